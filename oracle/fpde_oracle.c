/*
 * Plain FP64 CPU oracle for the P1 finite-element discretisation of the
 * steady Riesz fractional diffusion problem on a convex tetrahedral mesh
 * (Yang, Nie, Yuan & Wang, "Finite Element Methods for Fractional PDEs in
 * Three Dimensions").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file.  It shares no code with the
 * GPU library and is deliberately slow and literal: straight loops, a fixed
 * iteration order, FP64 throughout, no FMA contraction (built with
 * -ffp-contract=off).  The matrix-free products and the row-restricted form
 * split the Gauss points into one fixed block per OpenMP thread, each summed
 * into its own copy of the result; the copies are added in thread order, so
 * the thread count changes results only by rounding.
 *
 * What it computes (all citations are to the paper):
 *   - chord bounds a_i(x), b_i(x) of the convex domain along e_i (Sec. 1,
 *     eq. (1)): reached as the end of the walked path;
 *   - the integration path of a Gauss point: the ray-simplex intersection in
 *     volume coordinates (Sec. 2.2, eqs. eq:ck, eq:condrs2, eq:cond, equ:ac),
 *     the go-out m-face read from the zero pattern of the volume coordinates
 *     at r_max (Sec. 2.2, Fig. 2) and the move to the adjacent element;
 *   - the order-gamma left/right Riemann-Liouville derivatives (Sec. 1,
 *     eq. def, m = 1) of the P1 basis functions, summed segment by segment
 *     along the path (Sec. 2.1, the decomposition into D_{i,s_k}), in the
 *     closed form obtained by integrating the linear basis function by parts
 *     on each segment;
 *   - the element quadrature of the bilinear form (Sec. 2.1, (K_E)_kl) and
 *     the global dense matrix K = sum_E K_E, here for the Riesz operator split
 *     into (D_L^gamma u, D_R^gamma v) + (D_R^gamma u, D_L^gamma v)
 *     (form 1 of eq. equ:varsss with alpha = beta = gamma);
 *   - the load vector, a matrix-free product with K (walking every path, or
 *     from the derivative vectors walked once and kept) and the sums needed
 *     for the adjoint derivatives with respect to the order and the
 *     coefficients;
 *   - the non-symmetric matrix of the divergence-form two-sided problem of
 *     Sec. 3 (eq. equ:sfde2): order-beta_i trial derivatives along e_i with
 *     variable coefficients p_i, q_i, against the classical derivative of the
 *     test function on the Gauss point's own element;
 *   - the general uniform form (c D^alpha u, D^beta v) of Sec. 1 with the
 *     test operator on the opposite side, per-axis orders in [0, 1] and a
 *     coefficient per side.
 *
 * Readings where the paper is silent (each one is stated where it is used):
 *   - zero component of a volume coordinate: |k| <= 1e-12 max(1, |b~|, |r d~|),
 *     and the coordinate that set r_max is always zero;
 *   - several elements share the go-out edge/vertex: take the one with the
 *     smallest id among those in which the ray advances (relative 1e-12);
 *   - the ray origin u0 stays the Gauss point for every element it crosses.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS_BARY 1e-12   /* zero test on a volume coordinate */
#define ORC_EPS_ADV 1e-12    /* relative advance required past an edge/vertex */

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENONMANIFOLD = -2,
  ORC_EDEGENERATE = -3,
  ORC_ENONCONVEX = -4,
  ORC_EPATH = -5,
  ORC_ENOMEM = -10
};

typedef struct {
  int64_t nv, nt;
  double *xyz;      /* nv*3 */
  int32_t *tet;     /* nt*4 */
  int32_t *nbr;     /* nt*4: across face f (opposite local vertex f), -1 = boundary */
  double *M;        /* nt*9: A^{-1}, row r = gradient of volume coordinate k_{r+1} */
  double *vol;      /* nt */
  int32_t *vt_off;  /* nv+1 */
  int32_t *vt_tet;  /* 4*nt, ascending tet id per vertex */
  int32_t *dof;     /* nv: interior degree of freedom or -1 */
  int64_t ndof;
} orc_mesh;

/* ------------------------------------------------------------------------ */
/* Quadrature on the reference tetrahedron (Sec. 2.1 uses "Gaussian         */
/* quadrature" without naming a rule).  Barycentric points, weights sum 1.  */
/* ------------------------------------------------------------------------ */
int orc_quadrature(int nq, double *bary /* nq*4 */, double *w /* nq */) {
  if (nq == 1) {
    for (int j = 0; j < 4; j++) bary[j] = 0.25;
    w[0] = 1.0;
    return ORC_OK;
  }
  if (nq == 4) {
    /* degree 2: permutations of (a,b,b,b) */
    double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
    double b = (5.0 - sqrt(5.0)) / 20.0;
    for (int q = 0; q < 4; q++) {
      for (int j = 0; j < 4; j++) bary[q * 4 + j] = (j == q) ? a : b;
      w[q] = 0.25;
    }
    return ORC_OK;
  }
  if (nq == 11) {
    /* degree 4 (Keast): centroid (negative weight), a 4-point orbit of
       (11/14, 1/14, 1/14, 1/14) and a 6-point orbit of (a, a, b, b) with
       a,b = (1 +- sqrt(5/14))/4. */
    int q = 0;
    for (int j = 0; j < 4; j++) bary[j] = 0.25;
    w[q++] = -148.0 / 1875.0;
    for (int v = 0; v < 4; v++, q++) {
      for (int j = 0; j < 4; j++) bary[q * 4 + j] = (j == v) ? 11.0 / 14.0 : 1.0 / 14.0;
      w[q] = 343.0 / 7500.0;
    }
    double a = (1.0 + sqrt(5.0 / 14.0)) / 4.0;
    double b = (1.0 - sqrt(5.0 / 14.0)) / 4.0;
    static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int p = 0; p < 6; p++, q++) {
      for (int j = 0; j < 4; j++) bary[q * 4 + j] = b;
      bary[q * 4 + pairs[p][0]] = a;
      bary[q * 4 + pairs[p][1]] = a;
      w[q] = 56.0 / 375.0;
    }
    return ORC_OK;
  }
  return ORC_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Mesh: element adjacency ("adjacent information of the triangulation",    */
/* Sec. 2.2), m-face incidence via vertex->element lists, and A^{-1} per    */
/* element (Sec. 2.2: A = (e~1, e~2, e~3), e~i = v_i - v_0).                */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t v[3]; int32_t t; int32_t f; } orc_face;

static int face_cmp(const void *pa, const void *pb) {
  const orc_face *a = (const orc_face *)pa, *b = (const orc_face *)pb;
  for (int k = 0; k < 3; k++) {
    if (a->v[k] != b->v[k]) return a->v[k] < b->v[k] ? -1 : 1;
  }
  if (a->t != b->t) return a->t < b->t ? -1 : 1;
  return a->f - b->f;
}

static void sort3(int32_t *v) {
  int32_t t;
  if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
  if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
  if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

void orc_mesh_free(orc_mesh *m) {
  if (!m) return;
  free(m->xyz); free(m->tet); free(m->nbr); free(m->M); free(m->vol);
  free(m->vt_off); free(m->vt_tet); free(m->dof);
  free(m);
}

static double orc_cross_x(const double *a, const double *b) { return a[1] * b[2] - a[2] * b[1]; }
static double orc_cross_y(const double *a, const double *b) { return a[2] * b[0] - a[0] * b[2]; }
static double orc_cross_z(const double *a, const double *b) { return a[0] * b[1] - a[1] * b[0]; }

orc_mesh *orc_mesh_create(const double *xyz, int64_t nv, const int32_t *tet, int64_t nt, int *status) {
  *status = ORC_OK;
  if (nv <= 0 || nt <= 0 || !xyz || !tet) { *status = ORC_EINVAL; return NULL; }
  for (int64_t k = 0; k < 4 * nt; k++) {
    if (tet[k] < 0 || tet[k] >= nv) { *status = ORC_EINVAL; return NULL; }
  }
  orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
  m->nv = nv; m->nt = nt;
  m->xyz = (double *)malloc(sizeof(double) * 3 * nv);
  m->tet = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
  m->nbr = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
  m->M = (double *)malloc(sizeof(double) * 9 * nt);
  m->vol = (double *)malloc(sizeof(double) * nt);
  m->vt_off = (int32_t *)calloc(nv + 1, sizeof(int32_t));
  m->vt_tet = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
  m->dof = (int32_t *)malloc(sizeof(int32_t) * nv);
  memcpy(m->xyz, xyz, sizeof(double) * 3 * nv);
  memcpy(m->tet, tet, sizeof(int32_t) * 4 * nt);

  /* A^{-1} by the adjugate: rows (e2 x e3, e3 x e1, e1 x e2) / det */
  for (int64_t t = 0; t < nt; t++) {
    const double *v0 = xyz + 3 * (int64_t)tet[4 * t + 0];
    double e[3][3];
    for (int c = 1; c <= 3; c++) {
      const double *vc = xyz + 3 * (int64_t)tet[4 * t + c];
      for (int d = 0; d < 3; d++) e[c - 1][d] = vc[d] - v0[d];
    }
    double c1[3] = {orc_cross_x(e[1], e[2]), orc_cross_y(e[1], e[2]), orc_cross_z(e[1], e[2])};
    double c2[3] = {orc_cross_x(e[2], e[0]), orc_cross_y(e[2], e[0]), orc_cross_z(e[2], e[0])};
    double c3[3] = {orc_cross_x(e[0], e[1]), orc_cross_y(e[0], e[1]), orc_cross_z(e[0], e[1])};
    double det = e[0][0] * c1[0] + e[0][1] * c1[1] + e[0][2] * c1[2];
    double L = 0.0;
    for (int c = 0; c < 3; c++) {
      double l = sqrt(e[c][0] * e[c][0] + e[c][1] * e[c][1] + e[c][2] * e[c][2]);
      if (l > L) L = l;
    }
    if (!(fabs(det) > 1e-13 * L * L * L)) { *status = ORC_EDEGENERATE; orc_mesh_free(m); return NULL; }
    double *Mt = m->M + 9 * t;
    for (int d = 0; d < 3; d++) {
      Mt[0 + d] = c1[d] / det;
      Mt[3 + d] = c2[d] / det;
      Mt[6 + d] = c3[d] / det;
    }
    m->vol[t] = fabs(det) / 6.0;
  }

  /* face matching: face f of element t is opposite local vertex f */
  orc_face *F = (orc_face *)malloc(sizeof(orc_face) * 4 * nt);
  for (int64_t t = 0; t < nt; t++) {
    for (int f = 0; f < 4; f++) {
      orc_face *x = &F[4 * t + f];
      int k = 0;
      for (int j = 0; j < 4; j++) if (j != f) x->v[k++] = tet[4 * t + j];
      sort3(x->v);
      if (x->v[0] == x->v[1] || x->v[1] == x->v[2]) { free(F); *status = ORC_EDEGENERATE; orc_mesh_free(m); return NULL; }
      x->t = (int32_t)t; x->f = f;
      m->nbr[4 * t + f] = -1;
    }
  }
  qsort(F, 4 * nt, sizeof(orc_face), face_cmp);
  int64_t a = 0;
  while (a < 4 * nt) {
    int64_t b = a + 1;
    while (b < 4 * nt && F[b].v[0] == F[a].v[0] && F[b].v[1] == F[a].v[1] && F[b].v[2] == F[a].v[2]) b++;
    if (b - a > 2) { free(F); *status = ORC_ENONMANIFOLD; orc_mesh_free(m); return NULL; }
    if (b - a == 2) {
      m->nbr[4 * F[a].t + F[a].f] = F[a + 1].t;
      m->nbr[4 * F[a + 1].t + F[a + 1].f] = F[a].t;
    }
    a = b;
  }
  free(F);

  /* boundary vertices: vertices of faces without a neighbour */
  char *bnd = (char *)calloc(nv, 1);
  char *used = (char *)calloc(nv, 1);
  for (int64_t t = 0; t < nt; t++) {
    for (int j = 0; j < 4; j++) used[tet[4 * t + j]] = 1;
    for (int f = 0; f < 4; f++) {
      if (m->nbr[4 * t + f] < 0) {
        for (int j = 0; j < 4; j++) if (j != f) bnd[tet[4 * t + j]] = 1;
      }
    }
  }
  m->ndof = 0;
  for (int64_t v = 0; v < nv; v++) m->dof[v] = (used[v] && !bnd[v]) ? (int32_t)(m->ndof++) : -1;
  free(bnd);

  /* The chord bounds a_i(x), b_i(x) of Sec. 1 eq. (1) assume a convex domain.
     A polyhedron is convex exactly when each of its vertices lies on the
     inner side of the plane of each boundary face (each face plane supports
     it).  Tolerance: 1e-12 of the diagonal of the vertices' bounding box. */
  double lo[3], hi[3], diag = 0.0;
  for (int d = 0; d < 3; d++) lo[d] = hi[d] = xyz[d];
  for (int64_t v = 0; v < nv; v++) {
    for (int d = 0; d < 3; d++) {
      if (xyz[3 * v + d] < lo[d]) lo[d] = xyz[3 * v + d];
      if (xyz[3 * v + d] > hi[d]) hi[d] = xyz[3 * v + d];
    }
  }
  for (int d = 0; d < 3; d++) diag += (hi[d] - lo[d]) * (hi[d] - lo[d]);
  const double tol = 1e-12 * sqrt(diag);
  for (int64_t t = 0; t < nt; t++) {
    for (int f = 0; f < 4; f++) {
      if (m->nbr[4 * t + f] >= 0) continue;
      const double *p[3];
      int k = 0;
      for (int j = 0; j < 4; j++) if (j != f) p[k++] = xyz + 3 * (int64_t)tet[4 * t + j];
      const double *q = xyz + 3 * (int64_t)tet[4 * t + f];
      double a[3], b[3];
      for (int d = 0; d < 3; d++) { a[d] = p[1][d] - p[0][d]; b[d] = p[2][d] - p[0][d]; }
      double n[3] = {orc_cross_x(a, b), orc_cross_y(a, b), orc_cross_z(a, b)};
      double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int d = 0; d < 3; d++) n[d] /= len;
      /* outward: away from the element's own opposite vertex */
      if (n[0] * (q[0] - p[0][0]) + n[1] * (q[1] - p[0][1]) + n[2] * (q[2] - p[0][2]) > 0.0)
        for (int d = 0; d < 3; d++) n[d] = -n[d];
      for (int64_t v = 0; v < nv; v++) {
        if (!used[v]) continue;
        const double *x = xyz + 3 * v;
        double dist = n[0] * (x[0] - p[0][0]) + n[1] * (x[1] - p[0][1]) + n[2] * (x[2] - p[0][2]);
        if (dist > tol) { free(used); *status = ORC_ENONCONVEX; orc_mesh_free(m); return NULL; }
      }
    }
  }
  free(used);

  /* vertex -> element lists, ascending element id */
  for (int64_t k = 0; k < 4 * nt; k++) m->vt_off[tet[k] + 1]++;
  for (int64_t v = 0; v < nv; v++) m->vt_off[v + 1] += m->vt_off[v];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * nv);
  for (int64_t v = 0; v < nv; v++) fill[v] = m->vt_off[v];
  for (int64_t t = 0; t < nt; t++)
    for (int j = 0; j < 4; j++) m->vt_tet[fill[tet[4 * t + j]]++] = (int32_t)t;
  free(fill);
  return m;
}

int64_t orc_mesh_ndof(const orc_mesh *m) { return m->ndof; }
void orc_mesh_dof(const orc_mesh *m, int32_t *out) { memcpy(out, m->dof, sizeof(int32_t) * m->nv); }
void orc_mesh_nbr(const orc_mesh *m, int32_t *out) { memcpy(out, m->nbr, sizeof(int32_t) * 4 * m->nt); }
void orc_mesh_affine(const orc_mesh *m, double *M, double *vol) {
  memcpy(M, m->M, sizeof(double) * 9 * m->nt);
  memcpy(vol, m->vol, sizeof(double) * m->nt);
}

/* Gauss points x_g = sum_q beta_q v_q, summed in vertex order without FMA,
   and weights w_g = w_q |E|; g = element * nq + q. */
int orc_gauss_points(const orc_mesh *m, int nq, double *x /* G*3 */, double *w /* G */) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  for (int64_t t = 0; t < m->nt; t++) {
    for (int q = 0; q < nq; q++) {
      int64_t g = t * nq + q;
      for (int d = 0; d < 3; d++) {
        double s = 0.0;
        for (int j = 0; j < 4; j++) s = s + bary[q * 4 + j] * m->xyz[3 * (int64_t)m->tet[4 * t + j] + d];
        x[3 * g + d] = s;
      }
      w[g] = wq[q] * m->vol[t];
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Ray-simplex intersection in volume coordinates (Sec. 2.2).               */
/* For the ray u0 + r d, d = s e_i: b~ = (A^{-1}(u0 - v0), 1 - e^T A^{-1} b)  */
/* and d~ = (A^{-1} d, -e^T A^{-1} d); the ray is inside while              */
/* b~ + r d~ >= 0.  Index 0 of the arrays below is the coordinate k_0 = 1 - */
/* sum k_i (vertex v_0); index j = 1..3 is k_j (vertex v_j).               */
/* ------------------------------------------------------------------------ */
typedef struct {
  double bt[4], dt[4];
  double r_min, r_max;
  double kmax[4];
  int jexit;        /* coordinate whose ratio set r_max (first one on ties) */
} orc_isect;

/* Zero test on the volume coordinate k~_j at the go-out point: |k~_j| is
   compared with 1e-12 times the size of the terms b~_j and r_max d~_j it is
   the difference of (at least 1e-12), because for elements far from the ray
   origin or badly shaped the rounding error of b~ + r d~ grows with them.
   The coordinate that set r_max is zero by construction. */
static int orc_is_zero(const orc_isect *o, int j) {
  if (j == o->jexit) return 1;
  double s = fabs(o->bt[j]);
  double t = fabs(o->r_max * o->dt[j]);
  if (t > s) s = t;
  if (s < 1.0) s = 1.0;
  return fabs(o->kmax[j]) <= ORC_EPS_BARY * s;
}

static void orc_intersect(const orc_mesh *m, int64_t t, const double *u0, int i, int s, orc_isect *o) {
  const double *Mt = m->M + 9 * t;
  const double *v0 = m->xyz + 3 * (int64_t)m->tet[4 * t];
  double b[3] = {u0[0] - v0[0], u0[1] - v0[1], u0[2] - v0[2]};
  for (int r = 0; r < 3; r++) {
    o->bt[r + 1] = (Mt[3 * r + 0] * b[0] + Mt[3 * r + 1] * b[1]) + Mt[3 * r + 2] * b[2];
    o->dt[r + 1] = (s > 0) ? Mt[3 * r + i] : -Mt[3 * r + i];
  }
  o->bt[0] = 1.0 - ((o->bt[1] + o->bt[2]) + o->bt[3]);
  o->dt[0] = -((o->dt[1] + o->dt[2]) + o->dt[3]);
  /* eq:cond: r >= 0 and b~_j + r d~_j >= 0 for every j */
  o->r_max = INFINITY;
  o->r_min = 0.0;
  o->jexit = -1;
  for (int j = 0; j < 4; j++) {
    if (o->dt[j] < 0.0) {
      double r = -o->bt[j] / o->dt[j];
      if (r < o->r_max) {
        o->r_max = r;
        o->jexit = j;
      }
    } else if (o->dt[j] > 0.0) {
      double r = -o->bt[j] / o->dt[j];
      if (r > o->r_min) o->r_min = r;
    }
  }
  /* equ:ac: volume coordinates of the go-out point */
  for (int j = 0; j < 4; j++) {
    double p = o->r_max * o->dt[j];
    o->kmax[j] = o->bt[j] + p;
  }
}

/* Exposed for the face-classification test: volume coordinates at the
   go-out point and its zero pattern (bit j set <=> k_j is zero). */
int orc_exit_pattern(const orc_mesh *m, int64_t t, const double *u0, int i, int s,
                     double *kmax /* 4 */, double *rminmax /* 2 */) {
  orc_isect o;
  orc_intersect(m, t, u0, i, s, &o);
  int z = 0;
  for (int j = 0; j < 4; j++) {
    kmax[j] = o.kmax[j];
    if (orc_is_zero(&o, j)) z |= 1 << j;
  }
  rminmax[0] = o.r_min;
  rminmax[1] = o.r_max;
  return z;
}

/* The path of one half-ray (Sec. 2.2): start in the Gauss point's own
   element; in each element take the go-out point r_max and its zero pattern
   Z.  |Z| = 1: go-out point on a face -> the (at most one) element across it,
   none = boundary reached.  |Z| >= 2: an edge or vertex; search the elements
   that contain that m-face and continue in the one (smallest id) in which
   the ray advances; none = boundary reached.
   Emits (element, r_max) for every element in which the ray advances. */
int orc_walk(const orc_mesh *m, int64_t t0, const double *u0, int i, int s, int cap,
             int32_t *tets, double *r_end, int *n_out) {
  int64_t t = t0;
  double r_cur = 0.0;
  int n = 0;
  for (int step = 0; step < cap + 64; step++) {
    orc_isect o;
    orc_intersect(m, t, u0, i, s, &o);
    if (!(o.r_max < INFINITY)) return ORC_EPATH;
    if (o.r_max > r_cur) {
      if (n >= cap) return ORC_EPATH;
      tets[n] = (int32_t)t;
      r_end[n] = o.r_max;
      n++;
      r_cur = o.r_max;
    }
    int Z[4], nz = 0;
    for (int j = 0; j < 4; j++) if (orc_is_zero(&o, j)) Z[nz++] = j;
    if (nz == 0) return ORC_EPATH;
    if (nz == 1) {
      int32_t nx = m->nbr[4 * t + Z[0]];
      if (nx < 0) { *n_out = n; return ORC_OK; }
      t = nx;
      continue;
    }
    /* edge (|Z| = 2) or vertex (|Z| = 3): the m-face spanned by the
       vertices whose volume coordinate is not zero (Fig. 2) */
    int32_t keep[4];
    int nk = 0;
    for (int j = 0; j < 4; j++) {
      int in_z = 0;
      for (int k = 0; k < nz; k++) if (Z[k] == j) in_z = 1;
      if (!in_z) keep[nk++] = m->tet[4 * t + j];
    }
    if (nk == 0) return ORC_EPATH;
    int64_t best = -1;
    for (int32_t p = m->vt_off[keep[0]]; p < m->vt_off[keep[0] + 1]; p++) {
      int64_t c = m->vt_tet[p];
      if (c == t) continue;
      int has_all = 1;
      for (int k = 1; k < nk; k++) {
        int found = 0;
        for (int j = 0; j < 4; j++) if (m->tet[4 * c + j] == keep[k]) found = 1;
        if (!found) has_all = 0;
      }
      if (!has_all) continue;
      orc_isect oc;
      orc_intersect(m, c, u0, i, s, &oc);
      if (oc.r_max - r_cur > ORC_EPS_ADV * r_cur) { best = c; break; }
    }
    if (best < 0) { *n_out = n; return ORC_OK; }
    t = best;
  }
  return ORC_EPATH;
}

/* FNV-1a (64 bit) over the element ids of a path, 4 little-endian bytes each */
static uint64_t orc_fnv1a(const int32_t *ids, int n) {
  uint64_t h = 14695981039346656037ULL;
  for (int k = 0; k < n; k++) {
    uint32_t u = (uint32_t)ids[k];
    for (int b = 0; b < 4; b++) {
      h ^= (uint64_t)((u >> (8 * b)) & 0xffu);
      h *= 1099511628211ULL;
    }
  }
  return h;
}

/* Half-ray h = g*6 + 2*i + side (side 0: -e_i, side 1: +e_i). */
static void orc_ray_origin(const orc_mesh *m, int nq, const double *bary, int64_t g, double *u0) {
  int64_t t = g / nq;
  int q = (int)(g % nq);
  for (int d = 0; d < 3; d++) {
    double s = 0.0;
    for (int j = 0; j < 4; j++) s = s + bary[q * 4 + j] * m->xyz[3 * (int64_t)m->tet[4 * t + j] + d];
    u0[d] = s;
  }
}

int orc_paths(const orc_mesh *m, int nq, int64_t h0, int64_t count, int cap,
              int32_t *len, uint64_t *hash, int32_t *ids /* count*cap or NULL */,
              double *rend /* count*cap or NULL */) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int st = ORC_OK;
  for (int64_t k = 0; k < count; k++) {
    int64_t h = h0 + k;
    int64_t g = h / 6;
    int dir = (int)(h % 6), i = dir / 2, s = (dir & 1) ? 1 : -1;
    double u0[3];
    orc_ray_origin(m, nq, bary, g, u0);
    int n = 0;
    st = orc_walk(m, g / nq, u0, i, s, cap, tb, rb, &n);
    if (st != ORC_OK) break;
    len[k] = n;
    hash[k] = orc_fnv1a(tb, n);
    if (ids) for (int j = 0; j < n; j++) ids[k * cap + j] = tb[j];
    if (rend) for (int j = 0; j < n; j++) rend[k * cap + j] = rb[j];
  }
  free(tb); free(rb);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Closed-form RL derivative of the P1 basis functions along a path.        */
/* On segment s_k = [r_{k-1}, r_k] (distances from the Gauss point x along   */
/* the ray) the basis function psi_l has the constant slope                  */
/* sigma_{k,l} = d psi_l / d x_i on E_k.  From eq. def with m = 1 and         */
/* integration by parts, each segment contributes                            */
/*   left  (ray -e_i):  +sigma (r_k^{1-g} - r_{k-1}^{1-g}) / Gamma(2-g)       */
/*   right (ray +e_i):  -sigma (r_k^{1-g} - r_{k-1}^{1-g}) / Gamma(2-g)       */
/* with 0^{1-g} = 0 at the Gauss point itself, plus for a basis function    */
/* that is non-zero at the path end p_a (p_b) the boundary term             */
/*   psi_l(p_end) * r_end^{-g} / Gamma(1-g)                                  */
/* (zero for every interior node, kept for the all-nodes check).            */
/* ------------------------------------------------------------------------ */
typedef struct {
  double *acc;     /* nv, zero outside calls */
  int32_t *touched; int nt_; char *mark;
} orc_work;

static orc_work *orc_work_new(int64_t nv) {
  orc_work *w = (orc_work *)malloc(sizeof(orc_work));
  w->acc = (double *)calloc(nv, sizeof(double));
  w->mark = (char *)calloc(nv, 1);
  w->touched = (int32_t *)malloc(sizeof(int32_t) * nv);
  w->nt_ = 0;
  return w;
}
static void orc_work_free(orc_work *w) { free(w->acc); free(w->mark); free(w->touched); free(w); }

static void orc_touch(orc_work *w, int32_t v, double val) {
  if (!w->mark[v]) { w->mark[v] = 1; w->touched[w->nt_++] = v; }
  w->acc[v] += val;
}

static int icmp32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* slope of the volume coordinate of local vertex j along e_i on element t */
static double orc_slope(const orc_mesh *m, int64_t t, int j, int i) {
  const double *Mt = m->M + 9 * t;
  if (j > 0) return Mt[3 * (j - 1) + i];
  return -((Mt[0 + i] + Mt[3 + i]) + Mt[6 + i]);
}

typedef struct {
  double gamma;
  double inv_g2;   /* 1/Gamma(2-gamma) */
  double inv_g1;   /* 1/Gamma(1-gamma) (0 at gamma = 1) */
  double half_psi0;/* psi(2-gamma)/2, for the alpha-derivative */
} orc_order;

static double orc_pow_seg(double r, double e) { return (r > 0.0) ? pow(r, e) : 0.0; }
static double orc_lnpow(double r, double e) { return (r > 0.0) ? log(r) * pow(r, e) : 0.0; }

/* Sparse vector of D^gamma psi_l (x) over nodes for one half-ray.
   mode 0: interior dofs, value; mode 1: all nodes incl. boundary term;
   mode 2: interior dofs, derivative of the value with respect to alpha
   (gamma = alpha/2).  Output: node ids (vertex ids for mode 1, dofs else),
   ascending, and values.  Returns count or a negative status. */
static int orc_ray_vector(const orc_mesh *m, int nq, const double *bary, int64_t g, int i, int side,
                          const orc_order *ord, int mode, int cap, orc_work *w,
                          int32_t *out_id, double *out_val, int32_t *tb, double *rb) {
  double u0[3];
  orc_ray_origin(m, nq, bary, g, u0);
  int s = side ? 1 : -1;
  int n = 0;
  int st = orc_walk(m, g / nq, u0, i, s, cap, tb, rb, &n);
  if (st != ORC_OK) return st;
  double e = 1.0 - ord->gamma;
  double sgn = side ? -1.0 : 1.0;
  double r_lo = 0.0;
  for (int k = 0; k < n; k++) {
    int64_t t = tb[k];
    double r_hi = rb[k];
    double dP;
    if (mode == 2) {
      /* d/dalpha of r^{1-g}/Gamma(2-g): -(1/2) ln r r^{1-g} G + (psi0/2) r^{1-g} G */
      double P = orc_pow_seg(r_hi, e) - orc_pow_seg(r_lo, e);
      double Q = orc_lnpow(r_hi, e) - orc_lnpow(r_lo, e);
      dP = ord->inv_g2 * (ord->half_psi0 * P - 0.5 * Q);
    } else {
      dP = ord->inv_g2 * (orc_pow_seg(r_hi, e) - orc_pow_seg(r_lo, e));
    }
    for (int j = 0; j < 4; j++) {
      int32_t v = m->tet[4 * t + j];
      if (mode != 1 && m->dof[v] < 0) continue;
      double sigma = orc_slope(m, t, j, i);
      orc_touch(w, v, sgn * sigma * dP);
    }
    r_lo = r_hi;
  }
  if (mode == 1 && n > 0) {
    /* boundary term at the path end: psi_l(p_end) (r_end)^{-gamma}/Gamma(1-gamma) */
    orc_isect o;
    int64_t t = tb[n - 1];
    orc_intersect(m, t, u0, i, s, &o);
    double rend = rb[n - 1];
    double c = ord->inv_g1 * pow(rend, -ord->gamma);
    for (int j = 0; j < 4; j++) {
      double lam = o.kmax[j];
      if (lam != 0.0) orc_touch(w, m->tet[4 * t + j], lam * c);
    }
  }
  int cnt = w->nt_;
  qsort(w->touched, cnt, sizeof(int32_t), icmp32);
  for (int k = 0; k < cnt; k++) {
    int32_t v = w->touched[k];
    out_id[k] = (mode == 1) ? v : m->dof[v];
    out_val[k] = w->acc[v];
    w->acc[v] = 0.0;
    w->mark[v] = 0;
  }
  w->nt_ = 0;
  return cnt;
}

static void orc_fill_order(orc_order *o, double gamma, double inv_g2, double inv_g1, double half_psi0) {
  o->gamma = gamma; o->inv_g2 = inv_g2; o->inv_g1 = inv_g1; o->half_psi0 = half_psi0;
}

/* One half-ray's vector for the tests (mode as in orc_ray_vector). */
int orc_ray_values(const orc_mesh *m, int nq, int64_t g, int i, int side, double gamma,
                   double inv_g2, double inv_g1, double half_psi0, int mode, int cap,
                   int32_t *out_id, double *out_val) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  orc_order ord;
  orc_fill_order(&ord, gamma, inv_g2, inv_g1, half_psi0);
  orc_work *w = orc_work_new(m->nv);
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int r = orc_ray_vector(m, nq, bary, g, i, side, &ord, mode, cap, w, out_id, out_val, tb, rb);
  free(tb); free(rb); orc_work_free(w);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Dense assembly (Sec. 2.1):                                              */
/*   K_jk = sum_i K_i c_alpha sum_g w_g [L_gi(k) R_gi(j) + R_gi(k) L_gi(j)]  */
/* with L = D_L^gamma psi, R = D_R^gamma psi at the Gauss point and          */
/* c_alpha = 1/(2 cos(pi alpha/2)).  Both products are written out as        */
/* separate (j,k) loops.  A is ndof x ndof row-major, zeroed by the caller.  */
/* ------------------------------------------------------------------------ */
int orc_assemble(const orc_mesh *m, int nq, double gamma, double inv_g2, double c_alpha,
                 const double *Kc, int cap, double *A) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  orc_order ord;
  orc_fill_order(&ord, gamma, inv_g2, 0.0, 0.0);
  orc_work *w = orc_work_new(m->nv);
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int32_t *Li = (int32_t *)malloc(sizeof(int32_t) * 4 * cap), *Ri = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
  double *Lv = (double *)malloc(sizeof(double) * 4 * cap), *Rv = (double *)malloc(sizeof(double) * 4 * cap);
  int64_t n = m->ndof;
  int st = ORC_OK;
  for (int64_t g = 0; g < m->nt * nq && st == ORC_OK; g++) {
    double wg = wq[g % nq] * m->vol[g / nq];
    for (int i = 0; i < 3; i++) {
      int nl = orc_ray_vector(m, nq, bary, g, i, 0, &ord, 0, cap, w, Li, Lv, tb, rb);
      if (nl < 0) { st = nl; break; }
      int nr = orc_ray_vector(m, nq, bary, g, i, 1, &ord, 0, cap, w, Ri, Rv, tb, rb);
      if (nr < 0) { st = nr; break; }
      double W = wg * Kc[i] * c_alpha;
      for (int a = 0; a < nr; a++)
        for (int b = 0; b < nl; b++) A[Ri[a] * n + Li[b]] += W * (Rv[a] * Lv[b]);
      for (int a = 0; a < nl; a++)
        for (int b = 0; b < nr; b++) A[Li[a] * n + Ri[b]] += W * (Lv[a] * Rv[b]);
    }
  }
  free(tb); free(rb); free(Li); free(Ri); free(Lv); free(Rv); orc_work_free(w);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Divergence-form two-sided problem (Sec. 3, eq. equ:sfde2):               */
/*   sum_i D_i (p_i D_L^{beta_i} u - q_i D_R^{beta_i} u) = f,                */
/* whose variational form, after one classical integration by parts on the  */
/* test side, is a(u, v) = -sum_i [(p_i D_L u, D_i v) - (q_i D_R u, D_i v)].  */
/* With u = psi_k (trial) and v = psi_j (test) and the element quadrature of */
/* Sec. 2.1 this is                                                           */
/*   K_jk = -sum_i sum_g w_g d_i psi_j(x_g) [p_i L_gi(k) - q_i R_gi(k)]        */
/* where L_gi, R_gi are the order-beta_i vectors of the walked half-rays and  */
/* d_i psi_j(x_g) is the constant slope of psi_j on the Gauss point's own     */
/* element (zero for the other nodes).  pq holds p_i(x_g) at [i G + g] and    */
/* q_i(x_g) at [(3 + i) G + g].  A is ndof x ndof row-major (row = test),     */
/* zeroed by the caller.                                                      */
/* ------------------------------------------------------------------------ */
/* rows: NULL for the whole matrix (A is ndof x ndof), or the list of nrows
   rows to keep (A is nrows x ndof, row r of A = row rows[r] of K; each
   listed row at most once). */
static int orc_div_sums(const orc_mesh *m, int nq, const double *gamma, const double *inv_g2,
                        const double *pq, int cap, const int64_t *slot, double *A) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  orc_order ord[3];
  for (int i = 0; i < 3; i++) orc_fill_order(&ord[i], gamma[i], inv_g2[i], 0.0, 0.0);
  orc_work *w = orc_work_new(m->nv);
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int32_t *Li = (int32_t *)malloc(sizeof(int32_t) * 4 * cap), *Ri = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
  double *Lv = (double *)malloc(sizeof(double) * 4 * cap), *Rv = (double *)malloc(sizeof(double) * 4 * cap);
  int64_t n = m->ndof, G = m->nt * nq;
  int st = ORC_OK;
  for (int64_t g = 0; g < G && st == ORC_OK; g++) {
    int64_t t = g / nq;
    if (slot) {  /* skip Gauss points whose element has no kept row */
      int any = 0;
      for (int jl = 0; jl < 4; jl++) {
        int32_t j = m->dof[m->tet[4 * t + jl]];
        if (j >= 0 && slot[j] >= 0) any = 1;
      }
      if (!any) continue;
    }
    double wg = wq[g % nq] * m->vol[t];
    for (int i = 0; i < 3; i++) {
      int nl = orc_ray_vector(m, nq, bary, g, i, 0, &ord[i], 0, cap, w, Li, Lv, tb, rb);
      if (nl < 0) { st = nl; break; }
      int nr = orc_ray_vector(m, nq, bary, g, i, 1, &ord[i], 0, cap, w, Ri, Rv, tb, rb);
      if (nr < 0) { st = nr; break; }
      double p = pq[(int64_t)i * G + g], q = pq[(int64_t)(3 + i) * G + g];
      for (int jl = 0; jl < 4; jl++) {
        int32_t j = m->dof[m->tet[4 * t + jl]];
        if (j < 0) continue;
        int64_t row = slot ? slot[j] : j;
        if (row < 0) continue;
        double dpsi = orc_slope(m, t, jl, i);
        for (int b = 0; b < nl; b++) A[row * n + Li[b]] += -(wg * dpsi * p) * Lv[b];
        for (int b = 0; b < nr; b++) A[row * n + Ri[b]] += (wg * dpsi * q) * Rv[b];
      }
    }
  }
  free(tb); free(rb); free(Li); free(Ri); free(Lv); free(Rv); orc_work_free(w);
  return st;
}

int orc_assemble_div(const orc_mesh *m, int nq, const double *gamma /* 3 */, const double *inv_g2 /* 3 */,
                     const double *pq, int cap, double *A) {
  return orc_div_sums(m, nq, gamma, inv_g2, pq, cap, NULL, A);
}

/* Rows rows[0..nrows) of the same matrix (A: nrows x ndof, zeroed by the
   caller), for checks at sizes where the whole matrix is too large. */
int orc_assemble_div_rows(const orc_mesh *m, int nq, const double *gamma, const double *inv_g2,
                          const double *pq, int cap, int64_t nrows, const int64_t *rows, double *A) {
  int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (m->ndof > 0 ? m->ndof : 1));
  for (int64_t j = 0; j < m->ndof; j++) slot[j] = -1;
  for (int64_t r = 0; r < nrows; r++) {
    if (rows[r] < 0 || rows[r] >= m->ndof || slot[rows[r]] >= 0) { free(slot); return ORC_EINVAL; }
    slot[rows[r]] = r;
  }
  int st = orc_div_sums(m, nq, gamma, inv_g2, pq, cap, slot, A);
  free(slot);
  return st;
}

/* ------------------------------------------------------------------------ */
/* The uniform form of Sec. 1 (eq. equ:varsss) with its element quadrature  */
/* (Sec. 2.1, (K_E)_kl): per axis i a trial order alpha_i and a test order  */
/* beta_i in [0, 1], the test operator on the side opposite to the trial     */
/* one, and a coefficient per side:                                          */
/*   K_kl = sum_i sum_g w_g [cl_i(x_g) D_L^{a_i} psi_l(x_g) D_R^{b_i} psi_k(x_g) */
/*                         + cr_i(x_g) D_R^{a_i} psi_l(x_g) D_L^{b_i} psi_k(x_g)] */
/* (row k = test function).  coef holds cl_i(x_g) at [i G + g] and cr_i(x_g) */
/* at [(3 + i) G + g].  A is ndof x ndof row-major, zeroed by the caller.    */
/* ------------------------------------------------------------------------ */
/* slot: NULL for the whole matrix, else slot[k] = the row of A that keeps
   row k of K, or -1 (A is then nrows x ndof). */
static int orc_form_sums(const orc_mesh *m, int nq, const double *ga, const double *iga, const double *gb,
                         const double *igb, const double *coef, int cap, const int64_t *slot, int64_t nrows,
                         double *A) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  orc_order oa[3], ob[3];
  for (int i = 0; i < 3; i++) {
    orc_fill_order(&oa[i], ga[i], iga[i], 0.0, 0.0);
    orc_fill_order(&ob[i], gb[i], igb[i], 0.0, 0.0);
  }
  int64_t n = m->ndof, G = m->nt * nq;
  /* With a row list each OpenMP thread adds its block of Gauss points into
     its own copy of the rows, and the copies are added in thread order; the
     whole matrix is summed by one thread. */
  int nth = 1;
#ifdef _OPENMP
  if (slot) nth = omp_get_max_threads();
#endif
  const size_t asz = slot ? (size_t)nrows * (size_t)n : 0;
  double *At = (slot && nth > 1) ? (double *)calloc((size_t)nth * (asz > 0 ? asz : 1), sizeof(double)) : NULL;
  int st = ORC_OK;
#pragma omp parallel num_threads(nth)
  {
    int me = 0;
#ifdef _OPENMP
    me = omp_get_thread_num();
#endif
    double *Al = At ? At + (size_t)me * (asz > 0 ? asz : 1) : A;
    orc_work *w = orc_work_new(m->nv);
    int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *rb = (double *)malloc(sizeof(double) * cap);
    int32_t *id[4];
    double *v[4];
    for (int k = 0; k < 4; k++) {
      id[k] = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
      v[k] = (double *)malloc(sizeof(double) * 4 * cap);
    }
    int my_st = ORC_OK;
#pragma omp for schedule(static)
    for (int64_t g = 0; g < G; g++) {
      if (my_st != ORC_OK) continue;
      double wg = wq[g % nq] * m->vol[g / nq];
      for (int i = 0; i < 3; i++) {
        /* 0: D_L^a, 1: D_R^a (trial); 2: D_L^b, 3: D_R^b (test).  The test
           vectors are walked first: with a row list, a point whose test
           vectors touch no kept row adds nothing. */
        int cnt[4];
        for (int k = 3; k >= 0; k--) {
          if (k == 1 && slot) {
            int any = 0;
            for (int a = 0; a < cnt[3] && !any; a++) any = slot[id[3][a]] >= 0;
            for (int a = 0; a < cnt[2] && !any; a++) any = slot[id[2][a]] >= 0;
            if (!any) break;
          }
          cnt[k] = orc_ray_vector(m, nq, bary, g, i, k & 1, k < 2 ? &oa[i] : &ob[i], 0, cap, w, id[k], v[k], tb, rb);
          if (cnt[k] < 0) { my_st = cnt[k]; break; }
          if (k == 0) {
            double cl = coef[(int64_t)i * G + g], cr = coef[(int64_t)(3 + i) * G + g];
            for (int a = 0; a < cnt[3]; a++) {
              int64_t row = slot ? slot[id[3][a]] : id[3][a];
              if (row < 0) continue;
              for (int b = 0; b < cnt[0]; b++) Al[row * n + id[0][b]] += (wg * cl) * (v[3][a] * v[0][b]);
            }
            for (int a = 0; a < cnt[2]; a++) {
              int64_t row = slot ? slot[id[2][a]] : id[2][a];
              if (row < 0) continue;
              for (int b = 0; b < cnt[1]; b++) Al[row * n + id[1][b]] += (wg * cr) * (v[2][a] * v[1][b]);
            }
          }
        }
        if (my_st != ORC_OK) break;
      }
    }
#pragma omp critical
    if (my_st != ORC_OK && st == ORC_OK) st = my_st;
    free(tb); free(rb);
    for (int k = 0; k < 4; k++) { free(id[k]); free(v[k]); }
    orc_work_free(w);
  }
  if (At) {
    for (size_t e = 0; e < asz; e++) {
      double acc = 0.0;
      for (int t = 0; t < nth; t++) acc += At[(size_t)t * asz + e];
      A[e] += acc;
    }
    free(At);
  }
  return st;
}

int orc_assemble_form(const orc_mesh *m, int nq, const double *ga /* 3 */, const double *iga /* 3 */,
                      const double *gb /* 3 */, const double *igb /* 3 */, const double *coef, int cap,
                      double *A) {
  return orc_form_sums(m, nq, ga, iga, gb, igb, coef, cap, NULL, 0, A);
}

/* Rows rows[0..nrows) of the same matrix (A: nrows x ndof, zeroed by the
   caller, each row listed at most once), for checks at sizes where the
   whole matrix is too large. */
int orc_assemble_form_rows(const orc_mesh *m, int nq, const double *ga, const double *iga, const double *gb,
                           const double *igb, const double *coef, int cap, int64_t nrows, const int64_t *rows,
                           double *A) {
  int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (m->ndof > 0 ? m->ndof : 1));
  for (int64_t j = 0; j < m->ndof; j++) slot[j] = -1;
  for (int64_t r = 0; r < nrows; r++) {
    if (rows[r] < 0 || rows[r] >= m->ndof || slot[rows[r]] >= 0) { free(slot); return ORC_EINVAL; }
    slot[rows[r]] = r;
  }
  int st = orc_form_sums(m, nq, ga, iga, gb, igb, coef, cap, slot, nrows, A);
  free(slot);
  return st;
}

/* Matrix-free product y = K x (same sums as orc_assemble, never forming K),
   restricted to the Gauss points g in [g0, g1): the whole product for
   g0 = 0, g1 = G.  Each OpenMP thread walks a fixed block of Gauss points and
   sums into its own copy of y; the copies are added in thread order. */
int orc_apply_range(const orc_mesh *m, int nq, double gamma, double inv_g2, double c_alpha,
                    const double *Kc, int cap, const double *x, int64_t g0, int64_t g1, double *y) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  if (g0 < 0 || g1 > m->nt * nq || g0 > g1) return ORC_EINVAL;
  orc_order ord;
  orc_fill_order(&ord, gamma, inv_g2, 0.0, 0.0);
  const int64_t n = m->ndof;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  double *yt = (double *)calloc((size_t)nth * (size_t)(n > 0 ? n : 1), sizeof(double));
  int st = ORC_OK;
#pragma omp parallel num_threads(nth)
  {
    int me = 0;
#ifdef _OPENMP
    me = omp_get_thread_num();
#endif
    double *yl = yt + (size_t)me * (size_t)(n > 0 ? n : 1);
    orc_work *w = orc_work_new(m->nv);
    int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *rb = (double *)malloc(sizeof(double) * cap);
    int32_t *Li = (int32_t *)malloc(sizeof(int32_t) * 4 * cap), *Ri = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
    double *Lv = (double *)malloc(sizeof(double) * 4 * cap), *Rv = (double *)malloc(sizeof(double) * 4 * cap);
    int my_st = ORC_OK;
#pragma omp for schedule(static)
    for (int64_t g = g0; g < g1; g++) {
      if (my_st != ORC_OK) continue;
      double wg = wq[g % nq] * m->vol[g / nq];
      for (int i = 0; i < 3; i++) {
        int nl = orc_ray_vector(m, nq, bary, g, i, 0, &ord, 0, cap, w, Li, Lv, tb, rb);
        if (nl < 0) { my_st = nl; break; }
        int nr = orc_ray_vector(m, nq, bary, g, i, 1, &ord, 0, cap, w, Ri, Rv, tb, rb);
        if (nr < 0) { my_st = nr; break; }
        double W = wg * Kc[i] * c_alpha;
        double lx = 0.0, rx = 0.0;
        for (int b = 0; b < nl; b++) lx += Lv[b] * x[Li[b]];
        for (int b = 0; b < nr; b++) rx += Rv[b] * x[Ri[b]];
        for (int a = 0; a < nr; a++) yl[Ri[a]] += W * (Rv[a] * lx);
        for (int a = 0; a < nl; a++) yl[Li[a]] += W * (Lv[a] * rx);
      }
    }
#pragma omp critical
    if (my_st != ORC_OK && st == ORC_OK) st = my_st;
    free(tb); free(rb); free(Li); free(Ri); free(Lv); free(Rv); orc_work_free(w);
  }
  for (int64_t j = 0; j < n; j++) {
    double acc = 0.0;
    for (int t = 0; t < nth; t++) acc += yt[(size_t)t * (size_t)n + j];
    y[j] = acc;
  }
  free(yt);
  return st;
}

int orc_apply(const orc_mesh *m, int nq, double gamma, double inv_g2, double c_alpha,
              const double *Kc, int cap, const double *x, double *y) {
  return orc_apply_range(m, nq, gamma, inv_g2, c_alpha, Kc, cap, x, 0, m->nt * nq, y);
}

/* The same operator with its derivative vectors kept: every half-ray is
   walked once (orc_ray_vector, as above) and its sparse vector stored, so
   repeated products (conjugate gradients at sizes where the dense matrix is
   out of reach) cost two passes over the stored entries each.  The Gauss
   points are cut into one contiguous chunk per OpenMP thread at creation;
   chunk c holds, per point g and axis i, the weight W = w_g K_i c_alpha and
   the entries of L (side 0) then R (side 1). */
typedef struct {
  int64_t g0, g1, n_ent, cap_ent;
  int32_t *cnt;  /* (g1 - g0) * 6: entries of (g, i, side) at [6 (g - g0) + 2 i + side] */
  double *W;     /* (g1 - g0) * 3 */
  int32_t *id;
  double *val;
} orc_op_chunk;

typedef struct {
  int64_t n, nchunk;
  orc_op_chunk *c;
} orc_operator;

void orc_operator_free(orc_operator *op) {
  if (!op) return;
  for (int64_t k = 0; k < op->nchunk; k++) {
    free(op->c[k].cnt); free(op->c[k].W); free(op->c[k].id); free(op->c[k].val);
  }
  free(op->c);
  free(op);
}

orc_operator *orc_operator_create(const orc_mesh *m, int nq, double gamma, double inv_g2, double c_alpha,
                                  const double *Kc, int cap, int *status) {
  double bary[44], wq[11];
  *status = ORC_OK;
  if (orc_quadrature(nq, bary, wq) != ORC_OK) { *status = ORC_EINVAL; return NULL; }
  orc_order ord;
  orc_fill_order(&ord, gamma, inv_g2, 0.0, 0.0);
  const int64_t G = m->nt * nq;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  orc_operator *op = (orc_operator *)calloc(1, sizeof(orc_operator));
  op->n = m->ndof;
  op->nchunk = nth;
  op->c = (orc_op_chunk *)calloc((size_t)nth, sizeof(orc_op_chunk));
  int st = ORC_OK;
#pragma omp parallel num_threads(nth)
  {
    int me = 0;
#ifdef _OPENMP
    me = omp_get_thread_num();
#endif
    orc_op_chunk *c = &op->c[me];
    c->g0 = G * me / nth;
    c->g1 = G * (me + 1) / nth;
    const int64_t ng = c->g1 - c->g0;
    c->cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(6 * ng + 1));
    c->W = (double *)malloc(sizeof(double) * (size_t)(3 * ng + 1));
    c->cap_ent = 64 * ng + 1024;
    c->id = (int32_t *)malloc(sizeof(int32_t) * (size_t)c->cap_ent);
    c->val = (double *)malloc(sizeof(double) * (size_t)c->cap_ent);
    orc_work *w = orc_work_new(m->nv);
    int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *rb = (double *)malloc(sizeof(double) * cap);
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
    double *vals = (double *)malloc(sizeof(double) * 4 * cap);
    int my_st = ORC_OK;
    for (int64_t g = c->g0; g < c->g1 && my_st == ORC_OK; g++) {
      double wg = wq[g % nq] * m->vol[g / nq];
      for (int i = 0; i < 3 && my_st == ORC_OK; i++) {
        c->W[3 * (g - c->g0) + i] = wg * Kc[i] * c_alpha;
        for (int side = 0; side < 2; side++) {
          int nn = orc_ray_vector(m, nq, bary, g, i, side, &ord, 0, cap, w, ids, vals, tb, rb);
          if (nn < 0) { my_st = nn; break; }
          if (c->n_ent + nn > c->cap_ent) {
            c->cap_ent = 2 * (c->n_ent + nn);
            c->id = (int32_t *)realloc(c->id, sizeof(int32_t) * (size_t)c->cap_ent);
            c->val = (double *)realloc(c->val, sizeof(double) * (size_t)c->cap_ent);
          }
          memcpy(c->id + c->n_ent, ids, sizeof(int32_t) * nn);
          memcpy(c->val + c->n_ent, vals, sizeof(double) * nn);
          c->n_ent += nn;
          c->cnt[6 * (g - c->g0) + 2 * i + side] = nn;
        }
      }
    }
#pragma omp critical
    if (my_st != ORC_OK && st == ORC_OK) st = my_st;
    free(tb); free(rb); free(ids); free(vals); orc_work_free(w);
  }
  if (st != ORC_OK) { orc_operator_free(op); *status = st; return NULL; }
  return op;
}

int64_t orc_operator_entries(const orc_operator *op) {
  int64_t t = 0;
  for (int64_t k = 0; k < op->nchunk; k++) t += op->c[k].n_ent;
  return t;
}

/* y = K x from the stored vectors: per (g, i), y += W [R (L.x) + L (R.x)].
   Chunk k adds into its own copy of y; the copies are added in chunk order. */
void orc_operator_apply(const orc_operator *op, const double *x, double *y) {
  const int64_t n = op->n > 0 ? op->n : 1;
  double *yt = (double *)calloc((size_t)op->nchunk * (size_t)n, sizeof(double));
#pragma omp parallel for schedule(static, 1)
  for (int64_t k = 0; k < op->nchunk; k++) {
    const orc_op_chunk *c = &op->c[k];
    double *yl = yt + (size_t)k * (size_t)n;
    int64_t e = 0;
    for (int64_t g = c->g0; g < c->g1; g++) {
      for (int i = 0; i < 3; i++) {
        const int64_t q = 6 * (g - c->g0) + 2 * i;
        const int nl = c->cnt[q], nr = c->cnt[q + 1];
        const int32_t *Li = c->id + e, *Ri = c->id + e + nl;
        const double *Lv = c->val + e, *Rv = c->val + e + nl;
        double lx = 0.0, rx = 0.0;
        for (int b = 0; b < nl; b++) lx += Lv[b] * x[Li[b]];
        for (int b = 0; b < nr; b++) rx += Rv[b] * x[Ri[b]];
        const double W = c->W[3 * (g - c->g0) + i];
        for (int a = 0; a < nr; a++) yl[Ri[a]] += W * (Rv[a] * lx);
        for (int a = 0; a < nl; a++) yl[Li[a]] += W * (Lv[a] * rx);
        e += nl + nr;
      }
    }
  }
  for (int64_t j = 0; j < op->n; j++) {
    double acc = 0.0;
    for (int64_t k = 0; k < op->nchunk; k++) acc += yt[(size_t)k * (size_t)n + j];
    y[j] = acc;
  }
  free(yt);
}

/* Diagonal of K from the stored vectors: K_jj = sum over (g, i) of
   2 W L(j) R(j) (the ids of each vector are ascending, so a merge finds the
   nodes on both sides). */
void orc_operator_diagonal(const orc_operator *op, double *d) {
  const int64_t n = op->n > 0 ? op->n : 1;
  double *dt = (double *)calloc((size_t)op->nchunk * (size_t)n, sizeof(double));
#pragma omp parallel for schedule(static, 1)
  for (int64_t k = 0; k < op->nchunk; k++) {
    const orc_op_chunk *c = &op->c[k];
    double *dl = dt + (size_t)k * (size_t)n;
    int64_t e = 0;
    for (int64_t g = c->g0; g < c->g1; g++) {
      for (int i = 0; i < 3; i++) {
        const int64_t q = 6 * (g - c->g0) + 2 * i;
        const int nl = c->cnt[q], nr = c->cnt[q + 1];
        const int32_t *Li = c->id + e, *Ri = c->id + e + nl;
        const double *Lv = c->val + e, *Rv = c->val + e + nl;
        const double W = c->W[3 * (g - c->g0) + i];
        int a = 0, b = 0;
        while (a < nl && b < nr) {
          if (Li[a] < Ri[b]) a++;
          else if (Ri[b] < Li[a]) b++;
          else { dl[Li[a]] += 2.0 * W * (Lv[a] * Rv[b]); a++; b++; }
        }
        e += nl + nr;
      }
    }
  }
  for (int64_t j = 0; j < op->n; j++) {
    double acc = 0.0;
    for (int64_t k = 0; k < op->nchunk; k++) acc += dt[(size_t)k * (size_t)n + j];
    d[j] = acc;
  }
  free(dt);
}

/* OpenMP threads of the parallel oracle loops (0 or less: leave unchanged);
   returns the number now in use. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Sums for the adjoint (lambda = K^{-1} dJ/du, K symmetric):
     S_i = sum_g w_g [(lam.R)(L.u) + (lam.L)(R.u)]
     T_i = sum_g w_g [(lam.R')(L.u) + (lam.R)(L'.u) + (lam.L')(R.u) + (lam.L)(R'.u)]
   with ' = d/dalpha.  Then dJ/dK_i = -c_alpha S_i and
   dJ/dalpha = -sum_i K_i (c'_alpha S_i + c_alpha T_i). */
int orc_adjoint_sums(const orc_mesh *m, int nq, double gamma, double inv_g2, double half_psi0,
                     int cap, const double *u, const double *lam, double *S /* 3 */, double *T /* 3 */) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  orc_order ord;
  orc_fill_order(&ord, gamma, inv_g2, 0.0, half_psi0);
  orc_work *w = orc_work_new(m->nv);
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int32_t *id = (int32_t *)malloc(sizeof(int32_t) * 4 * cap);
  double *v = (double *)malloc(sizeof(double) * 4 * cap);
  int st = ORC_OK;
  for (int i = 0; i < 3; i++) { S[i] = 0.0; T[i] = 0.0; }
  for (int64_t g = 0; g < m->nt * nq && st == ORC_OK; g++) {
    double wg = wq[g % nq] * m->vol[g / nq];
    for (int i = 0; i < 3; i++) {
      double d[2][2][2]; /* [side][value|alpha-derivative][dot with u | lam] */
      for (int side = 0; side < 2 && st == ORC_OK; side++) {
        for (int mode = 0; mode < 2; mode++) {
          int nn = orc_ray_vector(m, nq, bary, g, i, side, &ord, mode ? 2 : 0, cap, w, id, v, tb, rb);
          if (nn < 0) { st = nn; break; }
          double du = 0.0, dl = 0.0;
          for (int k = 0; k < nn; k++) { du += v[k] * u[id[k]]; dl += v[k] * lam[id[k]]; }
          d[side][mode][0] = du;
          d[side][mode][1] = dl;
        }
      }
      if (st != ORC_OK) break;
      /* side 0 = L, side 1 = R; mode 0 = value, 1 = d/dalpha */
      double lamR = d[1][0][1], Lu = d[0][0][0], lamL = d[0][0][1], Ru = d[1][0][0];
      double lamRp = d[1][1][1], Lpu = d[0][1][0], lamLp = d[0][1][1], Rpu = d[1][1][0];
      S[i] += wg * (lamR * Lu + lamL * Ru);
      T[i] += wg * (lamRp * Lu + lamR * Lpu + lamLp * Ru + lamL * Rpu);
    }
  }
  free(tb); free(rb); free(id); free(v); orc_work_free(w);
  return st;
}

/* Load vector b_j = sum_g w_g f(x_g) psi_j(x_g); f_gauss may be NULL (f = 1). */
int orc_load(const orc_mesh *m, int nq, const double *f_gauss, double *b) {
  double bary[44], wq[11];
  if (orc_quadrature(nq, bary, wq) != ORC_OK) return ORC_EINVAL;
  for (int64_t j = 0; j < m->ndof; j++) b[j] = 0.0;
  for (int64_t t = 0; t < m->nt; t++) {
    for (int q = 0; q < nq; q++) {
      int64_t g = t * nq + q;
      double f = f_gauss ? f_gauss[g] : 1.0;
      double wg = wq[q] * m->vol[t];
      for (int j = 0; j < 4; j++) {
        int32_t d = m->dof[m->tet[4 * t + j]];
        if (d >= 0) b[d] += wg * f * bary[q * 4 + j];
      }
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive line/element intersection, the method the path search          */
/* replaces (Sec. 2.2): every element is clipped against its four face       */
/* planes (outward normals from vertex cross products, no A^{-1}).            */
/* lo/hi receive the parameter interval along u0 + r d (r unrestricted), or */
/* lo > hi when the line misses the element.                                 */
/* ------------------------------------------------------------------------ */
void orc_exhaustive(const orc_mesh *m, const double *u0, const double *d, double *lo, double *hi) {
  static const int fv[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
  for (int64_t t = 0; t < m->nt; t++) {
    double a = -INFINITY, b = INFINITY;
    for (int f = 0; f < 4; f++) {
      const double *p0 = m->xyz + 3 * (int64_t)m->tet[4 * t + fv[f][0]];
      const double *p1 = m->xyz + 3 * (int64_t)m->tet[4 * t + fv[f][1]];
      const double *p2 = m->xyz + 3 * (int64_t)m->tet[4 * t + fv[f][2]];
      const double *po = m->xyz + 3 * (int64_t)m->tet[4 * t + f];
      double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
      double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
      double nrm[3] = {orc_cross_x(e1, e2), orc_cross_y(e1, e2), orc_cross_z(e1, e2)};
      double side = nrm[0] * (po[0] - p0[0]) + nrm[1] * (po[1] - p0[1]) + nrm[2] * (po[2] - p0[2]);
      if (side > 0) { nrm[0] = -nrm[0]; nrm[1] = -nrm[1]; nrm[2] = -nrm[2]; }
      /* inside: nrm.(u0 + r d - p0) <= 0 */
      double c0 = nrm[0] * (u0[0] - p0[0]) + nrm[1] * (u0[1] - p0[1]) + nrm[2] * (u0[2] - p0[2]);
      double c1 = nrm[0] * d[0] + nrm[1] * d[1] + nrm[2] * d[2];
      if (c1 == 0.0) {
        if (c0 > 0.0) { a = 1.0; b = 0.0; }
      } else if (c1 > 0.0) {
        double r = -c0 / c1;
        if (r < b) b = r;
      } else {
        double r = -c0 / c1;
        if (r > a) a = r;
      }
    }
    lo[t] = a;
    hi[t] = b;
  }
}

/* The walk from an arbitrary point u0 inside element t0 (test helper). */
int orc_walk_from(const orc_mesh *m, int64_t t0, const double *u0, int i, int s, int cap,
                  int32_t *tets, double *r_end, int *n_out) {
  return orc_walk(m, t0, u0, i, s, cap, tets, r_end, n_out);
}
