/*
 * Plain FP64 CPU oracle for the two-dimensional variant (n = 2) of the
 * method: P1 elements on a convex triangulated polygon, paths along +-e_1,
 * +-e_2 (Sec. 1 with n = 2, Fig. 1a; Sec. 2.2 with three area coordinates).
 *
 * TEST INFRASTRUCTURE ONLY, like fpde_oracle.c: loaded only by the tests,
 * the smoke check and the benchmark's CPU-baseline leg; it shares no code
 * with the GPU library (nor with the 3-D oracle: its helpers are its own).
 * FP64 throughout, no FMA contraction.
 *
 * What it computes:
 *   - per triangle A^{-1}, A = (v1 - v0, v2 - v0) (Sec. 2.2 in n = 2), its
 *     area, the neighbour across each edge (edge f opposite local vertex f),
 *     the interior numbering (vertices on no boundary edge, increasing id)
 *     and vertex -> triangle lists;
 *   - the path of a ray u0 + r s e_i: area coordinates b~ = (A^{-1}(u0 - v0),
 *     1 - sum), rates d~ = (s A^{-1} e_i, -sum), r_max = min over d~_j < 0 of
 *     -b~_j / d~_j; the zero pattern of b~ + r_max d~ names the go-out
 *     m-face: one zero = an edge (the triangle across it), two = a vertex
 *     (the smallest-id triangle containing it in which the ray advances);
 *   - the order-gamma derivatives of the P1 basis along the path in the same
 *     closed form as in 3-D (integration by parts of eq. def, m = 1);
 *   - the split Riesz stiffness matrix
 *       K_jk = c_alpha sum_i K_i sum_g w_g [L_gi(k) R_gi(j) + R_gi(k) L_gi(j)],
 *     i = 1, 2, and the load vector.
 * Readings (identical to the 3-D oracle's): a coordinate is zero when
 * |k_j| <= 1e-12 max(1, |b~_j|, |r_max d~_j|), the coordinate that set r_max
 * always counts as zero; after a vertex go-out the ray must advance by more
 * than 1e-12 r; the ray origin stays the Gauss point.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { O2_OK = 0, O2_EINVAL = -1, O2_ENONMANIFOLD = -2, O2_EDEGENERATE = -3, O2_EPATH = -5 };

typedef struct {
  int64_t nv, nt, ndof;
  double *xy;       /* nv*2 */
  int32_t *tri;     /* nt*3 */
  int32_t *nbr;     /* nt*3: across edge f (opposite local vertex f), -1 = boundary */
  double *M;        /* nt*4: A^{-1} row-major, row r = gradient of area coordinate k_{r+1} */
  double *area;     /* nt */
  int32_t *vt_off;  /* nv+1 */
  int32_t *vt_tri;  /* 3*nt, ascending triangle id per vertex */
  int32_t *dof;     /* nv */
} o2_mesh;

/* ------------------------------------------------------------------------ */
/* Quadrature on the reference triangle, barycentric points, weights sum 1: */
/* 3 points (degree 2): permutations of (2/3, 1/6, 1/6), weight 1/3;        */
/* 7 points (degree 5, Radon): the centroid (9/40), permutations of          */
/* (1 - 2a, a, a) with a = (6 - sqrt 15)/21 (weight (155 - sqrt 15)/1200) and */
/* with a = (6 + sqrt 15)/21 (weight (155 + sqrt 15)/1200).                  */
/* ------------------------------------------------------------------------ */
int o2_quadrature(int nq, double *bary /* nq*3 */, double *w /* nq */) {
  if (nq == 3) {
    for (int q = 0; q < 3; q++) {
      for (int j = 0; j < 3; j++) bary[3 * q + j] = (j == q) ? 2.0 / 3.0 : 1.0 / 6.0;
      w[q] = 1.0 / 3.0;
    }
    return O2_OK;
  }
  if (nq == 7) {
    const double r15 = sqrt(15.0);
    const double a[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
    const double wa[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
    for (int j = 0; j < 3; j++) bary[j] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    int q = 1;
    for (int o = 0; o < 2; o++) {
      for (int v = 0; v < 3; v++, q++) {
        for (int j = 0; j < 3; j++) bary[3 * q + j] = (j == v) ? 1.0 - 2.0 * a[o] : a[o];
        w[q] = wa[o];
      }
    }
    return O2_OK;
  }
  return O2_EINVAL;
}

typedef struct { int32_t a, b, t, f; } o2_edge;

static int o2_edge_cmp(const void *pa, const void *pb) {
  const o2_edge *x = (const o2_edge *)pa, *y = (const o2_edge *)pb;
  if (x->a != y->a) return x->a < y->a ? -1 : 1;
  if (x->b != y->b) return x->b < y->b ? -1 : 1;
  if (x->t != y->t) return x->t < y->t ? -1 : 1;
  return x->f - y->f;
}

void o2_mesh_free(o2_mesh *m) {
  if (!m) return;
  free(m->xy); free(m->tri); free(m->nbr); free(m->M); free(m->area);
  free(m->vt_off); free(m->vt_tri); free(m->dof);
  free(m);
}

o2_mesh *o2_mesh_create(const double *xy, int64_t nv, const int32_t *tri, int64_t nt, int *status) {
  *status = O2_OK;
  if (nv <= 0 || nt <= 0 || !xy || !tri) { *status = O2_EINVAL; return NULL; }
  for (int64_t k = 0; k < 3 * nt; k++)
    if (tri[k] < 0 || tri[k] >= nv) { *status = O2_EINVAL; return NULL; }
  o2_mesh *m = (o2_mesh *)calloc(1, sizeof(o2_mesh));
  m->nv = nv; m->nt = nt;
  m->xy = (double *)malloc(sizeof(double) * 2 * nv);
  m->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
  m->nbr = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
  m->M = (double *)malloc(sizeof(double) * 4 * nt);
  m->area = (double *)malloc(sizeof(double) * nt);
  m->vt_off = (int32_t *)calloc(nv + 1, sizeof(int32_t));
  m->vt_tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
  m->dof = (int32_t *)malloc(sizeof(int32_t) * nv);
  memcpy(m->xy, xy, sizeof(double) * 2 * nv);
  memcpy(m->tri, tri, sizeof(int32_t) * 3 * nt);
  /* A^{-1} by the adjugate: (1/det) [[e2y, -e2x], [-e1y, e1x]] */
  for (int64_t t = 0; t < nt; t++) {
    const double *v0 = xy + 2 * (int64_t)tri[3 * t];
    const double *v1 = xy + 2 * (int64_t)tri[3 * t + 1];
    const double *v2 = xy + 2 * (int64_t)tri[3 * t + 2];
    double e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e2x = v2[0] - v0[0], e2y = v2[1] - v0[1];
    double det = e1x * e2y - e2x * e1y;
    double l1 = sqrt(e1x * e1x + e1y * e1y), l2 = sqrt(e2x * e2x + e2y * e2y);
    double L = l1 > l2 ? l1 : l2;
    if (!(fabs(det) > 1e-13 * L * L)) { *status = O2_EDEGENERATE; o2_mesh_free(m); return NULL; }
    double *Mt = m->M + 4 * t;
    Mt[0] = e2y / det;
    Mt[1] = -e2x / det;
    Mt[2] = -e1y / det;
    Mt[3] = e1x / det;
    m->area[t] = fabs(det) / 2.0;
  }
  /* edge matching: edge f of triangle t is opposite local vertex f */
  o2_edge *E = (o2_edge *)malloc(sizeof(o2_edge) * 3 * nt);
  for (int64_t t = 0; t < nt; t++)
    for (int f = 0; f < 3; f++) {
      int32_t p = tri[3 * t + (f + 1) % 3], q = tri[3 * t + (f + 2) % 3];
      if (p == q) { free(E); *status = O2_EDEGENERATE; o2_mesh_free(m); return NULL; }
      o2_edge *x = &E[3 * t + f];
      x->a = p < q ? p : q;
      x->b = p < q ? q : p;
      x->t = (int32_t)t;
      x->f = f;
      m->nbr[3 * t + f] = -1;
    }
  qsort(E, 3 * nt, sizeof(o2_edge), o2_edge_cmp);
  for (int64_t a = 0; a < 3 * nt;) {
    int64_t b = a + 1;
    while (b < 3 * nt && E[b].a == E[a].a && E[b].b == E[a].b) b++;
    if (b - a > 2) { free(E); *status = O2_ENONMANIFOLD; o2_mesh_free(m); return NULL; }
    if (b - a == 2) {
      m->nbr[3 * E[a].t + E[a].f] = E[a + 1].t;
      m->nbr[3 * E[a + 1].t + E[a + 1].f] = E[a].t;
    }
    a = b;
  }
  free(E);
  char *bnd = (char *)calloc(nv, 1), *used = (char *)calloc(nv, 1);
  for (int64_t t = 0; t < nt; t++) {
    for (int j = 0; j < 3; j++) used[tri[3 * t + j]] = 1;
    for (int f = 0; f < 3; f++)
      if (m->nbr[3 * t + f] < 0) {
        bnd[tri[3 * t + (f + 1) % 3]] = 1;
        bnd[tri[3 * t + (f + 2) % 3]] = 1;
      }
  }
  m->ndof = 0;
  for (int64_t v = 0; v < nv; v++) m->dof[v] = (used[v] && !bnd[v]) ? (int32_t)(m->ndof++) : -1;
  free(bnd); free(used);
  for (int64_t k = 0; k < 3 * nt; k++) m->vt_off[tri[k] + 1]++;
  for (int64_t v = 0; v < nv; v++) m->vt_off[v + 1] += m->vt_off[v];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * nv);
  for (int64_t v = 0; v < nv; v++) fill[v] = m->vt_off[v];
  for (int64_t t = 0; t < nt; t++)
    for (int j = 0; j < 3; j++) m->vt_tri[fill[tri[3 * t + j]]++] = (int32_t)t;
  free(fill);
  return m;
}

int64_t o2_mesh_ndof(const o2_mesh *m) { return m->ndof; }
void o2_mesh_dof(const o2_mesh *m, int32_t *out) { memcpy(out, m->dof, sizeof(int32_t) * m->nv); }
void o2_mesh_nbr(const o2_mesh *m, int32_t *out) { memcpy(out, m->nbr, sizeof(int32_t) * 3 * m->nt); }
void o2_mesh_affine(const o2_mesh *m, double *M, double *area) {
  memcpy(M, m->M, sizeof(double) * 4 * m->nt);
  memcpy(area, m->area, sizeof(double) * m->nt);
}

/* Gauss point g = triangle * nq + q: x_g = ((0 + b0 v0) + b1 v1) + b2 v2 */
static void o2_origin(const o2_mesh *m, int nq, const double *bary, int64_t g, double *u0) {
  int64_t t = g / nq;
  int q = (int)(g % nq);
  for (int d = 0; d < 2; d++) {
    double s = 0.0;
    for (int j = 0; j < 3; j++) s = s + bary[3 * q + j] * m->xy[2 * (int64_t)m->tri[3 * t + j] + d];
    u0[d] = s;
  }
}

int o2_gauss_points(const o2_mesh *m, int nq, double *x /* G*2 */, double *w /* G */) {
  double bary[21], wq[7];
  if (o2_quadrature(nq, bary, wq) != O2_OK) return O2_EINVAL;
  for (int64_t g = 0; g < m->nt * nq; g++) {
    o2_origin(m, nq, bary, g, x + 2 * g);
    w[g] = wq[g % nq] * m->area[g / nq];
  }
  return O2_OK;
}

typedef struct {
  double bt[3], dt[3], kmax[3];
  double r_max;
  int jexit;
} o2_isect;

static void o2_intersect(const o2_mesh *m, int64_t t, const double *u0, int i, int s, o2_isect *o) {
  const double *Mt = m->M + 4 * t;
  const double *v0 = m->xy + 2 * (int64_t)m->tri[3 * t];
  double b0 = u0[0] - v0[0], b1 = u0[1] - v0[1];
  for (int r = 0; r < 2; r++) {
    o->bt[r + 1] = Mt[2 * r] * b0 + Mt[2 * r + 1] * b1;
    o->dt[r + 1] = (s > 0) ? Mt[2 * r + i] : -Mt[2 * r + i];
  }
  o->bt[0] = 1.0 - (o->bt[1] + o->bt[2]);
  o->dt[0] = -(o->dt[1] + o->dt[2]);
  o->r_max = INFINITY;
  o->jexit = -1;
  for (int j = 0; j < 3; j++)
    if (o->dt[j] < 0.0) {
      double r = -o->bt[j] / o->dt[j];
      if (r < o->r_max) { o->r_max = r; o->jexit = j; }
    }
  for (int j = 0; j < 3; j++) o->kmax[j] = o->bt[j] + o->r_max * o->dt[j];
}

static int o2_is_zero(const o2_isect *o, int j) {
  if (j == o->jexit) return 1;
  double s = fabs(o->bt[j]), p = fabs(o->r_max * o->dt[j]);
  if (p > s) s = p;
  if (s < 1.0) s = 1.0;
  return fabs(o->kmax[j]) <= 1e-12 * s;
}

int o2_walk(const o2_mesh *m, int64_t t0, const double *u0, int i, int s, int cap, int32_t *tris, double *r_end,
            int *n_out) {
  int64_t t = t0;
  double r_cur = 0.0;
  int n = 0;
  for (int step = 0; step < cap + 64; step++) {
    o2_isect o;
    o2_intersect(m, t, u0, i, s, &o);
    if (!(o.r_max < INFINITY)) return O2_EPATH;
    if (o.r_max > r_cur) {
      if (n >= cap) return O2_EPATH;
      tris[n] = (int32_t)t;
      r_end[n] = o.r_max;
      n++;
      r_cur = o.r_max;
    }
    int Z[3], nz = 0;
    for (int j = 0; j < 3; j++) if (o2_is_zero(&o, j)) Z[nz++] = j;
    if (nz == 0 || nz == 3) return O2_EPATH;
    if (nz == 1) {
      int32_t nx = m->nbr[3 * t + Z[0]];
      if (nx < 0) { *n_out = n; return O2_OK; }
      t = nx;
      continue;
    }
    /* vertex go-out: the vertex whose coordinate is not zero */
    int keep = 0;
    for (int j = 0; j < 3; j++) if (j != Z[0] && j != Z[1]) keep = j;
    int32_t v = m->tri[3 * t + keep];
    int64_t best = -1;
    for (int32_t p = m->vt_off[v]; p < m->vt_off[v + 1]; p++) {
      int64_t c = m->vt_tri[p];
      if (c == t) continue;
      o2_isect oc;
      o2_intersect(m, c, u0, i, s, &oc);
      if (oc.r_max - r_cur > 1e-12 * r_cur) { best = c; break; }
    }
    if (best < 0) { *n_out = n; return O2_OK; }
    t = best;
  }
  return O2_EPATH;
}

static uint64_t o2_fnv1a(const int32_t *ids, int n) {
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

/* half-ray h = g * 4 + 2 i + side (side 0: -e_i, side 1: +e_i) */
int o2_paths(const o2_mesh *m, int nq, int64_t h0, int64_t count, int cap, int32_t *len, uint64_t *hash,
             int32_t *ids, double *rend) {
  double bary[21], wq[7];
  if (o2_quadrature(nq, bary, wq) != O2_OK) return O2_EINVAL;
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int st = O2_OK;
  for (int64_t k = 0; k < count && st == O2_OK; k++) {
    int64_t h = h0 + k, g = h / 4;
    int dir = (int)(h % 4), i = dir / 2, s = (dir & 1) ? 1 : -1;
    double u0[2];
    o2_origin(m, nq, bary, g, u0);
    int n = 0;
    st = o2_walk(m, g / nq, u0, i, s, cap, tb, rb, &n);
    if (st != O2_OK) break;
    len[k] = n;
    hash[k] = o2_fnv1a(tb, n);
    if (ids) for (int j = 0; j < n; j++) ids[k * cap + j] = tb[j];
    if (rend) for (int j = 0; j < n; j++) rend[k * cap + j] = rb[j];
  }
  free(tb); free(rb);
  return st;
}

int o2_walk_from(const o2_mesh *m, int64_t t0, const double *u0, int i, int s, int cap, int32_t *tris,
                 double *r_end, int *n_out) {
  return o2_walk(m, t0, u0, i, s, cap, tris, r_end, n_out);
}

/* slope of area coordinate j along e_i on triangle t */
static double o2_slope(const o2_mesh *m, int64_t t, int j, int i) {
  const double *Mt = m->M + 4 * t;
  if (j > 0) return Mt[2 * (j - 1) + i];
  return -(Mt[i] + Mt[2 + i]);
}

static double o2_pow(double r, double e) { return r > 0.0 ? pow(r, e) : 0.0; }

/* Sparse vector of D^gamma psi_l(x_g) along e_i, side 0 left / 1 right.
   mode 0: interior dofs; mode 1: all vertices with the end-point term
   psi_l(p_end) r_end^{-gamma} / Gamma(1 - gamma).  ids ascending.
   acc/mark: nv scratch, zero on entry and on exit. */
static int o2_vector(const o2_mesh *m, int nq, const double *bary, int64_t g, int i, int side, double gamma,
                     double inv_g2, double inv_g1, int mode, int cap, double *acc, char *mark, int32_t *touched,
                     int32_t *out_id, double *out_val) {
  double u0[2];
  o2_origin(m, nq, bary, g, u0);
  int s = side ? 1 : -1;
  int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * cap);
  double *rb = (double *)malloc(sizeof(double) * cap);
  int n = 0;
  int st = o2_walk(m, g / nq, u0, i, s, cap, tb, rb, &n);
  if (st != O2_OK) { free(tb); free(rb); return st; }
  double e = 1.0 - gamma, sgn = side ? -1.0 : 1.0, r_lo = 0.0;
  int nt_ = 0;
  for (int k = 0; k < n; k++) {
    int64_t t = tb[k];
    double dP = inv_g2 * (o2_pow(rb[k], e) - o2_pow(r_lo, e));
    for (int j = 0; j < 3; j++) {
      int32_t v = m->tri[3 * t + j];
      if (mode == 0 && m->dof[v] < 0) continue;
      if (!mark[v]) { mark[v] = 1; touched[nt_++] = v; }
      acc[v] += sgn * o2_slope(m, t, j, i) * dP;
    }
    r_lo = rb[k];
  }
  if (mode == 1 && n > 0) {
    o2_isect o;
    int64_t t = tb[n - 1];
    o2_intersect(m, t, u0, i, s, &o);
    double c = inv_g1 * pow(rb[n - 1], -gamma);
    for (int j = 0; j < 3; j++) {
      if (o.kmax[j] == 0.0) continue;
      int32_t v = m->tri[3 * t + j];
      if (!mark[v]) { mark[v] = 1; touched[nt_++] = v; }
      acc[v] += o.kmax[j] * c;
    }
  }
  /* ascending ids (insertion sort: a vector has a few dozen entries) */
  for (int a = 1; a < nt_; a++) {
    int32_t x = touched[a];
    int b = a - 1;
    while (b >= 0 && touched[b] > x) { touched[b + 1] = touched[b]; b--; }
    touched[b + 1] = x;
  }
  for (int k = 0; k < nt_; k++) {
    int32_t v = touched[k];
    out_id[k] = mode == 1 ? v : m->dof[v];
    out_val[k] = acc[v];
    acc[v] = 0.0;
    mark[v] = 0;
  }
  free(tb); free(rb);
  return nt_;
}

int o2_ray_values(const o2_mesh *m, int nq, int64_t g, int i, int side, double gamma, double inv_g2,
                  double inv_g1, int mode, int cap, int32_t *out_id, double *out_val) {
  double bary[21], wq[7];
  if (o2_quadrature(nq, bary, wq) != O2_OK) return O2_EINVAL;
  double *acc = (double *)calloc(m->nv, sizeof(double));
  char *mark = (char *)calloc(m->nv, 1);
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * m->nv);
  int r = o2_vector(m, nq, bary, g, i, side, gamma, inv_g2, inv_g1, mode, cap, acc, mark, touched, out_id,
                    out_val);
  free(acc); free(mark); free(touched);
  return r;
}

/* K_jk = c_alpha sum_i K_i sum_g w_g [L(k) R(j) + R(k) L(j)]; A zeroed by the caller */
int o2_assemble(const o2_mesh *m, int nq, double gamma, double inv_g2, double c_alpha, const double *Kc, int cap,
                double *A) {
  double bary[21], wq[7];
  if (o2_quadrature(nq, bary, wq) != O2_OK) return O2_EINVAL;
  double *acc = (double *)calloc(m->nv, sizeof(double));
  char *mark = (char *)calloc(m->nv, 1);
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * m->nv);
  int32_t *Li = (int32_t *)malloc(sizeof(int32_t) * 3 * cap), *Ri = (int32_t *)malloc(sizeof(int32_t) * 3 * cap);
  double *Lv = (double *)malloc(sizeof(double) * 3 * cap), *Rv = (double *)malloc(sizeof(double) * 3 * cap);
  int64_t n = m->ndof;
  int st = O2_OK;
  for (int64_t g = 0; g < m->nt * nq && st == O2_OK; g++) {
    double wg = wq[g % nq] * m->area[g / nq];
    for (int i = 0; i < 2; i++) {
      int nl = o2_vector(m, nq, bary, g, i, 0, gamma, inv_g2, 0.0, 0, cap, acc, mark, touched, Li, Lv);
      if (nl < 0) { st = nl; break; }
      int nr = o2_vector(m, nq, bary, g, i, 1, gamma, inv_g2, 0.0, 0, cap, acc, mark, touched, Ri, Rv);
      if (nr < 0) { st = nr; break; }
      double W = wg * Kc[i] * c_alpha;
      for (int a = 0; a < nr; a++)
        for (int b = 0; b < nl; b++) A[Ri[a] * n + Li[b]] += W * (Rv[a] * Lv[b]);
      for (int a = 0; a < nl; a++)
        for (int b = 0; b < nr; b++) A[Li[a] * n + Ri[b]] += W * (Lv[a] * Rv[b]);
    }
  }
  free(acc); free(mark); free(touched); free(Li); free(Ri); free(Lv); free(Rv);
  return st;
}

/* b_j = sum_g w_g f(x_g) psi_j(x_g); f_gauss may be NULL (f = 1) */
int o2_load(const o2_mesh *m, int nq, const double *f_gauss, double *b) {
  double bary[21], wq[7];
  if (o2_quadrature(nq, bary, wq) != O2_OK) return O2_EINVAL;
  for (int64_t j = 0; j < m->ndof; j++) b[j] = 0.0;
  for (int64_t t = 0; t < m->nt; t++)
    for (int q = 0; q < nq; q++) {
      double f = f_gauss ? f_gauss[t * nq + q] : 1.0;
      double wg = wq[q] * m->area[t];
      for (int j = 0; j < 3; j++) {
        int32_t d = m->dof[m->tri[3 * t + j]];
        if (d >= 0) b[d] += wg * f * bary[3 * q + j];
      }
    }
  return O2_OK;
}

/* exhaustive clipping of the line u0 + r d against every triangle (the
   search the walk replaces): parameter interval [lo, hi], lo > hi if missed */
void o2_exhaustive(const o2_mesh *m, const double *u0, const double *d, double *lo, double *hi) {
  for (int64_t t = 0; t < m->nt; t++) {
    double a = -INFINITY, b = INFINITY;
    for (int f = 0; f < 3; f++) {
      const double *p = m->xy + 2 * (int64_t)m->tri[3 * t + (f + 1) % 3];
      const double *q = m->xy + 2 * (int64_t)m->tri[3 * t + (f + 2) % 3];
      const double *o = m->xy + 2 * (int64_t)m->tri[3 * t + f];
      double nx = q[1] - p[1], ny = -(q[0] - p[0]);
      if (nx * (o[0] - p[0]) + ny * (o[1] - p[1]) > 0) { nx = -nx; ny = -ny; }
      double c0 = nx * (u0[0] - p[0]) + ny * (u0[1] - p[1]);
      double c1 = nx * d[0] + ny * d[1];
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
