// Mesh set-up on the device: per-element affine data, face adjacency,
// boundary detection, interior numbering and vertex -> element lists.
//
// The walk of Sec. 2.2 needs A^{-1} of every element (volume coordinates
// k = A^{-1}(x - v0)), the element across each face ("adjacent information
// of the triangulation") and, for edge/vertex go-out points, the elements
// that contain a given m-face (found through vertex -> element lists).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

// ---------------------------------------------------------------------------
// Quadrature (Sec. 2.1 uses Gaussian quadrature on each element without
// naming the rule): degree-2 4-point rule and the degree-4 11-point rule of
// Keast (centroid with a negative weight, a 4-orbit and a 6-orbit).
// ---------------------------------------------------------------------------
int quad_rule(int nq, QuadRule *r) {
  std::memset(r, 0, sizeof(*r));
  r->nq = nq;
  if (nq == 4) {
    const double a = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0;
    const double b = (5.0 - std::sqrt(5.0)) / 20.0;
    for (int q = 0; q < 4; q++) {
      for (int j = 0; j < 4; j++) r->bary[q][j] = (j == q) ? a : b;
      r->w[q] = 0.25;
    }
    return FPDE_OK;
  }
  if (nq == 11) {
    for (int j = 0; j < 4; j++) r->bary[0][j] = 0.25;
    r->w[0] = -148.0 / 1875.0;
    for (int v = 0; v < 4; v++) {
      for (int j = 0; j < 4; j++) r->bary[1 + v][j] = (j == v) ? 11.0 / 14.0 : 1.0 / 14.0;
      r->w[1 + v] = 343.0 / 7500.0;
    }
    const double a = (1.0 + std::sqrt(5.0 / 14.0)) / 4.0;
    const double b = (1.0 - std::sqrt(5.0 / 14.0)) / 4.0;
    const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int p = 0; p < 6; p++) {
      for (int j = 0; j < 4; j++) r->bary[5 + p][j] = b;
      r->bary[5 + p][pr[p][0]] = a;
      r->bary[5 + p][pr[p][1]] = a;
      r->w[5 + p] = 56.0 / 375.0;
    }
    return FPDE_OK;
  }
  return FPDE_EINVAL;
}

// digamma by upward recurrence to x >= 10 and the asymptotic series
// psi(x) ~ ln x - 1/(2x) - sum_k B_2k / (2k x^2k)
static double digamma(double x) {
  double acc = 0.0;
  while (x < 10.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double x2 = 1.0 / (x * x);
  double s = x2 * (1.0 / 12.0 -
              x2 * (1.0 / 120.0 -
              x2 * (1.0 / 252.0 -
              x2 * (1.0 / 240.0 -
              x2 * (1.0 / 132.0 -
              x2 * (691.0 / 32760.0 -
              x2 * (1.0 / 12.0)))))));
  return acc + std::log(x) - 0.5 / x - s;
}

Order order_scalars(double alpha) {
  Order o;
  o.gamma = 0.5 * alpha;
  o.e = 1.0 - o.gamma;
  o.inv_g2 = 1.0 / std::tgamma(2.0 - o.gamma);
  o.half_psi0 = 0.5 * digamma(2.0 - o.gamma);
  const double c = std::cos(M_PI * alpha / 2.0);
  o.c_alpha = 1.0 / (2.0 * c);
  o.dc_alpha = (M_PI / 4.0) * std::sin(M_PI * alpha / 2.0) / (c * c);
  return o;
}

int check_params(const fpde_mesh *m, const fpde_params *p) {
  if (!m || !p) return FPDE_EINVAL;
  if (!(p->alpha > 1.0 && p->alpha <= 2.0)) return FPDE_EALPHA;
  for (int i = 0; i < 3; i++)
    if (!(p->K[i] > 0.0) || !std::isfinite(p->K[i])) return FPDE_EALPHA;
  if (p->quad_points != 4 && p->quad_points != 11) return FPDE_EINVAL;
  if (p->precision != FPDE_FP64 && p->precision != FPDE_MIXED) return FPDE_EINVAL;
  if (p->source < FPDE_SRC_ONE || p->source > FPDE_SRC_CUBE_MMS) return FPDE_EINVAL;
  if (p->max_steps < 0) return FPDE_EINVAL;
  return FPDE_OK;
}

// The status word and the failure detail share one 16-byte device block,
// read back with one transfer into pinned host memory.
static int alloc_flags(fpde_mesh *m) {
  FPDE_TRY(dalloc(&m->flag_blk, 2));
  m->flag = reinterpret_cast<int32_t *>(m->flag_blk);
  m->flag_aux = m->flag_blk + 1;
  if (hipHostMalloc((void **)&m->hflag, 2 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    m->hflag = nullptr;
    return FPDE_ENOMEM;
  }
  return FPDE_OK;
}

int take_flag(fpde_mesh *m, hipStream_t s, int64_t *aux) {
  int32_t f = 0;
  int64_t a = -1;
  FPDE_HIP(hipMemcpyAsync(m->hflag, m->flag_blk, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipStreamSynchronize(s));
  std::memcpy(&f, m->hflag, sizeof(f));
  a = m->hflag[1];
  if (f != 0) {
    int32_t z = 0;
    int64_t mz = -1;
    FPDE_HIP(hipMemcpyAsync(m->flag, &z, sizeof(z), hipMemcpyHostToDevice, s));
    FPDE_HIP(hipMemcpyAsync(m->flag_aux, &mz, sizeof(mz), hipMemcpyHostToDevice, s));
    FPDE_HIP(hipStreamSynchronize(s));
  }
  if (aux) *aux = a;
  return f;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_affine(const double *__restrict__ xyz, const int32_t *__restrict__ tet, int64_t nt,
                         TetRec *__restrict__ rec, double *__restrict__ vol, int32_t *flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t v[4];
  for (int j = 0; j < 4; j++) v[j] = tet[4 * t + j];
  const double *p0 = xyz + 3 * (int64_t)v[0];
  double e[3][3];
  for (int c = 0; c < 3; c++) {
    const double *pc = xyz + 3 * (int64_t)v[c + 1];
    for (int d = 0; d < 3; d++) e[c][d] = pc[d] - p0[d];
  }
  // rows of A^{-1} = (e2 x e3, e3 x e1, e1 x e2) / det(e1, e2, e3)
  double r[3][3];
  const int a_[3] = {1, 2, 0}, b_[3] = {2, 0, 1};
  for (int k = 0; k < 3; k++) {
    const double *A = e[a_[k]], *B = e[b_[k]];
    r[k][0] = A[1] * B[2] - A[2] * B[1];
    r[k][1] = A[2] * B[0] - A[0] * B[2];
    r[k][2] = A[0] * B[1] - A[1] * B[0];
  }
  double det = e[0][0] * r[0][0] + e[0][1] * r[0][1] + e[0][2] * r[0][2];
  double L = 0.0;
  for (int c = 0; c < 3; c++) {
    double l = sqrt(e[c][0] * e[c][0] + e[c][1] * e[c][1] + e[c][2] * e[c][2]);
    L = l > L ? l : L;
  }
  bool rep = v[0] == v[1] || v[0] == v[2] || v[0] == v[3] || v[1] == v[2] || v[1] == v[3] || v[2] == v[3];
  if (rep || !(fabs(det) > 1e-13 * L * L * L)) {
    set_flag(flag, FPDE_EMESH_DEGENERATE);
    return;
  }
  TetRec R;
  for (int k = 0; k < 3; k++)
    for (int d = 0; d < 3; d++) R.M[3 * k + d] = r[k][d] / det;
  for (int d = 0; d < 3; d++) R.v0[d] = p0[d];
  for (int j = 0; j < 4; j++) {
    R.nbr[j] = -1;
    R.dof[j] = -1;
  }
  rec[t] = R;
  vol[t] = fabs(det) / 6.0;
}

// face f of element t (opposite local vertex f) -> sorted vertex triple key
__global__ void k_face_keys(const int32_t *__restrict__ tet, int64_t nt, uint64_t *__restrict__ key,
                            int32_t *__restrict__ val) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * nt) return;
  int64_t t = k >> 2;
  int f = (int)(k & 3);
  uint32_t a[3];
  int n = 0;
  for (int j = 0; j < 4; j++)
    if (j != f) a[n++] = (uint32_t)tet[4 * t + j];
  uint32_t x;
  if (a[0] > a[1]) { x = a[0]; a[0] = a[1]; a[1] = x; }
  if (a[1] > a[2]) { x = a[1]; a[1] = a[2]; a[2] = x; }
  if (a[0] > a[1]) { x = a[0]; a[0] = a[1]; a[1] = x; }
  key[k] = ((uint64_t)a[0] << 42) | ((uint64_t)a[1] << 21) | (uint64_t)a[2];
  val[k] = (int32_t)k;
}

__global__ void k_face_match(const uint64_t *__restrict__ key, const int32_t *__restrict__ val, int64_t n,
                             int32_t *__restrict__ nbr4, int32_t *flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (p > 0 && key[p - 1] == key[p]) return;  // not the first of its run
  if (p + 1 < n && key[p + 1] == key[p]) {
    if (p + 2 < n && key[p + 2] == key[p]) {
      set_flag(flag, FPDE_EMESH_NONMANIFOLD);
      return;
    }
    int32_t a = val[p], b = val[p + 1];
    nbr4[a] = b >> 2;
    nbr4[b] = a >> 2;
  }
}

__global__ void k_boundary(const int32_t *__restrict__ tet, const int32_t *__restrict__ nbr4, int64_t nt,
                           int32_t *__restrict__ used, int32_t *__restrict__ bnd,
                           unsigned long long *__restrict__ nbf) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * nt) return;
  int64_t t = k >> 2;
  int f = (int)(k & 3);
  used[tet[k]] = 1;
  if (nbr4[k] < 0) {
    for (int j = 0; j < 4; j++)
      if (j != f) bnd[tet[4 * t + j]] = 1;
    atomicAdd(nbf, 1ull);
  }
}

// Convexity of the domain (the chord bounds a_i(x), b_i(x) of Sec. 1 eq. (1)
// assume a convex domain).  A polyhedron is convex exactly when every one of
// its vertices lies on the inner side of the plane of every boundary face.
// Plane of boundary face f of element t: unit normal pointing away from the
// element's opposite vertex f, offset n . p0.
__global__ void k_bface_planes(const double *__restrict__ xyz, const int32_t *__restrict__ tet,
                               const int32_t *__restrict__ nbr4, int64_t nt, double4 *__restrict__ planes,
                               unsigned long long *__restrict__ count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * nt || nbr4[k] >= 0) return;
  const int64_t t = k >> 2;
  const int f = (int)(k & 3);
  double p[3][3];
  int n = 0;
  for (int j = 0; j < 4; j++) {
    if (j == f) continue;
    for (int d = 0; d < 3; d++) p[n][d] = xyz[3 * (int64_t)tet[4 * t + j] + d];
    n++;
  }
  const double *q = xyz + 3 * (int64_t)tet[4 * t + f];
  double a[3], b[3];
  for (int d = 0; d < 3; d++) {
    a[d] = p[1][d] - p[0][d];
    b[d] = p[2][d] - p[0][d];
  }
  double nx = a[1] * b[2] - a[2] * b[1];
  double ny = a[2] * b[0] - a[0] * b[2];
  double nz = a[0] * b[1] - a[1] * b[0];
  const double len = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= len;
  ny /= len;
  nz /= len;
  if (nx * (q[0] - p[0][0]) + ny * (q[1] - p[0][1]) + nz * (q[2] - p[0][2]) > 0.0) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  const unsigned long long slot = atomicAdd(count, 1ull);
  planes[slot] = make_double4(nx, ny, nz, nx * p[0][0] + ny * p[0][1] + nz * p[0][2]);
}

// every used vertex against every boundary plane, planes staged through LDS
// 256 at a time; a vertex more than tol outside a plane marks the mesh
// non-convex (aux = that vertex)
__global__ void __launch_bounds__(256) k_convex(const double *__restrict__ xyz, const int32_t *__restrict__ used,
                                                int64_t nv, const double4 *__restrict__ planes,
                                                const unsigned long long *__restrict__ count, double tol,
                                                int32_t *flag, int64_t *flag_aux) {
  __shared__ double4 pl[256];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = v < nv && used[v];
  double x = 0.0, y = 0.0, z = 0.0;
  if (live) {
    x = xyz[3 * v];
    y = xyz[3 * v + 1];
    z = xyz[3 * v + 2];
  }
  const int64_t nb = (int64_t)*count;
  bool out = false;
  for (int64_t c0 = 0; c0 < nb; c0 += 256) {
    __syncthreads();
    if (c0 + threadIdx.x < nb) pl[threadIdx.x] = planes[c0 + threadIdx.x];
    __syncthreads();
    const int cn = (int)(nb - c0 < 256 ? nb - c0 : 256);
    for (int c = 0; c < cn; c++) {
      const double4 P = pl[c];
      out |= (P.x * x + P.y * y + P.z * z) - P.w > tol;
    }
  }
  if (live && out) {
    set_flag(flag, FPDE_EMESH_NONCONVEX);
    atomicCAS((unsigned long long *)flag_aux, ~0ull, (unsigned long long)v);
  }
}

__global__ void k_isdof(const int32_t *__restrict__ used, const int32_t *__restrict__ bnd, int64_t nv,
                        int32_t *__restrict__ isdof) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  isdof[v] = (used[v] && !bnd[v]) ? 1 : 0;
}

__global__ void k_dof(const int32_t *__restrict__ isdof, const int32_t *__restrict__ scan, int64_t nv,
                      int32_t *__restrict__ dof, int32_t *__restrict__ vert_of_dof) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  if (isdof[v]) {
    dof[v] = scan[v];
    vert_of_dof[scan[v]] = (int32_t)v;
  } else {
    dof[v] = -1;
  }
}

__global__ void k_finalize(const int32_t *__restrict__ tet, const int32_t *__restrict__ nbr4,
                           const int32_t *__restrict__ dof, int64_t nt, TetRec *__restrict__ rec) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  for (int j = 0; j < 4; j++) {
    rec[t].nbr[j] = nbr4[4 * t + j];
    rec[t].dof[j] = dof[tet[4 * t + j]];
  }
}

__global__ void k_vt_keys(const int32_t *__restrict__ tet, int64_t nt, uint32_t *__restrict__ key,
                          int32_t *__restrict__ val, int32_t *__restrict__ count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * nt) return;
  key[k] = (uint32_t)tet[k];
  val[k] = (int32_t)(k >> 2);
  atomicAdd(&count[tet[k]], 1);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

}  // namespace fpde

using namespace fpde;

extern "C" const char *fpde_status_string(int s) {
  switch (s) {
    case FPDE_OK: return "ok";
    case FPDE_EINVAL: return "invalid argument";
    case FPDE_EMESH_NONMANIFOLD: return "non-manifold mesh: a face is shared by more than two elements";
    case FPDE_EMESH_DEGENERATE: return "degenerate element (zero volume or repeated vertex)";
    case FPDE_EMESH_NONCONVEX: return "non-convex domain: a vertex lies outside the plane of a boundary face";
    case FPDE_EPATH: return "integration path: no continuation found or max_steps exceeded";
    case FPDE_EALPHA: return "alpha outside (1, 2] or a coefficient K_i <= 0";
    case FPDE_ENOTSPD: return "Cholesky pivot <= 0: matrix not positive definite";
    case FPDE_ENOCONV: return "iterative refinement did not reach its tolerance";
    case FPDE_EHIP: return "HIP runtime error";
    case FPDE_ENOMEM: return "device allocation failed";
    case FPDE_EUNSUPPORTED: return "unsupported combination";
    case FPDE_ESINGULAR: return "LU without pivoting met a zero or non-finite pivot";
    default: return "unknown status";
  }
}

static int mesh_build(fpde_mesh *m, const double *xyz, const int32_t *tet, double convex_tol, hipStream_t s) {
  const int64_t nv = m->nv, nt = m->nt, nf = 4 * nt;
  FPDE_HIP(hipGetDevice(&m->device));
  FPDE_TRY(dalloc(&m->xyz, 3 * nv));
  FPDE_TRY(dalloc(&m->tet, 4 * nt));
  FPDE_TRY(dalloc(&m->rec, nt));
  FPDE_TRY(dalloc(&m->vol, nt));
  FPDE_TRY(dalloc(&m->vt_off, nv + 1));
  FPDE_TRY(dalloc(&m->vt_tet, nf));
  FPDE_TRY(dalloc(&m->dof, nv));
  FPDE_TRY(alloc_flags(m));
  {
    double tab[4 * 5 + 11 * 5];
    for (int nq : {4, 11}) {
      QuadRule r;
      FPDE_TRY(quad_rule(nq, &r));
      double *o = tab + rule_offset(nq);
      for (int q = 0; q < nq; q++) {
        for (int j = 0; j < 4; j++) o[4 * q + j] = r.bary[q][j];
        o[4 * nq + q] = r.w[q];
      }
    }
    FPDE_TRY(dalloc(&m->rules, sizeof(tab) / sizeof(double)));
    FPDE_HIP(hipMemcpyAsync(m->rules, tab, sizeof(tab), hipMemcpyHostToDevice, s));
  }
  FPDE_HIP(hipMemsetAsync(m->flag, 0, sizeof(int32_t), s));
  FPDE_HIP(hipMemsetAsync(m->flag_aux, 0xff, sizeof(int64_t), s));
  FPDE_HIP(hipMemcpyAsync(m->xyz, xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s));
  FPDE_HIP(hipMemcpyAsync(m->tet, tet, sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, s));

  k_affine<<<nblk(nt), 256, 0, s>>>(m->xyz, m->tet, nt, m->rec, m->vol, m->flag);

  // face adjacency by sorting sorted vertex triples
  uint64_t *key = nullptr, *key2 = nullptr;
  int32_t *val = nullptr, *val2 = nullptr, *nbr4 = nullptr;
  int32_t *used = nullptr, *bnd = nullptr, *isdof = nullptr, *scan = nullptr, *cnt = nullptr;
  uint32_t *vkey = nullptr, *vkey2 = nullptr;
  unsigned long long *nbf = nullptr, *nplanes = nullptr;
  double4 *planes = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  int st = FPDE_OK;
  auto cleanup = [&]() {
    dfree(key); dfree(key2); dfree(val); dfree(val2); dfree(nbr4); dfree(used); dfree(bnd);
    dfree(isdof); dfree(scan); dfree(cnt); dfree(vkey); dfree(vkey2); dfree(nbf); dfree(nplanes);
    dfree(planes);
    if (tmp) (void)hipFree(tmp);
  };
#define STEP(x)                \
  do {                         \
    st = (x);                  \
    if (st != FPDE_OK) {       \
      cleanup();               \
      return st;               \
    }                          \
  } while (0)
#define STEPH(x) STEP(((x) == hipSuccess) ? FPDE_OK : FPDE_EHIP)
  STEP(dalloc(&key, nf));
  STEP(dalloc(&key2, nf));
  STEP(dalloc(&val, nf));
  STEP(dalloc(&val2, nf));
  STEP(dalloc(&nbr4, nf));
  STEP(dalloc(&used, nv));
  STEP(dalloc(&bnd, nv));
  STEP(dalloc(&isdof, nv + 1));
  STEP(dalloc(&scan, nv + 1));
  STEP(dalloc(&cnt, nv + 1));
  STEP(dalloc(&vkey, nf));
  STEP(dalloc(&vkey2, nf));
  STEP(dalloc(&nbf, 1));
  STEP(dalloc(&nplanes, 1));

  k_face_keys<<<nblk(nf), 256, 0, s>>>(m->tet, nt, key, val);
  int end_bit = 42 + bits_for((uint64_t)nv);
  size_t need = 0;
  STEPH(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key, key2, val, val2, (int)nf, 0, end_bit, s));
  size_t need2 = 0;
  STEPH(hipcub::DeviceRadixSort::SortPairs(nullptr, need2, vkey, vkey2, val, val2, (int)nf, 0,
                                           bits_for((uint64_t)nv), s));
  size_t need3 = 0;
  STEPH(hipcub::DeviceScan::ExclusiveSum(nullptr, need3, isdof, scan, (int)(nv + 1), s));
  tmp_bytes = std::max(need, std::max(need2, need3));
  STEPH(hipMalloc(&tmp, tmp_bytes));
  STEPH(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, val2, (int)nf, 0, end_bit, s));
  k_fill_i32<<<nblk(nf), 256, 0, s>>>(nbr4, nf, -1);
  k_face_match<<<nblk(nf), 256, 0, s>>>(key2, val2, nf, nbr4, m->flag);

  STEPH(hipMemsetAsync(used, 0, sizeof(int32_t) * nv, s));
  STEPH(hipMemsetAsync(bnd, 0, sizeof(int32_t) * nv, s));
  STEPH(hipMemsetAsync(nbf, 0, sizeof(unsigned long long), s));
  STEPH(hipMemsetAsync(isdof, 0, sizeof(int32_t) * (nv + 1), s));
  k_boundary<<<nblk(nf), 256, 0, s>>>(m->tet, nbr4, nt, used, bnd, nbf);
  k_isdof<<<nblk(nv), 256, 0, s>>>(used, bnd, nv, isdof);
  STEPH(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, isdof, scan, (int)(nv + 1), s));
  int32_t ndof = 0;
  unsigned long long nbf_h = 0;
  STEPH(hipMemcpyAsync(&ndof, scan + nv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  STEPH(hipMemcpyAsync(&nbf_h, nbf, sizeof(nbf_h), hipMemcpyDeviceToHost, s));
  STEPH(hipStreamSynchronize(s));
  m->ndof = ndof;
  m->nbf = (int64_t)nbf_h;
  // the domain must be convex: every vertex inside every boundary-face plane
  STEP(dalloc(&planes, nbf_h > 0 ? nbf_h : 1));
  STEPH(hipMemsetAsync(nplanes, 0, sizeof(unsigned long long), s));
  k_bface_planes<<<nblk(nf), 256, 0, s>>>(m->xyz, m->tet, nbr4, nt, planes, nplanes);
  k_convex<<<nblk(nv), 256, 0, s>>>(m->xyz, used, nv, planes, nplanes, convex_tol, m->flag, m->flag_aux);
  STEP(dalloc(&m->vert_of_dof, ndof > 0 ? ndof : 1));
  k_dof<<<nblk(nv), 256, 0, s>>>(isdof, scan, nv, m->dof, m->vert_of_dof);
  k_finalize<<<nblk(nt), 256, 0, s>>>(m->tet, nbr4, m->dof, nt, m->rec);

  // vertex -> element lists, ascending element id (stable sort by vertex)
  STEPH(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nv + 1), s));
  k_vt_keys<<<nblk(nf), 256, 0, s>>>(m->tet, nt, vkey, val, cnt);
  STEPH(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, vkey, vkey2, val, m->vt_tet, (int)nf, 0,
                                           bits_for((uint64_t)nv), s));
  STEPH(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, m->vt_off, (int)(nv + 1), s));
  STEPH(hipGetLastError());
  int f = take_flag(m, s);
  cleanup();
  if (f < 0) return f;
  if (f > 0) return FPDE_EHIP;
  return FPDE_OK;
#undef STEP
#undef STEPH
}

namespace fpde {

int workspace_new(int64_t ndof, fpde_mesh **out) {
  *out = nullptr;
  fpde_mesh *m = new fpde_mesh();
  m->ndof = ndof;
  if (hipGetDevice(&m->device) != hipSuccess || alloc_flags(m) != FPDE_OK) {
    fpde_mesh_destroy(m);
    return FPDE_ENOMEM;
  }
  const int32_t z = 0;
  const int64_t mz = -1;
  if (hipMemcpy(m->flag, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->flag_aux, &mz, sizeof(mz), hipMemcpyHostToDevice) != hipSuccess) {
    fpde_mesh_destroy(m);
    return FPDE_EHIP;
  }
  *out = m;
  return FPDE_OK;
}

}  // namespace fpde

extern "C" int fpde_mesh_create(const double *xyz, int64_t n_vert, const int32_t *tet, int64_t n_tet,
                                void *stream, fpde_mesh **out) {
  if (!out) return FPDE_EINVAL;
  *out = nullptr;
  if (!xyz || !tet || n_vert < 4 || n_tet < 1) return FPDE_EINVAL;
  if (n_vert >= (int64_t(1) << 21) || n_tet >= (int64_t(1) << 29)) return FPDE_EUNSUPPORTED;
  for (int64_t k = 0; k < 4 * n_tet; k++)
    if (tet[k] < 0 || tet[k] >= n_vert) return FPDE_EINVAL;
  for (int64_t k = 0; k < 3 * n_vert; k++)
    if (!std::isfinite(xyz[k])) return FPDE_EINVAL;
  // convexity tolerance: 1e-12 of the diagonal of the vertices' bounding box
  // (an upper bound of the domain's diameter)
  double lo[3], hi[3];
  for (int d = 0; d < 3; d++) lo[d] = hi[d] = xyz[d];
  for (int64_t v = 1; v < n_vert; v++)
    for (int d = 0; d < 3; d++) {
      lo[d] = std::min(lo[d], xyz[3 * v + d]);
      hi[d] = std::max(hi[d], xyz[3 * v + d]);
    }
  double diag = 0.0;
  for (int d = 0; d < 3; d++) diag += (hi[d] - lo[d]) * (hi[d] - lo[d]);
  diag = std::sqrt(diag);
  fpde_mesh *m = new fpde_mesh();
  m->nv = n_vert;
  m->nt = n_tet;
  int st = mesh_build(m, xyz, tet, 1e-12 * diag, S(stream));
  if (st != FPDE_OK) {
    fpde_mesh_destroy(m);
    return st;
  }
  *out = m;
  return FPDE_OK;
}

extern "C" void fpde_mesh_destroy(fpde_mesh *m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  dfree(m->xyz); dfree(m->tet); dfree(m->rec); dfree(m->vol); dfree(m->vt_off); dfree(m->vt_tet);
  dfree(m->dof); dfree(m->vert_of_dof); dfree(m->rules); dfree(m->flag_blk);
  if (m->hflag) (void)hipHostFree(m->hflag);
  dfree(m->vec); dfree(m->red);
  for (auto &P : m->plan) free_plan(P);
  for (hipEvent_t e : m->timer.pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : m->bev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : m->lev)
    if (e) (void)hipEventDestroy(e);
  if (m->side) (void)hipStreamDestroy(m->side);
  if (m->linv) (void)hipFree(m->linv);
  dfree(m->tsync);
  dfree(m->batch_aux);
  dfree(m->escale);
  dfree(m->xsplit);
  dfree(m->bvec);
  dfree(m->pbox);
  dfree(m->cg);
  delete m;
}

extern "C" int fpde_mesh_info(const fpde_mesh *m, int64_t *n_dof, int64_t *n_boundary_faces, int64_t *n_tet) {
  if (!m) return FPDE_EINVAL;
  if (n_dof) *n_dof = m->ndof;
  if (n_boundary_faces) *n_boundary_faces = m->nbf;
  if (n_tet) *n_tet = m->nt;
  return FPDE_OK;
}

extern "C" int fpde_dof_map(const fpde_mesh *m, int32_t *dof) {
  if (!m || !dof) return FPDE_EINVAL;
  FPDE_HIP(hipMemcpy(dof, m->dof, sizeof(int32_t) * m->nv, hipMemcpyDeviceToHost));
  return FPDE_OK;
}

namespace fpde {

// Stage timers only take timestamps: their records need no system-scope
// cache writeback (the times are read after the caller has synchronised),
// which would otherwise cost every recorded stage a flush.
constexpr unsigned kTimerEventFlags = hipEventDisableSystemFence;

long timer_begin(fpde_mesh *m, hipStream_t s, int stage) {
  StageTimer &T = m->timer;
  if (!T.on || !((T.mask >> stage) & 1u)) return -1;
  if (T.used >= T.pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, kTimerEventFlags) != hipSuccess) return -1;
    T.pool.push_back(e);
  }
  const size_t i = T.used++;
  if (hipEventRecord(T.pool[i], s) != hipSuccess) return -1;
  return (long)i;
}

void timer_end(fpde_mesh *m, int stage, long t, hipStream_t s, int weight) {
  StageTimer &T = m->timer;
  if (t < 0 || !T.on) return;
  if (T.used >= T.pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, kTimerEventFlags) != hipSuccess) return;
    T.pool.push_back(e);
  }
  const size_t i = T.used++;
  if (hipEventRecord(T.pool[i], s) != hipSuccess) return;
  T.marks.push_back({stage, (size_t)t, i, weight});
}

}  // namespace fpde

extern "C" int fpde_timing_stages(fpde_mesh *m, unsigned mask) {
  if (!m) return FPDE_EINVAL;
  if (mask) {
    FPDE_HIP(hipDeviceSynchronize());
    m->timer.used = 0;
    m->timer.marks.clear();
  }
  m->timer.on = mask != 0;
  m->timer.mask = mask;
  return FPDE_OK;
}

extern "C" int fpde_timing(fpde_mesh *m, int enable) { return fpde_timing_stages(m, enable ? ~0u : 0u); }

extern "C" int fpde_stage_times(fpde_mesh *m, double *ms, int64_t *count) {
  if (!m) return FPDE_EINVAL;
  double t[FPDE_NSTAGES] = {0};
  int64_t c[FPDE_NSTAGES] = {0};
  for (const auto &mk : m->timer.marks) {
    FPDE_HIP(hipEventSynchronize(m->timer.pool[mk.b]));
    float e = 0.f;
    FPDE_HIP(hipEventElapsedTime(&e, m->timer.pool[mk.a], m->timer.pool[mk.b]));
    t[mk.stage] += (double)e;
    c[mk.stage] += mk.weight;
  }
  for (int k = 0; k < FPDE_NSTAGES; k++) {
    if (ms) ms[k] = t[k];
    if (count) count[k] = c[k];
  }
  return FPDE_OK;
}
