// Sparse storage of the fractional stiffness matrix on the template of
// Sec. 2.3 (Table 1), and a Krylov solve that needs no dense matrix.
//
// The template T (node j, node k) is set when, for some axis i, the boxes of
// the two element patches overlap in both coordinates other than i; it
// contains the nonzero pattern of K and its density falls like 1/N^(2/3) as
// the mesh is refined, so at large N K is kept as a CSR matrix on T instead
// of densely:
//   k_tpl_count / k_tpl_fill  one workgroup per row: every node's box tested
//                             against the row's (the patch boxes are the
//                             template's), counted, then written in column
//                             order (ballot + prefix within the workgroup);
//   assembly                  the tube accumulation, its row pass keeping the
//                             template's columns only (tubes.hip);
//   k_csr_apply               y = K x, one wavefront per row;
//   CG                        Jacobi-preconditioned conjugate gradients on
//                             either the CSR matrix or the matrix-free
//                             product of the derivative vectors (no N^2
//                             storage at all); the diagonal of K comes from
//                             the CSR row or, matrix-free, from each node's
//                             entries and the matching entries of their
//                             partner half-rays.
#include <cmath>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

namespace {

__device__ __forceinline__ bool boxes_meet2(const double *a, const double *b) {
  bool ov[3];
#pragma unroll
  for (int d = 0; d < 3; d++) ov[d] = a[d] <= b[3 + d] && b[d] <= a[3 + d];
  return (ov[1] && ov[2]) || (ov[2] && ov[0]) || (ov[0] && ov[1]);
}

__global__ void __launch_bounds__(256) k_tpl_count(const double *__restrict__ box, int64_t n,
                                                   int64_t *__restrict__ cnt) {
  __shared__ int64_t red[4];
  const int64_t j = blockIdx.x;
  double bj[6];
#pragma unroll
  for (int d = 0; d < 6; d++) bj[d] = box[6 * j + d];
  int64_t c = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    double bk[6];
#pragma unroll
    for (int d = 0; d < 6; d++) bk[d] = box[6 * k + d];
    c += boxes_meet2(bj, bk) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// columns of row j in increasing order: 256 candidates per round, each
// thread's position = set flags before it (wave ballots + wave totals)
__global__ void __launch_bounds__(256) k_tpl_fill(const double *__restrict__ box, int64_t n,
                                                  const int64_t *__restrict__ row_ptr,
                                                  int32_t *__restrict__ col) {
  __shared__ int wtot[4];
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double bj[6];
#pragma unroll
  for (int d = 0; d < 6; d++) bj[d] = box[6 * j + d];
  int64_t base = row_ptr[j];
  for (int64_t k0 = 0; k0 < n; k0 += blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    bool hit = false;
    if (k < n) {
      double bk[6];
#pragma unroll
      for (int d = 0; d < 6; d++) bk[d] = box[6 * k + d];
      hit = boxes_meet2(bj, bk);
    }
    const unsigned long long bal = __ballot(hit);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[w] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int v = 0; v < w; v++) off += wtot[v];
    const int tot = (wtot[0] + wtot[1]) + (wtot[2] + wtot[3]);
    if (hit) col[base + off + before] = (int32_t)k;
    base += tot;
    __syncthreads();  // wtot is rewritten next round
  }
}

// y = K x, one wavefront per row (4 rows per workgroup)
__global__ void __launch_bounds__(256) k_csr_apply(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                                   const double *__restrict__ x, int64_t n, double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double s = 0.0;
  for (int64_t q = row_ptr[j] + lane; q < row_ptr[j + 1]; q += 64) s = fma(val[q], x[col[q]], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[j] = s;
}

// d_j = K_jj from the CSR row (binary search of the sorted columns)
__global__ void k_csr_diag(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, int64_t n, double *__restrict__ d) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int64_t lo = row_ptr[j], hi = row_ptr[j + 1];
  double v = 0.0;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    const int32_t c = col[mid];
    if (c == (int32_t)j) {
      v = val[mid];
      break;
    }
    if (c < (int32_t)j) lo = mid + 1;
    else hi = mid;
  }
  d[j] = v;
}

// d_j = K_jj matrix-free: K_jj = sum_i K_i c_alpha sum_g w_g 2 L_gi(j) R_gi(j);
// over the incidences of node j (entry e of half-ray h, partner half-ray h'
// on the other side of the same (g, i)): W v_e (sum of h' entries at j).
// Every (g, i) in which j has entries on both sides is seen from both sides,
// which gives the factor 2.
struct DiagArgs {
  const int64_t *row_off;
  const int4 *meta;
  const double *w;
  const int32_t *ent_dof;
  const double *ent_val;
  int64_t ndof;
  double KC0, KC1, KC2;
};

__global__ void __launch_bounds__(256) k_matfree_diag(DiagArgs a, double *__restrict__ d) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= a.ndof) return;
  double s = 0.0;
  for (int64_t p = a.row_off[j] + lane; p < a.row_off[j + 1]; p += 64) {
    const int4 mt = a.meta[p];
    const int64_t po = mt.y, pl = mt.z >> 2;
    const int ax = mt.z & 3;
    double pv = 0.0;
    for (int64_t q = po; q < po + pl; q++)
      if (a.ent_dof[q] == (int32_t)j) pv += a.ent_val[q];
    const double kc = ax == 0 ? a.KC0 : (ax == 1 ? a.KC1 : a.KC2);
    s += a.w[p] * kc * a.ent_val[mt.x] * pv;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) d[j] = s;
}

// Per-block partial sums of x.y (blocks of 256 threads, grid-stride)
__global__ void __launch_bounds__(256) k_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                                             double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    s = fma(x[k], y[k], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// u += al p; r -= al q; z = r / d
__global__ void k_cg_update(double *__restrict__ u, double *__restrict__ r, double *__restrict__ z,
                            const double *__restrict__ p, const double *__restrict__ q,
                            const double *__restrict__ dinv, double al, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  u[k] = fma(al, p[k], u[k]);
  const double rk = fma(-al, q[k], r[k]);
  r[k] = rk;
  z[k] = rk * dinv[k];
}

// p = z + be p
__global__ void k_cg_dir(double *__restrict__ p, const double *__restrict__ z, double be, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  p[k] = fma(be, p[k], z[k]);
}

__global__ void k_zero1(int32_t *p) { *p = 0; }

// start: r = b, z = p = r / d, u = 0
__global__ void k_cg_start(const double *__restrict__ b, const double *__restrict__ d, double *__restrict__ u,
                           double *__restrict__ r, double *__restrict__ z, double *__restrict__ p,
                           double *__restrict__ dinv, int64_t n, int32_t *bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double dk = d[k];
  if (!(dk > 0.0)) atomicOr(bad, 1);
  const double di = dk > 0.0 ? 1.0 / dk : 1.0;
  dinv[k] = di;
  u[k] = 0.0;
  r[k] = b[k];
  z[k] = b[k] * di;
  p[k] = b[k] * di;
}

inline unsigned blocks_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

constexpr unsigned kDotBlocks = 256;

// CG scratch in the mesh handle: r, z, p, q, d, dinv (6 N), partial sums, a flag
struct CgWork {
  double *r, *z, *p, *q, *d, *dinv, *part;
  int32_t *bad;
};

}  // namespace

static int ensure_cg(fpde_mesh *m, CgWork *w) {
  const int64_t n = m->ndof > 0 ? m->ndof : 1;
  const int64_t need = 6 * n + kDotBlocks + 1;
  if (m->cg_n < need) {
    dfree(m->cg);
    m->cg_n = 0;
    FPDE_TRY(dalloc(&m->cg, (size_t)need));
    m->cg_n = need;
  }
  w->r = m->cg;
  w->z = w->r + n;
  w->p = w->z + n;
  w->q = w->p + n;
  w->d = w->q + n;
  w->dinv = w->d + n;
  w->part = w->dinv + n;
  w->bad = (int32_t *)(w->part + kDotBlocks);
  return FPDE_OK;
}

static int dot(const double *x, const double *y, int64_t n, double *part, double *out, hipStream_t s) {
  k_dot<<<kDotBlocks, 256, 0, s>>>(x, y, n, part);
  double h[kDotBlocks];
  FPDE_HIP(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (unsigned k = 0; k < kDotBlocks; k++) t += h[k];
  *out = t;
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_template_csr(fpde_mesh *m, int64_t *row_ptr, int32_t *col, int64_t capacity, int64_t *nnz,
                                 void *stream) {
  if (!m || !row_ptr || !nnz) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  const int64_t n = m->ndof;
  *nnz = 0;
  if (n == 0) {
    FPDE_HIP(hipMemsetAsync(row_ptr, 0, sizeof(int64_t), s));
    FPDE_HIP(hipStreamSynchronize(s));
    return FPDE_OK;
  }
  if (n >= (int64_t(1) << 31)) return FPDE_EUNSUPPORTED;
  FPDE_TRY(ensure_patch_boxes(m, s));
  int64_t *cnt = nullptr;
  FPDE_TRY(dalloc(&cnt, (size_t)(n + 1)));
  int st = FPDE_OK;
  const long t = timer_begin(m, s, FPDE_STAGE_PLAN);
  k_tpl_count<<<(unsigned)n, 256, 0, s>>>(m->pbox, n, cnt);
  if (hipGetLastError() != hipSuccess) st = FPDE_EHIP;
  // row_ptr = exclusive prefix of the counts (host: N + 1 values)
  std::vector<int64_t> h(n + 1);
  if (st == FPDE_OK && hipMemcpyAsync(h.data(), cnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
    st = FPDE_EHIP;
  if (st == FPDE_OK && hipStreamSynchronize(s) != hipSuccess) st = FPDE_EHIP;
  if (st == FPDE_OK) {
    int64_t acc = 0;
    for (int64_t j = 0; j < n; j++) {
      const int64_t c = h[j];
      h[j] = acc;
      acc += c;
    }
    h[n] = acc;
    *nnz = acc;
    if (hipMemcpyAsync(row_ptr, h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s) != hipSuccess)
      st = FPDE_EHIP;
  }
  if (st == FPDE_OK && col) {
    if (capacity < *nnz) {
      st = FPDE_EINVAL;
    } else {
      k_tpl_fill<<<(unsigned)n, 256, 0, s>>>(m->pbox, n, row_ptr, col);
      if (hipGetLastError() != hipSuccess) st = FPDE_EHIP;
    }
  }
  timer_end(m, FPDE_STAGE_PLAN, t, s);
  if (hipStreamSynchronize(s) != hipSuccess && st == FPDE_OK) st = FPDE_EHIP;
  dfree(cnt);
  return st;
}

extern "C" int fpde_assemble_csr(fpde_mesh *m, const fpde_params *p, const int64_t *row_ptr, const int32_t *col,
                                 double *val, double *b, const double *f_gauss, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!row_ptr || !col || !val) return FPDE_EINVAL;
  if (p->precision != FPDE_FP64) return FPDE_EUNSUPPORTED;
  if (p->source == FPDE_SRC_USER && !f_gauss && b) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values(m, P, p->alpha, s));
  FPDE_TRY(launch_contract_tubes_csr(m, *P, p, row_ptr, col, val, s));
  if (b) FPDE_TRY(launch_load(m, p, b, f_gauss, s));
  const int f = take_flag(m, s);
  if (f != 0) {
    invalidate_values(P);
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}

extern "C" int fpde_csr_apply(fpde_mesh *m, const int64_t *row_ptr, const int32_t *col, const double *val,
                              const double *x, double *y, void *stream) {
  if (!m || !row_ptr || !col || !val || !x || !y) return FPDE_EINVAL;
  if (m->ndof == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  const long t = timer_begin(m, s, FPDE_STAGE_SPMV);
  k_csr_apply<<<blocks_of(m->ndof, 4), 256, 0, s>>>(row_ptr, col, val, x, m->ndof, y);
  timer_end(m, FPDE_STAGE_SPMV, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

extern "C" int fpde_cg_solve(fpde_mesh *m, const fpde_params *p, const int64_t *row_ptr, const int32_t *col,
                             const double *val, const double *b, double *u, double tol, int max_iter,
                             fpde_solve_info *info, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!b || !u || b == u) return FPDE_EINVAL;
  const bool csr = row_ptr != nullptr;
  if (csr && (!col || !val)) return FPDE_EINVAL;
  if (info) {
    info->ir_iters = 0;
    info->final_rel_residual = 0.0;
    info->failed_pivot = -1;
  }
  const int64_t n = m->ndof;
  if (n == 0) return FPDE_OK;
  if (!(tol > 0.0)) tol = 1e-10;
  if (max_iter <= 0) max_iter = 10000;
  hipStream_t s = S(stream);
  CgWork w;
  FPDE_TRY(ensure_cg(m, &w));
  Plan *P = nullptr;
  double *dsc = nullptr;
  const Order o = order_scalars(p->alpha);
  if (!csr) {
    FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
    FPDE_TRY(ensure_values(m, P, p->alpha, s));
    FPDE_TRY(apply_scratch(m, P, &dsc));
  }
  auto op = [&](const double *x, double *y) -> int {
    if (csr) {
      const long t = timer_begin(m, s, FPDE_STAGE_SPMV);
      k_csr_apply<<<blocks_of(n, 4), 256, 0, s>>>(row_ptr, col, val, x, n, y);
      timer_end(m, FPDE_STAGE_SPMV, t, s);
      return hipGetLastError() == hipSuccess ? FPDE_OK : FPDE_EHIP;
    }
    return apply_matfree(m, P, p, x, y, dsc, s);
  };
  const long t_all = timer_begin(m, s, FPDE_STAGE_CG);
  // diagonal of K for the Jacobi preconditioner
  if (csr) {
    k_csr_diag<<<blocks_of(n), 256, 0, s>>>(row_ptr, col, val, n, w.d);
  } else {
    DiagArgs da{};
    da.row_off = P->row_off;
    da.meta = P->inc_meta;
    da.w = P->inc_w;
    da.ent_dof = P->ent_dof;
    da.ent_val = P->ent_val;
    da.ndof = n;
    da.KC0 = p->K[0] * o.c_alpha;
    da.KC1 = p->K[1] * o.c_alpha;
    da.KC2 = p->K[2] * o.c_alpha;
    k_matfree_diag<<<blocks_of(n, 4), 256, 0, s>>>(da, w.d);
  }
  k_zero1<<<1, 1, 0, s>>>(w.bad);
  k_cg_start<<<blocks_of(n), 256, 0, s>>>(b, w.d, u, w.r, w.z, w.p, w.dinv, n, w.bad);
  FPDE_HIP(hipGetLastError());
  int32_t bad = 0;
  FPDE_HIP(hipMemcpyAsync(&bad, w.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
  double bn2 = 0.0, rz = 0.0;
  FPDE_TRY(dot(b, b, n, w.part, &bn2, s));
  if (bad) return FPDE_ENOTSPD;  // a diagonal entry <= 0: K is not SPD
  FPDE_TRY(dot(w.r, w.z, n, w.part, &rz, s));
  const double bn = std::sqrt(bn2);
  double rel = bn > 0 ? 1.0 : 0.0;
  int it = 0;
  while (rel > tol && it < max_iter) {
    FPDE_TRY(op(w.p, w.q));
    double pq = 0.0;
    FPDE_TRY(dot(w.p, w.q, n, w.part, &pq, s));
    if (!(pq > 0.0)) return FPDE_ENOTSPD;
    const double al = rz / pq;
    k_cg_update<<<blocks_of(n), 256, 0, s>>>(u, w.r, w.z, w.p, w.q, w.dinv, al, n);
    double rr = 0.0, rz2 = 0.0;
    FPDE_TRY(dot(w.r, w.r, n, w.part, &rr, s));
    FPDE_TRY(dot(w.r, w.z, n, w.part, &rz2, s));
    it++;
    rel = std::sqrt(rr) / bn;
    if (rel <= tol) break;
    const double be = rz2 / rz;
    rz = rz2;
    k_cg_dir<<<blocks_of(n), 256, 0, s>>>(w.p, w.z, be, n);
  }
  timer_end(m, FPDE_STAGE_CG, t_all, s);
  FPDE_HIP(hipGetLastError());
  // the true residual b - K u of the result, not the recursively updated one
  FPDE_TRY(op(u, w.q));
  k_cg_dir<<<blocks_of(n), 256, 0, s>>>(w.q, b, -1.0, n);  // q = b - q
  double rt = 0.0;
  FPDE_TRY(dot(w.q, w.q, n, w.part, &rt, s));
  if (info) {
    info->ir_iters = it;
    info->final_rel_residual = bn > 0 ? std::sqrt(rt) / bn : std::sqrt(rt);
  }
  const int f = take_flag(m, s);
  if (f != 0) return f < 0 ? f : FPDE_EHIP;
  return rel <= tol ? FPDE_OK : FPDE_ENOCONV;
}
