// Dense solve of K u = b ("Solve linear equations", Table 4) for the SPD
// fractional stiffness matrix.
//
// Blocked right-looking Cholesky K = L L^T on a row-major matrix (lower
// triangle), panel width NB = 64:
//   potrf : the NB x NB diagonal block, factored in LDS by one workgroup;
//   trsm  : the panel below it, X L_kk^T = B, one workgroup per 64-row strip;
//   syrk  : the trailing lower triangle, C -= P P^T, one workgroup per
//           64 x 64 output tile with an NB-deep inner product.
// Triangular solves run block by block (diagonal block in LDS + a GEMV over
// the remaining rows).  The same kernels are instantiated for FP32, which
// the mixed-precision path factors and then refines against FP64 residuals
// b - K u computed matrix-free from the FP64 derivative vectors.
#include <cmath>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

int apply_matfree(fpde_mesh *m, Plan *P, const fpde_params *p, const double *x, double *y, double *dscratch,
                  hipStream_t s);
int apply_scratch(fpde_mesh *m, Plan *P, double **d);

constexpr int NB = 64;

template <class T>
__global__ void __launch_bounds__(256) k_potrf_diag(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                    int32_t *flag, int64_t *aux) {
  __shared__ T a[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx / nb, c = idx % nb;
    a[r][c] = A[(k0 + r) * lda + k0 + c];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < nb; c++) {
    if (tid == 0) {
      T piv = a[c][c];
      if (!(piv > (T)0)) {
        if (!bad) {
          set_flag(flag, FPDE_ENOTSPD);
          atomicCAS((unsigned long long *)aux, ~0ull, (unsigned long long)(k0 + c));
        }
        bad = 1;
        piv = (T)1;
      }
      a[c][c] = sqrt(piv);
    }
    __syncthreads();
    const T d = a[c][c];
    for (int r = c + 1 + tid; r < nb; r += blockDim.x) a[r][c] = a[r][c] / d;
    __syncthreads();
    const int w = nb - c - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int r = c + 1 + idx / w, mm = c + 1 + idx % w;
      if (mm <= r) a[r][mm] -= a[r][c] * a[mm][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx / nb, c = idx % nb;
    if (c <= r) A[(k0 + r) * lda + k0 + c] = a[r][c];
  }
}

// rows [k0+NB+64 b, ...) of columns [k0, k0+NB): X L_kk^T = B
template <class T>
__global__ void __launch_bounds__(256) k_trsm(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0) {
  __shared__ T L[NB][NB + 1];
  __shared__ T X[64][NB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = k0 + NB + 64 * (int64_t)blockIdx.x;
  const int rows = (int)((n - r0) < 64 ? (n - r0) : 64);
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx % NB;
    L[r][c] = (c <= r) ? A[(k0 + r) * lda + k0 + c] : (T)0;
  }
  for (int idx = tid; idx < rows * NB; idx += blockDim.x) {
    const int r = idx / NB, c = idx % NB;
    X[r][c] = A[(r0 + r) * lda + k0 + c];
  }
  __syncthreads();
  // 4 threads per row: each owns columns c = q (mod 4) of the partial sums
  const int r = tid >> 2, q = tid & 3;
  for (int c = 0; c < NB; c++) {
    if (r < rows && q == 0) X[r][c] = X[r][c] / L[c][c];
    __syncthreads();
    if (r < rows) {
      const T xc = X[r][c];
      for (int cc = c + 1 + q; cc < NB; cc += 4) X[r][cc] -= xc * L[cc][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < rows * NB; idx += blockDim.x) {
    const int rr = idx / NB, c = idx % NB;
    A[(r0 + rr) * lda + k0 + c] = X[rr][c];
  }
}

// trailing update C[I,J] -= P_I P_J^T over lower tiles I >= J of the matrix
// starting at row/column k0 + NB; P = columns [k0, k0+NB)
template <class T>
__global__ void __launch_bounds__(256) k_syrk(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0) {
  constexpr int KB = 32;
  __shared__ T PI[64][KB + 1];
  __shared__ T PJ[64][KB + 1];
  const int64_t x = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= x) I++;
  while (I * (I + 1) / 2 > x) I--;
  const int64_t J = x - I * (I + 1) / 2;
  const int64_t base = k0 + NB;
  const int64_t ri = base + 64 * I, cj = base + 64 * J;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = (T)0;
  for (int kk = 0; kk < NB; kk += KB) {
    for (int idx = tid; idx < 64 * KB; idx += blockDim.x) {
      const int r = idx / KB, c = idx % KB;
      PI[r][c] = (ri + r < n) ? A[(ri + r) * lda + k0 + kk + c] : (T)0;
      PJ[r][c] = (cj + r < n) ? A[(cj + r) * lda + k0 + kk + c] : (T)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KB; k++) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; a++) av[a] = PI[ty + 16 * a][k];
#pragma unroll
      for (int b = 0; b < 4; b++) bv[b] = PJ[tx + 16 * b][k];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; a++) {
    const int64_t r = ri + ty + 16 * a;
    if (r >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int64_t c = cj + tx + 16 * b;
      if (c >= n || c > r) continue;
      A[r * lda + c] -= acc[a][b];
    }
  }
}

// forward: y[k0..k0+nb) solved with the diagonal block
template <class T>
__global__ void __launch_bounds__(64) k_trsv_lo_diag(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                     double *__restrict__ y) {
  __shared__ double Ld[NB][NB + 1];
  __shared__ double yy[NB];
  const int tid = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx / nb, c = idx % nb;
    Ld[r][c] = (c <= r) ? (double)L[(k0 + r) * lda + k0 + c] : 0.0;
  }
  if (tid < nb) yy[tid] = y[k0 + tid];
  __syncthreads();
  for (int c = 0; c < nb; c++) {
    if (tid == 0) yy[c] = yy[c] / Ld[c][c];
    __syncthreads();
    if (tid > c && tid < nb) yy[tid] -= Ld[tid][c] * yy[c];
    __syncthreads();
  }
  if (tid < nb) y[k0 + tid] = yy[tid];
}

// forward GEMV: rows r >= k0+NB: y[r] -= L[r, k0:k0+NB] . y[k0:k0+NB]; one wavefront per row
template <class T>
__global__ void __launch_bounds__(256) k_gemv_lo(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                 double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = k0 + NB + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  double v = (double)L[r * lda + k0 + lane] * y[k0 + lane];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) y[r] -= v;
}

// backward: L_kk^T u_k = y_k
template <class T>
__global__ void __launch_bounds__(64) k_trsv_up_diag(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                     double *__restrict__ y) {
  __shared__ double Ld[NB][NB + 1];
  __shared__ double yy[NB];
  const int tid = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx / nb, c = idx % nb;
    Ld[r][c] = (c <= r) ? (double)L[(k0 + r) * lda + k0 + c] : 0.0;
  }
  if (tid < nb) yy[tid] = y[k0 + tid];
  __syncthreads();
  for (int c = nb - 1; c >= 0; c--) {
    if (tid == 0) yy[c] = yy[c] / Ld[c][c];
    __syncthreads();
    if (tid < c) yy[tid] -= Ld[c][tid] * yy[c];
    __syncthreads();
  }
  if (tid < nb) y[k0 + tid] = yy[tid];
}

// backward GEMV: rows r < k0: y[r] -= sum_c L[k0+c][r] u[k0+c]
template <class T>
__global__ void __launch_bounds__(256) k_gemv_up(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                 double *__restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= k0) return;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  double s = 0.0;
  for (int c = 0; c < nb; c++) s += (double)L[(k0 + c) * lda + r] * y[k0 + c];
  y[r] -= s;
}

__global__ void k_axpy_copy(double *__restrict__ u, const double *__restrict__ c, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) u[k] += c[k];
}
__global__ void k_sub(const double *__restrict__ b, const double *__restrict__ y, double *__restrict__ r, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) r[k] = b[k] - y[k];
}
// sum of squares, per-block partials
__global__ void __launch_bounds__(256) k_sumsq(const double *__restrict__ x, int64_t n, double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    s += x[k] * x[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <class T>
static int potrf(T *A, int64_t lda, int64_t n, fpde_mesh *m, hipStream_t s) {
  const long t = timer_begin(m, s);
  struct End {
    fpde_mesh *m;
    long t;
    hipStream_t s;
    ~End() { timer_end(m, FPDE_STAGE_POTRF, t, s); }
  } end{m, t, s};
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    k_potrf_diag<T><<<1, 256, 0, s>>>(A, lda, n, k0, m->flag, m->flag_aux);
    const int64_t rest = n - k0 - NB;
    if (rest > 0) {
      k_trsm<T><<<nblk(rest, 64), 256, 0, s>>>(A, lda, n, k0);
      const int64_t Tn = (rest + 63) / 64;
      k_syrk<T><<<(unsigned)(Tn * (Tn + 1) / 2), 256, 0, s>>>(A, lda, n, k0);
    }
  }
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

template <class T>
static int trsv_pair(const T *L, int64_t lda, int64_t n, double *y, fpde_mesh *m, hipStream_t s) {
  const long t = timer_begin(m, s);
  struct End {
    fpde_mesh *m;
    long t;
    hipStream_t s;
    ~End() { timer_end(m, FPDE_STAGE_TRSV, t, s); }
  } end{m, t, s};
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    k_trsv_lo_diag<T><<<1, 64, 0, s>>>(L, lda, n, k0, y);
    const int64_t rest = n - k0 - NB;
    if (rest > 0) k_gemv_lo<T><<<nblk(rest, 4), 256, 0, s>>>(L, lda, n, k0, y);
  }
  const int64_t last = ((n - 1) / NB) * NB;
  for (int64_t k0 = last; k0 >= 0; k0 -= NB) {
    k_trsv_up_diag<T><<<1, 64, 0, s>>>(L, lda, n, k0, y);
    if (k0 > 0) k_gemv_up<T><<<nblk(k0), 256, 0, s>>>(L, lda, n, k0, y);
  }
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

static int ensure_vec(fpde_mesh *m) {
  if (!m->vec) FPDE_TRY(dalloc(&m->vec, 4 * (m->ndof > 0 ? m->ndof : 1)));
  if (!m->red) {
    FPDE_TRY(dalloc(&m->red, 1024));
    m->red_n = 1024;
  }
  return FPDE_OK;
}

static int norm2(fpde_mesh *m, const double *x, double *out, hipStream_t s) {
  const unsigned nb = 256;
  k_sumsq<<<nb, 256, 0, s>>>(x, m->ndof, m->red);
  double h[256];
  FPDE_HIP(hipMemcpyAsync(h, m->red, sizeof(h), hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (unsigned k = 0; k < nb; k++) t += h[k];
  *out = std::sqrt(t);
  return FPDE_OK;
}

static int solve_with_factor(fpde_mesh *m, const fpde_params *p, const void *L, int64_t lda, const double *b,
                             double *u, fpde_solve_info *info, hipStream_t s) {
  const int64_t n = m->ndof;
  if (info) {
    info->ir_iters = 0;
    info->final_rel_residual = 0.0;
    info->failed_pivot = -1;
  }
  if (n == 0) return FPDE_OK;
  FPDE_TRY(ensure_vec(m));
  if (p->precision == FPDE_FP64) {
    if (u != b) FPDE_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    FPDE_TRY(trsv_pair<double>((const double *)L, lda, n, u, m, s));
    if (info) {
      double *y = m->vec, *r = m->vec + n;
      Plan *P = nullptr;
      FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
      FPDE_TRY(ensure_values(m, P, p->alpha, s));
      double *d = nullptr;
      FPDE_TRY(apply_scratch(m, P, &d));
      FPDE_TRY(apply_matfree(m, P, p, u, y, d, s));
      k_sub<<<nblk(n), 256, 0, s>>>(b, y, r, n);
      double rn = 0, bn = 0;
      FPDE_TRY(norm2(m, r, &rn, s));
      FPDE_TRY(norm2(m, b, &bn, s));
      info->final_rel_residual = bn > 0 ? rn / bn : rn;
    }
    return FPDE_OK;
  }
  // mixed: FP32 factor, FP64 residuals from the matrix-free product
  const double tol = p->ir_tol > 0 ? p->ir_tol : 1e-8;
  const int maxit = p->ir_max_iter > 0 ? p->ir_max_iter : 30;
  double *y = m->vec, *r = m->vec + n, *bb = m->vec + 2 * n;
  FPDE_HIP(hipMemcpyAsync(bb, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_HIP(hipMemcpyAsync(u, bb, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_TRY(trsv_pair<float>((const float *)L, lda, n, u, m, s));
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values(m, P, p->alpha, s));
  double *d = nullptr;
  FPDE_TRY(apply_scratch(m, P, &d));
  double bn = 0;
  FPDE_TRY(norm2(m, bb, &bn, s));
  double rel = 0;
  int it = 0;
  for (;;) {
    FPDE_TRY(apply_matfree(m, P, p, u, y, d, s));
    k_sub<<<nblk(n), 256, 0, s>>>(bb, y, r, n);
    double rn = 0;
    FPDE_TRY(norm2(m, r, &rn, s));
    rel = bn > 0 ? rn / bn : rn;
    if (rel <= tol || it >= maxit) break;
    FPDE_TRY(trsv_pair<float>((const float *)L, lda, n, r, m, s));
    k_axpy_copy<<<nblk(n), 256, 0, s>>>(u, r, n);
    it++;
  }
  if (info) {
    info->ir_iters = it;
    info->final_rel_residual = rel;
  }
  int f = take_flag(m, s);
  if (f != 0) return f < 0 ? f : FPDE_EHIP;
  return rel <= tol ? FPDE_OK : FPDE_ENOCONV;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_solve(fpde_mesh *m, const fpde_params *p, void *A, int64_t lda, const double *b, double *u,
                          fpde_solve_info *info, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!A || !b || !u || lda < m->ndof) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  const int64_t n = m->ndof;
  if (p->precision == FPDE_MIXED)
    FPDE_TRY(potrf<float>((float *)A, lda, n, m, s));
  else
    FPDE_TRY(potrf<double>((double *)A, lda, n, m, s));
  int64_t col = -1;
  int f = take_flag(m, s, &col);
  if (f != 0) {
    if (info) {
      info->ir_iters = 0;
      info->final_rel_residual = -1.0;
      info->failed_pivot = col;
    }
    return f < 0 ? f : FPDE_EHIP;
  }
  return solve_with_factor(m, p, A, lda, b, u, info, s);
}

extern "C" int fpde_solve_factored(fpde_mesh *m, const fpde_params *p, const void *L, int64_t lda, const double *b,
                                   double *u, fpde_solve_info *info, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!L || !b || !u || lda < m->ndof) return FPDE_EINVAL;
  return solve_with_factor(m, p, L, lda, b, u, info, S(stream));
}
