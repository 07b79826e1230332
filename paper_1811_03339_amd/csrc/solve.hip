// Dense solve of K u = b ("Solve linear equations", Table 4) for the SPD
// fractional stiffness matrix.
//
// Blocked right-looking Cholesky K = L L^T on a row-major matrix (lower
// triangle), panel width NB = 64, two launches per panel:
//   diag  : one workgroup factors the 64 x 64 diagonal block in 4-column
//           strips and forms inv(L_kk); for every panel after the first this
//           runs inside the previous trailing update (its tile (0, 0));
//   panel : X = B inv(L_kk)^T for every 64-row strip below (a plain GEMM,
//           no sequential dependency), one workgroup per strip;
//   syrk  : the trailing lower triangle, C -= X X^T, one workgroup per
//           64 x 64 output tile.
// Triangular solves use the stored inv(L_kk): one launch per block applies
// the diagonal inverse and the off-diagonal update together (forward
// x_k = inv(L_kk) y_k, y_below -= L_below,k x_k; backward
// u_k = inv(L_kk)^T x_k, x_above -= L_k,above^T u_k).  The same kernels are
// instantiated for FP32 storage, which the mixed-precision path factors and
// then refines against FP64 residuals b - K u computed matrix-free from the
// FP64 derivative vectors.
#include <cmath>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

int apply_matfree(fpde_mesh *m, Plan *P, const fpde_params *p, const double *x, double *y, double *dscratch,
                  hipStream_t s);
int apply_scratch(fpde_mesh *m, Plan *P, double **d);

constexpr int NB = 64;

// inverse of the lower-triangular L held in LDS (rows >= nb are identity);
// lane j builds column j of inv(L) in X by forward substitution (L reads
// are broadcasts, X accesses are one column per lane) and stores it to Linv
// (row-major 64 x 64).  One wavefront.
template <class T>
__device__ __forceinline__ void tri_inverse_to(const double (*Lsh)[NB + 1], double (*X)[NB + 1],
                                               T *__restrict__ Linv) {
  const int j = threadIdx.x;
  for (int i = 0; i < NB; i++) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int k = j; k < i; k++) s = fma(-Lsh[i][k], X[k][j], s);
    X[i][j] = (i < j) ? 0.0 : s / Lsh[i][i];
  }
  for (int i = 0; i < NB; i++) Linv[i * NB + j] = (T)X[i][j];
}

// LDS used by one diagonal-block factorization.
struct DiagSmem {
  double L[NB][NB + 1];  // the block on entry (lower part; identity past the matrix end), L on exit
  double S[NB][5];
  double rowb4[4][NB];
};

// Factor the 64 x 64 diagonal block held in sm.L (rows/columns >= nb are
// identity), write L over A's block at (k0, k0) and inv(L) to Linv.  256
// threads in a 16 x 16 grid, each holding a 4 x 4 register tile (rows 4ty..,
// columns 4tx..).  The factorization walks 4-column strips: the strip is
// factored by one wavefront (lane = row, pivots and multipliers exchanged by
// shuffles), then every thread applies the rank-4 update to its tile.  The
// inverse X = L^{-1} proceeds by 4-row blocks in the same way.
template <class T>
__device__ __forceinline__ void diag_factor(DiagSmem &sm, int nb, T *__restrict__ A, int64_t lda, int64_t k0,
                            T *__restrict__ Linv, int32_t *flag, int64_t *aux) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double a[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int r = 4 * ty + i, m = 4 * tx + j;
      a[i][j] = (m <= r) ? sm.L[r][m] : 0.0;
    }
  bool bad = false;
#pragma unroll 1
  for (int cb = 0; cb < 16; cb++) {
    if (tx == cb) {
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) sm.S[4 * ty + i][j] = a[i][j];
    }
    __syncthreads();
    if (tid < 64) {
      const int r = tid;
      double s4[4];
#pragma unroll
      for (int j = 0; j < 4; j++) s4[j] = sm.S[r][j];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int c = 4 * cb + j;
        const double piv = __shfl(s4[j], c, 64);
        const bool ok = piv > 0.0;
        if (r == c && !ok) bad = true;
        const double d = sqrt(ok ? piv : 1.0);
        if (r == c) s4[j] = d;
        else if (r > c) s4[j] = s4[j] / d;
#pragma unroll
        for (int jj = j + 1; jj < 4; jj++) {
          const double lc = __shfl(s4[j], 4 * cb + jj, 64);
          if (r >= 4 * cb + jj) s4[jj] = fma(-s4[j], lc, s4[jj]);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; j++) sm.S[r][j] = s4[j];
    }
    __syncthreads();
    if (tx == cb) {
      if (ty >= cb) {
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) a[i][j] = sm.S[4 * ty + i][j];
      }
    } else if (tx > cb && ty >= tx) {
#pragma unroll
      for (int k = 0; k < 4; k++) {
        double lr[4], lm[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
          lr[i] = sm.S[4 * ty + i][k];
          lm[i] = sm.S[4 * tx + i][k];
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++)
            if (ty != tx || j <= i) a[i][j] = fma(-lr[i], lm[j], a[i][j]);  // skip a diagonal tile's upper part
      }
    }
    __syncthreads();
  }
  if (bad) {
    set_flag(flag, FPDE_ENOTSPD);
    atomicCAS((unsigned long long *)aux, ~0ull, (unsigned long long)k0);
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int r = 4 * ty + i, m = 4 * tx + j;
      const double v = (m <= r) ? a[i][j] : 0.0;
      sm.L[r][m] = v;
      if (r < nb && m < nb && m <= r) A[(k0 + r) * lda + k0 + m] = (T)v;
    }
  // inverse: X = I, then blocks of 4 rows: the owners of rows 4cb..4cb+3
  // finish them with the 4 x 4 diagonal block of L (inside one thread's
  // tile), publish them, and the rows below subtract L[r, block] X[block, :]
  double x[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) x[i][j] = (4 * ty + i == 4 * tx + j) ? 1.0 : 0.0;
  __syncthreads();
#pragma unroll 1
  for (int cb = 0; cb < 16; cb++) {
    if (ty == cb && tx <= cb) {  // X is lower triangular: columns beyond stay 0
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int c = 4 * cb + i;
#pragma unroll
        for (int k = 0; k < i; k++) {
          const double l = sm.L[c][4 * cb + k];
#pragma unroll
          for (int j = 0; j < 4; j++) x[i][j] = fma(-l, x[k][j], x[i][j]);
        }
        const double dinv = 1.0 / sm.L[c][c];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          x[i][j] = x[i][j] * dinv;
          sm.rowb4[i][4 * tx + j] = x[i][j];
        }
      }
    }
    __syncthreads();
    if (ty > cb && tx <= cb) {
#pragma unroll
      for (int k = 0; k < 4; k++) {
        double xr[4], l[4];
#pragma unroll
        for (int j = 0; j < 4; j++) xr[j] = sm.rowb4[k][4 * tx + j];
#pragma unroll
        for (int i = 0; i < 4; i++) l[i] = sm.L[4 * ty + i][4 * cb + k];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) x[i][j] = fma(-l[i], xr[j], x[i][j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) Linv[(4 * ty + i) * NB + 4 * tx + j] = (T)x[i][j];
}

// Factor the diagonal block at (k0, k0) on its own (the first panel).
template <class T>
__global__ void __launch_bounds__(256) k_potrf_diag(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                    T *__restrict__ Linv, int32_t *flag, int64_t *aux) {
  __shared__ DiagSmem sm;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int r = idx >> 6, m = idx & 63;
    double v;
    if (r < nb && m < nb) v = (m <= r) ? (double)A[(k0 + r) * lda + k0 + m] : 0.0;
    else v = (r == m) ? 1.0 : 0.0;
    sm.L[r][m] = v;
  }
  __syncthreads();
  diag_factor<T>(sm, nb, A, lda, k0, Linv, flag, aux);
}

// inv(L_kk) for every diagonal block of an existing factor (one wave per block)
template <class T>
__global__ void __launch_bounds__(64) k_trinv(const T *__restrict__ A, int64_t lda, int64_t n, T *__restrict__ Linv) {
  __shared__ double Lsh[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int64_t k0 = (int64_t)blockIdx.x * NB;
  const int r = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  for (int m = 0; m < NB; m++) {
    double v;
    if (r < nb) v = (m <= r && m < nb) ? (double)A[(k0 + r) * lda + k0 + m] : 0.0;
    else v = (m == r) ? 1.0 : 0.0;
    Lsh[r][m] = v;
  }
  __syncthreads();
  tri_inverse_to<T>(Lsh, X, Linv + (int64_t)blockIdx.x * NB * NB);
}

// 64 x 64 tile product acc = P Q^T over a 64-deep inner dimension, P and Q
// given as row pointers with leading dimensions; rows past `prow`/`qrow`
// read as zero.  256 threads, 4 x 4 outputs each (rows ty + 16a, cols tx + 16b).
template <class T>
__device__ __forceinline__ void tile_nt(const T *__restrict__ P, int64_t ldp, int prow, const T *__restrict__ Q,
                                        int64_t ldq, int qrow, T (*sP)[33], T (*sQ)[33], T acc[4][4]) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = (T)0;
  for (int kk = 0; kk < NB; kk += 32) {
    for (int idx = tid; idx < 64 * 32; idx += 256) {
      const int rr = idx >> 5, c = idx & 31;
      sP[rr][c] = (rr < prow) ? P[rr * ldp + kk + c] : (T)0;
      sQ[rr][c] = (rr < qrow) ? Q[rr * ldq + kk + c] : (T)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < 32; k++) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; a++) av[a] = sP[ty + 16 * a][k];
#pragma unroll
      for (int b = 0; b < 4; b++) bv[b] = sQ[tx + 16 * b][k];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
}

// panel: rows [k0+NB+64 b, +64) of columns [k0, k0+NB) become B inv(L_kk)^T
template <class T>
__global__ void __launch_bounds__(256) k_panel(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                               const T *__restrict__ Linv) {
  __shared__ T sP[64][33], sQ[64][33];
  const int64_t r0 = k0 + NB + 64 * (int64_t)blockIdx.x;
  const int rows = (int)((n - r0) < 64 ? (n - r0) : 64);
  T acc[4][4];
  tile_nt<T>(A + r0 * lda + k0, lda, rows, Linv, NB, NB, sP, sQ, acc);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int a = 0; a < 4; a++) {
    const int rr = ty + 16 * a;
    if (rr >= rows) continue;
#pragma unroll
    for (int b = 0; b < 4; b++) A[(r0 + rr) * lda + k0 + tx + 16 * b] = acc[a][b];
  }
}

// trailing update C[I,J] -= X_I X_J^T over lower tiles I >= J of the matrix
// starting at row/column k1 = k0 + NB; X = columns [k0, k0+NB).  The
// workgroup of tile (0, 0) -- the next diagonal block -- keeps its updated
// tile in LDS and factors it at once (diag_factor), so the next panel's
// diagonal factorization runs beside the rest of this update instead of
// after it.
template <class T>
__global__ void __launch_bounds__(256) k_syrk(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                              T *__restrict__ Linv_next, int32_t *flag, int64_t *aux) {
  struct Gemm {
    T sP[64][33], sQ[64][33];
  };
  __shared__ union {
    Gemm g;
    DiagSmem d;
  } sm;
  const int64_t x = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= x) I++;
  while (I * (I + 1) / 2 > x) I--;
  const int64_t J = x - I * (I + 1) / 2;
  const int64_t base = k0 + NB;
  const int64_t ri = base + 64 * I, cj = base + 64 * J;
  const int prow = (int)((n - ri) < 64 ? (n - ri) : 64);
  const int qrow = (int)((n - cj) < 64 ? (n - cj) : 64);
  T acc[4][4];
  tile_nt<T>(A + ri * lda + k0, lda, prow, A + cj * lda + k0, lda, qrow, sm.g.sP, sm.g.sQ, acc);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  if (x == 0) {
    const int nb = prow;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) {
        const int r = ty + 16 * a, c = tx + 16 * b;
        double v;
        if (r < nb && c < nb) v = (c <= r) ? (double)A[(ri + r) * lda + ri + c] - (double)acc[a][b] : 0.0;
        else v = (r == c) ? 1.0 : 0.0;
        sm.d.L[r][c] = v;
      }
    __syncthreads();
    diag_factor<T>(sm.d, nb, A, lda, ri, Linv_next, flag, aux);
    return;
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

// forward block k: x_k = inv(L_kk) y_k (written by block 0), and
// y[r] -= L[r, k-block] . x_k for the 64 rows r >= k0 + NB of this workgroup
template <class T>
__global__ void __launch_bounds__(256) k_fwd_block(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                   const T *__restrict__ Linv, double *__restrict__ y,
                                                   double *__restrict__ x) {
  __shared__ double yk[NB], xk[NB];
  const int tid = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  if (tid < NB) yk[tid] = (tid < nb) ? y[k0 + tid] : 0.0;
  __syncthreads();
  if (tid < NB) {
    double s = 0.0;
    for (int m = 0; m < NB; m++) s = fma((double)Linv[tid * NB + m], yk[m], s);
    xk[tid] = s;
    if (blockIdx.x == 0 && tid < nb) x[k0 + tid] = s;
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int64_t rbase = k0 + NB + 64 * (int64_t)blockIdx.x;
  for (int q = w; q < 64; q += 4) {
    const int64_t r = rbase + q;
    if (r >= n) break;
    double v = (double)L[r * lda + k0 + lane] * xk[lane];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) y[r] -= v;
  }
}

// backward block k: u_k = inv(L_kk)^T x_k (written by block 0), and
// x[r] -= sum_c L[k0+c][r] u_k[c] for rows r < k0 (256 per workgroup)
template <class T>
__global__ void __launch_bounds__(256) k_bwd_block(const T *__restrict__ L, int64_t lda, int64_t n, int64_t k0,
                                                   const T *__restrict__ Linv, double *__restrict__ x,
                                                   double *__restrict__ u) {
  __shared__ double xk[NB], uk[NB];
  const int tid = threadIdx.x;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  if (tid < NB) xk[tid] = (tid < nb) ? x[k0 + tid] : 0.0;
  __syncthreads();
  if (tid < NB) {
    double s = 0.0;
    for (int m = 0; m < NB; m++) s = fma((double)Linv[m * NB + tid], xk[m], s);
    uk[tid] = s;
    if (blockIdx.x == 0 && tid < nb) u[k0 + tid] = s;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + tid;
  if (r < k0) {
    double s = 0.0;
    for (int c = 0; c < nb; c++) s = fma((double)L[(k0 + c) * lda + r], uk[c], s);
    x[r] -= s;
  }
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

// device buffer for the inverses of the diagonal blocks (bytes, reused)
static int ensure_linv(fpde_mesh *m, int64_t n, size_t elem, void **out) {
  const size_t need = (size_t)((n + NB - 1) / NB) * NB * NB * elem;
  if (m->linv_bytes < need) {
    if (m->linv) (void)hipFree(m->linv);
    m->linv = nullptr;
    m->linv_bytes = 0;
    if (hipMalloc(&m->linv, need) != hipSuccess) return FPDE_ENOMEM;
    m->linv_bytes = need;
  }
  *out = m->linv;
  return FPDE_OK;
}

template <class T>
static int potrf(T *A, int64_t lda, int64_t n, fpde_mesh *m, hipStream_t s) {
  void *lv = nullptr;
  FPDE_TRY(ensure_linv(m, n, sizeof(T), &lv));
  T *Linv = (T *)lv;
  const long t = timer_begin(m, s);
  // the first diagonal block on its own; every later one is factored by the
  // workgroup of tile (0, 0) inside the preceding trailing update
  k_potrf_diag<T><<<1, 256, 0, s>>>(A, lda, n, 0, Linv, m->flag, m->flag_aux);
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    T *Lk = Linv + (k0 / NB) * NB * NB;
    const int64_t rest = n - k0 - NB;
    if (rest > 0) {
      k_panel<T><<<nblk(rest, 64), 256, 0, s>>>(A, lda, n, k0, Lk);
      const int64_t Tn = (rest + 63) / 64;
      k_syrk<T><<<(unsigned)(Tn * (Tn + 1) / 2), 256, 0, s>>>(A, lda, n, k0, Lk + NB * NB, m->flag,
                                                                m->flag_aux);
    }
  }
  timer_end(m, FPDE_STAGE_POTRF, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

// y (n) holds the right-hand side on entry and the solution on exit;
// x (n) is scratch
template <class T>
static int trsv_pair(const T *L, int64_t lda, int64_t n, const T *Linv, double *y, double *x, fpde_mesh *m,
                     hipStream_t s) {
  const long t = timer_begin(m, s);
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int64_t rest = n - k0 - NB;
    const unsigned g = rest > 0 ? nblk(rest, 64) : 1;
    k_fwd_block<T><<<g, 256, 0, s>>>(L, lda, n, k0, Linv + (k0 / NB) * NB * NB, y, x);
  }
  const int64_t last = ((n - 1) / NB) * NB;
  for (int64_t k0 = last; k0 >= 0; k0 -= NB) {
    const unsigned g = k0 > 0 ? nblk(k0, 256) : 1;
    k_bwd_block<T><<<g, 256, 0, s>>>(L, lda, n, k0, Linv + (k0 / NB) * NB * NB, x, y);
  }
  timer_end(m, FPDE_STAGE_TRSV, t, s);
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

// Linv must hold the inverses of L's diagonal blocks
static int solve_with_factor(fpde_mesh *m, const fpde_params *p, const void *L, int64_t lda, const void *Linv,
                             const double *b, double *u, fpde_solve_info *info, hipStream_t s) {
  const int64_t n = m->ndof;
  if (info) {
    info->ir_iters = 0;
    info->final_rel_residual = 0.0;
    info->failed_pivot = -1;
  }
  if (n == 0) return FPDE_OK;
  FPDE_TRY(ensure_vec(m));
  double *y = m->vec, *r = m->vec + n, *bb = m->vec + 2 * n, *xs = m->vec + 3 * n;
  if (p->precision == FPDE_FP64) {
    if (u != b) FPDE_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    FPDE_TRY(trsv_pair<double>((const double *)L, lda, n, (const double *)Linv, u, xs, m, s));
    if (info) {
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
  FPDE_HIP(hipMemcpyAsync(bb, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_HIP(hipMemcpyAsync(u, bb, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_TRY(trsv_pair<float>((const float *)L, lda, n, (const float *)Linv, u, xs, m, s));
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
    FPDE_TRY(trsv_pair<float>((const float *)L, lda, n, (const float *)Linv, r, xs, m, s));
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
  return solve_with_factor(m, p, A, lda, m->linv, b, u, info, s);
}

extern "C" int fpde_solve_factored(fpde_mesh *m, const fpde_params *p, const void *L, int64_t lda, const double *b,
                                   double *u, fpde_solve_info *info, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!L || !b || !u || lda < m->ndof) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  const int64_t n = m->ndof;
  if (n == 0) return solve_with_factor(m, p, L, lda, nullptr, b, u, info, s);
  void *lv = nullptr;
  const size_t elem = p->precision == FPDE_MIXED ? sizeof(float) : sizeof(double);
  FPDE_TRY(ensure_linv(m, n, elem, &lv));
  const unsigned nbk = (unsigned)((n + NB - 1) / NB);
  if (p->precision == FPDE_MIXED)
    k_trinv<float><<<nbk, 64, 0, s>>>((const float *)L, lda, n, (float *)lv);
  else
    k_trinv<double><<<nbk, 64, 0, s>>>((const double *)L, lda, n, (double *)lv);
  FPDE_HIP(hipGetLastError());
  return solve_with_factor(m, p, L, lda, lv, b, u, info, s);
}
