// Dense LU factorization without pivoting, A = L U (L unit lower, U upper,
// both kept in A), and the solve A u = b, for the non-symmetric matrix of
// the divergence-form two-sided problem (Sec. 3).  Its bilinear form is
// coercive (the symmetric part of -A is positive definite), so every leading
// block is nonsingular and no row exchange is needed; a zero or non-finite
// pivot is reported, not worked around.
//
// Blocked right-looking, panel width NB = 64, three launches per panel k:
//   diag   : one workgroup factors A_kk = L_kk U_kk in registers and forms
//            inv(L_kk) (the same row operations applied to I) and inv(U_kk);
//   panels : L_ik = A_ik inv(U_kk) for every 64-row strip below and
//            U_kj = inv(L_kk) A_kj for every 64-column strip to the right,
//            each a 64 x 64 x 64 tile product (no sequential dependency);
//   update : C_ij -= L_ik U_kj over the whole trailing square, one workgroup
//            per 64 x 64 output tile.
// The solve runs the block-row triangular solves of dense.h forward with L
// (inv(L_bb) per block) and backward with U (inv(U_bb)).
#include <cmath>

#include "dense.h"

namespace fpde {

namespace {

struct LuSmem {
  double row[2][2][NB];  // [buffer][factor | inverse][column]: the pivot row
  double col[2][NB];     // [buffer][row]: the pivot column
};

// Thread t owns row r = t >> 2 of the 64 x 64 block and 16 of its columns
// (the four threads of a row are neighbouring lanes of one wavefront).
// FACTOR: a holds the block and becomes L (strict lower, multipliers) + U
// (upper); otherwise a holds an existing factor.  On exit y = inv(L) and
// z = inv(U) in the same layout.  Rows/columns past nb are identity.
// Returns false when a pivot was zero or not finite (FACTOR).
//
// One pass over the pivots j = 0..63, one barrier each.  Row j and column j
// of the partly eliminated block are final when step j starts; they are
// published to LDS (two alternating buffers, so the next step's writes
// cannot overtake this step's reads), then
//   rows r > j:  l = A_rj / U_jj, A_rc -= l U_jc (c > j), A_rj = l, and the
//                same row operation on Y (Y = I at the start, inv(L) at the
//                end: inv(L) is the product of the elimination steps);
//   rows r <= j: column j of W = inv(U) from W U = I,
//                W_rj = (delta_rj - sum_{k<j} W_rk U_kj) / U_jj, whose
//                column of U is the published column j and whose W_rk were
//                formed at the earlier steps (a 4-lane sum over the row's
//                threads).
// The pivots run in 16 blocks of 4 (a runtime loop over the blocks, the 4
// steps of a block unrolled), so the code stays small.  To keep register
// indices static, the three arrays rotate by one slot after each block: in
// block kb, slot s of a thread with t & 3 = cl holds column
// cl + 4 ((s + kb) mod 16), so the block's own columns are in slot 0.  The
// LDS row buffer is kept in slot order; the column buffer (indexed by row)
// in the same rotated order, row r at (r & 3) + 4 ((r / 4 - kb) mod 16).
template <bool FACTOR>
__device__ __forceinline__ bool lu_block(LuSmem &sm, double (&a)[16], double (&y)[16], double (&z)[16]) {
  const int tid = threadIdx.x, r = tid >> 2, cls = tid & 3;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    y[k] = (cls + 4 * k == r) ? 1.0 : 0.0;
    z[k] = 0.0;
  }
#pragma unroll 1
  for (int kb = 0; kb < 16; kb++) {
    const int own = (r & 3) + 4 * (((r >> 2) - kb) & 15);  // this row's slot in the column buffer
    const int live = 15 - kb;  // slots 1..live hold columns right of the block
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int j = 4 * kb + c, buf = c & 1;
      if (r == j) {
#pragma unroll
        for (int s = 0; s < 16; s++) {
          sm.row[buf][0][cls + 4 * s] = a[s];
          sm.row[buf][1][cls + 4 * s] = y[s];
        }
      }
      if (cls == c) sm.col[buf][own] = a[0];
      __syncthreads();
      // everything this step reads from LDS, loaded before any use
      double ra[16], ry[16], rc[16];
#pragma unroll
      for (int s = 0; s < 16; s++) {
        ra[s] = sm.row[buf][0][cls + 4 * s];
        ry[s] = sm.row[buf][1][cls + 4 * s];
        rc[s] = sm.col[buf][cls + 4 * s];
      }
      const double piv = sm.row[buf][0][c];  // U_jj: column j is slot 0 of lane class c
      const double cown = sm.col[buf][own];
      const double rp = 1.0 / piv;
      // column j of inv(U): sum over the columns left of j (inactive slots
      // contribute an exact zero)
      double part = 0.0;
#pragma unroll
      for (int s = 0; s < 16; s++) {
        const bool left = s == 0 ? cls < c : s > live;
        part = fma(left ? z[s] : 0.0, rc[s], part);
      }
      part += __shfl_xor(part, 1, 64);
      part += __shfl_xor(part, 2, 64);
      if (cls == c && r <= j) z[0] = ((r == j ? 1.0 : 0.0) - part) * rp;
      // elimination below the pivot: multipliers are zero where a slot does
      // not take part, which leaves it unchanged
      const double l = r > j ? (FACTOR ? cown * rp : cown) : 0.0;
#pragma unroll
      for (int s = 0; s < 16; s++) {
        const bool right = s == 0 ? cls > c : s <= live;
        if (FACTOR) a[s] = fma(right ? -l : 0.0, ra[s], a[s]);
        y[s] = fma(right ? 0.0 : -l, ry[s], y[s]);
      }
      if (FACTOR && cls == c && r > j) a[0] = l;
    }
    // rotate: slot s takes slot s + 1, slot 15 takes slot 0
    const double a0 = a[0], y0 = y[0], z0 = z[0];
#pragma unroll
    for (int s = 0; s < 15; s++) {
      a[s] = a[s + 1];
      y[s] = y[s + 1];
      z[s] = z[s + 1];
    }
    a[15] = a0;
    y[15] = y0;
    z[15] = z0;
  }
  // after 16 rotations every slot is back at column cls + 4 s; every pivot,
  // the last row's included, is a diagonal entry of U
  bool good = true;
  if (FACTOR) {
#pragma unroll
    for (int k = 0; k < 16; k++)
      if (cls + 4 * k == r && !(fabs(a[k]) > 0.0 && isfinite(a[k]))) good = false;
  }
  return good;
}

// FACTOR: one workgroup factors the diagonal block b = kfac / 64 and writes
// L / U over it; otherwise one workgroup per block b = blockIdx.x reads the
// existing factor.  Either way it writes inv(L_bb) (row-major), its
// transpose, and inv(U_bb)^T for block b.
template <bool FACTOR>
__global__ void __launch_bounds__(256) k_lu_diag(double *__restrict__ A, int64_t lda, int64_t n, int64_t kfac,
                                                 double *__restrict__ Linv, double *__restrict__ LinvT,
                                                 double *__restrict__ UinvT, int32_t *flag, int64_t *aux) {
  __shared__ LuSmem sm;
  const int64_t b = FACTOR ? kfac / NB : (int64_t)blockIdx.x;
  const int64_t k0 = b * NB;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  const int tid = threadIdx.x, r = tid >> 2, cls = tid & 3;
  double a[16], y[16], z[16];
  const int rr = r < nb ? r : nb - 1;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int c = cls + 4 * k;
    a[k] = A[(k0 + rr) * lda + k0 + (c < nb ? c : nb - 1)];
  }
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int c = cls + 4 * k;
    if (r >= nb || c >= nb) a[k] = (r == c) ? 1.0 : 0.0;
  }
  const bool good = lu_block<FACTOR>(sm, a, y, z);
  if (FACTOR && !good) {
    set_flag(flag, FPDE_ESINGULAR);
    atomicCAS((unsigned long long *)aux, ~0ull, (unsigned long long)k0);
  }
  const int64_t o = b * NB * NB;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int c = cls + 4 * k;
    if (FACTOR && r < nb && c < nb) A[(k0 + r) * lda + k0 + c] = a[k];
    Linv[o + r * NB + c] = y[k];
    LinvT[o + c * NB + r] = y[k];
    UinvT[o + c * NB + r] = z[k];
  }
}

// out = P Q over a 64-deep inner dimension: P is 64 x 64 (rows past `prow`
// read as zero), Q is 64 x 64 row-major by inner index (columns past `qcol`
// read as zero).  Two 32-deep chunks staged through LDS as in tile_product (Q
// transposed on the way in, every load at a valid address), multiplied on
// the matrix cores; value q of a thread's 16 sits at (frag_row<double>(q),
// frag_col<double>(q)).
template <int KD = NB>
__device__ __forceinline__ void tile_nn(const double *__restrict__ P, int64_t ldp, int prow,
                                        const double *__restrict__ Q, int64_t ldq, int qcol, double (*sP)[33],
                                        double (*sQ)[33], double out[16]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lc = tid & 31, lr = tid >> 5;  // P: rows lr + 8 it, column lc of a chunk
  const int qc = tid & 63, qr = tid >> 6;  // Q: column qc, inner rows qr + 4 it of a chunk
  const int qcc = qc < qcol ? qc : qcol - 1;
  const int rm = 32 * (w >> 1) + (lane & 15), cm = 32 * (w & 1) + (lane & 15), kq = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double pr[8], qv[8];
  auto load = [&](int kk) {
#pragma unroll
    for (int it = 0; it < 8; it++) {
      const int rr = lr + 8 * it;
      pr[it] = P[(int64_t)(rr < prow ? rr : prow - 1) * ldp + kk + lc];
      qv[it] = Q[(int64_t)(kk + qr + 4 * it) * ldq + qcc];
    }
  };
  load(0);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 32) {
#pragma unroll
    for (int it = 0; it < 8; it++) {
      const int rr = lr + 8 * it;
      sP[rr][lc] = rr < prow ? pr[it] : 0.0;
      sQ[qc][qr + 4 * it] = qc < qcol ? qv[it] : 0.0;
    }
    __syncthreads();
    if (kk + 32 < KD) load(kk + 32);
    mfma_chunk(sP, sQ, rm, cm, kq, acc);
    __syncthreads();
  }
  mfma_out(acc, out);
}

// Workgroups [0, ns): L strips (rows k1 + 64 x, columns of panel k);
// [ns, 2 ns): U strips (rows of panel k, columns k1 + 64 (x - ns)).
__global__ void __launch_bounds__(256) k_lu_panels(double *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                   int ns, const double *__restrict__ Linv_k,
                                                   const double *__restrict__ UinvT_k) {
  __shared__ double sP[64][33], sQ[64][33];
  const int64_t k1 = k0 + NB;
  const int x = blockIdx.x;
  double out[16];
  if (x < ns) {
    const int64_t r0 = k1 + 64 * (int64_t)x;
    const int rows = (int)((n - r0) < 64 ? (n - r0) : 64);
    tile_product(A + r0 * lda + k0, lda, rows, UinvT_k, NB, NB, sP, sQ, out);
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int rr = frag_row<double>(q);
      if (rr < rows) A[(r0 + rr) * lda + k0 + frag_col<double>(q)] = out[q];
    }
  } else {
    const int64_t c0 = k1 + 64 * (int64_t)(x - ns);
    const int cols = (int)((n - c0) < 64 ? (n - c0) : 64);
    tile_nn(Linv_k, NB, NB, A + k0 * lda + c0, lda, cols, sP, sQ, out);
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int cc = frag_col<double>(q);
      if (cc < cols) A[(k0 + frag_row<double>(q)) * lda + c0 + cc] = out[q];
    }
  }
}

// Diagonal block at (k0, k0) from registers a (thread t: row t >> 2,
// columns (t & 3) + 4 k; rows/columns past nb identity): factor it, write
// L + U over A's block and inv(L), inv(L)^T, inv(U)^T of block k0 / 64.
__device__ __forceinline__ void lu_diag_from(LuSmem &sm, double (&a)[16], int nb, double *__restrict__ A, int64_t lda,
                                             int64_t k0, double *__restrict__ Linv, double *__restrict__ LinvT,
                                             double *__restrict__ UinvT, int32_t *flag, int64_t *aux) {
  const int tid = threadIdx.x, r = tid >> 2, cls = tid & 3;
  double y[16], z[16];
  const bool good = lu_block<true>(sm, a, y, z);
  if (!good) {
    set_flag(flag, FPDE_ESINGULAR);
    atomicCAS((unsigned long long *)aux, ~0ull, (unsigned long long)k0);
  }
  const int64_t o = (k0 / NB) * NB * NB;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const int c = cls + 4 * k;
    if (r < nb && c < nb) A[(k0 + r) * lda + k0 + c] = a[k];
    Linv[o + r * NB + c] = y[k];
    LinvT[o + c * NB + r] = y[k];
    UinvT[o + c * NB + r] = z[k];
  }
}

// C_IJ -= L_I,K U_K,J over the trailing square from k1 = k0 + KD (T x T
// tiles), K = columns of L / rows of U [k0, k0 + KD): one panel (KD = 64) or
// two consecutive panels (KD = 128).  cross: only the block column and the
// block row at k1 (tiles (x, 0), x < T, then (0, x - T + 1): 2T - 1 tiles).
// The workgroup of tile (0, 0) -- the next diagonal block -- then factors
// that block at once (lu_diag_from), so the next step's diagonal
// factorization runs beside the rest of this update.
template <int KD>
__global__ void __launch_bounds__(256) k_lu_update(double *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                   int T, double *__restrict__ Linv, double *__restrict__ LinvT,
                                                   double *__restrict__ UinvT, int32_t *flag, int64_t *aux,
                                                   int cross) {
  struct Gemm {
    double sP[64][33], sQ[64][33];
  };
  struct Diag {
    double blk[64][65];
    LuSmem lu;
  };
  __shared__ union {
    Gemm g;
    Diag d;
  } sm;
  const int64_t k1 = k0 + KD;
  const int64_t x = blockIdx.x;
  int64_t I, J;
  if (cross) {
    I = x < T ? x : 0;
    J = x < T ? 0 : x - T + 1;
  } else {
    I = x / T;
    J = x - I * T;
  }
  const int64_t ri = k1 + 64 * I, cj = k1 + 64 * J;
  const int prow = (int)((n - ri) < 64 ? (n - ri) : 64);
  const int qcol = (int)((n - cj) < 64 ? (n - cj) : 64);
  double out[16];
  tile_nn<KD>(A + ri * lda + k0, lda, prow, A + k0 * lda + cj, lda, qcol, sm.g.sP, sm.g.sQ, out);
  double cv[16];
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int64_t r = ri + frag_row<double>(q), c = cj + frag_col<double>(q);
    cv[q] = A[(r < n ? r : n - 1) * lda + (c < n ? c : n - 1)];
  }
  if (x == 0) {
    const int nb = prow;
#pragma unroll
    for (int q = 0; q < 16; q++) sm.d.blk[frag_row<double>(q)][frag_col<double>(q)] = cv[q] - out[q];
    __syncthreads();
    const int tid = threadIdx.x, r = tid >> 2, cls = tid & 3;
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const int c = cls + 4 * k;
      a[k] = (r < nb && c < nb) ? sm.d.blk[r][c] : ((r == c) ? 1.0 : 0.0);
    }
    lu_diag_from(sm.d.lu, a, nb, A, lda, k1, Linv, LinvT, UinvT, flag, aux);
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int64_t r = ri + frag_row<double>(q), c = cj + frag_col<double>(q);
    if (r < n && c < n) A[r * lda + c] = cv[q] - out[q];
  }
}

inline unsigned blocks_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__global__ void k_copy_f64(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = a[k];
}

}  // namespace

// the three inverse sets of the LU blocks inside the mesh's buffer
static int lu_inverses(fpde_mesh *m, int64_t n, double **Linv, double **LinvT, double **UinvT) {
  void *lv = nullptr;
  FPDE_TRY(ensure_linv(m, n, sizeof(double), 3, &lv));
  const int64_t per = ((n + NB - 1) / NB) * NB * NB;
  *Linv = (double *)lv;
  *LinvT = *Linv + per;
  *UinvT = *LinvT + per;
  return FPDE_OK;
}

int lu_factor(fpde_mesh *m, double *A, int64_t lda, int64_t n, hipStream_t s) {
  double *Linv, *LinvT, *UinvT;
  FPDE_TRY(lu_inverses(m, n, &Linv, &LinvT, &UinvT));
  const long t = timer_begin(m, s, FPDE_STAGE_LU);
  for (int64_t k0 = 0; k0 < n; k0 += 2 * NB) {
    // the first diagonal block on its own (the kernel indexes the sets by its
    // block itself: base pointers); every later one is factored by tile
    // (0, 0) of the preceding update.  Panels in pairs: panel k0, the cross
    // at k1 = k0 + 64 (its block column and block row) updated by it alone,
    // panel k1, then the trailing square from k1 + 64 updated once by both
    // (128 columns of L, 128 rows of U): the trailing square is read and
    // written once per two panels.
    if (k0 == 0) k_lu_diag<true><<<1, 256, 0, s>>>(A, lda, n, k0, Linv, LinvT, UinvT, m->flag, m->flag_aux);
    const int64_t rest = n - k0 - NB;
    if (rest <= 0) break;
    const int64_t o = (k0 / NB) * NB * NB;  // block k0 / 64 of each inverse set
    const int ns = (int)((rest + 63) / 64);
    k_lu_panels<<<2 * ns, 256, 0, s>>>(A, lda, n, k0, ns, Linv + o, UinvT + o);
    if (rest <= NB) {  // one block left
      k_lu_update<NB><<<(unsigned)((int64_t)ns * ns), 256, 0, s>>>(A, lda, n, k0, ns, Linv, LinvT, UinvT, m->flag,
                                                                    m->flag_aux, 0);
      break;
    }
    k_lu_update<NB><<<(unsigned)(2 * ns - 1), 256, 0, s>>>(A, lda, n, k0, ns, Linv, LinvT, UinvT, m->flag,
                                                            m->flag_aux, 1);
    const int64_t k1 = k0 + NB, rest1 = rest - NB, o1 = o + NB * NB;
    const int ns1 = (int)((rest1 + 63) / 64);
    k_lu_panels<<<2 * ns1, 256, 0, s>>>(A, lda, n, k1, ns1, Linv + o1, UinvT + o1);
    k_lu_update<2 * NB><<<(unsigned)((int64_t)ns1 * ns1), 256, 0, s>>>(A, lda, n, k0, ns1, Linv, LinvT, UinvT,
                                                                        m->flag, m->flag_aux, 0);
  }
  timer_end(m, FPDE_STAGE_LU, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

// u = U^{-1} L^{-1} b from an existing factor; the inverses of its diagonal
// blocks are formed first (one workgroup per block).
int lu_solve(fpde_mesh *m, const double *LU, int64_t lda, int64_t n, const double *b, double *u, double *xs,
             hipStream_t s) {
  if (n == 0) return FPDE_OK;
  double *Linv, *LinvT, *UinvT;
  FPDE_TRY(lu_inverses(m, n, &Linv, &LinvT, &UinvT));
  const int nblk = (int)((n + NB - 1) / NB);
  FPDE_TRY(ensure_trsv_sync(m, nblk, s));
  const int epoch = ++m->tsync_epoch;
  int *fflags = m->tsync, *bflags = m->tsync + nblk, *tickets = m->tsync + 2 * nblk;
  const long t = timer_begin(m, s, FPDE_STAGE_TRSV);
  k_lu_diag<false><<<nblk, 256, 0, s>>>(const_cast<double *>(LU), lda, n, 0, Linv, LinvT, UinvT, m->flag,
                                        m->flag_aux);
  if (u != b) k_copy_f64<<<blocks_of(n), 256, 0, s>>>(b, u, n);
  FPDE_TRY(zero_ints(tickets, 2, s));
  k_trsv_rows<double, false><<<nblk, 256, 0, s>>>(LU, lda, n, nblk, LinvT, u, xs, fflags, tickets, epoch, m->flag,
                                                  BatchStrides{});
  k_trsv_rows<double, true><<<nblk, 256, 0, s>>>(LU, lda, n, nblk, UinvT, xs, u, bflags, tickets + 1, epoch,
                                                 m->flag, BatchStrides{});
  timer_end(m, FPDE_STAGE_TRSV, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_lu_factor(fpde_mesh *m, double *A, int64_t lda, int64_t *failed_pivot, void *stream) {
  if (!m || !A || lda < m->ndof) return FPDE_EINVAL;
  if (failed_pivot) *failed_pivot = -1;
  hipStream_t s = S(stream);
  const int64_t n = m->ndof;
  if (n == 0) return FPDE_OK;
  FPDE_TRY(lu_factor(m, A, lda, n, s));
  int64_t col = -1;
  const int f = take_flag(m, s, &col);
  if (f != 0) {
    if (failed_pivot) *failed_pivot = col;
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}

extern "C" int fpde_lu_solve(fpde_mesh *m, const double *LU, int64_t lda, const double *b, double *u,
                             void *stream) {
  if (!m || !LU || !b || !u || lda < m->ndof) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  const int64_t n = m->ndof;
  if (n == 0) return FPDE_OK;
  double *xs = nullptr;
  FPDE_TRY(dalloc(&xs, (size_t)n));
  int st = lu_solve(m, LU, lda, n, b, u, xs, s);
  const int f = take_flag(m, s);
  dfree(xs);
  if (st != FPDE_OK) return st;
  return f < 0 ? f : (f > 0 ? FPDE_EHIP : FPDE_OK);
}
