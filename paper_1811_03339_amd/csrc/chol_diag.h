// Factorization of one 64 x 64 diagonal block of the blocked Cholesky in
// LDS (256 threads), shared by the first-panel kernel and the trailing
// updates whose tile (0, 0) factors the next diagonal block.
#pragma once

#include "dense.h"

namespace fpde {

// LDS used by one diagonal-block factorization: the block on entry (lower
// part; identity past the matrix end); on exit L in the lower triangle and
// X = inv(L) transposed in the strict upper triangle (X[r][c], r > c, kept at
// L[c][r]) with X's diagonal in dinv.  XcT holds inv(L_cb)^T of the 16 x 16
// diagonal block being processed, dense (zeros included).
struct DiagSmem {
  double L[NB][NB + 1];
  double XcT[16][17];
  double dinv[NB];
};

// Factor the 64 x 64 diagonal block held in sm.L (rows/columns >= nb are
// identity), write L over A's block at (k0, k0), inv(L) to Linv and
// inv(L)^T to LinvT.  The first 256 threads of the workgroup work
// (wavefront w owns block row w of the four 16-row block rows); further
// threads only take part in its barriers.  Right-looking over 16-column
// blocks cb:
//   1. wavefront cb factors the 16 x 16 diagonal block in registers (lane =
//      row, pivots and multipliers broadcast across lanes, one rsqrt per
//      pivot) and, interleaved, inverts it (lane = column); it then scales
//      its block row of inv(L) by that inverse;
//   2. every wavefront below forms its block L[w][cb] = A[w][cb] inv(L_cb)^T
//      and updates its block row of inv(L) (product form
//      inv(L) = L_3^{-1} L_2^{-1} L_1^{-1} L_0^{-1}, one block column per step);
//   3. every thread applies the rank-16 update to its 4 x 4 tile (rows
//      4ty.., columns 4tx..) of the trailing lower triangle, in LDS.
// Two workgroup barriers per block column.
template <class T>
__device__ __forceinline__ void diag_factor(DiagSmem &sm, int nb, T *__restrict__ A, int64_t lda, int64_t k0,
                                            T *__restrict__ Linv, T *__restrict__ LinvT, int32_t *flag,
                                            int64_t *aux) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ty = tid >> 4, tx = tid & 15;
  bool bad = false;
#pragma unroll 1
  for (int cb = 0; cb < 4; cb++) {
    const int c0 = 16 * cb;
    // the trailing updates of the previous step to this wavefront's block
    // row (the only rows it reads before the next barrier) are in LDS
    wave_lds_sync();
    if (wv == cb) {
      const int r = opaque(lane & 15);  // lanes 16..63 repeat lanes 0..15
      // Lanes 0..15 (v = row r of the block -> row r of L) factor; lanes
      // 16..31 (v = column r of the identity -> column r of inv(L_cb))
      // run the same instruction stream, which is forward substitution for
      // them: both updates read v[k] -= v[j] L[k][j].  The strict upper part
      // of a factor row starts at zero and only ever holds values that no
      // lower entry depends on.  At pivot j the factor lanes store L[r][j] to
      // its place in LDS and every lane reads the multipliers L[k][j], k > j,
      // back as broadcasts; lane j + 1 forms the next pivot from its own
      // registers (its multiplier is its own L[j+1][j]), off the LDS path.
      const bool frow = lane < 16;
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; k++) {
        const double a = sm.L[c0 + r][c0 + k];
        v[k] = frow ? a : ((k == r) ? 1.0 : 0.0);
      }
      double piv = read_lane(v[0], 0);
#pragma unroll
      for (int j = 0; j < 16; j++) {
        if (!(piv > 0.0)) {
          bad = true;
          piv = 1.0;
        }
        const double rs = rsqrt(piv);
        v[j] *= rs;  // L[r][j] below the pivot, sqrt(piv) at it; inv(L)[j][r] on the other lanes
        if (j + 1 < 16) piv = read_lane(fma(-v[j], v[j], v[j + 1]), j + 1);
        if (frow) sm.L[c0 + r][c0 + j] = v[j];
        wave_lds_sync();
#pragma unroll
        for (int k = j + 1; k < 16; k++) pin(v[k]);  // the previous pivot's updates are done
#pragma unroll
        for (int k = j + 1; k < 16; k++) v[k] = fma(-v[j], sm.L[c0 + k][c0 + j], v[k]);
      }
      if (lane >= 16 && lane < 32) {
        double dg = 0.0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
          if (k > r) sm.L[c0 + r][c0 + k] = v[k];  // column r of inv(L) transposed; L is in place
          sm.XcT[r][k] = v[k];
          dg = (k == r) ? v[k] : dg;
        }
        sm.dinv[c0 + r] = dg;
      }
      wave_lds_sync();
      // block row cb of inv(L): X[cb][K] = inv(L_cb) * (accumulated X[cb][K]), K < cb
      const int c = lane & 15, rg = lane >> 4;
      for (int K = 0; K < cb; K++) {
        double nx[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k = 0; k < 16; k++) {
          const double xo = sm.L[16 * K + c][c0 + k];
#pragma unroll
          for (int q = 0; q < 4; q++) nx[q] = fma(sm.XcT[k][4 * rg + q], xo, nx[q]);
        }
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 4; q++) sm.L[16 * K + c][c0 + 4 * rg + q] = nx[q];
        wave_lds_sync();
      }
    }
    __syncthreads();
    if (wv > cb && wv < 4) {
      const int rb = 16 * wv, r = lane >> 2, cg = lane & 3;
      // L[wv][cb] = A[wv][cb] inv(L_cb)^T  (lane: row r, columns 4cg..4cg+3;
      // row values streamed from LDS, a few k at a time, to bound live registers)
      double lo[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k = 0; k < 16; k++) {
        const double av = sm.L[rb + r][c0 + k];
#pragma unroll
        for (int q = 0; q < 4; q++) lo[q] = fma(av, sm.XcT[k][4 * cg + q], lo[q]);
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; q++) sm.L[rb + r][c0 + 4 * cg + q] = lo[q];
      wave_lds_sync();
      // block row wv of inv(L): X[wv][K] -= L[wv][cb] X[cb][K] (K < cb), X[wv][cb] = -L[wv][cb] inv(L_cb)
      for (int K = 0; K <= cb; K++) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (K < cb) {
#pragma unroll 4
          for (int k = 0; k < 16; k++) {
            const double lv = sm.L[rb + r][c0 + k];
#pragma unroll
            for (int q = 0; q < 4; q++) acc[q] = fma(lv, sm.L[16 * K + 4 * cg + q][c0 + k], acc[q]);
          }
#pragma unroll
          for (int q = 0; q < 4; q++) sm.L[16 * K + 4 * cg + q][rb + r] -= acc[q];
        } else {
#pragma unroll 4
          for (int k = 0; k < 16; k++) {
            const double lv = sm.L[rb + r][c0 + k];
#pragma unroll
            for (int q = 0; q < 4; q++) acc[q] = fma(lv, sm.XcT[4 * cg + q][k], acc[q]);
          }
#pragma unroll
          for (int q = 0; q < 4; q++) sm.L[16 * K + 4 * cg + q][rb + r] = -acc[q];
        }
      }
    }
    __syncthreads();
    // trailing lower triangle, in place: 4 x 4 tile (rows 4ty.., columns 4tx..)
    // -= L[rows][cb] L[columns][cb]^T (upper halves of diagonal tiles untouched)
    if (ty < 16 && (tx >> 2) > cb && ty >= tx) {
      double t[4][4];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) t[i][j] = 0.0;
#pragma unroll 4
      for (int k = 0; k < 16; k++) {
        double lr[4], lm[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
          lr[i] = sm.L[4 * ty + i][c0 + k];
          lm[i] = sm.L[4 * tx + i][c0 + k];
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) t[i][j] = fma(lr[i], lm[j], t[i][j]);
      }
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
          if (ty != tx || j <= i) sm.L[4 * ty + i][4 * tx + j] -= t[i][j];
    }
  }
  if (bad) {
    set_flag(flag, FPDE_ENOTSPD);
    atomicCAS((unsigned long long *)aux, ~0ull, (unsigned long long)k0);
  }
  // L to A (lower part inside the matrix), X row-major to Linv, X^T to LinvT
  if (tid >= 256) return;
#pragma unroll 4
  for (int it = 0; it < 16; it++) {
    const int idx = tid + 256 * it, r = idx >> 6, m = idx & 63;
    const double lrm = sm.L[r][m], lmr = sm.L[m][r], dr = sm.dinv[r];
    if (r < nb && m < nb && m <= r) A[(k0 + r) * lda + k0 + m] = (T)lrm;
    Linv[idx] = (T)((m < r) ? lmr : ((m == r) ? dr : 0.0));   // X[r][m]
    LinvT[idx] = (T)((r < m) ? lrm : ((m == r) ? dr : 0.0));  // X[m][r]
  }
}

}  // namespace fpde
