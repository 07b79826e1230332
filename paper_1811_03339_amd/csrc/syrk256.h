// FP32 trailing update of the blocked Cholesky on 256 x 256 output tiles,
// split FP16 on the matrix cores (the arithmetic of k_syrk128<float>: per-row
// power-of-two scaling, x = hi + lo, hi hi^T + hi lo^T + lo hi^T in FP32).
// One workgroup of eight wavefronts (2 x 4, 128 x 64 each) per tile, one
// workgroup per compute unit (128 KB of LDS: two buffers of a 32-column
// chunk of X_I and X_J, hi and lo).  Against 128 x 128 tiles of four 64 x 64
// wavefronts, a 32-column chunk costs a compute unit 192 KB of LDS operand
// reads and 64 KB of staging writes (2048 LDS cycles) for 3072 cycles of
// matrix-core work per SIMD, where the 128-wide tiles load LDS and matrix
// cores alike (1536 cycles each), and the tiles read half the split rows of
// X per output entry.
#pragma once

#include "syrk128.h"

namespace fpde {

constexpr int T256 = 256;
constexpr int kSuper256 = 4;  // super-blocks of 4 x 4 tiles

struct Split256Smem {
  half8 a[2][2][T256][KC16 / 8];
  half8 b[2][2][T256][KC16 / 8];
};
struct Syrk256Smem {
  union {
    Split256Smem g;
    DiagSmem d;
  };
};

// work items of one system: super-blocks of the lower 256 x 256 tiles of a
// trailing matrix of m rows
__host__ __device__ inline int64_t syrk256_slots(int64_t m) {
  const int64_t t2 = (m + T256 - 1) / T256, s2 = (t2 + kSuper256 - 1) / kSuper256;
  return s2 * (s2 + 1) / 2 * kSuper256 * kSuper256;
}

// acc[x][y] (wavefront tile rows 16 x.., columns 16 y..) = X_I X_J^T over KD
// columns from the split rows xi, xj (prow, qrow of them inside the matrix),
// 512 threads: wavefront w holds rows 128 (w >> 2).., columns 64 (w & 3)...
// Thread t stages row t >> 1, groups 2 (t & 1) and 2 (t & 1) + 1 of both
// planes (split_load / split_put).  One chunk is staged in registers: while
// chunk c is multiplied from one LDS buffer, chunk c + 1 (loaded during
// chunk c - 1) waits in registers for the end of the products, then goes to
// the other buffer, and chunk c + 2 is requested.  Result layout: lane l
// holds rows 4 (l >> 4) + i, column l & 15 of each 16 x 16 tile.
template <int KD>
__device__ __forceinline__ void product_split256(const _Float16 *__restrict__ xi, const _Float16 *__restrict__ xj,
                                                 int prow, int qrow, Split256Smem &sm, f32x4v (&acc)[8][4]) {
  static_assert(KD % KC16 == 0, "split rows hold whole chunks");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 2, wc = w & 3;
  const int rr = t >> 1;
  const bool plive = rr < prow, qlive = rr < qrow;
  const _Float16 *pr = xi + (int64_t)(plive ? rr : prow - 1) * (2 * KD);
  const _Float16 *qr = xj + (int64_t)(qlive ? rr : qrow - 1) * (2 * KD);
#pragma unroll
  for (int x = 0; x < 8; x++)
#pragma unroll
    for (int y = 0; y < 4; y++) acc[x][y] = f32x4v{0.f, 0.f, 0.f, 0.f};
  SplitChunk pc, qc;
  split_load<KD>(pr, 0, pc);
  split_load<KD>(qr, 0, qc);
  split_put(pc, plive, sm.a[0][0], sm.a[0][1]);
  split_put(qc, qlive, sm.b[0][0], sm.b[0][1]);
  if (KC16 < KD) {
    split_load<KD>(pr, KC16, pc);
    split_load<KD>(qr, KC16, qc);
  }
  __syncthreads();
  const int q = lane >> 4;
#pragma unroll 1
  for (int kk = 0; kk < KD; kk += KC16) {
    const int buf = (kk / KC16) & 1;
    half8 bh[4], bl[4];
#pragma unroll
    for (int y = 0; y < 4; y++) {
      const int br = 64 * wc + 16 * y + (lane & 15);
      bh[y] = sm.b[buf][0][br][swz(br, q)];
      bl[y] = sm.b[buf][1][br][swz(br, q)];
    }
    // per 16-row block of the wavefront's rows: hi hi, hi lo, lo hi over
    // its four column tiles (consecutive operations write different
    // accumulators)
#pragma unroll
    for (int x = 0; x < 8; x++) {
      const int ar = 128 * wr + 16 * x + (lane & 15);
      const half8 ah = sm.a[buf][0][ar][swz(ar, q)];
      const half8 al = sm.a[buf][1][ar][swz(ar, q)];
#pragma unroll
      for (int y = 0; y < 4; y++) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[y], acc[x][y], 0, 0, 0);
#pragma unroll
      for (int y = 0; y < 4; y++) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[y], acc[x][y], 0, 0, 0);
#pragma unroll
      for (int y = 0; y < 4; y++) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[y], acc[x][y], 0, 0, 0);
    }
    if (kk + KC16 < KD) {
      // the other buffer was last read in the previous chunk, before the
      // barrier that ended it
      split_put(pc, plive, sm.a[buf ^ 1][0], sm.a[buf ^ 1][1]);
      split_put(qc, qlive, sm.b[buf ^ 1][0], sm.b[buf ^ 1][1]);
      if (kk + 2 * KC16 < KD) {
        split_load<KD>(pr, kk + 2 * KC16, pc);
        split_load<KD>(qr, kk + 2 * KC16, qc);
      }
    }
    __syncthreads();
  }
}

// Trailing update over the lower 256 x 256 tiles of the region of the
// matrix from row/column base (at least k0 + KD), X = columns [k0, k0 + KD)
// as split rows (xs, from k_row_split) with per-row exponents (escale); with
// factor set, the workgroup of tile (0, 0) factors the 64 x 64 diagonal
// block at base.  Tiles in super-blocks
// of kSuper256 x kSuper256, in row-major lower-triangular order (items above
// the diagonal of a diagonal super-block or past the matrix end are empty),
// nwork = nz slots work items (item 0 of every system first, then system
// by system its other items); the grid is 8 ceil(nwork / 8) blocks
// dealt to the XCDs in contiguous ranges of b (xcd_deal).  An XCD runs 32
// workgroups at once, two super-blocks, which share their block rows of X.
template <int KD>
__global__ void __launch_bounds__(512) k_syrk256(float *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                 int64_t base, int factor, float *__restrict__ Linv_next,
                                                 float *__restrict__ LinvT_next,
                                                 int32_t *flag, int64_t *aux, int64_t sA, int64_t sL,
                                                 const int *__restrict__ escale, int64_t se,
                                                 const _Float16 *__restrict__ xs, int64_t sx, int nz,
                                                 int64_t nwork) {
  const int64_t bw = xcd_deal(blockIdx.x, gridDim.x);
  if (bw >= nwork) return;
  // the tiles (0, 0) of all systems first (they factor the next diagonal
  // blocks, on which the next panel waits), then each system's other items
  const int64_t slots = nwork / nz;
  int64_t z, x;
  if (bw < nz) {
    z = bw;
    x = 0;
  } else {
    z = (bw - nz) / (slots - 1);
    x = 1 + (bw - nz) % (slots - 1);
  }
  constexpr int S = kSuper256;
  const int64_t sb = x / (S * S), si = x % (S * S);
  int64_t P = (int64_t)((sqrt(8.0 * (double)sb + 1.0) - 1.0) * 0.5);
  while ((P + 1) * (P + 2) / 2 <= sb) P++;
  while (P * (P + 1) / 2 > sb) P--;
  const int64_t I = S * P + si / S, J = S * (sb - P * (P + 1) / 2) + si % S;
  if (J > I || base + T256 * I >= n) return;  // an empty item
  A += z * sA;
  Linv_next += z * sL;
  LinvT_next += z * sL;
  aux += z;
  __shared__ Syrk256Smem sm;
  const int64_t ri = base + T256 * I, cj = base + T256 * J;
  const int prow = (int)((n - ri) < T256 ? (n - ri) : T256);
  const int qrow = (int)((n - cj) < T256 ? (n - cj) : T256);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 2, wc = w & 3;
  const int *es = escale + z * se;
  const _Float16 *x0 = xs + z * sx;
  f32x4v acc[8][4];
  product_split256<KD>(x0 + ri * (2 * KD), x0 + cj * (2 * KD), prow, qrow, sm.g, acc);
  int ec[4];
#pragma unroll
  for (int b = 0; b < 4; b++) {
    const int c = 64 * wc + 16 * b + (lane & 15);
    ec[b] = es[cj + (c < qrow ? c : qrow - 1)];
  }
  auto frow = [&](int a, int i) { return 128 * wr + 16 * a + 4 * (lane >> 4) + i; };
  auto fcol = [&](int b) { return 64 * wc + 16 * b + (lane & 15); };
  // wavefront 0 of tile (0, 0) holds the next diagonal block in its rows
  // 0..63 (blocks a < 4), factored below; its other rows are stored
  const bool keepw = factor && x == 0 && w == 0;
  // a tile strictly below the diagonal and inside the matrix needs neither
  // clamped loads nor guarded stores: 32-bit offsets from this lane's first
  // entry (256 lda < 2^31)
  const bool interior = J < I && ri + T256 <= n && cj + T256 <= n;
#pragma unroll
  for (int a = 0; a < 8; a++) {
    int er[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = frow(a, i);
      er[i] = es[ri + (r < prow ? r : prow - 1)];
    }
    if (interior) {
      float *p0 = A + (ri + frow(a, 0)) * lda + cj + fcol(0);
      float cv[4][4];
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) cv[b][i] = p0[i * (int)lda + 16 * b];
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) p0[i * (int)lda + 16 * b] = cv[b][i] - ldexpf(acc[a][b][i], er[i] + ec[b]);
    } else if (!(keepw && a < 4)) {
      float cv[4][4];
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t r = ri + frow(a, i), c = cj + fcol(b);
          cv[b][i] = A[(r < n ? r : n - 1) * lda + (c < n ? c : n - 1)];
        }
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t r = ri + frow(a, i), c = cj + fcol(b);
          if (r < n && c < n && c <= r) A[r * lda + c] = cv[b][i] - ldexpf(acc[a][b][i], er[i] + ec[b]);
        }
    }
  }
  if (x != 0 || !factor) return;
  // tile (0, 0): stage the next diagonal block in LDS (lower part; identity
  // past the matrix end) and factor it
  __syncthreads();  // the product's LDS is free
  const int nb = prow < NB ? prow : NB;
  if (keepw) {
#pragma unroll
    for (int a = 0; a < 4; a++) {
      int er[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = frow(a, i);
        er[i] = es[ri + (r < prow ? r : prow - 1)];
      }
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int r = frow(a, i), c = fcol(b);
          double v;
          if (r < nb && c < nb) {
            const float cold = A[(ri + r) * lda + cj + c];
            v = (c <= r) ? (double)(cold - ldexpf(acc[a][b][i], er[i] + ec[b])) : 0.0;
          } else {
            v = (r == c) ? 1.0 : 0.0;
          }
          sm.d.L[r][c] = v;
        }
    }
  }
  __syncthreads();
  diag_factor<float>(sm.d, nb, A, lda, ri, Linv_next, LinvT_next, flag, aux);
}

}  // namespace fpde
