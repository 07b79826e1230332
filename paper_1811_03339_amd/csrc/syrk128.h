// Trailing update of the blocked Cholesky on 128 x 128 output tiles:
//   C[I, J] -= X_I X_J^T  over the lower tiles I >= J of the trailing matrix,
// X = the KD columns of the panels just factored (2048 for a whole group,
// 256 to 1024 inside one).  One
// workgroup per output tile reads and writes its tile of C once and streams
// X_I and X_J through LDS in chunks of the inner dimension, double-buffered:
// a 128-wide tile halves the reads of X per output entry compared with
// 64-wide tiles.
//
// Two arithmetic forms:
//  * FP64 storage: v_mfma_f64_16x16x4f64 tiles, 16-deep chunks; eight
//    wavefronts in a 2 x 4 arrangement (64 x 32 each, 4 x 2 accumulators of
//    16 x 16), so that a wavefront holds 64 accumulator registers and two
//    workgroups give every SIMD four wavefronts to cover barrier and LDS
//    waits (the FP64 matrix cores need few LDS bytes per operation).
//  * FP32 storage (the factor of the mixed-precision solve): split FP16 on
//    the FP16 matrix cores, 32-deep chunks; four wavefronts in a 2 x 2
//    arrangement (64 x 64 each: the split operands need twice the LDS bytes
//    per operation, and smaller wavefront tiles would make the LDS the
//    bound).  Row r of X is scaled by a power
//    of two 2^-e_r (e_r from the row's largest magnitude over the KD
//    columns, computed by k_row_split before the update) so that its largest
//    entry lies in [2^13, 2^14), then split as x = hi + lo with hi = fp16(x)
//    and lo = fp16(x - hi) (22 significant bits).  The product accumulates
//    hi hi^T + hi lo^T + lo hi^T in FP32 with v_mfma_f32_16x16x32_f16 (the
//    dropped lo lo^T term is below 2^-22 of each product) and the update is
//    C -= 2^(e_r + e_c) acc.  Entries far below their row's largest lose
//    relative precision in lo, but their absolute error stays below 2^-24
//    of that largest entry: the FP32 rounding of the stored factor.
//
// The workgroup of tile (0, 0) keeps the top-left 64 x 64 quadrant of its
// updated tile -- the next diagonal block -- and factors it at once
// (diag_factor), as the 64-wide trailing update does.
#pragma once

#include <type_traits>

#include "chol_diag.h"
#include "dense.h"

namespace fpde {

constexpr int T128 = 128;

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// The group's columns of X in split FP16, once per group (every trailing
// tile then stages them as they are): for each row r in [r0, n) of the KD
// columns at k0, the exponent e_r with max_k |A[r][k0 + k]| 2^-e_r in
// [2^13, 2^14) (e_r within [-110, 110], 0 for an all-zero row), and
// x 2^-e_r = hi + lo, hi = fp16(x 2^-e_r), lo = fp16(x 2^-e_r - hi), stored
// row-major: xs[r][0][k] = hi, xs[r][1][k] = lo (KD halfs each).  One
// wavefront per row, KD / 64 columns per lane; batch z = blockIdx.y (rows of
// system z at A + z sA, exponents at escale + z se, split rows at xs + z sx).
template <int KD>
__global__ void __launch_bounds__(256) k_row_split(const float *__restrict__ A, int64_t lda, int64_t n, int64_t r0,
                                                   int64_t k0, int *__restrict__ escale, _Float16 *__restrict__ xs,
                                                   int64_t sA, int64_t se, int64_t sx) {
  constexpr int PL = KD / 64;  // consecutive columns per lane
  const int lane = threadIdx.x & 63;
  const int64_t r = r0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  A += (int64_t)blockIdx.y * sA;
  escale += (int64_t)blockIdx.y * se;
  xs += (int64_t)blockIdx.y * sx;
  if (r >= n) return;
  float v[PL];
  float mx = 0.f;
#pragma unroll
  for (int j = 0; j < PL; j++) {
    v[j] = A[r * lda + k0 + PL * lane + j];
    mx = fmaxf(mx, fabsf(v[j]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  int e = mx > 0.f ? ilogbf(mx) - 13 : 0;
  e = e < -110 ? -110 : (e > 110 ? 110 : e);
  if (lane == 0) escale[r] = e;
  _Float16 hi[PL], lo[PL];
#pragma unroll
  for (int j = 0; j < PL; j++) {
    const float x = ldexpf(v[j], -e);
    hi[j] = (_Float16)x;
    lo[j] = (_Float16)(x - (float)hi[j]);
  }
  _Float16 *row = xs + r * (2 * KD);
#pragma unroll
  for (int j = 0; j < PL; j++) {
    row[PL * lane + j] = hi[j];
    row[KD + PL * lane + j] = lo[j];
  }
}

// Split FP16 chunks: [buffer][hi, lo][row][k], 32 halfs per row (64 bytes).
// The four 16-byte groups of a row (k 8q..8q+7, q < 4) sit at group q ^ h(row),
// h = (r1 ^ r2) | (r1 ^ r3) << 1 over the bits r_i of the row.  A 16-byte
// read or write is served a few lanes at a time; h makes every such set
// of lanes hit distinct 16-byte slots, both for 8 lanes in a 128-byte
// window and for 16 lanes in a 256-byte window: reads of 16 consecutive
// rows (one q), and the staging writes (two lanes per row, groups
// 2 (t & 1) + g).
constexpr int KC16 = 32;
// The arrays are declared as 16-byte groups so that every operand read and
// staging write is one ds_read_b128 / ds_write_b128 (with _Float16 arrays
// the compiler cannot prove the alignment of a swizzled address and splits
// the reads into ds_read2_b64, whose 8-byte halves conflict).
struct Split16Smem {
  half8 a[2][2][T128][KC16 / 8];
  half8 b[2][2][T128][KC16 / 8];
};
// group slot of 16-byte group q in row `row`
__device__ __forceinline__ int swz(int row, int q) {
  return q ^ ((((row >> 1) ^ (row >> 2)) & 1) | ((((row >> 1) ^ (row >> 3)) & 1) << 1));
}

// FP64 chunks: [buffer][row][k], padded to an odd number of doubles per row
constexpr int KC64 = 16;
struct F64Smem {
  double a[2][T128][KC64 + 1];
  double b[2][T128][KC64 + 1];
};

// workgroup shape: WC wavefronts across the tile's columns (two down its
// rows), each holding BN 16-column blocks of its 64 rows
template <class T>
struct Syrk128Shape;
template <>
struct Syrk128Shape<float> {
  static constexpr int WC = 2, BN = 4, THREADS = 256;
};
template <>
struct Syrk128Shape<double> {
  static constexpr int WC = 4, BN = 2, THREADS = 512;
};

template <class T>
struct Syrk128Smem;
template <>
struct Syrk128Smem<float> {
  union {
    Split16Smem g;
    DiagSmem d;
  };
};
template <>
struct Syrk128Smem<double> {
  union {
    F64Smem g;
    DiagSmem d;
  };
};

// FP64 global loads of one 16-column chunk (512 threads), coalesced: the
// sixteen lanes of a row group read one 128-byte row segment; thread t reads
// column t & 15 of rows (t >> 4) + 32 it, it < 4.  Rows at or past the
// matrix end read a valid row and are zeroed when stored.
__device__ __forceinline__ int stage_row(int it) { return (threadIdx.x >> 4) + 32 * it; }

// element offsets (row r clamped into [0, rows)) * lda + this thread's
// column, for the four staged rows; they fit 32 bits (128 lda < 2^31)
__device__ __forceinline__ void stage_offsets(int rows, int64_t lda, int (&off)[4]) {
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int r = stage_row(it);
    off[it] = (r < rows ? r : rows - 1) * (int)lda + (threadIdx.x & 15);
  }
}

__device__ __forceinline__ void chunk_load(const double *__restrict__ P, const double *__restrict__ Q,
                                          const int (&po)[4], const int (&qo)[4], double (&pv)[4],
                                          double (&qv)[4]) {
#pragma unroll
  for (int it = 0; it < 4; it++) {
    pv[it] = P[po[it]];
    qv[it] = Q[qo[it]];
  }
}

// Staging of the split X: one chunk is, per row, 32 hi and 32 lo halfs
// (four 16-byte groups each).  Thread t moves groups 2 (t & 1) and
// 2 (t & 1) + 1 of both planes of row t >> 1 (rows past the tile's end read
// the last row and are zeroed).
struct SplitChunk {
  half8 v[4];  // [plane][group]: hi g0, hi g1, lo g0, lo g1
};

template <int KD>
__device__ __forceinline__ void split_load(const _Float16 *__restrict__ xrow, int kk, SplitChunk &c) {
  const int g0 = 2 * (threadIdx.x & 1);
#pragma unroll
  for (int pl = 0; pl < 2; pl++)
#pragma unroll
    for (int g = 0; g < 2; g++) c.v[2 * pl + g] = *(const half8 *)(xrow + pl * KD + kk + 8 * (g0 + g));
}

__device__ __forceinline__ void split_put(const SplitChunk &c, bool live, half8 (*hi)[KC16 / 8],
                                          half8 (*lo)[KC16 / 8]) {
  const int r = threadIdx.x >> 1, g0 = 2 * (threadIdx.x & 1);
  const half8 z = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int g = 0; g < 2; g++) {
    hi[r][swz(r, g0 + g)] = live ? c.v[g] : z;
    lo[r][swz(r, g0 + g)] = live ? c.v[2 + g] : z;
  }
}

// acc[a][b] (wavefront tile rows 16 a.., columns 16 b..) = X_I X_J^T over KD
// columns, split FP16, from the split rows xi (of X_I) and xj (of X_J).
// Result layout: lane l holds rows 4 (l >> 4) + i, column l & 15 of each
// 16 x 16 tile.
template <int KD>
__device__ __forceinline__ void product_split16(const _Float16 *__restrict__ xi, const _Float16 *__restrict__ xj,
                                                int prow, int qrow, Split16Smem &sm, f32x4v (&acc)[4][4]) {
  static_assert(KD % KC16 == 0, "split rows hold whole chunks");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  const int rr = t >> 1;
  const bool plive = rr < prow, qlive = rr < qrow;
  const _Float16 *pr = xi + (int64_t)(plive ? rr : prow - 1) * (2 * KD);
  const _Float16 *qr = xj + (int64_t)(qlive ? rr : qrow - 1) * (2 * KD);
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = f32x4v{0.f, 0.f, 0.f, 0.f};
  // Two chunks in flight: while chunk c is multiplied from LDS, chunk c + 1
  // (loaded during the previous chunk) is written to the other LDS buffer
  // and chunk c + 2 is loaded into registers.  The register sets A and B
  // alternate, so the loop body is unrolled by two.
  SplitChunk pA, qA, pB, qB;
  split_load<KD>(pr, 0, pA);
  split_load<KD>(qr, 0, qA);
  split_put(pA, plive, sm.a[0][0], sm.a[0][1]);
  split_put(qA, qlive, sm.b[0][0], sm.b[0][1]);
  if (KC16 < KD) {
    split_load<KD>(pr, KC16, pA);
    split_load<KD>(qr, KC16, qA);
  }
  __syncthreads();
  const int q = lane >> 4;
  auto step = [&](int kk, SplitChunk &pn, SplitChunk &qn, SplitChunk &pf, SplitChunk &qf) {
    const int buf = (kk / KC16) & 1;
    if (kk + 2 * KC16 < KD) {
      split_load<KD>(pr, kk + 2 * KC16, pf);
      split_load<KD>(qr, kk + 2 * KC16, qf);
    }
    half8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int x = 0; x < 4; x++) {
      const int ar = 64 * wr + 16 * x + (lane & 15), br = 64 * wc + 16 * x + (lane & 15);
      ah[x] = sm.a[buf][0][ar][swz(ar, q)];
      al[x] = sm.a[buf][1][ar][swz(ar, q)];
      bh[x] = sm.b[buf][0][br][swz(br, q)];
      bl[x] = sm.b[buf][1][br][swz(br, q)];
    }
    // hi hi, then hi lo, then lo hi over all 16 tiles: consecutive matrix-core
    // operations write different accumulators
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bh[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bl[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[a], bh[b], acc[a][b], 0, 0, 0);
    if (kk + KC16 < KD) {
      split_put(pn, plive, sm.a[buf ^ 1][0], sm.a[buf ^ 1][1]);
      split_put(qn, qlive, sm.b[buf ^ 1][0], sm.b[buf ^ 1][1]);
    }
    __syncthreads();
  };
#pragma unroll 1
  for (int kk = 0; kk < KD; kk += 2 * KC16) {
    step(kk, pA, qA, pB, qB);
    if (kk + KC16 < KD) step(kk + KC16, pB, qB, pA, qA);
  }
}

// The same product in FP64 on v_mfma_f64_16x16x4f64, eight wavefronts:
// wavefront w holds rows 64 (w >> 2).., columns 32 (w & 3)...  Result
// layout: lane l holds rows 4 i + (l >> 4), column l & 15 of each 16 x 16
// tile.
template <int KD>
__device__ __forceinline__ void product_f64(const double *__restrict__ P, const double *__restrict__ Q, int64_t lda,
                                            int prow, int qrow, F64Smem &sm, f64x4 (&acc)[4][2]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 2, wc = w & 3;
  const int c = t & 15;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  int po[4], qo[4];
  stage_offsets(prow, lda, po);
  stage_offsets(qrow, lda, qo);
  double pv[4], qv[4];
  chunk_load(P, Q, po, qo, pv, qv);
#pragma unroll
  for (int it = 0; it < 4; it++) {
    const int r = stage_row(it);
    sm.a[0][r][c] = r < prow ? pv[it] : 0.0;
    sm.b[0][r][c] = r < qrow ? qv[it] : 0.0;
  }
  __syncthreads();
  const int kq = lane >> 4;
#pragma unroll 1
  for (int kk = 0; kk < KD; kk += KC64) {
    const int buf = (kk / KC64) & 1;
    const bool more = kk + KC64 < KD;
    if (more) chunk_load(P + kk + KC64, Q + kk + KC64, po, qo, pv, qv);
#pragma unroll
    for (int k4 = 0; k4 < KC64; k4 += 4) {
      double av[4], bv[2];
#pragma unroll
      for (int x = 0; x < 4; x++) av[x] = sm.a[buf][64 * wr + 16 * x + (lane & 15)][k4 + kq];
#pragma unroll
      for (int y = 0; y < 2; y++) bv[y] = sm.b[buf][32 * wc + 16 * y + (lane & 15)][k4 + kq];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int it = 0; it < 4; it++) {
        const int r = stage_row(it);
        sm.a[buf ^ 1][r][c] = r < prow ? pv[it] : 0.0;
        sm.b[buf ^ 1][r][c] = r < qrow ? qv[it] : 0.0;
      }
    }
    __syncthreads();
  }
}

// Trailing update over the lower 128 x 128 tiles of the region of the
// matrix from row/column base (at least k0 + KD), with X = columns
// [k0, k0 + KD); with factor set, the workgroup of tile (0, 0) factors the
// 64 x 64 diagonal block at base.  ntc > 0: only the tiles of the region's
// first ntc tile columns (a strip; work items row by row, syrk128_strip_slots).
// ntc = 0: all its lower tiles, taken in super-blocks of kSuper x kSuper:
// super-block (P, Q), Q <= P, in
// row-major lower-triangular order, each kSuper^2 consecutive work items
// (tile rows 8 P + (s >> 3), columns 8 Q + (s & 7) for item s of the
// super-block); items above the diagonal of a diagonal super-block or past
// the matrix end are empty.  nwork = nz slots work items: first item 0 of
// every system, then system by system its items 1 .. slots - 1; the grid
// is 8 ceil(nwork / 8) blocks, dealt to the eight
// XCDs (which take workgroups round-robin) in contiguous ranges of b.  An
// XCD runs about 64 workgroups at once (32 compute units, two each): one
// super-block, whose tiles share 8 block rows and 8 block columns of X, so
// that each chunk of X that its L2 fetches serves eight tiles (64 tiles of
// one tile row would fetch 64 distinct blocks of X_J, each for one tile).
// FP32 only: escale and xs, the per-row exponents and split rows of X from
// k_row_split, system z at escale + z se and xs + z sx.
constexpr int kSuper = 8;
__device__ __forceinline__ int64_t xcd_deal(int64_t b, int64_t nblocks) {
  const int64_t per = nblocks / 8;  // nblocks is a multiple of 8
  return (b % 8) * per + b / 8;
}

// work items of one system: super-blocks of the lower tiles of a trailing
// matrix of m rows
__host__ __device__ inline int64_t syrk128_slots(int64_t m) {
  const int64_t t2 = (m + T128 - 1) / T128, s2 = (t2 + kSuper - 1) / kSuper;
  return s2 * (s2 + 1) / 2 * kSuper * kSuper;
}

// work items of one system in strip mode: the lower tiles of the first ntc
// tile columns of a trailing matrix of m rows (a triangle of ntc rows, then
// ntc per tile row; items of the triangle past the matrix end are empty)
__host__ __device__ inline int64_t syrk128_strip_slots(int64_t m, int ntc) {
  const int64_t t2 = (m + T128 - 1) / T128, tri = (int64_t)ntc * (ntc + 1) / 2;
  return t2 <= ntc ? tri : tri + (t2 - ntc) * ntc;
}

// FP64: the allocator is held to 128 registers (the 64 x 32 FP64
// accumulators take 64) so that two 512-thread workgroups (four wavefronts
// per SIMD, 2 x 68 KB of LDS) share a compute unit.
template <class T, int KD>
__global__ void __launch_bounds__(Syrk128Shape<T>::THREADS)
__attribute__((amdgpu_waves_per_eu(std::is_same<T, double>::value ? 4 : 1)))
k_syrk128(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0, int64_t base, int ntc, int factor,
          T *__restrict__ Linv_next, T *__restrict__ LinvT_next, int32_t *flag, int64_t *aux, int64_t sA,
          int64_t sL, const int *__restrict__ escale, int64_t se, const _Float16 *__restrict__ xs, int64_t sx,
          int nz, int64_t nwork) {
  constexpr bool F32 = std::is_same<T, float>::value;
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
  int64_t I, J;
  if (ntc > 0) {
    const int64_t tri = (int64_t)ntc * (ntc + 1) / 2;
    if (x < tri) {
      I = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
      while ((I + 1) * (I + 2) / 2 <= x) I++;
      while (I * (I + 1) / 2 > x) I--;
      J = x - I * (I + 1) / 2;
    } else {
      I = ntc + (x - tri) / ntc;
      J = (x - tri) % ntc;
    }
  } else {
    const int64_t sb = x / (kSuper * kSuper), si = x % (kSuper * kSuper);
    int64_t P = (int64_t)((sqrt(8.0 * (double)sb + 1.0) - 1.0) * 0.5);
    while ((P + 1) * (P + 2) / 2 <= sb) P++;
    while (P * (P + 1) / 2 > sb) P--;
    I = kSuper * P + si / kSuper;
    J = kSuper * (sb - P * (P + 1) / 2) + si % kSuper;
  }
  if (J > I || base + T128 * I >= n) return;  // an empty item
  A += z * sA;
  Linv_next += z * sL;
  LinvT_next += z * sL;
  aux += z;
  __shared__ Syrk128Smem<T> sm;
  const int64_t ri = base + T128 * I, cj = base + T128 * J;
  const int prow = (int)((n - ri) < T128 ? (n - ri) : T128);
  const int qrow = (int)((n - cj) < T128 ? (n - cj) : T128);
  constexpr int WC = Syrk128Shape<T>::WC, BN = Syrk128Shape<T>::BN, WCOL = T128 / WC;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w / WC, wc = w % WC;
  // the product: val(a, b, i) at tile row frow(a, i), column fcol(b)
  using Acc = std::conditional_t<F32, f32x4v, f64x4>;
  Acc acc[4][BN];
  int ec[BN] = {}, er[4][4] = {};
  if constexpr (F32) {
    const int *es = escale + z * se;
    const _Float16 *x0 = xs + z * sx;
    product_split16<KD>(x0 + ri * (2 * KD), x0 + cj * (2 * KD), prow, qrow, sm.g, acc);
#pragma unroll
    for (int b = 0; b < BN; b++) {
      const int c = WCOL * wc + 16 * b + (lane & 15);
      ec[b] = es[cj + (c < qrow ? c : qrow - 1)];
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = 64 * wr + 16 * a + 4 * (lane >> 4) + i;
        er[a][i] = es[ri + (r < prow ? r : prow - 1)];
      }
  } else {
    product_f64<KD>(A + ri * lda + k0, A + cj * lda + k0, lda, prow, qrow, sm.g, acc);
  }
  auto frow = [&](int a, int i) {
    return F32 ? 64 * wr + 16 * a + 4 * (lane >> 4) + i : 64 * wr + 16 * a + 4 * i + (lane >> 4);
  };
  auto fcol = [&](int b) { return WCOL * wc + 16 * b + (lane & 15); };
  auto val = [&](int a, int b, int i) -> T {
    if constexpr (F32) return ldexpf(acc[a][b][i], er[a][i] + ec[b]);
    else return acc[a][b][i];
  };
  // the next diagonal block (the tile's top-left 64 x 64), factored below
  const bool keep = factor && x == 0 && wr == 0 && WCOL * wc < NB;
  // a tile strictly below the diagonal and inside the matrix needs neither
  // clamped loads nor guarded stores: 32-bit offsets from this lane's first
  // entry (128 lda < 2^31)
  const bool interior = J < I && ri + T128 <= n && cj + T128 <= n;
  if (interior) {
    T *p0 = A + (ri + frow(0, 0)) * lda + cj + fcol(0);
#pragma unroll
    for (int a = 0; a < 4; a++) {
      T cv[BN][4];
#pragma unroll
      for (int b = 0; b < BN; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) cv[b][i] = p0[(frow(a, i) - frow(0, 0)) * (int)lda + 16 * b];
#pragma unroll
      for (int b = 0; b < BN; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) p0[(frow(a, i) - frow(0, 0)) * (int)lda + 16 * b] = cv[b][i] - val(a, b, i);
    }
  } else if (!keep) {
    // one block row of 16 at a time: its 16 entries of C loaded first
    // (indices clamped into the matrix), then updated and stored
#pragma unroll
    for (int a = 0; a < 4; a++) {
      T cv[BN][4];
#pragma unroll
      for (int b = 0; b < BN; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t r = ri + frow(a, i), c = cj + fcol(b);
          cv[b][i] = A[(r < n ? r : n - 1) * lda + (c < n ? c : n - 1)];
        }
#pragma unroll
      for (int b = 0; b < BN; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t r = ri + frow(a, i), c = cj + fcol(b);
          if (r < n && c < n && c <= r) A[r * lda + c] = cv[b][i] - val(a, b, i);
        }
    }
  }
  if (x != 0 || !factor) return;
  // tile (0, 0): the keep wavefronts hold the next 64 x 64 diagonal block;
  // stage it in LDS (lower part; identity past the matrix end) and factor it
  __syncthreads();  // the product's LDS is free
  const int nb = prow < NB ? prow : NB;
  if (keep) {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < BN; b++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int r = frow(a, i), c = fcol(b);
          double v;
          if (r < nb && c < nb) {
            const T cold = A[(ri + r) * lda + cj + c];
            v = (c <= r) ? (double)(cold - val(a, b, i)) : 0.0;
          } else {
            v = (r == c) ? 1.0 : 0.0;
          }
          sm.d.L[r][c] = v;
        }
  }
  __syncthreads();
  diag_factor<T>(sm.d, nb, A, lda, ri, Linv_next, LinvT_next, flag, aux);
}

}  // namespace fpde
