// Dense 64-wide building blocks shared by the Cholesky (SPD) and LU
// (non-symmetric) factorizations and their triangular solves: the tile
// product staged through LDS, wavefront helpers, and the block-row
// triangular solve with ticket ordering and per-block flags.
#pragma once

#include "fpde_internal.h"

namespace fpde {

constexpr int NB = 64;

// LDS written by some lanes of a wavefront and then read by other lanes of
// the same wavefront (the wavefront's LDS operations complete in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Forces v to be computed at this point of the program.
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

// Lane-dependent index whose comparisons the compiler must not hoist out of
// the enclosing loop (each hoisted comparison pins a 64-bit lane mask).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Staging of the 64 x 64 tile products P Q^T over a 64-deep inner dimension
// (P and Q given as row pointers with leading dimensions; rows past
// `prow`/`qrow` (>= 1) read as zero): 256 threads load rows lr + 8 it,
// column lc of a 32-deep chunk.  The second chunk's global loads are issued
// before the first chunk's arithmetic, and every load reads a valid address
// (rows clamped, then zeroed), so a thread's loads are all in flight
// together.
template <class T>
__device__ __forceinline__ void stage_load(const T *__restrict__ P, int64_t ldp, int prow, const T *__restrict__ Q,
                                           int64_t ldq, int qrow, int kk, int lr, int lc, T (&pr)[8], T (&qr)[8]) {
#pragma unroll
  for (int it = 0; it < 8; it++) {
    const int rr = lr + 8 * it;
    pr[it] = P[(int64_t)(rr < prow ? rr : prow - 1) * ldp + kk + lc];
    qr[it] = Q[(int64_t)(rr < qrow ? rr : qrow - 1) * ldq + kk + lc];
  }
}


typedef double f64x4 __attribute__((ext_vector_type(4)));

// acc += sP[rows][0..32) sQ[columns][0..32)^T for this wavefront's 32 x 32
// quarter (rows rm, rm + 16, columns cm, cm + 16 of the lane's 16-groups;
// kq = lane >> 4 picks the slice row of the 4-deep operands)
__device__ __forceinline__ void mfma_chunk(const double (*sP)[33], const double (*sQ)[33], int rm, int cm, int kq,
                                           f64x4 acc[2][2]) {
#pragma unroll
  for (int k4 = 0; k4 < 32; k4 += 4) {
    const double a0 = sP[rm][k4 + kq], a1 = sP[rm + 16][k4 + kq];
    const double b0 = sQ[cm][k4 + kq], b1 = sQ[cm + 16][k4 + kq];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ __forceinline__ void mfma_out(const f64x4 acc[2][2], double out[16]) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int i = 0; i < 4; i++) out[(2 * a + b) * 4 + i] = acc[a][b][i];
}

// The same 64 x 64 product on the matrix cores, FP64: wavefront w owns the
// 32 x 32 quarter (w >> 1, w & 1) as four 16 x 16 tiles, each accumulated
// by v_mfma_f64_16x16x4f64 over 4-deep slices of the inner dimension
// (A operand: lane l holds P[row l & 15][k + (l >> 4)]; B operand:
// Q[column l & 15][k + (l >> 4)]).  Result: out[(2 a + b) 4 + i] is tile
// (a, b) of the quarter at row 4 i + (l >> 4), column l & 15.
template <int KD = NB>
__device__ __forceinline__ void tile_nt_mfma(const double *__restrict__ P, int64_t ldp, int prow,
                                             const double *__restrict__ Q, int64_t ldq, int qrow, double (*sP)[33],
                                             double (*sQ)[33], double out[16]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lc = tid & 31, lr = tid >> 5;
  const int rm = 32 * (w >> 1) + (lane & 15), cm = 32 * (w & 1) + (lane & 15), kq = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double pr[8], qr[8];
  stage_load<double>(P, ldp, prow, Q, ldq, qrow, 0, lr, lc, pr, qr);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 32) {
#pragma unroll
    for (int it = 0; it < 8; it++) {
      const int rr = lr + 8 * it;
      sP[rr][lc] = rr < prow ? pr[it] : 0.0;
      sQ[rr][lc] = rr < qrow ? qr[it] : 0.0;
    }
    __syncthreads();
    if (kk + 32 < KD) stage_load<double>(P, ldp, prow, Q, ldq, qrow, kk + 32, lr, lc, pr, qr);
    mfma_chunk(sP, sQ, rm, cm, kq, acc);
    __syncthreads();
  }
  mfma_out(acc, out);
}

// 64 x 64 tile product over a KD-deep inner dimension (a multiple of 32)
// for the factorization kernels, on the matrix cores in FP64 and in FP32.  Value q of the 16 a thread holds sits at tile row
// frag_row<T>(q), column frag_col<T>(q).
template <int KD = NB>
__device__ __forceinline__ void tile_product(const double *__restrict__ P, int64_t ldp, int prow,
                                             const double *__restrict__ Q, int64_t ldq, int qrow, double (*sP)[33],
                                             double (*sQ)[33], double out[16]) {
  tile_nt_mfma<KD>(P, ldp, prow, Q, ldq, qrow, sP, sQ, out);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 on the matrix cores (v_mfma_f32_16x16x4f32), same quarters and
// operand layout as the FP64 product; this instruction's result is blocked:
// lane l holds rows 4 (l >> 4) + i, column l & 15 of each 16 x 16 tile.
template <int KD = NB>
__device__ __forceinline__ void tile_product(const float *__restrict__ P, int64_t ldp, int prow,
                                             const float *__restrict__ Q, int64_t ldq, int qrow, float (*sP)[33],
                                             float (*sQ)[33], float out[16]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lc = tid & 31, lr = tid >> 5;
  const int rm = 32 * (w >> 1) + (lane & 15), cm = 32 * (w & 1) + (lane & 15), kq = lane >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  float pr[8], qr[8];
  stage_load<float>(P, ldp, prow, Q, ldq, qrow, 0, lr, lc, pr, qr);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 32) {
#pragma unroll
    for (int it = 0; it < 8; it++) {
      const int rr = lr + 8 * it;
      sP[rr][lc] = rr < prow ? pr[it] : 0.f;
      sQ[rr][lc] = rr < qrow ? qr[it] : 0.f;
    }
    __syncthreads();
    if (kk + 32 < KD) stage_load<float>(P, ldp, prow, Q, ldq, qrow, kk + 32, lr, lc, pr, qr);
#pragma unroll
    for (int k4 = 0; k4 < 32; k4 += 4) {
      const float a0 = sP[rm][k4 + kq], a1 = sP[rm + 16][k4 + kq];
      const float b0 = sQ[cm][k4 + kq], b1 = sQ[cm + 16][k4 + kq];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int i = 0; i < 4; i++) out[(2 * a + b) * 4 + i] = acc[a][b][i];
}

template <class T>
__device__ __forceinline__ int frag_row(int q);
template <class T>
__device__ __forceinline__ int frag_col(int q);
template <>
__device__ __forceinline__ int frag_row<double>(int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 32 * (w >> 1) + 16 * (q >> 3) + 4 * (q & 3) + (lane >> 4);
}
template <>
__device__ __forceinline__ int frag_col<double>(int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 32 * (w & 1) + 16 * ((q >> 2) & 1) + (lane & 15);
}
template <>
__device__ __forceinline__ int frag_row<float>(int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 32 * (w >> 1) + 16 * (q >> 3) + 4 * (lane >> 4) + (q & 3);
}
template <>
__device__ __forceinline__ int frag_col<float>(int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 32 * (w & 1) + 16 * ((q >> 2) & 1) + (lane & 15);
}

// Element strides between the systems of a strided batch (grid.y = system):
// matrix, diagonal-block inverses, vectors, per-block flags, tickets.  All
// zero for a single system.
struct BatchStrides {
  int64_t a = 0, l = 0, v = 0, x = 0;  // v: right-hand side / solution, x: intermediate vector
  int f = 0, t = 0;
};
constexpr int kMaxBatch = 16;

constexpr int64_t kSpinLimit = int64_t(1) << 22;

// The blocks of a vector that the workgroups of one triangular-solve launch
// publish to each other are stored and loaded with relaxed device-scope
// atomic accesses, which are coherent across the XCDs' L2 caches by
// themselves: a publisher stores its block, waits until the stores have
// completed (s_waitcnt), then sets the block's flag with a relaxed
// device-scope store; a reader issues its loads of the block only after it
// has seen the flag.  No release or acquire fence is needed, so no L2
// write-back or invalidation (which would also evict the cached factor).
__device__ __forceinline__ double ld_dev(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// After a workgroup's st_dev stores: every store has completed, then the
// flag of block b carries `epoch` (thread 0).
__device__ __forceinline__ void publish_block(int *flags, int b, int epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[b], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole-wave poll of the flags of blocks c, c + dir, ..., (count <= 64 of
// them).  Returns how many leading ones carry `epoch` (>= 1), or 0 after
// kSpinLimit polls without flag c.  The polls are relaxed device-scope
// loads; the published blocks are then read with ld_dev.
__device__ __forceinline__ int poll_run(const int *flags, int c, int dir, int count, int epoch) {
  const int lane = threadIdx.x & 63;
  const int k = lane < count ? lane : count - 1;
  for (int64_t it = 0; it <= kSpinLimit; it++) {
    const int v = __hip_atomic_load(&flags[c + dir * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long pub = __ballot(v == epoch);
    if (pub & 1ull) {
      const unsigned long long gap = ~pub;
      const int run = gap ? __ffsll((long long)gap) - 1 : 64;
      return run < count ? run : count;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return 0;
}

// Sixteen per-lane values a[q] -> sum over the wave's 64 lanes of a[q], left
// in every lane with (lane >> 2) & 15 == q (butterfly that halves the
// vector at each exchange: 8 + 4 + 2 + 1 + 1 + 1 shuffles).
__device__ __forceinline__ double wave_sum16(const double (&a)[16]) {
  const int lane = threadIdx.x & 63;
  double b[8], c[4], d[2];
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 8; k++) b[k] = (h5 ? a[k + 8] : a[k]) + __shfl_xor(h5 ? a[k] : a[k + 8], 32, 64);
#pragma unroll
  for (int k = 0; k < 4; k++) c[k] = (h4 ? b[k + 4] : b[k]) + __shfl_xor(h4 ? b[k] : b[k + 4], 16, 64);
#pragma unroll
  for (int k = 0; k < 2; k++) d[k] = (h3 ? c[k + 2] : c[k]) + __shfl_xor(h3 ? c[k] : c[k + 2], 8, 64);
  double e = (h2 ? d[1] : d[0]) + __shfl_xor(h2 ? d[0] : d[1], 4, 64);
  e += __shfl_xor(e, 2, 64);
  e += __shfl_xor(e, 1, 64);
  return e;
}

// Block-row triangular solve in one launch:
//   x_b = D_b^{-1} (y_b - sum_{c in S(b)} A_bc x_c),
// S(b) = {c < b} (UP = false, block rows handed out top to bottom) or
// {c > b} (UP = true, bottom to top); DinvT holds (D_b^{-1})^T, 64 x 64
// row-major per block.  Used for L (Cholesky forward; LU forward with the
// unit lower factor) and U (LU backward), all read by block rows, so the
// loads of A are whole 64-wide row segments.  Each workgroup takes the next
// block row from an atomic ticket, so it only waits for block rows whose
// tickets were taken before its own by workgroups that are already running.
// Wave w owns rows 16w..16w+15 of the block row; lane = column within
// block c.
template <class T, bool UP>
__global__ void __launch_bounds__(256) k_trsv_rows(const T *__restrict__ A, int64_t lda, int64_t n, int nblk,
                                                   const T *__restrict__ DinvT, const double *__restrict__ y,
                                                   double *__restrict__ x, int *flags, int *ticket, int epoch,
                                                   int32_t *err, BatchStrides bs) {
  __shared__ int sb, ok;
  __shared__ double rhs[NB];
  __shared__ double red[4][NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {
    const int64_t z = blockIdx.y;  // system z of a strided batch (its own tickets and flags)
    A += z * bs.a;
    DinvT += z * bs.l;
    y += z * bs.v;
    x += z * bs.x;
    flags += z * bs.f;
    ticket += z * bs.t;
  }
  if (tid == 0) {
    sb = atomicAdd(ticket, 1);
    ok = 1;
  }
  __syncthreads();
  if (sb >= nblk) return;
  const int b = UP ? nblk - 1 - sb : sb;
  const int nc = UP ? nblk - 1 - b : b;  // blocks of S(b)
  const int c_first = UP ? nblk - 1 : 0, step = UP ? -1 : 1;
  const int64_t r0 = (int64_t)b * NB;
  const int nb = (int)((n - r0) < NB ? (n - r0) : NB);
  // D_b^{-1}[lane][16w + q], read before any wait
  double li[16];
#pragma unroll
  for (int q = 0; q < 16; q++) li[q] = (double)DinvT[(int64_t)b * NB * NB + (int64_t)(16 * w + q) * NB + lane];
  int64_t roff[16];  // rows past the matrix end repeat the last row; their sums are dropped
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int r = 16 * w + q;
    roff[q] = (r0 + (r < nb ? r : nb - 1)) * lda;
  }
  // column of block c read by this lane (only the last block can be
  // partial: its missing columns load a valid entry and multiply zero)
  auto col_of = [&](int c) {
    const int64_t cc = (int64_t)c * NB + lane;
    return cc < n ? cc : n - 1;
  };
  double part[16];
  T cur[16];
#pragma unroll
  for (int q = 0; q < 16; q++) {
    part[q] = 0.0;
    cur[q] = (T)0;
  }
  if (nc > 0) {
    const int64_t cc = col_of(c_first);
#pragma unroll
    for (int q = 0; q < 16; q++) cur[q] = A[roff[q] + cc];
  }
  bool good = true;
  int ready = 0;  // the first `ready` blocks of S(b), in visiting order, are published
  for (int it = 0; it < nc; it++) {
    const int c = c_first + step * it;
    if (it >= ready) {
      const int k = poll_run(flags, c, step, (nc - it) < 64 ? (nc - it) : 64, epoch);
      if (k == 0) {
        good = false;
        break;
      }
      ready = it + k;
    }
    const int64_t cc = (int64_t)c * NB + lane;
    const double xv = cc < n ? ld_dev(&x[cc]) : 0.0;
    const int64_t cn = col_of(it + 1 < nc ? c + step : c);
    T nxt[16];
#pragma unroll
    for (int q = 0; q < 16; q++) nxt[q] = A[roff[q] + cn];
#pragma unroll
    for (int q = 0; q < 16; q++) {
      part[q] = fma((double)cur[q], xv, part[q]);
      cur[q] = nxt[q];
    }
  }
  if (!good && lane == 0) ok = 0;
  const double sum = wave_sum16(part);
  if ((lane & 3) == 0) {
    const int r = 16 * w + (lane >> 2);
    rhs[r] = (r < nb) ? y[r0 + r] - sum : 0.0;
  }
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; q++) s = fma(li[q], rhs[16 * w + q], s);
  red[w][lane] = s;
  __syncthreads();
  // the block of x, written by wavefront 0 and published
  if (tid < nb) st_dev(&x[r0 + tid], (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
  publish_block(flags, b, epoch);
  if (tid == 0 && !ok) set_flag(err, FPDE_EHIP);
}

// Host helpers (solve.hip).
// Device buffer of `sets` x ceil(n / 64) inverses of 64 x 64 diagonal blocks
// (elements of `elem` bytes), kept in the mesh handle and grown on demand.
int ensure_linv(fpde_mesh *m, int64_t n, size_t elem, int sets, void **out);
// Per-block flags (two sets of nblk) and two tickets for the solves.
// per-system flags (2 nblk each) then tickets (2 each) for `count` systems
int ensure_trsv_sync(fpde_mesh *m, int nblk, hipStream_t s, int count = 1);
// p[0..n) = 0 with a kernel (no memset node when a caller captures a graph).
int zero_ints(int *p, int n, hipStream_t s);

}  // namespace fpde
