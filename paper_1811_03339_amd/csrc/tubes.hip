// Accumulation of the dense stiffness matrix by tubes (Sec. 2.1 assembly,
// Sec. 2.3 sparsity).
//
// Every Gauss point g and axis i contribute the rank-2 update
//   A += w_g K_i c_alpha (l r^T + r l^T)
// where l and r are the derivative vectors of the two half-rays of the
// chord through x_g parallel to e_i.  Chords of nearby Gauss points run
// through nearly the same elements, so the pairs (g, i) are grouped into
// tubes: axis i and the square cell of the plane orthogonal to e_i that
// holds x_g.  A tube's chords touch a small node set U_T (the union of its
// half-rays' entries), and its whole contribution is a dense |U_T| x |U_T|
// block.
//
//   plan (once per mesh and rule, independent of alpha and K):
//     tubes, the sorted node list U_T of each tube, for every entry its slot
//     (position of its node in U_T), and for every row the (tube, slot)
//     places where that node appears;
//   pass 1: one workgroup per (tube, band of block rows) reads the tube's
//     entries once and adds every product l_p r_q into an LDS band of the
//     block; the band goes to a scratch block in HBM.  The block is
//     symmetric, B = S + S^T with S = sum w l r^T, so a tube that fits in
//     LDS whole (the square for |U_T| <= 141, else the packed upper
//     triangle for |U_T| <= 200) is one band that adds each product of S
//     once, at (min, max), and expands it as it writes;
//   pass 2: one workgroup per row of A sums that row's slices of the tube
//     blocks into an LDS row and writes the row once.
// Each entry is read once per band of its tube (not once per node of its
// partner half-ray), and A is written once, without global atomics.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kHash = 8192;         // LDS hash slots per tube (int32 keys)
constexpr int kMaxU = kHash / 2;    // largest node set a tube may have
constexpr int kBandDoubles = 20160;  // LDS doubles of one pass-1 band (157.5 KB: the packed triangle of |U_T| <= 200)

// row stride of a band in LDS: odd, so the rows of one column fall in distinct bank pairs
__host__ __device__ inline int band_stride(int U) { return U | 1; }

// A tube whose packed upper triangle fits in LDS is one band (its whole
// block); a larger one is cut into bands of full rows.
__host__ __device__ inline int band_rows(int U) {
  if (U <= 0) return 1;
  if ((int64_t)U * (U + 1) / 2 <= kBandDoubles) return U;
  const int R = kBandDoubles / band_stride(U);
  return R < U ? R : U;
}

// position of (lo, hi), lo <= hi, in the row-packed upper triangle of a
// U x U block: tri_base(lo, U) + hi
__host__ __device__ inline int tri_base(int lo, int U) { return lo * (2 * U - lo + 1) / 2 - lo; }

inline unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Pair id P = i * G + g.  Key = tube cell of x_g in the plane orthogonal to
// e_i; x_g summed in the walk's order ((0 + b0 v0) + b1 v1) + ...
__global__ void k_pair_keys(const int32_t *__restrict__ tet, const double *__restrict__ xyz,
                            const double *__restrict__ qbary, int nq, int64_t G, double lo0, double lo1, double lo2,
                            double inv_c, int ncell, uint32_t *__restrict__ key, int32_t *__restrict__ val) {
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= 3 * G) return;
  const int i = (int)(P / G);
  const int64_t g = P - (int64_t)i * G;
  const int64_t t = g / nq;
  const int q = (int)(g - t * nq);
  double x[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < 4; m++) {
    const double b = qbary[4 * q + m];
    const double *v = xyz + 3 * (int64_t)tet[4 * t + m];
    for (int d = 0; d < 3; d++) x[d] = x[d] + b * v[d];
  }
  const double lo[3] = {lo0, lo1, lo2};
  const int a1 = (i + 1) % 3, a2 = (i + 2) % 3;
  int c1 = (int)floor((x[a1] - lo[a1]) * inv_c), c2 = (int)floor((x[a2] - lo[a2]) * inv_c);
  c1 = c1 < 0 ? 0 : (c1 >= ncell ? ncell - 1 : c1);
  c2 = c2 < 0 ? 0 : (c2 >= ncell ? ncell - 1 : c2);
  key[P] = ((uint32_t)i * (uint32_t)ncell + (uint32_t)c1) * (uint32_t)ncell + (uint32_t)c2;
  val[P] = (int32_t)P;
}

__global__ void k_heads(const uint32_t *__restrict__ key, int64_t n, int32_t *__restrict__ head) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) head[k] = (k == 0 || key[k] != key[k - 1]) ? 1 : 0;
}

// tube_off[T] = first sorted position of tube T; tube_off[n_tubes] = n
__global__ void k_tube_off(const int32_t *__restrict__ head, const int32_t *__restrict__ tid, int64_t n,
                           int64_t *__restrict__ tube_off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && head[k]) tube_off[tid[k]] = k;
  if (k == n - 1) tube_off[tid[k] + head[k]] = n;
}

// per sorted pair: {l first entry, r first entry, |l|, |r| | axis << 30} and w_g
__global__ void k_pair_meta(const int32_t *__restrict__ pair_sorted, int64_t n, int64_t G, int nq,
                            const int64_t *__restrict__ off, const double *__restrict__ qw,
                            const double *__restrict__ vol, int4 *__restrict__ pm, double *__restrict__ pw) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t P = pair_sorted[k];
  const int i = (int)(P / G);
  const int64_t g = P - (int64_t)i * G;
  const int64_t hl = (int64_t)(2 * i) * G + g, hr = hl + G;
  int4 m;
  m.x = (int)off[hl];
  m.y = (int)off[hr];
  m.z = (int)(off[hl + 1] - off[hl]);
  m.w = (int)(off[hr + 1] - off[hr]) | (i << 30);
  pm[k] = m;
  const int64_t t = g / nq;
  pw[k] = qw[g - t * nq] * vol[t];
}

__device__ __forceinline__ unsigned hash_slot(int32_t d) { return ((uint32_t)d * 2654435761u) >> (32 - 13); }

// insert every node of the tube's entries into the LDS hash; returns through
// `cnt` the number of distinct nodes (kMaxU + 1 on overflow)
__device__ void tube_insert(int32_t *hk, int *cnt, const int4 *__restrict__ pm, int64_t k0, int64_t k1,
                            const int32_t *__restrict__ ent_dof) {
  for (int j = threadIdx.x; j < kHash; j += blockDim.x) hk[j] = -1;
  if (threadIdx.x == 0) *cnt = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t k = k0 + wave; k < k1; k += nw) {
    const int4 m = pm[k];
    const int nl = m.z, nr = m.w & 0x3fffffff;
    for (int e = lane; e < nl + nr; e += 64) {
      const int32_t d = ent_dof[e < nl ? m.x + e : m.y + (e - nl)];
      unsigned h = hash_slot(d);
      for (int probe = 0; probe < kHash; probe++) {
        const int32_t old = atomicCAS(&hk[h], -1, d);
        if (old == -1) {
          atomicAdd(cnt, 1);
          break;
        }
        if (old == d) break;
        h = (h + 1) & (kHash - 1);
      }
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_tube_count(const int64_t *__restrict__ tube_off, const int4 *__restrict__ pm,
                                                    const int32_t *__restrict__ ent_dof, int64_t *__restrict__ u_cnt,
                                                    int32_t *flag) {
  __shared__ int32_t hk[kHash];
  __shared__ int cnt;
  const int64_t T = blockIdx.x;
  tube_insert(hk, &cnt, pm, tube_off[T], tube_off[T + 1], ent_dof);
  if (threadIdx.x == 0) {
    u_cnt[T] = cnt;
    if (cnt > kMaxU) set_flag(flag, FPDE_EUNSUPPORTED);
  }
}

// U_T sorted, the slot of every entry, and per-row counts of (tube, slot) places
__global__ void __launch_bounds__(256) k_tube_fill(const int64_t *__restrict__ tube_off, const int4 *__restrict__ pm,
                                                   const int32_t *__restrict__ ent_dof,
                                                   const int64_t *__restrict__ u_off, int32_t *__restrict__ tube_u,
                                                   int32_t *__restrict__ ent_slot, int64_t *__restrict__ row_cnt) {
  __shared__ int32_t hk[kHash];
  __shared__ int32_t su[kMaxU];
  __shared__ int cnt, cnt2;
  const int64_t T = blockIdx.x;
  const int64_t k0 = tube_off[T], k1 = tube_off[T + 1];
  tube_insert(hk, &cnt, pm, k0, k1, ent_dof);
  const int U = cnt;
  int P2 = 1;
  while (P2 < U) P2 <<= 1;
  if (threadIdx.x == 0) cnt2 = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < kHash; j += blockDim.x)
    if (hk[j] >= 0) su[atomicAdd(&cnt2, 1)] = hk[j];
  __syncthreads();
  for (int j = U + threadIdx.x; j < P2; j += blockDim.x) su[j] = 0x7fffffff;
  __syncthreads();
  // bitonic sort of su[0, P2)
  for (int size = 2; size <= P2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = threadIdx.x; j < P2; j += blockDim.x) {
        const int o = j ^ stride;
        if (o > j) {
          const bool up = (j & size) == 0;
          const int32_t x = su[j], y = su[o];
          if ((x > y) == up) {
            su[j] = y;
            su[o] = x;
          }
        }
      }
      __syncthreads();
    }
  const int64_t ub = u_off[T];
  for (int j = threadIdx.x; j < U; j += blockDim.x) {
    tube_u[ub + j] = su[j];
    atomicAdd((unsigned long long *)&row_cnt[su[j]], 1ull);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t k = k0 + wave; k < k1; k += nw) {
    const int4 m = pm[k];
    const int nl = m.z, nr = m.w & 0x3fffffff;
    for (int e = lane; e < nl + nr; e += 64) {
      const int64_t ei = e < nl ? m.x + e : m.y + (e - nl);
      const int32_t d = ent_dof[ei];
      int lo = 0, hi = U - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (su[mid] < d) lo = mid + 1;
        else hi = mid;
      }
      ent_slot[ei] = lo;
    }
  }
}

__global__ void k_row_places(const int64_t *__restrict__ u_off, int64_t n_tubes, const int32_t *__restrict__ tube_u,
                             int64_t *__restrict__ cursor, int2 *__restrict__ row_ts) {
  const int64_t T = blockIdx.x;
  if (T >= n_tubes) return;
  const int64_t u0 = u_off[T], U = u_off[T + 1] - u0;
  for (int64_t s = threadIdx.x; s < U; s += blockDim.x) {
    const int32_t d = tube_u[u0 + s];
    const unsigned long long pos = atomicAdd((unsigned long long *)&cursor[d], 1ull);
    row_ts[pos] = make_int2((int)T, (int)s);
  }
}

// pass-1 work items {tube, first block row, rows}
__global__ void k_bands(const int64_t *__restrict__ u_off, int64_t n_tubes, const int64_t *__restrict__ band_off,
                        int4 *__restrict__ items) {
  const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= n_tubes) return;
  const int U = (int)(u_off[T + 1] - u_off[T]);
  const int R = band_rows(U);
  int64_t w = band_off[T];
  for (int r0 = 0; r0 < U; r0 += R) items[w++] = make_int4((int)T, r0, (U - r0) < R ? (U - r0) : R, U);
}

__global__ void k_band_count(const int64_t *__restrict__ u_off, int64_t n_tubes, int64_t *__restrict__ nb,
                             int64_t *__restrict__ usq) {
  const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= n_tubes) return;
  const int64_t U = u_off[T + 1] - u_off[T];
  const int64_t R = band_rows((int)U);
  nb[T] = U > 0 ? (U + R - 1) / R : 0;
  usq[T] = U * U;
}

struct AccumArgs {
  const int64_t *tube_off;
  const int4 *pm;
  const double *pw;
  const int4 *items;
  const int32_t *ent_slot;
  const double *ent_val;
  const int64_t *blk_off;
  double *blk;
  double KC0, KC1, KC2;
  // general form (k_tube_form): test-order values and constant coefficients
  const double *val_b;
  double cl[3], cr[3];
};

__device__ __forceinline__ double read_lane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// A pair held in registers: entry `lane` and `lane + 64` of l and of r.
struct PairRegs {
  int4 m;
  double w;
  int ls[2], rs[2];
  double lv[2], rv[2];
};

constexpr int kRegEntries = 128;  // entries per half-ray the register path holds

__device__ __forceinline__ int pair_nl(const int4 &m) { return m.z; }
__device__ __forceinline__ int pair_nr(const int4 &m) { return m.w & 0x3fffffff; }

__device__ __forceinline__ void load_entries(PairRegs &p, const int32_t *__restrict__ slot,
                                             const double *__restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int nl = pair_nl(p.m), nr = pair_nr(p.m);
  // indices clamped to a valid entry (the pair's first, or entry 0 for an
  // empty side, whose offset may equal the entry count) so every load is in
  // bounds; lanes past the end are masked by the counts when used
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int kl = 64 * h + lane;
    const int il = nl > 0 ? p.m.x + (kl < nl ? kl : 0) : 0;
    const int ir = nr > 0 ? p.m.y + (kl < nr ? kl : 0) : 0;
    p.ls[h] = slot[il];
    p.lv[h] = val[il];
    p.rs[h] = slot[ir];
    p.rv[h] = val[ir];
  }
}

// Row-side entries one per lane (in-band ones active); the column side is
// swept one entry at a time, broadcast with readlane:
//   acc[s_row - r0][s_col] += v_row (w v_col).
// One LDS update per column touches one column of distinct rows: with an
// odd row stride these land in distinct bank pairs.
// Forces v to be computed at this point with the current (full) lane mask.
__device__ __forceinline__ void in_all_lanes(int &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void in_all_lanes(double &v) { asm volatile("" : "+v"(v)); }

// cv_reg already carries the pair weight; ncol is wave-uniform.  The column
// registers are read with readlane from lanes that may be masked off below:
// they are materialised in every lane before the branch (otherwise the
// compiler may sink their loads into it, leaving inactive lanes stale).
// Layouts of a pass-1 band in LDS:
//   kBand2: rows [r0, r0 + R) of the block, row stride Up; both products of
//           every pair (acc[rowbase + cs], rowbase = (xs - r0) Up);
//   kSquare1: the whole block, row stride Up, each product once at
//           (min, max) (lo Up + hi);
//   kTri1: the whole block as a row-packed upper triangle, each product once
//           at tri_base(lo, U) + hi (rowbase = tri_base(xs, U)).
// With the odd stride, the rows of one column sweep fall in distinct bank
// pairs in kBand2 and kSquare1 (stride Up when xs < cs, consecutive when
// xs > cs).
enum BandLayout { kBand2 = 0, kSquare1 = 1, kTri1 = 2 };

template <int LAYOUT>
__device__ __forceinline__ void sweep_cols(double *acc, int rowbase, int xs, int U, int Up, double xv, bool xok,
                                           int cs_reg, double cv_reg, int ncol) {
  in_all_lanes(cs_reg);
  in_all_lanes(cv_reg);
  if (xok) {
#pragma unroll 4
    for (int j = 0; j < ncol; j++) {
      const int cs = __builtin_amdgcn_readlane(cs_reg, j);
      const double cv = read_lane_f64(cv_reg, j);
      int idx;
      if (LAYOUT == kTri1) idx = xs <= cs ? rowbase + cs : tri_base(cs, U) + xs;
      else if (LAYOUT == kSquare1) idx = xs <= cs ? rowbase + cs : cs * Up + xs;
      else idx = rowbase + cs;
      atomicAdd(&acc[idx], xv * cv);
    }
  }
}

// one pair from registers (|l|, |r| <= kRegEntries).  kBand2: role 0 adds
// l (w r)^T, role 1 adds r (w l)^T to the rows in the band.  kSquare1,
// kTri1 (the whole block): role 0 only, each product at (min, max), which
// sums both roles (B = S + S^T, diagonal doubled when written).
template <int LAYOUT>
__device__ __forceinline__ void pair_products_reg(double *acc, int Up, int r0, int R, int U, const PairRegs &p) {
  const int lane = threadIdx.x & 63;
  // the pair is the wave's: its counts are uniform (scalar loop bounds)
  const int nl = __builtin_amdgcn_readfirstlane(pair_nl(p.m)), nr = __builtin_amdgcn_readfirstlane(pair_nr(p.m));
  // column-side values scaled by the pair weight once
  const double lw0 = p.lv[0] * p.w, lw1 = p.lv[1] * p.w, rw0 = p.rv[0] * p.w, rw1 = p.rv[1] * p.w;
#pragma unroll
  for (int role = 0; role < (LAYOUT == kBand2 ? 2 : 1); role++) {
    const int nrow = role ? nr : nl, ncol = role ? nl : nr;
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int xs = role ? p.rs[h] : p.ls[h];
      const double xv = role ? p.rv[h] : p.lv[h];
      const bool xok = 64 * h + lane < nrow && xs >= r0 && xs < r0 + R;
      if (__ballot(xok) == 0) continue;
      const int rowbase = LAYOUT == kTri1 ? tri_base(xs, U) : (xs - r0) * Up;
      sweep_cols<LAYOUT>(acc, rowbase, xs, U, Up, xv, xok, role ? p.ls[0] : p.rs[0], role ? lw0 : rw0,
                         ncol < 64 ? ncol : 64);
      if (ncol > 64)
        sweep_cols<LAYOUT>(acc, rowbase, xs, U, Up, xv, xok, role ? p.ls[1] : p.rs[1], role ? lw1 : rw1,
                           ncol - 64);
    }
  }
}

// the same from memory, for pairs with a longer half-ray
template <int LAYOUT>
__device__ void pair_products_mem(double *acc, int Up, int r0, int R, int U, const int4 m, double w,
                                  const int32_t *__restrict__ slot, const double *__restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int nl = __builtin_amdgcn_readfirstlane(pair_nl(m)), nr = __builtin_amdgcn_readfirstlane(pair_nr(m));
  for (int role = 0; role < (LAYOUT == kBand2 ? 2 : 1); role++) {
    const int nrow = role ? nr : nl, ncol = role ? nl : nr;
    const int erow = role ? m.y : m.x, ecol = role ? m.x : m.y;
    for (int j0 = 0; j0 < nrow; j0 += 64) {
      const int ex = erow + (j0 + lane < nrow ? j0 + lane : j0);
      const int xs = slot[ex];
      const double xv = val[ex];
      const bool xok = j0 + lane < nrow && xs >= r0 && xs < r0 + R;
      if (__ballot(xok) == 0) continue;
      const int rowbase = LAYOUT == kTri1 ? tri_base(xs, U) : (xs - r0) * Up;
      for (int c0 = 0; c0 < ncol; c0 += 64) {
        const int ec = ecol + (c0 + lane < ncol ? c0 + lane : c0);
        const int cn = ncol - c0 < 64 ? ncol - c0 : 64;
        sweep_cols<LAYOUT>(acc, rowbase, xs, U, Up, xv, xok, slot[ec], val[ec] * w, cn);
      }
    }
  }
}

__global__ void __launch_bounds__(1024) k_tube_accum(AccumArgs a) {
  extern __shared__ double acc[];
  const int4 it = a.items[blockIdx.x];
  const int64_t T = it.x;
  const int r0 = it.y, R = it.z, U = it.w, Up = band_stride(U);
  // B = S + S^T with S = sum_p w_p l_p r_p^T.  A tube that is one band
  // (band_rows) adds each product of S once, at (min, max): half the LDS
  // updates of the two products, in the full square when it fits (bank
  // conflict free), else in the packed upper triangle; a band of a larger
  // block takes both products into full rows.
  const int layout = R != U ? kBand2 : (U * Up <= kBandDoubles ? kSquare1 : kTri1);
  const int nacc = layout == kTri1 ? U * (U + 1) / 2 : R * Up;
  for (int j = threadIdx.x; j < nacc; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  // wave-uniform (readfirstlane), so the pair loop, its metadata and the
  // column sweeps are scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int64_t k0 = a.tube_off[T], k1 = a.tube_off[T + 1];
  auto meta = [&](int64_t k, PairRegs &p) {
    const int64_t kk = k < k1 ? k : k0;
    p.m = a.pm[kk];
    p.w = a.pw[kk];
  };
  // K_i c_alpha in registers (selected, not indexed, so no memory access sits
  // behind the pipelined loads)
  const double kc0 = a.KC0, kc1 = a.KC1, kc2 = a.KC2;
  auto weight = [kc0, kc1, kc2](const PairRegs &p) {
    const int axis = (int)((unsigned)p.m.w >> 30);
    return p.w * (axis == 0 ? kc0 : (axis == 1 ? kc1 : kc2));
  };
  // register path, software-pipelined: pair k in registers, the entries of
  // pair k + nw in flight, the metadata of pair k + 2 nw in flight (issued
  // first, so each wait leaves the newer loads outstanding)
  int64_t k = k0 + wave;
  bool long_pairs = false;
  if (k < k1) {
    PairRegs cur, nxt, far;
    meta(k, cur);
    load_entries(cur, a.ent_slot, a.ent_val);
    meta(k + nw, nxt);
    while (k < k1) {
      meta(k + 2 * nw, far);
      load_entries(nxt, a.ent_slot, a.ent_val);
      PairRegs p = cur;
      p.w = weight(cur);
      if (pair_nl(p.m) <= kRegEntries && pair_nr(p.m) <= kRegEntries) {
        if (layout == kSquare1) pair_products_reg<kSquare1>(acc, Up, r0, R, U, p);
        else if (layout == kTri1) pair_products_reg<kTri1>(acc, Up, r0, R, U, p);
        else pair_products_reg<kBand2>(acc, Up, r0, R, U, p);
      } else {
        long_pairs = true;
      }
      cur = nxt;
      nxt = far;
      k += nw;
    }
  }
  // pairs with a half-ray longer than the register path holds
  if (__ballot(long_pairs)) {
    for (k = k0 + wave; k < k1; k += nw) {
      PairRegs p;
      meta(k, p);
      if (pair_nl(p.m) > kRegEntries || pair_nr(p.m) > kRegEntries)
        if (layout == kSquare1) pair_products_mem<kSquare1>(acc, Up, r0, R, U, p.m, weight(p), a.ent_slot, a.ent_val);
        else if (layout == kTri1) pair_products_mem<kTri1>(acc, Up, r0, R, U, p.m, weight(p), a.ent_slot, a.ent_val);
        else pair_products_mem<kBand2>(acc, Up, r0, R, U, p.m, weight(p), a.ent_slot, a.ent_val);
    }
  }
  __syncthreads();
  double *out = a.blk + a.blk_off[T] + (int64_t)r0 * U;
  if (layout != kBand2) {
    for (int j = threadIdx.x; j < U * U; j += blockDim.x) {
      const int i = j / U, t = j - i * U;
      const int lo = i < t ? i : t, hi = i < t ? t : i;
      const double v = acc[(layout == kTri1 ? tri_base(lo, U) : lo * Up) + hi];
      out[j] = i == t ? v + v : v;
    }
  } else {
    for (int j = threadIdx.x; j < R * U; j += blockDim.x) {
      const int i = j / U, t = j - i * U;
      out[j] = acc[i * Up + t];
    }
  }
}

// General form with constant coefficients (Sec. 1, the test operator on
// the side opposite to the trial one): per pair, with l / r the left / right
// half-rays, the trial values at orders alpha (a.ent_val) and the test
// values at orders beta (a.val_b),
//   B[k][l] += w cl_i r_beta[k] l_alpha[l] + w cr_i l_beta[k] r_alpha[l]
// (rows: test node, columns: trial node).  Not symmetric, so both products
// of every pair go into full rows; an item is processed in row bands that
// fit the square layout, the pairs re-read per band.
__device__ void form_products_mem(double *acc, int Up, int rb, int Rb, const int4 m, double wl, double wr,
                                  const int32_t *__restrict__ slot, const double *__restrict__ va,
                                  const double *__restrict__ vb) {
  const int lane = threadIdx.x & 63;
  const int nl = __builtin_amdgcn_readfirstlane(pair_nl(m)), nr = __builtin_amdgcn_readfirstlane(pair_nr(m));
  for (int role = 0; role < 2; role++) {
    // role 0: rows r (beta), columns l (alpha, w cl); role 1: rows l, columns r (w cr)
    const int nrow = role ? nl : nr, ncol = role ? nr : nl;
    const int erow = role ? m.x : m.y, ecol = role ? m.y : m.x;
    const double w = role ? wr : wl;
    for (int j0 = 0; j0 < nrow; j0 += 64) {
      const int ex = erow + (j0 + lane < nrow ? j0 + lane : j0);
      const int xs = slot[ex];
      const double xv = vb[ex];
      const bool xok = j0 + lane < nrow && xs >= rb && xs < rb + Rb;
      if (__ballot(xok) == 0) continue;
      for (int c0 = 0; c0 < ncol; c0 += 64) {
        const int ec = ecol + (c0 + lane < ncol ? c0 + lane : c0);
        const int cn = ncol - c0 < 64 ? ncol - c0 : 64;
        sweep_cols<kBand2>(acc, (xs - rb) * Up, xs, 0, Up, xv, xok, slot[ec], va[ec] * w, cn);
      }
    }
  }
}

__global__ void __launch_bounds__(1024) k_tube_form(AccumArgs a) {
  extern __shared__ double acc[];
  const int4 it = a.items[blockIdx.x];
  const int64_t T = it.x;
  const int r0 = it.y, R = it.z, U = it.w, Up = band_stride(U);
  const int Rsq = kBandDoubles / Up;  // rows of one square band (>= 39 for |U_T| <= 512)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t k0 = a.tube_off[T], k1 = a.tube_off[T + 1];
  for (int rb = r0; rb < r0 + R; rb += Rsq) {
    const int Rb = (r0 + R - rb) < Rsq ? (r0 + R - rb) : Rsq;
    for (int j = threadIdx.x; j < Rb * Up; j += blockDim.x) acc[j] = 0.0;
    __syncthreads();
    for (int64_t k = k0 + wave; k < k1; k += nw) {
      PairRegs p;
      p.m = a.pm[k];
      p.w = a.pw[k];
      const int axis = (int)((unsigned)p.m.w >> 30);
      const double wl = p.w * (axis == 0 ? a.cl[0] : (axis == 1 ? a.cl[1] : a.cl[2]));
      const double wr = p.w * (axis == 0 ? a.cr[0] : (axis == 1 ? a.cr[1] : a.cr[2]));
      const int nl = __builtin_amdgcn_readfirstlane(pair_nl(p.m)), nr = __builtin_amdgcn_readfirstlane(pair_nr(p.m));
      if (nl > kRegEntries || nr > kRegEntries) {
        form_products_mem(acc, Up, rb, Rb, p.m, wl, wr, a.ent_slot, a.ent_val, a.val_b);
        continue;
      }
      // entries `lane` and `lane + 64` of both sides, both value sets
      // (indices clamped to a valid entry; lanes past the end are masked)
      int ls[2], rs[2];
      double la[2], ra[2], lb[2], rbv[2];
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int kl = 64 * h + lane;
        const int il = nl > 0 ? p.m.x + (kl < nl ? kl : 0) : 0;
        const int ir = nr > 0 ? p.m.y + (kl < nr ? kl : 0) : 0;
        ls[h] = a.ent_slot[il];
        rs[h] = a.ent_slot[ir];
        la[h] = a.ent_val[il];
        ra[h] = a.ent_val[ir];
        lb[h] = a.val_b[il];
        rbv[h] = a.val_b[ir];
      }
#pragma unroll
      for (int role = 0; role < 2; role++) {
        const int nrow = role ? nl : nr, ncol = role ? nr : nl;
        const double w = role ? wr : wl;
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int xs = role ? ls[h] : rs[h];
          const double xv = role ? lb[h] : rbv[h];
          const bool xok = 64 * h + lane < nrow && xs >= rb && xs < rb + Rb;
          if (__ballot(xok) == 0) continue;
          const int rowbase = (xs - rb) * Up;
          sweep_cols<kBand2>(acc, rowbase, xs, 0, Up, xv, xok, role ? rs[0] : ls[0], (role ? ra[0] : la[0]) * w,
                             ncol < 64 ? ncol : 64);
          if (ncol > 64)
            sweep_cols<kBand2>(acc, rowbase, xs, 0, Up, xv, xok, role ? rs[1] : ls[1], (role ? ra[1] : la[1]) * w,
                               ncol - 64);
        }
      }
    }
    __syncthreads();
    double *out = a.blk + a.blk_off[T] + (int64_t)rb * U;
    for (int j = threadIdx.x; j < Rb * U; j += blockDim.x) {
      const int i = j / U, t = j - i * U;
      out[j] = acc[i * Up + t];
    }
    __syncthreads();  // the band is written before the next one is cleared
  }
}

struct GatherArgs {
  const int64_t *row_off;
  const int2 *row_ts;
  const int64_t *u_off;
  const int32_t *tube_u;
  const int64_t *blk_off;
  const double *blk;
  // per tube, the first position in U_T of every column chunk: cstart[T
  // (nch + 1) + c] = #{nodes of U_T below c chunk} (U_T is increasing)
  const int32_t *cstart;
  int64_t ndof, lda;
  int chunk, nch;
};

// cstart for every (tube, chunk boundary): a binary search in U_T
__global__ void k_chunk_starts(const int64_t *__restrict__ u_off, const int32_t *__restrict__ tube_u, int64_t n_tubes,
                               int chunk, int nch, int32_t *__restrict__ cstart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tubes * (nch + 1)) return;
  const int64_t T = i / (nch + 1);
  const int64_t lim = (int64_t)(i % (nch + 1)) * chunk;
  int64_t lo = u_off[T], hi = u_off[T + 1];
  const int64_t first = lo;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (tube_u[mid] < lim) lo = mid + 1;
    else hi = mid;
  }
  cstart[i] = (int32_t)(lo - first);
}

__device__ __forceinline__ int64_t lane64(int64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Row `row`, column chunk ci ([c0, c0 + cw)) of K into the LDS chunk racc:
// the sum over the (tube, slot) places of the node of that slot's row of
// the tube block, scattered through U_T (one wavefront per place).  Only
// the part of the block row whose nodes fall in the chunk is read (U_T is
// increasing, so it is the range [cstart(T, ci), cstart(T, ci + 1))).  The
// places' metadata (tube, slot, node-set offset, block offset, range) is
// loaded 64 places at a time, one per lane, and broadcast from there.
// Ends with the chunk complete and visible to the whole workgroup.
__device__ __forceinline__ void gather_row_chunk(const GatherArgs &a, int64_t row, int ci, int64_t c0, int64_t cw,
                                                 double *racc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int64_t p0 = a.row_off[row], np = a.row_off[row + 1] - p0;
  for (int64_t j = threadIdx.x; j < cw; j += blockDim.x) racc[j] = 0.0;
  __syncthreads();
  for (int64_t pb = 0; pb < np; pb += 64) {
    int64_t u0 = 0, brow0 = 0;
    int t0 = 0, t1 = 0;
    if (pb + lane < np) {
      const int2 ts = a.row_ts[p0 + pb + lane];
      u0 = a.u_off[ts.x];
      const int64_t U = a.u_off[ts.x + 1] - u0;
      brow0 = a.blk_off[ts.x] + (int64_t)ts.y * U;
      const int32_t *cs = a.cstart + (int64_t)ts.x * (a.nch + 1) + ci;
      t0 = cs[0];
      t1 = cs[1];
    }
    const int cnt = (int)((np - pb) < 64 ? (np - pb) : 64);
    for (int k = wave; k < cnt; k += nwave) {
      const int64_t uk = lane64(u0, k);
      const double *brow = a.blk + lane64(brow0, k);
      const int tk1 = __builtin_amdgcn_readlane(t1, k);
      for (int t = __builtin_amdgcn_readlane(t0, k) + lane; t < tk1; t += 64)
        atomicAdd(&racc[(int64_t)a.tube_u[uk + t] - c0], brow[t]);
    }
  }
  __syncthreads();
}

// row of the dealt slot b: rows dealt XCD by XCD in contiguous ranges
// (workgroups go round-robin to the 8 XCDs)
__device__ __forceinline__ int64_t dealt_row(int64_t b, int64_t ndof) {
  const int64_t per_xcd = (ndof + 7) / 8;
  return (b % 8) * per_xcd + b / 8;
}

// A[p, :] = row p of K, written densely, once.
template <class TO>
__global__ void __launch_bounds__(256) k_tube_gather(GatherArgs a, TO *__restrict__ A) {
  extern __shared__ double racc[];
  const int64_t slots = 8 * ((a.ndof + 7) / 8);
  for (int64_t b = blockIdx.x; b < slots; b += gridDim.x) {
    const int64_t row = dealt_row(b, a.ndof);
    if (row >= a.ndof) continue;
    for (int ci = 0; ci < a.nch; ci++) {
      const int64_t c0 = (int64_t)ci * a.chunk;
      const int64_t cw = (a.ndof - c0) < a.chunk ? (a.ndof - c0) : a.chunk;
      gather_row_chunk(a, row, ci, c0, cw, racc);
      TO *out = A + row * a.lda + c0;
      for (int64_t j = threadIdx.x; j < cw; j += blockDim.x) out[j] = (TO)racc[j];
      __syncthreads();
    }
  }
}

// The same rows, kept only at the columns of a CSR pattern (sorted columns
// per row): val[q] = K[row, col[q]] for q in [row_ptr[row], row_ptr[row+1]).
__global__ void __launch_bounds__(256) k_tube_gather_csr(GatherArgs a, const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         double *__restrict__ val) {
  extern __shared__ double racc[];
  const int64_t slots = 8 * ((a.ndof + 7) / 8);
  for (int64_t b = blockIdx.x; b < slots; b += gridDim.x) {
    const int64_t row = dealt_row(b, a.ndof);
    if (row >= a.ndof) continue;
    const int64_t q0 = row_ptr[row], q1 = row_ptr[row + 1];
    for (int ci = 0; ci < a.nch; ci++) {
      const int64_t c0 = (int64_t)ci * a.chunk;
      const int64_t cw = (a.ndof - c0) < a.chunk ? (a.ndof - c0) : a.chunk;
      gather_row_chunk(a, row, ci, c0, cw, racc);
      for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const int64_t d = (int64_t)col[q] - c0;
        if ((uint64_t)d < (uint64_t)cw) val[q] = racc[d];
      }
      __syncthreads();
    }
  }
}

// ---- Tube blocks on the matrix cores in split FP16 (mixed precision) ----
//
// The block of a tube is one product B = X Y^T with an inner dimension of
// two columns per pair p: X_{:,2p} = W_p l_p, X_{:,2p+1} = W_p r_p,
// Y_{:,2p} = r_p, Y_{:,2p+1} = l_p (W_p = w_g K_i c_alpha), so that
// (X Y^T)_jk = sum_p W_p (l_j r_k + r_j l_k): the L W R^T contraction of the
// element quadrature, symmetric.  A node appears several times in one
// half-ray (once per element the ray crosses around it); those entries are
// summed first (in FP64, per assembly), so that a pair's side has one
// merged entry per node and every inner column of X and Y receives each of
// its rows at most once.  One workgroup (eight wavefronts, 64 x 32 each)
// computes a 128 x 128 region (I, J), I <= J, of B and writes it and its
// mirror into the tube's block.  The pairs go through LDS sixteen at a
// time (32 inner columns, one depth of v_mfma_f32_16x16x32_f16): the merged
// entries, scaled by the tube's powers of two (largest magnitude of X and
// of Y in [2^13, 2^14)), are split into FP16 hi + lo and stored straight
// into the operand panels, and the region accumulates hi hi + hi lo + lo hi
// in FP32 (22 significant bits per operand; the dropped lo lo term is
// below 2^-22 of each product).
constexpr int kRegion = 128;
constexpr int kChunkPairs = 16;
constexpr int kTubeThreads = 512;  // eight wavefronts per region, 64 x 32 of it each
constexpr int kMergeSlots = 4096;  // largest tube (|U_T|) of the matrix-core path
constexpr int kMergeMax = 512;     // most merged entries of one pair on that path

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// 16-byte group q of row `row` (64-byte rows): q ^ h(row) with
// h = (r1 ^ r2) | (r1 ^ r3) << 1 over the row's bits, so the lanes of one
// operand read (16 consecutive rows, one q) hit distinct 16-byte slots
// whether the LDS serves them 8 at a time in a 128-byte window or 16 at a
// time in a 256-byte window
__device__ __forceinline__ int tswz(int row, int q) {
  return q ^ ((((row >> 1) ^ (row >> 2)) & 1) | ((((row >> 1) ^ (row >> 3)) & 1) << 1));
}

// [buffer][hi, lo][row][16-byte group]: declared as 16-byte groups so that
// the operand reads are single ds_read_b128
struct TubeMfmaSmem {
  half8 hx[2][2][kRegion][2 * kChunkPairs / 8];
  half8 hy[2][2][kRegion][2 * kChunkPairs / 8];
};

// Merge structure of every sorted pair (plan time), one wavefront per pair:
// the merged entries of a side are its distinct tube slots in order of first
// occurrence (l's first, then r's).  COUNT: cnt[k] = the pair's merged
// entries.  FILL: for every entry its merged index within the pair (midx),
// and per merged entry slot | (inner column << 16), the column being
// 2 (pair mod 16) + side, its node and its pair; the pair's tube into
// pk_tube.  Slots must be
// below kMergeSlots; COUNT also takes into *maxc (zero on entry) the
// largest count above kMergeMax.
template <bool FILL>
__global__ void __launch_bounds__(64) k_merge_pairs(const int64_t *__restrict__ tube_off, int64_t n_tubes,
                                                    const int4 *__restrict__ pm, int64_t n_pairs,
                                                    const int32_t *__restrict__ ent_slot, int64_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ mk_pair, uint16_t *__restrict__ midx,
                                                    uint32_t *__restrict__ mk_meta, int32_t *__restrict__ pk_tube,
                                                    int *__restrict__ maxc, const int64_t *__restrict__ u_off,
                                                    const int32_t *__restrict__ tube_u, int32_t *__restrict__ mg_node,
                                                    int32_t *__restrict__ mg_pair) {
  __shared__ int tbl[kMergeSlots];
  const int lane = threadIdx.x;
  const int64_t k = blockIdx.x;
  if (k >= n_pairs) return;  // the whole block (one wavefront)
  const int4 m = pm[k];
  uint32_t col0 = 0;
  int64_t u0 = 0;
  if (FILL) {
    int64_t lo = 0, hi = n_tubes - 1;  // the pair's tube: the last T with tube_off[T] <= k
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (tube_off[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    col0 = 2u * (uint32_t)((k - tube_off[lo]) % kChunkPairs);
    if (lane == 0) pk_tube[k] = (int32_t)lo;
    u0 = u_off[lo];
  }
  int merged = 0;
  for (int side = 0; side < 2; side++) {
    const int64_t base = side ? (int64_t)m.y : (int64_t)m.x;
    const int n = side ? pair_nr(m) : pair_nl(m);
    for (int e = lane; e < n; e += 64) tbl[ent_slot[base + e]] = INT_MAX;
    __syncthreads();
    for (int e = lane; e < n; e += 64) atomicMin(&tbl[ent_slot[base + e]], e);
    __syncthreads();
    // first occurrences in order; each overwrites its slot's cell with
    // -(merged index + 1) (no other entry of that slot can be a first)
    for (int e0 = 0; e0 < n; e0 += 64) {
      const int e = e0 + lane;
      const int sl = e < n ? ent_slot[base + e] : 0;
      const bool first = e < n && tbl[sl] == e;
      const uint64_t bal = __ballot(first);
      const int r = merged + __popcll(bal & ((1ull << lane) - 1ull));
      if (first) {
        tbl[sl] = -(r + 1);
        if (FILL) {
          const int64_t q = mk_pair[k] + r;
          mk_meta[q] = (uint32_t)sl | ((col0 + (uint32_t)side) << 16);
          mg_node[q] = tube_u[u0 + sl];
          mg_pair[q] = (int32_t)k;
        }
      }
      merged += __popcll(bal);
    }
    __syncthreads();
    if (FILL)
      for (int e = lane; e < n; e += 64) midx[base + e] = (uint16_t)(-tbl[ent_slot[base + e]] - 1);
    __syncthreads();
  }
  if (!FILL && lane == 0) {
    cnt[k] = merged;
    if (merged > kMergeMax) atomicMax(maxc, merged);  // only the pairs over the limit
  }
}

__global__ void k_fill_int2(int2 *__restrict__ p, int64_t n, int2 v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Orders a wavefront's LDS accesses before and after it (no other
// wavefront shares the data).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The merged values (every assembly): each entry's value added in FP64 into
// its merged entry (LDS), kept in FP64 (mk_val64) and, times w_g, at its
// node-order position mpos (mwv) for the matrix-free product (when mwv is
// not null), and rounded to FP32 (mk_val, for the tube blocks); and per tube the
// largest binary exponents of X (W_p |v|) and of Y (|v|) over the merged
// values: texp must hold {INT_MIN, INT_MIN} per tube on entry and receives
// atomic maxima (ilogb is monotone, so the maximum of the exponents is the
// exponent of the maximum).  Every wavefront walks pairs k = wave, wave +
// waves, ... with the next pair's metadata loaded while the current one is
// merged; its LDS row is its own, so no workgroup barrier is needed (a
// wavefront's LDS operations complete in order).
__global__ void __launch_bounds__(256) k_merge_vals(const int4 *__restrict__ pm, const double *__restrict__ pw,
                                                    const int64_t *__restrict__ mk_pair,
                                                    const int32_t *__restrict__ pk_tube,
                                                    const uint16_t *__restrict__ midx, int64_t n_pairs,
                                                    const double *__restrict__ val, double KC0, double KC1, double KC2,
                                                    float *__restrict__ mk_val, double *__restrict__ mk_val64,
                                                    const int32_t *__restrict__ mpos, double *__restrict__ mwv,
                                                    int2 *__restrict__ texp) {
  __shared__ double acc[4][kMergeMax];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t waves = (int64_t)gridDim.x * 4;
  double *a = acc[w];
  int64_t k = (int64_t)blockIdx.x * 4 + w;
  int4 m{};
  int64_t b0 = 0, b1 = 0;
  double wk = 0.0;
  int tube = 0;
  auto meta = [&](int64_t kk, int4 &mm, int64_t &c0, int64_t &c1, double &ww, int &tt) {
    if (kk < n_pairs) {
      mm = pm[kk];
      c0 = mk_pair[kk];
      c1 = mk_pair[kk + 1];
      ww = pw[kk];
      tt = pk_tube[kk];
    }
  };
  meta(k, m, b0, b1, wk, tube);
  for (; k < n_pairs; k += waves) {
    const int nm = (int)(b1 - b0);
    for (int j = lane; j < nm; j += 64) a[j] = 0.0;
    wave_lds_sync();
    // entries e < nl of l, then of r, 256 at a time: all loads of a round
    // issued before its additions; the next pair's metadata is requested
    // after the first round, so waiting for that round leaves it in flight
    const int nl = pair_nl(m), ne = nl + pair_nr(m);
    int mi[4];
    double v[4];
    auto load_round = [&](int e0) {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int e = e0 + lane + 64 * j;
        const int64_t ei = e < nl ? (int64_t)m.x + e : (int64_t)m.y + (e - nl);
        mi[j] = e < ne ? (int)midx[ei] : -1;
        v[j] = e < ne ? val[ei] : 0.0;
      }
    };
    auto add_round = [&]() {
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (mi[j] >= 0) atomicAdd(&a[mi[j]], v[j]);
    };
    load_round(0);
    int4 mn{};
    int64_t n0 = 0, n1 = 0;
    double wn = 0.0;
    int tn = 0;
    meta(k + waves, mn, n0, n1, wn, tn);
    add_round();
    for (int e0 = 256; e0 < ne; e0 += 256) {
      load_round(e0);
      add_round();
    }
    wave_lds_sync();
    float vm = 0.f;
    for (int j = lane; j < nm; j += 64) {
      const double dv = a[j];
      const float fv = (float)dv;
      mk_val64[b0 + j] = dv;
      mk_val[b0 + j] = fv;
      if (mwv) mwv[mpos[b0 + j]] = wk * dv;
      vm = fmaxf(vm, fabsf(fv));
    }
    wave_lds_sync();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) vm = fmaxf(vm, __shfl_xor(vm, o, 64));
    if (lane == 0 && vm > 0.f) {
      const int axis = (int)((unsigned)m.w >> 30);
      const double mx = fabs(wk) * fabs(axis == 0 ? KC0 : (axis == 1 ? KC1 : KC2)) * (double)vm;
      int *te = (int *)&texp[tube];
      if (mx > 0.0) atomicMax(te, ilogb(mx));
      atomicMax(te + 1, ilogb((double)vm));
    }
    m = mn;
    b0 = n0;
    b1 = n1;
    wk = wn;
    tube = tn;
  }
}

// scale exponent of an operand from its largest exponent: the largest
// magnitude lands in [2^13, 2^14) (0 for an all-zero operand)
__device__ __forceinline__ int tube_scale_exp(int e) {
  if (e == INT_MIN) return 0;
  e -= 13;
  return e < -120 ? -120 : (e > 120 ? 120 : e);
}

// ---- The FP64 matrix-free product on the merged entries ----
// With d(k, s) = sum over the merged entries m of side s of pair k of
// v_m x[node_m], (K x)_j = sum over the merged entries m at node j of
// K_i c_alpha w_g v_m d(k_m, 1 - s_m): the quadrature of the element
// products over the half-ray pairs, with the entries of one node in a
// half-ray summed first (a third of the plan's entries at C5).  The
// node -> merged entry lists keep increasing merged index (a stable sort),
// so every sum has a fixed order.

// off[j] = the first position of node j in the sorted node keys, j <= nd
__global__ void k_node_bounds(const int32_t *__restrict__ keys, int64_t n, int64_t nd, int64_t *__restrict__ off) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nd) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  off[j] = lo;
}

__global__ void k_iota32(int32_t *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// per node-ordered merged incidence q: the index 2 k + (1 - s) of its
// partner's dot | axis << 30
__global__ void k_mpart(const int32_t *__restrict__ mrow_q, const int32_t *__restrict__ mg_pair,
                        const uint32_t *__restrict__ mk_meta, const int4 *__restrict__ pm, int64_t n,
                        uint32_t *__restrict__ mpart) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t mq = mrow_q[q];
  const int64_t k = mg_pair[mq];
  const uint32_t side = (mk_meta[mq] >> 16) & 1u;
  const uint32_t axis = (uint32_t)pm[k].w >> 30;
  mpart[q] = (uint32_t)(2 * k + 1 - side) | (axis << 30);
}

// mpos[m] = the position of merged entry m in node order
__global__ void k_inverse32(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ inv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) inv[perm[q]] = (int32_t)q;
}

// U entries per lane of the sixteen for one pair in flight at once: the
// loads of all U first, then the gathers of x, then the sums in entry order
template <int U>
__device__ __forceinline__ void pair_dot_run(int64_t &q, int64_t qe, const uint32_t *__restrict__ mk_meta,
                                             const double *__restrict__ mk_val64,
                                             const int32_t *__restrict__ mg_node, const double *__restrict__ x,
                                             double &s0, double &s1) {
  for (; q + 16 * (U - 1) < qe; q += 16 * U) {
    double w[U], xv[U];
    int32_t nd[U];
    uint32_t mt[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      w[u] = mk_val64[q + 16 * u];
      nd[u] = mg_node[q + 16 * u];
      mt[u] = mk_meta[q + 16 * u];
    }
#pragma unroll
    for (int u = 0; u < U; u++) xv[u] = x[nd[u]];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const double v = w[u] * xv[u];
      if ((mt[u] >> 16) & 1u) s1 += v;
      else s0 += v;
    }
  }
}

// dp[2 k + s] = d(k, s); sixteen lanes per pair, each summing its entries in
// ascending merged order
__global__ void __launch_bounds__(256) k_mpair_dot(const int64_t *__restrict__ mk_pair,
                                                   const uint32_t *__restrict__ mk_meta,
                                                   const double *__restrict__ mk_val64,
                                                   const int32_t *__restrict__ mg_node, const double *__restrict__ x,
                                                   int64_t n_pairs, double *__restrict__ dp) {
  const int gl = threadIdx.x & 15;
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (k >= n_pairs) return;  // the whole group of 16 shares k
  double s0 = 0.0, s1 = 0.0;
  const int64_t qe = mk_pair[k + 1];
  int64_t q = mk_pair[k] + gl;
  pair_dot_run<8>(q, qe, mk_meta, mk_val64, mg_node, x, s0, s1);
  pair_dot_run<2>(q, qe, mk_meta, mk_val64, mg_node, x, s0, s1);
  pair_dot_run<1>(q, qe, mk_meta, mk_val64, mg_node, x, s0, s1);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 16);
    s1 += __shfl_xor(s1, o, 16);
  }
  if (gl == 0) {
    dp[2 * k] = s0;
    dp[2 * k + 1] = s1;
  }
}

// U incidences per lane of node j's wavefront in flight at once, summed in
// ascending order
template <int U>
__device__ __forceinline__ void row_apply_run(int64_t &q, int64_t qe, const uint32_t *__restrict__ mpart,
                                              const double *__restrict__ mwv, const double *__restrict__ dp,
                                              double KC0, double KC1, double KC2, double &s) {
  for (; q + 64 * (U - 1) < qe; q += 64 * U) {
    uint32_t pt[U];
    double w[U], d[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      pt[u] = mpart[q + 64 * u];
      w[u] = mwv[q + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < U; u++) d[u] = dp[pt[u] & 0x3fffffffu];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t ax = pt[u] >> 30;
      s += w[u] * (ax == 0 ? KC0 : (ax == 1 ? KC1 : KC2)) * d[u];
    }
  }
}

// y_j over node j's merged incidences; one wavefront per node, four nodes
// per workgroup, the groups of four dealt to the XCDs in contiguous ranges
// (neighbouring nodes read the dots of the same tubes' pairs, which then
// stay in one L2); the grid is 8 ceil(ceil(ndof / 4) / 8) workgroups
__global__ void __launch_bounds__(256) k_mapply_rows(const int64_t *__restrict__ mrow_off,
                                                     const uint32_t *__restrict__ mpart,
                                                     const double *__restrict__ mwv, const double *__restrict__ dp,
                                                     double KC0, double KC1, double KC2, int64_t ndof,
                                                     double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = dealt_row(blockIdx.x, (ndof + 3) / 4) * 4 + (threadIdx.x >> 6);
  if (j >= ndof) return;
  double s = 0.0;
  const int64_t qe = mrow_off[j + 1];
  int64_t q = mrow_off[j] + lane;
  row_apply_run<4>(q, qe, mpart, mwv, dp, KC0, KC1, KC2, s);
  row_apply_run<2>(q, qe, mpart, mwv, dp, KC0, KC1, KC2, s);
  row_apply_run<1>(q, qe, mpart, mwv, dp, KC0, KC1, KC2, s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[j] = s;
}

struct TubeMfmaArgs {
  const int64_t *tube_off;
  const int4 *pm;
  const double *pw;
  const int64_t *mk_pair;
  const uint32_t *mk_meta;
  const float *mk_val;
  const int64_t *blk_off;
  double *blk;
  double KC0, KC1, KC2;
};

// One merged entry into the operand panels of buffer `b`: row slot - rx0
// of X (column c, W_p v) and row slot - ry0 of Y (column c ^ 1, v), each
// as hi and lo.
__device__ __forceinline__ void tube_put(TubeMfmaSmem &sm, int b, uint32_t mt, float v, const float *wv, float ysc,
                                         int rx0, int ry0) {
  const int sl = (int)(mt & 0xffffu), c = (int)(mt >> 16);
  const int rx = sl - rx0, ry = sl - ry0;
  if ((unsigned)rx < (unsigned)kRegion) {
    const float x = wv[c >> 1] * v;
    const _Float16 h = (_Float16)x;
    const int g = tswz(rx, c >> 3);
    ((_Float16 *)&sm.hx[b][0][rx][g])[c & 7] = h;
    ((_Float16 *)&sm.hx[b][1][rx][g])[c & 7] = (_Float16)(x - (float)h);
  }
  if ((unsigned)ry < (unsigned)kRegion) {
    const float y = v * ysc;
    const _Float16 h = (_Float16)y;
    const int cy = c ^ 1;
    const int g = tswz(ry, cy >> 3);
    ((_Float16 *)&sm.hy[b][0][ry][g])[cy & 7] = h;
    ((_Float16 *)&sm.hy[b][1][ry][g])[cy & 7] = (_Float16)(y - (float)h);
  }
}

// Work item b = blockIdx.x of n_items (the grid); items {-1, ..} pad the
// per-XCD lists and exit.
__global__ void __launch_bounds__(kTubeThreads) k_tube_mfma(TubeMfmaArgs a, const int4 *__restrict__ items, int64_t n_items,
                                                   const int2 *__restrict__ texp) {
  __shared__ TubeMfmaSmem sm;
  __shared__ float sw[2][kChunkPairs];  // W_p 2^-ex of the chunk's pairs (double-buffered)
  const int64_t bw = blockIdx.x;
  if (bw >= n_items) return;
  const int4 it = items[bw];
  if (it.x < 0) return;
  const int64_t T = it.x;
  const int U = it.w, rx0 = kRegion * it.y, ry0 = kRegion * it.z;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 2, wc = w & 3;
  const int64_t *__restrict__ mk_pair = a.mk_pair;
  const uint32_t *__restrict__ mk_meta = a.mk_meta;
  const float *__restrict__ mk_val = a.mk_val;
  const double *__restrict__ pw = a.pw;
  const int64_t k0 = a.tube_off[T], k1 = a.tube_off[T + 1];
  const int2 te0 = texp[T];
  const int2 te = make_int2(tube_scale_exp(te0.x), tube_scale_exp(te0.y));
  // the tube's pairs share one axis, so one coefficient
  const int axis = k1 > k0 ? (int)((unsigned)a.pm[k0].w >> 30) : 0;
  const double xsc = (axis == 0 ? a.KC0 : (axis == 1 ? a.KC1 : a.KC2)) * ldexp(1.0, -te.x);
  const float ysc = ldexpf(1.f, -te.y);
  // both panel buffers start at zero; a clear is 2 x 16 bytes per thread
  // of the buffer's hx and of its hy (16 KB each), consecutive lanes on
  // consecutive 16-byte slots
  const half8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
  auto clear = [&](int b) {
    half8 *px = &sm.hx[b][0][0][0], *py = &sm.hy[b][0][0][0];
#pragma unroll
    for (int j = 0; j < 1024 / kTubeThreads; j++) {
      px[t + kTubeThreads * j] = z8;
      py[t + kTubeThreads * j] = z8;
    }
  };
  clear(0);
  clear(1);
  f32x4v acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = f32x4v{0.f, 0.f, 0.f, 0.f};
  const int q = lane >> 4;
  // A chunk's merged entries are one contiguous range [e0, e1); thread t
  // takes e0 + t + kTubeThreads j.  Loads run ahead of their use: while chunk c is
  // scattered and multiplied, the entries of chunks c + 1 and c + 2, the
  // bounds of chunk c + 3 and the pair weights of chunk c + 2 are in flight.
  constexpr int kPre = 4;
  uint32_t cm[kPre], nm[kPre], fm[kPre];
  float cv[kPre], nv[kPre], fv[kPre];
  auto bounds = [&](int64_t kc, int64_t &b0, int64_t &b1) {
    if (kc < k1) {
      b0 = mk_pair[kc];
      b1 = mk_pair[kc + kChunkPairs < k1 ? kc + kChunkPairs : k1];
    } else {
      b0 = b1 = 0;
    }
  };
  auto entries = [&](int64_t b0, int64_t b1, uint32_t(&em)[kPre], float(&ev)[kPre]) {
#pragma unroll
    for (int j = 0; j < kPre; j++) {
      const int64_t i = b0 + t + kTubeThreads * j;
      const int64_t ic = i < b1 ? i : b0;
      em[j] = b1 > b0 ? mk_meta[ic] : 0u;
      ev[j] = b1 > b0 ? mk_val[ic] : 0.f;
    }
  };
  auto weight = [&](int64_t kc) { return t < kChunkPairs && kc + t < k1 ? (float)(pw[kc + t] * xsc) : 0.f; };
  // bounds of chunks c, c + 1, c + 2 (c = the current chunk)
  int64_t c0, c1, n0, n1, f0, f1;
  bounds(k0, c0, c1);
  bounds(k0 + kChunkPairs, n0, n1);
  bounds(k0 + 2 * kChunkPairs, f0, f1);
  entries(c0, c1, cm, cv);
  entries(n0, n1, nm, nv);
  if (t < kChunkPairs) sw[0][t] = weight(k0);
  float wnext = weight(k0 + kChunkPairs);
  int buf = 0;
  for (int64_t kc = k0; kc < k1; kc += kChunkPairs) {
    // issued now, used two iterations later: the entries of chunk c + 2;
    // one iteration later: the bounds of chunk c + 3, the weights of c + 2
    entries(f0, f1, fm, fv);
    int64_t g0, g1;
    bounds(kc + 3 * kChunkPairs, g0, g1);
    const float wfar = weight(kc + 2 * kChunkPairs);
    // buffer buf ^ 1 was read by the previous chunk's products, which every
    // wavefront finished before this barrier; buffer buf was cleared during
    // the previous chunk
    __syncthreads();
    clear(buf ^ 1);
#pragma unroll
    for (int j = 0; j < kPre; j++)
      if (c0 + t + kTubeThreads * j < c1) tube_put(sm, buf, cm[j], cv[j], sw[buf], ysc, rx0, ry0);
    for (int64_t i = c0 + t + kTubeThreads * kPre; i < c1; i += kTubeThreads) tube_put(sm, buf, mk_meta[i], mk_val[i], sw[buf], ysc, rx0, ry0);
    if (t < kChunkPairs) sw[buf ^ 1][t] = wnext;
    __syncthreads();
    half8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
    for (int x = 0; x < 4; x++) {
      const int ar = 64 * wr + 16 * x + (lane & 15);
      ah[x] = sm.hx[buf][0][ar][tswz(ar, q)];
      al[x] = sm.hx[buf][1][ar][tswz(ar, q)];
    }
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int br = 32 * wc + 16 * y + (lane & 15);
      bh[y] = sm.hy[buf][0][br][tswz(br, q)];
      bl[y] = sm.hy[buf][1][br][tswz(br, q)];
    }
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int y = 0; y < 2; y++) {
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[x], bh[y], acc[x][y], 0, 0, 0);
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[x], bl[y], acc[x][y], 0, 0, 0);
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[x], bh[y], acc[x][y], 0, 0, 0);
      }
    buf ^= 1;
#pragma unroll
    for (int j = 0; j < kPre; j++) {
      cm[j] = nm[j];
      cv[j] = nv[j];
      nm[j] = fm[j];
      nv[j] = fv[j];
    }
    c0 = n0;
    c1 = n1;
    n0 = f0;
    n1 = f1;
    f0 = g0;
    f1 = g1;
    wnext = wfar;
  }
  // region (I, J) of the block and, off the diagonal of regions, its mirror
  double *out = a.blk + a.blk_off[T];
  const int eu = te.x + te.y;
#pragma unroll
  for (int x = 0; x < 4; x++)
#pragma unroll
    for (int y = 0; y < 2; y++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = rx0 + 64 * wr + 16 * x + 4 * (lane >> 4) + i;
        const int c = ry0 + 32 * wc + 16 * y + (lane & 15);
        if (r < U && c < U) {
          const double v = ldexp((double)acc[x][y][i], eu);
          out[(int64_t)r * U + c] = v;
          if (it.y != it.z) out[(int64_t)c * U + r] = v;
        }
      }
}

}  // namespace

void free_tubes(TubePlan &tp) {
  dfree(tp.pair_sorted); dfree(tp.pm); dfree(tp.pw); dfree(tp.tube_off); dfree(tp.u_off); dfree(tp.tube_u); dfree(tp.ent_slot);
  dfree(tp.row_off); dfree(tp.row_ts); dfree(tp.items); dfree(tp.blk_off); dfree(tp.blk);
  dfree(tp.mitems); dfree(tp.texp);
  dfree(tp.mk_pair); dfree(tp.mk_meta); dfree(tp.mk_val); dfree(tp.mg_idx); dfree(tp.pk_tube);
  dfree(tp.cstart);
  dfree(tp.mg_node); dfree(tp.mg_pair); dfree(tp.mrow_q); dfree(tp.mrow_off); dfree(tp.mpart); dfree(tp.mpos);
  dfree(tp.mk_val64); dfree(tp.mwv); dfree(tp.mdp);
  tp = TubePlan();
}

int build_tubes(fpde_mesh *m, Plan &P, double kappa, hipStream_t s) {
  TubePlan &tp = P.tubes;
  free_tubes(tp);
  if (m->ndof == 0 || P.G == 0) return FPDE_OK;
  const int64_t n = 3 * P.G;
  if (n >= (int64_t(1) << 31)) return FPDE_EUNSUPPORTED;
  // cell size from the mean element size: edge of the regular tet of mean volume
  std::vector<double> xyz(3 * m->nv), vol(m->nt);
  FPDE_HIP(hipMemcpyAsync(xyz.data(), m->xyz, sizeof(double) * 3 * m->nv, hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipMemcpyAsync(vol.data(), m->vol, sizeof(double) * m->nt, hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipStreamSynchronize(s));
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, V = 0.0;
  for (int64_t v = 0; v < m->nv; v++)
    for (int d = 0; d < 3; d++) {
      lo[d] = std::min(lo[d], xyz[3 * v + d]);
      hi[d] = std::max(hi[d], xyz[3 * v + d]);
    }
  for (double x : vol) V += x;
  const double h = std::cbrt(6.0 * std::sqrt(2.0) * V / (double)m->nt);
  const double c = kappa * h;
  double ext = 0.0;
  for (int d = 0; d < 3; d++) ext = std::max(ext, hi[d] - lo[d]);
  const int ncell = std::max(1, (int)std::ceil(ext / c) + 1);
  if ((double)3 * ncell * ncell >= 4294967295.0) return FPDE_EUNSUPPORTED;
  tp.cell = c;

  uint32_t *key = nullptr, *key2 = nullptr;
  int32_t *val = nullptr, *head = nullptr, *tid = nullptr;
  int64_t *u_cnt = nullptr, *row_cnt = nullptr, *cursor = nullptr, *nb = nullptr, *usq = nullptr,
          *band_off = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  auto cleanup = [&]() {
    dfree(key); dfree(key2); dfree(val); dfree(head); dfree(tid);
    dfree(u_cnt); dfree(row_cnt); dfree(cursor); dfree(nb); dfree(usq); dfree(band_off);
    if (tmp) (void)hipFree(tmp);
    tmp = nullptr;
  };
  auto fail = [&](int code) {
    cleanup();
    free_tubes(tp);
    return code;
  };
  auto scratch = [&](size_t need) -> int {
    if (need <= tmp_bytes) return FPDE_OK;
    if (tmp) (void)hipFree(tmp);
    tmp = nullptr;
    tmp_bytes = 0;
    if (hipMalloc(&tmp, need) != hipSuccess) return FPDE_ENOMEM;
    tmp_bytes = need;
    return FPDE_OK;
  };
#define TRY_T(x)                          \
  do {                                    \
    int st_ = (x);                        \
    if (st_ != FPDE_OK) return fail(st_); \
  } while (0)
#define HIP_T(x)                                     \
  do {                                               \
    if ((x) != hipSuccess) return fail(FPDE_EHIP);   \
  } while (0)
  int st;
  TRY_T(dalloc(&key, n));
  TRY_T(dalloc(&key2, n));
  TRY_T(dalloc(&val, n));
  TRY_T(dalloc(&tp.pair_sorted, n));
  const double *qtab = m->rules + rule_offset(P.nq);
  k_pair_keys<<<nblocks(n), 256, 0, s>>>(m->tet, m->xyz, qtab, P.nq, P.G, lo[0], lo[1], lo[2], 1.0 / c, ncell, key,
                                         val);
  size_t need = 0;
  const int end_bit = 32;
  HIP_T(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key, key2, val, tp.pair_sorted, (int)n, 0, end_bit, s));
  TRY_T(scratch(need));
  HIP_T(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, tp.pair_sorted, (int)n, 0, end_bit, s));
  TRY_T(dalloc(&head, n));
  TRY_T(dalloc(&tid, n));
  k_heads<<<nblocks(n), 256, 0, s>>>(key2, n, head);
  HIP_T(hipcub::DeviceScan::ExclusiveSum(nullptr, need, head, tid, (int)n, s));
  TRY_T(scratch(need));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, head, tid, (int)n, s));
  int32_t last_tid = 0, last_head = 0;
  HIP_T(hipMemcpyAsync(&last_tid, tid + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_T(hipMemcpyAsync(&last_head, head + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_T(hipStreamSynchronize(s));
  tp.n_tubes = (int64_t)last_tid + last_head;
  const int64_t nT = tp.n_tubes;
  TRY_T(dalloc(&tp.tube_off, nT + 1));
  k_tube_off<<<nblocks(n), 256, 0, s>>>(head, tid, n, tp.tube_off);
  TRY_T(dalloc(&tp.pm, n));
  TRY_T(dalloc(&tp.pw, n));
  k_pair_meta<<<nblocks(n), 256, 0, s>>>(tp.pair_sorted, n, P.G, P.nq, P.off, qtab + 4 * P.nq, m->vol, tp.pm, tp.pw);
  dfree(key); dfree(key2); dfree(val); dfree(head); dfree(tid);

  // node sets
  TRY_T(dalloc(&u_cnt, nT + 1));
  TRY_T(dalloc(&tp.u_off, nT + 1));
  HIP_T(hipMemsetAsync(u_cnt, 0, sizeof(int64_t) * (nT + 1), s));
  k_tube_count<<<(unsigned)nT, 256, 0, s>>>(tp.tube_off, tp.pm, P.ent_dof, u_cnt, m->flag);
  int f = take_flag(m, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);
  HIP_T(hipcub::DeviceScan::ExclusiveSum(nullptr, need, u_cnt, tp.u_off, (int)(nT + 1), s));
  TRY_T(scratch(need));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, u_cnt, tp.u_off, (int)(nT + 1), s));
  HIP_T(hipMemcpyAsync(&tp.n_u, tp.u_off + nT, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_T(hipStreamSynchronize(s));
  TRY_T(dalloc(&tp.tube_u, tp.n_u));
  TRY_T(dalloc(&tp.ent_slot, P.n_ent));
  TRY_T(dalloc(&row_cnt, m->ndof + 1));
  HIP_T(hipMemsetAsync(row_cnt, 0, sizeof(int64_t) * (m->ndof + 1), s));
  k_tube_fill<<<(unsigned)nT, 256, 0, s>>>(tp.tube_off, tp.pm, P.ent_dof, tp.u_off, tp.tube_u, tp.ent_slot, row_cnt);
  TRY_T(dalloc(&tp.row_off, m->ndof + 1));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(nullptr, need, row_cnt, tp.row_off, (int)(m->ndof + 1), s));
  TRY_T(scratch(need));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, row_cnt, tp.row_off, (int)(m->ndof + 1), s));
  TRY_T(dalloc(&cursor, m->ndof + 1));
  HIP_T(hipMemcpyAsync(cursor, tp.row_off, sizeof(int64_t) * (m->ndof + 1), hipMemcpyDeviceToDevice, s));
  TRY_T(dalloc(&tp.row_ts, tp.n_u));
  k_row_places<<<(unsigned)nT, 256, 0, s>>>(tp.u_off, nT, tp.tube_u, cursor, tp.row_ts);

  // pass-1 bands and block offsets
  TRY_T(dalloc(&nb, nT + 1));
  TRY_T(dalloc(&usq, nT + 1));
  TRY_T(dalloc(&band_off, nT + 1));
  TRY_T(dalloc(&tp.blk_off, nT + 1));
  HIP_T(hipMemsetAsync(nb, 0, sizeof(int64_t) * (nT + 1), s));
  HIP_T(hipMemsetAsync(usq, 0, sizeof(int64_t) * (nT + 1), s));
  k_band_count<<<nblocks(nT), 256, 0, s>>>(tp.u_off, nT, nb, usq);
  HIP_T(hipcub::DeviceScan::ExclusiveSum(nullptr, need, nb, band_off, (int)(nT + 1), s));
  TRY_T(scratch(need));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, nb, band_off, (int)(nT + 1), s));
  HIP_T(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, usq, tp.blk_off, (int)(nT + 1), s));
  HIP_T(hipMemcpyAsync(&tp.n_items, band_off + nT, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_T(hipMemcpyAsync(&tp.blk_n, tp.blk_off + nT, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_T(hipStreamSynchronize(s));
  TRY_T(dalloc(&tp.items, tp.n_items));
  k_bands<<<nblocks(nT), 256, 0, s>>>(tp.u_off, nT, band_off, tp.items);
  // size statistics
  {
    std::vector<int64_t> uo(nT + 1);
    HIP_T(hipMemcpyAsync(uo.data(), tp.u_off, sizeof(int64_t) * (nT + 1), hipMemcpyDeviceToHost, s));
    HIP_T(hipStreamSynchronize(s));
    tp.max_u = 0;
    for (int64_t T = 0; T < nT; T++) tp.max_u = std::max<int64_t>(tp.max_u, uo[T + 1] - uo[T]);
  }
  HIP_T(hipGetLastError());
  f = take_flag(m, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);
  cleanup();
  return FPDE_OK;
#undef TRY_T
#undef HIP_T
}

// Plan of the matrix-core contraction: work items over the upper 128 x 128
// regions of every tube block, and the merge structure of every pair (merged
// index per entry, slot and inner column per merged entry).  Tubes larger
// than kMergeSlots or pairs with more than kMergeMax merged entries leave
// mfma_ok false (the FP64 accumulation then serves the mixed path).
static int build_mfma_plan(fpde_mesh *m, Plan &P, TubePlan &tp, hipStream_t s) {
  const int64_t nT = tp.n_tubes, nP = 3 * P.G;
  tp.mfma_ok = false;
  if (nT == 0 || tp.max_u > kMergeSlots) return FPDE_OK;
  int64_t *pcnt = nullptr;
  int *maxc = nullptr;
  void *tmp = nullptr;
  size_t need = 0, have = 0;
  int st = FPDE_OK;
  auto done = [&](int code) {
    dfree(pcnt);
    dfree(maxc);
    if (tmp) (void)hipFree(tmp);
    return code;
  };
  auto scan = [&](const int64_t *in, int64_t *out, int64_t n) {
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, (int)n, s) != hipSuccess) return FPDE_EHIP;
    if (need > have) {
      if (tmp) (void)hipFree(tmp);
      tmp = nullptr;
      if (hipMalloc(&tmp, need) != hipSuccess) return FPDE_ENOMEM;
      have = need;
    }
    return hipcub::DeviceScan::ExclusiveSum(tmp, need, in, out, (int)n, s) == hipSuccess ? FPDE_OK : FPDE_EHIP;
  };
  auto to_host = [&](const void *src, void *dst, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
  };
  // merged entries per pair, scanned
  if ((st = dalloc(&pcnt, nP + 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&maxc, 1)) != FPDE_OK) return done(st);
  if (hipMemsetAsync(pcnt, 0, sizeof(int64_t) * (nP + 1), s) != hipSuccess) return done(FPDE_EHIP);
  if (hipMemsetAsync(maxc, 0, sizeof(int), s) != hipSuccess) return done(FPDE_EHIP);
  k_merge_pairs<false><<<(unsigned)nP, 64, 0, s>>>(tp.tube_off, nT, tp.pm, nP, tp.ent_slot, pcnt, nullptr, nullptr,
                                                    nullptr, nullptr, maxc, nullptr, nullptr, nullptr, nullptr);
  int mc = 0;
  if (!to_host(maxc, &mc, sizeof(int))) return done(FPDE_EHIP);
  if (mc > kMergeMax) return done(FPDE_OK);
  if ((st = dalloc(&tp.mk_pair, nP + 1)) != FPDE_OK) return done(st);
  if ((st = scan(pcnt, tp.mk_pair, nP + 1)) != FPDE_OK) return done(st);
  int64_t n_mk = 0;
  if (!to_host(tp.mk_pair + nP, &n_mk, sizeof(int64_t))) return done(FPDE_EHIP);
  if ((st = dalloc(&tp.mk_meta, n_mk > 0 ? n_mk : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.mk_val, n_mk > 0 ? n_mk : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.mg_idx, P.n_ent > 0 ? P.n_ent : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.pk_tube, nP > 0 ? nP : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.mg_node, n_mk > 0 ? n_mk : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.mg_pair, n_mk > 0 ? n_mk : 1)) != FPDE_OK) return done(st);
  if ((st = dalloc(&tp.mk_val64, n_mk > 0 ? n_mk : 1)) != FPDE_OK) return done(st);
  k_merge_pairs<true><<<(unsigned)nP, 64, 0, s>>>(tp.tube_off, nT, tp.pm, nP, tp.ent_slot, nullptr, tp.mk_pair,
                                                   tp.mg_idx, tp.mk_meta, tp.pk_tube, nullptr, tp.u_off, tp.tube_u,
                                                   tp.mg_node, tp.mg_pair);
  tp.n_mk = n_mk;
  // node -> merged entries (stable by merged index) for the matrix-free
  // product; its partner indices need 2 nP < 2^30
  if (n_mk > 0 && n_mk < (int64_t(1) << 31) && 2 * nP + 1 < (int64_t(1) << 30)) {
    const int64_t nd = m->ndof;
    int32_t *keys = nullptr, *iota = nullptr;
    auto fail_m = [&](int code) {
      dfree(keys);
      dfree(iota);
      return done(code);
    };
    if ((st = dalloc(&keys, n_mk)) != FPDE_OK) return fail_m(st);
    if ((st = dalloc(&iota, n_mk)) != FPDE_OK) return fail_m(st);
    if ((st = dalloc(&tp.mrow_q, n_mk)) != FPDE_OK) return fail_m(st);
    k_iota32<<<nblocks(n_mk), 256, 0, s>>>(iota, n_mk);
    int bits = 1;
    while ((int64_t(1) << bits) < nd) bits++;
    size_t sneed = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, sneed, tp.mg_node, keys, iota, tp.mrow_q, (int)n_mk, 0, bits, s) !=
        hipSuccess)
      return fail_m(FPDE_EHIP);
    if (sneed > have) {
      if (tmp) (void)hipFree(tmp);
      tmp = nullptr;
      if (hipMalloc(&tmp, sneed) != hipSuccess) return fail_m(FPDE_ENOMEM);
      have = sneed;
    }
    if (hipcub::DeviceRadixSort::SortPairs(tmp, sneed, tp.mg_node, keys, iota, tp.mrow_q, (int)n_mk, 0, bits, s) !=
        hipSuccess)
      return fail_m(FPDE_EHIP);
    if ((st = dalloc(&tp.mrow_off, nd + 1)) != FPDE_OK) return fail_m(st);
    k_node_bounds<<<nblocks(nd + 1), 256, 0, s>>>(keys, n_mk, nd, tp.mrow_off);
    if ((st = dalloc(&tp.mpart, n_mk)) != FPDE_OK) return fail_m(st);
    k_mpart<<<nblocks(n_mk), 256, 0, s>>>(tp.mrow_q, tp.mg_pair, tp.mk_meta, tp.pm, n_mk, tp.mpart);
    if ((st = dalloc(&tp.mpos, n_mk)) != FPDE_OK) return fail_m(st);
    k_inverse32<<<nblocks(n_mk), 256, 0, s>>>(tp.mrow_q, n_mk, tp.mpos);
    if ((st = dalloc(&tp.mwv, n_mk)) != FPDE_OK) return fail_m(st);
    if ((st = dalloc(&tp.mdp, 2 * nP)) != FPDE_OK) return fail_m(st);
    if (hipStreamSynchronize(s) != hipSuccess) return fail_m(FPDE_EHIP);
    dfree(keys);
    dfree(iota);
    dfree(tp.mrow_q);
    dfree(tp.mg_pair);
    tp.mapply_ok = true;
  }
  // Region work items, balanced over the eight XCDs (the hardware deals
  // workgroup b to XCD b mod 8): whole tubes, largest cost first, each to
  // the XCD with the least work so far (cost = regions x chunks of 16
  // pairs); the items of XCD x at positions 8 j + x in tube order, padded
  // with {-1} at the end.  A tube's regions stay on one XCD, whose L2 then
  // serves its merged entries to all of them.
  std::vector<int64_t> toff(nT + 1), uoff(nT + 1);
  if (!to_host(tp.tube_off, toff.data(), sizeof(int64_t) * (nT + 1))) return done(FPDE_EHIP);
  if (!to_host(tp.u_off, uoff.data(), sizeof(int64_t) * (nT + 1))) return done(FPDE_EHIP);
  std::vector<int64_t> cost(nT), order(nT);
  for (int64_t T = 0; T < nT; T++) {
    const int64_t nr = (uoff[T + 1] - uoff[T] + kRegion - 1) / kRegion;
    const int64_t chunks = (toff[T + 1] - toff[T] + kChunkPairs - 1) / kChunkPairs;
    cost[T] = nr * (nr + 1) / 2 * (chunks + 1);
    order[T] = T;
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
  std::vector<int4> lists[8];
  int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (const int64_t T : order) {
    const int x = (int)(std::min_element(load, load + 8) - load);
    load[x] += cost[T];
    const int U = (int)(uoff[T + 1] - uoff[T]);
    const int nr = (U + kRegion - 1) / kRegion;
    for (int I = 0; I < nr; I++)
      for (int J = I; J < nr; J++) lists[x].push_back(make_int4((int)T, I, J, U));
  }
  size_t per = 0;
  for (int x = 0; x < 8; x++) per = std::max(per, lists[x].size());
  if (8 * (int64_t)per >= (int64_t(1) << 31)) return done(FPDE_EUNSUPPORTED);
  std::vector<int4> items(8 * per, make_int4(-1, 0, 0, 0));
  for (int x = 0; x < 8; x++)
    for (size_t j = 0; j < lists[x].size(); j++) items[8 * j + x] = lists[x][j];
  if ((st = dalloc(&tp.mitems, items.size() > 0 ? items.size() : 1)) != FPDE_OK) return done(st);
  if (!items.empty() && (hipMemcpyAsync(tp.mitems, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice,
                                        s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
    return done(FPDE_EHIP);
  tp.n_mitems = (int64_t)items.size();
  if (hipGetLastError() != hipSuccess) return done(FPDE_EHIP);
  tp.mfma_ok = true;
  return done(FPDE_OK);
}

// Pass 1 (the tube blocks) for order p->alpha and coefficients p->K:
// FP64 LDS accumulation, or for the mixed-precision matrix the split-FP16
// matrix-core contraction.
static int accumulate_tube_blocks(fpde_mesh *m, Plan &P, const fpde_params *p, hipStream_t s) {
  TubePlan &tp = P.tubes;
  if (!tp.blk) {
    FPDE_TRY(dalloc(&tp.blk, tp.blk_n > 0 ? tp.blk_n : 1));
  }
  Order o = order_scalars(p->alpha);
  AccumArgs a{};
  a.tube_off = tp.tube_off;
  a.pm = tp.pm;
  a.pw = tp.pw;
  a.items = tp.items;
  a.ent_slot = tp.ent_slot;
  a.ent_val = P.ent_val;
  a.blk_off = tp.blk_off;
  a.blk = tp.blk;
  a.KC0 = p->K[0] * o.c_alpha;
  a.KC1 = p->K[1] * o.c_alpha;
  a.KC2 = p->K[2] * o.c_alpha;
  // split FP16 on the matrix cores for the mixed-precision matrix (planned
  // once: work items and merge structure; merged values and exponents at
  // every assembly, as they follow the values)
  if (p->precision == FPDE_MIXED && !tp.mfma_planned) {
    FPDE_TRY(build_mfma_plan(m, P, tp, s));
    tp.mfma_planned = true;
  }
  if (p->precision == FPDE_MIXED && tp.mfma_ok) {
    if (!tp.texp) FPDE_TRY(dalloc(&tp.texp, tp.n_tubes > 0 ? tp.n_tubes : 1));
    const int64_t nP = 3 * P.G;
    const long ta = timer_begin(m, s, FPDE_STAGE_ACCUM);
    k_fill_int2<<<nblocks(tp.n_tubes), 256, 0, s>>>(tp.texp, tp.n_tubes, make_int2(INT_MIN, INT_MIN));
    // eight workgroups of four wavefronts per CU, each wavefront looping
    const unsigned mgrid = (unsigned)std::min<int64_t>(nblocks(nP, 4), 256 * 8);
    k_merge_vals<<<mgrid, 256, 0, s>>>(tp.pm, tp.pw, tp.mk_pair, tp.pk_tube, tp.mg_idx, nP, P.ent_val, a.KC0, a.KC1,
                                       a.KC2, tp.mk_val, tp.mk_val64, tp.mapply_ok ? tp.mpos : nullptr,
                                       tp.mapply_ok ? tp.mwv : nullptr, tp.texp);
    tp.mk_version = P.values_version;
    if (tp.n_mitems > 0) {
      TubeMfmaArgs ma{tp.tube_off, tp.pm, tp.pw, tp.mk_pair, tp.mk_meta, tp.mk_val, tp.blk_off, tp.blk,
                      a.KC0, a.KC1, a.KC2};
      k_tube_mfma<<<(unsigned)tp.n_mitems, kTubeThreads, 0, s>>>(ma, tp.mitems, tp.n_mitems, tp.texp);
    }
    timer_end(m, FPDE_STAGE_ACCUM, ta, s);
    return FPDE_OK;
  }
  const long ta = timer_begin(m, s, FPDE_STAGE_ACCUM);
  // deterministic: one wavefront per item walks the tube's pairs in order
  if (tp.n_items > 0)
    k_tube_accum<<<(unsigned)tp.n_items, p->deterministic ? 64 : 1024, sizeof(double) * kBandDoubles, s>>>(a);
  timer_end(m, FPDE_STAGE_ACCUM, ta, s);
  return FPDE_OK;
}

// Arguments of the row pass; the chunk starts of every tube are computed
// on first use (and again if the chunk width changes).
static int gather_args(fpde_mesh *m, Plan &P, int64_t lda, hipStream_t s, GatherArgs &gch) {
  TubePlan &tp = P.tubes;
  const int chunk = (int)(m->ndof < 8192 ? m->ndof : 8192);
  const int nch = (int)((m->ndof + chunk - 1) / chunk);
  if (!tp.cstart || tp.cs_chunk != chunk) {
    dfree(tp.cstart);
    tp.cs_chunk = 0;
    const int64_t ncs = tp.n_tubes * (nch + 1);
    FPDE_TRY(dalloc(&tp.cstart, ncs > 0 ? ncs : 1));
    if (ncs > 0) k_chunk_starts<<<nblocks(ncs), 256, 0, s>>>(tp.u_off, tp.tube_u, tp.n_tubes, chunk, nch, tp.cstart);
    FPDE_HIP(hipGetLastError());
    tp.cs_chunk = chunk;
  }
  gch = GatherArgs{};
  gch.row_off = tp.row_off;
  gch.row_ts = tp.row_ts;
  gch.u_off = tp.u_off;
  gch.tube_u = tp.tube_u;
  gch.blk_off = tp.blk_off;
  gch.blk = tp.blk;
  gch.cstart = tp.cstart;
  gch.ndof = m->ndof;
  gch.lda = lda;
  gch.chunk = chunk;
  gch.nch = nch;
  return FPDE_OK;
}

static unsigned gather_grid(int64_t ndof) {
  const int64_t slots = 8 * ((ndof + 7) / 8);
  return (unsigned)(slots < 65536 ? slots : 65536);
}

bool merged_apply_ready(const Plan &P) {
  const TubePlan &tp = P.tubes;
  return tp.mfma_ok && tp.mapply_ok && tp.mk_version == P.values_version;
}

int apply_merged(fpde_mesh *m, Plan &P, const fpde_params *p, const double *x, double *y, hipStream_t s) {
  TubePlan &tp = P.tubes;
  const int64_t nP = 3 * P.G;
  Order o = order_scalars(p->alpha);
  const long t = timer_begin(m, s, FPDE_STAGE_APPLY);
  k_mpair_dot<<<nblocks(16 * nP), 256, 0, s>>>(tp.mk_pair, tp.mk_meta, tp.mk_val64, tp.mg_node, x, nP, tp.mdp);
  k_mapply_rows<<<(unsigned)(8 * (((m->ndof + 3) / 4 + 7) / 8)), 256, 0, s>>>(tp.mrow_off, tp.mpart, tp.mwv, tp.mdp, p->K[0] * o.c_alpha,
                                                    p->K[1] * o.c_alpha, p->K[2] * o.c_alpha, m->ndof, y);
  timer_end(m, FPDE_STAGE_APPLY, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

int launch_contract_tubes(fpde_mesh *m, Plan &P, const fpde_params *p, void *A, int64_t lda, hipStream_t s) {
  if (m->ndof == 0) return FPDE_OK;
  const long t = timer_begin(m, s, FPDE_STAGE_CONTRACT);
  FPDE_TRY(accumulate_tube_blocks(m, P, p, s));
  GatherArgs gch;
  FPDE_TRY(gather_args(m, P, lda, s, gch));
  const unsigned grid = gather_grid(m->ndof);
  // deterministic: one wavefront per row takes the row's tube slices in order
  const unsigned gthreads = p->deterministic ? 64 : 256;
  if (p->precision == FPDE_MIXED)
    k_tube_gather<float><<<grid, gthreads, sizeof(double) * gch.chunk, s>>>(gch, (float *)A);
  else
    k_tube_gather<double><<<grid, gthreads, sizeof(double) * gch.chunk, s>>>(gch, (double *)A);
  timer_end(m, FPDE_STAGE_CONTRACT, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

// General form with constant coefficients: blocks by k_tube_form from the
// plan's two value sets (trial orders in ent_val, test orders in ent_val2),
// then the same row pass as the Riesz matrix.
int launch_form_tubes(fpde_mesh *m, Plan &P, const double cl[3], const double cr[3], double *A, int64_t lda,
                      hipStream_t s) {
  if (m->ndof == 0) return FPDE_OK;
  TubePlan &tp = P.tubes;
  if (!tp.blk) FPDE_TRY(dalloc(&tp.blk, tp.blk_n > 0 ? tp.blk_n : 1));
  AccumArgs a{};
  a.tube_off = tp.tube_off;
  a.pm = tp.pm;
  a.pw = tp.pw;
  a.items = tp.items;
  a.ent_slot = tp.ent_slot;
  a.ent_val = P.ent_val;
  a.val_b = P.ent_val2;
  a.blk_off = tp.blk_off;
  a.blk = tp.blk;
  for (int i = 0; i < 3; i++) {
    a.cl[i] = cl[i];
    a.cr[i] = cr[i];
  }
  if (tp.n_items > 0) k_tube_form<<<(unsigned)tp.n_items, 1024, sizeof(double) * kBandDoubles, s>>>(a);
  GatherArgs gch;
  FPDE_TRY(gather_args(m, P, lda, s, gch));
  k_tube_gather<double><<<gather_grid(m->ndof), 256, sizeof(double) * gch.chunk, s>>>(gch, A);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

int launch_contract_tubes_csr(fpde_mesh *m, Plan &P, const fpde_params *p, const int64_t *row_ptr,
                              const int32_t *col, double *val, hipStream_t s) {
  if (m->ndof == 0) return FPDE_OK;
  const long t = timer_begin(m, s, FPDE_STAGE_CONTRACT);
  FPDE_TRY(accumulate_tube_blocks(m, P, p, s));
  GatherArgs gch;
  FPDE_TRY(gather_args(m, P, 0, s, gch));
  k_tube_gather_csr<<<gather_grid(m->ndof), p->deterministic ? 64 : 256, sizeof(double) * gch.chunk, s>>>(
      gch, row_ptr, col, val);
  timer_end(m, FPDE_STAGE_CONTRACT, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

}  // namespace fpde
