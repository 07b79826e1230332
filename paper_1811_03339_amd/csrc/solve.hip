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
// Triangular solves use the stored inv(L_kk) and take one launch per
// direction: block rows are handed out in dependency order by an atomic
// ticket and wait for the blocks they need through per-block flags.  The same kernels are
// instantiated for FP32 storage, which the mixed-precision path factors and
// then refines against FP64 residuals b - K u computed matrix-free from the
// FP64 derivative vectors.
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "chol_diag.h"
#include "dense.h"
#include "syrk128.h"
#include "syrk256.h"

namespace fpde {

int apply_matfree(fpde_mesh *m, Plan *P, const fpde_params *p, const double *x, double *y, double *dscratch,
                  hipStream_t s);
int apply_scratch(fpde_mesh *m, Plan *P, double **d);

// inverse of the lower-triangular L held in LDS (rows >= nb are identity);
// lane j builds column j of inv(L) in X by forward substitution (L reads
// are broadcasts, X accesses are one column per lane) and stores it to Linv
// (row-major 64 x 64).  One wavefront.
template <class T>
__device__ __forceinline__ void tri_inverse_to(const double (*Lsh)[NB + 1], double (*X)[NB + 1],
                                               T *__restrict__ Linv, T *__restrict__ LinvT) {
  const int j = threadIdx.x;
  for (int i = 0; i < NB; i++) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int k = j; k < i; k++) s = fma(-Lsh[i][k], X[k][j], s);
    X[i][j] = (i < j) ? 0.0 : s / Lsh[i][i];
  }
  for (int i = 0; i < NB; i++) {
    Linv[i * NB + j] = (T)X[i][j];
    LinvT[j * NB + i] = (T)X[i][j];
  }
}

// Factor the diagonal block at (k0, k0) on its own (the first panel).
template <class T>
__global__ void __launch_bounds__(256) k_potrf_diag(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                    T *__restrict__ Linv, T *__restrict__ LinvT, int32_t *flag,
                                                    int64_t *aux, int64_t sA, int64_t sL) {
  __shared__ DiagSmem sm;
  A += (int64_t)blockIdx.y * sA;  // matrix blockIdx.y of a strided batch
  Linv += (int64_t)blockIdx.y * sL;
  LinvT += (int64_t)blockIdx.y * sL;
  aux += blockIdx.y;
  const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
  T av[16];  // all loads first (indices clamped into the block), then the selects
#pragma unroll
  for (int it = 0; it < 16; it++) {
    const int idx = threadIdx.x + 256 * it, r = idx >> 6, m = idx & 63;
    av[it] = A[(k0 + (r < nb ? r : nb - 1)) * lda + k0 + (m < nb ? m : nb - 1)];
  }
#pragma unroll
  for (int it = 0; it < 16; it++) {
    const int idx = threadIdx.x + 256 * it, r = idx >> 6, m = idx & 63;
    double v;
    if (r < nb && m < nb) v = (m <= r) ? (double)av[it] : 0.0;
    else v = (r == m) ? 1.0 : 0.0;
    sm.L[r][m] = v;
  }
  __syncthreads();
  diag_factor<T>(sm, nb, A, lda, k0, Linv, LinvT, flag, aux);
}

// inv(L_kk) for every diagonal block of an existing factor (one wave per block)
template <class T>
__global__ void __launch_bounds__(64) k_trinv(const T *__restrict__ A, int64_t lda, int64_t n, T *__restrict__ Linv,
                                              T *__restrict__ LinvT) {
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
  tri_inverse_to<T>(Lsh, X, Linv + (int64_t)blockIdx.x * NB * NB, LinvT + (int64_t)blockIdx.x * NB * NB);
}

// panel: rows [k0+NB+64 b, +64) of columns [k0, k0+NB) become B inv(L_kk)^T
template <class T>
__global__ void __launch_bounds__(256) k_panel(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                               const T *__restrict__ Linv, int64_t sA, int64_t sL) {
  __shared__ T sP[64][33], sQ[64][33];
  A += (int64_t)blockIdx.y * sA;
  Linv += (int64_t)blockIdx.y * sL;
  const int64_t r0 = k0 + NB + 64 * (int64_t)blockIdx.x;
  const int rows = (int)((n - r0) < 64 ? (n - r0) : 64);
  T out[16];
  tile_product(A + r0 * lda + k0, lda, rows, Linv, NB, NB, sP, sQ, out);
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int rr = frag_row<T>(q);
    if (rr < rows) A[(r0 + rr) * lda + k0 + frag_col<T>(q)] = out[q];
  }
}

// update C[I,J] -= X_I X_J^T over lower 64 x 64 tiles I >= J of the matrix
// starting at row/column k1 = k0 + KD; X = columns [k0, k0 + KD) (one panel,
// KD = 64).  ncol = 0: the whole lower triangle; ncol >= 1: only the strip
// of the first ncol block columns (tiles (I, J), J < ncol, I >= J), the
// block columns that the later panels of a group still need.  The workgroup
// of tile (0, 0) -- the next diagonal block -- keeps its updated tile in LDS
// and factors it at once (diag_factor), so the next panel's diagonal
// factorization runs beside the rest of this update instead of after it.
template <class T, int KD>
__global__ void __launch_bounds__(256) k_syrk(T *__restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                              T *__restrict__ Linv_next, T *__restrict__ LinvT_next, int32_t *flag,
                                              int64_t *aux, int64_t sA, int64_t sL, int nz, int ncol) {
  // block b = tile * nz + system: the tiles (0, 0) of all systems, which
  // carry the next diagonal factorizations, are dispatched first
  const int64_t z = (int64_t)blockIdx.x % nz;
  const int64_t x = (int64_t)blockIdx.x / nz;
  A += z * sA;
  Linv_next += z * sL;
  LinvT_next += z * sL;
  aux += z;
  struct Gemm {
    T sP[64][33], sQ[64][33];
  };
  __shared__ union {
    Gemm g;
    DiagSmem d;
  } sm;
  const int64_t base = k0 + KD;
  int64_t I = 0, J = 0;
  if (ncol == 0) {
    I = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= x) I++;
    while (I * (I + 1) / 2 > x) I--;
    J = x - I * (I + 1) / 2;
  } else {
    // strip tiles column by column: block column J holds Tn - J tiles
    const int64_t Tn = (n - base + 63) / 64;
    int64_t first = 0;
    while (J + 1 < ncol && x >= first + (Tn - J)) {
      first += Tn - J;
      J++;
    }
    I = J + (x - first);
  }
  const int64_t ri = base + 64 * I, cj = base + 64 * J;
  const int prow = (int)((n - ri) < 64 ? (n - ri) : 64);
  const int qrow = (int)((n - cj) < 64 ? (n - cj) : 64);
  T out[16];
  tile_product<KD>(A + ri * lda + k0, lda, prow, A + cj * lda + k0, lda, qrow, sm.g.sP, sm.g.sQ, out);
  // this thread's 16 entries of C, read before any is used (indices clamped
  // into the matrix so the loads need no guard)
  T cv[16];
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int64_t r = ri + frag_row<T>(q), c = cj + frag_col<T>(q);
    cv[q] = A[(r < n ? r : n - 1) * lda + (c < n ? c : n - 1)];
  }
  if (x == 0) {
    const int nb = prow;
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int r = frag_row<T>(q), c = frag_col<T>(q);
      double v;
      if (r < nb && c < nb) v = (c <= r) ? (double)cv[q] - (double)out[q] : 0.0;
      else v = (r == c) ? 1.0 : 0.0;
      sm.d.L[r][c] = v;
    }
    __syncthreads();
    diag_factor<T>(sm.d, nb, A, lda, ri, Linv_next, LinvT_next, flag, aux);
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int64_t r = ri + frag_row<T>(q), c = cj + frag_col<T>(q);
    if (r < n && c < n && c <= r) A[r * lda + c] = cv[q] - out[q];
  }
}

// Triangular solves in one launch per direction.  Each workgroup takes the
// next block row from an atomic ticket (forward: top to bottom; backward:
// bottom to top), so block rows are handed out in dependency order: a
// workgroup only ever waits for block rows whose tickets were taken before
// its own, by workgroups that are already running, and the first ticket
// waits for nothing -- no deadlock whatever the residency.  Solved blocks are
// published with a release store of the call's epoch into a per-block flag.
// Every wave polls the flags it needs by itself (acquire loads, up to 64
// flags per poll), so the loop over earlier blocks has no barrier; a poll
// that exceeds kSpinLimit marks the call failed and every wave still exits.
// backward: u_b = inv(L_bb)^T (x_b - sum_{c>b} L_cb^T u_c).  Lane = row of
// the result block (column r0 + lane of L); wave w owns rows 16w..16w+15 of
// block c.
template <class T>
__global__ void __launch_bounds__(256) k_trsv_bwd(const T *__restrict__ L, int64_t lda, int64_t n, int nblk,
                                                  const T *__restrict__ Linv, const double *__restrict__ x,
                                                  double *__restrict__ u, int *flags, int *ticket, int epoch,
                                                  int32_t *err, BatchStrides bs) {
  __shared__ int sb, ok;
  __shared__ double rhs[NB];
  __shared__ double red[4][NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {
    const int64_t z = blockIdx.y;
    L += z * bs.a;
    Linv += z * bs.l;
    x += z * bs.x;
    u += z * bs.v;
    flags += z * bs.f;
    ticket += z * bs.t;
  }
  if (tid == 0) {
    sb = atomicAdd(ticket, 1);
    ok = 1;
  }
  __syncthreads();
  if (sb >= nblk) return;
  const int b = nblk - 1 - sb;
  const int64_t r0 = (int64_t)b * NB;
  const int nb = (int)((n - r0) < NB ? (n - r0) : NB);
  // inv(L_bb)[16w + q][lane], read before any wait
  double li[16];
#pragma unroll
  for (int q = 0; q < 16; q++) li[q] = (double)Linv[(int64_t)b * NB * NB + (int64_t)(16 * w + q) * NB + lane];
  // only the last block can be partial, and it has no blocks below it, so
  // every block c > b read here has nbc rows and columns r0 + lane < n
  auto rows_of = [&](int c) { return (int)((n - (int64_t)c * NB) < NB ? (n - (int64_t)c * NB) : NB); };
  double part = 0.0;
  T cur[16];
#pragma unroll
  for (int q = 0; q < 16; q++) cur[q] = (T)0;
  if (nblk - 1 > b) {  // the last block row lies below this block
    const int c = nblk - 1;
    const int nbc = rows_of(c);
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int j = 16 * w + q;
      cur[q] = L[((int64_t)c * NB + (j < nbc ? j : nbc - 1)) * lda + r0 + lane];
    }
  }
  bool good = true;
  int ready = nblk;  // blocks [ready, nblk) known to be published
  for (int c = nblk - 1; c > b; c--) {
    if (c < ready) {
      const int k = poll_run(flags, c, -1, (c - b) < 64 ? (c - b) : 64, epoch);
      if (k == 0) {
        good = false;
        break;
      }
      ready = c - k + 1;
    }
    const int64_t c0 = (int64_t)c * NB;
    const int nbc = rows_of(c);
    const int jl = 16 * w + (lane & 15);
    const double ub = jl < nbc ? ld_dev(&u[c0 + jl]) : 0.0;
    const int cn = (c - 1 > b) ? c - 1 : c;
    const int nbn = rows_of(cn);
    T nxt[16];
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int j = 16 * w + q;
      nxt[q] = L[((int64_t)cn * NB + (j < nbn ? j : nbn - 1)) * lda + r0 + lane];
    }
#pragma unroll
    for (int q = 0; q < 16; q++) {
      part = fma((double)cur[q], read_lane(ub, q), part);
      cur[q] = nxt[q];
    }
  }
  if (!good && lane == 0) ok = 0;
  red[w][lane] = part;
  __syncthreads();
  if (tid < NB) rhs[tid] = (tid < nb) ? x[r0 + tid] - ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) : 0.0;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; q++) s = fma(li[q], rhs[16 * w + q], s);
  __syncthreads();  // red is reused
  red[w][lane] = s;
  __syncthreads();
  // written by wavefront 0 and published (as in the forward solve)
  if (tid < nb) st_dev(&u[r0 + tid], (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
  publish_block(flags, b, epoch);
  if (tid == 0 && !ok) set_flag(err, FPDE_EHIP);
}

__global__ void k_fill_i64(int64_t *p, int n, int64_t v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// u + z sv = b + z sv for the systems z = blockIdx.y of a batch
__global__ void k_copy_strided(const double *__restrict__ b, double *__restrict__ u, int64_t n, int64_t sv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = (int64_t)blockIdx.y * sv;
  if (k < n) u[o + k] = b[o + k];
}

__global__ void k_zero_i32(int *p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
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

int ensure_linv(fpde_mesh *m, int64_t n, size_t elem, int sets, void **out) {
  const size_t need = (size_t)sets * (size_t)((n + NB - 1) / NB) * NB * NB * elem;
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

// Inside a panel group: the KD / 64 block columns from hb on, every row
// from hb, by the KD columns of the group just before hb (X = columns
// [hb - KD, hb)), as a strip of 128 x 128 tiles (FP32: split FP16 rows of
// X first, into xq and es); its tile (0, 0) factors the diagonal block at
// hb into Ln, LnT.
template <class T, int KD>
static void group_part_update(T *A, int64_t lda, int64_t sA, int64_t n, int count, int64_t hb, T *Ln, T *LnT,
                              int64_t sL, int64_t *aux, int32_t *flag, int *es, _Float16 *xq, int64_t sx,
                              hipStream_t s) {
  const int64_t kx = hb - KD;
  if constexpr (std::is_same<T, float>::value)
    k_row_split<KD><<<dim3((unsigned)((n - hb + 3) / 4), (unsigned)count), 256, 0, s>>>(
        (const float *)A, lda, n, hb, kx, es, xq, sA, n, sx);
  const int ntc = KD / T128;
  const int64_t work = syrk128_strip_slots(n - hb, ntc) * count;
  k_syrk128<T, KD><<<(unsigned)(8 * ((work + 7) / 8)), Syrk128Shape<T>::THREADS, 0, s>>>(
      A, lda, n, kx, hb, ntc, 1, Ln, LnT, flag, aux, sA, sL, es, n, xq, sx, count, work);
}

// Factor `count` matrices of a strided batch (A + z sA, z < count) with one
// launch sequence: grid.y is the system, so the diagonal-block chains of the
// systems run side by side.  Linv holds 2 nblk inverse blocks per system
// (inverses, then transposes) at stride sL; aux[z] receives system z's
// failing column.
template <class T, int kGroup, int kPart>
static int potrf_batch_g(T *A, int64_t lda, int64_t sA, int64_t n, int count, T *Linv, int64_t sL, int64_t *aux,
                         fpde_mesh *m, hipStream_t s) {
  // Panels per group: kGroup (16 or 32), so that the trailing matrix is
  // read and written once per 64 kGroup columns (its traffic, 8 (n - k)^2
  // bytes per FP64 update, would otherwise compete with the matrix cores).
  // Inside a group the panels update the later block columns of their own
  // part of kPart panels one by one (strips of at most kPart - 1 block
  // columns).  With kPart < kGroup the update is recursive: whenever the
  // group's first kPart d panels are done (d the largest power of two
  // dividing the count over kPart, up to kGroup / 2 panels) the next kPart d
  // panels' columns are updated by those kPart d at once, on 128 x 128 tiles
  // with KD = 64 kPart d.  FP32: per-row exponents and split rows
  // (2 x 64 kGroup halfs) of the trailing updates, count x n of each, which
  // the parts inside the group use too.
  // FP32 trailing matrices of at least this many rows take 256 x 256 tiles
  // (measured at N = 66 822: 8-11% faster above it, alike from 12k rows
  // down to it, slower below: fewer tiles than the CUs can run at once)
  constexpr int64_t kTiles256From = 16384;
  // Look-ahead from this size on: a group's trailing update is split into
  // (a) the next group's 64 kGroup columns (every row from there; its tile (0, 0)
  // factors the next diagonal block) on the caller's stream and (b) the rest
  // on the side stream, so that the next group's panel chain (strips,
  // diagonal blocks, panels: a dependent sequence of small launches) runs
  // beside (b).  (a) of the next group waits for (b), which updated its
  // columns; the FP32 split rows alternate between two sets, so that a
  // group's split does not overwrite the rows that the previous (b) reads.
  constexpr int64_t kLookaheadFrom = 16384;
  const bool la = n >= kLookaheadFrom;
  if (la) {
    if (!m->side && hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess) {
      m->side = nullptr;
      return FPDE_EHIP;
    }
    for (hipEvent_t &e : m->lev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
        return FPDE_EHIP;
  }
  const int nset = la ? 2 : 1;
  int *escale = nullptr;
  _Float16 *xsplit = nullptr;
  const int64_t sx = n * 2 * kGroup * NB;
  if (std::is_same<T, float>::value) {
    const int64_t need = (int64_t)nset * count * n, xneed = (int64_t)nset * count * sx;
    if (m->escale_n < need || m->xsplit_n < xneed) {
      dfree(m->escale);
      dfree(m->xsplit);
      m->escale_n = m->xsplit_n = 0;
      FPDE_TRY(dalloc(&m->escale, (size_t)need));
      FPDE_TRY(dalloc(&m->xsplit, (size_t)xneed));
      m->escale_n = need;
      m->xsplit_n = xneed;
    }
    escale = m->escale;
    xsplit = m->xsplit;
  }
  bool pending_b = false;  // a (b) update is enqueued on the side stream
  const long t = timer_begin(m, s, FPDE_STAGE_POTRF);
  // the first diagonal block on its own; every later one is factored by the
  // workgroup of tile (0, 0) inside the preceding trailing update
  const int64_t nbk = (n + NB - 1) / NB;
  T *LinvT = Linv + nbk * NB * NB;
  const unsigned z = (unsigned)count;
  k_potrf_diag<T><<<dim3(1, z), 256, 0, s>>>(A, lda, n, 0, Linv, LinvT, m->flag, aux, sA, sL);
  // Panels in groups of kGroup: after panel s of a group (X_s = B inv(L)^T
  // for the 64 columns at ks, every row below), only later block columns of
  // its part of the group are updated by it (a strip, KD = 64; its tile
  // (0, 0) factors the next diagonal block), at the end of a part the next
  // part's columns by the part's panels, and the trailing matrix beyond the
  // group once by the whole group (KD = 64 kGroup): the trailing matrix is
  // read and written once per kGroup panels.
  for (int64_t k0 = 0; k0 < n; k0 += kGroup * NB) {
    for (int sp = 0; sp < kGroup; sp++) {
      const int64_t ks = k0 + sp * NB;
      const int64_t rest = n - ks - NB;  // rows below panel sp
      if (rest <= 0) goto factored;      // the last diagonal block is factored
      T *Lk = Linv + (ks / NB) * NB * NB;
      T *Ln = Lk + NB * NB, *LnT = LinvT + (ks / NB + 1) * NB * NB;
      k_panel<T><<<dim3(nblk(rest, 64), z), 256, 0, s>>>(A, lda, n, ks, Lk, sA, sL);
      const int64_t Tn = (rest + 63) / 64;              // block rows (and columns) below panel sp
      const int inner = kPart - 1 - sp % kPart;  // block columns of the part after panel sp
      if (Tn <= inner) {
        // the rest of the matrix lies inside the part: all of it, by this panel
        k_syrk<T, NB><<<(unsigned)(Tn * (Tn + 1) / 2 * count), 256, 0, s>>>(A, lda, n, ks, Ln, LnT, m->flag,
                                                                                aux, sA, sL, count, 0);
      } else if (inner > 0) {
        const int64_t tiles = (int64_t)inner * Tn - (int64_t)inner * (inner - 1) / 2;
        k_syrk<T, NB><<<(unsigned)(tiles * count), 256, 0, s>>>(A, lda, n, ks, Ln, LnT, m->flag, aux, sA, sL,
                                                                 count, inner);
      } else if (sp + 1 < kGroup) {
        // end of a part of the group: the next d panels' columns, every row
        // from there, by the d panels just factored, at once.  FP32: the
        // split rows go to this group's set, which nothing else reads
        // before the group's own split.
        const int64_t q = la ? (k0 / (kGroup * NB)) & 1 : 0;
        int *es = escale ? escale + q * count * n : nullptr;
        _Float16 *xq = xsplit ? xsplit + q * count * sx : nullptr;
        // panels updating at once: the largest power of two dividing sp + 1
        // (a multiple of kPart, at most kGroup / 2)
        const int d = (sp + 1) & -(sp + 1);
        static_assert((kGroup <= 32 && kPart == 4) || kPart == kGroup, "parts of 4 panels, or none");
        if (d == 16)
          group_part_update<T, 16 * NB>(A, lda, sA, n, count, ks + NB, Ln, LnT, sL, aux, m->flag, es, xq, sx, s);
        else if (d == 8)
          group_part_update<T, 8 * NB>(A, lda, sA, n, count, ks + NB, Ln, LnT, sL, aux, m->flag, es, xq, sx, s);
        else
          group_part_update<T, 4 * NB>(A, lda, sA, n, count, ks + NB, Ln, LnT, sL, aux, m->flag, es, xq, sx, s);
      } else {
        // the group's update of the trailing matrix from k0 + 64 kGroup on
        // 128 x 128 or 256 x 256 tiles (FP32: split FP16 with per-row
        // exponents over the group's 64 kGroup columns)
        const int64_t base = k0 + kGroup * NB;
        // this group's set of split rows
        const int64_t q = la ? (k0 / (kGroup * NB)) & 1 : 0;
        int *es = escale ? escale + q * count * n : nullptr;
        _Float16 *xq = xsplit ? xsplit + q * count * sx : nullptr;
        if constexpr (std::is_same<T, float>::value)
          k_row_split<kGroup * NB><<<dim3((unsigned)((n - base + 3) / 4), z), 256, 0, s>>>(
              (const float *)A, lda, n, base, k0, es, xq, sA, n, sx);
        // update of the region from rb on (lower tiles), X = the group's
        // columns; factor: its tile (0, 0) factors the diagonal block at rb
        auto region = [&](int64_t rb, int factor, hipStream_t st) {
          const int64_t mr = n - rb;
          if (std::is_same<T, float>::value && mr >= kTiles256From) {
            // 256 x 256 tiles of eight 128 x 64 wavefronts, one per CU
            const int64_t work = syrk256_slots(mr) * count;
            k_syrk256<kGroup * NB><<<(unsigned)(8 * ((work + 7) / 8)), 512, 0, st>>>(
                (float *)A, lda, n, k0, rb, factor, (float *)Ln, (float *)LnT, m->flag, aux, sA, sL, es, n, xq, sx,
                count, work);
          } else {
            // 128 x 128 tiles
            const int64_t work = syrk128_slots(mr) * count;
            k_syrk128<T, kGroup * NB><<<(unsigned)(8 * ((work + 7) / 8)), Syrk128Shape<T>::THREADS, 0, st>>>(
                A, lda, n, k0, rb, 0, factor, Ln, LnT, m->flag, aux, sA, sL, es, n, xq, sx, count, work);
          }
        };
        if (!la) {
          region(base, 1, s);
        } else {
          // (a) waits for the previous group's (b), which updated its columns
          if (pending_b) FPDE_HIP(hipStreamWaitEvent(s, m->lev[1], 0));
          const int ntc = kGroup * NB / T128;
          const int64_t work = syrk128_strip_slots(n - base, ntc) * count;
          k_syrk128<T, kGroup * NB><<<(unsigned)(8 * ((work + 7) / 8)), Syrk128Shape<T>::THREADS, 0, s>>>(
              A, lda, n, k0, base, ntc, 1, Ln, LnT, m->flag, aux, sA, sL, es, n, xq, sx, count, work);
          if (n - base > kGroup * NB) {
            // (b) after the split rows (and everything before them on s)
            FPDE_HIP(hipEventRecord(m->lev[0], s));
            FPDE_HIP(hipStreamWaitEvent(m->side, m->lev[0], 0));
            region(base + kGroup * NB, 0, m->side);
            FPDE_HIP(hipEventRecord(m->lev[1], m->side));
            pending_b = true;
          }
        }
      }
    }
  }
factored:
  if (pending_b) FPDE_HIP(hipStreamWaitEvent(s, m->lev[1], 0));  // the last (b) before anything after
  timer_end(m, FPDE_STAGE_POTRF, t, s, count);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

// From 16 384 unknowns on, groups of 32 panels in parts of 4; below, groups
// of 16 with per-panel strips over the rest of the group.  Measured, FP32 /
// FP64 factorization at N = 66 822: groups of 8 with per-panel strips
// 415 ms / 1.83 s; of 16: 375 ms / 1.78 s; of 16 in halves: 353 ms /
// 1.75 s; in parts of 4: 347 ms / 1.74 s; of 32 in parts of 4: 331 ms /
// 1.70 s; of 64: 348 ms / 1.69 s.  At N = 3 072 (six systems) and
// N = 4 494 (one system) the parts cost more launches than they save:
// 3.6 / 4.7 ms against 3.1 / 4.0 ms with per-panel strips.
template <class T>
static int potrf_batch(T *A, int64_t lda, int64_t sA, int64_t n, int count, T *Linv, int64_t sL, int64_t *aux,
                       fpde_mesh *m, hipStream_t s) {
  if (n >= 16384) return potrf_batch_g<T, 32, 4>(A, lda, sA, n, count, Linv, sL, aux, m, s);
  return potrf_batch_g<T, 16, 16>(A, lda, sA, n, count, Linv, sL, aux, m, s);
}

template <class T>
static int potrf(T *A, int64_t lda, int64_t n, fpde_mesh *m, hipStream_t s) {
  void *lv = nullptr;
  FPDE_TRY(ensure_linv(m, n, sizeof(T), 2, &lv));  // inverses, then their transposes
  return potrf_batch<T>(A, lda, 0, n, 1, (T *)lv, 0, m->flag_aux, m, s);
}

// y (n) holds the right-hand side on entry and the solution on exit;
// x (n) is scratch.  Two launches (forward, backward), each preceded by a
// reset of its ticket counter.
int zero_ints(int *p, int n, hipStream_t s) {
  if (n <= 0) return FPDE_OK;
  k_zero_i32<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

int ensure_trsv_sync(fpde_mesh *m, int nblk, hipStream_t s, int count) {
  const int cnt = count * (2 * nblk + 2);
  if (m->tsync_n < cnt) {
    dfree(m->tsync);
    m->tsync_n = 0;
    FPDE_TRY(dalloc(&m->tsync, (size_t)cnt));
    k_zero_i32<<<(cnt + 255) / 256, 256, 0, s>>>(m->tsync, cnt);
    m->tsync_n = cnt;
    m->tsync_epoch = 0;  // every flag is below the next epoch
  }
  return FPDE_OK;
}

// Forward and backward solves of `count` systems (strided batch, grid.y =
// system): y + z sv holds system z's right-hand side on entry and its
// solution on exit; x + z sx is scratch.
// The launches of trsv_batch with its flags and tickets given: tsync holds
// count x 2 nblk flags (below `epoch` on entry) then 2 count tickets.
template <class T>
static int trsv_batch_sync(const T *L, int64_t lda, int64_t sA, int64_t n, int count, const T *Linv, int64_t sL,
                           double *y, int64_t sv, double *x, int64_t sx, int *tsync, int epoch, fpde_mesh *m,
                           hipStream_t s) {
  const int nblk = (int)((n + NB - 1) / NB);
  int *fflags = tsync, *bflags = tsync + nblk, *tickets = tsync + (int64_t)count * 2 * nblk;
  const T *LinvT = Linv + (size_t)nblk * NB * NB;
  BatchStrides bs;
  bs.a = sA;
  bs.l = sL;
  bs.v = sv;
  bs.x = sx;
  bs.f = 2 * nblk;
  bs.t = 2;
  const dim3 grid((unsigned)nblk, (unsigned)count);
  const long t = timer_begin(m, s, FPDE_STAGE_TRSV);
  k_zero_i32<<<1, 64, 0, s>>>(tickets, 2 * count);
  k_trsv_rows<T, false><<<grid, 256, 0, s>>>(L, lda, n, nblk, LinvT, y, x, fflags, tickets, epoch, m->flag, bs);
  k_trsv_bwd<T><<<grid, 256, 0, s>>>(L, lda, n, nblk, Linv, x, y, bflags, tickets + 1, epoch, m->flag, bs);
  timer_end(m, FPDE_STAGE_TRSV, t, s, count);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

template <class T>
static int trsv_batch(const T *L, int64_t lda, int64_t sA, int64_t n, int count, const T *Linv, int64_t sL,
                      double *y, int64_t sv, double *x, int64_t sx, fpde_mesh *m, hipStream_t s) {
  const int nblk = (int)((n + NB - 1) / NB);
  FPDE_TRY(ensure_trsv_sync(m, nblk, s, count));
  const int epoch = ++m->tsync_epoch;
  return trsv_batch_sync<T>(L, lda, sA, n, count, Linv, sL, y, sv, x, sx, m->tsync, epoch, m, s);
}

template <class T>
static int trsv_pair(const T *L, int64_t lda, int64_t n, const T *Linv, double *y, double *x, fpde_mesh *m,
                     hipStream_t s) {
  return trsv_batch<T>(L, lda, 0, n, 1, Linv, 0, y, 0, x, 0, m, s);
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

// Dense SPD solve for a matrix that is not the Riesz matrix of a 3-D mesh
// (the two-dimensional variant): ws is a workspace handle (flags, timers,
// scratch) with ws->ndof = n.  A is overwritten by its Cholesky factor.
int dense_spd_solve(fpde_mesh *ws, double *A, int64_t lda, int64_t n, const double *b, double *u,
                    int64_t *failed, hipStream_t s) {
  if (failed) *failed = -1;
  if (n == 0) return FPDE_OK;
  FPDE_TRY(potrf<double>(A, lda, n, ws, s));
  int64_t col = -1;
  int f = take_flag(ws, s, &col);
  if (f != 0) {
    if (failed) *failed = col;
    return f < 0 ? f : FPDE_EHIP;
  }
  FPDE_TRY(ensure_vec(ws));
  if (u != b) FPDE_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_TRY(trsv_pair<double>(A, lda, n, (const double *)ws->linv, u, ws->vec + 3 * n, ws, s));
  f = take_flag(ws, s);
  return f < 0 ? f : (f > 0 ? FPDE_EHIP : FPDE_OK);
}

// ---- Dense FP64 solve whose scratch is a static device array ----
//
// For callers that cannot allocate: the diagonal-block inverses (and their
// transposes), the triangular solves' flags and tickets and the intermediate
// vector of fpde_solve's FP64 path live in `scratch`, one copy per device
// (the library's code object is loaded on every device it runs on), sized
// for kNoAllocMaxN unknowns.  Host code reaches the array through the device
// address hipGetSymbolAddress returns on each device (looked up once per
// device, on the first call there), never through its name.
constexpr int64_t kNoAllocMaxN = 8192;
constexpr int64_t kNoAllocBlk = (kNoAllocMaxN + NB - 1) / NB;
constexpr size_t kNoAllocLinv = 2 * (size_t)kNoAllocBlk * NB * NB;  // doubles
constexpr size_t kNoAllocVec = (size_t)kNoAllocMaxN;                // doubles
constexpr size_t kNoAllocInts = 2 * (size_t)kNoAllocBlk + 2;        // flags, tickets
constexpr size_t kNoAllocBytes = (kNoAllocLinv + kNoAllocVec) * sizeof(double) + kNoAllocInts * sizeof(int);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (`dev`)
static int scratch_address(int dev, void **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return FPDE_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FPDE_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_solve_noalloc(fpde_mesh *m, double *A, int64_t lda, const double *b, double *u,
                                  int64_t *failed_pivot, void *stream) {
  if (failed_pivot) *failed_pivot = -1;
  if (!m || !A || !b || !u) return FPDE_EINVAL;
  const int64_t n = m->ndof;
  if (lda < n || n > kNoAllocMaxN) return FPDE_EINVAL;
  if (m->timer.on) return FPDE_EINVAL;  // stage timers create events
  int dev = -1;
  FPDE_HIP(hipGetDevice(&dev));
  if (dev != m->device) return FPDE_EINVAL;
  if (n == 0) return FPDE_OK;
  void *base = nullptr;
  FPDE_TRY(scratch_address(dev, &base));
  double *lv = (double *)base;
  double *xs = lv + kNoAllocLinv;
  int *tsync = (int *)(xs + kNoAllocVec);
  const int nblk = (int)((n + NB - 1) / NB);
  hipStream_t s = S(stream);
  // the flags and tickets keep the previous call's values: cleared by a
  // kernel (no memset node if the caller captures a graph)
  FPDE_TRY(zero_ints(tsync, 2 * nblk + 2, s));
  FPDE_TRY(potrf_batch<double>(A, lda, 0, n, 1, lv, 0, m->flag_aux, m, s));
  if (u != b) FPDE_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FPDE_TRY(trsv_batch_sync<double>(A, lda, 0, n, 1, lv, 0, u, 0, xs, 0, tsync, 1, m, s));
  int64_t col = -1;
  int f = take_flag(m, s, &col);
  if (f == FPDE_ENOTSPD && failed_pivot) *failed_pivot = col;
  return f < 0 ? f : (f > 0 ? FPDE_EHIP : FPDE_OK);
}

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
  FPDE_TRY(ensure_linv(m, n, elem, 2, &lv));
  const unsigned nbk = (unsigned)((n + NB - 1) / NB);
  if (p->precision == FPDE_MIXED)
    k_trinv<float><<<nbk, 64, 0, s>>>((const float *)L, lda, n, (float *)lv, (float *)lv + (size_t)nbk * NB * NB);
  else
    k_trinv<double><<<nbk, 64, 0, s>>>((const double *)L, lda, n, (double *)lv,
                                        (double *)lv + (size_t)nbk * NB * NB);
  FPDE_HIP(hipGetLastError());
  return solve_with_factor(m, p, L, lda, lv, b, u, info, s);
}

extern "C" int fpde_solve_batch(fpde_mesh *m, int count, double *A, int64_t lda, int64_t stride_A, const double *b,
                                double *u, int64_t stride_v, int64_t *failed_pivot, void *stream) {
  if (!m || count < 1 || count > kMaxBatch) return FPDE_EINVAL;
  const int64_t n = m->ndof;
  if (!A || !b || !u || lda < n) return FPDE_EINVAL;
  if (count > 1 && (stride_A < n * lda || stride_v < n)) return FPDE_EINVAL;
  if (failed_pivot)
    for (int z = 0; z < count; z++) failed_pivot[z] = -1;
  if (n == 0) return FPDE_OK;
  const int64_t sA = count > 1 ? stride_A : 0, sv = count > 1 ? stride_v : 0;
  hipStream_t s = S(stream);
  if (!m->batch_aux) FPDE_TRY(dalloc(&m->batch_aux, (size_t)kMaxBatch));
  if (m->bvec_n < (int64_t)count * n) {
    dfree(m->bvec);
    m->bvec_n = 0;
    FPDE_TRY(dalloc(&m->bvec, (size_t)count * (size_t)n));
    m->bvec_n = (int64_t)count * n;
  }
  const int64_t nbk = (n + NB - 1) / NB, sL = 2 * nbk * NB * NB;
  void *lv = nullptr;
  FPDE_TRY(ensure_linv(m, n, sizeof(double), 2 * count, &lv));
  k_fill_i64<<<1, 64, 0, s>>>(m->batch_aux, count, -1);
  FPDE_TRY(potrf_batch<double>(A, lda, sA, n, count, (double *)lv, sL, m->batch_aux, m, s));
  // the solves follow at once: they finish whatever the factor holds (every
  // block flag is published, every wait bounded), and one status check at
  // the end covers both; a failed factorization reports no solution
  if (u != b) {
    k_copy_strided<<<dim3(nblk(n), (unsigned)count), 256, 0, s>>>(b, u, n, sv);
    FPDE_HIP(hipGetLastError());
  }
  FPDE_TRY(trsv_batch<double>(A, lda, sA, n, count, (const double *)lv, sL, u, sv, m->bvec, n, m, s));
  int f = take_flag(m, s);
  if (f == FPDE_ENOTSPD) {
    int64_t col[kMaxBatch];
    FPDE_HIP(hipMemcpyAsync(col, m->batch_aux, sizeof(int64_t) * count, hipMemcpyDeviceToHost, s));
    FPDE_HIP(hipStreamSynchronize(s));
    if (failed_pivot)
      for (int z = 0; z < count; z++) failed_pivot[z] = col[z];
  }
  return f < 0 ? f : (f > 0 ? FPDE_EHIP : FPDE_OK);
}
