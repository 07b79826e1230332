// Integration-path walk (Sec. 2.2) fused with the closed-form order-gamma
// Riemann-Liouville derivatives of the P1 basis functions (Sec. 2.1).
//
// One thread owns one half-ray (Gauss point x_g, direction s e_i).  Threads
// are numbered direction-major, h = dir * G + g, so a wavefront walks 64
// neighbouring Gauss points (Morton-ordered elements) in the same direction:
// similar path lengths, and the element records they touch overlap in L2.
//
// Per element E on the path, with u0 = x_g fixed for the whole walk:
//   b~ = (A^{-1}(u0 - v0), 1 - e^T A^{-1}(u0 - v0)),  d~ = (s A^{-1} e_i, -e^T s A^{-1} e_i)
//   r_max = min_{d~_j < 0} -b~_j / d~_j          (eq:cond)
//   k~_max = b~ + r_max d~                          (equ:ac)
// and the zero pattern of k~_max names the go-out m-face (Fig. 2): one zero
// -> the element across that face; more -> an element sharing the edge or
// vertex in which the ray advances (smallest id); none -> boundary reached.
// The arithmetic of the walk is IEEE FP64 without FMA contraction, in the
// same operation order as the reference definition, so element ids are
// reproducible bit for bit.
//
// On the segment [r_{k-1}, r_k] of element E_k the basis function of local
// vertex j has slope sigma = d psi / d x_i = (grad k_j)_i, and contributes
//   -s sigma (r_k^{1-gamma} - r_{k-1}^{1-gamma}) / Gamma(2 - gamma)
// to the side-s derivative at x_g (integration by parts of eq. def, m = 1;
// interior basis functions vanish at the path end, so no end-point term).
// A 4-slot window keyed by the current element's vertices accumulates these
// sums; a vertex that leaves the window is emitted as one (dof, value)
// entry, so a vector has about (segments + 3) entries.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "fpde_internal.h"

namespace fpde {

enum WalkMode { W_COUNT = 0, W_STRUCT = 1, W_VALUES = 2, W_ADJ = 3 };

struct WalkArgs {
  const TetRec *rec;
  const double *xyz;
  const int32_t *tet;
  const int32_t *vt_off;
  const int32_t *vt_tet;
  int32_t *flag;
  int64_t *flag_aux;
  int64_t G;
  int64_t h0, n;   // half-rays [h0, h0 + n)
  int cap;         // max elements per half-ray
  int nq;
  const double *qbary;  // device: nq x 4 barycentric coordinates of the rule
  // per axis: 1 - gamma_i, 1/Gamma(2 - gamma_i); psi(2 - gamma)/2 (one order)
  double e[3], inv_g2[3], half_psi0;
  // W_COUNT
  int32_t *cnt;    // n: entries per half-ray
  int32_t *len;    // n or null: elements per path
  uint64_t *hash;  // n or null
  int32_t *ids;    // n*cap or null
  double *rend;    // n*cap or null
  // W_STRUCT / W_VALUES
  const int64_t *off;  // indexed by h (global)
  int32_t *ent_dof;
  int32_t *ent_ray;
  double *ent_val;
  // W_ADJ
  const double *u, *lam;
  double *adj;     // 4 per half-ray (global h)
};

struct Isect {
  double bt[4], dt[4];
  double r_max;
  int jexit;  // coordinate whose ratio set r_max (first one on ties)
};

// entry (r, i) of A^{-1} with a lane-varying axis i, without indexing the
// record dynamically (which would spill it to scratch)
__device__ __forceinline__ double Mcol(const TetRec &R, int r, int i) {
  const double a = R.M[3 * r], b = R.M[3 * r + 1], c = R.M[3 * r + 2];
  return i == 0 ? a : (i == 1 ? b : c);
}

__device__ __forceinline__ void isect(const TetRec &R, const double *u0, int i, int s, Isect &o) {
  const double b0 = u0[0] - R.v0[0];
  const double b1 = u0[1] - R.v0[1];
  const double b2 = u0[2] - R.v0[2];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    o.bt[r + 1] = (R.M[3 * r + 0] * b0 + R.M[3 * r + 1] * b1) + R.M[3 * r + 2] * b2;
    const double m = Mcol(R, r, i);
    o.dt[r + 1] = (s > 0) ? m : -m;
  }
  o.bt[0] = 1.0 - ((o.bt[1] + o.bt[2]) + o.bt[3]);
  o.dt[0] = -((o.dt[1] + o.dt[2]) + o.dt[3]);
  double rm = INFINITY;
  int je = -1;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    if (o.dt[j] < 0.0) {
      const double r = -o.bt[j] / o.dt[j];
      if (r < rm) {
        rm = r;
        je = j;
      }
    }
  }
  o.r_max = rm;
  o.jexit = je;
}

__device__ __forceinline__ TetRec load_rec(const TetRec *rec, int64_t t) {
  TetRec R;
  const double4 *p = reinterpret_cast<const double4 *>(rec + t);
  double4 a = p[0], b = p[1], c = p[2], d = p[3];
  R.M[0] = a.x; R.M[1] = a.y; R.M[2] = a.z; R.M[3] = a.w;
  R.M[4] = b.x; R.M[5] = b.y; R.M[6] = b.z; R.M[7] = b.w;
  R.M[8] = c.x; R.v0[0] = c.y; R.v0[1] = c.z; R.v0[2] = c.w;
  const int4 *q = reinterpret_cast<const int4 *>(&d);
  int4 n = q[0], f = q[1];
  R.nbr[0] = n.x; R.nbr[1] = n.y; R.nbr[2] = n.z; R.nbr[3] = n.w;
  R.dof[0] = f.x; R.dof[1] = f.y; R.dof[2] = f.z; R.dof[3] = f.w;
  return R;
}

// slope of the volume coordinate of local vertex j along e_i
__device__ __forceinline__ double slope(const TetRec &R, int j, int i) {
  if (j > 0) return Mcol(R, j - 1, i);
  return -((Mcol(R, 0, i) + Mcol(R, 1, i)) + Mcol(R, 2, i));
}

// r^e for r > 0 as exp(e ln r): the exponent e = 1 - gamma lies in (0, 1]
// and r is a chord length (well inside (0, 1e3)), so |e ln r| is small and
// the result is within a few ulp of the correctly rounded power -- the
// values need 1e-10, not bit equality (only the element ids are bit-exact)
__device__ __forceinline__ double powr(double r, double e) { return r > 0.0 ? exp(e * log(r)) : 0.0; }
__device__ __forceinline__ double lnpowr(double r, double e) {
  if (!(r > 0.0)) return 0.0;
  const double l = log(r);
  return l * exp(e * l);
}

// Per-thread staging of a half-ray's consecutive outputs.  A thread writes
// its entries one at a time as the walk proceeds, and its neighbours in the
// wavefront write other half-rays' ranges, so plain stores leave every
// 64-byte segment of the output partly written for many steps (the caches
// evict such segments and the memory takes several partial writes per
// segment).  Instead each output goes to LDS slot (index mod L) of the
// thread's column, and an aligned run of L outputs leaves as 16-byte stores
// once its last element is known; the first and last runs of a half-ray,
// which it shares with its neighbours, are written element by element.
// The destination arrays are 256-byte aligned (device allocations).
template <class T, int L>
__device__ __forceinline__ void stage_put(T (*st)[256], T *__restrict__ out, int64_t base, int64_t e, T v) {
  static_assert(L * sizeof(T) == 64, "runs are 64-byte segments");
  const int tid = threadIdx.x;
  const int sl = (int)(e & (L - 1));
  st[sl][tid] = v;
  if (sl != L - 1) return;
  const int64_t c0 = e - (L - 1);
  if (c0 >= base) {
    if constexpr (sizeof(T) == 8) {
      double2 *p = reinterpret_cast<double2 *>(out + c0);
#pragma unroll
      for (int u = 0; u < L / 2; u++) p[u] = make_double2(st[2 * u][tid], st[2 * u + 1][tid]);
    } else {
      int4 *p = reinterpret_cast<int4 *>(out + c0);
#pragma unroll
      for (int u = 0; u < L / 4; u++)
        p[u] = make_int4(st[4 * u][tid], st[4 * u + 1][tid], st[4 * u + 2][tid], st[4 * u + 3][tid]);
    }
  } else {
    for (int64_t q = base; q <= e; q++) out[q] = st[q & (L - 1)][tid];
  }
}

// the outputs of the last, incomplete run [max(base, end rounded down), end)
template <class T, int L>
__device__ __forceinline__ void stage_flush(T (*st)[256], T *__restrict__ out, int64_t base, int64_t end) {
  const int64_t c0 = end & ~(int64_t)(L - 1);
  for (int64_t q = c0 > base ? c0 : base; q < end; q++) out[q] = st[q & (L - 1)][threadIdx.x];
}

// The walk is a chain of dependent element-record loads per thread; the
// value pass is asked for 4 wavefronts per SIMD (at most 128 VGPRs) so more
// chains are in flight.
template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == W_VALUES ? 4 : 1)))
k_walk(WalkArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const int64_t h = a.h0 + k;
  const int dir = (int)(h / a.G);
  const int64_t g = h - (int64_t)dir * a.G;
  const int i = dir >> 1, side = dir & 1;
  const int s = side ? 1 : -1;
  const int nq = a.nq;
  const int64_t t0 = g / nq;
  const int q = (int)(g - t0 * nq);

  // Gauss point x_g = sum_j beta_qj v_j, summed in vertex order
  double u0[3];
  {
    int32_t vv[4];
#pragma unroll
    for (int j = 0; j < 4; j++) vv[j] = a.tet[4 * t0 + j];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 4; j++) acc = acc + a.qbary[4 * q + j] * a.xyz[3 * (int64_t)vv[j] + d];
      u0[d] = acc;
    }
  }

  // window of the current element's vertices
  int32_t wd[4] = {-1, -1, -1, -1};
  double wv[4] = {0.0, 0.0, 0.0, 0.0};
  double wdv[4] = {0.0, 0.0, 0.0, 0.0};  // d/dalpha (W_ADJ)
  int64_t nemit = 0;
  int64_t base = 0;
  if (MODE == W_STRUCT || MODE == W_VALUES) base = a.off[h];
  double dot_u = 0.0, dot_l = 0.0, ddot_u = 0.0, ddot_l = 0.0;
  const double sgn = side ? -1.0 : 1.0;

  // staging runs of the structure pass (node and half-ray ids) and of the
  // value pass (values)
  __shared__ int32_t st_dof[MODE == W_STRUCT ? 16 : 1][256], st_ray[MODE == W_STRUCT ? 16 : 1][256];
  __shared__ double st_val[MODE == W_VALUES ? 8 : 1][256];
  auto emit = [&](int32_t d, double v, double dv) {
    if constexpr (MODE == W_STRUCT) {
      stage_put<int32_t, 16>(st_dof, a.ent_dof, base, base + nemit, d);
      stage_put<int32_t, 16>(st_ray, a.ent_ray, base, base + nemit, (int32_t)h);
    } else if constexpr (MODE == W_VALUES) {
      stage_put<double, 8>(st_val, a.ent_val, base, base + nemit, v);
    } else if constexpr (MODE == W_ADJ) {
      const double uu = a.u[d], ll = a.lam[d];
      dot_u += v * uu;
      dot_l += v * ll;
      ddot_u += dv * uu;
      ddot_l += dv * ll;
    }
    nemit++;
  };

  uint64_t hsh = 14695981039346656037ull;
  int64_t t = t0;
  double r_cur = 0.0;
  double P_lo = 0.0, Q_lo = 0.0;
  int nseg = 0;
  int status = FPDE_EPATH;  // cleared when the walk reaches the boundary
  for (int step = 0; step < a.cap + 64; step++) {
    const TetRec R = load_rec(a.rec, t);
    Isect o;
    isect(R, u0, i, s, o);
    if (!(o.r_max < INFINITY)) {
      status = FPDE_EPATH;
      break;
    }
    if (o.r_max > r_cur) {
      // segment [r_cur, r_max] in element t
      if (nseg >= a.cap) {
        status = FPDE_EPATH;
        break;
      }
      if (MODE == W_COUNT) {
        const uint32_t uid = (uint32_t)t;
#pragma unroll
        for (int b = 0; b < 4; b++) {
          hsh ^= (uint64_t)((uid >> (8 * b)) & 0xffu);
          hsh *= 1099511628211ull;
        }
        if (a.ids) a.ids[k * a.cap + nseg] = (int32_t)t;
        if (a.rend) a.rend[k * a.cap + nseg] = o.r_max;
      }
      // move the window onto this element's vertices
      {
        int32_t nd[4] = {R.dof[0], R.dof[1], R.dof[2], R.dof[3]};
        double na[4] = {0.0, 0.0, 0.0, 0.0}, nda[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 4; j++) {
          if (wd[j] < 0) continue;
          bool kept = false;
#pragma unroll
          for (int m = 0; m < 4; m++) {
            if (nd[m] == wd[j]) {
              na[m] = wv[j];
              nda[m] = wdv[j];
              kept = true;
            }
          }
          if (!kept) emit(wd[j], wv[j], wdv[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
          wd[j] = nd[j];
          wv[j] = na[j];
          wdv[j] = nda[j];
        }
      }
      if (MODE == W_VALUES || MODE == W_ADJ) {
        const double ei = i == 0 ? a.e[0] : (i == 1 ? a.e[1] : a.e[2]);
        const double gi = i == 0 ? a.inv_g2[0] : (i == 1 ? a.inv_g2[1] : a.inv_g2[2]);
        const double P_hi = powr(o.r_max, ei);
        double dP = gi * (P_hi - P_lo);
        double dQ = 0.0;
        if (MODE == W_ADJ) {
          const double Q_hi = lnpowr(o.r_max, ei);
          dQ = gi * (a.half_psi0 * (P_hi - P_lo) - 0.5 * (Q_hi - Q_lo));
          Q_lo = Q_hi;
        }
        P_lo = P_hi;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          if (wd[j] < 0) continue;
          const double sg = sgn * slope(R, j, i);
          wv[j] += sg * dP;
          if (MODE == W_ADJ) wdv[j] += sg * dQ;
        }
      }
      nseg++;
      r_cur = o.r_max;
    }
    // zero pattern of the volume coordinates at the go-out point: |k_j| is
    // compared with 1e-12 times the size of the two terms it is the
    // difference of (at least 1e-12); the coordinate that set r_max is zero
    // by construction
    int zmask = 0, nz = 0, zf = -1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const double p = o.r_max * o.dt[j];
      const double kj = o.bt[j] + p;
      double sc = fabs(o.bt[j]);
      sc = fabs(p) > sc ? fabs(p) : sc;
      sc = sc < 1.0 ? 1.0 : sc;
      if (j == o.jexit || fabs(kj) <= 1e-12 * sc) {
        zmask |= 1 << j;
        nz++;
        zf = j;
      }
    }
    if (nz == 0 || nz == 4) {
      status = FPDE_EPATH;
      break;
    }
    if (nz == 1) {
      const int32_t nx = zf == 0 ? R.nbr[0] : (zf == 1 ? R.nbr[1] : (zf == 2 ? R.nbr[2] : R.nbr[3]));
      if (nx < 0) {  // boundary reached
        status = 0;
        break;
      }
      t = nx;
      continue;
    }
    // edge or vertex: elements containing every vertex whose k != 0
    int32_t tv[4];
#pragma unroll
    for (int j = 0; j < 4; j++) tv[j] = a.tet[4 * t + j];
    const int first = __builtin_ctz((~zmask) & 0xf);  // nz <= 3, so one vertex is kept
    const int32_t v_first = (first == 0) ? tv[0] : (first == 1) ? tv[1] : (first == 2) ? tv[2] : tv[3];
    int64_t best = -1;
    for (int32_t p = a.vt_off[v_first]; p < a.vt_off[v_first + 1]; p++) {
      const int64_t c = a.vt_tet[p];
      if (c == t) continue;
      int32_t cv[4];
#pragma unroll
      for (int j = 0; j < 4; j++) cv[j] = a.tet[4 * c + j];
      bool all = true;
#pragma unroll
      for (int m = 0; m < 4; m++) {
        if ((zmask >> m) & 1) continue;
        const bool f = (cv[0] == tv[m]) || (cv[1] == tv[m]) || (cv[2] == tv[m]) || (cv[3] == tv[m]);
        all = all && f;
      }
      if (!all) continue;
      const TetRec Rc = load_rec(a.rec, c);
      Isect oc;
      isect(Rc, u0, i, s, oc);
      if (oc.r_max - r_cur > 1e-12 * r_cur) {
        best = c;
        break;
      }
    }
    if (best < 0) {  // boundary reached through an edge or vertex
      status = 0;
      break;
    }
    t = best;
  }
  if (status == 0 && nseg == 0) status = FPDE_EPATH;
  if (status != 0) {
    set_flag(a.flag, status);
    atomicCAS((unsigned long long *)a.flag_aux, ~0ull, (unsigned long long)h);
    if (MODE == W_COUNT) a.cnt[k] = 0;
    return;
  }
  // flush the last element's vertices
#pragma unroll
  for (int j = 0; j < 4; j++)
    if (wd[j] >= 0) emit(wd[j], wv[j], wdv[j]);
  if constexpr (MODE == W_STRUCT) {
    stage_flush<int32_t, 16>(st_dof, a.ent_dof, base, base + nemit);
    stage_flush<int32_t, 16>(st_ray, a.ent_ray, base, base + nemit);
  } else if constexpr (MODE == W_VALUES) {
    stage_flush<double, 8>(st_val, a.ent_val, base, base + nemit);
  }
  if (MODE == W_COUNT) {
    a.cnt[k] = (int32_t)nemit;
    if (a.len) a.len[k] = nseg;
    if (a.hash) a.hash[k] = hsh;
  }
  if (MODE == W_ADJ) {
    a.adj[4 * h + 0] = dot_u;
    a.adj[4 * h + 1] = dot_l;
    a.adj[4 * h + 2] = ddot_u;
    a.adj[4 * h + 3] = ddot_l;
  }
}

__global__ void k_row_count(const int32_t *__restrict__ ent_dof, int64_t n, int64_t *__restrict__ cnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) atomicAdd((unsigned long long *)&cnt[ent_dof[e]], 1ull);
}

__global__ void k_row_fill(const int32_t *__restrict__ ent_dof, int64_t n, int64_t *__restrict__ cursor,
                           int64_t *__restrict__ inc) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    int64_t p = (int64_t)atomicAdd((unsigned long long *)&cursor[ent_dof[e]], 1ull);
    inc[p] = e;
  }
}

// flattened per-incidence data for the accumulation (see Plan::inc_meta)
__global__ void k_inc_meta(const int64_t *__restrict__ inc, const int32_t *__restrict__ ent_ray,
                           const int64_t *__restrict__ off, const double *__restrict__ vol,
                           const double *__restrict__ wq, int64_t G, int nq, int64_t n, int4 *__restrict__ meta,
                           double *__restrict__ w) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t e = inc[p];
  const int64_t h = ent_ray[e];
  const int dir = (int)(h / G);
  const int64_t g = h - (int64_t)dir * G;
  const int64_t partner = (dir & 1) ? h - G : h + G;
  const int64_t po = off[partner];
  const int64_t pl = off[partner + 1] - po;
  meta[p] = make_int4((int)e, (int)po, (int)((pl << 2) | (dir >> 1)), (int)partner);
  w[p] = wq[g % nq] * vol[g / nq];
}

__global__ void k_i32_to_i64(const int32_t *__restrict__ a, int64_t n, int64_t *__restrict__ b) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = a[k];
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static WalkArgs base_args(fpde_mesh *m, const Plan &P, const QuadRule &rule) {
  WalkArgs a{};
  a.rec = m->rec;
  a.xyz = m->xyz;
  a.tet = m->tet;
  a.vt_off = m->vt_off;
  a.vt_tet = m->vt_tet;
  a.flag = m->flag;
  a.flag_aux = m->flag_aux;
  a.G = P.G;
  a.cap = P.max_steps;
  a.nq = rule.nq;
  a.qbary = m->rules + rule_offset(rule.nq);
  return a;
}

template <int MODE>
static void launch_walk(const WalkArgs &a, hipStream_t s) {
  if (a.n <= 0) return;
  k_walk<MODE><<<nblk(a.n), 256, 0, s>>>(a);
}

void free_plan(Plan &P) {
  dfree(P.off); dfree(P.ent_dof); dfree(P.ent_ray); dfree(P.ent_val); dfree(P.ent_val2); dfree(P.row_off); dfree(P.inc);
  dfree(P.adj); dfree(P.inc_meta); dfree(P.inc_w); dfree(P.inc_wv);
  free_tubes(P.tubes);
  P = Plan();
}

// tube cell edge of the accumulation, in mean element edges
constexpr double kTubeCell = 1.0;

static int build_plan(fpde_mesh *m, Plan &P, int nq, int max_steps, hipStream_t s) {
  QuadRule rule;
  FPDE_TRY(quad_rule(nq, &rule));
  P.nq = nq;
  P.max_steps = max_steps;
  P.G = m->nt * nq;
  P.n_half = 6 * P.G;
  int32_t *cnt = nullptr;
  int64_t *cnt64 = nullptr, *rowcnt = nullptr, *cursor = nullptr;
  void *tmp = nullptr;
  int st = FPDE_OK;
  auto fail = [&](int code) {
    dfree(cnt); dfree(cnt64); dfree(rowcnt); dfree(cursor);
    if (tmp) (void)hipFree(tmp);
    free_plan(P);
    return code;
  };
  if ((st = dalloc(&cnt, P.n_half + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&cnt64, P.n_half + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.off, P.n_half + 1)) != FPDE_OK) return fail(st);
  if (hipMemsetAsync(cnt, 0, sizeof(int32_t) * (P.n_half + 1), s) != hipSuccess) return fail(FPDE_EHIP);

  WalkArgs a = base_args(m, P, rule);
  a.h0 = 0;
  a.n = P.n_half;
  a.cnt = cnt;
  launch_walk<W_COUNT>(a, s);
  k_i32_to_i64<<<nblk(P.n_half + 1), 256, 0, s>>>(cnt, P.n_half + 1, cnt64);
  size_t need = 0, need2 = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, need, cnt64, P.off, (int)(P.n_half + 1), s) != hipSuccess)
    return fail(FPDE_EHIP);
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, need2, cnt64, P.off, (int)(m->ndof + 1), s) != hipSuccess)
    return fail(FPDE_EHIP);
  size_t tb = need > need2 ? need : need2;
  if (hipMalloc(&tmp, tb) != hipSuccess) return fail(FPDE_ENOMEM);
  if (hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt64, P.off, (int)(P.n_half + 1), s) != hipSuccess)
    return fail(FPDE_EHIP);
  if (hipMemcpyAsync(&P.n_ent, P.off + P.n_half, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(FPDE_EHIP);
  int f = take_flag(m, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);

  if (P.n_ent >= (int64_t(1) << 31)) return fail(FPDE_EUNSUPPORTED);  // 32-bit entry ids below
  if ((st = dalloc(&P.ent_dof, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.ent_ray, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.ent_val, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.inc, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.row_off, m->ndof + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&rowcnt, m->ndof + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&cursor, m->ndof + 1)) != FPDE_OK) return fail(st);
  a.off = P.off;
  a.ent_dof = P.ent_dof;
  a.ent_ray = P.ent_ray;
  launch_walk<W_STRUCT>(a, s);
  // node -> entries transpose (counting sort)
  if (hipMemsetAsync(rowcnt, 0, sizeof(int64_t) * (m->ndof + 1), s) != hipSuccess) return fail(FPDE_EHIP);
  if (P.n_ent > 0) k_row_count<<<nblk(P.n_ent), 256, 0, s>>>(P.ent_dof, P.n_ent, rowcnt);
  if (hipcub::DeviceScan::ExclusiveSum(tmp, tb, rowcnt, P.row_off, (int)(m->ndof + 1), s) != hipSuccess)
    return fail(FPDE_EHIP);
  if (hipMemcpyAsync(cursor, P.row_off, sizeof(int64_t) * (m->ndof + 1), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return fail(FPDE_EHIP);
  if (P.n_ent > 0) k_row_fill<<<nblk(P.n_ent), 256, 0, s>>>(P.ent_dof, P.n_ent, cursor, P.inc);
  if ((st = dalloc(&P.inc_meta, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.inc_w, P.n_ent)) != FPDE_OK) return fail(st);
  if (P.n_ent > 0)
    k_inc_meta<<<nblk(P.n_ent), 256, 0, s>>>(P.inc, P.ent_ray, P.off, m->vol,
                                             m->rules + rule_offset(nq) + 4 * nq, P.G, nq, P.n_ent,
                                             P.inc_meta, P.inc_w);
  if (hipGetLastError() != hipSuccess) return fail(FPDE_EHIP);
  f = take_flag(m, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);
  dfree(cnt); dfree(cnt64); dfree(rowcnt); dfree(cursor);
  (void)hipFree(tmp);
  // sizes for reporting: entry pairs the accumulation multiplies
  {
    std::vector<int64_t> off(P.n_half + 1);
    if (hipMemcpy(off.data(), P.off, sizeof(int64_t) * (P.n_half + 1), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(FPDE_EHIP);
    P.pairs = 0;
    P.max_ent = 0;
    for (int i = 0; i < 3; i++)
      for (int64_t g = 0; g < P.G; g++) {
        const int64_t hl = (int64_t)(2 * i) * P.G + g, hr = hl + P.G;
        const int64_t nl = off[hl + 1] - off[hl], nr = off[hr + 1] - off[hr];
        P.pairs += nl * nr;
        P.max_ent = std::max(P.max_ent, std::max(nl, nr));
      }
  }
  if ((st = build_tubes(m, P, kTubeCell, s)) != FPDE_OK) return fail(st);
  invalidate_values(&P);
  return FPDE_OK;
}

int plan_for(fpde_mesh *m, int nq, int max_steps, hipStream_t s, Plan **out) {
  if (nq != 4 && nq != 11) return FPDE_EINVAL;
  if (max_steps <= 0) max_steps = 4096;
  Plan &P = m->plan[nq == 4 ? 0 : 1];
  if (P.nq == nq && P.max_steps == max_steps) {
    *out = &P;
    return FPDE_OK;
  }
  free_plan(P);
  const long t = timer_begin(m, s, FPDE_STAGE_PLAN);
  FPDE_TRY(build_plan(m, P, nq, max_steps, s));
  timer_end(m, FPDE_STAGE_PLAN, t, s);
  *out = &P;
  return FPDE_OK;
}

// Fills the plan's entry values (walk + closed-form eval) for the axes whose
// order changed, in one launch over the contiguous range of half-rays that
// covers them (the half-rays along e_i are dir = 2i, 2i + 1, i.e.
// [2 i G, (2 i + 2) G)); each thread takes its axis's order.
int ensure_values_axes(fpde_mesh *m, Plan *P, const double gamma[3], hipStream_t s, int slot) {
  double *cache = slot == 0 ? P->val_gamma : P->val_gamma2;
  if (slot == 1 && !P->ent_val2) FPDE_TRY(dalloc(&P->ent_val2, P->n_ent));
  double *dest = slot == 0 ? P->ent_val : P->ent_val2;
  int i0 = 3, i1 = -1;
  for (int i = 0; i < 3; i++)
    if (cache[i] != gamma[i]) {
      i0 = i < i0 ? i : i0;
      i1 = i;
    }
  if (i1 < 0) return FPDE_OK;
  QuadRule rule;
  FPDE_TRY(quad_rule(P->nq, &rule));
  WalkArgs a = base_args(m, *P, rule);
  for (int i = 0; i < 3; i++) {
    const Order o = gamma_scalars(gamma[i]);
    a.e[i] = o.e;
    a.inv_g2[i] = o.inv_g2;
  }
  a.h0 = (int64_t)(2 * i0) * P->G;
  a.n = (int64_t)(2 * (i1 - i0 + 1)) * P->G;
  a.off = P->off;
  a.ent_val = dest;
  const long t = timer_begin(m, s, FPDE_STAGE_WALK);
  launch_walk<W_VALUES>(a, s);
  timer_end(m, FPDE_STAGE_WALK, t, s);
  if (hipGetLastError() != hipSuccess) {
    invalidate_values(P);
    return FPDE_EHIP;
  }
  for (int i = i0; i <= i1; i++) cache[i] = gamma[i];
  if (slot == 0) P->values_version++;
  return FPDE_OK;
}

int ensure_values(fpde_mesh *m, Plan *P, double alpha, hipStream_t s) {
  const double g[3] = {0.5 * alpha, 0.5 * alpha, 0.5 * alpha};
  return ensure_values_axes(m, P, g, s);
}

// Adjoint dots per half-ray (re-walks every path): value.u, value.lam,
// (d/dalpha value).u, (d/dalpha value).lam.
int walk_adjoint(fpde_mesh *m, Plan *P, double alpha, const double *u, const double *lam, hipStream_t s) {
  QuadRule rule;
  FPDE_TRY(quad_rule(P->nq, &rule));
  Order o = order_scalars(alpha);
  if (!P->adj) FPDE_TRY(dalloc(&P->adj, 4 * P->n_half));
  WalkArgs a = base_args(m, *P, rule);
  a.h0 = 0;
  a.n = P->n_half;
  for (int i = 0; i < 3; i++) {
    a.e[i] = o.e;
    a.inv_g2[i] = o.inv_g2;
  }
  a.half_psi0 = o.half_psi0;
  a.u = u;
  a.lam = lam;
  a.adj = P->adj;
  const long t = timer_begin(m, s, FPDE_STAGE_ADJOINT);
  launch_walk<W_ADJ>(a, s);
  timer_end(m, FPDE_STAGE_ADJOINT, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_plan(fpde_mesh *m, int quad_points, int max_steps, void *stream) {
  if (!m) return FPDE_EINVAL;
  Plan *P = nullptr;
  return plan_for(m, quad_points, max_steps, S(stream), &P);
}

extern "C" int fpde_paths(fpde_mesh *m, int quad_points, int dir, int64_t g0, int64_t count, int max_steps,
                          int32_t *len, uint64_t *hash, int32_t *ids, double *rend, void *stream) {
  if (!m || dir < 0 || dir > 5 || g0 < 0 || count < 0 || !len || !hash) return FPDE_EINVAL;
  QuadRule rule;
  FPDE_TRY(quad_rule(quad_points, &rule));
  if (max_steps <= 0) max_steps = 4096;
  const int64_t G = m->nt * quad_points;
  if (g0 + count > G) return FPDE_EINVAL;
  if (count == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  Plan tmp;
  tmp.G = G;
  tmp.max_steps = max_steps;
  int32_t *cnt = nullptr;
  FPDE_TRY(dalloc(&cnt, count));
  WalkArgs a = base_args(m, tmp, rule);
  a.h0 = (int64_t)dir * G + g0;
  a.n = count;
  a.cnt = cnt;
  a.len = len;
  a.hash = hash;
  a.ids = ids;
  a.rend = rend;
  launch_walk<W_COUNT>(a, s);
  int f = (hipGetLastError() == hipSuccess) ? take_flag(m, s) : FPDE_EHIP;
  dfree(cnt);
  return f;
}

extern "C" int fpde_ray_values(fpde_mesh *m, int quad_points, double alpha, int dir, int64_t g0, int64_t count,
                               int64_t *off, int32_t *dof, double *val, int64_t capacity, void *stream) {
  if (!m || !off || dir < 0 || dir > 5 || g0 < 0 || count < 0) return FPDE_EINVAL;
  if (!(alpha > 1.0 && alpha <= 2.0)) return FPDE_EALPHA;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, quad_points, 0, s, &P));
  if (g0 + count > P->G) return FPDE_EINVAL;
  FPDE_TRY(ensure_values(m, P, alpha, s));
  const int64_t h0 = (int64_t)dir * P->G + g0;
  FPDE_HIP(hipMemcpyAsync(off, P->off + h0, sizeof(int64_t) * (count + 1), hipMemcpyDeviceToHost, s));
  FPDE_HIP(hipStreamSynchronize(s));
  const int64_t e0 = off[0];
  for (int64_t k = 0; k <= count; k++) off[k] -= e0;
  const int64_t n = off[count];
  int f = take_flag(m, s);
  if (f != 0) return f;
  if (n > capacity || (n > 0 && (!dof || !val))) return FPDE_EINVAL;
  if (n > 0) {
    FPDE_HIP(hipMemcpyAsync(dof, P->ent_dof + e0, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    FPDE_HIP(hipMemcpyAsync(val, P->ent_val + e0, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    FPDE_HIP(hipStreamSynchronize(s));
  }
  return FPDE_OK;
}

extern "C" int fpde_plan_info(fpde_mesh *m, int quad_points, int64_t *out, void *stream) {
  if (!m || !out) return FPDE_EINVAL;
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, quad_points, 0, S(stream), &P));
  out[0] = P->n_half;
  out[1] = P->n_ent;
  out[2] = P->pairs;
  out[3] = P->max_ent;
  out[4] = P->tubes.n_tubes;
  out[5] = P->tubes.n_u;
  out[6] = P->tubes.max_u;
  out[7] = P->tubes.blk_n * (int64_t)sizeof(double);
  return FPDE_OK;
}
