// The two-dimensional variant (n = 2): P1 elements on a convex triangulated
// polygon, integration paths along +-e_1 and +-e_2 (Sec. 1 with n = 2,
// Fig. 1a; the walk of Sec. 2.2 with three area coordinates), the split Riesz
// stiffness
//
//   K_jk = c_alpha sum_i K_i sum_g w_g [L_gi(k) R_gi(j) + R_gi(k) L_gi(j)],  i = 1, 2,
//
// its load vector and the dense solve.  Everything runs on the GPU:
//   mesh set-up   A^{-1} per triangle (adjugate), edge adjacency by sorting
//                 sorted vertex pairs, boundary, interior numbering, vertex
//                 -> triangle lists;
//   k2_walk       one thread per half-ray (h = dir G + g, dir = 2 i + side):
//                 the path (edge go-out: the triangle across it; vertex
//                 go-out: the smallest-id triangle around the vertex in which
//                 the ray advances), fused with the closed-form order-gamma
//                 derivatives of the P1 basis (a 3-slot window over the
//                 current triangle's vertices); the same IEEE arithmetic as
//                 the reference definition, no FMA contraction, so element
//                 ids are reproducible bit for bit;
//   plan          entry counts and offsets, node -> entry transpose with the
//                 partner half-ray of every incidence;
//   k2_rows       one workgroup per (row, column chunk): row j adds, for each
//                 incidence of node j, W value times the partner half-ray's
//                 vector into an LDS row chunk (16 lanes per vector); the
//                 chunk is written once;
//   solve         the dense FP64 Cholesky of the 3-D path.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "fpde_internal.h"

namespace fpde {

// One triangle as the walk reads it: A^{-1} row-major (row r = gradient of
// area coordinate k_{r+1}), vertex 0, neighbour across edge f (opposite
// local vertex f, -1 = boundary), unknown of local vertex f (-1 = boundary).
struct TriRec {
  double M[4];
  double v0[2];
  int32_t nbr[3];
  int32_t dof[3];
};

struct Plan2 {
  int nq = 0, max_steps = 0;
  int64_t G = 0, n_half = 0, n_ent = 0;
  int64_t *off = nullptr;
  int32_t *ent_dof = nullptr, *ent_ray = nullptr;
  double *ent_val = nullptr;
  double val_alpha = -1.0;
  int64_t *row_off = nullptr;
  int4 *inc_meta = nullptr;  // entry, partner offset, partner length << 1 | axis, partner
  double *inc_w = nullptr;
};

}  // namespace fpde

struct fpde_mesh2d {
  int64_t nv = 0, nt = 0, ndof = 0, nbe = 0;
  double *xy = nullptr;
  int32_t *tri = nullptr;
  fpde::TriRec *rec = nullptr;
  double *area = nullptr;
  int32_t *vt_off = nullptr, *vt_tri = nullptr, *dof = nullptr, *vert_of_dof = nullptr;
  double *rules = nullptr;  // [3-point | 7-point]: nq x 3 barycentric coordinates, then nq weights
  fpde::Plan2 plan[2];
  fpde_mesh *ws = nullptr;  // flags, timers and dense-solve scratch
};

namespace fpde {

namespace {

inline unsigned nblk2(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
inline int rule2_offset(int nq) { return nq == 3 ? 0 : 3 * 4; }

int quad_rule2(int nq, double *bary, double *w) {
  if (nq == 3) {
    for (int q = 0; q < 3; q++) {
      for (int j = 0; j < 3; j++) bary[3 * q + j] = (j == q) ? 2.0 / 3.0 : 1.0 / 6.0;
      w[q] = 1.0 / 3.0;
    }
    return FPDE_OK;
  }
  if (nq == 7) {  // Radon's degree-5 rule
    const double r15 = std::sqrt(15.0);
    const double a[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
    const double wa[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
    for (int j = 0; j < 3; j++) bary[j] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    int q = 1;
    for (int o = 0; o < 2; o++)
      for (int v = 0; v < 3; v++, q++) {
        for (int j = 0; j < 3; j++) bary[3 * q + j] = (j == v) ? 1.0 - 2.0 * a[o] : a[o];
        w[q] = wa[o];
      }
    return FPDE_OK;
  }
  return FPDE_EINVAL;
}

// ---------------------------------------------------------------------------
// mesh set-up
// ---------------------------------------------------------------------------
__global__ void k2_affine(const double *__restrict__ xy, const int32_t *__restrict__ tri, int64_t nt,
                          TriRec *__restrict__ rec, double *__restrict__ area, int32_t *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  const double *v0 = xy + 2 * (int64_t)a, *v1 = xy + 2 * (int64_t)b, *v2 = xy + 2 * (int64_t)c;
  const double e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e2x = v2[0] - v0[0], e2y = v2[1] - v0[1];
  const double det = e1x * e2y - e2x * e1y;
  const double l1 = sqrt(e1x * e1x + e1y * e1y), l2 = sqrt(e2x * e2x + e2y * e2y);
  const double L = l1 > l2 ? l1 : l2;
  if (a == b || a == c || b == c || !(fabs(det) > 1e-13 * L * L)) {
    set_flag(flag, FPDE_EMESH_DEGENERATE);
    return;
  }
  TriRec R;
  R.M[0] = e2y / det;
  R.M[1] = -e2x / det;
  R.M[2] = -e1y / det;
  R.M[3] = e1x / det;
  R.v0[0] = v0[0];
  R.v0[1] = v0[1];
  for (int j = 0; j < 3; j++) {
    R.nbr[j] = -1;
    R.dof[j] = -1;
  }
  rec[t] = R;
  area[t] = fabs(det) / 2.0;
}

// edge f of triangle t (opposite local vertex f) -> sorted vertex pair key
__global__ void k2_edge_keys(const int32_t *__restrict__ tri, int64_t nt, uint64_t *__restrict__ key,
                             int32_t *__restrict__ val) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * nt) return;
  const int64_t t = k / 3;
  const int f = (int)(k - 3 * t);
  const uint32_t p = (uint32_t)tri[3 * t + (f + 1) % 3], q = (uint32_t)tri[3 * t + (f + 2) % 3];
  key[k] = p < q ? (((uint64_t)p << 32) | q) : (((uint64_t)q << 32) | p);
  val[k] = (int32_t)k;
}

__global__ void k2_edge_match(const uint64_t *__restrict__ key, const int32_t *__restrict__ val, int64_t n,
                              int32_t *__restrict__ nbr3, int32_t *flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (p > 0 && key[p - 1] == key[p]) return;
  if (p + 1 < n && key[p + 1] == key[p]) {
    if (p + 2 < n && key[p + 2] == key[p]) {
      set_flag(flag, FPDE_EMESH_NONMANIFOLD);
      return;
    }
    const int32_t a = val[p], b = val[p + 1];
    nbr3[a] = b / 3;
    nbr3[b] = a / 3;
  }
}

__global__ void k2_boundary(const int32_t *__restrict__ tri, const int32_t *__restrict__ nbr3, int64_t nt,
                            int32_t *__restrict__ used, int32_t *__restrict__ bnd,
                            unsigned long long *__restrict__ nbe) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * nt) return;
  const int64_t t = k / 3;
  const int f = (int)(k - 3 * t);
  used[tri[k]] = 1;
  if (nbr3[k] < 0) {
    bnd[tri[3 * t + (f + 1) % 3]] = 1;
    bnd[tri[3 * t + (f + 2) % 3]] = 1;
    atomicAdd(nbe, 1ull);
  }
}

__global__ void k2_isdof(const int32_t *__restrict__ used, const int32_t *__restrict__ bnd, int64_t nv,
                         int32_t *__restrict__ isdof) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) isdof[v] = (used[v] && !bnd[v]) ? 1 : 0;
}

__global__ void k2_dof(const int32_t *__restrict__ isdof, const int32_t *__restrict__ scan, int64_t nv,
                       int32_t *__restrict__ dof, int32_t *__restrict__ vert_of_dof) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  if (isdof[v]) {
    dof[v] = scan[v];
    vert_of_dof[scan[v]] = (int32_t)v;
  } else {
    dof[v] = -1;
  }
}

__global__ void k2_finalize(const int32_t *__restrict__ tri, const int32_t *__restrict__ nbr3,
                            const int32_t *__restrict__ dof, int64_t nt, TriRec *__restrict__ rec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  for (int j = 0; j < 3; j++) {
    rec[t].nbr[j] = nbr3[3 * t + j];
    rec[t].dof[j] = dof[tri[3 * t + j]];
  }
}

__global__ void k2_vt_keys(const int32_t *__restrict__ tri, int64_t nt, uint32_t *__restrict__ key,
                           int32_t *__restrict__ val, int32_t *__restrict__ count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * nt) return;
  key[k] = (uint32_t)tri[k];
  val[k] = (int32_t)(k / 3);
  atomicAdd(&count[tri[k]], 1);
}

__global__ void k2_fill(int32_t *p, int64_t n, int32_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

int bits2(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

// ---------------------------------------------------------------------------
// walk + closed-form derivatives
// ---------------------------------------------------------------------------
enum Walk2Mode { W2_COUNT = 0, W2_STRUCT = 1, W2_VALUES = 2 };

struct Walk2Args {
  const TriRec *rec;
  const double *xy;
  const int32_t *tri, *vt_off, *vt_tri;
  int32_t *flag;
  int64_t *flag_aux;
  int64_t G, h0, n;
  int cap, nq;
  const double *qbary;  // nq x 3
  double e, inv_g2;     // 1 - gamma, 1/Gamma(2 - gamma)
  int32_t *cnt, *len;   // W2_COUNT
  uint64_t *hash;
  int32_t *ids;
  double *rend;
  const int64_t *off;   // W2_STRUCT / W2_VALUES
  int32_t *ent_dof, *ent_ray;
  double *ent_val;
};

struct Isect2 {
  double bt[3], dt[3], r_max;
  int jexit;
};

__device__ __forceinline__ double mcol2(const TriRec &R, int r, int i) { return i == 0 ? R.M[2 * r] : R.M[2 * r + 1]; }

__device__ __forceinline__ void isect2(const TriRec &R, const double *u0, int i, int s, Isect2 &o) {
  const double b0 = u0[0] - R.v0[0], b1 = u0[1] - R.v0[1];
#pragma unroll
  for (int r = 0; r < 2; r++) {
    o.bt[r + 1] = R.M[2 * r] * b0 + R.M[2 * r + 1] * b1;
    const double m = mcol2(R, r, i);
    o.dt[r + 1] = (s > 0) ? m : -m;
  }
  o.bt[0] = 1.0 - (o.bt[1] + o.bt[2]);
  o.dt[0] = -(o.dt[1] + o.dt[2]);
  double rm = INFINITY;
  int je = -1;
#pragma unroll
  for (int j = 0; j < 3; j++)
    if (o.dt[j] < 0.0) {
      const double r = -o.bt[j] / o.dt[j];
      if (r < rm) {
        rm = r;
        je = j;
      }
    }
  o.r_max = rm;
  o.jexit = je;
}

__device__ __forceinline__ double slope2(const TriRec &R, int j, int i) {
  if (j > 0) return mcol2(R, j - 1, i);
  return -(mcol2(R, 0, i) + mcol2(R, 1, i));
}

// r^e for r > 0 as exp(e ln r) (e in (0, 1], r a chord length): a few ulp
// from the correctly rounded power; the values need 1e-10, not bit equality
__device__ __forceinline__ double powr2(double r, double e) { return r > 0.0 ? exp(e * log(r)) : 0.0; }

template <int MODE>
__global__ void __launch_bounds__(256) k2_walk(Walk2Args a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const int64_t h = a.h0 + k;
  const int dir = (int)(h / a.G);
  const int64_t g = h - (int64_t)dir * a.G;
  const int i = dir >> 1, side = dir & 1;
  const int s = side ? 1 : -1;
  const int64_t t0 = g / a.nq;
  const int q = (int)(g - t0 * a.nq);
  double u0[2];
#pragma unroll
  for (int d = 0; d < 2; d++) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 3; j++) acc = acc + a.qbary[3 * q + j] * a.xy[2 * (int64_t)a.tri[3 * t0 + j] + d];
    u0[d] = acc;
  }
  int32_t wd[3] = {-1, -1, -1};
  double wv[3] = {0.0, 0.0, 0.0};
  int64_t nemit = 0, base = 0;
  if (MODE != W2_COUNT) base = a.off[h];
  const double sgn = side ? -1.0 : 1.0;
  auto emit = [&](int32_t d, double v) {
    if (MODE == W2_STRUCT) {
      a.ent_dof[base + nemit] = d;
      a.ent_ray[base + nemit] = (int32_t)h;
    } else if (MODE == W2_VALUES) {
      a.ent_val[base + nemit] = v;
    }
    nemit++;
  };
  uint64_t hsh = 14695981039346656037ull;
  int64_t t = t0;
  double r_cur = 0.0, P_lo = 0.0;
  int nseg = 0;
  int status = FPDE_EPATH;
  for (int step = 0; step < a.cap + 64; step++) {
    const TriRec R = a.rec[t];
    Isect2 o;
    isect2(R, u0, i, s, o);
    if (!(o.r_max < INFINITY)) break;
    if (o.r_max > r_cur) {
      if (nseg >= a.cap) break;
      if (MODE == W2_COUNT) {
        const uint32_t uid = (uint32_t)t;
#pragma unroll
        for (int b = 0; b < 4; b++) {
          hsh ^= (uint64_t)((uid >> (8 * b)) & 0xffu);
          hsh *= 1099511628211ull;
        }
        if (a.ids) a.ids[k * a.cap + nseg] = (int32_t)t;
        if (a.rend) a.rend[k * a.cap + nseg] = o.r_max;
      }
      {
        const int32_t nd[3] = {R.dof[0], R.dof[1], R.dof[2]};
        double na[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; j++) {
          if (wd[j] < 0) continue;
          bool kept = false;
#pragma unroll
          for (int m = 0; m < 3; m++)
            if (nd[m] == wd[j]) {
              na[m] = wv[j];
              kept = true;
            }
          if (!kept) emit(wd[j], wv[j]);
        }
#pragma unroll
        for (int j = 0; j < 3; j++) {
          wd[j] = nd[j];
          wv[j] = na[j];
        }
      }
      if (MODE == W2_VALUES) {
        const double P_hi = powr2(o.r_max, a.e);
        const double dP = a.inv_g2 * (P_hi - P_lo);
        P_lo = P_hi;
#pragma unroll
        for (int j = 0; j < 3; j++)
          if (wd[j] >= 0) wv[j] += sgn * slope2(R, j, i) * dP;
      }
      nseg++;
      r_cur = o.r_max;
    }
    int zmask = 0, nz = 0, zf = -1;
#pragma unroll
    for (int j = 0; j < 3; j++) {
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
    if (nz == 0 || nz == 3) break;
    if (nz == 1) {
      const int32_t nx = zf == 0 ? R.nbr[0] : (zf == 1 ? R.nbr[1] : R.nbr[2]);
      if (nx < 0) {
        status = 0;
        break;
      }
      t = nx;
      continue;
    }
    // vertex go-out: the vertex whose coordinate is not zero
    const int keep = __builtin_ctz((~zmask) & 0x7);
    const int32_t v = a.tri[3 * t + keep];
    int64_t best = -1;
    for (int32_t p = a.vt_off[v]; p < a.vt_off[v + 1]; p++) {
      const int64_t c = a.vt_tri[p];
      if (c == t) continue;
      const TriRec Rc = a.rec[c];
      Isect2 oc;
      isect2(Rc, u0, i, s, oc);
      if (oc.r_max - r_cur > 1e-12 * r_cur) {
        best = c;
        break;
      }
    }
    if (best < 0) {
      status = 0;
      break;
    }
    t = best;
  }
  if (status == 0 && nseg == 0) status = FPDE_EPATH;
  if (status != 0) {
    set_flag(a.flag, status);
    atomicCAS((unsigned long long *)a.flag_aux, ~0ull, (unsigned long long)h);
    if (MODE == W2_COUNT) a.cnt[k] = 0;
    return;
  }
#pragma unroll
  for (int j = 0; j < 3; j++)
    if (wd[j] >= 0) emit(wd[j], wv[j]);
  if (MODE == W2_COUNT) {
    a.cnt[k] = (int32_t)nemit;
    if (a.len) a.len[k] = nseg;
    if (a.hash) a.hash[k] = hsh;
  }
}

__global__ void k2_i32_to_i64(const int32_t *__restrict__ a, int64_t n, int64_t *__restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = a[k];
}

__global__ void k2_row_count(const int32_t *__restrict__ ent_dof, int64_t n, int64_t *__restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) atomicAdd((unsigned long long *)&cnt[ent_dof[e]], 1ull);
}

// incidence record of entry e, placed at its node's next free slot
__global__ void k2_inc_fill(const int32_t *__restrict__ ent_dof, const int32_t *__restrict__ ent_ray,
                            const int64_t *__restrict__ off, const double *__restrict__ area,
                            const double *__restrict__ wq, int64_t G, int nq, int64_t n,
                            int64_t *__restrict__ cursor, int4 *__restrict__ meta, double *__restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t p = (int64_t)atomicAdd((unsigned long long *)&cursor[ent_dof[e]], 1ull);
  const int64_t h = ent_ray[e];
  const int dir = (int)(h / G);
  const int64_t g = h - (int64_t)dir * G;
  const int64_t partner = (dir & 1) ? h - G : h + G;
  const int64_t po = off[partner], pl = off[partner + 1] - po;
  meta[p] = make_int4((int)e, (int)po, (int)((pl << 1) | (dir >> 1)), (int)partner);
  w[p] = wq[g % nq] * area[g / nq];
}

// ---------------------------------------------------------------------------
// accumulation: row j = sum over incidences of node j of W value(e) x partner vector
// ---------------------------------------------------------------------------
constexpr int kChunk2 = 8192;
constexpr int kBatch2 = 512;

struct Rows2Args {
  const int64_t *row_off;
  const int4 *meta;
  const double *w;
  const int32_t *ent_dof;
  const double *ent_val;
  int64_t ndof, lda;
  int chunk;
  double KC0, KC1;  // K_i c_alpha
};

struct Inc2 {
  int32_t p0, n;
  double c;
};

__device__ __forceinline__ int64_t clamp2(int32_t e0, int32_t n, int k) {
  return n > 0 ? (int64_t)e0 + (k < n ? k : n - 1) : 0;
}

__global__ void __launch_bounds__(256) k2_rows(Rows2Args a, double *__restrict__ A) {
  __shared__ double row[kChunk2];
  __shared__ Inc2 its[kBatch2];
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  const int64_t j = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * a.chunk;
  const int cw = (int)((a.ndof - c0) < a.chunk ? (a.ndof - c0) : a.chunk);
  for (int q = tid; q < cw; q += blockDim.x) row[q] = 0.0;
  const int64_t q0 = a.row_off[j], nin = a.row_off[j + 1] - q0;
  for (int64_t i0 = 0; i0 < nin; i0 += kBatch2) {
    const int nb = (int)((nin - i0) < kBatch2 ? (nin - i0) : kBatch2);
    for (int t = tid; t < nb; t += blockDim.x) {
      const int64_t p = q0 + i0 + t;
      const int4 mt = a.meta[p];
      Inc2 d;
      d.p0 = mt.y;
      d.n = mt.z >> 1;
      d.c = a.w[p] * ((mt.z & 1) ? a.KC1 : a.KC0) * a.ent_val[mt.x];
      its[t] = d;
    }
    __syncthreads();
    for (int t = grp; t < nb; t += 32) {
      const Inc2 P = its[t];
      Inc2 Q = P;
      if (t + 16 < nb) Q = its[t + 16];
      else Q.n = 0;
      const int nmax = P.n > Q.n ? P.n : Q.n;
      for (int b = 0; b < nmax; b += 16) {
        const int kk = b + gl;
        const int64_t ep = clamp2(P.p0, P.n, kk), eq = clamp2(Q.p0, Q.n, kk);
        const int32_t dp = a.ent_dof[ep], dq = a.ent_dof[eq];
        const double vp = a.ent_val[ep], vq = a.ent_val[eq];
        const int64_t cp = (int64_t)dp - c0, cq = (int64_t)dq - c0;
        if (kk < P.n && (uint64_t)cp < (uint64_t)cw) atomicAdd(&row[cp], P.c * vp);
        if (kk < Q.n && (uint64_t)cq < (uint64_t)cw) atomicAdd(&row[cq], Q.c * vq);
      }
    }
    __syncthreads();
  }
  __syncthreads();
  double *out = A + j * a.lda + c0;
  for (int q = tid; q < cw; q += blockDim.x) out[q] = row[q];
}

// ---------------------------------------------------------------------------
// load: b_j = sum over triangles of node j, points q: w_q |T| f(x_q) lambda_j(x_q)
// ---------------------------------------------------------------------------
struct Load2Args {
  const int32_t *vert_of_dof, *vt_off, *vt_tri, *tri;
  const double *xy, *area, *f_gauss, *qtab;
  int64_t ndof;
  int nq, src;
  double K0, K1, c_alpha, alpha, rg3, rg4, rg5;
};

__device__ __forceinline__ double mms_phi2(double s) { return s * s * (1.0 - s) * (1.0 - s); }
__device__ __forceinline__ double mms_Phi2(double s, const Load2Args &a) {
  return 2.0 * pow(s, 2.0 - a.alpha) * a.rg3 - 12.0 * pow(s, 3.0 - a.alpha) * a.rg4 +
         24.0 * pow(s, 4.0 - a.alpha) * a.rg5;
}

__global__ void k2_load(Load2Args a, double *__restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.ndof) return;
  const int32_t v = a.vert_of_dof[j];
  double sum = 0.0;
  for (int32_t p = a.vt_off[v]; p < a.vt_off[v + 1]; p++) {
    const int64_t t = a.vt_tri[p];
    int jl = 0;
    int32_t vv[3];
    for (int m = 0; m < 3; m++) {
      vv[m] = a.tri[3 * t + m];
      if (vv[m] == v) jl = m;
    }
    for (int q = 0; q < a.nq; q++) {
      double f = 1.0;
      if (a.src == FPDE_SRC_USER) {
        f = a.f_gauss[t * a.nq + q];
      } else if (a.src == FPDE_SRC_SQUARE_MMS) {
        double x[2];
        for (int d = 0; d < 2; d++) {
          double s = 0.0;
          for (int m = 0; m < 3; m++) s = s + a.qtab[3 * q + m] * a.xy[2 * (int64_t)vv[m] + d];
          x[d] = s;
        }
        f = a.K0 * a.c_alpha * (mms_Phi2(x[0], a) + mms_Phi2(1.0 - x[0], a)) * mms_phi2(x[1]) +
            a.K1 * a.c_alpha * (mms_Phi2(x[1], a) + mms_Phi2(1.0 - x[1], a)) * mms_phi2(x[0]);
      }
      sum += a.qtab[3 * a.nq + q] * a.area[t] * f * a.qtab[3 * q + jl];
    }
  }
  b[j] = sum;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void free_plan2(Plan2 &P) {
  dfree(P.off); dfree(P.ent_dof); dfree(P.ent_ray); dfree(P.ent_val); dfree(P.row_off); dfree(P.inc_meta);
  dfree(P.inc_w);
  P = Plan2();
}

static Walk2Args walk2_args(fpde_mesh2d *m, const Plan2 &P) {
  Walk2Args a{};
  a.rec = m->rec;
  a.xy = m->xy;
  a.tri = m->tri;
  a.vt_off = m->vt_off;
  a.vt_tri = m->vt_tri;
  a.flag = m->ws->flag;
  a.flag_aux = m->ws->flag_aux;
  a.G = P.G;
  a.cap = P.max_steps;
  a.nq = P.nq;
  a.qbary = m->rules + rule2_offset(P.nq);
  return a;
}

template <int MODE>
static void launch_walk2(const Walk2Args &a, hipStream_t s) {
  if (a.n > 0) k2_walk<MODE><<<nblk2(a.n), 256, 0, s>>>(a);
}

static int build_plan2(fpde_mesh2d *m, Plan2 &P, int nq, int max_steps, hipStream_t s) {
  P.nq = nq;
  P.max_steps = max_steps;
  P.G = m->nt * nq;
  P.n_half = 4 * P.G;
  int32_t *cnt = nullptr;
  int64_t *cnt64 = nullptr, *rowcnt = nullptr, *cursor = nullptr;
  void *tmp = nullptr;
  auto fail = [&](int code) {
    dfree(cnt); dfree(cnt64); dfree(rowcnt); dfree(cursor);
    if (tmp) (void)hipFree(tmp);
    free_plan2(P);
    return code;
  };
  int st;
  if ((st = dalloc(&cnt, P.n_half + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&cnt64, P.n_half + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.off, P.n_half + 1)) != FPDE_OK) return fail(st);
  k2_fill<<<nblk2(P.n_half + 1), 256, 0, s>>>(cnt, P.n_half + 1, 0);
  Walk2Args a = walk2_args(m, P);
  a.h0 = 0;
  a.n = P.n_half;
  a.cnt = cnt;
  launch_walk2<W2_COUNT>(a, s);
  k2_i32_to_i64<<<nblk2(P.n_half + 1), 256, 0, s>>>(cnt, P.n_half + 1, cnt64);
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
  int f = take_flag(m->ws, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);
  if (P.n_ent >= (int64_t(1) << 31)) return fail(FPDE_EUNSUPPORTED);
  if ((st = dalloc(&P.ent_dof, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.ent_ray, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.ent_val, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.row_off, m->ndof + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&rowcnt, m->ndof + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&cursor, m->ndof + 1)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.inc_meta, P.n_ent)) != FPDE_OK) return fail(st);
  if ((st = dalloc(&P.inc_w, P.n_ent)) != FPDE_OK) return fail(st);
  a.off = P.off;
  a.ent_dof = P.ent_dof;
  a.ent_ray = P.ent_ray;
  launch_walk2<W2_STRUCT>(a, s);
  if (hipMemsetAsync(rowcnt, 0, sizeof(int64_t) * (m->ndof + 1), s) != hipSuccess) return fail(FPDE_EHIP);
  if (P.n_ent > 0) k2_row_count<<<nblk2(P.n_ent), 256, 0, s>>>(P.ent_dof, P.n_ent, rowcnt);
  if (hipcub::DeviceScan::ExclusiveSum(tmp, tb, rowcnt, P.row_off, (int)(m->ndof + 1), s) != hipSuccess)
    return fail(FPDE_EHIP);
  if (hipMemcpyAsync(cursor, P.row_off, sizeof(int64_t) * (m->ndof + 1), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return fail(FPDE_EHIP);
  if (P.n_ent > 0)
    k2_inc_fill<<<nblk2(P.n_ent), 256, 0, s>>>(P.ent_dof, P.ent_ray, P.off, m->area,
                                               m->rules + rule2_offset(nq) + 3 * nq, P.G, nq, P.n_ent, cursor,
                                               P.inc_meta, P.inc_w);
  if (hipGetLastError() != hipSuccess) return fail(FPDE_EHIP);
  f = take_flag(m->ws, s);
  if (f != 0) return fail(f < 0 ? f : FPDE_EHIP);
  dfree(cnt); dfree(cnt64); dfree(rowcnt); dfree(cursor);
  (void)hipFree(tmp);
  P.val_alpha = -1.0;
  return FPDE_OK;
}

static int plan2_for(fpde_mesh2d *m, int nq, int max_steps, hipStream_t s, Plan2 **out) {
  if (nq != 3 && nq != 7) return FPDE_EINVAL;
  if (max_steps <= 0) max_steps = 4096;
  Plan2 &P = m->plan[nq == 3 ? 0 : 1];
  if (P.nq == nq && P.max_steps == max_steps) {
    *out = &P;
    return FPDE_OK;
  }
  free_plan2(P);
  const long t = timer_begin(m->ws, s, FPDE_STAGE_PLAN);
  FPDE_TRY(build_plan2(m, P, nq, max_steps, s));
  timer_end(m->ws, FPDE_STAGE_PLAN, t, s);
  *out = &P;
  return FPDE_OK;
}

static int mesh2_build(fpde_mesh2d *m, const double *xy, const int32_t *tri, hipStream_t s) {
  const int64_t nv = m->nv, nt = m->nt, ne = 3 * nt;
  FPDE_TRY(dalloc(&m->xy, 2 * nv));
  FPDE_TRY(dalloc(&m->tri, ne));
  FPDE_TRY(dalloc(&m->rec, nt));
  FPDE_TRY(dalloc(&m->area, nt));
  FPDE_TRY(dalloc(&m->vt_off, nv + 1));
  FPDE_TRY(dalloc(&m->vt_tri, ne));
  FPDE_TRY(dalloc(&m->dof, nv));
  {
    double tab[3 * 4 + 7 * 4];
    for (int nq : {3, 7}) {
      double *o = tab + rule2_offset(nq);
      FPDE_TRY(quad_rule2(nq, o, o + 3 * nq));
    }
    FPDE_TRY(dalloc(&m->rules, sizeof(tab) / sizeof(double)));
    FPDE_HIP(hipMemcpyAsync(m->rules, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    FPDE_HIP(hipStreamSynchronize(s));
  }
  FPDE_HIP(hipMemcpyAsync(m->xy, xy, sizeof(double) * 2 * nv, hipMemcpyHostToDevice, s));
  FPDE_HIP(hipMemcpyAsync(m->tri, tri, sizeof(int32_t) * ne, hipMemcpyHostToDevice, s));
  k2_affine<<<nblk2(nt), 256, 0, s>>>(m->xy, m->tri, nt, m->rec, m->area, m->ws->flag);
  uint64_t *key = nullptr, *key2 = nullptr;
  int32_t *val = nullptr, *val2 = nullptr, *nbr3 = nullptr, *used = nullptr, *bnd = nullptr, *isdof = nullptr,
          *scan = nullptr, *cnt = nullptr;
  uint32_t *vkey = nullptr, *vkey2 = nullptr;
  unsigned long long *nbe = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  int st = FPDE_OK;
  auto cleanup = [&]() {
    dfree(key); dfree(key2); dfree(val); dfree(val2); dfree(nbr3); dfree(used); dfree(bnd);
    dfree(isdof); dfree(scan); dfree(cnt); dfree(vkey); dfree(vkey2); dfree(nbe);
    if (tmp) (void)hipFree(tmp);
  };
#define STEP2(x)         \
  do {                   \
    st = (x);            \
    if (st != FPDE_OK) { \
      cleanup();         \
      return st;         \
    }                    \
  } while (0)
#define STEPH2(x) STEP2(((x) == hipSuccess) ? FPDE_OK : FPDE_EHIP)
  STEP2(dalloc(&key, ne));
  STEP2(dalloc(&key2, ne));
  STEP2(dalloc(&val, ne));
  STEP2(dalloc(&val2, ne));
  STEP2(dalloc(&nbr3, ne));
  STEP2(dalloc(&used, nv));
  STEP2(dalloc(&bnd, nv));
  STEP2(dalloc(&isdof, nv + 1));
  STEP2(dalloc(&scan, nv + 1));
  STEP2(dalloc(&cnt, nv + 1));
  STEP2(dalloc(&vkey, ne));
  STEP2(dalloc(&vkey2, ne));
  STEP2(dalloc(&nbe, 1));
  k2_edge_keys<<<nblk2(ne), 256, 0, s>>>(m->tri, nt, key, val);
  const int end_bit = 32 + bits2((uint64_t)nv);
  size_t need = 0, need2 = 0, need3 = 0;
  STEPH2(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key, key2, val, val2, (int)ne, 0, end_bit, s));
  STEPH2(hipcub::DeviceRadixSort::SortPairs(nullptr, need2, vkey, vkey2, val, val2, (int)ne, 0,
                                            bits2((uint64_t)nv), s));
  STEPH2(hipcub::DeviceScan::ExclusiveSum(nullptr, need3, isdof, scan, (int)(nv + 1), s));
  tmp_bytes = std::max(need, std::max(need2, need3));
  STEPH2(hipMalloc(&tmp, tmp_bytes));
  STEPH2(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, val2, (int)ne, 0, end_bit, s));
  k2_fill<<<nblk2(ne), 256, 0, s>>>(nbr3, ne, -1);
  k2_edge_match<<<nblk2(ne), 256, 0, s>>>(key2, val2, ne, nbr3, m->ws->flag);
  k2_fill<<<nblk2(nv), 256, 0, s>>>(used, nv, 0);
  k2_fill<<<nblk2(nv), 256, 0, s>>>(bnd, nv, 0);
  k2_fill<<<1, 256, 0, s>>>(isdof + nv, 1, 0);
  STEPH2(hipMemsetAsync(nbe, 0, sizeof(unsigned long long), s));
  k2_boundary<<<nblk2(ne), 256, 0, s>>>(m->tri, nbr3, nt, used, bnd, nbe);
  k2_isdof<<<nblk2(nv), 256, 0, s>>>(used, bnd, nv, isdof);
  STEPH2(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, isdof, scan, (int)(nv + 1), s));
  int32_t ndof = 0;
  unsigned long long nbe_h = 0;
  STEPH2(hipMemcpyAsync(&ndof, scan + nv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  STEPH2(hipMemcpyAsync(&nbe_h, nbe, sizeof(nbe_h), hipMemcpyDeviceToHost, s));
  STEPH2(hipStreamSynchronize(s));
  m->ndof = ndof;
  m->nbe = (int64_t)nbe_h;
  m->ws->ndof = ndof;
  STEP2(dalloc(&m->vert_of_dof, ndof > 0 ? ndof : 1));
  k2_dof<<<nblk2(nv), 256, 0, s>>>(isdof, scan, nv, m->dof, m->vert_of_dof);
  k2_finalize<<<nblk2(nt), 256, 0, s>>>(m->tri, nbr3, m->dof, nt, m->rec);
  k2_fill<<<nblk2(nv + 1), 256, 0, s>>>(cnt, nv + 1, 0);
  k2_vt_keys<<<nblk2(ne), 256, 0, s>>>(m->tri, nt, vkey, val, cnt);
  STEPH2(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, vkey, vkey2, val, m->vt_tri, (int)ne, 0,
                                            bits2((uint64_t)nv), s));
  STEPH2(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, m->vt_off, (int)(nv + 1), s));
  STEPH2(hipGetLastError());
  const int f = take_flag(m->ws, s);
  cleanup();
  if (f != 0) return f < 0 ? f : FPDE_EHIP;
  return FPDE_OK;
#undef STEP2
#undef STEPH2
}

static int ensure_values2(fpde_mesh2d *m, Plan2 *P, double alpha, hipStream_t s) {
  if (P->val_alpha == alpha) return FPDE_OK;
  const Order o = order_scalars(alpha);
  Walk2Args a = walk2_args(m, *P);
  a.h0 = 0;
  a.n = P->n_half;
  a.e = o.e;
  a.inv_g2 = o.inv_g2;
  a.off = P->off;
  a.ent_val = P->ent_val;
  const long t = timer_begin(m->ws, s, FPDE_STAGE_WALK);
  launch_walk2<W2_VALUES>(a, s);
  timer_end(m->ws, FPDE_STAGE_WALK, t, s);
  FPDE_HIP(hipGetLastError());
  P->val_alpha = alpha;
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" void fpde_mesh2d_destroy(fpde_mesh2d *m) {
  if (!m) return;
  dfree(m->xy); dfree(m->tri); dfree(m->rec); dfree(m->area); dfree(m->vt_off); dfree(m->vt_tri);
  dfree(m->dof); dfree(m->vert_of_dof); dfree(m->rules);
  for (auto &P : m->plan) free_plan2(P);
  if (m->ws) fpde_mesh_destroy(m->ws);
  delete m;
}

extern "C" int fpde_mesh2d_create(const double *xy, int64_t n_vert, const int32_t *tri, int64_t n_tri,
                                  void *stream, fpde_mesh2d **out) {
  if (!out) return FPDE_EINVAL;
  *out = nullptr;
  if (!xy || !tri || n_vert < 3 || n_tri < 1) return FPDE_EINVAL;
  if (n_vert >= (int64_t(1) << 31) || 3 * n_tri >= (int64_t(1) << 31)) return FPDE_EUNSUPPORTED;
  for (int64_t k = 0; k < 3 * n_tri; k++)
    if (tri[k] < 0 || tri[k] >= n_vert) return FPDE_EINVAL;
  for (int64_t k = 0; k < 2 * n_vert; k++)
    if (!std::isfinite(xy[k])) return FPDE_EINVAL;
  fpde_mesh2d *m = new fpde_mesh2d();
  m->nv = n_vert;
  m->nt = n_tri;
  int st = workspace_new(0, &m->ws);
  if (st == FPDE_OK) st = mesh2_build(m, xy, tri, S(stream));
  if (st != FPDE_OK) {
    fpde_mesh2d_destroy(m);
    return st;
  }
  *out = m;
  return FPDE_OK;
}

extern "C" int fpde_mesh2d_info(const fpde_mesh2d *m, int64_t *n_dof, int64_t *n_boundary_edges, int64_t *n_tri) {
  if (!m) return FPDE_EINVAL;
  if (n_dof) *n_dof = m->ndof;
  if (n_boundary_edges) *n_boundary_edges = m->nbe;
  if (n_tri) *n_tri = m->nt;
  return FPDE_OK;
}

extern "C" int fpde_dof_map2d(const fpde_mesh2d *m, int32_t *dof) {
  if (!m || !dof) return FPDE_EINVAL;
  FPDE_HIP(hipMemcpy(dof, m->dof, sizeof(int32_t) * m->nv, hipMemcpyDeviceToHost));
  return FPDE_OK;
}

extern "C" int fpde_paths2d(fpde_mesh2d *m, int quad_points, int dir, int64_t g0, int64_t count, int max_steps,
                            int32_t *len, uint64_t *hash, int32_t *ids, double *rend, void *stream) {
  if (!m || dir < 0 || dir > 3 || g0 < 0 || count < 0 || !len || !hash) return FPDE_EINVAL;
  if (quad_points != 3 && quad_points != 7) return FPDE_EINVAL;
  if (max_steps <= 0) max_steps = 4096;
  const int64_t G = m->nt * quad_points;
  if (g0 + count > G) return FPDE_EINVAL;
  if (count == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  Plan2 tmp;
  tmp.G = G;
  tmp.nq = quad_points;
  tmp.max_steps = max_steps;
  int32_t *cnt = nullptr;
  FPDE_TRY(dalloc(&cnt, count));
  Walk2Args a = walk2_args(m, tmp);
  a.h0 = (int64_t)dir * G + g0;
  a.n = count;
  a.cnt = cnt;
  a.len = len;
  a.hash = hash;
  a.ids = ids;
  a.rend = rend;
  launch_walk2<W2_COUNT>(a, s);
  const int f = (hipGetLastError() == hipSuccess) ? take_flag(m->ws, s) : FPDE_EHIP;
  dfree(cnt);
  return f;
}

extern "C" int fpde_assemble2d(fpde_mesh2d *m, const fpde_params2d *p, double *A, int64_t lda, double *b,
                               const double *f_gauss, void *stream) {
  if (!m || !p || !A || lda < m->ndof) return FPDE_EINVAL;
  if (!(p->alpha > 1.0 && p->alpha <= 2.0) || !(p->K[0] > 0.0) || !(p->K[1] > 0.0)) return FPDE_EALPHA;
  if (p->quad_points != 3 && p->quad_points != 7) return FPDE_EINVAL;
  if (p->source != FPDE_SRC_ONE && p->source != FPDE_SRC_USER && p->source != FPDE_SRC_SQUARE_MMS)
    return FPDE_EINVAL;
  if (b && p->source == FPDE_SRC_USER && !f_gauss) return FPDE_EINVAL;
  if (m->ndof == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  Plan2 *P = nullptr;
  FPDE_TRY(plan2_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values2(m, P, p->alpha, s));
  const Order o = order_scalars(p->alpha);
  Rows2Args a{};
  a.row_off = P->row_off;
  a.meta = P->inc_meta;
  a.w = P->inc_w;
  a.ent_dof = P->ent_dof;
  a.ent_val = P->ent_val;
  a.ndof = m->ndof;
  a.lda = lda;
  a.chunk = (int)(m->ndof < kChunk2 ? m->ndof : kChunk2);
  a.KC0 = p->K[0] * o.c_alpha;
  a.KC1 = p->K[1] * o.c_alpha;
  const unsigned nchunk = (unsigned)((m->ndof + a.chunk - 1) / a.chunk);
  const long t = timer_begin(m->ws, s, FPDE_STAGE_CONTRACT);
  k2_rows<<<dim3((unsigned)m->ndof, nchunk), 256, 0, s>>>(a, A);
  timer_end(m->ws, FPDE_STAGE_CONTRACT, t, s);
  FPDE_HIP(hipGetLastError());
  if (b) {
    Load2Args l{};
    l.vert_of_dof = m->vert_of_dof;
    l.vt_off = m->vt_off;
    l.vt_tri = m->vt_tri;
    l.tri = m->tri;
    l.xy = m->xy;
    l.area = m->area;
    l.f_gauss = f_gauss;
    l.qtab = m->rules + rule2_offset(p->quad_points);
    l.ndof = m->ndof;
    l.nq = p->quad_points;
    l.src = p->source;
    l.K0 = p->K[0];
    l.K1 = p->K[1];
    l.c_alpha = o.c_alpha;
    l.alpha = p->alpha;
    l.rg3 = 1.0 / std::tgamma(3.0 - p->alpha);
    l.rg4 = 1.0 / std::tgamma(4.0 - p->alpha);
    l.rg5 = 1.0 / std::tgamma(5.0 - p->alpha);
    const long t2 = timer_begin(m->ws, s, FPDE_STAGE_LOAD);
    k2_load<<<nblk2(m->ndof), 256, 0, s>>>(l, b);
    timer_end(m->ws, FPDE_STAGE_LOAD, t2, s);
    FPDE_HIP(hipGetLastError());
  }
  const int f = take_flag(m->ws, s);
  if (f != 0) {
    P->val_alpha = -1.0;
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}

extern "C" int fpde_solve2d(fpde_mesh2d *m, double *A, int64_t lda, const double *b, double *u,
                            int64_t *failed_pivot, void *stream) {
  if (!m || !A || !b || !u || lda < m->ndof) return FPDE_EINVAL;
  return dense_spd_solve(m->ws, A, lda, m->ndof, b, u, failed_pivot, S(stream));
}

extern "C" int fpde_timing2d(fpde_mesh2d *m, int enable) {
  if (!m) return FPDE_EINVAL;
  return fpde_timing(m->ws, enable);
}

extern "C" int fpde_stage_times2d(fpde_mesh2d *m, double *ms, int64_t *count) {
  if (!m) return FPDE_EINVAL;
  return fpde_stage_times(m->ws, ms, count);
}
