// The divergence-form two-sided problem of Sec. 3 (eq. equ:sfde2):
//
//   sum_i D_i (p_i D_L^{beta_i} u - q_i D_R^{beta_i} u) = f,  u = 0 outside,
//
// in the weak form obtained by one classical integration by parts on the
// test side, a(u, v) = -sum_i [(p_i D_L u, D_i v) - (q_i D_R u, D_i v)].
// With the element quadrature of Sec. 2.1,
//
//   K_jk = -sum_i sum_g w_g (d_i psi_j)(x_g) [p_i(x_g) L_gi(k) - q_i(x_g) R_gi(k)],
//
// where L_gi / R_gi are the order-beta_i derivative vectors of the walked
// half-rays along e_i (the same walk and closed-form evaluation as the Riesz
// path, one order per axis) and d_i psi_j is the constant slope of psi_j on
// the Gauss point's own element.  Row j therefore collects, over the
// elements of its patch, every Gauss point and axis, two derivative vectors
// scaled by -w_g sigma_ji p_i and +w_g sigma_ji q_i.
//
//   k_div_rows  one workgroup per (row, column chunk): the chunk of the row
//               lives in LDS.  The row's (element, Gauss point, axis) items
//               are set up one per thread (coefficients, vector extents) into
//               LDS, then groups of 16 lanes sweep the items' vectors, each
//               group reading 16 consecutive entries of a vector per load
//               (a few cache lines per instruction), and add them with LDS
//               atomics; the chunk is then written to K once.
//   k_div_load  b_j = sum_g w_g f(x_g) psi_j(x_g), f = 1, user values, or
//               the closed-form source of u = (|x|^2 - r^2)^2 on the ball.
#include <cmath>

#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kDivChunk = 8192;  // doubles of one row chunk in LDS (64 KB)

struct DivArgs {
  const TetRec *rec;
  const int32_t *tet, *vt_off, *vt_tet, *vert_of_dof;
  const double *xyz, *vol;
  const double *qtab;  // nq x 4 barycentric coordinates, then nq weights
  int nq;
  int64_t G, ndof, lda;
  const int64_t *off;
  const int32_t *ent_dof;
  const double *ent_val;
  const double *pq;    // FPDE_COEF_USER: p_i at [i G + g], q_i at [(3 + i) G + g]; else null
  int chunk;
};

// slope of the volume coordinate of local vertex j along e_i
__device__ __forceinline__ double vslope(const TetRec &R, int j, int i) {
  const double a = R.M[i], b = R.M[3 + i], c = R.M[6 + i];
  if (j == 1) return a;
  if (j == 2) return b;
  if (j == 3) return c;
  return -((a + b) + c);
}

// coordinate d of Gauss point q of element t, summed in vertex order
__device__ __forceinline__ double gauss_coord(const DivArgs &a, int64_t t, int q, int d) {
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 4; m++) acc = acc + a.qtab[4 * q + m] * a.xyz[3 * (int64_t)a.tet[4 * t + m] + d];
  return acc;
}

// One (element, Gauss point, axis) item of a row: its two derivative
// vectors (first entry and length) and their scale factors.
struct DivItem {
  int32_t l0, nl, r0, nr;
  double cl, cr;
};
constexpr int kItemBatch = 512;

// entry k of a vector [e0, e0 + n), clamped into it; an empty vector reads
// entry 0 of the plan (the value is discarded by the caller)
__device__ __forceinline__ int64_t clamp_entry(int32_t e0, int32_t n, int k) {
  return n > 0 ? (int64_t)e0 + (k < n ? k : n - 1) : 0;
}

__global__ void __launch_bounds__(256) k_div_rows(DivArgs a, double *__restrict__ A) {
  __shared__ double row[kDivChunk];
  __shared__ DivItem its[kItemBatch];
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  const int64_t j = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * a.chunk;
  const int cw = (int)((a.ndof - c0) < a.chunk ? (a.ndof - c0) : a.chunk);
  for (int k = tid; k < cw; k += blockDim.x) row[k] = 0.0;
  const int32_t v = a.vert_of_dof[j];
  const int32_t p0 = a.vt_off[v];
  const int per = 3 * a.nq;
  const int items = (a.vt_off[v + 1] - p0) * per;
  const double *wq = a.qtab + 4 * a.nq;
  for (int i0 = 0; i0 < items; i0 += kItemBatch) {
    const int nb = (items - i0) < kItemBatch ? (items - i0) : kItemBatch;
    // phase A: one thread per item
    for (int k = tid; k < nb; k += blockDim.x) {
      const int it = i0 + k;
      const int pt = it / per, rem = it - pt * per;
      const int q = rem / 3, i = rem - 3 * q;
      const int64_t t = a.vt_tet[p0 + pt];
      const TetRec &R = a.rec[t];
      int jl = 0;
#pragma unroll
      for (int m = 1; m < 4; m++)
        if (R.dof[m] == (int32_t)j) jl = m;
      const double sigma = vslope(R, jl, i);
      const int64_t g = t * a.nq + q;
      const double wg = wq[q] * a.vol[t];
      double p, qc;
      if (a.pq) {
        p = a.pq[(int64_t)i * a.G + g];
        qc = a.pq[(int64_t)(3 + i) * a.G + g];
      } else {
        p = cos(gauss_coord(a, t, q, i));
        qc = 1.0 - p;
      }
      const int64_t hl = (int64_t)(2 * i) * a.G + g, hr = hl + a.G;
      const int64_t l0 = a.off[hl], l1 = a.off[hl + 1], r0 = a.off[hr], r1 = a.off[hr + 1];
      DivItem d;
      d.l0 = (int32_t)l0;
      d.nl = (int32_t)(l1 - l0);
      d.r0 = (int32_t)r0;
      d.nr = (int32_t)(r1 - r0);
      d.cl = -(wg * sigma * p);
      d.cr = wg * sigma * qc;
      its[k] = d;
    }
    __syncthreads();
    // phase B: a group of 16 lanes sweeps two items' four vectors, 16
    // consecutive entries of each per round (loads first, then the adds)
    for (int k = grp; k < nb; k += 32) {
      const DivItem P = its[k];
      DivItem Q = P;
      if (k + 16 < nb) {
        Q = its[k + 16];
      } else {
        Q.nl = 0;
        Q.nr = 0;
      }
      int nmax = P.nl > P.nr ? P.nl : P.nr;
      nmax = Q.nl > nmax ? Q.nl : nmax;
      nmax = Q.nr > nmax ? Q.nr : nmax;
      for (int b = 0; b < nmax; b += 16) {
        const int kk = b + gl;
        const int64_t e[4] = {clamp_entry(P.l0, P.nl, kk), clamp_entry(P.r0, P.nr, kk),
                              clamp_entry(Q.l0, Q.nl, kk), clamp_entry(Q.r0, Q.nr, kk)};
        int32_t d[4];
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          d[u] = a.ent_dof[e[u]];
          x[u] = a.ent_val[e[u]];
        }
        const int32_t n[4] = {P.nl, P.nr, Q.nl, Q.nr};
        const double cf[4] = {P.cl, P.cr, Q.cl, Q.cr};
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int64_t col = (int64_t)d[u] - c0;
          if (kk < n[u] && (uint64_t)col < (uint64_t)cw) atomicAdd(&row[col], cf[u] * x[u]);
        }
      }
    }
    __syncthreads();  // the batch's items are done before the next batch overwrites them
  }
  double *out = A + j * a.lda + c0;
  for (int k = tid; k < cw; k += blockDim.x) out[k] = row[k];
}

// Closed-form source of the exact solution u = (|x|^2 - r^2)^2 with
// p_i = cos x_i, q_i = 1 - cos x_i.  Along e_i the chord through x is
// |y_i| <= c, c^2 = r^2 - sum_{m != i} x_m^2, and in the distance s from
// either end u = s^4 - 4 c s^3 + 4 c^2 s^2, whose order-beta RL derivative
// from that end is Phi(s) = 24 s^{4-b}/G(5-b) - 24 c s^{3-b}/G(4-b)
// + 8 c^2 s^{2-b}/G(3-b); D_L u = Phi(x_i + c), D_R u = Phi(c - x_i) and
// f = sum_i [-sin x_i Phi(xi) + cos x_i Phi'(xi) - sin x_i Phi(eta)
//            + (1 - cos x_i) Phi'(eta)].
struct BallSrc {
  double r;
  double beta[3];
  double rg[3][4];  // 1/Gamma(k - beta_i), k = 2..5
};

__device__ __forceinline__ void chord_phi(double s, double c, double b, const double *rg, double &phi,
                                          double &dphi) {
  if (!(s > 0.0)) {
    phi = 0.0;
    dphi = 0.0;
    return;
  }
  const double s1 = pow(s, 1.0 - b), s2 = s1 * s, s3 = s2 * s, s4 = s3 * s;
  phi = 8.0 * c * c * rg[1] * s2 - 24.0 * c * rg[2] * s3 + 24.0 * rg[3] * s4;
  dphi = 8.0 * c * c * rg[0] * s1 - 24.0 * c * rg[1] * s2 + 24.0 * rg[2] * s3;
}

__device__ double ball_source(const double x[3], const BallSrc &b) {
  const double n2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
  double f = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const double c2 = b.r * b.r - (n2 - x[i] * x[i]);
    const double c = c2 > 0.0 ? sqrt(c2) : 0.0;
    double pl, dpl, pr, dpr;
    chord_phi(x[i] + c, c, b.beta[i], b.rg[i], pl, dpl);
    chord_phi(c - x[i], c, b.beta[i], b.rg[i], pr, dpr);
    const double sn = sin(x[i]), cs = cos(x[i]);
    f += -sn * pl + cs * dpl - sn * pr + (1.0 - cs) * dpr;
  }
  return f;
}

struct DivLoadArgs {
  const int32_t *vert_of_dof, *vt_off, *vt_tet, *tet;
  const double *xyz, *vol, *f_gauss, *qtab;
  int64_t ndof;
  int nq, src;
  BallSrc ball;
};

__global__ void k_div_load(DivLoadArgs a, double *__restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.ndof) return;
  const int32_t v = a.vert_of_dof[j];
  double sum = 0.0;
  for (int32_t p = a.vt_off[v]; p < a.vt_off[v + 1]; p++) {
    const int64_t t = a.vt_tet[p];
    int jl = 0;
    int32_t vv[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
      vv[m] = a.tet[4 * t + m];
      if (vv[m] == v) jl = m;
    }
    for (int q = 0; q < a.nq; q++) {
      double f = 1.0;
      if (a.src == FPDE_SRC_USER) {
        f = a.f_gauss[t * a.nq + q];
      } else if (a.src == FPDE_SRC_BALL_MMS) {
        double x[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < 4; m++) s = s + a.qtab[4 * q + m] * a.xyz[3 * (int64_t)vv[m] + d];
          x[d] = s;
        }
        f = ball_source(x, a.ball);
      }
      const double wg = a.qtab[4 * a.nq + q] * a.vol[t];
      sum += wg * f * a.qtab[4 * q + jl];
    }
  }
  b[j] = sum;
}

inline unsigned blocks_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int check_div(const fpde_mesh *m, const fpde_div_params *p) {
  if (!m || !p) return FPDE_EINVAL;
  for (int i = 0; i < 3; i++)
    if (!(p->beta[i] > 0.0 && p->beta[i] <= 1.0)) return FPDE_EALPHA;
  if (p->quad_points != 4 && p->quad_points != 11) return FPDE_EINVAL;
  if (p->coef != FPDE_COEF_SEC3 && p->coef != FPDE_COEF_USER) return FPDE_EINVAL;
  if (p->source != FPDE_SRC_ONE && p->source != FPDE_SRC_USER && p->source != FPDE_SRC_BALL_MMS)
    return FPDE_EINVAL;
  if (p->source == FPDE_SRC_BALL_MMS && !(p->radius > 0.0)) return FPDE_EINVAL;
  return FPDE_OK;
}

}  // namespace

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_div_assemble(fpde_mesh *m, const fpde_div_params *p, const double *pq, double *A, int64_t lda,
                                 double *b, const double *f_gauss, void *stream) {
  FPDE_TRY(check_div(m, p));
  if (!A || lda < m->ndof) return FPDE_EINVAL;
  if (p->coef == FPDE_COEF_USER && !pq) return FPDE_EINVAL;
  if (b && p->source == FPDE_SRC_USER && !f_gauss) return FPDE_EINVAL;
  if (m->ndof == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values_axes(m, P, p->beta, s));
  DivArgs a{};
  a.rec = m->rec;
  a.tet = m->tet;
  a.vt_off = m->vt_off;
  a.vt_tet = m->vt_tet;
  a.vert_of_dof = m->vert_of_dof;
  a.xyz = m->xyz;
  a.vol = m->vol;
  a.qtab = m->rules + rule_offset(p->quad_points);
  a.nq = p->quad_points;
  a.G = P->G;
  a.ndof = m->ndof;
  a.lda = lda;
  a.off = P->off;
  a.ent_dof = P->ent_dof;
  a.ent_val = P->ent_val;
  a.pq = p->coef == FPDE_COEF_USER ? pq : nullptr;
  a.chunk = (int)(m->ndof < kDivChunk ? m->ndof : kDivChunk);
  const unsigned nchunk = (unsigned)((m->ndof + a.chunk - 1) / a.chunk);
  const long t = timer_begin(m, s, FPDE_STAGE_DIV);
  k_div_rows<<<dim3((unsigned)m->ndof, nchunk), 256, 0, s>>>(a, A);
  timer_end(m, FPDE_STAGE_DIV, t, s);
  FPDE_HIP(hipGetLastError());
  if (b) {
    DivLoadArgs l{};
    l.vert_of_dof = m->vert_of_dof;
    l.vt_off = m->vt_off;
    l.vt_tet = m->vt_tet;
    l.tet = m->tet;
    l.xyz = m->xyz;
    l.vol = m->vol;
    l.f_gauss = f_gauss;
    l.qtab = a.qtab;
    l.ndof = m->ndof;
    l.nq = p->quad_points;
    l.src = p->source;
    l.ball.r = p->radius;
    for (int i = 0; i < 3; i++) {
      l.ball.beta[i] = p->beta[i];
      for (int k = 0; k < 4; k++) l.ball.rg[i][k] = 1.0 / std::tgamma((double)(k + 2) - p->beta[i]);
    }
    const long t2 = timer_begin(m, s, FPDE_STAGE_LOAD);
    k_div_load<<<blocks_of(m->ndof), 256, 0, s>>>(l, b);
    timer_end(m, FPDE_STAGE_LOAD, t2, s);
    FPDE_HIP(hipGetLastError());
  }
  const int f = take_flag(m, s);
  if (f != 0) {
    invalidate_values(P);
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}
