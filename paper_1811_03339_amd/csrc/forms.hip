// The general uniform form of Sec. 1 (eq. equ:varsss), the test operator
// on the side opposite to the trial one, with the element quadrature of
// Sec. 2.1:
//
//   K_kl = sum_i sum_g w_g [cl_i(x_g) D_L^{a_i} psi_l(x_g) D_R^{b_i} psi_k(x_g)
//                         + cr_i(x_g) D_R^{a_i} psi_l(x_g) D_L^{b_i} psi_k(x_g)],
//
// trial orders a_i and test orders b_i in [0, 1] (order 0 is the identity,
// order 1 the classical derivative, D_R^1 = -d/dx), row k = test function.
// The Riesz split (a = b, cl = cr = K_i c_alpha) and the problem of Sec. 3
// (b = 1, cl = p_i, cr = q_i) are instances.
//
// The walk evaluates every half-ray twice: at the trial orders into the
// plan's first value set and at the test orders into its second.  With
// constant coefficients the products are accumulated by tubes (the two
// products of every pair into a tube block, then the row pass of the
// Riesz matrix); with coefficients per Gauss point, row k
// then collects, over the incidences of node k (entry e of half-ray h in the
// plan's node -> entry transpose, partner half-ray h' on the other side of
// the same (g, i)), the partner's trial vector scaled by w_g c val_b(e), with
// c = cl_i when h is a right half-ray (its test operator is D_R) and cr_i when
// it is a left one:
//   k_form_rows  one workgroup per (row, column chunk): the row chunk lives in
//                LDS; the incidences are set up one per thread into LDS, then
//                groups of 16 lanes sweep 16 consecutive entries of a partner
//                vector per load and add them with LDS atomics; the chunk is
//                written to K once.
#include <cmath>

#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kFormChunk = 8192;  // doubles of one row chunk in LDS (64 KB)
constexpr int kIncBatch = 512;

struct FormArgs {
  const int64_t *row_off;  // node -> incidences
  const int4 *meta;        // per incidence: entry, partner offset, partner length << 2 | axis, partner
  const double *w;         // per incidence: w_g
  const int32_t *ent_dof;
  const double *val_a;     // trial orders
  const double *val_b;     // test orders
  const double *coef;      // FPDE_COEF_USER: cl_i at [i G + g], cr_i at [(3 + i) G + g]; else null
  double cl[3], cr[3];     // constant coefficients
  int64_t G, ndof, lda;
  int chunk;
};

struct Inc {
  int32_t p0, n;  // partner vector: first entry, length
  double c;       // scale of the partner's trial values
};

__device__ __forceinline__ int64_t clamp_entry(int32_t e0, int32_t n, int k) {
  return n > 0 ? (int64_t)e0 + (k < n ? k : n - 1) : 0;
}

__global__ void __launch_bounds__(256) k_form_rows(FormArgs a, double *__restrict__ A) {
  __shared__ double row[kFormChunk];
  __shared__ Inc its[kIncBatch];
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  const int64_t k = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * a.chunk;
  const int cw = (int)((a.ndof - c0) < a.chunk ? (a.ndof - c0) : a.chunk);
  for (int q = tid; q < cw; q += blockDim.x) row[q] = 0.0;
  const int64_t q0 = a.row_off[k], nin = a.row_off[k + 1] - q0;
  for (int64_t i0 = 0; i0 < nin; i0 += kIncBatch) {
    const int nb = (int)((nin - i0) < kIncBatch ? (nin - i0) : kIncBatch);
    for (int t = tid; t < nb; t += blockDim.x) {
      const int64_t p = q0 + i0 + t;
      const int4 mt = a.meta[p];
      const int ax = mt.z & 3;
      const int64_t hp = mt.w;                  // partner half-ray
      const int dirp = (int)(hp / a.G);
      const int64_t g = hp - (int64_t)dirp * a.G;
      const bool test_right = (dirp & 1) == 0;  // partner is a left half-ray
      double c;
      if (a.coef) {
        c = a.coef[(int64_t)(test_right ? ax : 3 + ax) * a.G + g];
      } else {
        c = test_right ? (ax == 0 ? a.cl[0] : (ax == 1 ? a.cl[1] : a.cl[2]))
                       : (ax == 0 ? a.cr[0] : (ax == 1 ? a.cr[1] : a.cr[2]));
      }
      Inc d;
      d.p0 = mt.y;
      d.n = mt.z >> 2;
      d.c = a.w[p] * c * a.val_b[mt.x];
      its[t] = d;
    }
    __syncthreads();
    for (int t = grp; t < nb; t += 32) {
      const Inc P = its[t];
      Inc Q = P;
      if (t + 16 < nb) Q = its[t + 16];
      else Q.n = 0;
      const int nmax = P.n > Q.n ? P.n : Q.n;
      for (int b = 0; b < nmax; b += 16) {
        const int kk = b + gl;
        const int64_t ep = clamp_entry(P.p0, P.n, kk), eq = clamp_entry(Q.p0, Q.n, kk);
        const int32_t dp = a.ent_dof[ep], dq = a.ent_dof[eq];
        const double vp = a.val_a[ep], vq = a.val_a[eq];
        const int64_t cp = (int64_t)dp - c0, cq = (int64_t)dq - c0;
        if (kk < P.n && (uint64_t)cp < (uint64_t)cw) atomicAdd(&row[cp], P.c * vp);
        if (kk < Q.n && (uint64_t)cq < (uint64_t)cw) atomicAdd(&row[cq], Q.c * vq);
      }
    }
    __syncthreads();  // the batch is done before the next one overwrites it
  }
  __syncthreads();
  double *out = A + k * a.lda + c0;
  for (int q = tid; q < cw; q += blockDim.x) out[q] = row[q];
}

int check_form(const fpde_mesh *m, const fpde_form_params *p) {
  if (!m || !p) return FPDE_EINVAL;
  for (int i = 0; i < 3; i++) {
    if (!(p->alpha[i] >= 0.0 && p->alpha[i] <= 1.0)) return FPDE_EALPHA;
    if (!(p->beta[i] >= 0.0 && p->beta[i] <= 1.0)) return FPDE_EALPHA;
    if (!std::isfinite(p->cl[i]) || !std::isfinite(p->cr[i])) return FPDE_EINVAL;
  }
  if (p->quad_points != 4 && p->quad_points != 11) return FPDE_EINVAL;
  if (p->coef != FPDE_COEF_CONST && p->coef != FPDE_COEF_USER) return FPDE_EINVAL;
  return FPDE_OK;
}

}  // namespace

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_form_assemble(fpde_mesh *m, const fpde_form_params *p, const double *coef, double *A,
                                  int64_t lda, void *stream) {
  FPDE_TRY(check_form(m, p));
  if (!A || lda < m->ndof) return FPDE_EINVAL;
  if (p->coef == FPDE_COEF_USER && !coef) return FPDE_EINVAL;
  if (m->ndof == 0) return FPDE_OK;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values_axes(m, P, p->alpha, s, 0));
  FPDE_TRY(ensure_values_axes(m, P, p->beta, s, 1));
  FormArgs a{};
  a.row_off = P->row_off;
  a.meta = P->inc_meta;
  a.w = P->inc_w;
  a.ent_dof = P->ent_dof;
  a.val_a = P->ent_val;
  a.val_b = P->ent_val2;
  a.coef = p->coef == FPDE_COEF_USER ? coef : nullptr;
  for (int i = 0; i < 3; i++) {
    a.cl[i] = p->cl[i];
    a.cr[i] = p->cr[i];
  }
  a.G = P->G;
  a.ndof = m->ndof;
  a.lda = lda;
  a.chunk = (int)(m->ndof < kFormChunk ? m->ndof : kFormChunk);
  const unsigned nchunk = (unsigned)((m->ndof + a.chunk - 1) / a.chunk);
  const long t = timer_begin(m, s, FPDE_STAGE_FORM);
  if (p->coef == FPDE_COEF_CONST) {
    // constant coefficients: the pairs' products by tubes, then the row pass
    FPDE_TRY(launch_form_tubes(m, *P, p->cl, p->cr, A, lda, s));
  } else {
    k_form_rows<<<dim3((unsigned)m->ndof, nchunk), 256, 0, s>>>(a, A);
  }
  timer_end(m, FPDE_STAGE_FORM, t, s);
  FPDE_HIP(hipGetLastError());
  const int f = take_flag(m, s);
  if (f != 0) {
    invalidate_values(P);
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}
