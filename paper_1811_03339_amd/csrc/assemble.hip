// Load vector, matrix-free product and adjoint sums (Sec. 2.1: K = sum_E K_E
// with element quadrature); the dense accumulation of K itself is in the
// tube pass (one block per group of parallel chords).
//
//   K_jk = sum_i K_i c_alpha sum_g w_g [R_gi(j) L_gi(k) + L_gi(j) R_gi(k)]
//
// The matrix-free product y = K x takes the dots of every half-ray vector
// with x and then, row by row, gathers W * value * (partner's dot) over the
// node -> entry transpose built once per mesh and rule.
#include <cmath>

#include "fpde_internal.h"

namespace fpde {

int walk_adjoint(fpde_mesh *m, Plan *P, double alpha, const double *u, const double *lam, hipStream_t s);

struct ContractArgs {
  const int64_t *row_off;
  const int4 *meta;       // per incidence: entry, partner offset, partner length << 2 | axis, partner
  const double *w;        // per incidence: Gauss weight w_g
  const double *wv;       // per incidence: w_g times its entry's value (matrix-free product)
  const int32_t *ent_dof;
  const double *ent_val;
  int64_t ndof, lda;
  int chunk;
  double KC0, KC1, KC2;   // K_i c_alpha
  __device__ __forceinline__ double KC(int i) const { return i == 0 ? KC0 : (i == 1 ? KC1 : KC2); }
};

struct LoadArgs {
  const int32_t *vert_of_dof, *vt_off, *vt_tet, *tet;
  const double *xyz, *vol, *f_gauss;
  int64_t ndof;
  int src;
  int nq;
  const double *qtab;  // device: nq x 4 barycentric coordinates, then nq weights
  double K[3], c_alpha, alpha, rg3, rg4, rg5;  // 1/Gamma(3-a), 1/Gamma(4-a), 1/Gamma(5-a)
};

__device__ inline double mms_phi(double s) { return s * s * (1.0 - s) * (1.0 - s); }
__device__ inline double mms_Phi(double s, const LoadArgs &a) {
  return 2.0 * pow(s, 2.0 - a.alpha) * a.rg3 - 12.0 * pow(s, 3.0 - a.alpha) * a.rg4 +
         24.0 * pow(s, 4.0 - a.alpha) * a.rg5;
}

// b_j = sum over elements E containing node j, points q: w_q |E| f(x_q) lambda_j(x_q).
// One wavefront per node: its lanes take the node's (element, point) pairs,
// then a butterfly sum in a fixed order (one node's few hundred terms would
// otherwise be a serial loop for a handful of workgroups).
__global__ void __launch_bounds__(256) k_load(LoadArgs a, double *__restrict__ b) {
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (j >= a.ndof) return;  // whole wavefronts
  const int32_t v = a.vert_of_dof[j];
  const int32_t p0 = a.vt_off[v];
  const int items = (a.vt_off[v + 1] - p0) * a.nq;
  double sum = 0.0;
  for (int k = lane; k < items; k += 64) {
    const int pi = k / a.nq, q = k - pi * a.nq;
    const int64_t t = a.vt_tet[p0 + pi];
    int jl = 0;
    int32_t vv[4];
    for (int m = 0; m < 4; m++) {
      vv[m] = a.tet[4 * t + m];
      if (vv[m] == v) jl = m;
    }
    double f = 1.0;
    if (a.src == FPDE_SRC_USER) {
      f = a.f_gauss[t * a.nq + q];
    } else if (a.src == FPDE_SRC_CUBE_MMS) {
      double x[3];
      for (int d = 0; d < 3; d++) {
        double s = 0.0;
        for (int m = 0; m < 4; m++) s = s + a.qtab[4 * q + m] * a.xyz[3 * (int64_t)vv[m] + d];
        x[d] = s;
      }
      const double ph[3] = {mms_phi(x[0]), mms_phi(x[1]), mms_phi(x[2])};
      f = 0.0;
      for (int i = 0; i < 3; i++) {
        double other = 1.0;
        for (int d = 0; d < 3; d++)
          if (d != i) other *= ph[d];
        f += a.K[i] * a.c_alpha * (mms_Phi(x[i], a) + mms_Phi(1.0 - x[i], a)) * other;
      }
    }
    const double wg = a.qtab[4 * a.nq + q] * a.vol[t];
    sum += wg * f * a.qtab[4 * q + jl];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) b[j] = sum;
}

// d[h] = sum over entries of half-ray h of value * x[dof]; 16 lanes per
// half-ray, so a load instruction reads 16 consecutive entries of each of
// four half-rays
__global__ void __launch_bounds__(256) k_ray_dot(const int64_t *__restrict__ off, const int32_t *__restrict__ dof,
                                                 const double *__restrict__ val, const double *__restrict__ x,
                                                 int64_t n_half, double *__restrict__ d) {
  const int gl = threadIdx.x & 15;
  const int64_t h = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (h >= n_half) return;  // the whole group of 16 shares h
  double s = 0.0;
  for (int64_t e = off[h] + gl; e < off[h + 1]; e += 16) s = fma(val[e], x[dof[e]], s);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
  if (gl == 0) d[h] = s;
}

// wv[p] = w_g value_e for incidence p (entry e = meta[p].x): the entry
// values in the node -> entry order, so the product streams them
__global__ void k_inc_wv(const int4 *__restrict__ meta, const double *__restrict__ w,
                         const double *__restrict__ ent_val, int64_t n, double *__restrict__ wv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) wv[p] = w[p] * ent_val[meta[p].x];
}

// y_j = sum over entries e on node j of W(h_e) value_e d[partner(h_e)];
// one wavefront per row, lanes stride over the row's entries
__global__ void __launch_bounds__(256) k_apply_rows(ContractArgs c, const double *__restrict__ d,
                                                    double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= c.ndof) return;
  double s = 0.0;
  for (int64_t p = c.row_off[j] + lane; p < c.row_off[j + 1]; p += 64) {
    const int4 mt = c.meta[p];
    s += c.wv[p] * c.KC(mt.z & 3) * d[mt.w];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[j] = s;
}

// Per-block partial sums of S_i, T_i (6 values) over Gauss points.
__global__ void __launch_bounds__(256) k_adjoint_partial(const double *__restrict__ adj, const double *__restrict__ vol,
                                                         int64_t G, int nq, const double *__restrict__ wq,
                                                         double *__restrict__ part) {
  __shared__ double red[6][256];
  const int tid = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + tid; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const double wg = wq[g % nq] * vol[g / nq];
    for (int i = 0; i < 3; i++) {
      const double *L = adj + 4 * ((int64_t)(2 * i) * G + g);
      const double *R = adj + 4 * ((int64_t)(2 * i + 1) * G + g);
      // [0] value.u  [1] value.lam  [2] d/da value.u  [3] d/da value.lam
      acc[i] += wg * (R[1] * L[0] + L[1] * R[0]);
      acc[3 + i] += wg * (R[3] * L[0] + R[1] * L[2] + L[3] * R[0] + L[1] * R[2]);
    }
  }
  for (int k = 0; k < 6; k++) red[k][tid] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < 6; k++) red[k][tid] += red[k][tid + w];
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < 6; k++) part[6 * blockIdx.x + k] = red[k][0];
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static ContractArgs contract_args(fpde_mesh *m, const Plan &P, const fpde_params *p, int64_t lda) {
  Order o = order_scalars(p->alpha);
  ContractArgs c{};
  c.row_off = P.row_off;
  c.meta = P.inc_meta;
  c.w = P.inc_w;
  c.ent_dof = P.ent_dof;
  c.ent_val = P.ent_val;
  c.ndof = m->ndof;
  c.lda = lda;
  c.chunk = (int)(m->ndof < 8192 ? (m->ndof > 0 ? m->ndof : 1) : 8192);
  c.KC0 = p->K[0] * o.c_alpha;
  c.KC1 = p->K[1] * o.c_alpha;
  c.KC2 = p->K[2] * o.c_alpha;
  return c;
}

int launch_load(fpde_mesh *m, const fpde_params *p, double *b, const double *f_gauss, hipStream_t s) {
  if (m->ndof == 0) return FPDE_OK;
  LoadArgs a{};
  a.vert_of_dof = m->vert_of_dof;
  a.vt_off = m->vt_off;
  a.vt_tet = m->vt_tet;
  a.tet = m->tet;
  a.xyz = m->xyz;
  a.vol = m->vol;
  a.f_gauss = f_gauss;
  a.ndof = m->ndof;
  a.src = p->source;
  a.nq = p->quad_points;
  a.qtab = m->rules + rule_offset(a.nq);
  Order o = order_scalars(p->alpha);
  for (int i = 0; i < 3; i++) a.K[i] = p->K[i];
  a.c_alpha = o.c_alpha;
  a.alpha = p->alpha;
  a.rg3 = 1.0 / std::tgamma(3.0 - p->alpha);
  a.rg4 = 1.0 / std::tgamma(4.0 - p->alpha);
  a.rg5 = 1.0 / std::tgamma(5.0 - p->alpha);
  const long t = timer_begin(m, s, FPDE_STAGE_LOAD);
  k_load<<<nblk(m->ndof * 64), 256, 0, s>>>(a, b);
  timer_end(m, FPDE_STAGE_LOAD, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

// y = K x from the stored derivative vectors (plan + values for p->alpha)
int apply_matfree(fpde_mesh *m, Plan *P, const fpde_params *p, const double *x, double *y, double *dscratch,
                  hipStream_t s) {
  // the merged entries of the mixed-precision plan, when they hold these values
  if (m->ndof > 0 && merged_apply_ready(*P)) return apply_merged(m, *P, p, x, y, s);
  if (!P->inc_wv) FPDE_TRY(dalloc(&P->inc_wv, P->n_ent > 0 ? P->n_ent : 1));
  ContractArgs c = contract_args(m, *P, p, 0);
  c.wv = P->inc_wv;
  const long t = timer_begin(m, s, FPDE_STAGE_APPLY);
  if (P->inc_wv_version != P->values_version) {
    if (P->n_ent > 0) k_inc_wv<<<nblk(P->n_ent), 256, 0, s>>>(P->inc_meta, P->inc_w, P->ent_val, P->n_ent, P->inc_wv);
    P->inc_wv_version = P->values_version;
  }
  k_ray_dot<<<nblk(16 * P->n_half), 256, 0, s>>>(P->off, P->ent_dof, P->ent_val, x, P->n_half, dscratch);
  k_apply_rows<<<nblk(m->ndof, 4), 256, 0, s>>>(c, dscratch, y);
  timer_end(m, FPDE_STAGE_APPLY, t, s);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

int apply_scratch(fpde_mesh *m, Plan *P, double **d) {
  // the adjoint buffer (4 per half-ray) doubles as the per-half-ray dot scratch
  if (!P->adj) FPDE_TRY(dalloc(&P->adj, 4 * P->n_half));
  *d = P->adj;
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_assemble(fpde_mesh *m, const fpde_params *p, void *A, int64_t lda, double *b,
                             const double *f_gauss, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!A || lda < m->ndof) return FPDE_EINVAL;
  if (p->source == FPDE_SRC_USER && !f_gauss && b) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values(m, P, p->alpha, s));
  FPDE_TRY(launch_contract_tubes(m, *P, p, A, lda, s));
  if (b) FPDE_TRY(launch_load(m, p, b, f_gauss, s));
  int f = take_flag(m, s);
  if (f != 0) {
    invalidate_values(P);
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}

extern "C" int fpde_assemble_batch(fpde_mesh *m, int count, const fpde_params *p, void *A, int64_t lda,
                                   int64_t stride_A, double *b, int64_t stride_b, void *stream) {
  if (!m || !p || count < 1 || count > 16 || !A || lda < m->ndof) return FPDE_EINVAL;
  for (int z = 0; z < count; z++) {
    FPDE_TRY(check_params(m, &p[z]));
    if (p[z].source == FPDE_SRC_USER || p[z].precision != p[0].precision) return FPDE_EINVAL;
  }
  if (count > 1 && (stride_A < m->ndof * lda || (b && stride_b < m->ndof))) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  const size_t elem = p[0].precision == FPDE_MIXED ? sizeof(float) : sizeof(double);
  Plan *used[16] = {};
  for (int z = 0; z < count; z++) FPDE_TRY(plan_for(m, p[z].quad_points, p[z].max_steps, s, &used[z]));
  // The walks run on a second stream: the walk of a system overlaps the
  // accumulation of the previous one when that one belongs to the other
  // rule (another plan, another value buffer).  Systems are taken with the
  // rules alternating; a walk waits for the caller's earlier work and for
  // the last accumulation that read its plan's values, an accumulation for
  // its walk (events; the values are re-walked only when the orders
  // changed, as in fpde_assemble).
  if (!m->side && hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess) m->side = nullptr;
  for (int k = 0; k < 2 * count + 1 && m->side; k++)
    if (!m->bev[k] && hipEventCreateWithFlags(&m->bev[k], hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess) return FPDE_EHIP;
  int order[16], no = 0;
  {
    int q4[16], q11[16], n4 = 0, n11 = 0;
    for (int z = 0; z < count; z++) (used[z] == used[0] ? q4[n4++] : q11[n11++]) = z;
    for (int k = 0; k < n4 || k < n11; k++) {
      if (k < n4) order[no++] = q4[k];
      if (k < n11) order[no++] = q11[k];
    }
  }
  hipStream_t w = m->side ? m->side : s;
  if (m->side) {
    FPDE_HIP(hipEventRecord(m->bev[2 * count], s));
    FPDE_HIP(hipStreamWaitEvent(w, m->bev[2 * count], 0));
  }
  int last_acc[2] = {-1, -1};  // per plan: the last system whose accumulation was enqueued
  for (int k = 0; k < count; k++) {
    const int z = order[k];
    Plan *P = used[z];
    const int pl = P == used[0] ? 0 : 1;
    if (m->side && last_acc[pl] >= 0) FPDE_HIP(hipStreamWaitEvent(w, m->bev[2 * last_acc[pl] + 1], 0));
    FPDE_TRY(ensure_values(m, P, p[z].alpha, w));
    if (m->side) {
      FPDE_HIP(hipEventRecord(m->bev[2 * z], w));
      FPDE_HIP(hipStreamWaitEvent(s, m->bev[2 * z], 0));
    }
    FPDE_TRY(launch_contract_tubes(m, *P, &p[z], (char *)A + (size_t)z * (size_t)stride_A * elem, lda, s));
    if (b) FPDE_TRY(launch_load(m, &p[z], b + (size_t)z * (size_t)stride_b, nullptr, s));
    if (m->side) FPDE_HIP(hipEventRecord(m->bev[2 * z + 1], s));
    last_acc[pl] = z;
  }
  int f = take_flag(m, s);  // every walk is ordered before an accumulation on s
  if (f != 0) {
    for (int z = 0; z < count; z++) invalidate_values(used[z]);
    return f < 0 ? f : FPDE_EHIP;
  }
  return FPDE_OK;
}

extern "C" int fpde_apply(fpde_mesh *m, const fpde_params *p, const double *x, double *y, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!x || !y) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(ensure_values(m, P, p->alpha, s));
  double *d = nullptr;
  FPDE_TRY(apply_scratch(m, P, &d));
  FPDE_TRY(apply_matfree(m, P, p, x, y, d, s));
  int f = take_flag(m, s);
  return f < 0 ? f : (f > 0 ? FPDE_EHIP : FPDE_OK);
}

extern "C" int fpde_adjoint(fpde_mesh *m, const fpde_params *p, const double *u, const double *lam,
                            double *grad_alpha, double *grad_K, void *stream) {
  FPDE_TRY(check_params(m, p));
  if (!u || !lam || !grad_alpha || !grad_K) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  Plan *P = nullptr;
  FPDE_TRY(plan_for(m, p->quad_points, p->max_steps, s, &P));
  FPDE_TRY(walk_adjoint(m, P, p->alpha, u, lam, s));
  const unsigned nb = 512;
  double *part = nullptr;
  FPDE_TRY(dalloc(&part, 6 * nb));
  k_adjoint_partial<<<nb, 256, 0, s>>>(P->adj, m->vol, P->G, P->nq,
                                       m->rules + rule_offset(P->nq) + 4 * P->nq, part);
  double h[6 * 512];
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpyAsync(h, part, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, s);
  int f = (e1 == hipSuccess && e2 == hipSuccess) ? take_flag(m, s) : FPDE_EHIP;
  dfree(part);
  if (f != 0) return f < 0 ? f : FPDE_EHIP;
  double S_[3] = {0, 0, 0}, T_[3] = {0, 0, 0};
  for (unsigned b = 0; b < nb; b++)
    for (int i = 0; i < 3; i++) {
      S_[i] += h[6 * b + i];
      T_[i] += h[6 * b + 3 + i];
    }
  Order o = order_scalars(p->alpha);
  double ga = 0.0;
  for (int i = 0; i < 3; i++) {
    grad_K[i] = -o.c_alpha * S_[i];
    ga -= p->K[i] * (o.dc_alpha * S_[i] + o.c_alpha * T_[i]);
  }
  *grad_alpha = ga;
  return FPDE_OK;
}
