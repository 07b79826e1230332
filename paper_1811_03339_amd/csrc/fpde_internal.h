// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <vector>

#include "fpde.h"

namespace fpde {

// One element as the walk reads it: a single 128-byte record (one cache line
// of the MI355X L2), so each step of the pointer-chasing walk costs one line.
//   M[9]   : A^{-1} row-major, row r = gradient of volume coordinate k_{r+1}
//            (Sec. 2.2: k = A^{-1}(x - v0), A = (v1-v0, v2-v0, v3-v0))
//   v0[3]  : vertex 0
//   nbr[4] : element across face f (opposite local vertex f), -1 = boundary
//   dof[4] : unknown index of local vertex f, -1 on the boundary
struct alignas(128) TetRec {
  double M[9];
  double v0[3];
  int32_t nbr[4];
  int32_t dof[4];
};
static_assert(sizeof(TetRec) == 128, "element record must be one 128-byte line");

// Element quadrature rule in barycentric coordinates, weights summing to 1.
struct QuadRule {
  int nq;
  double bary[11][4];
  double w[11];
};
int quad_rule(int nq, QuadRule *out);  // FPDE_OK or FPDE_EINVAL
// offset of the nq-point table inside fpde_mesh::rules
inline int rule_offset(int nq) { return nq == 4 ? 0 : 4 * 5; }

// Tubes of the accumulation: pairs (g, i) grouped by axis i and the cell of
// x_g in the plane orthogonal to e_i; U_T = the tube's nodes (sorted).
struct TubePlan {
  double cell = 0.0;              // cell edge
  int64_t n_tubes = 0, n_u = 0, n_items = 0, blk_n = 0, max_u = 0;
  int32_t *pair_sorted = nullptr; // 3 G pair ids i * G + g, tube by tube
  int4 *pm = nullptr;             // per sorted pair {l first entry, r first entry, |l|, |r| | axis << 30}
  double *pw = nullptr;           // per sorted pair: w_g
  int64_t *tube_off = nullptr;    // n_tubes + 1 into the sorted pairs
  int64_t *u_off = nullptr;       // n_tubes + 1 into tube_u
  int32_t *tube_u = nullptr;      // n_u: U_T, increasing
  int32_t *ent_slot = nullptr;    // n_ent: position of the entry's node in its tube's U_T
  int64_t *row_off = nullptr;     // n_dof + 1 into row_ts
  int2 *row_ts = nullptr;         // n_u: (tube, slot) places of each node, grouped by node
  int4 *items = nullptr;          // pass-1 work: {tube, first block row, rows, |U_T|}
  int64_t *blk_off = nullptr;     // n_tubes + 1: offsets (doubles) of the |U_T|^2 blocks
  double *blk = nullptr;          // blk_n doubles of block scratch, allocated on first use
  int32_t *cstart = nullptr;      // row pass: per tube, the first U_T position of every column chunk
  int cs_chunk = 0;               // the chunk width cstart was built for
  // the matrix-core contraction (mixed precision): work items {tube, region
  // row, region column, |U_T|} over the upper 128 x 128 regions of every
  // block, and per tube the largest binary exponents of its two operands;
  // the merged entries (one per node and side of a pair, in sorted-pair
  // order): first merged entry of every pair, per merged entry its tube
  // slot | (inner column << 16) (column 2 (pair mod 16) + side) and its
  // value in FP32 (rebuilt at every assembly), per plan entry its merged
  // index within its pair, and per sorted pair its tube
  bool mfma_planned = false, mfma_ok = false;
  int4 *mitems = nullptr;
  int64_t n_mitems = 0, n_mk = 0;
  int2 *texp = nullptr;
  int64_t *mk_pair = nullptr;
  uint32_t *mk_meta = nullptr;
  float *mk_val = nullptr;
  uint16_t *mg_idx = nullptr;
  int32_t *pk_tube = nullptr;
  // the FP64 matrix-free product on the merged entries: per merged entry
  // its node, FP64 value and position in node order (mpos); per node its
  // merged entries (mrow_off; ascending merged index), per such incidence
  // the partner's dot index | axis << 30 and w_g v; the per-pair-side
  // dots.  The values are rebuilt at every assembly (version mk_version of
  // the plan's values); mg_pair and mrow_q serve the plan only.
  bool mapply_ok = false;
  int32_t *mg_node = nullptr, *mg_pair = nullptr, *mrow_q = nullptr, *mpos = nullptr;
  int64_t *mrow_off = nullptr;
  uint32_t *mpart = nullptr;
  double *mk_val64 = nullptr, *mwv = nullptr, *mdp = nullptr;
  int64_t mk_version = -1;
};

// Symbolic phase of one rule: derivative-vector sizes and the row transpose.
// Half-ray index (direction-major): h = dir * G + g, dir = 2 i + side.
struct Plan {
  int nq = 0;
  int max_steps = 0;
  int64_t G = 0;          // Gauss points
  int64_t n_half = 0;     // 6 G half-rays
  int64_t n_ent = 0;      // entries over all half-rays
  int64_t *off = nullptr;     // n_half + 1: entries of half-ray h
  int32_t *ent_dof = nullptr; // n_ent
  int32_t *ent_ray = nullptr; // n_ent: owning half-ray
  double *ent_val = nullptr;  // n_ent: values, half-rays along e_i at order val_gamma[i]
  double val_gamma[3] = {-1.0, -1.0, -1.0};  // per axis; -1 = not computed
  double *ent_val2 = nullptr;  // n_ent: a second set of values (allocated on first use)
  double val_gamma2[3] = {-1.0, -1.0, -1.0};
  int64_t *row_off = nullptr; // n_dof + 1
  int64_t *inc = nullptr;     // n_ent: entry ids grouped by their dof
  // per incidence (row order): {entry id, partner offset, partner length << 2 | axis,
  // partner half-ray} and the quadrature weight w_g of its Gauss point
  int4 *inc_meta = nullptr;
  double *inc_w = nullptr;
  // per incidence: w_g times its entry's value (first value set), built by
  // the matrix-free product when the values changed since (versions)
  double *inc_wv = nullptr;
  int64_t values_version = 0, inc_wv_version = -1;
  double *adj = nullptr;      // 4 n_half scratch for the adjoint dots
  int64_t pairs = 0;          // sum over (g, i) of |L| |R|
  int64_t max_ent = 0;        // largest entry count of one half-ray
  TubePlan tubes;
};

// HIP events around stage launches on the caller's stream (fpde_timing).
struct StageTimer {
  bool on = false;
  unsigned mask = ~0u;  // stages recorded while on (bit 1 << stage)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Mark {
    int stage;
    size_t a, b;
    int weight;  // units the interval covers (systems of a batch)
  };
  std::vector<Mark> marks;
};

}  // namespace fpde

struct fpde_mesh {
  int device = 0;
  int64_t nv = 0, nt = 0, ndof = 0, nbf = 0;
  double *xyz = nullptr;          // nv*3
  int32_t *tet = nullptr;         // nt*4
  fpde::TetRec *rec = nullptr;    // nt
  double *vol = nullptr;          // nt
  int32_t *vt_off = nullptr;      // nv+1
  int32_t *vt_tet = nullptr;      // 4 nt
  int32_t *dof = nullptr;         // nv
  int32_t *vert_of_dof = nullptr; // ndof
  double *rules = nullptr;        // device quadrature tables: [4-point | 11-point],
                                  // each nq*4 barycentric coordinates then nq weights
  double *pbox = nullptr;         // ndof x 6: box of each node's element patch (lo xyz, hi xyz)
  int32_t *flag = nullptr;        // device status word (0 = ok)
  int64_t *flag_aux = nullptr;    // device: failing column / ray
  int64_t *flag_blk = nullptr;    // device block holding both: {flag (low word), flag_aux}
  int64_t *hflag = nullptr;       // pinned host copy of flag_blk (one transfer per status check)
  fpde::Plan plan[2];             // rules with 4 and 11 points
  // solve scratch
  double *vec = nullptr;          // 4 ndof FP64
  double *red = nullptr;          // reduction scratch
  int64_t red_n = 0;
  void *linv = nullptr;           // inverses of the factor's 64 x 64 diagonal blocks (+ transposes)
  size_t linv_bytes = 0;
  double *cg = nullptr;           // conjugate-gradient vectors and partial sums
  int64_t cg_n = 0;
  int *tsync = nullptr;           // triangular solves: per-system block flags (2 nblk) and tickets (2)
  int tsync_n = 0;                // ints allocated
  int64_t *batch_aux = nullptr;   // device, kMaxBatch: failing column per system of a batched factorization
  int *escale = nullptr;          // device: per-row exponents of the split-FP16 trailing updates
  _Float16 *xsplit = nullptr;     // device: the split rows (hi, lo) of X for those updates
  int64_t escale_n = 0, xsplit_n = 0;  // entries allocated in escale, xsplit
  double *bvec = nullptr;         // device: intermediate vectors of a batched solve
  int64_t bvec_n = 0;
  int tsync_epoch = 0;
  fpde::StageTimer timer;
  // batched assembly: a second stream for the walks and events ordering it
  // against the caller's stream (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t bev[33] = {};
  hipEvent_t lev[2] = {};  // factorization look-ahead: split rows ready, side update done
};

namespace fpde {

#define FPDE_HIP(call)                        \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return FPDE_EHIP;   \
  } while (0)

#define FPDE_TRY(call)             \
  do {                             \
    int s_ = (call);               \
    if (s_ != FPDE_OK) return s_;  \
  } while (0)

template <class T>
int dalloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return FPDE_ENOMEM;
  }
  return FPDE_OK;
}
template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

inline hipStream_t S(void *s) { return (hipStream_t)s; }

// Device status word: keeps the first error reported by any thread.
__device__ inline void set_flag(int32_t *flag, int code) { atomicCAS(flag, 0, code); }

// Reads (and clears) the device status word; synchronises the stream.
int take_flag(fpde_mesh *m, hipStream_t s, int64_t *aux = nullptr);

int plan_for(fpde_mesh *m, int nq, int max_steps, hipStream_t s, Plan **out);
// entry values at order gamma = alpha/2 on every axis
int ensure_values(fpde_mesh *m, Plan *P, double alpha, hipStream_t s);
// entry values at order gamma[i] along e_i (recomputes only the axes that
// changed); slot 0 = ent_val, slot 1 = ent_val2
int ensure_values_axes(fpde_mesh *m, Plan *P, const double gamma[3], hipStream_t s, int slot = 0);
inline void invalidate_values(Plan *P) {
  for (int i = 0; i < 3; i++) P->val_gamma[i] = P->val_gamma2[i] = -1.0;
}
int check_params(const fpde_mesh *m, const fpde_params *p);
void free_plan(Plan &P);
// tube plan of a rule whose entries exist (cell edge = kappa x mean element edge)
int build_tubes(fpde_mesh *m, Plan &P, double kappa, hipStream_t s);
void free_tubes(TubePlan &tp);
int launch_contract_tubes(fpde_mesh *m, Plan &P, const fpde_params *p, void *A, int64_t lda, hipStream_t s);
// the same sums kept at the columns of a CSR pattern (FP64)
// general form with constant coefficients from the plan's two value sets
int launch_form_tubes(fpde_mesh *m, Plan &P, const double cl[3], const double cr[3], double *A, int64_t lda,
                      hipStream_t s);
int launch_contract_tubes_csr(fpde_mesh *m, Plan &P, const fpde_params *p, const int64_t *row_ptr,
                              const int32_t *col, double *val, hipStream_t s);
// matrix-free y = K x and its scratch (assemble.hip)
// y = K x on the merged entries of the mixed-precision tube plan, when they
// hold the plan's current values (merged_apply_ready); FPDE_OK or an error.
bool merged_apply_ready(const Plan &P);
int apply_merged(fpde_mesh *m, Plan &P, const fpde_params *p, const double *x, double *y, hipStream_t s);
int apply_matfree(fpde_mesh *m, Plan *P, const fpde_params *p, const double *x, double *y, double *dscratch,
                  hipStream_t s);
int apply_scratch(fpde_mesh *m, Plan *P, double **d);
// load vector b for the Riesz problem (assemble.hip)
int launch_load(fpde_mesh *m, const fpde_params *p, double *b, const double *f_gauss, hipStream_t s);
// dense SPD solve with a workspace handle (solve.hip); a workspace handle
// holding only flags, timers and solve scratch for n unknowns (mesh.hip)
int dense_spd_solve(fpde_mesh *ws, double *A, int64_t lda, int64_t n, const double *b, double *u,
                    int64_t *failed, hipStream_t s);
int workspace_new(int64_t ndof, fpde_mesh **out);
// patch boxes of the template (built once per mesh)
int ensure_patch_boxes(fpde_mesh *m, hipStream_t s);

// Stage timing: t = timer_begin(m, s, stage); ...launches...;
// timer_end(m, stage, t, s).  Records nothing (t = -1) unless timing is on
// for that stage.
long timer_begin(fpde_mesh *m, hipStream_t s, int stage);
void timer_end(fpde_mesh *m, int stage, long t, hipStream_t s, int weight = 1);

// host-side order scalars
struct Order {
  double gamma, e;        // gamma = alpha/2, e = 1 - gamma
  double inv_g2;          // 1/Gamma(2-gamma)
  double half_psi0;       // psi(2-gamma)/2
  double c_alpha, dc_alpha;
};
Order order_scalars(double alpha);
// the same scalars for a one-sided order gamma in (0, 1] (alpha = 2 gamma)
inline Order gamma_scalars(double gamma) { return order_scalars(2.0 * gamma); }

}  // namespace fpde
