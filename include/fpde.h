/*
 * fpde.h - C ABI of the MI355X (gfx950) library for the P1 finite-element
 * discretisation of steady Riesz fractional diffusion on convex tetrahedral
 * meshes (Yang, Nie, Yuan & Wang, "Finite Element Methods for Fractional
 * PDEs in Three Dimensions").
 *
 * Problem: -sum_i K_i d^alpha u / d|x_i|^alpha = f in a convex polyhedron,
 * u = 0 outside (Sec. 1 eq. (1) for the chord bounds a_i(x), b_i(x); Sec. 3
 * for the zero extension), 1 < alpha <= 2.  The Riesz operator is
 * -(D_L^alpha + D_R^alpha) / (2 cos(pi alpha / 2)) and its weak form is
 * split into order-gamma = alpha/2 left/right Riemann-Liouville derivatives
 * (Sec. 1 eq. def, form 1 of eq. equ:varsss with alpha = beta):
 *
 *   K_jk = c_alpha sum_i K_i sum_g w_g [L_gi(k) R_gi(j) + R_gi(k) L_gi(j)],
 *   c_alpha = 1 / (2 cos(pi alpha / 2)),
 *
 * with L_gi(l) = D_L^gamma psi_l(x_g), R_gi(l) = D_R^gamma psi_l(x_g) along
 * e_i at Gauss point x_g with weight w_g (Sec. 2.1, element quadrature of
 * (K_E)_kl).  Each derivative is summed over the segments of the Gauss
 * point's integration path (Sec. 2.1) found by the ray-simplex walk of
 * Sec. 2.2.  Unknowns are the interior nodes (not on a boundary face),
 * numbered by increasing vertex id.
 *
 * Conventions for every call:
 *   - Return value: FPDE_OK (0) or a negative fpde_status; outputs are
 *     unspecified after an error.  No C++ exception crosses the ABI.
 *   - "dev" pointers are device memory on the mesh's device, owned by the
 *     caller; "host" pointers are host memory owned by the caller.  The
 *     library owns only the mesh handle, its device copy of the mesh and its
 *     scratch buffers (freed by fpde_mesh_destroy).
 *   - stream: a hipStream_t (NULL = legacy default stream).  Kernels are
 *     enqueued on it; calls that must report a device-side status or a size
 *     synchronise it once before returning (stated per call).
 *   - Matrices are dense, row-major with leading dimension lda >= n_dof.
 *     The Riesz stiffness matrix is symmetric, so row/column order is
 *     immaterial there; the Sec. 3 matrix (below) has the test function as
 *     its row.
 *   - One handle must not be used by two host threads at once.
 */
#ifndef FPDE_H
#define FPDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpde_mesh fpde_mesh; /* opaque, library-owned */

typedef enum {
  FPDE_OK = 0,
  FPDE_EINVAL = -1,            /* bad argument (null pointer, size, lda, rule) */
  FPDE_EMESH_NONMANIFOLD = -2, /* a face shared by more than two elements */
  FPDE_EMESH_DEGENERATE = -3,  /* zero-volume element or repeated vertex */
  FPDE_EMESH_NONCONVEX = -4,   /* a vertex lies outside the plane of a boundary face */
  FPDE_EPATH = -5,             /* a walk found no continuation or exceeded max_steps */
  FPDE_EALPHA = -6,            /* alpha outside (1, 2] or K_i <= 0 */
  FPDE_ENOTSPD = -7,           /* Cholesky met a pivot <= 0 */
  FPDE_ENOCONV = -8,           /* iterative refinement missed its tolerance */
  FPDE_EHIP = -9,              /* a HIP runtime call failed */
  FPDE_ENOMEM = -10,           /* device allocation failed */
  FPDE_EUNSUPPORTED = -11,     /* valid but not implemented combination */
  FPDE_ESINGULAR = -12         /* LU without pivoting met a zero or non-finite pivot */
} fpde_status;

enum { FPDE_FP64 = 0, FPDE_MIXED = 1 };
enum { FPDE_SRC_ONE = 0, FPDE_SRC_USER = 1, FPDE_SRC_CUBE_MMS = 2, FPDE_SRC_BALL_MMS = 3, FPDE_SRC_SQUARE_MMS = 4 };

typedef struct {
  double alpha;     /* Riesz order, 1 < alpha <= 2 */
  double K[3];      /* diffusion coefficients K_1..K_3 > 0 */
  int quad_points;  /* element rule: 4 (degree 2) or 11 (degree 4) points */
  int precision;    /* FPDE_FP64 or FPDE_MIXED */
  int source;       /* FPDE_SRC_ONE (f = 1), FPDE_SRC_USER (f given at the
                       Gauss points), FPDE_SRC_CUBE_MMS (manufactured source
                       of u = prod x_i^2 (1 - x_i)^2 on the unit cube) */
  int max_steps;    /* cap on elements per half-ray, 0 = 4096 */
  double ir_tol;    /* FPDE_MIXED: stop at ||b - K u|| / ||b|| <= ir_tol, 0 = 1e-8 */
  int ir_max_iter;  /* FPDE_MIXED: refinement sweeps, 0 = 30 */
  int deterministic; /* 1: the sums that build K (tube blocks, rows) run in one
                        wavefront per work item, so their additions come in a
                        fixed order and K is the same bit for bit on every run
                        (for parity runs; the FP64 accumulation is several
                        times slower); 0: the fastest order, K reproducible to
                        rounding only.  Occupies the struct's tail padding. */
} fpde_params;

typedef struct {
  int ir_iters;              /* refinement sweeps done (0 for FPDE_FP64) */
  double final_rel_residual; /* ||b - K u||_2 / ||b||_2 in FP64 */
  int64_t failed_pivot;      /* column of the first pivot <= 0, or -1 */
} fpde_solve_info;

/* Status text (static storage). */
const char *fpde_status_string(int status);

/*
 * Mesh set-up (Sec. 2.1 partition T_h; Sec. 2.2 "adjacent information of the
 * triangulation" and the m-face incidence used at edge/vertex go-out points).
 *   xyz:  host, n_vert x 3 FP64 vertex coordinates.
 *   tet:  host, n_tet x 4 int32 vertex ids in [0, n_vert), any orientation.
 * Copies both to the current HIP device, then builds on the device: per
 * element A^{-1} (A = (v1-v0, v2-v0, v3-v0)) and |E|, the neighbour across
 * each face (face f opposite local vertex f), boundary faces and nodes, the
 * interior numbering and vertex -> element lists.  The domain must be
 * convex (the chord bounds a_i(x), b_i(x) of Sec. 1 eq. (1) are the two ends
 * of one chord only then): every vertex used by an element must lie on the
 * inner side of the plane of every boundary face, within 1e-12 times the
 * diagonal of the vertices' bounding box, else FPDE_EMESH_NONCONVEX.
 * Synchronises `stream`.
 * Errors: FPDE_EINVAL (sizes, ids out of range), FPDE_EMESH_NONMANIFOLD,
 * FPDE_EMESH_DEGENERATE, FPDE_EMESH_NONCONVEX, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_mesh_create(const double *xyz, int64_t n_vert, const int32_t *tet, int64_t n_tet,
                     void *stream, fpde_mesh **out);
void fpde_mesh_destroy(fpde_mesh *m);

/* Sizes: interior unknowns, boundary faces, elements (any pointer may be NULL). */
int fpde_mesh_info(const fpde_mesh *m, int64_t *n_dof, int64_t *n_boundary_faces, int64_t *n_tet);

/* host, n_vert int32: unknown index of each vertex, -1 on the boundary. */
int fpde_dof_map(const fpde_mesh *m, int32_t *dof);

/*
 * Symbolic phase ("template", Sec. 2.3): walks every half-ray of the
 * quad_points rule once, records how many entries each derivative vector has
 * and builds the node -> entry transpose used by the accumulation.  Depends
 * on the mesh and rule only, so it is reused for every alpha and K.  Called
 * implicitly by fpde_assemble when missing; synchronises `stream`.
 * Errors: FPDE_EINVAL (rule), FPDE_EPATH, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_plan(fpde_mesh *m, int quad_points, int max_steps, void *stream);

/*
 * Integration paths (Sec. 2.2) of the half-rays (g, dir) for Gauss points
 * g in [g0, g0 + count) of the quad_points rule, dir = 2 i + side
 * (i = axis 0..2, side 0: -e_i, side 1: +e_i).  Gauss point g lies in element
 * g / quad_points.
 *   len:  dev, count int32: elements on the path.
 *   hash: dev, count uint64: FNV-1a 64 over the element ids (4 little-endian
 *         bytes each, in path order).
 *   ids:  dev or NULL, count x max_steps int32: the element ids.
 *   rend: dev or NULL, count x max_steps FP64: distance from x_g at which the
 *         path leaves each element.
 * Synchronises `stream`.  Errors: FPDE_EINVAL, FPDE_EPATH.
 */
int fpde_paths(fpde_mesh *m, int quad_points, int dir, int64_t g0, int64_t count, int max_steps,
               int32_t *len, uint64_t *hash, int32_t *ids, double *rend, void *stream);

/*
 * Derivative vectors of one direction: for Gauss points g in [g0, g0+count)
 * and dir = 2 i + side, the sparse vector D^gamma psi_l(x_g) (left for
 * side 0, right for side 1) over interior nodes l, gamma = alpha / 2.
 *   off:  host, count + 1 int64 (written): entries of ray k are
 *         [off[k], off[k+1]) of dof/val.
 *   dof:  host, capacity int32; val: host, capacity FP64.  A node may appear
 *         more than once in one ray (the values then add up).
 * Requires fpde_plan for the rule.  Synchronises `stream`.
 * Errors: FPDE_EINVAL (capacity too small: off[count] is still written),
 * FPDE_EALPHA, FPDE_EPATH.
 */
int fpde_ray_values(fpde_mesh *m, int quad_points, double alpha, int dir, int64_t g0, int64_t count,
                    int64_t *off, int32_t *dof, double *val, int64_t capacity, void *stream);

/*
 * Assembly (Sec. 2.1-2.3): the stiffness matrix and load vector.
 *   A: dev, n_dof x lda, FP64 (precision FPDE_FP64) or FP32 (FPDE_MIXED);
 *      every entry of the leading n_dof x n_dof block is written.
 *   b: dev, n_dof FP64, b_j = sum_g w_g f(x_g) psi_j(x_g); may be NULL.
 *   f_gauss: dev, n_tet * quad_points FP64 source values at the Gauss points
 *      (index element * quad_points + q) for FPDE_SRC_USER, else ignored.
 * Synchronises `stream` (walk status).
 * Errors: FPDE_EINVAL, FPDE_EALPHA, FPDE_EPATH, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_assemble(fpde_mesh *m, const fpde_params *p, void *A, int64_t lda, double *b,
                  const double *f_gauss, void *stream);

/*
 * fpde_assemble for `count` systems (1..16) of one mesh with one status
 * check at the end: system z (parameters p[z], host array; every p[z] of
 * one precision, no FPDE_SRC_USER) goes to A + z stride_A (elements of that
 * precision, stride_A >= n_dof lda when count > 1) and, when b is not NULL,
 * its load vector to b + z stride_b (stride_b >= n_dof).  The systems'
 * kernels are enqueued back to back; the caller of a batch solve
 * (fpde_solve_batch) assembles with this and synchronises twice per batch
 * instead of once per system.  The walks (derivative values) run on a
 * second stream owned by the mesh handle, each beside the previous
 * system's accumulation when that one uses the other quadrature rule;
 * events order them after the work already on `stream` and before the
 * accumulations on `stream`, so on return all of it is complete.
 * Synchronises `stream`.  Errors: as fpde_assemble; on a walk failure
 * every touched value set is invalidated and no system is to be used.
 */
int fpde_assemble_batch(fpde_mesh *m, int count, const fpde_params *p, void *A, int64_t lda, int64_t stride_A,
                        double *b, int64_t stride_b, void *stream);

/*
 * Matrix-free product y = K x in FP64 (the sums of fpde_assemble, never
 * forming K): the residual of the refinement in FPDE_MIXED.
 *   x, y: dev, n_dof FP64.  Synchronises `stream`.
 */
int fpde_apply(fpde_mesh *m, const fpde_params *p, const double *x, double *y, void *stream);

/*
 * Dense solve of K u = b (the "Solve linear equations" stage, Table 4).
 *   FPDE_FP64:  A (FP64, from fpde_assemble) is overwritten by its Cholesky
 *               factor L (lower triangle, K = L L^T); u = L^{-T} L^{-1} b.
 *   FPDE_MIXED: A (FP32) is overwritten by its FP32 Cholesky factor; u is
 *               refined with FP64 residuals b - K u from fpde_apply until
 *               ||r|| / ||b|| <= ir_tol.
 *   b, u: dev, n_dof FP64 (may alias).  info: host, may be NULL.
 * Synchronises `stream`.
 * Errors: FPDE_EINVAL, FPDE_ENOTSPD, FPDE_ENOCONV, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_solve(fpde_mesh *m, const fpde_params *p, void *A, int64_t lda, const double *b, double *u,
               fpde_solve_info *info, void *stream);

/*
 * Solve with an existing factor (from fpde_solve): u = K^{-1} b with the same
 * precision handling (FPDE_MIXED refines against fpde_apply).  Used for the
 * adjoint solve K lam = dJ/du (K is symmetric).
 */
int fpde_solve_factored(fpde_mesh *m, const fpde_params *p, const void *L, int64_t lda,
                        const double *b, double *u, fpde_solve_info *info, void *stream);

/*
 * FP64 dense solves of `count` independent systems K_z u_z = b_z, z < count
 * (the "Solve linear equations" stage, Table 4, for several alpha or rules at
 * once), with one launch sequence: the systems' Cholesky factorizations and
 * triangular solves run side by side on the device.
 *   A: dev FP64, count matrices of n_dof x n_dof (row-major, leading
 *      dimension lda >= n_dof), matrix z at A + z stride_A
 *      (stride_A >= n_dof lda when count > 1); each is overwritten by its
 *      Cholesky factor L_z (lower triangle), exactly as fpde_solve does.
 *   b, u: dev FP64, vector z at b + z stride_v and u + z stride_v
 *      (stride_v >= n_dof when count > 1); u may alias b.
 *   count: 1..16.  failed_pivot: host, count entries, may be NULL; entry z
 *      is the first column of the block where K_z was found not positive
 *      definite, else -1.
 * Synchronises `stream`.  The mesh handle's scratch is shared, so calls on
 * one handle must not overlap.
 * Errors: FPDE_EINVAL, FPDE_ENOTSPD (u then holds no solution), FPDE_ENOMEM,
 * FPDE_EHIP.
 */
int fpde_solve_batch(fpde_mesh *m, int count, double *A, int64_t lda, int64_t stride_A, const double *b,
                     double *u, int64_t stride_v, int64_t *failed_pivot, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * path of fpde_solve without its residual -- A (dev, n_dof x lda FP64, from
 * fpde_assemble) is overwritten by its Cholesky factor and u = K^{-1} b
 * (b, u: dev, n_dof FP64, may alias) -- with every scratch buffer (the
 * diagonal-block inverses, the triangular solves' flags and tickets, one
 * intermediate vector; 8.4 MB) in a static device array of the library
 * instead of the handle: no hipMalloc, hipFree or allocating library call.
 * Limit: n_dof <= 8192.  Each device holds one copy of the array for the
 * life of the process, shared by every call on that device: calls that
 * overlap on one device (other streams, other threads, other handles) race.
 * The current device must be the mesh's; stage timing must be off.
 * failed_pivot: host, may be NULL (as in fpde_solve_batch).  Synchronises
 * `stream` (one status check).
 * Errors: FPDE_EINVAL (null pointer, lda, n_dof > 8192, timing on, other
 * device), FPDE_ENOTSPD, FPDE_EHIP.
 */
int fpde_solve_noalloc(fpde_mesh *m, double *A, int64_t lda, const double *b, double *u, int64_t *failed_pivot,
                       void *stream);

/*
 * Adjoint sums for the gradient of a loss J(u) through assembly and solve
 * (u = K^{-1} b, b independent of alpha and K): with lam = K^{-1} dJ/du,
 *   dJ/dK_i   = -c_alpha S_i
 *   dJ/dalpha = -sum_i K_i (c'_alpha S_i + c_alpha T_i)
 *   S_i = sum_g w_g [(lam.R)(L.u) + (lam.L)(R.u)]
 *   T_i = sum_g w_g [(lam.R')(L.u) + (lam.R)(L'.u) + (lam.L')(R.u) + (lam.L)(R'.u)]
 * (' = d/dalpha).  The paths are walked again (recomputed, not stored).
 *   u, lam: dev, n_dof FP64.  grad_alpha, grad_K: host (1 and 3 FP64).
 * Synchronises `stream`.  Errors: FPDE_EINVAL, FPDE_EALPHA, FPDE_EPATH.
 */
int fpde_adjoint(fpde_mesh *m, const fpde_params *p, const double *u, const double *lam,
                 double *grad_alpha, double *grad_K, void *stream);

/*
 * Stage timing with HIP events recorded on the caller's stream around each
 * stage launch (no extra synchronisation while recording).
 * Stages: walk + closed-form evaluation, accumulation (both tube passes),
 * load vector, Cholesky factorisation (all panels), triangular solves,
 * matrix-free product, symbolic plan, adjoint re-walk, the tube products
 * pass timed again on its own inside CONTRACT, for the problem of Sec. 3
 * its LU factorisation and its accumulation, and the sparse products and
 * conjugate-gradient solves.
 *   fpde_timing(m, 1) clears the totals and starts recording; (m, 0) stops.
 *   fpde_timing_stages(m, mask) does the same for the stages whose bit
 *   (1u << FPDE_STAGE_x) is set in mask only (mask 0 stops; fpde_timing(m, 1)
 *   is mask ~0u).  Every timed stage costs two event records per interval on
 *   the stream, so a throughput measurement times only what it reports.
 *   fpde_stage_times waits for the recorded events, then writes per stage
 *   the summed milliseconds (host, FPDE_NSTAGES doubles) and the number of
 *   timed intervals (host, FPDE_NSTAGES int64; either pointer may be NULL).
 */
enum {
  FPDE_STAGE_WALK = 0,
  FPDE_STAGE_CONTRACT = 1,
  FPDE_STAGE_LOAD = 2,
  FPDE_STAGE_POTRF = 3,
  FPDE_STAGE_TRSV = 4,
  FPDE_STAGE_APPLY = 5,
  FPDE_STAGE_PLAN = 6,
  FPDE_STAGE_ADJOINT = 7,
  FPDE_STAGE_ACCUM = 8,
  FPDE_STAGE_LU = 9,    /* LU factorisation of the Sec. 3 matrix (all panels) */
  FPDE_STAGE_DIV = 10,  /* accumulation of the Sec. 3 matrix */
  FPDE_STAGE_SPMV = 11, /* CSR products (fpde_csr_apply and inside fpde_cg_solve) */
  FPDE_STAGE_CG = 12,   /* a whole conjugate-gradient solve */
  FPDE_STAGE_FORM = 13, /* accumulation of a general uniform form (fpde_form_assemble) */
  FPDE_NSTAGES = 14
};
int fpde_timing(fpde_mesh *m, int enable);
int fpde_timing_stages(fpde_mesh *m, unsigned mask);
int fpde_stage_times(fpde_mesh *m, double *ms, int64_t *count);

/*
 * The template T of Sec. 2.3 (Table 1): T_jk = 1 when, for some axis i, the
 * axis-aligned boxes of the element patches of nodes j and k overlap (closed
 * intervals) in both coordinates other than i -- the only case in which a
 * line parallel to e_i meets both supports, so T contains the nonzero
 * pattern of K.  The patch boxes are computed once per mesh and kept.
 *   tile  : tile edge in unknowns, 1..256.
 *   tiles : host, nt x nt uint8 row-major, nt = ceil(n_dof / tile): 1 when
 *           any (j, k) of the tile has T_jk = 1.
 *   nnz   : host int64, the number of (j, k) with T_jk = 1.
 * Synchronises `stream`.  FPDE_EINVAL for a tile outside 1..256.
 */
int fpde_template(fpde_mesh *m, int tile, uint8_t *tiles, int64_t *nnz, void *stream);

/*
 * Sizes of the symbolic plan of a rule (built on demand; see fpde_plan):
 *   out[0] half-rays (6 G), out[1] derivative-vector entries over all
 *   half-rays, out[2] sum over (g, i) of |L_gi| |R_gi| (entry pairs the
 *   accumulation multiplies), out[3] largest number of entries of one
 *   half-ray, out[4] tubes (groups of chords of one axis through one cell of
 *   the orthogonal plane, Sec. 2.3), out[5] sum over tubes of the number of
 *   nodes the tube's chords touch, out[6] the largest such number, out[7]
 *   bytes of the per-tube block scratch the accumulation uses.
 *   host, 8 int64.  Synchronises `stream`.
 */
int fpde_plan_info(fpde_mesh *m, int quad_points, int64_t *out, void *stream);

/*
 * ---- Sparse storage on the template (Sec. 2.3, Table 1) and a Krylov solve ----
 *
 * K stored as CSR on the template T (the pattern of fpde_template, at node
 * granularity): rows are unknowns, columns increasing, the diagonal always
 * present.  T contains the nonzero pattern of K, so nothing is dropped.
 */

/*
 * The template as CSR.  row_ptr: dev, n_dof + 1 int64 (always written);
 * nnz: host int64 (always written).  col: dev, capacity int32, written when
 * not NULL (call once with col = NULL to learn nnz).  O(n_dof^2) box tests,
 * once per mesh.  Synchronises `stream`.
 * Errors: FPDE_EINVAL (capacity < nnz), FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_template_csr(fpde_mesh *m, int64_t *row_ptr, int32_t *col, int64_t capacity, int64_t *nnz,
                      void *stream);

/*
 * Assembly of K (the same sums as fpde_assemble) into val (dev, nnz FP64)
 * on the pattern row_ptr / col from fpde_template_csr, and of b (dev, n_dof,
 * may be NULL).  FPDE_FP64 only.  Synchronises `stream`.
 * Errors: FPDE_EINVAL, FPDE_EALPHA, FPDE_EUNSUPPORTED (mixed), FPDE_EPATH,
 * FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_assemble_csr(fpde_mesh *m, const fpde_params *p, const int64_t *row_ptr, const int32_t *col,
                      double *val, double *b, const double *f_gauss, void *stream);

/* y = K x for the CSR matrix (all dev, FP64).  Does not synchronise. */
int fpde_csr_apply(fpde_mesh *m, const int64_t *row_ptr, const int32_t *col, const double *val,
                   const double *x, double *y, void *stream);

/*
 * K u = b by conjugate gradients with the Jacobi preconditioner (K is
 * symmetric positive definite), from u = 0, until ||b - K u|| / ||b|| <= tol
 * in the recurrence; info->final_rel_residual is then recomputed from
 * b - K u.  The operator is the CSR matrix when row_ptr is not NULL, else the
 * matrix-free product of fpde_apply (no N^2 storage at all).
 *   b, u: dev, n_dof FP64, distinct.  tol: 0 = 1e-10.  max_iter: 0 = 10000.
 *   info: host, may be NULL (ir_iters = CG iterations).
 * Synchronises `stream` every iteration.
 * Errors: FPDE_EINVAL, FPDE_EALPHA, FPDE_ENOTSPD (a diagonal entry or p.Kp
 * <= 0), FPDE_ENOCONV (max_iter reached), FPDE_EPATH, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_cg_solve(fpde_mesh *m, const fpde_params *p, const int64_t *row_ptr, const int32_t *col,
                  const double *val, const double *b, double *u, double tol, int max_iter,
                  fpde_solve_info *info, void *stream);

/*
 * ---- The divergence-form two-sided problem of Sec. 3 (eq. equ:sfde2) ----
 *
 *   sum_i D_i (p_i D_L^{beta_i} u - q_i D_R^{beta_i} u) = f,  u = 0 outside,
 *
 * 0 < beta_i <= 1, on the same convex meshes.  Its weak form (one classical
 * integration by parts on the test side) is
 *   a(u, v) = -sum_i [(p_i D_L^{beta_i} u, D_i v) - (q_i D_R^{beta_i} u, D_i v)],
 * so with the element quadrature of Sec. 2.1
 *   K_jk = -sum_i sum_g w_g (d_i psi_j)(x_g) [p_i(x_g) L_gi(k) - q_i(x_g) R_gi(k)],
 * L_gi / R_gi the order-beta_i derivative vectors of the half-rays along e_i
 * (the walk of Sec. 2.2) and d_i psi_j the slope of psi_j on the Gauss
 * point's own element.  K is not symmetric: row j is the test function.
 */
enum { FPDE_COEF_SEC3 = 0, FPDE_COEF_USER = 1, FPDE_COEF_CONST = 2 };

typedef struct {
  double beta[3];   /* orders beta_1..beta_3, each in (0, 1] */
  int quad_points;  /* element rule: 4 or 11 points */
  int coef;         /* FPDE_COEF_SEC3: p_i = cos x_i, q_i = 1 - cos x_i (Sec. 3);
                       FPDE_COEF_USER: p_i, q_i given at the Gauss points */
  int source;       /* FPDE_SRC_ONE, FPDE_SRC_USER, or FPDE_SRC_BALL_MMS: the
                       source of u = (|x|^2 - r^2)^2 on the ball |x| < radius
                       with the coefficients of Sec. 3 (its closed form along
                       each chord) */
  double radius;    /* FPDE_SRC_BALL_MMS: r > 0 */
  int max_steps;    /* cap on elements per half-ray, 0 = 4096 */
} fpde_div_params;

/*
 * Assembly of K (above) and b_j = sum_g w_g f(x_g) psi_j(x_g).
 *   pq: dev, 6 G FP64 for FPDE_COEF_USER (G = n_tet * quad_points Gauss
 *       points, index element * quad_points + q): p_i(x_g) at [i G + g],
 *       q_i(x_g) at [(3 + i) G + g]; else ignored (may be NULL).
 *   A:  dev, n_dof x lda FP64; every entry of the leading n_dof x n_dof block
 *       is written.
 *   b:  dev, n_dof FP64, or NULL.  f_gauss: dev, G FP64 for FPDE_SRC_USER.
 * Shares the symbolic plan (fpde_plan) with the Riesz problem; the entry
 * values are recomputed only for the axes whose order changed.
 * Synchronises `stream`.
 * Errors: FPDE_EINVAL, FPDE_EALPHA (beta_i outside (0, 1]), FPDE_EPATH,
 * FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_div_assemble(fpde_mesh *m, const fpde_div_params *p, const double *pq, double *A, int64_t lda,
                      double *b, const double *f_gauss, void *stream);

/*
 * LU factorisation without pivoting of the n_dof x n_dof matrix in A
 * (dev, FP64, lda >= n_dof), in place: A = L U with L unit lower (strict
 * lower triangle of A) and U upper (upper triangle with the diagonal).
 * Meant for the Sec. 3 matrix, whose symmetric part is definite (the form is
 * coercive), so every leading block is nonsingular.  A zero or non-finite
 * pivot gives FPDE_ESINGULAR and, if failed_pivot (host) is not NULL, the
 * first column of the 64-wide block where it occurred.  Synchronises
 * `stream`.  Errors: FPDE_EINVAL, FPDE_ESINGULAR, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_lu_factor(fpde_mesh *m, double *A, int64_t lda, int64_t *failed_pivot, void *stream);

/*
 * u = U^{-1} L^{-1} b with the factor from fpde_lu_factor.
 *   LU: dev, n_dof x lda FP64 (unchanged); b, u: dev, n_dof FP64 (may alias).
 * Synchronises `stream`.  Errors: FPDE_EINVAL, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_lu_solve(fpde_mesh *m, const double *LU, int64_t lda, const double *b, double *u, void *stream);

/*
 * ---- The general uniform form of Sec. 1 (eq. equ:varsss) ----
 *
 *   K_kl = sum_i sum_g w_g [cl_i(x_g) D_L^{alpha_i} psi_l(x_g) D_R^{beta_i} psi_k(x_g)
 *                         + cr_i(x_g) D_R^{alpha_i} psi_l(x_g) D_L^{beta_i} psi_k(x_g)]
 *
 * (c D^alpha u, D^beta v) with the test operator on the side opposite to the
 * trial one, per axis, with the element quadrature of Sec. 2.1; row k is the
 * test function.  Orders in [0, 1]: 0 is the identity, 1 the classical
 * derivative (D_L^1 = d/dx_i, D_R^1 = -d/dx_i), so the three operator forms
 * of Sec. 1 and the problems of fpde_assemble (alpha_i = beta_i = alpha/2,
 * cl = cr = K_i c_alpha) and fpde_div_assemble (beta_i = 1, cl = p_i,
 * cr = q_i) are instances.
 */
typedef struct {
  double alpha[3];  /* trial orders, each in [0, 1] */
  double beta[3];   /* test orders, each in [0, 1] */
  int quad_points;  /* 4 or 11 */
  int coef;         /* FPDE_COEF_CONST: cl, cr below; FPDE_COEF_USER: at the Gauss points */
  double cl[3];     /* FPDE_COEF_CONST: coefficient of the (D_L^alpha u, D_R^beta v) term per axis */
  double cr[3];     /* FPDE_COEF_CONST: coefficient of the (D_R^alpha u, D_L^beta v) term per axis */
  int max_steps;    /* cap on elements per half-ray, 0 = 4096 */
} fpde_form_params;

/*
 * Assembly of K (above) into A (dev, n_dof x lda FP64; the leading
 * n_dof x n_dof block is written).  coef: dev, 6 G FP64 for
 * FPDE_COEF_USER (cl_i(x_g) at [i G + g], cr_i(x_g) at [(3 + i) G + g],
 * g = element * quad_points + q), else ignored.  Every half-ray is evaluated
 * at the trial and at the test orders (two value sets in the plan, each
 * recomputed only for the axes whose order changed).  Synchronises `stream`.
 * Errors: FPDE_EINVAL, FPDE_EALPHA (an order outside [0, 1]), FPDE_EPATH,
 * FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_form_assemble(fpde_mesh *m, const fpde_form_params *p, const double *coef, double *A, int64_t lda,
                       void *stream);

/*
 * ---- The two-dimensional variant (n = 2; Sec. 1 with n = 2, Fig. 1a) ----
 *
 * P1 elements on a convex triangulated polygon, paths along +-e_1, +-e_2
 * (the walk of Sec. 2.2 with three area coordinates: an edge go-out leads
 * to the triangle across it, a vertex go-out to the smallest-id triangle
 * around the vertex in which the ray advances), the split Riesz stiffness
 *   K_jk = c_alpha sum_{i=1,2} K_i sum_g w_g [L_gi(k) R_gi(j) + R_gi(k) L_gi(j)],
 * the load vector and the dense FP64 Cholesky solve.  Element rules: 3
 * points (degree 2) and 7 points (degree 5, Radon).  Unknowns are the
 * vertices on no boundary edge, by increasing vertex id.  Conventions as for
 * the 3-D calls.
 */
typedef struct fpde_mesh2d fpde_mesh2d; /* opaque, library-owned */

typedef struct {
  double alpha;     /* Riesz order, 1 < alpha <= 2 */
  double K[2];      /* K_1, K_2 > 0 */
  int quad_points;  /* 3 or 7 */
  int source;       /* FPDE_SRC_ONE, FPDE_SRC_USER, or FPDE_SRC_SQUARE_MMS: the
                       manufactured source of u = phi(x) phi(y),
                       phi(s) = s^2 (1 - s)^2, on the unit square */
  int max_steps;    /* cap on elements per half-ray, 0 = 4096 */
} fpde_params2d;

/*
 * xy: host, n_vert x 2 FP64; tri: host, n_tri x 3 int32 (any orientation).
 * Builds on the device: A^{-1} and area per triangle, edge adjacency (edge f
 * opposite local vertex f), boundary, numbering, vertex -> triangle lists.
 * Synchronises `stream`.  Errors: FPDE_EINVAL, FPDE_EMESH_NONMANIFOLD,
 * FPDE_EMESH_DEGENERATE, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_mesh2d_create(const double *xy, int64_t n_vert, const int32_t *tri, int64_t n_tri, void *stream,
                       fpde_mesh2d **out);
void fpde_mesh2d_destroy(fpde_mesh2d *m);
int fpde_mesh2d_info(const fpde_mesh2d *m, int64_t *n_dof, int64_t *n_boundary_edges, int64_t *n_tri);
/* host, n_vert int32: unknown of each vertex, -1 on the boundary */
int fpde_dof_map2d(const fpde_mesh2d *m, int32_t *dof);

/*
 * Paths of the half-rays (g, dir) for Gauss points g in [g0, g0 + count),
 * dir = 2 i + side (i = 0, 1; side 0: -e_i, side 1: +e_i); g lies in
 * triangle g / quad_points.  Outputs as fpde_paths (len, FNV-1a hash of the
 * triangle ids, optional ids and break points).  Synchronises `stream`.
 */
int fpde_paths2d(fpde_mesh2d *m, int quad_points, int dir, int64_t g0, int64_t count, int max_steps,
                 int32_t *len, uint64_t *hash, int32_t *ids, double *rend, void *stream);

/*
 * K (dev, n_dof x lda FP64, leading block written) and b (dev, n_dof, may be
 * NULL); f_gauss: dev, n_tri * quad_points for FPDE_SRC_USER.  The symbolic
 * plan (paths, entry counts, node -> entry transpose) is built on first use
 * per rule.  Synchronises `stream`.
 * Errors: FPDE_EINVAL, FPDE_EALPHA, FPDE_EPATH, FPDE_ENOMEM, FPDE_EHIP.
 */
int fpde_assemble2d(fpde_mesh2d *m, const fpde_params2d *p, double *A, int64_t lda, double *b,
                    const double *f_gauss, void *stream);

/*
 * K u = b by the FP64 Cholesky of the 3-D path; A is overwritten by its
 * factor.  b, u: dev (may alias).  failed_pivot: host, may be NULL.
 * Synchronises `stream`.  Errors: FPDE_EINVAL, FPDE_ENOTSPD, FPDE_ENOMEM,
 * FPDE_EHIP.
 */
int fpde_solve2d(fpde_mesh2d *m, double *A, int64_t lda, const double *b, double *u, int64_t *failed_pivot,
                 void *stream);

/* stage timing of a 2-D handle (as fpde_timing / fpde_stage_times) */
int fpde_timing2d(fpde_mesh2d *m, int enable);
int fpde_stage_times2d(fpde_mesh2d *m, double *ms, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* FPDE_H */
