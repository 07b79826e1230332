// The template T of Sec. 2.3: the 0/1 pattern of the fractional stiffness
// matrix, known before any path is walked.
//
// Node j's basis function lives on its element patch omega_j (the elements
// containing z_j).  K_jk can be nonzero through axis i only if some line
// parallel to e_i meets both omega_j and omega_k, i.e. only if their
// projections on the plane orthogonal to e_i meet; with axis-aligned boxes
// of the patches that is: the boxes overlap in both coordinates other than i.
// T_jk = 1 when that holds for some i (a superset of the pattern of K; the
// printed one-coordinate test is read this way).  Its density falls like
// 1/N^2 in 3-D (Table 1), so most 64 x 64 tiles of a large K are empty.
//
//   k_patch_boxes     per node: min / max of its patch's vertex coordinates
//                     (cached in the mesh, built once);
//   k_template_tiles  per pair of tiles: every node pair of the two tiles
//                     tested from the boxes staged in LDS; the tile's flag
//                     and the count of set pairs.
#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kMaxTile = 256;

__global__ void k_patch_boxes(const int32_t *__restrict__ vert_of_dof, const int32_t *__restrict__ vt_off,
                              const int32_t *__restrict__ vt_tet, const int32_t *__restrict__ tet,
                              const double *__restrict__ xyz, int64_t ndof, double *__restrict__ box) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ndof) return;
  const int32_t v = vert_of_dof[j];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t p = vt_off[v]; p < vt_off[v + 1]; p++) {
    const int64_t t = vt_tet[p];
    for (int m = 0; m < 4; m++) {
      const double *x = xyz + 3 * (int64_t)tet[4 * t + m];
      for (int d = 0; d < 3; d++) {
        lo[d] = fmin(lo[d], x[d]);
        hi[d] = fmax(hi[d], x[d]);
      }
    }
  }
  for (int d = 0; d < 3; d++) {
    box[6 * j + d] = lo[d];
    box[6 * j + 3 + d] = hi[d];
  }
}

__device__ __forceinline__ bool boxes_meet(const double *a, const double *b) {
  bool ov[3];
#pragma unroll
  for (int d = 0; d < 3; d++) ov[d] = a[d] <= b[3 + d] && b[d] <= a[3 + d];
  return (ov[1] && ov[2]) || (ov[2] && ov[0]) || (ov[0] && ov[1]);
}

// one workgroup per tile pair (P, Q), P <= Q; the result is mirrored to (Q, P)
__global__ void __launch_bounds__(256) k_template_tiles(const double *__restrict__ box, int64_t ndof, int tile,
                                                        int64_t nt, uint8_t *__restrict__ tiles,
                                                        unsigned long long *__restrict__ nnz) {
  __shared__ double bp[kMaxTile * 6], bq[kMaxTile * 6];
  __shared__ int cnt;
  const int64_t x = blockIdx.x;
  const int64_t P = x / nt, Q = x - P * nt;
  if (P > Q) return;  // uniform per workgroup
  const int64_t p0 = P * tile, q0 = Q * tile;
  const int np = (int)((ndof - p0) < tile ? (ndof - p0) : tile);
  const int nq = (int)((ndof - q0) < tile ? (ndof - q0) : tile);
  for (int k = threadIdx.x; k < 6 * np; k += blockDim.x) bp[k] = box[6 * p0 + k];
  for (int k = threadIdx.x; k < 6 * nq; k += blockDim.x) bq[k] = box[6 * q0 + k];
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int idx = threadIdx.x; idx < np * nq; idx += blockDim.x) {
    const int a = idx / nq, b = idx - a * nq;
    c += boxes_meet(bp + 6 * a, bq + 6 * b) ? 1 : 0;
  }
  if (c) atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint8_t f = cnt > 0 ? 1 : 0;
    tiles[P * nt + Q] = f;
    tiles[Q * nt + P] = f;
    if (cnt) atomicAdd(nnz, (unsigned long long)cnt * (P == Q ? 1ull : 2ull));
  }
}

}  // namespace

int ensure_patch_boxes(fpde_mesh *m, hipStream_t s) {
  if (m->pbox || m->ndof == 0) return FPDE_OK;
  FPDE_TRY(dalloc(&m->pbox, 6 * (size_t)m->ndof));
  k_patch_boxes<<<(unsigned)((m->ndof + 255) / 256), 256, 0, s>>>(m->vert_of_dof, m->vt_off, m->vt_tet, m->tet,
                                                                  m->xyz, m->ndof, m->pbox);
  FPDE_HIP(hipGetLastError());
  return FPDE_OK;
}

}  // namespace fpde

using namespace fpde;

extern "C" int fpde_template(fpde_mesh *m, int tile, uint8_t *tiles, int64_t *nnz, void *stream) {
  if (!m || !tiles || !nnz || tile < 1 || tile > kMaxTile) return FPDE_EINVAL;
  hipStream_t s = S(stream);
  *nnz = 0;
  if (m->ndof == 0) return FPDE_OK;
  FPDE_TRY(ensure_patch_boxes(m, s));
  const int64_t nt = (m->ndof + tile - 1) / tile;
  uint8_t *dt = nullptr;
  unsigned long long *dn = nullptr;
  FPDE_TRY(dalloc(&dt, (size_t)(nt * nt)));
  if (dalloc(&dn, 1) != FPDE_OK) {
    dfree(dt);
    return FPDE_ENOMEM;
  }
  int st = FPDE_OK;
  unsigned long long hn = 0;
  if (hipMemsetAsync(dn, 0, sizeof(*dn), s) != hipSuccess) st = FPDE_EHIP;
  const long t = timer_begin(m, s, FPDE_STAGE_PLAN);
  if (st == FPDE_OK) k_template_tiles<<<(unsigned)(nt * nt), 256, 0, s>>>(m->pbox, m->ndof, tile, nt, dt, dn);
  timer_end(m, FPDE_STAGE_PLAN, t, s);
  if (st == FPDE_OK && hipGetLastError() != hipSuccess) st = FPDE_EHIP;
  if (st == FPDE_OK && hipMemcpyAsync(tiles, dt, (size_t)(nt * nt), hipMemcpyDeviceToHost, s) != hipSuccess)
    st = FPDE_EHIP;
  if (st == FPDE_OK && hipMemcpyAsync(&hn, dn, sizeof(hn), hipMemcpyDeviceToHost, s) != hipSuccess)
    st = FPDE_EHIP;
  if (st == FPDE_OK && hipStreamSynchronize(s) != hipSuccess) st = FPDE_EHIP;
  dfree(dt);
  dfree(dn);
  if (st == FPDE_OK) *nnz = (int64_t)hn;
  return st;
}
