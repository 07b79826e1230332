"""The dense Cholesky solve (Table 4's solve stage) on its own, through the
C ABI, at sizes that take every branch of the blocked factorization: one
partial block, exactly one block, panels inside one group of sixteen that
end exactly at N or in a partial last block, a whole group and its
in-group strips only (N = 1000), and a group followed by a trailing update
of five full and one partial 128 x 128 tile rows (N = 1728).

The FP32 factorization (split-FP16 trailing updates; groups of sixteen
panels with per-panel strips below 16 384 unknowns, of 32 panels updated in
four-panel parts from there) is checked on assembled mixed-precision
matrices: part of one group (N = 512, 1000), one group then a trailing
update with a ragged tail (1728), whole groups (4096) and 19 683 unknowns
(parts, look-ahead, 256 x 256 tiles).  Its
factor must lie within 16 times LAPACK's own FP32 factorization's
(spotrf) distance from the FP64 Cholesky factor of the same FP32 matrix:
the panels apply each 64 x 64 diagonal block through its explicit inverse
(X = B inv(L_bb)^T) rather than a triangular solve, which adds rounding
that grows with the block's condition number.  The refined solution must
equal the FP64 solve's within 1e-8.

The matrices are seeded random SPD matrices (any SPD matrix of the mesh's
size is a valid input); the factor must equal LAPACK's Cholesky factor and
the solution LAPACK's solution within 1e-10 (max-norm relative), one system
at a time and as a batch.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import paper_1811_03339_amd as F
from fpde_inputs import kuhn_cube

pytestmark = pytest.mark.gpu

# unit cube with k^3 sub-cubes: (k - 1)^3 unknowns
SIZES = {2: 1, 3: 8, 5: 64, 6: 125, 7: 216, 8: 343, 9: 512, 10: 729, 11: 1000, 13: 1728}
_MESHES = {}


def mesh(k):
    if k not in _MESHES:
        m = kuhn_cube(k)
        _MESHES[k] = F.Mesh(m.xyz, m.tet)
        assert _MESHES[k].n_dof == SIZES[k]
    return _MESHES[k]


def spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(n, n))
    return M @ M.T / n + np.eye(n), rng.normal(size=n)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("k", sorted(SIZES))
def test_factor_and_solve_match_lapack(k):
    gm = mesh(k)
    n = gm.n_dof
    print(f"[cholesky] n={n}", flush=True)
    S, rhs = spd(n, 100 + k)
    A = torch.tensor(S, device="cuda")
    b = torch.tensor(rhs, device="cuda")
    u = torch.empty_like(b)
    gm.solve(F.params(1.5), A, b, u, info=False)
    torch.cuda.synchronize()
    assert rel(np.tril(A.cpu().numpy()), np.linalg.cholesky(S)) <= 1e-10
    assert rel(u.cpu().numpy(), np.linalg.solve(S, rhs)) <= 1e-10


def test_fp64_factor_groups_of_32_match_lapack():
    """17 576 unknowns: groups of 32 panels updated in four-panel parts (part
    updates over 256, 512 and 1024 columns), look-ahead on the side stream.
    A missed or repeated contribution of any panel to any block column would
    put the factor far outside the bound.  The matrix is a seeded random
    symmetric one made diagonally dominant (SPD by Gershgorin)."""
    cube = kuhn_cube(27)
    gm = F.Mesh(cube.xyz, cube.tet)
    n = gm.n_dof
    print(f"[cholesky] groups of 32, n={n}", flush=True)
    rng = np.random.default_rng(327)
    S = rng.random((n, n))
    S += S.T
    S[np.diag_indices(n)] += 2.0 * n
    rhs = rng.normal(size=n)
    A = torch.tensor(S, device="cuda")
    b = torch.tensor(rhs, device="cuda")
    u = torch.empty_like(b)
    gm.solve(F.params(1.5), A, b, u, info=False)
    torch.cuda.synchronize()
    L = np.linalg.cholesky(S)
    assert rel(np.tril(A.cpu().numpy()), L) <= 1e-10
    ref = scipy.linalg.cho_solve((L, True), rhs)
    assert rel(u.cpu().numpy(), ref) <= 1e-10


@pytest.mark.parametrize("k", [3, 6, 7, 9, 10, 11])
def test_batch_matches_lapack(k):
    gm = mesh(k)
    n = gm.n_dof
    print(f"[cholesky batch] n={n}", flush=True)
    mats = [spd(n, 200 + 10 * k + z) for z in range(3)]
    A = torch.tensor(np.stack([S for S, _ in mats]), device="cuda")
    b = torch.tensor(np.stack([r for _, r in mats]), device="cuda")
    u = torch.empty_like(b)
    gm.solve_batch(A, b, u)
    torch.cuda.synchronize()
    for z, (S, rhs) in enumerate(mats):
        assert rel(np.tril(A[z].cpu().numpy()), np.linalg.cholesky(S)) <= 1e-10, z
        assert rel(u[z].cpu().numpy(), np.linalg.solve(S, rhs)) <= 1e-10, z


# n = 512 ... 4096, and 19683 (groups of 32 panels in parts of four), whose
# first trailing update (17 635 rows) takes the 256 x 256 tiles with a ragged
# last tile row, under the look-ahead
@pytest.mark.parametrize("k", [9, 11, 13, 17, 28])
def test_fp32_factor_as_accurate_as_spotrf(k):
    if k in SIZES:
        gm = mesh(k)
    else:
        cube = kuhn_cube(k)
        gm = F.Mesh(cube.xyz, cube.tet)
    n = gm.n_dof
    print(f"[cholesky fp32] n={n}", flush=True)
    pm = F.params(1.5, quad_points=4, precision=F.FPDE_MIXED, ir_tol=1e-10)
    A = torch.empty((n, n), dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    gm.assemble(pm, A, b)
    K32 = A.cpu().numpy()
    u = torch.empty_like(b)
    gm.solve(pm, A, b, u)
    torch.cuda.synchronize()
    L64 = np.linalg.cholesky(K32.astype(np.float64))
    L32 = np.linalg.cholesky(K32).astype(np.float64)  # LAPACK spotrf
    bar = rel(L32, L64)
    got = rel(np.tril(A.cpu().numpy()).astype(np.float64), L64)
    print(f"[cholesky fp32] n={n} factor {got:.2e} vs spotrf {bar:.2e}", flush=True)
    assert got <= 16.0 * bar + 1e-12
    A64 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    b64 = torch.empty_like(b)
    p64 = F.params(1.5, quad_points=4)
    gm.assemble(p64, A64, b64)
    u64 = torch.empty_like(b)
    gm.solve(p64, A64, b64, u64, info=False)
    torch.cuda.synchronize()
    assert rel(u.cpu().numpy(), u64.cpu().numpy()) <= 1e-8
