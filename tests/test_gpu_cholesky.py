"""The dense Cholesky solve (Table 4's solve stage) on its own, through the
C ABI, at sizes that take every branch of the blocked factorization: one
partial block, exactly one block, a pair of 64-column panels followed by a
single last panel, pairs that end exactly at N, a partial last block, and
trailing matrices of one and of several 128 x 128 update tiles, full and
partial (N = 1000, 1728).

The matrices are seeded random SPD matrices (any SPD matrix of the mesh's
size is a valid input); the factor must equal LAPACK's Cholesky factor and
the solution LAPACK's solution within 1e-10 (max-norm relative), one system
at a time and as a batch.
"""
import numpy as np
import pytest
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
