"""Parity of the HIP path for the divergence-form problem of Sec. 3 with the
FP64 CPU oracle, through the C ABI.

* K (non-symmetric, row = test function) and b element by element within
  1e-11 (max-norm relative; the accumulation order differs), for both rules,
  the orders of Table 3 and an order below 1/2, the coefficients of Sec. 3
  and user coefficients; the per-axis reuse of derivative values.
* The LU factorization without pivoting against a textbook right-looking
  elimination in NumPy, on single, exact-multiple and ragged block counts;
  a zero pivot is reported with its block.
* Whole solves against the oracle's LAPACK LU solution within 1e-9, and the
  discrete error against the exact solution equal to the oracle's.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_03339_amd as F
from fpde_inputs import kuhn_cube, workload_mesh

pytestmark = pytest.mark.gpu

R = 0.5
_MESHES = {}


def mesh_pair(name):
    if name not in _MESHES:
        if name.startswith("cube"):
            m = kuhn_cube(int(name[4:]))
        else:
            m = workload_mesh(name)
        print(f"[mesh] {name}: {m.n_vert} vertices, {m.n_tet} elements", flush=True)
        _MESHES[name] = (m, oracle.OracleMesh(m.xyz, m.tet), F.Mesh(m.xyz, m.tet))
    return _MESHES[name]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_div(gm, p, pq=None, f_gauss=None, with_b=True):
    A = F.new_matrix(gm)
    b = torch.empty(max(gm.n_dof, 1), dtype=torch.float64, device="cuda") if with_b else None
    gm.div_assemble(p, A, b, pq, f_gauss)
    torch.cuda.synchronize()
    return A, b


BETAS = [(0.8, 0.8, 0.8), (0.6, 0.7, 0.8), (0.3, 0.95, 0.45)]


@pytest.mark.parametrize("name,nq", [("cube4", 4), ("cube4", 11), ("sphere_small", 11), ("ball_h139", 4),
                                     ("ball_h139", 11)])
@pytest.mark.parametrize("beta", BETAS)
def test_matrix_matches_oracle(name, nq, beta):
    print(f"[case] matrix {name} nq={nq} beta={beta}", flush=True)
    m, om, gm = mesh_pair(name)
    A, _ = gpu_div(gm, F.div_params(beta, nq), with_b=False)
    want = om.assemble_div(nq, beta)
    assert rel(A.cpu().numpy(), want) <= 1e-11


def test_user_coefficients_match_oracle():
    m, om, gm = mesh_pair("ball_h139")
    nq, beta = 4, (0.6, 0.7, 0.8)
    G = m.n_tet * nq
    rng = np.random.default_rng(31)
    pq = rng.uniform(0.2, 1.5, size=(6, G))
    p = F.div_params(beta, nq, coef=F.FPDE_COEF_USER)
    A, _ = gpu_div(gm, p, pq=torch.tensor(pq, device="cuda"), with_b=False)
    assert rel(A.cpu().numpy(), om.assemble_div(nq, beta, pq)) <= 1e-11


@pytest.mark.parametrize("nq", [4, 11])
def test_load_vectors_match_oracle(nq):
    m, om, gm = mesh_pair("ball_h139")
    beta = (0.6, 0.7, 0.8)
    x, _ = om.gauss_points(nq)
    _, b = gpu_div(gm, F.div_params(beta, nq, source=F.FPDE_SRC_BALL_MMS, radius=R))
    assert rel(b.cpu().numpy(), om.load(nq, oracle.ball_source(x, beta, R))) <= 1e-11
    _, b = gpu_div(gm, F.div_params(beta, nq, source=F.FPDE_SRC_ONE))
    assert rel(b.cpu().numpy(), om.load(nq)) <= 1e-12
    f = np.sin(3 * x[:, 0]) + x[:, 1] * x[:, 2]
    _, b = gpu_div(gm, F.div_params(beta, nq, source=F.FPDE_SRC_USER), f_gauss=torch.tensor(f, device="cuda"))
    assert rel(b.cpu().numpy(), om.load(nq, f)) <= 1e-12


def test_axis_values_are_reused_and_refreshed():
    """Orders that change on one axis only, and the Riesz path in between
    (all axes at alpha / 2), must never leave stale values behind."""
    m, om, gm = mesh_pair("sphere_small")
    nq = 4
    for beta in [(0.6, 0.7, 0.8), (0.6, 0.9, 0.8), (0.6, 0.9, 0.8), (0.75, 0.75, 0.75)]:
        A, _ = gpu_div(gm, F.div_params(beta, nq), with_b=False)
        assert rel(A.cpu().numpy(), om.assemble_div(nq, beta)) <= 1e-11, beta
        # a Riesz assembly in between sets every axis to alpha / 2 = 0.75
        K = F.new_matrix(gm)
        gm.assemble(F.params(1.5, quad_points=nq), K)
        torch.cuda.synchronize()
        assert rel(K.cpu().numpy(), om.assemble(nq, 1.5)) <= 1e-10


def lu_nopivot(A):
    """Textbook right-looking elimination without row exchanges."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    for k in range(n - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


@pytest.mark.parametrize("cube", ["cube2", "cube3", "cube5", "cube6", "cube9", "cube10"])
def test_lu_matches_textbook_elimination(cube):
    # n_dof = 1, 8, 64 (one full block), 125, 512 (8 blocks), 729 (11 + a ragged 25)
    m, om, gm = mesh_pair(cube)
    n = gm.n_dof
    print(f"[case] lu n={n}", flush=True)
    rng = np.random.default_rng(n)
    A0 = rng.uniform(-1, 1, size=(n, n)) + np.diag(rng.uniform(0.5, 1.5, size=n) * n)
    A = torch.tensor(A0, device="cuda")
    assert gm.lu_factor(A) == -1
    torch.cuda.synchronize()
    want = lu_nopivot(A0)
    assert rel(A.cpu().numpy(), want) <= 1e-12
    b0 = rng.normal(size=n)
    b = torch.tensor(b0, device="cuda")
    u = torch.empty_like(b)
    gm.lu_solve(A, b, u)
    torch.cuda.synchronize()
    assert rel(u.cpu().numpy(), np.linalg.solve(A0, b0)) <= 1e-11
    gm.lu_solve(A, b, b)  # aliased right-hand side and solution
    torch.cuda.synchronize()
    assert rel(b.cpu().numpy(), u.cpu().numpy()) == 0.0


@pytest.mark.parametrize("where", [0, 67])
def test_zero_pivot_is_reported(where):
    m, om, gm = mesh_pair("cube6")  # 125 unknowns, two blocks
    n = gm.n_dof
    A0 = np.eye(n) * 2.0
    A0[where, where] = 0.0
    A = torch.tensor(A0, device="cuda")
    with pytest.raises(F.FpdeError) as e:
        gm.lu_factor(A)
    assert e.value.status == -12
    assert e.value.failed_pivot == 64 * (where // 64)


@pytest.mark.parametrize("beta", [(0.8, 0.8, 0.8), (0.6, 0.7, 0.8)])
def test_solution_matches_oracle(beta):
    m, om, gm = mesh_pair("ball_h139")
    nq = 4
    print(f"[case] solve ball_h139 beta={beta}", flush=True)
    u, _, _ = F.solve_div_problem(gm, F.div_params(beta, nq, source=F.FPDE_SRC_BALL_MMS, radius=R))
    torch.cuda.synchronize()
    _, _, uo = oracle.solve_div(om, nq, beta, R)
    ug = u.cpu().numpy()
    assert rel(ug, uo) <= 1e-9
    eg = oracle.l2_error(om, ug, lambda x: oracle.ball_exact(x, R))
    eo = oracle.l2_error(om, uo, lambda x: oracle.ball_exact(x, R))
    assert abs(eg - eo) <= 1e-9 * eo and eo < 5e-4


def test_bad_orders_and_modes_rejected():
    m, om, gm = mesh_pair("cube3")
    A = F.new_matrix(gm)
    for beta in [(0.0, 0.5, 0.5), (0.5, 1.2, 0.5), (0.5, 0.5, float("nan"))]:
        with pytest.raises(F.FpdeError) as e:
            gm.div_assemble(F.div_params(beta), A)
        assert e.value.status == -6
    with pytest.raises(F.FpdeError):
        gm.div_assemble(F.div_params((0.5, 0.5, 0.5), coef=F.FPDE_COEF_USER), A)  # pq missing
    with pytest.raises(F.FpdeError):
        gm.div_assemble(F.div_params((0.5, 0.5, 0.5), source=F.FPDE_SRC_BALL_MMS, radius=0.0), A, A[0])
