"""Sparse storage on the template of Sec. 2.3 and the conjugate-gradient
solve, through the C ABI, against the FP64 CPU oracle.

* The template as CSR equals the oracle's template (bit-exact pattern).
* K assembled on that pattern equals the oracle's dense K at every stored
  entry (1e-10, max-norm relative), and the oracle's K has no nonzero off
  the pattern; the CSR product equals K x.
* CG (Jacobi) on the CSR matrix and on the matrix-free operator reaches the
  oracle's dense (LAPACK Cholesky) solution within 1e-8, with the true
  residual b - K u at the requested tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_03339_amd as F
from fpde_inputs import kuhn_cube, workload_mesh

pytestmark = pytest.mark.gpu

_MESHES = {}


def mesh_pair(name):
    if name not in _MESHES:
        m = kuhn_cube(int(name[4:])) if name.startswith("cube") else workload_mesh(name)
        print(f"[mesh] {name}: {m.n_vert} vertices, {m.n_tet} elements", flush=True)
        _MESHES[name] = (m, oracle.OracleMesh(m.xyz, m.tet), F.Mesh(m.xyz, m.tet))
    return _MESHES[name]


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("name", ["cube3", "cube8", "sphere_small", "sphere20k"])
def test_template_csr_matches_oracle(name):
    m, om, gm = mesh_pair(name)
    rp, col = gm.template_csr()
    T = om.template()
    rows, cols = np.nonzero(T)  # row-major order, columns increasing
    want_rp = np.concatenate([[0], np.cumsum(T.sum(axis=1))])
    assert np.array_equal(rp.cpu().numpy(), want_rp)
    assert np.array_equal(col.cpu().numpy(), cols.astype(np.int32))
    assert all(T[j, j] for j in range(om.ndof))


@pytest.mark.parametrize("name,alpha,nq", [("cube8", 1.5, 4), ("sphere_small", 1.3, 11), ("sphere20k", 1.7, 4)])
def test_csr_assembly_and_product(name, alpha, nq):
    print(f"[case] csr {name} alpha={alpha} nq={nq}", flush=True)
    m, om, gm = mesh_pair(name)
    K = (1.0, 0.5, 2.0)
    p = F.params(alpha, K, quad_points=nq)
    rp, col = gm.template_csr()
    val = torch.empty(col.numel(), dtype=torch.float64, device="cuda")
    b = torch.empty(gm.n_dof, dtype=torch.float64, device="cuda")
    gm.assemble_csr(p, rp, col, val, b)
    torch.cuda.synchronize()
    Ko = om.assemble(nq, alpha, K)
    rpn, cn = rp.cpu().numpy(), col.cpu().numpy()
    rows = np.repeat(np.arange(gm.n_dof), np.diff(rpn))
    assert rel(val.cpu().numpy(), Ko[rows, cn]) <= 1e-10
    off = np.ones_like(Ko, dtype=bool)
    off[rows, cn] = False
    assert np.abs(Ko[off]).max(initial=0.0) == 0.0  # nothing dropped
    assert rel(b.cpu().numpy(), om.load(nq)) <= 1e-10
    x = np.random.default_rng(7).normal(size=gm.n_dof)
    y = torch.empty_like(b)
    gm.csr_apply(rp, col, val, torch.tensor(x, device="cuda"), y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), Ko @ x) <= 1e-10


@pytest.mark.parametrize("name,alpha,nq", [("cube8", 1.5, 4), ("sphere20k", 1.4, 11)])
def test_cg_csr_and_matrix_free(name, alpha, nq):
    print(f"[case] cg {name} alpha={alpha} nq={nq}", flush=True)
    m, om, gm = mesh_pair(name)
    K = (1.0, 1.0, 1.0)
    p = F.params(alpha, K, quad_points=nq)
    rp, col = gm.template_csr()
    val = torch.empty(col.numel(), dtype=torch.float64, device="cuda")
    b = torch.empty(gm.n_dof, dtype=torch.float64, device="cuda")
    gm.assemble_csr(p, rp, col, val, b)
    Ko = om.assemble(nq, alpha, K)
    uo = oracle.solve_spd(Ko, b.cpu().numpy())
    for csr in ((rp, col, val), None):
        u = torch.empty_like(b)
        info = gm.cg_solve(p, b, u, csr=csr, tol=1e-12)
        torch.cuda.synchronize()
        assert info.ir_iters > 0
        assert info.final_rel_residual <= 1e-11
        assert rel(u.cpu().numpy(), uo) <= 1e-8, ("csr" if csr else "matrix-free", info.ir_iters)


def test_cg_rejects_aliased_vectors_and_reports_no_convergence():
    m, om, gm = mesh_pair("cube8")
    p = F.params(1.5)
    b = torch.ones(gm.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FpdeError) as e:
        gm.cg_solve(p, b, b)
    assert e.value.status == -1
    u = torch.empty_like(b)
    with pytest.raises(F.FpdeError) as e:
        gm.cg_solve(p, b, u, tol=1e-14, max_iter=2)
    assert e.value.status == -8
