"""fpde_solve_noalloc (for callers that cannot allocate) against fpde_solve:
the same FP64 Cholesky factor and solution, on two calls in a row with the
second on a smaller system (the static scratch keeps the first call's
contents), both against the oracle (LAPACK Cholesky of the oracle's matrix)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_03339_amd as F
from fpde_inputs import kuhn_cube, workload_mesh

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def one(name, m, alpha, nq):
    print(f"[noalloc] {name} alpha={alpha} nq={nq}", flush=True)
    gm = F.Mesh(m.xyz, m.tet)
    om = oracle.OracleMesh(m.xyz, m.tet)
    n = gm.n_dof
    p = F.params(alpha, (1.0, 0.5, 2.0), quad_points=nq)
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    gm.assemble(p, A, b)
    A2 = A.clone()
    u_ref = torch.empty_like(b)
    gm.solve(p, A, b, u_ref, info=False)
    u = torch.empty_like(b)
    gm.solve_noalloc(A2, b, u)
    torch.cuda.synchronize()
    # same kernels on the same input: the same factor and solution
    assert torch.equal(torch.tril(A2), torch.tril(A))
    assert rel(u.cpu().numpy(), u_ref.cpu().numpy()) <= 1e-10
    u_o = oracle.solve_spd(om.assemble(nq, alpha, (1.0, 0.5, 2.0)), om.load(nq))
    assert rel(u.cpu().numpy(), u_o) <= 1e-10
    return gm


def test_noalloc_solve_twice_second_smaller():
    g1 = one("sphere20k", workload_mesh("sphere20k"), 1.5, 4)
    assert g1.n_dof > 3000
    g2 = one("cube384", kuhn_cube(4), 1.3, 11)
    assert g2.n_dof == 27


def test_noalloc_rejects_what_it_cannot_hold():
    m = kuhn_cube(4)
    gm = F.Mesh(m.xyz, m.tet)
    n = gm.n_dof
    A = -torch.eye(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.empty_like(b)
    with pytest.raises(F.FpdeError) as e:
        gm.solve_noalloc(A, b, u)
    assert e.value.status == -7 and e.value.failed_pivot == 0
    gm.timing(True)
    with pytest.raises(F.FpdeError) as e:
        gm.solve_noalloc(torch.eye(n, dtype=torch.float64, device="cuda"), b, u)
    assert e.value.status == -1
    gm.timing(False)
    # a well-posed call still works after the failures
    B = torch.eye(n, dtype=torch.float64, device="cuda") * 4.0
    gm.solve_noalloc(B, b, u)
    assert torch.allclose(u, b / 4.0, rtol=0, atol=1e-15)
