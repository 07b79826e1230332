"""Batched FP64 dense solves (several systems, one launch sequence) through
the C ABI.

* Every system of a batch gets bit-for-bit the factor and solution that the
  single-system solve gives (the same kernels and order of operations).
* The solutions equal the FP64 CPU oracle's (dense assembly + Cholesky)
  within 1e-10, max-norm relative.
* A system that is not positive definite is reported for itself alone; the
  sizes cover one partial block (n < 64), several blocks with a ragged
  tail, the look-ahead factorization (n = 17 576) and the largest batch (16).
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
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def systems(gm, cases):
    n = gm.n_dof
    A = torch.empty((len(cases), n, n), dtype=torch.float64, device="cuda")
    b = torch.empty((len(cases), n), dtype=torch.float64, device="cuda")
    for z, (alpha, nq) in enumerate(cases):
        gm.assemble(F.params(alpha, (1.0, 0.5, 2.0), quad_points=nq), A[z], b[z])
    return A, b


@pytest.mark.parametrize("name,cases", [
    ("cube8", [(1.2, 4), (1.5, 4), (1.8, 11)]),
    ("sphere_small", [(1.3, 4), (1.6, 11)]),
    ("sphere20k", [(1.2, 4), (1.5, 4), (1.8, 4), (1.2, 11), (1.5, 11), (1.8, 11)]),
    # 17 576 unknowns: the factorization looks ahead (side-stream trailing
    # updates) with two systems at once
    ("cube27", [(1.3, 4), (1.6, 4)]),
])
def test_batch_equals_single_and_oracle(name, cases):
    print(f"[case] batch {name} {cases}", flush=True)
    m, om, gm = mesh_pair(name)
    A, b = systems(gm, cases)
    A1, b1 = A.clone(), b.clone()
    u = torch.empty_like(b)
    gm.solve_batch(A, b, u)
    torch.cuda.synchronize()
    for z, (alpha, nq) in enumerate(cases):
        us = torch.empty_like(b1[z])
        gm.solve(F.params(alpha, (1.0, 0.5, 2.0), quad_points=nq), A1[z], b1[z], us, info=False)
        torch.cuda.synchronize()
        assert torch.equal(torch.tril(A[z]), torch.tril(A1[z])), (name, z)
        assert torch.equal(u[z], us), (name, z)
    if gm.n_dof <= 1200:
        for z, (alpha, nq) in enumerate(cases[:2]):
            Ko = om.assemble(nq, alpha, (1.0, 0.5, 2.0))
            uo = oracle.solve_spd(Ko, om.load(nq))
            assert rel(u[z].cpu().numpy(), uo) <= 1e-10, (name, z)


def test_batch_reports_the_failing_system_only():
    m, om, gm = mesh_pair("cube8")
    A, b = systems(gm, [(1.5, 4)] * 4)
    A[2, 70, 70] = -1.0  # block starting at column 64 has a negative pivot
    u = torch.empty_like(b)
    with pytest.raises(F.FpdeError) as e:
        gm.solve_batch(A, b, u)
    assert e.value.status == -7
    assert e.value.failed_pivot == [-1, -1, 64, -1]
    # the handle is usable afterwards
    A, b = systems(gm, [(1.5, 4)] * 2)
    gm.solve_batch(A, b, b)  # in place
    torch.cuda.synchronize()
    assert torch.isfinite(b).all()


def test_batch_sixteen_small_systems_in_place():
    m, om, gm = mesh_pair("cube3")  # 8 unknowns: one partial block
    cases = [(1.1 + 0.05 * z, 4 if z % 2 == 0 else 11) for z in range(16)]
    A, b = systems(gm, cases)
    want = []
    for z, (alpha, nq) in enumerate(cases):
        Ko = om.assemble(nq, alpha, (1.0, 0.5, 2.0))
        want.append(oracle.solve_spd(Ko, om.load(nq)))
    gm.solve_batch(A, b, b)
    torch.cuda.synchronize()
    for z in range(16):
        assert rel(b[z].cpu().numpy(), want[z]) <= 1e-10, z


def test_batch_rejects():
    m, om, gm = mesh_pair("cube3")
    n = gm.n_dof
    lib = F._lib()
    A = torch.eye(n, dtype=torch.float64, device="cuda").repeat(17, 1, 1)
    b = torch.ones((17, n), dtype=torch.float64, device="cuda")
    h, s = gm._h, F._stream()
    for count, sa, sv in ((0, n * n, n), (17, n * n, n), (2, n * n - 1, n), (2, n * n, n - 1)):
        st = lib.fpde_solve_batch(h, count, F._ptr(A), n, sa, F._ptr(b), F._ptr(b), sv, None, s)
        assert st == -1, (count, sa, sv)
    st = lib.fpde_solve_batch(h, 2, None, n, n * n, F._ptr(b), F._ptr(b), n, None, s)
    assert st == -1


@pytest.mark.parametrize("name", ["cube8", "sphere20k"])
def test_assemble_batch_equals_single(name):
    """fpde_assemble_batch gives each system the matrix and load of fpde_assemble
    (to the rounding of the LDS accumulation order)."""
    print(f"[case] assemble_batch {name}", flush=True)
    m, om, gm = mesh_pair(name)
    cases = [(1.2, 4), (1.5, 11), (1.8, 4), (1.3, 11)]
    ps = [F.params(a, (1.0, 0.5, 2.0), quad_points=nq) for a, nq in cases]
    n = gm.n_dof
    A = torch.empty((len(cases), n, n), dtype=torch.float64, device="cuda")
    b = torch.empty((len(cases), n), dtype=torch.float64, device="cuda")
    gm.assemble_batch(ps, A, b)
    A1, b1 = systems(gm, cases)
    torch.cuda.synchronize()
    for z in range(len(cases)):
        assert rel(A[z].cpu().numpy(), A1[z].cpu().numpy()) <= 1e-13, z
        assert rel(b[z].cpu().numpy(), b1[z].cpu().numpy()) <= 1e-14, z


def test_assemble_batch_rejects():
    m, om, gm = mesh_pair("cube3")
    n = gm.n_dof
    lib = F._lib()
    A = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    h, s = gm._h, F._stream()
    mixed = (F.fpde_params * 2)(F.params(1.5), F.params(1.5, precision=F.FPDE_MIXED))
    assert lib.fpde_assemble_batch(h, 2, mixed, F._ptr(A), n, n * n, None, 0, s) == -1
    user = (F.fpde_params * 1)(F.params(1.5, source=F.FPDE_SRC_USER))
    assert lib.fpde_assemble_batch(h, 1, user, F._ptr(A), n, n * n, None, 0, s) == -1
    ok = (F.fpde_params * 2)(F.params(1.5), F.params(1.6))
    assert lib.fpde_assemble_batch(h, 0, ok, F._ptr(A), n, n * n, None, 0, s) == -1
    assert lib.fpde_assemble_batch(h, 2, ok, F._ptr(A), n, n * n - 1, None, 0, s) == -1


def test_assemble_batch_fp32_and_single_rule():
    """FP32 matrices (the mixed arm) and a batch whose systems all use one rule
    (every walk waits for the previous accumulation of the same plan)."""
    m, om, gm = mesh_pair("sphere_small")
    n = gm.n_dof
    cases = [(1.2, 11), (1.5, 11), (1.8, 11)]
    ps = [F.params(a, (1.0, 0.5, 2.0), quad_points=nq, precision=F.FPDE_MIXED) for a, nq in cases]
    A = torch.empty((3, n, n), dtype=torch.float32, device="cuda")
    b = torch.empty((3, n), dtype=torch.float64, device="cuda")
    gm.assemble_batch(ps, A, b)
    for z, p in enumerate(ps):
        A1 = torch.empty((n, n), dtype=torch.float32, device="cuda")
        b1 = torch.empty(n, dtype=torch.float64, device="cuda")
        gm.assemble(p, A1, b1)
        torch.cuda.synchronize()
        assert rel(A[z].cpu().numpy(), A1.cpu().numpy()) <= 1e-6, z
        assert rel(b[z].cpu().numpy(), b1.cpu().numpy()) <= 1e-14, z
    ps64 = [F.params(a, (1.0, 0.5, 2.0), quad_points=nq) for a, nq in cases]
    A64 = torch.empty((3, n, n), dtype=torch.float64, device="cuda")
    gm.assemble_batch(ps64, A64, None)
    torch.cuda.synchronize()
    for z, (a, nq) in enumerate(cases):
        assert rel(A64[z].cpu().numpy(), om.assemble(nq, a, (1.0, 0.5, 2.0))) <= 1e-10, z


def test_timing_chosen_stages_only():
    # fpde_timing_stages: only the chosen stages record intervals (the batch
    # assembly's accumulations here); stopping keeps what was recorded
    m, om, gm = mesh_pair("cube4")
    n = gm.n_dof
    cases = [(4, 1.3), (11, 1.6), (4, 1.7)]
    params = [F.params(a, (1.0, 0.5, 2.0), quad_points=nq) for nq, a in cases]
    A = torch.empty((len(cases), n, n), dtype=torch.float64, device="cuda")
    b = torch.empty((len(cases), n), dtype=torch.float64, device="cuda")
    print("[case] timing accum only, cube4", flush=True)
    gm.timing(True, stages=["accum"])
    gm.assemble_batch(params, A, b)
    torch.cuda.synchronize()
    gm.timing(False)
    st = gm.stage_times()
    assert st["accum"][1] == len(cases) and st["accum"][0] > 0.0
    assert all(c == 0 for k, (t, c) in st.items() if k != "accum")
    gm.timing(True)
    gm.assemble_batch(params, A, b)
    torch.cuda.synchronize()
    gm.timing(False)
    st = gm.stage_times()
    assert st["accum"][1] == len(cases) and st["walk"][1] >= 1 and st["contract"][1] == len(cases)
