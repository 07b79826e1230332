"""Parity of the two-dimensional variant on the GPU with the FP64 CPU oracle,
through the C ABI.

Bars: element ids of every half-ray bit-exact (structured square, Delaunay
disks, both rules); K, b and the FP64 solution within 1e-10 (max-norm
relative); the manufactured-solution error on the square equal to the
oracle's.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_03339_amd as F
from fpde_inputs import kuhn_square, workload_mesh

pytestmark = pytest.mark.gpu

_MESHES = {}


def mesh_pair(name):
    if name not in _MESHES:
        m = kuhn_square(int(name[6:])) if name.startswith("square") else workload_mesh(name)
        print(f"[mesh2d] {name}: {m.n_vert} vertices, {m.n_tet} triangles", flush=True)
        _MESHES[name] = (m, oracle.OracleMesh2D(m.xyz, m.tet), F.Mesh2D(m.xyz, m.tet))
    return _MESHES[name]


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("name", ["square8", "disk_small", "disk4k"])
def test_numbering(name):
    m, om, gm = mesh_pair(name)
    assert gm.n_dof == om.ndof
    assert np.array_equal(gm.dof_map(), om.dof)


@pytest.mark.parametrize("name,nq", [("square8", 3), ("square8", 7), ("disk_small", 7), ("disk4k", 3),
                                     ("disk4k", 7)])
def test_paths_bit_exact(name, nq):
    m, om, gm = mesh_pair(name)
    G = m.n_tet * nq
    ln_o, hs_o = om.paths(nq)
    ln_o, hs_o = ln_o.reshape(G, 4), hs_o.reshape(G, 4)
    for d in range(4):
        ln, hs, _, _ = gm.paths(nq, d, 0, G)
        assert np.array_equal(ln.cpu().numpy(), ln_o[:, d]), (name, nq, d)
        assert np.array_equal(hs.cpu().numpy().view(np.uint64), hs_o[:, d]), (name, nq, d)


def test_break_points_bit_equal():
    m, om, gm = mesh_pair("disk4k")
    nq, cap, g0, count = 7, 256, 500, 200
    ln_o, _, ids_o, rend_o = oracle.OracleMesh2D(m.xyz, m.tet, cap=cap).paths(nq, 4 * g0, 4 * count, lists=True)
    for d in range(4):
        ln, _, ids, rend = gm.paths(nq, d, g0, count, max_steps=cap, lists=True)
        ln, ids, rend = ln.cpu().numpy(), ids.cpu().numpy(), rend.cpu().numpy()
        for k in range(count):
            n = ln[k]
            assert np.array_equal(ids[k, :n], ids_o[4 * k + d, :n])
            assert np.array_equal(rend[k, :n], rend_o[4 * k + d, :n])


@pytest.mark.parametrize("name,alpha,K,nq,src", [("square8", 1.5, (1.0, 1.0), 7, "mms"),
                                                 ("disk_small", 1.3, (1.0, 0.4), 3, "one"),
                                                 ("disk4k", 1.7, (2.0, 1.0), 7, "one")])
def test_assembly_and_solve(name, alpha, K, nq, src):
    print(f"[case] 2d {name} alpha={alpha} nq={nq}", flush=True)
    m, om, gm = mesh_pair(name)
    p = F.params2d(alpha, K, nq, source=F.FPDE_SRC_SQUARE_MMS if src == "mms" else F.FPDE_SRC_ONE)
    n = gm.n_dof
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    gm.assemble(p, A, b)
    torch.cuda.synchronize()
    Ao = om.assemble(nq, alpha, K)
    x, _ = om.gauss_points(nq)
    bo = om.load(nq, oracle.mms_source2d(x, alpha, K) if src == "mms" else None)
    assert rel(A.cpu().numpy(), Ao) <= 1e-10
    assert rel(b.cpu().numpy(), bo) <= 1e-10
    u = torch.empty_like(b)
    gm.solve(A, b, u)
    torch.cuda.synchronize()
    uo = oracle.solve_spd(Ao, bo)
    assert rel(u.cpu().numpy(), uo) <= 1e-10
    if src == "mms":
        eg = oracle.l2_error2d(om, u.cpu().numpy(), oracle.mms_exact2d)
        eo = oracle.l2_error2d(om, uo, oracle.mms_exact2d)
        assert abs(eg - eo) <= 1e-9 * eo


def test_bad_parameters_rejected():
    m, om, gm = mesh_pair("square8")
    n = gm.n_dof
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    for p in (F.params2d(0.9), F.params2d(1.5, (1.0, 0.0)), F.params2d(1.5, quad_points=4)):
        with pytest.raises(F.FpdeError):
            gm.assemble(p, A)
