"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: element ids of every path bit-exact; derivative vectors, stiffness,
load, FP64 solution and adjoint gradients within 1e-10 (max-norm relative);
the mixed-precision solution within 1e-6 of the oracle's FP64 solution.
"""
import math

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
        m = kuhn_cube(4) if name == "cube384" else workload_mesh(name)
        print(f"[mesh] {name}: {m.n_vert} vertices, {m.n_tet} elements", flush=True)
        _MESHES[name] = (m, oracle.OracleMesh(m.xyz, m.tet), F.Mesh(m.xyz, m.tet))
    return _MESHES[name]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_mesh_numbering_matches():
    for name in ("cube384", "sphere_small"):
        m, om, gm = mesh_pair(name)
        assert gm.n_dof == om.ndof
        assert np.array_equal(gm.dof_map(), om.dof)


@pytest.mark.parametrize("name,nq", [("cube384", 4), ("cube384", 11), ("sphere_small", 11), ("sphere20k", 4),
                                     ("sphere20k", 11)])
def test_paths_bit_exact(name, nq):
    m, om, gm = mesh_pair(name)
    G = m.n_tet * nq
    ln_o, hs_o = om.paths(nq)
    ln_o = ln_o.reshape(G, 6)
    hs_o = hs_o.reshape(G, 6)
    for d in range(6):
        ln, hs, _, _ = gm.paths(nq, d, 0, G)
        assert np.array_equal(ln.cpu().numpy(), ln_o[:, d]), (name, nq, d)
        assert np.array_equal(hs.cpu().numpy().view(np.uint64), hs_o[:, d]), (name, nq, d)


def test_path_lists_and_breakpoints():
    m, om, gm = mesh_pair("sphere20k")
    nq, cap = 4, 256
    g0, count = 1000, 300
    for d in range(6):
        ln, hs, ids, rend = gm.paths(nq, d, g0, count, max_steps=cap, lists=True)
        ln = ln.cpu().numpy()
        ids = ids.cpu().numpy()
        rend = rend.cpu().numpy()
        for k in range(0, count, 7):
            h = (g0 + k) * 6 + d
            lo, _, io, ro = om.paths(nq, h, 1, lists=True)
            n = int(lo[0])
            assert ln[k] == n
            assert np.array_equal(ids[k, :n], io[0, :n])
            assert np.array_equal(rend[k, :n], ro[0, :n])  # same FP64 operations, same bits


def merged(dof, val):
    out = {}
    for d, v in zip(dof, val):
        out[int(d)] = out.get(int(d), 0.0) + float(v)
    return out


@pytest.mark.parametrize("alpha", [1.2, 1.5, 2.0])
def test_derivative_vectors(alpha):
    m, om, gm = mesh_pair("sphere20k")
    nq = 4
    g0, count = 5000, 120
    for d in range(6):
        off, dof, val = gm.ray_values(nq, alpha, d, g0, count)
        i, side = divmod(d, 2)
        for k in range(count):
            got = merged(dof[off[k]:off[k + 1]], val[off[k]:off[k + 1]])
            ids, vals = om.ray_values(nq, g0 + k, i, side, alpha)
            want = dict(zip(ids.tolist(), vals.tolist()))
            assert set(got) == set(want)
            scale = max(abs(v) for v in want.values()) if want else 1.0
            for key, v in want.items():
                assert abs(got[key] - v) <= 1e-10 * scale


CASES = [
    ("cube384", 1.5, (1.0, 1.0, 1.0), 4, "mms"),
    ("sphere_small", 1.2, (1.0, 0.5, 2.0), 11, "one"),
    ("sphere_small", 1.8, (1.0, 0.5, 2.0), 4, "one"),
    ("sphere20k", 1.5, (1.0, 0.5, 2.0), 4, "one"),
    ("sphere20k", 1.8, (1.0, 0.5, 2.0), 11, "one"),
]


def oracle_system(om, nq, alpha, K, src):
    f = None
    if src == "mms":
        x, _ = om.gauss_points(nq)
        f = oracle.mms_source(x, alpha, K)
    return om.assemble(nq, alpha, K), om.load(nq, f)


@pytest.mark.parametrize("name,alpha,K,nq,src", CASES)
def test_assembly_and_fp64_solve(name, alpha, K, nq, src):
    m, om, gm = mesh_pair(name)
    print(f"[assemble] {name} alpha={alpha} nq={nq}", flush=True)
    A_o, b_o = oracle_system(om, nq, alpha, K, src)
    u_o = oracle.solve_spd(A_o, b_o)
    source = F.FPDE_SRC_CUBE_MMS if src == "mms" else F.FPDE_SRC_ONE
    p = F.params(alpha, K, quad_points=nq, source=source)
    A = F.new_matrix(gm)
    b = torch.empty(gm.n_dof, dtype=torch.float64, device="cuda")
    gm.assemble(p, A, b)
    A_g = A.cpu().numpy()
    assert rel(A_g, A_o) <= 1e-10
    assert rel(b.cpu().numpy(), b_o) <= 1e-10
    # matrix-free product
    x = torch.tensor(np.random.default_rng(0).normal(size=gm.n_dof), device="cuda")
    y = torch.empty_like(x)
    gm.apply(p, x, y)
    assert rel(y.cpu().numpy(), A_o @ x.cpu().numpy()) <= 1e-10
    u = torch.empty_like(b)
    info = gm.solve(p, A, b, u)
    assert rel(u.cpu().numpy(), u_o) <= 1e-10
    assert info.final_rel_residual < 1e-12
    # the factor: lower triangle of A holds L with L L^T = K
    if gm.n_dof <= 400:
        Lg = np.tril(A.cpu().numpy())
        assert rel(Lg @ Lg.T, A_o) <= 1e-12


@pytest.mark.parametrize("name,alpha,nq", [("sphere_small", 1.7, 11), ("sphere20k", 1.7, 11)])
def test_mixed_precision_solve(name, alpha, nq):
    m, om, gm = mesh_pair(name)
    K = (1.0, 1.0, 1.0)
    print(f"[mixed] {name} alpha={alpha} nq={nq}", flush=True)
    A_o, b_o = oracle_system(om, nq, alpha, K, "one")
    u_o = oracle.solve_spd(A_o, b_o)
    p = F.params(alpha, K, quad_points=nq, precision=F.FPDE_MIXED, ir_tol=1e-8)
    u, A, info = F.solve_problem(gm, p)
    assert info.final_rel_residual <= 1e-8
    # the FP32 factor (split-FP16 trailing updates) is close enough to K that
    # the FP64 refinement converges at once
    assert info.ir_iters <= 2
    assert rel(u.cpu().numpy(), u_o) <= 1e-6
    # the FP32 matrix (split-FP16 tube contraction) against the oracle's FP64 one
    A32 = F.new_matrix(gm, F.FPDE_MIXED)
    gm.assemble(p, A32)
    assert rel(A32.cpu().numpy().astype(np.float64), A_o) <= 1e-6


@pytest.mark.parametrize("name", ["cube384", "sphere_small"])
def test_adjoint_matches_oracle_and_finite_differences(name):
    m, om, gm = mesh_pair(name)
    nq = 4
    alpha, K = 1.4, np.array([1.0, 1.0, 1.0])
    b_o = om.load(nq)
    rng = np.random.default_rng(40)
    u_obs = oracle.solve_spd(om.assemble(nq, 1.6, (1.2, 0.8, 1.0)), b_o) + 1e-3 * rng.normal(size=om.ndof)
    u_o = oracle.solve_spd(om.assemble(nq, alpha, K), b_o)
    ga_o, gk_o = om.gradient(nq, alpha, K, u_o, 2 * (u_o - u_obs))

    a_t = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    k_t = torch.tensor(K, dtype=torch.float64, requires_grad=True)
    u = F.FracSolve.apply(a_t, k_t, gm, nq)
    obs = torch.tensor(u_obs, device="cuda")
    J = torch.sum((u - obs) ** 2)
    J.backward()
    assert abs(a_t.grad.item() - ga_o) <= 1e-10 * abs(ga_o)
    assert rel(k_t.grad.numpy(), gk_o) <= 1e-10

    def loss(a, k):
        p = F.params(a, k, quad_points=nq)
        uu, _, _ = F.solve_problem(gm, p)
        return float(torch.sum((uu - obs) ** 2))

    h = 1e-6
    fd = (loss(alpha + h, K) - loss(alpha - h, K)) / (2 * h)
    assert abs(a_t.grad.item() - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("name,tile", [("cube_n8", 64), ("cube_n8", 7), ("sphere_small", 64), ("sphere20k", 64),
                                       ("sphere20k", 256)])
def test_template_matches_oracle(name, tile):
    if name == "cube_n8":
        m = kuhn_cube(8)
        om, gm = oracle.OracleMesh(m.xyz, m.tet), F.Mesh(m.xyz, m.tet)
    else:
        m, om, gm = mesh_pair(name)
    tiles, nnz = gm.template(tile)
    T = om.template()
    assert nnz == int(T.sum())
    assert np.array_equal(tiles, om.template_tiles(tile))


def test_template_covers_assembled_pattern():
    m, om, gm = mesh_pair("sphere20k")
    n, tile = gm.n_dof, 64
    tiles, nnz = gm.template(tile)
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    gm.assemble(F.params(1.4, (1.0, 2.0, 0.5), quad_points=11), A, None)
    nt = tiles.shape[0]
    pad = torch.zeros((nt * tile, nt * tile), dtype=torch.float64, device="cuda")
    pad[:n, :n] = A.abs()
    occupied = (pad.reshape(nt, tile, nt, tile).amax(dim=(1, 3)) > 0).cpu().numpy()
    assert not (occupied & (tiles == 0)).any()
    assert tiles.mean() < 1.0 and nnz < n * n
    with pytest.raises(F.FpdeError):
        gm.template(0)
    with pytest.raises(F.FpdeError):
        gm.template(257)


def test_error_paths_forced_from_host():
    m, om, gm = mesh_pair("sphere_small")
    A = F.new_matrix(gm)
    with pytest.raises(F.FpdeError) as e:
        gm.assemble(F.params(1.0), A)
    assert e.value.status == -6
    with pytest.raises(F.FpdeError) as e:
        gm.assemble(F.params(1.5, (1.0, -1.0, 1.0)), A)
    assert e.value.status == -6
    # a cap of two elements per half-ray is exceeded by most paths
    ln, hs, _, _ = gm.paths(4, 0, 0, 10, max_steps=64)
    assert int(ln.max()) > 2
    with pytest.raises(F.FpdeError) as e:
        gm.paths(4, 0, 0, 10, max_steps=2)
    assert e.value.status == -5
    # a matrix that is not positive definite
    n = gm.n_dof
    A = -torch.eye(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.empty_like(b)
    with pytest.raises(F.FpdeError) as e:
        gm.solve(F.params(1.5), A, b, u)
    assert e.value.status == -7
    # the handle still works afterwards
    u2, _, info = F.solve_problem(gm, F.params(1.5))
    assert info.final_rel_residual < 1e-12


def test_mesh_errors():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [-1, -1, -1]], dtype=float)
    # three elements on one face
    tet = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], dtype=np.int32)
    with pytest.raises(F.FpdeError) as e:
        F.Mesh(xyz, tet)
    assert e.value.status == -2
    flat = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=float)
    with pytest.raises(F.FpdeError) as e:
        F.Mesh(flat, np.array([[0, 1, 2, 3]], dtype=np.int32))
    assert e.value.status == -3


def test_nonconvex_meshes_are_rejected():
    """The chord bounds of Sec. 1 eq. (1) need a convex domain: the L-shaped
    prism and a cube with a 1e-9 bump or dent in one face are refused with
    FPDE_EMESH_NONCONVEX (as by the oracle); a 1e-15 move is inside the
    tolerance and accepted."""
    from fpde_inputs import notched_cube
    m = notched_cube(4)
    print(f"[nonconvex] notched cube {m.n_tet} elements", flush=True)
    with pytest.raises(F.FpdeError) as e:
        F.Mesh(m.xyz, m.tet)
    assert e.value.status == -4
    c = kuhn_cube(4)
    v = int(np.flatnonzero(np.all(np.abs(c.xyz - [0.5, 0.5, 1.0]) < 1e-14, axis=1))[0])
    for dz, ok in ((1e-9, False), (-1e-9, False), (1e-15, True), (-1e-15, True)):
        xyz = c.xyz.copy()
        xyz[v, 2] += dz
        if ok:
            assert F.Mesh(xyz, c.tet).n_dof == 27
        else:
            with pytest.raises(F.FpdeError) as e:
                F.Mesh(xyz, c.tet)
            assert e.value.status == -4
    # a handle made afterwards works
    assert F.Mesh(c.xyz, c.tet).n_dof == 27


def test_refinement_that_misses_its_tolerance_reports_enoconv():
    """FPDE_ENOCONV with the sweep count and residual filled in: one sweep
    cannot reach a relative residual of 1e-30."""
    import ctypes
    m, om, gm = mesh_pair("sphere_small")
    print("[enoconv] sphere_small mixed, ir_max_iter = 1", flush=True)
    p = F.params(1.5, quad_points=4, precision=F.FPDE_MIXED, ir_tol=1e-30, ir_max_iter=1)
    A = F.new_matrix(gm, F.FPDE_MIXED)
    b = torch.empty(gm.n_dof, dtype=torch.float64, device="cuda")
    gm.assemble(p, A, b)
    u = torch.empty_like(b)
    info = F.fpde_solve_info()
    st = F._lib().fpde_solve(gm._h, ctypes.byref(p), F._ptr(A), A.stride(0), F._ptr(b), F._ptr(u),
                             ctypes.byref(info), F._stream())
    assert st == -8
    assert info.ir_iters == 1
    assert 0.0 < info.final_rel_residual < 1e-6
    # the same factor refined to a reachable tolerance converges
    p2 = F.params(1.5, quad_points=4, precision=F.FPDE_MIXED, ir_tol=1e-8)
    info2 = gm.solve_factored(p2, A, b, u)
    assert info2.final_rel_residual <= 1e-8
