"""Pins for the oracle's two-dimensional variant (n = 2: triangles, paths
along +-e_1, +-e_2; Sec. 1 with n = 2, Fig. 1a; Sec. 2.2 with area
coordinates).

* Paths: the walked triangles and break points equal an exhaustive clipping
  of the ray against every triangle (edge half-planes from the vertex
  coordinates), and the path ends on the convex hull (Qhull).
* Linear functions are reproduced by the derivative vectors with the
  end-point term: sum_l g(z_l) D_L^gamma psi_l(x) equals the textbook
  derivative of a linear function on the chord.
* alpha = 2: K equals the classical anisotropic P1 stiffness; K is
  symmetric positive definite.
* f = 1: b_j = |patch(j)| / 3.
* Manufactured solution phi(x) phi(y) on the unit square: L2 order near 2.
"""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull
from scipy.special import rgamma

import oracle
from fpde_inputs import kuhn_square, workload_mesh


def mesh2(name):
    if name.startswith("square"):
        m = kuhn_square(int(name[6:]))
    else:
        m = workload_mesh(name)
    return m, oracle.OracleMesh2D(m.xyz, m.tet)


def chord2(hull, u0, d):
    n, off = hull.equations[:, :2], hull.equations[:, 2]
    nd = n @ d
    return float((-(n @ u0 + off)[nd > 0] / nd[nd > 0]).min())


@pytest.mark.parametrize("name", ["square5", "disk_small"])
def test_walk_equals_exhaustive_clipping(name):
    m, om = mesh2(name)
    hull = ConvexHull(m.xyz)
    x, _ = om.gauss_points(3)
    rng = np.random.default_rng(21)
    for g in rng.choice(len(x), size=40, replace=False):
        for i in range(2):
            for s in (-1, 1):
                ids, rend = om.walk(int(g) // 3, x[g], i, s)
                d = np.zeros(2)
                d[i] = s
                lo, hi = om.exhaustive(x[g], d)
                r_end = chord2(hull, x[g], d)
                assert abs(rend[-1] - r_end) <= 1e-12 * max(1.0, r_end)
                seg = (hi > np.maximum(lo, 0.0) + 1e-12) & (hi > 1e-14)
                assert set(ids.tolist()) == set(np.nonzero(seg)[0].tolist()), (g, i, s)
                assert np.allclose(np.sort(rend), np.sort(hi[ids]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("alpha", [0.8, 1.3, 1.9])
def test_linear_function_reproduced(alpha):
    m, om = mesh2("disk_small")
    hull = ConvexHull(m.xyz)
    x, _ = om.gauss_points(7)
    gm = alpha / 2
    rng = np.random.default_rng(22)
    c = rng.normal(size=2)
    d0 = rng.normal()
    gz = m.xyz @ c + d0
    for g in rng.choice(len(x), size=40, replace=False):
        for i in range(2):
            for side in (0, 1):
                ids, vals = om.ray_values(7, int(g), i, side, alpha, mode=1)
                got = float(np.sum(gz[ids] * vals))
                e = np.zeros(2)
                e[i] = 1.0 if side else -1.0
                r = chord2(hull, x[g], e)
                gend = float((x[g] + r * e) @ c + d0)
                sgn = -1.0 if side else 1.0
                want = gend * r ** (-gm) * rgamma(1 - gm) + sgn * c[i] * r ** (1 - gm) * rgamma(2 - gm)
                assert abs(got - want) <= 1e-12 * (abs(want) + abs(gend) + abs(c[i])), (g, i, side)


def classical_stiffness2d(xy, tri, dof, ndof, K):
    A = np.zeros((ndof, ndof))
    for t in tri:
        P = xy[t]
        C = np.linalg.inv(np.hstack([np.ones((3, 1)), P]))
        grads = C[1:, :].T
        area = abs(np.linalg.det(P[1:] - P[0])) / 2.0
        Ke = area * grads @ np.diag(K) @ grads.T
        for a in range(3):
            for b in range(3):
                da, db = dof[t[a]], dof[t[b]]
                if da >= 0 and db >= 0:
                    A[da, db] += Ke[a, b]
    return A


@pytest.mark.parametrize("name", ["square5", "disk_small"])
def test_order_two_is_classical_stiffness(name):
    m, om = mesh2(name)
    K = (1.0, 0.4)
    for nq in (3, 7):
        A = om.assemble(nq, 2.0, K)
        S = classical_stiffness2d(m.xyz, m.tet, om.dof, om.ndof, K)
        assert np.abs(A - S).max() <= 1e-13 * np.abs(S).max()


def test_symmetric_positive_definite_and_load():
    m, om = mesh2("disk_small")
    A = om.assemble(7, 1.4, (1.0, 2.0))
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
    b = om.load(3)
    _, area = om.affine()
    dof = om.dof
    want = np.zeros(om.ndof)
    for t, tri in enumerate(m.tet):
        for v in tri:
            if dof[v] >= 0:
                want[dof[v]] += area[t] / 3.0
    assert np.abs(b - want).max() <= 1e-15 * np.abs(want).max()


@pytest.mark.slow
@pytest.mark.parametrize("alpha", [1.4, 1.8])
def test_manufactured_solution_order(alpha):
    errs, hs = [], []
    for n in (8, 16, 32):
        m, om = mesh2(f"square{n}")
        x, _ = om.gauss_points(7)
        A = om.assemble(7, alpha)
        b = om.load(7, oracle.mms_source2d(x, alpha))
        u = oracle.solve_spd(A, b)
        errs.append(oracle.l2_error2d(om, u, oracle.mms_exact2d))
        hs.append(1.0 / n)
    orders = [math.log(errs[k] / errs[k + 1]) / math.log(2.0) for k in range(2)]
    assert all(1.7 <= o <= 2.4 for o in orders), (errs, orders)
