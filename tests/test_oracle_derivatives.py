"""Pins for the oracle's closed-form RL derivatives of the P1 basis (Sec. 2.1).

* Linear functions: for g(x) = c.x + d with nodal values on every vertex,
  sum_l g(z_l) D_L^gamma psi_l(x) must equal the textbook derivative of a
  linear function on [a, x] (Sec. 1 eq. def, m = 1):
      g(a) (x - a)^(-gamma) / Gamma(1 - gamma) + c_i (x - a)^(1-gamma) / Gamma(2 - gamma)
  and for the right side
      g(b) (b - x)^(-gamma) / Gamma(1 - gamma) - c_i (b - x)^(1-gamma) / Gamma(2 - gamma),
  with the chord ends a, b taken from the convex hull of the vertices (Qhull).
* The literal definition: D_L^gamma psi(x) = d/dx [I^{1-gamma} psi](x) with the
  fractional integral of eq. fcl evaluated exactly piece by piece in 40-digit
  arithmetic (break points from brute-force plane crossings, psi from
  brute-force point location) and differentiated numerically in x.
* gamma = 1 (alpha = 2): the derivative is the own-element slope.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.spatial import ConvexHull
from scipy.special import rgamma

import oracle
from fpde_inputs import kuhn_cube, workload_mesh


def chord(hull, u0, d):
    n, off = hull.equations[:, :3], hull.equations[:, 3]
    nd = n @ d
    return float((-(n @ u0 + off)[nd > 0] / nd[nd > 0]).min())


@pytest.mark.parametrize("name", ["cube3", "sphere_small"])
@pytest.mark.parametrize("alpha", [0.8, 1.2, 1.5, 1.9])
def test_linear_function_reproduced(name, alpha):
    m = kuhn_cube(3) if name == "cube3" else workload_mesh(name)
    om = oracle.OracleMesh(m.xyz, m.tet)
    hull = ConvexHull(m.xyz)
    x, _ = om.gauss_points(4)
    gm = alpha / 2
    rng = np.random.default_rng(3)
    c = rng.normal(size=3)
    d0 = rng.normal()
    gz = m.xyz @ c + d0
    for g in rng.choice(len(x), size=40, replace=False):
        for i in range(3):
            for side in (0, 1):
                ids, vals = om.ray_values(4, int(g), i, side, alpha, mode=1)
                got = float(np.sum(gz[ids] * vals))
                e = np.zeros(3)
                e[i] = 1.0 if side else -1.0
                r = chord(hull, x[g], e)
                p_end = x[g] + r * e
                gend = float(p_end @ c + d0)
                sgn = -1.0 if side else 1.0
                want = gend * r ** (-gm) * rgamma(1 - gm) + sgn * c[i] * r ** (1 - gm) * rgamma(2 - gm)
                assert abs(got - want) <= 1e-12 * (abs(want) + abs(gend) + abs(c[i])), (g, i, side)


def brute_pieces(xyz, tet, u0, i, side, r_end):
    """Break points of the ray where it crosses any face plane of any element
    (brute force), and psi_l at both ends of every piece by point location."""
    e = np.zeros(3)
    e[i] = 1.0 if side else -1.0
    ts = {0.0, r_end}
    P = xyz[tet]
    for f in [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]:
        a, b, c = P[:, f[0]], P[:, f[1]], P[:, f[2]]
        n = np.cross(b - a, c - a)
        nd = n @ e
        ok = np.abs(nd) > 1e-300
        r = np.einsum("ij,ij->i", n[ok], a[ok] - u0) / nd[ok]
        for rr in r[(r > 0) & (r < r_end)]:
            ts.add(float(rr))
    ts = sorted(ts)
    merged = [ts[0]]
    for t in ts[1:]:
        if t - merged[-1] > 1e-11:
            merged.append(t)
    merged[-1] = r_end
    T = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    Tinv = np.linalg.inv(T)

    def locate(p):
        lam = np.einsum("tij,tj->ti", Tinv, p - P[:, 0])
        lam = np.concatenate([1 - lam.sum(1, keepdims=True), lam], 1)
        t = int(np.argmax(lam.min(1)))
        assert lam[t].min() > -1e-9
        return t, lam[t]

    pieces = []
    for r0, r1 in zip(merged[:-1], merged[1:]):
        vals = []
        for frac in (0.25, 0.75):
            t, lam = locate(u0 + (r0 + frac * (r1 - r0)) * e)
            vals.append({int(tet[t, j]): lam[j] for j in range(4)})
        pieces.append((r0, r1, vals))
    return pieces


def literal_derivative(pieces, node, gamma, dps=40):
    """D^gamma psi_node at the ray origin from the literal definition.

    Along the ray r (distance from x), psi is linear on each piece.  With the
    origin moved by h along the ray direction, the fractional integral of
    eq. fcl / fcr is F(h) = (1/Gamma(1-g)) int_{pieces} (r - h)^(-g) psi(r) dr
    over r in [h, r_end]; D_L = -dF/dh for the left ray (x moves away from a as
    h decreases) and D_R = -dF/dh for the right ray (eq. def carries (-1)^m).
    Both reduce to -dF/dh in the ray coordinate.
    """
    mp.mp.dps = dps
    g = mp.mpf(gamma)

    def lin(piece):
        r0, r1, vals = piece
        v25 = mp.mpf(vals[0].get(node, 0.0))
        v75 = mp.mpf(vals[1].get(node, 0.0))
        slope = (v75 - v25) / (mp.mpf(0.5) * (mp.mpf(r1) - mp.mpf(r0)))
        at0 = v25 - slope * mp.mpf(0.25) * (mp.mpf(r1) - mp.mpf(r0))
        return mp.mpf(r0), mp.mpf(r1), at0, slope

    parts = [lin(p) for p in pieces]

    def F(h):
        tot = mp.mpf(0)
        for k, (r0, r1, at0, slope) in enumerate(parts):
            # the first piece (own element) extends linearly past the origin
            lo = h if k == 0 else max(r0, h)
            if r1 <= lo:
                continue
            # psi(r) = at0 + slope (r - r0) = A + B (r - h), with s = r - h
            B = slope
            A = at0 + slope * (h - r0)
            s0, s1 = lo - h, r1 - h
            I0 = (s1 ** (1 - g) - (s0 ** (1 - g) if s0 > 0 else 0)) / (1 - g)
            I1 = (s1 ** (2 - g) - (s0 ** (2 - g) if s0 > 0 else 0)) / (2 - g)
            tot += A * I0 + B * I1
        return tot / mp.gamma(1 - g)

    return float(-mp.diff(F, mp.mpf(0)))


@pytest.mark.parametrize("alpha", [0.6, 1.3, 1.7])
def test_literal_definition_on_tiny_mesh(alpha):
    m = kuhn_cube(2)
    om = oracle.OracleMesh(m.xyz, m.tet)
    hull = ConvexHull(m.xyz)
    x, _ = om.gauss_points(4)
    rng = np.random.default_rng(5)
    checked = 0
    for g in rng.choice(len(x), size=6, replace=False):
        for i in range(3):
            for side in (0, 1):
                e = np.zeros(3)
                e[i] = 1.0 if side else -1.0
                r_end = chord(hull, x[g], e)
                pieces = brute_pieces(m.xyz, m.tet, x[g], i, side, r_end)
                ids, vals = om.ray_values(4, int(g), i, side, alpha, mode=1)
                scale = np.abs(vals).max()
                for node, v in zip(ids, vals):
                    want = literal_derivative(pieces, int(node), alpha / 2)
                    assert abs(v - want) <= 1e-10 * scale, (g, i, side, node, v, want)
                    checked += 1
    assert checked > 100


def test_order_one_limit_is_own_element_slope():
    m = workload_mesh("sphere_tiny")
    om = oracle.OracleMesh(m.xyz, m.tet)
    M, _ = om.affine()
    dof = om.dof
    for g in range(0, om.n_tet * 4, 37):
        t = g // 4
        grads = np.vstack([-M[t].sum(0), M[t]])  # gradients of k_0..k_3
        for i in range(3):
            for side in (0, 1):
                ids, vals = om.ray_values(4, g, i, side, 2.0)
                want = {}
                for j in range(4):
                    d = dof[m.tet[t, j]]
                    if d >= 0:
                        want[d] = (grads[j, i] if side == 0 else -grads[j, i])
                got = {int(a): b for a, b in zip(ids, vals) if abs(b) > 1e-13}
                assert set(got) <= set(want)
                for d, v in want.items():
                    assert abs(got.get(d, 0.0) - v) < 1e-12 * max(1.0, abs(v))


def test_alpha_derivative_matches_finite_difference():
    m = workload_mesh("sphere_tiny")
    om = oracle.OracleMesh(m.xyz, m.tet)
    a, h = 1.45, 1e-6
    for g in (3, 50, 111):
        for i in range(3):
            for side in (0, 1):
                ids, dv = om.ray_values(4, g, i, side, a, mode=2)
                i1, vp = om.ray_values(4, g, i, side, a + h)
                i2, vm = om.ray_values(4, g, i, side, a - h)
                assert list(ids) == list(i1) == list(i2)
                fd = (vp - vm) / (2 * h)
                assert np.abs(dv - fd).max() <= 1e-7 * max(1.0, np.abs(dv).max())
