"""Pins for the oracle's quadrature rules and Gauss points (Sec. 2.1, (K_E)_kl).

A rule with weights summing to 1 is exact for a monomial x^a y^b z^c on the
reference tetrahedron when sum_q w_q x^a y^b z^c = 6 a! b! c! / (a+b+c+3)!
(the classical Dirichlet integral; the reference volume is 1/6).
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle
from fpde_inputs import kuhn_cube, workload_mesh


def exact_moment(a, b, c):
    return Fraction(6 * factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))


def max_defect(nq, degree):
    bary, w = oracle.quadrature(nq)
    worst = 0.0
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            for c in range(degree + 1 - a - b):
                q = float(np.sum(w * bary[:, 1] ** a * bary[:, 2] ** b * bary[:, 3] ** c))
                worst = max(worst, abs(q - float(exact_moment(a, b, c))))
    return worst


@pytest.mark.parametrize("nq,degree", [(1, 1), (4, 2), (11, 4)])
def test_rule_exact_to_its_degree(nq, degree):
    assert max_defect(nq, degree) < 2e-16 * 10


@pytest.mark.parametrize("nq,degree", [(1, 2), (4, 3), (11, 5)])
def test_rule_not_exact_beyond_its_degree(nq, degree):
    # the moment check is discriminating: one degree more must fail
    assert max_defect(nq, degree) > 1e-6


def test_eleven_point_rule_has_negative_centroid_weight():
    bary, w = oracle.quadrature(11)
    assert np.allclose(bary[0], 0.25) and w[0] < 0
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(bary > 0) and np.allclose(bary.sum(1), 1.0, atol=1e-15)


@pytest.mark.parametrize("nq", [4, 11])
def test_gauss_weights_sum_to_domain_volume(nq):
    m = kuhn_cube(3)
    om = oracle.OracleMesh(m.xyz, m.tet)
    x, w = om.gauss_points(nq)
    assert abs(w.sum() - 1.0) < 1e-13
    # every Gauss point strictly inside its own element
    t = np.repeat(np.arange(m.n_tet), nq)
    P = m.xyz[m.tet[t]]
    T = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    lam = np.linalg.solve(T, (x - P[:, 0])[..., None])[..., 0]
    lam0 = 1 - lam.sum(1)
    assert lam.min() > 1e-3 and lam0.min() > 1e-3


def test_gauss_points_integrate_quadratics_on_hull_mesh():
    m = workload_mesh("sphere_tiny")
    om = oracle.OracleMesh(m.xyz, m.tet)
    x, w = om.gauss_points(4)
    # integral of x^2 over the polyhedron = sum over tets of the exact
    # per-tet second moment (Dirichlet formula in barycentric form)
    P = m.xyz[m.tet]
    vol = np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0],
                           np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6
    X = P[:, :, 0]
    exact = float(np.sum(vol * (X.sum(1) ** 2 + (X ** 2).sum(1)) / 20.0))
    assert abs(float(np.sum(w * x[:, 0] ** 2)) - exact) < 1e-13 * max(1.0, abs(exact))
