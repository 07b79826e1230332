"""Pins for the oracle's adjoint gradients of J = ||u_h - u_obs||^2.

u_h = K(alpha, K_1..3)^{-1} b; the oracle's gradient uses lam = K^{-1} dJ/du
and the closed-form alpha-derivatives of the basis-function derivatives
(ln-terms and the digamma term).  Checked against central differences
(h = 1e-6) of the oracle's own forward solve.
"""
import numpy as np
import pytest

import oracle
from fpde_inputs import kuhn_cube, workload_mesh


def loss(om, nq, alpha, K, b, u_obs):
    u = oracle.solve_spd(om.assemble(nq, alpha, K), b)
    return float(np.sum((u - u_obs) ** 2)), u


@pytest.mark.parametrize("name", ["cube3", "sphere_tiny"])
def test_gradient_matches_central_differences(name):
    m = kuhn_cube(3) if name == "cube3" else workload_mesh(name)
    om = oracle.OracleMesh(m.xyz, m.tet)
    nq = 4
    b = om.load(nq)
    rng = np.random.default_rng(40)
    u_obs = oracle.solve_spd(om.assemble(nq, 1.6, (1.2, 0.8, 1.0)), b)
    u_obs = u_obs + 1e-3 * rng.normal(size=u_obs.shape)
    alpha, K = 1.4, np.array([1.0, 1.0, 1.0])
    J, u = loss(om, nq, alpha, K, b, u_obs)
    da, dK = om.gradient(nq, alpha, K, u, 2.0 * (u - u_obs))
    h = 1e-6
    fd_a = (loss(om, nq, alpha + h, K, b, u_obs)[0] - loss(om, nq, alpha - h, K, b, u_obs)[0]) / (2 * h)
    assert abs(da - fd_a) <= 1e-6 * abs(fd_a)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (loss(om, nq, alpha, K + e, b, u_obs)[0] - loss(om, nq, alpha, K - e, b, u_obs)[0]) / (2 * h)
        assert abs(dK[i] - fd) <= 1e-6 * abs(fd)
