"""Pins for the oracle's general uniform form (Sec. 1, eq. equ:varsss):

    K_kl = sum_i sum_g w_g [cl_i D_L^{a_i} psi_l D_R^{b_i} psi_k + cr_i D_R^{a_i} psi_l D_L^{b_i} psi_k](x_g),

test operator on the side opposite to the trial one, orders in [0, 1].

* a = b = 1 (D_L^1 = d/dx, D_R^1 = -d/dx): with cl = cr = 1/2 on every axis
  K = -(grad psi_l, grad psi_k), minus the classical stiffness matrix.
* a = b = 0 (the identity): with cl_i + cr_i summing to 1 over the axes K is
  the P1 mass matrix |E|/20 (1 + delta_kl), exact for the 4-point rule.
* a = 1, b = 0 on axis 0 only (cl - cr = 1): K_kl = (d_0 psi_l, psi_k), the
  P1 convection matrix, |E|/4 d_0 lambda_l per element.
* Transposition: K(a, b, cl, cr)^T = K(b, a, cr, cl).
* The Riesz split (a = b = alpha/2, cl = cr = K_i c_alpha) and the problem of
  Sec. 3 (a = beta_i, b = 1, cl = p_i, cr = q_i) are instances: both equal
  the oracle's own assemblies of those problems, which are pinned on their
  own.
"""
import numpy as np
import pytest

import oracle
from fpde_inputs import kuhn_cube, workload_mesh

from test_oracle_assembly import classical_stiffness


def element_data(m, om):
    dof = om.dof
    out = []
    for t in m.tet:
        P = m.xyz[t]
        C = np.linalg.inv(np.hstack([np.ones((4, 1)), P]))
        out.append((t, C[1:, :].T, abs(np.linalg.det(P[1:] - P[0])) / 6.0))
    return dof, out


@pytest.mark.parametrize("name", ["cube3", "sphere_small"])
def test_order_one_both_sides_is_minus_stiffness(name):
    m = kuhn_cube(3) if name == "cube3" else workload_mesh(name)
    om = oracle.OracleMesh(m.xyz, m.tet)
    K = om.assemble_form(4, (1.0, 1.0, 1.0), (1.0, 1.0, 1.0), [0.5] * 6)
    S = classical_stiffness(m.xyz, m.tet, om.dof, om.ndof, (1.0, 1.0, 1.0))
    assert np.abs(K + S).max() <= 1e-13 * np.abs(S).max()


@pytest.mark.parametrize("name", ["cube3", "sphere_small"])
def test_order_zero_is_mass_matrix(name):
    m = kuhn_cube(3) if name == "cube3" else workload_mesh(name)
    om = oracle.OracleMesh(m.xyz, m.tet)
    K = om.assemble_form(4, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), [0.2, 0.1, 0.2, 0.15, 0.25, 0.1])
    dof, els = element_data(m, om)
    M = np.zeros_like(K)
    for t, _, vol in els:
        for a in range(4):
            for b in range(4):
                da, db = dof[t[a]], dof[t[b]]
                if da >= 0 and db >= 0:
                    M[da, db] += vol / 20.0 * (2.0 if a == b else 1.0)
    assert np.abs(K - M).max() <= 1e-12 * np.abs(M).max()


def test_order_one_against_zero_is_convection_matrix():
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    K = om.assemble_form(4, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), [0.75, 0.0, 0.0, -0.25, 0.0, 0.0])
    dof, els = element_data(m, om)
    C = np.zeros_like(K)
    for t, grads, vol in els:
        for k in range(4):
            for l in range(4):
                dk, dl = dof[t[k]], dof[t[l]]
                if dk >= 0 and dl >= 0:
                    C[dk, dl] += vol / 4.0 * grads[l, 0]
    assert np.abs(K - C).max() <= 1e-12 * np.abs(C).max()


def test_transposition_swaps_orders_and_sides():
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    G = m.n_tet * 11
    rng = np.random.default_rng(12)
    c = rng.uniform(0.2, 1.0, size=(6, G))
    a, b = (0.3, 0.8, 0.55), (0.9, 0.4, 0.7)
    K1 = om.assemble_form(11, a, b, c)
    K2 = om.assemble_form(11, b, a, np.ascontiguousarray(c[[3, 4, 5, 0, 1, 2]]))
    assert np.abs(K1.T - K2).max() <= 1e-13 * np.abs(K1).max()
    assert np.abs(K1 - K1.T).max() > 1e-3 * np.abs(K1).max()


def test_riesz_and_sec3_are_instances():
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    alpha, Kc = 1.5, (1.0, 0.5, 2.0)
    g, ca = alpha / 2, oracle.c_alpha(alpha)
    A1 = om.assemble(4, alpha, Kc)
    A2 = om.assemble_form(4, (g, g, g), (g, g, g), [Kc[0] * ca, Kc[1] * ca, Kc[2] * ca] * 2)
    assert np.abs(A1 - A2).max() <= 1e-15 * np.abs(A1).max()
    beta = (0.6, 0.7, 0.8)
    x, _ = om.gauss_points(4)
    B1 = om.assemble_div(4, beta)
    B2 = om.assemble_form(4, beta, (1.0, 1.0, 1.0), oracle.div_coefficients(x))
    assert np.abs(B1 - B2).max() <= 1e-14 * np.abs(B1).max()


def test_rows_variant_keeps_the_listed_rows():
    # the row list only selects which rows are kept: every kept row equals
    # the whole matrix's, in any order, including the first and last rows
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    a, b = (0.3, 0.8, 0.55), (0.9, 0.4, 0.7)
    coef = (1.0, 0.5, 2.0, 0.7, 1.5, 0.3)
    K = om.assemble_form(4, a, b, coef)
    n = K.shape[0]
    rows = np.array([n - 1, 0, 17, n // 2, 5])
    # one thread sums in the whole matrix's order: the same bits
    before = oracle.set_threads()
    try:
        oracle.set_threads(1)
        R = om.assemble_form(4, a, b, coef, rows=rows)
    finally:
        oracle.set_threads(before)
    assert np.array_equal(R, K[rows])
    # several threads add their Gauss points' parts in thread order
    R = om.assemble_form(4, a, b, coef, rows=rows)
    assert np.abs(R - K[rows]).max() <= 1e-14 * np.abs(K).max()
    with pytest.raises(oracle.OracleError):
        om.assemble_form(4, a, b, coef, rows=np.array([3, 3]))
