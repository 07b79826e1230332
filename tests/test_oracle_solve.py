"""Pins for the oracle's large-size tools: its matrix-free product split over
OpenMP threads and Gauss-point ranges, and its conjugate-gradient solve.

* The matrix-free product of the stiffness matrix (the sums of Sec. 2.1,
  never forming K) does not depend on the number of threads beyond rounding,
  and the products over disjoint Gauss-point ranges add up to the whole one.
* Conjugate gradients (a textbook method, written out plainly in the oracle)
  terminates in at most k steps on a matrix with k distinct eigenvalues (exact
  arithmetic; here to rounding), and on the stiffness matrix of a hull mesh,
  driven by the matrix-free product, it agrees with LAPACK's Cholesky solve
  of the densely assembled matrix.
* The operator that keeps the walked vectors gives the same products, its
  diagonal is the dense matrix's, and Jacobi-preconditioned CG on it gives
  the same solution.
"""
import numpy as np

import oracle
from fpde_inputs import workload_mesh


def test_product_is_independent_of_threads_and_splits_by_gauss_point():
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    nq, alpha, K = 11, 1.3, (1.0, 0.7, 1.6)
    x = np.random.default_rng(3).normal(size=om.ndof)
    before = oracle.set_threads()
    try:
        oracle.set_threads(1)
        y1 = om.apply(nq, alpha, K, x)
        oracle.set_threads(max(before, 4))
        y4 = om.apply(nq, alpha, K, x)
    finally:
        oracle.set_threads(before)
    assert np.abs(y4 - y1).max() <= 1e-14 * np.abs(y1).max()
    G = m.n_tet * nq
    cuts = [0, 17, G // 3, G // 3 + 1, G]
    parts = sum(om.apply_range(nq, alpha, K, x, a, b) for a, b in zip(cuts[:-1], cuts[1:]))
    assert np.abs(parts - y1).max() <= 1e-13 * np.abs(y1).max()
    assert not om.apply_range(nq, alpha, K, x, 5, 5).any()


def test_cg_terminates_in_as_many_steps_as_distinct_eigenvalues():
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(40, 40)))
    lam = np.repeat([0.5, 2.0, 3.0, 11.0], 10)
    A = (Q * lam) @ Q.T
    b = rng.normal(size=40)
    x, it = oracle.cg(lambda v: A @ v, b, tol=1e-12)
    assert it <= 4 + 1  # four distinct eigenvalues (one more step for rounding)
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-10 * np.abs(x).max()


def test_matrix_free_cg_equals_lapack_cholesky():
    m = workload_mesh("sphere_small")
    om = oracle.OracleMesh(m.xyz, m.tet)
    nq, alpha, K = 4, 1.7, (1.0, 1.0, 1.0)
    b = om.load(nq)
    u_chol = oracle.solve_spd(om.assemble(nq, alpha, K), b)
    u_cg, it = oracle.cg(lambda v: om.apply(nq, alpha, K, v), b, tol=1e-13)
    assert 0 < it < om.ndof
    assert np.abs(u_cg - u_chol).max() <= 1e-10 * np.abs(u_chol).max()
    # the operator with stored vectors gives the same products and solution
    op = oracle.OracleOperator(om, nq, alpha, K)
    x = np.random.default_rng(5).normal(size=om.ndof)
    y = om.apply(nq, alpha, K, x)
    assert np.abs(op.apply(x) - y).max() <= 1e-14 * np.abs(y).max()
    u_op, it2 = oracle.cg(op.apply, b, tol=1e-13)
    assert np.abs(u_op - u_chol).max() <= 1e-10 * np.abs(u_chol).max()
    # its diagonal is the dense matrix's, and the Jacobi-preconditioned
    # iteration reaches the same solution
    A = om.assemble(nq, alpha, K)
    assert np.abs(op.diagonal() - np.diag(A)).max() <= 1e-14 * np.abs(np.diag(A)).max()
    u_pc, it3 = oracle.cg(op.apply, b, tol=1e-13, dinv=1.0 / op.diagonal())
    assert np.abs(u_pc - u_chol).max() <= 1e-10 * np.abs(u_chol).max()
