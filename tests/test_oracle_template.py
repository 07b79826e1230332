"""Pins of the oracle's template (Sec. 2.3, Table 1).

* On the Kuhn cube with n intervals every interior node's patch box is the
  cube of half-width h = 1/n around it, so T_jk holds exactly when at least
  two of the three index differences are <= 2: with m = n - 1 interior nodes
  per axis, p = m + 2(m-1) + 2(m-2) index pairs per axis are within 2 and
  q = m^2 - p are not, so nnz(T) = 3 p^2 q + p^3 (counted by hand, not by
  the oracle's code).  Its density falls like 1/N^2 (Table 1's 3-D row).
* T contains the nonzero pattern of the stiffness matrix the oracle
  assembles (on the cube and on a hull mesh, both rules).
"""
import numpy as np
import pytest

import oracle
from fpde_inputs import kuhn_cube, workload_mesh


def kuhn_count(n):
    m = n - 1
    p = m + 2 * (m - 1) + 2 * (m - 2)
    q = m * m - p
    return 3 * p * p * q + p ** 3


@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_template_count_on_kuhn_cube(n):
    mesh = kuhn_cube(n)
    om = oracle.OracleMesh(mesh.xyz, mesh.tet)
    T = om.template()
    assert om.ndof == (n - 1) ** 3
    assert int(T.sum()) == kuhn_count(n)
    assert (T == T.T).all()


def test_template_density_falls_like_one_over_n_squared():
    # closed form: density * m^2 rises to 75 as the grid is refined (Table 1, 3-D, fractional),
    # so the density itself falls like 1/N^2, not like 1/N^3 as for a classical stiffness
    dens = {n: kuhn_count(n) / float((n - 1) ** 6) for n in (8, 16, 32, 64, 512)}
    scaled = [dens[n] * (n - 1) ** 2 for n in (8, 16, 32, 64, 512)]
    assert all(a < b < 75.0 for a, b in zip(scaled, scaled[1:]))
    assert scaled[-1] > 74.0
    om = oracle.OracleMesh(*[getattr(kuhn_cube(16), k) for k in ("xyz", "tet")])
    assert om.template().mean() == pytest.approx(dens[16], rel=1e-12)


@pytest.mark.parametrize("name,nq,alpha", [("cube_n8", 4, 1.5), ("sphere_small", 4, 1.3),
                                           ("sphere_small", 11, 1.8)])
def test_template_contains_stiffness_pattern(name, nq, alpha):
    mesh = kuhn_cube(8) if name == "cube_n8" else workload_mesh(name)
    om = oracle.OracleMesh(mesh.xyz, mesh.tet)
    A = om.assemble(nq, alpha, (1.0, 0.7, 1.3))
    T = om.template()
    nz = np.abs(A) > 0.0
    assert not (nz & ~T).any()
    assert T.mean() < 1.0 and nz.mean() <= T.mean()


def test_template_tiles_are_any_over_tile():
    mesh = kuhn_cube(8)
    om = oracle.OracleMesh(mesh.xyz, mesh.tet)
    T = om.template()
    tiles = om.template_tiles(64)
    nt = tiles.shape[0]
    assert nt == -(-om.ndof // 64)
    for P in range(nt):
        for Q in range(nt):
            assert tiles[P, Q] == T[64 * P:64 * P + 64, 64 * Q:64 * Q + 64].any()
