"""Pins for the oracle's mesh checks: the domain must be convex.

The chord bounds a_i(x), b_i(x) of Sec. 1 eq. (1) describe one chord of the
domain through x, which is its intersection with the line only when the
domain is convex.  A polyhedron is convex exactly when every vertex lies on
the inner side of the plane of every boundary face; the oracle rejects other
meshes with status -4 (tolerance 1e-12 of the bounding-box diagonal).

Pinned here by shapes whose convexity is known without computation: the
cube and random convex hulls (accepted), the L-shaped prism (a cube with a
quarter removed), and the cube with one boundary vertex moved out of or into
its face by 1e-9 (a bump or a dent: rejected) or by 1e-15 (inside the
tolerance: accepted).
"""
import numpy as np
import pytest

import oracle
from fpde_inputs import kuhn_cube, notched_cube, workload_mesh

NONCONVEX = -4


def test_convex_meshes_are_accepted():
    for m in (kuhn_cube(2), kuhn_cube(4), workload_mesh("sphere_tiny"), workload_mesh("sphere_small")):
        om = oracle.OracleMesh(m.xyz, m.tet)
        assert om.ndof >= 1


@pytest.mark.parametrize("n", [2, 4])
def test_l_shaped_prism_is_rejected(n):
    m = notched_cube(n)
    assert m.n_tet == 6 * n ** 3 * 3 // 4
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(m.xyz, m.tet)
    assert e.value.status == NONCONVEX


def face_centre_vertex(m):
    """Index of the vertex at the centre of the face z = 1 of a Kuhn cube."""
    k = np.flatnonzero(np.all(np.abs(m.xyz - [0.5, 0.5, 1.0]) < 1e-14, axis=1))
    assert len(k) == 1
    return int(k[0])


@pytest.mark.parametrize("dz", [1e-9, -1e-9])
def test_bump_or_dent_in_a_face_is_rejected(dz):
    m = kuhn_cube(4)
    v = face_centre_vertex(m)
    xyz = m.xyz.copy()
    xyz[v, 2] += dz
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(xyz, m.tet)
    assert e.value.status == NONCONVEX


@pytest.mark.parametrize("dz", [1e-15, -1e-15])
def test_perturbation_inside_the_tolerance_is_accepted(dz):
    m = kuhn_cube(4)
    v = face_centre_vertex(m)
    xyz = m.xyz.copy()
    xyz[v, 2] += dz
    assert oracle.OracleMesh(xyz, m.tet).ndof == 27
