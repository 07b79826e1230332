"""Pins for the oracle's integration-path search (Sec. 2.2).

* Fig. 2 (completed): the zero pattern of the volume coordinates at the
  go-out point names the face, edge or vertex the ray leaves through.
* The walk against the exhaustive search it replaces (every element clipped
  by its four face planes, no volume coordinates involved): same elements in
  the same order, same break points, and the path ends on the chord bound
  b_i(x) / a_i(x) of Sec. 1 eq. (1), which is computed here from the convex
  hull of the mesh vertices (Qhull), independently of the mesh connectivity.
"""
import os

import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle
from fpde_inputs import kuhn_cube, workload_mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig2_volume_coordinates.txt")
FIG2_TET = np.array([[0.5, 0.75, 0.433], [0.0, 0.0, 0.0], [0.5, 0.0, 0.866], [1.0, 0.0, 0.0]])


def read_fig2():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows.append((parts[0], parts[1]))
    return rows


def rotation_to_e(d, axis):
    """Orthogonal matrix R with R d = e_axis (Householder reflection)."""
    e = np.zeros(3)
    e[axis] = 1.0
    v = d - e
    if np.linalg.norm(v) < 1e-14:
        return np.eye(3)
    v /= np.linalg.norm(v)
    return np.eye(3) - 2.0 * np.outer(v, v)


@pytest.mark.parametrize("axis,sign", [(0, 1), (1, -1), (2, 1)])
def test_fig2_exit_subface_from_zero_pattern(axis, sign):
    rows = read_fig2()
    assert len(rows) == 14  # 4 faces, 6 edges, 4 vertices
    names = "ABCD"
    centroid = FIG2_TET.mean(0)
    for label, pattern in rows:
        verts = [names.index(c) for c in label]
        # a point inside the sub-face: a generic convex combination of its vertices
        wts = np.array([1.0, 1.3, 0.7][: len(verts)])
        p = (wts[:, None] * FIG2_TET[verts]).sum(0) / wts.sum()
        d = (p - centroid) / np.linalg.norm(p - centroid)
        R = rotation_to_e(d * sign, axis)
        xyz = FIG2_TET @ R.T
        om = oracle.OracleMesh(xyz, np.array([[0, 1, 2, 3]], dtype=np.int32))
        z, k, rr = om.exit_pattern(0, R @ centroid, axis, sign)
        got = "".join("0" if (z >> j) & 1 else "1" for j in range(4))
        assert got == pattern, (label, got, k)
        # the go-out point is the chosen point
        assert abs(rr[1] - np.linalg.norm(p - centroid)) < 1e-13


def hull_chord_end(hull, u0, d):
    """Largest r with u0 + r d in the convex hull (Sec. 1 eq. (1))."""
    n, off = hull.equations[:, :3], hull.equations[:, 3]
    nd = n @ d
    r = -(n @ u0 + off)[nd > 0] / nd[nd > 0]
    return float(r.min())


def exhaustive_path(om, u0, d, tol):
    lo, hi = om.exhaustive(u0, d)
    lo = np.maximum(lo, 0.0)
    keep = np.nonzero(hi - lo > tol)[0]
    order = keep[np.argsort(lo[keep], kind="stable")]
    return order, lo[order], hi[order]


@pytest.mark.parametrize("name,nq", [("cube4", 4), ("cube4", 11), ("sphere_small", 4), ("sphere_small", 11)])
def test_walk_matches_exhaustive_search_and_chord(name, nq):
    m = kuhn_cube(4) if name == "cube4" else workload_mesh(name)
    om = oracle.OracleMesh(m.xyz, m.tet)
    hull = ConvexHull(m.xyz)
    x, _ = om.gauss_points(nq)
    n_rays = om.n_tet * nq * 6
    rng = np.random.default_rng(7)
    sample = rng.choice(n_rays, size=min(300, n_rays), replace=False)
    diam = float(np.linalg.norm(m.xyz.max(0) - m.xyz.min(0)))
    for h in sample:
        ln, hs, ids, rend = om.paths(nq, int(h), 1, lists=True)
        n = int(ln[0])
        g, dirn = divmod(int(h), 6)
        i, side = divmod(dirn, 2)
        d = np.zeros(3)
        d[i] = 1.0 if side else -1.0
        order, lo, hi = exhaustive_path(om, x[g], d, 1e-12 * diam)
        assert list(ids[0, :n]) == list(order), (h, ids[0, :n], order)
        assert np.allclose(rend[0, :n], hi, rtol=0, atol=1e-12 * diam)
        # contiguous cover: each element is entered where the previous one is left
        assert np.allclose(lo[1:], hi[:-1], rtol=0, atol=1e-12 * diam)
        assert lo[0] == 0.0
        # the path ends on the domain boundary: b_i(x) - x_i (or x_i - a_i(x))
        assert abs(rend[0, n - 1] - hull_chord_end(hull, x[g], d)) < 1e-12 * diam


def test_path_hash_is_fnv1a_of_ids():
    m = workload_mesh("sphere_tiny")
    om = oracle.OracleMesh(m.xyz, m.tet)
    ln, hs, ids, _ = om.paths(4, 0, 24, lists=True)
    for k in range(24):
        h = 14695981039346656037
        for t in ids[k, : ln[k]]:
            for b in int(t).to_bytes(4, "little"):
                h ^= b
                h = (h * 1099511628211) % (1 << 64)
        assert h == int(hs[k])


def test_two_tet_face_crossing():
    # Fig. 1(b): a path that crosses two elements through their shared face
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=float)
    tet = np.array([[0, 1, 2, 3], [4, 1, 2, 3]], dtype=np.int32)
    om = oracle.OracleMesh(xyz, tet)
    assert om.nbr[0, 0] == 1 and om.nbr[1, 0] == 0
    # Gauss points of element 0, ray +e1: leaves element 0 through face
    # (1,2,3) into element 1 whenever the line meets element 1
    x, _ = om.gauss_points(4)
    ln, hs, ids, rend = om.paths(4, 0 * 6 + 1, 1, lists=True)
    assert ln[0] == 2 and list(ids[0, :2]) == [0, 1]
    # exit of element 0 on the plane x+y+z = 1, exit of element 1 on x = 1... or
    # y/z faces of element 1; compare with the exhaustive clip
    order, lo, hi = exhaustive_path(om, x[0], np.array([1.0, 0, 0]), 1e-12)
    assert list(order) == [0, 1] and np.allclose(rend[0, :2], hi, atol=1e-14)


def test_edge_exit_searches_elements_sharing_the_edge():
    # four elements around the z-axis edge (0,0,-1)-(0,0,1), their outer
    # vertices at angles 45 + 90k degrees; a +x ray at y = 0 starting in
    # element 1 (around 180 degrees) leaves it exactly through the z-axis edge
    # and must continue in element 3 (around 0 degrees), the only element
    # sharing that edge in which it advances (Sec. 2.2: m-face search)
    ang = np.deg2rad(45.0 + 90.0 * np.arange(4))
    c = np.stack([np.cos(ang), np.sin(ang), np.zeros(4)], 1)
    xyz = np.vstack([[0, 0, -1.0], [0, 0, 1.0], c])
    tet = np.array([[0, 1, 2 + k, 2 + (k + 1) % 4] for k in range(4)], dtype=np.int32)
    om = oracle.OracleMesh(xyz, tet)
    u0 = np.array([-0.3, 0.0, 0.1])
    z, k, rr = om.exit_pattern(1, u0, 0, 1)
    assert bin(z).count("1") == 2 and (z >> 0) & 1 == 0 and (z >> 1) & 1 == 0
    assert abs(rr[1] - 0.3) < 1e-15
    ids, rend = om.walk(1, u0, 0, 1)
    assert list(ids) == [1, 3]
    order, lo, hi = exhaustive_path(om, u0, np.array([1.0, 0, 0]), 1e-12)
    assert list(order) == [1, 3] and np.allclose(rend, hi, atol=1e-14)


def test_vertex_exit_searches_elements_sharing_the_vertex():
    # eight elements around the vertex O = 0: O joined to the faces of an
    # octahedron in generic orientation.  The +x axis meets O from inside one
    # element and leaves into another: a 0-face exit (three zero coordinates)
    th = 0.37
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    ph = 0.61
    Rx = np.array([[1, 0, 0], [0, np.cos(ph), -np.sin(ph)], [0, np.sin(ph), np.cos(ph)]])
    R = Rz @ Rx
    oct_v = np.vstack([R @ (s * e) for e in np.eye(3) for s in (1.0, -1.0)])  # 6 vertices
    xyz = np.vstack([[0.0, 0.0, 0.0], oct_v])
    tets = []
    for s1 in (0, 1):
        for s2 in (0, 1):
            for s3 in (0, 1):
                tets.append([0, 1 + s1, 3 + s2, 5 + s3])
    tet = np.array(tets, dtype=np.int32)
    om = oracle.OracleMesh(xyz, tet)

    def containing(p):
        for t, tt in enumerate(tet):
            P = xyz[tt]
            lam = np.linalg.solve((P[1:] - P[0]).T, p - P[0])
            if lam.min() > 1e-9 and lam.sum() < 1 - 1e-9:
                return t
        return -1

    t_in, t_out = containing(np.array([-0.3, 0, 0])), containing(np.array([0.3, 0, 0]))
    assert t_in >= 0 and t_out >= 0 and t_in != t_out
    u0 = np.array([-0.3, 0.0, 0.0])
    z, k, rr = om.exit_pattern(t_in, u0, 0, 1)
    assert bin(z).count("1") == 3
    ids, rend = om.walk(t_in, u0, 0, 1)
    assert list(ids) == [t_in, t_out]
    order, lo, hi = exhaustive_path(om, u0, np.array([1.0, 0, 0]), 1e-12)
    assert list(order) == [t_in, t_out] and np.allclose(rend, hi, atol=1e-14)
