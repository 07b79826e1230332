"""Seeded synthetic tetrahedral meshes shaped like the paper's workloads.

This module only *makes inputs*: vertex coordinates and tetrahedra (plus a
few descriptive statistics).  It holds none of the finite-element method's
arithmetic (no basis functions, quadrature, path search or assembly), so the
CPU oracle and the GPU library can both take their meshes from here while
sharing no code with each other.

The paper solves on convex domains (the chord bounds of Section 1 need
convexity) meshed by simplices (Section 2.1); its own meshes are not
published, so these generators stand in for them:

* ``kuhn_cube(n)``: the unit cube cut into n^3 sub-cubes, each split into the
  six Kuhn tetrahedra that share the sub-cube's (0,0,0)-(1,1,1) diagonal.
  The split is conforming across sub-cubes.
* ``hull_mesh(...)``: the convex hull of seeded random points (on a sphere,
  or inside an ellipsoid), filled with a jittered body-centred-cubic lattice
  of interior points kept at least half a spacing inside every hull facet,
  Delaunay tetrahedralised (Qhull), with a vertex re-jitter loop that raises
  the worst radius ratio.

Vertices and tetrahedra are renumbered in Morton (Z-curve) order of their
positions / centroids, so ids are spatially coherent and identical for every
consumer of the same (generator, parameters, seed).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Mesh", "kuhn_cube", "notched_cube", "hull_mesh", "radius_ratio", "workload_mesh", "fibonacci_sphere",
    "kuhn_square", "polygon_mesh", "circle_points",
    "WORKLOADS",
]


@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray          # (n_vert, 3) float64
    tet: np.ndarray          # (n_tet, 4) int32
    name: str = ""
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tet(self) -> int:
        return int(self.tet.shape[0])


# --------------------------------------------------------------------------
# Morton ordering
# --------------------------------------------------------------------------
def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def _morton_keys(p: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    span = np.maximum(hi - lo, 1e-300)
    q = np.clip(((p - lo) / span) * float((1 << 21) - 1), 0, (1 << 21) - 1)
    q = q.astype(np.uint64)
    return _part1by2(q[:, 0]) | (_part1by2(q[:, 1]) << np.uint64(1)) | \
        (_part1by2(q[:, 2]) << np.uint64(2))


def morton_renumber(xyz: np.ndarray, tet: np.ndarray):
    """Renumber vertices and tetrahedra along the Z-curve (stable, ties by id)."""
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    vkey = _morton_keys(xyz, lo, hi)
    vperm = np.lexsort((np.arange(len(xyz)), vkey))
    inv = np.empty_like(vperm)
    inv[vperm] = np.arange(len(vperm))
    xyz2 = np.ascontiguousarray(xyz[vperm])
    tet2 = inv[tet]
    cen = xyz2[tet2].mean(axis=1)
    tkey = _morton_keys(cen, lo, hi)
    tperm = np.lexsort((np.arange(len(tet2)), tkey))
    return xyz2, np.ascontiguousarray(tet2[tperm].astype(np.int32))


# --------------------------------------------------------------------------
# Kuhn cube
# --------------------------------------------------------------------------
def kuhn_cube(n: int, lo: float = 0.0, hi: float = 1.0, morton: bool = False) -> Mesh:
    """Unit cube, n^3 sub-cubes x 6 Kuhn tetrahedra (6 n^3 tets, (n+1)^3 nodes)."""
    m = n + 1
    g = np.linspace(lo, hi, m)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)

    def vid(i, j, k):
        return (i * m + j) * m + k

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for p in perms:
                    c = [i, j, k]
                    t = [vid(*c)]
                    for ax in p:
                        c[ax] += 1
                        t.append(vid(*c))
                    tets.append(t)
    tet = np.asarray(tets, dtype=np.int32)
    if morton:
        xyz, tet = morton_renumber(xyz, tet)
    return Mesh(xyz, tet, name=f"kuhn_cube_{n}", info={"n": n})


def notched_cube(n: int) -> Mesh:
    """A non-convex input: the Kuhn cube of ``kuhn_cube(n)`` (n even) with the
    sub-cubes of the quarter x > 1/2, y > 1/2 removed (an L-shaped prism).
    Vertices no longer used by any tetrahedron are dropped."""
    if n < 2 or n % 2:
        raise ValueError("notched_cube needs an even n >= 2")
    c = kuhn_cube(n)
    cen = c.xyz[c.tet].mean(axis=1)
    keep = ~((cen[:, 0] > 0.5) & (cen[:, 1] > 0.5))
    tet = c.tet[keep]
    used = np.unique(tet)
    remap = np.full(c.n_vert, -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return Mesh(c.xyz[used].copy(), remap[tet].astype(np.int32), name=f"notched_cube_{n}", info={"n": n})


# --------------------------------------------------------------------------
# Quality measure (input statistics only)
# --------------------------------------------------------------------------
def kuhn_square(n: int, lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """The unit square cut into n x n sub-squares, each split into two
    triangles along its (0,0)-(1,1) diagonal (a two-dimensional input: xyz
    has two columns, tet holds triangles)."""
    t = np.linspace(lo, hi, n + 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: i * (n + 1) + j  # noqa: E731
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    return Mesh(xy, np.array(tris, dtype=np.int32), name=f"square{n}")


def polygon_mesh(hull_points: np.ndarray, spacing: float, seed: int, jitter: float = 0.1,
                 name: str = "polygon") -> Mesh:
    """Delaunay triangulation of conv(hull_points) (2-D) with a jittered
    triangular lattice of interior points kept at least half a spacing
    inside every edge; vertices and triangles in Morton order of their
    positions / centroids."""
    from scipy.spatial import ConvexHull, Delaunay
    rng = np.random.default_rng(seed)
    h = ConvexHull(hull_points)
    bpts = hull_points[h.vertices]
    eq = h.equations
    lo, hi = bpts.min(0), bpts.max(0)
    xs = np.arange(lo[0], hi[0] + spacing, spacing)
    ys = np.arange(lo[1], hi[1] + spacing, spacing * np.sqrt(3) / 2)
    G = np.array([(x + (0.5 * spacing if k % 2 else 0.0), y) for k, y in enumerate(ys) for x in xs])
    G = G + rng.uniform(-jitter * spacing, jitter * spacing, size=G.shape)
    inside = (G @ eq[:, :2].T + eq[:, 2]).max(axis=1) <= -0.5 * spacing
    P = np.concatenate([bpts, G[inside]])
    tri = Delaunay(P).simplices.astype(np.int64)
    p = P[tri]
    area2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    tri = tri[np.abs(area2) > 1e-12 * spacing ** 2]
    keys = _morton_keys(np.concatenate([P, np.zeros((len(P), 1))], axis=1),
                        np.append(lo, 0.0), np.append(hi, 1.0))
    order = np.argsort(keys, kind="stable")
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    P = P[order]
    tri = inv[tri]
    c = P[tri].mean(axis=1)
    tkeys = _morton_keys(np.concatenate([c, np.zeros((len(c), 1))], axis=1), np.append(lo, 0.0), np.append(hi, 1.0))
    tri = tri[np.argsort(tkeys, kind="stable")]
    return Mesh(P, tri.astype(np.int32), name=name)


def circle_points(n: int, radius: float = 1.0) -> np.ndarray:
    k = np.arange(n) * 2.0 * np.pi / n
    return radius * np.stack([np.cos(k), np.sin(k)], axis=1)


def radius_ratio(xyz: np.ndarray, tet: np.ndarray) -> np.ndarray:
    """rho = 3 r_in / R_circ per tetrahedron (1 for the regular one)."""
    p = xyz[tet]
    a = p[:, 1] - p[:, 0]
    b = p[:, 2] - p[:, 0]
    c = p[:, 3] - p[:, 0]
    vol6 = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    def area(u, v, w):
        return 0.5 * np.linalg.norm(np.cross(v - u, w - u), axis=1)
    s = area(p[:, 1], p[:, 2], p[:, 3]) + area(p[:, 0], p[:, 2], p[:, 3]) + \
        area(p[:, 0], p[:, 1], p[:, 3]) + area(p[:, 0], p[:, 1], p[:, 2])
    r_in = (vol6 / 2.0) / np.maximum(s, 1e-300)       # 3V / S, V = vol6/6
    # circumradius: |a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b) over 2 det
    num = (np.sum(a * a, 1)[:, None] * np.cross(b, c)
           + np.sum(b * b, 1)[:, None] * np.cross(c, a)
           + np.sum(c * c, 1)[:, None] * np.cross(a, b))
    R = np.linalg.norm(num, axis=1) / np.maximum(2.0 * vol6, 1e-300)
    return 3.0 * r_in / np.maximum(R, 1e-300)


# --------------------------------------------------------------------------
# Convex-hull meshes
# --------------------------------------------------------------------------
def _hull(points: np.ndarray):
    from scipy.spatial import ConvexHull
    h = ConvexHull(points)
    return h


def hull_mesh(hull_points: np.ndarray, spacing: float, seed: int,
              rho_min: float = 0.2, max_rounds: int = 12,
              jitter: float = 0.1, name: str = "hull") -> Mesh:
    """Delaunay mesh of conv(hull_points) with a jittered interior lattice.

    Only the hull vertices of ``hull_points`` are kept on the boundary, so the
    domain is exactly their convex hull.  Interior body-centred-cubic lattice
    points (density of a cubic lattice of step ``spacing``, jitter
    +-``jitter``*spacing per axis) are kept when they lie at least
    0.5*spacing inside every facet plane.  Tetrahedra whose radius ratio is
    below ``rho_min`` have their interior vertices re-jittered and the point
    set is re-triangulated, up to ``max_rounds`` times.  Tets standing on a
    hull facet keep that facet's shape (random hulls have skinny facets), so
    ``info`` reports the worst radius ratio with and without them.
    """
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    h = _hull(hull_points)
    bpts = hull_points[np.unique(h.simplices)]
    eq = h.equations                       # n.x + d <= 0 inside
    lo, hi = bpts.min(0), bpts.max(0)
    # body-centred cubic lattice with the same point density as a cubic one of
    # step ``spacing`` (its Delaunay cells are well shaped and non-degenerate)
    a = spacing * 2.0 ** (1.0 / 3.0)
    axes = [np.arange(lo[d] + 0.25 * a, hi[d], a) for d in range(3)]
    G0 = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    G = np.concatenate([G0, G0 + 0.5 * a])
    G = G + rng.uniform(-jitter * spacing, jitter * spacing, size=G.shape)
    inside = (G @ eq[:, :3].T + eq[:, 3]).max(axis=1) <= -0.5 * spacing
    ipts = G[inside]
    nb = len(bpts)
    P = np.concatenate([bpts, ipts])

    def triangulate(P):
        d = Delaunay(P)
        t = d.simplices.astype(np.int64)
        p = P[t]
        vol6 = np.einsum("ij,ij->i", p[:, 1] - p[:, 0],
                         np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
        keep = np.abs(vol6) > 1e-12 * spacing ** 3
        return t[keep]

    def interior_min(t):
        rho = radius_ratio(P, t)
        movable = (t >= nb).any(axis=1)
        return rho, movable

    t = triangulate(P)
    rho, movable = interior_min(t)
    rounds = 0
    amp = 0.1 * spacing
    while rounds < max_rounds:
        badmask = (rho < rho_min) & movable
        if not badmask.any():
            break
        bad = np.unique(t[badmask].ravel())
        bad = bad[bad >= nb]               # hull vertices never move
        trial = P[bad] + rng.uniform(-amp, amp, size=(len(bad), 3))
        ok = (trial @ eq[:, :3].T + eq[:, 3]).max(axis=1) <= -0.25 * spacing
        P[bad[ok]] = trial[ok]
        t = triangulate(P)
        rho, movable = interior_min(t)
        rounds += 1
    # tets with a hull facet (3 hull vertices) inherit that facet's shape,
    # which the generator cannot change; report both minima
    on_hull = (t < nb).sum(axis=1) >= 3
    info = {"spacing": spacing, "seed": seed, "n_hull_vertices": int(nb),
            "rho_min": float(rho.min()), "rho_mean": float(rho.mean()),
            "rho_min_off_hull_facets": float(rho[~on_hull].min()),
            "rejitter_rounds": rounds}
    xyz, tet = morton_renumber(P, t.astype(np.int32))
    return Mesh(xyz, tet, name=name, info=info)


def sphere_points(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(n, 3))
    return p / np.linalg.norm(p, axis=1, keepdims=True)


def fibonacci_sphere(n: int, radius: float = 1.0) -> np.ndarray:
    """n points on the sphere of the given radius along the golden-angle
    spiral (equal-area latitude bands): a quasi-uniform, deterministic hull
    whose facets shrink evenly as n grows, for mesh-refinement families."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    phi = np.pi * (1.0 + 5.0 ** 0.5) * k
    s = np.sqrt(1.0 - z * z)
    return radius * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def ellipsoid_points(n: int, axes, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    r = rng.uniform(size=(n, 1)) ** (1.0 / 3.0)
    return p * r * np.asarray(axes, dtype=np.float64)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    # unit cube, 4x4x4 sub-cubes x 6 Kuhn tets: 384 tets, 125 nodes, 27 interior
    "cube384": dict(kind="cube", n=4),
    # hull of 400 random points on the unit sphere + lattice: ~20k tets, ~4k nodes
    "sphere20k": dict(kind="sphere", n_surface=400, spacing=0.104, seed=2),
    # same generator, ~150k tets / ~27k nodes
    "sphere150k": dict(kind="sphere", n_surface=400, spacing=0.053, seed=3),
    # unit-ball hull (800 points on S^2), ~40k tets / ~8k nodes
    "ball40k": dict(kind="sphere", n_surface=800, spacing=0.082, seed=4),
    # hull of 2000 points in the ellipsoid (1, 0.7, 0.4), ~400k tets / ~70k nodes
    "ellipsoid400k": dict(kind="ellipsoid", n_points=2000, axes=(1.0, 0.7, 0.4),
                          spacing=0.0246, seed=5),
    # the ball |x| < 0.5 of the divergence-form problem (Sec. 3): a
    # refinement family whose largest element diameter matches the h column
    # of Table 3 (0.270, 0.139, 0.0757) and the mesh of Fig. 3 (0.0894)
    "ball_h270": dict(kind="ball", radius=0.5, n_surface=122, spacing=0.14021, seed=21),
    "ball_h139": dict(kind="ball", radius=0.5, n_surface=469, spacing=0.07152, seed=22),
    "ball_h089": dict(kind="ball", radius=0.5, n_surface=1215, spacing=0.04445, seed=23),
    "ball_h076": dict(kind="ball", radius=0.5, n_surface=1628, spacing=0.03840, seed=24),
    # two dimensions: the unit disk as a 64-gon filled with a jittered
    # triangular lattice (~4.5k nodes) and a small one for tests
    "disk4k": dict(kind="disk", n_boundary=160, spacing=0.028, seed=31),
    "disk_small": dict(kind="disk", n_boundary=24, spacing=0.2, seed=32),
    # small hull meshes for tests
    "sphere_tiny": dict(kind="sphere", n_surface=40, spacing=0.45, seed=11),
    "sphere_small": dict(kind="sphere", n_surface=100, spacing=0.22, seed=12),
}


def workload_mesh(name: str, **overrides) -> Mesh:
    spec = dict(WORKLOADS[name])
    spec.update(overrides)
    kind = spec.pop("kind")
    if kind == "cube":
        m = kuhn_cube(spec["n"])
    elif kind == "sphere":
        pts = sphere_points(spec["n_surface"], spec["seed"])
        m = hull_mesh(pts, spec["spacing"], spec["seed"], name=name)
    elif kind == "disk":
        m = polygon_mesh(circle_points(spec["n_boundary"]), spec["spacing"], spec["seed"], name=name)
    elif kind == "ball":
        pts = fibonacci_sphere(spec["n_surface"], spec["radius"])
        m = hull_mesh(pts, spec["spacing"], spec["seed"], name=name)
    elif kind == "ellipsoid":
        pts = ellipsoid_points(spec["n_points"], spec["axes"], spec["seed"])
        m = hull_mesh(pts, spec["spacing"], spec["seed"], name=name)
    else:
        raise ValueError(kind)
    m.name = name
    return m
