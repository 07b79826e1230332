"""Plain FP64 CPU oracle for the 3-D fractional FEM stiffness assembly and solve.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the GPU library.  The heavy loops
live in ``fpde_oracle.c`` (plain C, ``-O2 -ffp-contract=off``); this module
marshals arguments, supplies the closed-form scalars (Gamma, digamma, the
Riesz constant), the textbook solves (LAPACK Cholesky through SciPy, plain
CG) and the manufactured solution on the unit cube.

Problem (the Riesz instance of form 1 of the paper's uniform variational
form, Sec. 1 eq. equ:varsss, on a convex polyhedron with zero extension):

    -sum_i K_i d^alpha u / d|x_i|^alpha = f,   1 < alpha <= 2,

with d^alpha/d|x|^alpha = -(D_L^alpha + D_R^alpha) / (2 cos(pi alpha / 2)).
Splitting each one-sided operator into two of order gamma = alpha/2 gives

    a(u, v) = c_alpha sum_i K_i [(D_L^g u, D_R^g v) + (D_R^g u, D_L^g v)],
    c_alpha = 1 / (2 cos(pi alpha / 2))  (< 0 on (1, 2); -1/2 at alpha = 2),

which is symmetric positive definite and equals sum_i K_i (d_i u, d_i v) at
alpha = 2.

Also the divergence-form two-sided problem of Sec. 3 (eq. equ:sfde2) on the
ball |x| < r: order-beta_i one-sided derivatives with coefficients
p_i = cos x_i, q_i = 1 - cos x_i on the trial side, the classical derivative
on the test side (a non-symmetric matrix, solved by LAPACK LU), and the
closed-form source of its exact solution u = (|x|^2 - r^2)^2.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "fpde_oracle.c"
_SRC2 = _HERE / "fpde_oracle2d.c"
_LIB = _HERE / "_fpde_oracle.so"

ORC_EPATH = -5
DEFAULT_CAP = 4096


def build(force: bool = True) -> Path:
    """Compile the C oracle with gcc (plain FP64, no FMA contraction)."""
    if force or _stale():
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                        "-fPIC", "-shared", "-o", str(tmp), str(_SRC), str(_SRC2), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _stale() -> bool:
    if not _LIB.exists():
        return True
    t = _LIB.stat().st_mtime
    return t < _SRC.stat().st_mtime or t < _SRC2.stat().st_mtime


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _stale():
        build(force=True)
    L = ctypes.CDLL(str(_LIB))
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.orc_mesh_create.restype = P
    L.orc_mesh_create.argtypes = [P, i64, P, i64, P]
    L.orc_mesh_free.argtypes = [P]
    L.orc_mesh_ndof.restype = i64
    L.orc_mesh_ndof.argtypes = [P]
    L.orc_mesh_dof.argtypes = [P, P]
    L.orc_mesh_nbr.argtypes = [P, P]
    L.orc_mesh_affine.argtypes = [P, P, P]
    L.orc_quadrature.argtypes = [i32, P, P]
    L.orc_gauss_points.argtypes = [P, i32, P, P]
    L.orc_paths.argtypes = [P, i32, i64, i64, i32, P, P, P, P]
    L.orc_exit_pattern.argtypes = [P, i64, P, i32, i32, P, P]
    L.orc_ray_values.argtypes = [P, i32, i64, i32, i32, dbl, dbl, dbl, dbl, i32, i32, P, P]
    L.orc_assemble.argtypes = [P, i32, dbl, dbl, dbl, P, i32, P]
    L.orc_assemble_div.argtypes = [P, i32, P, P, P, i32, P]
    L.orc_assemble_div_rows.argtypes = [P, i32, P, P, P, i32, i64, P, P]
    L.orc_assemble_form.argtypes = [P, i32, P, P, P, P, P, i32, P]
    L.orc_assemble_form_rows.argtypes = [P, i32, P, P, P, P, P, i32, i64, P, P]
    # two dimensions
    L.o2_mesh_create.restype = P
    L.o2_mesh_create.argtypes = [P, i64, P, i64, P]
    L.o2_mesh_free.argtypes = [P]
    L.o2_mesh_ndof.restype = i64
    L.o2_mesh_ndof.argtypes = [P]
    L.o2_mesh_dof.argtypes = [P, P]
    L.o2_mesh_nbr.argtypes = [P, P]
    L.o2_mesh_affine.argtypes = [P, P, P]
    L.o2_quadrature.argtypes = [i32, P, P]
    L.o2_gauss_points.argtypes = [P, i32, P, P]
    L.o2_paths.argtypes = [P, i32, i64, i64, i32, P, P, P, P]
    L.o2_walk_from.argtypes = [P, i64, P, i32, i32, i32, P, P, P]
    L.o2_ray_values.argtypes = [P, i32, i64, i32, i32, dbl, dbl, dbl, i32, i32, P, P]
    L.o2_assemble.argtypes = [P, i32, dbl, dbl, dbl, P, i32, P]
    L.o2_load.argtypes = [P, i32, P, P]
    L.o2_exhaustive.argtypes = [P, P, P, P, P]
    L.orc_apply.argtypes = [P, i32, dbl, dbl, dbl, P, i32, P, P]
    L.orc_apply_range.argtypes = [P, i32, dbl, dbl, dbl, P, i32, P, i64, i64, P]
    L.orc_operator_create.restype = P
    L.orc_operator_create.argtypes = [P, i32, dbl, dbl, dbl, P, i32, P]
    L.orc_operator_free.argtypes = [P]
    L.orc_operator_apply.argtypes = [P, P, P]
    L.orc_operator_diagonal.argtypes = [P, P]
    L.orc_operator_entries.restype = i64
    L.orc_operator_entries.argtypes = [P]
    L.orc_set_threads.argtypes = [i32]
    L.orc_set_threads.restype = i32
    L.orc_adjoint_sums.argtypes = [P, i32, dbl, dbl, dbl, i32, P, P, P, P]
    L.orc_load.argtypes = [P, i32, P, P]
    L.orc_exhaustive.argtypes = [P, P, P, P, P]
    L.orc_walk_from.argtypes = [P, i64, P, i32, i32, i32, P, P, P]
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__(f"oracle status {status} {what}")
        self.status = status


# --------------------------------------------------------------------------
# Closed-form scalars
# --------------------------------------------------------------------------
def c_alpha(alpha: float) -> float:
    """c_alpha = 1 / (2 cos(pi alpha / 2)): minus the Riesz normalisation."""
    return 1.0 / (2.0 * math.cos(math.pi * alpha / 2.0))


def dc_alpha(alpha: float) -> float:
    """d c_alpha / d alpha = (pi/4) sin(pi alpha/2) / cos^2(pi alpha/2)."""
    c = math.cos(math.pi * alpha / 2.0)
    return (math.pi / 4.0) * math.sin(math.pi * alpha / 2.0) / (c * c)


def order_scalars(alpha: float):
    """gamma = alpha/2, 1/Gamma(2-gamma), 1/Gamma(1-gamma), psi(2-gamma)/2."""
    from scipy.special import rgamma, digamma
    g = alpha / 2.0
    return g, float(rgamma(2.0 - g)), float(rgamma(1.0 - g)), 0.5 * float(digamma(2.0 - g))


def quadrature(nq: int):
    L = _load()
    bary = np.zeros((nq, 4))
    w = np.zeros(nq)
    st = L.orc_quadrature(nq, _p(bary), _p(w))
    if st != 0:
        raise OracleError(st, f"no {nq}-point rule")
    return bary, w


# --------------------------------------------------------------------------
# Mesh-bound operations
# --------------------------------------------------------------------------
class OracleMesh:
    def __init__(self, xyz, tet, cap: int = DEFAULT_CAP):
        L = _load()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tet = np.ascontiguousarray(tet, dtype=np.int32)
        self.cap = int(cap)
        st = ctypes.c_int(0)
        h = L.orc_mesh_create(_p(self.xyz), self.xyz.shape[0], _p(self.tet), self.tet.shape[0],
                              ctypes.byref(st))
        if not h:
            raise OracleError(st.value, "mesh")
        self._h = ctypes.c_void_p(h)
        self.n_vert = self.xyz.shape[0]
        self.n_tet = self.tet.shape[0]
        self.ndof = int(L.orc_mesh_ndof(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_mesh_free(self._h)
            self._h = None

    # mesh data -----------------------------------------------------------
    @property
    def dof(self) -> np.ndarray:
        out = np.empty(self.n_vert, dtype=np.int32)
        _lib.orc_mesh_dof(self._h, _p(out))
        return out

    @property
    def nbr(self) -> np.ndarray:
        out = np.empty((self.n_tet, 4), dtype=np.int32)
        _lib.orc_mesh_nbr(self._h, _p(out))
        return out

    def affine(self):
        M = np.empty((self.n_tet, 3, 3))
        vol = np.empty(self.n_tet)
        _lib.orc_mesh_affine(self._h, _p(M), _p(vol))
        return M, vol

    def gauss_points(self, nq: int):
        G = self.n_tet * nq
        x = np.empty((G, 3))
        w = np.empty(G)
        st = _lib.orc_gauss_points(self._h, nq, _p(x), _p(w))
        if st != 0:
            raise OracleError(st)
        return x, w

    # template (Sec. 2.3) ---------------------------------------------------
    def patch_boxes(self):
        """Axis-aligned bounding box of the element patch omega_j (the union of
        the elements containing node z_j, Sec. 2.3) of every interior node:
        (lo, hi), each (ndof, 3), by min / max over the patch's vertices."""
        dof = self.dof
        lo = np.full((self.ndof, 3), np.inf)
        hi = np.full((self.ndof, 3), -np.inf)
        pts = self.xyz[self.tet]
        elo, ehi = pts.min(axis=1), pts.max(axis=1)
        for m in range(4):
            d = dof[self.tet[:, m]]
            ok = d >= 0
            np.minimum.at(lo, d[ok], elo[ok])
            np.maximum.at(hi, d[ok], ehi[ok])
        return lo, hi

    def template(self) -> np.ndarray:
        """The template T of Sec. 2.3 as a dense boolean matrix.

        T_jk is set when, for some axis i, the patch boxes of j and k overlap
        (closed intervals) in both coordinates other than i: only then can a
        line parallel to e_i meet both supports.  When it is clear for every
        i, every chord misses one of the two supports and K_jk = 0, so T is a
        superset of the nonzero pattern of K.  (The printed criterion, one
        overlap test in the coordinate i itself, is garbled; this is the
        reading used.)"""
        lo, hi = self.patch_boxes()
        ov = (lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :])
        T = np.zeros((self.ndof, self.ndof), dtype=bool)
        for i in range(3):
            T |= ov[:, :, (i + 1) % 3] & ov[:, :, (i + 2) % 3]
        return T

    def template_tiles(self, tile: int) -> np.ndarray:
        """T at tile granularity: (nt, nt) uint8, 1 when any (j, k) of the tile is set."""
        T = self.template()
        nt = -(-self.ndof // tile)
        out = np.zeros((nt, nt), dtype=np.uint8)
        for P in range(nt):
            for Q in range(nt):
                out[P, Q] = T[P * tile:(P + 1) * tile, Q * tile:(Q + 1) * tile].any()
        return out

    # paths ---------------------------------------------------------------
    def paths(self, nq: int, h0: int = 0, count: int | None = None, lists: bool = False):
        """Half-ray h = g*6 + 2*i + side: (length, FNV-1a hash[, ids, r_end])."""
        if count is None:
            count = self.n_tet * nq * 6 - h0
        ln = np.zeros(count, dtype=np.int32)
        hs = np.zeros(count, dtype=np.uint64)
        ids = np.full((count, self.cap), -1, dtype=np.int32) if lists else None
        rend = np.zeros((count, self.cap)) if lists else None
        st = _lib.orc_paths(self._h, nq, h0, count, self.cap, _p(ln), _p(hs),
                            _p(ids) if lists else None, _p(rend) if lists else None)
        if st != 0:
            raise OracleError(st, "paths")
        if lists:
            return ln, hs, ids, rend
        return ln, hs

    def exit_pattern(self, t: int, u0, i: int, s: int):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        k = np.zeros(4)
        rr = np.zeros(2)
        z = _lib.orc_exit_pattern(self._h, t, _p(u0), i, s, _p(k), _p(rr))
        return z, k, rr

    def walk(self, t0: int, u0, i: int, s: int):
        """Path of the ray u0 + r s e_i from inside element t0: (ids, r_end)."""
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        ids = np.empty(self.cap, dtype=np.int32)
        rend = np.empty(self.cap)
        n = ctypes.c_int(0)
        st = _lib.orc_walk_from(self._h, t0, _p(u0), i, s, self.cap, _p(ids), _p(rend), ctypes.byref(n))
        if st != 0:
            raise OracleError(st, "walk")
        return ids[: n.value].copy(), rend[: n.value].copy()

    def exhaustive(self, u0, d):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        lo = np.empty(self.n_tet)
        hi = np.empty(self.n_tet)
        _lib.orc_exhaustive(self._h, _p(u0), _p(d), _p(lo), _p(hi))
        return lo, hi

    # derivative vectors --------------------------------------------------
    def ray_values(self, nq: int, g: int, i: int, side: int, alpha: float, mode: int = 0):
        """mode 0: interior dofs; 1: all vertices with the end-point term;
        2: d/dalpha of mode 0."""
        gm, ig2, ig1, hp = order_scalars(alpha)
        ids = np.empty(4 * self.cap, dtype=np.int32)
        vals = np.empty(4 * self.cap)
        n = _lib.orc_ray_values(self._h, nq, g, i, side, gm, ig2, ig1, hp, mode, self.cap,
                                _p(ids), _p(vals))
        if n < 0:
            raise OracleError(n, "ray")
        return ids[:n].copy(), vals[:n].copy()

    # assembly ------------------------------------------------------------
    def assemble(self, nq: int, alpha: float, K=(1.0, 1.0, 1.0)) -> np.ndarray:
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        A = np.zeros((self.ndof, self.ndof))
        st = _lib.orc_assemble(self._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), self.cap, _p(A))
        if st != 0:
            raise OracleError(st, "assemble")
        return A

    def assemble_div(self, nq: int, beta, pq=None, rows=None) -> np.ndarray:
        """Non-symmetric matrix of the divergence-form problem of Sec. 3:
        K_jk = a(psi_k, psi_j) with trial derivatives of order beta_i along
        e_i and the classical d_i psi_j of the own element on the test side.
        pq: (6, G) with p_i(x_g) in rows 0..2 and q_i(x_g) in rows 3..5;
        default the coefficients of Sec. 3 (div_coefficients).  rows: only
        these rows (len(rows) x ndof), else the whole matrix."""
        beta = np.asarray(beta, dtype=np.float64)
        if pq is None:
            x, _ = self.gauss_points(nq)
            pq = div_coefficients(x)
        pq = np.ascontiguousarray(pq, dtype=np.float64)
        if pq.shape != (6, self.n_tet * nq):
            raise ValueError("pq must be (6, G)")
        gm = np.ascontiguousarray(beta)
        ig2 = np.array([rgamma_(2.0 - b) for b in beta])
        if rows is None:
            A = np.zeros((self.ndof, self.ndof))
            st = _lib.orc_assemble_div(self._h, nq, _p(gm), _p(ig2), _p(pq), self.cap, _p(A))
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            A = np.zeros((len(rows), self.ndof))
            st = _lib.orc_assemble_div_rows(self._h, nq, _p(gm), _p(ig2), _p(pq), self.cap, len(rows),
                                            _p(rows), _p(A))
        if st != 0:
            raise OracleError(st, "assemble_div")
        return A

    def assemble_form(self, nq: int, alpha, beta, coef, rows=None) -> np.ndarray:
        """The uniform form of Sec. 1 (eq. equ:varsss), test operator on the
        side opposite to the trial one:
        K_kl = sum_i sum_g w_g [cl_i D_L^{alpha_i} psi_l D_R^{beta_i} psi_k
                                + cr_i D_R^{alpha_i} psi_l D_L^{beta_i} psi_k](x_g),
        orders in [0, 1] per axis; coef: (6, G) with cl_i in rows 0..2 and
        cr_i in rows 3..5, or 6 constants.  rows: only these rows
        (len(rows) x ndof), else the whole matrix."""
        G = self.n_tet * nq
        coef = np.asarray(coef, dtype=np.float64)
        if coef.shape == (6,):
            coef = np.repeat(coef[:, None], G, axis=1)
        coef = np.ascontiguousarray(coef)
        if coef.shape != (6, G):
            raise ValueError("coef must be (6,) or (6, G)")
        ga = np.ascontiguousarray(alpha, dtype=np.float64)
        gb = np.ascontiguousarray(beta, dtype=np.float64)
        iga = np.array([rgamma_(2.0 - a) for a in ga])
        igb = np.array([rgamma_(2.0 - b) for b in gb])
        if rows is None:
            A = np.zeros((self.ndof, self.ndof))
            st = _lib.orc_assemble_form(self._h, nq, _p(ga), _p(iga), _p(gb), _p(igb), _p(coef), self.cap, _p(A))
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            A = np.zeros((len(rows), self.ndof))
            st = _lib.orc_assemble_form_rows(self._h, nq, _p(ga), _p(iga), _p(gb), _p(igb), _p(coef), self.cap,
                                             len(rows), _p(rows), _p(A))
        if st != 0:
            raise OracleError(st, "assemble_form")
        return A

    def apply(self, nq: int, alpha: float, K, x) -> np.ndarray:
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.ndof)
        st = _lib.orc_apply(self._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), self.cap, _p(x), _p(y))
        if st != 0:
            raise OracleError(st, "apply")
        return y

    def apply_range(self, nq: int, alpha: float, K, x, g0: int, g1: int) -> np.ndarray:
        """The part of K x summed over the Gauss points g0 <= g < g1 only."""
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.ndof)
        st = _lib.orc_apply_range(self._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), self.cap, _p(x), int(g0), int(g1),
                                  _p(y))
        if st != 0:
            raise OracleError(st, "apply_range")
        return y

    def load(self, nq: int, f_gauss=None) -> np.ndarray:
        b = np.zeros(self.ndof)
        f = None if f_gauss is None else np.ascontiguousarray(f_gauss, dtype=np.float64)
        st = _lib.orc_load(self._h, nq, _p(f) if f is not None else None, _p(b))
        if st != 0:
            raise OracleError(st, "load")
        return b

    def adjoint_sums(self, nq: int, alpha: float, u, lam):
        gm, ig2, _, hp = order_scalars(alpha)
        u = np.ascontiguousarray(u, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        S = np.zeros(3)
        T = np.zeros(3)
        st = _lib.orc_adjoint_sums(self._h, nq, gm, ig2, hp, self.cap, _p(u), _p(lam), _p(S), _p(T))
        if st != 0:
            raise OracleError(st, "adjoint")
        return S, T

    # whole problems ------------------------------------------------------
    def gradient(self, nq: int, alpha: float, K, u, gbar, A=None):
        """d(loss)/d(alpha), d(loss)/dK for u = A(alpha,K)^{-1} b with
        dloss/du = gbar: lam = A^{-1} gbar, dJ/dtheta = -lam^T (dA/dtheta) u."""
        if A is None:
            A = self.assemble(nq, alpha, K)
        lam = solve_spd(A, gbar)
        S, T = self.adjoint_sums(nq, alpha, u, lam)
        ca, dca = c_alpha(alpha), dc_alpha(alpha)
        K = np.asarray(K, dtype=np.float64)
        dK = -ca * S
        da = -float(np.sum(K * (dca * S + ca * T)))
        return da, dK


# --------------------------------------------------------------------------
# The two-dimensional variant (n = 2): triangles, paths along +-e_1, +-e_2
# --------------------------------------------------------------------------
def quadrature2d(nq: int):
    L = _load()
    bary = np.empty(3 * nq)
    w = np.empty(nq)
    if L.o2_quadrature(nq, _p(bary), _p(w)) != 0:
        raise OracleError(-1, "quadrature2d")
    return bary.reshape(nq, 3), w


class OracleMesh2D:
    def __init__(self, xy, tri, cap: int = DEFAULT_CAP):
        L = _load()
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.cap = int(cap)
        st = ctypes.c_int(0)
        h = L.o2_mesh_create(_p(self.xy), self.xy.shape[0], _p(self.tri), self.tri.shape[0], ctypes.byref(st))
        if not h:
            raise OracleError(st.value, "mesh2d")
        self._h = ctypes.c_void_p(h)
        self.n_vert = self.xy.shape[0]
        self.n_tri = self.tri.shape[0]
        self.ndof = int(L.o2_mesh_ndof(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.o2_mesh_free(self._h)
            self._h = None

    @property
    def dof(self) -> np.ndarray:
        out = np.empty(self.n_vert, dtype=np.int32)
        _lib.o2_mesh_dof(self._h, _p(out))
        return out

    @property
    def nbr(self) -> np.ndarray:
        out = np.empty((self.n_tri, 3), dtype=np.int32)
        _lib.o2_mesh_nbr(self._h, _p(out))
        return out

    def affine(self):
        M = np.empty((self.n_tri, 2, 2))
        area = np.empty(self.n_tri)
        _lib.o2_mesh_affine(self._h, _p(M), _p(area))
        return M, area

    def gauss_points(self, nq: int):
        G = self.n_tri * nq
        x = np.empty((G, 2))
        w = np.empty(G)
        if _lib.o2_gauss_points(self._h, nq, _p(x), _p(w)) != 0:
            raise OracleError(-1, "gauss2d")
        return x, w

    def paths(self, nq: int, h0: int = 0, count: int | None = None, lists: bool = False):
        """Half-ray h = g*4 + 2*i + side: (length, FNV-1a hash[, ids, r_end])."""
        if count is None:
            count = self.n_tri * nq * 4 - h0
        ln = np.zeros(count, dtype=np.int32)
        hs = np.zeros(count, dtype=np.uint64)
        ids = np.full((count, self.cap), -1, dtype=np.int32) if lists else None
        rend = np.zeros((count, self.cap)) if lists else None
        st = _lib.o2_paths(self._h, nq, h0, count, self.cap, _p(ln), _p(hs),
                           _p(ids) if lists else None, _p(rend) if lists else None)
        if st != 0:
            raise OracleError(st, "paths2d")
        return (ln, hs, ids, rend) if lists else (ln, hs)

    def walk(self, t0: int, u0, i: int, s: int):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        ids = np.empty(self.cap, dtype=np.int32)
        rend = np.empty(self.cap)
        n = ctypes.c_int(0)
        st = _lib.o2_walk_from(self._h, t0, _p(u0), i, s, self.cap, _p(ids), _p(rend), ctypes.byref(n))
        if st != 0:
            raise OracleError(st, "walk2d")
        return ids[: n.value].copy(), rend[: n.value].copy()

    def exhaustive(self, u0, d):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        lo = np.empty(self.n_tri)
        hi = np.empty(self.n_tri)
        _lib.o2_exhaustive(self._h, _p(u0), _p(d), _p(lo), _p(hi))
        return lo, hi

    def ray_values(self, nq: int, g: int, i: int, side: int, alpha: float, mode: int = 0):
        gm, ig2, ig1, _ = order_scalars(alpha)
        ids = np.empty(3 * self.cap, dtype=np.int32)
        vals = np.empty(3 * self.cap)
        n = _lib.o2_ray_values(self._h, nq, g, i, side, gm, ig2, ig1, mode, self.cap, _p(ids), _p(vals))
        if n < 0:
            raise OracleError(n, "ray2d")
        return ids[:n].copy(), vals[:n].copy()

    def assemble(self, nq: int, alpha: float, K=(1.0, 1.0)) -> np.ndarray:
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        A = np.zeros((self.ndof, self.ndof))
        st = _lib.o2_assemble(self._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), self.cap, _p(A))
        if st != 0:
            raise OracleError(st, "assemble2d")
        return A

    def apply_range(self, nq: int, alpha: float, K, x, g0: int, g1: int) -> np.ndarray:
        """The part of K x summed over the Gauss points g0 <= g < g1 only."""
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.ndof)
        st = _lib.orc_apply_range(self._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), self.cap, _p(x), int(g0), int(g1),
                                  _p(y))
        if st != 0:
            raise OracleError(st, "apply_range")
        return y

    def load(self, nq: int, f_gauss=None) -> np.ndarray:
        b = np.zeros(self.ndof)
        f = None if f_gauss is None else np.ascontiguousarray(f_gauss, dtype=np.float64)
        if _lib.o2_load(self._h, nq, _p(f) if f is not None else None, _p(b)) != 0:
            raise OracleError(-1, "load2d")
        return b


def mms_exact2d(x: np.ndarray) -> np.ndarray:
    return mms_phi(x[:, 0]) * mms_phi(x[:, 1])


def mms_source2d(x: np.ndarray, alpha: float, K=(1.0, 1.0)) -> np.ndarray:
    """Source of u = phi(x) phi(y) on the unit square for the Riesz problem:
    f = sum_i K_i c_alpha [Phi(x_i) + Phi(1 - x_i)] phi(x_other)."""
    ca = c_alpha(alpha)
    ph = [mms_phi(x[:, 0]), mms_phi(x[:, 1])]
    return sum(K[i] * ca * (mms_Phi(x[:, i], alpha) + mms_Phi(1.0 - x[:, i], alpha)) * ph[1 - i]
               for i in range(2))


def l2_error2d(mesh: OracleMesh2D, u_dof: np.ndarray, exact, nq: int = 7) -> float:
    bary, _ = quadrature2d(nq)
    x, w = mesh.gauss_points(nq)
    dof = mesh.dof
    full = np.zeros(mesh.n_vert)
    full[dof >= 0] = u_dof[dof[dof >= 0]]
    uh = np.einsum("qj,tj->tq", bary, full[mesh.tri]).reshape(-1)
    e = exact(x) - uh
    return math.sqrt(float(np.sum(w * e * e)))


class OracleOperator:
    """The stiffness matrix of OracleMesh.apply as an operator whose
    derivative vectors are walked once and kept (host memory: 12 bytes per
    entry), for repeated products (conjugate gradients at large N)."""

    def __init__(self, mesh: OracleMesh, nq: int, alpha: float, K=(1.0, 1.0, 1.0)):
        gm, ig2, _, _ = order_scalars(alpha)
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        st = ctypes.c_int(0)
        h = _lib.orc_operator_create(mesh._h, nq, gm, ig2, c_alpha(alpha), _p(Kc), mesh.cap, ctypes.byref(st))
        if not h:
            raise OracleError(st.value, "operator")
        self._h = ctypes.c_void_p(h)
        self.n = mesh.ndof
        self.entries = int(_lib.orc_operator_entries(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_operator_free(self._h)
            self._h = None

    def apply(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        _lib.orc_operator_apply(self._h, _p(x), _p(y))
        return y

    def diagonal(self) -> np.ndarray:
        d = np.zeros(self.n)
        _lib.orc_operator_diagonal(self._h, _p(d))
        return d


# --------------------------------------------------------------------------
# Solves (textbook routines)
# --------------------------------------------------------------------------
def set_threads(n: int = 0) -> int:
    """OpenMP threads of the oracle's parallel loops (the matrix-free
    product, the row-restricted forms); n <= 0 only reports the count."""
    return int(_load().orc_set_threads(int(n)))


def solve_spd(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """LAPACK Cholesky (dpotrf/dpotrs via SciPy)."""
    from scipy.linalg import cho_factor, cho_solve
    return cho_solve(cho_factor(A, lower=True), b)


def cg(apply, b: np.ndarray, tol: float = 1e-13, maxiter: int = 10000, dinv=None):
    """Conjugate gradients on a symmetric positive definite operator, stopped
    at ||r|| <= tol ||b||; with dinv (the inverse of K's diagonal) the Jacobi
    preconditioned variant (the textbook recurrences with z = dinv r)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = r if dinv is None else dinv * r
    p = z.copy()
    rz = float(r @ z)
    bn = math.sqrt(float(b @ b))
    it = 0
    while math.sqrt(float(r @ r)) > tol * bn and it < maxiter:
        q = apply(p)
        a = rz / float(p @ q)
        x += a * p
        r -= a * q
        z = r if dinv is None else dinv * r
        rz2 = float(r @ z)
        p = z + (rz2 / rz) * p
        rz = rz2
        it += 1
    return x, it


# --------------------------------------------------------------------------
# Manufactured solution on the unit cube
# --------------------------------------------------------------------------
def mms_phi(s):
    return s * s * (1.0 - s) ** 2


def mms_Phi(s, alpha: float):
    """Left RL derivative of order alpha of s^2 - 2 s^3 + s^4 from 0:
    D^alpha s^n = Gamma(n+1)/Gamma(n+1-alpha) s^(n-alpha)."""
    from scipy.special import rgamma
    s = np.asarray(s, dtype=np.float64)
    return (2.0 * s ** (2 - alpha) * rgamma(3 - alpha)
            - 12.0 * s ** (3 - alpha) * rgamma(4 - alpha)
            + 24.0 * s ** (4 - alpha) * rgamma(5 - alpha))


def mms_exact(x: np.ndarray) -> np.ndarray:
    return mms_phi(x[:, 0]) * mms_phi(x[:, 1]) * mms_phi(x[:, 2])


def mms_source(x: np.ndarray, alpha: float, K=(1.0, 1.0, 1.0)) -> np.ndarray:
    """f = sum_i K_i c_alpha [Phi(x_i) + Phi(1 - x_i)] prod_{m != i} phi(x_m)."""
    ca = c_alpha(alpha)
    f = np.zeros(x.shape[0])
    ph = [mms_phi(x[:, d]) for d in range(3)]
    for i in range(3):
        other = np.ones(x.shape[0])
        for d in range(3):
            if d != i:
                other = other * ph[d]
        f += K[i] * ca * (mms_Phi(x[:, i], alpha) + mms_Phi(1.0 - x[:, i], alpha)) * other
    return f


# --------------------------------------------------------------------------
# The divergence-form problem of Sec. 3 on the ball |x| < r
# --------------------------------------------------------------------------
def rgamma_(z: float) -> float:
    from scipy.special import rgamma
    return float(rgamma(z))


def div_coefficients(x: np.ndarray) -> np.ndarray:
    """p_i = cos x_i, q_i = 1 - cos x_i at the points x (G, 3) (Sec. 3), as
    the (6, G) array the assembly takes."""
    c = np.cos(x.T)
    return np.ascontiguousarray(np.concatenate([c, 1.0 - c]))


def ball_exact(x: np.ndarray, r: float = 0.5) -> np.ndarray:
    """u = (|x|^2 - r^2)^2 inside the ball, 0 outside (Sec. 3)."""
    s = np.sum(x * x, axis=1) - r * r
    return np.where(s < 0.0, s * s, 0.0)


def _chord_Phi(s, c, beta, deriv: bool):
    """On the chord of half-length c the exact solution is, in the distance s
    from either end, s^2 (s - 2c)^2 = s^4 - 4 c s^3 + 4 c^2 s^2; its order-beta
    Riemann-Liouville derivative from that end (term by term,
    D^beta s^n = Gamma(n+1)/Gamma(n+1-beta) s^(n-beta)) and, with deriv,
    the s-derivative of that."""
    g = rgamma_
    if deriv:
        return (8.0 * c * c * g(2.0 - beta) * s ** (1.0 - beta)
                - 24.0 * c * g(3.0 - beta) * s ** (2.0 - beta)
                + 24.0 * g(4.0 - beta) * s ** (3.0 - beta))
    return (8.0 * c * c * g(3.0 - beta) * s ** (2.0 - beta)
            - 24.0 * c * g(4.0 - beta) * s ** (3.0 - beta)
            + 24.0 * g(5.0 - beta) * s ** (4.0 - beta))


def ball_flux(x: np.ndarray, beta, r: float = 0.5, i: int = 0):
    """(D_L^{beta_i} u, D_R^{beta_i} u) along e_i at x for the exact solution:
    the chord through x is |y_i| <= c with c^2 = r^2 - sum_{m != i} x_m^2."""
    c2 = r * r - (np.sum(x * x, axis=1) - x[:, i] ** 2)
    c = np.sqrt(np.maximum(c2, 0.0))
    xi = np.maximum(x[:, i] + c, 0.0)
    eta = np.maximum(c - x[:, i], 0.0)
    b = float(beta[i])
    return _chord_Phi(xi, c, b, False), _chord_Phi(eta, c, b, False)


def ball_source(x: np.ndarray, beta, r: float = 0.5) -> np.ndarray:
    """f = sum_i D_i (p_i D_L^{beta_i} u - q_i D_R^{beta_i} u) for the exact
    solution and the coefficients of Sec. 3, by the product rule:
    D_i [cos x_i Phi(xi)] - D_i [(1 - cos x_i) Phi(eta)] with xi = x_i + c and
    eta = c - x_i the distances to the chord ends (d eta / d x_i = -1)."""
    f = np.zeros(x.shape[0])
    for i in range(3):
        c2 = r * r - (np.sum(x * x, axis=1) - x[:, i] ** 2)
        c = np.sqrt(np.maximum(c2, 0.0))
        xi = np.maximum(x[:, i] + c, 0.0)
        eta = np.maximum(c - x[:, i], 0.0)
        b = float(beta[i])
        s, co = np.sin(x[:, i]), np.cos(x[:, i])
        f += (-s * _chord_Phi(xi, c, b, False) + co * _chord_Phi(xi, c, b, True)
              - s * _chord_Phi(eta, c, b, False) + (1.0 - co) * _chord_Phi(eta, c, b, True))
    return f


def solve_div(mesh: OracleMesh, nq: int, beta, r: float = 0.5, f_gauss=None):
    """K, b and u = K^{-1} b for the problem of Sec. 3 (LAPACK LU with partial
    pivoting; K is not symmetric).  f defaults to the exact solution's source."""
    from scipy.linalg import lu_factor, lu_solve
    K = mesh.assemble_div(nq, beta)
    if f_gauss is None:
        x, _ = mesh.gauss_points(nq)
        f_gauss = ball_source(x, beta, r)
    b = mesh.load(nq, f_gauss)
    return K, b, lu_solve(lu_factor(K), b)


def solve_problem(mesh: OracleMesh, nq: int, alpha: float, K=(1.0, 1.0, 1.0), f_gauss=None):
    A = mesh.assemble(nq, alpha, K)
    b = mesh.load(nq, f_gauss)
    return A, b, solve_spd(A, b)


def nodal_full(mesh: OracleMesh, u_dof: np.ndarray) -> np.ndarray:
    """Nodal values on all vertices (zero on the boundary)."""
    dof = mesh.dof
    full = np.zeros(mesh.n_vert)
    full[dof >= 0] = u_dof[dof[dof >= 0]]
    return full


def l2_error(mesh: OracleMesh, u_dof: np.ndarray, exact, nq: int = 11) -> float:
    """||u - u_h||_{L2} with the nq-point rule on every element."""
    bary, _ = quadrature(nq)
    x, w = mesh.gauss_points(nq)
    full = nodal_full(mesh, u_dof)
    uh = np.einsum("qj,tj->tq", bary, full[mesh.tet]).reshape(-1)
    e = exact(x) - uh
    return math.sqrt(float(np.sum(w * e * e)))


def h_max(mesh: OracleMesh) -> float:
    p = mesh.xyz[mesh.tet]
    h = 0.0
    for a in range(4):
        for b in range(a + 1, 4):
            h = max(h, float(np.linalg.norm(p[:, a] - p[:, b], axis=1).max()))
    return h
