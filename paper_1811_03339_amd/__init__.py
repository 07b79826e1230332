"""MI355X (gfx950) library for the 3-D P1 finite-element discretisation of
steady Riesz fractional diffusion (Yang, Nie, Yuan & Wang, "Finite Element
Methods for Fractional PDEs in Three Dimensions").

Thin ctypes binding of ``libfpde.so`` (C ABI declared in ``include/fpde.h``):
argument marshalling only.  Every step (mesh set-up, path walk, closed-form
derivatives, accumulation, load vector, Cholesky, refinement, adjoint, and for
the divergence-form problem of Sec. 3 its accumulation and LU) runs in the
library's HIP kernels; PyTorch supplies device memory and the stream.
If the library is missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libfpde.so"

FPDE_OK = 0
FPDE_FP64, FPDE_MIXED = 0, 1
FPDE_SRC_ONE, FPDE_SRC_USER, FPDE_SRC_CUBE_MMS, FPDE_SRC_BALL_MMS, FPDE_SRC_SQUARE_MMS = 0, 1, 2, 3, 4
FPDE_COEF_SEC3, FPDE_COEF_USER, FPDE_COEF_CONST = 0, 1, 2

STATUS = {
    0: "FPDE_OK", -1: "FPDE_EINVAL", -2: "FPDE_EMESH_NONMANIFOLD", -3: "FPDE_EMESH_DEGENERATE", -4: "FPDE_EMESH_NONCONVEX",
    -5: "FPDE_EPATH", -6: "FPDE_EALPHA", -7: "FPDE_ENOTSPD", -8: "FPDE_ENOCONV", -9: "FPDE_EHIP",
    -10: "FPDE_ENOMEM", -11: "FPDE_EUNSUPPORTED", -12: "FPDE_ESINGULAR",
}

EXPORTS = [
    "fpde_status_string", "fpde_mesh_create", "fpde_mesh_destroy", "fpde_mesh_info", "fpde_dof_map",
    "fpde_plan", "fpde_paths", "fpde_ray_values", "fpde_assemble", "fpde_apply", "fpde_solve",
    "fpde_solve_factored", "fpde_adjoint", "fpde_timing", "fpde_timing_stages", "fpde_stage_times", "fpde_plan_info",
    "fpde_template", "fpde_div_assemble", "fpde_lu_factor", "fpde_lu_solve", "fpde_template_csr",
    "fpde_assemble_csr", "fpde_csr_apply", "fpde_cg_solve", "fpde_form_assemble", "fpde_mesh2d_create",
    "fpde_mesh2d_destroy", "fpde_mesh2d_info", "fpde_dof_map2d", "fpde_paths2d", "fpde_assemble2d",
    "fpde_solve2d", "fpde_timing2d", "fpde_stage_times2d", "fpde_solve_batch", "fpde_assemble_batch",
    "fpde_solve_noalloc",
]

STAGES = ["walk", "contract", "load", "potrf", "trsv", "apply", "plan", "adjoint", "accum", "lu", "div", "spmv",
          "cg", "form"]


class FpdeError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        name = STATUS.get(status, str(status))
        text = ""
        try:
            text = _lib().fpde_status_string(status).decode()
        except Exception:  # noqa: BLE001 - message only
            pass
        super().__init__(f"{what}: {name} ({text})")
        self.status = status


class fpde_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("K", ctypes.c_double * 3), ("quad_points", ctypes.c_int),
                ("precision", ctypes.c_int), ("source", ctypes.c_int), ("max_steps", ctypes.c_int),
                ("ir_tol", ctypes.c_double), ("ir_max_iter", ctypes.c_int), ("deterministic", ctypes.c_int)]


class fpde_div_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double * 3), ("quad_points", ctypes.c_int), ("coef", ctypes.c_int),
                ("source", ctypes.c_int), ("radius", ctypes.c_double), ("max_steps", ctypes.c_int)]


class fpde_form_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double * 3), ("beta", ctypes.c_double * 3), ("quad_points", ctypes.c_int),
                ("coef", ctypes.c_int), ("cl", ctypes.c_double * 3), ("cr", ctypes.c_double * 3),
                ("max_steps", ctypes.c_int)]


class fpde_params2d(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("K", ctypes.c_double * 2), ("quad_points", ctypes.c_int),
                ("source", ctypes.c_int), ("max_steps", ctypes.c_int)]


class fpde_solve_info(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int), ("final_rel_residual", ctypes.c_double),
                ("failed_pivot", ctypes.c_int64)]


_L = None


def _lib():
    global _L
    if _L is not None:
        return _L
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1811_03339_amd.build")
    L = ctypes.CDLL(str(LIB_PATH))
    P, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.fpde_status_string.restype = ctypes.c_char_p
    L.fpde_status_string.argtypes = [i32]
    L.fpde_mesh_create.argtypes = [P, i64, P, i64, P, ctypes.POINTER(P)]
    L.fpde_mesh_destroy.argtypes = [P]
    L.fpde_mesh_destroy.restype = None
    L.fpde_mesh_info.argtypes = [P, P, P, P]
    L.fpde_dof_map.argtypes = [P, P]
    L.fpde_plan.argtypes = [P, i32, i32, P]
    L.fpde_paths.argtypes = [P, i32, i32, i64, i64, i32, P, P, P, P, P]
    L.fpde_ray_values.argtypes = [P, i32, dbl, i32, i64, i64, P, P, P, i64, P]
    L.fpde_assemble.argtypes = [P, P, P, i64, P, P, P]
    L.fpde_apply.argtypes = [P, P, P, P, P]
    L.fpde_solve.argtypes = [P, P, P, i64, P, P, P, P]
    L.fpde_solve_factored.argtypes = [P, P, P, i64, P, P, P, P]
    L.fpde_solve_batch.argtypes = [P, i32, P, i64, i64, P, P, i64, P, P]
    L.fpde_solve_noalloc.argtypes = [P, P, i64, P, P, P, P]
    L.fpde_assemble_batch.argtypes = [P, i32, P, P, i64, i64, P, i64, P]
    L.fpde_adjoint.argtypes = [P, P, P, P, P, P, P]
    L.fpde_timing.argtypes = [P, i32]
    L.fpde_timing_stages.argtypes = [P, ctypes.c_uint]
    L.fpde_stage_times.argtypes = [P, P, P]
    L.fpde_plan_info.argtypes = [P, i32, P, P]
    L.fpde_template.argtypes = [P, i32, P, P, P]
    L.fpde_div_assemble.argtypes = [P, P, P, P, i64, P, P, P]
    L.fpde_lu_factor.argtypes = [P, P, i64, P, P]
    L.fpde_lu_solve.argtypes = [P, P, i64, P, P, P]
    L.fpde_template_csr.argtypes = [P, P, P, i64, P, P]
    L.fpde_assemble_csr.argtypes = [P, P, P, P, P, P, P, P]
    L.fpde_csr_apply.argtypes = [P, P, P, P, P, P, P]
    L.fpde_cg_solve.argtypes = [P, P, P, P, P, P, P, dbl, i32, P, P]
    L.fpde_form_assemble.argtypes = [P, P, P, P, i64, P]
    L.fpde_mesh2d_create.argtypes = [P, i64, P, i64, P, ctypes.POINTER(P)]
    L.fpde_mesh2d_destroy.argtypes = [P]
    L.fpde_mesh2d_info.argtypes = [P, P, P, P]
    L.fpde_dof_map2d.argtypes = [P, P]
    L.fpde_paths2d.argtypes = [P, i32, i32, i64, i64, i32, P, P, P, P, P]
    L.fpde_assemble2d.argtypes = [P, P, P, i64, P, P, P]
    L.fpde_solve2d.argtypes = [P, P, i64, P, P, P, P]
    L.fpde_timing2d.argtypes = [P, i32]
    L.fpde_stage_times2d.argtypes = [P, P, P]
    for name in EXPORTS:
        getattr(L, name).restype = L.fpde_status_string.restype if name == "fpde_status_string" else (
            None if name in ("fpde_mesh_destroy", "fpde_mesh2d_destroy") else ctypes.c_int)
    _L = L
    return L


def _check(st: int, what: str):
    if st != FPDE_OK:
        raise FpdeError(st, what)


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _np(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def params(alpha: float, K=(1.0, 1.0, 1.0), quad_points: int = 4, precision: int = FPDE_FP64,
           source: int = FPDE_SRC_ONE, max_steps: int = 0, ir_tol: float = 0.0, ir_max_iter: int = 0,
           deterministic: bool = False):
    p = fpde_params()
    p.alpha = float(alpha)
    for i in range(3):
        p.K[i] = float(K[i])
    p.quad_points = int(quad_points)
    p.precision = int(precision)
    p.source = int(source)
    p.max_steps = int(max_steps)
    p.ir_tol = float(ir_tol)
    p.ir_max_iter = int(ir_max_iter)
    p.deterministic = int(bool(deterministic))
    return p


def div_params(beta, quad_points: int = 4, coef: int = FPDE_COEF_SEC3, source: int = FPDE_SRC_ONE,
               radius: float = 0.5, max_steps: int = 0):
    """Parameters of the divergence-form problem of Sec. 3."""
    p = fpde_div_params()
    for i in range(3):
        p.beta[i] = float(beta[i])
    p.quad_points = int(quad_points)
    p.coef = int(coef)
    p.source = int(source)
    p.radius = float(radius)
    p.max_steps = int(max_steps)
    return p


def form_params(alpha, beta, cl=(1.0, 1.0, 1.0), cr=(1.0, 1.0, 1.0), quad_points: int = 4,
                coef: int = FPDE_COEF_CONST, max_steps: int = 0):
    """Parameters of the general uniform form (c D^alpha u, D^beta v)."""
    p = fpde_form_params()
    for i in range(3):
        p.alpha[i] = float(alpha[i])
        p.beta[i] = float(beta[i])
        p.cl[i] = float(cl[i])
        p.cr[i] = float(cr[i])
    p.quad_points = int(quad_points)
    p.coef = int(coef)
    p.max_steps = int(max_steps)
    return p


class Mesh:
    """Device-resident mesh handle (fpde_mesh_create / fpde_mesh_destroy)."""

    def __init__(self, xyz, tet, stream=None):
        L = _lib()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tet = np.ascontiguousarray(tet, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.fpde_mesh_create(_np(self.xyz), self.xyz.shape[0], _np(self.tet), self.tet.shape[0],
                                  _stream(stream), ctypes.byref(h)), "fpde_mesh_create")
        self._h = h
        nd, nb, nt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.fpde_mesh_info(h, ctypes.byref(nd), ctypes.byref(nb), ctypes.byref(nt)), "fpde_mesh_info")
        self.n_dof, self.n_boundary_faces, self.n_tet = nd.value, nb.value, nt.value
        self.n_vert = self.xyz.shape[0]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().fpde_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def dof_map(self) -> np.ndarray:
        out = np.empty(self.n_vert, dtype=np.int32)
        _check(_lib().fpde_dof_map(self._h, _np(out)), "fpde_dof_map")
        return out

    def plan(self, quad_points: int, max_steps: int = 0, stream=None):
        _check(_lib().fpde_plan(self._h, quad_points, max_steps, _stream(stream)), "fpde_plan")

    def plan_info(self, quad_points: int, stream=None) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(_lib().fpde_plan_info(self._h, quad_points, _np(out), _stream(stream)), "fpde_plan_info")
        return {"half_rays": int(out[0]), "entries": int(out[1]), "pairs": int(out[2]), "max_entries": int(out[3]),
                "tubes": int(out[4]), "tube_nodes": int(out[5]), "max_tube_nodes": int(out[6]),
                "block_bytes": int(out[7])}

    def template(self, tile: int = 64, stream=None):
        """Template of Sec. 2.3 at tile granularity: (tiles uint8 (nt, nt), nnz)."""
        nt = -(-self.n_dof // tile) if (self.n_dof and tile >= 1) else 0  # the library rejects bad tiles
        tiles = np.zeros((nt, nt), dtype=np.uint8)
        nnz = np.zeros(1, dtype=np.int64)
        _check(_lib().fpde_template(self._h, tile, _np(tiles), _np(nnz), _stream(stream)), "fpde_template")
        return tiles, int(nnz[0])

    def timing(self, enable: bool, stages=None):
        """Start (clearing the totals) or stop stage timing; stages: names
        from STAGES to time only those (default: every stage)."""
        if not enable:
            _check(_lib().fpde_timing_stages(self._h, 0), "fpde_timing_stages")
        elif stages is None:
            _check(_lib().fpde_timing(self._h, 1), "fpde_timing")
        else:
            mask = 0
            for name in stages:
                mask |= 1 << STAGES.index(name)
            _check(_lib().fpde_timing_stages(self._h, mask), "fpde_timing_stages")

    def stage_times(self) -> dict:
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), dtype=np.int64)
        _check(_lib().fpde_stage_times(self._h, _np(ms), _np(cnt)), "fpde_stage_times")
        return {s: (float(ms[k]), int(cnt[k])) for k, s in enumerate(STAGES)}

    def paths(self, quad_points: int, dir: int, g0: int, count: int, max_steps: int = 4096,
              lists: bool = False, stream=None):
        import torch
        dev = torch.device("cuda")
        ln = torch.empty(count, dtype=torch.int32, device=dev)
        hs = torch.empty(count, dtype=torch.int64, device=dev)
        ids = torch.empty((count, max_steps), dtype=torch.int32, device=dev) if lists else None
        rend = torch.empty((count, max_steps), dtype=torch.float64, device=dev) if lists else None
        _check(_lib().fpde_paths(self._h, quad_points, dir, g0, count, max_steps, _ptr(ln), _ptr(hs),
                                 _ptr(ids), _ptr(rend), _stream(stream)), "fpde_paths")
        return ln, hs, ids, rend

    def ray_values(self, quad_points: int, alpha: float, dir: int, g0: int, count: int, stream=None):
        off = np.zeros(count + 1, dtype=np.int64)
        L = _lib()
        st = L.fpde_ray_values(self._h, quad_points, alpha, dir, g0, count, _np(off), None, None, 0,
                               _stream(stream))
        if st not in (FPDE_OK, -1):
            _check(st, "fpde_ray_values")
        n = int(off[-1])
        dof = np.empty(max(n, 1), dtype=np.int32)
        val = np.empty(max(n, 1), dtype=np.float64)
        _check(L.fpde_ray_values(self._h, quad_points, alpha, dir, g0, count, _np(off), _np(dof), _np(val), n,
                                 _stream(stream)), "fpde_ray_values")
        return off, dof[:n], val[:n]

    def assemble(self, p, A, b=None, f_gauss=None, stream=None):
        _check(_lib().fpde_assemble(self._h, ctypes.byref(p), _ptr(A), A.stride(0), _ptr(b), _ptr(f_gauss),
                                    _stream(stream)), "fpde_assemble")

    def apply(self, p, x, y, stream=None):
        _check(_lib().fpde_apply(self._h, ctypes.byref(p), _ptr(x), _ptr(y), _stream(stream)), "fpde_apply")

    def solve(self, p, A, b, u, stream=None, info: bool = True):
        """FP64: Cholesky + triangular solves (with info: the FP64 residual is
        also measured); mixed: FP32 Cholesky + refinement (info always)."""
        out = fpde_solve_info()
        _check(_lib().fpde_solve(self._h, ctypes.byref(p), _ptr(A), A.stride(0), _ptr(b), _ptr(u),
                                 ctypes.byref(out) if info else None, _stream(stream)), "fpde_solve")
        return out if info else None

    def assemble_batch(self, params_list, A, b=None, stream=None):
        """fpde_assemble for the systems params_list[z] into A[z] (and b[z]),
        one status check at the end."""
        count = len(params_list)
        if A.shape[0] != count or A.stride(2) != 1 or (b is not None and (b.shape[0] != count or b.stride(1) != 1)):
            raise ValueError("assemble_batch: A (count, n, n) and b (count, n) with contiguous rows")
        arr = (fpde_params * count)(*params_list)
        _check(_lib().fpde_assemble_batch(self._h, count, arr, _ptr(A), A.stride(1), A.stride(0), _ptr(b),
                                          b.stride(0) if b is not None else 0, _stream(stream)),
               "fpde_assemble_batch")

    def solve_batch(self, A, b, u, stream=None):
        """FP64 Cholesky solves of A[z] u[z] = b[z] for every z < A.shape[0]
        (1..16) in one launch sequence; A (count, n, n) is overwritten by the
        factors.  Raises FpdeError with .failed_pivot (per system) on failure."""
        count = A.shape[0]
        if A.stride(2) != 1 or b.stride(-1) != 1 or u.stride(-1) != 1 or u.stride(0) != b.stride(0):
            raise ValueError("solve_batch: rows of A and the vectors must be contiguous, b and u alike strided")
        piv = (ctypes.c_int64 * max(count, 1))()
        st = _lib().fpde_solve_batch(self._h, count, _ptr(A), A.stride(1), A.stride(0), _ptr(b), _ptr(u),
                                     b.stride(0), piv, _stream(stream))
        if st != FPDE_OK:
            e = FpdeError(st, "fpde_solve_batch")
            e.failed_pivot = [piv[z] for z in range(count)]
            raise e

    def solve_noalloc(self, A, b, u, stream=None):
        """FP64 Cholesky solve with the library's static scratch (no device
        allocation; n_dof <= 8192).  Raises FpdeError with .failed_pivot."""
        piv = ctypes.c_int64(-1)
        st = _lib().fpde_solve_noalloc(self._h, _ptr(A), A.stride(0), _ptr(b), _ptr(u), ctypes.byref(piv),
                                       _stream(stream))
        if st != FPDE_OK:
            e = FpdeError(st, "fpde_solve_noalloc")
            e.failed_pivot = piv.value
            raise e

    def solve_factored(self, p, L, b, u, stream=None, info: bool = True):
        out = fpde_solve_info()
        _check(_lib().fpde_solve_factored(self._h, ctypes.byref(p), _ptr(L), L.stride(0), _ptr(b), _ptr(u),
                                          ctypes.byref(out) if info else None, _stream(stream)),
               "fpde_solve_factored")
        return out if info else None

    # sparse storage on the template, conjugate gradients ------------------
    def template_csr(self, stream=None):
        """The template of Sec. 2.3 as CSR: (row_ptr int64, col int32), device tensors."""
        import torch
        L = _lib()
        rp = torch.empty(self.n_dof + 1, dtype=torch.int64, device="cuda")
        nnz = ctypes.c_int64()
        _check(L.fpde_template_csr(self._h, _ptr(rp), None, 0, ctypes.byref(nnz), _stream(stream)),
               "fpde_template_csr")
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
        _check(L.fpde_template_csr(self._h, _ptr(rp), _ptr(col), nnz.value, ctypes.byref(nnz), _stream(stream)),
               "fpde_template_csr")
        return rp, col[:nnz.value]

    def assemble_csr(self, p, row_ptr, col, val, b=None, f_gauss=None, stream=None):
        _check(_lib().fpde_assemble_csr(self._h, ctypes.byref(p), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(b),
                                        _ptr(f_gauss), _stream(stream)), "fpde_assemble_csr")

    def csr_apply(self, row_ptr, col, val, x, y, stream=None):
        _check(_lib().fpde_csr_apply(self._h, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y),
                                     _stream(stream)), "fpde_csr_apply")

    def cg_solve(self, p, b, u, csr=None, tol: float = 1e-10, max_iter: int = 0, stream=None):
        """CG with the Jacobi preconditioner; csr = (row_ptr, col, val) or None
        for the matrix-free operator.  Returns fpde_solve_info."""
        out = fpde_solve_info()
        rp, ci, va = csr if csr is not None else (None, None, None)
        _check(_lib().fpde_cg_solve(self._h, ctypes.byref(p), _ptr(rp), _ptr(ci), _ptr(va), _ptr(b), _ptr(u),
                                    float(tol), int(max_iter), ctypes.byref(out), _stream(stream)),
               "fpde_cg_solve")
        return out

    # the general uniform form --------------------------------------------
    def form_assemble(self, p, A, coef=None, stream=None):
        _check(_lib().fpde_form_assemble(self._h, ctypes.byref(p), _ptr(coef), _ptr(A), A.stride(0),
                                         _stream(stream)), "fpde_form_assemble")

    # the divergence-form problem of Sec. 3 -------------------------------
    def div_assemble(self, p, A, b=None, pq=None, f_gauss=None, stream=None):
        _check(_lib().fpde_div_assemble(self._h, ctypes.byref(p), _ptr(pq), _ptr(A), A.stride(0), _ptr(b),
                                        _ptr(f_gauss), _stream(stream)), "fpde_div_assemble")

    def lu_factor(self, A, stream=None) -> int:
        """In-place LU without pivoting; returns -1 (FpdeError on failure,
        with .failed_pivot set to the failing block's first column)."""
        piv = ctypes.c_int64(-1)
        st = _lib().fpde_lu_factor(self._h, _ptr(A), A.stride(0), ctypes.byref(piv), _stream(stream))
        if st != FPDE_OK:
            e = FpdeError(st, "fpde_lu_factor")
            e.failed_pivot = piv.value
            raise e
        return piv.value

    def lu_solve(self, LU, b, u, stream=None):
        _check(_lib().fpde_lu_solve(self._h, _ptr(LU), LU.stride(0), _ptr(b), _ptr(u), _stream(stream)),
               "fpde_lu_solve")

    def adjoint(self, p, u, lam, stream=None):
        ga = ctypes.c_double()
        gk = (ctypes.c_double * 3)()
        _check(_lib().fpde_adjoint(self._h, ctypes.byref(p), _ptr(u), _ptr(lam), ctypes.byref(ga), gk,
                                   _stream(stream)), "fpde_adjoint")
        return ga.value, np.array(list(gk))


def params2d(alpha: float, K=(1.0, 1.0), quad_points: int = 3, source: int = FPDE_SRC_ONE, max_steps: int = 0):
    p = fpde_params2d()
    p.alpha = float(alpha)
    p.K[0], p.K[1] = float(K[0]), float(K[1])
    p.quad_points = int(quad_points)
    p.source = int(source)
    p.max_steps = int(max_steps)
    return p


class Mesh2D:
    """Device-resident two-dimensional mesh handle (fpde_mesh2d_*)."""

    def __init__(self, xy, tri, stream=None):
        L = _lib()
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.fpde_mesh2d_create(_np(self.xy), self.xy.shape[0], _np(self.tri), self.tri.shape[0],
                                    _stream(stream), ctypes.byref(h)), "fpde_mesh2d_create")
        self._h = h
        nd, nb, nt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.fpde_mesh2d_info(h, ctypes.byref(nd), ctypes.byref(nb), ctypes.byref(nt)), "fpde_mesh2d_info")
        self.n_dof, self.n_boundary_edges, self.n_tri = nd.value, nb.value, nt.value
        self.n_vert = self.xy.shape[0]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().fpde_mesh2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def dof_map(self) -> np.ndarray:
        out = np.empty(self.n_vert, dtype=np.int32)
        _check(_lib().fpde_dof_map2d(self._h, _np(out)), "fpde_dof_map2d")
        return out

    def paths(self, quad_points: int, dir: int, g0: int, count: int, max_steps: int = 4096, lists: bool = False,
              stream=None):
        import torch
        ln = torch.empty(count, dtype=torch.int32, device="cuda")
        hs = torch.empty(count, dtype=torch.int64, device="cuda")
        ids = torch.empty((count, max_steps), dtype=torch.int32, device="cuda") if lists else None
        rend = torch.empty((count, max_steps), dtype=torch.float64, device="cuda") if lists else None
        _check(_lib().fpde_paths2d(self._h, quad_points, dir, g0, count, max_steps, _ptr(ln), _ptr(hs), _ptr(ids),
                                   _ptr(rend), _stream(stream)), "fpde_paths2d")
        return ln, hs, ids, rend

    def assemble(self, p, A, b=None, f_gauss=None, stream=None):
        _check(_lib().fpde_assemble2d(self._h, ctypes.byref(p), _ptr(A), A.stride(0), _ptr(b), _ptr(f_gauss),
                                      _stream(stream)), "fpde_assemble2d")

    def solve(self, A, b, u, stream=None):
        piv = ctypes.c_int64(-1)
        _check(_lib().fpde_solve2d(self._h, _ptr(A), A.stride(0), _ptr(b), _ptr(u), ctypes.byref(piv),
                                   _stream(stream)), "fpde_solve2d")

    def timing(self, enable: bool):
        _check(_lib().fpde_timing2d(self._h, 1 if enable else 0), "fpde_timing2d")

    def stage_times(self) -> dict:
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), dtype=np.int64)
        _check(_lib().fpde_stage_times2d(self._h, _np(ms), _np(cnt)), "fpde_stage_times2d")
        return {s: (float(ms[k]), int(cnt[k])) for k, s in enumerate(STAGES)}


def new_matrix(mesh: Mesh, precision: int = FPDE_FP64):
    import torch
    dt = torch.float64 if precision == FPDE_FP64 else torch.float32
    n = max(mesh.n_dof, 1)
    return torch.empty((n, n), dtype=dt, device="cuda")


def solve_problem(mesh: Mesh, p, f_gauss=None, stream=None, info: bool = True):
    """Assemble and solve: returns (u, factor, info) with device tensors."""
    import torch
    A = new_matrix(mesh, p.precision)
    b = torch.empty(max(mesh.n_dof, 1), dtype=torch.float64, device="cuda")
    mesh.assemble(p, A, b, f_gauss, stream)
    u = torch.empty_like(b)
    out = mesh.solve(p, A, b, u, stream, info=info)
    return u, A, out


def solve_div_problem(mesh: Mesh, p, pq=None, f_gauss=None, stream=None):
    """Assemble the Sec. 3 system and solve it by LU: returns (u, LU, b)."""
    import torch
    A = new_matrix(mesh, FPDE_FP64)
    b = torch.empty(max(mesh.n_dof, 1), dtype=torch.float64, device="cuda")
    mesh.div_assemble(p, A, b, pq, f_gauss, stream)
    mesh.lu_factor(A, stream)
    u = torch.empty_like(b)
    mesh.lu_solve(A, b, u, stream)
    return u, A, b


from .autograd import FracSolve  # noqa: E402

__all__ = ["Mesh", "params", "div_params", "solve_problem", "solve_div_problem", "new_matrix", "FracSolve",
           "FpdeError", "fpde_params", "fpde_div_params", "fpde_solve_info", "FPDE_FP64", "FPDE_MIXED",
           "FPDE_SRC_ONE", "FPDE_SRC_USER", "FPDE_SRC_CUBE_MMS", "FPDE_SRC_BALL_MMS", "FPDE_COEF_SEC3",
           "FPDE_COEF_USER", "FPDE_COEF_CONST", "form_params", "fpde_form_params", "Mesh2D", "params2d",
           "fpde_params2d", "FPDE_SRC_SQUARE_MMS", "EXPORTS", "LIB_PATH"]
