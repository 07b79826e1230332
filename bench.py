#!/usr/bin/env python3
"""Benchmark of the fractional FEM hot path on one MI355X.

Headline workload (synthetic, seeded): the convex hull of 2000 random points
in the ellipsoid with semi-axes (1, 0.7, 0.4), filled with a jittered
body-centred-cubic lattice (~400k elements, ~67k nodes), Riesz order
alpha = 1.3 (the timed passes alternate 1.30 / 1.31 so every pass walks its
paths again instead of reusing the previous pass's derivative values),
K = (1, 1, 1), the 11-point element rule.

One step = one mixed-precision assembly + solve pass on that mesh: path walk
and closed-form derivatives (FP64), accumulation of the dense stiffness
matrix stored in FP32 (~18 GB), load vector, FP32 Cholesky, then refinement
with FP64 residuals from the matrix-free product until ||b - K u|| / ||b||
<= 1e-8.  Inputs are resident on the device when the timed region starts;
the mesh set-up and the symbolic plan (built once per mesh and rule) happen
before it and are reported apart.

value = Gauss-point paths per second of the whole step (6 half-rays per
Gauss point divided by the step time).  Beside it on the single JSON line:
assembly+solve seconds per step, paths/s of walk+eval alone, the FP64 arm on
the same mesh (FP64 matrix, ~36 GB, FP64 Cholesky) with the mixed/FP64
speedup and the distance between the two solutions, the per-stage times, the
roofline of the step's dominant kernel (launch durations measured over the
timed steps with HIP events inside the library on the launch stream), and
the CPU oracle on a bounded sample of the same workload.  Secondary sections
(not the headline): FP64 vs mixed on the ~150k-element sphere hull, the
adjoint gradient on the ~40k-element ball, the six-system batch on the
~20k-element sphere hull, sparse template storage with CG, the general
uniform form, the two-dimensional variant and the divergence-form problem of
Sec. 3.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "assembly+solve s & Gauss-pt paths/s at N nodes, FP64 vs mixed @1e-6 rel err"
WORKLOAD = "ellipsoid400k"
HEAD_ALPHAS = (1.30, 1.31)
HEAD_NQ = 11
HEAD_K = (1.0, 1.0, 1.0)
C2_WORKLOAD = "sphere20k"
ALPHAS = (1.2, 1.5, 1.8)
RULES = (4, 11)
BREAKDOWN_STEPS = 5  # steps with every stage timed, after the timed steps
KCOEF = (1.0, 0.5, 2.0)
HBM_PEAK = 8.0e12        # B/s
FP64_PEAK = 78.6e12      # FLOP/s, vector and matrix
FP32_PEAK = 157.3e12     # FLOP/s, matrix cores
FP16_PEAK = 2.5e15       # FLOP/s, dense matrix cores
CSRC = os.path.join(ROOT, "paper_1811_03339_amd", "csrc")
# HBM counter summaries (profiles/): unit -> (file, sources its kernels are built from)
FACT_SRC = [os.path.join(CSRC, f) for f in ("solve.hip", "syrk128.h", "chol_diag.h", "dense.h", "syrk256.h")]
PMC = {
    "factorization_fp32_c5": (os.path.join(ROOT, "profiles", "potrf_fp32_ellipsoid400k_pmc.txt"), FACT_SRC),
    "factorization_fp64_c5": (os.path.join(ROOT, "profiles", "potrf_fp64_ellipsoid400k_pmc.txt"), FACT_SRC),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_sha1(paths):
    h = hashlib.sha1()
    for path in paths:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def read_traffic(kernel):
    """HBM bytes per unit (launch, or factorization) from the committed PMC
    summary, or None when it is missing or was taken on another version of
    the source."""
    path, src = PMC[kernel]
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha1") != src_sha1(src):
        return None
    try:
        return float(kv["hbm_bytes_per_unit"])
    except (KeyError, ValueError):
        return None


SEC3_WORKLOAD = "ball_h076"
SEC3_BETAS = ((0.6, 0.7, 0.8), (0.8, 0.8, 0.8))
SEC3_R = 0.5


MIXED_LARGE = "sphere150k"


def bench_mixed_large(F, torch, dev, reps=3):
    """FP64 against the mixed arm where the factorization dominates: the
    convex-hull mesh of 400 sphere points with ~150k elements (~25k
    unknowns), 11-point rule, K = (1, 1, 1), alpha alternating 1.70 / 1.69
    so that every pass re-walks.  Per pass and arm: assembly + solve (FP64:
    FP64 matrix, Cholesky, two triangular solves; mixed: FP32 matrix, FP32
    Cholesky, refinement with FP64 matrix-free residuals to 1e-8).  Median of
    `reps` passes after one warm-up pass of each arm."""
    from fpde_inputs import workload_mesh
    mesh = workload_mesh(MIXED_LARGE)
    g = F.Mesh(mesh.xyz, mesh.tet)
    nq, K = 11, (1.0, 1.0, 1.0)
    g.plan(nq)
    n = g.n_dof
    b = torch.empty(n, dtype=torch.float64, device=dev)
    u64 = torch.empty_like(b)
    u32 = torch.empty_like(b)
    alphas = (1.70, 1.69)

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), r

    def arm(precision, A, u):
        ts, info = [], None
        g.timing(True)
        for k in range(reps + 1):
            a = alphas[k % 2]
            p = F.params(a, K, quad_points=nq, precision=precision, ir_tol=1e-8)

            def run():
                g.assemble(p, A, b)
                return g.solve(p, A, b, u, info=(precision == F.FPDE_MIXED))
            t, info = timed(run)
            if k > 0:
                ts.append(t)
        g.timing(False)
        st = g.stage_times()
        return sorted(ts)[len(ts) // 2], info, st

    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    t64, _, st64 = arm(F.FPDE_FP64, A, u64)
    del A
    torch.cuda.empty_cache()
    A32 = torch.empty((n, n), dtype=torch.float32, device=dev)
    tmx, info, stmx = arm(F.FPDE_MIXED, A32, u32)
    del A32
    torch.cuda.empty_cache()
    err = float((u32 - u64).abs().max() / u64.abs().max())  # both at the last alpha of the sequence
    fl = n ** 3 / 3.0

    def tf(st):
        return fl / (st["potrf"][0] / st["potrf"][1] / 1e3) / 1e12 if st["potrf"][1] else None
    return {"workload": f"{MIXED_LARGE}: hull of 400 seeded points on the unit sphere + BCC lattice, {g.n_tet} "
                        f"tets, {n} unknowns, 11-point rule, K = (1, 1, 1), alpha alternating 1.70 / 1.69",
            "n_dof": n, "fp64_assembly_solve_s": t64 / 1e3, "mixed_assembly_solve_s": tmx / 1e3,
            "speedup_vs_fp64": t64 / tmx, "rel_err_vs_fp64": err, "ir_iters": info.ir_iters,
            "final_rel_residual": info.final_rel_residual,
            "factorization_TFLOP_s": {"fp64": tf(st64), "fp32": tf(stmx)},
            "factorization_ms": {"fp64": st64["potrf"][0] / max(st64["potrf"][1], 1),
                                 "fp32": stmx["potrf"][0] / max(stmx["potrf"][1], 1)},
            "stages_ms_per_pass": {"fp64": {k: v[0] / (reps + 1) for k, v in st64.items() if v[1] > 0},
                                   "mixed": {k: v[0] / (reps + 1) for k, v in stmx.items() if v[1] > 0}}}


def bench_sec3(F, torch, dev, reps=4):
    """The divergence-form problem of Sec. 3 on the finest mesh of Table 3
    (ball |x| < 0.5, largest element diameter 0.0757): per pass the Sec. 3
    assembly (walk values at the pass's orders, row accumulation, closed-form
    source), the LU factorization and the two triangular solves.  Passes
    alternate the two order sets of Table 3, so the walk re-evaluates the
    axes whose order changed."""
    import numpy as np
    from fpde_inputs import workload_mesh
    mesh = workload_mesh(SEC3_WORKLOAD)
    g3 = F.Mesh(mesh.xyz, mesh.tet)
    g3.plan(4)
    n = g3.n_dof
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)

    def one(beta):
        p = F.div_params(beta, 4, source=F.FPDE_SRC_BALL_MMS, radius=SEC3_R)
        g3.div_assemble(p, A, b)
        g3.lu_factor(A)
        g3.lu_solve(A, b, u)

    one(SEC3_BETAS[1])  # warm-up
    torch.cuda.synchronize()
    g3.timing(True)
    ts = []
    for k in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        one(SEC3_BETAS[k % 2])
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    g3.timing(False)
    st = g3.stage_times()
    # nodal error against the exact solution of the last pass's orders
    dof = g3.dof_map()
    x = mesh.xyz[dof >= 0]
    exact = (np.sum(x * x, axis=1) - SEC3_R ** 2) ** 2
    uh = u.cpu().numpy()[dof[dof >= 0]]
    lu_t = st["lu"][0] / max(st["lu"][1], 1) / 1e3
    fl = 2.0 * n ** 3 / 3.0
    out = {
        "workload": f"{SEC3_WORKLOAD}: ball |x| < 0.5, {g3.n_tet} tets, {mesh.n_vert} nodes ({n} interior), "
                    f"largest element diameter 0.0757 (Table 3), 4-point rule, p_i = cos x_i, "
                    f"q_i = 1 - cos x_i, beta alternating {list(SEC3_BETAS)}",
        "n_dof": n,
        "pass_ms": sorted(ts)[len(ts) // 2],
        "stages_ms_per_pass": {k: v[0] / reps for k, v in st.items() if v[1] > 0},
        "lu": {"bound": "mfma", "flops_per_factorization": fl, "ms": lu_t * 1e3,
               "achieved": fl / lu_t / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
               "frac": fl / lu_t / FP64_PEAK},
        "max_nodal_error": float(np.abs(uh - exact).max()),
    }
    g3.close()
    return out


def bench_sparse(F, torch, gm, reps=3):
    """K on the template of Sec. 2.3 as CSR, on the bench mesh: the pattern
    (once per mesh), the CSR assembly, the CSR product against its HBM
    roofline, and conjugate gradients on the CSR matrix and matrix-free,
    compared with the dense FP64 Cholesky solution."""
    n = gm.n_dof
    p = F.params(1.5, KCOEF, quad_points=4)

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), r

    t_tpl, (rp, col) = timed(lambda: gm.template_csr())
    nnz = col.numel()
    val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    t_asm = sorted(timed(lambda: gm.assemble_csr(p, rp, col, val, b))[0] for _ in range(reps))[reps // 2]
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    gm.csr_apply(rp, col, val, x, y)
    k = 50
    t_mv = timed(lambda: [gm.csr_apply(rp, col, val, x, y) for _ in range(k)])[0] / k
    by = nnz * 12.0 + (n + 1) * 8.0 + 2.0 * n * 8.0
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ud = torch.empty_like(b)
    gm.assemble(p, A, b)
    gm.solve(p, A, b, ud, info=False)
    del A
    out = {"workload": f"{C2_WORKLOAD}, alpha = 1.5, 4-point rule", "template_ms": t_tpl, "nnz": nnz,
           "density": nnz / float(n * n), "csr_bytes": nnz * 12 + (n + 1) * 8, "dense_bytes": n * n * 8,
           "csr_assembly_ms": t_asm,
           "spmv": {"ms": t_mv, "bound": "hbm", "algorithmic_bytes": by, "achieved": by / (t_mv / 1e3) / 1e9,
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": by / (t_mv / 1e3) / HBM_PEAK}}
    for name, csr in (("cg_csr", (rp, col, val)), ("cg_matrix_free", None)):
        u = torch.empty_like(b)
        t, info = timed(lambda: gm.cg_solve(p, b, u, csr=csr, tol=1e-10))
        out[name] = {"ms": t, "iterations": info.ir_iters, "rel_residual": info.final_rel_residual,
                     "rel_diff_vs_cholesky": float((u - ud).abs().max() / ud.abs().max())}
    return out


FORM_ALPHA = (0.3, 0.8, 0.55)
FORM_BETA = (0.9, 0.4, 0.7)


def bench_form(F, torch, gm, info4, reps=3):
    """The general uniform form (c D^alpha u, D^beta v) with per-axis orders
    on the bench mesh (4-point rule), constant coefficients: both value sets
    re-walked every pass (the orders alternate), the two products of every
    pair accumulated by tubes (k_tube_form), then the row pass of K."""
    n = gm.n_dof
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    gm.timing(True)
    ts = []
    for k in range(reps):
        a, b = (FORM_ALPHA, FORM_BETA) if k % 2 == 0 else (FORM_BETA, FORM_ALPHA)
        p = F.form_params(a, b, (1.0, 0.5, 2.0), (0.7, 1.5, 0.3), 4)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        gm.form_assemble(p, A)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    gm.timing(False)
    st = gm.stage_times()
    t_form = st["form"][0] / max(st["form"][1], 1) / 1e3
    # algorithmic work: per entry product of a pair two products (trial x
    # test scaled by cl, test x trial scaled by cr), a multiply-add each
    fl = 4.0 * info4["pairs"]
    return {"workload": f"{C2_WORKLOAD}, 4-point rule, alpha {list(FORM_ALPHA)}, beta {list(FORM_BETA)} "
                        f"(alternating), constant coefficients",
            "pass_ms": sorted(ts)[len(ts) // 2],
            "stages_ms_per_pass": {k: v[0] / reps for k, v in st.items() if v[1] > 0},
            "tubes": {"bound": "alu", "ms": t_form * 1e3, "flops": fl,
                      "achieved": fl / t_form / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                      "frac": fl / t_form / FP64_PEAK,
                      "kernel": "k_tube_form + k_tube_gather<double> (vector FMA, LDS atomics)"}}


PLANE_WORKLOAD = "disk4k"


def bench_plane(F, torch, reps=3):
    """The two-dimensional variant on the disk (4654 nodes), 7-point rule:
    per pass the walk at the pass's order, the row accumulation, the load
    vector and the dense Cholesky solve (orders alternate so every pass
    re-walks)."""
    from fpde_inputs import workload_mesh
    mesh = workload_mesh(PLANE_WORKLOAD)
    g2 = F.Mesh2D(mesh.xyz, mesh.tet)
    n = g2.n_dof
    A = torch.empty((n, n), dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    u = torch.empty_like(b)

    def one(alpha):
        g2.assemble(F.params2d(alpha, (1.0, 0.5), 7), A, b)
        g2.solve(A, b, u)

    one(1.8)  # plan + warm-up
    torch.cuda.synchronize()
    g2.timing(True)
    ts = []
    for k in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        one(1.3 if k % 2 == 0 else 1.6)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    g2.timing(False)
    st = g2.stage_times()
    t = sorted(ts)[len(ts) // 2]
    rays = 4 * g2.n_tri * 7
    out = {"workload": f"{PLANE_WORKLOAD}: unit disk (160-gon) + jittered triangular lattice, {g2.n_tri} triangles, "
                       f"{mesh.n_vert} nodes ({n} interior), 7-point rule, K = (1, 0.5), alpha alternating 1.3 / 1.6",
           "n_dof": n, "pass_ms": t, "paths_per_s": rays / (t / 1e3),
           "stages_ms_per_pass": {k: v[0] / reps for k, v in st.items() if v[1] > 0}}
    g2.close()
    return out


ADJ_WORKLOAD = "ball40k"


def bench_adjoint(F, torch, dev):
    """Adjoint gradients on the unit-ball hull (~42k elements): loss
    J = ||u_h - u_obs||^2 at alpha = 1.4, K = (1, 1, 1) (4-point rule), u_obs
    from alpha = 1.6, K = (1.2, 0.8, 1.0) plus N(0, 1e-3^2) noise (seed 40).
    One forward (assembly + FP64 solve) and backward (adjoint solve with the
    stored factor + the adjoint kernel re-walking every path), timed, and the
    gradient against central differences with h = 1e-6."""
    import numpy as np
    from fpde_inputs import workload_mesh
    mesh = workload_mesh(ADJ_WORKLOAD)
    g = F.Mesh(mesh.xyz, mesh.tet)
    nq = 4
    g.plan(nq)
    rng = np.random.default_rng(40)
    u_obs, _, _ = F.solve_problem(g, F.params(1.6, (1.2, 0.8, 1.0), quad_points=nq), info=False)
    obs = u_obs + 1e-3 * torch.tensor(rng.normal(size=g.n_dof), device=dev)
    alpha, K = 1.4, np.array([1.0, 1.0, 1.0])

    def fwd_bwd():
        a_t = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
        k_t = torch.tensor(K, dtype=torch.float64, requires_grad=True)
        u = F.FracSolve.apply(a_t, k_t, g, nq)
        J = torch.sum((u - obs) ** 2)
        J.backward()
        return a_t.grad.item(), k_t.grad.numpy().copy()

    fwd_bwd()  # warm-up (values, factor scratch)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ga, gk = fwd_bwd()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)

    def loss(a, k):
        uu, _, _ = F.solve_problem(g, F.params(a, k, quad_points=nq), info=False)
        return float(torch.sum((uu - obs) ** 2))

    h = 1e-6
    fd_a = (loss(alpha + h, K) - loss(alpha - h, K)) / (2 * h)
    fd_k = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd_k.append((loss(alpha, K + e) - loss(alpha, K - e)) / (2 * h))
    fd_k = np.array(fd_k)
    out = {"workload": f"{ADJ_WORKLOAD}: hull of 800 seeded points on the unit sphere + BCC lattice, {g.n_tet} tets, "
                       f"{mesh.n_vert} nodes ({g.n_dof} interior), 4-point rule, alpha = 1.4, K = (1, 1, 1)",
           "forward_backward_s": sorted(ts)[1], "dJ_dalpha": ga, "dJ_dK": gk.tolist(),
           "fd_dalpha": fd_a, "fd_dK": fd_k.tolist(),
           "rel_err_dalpha_vs_fd": abs(ga - fd_a) / abs(fd_a),
           "rel_err_dK_vs_fd": float(np.abs(gk - fd_k).max() / np.abs(fd_k).max()),
           "fd_step": h}
    g.close()
    return out


def bench_c2(F, torch, dev, steps=20, warmup=2):
    """The six-system batch on the ~20k-element sphere hull (3 alphas x 2
    rules, K = (1, 0.5, 2)): per step the six systems are assembled as one
    batch (walks beside the accumulations) and factored and solved as one
    batch.  Also the mixed arm at this size (alpha alternating so that every
    pass walks again), the template CSR / CG and the general-form sections."""
    from fpde_inputs import workload_mesh
    mesh = workload_mesh(C2_WORKLOAD)
    gm = F.Mesh(mesh.xyz, mesh.tet)
    info = {}
    for nq in RULES:
        gm.plan(nq)
        info[nq] = gm.plan_info(nq)
    n = gm.n_dof
    cases = [(nq, a) for nq in RULES for a in ALPHAS]
    A = torch.empty((len(cases), n, n), dtype=torch.float64, device=dev)
    b = torch.empty((len(cases), n), dtype=torch.float64, device=dev)
    u = torch.empty((len(cases), n), dtype=torch.float64, device=dev)
    rays_per_step = sum(6 * gm.n_tet * nq for nq in RULES) * len(ALPHAS)
    step_params = [F.params(a, KCOEF, quad_points=nq) for nq, a in cases]

    def step():
        gm.assemble_batch(step_params, A, b)
        gm.solve_batch(A, b, u)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    gm.timing(True)
    for _ in range(BREAKDOWN_STEPS):
        step()
    torch.cuda.synchronize()
    gm.timing(False)
    st = gm.stage_times()
    out = {"workload": f"{C2_WORKLOAD}: hull of 400 seeded points on the unit sphere + BCC lattice, {gm.n_tet} tets, "
                       f"{mesh.n_vert} nodes ({n} interior); alpha {list(ALPHAS)}, K={list(KCOEF)}, rules "
                       f"{list(RULES)}; six FP64 systems per step, assembled and solved as batches",
           "n_dof": n, "ms_per_step": ms, "paths_per_s": rays_per_step / (ms / 1e3),
           "stages_ms_per_step": {k: v[0] / BREAKDOWN_STEPS for k, v in st.items() if v[1] > 0},
           "tube_accum": None}
    if st["accum"][1]:
        t = st["accum"][0] / st["accum"][1] / 1e3
        fl = sum(4 * info[nq]["pairs"] for nq in RULES) / len(RULES)
        out["tube_accum"] = {"bound": "alu", "ms_per_launch": t * 1e3, "flops_per_launch": fl,
                             "achieved": fl / t / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                             "frac": fl / t / FP64_PEAK,
                             "note": "4 |L| |R| flops per (g, i): both products W (R L^T + L R^T)"}
    # mixed arm at this size, alpha alternating so every pass walks again
    p64s = [F.params(a, KCOEF, quad_points=11) for a in (1.5, 1.51)]
    pmxs = [F.params(a, KCOEF, quad_points=11, precision=F.FPDE_MIXED, ir_tol=1e-8) for a in (1.5, 1.51)]
    A32 = torch.empty((n, n), dtype=torch.float32, device=dev)
    u32 = torch.empty_like(u[0])

    def timed(fn, reps=4):
        ts, r = [], None
        for k in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn(k)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2], r

    def run64(k):
        p = p64s[k % 2]
        gm.assemble(p, A[0], b[0])
        gm.solve(p, A[0], b[0], u[0], info=False)

    def runmx(k):
        p = pmxs[k % 2]
        gm.assemble(p, A32, b[0])
        return gm.solve(p, A32, b[0], u32)

    t64, _ = timed(run64)
    tmx, inf = timed(runmx)
    err = float((u32 - u[0]).abs().max() / u[0].abs().max())  # both at alpha = 1.51
    out["mixed"] = {"workload": "alpha alternating 1.50 / 1.51, 11-point rule", "fp64_assembly_solve_s": t64 / 1e3,
                    "mixed_assembly_solve_s": tmx / 1e3, "speedup_vs_fp64": t64 / tmx, "rel_err_vs_fp64": err,
                    "ir_iters": inf.ir_iters, "final_rel_residual": inf.final_rel_residual}
    del A32, A
    torch.cuda.empty_cache()
    out["sparse"] = bench_sparse(F, torch, gm)
    out["form"] = bench_form(F, torch, gm, info[4])
    gm.close()
    return out


def cpu_baseline(om, alpha, K, nq, G, budget_s=10.0):
    """The oracle as it stands on a bounded sample of the headline workload:
    its matrix-free product (walk, closed-form derivatives and the sums of
    Sec. 2.1 for every half-ray of the sampled Gauss points) restricted to a
    contiguous range of Gauss points sized for about `budget_s` seconds, at
    one thread and at every host thread.  Gauss-point paths per second."""
    import numpy as np

    import oracle
    x = np.random.default_rng(0).normal(size=om.ndof)
    before = oracle.set_threads()
    out = {}
    try:
        for th in (1, before):
            oracle.set_threads(th)
            cal = 2000 * th
            t0 = time.perf_counter()
            om.apply_range(nq, alpha, K, x, 0, cal)
            dt = time.perf_counter() - t0
            cnt = int(min(G, max(cal, cal * budget_s / max(dt, 1e-3))))
            g0 = (G - cnt) // 2
            t0 = time.perf_counter()
            om.apply_range(nq, alpha, K, x, g0, g0 + cnt)
            dt = time.perf_counter() - t0
            out[th] = (6 * cnt / dt, cnt, dt)
    finally:
        oracle.set_threads(before)
    v1, c1, d1 = out[1]
    vn, cn, dn = out[before]
    return {"value": vn, "unit": "Gauss-pt paths/s", "cores": before, "kind": "oracle",
            "sample": f"{WORKLOAD}, alpha {alpha}, {nq}-point rule: the oracle's matrix-free product (walk + "
                      f"closed-form derivatives + the sums of K x, FP64) over {cn} contiguous Gauss points "
                      f"({6 * cn} half-rays) of {G} in {dn:.1f} s on {before} threads; one thread: {c1} points "
                      f"in {d1:.1f} s",
            "single_thread_value": v1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 arm of the headline workload")
    ap.add_argument("--no-sections", action="store_true", help="only the headline workload")
    ap.add_argument("--no-sec3", action="store_true", help="skip the Sec. 3 divergence-form problem")
    ap.add_argument("--no-c2", action="store_true", help="skip the six-system batch section (and sparse, form)")
    ap.add_argument("--no-plane", action="store_true", help="skip the two-dimensional section")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint section")
    ap.add_argument("--no-mixed-large", action="store_true",
                    help="skip FP64 vs mixed at the 25k-unknown mesh")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the library runs on one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_03339_amd as F
    from fpde_inputs import workload_mesh

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t = time.perf_counter()
    mesh = workload_mesh(WORKLOAD)
    gen_s = time.perf_counter() - t
    log(f"[bench] mesh {WORKLOAD}: {mesh.n_vert} nodes, {mesh.n_tet} elements ({gen_s:.1f} s to generate)")

    torch.cuda.synchronize()
    t = time.perf_counter()
    gm = F.Mesh(mesh.xyz, mesh.tet)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    gm.plan(HEAD_NQ)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t)
    info = gm.plan_info(HEAD_NQ)
    n = gm.n_dof
    G = gm.n_tet * HEAD_NQ
    rays = 6 * G
    log(f"[bench] n_dof {n}, mesh set-up {setup_ms:.1f} ms, plan {plan_ms:.1f} ms, {info}")

    b = torch.empty(n, dtype=torch.float64, device=dev)
    u = torch.empty_like(b)
    A32 = torch.empty((n, n), dtype=torch.float32, device=dev)
    pm = [F.params(a, HEAD_K, quad_points=HEAD_NQ, precision=F.FPDE_MIXED, ir_tol=1e-8) for a in HEAD_ALPHAS]
    last = {}

    def step(k):
        p = pm[k % 2]
        gm.assemble(p, A32, b)
        last["info"] = gm.solve(p, A32, b, u)
        last["alpha"] = p.alpha

    for k in range(args.warmup):
        step(k + 1)  # ends on the alpha the first timed step does not use
    torch.cuda.synchronize()
    # inside the timed steps only the two roofline candidates carry stage
    # events (each timed stage costs two event records per launch)
    gm.timing(True, stages=["accum", "potrf"])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        step(k)
        log(f"[bench] step {k + 1}/{args.steps} done (ir_iters {last['info'].ir_iters}, residual "
            f"{last['info'].final_rel_residual:.2e})")
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    gm.timing(False)
    live = gm.stage_times()
    ms_per_step = total_ms / args.steps
    value = rays * args.steps / (total_ms / 1e3)
    log(f"[bench] {ms_per_step:.1f} ms/step, {value:.3e} paths/s, timed-step stages {live}")
    mixed_info = last["info"]
    # device memory held after the timed steps: mesh, plan (entries, tube
    # plan, packed operands, blocks), the FP32 matrix and the solve's scratch
    free_b, total_b = torch.cuda.mem_get_info()
    mem_used_gb = (total_b - free_b) / 1e9
    log(f"[bench] device memory in use {mem_used_gb:.1f} GB of {total_b / 1e9:.1f} GB")
    # per-stage breakdown from one further step with every stage timed
    gm.timing(True)
    step(args.steps)
    torch.cuda.synchronize()
    gm.timing(False)
    stages = gm.stage_times()
    log(f"[bench] stage breakdown (one step): {stages}")
    walk_ms = stages["walk"][0]
    u_mixed = u.clone()
    alpha_mixed = last["alpha"]

    # roofline of the step's dominant kernel, by time per step: the FP32
    # factorization (one unit = one factorization of the n x n matrix:
    # n^3 / 3 algorithmic flops; its trailing updates run as split-FP16
    # products, three FP16 matrix-core products per FP32 product, so its
    # ceiling is the dense FP16 peak / 3) or the tube accumulation (one unit =
    # the accumulation of one assembly: 4 |L| |R| flops per (g, i))
    cand = []
    if live["potrf"][1]:
        t_f = live["potrf"][0] / live["potrf"][1] / 1e3
        fl = n ** 3 / 3.0
        peak = FP16_PEAK / 3.0
        cand.append((live["potrf"][0], {
            "bound": "mfma", "achieved": fl / t_f / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": fl / t_f / peak, "traffic": read_traffic("factorization_fp32_c5"),
            "kernel": "FP32 Cholesky of the n x n matrix: per group of sixteen 64-column panels k_panel and the "
                      "k_syrk<float, 64> strip update of the group's later block columns, then k_row_split<1024> "
                      "and k_syrk256<1024> on the trailing matrix (256 x 256 tiles)",
            "peak_note": "dense FP16 matrix-core peak (2.5 PFLOP/s) / 3: each FP32 product of the trailing "
                         "update is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16",
            "avg_launch_ms": t_f * 1e3, "flops_per_unit": fl,
            "dtype": "f32 factor; trailing update in split f16 (hi + lo) with f32 accumulation"}))
    if live["accum"][1]:
        t_a = live["accum"][0] / live["accum"][1] / 1e3
        fl = 4.0 * info["pairs"]
        cand.append((live["accum"][0], {
            "bound": "mfma", "achieved": fl / t_a / 1e12, "peak": FP16_PEAK / 3.0 / 1e12, "unit": "TFLOP/s",
            "frac": fl / t_a / (FP16_PEAK / 3.0), "traffic": None,
            "kernel": "k_merge_vals + k_tube_mfma (entries merged per node and side, tube blocks as split-FP16 "
                      "products on 128 x 128 regions, one pass per assembly)",
            "note": "achieved counts the method's products over entries (4 |L| |R| per pair); the kernel computes "
                    "each 128 x 128 region of a tube block densely over the tube's pairs, so the matrix-core work "
                    "it issues is larger than this count",
            "avg_launch_ms": t_a * 1e3, "flops_per_unit": fl, "dtype": "f32 operands split into f16 hi + lo"}))
    roofline = max(cand, key=lambda c: c[0])[1] if cand else None
    other_roofline = min(cand, key=lambda c: c[0])[1] if len(cand) > 1 else None

    # the FP64 arm on the same mesh: FP64 matrix (n^2 x 8 bytes), FP64
    # Cholesky, two triangular solves; alpha alternating as above
    fp64 = None
    if not args.no_fp64:
        del A32
        torch.cuda.empty_cache()
        A64 = torch.empty((n, n), dtype=torch.float64, device=dev)
        u64 = torch.empty_like(b)
        p64 = [F.params(a, HEAD_K, quad_points=HEAD_NQ) for a in HEAD_ALPHAS]
        ts = []
        gm.timing(True)
        # pass 0 (untimed) warms the FP64 scratch; the timed passes 1 and 2
        # each take the alpha the previous pass did not (so both walk), and
        # the last is the mixed solution's
        mi = HEAD_ALPHAS.index(alpha_mixed)
        seq = [p64[mi], p64[1 - mi], p64[mi]]
        for k in range(3):
            p = seq[k]
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            gm.assemble(p, A64, b)
            gm.solve(p, A64, b, u64, info=False)
            e1.record()
            torch.cuda.synchronize()
            if k > 0:
                ts.append(e0.elapsed_time(e1))
            log(f"[bench] FP64 pass {k} {e0.elapsed_time(e1):.1f} ms")
        gm.timing(False)
        st64 = gm.stage_times()
        assert abs(p.alpha - alpha_mixed) < 1e-15  # the last FP64 pass solved the mixed solution's alpha
        t64 = sum(ts) / len(ts)
        err = float((u_mixed - u64).abs().max() / u64.abs().max())
        potrf64 = st64["potrf"][0] / max(st64["potrf"][1], 1) / 1e3
        fp64 = {"assembly_solve_s": t64 / 1e3, "speedup_mixed_vs_fp64": t64 / ms_per_step,
                "mixed_rel_err_vs_fp64": err, "alpha_compared": alpha_mixed,
                "matrix_bytes": n * n * 8,
                "stages_ms_per_pass": {k: v[0] / 3 for k, v in st64.items() if v[1] > 0},
                "factorization": {"bound": "mfma", "ms": potrf64 * 1e3,
                                  "achieved": n ** 3 / 3.0 / potrf64 / 1e12, "peak": FP64_PEAK / 1e12,
                                  "unit": "TFLOP/s", "frac": n ** 3 / 3.0 / potrf64 / FP64_PEAK,
                                  "traffic": read_traffic("factorization_fp64_c5")}}
        log(f"[bench] FP64 arm {fp64}")
        del A64
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        import oracle
        om = oracle.OracleMesh(mesh.xyz, mesh.tet)
        cpu = cpu_baseline(om, HEAD_ALPHAS[0], HEAD_K, HEAD_NQ, G)
        log(f"[bench] cpu oracle {cpu}")
        del om
    gm.close()
    torch.cuda.empty_cache()

    sections = {}
    if not args.no_sections:
        if not args.no_mixed_large:
            sections["sphere150k_fp64_vs_mixed"] = bench_mixed_large(F, torch, dev)
            log(f"[bench] sphere150k {sections['sphere150k_fp64_vs_mixed']}")
        if not args.no_adjoint:
            sections["ball40k_adjoint"] = bench_adjoint(F, torch, dev)
            log(f"[bench] adjoint {sections['ball40k_adjoint']}")
        if not args.no_c2:
            sections["sphere20k_batch"] = bench_c2(F, torch, dev)
            log(f"[bench] sphere20k {sections['sphere20k_batch']}")
        if not args.no_plane:
            sections["plane"] = bench_plane(F, torch)
            log(f"[bench] plane {sections['plane']}")
        if not args.no_sec3:
            sections["sec3"] = bench_sec3(F, torch, dev)
            log(f"[bench] sec3 {sections['sec3']}")

    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB device-to-device copy done")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gauss-pt paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 paths/derivatives/residuals, f32 matrix and factor",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: hull of 2000 seeded points in the ellipsoid (1, 0.7, 0.4) + BCC lattice, "
                        f"{gm.n_tet} tets, {mesh.n_vert} nodes ({n} interior); alpha {HEAD_ALPHAS[0]} "
                        f"(timed passes alternate {list(HEAD_ALPHAS)}), K={list(HEAD_K)}, {HEAD_NQ}-point rule; "
                        f"mixed precision: FP32 dense matrix + FP32 Cholesky + FP64 matrix-free refinement to 1e-8",
            "n_nodes": mesh.n_vert, "n_dof": n, "n_tet": gm.n_tet, "gauss_points": G,
            "parallelism": "single GPU",
        },
        "assembly_solve_s": ms_per_step / 1e3,
        "walk_eval_paths_per_s": rays / (walk_ms / 1e3) if walk_ms > 0 else None,
        "mixed": {"ir_iters": mixed_info.ir_iters, "final_rel_residual": mixed_info.final_rel_residual,
                  "matrix_bytes": n * n * 4},
        "fp64": fp64,
        "stages_ms_per_step": {k: v[0] for k, v in stages.items() if v[1] > 0},
        "stages_note": ("launch times per stage from one further step with every stage timed; inside the timed "
                        "steps only the accumulation and the factorization carry events (the roofline's launch "
                        "durations)"),
        "setup_ms": setup_ms,
        "plan_ms": plan_ms,
        "mesh_generation_s": gen_s,
        "end_to_end_first_pass_s": (setup_ms + plan_ms) / 1e3 + ms_per_step / 1e3,
        "plan": info,
        "device_mem_used_gb": mem_used_gb,
        "roofline": roofline,
        "roofline_other": other_roofline,
        "sections": sections,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
