#!/usr/bin/env python3
"""Benchmark of the fractional FEM hot path on one MI355X.

Workload (synthetic, seeded): the convex hull of 400 random points on the
unit sphere filled with a jittered body-centred-cubic lattice (19 689
elements, 3 472 nodes, 3 072 interior unknowns), Riesz orders
alpha in {1.2, 1.5, 1.8}, K = (1, 0.5, 2), the 4- and 11-point element rules.

One step = for each rule and each alpha: assemble (path walk + closed-form
derivatives, accumulation of the dense FP64 stiffness matrix, load vector)
and solve (dense FP64 Cholesky + triangular solves) -- six assembly+solve
passes.  The mesh set-up and the symbolic plan (the template, built once per
mesh and rule) happen before the timed region and are reported apart.

value = Gauss-point paths per second over the timed steps (6 half-rays per
Gauss point, summed over the six passes, divided by the step time).
The single JSON line on stdout also carries the per-stage times (from a few
further steps with every stage timed), the roofline of the dominant kernel
(its launch durations measured over the timed steps with HIP events inside
the library on the launch stream; only the two candidate stages carry
events there), the mixed-precision arm, K on the template of Sec. 2.3
as CSR with conjugate gradients (CSR and matrix-free), the general uniform
form (c D^alpha u, D^beta v) with per-axis orders, the two-dimensional
variant on a disk, the divergence-form
problem of Sec. 3 on the finest mesh of Table 3 (assembly + LU + solve, with the LU
against its FP64 roofline) and the CPU oracle baseline.
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
WORKLOAD = "sphere20k"
ALPHAS = (1.2, 1.5, 1.8)
RULES = (4, 11)
BREAKDOWN_STEPS = 5  # steps with every stage timed, after the timed steps
KCOEF = (1.0, 0.5, 2.0)
HBM_PEAK = 8.0e12        # B/s
FP64_PEAK = 78.6e12      # FLOP/s, vector and matrix
CSRC = os.path.join(ROOT, "paper_1811_03339_amd", "csrc")
# HBM counter summaries (profiles/): unit -> (file, sources its kernels are built from)
PMC = {
    "factorization": (os.path.join(ROOT, "profiles", "potrf_sphere20k_pmc.txt"),
                      [os.path.join(CSRC, "solve.hip"), os.path.join(CSRC, "dense.h")]),
    "k_tube_accum": (os.path.join(ROOT, "profiles", "tube_accum_sphere20k_pmc.txt"),
                     [os.path.join(CSRC, "tubes.hip")]),
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
    out = {"workload": f"{WORKLOAD}, alpha = 1.5, 4-point rule", "template_ms": t_tpl, "nnz": nnz,
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
    return {"workload": f"{WORKLOAD}, 4-point rule, alpha {list(FORM_ALPHA)}, beta {list(FORM_BETA)} "
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


def cpu_baseline(mesh_np):
    """The oracle, unchanged, single-threaded, on one full step."""
    from threadpoolctl import threadpool_limits

    import oracle
    with threadpool_limits(limits=1):
        om = oracle.OracleMesh(mesh_np.xyz, mesh_np.tet)
        rays = 0
        t0 = time.perf_counter()
        for nq in RULES:
            for a in ALPHAS:
                A = om.assemble(nq, a, KCOEF)
                b = om.load(nq)
                oracle.solve_spd(A, b)
                rays += 6 * om.n_tet * nq
        dt = time.perf_counter() - t0
    return {"value": rays / dt, "unit": "Gauss-pt paths/s", "cores": 1, "kind": "oracle",
            "sample": f"one full step ({len(RULES)} rules x {len(ALPHAS)} alphas): dense assembly + load + "
                      f"LAPACK Cholesky, FP64, 1 thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision arm")
    ap.add_argument("--no-sec3", action="store_true", help="skip the Sec. 3 divergence-form problem")
    ap.add_argument("--no-sparse", action="store_true", help="skip the template-CSR / CG section")
    ap.add_argument("--no-form", action="store_true", help="skip the general-form section")
    ap.add_argument("--no-plane", action="store_true", help="skip the two-dimensional section")
    ap.add_argument("--no-mixed-large", action="store_true",
                    help="skip FP64 vs mixed at the 25k-unknown mesh")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the one-step comparison that solves the systems one at a time")
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
    info = {}
    for nq in RULES:
        gm.plan(nq)
        info[nq] = gm.plan_info(nq)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t)
    n = gm.n_dof
    log(f"[bench] n_dof {n}, mesh set-up {setup_ms:.1f} ms, plans {plan_ms:.1f} ms, {info}")
    t = time.perf_counter()
    tiles, t_nnz = gm.template(64)
    template = {"tile": 64, "tiles_set": float(tiles.mean()), "pair_density": t_nnz / float(n * n),
                "ms": 1e3 * (time.perf_counter() - t)}
    log(f"[bench] template {template}")

    cases = [(nq, a) for nq in RULES for a in ALPHAS]
    A = torch.empty((len(cases), n, n), dtype=torch.float64, device=dev)
    b = torch.empty((len(cases), n), dtype=torch.float64, device=dev)
    u = torch.empty((len(cases), n), dtype=torch.float64, device=dev)
    rays_per_step = sum(6 * gm.n_tet * nq for nq in RULES) * len(ALPHAS)

    step_params = [F.params(a, KCOEF, quad_points=nq) for nq, a in cases]

    def step():
        # the step's systems are assembled one after another (each fills the
        # device; one status check for all, each walk beside the previous
        # system's accumulation), then factored and solved together: their
        # Cholesky and triangular-solve chains, latency-bound one by one, run
        # side by side
        gm.assemble_batch(step_params, A, b)
        gm.solve_batch(A, b, u)

    def step_sequential():
        for z, (nq, a) in enumerate(cases):
            p = F.params(a, KCOEF, quad_points=nq)
            gm.assemble(p, A[z], b[z])
            gm.solve(p, A[z], b[z], u[z], info=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # inside the timed steps only the two roofline candidates carry stage
    # events (each timed stage costs two event records per launch)
    gm.timing(True, stages=["accum", "potrf"])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        step()
        log(f"[bench] step {k + 1}/{args.steps} done")
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    gm.timing(False)
    live = gm.stage_times()  # accumulation and factorization over the timed steps
    ms_per_step = total_ms / args.steps
    value = rays_per_step * args.steps / (total_ms / 1e3)
    log(f"[bench] {ms_per_step:.2f} ms/step, {value:.3e} paths/s, timed-step stages {live}")
    # the per-stage breakdown from further steps with every stage timed
    # (outside the timed region)
    gm.timing(True)
    for _ in range(BREAKDOWN_STEPS):
        step()
    torch.cuda.synchronize()
    gm.timing(False)
    stages = gm.stage_times()
    log(f"[bench] stage breakdown over {BREAKDOWN_STEPS} steps: {stages}")

    # the same systems one at a time (assemble, factor, solve per system), one
    # step, outside the timed region: the per-system latency beside the
    # batched throughput
    seq_ms = None
    if not args.no_sequential:
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step_sequential()
        e1.record()
        torch.cuda.synchronize()
        seq_ms = e0.elapsed_time(e1)
        log(f"[bench] one step with the systems solved one at a time: {seq_ms:.2f} ms")

    # Roofline of the dominant kernel of the step, by time per step: either
    # the batched dense factorization (one unit = k_potrf_diag once, then per
    # pair of 64-column panels two k_panel and two k_syrk launches over all
    # systems, timed with one
    # event pair per call on the launch stream; algorithmic work
    # systems x n^3 / 3 FP64 flops, on the matrix cores: FP64 peak
    # 78.6 TFLOP/s) or the tube accumulation (one unit = one k_tube_accum
    # launch, one per system; algorithmic work one multiply-add per entry
    # product of S = sum w l r^T, B = S + S^T, i.e. 2 flops x pairs, on the
    # vector ALUs with LDS atomics: FP64 peak 78.6 TFLOP/s).
    passes = len(cases)
    factorizations = live["potrf"][1]
    cand = []
    if factorizations:
        calls = factorizations / passes
        avg_s = live["potrf"][0] / calls / 1e3
        fl = passes * n ** 3 / 3.0
        ach = fl / avg_s / 1e12
        cand.append((live["potrf"][0], {
            "bound": "mfma", "achieved": ach, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / (FP64_PEAK / 1e12), "traffic": read_traffic("factorization"),
            "kernel": f"batched factorization of {passes} systems: k_potrf_diag<double>, then per pair of "
                      f"64-column panels k_panel, k_syrk<double, 64> (block column), k_panel, "
                      f"k_syrk<double, 128> (trailing matrix)",
            "avg_launch_ms": avg_s * 1e3, "flops_per_unit": fl, "dtype": "f64 (v_mfma_f64_16x16x4f64 tiles)"}))
    if live["accum"][1]:
        avg_s = live["accum"][0] / live["accum"][1] / 1e3
        fl = sum(2 * info[nq]["pairs"] for nq in RULES) / len(RULES)  # launches alternate the rules evenly
        ach = fl / avg_s / 1e12
        cand.append((live["accum"][0], {
            "bound": "alu", "achieved": ach, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / (FP64_PEAK / 1e12), "traffic": read_traffic("k_tube_accum"),
            "kernel": "k_tube_accum (tube blocks, one launch per system)",
            "avg_launch_ms": avg_s * 1e3, "flops_per_unit": fl, "dtype": "f64 (vector FMA, LDS atomics)"}))
    roofline = max(cand, key=lambda c: c[0])[1] if cand else None
    other_roofline = min(cand, key=lambda c: c[0])[1] if len(cand) > 1 else None
    # every stage against its own bound (algorithmic work / measured time)
    stage_roof = {}
    if stages["potrf"][1]:
        t = stages["potrf"][0] / stages["potrf"][1] / 1e3
        fl = n ** 3 / 3.0
        stage_roof["potrf"] = {"flops_per_factorization": fl, "TFLOP/s": fl / t / 1e12,
                               "frac_fp64": fl / t / FP64_PEAK}
    if stages["trsv"][1]:
        t = stages["trsv"][0] / stages["trsv"][1] / 1e3
        by = n * n * 8.0  # the lower triangle read once forward, once backward
        stage_roof["trsv"] = {"bytes_per_solve": by, "GB/s": by / t / 1e9, "frac_hbm": by / t / HBM_PEAK}
    if stages["contract"][1]:
        t = stages["contract"][0] / stages["contract"][1] / 1e3
        by = n * n * 8.0 + sum(12.0 * info[nq]["entries"] for nq in RULES) / len(RULES)
        stage_roof["contract"] = {"algorithmic_bytes": by, "GB/s": by / t / 1e9, "frac_hbm": by / t / HBM_PEAK,
                                  "note": "K written once + every derivative entry read once"}
    if stages["accum"][1]:
        t = stages["accum"][0] / stages["accum"][1] / 1e3
        fl = sum(2 * info[nq]["pairs"] for nq in RULES) / len(RULES)
        stage_roof["accum"] = {"flops_per_launch": fl, "TFLOP/s": fl / t / 1e12, "frac_fp64": fl / t / FP64_PEAK,
                               "note": "one multiply-add per entry product of S (B = S + S^T)"}
    if stages["walk"][1]:
        stage_roof["walk"] = {"paths_per_s": rays_per_step * BREAKDOWN_STEPS / (stages["walk"][0] / 1e3)}

    # mixed-precision arm at alpha = 1.5, 11-point rule
    mixed = None
    if not args.no_mixed:
        p64 = F.params(1.5, KCOEF, quad_points=11)
        pmx = F.params(1.5, KCOEF, quad_points=11, precision=F.FPDE_MIXED, ir_tol=1e-8)
        A32 = torch.empty((n, n), dtype=torch.float32, device=dev)
        A0, b0, u0 = A[0], b[0], u[0]
        u32 = torch.empty_like(u0)

        def timed(fn, reps=3):
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                r = fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return sorted(ts)[len(ts) // 2], r

        def run64():
            gm.assemble(p64, A0, b0)
            gm.solve(p64, A0, b0, u0, info=False)

        def runmx():
            gm.assemble(pmx, A32, b0)
            return gm.solve(pmx, A32, b0, u32)

        t64, _ = timed(run64)
        tmx, inf = timed(runmx)
        err = float((u32 - u0).abs().max() / u0.abs().max())
        mixed = {"workload": "alpha=1.5, 11-point rule", "fp64_assembly_solve_s": t64 / 1e3,
                 "mixed_assembly_solve_s": tmx / 1e3, "speedup_vs_fp64": t64 / tmx,
                 "rel_err_vs_fp64": err, "ir_iters": inf.ir_iters,
                 "final_rel_residual": inf.final_rel_residual}
        log(f"[bench] mixed {mixed}")

    sparse = None
    if not args.no_sparse:
        sparse = bench_sparse(F, torch, gm)
        log(f"[bench] sparse {sparse}")

    form = None
    if not args.no_form:
        form = bench_form(F, torch, gm, info[4])
        log(f"[bench] form {form}")

    plane = None
    if not args.no_plane:
        plane = bench_plane(F, torch)
        log(f"[bench] plane {plane}")

    mixed_large = None
    if not args.no_mixed_large:
        mixed_large = bench_mixed_large(F, torch, dev)
        log(f"[bench] mixed_large {mixed_large}")

    sec3 = None
    if not args.no_sec3:
        sec3 = bench_sec3(F, torch, dev)
        log(f"[bench] sec3 {sec3}")

    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB device-to-device copy done")

    cpu = None if args.no_cpu else cpu_baseline(mesh)
    if cpu:
        log(f"[bench] cpu oracle {cpu}")

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: hull of 400 seeded points on the unit sphere + BCC lattice, "
                        f"{gm.n_tet} tets, {mesh.n_vert} nodes ({n} interior); alpha {list(ALPHAS)}, "
                        f"K={list(KCOEF)}, rules {list(RULES)}; FP64 assembly + dense Cholesky; "
                        f"{passes} systems per step, assembled as one batch (walks beside the accumulations), "
                        f"factored and solved as one batch",
            "n_nodes": mesh.n_vert, "n_dof": n, "n_tet": gm.n_tet,
            "gauss_points": {str(nq): gm.n_tet * nq for nq in RULES},
            "parallelism": "single GPU",
        },
        "assembly_solve_s_per_pass": ms_per_step / passes / 1e3,
        "sequential_ms_per_step": seq_ms,
        "sequential_assembly_solve_s_per_system": seq_ms / passes / 1e3 if seq_ms else None,
        "stages_ms_per_step": {k: v[0] / BREAKDOWN_STEPS for k, v in stages.items() if v[1] > 0},
        "stages_note": (f"launch times per stage from {BREAKDOWN_STEPS} further steps with every stage timed; "
                        f"inside the timed steps only the accumulation and the factorization carry events "
                        f"(the roofline's launch durations)"),
        "walk_eval_paths_per_s": (rays_per_step * BREAKDOWN_STEPS / (stages["walk"][0] / 1e3)
                                  if stages["walk"][0] > 0 else None),
        "setup_ms": setup_ms,
        "template_plan_ms": plan_ms,
        "template": template,
        "plan": {str(k): v for k, v in info.items()},
        "roofline": roofline,
        "roofline_other": other_roofline,
        "stage_rooflines": stage_roof,
        "mixed": mixed,
        "mixed_large": mixed_large,
        "sparse": sparse,
        "form": form,
        "plane": plane,
        "sec3": sec3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
