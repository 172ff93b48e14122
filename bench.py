"""Throughput benchmark of the truncated-Newton entropic-OT hot path.

Workload: n = m = 16384 (128 x 128 pixel grid), 3-blob histogram marginals
(seed 3000), dense FP32 squared-L2 grid cost normalised to max 1 (1 GiB,
resident in HBM), temperature annealed 1/32 -> 1e-5, target L1 marginal
error 1e-6.

A step is one full solve (MDOT + TruncatedNewtonProject + NewtonSolve/CG +
line search + ChiSinkhorn) in mixed precision, ending with the FP64
verification projection. `value` is the solve's streamed throughput: every
O(nm) pass reads the 4nm-byte cost once, so value = passes x 4nm / time.
Also reported: the HVP kernel's own GB/s against the 8 TB/s HBM peak
(roofline), the time to 1e-6 marginal error of the same solve in plain FP64
(the comparison the metric names), and the FP64 CPU oracle timed on a
bounded sample of the same HVP pass.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic():
    """HBM bytes per launch of the mixed HVP pass from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hvp_grid16384_memory_counters.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            kv[k] = v
    h = hashlib.sha256()
    for f in ("eot_kernels.hip", "eot_internal.h", "eot_lanes.h"):
        h.update(open(os.path.join(ROOT, "paper_2504_02067_amd", "csrc", f), "rb").read())
    if kv.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def oracle_hvp_band(p, C_rows_fn, budget_s, max_rows=None):
    """The FP64 oracle's HVP on a row band of the grid128 cost: the band grows
    until one call takes ~0.5 s (or reaches max_rows / every row), then calls
    repeat until the time budget is spent. Returns (GB/s of FP32-cost-equivalent
    bytes, rows, calls, seconds)."""
    import oracle as O
    n = p.n
    gamma = 1e-3
    rng = np.random.default_rng(1)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(n)
    rows = 16
    limit = n if max_rows is None else min(n, max_rows)
    while True:
        # the oracle takes FP64 costs: convert the band once, outside the timing
        Cs = np.ascontiguousarray(C_rows_fn(np.arange(rows)), dtype=np.float64)
        x = rng.standard_normal(rows)
        y = rng.standard_normal(n)
        t0 = time.perf_counter()
        O.hvp(Cs, 1.0 / gamma, u[:rows], v, 1.0, x, y)
        dt = time.perf_counter() - t0
        if dt > 0.5 or rows >= limit:
            break
        rows = min(limit, rows * 4)
    calls, total = 1, dt
    while total < budget_s:
        t0 = time.perf_counter()
        O.hvp(Cs, 1.0 / gamma, u[:rows], v, 1.0, x, y)
        total += time.perf_counter() - t0
        calls += 1
    return 4.0 * rows * n * calls / total / 1e9, rows, calls, total


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, C_rows_fn, W, batch=None, budget_s=6.0):
    """The FP64 oracle timed on the host cores (it is never tuned for this):
    its HVP on a row band of the grid128 cost with every thread and with one
    (a child process with OMP_NUM_THREADS=1, CPU only), full oracle solves of
    the 64-point instance (points64, seed 1000) and of the 28 x 28 grid with the
    squared-L2 cost (seed 2000), time per pass / CG iteration / Newton step from
    that solve, and estimates for the 28 x 28 L1 instance and the 512-problem
    batch from the oracle's time per plan entry and pass times the passes the
    same algorithm takes on the GPU (the oracle solve of the L1 instance alone
    takes ~30 s, the batch's largest problem ~50 s)."""
    import subprocess
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    threads = os.environ.get("OMP_NUM_THREADS", str(cores))
    gbs, rows, calls, total = oracle_hvp_band(p, C_rows_fn, budget_s, 1024)
    out = {"value": gbs, "unit": "GB/s", "cores": int(threads) if threads.isdigit() else cores,
           "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": cores,
           "sample": f"oracle HVP (FP64, row and column reductions) on a {rows} x {p.n} row band of "
                     f"the grid128 cost, {calls} calls in {total:.1f} s; OpenMP threads = {threads}"}
    # one thread, in a CPU-only child process (the oracle library reads its thread
    # count when loaded)
    code = ("import sys, json; sys.path.insert(0, %r); import bench, numpy as np; "
            "from paper_2504_02067_amd import workloads as W; p = W.large_grid_problem(3000); "
            "r = bench.oracle_hvp_band(p, lambda rows: W.grid_cost_rows(128, rows), 3.0, 1024); "
            "print(json.dumps(r))") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=120)
        g1, r1, c1, t1 = json.loads(res.stdout.strip().splitlines()[-1])
        out["single_core"] = {"value": g1, "unit": "GB/s",
                              "sample": f"{r1} x {p.n} row band, {c1} calls in {t1:.1f} s, 1 thread"}
    except Exception as e:                      # reported, not fatal
        out["single_core"] = {"error": str(e)[:200]}
    solves = {}
    q = W.small_points_problem(1000)
    t0 = time.perf_counter()
    _, _, st = O.solve(q.C, q.r, q.c, gamma_init=q.gamma_init, gamma_final=q.gamma_final, tol=q.tol)
    solves["points64"] = {"seconds": time.perf_counter() - t0, "newton_steps": st["newton_steps"],
                          "cg_iters": st["cg_iters"], "status": st["status"]}
    q = W.mnist_like_problem(2000, "sqeuclid")
    t0 = time.perf_counter()
    _, _, st = O.solve(q.C, q.r, q.c, gamma_init=q.gamma_init, gamma_final=q.gamma_final, tol=q.tol)
    dt = time.perf_counter() - t0
    passes = (st["passes_newton"] + st["passes_linesearch"] + st["passes_sinkhorn"]
              + st["passes_projection"])
    s_entry = dt / (passes * float(q.n) * q.m)             # seconds per plan entry and pass
    solves["grid28_sqeuclid_s2000"] = {
        "seconds": dt, "newton_steps": st["newton_steps"], "cg_iters": st["cg_iters"],
        "passes": passes, "status": st["status"], "ms_per_pass": 1e3 * dt / passes,
        "ms_per_cg_iter": 2e3 * dt / passes,             # a CG iteration is two passes
        "ms_per_newton_step": 1e3 * dt / max(1, st["newton_steps"]),
        "ns_per_entry_pass": 1e9 * s_entry}
    out["solves"] = solves
    est = {"basis": "oracle seconds per plan entry and pass (grid28 squared-L2 solve above) "
                    "x passes the same algorithm takes on the GPU x n m"}
    if batch is not None and "entry_passes" in batch.get("fp64", {}):
        est["batch512_seconds"] = s_entry * batch["fp64"]["entry_passes"]
    out["estimates"] = est
    return out


def valu_cycles_points_hvp(d):
    """FP32 vector lane operations per plan entry of the method's own work in
    the point-cloud HVP with the marginals given: d subtractions and d
    multiply-adds for |x - y|^2, two for the exponent (sum of the row and
    column parts, one multiply-add with the cost), exp, and one accumulation
    each for the row and the column sum (11 at d = 3). The implementation
    issues about 13.5 per entry (the lo part of beta, per-row reductions, loop
    control)."""
    return 2 * d + 2 + 1 + 2


# FP32 vector lane operations per second: the published FP32 vector peak
# (157.3 TFLOP/s, a multiply-add counted as two flops) over two.
FP32_LANE_OPS = 157.3e12 / 2


def points_measure(args, eot, W, dev, iters=4):
    """Mixed HVP pass on the n = m = 2^20 Gaussian-mixture clouds in R^3 with
    the cost recomputed on the fly (1.1e12 plan elements per pass)."""
    import torch
    p = W.point_cloud_problem()
    n, m = p.n, p.m
    pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
    gamma = 1e-2
    rng = np.random.default_rng(1)
    f = torch.from_numpy(gamma * (np.log(p.r) + 0.5 * rng.standard_normal(n))).to(dev)
    g = torch.from_numpy(gamma * (np.log(p.c) + 0.5 * rng.standard_normal(m))).to(dev)
    x = torch.from_numpy(rng.standard_normal(n)).to(dev)
    y = torch.from_numpy(rng.standard_normal(m)).to(dev)
    log(f"points: n = m = {n}, d = 3, row shift")
    shift = eot.eot_marginals(pc, gamma, f, g, precision="mixed", want=("log_rP",))["log_rP"]
    eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    torch.cuda.synchronize()
    eot.eot_pass_timing(True)
    for _ in range(iters):
        eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    torch.cuda.synchronize()
    k, ms = eot.eot_pass_timing_read(fused_hvp=1, precision="mixed")
    eot.eot_pass_timing(False)
    sec = ms / 1e3 / k
    elems = float(n) * float(m)
    cyc = valu_cycles_points_hvp(3)
    peak_eps = FP32_LANE_OPS / cyc
    log(f"points HVP {sec * 1e3:.1f} ms per pass, {elems / sec / 1e12:.3f} T elements/s")
    # the same product with r(P), c(P) given (one weighted sum per direction)
    mg = eot.eot_marginals(pc, gamma, f, g, row_shift=shift, precision="mixed",
                           want=("log_rP", "log_cP"))
    eot.eot_hvp_with_marginals(pc, gamma, f, g, mg["log_rP"], mg["log_cP"], 1.0, x, y,
                               precision="mixed")
    torch.cuda.synchronize()
    eot.eot_pass_timing(True)
    for _ in range(iters):
        eot.eot_hvp_with_marginals(pc, gamma, f, g, mg["log_rP"], mg["log_cP"], 1.0, x, y,
                                   precision="mixed")
    torch.cuda.synchronize()
    k2, ms2 = eot.eot_pass_timing_read(nr=1, nc=1, fused_hvp=0, precision="mixed")
    eot.eot_pass_timing(False)
    sec_m = ms2 / 1e3 / k2
    log(f"points HVP with marginals {sec_m * 1e3:.1f} ms per pass, "
        f"{elems / sec_m / 1e12:.3f} T elements/s")
    # the CG's two single-sum passes on the same clouds (row sums: rows on the lanes)
    cgp = {}
    for name, want, filt in (("row", ("log_rP",), dict(nr=1, nc=0)),
                             ("col", ("log_cP",), dict(nr=0, nc=1))):
        fn = lambda: eot.eot_marginals(pc, gamma, f, g, row_shift=shift, precision="mixed",
                                       want=want)
        fn()
        torch.cuda.synchronize()
        eot.eot_pass_timing(True)
        for _ in range(iters):
            fn()
        torch.cuda.synchronize()
        k3, ms3 = eot.eot_pass_timing_read(precision="mixed", **filt)
        eot.eot_pass_timing(False)
        cgp[f"{name}_ms"] = ms3 / k3
        cgp[f"{name}_entries_per_s"] = elems / (ms3 / k3 / 1e3)
    log(f"points CG passes: row {cgp['row_ms']:.1f} ms, column {cgp['col_ms']:.1f} ms")
    # a full solve on the same mixtures at n = m = 65536 (temperature 1/32 -> 1e-4, tol 1e-4)
    q = W.point_cloud_problem(n=1 << 16)
    qc = eot.PointCloud(torch.from_numpy(q.X).to(dev), torch.from_numpy(q.Y).to(dev), q.scale)
    qr, qcm = torch.from_numpy(q.r).to(dev), torch.from_numpy(q.c).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qf, qg, qs = eot.eot_solve(qc, qr, qcm, gamma_init=q.gamma_init, gamma_final=q.gamma_final,
                               tol=q.tol, precision="mixed")
    torch.cuda.synchronize()
    qt = time.perf_counter() - t0
    qp = sum(v for k, v in qs.items() if k.startswith("passes_"))
    log(f"points solve n = m = {q.n}: {qt:.2f} s, {qp} passes, error {qs['err_r'] + qs['err_c']:.1e}")
    mf = points_mfma_form(eot, pc, p, f, g, x, y, shift, gamma, iters, sec,
                          cold=(qc, q, qf, qg))
    return {"workload": f"gmm3d n=m={n} d=3 on-the-fly |x-y|^2/s, mixed HVP pass "
                        "(eot_hvp_with_marginals: r(P), c(P) given, P y and P^T x in one pass)",
            "kernel_ms": sec_m * 1e3, "elements_per_s": elems / sec_m,
            "roofline": {"bound": "alu", "achieved": elems / sec_m / 1e12,
                         "peak": peak_eps / 1e12, "unit": "T elements/s",
                         "frac": elems / sec_m / peak_eps,
                         "fp32_lane_ops_per_element": cyc},
            "cg_passes": cgp,
            "fused_hvp": {
                "note": "eot_hvp: r(P), c(P) formed in the same pass (two sums per direction)",
                "kernel_ms": sec * 1e3, "elements_per_s": elems / sec,
                "frac": elems / sec / peak_eps},
            "mfma_form": mf,
            "solve": {"workload": f"gmm3d n=m={q.n} d=3, temperature {q.gamma_init} -> "
                                  f"{q.gamma_final}, tol {q.tol}, mixed",
                      "seconds": qt, "passes": qp, "newton_steps": qs["newton_steps"],
                      "cg_iters": qs["cg_iters"], "err": qs["err_r"] + qs["err_c"],
                      "status": qs["status"]}}


def _pad16(cloud, eot):
    """The same points with coordinates zero-padded to d = 16 (the padding adds
    nothing to any distance)."""
    import torch
    X16 = torch.zeros(cloud.X.shape[0], 16, dtype=torch.float32, device=cloud.X.device)
    Y16 = torch.zeros(cloud.Y.shape[0], 16, dtype=torch.float32, device=cloud.X.device)
    X16[:, :cloud.X.shape[1]] = cloud.X
    Y16[:, :cloud.Y.shape[1]] = cloud.Y
    return eot.PointCloud(X16, Y16, cloud.scale)


def _marginal_errors(eot, clouds, gam, f, g):
    """Max |log r(P) - ref| and |log c(P) - ref| of each mixed form, the
    reference being the FP64 difference form (its log r(P) is the row shift)."""
    want = ("log_rP", "log_cP")
    ref = eot.eot_marginals(clouds["difference"], gam, f, g, precision="fp64", want=want)
    out = {}
    for name, cloud in clouds.items():
        o = eot.eot_marginals(cloud, gam, f, g, row_shift=ref["log_rP"], precision="mixed",
                              want=want)
        out[name] = max(float((o[w] - ref[w]).abs().max()) for w in want)
    return out


def points_mfma_form(eot, pc, p, f, g, x, y, shift, gamma, iters, diff_sec, cold):
    """The d = 3 pass with |x - y|^2 = |x|^2 + |y|^2 - 2 x . y and x . y on the
    matrix cores (the high-dimensional kernel on the coordinates zero-padded to
    16) against the difference form on the vector units: time per HVP pass on
    the 2^20-point clouds, and the error of each form's log marginals against
    the FP64 difference form, at the benchmark temperature and at the final
    temperature of the 65536-point solve (its converged potentials)."""
    import torch
    n, m = p.n, p.m
    pc16 = _pad16(pc, eot)
    eot.eot_hvp(pc16, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    torch.cuda.synchronize()
    eot.eot_pass_timing(True)
    for _ in range(iters):
        eot.eot_hvp(pc16, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    torch.cuda.synchronize()
    k, ms = eot.eot_pass_timing_read(fused_hvp=1, precision="mixed")
    eot.eot_pass_timing(False)
    sec = ms / 1e3 / k
    res = {"note": "x . y on the matrix cores (BF16 hi/lo, coordinates zero-padded to d = 16) "
                   "against the difference form on the vector units; errors: max |log r(P) - ref| "
                   "over rows and |log c(P) - ref| over columns, ref = FP64 difference form",
           "mfma_hvp_ms": sec * 1e3, "difference_hvp_ms": diff_sec * 1e3,
           "mfma_elements_per_s": float(n) * m / sec, "speedup_vs_difference": diff_sec / sec}
    e1 = _marginal_errors(eot, {"difference": pc, "mfma": pc16}, gamma, f, g)
    del pc16
    qc, q, qf, qg = cold
    qc16 = _pad16(qc, eot)
    e2 = _marginal_errors(eot, {"difference": qc, "mfma": qc16}, q.gamma_final, qf, qg)
    del qc16
    torch.cuda.synchronize()
    for name in ("difference", "mfma"):
        res[f"{name}_err_n2^20_gamma_{gamma:g}"] = e1[name]
        res[f"{name}_err_n65536_solution_gamma_{q.gamma_final:g}"] = e2[name]
    log(f"points MFMA form (d padded to 16): {sec * 1e3:.1f} ms per HVP pass "
        f"({diff_sec / sec:.2f}x the difference form); log-marginal error vs FP64: "
        f"gamma {gamma:g}: difference {e1['difference']:.1e}, MFMA {e1['mfma']:.1e}; "
        f"solution at gamma {q.gamma_final:g}: difference {e2['difference']:.1e}, "
        f"MFMA {e2['mfma']:.1e}")
    return res


def highd_measure(args, eot, W, dev, iters=5):
    """Mixed HVP pass on n = m = 65536 unit-norm embeddings in R^64, cost recomputed
    on the fly with the x . y contraction on the matrix cores (BF16 hi/lo, three
    MFMAs per 32 dimensions)."""
    import torch
    p = W.embedding_problem(1 << 16, d=64)
    n, m, d = p.n, p.m, 64
    pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
    gamma = 1e-2
    rng = np.random.default_rng(1)
    f = torch.from_numpy(gamma * (np.log(p.r) + 0.5 * rng.standard_normal(n))).to(dev)
    g = torch.from_numpy(gamma * (np.log(p.c) + 0.5 * rng.standard_normal(m))).to(dev)
    x = torch.from_numpy(rng.standard_normal(n)).to(dev)
    y = torch.from_numpy(rng.standard_normal(m)).to(dev)
    log(f"high-d: n = m = {n}, d = {d}")
    shift = eot.eot_marginals(pc, gamma, f, g, precision="mixed", want=("log_rP",))["log_rP"]
    res = {"workload": f"unit-norm embeddings n=m={n} d={d}, on-the-fly |x-y|^2/4, mixed HVP pass"}
    for prec in ("mixed", "fp64"):
        eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision=prec)
        torch.cuda.synchronize()
        eot.eot_pass_timing(True)
        for _ in range(iters):
            eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision=prec)
        torch.cuda.synchronize()
        k, ms = eot.eot_pass_timing_read(fused_hvp=1, precision=prec)
        eot.eot_pass_timing(False)
        sec = ms / 1e3 / k
        res[f"{prec}_ms"] = sec * 1e3
        res[f"{prec}_entries_per_s"] = float(n) * m / sec
    # the HVP with the marginals given (one weighted sum per direction), mixed
    mg = eot.eot_marginals(pc, gamma, f, g, row_shift=shift, precision="mixed",
                           want=("log_rP", "log_cP"))
    fn = lambda: eot.eot_hvp_with_marginals(pc, gamma, f, g, mg["log_rP"], mg["log_cP"], 1.0, x,
                                            y, precision="mixed")
    fn()
    torch.cuda.synchronize()
    eot.eot_pass_timing(True)
    for _ in range(iters):
        fn()
    torch.cuda.synchronize()
    k, ms = eot.eot_pass_timing_read(precision="mixed", nr=1, nc=1, fused_hvp=0)
    eot.eot_pass_timing(False)
    sec = ms / 1e3 / k
    res["with_marginals_mixed_ms"] = sec * 1e3
    res["with_marginals_mfma_frac"] = 3 * 2 * d * float(n) * m / sec / 2.5e15
    res["with_marginals_mfma_method_frac"] = 2 * d * float(n) * m / sec / 2.5e15
    # the CG's single-sum passes (column sums, then row sums), mixed
    for name, want, filt in (("colpass", ("log_cP",), dict(nr=0, nc=1)),
                             ("rowpass", ("log_rP",), dict(nr=1, nc=0))):
        fn = lambda: eot.eot_marginals(pc, gamma, f, g, row_shift=shift, precision="mixed", want=want)
        fn()
        torch.cuda.synchronize()
        eot.eot_pass_timing(True)
        for _ in range(iters):
            fn()
        torch.cuda.synchronize()
        k, ms = eot.eot_pass_timing_read(precision="mixed", **filt)
        eot.eot_pass_timing(False)
        sec = ms / 1e3 / k
        res[f"{name}_mixed_ms"] = sec * 1e3
        res[f"{name}_mfma_frac"] = 3 * 2 * d * float(n) * m / sec / 2.5e15
        res[f"{name}_mfma_method_frac"] = 2 * d * float(n) * m / sec / 2.5e15
    want = ("log_rP", "log_cP")
    ref = eot.eot_marginals(pc, gamma, f, g, precision="fp64", want=want)
    mx = eot.eot_marginals(pc, gamma, f, g, row_shift=ref["log_rP"], precision="mixed", want=want)
    res["mixed_log_marginal_err_vs_fp64"] = max(float((mx[w] - ref[w]).abs().max()) for w in want)
    res["beta_over_scale"] = 1.0 / gamma / p.scale
    eps = res["mixed_entries_per_s"]
    mfma = 3 * 2 * d * eps                      # BF16 hi/lo: three products per dimension pair
    res["mfma"] = {"achieved": mfma / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                   "frac": mfma / 2.5e15,
                   "method_frac": 2 * d * eps / 2.5e15,
                   "note": "dense BF16 matrix-core peak; frac counts the three hi/lo products the "
                           "matrix cores execute (3 x 2d flops per entry), method_frac only the "
                           "method's own x . y (2d flops per entry); the pass also evaluates exp and "
                           "the row and column sums per entry on the vector units"}
    mfma64 = 2 * d * res["fp64_entries_per_s"]  # FP64: one product per dimension pair
    res["mfma_fp64"] = {"achieved": mfma64 / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                        "frac": mfma64 / 78.6e12,
                        "note": "FP64 mode (line search, verification): x . y on the FP64 matrix "
                                "cores against their dense peak; exp and sums in FP64 on the vector units"}
    log(f"high-d HVP mixed {res['mixed_ms']:.2f} ms ({eps / 1e12:.2f} T entries/s, MFMA "
        f"{mfma / 1e12:.0f} TFLOP/s = {100 * mfma / 2.5e15:.1f}% of BF16 peak), FP64 {res['fp64_ms']:.2f} ms "
        f"(FP64 MFMA {mfma64 / 1e12:.1f} TFLOP/s = {100 * mfma64 / 78.6e12:.0f}% of FP64 peak)")
    log(f"high-d mixed log-marginal error vs FP64 at gamma {gamma:g}: "
        f"{res['mixed_log_marginal_err_vs_fp64']:.1e}")
    log(f"high-d HVP with marginals mixed {res['with_marginals_mixed_ms']:.2f} ms "
        f"({100 * res['with_marginals_mfma_frac']:.1f}% of BF16 peak)")
    log(f"high-d CG passes mixed: column {res['colpass_mixed_ms']:.2f} ms "
        f"({100 * res['colpass_mfma_frac']:.1f}% of BF16 peak), row {res['rowpass_mixed_ms']:.2f} ms "
        f"({100 * res['rowpass_mfma_frac']:.1f}%)")
    return res


def round_measure(eot, C, gamma, f, g, r, c):
    """Rounding of the solve's plan onto U(r, c) (three FP64 passes over the
    cost): time, the cost of the rounded plan and its gap to <P, C>."""
    import torch
    eot.eot_round(C, gamma, f, g, r, c)                  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = eot.eot_round(C, gamma, f, g, r, c)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"round: {dt * 1e3:.2f} ms, cost {out['cost_round']:.9f} (plan {out['cost_plan']:.9f})")
    return {"seconds": dt, "cost_round": out["cost_round"], "cost_plan": out["cost_plan"],
            "rel_gap": (out["cost_round"] - out["cost_plan"]) / out["cost_plan"]}


def grad_measure(eot, W, dev):
    """Backward of (W, S) for the largest batch problem (64 x 64 grid, 2-D
    points, temperature 1e-3): the S part solves the Hessian system by CG;
    gradients for X, Y, r and c, in FP64 and in mixed precision."""
    import torch
    sides = W.batch_sides()
    k = int(np.argmax(sides))
    p = W.batch_problem(k, sides=sides)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
    r = torch.from_numpy(p.r).to(dev)
    c = torch.from_numpy(p.c).to(dev)
    gamma = 1e-3
    f, g, st = eot.eot_solve(pc, r, c, gamma_init=1.0 / 32.0, gamma_final=gamma, tol=1e-6)
    res = {"workload": f"batch problem {k}: n = m = {p.n} (2-D points), temperature {gamma}, "
                       f"w_W = w_S = 1, outputs X, Y, r, c"}
    for prec in ("fp64", "mixed"):
        eot.eot_gradient(pc, gamma, f, g, 1.0, 1.0, want=("X", "Y", "r", "c"), precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = eot.eot_gradient(pc, gamma, f, g, 1.0, 1.0, want=("X", "Y", "r", "c"), precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = {"seconds": dt, "cg_iters": int(out["cg_iters"]),
                     "cg_residual": float(out["cg_residual"])}
        log(f"gradient {prec}: {dt * 1e3:.1f} ms, {out['cg_iters']} CG iterations")
    return res


def c1_measure(eot, W, dev, seeds=range(1000, 1010)):
    """The 64-point instances (n = m = 64, FP64 cost, temperature 1e-1 -> 1e-3,
    tol 1e-9), FP64 solves on the GPU: time per solve and per CG iteration
    (wall clock of the whole solve over its CG iterations), seeds 1000..1009."""
    import torch
    rows = []
    for s in seeds:
        q = W.small_points_problem(s)
        C = torch.from_numpy(q.C).to(dev)
        r, c = torch.from_numpy(q.r).to(dev), torch.from_numpy(q.c).to(dev)
        eot.eot_solve(C, r, c, gamma_init=q.gamma_init, gamma_final=q.gamma_final, tol=q.tol,
                      precision="fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st = eot.eot_solve(C, r, c, gamma_init=q.gamma_init, gamma_final=q.gamma_final,
                                 tol=q.tol, precision="fp64")
        torch.cuda.synchronize()
        rows.append((time.perf_counter() - t0, st["cg_iters"], st["newton_steps"],
                     st["err_r"] + st["err_c"]))
    sec = [x[0] for x in rows]
    res = {"workload": "points64 n=m=64, FP64 cost, temperature 0.1 -> 1e-3, tol 1e-9, FP64, "
                       f"seeds {seeds[0]}..{seeds[-1]}",
           "median_ms": float(np.median(sec)) * 1e3,
           "us_per_cg_iter": float(np.median([x[0] / max(x[1], 1) for x in rows])) * 1e6,
           "cg_iters_median": float(np.median([x[1] for x in rows])),
           "newton_steps_median": float(np.median([x[2] for x in rows])),
           "max_err": float(max(x[3] for x in rows))}
    log(f"C1 points64: median {res['median_ms']:.1f} ms per FP64 solve, "
        f"{res['us_per_cg_iter']:.0f} us per CG iteration (whole solve), max error {res['max_err']:.1e}")
    return res


def grid28_measure(eot, W, dev, seeds=3):
    """Time to 1e-6 marginal error on the 28 x 28 grid (n = m = 784, dense FP32
    cost, temperature 1/32 -> 1e-4), L1 and squared-L2 costs, mixed against plain
    FP64; medians over seeds 2000.. (each solve timed after one untimed solve of
    the same instance). Small problems: the solve is bound by latency (each CG
    solve is one cooperative launch, the rest of Alg. 4 launches per step), not
    by the passes. For comparison, the FP64 solve of the first seed also with
    the CG launched per iteration (eot_set_cg_persist(0))."""
    import torch
    res = {"workload": f"grid28 n=m=784 dense FP32 cost, 3-blob marginals seeds 2000..{2000 + seeds - 1}, "
                       "temperature 1/32 -> 1e-4, tol 1e-6"}
    for kind in ("l1", "sqeuclid"):
        rows = {"mixed": [], "fp64": []}
        costs = {"mixed": [], "fp64": []}
        errs = {"mixed": [], "fp64": []}
        per_cg = {"mixed": [], "fp64": []}
        for s in range(seeds):
            p = W.mnist_like_problem(2000 + s, kind)
            C = torch.from_numpy(p.C).to(dev)
            r = torch.from_numpy(p.r).to(dev)
            c = torch.from_numpy(p.c).to(dev)
            for prec in ("mixed", "fp64"):
                o = eot.default_solve_opts(gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                                           tol=p.tol, precision=prec)
                eot.eot_solve(C, r, c, opts=o)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, st = eot.eot_solve(C, r, c, opts=o)
                torch.cuda.synchronize()
                rows[prec].append(time.perf_counter() - t0)
                per_cg[prec].append(rows[prec][-1] / max(1, st["cg_iters"]))
                costs[prec].append(st["cost"])
                errs[prec].append(st["err_r"] + st["err_c"])
        med = {k: float(np.median(v)) for k, v in rows.items()}
        p = W.mnist_like_problem(2000, kind)
        C = torch.from_numpy(p.C).to(dev)
        r = torch.from_numpy(p.r).to(dev)
        c = torch.from_numpy(p.c).to(dev)
        o = eot.default_solve_opts(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol,
                                   precision="fp64")
        eot.eot_set_cg_persist(0, 0)
        try:
            eot.eot_solve(C, r, c, opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eot.eot_solve(C, r, c, opts=o)
            torch.cuda.synchronize()
            launches_s = time.perf_counter() - t0
        finally:
            eot.eot_set_cg_persist(1, 0)
        res[kind] = {"mixed_ms": 1e3 * med["mixed"], "fp64_ms": 1e3 * med["fp64"],
                     "fp64_cg_launched_per_iteration_ms_seed2000": 1e3 * launches_s,
                     "mixed_us_per_cg_iter": 1e6 * float(np.median(per_cg["mixed"])),
                     "fp64_us_per_cg_iter": 1e6 * float(np.median(per_cg["fp64"])),
                     "speedup_mixed_vs_fp64": med["fp64"] / med["mixed"],
                     "max_err": float(max(errs["mixed"] + errs["fp64"])),
                     "max_cost_rel_diff": float(max(abs(a - b) / b for a, b in
                                                    zip(costs["mixed"], costs["fp64"])))}
        log(f"grid28 {kind}: mixed {res[kind]['mixed_ms']:.1f} ms, fp64 {res[kind]['fp64_ms']:.1f} ms "
            f"(CG launched per iteration: {1e3 * launches_s:.1f} ms), "
            f"cost rel diff {res[kind]['max_cost_rel_diff']:.1e}")
    return res


def batch_measure(args, eot, W, dev, host_path=True):
    """The ragged batch: 512 grid problems, sides uniform on 16..64 (n = side^2
    in [256, 4096]), integer grid positions as 2-D points with the cost
    recomputed on the fly, temperature 1/32 -> 1e-3, tol 1e-6; one
    eot_solve_batched call per precision on the persistent single-launch path,
    and (host_path) the host-worker path in mixed precision for comparison."""
    import torch
    sides = W.batch_sides()
    items = []
    for k in range(len(sides)):
        p = W.batch_problem(k, sides=sides)
        pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
        items.append((pc, torch.from_numpy(p.r).to(dev), torch.from_numpy(p.c).to(dev)))
    torch.cuda.synchronize()
    res = {"workload": f"{len(items)} grid problems, n = side^2, side uniform on 16..64, "
                       f"on-the-fly 2-D points, temperature 1/32 -> 1e-3, tol 1e-6",
           "problems": len(items), "mean_n2": float(np.mean([float(s) ** 4 for s in sides])),
           "workers": args.batch_workers}
    legs = [("mixed", 1), ("fp64", 1)] + ([("mixed", 0)] if host_path else [])
    for prec, pers in legs:
        key = prec if pers else f"{prec}_host_workers"
        log(f"batch: {len(items)} problems, {prec}, "
            + ("one persistent launch" if pers else f"{args.batch_workers} host workers"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs, stats, status = eot.eot_solve_batched(items, workers=args.batch_workers,
                                                    gamma_init=1.0 / 32.0, gamma_final=1e-3,
                                                    tol=1e-6, precision=prec, check=False,
                                                    batch_persistent=pers)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        errs = [st["err_r"] + st["err_c"] for st in stats]
        # plan entries evaluated: passes x n m of every problem
        ent = float(sum(sum(v for k, v in st.items() if k.startswith("passes_")) * float(s) ** 4
                        for st, s in zip(stats, sides)))
        res[key] = {"seconds": dt, "problems_per_s": len(items) / dt,
                    "failed": int(sum(1 for x in status if x != 0)),
                    "max_err": float(max(errs)),
                    "newton_steps": int(sum(st["newton_steps"] for st in stats)),
                    "cg_iters": int(sum(st["cg_iters"] for st in stats)),
                    "mixed_stalls": int(sum(st["mixed_stalls"] for st in stats)),
                    "range_retries": int(sum(st["range_retries"] for st in stats)),
                    "entry_passes": ent, "entries_per_s": ent / dt}
        log(f"  {dt:.2f} s, failed {res[key]['failed']}, max err {max(errs):.2e}, "
            f"{ent / dt / 1e12:.2f} T plan entries/s")
        if key == "fp64":
            sol64 = outs
    # the backward over the whole batch (eot_gradient_batched) at the FP64
    # solutions: d(W + S) for X, Y, r, c of every problem
    gprobs = [(pc, 1e-3, f, g) for (pc, _, _), (f, g) in zip(items, sol64)]
    res["backward"] = {"workload": f"eot_gradient_batched over the {len(items)} FP64 solutions, "
                                   f"w_W = w_S = 1, outputs X, Y, r, c",
                       "workers": args.batch_workers}
    for prec, tol in (("fp64", 1e-11), ("mixed", 1e-5)):
        eot.eot_gradient_batched(gprobs[:8], w_W=1.0, w_S=1.0, tol=tol, precision=prec,
                                 workers=args.batch_workers, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gout = eot.eot_gradient_batched(gprobs, w_W=1.0, w_S=1.0, tol=tol, precision=prec,
                                        workers=args.batch_workers, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res["backward"][prec] = {"seconds": dt, "problems_per_s": len(gprobs) / dt, "cg_tol": tol,
                                 "failed": int(sum(1 for o in gout if o["status"] != 0)),
                                 "cg_iters": int(sum(o["cg_iters"] for o in gout))}
        log(f"batch backward {prec}: {dt:.2f} s, {res['backward'][prec]['cg_iters']} CG iterations, "
            f"failed {res['backward'][prec]['failed']}")
    res["speedup_mixed_vs_fp64"] = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    if host_path:
        res["speedup_persistent_vs_host_workers"] = (res["mixed_host_workers"]["seconds"]
                                                     / res["mixed"]["seconds"])
    return res


def points_only(eot, W, dev, iters=2):
    """The point-cloud mixed HVP of points_measure alone (one warm-up pass, then
    `iters` passes), for counter runs."""
    import torch
    p = W.point_cloud_problem()
    n, m = p.n, p.m
    pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
    gamma = 1e-2
    rng = np.random.default_rng(1)
    f = torch.from_numpy(gamma * (np.log(p.r) + 0.5 * rng.standard_normal(n))).to(dev)
    g = torch.from_numpy(gamma * (np.log(p.c) + 0.5 * rng.standard_normal(m))).to(dev)
    x = torch.from_numpy(rng.standard_normal(n)).to(dev)
    y = torch.from_numpy(rng.standard_normal(m)).to(dev)
    shift = eot.eot_marginals(pc, gamma, f, g, precision="mixed", want=("log_rP",))["log_rP"]
    for _ in range(1 + iters):
        eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    # then the product with the marginals given: one marginal pass and 1 + iters
    # HVP passes of the same kernel (k_pass<..., 1, 1, 0, ...>)
    mg = eot.eot_marginals(pc, gamma, f, g, row_shift=shift, precision="mixed",
                           want=("log_rP", "log_cP"))
    for _ in range(1 + iters):
        eot.eot_hvp_with_marginals(pc, gamma, f, g, mg["log_rP"], mg["log_cP"], 1.0, x, y,
                                   precision="mixed")
    torch.cuda.synchronize()
    print(json.dumps({"mode": "points-only", "hvp_launches": 1 + iters,
                      "hvp_with_marginals_launches": 1 + iters, "entries": float(n) * m}),
          flush=True)


def highd_only(eot, W, dev, iters=5):
    """The high-dimensional mixed HVP of highd_measure alone (one warm-up pass,
    then `iters` passes), for counter runs."""
    import torch
    p = W.embedding_problem(1 << 16, d=64)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(dev), torch.from_numpy(p.Y).to(dev), p.scale)
    gamma = 1e-2
    rng = np.random.default_rng(1)
    f = torch.from_numpy(gamma * (np.log(p.r) + 0.5 * rng.standard_normal(p.n))).to(dev)
    g = torch.from_numpy(gamma * (np.log(p.c) + 0.5 * rng.standard_normal(p.m))).to(dev)
    x = torch.from_numpy(rng.standard_normal(p.n)).to(dev)
    y = torch.from_numpy(rng.standard_normal(p.m)).to(dev)
    shift = eot.eot_marginals(pc, gamma, f, g, precision="mixed", want=("log_rP",))["log_rP"]
    for _ in range(1 + iters):
        eot.eot_hvp(pc, gamma, f, g, 1.0, x, y, row_shift=shift, precision="mixed")
    torch.cuda.synchronize()
    log(f"high-d only: {1 + iters} mixed HVP passes at n = m = {p.n}, d = 64")


def kernels_only(args, eot, W, p, C, dev):
    """The HVP pass (as in the full run, in --kernels-prec) and a 1 GiB
    device-to-device copy whose fetched / written bytes calibrate the memory
    counters."""
    import torch
    n, m = p.n, p.m
    gamma = p.gamma_final
    rng = np.random.default_rng(1)
    f = torch.from_numpy(gamma * (np.log(p.r) + 0.5 * rng.standard_normal(n))).to(dev)
    g = torch.from_numpy(gamma * (np.log(p.c) + 0.5 * rng.standard_normal(m))).to(dev)
    x = torch.from_numpy(rng.standard_normal(n)).to(dev)
    y = torch.from_numpy(rng.standard_normal(m)).to(dev)
    shift = eot.eot_marginals(C, gamma, f, g, precision="mixed", want=("log_rP",))["log_rP"]
    for _ in range(args.hvp_iters):
        eot.eot_hvp(C, gamma, f, g, 1.0, x, y, row_shift=shift, precision=args.kernels_prec)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(args.hvp_iters):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernels-only", "precision": args.kernels_prec,
                      "hvp_launches": args.hvp_iters,
                      "copy_bytes": 4 * src.numel(), "copy_launches": args.hvp_iters}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hvp-iters", type=int, default=20)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-points", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grid28", action="store_true")
    ap.add_argument("--no-sinkhorn", action="store_true")
    ap.add_argument("--sinkhorn-sweeps", type=int, default=2000,
                    help="cap of Sinkhorn sweeps per temperature for the baseline run")
    ap.add_argument("--batch-workers", type=int, default=8)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the HVP kernel loop and a 1 GiB device copy (for counter runs)")
    ap.add_argument("--kernels-prec", choices=("mixed", "fp64"), default="mixed",
                    help="precision of the --kernels-only HVP passes")
    ap.add_argument("--points-only", action="store_true",
                    help="only 1 + 2 mixed point-cloud HVP passes (n = m = 2^20, d = 3; for "
                         "counter runs)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 512-problem batch in both precisions (for trace runs)")
    ap.add_argument("--grid28-only", choices=("l1", "sqeuclid"),
                    help="only one FP64 solve of the 28 x 28 grid (seed 2000) with that cost, after "
                         "one untimed solve (for trace runs)")
    ap.add_argument("--points-solve-only", action="store_true",
                    help="only the mixed solve of the n = m = 65536 Gaussian-mixture clouds in R^3 "
                         "(temperature 1/32 -> 1e-4, tol 1e-4; for trace runs)")
    ap.add_argument("--highd-only", action="store_true",
                    help="only 1 + 5 mixed high-dimensional HVP passes (n = m = 65536, d = 64; "
                         "for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_02067_amd import eot, workloads as W

    dev = torch.device("cuda:0")
    if args.grid28_only:
        p = W.mnist_like_problem(2000, args.grid28_only)
        C = torch.from_numpy(p.C).to(dev)
        r = torch.from_numpy(p.r).to(dev)
        c = torch.from_numpy(p.c).to(dev)
        o = eot.default_solve_opts(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol,
                                   precision="fp64")
        eot.eot_solve(C, r, c, opts=o)
        _, _, st = eot.eot_solve(C, r, c, opts=o)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "grid28-only", "cost": args.grid28_only,
                          "cg_iters": st["cg_iters"], "newton_steps": st["newton_steps"],
                          "seconds": st["seconds"]}), flush=True)
        return
    if args.highd_only:
        highd_only(eot, W, dev)
        return
    if args.points_solve_only:
        q = W.point_cloud_problem(n=1 << 16)
        qc = eot.PointCloud(torch.from_numpy(q.X).to(dev), torch.from_numpy(q.Y).to(dev), q.scale)
        t0 = time.perf_counter()
        _, _, st = eot.eot_solve(qc, torch.from_numpy(q.r).to(dev), torch.from_numpy(q.c).to(dev),
                                 gamma_init=q.gamma_init, gamma_final=q.gamma_final, tol=q.tol,
                                 precision="mixed")
        torch.cuda.synchronize()
        print(json.dumps({"mode": "points-solve-only", "n": q.n, "seconds": time.perf_counter() - t0,
                          "passes": sum(v for k, v in st.items() if k.startswith("passes_")),
                          "cg_iters": st["cg_iters"], "newton_steps": st["newton_steps"],
                          "err": st["err_r"] + st["err_c"]}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"mode": "batch-only",
                          "batch": batch_measure(args, eot, W, dev, host_path=False)}), flush=True)
        return
    if args.points_only:
        points_only(eot, W, dev)
        return
    side = 128
    p = W.large_grid_problem(args.seed)
    n = m = p.n
    log(f"building {n}x{m} FP32 cost on {torch.cuda.get_device_name(0)}")
    C = W.grid_cost_device(side, "sqeuclid", dev)
    r = torch.from_numpy(p.r).to(dev)
    c = torch.from_numpy(p.c).to(dev)
    torch.cuda.synchronize()
    cost_bytes = 4.0 * n * m

    if args.kernels_only:
        kernels_only(args, eot, W, p, C, dev)
        return

    def solve(prec):
        o = eot.default_solve_opts(gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                                   tol=p.tol, precision=prec)
        return eot.eot_solve(C, r, c, opts=o)

    def timed_solve(prec):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        f, g, st = solve(prec)
        e1.record()
        torch.cuda.synchronize()
        return f, g, st, e0.elapsed_time(e1) / 1e3

    for w in range(args.warmup):
        log(f"warmup solve {w + 1}/{args.warmup} (mixed)")
        f, g, st, dt = timed_solve("mixed")
        log(f"  {dt:.3f} s status={st['status']} err={st['err_r'] + st['err_c']:.2e}")
    times, stats = [], []
    torch.cuda.synchronize()
    for k in range(args.steps):
        f, g, st, dt = timed_solve("mixed")
        times.append(dt)
        stats.append(st)
        log(f"step {k + 1}/{args.steps}: {dt:.3f} s err={st['err_r'] + st['err_c']:.2e} "
            f"newton={st['newton_steps']} cg={st['cg_iters']} mdot={st['mdot_steps']}")
    torch.cuda.synchronize()
    st = stats[-1]
    passes = (st["passes_newton"] + st["passes_linesearch"] + st["passes_sinkhorn"]
              + st["passes_projection"] + st["passes_other"])
    t_mixed = float(np.mean(times))
    value = passes * cost_bytes / t_mixed / 1e9

    fp64 = None
    if not args.no_fp64:
        log("FP64 solve (time to 1e-6 in plain FP64)")
        f64, g64, st64, t64 = timed_solve("fp64")
        log(f"  {t64:.3f} s err={st64['err_r'] + st64['err_c']:.2e} newton={st64['newton_steps']}")
        fp64 = {"seconds": t64, "err": st64["err_r"] + st64["err_c"], "cost": st64["cost"],
                "status": st64["status"], "newton_steps": st64["newton_steps"],
                "cg_iters": st64["cg_iters"]}

    # HVP kernel and the two CG pass kernels at the solution potentials.
    shift = eot.eot_marginals(C, p.gamma_final, f, g, want=("log_rP",))["log_rP"]
    gen = torch.Generator(device=dev).manual_seed(0)
    x = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
    y = torch.randn(m, dtype=torch.float64, device=dev, generator=gen)

    def time_calls(fn, iters):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / iters

    def kernel_us(fn, iters, **filt):
        """Average duration of the streaming-pass kernel alone: the library
        brackets each pass launch with HIP events on its stream."""
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        eot.eot_pass_timing(True)
        for _ in range(iters):
            fn()
        torch.cuda.synchronize()
        k, ms = eot.eot_pass_timing_read(**filt)
        eot.eot_pass_timing(False)
        return ms * 1e3 / k

    # Algorithmic bytes per launch: the FP32 cost once plus the FP64 vectors read
    # (potentials, shift, weights) and written (results).
    kern = {}
    hvp_bytes = cost_bytes + 8.0 * (3 * n + 2 * m) + 8.0 * (n + m)
    col_bytes = cost_bytes + 8.0 * (2 * n + m) + 8.0 * m
    row_bytes = cost_bytes + 8.0 * (2 * n + m) + 8.0 * n
    for prec in ("mixed", "fp64"):
        call_hvp = lambda: eot.eot_hvp(C, p.gamma_final, f, g, 1.0, x, y, row_shift=shift,
                                       precision=prec)
        call_col = lambda: eot.eot_marginals(C, p.gamma_final, f, g, row_shift=shift,
                                             precision=prec, want=("log_cP",))
        call_row = lambda: eot.eot_marginals(C, p.gamma_final, f, g, row_shift=shift,
                                             precision=prec, want=("log_rP",))
        mg = eot.eot_marginals(C, p.gamma_final, f, g, row_shift=shift, precision=prec,
                               want=("log_rP", "log_cP"))
        call_hvpm = lambda: eot.eot_hvp_with_marginals(C, p.gamma_final, f, g, mg["log_rP"],
                                                       mg["log_cP"], 1.0, x, y, precision=prec)
        for name, fn, nbytes, filt in (
                ("hvp", call_hvp, hvp_bytes, dict(fused_hvp=1)),
                ("hvp_with_marginals", call_hvpm, hvp_bytes, dict(nr=1, nc=1, fused_hvp=0)),
                ("colpass", call_col, col_bytes, dict(nr=0, nc=1)),
                ("rowpass", call_row, row_bytes, dict(nr=1, nc=0))):
            us = kernel_us(fn, args.hvp_iters, precision=prec, **filt)
            call = time_calls(fn, args.hvp_iters) * 1e6
            kern[f"{name}_{prec}"] = {"kernel_us": us, "gbs": nbytes / (us * 1e-6) / 1e9,
                                      "call_us": call, "bytes": nbytes}
        log(f"{prec}: hvp {kern[f'hvp_{prec}']['kernel_us']:.1f} us "
            f"({kern[f'hvp_{prec}']['gbs']:.0f} GB/s; with marginals "
            f"{kern[f'hvp_with_marginals_{prec}']['kernel_us']:.1f} us) "
            f"col {kern[f'colpass_{prec}']['kernel_us']:.1f} us "
            f"row {kern[f'rowpass_{prec}']['kernel_us']:.1f} us (kernel only)")
    hvp = kern["hvp_mixed"]

    sink = None
    if not args.no_sinkhorn:
        log(f"MDOT-Sinkhorn baseline (mixed, <= {args.sinkhorn_sweeps} sweeps per temperature)")
        o = eot.default_solve_opts(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol,
                                   precision="mixed", projection="sinkhorn",
                                   max_sinkhorn=args.sinkhorn_sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, sst = eot.eot_solve(C, r, c, opts=o, allow_not_converged=True)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
        sink = {"seconds": dts, "status": sst["status"], "err": sst["err_r"] + sst["err_c"],
                "sweeps": sst["sinkhorn_iters"], "mdot_steps": sst["mdot_steps"],
                "final_gamma": sst["final_gamma"],
                "note": "MDOT with Sinkhorn as the projection on the same passes; status 4 = "
                        "sweep cap reached before the target error"}
        log(f"  {dts:.2f} s status={sst['status']} err={sink['err']:.2e} sweeps={sst['sinkhorn_iters']} "
            f"final gamma={sst['final_gamma']:.1e}")

    rnd = round_measure(eot, C, p.gamma_final, f, g, r, c)

    pts = None
    if not args.no_points:
        del C
        torch.cuda.empty_cache()
        pts = points_measure(args, eot, W, dev)

    highd = None
    if not args.no_points:
        highd = highd_measure(args, eot, W, dev)

    grid28 = None if (args.no_fp64 or args.no_grid28) else grid28_measure(eot, W, dev)
    c1 = None if (args.no_fp64 or args.no_grid28) else c1_measure(eot, W, dev)

    batch = None
    grad = None
    if not args.no_batch:
        batch = batch_measure(args, eot, W, dev)
        grad = grad_measure(eot, W, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        cpu = cpu_baseline(p, lambda rows: W.grid_cost_rows(side, rows), W, batch)

    out = {
        "metric": "HVP GB/s (% HBM peak); time-to-1e-6 marginal error, mixed vs plain FP64",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-plan/f64-accum",
        "data": "synthetic",
        "config": {"workload": "grid128 n=m=16384 dense FP32 sqeuclid cost, 3-blob marginals "
                               "seed 3000, temperature 1/32 -> 1e-5, tol 1e-6, mixed precision "
                               "solve (1 step = 1 solve)",
                   "n": n, "m": m, "passes_per_step": passes,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": hvp["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hvp["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_pass<mixed, fused HVP>: one pass, row + column reductions",
                     "bytes_per_launch": hvp_bytes, "kernel_us": hvp["kernel_us"]},
        "time_to_1e6": {"mixed_s": t_mixed, "fp64_s": fp64["seconds"] if fp64 else None,
                        "speedup": (fp64["seconds"] / t_mixed) if fp64 else None,
                        "mixed_err": st["err_r"] + st["err_c"],
                        "fp64_err": fp64["err"] if fp64 else None,
                        "cost_rel_diff": (abs(st["cost"] - fp64["cost"]) / fp64["cost"]) if fp64 else None,
                        "mixed_newton_steps": st["newton_steps"], "mixed_cg_iters": st["cg_iters"],
                        "mixed_stalls": st["mixed_stalls"], "mixed_range_retries": st["range_retries"],
                        "fp64_newton_steps": fp64["newton_steps"] if fp64 else None,
                        "fp64_cg_iters": fp64["cg_iters"] if fp64 else None},
        "time_to_1e6_grid28": grid28,
        "points64_fp64": c1,
        "sinkhorn_baseline": sink,
        "kernels": kern,
        "round": rnd,
        "gradient": grad,
        "points": pts,
        "highd": highd,
        "batch": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
