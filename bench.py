"""Benchmark: IFMM factor + solve on one MI355X at N = 1,048,576, mixed
precision against FP64.

Workload (one step = the whole hot path on one batch of synthetic input):
  1,048,576 i.i.d. uniform points in [0,1]^2, K(r) = exp(-r/0.1) with
  A_ii = 1 + 1e-2 (sigma^2 = 1e-2), leaf size 64 (7 levels), 6 x 6 Chebyshev
  (rank 36), compression eps = 1e-8, one N(0,1) right-hand side; factor
  (assembly + Algorithm 1) then solve (Algorithm 2) with FP64 refinement
  until ||b - A x|| / ||b|| <= 1e-8 against the FMM matrix.
The headline runs the mixed-precision factor (FP32 blocks, Schur updates and
recompression; FP64 pivot inverses, top solve, FMM product, residuals and
vectors); the same steps with the FP64 factor are timed after it for the
speedup.  Inputs are resident in HBM before the timed regions; a timed
region covers K complete steps (ifmm_factor + ifmm_solve + ifmm_destroy).
Before the warmup, one untimed step times every launch family with HIP
events (the per-family breakdown in the output); the timed steps put HIP
events around the launches of the dominant single-kernel family only (the
roofline's live launch duration), so the other launches run back to back.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).  The
roofline's "traffic" is the HBM traffic per launch of its kernel from the
committed rocprofv3 counter runs (null once the kernel sources differ from the
ones measured); `--copy-cal` runs only the known-size copy those counter runs
are scaled by.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s IFMM factor+solve at N=1M, rel resid 1e-8: mixed vs FP64 GPU"
# MI355X peaks: HBM3E, FP64 and FP32 (vector and matrix alike) dense rates.
PEAK = {"hbm_GBs": 8000.0, "fp64_TFs": 78.6, "fp32_TFs": 157.3}
WORKLOAD = ("1,048,576 uniform points in [0,1]^2, exp(-r/0.1) + 1e-2 I, leaf 64, "
            "p=6 (rank 36), eps 1e-8, 1 rhs, factor+solve with FP64 refinement to 1e-8; "
            "value: mixed-precision factor (FP32 blocks), fp64 figures alongside")
# Profile slots whose launches are all one kernel instantiation, per factor
# precision (the pivoted QR, the inverse, the products slot (GEMMs and M2L
# assembly), the copies slot (adds and transitions), the other elimination
# steps and the solve sweeps (one kernel per step) span several kernels).
SINGLE_KERNEL = {
    "fp64": {"stackqr": "k_stackqr<double>", "elim": "k_elim<double, 2>",
             "touch_xform": "k_touch_xform<double>", "stack_win": "k_stackqr_win<double>"},
    "fp32": {"qr_f32": "k_qr<float>", "stackqr_f32": "k_stackqr<float>", "elim_f32": "k_elim<float, 2>",
             "touch_xform_f32": "k_touch_xform<float>", "stack_win_f32": "k_stackqr_win<float>"},
}


SUB_SIDE = 1.0 / 16  # sub-squares of the 1M point set: 16 x 16 of them


def _oracle_subsquare(args):
    """Factor + refined solve of one sub-square of the point set by the
    oracle on one core (one BLAS thread); returns (points, seconds)."""
    n_full, ix, iy = args
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle.ifmm import IFMM
    from oracle.kernels import Kernel

    pts = workloads.points_for("c3_exp_1m", n_full)
    b = workloads.rhs_for("c3_exp_1m", n_full)[:, 0]
    lo = (ix * SUB_SIDE, iy * SUB_SIDE)
    m = ((pts[:, 0] >= lo[0]) & (pts[:, 0] < lo[0] + SUB_SIDE) &
         (pts[:, 1] >= lo[1]) & (pts[:, 1] < lo[1] + SUB_SIDE))
    p, bb = pts[m], b[m]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = IFMM(p, Kernel("exp", 0.1), 1e-8, 64, 6, "const", 1.01, lo=lo, size=SUB_SIDE)
        o.factor()
        o.solve_refined(bb, 1e-8)
        dt = time.perf_counter() - t0
    return len(p), dt


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_full):
    """The oracle, untuned, on sub-squares of the same point set (same density
    and leaf-box width as the full problem): one core, then every usable core
    (one process per core, one sub-square at a time each).  Run before the GPU
    is touched, so the worker processes are plain forks."""
    import multiprocessing as mp

    single = [(n_full, 0, 0), (n_full, 1, 0), (n_full, 0, 1)]
    n1, t1 = 0, 0.0
    for a in single:
        n, dt = _oracle_subsquare(a)
        n1, t1 = n1 + n, t1 + dt
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    many = [(n_full, 2 + j % 14, 2 + j // 14) for j in range(2 * cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_subsquare, many, chunksize=1)
    tw = time.perf_counter() - t0
    nm = sum(n for n, _ in res)
    return {"value": nm / tw, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(many)} sub-squares of side 1/16 of the same 1M point set ({nm} points, "
                      f"leaf boxes of the full problem's width), same kernel, p, eps, FP64, refinement to "
                      f"1e-8, one process per core (one BLAS thread each); {tw:.1f} s wall",
            "single_core": {"value": n1 / t1, "unit": "unknowns/s", "cores": 1,
                            "sample": f"{len(single)} sub-squares ({n1} points), {t1:.1f} s on 1 thread"},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(),
                     "usable_cpus": len(os.sched_getaffinity(0))}}


def dominant(fam, prec):
    """The profile slot with the most kernel time among those whose launches
    are all one kernel instantiation."""
    single = [k for k in fam if k in SINGLE_KERNEL[prec] and fam[k]["launches"] > 0]
    return max(single, key=lambda k: fam[k]["ms"])


# HBM traffic per launch of the roofline kernel, from two rocprofv3 counter
# runs of `bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp64
# --no-extra` (pass 1 FETCH_SIZE, pass 2 WRITE_SIZE; KiB per dispatch,
# averaged over its 108 dispatches), each scaled by what the same counter
# reads for the known-size copy of `bench.py --copy-cal` (1 GiB read:
# FETCH_SIZE 524,303 KiB, factor 2.000; 1 GiB written: WRITE_SIZE 1,048,576
# KiB, factor 1.000); summary in profiles/ifmm_c3_1m_exp_mixed_pmc_traffic.md.
# Valid only for the kernel sources the counters were taken on (their
# SHA-256 below): traffic is null after any change to them.
PMC_TRAFFIC = {"kernel": "k_elim<float, 2>", "fetch_bytes": 3.3854e+08, "write_bytes": 2.6622e+08,
               "sources": ("paper_1407_1572_amd/csrc/ifmm_linalg.hip", "paper_1407_1572_amd/csrc/ifmm_internal.h"),
               "sha256": "b1c2f4f3530850eed8c87a996528bac5f72a7b982a1b548ed5ff622d35ee4868"}


def pmc_traffic(kernel):
    import hashlib
    if kernel != PMC_TRAFFIC["kernel"]:
        return None
    h = hashlib.sha256()
    for f in PMC_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != PMC_TRAFFIC["sha256"]:
        return None
    return PMC_TRAFFIC["fetch_bytes"] + PMC_TRAFFIC["write_bytes"]


def roofline(fam, dom, nrec, prec):
    d = fam[dom]
    t_s = d["ms"] / 1e3
    flops_rate = d["flops"] / t_s / 1e12 if t_s > 0 else 0.0
    bw = d["bytes"] / t_s / 1e9 if t_s > 0 else 0.0
    peak_f = PEAK["fp32_TFs"] if dom.endswith("_f32") else PEAK["fp64_TFs"]
    if d["bytes"] / (PEAK["hbm_GBs"] * 1e9) > d["flops"] / (peak_f * 1e12):
        roof = {"bound": "hbm", "achieved": bw, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": bw / PEAK["hbm_GBs"], "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": flops_rate, "peak": peak_f, "unit": "TFLOP/s",
                "frac": flops_rate / peak_f, "traffic": None}
    kern = SINGLE_KERNEL[prec][dom]
    traffic = pmc_traffic(kern)
    if traffic is not None and roof["bound"] == "hbm":
        roof["traffic"] = traffic
        roof["traffic_GBs"] = traffic / (d["ms"] / max(1, d["launches"]) / 1e3) / 1e9
        roof["traffic_over_algorithmic"] = traffic / (d["bytes"] / max(1, d["launches"]))
        roof["traffic_unit"] = "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    # both fractions of the Schur-update kernel (memory and matrix-core side)
    roof["frac_hbm"] = bw / PEAK["hbm_GBs"]
    roof["frac_mfma"] = flops_rate / peak_f
    roof.update({"kernel": kern, "launches_per_step": d["launches"] / nrec,
                 "avg_launch_ms": d["ms"] / max(1, d["launches"]),
                 "algorithmic_flops_per_launch": d["flops"] / max(1, d["launches"]),
                 "algorithmic_bytes_per_launch": d["bytes"] / max(1, d["launches"]),
                 "achieved_GBs": bw, "achieved_TFs": flops_rate,
                 "timing": "HIP events on the launch stream around every launch of this kernel, "
                           "over the timed steps"})
    return roof


def families(recs):
    fam = {}
    for st, _ in recs:
        for name, kv in st["kernels"].items():
            a = fam.setdefault(name, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
            for key in a:
                a[key] += kv[key]
    return fam


def run(prec, pts, b, steps, warmup, N):
    import torch

    from paper_1407_1572_amd import IFMMSolver

    def step(profile):
        t0 = time.perf_counter()
        s = IFMMSolver(pts, "exp", 0.1, "const", 1.01, 1e-8, 64, 36, refine_tol=1e-8, profile=profile,
                       precision=prec)
        t1 = time.perf_counter()
        s.solve(b)
        st, info = s.stats(), s.last_info
        t2 = time.perf_counter()
        s.close()
        t3 = time.perf_counter()
        st["wall_ms"] = {"factor_call": (t1 - t0) * 1e3, "solve_call": (t2 - t1) * 1e3, "destroy": (t3 - t2) * 1e3}
        return st, info

    def say(tag, st, info):
        print(f"{prec} {tag}: t_a {st['assembly_ms']:.0f} ms  t_f {st['factor_ms']:.0f} ms  "
              f"t_s {st['last_solve_ms']:.0f} ms  resid {info['residual']:.2e} ({info['iterations']} sweeps)  "
              f"wall {st['wall_ms']}", file=sys.stderr, flush=True)

    # One untimed step with every launch family timed by HIP events: the
    # per-family breakdown, and which single-kernel family dominates.  The
    # timed steps then put events around that kernel's launches only.
    full = step(True)
    say("profiled step", *full)
    fam_full = families([full])
    dom = dominant(fam_full, prec)
    only = [dom[:-4] if dom.endswith("_f32") else dom]
    for w in range(warmup):
        say(f"warmup {w}", *step(only))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(steps):
        recs.append(step(only))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    for k, r in enumerate(recs):
        say(f"step {k}", *r)
    fam = families(recs)
    st0, info0 = recs[-1]
    summary = {"unknowns_per_s": N / (ms / 1e3), "ms_per_step": ms,
               "t_assembly_ms": st0["assembly_ms"], "t_factor_ms": st0["factor_ms"],
               "t_solve_ms": st0["last_solve_ms"], "wall_ms": st0["wall_ms"],
               "refine_status": max(info["status"] for _, info in recs),
               "refine_iterations": info0["iterations"], "final_residual": info0["residual"],
               "residual_history": info0["history"], "max_rank": st0["max_rank"],
               "level_max_rank": st0["level_max_rank"], "level_mean_rank": st0["level_mean_rank"],
               "factor_bytes": st0["factor_bytes"], "factor_flops": st0["factor_flops"],
               "profiled_step_ms": sum(full[0]["wall_ms"].values()),
               "kernels_per_step": {k: {"ms": v["ms"], "launches": v["launches"], "gflop": v["flops"] / 1e9,
                                        "gbyte": v["bytes"] / 1e9}
                                    for k, v in fam_full.items() if v["launches"] > 0},
               "kernels_per_step_source": "one untimed step with HIP events around every launch"}
    return summary, roofline(fam, dom, len(recs), prec)


def accuracy(pts, b, N):
    """Outside the timed region, one factor of each precision: the refined
    solution's residual against the FMM matrix, against the true kernel on
    1,000 sampled rows, the paper's error (b = A~ x_exact, x_exact ~ N(0,1);
    the notation table of the numerical section), and the mixed solution
    against the FP64 one."""
    import numpy as np
    import torch

    from paper_1407_1572_amd import IFMMSolver

    gen = np.random.default_rng(3003)
    rows = torch.from_numpy(np.sort(gen.choice(N, 1000, replace=False))).to(pts.device)
    x_exact = torch.from_numpy(np.random.default_rng(3004).standard_normal(N)).to(pts.device)
    c0, ell = 1.01, 0.1

    def true_rows(x):
        """(A x)[rows] with the exact kernel exp(-r/ell), A_ii = c0 (FP64, plain torch ops)."""
        out = torch.empty(len(rows), dtype=torch.float64, device=pts.device)
        for a in range(0, len(rows), 50):
            rr = rows[a:a + 50]
            d = torch.cdist(pts[rr], pts)
            K = torch.exp(-d / ell)
            K[torch.arange(len(rr), device=pts.device), rr] = c0
            out[a:a + 50] = K @ x
        return out

    res, xs = {}, {}
    for prec in ("fp32", "fp64"):
        s = IFMMSolver(pts, "exp", ell, "const", c0, 1e-8, 64, 36, refine_tol=1e-8, precision=prec)
        x = s.solve(b)
        info = s.last_info
        r_fmm = (b - s.matvec(x)).norm() / b.norm()
        r_true = (b[rows] - true_rows(x)).norm() / b[rows].norm()
        r_fmm_rows = (b - s.matvec(x))[rows].norm() / b[rows].norm()
        be = s.matvec(x_exact)
        xe = s.solve(be)
        err = (xe - x_exact).norm() / x_exact.norm()
        xs[prec] = x
        res["mixed" if prec == "fp32" else "fp64"] = {
            "direct_residual": info["history"][0], "refined_residual": float(r_fmm),
            "sweeps": info["iterations"], "residual_fmm_sampled_rows": float(r_fmm_rows),
            "residual_true_kernel_sampled_rows": float(r_true),
            "paper_error_x_exact": float(err)}
        s.close()
        torch.cuda.synchronize()
    res["mixed_vs_fp64"] = float((xs["fp32"] - xs["fp64"]).norm() / xs["fp64"].norm())
    res["note"] = ("residual_true_kernel_sampled_rows: ||b - A x|| / ||b|| over 1,000 seeded rows with the exact "
                   "kernel (the FMM matrix A~ at p = 6 differs from it by its interpolation error); "
                   "paper_error_x_exact: ||x - x_exact|| / ||x_exact|| for b = A~ x_exact, refined to 1e-8")
    return res


def gradients():
    """Gradients of L = 1/2 y^T A^-1 y, A = exp(-r/0.08) + 5e-3 I, on 262,144
    uniform points (eps 1e-10, FP64 factor refined to 1e-12): forward (factor +
    solve) and backward (transposed solve + FMM of dK/d ell) times, and the
    gradients in ell and sigma^2 against central finite differences of the
    loss (step 1e-5)."""
    import numpy as np
    import torch

    from paper_1407_1572_amd.autograd import gp_loss

    n, ell0, s20 = 262144, 0.08, 5e-3
    pts = torch.from_numpy(np.random.default_rng(1005).uniform(size=(n, 2))).to("cuda:0")
    y = torch.from_numpy(np.random.default_rng(2005).standard_normal(n)).to("cuda:0")
    kw = dict(eps=1e-10, leaf_size=64, rank=36, refine_tol=1e-12)
    out = {}
    for rep in range(2):  # the second run is reported (the first warms the block cache)
        yy = y.clone().requires_grad_(True)
        ell = torch.tensor(ell0, dtype=torch.float64, requires_grad=True)
        s2 = torch.tensor(s20, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = gp_loss(pts, yy, ell, s2, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = {"n": n, "loss": float(L.detach()), "d_ell": float(ell.grad), "d_sigma2": float(s2.grad),
               "dy_norm": float(yy.grad.norm()), "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3}
    h = 1e-5

    def loss(e, q):
        with torch.no_grad():
            return float(gp_loss(pts, y, e, q, **kw))

    fd_ell = (loss(ell0 + h, s20) - loss(ell0 - h, s20)) / (2 * h)
    fd_s2 = (loss(ell0, s20 + h) - loss(ell0, s20 - h)) / (2 * h)
    out.update(fd_d_ell=fd_ell, fd_d_sigma2=fd_s2, rel_err_d_ell=abs(out["d_ell"] - fd_ell) / abs(fd_ell),
               rel_err_d_sigma2=abs(out["d_sigma2"] - fd_s2) / abs(fd_s2),
               workload="262,144 uniform points, exp(-r/0.08) + 5e-3 I, leaf 64, p = 6, eps 1e-10, FP64 factor, "
                        "solve refined to 1e-12; central differences with step 1e-5")
    return out


def batched():
    """256 independent problems of uneven size (N_j log-uniform in [1,024,
    32,768], points seed 4000 + j), kernels alternating between 1/r with the
    row-sum diagonal and exp(-r/0.1) + 1e-2 I, leaf 64, p = 6, eps 1e-8, 8
    right-hand sides each (seed 5000 + j), FP32 factor with FP64 refinement
    to 1e-10: ifmm_factor_batched + ifmm_solve_batched in chunks of 64
    problems (factor, solve, free), with 1, 4, 8 and 16 host threads (streams)."""
    import numpy as np
    import torch

    import workloads
    from paper_1407_1572_amd import factor_batched, release_cached_memory, solve_batched

    release_cached_memory()  # the 1M-point factors' cached blocks are not the batch's sizes
    count, chunk = 256, 64
    ns = [int(round(np.exp(np.random.default_rng(3000 + j).uniform(np.log(1024), np.log(32768)))))
          for j in range(count)]
    pts = [torch.from_numpy(workloads.uniform(n, 4000 + j)).to("cuda:0") for j, n in enumerate(ns)]
    rhs = [torch.from_numpy(workloads.rhs(n, 8, 5000 + j)).to("cuda:0") for j, n in enumerate(ns)]
    kern = [{"kind": "inv_r", "ell": 0.0, "diag": "rowsum", "c0": 1.0} if j % 2 == 0 else
            {"kind": "exp", "ell": 0.1, "diag": "const", "c0": 1.01} for j in range(count)]
    kw = dict(eps=1e-8, leaf_size=64, rank=36, refine_tol=1e-10, precision="fp32")
    out = {"problems": count, "unknowns": int(sum(ns)), "nrhs": 8, "chunk": chunk, "min_n": min(ns),
           "max_n": max(ns)}
    for threads in (1, 4, 8, 16):
        for rep in range(2):  # the second pass is reported (the first warms the block cache)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            worst, sweeps = 0.0, 0
            for c0 in range(0, count, chunk):
                sv = factor_batched(pts[c0:c0 + chunk], kern[c0:c0 + chunk], threads=threads, **kw)
                solve_batched(sv, rhs[c0:c0 + chunk], threads=threads)
                for s in sv:
                    worst = max(worst, s.last_info["residual"])
                    sweeps = max(sweeps, s.last_info["iterations"])
                    s.close()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        out[f"threads_{threads}"] = {"seconds": dt, "unknowns_per_s": sum(ns) / dt,
                                     "worst_residual": worst, "max_sweeps": sweeps}
        print(f"batched, {threads} threads: {out[f'threads_{threads}']}", file=sys.stderr, flush=True)
    return out


BATCH_HW_QUEUES = 16


def batched_child():
    """The batched section in a child process whose HIP runtime opens
    BATCH_HW_QUEUES hardware queues (GPU_MAX_HW_QUEUES; with the default 4 the
    worker streams of 8 or 16 host threads share 4 queues and their
    launch-latency-bound chains overlap less: 512k -> 596k unknowns/s at 8
    threads, measured).  The child's progress goes to this stderr."""
    import subprocess

    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(BATCH_HW_QUEUES))
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--batched-only"], env=env,
                       stdout=subprocess.PIPE, text=True, timeout=1200)
    if r.returncode != 0:
        raise RuntimeError(f"batched child exited with {r.returncode}")
    out = json.loads(r.stdout.strip().splitlines()[-1])["batched"]
    out["hw_queues"] = BATCH_HW_QUEUES
    return out


def scaling(prec):
    """Factor and solve time per unknown and the largest rank at N = 4^k * 64
    (same parameters, uniform points of the same seed), second of two runs."""
    import torch

    import workloads
    from paper_1407_1572_amd import IFMMSolver

    out = {}
    for n in (16384, 65536, 262144):
        pts = torch.from_numpy(workloads.points_for("c3_exp_1m", n)).to("cuda:0")
        b = torch.from_numpy(workloads.rhs_for("c3_exp_1m", n)[:, 0].copy()).to("cuda:0")
        for _ in range(2):
            s = IFMMSolver(pts, "exp", 0.1, "const", 1.01, 1e-8, 64, 36, refine_tol=1e-8, precision=prec)
            s.solve(b)
            st = s.stats()
            s.close()
        out[str(n)] = {"t_factor_ns_per_unknown": st["factor_ms"] * 1e6 / n,
                       "t_assembly_ns_per_unknown": st["assembly_ms"] * 1e6 / n,
                       "t_solve_ns_per_unknown": st["last_solve_ms"] * 1e6 / n,
                       "max_rank": st["max_rank"], "level_max_rank": st["level_max_rank"]}
    return out


# The numerical section's benchmark: sigma_i + sum_{j != i} K(r_ij) sigma_j =
# f_i with its three singular kernels (a = 1e-3), points uniform in
# [-1, 1]^2, 8 x 8 Chebyshev nodes, tolerance 1e-14 (FP64 factor, direct solve);
# N in thousands as in its tables.  The paper's own figures (one CPU at
# 2.1 GHz, its C++ code): t_f seconds and r_m per N.
PAPER_SIZES_K = (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000)
PAPER_TABLES = {
    "log_a": {"t_f": (0.35, 0.71, 1.68, 3.21, 6.78, 16.79, 34.93, 73.87, 189.63, 412.48),
              "t_s": (0.007, 0.009, 0.026, 0.06, 0.13, 0.32, 0.72, 1.54, 4.09, 8.87),
              "r_m": (29, 31, 30, 37, 36, 40, 44, 48, 47, 51)},
    "inv_r_a": {"t_f": (0.42, 1.00, 2.37, 4.94, 9.92, 27.39, 61.34, 142.38, 398.23, 803.85),
                "t_s": (0.005, 0.015, 0.035, 0.092, 0.192, 0.567, 1.213, 2.492, 5.781, 12.436),
                "r_m": (45, 43, 49, 51, 57, 54, 59, 65, 68, 67)},
    "r2log_a": {"t_f": (0.11, 0.27, 0.64, 1.42, 2.76, 5.34, 10.89, 26.47, 72.37, 153.93),
                "t_s": (0.003, 0.007, 0.017, 0.041, 0.091, 0.262, 0.554, 1.192, 2.873, 6.121),
                "r_m": (22, 21, 25, 24, 27, 26, 28, 31, 30, 32)},
}


def paper_kernels(max_k):
    """Factor time, solve time, largest rank and the error ||x - x_exact|| /
    ||x_exact|| (b = A~ x_exact) of the three kernels over the paper's sizes."""
    import numpy as np
    import torch

    from paper_1407_1572_amd import IFMMError, IFMMSolver

    out = {}
    for kind in ("log_a", "inv_r_a", "r2log_a"):
        rows = []
        for j, nk in enumerate(PAPER_SIZES_K):
            if nk > max_k:
                break
            n = nk * 1000
            pts = torch.from_numpy(2.0 * np.random.default_rng(6000 + nk).uniform(size=(n, 2)) - 1.0).to("cuda:0")
            xe = torch.from_numpy(np.random.default_rng(7000 + nk).standard_normal(n)).to("cuda:0")
            rec = {"n": n, "paper": {q: PAPER_TABLES[kind][q][j] for q in ("t_f", "t_s", "r_m")}}
            try:
                for _ in range(2):  # the second run is reported (the first warms the block cache)
                    s = IFMMSolver(pts, kind, 1e-3, "const", 1.0, 1e-14, 128, 64, box=(-1.0, -1.0, 2.0))
                    b = s.matvec(xe)
                    x = s.solve(b)
                    st = s.stats()
                    s.close()
                rec.update(t_a=st["assembly_ms"] / 1e3, t_f=st["factor_ms"] / 1e3, t_s=st["last_solve_ms"] / 1e3,
                           r_m=st["max_rank"], level_max_rank=st["level_max_rank"],
                           cap_hits=sum(st["level_cap_hits"].values()),
                           error=float((x - xe).norm() / xe.norm()), kappa=st["kappa"])
            except IFMMError as e:
                rec["status"] = str(e)
            torch.cuda.synchronize()
            print(f"paper kernel {kind} N={n}: {rec}", file=sys.stderr, flush=True)
            rows.append(rec)
        out[kind] = rows
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the untimed accuracy figures and the factor-time-per-unknown sweep over N")
    ap.add_argument("--paper-kernels", type=int, default=0, metavar="MAX_K",
                    help="only sweep the numerical section's three kernels up to N = MAX_K thousand "
                         "(p = 8, tolerance 1e-14, [-1,1]^2, FP64) and print that table as one JSON line")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 256-problem batched factor + solve and print its JSON")
    ap.add_argument("--fp64-only", action="store_true",
                    help="only run the FP64 factor + solve of the workload (for profiling that path) and print "
                         "its figures as one JSON line")
    ap.add_argument("--copy-cal", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write kernel (3 times): the known-size reference "
                         "for scaling the HBM counters (FETCH_SIZE / WRITE_SIZE) of a counter run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the IFMM factor+solve of one problem runs on a "
              "single MI355X here (multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads

    dev = torch.device("cuda:0")
    if args.copy_cal:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print("copy-cal: 3 x (read 1 GiB, write 1 GiB) by torch.mul", flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched()}))
        return
    if args.paper_kernels:
        res = paper_kernels(args.paper_kernels)
        print(json.dumps({"workload": "numerical-section kernels (i)-(iii), a = 1e-3, uniform points in [-1,1]^2, "
                          "unit diagonal, p = 8 (rank 64), leaf 128, tolerance 1e-14, FP64 factor, direct solve; "
                          "paper: one 2.1 GHz CPU", "results": res}))
        return
    N = args.n
    cpu = None if args.no_cpu_baseline else cpu_baseline(N)
    pts = torch.from_numpy(workloads.points_for("c3_exp_1m", N)).to(dev)
    b = torch.from_numpy(workloads.rhs_for("c3_exp_1m", N)[:, 0].copy()).to(dev)
    torch.cuda.synchronize()

    if args.fp64_only:
        fp64, roof64 = run("fp64", pts, b, args.steps, args.warmup, N)
        print(json.dumps({"workload": WORKLOAD, "n": N, "fp64": fp64, "roofline_fp64": roof64}))
        return
    mixed, roof = run("fp32", pts, b, args.steps, args.warmup, N)
    fp64, roof64 = (None, None) if args.no_fp64 else run("fp64", pts, b, args.steps, args.warmup, N)
    def extra(name, fn):
        """An extra section of the line; an error in it is reported there and
        the headline figures above stand."""
        try:
            r = fn()
        except Exception as e:
            r = {"error": f"{type(e).__name__}: {e}"}
        print(f"{name}: {r}", file=sys.stderr, flush=True)
        return r

    acc = None if args.no_fp64 or args.no_extra else extra("accuracy", lambda: accuracy(pts, b, N))
    scal = None
    if not args.no_extra:
        def scaling_all():
            sc = {"fp32": scaling("fp32"), "fp64": None if args.no_fp64 else scaling("fp64")}
            for prec, rec in (("fp32", mixed), ("fp64", fp64)):
                if rec is not None and sc[prec] is not None:
                    sc[prec][str(N)] = {"t_factor_ns_per_unknown": rec["t_factor_ms"] * 1e6 / N,
                                        "t_assembly_ns_per_unknown": rec["t_assembly_ms"] * 1e6 / N,
                                        "t_solve_ns_per_unknown": rec["t_solve_ms"] * 1e6 / N,
                                        "max_rank": rec["max_rank"], "level_max_rank": rec["level_max_rank"]}
            return sc
        scal = extra("scaling", scaling_all)
    grads = None if args.no_extra else extra("gradients", gradients)
    batch = None if args.no_extra else extra("batched", batched_child)
    out = {
        "metric": METRIC, "value": mixed["unknowns_per_s"], "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N, "mixed": mixed, "fp64": fp64,
                   "speedup_mixed_vs_fp64": (fp64["ms_per_step"] / mixed["ms_per_step"]) if fp64 else None,
                   "roofline_fp64": roof64, "accuracy": acc, "scaling_in_n": scal,
                   "gradients": grads, "batched": batch},
        "roofline": roof,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
