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


def cpu_baseline(n_full):
    """The oracle, untuned, on sub-squares of the same point set (same density
    and leaf-box width as the full problem), one BLAS thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle.ifmm import IFMM
    from oracle.kernels import Kernel

    pts = workloads.points_for("c3_exp_1m", n_full)
    b = workloads.rhs_for("c3_exp_1m", n_full)[:, 0]
    side = 1.0 / 16
    tot_n, tot_t = 0, 0.0
    subs = [(0.0, 0.0), (side, 0.0), (0.0, side)]
    with threadpool_limits(limits=1):
        for lo in subs:
            m = ((pts[:, 0] >= lo[0]) & (pts[:, 0] < lo[0] + side) &
                 (pts[:, 1] >= lo[1]) & (pts[:, 1] < lo[1] + side))
            p, bb = pts[m], b[m]
            t0 = time.perf_counter()
            o = IFMM(p, Kernel("exp", 0.1), 1e-8, 64, 6, "const", 1.01, lo=lo, size=side)
            o.factor()
            o.solve_refined(bb, 1e-8)
            tot_t += time.perf_counter() - t0
            tot_n += len(p)
    return {"value": tot_n / tot_t, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(subs)} sub-squares of side 1/16 of the same 1M point set "
                      f"({tot_n} points, leaf boxes of the full problem's width), same kernel, "
                      f"p, eps, FP64, refinement to 1e-8; {tot_t:.1f} s on 1 thread"}


def dominant(fam, prec):
    """The profile slot with the most kernel time among those whose launches
    are all one kernel instantiation."""
    single = [k for k in fam if k in SINGLE_KERNEL[prec] and fam[k]["launches"] > 0]
    return max(single, key=lambda k: fam[k]["ms"])


# HBM traffic per launch of the roofline kernel, from two rocprofv3 counter
# runs of `bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp64` (pass 1
# FETCH_SIZE, pass 2 WRITE_SIZE; KiB per dispatch, averaged over its 108
# dispatches), each scaled by what the same counter reads for the known-size
# copy of `bench.py --copy-cal` (1 GiB read: FETCH_SIZE 524,303 KiB, factor
# 2.000; 1 GiB written: WRITE_SIZE 1,048,576 KiB, factor 1.000); summary in
# profiles/ifmm_c3_1m_exp_mixed_pmc_traffic.md.  Valid only for the kernel
# sources the counters were taken on (their SHA-256 below): traffic is null
# after any change to them.
PMC_TRAFFIC = {"kernel": "k_elim<float, 2>", "fetch_bytes": 1.4827e9, "write_bytes": 2.7078e8,
               "sources": ("paper_1407_1572_amd/csrc/ifmm_linalg.hip", "paper_1407_1572_amd/csrc/ifmm_internal.h"),
               "sha256": "1d8a7f21954cf3f5b8e97c879f98b05cf925819a5b67fe151c15b2604eb76cc3"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
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
    N = args.n
    pts = torch.from_numpy(workloads.points_for("c3_exp_1m", N)).to(dev)
    b = torch.from_numpy(workloads.rhs_for("c3_exp_1m", N)[:, 0].copy()).to(dev)
    torch.cuda.synchronize()

    mixed, roof = run("fp32", pts, b, args.steps, args.warmup, N)
    fp64, roof64 = (None, None) if args.no_fp64 else run("fp64", pts, b, args.steps, args.warmup, N)
    out = {
        "metric": METRIC, "value": mixed["unknowns_per_s"], "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N, "mixed": mixed, "fp64": fp64,
                   "speedup_mixed_vs_fp64": (fp64["ms_per_step"] / mixed["ms_per_step"]) if fp64 else None,
                   "roofline_fp64": roof64},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
