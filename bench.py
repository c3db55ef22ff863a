#!/usr/bin/env python3
"""Benchmark of the short-characteristics + Jacobi ALI hot path on one MI355X.

A step is one whole pass of the hot path over the 128^3 scattering workload
(grey coherent scattering, eps = 1e-3, exponentially stratified opacity with a
vertical optical depth of 1e4, 48 rays): ingest of chi/eps/B with Lambda*, then
Jacobi ALI from S = B with FP32 difference-form sweeps and FP64 updates and
residuals until max |dS|/S <= 1e-6, then the moments epilogue (J, H, K, f = K/J,
Q and the heating sum) on the converged S.  Inputs are resident in HBM before the timed
region.  The JSON line reports cell*ray*bin updates per second over the timed
steps, ALI solves/s, p50/p99 solve latency, the sweep kernel against its roofline
(VALU-bound; durations from HIP events inside the library, see rt_problem_profile),
the plain FP64 GPU solve for comparison, and the FP64 CPU oracle on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell·ray·freq updates/s per formal solve; ALI solves/s; p50/p99 latency"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 VALU lane-operations/s
# (one non-packed FP32 op per lane per cycle; packed FP32 is disabled in this build).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU lane-operations of one FP32 difference-form update (closed-form
# branch): 3 bilinear interpolations (I-, S-, chi-: 4 each), dtau (2), exp (scale 1 +
# quarter-rate exp 4), g = (1 - E)/dtau (sub 1 + quarter-rate rcp 4 + mul 1),
# D update (3), accumulation of w D (1).
OPS_PER_UPDATE_F32 = 12 + 2 + 5 + 6 + 3 + 1


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_stage_f32_scattering128_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_kernels.hip")


def measured_traffic():
    """HBM bytes per sweep-stage launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (calibrated against a plain copy), or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        fields = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_launch:",
                                                                                   "kernel_source_sha256:")))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel_source_sha256", "").strip() != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(wl, sweeps):
    """FP64 oracle (single thread, as it stands) timed on a bounded number of formal
    solutions of the same workload."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    op = oracle.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi)
    S = wl.B.copy()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        op.sweep(S)
    dt = time.perf_counter() - t0
    updates = wl.cells * wl.na * wl.nf * sweeps
    return {"value": updates / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} formal solutions (sweeps) of the {wl.shape[0]}^3 x {wl.na}-ray workload, "
                      f"{updates / 1e6:.1f} M updates in {dt:.1f} s, FP64, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="grid edge of the scattering workload")
    ap.add_argument("--cpu-sweeps", type=int, default=2, help="oracle sweeps for the CPU baseline (0 = skip)")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 GPU comparison solve")
    ap.add_argument("--schedule", choices=["stages"], default="stages")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="profiling mode: run exactly this many ALI iterations per step instead of converging")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (for scaling rocprofv3 FETCH/WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(how the path would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1201_2222_amd as rt
    from paper_1201_2222_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "copies": 3}), flush=True)
        return
    wl = W.scattering(args.n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    chi, eps, B = dev(wl.chi), dev(wl.eps), dev(wl.B)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    cells = wl.cells
    mom = {k: torch.empty(m * cells, dtype=torch.float64, device="cuda")
           for k, m in (("J_int", 1), ("H_int", 3), ("K_int", 6), ("f_int", 6), ("Q_int", 1))}
    sched = rt.RT_SCHED_STAGES
    prob = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32,
                      schedule=sched)

    def step():
        prob.reset_periodic()
        prob.set_fields(chi, eps, B)
        status, st = prob.ali_solve(S, J, delta_c=wl.delta_c, max_iter=50000, per_bin_stop=True,
                                    fixed_iters=args.fixed_iters)
        if status != rt.RT_OK:
            raise RuntimeError(f"ALI did not converge: {st}")
        st["heating"] = prob.moments(S, want_heating=True, **mom)   # moments epilogue on the converged S
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rt.rt_problem_profile(prob.handle, True)
    lat, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        st = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        iters.append(st["iterations"])
        print(f"step: {lat[-1] * 1e3:.1f} ms, {st['iterations']} iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    prof = rt.rt_problem_profile_read(prob.handle)
    rt.rt_problem_profile(prob.handle, False)
    J32 = J.cpu().numpy()

    # one sweep per ALI iteration plus the moments sweep
    updates = float(wl.cells * wl.na * wl.nf * (sum(iters) + len(iters)))
    value = updates / total
    kernel_s = prof["kernel_ms"] / 1e3
    achieved = prof["updates"] * OPS_PER_UPDATE_F32 / kernel_s / 1e12 if kernel_s > 0 else 0.0
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "sweep_stage_kernel<float, true, 1, false>",
                "avg_launch_us": prof["kernel_ms"] * 1e3 / max(prof["launches"], 1),
                "timed_launches": prof["launches"],
                "ops_per_update": OPS_PER_UPDATE_F32}

    extra = {}
    if not args.no_f64:
        p64 = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F64,
                         schedule=sched)
        p64.set_fields(chi, eps, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, st64 = p64.ali_solve(S, J, delta_c=wl.delta_c, max_iter=50000, per_bin_stop=True)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        J64 = J.cpu().numpy()
        extra["f64_gpu_solve"] = {"seconds": t64, "iterations": st64["iterations"],
                                  "solves_per_s": 1.0 / t64,
                                  "updates_per_s": wl.cells * wl.na * wl.nf * st64["iterations"] / t64,
                                  "f32_vs_f64_max_rel_J": float(np.max(np.abs(J32 - J64) / np.abs(J64)))}
        p64.close()

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded, generated on the host)",
        "config": {"workload": f"scattering {wl.shape[0]}^3, 1 bin, {wl.na} rays, eps=1e-3, "
                               f"vertical tau 1e4, Jacobi ALI from S=B to max|dS/S|<=1e-6, "
                               f"FP32 sweeps + FP64 updates", "grid": list(wl.shape), "rays": wl.na,
                   "schedule": args.schedule,
                   "bins": wl.nf},
        "ali_solves_per_s": args.steps / total,
        "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
        "iterations": iters,
        "heating": st["heating"],
        "profiling_fixed_iters": args.fixed_iters or None,
        "roofline": roofline,
    }
    out.update(extra)
    if args.cpu_sweeps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sweeps)
    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
