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
(VALU-bound; durations from HIP events inside the library, see rt_problem_profile;
with --ali gauss-seidel the chain kernel of the downward pass against HBM),
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
# (one non-packed FP32 op per lane per cycle; the library is compiled without packed FP32).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU lane-operations of one FP32 difference-form update (closed-form
# branch): 3 bilinear interpolations (I-, S-, chi-: 4 each), dtau (2), exp (scale 1 +
# quarter-rate exp 4), g = (1 - E)/dtau (sub 1 + quarter-rate rcp 4 + mul 1),
# D update (3), accumulation of w D (1).
OPS_PER_UPDATE_F32 = 12 + 2 + 5 + 6 + 3 + 1
# Second-order (Bezier) FP32 update, closed-form branch: 5 bilinear interpolations
# (I-, S-, chi-, S+, chi+: 20), dtau- and dtau+ (4), exp (5), E + alpha and gamma from
# e1, e2 with one reciprocal (15), S- - S0 and S+ - S0 formed in FP64 and converted (4),
# the control point (t = h1/h2 by reciprocal 5, a - b t^2 2, / 2(1 + t) by reciprocal
# 6, clamp between a and 0 4: 17), D update (3), accumulation (1).
OPS_PER_UPDATE_BEZ_F32 = 20 + 4 + 5 + 15 + 4 + 17 + 3 + 1
# Monotone quadratic upwind intensity, FP32 difference form: I = D + S at the 3 x 3
# stencil (9, FP64), four 1D quadratic Bezier interpolations with the clamped
# control point (9 each: 36), I- - S- and its conversion (2), S- (FP64) and chi-
# bilinear (8), dtau (2), exp (5), g (6), D update (3), accumulation (1).
OPS_PER_UPDATE_QUAD_F32 = 9 + 36 + 2 + 8 + 2 + 5 + 6 + 3 + 1
# HBM: 8 TB/s.  The Gauss-Seidel chain kernel does 9 VALU operations per update
# (3 for the new intensity, 5 for the recomputed one, 1 for its weight) against 24
# bytes, so HBM is its roof.  Algorithmic bytes of one FP32 chain update (one vertex,
# one ray crossing an x or y face first, one bin, in a step that computes a plane and
# recomputes the one above): the four coefficients E and Q of the new and the
# recomputed intensity read (16), the new intensity and the weighted recomputed one
# written (8).
HBM_PEAK_GBS = 8000.0
BYTES_PER_CHAIN_UPDATE_F32 = 16 + 4 + 4
# Algorithmic bytes of the FP32 sweep kernel per cell and bin and formal solution: each
# of the 8 octant passes reads chi (4) and S (4 as FP32) and writes its J partial (4),
# 96 bytes, shared by the rays of the angle set: 1.2 bytes per update at 80 rays.
BYTES_PER_CELL_BIN_SWEEP_F32 = 8 * (4 + 4 + 4)
BYTES_PER_UPDATE_SWEEP_F32_80 = BYTES_PER_CELL_BIN_SWEEP_F32 / 80


TRAFFIC_PROFILE = {"multifreq": os.path.join(ROOT, "profiles", "sweep_stage_f32_multifreq192_traffic.md"),
                   "linear": os.path.join(ROOT, "profiles", "sweep_stage_f32_scattering128_traffic.md"),
                   "bezier": os.path.join(ROOT, "profiles", "sweep_stage_f32_bezier_scattering128_traffic.md"),
                   "quadratic": os.path.join(ROOT, "profiles", "plane_step_f32_quadratic_scattering128_traffic.md"),
                   "gauss-seidel": os.path.join(ROOT, "profiles", "gs_chain_f32_scattering128_traffic.md")}
KERNEL_SOURCE = {"multifreq": os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_kernels.hip"),
                 "linear": os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_kernels.hip"),
                 "bezier": os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_kernels.hip"),
                 "quadratic": os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_plane.hip"),
                 "gauss-seidel": os.path.join(ROOT, "paper_1201_2222_amd", "csrc", "rt_gs.hip")}


# device code every kernel above also compiles in
KERNEL_HEADERS = [os.path.join(ROOT, "paper_1201_2222_amd", "csrc", h) for h in ("rt_device.h", "rt_internal.h")]


def kernel_source_sha256(order):
    """SHA-256 over the kernel's source file and the device headers it includes."""
    import hashlib
    h = hashlib.sha256()
    for path in [KERNEL_SOURCE[order]] + KERNEL_HEADERS:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(order="linear", kernel=None):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (calibrated against a plain copy), or None when the
    kernel source or the device headers have changed since the counters were taken, or
    when the summary is of another kernel than `kernel`."""
    try:
        text = open(TRAFFIC_PROFILE[order]).read()
        fields = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_launch:",
                                                                                   "kernel_source_sha256:",
                                                                                   "kernel:")))
        sha = kernel_source_sha256(order)
    except OSError:
        return None
    if fields.get("kernel_source_sha256", "").strip() != sha:
        return None
    if kernel is not None and fields.get("kernel", "").strip() != kernel:
        return None
    return float(fields["traffic_bytes_per_launch"])


def _traffic_rate(roofline):
    """Measured HBM bytes of one launch over its average duration (GB/s), or None."""
    if roofline["traffic"] is None or roofline["avg_launch_us"] <= 0:
        return None
    return roofline["traffic"] / (roofline["avg_launch_us"] * 1e-6) / 1e9


def _chain_kernel_name(shape):
    """The FP32 Gauss-Seidel chain kernel that computes a plane and recomputes the one
    above, as the library picks it: M vertices per lane for the longer in-plane axis
    (64 M lanes' worth), FULL when both in-plane axes are exactly 64 M."""
    ne = max(shape[0], shape[1])
    m = 1 if ne <= 64 else (2 if ne <= 128 else 4)
    full = shape[0] == 64 * m and shape[1] == 64 * m
    return f"gs_chain_kernel<float, true, {m}, true, true, {'true' if full else 'false'}>"


def _schedule(args, rt):
    return rt.RT_SCHED_PERSISTENT if args.schedule == "persistent" else rt.RT_SCHED_STAGES


def _sweep_kernel_name(args, order, multi=False):
    """The FP32 sweep kernel the library launches (multi: fewer waves than rays per octant,
    each wave sweeping several rays)."""
    if args.schedule == "persistent":
        return "sweep_persistent_kernel<float, true>"
    return f"sweep_stage_kernel<float, true, 1, {'true' if multi else 'false'}, {order}, 8>"


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(wl, sweeps, order=0, interp=0):
    """FP64 oracle (single thread, as it stands) timed on a bounded number of formal
    solutions of the same workload."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    op = oracle.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, order=order,
                        interp=interp)
    S = wl.B.copy()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        op.sweep(S)
    dt = time.perf_counter() - t0
    updates = wl.cells * wl.na * wl.nf * sweeps
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": updates / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "host": {"cpu": model, "threads": os.cpu_count()},
            "sample": f"{sweeps} formal solutions (sweeps) of the {wl.shape[0]}^3 x {wl.na}-ray workload"
                      f"{' (second order)' if order else ''}{' (quadratic upwind intensity)' if interp else ''}, "
                      f"{updates / 1e6:.1f} M updates in {dt:.1f} s, FP64, one thread"}


def _wait_all(rt, srv, tickets, label):
    """Poll the server until every ticket has finished; one progress line per finished
    request (the work itself reports progress)."""
    done, t0 = {}, time.perf_counter()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = rt.rt_server_poll(srv, t)
            if r is not None:
                done[t] = r
                print(f"{label}: {len(done)}/{len(tickets)} done at {time.perf_counter() - t0:.2f} s "
                      f"({r[1]['iterations']} iterations)", file=sys.stderr, flush=True)
        time.sleep(0.001)
    return done


def bench_batched(args, rt, W, torch, np):
    """Many uneven problems solved together: one server, all requests submitted at once."""
    count = args.count
    free, _ = torch.cuda.mem_get_info()
    probs = []
    t_gen = time.perf_counter()
    for k in range(count):
        wl = W.batched_problem(k)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        p = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, w_nu=wl.w_nu,
                       precision=rt.RT_F32, schedule=_schedule(args, rt))
        p.set_fields(dev(wl.chi), dev(wl.eps), dev(wl.B))
        S = torch.empty(wl.chi.size, dtype=torch.float64, device="cuda")
        J = torch.empty_like(S)
        probs.append((p, S, J, wl.cells, wl.na, wl.nf))
        print(f"batched: problem {k} set up ({wl.shape[0]}x{wl.shape[1]}x{wl.shape[2]}, {wl.na} rays, "
              f"{wl.nf} bins, eps {wl.meta['eps']:.1e})", file=sys.stderr, flush=True)
        del wl
    torch.cuda.synchronize()
    print(f"batched: {count} problems set up in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    budget = int(0.8 * free)
    srv = rt.rt_server_create(budget, check_every=16)
    t0 = time.perf_counter()
    tickets = [rt.rt_server_submit(srv, p.handle, S, J, delta_c=1e-6, max_iter=args.max_iter,
                                   fixed_iters=args.fixed_iters) for p, S, J, *_ in probs]
    done = _wait_all(rt, srv, tickets, "batched")
    total = time.perf_counter() - t0
    rt.rt_server_destroy(srv)
    updates, lat, iters, notconv = 0.0, [], [], 0
    for (p, S, J, cells, na, nf), t in zip(probs, tickets):
        status, st = done[t]
        notconv += status != rt.RT_OK
        it_bins, _ = rt.rt_ali_bin_stats(p.handle, nf)
        updates += float(cells) * na * float(np.sum(it_bins))
        lat.append(st["seconds"])
        iters.append(st["iterations"])
    seq = None
    if args.seq_sample > 0:
        # the same kind of problems one at a time, for the batching gain
        k = min(args.seq_sample, count)
        t1 = time.perf_counter()
        seq_updates = 0.0
        for p, S, J, cells, na, nf in probs[:k]:
            p.ali_solve(S, J, delta_c=1e-6, max_iter=args.max_iter)
            it_bins, _ = rt.rt_ali_bin_stats(p.handle, nf)
            seq_updates += float(cells) * na * float(np.sum(it_bins))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        seq = {"problems": k, "seconds": dt, "updates_per_s": seq_updates / dt, "solves_per_s": k / dt}
        print(f"batched: {k} problems one at a time in {dt:.2f} s", file=sys.stderr, flush=True)
    for p, *_ in probs:
        p.close()
    return {
        "metric": METRIC, "value": updates / total, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": total * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded, generated on the host)",
        "config": {"workload": f"batched: {count} uneven problems (axes 24..96, 24/48/80 rays, 1..16 bins, "
                               f"eps 1e-4..1), Jacobi ALI to max|dS/S|<=1e-6 per bin, FP32 sweeps",
                   "problems": count, "schedule": args.schedule},
        "ali_solves_per_s": count / total,
        "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
        "iterations": {"min": int(min(iters)), "median": float(np.median(iters)), "max": int(max(iters))},
        "not_converged": notconv, "one_at_a_time": seq,
    }


def _host_threads():
    """Host cores this process may use (the affinity mask), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        return None


def oracle_rate(wl, units, threads, sweeps=1):
    """The FP64 oracle, as it stands, on independent (bin, ray subset) units of a
    workload: each unit is a one-bin oracle problem over some of the rays (rays and
    bins do not couple within one formal solution), swept ``sweeps`` times.  Units run
    on a thread pool of ``threads`` workers (the C sweep releases the GIL).  Returns
    (updates/s, updates, seconds)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.build(force=False)
    mu, w = oracle.quadrature(wl.n_mu)
    probs = []
    for b, rays in units:
        rays = np.asarray(rays)
        probs.append((oracle.Problem(wl.shape, wl.chi[b], wl.eps[b], wl.B[b], mu=mu[rays], w=w[rays],
                                     bc_lo=wl.bc_lo, bc_hi=wl.bc_hi), wl.B[b], len(rays)))

    def run(u):
        op, S, _ = u
        for _ in range(sweeps):
            op.sweep(S)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, probs))
    dt = time.perf_counter() - t0
    updates = float(sum(wl.cells * nr * sweeps for _, _, nr in probs))
    return updates / dt, updates, dt


def cpu_baseline_multifreq(n, nf_total, sample_bins, rays_per_octant=10, single_octants=2):
    """Oracle baseline on the multi-frequency workload: one thread over one bin and
    ``single_octants`` octants of its rays, and every host thread (at most 16) over
    (bin, octant) units of ``sample_bins``; one sweep each, extrapolated to the full
    workload through updates/s (sweeps cost the same per update in every bin)."""
    from paper_1201_2222_amd import workloads as W
    wl = W.multifreq(n=n, nf=nf_total, bins=sample_bins)
    oct_rays = lambda o: list(range(o * rays_per_octant, (o + 1) * rays_per_octant))
    r1, u1, t1 = oracle_rate(wl, [(0, sum((oct_rays(o) for o in range(single_octants)), []))], 1)
    threads = _host_threads()
    units = [(b, oct_rays(o)) for b in range(len(sample_bins)) for o in range(8)][:max(threads, 1) * 1]
    rN, uN, tN = oracle_rate(wl, units, threads)
    return {"value": rN, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "host": {"cpu": _cpu_model(), "threads_visible": os.cpu_count()},
            "sample": f"{len(units)} (bin, octant) units of bins {[int(b) for b in wl.meta['bins']]} of the "
                      f"{n}^3 x {nf_total}-bin x {wl.na}-ray workload, one sweep each on {threads} threads: "
                      f"{uN / 1e6:.0f} M updates in {tN:.1f} s, FP64; extrapolated to the full workload at "
                      f"this rate ({wl.cells * nf_total * wl.na / rN:.0f} s per sweep of all bins)",
            "single_thread": {"value": r1, "unit": "updates/s", "cores": 1,
                              "sample": f"bin {int(wl.meta['bins'][0])}, {single_octants} octants "
                                        f"({single_octants * rays_per_octant} rays), one sweep: "
                                        f"{u1 / 1e6:.0f} M updates in {t1:.1f} s"}}


def bench_multifreq(args, rt, W, torch, np):
    """Multi-frequency workload at full size: 192^3 x 64 bins x 80 rays in one problem
    (about 100 GB of device memory).  A step is one Jacobi ALI iteration over all 64
    bins (one formal solution of every bin plus the update); inputs are resident in
    HBM before the timed region."""
    nf_total = 64
    n = args.mf_n
    bins = np.arange(nf_total) if args.bins >= nf_total else \
        np.linspace(0, nf_total - 1, args.bins).round().astype(int)
    nfb = len(bins)
    cells = n ** 3
    chi = torch.empty(nfb * cells, dtype=torch.float64, device="cuda")
    eps = torch.empty_like(chi)
    B = torch.empty_like(chi)
    t_gen = time.perf_counter()
    w_nu = np.zeros(nfb)
    for c0 in range(0, nfb, 8):
        sel = bins[c0:c0 + 8]
        wl = W.multifreq(n=n, nf=nf_total, bins=sel)
        sl = slice(c0 * cells, (c0 + len(sel)) * cells)
        for dst, src in ((chi, wl.chi), (eps, wl.eps), (B, wl.B)):
            dst[sl].copy_(torch.from_numpy(np.ascontiguousarray(src).reshape(-1)))
        w_nu[c0:c0 + len(sel)] = wl.w_nu
        print(f"multifreq: bins {int(sel[0])}..{int(sel[-1])} generated and copied "
              f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    shape, n_mu, bc_lo, bc_hi = wl.shape, wl.n_mu, wl.bc_lo, wl.bc_hi
    na = n_mu * (n_mu + 2)
    del wl
    prob = rt.Problem(shape, nf=nfb, n_mu=n_mu, bc_lo=bc_lo, bc_hi=bc_hi, w_nu=w_nu, precision=rt.RT_F32,
                      schedule=_schedule(args, rt))
    desc_bytes = rt.rt_problem_bytes(prob.desc)
    prob.set_fields(chi, eps, B)
    torch.cuda.synchronize()
    del chi, eps, B          # the library keeps its own copies
    S = torch.empty(nfb * cells, dtype=torch.float64, device="cuda")
    J = torch.empty_like(S)
    free, total_mem = torch.cuda.mem_get_info()
    print(f"multifreq: {n}^3 x {nfb} bins x {na} rays set up, library state {desc_bytes / 1e9:.1f} GB, "
          f"{(total_mem - free) / 1e9:.1f} GB of device memory in use", file=sys.stderr, flush=True)

    K, Wm = args.steps, args.warmup
    gs = args.ali == "gauss-seidel"
    solve = prob.ali_solve_gs if gs else prob.ali_solve
    if Wm > 0:
        solve(S, J, fixed_iters=Wm, check_every=Wm)
    torch.cuda.synchronize()
    print(f"multifreq: {Wm} warm-up iterations done", file=sys.stderr, flush=True)
    # the library's launch-shape tuner picks the waves per sweep workgroup for this
    # problem (formal solutions timed per wave count; setup, not part of the timed step)
    waves, tune_ms = None, None
    if args.waves > 0:
        prob.set_waves(args.waves)
        waves = args.waves
    elif not args.no_tune and args.schedule == "stages":
        if Wm <= 0:
            solve(S, J, fixed_iters=1, check_every=1)
        waves, tune_ms = prob.tune(S, reps=2)
        torch.cuda.synchronize()
        print(f"multifreq: tuned {waves} waves per workgroup "
              f"({', '.join(f'{w}: {m:.1f}' for w, m in tune_ms.items())} ms per sweep)", file=sys.stderr, flush=True)
    # timed: K Jacobi iterations of all bins (the production path: graph-replayed chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, st = solve(S, J, fixed_iters=K, check_every=K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"multifreq: {K} timed iterations in {dt:.3f} s", file=sys.stderr, flush=True)
    updates = float(cells) * na * nfb * K
    # one more iteration with the sweep kernel's launches timed by events
    rt.rt_problem_profile(prob.handle, True)
    solve(S, J, fixed_iters=1, check_every=1)
    torch.cuda.synchronize()
    prof = rt.rt_problem_profile_read(prob.handle)
    rt.rt_problem_profile(prob.handle, False)
    kernel_s = prof["kernel_ms"] / 1e3
    sweep_rate = prof["updates"] / kernel_s if kernel_s > 0 else 0.0
    achieved = sweep_rate * OPS_PER_UPDATE_F32 / 1e12
    launches = max(prof["launches"], 1)
    # the committed byte counters were taken on the full 192^3 x 64-bin workload
    kname = _sweep_kernel_name(args, 0, multi=waves is not None and waves < na // 8)
    traffic = measured_traffic("multifreq", kname) if (n == 192 and nfb == 64 and args.schedule == "stages" and
                                                     not gs) else None
    avg_us = prof["kernel_ms"] * 1e3 / launches
    hbm_alg = sweep_rate * BYTES_PER_UPDATE_SWEEP_F32_80 / 1e9
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": kname,
                "avg_launch_us": avg_us, "timed_launches": prof["launches"],
                "ops_per_update": OPS_PER_UPDATE_F32, "sweep_updates_per_s": sweep_rate,
                "hbm": {"achieved": hbm_alg, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_alg / HBM_PEAK_GBS,
                        "bytes_per_update": BYTES_PER_UPDATE_SWEEP_F32_80,
                        "measured_gbs": (traffic / (avg_us * 1e-6) / 1e9) if traffic and avg_us > 0 else None,
                        "measured_frac": (traffic / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS)
                        if traffic and avg_us > 0 else None}}
    if gs:
        # the dominant kernel of Gauss-Seidel is the chain kernel of the downward pass
        chain_s = prof["chain_ms"] / 1e3
        ach = prof["chain_updates"] * BYTES_PER_CHAIN_UPDATE_F32 / chain_s / 1e9 if chain_s > 0 else 0.0
        roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS, "traffic": None,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": _chain_kernel_name(shape),
                    "avg_launch_us": prof["chain_ms"] * 1e3 / max(prof["chain_launches"], 1),
                    "timed_launches": prof["chain_launches"],
                    "bytes_per_update": BYTES_PER_CHAIN_UPDATE_F32,
                    "upward_sweep": {"kernel": "sweep_stage_kernel<float, true, 1, "
                                               f"{'true' if waves is not None and waves < na // 8 else 'false'}, 0, 4>",
                                     "avg_launch_us": avg_us, "updates_per_s": sweep_rate}}
    out = {
        "metric": METRIC, "value": updates / dt, "unit": "updates/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded, generated on the host)",
        "config": {"workload": f"multifreq {n}^3 x {nfb} bins x {na} rays (x_nu log-spaced in [0.05, 50], free-free "
                               f"chi_abs ~ x^-3 rho with rho lognormal(0.8), grey scattering tau 10, Planck B_nu "
                               f"with T lognormal(0.3)); a step is one Jacobi ALI iteration over all bins, "
                               f"FP32 sweeps + FP64 updates and residuals"
                               f"{'; Gauss-Seidel ALI (plane-block order)' if gs else ''}",
                   "grid": list(shape), "bins": nfb, "rays": na, "schedule": args.schedule, "ali": args.ali,
                   "waves_per_workgroup": waves, "tuner_ms_per_sweep": tune_ms,
                   "device_bytes_library": desc_bytes},
        "roofline": roofline,
    }
    if args.mf_converge:
        # the whole solve to max |dS/S| <= 1e-6 per bin from S = B, in chunks of 100
        # iterations (each later chunk continues from S; a bin already converged stops
        # after one iteration of the chunk)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it_total = np.zeros(nfb, dtype=np.int64)
        status = rt.RT_NOT_CONVERGED
        while status != rt.RT_OK and it_total.max() < args.max_iter:
            status, st = solve(S, J, delta_c=1e-6, max_iter=100, per_bin_stop=True,
                               warm_start=1 if it_total.max() > 0 else 0)
            it_bins, res = rt.rt_ali_bin_stats(prob.handle, nfb)
            it_total += it_bins
            print(f"multifreq: converging, {int(it_total.max())} iterations, max residual {float(res.max()):.2e} "
                  f"({time.perf_counter() - t1:.1f} s)", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t1
        out["converged_solve"] = {"seconds": tc, "status": int(status), "iterations_max": int(it_total.max()),
                                  "iterations_per_bin": it_total.tolist(),
                                  "updates_per_s": float(cells) * na * float(np.sum(it_total)) / tc}
    prob.close()
    del S, J
    torch.cuda.empty_cache()
    return out


class _ServingRun:
    """One serving run: requests arrive at given times, are created on the device (a
    new problem with its own fields, or the next snapshot of a drifting stream) and
    submitted to the server as long as the summed rt_problem_bytes of the requests in
    flight stays within the budget (oldest first; a stream's snapshot waits for its
    previous one), and their latency runs from arrival to completion."""

    def __init__(self, rt, W, torch, np, srv, budget, streams, max_iter, label, max_n=160):
        self.max_n = max_n
        self.rt, self.W, self.torch, self.np = rt, W, torch, np
        self.srv, self.budget, self.streams, self.max_iter, self.label = srv, budget, streams, max_iter, label
        self.inflight = {}        # ticket -> record
        self.bytes = 0
        self.done = []

    def _make(self, kind, key):
        rt, torch = self.rt, self.torch
        if kind == "stream":
            st = self.streams[key]
            if st["busy"]:
                return None
            if st["problem"] is None:
                req = self.W.serving_request(10_000 + key, n=st["n"], nf=st["nf"])
                p = rt.Problem(req["shape"], nf=req["nf"], n_mu=req["n_mu"], w_nu=req["w_nu"], precision=rt.RT_F32)
                p.set_fields(req["chi"], req["eps"], req["B"])
                st.update(problem=p, req=req, S=torch.empty_like(req["B"]), J=torch.empty_like(req["B"]),
                          bytes=rt.rt_problem_bytes(p.desc) + 2 * req["B"].numel() * 8, step=0, warm=0)
            else:
                st["step"] += 1
                B = self.W.serving_drift(st["req"], st["step"])
                st["problem"].set_fields(st["req"]["chi"], st["req"]["eps"], B)
                st["warm"] = 2     # S = eps B + (1 - eps) J of the previous snapshot, on the device
            st["busy"] = True
            return st["problem"], st["S"], st["J"], st["bytes"], st["warm"], False
        req = self.W.serving_request(key, max_n=self.max_n)
        desc = rt.make_desc(req["shape"], nf=req["nf"], n_mu=req["n_mu"], w_nu=req["w_nu"], precision=rt.RT_F32)
        nbytes = rt.rt_problem_bytes(desc) + 2 * req["B"].numel() * 8    # with the caller's S and J
        if self.inflight and self.bytes + nbytes > self.budget:
            return "full"
        p = rt.Problem(req["shape"], nf=req["nf"], n_mu=req["n_mu"], w_nu=req["w_nu"], precision=rt.RT_F32)
        p.set_fields(req["chi"], req["eps"], req["B"])
        S, J = torch.empty_like(req["B"]), torch.empty_like(req["B"])
        del req
        return p, S, J, nbytes, 0, True

    def run(self, arrivals, kinds, t_admit_end=None, drain=True):
        """arrivals: seconds from the start; kinds: ("fresh", index) or ("stream", s).
        Requests not admitted by t_admit_end (None: never stop) stay unserved."""
        import time
        rt = self.rt
        pending, nxt, t0 = [], 0, time.perf_counter()
        unserved = 0
        while True:
            now = time.perf_counter() - t0
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                pending.append((arrivals[nxt], kinds[nxt]))
                nxt += 1
            admitting = t_admit_end is None or now <= t_admit_end
            i = 0
            while admitting and i < len(pending):
                arr, (kind, key) = pending[i]
                if kind == "stream" and self.streams[key]["problem"] is not None and \
                        self.streams[key]["bytes"] + self.bytes > self.budget and self.inflight:
                    break
                made = self._make(kind, key)
                if made == "full":
                    break                      # oldest fresh request first
                if made is None:
                    i += 1                     # its stream is busy: later requests may go
                    continue
                p, S, J, nbytes, warm, fresh = made
                t = rt.rt_server_submit(self.srv, p.handle, S, J, delta_c=1e-6, max_iter=self.max_iter,
                                        warm_start=warm)
                self.inflight[t] = {"arr": arr, "p": p, "S": S, "J": J, "bytes": nbytes, "fresh": fresh,
                                    "kind": kind, "key": key, "cells": p.cells, "nf": p.nf,
                                    "t_submit": time.perf_counter() - t0}
                self.bytes += nbytes
                pending.pop(i)
                break          # one request per round, so completions are polled in between
            for t in list(self.inflight):
                r = rt.rt_server_poll(self.srv, t)
                if r is None:
                    continue
                rec = self.inflight.pop(t)
                now = time.perf_counter() - t0
                rt.rt_server_release(self.srv, t)
                it_bins, _ = rt.rt_ali_bin_stats(rec["p"].handle, rec["nf"])
                self.bytes -= rec["bytes"]
                if rec["fresh"]:
                    rec["p"].close()
                else:
                    self.streams[rec["key"]]["busy"] = False
                # arrival to submission (waiting, then the request's fields and problem
                # made on the device) plus the server's submission-to-completion time
                lat = rec["t_submit"] - rec["arr"] + r[1]["seconds"]
                self.done.append({"latency": lat, "iterations": r[1]["iterations"], "status": r[0],
                                  "kind": rec["kind"], "updates": float(rec["cells"]) * 48 * float(self.np.sum(it_bins)),
                                  "t_done": now})
                print(f"{self.label}: {len(self.done)} done ({rec['kind']}), latency {self.done[-1]['latency']:.2f} s, "
                      f"{r[1]['iterations']} iterations, {len(self.inflight)} in flight, {len(pending)} waiting",
                      file=sys.stderr, flush=True)
            if nxt >= len(arrivals) and not self.inflight and (not pending or not admitting):
                unserved = len(pending)
                break
            if not admitting and not self.inflight:
                unserved = len(pending) + (len(arrivals) - nxt)
                break
            time.sleep(0.0005)
        span = time.perf_counter() - t0
        return span, unserved


def bench_serving(args, rt, W, torch, np):
    """Serving loop at the workload's stated size: every request a new problem (cubic N
    log-uniform in 32..160, 8..32 bins, 48 rays, eps 10^U[-4,0]) generated on the device,
    30% of them successive snapshots of 16 drifting streams warm-started from their
    device-resident S and J; admission by HBM footprint.  First the capacity (a
    saturated window), then Poisson arrivals at 0.25, 0.5 and 0.9 of it and at 200
    requests/s over 30 s windows; latency from arrival to completion, queueing
    included.  At 200 requests/s the GPU is overloaded: requests still waiting when the
    window closes are reported as unserved (their latency exceeds the window)."""
    rng = np.random.default_rng(2005)
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    # the library's state and the callers' S and J of the admitted requests; the rest
    # of the memory is left to request generation
    budget = int(0.6 * free)
    srv = rt.rt_server_create(budget, check_every=16)
    runs = []
    srng = np.random.default_rng(3005)
    streams = [{"n": int(round(np.exp(srng.uniform(np.log(32), np.log(args.serve_max_n))))),
                "nf": int(srng.integers(8, 33)),
                "problem": None, "busy": False} for _ in range(args.streams)]
    try:
        counter = [0]

        def kinds_for(m):
            out = []
            for _ in range(m):
                if rng.random() < 0.3:
                    out.append(("stream", int(rng.integers(len(streams)))))
                else:
                    out.append(("fresh", counter[0]))
                    counter[0] += 1
            return out

        def summary(run, span, unserved, rate, window):
            lat = [d["latency"] for d in run.done]
            served = len(run.done)
            warm = [d["iterations"] for d in run.done if d["kind"] == "stream"]
            cold = [d["iterations"] for d in run.done if d["kind"] == "fresh"]
            out = {"rate_per_s": rate, "window_s": window, "arrived": served + unserved, "served": served,
                   "unserved": unserved, "solves_per_s": served / span if span > 0 else 0.0,
                   "updates_per_s": sum(d["updates"] for d in run.done) / span if span > 0 else 0.0,
                   "latency_ms": {"p50": _pct(lat, 50) * 1e3 if lat else None, "p99": _pct(lat, 99) * 1e3 if lat else None},
                   "iterations_cold_median": float(np.median(cold)) if cold else None,
                   "iterations_warm_median": float(np.median(warm)) if warm else None,
                   "not_converged": sum(d["status"] != rt.RT_OK for d in run.done)}
            if unserved:
                out["latency_note"] = (f"{unserved} requests were still waiting when the window closed; their latency "
                                       f"exceeds {window:.0f} s and is not in the percentiles")
            return out

        # capacity: a saturated window (requests always waiting)
        cap_window = args.serve_window / 2
        n_cap = 400
        cap_run = _ServingRun(rt, W, torch, np, srv, budget, streams, args.max_iter, "serving capacity", args.serve_max_n)
        runs.append(cap_run)
        span, _ = cap_run.run(np.zeros(n_cap), kinds_for(n_cap), t_admit_end=cap_window)
        capacity = len(cap_run.done) / span
        print(f"serving: capacity {capacity:.2f} solves/s ({len(cap_run.done)} in {span:.1f} s)", file=sys.stderr,
              flush=True)
        results = []
        for frac in (0.25, 0.5, 0.9):
            rate = frac * capacity
            arr = np.cumsum(rng.exponential(1.0 / rate, int(rate * args.serve_window * 2) + 8))
            arr = arr[arr < args.serve_window]
            run = _ServingRun(rt, W, torch, np, srv, budget, streams, args.max_iter, f"serving {frac:.2f}x", args.serve_max_n)
            runs.append(run)
            span, unserved = run.run(arr, kinds_for(len(arr)))
            results.append(summary(run, span, unserved, rate, args.serve_window))
        rate = 200.0
        arr = np.cumsum(rng.exponential(1.0 / rate, int(rate * args.serve_window * 1.2) + 8))
        arr = arr[arr < args.serve_window]
        run = _ServingRun(rt, W, torch, np, srv, budget, streams, args.max_iter, "serving 200/s", args.serve_max_n)
        runs.append(run)
        span, unserved = run.run(arr, kinds_for(len(arr)), t_admit_end=args.serve_window)
        over = summary(run, span, unserved, rate, args.serve_window)
    finally:
        # every request finishes before any of its problems is freed, also when a run
        # above raised
        rt.rt_server_destroy(srv)
        for r in runs:
            for rec in r.inflight.values():
                if rec["fresh"]:
                    rec["p"].close()
        for st in streams:
            if st.get("problem") is not None:
                st["problem"].close()
    return {
        "metric": METRIC, "value": over["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": over["served"], "warmup": 0,
        "ms_per_step": 1e3 / over["solves_per_s"] if over["solves_per_s"] > 0 else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded; every request's fields generated on the device)",
        "config": {"workload": f"serving: Poisson arrivals at 200 requests/s over {args.serve_window:.0f} s, each a "
                               f"new problem (N log-uniform 32..{args.serve_max_n} cubed, 8..32 bins, 48 rays, eps 10^U[-4,0]); 30% "
                               f"successive snapshots of {args.streams} drifting streams (T x (1 + 0.02 h) per step) "
                               "warm-started from device-resident S and J; HBM-bounded admission; Jacobi ALI to "
                               "1e-6 per bin, FP32 sweeps", "hbm_budget_bytes": budget},
        "capacity_solves_per_s": capacity, "latency_vs_rate": results, "overload_200_per_s": over,
    }


def bench_scattering(args, rt, W, torch, np, steps, warmup, cpu=True):
    """The 128^3 scattering workload: ALI solves from S = B to max |dS/S| <= 1e-6 plus the
    moments epilogue, timed per solve (the FP32 production path, graph-replayed chunks),
    the sweep kernel against its roofline, and the plain FP64 GPU solve."""
    wl = W.scattering(args.n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    chi, eps, B = dev(wl.chi), dev(wl.eps), dev(wl.B)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    cells = wl.cells
    mom = {k: torch.empty(m * cells, dtype=torch.float64, device="cuda")
           for k, m in (("J_int", 1), ("H_int", 3), ("K_int", 6), ("f_int", 6), ("Q_int", 1))}
    sched = _schedule(args, rt)
    order = rt.RT_SC_BEZIER if args.order == "bezier" else rt.RT_SC_LINEAR
    quad = args.interp == "quadratic"
    if quad and order:
        raise SystemExit("--interp quadratic is built with first-order segments only")
    interp = rt.RT_INTERP_QUADRATIC if quad else rt.RT_INTERP_BILINEAR
    gs = args.ali == "gauss-seidel"
    if gs and (quad or order):
        raise SystemExit("--ali gauss-seidel is built with first-order segments and bilinear I- only")
    kind = "quadratic" if quad else args.order
    ops_per_update = OPS_PER_UPDATE_QUAD_F32 if quad else (OPS_PER_UPDATE_BEZ_F32 if order else OPS_PER_UPDATE_F32)
    prob = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32,
                      schedule=sched, order=order, interp=interp)

    def step():
        prob.reset_periodic()
        prob.set_fields(chi, eps, B)
        solve = prob.ali_solve_gs if gs else prob.ali_solve
        status, st = solve(S, J, delta_c=wl.delta_c, max_iter=50000, per_bin_stop=True,
                           fixed_iters=args.fixed_iters)
        if status != rt.RT_OK:
            raise RuntimeError(f"ALI did not converge: {st}")
        # moments epilogue on the converged S
        st["heating"] = prob.moments(S, want_heating=True, **mom)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed steps: the production path (ALI chunks replayed as HIP graphs)
    lat, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        st = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        iters.append(st["iterations"])
        print(f"step: {lat[-1] * 1e3:.1f} ms, {st['iterations']} iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    J32 = J.cpu().numpy()
    # one more solve with the sweep timed by events (issued from the host, the same
    # launches) for the kernel's average launch duration
    rt.rt_problem_profile(prob.handle, True)
    step()
    torch.cuda.synchronize()
    prof = rt.rt_problem_profile_read(prob.handle)
    rt.rt_problem_profile(prob.handle, False)
    print(f"profiled step: {prof['launches']} timed sweep launches, {prof['chain_launches']} timed chain launches",
          file=sys.stderr, flush=True)

    # one sweep per ALI iteration plus the moments sweep
    updates = float(wl.cells * wl.na * wl.nf * (sum(iters) + len(iters)))
    profiled_size = args.n == 128   # the committed byte counters were taken on the 128^3 workload
    value = updates / total
    kernel_s = prof["kernel_ms"] / 1e3
    achieved = prof["updates"] * ops_per_update / kernel_s / 1e12 if kernel_s > 0 else 0.0
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(kind) if profiled_size and args.schedule == "stages" else None,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "plane_step_kernel<float, true, 1>" if quad else _sweep_kernel_name(args, order),
                "avg_launch_us": prof["kernel_ms"] * 1e3 / max(prof["launches"], 1),
                "timed_launches": prof["launches"],
                "ops_per_update": ops_per_update}
    roofline["traffic_gbs"] = _traffic_rate(roofline)
    if gs:
        # the dominant kernel of Gauss-Seidel is the chain kernel of the downward pass
        chain_s = prof["chain_ms"] / 1e3
        achieved = prof["chain_updates"] * BYTES_PER_CHAIN_UPDATE_F32 / chain_s / 1e9 if chain_s > 0 else 0.0
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic("gauss-seidel") if profiled_size else None,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": _chain_kernel_name(wl.shape),
                    "avg_launch_us": prof["chain_ms"] * 1e3 / max(prof["chain_launches"], 1),
                    "timed_launches": prof["chain_launches"],
                    "algorithmic_bytes_per_launch": prof["chain_updates"] * BYTES_PER_CHAIN_UPDATE_F32
                    / max(prof["chain_launches"], 1),
                    "bytes_per_update": BYTES_PER_CHAIN_UPDATE_F32}
        roofline["traffic_gbs"] = _traffic_rate(roofline)

    extra = {}
    if not args.no_f64:
        p64 = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F64,
                         schedule=sched, order=order, interp=interp)
        p64.set_fields(chi, eps, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, st64 = (p64.ali_solve_gs if gs else p64.ali_solve)(S, J, delta_c=wl.delta_c, max_iter=50000,
                                                                   per_bin_stop=True)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        J64 = J.cpu().numpy()
        extra["f64_gpu_solve"] = {"seconds": t64, "iterations": st64["iterations"],
                                  "solves_per_s": 1.0 / t64,
                                  "updates_per_s": wl.cells * wl.na * wl.nf * st64["iterations"] / t64,
                                  "f32_vs_f64_max_rel_J": float(np.max(np.abs(J32 - J64) / np.abs(J64)))}
        p64.close()

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": total / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded, generated on the host)",
        "config": {"workload": f"scattering {wl.shape[0]}^3, 1 bin, {wl.na} rays, eps=1e-3, "
                               f"vertical tau 1e4, {'Gauss-Seidel' if gs else 'Jacobi'} ALI from S=B to max|dS/S|<=1e-6, "
                               f"FP32 sweeps + FP64 updates"
                               f"{', second-order (Bezier) segments' if order else ''}"
                               f"{', monotone quadratic upwind intensity (plane order)' if quad else ''}",
                   "grid": list(wl.shape), "rays": wl.na, "order": args.order, "interp": args.interp,
                   "ali": args.ali,
                   "schedule": args.schedule,
                   "bins": wl.nf},
        "ali_solves_per_s": steps / total,
        "latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
        "iterations": iters,
        "heating": st["heating"],
        "profiling_fixed_iters": args.fixed_iters or None,
        "roofline": roofline,
    }
    out.update(extra)
    if cpu and args.cpu_sweeps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sweeps, order, 1 if quad else 0)
    prob.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (multifreq: ALI iterations over all bins)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="grid edge of the scattering workload")
    ap.add_argument("--cpu-sweeps", type=int, default=2, help="oracle sweeps for the CPU baseline (0 = skip)")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 GPU comparison solve")
    ap.add_argument("--schedule", choices=["stages", "persistent"], default="stages",
                    help="tile wavefront: one launch per hyperplane, or one persistent launch per sweep")
    ap.add_argument("--order", choices=["linear", "bezier"], default="linear",
                    help="scattering: first-order or second-order (Bezier) short characteristics")
    ap.add_argument("--interp", choices=["bilinear", "quadratic"], default="bilinear",
                    help="scattering: upwind intensity bilinear (tile wavefront) or monotone quadratic "
                         "(plane-ordered sweep)")
    ap.add_argument("--ali", choices=["jacobi", "gauss-seidel"], default="jacobi",
                    help="scattering: Jacobi ALI, or Gauss-Seidel with horizontal planes as the blocks")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="profiling mode: run exactly this many ALI iterations per step instead of converging")
    ap.add_argument("--streams", type=int, default=16, help="serving: drifting snapshot streams")
    ap.add_argument("--serve-window", type=float, default=30.0, help="serving: arrival window per rate (s)")
    ap.add_argument("--serve-max-n", type=int, default=160, help="serving: largest grid edge of a request")
    ap.add_argument("--workload", choices=["multifreq", "scattering", "batched", "serving"], default="multifreq",
                    help="multifreq: 192^3 x 64 bins x 80 rays, a step is one Jacobi iteration over all bins "
                         "(default; the 128^3 scattering solves are reported beside it); scattering: the 128^3 "
                         "single-bin solve; batched: many uneven problems; serving: the request loop")
    ap.add_argument("--bins", type=int, default=64, help="multifreq: bins of the 64 to run")
    ap.add_argument("--mf-n", type=int, default=192, help="multifreq: grid edge")
    ap.add_argument("--mf-converge", action="store_true", help="multifreq: also one whole solve to 1e-6 per bin")
    ap.add_argument("--no-tune", action="store_true", help="multifreq: keep the default waves per workgroup")
    ap.add_argument("--waves", type=int, default=0, help="multifreq: waves per sweep workgroup instead of the tuner's")
    ap.add_argument("--scattering-steps", type=int, default=3,
                    help="multifreq: converged 128^3 scattering solves reported beside the line (0 = skip)")
    ap.add_argument("--count", type=int, default=96, help="problems of the batched workload")
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--seq-sample", type=int, default=0,
                    help="batched workload: also solve this many of its problems one at a time")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (for scaling rocprofv3 FETCH/WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (bins and independent "
              "problems would shard across GPUs with no communication but a few reduced scalars)",
              file=sys.stderr)
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
    if args.workload == "batched":
        print(json.dumps(bench_batched(args, rt, W, torch, np)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(bench_serving(args, rt, W, torch, np)), flush=True)
        return
    if args.workload == "scattering":
        print(json.dumps(bench_scattering(args, rt, W, torch, np, args.steps, args.warmup)), flush=True)
        return
    out = bench_multifreq(args, rt, W, torch, np)
    if args.scattering_steps > 0:
        sc = bench_scattering(args, rt, W, torch, np, args.scattering_steps, 1, cpu=False)
        out["scattering_128"] = {k: sc[k] for k in ("config", "ali_solves_per_s", "latency_ms", "iterations",
                                                   "value", "unit", "ms_per_step", "steps")}
        out["scattering_128"]["roofline"] = {k: sc["roofline"][k] for k in ("bound", "achieved", "peak", "unit",
                                                                           "frac", "avg_launch_us")}
        if "f64_gpu_solve" in sc:
            out["scattering_128"]["f64_gpu_solve"] = sc["f64_gpu_solve"]
    if args.cpu_sweeps > 0:
        out["cpu_baseline"] = cpu_baseline_multifreq(args.mf_n, 64, [16, 48])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
