#!/usr/bin/env python
"""Benchmark: per-projection reconstruction solves on one MI355X.

Workload (paper-scale configuration): a 256x256x100 reference volume at
1.875x1.875x2.5 mm (seeded ellipsoid-thorax phantom), a K = 3 PCA motion model
trained on 10 analytic breathing phases, and 360 cone-beam projections (one
per degree, 11 projections/s, 4 s breathing period, 1.5x training amplitude)
on a 512x384 detector at 0.776 mm (SAD 1000 mm, SDD 1500 mm), ray step
0.9375 mm.  Each projection is solved warm-started from the previous w, up to
50 iterations, then the tumour is localised.  The measured projections are
synthetic (the truth-warped phantom projected by the library) and resident
in HBM before timing starts.

One step = one per-projection solve: DVF composition, warp, projection,
cost and gradient, Armijo trials, closed-form (a, b), iteration control and
tumour localisation.  `value` is solves/s over the timed steps.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "p50/p99 per-projection solve latency; solves/s served; ray-samples/s vs HBM peak"
# MI355X published peaks: HBM3E bandwidth, and dense FP32 vector throughput
# (an FMA counts as two flops)
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
CUS, CLOCK_HZ = 256, 2.4e9


def march_flops_per_sample(channels):
    """Algorithmic flops of one trilinear ray sample over `channels` channels:
    the sample position (3 FMAs = 6), floor and fraction (6), the weight
    complements (3), the 8 corner weights (12 multiplies) and one FMA per
    corner and channel (16 per channel)."""
    return 27 + 16 * channels


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------- workload ------
def samples_per_ray(grid, geom):
    """Samples each ray marches (global grid t = n step clipped to the
    interpolant's support), FP64 numpy; [nv][nu]."""
    st, ct = math.sin(geom.angle), math.cos(geom.angle)
    iso = np.asarray(geom.iso, float)
    s = iso + np.array([geom.sad * st, -geom.sad * ct, 0.0])
    c = iso + np.array([-(geom.sdd - geom.sad) * st, (geom.sdd - geom.sad) * ct, 0.0])
    eu, ev = np.array([ct, st, 0.0]), np.array([0.0, 0.0, 1.0])
    u = (np.arange(geom.nu) - 0.5 * (geom.nu - 1)) * geom.du + geom.off_u
    v = (np.arange(geom.nv) - 0.5 * (geom.nv - 1)) * geom.dv + geom.off_v
    pix = c[None, None, :] + u[None, :, None] * eu + v[:, None, None] * ev
    d = pix - s
    L = np.linalg.norm(d, axis=-1)
    d = d / L[..., None]
    lo = np.asarray(grid.origin) - np.asarray(grid.spacing)
    hi = np.asarray(grid.origin) + np.asarray(grid.n) * np.asarray(grid.spacing)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - s) / d
        t2 = (hi - s) / d
    tmin = np.maximum(0.0, np.nanmax(np.minimum(t1, t2), axis=-1))
    tmax = np.minimum(L, np.nanmin(np.maximum(t1, t2), axis=-1))
    n = np.floor(tmax / geom.step) - np.ceil(tmin / geom.step) + 1
    return np.where(tmax >= tmin, np.maximum(n, 0), 0)


def true_tumour(grid, phi, R, scale, p_ref):
    """Position p with p + x(p) = p_ref for the analytic test motion
    (continuous field, evaluated in closed form): the synthetic ground truth."""
    from paper_1004_0014_amd import synth as S
    L = grid.fov
    amps = (1.0, 0.3, 0.15, 0.1, 0.08)
    c = S.phase_coeffs(phi, R) * scale

    def x_at(p):
        g = math.exp(-(p[0] / (0.35 * L[0])) ** 2)
        hz, sx = p[2] / L[2], p[0] / L[0]
        comps = [(2, 1.0), (1, 1.0), (2, hz), (1, hz), (0, sx)]
        out = np.zeros(3)
        for i in range(R):
            ax, f = comps[i]
            out[ax] += 10.0 * amps[i] * g * f * c[i]
        return out

    p = np.array(p_ref, dtype=float)
    for _ in range(200):                  # contraction: |dx/dp| << 1 for this motion
        p_new = p_ref - x_at(p)
        if np.linalg.norm(p_new - p) < 1e-12:
            return p_new
        p = p_new
    return p


class Workload:
    def __init__(self, name, dev):
        import torch
        from paper_1004_0014_amd import synth as S, _lib
        self.name = name
        self.cfg = S.config(name)
        self.grid = S.grid_for(name)
        self.K = self.cfg["K"]
        t0 = time.time()
        self.f0_64 = S.phantom(self.grid)
        self.model = S.pca_model(self.grid, self.K)
        self.f0 = torch.tensor(self.f0_64, dtype=torch.float32, device=dev)
        self.mean = torch.tensor(self.model.mean, dtype=torch.float32, device=dev)
        self.U = torch.tensor(self.model.U, dtype=torch.float32, device=dev)
        self.dmodel = _lib.DeviceModel(self.mean, self.U)
        self.p_ref = S.tumor_center(self.grid)
        log("[bench] inputs for %s built in %.1fs" % (name, time.time() - t0))

    def frame(self, i):
        """Angle, time, breathing phase and truth w of projection i."""
        from paper_1004_0014_amd import synth as S
        angle = math.radians(i % 360)
        t = i / self.cfg["rate_hz"]
        phi = S.breathing_phase(t)
        return angle, t, phi, S.truth_w(self.model, phi)

    def measurements(self, idxs, fixed_angle=None):
        """Synthetic measured projections (truth-warped phantom, projected by
        the library in FP32), kept on the device.  With `fixed_angle` (rad)
        every frame is taken at that gantry angle (fluoroscopy)."""
        import torch
        from paper_1004_0014_amd import synth as S, _lib
        ys, geoms = [], []
        for i in idxs:
            angle, _, _, w = self.frame(i)
            G = S.geom_for(self.name, angle if fixed_angle is None else fixed_angle)
            dvf = _lib.dvf_compose(self.grid, self.dmodel, w)
            f = _lib.warp_volume(self.grid, self.f0, dvf)
            ys.append(_lib.forward_project(self.grid, G, f))
            geoms.append(G)
        torch.cuda.synchronize()
        return ys, geoms


def storage_model(W, storage, dev):
    """The motion model and reference image in 16-bit storage (FP16 fields are
    stored divided by their max |.| so that small entries stay normal)."""
    import torch
    from paper_1004_0014_amd import _lib
    dt = {"bf16": torch.bfloat16, "f16": torch.float16}[storage]
    if storage == "f16":
        scale = np.abs(W.model.U.reshape(W.K, -1)).max(axis=1)
        U = torch.tensor(W.model.U / scale[:, None, None, None, None], dtype=dt, device=dev)
    else:
        scale = None
        U = torch.tensor(W.model.U, dtype=dt, device=dev)
    mean = torch.tensor(W.model.mean, dtype=dt, device=dev)
    f0 = torch.tensor(W.f0_64, dtype=dt, device=dev)
    return _lib.DeviceModel(mean, U, scale=scale), f0


def carried_step0(step0, move):
    """First-trial distance of a solve under the carried-move rule: the
    distance the previous solve of the sequence moved w (from its start to its
    result), kept within [1e-3, 1] x the model's step0."""
    if move is None:
        return step0
    return min(max(move, 1e-3 * step0), step0)


def run_sequence(ctx, W, ys, geoms, idxs, opts, w0, profile=False, predict_order=0, hist=None,
                 chain_mu=False, carry_move=False, move=None, profile_kinds=None):
    """Solves the projections in order, each warm-started from the previous
    result, or with predict_order > 0 from the polynomial extrapolation of
    the last results to the frame's time (the prediction is inside the timed
    solve).  `hist` is a list of (t, w) carried across calls.  With chain_mu
    each solve's first trial uses the step size the previous solve ended with;
    with carry_move its first trial moves w by the distance the previous solve
    moved (`move`: that distance before the first solve here, or None)."""
    import torch
    from paper_1004_0014_amd import _lib
    if chain_mu and hist is None:
        opts.mu0 = 0.0        # a fresh sequence: the first solve's first trial from step0
    lat, iters, trials, werr, terr, evals, samples, ends, ws = [], [], [], [], [], [], [], [], []
    w = list(w0)
    hist = [] if hist is None else hist
    # each frame's time stamp arrives with the frame; the truth used to score
    # the results is looked up after the timed loop
    times = [W.frame(i)[1] for i in idxs]
    torch.cuda.synchronize()
    if profile:
        _lib.profile_enable(True, profile_kinds)
    t_start = time.perf_counter()
    for n, (y, G, i, t_i) in enumerate(zip(ys, geoms, idxs, times)):
        t0 = time.perf_counter()
        if predict_order > 0 and len(hist) >= 2:
            last = hist[-(predict_order + 1):]
            w = _lib.predict_w([h[1] for h in last], [h[0] for h in last], t_i, predict_order)
        if carry_move:
            opts.step0 = carried_step0(W.model.step0, move)
        w_start = list(w)
        w, ab, st = ctx.reconstruct(y, G, w, opts)
        lat.append(time.perf_counter() - t0)
        move = float(np.linalg.norm(np.array(w) - np.array(w_start)))
        if chain_mu:
            opts.mu0 = st["mu"]
        hist.append((t_i, list(w)))
        ws.append(list(w))
        if (n + 1) % 60 == 0:
            log("[bench]   %d solves, last %.2f ms, %d iterations" % (n + 1, 1e3 * lat[-1],
                                                                     st["iterations"]))
        iters.append(st["iterations"])
        trials.append(st["trials"])
        evals.append(st["trials"] + 1)
        samples.append(st["samples"])
        # how the solve ended: tolerance met, iteration cap, line search exhausted
        ends.append("tol" if st["status"] == 0 else
                    ("cap" if st["iterations"] >= opts.max_iter else "armijo"))
        terr.append(st["tumor_mm"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    for wi, i in zip(ws, idxs):
        wt = W.frame(i)[3]
        werr.append(float(np.linalg.norm(np.array(wi) - wt) / np.linalg.norm(wt)))
    prof = _lib.profile_read() if profile else None
    if profile:
        _lib.profile_enable(False)
    return dict(lat=np.array(lat), iters=np.array(iters), trials=np.array(trials),
                evals=np.array(evals), samples=np.array(samples), ends=ends, werr=np.array(werr),
                tumor=np.array(terr), w=w, ws=np.array(ws), move=move,
                elapsed=elapsed, prof=prof, hist=hist)


def summarise(res, W, idxs, samples_per_proj):
    lat = res["lat"] * 1e3
    tumour_err = []
    for i, p in zip(idxs, res["tumor"]):
        _, _, phi, _ = W.frame(i)
        tumour_err.append(float(np.linalg.norm(p - true_tumour(W.grid, phi, W.K, 1.5, W.p_ref))))
    # samples of the definition (every ray over the whole support box) and
    # samples actually marched (rays clipped to where the image can be nonzero)
    samples = float(np.sum(res["evals"] * samples_per_proj))
    marched = float(np.sum(res["samples"]))
    return {
        "solves_per_s": len(lat) / res["elapsed"],
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "mean_iterations": float(res["iters"].mean()),
        "mean_trials": float(res["trials"].mean()),
        "ray_samples_per_s": marched / res["elapsed"],
        "ray_samples_per_s_support_box": samples / res["elapsed"],
        "marched_fraction": marched / samples,
        "solve_end": {k: res["ends"].count(k) for k in ("tol", "cap", "armijo")},
        "w_rel_err_vs_truth_median": float(np.median(res["werr"])),
        "w_rel_err_vs_truth_max": float(np.max(res["werr"])),
        "tumour_err_mm_mean": float(np.mean(tumour_err)),
        "tumour_err_mm_max": float(np.max(tumour_err)),
    }


def kernel_table(prof):
    return {k: {"total_ms": v[0], "launches": v[1], "avg_us": 1e3 * v[0] / max(v[1], 1)}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}


def profiled_value(name, key):
    """A figure measured with rocprofv3 counters, from the line `<key>: <n>`
    of profiles/<name>.md (None if absent)."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    try:
        for line in open(path):
            if line.startswith(key + ":"):
                v = line.split(":", 1)[1].strip()
                return None if v in ("", "null", "None") else float(v)
    except OSError:
        pass
    return None


def profiled_traffic(name):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return profiled_value(name, "traffic_bytes_per_launch")


def roofline(W, prof, samples_per_launch, channels, cell_bytes, traffic_profile=None):
    """Roofline of the dominant kernel (largest total time in the timed region)."""
    kt = kernel_table(prof)
    dom = next(iter(kt))
    N = W.grid.N
    nx, ny, nz = W.grid.n
    cells = (nx + 3) * (ny + 3) * (nz + 3)
    K = W.K
    avg_s = kt[dom]["avg_us"] * 1e-6
    if dom == "march":
        flops = samples_per_launch * march_flops_per_sample(channels)
        achieved = flops / avg_s / 1e12
        traffic = profiled_traffic(traffic_profile) if traffic_profile else None
        # what binds it, from the counter profile of the same kernel: VALU
        # issue (wave-instructions per CU and clock, at most one), with the
        # vector L1's tag lookups beside it
        cprof = "march_counters_256x256x100_f32"
        tags = profiled_value(cprof, "l1_tag_lookups_per_cu_clock")
        taps_gbs = samples_per_launch * 8 * cell_bytes / avg_s / 1e9
        return {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                "avg_us": kt[dom]["avg_us"], "samples_per_launch": samples_per_launch,
                "flops_per_sample": march_flops_per_sample(channels),
                "algorithmic_flops_per_launch": flops,
                "binding_resource": {
                    "name": "VALU issue (SQ_ACTIVE_INST_VALU per CU and clock)",
                    "achieved_per_cu_clock": profiled_value(cprof, "valu_issue_fraction"),
                    "peak_per_cu_clock": 1.0, "frac": profiled_value(cprof, "valu_issue_fraction"),
                    "l1_tag_lookups_per_cu_clock": tags,
                    "source": "profiles/%s.md" % cprof},
                "hbm": {"dram_bytes_per_launch": traffic,
                        "GB_per_s": traffic / avg_s / 1e9 if traffic else None,
                        "frac_of_peak": traffic / avg_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                        "l2_hit_rate": profiled_value(cprof, "march_l2_hit_rate"),
                        "source": "profiles/%s.md, profiles/%s.md" % (traffic_profile, cprof)},
                # taps the samples request (8 cells each), served by the
                # caches: not HBM bytes
                "cache_served_tap_GB_per_s": taps_gbs,
                # the same command's kernel trace (march + final sum per launch)
                "rocprof_avg_us": profiled_value("march_bench_main_256x256x100_f32",
                                                 "rocprof_march_plus_final_sum_us"),
                "compulsory_hbm_bytes_per_launch": cells * cell_bytes + 4 * W.cfg["nu"] * W.cfg["nv"]}
    if dom == "warp_fused":
        # reads mean (3) and U (3K) fields and f0 once, writes the cells
        byts = N * (4 * 3 + 4 * 3 * K + 4 + cell_bytes)
        achieved = byts / avg_s / 1e9
        return {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_us": kt[dom]["avg_us"], "algorithmic_bytes_per_launch": byts}
    return {"kernel": dom, "avg_us": kt[dom]["avg_us"]}


# --------------------------------------------------------- cpu baseline ----
def host_cpu():
    """CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def cpu_baseline(W):
    """The FP64 oracle on this host, on a bounded sample of the workload:
    projections 0, 45 and 90 of the paper-scale rotation, each warm-started
    from the previous frame's true w and solved to the stopping rule, with
    all the oracle's threads (the `value`: solves/s); one iteration of
    projection 45 on one thread; and the tiny configuration's full 30-
    iteration solve from w = 0 on all threads and on one.  Inputs are the
    same FP32 values the GPU solves from, widened; measured projections come
    from the oracle (not timed)."""
    import oracle
    from paper_1004_0014_amd import synth as S
    model, cores = host_cpu()
    nth = oracle.num_threads()
    f0 = W.f0.cpu().double().numpy()
    mean = W.mean.cpu().double().numpy()
    U = W.U.cpu().double().numpy()

    def measured(i):
        angle, _, _, wt = W.frame(i)
        G = S.geom_for(W.name, angle)
        y = oracle.project(W.grid, G, oracle.warp(W.grid, f0, oracle.compose(W.grid, mean, U, wt)))
        return G, y, W.frame(i - 1)[3]

    def evals_samples(G, st):
        # the oracle marches every ray over the whole support: one projection
        # per trial and per gradient, one backprojection per gradient
        per = float(samples_per_ray(W.grid, G).sum())
        return per * (st["trials"] + 2 * (st["iterations"] + 1))

    rows, t_all, samp = [], 0.0, 0.0
    for i in (0, 45, 90):
        G, y, w0 = measured(i)
        opts = oracle.SolveOpts(max_iter=W.cfg["max_iter"], step0=W.model.step0)
        t0 = time.perf_counter()
        _, _, st, _ = oracle.solve(W.grid, G, f0, mean, U, y, w0, opts)
        T = time.perf_counter() - t0
        t_all += T
        samp += evals_samples(G, st)
        rows.append({"projection": i, "seconds": T, "iterations": st["iterations"],
                     "trials": st["trials"], "status": st["status"]})
        log("[bench] cpu baseline: projection %d, %d iterations, %.1f s on %d threads" % (
            i, st["iterations"], T, nth))
    # one thread: a single iteration of projection 45 (a full solve would take minutes)
    G, y, w0 = measured(45)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        _, _, st1, _ = oracle.solve(W.grid, G, f0, mean, U, y, w0,
                                    oracle.SolveOpts(max_iter=1, step0=W.model.step0))
        T1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nth)
    # the tiny configuration (64^3 at 4 mm, K = 3, 128x96 at 1.6 mm, 30 deg):
    # 30 iterations from w = 0, FP64 inputs, at w* of a seeded phase
    g0 = S.grid_for("tiny")
    G0 = S.geom_for("tiny")
    m0 = S.pca_model(g0, 3)
    f00 = S.phantom(g0)
    phi = float(np.random.default_rng(1).uniform(0, 2 * np.pi))
    y0 = oracle.project(g0, G0, oracle.warp(g0, f00, oracle.compose(g0, m0.mean, m0.U, S.truth_w(m0, phi))))
    tiny = {}
    for threads in (nth, 1):
        oracle.set_num_threads(threads)
        try:
            t0 = time.perf_counter()
            _, _, st0, _ = oracle.solve(g0, G0, f00, m0.mean, m0.U, y0, np.zeros(3),
                                        oracle.SolveOpts(max_iter=30, step0=m0.step0, eps_g=0.0))
            tiny["threads_%d" % threads] = {"seconds": time.perf_counter() - t0,
                                            "iterations": st0["iterations"], "trials": st0["trials"]}
        finally:
            oracle.set_num_threads(nth)
    per_it = t_all / max(1, sum(r["iterations"] for r in rows))
    return {"value": len(rows) / t_all, "unit": "solves/s", "cores": nth, "kind": "oracle",
            "sample": ("FP64 oracle solves of paper-scale projections 0, 45 and 90, each warm-started "
                       "from the previous frame's true w and run to the stopping rule (%s iterations, "
                       "%.1f s in all) on %d threads" % (
                           "/".join(str(r["iterations"]) for r in rows), t_all, nth)),
            "cpu_model": model, "host_cores": cores, "seconds_per_solve": t_all / len(rows),
            "seconds_per_iteration": per_it, "oracle_ray_samples_per_s": samp / t_all,
            "solves": rows,
            "one_thread": {"what": "projection 45 capped at one iteration",
                           "iterations": st1["iterations"], "trials": st1["trials"], "seconds": T1,
                           "seconds_per_iteration": T1 / max(1, st1["iterations"])},
            "tiny_30_iterations": tiny}


# ------------------------------------------------------------- serving -----
def serving_measure(dev, n_streams, seconds, slots, budget_gb=200.0):
    """The serving configuration, shortened: n_streams seeded patient streams
    (volumes 128x128x64 .. 512x512x160, K 2..5, detectors 256x192 ..
    1024x768, 11 Hz with 10 ms jitter, gantry at 6 deg/s) over `seconds` of
    arrivals, served by the continuous-batching engine with the streams'
    reference images and models stored BF16, then the same streams and
    arrivals stored FP32 (the plain path), on the same GPU."""
    import torch
    from paper_1004_0014_amd import serve
    t0 = time.time()
    streams = serve.build_streams(n_streams, seconds, 4, dev, storage=torch.float32)
    log("[bench] serving: %d streams built in %.1f s" % (n_streams, time.time() - t0))
    out = {"workload": ("%d streams (seed 4), %.1f s of arrivals at 11 Hz each, volumes 128x128x64.."
                        "512x512x160 over 480x480x320 mm, K 2..5, detectors 256x192..1024x768 "
                        "(397 mm / nu pitch), gantry 6 deg/s, %d slots, stale frames dropped"
                        % (n_streams, seconds, slots))}
    for name, dt, po, carry in (("bf16", torch.bfloat16, 0, False), ("fp32", torch.float32, 0, False),
                                ("bf16_predicted_start", torch.bfloat16, 1, True)):
        ss = [st.as_storage(dt) for st in streams] if dt != torch.float32 else streams
        torch.cuda.synchronize()
        res = serve.run(ss, seconds, slots, budget_gb, predict_order=po, carry_move=carry)
        if po:
            res["warm_start"] = ("linear extrapolation of the stream's last two results; first trial "
                                 "moves w by the distance the stream's previous solve moved it")
        out[name] = res
        log("[bench] serving %s: offered %.0f/s served %.1f/s dropped %d p50 %.1f ms p99 %.1f ms" % (
            name, res["offered_per_s"], res["served_per_s"], res["dropped"], res["p50_ms"] or -1,
            res["p99_ms"] or -1))
        del ss
    del streams
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------- precision -----
def precision_measure(dev, steps, oracle_frame):
    """The precision configuration (256x256x128, K = 4, 512x384 detector) over
    projections 0..steps-1 of its rotation, solved warm-started with the
    reference image and fields stored FP32, BF16 and FP16 (per-field scale);
    w and tumour differences against the FP32-storage path frame by frame and
    against the truth; the projection of the true deformation and one solve
    (frame `oracle_frame`, warm-started from the previous frame's true w)
    against the FP64 oracle on the unrounded inputs."""
    import torch
    import oracle
    from paper_1004_0014_amd import synth as S, _lib
    W = Workload("precision", dev)
    K = W.K
    idxs = list(range(steps))
    ys, geoms = W.measurements(idxs)
    opts = _lib.default_opts(max_iter=W.cfg["max_iter"], step0=W.model.step0, localize=1,
                             p_ref_mm=W.p_ref)
    # the oracle on the unrounded FP64 inputs
    i = oracle_frame
    angle, _, phi, wt = W.frame(i)
    Go = S.geom_for(W.name, angle)
    t0 = time.perf_counter()
    yo = oracle.project(W.grid, Go, oracle.warp(W.grid, W.f0_64,
                                                oracle.compose(W.grid, W.model.mean, W.model.U, wt)))
    wprev = W.frame(i - 1)[3]
    wo, _, sto, _ = oracle.solve(W.grid, Go, W.f0_64, W.model.mean, W.model.U, yo, wprev,
                                 oracle.SolveOpts(max_iter=W.cfg["max_iter"], step0=W.model.step0))
    po, _, _ = oracle.localize(W.grid, W.model.mean, W.model.U, wo, W.p_ref)
    log("[bench] precision: oracle frame %d solved in %.1f s (%d iterations)" % (
        i, time.perf_counter() - t0, sto["iterations"]))
    yo_d = torch.tensor(yo, dtype=torch.float32, device=dev)
    out = {"workload": "precision: %dx%dx%d volume (%s mm), K=%d, projections 0..%d at 1 deg steps, "
                       "%dx%d detector at %.3f mm, warm-started, <= %d iterations" % (
                           *W.grid.n, "x".join("%g" % v for v in W.grid.spacing), K, steps - 1,
                           W.cfg["nu"], W.cfg["nv"], W.cfg["du"], W.cfg["max_iter"]),
           "oracle_frame": {"projection": i, "iterations": sto["iterations"]}}
    spp = np.array([float(samples_per_ray(W.grid, G).sum()) for G in geoms[2:]])
    ref = None
    for storage in ("f32", "bf16", "f16"):
        if storage == "f32":
            dm, f0v = W.dmodel, W.f0
        else:
            dm, f0v = storage_model(W, storage, dev)
        ctx = _lib.Context(W.grid, dm, f0v)
        warm = run_sequence(ctx, W, ys[:2], geoms[:2], idxs[:2], opts, [0.0] * K)
        res = run_sequence(ctx, W, ys[2:], geoms[2:], idxs[2:], opts, warm["w"], hist=warm["hist"])
        # projection of the true deformation against the FP64 oracle
        p = _lib.forward_project(W.grid, Go, _lib.warp_volume(W.grid, f0v, _lib.dvf_compose(W.grid, dm, wt)))
        perr = float(torch.linalg.vector_norm((p.double() - yo_d.double())) /
                     torch.linalg.vector_norm(yo_d.double()))
        # one solve from the oracle's start and measurement
        wg, _, stg = ctx.reconstruct(yo_d, Go, list(wprev), opts)
        ctx.close()
        summ = summarise(res, W, idxs[2:], spp)
        row = {k: summ[k] for k in ("solves_per_s", "p50_ms", "p99_ms", "mean_iterations", "solve_end",
                                    "w_rel_err_vs_truth_median", "w_rel_err_vs_truth_max",
                                    "tumour_err_mm_mean", "tumour_err_mm_max")}
        row["projection_rel_err_vs_oracle"] = perr
        row["w_rel_err_vs_oracle"] = float(np.linalg.norm(np.array(wg) - wo) / np.linalg.norm(wo))
        row["tumour_diff_vs_oracle_mm"] = float(np.linalg.norm(np.array(stg["tumor_mm"]) - po))
        if ref is None:
            ref = res
        else:
            dw = np.linalg.norm(res["ws"] - ref["ws"], axis=1) / np.linalg.norm(ref["ws"], axis=1)
            dt = np.linalg.norm(res["tumor"] - ref["tumor"], axis=1)
            row["w_rel_diff_vs_fp32_median"] = float(np.median(dw))
            row["w_rel_diff_vs_fp32_max"] = float(np.max(dw))
            row["tumour_diff_vs_fp32_mm_mean"] = float(np.mean(dt))
            row["tumour_diff_vs_fp32_mm_max"] = float(np.max(dt))
        out[storage] = row
        log("[bench] precision %s: %.1f solves/s, projection err %.2e, w vs oracle %.2e, tumour vs "
            "oracle %.4f mm" % (storage, row["solves_per_s"], perr, row["w_rel_err_vs_oracle"],
                                 row["tumour_diff_vs_oracle_mm"]))
    return out


# ---------------------------------------------------------------- main -----
def pca_measure(W, dev, reps=5):
    """PCA training of the motion model (section 2.1) at the workload's size:
    the 9 training DVFs of phases 2 pi j / 10 (j = 1..9) as FP32 [9][3][N] on
    the device, K leading components.  Reports the wall time of the training
    call (it returns host values, so it ends synchronised), the HIP-event
    times of its two streaming passes against HBM peak on their algorithmic
    bytes, and the singular values against the exact ones of the model."""
    import torch
    from paper_1004_0014_amd import synth as S, _lib
    g, K, R, J = W.grid, W.K, W.model.R, 9
    d = torch.from_numpy(S.training_dvfs(g, R, n_phases=J + 1)).to(dev)
    torch.cuda.synchronize()
    _lib.pca_train(g, d, K)
    walls = []
    _lib.profile_enable(True)
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, sing, _ = _lib.pca_train(g, d, K)
        walls.append(time.perf_counter() - t0)
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    E = 3 * g.N
    algo = {"pca_gram": J * E * 4, "pca_fields": J * E * 4 + (K + 1) * E * 4}
    kern = {}
    for name, nbytes in algo.items():
        if name in prof:
            us = 1e3 * prof[name][0] / prof[name][1]
            kern[name] = {"avg_us": us, "algorithmic_bytes": nbytes,
                          "GB_per_s": nbytes / us * 1e-3, "frac_hbm": nbytes / us * 1e-3 / 8000.0}
    exact = np.asarray(W.model.sing[:K], float)
    del d
    return {"J": J, "K": K, "reps": reps, "ms_median": 1e3 * float(np.median(walls)),
            "kernels": kern,
            "sing_max_rel_err": float(np.max(np.abs(np.asarray(sing) - exact) / exact))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=360)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="paper")
    ap.add_argument("--grad-mode", default="fused", choices=["fused", "adjoint"])
    ap.add_argument("--variants", default="chain,carry-move,quadratic-step,bf16,f16,f16-image,adjoint,predict,predict-carry,fluoro,fluoro-predict-carry",
                    help="extra timed runs reported beside the main line (comma list; '' = none)")
    ap.add_argument("--variant-steps", type=int, default=0,
                    help="steps of each variant (0: as many as the main run; the adjoint "
                         "variant at most 60)")
    ap.add_argument("--predict-order", type=int, default=2,
                    help="polynomial order of the history predictor in the *predict variants")
    ap.add_argument("--fluoro-angle", type=float, default=30.0,
                    help="gantry angle (deg) of the fixed-angle variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pca", action="store_true", help="skip the PCA-training measurement")
    ap.add_argument("--serve-streams", type=int, default=64,
                    help="streams of the serving measurement (0: skip it)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--precision-steps", type=int, default=40,
                    help="projections of the precision-configuration measurement (0: skip it)")
    ap.add_argument("--precision-oracle-frame", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the per-projection solve is a one-GPU workload "
              "here (see the design notes for how it would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1004_0014_amd import _lib
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = Workload(args.config, dev)
    K, Wm, Ks = W.K, args.warmup, args.steps
    idxs = list(range(Wm + Ks))
    ys, geoms = W.measurements(idxs)
    spp = np.array([float(samples_per_ray(W.grid, G).sum()) for G in geoms])
    mode = _lib.GRAD_FUSED if args.grad_mode == "fused" else _lib.GRAD_ADJOINT
    opts = _lib.default_opts(max_iter=W.cfg["max_iter"], step0=W.model.step0, grad_mode=mode,
                             localize=1, p_ref_mm=W.p_ref)
    ctx = _lib.Context(W.grid, W.dmodel, W.f0)
    # channels of the padded image the march reads: (f, h_1..h_K) padded to 2/4/8
    channels = (2 if K + 1 <= 2 else 4 if K + 1 <= 4 else 8) if mode == _lib.GRAD_FUSED else 1
    # warmup: cold start at w = 0 on the first projection, then warm starts
    warm = run_sequence(ctx, W, ys[:Wm], geoms[:Wm], idxs[:Wm], opts, [0.0] * K)
    # The timed run carries no instrumentation (an event record between two
    # kernels costs ~10 us of GPU time).  A second timed pass over the same
    # projections records HIP events around the dominant kernel (the march)
    # only, on the stream it runs on: its average launch time is the
    # roofline's; a third pass over (at most) the first 60 projections times
    # every kernel.
    res = run_sequence(ctx, W, ys[Wm:], geoms[Wm:], idxs[Wm:], opts, warm["w"], hist=warm["hist"])
    summ = summarise(res, W, idxs[Wm:], spp[Wm:])
    mres = run_sequence(ctx, W, ys[Wm:], geoms[Wm:], idxs[Wm:], opts, warm["w"], profile=True,
                        profile_kinds=("march",))
    nk = min(Ks, 60)
    kres = run_sequence(ctx, W, ys[Wm:Wm + nk], geoms[Wm:Wm + nk], idxs[Wm:Wm + nk], opts,
                        warm["w"], profile=True)
    line = {
        "metric": METRIC, "value": summ["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": Ks, "warmup": Wm, "ms_per_step": 1e3 * res["elapsed"] / Ks,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d volume (%s mm), K=%d, %d projections at 1 deg steps, "
                               "%dx%d detector at %.3f mm, warm-started, <= %d iterations, "
                               "FP32 storage, %s gradient, Armijo line search with secant first "
                               "trials" % (
                                   args.config, *W.grid.n, "x".join("%g" % s for s in W.grid.spacing),
                                   K, Ks, W.cfg["nu"], W.cfg["nv"], W.cfg["du"], W.cfg["max_iter"],
                                   args.grad_mode),
                   "global_batch": 1, "parallelism": "single-gpu"},
        "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"],
        "ray_samples_per_s": summ["ray_samples_per_s"],
        "accuracy": {k: summ[k] for k in ("w_rel_err_vs_truth_median", "w_rel_err_vs_truth_max",
                                          "tumour_err_mm_mean", "tumour_err_mm_max",
                                          "mean_iterations", "mean_trials", "solve_end")},
        "kernels": {"march_events_pass": kernel_table(mres["prof"]),
                    "march_events_pass_solves_per_s": Ks / mres["elapsed"],
                    "all_kernels_first_%d_projections" % nk: kernel_table(kres["prof"])},
        "roofline": roofline(W, mres["prof"],
                             float(np.sum(mres["samples"])) / max(mres["prof"]["march"][1], 1), channels,
                             4 * channels, "march_fused_%dx%dx%d_f32" % tuple(W.grid.n)),
    }
    log("[bench] main: %.1f solves/s p50 %.2f ms p99 %.2f ms" % (summ["solves_per_s"], summ["p50_ms"],
                                                                 summ["p99_ms"]))
    log("[bench] main line: " + json.dumps(line))
    variants = {}
    fl = None
    for v in [s for s in args.variants.split(",") if s]:
        po, carry, chain = 0, False, False
        vsteps = min(Ks, args.variant_steps or (60 if v == "adjoint" else Ks))
        if v in ("bf16", "f16", "bf16-image", "f16-image"):
            dm, f0v = storage_model(W, v.split("-")[0], dev)
            cv = _lib.Context(W.grid, dm, f0v,
                              image_dtype=torch.float16 if v.endswith("image") else torch.float32)
            wv = run_sequence(cv, W, ys[:Wm], geoms[:Wm], idxs[:Wm], opts, [0.0] * K)
            rv = run_sequence(cv, W, ys[Wm:Wm + vsteps], geoms[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], opts, wv["w"], hist=wv["hist"])
            cv.close()
        elif v == "adjoint":
            o2 = _lib.default_opts(max_iter=W.cfg["max_iter"], step0=W.model.step0,
                                   grad_mode=_lib.GRAD_ADJOINT, localize=1, p_ref_mm=W.p_ref)
            wv = run_sequence(ctx, W, ys[:Wm], geoms[:Wm], idxs[:Wm], o2, [0.0] * K)
            rv = run_sequence(ctx, W, ys[Wm:Wm + vsteps], geoms[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], o2, wv["w"], hist=wv["hist"])
        elif v in ("predict", "fluoro", "fluoro-predict", "chain", "quadratic-step",
                   "carry-move", "predict-carry", "fluoro-predict-carry"):
            po = args.predict_order if "predict" in v else 0
            chain = v == "chain"
            carry = v.endswith("carry") or v == "carry-move"
            vo = _lib.default_opts(max_iter=W.cfg["max_iter"], step0=W.model.step0, grad_mode=mode,
                                   localize=1, p_ref_mm=W.p_ref)
            if v == "quadratic-step":
                vo.step_rule = _lib.PCR_STEP_QUADRATIC
            if v.startswith("fluoro"):
                if fl is None:
                    fl = W.measurements(idxs[:Wm + vsteps], fixed_angle=math.radians(args.fluoro_angle))
                vy, vg = fl
            else:
                vy, vg = ys, geoms
            wv = run_sequence(ctx, W, vy[:Wm], vg[:Wm], idxs[:Wm], vo, [0.0] * K,
                              predict_order=po, chain_mu=chain, carry_move=carry)
            rv = run_sequence(ctx, W, vy[Wm:Wm + vsteps], vg[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], vo, wv["w"], predict_order=po, hist=wv["hist"],
                              chain_mu=chain, carry_move=carry, move=wv["move"])
            if v.startswith("fluoro"):
                vspp = np.full(vsteps, float(samples_per_ray(W.grid, vg[Wm]).sum()))
        else:
            continue
        sv = summarise(rv, W, idxs[Wm:Wm + vsteps], vspp if v.startswith("fluoro") else spp[Wm:Wm + vsteps])
        if v.startswith("fluoro"):
            sv["angle_deg"] = args.fluoro_angle
        if po:
            sv["predict_order"] = po
        if chain:
            sv["step_size_carried"] = True
        if carry:
            sv["first_trial"] = "distance the previous solve moved w (carried move)"
        if v == "quadratic-step":
            sv["step_rule"] = "quadratic model"
        sv["steps"] = vsteps
        if rv["prof"]:
            sv["kernels"] = kernel_table(rv["prof"])
        variants[v] = sv
        log("[bench] %s: %.1f solves/s p50 %.2f ms p99 %.2f ms" % (v, sv["solves_per_s"], sv["p50_ms"],
                                                                   sv["p99_ms"]))
    if variants:
        line["variants"] = variants
    ctx.close()
    if not args.no_pca:
        line["pca_train"] = pca_measure(W, dev)
        log("[bench] pca_train: " + json.dumps(line["pca_train"]))
    if args.serve_streams > 0:
        line["serving"] = serving_measure(dev, args.serve_streams, args.serve_seconds, args.serve_slots)
    if args.precision_steps > 2:
        line["precision"] = precision_measure(dev, args.precision_steps, args.precision_oracle_frame)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W)
        log("[bench] cpu baseline %.4g solves/s on %d threads" % (line["cpu_baseline"]["value"],
                                                                  line["cpu_baseline"]["cores"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
