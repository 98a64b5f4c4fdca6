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
HBM_PEAK_GBS = 8000.0
# FP32 VALU issue rate without packed-FP32 instructions (which the library's
# compile flags disable): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions/s
# (78.6 TFLOP/s counting an FMA as two flops).
VALU_ISSUE_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


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


def run_sequence(ctx, W, ys, geoms, idxs, opts, w0, profile=False, predict_order=0, hist=None,
                 chain_mu=False):
    """Solves the projections in order, each warm-started from the previous
    result, or with predict_order > 0 from the polynomial extrapolation of
    the last results to the frame's time (the prediction is inside the timed
    solve).  `hist` is a list of (t, w) carried across calls.  With chain_mu
    each solve's first trial uses the step size the previous solve ended with."""
    import torch
    from paper_1004_0014_amd import _lib
    lat, iters, trials, werr, terr, evals, samples, ends = [], [], [], [], [], [], [], []
    w = list(w0)
    hist = [] if hist is None else hist
    torch.cuda.synchronize()
    if profile:
        _lib.profile_enable(True)
    t_start = time.perf_counter()
    for n, (y, G, i) in enumerate(zip(ys, geoms, idxs)):
        t_i = W.frame(i)[1]
        t0 = time.perf_counter()
        if predict_order > 0 and len(hist) >= 2:
            last = hist[-(predict_order + 1):]
            w = _lib.predict_w([h[1] for h in last], [h[0] for h in last], t_i, predict_order)
        w, ab, st = ctx.reconstruct(y, G, w, opts)
        lat.append(time.perf_counter() - t0)
        if chain_mu:
            opts.mu0 = st["mu"]
        hist.append((t_i, list(w)))
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
        _, _, phi, wt = W.frame(i)
        werr.append(float(np.linalg.norm(np.array(w) - wt) / np.linalg.norm(wt)))
        terr.append(st["tumor_mm"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = _lib.profile_read() if profile else None
    if profile:
        _lib.profile_enable(False)
    return dict(lat=np.array(lat), iters=np.array(iters), trials=np.array(trials),
                evals=np.array(evals), samples=np.array(samples), ends=ends, werr=np.array(werr),
                tumor=np.array(terr), w=w,
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
        # VALU lane-instructions per sample (the loop as compiled): position
        # FMAs, clamp, truncation, fractions and complements, the 8 trilinear
        # weights (12 multiplies), then 8 FMAs per channel -> 25 + 12 C (72
        # for C = 4 in the gfx950 code); an FMA is one issue slot here
        ops = samples_per_launch * (25 + 12 * channels)
        achieved = ops / avg_s / 1e12
        peak = VALU_ISSUE_PEAK_TOPS
        # what binds it, from the counter profile of the same kernel: the
        # vector memory path through the L1 (tag lookups per CU and clock,
        # peak 1; texture addresser busy fraction)
        cprof = "march_counters_256x256x100_f32"
        return {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TOP/s (fp32 VALU lane-instructions)", "frac": achieved / peak,
                "traffic": profiled_traffic(traffic_profile) if traffic_profile else None,
                "avg_us": kt[dom]["avg_us"], "samples_per_launch": samples_per_launch,
                "algorithmic_ops_per_launch": ops,
                "binding_path": "vector L1 (measured, profiles/%s.md)" % cprof,
                "l1_tag_lookups_per_cu_clock": profiled_value(cprof, "l1_tag_lookups_per_cu_clock"),
                "ta_busy_fraction": profiled_value(cprof, "ta_busy_fraction"),
                "l1_requested_bytes_per_sample_without_reuse": 8 * cell_bytes,
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
def cpu_baseline(W, idx, iters_cap, mean_gpu_iters):
    """The FP64 oracle on this host: one warm-started solve of one projection
    of the same workload, capped at `iters_cap` iterations, scaled to the
    GPU's mean iteration count."""
    import oracle
    from paper_1004_0014_amd import synth as S
    f0 = W.f0.cpu().double().numpy()
    mean = W.mean.cpu().double().numpy()
    U = W.U.cpu().double().numpy()
    angle, _, _, wt = W.frame(idx)
    _, _, _, wprev = W.frame(idx - 1)
    G = S.geom_for(W.name, angle)
    y = oracle.project(W.grid, G, oracle.warp(W.grid, f0, oracle.compose(W.grid, mean, U, wt)))
    opts = oracle.SolveOpts(max_iter=iters_cap, step0=W.model.step0)
    t0 = time.perf_counter()
    w, ab, st, _ = oracle.solve(W.grid, G, f0, mean, U, y, wprev, opts)
    T = time.perf_counter() - t0
    done = st["iterations"]
    t_solve = T * (mean_gpu_iters + 1.0) / (done + 1.0)
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": ("FP64 oracle, one solve of projection %d warm-started from the previous "
                       "frame's true w, capped at %d iterations (%d done, %d line-search trials, "
                       "%.1f s wall); scaled by (GPU mean iterations + 1) / (iterations + 1) = "
                       "(%.2f + 1) / (%d + 1)" % (idx, iters_cap, done, st["trials"], T,
                                                  mean_gpu_iters, done)),
            "seconds_measured": T}


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
    ap.add_argument("--variants", default="quadratic-step,bf16,f16,f16-image,bf16-image,adjoint,chain,predict,fluoro,fluoro-predict",
                    help="extra timed runs reported beside the main line (comma list; '' = none)")
    ap.add_argument("--variant-steps", type=int, default=0,
                    help="steps of each variant (0: as many as the main run; the adjoint "
                         "variant at most 60)")
    ap.add_argument("--predict-order", type=int, default=2,
                    help="polynomial order of the history predictor in the *predict variants")
    ap.add_argument("--fluoro-angle", type=float, default=30.0,
                    help="gantry angle (deg) of the fixed-angle variants")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pca", action="store_true", help="skip the PCA-training measurement")
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
    res = run_sequence(ctx, W, ys[Wm:], geoms[Wm:], idxs[Wm:], opts, warm["w"], profile=True)
    summ = summarise(res, W, idxs[Wm:], spp[Wm:])
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
        "kernels": kernel_table(res["prof"]),
        "roofline": roofline(W, res["prof"],
                             float(np.sum(res["samples"])) / max(res["prof"]["march"][1], 1), channels,
                             4 * channels, "march_fused_%dx%dx%d_f32" % tuple(W.grid.n)),
    }
    log("[bench] main: %.1f solves/s p50 %.2f ms p99 %.2f ms" % (summ["solves_per_s"], summ["p50_ms"],
                                                                 summ["p99_ms"]))
    log("[bench] main line: " + json.dumps(line))
    variants = {}
    fl = None
    for v in [s for s in args.variants.split(",") if s]:
        po = 0
        vsteps = min(Ks, args.variant_steps or (60 if v == "adjoint" else Ks))
        if v in ("bf16", "f16", "bf16-image", "f16-image"):
            dm, f0v = storage_model(W, v.split("-")[0], dev)
            cv = _lib.Context(W.grid, dm, f0v,
                              image_dtype=torch.float16 if v.endswith("image") else torch.float32)
            wv = run_sequence(cv, W, ys[:Wm], geoms[:Wm], idxs[:Wm], opts, [0.0] * K)
            rv = run_sequence(cv, W, ys[Wm:Wm + vsteps], geoms[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], opts, wv["w"], profile=True)
            cv.close()
        elif v == "adjoint":
            o2 = _lib.default_opts(max_iter=W.cfg["max_iter"], step0=W.model.step0,
                                   grad_mode=_lib.GRAD_ADJOINT, localize=1, p_ref_mm=W.p_ref)
            wv = run_sequence(ctx, W, ys[:Wm], geoms[:Wm], idxs[:Wm], o2, [0.0] * K)
            rv = run_sequence(ctx, W, ys[Wm:Wm + vsteps], geoms[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], o2, wv["w"], profile=True)
        elif v in ("predict", "fluoro", "fluoro-predict", "chain", "predict-chain", "quadratic-step"):
            po = args.predict_order if "predict" in v else 0
            chain = v.endswith("chain")
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
                              predict_order=po, chain_mu=chain)
            rv = run_sequence(ctx, W, vy[Wm:Wm + vsteps], vg[Wm:Wm + vsteps],
                              idxs[Wm:Wm + vsteps], vo, wv["w"], profile=True,
                              predict_order=po, hist=wv["hist"], chain_mu=chain)
            if v.startswith("fluoro"):
                vspp = np.full(vsteps, float(samples_per_ray(W.grid, vg[Wm]).sum()))
        else:
            continue
        sv = summarise(rv, W, idxs[Wm:Wm + vsteps], vspp if v.startswith("fluoro") else spp[Wm:Wm + vsteps])
        if v.startswith("fluoro"):
            sv["angle_deg"] = args.fluoro_angle
        if po:
            sv["predict_order"] = po
        if v.endswith("chain"):
            sv["step_size_carried"] = True
        if v == "quadratic-step":
            sv["step_rule"] = "quadratic model"
        sv["steps"] = vsteps
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
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, idxs[Wm], args.cpu_iters,
                                            float(res["iters"].mean()))
        log("[bench] cpu baseline %.4g solves/s on %d threads" % (line["cpu_baseline"]["value"],
                                                                  line["cpu_baseline"]["cores"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
