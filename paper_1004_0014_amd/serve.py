"""Serving harness: many simulated patient streams feeding the serving engine
(pcr_server_*, the C++ continuous-batching loop in csrc/serve.hip).

Workload (serving configuration): 64 streams; per stream a seeded volume
nx = ny ~ U{128..512} (multiples of 16), nz ~ U{64..160} (multiples of 8)
over a 480 x 480 x 320 mm field of view, K ~ U{2..5}, a detector
nu ~ U{256..1024} (multiples of 32), nv = 3/4 nu, 397 mm / nu pitch, one
projection every 1/11 s with N(0, 10 ms) jitter, gantry angle advancing at
6 deg/s from a seeded start (one rotation per minute, section 3), breathing
at 1.5x the training amplitude with a 4 s period.  Reference images and
eigenvector fields are stored BF16 on the device (FP32 with --storage f32);
compute is FP32.

Inputs are synthesised on the GPU with plain torch ops (ellipsoid thorax,
smoothed Gaussian texture, the analytic rank-K breathing motion and its PCA
through the K x K pattern Gram matrix) -- input plumbing only; every solve
runs in the HIP library.  Measured projections are the library's projections
of the truth-warped FP32 phantom.

    python -m paper_1004_0014_amd.serve --streams 64 --seconds 3
"""
from __future__ import annotations

import argparse
import copy
import json
import math
import sys
import threading
import time

import numpy as np
import torch

from . import _lib
from .synth import Geom, Grid, phase_coeffs

FOV = (480.0, 480.0, 320.0)
AMPS = (1.0, 0.3, 0.15, 0.1, 0.08)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ inputs -------
def stream_spec(rng: np.random.Generator):
    nxy = int(rng.integers(8, 33)) * 16             # 128..512
    nz = int(rng.integers(8, 21)) * 8               # 64..160
    K = int(rng.integers(2, 6))                     # 2..5
    nu = int(rng.integers(8, 33)) * 32              # 256..1024
    nv = nu * 3 // 4
    theta0 = float(rng.uniform(0, 2 * math.pi))
    grid = Grid((nxy, nxy, nz), (FOV[0] / nxy, FOV[1] / nxy, FOV[2] / nz))
    return dict(grid=grid, K=K, nu=nu, nv=nv, du=397.0 / nu, theta0=theta0)


def _mesh(grid, dev):
    ax = [torch.tensor(grid.origin[a] + grid.spacing[a] * np.arange(grid.n[a]), dtype=torch.float32,
                       device=dev) for a in range(3)]
    return ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None]


def gpu_phantom(grid, seed, dev):
    """Ellipsoid thorax (same construction as synth.phantom) with a
    seeded torch texture."""
    L = grid.fov
    px, py, pz = _mesh(grid, dev)
    mu = torch.zeros(grid.shape, dtype=torch.float32, device=dev)

    def inside(c, s):
        return ((px - c[0]) / s[0]) ** 2 + ((py - c[1]) / s[1]) ** 2 + ((pz - c[2]) / s[2]) ** 2 <= 1.0

    mu[inside((0, 0, 0), (0.40 * L[0], 0.30 * L[1], 0.60 * L[2]))] = 0.02
    for sx in (1, -1):
        mu[inside((sx * 0.17 * L[0], 0.02 * L[1], 0.05 * L[2]),
                  (0.13 * L[0], 0.20 * L[1], 0.30 * L[2]))] = 0.004
    tc = (-0.17 * L[0], 0.02 * L[1], -0.05 * L[2])
    mu[inside(tc, (10.0, 10.0, 10.0))] = 0.02
    g = torch.Generator(device=dev).manual_seed(seed)
    z = torch.randn(grid.shape, generator=g, device=dev, dtype=torch.float32)
    k = np.exp(-0.5 * np.arange(-4, 5) ** 2)
    k = k / k.sum()
    for ax in range(3):           # separable Gaussian (sigma = 1 voxel), zero padded
        n = z.shape[ax]
        pad = [0, 0] * 3
        pad[2 * (2 - ax)] = pad[2 * (2 - ax) + 1] = 4
        zp = torch.nn.functional.pad(z, pad)
        z = sum(float(k[j]) * zp.narrow(ax, j, n) for j in range(9))
    z = z / z.std()
    return (mu * (1.0 + 0.05 * z)).contiguous(), np.array(tc)


def gpu_model(grid, K, dev):
    """Rank-K analytic motion patterns and their PCA (training phases
    2 pi j / 10, j = 1..9) through the K x K pattern Gram matrix."""
    L = grid.fov
    px, py, pz = _mesh(grid, dev)
    gx = torch.exp(-(px / (0.35 * L[0])) ** 2).expand(grid.shape)
    hz = (pz / L[2]).expand(grid.shape)
    sx = (px / L[0]).expand(grid.shape)
    comps = [(2, gx), (1, gx), (2, gx * hz), (1, gx * hz), (0, gx * sx)]
    P = torch.zeros((K, 3) + grid.shape, dtype=torch.float32, device=dev)
    for i in range(K):
        ax, f = comps[i]
        P[i, ax] = 10.0 * AMPS[i] * f
    Pf = P.view(K, -1)
    Q = (Pf.double() @ Pf.double().T).cpu().numpy()
    phis = 2 * np.pi * np.arange(1, 10) / 10
    C = phase_coeffs(phis, K)
    cbar = C.mean(axis=1)
    Lc = np.linalg.cholesky(Q)
    A, _, _ = np.linalg.svd(Lc.T @ (C - cbar[:, None]), full_matrices=False)
    Z = np.linalg.solve(Lc.T, A)[:, :K]
    U = torch.stack([sum(float(Z[j, k]) * Pf[j] for j in range(K)) for k in range(K)]).view(
        (K, 3) + grid.shape)
    for k in range(K):
        j = int(torch.argmax(U[k].abs()))
        if float(U[k].reshape(-1)[j]) < 0:
            U[k] = -U[k]
            Z[:, k] = -Z[:, k]
    mean = sum(float(cbar[j]) * Pf[j] for j in range(K)).view((3,) + grid.shape)
    w_train = (C - cbar[:, None]).T @ Q @ Z
    step0 = 0.5 * float(np.sqrt(np.mean(np.sum(w_train ** 2, axis=1))))
    return mean.contiguous(), U.contiguous(), dict(Z=Z, Q=Q, cbar=cbar, step0=step0)


def truth_w(pca, K, phi, scale=1.5):
    c = phase_coeffs(phi, K) * scale - pca["cbar"]
    return pca["Z"].T @ pca["Q"] @ c


class SimStream:
    """One patient stream: model and reference image stored in `storage`
    (BF16 by default; FP32 keeps them as built), request schedule and
    measured projections (FP32, on the device)."""

    def __init__(self, idx, seed, seconds, dev, rate_hz=11.0, jitter_s=0.010,
                 storage=torch.bfloat16):
        rng = np.random.default_rng([seed, idx])
        sp = stream_spec(rng)
        self.idx, self.K, self.grid = idx, sp["K"], sp["grid"]
        f0, self.p_ref = gpu_phantom(self.grid, seed * 1000 + idx, dev)
        mean, U, self.pca = gpu_model(self.grid, self.K, dev)
        dm32 = _lib.DeviceModel(mean, U)
        n = int(math.floor(seconds * rate_hz))
        t = np.arange(n) / rate_hz + rng.normal(0.0, jitter_s, n) + rng.uniform(0, 1.0 / rate_hz)
        self.times = np.sort(np.maximum(t, 0.0))
        self.geoms, self.ys, self.w_true = [], [], []
        t_phase = rng.uniform(0, 4.0)
        for tk in self.times:
            ang = sp["theta0"] + math.radians(6.0) * tk
            G = Geom(ang, sp["nu"], sp["nv"], sp["du"], sp["du"], 0.5 * min(self.grid.spacing))
            w = truth_w(self.pca, self.K, 2 * math.pi * (tk + t_phase) / 4.0)
            dvf = _lib.dvf_compose(self.grid, dm32, w)
            f = _lib.warp_volume(self.grid, f0, dvf)
            self.ys.append(_lib.forward_project(self.grid, G, f))
            self.geoms.append(G)
            self.w_true.append(w)
            del dvf, f
        self.f0 = f0.to(storage)
        self.model = _lib.DeviceModel(mean.to(storage), U.to(storage))
        self.spec = sp
        del f0, mean, U, dm32

    def as_storage(self, storage):
        """The same stream (schedule, projections, truth) with its reference
        image and model converted to `storage`."""
        c = copy.copy(self)
        c.f0 = self.f0.to(storage)
        c.model = _lib.DeviceModel(self.model.mean.to(storage), self.model.U.to(storage))
        return c

    def opts(self):
        return _lib.default_opts(max_iter=50, step0=self.pca["step0"], localize=1, p_ref_mm=self.p_ref)


def build_streams(n_streams, seconds, seed, dev, storage=torch.bfloat16):
    t0 = time.time()
    out = []
    for i in range(n_streams):
        out.append(SimStream(i, seed, seconds, dev, storage=storage))
        if (i + 1) % 8 == 0:
            log("[serve] built %d/%d streams (%.1fs)" % (i + 1, n_streams, time.time() - t0))
    torch.cuda.synchronize()
    return out


# ----------------------------------------------------------------- run -----
def run(streams, seconds, max_slots, budget_gb, drop_stale=True, image_f16=False, predict_order=0,
        carry_move=False):
    srv = _lib.Server(hbm_budget_bytes=int(budget_gb * (1 << 30)), max_slots=max_slots,
                      drop_stale=drop_stale, image_f16=image_f16, predict_order=predict_order,
                      carry_move=carry_move)
    sids, rejected = [], 0
    for st in streams:
        try:
            sids.append(srv.add_stream(st.grid, st.model, st.f0, st.opts(), np.zeros(st.K)))
        except _lib.PCRError as e:
            if e.status != _lib.PCR_EBUSY:
                raise
            sids.append(None)
            rejected += 1
    events = sorted((t, i, j) for i, st in enumerate(streams) if sids[i] is not None
                    for j, t in enumerate(st.times))
    results, req_meta = [], {}
    done = threading.Event()

    def poller():
        while not done.is_set() or len(results) < len(req_meta):
            results.extend(srv.poll(512, wait_ms=20))
            if done.is_set() and len(results) >= len(req_meta):
                break

    th = threading.Thread(target=poller, daemon=True)
    th.start()
    t_start = time.perf_counter()
    for t, i, j in events:
        delay = t_start + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        rid = srv.submit(sids[i], streams[i].ys[j], streams[i].geoms[j])
        req_meta[rid] = (i, j)
    t_sub_end = time.perf_counter()
    srv.drain()
    t_end = time.perf_counter()
    done.set()
    th.join(timeout=60)
    srv.close()
    served = [r for r in results if r["status"] in (0, -4)]
    dropped = [r for r in results if r["status"] == _lib.PCR_EBUSY]
    failed = [r for r in results if r["status"] not in (0, -4, _lib.PCR_EBUSY)]
    lat = np.array([r["t_done_s"] - r["t_submit_s"] for r in served]) * 1e3
    wait = np.array([r["t_start_s"] - r["t_submit_s"] for r in served]) * 1e3
    werr = []
    for r in served:
        i, j = req_meta[r["req_id"]]
        wt = streams[i].w_true[j]
        werr.append(float(np.linalg.norm(np.array(r["w"]) - wt) / np.linalg.norm(wt)))
    span = t_end - t_start
    return {
        "streams": len(streams), "admitted": len(streams) - rejected, "rejected": rejected,
        "max_slots": max_slots, "requests": len(events),
        "offered_per_s": len(events) / seconds,
        "served": len(served), "dropped": len(dropped), "failed": len(failed),
        "served_per_s": len(served) / span, "makespan_s": span,
        "submit_window_s": t_sub_end - t_start,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "queue_wait_p50_ms": float(np.percentile(wait, 50)) if len(wait) else None,
        "mean_iterations": float(np.mean([r["iterations"] for r in served])) if served else None,
        # work-normalised rate: ray samples marched by the served solves per
        # second (mixes of different sizes are comparable on it)
        "served_gsamples_per_s": sum(r["samples"] for r in served) / span * 1e-9,
        "mean_gsamples_per_solve": float(np.mean([r["samples"] for r in served])) * 1e-9 if served else None,
        "w_rel_err_median": float(np.median(werr)) if werr else None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--streams", default="64", help="comma list of stream counts")
    ap.add_argument("--seconds", type=float, default=3.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--image-f16", action="store_true", help="FP16 fused images")
    ap.add_argument("--predict-order", type=int, default=0,
                    help="warm start from the extrapolation of each stream's last results")
    ap.add_argument("--carry-move", action="store_true",
                    help="first trial moves w by the distance the stream's last solve moved it")
    ap.add_argument("--storage", default="bf16", choices=["bf16", "f32"],
                    help="storage of the streams' reference images and models")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    counts = [int(s) for s in args.streams.split(",")]
    storage = torch.bfloat16 if args.storage == "bf16" else torch.float32
    streams = build_streams(max(counts), args.seconds, args.seed, dev, storage=storage)
    for n in counts:
        res = run(streams[:n], args.seconds, args.slots, args.budget_gb, image_f16=args.image_f16,
                  predict_order=args.predict_order, carry_move=args.carry_move)
        print(json.dumps({"serving": res}), flush=True)


if __name__ == "__main__":
    main()
