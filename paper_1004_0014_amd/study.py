"""Accuracy study on the synthetic ground truth (section 3's evaluation, and
the detector-resolution study of section 5).

For projections over one gantry rotation of the paper-scale workload it
reports, per projection and in summary:

* the relative image error e = sqrt(sum (f - f*)^2 / sum f*^2) of the
  reconstructed volume f = warp(f0, mean + U w) against the ground-truth
  volume f* = warp(f0, 1.5 x(t)) (the test motion lies in the model's span,
  so f* is exactly representable), beside the initial error of the reference
  image f0 against f*;
* the 3D tumour localisation error |p - p*| (p* from the analytic motion)
  and its RMS over the rotation;
* with --resolutions, the same at detector sizes from 40x30 to 1000x750
  pixels over the same 40 x 30 cm imager.

The solves run in the HIP library; e is an evaluation metric computed with
torch on the device.

    python -m paper_1004_0014_amd.study --every 10
    python -m paper_1004_0014_amd.study --resolutions 40,80,200,512,1000 --every 30
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch

from . import _lib, synth as S


def true_tumour(grid, phi, R, scale, p_ref):
    """p with p + x(p) = p_ref for the analytic test motion (closed-form field)."""
    L = grid.fov
    amps = (1.0, 0.3, 0.15, 0.1, 0.08)
    c = S.phase_coeffs(phi, R) * scale
    p = np.array(p_ref, dtype=float)
    for _ in range(200):
        g = math.exp(-(p[0] / (0.35 * L[0])) ** 2)
        hz, sx = p[2] / L[2], p[0] / L[0]
        comps = [(2, 1.0), (1, 1.0), (2, hz), (1, hz), (0, sx)]
        x = np.zeros(3)
        for i in range(R):
            ax, f = comps[i]
            x[ax] += 10.0 * amps[i] * g * f * c[i]
        pn = p_ref - x
        if np.linalg.norm(pn - p) < 1e-12:
            return pn
        p = pn
    return p


def rel_err(a, b):
    return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))


def run_rotation(name="paper", every=1, nu=None, dev="cuda", angles=None, measure=None):
    """Solves the projections at gantry angles `angles` (degrees; default
    every `every`-th degree of one rotation; projection i is taken at
    t = i / rate) in sequence, each warm-started from the previous result,
    and scores each against the ground truth.  measure(i, geom, w_true)
    returns the measured projection as an FP32 device tensor (default: the
    library projects the phantom warped by the true w).  Returns a summary and
    one row per projection (with the solved w and the localised tumour)."""
    cfg = S.config(name)
    g = S.grid_for(name)
    K = cfg["K"]
    rate = cfg.get("rate_hz", 11.0)
    m = S.pca_model(g, K)
    f0 = torch.tensor(S.phantom(g), dtype=torch.float32, device=dev)
    dm = _lib.DeviceModel(torch.tensor(m.mean, dtype=torch.float32, device=dev),
                          torch.tensor(m.U, dtype=torch.float32, device=dev))
    ctx = _lib.Context(g, dm, f0)
    p_ref = S.tumor_center(g)
    nu = nu or cfg["nu"]
    nv = max(1, round(nu * cfg["nv"] / cfg["nu"]))
    du = cfg["nu"] * cfg["du"] / nu
    opts = _lib.default_opts(max_iter=cfg["max_iter"], step0=m.step0, localize=1, p_ref_mm=p_ref)
    w = np.zeros(K)
    rows = []
    for i in (range(0, 360, every) if angles is None else angles):
        t = i / rate
        phi = S.breathing_phase(t)
        w_true = S.truth_w(m, phi)
        G = S.Geom(math.radians(i), nu, nv, du, du, cfg["step"])
        f_true = _lib.warp_volume(g, f0, _lib.dvf_compose(g, dm, w_true))
        if measure is None:
            y = _lib.forward_project(g, G, f_true)
        else:
            y = measure(i, G, w_true)
        w0 = np.array(w, dtype=float)
        w, ab, st = ctx.reconstruct(y, G, w, opts)
        f_rec = _lib.warp_volume(g, f0, _lib.dvf_compose(g, dm, w))
        pt = true_tumour(g, phi, K, 1.5, p_ref)
        rows.append(dict(angle=i, e=rel_err(f_rec, f_true), e_ref=rel_err(f0, f_true),
                         loc_mm=float(np.linalg.norm(np.array(st["tumor_mm"]) - pt)),
                         loc_xyz_mm=list(np.array(st["tumor_mm"]) - pt),
                         iterations=st["iterations"], w0=list(w0), w=list(np.asarray(w, float)),
                         w_true=list(w_true), tumor_mm=list(st["tumor_mm"]),
                         tumor_true_mm=list(pt), status=st["status"]))
    ctx.close()
    e = np.array([r["e"] for r in rows])
    loc = np.array([r["loc_mm"] for r in rows])
    xyz = np.array([r["loc_xyz_mm"] for r in rows])
    return {"config": name, "detector": [nu, nv], "pitch_mm": du, "projections": len(rows),
            "e_mean": float(e.mean()), "e_std": float(e.std()),
            "e_ref_mean": float(np.mean([r["e_ref"] for r in rows])),
            "loc_rms_mm": float(np.sqrt(np.mean(loc ** 2))), "loc_mean_mm": float(loc.mean()),
            "loc_std_mm": float(loc.std()),
            "loc_rms_lr_ap_si_mm": [float(np.sqrt(np.mean(xyz[:, a] ** 2))) for a in range(3)],
            "mean_iterations": float(np.mean([r["iterations"] for r in rows]))}, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="paper")
    ap.add_argument("--every", type=int, default=10, help="use every n-th projection (degree)")
    ap.add_argument("--resolutions", default="", help="comma list of detector widths (pixels)")
    ap.add_argument("--rows", action="store_true", help="print per-projection rows")
    args = ap.parse_args()
    widths = [int(v) for v in args.resolutions.split(",") if v] or [None]
    for nu in widths:
        summ, rows = run_rotation(args.config, args.every, nu)
        print(json.dumps({"study": summ}), flush=True)
        if args.rows:
            for r in rows:
                print(json.dumps(r), flush=True)
        print("[study] %s detector %s: e %.4f (ref %.4f), loc rms %.3f mm" % (
            args.config, summ["detector"], summ["e_mean"], summ["e_ref_mean"], summ["loc_rms_mm"]),
            file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
