"""Kernel-profiling driver: repeats one pass of the hot path at the
paper-scale workload (256x256x100 volume, K = 3, 512x384 detector) so that
`rocprofv3` can time it or read its counters, and runs a plain device copy of
a known size beside it to calibrate the byte counters.

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 -m paper_1004_0014_amd.kprof
    rocprofv3 --pmc FETCH_SIZE -d OUT -o run -- python3 -m paper_1004_0014_amd.kprof

Each repetition is one fused cost-and-gradient evaluation (warp + march +
reduce) at a fixed gantry angle, one backprojection with --what backproject,
or one PCA training of the motion model from its 9 training DVFs with --what pca.
--config serve-max takes the largest volume and detector of the serving
workload, where the image no longer fits the caches.
"""
from __future__ import annotations

import argparse
import math
import sys

import torch

from . import _lib, synth as S

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="paper",
                    help="paper, tiny, diff, precision, or serve-max: the largest volume and detector "
                         "of the serving configuration (512x512x160 over 480x480x320 mm, K = 5, "
                         "1024x768 at 397/1024 mm), whose fused image (1.04 GB) exceeds the caches")
    ap.add_argument("--angle", type=float, default=30.0)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--what", default="fused", choices=["fused", "adjoint", "backproject", "forward", "pca"])
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--image", default="f32", choices=["f32", "f16"],
                    help="element type of the fused image")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    if args.config == "serve-max":
        g = S.Grid((512, 512, 160), (480.0 / 512, 480.0 / 512, 320.0 / 160))
        K = 5
        G = S.Geom(math.radians(args.angle), 1024, 768, 397.0 / 1024, 397.0 / 1024, 0.5 * 480.0 / 512)
    else:
        g = S.grid_for(args.config)
        K = S.CONFIGS[args.config]["K"]
        G = S.geom_for(args.config, math.radians(args.angle))
    dt = torch.float32 if args.storage == "f32" else torch.bfloat16
    if args.config == "serve-max":
        # inputs synthesised on the device (the serving harness's generators)
        from . import serve
        f0, _ = serve.gpu_phantom(g, 4000, dev)
        mean, U, pca = serve.gpu_model(g, K, dev)
        dm32 = _lib.DeviceModel(mean, U)
        w = serve.truth_w(pca, K, 2.0)
        m = None
    else:
        m = S.pca_model(g, K)
        f0 = torch.tensor(S.phantom(g), dtype=torch.float32, device=dev)
        dm32 = _lib.DeviceModel(torch.tensor(m.mean, dtype=torch.float32, device=dev),
                                torch.tensor(m.U, dtype=torch.float32, device=dev))
        w = S.truth_w(m, 2.0)
    y = _lib.forward_project(g, G, _lib.warp_volume(g, f0, _lib.dvf_compose(g, dm32, w)))
    dm = dm32 if dt == torch.float32 else _lib.DeviceModel(dm32.mean.to(dt), dm32.U.to(dt))
    f0s = f0.to(dt)
    ctx = _lib.Context(g, dm, f0s, image_dtype=torch.float16 if args.image == "f16" else torch.float32)
    if args.what == "pca" and m is None:
        raise SystemExit("--what pca needs a configuration with an analytic model (not serve-max)")
    if args.what == "pca":
        d = torch.from_numpy(S.training_dvfs(g, m.R)).to(dev)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        if args.what in ("fused", "adjoint"):
            ctx.cost_grad(y, G, 0.9 * w, 1.0, 0.0, mode=0 if args.what == "fused" else 1)
        elif args.what == "backproject":
            _lib.backproject_residual(g, G, y)
        elif args.what == "pca":
            _lib.pca_train(g, d, K)
        else:
            _lib.forward_project(g, G, f0)
        dst.copy_(src)                       # calibration: 256 MiB read + 256 MiB written
    torch.cuda.synchronize()
    print("kprof done: %s x%d at %s, %s storage, %s image" % (args.what, args.reps, args.config,
                                                             args.storage, args.image), file=sys.stderr)


if __name__ == "__main__":
    main()
