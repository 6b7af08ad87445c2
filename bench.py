#!/usr/bin/env python3
"""Throughput of the progressive saliency-guided hologram on one MI355X.

One step = one full hot-path pass (fused DWT/saliency/masking, FP64 fringe
tables, both contractions, optional split-K reduce) producing one complex64
hologram from inputs already resident in HBM.  Default workload: a 2048 x 2048
object with a smooth depth map quantised to 8 planes (z = 0.1-0.3 m), ~20%
saliency, 3 Haar levels, lambda 532 nm, pitch 8 um (seeded, synthetic).

Prints one JSON line: holograms/s, ms per step, the dominant kernel's roofline
(second contraction: algorithmic flops per launch over its average duration,
from HIP events recorded on the launch stream) and the FP64 oracle timed on a
bounded pixel sample on the host cores (before the GPU is touched).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2211_09938_amd import scenes  # noqa: E402

PEAKS_TFLOPS = {"fp32": 157.3, "bf16_split": 2516.6, "fp16_split": 2516.6}
METRIC = "holograms/sec and Gpoint*pixel/s at 2048^2, FP32 vs BF16-split at stated rel-L2"

WORKLOADS = {
    "depth2048x8": (scenes.depth_2048,
                    "2048x2048 object, smooth depth quantised to 8 planes z=0.1-0.3 m, "
                    "~20% saliency (1 ellipse), 3 Haar levels, lambda 532 nm, pitch 8 um"),
    "plane1024": (scenes.plane_1024,
                  "1024x1024 object, one plane z=0.2 m, ~30% saliency (3 ellipses), "
                  "3 Haar levels, lambda 532 nm, pitch 8 um"),
    "tiny128": (scenes.tiny,
                "128x128 object, one plane z=0.2 m, ~25% saliency, 3 Haar levels"),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=sorted(PEAKS_TFLOPS))
    ap.add_argument("--workload", default="depth2048x8", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-pixels", type=int, default=1536,
                    help="hologram pixels the oracle evaluates for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference for scaling hardware byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 4, "launches": 5}), flush=True)


def cpu_baseline(scene, n_pixels, seed=12345):
    """FP64 oracle on a seeded pixel sample of the same hologram (host cores only)."""
    from oracle import fresnel, progressive

    ny, nx = scene.shape
    rng = np.random.default_rng(seed)
    ys = rng.integers(0, ny, n_pixels)
    xs = rng.integers(0, nx, n_pixels)
    obj = scene.obj.astype(np.float64)
    sal = None if scene.saliency is None else scene.saliency.astype(np.float64)
    t0 = time.perf_counter()
    recon = [progressive.masked_reconstruction(a, sal, scene.levels)
             for a in progressive.layer_split(obj, scene.layer, len(scene.z))]
    t1 = time.perf_counter()
    vals = np.zeros(n_pixels, dtype=np.complex128)
    for d, a_hat in enumerate(recon):
        vals += fresnel.direct_sum(a_hat, scene.lam, scene.pitch, scene.z[d], ys, xs)
    t2 = time.perf_counter()
    per_holo = (t1 - t0) + (t2 - t1) * (ny * nx) / n_pixels
    return {
        "value": 1.0 / per_holo,
        "unit": "holograms/s",
        "cores": fresnel.worker_count(),
        "kind": "oracle",
        "sample": (f"FP64 direct 2D point sum at {n_pixels} seeded pixels of the same hologram "
                   f"({t2 - t1:.1f} s) plus the masked reconstruction of every layer "
                   f"({t1 - t0:.1f} s), extrapolated linearly to all {ny * nx} pixels"),
        "_pixels": (ys, xs, vals),
    }


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the hologram would shard by column bands, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    make, desc = WORKLOADS[args.workload]
    scene = make()
    ny, nx = scene.shape

    base = None if args.no_cpu_baseline else cpu_baseline(scene, args.cpu_pixels)

    import torch

    from paper_2211_09938_amd import cgh

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    obj = torch.from_numpy(scene.obj).to(dev)
    sal = None if scene.saliency is None else torch.from_numpy(scene.saliency).to(dev)
    lay = None if scene.layer is None else torch.from_numpy(scene.layer).to(dev)
    n_layers = len(scene.z)
    ws = torch.empty(cgh.workspace_size(ny, nx, n_layers, scene.levels, args.precision),
                     dtype=torch.uint8, device=dev)
    out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)

    def step():
        cgh.progressive_hologram(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal, lay,
                                 precision=args.precision, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    cgh.profile_enable(True)
    cgh.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = cgh.profile_read(reset=True)
    cgh.profile_enable(False)
    stats = cgh.workspace_stats(ws, ny, nx, n_layers, scene.levels, args.precision)

    holo_s = args.steps / elapsed
    sec_ms, sec_n = prof["second"]
    avg_ms = sec_ms / max(1, sec_n)
    achieved = stats["flops_second"] / (avg_ms * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    points = float(ny * nx)
    line = {
        "metric": METRIC,
        "value": holo_s,
        "unit": "holograms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16_split": "bf16x3-split/f32-acc",
                  "fp16_split": "f16x3-split/f32-acc"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "ny": ny, "nx": nx,
                   "planes": n_layers, "levels": scene.levels, "precision": args.precision},
        "gpoint_pixel_per_s": holo_s * points * points / 1e9,
        "roofline": {
            "bound": "mfma",
            "kernel": ("second contraction (cgemm_f32_kernel<FwdS2>)" if args.precision == "fp32"
                       else "second contraction (cgemm_split_kernel<FwdS2>)"),
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "flops_per_launch": stats["flops_second"],
            "avg_launch_ms": avg_ms,
        },
        "stages_ms_per_step": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
        "work": stats,
    }
    if base is not None:
        ys, xs, vals = base.pop("_pixels")
        got = out.cpu().numpy()[ys, xs].astype(np.complex128)
        line["rel_l2_vs_oracle"] = float(np.linalg.norm(got - vals) / np.linalg.norm(vals))
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
