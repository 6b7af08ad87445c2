#!/usr/bin/env python3
"""Throughput of the progressive saliency-guided hologram on one MI355X.

One step = one full hot-path pass (fused DWT/saliency/masking, FP64 fringe
tables, active lists and operand panels, both contractions, optional split-K
reduce) producing one complex64 hologram per scene from inputs already resident
in HBM.  Default workload: a 2048 x 2048 object with a smooth depth map
quantised to 8 planes (z = 0.1-0.3 m), ~20% saliency, 3 Haar levels,
lambda 532 nm, pitch 8 um (seeded, synthetic).  The headline is the FP32 form;
the BF16 and FP16 split forms are measured on the same inputs in the same run
(``forms``), each with its relative L2 error against the FP64 oracle sample.

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
# real MFMA products issued per algorithmic real product: 128 x 128 tiles (four real
# products per complex product; the split forms issue three MFMAs per real product)
ISSUE_FACTOR = {"fp32": 1.0, "bf16_split": 3.0, "fp16_split": 3.0}
# the single-scene second contraction: FP32 runs 128 x 64 tiles with three real products
# per complex product (Gauss), so 3/4 of the algorithmic real products are issued
SECOND_ISSUE = {"fp32": 0.75, "bf16_split": 3.0, "fp16_split": 3.0}
SECOND_TILE = {"fp32": "128x64, 3 real products per complex product",
               "bf16_split": "256x128, one workgroup per CU",
               "fp16_split": "256x128, one workgroup per CU"}
SECOND_KERNEL = {"fp32": "nt_direct_kernel", "bf16_split": "nt_pp_kernel",
                 "fp16_split": "nt_pp_kernel"}
DTYPES = {"fp32": "f32", "bf16_split": "bf16x3-split/f32-acc", "fp16_split": "f16x3-split/f32-acc"}
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
    "grad1024": (scenes.differentiable,
                 "1024x1024 float32 amplitudes, one plane z=0.2 m, ~30% saliency, 3 Haar levels; "
                 "loss = sum (|Fresnel back-propagation of H| - T)^2 with a blob target; one "
                 "step = forward + back-propagation + loss + gradient through the adjoints"),
    "literal2048x8": (scenes.depth_2048,
                      "the 2048x2048, 8-plane scene of depth2048x8 by the paper-literal form: "
                      "approximation image and residual maps times uniform-block fringes, dense"),
    "fused2048x8": (scenes.depth_2048,
                    "the 2048x2048, 8-plane scene of depth2048x8 by the dense reconstruct-then-"
                    "contract form: masked reconstruction per layer, one dense Fresnel "
                    "contraction pair per layer (12 N^3 flops per layer, no saliency skipping)"),
    "stages256": (lambda: scenes.tiny(n=256),
                  "256x256 object (the paper's image size), one plane z=0.2 m, ~25% saliency, "
                  "3 levels: the four progressive stage holograms, their inverse "
                  "angular-spectrum reconstructions (and Fresnel back-propagations) and the SSIM "
                  "of each against the point-wise hologram's, with the operator counts of every "
                  "step"),
    "exact256": (lambda: scenes.tiny(n=256),
                 "256x256 object, one plane z=0.2 m, ~25% saliency, 3 Haar levels; Eq. 1 with the "
                 "exact distance and 1/r amplitude as a direct sum (evaluation of the Fresnel form)"),
    "recon2048": (lambda: {"n": 2048, "z": 0.2, "seed": 2211},
                  "inverse angular-spectrum reconstruction (the paper's reconstruction method) of "
                  "a 2048x2048 unit-modulus random-phase hologram recorded at z=0.2 m, lambda "
                  "532 nm, pitch 8 um"),
    "batch64": (scenes.batched,
                "64 scenes, sides uniform in {256,512,768,1024,1536,2048}, 1-4 depth planes, "
                "saliency 5-60% from 1-3 ellipses, 3 Haar levels; one batched plan "
                "(persistent contractions, autotuned tiles, HIP graph)"),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=sorted(PEAKS_TFLOPS),
                    help="form reported as the headline value")
    ap.add_argument("--forms", default="all", choices=["all", "one"],
                    help="also measure the other precision forms (all) or only --precision")
    ap.add_argument("--workload", default="depth2048x8", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-pixels", type=int, default=1536,
                    help="hologram pixels the oracle evaluates for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="tile-shape cache for batched plans")
    ap.add_argument("--mfma-peak", action="store_true",
                    help="only run the matrix-core throughput probe (register-resident MFMA "
                         "loops, no memory traffic) for FP32, BF16 and FP16 and exit")
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


# probe launches: (kind, iterations per wave) sized to about 20 ms at one wave per SIMD
PEAK_PROBES = {"fp32": ("fp32", 20000), "bf16_split": ("bf16", 40000),
               "fp16_split": ("fp16", 40000)}


def mfma_attainable(prec, blocks=256, zero=False, launches=3):
    """Sustained matrix-core rate (TFLOP/s) of the probe for the form's MFMA
    instruction: mean over `launches` timed launches after one warm-up."""
    import torch

    from paper_2211_09938_amd import cgh

    kind, iters = PEAK_PROBES[prec]
    sink, flops = cgh.mfma_peak(kind, blocks, iters, zero)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(launches):
        cgh.mfma_peak(kind, blocks, iters, zero, sink)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    return flops / (ms * 1e-3) / 1e12, ms


def mfma_peak_lines():
    """One JSON line per probe configuration (the attainable-peak calibration)."""
    for prec in ("fp32", "bf16_split", "fp16_split"):
        for blocks in (256, 512):
            for zero in (False, True):
                tf, ms = mfma_attainable(prec, blocks, zero)
                print(json.dumps({"probe": "mfma_peak", "instruction": PEAK_PROBES[prec][0],
                                  "waves_per_simd": blocks // 256, "operands":
                                  "zero" if zero else "random", "tflops": tf,
                                  "published_peak_tflops": PEAKS_TFLOPS[prec],
                                  "frac_of_published": tf / PEAKS_TFLOPS[prec],
                                  "avg_launch_ms": ms}), flush=True)


def host_cpu():
    """CPU model and core counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        affinity = None
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "cpus_in_affinity": affinity,
            "worker_cap": "the oracle's pool takes the process's CPU affinity, at most 16 "
                          "processes (one GPU's share of the host); ORACLE_WORKERS overrides"}


def crop_reference(scene, size=256, seed=2048):
    """FP64 window of the hologram (separable oracle) at a seeded offset: the 256 x 256
    crop the depth workload's parity is stated on (the same offset as its test)."""
    from oracle import separable

    ny, nx = scene.shape
    h, w = min(size, ny), min(size, nx)
    rng = np.random.default_rng(seed)
    y0, x0 = (int(v) for v in rng.integers(0, [ny - h + 1, nx - w + 1]))
    sal = None if scene.saliency is None else scene.saliency.astype(np.float64)
    ref = separable.window(scene.obj.astype(np.float64), scene.z, scene.lam, scene.pitch,
                           scene.levels, sal, scene.layer, y0=y0, x0=x0, h=h, w=w)
    return y0, x0, ref


def cpu_separable_baseline(scene):
    """The oracle's separable FP64 form (kernel-matrix products on the host's BLAS) timed on
    the whole hologram: a stronger CPU reference than the direct sum, reported beside it."""
    from oracle import separable

    sal = None if scene.saliency is None else scene.saliency.astype(np.float64)
    t0 = time.perf_counter()
    separable.window(scene.obj.astype(np.float64), scene.z, scene.lam, scene.pitch,
                     scene.levels, sal, scene.layer)
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "holograms/s", "kind": "oracle (separable FP64 BLAS form)",
            "threads": os.environ.get("OMP_NUM_THREADS", "BLAS default (all host CPUs)"),
            "sample": f"the whole {scene.shape[0]}x{scene.shape[1]} hologram, {len(scene.z)} "
                      f"layer(s), {t:.2f} s"}


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
        **host_cpu(),
        "kind": "oracle",
        "sample": (f"FP64 direct 2D point sum at {n_pixels} seeded pixels of the same hologram "
                   f"({t2 - t1:.1f} s) plus the masked reconstruction of every layer "
                   f"({t1 - t0:.1f} s), extrapolated linearly to all {ny * nx} pixels"),
        "_pixels": (ys, xs, vals),
    }


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# valid only while the kernel and plan sources hash to what they were when counted
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TRAFFIC_SOURCES = ("paper_2211_09938_amd/csrc/ntgemm.hip", "paper_2211_09938_amd/csrc/nt.h",
                   "paper_2211_09938_amd/csrc/plan.hip")


def sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, prec):
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha1") != sources_sha1():
        return None
    entry = rec.get("entries", {}).get(f"{workload}/{prec}")
    return None if entry is None else entry["bytes"]


# exact-distance kernel: VALU instructions per (point, pixel) term, counted in the
# gfx950 ISA of its inner loop; VALU issue peak = 256 CUs x 64 lanes per clock x 2.4 GHz
EXACT_VALU_PER_TERM = 79
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9


def run_exact(scene, steps, warmup):
    import torch

    from paper_2211_09938_amd import cgh

    dev = torch.device("cuda:0")
    ny, nx = scene.shape
    obj = torch.from_numpy(scene.obj).to(dev)
    sal = torch.from_numpy(scene.saliency).to(dev)
    ws = torch.empty(cgh.workspace_size(ny, nx, 1, scene.levels, "fp32"), dtype=torch.uint8,
                     device=dev)
    out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)

    def step():
        cgh.exact_hologram(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal, out=out,
                           workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = a.elapsed_time(b) / steps
    # every point of the blob object's masked reconstruction is nonzero: dense count
    terms = float(ny * nx) ** 2
    achieved = terms / (ms * 1e-3) / 1e9
    peak = VALU_LANE_OPS_PER_S / EXACT_VALU_PER_TERM / 1e9
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "roofline": {"bound": "alu", "kernel": "exact_kernel", "achieved": achieved,
                     "peak": peak, "unit": "Gterm/s", "frac": achieved / peak, "traffic": None,
                     "valu_per_term": EXACT_VALU_PER_TERM, "avg_launch_ms": ms},
        "_out": out.cpu().numpy(),
    }


def run_dense(scene, prec, steps, warmup, form):
    """The dense forms: paper-literal residual maps ("literal") or the masked
    reconstruction contracted once per layer ("fused")."""
    import torch

    from paper_2211_09938_amd import cgh

    dev = torch.device("cuda:0")
    ny, nx = scene.shape
    obj = torch.from_numpy(scene.obj).to(dev)
    sal = torch.from_numpy(scene.saliency).to(dev)
    lay = None if scene.layer is None else torch.from_numpy(scene.layer).to(dev)
    layers = len(scene.z)
    ws = torch.empty(cgh.workspace_size(ny, nx, layers, scene.levels, prec), dtype=torch.uint8,
                     device=dev)
    out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)
    fn = cgh.literal_hologram if form == "literal" else cgh.fused_hologram

    def step():
        fn(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal, lay, precision=prec, out=out,
           workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # dense work: per layer a real x complex product (ny x k) x (k x nx) and a complex product
    # (ny x k) x (k x nx) with k = nx >> b, ny >> b per image b of the literal form (block 2^b,
    # b = L..0), k = nx, ny once for the fused form; matrix-core flops issued: the FP32 complex
    # product takes the three-product form (3/4 of its real products)
    sizes = [(ny >> b, nx >> b) for b in range(scene.levels, -1, -1)] if form == "literal" \
        else [(ny, nx)]
    fl = 0.0
    fl_issued = 0.0
    for r, c in sizes:
        fl += layers * (4.0 * r * c * nx + 8.0 * ny * r * nx)
        fl_issued += layers * (ISSUE_FACTOR[prec] * 4.0 * r * c * nx
                               + SECOND_ISSUE[prec] * 8.0 * ny * r * nx)
    ms = 1e3 * elapsed / steps
    # achieved: the matrix-core flops the two contractions' algorithms perform (three-product
    # FP32 complex form, three products per real product in the split forms); the method's
    # count (8 real flops per complex multiply-add) beside it
    achieved = fl_issued / (ms * 1e-3) / 1e12
    return {
        "value": steps / elapsed,
        "ms_per_step": ms,
        "stages_ms_per_step": {},
        "work": {"flops_dense": fl},
        "roofline": {"bound": "mfma", "kernel": f"whole {form} step (both contractions dominate)",
                     "achieved": achieved, "peak": PEAKS_TFLOPS[prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAKS_TFLOPS[prec], "traffic": None,
                     "flops_per_launch": fl_issued, "flops_4m_per_launch": fl,
                     "achieved_4m": fl / (ms * 1e-3) / 1e12},
        "_out": out.cpu().numpy(),
    }


def run_stages(scene, prec, steps, warmup):
    import torch

    from paper_2211_09938_amd import cgh, quality

    dev = torch.device("cuda:0")
    ny, nx = scene.shape
    obj = torch.from_numpy(scene.obj).to(dev)
    sal = torch.from_numpy(scene.saliency).to(dev)
    ws = torch.empty(cgh.workspace_size(ny, nx, 1, scene.levels, prec), dtype=torch.uint8,
                     device=dev)
    st = torch.empty((scene.levels + 1, ny, nx), dtype=torch.complex64, device=dev)

    def step():
        cgh.progressive_stages(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal,
                               precision=prec, out=st, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = cgh.workspace_stats(ws, ny, nx, 1, scene.levels, prec)
    # every block salient = the point-wise hologram (each point its own fringe)
    full = cgh.progressive_hologram(obj, scene.z, scene.lam, scene.pitch, scene.levels, None,
                                    precision=prec)
    z = scene.z[0]

    def amp_angular(h):  # the paper's reconstruction: inverse angular spectrum
        return cgh.reconstruct(h, scene.lam, scene.pitch, z).abs().cpu().numpy().astype(np.float64)

    def amp_fresnel(h):
        return cgh.fresnel_backpropagate(h, scene.lam, scene.pitch, z, precision=prec).abs() \
            .cpu().numpy().astype(np.float64)

    refs = {k: f(full) for k, f in (("angular", amp_angular), ("fresnel", amp_fresnel))}
    rows = []
    cum = 0
    for j in range(scene.levels + 1):
        h = st[j].contiguous()
        cum += stats["operators"][j]
        row = {"stage": ["LLL", "LL", "L", "object"][j] if scene.levels == 3 else j}
        for k, f in (("angular", amp_angular), ("fresnel", amp_fresnel)):
            ref = refs[k]
            key = "ssim_vs_pointwise" if k == "angular" else "ssim_vs_pointwise_fresnel_recon"
            row[key] = quality.ssim(f(h), ref, float(ref.max() - ref.min()))
        row.update({"operators_cumulative": cum,
                    "operators_frac_of_pointwise": cum / stats["operators_pointwise"]})
        rows.append(row)
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "stages": rows,
        "operators_pointwise": stats["operators_pointwise"],
    }


def run_recon(spec, steps, warmup):
    """Inverse angular-spectrum reconstruction of one n x n field per step."""
    import torch

    from paper_2211_09938_amd import cgh

    n, z = spec["n"], spec["z"]
    rng = np.random.default_rng(spec["seed"])
    field_h = np.exp(2j * np.pi * rng.random((n, n))).astype(np.complex64)
    dev = torch.device("cuda:0")
    field = torch.from_numpy(field_h).to(dev)
    out = torch.empty_like(field)
    ws = torch.empty(cgh.lib().cgh_angular_spectrum_workspace_size(n, n), dtype=torch.uint8,
                     device=dev)

    def step():
        cgh.reconstruct(field, scenes.WAVELENGTH, scenes.PITCH, z, out=out, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the library launches on torch's current stream: events there bracket its kernels
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = a.elapsed_time(b) / steps
    alg = 16.0 * n * n  # the field read once, the reconstruction written once
    achieved = alg / (ms * 1e-3) / 1e9
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "roofline": {"bound": "hbm", "kernel": "cgh_angular_spectrum (five launches: row FFT, "
                     "transpose, column FFT x transfer x inverse FFT, transpose, row inverse FFT)",
                     "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "traffic": None, "bytes_per_call": alg,
                     "pass_bytes_per_call": 5 * alg, "avg_call_ms": ms},
        "_field": field_h,
        "_out": out.cpu().numpy(),
    }


def recon_cpu_baseline(field, z):
    from oracle import angular

    t0 = time.perf_counter()
    ref = angular.reconstruct(field.astype(np.complex128), scenes.WAVELENGTH, scenes.PITCH, z)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "reconstructions/s", "cores": 1, "kind": "oracle",
            "sample": f"one whole {field.shape[0]}x{field.shape[1]} reconstruction "
                      "(numpy FFT, complex128, one thread)", "_ref": ref}


def exact_cpu_baseline(scene, n_pixels=256):
    from oracle import exact, fresnel

    ny, nx = scene.shape
    rng = np.random.default_rng(12345)
    ys = rng.integers(0, ny, n_pixels)
    xs = rng.integers(0, nx, n_pixels)
    t0 = time.perf_counter()
    vals = exact.hologram_exact(scene.obj.astype(np.float64), scene.z, scene.lam, scene.pitch,
                                scene.levels, scene.saliency.astype(np.float64), None,
                                pixels=(ys, xs))
    t = time.perf_counter() - t0
    return {
        "value": 1.0 / (t * ny * nx / n_pixels),
        "unit": "holograms/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 exact-distance sum at {n_pixels} seeded pixels ({t:.1f} s), "
                  f"extrapolated linearly to all {ny * nx} pixels",
        "_pixels": (ys, xs, vals),
    }


def gauss_tile(prec, tm, tn):
    """FP32 complex tiles of 128 x 64 and smaller issue three real products per complex one."""
    return prec == "fp32" and tm * tn <= 128 * 64


def batch_second_kernel(prec, info):
    """The batch's second contraction: the ring kernel when the autotuner chose its tile."""
    return ("nt_pp_kernel" if prec != "fp32" and tuple(info["second_tile"]) == (256, 128)
            else "nt_persistent_kernel")


def roofline(stats, prec, avg_ms, kernel, traffic=None, issue=None, attainable=None):
    """Second contraction: the real flops its algorithm performs per launch over the
    average launch time, against the published dense peak of its MFMA type.

    The method's count (``flops_4m_per_launch``) is 8 real flops per complex
    multiply-add, 8 * ny * nx * active coefficient rows.  The kernel performs
    ``issue`` times that on the matrix cores: 3/4 in the three-product FP32 form,
    3x in the split forms (hi*hi + hi*lo + lo*hi per real product), so ``achieved``
    counts issue x the method's flops on the active rows and ``frac`` is a true
    fraction of the peak.  ``issued_mfma_frac`` adds the zero rows that pad every K
    segment to 16; ``attainable`` is the register-resident probe's rate for the same
    instruction on this GPU, measured in the same run.
    """
    issue = SECOND_ISSUE[prec] if issue is None else issue
    t = avg_ms * 1e-3
    flops = issue * stats["flops_second"]
    achieved = flops / t / 1e12
    peak = PEAKS_TFLOPS[prec]
    issued = issue * stats["flops_second_issued"] / t / 1e12
    frac = achieved / peak
    if frac > 1.0:
        print(f"bench.py: roofline fraction {frac:.3f} > 1 for {kernel}: flop count or timing "
              "is wrong", file=sys.stderr)
    out = {
        "bound": "mfma",
        "kernel": kernel,
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": frac,
        "traffic": traffic,
        "flops_per_launch": flops,
        "avg_launch_ms": avg_ms,
        "issued_mfma_frac": issued / peak,
        "flops_4m_per_launch": stats["flops_second"],
        "achieved_4m": stats["flops_second"] / t / 1e12,
        "mfma_flops_per_4m_flop": issue,
    }
    if attainable is not None:
        out["attainable"] = attainable
        out["frac_of_attainable"] = achieved / attainable
    return out


def timed_steps(step, steps):
    """Times `steps` calls of step() with a HIP event pair only around the second
    contraction (every recorded event idles the stream a few microseconds), then
    runs a few more steps with a pair at every stage for the per-stage breakdown.
    Returns (seconds, (second-contraction ms, launches), per-stage profile)."""
    import torch

    from paper_2211_09938_amd import cgh

    torch.cuda.synchronize()
    cgh.profile_stages(["second"])
    cgh.profile_enable(True)
    cgh.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    second = cgh.profile_read(reset=True)["second"]
    cgh.profile_stages(None)
    for _ in range(min(steps, 5)):
        step()
    torch.cuda.synchronize()
    prof = cgh.profile_read(reset=True)
    cgh.profile_enable(False)
    return elapsed, second, prof


def run_single(scene, prec, steps, warmup, workload):
    import torch

    from paper_2211_09938_amd import cgh

    dev = torch.device("cuda:0")
    ny, nx = scene.shape
    obj = torch.from_numpy(scene.obj).to(dev)
    sal = None if scene.saliency is None else torch.from_numpy(scene.saliency).to(dev)
    lay = None if scene.layer is None else torch.from_numpy(scene.layer).to(dev)
    n_layers = len(scene.z)
    ws = torch.empty(cgh.workspace_size(ny, nx, n_layers, scene.levels, prec), dtype=torch.uint8,
                     device=dev)
    out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)

    def step():
        cgh.progressive_hologram(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal, lay,
                                 precision=prec, out=out, workspace=ws)

    for _ in range(warmup):
        step()
    elapsed, (sec_ms, sec_n), prof = timed_steps(step, steps)
    stats = cgh.workspace_stats(ws, ny, nx, n_layers, scene.levels, prec)
    kernel = f"second contraction ({SECOND_KERNEL[prec]}<{prec}, complex A, {SECOND_TILE[prec]}>)"
    # the HBM-bound coefficient stage: flag clear + fused layer split / Haar / masks;
    # algorithmic bytes = object 4 B + layer id 1 B + saliency 4 B read per pixel,
    # 4 B written per pixel and layer
    coef_ms = prof["coef"][0] / max(1, prof["coef"][1])
    px = float(ny * nx)
    coef_bytes = px * (4 + (1 if lay is not None else 0) + (4 if sal is not None else 0)) \
        + px * 4 * n_layers
    hbm = {"kernel": "dwt_mask_kernel (coefficient stage)", "bound": "hbm",
           "achieved": coef_bytes / (coef_ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
           "bytes_per_launch": coef_bytes, "avg_launch_ms": coef_ms}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "stages_ms_per_step": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
        "work": stats,
        "roofline": roofline(stats, prec, sec_ms / max(1, sec_n), kernel,
                             measured_traffic(workload, prec),
                             attainable=mfma_attainable(prec)[0]),
        "hbm_roofline": hbm,
        "_out": out.cpu().numpy(),
    }


def run_grad(scene, prec, steps, warmup):
    import torch

    from paper_2211_09938_amd import cgh

    dev = torch.device("cuda:0")
    ny, nx = scene.shape
    obj = torch.from_numpy(scene.obj).to(dev).requires_grad_(True)
    sal = torch.from_numpy(scene.saliency).to(dev)
    target = torch.from_numpy(scene.extra["target"]).to(dev)
    z = scene.z[0]

    def step():
        obj.grad = None
        h = cgh.hologram_fn(obj, [z], scene.lam, scene.pitch, scene.levels, sal, None, None, prec)
        u = cgh.backprop_fn(h, scene.lam, scene.pitch, z, prec)
        loss = ((u.abs() - target) ** 2).sum()
        loss.backward()
        return loss

    for _ in range(warmup):
        step()
    elapsed, (sec_ms, sec_n), prof = timed_steps(step, steps)
    ws = torch.empty(cgh.workspace_size(ny, nx, 1, scene.levels, prec), dtype=torch.uint8, device=dev)
    cgh.progressive_hologram(obj.detach(), [z], scene.lam, scene.pitch, scene.levels, sal,
                             precision=prec, workspace=ws)
    stats = cgh.workspace_stats(ws, ny, nx, 1, scene.levels, prec)
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "stages_ms_per_step": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
        "work": stats,
        "roofline": roofline(stats, prec, sec_ms / max(1, sec_n),
                             f"forward second contraction inside the step ({SECOND_KERNEL[prec]}<{prec}>)"),
    }


def run_batch(batch, prec, steps, warmup, tune_cache):
    import torch

    from paper_2211_09938_amd import cgh

    dev = torch.device("cuda:0")
    descs = []
    for s in batch:
        d = {"obj": torch.from_numpy(s.obj).to(dev), "z": s.z,
             "saliency": torch.from_numpy(s.saliency).to(dev)}
        if s.layer is not None:
            d["layer_index"] = torch.from_numpy(s.layer).to(dev)
        descs.append(d)
    t_plan = time.perf_counter()
    plan = cgh.Plan(descs, scenes.WAVELENGTH, scenes.PITCH, precision=prec, tune_cache=tune_cache)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan
    for _ in range(warmup):
        plan.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-kernel durations: the same kernels launched eagerly with stage events
    cgh.profile_enable(True)
    cgh.profile_read(reset=True)
    for _ in range(3):
        plan.execute()
    torch.cuda.synchronize()
    prof = cgh.profile_read(reset=True)
    cgh.profile_enable(False)
    stats = plan.stats()
    info = plan.info()
    sec_ms, sec_n = prof["second"]
    n = len(batch)
    res = {
        "value": n * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "stages_ms_per_step": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
        "work": stats,
        "roofline": roofline(stats, prec, sec_ms / max(1, sec_n),
                             f"second contraction ({batch_second_kernel(prec, info)}<{prec}, "
                             f"{info['second_tile'][0]}x{info['second_tile'][1]}"
                             + (", 3 real products per complex product>)"
                                if gauss_tile(prec, *info["second_tile"]) else ">)"),
                             issue=(0.75 if gauss_tile(prec, *info["second_tile"])
                                    else ISSUE_FACTOR[prec])),
        "plan": dict(info, create_s=t_plan),
    }
    plan.close()
    return res


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.mfma_peak:
        mfma_peak_lines()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the hologram would shard by bands of hologram columns)", file=sys.stderr)
        sys.exit(2)
    make, desc = WORKLOADS[args.workload]
    work = make()
    if args.workload.startswith("stages"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("bench.py needs a GPU")
        res = run_stages(work, args.precision, args.steps, args.warmup)
        line = {"metric": "progressive stage sets/s (all levels+1 stage holograms) with SSIM "
                          "of each stage vs the point-wise hologram and operator counts",
                "value": res["value"], "unit": "stage sets/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": DTYPES[args.precision], "data": "synthetic",
                "config": {"workload": args.workload, "description": desc,
                           "ny": work.shape[0], "nx": work.shape[1]},
                "stages": res["stages"], "operators_pointwise": res["operators_pointwise"]}
        print(json.dumps(line), flush=True)
        return
    if args.workload.startswith("recon"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("bench.py needs a GPU")
        res = run_recon(work, args.steps, args.warmup)
        field, out = res.pop("_field"), res.pop("_out")
        line = {"metric": "inverse angular-spectrum reconstructions/s (the paper's "
                          "reconstruction method)",
                "value": res["value"], "unit": "reconstructions/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32 (f64 twiddles and transfer phase)", "data": "synthetic",
                "config": {"workload": args.workload, "description": desc, "ny": work["n"],
                           "nx": work["n"]},
                "roofline": res["roofline"]}
        if not args.no_cpu_baseline:
            base = recon_cpu_baseline(field, work["z"])
            ref = base.pop("_ref")
            line["rel_l2_vs_oracle"] = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
            line["cpu_baseline"] = base
        print(json.dumps(line), flush=True)
        return
    if args.workload.startswith("exact"):
        base = None if args.no_cpu_baseline else exact_cpu_baseline(work)
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("bench.py needs a GPU")
        res = run_exact(work, args.steps, args.warmup)
        out = res.pop("_out")
        line = {"metric": "exact-distance Eq. 1 holograms/s (evaluation kernel)",
                "value": res["value"], "unit": "holograms/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32 (f64 phase reduction and tile sums)", "data": "synthetic",
                "config": {"workload": args.workload, "description": desc,
                           "ny": work.shape[0], "nx": work.shape[1]},
                "roofline": res["roofline"]}
        if base is not None:
            ys, xs, vals = base.pop("_pixels")
            got = out[ys, xs].astype(np.complex128)
            line["rel_l2_vs_oracle"] = float(np.linalg.norm(got - vals) / np.linalg.norm(vals))
            line["cpu_baseline"] = base
        print(json.dumps(line), flush=True)
        return
    batch = isinstance(work, list)
    scene = work[0] if batch else work

    grad = args.workload.startswith("grad")
    base = None if (args.no_cpu_baseline or batch or grad) else cpu_baseline(scene, args.cpu_pixels)

    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    precs = [args.precision]
    if args.forms == "all":
        precs += [p for p in ("fp32", "bf16_split", "fp16_split") if p != args.precision]
    crop = None
    if base is not None and not args.workload.startswith(("literal", "fused")):
        crop = crop_reference(scene)
        base["separable"] = cpu_separable_baseline(scene)
    forms = {}
    for prec in precs:
        if batch:
            forms[prec] = run_batch(work, prec, args.steps, args.warmup, args.tune_cache)
        elif grad:
            forms[prec] = run_grad(scene, prec, args.steps, args.warmup)
        elif args.workload.startswith("literal"):
            forms[prec] = run_dense(scene, prec, args.steps, args.warmup, "literal")
        elif args.workload.startswith("fused"):
            forms[prec] = run_dense(scene, prec, args.steps, args.warmup, "fused")
        else:
            forms[prec] = run_single(scene, prec, args.steps, args.warmup, args.workload)
        out = forms[prec].pop("_out", None)
        if base is not None and out is not None:
            ys, xs, vals = base["_pixels"]
            got = out[ys, xs].astype(np.complex128)
            forms[prec]["rel_l2_vs_oracle"] = float(np.linalg.norm(got - vals) / np.linalg.norm(vals))
        if crop is not None and out is not None:
            y0, x0, ref = crop
            win = out[y0:y0 + ref.shape[0], x0:x0 + ref.shape[1]].astype(np.complex128)
            forms[prec]["crop_rel_l2_vs_oracle"] = {
                "value": float(np.linalg.norm(win - ref) / np.linalg.norm(ref)),
                "window": [y0, x0, ref.shape[0], ref.shape[1]]}
        forms[prec]["dtype"] = DTYPES[prec]
    head = forms[args.precision]
    if batch:
        points_pixels = sum(float(s.obj.size) ** 2 for s in work) / len(work)
        config = {"workload": args.workload, "description": desc, "scenes": len(work),
                  "sides": sorted({s.shape[0] for s in work}), "precision": args.precision}
    else:
        points_pixels = float(scene.obj.size) ** 2
        config = {"workload": args.workload, "description": desc, "ny": scene.shape[0],
                  "nx": scene.shape[1], "planes": len(scene.z), "levels": scene.levels,
                  "precision": args.precision}
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "loss+grad/s" if grad else "holograms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": config,
        "gpoint_pixel_per_s": head["value"] * points_pixels / 1e9,
        "roofline": head["roofline"],
        "stages_ms_per_step": head["stages_ms_per_step"],
        "hbm_roofline": head.get("hbm_roofline"),
        "work": head["work"],
    }
    if "rel_l2_vs_oracle" in head:
        line["rel_l2_vs_oracle"] = head["rel_l2_vs_oracle"]
    if "crop_rel_l2_vs_oracle" in head:
        line["crop_rel_l2_vs_oracle"] = head["crop_rel_l2_vs_oracle"]
    if batch:
        line["plan"] = head["plan"]
    line["forms"] = {p: {k: v for k, v in f.items() if k != "work"} for p, f in forms.items()}
    if base is not None:
        base.pop("_pixels")
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
