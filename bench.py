#!/usr/bin/env python3
"""Benchmark: simulated images/s + p50/p99 latency of the headline image
(200x200 px at 0.05"/px, supersampling 3, SIE + shear + 10,000 NFW subhalos,
one lens-light + two source Sersic components, 41x41 PSF) on one MI355X.

A step is one full simulated image: subhalo-table derivation, the fused
ray-shooting + surface-brightness + supersample kernel, and the PSF
convolution, with all inputs resident in HBM before the timed region.

Prints one JSON line.  `roofline` refers to the dominant kernel (the fused
simulate kernel); its duration comes from HIP events the library records on
the launch stream during the timed region.  `cpu_baseline` times the FP64
oracle on a bounded sample of the same image on this host.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "simulated images/s + p50/p99 latency (200² px, 10k NFW, 41² PSF); % FP32 peak"
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector, published
# Algorithmic FP32 work of one (sub-pixel, subhalo) NFW pair in this
# formulation (FMA = 2, transcendental = 1): dx, dy 2; r^2 3; x^2 1;
# rsq + log2 2; degree-8 polynomial 16; g 2; g/x^2 2; * c2 1; accumulate 4.
FLOP_PER_PAIR = 33
KERNEL_SOURCES = ["paper_2606_01547_amd/csrc/kernels.hip", "paper_2606_01547_amd/csrc/jt_device.hpp",
                  "paper_2606_01547_amd/csrc/nfw_poly.inc"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_simulate_headline_traffic.json")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, or None when absent or taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(scene, rows):
    """The FP64 oracle on `rows` pixel rows of the image (every sub-pixel of
    them through the full deflector sum and light), plus the full-image PSF
    convolution; extrapolated to one whole image."""
    import numpy as np
    import oracle as O
    g = scene.grid
    t0 = time.perf_counter()
    tx, ty = O.subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    tx, ty = tx[:rows], ty[:rows]
    bx, by = O.ray_shoot(tx, ty, scene.lens)
    sb = O.surface_brightness(tx, ty, bx, by, scene.source, scene.lens_light, scene.bn_exact)
    part = O.supersample_reduce(sb, g.pixel_scale)
    t1 = time.perf_counter()
    O.convolve_same(np.zeros((g.ny, g.nx)) + part.mean(), scene.psf)
    t2 = time.perf_counter()
    per_image = (t1 - t0) * g.ny / rows + (t2 - t1)
    pairs = rows * g.nx * g.supersample ** 2 * scene.lens.nfw.n
    return {"value": 1.0 / per_image, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": (f"{rows} of {g.ny} pixel rows ({pairs:.3g} sub-pixel x subhalo pairs) through the FP64 "
                       f"oracle in {t1 - t0:.1f} s plus one full-image convolution ({t2 - t1:.2f} s), "
                       f"extrapolated to a whole image; single NumPy process"),
            "seconds": round(t2 - t0, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--cpu-rows", type=int, default=10, help="pixel rows of the oracle sample (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times), to calibrate "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU figures are not produced",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2606_01547_amd import Context

    scene = W.config2_scene()
    g = scene.grid
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    # inputs resident in HBM before timing: subhalo SoA and the PSF as device tensors
    nfw = scene.lens.nfw
    dev_nfw = W.NFWTable(*[torch.from_numpy(np.asarray(a)).to(dev) for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)])
    lens = W.Lens(sie=scene.lens.sie, shear=scene.lens.shear, nfw=dev_nfw)
    psf = torch.from_numpy(scene.psf).to(dev)
    out = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)

    def step():
        ctx.simulate_image(g, lens, scene.source, scene.lens_light, psf, scene.bn_exact, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim_ms, sim_n = ctx.profile_read("sim")
    conv_ms, conv_n = ctx.profile_read("conv")
    prep_ms, prep_n = ctx.profile_read("prep")
    ctx.profile_enable(False)

    total = t1 - t0
    ms_per_step = 1e3 * total / args.steps
    value = args.steps / total

    # latency: one image at a time, host clock from call to completion
    lat = []
    for _ in range(args.latency_samples):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - a))
    lat = np.array(lat)

    pairs = g.nx * g.ny * g.supersample ** 2 * nfw.n
    sim_avg_s = 1e-3 * sim_ms / max(sim_n, 1)
    achieved = FLOP_PER_PAIR * pairs / sim_avg_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic_per_launch(),
                "kernel": "k_simulate", "avg_ms": round(1e3 * sim_avg_s, 4),
                "flop_per_launch": FLOP_PER_PAIR * pairs, "pairs_per_s": round(pairs / sim_avg_s, 1)}

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "200x200 px at 0.05\"/px, supersampling 3, SIE + shear + 10000 NFW, "
                               "1 lens-light + 2 source Sersic, 41x41 PSF (seed 1002)",
                   "global_batch": 1, "subhalos": nfw.n, "pixels": g.nx * g.ny, "supersample": g.supersample,
                   "psf": int(scene.psf.shape[0])},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4), "samples": int(lat.size)},
        "kernels_ms": {"simulate": round(sim_ms / max(sim_n, 1), 4), "convolve": round(conv_ms / max(conv_n, 1), 4),
                       "prep": round(prep_ms / max(prep_n, 1), 4)},
        "roofline": roofline,
    }
    if args.cpu_rows > 0:
        result["cpu_baseline"] = cpu_baseline(scene, args.cpu_rows)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
