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
PEAK_HBM_BYTES = 8.0e12           # MI355X HBM3E, published
# Algorithmic FP32 work of one (sub-pixel, subhalo) NFW pair in the form a
# distant pair takes (y = Rs/r below 0.125 for its group of four subhalos: at
# least 93% of the headline's pairs), FMA = 2: dx, dy 2; r^2 = dx dx + dy dy 3;
# x^2/4 = r^2 c1/4 1; rsq + log2 2; degree-4 polynomial (3 FMA) 6;
# g' = fma(R, y, log) 2; y^2 and g' y^2 2; * c2 1; two accumulating FMAs 4;
# the group's branch test 1.  The remaining pairs take the degree-8 form
# (33 FLOP), not counted, so `achieved` is a lower bound; the executed FLOP
# from the committed counters is reported beside it as executed_frac.
FLOP_PER_PAIR = 24
KERNEL_SOURCES = ["paper_2606_01547_amd/csrc/kernels.hip", "paper_2606_01547_amd/csrc/jt_device.hpp",
                  "paper_2606_01547_amd/csrc/nfw_poly.inc", "paper_2606_01547_amd/csrc/jt_sum.hpp",
                  "paper_2606_01547_amd/csrc/atan_poly.inc"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_simulate_headline_traffic.json")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters():
    """The committed rocprofv3 counter summary of the fused kernel (HBM bytes
    per launch, executed FLOP per pair), or {} when absent or taken on other
    kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_sources_sha256_16") != kernel_hash():
        return {}
    return t


def _oracle_rows(job):
    """The FP64 oracle on pixel rows [r0, r1) of a scene: every sub-pixel of
    them through the full deflector sum and light, then the supersample mean.
    Returns the seconds it took."""
    import oracle as O
    scene, r0, r1 = job
    g = scene.grid
    t0 = time.perf_counter()
    tx, ty = O.subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    tx, ty = tx[r0:r1], ty[r0:r1]
    bx, by = O.ray_shoot(tx, ty, scene.lens)
    sb = O.surface_brightness(tx, ty, bx, by, scene.source, scene.lens_light, scene.bn_exact)
    O.supersample_reduce(sb, g.pixel_scale)
    return time.perf_counter() - t0


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(scene, rows, workers, rows_per_worker=4):
    """The FP64 oracle timed on this host, extrapolated to one whole image:
    (i) one process on `rows` pixel rows; (ii) `workers` spawned processes,
    each on `rows_per_worker` rows, timed by the wall clock around the pool
    (start-up included).  Both add one full-image PSF convolution.  The value
    is the faster of the two."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    import oracle as O
    g = scene.grid
    t0 = time.perf_counter()
    O.convolve_same(np.zeros((g.ny, g.nx)), scene.psf)
    t_conv = time.perf_counter() - t0
    pairs_row = g.nx * g.supersample ** 2 * scene.lens.nfw.n
    t_single = _oracle_rows((scene, 0, rows))
    single = 1.0 / (t_single * g.ny / rows + t_conv)
    model, avail = host_cpu()
    out = {"value": single, "unit": "images/s", "cores": 1, "kind": "oracle",
           "sample": (f"{rows} of {g.ny} pixel rows ({rows * pairs_row:.3g} sub-pixel x subhalo pairs) through the "
                      f"FP64 oracle in {t_single:.1f} s in one NumPy process, plus one full-image convolution "
                      f"({t_conv:.2f} s), extrapolated to a whole image"),
           "seconds": round(t_single + t_conv, 2), "host_cpu": model, "host_cores_available": avail,
           "single_process_images_per_s": single}
    workers = min(workers, avail, g.ny // rows_per_worker)
    if workers > 1:
        jobs = [(scene, w * rows_per_worker, (w + 1) * rows_per_worker) for w in range(workers)]
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            busy = list(ex.map(_oracle_rows, jobs))
        wall = time.perf_counter() - t0
        done = workers * rows_per_worker
        pooled = 1.0 / (wall * g.ny / done + t_conv)
        out["pool"] = {"images_per_s": pooled, "processes": workers, "rows": done, "wall_s": round(wall, 2),
                       "mean_worker_busy_s": round(sum(busy) / workers, 2)}
        if pooled > single:
            out["value"] = pooled
            out["cores"] = workers
            out["sample"] = (f"{done} of {g.ny} pixel rows ({done * pairs_row:.3g} sub-pixel x subhalo pairs) "
                             f"through the FP64 oracle on {workers} spawned NumPy processes ({rows_per_worker} rows "
                             f"each) in {wall:.1f} s wall, plus one full-image convolution ({t_conv:.2f} s), "
                             f"extrapolated to a whole image; one process alone on {rows} rows: "
                             f"{single:.4g} images/s")
    return out


def serving_bench(ctx, n_requests, large_every, seed=1003, loads=(0.5, 0.8, 1.0)):
    """The request stream served by the continuous-batching server: a
    saturated calibration pass (everything submitted at once), then Poisson
    arrivals at each of `loads` times the saturated rate, each schedule also
    served by one jt_simulate_image call per request (FIFO, one stream, the
    same resident subhalo tables and device PSFs) for comparison."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_01547_amd import Server
    t_gen = time.perf_counter()
    scenes = W.config3_requests(n_requests, seed=seed)
    if large_every:
        for i in range(large_every - 1, n_requests, large_every):
            scenes[i] = W.config5_scene(seed=1005 + i)
    import types
    handles, outs, pairs, direct = [], [], 0.0, []
    for sc in scenes:
        hs = ctx.upload_subhalos(sc.lens.nfw) if sc.lens.nfw.n > 0 else 0
        hp = ctx.upload_psf(sc.psf)
        handles.append((hs, hp))
        outs.append(torch.empty((sc.grid.ny, sc.grid.nx), dtype=torch.float32, device="cuda"))
        # the per-image path gets the same resident subhalo table and a device PSF
        direct.append((types.SimpleNamespace(sie=sc.lens.sie, shear=sc.lens.shear, subhalo_handle=hs),
                       torch.from_numpy(np.ascontiguousarray(sc.psf, dtype=np.float32)).cuda()))
        pairs += sc.grid.nx * sc.grid.ny * sc.grid.supersample ** 2 * sc.lens.nfw.n
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t_gen
    cfg = dict(hbm_budget_bytes=4 << 30, max_batch_images=64, max_batch_pairs=4e9, max_inflight_batches=8,
               n_streams=4)

    def run(arrivals):
        srv = Server(ctx, **cfg)
        t0 = time.perf_counter()
        tickets = []
        for sc, (hs, hp), o, ta in zip(scenes, handles, outs, arrivals):
            while True:
                dt = t0 + ta - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 2e-3))
            tickets.append(srv.submit(sc.grid, sc.lens, sc.source, sc.lens_light, out=o, subhalo_handle=hs,
                                      psf_handle=hp))
        lat = np.array([srv.wait(t) for t in tickets])
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, wall, st

    def run_per_image(arrivals):
        # one jt_simulate_image per request, FIFO, waiting for each
        lat = []
        t0 = time.perf_counter()
        for sc, (lens, psf), o, ta in zip(scenes, direct, outs, arrivals):
            while True:
                dt = t0 + ta - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 2e-3))
            ctx.simulate_image(sc.grid, lens, sc.source, sc.lens_light, psf, getattr(sc, "bn_exact", False), out=o)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - (t0 + ta))
        return np.array(lat), time.perf_counter() - t0

    pct = lambda a, q: round(1e3 * float(np.percentile(a, q)), 3)
    lat_sat, wall_sat, st_sat = run(np.zeros(n_requests))
    rate_sat = n_requests / wall_sat
    poisson = {}
    for load in loads:
        lam = load * rate_sat
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / lam, n_requests))
        arrivals -= arrivals[0]
        lat, wall, st = run(arrivals)
        pimg, wall_pi = run_per_image(arrivals)
        poisson[f"{load:g}"] = {
            "arrival_rate_per_s": round(lam, 2),
            "server": {"images_per_s": round(n_requests / wall, 2), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                       "batches": int(st["batches"]), "arena_peak_bytes": int(st["arena_peak"])},
            "per_image_launches": {"images_per_s": round(n_requests / wall_pi, 2), "p50_ms": pct(pimg, 50),
                                   "p99_ms": pct(pimg, 99)}}
    for hs, hp in handles:
        for h in (hs, hp):
            if h:
                ctx.release(h)
    return {
        "workload": (f"{n_requests} seeded requests: grid from {{64,100,200,400}}^2, s from {{1,3}}, "
                     f"log-uniform 0-20000 NFW, PSF 21 or 41" +
                     (f"; every {large_every}th a 1000^2, s=5, 50000-NFW, 101^2-PSF image" if large_every else "")),
        "pairs": pairs, "generation_s": round(gen_s, 2),
        "saturated": {"images_per_s": round(rate_sat, 2), "p50_ms": pct(lat_sat, 50), "p99_ms": pct(lat_sat, 99),
                      "batches": int(st_sat["batches"])},
        "poisson_by_load": poisson,
        "server_config": cfg,
    }


def conv_sweep(ctx, reps=10):
    """Direct against FFT convolution, kernel time from the library's HIP
    events, on 200^2 and 1000^2 images for PSF sides 21..101, and the path
    method 0 picks."""
    import numpy as np
    import torch
    from paper_2606_01547_amd import convolve_auto_method
    rng = np.random.default_rng(7)
    rows = []
    for n in (200, 1000):
        img = torch.from_numpy(rng.uniform(0, 1, (n, n)).astype(np.float32)).cuda()
        out = torch.empty_like(img)
        for k in (21, 41, 61, 81, 101):
            psf = rng.uniform(0, 1, (k, k))
            psf = torch.from_numpy((psf / psf.sum()).astype(np.float32)).cuda()
            us = {}
            for name, m in (("direct", 1), ("fft", 2)):
                ctx.convolve(img, psf, method=m, out=out)
                torch.cuda.synchronize()
                ctx.profile_enable(True)
                ms0, n0 = ctx.profile_read("conv")
                for _ in range(reps):
                    ctx.convolve(img, psf, method=m, out=out)
                torch.cuda.synchronize()
                ms1, n1 = ctx.profile_read("conv")
                ctx.profile_enable(False)
                us[name] = round(1e3 * (ms1 - ms0) / (n1 - n0), 2)
            rows.append({"n": n, "k": k, "direct_us": us["direct"], "fft_us": us["fft"],
                         "direct_tflops": round(2.0 * n * n * k * k / us["direct"] / 1e6, 2),
                         "auto": {1: "direct", 2: "fft"}[convolve_auto_method(n, n, k)]})
    return rows


def large_image_bench(ctx, reps):
    """One 1000x1000 px image at s = 5 with 50,000 NFW subhalos, four Sersic
    components and a 101x101 PSF (the largest workload)."""
    import numpy as np
    import torch
    import workloads as W
    sc = W.config5_scene()
    g = sc.grid
    nfw = sc.lens.nfw
    dev_nfw = W.NFWTable(*[torch.from_numpy(np.asarray(a)).cuda() for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)])
    lens = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear, nfw=dev_nfw)
    psf = torch.from_numpy(sc.psf).cuda()
    out = torch.empty((g.ny, g.nx), dtype=torch.float32, device="cuda")
    step = lambda: ctx.simulate_image(g, lens, sc.source, sc.lens_light, psf, sc.bn_exact, out=out)
    step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    base = {k: ctx.profile_read(k) for k in ("sim", "conv")}
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    per = {}
    for k in ("sim", "conv"):
        ms, n = ctx.profile_read(k)
        per[k] = (ms - base[k][0]) / max(n - base[k][1], 1)
    ctx.profile_enable(False)
    pairs = g.nx * g.ny * g.supersample ** 2 * nfw.n
    achieved = FLOP_PER_PAIR * pairs / (1e-3 * per["sim"]) / 1e12
    return {"workload": "1000x1000 px at 0.11\"/px, s=5, SIE + shear + 50000 NFW, 1 lens-light + 3 source Sersic, "
                        "101x101 PSF (seed 1005)",
            "reps": reps, "ms_per_image": round(1e3 * wall, 2), "simulate_ms": round(per["sim"], 2),
            "convolve_ms": round(per["conv"], 3), "pairs": pairs,
            "pairs_per_s": round(pairs / (1e-3 * per["sim"]), 1),
            "simulate_frac_fp32_peak": round(achieved / PEAK_FP32_TFLOPS, 4)}


def _kernel_ms(ctx, fn, kernels, reps):
    """Average library-event time per launch of `kernels` over `reps` calls of
    fn, and the wall time per call."""
    import torch
    fn()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    base = {k: ctx.profile_read(k) for k in kernels}
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    per = {}
    for k in kernels:
        ms, n = ctx.profile_read(k)
        per[k] = (ms - base[k][0]) / max(n - base[k][1], 1)
    ctx.profile_enable(False)
    return per, wall


def profiles_bench(ctx, reps=20):
    """The profile-dispatch rows: (a) each main-deflector profile alone on a
    180x180 grid (the paper's deflection table), kernel time per call; (b) the
    headline image with an elliptical power-law main deflector, and with
    truncated subhalos, as images/s and (sub-pixel, subhalo) pairs/s."""
    import numpy as np
    import torch
    import workloads as W
    g = np.arange(180, dtype=np.float64) * 0.05 - 0.05 * 89.5
    gx, gy = np.meshgrid(g, g)
    x = torch.from_numpy(gx.astype(np.float32).ravel()).cuda()
    y = torch.from_numpy(gy.astype(np.float32).ravel()).cuda()
    ox, oy = torch.empty_like(x), torch.empty_like(y)
    rng = np.random.default_rng(2024)
    one = lambda **kw: W.NFWTable(*[torch.from_numpy(np.asarray(v, np.float32)).cuda()
                                    for v in ([0.3], [-0.2], [0.25], [0.02])], **kw)
    cases = {
        "SIE": W.Lens(sie=W.SIE(1.2, 0.7, 0.4, 0.0, 0.0)),
        "EPL": W.Lens(epl=W.EPL(1.2, 2.1, 0.7, 0.4, 0.0, 0.0)),
        "SHEAR": W.Lens(shear=W.Shear(0.03, -0.02)),
        "NFW": W.Lens(nfw=one()),
        "TNFW": W.Lens(nfw=one(r_trunc=torch.tensor([2.5], device="cuda"))),
    }
    table = {}
    for name, lens in cases.items():
        per, _ = _kernel_ms(ctx, lambda: ctx.deflection(x, y, lens, out=(ox, oy)), ("ray",), reps)
        table[name] = round(1e3 * per["ray"], 2)
    gs = [W.Gaussian(1.0 + k, 0.1 + 0.05 * k, 1.0, 0.0, 0.0, 0.0) for k in range(5)]
    ge = [W.Gaussian(1.0 + k, 0.1 + 0.05 * k, 0.7, 0.4, 0.0, 0.0) for k in range(5)]
    coef = lambda n: rng.normal(0, 1, (n + 1) * (n + 2) // 2)
    lights = {
        "GAUSSIAN": [gs[0]], "GAUSSIAN_ELLIPSE": [ge[0]], "MULTI_GAUSSIAN (5)": gs, "MULTI_GAUSSIAN_ELLIPSE (5)": ge,
        "SERSIC": [W.Sersic(1.0, 0.5, 3.0, 1.0, 0.0, 0.0, 0.0)], "SERSIC_ELLIPSE": [W.Sersic(1.0, 0.5, 3.0, 0.7, 0.4, 0.0, 0.0)],
        "CORE_SERSIC": [W.CoreSersic(1.0, 0.5, 0.05, 3.0, 0.3, 3.0, 0.7, 0.4, 0.0, 0.0)],
        "SHAPELETS (n_max=6)": [W.Shapelets(6, 0.2, 0.0, 0.0, coef(6))],
        "SHAPELETS (n_max=10)": [W.Shapelets(10, 0.2, 0.0, 0.0, coef(10))],
    }
    sb = torch.empty_like(x)
    light = {}
    for name, comps in lights.items():
        per, _ = _kernel_ms(ctx, lambda: ctx.source_sb(x, y, x, y, comps, [], out=sb), ("sb",), reps)
        light[name] = round(1e3 * per["sb"], 2)
    images = {}
    for name, sc in (("EPL main deflector", W.epl_scene()), ("TNFW subhalos", W.tnfw_scene())):
        gr = sc.grid
        nfw = sc.lens.nfw
        cols = [nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs]
        dev = [torch.from_numpy(np.asarray(a)).cuda() for a in cols]
        rt = torch.from_numpy(np.asarray(nfw.r_trunc)).cuda() if nfw.r_trunc is not None else None
        lens = W.Lens(sie=sc.lens.sie, epl=sc.lens.epl, shear=sc.lens.shear, nfw=W.NFWTable(*dev, r_trunc=rt))
        psf = torch.from_numpy(sc.psf).cuda()
        out = torch.empty((gr.ny, gr.nx), dtype=torch.float32, device="cuda")
        per, wall = _kernel_ms(ctx, lambda: ctx.simulate_image(gr, lens, sc.source, sc.lens_light, psf, sc.bn_exact,
                                                               out=out), ("sim", "conv", "prep"), reps)
        pairs = gr.nx * gr.ny * gr.supersample ** 2 * nfw.n
        images[name] = {"images_per_s": round(1.0 / wall, 2), "simulate_ms": round(per["sim"], 4),
                        "convolve_ms": round(per["conv"], 4), "prep_ms": round(per["prep"], 4),
                        "pairs_per_s": round(pairs / (1e-3 * per["sim"]), 1)}
    return {"deflection_180x180_us": table, "light_180x180_us": light,
            "deflection_workload": "32,400 points of a 180x180 grid at 0.05\"/px; one deflector of each profile",
            "images": images,
            "images_workload": ("200x200 px, s = 3, shear + 10,000 subhalos, 1 lens-light + 2 source Sersic, "
                                "41x41 PSF: EPL (gamma in [1.8, 2.2]) + NFW (seed 1006); SIE + TNFW with "
                                "tau = r_trunc/Rs log-uniform in [3, 30] (seed 1007)")}


def stages_bench(ctx, reps=10):
    """The three steps as separate calls, with their algorithmic bytes or
    pairs: step 1 (jt_ray_shoot) and step 2 (jt_source_sb) streaming over the
    1000x1000 px, s = 5 image's 25 million sub-pixels (macro lens only for
    step 1, the image's four Sersic components for step 2), and step 1 with
    the headline's 10,000 NFW at its 360,000 sub-pixels.  Kernel time from
    the library's HIP events."""
    import numpy as np
    import torch
    import workloads as W
    out = {}
    sc = W.config5_scene()
    g = sc.grid
    n1 = g.nx * g.supersample
    d = g.pixel_scale / g.supersample
    ax = (torch.arange(n1, device="cuda", dtype=torch.float64) - 0.5 * (n1 - 1)) * d
    yy, xx = torch.meshgrid(ax, ax, indexing="ij")
    x, y = xx.float().contiguous().view(-1), yy.float().contiguous().view(-1)
    del xx, yy
    n = x.numel()
    bx, by = torch.empty_like(x), torch.empty_like(y)
    macro = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear)
    per, _ = _kernel_ms(ctx, lambda: ctx.ray_shoot(x, y, macro, out=(bx, by)), ("ray",), reps)
    t = 1e-3 * per["ray"]
    out["ray_shoot_macro"] = {"points": n, "us": round(1e6 * t, 1), "bytes_per_point": 16,
                              "GB_per_s": round(16 * n / t / 1e9, 1),
                              "frac_hbm_peak": round(16 * n / t / PEAK_HBM_BYTES, 4),
                              "note": "SIE + shear in FP64 per point (atan/atanh): FP64 VALU work beside 16 B of HBM"}
    sb = torch.empty_like(x)
    per, _ = _kernel_ms(ctx, lambda: ctx.source_sb(x, y, bx, by, sc.source, sc.lens_light, sc.bn_exact, out=sb),
                        ("sb",), reps)
    t = 1e-3 * per["sb"]
    out["source_sb"] = {"points": n, "components": len(sc.source) + len(sc.lens_light), "us": round(1e6 * t, 1),
                        "bytes_per_point": 20, "GB_per_s": round(20 * n / t / 1e9, 1),
                        "frac_hbm_peak": round(20 * n / t / PEAK_HBM_BYTES, 4)}
    del x, y, bx, by, sb
    sc2 = W.config2_scene()
    g2 = sc2.grid
    m = g2.nx * g2.supersample
    d2 = g2.pixel_scale / g2.supersample
    ax2 = (torch.arange(m, device="cuda", dtype=torch.float64) - 0.5 * (m - 1)) * d2
    yy, xx = torch.meshgrid(ax2, ax2, indexing="ij")
    x, y = xx.float().contiguous().view(-1), yy.float().contiguous().view(-1)
    bx, by = torch.empty_like(x), torch.empty_like(y)
    nfw = sc2.lens.nfw
    dev = W.NFWTable(*[torch.from_numpy(np.asarray(a)).cuda() for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)])
    lens = W.Lens(sie=sc2.lens.sie, shear=sc2.lens.shear, nfw=dev)
    per, _ = _kernel_ms(ctx, lambda: ctx.ray_shoot(x, y, lens, out=(bx, by)), ("ray", "prep"), reps)
    t = 1e-3 * per["ray"]
    pairs = x.numel() * nfw.n
    out["ray_shoot_subhalos"] = {"points": x.numel(), "subhalos": nfw.n, "us": round(1e6 * t, 1),
                                 "pairs_per_s": round(pairs / t, 1),
                                 "frac_fp32_peak": round(FLOP_PER_PAIR * pairs / t / 1e12 / PEAK_FP32_TFLOPS, 4)}
    out["workload"] = ("steps 1 and 2 alone on the 1000x1000 px, s = 5 image's 5000x5000 sub-pixel grid "
                       "(seed 1005); step 1 with the headline's 10,000 NFW on its 600x600 sub-pixels (seed 1002)")
    return out


def linear_bench(ctx, reps=20):
    """The linear amplitude solver on the headline image (four components:
    the two sources, a third added source and the lens light) against
    seeded noisy data: wall time per call, and the basis, convolution and
    plain-image kernel times."""
    import numpy as np
    import torch
    import workloads as W
    sc = W.config2_scene()
    sc.source.append(W.Sersic(amp=3.0, R_sersic=0.25, n_sersic=1.2, q=0.8, phi=1.1, cx=-0.15, cy=0.1))
    g = sc.grid
    nfw = sc.lens.nfw
    dev = W.NFWTable(*[torch.from_numpy(np.asarray(a)).cuda() for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)])
    lens = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear, nfw=dev)
    psf = torch.from_numpy(sc.psf).cuda()
    img = ctx.simulate_image(g, lens, sc.source, sc.lens_light, psf, sc.bn_exact)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    m = img.cpu().numpy().astype(np.float64)
    d = rng.poisson(1000.0 * np.maximum(m, 0.0)) / 1000.0 + rng.normal(0.0, 0.01, m.shape)
    data = torch.from_numpy(d.astype(np.float32)).cuda()
    w = 1.0 / (0.01 ** 2 + torch.clamp(data, min=0.0) / 1000.0)
    model = torch.empty_like(data)
    fn = lambda: ctx.linear_amplitudes(g, lens, sc.source, sc.lens_light, data, w, psf=psf, bn_exact=sc.bn_exact)
    per, wall = _kernel_ms(ctx, fn, ("sim", "conv", "prep"), reps)
    amps, _, logL = fn()
    torch.cuda.synchronize()
    return {"workload": "headline image with 4 light components (3 sources + lens light), seeded noisy data",
            "ms_per_solve": round(1e3 * wall, 4), "basis_kernel_ms": round(per["sim"], 4),
            "convolution_ms": round(per["conv"], 4), "amplitudes": [round(float(a), 6) for a in amps.cpu()],
            "true_amplitudes": [c.amp for c in sc.source] + [c.amp for c in sc.lens_light],
            "logL": float(logL.cpu()[0])}


def fitting_bench(ctx, steps=20):
    """The paper's swarm-fitting case without its point source: 100x100 px
    (0.05"/px), 13x13 PSF, SIE + shear, an elliptical Sersic source and lens
    light (21 parameters), seeded noisy data.  Swarm steps for 64..512
    particles (wall time per step: one batched likelihood launch plus the
    host update), and L-BFGS from 8 starts at once."""
    import numpy as np
    import torch
    import workloads as W
    rng = np.random.default_rng(2025)
    sc = W.config1_scene(draw=7)
    sc.grid = W.Grid(nx=100, ny=100, pixel_scale=0.05, supersample=1)
    sc.lens_light = [W.Sersic(amp=5.0, R_sersic=0.8, n_sersic=3.0, q=0.8, phi=0.5, cx=sc.lens.sie.cx,
                              cy=sc.lens.sie.cy)]
    sc.psf = W.gaussian_psf(13, 2.0)
    img = ctx.simulate_scene(sc)
    torch.cuda.synchronize()
    m = img.cpu().numpy().astype(np.float64)
    d = (rng.poisson(1000.0 * np.maximum(m, 0.0)) / 1000.0 + rng.normal(0.0, 0.01, m.shape)).astype(np.float32)
    w = (1.0 / (0.01 ** 2 + np.maximum(d, 0.0) / 1000.0)).astype(np.float32)
    data, inv_var = torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda()
    psf = torch.from_numpy(sc.psf).cuda()
    t = np.array([sc.lens.sie.theta_E, sc.lens.sie.q, sc.lens.sie.phi, sc.lens.sie.cx, sc.lens.sie.cy,
                  sc.lens.shear.gamma1, sc.lens.shear.gamma2] +
                 [v for c in sc.source + sc.lens_light for v in (c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy)])
    half = np.array([0.2, 0.2, 0.5, 0.1, 0.1, 0.05, 0.05] + [0.5 * t[7], 0.5 * t[8], 1.0, 0.2, 0.5, 0.1, 0.1] +
                    [0.5 * t[14], 0.5 * t[15], 1.0, 0.2, 0.5, 0.1, 0.1])
    lo, hi = t - half, t + half
    for i in (1, 10, 17):
        lo[i], hi[i] = max(lo[i], 0.3), min(hi[i], 1.0)
    for i in (9, 16):
        lo[i] = max(lo[i], 0.5)
    swarm = []
    for N in (64, 128, 256, 512):
        ctx.pso(sc.grid, 1, 1, lo, hi, data, inv_var, psf=psf, n_particles=N, n_iterations=2, seed=1)
        t0 = time.perf_counter()
        best, bl, hist = ctx.pso(sc.grid, 1, 1, lo, hi, data, inv_var, psf=psf, n_particles=N, n_iterations=steps,
                                 seed=1)
        wall = time.perf_counter() - t0
        swarm.append({"particles": N, "steps": steps, "ms_per_step": round(1e3 * wall / (steps + 1), 3),
                      "us_per_particle_evaluation": round(1e6 * wall / ((steps + 1) * N), 3),
                      "best_logL": round(float(bl), 3)})
    starts = t + half * rng.uniform(-0.5, 0.5, (8, t.size))
    starts = np.clip(starts, lo, hi)
    t0 = time.perf_counter()
    x, ll, its = ctx.lbfgs(sc.grid, 1, 1, lo, hi, data, inv_var, starts, psf=psf, max_iter=300)
    wall = time.perf_counter() - t0
    return {"workload": "100x100 px at 0.05\"/px, 13x13 PSF, SIE + shear + Sersic source + Sersic lens light "
                        "(21 parameters), seeded noisy data; no point source",
            "pso": swarm,
            "lbfgs": {"starts": 8, "seconds": round(wall, 3), "iterations": [int(i) for i in its],
                      "best_logL": round(float(ll.max()), 3), "logL_at_truth_params_note":
                      "the data are noisy, so the optimum lies near, not at, the generating parameters"}}


def adjoint_bench(ctx, draws, reps):
    """Gradient of the chi^2 log-likelihood for a batch of parameter draws
    (100x100 px, 1000 NFW, 21x21 PSF) against the forward alone and the plain
    per-image path."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_01547_amd.grad import DrawBatch, macro_row
    truth, scenes = W.config4_draws(B=draws)
    macro = np.stack([macro_row(s.lens, s.source, s.lens_light) for s in scenes])
    st = lambda a: torch.from_numpy(np.stack([getattr(s.lens.nfw, a) for s in scenes])).cuda()
    batch = DrawBatch(macro, 1, 0, st("x"), st("y"), st("Rs"), st("alpha_Rs"))
    m = ctx.simulate_scene(truth)
    torch.cuda.synchronize()
    d = W.noisy_image(m.cpu().numpy(), seed=1)
    w = (1.0 / (0.01 ** 2 + np.maximum(d, 0) / 1000.0)).astype(np.float32)
    dt, wt, psf = torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(truth.psf).cuda()

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_grad = timeit(lambda: ctx.chi2_grad(truth.grid, batch, dt, wt, psf))
    t_kept = timeit(lambda: ctx.chi2_grad(truth.grid, batch, dt, wt, psf, keep_positions=True))
    t_fwd = timeit(lambda: ctx.chi2(truth.grid, batch, dt, wt, psf))
    out = torch.empty((truth.grid.ny, truth.grid.nx), dtype=torch.float32, device="cuda")
    # the per-image path with its inputs resident too: each draw's subhalo SoA
    # and the PSF on the device before the timed region, one call per draw
    resident = []
    for sc in scenes:
        nfw = sc.lens.nfw
        dev = W.NFWTable(*[torch.from_numpy(np.asarray(a)).cuda() for a in (nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs)])
        resident.append((W.Lens(sie=sc.lens.sie, shear=sc.lens.shear, nfw=dev), sc.source, sc.lens_light))
    torch.cuda.synchronize()

    def per_image():
        for lens, src, ll in resident:
            ctx.simulate_image(truth.grid, lens, src, ll, psf, out=out)
    t_pi = timeit(per_image)
    # the same case with an EPL main deflector and truncated subhalos
    truth_p, scenes_p = W.config4_profile_draws(B=draws, n_sub=scenes[0].lens.nfw.n, grid=truth.grid, epl=True,
                                                tnfw=True, psf_size=21)
    macro_p = np.stack([macro_row(s.lens, s.source, s.lens_light) for s in scenes_p])
    stp = lambda a: torch.from_numpy(np.stack([getattr(s.lens.nfw, a) for s in scenes_p])).cuda()
    batch_p = DrawBatch(macro_p, 1, 0, stp("x"), stp("y"), stp("Rs"), stp("alpha_Rs"), main="epl",
                        sub_r_trunc=stp("r_trunc"))
    t_grad_p = timeit(lambda: ctx.chi2_grad(truth.grid, batch_p, dt, wt, psf))
    t_fwd_p = timeit(lambda: ctx.chi2(truth.grid, batch_p, dt, wt, psf))
    return {"workload": f"{draws} draws of 100x100 px, s=1, SIE + shear + 1000 NFW, 1 source, 21x21 PSF",
            "gradient_ms_per_batch": round(1e3 * t_grad, 3), "forward_ms_per_batch": round(1e3 * t_fwd, 3),
            "per_image_forward_ms_per_batch": round(1e3 * t_pi, 3),
            "per_image_path": "one jt_simulate_image call per draw, subhalo SoA and PSF resident on the device",
            "gradients_per_s": round(draws / t_grad, 1), "adjoint_over_forward": round(t_grad / t_fwd, 3),
            "kept_positions_gradient_ms_per_batch": round(1e3 * t_kept, 3),
            "kept_positions_over_forward": round(t_kept / t_fwd, 3),
            "params_per_draw": int(macro.shape[1] + 3 * scenes[0].lens.nfw.n),
            "epl_tnfw": {"workload": "the same draws with an EPL main deflector (slope 1.9 +- 1%) and truncated "
                                     "subhalos (tau log-uniform in [3, 30])",
                         "gradient_ms_per_batch": round(1e3 * t_grad_p, 3),
                         "forward_ms_per_batch": round(1e3 * t_fwd_p, 3),
                         "params_per_draw": int(macro_p.shape[1] + 3 * scenes_p[0].lens.nfw.n)}}


# Lane-operations per round of each calibration kind (jt_calibrate_valu) and
# FLOP per lane-operation (FMA = 2).
CALIB_KINDS = {0: ("fma", 8, 2.0), 1: ("rsq", 8, 1.0), 2: ("16 fma + 2 rsq", 18, 34.0 / 18.0),
               3: ("mul", 16, 1.0), 4: ("fma with literal", 8, 2.0), 5: ("log + add", 16, 1.0),
               6: ("fmac, sgpr operand", 8, 2.0), 7: ("fma, three vgprs", 8, 2.0)}
CLOCK_HZ = 2.4e9   # MI355X peak engine clock (published)
N_CU = 256


def valu_calibration(iters):
    """FP32 issue rates measured by the library's calibration kernels: for
    each instruction class and 1, 2, 4, 8 waves per SIMD, lane-operations per
    second, per CU per clock (at the published 2.4 GHz) and the implied SIMD
    cycles per wave64 instruction."""
    from paper_2606_01547_amd import Context
    ctx = Context(0)
    rows = []
    for kind, (name, ops, flop_per_op) in CALIB_KINDS.items():
        for waves in (1, 2, 4, 8):
            blocks = N_CU * waves              # 4 waves per block, 4 SIMDs per CU
            ms = ctx.calibrate_valu(kind, blocks, iters)
            lane_ops = blocks * 256.0 * iters * ops
            rate = lane_ops / (1e-3 * ms)
            per_cu_clk = rate / (N_CU * CLOCK_HZ)
            rows.append({"kind": kind, "class": name, "waves_per_simd": waves, "ms": round(ms, 4),
                         "lane_ops_per_s": float(f"{rate:.4g}"), "lane_ops_per_cu_clock": round(per_cu_clk, 2),
                         "simd_cycles_per_wave_instruction": round(4 * 64 / per_cu_clk, 3),
                         "fp32_tflops": round(rate * flop_per_op / 1e12, 2)})
    ctx.close()
    return {"valu_calibration": rows, "iters": iters, "clock_hz": CLOCK_HZ, "cus": N_CU,
            "note": "lane_ops_per_cu_clock assumes the published 2.4 GHz; rates are measured"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-samples", type=int, default=200)
    ap.add_argument("--cpu-rows", type=int, default=30, help="pixel rows of the oracle sample (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle processes of the pooled baseline")
    ap.add_argument("--serve-requests", type=int, default=4096, help="serving stream length (0 = skip)")
    ap.add_argument("--serve-large-every", type=int, default=512,
                    help="every n-th request is a large 1000x1000 image (0 = none)")
    ap.add_argument("--adjoint-draws", type=int, default=256, help="parameter draws per gradient (0 = skip)")
    ap.add_argument("--large-reps", type=int, default=3, help="timed 1000^2-px images (0 = skip)")
    ap.add_argument("--conv-sweep", type=int, default=1, help="direct/FFT convolution sweep (0 = skip)")
    ap.add_argument("--profiles", type=int, default=1, help="EPL / TNFW profile rows (0 = skip)")
    ap.add_argument("--linear", type=int, default=1, help="linear amplitude solver row (0 = skip)")
    ap.add_argument("--stages", type=int, default=1, help="steps 1 and 2 as separate calls (0 = skip)")
    ap.add_argument("--fitting", type=int, default=1, help="swarm and L-BFGS fitting row (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times), to calibrate "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--valu-calibration", type=int, default=0, metavar="ITERS",
                    help="only run the FP32 issue-rate calibration kernels (ITERS rounds per lane) at 1, 2, 4 "
                         "and 8 waves per SIMD and print their rates")
    args = ap.parse_args()
    if args.valu_calibration:
        print(json.dumps(valu_calibration(args.valu_calibration)), flush=True)
        return
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
    cnt = counters()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": cnt.get("bytes_per_launch"),
                "kernel": "k_simulate", "avg_ms": round(1e3 * sim_avg_s, 4),
                "flop_per_launch": FLOP_PER_PAIR * pairs, "flop_per_pair": FLOP_PER_PAIR,
                "pairs_per_s": round(pairs / sim_avg_s, 1)}
    if cnt.get("executed_flop_per_pair"):
        ex = cnt["executed_flop_per_pair"] * pairs / sim_avg_s / 1e12
        roofline["executed_flop_per_pair"] = cnt["executed_flop_per_pair"]
        roofline["executed_frac"] = round(ex / PEAK_FP32_TFLOPS, 4)

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
    if args.conv_sweep:
        result["conv_sweep"] = conv_sweep(ctx)
    if args.large_reps > 0:
        result["large_image"] = large_image_bench(ctx, args.large_reps)
    if args.profiles:
        result["profiles"] = profiles_bench(ctx)
    if args.stages:
        result["stages"] = stages_bench(ctx)
    if args.linear:
        result["linear_amplitudes"] = linear_bench(ctx)
    if args.fitting:
        result["fitting"] = fitting_bench(ctx)
    if args.adjoint_draws > 0:
        result["adjoint"] = adjoint_bench(ctx, args.adjoint_draws, reps=10)
    if args.serve_requests > 0:
        result["serving"] = serving_bench(ctx, args.serve_requests, args.serve_large_every)
    if args.cpu_rows > 0:
        result["cpu_baseline"] = cpu_baseline(scene, args.cpu_rows, args.cpu_workers)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
