#!/usr/bin/env python
"""Benchmark of the ILS hot path on one MI355X.

A step is one full ILS smoothing (Algorithm 1, N = 4 iterations:
2N + 1 = 9 fused passes) of one 1920 x 1080 RGB float32 frame
(lambda = 1, p = 0.8, eps = 1e-4), the frames taken in turn from a ring of
distinct seeded synthetic frames that are resident in HBM before timing
starts (the ring is larger than the 256 MB last-level cache).

Prints one JSON line with throughput (Mpixel/s, an RGB pixel counted once),
fps, the roofline of the dominant kernel (per-launch durations from HIP
events on the library's stream, algorithmic bytes per launch), the FP64
oracle timed on the host cores, and secondary figures (hot single frame,
batched frames).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s and fps at 1080p RGB N=4 (FP32 ILS vs surrogate), HBM GB/s % peak"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one non-packed VALU instruction per lane per clock
VALU_PEAK_TLANE = round(256 * 4 * 16 * 2.4e9 / 1e12, 2)
PAPER_1080P_RGB_MPX_S = 1920 * 1080 * 20 / 1e6  # 20 fps on a GTX 1080 (paper's GPU timing table)


def pass_bytes(H, W, C):
    """Algorithmic HBM bytes of each pass kind for one frame (all channels)."""
    img = C * H * W * 4
    spec = C * H * (W // 2 + 1) * 8
    return {"row_first": img + spec, "row_mid": img + 2 * spec, "row_final": spec + img, "column": 2 * spec}


def step_bytes(H, W, C, N):
    b = pass_bytes(H, W, C)
    return b["row_first"] + (N - 1) * b["row_mid"] + N * b["column"] + b["row_final"]


def profile_entry(kernel, H, W, C):
    """Counter figures per launch measured with rocprofv3 (committed under
    profiles/), or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(f"{kernel}@{H}x{W}x{C}")
    from paper_2003_07504_amd.build import source_hash
    if not e or e.get("source_hash") != source_hash() or "bytes_per_launch" not in e:
        return None
    return e


def roofline_of(kernel, avg_us, alg_bytes, H, W, C):
    """Roofline of the dominant kernel against HBM: algorithmic bytes per
    launch (20N+4 model, per pass kind) / the kernel's average launch
    duration (events around a run of un-bracketed launches) / 8 TB/s.
    `traffic` is the measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy of known size) when the committed counter file was taken
    on the current kernel sources, else null.  The kernel's vector issue rate
    (SQ_INSTS_VALU x 64 lanes against 256 CUs x 64 lanes x 2.4 GHz, packed
    FP32 off) is reported beside it as `alu`."""
    ach = alg_bytes / (avg_us * 1e-6) / 1e9
    e = profile_entry(kernel, H, W, C)
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": e["bytes_per_launch"] if e else None,
           "kernel": kernel, "avg_launch_us": avg_us, "alg_bytes_per_launch": alg_bytes}
    valu = (e or {}).get("sq", {}).get("SQ_INSTS_VALU")
    if valu:
        lane = float(valu) * 64.0
        a = lane / (avg_us * 1e-6) / 1e12
        out["alu"] = {"achieved": round(a, 2), "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instr/s",
                      "frac": round(a / VALU_PEAK_TLANE, 4), "valu_lane_instr_per_launch": int(lane)}
    if e:
        out["traffic_read_write"] = [e.get("read_bytes"), e.get("write_bytes")]
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames_np, H, W, C, lam, p, eps, N, seconds):
    """The FP64 oracle (scipy.fft) on whole frames of the workload, first with
    all host threads (up to 16), then with one; about `seconds` each."""
    from oracle.ils import ils_channels

    def leg(workers, budget):
        t0 = time.perf_counter()
        done = 0
        while True:
            ils_channels(frames_np[done % len(frames_np)].astype("float64"), lam, p, eps, N, workers=workers)
            done += 1
            if time.perf_counter() - t0 >= budget:
                break
        el = time.perf_counter() - t0
        return done, el

    workers = min(16, os.cpu_count() or 1)
    done, el = leg(workers, seconds)
    d1, e1 = leg(1, seconds * 0.75)
    return {"value": round(done * H * W / el / 1e6, 4), "unit": "Mpixel/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} frame(s) of {W}x{H}x{C}, N={N}, FP64 NumPy/SciPy oracle (scipy.fft workers={workers})",
            "fps": round(done / el, 4), "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": round(d1 * H * W / e1 / 1e6, 4), "unit": "Mpixel/s", "cores": 1,
                              "sample": f"{d1} frame(s), scipy.fft workers=1", "fps": round(d1 / e1, 4)}}


def surrogate_gain(ring, H, W, weights, say):
    """Learned surrogate with the residual gate against plain ILS at
    N = 1..4 on the same frames (16 x 1080p RGB, per-frame lambda ~ U[0.5, 2],
    p ~ U[0.5, 1]): time per frame and PSNR against plain ILS N = 4."""
    import numpy as np
    import torch

    from paper_2003_07504_amd import ils, surrogate

    B = len(ring)
    rng = np.random.default_rng(3)
    lam = rng.uniform(0.5, 2.0, B).astype(np.float32)
    p = rng.uniform(0.5, 1.0, B).astype(np.float32)
    f = torch.stack(ring).contiguous()
    plan = ils.Plan(H, W, 3)
    z = np.load(weights, allow_pickle=False)
    tau = float(z["tau"])
    net = surrogate.Net(B, H, W, params=z["params"])

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps, out

    res = {"frames": B, "tau": tau, "plain": {}}
    refs = {}
    for N in (1, 2, 3, 4):
        outs = [torch.empty_like(ring[0]) for _ in range(B)]

        def run_plain(N=N, outs=outs):
            for b in range(B):
                plan.smooth(f[b], float(lam[b]), float(p[b]), 1e-4, N, out=outs[b])
            return outs
        t, o = timed(run_plain)
        refs[N] = torch.stack(o)
        res["plain"][f"N{N}"] = {"ms_per_frame": round(t * 1e3 / B, 4)}

    def psnr(a, b):
        mse = torch.mean((a - b) ** 2, dim=(1, 2, 3))
        return (10 * torch.log10(1.0 / mse)).cpu().numpy()

    for N in (1, 2, 3):
        res["plain"][f"N{N}"]["psnr_vs_N4_db"] = round(float(np.mean(psnr(refs[N], refs[4]))), 2)
    say("surrogate: network forward and gated inference")
    tnet, v = timed(lambda: net.forward(f, lam, p))
    tg, (out, r, fb) = timed(lambda: net.infer_gated(plan, f, lam, p, 1e-4, 4, tau), reps=2)
    ps_v = psnr(v, refs[4])
    # gated output: frames that fell back equal plain N = 4 exactly, so the
    # PSNR is taken over the mean squared error of the whole set
    mse_g = float(torch.mean((out - refs[4]) ** 2))
    passed = ~np.asarray(fb, dtype=bool)
    res["surrogate"] = {
        "network_ms_per_frame": round(tnet * 1e3 / B, 4),
        "gated_ms_per_frame": round(tg * 1e3 / B, 4),
        "psnr_vs_plain_N4_db_mean": round(float(np.mean(ps_v)), 2),
        "psnr_vs_plain_N4_db_min": round(float(np.min(ps_v)), 2),
        "gated_psnr_vs_plain_N4_db_of_mean_mse": (round(10 * float(np.log10(1.0 / mse_g)), 2) if mse_g > 0 else None),
        "psnr_of_frames_passing_gate_db_min": (round(float(np.min(ps_v[passed])), 2) if passed.any() else None),
        "fallback_rate": round(float(np.mean(fb)), 4),
        "residual_median": float(np.median(r)),
        "weights_step": int(z["step"]),
    }
    res["gain_vs_plain_N4"] = round(res["plain"]["N4"]["ms_per_frame"] / res["surrogate"]["gated_ms_per_frame"], 3)
    # like for like with batches: plain N = 4 as one 16-frame batched call
    # against gated inference whose T(v) and fallback are batched calls too
    say("surrogate: batched plain ILS and batched gated inference")
    plan_b = ils.Plan(H, W, 3, max_frames=B)
    outs_b = [torch.empty_like(ring[0]) for _ in range(B)]
    frames_b = [(f[b], float(lam[b]), float(p[b]), 1e-4, 4) for b in range(B)]
    tpb, _ = timed(lambda: plan_b.smooth_batch(frames_b, outs=outs_b))
    tgb, (out_b, _, fb_b) = timed(lambda: net.infer_gated(plan_b, f, lam, p, 1e-4, 4, tau), reps=2)
    torch.cuda.synchronize()
    if not torch.equal(out_b, out) or list(fb_b) != list(fb):
        raise RuntimeError("batched gated inference differs from the per-image one")
    res["batched"] = {"plain_N4_ms_per_frame": round(tpb * 1e3 / B, 4), "gated_ms_per_frame": round(tgb * 1e3 / B, 4),
                      "gain_vs_plain_N4": round(tpb / tgb, 3)}
    plan_b.close()
    net.close()
    plan.close()
    return res


def two_stream_figures(plan, plan2, s1, ring, outs, H, W, C, lam, p, eps, N, shapes, steps):
    """Frames alternate between two plans on two streams (default priority),
    so that one frame's passes can use the compute units the other frame's
    passes leave idle (pass tails, load and store phases).  Each frame still
    takes the whole path; only two are in flight.  s1 is created before any
    other stream of the process."""
    import torch

    plan2.set_shapes(H, W, C, shapes["row_shape"], shapes["col_shape"])
    outs2 = [torch.empty_like(f) for f in ring]
    torch.cuda.synchronize()

    def go(n):
        for i in range(n):
            j = i % len(ring)
            if i % 2 == 0:
                plan.smooth(ring[j], lam, p, eps, N, out=outs[j])
            else:
                with torch.cuda.stream(s1):
                    plan2.smooth(ring[j], lam, p, eps, N, out=outs2[j])

    go(32)
    torch.cuda.synchronize()
    a = time.perf_counter()
    go(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / steps
    if plan2.last_error() != 0:
        raise RuntimeError("HIP error in the two-stream figure")
    return {"ms_per_frame": round(dt * 1e3, 4), "fps": round(1 / dt, 1), "Mpixel_s": round(H * W / dt / 1e6, 1)}


def small_image_figures(say, reps=200):
    """256 x 256 grey, N = 4 (lambda = 1, p = 0.8): a latency-bound size.
    Per image: calls queued back to back, one-frame batched calls (enqueued
    directly: a batch of one part builds no graph), and a call followed by a
    stream synchronisation.  Also one grey
    1080p frame per call (a third of the RGB work on the same grid shape)."""
    import torch

    from paper_2003_07504_amd import ils
    from synth import voronoi_image

    f = torch.from_numpy(voronoi_image(256, 256, 1, 40, 0.05, seed=0)).cuda()
    out = torch.empty_like(f)
    plan = ils.Plan(256, 256, 1)
    res = {}

    def timeit(fn, sync_each=False):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
            if sync_each:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps * 1e6

    res["queued_us_per_image"] = round(timeit(lambda: plan.smooth(f, 1.0, 0.8, 1e-4, 4, out=out)), 2)
    res["batch_of_1_us_per_image"] = round(timeit(
        lambda: plan.smooth_batch([(f, 1.0, 0.8, 1e-4, 4)], outs=[out])), 2)
    res["synchronous_us_per_call"] = round(timeit(lambda: plan.smooth(f, 1.0, 0.8, 1e-4, 4, out=out), True), 2)
    plan.close()
    g = torch.from_numpy(voronoi_image(1080, 1920, 1, 400, 0.05, seed=1)).cuda()
    og = torch.empty_like(g)
    pg = ils.Plan(1080, 1920, 1)
    t = timeit(lambda: pg.smooth(g, 1.0, 0.8, 1e-4, 4, out=og)) * 1e-6
    res["grey_1080p_n4_Mpixel_s"] = round(1920 * 1080 / t / 1e6, 1)
    res["grey_1080p_tile_shapes"] = pg.tune(1080, 1920, 1)
    pg.close()
    say(f"256x256 grey N=4: {res}")
    return res


def convergence_figures(ring, say, n_max=30):
    """Energy of Eq. (1) along the iteration on one 1080p RGB frame (device
    energy kernel, iterations one at a time from the previous iterate): the
    share of the N = n_max energy decrease reached at N = 1, 2, 4, 6, 10
    (the paper quotes 74-90 % at N = 4 and 81-96 % at N = 6 on photographs)."""
    import torch

    from paper_2003_07504_amd import ils

    f = ring[0]
    C, H, W = f.shape
    plan = ils.Plan(H, W, C)
    u = f.clone()
    nxt = torch.empty_like(f)
    energies = [float(plan.energy(f, u, 1.0, 0.8, 1e-4).cpu())]
    for _ in range(n_max):
        plan.iterate_from(f, u, 1.0, 0.8, 1e-4, 1, out=nxt)
        u, nxt = nxt, u
        energies.append(float(plan.energy(f, u, 1.0, 0.8, 1e-4).cpu()))
    plan.close()
    total = energies[0] - energies[-1]
    res = {"lambda": 1.0, "p": 0.8, "E0": energies[0], f"E{n_max}": energies[-1],
           "share_of_decrease": {f"N{n}": round((energies[0] - energies[n]) / total, 4) for n in (1, 2, 4, 6, 10)},
           "monotone": all(b <= a for a, b in zip(energies, energies[1:]))}
    say(f"convergence: {res['share_of_decrease']}")
    return res


def convergence_sweeps(ring, say, n_max=30):
    """Energy-decrease trends of Sec. 3.2 and Sec. 3.3.4 on one channel of a
    1080p frame (device energy kernel, iterations one at a time): for
    lambda in {0.1, 0.5, 1, 5, 10} x p in {0.2, 0.5, 0.8, 1} (eps = 1e-4) and
    for eps in {1e-2, 1e-4, 1e-5} (lambda = 1, p = 0.8), the share of the
    N = n_max energy decrease reached at N = 1, 2, 4, 6, 10, and whether the
    energy decreased at every iteration."""
    import torch

    from paper_2003_07504_amd import ils

    f = ring[0][:1].contiguous()
    C, H, W = f.shape
    plan = ils.Plan(H, W, C)

    def curve(lam, p, eps):
        u = f.clone()
        nxt = torch.empty_like(f)
        es = [plan.energy(f, u, lam, p, eps)]
        for _ in range(n_max):
            plan.iterate_from(f, u, lam, p, eps, 1, out=nxt)
            u, nxt = nxt, u
            es.append(plan.energy(f, u, lam, p, eps))
        es = [float(e) for e in torch.stack(es).cpu()]
        total = es[0] - es[-1]
        share = {f"N{n}": round((es[0] - es[n]) / total, 4) if total > 0 else None for n in (1, 2, 4, 6, 10)}
        return {"share_of_decrease": share, "monotone": all(b <= a * (1 + 1e-12) for a, b in zip(es, es[1:])),
                "E_ratio_N30": round(es[-1] / es[0], 5)}

    grid = {}
    for lam in (0.1, 0.5, 1.0, 5.0, 10.0):
        for p in (0.2, 0.5, 0.8, 1.0):
            grid[f"lambda={lam},p={p}"] = curve(lam, p, 1e-4)
    eps_sweep = {f"eps={e:g}": curve(1.0, 0.8, e) for e in (1e-2, 1e-4, 1e-5)}
    plan.close()
    res = {"frame": f"1920x1080, channel 0 of ring frame 0, N up to {n_max}", "lambda_x_p": grid, "eps": eps_sweep}
    say(f"eps sweep share at N=1: { {k: v['share_of_decrease']['N1'] for k, v in eps_sweep.items()} }")
    return res


def batch_mix_figures(say, reps=3):
    """Uneven-size batch: 64 frames drawn from {640x480, 1280x720, 1920x1080,
    3840x2160} x {grey, RGB} with per-frame lambda ~ U[0.5, 2], p ~ U[0.5, 1],
    N = 4, smoothed by one ils_smooth_batch call (one graph replay).  One
    distinct image per (size, channels) class is generated and shared by the
    frames of that class (each frame keeps its own parameters and output)."""
    import torch

    from paper_2003_07504_amd import ils
    from synth import batch_mix, voronoi_image

    specs = batch_mix(n=64, seed=2)
    imgs = {}
    for s in specs:
        if (s.H, s.W, s.C) not in imgs:
            imgs[(s.H, s.W, s.C)] = torch.from_numpy(voronoi_image(s.H, s.W, s.C, s.K, s.sigma, s.seed)).cuda()
    frames = [(imgs[(s.H, s.W, s.C)], s.lam, s.p, s.eps, s.N) for s in specs]
    outs = [torch.empty_like(f[0]) for f in frames]
    pxch = sum(s.H * s.W * s.C for s in specs)
    px = sum(s.H * s.W for s in specs)
    nbytes = sum(step_bytes(s.H, s.W, s.C, s.N) for s in specs)
    from paper_2003_07504_amd._lib import IlsFrame, load
    arr = (IlsFrame * len(frames))()
    for i, (f, lam, p_, eps, N) in enumerate(frames):
        C, H, W = f.shape
        arr[i] = IlsFrame(f.data_ptr(), outs[i].data_ptr(), H, W, C, lam, p_, eps, N, 0)
    need = int(load().ils_batch_workspace_bytes(arr, len(frames)))
    plan = ils.Plan(2160, 3840, 3, max_frames=64, ws_bytes=need)
    plan.smooth_batch(frames, outs=outs)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        plan.smooth_batch(frames, outs=outs)
    torch.cuda.synchronize()
    t = (time.perf_counter() - a) / reps
    plan.close()
    return {"frames": len(specs), "Mpx_ch": round(pxch / 1e6, 1), "ms_per_batch": round(t * 1e3, 3),
            "fps": round(len(specs) / t, 1), "Mpixel_s": round(px / t / 1e6, 1),
            "alg_GBs": round(nbytes / t / 1e9, 1), "distinct_images": len(imgs)}


def stress_4k_figures(say, reps=2, distinct=8):
    """32 x 3840x2160 RGB frames (2000 cells, sigma 0.08), lambda = 2,
    p = 0.5, N = 10 in one batched call; `distinct` different frames cycled."""
    import torch

    from paper_2003_07504_amd import ils
    from synth import voronoi_image

    H, W, C, N = 2160, 3840, 3, 10
    base = [torch.from_numpy(voronoi_image(H, W, C, 2000, 0.08, seed=5000 + i)).cuda() for i in range(distinct)]
    frames = [(base[i % distinct], 2.0, 0.5, 1e-4, N) for i in range(32)]
    outs = [torch.empty_like(base[0]) for _ in range(32)]
    plan = ils.Plan(H, W, C, max_frames=32)  # 32 x 4K RGB spectra resident
    plan.smooth_batch(frames, outs=outs)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        plan.smooth_batch(frames, outs=outs)
    torch.cuda.synchronize()
    t = (time.perf_counter() - a) / reps
    plan.close()
    nbytes = 32 * step_bytes(H, W, C, N)
    return {"frames": 32, "N": N, "ms_per_batch": round(t * 1e3, 2), "fps": round(32 / t, 1),
            "alg_GBs": round(nbytes / t / 1e9, 1), "alg_frac_of_8TBs": round(nbytes / t / 8e12, 4),
            "distinct_frames": distinct}


def application_figures(ring, say, reps=32):
    """Per-frame time of the applications on the 1080p RGB ring (luminance-only
    smoothing, detail enhancement k = 3, HDR tone mapping of a synthetic
    radiance map) and of the Welsch-penalty smoother at
    the paper's clip-art (lambda 20, gamma 10/255, N 10) and texture (lambda 30,
    gamma 10/255, N 15) settings on the nearest compiled sizes."""
    import torch

    from paper_2003_07504_amd import ils
    from synth import clipart_image, texture_image

    def per_frame(fn, n):
        for i in range(2):
            fn(i)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i in range(n):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / n

    res = {}
    C, H, W = ring[0].shape
    plan = ils.Plan(H, W, C)
    out = torch.empty_like(ring[0])
    t = per_frame(lambda i: plan.smooth_luminance(ring[i % len(ring)], 1.0, 0.8, 1e-4, 4, 0.0, out=out), reps)
    res["luminance_only_1080p_rgb_n4"] = {"ms_per_frame": round(t * 1e3, 4), "Mpixel_s": round(H * W / t / 1e6, 1)}
    t = per_frame(lambda i: plan.detail_enhance(ring[i % len(ring)], 1.0, 0.8, 1e-4, 4, 3.0, out=out), reps)
    res["detail_enhance_k3_1080p_rgb_n4"] = {"ms_per_frame": round(t * 1e3, 4), "Mpixel_s": round(H * W / t / 1e6, 1)}
    from synth import hdr_image
    hdr = torch.from_numpy(hdr_image(H, W, K=400, seed=9)).cuda()
    t = per_frame(lambda i: plan.tone_map(hdr, 10.0, 1.0, 1e-4, 4, 100.0, 1.0, out=out), reps)
    res["tone_map_1080p_rgb_lambda10_p1_n4"] = {"ms_per_frame": round(t * 1e3, 4), "Mpixel_s": round(H * W / t / 1e6, 1)}
    plan.close()
    for name, (Hh, Ww, lam, gam, N, img) in {
            "welsch_clipart_540x1024_rgb_n10": (540, 1024, 20.0, 10 / 255, 10, clipart_image(540, 1024, 3, seed=7)),
            "welsch_texture_480x640_rgb_n15": (480, 640, 30.0, 10 / 255, 15, texture_image(480, 640, 3, seed=8))}.items():
        ft = torch.from_numpy(img).cuda()
        o = torch.empty_like(ft)
        pw = ils.Plan(Hh, Ww, 3)
        t = per_frame(lambda i: pw.smooth_welsch(ft, lam, gam, N, out=o), reps)
        res[name] = {"ms_per_frame": round(t * 1e3, 4), "fps": round(1 / t, 1)}
        pw.close()
    say(f"applications: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--ring", type=int, default=32, help="distinct frames cycled through")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the hot-frame, batched and surrogate figures")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one 512 MiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--small", action="store_true",
                    help="the 256x256 grey workload (40 Voronoi cells) in place of 1080p RGB, for profiling; "
                         "implies --no-extras and --no-cpu-baseline")
    ap.add_argument("--stress", action="store_true",
                    help="single 3840x2160 RGB frames of the stress workload (2000 cells, sigma 0.08, lambda 2, "
                         "p 0.5, N 10; ring of 8) in place of 1080p RGB, for profiling; implies --no-extras and "
                         "--no-cpu-baseline")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2003_07504_amd", "weights", "surrogate.npz"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the library runs on one GPU only "
              "(frames would shard across GPUs with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2003_07504_amd import ils
    from synth import voronoi_image

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    H, W, C, lam, p, eps, N = 1080, 1920, 3, 1.0, 0.8, 1e-4, 4
    cells, sigma = 400, 0.05
    if args.small:
        H, W, C, cells = 256, 256, 1, 40
        args.no_extras = args.no_cpu_baseline = True
    if args.stress:
        H, W, C, lam, p, N, cells, sigma = 2160, 3840, 3, 2.0, 0.5, 10, 2000, 0.08
        args.ring = min(args.ring, 8)
        args.no_extras = args.no_cpu_baseline = True
    say(f"generating {args.ring} frames {W}x{H}x{C}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s1 = torch.cuda.Stream(device=dev)  # second stream of the two-stream figure, first of the process
    frames_np = [voronoi_image(H, W, C, cells, sigma, seed=1 + i) for i in range(args.ring)]
    ring = [torch.from_numpy(f).to(dev) for f in frames_np]
    outs = [torch.empty_like(f) for f in ring]
    plan = ils.Plan(H, W, C, max_frames=8)
    plan2 = ils.Plan(H, W, C)  # the two-stream figure's second plan
    torch.cuda.synchronize()

    def run(k0, k):
        for i in range(k0, k0 + k):
            j = i % len(ring)
            plan.smooth(ring[j], lam, p, eps, N, out=outs[j])

    say(f"warmup {args.warmup} steps")
    run(0, args.warmup)
    torch.cuda.synchronize()
    shapes = dict(zip(("row_shape", "col_shape"), plan.tune(H, W, C)))
    say(f"tile shapes chosen by the tuner: {shapes} of {ils.shape_variants(H, W)}")
    say(f"timed region {args.steps} steps")
    # ---- timed region
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    run(args.warmup, args.steps)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    host_s = t1 - t0
    gpu_ms = ev0.elapsed_time(ev1)
    if plan.last_error() != 0:
        raise RuntimeError("HIP error during the timed region")
    elapsed = max(host_s, gpu_ms / 1e3)
    ms_per_step = elapsed * 1e3 / args.steps
    mpx = args.steps * H * W / elapsed / 1e6
    fps = args.steps / elapsed

    # ---- median step time: one event before every step, >= 50 steps
    n_med = max(64, args.steps)
    say(f"median leg: {n_med} steps with an event before each")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_med + 1)]
    k0 = args.warmup + args.steps
    for i in range(n_med):
        evs[i].record()
        run(k0 + i, 1)
    evs[n_med].record()
    torch.cuda.synchronize()
    step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(n_med))
    median_ms = step_ms[n_med // 2]

    # ---- per-pass durations: a run of launches of one pass kind, back to
    # back on the plan's stream (f cycling through the ring as in the steps),
    # with one event pair around the run: no event between launches
    say("per-pass timing (runs of un-bracketed launches)")
    pb = pass_bytes(H, W, C)
    per_step = {"row_first": 1, "row_mid": N - 1, "row_final": 1, "column": N}
    reps = 64
    per_kind = {}
    for kind in ils.Plan.PASS_KINDS:
        for i in range(4):
            plan.enqueue_pass(kind, ring[i % len(ring)], lam, p, eps, out=outs[i % len(ring)])
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(reps):
            plan.enqueue_pass(kind, ring[i % len(ring)], lam, p, eps, out=outs[i % len(ring)])
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / reps
        per_kind[kind] = {"avg_us": round(us, 3), "launches_timed": reps, "per_step": per_step[kind],
                          "alg_bytes": pb[kind], "alg_GBs": round(pb[kind] / (us * 1e-6) / 1e9, 1)}
    if plan.last_error() != 0:
        raise RuntimeError("HIP error during pass timing")
    dom = max(per_kind, key=lambda k: per_kind[k]["avg_us"] * per_kind[k]["per_step"])
    dk = per_kind[dom]
    roofline = roofline_of(dom, dk["avg_us"], dk["alg_bytes"], H, W, C)
    step_alg = step_bytes(H, W, C, N)

    if args.copy_ref:  # a copy of known size, to scale the profiler's byte counters
        src = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    extras = {}
    if not args.no_extras:
        # first of the extras: the second stream's first launches come before
        # any batch graph has run (when they came after, the two streams ran
        # one after the other in some runs)
        say("two frames in flight on two streams")
        extras["two_streams_1080p_rgb_n4"] = two_stream_figures(plan, plan2, s1, ring, outs, H, W, C, lam, p, eps,
                                                                N, shapes, args.steps)
        say("hot single frame and batched figures")
        # hot: the same frame over and over (working set resident in the last-level cache)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            plan.smooth(ring[0], lam, p, eps, N, out=outs[0])
        torch.cuda.synchronize()
        hot = (time.perf_counter() - a) / args.steps
        extras["hot_single_frame"] = {"ms_per_frame": round(hot * 1e3, 4), "fps": round(1 / hot, 1),
                                      "Mpixel_s": round(H * W / hot / 1e6, 1)}
        # batched: 8 frames per ils_smooth_batch call
        nb = 8
        batches = max(1, args.steps // nb)
        frames = [(ring[j], lam, p, eps, N) for j in range(nb)]
        for _ in range(2):
            plan.smooth_batch(frames, outs=outs[:nb])
        torch.cuda.synchronize()
        a = time.perf_counter()
        for bi in range(batches):
            off = (bi * nb) % len(ring)
            idx = [(off + j) % len(ring) for j in range(nb)]
            plan.smooth_batch([(ring[j], lam, p, eps, N) for j in idx], outs=[outs[j] for j in idx])
        torch.cuda.synchronize()
        bt = (time.perf_counter() - a) / (batches * nb)
        extras["batched_8_frames"] = {"ms_per_frame": round(bt * 1e3, 4), "fps": round(1 / bt, 1),
                                      "Mpixel_s": round(H * W / bt / 1e6, 1)}
        say("uneven-size batch of 64 frames")
        extras["batch_mix_64"] = batch_mix_figures(say)
        say("energy along the iteration (1080p RGB, N up to 30)")
        extras["convergence_1080p_rgb"] = convergence_figures(ring, say)
        say("convergence sweeps: lambda x p grid and eps (one 1080p channel, N up to 30)")
        extras["convergence_sweeps"] = convergence_sweeps(ring, say)
        say("256x256 grey latency figures")
        extras["small_256x256_grey_n4"] = small_image_figures(say)
        say("applications (luminance mode, detail enhancement, Welsch penalty)")
        extras["applications"] = application_figures(ring, say)
        say("4K RGB N=10 stress batch of 32 frames")
        extras["stress_4k_n10_32"] = stress_4k_figures(say)
        if os.path.exists(args.weights):
            extras["surrogate_gain"] = surrogate_gain(ring, H, W, args.weights, say)

    cpu = None
    if not args.no_cpu_baseline:
        say(f"cpu baseline (oracle) for about {args.cpu_seconds} s")
        cpu = cpu_baseline(frames_np, H, W, C, lam, p, eps, N, args.cpu_seconds)

    line = {
        "metric": METRIC,
        "value": round(mpx, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(mpx / PAPER_1080P_RGB_MPX_S, 2) if (H, W, C) == (1080, 1920, 3) else None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ILS {W}x{H} {'RGB' if C == 3 else 'grey'} float32, N={N}, lambda={lam:g}, "
                               f"p={p:g}, eps=1e-4, one frame per step from a ring of {args.ring} distinct "
                               "Voronoi+Gaussian frames",
                   "H": H, "W": W, "C": C, "N": N, "lambda": lam, "p": p, "eps": eps,
                   "global_batch": 1, "parallelism": "none (1 GPU)"},
        "fps": round(fps, 1),
        "alg_GBs_whole_step": round(step_alg / (ms_per_step * 1e-3) / 1e9, 1),
        "alg_bytes_per_step": step_alg,
        "median_ms_per_step": round(median_ms, 5),
        "median_steps": n_med,
        "step_ms_p10_p90": [round(step_ms[n_med // 10], 5), round(step_ms[(9 * n_med) // 10], 5)],
        "host_s": round(host_s, 6),
        "gpu_event_ms": round(gpu_ms, 4),
        "roofline": roofline,
        "passes": per_kind,
        "tile_shapes": shapes,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
