#!/usr/bin/env python3
"""Benchmark of the LumiPath light-field path on one MI355X.

The timed step runs on the precision workload, the largest one a single GPU
holds: 512^3 u16 CT-like phantom (40 nested ellipsoids) in 8^3 bricks,
M = N = 32768 spherical-Fibonacci points (1.07B rays), 16 samples per ray,
8 bounces, HG g = 0.3, area light, 8^3 majorant grid:
  lf_points (SF table) -> lf_generate (FP32 light field, 12.9 GB) -> lf_lookup
  (32 views of 1920 x 1080, K = 5).
`value` = M*N*spp path samples per second of that step.  Next to it: the
same field stored as FP16 and BF16 (time, memory, error against the FP64
oracle on a seeded 1 % ray subset), the CT-like step with the adjoint
(256^3 phantom, N = 2048, 64 spp: generation keeping each sample's radiance,
lookup fused with an L2 loss gradient and its transpose, path-replay adjoint;
only rays the views reach carry an adjoint), and the dense adjoint of the
differentiation workload (128^3 f32, N = 1024, 32 spp: every ray carries an
adjoint, two replays per sample).  One JSON line on stdout; progress on
stderr.  Inputs are seeded synthetic data (lfsynth).
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of generation per tentative point (a delta-tracking
# collision or a ratio-tracking step): ~40 FP32 operations (position,
# trilinear interpolation, classification, accept or transmittance update),
# one Philox4x32-10 call (60 32-bit operations: 10 rounds of 2 wide
# multiplies and 4 xors) and one logarithm (4).  Peak: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz, one 32-bit lane operation per lane and clock.
OPS_POINT = 40 + 60 + 4
# Resident waves per SIMD of the forward tracer (lf_gen_params.waves_per_simd;
# results do not depend on it).  Four is the library's default and the faster
# choice on every workload measured but the precision workload, whose
# transfer function makes the tracer run HBM at ~77 % of its peak: there four
# waves' extra concurrent misses cost more than the latency they hide
# (4776 against 4530 ms per generation).
WAVES = {4: 3}
PEAK_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the code the generation kernel and its launch are built from
    (the kernel, its headers, the set-up kernels and the entry points), with
    comments and blank space removed so that editing a comment keeps a
    profile valid; the lookup and metric kernels are not part of it."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_03837_amd", "csrc")
    for f in ("api.cpp", "generate.hip", "internal.hpp", "sf_device.hpp", "tracer_device.hpp", "wave.hip"):
        text = open(os.path.join(csrc, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash, name):
    """HBM bytes per generation launch from a committed rocprofv3 PMC summary,
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def sweep_configs(configs, with_oracle=True, calib_copy_mb=0):
    """Generation on each workload c1..c5 at full size: throughput, work
    counts, error against the FP64 oracle on seeded ray samples, FP16/BF16
    storage error (c4), adjoint checks and timing (c5).  One JSON line per
    workload on stdout.  Without the oracle (counter runs) the error and
    oracle fields are left out."""
    import numpy as np
    import torch

    import lfsynth as S
    import paper_1903_03837_amd as lp

    dev = "cuda"
    if with_oracle:
        # the CPU baseline and error reference of each workload
        from oracle import oracle as orc
        threads = orc.default_threads()
    sample_rays = {1: None, 2: 20000, 3: 50000, 4: None, 5: 20000}

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def rel_errors(got, ref):
        # aggregate L1 ratio, then per-value relative errors (values below
        # 1e-3 of the mean radiance are measured against that floor)
        den = np.abs(ref).sum()
        floor = 1e-3 * np.abs(ref).mean()
        rel = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
        return {"rel_l1": float(np.abs(got - ref).sum() / den), "mean_rel": float(rel.mean()),
                "median_rel": float(np.median(rel)), "p99_rel": float(np.quantile(rel, 0.99)),
                "max_rel": float(rel.max()), "frac_within_1e-3": float((rel <= 1e-3).mean())}

    def storage_rounding(low, f32, tiny):
        # relative change made by storing the same FP32 values in a narrower
        # type, over values in that type's normal range
        m = np.abs(f32) >= tiny
        return {"rel_l1": float(np.abs(low - f32).sum() / np.abs(f32).sum()),
                "max_rel_normal": float((np.abs(low - f32)[m] / np.abs(f32)[m]).max())}

    for c in configs:
        log(f"configs: workload c{c}")
        sc = S.config(c)
        vol, med, light, prm, cams = lp.device_scene(sc)
        prm = dataclasses.replace(prm, waves_per_simd=WAVES.get(c, 0))
        M, N, spp = prm.M, prm.N, prm.spp
        stats = torch.zeros(5, dtype=torch.int64, device=dev)
        lf = lp.generate(vol, med, light, prm, stats=stats)
        torch.cuda.synchronize()
        tent, shadow, real, samples, cells = (int(x) for x in stats.cpu().numpy())
        reps = 2 if M * N > 10_000_000 else 5
        ms = timed(lambda: lp.generate(vol, med, light, prm, out=lf), reps)
        log(f"configs: c{c} generation {ms:.2f} ms")
        rays = M * N - (M if M == N else 0)
        row = {"workload": sc.name, "M": M, "N": N, "spp": spp, "grid": prm.grid, "rays": rays,
               "generate_ms": ms, "samples_per_s": M * N * spp / (ms / 1e3),
               "tentative_collisions_per_s": tent / (ms / 1e3), "collisions_per_sample": tent / samples,
               "cell_steps_per_sample": cells / samples,
               "gather_GBps": (tent + shadow) * 8 * np.dtype(sc.volume.data.dtype).itemsize / (ms / 1e3) / 1e9,
               "real_collisions_per_sample": real / samples, "field_bytes_f32": lf.numel() * 4}
        if c == 1:
            ks = np.arange(M * N)
            ks = ks[(ks // N) != (ks % N)]
        elif sample_rays[c] is None:
            ks = S.random_rays(M, N, (M * N) // 100, 9000 + c)
        else:
            ks = S.random_rays(M, N, sample_rays[c], 9000 + c)
        idx = torch.from_numpy(ks).to(dev)
        got = lf.reshape(-1, 3)[idx].double().cpu().numpy()
        ref = None
        if with_oracle:
            t0 = time.perf_counter()
            ref = orc.generate(sc, ks, nthreads=threads)
            t_orc = time.perf_counter() - t0
            log(f"configs: c{c} oracle on {len(ks)} rays {t_orc:.1f} s")
            row["f32_vs_oracle"] = dict(rays=int(len(ks)), **rel_errors(got, ref))
            row["oracle_samples_per_s"] = len(ks) * spp / t_orc
            row["oracle_cores"] = threads
        if c == 4:
            for name in ("f16", "bf16"):
                low = lp.generate(vol, med, light, prm, dtype=name)
                torch.cuda.synchronize()
                ms_low = timed(lambda: lp.generate(vol, med, light, prm, dtype=name, out=low), reps)
                log(f"configs: c{c} {name} generation {ms_low:.2f} ms")
                g = low.reshape(-1, 3)[idx].double().cpu().numpy()
                if ref is not None:
                    row[f"{name}_vs_oracle"] = rel_errors(g, ref)
                row[f"{name}_generate_ms"] = ms_low
                row[f"{name}_field_bytes"] = low.numel() * low.element_size()
                row[f"{name}_vs_f32"] = storage_rounding(g, got, 6.1e-5 if name == "f16" else 1.2e-38)
                del low
                torch.cuda.empty_cache()
        if c == 5:
            # adjoint of 1/2 |views - targets|^2 over 16 views of 512^2, and its checks
            W, H = sc.width, sc.height
            tm = S.target_medium(sc)
            tmed = lp.Medium(torch.from_numpy(tm.lut).to(dev), tm.scale)
            target = lp.lookup(lp.generate(vol, tmed, light, prm), prm, cams, W, H, sc.K)
            img = lp.lookup(lf, prm, cams, W, H, sc.K)
            d_lf = lp.lookup_adjoint(img - target, prm, cams, sc.K)
            ms_bwd = timed(lambda: lp.generate_backward(vol, med, light, prm, d_lf), 5)
            # the same adjoint from the radiance a forward kept
            srad = torch.empty((M, N, spp, 3), dtype=torch.float32, device=dev)
            ms_keep = timed(lambda: lp.generate(vol, med, light, prm, out=lf, sample_radiance=srad), 5)
            ms_bwd_keep = timed(lambda: lp.generate_backward(vol, med, light, prm, d_lf, sample_radiance=srad), 5)
            del srad
            log(f"configs: c{c} adjoint {ms_bwd:.2f} ms; keeping samples: forward {ms_keep:.2f}, adjoint {ms_bwd_keep:.2f} ms")
            d_lut, d_scale = lp.generate_backward(vol, med, light, prm, d_lf)
            torch.cuda.synchronize()
            g = np.concatenate([d_lut.cpu().numpy().reshape(-1), d_scale.cpu().numpy()]).astype(np.float64)
            adj = d_lf.double()
            lut0 = sc.medium.lut

            def loss(lut, scale):
                m = lp.Medium(torch.from_numpy(lut).to(dev), scale)
                L = lp.generate(vol, m, light, prm, sample=med)
                return float((L.double() * adj).sum())

            # central differences in frozen sampling on the 24 largest LUT
            # coordinates of the gradient and the density scale
            order = np.argsort(-np.abs(g[:-1]))[:24]
            h = 1e-3
            fd, gv = [], []
            for e in order:
                a, b = divmod(int(e), 4)
                lp_, lm = lut0.copy(), lut0.copy()
                lp_[a, b] += h
                lm[a, b] -= h
                fd.append((loss(lp_, sc.medium.scale) - loss(lm, sc.medium.scale)) / (float(lp_[a, b]) - float(lm[a, b])))
                gv.append(g[e])
            fd.append((loss(lut0, sc.medium.scale + h) - loss(lut0, sc.medium.scale - h)) / (2 * h))
            gv.append(g[-1])
            fd, gv = np.array(fd), np.array(gv)
            row["adjoint"] = {"views": len(cams), "width": W, "height": H, "backward_ms": ms_bwd,
                              "adjoint_forward_ratio": ms_bwd / ms,
                              "kept_samples": {"forward_ms": ms_keep, "backward_ms": ms_bwd_keep,
                                               "adjoint_forward_ratio": ms_bwd_keep / ms_keep},
                              "vs_central_differences_h1e-3": float(np.linalg.norm(gv - fd) / np.linalg.norm(fd)),
                              "fd_coordinates": len(fd)}
            if with_oracle:
                # the oracle gradient of the same adjoint restricted to a ray subset
                sub = S.random_rays(M, N, 20000, 9105)
                adj_sub = torch.zeros_like(d_lf)
                sidx = torch.from_numpy(sub).to(dev)
                adj_sub.view(-1, 3)[sidx] = d_lf.view(-1, 3)[sidx]
                gs_lut, gs_scale = lp.generate_backward(vol, med, light, prm, adj_sub)
                o_lut, o_scale = orc.gradient(sc, sub, adj_sub.view(-1, 3)[sidx].double().cpu().numpy())
                gs = np.concatenate([gs_lut.cpu().numpy().reshape(-1), [float(gs_scale)]]).astype(np.float64)
                os_ = np.concatenate([o_lut.reshape(-1), [o_scale]])
                row["adjoint"]["vs_oracle_gradient_20000_rays"] = float(np.linalg.norm(gs - os_) / np.linalg.norm(os_))
        print(json.dumps(row), flush=True)
        del lf
        torch.cuda.empty_cache()
    if calib_copy_mb:
        # counter calibration: a plain device copy of calib_copy_mb MiB, then
        # gathers of 4 and of 16 bytes from each 128-byte line of it, lines
        # in random order (64-bit indices, one per line)
        n = calib_copy_mb * (1 << 20) // 4
        a_ = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        lines = torch.randperm(n // 32, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
        g4 = a_[lines * 32]
        g16 = a_.view(-1, 4)[lines * 8]
        torch.cuda.synchronize()
        del g4, g16, lines, a_, b_


def timed_ms(fn, reps, stream):
    import numpy as np
    import torch
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def missing_rays(prm, pad):
    """Rays of the SF ray set whose chord misses the volume box grown by
    `pad` (FP64, on the GPU in row chunks): the generation kernel finishes
    them without tracing (their samples are the environment)."""
    import math
    import torch
    dev = "cuda"
    phi = (math.sqrt(5.0) - 1.0) / 2.0

    def sf(n):
        i = torch.arange(n, dtype=torch.float64, device=dev)
        z = 1.0 - (2.0 * i + 1.0) / n
        st = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
        ph = 2.0 * math.pi * torch.frac(i * phi)
        return torch.stack([torch.cos(ph) * st, torch.sin(ph) * st, z], 1)

    po, pd = sf(prm.M), sf(prm.N)
    lo, hi = -1.0 - pad, 1.0 + pad
    R = prm.radius
    count = 0
    for r0 in range(0, prm.rows, 1024):
        o = po[r0:min(prm.rows, r0 + 1024)]
        d = pd[None, :, :] - o[:, None, :]
        d = d / torch.clamp(d.norm(dim=-1, keepdim=True), min=1e-300)
        x = (R * o)[:, None, :]
        with torch.no_grad():
            t1 = (lo - x) / d
            t2 = (hi - x) / d
        tn = torch.clamp(torch.nan_to_num(torch.minimum(t1, t2), nan=-1e300).amax(-1), min=0.0)
        tf = torch.nan_to_num(torch.maximum(t1, t2), nan=1e300).amin(-1)
        miss = ~(tn < tf)
        if prm.M == prm.N:  # texels i == j have no direction and are not traced either
            idx = torch.arange(o.shape[0], device=dev)
            miss[idx, r0 + idx] = False
        count += int(miss.sum())
        del d, t1, t2
    return count


def c2_step_extra(steps, warmup):
    """The CT-like step with the adjoint (extra keys of the bench line)."""
    import numpy as np
    import torch

    import lfsynth as S
    import paper_1903_03837_amd as lp

    dev = "cuda"
    sc = S.config(2)
    vol, med, light, prm, cams = lp.device_scene(sc)
    V, W, H, K = len(cams), sc.width, sc.height, sc.K
    M, N, spp = prm.M, prm.N, prm.spp
    lf = torch.empty((M, N, 3), dtype=torch.float32, device=dev)
    img = torch.empty((V, H, W, 3), dtype=torch.float32, device=dev)
    d_lf = torch.empty((M, N, 3), dtype=torch.float32, device=dev)
    srad = torch.empty((M, N, spp, 3), dtype=torch.float32, device=dev)
    tm = S.target_medium(sc)
    tmed = lp.Medium(torch.from_numpy(tm.lut).to(dev), tm.scale)
    target = lp.lookup(lp.generate(vol, tmed, light, prm), prm, cams, W, H, K)
    stream = torch.cuda.current_stream()

    def step(evs):
        evs[0].record(stream)
        lp.points(M)
        evs[1].record(stream)
        lp.generate(vol, med, light, prm, out=lf, sample_radiance=srad)
        evs[2].record(stream)
        d_lf.zero_()
        lp.lookup_l2(lf, prm, cams, target, K, img=img, d_lf=d_lf)
        evs[3].record(stream)
        lp.generate_backward(vol, med, light, prm, d_lf, sample_radiance=srad)
        evs[4].record(stream)

    for _ in range(warmup):
        step([torch.cuda.Event(enable_timing=True) for _ in range(5)])
    torch.cuda.synchronize()
    all_evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(all_evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    names = ["points", "generate", "lookup_loss_adjoint", "generate_backward"]
    legs = {nm: float(np.mean([e[a].elapsed_time(e[a + 1]) for e in all_evs])) for a, nm in enumerate(names)}
    listed = int((d_lf.abs().sum(-1) != 0).sum())
    # the same adjoint tracing each sample twice (no kept radiance)
    bwd2 = timed_ms(lambda: lp.generate_backward(vol, med, light, prm, d_lf), 3, stream)
    gen_plain = timed_ms(lambda: lp.generate(vol, med, light, prm, out=lf), 3, stream)
    lookup_ms = timed_ms(lambda: lp.lookup(lf, prm, cams, W, H, K, img=img), 3, stream)
    # image quality against path-traced views (4 of the views at 480 x 270, 256 spp)
    qv, qw, qh, qspp = 4, 480, 270, 256
    qcams = cams[:qv]
    gt_prm = dataclasses.replace(prm, spp=qspp)
    gt = lp.render_views(vol, med, light, gt_prm, qcams, qw, qh)
    render_ms = timed_ms(lambda: lp.render_views(vol, med, light, gt_prm, qcams, qw, qh, img=gt), 1, stream)
    gmax = float(gt.max())
    quality = {"views": qv, "width": qw, "height": qh, "ground_truth_spp": qspp, "render_ms": render_ms,
               "render_samples_per_s": qv * qw * qh * qspp / (render_ms / 1e3)}
    for kk in (1, K):
        v_img = lp.lookup(lf, prm, qcams, qw, qh, kk)
        quality[f"ssim_K{kk}"] = float(lp.ssim(v_img, gt, data_range=gmax).mean())
        quality[f"cw_ssim_K{kk}"] = float(lp.cw_ssim(v_img, gt, data_range=gmax).mean())
        quality[f"rel_l1_K{kk}"] = float((v_img - gt).abs().sum() / gt.abs().sum())
    out = {
        "workload": "CT-like phantom 256^3 u16, M=N=2048 (4.19M rays), 64 spp, 8 bounces, HG g=0.3, area light, "
                    "5^3 majorant grid; FP32 field keeping each sample's radiance; lookup of 32 views 1920x1080 "
                    "K=5 fused with the loss 1/2 |views - targets|^2 and its transpose; path-replay adjoint",
        "steps": steps, "ms_per_step": ms, "path_samples_per_s": M * N * spp / (ms / 1e3), "legs_ms": legs,
        "generate_ms_without_kept_radiance": gen_plain, "lookup_ms": lookup_ms,
        "lookup_pixels_per_s": V * W * H / (lookup_ms / 1e3),
        "adjoint_rays": listed, "adjoint_rays_frac": listed / (M * N),
        "adjoint_forward_ratio_sparse": legs["generate_backward"] / legs["generate"],
        "adjoint_two_replays_ms": bwd2,
        "adjoint_forward_ratio_sparse_two_replays": bwd2 / gen_plain,
        "quality_vs_ground_truth": quality,
    }
    del srad, lf, img, d_lf, target
    torch.cuda.empty_cache()
    return out


def c5_dense_adjoint():
    """Differentiation workload: forward, and the adjoint with every
    non-degenerate ray carrying a (seeded) adjoint value: two replays per
    sample, nothing kept from the forward."""
    import numpy as np
    import torch

    import lfsynth as S
    import paper_1903_03837_amd as lp

    sc = S.config(5)
    vol, med, light, prm, cams = lp.device_scene(sc)
    M, N = prm.M, prm.N
    stream = torch.cuda.current_stream()
    lf = lp.generate(vol, med, light, prm)
    fwd = timed_ms(lambda: lp.generate(vol, med, light, prm, out=lf), 5, stream)
    g = torch.Generator(device="cuda").manual_seed(505)
    d_lf = torch.randn((M, N, 3), generator=g, device="cuda")
    d_lf.view(M * N, 3)[torch.arange(M, device="cuda") * (N + 1)] = 0.0
    lp.generate_backward(vol, med, light, prm, d_lf)
    bwd = timed_ms(lambda: lp.generate_backward(vol, med, light, prm, d_lf), 5, stream)
    return {"workload": "128^3 f32 blobs, M=N=1024, 32 spp, 4 bounces, directional light, 8^3 majorant grid; "
                        "seeded adjoint on every non-degenerate ray",
            "forward_ms": fwd, "adjoint_ms": bwd, "adjoint_forward_ratio_dense": bwd / fwd}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed step and its work counts (for profiler runs)")
    ap.add_argument("--subset-frac", type=float, default=0.01,
                    help="share of the rays in the seeded subset the oracle traces")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--configs", type=str, default="",
                    help="instead of the step, measure generation on these workloads (e.g. 1,2,3,4,5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the light field would shard by "
              "slabs of origin rows, one per GPU). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.configs:
        sweep_configs([int(c) for c in args.configs.split(",")], with_oracle=not args.no_cpu_baseline,
                      calib_copy_mb=args.calib_copy_mb)
        return

    import math

    import numpy as np
    import torch

    import lfsynth as S
    import paper_1903_03837_amd as lp

    torch.cuda.set_device(0)
    lp.library()
    dev = "cuda"
    log("bench: building the precision workload (512^3 u16 phantom in 8^3 bricks, N=32768, 16 spp)")
    sc = S.config(4, views=32, width=1920, height=1080)
    vol, med, light, prm, cams = lp.device_scene(sc)
    prm = dataclasses.replace(prm, waves_per_simd=WAVES[4])
    V, W, H, K = len(cams), sc.width, sc.height, sc.K
    M, N, spp = prm.M, prm.N, prm.spp
    lf = torch.empty((M, N, 3), dtype=torch.float32, device=dev)
    img = torch.empty((V, H, W, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(evs):
        evs[0].record(stream)
        lp.points(M)
        evs[1].record(stream)
        lp.generate(vol, med, light, prm, out=lf)
        evs[2].record(stream)
        lp.lookup(lf, prm, cams, W, H, K, img=img)
        evs[3].record(stream)

    log(f"bench: {args.warmup} warmup + {args.steps} timed steps")
    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True) for _ in range(4)])
        torch.cuda.synchronize()
        log("bench: warmup step done")
    all_evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(all_evs[k])
        if k % 4 == 3:  # progress (the queue stays full: the next step is already enqueued)
            all_evs[k][3].synchronize()
            log(f"bench: {k + 1} steps done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    names = ["points", "generate", "lookup"]
    legs = {nm: float(np.mean([e[a].elapsed_time(e[a + 1]) for e in all_evs])) for a, nm in enumerate(names)}
    ms_per_step = elapsed * 1e3 / args.steps
    log("bench: legs (ms) " + ", ".join(f"{k} {v:.2f}" for k, v in legs.items()))
    gen_s = legs["generate"] / 1e3
    khash = kernel_source_hash()

    # work counts of one launch (deterministic for the fixed stream)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    lp.generate(vol, med, light, prm, out=lf, stats=stats)
    torch.cuda.synchronize()
    tent, shadow, real, samples, cells = (int(x) for x in stats.cpu().numpy())
    rays = prm.rows * N - (M if M == N else 0)
    pad = 2.0 * prm.radius / math.sqrt(M) * 1.001 + 1e-5 * prm.radius
    n_miss = missing_rays(prm, pad)
    traced = (rays - n_miss) * spp
    points = tent + shadow
    achieved = OPS_POINT * points / gen_s
    traffic = measured_traffic(khash, "gen_c4_traffic.json")
    log(f"bench: {points} tentative points, {n_miss} of {rays} rays miss the box")

    # the same field stored as FP16 and BF16
    low = {}
    for name in (() if args.no_extras else ("f16", "bf16")):
        t = lp.generate(vol, med, light, prm, dtype=name)
        ms_low = timed_ms(lambda: lp.generate(vol, med, light, prm, dtype=name, out=t), 1, stream)
        low[name] = (t, ms_low)
        log(f"bench: {name} generation {ms_low:.1f} ms")

    def rel(got, ref):
        den = np.abs(ref).sum()
        floor = 1e-3 * np.abs(ref).mean()
        r = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
        return {"rel_l1": float(np.abs(got - ref).sum() / den), "mean_rel": float(r.mean()),
                "p99_rel": float(np.quantile(r, 0.99)), "max_rel": float(r.max()),
                "flip_frac": float((r > 1e-2).mean()), "frac_within_1e-3": float((r <= 1e-3).mean())}

    precision = {"f32": {"generate_ms": legs["generate"], "field_bytes": lf.numel() * 4}}
    for name, (t, ms_low) in low.items():
        f = t.float()
        den = float(lf.abs().sum())
        precision[name] = {"generate_ms": ms_low, "field_bytes": t.numel() * t.element_size(),
                           "memory_vs_f32": t.numel() * t.element_size() / (lf.numel() * 4),
                           "throughput_vs_f32": legs["generate"] / ms_low,
                           "rel_l1_vs_f32": float((f - lf).abs().sum()) / den}
        del f

    out = {
        "metric": "LF path samples/s + %HBM roofline; FP16 vs FP32 err; adjoint/forward time",
        "value": M * N * spp / (ms_per_step / 1e3),
        "unit": "path samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded CT-like phantom, transfer function, area light, cameras)",
        "config": {
            "workload": "precision workload: CT-like phantom 512^3 u16 (40 nested ellipsoids) in 8^3 bricks, "
                        "M=N=32768 SF points (1.07B rays), 16 spp, 8 bounces, HG g=0.3, area light, 8^3 majorant "
                        "grid, FP32 light field (12.9 GB); lookup of 32 views 1920x1080 K=5",
            "M": M, "N": N, "spp": spp, "max_bounces": prm.max_bounces, "views": V, "width": W, "height": H,
            "K": K, "volume": "512^3 u16 8^3-bricked", "majorant_grid": prm.grid,
            "waves_per_simd": prm.waves_per_simd,
        },
        "roofline": {
            "kernel": f"gen_wave_kernel<u16, forward, {prm.waves_per_simd or 4} waves per SIMD> (lf_generate)",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_OPS / 1e12,
            "unit": "Top/s (32-bit lane ops)",
            "frac": achieved / PEAK_OPS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_GBps": (traffic / gen_s / 1e9) if traffic else None,
            "hbm_frac": (traffic / gen_s / PEAK_HBM) if traffic else None,
            "launch_ms": legs["generate"],
            "ops_per_point": OPS_POINT,
            "ops_model": "algorithmic count, not counters: per tentative point (tentative collision or shadow "
                         "step) ~40 FP32 ops + one Philox4x32-10 call (60) + one logarithm (4)",
            "ops_per_launch": OPS_POINT * points,
            "units_per_launch": {"tentative_points": points, "tentative_collisions": tent, "shadow_steps": shadow,
                                 "real_collisions": real, "samples": samples, "traced_samples": traced,
                                 "rays": rays, "rays_missing_the_box": n_miss, "majorant_cell_steps": cells},
        },
        "legs_ms": legs,
        "generate_samples_per_s": M * N * spp / gen_s,
        "traced_samples_per_s": traced / gen_s,
        "tentative_points_per_s": points / gen_s,
        "lookup_pixels_per_s": V * W * H / (legs["lookup"] / 1e3),
        "precision": precision,
        "kernel_hash": khash,
    }
    del img
    torch.cuda.empty_cache()
    if args.no_extras:
        print(json.dumps(out), flush=True)
        return

    if not args.no_cpu_baseline:
        # the oracle on the seeded ray subset: the CPU baseline and the error
        # of each storage type against FP64
        from oracle import oracle as orc
        threads = orc.default_threads()
        ks = S.random_rays(M, N, int(M * N * args.subset_frac), 9004)
        log(f"bench: FP64 oracle on {len(ks)} rays ({100 * args.subset_frac:g} % subset), {threads} threads")
        t0 = time.perf_counter()
        ref = orc.generate(sc, ks, nthreads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(ks) * spp / dt, "unit": "path samples/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"seeded {100 * args.subset_frac:g} % ray subset of the precision workload: "
                                         f"{len(ks)} rays x {spp} spp ({dt:.1f} s, FP64 C, pthreads)"}
        idx = torch.from_numpy(ks).to(dev)
        for name, t in (("f32", lf), ("f16", low["f16"][0]), ("bf16", low["bf16"][0])):
            got = t.reshape(-1, 3)[idx].double().cpu().numpy()
            out["precision"][name]["vs_fp64_oracle"] = dict(rays=int(len(ks)), **rel(got, ref))
        del ref
    del low, lf
    torch.cuda.empty_cache()

    log("bench: CT-like step with the adjoint")
    out["ct_like_step"] = c2_step_extra(max(5, args.steps // 2), 2)
    log("bench: dense adjoint of the differentiation workload")
    out["dense_adjoint"] = c5_dense_adjoint()
    out["adjoint_forward_ratio_dense"] = out["dense_adjoint"]["adjoint_forward_ratio_dense"]
    out["adjoint_forward_ratio_sparse"] = out["ct_like_step"]["adjoint_forward_ratio_sparse"]
    out["fp16_vs_fp32_rel_err"] = out["precision"]["f16"]["rel_l1_vs_f32"]
    out["bf16_vs_fp32_rel_err"] = out["precision"]["bf16"]["rel_l1_vs_f32"]
    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        a_ = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
