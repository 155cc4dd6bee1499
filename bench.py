#!/usr/bin/env python3
"""Benchmark of the LumiPath light-field path on one MI355X.

One step = one pass of the whole path over the CT-like workload (256^3 u16
phantom, M = N = 2048 spherical-Fibonacci points, 4.19M rays, 64 samples per
ray, 8 bounces, HG g = 0.3, area light):
  lf_points (SF table) -> lf_generate (FP32 light field, 5^3 majorant grid, keeping
  every sample's radiance) -> lf_lookup_l2 (32 views of 1920 x 1080, K = 5, the
  gradient of 1/2 |views - targets|^2 and its lookup transpose, in one pass) ->
  lf_generate_backward (d LUT, d density scale; one replay per sample, from the
  kept radiance).
`value` = M*N*spp path samples per second of the whole step.  One JSON line
on stdout; progress on stderr.  Inputs are seeded synthetic data (lfsynth).
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

# Algorithmic 32-bit ALU operations per unit of work (see the design notes,
# "roofline of generation"): counted from the estimator's definition, one op
# per add/mul/fma/compare/convert/logic, four per transcendental, 60 per
# Philox4x32-10 block (10 rounds x (2 wide multiplies + 4 xor)).
OPS_TENTATIVE = 113     # free-flight step: 1/2 Philox, log, trilinear fetch, classify, accept
OPS_SHADOW = 90         # ratio-tracking step: 1/4 Philox, log, trilinear fetch, alpha, Tr update
OPS_REAL = 270          # scatter vertex: albedo, Philox block, light sample, phase eval/sample, clips
OPS_SAMPLE = 140        # jitter (Philox block, sqrt, sincos, frame), first clip, escape, accumulate
OPS_RAY = 80            # two SF points (FP64 frac), direction, store
OPS_CELL = 16           # majorant-grid step: cell majorant read, 3-way min, spend/compare, advance
PEAK_OPS = 256 * 4 * 16 * 2.4e9   # 32-bit lane ops per second: CUs x SIMDs x lanes x clock
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_03837_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per generation launch from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "gen_c2_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(scene, seconds, nrays_probe=20000):
    """The FP64 oracle on a bounded seeded sample of the same rays."""
    import numpy as np

    import lfsynth as S
    from oracle import oracle as orc

    threads = orc.default_threads()
    M, N = scene.params.M, scene.params.N
    ks = S.random_rays(M, N, nrays_probe, 777)
    t0 = time.perf_counter()
    orc.generate(scene, ks, nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(min(M * N, max(nrays_probe, nrays_probe * seconds / max(dt, 1e-3))))
    ks = S.random_rays(M, N, n, 778)
    t0 = time.perf_counter()
    ref = orc.generate(scene, ks, nthreads=threads)
    dt = time.perf_counter() - t0
    samples = len(ks) * scene.params.spp
    return {"value": samples / dt, "unit": "path samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(ks)} seeded random rays of the same workload x {scene.params.spp} spp "
                      f"({dt:.1f} s, FP64 C, pthreads)"}, ks, ref


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
        n = calib_copy_mb * (1 << 20) // 4
        a_ = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--configs", type=str, default="",
                    help="instead of the step, measure generation on these workloads (e.g. 1,2,3,4,5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the light field shards by rows "
              "of origins; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.configs:
        sweep_configs([int(c) for c in args.configs.split(",")], with_oracle=not args.no_cpu_baseline,
                      calib_copy_mb=args.calib_copy_mb)
        return

    import numpy as np
    import torch

    import lfsynth as S
    import paper_1903_03837_amd as lp

    torch.cuda.set_device(0)
    lp.library()
    log("bench: building the CT-like workload (256^3 u16 phantom, N=2048, 64 spp)")
    sc = S.config(2)
    vol, med, light, prm, cams = lp.device_scene(sc)
    V, W, H, K = len(cams), sc.width, sc.height, sc.K
    M, N, spp = prm.M, prm.N, prm.spp
    dev = "cuda"
    lf = torch.empty((M, N, 3), dtype=torch.float32, device=dev)
    img = torch.empty((V, H, W, 3), dtype=torch.float32, device=dev)
    dimg = torch.empty_like(img)
    d_lf = torch.empty((M, N, 3), dtype=torch.float32, device=dev)
    # every sample's radiance, kept by the forward for the adjoint (3.2 GB)
    srad = torch.empty((M, N, spp, 3), dtype=torch.float32, device=dev)

    # seeded target views: the same scene under the perturbed medium
    tm = S.target_medium(sc)
    tmed = lp.Medium(torch.from_numpy(tm.lut).to(dev), tm.scale)
    target = lp.lookup(lp.generate(vol, tmed, light, prm), prm, cams, W, H, K)

    # counts of the units of work (deterministic for the fixed stream)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    lp.generate(vol, med, light, prm, out=lf, stats=stats)
    torch.cuda.synchronize()
    tent, shadow, real, samples, cells = (int(x) for x in stats.cpu().numpy())
    rays = M * N - (M if M == N else 0)
    alg_ops = (tent * OPS_TENTATIVE + shadow * OPS_SHADOW + real * OPS_REAL + samples * OPS_SAMPLE
               + rays * OPS_RAY + cells * OPS_CELL)

    stream = torch.cuda.current_stream()
    nev = 5

    def step(evs):
        evs[0].record(stream)
        lp.points(M)
        evs[1].record(stream)
        lp.generate(vol, med, light, prm, out=lf, sample_radiance=srad)
        evs[2].record(stream)
        # views, the gradient of 1/2 |views - targets|^2 and its transpose, in one pass
        d_lf.zero_()
        lp.lookup_l2(lf, prm, cams, target, K, img=img, d_lf=d_lf)
        evs[3].record(stream)
        d_lut, d_scale = lp.generate_backward(vol, med, light, prm, d_lf, sample_radiance=srad)
        evs[4].record(stream)
        return d_lut, d_scale

    log(f"bench: {args.warmup} warmup + {args.steps} timed steps")
    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True) for _ in range(nev)])
    torch.cuda.synchronize()
    all_evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(all_evs[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    legs = {}
    names = ["points", "generate", "lookup_loss_adjoint", "generate_backward"]
    for a, name in enumerate(names):
        legs[name] = float(np.mean([e[a].elapsed_time(e[a + 1]) for e in all_evs]))
    ms_per_step = elapsed * 1e3 / args.steps
    log("bench: legs (ms) " + ", ".join(f"{k} {v:.2f}" for k, v in legs.items()))

    # the plain lookup alone (outside the timed step), for its own throughput
    lk = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lp.lookup(lf, prm, cams, W, H, K, img=dimg)
        e1.record(stream)
        torch.cuda.synchronize()
        lk.append(e0.elapsed_time(e1))
    lookup_ms = float(np.median(lk))

    gen_s = legs["generate"] / 1e3
    # voxel bytes the estimator reads: 8 voxels per tentative point (u16)
    tent_bytes = (tent + shadow) * 8 * 2
    achieved = alg_ops / gen_s
    khash = kernel_source_hash()
    traffic = measured_traffic(khash)

    # storage precision: FP16 / BF16 fields against the FP32 field
    f32 = lf.clone()
    f16 = lp.generate(vol, med, light, prm, dtype="f16").float()
    b16 = lp.generate(vol, med, light, prm, dtype="bf16").float()
    torch.cuda.synchronize()
    denom = f32.abs().sum().item()
    err16 = (f16 - f32).abs().sum().item() / denom
    errb16 = (b16 - f32).abs().sum().item() / denom

    # image quality against path-traced views (not part of the timed step):
    # 4 of the views at 480 x 270, ground truth at 256 spp
    qv, qw, qh, qspp = 4, 480, 270, 256
    qcams = cams[:qv]
    gt_prm = dataclasses.replace(prm, spp=qspp)
    gt = lp.render_views(vol, med, light, gt_prm, qcams, qw, qh)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lp.render_views(vol, med, light, gt_prm, qcams, qw, qh, img=gt)
    e1.record(stream)
    torch.cuda.synchronize()
    render_ms = e0.elapsed_time(e1)
    gmax = float(gt.max())
    quality = {"views": qv, "width": qw, "height": qh, "ground_truth_spp": qspp,
               "render_ms": render_ms, "render_samples_per_s": qv * qw * qh * qspp / (render_ms / 1e3)}
    for kk in (1, K):
        v_img = lp.lookup(lf, prm, qcams, qw, qh, kk)
        quality[f"ssim_K{kk}"] = float(lp.ssim(v_img, gt, data_range=gmax).mean())
        quality[f"cw_ssim_K{kk}"] = float(lp.cw_ssim(v_img, gt, data_range=gmax).mean())
        quality[f"rel_l1_K{kk}"] = float((v_img - gt).abs().sum() / gt.abs().sum())
    log("bench: light-field views vs ground truth " + json.dumps(quality))

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        a_ = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()

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
            "workload": "CT-like phantom 256^3 u16 (12 nested ellipsoids), M=N=2048 SF points (4.19M rays), "
                        "64 spp, 8 bounces, HG g=0.3, area light, 5^3 majorant grid, FP32 light field; lookup of "
                        "32 views 1920x1080 K=5 fused with the loss 1/2 |views - targets|^2 and its lookup transpose; adjoint by path replay from the forward's per-sample radiance",
            "M": M, "N": N, "spp": spp, "max_bounces": prm.max_bounces, "views": V, "width": W, "height": H,
            "K": K, "volume": "256^3 u16 linear", "majorant_grid": prm.grid,
        },
        "roofline": {
            "kernel": "gen_wave_kernel<u16, forward> (lf_generate)",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_OPS / 1e12,
            "unit": "Top/s (32-bit lane ops)",
            "frac": achieved / PEAK_OPS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_GBps": (traffic / gen_s / 1e9) if traffic else None,
            "gather_GBps": tent_bytes / gen_s / 1e9,
            "launch_ms": legs["generate"],
            "ops_per_launch": alg_ops,
            "units_per_launch": {"tentative_collisions": tent, "shadow_steps": shadow, "real_collisions": real,
                                 "samples": samples, "rays": rays, "majorant_cell_steps": cells},
        },
        "legs_ms": legs,
        "generate_samples_per_s": M * N * spp / gen_s,
        "lookup_ms": lookup_ms,
        "lookup_pixels_per_s": V * W * H / (lookup_ms / 1e3),
        "lookup_gather_GBps": V * W * H * 312 / (lookup_ms / 1e3) / 1e9,
        "adjoint_forward_ratio": legs["generate_backward"] / legs["generate"],
        "fp16_vs_fp32_rel_err": err16,
        "bf16_vs_fp32_rel_err": errb16,
        "quality_vs_ground_truth": quality,
        "collisions_per_sample": tent / samples,
        "cell_steps_per_sample": cells / samples,
        "kernel_hash": khash,
    }
    if not args.no_cpu_baseline:
        log(f"bench: oracle CPU baseline (~{args.cpu_seconds:.0f} s)")
        base, ks, ref = cpu_baseline(sc, args.cpu_seconds)
        out["cpu_baseline"] = base
        got = f32.reshape(-1, 3)[torch.from_numpy(ks).to(dev)].double().cpu().numpy()
        got16 = f16.reshape(-1, 3)[torch.from_numpy(ks).to(dev)].double().cpu().numpy()
        den = np.abs(ref).sum()
        out["fp32_vs_oracle_rel_err"] = float(np.abs(got - ref).sum() / den)
        out["fp16_vs_oracle_rel_err"] = float(np.abs(got16 - ref).sum() / den)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
