#!/usr/bin/env python3
"""Benchmark: Monte Carlo path tracing of the 5.5M-primitive room workload on
one MI355X, reported as traversal queries per second (Mrays/s).

One step = one sample pass over the whole hot path: camera rays for every
pixel of the 1920x1080 image, then per vertex (max depth 12) primitive-level
free-flight sampling, emission pick-up, next-event estimation (emitter query
toward a point drawn from the emitter's Gaussian) and phase sampling, then
accumulation.  A
"ray" is one traversal query (collision, emitter or environment query).

The scene, camera and seeds are synthetic and fixed (see
paper_2406_09733_amd/scenes.py); inputs are resident in HBM before timing.

Besides the JSON line's throughput it reports:
  roofline     the dominant kernel (the collision kernel): algorithmic bytes
               per launch divided by its mean launch duration from HIP events
               recorded around every launch during the timed run, against
               8 TB/s HBM.  Algorithmic bytes per collision ray = 64 n_node +
               64 n_prim + 32 (a node visit reads two child boxes' worth, a
               primitive chord test one 64-B record, the ray 32 B), with
               n_node and n_prim the measured means of an instrumented pass.
               `traffic` is the HBM bytes per launch of this run: HBM bytes per
               collision ray measured with rocprofv3 counters (the summary
               under profiles/) times the collision rays per launch, reported
               only while the kernel sources still hash to the value recorded
               there.  `layout_model` gives the bytes of this build's own
               layout (128-B 4-wide nodes, re-read records, the path record)
               for comparison;
  cpu_baseline the FP64 CPU oracle on a bounded pixel subset of the same
               workload, on this host's cores and on one core, with the CPU model;
  time_to_rmse the second half of the metric, bounded: plain (45 s, then
               extrapolated), cached (up to 110 s, enough to reach the
               target), untrained-cache and cache-free-termination (10 s)
               tracers at 240x135 (1/64 of the pixels of 1920x1080) against
               a 4096-spp plain reference, at exposure 1 (see time_to_rmse).

With --time-to-rmse it instead runs the second half of the metric on the same
scene at 300-s caps: progressive renders of the plain tracer and of the
neural-cache tracer (paths end in the cache after two scattering events; the
cache trains online, 16 Adam steps per render call of 128 samples per pixel)
against a 4096-spp plain reference, RMSE over all pixels and channels of the
images clamped to [0, 1] with the reference's own noise removed, against
wall time.  It prints one JSON line of its own (see time_to_rmse).

Other modes, each printing one JSON line of its own: --queries (per-ray query
rates), --sggx (SGGX phase functions), --transport (the linear model against
its exponential variant as renders), --fit, --radiance-fit, --shading-fit,
--rf and --albedo-grad (differentiation).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mrays/s at 5.5M prims; time-to-RMSE 0.01, plain vs neural-cache tracer"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the method (per node visit, per primitive chord test,
# per ray) and, separately, of this build's layout (4-wide 128-B nodes,
# re-read records, 48-B path record + 4-B sort index + 8-B hit)
ALG_NODE_B, ALG_PRIM_B, ALG_RAY_B = 64, 64, 32
NODE_B, PRIM_B, PATH_B = 128, 64, 60
COUNTERS = os.path.join(ROOT, "profiles", "k_collide_room_5p5m_hbm_counters.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per collision ray of k_collide from the committed counter
    summary, or None when the kernel sources changed since the counters were
    taken."""
    import glob
    import hashlib
    import re
    if not os.path.exists(COUNTERS):
        return None
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2406_09733_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    text = open(COUNTERS).read()
    m1 = re.search(r"kernel_sources_sha256: ([0-9a-f]+)", text)
    m2 = re.search(r"traffic_bytes_per_collision_ray: ([0-9.e+]+)", text)
    if not (m1 and m2) or m1.group(1) != h.hexdigest():
        return None
    return float(m2.group(1))


def cpu_baseline(sc, cam, params, target_s: float):
    """Time the FP64 oracle on an evenly spaced pixel subset at 1 spp."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    S = oracle.Scene(sc)
    log(f"[cpu] oracle scene + BVH ready in {time.perf_counter() - t0:.1f}s")
    npix = cam["width"] * cam["height"]
    nthreads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1))
    p = dict(params, spp=1, sample_offset=0)
    # calibrate on a small subset, then size the timed subset to ~target_s
    stride = max(1, npix // 512)
    pix = np.arange(0, npix, stride, dtype=np.int64)
    t0 = time.perf_counter()
    _, _, rays = S.render(cam, p, pixels=pix, nthreads=nthreads)
    dt = time.perf_counter() - t0
    want = int(len(pix) * target_s / max(dt, 1e-3))
    stride = max(1, npix // max(want, 1))
    pix = np.arange(0, npix, stride, dtype=np.int64)
    t0 = time.perf_counter()
    _, _, rays = S.render(cam, dict(p, sample_offset=1), pixels=pix, nthreads=nthreads)
    dt = time.perf_counter() - t0
    rate = rays / dt / 1e6
    # one core, on a subset sized to about a third of the time
    want1 = max(64, int(len(pix) * (target_s / 3) / (dt * nthreads)))
    stride1 = max(1, npix // want1)
    pix1 = np.arange(0, npix, stride1, dtype=np.int64)
    t0 = time.perf_counter()
    _, _, rays1 = S.render(cam, dict(p, sample_offset=2), pixels=pix1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": rate, "unit": "Mrays/s", "cores": nthreads, "kind": "oracle",
            "sample": f"every {stride}th pixel of 1920x1080 ({len(pix)} camera paths), 1 spp, "
                      f"max depth {params['max_depth']}, {rays} rays in {dt:.1f}s",
            "cpu_model": _cpu_model(), "value_1_core": rays1 / dt1 / 1e6,
            "sample_1_core": f"every {stride1}th pixel ({len(pix1)} camera paths), {rays1} rays in {dt1:.1f}s"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


class _Reference:
    """A plain-tracer reference of ref_spp samples per pixel in two halves a, b
    (disjoint sample indices), for RMSE at exposure k of images clamped to
    [0, 1].  The reference itself is noisy: for a test image t independent of
    it, E|clamp(k t) - clamp(k r)|^2 = E|clamp(k t) - truth|^2 + Var(clamp(k r)),
    and Var(clamp(k r)) is estimated per pixel from the halves as
    (clamp(k a) - clamp(k b))^2 / 4.  `rmse` returns both the plain RMSE against
    the reference and this noise-corrected estimate of the RMSE against the
    converged image."""

    def __init__(self, a, b):
        self.a, self.b = a, b
        self.r = 0.5 * (a + b)
        self._k = {}

    def _at(self, k):
        if k not in self._k:
            ref = (k * self.r).clamp(0, 1)
            var = ((k * self.a).clamp(0, 1) - (k * self.b).clamp(0, 1)) ** 2 / 4
            self._k[k] = (ref, float(var.mean()))
        return self._k[k]

    def noise(self, k=1.0):
        return self._at(k)[1] ** 0.5

    def rmse(self, img, k=1.0):
        import torch
        ref, var = self._at(k)
        mse = float(torch.mean(((k * img).clamp(0, 1) - ref) ** 2))
        return mse ** 0.5, max(0.0, mse - var) ** 0.5


def _nrc_weights0():
    import numpy as np
    rng = np.random.default_rng(0)
    layers = [(64, 96), (64, 64), (64, 64), (64, 64), (3, 64)]
    return np.concatenate([rng.uniform(-1, 1, o * i) * np.sqrt(6.0 / i) for (o, i) in layers]).astype(np.float32)


def time_to_rmse(args, ctx=None, sc=None, bounded=False):
    """Time to RMSE 0.01 of the plain and the neural-cache tracer on the room.

    Images are compared at exposure 1, clamped to [0, 1], over all pixels and
    channels, against a 4096-spp plain reference (two halves of 2048 with
    disjoint sample indices).  At exposure 1 that reference is itself far
    noisier than 0.01 (its own RMSE is ~0.03: two 1 x 1 m panels light an
    8 x 3 x 8 m room), so an RMSE against it cannot fall below ~0.03; the
    criterion is therefore the noise-corrected RMSE, the RMSE against the
    converged image estimated by subtracting the reference's own variance
    (from its halves) from the mean squared difference (see _Reference).  The
    plain RMSE against the reference is reported beside it.

    Each tracer renders progressively from sample 0 with another seed, one
    wavefront (all pixels x several samples) per call; the wall time of the
    render calls is accumulated and the RMSE is taken after every call
    (outside the clock).  Runs: plain; the cache trained online from fixed
    initial weights (paths end in it after two scattering events); the same
    initial cache untrained (inference only); paths ending after two
    scattering events with nothing added.  bounded=True is the default
    benchmark's leg (caps per run).
    """
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    W, H = (int(v) for v in args.rmse_res.split("x"))
    if sc is None:
        sc = scenes.room_5p5m()
    cam = dict(scenes.camera("room_5p5m"), width=W, height=H)
    rs = scenes.render_settings("room_5p5m")
    if ctx is None:
        ctx = P.Context(0)
        ctx.build_bvh(sc)
        ctx.sync()
    ctx.set_profiling(0)
    base = {"max_depth": rs["max_depth"], "seed": rs["seed"]}
    wf = max(1, min(args.ref_spp // 2, args.rmse_wavefront))
    t_ref = 0.0
    halves = []
    half = args.ref_spp // 2
    for h in range(2):
        acc = torch.zeros((H, W, 3), device="cuda", dtype=torch.float32)
        done = 0
        while done < half:
            n = min(4 * wf, half - done)
            t0 = time.perf_counter()
            ctx.render(cam, dict(base, spp=n, sample_offset=h * half + done, want_sumsq=False), acc)
            ctx.sync()
            t_ref += time.perf_counter() - t0
            done += n
        log(f"[rmse] reference half {h}: {done} spp ({t_ref:.1f} s)")
        halves.append(acc / half)
    R = _Reference(*halves)
    black = R.rmse(torch.zeros_like(R.r))
    log(f"[rmse] reference noise at exposure 1: {R.noise():.5f}; mean clamped pixel "
        f"{float(R.r.clamp(0, 1).mean()):.4f}; RMSE of a black image {black[1]:.4f}")
    target = args.rmse_target
    caps = {"plain": args.rmse_seconds, "nrc": getattr(args, "rmse_seconds_nrc", None) or args.rmse_seconds,
            "nrc_untrained": args.rmse_seconds_ablation, "terminate": args.rmse_seconds_ablation}

    def run(label, extra, weights=None, warmup=0):
        if weights is not None:
            ctx.nrc_set_weights(weights)
        acc = torch.zeros((H, W, 3), device="cuda", dtype=torch.float32)
        t, spp, curve = 0.0, 0, []
        # warm-up calls train the cache on their own samples without adding
        # them to the image (their time counts): the image then averages only
        # samples rendered with a cache that has learned something
        for k in range(warmup):
            t0 = time.perf_counter()
            ctx.render(cam, dict(base, seed=778, spp=wf, sample_offset=k * wf, want_sumsq=False, **extra))
            ctx.sync()
            t += time.perf_counter() - t0
        while t < caps[label] and spp < args.rmse_max_spp:
            t0 = time.perf_counter()
            ctx.render(cam, dict(base, seed=777, spp=wf, sample_offset=spp, want_sumsq=False, **extra), acc)
            ctx.sync()
            t += time.perf_counter() - t0
            spp += wf
            raw, true = R.rmse(acc / spp)
            curve.append((round(t, 4), spp, round(true, 6), round(raw, 6)))
            if len(curve) % 20 == 1:
                log(f"[rmse] {label}: {spp} spp, {t:.2f} s, RMSE {true:.5f} (vs reference {raw:.5f})")
            if true <= target:
                break
        hit = next((c for c in curve if c[2] <= target), None)
        out = {"time_to_target_s": hit[0] if hit else None, "spp_at_target": hit[1] if hit else None,
               "final": {"t_s": curve[-1][0], "spp": curve[-1][1], "rmse": curve[-1][2],
                         "rmse_vs_reference": curve[-1][3]},
               "ms_per_call": round(1e3 * curve[-1][0] / len(curve), 2),
               "curve": [c[:3] for c in curve[:: max(1, len(curve) // 30)]]}
        if hit is None and label == "plain":
            # unbiased: the squared error falls as 1/t, so the time to the target
            # follows from the last point (an extrapolation, labelled as such)
            out["time_to_target_extrapolated_s"] = round(curve[-1][0] * (curve[-1][2] / target) ** 2, 2)
        if extra.get("nrc_mode", 0) == 1:
            out["last_loss"] = ctx.render_stats()["nrc_loss"]
        log(f"[rmse] {label}: {json.dumps({k: v for k, v in out.items() if k != 'curve'})}")
        return out, curve

    w0 = _nrc_weights0()
    nrc = {"nrc_mode": 1, "nrc_terminate_after": 2, "nrc_train_records": args.nrc_records, "nrc_lr": args.nrc_lr,
           "nrc_train_steps": args.nrc_steps, "nrc_target_clamp": args.nrc_clamp}
    runs = args.runs.split(",")
    res, curves = {}, {}
    if "plain" in runs:
        res["plain"], curves["plain"] = run("plain", {})
    if "nrc" in runs:
        res["nrc"], curves["nrc"] = run("nrc", nrc, w0, warmup=args.nrc_warmup_calls)
    if "nrc_untrained" in runs:
        res["nrc_untrained"], _ = run("nrc_untrained", dict(nrc, nrc_mode=2), w0)
    if "terminate" in runs:
        res["terminate_no_cache"], _ = run("terminate", {"nrc_mode": 3, "nrc_terminate_after": 2})

    def at(curve, t):
        prev = None
        for c in curve:
            if c[0] > t:
                break
            prev = c
        return prev[2] if prev else None

    cp, cn = curves.get("plain"), curves.get("nrc")
    t_eq = min(cp[-1][0], cn[-1][0]) if cp and cn else None
    vp_, vn = res.get("plain", {}).get("time_to_target_s"), res.get("nrc", {}).get("time_to_target_s")
    out = {"metric": "time to RMSE %.3g at exposure 1 (clamped [0,1] linear RGB, all pixels and channels, "
                     "noise of the %d-spp plain reference removed)" % (target, args.ref_spp),
           "unit": "s", "higher_is_better": False,
           "value_plain": vp_, "value_nrc": vn,
           "speedup_nrc": round(vp_ / vn, 3) if vp_ and vn else None,
           "value_plain_extrapolated": res.get("plain", {}).get("time_to_target_extrapolated_s"),
           "equal_time_s": t_eq,
           "rmse_at_equal_time": {"plain": at(cp, t_eq), "nrc": at(cn, t_eq)} if t_eq else None,
           "reference": {"spp": args.ref_spp, "noise_rmse": round(R.noise(), 6), "render_s": round(t_ref, 2),
                         "mean_clamped_pixel": round(float(R.r.clamp(0, 1).mean()), 5),
                         "black_image_rmse": round(black[1], 5)},
           "config": {"workload": f"room_5p5m at {W}x{H} ({W * H / (1920 * 1080):.4g} of the 1920x1080 "
                                  f"pixels), depth {rs['max_depth']}; the cache ends paths after 2 scattering "
                                  f"events and trains on {args.nrc_records} records per chunk of samples",
                      "spp_per_call": wf, "seconds_cap": caps, "nrc": nrc,
                      "nrc_warmup_calls": args.nrc_warmup_calls},
           "runs": res}
    return out


def copy_probe(nbytes: int):
    """A plain device copy of nbytes (three launches), the known-size kernel
    against which HBM byte counters are scaled."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 3}))


def transmittance_fit(args):
    """The transmittance optimisation of Sec. 7.2 on the 100K-primitive mixed
    scene: reference images of the scene from 8 views of 256x256 (16 jittered
    rays per pixel), a perturbed copy as the start, then Adam steps with one
    jittered ray per pixel per view, the hierarchy rebuilt every step.  Prints
    one JSON line: steps per second, rays per second through the CDF and its
    gradient, the loss at the start and the end."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import fit, scenes

    sc = scenes.mixed_100k()
    n = sc["mean"].shape[0]
    cams = scenes.ring_cameras((0.5, 0.5, 0.5), 2.2, n=8, size=256)
    ctx = P.Context(0)
    target = fit.reference_images(ctx, sc, cams, seed=3, samples=16)
    start = scenes.perturbed(sc, seed=11)
    params = {k: torch.tensor(np.asarray(start[k]), device="cuda").contiguous()
              for k in ("mean", "scale", "rotation", "density", "albedo", "roughness", "emission", "material")}
    # warm-up step on a copy (kernels loaded, allocations made), then the timed run
    warm = {k: v.clone() for k, v in params.items()}
    lr = tuple(float(x) for x in args.fit_lr.split(","))
    fit.fit_transmittance(ctx, warm, cams, target, iters=1, lr=lr)
    out = fit.fit_transmittance(ctx, params, cams, target, iters=args.fit_steps, lr=lr,
                                on_step=lambda it: log(f"[fit] step {it}") if it % 10 == 0 else None,
                                rebuild_every=args.fit_rebuild_every)
    ls = out["loss"]
    rays = args.fit_steps * sum(c["width"] * c["height"] for c in cams)
    res = {"metric": "transmittance-fit steps/s (Sec. 7.2) on the 100K mixed scene",
           "value": round(args.fit_steps / out["seconds"], 3), "unit": "steps/s",
           "ms_per_step": round(1e3 * out["seconds"] / args.fit_steps, 2),
           "rays_per_s": round(rays / out["seconds"], 1), "primitives": n, "views": len(cams),
           "resolution": "256x256", "steps": args.fit_steps, "lr_mean_logscale_rotation_density": lr,
           "rebuild_every": args.fit_rebuild_every,
           "loss_first": ls[0], "loss_last": ls[-1], "loss_ratio": round(ls[-1] / ls[0], 4),
           "loss_curve": [round(x, 7) for x in ls[:: max(1, len(ls) // 20)]]}
    print(json.dumps(res), flush=True)


def radiance_fit(args):
    """Differentiable fitting at the shape of the fitting workload: a target of
    the 100K mixed scene rendered by the plain tracer from 8 cameras on a ring
    of radius 1.5 around (0.5, 0.5, 0.5) at heights +-0.3 (alternating),
    256x256, 64 spp, depth 4, environment 0.3; a start of 200,000 primitives
    as in the 1K random scene (means U[0,1]^3, random rotations, densities
    U[0.5, 5]) with albedo 0.5 and roughness 0.5 (seed 4), its scales
    (log-uniform [0.005, 0.05] there) multiplied by (1000 / 200000)^(1/3) so
    that the start overlaps as the 1K scene does (0.9 primitives per point;
    at the 1K scene's scales 200K primitives overlap 176-fold, beyond the
    sweep's 64 entries).  Stage A fits the geometry (means, scales,
    rotations, densities) to the target's transmittance images with the
    accumulated free-flight CDF (Sec. 7.2; its Adam with clamps); stage B fits
    albedo, roughness and density to the target radiance images through the
    path tracer's adjoints (autograd.render, one view of 64 spp per step, the
    backward on another seed).  One JSON line: steps/s of each stage, the
    losses, and the image error of all views (at 64 spp) before and after."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import autograd as A
    from paper_2406_09733_amd import fit, scenes

    target_sc = scenes.mixed_100k()
    cams = []
    for k in range(8):
        a = 2 * np.pi * k / 8
        h = 0.3 if k % 2 == 0 else -0.3
        o = np.array([0.5, 0.5, 0.5]) + 1.5 * np.array([np.cos(a), h, np.sin(a)])
        cams.append({"origin": tuple(o.tolist()), "target": (0.5, 0.5, 0.5), "up": (0.0, 1.0, 0.0),
                     "vfov_deg": 45.0, "width": 256, "height": 256})
    rp = {"max_depth": 4, "env_radiance": (0.3, 0.3, 0.3), "spp": 64}
    ctx = P.Context(0)
    t0 = time.perf_counter()
    truth = {k: torch.tensor(np.asarray(v), device="cuda") for k, v in target_sc.items() if k != "bounds"}
    with torch.no_grad():
        targets = [A.render(ctx, truth, c, dict(rp, seed=900 + i)).detach() for i, c in enumerate(cams)]
    cdf_target = fit.reference_images(ctx, target_sc, cams, seed=3, samples=16)
    torch.cuda.synchronize()
    log(f"[radiance-fit] targets rendered in {time.perf_counter() - t0:.1f}s")
    init = scenes.tiny_random(seed=4, n=200_000, n_emit=0)
    init["scale"] = (init["scale"] * (1000.0 / 200_000) ** (1.0 / 3.0)).astype(np.float32)
    init["albedo"][:] = 0.5
    init["roughness"][:] = 0.5
    params = {k: torch.tensor(np.asarray(init[k]), device="cuda").contiguous()
              for k in ("mean", "scale", "rotation", "density", "albedo", "roughness", "emission", "material")}

    def image_error():
        with torch.no_grad():
            e = [float(((A.render(ctx, params, c, dict(rp, seed=700 + i)) - targets[i]) ** 2).mean())
                 for i, c in enumerate(cams)]
        return float(np.mean(e))

    err0 = image_error()
    log(f"[radiance-fit] start: image error {err0:.4e}")
    # stage A: geometry from the transmittance images (Sec. 7.2)
    outA = fit.fit_transmittance(ctx, params, cams, cdf_target, iters=args.fit_steps_geometry,
                                 lr=(5e-5, 1e-2, 2e-3, 1e-2), rebuild_every=1,
                                 on_step=lambda it: log(f"[radiance-fit] geometry step {it}") if it % 10 == 0 else None)
    errA = image_error()
    log(f"[radiance-fit] after the geometry stage: image error {errA:.4e}")
    # stage B: albedo, roughness and density through the path tracer
    alb = params["albedo"].clone().requires_grad_(True)
    rough = params["roughness"].clone().requires_grad_(True)
    logd = torch.log(params["density"].clamp(min=1e-4)).requires_grad_(True)
    opt = torch.optim.Adam([{"params": [alb], "lr": 0.02}, {"params": [rough], "lr": 0.01},
                            {"params": [logd], "lr": 0.02}])
    lossesB = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(args.fit_steps_appearance):
        v = it % len(cams)
        cur = dict(params, albedo=alb, roughness=rough, density=torch.exp(logd))
        img = A.render(ctx, cur, cams[v], dict(rp, seed=2000 + it), backward_params={"seed": 50000 + it})
        loss = ((img - targets[v]) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            alb.clamp_(0.01, 0.99)
            rough.clamp_(0.05, 1.0)
        lossesB.append(float(loss.item()))
        if it % 10 == 0:
            log(f"[radiance-fit] appearance step {it} loss {lossesB[-1]:.4e}")
    torch.cuda.synchronize()
    tB = time.perf_counter() - t0
    with torch.no_grad():
        params["albedo"], params["roughness"], params["density"] = alb.detach(), rough.detach(), torch.exp(logd).detach()
    errB = image_error()
    lsA = outA["loss"]
    res = {"metric": "differentiable fitting: 200K random primitives to 8 views of the 100K mixed scene at 256x256",
           "value": round(args.fit_steps_appearance / tB, 3), "unit": "appearance steps/s", "higher_is_better": True,
           "primitives": int(params["mean"].shape[0]), "target_primitives": int(target_sc["mean"].shape[0]),
           "views": len(cams), "resolution": "256x256", "spp": rp["spp"], "max_depth": rp["max_depth"],
           "stage_a": {"steps": args.fit_steps_geometry, "steps_per_s": round(args.fit_steps_geometry / outA["seconds"], 3),
                       "loss_first": lsA[0], "loss_last": lsA[-1]},
           "stage_b": {"steps": args.fit_steps_appearance, "ms_per_step": round(1e3 * tB / args.fit_steps_appearance, 1),
                       "loss_first5": float(np.mean(lossesB[:5])), "loss_last5": float(np.mean(lossesB[-5:]))},
           "image_error": {"start": round(err0, 6), "after_geometry": round(errA, 6), "after_appearance": round(errB, 6)}}
    print(json.dumps(res), flush=True)


def shading_fit(args):
    """Fit of the shading parameters through the path tracer's adjoints: the
    100K mixed scene rendered from 8 views of 256x256 (depth 4, environment
    0.3) as targets; a start with every albedo and roughness perturbed
    (geometry held); Adam on albedo and roughness through autograd.render,
    one view per step, each view rendered with its target's seed and spp
    (common random numbers: the loss is zero at the truth and measures the
    parameter error, not Monte Carlo noise).  Prints one JSON line: steps/s,
    the image loss of the first and last ten steps and the parameter errors
    of the primitives the views see most, at the start and the end."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import autograd as A
    from paper_2406_09733_amd import scenes

    sc = scenes.mixed_100k()
    n = sc["mean"].shape[0]
    cams = scenes.ring_cameras((0.5, 0.5, 0.5), 2.2, n=8, size=256)
    ctx = P.Context(0)
    truth = {k: torch.tensor(np.asarray(v), device="cuda") for k, v in sc.items() if k != "bounds"}
    spp = args.shading_fit_spp
    rp = {"max_depth": 4, "env_radiance": (0.3, 0.3, 0.3), "spp": spp}
    targets = [A.render(ctx, truth, c, dict(rp, seed=1000 + i)).detach() for i, c in enumerate(cams)]
    rng = np.random.default_rng(21)
    a_true = np.asarray(sc["albedo"], np.float64)
    r_true = np.asarray(sc["roughness"], np.float64)
    a0 = np.clip(a_true + rng.uniform(-0.3, 0.3, a_true.shape), 0.02, 0.98)
    r0 = np.clip(r_true + rng.uniform(-0.3, 0.3, n), 0.05, 1.0)
    params = dict(truth)
    params["albedo"] = torch.tensor(a0.astype(np.float32), device="cuda", requires_grad=True)
    params["roughness"] = torch.tensor(r0.astype(np.float32), device="cuda", requires_grad=True)
    opt = torch.optim.Adam([{"params": [params["albedo"]], "lr": args.shading_fit_lr[0]},
                            {"params": [params["roughness"]], "lr": args.shading_fit_lr[1]}])
    # the primitives the views see most: albedo gradient of a plain sum
    seen_w = torch.zeros(n, device="cuda")
    ctx.build_bvh(sc)
    for c in cams:
        g = torch.zeros((n, 3), device="cuda")
        ctx.render_albedo_grad(c, dict(rp, spp=1, seed=7), torch.ones((256, 256, 3), device="cuda"), g)
        seen_w += g.abs().sum(1)
    seen = torch.argsort(-seen_w)[:2000].cpu().numpy()
    glossy = seen[np.asarray(sc["material"])[seen] == 1]
    steps = args.shading_fit_steps
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        v = it % len(cams)
        img = A.render(ctx, params, cams[v], dict(rp, seed=1000 + v))
        loss = ((img - targets[v]) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            params["albedo"].clamp_(0.01, 0.99)
            params["roughness"].clamp_(0.05, 1.0)
        losses.append(float(loss.item()))
        if it % 40 == 0:
            log(f"[shading-fit] step {it} loss {losses[-1]:.4e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a1 = params["albedo"].detach().cpu().numpy().astype(np.float64)
    r1 = params["roughness"].detach().cpu().numpy().astype(np.float64)
    res = {"metric": "shading fit (albedo + roughness through the path-replay adjoints), 100K mixed scene, "
                     "8 views of 256x256",
           "value": round(steps / dt, 3), "unit": "steps/s", "ms_per_step": round(1e3 * dt / steps, 2),
           "steps": steps, "spp": spp, "max_depth": rp["max_depth"], "lr_albedo_roughness": args.shading_fit_lr,
           "loss_first10": float(np.mean(losses[:10])), "loss_last10": float(np.mean(losses[-10:])),
           "albedo_err_seen": [round(float(np.abs(a0[seen] - a_true[seen]).mean()), 4),
                               round(float(np.abs(a1[seen] - a_true[seen]).mean()), 4)],
           "roughness_err_seen_glossy": [round(float(np.abs(r0[glossy] - r_true[glossy]).mean()), 4),
                                         round(float(np.abs(r1[glossy] - r_true[glossy]).mean()), 4)],
           "seen_primitives": int(seen.size)}
    print(json.dumps(res), flush=True)


def rf_render_bench(args):
    """Radiance-field rendering (Sec. 8, eq. rf) at the resolution of the
    paper's timings (800x800, one ray per pixel) on a synthetic scene of
    300K primitives (the mixed generator at 3x: flat Gaussians on spheres and
    planes plus a cloud; every primitive emissive).  Prints one JSON line: ms
    per frame and rays/s (the saturation sweep and the emission-weighted sum)."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import fit, scenes

    sc = scenes.mixed_100k(n_flat=210_000, n_cloud=90_000, n_emit=0)
    rng = np.random.default_rng(5)
    sc["emission"] = rng.uniform(0.0, 1.0, (sc["mean"].shape[0], 3)).astype(np.float32)
    cams = scenes.ring_cameras((0.5, 0.5, 0.5), 2.2, n=8, size=800)
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    rays = [fit.view_rays(ctx, [c], 1, 0) for c in cams]
    for r in rays[:2]:
        ctx.rf_render(r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.rf_frames):
        ctx.rf_render(rays[k % len(rays)])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.rf_frames
    res = {"metric": "radiance-field render ms per 800x800 frame (Sec. 8, eq. rf)", "value": round(1e3 * dt, 3),
           "unit": "ms", "higher_is_better": False, "primitives": int(sc["mean"].shape[0]),
           "resolution": "800x800", "frames": args.rf_frames, "rays_per_s": round(800 * 800 / dt, 1)}
    print(json.dumps(res), flush=True)


def albedo_grad_bench(args):
    """Cost of the albedo adjoint (ugp_render_albedo_grad, path replay)
    against the plain render it differentiates: the 100K mixed scene, one
    view of 256x256 at 64 spp, depth 8 (the differentiable-fitting
    workload's view).  Prints one JSON line: ms per render, ms per adjoint
    (forward + replay), and camera paths/s of the adjoint."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    sc = scenes.mixed_100k()
    cam = dict(scenes.camera("mixed_100k"), width=256, height=256)
    rp = {"spp": 64, "max_depth": 8, "seed": 5, "env_radiance": (0.2, 0.2, 0.2), "want_sumsq": False}
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    d = torch.tensor(np.random.default_rng(1).uniform(-1, 1, (256, 256, 3)).astype(np.float32), device="cuda")
    g = torch.zeros((sc["mean"].shape[0], 3), device="cuda", dtype=torch.float32)
    ctx.render(cam, rp)
    ctx.render_albedo_grad(cam, rp, d, g)
    ctx.sync()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.render(cam, rp)
    ctx.sync()
    t_fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.render_albedo_grad(cam, rp, d, g)
    ctx.sync()
    t_adj = (time.perf_counter() - t0) / reps
    paths = 256 * 256 * rp["spp"]
    res = {"metric": "albedo adjoint (path replay) ms per 256x256 view at 64 spp, 100K mixed scene",
           "value": round(1e3 * t_adj, 2), "unit": "ms", "higher_is_better": False,
           "render_ms": round(1e3 * t_fwd, 2), "adjoint_over_render": round(t_adj / t_fwd, 3),
           "adjoint_paths_per_s": round(paths / t_adj, 1), "depth": rp["max_depth"], "spp": rp["spp"]}
    print(json.dumps(res), flush=True)


def sggx_bench(args):
    """Cost of the SGGX microflake phase functions in the path tracer: the
    100K mixed scene at 512x512, 16 spp, depth 8, rendered with its own
    delta-NDF materials, then with half of the primitives SGGX microflakes
    with a Lambertian base (material 2) and with a Disney-style base
    (material 3).  One JSON line: ms per frame, Mrays/s and the shading
    kernels' share per variant (kernel times from HIP events)."""
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    base_sc = scenes.mixed_100k()
    cam = dict(scenes.camera("mixed_100k"), width=512, height=512)
    rp = {"spp": 16, "max_depth": 8, "seed": 1, "env_radiance": (0.2, 0.2, 0.2)}
    ctx = P.Context(0)
    out = {}
    for name, sc in (("delta_ndf", base_sc), ("sggx_lambert", scenes.with_sggx(base_sc, seed=7, frac=0.5)),
                     ("sggx_disney", scenes.with_sggx(base_sc, seed=7, frac=0.5, base="disney"))):
        ctx.build_bvh(sc)
        ctx.set_profiling(0)
        ctx.render(cam, dict(rp, spp=2, sample_offset=1000))
        ctx.sync()
        ctx.set_profiling(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.render(cam, rp)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.render_stats()
        ctx.set_profiling(0)
        kern = st["ms_collide"] + st["ms_collide_wide"] + st["ms_light"] + st["ms_env"] + st["ms_shade"] + st["ms_sort"]
        out[name] = {"ms_per_frame": round(1e3 * dt, 2), "mrays_per_s": round(st["rays"] / dt / 1e6, 1),
                     "shade_ms": round(st["ms_shade"], 2), "shade_share": round(st["ms_shade"] / max(kern, 1e-9), 3),
                     "rays_per_path": round(st["rays"] / max(st["paths"], 1), 3)}
        log(f"[bench] {name}: {json.dumps(out[name])}")
    res = {"metric": "path tracing with SGGX microflake primitives, 100K mixed scene 512x512 16 spp depth 8",
           "value": out["sggx_disney"]["ms_per_frame"], "unit": "ms", "higher_is_better": False,
           "variants": out, "sggx_fraction": 0.5}
    print(json.dumps(res), flush=True)


def transport_bench(args):
    """The paper's comparison of transmittance models as renders: the 100K
    mixed scene (512x512, 16 spp, depth 8) and the room (480x270, 4 spp,
    depth 12) rendered with the linear model and with its exponential
    variant (decomposition tracking, App. D).  One JSON line: ms per frame,
    Mrays/s, collision and light-sample kernel times and the image mean per
    scene and model (kernel times from HIP events)."""
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    ctx = P.Context(0)
    out = {}
    for name, sc, cam, rp in (
            ("mixed_100k", scenes.mixed_100k(), dict(scenes.camera("mixed_100k"), width=512, height=512),
             {"spp": 16, "max_depth": 8, "seed": 1, "env_radiance": (0.2, 0.2, 0.2)}),
            ("room_5p5m", scenes.room_5p5m(), dict(scenes.camera("room_5p5m"), width=480, height=270),
             {"spp": 4, "max_depth": 12, "seed": 1})):
        ctx.build_bvh(sc)
        for tr, model in ((0, "linear"), (1, "exponential")):
            p = dict(rp, transport=tr)
            ctx.set_profiling(0)
            ctx.render(cam, dict(p, spp=1, sample_offset=1000))
            ctx.sync()
            ctx.set_profiling(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, _ = ctx.render(cam, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = ctx.render_stats()
            ctx.set_profiling(0)
            r = {"ms_per_frame": round(1e3 * dt, 2), "mrays_per_s": round(st["rays"] / dt / 1e6, 1),
                 "collide_ms": round(st["ms_collide"] + st["ms_collide_wide"] + st["ms_tail"], 2),
                 "light_ms": round(st["ms_light"], 2), "rays_per_path": round(st["rays"] / max(st["paths"], 1), 3),
                 "image_mean": round(float(s.mean()) / p["spp"], 5)}
            out[f"{name}_{model}"] = r
            log(f"[bench] {name} {model}: {json.dumps(r)}")
    res = {"metric": "path tracing under the linear model and its exponential variant (App. D)",
           "value": out["room_5p5m_exponential"]["mrays_per_s"], "unit": "Mrays/s", "higher_is_better": True,
           "runs": out}
    print(json.dumps(res), flush=True)


def query_bench(args):
    """Per-ray query rates on the room (5.5M primitives): linear-model
    transmittance and free-flight sampling (the ordered sweep) against the
    exponential variant's transmittance and analog decomposition tracking
    (App. D), on the same 4M rays (origins in the room, directions uniform,
    t in [0, inf)).  Prints one JSON line of Mrays/s per query."""
    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    sc = scenes.room_5p5m()
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    n = 1 << 22
    rng = np.random.default_rng(17)
    o = rng.uniform([0.5, 0.2, 0.5], [7.5, 2.8, 7.5], (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = torch.tensor(np.concatenate([o, d, np.zeros((n, 1)), np.full((n, 1), np.inf)], 1).astype(np.float32),
                        device="cuda")
    u = torch.tensor(rng.uniform(0, 1, n).astype(np.float32), device="cuda")
    runs = {"linear_transmittance": lambda: ctx.transmittance(rays),
            "linear_sample_collision": lambda: ctx.sample_collision(rays, u),
            "linear_saturation": lambda: ctx.saturation(rays),
            "exp_transmittance": lambda: ctx.exp_transmittance(rays),
            "exp_sample_collision": lambda: ctx.exp_sample_collision(rays, 5)}
    res = {"metric": "per-ray query Mrays/s on the room, 4M rays", "unit": "Mrays/s", "rays": n}
    for name, fn in runs.items():
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        res[name] = round(3 * n / (time.perf_counter() - t0) / 1e6, 2)
        log(f"[queries] {name}: {res[name]} Mrays/s")
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed sample passes")
    ap.add_argument("--warmup", type=int, default=2, help="untimed sample passes")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--time-to-rmse", action="store_true", help="run the full time-to-RMSE comparison instead")
    ap.add_argument("--no-time-to-rmse", action="store_true", help="skip the bounded time-to-RMSE leg")
    ap.add_argument("--rmse-res", default="240x135")
    ap.add_argument("--ref-spp", type=int, default=4096)
    ap.add_argument("--rmse-target", type=float, default=0.01)
    ap.add_argument("--rmse-seconds", type=float, default=300.0, help="wall-time cap of the plain and cached runs")
    ap.add_argument("--rmse-seconds-nrc", type=float, default=None,
                    help="wall-time cap of the cached run (default: --rmse-seconds)")
    ap.add_argument("--rmse-seconds-ablation", type=float, default=30.0,
                    help="wall-time cap of the untrained-cache and termination runs")
    ap.add_argument("--rmse-max-spp", type=int, default=1 << 18)
    ap.add_argument("--rmse-wavefront", type=int, default=128,
                    help="samples per pixel per render call (the RMSE is taken after each call)")
    ap.add_argument("--nrc-lr", type=float, default=1e-2)
    ap.add_argument("--nrc-records", type=int, default=262144, help="training records per chunk of samples")
    ap.add_argument("--nrc-warmup-calls", type=int, default=0,
                    help="first render calls of the cached tracer that only train the cache (timed, not accumulated)")
    ap.add_argument("--nrc-steps", type=int, default=16, help="Adam steps per chunk")
    ap.add_argument("--nrc-clamp", type=float, default=0.0, help="training target clamp (radiance units; 0 = none)")
    ap.add_argument("--runs", default="plain,nrc,nrc_untrained,terminate")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of BYTES (counter calibration) and exit")
    ap.add_argument("--fit", action="store_true", help="run the transmittance-optimisation benchmark instead")
    ap.add_argument("--rf", action="store_true", help="run the radiance-field rendering benchmark instead")
    ap.add_argument("--queries", action="store_true", help="run the per-ray query benchmark instead")
    ap.add_argument("--albedo-grad", action="store_true", help="run the albedo-adjoint benchmark instead")
    ap.add_argument("--sggx", action="store_true", help="run the SGGX phase-function benchmark instead")
    ap.add_argument("--transport", action="store_true",
                    help="render two scenes under the linear model and its exponential variant instead")
    ap.add_argument("--radiance-fit", action="store_true",
                    help="run the differentiable-fitting benchmark (200K primitives, 8 views) instead")
    ap.add_argument("--fit-steps-geometry", type=int, default=50, help="geometry (transmittance) steps")
    ap.add_argument("--fit-steps-appearance", type=int, default=40, help="appearance (path-traced) steps")
    ap.add_argument("--shading-fit", action="store_true",
                    help="run the albedo + roughness fit through the path tracer's adjoints instead")
    ap.add_argument("--shading-fit-steps", type=int, default=200)
    ap.add_argument("--shading-fit-spp", type=int, default=8)
    ap.add_argument("--shading-fit-lr", type=lambda v: [float(x) for x in v.split(",")], default=[0.02, 0.005],
                    help="Adam learning rates: albedo,roughness")
    ap.add_argument("--rf-frames", type=int, default=40)
    ap.add_argument("--fit-steps", type=int, default=50)
    ap.add_argument("--fit-rebuild-every", type=int, default=1,
                    help="new hierarchy every N fit steps, refitted in between (1: rebuild every step)")
    ap.add_argument("--fit-lr", default="5e-5,1e-2,2e-3,1e-2",
                    help="Adam rates of the means, log scales, rotations and densities")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path would shard by "
              "pixels, with no communication beyond a final image reduction)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.time_to_rmse:
        print(json.dumps(time_to_rmse(args)), flush=True)
        return
    if args.fit:
        transmittance_fit(args)
        return
    if args.rf:
        rf_render_bench(args)
        return
    if args.queries:
        query_bench(args)
        return
    if args.albedo_grad:
        albedo_grad_bench(args)
        return
    if args.transport:
        transport_bench(args)
        return
    if args.sggx:
        sggx_bench(args)
        return
    if args.shading_fit:
        shading_fit(args)
        return
    if args.radiance_fit:
        radiance_fit(args)
        return

    import numpy as np
    import torch

    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes

    name = "room_5p5m"
    t0 = time.perf_counter()
    sc = scenes.room_5p5m()
    cam = scenes.camera(name)
    rs = scenes.render_settings(name)
    log(f"[bench] scene {sc['mean'].shape[0]} primitives generated in {time.perf_counter() - t0:.1f}s")
    ctx = P.Context(0)
    t0 = time.perf_counter()
    ctx.build_bvh(sc)
    torch.cuda.synchronize()
    log(f"[bench] GPU BVH built in {time.perf_counter() - t0:.2f}s")
    H, W = cam["height"], cam["width"]
    base = {"max_depth": rs["max_depth"], "seed": rs["seed"]}

    # traversal counters of one pass (algorithmic bytes per ray), untimed
    ctx.set_profiling(2)
    s_img = torch.zeros((H, W, 3), device="cuda", dtype=torch.float32)
    s2_img = torch.zeros_like(s_img)
    ctx.render(cam, dict(base, spp=1, sample_offset=10_000), s_img, s2_img)
    cnt = ctx.render_stats()
    ctx.sync()
    log(f"[bench] counters: {json.dumps(cnt)}")
    coll_rays_c = max(cnt["collision_rays"], 1)
    n_node = cnt["cat_nodes"][0] / coll_rays_c
    n_prim = cnt["cat_prims"][0] / coll_rays_c
    n_reload = cnt["cat_reloads"][0] / coll_rays_c
    alg_bytes_per_ray = ALG_NODE_B * n_node + ALG_PRIM_B * n_prim + ALG_RAY_B
    layout_bytes_per_ray = NODE_B * n_node + PRIM_B * (n_prim + n_reload) + PATH_B

    # warm-up then timed passes (kernel durations from HIP events)
    ctx.set_profiling(1)
    s_img.zero_()
    s2_img.zero_()
    if args.warmup > 0:
        ctx.render(cam, dict(base, spp=args.warmup, sample_offset=0), s_img, s2_img)
    torch.cuda.synchronize()
    s_img.zero_()
    s2_img.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.render(cam, dict(base, spp=args.steps, sample_offset=args.warmup), s_img, s2_img)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.render_stats()
    ctx.sync()
    rays = st["rays"]
    mrays = rays / dt / 1e6
    img = (s_img / args.steps).clamp(0, 1)
    mean_pix = float(img.mean())
    log(f"[bench] {args.steps} passes in {dt:.3f}s: {rays} rays ({st['collision_rays']} collision, "
        f"{st['light_rays']} light, {st['env_rays']} env), {mrays:.1f} Mrays/s, "
        f"{st['paths'] / dt / 1e6:.2f} M paths/s; mean clamped pixel {mean_pix:.4f}")
    log(f"[bench] kernel ms: collide {st['ms_collide']:.1f} ({st['launches_collide']} launches), "
        f"overflow {st['ms_collide_wide']:.2f}, light {st['ms_light']:.1f}, env {st['ms_env']:.1f}, "
        f"shade {st['ms_shade']:.1f}, sort {st['ms_sort']:.1f}")

    launches = max(st["launches_collide"], 1)
    rays_per_launch = st["collision_rays"] / launches
    launch_s = st["ms_collide"] / launches * 1e-3
    achieved = alg_bytes_per_ray * rays_per_launch / launch_s / 1e9
    traffic = measured_traffic()
    if traffic is not None:
        traffic *= rays_per_launch  # HBM bytes per launch of this run
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch",
                "kernel": "k_collide (main)",
                "bytes_per_ray": round(alg_bytes_per_ray, 1),
                "bytes_formula": "64 n_node + 64 n_prim + 32 per collision ray",
                "nodes_per_ray": round(n_node, 2), "prims_per_ray": round(n_prim, 2),
                "rays_per_launch": round(rays_per_launch, 1),
                "mean_launch_ms": round(st["ms_collide"] / launches, 4), "launches": launches,
                "traffic_gbs": None if traffic is None else round(traffic / launch_s / 1e9, 1),
                "layout_model": {"bytes_per_ray": round(layout_bytes_per_ray, 1),
                                 "reloads_per_ray": round(n_reload, 2),
                                 "gbs": round(layout_bytes_per_ray * rays_per_launch / launch_s / 1e9, 1)}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, cam, base, args.cpu_seconds)

    ttr = None
    if not args.no_time_to_rmse:
        # the second half of the metric, bounded: 240x135 (1/64 of the pixels),
        # 128 spp per call, caps of 45 s (plain, then extrapolated from its
        # 1/t squared-error law), 110 s (cached: long enough to reach the
        # target) and 10 s (ablations)
        import copy
        a2 = copy.copy(args)
        a2.rmse_res, a2.rmse_wavefront = "240x135", 128
        a2.rmse_seconds, a2.rmse_seconds_nrc, a2.rmse_seconds_ablation = 45.0, 110.0, 10.0
        ttr = time_to_rmse(a2, ctx=ctx, sc=sc, bounded=True)
        for r in ttr["runs"].values():
            r.pop("curve", None)

    out = {"metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "room_5p5m: 5.5M Gaussian primitives (room of boxes and planes tiled "
                                  "with flat Gaussians, 40 clusters of elongated Gaussians, 2 emissive "
                                  "panels), 1920x1080, 1 spp per step, max depth 12",
                      "primitives": int(sc["mean"].shape[0]), "resolution": "1920x1080",
                      "max_depth": rs["max_depth"], "paths_per_s": round(st["paths"] / dt, 1),
                      "mean_clamped_pixel": round(mean_pix, 4)},
           "roofline": roofline, "cpu_baseline": cpu, "time_to_rmse": ttr}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
