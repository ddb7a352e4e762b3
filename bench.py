#!/usr/bin/env python3
"""Benchmark: Monte Carlo path tracing of the 5.5M-primitive room workload on
one MI355X, reported as traversal queries per second (Mrays/s).

One step = one sample pass over the whole hot path: camera rays for every
pixel of the 1920x1080 image, then per vertex (max depth 12) primitive-level
free-flight sampling, emission pick-up, next-event estimation (emitter query
along a sampled cone direction) and phase sampling, then accumulation.  A
"ray" is one traversal query (collision, emitter or environment query).

The scene, camera and seeds are synthetic and fixed (see
paper_2406_09733_amd/scenes.py); inputs are resident in HBM before timing.

Besides the JSON line's throughput it reports:
  roofline     the dominant kernel (the collision kernel): algorithmic bytes
               per launch (4-wide BVH node records 128 B, primitive records 64 B,
               re-read records 64 B, path-queue records 96 B per ray) divided
               by its mean launch duration from HIP events recorded around
               every launch during the timed run, against 8 TB/s HBM;
  cpu_baseline the FP64 CPU oracle on a bounded pixel subset of the same
               workload, on this host's cores.
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
NODE_B, PRIM_B, PATH_B = 128, 64, 96


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sc, cam, params, target_s: float):
    """Time the FP64 oracle on an evenly spaced pixel subset at 1 spp."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    S = oracle.Scene(sc)
    log(f"[cpu] oracle scene + BVH ready in {time.perf_counter() - t0:.1f}s")
    npix = cam["width"] * cam["height"]
    nthreads = os.cpu_count() or 1
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
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": nthreads, "kind": "oracle",
            "sample": f"every {stride}th pixel of 1920x1080 ({len(pix)} camera paths), 1 spp, "
                      f"max depth {params['max_depth']}, {rays} rays in {dt:.1f}s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed sample passes")
    ap.add_argument("--warmup", type=int, default=2, help="untimed sample passes")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path shards by "
              "pixels with no communication beyond a final image reduction; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

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
    bytes_per_coll_ray = (NODE_B * cnt["cat_nodes"][0] + PRIM_B * cnt["cat_prims"][0] +
                          PRIM_B * cnt["cat_reloads"][0]) / coll_rays_c + PATH_B

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
    achieved = (bytes_per_coll_ray * st["collision_rays"] / launches) / (st["ms_collide"] / launches * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_collide (main)", "bytes_per_ray": round(bytes_per_coll_ray, 1),
                "nodes_per_ray": round(cnt["cat_nodes"][0] / coll_rays_c, 2),
                "prims_per_ray": round(cnt["cat_prims"][0] / coll_rays_c, 2),
                "reloads_per_ray": round(cnt["cat_reloads"][0] / coll_rays_c, 2),
                "mean_launch_ms": round(st["ms_collide"] / launches, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, cam, base, args.cpu_seconds)

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
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
