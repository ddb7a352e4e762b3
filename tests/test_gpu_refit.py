"""GPU tests of ugp_refit_bvh: after new parameters are refitted into the
hierarchy of the old ones, every query matches the oracle of the NEW scene
(the same bar as the parity tests), also after large moves and for cut
(slab) primitives; a render after a refit that changes the emitters matches
a render of a fresh build; bad calls leave the scene unchanged.

Tolerances (as tests/test_gpu_parity.py):
  T        |dT| <= 1e-5
  t_sat    |dt| <= 1e-5 max(|t|, 1e-3), or F_oracle(t_gpu) within 2e-5 of 1
  prim     identical wherever the oracle's margin exceeds 1e-5
"""
import sys

import numpy as np
import pytest

from paper_2406_09733_amd import scenes

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2406_09733_amd as P
    return P.Context(0)


def _np(t):
    return t.detach().cpu().numpy()


def _check_queries(ctx, orc, sc, nr, seed):
    S = orc.Scene(sc)
    rays = scenes.probe_rays(sc, nr, seed=seed)
    F_ref, T_ref = S.transmittance(rays)
    T, _ = ctx.transmittance(rays)
    dT = np.abs(_np(T) - T_ref).max()
    assert dT <= 1e-5, dT
    u = np.random.default_rng(seed).uniform(0, 1, nr).astype(np.float32)
    ref = S.sample_collision(rays, u.astype(np.float64))
    prim, _ = ctx.sample_collision(rays, u)
    clear = ref["margin"] > 1e-5
    mism = int(((_np(prim) != ref["prim"]) & clear).sum())
    assert mism == 0, mism
    ts_ref = S.saturation(rays)
    ts = _np(ctx.saturation(rays)).astype(np.float64)
    t1 = rays[:, 7].astype(np.float64)
    assert ((ts == t1) == (ts_ref == t1)).mean() > 0.999
    sat = (ts_ref < t1) & (ts < t1)
    ok = np.abs(ts[sat] - ts_ref[sat]) <= 1e-5 * np.maximum(np.abs(ts_ref[sat]), 1e-3)
    ok |= np.abs(S.F_at(rays[sat], ts[sat]) - 1.0) <= 2e-5
    assert ok.all()
    ctx.sync()
    return dT


@pytest.mark.parametrize("name", ["tiny_random", "mixed_100k", "needles"])
def test_refit_queries_match_the_new_scene(ctx, orc, torch, name):
    _say("refit parity", name)
    sc = {"tiny_random": scenes.tiny_random, "mixed_100k": scenes.mixed_100k, "needles": scenes.needles}[name]()
    ctx.build_bvh(sc)
    moved = scenes.perturbed(sc, seed=7)
    ctx.refit_bvh(moved)
    dT = _check_queries(ctx, orc, moved, 2048, 401)
    _say(f"  max |dT| {dT:.2e}")


def test_refit_after_large_moves(ctx, orc, torch):
    _say("refit after the means are shuffled")
    sc = scenes.needles()
    ctx.build_bvh(sc)
    moved = dict(sc)
    perm = np.random.default_rng(3).permutation(sc["mean"].shape[0])
    moved["mean"] = np.ascontiguousarray(sc["mean"][perm])
    ctx.refit_bvh(moved)
    _check_queries(ctx, orc, moved, 2048, 402)


def test_refit_render_with_new_emitters(ctx, torch):
    _say("render after a refit that changes the emitters vs a fresh build")
    sc = scenes.tiny_random()
    moved = scenes.perturbed(sc, seed=9, pos=0.2)
    rng = np.random.default_rng(4)
    moved["emission"] = np.zeros_like(sc["emission"])
    moved["emission"][rng.choice(sc["mean"].shape[0], 25, replace=False)] = 4.0
    cam = dict(scenes.camera("tiny_random"), width=64, height=64)
    p = {"spp": 8, "max_depth": 4, "seed": 3, "want_sumsq": False}
    ctx.build_bvh(moved)
    ref, _ = ctx.render(cam, p)
    ref = _np(ref)
    ctx.build_bvh(sc)
    ctx.refit_bvh(moved)
    img, _ = ctx.render(cam, p)
    img = _np(img)
    ctx.sync()
    diff = np.abs(img - ref)
    # the same estimator on another hierarchy: equal up to float summation
    # order (a path may rarely take another decision near a margin)
    frac = float((diff > 1e-4 * max(1.0, ref.max())).mean())
    _say(f"  mean image {img.mean():.5f} vs {ref.mean():.5f}; values off by > 1e-4: {frac:.4f}")
    assert frac < 0.01
    assert abs(img.mean() - ref.mean()) <= 1e-3 * ref.mean()


def test_refit_rejects_bad_calls_and_keeps_the_scene(ctx, orc, torch):
    import paper_2406_09733_amd as P
    sc = scenes.tiny_random()
    ctx.build_bvh(sc)
    rays = scenes.probe_rays(sc, 512, seed=403)
    T0 = _np(ctx.transmittance(rays)[0])
    small = {k: (v[:10] if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    with pytest.raises(P.UGPError) as e:
        ctx.refit_bvh(small)
    assert e.value.code == 1
    bad = dict(sc)
    bad["scale"] = np.array(sc["scale"], copy=True)
    bad["scale"][5, 1] = -1.0
    with pytest.raises(P.UGPError) as e:
        ctx.refit_bvh(bad)
    assert e.value.code == 1
    T1 = _np(ctx.transmittance(rays)[0])
    ctx.sync()  # no deferred error is left behind by the rejected calls
    assert np.array_equal(T0, T1)
    # a rejected build keeps the built scene too
    with pytest.raises(P.UGPError) as e:
        ctx.build_bvh(bad)
    assert e.value.code == 1
    T2 = _np(ctx.transmittance(rays)[0])
    ctx.sync()
    assert np.array_equal(T0, T2)
