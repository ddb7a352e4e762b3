"""GPU tests of the roughness adjoint of the path tracer
(ugp_render_roughness_grad, path replay with d log f / d roughness of the
glossy lobe at every vertex).

* Direct lighting by light sampling only (mis_mode 2, max_depth 1): no
  sampling decision depends on the roughness there, so the image is a smooth
  function of it and central differences of the GPU's own render with the
  same random numbers give the derivative up to O(h^2) and float rounding;
  the same against FP64 central differences of the oracle's render.
* Several bounces: the phase samples move with the roughness, so the adjoint
  estimates the derivative of the expected image.  Light sampling only,
  phase sampling only and MIS estimate the same expected image, so their
  gradients must agree within their Monte Carlo errors (the phase-sampling
  estimator exercises the continuation's ratio alone).

Tolerances:
  vs GPU differences     |g - fd| <= 3e-3 |g| + 1e-3 (the O(h^2) term of the
                          difference at h = 0.004 reaches 1e-3 |g| at roughness 0.17)
  vs oracle differences  |g dr - d loss| <= 3e-2 |g dr| + 2e-5
  MIS modes              |g_a - g_b| <= 4.5 sigma (sigma from 8 independent renders each)
"""
import math
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


def _scene():
    sc = scenes.tiny_random(seed=3, n_emit=120)
    rng = np.random.default_rng(13)
    n = sc["mean"].shape[0]
    sc["material"] = (rng.uniform(0, 1, n) < 0.8).astype(np.int32)  # mostly glossy
    sc["roughness"] = rng.uniform(0.15, 0.9, n).astype(np.float32)
    sc["density"] = (np.asarray(sc["density"]) * 6.0).astype(np.float32)
    return sc


CAM = dict(scenes.camera("tiny_random"), width=48, height=48)
DIRECT = {"spp": 4, "max_depth": 1, "seed": 9, "env_radiance": (0.3, 0.3, 0.3), "mis_mode": 2}


def _weights(seed=2, res=48):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (res, res, 3)).astype(np.float32)


def _gpu_loss(ctx, sc, w, params):
    ctx.build_bvh(sc)
    s, _ = ctx.render(CAM, dict(params, want_sumsq=False))
    ctx.sync()
    img = s.cpu().numpy().astype(np.float64) / params["spp"]
    return float(np.sum(w.astype(np.float64) * img))


def _grad(ctx, torch, sc, w, params, cam=CAM):
    ctx.build_bvh(sc)
    g = torch.zeros(sc["mean"].shape[0], device="cuda", dtype=torch.float32)
    ctx.render_roughness_grad(cam, params, torch.tensor(w, device="cuda"), g)
    ctx.sync()
    return g.cpu().numpy().astype(np.float64)


def _probe(g, sc, k=8, seed=0):
    glossy = np.asarray(sc["material"]) == 1
    mag = np.where(glossy, np.abs(g), 0)
    top = list(np.argsort(-mag)[:6])
    rest = np.where(mag > 0)[0]
    rng = np.random.default_rng(seed)
    return top + [int(x) for x in rng.choice(np.setdiff1d(rest, top), 2, replace=False)]


def test_roughness_gradient_vs_gpu_differences(ctx, torch):
    _say("roughness adjoint vs central differences of the GPU render (direct light, light sampling)")
    sc = _scene()
    w = _weights()
    g = _grad(ctx, torch, sc, w, DIRECT)
    assert np.all(g[np.asarray(sc["material"]) == 0] == 0)
    h = 0.004
    for k in _probe(g, sc):
        vals = []
        for sgn in (1, -1):
            s2 = dict(sc)
            r = np.asarray(sc["roughness"], np.float32).copy()
            r[k] = np.float32(r[k] + sgn * h)
            s2["roughness"] = r
            vals.append(_gpu_loss(ctx, s2, w, DIRECT))
        fd = (vals[0] - vals[1]) / (2 * h)
        tol = 3e-3 * abs(g[k]) + 1e-3
        _say(f"  prim {k} (roughness {sc['roughness'][k]:.3f}): g {g[k]:.6e} fd {fd:.6e} |diff| {abs(g[k] - fd):.2e}"
             f" tol {tol:.2e}")
        assert abs(g[k] - fd) <= tol


def test_roughness_gradient_vs_oracle_differences(ctx, orc, torch):
    _say("roughness adjoint vs FP64 central differences of the oracle's render (direct light)")
    sc = _scene()
    w = _weights(3)
    g = _grad(ctx, torch, sc, w, DIRECT)

    def oracle_loss(s2):
        s, _, _ = orc.Scene(s2).render(CAM, DIRECT)
        return float(np.sum(w.reshape(-1, 3).astype(np.float64) * s / DIRECT["spp"]))

    h = 0.004
    for k in _probe(g, sc, seed=1)[:6]:
        vals = []
        for sgn in (1, -1):
            s2 = dict(sc)
            r = np.asarray(sc["roughness"], np.float32).copy()
            r[k] = np.float32(r[k] + sgn * h)
            s2["roughness"] = r
            vals.append((float(r[k]), oracle_loss(s2)))
        dr = vals[0][0] - vals[1][0]
        dl = vals[0][1] - vals[1][1]
        _say(f"  prim {k}: g dr {g[k] * dr:.6e} oracle difference {dl:.6e}")
        assert abs(g[k] * dr - dl) <= 3e-2 * abs(g[k] * dr) + 2e-5


def test_roughness_gradient_mis_modes_agree(ctx, torch):
    _say("roughness adjoint: light-only, phase-only and MIS estimates of the derivative agree (depth 3)")
    sc = _scene()
    cam = dict(CAM, width=64, height=64)
    w = _weights(4, 64)
    proj = np.random.default_rng(5).choice([-1.0, 1.0], sc["mean"].shape[0])
    res = {}
    for mode in (0, 1, 2):
        vals = []
        for rep in range(8):
            p = {"spp": 64, "max_depth": 3, "seed": 100 * mode + rep, "env_radiance": (0.3, 0.3, 0.3),
                 "mis_mode": mode}
            vals.append(float(_grad(ctx, torch, sc, w, p, cam) @ proj))
        res[mode] = (np.mean(vals), np.std(vals, ddof=1) / math.sqrt(len(vals)))
        _say(f"  mode {mode}: {res[mode][0]:.5e} +- {res[mode][1]:.2e}")
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(res[a][0] - res[b][0]) <= 4.5 * math.hypot(res[a][1], res[b][1]), res


def test_roughness_gradient_refusals(ctx, torch):
    import paper_2406_09733_amd as P
    sc = scenes.with_sggx(scenes.tiny_random(n=200, n_emit=5), seed=0, frac=0.5, base="disney")
    ctx.build_bvh(sc)
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    d_img = torch.ones((16, 16, 3), device="cuda")
    with pytest.raises(P.UGPError):
        ctx.render_roughness_grad(cam, {"spp": 1, "max_depth": 2, "seed": 0}, d_img,
                                  torch.zeros(200, device="cuda"))
    ctx.build_bvh(scenes.tiny_random(n=200, n_emit=5))
    with pytest.raises(P.UGPError):
        ctx.render_roughness_grad(cam, {"spp": 1, "max_depth": 2, "seed": 0, "nrc_mode": 2}, d_img,
                                  torch.zeros(200, device="cuda"))


def test_autograd_render_roughness_fit(ctx, torch):
    # gradient descent on the roughness through autograd.render under direct
    # light by light sampling with common random numbers: there the image is
    # a smooth function of the roughness and the adjoint is its exact
    # derivative, so the fit is a deterministic optimisation whose minimum is
    # the true roughness (with fresh seeds per step the roughness signal of
    # this scene drowns in the Monte Carlo noise of small renders)
    from paper_2406_09733_amd import autograd as A
    _say("autograd render: fit roughness to an image (direct light, light sampling, same seed)")
    sc = _scene()
    truth = {k: torch.tensor(np.asarray(v), device="cuda") for k, v in sc.items() if k != "bounds"}
    rp = dict(DIRECT, seed=50)
    target = A.render(ctx, truth, CAM, rp).detach()
    n = sc["mean"].shape[0]
    r_true = np.asarray(sc["roughness"], np.float64)
    r0 = np.clip(r_true + np.random.default_rng(7).uniform(-0.3, 0.3, n), 0.1, 0.95)
    params = dict(truth)
    params["roughness"] = torch.tensor(r0.astype(np.float32), device="cuda", requires_grad=True)
    opt = torch.optim.Adam([params["roughness"]], lr=0.02)
    losses = []
    for it in range(80):
        img = A.render(ctx, params, CAM, rp)
        loss = ((img - target) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            params["roughness"].clamp_(0.05, 1.0)
        losses.append(float(loss.item()))
    g = _grad(ctx, torch, sc, np.ones((48, 48, 3), np.float32), DIRECT)
    seen = np.argsort(-np.abs(g))[:20]
    r1 = params["roughness"].detach().cpu().numpy().astype(np.float64)
    err0 = np.abs(r0[seen] - r_true[seen]).mean()
    err1 = np.abs(r1[seen] - r_true[seen]).mean()
    _say(f"  image loss {losses[0]:.4e} -> {np.mean(losses[-5:]):.4e}; roughness error of the 20 most"
         f" sensitive primitives {err0:.3f} -> {err1:.3f}")
    assert np.mean(losses[-5:]) < 0.1 * losses[0]
    assert err1 < 0.5 * err0
