"""Density adjoint of the path tracer (ugp_render_density_grad, a
score-function estimate by path replay) against the derivative of the
expected image.

Depth 0 (the camera collision only): the expected image of given camera
rays is the radiance-field sum of eq. rf, sum_k W_k L_e,k, which the FP64
oracle evaluates exactly; its central differences in the densities (along
random directions and per primitive) are the exact derivative.  The oracle's
own camera rays of each sample are used (same jitter stream as the GPU's).
Depth 3 with light and environment samples: against central differences of
the GPU's expected image (common random numbers, many samples), and the
light-only and MIS estimates of the derivative agree.

The adjoint is a Monte Carlo estimate: each comparison runs B batches
(seeds) and requires the mean of (adjoint - reference) over the batches to lie
within 4.5 standard errors of zero, and the adjoint to carry most of the
reference's magnitude (a sign or a factor error fails that)."""
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
    c = P.Context(0)
    yield c
    c.close()


def _scene():
    # c0 with 100 emitters of varied colour and denser primitives, so that
    # rays saturate and t_sat terms occur
    sc = scenes.tiny_random(n_emit=0)
    rng = np.random.default_rng(31)
    sc["density"] = (sc["density"] * 4.0).astype(np.float32)
    idx = rng.choice(sc["mean"].shape[0], 100, replace=False)
    sc["emission"][idx] = rng.uniform(1.0, 6.0, (100, 3)).astype(np.float32)
    return sc


def _stats(d):
    d = np.asarray(d, np.float64)
    return d.mean(0), d.std(0, ddof=1) / np.sqrt(d.shape[0])


def test_density_adjoint_depth0_vs_oracle_exact(ctx, orc, torch):
    _say("density adjoint at depth 0 vs central differences of the oracle's expected image (eq. rf)")
    sc = _scene()
    n = sc["mean"].shape[0]
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    spp, B = 128, 12
    seeds = [500 + b for b in range(B)]
    rng = np.random.default_rng(5)
    g = rng.uniform(-1, 1, (16, 16, 3)).astype(np.float32)
    V = rng.normal(size=(3, n))
    ctx.build_bvh(sc)
    G = []
    for b in range(B):
        grad = torch.zeros(n, device="cuda", dtype=torch.float32)
        ctx.render_density_grad(cam, {"spp": spp, "max_depth": 0, "seed": seeds[b]}, g, grad)
        G.append(grad.cpu().numpy().astype(np.float64))
    ctx.sync()
    G = np.array(G)
    # the oracle's exact expectation for each batch's rays
    rays = [np.concatenate([orc.camera_rays(cam, seeds[b], s) for s in range(spp)]) for b in range(B)]
    gw = np.tile(g.reshape(-1, 3).astype(np.float64), (spp, 1)) / spp

    def loss(dens, b):
        s2 = dict(sc, density=dens.astype(np.float32))
        return float((orc.Scene(s2).rf_radiance(rays[b]) * gw).sum())

    d0 = sc["density"].astype(np.float64)
    # directional derivatives
    D, ref_mag = [], []
    for v in V:
        h = 1e-3 * d0 * v
        fd = np.array([(loss(d0 + h, b) - loss(d0 - h, b)) / 2e-3 for b in range(B)])
        D.append(G @ (d0 * v) - fd)
        ref_mag.append(np.abs(fd).mean())
    D = np.array(D).T  # [B, 3]
    m, se = _stats(D)
    _say(f"  directional: adjoint - FD mean {m}, s.e. {se}, |FD| {np.array(ref_mag)}")
    assert np.all(np.abs(m) <= 4.5 * se + 1e-9)
    # per primitive, for the primitives with the largest gradients
    top = np.argsort(-np.abs(G.mean(0)))[:5]
    Dp, mags = [], []
    for j in top:
        e = np.zeros(n)
        e[j] = 1e-3 * d0[j]
        fd = np.array([(loss(d0 + e, b) - loss(d0 - e, b)) / (2 * e[j]) for b in range(B)])
        Dp.append(G[:, j] - fd)
        mags.append(np.abs(fd.mean()))
    Dp = np.array(Dp).T
    m, se = _stats(Dp)
    _say(f"  per primitive {top.tolist()}: adjoint - FD mean {m}, s.e. {se}, |FD| {np.array(mags)}")
    assert np.all(np.abs(m) <= 4.5 * se + 1e-9)
    # the adjoint carries the reference's magnitude (not swamped by its noise)
    assert np.all(se < 0.35 * np.array(mags))


def _render_mean(ctx, torch, cam, p, g):
    s, _ = ctx.render(cam, dict(p, want_sumsq=False))
    return float((s.cpu().numpy().astype(np.float64) * g).sum()) / p["spp"]


@pytest.mark.parametrize("mis_mode", [0, 2])
def test_density_adjoint_depth3_vs_gpu_differences(ctx, torch, mis_mode):
    _say(f"density adjoint at depth 3 (mis_mode {mis_mode}) vs central differences of the expected image")
    sc = _scene()
    n = sc["mean"].shape[0]
    cam = dict(scenes.camera("tiny_random"), width=24, height=24)
    spp, B = 2048, 8
    rng = np.random.default_rng(6)
    g = rng.uniform(0, 1, (24, 24, 3)).astype(np.float64)
    v = rng.normal(size=n)
    d0 = sc["density"].astype(np.float64)
    base = {"spp": spp, "max_depth": 3, "env_radiance": (0.3, 0.35, 0.4), "mis_mode": mis_mode}
    D, F = [], []
    for b in range(B):
        p = dict(base, seed=300 + b)
        ctx.build_bvh(sc)
        grad = torch.zeros(n, device="cuda", dtype=torch.float32)
        ctx.render_density_grad(cam, p, g.astype(np.float32), grad)
        adj = float(grad.cpu().numpy().astype(np.float64) @ (d0 * v))
        h = 0.02
        ctx.build_bvh(dict(sc, density=(d0 * (1 + h * v)).astype(np.float32)))
        lp = _render_mean(ctx, torch, cam, p, g)
        ctx.build_bvh(dict(sc, density=(d0 * (1 - h * v)).astype(np.float32)))
        lm = _render_mean(ctx, torch, cam, p, g)
        fd = (lp - lm) / (2 * h)
        D.append(adj - fd)
        F.append(fd)
    ctx.sync()
    m, se = _stats(D)
    _say(f"  adjoint - FD mean {m:.4g}, s.e. {se:.3g}; FD mean {np.mean(F):.4g}")
    assert abs(m) <= 4.5 * se + 1e-9
    assert se < 0.35 * abs(np.mean(F))


def test_density_adjoint_refuses_the_cache(ctx, torch):
    import paper_2406_09733_amd as P
    sc = _scene()
    ctx.build_bvh(sc)
    cam = dict(scenes.camera("tiny_random"), width=8, height=8)
    with pytest.raises(P.UGPError):
        ctx.render_density_grad(cam, {"spp": 1, "max_depth": 2, "nrc_mode": 2}, np.ones((8, 8, 3), np.float32),
                                torch.zeros(sc["mean"].shape[0], device="cuda"))


def test_autograd_density_fit(ctx, torch):
    # densities perturbed by up to e^(+-0.7), recovered through autograd.render
    # (ugp_render_density_grad) with Adam against a 1024-spp target; each step
    # renders 64 spp with a fresh seed, and its backward another 64 spp with
    # another seed (a gradient from the image's own samples would be biased
    # by the correlation of the residual's noise with the score terms)
    from paper_2406_09733_amd import autograd as A
    _say("density fit through the path tracer's density adjoint")
    sc = scenes.tiny_random(n_emit=30)
    n = sc["mean"].shape[0]
    cam = dict(scenes.camera("tiny_random"), width=32, height=32)
    rp = {"max_depth": 2, "env_radiance": (0.3, 0.3, 0.3)}
    truth = {k: torch.tensor(np.asarray(v), device="cuda") for k, v in sc.items() if k != "bounds"}
    target = A.render(ctx, truth, cam, dict(rp, spp=1024, seed=1)).detach()
    d_true = np.asarray(sc["density"], np.float64)
    rng = np.random.default_rng(3)
    d0 = d_true * np.exp(rng.uniform(-0.7, 0.7, n))
    params = dict(truth)
    logd = torch.tensor(np.log(d0).astype(np.float32), device="cuda", requires_grad=True)
    opt = torch.optim.Adam([logd], lr=0.05)
    # the primitives the view sees most (density gradient of the plain image sum)
    ctx.build_bvh(sc)
    seen_g = torch.zeros(n, device="cuda")
    ctx.render_density_grad(cam, dict(rp, spp=64, seed=7), np.ones((32, 32, 3), np.float32), seen_g)
    seen = np.argsort(-np.abs(seen_g.cpu().numpy()))[:40]
    err0 = np.abs(np.log(d0[seen]) - np.log(d_true[seen])).mean()
    losses = []
    for it in range(80):
        params["density"] = torch.exp(logd)
        img = A.render(ctx, params, cam, dict(rp, spp=64, seed=100 + it), backward_params={"seed": 5000 + it})
        loss = ((img - target) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    d1 = np.exp(logd.detach().cpu().numpy().astype(np.float64))
    err1 = np.abs(np.log(d1[seen]) - np.log(d_true[seen])).mean()

    def image_err(d):
        # at 1024 spp (another seed): the per-step losses are dominated by the
        # 64-spp noise
        p = dict(params, density=torch.tensor(d.astype(np.float32), device="cuda"))
        with torch.no_grad():
            img = A.render(ctx, p, cam, dict(rp, spp=1024, seed=9))
        return float(((img - target) ** 2).mean())

    e0, e1 = image_err(d0), image_err(d1)
    _say(f"  per-step loss {np.mean(losses[:5]):.3e} -> {np.mean(losses[-5:]):.3e}; image error at 1024 spp "
         f"{e0:.3e} -> {e1:.3e}; log-density error of the 40 most visible primitives {err0:.3f} -> {err1:.3f}")
    assert e1 < 0.7 * e0
    assert err1 < 0.7 * err0
