"""GPU parity of the exponential variant (App. D; eq. exp_ff) with the oracle:
transmittance exp(-sum I_k), and analog decomposition tracking with the same
counter-based uniforms on both sides, per ray and as a render mode
(ugp_render_params.transport = 1).

Tolerances:
  T      |gpu - oracle| <= 1e-5 max(T, 1e-3)  (float sum of the ray integrals)
  prim   identical wherever the oracle's margin (collide-or-not decision and
         the gap between the two nearest collisions, relative) exceeds 1e-4
  t      |gpu - oracle| <= 1e-4 |t| + 1e-6 there (FP64 inverse of float chord data)
  image  at most 1% of pixels beyond 3 sigma of the two renders' Monte Carlo
         noise, image means within 3 standard errors (the same random numbers
         drive both, so most pixels agree to rounding)
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


@pytest.mark.parametrize("name", ["tiny_random", "mixed_100k", "needles"])
def test_exp_parity(ctx, orc, torch, name):
    sc = {"tiny_random": scenes.tiny_random, "mixed_100k": scenes.mixed_100k, "needles": scenes.needles}[name]()
    rays = scenes.probe_rays(sc, 4096, seed=301)
    rng = np.random.default_rng(8)
    ex = rng.integers(-1, sc["mean"].shape[0], rays.shape[0]).astype(np.int32)
    ex[::2] = -1
    S = orc.Scene(sc)
    T_ref = S.exp_transmittance(rays, ex)
    p_ref, t_ref, margin = S.exp_sample(rays, seed=77, exclude=ex)
    ctx.build_bvh(sc)
    T = ctx.exp_transmittance(rays, ex).cpu().numpy().astype(np.float64)
    p, t = ctx.exp_sample_collision(rays, 77, ex)
    p = p.cpu().numpy()
    t = t.cpu().numpy().astype(np.float64)
    ctx.sync()
    assert np.all(np.abs(T - T_ref) <= 1e-5 * np.maximum(T_ref, 1e-3))
    clear = margin > 1e-4
    _say(f"  {name}: collisions {np.mean(p_ref >= 0):.3f}; ambiguous {int((~clear).sum())} of {len(p)};"
         f" max |dT| {np.abs(T - T_ref).max():.2e}")
    assert np.array_equal(p[clear], p_ref[clear])
    hit = clear & (p_ref >= 0)
    assert np.all(np.abs(t[hit] - t_ref[hit]) <= 1e-4 * np.abs(t_ref[hit]) + 1e-6)
    assert np.all(np.isnan(t[clear & (p_ref < 0)]))


def _exp_image_parity(ctx, orc, sc, name, spp, depth, seed, res, extra=None):
    cam = dict(scenes.camera(name), width=res[0], height=res[1])
    p = {"spp": spp, "max_depth": depth, "seed": seed, "transport": 1}
    if extra:
        p.update(extra)
    s_ref, s2_ref, _ = orc.Scene(sc).render(cam, p)
    ctx.build_bvh(sc)
    s, s2 = ctx.render(cam, p)
    ctx.sync()
    s = s.cpu().numpy().reshape(-1, 3).astype(np.float64)
    s2 = s2.cpu().numpy().reshape(-1, 3).astype(np.float64)
    m, m_ref = s / spp, s_ref / spp
    v = np.maximum(s2 / spp - m ** 2, 0) / spp
    v_ref = np.maximum(s2_ref / spp - m_ref ** 2, 0) / spp
    z = np.abs(m - m_ref) / np.sqrt(v + v_ref + 1e-12)
    frac = float((z > 3).mean())
    gse = np.sqrt((v + v_ref).sum()) / m.size
    _say(f"  {name} (exponential): mean gpu {m.mean():.6f} oracle {m_ref.mean():.6f} se {gse:.2e};"
         f" pixels beyond 3 sigma {frac:.4f}; identical pixels {(np.abs(m - m_ref) < 1e-4).mean():.3f}")
    assert np.all(np.isfinite(m))
    return frac, abs(m.mean() - m_ref.mean()), gse, m_ref.mean()


@pytest.mark.parametrize("name,depth,res,extra", [
    ("tiny_random", 4, (96, 96), {"env_radiance": (0.2, 0.3, 0.4)}),
    ("mixed_100k", 6, (96, 96), None),
    ("needles", 5, (80, 80), {"env_radiance": (0.1, 0.1, 0.1)}),
])
def test_exp_render_parity(ctx, orc, torch, name, depth, res, extra):
    _say(f"exponential render parity {name} {res[0]}x{res[1]} 4 spp depth {depth}")
    sc = {"tiny_random": scenes.tiny_random, "mixed_100k": scenes.mixed_100k, "needles": scenes.needles}[name]()
    frac, d, se, mean = _exp_image_parity(ctx, orc, sc, name, 4, depth, 11, res, extra)
    assert frac < 0.01
    assert d <= 3 * se + 1e-6
    assert mean > 0


def test_exp_render_is_not_the_linear_render(ctx, torch):
    # the switch changes the transport: with no emitters, a unit environment
    # and no scattering (max_depth 0) a pixel is the probability of escape,
    # 1 - I/2 (clamped) against exp(-I); the image means differ far beyond
    # their standard errors (the oracle gives 0.893 and 0.819 here)
    sc = scenes.tiny_random(n_emit=0)
    ctx.build_bvh(sc)
    cam = dict(scenes.camera("tiny_random"), width=48, height=48)
    p = {"spp": 64, "max_depth": 0, "seed": 3, "env_radiance": (1.0, 1.0, 1.0)}
    out = {}
    for tr in (0, 1):
        s, s2 = ctx.render(cam, dict(p, transport=tr))
        ctx.sync()
        m = s.cpu().numpy().astype(np.float64)[..., 0] / 64
        q = s2.cpu().numpy().astype(np.float64)[..., 0] / 64
        out[tr] = (m, np.maximum(q - m * m, 0) / 64)
    d = abs(out[0][0].mean() - out[1][0].mean())
    se = np.sqrt(out[0][1].sum() + out[1][1].sum()) / out[0][0].size
    _say(f"  escape probability: linear {out[0][0].mean():.4f}, exponential {out[1][0].mean():.4f}"
         f" (standard error of the difference {se:.1e})")
    assert d > 10 * se


def test_exp_render_refusals(ctx, torch):
    import paper_2406_09733_amd as P
    sc = scenes.tiny_random()
    ctx.build_bvh(sc)
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    box = (-0.5, -0.5, -0.5, 1.5, 1.5, 1.5)
    with pytest.raises(P.UGPError) as e:  # no radiance cache in the exponential variant
        ctx.render(cam, {"spp": 1, "max_depth": 2, "transport": 1, "nrc_mode": 3, "nrc_box": box})
    assert e.value.code == 5
    with pytest.raises(P.UGPError) as e:
        ctx.render(cam, {"spp": 1, "max_depth": 2, "transport": 2})
    assert e.value.code == 1
    g = torch.zeros((sc["mean"].shape[0], 3), device="cuda", dtype=torch.float32)
    d = torch.zeros((16, 16, 3), device="cuda", dtype=torch.float32)
    with pytest.raises(P.UGPError) as e:  # nor adjoints
        ctx.render_albedo_grad(cam, {"spp": 1, "max_depth": 2, "transport": 1}, d, g)
    assert e.value.code == 5
    ctx.sync()
