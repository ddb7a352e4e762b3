"""GPU parity of the exponential variant (App. D; eq. exp_ff) with the oracle:
transmittance exp(-sum I_k), and analog decomposition tracking with the same
counter-based uniforms on both sides.

Tolerances:
  T     |gpu - oracle| <= 1e-5 max(T, 1e-3)  (float sum of the ray integrals)
  prim  identical wherever the oracle's margin (collide-or-not decision and
        the gap between the two nearest collisions, relative) exceeds 1e-4
  t     |gpu - oracle| <= 1e-4 |t| + 1e-6 there (FP64 inverse of float chord data)
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
