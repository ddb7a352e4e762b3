"""The allocation-free collision query (ugp_sample_collision_noalloc) against
ugp_sample_collision, through the C ABI: two calls in a row on the same GPU,
the second with fewer rays, on scenes whose rays overflow the 16-entry buffer
(so the fixed buffer's overflow list and saved states are used and reused).
Bar: the parity bar of the collision query -- the selected primitive equal
wherever the oracle's margin |u - boundary| > 1e-5 (the two entry points run
the same kernels; a ray whose saved state did not fit restarts and may round
t differently), t within 1e-5 relative."""
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


def _np(t):
    return t.detach().cpu().numpy()


def _compare(ctx, S, rays, u, ex):
    prim_a, t_a = ctx.sample_collision(rays, u, ex)
    prim_b, t_b = ctx.sample_collision_noalloc(rays, u, ex)
    ctx.sync()
    pa, pb = _np(prim_a), _np(prim_b)
    ta, tb = _np(t_a).astype(np.float64), _np(t_b).astype(np.float64)
    ref = S.sample_collision(rays, u.astype(np.float64), ex)
    clear = ref["margin"] > 1e-5
    assert np.all((pa == pb) | ~clear), np.where((pa != pb) & clear)[0][:10]
    both = (pa == pb) & (pa >= 0)
    assert np.all(np.abs(ta[both] - tb[both]) <= 1e-5 * np.maximum(np.abs(ta[both]), 1e-3))
    assert np.array_equal(np.isnan(ta), np.isnan(tb))
    # and both match the oracle
    assert np.all((pb == ref["prim"]) | ~clear)
    return float((pa == pb).mean()), float((pb >= 0).mean())


@pytest.mark.parametrize("name", ["overlap_pile", "needles"])
def test_noalloc_matches_the_allocating_query(torch, orc, name):
    import paper_2406_09733_amd as P
    sc = {"overlap_pile": scenes.overlap_pile, "needles": scenes.needles}[name]()
    S = orc.Scene(sc)
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    rng = np.random.default_rng(71)
    for n in (200_000, 3_001):
        _say(f"no-alloc collision query on {name}, {n} rays")
        rays = scenes.probe_rays(sc, n, seed=300 + n, aimed_frac=0.9)
        ex = rng.integers(-1, sc["mean"].shape[0], n).astype(np.int32)
        ex[::2] = -1
        u = rng.uniform(0, 1, n).astype(np.float32)
        same, hit = _compare(ctx, S, rays, u, ex)
        _say(f"  identical picks {same:.5f}, collisions {hit:.3f}")
    ctx.close()


def test_noalloc_rejects_too_many_rays(torch):
    import ctypes as C

    import paper_2406_09733_amd as P
    sc = scenes.tiny_random()
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    n = P.NOALLOC_MAX_RAYS + 1
    # the size check comes before any pointer is read: no buffers are needed
    dummy = torch.zeros(8, device="cuda")
    p = C.c_void_p(dummy.data_ptr())
    assert P.lib().ugp_sample_collision_noalloc(ctx.h, n, p, None, p, p, p) == 1
    ctx.sync()
    ctx.close()
