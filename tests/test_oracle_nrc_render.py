"""Pins of the oracle's path tracer with the neural radiance cache: paths
that end in the cache after a fixed number of scattering events, and the
training records of full-length paths.

  * ending paths with nothing added equals the plain tracer with that depth,
    path by path (the cache only replaces the continuation);
  * in a white furnace (albedo 1, unit environment, no emitters) the radiance
    scattered from any vertex is exactly 1, so a cache that predicts 1 gives
    exactly 1 per path under phase sampling, 1 in expectation under MIS, and
    the training targets average 1 (a dropped throughput, or the vertex's own
    light samples counted as 'radiance so far', breaks this);
  * a network built to output a constant c returns c (checked on the oracle's
    own forward pass, then used as that cache)."""
import numpy as np
import pytest

from paper_2406_09733_amd import scenes

Y00 = 0.28209479177387814  # band-0 real spherical harmonic


def const_cache(c):
    """Weights of a network whose output is the constant c: the band-0
    harmonic feature (index 72) drives hidden unit 0 of each layer to 1."""
    from oracle import NRC_LAYERS
    ws = []
    for li, (o, i) in enumerate(NRC_LAYERS):
        w = np.zeros((o, i))
        if li == 0:
            w[0, 72] = 1.0 / Y00
        elif li < 4:
            w[0, 0] = 1.0
        else:
            w[:, 0] = c
        ws.append(w.ravel())
    return np.concatenate(ws)


BOX = (-0.5, -0.5, -0.5, 1.5, 1.5, 1.5)


def _furnace():
    sc = scenes.tiny_random(seed=21, n_emit=0)
    sc["albedo"][:] = 1.0
    sc["material"][:] = 0
    return sc


def test_constant_network(orc):
    W = const_cache([0.3, 0.7, 1.1])
    rng = np.random.default_rng(0)
    x = np.zeros((20, 16), np.float32)
    x[:, :3] = rng.uniform(-0.5, 1.5, (20, 3))
    d = rng.normal(size=(20, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    x[:, 3:6] = d
    x[:, 6:13] = rng.uniform(0, 1, (20, 7))
    y = orc.nrc_forward(W, orc.nrc_encode(x, BOX[:3], BOX[3:]))
    assert np.allclose(y, [0.3, 0.7, 1.1], atol=1e-12)


def test_termination_without_cache_equals_shorter_paths(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    cam = dict(scenes.camera("tiny_random"), width=24, height=24)
    for k in (1, 2, 3):
        plain = {"spp": 1, "max_depth": k, "seed": 11}
        cut = {"spp": 1, "max_depth": 6, "seed": 11, "nrc_mode": 3, "nrc_terminate_after": k, "nrc_box": BOX}
        zero = dict(cut, nrc_mode=2, nrc_weights=const_cache([0, 0, 0]))
        for pix in range(0, 24 * 24, 7):
            a = S.path_radiance(cam, plain, pix, 0)
            assert np.array_equal(a, S.path_radiance(cam, cut, pix, 0))
            assert np.array_equal(a, S.path_radiance(cam, zero, pix, 0))


def test_exact_cache_in_furnace_phase_sampling(orc):
    S = orc.Scene(_furnace())
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    p = {"spp": 4, "max_depth": 1000, "seed": 3, "env_radiance": (1, 1, 1), "mis_mode": 1,
         "nrc_mode": 2, "nrc_terminate_after": 2, "nrc_box": BOX, "nrc_weights": const_cache([1, 1, 1])}
    for term in (1, 2):
        s, _, _ = S.render(cam, dict(p, nrc_terminate_after=term))
        assert np.allclose(s / 4, 1.0, rtol=0, atol=1e-12)
    # a cache predicting 0.5 lowers exactly the paths that reach it (by 1/2 each)
    s2, _, _ = S.render(cam, dict(p, nrc_terminate_after=1, nrc_weights=const_cache([0.5, 0.5, 0.5])))
    cached = 2 * 4 * (1 - s2 / 4)
    assert np.allclose(cached, np.round(cached), atol=1e-9) and cached.sum() > 10


def test_exact_cache_in_furnace_with_mis(orc):
    S = orc.Scene(_furnace())
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    spp = 16
    p = {"spp": spp, "max_depth": 1000, "seed": 4, "env_radiance": (1, 1, 1), "nrc_mode": 2,
         "nrc_terminate_after": 2, "nrc_box": BOX, "nrc_weights": const_cache([1, 1, 1])}
    s, s2, _ = S.render(cam, p)
    m = s.sum(0) / (s.shape[0] * spp)
    var = s2.sum(0) / (s.shape[0] * spp) - m ** 2
    err = np.sqrt(var / (s.shape[0] * spp))
    assert np.all(np.abs(m - 1.0) <= 3 * err + 1e-12), (m, err)


def test_training_records_in_furnace(orc):
    # a denser furnace (scales x4) so that paths scatter many times; paths
    # end only by escaping, so the radiance scattered from every vertex is 1
    sc = _furnace()
    sc["scale"] *= 4
    S = orc.Scene(sc)
    cam = dict(scenes.camera("tiny_random"), width=32, height=32)
    p = {"spp": 1, "max_depth": 1000, "seed": 8, "env_radiance": (1, 1, 1), "nrc_mode": 1,
         "nrc_terminate_after": 2, "nrc_train_frac": 1.0, "nrc_box": BOX,
         "nrc_weights": const_cache([0.0, 0.0, 0.0])}
    plain = {"spp": 1, "max_depth": 1000, "seed": 8, "env_radiance": (1, 1, 1)}
    targets = []
    for pix in range(32 * 32):
        for smp in range(2):
            L, rec = S.path_records(cam, p, pix, smp, max_rec=4000)
            if pix % 16 == 0:
                # a training path is a full path: same radiance as the plain tracer
                assert np.array_equal(L, S.path_radiance(cam, plain, pix, smp))
            if len(rec) == 0:
                continue
            assert np.array_equal(rec[:, 23], np.arange(1, len(rec) + 1))
            assert np.all(rec[:, 19] == pix)
            wo, nrm = rec[:, 3:6], rec[:, 6:9]
            assert np.allclose(np.linalg.norm(wo, axis=1), 1, atol=1e-6)
            assert np.all(np.sum(wo * nrm, axis=1) >= -1e-6)
            assert np.allclose(rec[0, 16:19], 1.0) and np.allclose(rec[0, 20:23], 0.0)
            targets.append((L[None, :] - rec[:, 20:23]) / rec[:, 16:19])
    t = np.concatenate(targets)
    assert t.shape[0] > 10000
    m, se = t.mean(), t.std() / np.sqrt(t.size)
    assert abs(m - 1.0) < 4 * se, (m, se)


def test_no_training_paths_equals_inference_only(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    W = const_cache([0.2, 0.1, 0.05])
    a = {"spp": 1, "max_depth": 5, "seed": 2, "nrc_mode": 1, "nrc_train_frac": 0.0, "nrc_box": BOX,
         "nrc_weights": W}
    b = dict(a, nrc_mode=2)
    for pix in range(0, 256, 3):
        assert np.array_equal(S.path_radiance(cam, a, pix, 0), S.path_radiance(cam, b, pix, 0))
