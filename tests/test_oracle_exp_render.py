"""Pins of the oracle's path tracer in the exponential transport model (App. D,
Sec. 4 eq. exp_ff; the comparison variant of the paper's linear-vs-exponential
study): collisions and light samples by analog decomposition tracking,
environment samples by exp(-sum I_k), no primitive skipped after a scatter.
Checked against the exponential model's first-collision law by independent
quadrature, the white furnace and the agreement of the light-sampling,
phase-sampling and MIS estimators."""
import math

import numpy as np
import pytest
from scipy import integrate

import indep
from paper_2406_09733_amd import scenes

EXP = {"transport": 1}


def _furnace_scene():
    sc = scenes.tiny_random(seed=21, n_emit=0)
    sc["albedo"][:] = 1.0
    sc["material"][:] = 0
    return sc


def _prims(mu, s, q, d, emission):
    n = len(d)
    return {"mean": np.array(mu, np.float32).reshape(-1, 3), "scale": np.array(s, np.float32).reshape(-1, 3),
            "rotation": np.array(q, np.float32).reshape(-1, 4), "density": np.array(d, np.float32),
            "albedo": np.full((n, 3), 0.5, np.float32), "roughness": np.full(n, 0.5, np.float32),
            "emission": np.array(emission, np.float32).reshape(-1, 3), "material": np.zeros(n, np.int32)}


# a near-pinpoint camera looking along +z: every sample takes the same ray
_PIN = {"origin": (0.5, 0.52, -1.0), "target": (0.5, 0.52, 0.5), "up": (0, 1, 0), "vfov_deg": 1e-6,
        "width": 1, "height": 1}


def _mean_radiance(S, params, n):
    Ls = np.array([S.path_radiance(_PIN, params, 0, i) for i in range(n)])
    return Ls.mean(0), Ls.std(0) / np.sqrt(n)


def test_exp_white_furnace_phase_sampling_is_exact(orc):
    # albedo 1, a Lambert phase function, unit environment, no emitters: every
    # path escapes carrying exactly 1, whatever the free flights were
    S = orc.Scene(_furnace_scene())
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    s, _, _ = S.render(cam, dict(EXP, spp=8, max_depth=1000, seed=3, env_radiance=(1, 1, 1), mis_mode=1))
    assert np.allclose(s / 8, 1.0, rtol=0, atol=1e-12)


def test_exp_white_furnace_with_mis(orc):
    S = orc.Scene(_furnace_scene())
    cam = dict(scenes.camera("tiny_random"), width=16, height=16)
    spp = 16
    s, s2, _ = S.render(cam, dict(EXP, spp=spp, max_depth=1000, seed=4, env_radiance=(1, 1, 1)))
    mean = s.sum(0) / (s.shape[0] * spp)
    var = s2.sum(0) / (s.shape[0] * spp) - mean ** 2
    err = np.sqrt(var / (s.shape[0] * spp))
    assert np.all(np.abs(mean - 1.0) <= 3 * err + 1e-12), (mean, err)


def test_exp_direct_view_expected_value(orc):
    # max_depth 0: a camera path only picks up the emission of the Gaussian
    # it collides in; in an exponential medium the ray collides with
    # probability 1 - exp(-I) (the linear model's is I/2)
    sc = _prims([[0.5, 0.5, 0.5]], [[0.1, 0.2, 0.15]], [[0.9, 0.2, 0.1, 0.3]], [3.0], [[2.0, 3.0, 4.0]])
    S = orc.Scene(sc)
    m, se = _mean_radiance(S, dict(EXP, spp=1, max_depth=0, seed=5), 4000)
    o = np.float32([0.5, 0.52, -1.0]).astype(np.float64)
    I = indep.integral(sc, 0, o, np.array([0.0, 0.0, 1.0]), 0.0, np.inf)
    ref = (1.0 - math.exp(-I)) * np.array([2.0, 3.0, 4.0])
    assert 0.2 < 1.0 - math.exp(-I) < 0.95
    assert np.all(np.abs(m - ref) <= 3.5 * se + 1e-4), (m, ref, se)


def test_exp_first_collision_law_with_overlap(orc):
    # an absorber overlapping an emitter along the ray: the emitter is hit
    # first with probability int T(t) G_e(t) dt, T(t) = exp(-int_0^t (G_1 + G_e))
    # (the exponential free-flight law of the summed extinction), by nested
    # quadrature of the kernels
    sc = _prims([[0.5, 0.52, 0.45], [0.5, 0.52, 0.55]], [[0.2, 0.2, 0.12], [0.15, 0.15, 0.1]],
                [[1, 0, 0, 0], [0.95, 0.1, 0.2, 0.2]], [4.0, 5.0], [[0, 0, 0], [1.0, 2.0, 3.0]])
    sc["albedo"][0] = 0.0
    S = orc.Scene(sc)
    o = np.float32([0.5, 0.52, -1.0]).astype(np.float64)
    w = np.array([0.0, 0.0, 1.0])
    c0, c1 = indep.chord(sc, 0, o, w), indep.chord(sc, 1, o, w)
    assert c0[0] < c1[0] < c0[1]  # the chords overlap
    lo, hi = min(c0[0], c1[0]), max(c0[1], c1[1])

    def tau(t):
        return indep.integral(sc, 0, o, w, 0.0, t) + indep.integral(sc, 1, o, w, 0.0, t)

    def g1(t):
        return indep.kernel(sc, 1, o + t * w)

    P, _ = integrate.quad(lambda t: math.exp(-tau(t)) * g1(t), lo, hi, epsabs=1e-10, limit=200)
    m, se = _mean_radiance(S, dict(EXP, spp=1, max_depth=0, seed=6), 6000)
    ref = P * np.array([1.0, 2.0, 3.0])
    assert 0.1 < P < 0.9
    assert np.all(np.abs(m - ref) <= 3.5 * se + 1e-4), (m, ref, se)


@pytest.mark.slow
def test_exp_mis_estimators_agree(orc):
    # light sampling only, phase sampling only and the balance heuristic
    # estimate the same image in the exponential model too
    sc = scenes.tiny_random(seed=0, n_emit=200)
    sc["material"][::2] = 1
    sc["roughness"][:] = np.linspace(0.1, 1.0, sc["roughness"].size, dtype=np.float32)
    S = orc.Scene(sc)
    cam = dict(scenes.camera("tiny_random"), width=32, height=32)
    spp = 512
    res = {}
    for mode in (0, 1, 2):
        s, s2, _ = S.render(cam, dict(EXP, spp=spp, max_depth=3, seed=7 + mode, mis_mode=mode))
        npx = s.shape[0]
        mean = s.sum() / (npx * spp * 3)
        per = s.sum(1) / 3 / spp
        var = (s2.sum(1) / 3 / spp - per ** 2).mean()
        res[mode] = (mean, math.sqrt(max(var, 0) / (npx * spp)))
    for a in (1, 2):
        d = abs(res[a][0] - res[0][0])
        assert d <= 3 * math.hypot(res[a][1], res[0][1]), res


def test_exp_and_linear_models_differ(orc):
    # the same scene under the two models: the linear model's direct-view
    # pick-up I/2 against the exponential 1 - exp(-I) (a switch that did
    # nothing would pass the tests above only by accident of the scene)
    sc = _prims([[0.5, 0.5, 0.5]], [[0.1, 0.2, 0.15]], [[0.9, 0.2, 0.1, 0.3]], [3.0], [[2.0, 3.0, 4.0]])
    S = orc.Scene(sc)
    me, se_e = _mean_radiance(S, dict(EXP, spp=1, max_depth=0, seed=5), 3000)
    ml, se_l = _mean_radiance(S, dict(spp=1, max_depth=0, seed=5), 3000)
    assert np.all(np.abs(me - ml) > 5 * np.hypot(se_e, se_l))


def test_exp_scatter_keeps_the_gaussian(orc):
    # one dense Gaussian of albedo 1 in a unit environment, one scattering
    # event, phase sampling only: the linear model skips the primitive after
    # its scatter, so every path escapes carrying exactly 1; the exponential
    # variant scatters inside the Gaussian, whose rest still attenuates the
    # second flight, so some paths end there and the mean falls below 1
    sc = _prims([[0.5, 0.52, 0.5]], [[0.2, 0.2, 0.2]], [[1, 0, 0, 0]], [6.0], [[0, 0, 0]])
    sc["albedo"][:] = 1.0
    S = orc.Scene(sc)
    p = {"spp": 1, "max_depth": 1, "seed": 8, "env_radiance": (1, 1, 1), "mis_mode": 1}
    lin = np.array([S.path_radiance(_PIN, p, 0, i) for i in range(400)])
    assert np.allclose(lin, 1.0, rtol=0, atol=1e-12)
    m, se = _mean_radiance(S, dict(EXP, **p), 3000)
    assert np.all(m < 1.0 - 10 * se), (m, se)
