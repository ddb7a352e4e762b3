"""The scene generators build what their recipes state: surface primitives
100x thinner than wide with a normal-incidence opacity alpha ~ U[0.6, 1], the
room's primitive, emitter and cluster counts, and (through the oracle) the
mean free-flight CDF of a tiled surface at normal incidence: the cover of the
tiling (k eps times the truncated kernel's footprint) times E[alpha]."""
import math

import numpy as np
import pytest

from paper_2406_09733_amd import scenes

R_CUT = math.sqrt(-2.0 * math.log(0.01))
CENTRE = math.sqrt(2.0 * math.pi) * math.erf(R_CUT / math.sqrt(2.0))


def _flat_part(sc):
    s = np.sort(sc["scale"].astype(np.float64), axis=1)
    flat = s[:, 0] < 0.05 * s[:, 1]
    return flat, s


def _alpha(sc, flat, s):
    # half the ray integral through the centre at normal incidence
    return 0.5 * sc["density"][flat].astype(np.float64) * CENTRE * s[flat, 0]


def test_mixed_recipe():
    sc = scenes.mixed_100k()
    flat, s = _flat_part(sc)
    assert flat.sum() == pytest.approx(70_000, rel=0.02)
    assert np.allclose(s[flat, 0] / s[flat, 1], 0.01, rtol=1e-5)
    assert np.allclose(s[flat, 1], s[flat, 2], rtol=1e-6)
    a = _alpha(sc, flat, s)
    assert a.min() >= 0.6 - 1e-5 and a.max() <= 1.0 + 1e-5
    assert abs(a.mean() - 0.8) < 0.005
    assert (sc["emission"].max(1) > 0).sum() == 1000


@pytest.mark.slow
def test_room_recipe():
    sc = scenes.room_5p5m()
    n = sc["mean"].shape[0]
    assert 5_400_000 <= n <= 5_600_000
    flat, s = _flat_part(sc)
    assert flat.sum() == n - 40 * 30_000
    assert np.allclose(s[flat, 0] / s[flat, 1], 0.01, rtol=1e-5)
    a = _alpha(sc, flat, s)
    assert a.min() >= 0.6 - 1e-5 and a.max() <= 1.0 + 1e-5
    # tangent scale sqrt(0.16 A / N), about 4 mm
    assert 0.003 < float(np.median(s[flat, 1])) < 0.006
    # clusters: 20:1:1, short scale in [0.5, 2] mm
    c = ~flat
    assert np.allclose(s[c, 2] / s[c, 1], 20.0, rtol=1e-5)
    assert s[c, 0].min() >= 0.0005 * (1 - 1e-6) and s[c, 0].max() <= 0.002 * (1 + 1e-6)
    em = sc["emission"].max(1) > 0
    assert 15_000 < em.sum() < 25_000 and np.all(flat[em])
    # emitters lie in the two 1 x 1 m panels 1 cm under the ceiling
    assert np.allclose(sc["mean"][em, 1], 2.99, atol=1e-5)


def _cover():
    # k eps / s_t^2 times the area integral of half the normal-incidence ray
    # integral of a flat primitive of centre opacity 1: in units of s_t,
    # 2 pi int_0^r rho e^(-rho^2/2) erf(sqrt((r^2 - rho^2)/2)) drho / erf(r/sqrt 2)
    from scipy import integrate
    f = lambda p: p * math.exp(-p * p / 2) * math.erf(math.sqrt((R_CUT ** 2 - p * p) / 2))
    v, _ = integrate.quad(f, 0, R_CUT, epsabs=0, epsrel=1e-12)
    return 0.16 * 2 * math.pi * v / math.erf(R_CUT / math.sqrt(2))


def test_tiled_plane_is_semi_transparent_at_normal_incidence(orc):
    # a square of flat primitives from the generators' tiling recipe: the mean
    # of F over uniform ray positions is the tiling's cover (0.981) times the
    # primitives' mean opacity, so most normal-incidence rays pass partially
    rng = np.random.Generator(np.random.PCG64(3))
    side, n = 0.5, 40_000
    cell = side / math.sqrt(n)
    s_t = math.sqrt(0.16) * cell
    pts = scenes._grid_on_rect(rng, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), side, side, cell)
    nrm = np.tile([0.0, 0.0, 1.0], (pts.shape[0], 1))
    m, scale, q, d = scenes._flat(rng, pts, nrm, s_t, 0.01)
    k = m.shape[0]
    sc = {"mean": m.astype(np.float32), "scale": scale.astype(np.float32), "rotation": q.astype(np.float32),
          "density": d.astype(np.float32), "albedo": np.full((k, 3), 0.5, np.float32),
          "roughness": np.full(k, 0.5, np.float32), "emission": np.zeros((k, 3), np.float32),
          "material": np.zeros(k, np.int32)}
    S = orc.Scene(sc)
    nr = 20000
    o = np.concatenate([rng.uniform(0.1, 0.4, (nr, 2)), np.full((nr, 1), -1.0)], 1)
    rays = np.concatenate([o, np.tile([0.0, 0.0, 1.0], (nr, 1)), np.zeros((nr, 1)), np.full((nr, 1), np.inf)],
                          1).astype(np.float32)
    F, T = S.transmittance(rays)
    alpha = 0.5 * sc["density"].astype(np.float64) * CENTRE * sc["scale"][:, 2]
    want = _cover() * alpha.mean()
    assert abs(F.mean() - want) < 3.5 * F.std() / math.sqrt(nr), (F.mean(), want)
    assert 0.5 < (T > 0).mean() < 0.95  # most rays pass partially, some saturate
