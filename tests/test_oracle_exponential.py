"""The oracle's exponential variant (App. D; eq. exp_ff) against what the
exponential model fixes: a ray escapes the decomposition-tracking sampler
with probability exp(-sum_k I_k) = T, and the free-flight distance inside a
single Gaussian has CDF 1 - exp(-I(a, t))."""
import numpy as np

from paper_2406_09733_amd import scenes


def _single(d=3.0):
    # one isotropic Gaussian at the origin
    one = lambda v, w: np.asarray(v, np.float32).reshape(1, w)
    return {"mean": one([0, 0, 0], 3), "scale": one([0.2, 0.2, 0.2], 3), "rotation": one([1, 0, 0, 0], 4),
            "density": one([d], 1).reshape(1), "albedo": one([0.5] * 3, 3), "roughness": one([0.5], 1).reshape(1),
            "emission": one([0, 0, 0], 3), "material": np.zeros(1, np.int32)}


def test_exp_escape_probability_is_the_transmittance(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    rays = scenes.probe_rays(tiny_scene, 40, seed=41, aimed_frac=1.0, finite_frac=0.0)
    T = S.exp_transmittance(rays)
    reps = 3000
    rr = np.repeat(rays, 1, axis=0)
    esc = np.zeros(len(rays))
    for s in range(reps):
        prim, t, _ = S.exp_sample(rr, seed=1000 + s)
        esc += prim < 0
    p = esc / reps
    se = np.sqrt(np.maximum(T * (1 - T), 1e-4) / reps)
    assert np.all(np.abs(p - T) <= 4.5 * se + 1e-3), np.abs(p - T) / se
    assert T.min() < 0.9


def test_exp_free_flight_cdf_inside_one_gaussian(orc):
    sc = _single()
    S = orc.Scene(sc)
    ray = np.array([[-1.0, 0.01, 0.02, 1.0, 0.0, 0.0, 0.0, np.inf]], np.float32)
    n = 4000
    rays = np.repeat(ray, n, axis=0)
    # one seed, many rays: ray index i is in the counter, so every ray draws its own uniform
    prim, t, _ = S.exp_sample(rays, seed=7)
    hit = prim >= 0
    T = S.exp_transmittance(ray)[0]
    assert abs((~hit).mean() - T) <= 4.5 * np.sqrt(T * (1 - T) / n) + 1e-3
    # sampled distances: F(t) = (1 - exp(-I(a, t))) / (1 - T) given a collision
    ts = np.sort(t[hit])
    grid = np.linspace(ts[0], ts[-1], 25)
    rr = np.repeat(ray, len(grid), axis=0).copy()
    rr[:, 7] = grid
    I_t = -np.log(S.exp_transmittance(rr))
    F_model = (1 - np.exp(-I_t)) / (1 - T)
    F_emp = np.searchsorted(ts, grid, side="right") / len(ts)
    assert np.max(np.abs(F_emp - F_model)) <= 1.36 * np.sqrt(2.0 / len(ts)) + 0.01
