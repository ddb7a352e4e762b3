"""Pins of the oracle's primitive geometry and ray integral (Sec. 3.1, Sec. 4.1,
App. A, App. C) against quadrature, closed forms and identities."""
import math

import numpy as np
import pytest
from scipy.special import erf

import indep

R = indep.R_CUT


def _ray(o, w, t0=0.0, t1=np.inf):
    return np.array([*o, *w, t0, t1], dtype=np.float64)


def _scene_one(mu, s, q, d):
    return {"mean": np.array([mu], np.float32), "scale": np.array([s], np.float32),
            "rotation": np.array([q], np.float32), "density": np.array([d], np.float32),
            "albedo": np.full((1, 3), 0.5, np.float32), "roughness": np.full(1, 0.5, np.float32),
            "emission": np.zeros((1, 3), np.float32), "material": np.zeros(1, np.int32)}


def test_cutoff_radius(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    # eq. cutoff_threshold: G/G(mu) = eps on |x'| = r  =>  exp(-r^2/2) = eps
    assert math.isclose(math.exp(-0.5 * S.cutoff_radius ** 2), 0.01, rel_tol=1e-14)


def test_frame_against_scipy(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    for k in range(0, 1000, 97):
        M, nrm, lo, hi = S.prim_frame(k)
        mu, s, Rm, Sigma, d = indep.prim(tiny_scene, k)
        # M^T M = Sigma^-1 (eq. covariance_decomposition)
        assert np.allclose(M.T @ M, np.linalg.inv(Sigma), rtol=1e-10, atol=0)
        # facet normal is the eigenvector of the smallest scale
        evals, evecs = np.linalg.eigh(Sigma)
        assert abs(abs(evecs[:, 0] @ nrm) - 1) < 1e-9
        # the box contains the ellipsoid's extreme points along each axis
        ext = R * np.sqrt(np.diag(Sigma))
        assert np.allclose(hi - mu, ext, rtol=1e-9) and np.allclose(mu - lo, ext, rtol=1e-9)


def test_ray_integral_matches_quadrature(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    rng = np.random.default_rng(5)
    checked = 0
    for k in rng.choice(1000, 60, replace=False):
        mu = tiny_scene["mean"][k].astype(np.float64)
        s = tiny_scene["scale"][k].astype(np.float64)
        o = mu + rng.normal(size=3) * 0.3
        tgt = mu + rng.normal(size=3) * s.max()
        w = (tgt - o) / np.linalg.norm(tgt - o)
        ch = indep.chord(tiny_scene, k, o, w)
        if ch is None:
            continue
        for (x, y) in [(-np.inf, np.inf), (ch[0] + 0.3 * (ch[1] - ch[0]), np.inf),
                       (ch[0] + 0.2 * (ch[1] - ch[0]), ch[0] + 0.7 * (ch[1] - ch[0]))]:
            got = S.ray_integral(k, _ray(o, w), x, y)
            ref = indep.integral(tiny_scene, k, o, w, x, y)
            assert got == pytest.approx(ref, rel=1e-11, abs=1e-300)
            checked += 1
    assert checked > 60


def test_axis_aligned_closed_form(orc):
    # a ray along local axis i through the mean: rho = 0, A = 1/s_i^2, so the
    # truncated integral is d sqrt(2 pi) s_i erf(r / sqrt 2)
    sc = _scene_one([0.1, -0.2, 0.3], [0.02, 0.05, 0.3], [1, 0, 0, 0], 3.0)
    S = orc.Scene(sc, bvh=False)
    assert math.isclose(erf(R / math.sqrt(2)), 0.9975934800, rel_tol=1e-9)
    for i, si in enumerate(np.float32([0.02, 0.05, 0.3]).astype(np.float64)):
        w = np.zeros(3); w[i] = 1.0
        o = np.float32([0.1, -0.2, 0.3]).astype(np.float64) - 5.0 * w
        got = S.ray_integral(0, _ray(o, w), -np.inf, np.inf)
        ref = 3.0 * math.sqrt(2 * math.pi) * si * erf(R / math.sqrt(2))
        assert got == pytest.approx(ref, rel=1e-13)


def test_projected_2d_gaussian_identity(orc, tiny_scene):
    # App. C: the integral of the normalised 3D Gaussian along an infinite ray
    # equals the normalised 2D Gaussian of the projection (mu_hat, Sigma_hat);
    # truncation at r multiplies the integral by erf(sqrt((r^2 - rho^2)/2)),
    # with rho^2 = mu_hat^T Sigma_hat^-1 mu_hat.
    S = orc.Scene(tiny_scene)
    rng = np.random.default_rng(9)
    n_ok = 0
    for k in rng.choice(1000, 40, replace=False):
        mu, s, Rm, Sigma, d = indep.prim(tiny_scene, k)
        w = rng.normal(size=3); w /= np.linalg.norm(w)
        u = np.cross(w, [0.3, 0.5, 0.8]); u /= np.linalg.norm(u)
        v = np.cross(w, u)
        B = np.stack([u, v, w], axis=1)
        o = mu + (rng.normal(size=2) * s.min()) @ np.stack([u, v])
        mu_hat = (B.T @ (mu - o))[:2]
        Sig_hat = (B.T @ Sigma @ B)[:2, :2]
        rho2 = mu_hat @ np.linalg.solve(Sig_hat, mu_hat)
        if rho2 >= R * R:
            continue
        c = d * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(Sigma))
        pdf2 = math.exp(-0.5 * rho2) / (2 * math.pi * math.sqrt(np.linalg.det(Sig_hat)))
        ref = c * pdf2 * erf(math.sqrt((R * R - rho2) / 2))
        got = S.ray_integral(k, _ray(o, w, -np.inf, np.inf), -np.inf, np.inf)
        assert got == pytest.approx(ref, rel=1e-10)
        n_ok += 1
    assert n_ok > 20


def test_additivity_and_reversal(orc, tiny_scene):
    S = orc.Scene(tiny_scene)
    rng = np.random.default_rng(2)
    for k in rng.choice(1000, 30, replace=False):
        mu = tiny_scene["mean"][k].astype(np.float64)
        o = mu - np.array([0.4, 0.1, 0.2]); w = (mu - o) / np.linalg.norm(mu - o)
        ch = indep.chord(tiny_scene, k, o, w)
        a, b = ch
        m = a + 0.37 * (b - a)
        r = _ray(o, w)
        I_ab = S.ray_integral(k, r, -np.inf, np.inf)
        assert I_ab == pytest.approx(S.ray_integral(k, r, -np.inf, m) + S.ray_integral(k, r, m, np.inf),
                                     rel=1e-13)
        # reversed ray from beyond the chord covers the same segment
        o2 = o + (b + 0.5) * w
        r2 = _ray(o2, -w)
        assert S.ray_integral(k, r2, -np.inf, np.inf) == pytest.approx(I_ab, rel=1e-12)
        assert S.ray_integral(k, r2, (b + 0.5) - m, np.inf) == pytest.approx(
            S.ray_integral(k, r, -np.inf, m), rel=1e-11)
