"""Pins of the oracle's light sampling (reading C12): an emissive primitive is
picked uniformly, a point y of its untruncated Gaussian N(mu, Sigma) is drawn
and the light ray aims at it.  The solid-angle pdf of the direction is the
density of y integrated along the ray, int_0^inf N(x + t w) t^2 dt; the
oracle evaluates it in closed form.

* the closed form against adaptive quadrature of that integral, with Sigma
  from scipy's rotation of the quaternion (near and far outside the cut-off
  ellipsoid; toward, across and away from the centre), and 0 from inside it
  (no light sample is taken toward an emitter from within its support);
* the pdf integrates to 1 over the sphere of directions;
* the sampled directions follow the pdf (chi-square over solid-angle bins),
  and the points behind them are Gaussian (the directions toward the mean of
  an isotropic emitter seen from afar spread as the 2-D normal of its
  projected width).
The renderer's use of both (MIS weights at emission pick-ups, the light
estimate) is pinned by the agreement of the light-only, phase-only and MIS
images (test_oracle_render.py)."""
import numpy as np
import pytest
from scipy import integrate, stats

import indep


def _emitters(n=6, seed=3):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    # flat, elongated and round emitters (aspect up to 100, as the room's panels)
    scale = np.array([[0.2, 0.2, 0.002], [0.3, 0.05, 0.05], [0.1, 0.1, 0.1],
                      [0.25, 0.12, 0.03], [0.04, 0.3, 0.006], [0.15, 0.08, 0.2]])[:n]
    sc = {"mean": rng.uniform(-0.5, 0.5, (n, 3)).astype(np.float32), "scale": scale.astype(np.float32),
          "rotation": q.astype(np.float32), "density": np.full(n, 2.0, np.float32),
          "albedo": np.full((n, 3), 0.5, np.float32), "roughness": np.full(n, 0.5, np.float32),
          "emission": np.ones((n, 3), np.float32), "material": np.zeros(n, np.int32)}
    return sc


def _pdf_quad(sc, k, x, w):
    """int_0^inf N(x + t w; mu, Sigma) t^2 dt by adaptive quadrature; along
    the line the density is a 1-D Gaussian in t (centre t_m, width sd), so
    the interval is split there."""
    mu, s, R, Sigma, _ = indep.prim(sc, k)
    N = stats.multivariate_normal(mean=mu, cov=Sigma)
    f = lambda t: N.pdf(x + t * w) * t * t
    Si = np.linalg.inv(Sigma)
    a2 = float(w @ Si @ w)
    t_m, sd = float((mu - x) @ Si @ w) / a2, 1.0 / np.sqrt(a2)
    lo, hi = max(0.0, t_m - 14 * sd), max(0.0, t_m + 14 * sd)
    total = 0.0
    if lo > 0:
        total += integrate.quad(f, 0.0, lo, limit=200)[0]
    if hi > lo:
        pts = [t for t in t_m + sd * np.arange(-13, 14) if lo < t < hi]
        total += integrate.quad(f, lo, hi, points=pts, limit=800, epsabs=0, epsrel=1e-12)[0]
    total += integrate.quad(f, hi, np.inf, limit=200)[0]
    return total


def test_light_pdf_matches_its_integral_definition(orc):
    sc = _emitters()
    S = orc.Scene(sc)
    n_emit = sc["mean"].shape[0]
    rng = np.random.default_rng(7)
    worst = 0.0
    checked = inside = 0
    for k in range(n_emit):
        mu, s, R, Sigma, _ = indep.prim(sc, k)
        for dist in (0.05, 0.5, 2.0, 8.0):  # in units of the largest scale: inside .. far
            for _ in range(4):
                x = mu + dist * float(np.max(s)) * rng.normal(size=3) / np.sqrt(3.0)
                c = (mu - x) / np.linalg.norm(mu - x)
                # toward the centre, across the emitter, at random
                for w in (c, c + 0.5 * float(np.max(s)) / max(np.linalg.norm(mu - x), 1e-3) * rng.normal(size=3),
                          rng.normal(size=3)):
                    w = w / np.linalg.norm(w)
                    got = S.light_pdf(k, x, w) * n_emit
                    if indep.mahal2(sc, k, x) <= indep.R_CUT ** 2:
                        # no light sample from inside the cut-off ellipsoid
                        assert got == 0.0
                        inside += 1
                        continue
                    ref = _pdf_quad(sc, k, x, w)
                    # relative agreement wherever the density is not
                    # vanishingly small (far behind the emitter both forms
                    # lose relative precision in the exp(-s^2/2) tail)
                    if ref > 1e-30:
                        worst = max(worst, abs(got - ref) / ref)
                        checked += 1
                    else:
                        assert got <= 1e-25
    assert checked > 120 and inside > 30
    assert worst < 1e-7, worst


@pytest.mark.parametrize("dist", [0.7, 3.0])
def test_light_pdf_integrates_to_one(orc, dist):
    # Gauss-Legendre in cos(theta) about the direction to the mean (split
    # where the emitter's cone ends), trapezoid in phi (periodic)
    sc = _emitters()
    S = orc.Scene(sc)
    n_emit = sc["mean"].shape[0]
    for k in (0, 1, 4):
        mu, s, R, Sigma, _ = indep.prim(sc, k)
        x = mu + dist * np.array([0.3, 0.8, -0.52]) / np.linalg.norm([0.3, 0.8, -0.52])
        assert indep.mahal2(sc, k, x) > indep.R_CUT ** 2
        c = (mu - x) / np.linalg.norm(mu - x)
        b1 = np.cross(c, [1.0, 0.0, 0.0] if abs(c[0]) < 0.9 else [0.0, 1.0, 0.0])
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(c, b1)
        reach = min(1.0, 7.0 * float(np.max(s)) / dist)
        cut = np.cos(np.arcsin(reach)) if reach < 1.0 else -1.0
        total = 0.0
        for lo, hi, m in ((cut, 1.0, 400), (-1.0, cut, 60)):
            if hi <= lo:
                continue
            xs, ws = np.polynomial.legendre.leggauss(m)
            ct = 0.5 * (hi - lo) * xs + 0.5 * (hi + lo)
            wt = 0.5 * (hi - lo) * ws
            nphi = 256
            for cti, wti in zip(ct, wt):
                st = np.sqrt(max(0.0, 1.0 - cti * cti))
                acc = 0.0
                for ph in np.arange(nphi) * (2 * np.pi / nphi):
                    w = cti * c + st * (np.cos(ph) * b1 + np.sin(ph) * b2)
                    acc += S.light_pdf(k, x, w)
                total += wti * acc * (2 * np.pi / nphi)
        assert abs(total * n_emit - 1.0) < 2e-3, (k, dist, total * n_emit)


def test_light_directions_follow_the_pdf(orc):
    # a flat emitter seen obliquely from 1.5 of its scale: bins in
    # (cos theta, phi) about the direction to the mean; expected counts by
    # quadrature of the pdf over each bin
    sc = _emitters()
    S = orc.Scene(sc)
    n_emit = sc["mean"].shape[0]
    k = 0
    mu, s, R, Sigma, _ = indep.prim(sc, k)
    x = mu + 0.3 * np.array([0.6, 0.0, 0.8])
    assert indep.mahal2(sc, k, x) > indep.R_CUT ** 2
    c = (mu - x) / np.linalg.norm(mu - x)
    b1 = np.cross(c, [0.0, 1.0, 0.0])
    b1 /= np.linalg.norm(b1)
    b2 = np.cross(c, b1)
    rng = np.random.default_rng(11)
    n = 60000
    U = rng.uniform(size=(n, 4))
    W = np.array([S.light_dir(k, x, u) for u in U])
    ct = W @ c
    ph = np.mod(np.arctan2(W @ b2, W @ b1), 2 * np.pi)
    ce = np.array([-1.0, 0.0, 0.5, 0.75, 0.87, 0.93, 0.965, 0.985, 1.0])
    pe = np.linspace(0, 2 * np.pi, 9)
    obs, _, _ = np.histogram2d(ct, ph, bins=[ce, pe])
    exp = np.zeros_like(obs)
    xs, ws = np.polynomial.legendre.leggauss(24)
    for i in range(len(ce) - 1):
        for j in range(len(pe) - 1):
            a0, a1, p0, p1 = ce[i], ce[i + 1], pe[j], pe[j + 1]
            tot = 0.0
            for xi, wi in zip(xs, ws):
                cti = 0.5 * (a1 - a0) * xi + 0.5 * (a1 + a0)
                st = np.sqrt(max(0.0, 1 - cti * cti))
                for xj, wj in zip(xs, ws):
                    phj = 0.5 * (p1 - p0) * xj + 0.5 * (p1 + p0)
                    w = cti * c + st * (np.cos(phj) * b1 + np.sin(phj) * b2)
                    tot += wi * wj * S.light_pdf(k, x, w)
            exp[i, j] = tot * 0.25 * (a1 - a0) * (p1 - p0) * n_emit * n
    keep = exp > 20
    assert keep.sum() >= 30
    chi2 = float((((obs - exp) ** 2) / exp)[keep].sum())
    dof = int(keep.sum()) - 1
    assert stats.chi2.sf(chi2, dof) > 1e-3, (chi2, dof)
    assert abs(obs.sum() - exp.sum()) < 4 * np.sqrt(n) + 1e-3 * n


def test_light_points_are_gaussian(orc):
    # round emitter far away: the directions' offsets from the centre
    # direction, scaled by the distance, are its N(0, sigma^2 I) projection
    sc = _emitters()
    S = orc.Scene(sc)
    k = 2
    mu, s, R, Sigma, _ = indep.prim(sc, k)
    D = 500.0
    x = mu - D * np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(12)
    W = np.array([S.light_dir(k, x, u) for u in rng.uniform(size=(20000, 4))])
    off = W[:, :2] / W[:, 2:3] * D / float(s[0])
    for col in off.T:
        assert stats.kstest(col, "norm").pvalue > 1e-3


def _panel_and_floor():
    # a panel of overlapping flat emitters (thin axis 1/100) 1 above a floor
    # of flat diffuse primitives, both facing each other
    g = np.arange(12) * 0.05 - 0.275
    px, pz = np.meshgrid(g, g)
    fg = np.arange(16) * 0.12 - 0.9
    fx, fz = np.meshgrid(fg, fg)
    n_p, n_f = px.size, fx.size
    mean = np.concatenate([np.stack([px.ravel(), np.full(n_p, 1.0), pz.ravel()], 1),
                           np.stack([fx.ravel(), np.zeros(n_f), fz.ravel()], 1)])
    s_p, s_f = 0.04, 0.1
    scale = np.concatenate([np.tile([s_p, s_p, s_p / 100], (n_p, 1)), np.tile([s_f, s_f, s_f / 100], (n_f, 1))])
    q = np.tile([np.cos(np.pi / 4), np.sin(np.pi / 4), 0.0, 0.0], (n_p + n_f, 1))  # thin axis -> y
    alpha = 0.8
    dens = 2 * alpha / (np.sqrt(2 * np.pi) * scale[:, 2])
    emis = np.zeros((n_p + n_f, 3))
    emis[:n_p] = 4.0
    return {"mean": mean.astype(np.float32), "scale": scale.astype(np.float32), "rotation": q.astype(np.float32),
            "density": dens.astype(np.float32), "albedo": np.full((n_p + n_f, 3), 0.7, np.float32),
            "roughness": np.full(n_p + n_f, 0.5, np.float32), "emission": emis.astype(np.float32),
            "material": np.zeros(n_p + n_f, np.int32)}


@pytest.mark.slow
def test_mis_estimators_agree_with_overlapping_flat_emitters(orc):
    # paths scatter inside the panel's overlapping emitters and on the floor:
    # light-only, phase-only and MIS estimates of the image agree
    sc = _panel_and_floor()
    S = orc.Scene(sc)
    cam = {"origin": (0.0, 0.5, -2.0), "target": (0.0, 0.55, 0.0), "up": (0, 1, 0), "vfov_deg": 50.0,
           "width": 24, "height": 24}
    spp = 192
    res = {}
    for mode in (0, 1, 2):
        s, s2, _ = S.render(cam, {"spp": spp, "max_depth": 2, "seed": 70 + mode, "mis_mode": mode})
        per = s / spp
        var = np.maximum(s2 / spp - per ** 2, 0.0)
        res[mode] = (float(per.mean()), float(np.sqrt(var.mean() / (spp * s.shape[0]))))
    for a in (1, 2):
        assert abs(res[a][0] - res[0][0]) <= 4 * np.hypot(res[a][1], res[0][1]), res
    assert all(v[1] < 0.03 * v[0] for v in res.values()), res
