"""Pins of the oracle's SGGX microflakes with a Disney-style base BSDF
(material 3; Sec. 4.2: the improved stochastic evaluation with internal MIS
for the specular and the diffuse lobe, importance sampling by visible normals
then the base BSDF, App. B: the approximate MIS pdf with a roughened SGGX).

Independent anchors:
  * a flat S with metallic 1 is the delta-NDF GGX material (its own pins in
    test_oracle_phase.py): Sec. 4.2's statement that a delta NDF falls back to
    the surface BSDF times the cosine;
  * normal incidence of the diffuse lobe is base colour / pi exactly (every
    retro-reflection factor is 1), F0 = 0.04 for a dielectric;
  * the base BSDF divided by the incident cosine is symmetric in the two
    directions;
  * the stochastic estimate's mean equals the quadrature of eq. phase_function;
  * importance-sampling weights and 4 pi times the estimate at uniform
    directions estimate the same directional albedo (sampling and evaluation
    agree);
  * the roughened SGGX has the eigenvalues App. B states, checked against
    numpy's symmetric eigen-solver;
  * light sampling, phase sampling and MIS render the same image.
"""
import math

import numpy as np
import pytest

from paper_2406_09733_amd import scenes


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _s6(S):
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


def _rand_spd(rng, lam):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q @ np.diag(lam) @ q.T


def _flat(n, eps=1e-8):
    return _s6(np.outer(n, n) + eps * (np.eye(3) - np.outer(n, n)))


def test_flat_metallic_is_the_delta_ndf_ggx(orc):
    rng = np.random.default_rng(0)
    n = _unit([0.3, -0.4, 0.85])
    c = np.array([0.9, 0.6, 0.3])
    u = rng.uniform(0, 1, (2000, 6))
    for rough in [0.3, 0.6, 1.0]:
        for _ in range(3):
            wo = _unit(rng.normal(size=3)); wi = _unit(rng.normal(size=3))
            if (wo @ n) * (wi @ n) <= 0.05:
                wi = wi - 2 * (wi @ n) * n if (wo @ n) * (wi @ n) < 0 else _unit(wi + n * np.sign(wo @ n))
            ref, _ = orc.phase_eval(1, c, rough, n, wo, wi)
            est = orc.sggx_disney_est(_flat(n), c, rough, 1.0, wo, wi, u).mean(0)
            assert np.allclose(est, ref, rtol=3e-3, atol=1e-6), (rough, est, ref)


def test_base_bsdf_normal_incidence_and_symmetry(orc):
    rng = np.random.default_rng(1)
    n = _unit([0.1, 0.2, 0.97])
    c = np.array([0.2, 0.5, 0.8])
    for rough in [0.1, 0.5, 1.0]:
        fs, fd = orc.disney_base(c, rough, 0.0, n, n, n)
        assert np.allclose(fd, c / math.pi, rtol=1e-12)
        a = max(rough * rough, 1e-4)
        assert np.allclose(fs, 0.04 * (1 / (math.pi * a * a)) / 4, rtol=1e-10)  # F0 D(1) G2(1,1) / 4
        fs, fd = orc.disney_base(c, rough, 0.4, n, n, n)
        assert np.allclose(fd, 0.6 * c / math.pi, rtol=1e-12)
        for _ in range(5):
            wo = _unit(n + 0.8 * rng.normal(size=3)); wi = _unit(n + 0.8 * rng.normal(size=3))
            if wo @ n <= 0 or wi @ n <= 0:
                continue
            f1 = np.add(*orc.disney_base(c, rough, 0.3, n, wo, wi)) / (wi @ n)
            f2 = np.add(*orc.disney_base(c, rough, 0.3, n, wi, wo)) / (wo @ n)
            assert np.allclose(f1, f2, rtol=1e-12)
        fs, fd = orc.disney_base(c, rough, 0.3, n, n, -n)
        assert np.all(fs == 0) and np.all(fd == 0)


def test_estimator_is_unbiased_against_quadrature(orc):
    rng = np.random.default_rng(2)
    c = np.array([0.7, 0.5, 0.3])
    for lam, rough, met in [((1.0, 0.2, 0.2), 0.3, 0.0), ((1.0, 1.0, 0.05), 0.7, 1.0),
                            ((1.0, 0.5, 0.1), 1.0, 0.5), ((1.0, 1.0, 1.0), 0.2, 0.2)]:
        s6 = _s6(_rand_spd(rng, lam))
        for _ in range(2):
            wo = _unit(rng.normal(size=3)); wi = _unit(rng.normal(size=3))
            ref = orc.sggx_disney_quad(s6, c, rough, met, wo, wi, 700, 1400)
            est = orc.sggx_disney_est(s6, c, rough, met, wo, wi, rng.uniform(0, 1, (30000, 6)))
            se = est.std(0) / math.sqrt(est.shape[0])
            assert np.all(np.abs(est.mean(0) - ref) <= 5 * se + 1e-3 * ref + 1e-7), (lam, est.mean(0), ref, se)


def test_sampling_and_evaluation_agree(orc):
    # E[weight] over importance samples = integral of f_p over incident
    # directions = 4 pi E[estimate] over uniform directions
    rng = np.random.default_rng(3)
    c = np.array([0.6, 0.6, 0.6])
    for lam, rough, met in [((1.0, 0.1, 0.1), 0.4, 0.0), ((1.0, 1.0, 0.1), 0.8, 1.0), ((1.0, 0.6, 0.3), 0.5, 0.5)]:
        s6 = _s6(_rand_spd(rng, lam))
        wo = _unit(rng.normal(size=3))
        _, w, ok = orc.sggx_disney_sample(s6, c, rough, met, wo, rng.uniform(0, 1, (40000, 5)))
        ws = w[:, 0]
        m1, s1 = ws.mean(), ws.std() / math.sqrt(ws.size)
        dirs = rng.normal(size=(8000, 3)); dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        e = np.array([orc.sggx_disney_est(s6, c, rough, met, wo, d, rng.uniform(0, 1, (2, 6)))[:, 0].mean()
                      for d in dirs]) * 4 * math.pi
        m2, s2 = e.mean(), e.std() / math.sqrt(e.size)
        assert abs(m1 - m2) <= 4.5 * math.hypot(s1, s2), (lam, rough, met, m1, m2, s1, s2)
        assert ok.mean() > 0.5


def test_roughened_sggx_eigenvalues(orc):
    rng = np.random.default_rng(4)
    for lam in [(0.02, 0.3, 1.0), (0.1, 0.5, 0.9), (0.5, 0.05, 2.0)]:
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        S = Q @ np.diag(lam) @ Q.T
        for rough in [0.1, 0.5, 1.0]:
            a2 = max(rough * rough, 1e-4) ** 2
            r6 = orc.sggx_roughened(_s6(S), rough)
            R = np.array([[r6[0], r6[3], r6[4]], [r6[3], r6[1], r6[5]], [r6[4], r6[5], r6[2]]])
            s = np.sort(lam)
            want = np.sort([s[0] + a2 * s[2], s[1] + a2 * s[2], s[2]])
            got, V = np.linalg.eigh(R)
            assert np.allclose(got, want, rtol=1e-10)
            # same eigenvectors: R commutes with S
            assert np.allclose(R @ S, S @ R, atol=1e-10)


def test_approximate_pdf_limits(orc):
    c = np.array([0.4, 0.5, 0.6])
    wo = _unit([0.2, 0.1, 0.97])
    for met in [0.0, 1.0]:
        ps = orc.disney_spec_prob(c, met)
        lum = 0.2126 * 0.4 + 0.7152 * 0.5 + 0.0722 * 0.6
        assert ps == pytest.approx(1 / (1 + (1 - met) * lum), rel=1e-14)
        # at w_i = w_o the half vector is w_o: ps D~_wo(w_o) + (1 - ps) / pi
        s6 = _s6(np.diag([1.0, 0.3, 0.2]))
        r6 = orc.sggx_roughened(s6, 0.5)
        ref = ps * orc.sggx_vndf(r6, wo, wo[None])[0] + (1 - ps) / math.pi
        assert orc.sggx_disney_pdf_approx(s6, c, 0.5, met, wo, wo) == pytest.approx(ref, rel=1e-12)
        assert orc.sggx_disney_pdf_approx(s6, c, 0.5, met, wo, -wo) == 0.0


def _disney_scene(seed, n_emit, frac):
    return scenes.with_sggx(scenes.tiny_random(seed=seed, n_emit=n_emit), seed=seed + 1, frac=frac, base="disney")


def test_disney_mis_estimators_agree(orc):
    sc = _disney_scene(0, 200, 0.7)
    S = orc.Scene(sc)
    cam = dict(scenes.camera("tiny_random"), width=24, height=24)
    spp = 256
    res = {}
    for mode in (0, 1, 2):
        s, s2, _ = S.render(cam, {"spp": spp, "max_depth": 3, "seed": 7 + mode, "mis_mode": mode})
        npx = s.shape[0]
        per = s.sum(1) / 3 / spp
        var = (s2.sum(1) / 3 / spp - per ** 2).mean()
        res[mode] = (s.sum() / (npx * spp * 3), math.sqrt(max(var, 0) / (npx * spp)))
    for a in (1, 2):
        assert abs(res[a][0] - res[0][0]) <= 3 * math.hypot(res[a][1], res[0][1]), res


def test_scene_rejects_bad_metallic(orc):
    sc = _disney_scene(0, 2, 1.0)
    sc["metallic"][4] = 1.5
    with pytest.raises(ValueError):
        orc.Scene(sc)
