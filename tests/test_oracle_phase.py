"""Pins of the oracle's delta-NDF phase functions (Sec. 6: a single facet
normal reduces eq. phase_function to the surface BSDF times the cosine)."""
import numpy as np
import pytest


def _sphere_grid(n):
    # golden-spiral quadrature nodes with equal weights 4 pi / n
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    phi = np.pi * (3 - np.sqrt(5)) * np.arange(n)
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1), 4 * np.pi / n


def _rand_dir(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_lambert_integrates_to_albedo(orc):
    rng = np.random.default_rng(0)
    dirs, dw = _sphere_grid(200000)
    for _ in range(3):
        nrm, wo = _rand_dir(rng), _rand_dir(rng)
        alb = rng.uniform(0.1, 1.0, 3)
        tot = np.zeros(3); pdf_tot = 0.0
        for wi in dirs[::50]:
            f, p = orc.phase_eval(0, alb, 0.5, nrm, wo, wi)
            tot += f; pdf_tot += p
        tot *= dw * 50; pdf_tot *= dw * 50
        assert np.allclose(tot, alb, rtol=5e-3)
        assert pdf_tot == pytest.approx(1.0, rel=5e-3)


def test_ggx_energy_and_sample_consistency(orc):
    rng = np.random.default_rng(1)
    for rough in [0.3, 0.6, 1.0]:
        nrm, wo = _rand_dir(rng), _rand_dir(rng)
        alb = np.ones(3)
        # MC with the sampler: E[f/pdf] over accepted samples = int f
        n = 20000
        u = rng.uniform(size=(n, 2))
        acc = 0.0; nacc = 0
        for i in range(n):
            wi, wgt, p = orc.phase_sample(1, alb, rough, nrm, wo, u[i, 0], u[i, 1])
            if p > 0:
                f, pe = orc.phase_eval(1, alb, rough, nrm, wo, wi)
                assert pe == pytest.approx(p, rel=1e-9)
                assert np.allclose(f / pe, wgt, rtol=1e-9)
                acc += wgt[0]; nacc += 1
        albedo_est = acc / n
        assert 0.3 < albedo_est <= 1.0 + 3 * np.sqrt(1.0 / n)
        # the pdf integrates to the accepted fraction (samples below the facet are dropped)
        dirs, dw = _sphere_grid(400000)
        ptot = sum(orc.phase_eval(1, alb, rough, nrm, wo, wi)[1] for wi in dirs[::20]) * dw * 20
        assert ptot == pytest.approx(nacc / n, abs=0.02)


def test_ggx_reciprocity(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        nrm = _rand_dir(rng)
        wo, wi = _rand_dir(rng), _rand_dir(rng)
        if (nrm @ wo) * (nrm @ wi) <= 0:
            continue
        alb = rng.uniform(0, 1, 3); rough = rng.uniform(0.05, 1)
        f1, _ = orc.phase_eval(1, alb, rough, nrm, wo, wi)
        f2, _ = orc.phase_eval(1, alb, rough, nrm, wi, wo)
        n = nrm * np.sign(nrm @ wo)
        assert np.allclose(f1 / (n @ wi), f2 / (n @ wo), rtol=1e-10)


def test_phase_sample_histogram_matches_pdf(orc):
    # chi-square of sampled directions against the pdf integrated over bins
    rng = np.random.default_rng(3)
    nrm = np.array([0.0, 0.0, 1.0]); wo = np.array([0.6, 0.0, 0.8])
    for mat, rough in [(0, 0.5), (1, 0.5)]:
        n = 40000
        u = rng.uniform(size=(n, 2))
        cz = []
        for i in range(n):
            wi, wgt, p = orc.phase_sample(mat, np.ones(3), rough, nrm, wo, u[i, 0], u[i, 1])
            if p > 0:
                cz.append(wi[2])
        cz = np.array(cz)
        edges = np.linspace(0, 1, 11)
        hist = np.histogram(cz, edges)[0]
        # expected mass per bin of cos(theta) by quadrature of the pdf
        dirs, dw = _sphere_grid(400000)
        pd = np.array([orc.phase_eval(mat, np.ones(3), rough, nrm, wo, d)[1] for d in dirs[::4]])
        zz = dirs[::4, 2]
        exp = np.array([(pd[(zz >= edges[j]) & (zz < edges[j + 1])]).sum() * dw * 4 for j in range(10)])
        exp = exp / exp.sum() * hist.sum()
        m = exp > 20
        chi2 = (((hist - exp) ** 2) / exp)[m].sum()
        assert chi2 < 40, (mat, chi2)


def _ggx_slope_pdf(a, x, y):
    # the GGX (Trowbridge-Reitz) distribution of microfacet slopes of roughness a
    return 1.0 / (np.pi * a * a * (1.0 + (x * x + y * y) / (a * a)) ** 2)


def _smith_lambda_by_definition(a, cos_t):
    # Smith's Lambda from its definition over the slope distribution:
    # Lambda = (1/mu) int_mu^inf (q - mu) P2(q) dq, mu = cot(theta), with the
    # marginal P2(q) = int P22(q, y) dy taken by quadrature too
    from scipy import integrate
    mu = cos_t / np.sqrt(max(0.0, 1.0 - cos_t * cos_t))
    P2 = lambda q: integrate.quad(lambda y: _ggx_slope_pdf(a, q, y), -np.inf, np.inf, epsabs=0, epsrel=1e-12)[0]
    val = integrate.quad(lambda q: (q - mu) * P2(q), mu, np.inf, epsabs=0, epsrel=1e-10, limit=200)[0]
    return val / mu


def test_ggx_form_against_the_microfacet_definitions(orc):
    # With albedo 1 (Schlick F = 1) the glossy delta-NDF phase function is
    # D(h) G2(w_o, w_i) / (4 cos_o) and its sampling pdf G1(w_o) D(h) / (4
    # cos_o).  Here D comes from the slope distribution (D(h) = P22(slope)
    # / cos^4 theta_h), G1 = 1/(1 + Lambda(w_o)) and the height-correlated
    # G2 = 1/(1 + Lambda(w_o) + Lambda(w_i)) with Lambda integrated from its
    # definition, so a wrong exponent, a dropped term or the uncorrelated
    # form G1 G1 fails it
    rng = np.random.default_rng(21)
    nrm = np.array([0.0, 0.0, 1.0])
    for _ in range(12):
        rough = rng.uniform(0.3, 1.0)
        a = rough * rough
        wo, wi = _rand_dir(rng), _rand_dir(rng)
        wo[2], wi[2] = abs(wo[2]) + 0.05, abs(wi[2]) + 0.05
        wo /= np.linalg.norm(wo)
        wi /= np.linalg.norm(wi)
        f, pdf = orc.phase_eval(1, np.ones(3), rough, nrm, wo, wi)
        h = wo + wi
        h /= np.linalg.norm(h)
        D = _ggx_slope_pdf(a, -h[0] / h[2], -h[1] / h[2]) / h[2] ** 4
        lo, li = _smith_lambda_by_definition(a, wo[2]), _smith_lambda_by_definition(a, wi[2])
        f_ref = D / (1.0 + lo + li) / (4.0 * wo[2])
        pdf_ref = D / (1.0 + lo) / (4.0 * wo[2])
        assert np.allclose(f, f_ref, rtol=1e-7), (f, f_ref)
        assert pdf == pytest.approx(pdf_ref, rel=1e-7)


def test_ggx_fresnel_limits(orc):
    # Schlick's Fresnel with F0 = albedo: at w_i = w_o (half vector along both,
    # normal incidence on the microfacet) the reflectance is the albedo, so
    # f(albedo) / f(1) = albedo; at grazing microfacet incidence (w_i = -w_o
    # mirrored about a half vector nearly perpendicular to w_o) it tends to 1
    rng = np.random.default_rng(22)
    nrm = np.array([0.0, 0.0, 1.0])
    for _ in range(6):
        alb = rng.uniform(0.05, 0.9, 3)
        w = _rand_dir(rng)
        w[2] = abs(w[2]) + 0.1
        w /= np.linalg.norm(w)
        f1, _ = orc.phase_eval(1, np.ones(3), 0.6, nrm, w, w)
        fa, _ = orc.phase_eval(1, alb, 0.6, nrm, w, w)
        assert np.allclose(fa / f1, alb, rtol=1e-12)
    # nearly opposite directions in the upper hemisphere: w_i . h -> 0
    wo = np.array([np.sin(1.5), 0.0, np.cos(1.5)])
    wi = np.array([-np.sin(1.5), 1e-3, np.cos(1.5)])
    wi /= np.linalg.norm(wi)
    f1, _ = orc.phase_eval(1, np.ones(3), 0.8, nrm, wo, wi)
    fa, _ = orc.phase_eval(1, np.full(3, 0.2), 0.8, nrm, wo, wi)
    h = (wo + wi) / np.linalg.norm(wo + wi)
    c = float(wi @ h)
    assert c < 0.08
    # reflectance rises from 0.2 toward 1: above 0.2 + 0.8 * 0.92^5 = 0.727
    # there, and below 1
    assert np.all(fa / f1 > 0.72) and np.all(fa / f1 < 1.0)
