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
