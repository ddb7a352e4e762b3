"""Independent numerical routes used to pin the oracle (test helpers only).

Nothing here calls the oracle's arithmetic: rotations come from scipy, chord
end points from fitting the exact quadratic through three samples, and ray
integrals from adaptive quadrature of the truncated kernel.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate
from scipy.spatial.transform import Rotation

R_CUT = float(np.sqrt(-2.0 * np.log(0.01)))


def rotation(q):
    return Rotation.from_quat(np.asarray(q, np.float64), scalar_first=True).as_matrix()


def prim(sc, k):
    mu = sc["mean"][k].astype(np.float64)
    s = sc["scale"][k].astype(np.float64)
    R = rotation(sc["rotation"][k])
    Sigma = R @ np.diag(s * s) @ R.T
    return mu, s, R, Sigma, float(sc["density"][k])


def mahal2(sc, k, p):
    mu, s, R, Sigma, d = prim(sc, k)
    x = np.asarray(p, np.float64) - mu
    return float(x @ np.linalg.solve(Sigma, x))


def kernel(sc, k, p):
    """Truncated Gaussian G_k(p) = d exp(-q/2) for q <= r^2, else 0."""
    q = mahal2(sc, k, p)
    return prim(sc, k)[4] * np.exp(-0.5 * q) if q <= R_CUT ** 2 else 0.0


def chord(sc, k, o, w):
    """Chord of the cut-off ellipsoid along o + t w (None if missed); the
    quadratic q(t) - r^2 is fitted exactly from three samples."""
    o = np.asarray(o, np.float64); w = np.asarray(w, np.float64)
    ts = np.array([0.0, 1.0, 2.0])
    qs = np.array([mahal2(sc, k, o + t * w) for t in ts])
    c2 = 0.5 * (qs[2] - 2 * qs[1] + qs[0])
    c1 = qs[1] - qs[0] - c2
    c0 = qs[0] - R_CUT ** 2
    disc = c1 * c1 - 4 * c2 * c0
    if disc <= 0:
        return None
    sq = np.sqrt(disc)
    return (-c1 - sq) / (2 * c2), (-c1 + sq) / (2 * c2)


def integral(sc, k, o, w, x, y):
    """int_x^y G_k(o + t w) dt by adaptive quadrature inside the chord."""
    ch = chord(sc, k, o, w)
    if ch is None:
        return 0.0
    a, b = max(x, ch[0]), min(y, ch[1])
    if not a < b:
        return 0.0
    o = np.asarray(o, np.float64); w = np.asarray(w, np.float64)
    mu, s, R, Sigma, d = prim(sc, k)
    Si = np.linalg.inv(Sigma)
    f = lambda t: d * np.exp(-0.5 * (o + t * w - mu) @ Si @ (o + t * w - mu))
    val, err = integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)
    return val
