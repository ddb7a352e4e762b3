"""Pins of the oracle's neural radiance cache: the input encoding (sinusoids,
real spherical harmonics), the MLP forward pass and its hand-written
gradient, and the Adam step -- against quadrature, torch autograd, central
finite differences and torch.optim.Adam (independent routes)."""
import numpy as np
import pytest
import torch


def _weights(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    from oracle import NRC_LAYERS
    ws = []
    for (o, i) in NRC_LAYERS:
        ws.append(rng.uniform(-1, 1, (o, i)) * scale * np.sqrt(6.0 / i))
    return np.concatenate([w.ravel() for w in ws])


def _inputs(n, seed=1):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3))
    wo = rng.normal(size=(n, 3)); wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    nrm = rng.normal(size=(n, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    rough = rng.uniform(0.02, 1, (n, 1)); alb = rng.uniform(0, 1, (n, 3))
    return np.concatenate([pos, wo, nrm, rough, alb, np.zeros((n, 3))], 1).astype(np.float32)


def test_encoding_layout_and_sinusoids(orc):
    x = _inputs(50)
    lo, hi = np.array([-1.0, 0.0, 0.5]), np.array([2.0, 1.0, 1.5])
    f = orc.nrc_encode(x, lo, hi)
    assert f.shape == (50, 96)
    xh = (x[:, :3].astype(np.float64) - lo) / (hi - lo)
    for a in range(3):
        for j in range(12):
            assert np.allclose(f[:, 24 * a + 2 * j], np.sin(2.0 ** j * np.pi * xh[:, a]), atol=1e-12)
            assert np.allclose(f[:, 24 * a + 2 * j + 1], np.cos(2.0 ** j * np.pi * xh[:, a]), atol=1e-12)
    assert np.allclose(f[:, 88:95], x[:, 6:13])
    assert np.all(f[:, 95] == 0.0)


def test_spherical_harmonics_are_orthonormal(orc):
    # Gauss-Legendre x uniform-phi quadrature of Y_i Y_j over the sphere
    nt, nph = 40, 80
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    C, P = np.meshgrid(ct, ph, indexing="ij")
    st = np.sqrt(1 - C ** 2)
    d = np.stack([st * np.cos(P), st * np.sin(P), C], -1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    x = np.zeros((d.shape[0], 16), np.float32)
    x[:, 3:6] = d
    Y = orc.nrc_encode(x, np.zeros(3), np.ones(3))[:, 72:88]
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-5), np.abs(G - np.eye(16)).max()


def _torch_mlp(W, feat):
    from oracle import NRC_LAYERS
    Wt = torch.tensor(W, dtype=torch.float64, requires_grad=True)
    x = torch.tensor(feat, dtype=torch.float64)
    off = 0
    h = x
    for li, (o, i) in enumerate(NRC_LAYERS):
        w = Wt[off:off + o * i].reshape(o, i)
        off += o * i
        h = h @ w.T
        if li < 4:
            h = torch.relu(h)
    return Wt, h


def test_forward_matches_torch(orc):
    W = _weights(0)
    feat = orc.nrc_encode(_inputs(64), np.zeros(3), np.ones(3))
    _, y = _torch_mlp(W, feat)
    assert np.allclose(orc.nrc_forward(W, feat), y.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gradient_matches_autograd_and_finite_differences(orc):
    W = _weights(2)
    feat = orc.nrc_encode(_inputs(32, 3), np.zeros(3), np.ones(3))
    tgt = np.random.default_rng(4).uniform(0, 2, (32, 3))
    loss, g = orc.nrc_loss_grad(W, feat, tgt)
    Wt, y = _torch_mlp(W, feat)
    t = torch.tensor(tgt)
    L = (((y - t) ** 2) / (y.detach() ** 2 + 0.01)).mean()
    L.backward()
    assert loss == pytest.approx(L.item(), rel=1e-12)
    assert np.allclose(g, Wt.grad.numpy(), rtol=1e-9, atol=1e-14)
    # central finite differences of the oracle's own loss (sg(y) held fixed
    # means the denominator uses y at the perturbed point; compare on a
    # loss with a frozen denominator instead)
    y0 = orc.nrc_forward(W, feat)
    den = y0 ** 2 + 0.01

    def frozen(Wp):
        yp = orc.nrc_forward(Wp, feat)
        return np.mean((yp - tgt) ** 2 / den)

    rng = np.random.default_rng(5)
    for p in rng.choice(W.size, 40, replace=False):
        h = 1e-6 * max(1.0, abs(W[p]))
        Wp, Wm = W.copy(), W.copy()
        Wp[p] += h
        Wm[p] -= h
        fd = (frozen(Wp) - frozen(Wm)) / (2 * h)
        assert fd == pytest.approx(g[p], rel=1e-5, abs=1e-10)


def test_adam_matches_torch(orc):
    W = _weights(6)
    rng = np.random.default_rng(7)
    m = np.zeros_like(W); v = np.zeros_like(W)
    p = torch.nn.Parameter(torch.tensor(W, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.99), eps=1e-8)
    Wc = W.copy()
    for t in range(1, 6):
        g = rng.normal(size=W.size)
        Wc, m, v = orc.nrc_adam(Wc, m, v, g, t)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(Wc, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_emulation_without_rounding_is_the_oracle(orc):
    # the test helper that emulates the kernels' bf16 arithmetic computes the
    # oracle's FP64 loss and gradient when its rounding is switched off
    import nrc_emul
    rng = np.random.default_rng(8)
    W = np.concatenate([rng.uniform(-1, 1, o * i) * np.sqrt(6.0 / i) for (o, i) in orc.NRC_LAYERS])
    feat = rng.uniform(-1, 1, (97, 96))
    tgt = rng.uniform(0, 2, (97, 3))
    l_ref, g_ref = orc.nrc_loss_grad(W, feat, tgt)
    l, g = nrc_emul.train_grad(W, feat, tgt, rounding=False)
    assert abs(l - l_ref) <= 1e-12 * abs(l_ref)
    assert np.allclose(g, g_ref, rtol=1e-10, atol=1e-14)
