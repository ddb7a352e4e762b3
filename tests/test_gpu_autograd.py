"""GPU tests of the torch.autograd functions over the differentiable images
(Sec. 7.2 eq. accum_cdf; Sec. 8 eq. rf), whose backward is the library's
vector-Jacobian product: against the fused loss gradient of the same entry
points, against FP64 central finite differences of the oracle for a loss
that is not the fused one (a weighted sum of the images), and across a
hierarchy rebuilt between forward and backward.

Tolerances:
  forward      identical to the plain entry point (same kernels, same input)
  vs fused     per primitive, every component within 1e-4 of that primitive's
               largest component (float atomics in another order; dLoss/dC
               formed in float by torch instead of in double)
  vs FD        per primitive, within 2% of its largest finite-difference
               component (as the fused gradient's own test), over the
               components whose quotient does not depend on the step
"""
import sys

import numpy as np
import pytest

from paper_2406_09733_amd import scenes

pytestmark = pytest.mark.gpu

_SHAPE = [("mean", 0, 3), ("scale", 3, 3), ("rotation", 6, 4), ("density", 10, 1)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2406_09733_amd as P
    return P.Context(0)


def _dense_tiny(seed=None):
    sc = scenes.tiny_random() if seed is None else scenes.tiny_random(seed=seed)
    sc["density"] = (np.asarray(sc["density"], np.float32) * 8.0).astype(np.float32)
    rng = np.random.default_rng(7)
    sc["emission"] = rng.uniform(0.0, 2.0, (sc["mean"].shape[0], 3)).astype(np.float32)
    return sc


def _params(torch, sc, rgb=False):
    p = {}
    for k in ("mean", "scale", "rotation", "density", "emission", "albedo", "roughness"):
        p[k] = torch.tensor(np.asarray(sc[k], np.float32), device="cuda")
    p["material"] = torch.tensor(np.asarray(sc["material"], np.int32), device="cuda")
    for k in ("mean", "scale", "rotation", "density") + (("emission",) if rgb else ()):
        p[k].requires_grad_(True)
    return p


def _rows(p, rgb=False):
    parts = [p["mean"].grad, p["scale"].grad, p["rotation"].grad, p["density"].grad[:, None]]
    if rgb:
        parts.append(p["emission"].grad)
    import torch
    return torch.cat(parts, 1).cpu().numpy().astype(np.float64)


def _close_rows(a, b, tol):
    scale = np.maximum(np.abs(b).max(axis=1, keepdims=True), 1e-30)
    return np.abs(a - b) / scale


@pytest.mark.parametrize("rgb", [False, True])
def test_autograd_matches_the_fused_loss_gradient(ctx, torch, rgb):
    from paper_2406_09733_amd import autograd as A
    _say("autograd vs fused gradient", "rf" if rgb else "accum_cdf")
    sc = _dense_tiny()
    n = sc["mean"].shape[0]
    rays = scenes.probe_rays(sc, 1024, seed=231, aimed_frac=1.0, finite_frac=0.2)
    rng = np.random.default_rng(3)
    ex = rng.integers(-1, n, rays.shape[0]).astype(np.int32)
    ex[::2] = -1
    p = _params(torch, sc, rgb)
    img = (A.rf_render if rgb else A.accum_cdf)(ctx, p, rays, ex)
    ctx.build_bvh(sc)
    plain = ctx.rf_render(rays, exclude=ex) if rgb else ctx.accum_cdf(rays, exclude=ex)
    assert torch.equal(img.detach(), plain)
    target = (0.5 * plain + 0.05).detach()
    loss = ((img - target) ** 2).sum()
    loss.backward()
    ga = _rows(p, rgb)
    gf = torch.zeros((n, 14 if rgb else 11), device="cuda", dtype=torch.float32)
    lf = torch.zeros(1, device="cuda", dtype=torch.float32)
    (ctx.rf_render if rgb else ctx.accum_cdf)(rays, target=target, exclude=ex, loss=lf, grad=gf)
    ctx.sync()
    gf = gf.cpu().numpy().astype(np.float64)
    assert abs(float(lf.item()) - float(loss.item())) <= 1e-5 * float(loss.item())
    live = np.abs(gf).max(axis=1) > 0
    _say(f"  {live.sum()} primitives with gradient; max row-relative diff "
         f"{_close_rows(ga[live], gf[live], 0).max():.2e}")
    assert np.array_equal(np.abs(ga).max(axis=1) > 0, live)
    assert np.all(_close_rows(ga[live], gf[live], 0) <= 1e-4)


def test_autograd_weighted_image_vs_finite_differences(ctx, orc, torch):
    from paper_2406_09733_amd import autograd as A
    _say("autograd of a weighted sum of C vs FP64 central differences of the oracle")
    sc = _dense_tiny()
    n = sc["mean"].shape[0]
    rays = scenes.probe_rays(sc, 512, seed=232, aimed_frac=1.0, finite_frac=0.2)
    w = np.random.default_rng(4).uniform(-1.0, 1.0, rays.shape[0])
    p = _params(torch, sc)
    C = A.accum_cdf(ctx, p, rays)
    (C * torch.tensor(w, device="cuda", dtype=torch.float32)).sum().backward()
    g = _rows(p)
    _, ts0 = orc.Scene(sc).accum_cdf(rays)

    def obj(s2):
        C2, _ = orc.Scene(s2).accum_cdf(rays, tsat=ts0)
        return float(np.dot(w.astype(np.float32).astype(np.float64), C2))

    def quotient(k, name, j, h):
        base = np.asarray(sc[name], np.float32).reshape(n, -1)
        v = float(base[k, j])
        vals = []
        for sgn in (1, -1):
            arr = base.copy()
            arr[k, j] = np.float32(v + sgn * h)
            s2 = dict(sc)
            s2[name] = arr.reshape(np.asarray(sc[name]).shape)
            vals.append((float(arr[k, j]), obj(s2)))
        return (vals[0][1] - vals[1][1]) / (vals[0][0] - vals[1][0])

    # A component whose quotient changes with the step has a kink inside the
    # stencil (a ray's chord appearing or vanishing at the cut-off ellipsoid,
    # where the clipped integral grows like the square root of the overlap):
    # there the difference quotient is no derivative and is not compared.
    kinks = 0
    for k in np.argsort(-np.abs(g).max(axis=1))[:5]:
        fd = np.zeros(11)
        smooth = np.ones(11, bool)
        smin = float(np.min(sc["scale"][k]))
        for name, off, width in _SHAPE:
            for j in range(width):
                v = float(np.asarray(sc[name], np.float32).reshape(n, -1)[k, j])
                h = {"mean": 1e-3 * smin, "scale": 1e-3 * v, "rotation": 1e-3, "density": 1e-3 * v}[name]
                fd[off + j] = quotient(k, name, j, h)
                fd4 = quotient(k, name, j, h / 4)
                smooth[off + j] = abs(fd[off + j] - fd4) <= 1e-3 * max(abs(fd[off + j]), abs(fd4)) + 1e-9
        kinks += int((~smooth).sum())
        assert smooth.sum() >= 8, (k, fd)
        rel = np.abs(g[k] - fd)[smooth].max() / np.abs(fd[smooth]).max()
        _say(f"  prim {k}: max |g - fd| / max |fd| = {rel:.2e} ({int((~smooth).sum())} components at a kink)")
        assert rel <= 2e-2, (k, g[k], fd)
    assert kinks <= 10  # of 55 components (5 seen)


def test_autograd_backward_after_another_build(ctx, torch):
    from paper_2406_09733_amd import autograd as A
    _say("autograd backward after the hierarchy was rebuilt for another scene")
    sa, sb = _dense_tiny(), _dense_tiny(seed=11)
    rays = scenes.probe_rays(sa, 1024, seed=233, aimed_frac=1.0, finite_frac=0.2)
    w = torch.tensor(np.random.default_rng(5).uniform(0.0, 1.0, rays.shape[0]), device="cuda",
                     dtype=torch.float32)
    pa = _params(torch, sa)
    (A.accum_cdf(ctx, pa, rays) * w).sum().backward()
    ref = _rows(pa)
    pa2, pb = _params(torch, sa), _params(torch, sb)
    Ca = A.accum_cdf(ctx, pa2, rays)
    Cb = A.accum_cdf(ctx, pb, rays)  # replaces the hierarchy
    ((Ca + 0.0 * Cb) * w).sum().backward()
    got = _rows(pa2)
    live = np.abs(ref).max(axis=1) > 0
    assert live.sum() > 10
    assert np.all(_close_rows(got[live], ref[live], 0) <= 1e-5)
    assert np.all(got[~live] == 0)


def test_autograd_on_a_scene_with_sggx_primitives(ctx, torch):
    # the SGGX matrices and metallic values ride along as fixed fields, so the
    # hierarchy rebuilt for the image accepts material 3 primitives; the
    # transmittance image does not depend on the phase function
    from paper_2406_09733_amd import autograd as A
    _say("autograd accum_cdf on a scene with Disney-base SGGX primitives")
    sa = _dense_tiny()
    sg = scenes.with_sggx(sa, seed=3, frac=0.5, base="disney")
    rays = scenes.probe_rays(sa, 1024, seed=234, aimed_frac=1.0, finite_frac=0.2)
    w = torch.tensor(np.random.default_rng(6).uniform(0.0, 1.0, rays.shape[0]), device="cuda",
                     dtype=torch.float32)
    pa = _params(torch, sa)
    (A.accum_cdf(ctx, pa, rays) * w).sum().backward()
    pg = _params(torch, sg)
    pg["sggx"] = torch.tensor(sg["sggx"], device="cuda")
    pg["metallic"] = torch.tensor(sg["metallic"], device="cuda")
    pg["material"] = torch.tensor(sg["material"], device="cuda")
    (A.accum_cdf(ctx, pg, rays) * w).sum().backward()
    ref, got = _rows(pa), _rows(pg)
    live = np.abs(ref).max(axis=1) > 0
    assert live.sum() > 10
    # float atomics add in any order
    assert np.all(_close_rows(got[live], ref[live], 0) <= 1e-5)
    assert np.all(got[~live] == 0)
