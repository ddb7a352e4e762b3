"""GPU parity of the neural radiance cache (nrc.hip) against the FP64 oracle,
through the C ABI.

Arithmetic of the kernels: bf16 weights and activations, float32
accumulation on the matrix cores, float32 master weights for Adam.  The
oracle runs in FP64 on the same bf16-rounded weights and features, so the
tolerances below come from rounding each hidden activation (and, in the
backward pass, each back-propagated error) to bf16, unit roundoff u = 2^-9,
a rounding error uniform in +-u|x| with variance (u x)^2 / 3:
  encoding        |d| <= 2e-6 (float sincospi of an exactly reduced argument;
                  float products for the harmonics)
  forward         |dy| <= 6 sigma_y + 1e-6, sigma_y^2 the variance of the
                  output error, propagated layer by layer with the squared
                  weights from the oracle's exact activations (on a CPU
                  emulation of the kernel's arithmetic, 60K outputs stay
                  below 3.4 sigma; the kernel agrees with that emulation to
                  ~2e-6)
  fused encoding  the forward pass on raw inputs equals the forward pass on
                  the GPU's own features bit for bit
  loss            |dL| <= 6 sigma_L + 1e-5 L, sigma_L from sigma_y through dL/dy
  gradient        per element against an emulation of the kernels' bf16
                  arithmetic (tests/nrc_emul.py: the same roundings of
                  activations, loss gradient and back-propagated errors;
                  FP64 sums, pinned to the oracle with rounding off):
                  |dg| <= 2^-9 (|g| + 0.02 max|g| of its layer), except for
                  at most 2% of a layer's elements (at most 8x the bar: a
                  ReLU unit whose pre-activation is within float32 rounding
                  of zero switches and moves a row), and normwise within
                  2^-9 of the emulation; and against
                  the exact FP64 gradient of the oracle per layer
                  ||dg|| <= 0.08 ||g|| and cosine > 0.995 (about a dozen
                  roundings lie between the loss and each weight, ~12 u =
                  2.3%, plus ReLU units whose pre-activation lies within
                  rounding of zero and switch)
  Adam            the master weights after each step equal the oracle's Adam
                  step on the kernel's gradient to float32 rounding
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U = 2.0 ** -9


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


def bf16(x):
    import torch
    return torch.tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def weights(seed, scale=1.0):
    from oracle import NRC_LAYERS
    rng = np.random.default_rng(seed)
    ws = [rng.uniform(-1, 1, (o, i)) * scale * np.sqrt(6.0 / i) for (o, i) in NRC_LAYERS]
    return bf16(np.concatenate([w.ravel() for w in ws]))


def inputs(n, seed, box=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0)):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(box[:3]), np.array(box[3:])
    pos = lo + (hi - lo) * rng.uniform(-0.05, 1.05, (n, 3))
    wo = rng.normal(size=(n, 3)); wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    nrm = rng.normal(size=(n, 3)); nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    x = np.concatenate([pos, wo, nrm, rng.uniform(0.02, 1, (n, 1)), rng.uniform(0, 1, (n, 3)),
                        np.zeros((n, 3))], 1)
    return x.astype(np.float32)


def split(W):
    from oracle import NRC_LAYERS
    out, off = [], 0
    for (o, i) in NRC_LAYERS:
        out.append(W[off:off + o * i].reshape(o, i))
        off += o * i
    return out


def forward_sigma(W, feat):
    """standard deviation of the output error from rounding every hidden
    activation to bf16 (variance (u a)^2 / 3 per activation), propagated with
    the squared weights; errors pass through inactive ReLU units as well,
    which covers units whose pre-activation is within rounding of zero"""
    h, v = feat, np.zeros_like(feat)
    for l, w in enumerate(split(W)):
        z = h @ w.T
        v = v @ (w ** 2).T
        if l < 4:
            h = np.maximum(z, 0)
            v = v + (U * h) ** 2 / 3
    return np.sqrt(v)


def loss_sigma(y, t, sy):
    n = y.shape[0]
    den = y * y + 0.01
    dL = (2 * (y - t) / den - 2 * y * (y - t) ** 2 / den ** 2) / (3 * n)
    return np.sqrt(np.sum((dL * sy) ** 2))


BOX = (-1.0, 0.0, 0.5, 2.0, 1.0, 1.5)


def test_encoding_parity(ctx, torch, orc):
    _say("nrc encode parity")
    for n, seed in ((1, 0), (1000, 1), (4099, 2)):
        x = inputs(n, seed, BOX)
        got = ctx.nrc_encode(x, box=BOX).cpu().numpy()
        ref = orc.nrc_encode(x, BOX[:3], BOX[3:])
        err = np.abs(got - ref).max()
        _say(f"  n={n}: max |d| {err:.2e}")
        assert err <= 2e-6


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 4097])
def test_forward_parity(ctx, torch, orc, n):
    _say(f"nrc forward parity n={n}")
    W = weights(3)
    ctx.nrc_set_weights(W.astype(np.float32))
    x = inputs(n, 10 + n, BOX)
    feat = bf16(orc.nrc_encode(x, BOX[:3], BOX[3:]))
    y = ctx.nrc_forward(feat.astype(np.float32)).cpu().numpy().astype(np.float64)
    ref = orc.nrc_forward(W, feat)
    sig = forward_sigma(W, feat)
    err = np.abs(y - ref)
    _say(f"  max |dy| {err.max():.3e}, max |dy|/sigma {np.max(err / (sig + 1e-12)):.2f}, "
         f"rms y {np.sqrt((ref ** 2).mean()):.3e}")
    assert np.all(err <= 6 * sig + 1e-6)
    # the fused encoding gives the same result as the GPU's own features
    f_gpu = ctx.nrc_encode(x, box=BOX)
    y1 = ctx.nrc_forward(f_gpu).cpu().numpy()
    y0 = ctx.nrc_forward(x, box=BOX).cpu().numpy()
    assert np.array_equal(y0, y1)


def test_weights_roundtrip(ctx, torch):
    W = np.random.default_rng(5).normal(size=18624).astype(np.float32)
    ctx.nrc_set_weights(W)
    assert np.array_equal(ctx.nrc_get_weights().cpu().numpy(), W)


@pytest.mark.parametrize("n", [1, 33, 3001, 65536])
def test_train_step_parity(ctx, torch, orc, n):
    _say(f"nrc train step parity n={n}")
    from oracle import NRC_LAYERS
    W = weights(7)
    ctx.nrc_set_weights(W.astype(np.float32))
    x = inputs(n, 20 + n, BOX)
    feat = bf16(orc.nrc_encode(x, BOX[:3], BOX[3:]))
    tgt = np.random.default_rng(n).uniform(0, 2, (n, 3)).astype(np.float32)
    loss, g = ctx.nrc_train_step(feat.astype(np.float32), tgt, lr=1e-3, want_grad=True)
    loss, g = float(loss.cpu().numpy()[0]), g.cpu().numpy().astype(np.float64)
    lref, gref = orc.nrc_loss_grad(W, feat, tgt.astype(np.float64))
    yref = orc.nrc_forward(W, feat)
    sl = loss_sigma(yref, tgt.astype(np.float64), forward_sigma(W, feat))
    _say(f"  loss gpu {loss:.6f} oracle {lref:.6f} (|d| / sigma {abs(loss - lref) / sl:.2f})")
    assert abs(loss - lref) <= 6 * sl + 1e-5 * lref
    # per element against the emulation of the kernels' bf16 arithmetic (the
    # same roundings at the same points; sums in FP64 instead of FP32):
    # |dg| <= 2^-9 (|g| + 0.02 max|g| of the layer), and normwise against the
    # exact FP64 gradient of the oracle
    import nrc_emul
    _, gem = nrc_emul.train_grad(W, feat, tgt.astype(np.float64))
    off = 0
    for l, (o, i) in enumerate(NRC_LAYERS):
        a, b, e = g[off:off + o * i], gref[off:off + o * i], gem[off:off + o * i]
        off += o * i
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        tol = U * (np.abs(e) + 0.02 * np.abs(e).max()) + 1e-12
        ratio = np.abs(a - e) / tol
        worst, beyond = float(ratio.max()), int((ratio > 1.0).sum())
        _say(f"  layer {l}: vs bf16 emulation worst |dg|/bar {worst:.3f}, {beyond} of {ratio.size} beyond (max rel "
             f"{np.max(np.abs(a - e) / (np.abs(e) + 1e-30 + 0.02 * np.abs(e).max())):.2e}); "
             f"vs FP64 normwise {rel:.3e}, cosine {cos:.6f}")
        # a ReLU unit whose pre-activation lies within float32 rounding of
        # zero can switch between the matrix-core sum and the emulation's FP64
        # sum, which moves a row of the layer's gradient (up to 96 elements) by
        # that record's terms; a bf16 rounding that lands on the other side
        # moves single terms by an ulp: at most 2% of a layer's elements may
        # exceed the bar, by a bounded factor, and normwise the layer stays
        # within the bar's 2^-9
        assert beyond <= max(2, ratio.size // 50) and worst <= 8.0
        assert np.linalg.norm(a - e) <= U * np.linalg.norm(e)
        assert rel <= 0.08 and cos > 0.995
    # Adam on the master weights: one step from zero moments
    Wn = ctx.nrc_get_weights().cpu().numpy().astype(np.float64)
    Wa, _, _ = orc.nrc_adam(W, np.zeros_like(W), np.zeros_like(W), g.astype(np.float32).astype(np.float64), 1)
    assert np.allclose(Wn, Wa, rtol=1e-6, atol=1e-9), np.abs(Wn - Wa).max()


def test_adam_sequence(ctx, torch, orc):
    _say("nrc adam over 4 steps")
    W = weights(9)
    ctx.nrc_set_weights(W.astype(np.float32))
    n = 2048
    x = inputs(n, 99, BOX)
    tgt = np.random.default_rng(4).uniform(0, 1, (n, 3)).astype(np.float32)
    Wc, m, v = W.copy(), np.zeros_like(W), np.zeros_like(W)
    for t in range(1, 5):
        _, g = ctx.nrc_train_step(x, tgt, lr=3e-3, box=BOX, want_grad=True)
        Wc, m, v = orc.nrc_adam(Wc, m, v, g.cpu().numpy().astype(np.float64), t, lr=3e-3)
        Wn = ctx.nrc_get_weights().cpu().numpy().astype(np.float64)
        assert np.allclose(Wn, Wc, rtol=1e-5, atol=1e-7), (t, np.abs(Wn - Wc).max())


def test_training_fits_a_smooth_function(ctx, torch):
    # the cache learns: the loss on a smooth target field falls by 10x
    _say("nrc training convergence")
    from oracle import NRC_LAYERS
    rng = np.random.default_rng(1)
    W = np.concatenate([rng.uniform(-1, 1, o * i) * np.sqrt(6.0 / i) for (o, i) in NRC_LAYERS])
    ctx.nrc_set_weights(W.astype(np.float32))
    n = 16384
    losses = []
    for it in range(300):
        x = inputs(n, 1000 + it, BOX)
        p = x[:, :3]
        t = np.stack([0.5 + 0.4 * np.sin(2 * p[:, 0]), 0.3 + 0.2 * p[:, 1] * x[:, 5], 0.2 + 0.1 * x[:, 10]], 1)
        loss, _ = ctx.nrc_train_step(x, t.astype(np.float32), lr=1e-2, box=BOX)
        if it % 50 == 0 or it == 299:
            losses.append(float(loss.cpu().numpy()[0]))
    _say(f"  losses {['%.4f' % l for l in losses]}")
    assert losses[-1] < 0.1 * losses[0]


# ---------------------------------------------------------------------------
# the cache inside the path tracer
# ---------------------------------------------------------------------------
def albedo_cache(c):
    """network whose output is exactly c wherever the albedo's red channel is
    1 (feature 92): every product is exact in bf16 for bf16-exact c"""
    from oracle import NRC_LAYERS
    ws = []
    for li, (o, i) in enumerate(NRC_LAYERS):
        w = np.zeros((o, i))
        if li == 0:
            w[0, 92] = 1.0
        elif li < 4:
            w[0, 0] = 1.0
        else:
            w[:, 0] = c
        ws.append(w.ravel())
    return np.concatenate(ws)


def _np(t):
    return t.detach().cpu().numpy()


def test_render_termination_equals_shorter_paths(ctx, torch):
    from paper_2406_09733_amd import scenes
    _say("nrc render: termination without a cache == plain tracer of that depth")
    ctx.build_bvh(scenes.tiny_random())
    cam = dict(scenes.camera("tiny_random"), width=64, height=64)
    for k in (1, 2):
        a, _ = ctx.render(cam, {"spp": 4, "max_depth": k, "seed": 5})
        b, _ = ctx.render(cam, {"spp": 4, "max_depth": 6, "seed": 5, "nrc_mode": 3, "nrc_terminate_after": k})
        ctx.sync()
        assert np.array_equal(_np(a), _np(b))


def test_render_exact_cache_furnace(ctx, torch):
    from paper_2406_09733_amd import scenes
    _say("nrc render: exact cache in the white furnace")
    sc = scenes.tiny_random(seed=21, n_emit=0)
    sc["albedo"][:] = 1.0
    sc["material"][:] = 0
    sc["scale"] *= 3  # up to ~38 primitives overlap a point (the kernels hold 64)
    ctx.build_bvh(sc)
    ctx.nrc_set_weights(albedo_cache([1.0, 1.0, 1.0]).astype(np.float32))
    cam = dict(scenes.camera("tiny_random"), width=64, height=64)
    p = {"spp": 4, "max_depth": 1000, "seed": 3, "env_radiance": (1, 1, 1), "mis_mode": 1, "nrc_mode": 2,
         "nrc_terminate_after": 2}
    s, _ = ctx.render(cam, p)
    ctx.sync()
    st = ctx.render_stats()
    m = _np(s) / 4
    _say(f"  cached paths {st['nrc_queries']}, max |pixel - 1| {np.abs(m - 1).max():.2e}")
    assert st["nrc_queries"] > 1000
    assert np.allclose(m, 1.0, atol=2e-5)


def _cache_image_parity(ctx, orc, sc, name, res, spp, depth, W, extra=None):
    from paper_2406_09733_amd import scenes
    cam = dict(scenes.camera(name), width=res[0], height=res[1])
    box = tuple(np.concatenate([sc["mean"].min(0) - 0.1, sc["mean"].max(0) + 0.1]).tolist())
    p = {"spp": spp, "max_depth": depth, "seed": 6, "nrc_mode": 2, "nrc_terminate_after": 2, "nrc_box": box}
    if extra:
        p.update(extra)
    S = orc.Scene(sc)
    ref2, _, _ = S.render(cam, dict(p, nrc_weights=W))
    ref3, _, _ = S.render(cam, dict(p, nrc_mode=3))
    ctx.build_bvh(sc)
    ctx.nrc_set_weights(W.astype(np.float32))
    g, _ = ctx.render(cam, p)
    ctx.sync()
    g = _np(g).reshape(-1, 3).astype(np.float64)
    cache = np.abs(ref2 - ref3)
    tol = 1e-4 * np.abs(ref2) + 0.05 * cache + 1e-5
    bad = float((np.abs(g - ref2) > tol).mean())
    _say(f"  {name}: cache share of the image {cache.sum() / max(np.abs(ref2).sum(), 1e-30):.3f}; "
         f"pixels beyond tolerance {bad:.4f}; mean gpu {g.mean():.6f} oracle {ref2.mean():.6f}")
    return bad, g, ref2


def test_render_cache_parity_tiny(ctx, torch, orc):
    from paper_2406_09733_amd import scenes
    _say("nrc render parity tiny_random 96x96 2 spp depth 6")
    W = weights(11, scale=0.5)
    bad, g, ref = _cache_image_parity(ctx, orc, scenes.tiny_random(), "tiny_random", (96, 96), 2, 6, W)
    assert bad < 0.01


def test_render_cache_parity_mixed(ctx, torch, orc):
    from paper_2406_09733_amd import scenes
    _say("nrc render parity mixed_100k 64x64 2 spp depth 8")
    W = weights(12, scale=0.5)
    bad, g, ref = _cache_image_parity(ctx, orc, scenes.mixed_100k(), "mixed_100k", (64, 64), 2, 8, W)
    assert bad < 0.01


def test_render_training_records_parity(ctx, torch, orc):
    from paper_2406_09733_amd import scenes
    _say("nrc render: training records and targets vs oracle (tiny_random 32x32, depth 4)")
    sc = scenes.tiny_random(seed=3, n_emit=50)
    sc["scale"] *= 2
    box = (-0.5, -0.5, -0.5, 1.5, 1.5, 1.5)
    import paper_2406_09733_amd as P
    c2 = P.Context(0)  # fresh context: the training-path probability starts at its initial value
    c2.build_bvh(sc)
    W = weights(13, scale=0.5)
    c2.nrc_set_weights(W.astype(np.float32))
    cam = dict(scenes.camera("tiny_random"), width=32, height=32)
    R = 65536
    p = {"spp": 1, "max_depth": 4, "seed": 9, "nrc_mode": 1, "nrc_terminate_after": 2, "nrc_train_records": R,
         "nrc_box": box}
    img, _ = c2.render(cam, p)
    rec, tgt = c2.nrc_records(R)
    c2.sync()
    rec32 = _np(rec)
    pix_gpu = np.ascontiguousarray(rec32[:, 19]).view(np.int32)
    rec, tgt = rec32.astype(np.float64), _np(tgt).astype(np.float64)
    frac = min(1.0, R / (8.0 * 32 * 32))  # the training-path probability's start
    assert frac == 1.0
    # every path is a training path: the image is the plain tracer's, bit for bit
    ctx.build_bvh(sc)
    plain, _ = ctx.render(cam, {"spp": 1, "max_depth": 4, "seed": 9})
    ctx.sync()
    assert np.array_equal(_np(img), _np(plain))
    S = orc.Scene(sc)
    po = dict(p, nrc_train_frac=frac, nrc_weights=W)
    order = np.lexsort((rec[:, 23], pix_gpu))
    rec, tgt, pix_gpu = rec[order], tgt[order], pix_gpu[order]
    ok = total = 0
    for pix in range(32 * 32):
        L, r = S.path_records(cam, po, pix, 0)
        sel = pix_gpu == pix
        total += 1
        g, gt = rec[sel], tgt[sel]
        if len(g) != len(r):
            continue
        if len(r) == 0:
            ok += 1
            continue
        t_ref = np.where(r[:, 16:19] > 0, (L[None, :] - r[:, 20:23]) / np.where(r[:, 16:19] > 0, r[:, 16:19], 1), 0)
        t_ref = np.maximum(t_ref, 0)
        good = (np.allclose(g[:, :16], r[:, :16], rtol=1e-4, atol=2e-5) and
                np.allclose(g[:, 16:19], r[:, 16:19], rtol=1e-4, atol=1e-7) and
                np.allclose(g[:, 20:23], r[:, 20:23], rtol=1e-4, atol=1e-6) and
                np.array_equal(g[:, 23], r[:, 23]) and
                np.allclose(gt, t_ref, rtol=1e-3, atol=1e-4 * max(1.0, np.abs(t_ref).max())))
        ok += int(good)
    _say(f"  {len(rec)} records; pixels whose records match the oracle: {ok}/{total}")
    assert len(rec) > 500
    assert ok >= 0.99 * total
    c2.close()


def test_cached_renders_repeat_exactly(torch):
    # Training records are appended by atomics in whatever order the waves
    # reach them; the renderer orders a chunk's records by path before it
    # trains, so runs from the same weights give the same records, weights and
    # images bit for bit -- also with a bounded path pool and no tail kernel
    # (other append orders), when a chunk attempts more records than it
    # trains on (the cap then keeps the same paths), and in a context that
    # trained before and was given the initial weights again.  The room at 64x36, depth
    # 30: a closed scene, so a training path records many vertices and the
    # first call attempts more than the cap.
    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes
    _say("cached renders repeat exactly (room 64x36, depth 30, 3 calls of 4 spp, 2048 records per step)")
    sc = scenes.room_5p5m()
    cam = dict(scenes.camera("room_5p5m"), width=64, height=36)
    rng = np.random.default_rng(1)
    w0 = (0.1 * rng.uniform(-1, 1, P.nrc_num_params())).astype(np.float32)
    cap = 2048
    p = {"max_depth": 30, "seed": 4, "spp": 4, "nrc_mode": 1, "nrc_terminate_after": 2, "nrc_train_records": cap,
         "nrc_train_steps": 4}

    def run(pool, tail, again=False):
        ctx = P.Context(0)
        ctx.build_bvh(sc)
        ctx.set_path_pool(pool)
        ctx.set_tail_paths(tail)
        for _ in range(2 if again else 1):
            # setting the weights again restarts the training state (Adam,
            # radiance unit, training-path probability)
            ctx.nrc_set_weights(w0)
            imgs, att = [], []
            for k in range(3):
                s, _ = ctx.render(cam, dict(p, sample_offset=4 * k))
                att.append(int(ctx.render_stats()["nrc_records"]))
                imgs.append(_np(s).copy())
        rec, tgt = ctx.nrc_records(cap)
        out = imgs, att, _np(ctx.nrc_get_weights()).copy(), _np(rec).copy(), _np(tgt).copy()
        ctx.close()
        return out

    a = run(0, 65536)
    b = run(0, 65536, again=True)
    c = run(64 * 36, 0)
    _say(f"  records attempted per call: {a[1]} (cap {cap}); kept in the last: {len(a[3])}")
    assert a[1] == b[1] == c[1]
    # the first call attempts more than it trains on; the weights after the
    # third call carry what its cap kept
    assert a[1][0] > cap and len(a[3]) == min(a[1][-1], cap)
    for other in (b, c):
        for x, y in zip(a[0], other[0]):
            assert np.array_equal(x, y)
        assert np.array_equal(a[2], other[2])
        assert np.array_equal(a[3], other[3]) and np.array_equal(a[4], other[4])
    assert not np.array_equal(a[2], w0)  # the training moved the weights


def test_trained_cache_gains_over_untrained_and_termination(torch):
    # On the room at 160x90 (its configuration's depth 12, exposure 1): a
    # cache trained online on the tracer's own records (2048 spp of training,
    # 16 Adam steps on 262,144 records per chunk) leaves a smaller error against a converged plain
    # reference than the same network untrained and than ending paths after two
    # scattering events with nothing added, at equal spp (1024) and on the same
    # random numbers (identical path prefixes: the images differ only in what
    # the cache adds).  Error = the bias, estimated over pixels whose reference
    # is below 0.9: mean (t - r)^2 minus the variance of t (from its per-pixel
    # sums of squares) minus the variance of the reference r (from its two
    # halves), which leaves mean (E t - E r)^2.  The clamped RMSE at exposure 1
    # with the reference's noise removed (the benchmark's criterion) is
    # reported beside it.
    import paper_2406_09733_amd as P
    from paper_2406_09733_amd import scenes
    _say("trained cache vs untrained cache vs termination on the room at 160x90")
    sc = scenes.room_5p5m()
    ctx = P.Context(0)
    ctx.build_bvh(sc)
    cam = dict(scenes.camera("room_5p5m"), width=160, height=90)
    base = {"max_depth": 12, "seed": 2}
    halves = []
    for h in range(2):
        s, _ = ctx.render(cam, dict(base, spp=4096, sample_offset=4096 * h))
        halves.append(s.double() / 4096)
    ctx.sync()
    a, b = halves
    r = 0.5 * (a + b)
    var_r = (a - b) ** 2 / 4
    rng = np.random.default_rng(0)
    from oracle import NRC_LAYERS
    w0 = np.concatenate([rng.uniform(-1, 1, o * i) * np.sqrt(6.0 / i) for (o, i) in NRC_LAYERS]).astype(np.float32)
    nrc = {"nrc_terminate_after": 2, "nrc_train_records": 262144, "nrc_lr": 1e-2, "nrc_train_steps": 16,
           "nrc_target_clamp": 0.0}
    ctx.nrc_set_weights(w0)
    for k in range(16):
        ctx.render(cam, dict(base, seed=5, spp=128, sample_offset=128 * k, want_sumsq=False, nrc_mode=1, **nrc))
    ctx.sync()
    spp = 1024
    test = {"seed": 9, "spp": spp}

    def err(mode, weights=None):
        if weights is not None:
            ctx.nrc_set_weights(weights)
        # (nrc_radiance_scale 0 keeps the radiance unit the training set;
        # setting weights clears it to 1)
        s, s2 = ctx.render(cam, dict(base, **test, nrc_mode=mode, **nrc))
        ctx.sync()
        t = s.double() / spp
        var_t = torch.clamp(s2.double() / spp - t * t, min=0) / spp
        live = r.max(dim=2, keepdim=True).values.expand_as(r) < 0.9
        bias2 = float(((t - r) ** 2 - var_t - var_r)[live].mean())
        mse_c = float(((t.clamp(0, 1) - r.clamp(0, 1)) ** 2).mean())
        noise_c = float(((a.clamp(0, 1) - b.clamp(0, 1)) ** 2 / 4).mean())
        return bias2, max(0.0, mse_c - noise_c) ** 0.5

    e_trained = err(2)  # the weights and unit the training left
    e_term = err(3)
    e_untrained = err(2, w0)
    _say(f"  bias^2 (unsaturated pixels): trained {e_trained[0]:.3e}, untrained {e_untrained[0]:.3e}, "
         f"termination {e_term[0]:.3e}")
    _say(f"  clamped RMSE at exposure 1, reference noise removed: trained {e_trained[1]:.4f}, "
         f"untrained {e_untrained[1]:.4f}, termination {e_term[1]:.4f}")
    assert e_trained[0] < e_term[0] and e_trained[0] < e_untrained[0]
    assert e_trained[1] < e_term[1] and e_trained[1] < e_untrained[1]
    ctx.close()
