"""GPU parity of the learned arrangement selector against oracle/selector.py:
the matrix-core GEMM, the band features, the network's logits and gradients,
one AdamW step, and the compress path with the selector (lossless, equal to
compressing with the predicted ids forced, equal to exhaustive judging when
every band falls back)."""
import numpy as np
import pytest

from oracle import selector as OS
from paper_2310_09467_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_09467_amd import pcbz

    return torch, pcbz, pcbz.Context(0)


def _bf16_bits(torch, x):
    """float64 array (already bf16-representable) -> device int16 tensor of its bf16 bits."""
    a = np.asarray(x, np.float32).view(np.uint32) >> 16
    return torch.from_numpy(a.astype(np.uint16).view(np.int16)).cuda()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 16), (17, 33, 48), (100, 70, 300), (64, 64, 16),
                                   (5, 130, 2049), (257, 3, 77)])
def test_gemm_bf16_lane_layout(env, M, N, K):
    torch, pcbz, _ = env
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    a = OS.bf16(rng.normal(size=(M, K)))
    b = OS.bf16(rng.normal(size=(K, N)))
    c = pcbz.gemm_bf16(_bf16_bits(torch, a), _bf16_bits(torch, b)).cpu().numpy()
    ref = a @ b
    # FP32 accumulation of K exact bf16 products
    tol = 2e-6 * np.sqrt(K) * (np.abs(a) @ np.abs(b)) + 1e-30
    assert np.all(np.abs(c - ref) <= tol), np.max(np.abs(c - ref) / tol)


def _frames():
    f1 = synth.config1_frame(11)
    f0 = synth.config1_frame(12)
    big, _ = synth.beads_frame(450, 300, 40, 300.0, seed=13)
    return [(f1, None, 1), (f1, f0, 1), (big, None, 2)]


def test_features_match_oracle(env):
    torch, pcbz, ctx = env
    for frame, prev, level in _frames():
        got = ctx.features(frame, prev, 15, level, 0xF if prev is not None else 0x7).cpu().numpy()
        ref = OS.features(frame, prev, 15, level)
        assert got.shape == ref.shape
        # FP64 sums of integers on both sides; only the final FP32 rounding may differ
        np.testing.assert_allclose(got, ref, rtol=2e-7, atol=1e-7)


def _setup(env, seed=0, n=6):
    torch, pcbz, ctx = env
    rng = np.random.default_rng(seed)
    theta = OS.init_params(seed)
    theta[OS.NUM_PARAMS - 4:] = rng.normal(0, 0.1, 4)
    norm = np.array([5.0, 8.0, 2.0, 0.5, 1.5, 3.0, 1.0, 1.0], np.float32)
    feats = []
    for frame, prev, level in _frames():
        feats.append(OS.features(frame, prev, 15, level))
    feat = np.concatenate(feats)[:n].astype(np.float32)
    sel = pcbz.Selector(ctx, theta.astype(np.float32), norm)
    return torch, pcbz, ctx, sel, theta, norm.astype(np.float64), feat


def test_forward_batch_invariant(env):
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 2)
    f = torch.from_numpy(feat).cuda()
    whole = sel.forward(f).cpu().numpy()
    for i in range(len(feat)):
        one = sel.forward(f[i:i + 1]).cpu().numpy()
        np.testing.assert_array_equal(one[0], whole[i])


U32 = 2.0 ** -24  # unit roundoff of FP32


def _acc_bound(a, b, k, extra=0.0):
    """Worst-case error of an FP32 sum of k exact products (bf16 x bf16 fits
    FP32's significand) plus one more addition, in any order:
    (k + 1) u sum |terms| (Higham's gamma bound, u = 2^-24, k u << 1)."""
    return (k + 1) * U32 * 1.0001 * ((np.abs(a) @ np.abs(b)) + np.abs(extra)) + 1e-30


def _bf16_halfulp(v):
    """Half a bfloat16 unit in the last place at |v| (8 significand bits)."""
    m = np.maximum(np.abs(v), 2.0 ** -126)
    return np.ldexp(1.0, np.floor(np.log2(m)).astype(int) - 8)


def _rounded_ok(got, exact, bound):
    """got (a bf16 value) is the bf16 rounding of some FP32 value within
    `bound` of the exact value: |got - exact| <= half an ulp + bound."""
    slack = _bf16_halfulp(np.maximum(np.abs(exact) + bound, np.abs(got))) + bound * 1.0001
    return np.abs(got - exact) <= slack


def _check(name, ok, got, ref):
    bad = ~ok
    assert not bad.any(), (name, int(bad.sum()), got[bad][:5], ref[bad][:5])


def _layers(env, seed, labels, cw):
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, seed)
    n = len(feat)
    g, loss = sel.gradients(torch.from_numpy(feat).cuda(), torch.from_numpy(labels).cuda(), cw)
    T = {nm: sel.inspect(nm, n).astype(np.float64) for nm, _, _ in pcbz.Selector.INSPECT}
    return theta, norm, feat, g.cpu().numpy().astype(np.float64), loss, T


def test_forward_layers_match_oracle_elementwise(env):
    """Every layer of the training forward pass, element by element: each
    layer's FP32 pre-activation against the oracle's product of the GPU's own
    bf16 layer input (so that rounding flips upstream do not propagate), within
    the worst-case FP32 accumulation bound; each bf16 output equals the
    oracle's bf16 rounding of the GPU's FP32 value; the normalised input is
    the bf16 rounding of the exact (f - mean) / std within FP32 arithmetic."""
    labels = np.array([0, 1, 2, 1, 0, 2])
    theta, norm, feat, _, _, T = _layers(env, 1, labels, None)
    n = len(feat)
    P = OS.unpack(theta)
    x0 = (feat.astype(np.float64) - norm[:4]) / norm[4:]
    _check("x0", _rounded_ok(T["x0"], x0, 2 * U32 * (np.abs(x0) + np.abs(norm[:4] / norm[4:]))), T["x0"], x0)
    x = T["x0"]
    for i, (H, C) in enumerate(((64, 4), (32, 32), (16, 32)), start=1):
        col = OS.im2col(x)
        Wk = OS.bf16(P[f"W{i}"].reshape(32, 9 * C))
        ref = col @ Wk.T + P[f"b{i}"]
        pre = T[f"pre{i}"].reshape(ref.shape)
        _check(f"pre{i}", np.abs(pre - ref) <= _acc_bound(col, Wk.T, 9 * C, P[f"b{i}"]), pre, ref)
        nxt = T[f"x{i}"].reshape(ref.shape)
        np.testing.assert_array_equal(nxt, OS.bf16(np.maximum(pre.astype(np.float32), 0.0)))
        x = T[f"x{i}"].reshape(n, H // 2, H // 2, 32)
    x3 = T["x3"]
    W4 = OS.bf16(P["W4"])
    ref4 = x3 @ W4.T + P["b4"]
    _check("pre4", np.abs(T["pre4"] - ref4) <= _acc_bound(x3, W4.T, 2048, P["b4"]), T["pre4"], ref4)
    np.testing.assert_array_equal(T["x4"], OS.bf16(np.maximum(T["pre4"].astype(np.float32), 0.0)))
    W5 = OS.bf16(P["W5"])
    ref5 = T["x4"] @ W5.T + P["b5"]
    _check("logits", np.abs(T["logits"] - ref5) <= _acc_bound(T["x4"], W5.T, 64, P["b5"]), T["logits"], ref5)


def test_backward_layers_match_oracle_elementwise(env):
    """Every gradient of the backward pass, element by element, from the GPU's
    own layer inputs and upstream bf16 gradients: dloss/dlogits against the
    oracle's softmax cross-entropy of the GPU logits; each weight and bias
    gradient against the oracle's product within the worst-case FP32
    accumulation bound; each bf16 upstream gradient against the oracle's
    masked product (ReLU mask from the GPU's pre-activations) within half a
    bf16 ulp plus that bound, and exactly zero where the mask is off."""
    labels = np.array([0, 1, 2, 1, 0, 2])
    cw = [1.0, 2.0, 0.5, 1.0]
    theta, norm, feat, g, loss, T = _layers(env, 3, labels, cw)
    n = len(feat)
    P = OS.unpack(theta)
    G = OS.unpack(g)
    ref_loss, dlog = OS.softmax_ce(T["logits"], labels, cw)
    assert abs(loss - ref_loss) <= 1e-6 * abs(ref_loss) + 1e-7, (loss, ref_loss)
    wscale = (np.asarray(cw)[labels] / np.asarray(cw)[labels].sum())[:, None]
    _check("dlogits", np.abs(T["dlogits"] - dlog) <= 32 * U32 * wscale, T["dlogits"], dlog)
    np.testing.assert_array_equal(T["g5"], OS.bf16(T["dlogits"].astype(np.float32)))

    def wgrad(name, gup, xin):
        ref = gup.T @ xin
        got = G[name].reshape(ref.shape)
        _check(name, np.abs(got - ref) <= _acc_bound(gup.T, xin, gup.shape[0]), got, ref)

    def bgrad(name, gup):
        ref = gup.sum(0)
        _check(name, np.abs(G[name] - ref) <= (gup.shape[0] + 1) * U32 * np.abs(gup).sum(0) + 1e-30, G[name], ref)

    def upstream(name, gup, W, pre, shape=None, k=None):
        dx = gup @ W
        bound = _acc_bound(gup, W, k or gup.shape[1])
        if shape is not None:  # conv input gradient: col2im adds up to four products per pixel
            absum = OS.col2im(np.abs(dx), shape).reshape(pre.shape)
            dx = OS.col2im(dx, shape).reshape(pre.shape)
            bound = OS.col2im(bound, shape).reshape(pre.shape) * 1.0001 + 4 * U32 * absum
        got = T[name].reshape(pre.shape)
        on = pre > 0
        _check(name + " (masked)", got[~on] == 0.0, got[~on], dx[~on])
        _check(name, _rounded_ok(got[on], dx[on], bound[on]), got[on], dx[on])

    # FC5 and FC4
    wgrad("W5", T["g5"], T["x4"])
    bgrad("b5", T["g5"])
    upstream("g4", T["g5"], OS.bf16(P["W5"]), T["pre4"])
    wgrad("W4", T["g4"], T["x3"])
    bgrad("b4", T["g4"])
    # the conv3 output gradient, flattened (y, x, c) like x3
    upstream("g3", T["g4"], OS.bf16(P["W4"]), T["pre3"].reshape(n, 2048))
    # convolutions: gradient [n*Ho*Wo][32] against im2col of the layer input
    xs = {3: T["x2"], 2: T["x1"], 1: T["x0"]}
    for i, C in ((3, 32), (2, 32), (1, 4)):
        gi = T[f"g{i}"].reshape(-1, 32)
        col = OS.im2col(xs[i])
        wgrad(f"W{i}", gi, col)
        bgrad(f"b{i}", gi)
        if i > 1:
            Wk = OS.bf16(P[f"W{i}"].reshape(32, 9 * C))
            upstream(f"g{i - 1}", gi, Wk, T[f"pre{i - 1}"].reshape(-1, 32), shape=xs[i].shape, k=32)


def test_train_steps_match_oracle_adamw_elementwise(env):
    """Two AdamW steps, element by element: the oracle's AdamW applied to the
    GPU's parameters and the GPU's gradient at each step (the gradient itself
    is checked layer by layer above), with the moment decay rates the kernel
    holds (0.9 and 0.999 as FP32 numbers), within the FP32 arithmetic of the
    update: the bias corrections 1 - beta^t lose about u beta^t / (1 - beta^t)
    of relative precision to cancellation, the rest a few u."""
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 4)
    labels = np.array([2, 0, 1, 1, 0, 2][:len(feat)])
    lr, wd = 1e-3, 1e-2
    f = torch.from_numpy(feat).cuda()
    lab = torch.from_numpy(labels).cuda()
    th = theta.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in (1, 2):
        g, _ = sel.gradients(f, lab)
        g = g.cpu().numpy().astype(np.float64)
        sel.train_step(f, lab, None, lr, wd)
        got, _ = sel.params()
        b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
        ref, m, v = OS.adamw(th, m, v, g, step, lr, wd, b1, b2)
        upd = np.abs(th * (1 - lr * wd) - ref) / lr
        rel = 2 * U32 * (b1 ** step / (1 - b1 ** step) + b2 ** step / (1 - b2 ** step)) + 32 * U32
        tol = 4 * U32 * np.abs(th) + lr * upd * rel + 16 * U32 * lr
        _check(f"adamw step {step}", np.abs(got - ref) <= tol, got, ref)
        th = got.astype(np.float64)


def test_save_load_roundtrip(env, tmp_path):
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 5)
    path = tmp_path / "sel.bin"
    sel.save(path)
    s2 = pcbz.Selector.load_file(ctx, path)
    p1, n1 = sel.params()
    p2, n2 = s2.params()
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(n1, n2)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"PCBZSEL0" + bytes(64))
    with pytest.raises(pcbz.PcbzError):
        pcbz.Selector.load_file(ctx, bad)


def test_compress_with_selector(env, orc):
    """With the selector, containers equal the oracle's for the ids used: the
    exhaustive ones when every band falls back, the predicted ones (the
    oracle's thresholded choice of the GPU logits) when every band is trusted."""
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 6)
    frames = _frames()
    try:
        for frame, prev, level in frames:
            mask = 0xF if prev is not None else 0x7
            plain, _ = orc.compress(frame, prev, 15, level, mask)
            # every band falls back: exhaustive bytes
            ctx.set_selector(sel, 2.0)
            blob = ctx.compress(frame, prev, 15, level, mask)
            nb, judged = ctx.selector_stats()
            assert blob == plain and judged == nb > 0
            # every band trusted: the predicted ids, lossless
            ctx.set_selector(sel, 0.0)
            blob, ids = ctx.compress(frame, prev, 15, level, mask, return_choice=True)
            nb, judged = ctx.selector_stats()
            assert judged == 0
            logits = sel.forward(ctx.features(frame, prev, 15, level, mask)).cpu().numpy()
            pred = OS.predict(logits, mask, 0.0)
            np.testing.assert_array_equal(ids, pred)
            ctx.set_selector(None)
            assert blob == orc.compress(frame, prev, 15, level, mask, forced_choice=ids)[0]
            out = pcbz.as_uint16(ctx.decompress(blob, prev))
            np.testing.assert_array_equal(out, frame)
    finally:
        ctx.set_selector(None)


def test_selector_in_batch_graph(env, orc):
    """Captured batch replays with the selector equal the oracle's containers
    for the expected ids: the prediction where it is confident, the oracle's
    judgement elsewhere."""
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 7)
    frames = [f for f, _, _ in _frames()]
    params = [(15, 1, 0x7), (15, 1, 0x7), (15, 2, 0x7)]
    try:
        ctx.set_graphs(2)  # replay graphs even where an eager call would be faster
        first = ctx.compress_batch(frames, None, params, selector=sel, min_conf=0.6)
        for _ in range(3):
            again = ctx.compress_batch(frames, None, params, selector=sel, min_conf=0.6)
            assert again == first
        # the call's selector applies to that call only
        assert ctx.compress_batch(frames, None, params) == [orc.compress(f, None, p, lv, m)[0]
                                                           for f, (p, lv, m) in zip(frames, params)]
        ctx.set_graphs(1)
        for blob, frame, (p, lv, m) in zip(first, frames, params):
            # expected ids: the prediction where it is confident, the judgement elsewhere
            logits = sel.forward(ctx.features(frame, None, p, lv, m)).cpu().numpy()
            pred = OS.predict(logits, m, 0.6)
            judged = orc.judge(frame, None, p, lv, m)[0]
            ids = np.where(pred == 0xFF, judged, pred).astype(np.uint8)
            assert blob == orc.compress(frame, None, p, lv, m, forced_choice=ids)[0]
            out = pcbz.as_uint16(ctx.decompress(blob))
            np.testing.assert_array_equal(out, frame)
    finally:
        ctx.set_selector(None)


def test_fused_inference_matches_layer_path(env):
    """The fused inference kernel and the layer-by-layer training forward give
    the same logits (same k order on the matrix cores): the loss the training
    path reports equals the loss of the fused logits."""
    torch, pcbz, ctx, sel, theta, norm, feat = _setup(env, 8)
    labels = np.array([3, 1, 0, 2, 1, 0][:len(feat)])
    f = torch.from_numpy(feat).cuda()
    logits = sel.forward(f).cpu().numpy().astype(np.float64)
    _, loss = sel.gradients(f, torch.from_numpy(labels).cuda())
    ref, _ = OS.softmax_ce(logits, labels)
    assert abs(loss - ref) <= 2e-6 * abs(ref) + 1e-7, (loss, ref)


def test_trained_selector_gain(env):
    """The committed trained selector on the three 2040x2040 bead frames:
    most bands skip the judgement, the size regret stays within 0.5 %, and
    the output stays lossless."""
    import json
    import os

    torch, pcbz, ctx = env
    from paper_2310_09467_amd import cameras

    path = cameras.DEFAULT_SELECTOR
    tau = json.load(open(path.replace(".bin", "_report.json")))["picked"]["min_conf"]
    sel = pcbz.Selector.load_file(ctx, path)
    total_sel = total_exh = bands = judged = 0
    try:
        for peak in (20.0, 100.0, 1000.0):
            f = synth.config2_frame(peak)
            exh = ctx.compress(f, None, 15, 9, 0x7)
            ctx.set_selector(sel, tau)
            blob = ctx.compress(f, None, 15, 9, 0x7)
            nb, nj = ctx.selector_stats()
            ctx.set_selector(None)
            bands += nb
            judged += nj
            total_sel += len(blob)
            total_exh += len(exh)
            np.testing.assert_array_equal(pcbz.as_uint16(ctx.decompress(blob)), f)
    finally:
        ctx.set_selector(None)
    assert judged <= 0.1 * bands, (judged, bands)
    assert total_sel <= 1.005 * total_exh, (total_sel, total_exh)
    assert os.path.getsize(path) > 0
