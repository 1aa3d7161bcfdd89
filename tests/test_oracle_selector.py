"""Pins of the selector oracle (oracle/selector.py) against definitions that do
not go through its own code: torch's bfloat16 conversion, direct-loop
convolution, closed forms and central differences."""
import numpy as np
import pytest

from oracle import selector as S


def test_num_params():
    assert S.NUM_PARAMS == 151076


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-30, 50), rng.normal(0, 1e30, 50),
                        [1 + 2 ** -8, 1 + 2 ** -7 + 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0, 3.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), ref)
    # ties to even, by hand
    assert S.bf16(1 + 2 ** -8) == 1.0
    assert S.bf16(1 + 2 ** -7 + 2 ** -8) == 1 + 2 ** -6


def _direct_conv(x, Wt, b):
    """3x3 stride-2 pad-1 convolution by nested loops, weights [out][ky][kx][in]."""
    n, H, W, C = x.shape
    O = Wt.shape[0]
    out = np.zeros((n, H // 2, W // 2, O))
    for i in range(n):
        for oy in range(H // 2):
            for ox in range(W // 2):
                for o in range(O):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            y, xx = 2 * oy - 1 + ky, 2 * ox - 1 + kx
                            if 0 <= y < H and 0 <= xx < W:
                                s += float(np.dot(Wt[o, ky, kx], x[i, y, xx]))
                    out[i, oy, ox, o] = s
    return out


def test_im2col_product_is_the_direct_convolution():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 6, 8, 3))
    Wt = rng.normal(size=(5, 3, 3, 3))
    b = rng.normal(size=5)
    got = (S.im2col(x) @ Wt.reshape(5, 27).T + b).reshape(2, 3, 4, 5)
    np.testing.assert_allclose(got, _direct_conv(x, Wt, b), rtol=1e-12, atol=1e-12)


def test_col2im_is_the_adjoint_of_im2col():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 6, 3))
    d = rng.normal(size=(2 * 4 * 3, 27))
    # <im2col(x), d> == <x, col2im(d)>
    assert np.isclose((S.im2col(x) * d).sum(), (x * S.col2im(d, x.shape)).sum(), rtol=1e-12)


def test_forward_layers_against_direct_loops():
    """First conv layer of the network equals the direct loop (rounding off)."""
    rng = np.random.default_rng(3)
    theta = S.init_params(3)
    P = S.unpack(theta)
    feat = rng.normal(size=(1, 64, 64, 4))
    norm = np.array([0.1, 0.2, 0.3, 0.4, 1.5, 2.0, 0.5, 1.0])
    _, cache = S.forward(theta, norm, feat, bf16_round=False)
    x0 = (feat - norm[:4]) / norm[4:]
    # direct loop on a corner patch: the outputs at (oy, ox) < 3 read input rows/cols < 6
    ref = _direct_conv(x0[:, :6, :6], P["W1"], P["b1"])
    got = cache["pre1"].reshape(1, 32, 32, 32)[:, :3, :3]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_flatten_order_is_y_x_c():
    """W4 row 0 reading only element (y=1, x=2, c=3) of the 8x8x32 map returns it."""
    rng = np.random.default_rng(4)
    theta = S.init_params(4)
    P = {k: v.copy() for k, v in S.unpack(theta).items()}
    P["W4"][:] = 0.0
    P["W4"][0, (1 * 8 + 2) * 32 + 3] = 1.0
    P["b4"][:] = 0.0
    P["W5"][:] = 0.0
    P["W5"][0, 0] = 1.0
    P["b5"][:] = 0.0
    feat = rng.normal(size=(2, 64, 64, 4))
    logits, cache = S.forward(S.pack(P), np.array([0, 0, 0, 0, 1, 1, 1, 1.0]), feat, bf16_round=False)
    conv3 = np.maximum(cache["pre3"], 0).reshape(2, 8, 8, 32)
    np.testing.assert_allclose(logits[:, 0], conv3[:, 1, 2, 3], rtol=1e-12)


def test_softmax_ce_closed_form_at_equal_logits():
    z = np.zeros((3, 4))
    y = np.array([0, 2, 3])
    cw = np.array([1.0, 2.0, 3.0, 4.0])
    loss, d = S.softmax_ce(z, y, cw)
    assert np.isclose(loss, np.log(4))
    W = cw[y].sum()
    ref = (cw[y] / W)[:, None] * (0.25 - np.eye(4)[y])
    np.testing.assert_allclose(d, ref, rtol=1e-14)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(5)
    theta = S.init_params(5) * 0.5
    theta += rng.normal(0, 0.01, theta.size)  # nonzero biases
    norm = np.array([4.0, 3.0, 1.0, 0.5, 1.0, 2.0, 1.0, 1.0])
    feat = norm[:4] + rng.normal(size=(3, 64, 64, 4))
    labels = np.array([1, 0, 3])
    cw = np.array([1.0, 0.5, 2.0, 1.5])
    _, g = S.loss_and_grad(theta, norm, feat, labels, cw, bf16_round=False)
    # every bias, and a sample of weights of every layer
    idx, off = [], 0
    for name, shape in S.LAYOUT:
        n = int(np.prod(shape))
        if name.startswith("b"):
            idx += list(range(off, off + n))[:8]
        else:
            idx += list(off + rng.choice(n, 6, replace=False))
        off += n
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp, _ = S.loss_and_grad(tp, norm, feat, labels, cw, bf16_round=False)
        lm, _ = S.loss_and_grad(tm, norm, feat, labels, cw, bf16_round=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(6)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, wd = 1e-3, 0.01
    out, m, v = S.adamw(th, np.zeros(50), np.zeros(50), g, 1, lr, wd)
    # first step: bias-corrected m = g, v = g^2
    np.testing.assert_allclose(out, th * (1 - lr * wd) - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_closed_forms():
    p = 5
    const = np.full((50, 60), 700, np.uint16)
    prev = np.full((50, 60), 690, np.uint16)
    f = S.features(const, prev, pitch=p, level=1)
    R, nb = S.band_rows(50, 60, p, 1)
    assert f.shape == (nb, 64, 64, 4)
    nz = f[..., 0] != 0
    assert nz.any()
    np.testing.assert_allclose(f[..., 0][nz], np.log1p(700))
    np.testing.assert_allclose(f[..., 1][nz], 0.0)
    np.testing.assert_allclose(f[..., 2][nz], 0.0)
    np.testing.assert_allclose(f[..., 3][nz], np.log1p(10))
    # ramp along x: |x - x(left lens)| = p on every pixel past the first lens column
    ramp = np.tile(np.arange(60, dtype=np.uint16) * 3, (50, 1))
    f = S.features(ramp, None, pitch=p, level=1)
    last = f[0, :, -1, 2]  # last column of cells: x >= p everywhere
    np.testing.assert_allclose(last[last != 0], np.log1p(3 * p))
    assert np.all(f[..., 3] == 0)


def test_features_brute_force_cell():
    rng = np.random.default_rng(7)
    p, h, w = 15, 225, 225
    x = rng.integers(0, 2000, size=(h, w)).astype(np.uint16)
    pv = rng.integers(0, 2000, size=(h, w)).astype(np.uint16)
    f = S.features(x, pv, p, 1)
    R, nb = S.band_rows(h, w, p, 1)
    b = nb - 1
    rb = min(R, h // p - b * R)
    hb = rb * p
    for ci, cj in [(0, 0), (63, 63), (17, 40)]:
        ya, yb = b * R * p + ci * hb // 64, b * R * p + (ci + 1) * hb // 64
        xa, xb = cj * w // 64, (cj + 1) * w // 64
        vals, dxs, dts = [], [], []
        for yy in range(ya, yb):
            for xx in range(xa, xb):
                v = int(x[yy, xx])
                vals.append(v)
                dxs.append(abs(v - int(x[yy, xx - p])) if xx >= p else 0)
                dts.append(abs(v - int(pv[yy, xx])))
        if not vals:
            assert np.all(f[b, ci, cj] == 0)
            continue
        m = np.mean(vals)
        np.testing.assert_allclose(f[b, ci, cj], [np.log1p(m), np.log1p(np.var(vals)), np.log1p(np.mean(dxs)),
                                                  np.log1p(np.mean(dts))], rtol=1e-12)


def test_predict_threshold_and_mask():
    z = np.array([[0.0, 5.0, 0.0, 9.0], [1.0, 1.0, 1.0, 1.0], [2.0, 0.0, 0.0, 0.0]])
    # mask 0x7 hides id 3
    out = S.predict(z, 0x7, 0.9)
    assert out[0] == 1
    assert out[1] == 0xFF
    p2 = np.exp(2) / (np.exp(2) + 2)
    assert S.predict(z, 0x7, p2 - 1e-12)[2] == 0
    assert S.predict(z, 0x7, p2 + 1e-9)[2] == 0xFF
    assert list(S.predict(z, 0x7, 0.0)) == [1, 0, 0]  # ties go to the lowest id
