"""CPU oracle of the learned arrangement selector (numpy, FP64).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests,
``__graft_entry__.smoke()`` and the CPU baseline leg of ``bench.py`` may use it;
the GPU library and its binding never do.

The selector is not part of the paper's method.  The paper scores every
candidate arrangement of every band with the 2D image entropy (Sec. 2.1.2,
Eq. 1) and lists a faster decision criterion as future work (Sec. 4); the
selector predicts the judgement's choice so that confident bands skip it.
Its definition (features, network, loss, optimiser) is the one the library's
C header states; this module writes it out plainly:

* features: per band, 64 x 64 cells, each giving log1p of the mean, the
  population variance, the mean absolute difference to the pixel one lens to
  the left and the mean absolute difference to the previous frame;
* network: three 3x3 stride-2 pad-1 convolutions (4->32->32->32 channels,
  ReLU), a 2048->64 fully connected layer with ReLU and a 64->4 output layer,
  channels-last tensors, weights [out][ky][kx][in];
* arithmetic: FP64, with every layer input (normalised features,
  activations, upstream gradients fed to a product) and every weight used in
  a product rounded to bfloat16 (round to nearest, ties to even), as the
  matrix-core kernels do; ``bf16=False`` turns the rounding off, which is how
  the finite-difference pins check the gradients;
* loss: class-weighted softmax cross-entropy, sum_i w[y_i] loss_i / sum_i w[y_i];
* optimiser: AdamW (beta1 0.9, beta2 0.999, eps 1e-8, decoupled decay).

Pins (tests/test_oracle_selector.py): bf16 rounding against torch's own
conversion; convolution against a direct loop; flatten order against a
one-hot readout; loss and gradient closed forms at equal logits; the whole
backward pass against central differences of the forward pass (rounding off);
AdamW's first step against its closed form; features against brute-force
loops and closed forms on constant and ramp frames.
"""
from __future__ import annotations

import numpy as np

N_CELLS = 64
CONV_CH = 32
HIDDEN = 64
N_CLASSES = 4

# parameter layout (name, shape) in storage order
LAYOUT = (
    ("W1", (32, 3, 3, 4)), ("b1", (32,)),
    ("W2", (32, 3, 3, 32)), ("b2", (32,)),
    ("W3", (32, 3, 3, 32)), ("b3", (32,)),
    ("W4", (64, 2048)), ("b4", (64,)),
    ("W5", (4, 64)), ("b5", (4,)),
)
NUM_PARAMS = int(sum(np.prod(s) for _, s in LAYOUT))


# ----------------------------------------------------------------- helpers
def bf16(x):
    """Round to the nearest bfloat16 value (ties to even); returns float64.

    The value is first taken to FP32 (as the kernels hold it), then its low
    16 bits are rounded away.  NaN stays NaN.
    """
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def unpack(theta):
    """Flat parameter vector -> dict of arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.size != NUM_PARAMS:
        raise ValueError(f"expected {NUM_PARAMS} parameters")
    out, off = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in LAYOUT])


def init_params(seed=0):
    """He-normal weights (fan-in), zero biases; FP32-representable values."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in LAYOUT:
        if name.startswith("b"):
            d[name] = np.zeros(shape)
        else:
            fan_in = int(np.prod(shape[1:]))
            d[name] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=shape)
    return pack(d).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------- features
def band_rows(h, w, pitch, level):
    """Lens rows per band and band count (the band plan of Sec. 2.1.3)."""
    lim = 100000 * level - 19
    R = max(1, lim // (2 * pitch * w))
    ns = h // pitch
    return R, (ns + R - 1) // R


def features(frame, prev=None, pitch=15, level=9):
    """Per-band features [n_bands, 64, 64, 4] (float64)."""
    x = np.asarray(frame, dtype=np.float64)
    pv = None if prev is None else np.asarray(prev, dtype=np.float64)
    h, w = x.shape
    R, nb = band_rows(h, w, pitch, level)
    ns = h // pitch
    out = np.zeros((nb, N_CELLS, N_CELLS, 4))
    # |x - x one lens to the left|, zero (excluded) in the first lens column
    dx = np.zeros_like(x)
    dx[:, pitch:] = np.abs(x[:, pitch:] - x[:, :-pitch])
    dt = np.zeros_like(x) if pv is None else np.abs(x - pv)
    for b in range(nb):
        rb = min(R, ns - b * R)
        y0, hb = b * R * pitch, rb * pitch
        for ci in range(N_CELLS):
            ya, yb = y0 + ci * hb // N_CELLS, y0 + (ci + 1) * hb // N_CELLS
            for cj in range(N_CELLS):
                xa, xb = cj * w // N_CELLS, (cj + 1) * w // N_CELLS
                cnt = (yb - ya) * (xb - xa)
                if cnt == 0:
                    continue
                cell = x[ya:yb, xa:xb]
                m = cell.sum() / cnt
                var = max(float((cell * cell).sum()) / cnt - m * m, 0.0)
                out[b, ci, cj, 0] = np.log1p(m)
                out[b, ci, cj, 1] = np.log1p(var)
                out[b, ci, cj, 2] = np.log1p(dx[ya:yb, xa:xb].sum() / cnt)
                out[b, ci, cj, 3] = np.log1p(dt[ya:yb, xa:xb].sum() / cnt)
    return out


# ----------------------------------------------------------------- network
def im2col(x):
    """x [n, H, W, C] -> columns [n*(H/2)*(W/2), 9*C] for a 3x3 stride-2 pad-1
    convolution; column index (ky*3 + kx)*C + c reads input pixel
    (2*oy - 1 + ky, 2*ox - 1 + kx), zero outside."""
    n, H, W, C = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((n, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    cols = np.empty((n, Ho, Wo, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx, :] = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
    return cols.reshape(n * Ho * Wo, 9 * C)


def col2im(dcol, shape):
    """Adjoint of im2col: adds each column entry back to the pixel it read."""
    n, H, W, C = shape
    Ho, Wo = H // 2, W // 2
    d = dcol.reshape(n, Ho, Wo, 3, 3, C)
    dxp = np.zeros((n, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += d[:, :, :, ky, kx, :]
    return dxp[:, 1:H + 1, 1:W + 1]


def forward(theta, norm, feat, bf16_round=True):
    """Logits [n, 4] and the activations the backward pass needs."""
    r = bf16 if bf16_round else _id
    P = unpack(theta)
    norm = np.asarray(norm, np.float64).reshape(8)
    f = np.asarray(feat, np.float64)
    n = f.shape[0]
    cache = {}
    x = r((f - norm[:4]) / norm[4:])
    for i, (H, C) in enumerate(((64, 4), (32, 32), (16, 32)), start=1):
        col = im2col(x)
        Wk = r(P[f"W{i}"].reshape(CONV_CH, 9 * C))
        pre = col @ Wk.T + P[f"b{i}"]
        cache[f"col{i}"], cache[f"pre{i}"], cache[f"shape{i}"] = col, pre, x.shape
        x = r(np.maximum(pre, 0.0)).reshape(n, H // 2, H // 2, CONV_CH)
    x3 = x.reshape(n, 2048)  # flatten (y, x, c)
    pre4 = x3 @ r(P["W4"]).T + P["b4"]
    x4 = r(np.maximum(pre4, 0.0))
    logits = x4 @ r(P["W5"]).T + P["b5"]
    cache.update(x3=x3, pre4=pre4, x4=x4)
    return logits, cache


def softmax_ce(logits, labels, class_w=None):
    """(loss, dloss/dlogits) of the class-weighted mean cross-entropy."""
    z = np.asarray(logits, np.float64)
    y = np.asarray(labels, np.int64)
    cw = np.ones(N_CLASSES) if class_w is None else np.asarray(class_w, np.float64)
    z = z - z.max(axis=1, keepdims=True)
    p = np.exp(z) / np.exp(z).sum(axis=1, keepdims=True)
    wi = cw[y]
    W = wi.sum()
    loss = float((wi * -np.log(p[np.arange(len(y)), y])).sum() / W)
    onehot = np.zeros_like(p)
    onehot[np.arange(len(y)), y] = 1.0
    return loss, (wi / W)[:, None] * (p - onehot)


def backward(theta, cache, dlogits, bf16_round=True):
    """Gradient of the loss w.r.t. the flat parameters, from dloss/dlogits."""
    r = bf16 if bf16_round else _id
    P = unpack(theta)
    G = {}
    g = r(dlogits)
    G["W5"] = g.T @ cache["x4"]
    G["b5"] = g.sum(0)
    dx = g @ r(P["W5"])
    g = r(np.where(cache["pre4"] > 0, dx, 0.0))
    G["W4"] = g.T @ cache["x3"]
    G["b4"] = g.sum(0)
    dx = g @ r(P["W4"])  # [n, 2048]: gradient of the flattened conv3 output
    for i, C in ((3, 32), (2, 32), (1, 4)):
        g = r(np.where(cache[f"pre{i}"] > 0, dx.reshape(cache[f"pre{i}"].shape), 0.0))
        G[f"W{i}"] = (g.T @ cache[f"col{i}"]).reshape(CONV_CH, 3, 3, C)
        G[f"b{i}"] = g.sum(0)
        if i > 1:
            dcol = g @ r(P[f"W{i}"].reshape(CONV_CH, 9 * C))
            dx = col2im(dcol, cache[f"shape{i}"])
    return pack(G)


def loss_and_grad(theta, norm, feat, labels, class_w=None, bf16_round=True):
    logits, cache = forward(theta, norm, feat, bf16_round)
    loss, dlog = softmax_ce(logits, labels, class_w)
    return loss, backward(theta, cache, dlog, bf16_round)


def adamw(theta, m, v, grad, step, lr, weight_decay, b1=0.9, b2=0.999, eps=1e-8):
    """One AdamW step (step counts from 1); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta = theta * (1 - lr * weight_decay) - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


def predict(logits, cand_mask, min_conf):
    """Per band: the most probable enabled id if its probability (softmax over
    the enabled ids) reaches min_conf, else 0xFF (left to the judgement)."""
    z = np.asarray(logits, np.float64)
    ids = [c for c in range(N_CLASSES) if (cand_mask >> c) & 1]
    out = np.full(len(z), 0xFF, np.uint8)
    if cand_mask >> N_CLASSES:  # ids beyond the network's classes: every band is judged
        return out
    for b, row in enumerate(z):
        best = max(ids, key=lambda c: (row[c], -c))
        p = 1.0 / np.exp(row[ids] - row[best]).sum()
        if p >= min_conf:
            out[b] = best
    return out
