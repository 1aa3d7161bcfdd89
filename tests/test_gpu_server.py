"""GPU tests of the serving loop: every container equals the one-frame call
with the same previous frame, also when admission has to wait for memory,
with several workers and with the learned selector."""
import numpy as np
import pytest

from paper_2310_09467_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_09467_amd import pcbz

    return torch, pcbz, pcbz.Context(0)


def _frames():
    """Two cameras x two shapes x four time steps (beads drifting)."""
    out = {}
    for cam in range(2):
        for shape in ((450, 300), (225, 225)):
            _, pos = synth.beads_frame(*shape, 40, 200.0 + 100 * cam, seed=31 + cam)
            seq = []
            for k in range(4):
                f, _ = synth.beads_frame(*shape, 40, 200.0 + 100 * cam, seed=1000 * cam + 10 * k + shape[0],
                                         positions=pos)
                seq.append(f)
                pos = pos + np.array([0.03, -0.02, 0.0])
            out[(cam, shape)] = seq
    return out


def _run(pcbz, srv, frames, mask=0xF, level=1):
    order = []
    for k in range(4):
        for (cam, shape), seq in sorted(frames.items()):
            order.append((cam, shape, k))
    for tag, (cam, shape, k) in enumerate(order):
        srv.submit(frames[(cam, shape)][k], tag, cam, 15, level, mask)
    res = {}
    while len(res) < len(order):
        for r in srv.poll(64, 1000):
            res[r["tag"]] = r
    return order, res


def _check(ctx, frames, order, res, mask=0xF, level=1):
    tag_of = {o: t for t, o in enumerate(order)}
    for tag, (cam, shape, k) in enumerate(order):
        r = res[tag]
        assert r["status"] == 0
        f = frames[(cam, shape)][k]
        if k == 0 or not (mask & 8):
            assert r["prev_tag"] is None
            prev = None
        else:
            assert r["prev_tag"] == tag_of[(cam, shape, k - 1)]
            prev = frames[(cam, shape)][k - 1]
        m = mask if prev is not None else mask & 7
        assert r["data"] == ctx.compress(f, prev, 15, level, m), (tag, cam, shape, k)


@pytest.mark.parametrize("workers", [1, 3])
def test_server_equals_alone(env, workers):
    torch, pcbz, ctx = env
    frames = _frames()
    srv = pcbz.Server(0, 1 << 30, workers)
    try:
        order, res = _run(pcbz, srv, frames)
        st = srv.stats()
        assert st["completed"] == len(order) and st["pending"] == 0 and st["admitted"] == 0
    finally:
        srv.close()
    _check(ctx, frames, order, res)


def test_server_admission_waits_for_memory(env):
    """A budget whose pool holds only a few frames: submissions queue on the
    host, all finish, bytes unchanged."""
    torch, pcbz, ctx = env
    frames = _frames()
    srv = pcbz.Server(0, 64 << 20, 1)
    try:
        order, res = _run(pcbz, srv, frames)
        st = srv.stats()
        assert st["pool_peak"] <= st["pool_bytes"]
        assert st["completed"] == len(order)
    finally:
        srv.close()
    _check(ctx, frames, order, res)


def test_server_with_selector(env):
    torch, pcbz, ctx = env
    from oracle import selector as OS

    frames = _frames()
    theta = OS.init_params(9).astype(np.float32)
    norm = np.array([5.0, 8.0, 2.0, 0.5, 1.5, 3.0, 1.0, 1.0], np.float32)
    sel = pcbz.Selector(ctx, theta, norm)
    srv = pcbz.Server(0, 1 << 30, 2, 0, sel, 0.7)
    try:
        order, res = _run(pcbz, srv, frames)
    finally:
        srv.close()
    ctx.set_selector(sel, 0.7)
    try:
        _check(ctx, frames, order, res)
    finally:
        ctx.set_selector(None)


def test_server_rejects_frames_that_never_fit(env):
    torch, pcbz, ctx = env
    srv = pcbz.Server(0, 64 << 20, 1)
    try:
        big = np.zeros((2040, 2040), np.uint16)
        with pytest.raises(pcbz.PcbzError):
            srv.submit(big, 0, 0, 15, 9, 0x7)
    finally:
        srv.close()
