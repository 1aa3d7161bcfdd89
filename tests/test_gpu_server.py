"""GPU tests of the serving loop: every container equals the oracle's for that
frame with the same previous frame, also when admission has to wait for
memory, with several workers and with the learned selector; frames that
cannot be coded are refused on their own."""
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


def _check(orc, frames, order, res, mask=0xF, level=1, expected_ids=None):
    """Every served container equals the oracle's container of that frame
    with the same previous frame and the ids the server chose; the ids are the
    oracle's judgement (or what expected_ids(frame, prev, mask) gives)."""
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
        ids = orc.peek(r["data"])["ids"]
        want = orc.judge(f, prev, 15, level, m)[0] if expected_ids is None else expected_ids(f, prev, m)
        np.testing.assert_array_equal(ids, want, err_msg=str((tag, cam, shape, k)))
        assert r["data"] == orc.compress(f, prev, 15, level, m, forced_choice=ids)[0], (tag, cam, shape, k)


@pytest.mark.parametrize("workers", [1, 3])
def test_server_equals_alone(env, orc, workers):
    torch, pcbz, ctx = env
    frames = _frames()
    srv = pcbz.Server(0, 1 << 30, workers)
    try:
        order, res = _run(pcbz, srv, frames)
        st = srv.stats()
        assert st["completed"] == len(order) and st["pending"] == 0 and st["admitted"] == 0
    finally:
        srv.close()
    _check(orc, frames, order, res)


def test_server_admission_waits_for_memory(env, orc):
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
    _check(orc, frames, order, res)


def test_server_with_selector(env, orc):
    torch, pcbz, ctx = env
    frames = _frames()
    theta = OS.init_params(9).astype(np.float32)
    norm = np.array([5.0, 8.0, 2.0, 0.5, 1.5, 3.0, 1.0, 1.0], np.float32)
    sel = pcbz.Selector(ctx, theta, norm)
    srv = pcbz.Server(0, 1 << 30, 2, 0, sel, 0.7)
    try:
        order, res = _run(pcbz, srv, frames)
    finally:
        srv.close()

    def expected(f, prev, m):
        # the selector's confident predictions (the oracle's thresholded
        # choice of the GPU logits), the oracle's judgement elsewhere
        logits = sel.forward(ctx.features(f, prev, 15, 1, m)).cpu().numpy()
        pred = OS.predict(logits, m, 0.7)
        return np.where(pred == 0xFF, orc.judge(f, prev, 15, 1, m)[0], pred).astype(np.uint8)

    _check(orc, frames, order, res, expected_ids=expected)


def test_server_per_frame_status(env, orc):
    """A camera's first frame whose only candidate is the temporal one is
    refused at submit (it has no previous frame); frames submitted around it
    complete and equal the oracle's."""
    torch, pcbz, ctx = env
    frames = _frames()
    a = frames[(0, (225, 225))]
    srv = pcbz.Server(0, 1 << 30, 1)
    try:
        srv.submit(a[0], 0, 0, 15, 1, 0x7)
        with pytest.raises(pcbz.PcbzError) as e:
            srv.submit(a[0], 1, 5, 15, 1, 0x8)
        assert e.value.code == pcbz.ENEEDPREV
        srv.submit(a[1], 2, 0, 15, 1, 0x8)  # camera 0 has a previous frame of this shape
        srv.submit(a[2], 3, 0, 15, 1, 0x3)
        res = {}
        while len(res) < 3:
            for r in srv.poll(8, 1000):
                res[r["tag"]] = r
    finally:
        srv.close()
    assert [res[t]["status"] for t in (0, 2, 3)] == [0, 0, 0]
    assert res[2]["prev_tag"] == 0
    assert res[0]["data"] == orc.compress(a[0], None, 15, 1, 0x7)[0]
    assert res[2]["data"] == orc.compress(a[1], a[0], 15, 1, 0x8)[0]
    assert res[3]["data"] == orc.compress(a[2], None, 15, 1, 0x3)[0]


def test_server_rejects_frames_that_never_fit(env):
    torch, pcbz, ctx = env
    srv = pcbz.Server(0, 64 << 20, 1)
    try:
        big = np.zeros((2040, 2040), np.uint16)
        with pytest.raises(pcbz.PcbzError):
            srv.submit(big, 0, 0, 15, 9, 0x7)
    finally:
        srv.close()
