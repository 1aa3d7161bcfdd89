"""The predictor family (arrangement ids 4..15) on the GPU against the
oracle: judgement over all sixteen ids (choices and every fixed-point score
exact), containers byte for byte with judged and forced ids, and GPU
decompression of those containers back to the frame."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [((450, 300), 15, 9), ((90, 3345), 15, 2), ((64, 56), 8, 1), ((35, 21), 7, 9), ((30, 30), 15, 9),
         ((600, 90), 15, 9)]


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_09467_amd import pcbz

    c = pcbz.Context(0)
    yield c
    c.close()


def _frame(shape, pitch, seed):
    from paper_2310_09467_amd import synth

    f, pos = synth.beads_frame(shape[0], shape[1], 60, 300.0, seed, pitch=pitch)
    prev, _ = synth.beads_frame(shape[0], shape[1], 60, 300.0, seed + 100, pitch=pitch, positions=pos)
    # smooth structure too, so that the predictors have something to win on
    yy, xx = np.mgrid[0:shape[0], 0:shape[1]]
    f = (f.astype(np.int64) + (yy * 3 + xx * 2) % 400).clip(0, 65535).astype(np.uint16)
    return f, prev


@pytest.mark.parametrize("shape,pitch,level", CASES)
def test_judge_all_sixteen(ctx, orc, shape, pitch, level):
    f, prev = _frame(shape, pitch, 51)
    for mask, pv in ((0xFFFF, prev), (0xFFF7, None), (0xFFF0, None)):
        print("judge", shape, pitch, level, hex(mask), flush=True)
        c, e, s = ctx.judge(f, pv, pitch, level, mask)
        oc, oS, oH = orc.judge(f, pv, pitch, level, mask)
        np.testing.assert_array_equal(c.cpu().numpy(), oc)
        np.testing.assert_array_equal(s.cpu().numpy(), oS)
        ge = e.cpu().numpy()
        fin = ~np.isnan(oH)
        assert np.array_equal(np.isnan(ge), ~fin)
        np.testing.assert_allclose(ge[fin], oH[fin], rtol=0, atol=1e-9)


@pytest.mark.parametrize("shape,pitch,level", CASES)
def test_containers_and_decode(ctx, orc, shape, pitch, level):
    from paper_2310_09467_amd import pcbz

    f, prev = _frame(shape, pitch, 61)
    nb = orc.plan(shape[0], shape[1], pitch, level)[1]
    print("judged", shape, pitch, level, flush=True)
    blob, ch = ctx.compress(f, prev, pitch, level, 0xFFFF, return_choice=True)
    ob, oc = orc.compress(f, prev, pitch, level, 0xFFFF)
    np.testing.assert_array_equal(ch, oc)
    assert blob == ob
    np.testing.assert_array_equal(pcbz.as_uint16(ctx.decompress(blob, prev=prev)), f)
    for cid in range(4, 16):
        print("forced", cid, flush=True)
        ids = np.full(nb, cid, np.uint8)
        blob = ctx.compress(f, None, pitch, level, 0x7, forced=ids)
        assert blob == orc.compress(f, None, pitch, level, 0x7, forced_choice=ids)[0]
        np.testing.assert_array_equal(pcbz.as_uint16(ctx.decompress(blob)), f)


def test_mixed_ids_in_one_batch(ctx, orc):
    """Frames of several shapes with random ids over all sixteen, coded in one
    batch and decoded in one call."""
    from paper_2310_09467_amd import pcbz

    rng = np.random.default_rng(77)
    frames, prevs, params, forced = [], [], [], []
    for k, (shape, pitch, level) in enumerate(CASES):
        f, prev = _frame(shape, pitch, 71 + k)
        nb = orc.plan(shape[0], shape[1], pitch, level)[1]
        frames.append(f)
        prevs.append(prev)
        params.append((pitch, level, 0xFFFF))
        forced.append(rng.integers(0, 16, nb).astype(np.uint8))
    blobs = ctx.compress_batch(frames, prevs, params, forced=forced)
    for f, pv, (pitch, level, m), fc, b in zip(frames, prevs, params, forced, blobs):
        assert b == orc.compress(f, pv, pitch, level, m, forced_choice=fc)[0]
    outs = ctx.decompress_batch(blobs, prevs)
    for f, o in zip(frames, outs):
        np.testing.assert_array_equal(pcbz.as_uint16(o), f)
