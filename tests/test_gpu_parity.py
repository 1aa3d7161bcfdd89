"""GPU parity: the HIP library (called through its C ABI) against the CPU oracle.

Integer and byte work must be bit-exact: per-band choices, the fixed-point
entropy scores and every container byte.  The entropy in bits is a float
report; it must agree with the oracle's within 1e-9 bits."""
import bz2

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2310_09467_amd import pcbz

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = pcbz.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def check_judge(ctx, orc, f, prev=None, pitch=15, level=9, mask=0x7):
    c, e, s = ctx.judge(f, prev, pitch, level, mask)
    oc, oS, oH = orc.judge(f, prev, pitch, level, mask)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(s.cpu().numpy(), oS)
    ge = e.cpu().numpy()
    fin = ~np.isnan(oH)
    assert np.array_equal(np.isnan(ge), ~fin)
    np.testing.assert_allclose(ge[fin], oH[fin], rtol=0, atol=1e-9)


def check_compress(ctx, orc, f, prev=None, pitch=15, level=9, mask=0x7, forced=None):
    blob, ch = ctx.compress(f, prev, pitch, level, mask, forced=forced, return_choice=True)
    ob, oc = orc.compress(f, prev, pitch, level, mask, forced_choice=forced)
    np.testing.assert_array_equal(ch, oc)
    assert len(blob) == len(ob)
    assert blob == ob
    return blob


def test_c1_frame(ctx, orc):
    from paper_2310_09467_amd import synth

    _say("c1 225x225 level 1")
    f = synth.config1_frame()
    check_judge(ctx, orc, f, level=1, mask=0x3)
    blob = check_compress(ctx, orc, f, level=1, mask=0x3)
    hdr = orc.header_bytes(2)
    assert bz2.decompress(blob[hdr:]) == b"".join(
        orc.to_bytes(orc.arrange(f, b, int(blob[20 + 5 * b]), level=1)).tobytes() for b in range(2))


@pytest.mark.parametrize("name", ["zeros", "const_0101", "alt_0100", "index", "saturated", "uniform", "four_run",
                                  "period2", "period7"])
@pytest.mark.parametrize("level", [1, 9])
def test_adversarial(ctx, orc, name, level):
    from paper_2310_09467_amd import synth

    f = synth.adversarial_frames(180, 180)[name]
    _say("adversarial", name, level)
    check_judge(ctx, orc, f, level=level, mask=0x7)
    check_compress(ctx, orc, f, level=level, mask=0x7)


@pytest.mark.parametrize("shape,pitch,level", [((450, 300), 15, 1), ((465, 225), 15, 2), ((96, 120), 8, 1),
                                               ((63, 49), 7, 1), ((90, 3345), 15, 1), ((30, 30), 15, 9)])
def test_shapes_and_ragged_tails(ctx, orc, shape, pitch, level):
    from paper_2310_09467_amd import synth

    h, w = shape
    _say("shape", shape, pitch, level)
    f, pos = synth.beads_frame(h, w, 30, 300.0, 11, pitch=pitch)
    prev, _ = synth.beads_frame(h, w, 30, 300.0, 12, pitch=pitch, positions=pos)
    check_judge(ctx, orc, f, prev, pitch, level, 0xF)
    check_compress(ctx, orc, f, prev, pitch, level, 0xF)


def test_forced_choices_and_temporal(ctx, orc):
    from paper_2310_09467_amd import synth

    rng = np.random.default_rng(21)
    f, pos = synth.beads_frame(450, 300, 40, 300.0, 5)
    prev, _ = synth.beads_frame(450, 300, 40, 300.0, 6, positions=pos)
    nb = orc.plan(450, 300, 15, 1)[1]
    for trial in range(4):
        forced = rng.integers(0, 4, nb).astype(np.uint8)
        _say("forced", forced)
        check_compress(ctx, orc, f, prev, 15, 1, 0xF, forced=forced)


@pytest.mark.parametrize("peak", [20.0, 100.0, 1000.0])
def test_c2_full_frame(ctx, orc, peak):
    """2040x2040, level 9, three candidates: the full frame the benchmark times."""
    from paper_2310_09467_amd import synth

    _say("c2 peak", peak)
    f = synth.config2_frame(peak)
    check_judge(ctx, orc, f, level=9, mask=0x7)
    check_compress(ctx, orc, f, level=9, mask=0x7)


def test_roundtrip_through_library_decoder(ctx, orc):
    from paper_2310_09467_amd import pcbz, synth

    f, pos = synth.beads_frame(900, 600, 200, 500.0, 31)
    prev, _ = synth.beads_frame(900, 600, 200, 500.0, 32, positions=pos)
    for mask in (0x1, 0x3, 0x7, 0xF):
        blob = ctx.compress(f, prev, 15, 2, mask)
        back = pcbz.as_uint16(ctx.decompress(blob, prev=prev))
        np.testing.assert_array_equal(back, f)


def test_decoder_rejects_corruption(ctx, orc):
    from paper_2310_09467_amd import pcbz, synth

    f = synth.config1_frame()
    blob = bytearray(ctx.compress(f, None, 15, 1, 0x3))
    hdr = orc.header_bytes(2)
    bad = bytearray(blob)
    bad[hdr + 40] ^= 0x10
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.decompress(bytes(bad))
    assert e.value.code == pcbz.EDATA
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.decompress(bytes(blob[:-5]))
    assert e.value.code == pcbz.EDATA


def test_errors(ctx, orc):
    import ctypes

    import torch

    from paper_2310_09467_amd import pcbz, synth

    f = synth.config1_frame()
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.compress(f, None, 15, 1, 0xF)
    assert e.value.code == pcbz.ENEEDPREV
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.compress(f, None, 15, 1, 0x3, forced=[3, 0])
    assert e.value.code == pcbz.ENEEDPREV
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.compress(f, None, 15, 1, 0x3, forced=[16, 0])
    assert e.value.code == pcbz.EINVAL
    blob = ctx.compress(f, None, 15, 1, 0x3)
    dev = pcbz.to_device(f)
    out = torch.zeros(100, dtype=torch.uint8, device=dev.device)
    with pytest.raises(pcbz.PcbzError) as e:
        ctx.compress_into(dev, None, pcbz.Params(225, 225, 15, 1, 0x3), out)
    assert e.value.code == pcbz.ENOSPC and str(len(blob)) in str(e.value)
    assert not out.any().item()  # nothing written past a too-small buffer


def test_repeat_calls_are_deterministic(ctx, orc):
    from paper_2310_09467_amd import synth

    f = synth.config2_frame(100.0)
    a = ctx.compress(f, None, 15, 9, 0x7)
    small = synth.config1_frame()
    ctx.compress(small, None, 15, 1, 0x3)
    b = ctx.compress(f, None, 15, 9, 0x7)
    assert a == b


def test_known_shape_schedule(ctx, orc):
    """A shape seen before runs the round schedule its last read-back call
    needed, without read-backs; a frame that needs more rounds than that (or
    has a group too large for the in-group sort) is redone with read-backs.
    The adversarial frames share one shape and need very different rounds."""
    from paper_2310_09467_amd import synth

    frames = synth.adversarial_frames(150, 150)
    for rep in range(2):
        for name in sorted(frames):
            f = frames[name]
            _say("known shape", rep, name)
            assert ctx.compress(f, None, 15, 9, 0x7) == orc.compress(f, None, 15, 9, 0x7)[0]


def test_batch_equals_single_frames(ctx, orc):
    from paper_2310_09467_amd import synth

    frames = [synth.config1_frame()]
    params = [(15, 1, 0x3)]
    for i, (h, w) in enumerate([(450, 300), (300, 450), (225, 225)]):
        f, _ = synth.beads_frame(h, w, 50, 200.0 + 100 * i, 40 + i)
        frames.append(f)
        params.append((15, 9, 0x7))
    f2 = synth.config2_frame(100.0)
    frames.append(f2)
    params.append((15, 9, 0x7))
    _say("batch of", len(frames))
    blobs = ctx.compress_batch(frames, params=params)
    for f, (p, lv, m), blob in zip(frames, params, blobs):
        assert blob == ctx.compress(f, None, p, lv, m)
        assert blob == orc.compress(f, None, p, lv, m)[0]


def _periodic(h, w, period=50, seed=3):
    """Raster bytes repeating a random pattern: the band's single block keeps
    groups of (length / period) rotations in every doubling round."""
    rng = np.random.default_rng(seed)
    pat = rng.integers(0, 256, period, dtype=np.uint8)
    return np.resize(pat, 2 * h * w).view(np.uint16).reshape(h, w).copy()


@pytest.mark.parametrize("w,largest", [(330, 3960), (345, 4140)])
def test_group_sort_limit(ctx, orc, capfd, monkeypatch, w, largest):
    """Groups of 3960 rotations are sorted group by group in LDS, groups of
    4140 exceed the 4096 limit and take the radix sort; both are exact."""
    monkeypatch.setenv("PCBZ_DEBUG_BWT", "1")
    f = _periodic(300, w)
    nb = orc.plan(300, w, 15, 9)[1]
    _say("periodic 300 x", w)
    check_compress(ctx, orc, f, level=9, mask=0x7, forced=np.zeros(nb, np.uint8))
    err = capfd.readouterr().err
    assert f"largest group={largest}" in err


def test_many_blocks_one_frame(ctx, orc):
    """2040x2040 at level 1 (100 kB blocks): more than 64 blocks in one call,
    so the block lookups take their searched path instead of the per-lane
    table."""
    from paper_2310_09467_amd import synth

    f = synth.config2_frame(100.0)
    _say("c2 level 1")
    blob = check_compress(ctx, orc, f, level=1, mask=0x7)
    assert ctx.last_stats()["blocks"] > 64


def test_many_tiny_frames_in_one_batch(ctx, orc):
    """Eighty 30x30 frames in one call: blocks of about 1.8 kB, so a 4096-entry
    tile of every scan and sort spans several blocks."""
    from paper_2310_09467_amd import synth

    frames, params = [], []
    for i in range(80):
        f, _ = synth.beads_frame(30, 30, 3, 50.0 + 10 * i, 300 + i)
        frames.append(f)
        params.append((15, 9 if i % 2 else 1, 0x7))
    _say("batch of 80 tiny frames")
    blobs = ctx.compress_batch(frames, params=params)
    for f, (p, lv, m), blob in zip(frames, params, blobs):
        assert blob == orc.compress(f, None, p, lv, m)[0]
