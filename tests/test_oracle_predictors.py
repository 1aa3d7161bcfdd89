"""Pins of the oracle's predictor family (arrangement ids 4..15: the four
multi-neighbour lossless-JPEG functions over pixel, lens and phase-space
neighbours, Sec. 2.1.1, Fig. 1b, Fig. 3b/3c): hand-derived residuals on
constant frames and on planes (rising and falling, so that floor and
truncation differ), the boundary rule, the zigzag map, reductions at pitch 1,
and exact inversion."""
import numpy as np
import pytest


def zz(r):
    """0, -1, 1, -2, 2 ... -> 0, 1, 2, 3, 4 (hand table below pins it)"""
    return 2 * r if r >= 0 else -2 * r - 1


def test_zigzag_closed_forms(orc):
    assert [orc.zigzag16(v) for v in (0, 0xFFFF, 1, 0xFFFE, 2, 0x7FFF, 0x8000)] == [0, 1, 2, 3, 4, 65534, 65535]
    z = [orc.unzigzag16(v) for v in range(65536)]
    assert sorted(z) == list(range(65536))  # a bijection on 16 bits
    assert all(orc.zigzag16(orc.unzigzag16(v)) == v for v in range(0, 65536, 97))


def _residuals(orc, f, band, cid, pitch, level=9):
    r = orc.arrange(f, band, cid, None, pitch, level).astype(np.int64)
    return np.array([orc.unzigzag16(v) for v in r.ravel()], np.int64).astype(np.int16).reshape(-1, f.shape[1])


@pytest.mark.parametrize("cid", range(4, 16))
def test_constant_frame(orc, cid):
    p, c = 5, 1234
    f = np.full((30, 40), c, np.uint16)
    r = _residuals(orc, f, 0, cid, p)
    domain = (cid - 4) // 4
    yy, x = np.mgrid[0:30, 0:40]
    if domain == 0:
        first = (yy == 0) & (x == 0)
    elif domain == 1:
        first = (yy < p) & (x < p)
    else:
        first = (yy % p == 0) & (x < p)
    assert np.all(r[first] == c) and np.all(r[~first] == 0)


def _ceil_half(v):
    return -((-v) // 2)


@pytest.mark.parametrize("a,b", [(3, 5), (-3, -5), (7, -2), (0, 1)])
@pytest.mark.parametrize("cid", range(4, 16))
def test_plane(orc, cid, a, b):
    """X = c0 + a*yy + b*x.  Interior residuals (A, B, C one step back along
    each neighbour's axis; dA, dB their distances in value):
    A+B-C -> 0, A+floor((B-C)/2) -> ceil(dA/2), B+floor((A-C)/2) -> ceil(dB/2),
    floor((A+B)/2) -> ceil((dA+dB)/2).  Edges: only A -> dA, only B -> dB,
    neither -> X."""
    p, c0, H, W = 4, 20000, 24, 36
    yy, x = np.mgrid[0:H, 0:W]
    f = (c0 + a * yy + b * x).astype(np.uint16)
    domain, fn = (cid - 4) // 4, (cid - 4) % 4
    if domain == 0:
        dA, dB, hasA, hasB = b, a, x >= 1, yy >= 1
    elif domain == 1:
        dA, dB, hasA, hasB = b * p, a * p, x >= p, yy >= p
    else:
        dA, dB, hasA, hasB = b * p, a, x >= p, yy % p >= 1
    inner = [0, _ceil_half(dA), _ceil_half(dB), _ceil_half(dA + dB)][fn]
    want = np.where(hasA & hasB, inner, np.where(hasA, dA, np.where(hasB, dB, f.astype(np.int64))))
    r = _residuals(orc, f, 0, cid, p)
    np.testing.assert_array_equal(r, want.astype(np.int16))


def test_boundaries_are_band_local(orc):
    """With bands of 2 lens rows (level 1, wide frame), the first pixel row of
    the second band has no B neighbour in the pixel and lens domains."""
    p = 15
    w = 15 * 170  # a lens row is 2 * 15 * 2550 = 76500 bytes: one lens row per band at level 1
    f = np.full((30, w), 77, np.uint16)
    assert orc.plan(30, w, p, 1)[1] == 2
    for cid in (4, 8, 12):
        r = _residuals(orc, f, 1, cid, p, level=1)
        assert r[0, 0] == 77  # the band starts afresh


@pytest.mark.parametrize("fn", range(4))
def test_pitch_one_reductions(orc, fn):
    """At pitch 1 every lens is one pixel: the lens domain is the pixel
    domain, and the phase-space B (the pixel above inside the lens) never
    exists, so that domain predicts from the left pixel only."""
    rng = np.random.default_rng(fn)
    f = rng.integers(0, 65536, size=(12, 17), dtype=np.uint16)
    px = orc.arrange(f, 0, 4 + fn, None, 1, 9)
    ln = orc.arrange(f, 0, 8 + fn, None, 1, 9)
    ph = orc.arrange(f, 0, 12 + fn, None, 1, 9)
    np.testing.assert_array_equal(px, ln)
    left = np.zeros_like(f, dtype=np.int64)
    left[:, 1:] = f[:, :-1]
    want = [zz(int(np.int16(np.uint16((int(v) - int(l)) & 0xFFFF)))) for v, l in zip(f.ravel(), left.ravel())]
    np.testing.assert_array_equal(ph, np.array(want, np.uint16))


@pytest.mark.parametrize("cid", range(4, 16))
def test_inverse_roundtrip(orc, cid):
    rng = np.random.default_rng(cid)
    for shape, pitch, level in (((30, 45), 15, 1), ((64, 56), 8, 1), ((35, 21), 7, 9), ((9, 13), 1, 1)):
        f = rng.integers(0, 65536, size=shape, dtype=np.uint16)
        nb = orc.plan(shape[0], shape[1], pitch, level)[1]
        back = np.zeros_like(f)
        for b in range(nb):
            a = orc.arrange(f, b, cid, None, pitch, level)
            orc.unarrange(a, shape, b, cid, None, pitch, level, into=back)
        np.testing.assert_array_equal(back, f)


def test_container_roundtrip_with_predictors(orc):
    from paper_2310_09467_amd import synth

    f, _ = synth.beads_frame(90, 60, 20, 300.0, 5)
    nb = orc.plan(90, 60, 15, 1)[1]
    for cid in range(4, 16):
        blob, ch = orc.compress(f, None, 15, 1, 0xFFF7, forced_choice=np.full(nb, cid, np.uint8))
        assert list(orc.peek(blob)["ids"]) == [cid] * nb
        np.testing.assert_array_equal(orc.decompress(blob), f)


def test_judge_over_all_sixteen(orc):
    """The judgement over every arrangement id picks the float argmin of the
    brute-force pair entropies (rotation lists built explicitly)."""
    from test_oracle_judge import brute_lastcol, float_entropy

    rng = np.random.default_rng(21)
    for trial in range(2):
        base = np.add.outer(np.arange(30) * 3, np.arange(45) * 2) + np.tile(rng.integers(0, 5, (15, 15)), (2, 3))
        f = (base + rng.integers(0, 2, size=base.shape)).astype(np.uint16)
        prev = f ^ rng.integers(0, 2, size=f.shape).astype(np.uint16)
        choice, S, H = orc.judge(f, prev=prev, pitch=15, level=1, cand_mask=0xFFFF)
        for b in range(choice.size):
            Hf = []
            for cid in range(16):
                x = orc.to_bytes(orc.arrange(f, b, cid, prev=prev, pitch=15, level=1))
                Hf.append(float_entropy(brute_lastcol(x.tolist())))
                assert abs(Hf[-1] - H[b, cid]) < 1e-6
            best = min(Hf)
            assert Hf[choice[b]] - best < 1e-9
