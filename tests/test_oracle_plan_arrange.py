"""Pins for the oracle's band plan and arrangements (paper Sec. 2.1.1, Fig. 1a,
Fig. 3a; the sub-aperture view of a lenslet image is the strided slice
frame[u::p, v::p])."""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_block_limit(orc):
    assert orc.block_limit(1) == 99981
    assert orc.block_limit(9) == 899981


@pytest.mark.parametrize("case", GOLD["band_plan"]["cases"])
def test_band_plan_closed_form(orc, case):
    R, nb = orc.plan(case["h"], case["w"], case["pitch"], case["level"])
    assert R == case["R"]
    assert nb == len(case["band_bytes"])
    got = []
    for b in range(nb):
        _, rows = orc.band_geometry(case["h"], case["w"], case["pitch"], case["level"], b)
        got.append(2 * rows * case["pitch"] * case["w"])
    assert got == case["band_bytes"]
    assert sum(got) == 2 * case["h"] * case["w"]


@pytest.mark.parametrize("h,w,pitch,level,mask", [
    (224, 225, 15, 9, 7), (225, 224, 15, 9, 7), (225, 225, 15, 0, 7), (225, 225, 15, 10, 7),
    (225, 225, 15, 9, 0), (225, 225, 15, 9, 1 << 16), (0, 225, 15, 9, 7), (225, 225, 0, 9, 7)])
def test_plan_rejects(orc, h, w, pitch, level, mask):
    with pytest.raises(orc.OracleError) as e:
        orc.plan(h, w, pitch, level, mask)
    assert e.value.code == orc.EINVAL


def test_wide_frame_forces_one_lens_row(orc):
    # 2*p*W above the block limit: R clamps to 1 lens row per band.
    R, nb = orc.plan(45, 3345, 15, 1)
    assert (R, nb) == (1, 3)


def _band(frame, orc, b, pitch=15, level=9):
    y0, rows = orc.band_geometry(frame.shape[0], frame.shape[1], pitch, level, b)
    return frame[y0 * pitch:(y0 + rows) * pitch], rows


@pytest.mark.parametrize("shape,pitch,level", [((225, 225), 15, 1), ((450, 300), 15, 1), ((60, 84), 6, 1)])
def test_view_equals_subaperture_slices(orc, shape, pitch, level):
    rng = np.random.default_rng(3)
    f = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    _, nb = orc.plan(*shape, pitch, level)
    for b in range(nb):
        band, rows = _band(f, orc, b, pitch, level)
        got = orc.arrange(f, b, orc.VIEW, pitch=pitch, level=level)
        nt = shape[1] // pitch
        views = got.reshape(pitch, pitch, rows, nt)
        for u in range(pitch):
            for v in range(pitch):
                np.testing.assert_array_equal(views[u, v], band[u::pitch, v::pitch])


def test_raster_is_band(orc):
    rng = np.random.default_rng(4)
    f = rng.integers(0, 65536, size=(225, 225), dtype=np.uint16)
    for b in range(2):
        band, _ = _band(f, orc, b, 15, 1)
        np.testing.assert_array_equal(orc.arrange(f, b, orc.RASTER, level=1), band.ravel())


def test_view_dx_constant(orc):
    f = np.full((225, 225), 1234, np.uint16)
    out = orc.arrange(f, 0, orc.VIEW_DX, level=1).reshape(225, 14, 15)
    assert np.all(out[:, 0, 0] == 1234)
    out[:, 0, 0] = 0
    assert not out.any()


def test_view_dx_ramp_along_lens_columns(orc):
    p = 15
    y, x = np.mgrid[0:225, 0:225]
    base = (1000 + 37 * (x % p) + 91 * (y % p)).astype(np.int64)
    f = ((base + 5 * (x // p)) % 65536).astype(np.uint16)
    out = orc.arrange(f, 0, orc.VIEW_DX, level=1).reshape(p * p, 14, 15)
    assert np.all(out[:, :, 1:] == 5)
    assert np.all(out[:, 1:, 0] == 0)
    uv = np.arange(p * p)
    np.testing.assert_array_equal(out[:, 0, 0], (1000 + 37 * (uv % p) + 91 * (uv // p)).astype(np.uint16))


def test_view_dx_wraps(orc):
    p = 3
    f = np.zeros((3, 6), np.uint16)
    f[0, 3] = 65535  # view (0,0): lens t=0 value 0, t=1 value 65535
    out = orc.arrange(f, 0, orc.VIEW_DX, pitch=p, level=1).reshape(9, 1, 2)
    assert out[0, 0, 1] == 65535
    g = np.zeros((3, 6), np.uint16)
    g[0, 0] = 65535
    out = orc.arrange(g, 0, orc.VIEW_DX, pitch=p, level=1).reshape(9, 1, 2)
    assert out[0, 0, 0] == 65535 and out[0, 0, 1] == 1


def test_view_dx_matches_numpy_differences(orc):
    rng = np.random.default_rng(5)
    f = rng.integers(0, 65536, size=(450, 225), dtype=np.uint16)
    view = orc.arrange(f, 0, orc.VIEW, level=1).reshape(225, 14, 15).astype(np.int64)
    want = view.copy()
    want[:, :, 1:] = view[:, :, 1:] - view[:, :, :-1]
    want[:, 1:, 0] = view[:, 1:, 0] - view[:, :-1, 0]
    got = orc.arrange(f, 0, orc.VIEW_DX, level=1).reshape(225, 14, 15)
    np.testing.assert_array_equal(got, (want % 65536).astype(np.uint16))


def test_view_dt(orc):
    rng = np.random.default_rng(6)
    f = rng.integers(0, 65536, size=(225, 225), dtype=np.uint16)
    assert not orc.arrange(f, 0, orc.VIEW_DT, prev=f, level=1).any()
    prev = rng.integers(0, 65536, size=(225, 225), dtype=np.uint16)
    d = ((f.astype(np.int64) - prev) % 65536).astype(np.uint16)
    np.testing.assert_array_equal(orc.arrange(f, 0, orc.VIEW_DT, prev=prev, level=1),
                                  orc.arrange(d, 0, orc.VIEW, level=1))
    with pytest.raises(orc.OracleError) as e:
        orc.arrange(f, 0, orc.VIEW_DT, level=1)
    assert e.value.code == orc.ENEEDPREV


@pytest.mark.parametrize("cid", [0, 1, 2, 3])
def test_inverse_roundtrip(orc, cid):
    rng = np.random.default_rng(7 + cid)
    shape, pitch, level = (90, 75), 15, 1
    f = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    prev = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    _, nb = orc.plan(*shape, pitch, level)
    back = np.zeros(shape, np.uint16)
    for b in range(nb):
        a = orc.arrange(f, b, cid, prev=prev, pitch=pitch, level=level)
        orc.unarrange(a, shape, b, cid, prev=prev, pitch=pitch, level=level, into=back)
    np.testing.assert_array_equal(back, f)


def test_to_bytes_little_endian(orc):
    assert list(orc.to_bytes(np.array([0x1234, 0xABCD], np.uint16))) == [0x34, 0x12, 0xCD, 0xAB]
