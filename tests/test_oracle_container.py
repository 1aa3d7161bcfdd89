"""Pins for the oracle's container and whole-frame round trip (paper Sec. 2.1.4:
an 8-bit predictor id is stored with the coded data; Sec. 3 / Supp. Fig. S2:
decompression restores the frame exactly).  The bzip2 layer is decoded by the
stock bz2 module, independently of the oracle."""
import bz2
import ctypes

import numpy as np
import pytest


def decode_with_bz2(orc, blob, prev=None):
    info = orc.peek(blob)
    h, w, pitch, level = info["h"], info["w"], info["pitch"], info["level"]
    frame = np.zeros((h, w), np.uint16)
    pos = orc.header_bytes(info["n_bands"])
    for b in range(info["n_bands"]):
        ln = int(info["band_len"][b])
        raw = bz2.decompress(blob[pos:pos + ln])
        pos += ln
        arr = np.frombuffer(raw, np.uint16)
        orc.unarrange(arr, (h, w), b, int(info["ids"][b]), prev=prev, pitch=pitch, level=level, into=frame)
    return frame, info


def test_c1_roundtrip_and_header(orc):
    from paper_2310_09467_amd import synth

    f = synth.config1_frame()
    blob, choice = orc.compress(f, pitch=15, level=1, cand_mask=0x3)
    assert blob[:4] == b"PCBZ" and blob[4] == 1 and blob[5] == 1
    back, info = decode_with_bz2(orc, blob)
    np.testing.assert_array_equal(back, f)
    assert (info["h"], info["w"], info["pitch"], info["level"], info["n_bands"]) == (225, 225, 15, 1, 2)
    assert list(info["ids"]) == list(choice)
    assert orc.header_bytes(2) + int(info["band_len"].sum()) == len(blob)


def test_payload_is_arranged_band_bytes(orc):
    from paper_2310_09467_amd import synth

    f = synth.config1_frame()
    blob, choice = orc.compress(f, pitch=15, level=1, cand_mask=0x3)
    payload = bz2.decompress(blob[orc.header_bytes(2):])
    want = b"".join(orc.to_bytes(orc.arrange(f, b, int(choice[b]), level=1)).tobytes() for b in range(2))
    assert payload == want


def test_choice_matches_judge(orc):
    from paper_2310_09467_amd import synth

    f = synth.config1_frame()
    c_judge, _, _ = orc.judge(f, pitch=15, level=1, cand_mask=0x7)
    _, choice = orc.compress(f, pitch=15, level=1, cand_mask=0x7)
    assert list(choice) == list(c_judge)


@pytest.mark.parametrize("seed", [1, 2])
def test_forced_choices_stay_lossless(orc, seed):
    rng = np.random.default_rng(seed)
    from paper_2310_09467_amd import synth

    f, pos = synth.beads_frame(450, 300, 40, 300.0, seed)
    prev, _ = synth.beads_frame(450, 300, 40, 300.0, seed + 100, positions=pos)
    _, nb = orc.plan(450, 300, 15, 1)
    forced = rng.integers(0, 4, nb).astype(np.uint8)
    blob, choice = orc.compress(f, prev=prev, pitch=15, level=1, cand_mask=0xF, forced_choice=forced)
    assert list(choice) == list(forced)
    assert blob[18] == (1 if (forced == 3).any() else 0)
    back, _ = decode_with_bz2(orc, blob, prev=prev)
    np.testing.assert_array_equal(back, f)


def test_adversarial_roundtrip(orc):
    from paper_2310_09467_amd import synth

    for name, f in synth.adversarial_frames(180, 180).items():
        blob, _ = orc.compress(f, pitch=15, level=1, cand_mask=0x7)
        back, _ = decode_with_bz2(orc, blob)
        np.testing.assert_array_equal(back, f, err_msg=name)


def test_enospc_reports_required_size(orc):
    from paper_2310_09467_amd import synth

    f = np.ascontiguousarray(synth.config1_frame())
    blob, _ = orc.compress(f, pitch=15, level=1, cand_mask=0x3)
    p = orc.params(225, 225, 15, 1, 0x3)
    out = np.zeros(100, np.uint8)
    ln = np.zeros(1, np.uintp)
    st = orc.lib().orc_compress(ctypes.byref(p), f.ctypes.data_as(ctypes.c_void_p), None, None,
                                out.ctypes.data_as(ctypes.c_void_p), out.size, ln.ctypes.data_as(ctypes.c_void_p),
                                None)
    assert st == orc.ENOSPC and int(ln[0]) == len(blob)


def test_peek_rejects_damage(orc):
    from paper_2310_09467_amd import synth

    blob, _ = orc.compress(synth.config1_frame(), pitch=15, level=1, cand_mask=0x3)
    for bad in (b"XCBZ" + blob[4:], blob[:-1], blob[:10]):
        with pytest.raises(orc.OracleError) as e:
            orc.peek(bad)
        assert e.value.code == orc.EDATA


def test_oracle_decompress_roundtrip(orc):
    """The oracle's decoder (stock bz2 per band, then the inverse
    arrangement) gives back the frame for every arrangement id."""
    from paper_2310_09467_amd import synth

    f, pos = synth.beads_frame(90, 60, 20, 300.0, 5)
    prev, _ = synth.beads_frame(90, 60, 20, 300.0, 6, positions=pos)
    nb = orc.plan(90, 60, 15, 1)[1]
    for cid in range(4):
        blob, _ = orc.compress(f, prev, 15, 1, 0xF, forced_choice=np.full(nb, cid, np.uint8))
        np.testing.assert_array_equal(orc.decompress(blob, prev), f)

