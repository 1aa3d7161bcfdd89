"""Pins for the oracle's entropy judgement (paper Sec. 2.1.2, Eq. 1, Fig. 2c):
brute-force rotation matrices, closed-form entropies and invariants."""
import itertools
import json
import math
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def brute_lastcol(x):
    """Build every rotation, stably sort on the first byte only, take last bytes."""
    x = list(x)
    n = len(x)
    rots = [x[i:] + x[:i] for i in range(n)]
    order = sorted(range(n), key=lambda i: rots[i][0])  # Python's sort is stable
    return [rots[i][-1] for i in order]


def float_entropy(T):
    T = np.asarray(T, np.int64)
    q = T[:-1] * 256 + T[1:]
    _, cnt = np.unique(q, return_counts=True)
    p = cnt / cnt.sum()
    return float(-(p * np.log2(p)).sum())


def test_lastcol_all_ternary_strings(orc):
    for n in range(1, 9):
        for s in itertools.product(range(3), repeat=n):
            x = np.array(s, np.uint8)
            assert list(orc.order1_lastcol(x)) == brute_lastcol(s), s


@pytest.mark.parametrize("alpha,n,seed", [(2, 4096, 1), (16, 3001, 2), (256, 4096, 3), (3, 17, 4)])
def test_lastcol_random(orc, alpha, n, seed):
    x = np.random.default_rng(seed).integers(0, alpha, n).astype(np.uint8)
    assert list(orc.order1_lastcol(x)) == brute_lastcol(x.tolist())


def test_entropy_alternating_bytes(orc):
    g = GOLD["entropy_alternating_0100"]
    x = np.array(g["x"], np.uint8)
    T = orc.order1_lastcol(x)
    assert list(T) == g["T"]
    S = orc.band_score(x)
    assert abs(orc.entropy_bits(S, 8) - g["H_bits"]) < 1e-6
    # the 16-bit frame 0x0100 is exactly these bytes
    fr = np.full((15, 15), 0x0100, np.uint16)
    assert list(orc.to_bytes(fr)[:8]) == g["x"]


def test_entropy_constant_is_zero(orc):
    for n in (2, 3, 1000):
        x = np.full(n, 7, np.uint8)
        S = orc.band_score(x)
        assert S == orc.tq(n - 1)
        assert abs(orc.entropy_bits(S, n)) < 1e-9


def test_tq_powers_of_two(orc):
    assert orc.tq(0) == 0 and orc.tq(1) == 0
    for k in range(1, 21):
        assert orc.tq(2**k) == k * 2**k * 2**20


@pytest.mark.parametrize("k,c", [(1, 5), (2, 3), (7, 11), (256, 1), (4096, 9), (65536, 2)])
def test_equal_bins_give_log2k(orc, k, c):
    P = np.zeros(65536, np.uint32)
    idx = np.random.default_rng(k).choice(65536, k, replace=False)
    P[idx] = c
    S = orc.score(P)
    H = orc.entropy_bits(S, k * c + 1)
    assert abs(H - math.log2(k)) <= 2.0**-20 * max(1.0, math.log2(k)) + 1e-12


def test_distinct_pairs(orc):
    T = np.arange(256, dtype=np.uint8)
    P = orc.pair_hist(T)
    assert P.sum() == 255 and P.max() == 1
    assert P[0x0001] == 1 and P[0xFEFF] == 1 and P[0x0100] == 0


@pytest.mark.parametrize("alpha,seed", [(2, 1), (5, 2), (40, 3), (256, 4)])
def test_entropy_matches_float_and_bounds(orc, alpha, seed):
    x = np.random.default_rng(seed).integers(0, alpha, 5000).astype(np.uint8)
    S = orc.band_score(x)
    H = orc.entropy_bits(S, x.size)
    Hf = float_entropy(brute_lastcol(x.tolist()))
    assert abs(H - Hf) < 1e-6
    assert 0.0 <= H <= min(16.0, math.log2(x.size - 1)) + 1e-9


def test_judge_tie_goes_to_lowest_id(orc):
    f = np.full((225, 225), 0x0101, np.uint16)
    choice, S, _ = orc.judge(f, pitch=15, level=1, cand_mask=0x3)
    assert list(choice) == [0, 0]
    assert S[0, 0] == S[0, 1]


def test_judge_picks_view_dx_on_lens_constant_frame(orc):
    # value depends only on the in-lens position: every view is constant
    rng = np.random.default_rng(8)
    tile = rng.integers(0, 65536, size=(15, 15), dtype=np.uint16)
    f = np.tile(tile, (15, 15))
    choice, S, H = orc.judge(f, pitch=15, level=1, cand_mask=0x7)
    assert list(choice) == [2, 2]
    assert np.isnan(H[0, 3]) and S[0, 3] == orc.INT64_MIN


def test_judge_matches_float_argmin(orc):
    rng = np.random.default_rng(9)
    for trial in range(6):
        f = (rng.integers(0, 3, size=(30, 45)) * 3 + np.tile(rng.integers(0, 4, (15, 15)), (2, 3))).astype(np.uint16)
        prev = f ^ rng.integers(0, 2, size=f.shape).astype(np.uint16)
        choice, S, H = orc.judge(f, prev=prev, pitch=15, level=1, cand_mask=0xF)
        for b in range(choice.size):
            Hf = []
            for cid in range(4):
                x = orc.to_bytes(orc.arrange(f, b, cid, prev=prev, pitch=15, level=1))
                Hf.append(float_entropy(brute_lastcol(x.tolist())))
                assert abs(Hf[-1] - H[b, cid]) < 1e-6
            best = min(Hf)
            assert Hf[choice[b]] - best < 1e-9
            assert choice[b] == min(i for i in range(4) if Hf[i] - best < 1e-9) or \
                abs(Hf[choice[b]] - best) < 1e-5


def test_judge_needs_prev(orc):
    f = np.zeros((225, 225), np.uint16)
    with pytest.raises(orc.OracleError) as e:
        orc.judge(f, pitch=15, level=1, cand_mask=0xF)
    assert e.value.code == orc.ENEEDPREV
