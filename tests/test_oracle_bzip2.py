"""Pins for the oracle's bzip2 block coding (paper Sec. 2.1.3 uses bzip2; the
stream layout is the public bzip2 format).  Independent checks: brute-force
rotation sorting, inverse transforms, exhaustive optimal-code search, a
textbook Huffman, zlib's reflected CRC-32, and the stock decoders (Python's
bz2 module and the bzip2 command)."""
import bz2
import heapq
import itertools
import json
import os
import shutil
import subprocess
import zlib

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
_REV8 = np.array([int(f"{i:08b}"[::-1], 2) for i in range(256)], np.uint8)


def _rev32(v):
    return int(f"{v:032b}"[::-1], 2)


# ------------------------------------------------------------------ CRC
def test_crc_check_value(orc):
    g = GOLD["crc32_bzip2_check"]
    assert orc.crc32_bzip2(g["input"].encode()) == g["crc"]


def test_crc_equals_bit_reflected_zlib(orc):
    rng = np.random.default_rng(1)
    for n in (0, 1, 7, 1000, 65537):
        x = rng.integers(0, 256, n).astype(np.uint8)
        want = _rev32(zlib.crc32(_REV8[x].tobytes()) & 0xFFFFFFFF)
        assert orc.crc32_bzip2(x) == want


# ------------------------------------------------------------------ RLE1 and block cut
@pytest.mark.parametrize("case", GOLD["rle1_runs"]["cases"])
def test_rle1_runs(orc, case):
    raw = np.full(case["run"], 97, np.uint8)
    out, rs, os_ = orc.rle1_blocks(raw, level=9)
    assert list(out) == case["out"]
    assert list(rs) == [0] and list(os_) == [0]


def test_rle1_mixed_runs(orc):
    raw = np.frombuffer(b"abbbbbcccd" + b"e" * 300 + b"f", np.uint8)
    out, _, _ = orc.rle1_blocks(raw, level=9)
    want = b"abbbb\x01cccd" + b"eeee\xfb" + b"eeee\x29" + b"f"
    assert out.tobytes() == want


def test_four_run_cut(orc):
    g = GOLD["four_run_cut"]
    raw = np.frombuffer(b"aaaab" * (g["n"] // 5), np.uint8)
    out, rs, os_ = orc.rle1_blocks(raw, level=g["level"])
    assert list(rs) == g["raw_start"] and list(os_) == g["rle_start"]
    assert out.size == 6 * (g["n"] // 5)


def test_cut_respects_limit_and_pieces(orc):
    rng = np.random.default_rng(2)
    raw = np.repeat(rng.integers(0, 3, 4000).astype(np.uint8), rng.integers(1, 9, 4000))
    out, rs, os_ = orc.rle1_blocks(raw, limit=997)
    ends = list(os_[1:]) + [out.size]
    assert all(e - s <= 997 for s, e in zip(os_, ends))
    assert all(e - s >= 997 - 4 for s, e in zip(os_[:-1], ends[:-1]))  # a piece is at most 5 bytes


# ------------------------------------------------------------------ BWT
def brute_bwt(s):
    m = len(s)
    sa = sorted(range(m), key=lambda i: (s[i:] + s[:i], i))
    L = [s[(i - 1) % m] for i in sa]
    return sa, L, sa.index(0)


def ibwt(L, orig):
    L = np.asarray(L, np.uint8)
    order = np.argsort(L, kind="stable")
    out = np.empty(L.size, np.uint8)
    i = int(order[orig])
    for k in range(L.size):
        out[k] = L[i]
        i = int(order[i])
    return out


@pytest.mark.parametrize("case", GOLD["bwt_cyclic"]["cases"])
def test_bwt_golden(orc, case):
    sa, L, orig = orc.bwt(np.frombuffer(case["block"].encode(), np.uint8))
    assert list(sa) == case["sa"] and L.tobytes().decode() == case["L"] and orig == case["orig"]


def test_bwt_all_binary_strings(orc):
    for m in range(1, 13):
        for s in itertools.product(b"ab", repeat=m):
            sa, L, orig = orc.bwt(np.array(s, np.uint8))
            bsa, bL, borig = brute_bwt(list(s))
            assert list(sa) == bsa and list(L) == bL and orig == borig, bytes(s)


@pytest.mark.parametrize("alpha,m,seed", [(2, 2000, 1), (4, 1500, 2), (256, 2000, 3), (1, 64, 4), (3, 999, 5)])
def test_bwt_random(orc, alpha, m, seed):
    s = np.random.default_rng(seed).integers(0, alpha, m).astype(np.uint8)
    sa, L, orig = orc.bwt(s)
    bsa, bL, borig = brute_bwt(s.tolist())
    assert list(sa) == bsa and list(L) == bL and orig == borig


def test_bwt_periodic_ties_by_index(orc):
    s = np.frombuffer(b"abc" * 50, np.uint8)
    sa, L, orig = orc.bwt(s)
    assert list(sa) == brute_bwt(list(s))[0]
    assert list(sa[:50]) == list(range(0, 150, 3))


def test_inverse_bwt_large_block(orc):
    rng = np.random.default_rng(6)
    blk = np.repeat(rng.integers(0, 20, 60000).astype(np.uint8), rng.integers(1, 30, 60000))[:899981]
    sa, L, orig = orc.bwt(blk)
    assert np.array_equal(np.sort(sa), np.arange(blk.size))
    np.testing.assert_array_equal(ibwt(L, orig), blk)
    # adjacent rotations are in order on a sample
    for j in rng.integers(0, blk.size - 1, 50):
        a, b = int(sa[j]), int(sa[j + 1])
        ra = np.concatenate([blk[a:], blk[:a]])[:4096]
        rb = np.concatenate([blk[b:], blk[:b]])[:4096]
        assert (ra.tobytes(), a) < (rb.tobytes(), b) or ra.tobytes() < rb.tobytes()


# ------------------------------------------------------------------ MTF + RLE2
def inverse_mtf_rle2(sym, used):
    nu = len(used)
    out, lst, i, run, weight = [], list(range(nu)), 0, 0, 1
    for s in sym:
        if s in (0, 1):
            run += weight * (s + 1)
            weight *= 2
            continue
        out.extend([used[lst[0]]] * run)
        run, weight = 0, 1
        if s == nu + 1:
            break
        v = lst.pop(s - 1)
        lst.insert(0, v)
        out.append(used[v])
    return out


def test_mtf_rle2_golden(orc):
    g = GOLD["mtf_rle2"]
    sym, freq, nu = orc.mtf_rle2(np.frombuffer(g["L"].encode(), np.uint8))
    assert list(sym) == g["sym"] and nu == 3
    assert list(freq[:5]) == [0, 2, 2, 1, 1]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mtf_rle2_inverse(orc, seed):
    rng = np.random.default_rng(seed)
    L = np.repeat(rng.choice([0, 5, 17, 200, 255], 3000).astype(np.uint8), rng.integers(1, 40, 3000))
    sym, freq, nu = orc.mtf_rle2(L)
    used = sorted(set(L.tolist()))
    assert nu == len(used)
    assert inverse_mtf_rle2(sym.tolist(), used) == L.tolist()
    assert np.array_equal(np.bincount(sym, minlength=258)[:258], freq)
    assert sym[-1] == nu + 1


def test_zero_run_digits(orc):
    # a run of r equal bytes after the first occurrence gives r-1 MTF zeros
    for r in range(1, 70):
        L = np.array([1] + [2] * r, np.uint8)
        sym, _, _ = orc.mtf_rle2(L)
        body = sym[2:-1].tolist()
        val, w = 0, 1
        for d in body:
            assert d in (0, 1)
            val += w * (d + 1)
            w *= 2
        assert val == r - 1


# ------------------------------------------------------------------ Huffman lengths
def opt_cost_exhaustive(w, limit):
    n, best = len(w), None
    for lens in itertools.product(range(1, limit + 1), repeat=n):
        if sum(2.0**-l for l in lens) <= 1.0 + 1e-12:
            c = sum(a * b for a, b in zip(w, lens))
            best = c if best is None else min(best, c)
    return best


def huffman_cost(w):
    h = list(w)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("n,limit,seed", [(3, 2, 1), (4, 2, 2), (5, 3, 3), (6, 3, 4), (7, 3, 5), (7, 4, 6), (8, 3, 7)])
def test_package_merge_optimal(orc, n, limit, seed):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        w = rng.integers(1, 60, n).astype(np.uint32)
        if rng.random() < 0.5:
            w = (2 ** rng.integers(0, 12, n)).astype(np.uint32)  # skewed: limit binds
        ln = orc.package_merge(w, limit)
        assert ln.max() <= limit and ln.min() >= 1
        assert sum(2.0 ** -int(l) for l in ln) == 1.0
        assert int((w.astype(np.int64) * ln).sum()) == opt_cost_exhaustive(w.tolist(), limit)


@pytest.mark.parametrize("n,seed", [(3, 1), (40, 2), (258, 3), (258, 4)])
def test_package_merge_equals_huffman_when_unconstrained(orc, n, seed):
    w = np.random.default_rng(seed).integers(1, 5000, n).astype(np.uint32)
    ln = orc.package_merge(w, 17)
    assert int((w.astype(np.int64) * ln).sum()) == huffman_cost(w.tolist())
    assert sum(2.0 ** -int(l) for l in ln) == 1.0


def test_limit_17_binds_on_fibonacci_weights(orc):
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    ln = orc.package_merge(np.array(fib, np.uint32), 17)
    assert ln.max() == 17
    assert sum(2.0 ** -int(l) for l in ln) == 1.0


def test_canonical_codes_prefix_free(orc):
    lens = orc.package_merge(np.random.default_rng(3).integers(1, 900, 100).astype(np.uint32), 17)
    codes = orc.canonical_codes(lens)
    words = sorted(format(int(c), f"0{int(l)}b") for c, l in zip(codes, lens))
    for a, b in zip(words, words[1:]):
        assert not b.startswith(a)


def test_table_count_thresholds(orc):
    for n, G in [(50, 2), (199, 2), (200, 3), (799, 3), (800, 4), (2399, 4), (2400, 5), (5999, 5), (6000, 6)]:
        sym = (np.arange(n) % 20).astype(np.uint16)
        g, sel, lens = orc.huff_tables(sym, 22)
        assert g == G and sel.size == (n + 49) // 50 and lens.shape == (G, 22)
    g, _, _ = orc.huff_tables(np.zeros(7000, np.uint16), 3)
    assert g == 3


# ------------------------------------------------------------------ whole streams
def _inputs():
    rng = np.random.default_rng(11)
    from paper_2310_09467_amd import synth

    yield "random", rng.integers(0, 256, 50000).astype(np.uint8)
    yield "runs", np.repeat(rng.integers(0, 4, 5000).astype(np.uint8), rng.integers(1, 600, 5000))[:300000]
    yield "single", np.array([42], np.uint8)
    yield "two", np.array([1, 2], np.uint8)
    yield "zeros", np.zeros(899981, np.uint8)
    yield "beads", synth.config1_frame().view(np.uint8).ravel().copy()
    for name, f in synth.adversarial_frames(90, 90).items():
        yield "adv_" + name, f.view(np.uint8).ravel().copy()


@pytest.mark.parametrize("level", [1, 9])
def test_streams_decode_with_stock_bz2(orc, level):
    for name, raw in _inputs():
        s, nb = orc.band_streams(raw, level)
        assert bz2.decompress(s) == raw.tobytes(), name
        assert s.startswith(b"BZh" + str(level).encode())


def test_four_run_band_two_streams(orc):
    raw = np.frombuffer(b"aaaab" * 18900, np.uint8)
    s, nb = orc.band_streams(raw, 1)
    assert nb == 2 and bz2.decompress(s) == raw.tobytes()
    assert s.count(b"BZh1") >= 2


@pytest.mark.skipif(shutil.which("bzip2") is None, reason="bzip2 command not installed")
def test_stream_decodes_with_bzip2_command(orc):
    from paper_2310_09467_amd import synth

    raw = synth.config1_frame().view(np.uint8).ravel()
    s, _ = orc.band_streams(raw, 9)
    out = subprocess.run(["bzip2", "-dc"], input=s, capture_output=True, check=True).stdout
    assert out == raw.tobytes()


def test_block_crc_in_header(orc):
    raw = np.frombuffer(b"123456789", np.uint8)
    s, _ = orc.band_streams(raw, 9)
    assert s[4:10] == bytes.fromhex("314159265359")
    assert int.from_bytes(s[10:14], "big") == 0xFC891918


def test_ratio_close_to_bzip2_9(orc):
    from paper_2310_09467_amd import synth

    raw = synth.config1_frame().view(np.uint8).ravel()
    s, _ = orc.band_streams(raw, 9)
    ref = len(bz2.compress(raw.tobytes(), 9))
    assert len(s) < 1.05 * ref


# ------------------------------------------------------------------ hand-derived table and stream pins
# These fix the choices that several valid outputs leave open (every
# selector vector decodes, optimal code lengths are not unique), so that a
# plausible slip -- a strict comparison in the initial ranges, a tie going to
# a later table, packages before leaves on equal weight, another start value
# for the code lengths -- changes a value below.
@pytest.mark.parametrize("case", GOLD["huff_init_ranges"]["cases"])
def test_huff_initial_ranges_hand_cases(orc, case):
    assert orc.huff_init_ranges(case["freq"], case["G"]).tolist() == case["end"]


def test_huff_select_tie_goes_to_lowest_table(orc):
    g = GOLD["huff_select_tie"]
    assert orc.huff_select(g["sym"], g["cost"]).tolist() == g["sel"]


def _groups_to_sym(groups):
    if isinstance(groups, str):  # the clamp case: ten groups of s0, six of s1, four of s2
        return np.array([0] * 500 + [1] * 300 + [2] * 200, np.uint16)
    return np.array([s for grp in groups for s, c in grp for _ in range(c)], np.uint16)


@pytest.mark.parametrize("case", GOLD["huff_tables"]["cases"])
def test_huff_tables_hand_cases(orc, case):
    sym = _groups_to_sym(case["groups"])
    G, sel, lens = orc.huff_tables(sym, case["alpha"])
    assert G == case["G"]
    assert sel.tolist() == case["sel"]
    assert lens.tolist() == case["len"]


@pytest.mark.parametrize("case", GOLD["package_merge_ties"]["cases"])
def test_package_merge_tie_order(orc, case):
    w = np.array(case["w"], np.uint32)
    ln = orc.package_merge(w, case["limit"])
    assert ln.tolist() == case["len"]
    assert int((w.astype(np.int64) * ln).sum()) == opt_cost_exhaustive(case["w"], case["limit"])


def test_stream_of_aaa_hand_derived(orc):
    g = GOLD["stream_aaa"]
    raw = np.frombuffer(g["block"].encode(), np.uint8)
    crc = _rev32(zlib.crc32(_REV8[raw].tobytes()) & 0xFFFFFFFF)
    bits = "".join(format(crc if v == "crc" else v, f"0{n}b") for _, n, v in g["fields"])
    bits += "0" * (-len(bits) % 8)
    want = int(bits, 2).to_bytes(len(bits) // 8, "big")
    got = orc.block_stream(raw, crc, g["level"])
    assert got == want
    assert bz2.decompress(got) == raw.tobytes()
