"""The oracle's pins have teeth: each test builds a copy of the oracle with one
plausible slip planted in it (on the CPU, in a temporary directory) and shows
that the matching hand-derived golden rejects it.  The slips are the open
choices of the bzip2 encoder that no decoder can see: the initial table
ranges (E11), the table chosen on equal cost (E12), the order of a leaf and a
package of equal weight (E13) and the start value of the code-length coding
(E16)."""
import ctypes
import json
import os
import subprocess
import tempfile
import zlib

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "pcbz_oracle.c")
GOLD = json.load(open(os.path.join(HERE, "golden", "closed_forms.json")))
_REV8 = np.array([int(f"{i:08b}"[::-1], 2) for i in range(256)], np.uint8)

MUTANTS = {
    "e11_strict": ("if (acc * (uint64_t)left >= remaining) break;", "if (acc * (uint64_t)left > remaining) break;"),
    "e12_tie_high": ("if (g == 0 || c < best_c) {", "if (g == 0 || c <= best_c) {"),
    "e13_packages_first": ("(uint64_t)w[order[li]] <= pw", "(uint64_t)w[order[li]] < pw"),
    "e16_start_last": ("int cur = lens[g * 258];", "int cur = lens[g * 258 + alpha - 1];"),
}


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _build(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found once"
    path = os.path.join(tmp, f"{name}.c")
    open(path, "w").write(src.replace(old, new))
    so = os.path.join(tmp, f"lib{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-I", os.path.dirname(SRC),
                           "-o", so, path, "-lm"])
    return ctypes.CDLL(so)


def _init_ranges(L, freq, G):
    f = np.ascontiguousarray(freq, np.uint32)
    end = np.zeros(G, np.int32)
    L.orc_huff_init_ranges.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p]
    L.orc_huff_init_ranges(_p(f), f.size, G, int(f.sum()), _p(end))
    return end.tolist()


def _select(L, sym, cost):
    s = np.ascontiguousarray(sym, np.uint16)
    c = np.zeros((len(cost), 258), np.uint32)
    c[:, : len(cost[0])] = cost
    sel = np.zeros((s.size + 49) // 50, np.uint8)
    L.orc_huff_select.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    L.orc_huff_select(_p(s), s.size, _p(c), len(cost), _p(sel))
    return sel.tolist()


def _pm(L, w, limit):
    w = np.ascontiguousarray(w, np.uint32)
    ln = np.zeros(w.size, np.uint8)
    L.orc_package_merge.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    L.orc_package_merge(_p(w), w.size, limit, _p(ln))
    return ln.tolist()


def _stream(L, raw, crc, level):
    out = np.zeros(4096, np.uint8)
    ln = np.zeros(1, np.uintp)
    L.orc_block_stream.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    assert L.orc_block_stream(_p(raw), raw.size, crc, level, _p(out), out.size, _p(ln)) == 0
    return bytes(out[: int(ln[0])])


def _goldens_pass(L):
    """True when every table and stream golden holds for library L."""
    ok = all(_init_ranges(L, c["freq"], c["G"]) == c["end"] for c in GOLD["huff_init_ranges"]["cases"])
    g = GOLD["huff_select_tie"]
    ok &= _select(L, g["sym"], g["cost"]) == g["sel"]
    ok &= all(_pm(L, c["w"], c["limit"]) == c["len"] for c in GOLD["package_merge_ties"]["cases"])
    g = GOLD["stream_aaa"]
    raw = np.frombuffer(g["block"].encode(), np.uint8)
    crc = int(f"{zlib.crc32(_REV8[raw].tobytes()) & 0xFFFFFFFF:032b}"[::-1], 2)
    bits = "".join(format(crc if v == "crc" else v, f"0{n}b") for _, n, v in g["fields"])
    bits += "0" * (-len(bits) % 8)
    ok &= _stream(L, raw, crc, g["level"]) == int(bits, 2).to_bytes(len(bits) // 8, "big")
    return ok


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "plain.c")
        open(src, "w").write(open(SRC).read())
        so = os.path.join(tmp, "libplain.so")
        subprocess.check_call(["gcc", "-O1", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-I", os.path.dirname(SRC),
                               "-o", so, src, "-lm"])
        assert _goldens_pass(ctypes.CDLL(so))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_slip_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        assert not _goldens_pass(_build(name, tmp)), f"the goldens do not catch {name}"
