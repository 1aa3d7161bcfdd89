"""CPU oracle for the PC-bzip2 hot path (ctypes wrapper over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the GPU library and its
Python binding never do.  The C code (pcbz_oracle.c) is a plain sequential
implementation of the paper's steps (arXiv 2310.09467 Sec. 2.1.1-2.1.4,
Eq. 1, Fig. 2) plus the public bzip2 stream format; every bzip2 encoder choice
the format leaves open is pinned by the PCBZ-1 profile documented there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcbz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOSPC, EDATA, ENEEDPREV, ENOMEM = 0, -1, -2, -3, -4, -5
RASTER, VIEW, VIEW_DX, VIEW_DT = 0, 1, 2, 3
INT64_MIN = -(2**63)
NCAND = 16  # arrangement ids 0..15 (4..15: the predictor family)
PRED_FIRST = 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, plain C99)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_uint32), ("w", ctypes.c_uint32), ("pitch", ctypes.c_uint32),
                ("level", ctypes.c_uint32), ("cand_mask", ctypes.c_uint32)]


def _P(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, u32, u64, sz, i32, i64 = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t,
                                      ctypes.c_int, ctypes.c_int64)
        pp = ctypes.POINTER(_Params)
        sigs = {
            "orc_block_limit": (u32, [u32]),
            "orc_check_params": (i32, [pp]),
            "orc_plan": (i32, [pp, vp, vp]),
            "orc_band_geometry": (i32, [pp, u32, vp, vp]),
            "orc_arrange": (i32, [pp, u32, i32, vp, vp, vp]),
            "orc_unarrange": (i32, [pp, u32, i32, vp, vp, vp]),
            "orc_to_bytes": (None, [vp, sz, vp]),
            "orc_order1_lastcol": (None, [vp, sz, vp]),
            "orc_pair_hist": (None, [vp, sz, vp]),
            "orc_tq": (i64, [u64]),
            "orc_score": (i64, [vp]),
            "orc_entropy_bits": (ctypes.c_double, [i64, sz]),
            "orc_band_score": (i64, [vp, sz]),
            "orc_judge": (i32, [pp, vp, vp, vp, vp, vp]),
            "orc_crc32_bzip2": (u32, [vp, sz]),
            "orc_rle1_blocks": (sz, [vp, sz, u32, vp, vp, vp, sz, vp]),
            "orc_bwt": (None, [vp, sz, vp, vp, vp]),
            "orc_mtf_rle2": (sz, [vp, sz, vp, vp, vp]),
            "orc_package_merge": (None, [vp, i32, i32, vp]),
            "orc_canonical_codes": (None, [vp, i32, vp]),
            "orc_huff_init_ranges": (None, [vp, i32, i32, u64, vp]),
            "orc_huff_select": (None, [vp, sz, vp, i32, vp]),
            "orc_huff_tables": (i32, [vp, sz, i32, vp, vp, vp, vp]),
            "orc_block_stream": (i32, [vp, sz, u32, u32, vp, sz, vp]),
            "orc_band_streams": (i32, [vp, sz, u32, vp, sz, vp, vp]),
            "orc_container_header_bytes": (sz, [u32]),
            "orc_compress": (i32, [pp, vp, vp, vp, vp, sz, vp, vp]),
            "orc_peek": (i32, [vp, sz, pp, vp, vp, vp]),
            "orc_zigzag16": (ctypes.c_uint16, [ctypes.c_uint16]),
            "orc_unzigzag16": (ctypes.c_uint16, [ctypes.c_uint16]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


def params(h, w, pitch=15, level=9, cand_mask=0x7):
    return _Params(h, w, pitch, level, cand_mask)


# ---------------------------------------------------------------- band plan
def block_limit(level):
    return lib().orc_block_limit(level)


def plan(h, w, pitch=15, level=9, cand_mask=0x7):
    p = params(h, w, pitch, level, cand_mask)
    R, nb = np.zeros(1, np.uint32), np.zeros(1, np.uint32)
    _check(lib().orc_plan(ctypes.byref(p), _P(R), _P(nb)), "plan")
    return int(R[0]), int(nb[0])


def band_geometry(h, w, pitch, level, band):
    p = params(h, w, pitch, level, 1)
    y0, rb = np.zeros(1, np.uint32), np.zeros(1, np.uint32)
    _check(lib().orc_band_geometry(ctypes.byref(p), band, _P(y0), _P(rb)), "band_geometry")
    return int(y0[0]), int(rb[0])


def arrange(frame, band, cid, prev=None, pitch=15, level=9):
    frame = np.ascontiguousarray(frame, np.uint16)
    h, w = frame.shape
    y0, rb = band_geometry(h, w, pitch, level, band)
    out = np.zeros(rb * pitch * w, np.uint16)
    pr = None if prev is None else np.ascontiguousarray(prev, np.uint16)
    p = params(h, w, pitch, level, 1)
    _check(lib().orc_arrange(ctypes.byref(p), band, cid, _P(frame), _P(pr), _P(out)), "arrange")
    return out


def unarrange(arranged, frame_shape, band, cid, prev=None, pitch=15, level=9, into=None):
    h, w = frame_shape
    arranged = np.ascontiguousarray(arranged, np.uint16)
    frame = np.zeros((h, w), np.uint16) if into is None else into
    pr = None if prev is None else np.ascontiguousarray(prev, np.uint16)
    p = params(h, w, pitch, level, 1)
    _check(lib().orc_unarrange(ctypes.byref(p), band, cid, _P(arranged), _P(pr), _P(frame)), "unarrange")
    return frame


def zigzag16(r):
    return int(lib().orc_zigzag16(int(r) & 0xFFFF))


def unzigzag16(z):
    return int(lib().orc_unzigzag16(int(z) & 0xFFFF))


def to_bytes(v):
    v = np.ascontiguousarray(v, np.uint16).ravel()
    out = np.zeros(2 * v.size, np.uint8)
    lib().orc_to_bytes(_P(v), v.size, _P(out))
    return out


# ---------------------------------------------------------------- judgement
def order1_lastcol(x):
    x = np.ascontiguousarray(x, np.uint8)
    T = np.zeros(x.size, np.uint8)
    lib().orc_order1_lastcol(_P(x), x.size, _P(T))
    return T


def pair_hist(T):
    T = np.ascontiguousarray(T, np.uint8)
    P = np.zeros(65536, np.uint32)
    lib().orc_pair_hist(_P(T), T.size, _P(P))
    return P


def tq(c):
    return lib().orc_tq(int(c))


def score(P):
    P = np.ascontiguousarray(P, np.uint32)
    return lib().orc_score(_P(P))


def entropy_bits(S, n):
    return lib().orc_entropy_bits(int(S), int(n))


def band_score(x):
    x = np.ascontiguousarray(x, np.uint8)
    return lib().orc_band_score(_P(x), x.size)


def judge(frame, prev=None, pitch=15, level=9, cand_mask=0x7):
    frame = np.ascontiguousarray(frame, np.uint16)
    h, w = frame.shape
    _, nb = plan(h, w, pitch, level, cand_mask)
    p = params(h, w, pitch, level, cand_mask)
    choice = np.zeros(nb, np.uint8)
    S = np.zeros(nb * NCAND, np.int64)
    H = np.zeros(nb * NCAND, np.float64)
    pr = None if prev is None else np.ascontiguousarray(prev, np.uint16)
    _check(lib().orc_judge(ctypes.byref(p), _P(frame), _P(pr), _P(choice), _P(S), _P(H)), "judge")
    return choice, S.reshape(nb, NCAND), H.reshape(nb, NCAND)


# ---------------------------------------------------------------- bzip2 stages
def crc32_bzip2(data):
    d = np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else np.ascontiguousarray(data, np.uint8)
    return lib().orc_crc32_bzip2(_P(d), d.size)


def rle1_blocks(raw, level=9, limit=None):
    raw = np.ascontiguousarray(raw, np.uint8)
    n = raw.size
    lim = block_limit(level) if limit is None else limit
    out = np.zeros(n + n // 4 + 8, np.uint8)
    maxb = n // 4 + 4
    rs, os_ = np.zeros(maxb, np.uintp), np.zeros(maxb, np.uintp)
    nb = np.zeros(1, np.uintp)
    o = lib().orc_rle1_blocks(_P(raw), n, lim, _P(out), _P(rs), _P(os_), maxb, _P(nb))
    k = int(nb[0])
    return out[:o].copy(), rs[:k].astype(np.int64), os_[:k].astype(np.int64)


def bwt(blk):
    blk = np.ascontiguousarray(blk, np.uint8)
    m = blk.size
    sa = np.zeros(max(m, 1), np.uint32)
    L = np.zeros(max(m, 1), np.uint8)
    orig = np.zeros(1, np.uint32)
    lib().orc_bwt(_P(blk), m, _P(sa), _P(L), _P(orig))
    return sa[:m], L[:m], int(orig[0])


def mtf_rle2(L):
    L = np.ascontiguousarray(L, np.uint8)
    sym = np.zeros(L.size + 2, np.uint16)
    freq = np.zeros(258, np.uint32)
    nu = np.zeros(1, np.uint32)
    n = lib().orc_mtf_rle2(_P(L), L.size, _P(sym), _P(freq), _P(nu))
    return sym[:n].copy(), freq, int(nu[0])


def package_merge(w, limit=17):
    w = np.ascontiguousarray(w, np.uint32)
    ln = np.zeros(w.size, np.uint8)
    lib().orc_package_merge(_P(w), w.size, limit, _P(ln))
    return ln


def canonical_codes(lens):
    lens = np.ascontiguousarray(lens, np.uint8)
    code = np.zeros(lens.size, np.uint32)
    lib().orc_canonical_codes(_P(lens), lens.size, _P(code))
    return code


def huff_init_ranges(freq, G):
    """Last symbol of each of the G initial table ranges (E11)."""
    freq = np.ascontiguousarray(freq, np.uint32)
    end = np.zeros(G, np.int32)
    lib().orc_huff_init_ranges(_P(freq), freq.size, G, int(freq.astype(np.uint64).sum()), _P(end))
    return end


def huff_select(sym, cost):
    """Table per group of 50 symbols for cost tables cost[G][alpha] (E12 a)."""
    sym = np.ascontiguousarray(sym, np.uint16)
    cost = np.asarray(cost, np.uint32)
    G = cost.shape[0]
    c = np.zeros((G, 258), np.uint32)
    c[:, : cost.shape[1]] = cost
    sel = np.zeros((sym.size + 49) // 50, np.uint8)
    lib().orc_huff_select(_P(sym), sym.size, _P(c), G, _P(sel))
    return sel


def huff_tables(sym, alpha):
    sym = np.ascontiguousarray(sym, np.uint16)
    G, nsel = np.zeros(1, np.int32), np.zeros(1, np.uint32)
    sel = np.zeros(sym.size // 50 + 2, np.uint8)
    lens = np.zeros(6 * 258, np.uint8)
    _check(lib().orc_huff_tables(_P(sym), sym.size, alpha, _P(G), _P(nsel), _P(sel), _P(lens)), "huff_tables")
    g = int(G[0])
    return g, sel[: int(nsel[0])].copy(), lens.reshape(6, 258)[:g, :alpha].copy()


def block_stream(rle_block, block_crc, level=9):
    rle_block = np.ascontiguousarray(rle_block, np.uint8)
    cap = rle_block.size * 2 + 4096
    out = np.zeros(cap, np.uint8)
    ln = np.zeros(1, np.uintp)
    _check(lib().orc_block_stream(_P(rle_block), rle_block.size, block_crc, level, _P(out), cap, _P(ln)),
           "block_stream")
    return bytes(out[: int(ln[0])])


def band_streams(raw, level=9):
    raw = np.ascontiguousarray(raw, np.uint8)
    cap = raw.size * 3 + 8192
    out = np.zeros(cap, np.uint8)
    ln, nb = np.zeros(1, np.uintp), np.zeros(1, np.uintp)
    _check(lib().orc_band_streams(_P(raw), raw.size, level, _P(out), cap, _P(ln), _P(nb)), "band_streams")
    return bytes(out[: int(ln[0])]), int(nb[0])


# ---------------------------------------------------------------- whole frame
def header_bytes(n_bands):
    return lib().orc_container_header_bytes(n_bands)


def compress(frame, prev=None, pitch=15, level=9, cand_mask=0x7, forced_choice=None):
    """Compress one frame; returns (container bytes, per-band choice)."""
    frame = np.ascontiguousarray(frame, np.uint16)
    h, w = frame.shape
    _, nb = plan(h, w, pitch, level, cand_mask)
    p = params(h, w, pitch, level, cand_mask)
    cap = header_bytes(nb) + 3 * h * w + 4096 * nb
    out = np.zeros(cap, np.uint8)
    ln = np.zeros(1, np.uintp)
    choice = np.zeros(nb, np.uint8)
    pr = None if prev is None else np.ascontiguousarray(prev, np.uint16)
    fc = None if forced_choice is None else np.ascontiguousarray(forced_choice, np.uint8)
    _check(lib().orc_compress(ctypes.byref(p), _P(frame), _P(pr), _P(fc), _P(out), cap, _P(ln), _P(choice)),
           "compress")
    return bytes(out[: int(ln[0])]), choice


def peek(blob):
    b = np.frombuffer(bytes(blob), np.uint8)
    p = _Params()
    nb = np.zeros(1, np.uint32)
    ids = np.zeros(65536, np.uint8)
    bl = np.zeros(65536, np.uint64)
    _check(lib().orc_peek(_P(b), b.size, ctypes.byref(p), _P(nb), _P(ids), _P(bl)), "peek")
    k = int(nb[0])
    return dict(h=p.h, w=p.w, pitch=p.pitch, level=p.level, n_bands=k, ids=ids[:k].copy(),
                band_len=bl[:k].astype(np.int64))


def decompress(blob, prev=None):
    """Decode a container (test infrastructure): each band's streams with the
    stock bz2 decoder, then the inverse arrangement named by the band's id
    (orc_unarrange).  Returns the frame."""
    import bz2

    info = peek(blob)
    h, w, pitch, level, nb = info["h"], info["w"], info["pitch"], info["level"], info["n_bands"]
    frame = np.zeros((h, w), np.uint16)
    pos = header_bytes(nb)
    for b in range(nb):
        ln = int(info["band_len"][b])
        data = bz2.decompress(bytes(blob[pos:pos + ln]))
        unarrange(np.frombuffer(data, "<u2"), (h, w), b, int(info["ids"][b]), prev, pitch, level, into=frame)
        pos += ln
    return frame

