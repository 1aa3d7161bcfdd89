"""Python binding of libpcbz (argument marshalling only).

Every compute step runs in the library's HIP kernels; torch provides device
memory and the stream handle.  Importing this module never falls back to a
CPU path: if lib/libpcbz.so is missing, the functions raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libpcbz.so")

OK, EINVAL, ENOSPC, EDATA, ENEEDPREV, ENOMEM, EDEVICE = 0, -1, -2, -3, -4, -5, -6
RASTER, VIEW, VIEW_DX, VIEW_DT = 0, 1, 2, 3
_NAMES = {EINVAL: "EINVAL", ENOSPC: "ENOSPC", EDATA: "EDATA", ENEEDPREV: "ENEEDPREV", ENOMEM: "ENOMEM",
          EDEVICE: "EDEVICE"}

EXPORTS = ("pcbz_create", "pcbz_destroy", "pcbz_last_error", "pcbz_plan", "pcbz_judge", "pcbz_compress",
           "pcbz_compress_batch", "pcbz_peek", "pcbz_decompress", "pcbz_last_stats", "pcbz_trace_enable",
           "pcbz_trace_read")


class PcbzError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"pcbz {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_uint32), ("w", ctypes.c_uint32), ("pitch", ctypes.c_uint32),
                ("level", ctypes.c_uint32), ("cand_mask", ctypes.c_uint32)]


_lib = None


def load():
    """Loads libpcbz.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
        # torch's wheel carries its own HIP runtime with the same soname as the
        # one libpcbz links; loading torch first makes the process use a single
        # runtime, so torch's device memory and stream handles are the
        # library's too.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int
        pp = ctypes.POINTER(Params)
        sig = {
            "pcbz_create": (i32, [ctypes.POINTER(vp), i32, sz]),
            "pcbz_destroy": (None, [vp]),
            "pcbz_last_error": (ctypes.c_char_p, [vp]),
            "pcbz_plan": (i32, [pp, vp, vp]),
            "pcbz_judge": (i32, [vp, pp, vp, vp, vp, vp, vp, vp]),
            "pcbz_compress": (i32, [vp, pp, vp, vp, vp, vp, sz, vp, vp, vp]),
            "pcbz_compress_batch": (i32, [vp, u32, pp, vp, vp, vp, vp, vp, vp, vp]),
            "pcbz_peek": (i32, [vp, sz, pp, vp]),
            "pcbz_decompress": (i32, [vp, vp, sz, vp, vp, sz, vp]),
            "pcbz_last_stats": (i32, [vp, vp, vp, vp, vp]),
            "pcbz_trace_enable": (i32, [vp, i32, ctypes.c_char_p]),
            "pcbz_trace_read": (i32, [vp, vp, sz, vp, vp, vp, u32, vp, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def plan(h, w, pitch=15, level=9, cand_mask=0x7):
    p = Params(h, w, pitch, level, cand_mask)
    nb = ctypes.c_uint32()
    bound = ctypes.c_size_t()
    st = load().pcbz_plan(ctypes.byref(p), ctypes.byref(nb), ctypes.byref(bound))
    if st:
        raise PcbzError(st, "plan")
    return nb.value, bound.value


def peek(blob):
    b = np.frombuffer(bytes(blob), np.uint8)
    p = Params()
    nb = ctypes.c_uint32()
    st = load().pcbz_peek(b.ctypes.data_as(ctypes.c_void_p), b.size, ctypes.byref(p), ctypes.byref(nb))
    if st:
        raise PcbzError(st, "peek")
    return dict(h=p.h, w=p.w, pitch=p.pitch, level=p.level, n_bands=nb.value, id_mask=p.cand_mask)


def _torch():
    import torch

    return torch


def to_device(frame, device="cuda"):
    """uint16 frame (numpy or torch) -> contiguous device int16 tensor with the same bits."""
    torch = _torch()
    if isinstance(frame, np.ndarray):
        a = np.ascontiguousarray(frame, np.uint16)
        return torch.from_numpy(a.view(np.int16)).to(device)
    t = frame
    if t.dtype != torch.int16:
        t = t.view(torch.int16) if t.element_size() == 2 else t.to(torch.int16)
    return t.to(device).contiguous()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


class Context:
    """One library context (device workspace, tables); not thread-safe."""

    def __init__(self, device=0, hbm_budget=0):
        h = ctypes.c_void_p()
        st = load().pcbz_create(ctypes.byref(h), device, hbm_budget)
        if st:
            raise PcbzError(st, f"create on device {device}")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().pcbz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, what):
        msg = load().pcbz_last_error(self._h)
        raise PcbzError(st, f"{what}: {msg.decode() if msg else ''}")

    def judge(self, frame, prev=None, pitch=15, level=9, cand_mask=0x7):
        """Returns (choice uint8[n_bands], entropy float64[n_bands,4], score int64[n_bands,4]) on the device."""
        torch = _torch()
        f = to_device(frame)
        pv = None if prev is None else to_device(prev)
        h, w = f.shape
        nb, _ = plan(h, w, pitch, level, cand_mask)
        choice = torch.empty(nb, dtype=torch.uint8, device=f.device)
        ent = torch.empty(nb * 4, dtype=torch.float64, device=f.device)
        score = torch.empty(nb * 4, dtype=torch.int64, device=f.device)
        p = Params(h, w, pitch, level, cand_mask)
        st = load().pcbz_judge(self._h, ctypes.byref(p), _ptr(f), _ptr(pv), _ptr(choice), _ptr(ent), _ptr(score),
                               _stream())
        if st:
            self._err(st, "judge")
        return choice, ent.view(nb, 4), score.view(nb, 4)

    def compress_into(self, f, pv, p, out, forced=None, choice_out=None):
        """Device-level call: f/pv device int16 tensors, out device uint8 tensor.  Returns the length."""
        ln = ctypes.c_size_t()
        st = load().pcbz_compress(self._h, ctypes.byref(p), _ptr(f), _ptr(pv), _ptr(forced), _ptr(out), out.numel(),
                                  ctypes.byref(ln), _ptr(choice_out), _stream())
        if st:
            if st == ENOSPC:
                raise PcbzError(st, f"needs {ln.value} bytes")
            self._err(st, "compress")
        return ln.value

    def compress(self, frame, prev=None, pitch=15, level=9, cand_mask=0x7, forced=None, return_choice=False):
        """Compresses one frame; returns the container as bytes (and the per-band ids)."""
        torch = _torch()
        f = to_device(frame)
        pv = None if prev is None else to_device(prev)
        h, w = f.shape
        nb, bound = plan(h, w, pitch, level, cand_mask)
        out = torch.empty(bound, dtype=torch.uint8, device=f.device)
        fc = None
        if forced is not None:
            fc = torch.as_tensor(np.asarray(forced, np.uint8)).to(f.device)
        choice = torch.empty(nb, dtype=torch.uint8, device=f.device)
        p = Params(h, w, pitch, level, cand_mask)
        ln = self.compress_into(f, pv, p, out, fc, choice)
        blob = out[:ln].cpu().numpy().tobytes()
        if return_choice:
            return blob, choice.cpu().numpy()
        return blob

    def compress_batch(self, frames, prevs=None, params=None, forced=None):
        """Compresses several frames in one pass; returns a list of containers (bytes)."""
        torch = _torch()
        n = len(frames)
        fs = [to_device(f) for f in frames]
        pvs = [None if (prevs is None or prevs[i] is None) else to_device(prevs[i]) for i in range(n)]
        prm = (Params * n)()
        outs, caps = [], (ctypes.c_size_t * n)()
        for i in range(n):
            h, w = fs[i].shape
            pitch, level, mask = params[i] if params is not None else (15, 9, 0x7)
            prm[i] = Params(h, w, pitch, level, mask)
            _, bound = plan(h, w, pitch, level, mask)
            outs.append(torch.empty(bound, dtype=torch.uint8, device=fs[i].device))
            caps[i] = bound
        fcs = None
        if forced is not None:
            fcs = [None if forced[i] is None else torch.as_tensor(np.asarray(forced[i], np.uint8)).to(fs[i].device)
                   for i in range(n)]
        VP = ctypes.c_void_p * n
        d_frames = VP(*[f.data_ptr() for f in fs])
        d_prevs = VP(*[0 if p is None else p.data_ptr() for p in pvs])
        d_outs = VP(*[o.data_ptr() for o in outs])
        d_forced = None if fcs is None else VP(*[0 if c is None else c.data_ptr() for c in fcs])
        lens = (ctypes.c_size_t * n)()
        st = load().pcbz_compress_batch(self._h, n, prm, d_frames, d_prevs, d_forced, d_outs, caps, lens, _stream())
        if st:
            self._err(st, "compress_batch")
        return [outs[i][: lens[i]].cpu().numpy().tobytes() for i in range(n)]

    def decompress(self, blob, prev=None):
        """Decodes a container (host bytes) into a device int16 tensor (uint16 bits)."""
        torch = _torch()
        info = peek(blob)
        out = torch.empty((info["h"], info["w"]), dtype=torch.int16, device=f"cuda:{self.device}")
        b = np.frombuffer(bytes(blob), np.uint8)
        pv = None if prev is None else to_device(prev)
        st = load().pcbz_decompress(self._h, b.ctypes.data_as(ctypes.c_void_p), b.size, _ptr(pv), _ptr(out),
                                    out.numel(), _stream())
        if st:
            self._err(st, "decompress")
        return out

    def trace(self, on=True, kernel=None):
        """Enables HIP-event timing of launches of `kernel` (all kernels when None)."""
        st = load().pcbz_trace_enable(self._h, 1 if on else 0, None if kernel is None else kernel.encode())
        if st:
            self._err(st, "trace_enable")

    def trace_read(self, reset=True, max_names=256):
        """Returns {kernel name: (total ms, launches, algorithmic bytes)} for the traced launches."""
        stride = 96
        names = ctypes.create_string_buffer(stride * max_names)
        ms = (ctypes.c_double * max_names)()
        calls = (ctypes.c_uint64 * max_names)()
        nbytes = (ctypes.c_uint64 * max_names)()
        n = ctypes.c_uint32()
        st = load().pcbz_trace_read(self._h, names, stride, ms, calls, nbytes, max_names, ctypes.byref(n),
                                    1 if reset else 0)
        if st:
            self._err(st, "trace_read")
        out = {}
        for i in range(min(n.value, max_names)):
            nm = names.raw[i * stride:(i + 1) * stride].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], calls[i], nbytes[i])
        return out

    def last_stats(self):
        r, q = ctypes.c_uint64(), ctypes.c_uint64()
        nb, rounds = ctypes.c_uint32(), ctypes.c_uint32()
        load().pcbz_last_stats(self._h, ctypes.byref(r), ctypes.byref(q), ctypes.byref(nb), ctypes.byref(rounds))
        return dict(raw_bytes=r.value, rle_bytes=q.value, blocks=nb.value, bwt_rounds=rounds.value)


def as_uint16(t):
    """Device int16 tensor -> host numpy uint16 array."""
    return t.cpu().numpy().view(np.uint16)
