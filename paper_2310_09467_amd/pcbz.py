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
NCAND = 16  # arrangement ids; 4 + 4 * domain + function: the predictor family
_NAMES = {EINVAL: "EINVAL", ENOSPC: "ENOSPC", EDATA: "EDATA", ENEEDPREV: "ENEEDPREV", ENOMEM: "ENOMEM",
          EDEVICE: "EDEVICE"}

EXPORTS = ("pcbz_create", "pcbz_destroy", "pcbz_last_error", "pcbz_plan", "pcbz_judge", "pcbz_compress",
           "pcbz_compress_batch", "pcbz_peek", "pcbz_decompress", "pcbz_last_stats", "pcbz_trace_enable",
           "pcbz_trace_read", "pcbz_selector_num_params", "pcbz_selector_create", "pcbz_selector_free",
           "pcbz_selector_get_params", "pcbz_selector_set_params", "pcbz_selector_save", "pcbz_selector_load",
           "pcbz_features", "pcbz_selector_forward", "pcbz_selector_gradients", "pcbz_selector_train_step",
           "pcbz_gemm_bf16", "pcbz_set_selector", "pcbz_selector_stats", "pcbz_set_graphs", "pcbz_server_create",
           "pcbz_server_submit", "pcbz_server_poll", "pcbz_server_stats", "pcbz_server_destroy",
           "pcbz_selector_inspect", "pcbz_judge_noalloc", "pcbz_decompress_batch", "pcbz_decompress_inspect")


class PcbzError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"pcbz {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_uint32), ("w", ctypes.c_uint32), ("pitch", ctypes.c_uint32),
                ("level", ctypes.c_uint32), ("cand_mask", ctypes.c_uint32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("prev_tag", ctypes.c_uint64), ("camera", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("data", ctypes.c_void_p), ("len", ctypes.c_size_t),
                ("latency_ms", ctypes.c_double), ("submit_ms", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "pending", "admitted", "in_flight",
                                               "batches", "batched_frames", "pool_bytes", "pool_used",
                                               "pool_peak")] + [("busy_ms", ctypes.c_double),
                                                                ("overlap_ms", ctypes.c_double)]


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
            "pcbz_judge_noalloc": (i32, [vp, pp, vp, vp, vp, vp, vp, vp]),
            "pcbz_compress": (i32, [vp, pp, vp, vp, vp, vp, sz, vp, vp, vp]),
            "pcbz_compress_batch": (i32, [vp, u32, pp, vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, vp]),
            "pcbz_peek": (i32, [vp, sz, pp, vp]),
            "pcbz_decompress": (i32, [vp, vp, sz, vp, vp, sz, vp]),
            "pcbz_decompress_batch": (i32, [vp, u32, vp, vp, vp, vp, vp, vp]),
            "pcbz_decompress_inspect": (i32, [vp, i32, vp, sz]),
            "pcbz_last_stats": (i32, [vp, vp, vp, vp, vp]),
            "pcbz_trace_enable": (i32, [vp, i32, ctypes.c_char_p]),
            "pcbz_trace_read": (i32, [vp, vp, sz, vp, vp, vp, u32, vp, i32]),
            "pcbz_selector_num_params": (sz, []),
            "pcbz_selector_create": (i32, [vp, vp, vp, ctypes.POINTER(vp)]),
            "pcbz_selector_free": (None, [vp]),
            "pcbz_selector_get_params": (i32, [vp, vp, vp]),
            "pcbz_selector_set_params": (i32, [vp, vp, vp]),
            "pcbz_selector_save": (i32, [vp, ctypes.c_char_p]),
            "pcbz_selector_load": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(vp)]),
            "pcbz_features": (i32, [vp, pp, vp, vp, vp, vp]),
            "pcbz_selector_forward": (i32, [vp, vp, u32, vp, vp]),
            "pcbz_selector_gradients": (i32, [vp, vp, vp, u32, vp, vp, vp, vp]),
            "pcbz_selector_train_step": (i32, [vp, vp, vp, u32, vp, ctypes.c_float, ctypes.c_float, vp, vp]),
            "pcbz_gemm_bf16": (i32, [i32, i32, i32, vp, vp, vp, vp]),
            "pcbz_selector_inspect": (i32, [vp, i32, vp, sz]),
            "pcbz_set_selector": (i32, [vp, vp, ctypes.c_float]),
            "pcbz_selector_stats": (i32, [vp, vp, vp]),
            "pcbz_set_graphs": (i32, [vp, i32]),
            "pcbz_server_create": (i32, [i32, sz, u32, sz, vp, ctypes.c_float, ctypes.POINTER(vp)]),
            "pcbz_server_submit": (i32, [vp, pp, vp, u32, ctypes.c_uint64]),
            "pcbz_server_poll": (i32, [vp, ctypes.POINTER(ServerResult), u32, vp, i32]),
            "pcbz_server_stats": (i32, [vp, ctypes.POINTER(ServerInfo)]),
            "pcbz_server_destroy": (None, [vp]),
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

    def judge(self, frame, prev=None, pitch=15, level=9, cand_mask=0x7, noalloc=False):
        """Returns (choice uint8[n_bands], entropy float64[n_bands,16], score int64[n_bands,16]) on the device.

        noalloc=True calls pcbz_judge_noalloc (fixed device workspace)."""
        torch = _torch()
        f = to_device(frame)
        pv = None if prev is None else to_device(prev)
        h, w = f.shape
        nb, _ = plan(h, w, pitch, level, cand_mask)
        choice = torch.empty(nb, dtype=torch.uint8, device=f.device)
        ent = torch.empty(nb * NCAND, dtype=torch.float64, device=f.device)
        score = torch.empty(nb * NCAND, dtype=torch.int64, device=f.device)
        self.judge_into(f, pv, Params(h, w, pitch, level, cand_mask), choice, ent, score, noalloc)
        return choice, ent.view(nb, NCAND), score.view(nb, NCAND)

    def judge_into(self, f, pv, p, choice, ent=None, score=None, noalloc=False):
        """Device-level judge: f/pv device tensors, outputs preallocated device tensors."""
        fn = load().pcbz_judge_noalloc if noalloc else load().pcbz_judge
        st = fn(self._h, ctypes.byref(p), _ptr(f), _ptr(pv), _ptr(choice), _ptr(ent), _ptr(score), _stream())
        if st:
            self._err(st, "judge_noalloc" if noalloc else "judge")

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

    def compress_batch(self, frames, prevs=None, params=None, forced=None, selector=None, min_conf=0.9):
        """Compresses several frames in one pass; returns a list of containers
        (bytes).  `selector` (a Selector, or None for the exhaustive judgement)
        and min_conf apply to this call only."""
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
        st = load().pcbz_compress_batch(self._h, n, prm, d_frames, d_prevs, d_forced,
                                        None if selector is None else selector._h, float(min_conf), d_outs, caps,
                                        lens, _stream())
        if st:
            self._err(st, "compress_batch")
        return [outs[i][: lens[i]].cpu().numpy().tobytes() for i in range(n)]

    def compress_batch_into(self, dev_frames, dev_prevs, params, outs, selector=None, min_conf=0.9):
        """Device-level batch call: device int16 frames (and prevs or None),
        Params list, device uint8 output tensors, optional Selector.  Returns
        the lengths."""
        n = len(dev_frames)
        prm = (Params * n)(*params)
        VP = ctypes.c_void_p * n
        caps = (ctypes.c_size_t * n)(*[o.numel() for o in outs])
        lens = (ctypes.c_size_t * n)()
        d_prevs = None if dev_prevs is None else VP(*[0 if p is None else p.data_ptr() for p in dev_prevs])
        st = load().pcbz_compress_batch(self._h, n, prm, VP(*[f.data_ptr() for f in dev_frames]), d_prevs, None,
                                        None if selector is None else selector._h, float(min_conf),
                                        VP(*[o.data_ptr() for o in outs]), caps, lens, _stream())
        if st:
            self._err(st, "compress_batch")
        return list(lens)

    def decompress(self, blob, prev=None):
        """Decodes a container (host bytes or a device uint8 tensor) into a
        device int16 tensor (uint16 bits) on the GPU."""
        return self.decompress_batch([blob], [prev])[0]

    def decompress_batch(self, blobs, prevs=None):
        """Decodes several containers in one call; returns device int16 tensors."""
        torch = _torch()
        n = len(blobs)
        dev = [b if hasattr(b, "data_ptr") else
               torch.from_numpy(np.frombuffer(bytes(b), np.uint8).copy()).to(f"cuda:{self.device}") for b in blobs]
        outs = []
        for b, d in zip(blobs, dev):
            head = bytes(b[:20].cpu().numpy().tobytes()) if hasattr(b, "data_ptr") else bytes(b[:20])
            h = int.from_bytes(head[8:12], "little") if len(head) >= 20 else 0
            w = int.from_bytes(head[12:16], "little") if len(head) >= 20 else 0
            outs.append(torch.empty((h, w), dtype=torch.int16, device=f"cuda:{self.device}"))
        pvs = [None if prevs is None or prevs[i] is None else to_device(prevs[i]) for i in range(n)]
        VP = ctypes.c_void_p * n
        SZ = ctypes.c_size_t * n
        st = load().pcbz_decompress_batch(self._h, n, VP(*[d.data_ptr() for d in dev]), SZ(*[d.numel() for d in dev]),
                                          VP(*[0 if p is None else p.data_ptr() for p in pvs]),
                                          VP(*[o.data_ptr() for o in outs]), SZ(*[o.numel() for o in outs]),
                                          _stream())
        if st:
            self._err(st, "decompress")
        return outs

    def decompress_batch_into(self, dev_blobs, lens, dev_prevs, outs):
        """Device-level batch decode: device uint8 containers with their lengths,
        device int16 previous frames (or None) and outputs."""
        n = len(dev_blobs)
        VP = ctypes.c_void_p * n
        SZ = ctypes.c_size_t * n
        pv = VP(*[0 if dev_prevs is None or dev_prevs[i] is None else dev_prevs[i].data_ptr() for i in range(n)])
        st = load().pcbz_decompress_batch(self._h, n, VP(*[d.data_ptr() for d in dev_blobs]), SZ(*lens), pv,
                                          VP(*[o.data_ptr() for o in outs]), SZ(*[o.numel() for o in outs]), _stream())
        if st:
            self._err(st, "decompress")

    def decompress_inspect(self, which, nbytes, dtype=np.uint8):
        """One intermediate array of the last decompression call (see the header)."""
        buf = np.zeros(nbytes, np.uint8)
        st = load().pcbz_decompress_inspect(self._h, int(which), buf.ctypes.data_as(ctypes.c_void_p), nbytes)
        if st:
            raise PcbzError(st, "decompress_inspect")
        return buf.view(dtype)

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

    def features(self, frame, prev=None, pitch=15, level=9, cand_mask=0x7):
        """Per-band selector features: device float32 tensor [n_bands, 64, 64, 4]."""
        torch = _torch()
        f = to_device(frame)
        pv = None if prev is None else to_device(prev)
        h, w = f.shape
        nb, _ = plan(h, w, pitch, level, cand_mask)
        out = torch.empty((nb, 64, 64, 4), dtype=torch.float32, device=f.device)
        p = Params(h, w, pitch, level, cand_mask)
        st = load().pcbz_features(self._h, ctypes.byref(p), _ptr(f), _ptr(pv), _ptr(out), _stream())
        if st:
            self._err(st, "features")
        return out

    def set_selector(self, sel, min_conf=0.9):
        """Compress calls consult `sel` (None: judge every band)."""
        st = load().pcbz_set_selector(self._h, None if sel is None else sel._h, float(min_conf))
        if st:
            self._err(st, "set_selector")
        self._sel = sel  # keeps the selector alive while it is set

    def set_graphs(self, on=True):
        """pcbz_compress_batch mode: True / 1 = graphs where the autotuner finds
        them faster than eager calls, 2 = always graphs, False / 0 = eager."""
        st = load().pcbz_set_graphs(self._h, int(on))
        if st:
            self._err(st, "set_graphs")

    def selector_stats(self):
        """(bands seen by the selector, bands judged) of the last compress call."""
        n, j = ctypes.c_uint32(), ctypes.c_uint32()
        load().pcbz_selector_stats(self._h, ctypes.byref(n), ctypes.byref(j))
        return n.value, j.value

    def last_stats(self):
        r, q = ctypes.c_uint64(), ctypes.c_uint64()
        nb, rounds = ctypes.c_uint32(), ctypes.c_uint32()
        load().pcbz_last_stats(self._h, ctypes.byref(r), ctypes.byref(q), ctypes.byref(nb), ctypes.byref(rounds))
        return dict(raw_bytes=r.value, rle_bytes=q.value, blocks=nb.value, bwt_rounds=rounds.value)


def selector_num_params():
    return int(load().pcbz_selector_num_params())


class Selector:
    """Learned arrangement selector (network parameters on the device)."""

    def __init__(self, ctx, params=None, norm=None, _handle=None):
        self.ctx = ctx
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        pa = None if params is None else np.ascontiguousarray(params, np.float32)
        if pa is not None and pa.size != selector_num_params():
            raise ValueError(f"expected {selector_num_params()} parameters, got {pa.size}")
        nm = None if norm is None else np.ascontiguousarray(norm, np.float32).reshape(8)
        st = load().pcbz_selector_create(ctx._h, None if pa is None else pa.ctypes.data_as(ctypes.c_void_p),
                                         None if nm is None else nm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
        if st:
            raise PcbzError(st, "selector_create")
        self._h = h

    @classmethod
    def load_file(cls, ctx, path):
        h = ctypes.c_void_p()
        st = load().pcbz_selector_load(ctx._h, str(path).encode(), ctypes.byref(h))
        if st:
            raise PcbzError(st, f"selector_load {path}")
        return cls(ctx, _handle=h)

    def save(self, path):
        st = load().pcbz_selector_save(self._h, str(path).encode())
        if st:
            raise PcbzError(st, f"selector_save {path}")

    def close(self):
        if getattr(self, "_h", None):
            load().pcbz_selector_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        """(parameters float32[num_params], norm float32[8]) on the host."""
        p = np.empty(selector_num_params(), np.float32)
        nm = np.empty(8, np.float32)
        st = load().pcbz_selector_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                             nm.ctypes.data_as(ctypes.c_void_p))
        if st:
            raise PcbzError(st, "selector_get_params")
        return p, nm

    def set_params(self, params, norm=None):
        pa = np.ascontiguousarray(params, np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, np.float32).reshape(8)
        st = load().pcbz_selector_set_params(self._h, pa.ctypes.data_as(ctypes.c_void_p),
                                             None if nm is None else nm.ctypes.data_as(ctypes.c_void_p))
        if st:
            raise PcbzError(st, "selector_set_params")

    def forward(self, feat):
        """feat: device float32 [n, 64, 64, 4] -> device float32 logits [n, 4]."""
        torch = _torch()
        feat = feat.contiguous()
        n = feat.shape[0]
        out = torch.empty((n, 4), dtype=torch.float32, device=feat.device)
        st = load().pcbz_selector_forward(self._h, _ptr(feat), n, _ptr(out), _stream())
        if st:
            raise PcbzError(st, "selector_forward")
        return out

    @staticmethod
    def _cw(class_w):
        if class_w is None:
            return None
        return (ctypes.c_float * 4)(*[float(x) for x in class_w])

    def gradients(self, feat, labels, class_w=None):
        """Returns (device float32 gradient [num_params], loss)."""
        torch = _torch()
        feat = feat.contiguous()
        lab = labels.to(torch.uint8).contiguous()
        g = torch.empty(selector_num_params(), dtype=torch.float32, device=feat.device)
        loss = ctypes.c_float()
        st = load().pcbz_selector_gradients(self._h, _ptr(feat), _ptr(lab), feat.shape[0], self._cw(class_w), _ptr(g),
                                            ctypes.byref(loss), _stream())
        if st:
            raise PcbzError(st, "selector_gradients")
        return g, loss.value

    # (name, dtype, per-sample shape) of pcbz_selector_inspect's tensors, by index
    INSPECT = (("x0", "bf16", (64, 64, 4)), ("x1", "bf16", (32, 32, 32)), ("x2", "bf16", (16, 16, 32)),
               ("x3", "bf16", (2048,)), ("x4", "bf16", (64,)), ("pre1", "f32", (1024, 32)),
               ("pre2", "f32", (256, 32)), ("pre3", "f32", (64, 32)), ("pre4", "f32", (64,)),
               ("logits", "f32", (4,)), ("dlogits", "f32", (4,)), ("g5", "bf16", (4,)), ("g4", "bf16", (64,)),
               ("g3", "bf16", (64, 32)), ("g2", "bf16", (256, 32)), ("g1", "bf16", (1024, 32)))

    def inspect(self, name, n):
        """A tensor of the last gradients call (n samples) as a numpy array:
        bf16 tensors come back as float32 values, FP32 ones as they are."""
        which = [nm for nm, _, _ in self.INSPECT].index(name)
        _, kind, shape = self.INSPECT[which]
        count = n * int(np.prod(shape))
        if kind == "bf16":
            buf = np.empty(count, np.uint16)
        else:
            buf = np.empty(count, np.float32)
        st = load().pcbz_selector_inspect(self._h, which, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes)
        if st:
            raise PcbzError(st, "selector_inspect")
        if kind == "bf16":
            buf = (buf.astype(np.uint32) << 16).view(np.float32)
        return buf.reshape((n,) + shape)

    def train_step(self, feat, labels, class_w=None, lr=1e-3, weight_decay=1e-4):
        """One AdamW step; returns the batch loss before the step."""
        torch = _torch()
        feat = feat.contiguous()
        lab = labels.to(torch.uint8).contiguous()
        loss = ctypes.c_float()
        st = load().pcbz_selector_train_step(self._h, _ptr(feat), _ptr(lab), feat.shape[0], self._cw(class_w),
                                             float(lr), float(weight_decay), ctypes.byref(loss), _stream())
        if st:
            raise PcbzError(st, "selector_train_step")
        return loss.value


class Server:
    """Serving loop: submit host frames as they arrive, poll finished containers.

    Host frames must stay alive (and unchanged) until their result is polled;
    pinned host memory makes the uploads asynchronous.
    """

    def __init__(self, device=0, hbm_budget=32 << 30, workers=2, max_batch_bytes=0, selector=None,
                 min_conf=1.01):
        h = ctypes.c_void_p()
        st = load().pcbz_server_create(device, int(hbm_budget), int(workers), int(max_batch_bytes),
                                       None if selector is None else selector._h, float(min_conf),
                                       ctypes.byref(h))
        if st:
            raise PcbzError(st, "server_create")
        self._h = h
        self._keep = {}  # tag -> host frame, alive until polled

    def submit(self, frame, tag, camera=0, pitch=15, level=9, cand_mask=0x7):
        """frame: host uint16 array or tensor (pinned for asynchronous upload)."""
        if hasattr(frame, "data_ptr"):
            ptr, (h, w) = frame.data_ptr(), tuple(frame.shape)
        else:
            frame = np.ascontiguousarray(frame, np.uint16)
            ptr, (h, w) = frame.ctypes.data, frame.shape
        p = Params(h, w, pitch, level, cand_mask)
        self._keep[int(tag)] = frame
        st = load().pcbz_server_submit(self._h, ctypes.byref(p), ctypes.c_void_p(ptr), int(camera), int(tag))
        if st:
            self._keep.pop(int(tag), None)
            raise PcbzError(st, f"server_submit tag {tag}")

    def poll(self, max_results=256, timeout_ms=0):
        """List of dicts (tag, prev_tag, camera, status, data bytes, latency_ms, submit_ms)."""
        res = (ServerResult * max_results)()
        n = ctypes.c_uint32()
        st = load().pcbz_server_poll(self._h, res, max_results, ctypes.byref(n), int(timeout_ms))
        if st:
            raise PcbzError(st, "server_poll")
        out = []
        for i in range(n.value):
            r = res[i]
            data = ctypes.string_at(r.data, r.len) if r.len else b""
            self._keep.pop(int(r.tag), None)
            out.append(dict(tag=r.tag, prev_tag=None if r.prev_tag == 2 ** 64 - 1 else r.prev_tag,
                            camera=r.camera, status=r.status, data=data, latency_ms=r.latency_ms,
                            submit_ms=r.submit_ms))
        return out

    def stats(self):
        info = ServerInfo()
        load().pcbz_server_stats(self._h, ctypes.byref(info))
        return {n: getattr(info, n) for n, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().pcbz_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(a16, b16):
    """C = A x B on the selector's matrix-core kernel; a16 [M, K], b16 [K, N] device int16 (bf16 bits)."""
    torch = _torch()
    a16, b16 = a16.contiguous(), b16.contiguous()
    M, K = a16.shape
    K2, N = b16.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    c = torch.empty((M, N), dtype=torch.float32, device=a16.device)
    st = load().pcbz_gemm_bf16(M, N, K, _ptr(a16), _ptr(b16), _ptr(c), _stream())
    if st:
        raise PcbzError(st, "gemm_bf16")
    return c


def as_uint16(t):
    """Device int16 tensor -> host numpy uint16 array."""
    return t.cpu().numpy().view(np.uint16)
