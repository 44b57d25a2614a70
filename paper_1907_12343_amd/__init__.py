"""Python binding of libhrr.so, the gfx950 hierarchical Russian-roulette library.

Argument marshalling only: every step of the path runs in the HIP kernels
behind the C ABI declared in ``include/hrr.h``.  torch is used for device
memory (tensor storage) and streams.  There is no CPU fallback: if the
library is not built, importing the binding's entry points raises.

u32 quantities travel as torch.int32 tensors holding the same bits; use
``as_u32_numpy`` / ``u32_to_i64`` to read them as unsigned numbers.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrr.so")

HRR_OK, HRR_E_INVALID, HRR_E_NOMEM, HRR_E_OVERFLOW = 0, 1, 2, 3
HRR_E_DEVICE, HRR_E_NOTREADY, HRR_E_CANCELLED, HRR_E_BUSY = 4, 5, 6, 7
RMQ_PAPER, RMQ_DIRECT, RMQ_PAPER_FULL, RMQ_PAPER_LOOP = 0, 1, 2, 3
RMQ_DYADIC, RMQ_PAPER_NO_REUSE = 4, 5   # ablations; the second in traversals only
SPLIT_RADIX, SPLIT_POW2 = 0x000, 0x100   # hierarchy split rules, OR-ed into leaf_size
_SPLITS = {"radix": SPLIT_RADIX, "pow2": SPLIT_POW2}
F_STATS = 1
F_NO_REORDER = 2
F_TIMING = 4

_u32, _u64, _i32, _f32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_float
_P = ctypes.c_void_p


class HrrEyes(ctypes.Structure):
    _fields_ = [("xyz", _P), ("n", _u32), ("width", _u32), ("shift_offset", _u32),
                ("pixel_base", _u32)]


class HrrTraverseOpts(ctypes.Structure):
    _fields_ = [("eyes_per_wave", _u32), ("stack_entries", _u32), ("rmq_method", _u32),
                ("n_samples", _u32), ("psi_s0", _u32), ("flags", _u32)]


class HrrStats(ctypes.Structure):
    _fields_ = [("eyes", _u64), ("pairs", _u64), ("node_visits", _u64), ("rmq_calls", _u64),
                ("leaf_tests", _u64), ("spills", _u64), ("max_stack", _u64),
                ("kernel_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is ctypes.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class HrrHierarchyInfo(ctypes.Structure):
    _fields_ = [("n_lights", _u32), ("leaf_size", _u32), ("n_nodes", _u32), ("depth", _u32),
                ("device_bytes", _u64), ("box", _f32 * 6), ("split", _u32)]


class HrrWorkItem(ctypes.Structure):
    _fields_ = [("h", _P), ("eyes", HrrEyes), ("s", _f32), ("reserved", _u32),
                ("out_offset", _u64), ("out_capacity", _u64)]


class HrrTuneResult(ctypes.Structure):
    _fields_ = [("eyes_per_wave", _u32), ("stack_entries", _u32), ("leaf_size", _u32),
                ("ms", _f32)]


class HrrServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _u64), ("max_inflight", _u32), ("max_batch_eyes", _u32),
                ("max_batch_items", _u32), ("eyes_per_wave", _u32),
                ("pairs_per_eye_guess", _f32), ("overtake_ms", _f32)]


class HrrServerStats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("cancelled", _u64),
                ("rejected", _u64), ("launches", _u64), ("retries", _u64), ("pairs", _u64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("peak_bytes", _u64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is ctypes.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class HrrTicketInfo(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("n_pairs", _u64), ("launches", _u32)]


# every symbol declared in include/hrr.h, with (restype, argtypes)
SIGNATURES = {
    "hrr_create": (_i32, [_i32, _P, _P]),
    "hrr_destroy": (None, [_P]),
    "hrr_last_error": (ctypes.c_char_p, [_P]),
    "hrr_status_string": (ctypes.c_char_p, [_i32]),
    "hrr_version": (_i32, []),
    "hrr_range_min": (_i32, [_P, _P, _P, _P, _u64, _u32, _P, _P, _P, _P]),
    "hrr_build_hierarchy": (_i32, [_P, _P, _u32, _u32, _P, _P]),
    "hrr_build_hierarchy_device": (_i32, [_P, _P, _u32, _u32, _P, _P, _P]),
    "hrr_hierarchy_get_info": (_i32, [_P, _P]),
    "hrr_hierarchy_records": (_i32, [_P, _P]),
    "hrr_hierarchy_permutation": (_i32, [_P, _P]),
    "hrr_hierarchy_sorted_lights": (_i32, [_P, _P]),
    "hrr_free_hierarchy": (None, [_P, _P]),
    "hrr_traverse": (_i32, [_P, _P, _P, _f32, _P, _P, _P, _u64, _P, _P, _P]),
    "hrr_traverse_batched": (_i32, [_P, _P, _u32, _P, _P, _P, _P, _P, _P]),
    "hrr_traverse_noalloc": (_i32, [_P, _P, _P, _f32, _P, _P, _P, _u64, _P, _P]),
    "hrr_autotune": (_i32, [_P, _P, _u32, _P, _f32, _u32, _P, _P]),
    "hrr_autotune_batched": (_i32, [_P, _P, _u32, _u32, _P, _P]),
    "hrr_tuned_leaf_size": (_u32, [_P, _u32]),
    "hrr_server_start": (_i32, [_P, _P]),
    "hrr_server_stop": (_i32, [_P]),
    "hrr_submit": (_i32, [_P, _P, _P, _u32, _u32, _u32, _f32, _P]),
    "hrr_poll": (_i32, [_P, _u64, _P, _P, _P]),
    "hrr_wait": (_i32, [_P, _u64, _u32]),
    "hrr_result_copy": (_i32, [_P, _u64, _P, _u64, _P]),
    "hrr_cancel": (_i32, [_P, _u64]),
    "hrr_release": (_i32, [_P, _u64]),
    "hrr_server_get_stats": (_i32, [_P, _P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhrr.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            "libhrr.so is not built (expected %s); run "
            "`python paper_1907_12343_amd/build.py` -- there is no CPU fallback" % path)
    import torch  # noqa: F401  (its HIP runtime must be the one libhrr binds to)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HrrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class OverflowResult(HrrError):
    pass


def _check(st: int, what: str):
    if st != HRR_OK:
        msg = _lib.hrr_last_error(None).decode(errors="replace")
        raise HrrError(st, "%s: %s" % (what, msg))


def _dptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def as_u32_numpy(t) -> np.ndarray:
    """torch int32 tensor holding u32 bits -> numpy uint32 (host copy)."""
    return t.detach().cpu().numpy().view(np.uint32)


def u32_to_i64(t):
    import torch
    return t.to(torch.int64) & 0xFFFFFFFF


def u32_tensor(a, device):
    """numpy array of u32 values -> torch int32 tensor with the same bits."""
    import torch
    arr = np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)
    return torch.from_numpy(arr).to(device)


NODE_DTYPE = np.dtype([("lo_l", "<f4", 3), ("a", "<u4"), ("hi_l", "<f4", 3), ("c", "<u4"),
                       ("lo_r", "<f4", 3), ("b", "<u4"), ("hi_r", "<f4", 3), ("first", "<u4")])


class Hierarchy:
    """A light hierarchy resident on the context's device."""

    def __init__(self, ctx: "Context", handle: int):
        self._ctx = ctx
        self.handle = handle
        info = HrrHierarchyInfo()
        _check(_lib.hrr_hierarchy_get_info(handle, ctypes.byref(info)), "hierarchy info")
        self.n_lights = info.n_lights
        self.leaf_size = info.leaf_size
        self.n_nodes = info.n_nodes
        self.depth = info.depth
        self.device_bytes = info.device_bytes
        self.box = list(info.box)
        self.split = "pow2" if info.split == SPLIT_POW2 else "radix"

    def permutation(self) -> np.ndarray:
        out = np.empty(self.n_lights, np.uint32)
        _check(_lib.hrr_hierarchy_permutation(self.handle, out.ctypes.data_as(_P)),
               "hierarchy permutation")
        return out

    def sorted_lights(self) -> np.ndarray:
        out = np.empty((self.n_lights, 3), np.float32)
        _check(_lib.hrr_hierarchy_sorted_lights(self.handle, out.ctypes.data_as(_P)),
               "sorted lights")
        return out

    def records(self) -> np.ndarray:
        """Node records (sibling pairs, see include/hrr.h) as a structured array."""
        out = np.zeros(self.n_nodes, NODE_DTYPE)
        _check(_lib.hrr_hierarchy_records(self.handle, out.ctypes.data_as(_P)), "hierarchy records")
        return out

    def free(self):
        if self.handle:
            _lib.hrr_free_hierarchy(self._ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self._ctx.handle:
                self.free()
        except Exception:
            pass


def _opts(eyes_per_wave=0, stack_entries=0, rmq_method=RMQ_PAPER, n_samples=1, psi_s0=0,
          stats=False, reorder=True, timing=False):
    flags = (F_STATS if stats else 0) | (0 if reorder else F_NO_REORDER) | (F_TIMING if timing else 0)
    return HrrTraverseOpts(eyes_per_wave, stack_entries, rmq_method, n_samples,
                           psi_s0 & 0xFFFFFFFF, flags)


class Context:
    """hrr_ctx on one HIP device with a 64x64 dither tile."""

    def __init__(self, tile, device: int = 0):
        load_library()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the hrr library needs an MI355X")
        self.device = device
        self.torch_device = torch.device("cuda", device)
        tile = np.ascontiguousarray(tile, dtype=np.uint32)
        if tile.size != 4096:
            raise ValueError("tile must have 64*64 entries")
        torch.cuda.set_device(device)
        h = _P()
        _check(_lib.hrr_create(device, tile.ctypes.data_as(_P), ctypes.byref(h)), "hrr_create")
        self.handle = h.value

    def close(self):
        if getattr(self, "handle", None):
            _lib.hrr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- range minimum --------------------------------------------------------
    def range_min(self, a, b, r, method: int = RMQ_PAPER, out_k=None, out_v=None,
                  n_invalid=None, stream=None):
        """argmin / min of (bitrev32(i) + r) mod 2^32 over [a, b), per query.

        a, b, r: int32 cuda tensors (u32 bits).  Returns (k, v) int32 tensors.
        Asynchronous on the current stream.
        """
        import torch
        n = a.numel()
        for t in (a, b, r):
            if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous() and t.numel() == n):
                raise ValueError("a, b, r must be contiguous int32 cuda tensors of one size")
        if out_k is None:
            out_k = torch.empty_like(a)
        if out_v is None:
            out_v = torch.empty_like(a)
        _check(_lib.hrr_range_min(self.handle, _dptr(a), _dptr(b), _dptr(r), n, method,
                                  _dptr(out_k), _dptr(out_v), _dptr(n_invalid),
                                  _stream_handle(stream)), "hrr_range_min")
        return out_k, out_v

    # -- hierarchy ------------------------------------------------------------
    def build_hierarchy(self, lights_xyz, leaf_size: int = 1, box=None,
                        split: str = "radix") -> Hierarchy:
        """split: "radix" (highest differing Morton bit) or "pow2" (left child =
        largest power of two below the node's length)."""
        lights = np.ascontiguousarray(lights_xyz, dtype=np.float32).reshape(-1, 3)
        bx = None if box is None else np.ascontiguousarray(box, dtype=np.float32)
        h = _P()
        _check(_lib.hrr_build_hierarchy(self.handle, lights.ctypes.data_as(_P), lights.shape[0],
                                        leaf_size | _SPLITS[split],
                                        None if bx is None else bx.ctypes.data_as(_P),
                                        ctypes.byref(h)), "hrr_build_hierarchy")
        return Hierarchy(self, h.value)

    def build_hierarchy_device(self, lights_xyz, leaf_size: int = 1, box=None, stream=None,
                               split: str = "radix") -> Hierarchy:
        """The same hierarchy built on the GPU from a (n, 3) float32 cuda tensor."""
        import torch
        if not (lights_xyz.is_cuda and lights_xyz.dtype == torch.float32 and lights_xyz.is_contiguous()
                and lights_xyz.dim() == 2 and lights_xyz.shape[1] == 3):
            raise ValueError("lights must be a contiguous (n, 3) float32 cuda tensor")
        bx = None if box is None else np.ascontiguousarray(box, dtype=np.float32)
        h = _P()
        _check(_lib.hrr_build_hierarchy_device(self.handle, _dptr(lights_xyz), lights_xyz.shape[0],
                                               leaf_size | _SPLITS[split],
                                               None if bx is None else bx.ctypes.data_as(_P),
                                               _stream_handle(stream), ctypes.byref(h)),
               "hrr_build_hierarchy_device")
        return Hierarchy(self, h.value)

    # -- traversal ------------------------------------------------------------
    def _eyes(self, eyes, width, shift_offset, pixel_base):
        import torch
        if not (eyes.is_cuda and eyes.dtype == torch.float32 and eyes.is_contiguous()
                and eyes.dim() == 2 and eyes.shape[1] == 3):
            raise ValueError("eyes must be a contiguous (n, 3) float32 cuda tensor")
        return HrrEyes(_dptr(eyes), eyes.shape[0], width, shift_offset & 0xFFFFFFFF,
                       pixel_base)

    def traverse(self, h: Hierarchy, eyes, s: float, width: int, shift_offset: int = 0,
                 pixel_base: int = 0, capacity: Optional[int] = None, pairs=None,
                 weights=None, with_weights: bool = False, stream=None, **opt):
        """Cull eye x light pairs.  Returns (pairs[:n] as (n, 2) int32 view, n, stats)."""
        import torch
        E = self._eyes(eyes, width, shift_offset, pixel_base)
        o = _opts(**opt)
        if pairs is None:
            if capacity is None:
                capacity = 1 << 20
            pairs = torch.empty((capacity, 2), dtype=torch.int32, device=eyes.device)
        capacity = pairs.shape[0] if capacity is None else min(capacity, pairs.shape[0])
        if with_weights and weights is None:
            weights = torch.empty((capacity,), dtype=torch.float32, device=eyes.device)
        n = ctypes.c_uint64()
        st = HrrStats()
        code = _lib.hrr_traverse(self.handle, h.handle, ctypes.byref(E), float(s), ctypes.byref(o),
                                 _dptr(pairs), _dptr(weights), capacity, ctypes.byref(n),
                                 ctypes.byref(st), _stream_handle(stream))
        if code == HRR_E_OVERFLOW:
            err = OverflowResult(code, "hrr_traverse: %d pairs exceed capacity %d"
                                 % (n.value, capacity))
            err.count = int(n.value)
            raise err
        _check(code, "hrr_traverse")
        k = int(n.value)
        out = (pairs[:k], k, st.as_dict())
        if weights is not None:
            return out + (weights[:k],)
        return out

    def traverse_noalloc(self, h: Hierarchy, eyes, s: float, width: int, pairs, result,
                         weights=None, shift_offset: int = 0, pixel_base: int = 0,
                         capacity: Optional[int] = None, stream=None, **opt):
        """Enqueue the allocation-free traversal (nothing allocated, nothing
        read back).  pairs: (capacity, 2) int32 device tensor; result: int64
        device tensor of 2 elements that receives (true count, status)."""
        E = self._eyes(eyes, width, shift_offset, pixel_base)
        o = _opts(**opt)
        capacity = pairs.shape[0] if capacity is None else min(capacity, pairs.shape[0])
        _check(_lib.hrr_traverse_noalloc(self.handle, h.handle, ctypes.byref(E), float(s),
                                         ctypes.byref(o), _dptr(pairs), _dptr(weights), capacity,
                                         _dptr(result), _stream_handle(stream)),
               "hrr_traverse_noalloc")

    def traverse_all(self, h: Hierarchy, eyes, s, width, **kw):
        """traverse() after a count-only pass that sizes the output exactly."""
        cnt_kw = {k: v for k, v in kw.items() if k not in ("with_weights",)}
        n = self.count(h, eyes, s, width, **cnt_kw)
        return self.traverse(h, eyes, s, width, capacity=max(n, 1), **kw)

    def count(self, h: Hierarchy, eyes, s, width, **kw):
        import torch
        E = self._eyes(eyes, width, kw.pop("shift_offset", 0), kw.pop("pixel_base", 0))
        kw.pop("with_weights", None)
        stream = kw.pop("stream", None)
        o = _opts(**kw)
        n = ctypes.c_uint64()
        code = _lib.hrr_traverse(self.handle, h.handle, ctypes.byref(E), float(s), ctypes.byref(o),
                                 None, None, 0, ctypes.byref(n), None, _stream_handle(stream))
        if code not in (HRR_OK, HRR_E_OVERFLOW):
            _check(code, "hrr_traverse (count)")
        return int(n.value)

    def traverse_batched(self, items: Sequence[dict], pairs, weights=None, stream=None, **opt):
        """items: dicts with h, eyes, s, width, [shift_offset, pixel_base], out_offset,
        out_capacity.  Returns (counts np.uint64, stats)."""
        arr = (HrrWorkItem * len(items))()
        keep = []
        for k, it in enumerate(items):
            E = self._eyes(it["eyes"], it["width"], it.get("shift_offset", 0),
                           it.get("pixel_base", 0))
            keep.append(it["eyes"])
            arr[k] = HrrWorkItem(it["h"].handle, E, float(it["s"]), 0, int(it["out_offset"]),
                                 int(it["out_capacity"]))
        counts = np.zeros(len(items), np.uint64)
        st = HrrStats()
        o = _opts(**opt)
        code = _lib.hrr_traverse_batched(self.handle, arr, len(items), ctypes.byref(o),
                                         _dptr(pairs), _dptr(weights),
                                         counts.ctypes.data_as(_P), ctypes.byref(st),
                                         _stream_handle(stream))
        if code == HRR_E_OVERFLOW:
            err = OverflowResult(code, "hrr_traverse_batched: an item exceeded its capacity")
            err.counts = counts       # true count of every item
            raise err
        _check(code, "hrr_traverse_batched")
        return counts, st.as_dict()

    def autotune(self, hs: Sequence[Hierarchy], eyes, s: float, width: int,
                 max_probe_eyes: int = 4096, stream=None):
        arr = (_P * len(hs))(*[h.handle for h in hs])
        E = self._eyes(eyes, width, 0, 0)
        res = HrrTuneResult()
        _check(_lib.hrr_autotune(self.handle, arr, len(hs), ctypes.byref(E), float(s),
                                 max_probe_eyes, ctypes.byref(res), _stream_handle(stream)),
               "hrr_autotune")
        return dict(eyes_per_wave=res.eyes_per_wave, stack_entries=res.stack_entries,
                    leaf_size=res.leaf_size, ms=res.ms)

    def autotune_batched(self, sets: Sequence[Sequence[dict]], stream=None):
        """sets: equally long lists of dicts (h, eyes, s, width, [shift_offset,
        pixel_base]), set q built with its own leaf size; see hrr_autotune_batched."""
        n_items = len(sets[0])
        if any(len(x) != n_items for x in sets):
            raise ValueError("every set needs the same items")
        arr = (HrrWorkItem * (len(sets) * n_items))()
        keep = []
        for q, items in enumerate(sets):
            for k, it in enumerate(items):
                E = self._eyes(it["eyes"], it["width"], it.get("shift_offset", 0), it.get("pixel_base", 0))
                keep.append(it["eyes"])
                arr[q * n_items + k] = HrrWorkItem(it["h"].handle, E, float(it["s"]), 0, 0, 0)
        res = HrrTuneResult()
        _check(_lib.hrr_autotune_batched(self.handle, arr, len(sets), n_items, ctypes.byref(res),
                                         _stream_handle(stream)), "hrr_autotune_batched")
        return dict(eyes_per_wave=res.eyes_per_wave, stack_entries=res.stack_entries,
                    leaf_size=res.leaf_size, ms=res.ms)

    def tuned_leaf_size(self, n_lights: int) -> int:
        return int(_lib.hrr_tuned_leaf_size(self.handle, n_lights))

    # -- serving ------------------------------------------------------------------
    def server_start(self, hbm_budget_bytes: int, max_inflight: int = 2,
                     max_batch_eyes: int = 1 << 16, max_batch_items: int = 64,
                     eyes_per_wave: int = 0, pairs_per_eye_guess: float = 64.0,
                     overtake_ms: float = 100.0):
        cfg = HrrServerConfig(hbm_budget_bytes, max_inflight, max_batch_eyes, max_batch_items,
                              eyes_per_wave, pairs_per_eye_guess, overtake_ms)
        _check(_lib.hrr_server_start(self.handle, ctypes.byref(cfg)), "hrr_server_start")

    def server_stop(self):
        _check(_lib.hrr_server_stop(self.handle), "hrr_server_stop")

    def submit(self, h: Hierarchy, eyes_xyz, width: int, shift_offset: int, s: float) -> int:
        e = np.ascontiguousarray(eyes_xyz, dtype=np.float32).reshape(-1, 3)
        t = ctypes.c_uint64()
        _check(_lib.hrr_submit(self.handle, h.handle, e.ctypes.data_as(_P), e.shape[0], width,
                               shift_offset & 0xFFFFFFFF, float(s), ctypes.byref(t)),
               "hrr_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """None while running; else (device address, n_pairs, info dict)."""
        p = _P()
        n = ctypes.c_uint64()
        info = HrrTicketInfo()
        code = _lib.hrr_poll(self.handle, ticket, ctypes.byref(p), ctypes.byref(n),
                             ctypes.byref(info))
        if code == HRR_E_NOTREADY:
            return None
        _check(code, "hrr_poll")
        return (p.value or 0, int(n.value),
                dict(submit_s=info.submit_s, start_s=info.start_s, done_s=info.done_s,
                     n_pairs=int(info.n_pairs), launches=int(info.launches)))

    def wait(self, ticket: int, timeout_ms: int = 60000) -> bool:
        code = _lib.hrr_wait(self.handle, ticket, timeout_ms)
        if code == HRR_E_NOTREADY:
            return False
        _check(code, "hrr_wait")
        return True

    def cancel(self, ticket: int) -> int:
        return int(_lib.hrr_cancel(self.handle, ticket))

    def release(self, ticket: int):
        _check(_lib.hrr_release(self.handle, ticket), "hrr_release")

    def result(self, ticket: int, device=None, stream=None):
        """Copy a complete request's pairs into a new (n, 2) int32 cuda tensor."""
        import torch
        ready = self.poll(ticket)
        if ready is None:
            raise HrrError(HRR_E_NOTREADY, "request %d has not finished" % ticket)
        n = ready[1]
        dev = torch.device("cuda", self.device) if device is None else device
        out = torch.empty((max(n, 1), 2), dtype=torch.int32, device=dev)
        _check(_lib.hrr_result_copy(self.handle, ticket, _dptr(out), n, _stream_handle(stream)),
               "hrr_result_copy")
        return out[:n]

    def server_stats(self):
        st = HrrServerStats()
        _check(_lib.hrr_server_get_stats(self.handle, ctypes.byref(st)), "hrr_server_get_stats")
        return st.as_dict()
