"""CPU oracle for the hierarchical Russian-roulette hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  The arithmetic lives in
``hrr_oracle.c`` (plain C, one operation at a time); this module only
marshals numpy arrays into it.

What each function follows (Pantaleoni, "Blue-Noise Dithered QMC
Hierarchical Russian Roulette"):

* ``bitrev``/``phi``        Section 2, definition of the radical inverse
                            Phi_b; Section 1, the rotated sequence phi_j.
* ``rmq_scan``              Section 1, v(a,b) = min over [a,b) of phi_j, and
                            Section 2, its argmin k; by scanning every index.
* ``rmq_dyadic``            the same minimum in closed form over aligned
                            dyadic blocks, for ranges too long to scan; pinned
                            to ``rmq_scan`` by the tests.
* ``morton_order``          Section 1, light vertices sorted by a spatial
                            hierarchy so that the sort position is the
                            sequence index i.
* ``eye_shift``             Section 1 and the teaser figure: one rotation per
                            eye vertex from a 64x64 dither tile.
* ``accept``/``accept_eyes``  the all-pairs Russian-roulette test that
                            hierarchical culling must reproduce exactly.
* ``psi``                   Section 3, rank-1 golden-ratio lattice used as an
                            extra rotation per sample.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhrr_oracle.so")
_lib = None


def _threads(threads):
    if threads:
        return int(threads)
    return max(1, min(16, os.cpu_count() or 1))


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    u32, u64, i32, i64 = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                          ctypes.c_int64)
    P = ctypes.c_void_p
    L.or_bitrev.restype = u64
    L.or_bitrev.argtypes = [u64, i32]
    L.or_phi.restype = u64
    L.or_phi.argtypes = [u64, u64, i32]
    L.or_rmq_scan_one.restype = None
    L.or_rmq_scan_one.argtypes = [u64, u64, u64, i32, P, P]
    L.or_rmq_dyadic_one.restype = None
    L.or_rmq_dyadic_one.argtypes = [u64, u64, u64, i32, P, P]
    L.or_rmq_batch.restype = None
    L.or_rmq_batch.argtypes = [P, P, P, i64, i32, i32, P, P, i32]
    L.or_morton.restype = u64
    L.or_morton.argtypes = [ctypes.c_float] * 3 + [P]
    L.or_morton_order.restype = i32
    L.or_morton_order.argtypes = [P, u32, P, P]
    L.or_eye_shift.restype = u32
    L.or_eye_shift.argtypes = [P, u32, u32, u32]
    L.or_golden_alpha.restype = u32
    L.or_golden_alpha.argtypes = []
    L.or_psi.restype = u32
    L.or_psi.argtypes = [u32, u32]
    L.or_accept_prob.restype = ctypes.c_float
    L.or_accept_prob.argtypes = [P, P, ctypes.c_float]
    L.or_accept.restype = i32
    L.or_accept.argtypes = [P, P, ctypes.c_float, u32]
    L.or_accept_weight.restype = ctypes.c_float
    L.or_accept_weight.argtypes = [P, P, ctypes.c_float]
    L.or_fingerprint_hash.restype = u64
    L.or_fingerprint_hash.argtypes = [u64]
    L.or_accept_eyes.restype = None
    L.or_accept_eyes.argtypes = [P, P, i64, u32, u32, P, P, u32, ctypes.c_float,
                                 u32, u32, P, P, P, P, P, P, i32]
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# -- sequence ---------------------------------------------------------------

def bitrev(i: int, B: int = 32) -> int:
    return int(lib().or_bitrev(int(i), int(B)))


def phi(i: int, r: int, B: int = 32) -> int:
    return int(lib().or_phi(int(i), int(r), int(B)))


# -- range minimum ----------------------------------------------------------

def rmq_scan_one(a: int, b: int, r: int, B: int = 32):
    k, v = ctypes.c_uint64(), ctypes.c_uint64()
    lib().or_rmq_scan_one(int(a), int(b), int(r), int(B), ctypes.byref(k),
                          ctypes.byref(v))
    return int(k.value), int(v.value)


def rmq_dyadic_one(a: int, b: int, r: int, B: int = 32):
    k, v = ctypes.c_uint64(), ctypes.c_uint64()
    lib().or_rmq_dyadic_one(int(a), int(b), int(r), int(B), ctypes.byref(k),
                            ctypes.byref(v))
    return int(k.value), int(v.value)


def _rmq_batch(a, b, r, B, method, threads):
    a, b, r = _c(a, np.uint32), _c(b, np.uint32), _c(r, np.uint32)
    n = a.size
    k = np.empty(n, np.uint32)
    v = np.empty(n, np.uint32)
    lib().or_rmq_batch(_ptr(a), _ptr(b), _ptr(r), n, int(B), int(method),
                       _ptr(k), _ptr(v), _threads(threads))
    return k, v


def rmq_scan(a, b, r, B: int = 32, threads=None):
    """(argmin, min) of phi over [a,b) for each query, by scanning."""
    return _rmq_batch(a, b, r, B, 0, threads)


def rmq_dyadic(a, b, r, B: int = 32, threads=None):
    """(argmin, min) of phi over [a,b) for each query, dyadic closed form."""
    return _rmq_batch(a, b, r, B, 1, threads)


# -- light order --------------------------------------------------------------

def morton(x: float, y: float, z: float, box=None) -> int:
    bx = None if box is None else _c(box, np.float32)
    return int(lib().or_morton(float(x), float(y), float(z), _ptr(bx)))


def morton_order(xyz, box=None) -> np.ndarray:
    """perm[i] = original index of the light with sequence index i."""
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    bx = None if box is None else _c(box, np.float32)
    perm = np.empty(xyz.shape[0], np.uint32)
    if lib().or_morton_order(_ptr(xyz), xyz.shape[0], _ptr(bx), _ptr(perm)):
        raise MemoryError("oracle morton_order")
    return perm


# -- shifts and acceptance -----------------------------------------------------

def eye_shift(tile, j: int, width: int, offset: int = 0) -> int:
    tile = _c(tile, np.uint32)
    return int(lib().or_eye_shift(_ptr(tile), int(j), int(width), int(offset)))


def golden_alpha() -> int:
    return int(lib().or_golden_alpha())


def psi(n: int, s0: int = 0) -> int:
    return int(lib().or_psi(int(n), int(s0)))


def accept_prob(e, l, s: float) -> float:
    e, l = _c(e, np.float32), _c(l, np.float32)
    return float(lib().or_accept_prob(_ptr(e), _ptr(l), float(s)))


def accept(e, l, s: float, xi: int) -> bool:
    e, l = _c(e, np.float32), _c(l, np.float32)
    return bool(lib().or_accept(_ptr(e), _ptr(l), float(s), int(xi)))


def accept_weight(e, l, s: float) -> float:
    """1 / p of the pair in binary32."""
    e, l = _c(e, np.float32), _c(l, np.float32)
    return float(lib().or_accept_weight(_ptr(e), _ptr(l), float(s)))


def fingerprint_hash(i: int) -> int:
    return int(lib().or_fingerprint_hash(int(i)))


def accept_eyes(eyes, sel, width: int, offset: int, tile, lights_sorted,
                s: float, n_samples: int = 1, psi_s0: int = 0,
                lists: bool = False, threads=None):
    """All-pairs accepted set for the eyes ``sel``.

    Returns a dict with per-selected-eye ``count``, ``fp_sum`` and ``fp_xor``
    (sum / xor of SplitMix64 of ((n << 32) | i) over accepted pairs), and with
    ``lists=True`` also ``offsets`` (len(sel)+1), ``idx`` (accepted light
    indices in ascending order per eye and sample) and ``sample``.
    """
    eyes = _c(eyes, np.float32).reshape(-1, 3)
    sel = _c(sel, np.uint32)
    tile = _c(tile, np.uint32)
    lights_sorted = _c(lights_sorted, np.float32).reshape(-1, 3)
    n = sel.size
    cnt = np.zeros(n, np.uint64)
    fs = np.zeros(n, np.uint64)
    fx = np.zeros(n, np.uint64)
    L = lib()
    th = _threads(threads)
    args = (_ptr(eyes), _ptr(sel), n, int(width), int(offset) & 0xFFFFFFFF,
            _ptr(tile), _ptr(lights_sorted), lights_sorted.shape[0], float(s),
            int(n_samples), int(psi_s0) & 0xFFFFFFFF)
    L.or_accept_eyes(*args, _ptr(cnt), _ptr(fs), _ptr(fx), None, None, None, th)
    out = dict(count=cnt, fp_sum=fs, fp_xor=fx)
    if lists:
        off = np.zeros(n + 1, np.uint64)
        np.cumsum(cnt, out=off[1:])
        tot = int(off[-1])
        idx = np.empty(max(tot, 1), np.uint32)
        smp = np.empty(max(tot, 1), np.uint32)
        cnt2 = np.zeros(n, np.uint64)
        L.or_accept_eyes(*args, _ptr(cnt2), None, None, _ptr(off[:-1].copy()),
                         _ptr(idx), _ptr(smp), th)
        out.update(offsets=off, idx=idx[:tot], sample=smp[:tot])
    return out
