"""Python face of the CPU oracle (test infrastructure only).

Wraps oracle/liboracle.so (plain C, see nbb_oracle.c for the definitions and
their places in the paper).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product library never imports it.

Compact indices are canonical: i = sum_mu H_mu k^mu, H_mu the replica id of
the level-mu digit pair (section 3.1).  Outside coordinates map to -1 here.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence, Tuple

import numpy as np

from . import build_oracle

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        L = ctypes.CDLL(build_oracle.LIB)
        vp, i64, u64, u32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_double)
        L.orc_make.argtypes = [vp, i64, i64, vp, i64]
        L.orc_make.restype = ctypes.c_int
        L.orc_fractal_size.restype = ctypes.c_size_t
        L.orc_member.argtypes = [vp, i64, i64]
        L.orc_member.restype = ctypes.c_int
        L.orc_nu.argtypes = [vp, i64, i64]
        L.orc_nu.restype = i64
        L.orc_lambda.argtypes = [vp, i64, vp, vp]
        L.orc_nu_paper2d.argtypes = [vp, i64, i64, vp, vp]
        L.orc_nu_paper2d.restype = ctypes.c_int
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_splitmix64.restype = u64
        L.orc_threshold.argtypes = [dbl]
        L.orc_threshold.restype = u32
        L.orc_init_bbox.argtypes = [vp, vp, u64, dbl]
        L.orc_init_compact.argtypes = [vp, vp, u64, dbl]
        L.orc_member_mask.argtypes = [vp, vp]
        L.orc_bbox_step.argtypes = [vp, vp, vp, vp, u32]
        L.orc_compact_step.argtypes = [vp, vp, vp, u32]
        L.orc_gather.argtypes = [vp, vp, vp]
        L.orc_expand.argtypes = [vp, vp, vp]
        L.orc_lambda_many.argtypes = [vp, vp, i64, vp, vp]
        L.orc_nu_many.argtypes = [vp, vp, vp, i64, vp]
        L.orc_cells_after.argtypes = [vp, vp, vp, i64, u32, ctypes.c_int, vp]
        L.orc_cells_after_seeded.argtypes = [vp, u64, dbl, vp, i64, u32, ctypes.c_int, vp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def splitmix64(seed: int, key: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), key & (2**64 - 1)))


def threshold(p: float) -> int:
    return int(lib().orc_threshold(p))


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


class Fractal:
    """F^{k,s} at level r with replica offsets [(x0,y0), (x1,y1), ...]."""

    def __init__(self, s: int, offsets: Sequence[Tuple[int, int]], r: int):
        self.s, self.r = int(s), int(r)
        self.offsets = tuple((int(a), int(b)) for a, b in offsets)
        self.k = len(self.offsets)
        self.n = self.s ** self.r
        self.cells = self.k ** self.r
        self._buf = ctypes.create_string_buffer(int(lib().orc_fractal_size()))
        flat = np.array([c for o in self.offsets for c in o], dtype=np.int32)
        if lib().orc_make(self._buf, self.k, self.s, _ptr(flat), self.r) != 0:
            raise ValueError("not an NBB fractal the oracle accepts")
        self._h = ctypes.addressof(self._buf)

    # ---- maps -------------------------------------------------------------
    def member(self, x: int, y: int) -> bool:
        return bool(lib().orc_member(self._h, int(x), int(y)))

    def lam(self, i: int) -> Tuple[int, int]:
        if not 0 <= i < self.cells:
            raise IndexError(i)
        x, y = ctypes.c_int64(), ctypes.c_int64()
        lib().orc_lambda(self._h, int(i), ctypes.byref(x), ctypes.byref(y))
        return x.value, y.value

    def nu(self, x: int, y: int) -> int:
        return int(lib().orc_nu(self._h, int(x), int(y)))

    def nu_paper2d(self, x: int, y: int):
        nx, ny = ctypes.c_int64(), ctypes.c_int64()
        if not lib().orc_nu_paper2d(self._h, int(x), int(y), ctypes.byref(nx), ctypes.byref(ny)):
            return None
        return nx.value, ny.value

    def lam_many(self, idx) -> Tuple[np.ndarray, np.ndarray]:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= self.cells):
            raise IndexError("index out of range")
        x = np.empty_like(idx)
        y = np.empty_like(idx)
        lib().orc_lambda_many(self._h, _ptr(idx), idx.size, _ptr(x), _ptr(y))
        return x, y

    def nu_many(self, x, y) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.int64)
        y = np.ascontiguousarray(y, dtype=np.int64)
        out = np.empty_like(x)
        lib().orc_nu_many(self._h, _ptr(x), _ptr(y), x.size, _ptr(out))
        return out

    # ---- states -----------------------------------------------------------
    def member_mask(self) -> np.ndarray:
        m = np.empty((self.n, self.n), dtype=np.uint8)
        lib().orc_member_mask(self._h, _ptr(m))
        return m

    def init_bbox(self, seed: int, p: float) -> np.ndarray:
        st = np.empty((self.n, self.n), dtype=np.uint8)
        lib().orc_init_bbox(self._h, _ptr(st), seed & (2**64 - 1), float(p))
        return st

    def init_compact(self, seed: int, p: float) -> np.ndarray:
        st = np.empty(self.cells, dtype=np.uint8)
        lib().orc_init_compact(self._h, _ptr(st), seed & (2**64 - 1), float(p))
        return st

    def gather(self, bbox: np.ndarray) -> np.ndarray:
        bbox = np.ascontiguousarray(bbox, dtype=np.uint8)
        assert bbox.size == self.n * self.n
        out = np.empty(self.cells, dtype=np.uint8)
        lib().orc_gather(self._h, _ptr(bbox), _ptr(out))
        return out

    def expand(self, compact: np.ndarray) -> np.ndarray:
        compact = np.ascontiguousarray(compact, dtype=np.uint8)
        assert compact.size == self.cells
        out = np.empty((self.n, self.n), dtype=np.uint8)
        lib().orc_expand(self._h, _ptr(compact), _ptr(out))
        return out

    def bbox_steps(self, state: np.ndarray, rule: int, steps: int, mask=None) -> np.ndarray:
        a = np.ascontiguousarray(state, dtype=np.uint8).reshape(self.n, self.n).copy()
        b = np.empty_like(a)
        mask = self.member_mask() if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        for _ in range(int(steps)):
            lib().orc_bbox_step(self._h, _ptr(mask), _ptr(a), _ptr(b), int(rule))
            a, b = b, a
        return a

    def cells_after(self, state: np.ndarray, idx, rule: int, steps: int) -> np.ndarray:
        """States of the compact cells idx after `steps` generations (steps <= 3)."""
        st = np.ascontiguousarray(state, dtype=np.uint8)
        assert st.size == self.cells and 0 <= steps <= 3
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= self.cells):
            raise IndexError("index out of range")
        out = np.empty(idx.size, dtype=np.uint8)
        lib().orc_cells_after(self._h, _ptr(st), _ptr(idx), idx.size, int(rule), int(steps), _ptr(out))
        return out

    def cells_after_seeded(self, seed: int, p: float, idx, rule: int, steps: int) -> np.ndarray:
        """As cells_after, from the Bernoulli(p) initial state of `seed`,
        evaluated per cell (no whole-state array; steps <= 3)."""
        assert 0 <= steps <= 3
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= self.cells):
            raise IndexError("index out of range")
        out = np.empty(idx.size, dtype=np.uint8)
        lib().orc_cells_after_seeded(self._h, seed & (2 ** 64 - 1), float(p), _ptr(idx), idx.size, int(rule),
                                     int(steps), _ptr(out))
        return out

    def compact_steps(self, state: np.ndarray, rule: int, steps: int) -> np.ndarray:
        a = np.ascontiguousarray(state, dtype=np.uint8).copy()
        assert a.size == self.cells
        b = np.empty_like(a)
        for _ in range(int(steps)):
            lib().orc_compact_step(self._h, _ptr(a), _ptr(b), int(rule))
            a, b = b, a
        return a
