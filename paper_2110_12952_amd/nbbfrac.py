"""Python binding of libnbbfrac (include/nbbfrac.h): argument marshalling only.

Device memory and streams come from PyTorch-ROCm (torch.cuda tensors and the
current stream); every step of the computation runs in the library's HIP
kernels.  The library is loaded from this package directory; if it is missing
the import of the binding fails with an error that says how to build it --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# NBB_LIBRARY may name another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("NBB_LIBRARY") or os.path.join(HERE, "libnbbfrac.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nbbfrac.h")

NBB_OK, NBB_E_INVALID, NBB_E_RANGE, NBB_E_NOMEM, NBB_E_DEVICE = range(5)
NBB_OUTSIDE = 0xFFFFFFFF
NBB_RULE_B3S23 = (1 << 3) | ((1 << 2 | 1 << 3) << 16)
NBB_RULE_VON_NEUMANN = 1 << 31
NBB_BATCH_NO_RESIDENT = 1  # nbb_batch_create_ex: small instances stepped by the group launches too
NBB_BATCH_RESIDENT = 2     # nbb_batch_create_ex: every small instance stepped in LDS
(STRATEGY_AUTO, STRATEGY_TILED, STRATEGY_DIRECT, STRATEGY_TILED_WAVE, STRATEGY_TILED_BOX, STRATEGY_TEMPORAL,
 STRATEGY_TILED_EDGE) = range(7)
MAP_LUT, MAP_DIGITS, MAP_MFMA = 0, 1, 2


class NbbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


STATUS_NAMES = {0: "NBB_OK", 1: "NBB_E_INVALID", 2: "NBB_E_RANGE", 3: "NBB_E_NOMEM", 4: "NBB_E_DEVICE"}


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("cells", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
                ("k", ctypes.c_uint32), ("s", ctypes.c_uint32), ("r", ctypes.c_uint32),
                ("strategy", ctypes.c_uint32), ("tile_level", ctypes.c_uint32),
                ("tile_side", ctypes.c_uint32), ("halo_cells", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("bbox_pitch", ctypes.c_uint64),
                ("device_table_bytes", ctypes.c_uint64), ("box_low_side", ctypes.c_uint32),
                ("box_high_side", ctypes.c_uint32), ("tiled_form", ctypes.c_uint32),
                ("temporal_depth", ctypes.c_uint32)]


class TemporalView(ctypes.Structure):
    _fields_ = [("tile_level", ctypes.c_uint32), ("tile_side", ctypes.c_uint32), ("tile_cells", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("box_side", ctypes.c_uint32), ("box_pitch", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("halo_count", ctypes.c_uint32), ("tiles", ctypes.c_uint64),
                ("self_", ctypes.POINTER(ctypes.c_uint32)), ("halo", ctypes.POINTER(ctypes.c_uint32)),
                ("nbr", ctypes.POINTER(ctypes.c_uint32))]


class PlanView(ctypes.Structure):
    _fields_ = [("tile_level", ctypes.c_uint32), ("tile_side", ctypes.c_uint32),
                ("tile_cells", ctypes.c_uint32), ("block_level", ctypes.c_uint32),
                ("block_side", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("halo_count", ctypes.c_uint32), ("box_pitch", ctypes.c_uint32),
                ("box_rows", ctypes.c_uint32), ("lds_bytes", ctypes.c_uint32),
                ("tiles", ctypes.c_uint64),
                ("lut0", ctypes.POINTER(ctypes.c_uint16)), ("lut1", ctypes.POINTER(ctypes.c_uint16)),
                ("halo_src", ctypes.POINTER(ctypes.c_uint32)), ("halo_dst", ctypes.POINTER(ctypes.c_uint32)),
                ("nbr", ctypes.POINTER(ctypes.c_uint32)),
                ("edge_ok", ctypes.c_uint32), ("edge_grid", ctypes.c_uint32), ("edge_records", ctypes.c_uint32),
                ("edge_rec_bytes", ctypes.c_uint32), ("edge_halo_count", ctypes.c_uint32),
                ("edge_nsrc", ctypes.c_uint32),
                ("edge_unpack", ctypes.c_uint32 * 8), ("edge_pack", ctypes.c_uint32 * 8),
                ("edge_blk", ctypes.POINTER(ctypes.c_uint32)), ("edge_halo", ctypes.POINTER(ctypes.c_uint32))]


class BatchInfo(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_uint32), ("groups", ctypes.c_uint32), ("direct", ctypes.c_uint32),
                ("resident", ctypes.c_uint32), ("cells", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("device_table_bytes", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32p = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    st = ctypes.c_int
    L.nbb_create.argtypes = [u32, u32, vp, u32, ctypes.POINTER(vp)]
    L.nbb_create.restype = st
    L.nbb_destroy.argtypes = [vp]
    L.nbb_destroy.restype = None
    L.nbb_query.argtypes = [vp, ctypes.POINTER(Info)]
    L.nbb_query.restype = st
    L.nbb_configure.argtypes = [vp, u32, u32]
    L.nbb_configure.restype = st
    L.nbb_lambda.argtypes = [vp, vp, u64, vp, vp, vp]
    L.nbb_lambda.restype = st
    L.nbb_nu.argtypes = [vp, vp, vp, u64, vp, vp]
    L.nbb_nu.restype = st
    L.nbb_lambda_method.argtypes = [vp, u32, vp, u64, vp, vp, vp]
    L.nbb_lambda_method.restype = st
    L.nbb_nu_method.argtypes = [vp, u32, vp, vp, u64, vp, vp]
    L.nbb_nu_method.restype = st
    L.nbb_init_compact.argtypes = [vp, vp, u64, u64, ctypes.c_double, vp]
    L.nbb_init_compact.restype = st
    L.nbb_init_bbox.argtypes = [vp, vp, u64, u64, u64, ctypes.c_double, vp]
    L.nbb_init_bbox.restype = st
    L.nbb_step_compact.argtypes = [vp, vp, vp, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_step_compact.restype = st
    L.nbb_step_bbox.argtypes = [vp, vp, vp, u64, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_step_bbox.restype = st
    L.nbb_step_lambda.argtypes = [vp, vp, vp, u64, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_step_lambda.restype = st
    L.nbb_blocked_bytes.argtypes = [vp]
    L.nbb_blocked_bytes.restype = u64
    L.nbb_blocked_from_compact.argtypes = [vp, vp, vp, u64, vp]
    L.nbb_blocked_from_compact.restype = st
    L.nbb_blocked_to_compact.argtypes = [vp, vp, u64, vp, vp]
    L.nbb_blocked_to_compact.restype = st
    L.nbb_step_blocked.argtypes = [vp, vp, vp, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_step_blocked.restype = st
    L.nbb_packed_bytes.argtypes = [vp]
    L.nbb_packed_bytes.restype = u64
    L.nbb_pack.argtypes = [vp, vp, vp, u64, vp]
    L.nbb_pack.restype = st
    L.nbb_unpack.argtypes = [vp, vp, u64, vp, vp]
    L.nbb_unpack.restype = st
    L.nbb_step_packed.argtypes = [vp, vp, vp, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_step_packed.restype = st
    L.nbb_expand.argtypes = [vp, vp, vp, u64, u64, vp]
    L.nbb_expand.restype = st
    L.nbb_gather.argtypes = [vp, vp, u64, vp, u64, vp]
    L.nbb_gather.restype = st
    L.nbb_autotune.argtypes = [vp, vp, vp, u64, u32, u32, vp, ctypes.POINTER(Info)]
    L.nbb_autotune.restype = st
    L.nbb_batch_create.argtypes = [vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.nbb_batch_create.restype = st
    L.nbb_batch_create_ex.argtypes = [vp, vp, u32, u32, vp, ctypes.POINTER(vp)]
    L.nbb_batch_create_ex.restype = st
    L.nbb_batch_destroy.argtypes = [vp]
    L.nbb_batch_destroy.restype = None
    L.nbb_batch_query.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.nbb_batch_query.restype = st
    L.nbb_batch_step.argtypes = [vp, vp, vp, u64, u32, u32, ctypes.POINTER(ctypes.c_int), vp]
    L.nbb_batch_step.restype = st
    L.nbb_batch_step_each.argtypes = [vp, vp, vp, u64, vp, u32, vp]
    L.nbb_batch_step_each.restype = st
    L.nbb_batch_step_each_noalloc.argtypes = [vp, vp, u32, vp, vp, u64, vp, u32, vp]
    L.nbb_batch_step_each_noalloc.restype = st
    L.nbb_bbox_pitch.argtypes = [vp]
    L.nbb_bbox_pitch.restype = u64
    L.nbb_last_error.restype = ctypes.c_char_p
    L.nbb_status_string.argtypes = [st]
    L.nbb_status_string.restype = ctypes.c_char_p
    L.nbb_plan_build.argtypes = [u32, u32, vp, u32, u32, ctypes.POINTER(vp), ctypes.POINTER(PlanView)]
    L.nbb_plan_build.restype = st
    L.nbb_plan_free.argtypes = [vp]
    L.nbb_plan_free.restype = None
    L.nbb_batch_autotune.argtypes = [vp, vp, u32, vp, vp, u64, u32, u32, u32, vp]
    L.nbb_batch_autotune.restype = st
    L.nbb_configure_temporal.argtypes = [vp, u32, u32]
    L.nbb_configure_temporal.restype = st
    L.nbb_temporal_plan_build.argtypes = [u32, u32, vp, u32, u32, u32, u32, ctypes.POINTER(vp),
                                          ctypes.POINTER(TemporalView)]
    L.nbb_temporal_plan_build.restype = st
    L.nbb_temporal_plan_free.argtypes = [vp]
    L.nbb_temporal_plan_free.restype = None
    _lib = L
    return L


def header_symbols() -> list:
    """Names of the functions include/nbbfrac.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbb_[a-z_0-9]+)\s*\(", text)))


def _check(status: int) -> None:
    if status != NBB_OK:
        raise NbbError(status, lib().nbb_last_error().decode())


def _offsets_array(offsets: Sequence[Tuple[int, int]]) -> np.ndarray:
    return np.ascontiguousarray([c for o in offsets for c in o], dtype=np.int32)


def temporal_plan_tables(s: int, offsets: Sequence[Tuple[int, int]], r: int, tile_level: int, depth: int,
                         lds_limit: int = 0) -> dict:
    """Host-side temporal plan (nbb_temporal_plan_build; no device) as numpy arrays."""
    offs = _offsets_array(offsets)
    h = ctypes.c_void_p()
    v = TemporalView()
    _check(lib().nbb_temporal_plan_build(len(offsets), s, offs.ctypes.data, r, tile_level, depth, lds_limit,
                                         ctypes.byref(h), ctypes.byref(v)))
    try:
        out = {"tile_level": v.tile_level, "tile_side": v.tile_side, "K": v.tile_cells, "depth": v.depth,
               "B": v.box_side, "P": v.box_pitch, "lds_bytes": v.lds_bytes, "tiles": int(v.tiles)}
        out["self"] = np.ctypeslib.as_array(v.self_, (v.tile_cells,)).copy()
        out["halo"] = (np.ctypeslib.as_array(v.halo, (2 * v.halo_count,)).copy() if v.halo_count
                       else np.zeros(0, np.uint32))
        out["nbr"] = np.ctypeslib.as_array(v.nbr, (int(v.tiles) * 8,)).copy()
    finally:
        lib().nbb_temporal_plan_free(h)
    return out


def plan_tables(s: int, offsets: Sequence[Tuple[int, int]], r: int, tile_level: int = 0) -> dict:
    """Host-side tile plan (no device involved) as numpy arrays."""
    offs = _offsets_array(offsets)
    h = ctypes.c_void_p()
    v = PlanView()
    _check(lib().nbb_plan_build(len(offsets), s, offs.ctypes.data, r, tile_level, ctypes.byref(h),
                                ctypes.byref(v)))
    try:
        out = {f: getattr(v, f) for f in ("tile_level", "tile_side", "tile_cells", "block_level",
                                          "block_side", "blocks", "halo_count",
                                          "box_pitch", "box_rows", "lds_bytes", "tiles")}
        out["lut0"] = np.ctypeslib.as_array(v.lut0, (v.tile_cells,)).copy()
        out["lut1"] = np.ctypeslib.as_array(v.lut1, (v.blocks,)).copy()
        out["halo_src"] = np.ctypeslib.as_array(v.halo_src, (v.halo_count,)).copy() if v.halo_count else \
            np.zeros(0, np.uint32)
        out["halo_dst"] = np.ctypeslib.as_array(v.halo_dst, (v.halo_count,)).copy() if v.halo_count else \
            np.zeros(0, np.uint32)
        out["nbr"] = np.ctypeslib.as_array(v.nbr, (int(v.tiles) * 8,)).copy()
        out["edge_ok"] = bool(v.edge_ok)
        if v.edge_ok:
            for f in ("edge_grid", "edge_records", "edge_rec_bytes", "edge_halo_count", "edge_nsrc"):
                out[f] = getattr(v, f)
            out["edge_unpack"] = np.array(list(v.edge_unpack), np.uint32)
            out["edge_pack"] = np.array(list(v.edge_pack), np.uint32)
            out["edge_blk"] = np.ctypeslib.as_array(v.edge_blk, (4 * v.blocks,)).copy()
            out["edge_halo"] = np.ctypeslib.as_array(v.edge_halo, (2 * v.edge_halo_count,)).copy() \
                if v.edge_halo_count else np.zeros(0, np.uint32)
        return out
    finally:
        lib().nbb_plan_free(h)


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_ptr(t, dtype_name: str, numel: Optional[int] = None) -> int:
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


class Fractal:
    """Descriptor of F^{k,s} at level r (nbb_create / nbb_destroy)."""

    def __init__(self, s: int, offsets: Sequence[Tuple[int, int]], r: int):
        offs = _offsets_array(offsets)
        h = ctypes.c_void_p()
        _check(lib().nbb_create(len(offsets), s, offs.ctypes.data, r, ctypes.byref(h)))
        self._h = h
        self.s, self.r, self.k = int(s), int(r), len(offsets)
        self.offsets = tuple((int(a), int(b)) for a, b in offsets)
        inf = self.info()
        self.n, self.cells, self.pitch = int(inf.n), int(inf.cells), int(inf.bbox_pitch)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().nbb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Info:
        inf = Info()
        _check(lib().nbb_query(self._h, ctypes.byref(inf)))
        return inf

    def configure(self, strategy: int = STRATEGY_AUTO, tile_level: int = 0) -> None:
        _check(lib().nbb_configure(self._h, strategy, tile_level))

    def configure_temporal(self, tile_level: int = 0, depth: int = 0) -> None:
        """Several generations per launch (nbb_configure_temporal; 0 = automatic)."""
        _check(lib().nbb_configure_temporal(self._h, tile_level, depth))

    def autotune(self, a, b, steps: int = 5, rule: int = NBB_RULE_B3S23, stream=None) -> Info:
        """Time each candidate plan on a and b (both overwritten) and keep the fastest."""
        inf = Info()
        _check(lib().nbb_autotune(self._h, _dev_ptr(a, "uint8", self.cells), _dev_ptr(b, "uint8", self.cells),
                                  self.cells, int(steps), int(rule), _stream(stream), ctypes.byref(inf)))
        return inf

    # ---- maps ------------------------------------------------------------
    def lam(self, idx=None, count: Optional[int] = None, out=None, stream=None, method: int = MAP_LUT):
        import torch
        if idx is not None:
            count = idx.numel()
            ip = _dev_ptr(idx, "int32") if idx.dtype == torch.int32 else _dev_ptr(idx, "uint32")
        else:
            ip = None
            count = self.cells if count is None else int(count)
        dev = torch.device("cuda", torch.cuda.current_device())
        x, y = out if out is not None else (torch.empty(count, dtype=torch.int32, device=dev),
                                             torch.empty(count, dtype=torch.int32, device=dev))
        _check(lib().nbb_lambda_method(self._h, method, ip, count, _dev_ptr(x, "int32", count),
                                       _dev_ptr(y, "int32", count), _stream(stream)))
        return x, y

    def nu(self, x, y, out=None, stream=None, method: int = MAP_LUT):
        import torch
        count = x.numel()
        idx = out if out is not None else torch.empty(count, dtype=torch.int32, device=x.device)
        _check(lib().nbb_nu_method(self._h, method, _dev_ptr(x, "int32", count), _dev_ptr(y, "int32", count),
                                   count, _dev_ptr(idx, "int32", count), _stream(stream)))
        return idx  # int32 view of the uint32 result: NBB_OUTSIDE reads as -1

    # ---- states ----------------------------------------------------------
    def new_compact(self):
        import torch
        return torch.empty(self.cells, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))

    def new_bbox(self):
        import torch
        return torch.empty((self.n, self.pitch), dtype=torch.uint8,
                           device=torch.device("cuda", torch.cuda.current_device()))

    def init_compact(self, seed: int, p: float, out=None, stream=None):
        st = self.new_compact() if out is None else out
        _check(lib().nbb_init_compact(self._h, _dev_ptr(st, "uint8", self.cells), self.cells,
                                      seed & (2 ** 64 - 1), float(p), _stream(stream)))
        return st

    def init_bbox(self, seed: int, p: float, out=None, stream=None):
        st = self.new_bbox() if out is None else out
        pitch = st.shape[-1] if st.dim() == 2 else self.pitch
        _check(lib().nbb_init_bbox(self._h, _dev_ptr(st, "uint8"), pitch, st.numel(), seed & (2 ** 64 - 1),
                                   float(p), _stream(stream)))
        return st

    def step_compact(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        """Returns the tensor (a or b) that holds the result."""
        res = ctypes.c_int(0)
        _check(lib().nbb_step_compact(self._h, _dev_ptr(a, "uint8", self.cells), _dev_ptr(b, "uint8", self.cells),
                                      self.cells, int(steps), int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    def step_bbox(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        res = ctypes.c_int(0)
        pitch = a.shape[-1]
        _check(lib().nbb_step_bbox(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), pitch, a.numel(),
                                   int(steps), int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    def step_lambda(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        """The lambda approach on box buffers (threads over fractal cells)."""
        res = ctypes.c_int(0)
        pitch = a.shape[-1]
        _check(lib().nbb_step_lambda(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), pitch, a.numel(),
                                     int(steps), int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    # ---- blocked layout (one S x S square per tile) ------------------------
    def blocked_bytes(self) -> int:
        return int(lib().nbb_blocked_bytes(self._h))

    def to_blocked(self, compact, out=None, stream=None):
        import torch
        n = self.blocked_bytes()
        blk = torch.empty(max(n, 1), dtype=torch.uint8, device=compact.device)[:n] if out is None else out
        _check(lib().nbb_blocked_from_compact(self._h, _dev_ptr(compact, "uint8", self.cells), _dev_ptr(blk, "uint8"),
                                              blk.numel(), _stream(stream)))
        return blk

    def from_blocked(self, blocked, out=None, stream=None):
        c = self.new_compact() if out is None else out
        _check(lib().nbb_blocked_to_compact(self._h, _dev_ptr(blocked, "uint8"), blocked.numel(),
                                            _dev_ptr(c, "uint8", self.cells), _stream(stream)))
        return c

    def step_blocked(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        res = ctypes.c_int(0)
        _check(lib().nbb_step_blocked(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(), int(steps),
                                      int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    # ---- bit-packed state (cell i = bit i % 8 of byte i / 8) ---------------
    def packed_bytes(self) -> int:
        return int(lib().nbb_packed_bytes(self._h))

    def new_packed(self):
        import torch
        return torch.zeros(self.packed_bytes(), dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))

    def pack(self, compact, out=None, stream=None):
        pk = self.new_packed() if out is None else out
        _check(lib().nbb_pack(self._h, _dev_ptr(compact, "uint8", self.cells), _dev_ptr(pk, "uint8"), pk.numel(),
                              _stream(stream)))
        return pk

    def unpack(self, packed, out=None, stream=None):
        c = self.new_compact() if out is None else out
        _check(lib().nbb_unpack(self._h, _dev_ptr(packed, "uint8"), packed.numel(), _dev_ptr(c, "uint8", self.cells),
                                _stream(stream)))
        return c

    def step_packed(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        res = ctypes.c_int(0)
        _check(lib().nbb_step_packed(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(), int(steps),
                                     int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    def expand(self, compact, out=None, stream=None):
        box = self.new_bbox() if out is None else out
        _check(lib().nbb_expand(self._h, _dev_ptr(compact, "uint8", self.cells), _dev_ptr(box, "uint8"),
                                box.shape[-1], box.numel(), _stream(stream)))
        return box

    def gather(self, box, out=None, stream=None):
        c = self.new_compact() if out is None else out
        _check(lib().nbb_gather(self._h, _dev_ptr(box, "uint8"), box.shape[-1], _dev_ptr(c, "uint8", self.cells),
                                self.cells, _stream(stream)))
        return c


def shared_descriptors(specs: Sequence[Tuple[int, Sequence[Tuple[int, int]], int]]) -> list:
    """Descriptors for the instances (s, offsets, r) of a batch: one per
    distinct instance kind, shared by the instances of that kind.  Every
    descriptor of one fractal is configured to the automatic tile level of
    that fractal at its largest r (capped by its own r), so the batch steps
    all instances of a fractal with one launch per generation."""
    desc, top = {}, {}
    for s, offsets, r in specs:
        key = (int(s), tuple((int(a), int(b)) for a, b in offsets), int(r))
        if key not in desc:
            desc[key] = Fractal(key[0], key[1], key[2])
        fk = key[:2]
        if fk not in top or key[2] > top[fk][0]:
            top[fk] = (key[2], desc[key])
    for (s, offs, r), f in desc.items():
        big_r, big = top[(s, offs)]
        inf = big.info()
        if inf.strategy != STRATEGY_DIRECT and f.info().strategy != STRATEGY_DIRECT:
            f.configure(int(inf.strategy), min(r, int(inf.tile_level)))
    return [desc[(int(s), tuple((int(a), int(b)) for a, b in o), int(r))] for s, o, r in specs]


def pack_offsets(cells: Sequence[int]) -> Tuple[list, int]:
    """Consecutive 16-byte-aligned arena offsets for states of these sizes,
    and the arena length they need."""
    offs, o = [], 0
    for c in cells:
        offs.append(o)
        o += (int(c) + 15) & ~15
    return offs, max(o, 16)


NBB_TUNE_NO_CACHE = 1


def batch_autotune(fractals: Sequence["Fractal"], offsets: Sequence[int], a, b, steps: int = 10,
                   rule: int = NBB_RULE_B3S23, use_cache: bool = True, stream=None) -> None:
    """nbb_batch_autotune: per fractal of the batch, time the candidate tile
    plans on its instances (states in arenas a and b, which are stepped) and
    configure its descriptors to the fastest."""
    if a.numel() != b.numel():
        raise ValueError("arenas differ in length")
    n = len(fractals)
    hs = (ctypes.c_void_p * max(n, 1))(*[f._h.value for f in fractals])
    offs = (ctypes.c_uint64 * max(n, 1))(*[int(o) for o in offsets])
    _check(lib().nbb_batch_autotune(hs, offs, n, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(), int(steps),
                                    int(rule), 0 if use_cache else NBB_TUNE_NO_CACHE, _stream(stream)))


NOALLOC_SCRATCH_BYTES = 16 << 20  # NBB_NOALLOC_SCRATCH_BYTES


def batch_step_each_noalloc(fractals: Sequence["Fractal"], offsets: Sequence[int], a, b, steps: Sequence[int],
                            rule: int = NBB_RULE_B3S23, stream=None) -> None:
    """nbb_batch_step_each_noalloc: instance i (fractals[i], state at byte
    offsets[i] of both arenas) takes steps[i] generations, its result in b
    iff steps[i] is odd; the batch tables live in the library's static device
    array, so the call allocates no device memory."""
    if a.numel() != b.numel():
        raise ValueError("arenas differ in length")
    n = len(fractals)
    if len(offsets) != n or len(steps) != n:
        raise ValueError(f"expected {n} offsets and step counts")
    hs = (ctypes.c_void_p * max(n, 1))(*[f._h.value for f in fractals])
    offs = (ctypes.c_uint64 * max(n, 1))(*[int(o) for o in offsets])
    arr = np.ascontiguousarray(steps, dtype=np.uint32) if n else np.zeros(1, np.uint32)
    _check(lib().nbb_batch_step_each_noalloc(hs, offs, n, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(),
                                             arr.ctypes.data, int(rule), _stream(stream)))


class Batch:
    """Many automata stepped together (nbb_batch_create / nbb_batch_step).

    Instance i is the fractal fractals[i] with its state at byte offsets[i] of
    each arena (default: packed one after another).  The descriptors must stay
    alive and keep their configuration while the batch exists; the batch
    holds references to them.  resident: None = the library's choice, True =
    every small instance runs all generations in LDS, False = small instances
    go through the per-generation group launches like the rest."""

    def __init__(self, fractals: Sequence[Fractal], offsets: Optional[Sequence[int]] = None, stream=None,
                 resident: Optional[bool] = None):
        self.fractals = list(fractals)
        cells = [f.cells for f in self.fractals]
        if offsets is None:
            offsets, _ = pack_offsets(cells)
        self.offsets = [int(o) for o in offsets]
        self.cells = cells
        n = len(self.fractals)
        hs = (ctypes.c_void_p * max(n, 1))(*[f._h.value for f in self.fractals])
        offs = (ctypes.c_uint64 * max(n, 1))(*self.offsets)
        h = ctypes.c_void_p()
        flags = 0 if resident is None else (NBB_BATCH_RESIDENT if resident else NBB_BATCH_NO_RESIDENT)
        _check(lib().nbb_batch_create_ex(hs, offs, n, flags, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.arena_bytes = int(self.info().arena_bytes)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().nbb_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> BatchInfo:
        inf = BatchInfo()
        _check(lib().nbb_batch_query(self._h, ctypes.byref(inf)))
        return inf

    def new_arena(self):
        import torch
        return torch.zeros(max(self.arena_bytes, 16), dtype=torch.uint8,
                           device=torch.device("cuda", torch.cuda.current_device()))

    def state(self, arena, i: int):
        """Instance i's state inside an arena (a view)."""
        return arena[self.offsets[i]:self.offsets[i] + self.cells[i]]

    def step(self, a, b, steps: int, rule: int = NBB_RULE_B3S23, stream=None):
        """Returns the arena (a or b) that holds the result."""
        if a.numel() != b.numel():
            raise ValueError("arenas differ in length")
        res = ctypes.c_int(0)
        _check(lib().nbb_batch_step(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(), int(steps),
                                    int(rule), ctypes.byref(res), _stream(stream)))
        return b if res.value else a

    def step_each(self, a, b, steps: Sequence[int], rule: int = NBB_RULE_B3S23, stream=None) -> None:
        """Instance i takes steps[i] generations; its result is in b iff steps[i] is odd."""
        if a.numel() != b.numel():
            raise ValueError("arenas differ in length")
        n = len(self.fractals)
        if len(steps) != n:
            raise ValueError(f"expected {n} step counts")
        arr = np.ascontiguousarray(steps, dtype=np.uint32) if n else np.zeros(1, np.uint32)
        _check(lib().nbb_batch_step_each(self._h, _dev_ptr(a, "uint8"), _dev_ptr(b, "uint8"), a.numel(),
                                         arr.ctypes.data, int(rule), _stream(stream)))
