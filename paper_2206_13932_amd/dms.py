"""ctypes binding of libdms.so (the C ABI in include/dms.h).

Argument marshalling only: every step of the pipeline runs in the HIP
library. torch provides device memory and the stream. If the library is not
built, importing the binding raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdms.so")

DMS_OK, DMS_E_INVAL, DMS_E_NAN, DMS_E_NOMEM, DMS_E_CAPACITY, DMS_E_HIP, DMS_E_STATE, DMS_E_INTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7
DMS_VIRTUAL_MAX = 1
BUF_RANK, BUF_GRADIENT, BUF_CRIT0, BUF_ARCS0, BUF_ARCS2, BUF_STATS, BUF_D1LEN = 0, 1, 2, 6, 7, 8, 9
# most contributions dms_scatter_grad_noalloc takes (its static scratch)
NOALLOC_MAX_CONTRIB = 1 << 22
# debug options of a context (dms_set_option)
OPT_D1_SMALL_PASSES, OPT_LOG_PASSES, OPT_D1_NO_SANDWICH, OPT_D1_NO_CACHE, OPT_D1_HEAP_KEYS = 1, 2, 3, 4, 5
_ERRNAMES = {-1: "DMS_E_INVAL", -2: "DMS_E_NAN", -3: "DMS_E_NOMEM", -4: "DMS_E_CAPACITY", -5: "DMS_E_HIP",
             -6: "DMS_E_STATE", -7: "DMS_E_INTERNAL"}


class DmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class GradientInfo(ctypes.Structure):
    _fields_ = [("n_crit", ctypes.c_int64 * 4)]


_p = ctypes.c_void_p


class DiagramOut(ctypes.Structure):
    _fields_ = [("pairs", _p * 3), ("cap", ctypes.c_int64 * 3), ("n", ctypes.c_int64 * 3),
                ("birth_vertex", _p * 3), ("death_vertex", _p * 3),
                ("birth_value", _p * 3), ("death_value", _p * 3)]


class Item(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("offset", ctypes.c_int64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("cross_x", ctypes.c_int32), ("cross_y", ctypes.c_int32), ("z_quantum", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class BatchOut(ctypes.Structure):
    _fields_ = [("pairs", _p * 3), ("cap", ctypes.c_int64 * 3), ("n", ctypes.c_int64 * 3),
                ("item_start", _p * 3)]


_lib = None


def load_library() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2206_13932_amd/build.py (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    i64, u32 = ctypes.c_int64, ctypes.c_uint32
    lib.dms_create.argtypes = [ctypes.POINTER(_p), ctypes.c_int, _p, ctypes.c_size_t]
    lib.dms_create.restype = ctypes.c_int
    lib.dms_destroy.argtypes = [_p]
    lib.dms_destroy.restype = None
    lib.dms_last_error.argtypes = [_p]
    lib.dms_last_error.restype = ctypes.c_char_p
    lib.dms_gradient.argtypes = [_p, _p, Grid, u32, ctypes.POINTER(GradientInfo)]
    lib.dms_gradient.restype = ctypes.c_int
    lib.dms_pairs_d0_d2.argtypes = [_p, _p, i64, ctypes.POINTER(i64), _p, i64, ctypes.POINTER(i64)]
    lib.dms_pairs_d0_d2.restype = ctypes.c_int
    lib.dms_pairs_d1.argtypes = [_p, _p, i64, ctypes.POINTER(i64)]
    lib.dms_pairs_d1.restype = ctypes.c_int
    lib.dms_diagram.argtypes = [_p, _p, Grid, u32, ctypes.POINTER(DiagramOut)]
    lib.dms_diagram.restype = ctypes.c_int
    lib.dms_d1_generators.argtypes = [_p, _p, i64, _p, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.dms_d1_generators.restype = ctypes.c_int
    lib.dms_debug_copy.argtypes = [_p, ctypes.c_int, _p, i64]
    lib.dms_debug_copy.restype = i64
    lib.dms_set_option.argtypes = [_p, ctypes.c_int32, i64]
    lib.dms_set_option.restype = ctypes.c_int
    lib.dms_stage_ms.argtypes = [_p, ctypes.POINTER(ctypes.c_float * 8)]
    lib.dms_stage_ms.restype = ctypes.c_int
    lib.dms_scatter_grad.argtypes = [_p, i64, _p, _p, i64, _p]
    lib.dms_scatter_grad.restype = ctypes.c_int
    lib.dms_scatter_grad_noalloc.argtypes = [_p, i64, _p, _p, i64, _p]
    lib.dms_scatter_grad_noalloc.restype = ctypes.c_int
    lib.dms_diagram_batch.argtypes = [_p, _p, _p, ctypes.c_int32, u32, ctypes.POINTER(BatchOpts),
                                      ctypes.POINTER(BatchOut)]
    lib.dms_diagram_batch.restype = ctypes.c_int
    lib.dms_batch_layout.argtypes = [_p, ctypes.c_int32, ctypes.POINTER(BatchOpts), ctypes.POINTER(ctypes.c_int32 * 3),
                                     _p]
    lib.dms_batch_layout.restype = ctypes.c_int
    lib.dms_batch_info.argtypes = [_p, ctypes.POINTER(ctypes.c_int64 * 8)]
    lib.dms_batch_info.restype = ctypes.c_int
    _lib = lib
    return lib


def _grid_of(field: torch.Tensor) -> Grid:
    """[nz, ny, nx] is a 3D grid (nz = 1: the 2D grid of the plane z = 0);
    [ny, nx] is a 2D grid too."""
    if field.dim() == 2:
        ny, nx = field.shape
        return Grid(nx, ny, 1)
    if field.dim() != 3:
        raise ValueError("field must be shaped [nz, ny, nx] (or [ny, nx] for a 2D grid)")
    nz, ny, nx = field.shape
    return Grid(nx, ny, nz)


def _check_field(field: torch.Tensor) -> torch.Tensor:
    if not field.is_cuda:
        raise ValueError("field must be a device tensor")
    if field.dtype != torch.float32:
        raise ValueError("field must be float32")
    return field.contiguous()


class Context:
    """One library context: owns the device state of the last field."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, hbm_budget: int = 0):
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _p()
        rc = self.lib.dms_create(ctypes.byref(h), device, _p(self.stream.cuda_stream), hbm_budget)
        if rc != DMS_OK:
            raise DmsError(rc, "dms_create failed")
        self.h = h
        self.n_crit = None
        self._caps = [0, 0, 0]

    def close(self):
        if getattr(self, "h", None):
            self.lib.dms_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, rc: int):
        raise DmsError(rc, self.lib.dms_last_error(self.h).decode())

    # ---- the four calls of the ABI ----
    def gradient(self, field: torch.Tensor, flags: int = DMS_VIRTUAL_MAX):
        field = _check_field(field)
        info = GradientInfo()
        rc = self.lib.dms_gradient(self.h, _p(field.data_ptr()), _grid_of(field), flags, ctypes.byref(info))
        if rc != DMS_OK:
            self._raise(rc)
        self.n_crit = [int(x) for x in info.n_crit]
        return list(self.n_crit)

    def pairs_d0_d2(self):
        c = self.n_crit
        d0 = torch.empty((c[0] + 1, 2), dtype=torch.int64, device=self.device)
        d2 = torch.empty((c[2] + 1, 2), dtype=torch.int64, device=self.device)
        n0, n2 = ctypes.c_int64(), ctypes.c_int64()
        rc = self.lib.dms_pairs_d0_d2(self.h, _p(d0.data_ptr()), d0.shape[0], ctypes.byref(n0),
                                      _p(d2.data_ptr()), d2.shape[0], ctypes.byref(n2))
        if rc != DMS_OK:
            self._raise(rc)
        return d0[: n0.value], d2[: n2.value]

    def pairs_d1(self):
        c = self.n_crit
        d1 = torch.empty((c[1] + 1, 2), dtype=torch.int64, device=self.device)
        n1 = ctypes.c_int64()
        rc = self.lib.dms_pairs_d1(self.h, _p(d1.data_ptr()), d1.shape[0], ctypes.byref(n1))
        if rc != DMS_OK:
            self._raise(rc)
        return d1[: n1.value]

    def d1_generators(self):
        """Persistent 1-cycle generators of the finite D1 pairs of the last
        single-field run: (offsets [n + 1], edges [E]) LongTensors on the
        device; cycle i = edges[offsets[i]:offsets[i + 1]] (edge ids,
        ascending) belongs to the i-th finite pair of pairs_d1 / diagram."""
        n, e = ctypes.c_int64(), ctypes.c_int64()
        rc = self.lib.dms_d1_generators(self.h, None, 0, None, 0, ctypes.byref(n), ctypes.byref(e))
        if rc not in (DMS_OK, DMS_E_CAPACITY):
            self._raise(rc)
        offsets = torch.empty(n.value + 1, dtype=torch.int64, device=self.device)
        edges = torch.empty(max(e.value, 1), dtype=torch.int64, device=self.device)
        rc = self.lib.dms_d1_generators(self.h, _p(offsets.data_ptr()), offsets.numel(), _p(edges.data_ptr()),
                                        edges.numel(), ctypes.byref(n), ctypes.byref(e))
        if rc != DMS_OK:
            self._raise(rc)
        return offsets, edges[: e.value]

    def diagram(self, field: torch.Tensor, flags: int = DMS_VIRTUAL_MAX, with_values: bool = False):
        """Whole pipeline in one call. Returns {0: pairs, 1: pairs, 2: pairs}
        (LongTensor [n, 2] on the device) and, with_values, per dimension the
        birth/death highest vertices and their values."""
        field = _check_field(field)
        V = field.numel()
        for attempt in range(2):
            caps = [max(self._caps[d], V // 64 + 1024) for d in range(3)]
            out = DiagramOut()
            keep = []
            for d in range(3):
                t = torch.empty((caps[d], 2), dtype=torch.int64, device=self.device)
                keep.append(t)
                out.pairs[d] = t.data_ptr()
                out.cap[d] = caps[d]
                if with_values:
                    bv = torch.empty(caps[d], dtype=torch.int64, device=self.device)
                    dv = torch.empty(caps[d], dtype=torch.int64, device=self.device)
                    bf = torch.empty(caps[d], dtype=torch.float32, device=self.device)
                    df = torch.empty(caps[d], dtype=torch.float32, device=self.device)
                    keep += [bv, dv, bf, df]
                    out.birth_vertex[d], out.death_vertex[d] = bv.data_ptr(), dv.data_ptr()
                    out.birth_value[d], out.death_value[d] = bf.data_ptr(), df.data_ptr()
            rc = self.lib.dms_diagram(self.h, _p(field.data_ptr()), _grid_of(field), flags, ctypes.byref(out))
            if rc == DMS_E_CAPACITY and attempt == 0:
                self._caps = [int(out.n[d] * 1.25) + 16 for d in range(3)]
                continue
            if rc != DMS_OK:
                self._raise(rc)
            res = {}
            stride = 5 if with_values else 1
            for d in range(3):
                n = int(out.n[d])
                entry = keep[d * stride][:n]
                if with_values:
                    bv, dv, bf, df = keep[d * stride + 1: d * stride + 5]
                    entry = {"pairs": entry, "birth_vertex": bv[:n], "death_vertex": dv[:n],
                             "birth_value": bf[:n], "death_value": df[:n]}
                res[d] = entry
            return res
        raise DmsError(DMS_E_CAPACITY, "output capacity")

    # ---- inspection for tests ----
    def debug(self, what: int, dtype=np.uint32) -> np.ndarray:
        n = self.lib.dms_debug_copy(self.h, what, None, 0)
        if n < 0:
            self._raise(int(n))
        buf = np.empty(n, dtype=np.uint8)
        r = self.lib.dms_debug_copy(self.h, what, buf.ctypes.data_as(_p), n)
        if r < 0:
            self._raise(int(r))
        return buf.view(dtype)

    def scatter_grad(self, vertex: torch.Tensor, grad: torch.Tensor, nvert: int) -> torch.Tensor:
        """Deterministic scatter-add: out[v] = sum of grad[i] with vertex[i] == v
        (in increasing i), zero elsewhere; a float32 device tensor [nvert]."""
        vertex = vertex.to(device=self.device, dtype=torch.int64).contiguous()
        grad = grad.to(device=self.device, dtype=torch.float32).contiguous()
        if vertex.shape != grad.shape or vertex.dim() != 1:
            raise ValueError("vertex and grad must be 1-d tensors of the same length")
        out = torch.empty(nvert, dtype=torch.float32, device=self.device)
        rc = self.lib.dms_scatter_grad(self.h, vertex.numel(), _p(vertex.data_ptr()), _p(grad.data_ptr()), nvert,
                                       _p(out.data_ptr()))
        if rc != DMS_OK:
            self._raise(rc)
        return out

    def diagram_batch(self, fields, cross=(0, 0), z_quantum: int = 0, use_graph: bool = False,
                      flags: int = DMS_VIRTUAL_MAX):
        """Diagrams of several float32 device fields [nz, ny, nx] in one pipeline
        run. Returns a list with one {0, 1, 2: pairs} per field, as diagram()."""
        fields = [_check_field(f) for f in fields]
        n = len(fields)
        items = (Item * n)()
        off = 0
        for i, f in enumerate(fields):
            nz, ny, nx = f.shape
            items[i].nx, items[i].ny, items[i].nz, items[i].offset = nx, ny, nz, off
            off += f.numel()
        packed = torch.cat([f.reshape(-1) for f in fields]) if n > 1 else fields[0].reshape(-1)
        opts = BatchOpts(int(cross[0]), int(cross[1]), int(z_quantum), 1 if use_graph else 0)
        starts = [np.zeros(n + 1, dtype=np.int64) for _ in range(3)]
        caps = [max(c, off // 8 + 1024) for c in getattr(self, "_bcaps", [0, 0, 0])]
        for attempt in range(2):
            out = BatchOut()
            bufs = []
            for d in range(3):
                t = torch.empty((caps[d], 2), dtype=torch.int64, device=self.device)
                bufs.append(t)
                out.pairs[d] = t.data_ptr()
                out.cap[d] = caps[d]
                out.item_start[d] = starts[d].ctypes.data
            rc = self.lib.dms_diagram_batch(self.h, _p(packed.data_ptr()), ctypes.cast(items, _p), n, flags,
                                            ctypes.byref(opts), ctypes.byref(out))
            if rc == DMS_E_CAPACITY and attempt == 0:
                caps = [int(out.n[d] * 1.25) + 16 for d in range(3)]
                self._bcaps = caps
                continue
            if rc != DMS_OK:
                self._raise(rc)
            return [{d: bufs[d][int(starts[d][i]): int(starts[d][i + 1])] for d in range(3)} for i in range(n)]
        raise DmsError(DMS_E_CAPACITY, "output capacity")

    def scatter_grad_noalloc(self, vertex: torch.Tensor, grad: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """dms_scatter_grad_noalloc into a caller-owned float32 tensor out
        (nvert = out.numel()): no device allocation in the library; at most
        NOALLOC_MAX_CONTRIB contributions."""
        vertex = vertex.to(device=self.device, dtype=torch.int64).contiguous()
        grad = grad.to(device=self.device, dtype=torch.float32).contiguous()
        assert out.dtype == torch.float32 and out.is_contiguous() and out.device == vertex.device
        rc = self.lib.dms_scatter_grad_noalloc(self.h, vertex.numel(), _p(vertex.data_ptr()), _p(grad.data_ptr()),
                                               out.numel(), _p(out.data_ptr()))
        if rc != DMS_OK:
            self._raise(rc)
        return out

    def batch_info(self):
        arr = (ctypes.c_int64 * 8)()
        self.lib.dms_batch_info(self.h, ctypes.byref(arr))
        return list(arr)

    def set_option(self, option: int, value: int = 1):
        """Debug and ablation options (OPT_D1_SMALL_PASSES, OPT_LOG_PASSES,
        OPT_D1_NO_SANDWICH, OPT_D1_NO_CACHE, OPT_D1_HEAP_KEYS); they change how
        D1 splits, logs or repeats its work, never a result."""
        rc = self.lib.dms_set_option(self.h, int(option), int(value))
        if rc != DMS_OK:
            self._raise(rc)

    def stage_ms(self):
        arr = (ctypes.c_float * 8)()
        self.lib.dms_stage_ms(self.h, ctypes.byref(arr))
        return list(arr)


def batch_layout(shapes, cross=(0, 0), z_quantum: int = 0):
    """Host-only layout of a batch: ((X, Y, Z), origins [n, 3]) for grid shapes
    [(nz, ny, nx), ...]."""
    lib = load_library()
    n = len(shapes)
    items = (Item * n)()
    for i, (nz, ny, nx) in enumerate(shapes):
        items[i].nx, items[i].ny, items[i].nz = nx, ny, nz
    opts = BatchOpts(int(cross[0]), int(cross[1]), int(z_quantum), 0)
    dims = (ctypes.c_int32 * 3)()
    origins = np.zeros((n, 3), dtype=np.int32)
    rc = lib.dms_batch_layout(ctypes.cast(items, _p), n, ctypes.byref(opts), ctypes.byref(dims), origins.ctypes.data)
    if rc != DMS_OK:
        raise DmsError(rc, "dms_batch_layout failed")
    return (dims[0], dims[1], dims[2]), origins


def diagram(field: torch.Tensor, ctx: Context | None = None):
    """Persistence diagrams {0, 1, 2} of a float32 device field [nz, ny, nx]."""
    own = ctx is None
    ctx = ctx or Context(field.device.index or 0)
    try:
        return ctx.diagram(field)
    finally:
        if own:
            ctx.close()
