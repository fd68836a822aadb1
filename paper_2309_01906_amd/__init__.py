"""Hierarchical nested reductions on MI355X (gfx950): Python binding of libhp.so.

Argument marshalling only: every step of the reduction runs in the HIP kernels of
``libhp.so``; torch supplies device memory and streams.  The library must have
been built (``python paper_2309_01906_amd/build.py`` or ``__graft_entry__.build()``);
without it every call raises ``RuntimeError`` -- there is no fallback path.

Level maps are written per loop level as a string of scope letters, outermost
first: ``"G"`` grid (workgroups), ``"W"`` workgroup (waves), ``"V"`` wavefront
(lanes), ``"L"`` lane (serial), e.g. ``["G", "W", "VL"]``; optionally with unit
counts: ``("GW", {"G": 16, "W": 8})``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhp.so")

MAX_DEPTH = 8
NONE, SUM, MIN, MAX, ARGMIN, ARGMAX, PROD = 0, 1, 2, 3, 4, 5, 6
I32, F32, BF16, I64, F64, AFFINE64, MAT2X2_64 = 0, 1, 2, 3, 4, 5, 6
# uint64 words per element of the ordered-product types (tensors hold them as int64)
WIDTH = {AFFINE64: 2, MAT2X2_64: 4}
SCOPE = {"G": 1, "W": 2, "V": 4, "L": 8, "X": 16}
AXIS = {"G": 0, "W": 1, "V": 2}
FLAG_OUT_F32, FLAG_SCALAR, FLAG_NO_XCD, FLAG_GENERIC = 0x1, 0x2, 0x4, 0x10
OP_NAMES = {"NONE": NONE, "SUM": SUM, "MIN": MIN, "MAX": MAX, "ARGMIN": ARGMIN, "ARGMAX": ARGMAX, "PROD": PROD}
STATUS = ["HP_OK", "HP_EINVAL", "HP_EUNSUPPORTED", "HP_ENOMEM", "HP_EDEVICE", "HP_EAGAIN",
          "HP_ETOOBIG", "HP_ENOTREADY", "HP_ECANCELED", "HP_ESTATE"]


class HPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.status_name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{self.status_name}: {msg}")


class Nest(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("op", ctypes.c_int32 * MAX_DEPTH), ("extent", ctypes.c_int64 * MAX_DEPTH)]


class LevelMap(ctypes.Structure):
    _fields_ = [("scopes", ctypes.c_uint32 * MAX_DEPTH), ("units", (ctypes.c_uint32 * 3) * MAX_DEPTH)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("out_dtype", ctypes.c_int32), ("n_out", ctypes.c_int64),
                ("out_bytes", ctypes.c_size_t), ("in_elems", ctypes.c_int64), ("in_bytes", ctypes.c_size_t),
                ("grid", ctypes.c_int64), ("waves", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("gsplit", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t), ("lds_bytes", ctypes.c_size_t),
                ("scopes", ctypes.c_uint32 * MAX_DEPTH), ("units", (ctypes.c_uint32 * 3) * MAX_DEPTH),
                ("strips", ctypes.c_int64 * MAX_DEPTH), ("nseg", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("flat_block", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded libhp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2309_01906_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, st = ctypes.c_void_p, ctypes.c_int
        L.hp_plan_inspect.argtypes = [ctypes.POINTER(Nest), ctypes.POINTER(LevelMap), ctypes.c_uint32,
                                      ctypes.POINTER(PlanInfo)]
        L.hp_plan_inspect.restype = st
        L.hp_plan.argtypes = [ctypes.POINTER(Nest), ctypes.POINTER(LevelMap), ctypes.c_uint32,
                              ctypes.POINTER(vp)]
        L.hp_plan.restype = st
        L.hp_plan_info_get.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.hp_plan_info_get.restype = st
        L.hp_run.argtypes = [vp, vp, vp, vp]
        L.hp_run.restype = st
        L.hp_destroy.argtypes = [vp]
        L.hp_destroy.restype = st
        L.hp_last_error.argtypes = []
        L.hp_last_error.restype = ctypes.c_char_p
        L.hp_status_str.argtypes = [st]
        L.hp_status_str.restype = ctypes.c_char_p
        L.hp_stream_read.argtypes = [vp, ctypes.c_size_t, vp, ctypes.c_int32, vp]
        L.hp_stream_read.restype = st
        L.hp_reduce_static.argtypes = [ctypes.POINTER(Nest), ctypes.POINTER(LevelMap), ctypes.c_uint32, vp, vp, vp]
        L.hp_reduce_static.restype = st
        L.hp_xcd_ids.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t, vp]
        L.hp_xcd_ids.restype = st
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        raise HPError(status, lib().hp_last_error().decode(errors="replace"))


def _op(o):
    return OP_NAMES[o.upper()] if isinstance(o, str) else int(o)


def make_nest(extents, ops, dtype) -> Nest:
    n = Nest()
    if len(extents) != len(ops) or not 1 <= len(extents) <= MAX_DEPTH:
        raise ValueError("extents and ops must have the same length, 1..8")
    n.depth = len(extents)
    n.dtype = int(dtype)
    for i, (e, o) in enumerate(zip(extents, ops)):
        n.extent[i] = int(e)
        n.op[i] = _op(o)
    return n


def make_map(level_map) -> LevelMap | None:
    if level_map is None:
        return None
    m = LevelMap()
    for i, lv in enumerate(level_map):
        units = {}
        if isinstance(lv, (tuple, list)):
            lv, units = lv
        s = 0
        for ch in lv.replace("+", "").upper():
            s |= SCOPE[ch]
        m.scopes[i] = s
        for k, v in units.items():
            m.units[i][AXIS[k.upper()]] = int(v)
    return m


(KERNEL_LEAN, KERNEL_GENERIC4, KERNEL_GENERIC8, KERNEL_INT_FLAT, KERNEL_INT_SEG, KERNEL_INT_DEEP, KERNEL_ORDERED,
 KERNEL_INT_CHAIN) = range(8)
OP_TEMPLATE = {SUM: "1", MIN: "2", MAX: "3", ARGMIN: "4", ARGMAX: "5"}


def kernel_name(inf: PlanInfo, ops=None) -> str:
    """Symbol of the kernel hp_run launches for a plan (as profilers print it); the chain
    kernel's first template argument is the innermost operator (from ``ops``)."""
    c = inf.chunk
    if inf.kernel == KERNEL_ORDERED:
        return "hp::k_ordered<2, 8>" if inf.out_dtype == AFFINE64 else "hp::k_ordered<4, 4>"
    if inf.kernel == KERNEL_INT_CHAIN:
        return f"hp::k_nest_i32_chain<{OP_TEMPLATE[_op(ops[-1])] if ops else '?'}, {inf.nseg}>"
    if inf.kernel == KERNEL_INT_DEEP:
        bounds = "3, 4" if inf.depth <= 4 and inf.nseg <= 3 else f"{MAX_DEPTH}, {MAX_DEPTH}"
        return f"hp::k_nest_i32_deep<{c}, {bounds}>"
    if inf.kernel in (KERNEL_INT_FLAT, KERNEL_INT_SEG):
        kind = {KERNEL_INT_FLAT: "flat", KERNEL_INT_SEG: "seg"}[inf.kernel]
        return f"hp::k_nest_i32_{kind}<{c}>"
    t = "bf16" if inf.in_bytes == 2 * inf.in_elems else "f32"
    if inf.kernel == KERNEL_LEAN:
        return f"hp::k_nest_{t}_lean{'_flat' if inf.flat_block else ''}<{c}>"
    return f"hp::k_nest_{t}<{c}, {4 if inf.kernel == KERNEL_GENERIC4 else MAX_DEPTH}>"


def _info_dict(inf: PlanInfo, ops=None) -> dict:
    d = inf.depth
    names = "GWVL"
    return {
        "depth": d, "out_dtype": inf.out_dtype, "n_out": inf.n_out, "out_bytes": inf.out_bytes,
        "in_elems": inf.in_elems, "in_bytes": inf.in_bytes, "grid": inf.grid, "waves": inf.waves,
        "chunk": inf.chunk, "gsplit": inf.gsplit, "workspace_bytes": inf.workspace_bytes,
        "lds_bytes": inf.lds_bytes, "nseg": inf.nseg, "kernel": inf.kernel, "kernel_name": kernel_name(inf, ops),
        # a level on X reports "X" in place of the G it lowers to
        "map": [("X" if inf.scopes[i] & 16 else "") +
                "".join(names[b] for b in range(4) if inf.scopes[i] >> b & 1 and not (b == 0 and inf.scopes[i] & 16))
                for i in range(d)],
        "units": [tuple(inf.units[i][a] for a in range(3)) for i in range(d)],
        "strips": [inf.strips[i] for i in range(d)],
        "flat_block": inf.flat_block,
    }


def inspect(extents, ops, dtype, level_map=None, flags: int = 0) -> dict:
    """Plan without a device: validation and launch geometry (host only)."""
    n = make_nest(extents, ops, dtype)
    m = make_map(level_map)
    inf = PlanInfo()
    check(lib().hp_plan_inspect(ctypes.byref(n), ctypes.byref(m) if m is not None else None,
                                flags, ctypes.byref(inf)))
    return _info_dict(inf, ops)


def _torch():
    import torch
    return torch


def torch_out_dtype(code):
    torch = _torch()
    return {I32: torch.int32, I64: torch.int64, F32: torch.float32, F64: torch.float64,
            AFFINE64: torch.int64, MAT2X2_64: torch.int64}[code]


def dtype_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.float32:
        return F32
    if t.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return BF16
    raise TypeError(f"unsupported input dtype {t.dtype}")


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Plan:
    """A planned nest (hp_plan).  ``run`` launches it on a torch stream."""

    def __init__(self, extents, ops, dtype, level_map=None, flags: int = 0):
        self._h = ctypes.c_void_p()
        self.extents = tuple(int(e) for e in extents)
        self.ops = tuple(_op(o) for o in ops)
        self.dtype = int(dtype)
        n = make_nest(extents, ops, dtype)
        m = make_map(level_map)
        check(lib().hp_plan(ctypes.byref(n), ctypes.byref(m) if m is not None else None, flags,
                            ctypes.byref(self._h)))
        inf = PlanInfo()
        check(lib().hp_plan_info_get(self._h, ctypes.byref(inf)))
        self.info = _info_dict(inf, self.ops)

    def _out_shape(self):
        w = WIDTH.get(self.info["out_dtype"])
        return (self.info["n_out"],) if w is None else (self.info["n_out"], w)

    def empty_out(self, device):
        return _torch().empty(self._out_shape(), dtype=torch_out_dtype(self.info["out_dtype"]), device=device)

    def run(self, inp, out=None, stream=None):
        torch = _torch()
        if not inp.is_cuda:
            raise ValueError("input must be a device tensor")
        if not inp.is_contiguous():
            raise ValueError("input must be contiguous")
        w = WIDTH.get(self.dtype)
        if w is not None:  # ordered-product elements: int64 words, w per element
            if inp.dtype != torch.int64 or inp.numel() != self.info["in_elems"] * w:
                raise ValueError("input does not match the planned nest")
        elif inp.numel() != self.info["in_elems"] or dtype_of(inp) != self.dtype:
            raise ValueError("input does not match the planned nest")
        if out is None:
            out = self.empty_out(inp.device)
        if tuple(out.shape) != self._out_shape() or out.dtype != torch_out_dtype(self.info["out_dtype"]) \
                or not out.is_contiguous():
            raise ValueError("output does not match the plan")
        check(lib().hp_run(self._h, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                           _stream_handle(stream)))
        return out

    __call__ = run

    def close(self):
        if self._h:
            check(lib().hp_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.hp_destroy(self._h)
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


STENCIL_NO_XCD = 1


class Stencil:
    """`steps` five-point Jacobi sweeps of a 2-D float32 device array, tiled through
    LDS with a ghost surface (hp_stencil_*).  tile_rows (32 or 64) and
    sweeps_per_launch (1..8) default to the plan's choice; `info` holds what it chose."""

    def __init__(self, rows: int, cols: int, steps: int, c0: float, c1: float, tile_rows: int = 0,
                 sweeps_per_launch: int = 0, flags: int = 0):
        L = lib()
        L.hp_stencil_plan_ex.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_void_p)]
        L.hp_stencil_info.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int32)] * 4
        L.hp_stencil_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.hp_stencil_destroy.argtypes = [ctypes.c_void_p]
        self._h = ctypes.c_void_p()
        self.shape = (int(rows), int(cols))
        check(L.hp_stencil_plan_ex(int(rows), int(cols), int(steps), float(c0), float(c1), int(tile_rows),
                                   int(sweeps_per_launch), int(flags), ctypes.byref(self._h)))
        v = [ctypes.c_int32() for _ in range(4)]
        check(L.hp_stencil_info(self._h, *[ctypes.byref(x) for x in v]))
        self.info = dict(zip(("tile_rows", "tile_cols", "sweeps_per_launch", "launches"), (x.value for x in v)))

    def run(self, inp, out=None, stream=None):
        torch = _torch()
        if inp.dtype != torch.float32 or tuple(inp.shape) != self.shape or not inp.is_contiguous():
            raise ValueError("input must be a contiguous float32 array of the planned shape")
        if out is None:
            out = torch.empty_like(inp)
        if out.dtype != torch.float32 or tuple(out.shape) != self.shape or not out.is_contiguous():
            raise ValueError("output does not match the plan")
        check(lib().hp_stencil_run(self._h, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   _stream_handle(stream)))
        return out

    def close(self):
        if self._h:
            check(lib().hp_stencil_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def stream_read(inp, scratch, grid: int, stream=None):
    """Calibration read of the whole device tensor ``inp`` (hp_stream_read); ``scratch``
    is a float32 device tensor of at least ``grid`` elements."""
    if scratch.numel() < grid:
        raise ValueError("scratch needs one float per workgroup")
    check(lib().hp_stream_read(ctypes.c_void_p(inp.data_ptr()), inp.numel() * inp.element_size(),
                               ctypes.c_void_p(scratch.data_ptr()), int(grid), _stream_handle(stream)))


class LevelProps(ctypes.Structure):
    _fields_ = [("scope", ctypes.c_uint32), ("units", ctypes.c_int32), ("props", ctypes.c_uint32),
                ("shared_bytes", ctypes.c_int64)]


LP_BARRIER, LP_SHUFFLE, LP_LOCALMEM, LP_ATOMIC, LP_DYNAMIC, LP_LOCKSTEP, LP_SHARED_CACHE = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40)


def level_table():
    """hp_level_table: the device's hardware levels and their properties (host only).
    Returns (rows, fill_workgroups); a row is a dict with the scope letter."""
    L = lib()
    L.hp_level_table.argtypes = [ctypes.POINTER(LevelProps), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64)]
    L.hp_level_table.restype = ctypes.c_int
    rows = (LevelProps * 8)()
    n, fill = ctypes.c_int32(), ctypes.c_int64()
    check(L.hp_level_table(rows, 8, ctypes.byref(n), ctypes.byref(fill)))
    names = {v: k for k, v in SCOPE.items()}
    return ([{"scope": names[rows[i].scope], "units": rows[i].units, "props": rows[i].props,
              "shared_bytes": rows[i].shared_bytes} for i in range(n.value)], fill.value)


def xcd_ids(grid: int, threads: int = 256, lds_bytes: int = 0, stream=None):
    """hp_xcd_ids: the XCD that each of `grid` workgroups of `threads` threads runs on,
    as the hardware reports it (int32 device tensor of `grid` entries)."""
    torch = _torch()
    out = torch.full((int(grid),), -1, dtype=torch.int32, device="cuda")
    check(lib().hp_xcd_ids(ctypes.c_void_p(out.data_ptr()), int(grid), int(threads), int(lds_bytes),
                           _stream_handle(stream)))
    return out


def reduce(inp, extents, ops, level_map=None, flags: int = 0, stream=None):
    """One-shot: plan, run, return the output tensor (the plan is freed after the
    stream has finished with it)."""
    p = Plan(extents, ops, dtype_of(inp), level_map, flags)
    out = p.run(inp, stream=stream)
    _torch().cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    p.close()
    return out


def reduce_static(inp, out, extents, ops, level_map=None, flags: int = 0, stream=None):
    """hp_reduce_static: plan and run into ``out`` without allocating device memory
    (the library's static scratch holds the plan and partials).  Asynchronous on
    ``stream``; calls that overlap on one GPU race."""
    n = make_nest(extents, ops, dtype_of(inp))
    m = make_map(level_map)
    if not (inp.is_cuda and out.is_cuda and inp.is_contiguous() and out.is_contiguous()):
        raise ValueError("input and output must be contiguous device tensors")
    check(lib().hp_reduce_static(ctypes.byref(n), ctypes.byref(m) if m is not None else None, flags,
                                 ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 _stream_handle(stream)))
    return out


# ---------------------------------------------------------------------------
# batches and the autotuner

BATCH_GRAPH, BATCH_NO_TUNE = 0x100, 0x200
_batch_sigs_done = False


def _batch_sigs():
    global _batch_sigs_done
    if _batch_sigs_done:
        return
    L = lib()
    vp, st = ctypes.c_void_p, ctypes.c_int
    L.hp_batch_plan.argtypes = [ctypes.POINTER(Nest), ctypes.c_int64, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.hp_batch_info.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(PlanInfo)]
    L.hp_batch_plan_inspect.argtypes = [ctypes.POINTER(Nest), ctypes.c_int64, ctypes.c_uint32,
                                        ctypes.POINTER(PlanInfo)]
    L.hp_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    L.hp_batch_set_io.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.hp_batch_run.argtypes = [vp, vp]
    L.hp_batch_run_each.argtypes = [vp, vp, ctypes.c_int32]
    L.hp_batch_destroy.argtypes = [vp]
    L.hp_tune_nest.argtypes = [ctypes.POINTER(Nest), ctypes.c_uint32, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.hp_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.hp_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.hp_tune_cache_clear.argtypes = []
    L.hp_tune_cache_size.argtypes = [ctypes.POINTER(ctypes.c_int64)]
    for f in ("hp_batch_plan", "hp_batch_plan_inspect", "hp_batch_info", "hp_batch_stats", "hp_batch_set_io", "hp_batch_run",
              "hp_batch_run_each", "hp_batch_destroy", "hp_tune_nest", "hp_tune_cache_load",
              "hp_tune_cache_save", "hp_tune_cache_clear", "hp_tune_cache_size"):
        getattr(L, f).restype = st
    _batch_sigs_done = True


def batch_inspect(nests, flags: int = 0):
    """Host only: the plan of every nest of a batch (tuner cache included)."""
    _batch_sigs()
    arr = (Nest * len(nests))()
    for i, (ext, ops, dt) in enumerate(nests):
        arr[i] = make_nest(ext, ops, dt)
    infos = (PlanInfo * len(nests))()
    check(lib().hp_batch_plan_inspect(arr, len(nests), flags, infos))
    return [_info_dict(infos[i], nests[i][1]) for i in range(len(nests))]


class Batch:
    """hp_batch_*: many nests, one persistent launch per kernel family."""

    def __init__(self, nests, flags: int = 0):
        _batch_sigs()
        arr = (Nest * len(nests))()
        for i, (ext, ops, dt) in enumerate(nests):
            arr[i] = make_nest(ext, ops, dt)
        self._h = ctypes.c_void_p()
        self.n = len(nests)
        self._ops = [ops for _, ops, _ in nests]
        check(lib().hp_batch_plan(arr, self.n, flags, ctypes.byref(self._h)))

    def info(self, i: int) -> dict:
        inf = PlanInfo()
        check(lib().hp_batch_info(self._h, i, ctypes.byref(inf)))
        return _info_dict(inf, self._ops[i])

    def stats(self):
        a, b, w, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(lib().hp_batch_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(w), ctypes.byref(c)))
        return {"launches": a.value, "tasks": b.value, "workers": w.value, "bytes": c.value}

    def set_io_ptrs(self, in_ptrs, out_ptrs):
        ins = (ctypes.c_void_p * self.n)(*in_ptrs)
        outs = (ctypes.c_void_p * self.n)(*out_ptrs)
        check(lib().hp_batch_set_io(self._h, ins, outs))

    def set_io(self, ins, outs):
        self.set_io_ptrs([t.data_ptr() for t in ins], [t.data_ptr() for t in outs])

    def run(self, stream=None):
        check(lib().hp_batch_run(self._h, _stream_handle(stream)))

    def run_each(self, stream=None, graph: bool = False):
        check(lib().hp_batch_run_each(self._h, _stream_handle(stream), 1 if graph else 0))

    def close(self):
        if self._h:
            check(lib().hp_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.hp_batch_destroy(self._h)
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tune(extents, ops, dtype, reps: int = 20, flags: int = 0):
    """Time candidate maps for the nest's size class on the current device and
    cache the fastest; returns (best_us, auto_us)."""
    _batch_sigs()
    n = make_nest(extents, ops, dtype)
    b, a = ctypes.c_double(), ctypes.c_double()
    check(lib().hp_tune_nest(ctypes.byref(n), flags, reps, ctypes.byref(b), ctypes.byref(a)))
    return b.value, a.value


def tune_cache_load(path: str):
    _batch_sigs()
    check(lib().hp_tune_cache_load(path.encode()))


def tune_cache_save(path: str):
    _batch_sigs()
    check(lib().hp_tune_cache_save(path.encode()))


def tune_cache_clear():
    _batch_sigs()
    check(lib().hp_tune_cache_clear())


def tune_cache_size() -> int:
    _batch_sigs()
    n = ctypes.c_int64()
    check(lib().hp_tune_cache_size(ctypes.byref(n)))
    return n.value


# ---------------------------------------------------------------------------
# serving

SERVER_FAKE_DEVICE = 0x1000


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("slot_bytes", ctypes.c_size_t), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("window_us", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("fail_every_nth_batch", ctypes.c_int32), ("fail_step", ctypes.c_int32)]


class ReqInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("t_arrival_us", ctypes.c_double),
                ("t_admit_us", ctypes.c_double), ("t_launch_us", ctypes.c_double), ("t_done_us", ctypes.c_double),
                ("bytes", ctypes.c_int64), ("batch_id", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("pending", ctypes.c_int64), ("max_queue", ctypes.c_int64),
                ("max_in_use_bytes", ctypes.c_int64), ("in_use_bytes", ctypes.c_int64), ("bytes", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("p999_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("mean_us", ctypes.c_double), ("gbps", ctypes.c_double)]


_server_sigs_done = False


def _server_sigs():
    global _server_sigs_done
    if _server_sigs_done:
        return
    L = lib()
    vp, st, u64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
    L.hp_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
    L.hp_submit.argtypes = [vp, ctypes.POINTER(Nest), vp, vp, ctypes.c_double, u64p]
    L.hp_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ReqInfo)]
    L.hp_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ReqInfo)]
    L.hp_server_forget.argtypes = [vp, ctypes.c_uint64]
    L.hp_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.hp_server_now_us.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.hp_server_replay.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Nest), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double), u64p]
    L.hp_server_destroy.argtypes = [vp]
    for f in ("hp_server_create", "hp_submit", "hp_poll", "hp_wait", "hp_server_forget", "hp_server_get_stats",
              "hp_server_now_us", "hp_server_replay", "hp_server_destroy"):
        getattr(L, f).restype = st
    _server_sigs_done = True


def _info(ri: ReqInfo) -> dict:
    return {k: getattr(ri, k) for k, _ in ReqInfo._fields_ if k != "pad"}


class Server:
    """hp_server_*: continuous batching of nest-reduction requests."""

    def __init__(self, hbm_budget=64 << 30, slot_bytes=64 << 20, streams=4, max_batch=1024, window_us=30,
                 queue_cap=1 << 20, flags=0, fail_every_nth_batch=0, fail_step=0):
        _server_sigs()
        cfg = ServerCfg(hbm_budget, slot_bytes, streams, max_batch, window_us, queue_cap, flags,
                        fail_every_nth_batch, fail_step)
        self._h = ctypes.c_void_p()
        check(lib().hp_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def now_us(self) -> float:
        t = ctypes.c_double()
        check(lib().hp_server_now_us(self._h, ctypes.byref(t)))
        return t.value

    def submit(self, extents, ops, dtype, in_ptr: int, out_ptr: int, t_arrival_us: float = -1.0) -> int:
        n = make_nest(extents, ops, dtype)
        t = ctypes.c_uint64()
        check(lib().hp_submit(self._h, ctypes.byref(n), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                              t_arrival_us, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        ri = ReqInfo()
        s = lib().hp_poll(self._h, ticket, ctypes.byref(ri))
        if s == 7:  # HP_ENOTREADY
            return None
        check(s)
        return _info(ri)

    def wait(self, ticket: int) -> dict:
        ri = ReqInfo()
        check(lib().hp_wait(self._h, ticket, ctypes.byref(ri)))
        return _info(ri)

    def forget(self, ticket: int):
        check(lib().hp_server_forget(self._h, ticket))

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().hp_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def replay(self, nests, in_ptrs, out_ptrs, t_arrival_us):
        """Submit request i at server time t_arrival_us[i] (hp_server_replay)."""
        return self._replay(nests, in_ptrs, out_ptrs, lambda: t_arrival_us)[0]

    def replay_from_now(self, nests, in_ptrs, out_ptrs, offsets_us, lead_us: float = 5000.0):
        """Submit request i at t0 + offsets_us[i], with t0 = now + lead_us read after the
        arguments have been marshalled (for long streams that takes a noticeable time,
        which would otherwise delay the first arrivals).  Returns (tickets, t0)."""
        t0 = []

        def times():
            t0.append(self.now_us() + lead_us)
            return [t0[0] + o for o in offsets_us]
        tk = self._replay(nests, in_ptrs, out_ptrs, times)
        return tk[0], t0[0]

    def _replay(self, nests, in_ptrs, out_ptrs, times):
        n = len(nests)
        arr = (Nest * n)()
        for i, (ext, ops, dt) in enumerate(nests):
            arr[i] = make_nest(ext, ops, dt)
        ins = (ctypes.c_void_p * n)(*in_ptrs)
        outs = (ctypes.c_void_p * n)(*out_ptrs)
        tk = (ctypes.c_uint64 * n)()
        ts = (ctypes.c_double * n)()
        ts[:] = times()
        check(lib().hp_server_replay(self._h, n, arr, ins, outs, ts, tk))
        return list(tk), None

    def close(self):
        if self._h:
            check(lib().hp_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
