"""Reference oracle for nested multi-level reductions -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never does, and this package
imports nothing from it.  The arithmetic lives in ``oracle.c`` (plain
sequential C nested loops, see ``oracle.h`` for the definition and the
readings of the paper it follows); this file only builds and calls it.

Every function here is pinned by ``tests/test_oracle.py`` against closed
forms, exactly rounded sums (``math.fsum``), numpy library reductions,
brute force on tiny nests and invariants; nothing is left "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NONE, SUM, MIN, MAX, ARGMIN, ARGMAX, PROD = 0, 1, 2, 3, 4, 5, 6
I32, F32, BF16, AFFINE, MAT2 = 0, 1, 2, 5, 6
WIDTH = {AFFINE: 2, MAT2: 4}  # uint64 words per element of the ordered-product types
OUT_I32, OUT_I64, OUT_F64 = 0, 1, 2
_OUT_NP = {OUT_I32: np.int32, OUT_I64: np.int64, OUT_F64: np.float64}
_IN_NP = {I32: np.int32, F32: np.float32, BF16: np.uint16}

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_out_kind.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int]
        lib.oracle_out_kind.restype = ctypes.c_int
        lib.oracle_n_out.argtypes = [ctypes.c_int, i64p, ip]
        lib.oracle_n_out.restype = ctypes.c_int64
        lib.oracle_reduce_range.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        lib.oracle_reduce_range.restype = ctypes.c_int
        lib.oracle_abs_sum_range.argtypes = lib.oracle_reduce_range.argtypes
        lib.oracle_abs_sum_range.restype = ctypes.c_int
        lib.oracle_prod_range.argtypes = lib.oracle_reduce_range.argtypes
        lib.oracle_prod_range.restype = ctypes.c_int
        lib.oracle_stencil.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_stencil.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arrays(extents, ops):
    d = len(extents)
    e = (ctypes.c_int64 * d)(*[int(x) for x in extents])
    o = (ctypes.c_int * d)(*[int(x) for x in ops])
    return d, e, o


def out_kind(extents, ops, dtype) -> int:
    d, e, o = _arrays(extents, ops)
    k = _load().oracle_out_kind(d, e, o, int(dtype))
    if k < 0:
        raise ValueError("nest not defined for the oracle")
    return k


def n_out(extents, ops) -> int:
    d, e, o = _arrays(extents, ops)
    k = _load().oracle_n_out(d, e, o)
    if k < 0:
        raise ValueError("nest not defined for the oracle")
    return int(k)


def _check_input(x: np.ndarray, extents, dtype):
    want = _IN_NP[dtype]
    if x.dtype != want:
        raise TypeError(f"input dtype {x.dtype}, expected {np.dtype(want)}")
    if x.size != int(np.prod(extents, dtype=np.int64)):
        raise ValueError("input size does not match the extents")
    if not x.flags.c_contiguous:
        raise ValueError("input must be C-contiguous")


def reduce(x: np.ndarray, extents, ops, dtype, threads: int = 1, o_begin: int = 0,
           o_end: int | None = None) -> np.ndarray:
    """Outputs [o_begin, o_end) of the nest over the row-major input ``x``
    (int32, float32, or bfloat16 bit patterns as uint16)."""
    _check_input(x, extents, dtype)
    kind = out_kind(extents, ops, dtype)
    total = n_out(extents, ops)
    if o_end is None:
        o_end = total
    out = np.empty(o_end - o_begin, _OUT_NP[kind])
    d, e, o = _arrays(extents, ops)
    rc = _load().oracle_reduce_range(d, e, o, int(dtype), x.ctypes.data, out.ctypes.data,
                                     int(o_begin), int(o_end), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the nest or range")
    return out


def abs_sum(x: np.ndarray, extents, ops, dtype, threads: int = 1, o_begin: int = 0,
            o_end: int | None = None) -> np.ndarray:
    """Sum of |a| over each output's reduced block (float nests): the scale of
    the accuracy bound."""
    _check_input(x, extents, dtype)
    total = n_out(extents, ops)
    if o_end is None:
        o_end = total
    out = np.empty(o_end - o_begin, np.float64)
    d, e, o = _arrays(extents, ops)
    rc = _load().oracle_abs_sum_range(d, e, o, int(dtype), x.ctypes.data, out.ctypes.data,
                                      int(o_begin), int(o_end), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the nest or range")
    return out


def prod(x: np.ndarray, extents, ops, dtype, threads: int = 1, o_begin: int = 0,
         o_end: int | None = None) -> np.ndarray:
    """Ordered products (levels PROD, after a NONE prefix) over ``x``: uint64 of
    shape extents + (width,), width 2 for AFFINE and 4 for MAT2.  Returns the
    outputs [o_begin, o_end) as uint64 of shape (count, width)."""
    w = WIDTH[dtype]
    if x.dtype != np.uint64 or not x.flags.c_contiguous:
        raise TypeError("input must be C-contiguous uint64")
    if x.size != int(np.prod(extents, dtype=np.int64)) * w:
        raise ValueError("input size does not match the extents")
    p = next((i for i, o in enumerate(ops) if o != NONE), len(ops))
    total = int(np.prod(extents[:p], dtype=np.int64))
    if o_end is None:
        o_end = total
    out = np.empty((o_end - o_begin, w), np.uint64)
    d, e, o = _arrays(extents, ops)
    rc = _load().oracle_prod_range(d, e, o, int(dtype), x.ctypes.data, out.ctypes.data,
                                   int(o_begin), int(o_end), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the nest or range")
    return out


def stencil(x: np.ndarray, steps: int, c0: float, c1: float) -> np.ndarray:
    """`steps` five-point Jacobi sweeps of the float32 2-D array ``x`` (boundary
    cells fixed), in double precision."""
    if x.dtype != np.float32 or x.ndim != 2 or not x.flags.c_contiguous:
        raise TypeError("input must be a C-contiguous 2-D float32 array")
    out = np.empty(x.shape, np.float64)
    rc = _load().oracle_stencil(x.shape[0], x.shape[1], int(steps), float(c0), float(c1), x.ctypes.data,
                                out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the stencil")
    return out


def within_tolerance(got: np.ndarray, ref: np.ndarray, abs_sum_ref: np.ndarray, rel: float = 1e-6):
    """Float acceptance rule: |got - ref| <= rel * max(|ref|, 2^-24 * sum|a|).
    Returns (ok, max plain relative error, max scaled error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), abs_sum_ref * 2.0**-24)
    err = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        plain = np.where(ref != 0, err / np.abs(ref), np.where(err == 0, 0.0, np.inf))
        scaled = np.where(scale > 0, err / scale, np.where(err == 0, 0.0, np.inf))
    ok = bool(np.all(scaled <= rel))
    return ok, float(plain.max(initial=0.0)), float(scaled.max(initial=0.0))


def verify(cases, rel: float = 1e-6, workers: int | None = None) -> dict:
    """Check many device results against the oracle (a thread pool: the C calls
    release the GIL).  ``cases`` yields (x, extents, ops, dtype, got) per nest.
    Integer nests must match bit for bit; float nests must satisfy
    ``within_tolerance`` output by output.  Returns counts, the largest plain and
    scaled errors, the worst condition number sum|a| / |sum a| over the float
    outputs, and the first failing cases."""
    from concurrent.futures import ThreadPoolExecutor

    cases = list(cases)
    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))

    def one(k):
        x, ext, ops, dt, got = cases[k]
        ref = reduce(x, ext, ops, dt)
        got = np.asarray(got)
        if dt == I32:
            bad = int(np.count_nonzero(got.reshape(ref.shape) != ref)) if got.size == ref.size else ref.size
            return k, True, bad, None
        s = abs_sum(x, ext, ops, dt) if any(o != NONE for o in ops) else np.abs(ref.astype(np.float64))
        return k, False, None, (np.asarray(got, np.float64).reshape(-1), ref.astype(np.float64), s)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, range(len(cases))))
    n_int = sum(1 for r in res if r[1])
    int_bad = [(r[0], r[2]) for r in res if r[1] and r[2]]
    fl = [r for r in res if not r[1]]
    out = {"nests": len(cases), "int_nests": n_int, "int_nests_mismatched": len(int_bad),
           "float_nests": len(fl), "float_outputs": 0, "float_within": True, "max_rel_err": 0.0,
           "max_scaled_err": 0.0, "worst_condition_number": 0.0, "failures": [k for k, _ in int_bad[:5]]}
    if fl:
        got = np.concatenate([r[3][0] for r in fl])
        ref = np.concatenate([r[3][1] for r in fl])
        s = np.concatenate([r[3][2] for r in fl])
        ok, plain, scaled = within_tolerance(got, ref, s, rel)
        with np.errstate(divide="ignore"):
            cond = float(np.max(np.where(ref != 0, s / np.abs(ref), np.where(s == 0, 1.0, np.inf))))
        out.update(float_outputs=int(got.size), float_within=ok, max_rel_err=plain, max_scaled_err=scaled,
                   worst_condition_number=cond)
        if not ok:
            for r in fl:
                g, f, a = r[3]
                if not within_tolerance(g, f, a, rel)[0]:
                    out["failures"].append(r[0])
                    if len(out["failures"]) >= 10:
                        break
    out["ok"] = not int_bad and out["float_within"]
    return out
