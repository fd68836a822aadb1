"""Seeded synthetic workloads for the nested-reduction benchmarks and tests.

This module only produces inputs: element values (via the SplitMix64 counter
generator in ``gen.c``), nest shapes and request streams.  It contains no
reduction arithmetic, and it is the only code shared by the CPU oracle side
and the GPU side of the tests.

Workloads (seeds are ``BASE_SEED + n`` for workload n):

* ``c1``: 2-level nest, int32 1024x1024 uniform in [-1000, 1000], out[i] = sum_j.
* ``c2``: 3-level nest, fp32 4096x256x256 N(0,1), out[i] = sum_j sum_k.
* ``c3``: 4-level nest, int32 64x128x64x64 uniform in [0, 2^20),
  out[i] = sum_j max_k argmin_l.
* ``c4``: 10,000 bf16 nests of log-normal total length (median 4096,
  max 2^22), 3 levels (e0, j, k) with j k = ceil(L / e0), reduced levels SUM.
* ``c5``: open-loop Poisson request stream (20k req/s), 2-4 level nests of
  log-normal byte size (median 64 KiB, max 256 MiB), half int32, half fp32.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 230901906

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libhpgen.so")

K_U64, K_I32, K_F32N, K_BF16N, K_F64N = 0, 1, 2, 3, 4

# op / dtype codes used in nest descriptions (plain ints; both sides map them)
NONE, SUM, MIN, MAX, ARGMIN, ARGMAX = 0, 1, 2, 3, 4, 5
I32, F32, BF16 = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (no GPU code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.gen_fill.restype = ctypes.c_int
        lib.gen_fill.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _fill(kind, seed, start, out: np.ndarray, lo=0, hi=0):
    assert out.flags.c_contiguous
    rc = _load().gen_fill(kind, seed & (2**64 - 1), start, out.size, lo, hi,
                          out.ctypes.data, _threads())
    if rc != 0:
        raise ValueError("gen_fill rejected its arguments")
    return out


def u64(seed: int, n: int, start: int = 0) -> np.ndarray:
    return _fill(K_U64, seed, start, np.empty(n, np.uint64))


AFFINE, MAT2 = 5, 6  # element types of ordered products (uint64 words per element: 2, 4)


def monoid_input(seed: int, shape, kind: int, start: int = 0) -> np.ndarray:
    """Random elements of an ordered-product type, uint64 of shape shape + (w,).
    Affine maps (a, b) get an odd a and 2x2 matrices an odd determinant (odd
    diagonal, even upper-right entry), so long products stay invertible modulo
    2^64 instead of collapsing to multiples of large powers of two."""
    w = 2 if kind == AFFINE else 4
    n = int(np.prod(shape, dtype=np.int64))
    x = u64(seed, n * w, start).reshape(tuple(shape) + (w,))
    if kind == AFFINE:
        x[..., 0] |= np.uint64(1)
    else:
        x[..., 0] |= np.uint64(1)
        x[..., 3] |= np.uint64(1)
        x[..., 1] &= ~np.uint64(1)
    return x


def uniform_i32(seed: int, shape, lo: int, hi: int, start: int = 0) -> np.ndarray:
    out = np.empty(shape, np.int32)
    return _fill(K_I32, seed, start, out.reshape(-1), lo, hi).reshape(shape)


def normal_f32(seed: int, shape, start: int = 0) -> np.ndarray:
    out = np.empty(shape, np.float32)
    return _fill(K_F32N, seed, start, out.reshape(-1)).reshape(shape)


def normal_bf16_bits(seed: int, shape, start: int = 0) -> np.ndarray:
    """bfloat16 values as raw uint16 bit patterns (N(0,1) rounded RNE)."""
    out = np.empty(shape, np.uint16)
    return _fill(K_BF16N, seed, start, out.reshape(-1)).reshape(shape)


def normal_f64(seed: int, n: int, start: int = 0) -> np.ndarray:
    return _fill(K_F64N, seed, start, np.empty(n, np.float64))


def unit_f64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform draws in [0, 1)."""
    return (u64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (1.0 / 2**53)


# ---------------------------------------------------------------------------
# Fixed-shape workloads


@dataclass
class Nest:
    extents: tuple
    ops: tuple
    dtype: int

    @property
    def elems(self) -> int:
        return int(np.prod(self.extents, dtype=np.int64))

    @property
    def elem_bytes(self) -> int:
        return 2 if self.dtype == BF16 else 4


C1 = Nest((1024, 1024), (NONE, SUM), I32)
C2 = Nest((4096, 256, 256), (NONE, SUM, SUM), F32)
C3 = Nest((64, 128, 64, 64), (NONE, SUM, MAX, ARGMIN), I32)


def c1_input(shape=C1.extents) -> np.ndarray:
    return uniform_i32(BASE_SEED + 1, shape, -1000, 1000)


def c2_input(shape=C2.extents, start: int = 0) -> np.ndarray:
    return normal_f32(BASE_SEED + 2, shape, start)


def c3_input(shape=C3.extents) -> np.ndarray:
    return uniform_i32(BASE_SEED + 3, shape, 0, (1 << 20) - 1)


def lognormal_sigma(median: float, maximum: float, n: int) -> float:
    """sigma such that the 1 - 1/n quantile of LogNormal(ln median, sigma) is `maximum`."""
    from statistics import NormalDist
    return math.log(maximum / median) / NormalDist().inv_cdf(1.0 - 1.0 / n)


@dataclass
class BatchWorkload:
    nests: list                 # list[Nest], 3-level (e0, j, k)
    offsets: np.ndarray         # element offset of each nest in the packed buffer (multiple of 8)
    total_elems: int
    seed: int

    def payload_bf16(self) -> np.ndarray:
        return normal_bf16_bits(self.seed, (self.total_elems,))


def c4_batch(n: int = 10000, median: int = 4096, maximum: int = 1 << 22, seed: int = BASE_SEED + 4) -> BatchWorkload:
    """Uneven bf16 nests.  Total length L ~ LogNormal(ln median, sigma) clipped to
    [64, maximum]; e0 = 2^U with U uniform in {0..min(6, log2(L/64))}; reduced
    length I = ceil(L / e0), any integer; shape (e0, j, k) with k = gcd(I, 64) and
    j = I / k.  (How the reduced block meets the hardware is the planner's and the
    tuner's choice: a single reduction may be reshaped.)"""
    sigma = lognormal_sigma(median, maximum, n)
    z = normal_f64(seed, n, start=0)
    u = unit_f64(seed ^ 0x5DEECE66D, n)
    nests, offsets = [], np.zeros(n, np.int64)
    off = 0
    for i in range(n):
        L = int(round(math.exp(math.log(median) + sigma * z[i])))
        L = max(64, min(maximum, L))
        umax = min(6, int(math.floor(math.log2(L / 64)))) if L >= 64 else 0
        U = int(u[i] * (umax + 1))
        e0 = 1 << U
        I = (L + e0 - 1) // e0
        k = math.gcd(I, 64)
        nests.append(Nest((e0, I // k, k), (NONE, SUM, SUM), BF16))
        offsets[i] = off
        off += ((e0 * I + 7) // 8) * 8
    return BatchWorkload(nests, offsets, off, seed + 1000)


@dataclass
class Request:
    t_arrival_us: float
    nest: Nest
    pool: int           # 0: int32 pool, 1: fp32 pool
    offset: int         # element offset in its pool (multiple of 4)


@dataclass
class RequestStream:
    requests: list = field(default_factory=list)
    pool_elems: int = 0
    seed: int = 0

    def pool_i32(self) -> np.ndarray:
        return uniform_i32(self.seed, (self.pool_elems,), -1000, 1000)

    def pool_f32(self) -> np.ndarray:
        return normal_f32(self.seed + 1, (self.pool_elems,))


def c5_stream(duration_s: float = 1.0, rate: float = 20000.0, median_bytes: int = 64 << 10,
              max_bytes: int = 256 << 20, pool_elems: int = 1 << 28, seed: int = BASE_SEED + 5,
              max_requests: int | None = None) -> RequestStream:
    """Open-loop Poisson arrivals with log-normal payload sizes (bytes clipped to
    [256, max_bytes], further capped by the pool).  Depth uniform in {2,3,4};
    inner extents are powers of two; e0 = ceil(elements / prod(inner)).  Half of
    the requests are int32 with per-level ops drawn from {SUM, MAX, ARGMIN}, half
    fp32 with SUM at every reduced level."""
    n = int(duration_s * rate * 1.5) + 64
    if max_requests is not None:
        n = min(n, max_requests)
    sigma = lognormal_sigma(median_bytes, max_bytes, 200000)
    draws = unit_f64(seed, 16 * n).reshape(n, 16)
    z = normal_f64(seed + 7, n)
    t = 0.0
    st = RequestStream(pool_elems=pool_elems, seed=seed + 100)
    for r in range(n):
        d = draws[r]
        t += -math.log(1.0 - d[0]) / rate * 1e6
        if t > duration_s * 1e6:
            break
        nbytes = int(math.exp(math.log(median_bytes) + sigma * z[r]))
        nbytes = max(256, min(max_bytes, nbytes))
        elems = max(1, min(pool_elems // 2, nbytes // 4))
        is_int = d[1] < 0.5
        depth = 2 + int(d[2] * 3)
        inner = []
        rem = elems
        for lv in range(depth - 1):
            # power-of-two extents, innermost first, leaving at least one outer row
            cap = max(0, int(math.floor(math.log2(max(1, rem)))) - (depth - 2 - lv))
            k = int(d[3 + lv] * (min(cap, 10) + 1))
            inner.append(1 << k)
            rem = max(1, rem // (1 << k))
        inner = inner[::-1]
        e0 = max(1, -(-elems // int(np.prod(inner))))
        ext = (e0,) + tuple(inner)
        if is_int:
            ops = (NONE,) + tuple((SUM, MAX, ARGMIN)[int(d[8 + lv] * 3)] for lv in range(depth - 1))
            dt = I32
        else:
            ops = (NONE,) + (SUM,) * (depth - 1)
            dt = F32
        total = int(np.prod(ext))
        if total > pool_elems:
            continue
        off = int(d[12] * (pool_elems - total)) // 4 * 4
        st.requests.append(Request(t, Nest(ext, ops, dt), 0 if is_int else 1, off))
        if max_requests is not None and len(st.requests) >= max_requests:
            break
    return st
