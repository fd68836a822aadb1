"""Helpers shared by the GPU tests: move seeded host inputs to the device, run the
HIP path through the C ABI, and compare with the oracle."""
import os
import sys

import numpy as np

import oracle
import paper_2309_01906_amd as hp

OPS = hp.OP_NAMES
# the committed tuner cache the benchmark loads
ROOT_TUNE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2309_01906_amd",
                         "tune_gfx950.txt")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(x: np.ndarray):
    import torch
    if x.dtype == np.uint16:
        t = torch.from_numpy(x.view(np.int16).copy()).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to("cuda")


def np_dtype_code(x: np.ndarray) -> int:
    return {np.dtype(np.int32): hp.I32, np.dtype(np.float32): hp.F32, np.dtype(np.uint16): hp.BF16}[x.dtype]


def gpu_reduce(x, extents, ops, level_map=None, flags=0, dev=None):
    import torch
    ops = [OPS[o] if isinstance(o, str) else o for o in ops]
    d = to_device(x) if dev is None else dev
    with hp.Plan(extents, ops, np_dtype_code(x), level_map, flags) as p:
        out = p.run(d)
        torch.cuda.synchronize()
        return out.cpu().numpy(), p.info


def oracle_reduce(x, extents, ops, o_begin=0, o_end=None, threads=8):
    ops = [OPS[o] if isinstance(o, str) else o for o in ops]
    return oracle.reduce(x, extents, ops, np_dtype_code(x), threads=threads, o_begin=o_begin, o_end=o_end)


def assert_match(got, x, extents, ops, o_begin=0, o_end=None, rel=1e-6, what=""):
    ops_i = [OPS[o] if isinstance(o, str) else o for o in ops]
    ref = oracle_reduce(x, extents, ops_i, o_begin, o_end)
    got = np.asarray(got)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if x.dtype == np.int32:
        assert got.dtype == ref.dtype, (what, got.dtype, ref.dtype)
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}: got {got[bad[:5]]} want {ref[bad[:5]]}"
    else:
        s = oracle.abs_sum(x, extents, ops_i, np_dtype_code(x), threads=8, o_begin=o_begin,
                           o_end=o_end) if any(o != 0 for o in ops_i) else np.abs(ref)
        ok, plain, scaled = oracle.within_tolerance(got.astype(np.float64), ref, s, rel)
        assert ok, f"{what}: max scaled error {scaled:.3g} (plain relative {plain:.3g}) exceeds {rel}"
        return plain, scaled
    return 0.0, 0.0
