"""Tune the level maps of the batched workload's size classes on this GPU and write
the tuner cache that batched plans consult.

    python paper_2309_01906_amd/tune.py [--out FILE] [--reps N] [--limit K]

One representative nest per size class (input type, operators, log2 of the output
count and of the block length) is timed with every candidate map (hp_tune_nest);
the winners are saved with hp_tune_cache_save.  The default output file is the
one the benchmark loads.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def class_key(nest):
    import math
    outs = 1
    block = 1
    for e, o in zip(nest.extents, nest.ops):
        if o == 0:
            outs *= e
        else:
            block *= e
    return (nest.dtype, tuple(nest.ops), int(math.log2(outs)), int(math.log2(block)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.txt"))
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--limit", type=int, default=0, help="tune at most this many classes (0: all)")
    args = ap.parse_args()

    import torch

    import paper_2309_01906_amd as hp
    import workloads
    torch.cuda.set_device(0)
    bw = workloads.c4_batch()
    reps = {}
    for n in bw.nests:
        reps.setdefault(class_key(n), n)
    keys = sorted(reps)
    if args.limit:
        keys = keys[: args.limit]
    hp.tune_cache_clear()
    t0 = time.perf_counter()
    for i, k in enumerate(keys):
        n = reps[k]
        best, auto = hp.tune(n.extents, n.ops, n.dtype, reps=args.reps)
        print(f"class {i + 1}/{len(keys)} {k}: shape {n.extents} auto {auto:.1f} us -> tuned {best:.1f} us "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        hp.tune_cache_save(args.out)  # after every class, so an interrupted run keeps what it has
    print(f"{len(keys)} classes tuned in {time.perf_counter() - t0:.1f} s -> {args.out}", flush=True)


if __name__ == "__main__":
    main()
