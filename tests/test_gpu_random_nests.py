"""Seeded random nests against the oracle: depth 2 to 6, random extents (ragged
innermost lengths included), random operators on the integer levels, full-range
int32 values (so that ARG levels over SUMs see int64 values), fp32 and bf16 normals.
Each nest runs alone with its automatic plan, then all nests of one type run as one
batch; every output is checked (integers bit for bit, floats by the 1e-6 rule)."""
import random

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import say, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS_I = ("SUM", "MIN", "MAX", "ARGMIN", "ARGMAX")


def random_nests(rng, kind, n):
    nests = []
    for _ in range(n):
        depth = rng.randint(2, 6)
        p = rng.randint(1, depth - 1)
        ext = [rng.choice([1, 2, 3, 4, 5, 7, 8, 16, 33, 64]) for _ in range(depth)]
        ext[-1] = rng.choice([1, 3, 4, 7, 8, 16, 31, 64, 100, 256, 1000, 4099])
        ops = ("NONE",) * p + tuple(rng.choice(OPS_I) if kind == "i32" else "SUM" for _ in range(depth - p))
        nests.append((tuple(ext), ops))
    return nests


@pytest.mark.parametrize("kind", ["i32", "f32", "bf16"])
def test_random_nests_alone_and_batched(kind):
    import paper_2309_01906_amd as hp
    rng = random.Random({"i32": 5, "f32": 6, "bf16": 7}[kind])
    nests = random_nests(rng, kind, 150)
    offs, off = [], 0
    for ext, _ in nests:
        offs.append(off)
        off += (int(np.prod(ext)) + 7) // 8 * 8
    seed = 5000 + {"i32": 1, "f32": 2, "bf16": 3}[kind]
    if kind == "i32":
        host = workloads.uniform_i32(seed, (off,), -(1 << 31), (1 << 31) - 1)
    elif kind == "f32":
        host = workloads.normal_f32(seed, (off,))
    else:
        host = workloads.normal_bf16_bits(seed, (off,))
    dt = {"i32": hp.I32, "f32": hp.F32, "bf16": hp.BF16}[kind]
    odt = {"i32": oracle.I32, "f32": oracle.F32, "bf16": oracle.BF16}[kind]
    dev = to_device(host)
    say("case random nests", kind, len(nests))
    alone = []
    for (ext, ops), o in zip(nests, offs):
        n = int(np.prod(ext))
        with hp.Plan(ext, ops, dt) as p:
            out = p.empty_out(dev.device)
            p.run(dev[o:o + n], out)
            torch.cuda.synchronize()
            alone.append(out.cpu().numpy())
    with hp.Batch([(ext, ops, dt) for ext, ops in nests]) as b:
        outs = [torch.zeros(b.info(i)["n_out"], dtype=hp.torch_out_dtype(b.info(i)["out_dtype"]), device="cuda")
                for i in range(len(nests))]
        b.set_io([dev[o:o + int(np.prod(e))] for o, (e, _) in zip(offs, nests)], outs)
        b.run()
        torch.cuda.synchronize()
        batched = [t.cpu().numpy() for t in outs]
    for got, what in ((alone, "alone"), (batched, "batched")):
        cases = [(host[o:o + int(np.prod(e))].reshape(e), e, [hp.OP_NAMES[x] for x in ops], odt, g)
                 for o, (e, ops), g in zip(offs, nests, got)]
        v = oracle.verify(cases)
        say(kind, what, {k: v[k] for k in ("nests", "int_nests_mismatched", "max_scaled_err")})
        assert v["ok"], (what, [nests[k] for k in v["failures"]])


def large_nests(rng, kind, n, max_elems=1 << 23):
    """Blocks of 16 KiB to 16 MiB with 1 to 1,024 outputs: float sums of sums over 2
    to 4 levels, single-operator integer nests with few outputs."""
    nests = []
    while len(nests) < n:
        if kind == "i32":
            ext = (rng.choice([1, 2, 3, 5, 8, 64, 100, 512, 1000, 1024]),
                   rng.choice([1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 3 << 20]))
            ops = ("NONE", rng.choice(OPS_I))
        else:
            depth = rng.randint(2, 4)
            p = 1 if depth == 2 else rng.randint(1, depth - 2)
            ext = [rng.choice([1, 2, 3, 7, 16, 64, 256, 1024]) for _ in range(p)]
            ext += [rng.choice([1, 2, 3, 4, 8, 16, 64]) for _ in range(depth - p - 1)]
            ext = tuple(ext + [rng.choice([64, 256, 1024, 4096, 16384, 65536, 1 << 18])])
            ops = ("NONE",) * p + ("SUM",) * (depth - p)
        if (1 << 12) <= int(np.prod(ext)) <= max_elems:
            nests.append((ext, ops))
    return nests


@pytest.mark.parametrize("kind", ["i32", "f32", "bf16"])
def test_random_large_nests_alone(kind):
    """Larger blocks reach the planner's grid splits (and the integer fold on a whole
    wave), its wave rule and the one-level view of float sums of sums."""
    import paper_2309_01906_amd as hp
    rng = random.Random({"i32": 15, "f32": 16, "bf16": 17}[kind])
    dt = {"i32": hp.I32, "f32": hp.F32, "bf16": hp.BF16}[kind]
    odt = {"i32": oracle.I32, "f32": oracle.F32, "bf16": oracle.BF16}[kind]
    cases, plans = [], set()
    for i, (ext, ops) in enumerate(large_nests(rng, kind, 24)):
        n = int(np.prod(ext))
        if kind == "i32":
            x = workloads.uniform_i32(100 + i, (n,), -50, 50)  # many ties for the ARG levels
        elif kind == "f32":
            x = workloads.normal_f32(100 + i, (n,))
        else:
            x = workloads.normal_bf16_bits(100 + i, (n,))
        d = to_device(x)
        with hp.Plan(ext, ops, dt) as p:
            got = p.run(d).cpu().numpy()
            plans.add((p.info["kernel_name"], p.info["depth"], p.info["gsplit"] > 1))
        del d
        cases.append((x.reshape(ext), ext, [hp.OP_NAMES[o] for o in ops], odt, got))
    v = oracle.verify(cases)
    say("large", kind, len(cases), "nests, plans", sorted(plans))
    assert v["ok"], (v["failures"], [cases[k][1:3] for k in v["failures"]])
    assert any(split for _, _, split in plans)
