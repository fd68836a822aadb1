"""GPU tests of the persistent batched kernel: every nest of a batch gives the same
bits as the one-launch-per-nest baseline over the same plans, matches the oracle,
and graph replays reproduce the eager result."""
import numpy as np
import pytest

import workloads
from gpu_util import assert_match, say, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_01906_amd as hp
    hp.lib()
    yield


def packed(nests, seed, kind):
    """One device buffer holding every nest's input at 16-byte aligned offsets."""
    offs, off = [], 0
    for ext, ops, dt in nests:
        offs.append(off)
        off += (int(np.prod(ext)) + 7) // 8 * 8
    if kind == "bf16":
        host = workloads.normal_bf16_bits(seed, (off,))
    elif kind == "f32":
        host = workloads.normal_f32(seed, (off,))
    else:
        host = workloads.uniform_i32(seed, (off,), -1000, 1000)
    return host, offs


def run_batch(nests, host, offs, flags=0, graph_each=False, replays=1):
    import paper_2309_01906_amd as hp
    dev = to_device(host)
    with hp.Batch(nests, flags) as b:
        ins = [dev[o:o + int(np.prod(e))] for o, (e, _, _) in zip(offs, nests)]
        outs_b = [torch.zeros(b.info(i)["n_out"], dtype=hp.torch_out_dtype(b.info(i)["out_dtype"]), device="cuda")
                  for i in range(len(nests))]
        outs_e = [torch.zeros_like(t) for t in outs_b]
        b.set_io(ins, outs_b)
        results = []
        for r in range(replays):
            for t in outs_b:
                t.zero_()
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            results.append([t.cpu().numpy() for t in outs_b])
            torch.sum(dev[:1024].float()).item()  # eager work between replays
        b.set_io(ins, outs_e)
        b.run_each(graph=graph_each)
        torch.cuda.synchronize()
        each = [t.cpu().numpy() for t in outs_e]
        stats = b.stats()
    return results, each, stats


def uneven_bf16(n, seed):
    bw = workloads.c4_batch(n=n, median=4096, maximum=1 << 18, seed=seed)
    return [(nest.extents, nest.ops, workloads.BF16) for nest in bw.nests]


def test_batch_bf16_uneven_matches_each_and_oracle():
    nests = uneven_bf16(300, 91)
    host, offs = packed(nests, 92, "bf16")
    say("case batch bf16 uneven", len(nests), "nests")
    (res,), each, stats = run_batch(nests, host, offs)
    assert stats["launches"] == 1
    for i, (ext, ops, _) in enumerate(nests):
        np.testing.assert_array_equal(res[i], each[i], err_msg=f"nest {i} {ext}")
        x = host[offs[i]:offs[i] + int(np.prod(ext))].reshape(ext)
        assert_match(res[i], np.ascontiguousarray(x), ext, ops, what=f"nest {i} {ext}")


def test_batch_graph_replays_and_graph_each():
    import paper_2309_01906_amd as hp
    nests = uneven_bf16(200, 93)
    host, offs = packed(nests, 94, "bf16")
    say("case batch graph", len(nests), "nests")
    results, each, _ = run_batch(nests, host, offs, flags=hp.BATCH_GRAPH, graph_each=True, replays=4)
    for r in results:
        for i in range(len(nests)):
            np.testing.assert_array_equal(r[i], each[i], err_msg=f"replay nest {i}")


def test_batch_mixed_families():
    # int32 flat, int32 multi-segment, deep int32, fp32: four persistent launches
    nests = [((7, 300), ("NONE", "SUM"), 0), ((3, 64, 64), ("NONE", "MAX", "ARGMIN"), 0),
             ((2, 2, 2, 2, 2, 33), ("NONE", "SUM", "MAX", "ARGMIN", "SUM", "MIN"), 0),
             ((5, 4096), ("NONE", "SUM"), 1), ((1, 1 << 20), ("NONE", "SUM"), 1),
             ((1, 1 << 20), ("NONE", "ARGMAX"), 0), ((4, 5), ("NONE", "SUM"), 1), ((9,), ("NONE",), 0)]
    hi, offi = packed(nests, 95, "i32")
    hf, offf = packed(nests, 96, "f32")
    # one buffer per type: give each nest the buffer of its type
    import paper_2309_01906_amd as hp
    di, df = to_device(hi), to_device(hf)
    with hp.Batch(nests) as b:
        ins, outs = [], []
        for i, (ext, ops, dt) in enumerate(nests):
            n = int(np.prod(ext))
            ins.append(di[offi[i]:offi[i] + n] if dt == 0 else df[offf[i]:offf[i] + n])
            inf = b.info(i)
            outs.append(torch.zeros(inf["n_out"], dtype=hp.torch_out_dtype(inf["out_dtype"]), device="cuda"))
        b.set_io(ins, outs)
        st = b.stats()
        assert st["launches"] >= 3
        # several runs in a row: each must find its task counters cleared by the last
        for r in range(3):
            for t in outs:
                t.zero_()
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            for i, (ext, ops, dt) in enumerate(nests):
                n = int(np.prod(ext))
                x = (hi[offi[i]:offi[i] + n] if dt == 0 else hf[offf[i]:offf[i] + n]).reshape(ext)
                assert_match(outs[i].cpu().numpy(), np.ascontiguousarray(x), ext, ops, what=f"run {r} mixed nest {i}")


def test_batch_arg_over_wide_sums():
    """An ARG level over int64 sums of full-range int32 values cannot take 64-bit key
    carriers: the single-nest plan names the general kernel, and in a batch the
    segmented family carries (value, index) pairs.  Mixed with narrow nests of the
    same depth, every output matches the oracle bit for bit and one launch per nest."""
    import paper_2309_01906_amd as hp
    wide = [((6, 16, 64), ("NONE", "ARGMAX", "SUM"), 0), ((5, 7, 33), ("NONE", "ARGMIN", "SUM"), 0),
            ((3, 4, 8, 64), ("NONE", "SUM", "ARGMAX", "SUM"), 0)]
    narrow = [((6, 16, 64), ("NONE", "ARGMAX", "MAX"), 0), ((5, 7, 33), ("NONE", "SUM", "ARGMIN"), 0)]
    for ext, ops, _ in wide:
        assert hp.inspect(ext, ops, hp.I32)["kernel"] == hp.KERNEL_INT_DEEP, (ext, ops)
    for ext, ops, _ in narrow:
        assert hp.inspect(ext, ops, hp.I32)["kernel"] != hp.KERNEL_INT_DEEP, (ext, ops)
    nests = wide + narrow
    offs, off = [], 0
    for ext, _, _ in nests:
        offs.append(off)
        off += (int(np.prod(ext)) + 7) // 8 * 8
    host = workloads.uniform_i32(97, (off,), -(1 << 31), (1 << 31) - 1)
    say("case batch wide sums", len(nests))
    results, each, _ = run_batch(nests, host, offs)
    for i, (ext, ops, _) in enumerate(nests):
        n = int(np.prod(ext))
        np.testing.assert_array_equal(results[0][i], each[i], err_msg=f"nest {i}")
        assert_match(results[0][i], host[offs[i]:offs[i] + n].reshape(ext), ext, ops, what=f"wide nest {i}")


def test_batch_mixed_families_graph_replays():
    """The multi-launch batch replayed from a graph, with and without grid-split
    nests (the fold kernel, when there is one, clears the task counters for the
    next replay; otherwise each launch clears its own)."""
    import paper_2309_01906_amd as hp
    for split in (True, False):
        nests = [((7, 300), ("NONE", "SUM"), 0), ((3, 64, 64), ("NONE", "MAX", "ARGMIN"), 0),
                 ((5, 4096), ("NONE", "SUM"), 1), ((4, 5), ("NONE", "SUM"), 1)]
        if split:
            nests += [((1, 1 << 20), ("NONE", "SUM"), 1), ((1, 1 << 20), ("NONE", "ARGMAX"), 0)]
        hi, offi = packed(nests, 98, "i32")
        hf, offf = packed(nests, 99, "f32")
        di, df = to_device(hi), to_device(hf)
        say("case batch mixed graph", "split" if split else "no split")
        with hp.Batch(nests, hp.BATCH_GRAPH) as b:
            ins, outs = [], []
            for i, (ext, ops, dt) in enumerate(nests):
                n = int(np.prod(ext))
                ins.append(di[offi[i]:offi[i] + n] if dt == 0 else df[offf[i]:offf[i] + n])
                inf = b.info(i)
                outs.append(torch.zeros(inf["n_out"], dtype=hp.torch_out_dtype(inf["out_dtype"]), device="cuda"))
            b.set_io(ins, outs)
            assert b.stats()["launches"] >= 2
            assert any(b.info(i)["gsplit"] > 1 for i in range(len(nests))) == split
            for r in range(4):
                for t in outs:
                    t.zero_()
                torch.cuda.synchronize()
                b.run()
                torch.cuda.synchronize()
                for i, (ext, ops, dt) in enumerate(nests):
                    n = int(np.prod(ext))
                    x = (hi[offi[i]:offi[i] + n] if dt == 0 else hf[offf[i]:offf[i] + n]).reshape(ext)
                    assert_match(outs[i].cpu().numpy(), np.ascontiguousarray(x), ext, ops,
                                 what=f"replay {r} nest {i}")
                torch.sum(di[:1024].float()).item()  # eager work between replays


def test_tuner_then_batch():
    import paper_2309_01906_amd as hp
    hp.tune_cache_clear()
    ext, ops = (4, 256, 64), ("NONE", "SUM", "SUM")
    best, auto = hp.tune(ext, ops, hp.BF16, reps=5)
    assert best > 0 and auto > 0 and best <= auto * 1.0001
    assert hp.tune_cache_size() >= 1
    nests = [(ext, ops, hp.BF16)] * 3 + [((4, 512, 32), ops, hp.BF16)]
    host, offs = packed(nests, 97, "bf16")
    (res,), each, _ = run_batch(nests, host, offs)
    for i, (e, o, _) in enumerate(nests):
        np.testing.assert_array_equal(res[i], each[i])
        x = host[offs[i]:offs[i] + int(np.prod(e))].reshape(e)
        assert_match(res[i], np.ascontiguousarray(x), e, o, what=f"tuned nest {i}")
    hp.tune_cache_clear()
