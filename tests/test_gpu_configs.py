"""GPU parity at the benchmarked configurations, through the C ABI: the headline
3-level nest with every output checked; the 10,000-nest bf16 batch on the
committed tuner recipes, replayed from its graph exactly as the benchmark runs it;
a full-size request stream through the server; and the batch kernel families that
uneven or deep nests use.  Every result is checked against the oracle -- bit for
bit for integers, within |got - ref| <= 1e-6 * max(|ref|, 2^-24 * sum|a|) for
floats -- and the error statement is printed."""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ROOT_TUNE, say, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_01906_amd as hp
    hp.lib()
    yield
    hp.tune_cache_clear()


def test_c2_full_size_all_rows():
    import paper_2309_01906_amd as hp
    say("case c2 full 4096x256x256 fp32 (1 GiB), all rows")
    nest = workloads.C2
    x = workloads.c2_input()
    d = to_device(x)
    with hp.Plan(nest.extents, nest.ops, nest.dtype) as p:
        assert p.info["kernel_name"] == "hp::k_nest_f32_lean<4>"
        got = p.run(d).cpu().numpy()
    del d
    ref = oracle.reduce(x, nest.extents, nest.ops, oracle.F32, threads=16)
    s = oracle.abs_sum(x, nest.extents, nest.ops, oracle.F32, threads=16)
    ok, plain, scaled = oracle.within_tolerance(got, ref, s, 1e-6)
    say(f"c2 all 4096 rows: max rel err {plain:.3g}, max scaled {scaled:.3g}")
    assert ok, (plain, scaled)


def test_c4_full_batch_on_tuned_recipes():
    """All 10,000 nests of the batched workload, planned with the committed tuner
    cache (reshaped blocks and many-outputs-per-task recipes), one persistent launch
    replayed from a hipGraph: every output within the 1e-6 rule, replays identical,
    and the same bits as one launch per nest."""
    import paper_2309_01906_amd as hp
    hp.tune_cache_clear()
    hp.tune_cache_load(ROOT_TUNE)
    bw = workloads.c4_batch()
    nests = [(n.extents, n.ops, n.dtype) for n in bw.nests]
    tuned = hp.batch_inspect(nests)
    plain = hp.batch_inspect(nests, hp.BATCH_NO_TUNE)
    n_tuned = sum(1 for a, b in zip(tuned, plain) if (a["map"], a["units"], a["grid"]) != (b["map"], b["units"], b["grid"]))
    say("case c4 full:", len(nests), "nests,", n_tuned, "on tuned recipes")
    assert n_tuned > 1000
    host = bw.payload_bf16()
    dev = to_device(host)
    oo = np.concatenate([[0], np.cumsum([n.extents[0] for n in bw.nests])])
    out = torch.zeros(int(oo[-1]), dtype=torch.float64, device="cuda")
    out_each = torch.zeros_like(out)
    ins = [dev.data_ptr() + 2 * int(o) for o in bw.offsets]
    with hp.Batch(nests, hp.BATCH_GRAPH) as b:
        b.set_io_ptrs(ins, [out.data_ptr() + 8 * int(o) for o in oo[:-1]])
        reps = []
        for r in range(3):
            out.fill_(-1.0)
            b.run()
            torch.cuda.synchronize()
            reps.append(out.cpu().numpy())
            torch.sum(dev[:4096].float()).item()  # eager work between replays
        b.set_io_ptrs(ins, [out_each.data_ptr() + 8 * int(o) for o in oo[:-1]])
        b.run_each()
        torch.cuda.synchronize()
        each = out_each.cpu().numpy()
    for r in reps[1:]:
        np.testing.assert_array_equal(r, reps[0])
    np.testing.assert_array_equal(reps[0], each)
    got = reps[0]
    cases = []
    for i, n in enumerate(bw.nests):
        x = host[bw.offsets[i]:bw.offsets[i] + n.elems].reshape(n.extents)
        cases.append((x, n.extents, n.ops, oracle.BF16, got[oo[i]:oo[i + 1]]))
    v = oracle.verify(cases)
    say("c4 error statement:", {k: v[k] for k in ("nests", "float_outputs", "max_rel_err", "max_scaled_err",
                                                   "worst_condition_number")})
    assert v["ok"], v["failures"]
    hp.tune_cache_clear()


def test_c5_full_size_stream_served():
    """Two seconds of the full serving workload (Poisson 20k req/s, sizes log-normal
    with median 64 KiB up to 256 MiB, half int32 with mixed ops, half fp32) through a
    server configured as the benchmark's: every request completes and matches the
    oracle."""
    import paper_2309_01906_amd as hp
    hp.tune_cache_clear()
    hp.tune_cache_load(ROOT_TUNE)
    st = workloads.c5_stream(duration_s=2.0)
    pi, pf = st.pool_i32(), st.pool_f32()
    di, df = torch.from_numpy(pi).cuda(), torch.from_numpy(pf).cuda()
    reqs = st.requests
    say("case c5 full size:", len(reqs), "requests, largest", max(r.nest.elems for r in reqs) * 4 >> 20, "MiB")
    outs = []
    for r in reqs:
        inf = hp.inspect(r.nest.extents, r.nest.ops, r.nest.dtype)
        outs.append(torch.full((inf["n_out"],), -7, dtype=hp.torch_out_dtype(inf["out_dtype"]), device="cuda"))
    ins = [(di if r.pool == 0 else df).data_ptr() + 4 * r.offset for r in reqs]
    with hp.Server(hbm_budget=64 << 30, slot_bytes=256 << 20, streams=4, max_batch=512, window_us=30) as s:
        tk, t0 = s.replay_from_now([(r.nest.extents, r.nest.ops, r.nest.dtype) for r in reqs], ins,
                                   [o.data_ptr() for o in outs], [r.t_arrival_us for r in reqs])
        infos = [s.wait(t) for t in tk]
        stats = s.stats()
    assert all(i["status"] == 0 for i in infos) and stats["failed"] == 0
    say("served:", {k: round(stats[k], 1) for k in ("completed", "batches", "p50_us", "p99_us", "gbps")})
    cases = []
    for r, o in zip(reqs, outs):
        pool = pi if r.pool == 0 else pf
        x = pool[r.offset:r.offset + r.nest.elems].reshape(r.nest.extents)
        cases.append((x, r.nest.extents, r.nest.ops, r.nest.dtype, o.cpu().numpy()))
    v = oracle.verify(cases)
    say("c5 error statement:", {k: v[k] for k in ("int_nests", "float_nests", "max_rel_err", "max_scaled_err",
                                                   "worst_condition_number")})
    assert v["ok"], v["failures"]
    hp.tune_cache_clear()


def _run_batch_and_verify(nests, kind, seed):
    import paper_2309_01906_amd as hp
    offs, off = [], 0
    for ext, _, _ in nests:
        offs.append(off)
        off += (int(np.prod(ext)) + 7) // 8 * 8
    host = {"bf16": workloads.normal_bf16_bits, "f32": workloads.normal_f32}[kind](seed, (off,))
    dev = to_device(host)
    with hp.Batch(nests) as b:
        fams = {b.info(i)["kernel_name"] for i in range(len(nests))}
        outs = [torch.zeros(b.info(i)["n_out"], dtype=hp.torch_out_dtype(b.info(i)["out_dtype"]), device="cuda")
                for i in range(len(nests))]
        each = [torch.zeros_like(t) for t in outs]
        ins = [dev[o:o + int(np.prod(e))] for o, (e, _, _) in zip(offs, nests)]
        b.set_io(ins, outs)
        b.run()
        b.set_io(ins, each)
        b.run_each()
        torch.cuda.synchronize()
    dt = oracle.BF16 if kind == "bf16" else oracle.F32
    cases = []
    for i, (ext, ops, _) in enumerate(nests):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), each[i].cpu().numpy(), err_msg=f"nest {i} {ext}")
        x = host[offs[i]:offs[i] + int(np.prod(ext))].reshape(ext)
        cases.append((x, ext, [hp.OP_NAMES[o] for o in ops], dt, outs[i].cpu().numpy()))
    v = oracle.verify(cases)
    assert v["ok"], (v["failures"], [nests[k] for k in v["failures"]])
    return fams


@pytest.mark.parametrize("kind", ["bf16", "f32"])
def test_batch_families_ragged_and_deep(kind):
    """Uneven shapes reach every float batch family: innermost extents that are not
    a multiple of the 16-byte vector, and nests deeper than 4 levels."""
    rng = np.random.default_rng(7 if kind == "bf16" else 8)
    nests = []
    for i in range(120):
        depth = int(rng.integers(2, 7))
        ext = [int(rng.integers(1, 6))] + [int(rng.integers(1, 9)) for _ in range(depth - 2)] + \
              [int(rng.integers(1, 300))]
        nests.append((tuple(ext), ("NONE",) + ("SUM",) * (depth - 1), 2 if kind == "bf16" else 1))
    nests += [((3, 2, 2, 2, 2, 1001), ("NONE",) + ("SUM",) * 5, 2 if kind == "bf16" else 1),
              ((1, 77777), ("NONE", "SUM"), 2 if kind == "bf16" else 1)]
    say("case batch families", kind, len(nests))
    fams = _run_batch_and_verify(nests, kind, 310)
    say("families", sorted(fams))
