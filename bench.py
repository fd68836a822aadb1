#!/usr/bin/env python3
"""Benchmark of the nested multi-level reduction on one MI355X.

Headline workload: the plain 3-level nest, fp32 4096 x 256 x 256 (1 GiB, N(0,1)),
out[i] = sum_j sum_k A[i,j,k] with fp32 compensated accumulation and fp64 output,
levels mapped grid -> waves -> lanes.  A step is one hp_run over the whole array
(input resident in HBM); value = algorithmic bytes (input + output) per second.

Prints ONE JSON line (rank 0, N = 1).  Only one GPU is used; --gpus > 1 exits.
The CPU baseline leg times the oracle (test infrastructure) on the host cores and
states the error of the GPU results against it: the headline's, the ragged nest's,
the batch's and the served requests'.  Those checks read results the timed GPU runs
left behind; with --no-cpu-baseline nothing calls the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "achieved HBM GB/s (% of peak) for nested reduction; batched-vs-plain; p50/p99"
# the CPU baseline leg: the oracle checks of GPU results (off with --no-cpu-baseline)
ORACLE_CHECKS = True
PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
KERNEL_SOURCES = ["hp_nest.h", "hp_lanes.h", "hp_nest_f32.hip", "hp_internal.h", "hp_plan.cpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_01906_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def progress(msg: str):
    """A progress line on stderr as each part of the benchmark ends."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def time_plan(plan, dev_in, out, steps, warmup, stream):
    """Warmup, then `steps` runs bracketed by synchronize; per-run HIP events on the
    stream the kernel is launched on."""
    import torch
    for _ in range(warmup):
        plan.run(dev_in, out, stream=stream)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        plan.run(dev_in, out, stream=stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return wall, ev_ms


def counters_from_profiles():
    """The committed rocprofv3 counter summary of the headline kernel, if it was taken
    on the current kernel sources; else None."""
    p = COUNTERS_JSON
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d


def traffic_from_profiles(per_launch_bytes):
    """HBM bytes per launch from the committed counter summary, or None."""
    d = counters_from_profiles()
    return None if d is None else d.get("traffic_bytes_per_launch")


def utilisation_from_profiles(avg_ms):
    """VALU and LDS figures of the headline kernel: per-wave instruction counts from
    the committed SQ counters, and the share of the SIMDs' issue time the VALU work
    takes at this run's measured kernel time (a wave64 instruction occupies a 16-lane
    SIMD for 4 cycles; 1024 SIMDs at 2.4 GHz)."""
    d = counters_from_profiles()
    if d is None or "sq" not in d:
        return None
    sq = d["sq"]
    valu = sq.get("sq_insts_valu_per_wave", 0.0) * sq["waves"]
    return {"valu_insts_per_wave": sq.get("sq_insts_valu_per_wave"), "lds_insts_per_wave": sq.get("sq_insts_lds_per_wave"),
            "lds_bank_conflict_cycles_per_wave": sq.get("sq_lds_bank_conflict_per_wave"),
            "valu_share": round(valu * 4 / (1024 * 2.4e9 * avg_ms * 1e-3), 3)}


COUNTERS_JSON = os.path.join(ROOT, "profiles", "c2_nest_counters.json")


def ingest_counters(fetch_csv, write_csv, kernel, nbytes, copy_bytes=1 << 30, sq_csv=None):
    """Turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of a `bench.py --copy-calib` run into HBM bytes
    per launch of `kernel`.  Each counter is scaled by what it reads for the 1 GiB
    device copy of the same run (reads 1 GiB, writes 1 GiB)."""
    import csv

    def rows(path, counter):
        out = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
        return out

    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rs = rows(path, counter)
        ks = [v for n, _, v in rs if kernel in n]
        copies = [(g, v) for n, g, v in rs if "copyBuffer" in n]
        if not ks or not copies:
            raise SystemExit(f"{path}: no {counter} rows for {kernel} or for the calibration copy")
        calib = max(copies)[1]  # the largest copy dispatch is the 1 GiB calibration copy
        scale = copy_bytes / (calib * 1024.0)
        res[counter] = {"kib_per_dispatch": round(sum(ks) / len(ks), 3), "dispatches": len(ks),
                        "copy_kib": calib, "scale": round(scale, 6),
                        "bytes_per_launch": round(sum(ks) / len(ks) * 1024.0 * scale)}
    traffic = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    d = {"kernel": kernel, "kernel_hash": kernel_hash(), "algorithmic_bytes_per_launch": nbytes,
         "traffic_bytes_per_launch": traffic, "traffic_over_algorithmic": round(traffic / nbytes, 5),
         "counters": res, "calibration": f"device copy of {copy_bytes} bytes (reads and writes that many)"}
    if sq_csv:  # per-wave instruction counts (SQ block) of the same kernel
        sums, n = {}, {}
        with open(sq_csv) as fh:
            for r in csv.DictReader(fh):
                if kernel in r["Kernel_Name"]:
                    c = r["Counter_Name"]
                    sums[c] = sums.get(c, 0.0) + float(r["Counter_Value"])
                    n[c] = n.get(c, 0) + 1
        if "SQ_WAVES" in sums:
            waves = sums["SQ_WAVES"] / n["SQ_WAVES"]
            d["sq"] = {"waves": waves}
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_LDS_BANK_CONFLICT"):
                if c in sums:
                    d["sq"][c.lower() + "_per_wave"] = round(sums[c] / n[c] / waves, 2)
    os.makedirs(os.path.dirname(COUNTERS_JSON), exist_ok=True)
    with open(COUNTERS_JSON, "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    print(json.dumps(d))


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), as lscpu prints it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_host, ext, ops, got_rows):
    """Oracle on the host cores: the full workload with every core (median of the
    runs made in about 10 s), the same on one core, and the error statement of the
    GPU result against it."""
    import numpy as np

    import oracle
    threads = max(1, min(64, os.cpu_count() or 1))
    n_out = ext[0]
    nbytes = x_host.nbytes + n_out * 8

    def timed(th, budget_s, min_runs):
        times, ref = [], None
        t_start = time.perf_counter()
        while len(times) < min_runs or (time.perf_counter() - t_start < budget_s and len(times) < 1000):
            t0 = time.perf_counter()
            ref = oracle.reduce(x_host, ext, ops, oracle.F32, threads=th)
            times.append(time.perf_counter() - t0)
        return statistics.median(times), len(times), ref

    t, runs, ref = timed(threads, 10.0, 3)
    t1, runs1, ref1 = timed(1, 8.0, 2)
    s = oracle.abs_sum(x_host, ext, ops, oracle.F32, threads=threads)
    ok, plain, scaled = oracle.within_tolerance(got_rows, ref, s, 1e-6)
    return {
        "value": round(nbytes / t / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
        "sample": f"full workload ({n_out} outputs, {x_host.nbytes >> 20} MiB) repeated for ~10 s, median of {runs} runs, "
                  f"fp64 Neumaier sequential C, outputs split over {threads} threads",
        "seconds": round(t, 4), "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "single_core": {"value": round(nbytes / t1 / 1e9, 3), "unit": "GB/s", "cores": 1, "seconds": round(t1, 4),
                        "sample": f"the same full workload on one thread, median of {runs1} runs",
                        "bit_identical_to_all_cores": bool(np.array_equal(ref, ref1))},
    }, {"all_outputs_checked": int(n_out), "within_1e-6": ok, "max_rel_err": plain,
        "max_scaled_err": scaled,
        "worst_condition_number": float(np.max(s / np.maximum(np.abs(ref), 1e-300))),
        "rule": "|gpu - fp64 oracle| <= 1e-6 * max(|oracle|, 2^-24 * sum|a|) per output"}


def error_statement(v) -> dict:
    """The summary of oracle.verify that the bench line carries."""
    keys = ("ok", "nests", "int_nests", "int_nests_mismatched", "float_nests", "float_outputs", "max_rel_err",
            "max_scaled_err", "worst_condition_number")
    d = {k: v[k] for k in keys}
    d["rule"] = "ints bit-exact; floats |gpu - fp64 oracle| <= 1e-6 * max(|oracle|, 2^-24 * sum|a|) per output"
    return d


def extra_int_workloads(steps, warmup, stream):
    """C1 and C3: GB/s with the plan's default map (cache-resident sizes: labelled)."""
    import torch

    import paper_2309_01906_amd as hp
    import workloads
    res = {}
    # a 512 MiB read evicts the input from L2 and the 256 MB MALL without leaving
    # dirty lines behind (a fill would be written back during the timed run)
    flush = torch.zeros(128 << 20, dtype=torch.float32, device="cuda")
    for name, nest, gen in (("c1", workloads.C1, workloads.c1_input), ("c3", workloads.C3, workloads.c3_input)):
        x = gen()
        d = torch.from_numpy(x).cuda()
        with hp.Plan(nest.extents, nest.ops, nest.dtype) as p:
            out = p.empty_out(d.device)
            # warm (cache-resident) timing
            wall, ev = time_plan(p, d, out, steps, warmup, stream)
            # cold: flush L2 / MALL with a 512 MiB read between runs, outside the events
            cold = []
            for _ in range(min(steps, 50)):
                flush.sum()
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s.record(stream)
                p.run(d, out, stream=stream)
                e.record(stream)
                torch.cuda.synchronize()
                cold.append(s.elapsed_time(e))
            nbytes = x.nbytes + p.info["out_bytes"]
            res[name] = {
                "shape": list(nest.extents), "bytes": nbytes, "map": p.info["map"], "grid": p.info["grid"],
                "warm_p50_us": round(pct(ev, 50) * 1e3, 2), "warm_p99_us": round(pct(ev, 99) * 1e3, 2),
                "cold_p50_us": round(pct(cold, 50) * 1e3, 2), "cold_p99_us": round(pct(cold, 99) * 1e3, 2),
                "cold_GBps": round(nbytes / (pct(cold, 50) * 1e-3) / 1e9, 1),
            }
        del d
    del flush
    return res


def _time_cold(plan, d, out, stream, reps, flush):
    """p50 of `reps` runs, each after a 512 MiB read that evicts L2 and the MALL."""
    import torch
    ts = []
    for _ in range(reps):
        flush.sum()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        plan.run(d, out, stream=stream)
        e.record(stream)
        torch.cuda.synchronize()
        ts.append(s.elapsed_time(e))
    return pct(ts, 50)


def extra_ragged_and_xcd(steps, warmup, stream):
    """A 3-level-sized fp32 nest whose rows are not vector multiples, (4096, 65537)
    (flat blocks: 16-byte loads on each row's aligned interior), beside the headline;
    and the XCD scope: the 4-level int32 nest and a one-output 1 GiB fp32 sum
    (viewed as (1, 8, 2^25)) with the default numbering, with XCD numbering off
    (HP_FLAG_NO_XCD) and with an explicit X level."""
    import torch

    import paper_2309_01906_amd as hp
    import workloads
    res = {}
    flush = torch.zeros(128 << 20, dtype=torch.float32, device="cuda")
    ext = (4096, 65537)
    x = workloads.normal_f32(workloads.BASE_SEED + 6, ext)
    d = torch.from_numpy(x).cuda()
    with hp.Plan(ext, (hp.NONE, hp.SUM), hp.F32) as p:
        out = p.empty_out(d.device)
        wall, ev = time_plan(p, d, out, steps, warmup, stream)
        nb = x.nbytes + p.info["out_bytes"]
        got = out.cpu().numpy()
        res["ragged_fp32_4096x65537"] = {
            "bytes": nb, "kernel": p.info["kernel_name"], "flat_block": p.info["flat_block"],
            "p50_us": round(pct(ev, 50) * 1e3, 1), "GBps": round(nb / (pct(ev, 50) * 1e-3) / 1e9, 1)}
        if ORACLE_CHECKS:
            import oracle
            ref = oracle.reduce(x, ext, (0, 1), oracle.F32, threads=16)
            sa = oracle.abs_sum(x, ext, (0, 1), oracle.F32, threads=16)
            ok, plain, scaled = oracle.within_tolerance(got, ref, sa, 1e-6)
            res["ragged_fp32_4096x65537"].update({"all_outputs_within_1e-6": bool(ok), "max_rel_err": plain})
    del d, x
    xcd = {}
    c3 = workloads.C3
    xi = workloads.c3_input()
    d = torch.from_numpy(xi).cuda()
    for label, m, fl in (("default", None, 0), ("no_xcd_numbering", None, hp.FLAG_NO_XCD),
                         ("x_on_outputs", ["X", ("GW", {"G": 16, "W": 8}), ("V", {"V": 16}), ("V", {"V": 4})], 0)):
        with hp.Plan(c3.extents, c3.ops, c3.dtype, m, fl) as p:
            out = p.empty_out(d.device)
            for _ in range(warmup):
                p.run(d, out, stream=stream)
            xcd[f"c3_{label}_cold_us"] = round(_time_cold(p, d, out, stream, min(steps, 30), flush) * 1e3, 2)
    del d
    big = torch.randn(1 << 28, dtype=torch.float32, device="cuda")
    # one sum of 2^28 floats: (1, 2^28) with the automatic map, with and without the
    # XCD numbering; and viewed as (8, 2^25) with its first level on X
    for label, ext, ops, m, fl in (("default", (1, 1 << 28), (hp.NONE, hp.SUM), None, 0),
                                   ("no_xcd_numbering", (1, 1 << 28), (hp.NONE, hp.SUM), None, hp.FLAG_NO_XCD),
                                   ("x_level", (8, 1 << 25), (hp.SUM, hp.SUM),
                                    ["X", ("GWV", {"G": 256, "W": 8})], 0)):
        with hp.Plan(ext, ops, hp.F32, m, fl) as p:
            out = p.empty_out(big.device)
            for _ in range(warmup):
                p.run(big, out, stream=stream)
            xcd[f"sum_1GiB_{label}_cold_us"] = round(_time_cold(p, big, out, stream, min(steps, 30), flush) * 1e3, 2)
            xcd[f"sum_1GiB_{label}_map"] = p.info["map"]
    del big, flush
    res["xcd_scope"] = xcd
    return res


def ordered_products(stream, steps=20, warmup=3):
    """Ordered (non-commutative) products, 1 GiB each: 4096 recurrences of 16,384
    affine steps, and 4096 products of 8,192 2x2 matrices, modulo 2^64.  The values
    are random words (the product kernels do the same work for any value)."""
    import numpy as np
    import torch

    import paper_2309_01906_amd as hp
    res = {}
    for name, dt, ext in (("affine_4096x16384", hp.AFFINE64, (4096, 16384)), ("mat2x2_4096x8192", hp.MAT2X2_64, (4096, 8192))):
        g = torch.Generator(device="cuda").manual_seed(230901906)
        x = torch.randint(-2**62, 2**62, (int(np.prod(ext)) * hp.WIDTH[dt],), dtype=torch.int64, device="cuda",
                          generator=g)
        with hp.Plan(ext, (hp.NONE, hp.PROD), dt) as p:
            out = p.empty_out(x.device)
            wall, ev = time_plan(p, x, out, steps, warmup, stream)
            nb = p.info["in_bytes"] + p.info["out_bytes"]
            res[name] = {"bytes": nb, "kernel": p.info["kernel_name"], "p50_us": round(pct(ev, 50) * 1e3, 1),
                         "GBps": round(nb / (pct(ev, 50) * 1e-3) / 1e9, 1), "chunks_per_output": p.info["gsplit"]}
        del x
    return res


def stencils(stream, steps=20, warmup=3):
    """Five-point Jacobi sweeps of an 8192 x 8192 fp32 array (256 MiB): 1, 4 and 8
    sweeps in one launch and 16 in two, tiled through LDS with a ghost surface, the
    tiles dealt to the XCDs in bands; 1 and 8 sweeps also without the XCD bands.
    `effective_GBps` counts one read and one write of every cell per sweep (what
    separate sweeps would move); `launch_GBps` one read and one write of every cell
    per launch, which is what HBM carries when the ghost cells that neighbouring
    tiles share are read once (the HBM counters show this with the XCD bands, and
    about twice the reads without them at one sweep)."""
    import torch

    import paper_2309_01906_amd as hp
    import workloads
    R = C = 8192
    x = torch.from_numpy(workloads.normal_f32(230901906 + 7, (R, C))).cuda()
    y = torch.empty_like(x)
    res = {}
    # each no-band run right after its banded twin, so that both see the same clocks
    for t, flags in ((1, 0), (1, hp.STENCIL_NO_XCD), (4, 0), (8, 0), (8, hp.STENCIL_NO_XCD), (16, 0)):
        with hp.Stencil(R, C, t, 0.6, 0.1, flags=flags) as st:
            for _ in range(warmup):
                st.run(x, y, stream)
            torch.cuda.synchronize()
            ev = []
            for _ in range(steps):
                s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s_.record(stream)
                st.run(x, y, stream)
                e_.record(stream)
                e_.synchronize()
                ev.append(s_.elapsed_time(e_))
            inf = st.info
        us = pct(ev, 50) * 1e3
        key = f"sweeps_{t}" + ("_no_xcd" if flags else "")
        res[key] = {"p50_us": round(us, 1), "tile": [inf["tile_rows"], inf["tile_cols"]],
                    "sweeps_per_launch": inf["sweeps_per_launch"], "launches": inf["launches"],
                    "effective_GBps": round(8.0 * R * C * t / us / 1e3, 1),
                    "launch_GBps": round(inf["launches"] * 8.0 * R * C / us / 1e3, 1)}
    del x, y
    return res


def batched_vs_plain(stream, steps=20, warmup=3, plain=True, verify=True):
    """10,000 uneven bf16 nests: one persistent launch replayed from a hipGraph vs one
    launch per nest (eager, and all launches captured in one graph).  Same plans, so
    the outputs are compared bit for bit.  Latency: each run timed alone (p50/p99).
    Throughput: `back_to_back_*`, 50 runs enqueued back to back between two events;
    the same persistent launches also without the graph (`batched_direct`)."""
    import numpy as np
    import torch

    import paper_2309_01906_amd as hp
    import workloads
    bw = workloads.c4_batch()
    host = bw.payload_bf16()
    dev = torch.from_numpy(host.view(np.int16)).cuda().view(torch.bfloat16)
    nests = [(n.extents, n.ops, n.dtype) for n in bw.nests]
    out_elems = [n.extents[0] for n in bw.nests]
    oo = np.concatenate([[0], np.cumsum(out_elems)])
    out_a = torch.zeros(int(oo[-1]), dtype=torch.float64, device="cuda")
    out_b = torch.zeros_like(out_a)
    t_plan = time.perf_counter()
    b = hp.Batch(nests, hp.BATCH_GRAPH)
    t_plan = time.perf_counter() - t_plan
    base_in, base_a, base_b = dev.data_ptr(), out_a.data_ptr(), out_b.data_ptr()
    ins = [base_in + 2 * int(o) for o in bw.offsets]
    st = b.stats()

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        ev = []
        t0 = time.perf_counter()
        for _ in range(k):
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(stream)
            fn()
            e_.record(stream)
            e_.synchronize()
            ev.append(s_.elapsed_time(e_))
        return (time.perf_counter() - t0) / k * 1e3, ev

    def back_to_back(fn, k=50):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(stream)
        for _ in range(k):
            fn()
        e_.record(stream)
        e_.synchronize()
        return s_.elapsed_time(e_) / k

    b.set_io_ptrs(ins, [base_a + 8 * int(o) for o in oo[:-1]])
    wall_b, ev_b = timed(lambda: b.run(stream), steps, warmup)
    b2b_g = back_to_back(lambda: b.run(stream))
    got_b = out_a.cpu().numpy()
    with hp.Batch(nests) as bd:  # the same plans and launches, without the graph
        bd.set_io_ptrs(ins, [base_a + 8 * int(o) for o in oo[:-1]])
        _, ev_d = timed(lambda: bd.run(stream), steps, warmup)
        b2b_d = back_to_back(lambda: bd.run(stream))
        same_direct = bool(np.array_equal(out_a.cpu().numpy(), got_b))
    nbytes = st["bytes"]
    err = None
    if verify and ORACLE_CHECKS:
        import oracle
        cases = [(host[bw.offsets[i]:bw.offsets[i] + n.elems].reshape(n.extents), n.extents, n.ops, oracle.BF16,
                  got_b[oo[i]:oo[i + 1]]) for i, n in enumerate(bw.nests)]
        err = error_statement(oracle.verify(cases))
    def form(ev, b2b_ms):
        return {"p50_us": round(pct(ev, 50) * 1e3, 1), "p99_us": round(pct(ev, 99) * 1e3, 1),
                "GBps": round(nbytes / (pct(ev, 50) * 1e-3) / 1e9, 1),
                "back_to_back_us": round(b2b_ms * 1e3, 1), "back_to_back_GBps": round(nbytes / (b2b_ms * 1e-3) / 1e9, 1)}

    if not plain:
        b.close()
        return {"nests": len(nests), "bytes": nbytes, "persistent_launches": st["launches"], "tasks": st["tasks"],
                "wave_workers": st["workers"], "batched_graph": form(ev_b, b2b_g),
                "batched_direct": form(ev_d, b2b_d), "direct_bit_identical": same_direct}
    b.set_io_ptrs(ins, [base_b + 8 * int(o) for o in oo[:-1]])
    wall_p, ev_p = timed(lambda: b.run_each(stream, graph=False), max(3, steps // 4), 1)
    got_p = out_b.cpu().numpy()
    wall_g, ev_g = timed(lambda: b.run_each(stream, graph=True), max(3, steps // 4), 1)
    b.close()
    res = {
        "nests": len(nests), "bytes": nbytes, "persistent_launches": st["launches"], "tasks": st["tasks"],
        "wave_workers": st["workers"],
        "plan_seconds": round(t_plan, 3),
        "batched_graph": form(ev_b, b2b_g),
        "batched_direct": form(ev_d, b2b_d), "direct_bit_identical": same_direct,
        "plain_one_launch_per_nest": {"p50_us": round(pct(ev_p, 50) * 1e3, 1),
                                      "GBps": round(nbytes / (pct(ev_p, 50) * 1e-3) / 1e9, 1)},
        "plain_launches_in_one_graph": {"p50_us": round(pct(ev_g, 50) * 1e3, 1),
                                        "GBps": round(nbytes / (pct(ev_g, 50) * 1e-3) / 1e9, 1)},
        "bit_identical_to_plain": bool(np.array_equal(got_b, got_p)),
        "error_vs_fp64_oracle": err,
    }
    res["speedup_vs_plain"] = round(res["plain_one_launch_per_nest"]["p50_us"] / res["batched_graph"]["p50_us"], 2)
    del dev, out_a, out_b
    return res


class ServingPools:
    """The request stream's two 1 GiB payload pools (int32 and fp32), on the host and
    on the device, shared by the serving runs."""

    def __init__(self):
        import torch

        import workloads
        st = workloads.c5_stream(duration_s=0.0, pool_elems=1 << 28)
        self.seed = st.seed
        self.pi, self.pf = st.pool_i32(), st.pool_f32()
        self.di, self.df = torch.from_numpy(self.pi).cuda(), torch.from_numpy(self.pf).cuda()


def serve_stream(pools, duration_s, rate, warmup_s, verify):
    """Replay one open-loop Poisson stream through a server; latency is measured
    from each request's scheduled arrival to its observed completion."""
    import numpy as np
    import torch

    import paper_2309_01906_amd as hp
    import workloads
    st = workloads.c5_stream(duration_s=duration_s + warmup_s, rate=rate, pool_elems=1 << 28)
    assert st.seed == pools.seed
    reqs = st.requests
    out_sizes = [hp.inspect(r.nest.extents, r.nest.ops, r.nest.dtype)["n_out"] for r in reqs]
    out = torch.zeros(int(sum(out_sizes)) + len(reqs), dtype=torch.float64, device="cuda")  # 8 B per output
    offs = np.concatenate([[0], np.cumsum(out_sizes)])
    ins = [(pools.di if r.pool == 0 else pools.df).data_ptr() + 4 * r.offset for r in reqs]
    outs = [out.data_ptr() + 8 * int(o) for o in offs[:-1]]
    nests = [(r.nest.extents, r.nest.ops, r.nest.dtype) for r in reqs]
    with hp.Server(hbm_budget=64 << 30, slot_bytes=256 << 20, streams=4, max_batch=512, window_us=30) as srv:
        tk, t0 = srv.replay_from_now(nests, ins, outs, [r.t_arrival_us for r in reqs])
        infos = [srv.wait(t) for t in tk]
        stats = srv.stats()
    arr = np.array([i["t_arrival_us"] - t0 for i in infos])
    lat = np.array([i["t_done_us"] - i["t_arrival_us"] for i in infos])
    steady = arr >= warmup_s * 1e6
    ls = lat[steady]
    nb = sum(int(np.prod(r.nest.extents)) * 4 for r, k in zip(reqs, steady) if k)
    t_first = min(i["t_arrival_us"] for i, k in zip(infos, steady) if k)
    t_last = max(i["t_done_us"] for i, k in zip(infos, steady) if k)
    res = {
        "requests": len(reqs), "measured_requests": int(steady.sum()), "offered_rate_per_s": rate,
        "duration_s": duration_s, "warmup_s": warmup_s,
        "all_ok": all(i["status"] == 0 for i in infos), "failed": stats["failed"], "batches": stats["batches"],
        "p50_us": round(float(np.percentile(ls, 50)), 1), "p99_us": round(float(np.percentile(ls, 99)), 1),
        "p999_us": round(float(np.percentile(ls, 99.9)), 1), "max_us": round(float(ls.max()), 1),
        "GBps": round(nb / (t_last - t_first) / 1e3, 2),
    }
    if verify and ORACLE_CHECKS:
        import oracle
        got = out.cpu().numpy()
        cases = []
        for k, r in enumerate(reqs):
            pool = pools.pi if r.pool == 0 else pools.pf
            x = pool[r.offset:r.offset + r.nest.elems].reshape(r.nest.extents)
            g = got[offs[k]:offs[k + 1]]  # one 8-byte slot per output; int32 outputs fill the first half
            kind = hp.inspect(r.nest.extents, r.nest.ops, r.nest.dtype)["out_dtype"]
            g = g.view(np.int64) if kind == hp.I64 else g.view(np.int32)[:g.size].copy() if kind == hp.I32 else g
            cases.append((x, r.nest.extents, r.nest.ops, r.nest.dtype, g))
        res["error_vs_fp64_oracle"] = error_statement(oracle.verify(cases))
    if verify:
        # start-up: p99 per 100 ms of arrival time over the first two seconds
        res["startup_p99_us_per_100ms"] = [round(float(np.percentile(lat[(arr >= a) & (arr < a + 1e5)], 99)), 1)
                                           for a in np.arange(0, 2e6, 1e5) if np.any((arr >= a) & (arr < a + 1e5))]
        res["including_warmup"] = {"p50_us": round(stats["p50_us"], 1), "p99_us": round(stats["p99_us"], 1),
                                   "GBps": round(stats["gbps"], 2)}
        res["bytes"] = stats["bytes"]
        res["max_in_flight_bytes"] = stats["max_in_use_bytes"]
    del out
    return res


def serving(duration_s=10.0, rate=20000.0, warmup_s=1.0, sweep=True):
    """Open-loop Poisson stream of mixed 2-4 level requests admitted by a 64 GiB
    budget: 10 s measured after a 1 s warm-up at the offered 20k req/s, every result
    checked against the oracle; then a rate sweep (shorter runs) until p99 passes
    1 ms, to find the server's capacity."""
    pools = ServingPools()
    res = serve_stream(pools, duration_s, rate, warmup_s, verify=True)
    if sweep:
        res["rate_sweep"] = []
        r = 1.25 * rate
        while r <= 2.56e6:
            s = serve_stream(pools, 1.5, r, 0.5, verify=False)
            res["rate_sweep"].append({k: s[k] for k in ("offered_rate_per_s", "measured_requests", "all_ok", "p50_us",
                                                        "p99_us", "GBps", "batches")})
            if s["p99_us"] > 1000.0 or not s["all_ok"]:
                break
            r *= 1.25
    del pools
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-s", type=float, default=10.0, help="measured seconds of the serving run")
    ap.add_argument("--no-sweep", action="store_true", help="skip the serving rate sweep")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 1 GiB device copy (for scaling rocprofv3 byte counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the persistent batched run of the 10,000-nest workload (for profiling)")
    ap.add_argument("--ordered-only", action="store_true",
                    help="only the ordered products (for profiling the ordered kernels)")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only the stencil sweeps (for profiling the stencil kernels)")
    ap.add_argument("--int-only", action="store_true",
                    help="only the 2- and 4-level integer nests (for profiling)")
    ap.add_argument("--ingest-counters", nargs="+", metavar="CSV",
                    help="host only: FETCH_SIZE csv, WRITE_SIZE csv[, SQ counters csv] of rocprofv3 --pmc "
                         "runs -> the counter summary the bench reads; then exit")
    args = ap.parse_args()
    if args.ingest_counters:
        import paper_2309_01906_amd as hp
        import workloads
        info = hp.inspect(workloads.C2.extents, workloads.C2.ops, workloads.C2.dtype)
        if len(args.ingest_counters) not in (2, 3):
            raise SystemExit("--ingest-counters takes FETCH_CSV WRITE_CSV [SQ_CSV]")
        ingest_counters(args.ingest_counters[0], args.ingest_counters[1], info["kernel_name"],
                        info["in_bytes"] + info["out_bytes"],
                        sq_csv=args.ingest_counters[2] if len(args.ingest_counters) == 3 else None)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2309_01906_amd as hp
    import workloads

    torch.cuda.set_device(0)
    global ORACLE_CHECKS
    ORACLE_CHECKS = not args.no_cpu_baseline
    stream = torch.cuda.current_stream()
    if args.int_only:
        print(json.dumps({"int_nests": extra_int_workloads(args.steps, args.warmup, stream)}), flush=True)
        return
    if args.ordered_only:
        print(json.dumps({"ordered_products": ordered_products(stream, args.steps, args.warmup)}), flush=True)
        return
    if args.stencil_only:
        print(json.dumps({"stencils": stencils(stream, args.steps, args.warmup)}), flush=True)
        return
    if args.batched_only:
        tc = os.path.join(ROOT, "paper_2309_01906_amd", "tune_gfx950.txt")
        if os.path.exists(tc):
            hp.tune_cache_load(tc)
        print(json.dumps({"batched": batched_vs_plain(stream, args.steps, args.warmup, plain=False, verify=False)}),
              flush=True)
        return
    nest = workloads.C2
    x_host = workloads.c2_input()
    dev_in = torch.from_numpy(x_host).cuda()
    plan = hp.Plan(nest.extents, nest.ops, nest.dtype)
    out = plan.empty_out(dev_in.device)
    wall, ev_ms = time_plan(plan, dev_in, out, args.steps, args.warmup, stream)
    nbytes = x_host.nbytes + plan.info["out_bytes"]
    ms_per_step = wall / args.steps * 1e3
    value = nbytes / (ms_per_step * 1e-3) / 1e9
    avg_ev = sum(ev_ms) / len(ev_ms)
    achieved = nbytes / (avg_ev * 1e-3) / 1e9
    got = out.cpu().numpy()

    # the device's plain streaming-read ceiling on the same buffer (calibration kernel)
    ceiling = 0.0
    scratch = torch.empty(16384, dtype=torch.float32, device="cuda")
    for grid in (2048, 4096, 8192, 16384):
        for _ in range(3):
            hp.stream_read(dev_in, scratch, grid, stream)
        torch.cuda.synchronize()
        evs = []
        for _ in range(20):
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(stream)
            hp.stream_read(dev_in, scratch, grid, stream)
            e_.record(stream)
            e_.synchronize()
            evs.append(s_.elapsed_time(e_))
        ceiling = max(ceiling, x_host.nbytes / (pct(evs, 50) * 1e-3) / 1e9)
    del scratch

    if args.copy_calib:
        y = torch.empty_like(dev_in)
        y.copy_(dev_in)
        torch.cuda.synchronize()
        del y

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain 3-level nest fp32 4096x256x256 (1 GiB, N(0,1)), out[i]=sum_j sum_k A, "
                               "fp32 compensated pairs, fp64 output; grid->waves->lanes",
                   "shape": list(nest.extents), "map": plan.info["map"], "units": plan.info["units"],
                   "waves_per_workgroup": plan.info["waves"], "grid": plan.info["grid"],
                   "algorithmic_bytes": nbytes, "parallelism": "1 GPU"},
        "pct_of_peak": round(100.0 * value / PEAK_GBS, 2),
        "read_ceiling": {"GBps": round(ceiling, 1), "kernel": "hp_stream_read (plain nontemporal float4 read)",
                         "roofline_achieved_pct_of_ceiling": round(100.0 * achieved / ceiling, 1)},
        "p50_us": round(pct(ev_ms, 50) * 1e3, 2), "p99_us": round(pct(ev_ms, 99) * 1e3, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_GBS, 4), "traffic": traffic_from_profiles(nbytes),
                     "kernel": plan.info["kernel_name"], "algorithmic_bytes_per_launch": nbytes,
                     "kernel_hash": kernel_hash(), "utilisation": utilisation_from_profiles(avg_ev)},
    }
    progress(f"headline nest {round(achieved, 1)} GB/s by kernel events")
    if not args.no_cpu_baseline:
        cb, err = cpu_baseline(x_host, nest.extents, nest.ops, got)
        line["cpu_baseline"] = cb
        line["error_vs_fp64_oracle"] = err
        progress("oracle timed and outputs checked")
    if not args.no_extras:
        line["extras"] = extra_int_workloads(min(args.steps, 200), min(args.warmup, 20), stream)
        line["extras"].update(extra_ragged_and_xcd(min(args.steps, 50), min(args.warmup, 5), stream))
        progress("ragged and XCD extras done")
        progress("2- and 4-level integer nests done")
        tc = os.path.join(ROOT, "paper_2309_01906_amd", "tune_gfx950.txt")
        if os.path.exists(tc):
            hp.tune_cache_load(tc)
        if not args.no_batch:
            line["batched_vs_plain"] = batched_vs_plain(stream)
            progress("batched nests done")
        if not args.no_serving:
            line["serving"] = serving(duration_s=args.serving_s, sweep=not args.no_sweep)
            progress("serving done")
        line["ordered_products"] = ordered_products(stream)
        line["stencils"] = stencils(stream)
        progress("ordered products and stencils done")
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
