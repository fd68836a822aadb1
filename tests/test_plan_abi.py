"""Host-side tests of libhp.so: every declared entry point is exported, and the
planner (host only, no device) validates nests and maps and lowers them to
consistent launch geometry."""
import itertools
import os
import re

import numpy as np
import pytest

import paper_2309_01906_amd as hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(hp_\w+)\s*\(", txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = hp.lib()
    names = declared_functions()
    assert "hp_plan" in names and "hp_run" in names and "hp_destroy" in names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = hp.lib()
    for i, name in enumerate(hp.STATUS):
        assert L.hp_status_str(i).decode() == name


def err(extents, ops, dtype, m=None, flags=0):
    with pytest.raises(hp.HPError) as e:
        hp.inspect(extents, ops, dtype, m, flags)
    return e.value.status_name


def test_rejects_malformed_nests():
    assert err((4, 0), ("NONE", "SUM"), hp.I32) == "HP_EINVAL"
    assert err((4, 4), ("SUM", "NONE"), hp.I32) == "HP_EINVAL"
    assert err((4, 4), ("NONE", "MAX"), hp.F32) == "HP_EUNSUPPORTED"
    assert err((4, 4), ("NONE", "ARGMIN"), hp.BF16) == "HP_EUNSUPPORTED"
    assert err((4, 4), ("NONE", 9), hp.I32) == "HP_EINVAL"
    assert err((4, 4), ("NONE", "SUM"), 7) == "HP_EINVAL"
    assert err((4, 4), ("NONE", "SUM"), hp.I32, flags=0x100) == "HP_EINVAL"


def test_rejects_bad_maps():
    n = ((8, 8, 8), ("NONE", "SUM", "SUM"), hp.I32)
    assert err(*n, m=["W", "G", "V"]) == "HP_EINVAL"            # not monotone
    assert err(*n, m=["G", "GV", "L"]) == "HP_EINVAL"           # G+V is not a run of adjacent scopes
    assert err(*n, m=["G", ("W", {"W": 3}), "V"]) == "HP_EINVAL"  # not a power of two
    assert err(*n, m=["G", ("W", {"W": 32}), "V"]) == "HP_EINVAL"  # more than 16 waves
    assert err(*n, m=["G", ("W", {"V": 4}), "V"]) == "HP_EINVAL"  # units on an unused axis
    assert err(*n, m=["G", ("V", {"V": 16}), ("V", {"V": 16})]) == "HP_EINVAL"  # 256 lanes
    assert err(*n, m=["", "W", "V"]) == "HP_EINVAL"


SCOPE_SETS = ["G", "W", "V", "L", "GW", "WV", "VL", "GWV", "WVL", "GWVL"]
ORDER = "GWVL"


def monotone(m):
    # an L next to other scopes only marks strips; a level on L alone is serial
    for i, b in enumerate(m):
        for a in m[:i]:
            hi = a[-1] if a == "L" else a.replace("L", "")[-1]
            if ORDER.index(b[0]) < ORDER.index(hi):
                return False
    return True


def all_maps(depth):
    return [m for m in itertools.product(SCOPE_SETS, repeat=depth) if monotone(m)]


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_every_monotone_map_plans_consistently(depth):
    ext = (5, 7, 33)[:depth]
    for ops in [("SUM",) * depth, ("NONE",) + ("MAX",) * (depth - 1), ("NONE",) * depth]:
        for m in all_maps(depth):
            try:
                info = hp.inspect(ext, ops, hp.I32, list(m))
            except hp.HPError as e:
                # only the one-strip rule for reducing levels outside a grid-spanning
                # segment may refuse a well-formed monotone map
                assert e.status_name == "HP_EUNSUPPORTED", (m, ops, str(e))
                continue
            for l in range(depth):
                g, w, v = info["units"][l]
                chunk = info["chunk"] if l == depth - 1 else 1
                span = g * w * v * chunk
                assert info["strips"][l] == -(-ext[l] // span)
                assert (g > 1) <= ("G" in m[l]) and (w > 1) <= ("W" in m[l]) and (v > 1) <= ("V" in m[l])
            assert 1 <= info["waves"] <= 16
            assert info["grid"] >= 1


def test_auto_maps_for_the_workloads():
    c1 = hp.inspect((1024, 1024), ("NONE", "SUM"), hp.I32)
    assert c1["n_out"] == 1024 and c1["out_dtype"] == hp.I64 and c1["chunk"] == 4
    c2 = hp.inspect((4096, 256, 256), ("NONE", "SUM", "SUM"), hp.F32)
    assert c2["grid"] == 4096 and c2["gsplit"] == 1 and c2["out_dtype"] == hp.F64
    assert c2["map"][2] == "V" and c2["map"][1] == "W"
    c3 = hp.inspect((64, 128, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32)
    assert c3["nseg"] == 3 and c3["out_dtype"] == hp.I64 and c3["gsplit"] > 1
    big = hp.inspect((1, 1 << 28), ("NONE", "SUM"), hp.F32)
    assert big["gsplit"] > 1 and big["workspace_bytes"] > 0


def test_output_types_match_the_oracle_rule():
    import oracle
    for ops in [("NONE", "SUM"), ("NONE", "MAX"), ("NONE", "ARGMAX"), ("NONE", "MIN", "SUM"),
                ("NONE", "MAX", "ARGMIN", "SUM"), ("NONE", "SUM", "MAX", "ARGMIN"), ("NONE",), ("SUM", "MIN")]:
        ext = (3,) * len(ops)
        kind = oracle.out_kind(ext, [hp.OP_NAMES[o] for o in ops], 0)
        got = hp.inspect(ext, ops, hp.I32)["out_dtype"]
        assert got == {0: hp.I32, 1: hp.I64}[kind], ops
    assert hp.inspect((3, 3), ("NONE", "SUM"), hp.F32, flags=hp.FLAG_OUT_F32)["out_dtype"] == hp.F32


def test_scalar_chunk_when_extent_is_ragged():
    # blocks too short to hold an aligned vector wherever they start: one element per load
    assert hp.inspect((4, 6), ("NONE", "SUM"), hp.F32)["chunk"] == 1
    assert hp.inspect((4, 14), ("NONE", "SUM"), hp.BF16)["chunk"] == 1
    assert hp.inspect((4, 6, 3), ("NONE", "MAX", "ARGMIN"), hp.I32)["chunk"] == 1
    # long enough: flat blocks keep the 16-byte vector
    assert hp.inspect((4, 7), ("NONE", "SUM"), hp.F32)["chunk"] == 4
    assert hp.inspect((4, 8), ("NONE", "SUM"), hp.BF16)["chunk"] == 8
    assert hp.inspect((4, 8), ("NONE", "SUM"), hp.F32, flags=hp.FLAG_SCALAR)["chunk"] == 1


def test_batch_plans_are_wave_tasks_of_useful_size():
    import numpy as np

    import workloads
    bw = workloads.c4_batch(n=2000)
    nests = [(n.extents, n.ops, n.dtype) for n in bw.nests]
    infos = hp.batch_inspect(nests, 0x200)  # automatic maps, no tuner cache
    assert all(i["waves"] == 1 for i in infos)
    tasks = np.array([i["grid"] for i in infos])
    nbytes = np.array([i["in_bytes"] for i in infos])
    assert tasks.sum() < 4 * len(nests)           # small nests share tasks
    assert (nbytes / tasks).mean() > 8 << 10       # tasks carry kilobytes, not bytes
    for i, (ext, ops, dt) in zip(infos, nests):
        assert i["n_out"] == ext[0]


def test_ordered_products_plan_and_rejections():
    i = hp.inspect((4096, 16384), ("NONE", "PROD"), hp.AFFINE64)
    assert i["kernel"] == hp.KERNEL_ORDERED and i["out_dtype"] == hp.AFFINE64
    assert i["out_bytes"] == 4096 * 16 and i["in_bytes"] == 4096 * 16384 * 16
    assert i["workspace_bytes"] == (4096 * i["gsplit"] * 16 if i["gsplit"] > 1 else 0)
    one = hp.inspect((1, 1 << 22), ("NONE", "PROD"), hp.MAT2X2_64)
    assert one["gsplit"] > 1 and one["workspace_bytes"] == one["gsplit"] * 32
    # chunks cover the block exactly once
    span = -(-(1 << 22) // one["gsplit"])
    assert (one["gsplit"] - 1) * span < (1 << 22)
    assert err((4, 4), ("NONE", "PROD"), hp.I32) == "HP_EUNSUPPORTED"
    assert err((4, 4), ("NONE", "SUM"), hp.AFFINE64) == "HP_EUNSUPPORTED"
    assert err((4, 4), ("NONE", "PROD"), hp.MAT2X2_64, m=["G", "V"]) == "HP_EUNSUPPORTED"
    assert err((4, 4), ("NONE", "PROD"), hp.AFFINE64, flags=hp.FLAG_OUT_F32) == "HP_EINVAL"
    assert err((4, 4), ("PROD", "NONE"), hp.AFFINE64) == "HP_EINVAL"
    with pytest.raises(hp.HPError) as e:
        hp.batch_inspect([((4, 4), (0, hp.PROD), hp.AFFINE64)], 0)
    assert e.value.status_name == "HP_EUNSUPPORTED"


def test_stream_read_rejects_bad_arguments_without_a_device():
    L = hp.lib()
    assert L.hp_stream_read(None, 1024, None, 1, None) == 1                 # HP_EINVAL: null pointers
    assert L.hp_stream_read(16, 1000, 16, 1, None) == 1                     # size not a multiple of 16
    assert L.hp_stream_read(16, 1024, 16, 0, None) == 1                     # grid out of range


def test_stencil_plan_rejections():
    with pytest.raises(hp.HPError) as e:
        hp.Stencil(0, 10, 1, 0.5, 0.125)
    assert e.value.status_name == "HP_EINVAL"
    for kw in ({"tile_rows": 48}, {"sweeps_per_launch": 9}, {"flags": 2}):
        with pytest.raises(hp.HPError) as e:
            hp.Stencil(10, 10, 4, 0.5, 0.125, **kw)
        assert e.value.status_name == "HP_EINVAL", kw
    with pytest.raises(hp.HPError) as e:
        hp.Stencil(10, 10, 0, 0.5, 0.125)
    assert e.value.status_name == "HP_EINVAL"
    with pytest.raises(hp.HPError) as e:                            # more tiles than a launch holds
        hp.Stencil(1 << 31, 1 << 20, 1, 0.5, 0.125)
    assert e.value.status_name == "HP_EUNSUPPORTED"
    s = hp.Stencil(100, 200, 4, 0.5, 0.125)
    L = hp.lib()
    assert L.hp_stencil_run(s._h, None, None, None) == 1          # null arrays
    assert L.hp_stencil_run(s._h, 4096, 4096 + 64, None) == 1     # overlapping arrays
    s.close()


def test_stencil_plan_follows_the_workgroup_local_memory():
    """Tile rows and sweeps per launch follow the level-property table: every choice
    fits the W level's LDS; the 64-row tile is taken from 6 sweeps per launch when the
    array still gives the fill target of workgroups; a plan of one launch allocates
    nothing (these run without a device)."""
    rows, fill = hp.level_table()
    assert fill == 2048
    lds = next(r["shared_bytes"] for r in rows if r["scope"] == "W")

    def tile_bytes(th, t):
        return 2 * (th + 2 * t) * (64 + 2 * t + 1) * 4

    for (r, c, steps), want in {(100, 200, 4): (32, 4), (8192, 8192, 1): (32, 1), (8192, 8192, 4): (32, 4),
                                (8192, 8192, 5): (32, 5), (8192, 8192, 6): (64, 6), (8192, 8192, 8): (64, 8),
                                (1024, 8192, 8): (64, 8), (900, 8192, 8): (32, 8), (100, 200, 8): (32, 8)}.items():
        with hp.Stencil(r, c, steps, 0.6, 0.1) as s:
            i = s.info
            assert (i["tile_rows"], i["sweeps_per_launch"], i["launches"], i["tile_cols"]) == want + (1, 64)
            assert tile_bytes(i["tile_rows"], i["sweeps_per_launch"]) <= lds
    with hp.Stencil(300, 300, 5, 0.6, 0.1, tile_rows=64, sweeps_per_launch=5, flags=hp.STENCIL_NO_XCD) as s:
        assert s.info == {"tile_rows": 64, "tile_cols": 64, "sweeps_per_launch": 5, "launches": 1}


def test_xcd_scope_planning():
    """X: 8 grid units on the outermost grid digit (the XCD index under XCD-aware
    numbering), G for every other rule; the rejections name the broken rule."""
    c3 = ((64, 128, 64, 64), (hp.NONE, hp.SUM, hp.MAX, hp.ARGMIN), hp.I32)
    i = hp.inspect(*c3, ["X", ("GW", {"G": 16, "W": 8}), ("V", {"V": 16}), ("V", {"V": 4})])
    assert i["map"] == ["X", "GW", "V", "V"]
    assert i["units"][0][0] == 8 and i["grid"] == 8 * 16 and i["gsplit"] == 16
    i = hp.inspect((64, 64, 256), (hp.SUM, hp.SUM, hp.SUM), hp.F32, ["X", ("GW", {"G": 4, "W": 4}), "V"])
    assert i["map"] == ["X", "GW", "V"] and i["grid"] == 32 and i["gsplit"] == 32
    # a grid of exactly 8 (X alone, here collapsed with W): workgroup b is unit b
    i = hp.inspect((40, 64, 256), (hp.NONE, hp.SUM, hp.SUM), hp.F32, [("XW", {"W": 2}), ("W", {"W": 4}), "V"])
    assert i["map"][0] == "XW" and i["grid"] == 8 and i["units"][0] == (8, 2, 1)
    i = hp.inspect((4, 64), (hp.NONE, hp.SUM), hp.I32, ["X", "V"])
    assert i["grid"] == 8
    bad = [(c3, ["G", "X", "V", "L"], 0, "HP_EINVAL", "already uses the grid"),
           (c3, ["X", "GW", "V", "V"], hp.FLAG_NO_XCD, "HP_EINVAL", "NO_XCD"),
           (c3, ["X", "X", "V", "V"], 0, "HP_EINVAL", "both use"),
           (c3, [("X", {"G": 4}), "GW", "V", "V"], 0, "HP_EINVAL", "8 units"),
           (c3, ["XG", "W", "V", "V"], 0, "HP_EINVAL", "both X and G")]
    for (ext, ops, dt), m, fl, status, words in bad:
        with pytest.raises(hp.HPError) as e:
            hp.inspect(ext, ops, dt, m, fl)
        assert e.value.status_name == status and words in str(e.value), (m, str(e.value))


def test_flat_block_planning():
    """A single SUM / MIN / MAX reduction whose block is not a multiple of the 16-byte
    vector is planned as the aligned interior of each output's contiguous block (16-byte
    loads) plus a rest spread over the output's threads; other nests keep their plans."""
    cases = [((4096, 65537), ("NONE", "SUM"), hp.F32, 4), ((7, 3, 5, 7), ("NONE", "SUM", "SUM", "SUM"), hp.BF16, 8),
             ((100, 101), ("NONE", "MAX"), hp.I32, 4), ((1, 1000003), ("SUM", "SUM"), hp.F32, 4),
             ((3, 1001), ("NONE", "MIN"), hp.I32, 4), ((9, 2, 3, 5), ("NONE", "SUM", "SUM", "SUM"), hp.F32, 4)]
    for ext, ops, dt, c in cases:
        i = hp.inspect(ext, ops, dt)
        p = next(k for k, o in enumerate(ops) if o != "NONE")
        block = int(np.prod(ext[p:]))
        assert i["flat_block"] == block, (ext, i)
        assert i["in_elems"] == int(np.prod(ext)) and i["chunk"] == c
        assert i["depth"] == p + 1  # the interior view: one reducing level
    # the interior of a long row is whole strips: the stream stays unmasked
    i = hp.inspect((4096, 65537), ("NONE", "SUM"), hp.F32)
    span = i["units"][1][1] * i["units"][1][2] * 4
    assert i["strips"][1] * span <= 65537 - 3 and i["kernel_name"] == "hp::k_nest_f32_lean_flat<4>"
    # not flat: several segments, ARG, an explicit map, the scalar flag, blocks too short
    for ext, ops, dt, m, fl in [((64, 128, 64, 63), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32, None, 0),
                                ((10, 1001), ("NONE", "ARGMIN"), hp.I32, None, 0),
                                ((10, 1001), ("NONE", "SUM"), hp.F32, ["G", "V"], 0),
                                ((10, 1001), ("NONE", "SUM"), hp.F32, None, hp.FLAG_SCALAR),
                                ((10, 14), ("NONE", "SUM"), hp.BF16, None, 0),
                                ((10, 1024), ("NONE", "SUM"), hp.F32, None, 0)]:
        i = hp.inspect(ext, ops, dt, m, fl)
        assert i["flat_block"] == 0, (ext, ops, m, fl)
    # batched plans (default recipes and the committed tuner cache) use flat blocks too
    nests = [((8, 3, 333), ("NONE", "SUM", "SUM"), hp.BF16), ((1, 5, 4099), ("NONE", "SUM", "SUM"), hp.BF16)]
    infos = hp.batch_inspect(nests)
    assert all(x["flat_block"] == int(np.prod(n[0][1:])) for x, n in zip(infos, nests)), infos


def test_static_entry_host_errors():
    """hp_reduce_static rejects bad pointers and over-size nests before touching a device."""
    import ctypes
    L = hp.lib()
    n = hp.make_nest((8192, 1024), (0, 1), hp.F32)
    m = hp.make_map(["G", ("G", {"G": 64})])  # 8192 outputs x 64 partials x 16 B = 8 MiB of partials
    assert L.hp_reduce_static(ctypes.byref(n), ctypes.byref(m), 0, 4096, 4096, None) == 6  # HP_ETOOBIG
    assert b"static scratch" in L.hp_last_error()
    assert L.hp_reduce_static(ctypes.byref(n), None, 0, None, 4096, None) == 1  # null input
    assert L.hp_reduce_static(ctypes.byref(n), None, 0, 4100, 4096, None) == 1  # misaligned input
    assert L.hp_reduce_static(ctypes.byref(n), None, 0, 4096, 4100, None) == 1  # misaligned fp64 output
    bad = hp.make_nest((4, 0), (0, 1), hp.F32)
    assert L.hp_reduce_static(ctypes.byref(bad), None, 0, 4096, 4096, None) == 1  # extent < 1


def test_int_kernel_choice():
    """Integer plans: a chain of single-level segments that divides evenly goes to the
    chain kernel; masked levels to the segmented kernel; an ARG level over int64 sums
    (its (value, index) does not pack into one 64-bit key) to the general kernel."""
    i = hp.inspect((64, 128, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32)
    assert i["kernel"] == hp.KERNEL_INT_CHAIN and i["kernel_name"] == "hp::k_nest_i32_chain<4, 3>"
    i = hp.inspect((64, 128, 64), ("NONE", "MAX", "ARGMAX"), hp.I32)
    assert i["kernel"] == hp.KERNEL_INT_CHAIN and i["kernel_name"] == "hp::k_nest_i32_chain<5, 2>"
    assert hp.inspect((64, 100, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32)["kernel"] == hp.KERNEL_INT_SEG
    assert hp.inspect((64, 128, 60, 64), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32)["kernel"] == hp.KERNEL_INT_SEG
    assert hp.inspect((64, 128, 64), ("NONE", "ARGMIN", "SUM"), hp.I32)["kernel"] == hp.KERNEL_INT_DEEP
    assert hp.inspect((64, 128, 64), ("NONE", "ARGMIN", "MAX"), hp.I32)["kernel"] == hp.KERNEL_INT_CHAIN
    assert hp.inspect((64, 128, 64, 64), ("NONE", "SUM", "SUM", "MAX"), hp.I32)["kernel"] == hp.KERNEL_INT_SEG


def test_level_table_and_automatic_maps_follow_it():
    """The level-property table (the analogue of the paper's Table 2) and the automatic
    map's choices: a reducing level's lanes are on the level that shuffles, its waves on
    the level with a barrier and shared memory, the grid (no barrier) only through a
    fold; lanes and waves within the table's unit counts; the outermost reducing level
    split over the grid only when the outputs alone give fewer workgroups than the
    table's fill target; and never the XCD level (its shared cache pays only for data
    read more than once)."""
    rows, fill = hp.level_table()
    by = {r["scope"]: r for r in rows}
    assert [r["scope"] for r in rows] == ["G", "X", "W", "V", "L"]
    assert by["V"]["props"] & hp.LP_SHUFFLE and by["V"]["units"] == 64
    assert by["W"]["props"] & hp.LP_BARRIER and by["W"]["props"] & hp.LP_LOCALMEM and by["W"]["units"] == 16
    assert not by["G"]["props"] & (hp.LP_BARRIER | hp.LP_SHUFFLE) and by["X"]["units"] == 8
    assert fill == 2048
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(300):
        depth = int(rng.integers(2, 5))
        ext = tuple(int(x) for x in rng.integers(1, 300, size=depth))
        p = int(rng.integers(0, depth))
        ops = ["NONE"] * p + [str(rng.choice(["SUM", "MIN", "MAX", "ARGMIN"])) for _ in range(depth - p)]
        try:
            i = hp.inspect(ext, ops, hp.I32)
        except hp.HPError:
            continue
        if i["flat_block"]:
            continue
        checked += 1
        n_out = int(np.prod(ext[:p])) if p else 1
        lanes = waves = 1
        for lvl in range(i["depth"]):
            sc = i["map"][lvl]
            assert "X" not in sc, (ext, ops, i["map"])
            g, w, v = i["units"][lvl]
            lanes *= v
            waves *= w
            # one or two reducing levels fit a workgroup's lanes and waves: one on the
            # grid as well is only ever a split to fill the chip
            if lvl >= p and g > 1 and depth - p <= 2:
                assert n_out < fill and i["gsplit"] > 1, (ext, ops, i["map"], i["units"])
        assert lanes <= by["V"]["units"] and waves <= by["W"]["units"], (ext, ops, i["units"])
    assert checked > 150


def test_grid_split_and_wave_rules():
    """The automatic map's measured rules: outputs below half the 2,048-workgroup fill
    target split their outermost reducing level (floats over 4,096 workgroups of at most
    4 waves, integers over 2,048), 1,024 outputs run in one pass, and unsplit float
    plans of at most 1,024 outputs with 256-384 KiB blocks take 2 waves."""
    one_f = hp.inspect((1, 1 << 28), ("NONE", "SUM"), hp.F32)
    assert one_f["grid"] == 4096 and one_f["gsplit"] == 4096 and one_f["waves"] == 4
    one_i = hp.inspect((1, 1 << 26), ("NONE", "MAX"), hp.I32)
    assert one_i["grid"] == 2048 and one_i["gsplit"] == 2048
    few = hp.inspect((256, 1 << 20), ("NONE", "SUM"), hp.F32)
    assert few["grid"] == 4096 and few["gsplit"] == 16 and few["waves"] == 4
    for ext, dt, ops in [((1024, 65536), hp.I32, ("NONE", "SUM")), ((1024, 1 << 18), hp.F32, ("NONE", "SUM"))]:
        i = hp.inspect(ext, ops, dt)
        assert i["gsplit"] == 1 and i["grid"] == 1024, (ext, i["units"])
    assert hp.inspect((1024, 65536), ("NONE", "SUM"), hp.F32)["waves"] == 2
    assert hp.inspect((1024, 131072), ("NONE", "SUM"), hp.BF16)["waves"] == 2
    assert hp.inspect((1024, 98304), ("NONE", "SUM"), hp.F32)["waves"] == 8     # 384 KiB blocks
    assert hp.inspect((1024, 1 << 18), ("NONE", "SUM"), hp.F32)["waves"] == 8   # 1 MiB blocks
    assert hp.inspect((4096, 65536), ("NONE", "SUM"), hp.F32)["waves"] == 8     # 4,096 outputs
    # the 4-level integer chain keeps 16 workgroups per output
    c3 = hp.inspect((64, 128, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN"), hp.I32)
    assert c3["gsplit"] == 16 and c3["grid"] == 1024


def test_sums_of_sums_run_as_one_level_when_that_is_lean():
    for ext, dt in [((4096, 8, 1024), hp.F32), ((2048, 4, 8, 1024), hp.BF16), ((8192, 4, 2048), hp.F32)]:
        ops = ("NONE",) + ("SUM",) * (len(ext) - 1)
        i = hp.inspect(ext, ops, dt)
        assert i["depth"] == 2 and i["kernel"] == hp.KERNEL_LEAN, (ext, i["kernel_name"])
        assert i["n_out"] == ext[0] and i["in_elems"] == int(np.prod(ext))
        nested = hp.inspect(ext, ops, dt, ["G"] * (len(ext) - 2) + [("W", {"W": 2}), "V"])
        assert nested["depth"] == len(ext) and nested["kernel"] != hp.KERNEL_LEAN
        assert hp.inspect(ext, ops, dt, flags=hp.FLAG_GENERIC)["depth"] == len(ext)
    # already lean as nested (the headline): unchanged
    c2 = hp.inspect((4096, 256, 256), ("NONE", "SUM", "SUM"), hp.F32)
    assert c2["depth"] == 3 and c2["kernel"] == hp.KERNEL_LEAN
    # integers keep their nested plan
    assert hp.inspect((4096, 8, 1024), ("NONE", "SUM", "SUM"), hp.I32)["depth"] == 3
