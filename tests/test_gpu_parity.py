"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on seeded
inputs.  Integer, MIN/MAX and ARG results must be bit-exact; float sums must be
within |got - ref| <= 1e-6 * max(|ref|, 2^-24 * sum|a|) of the fp64 oracle."""
import itertools

import numpy as np
import pytest

import workloads
from gpu_util import assert_match, gpu_reduce, say, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_01906_amd as hp
    hp.lib()  # fails loudly if libhp.so is missing
    yield


# --------------------------------------------------------------------------
# the workloads at their full sizes


def test_c1_full_bit_exact():
    say("case c1 1024x1024 int32 SUM")
    x = workloads.c1_input()
    got, info = gpu_reduce(x, x.shape, ("NONE", "SUM"))
    assert_match(got, x, x.shape, ("NONE", "SUM"), what="c1")


def test_c2_reduced_rows_full_parity():
    say("case c2 shape 64x256x256 fp32")
    x = workloads.c2_input((64, 256, 256))
    got, info = gpu_reduce(x, x.shape, ("NONE", "SUM", "SUM"))
    assert got.dtype == np.float64
    assert_match(got, x, x.shape, ("NONE", "SUM", "SUM"), what="c2 small")


C3_OPS = ("NONE", "SUM", "MAX", "ARGMIN")
C3_MAPS = [
    None,
    ["G", "W", "V", "L"],                                   # the literal map of the workload
    ["G", ("GW", {"G": 8, "W": 4}), "V", "L"],              # level 1 split over the grid
    ["G", "W", ("V", {"V": 4}), ("V", {"V": 16})],          # partitions of 16 lanes
    ["G", ("W", {"W": 16}), "L", "L"],                       # lanes idle: level 2 and 3 serial
    ["G", "GW", ("WV", {"W": 2, "V": 8}), ("V", {"V": 8})],  # waves split between two levels
    [("GW", {"G": 16, "W": 4}), "L", "L", "L"],              # outputs over workgroups and waves
]


def test_c3_full_bit_exact_and_map_independent():
    x = workloads.c3_input()
    first = None
    for m in C3_MAPS:
        say("case c3 map", m)
        got, info = gpu_reduce(x, x.shape, C3_OPS, m)
        if first is None:
            assert_match(got, x, x.shape, C3_OPS, what=f"c3 map {m}")
            first = got
        else:
            np.testing.assert_array_equal(got, first, err_msg=f"c3 map {m}")


# --------------------------------------------------------------------------
# every monotone map of small nests, integer and float, ragged extents

SCOPE_SETS = ["G", "W", "V", "L", "GW", "WV", "VL", "GWV", "WVL", "GWVL"]
ORDER = "GWVL"


def monotone(m):
    for i, b in enumerate(m):
        for a in m[:i]:
            hi = a[-1] if a == "L" else a.replace("L", "")[-1]
            if ORDER.index(b[0]) < ORDER.index(hi):
                return False
    return True


def maps(depth):
    return [list(m) for m in itertools.product(SCOPE_SETS, repeat=depth) if monotone(m)]


INT_CHAINS_2 = [("NONE", "SUM"), ("NONE", "MIN"), ("NONE", "ARGMAX"), ("SUM", "SUM"), ("ARGMIN", "SUM"),
                ("NONE", "NONE")]
INT_CHAINS_3 = [("NONE", "SUM", "SUM"), ("NONE", "MAX", "ARGMIN"), ("NONE", "SUM", "MIN"), ("SUM", "ARGMAX", "MAX"),
                ("NONE", "NONE", "ARGMIN")]


@pytest.mark.parametrize("depth", [2, 3])
def test_all_maps_int(depth):
    import paper_2309_01906_amd as hp
    ext = (5, 37) if depth == 2 else (3, 7, 36)
    chains = INT_CHAINS_2 if depth == 2 else INT_CHAINS_3
    x = workloads.uniform_i32(40 + depth, ext, -3, 3)
    dev = to_device(x)
    n = 0
    for ops in chains:
        for m in maps(depth):
            try:
                got, info = gpu_reduce(x, ext, ops, m, dev=dev)
            except hp.HPError as e:
                assert e.status_name == "HP_EUNSUPPORTED", (ops, m, str(e))
                continue
            assert_match(got, x, ext, ops, what=f"ops {ops} map {m}")
            n += 1
    say("int maps checked:", n)
    assert n > 50


@pytest.mark.parametrize("depth", [2, 3])
def test_all_maps_float(depth):
    import paper_2309_01906_amd as hp
    ext = (5, 1000) if depth == 2 else (3, 9, 68)
    x = workloads.normal_f32(50 + depth, ext)
    dev = to_device(x)
    n = 0
    for ops in [("NONE",) + ("SUM",) * (depth - 1), ("SUM",) * depth]:
        for m in maps(depth):
            try:
                got, info = gpu_reduce(x, ext, ops, m, dev=dev)
            except hp.HPError as e:
                assert e.status_name == "HP_EUNSUPPORTED", (ops, m, str(e))
                continue
            assert_match(got, x, ext, ops, what=f"ops {ops} map {m}")
            n += 1
    say("float maps checked:", n)


def test_depth4_maps_sampled():
    ext = (3, 5, 6, 12)
    x = workloads.uniform_i32(61, ext, 0, 5)
    dev = to_device(x)
    rng = np.random.default_rng(3)
    all4 = maps(4)
    picks = [all4[i] for i in rng.choice(len(all4), size=min(120, len(all4)), replace=False)]
    for ops in [C3_OPS, ("NONE", "ARGMAX", "MIN", "SUM"), ("NONE", "NONE", "SUM", "SUM")]:
        for m in picks:
            try:
                got, _ = gpu_reduce(x, ext, ops, m, dev=dev)
            except Exception as e:  # only unsupported maps may be refused
                assert "HP_EUNSUPPORTED" in str(e), (ops, m, str(e))
                continue
            assert_match(got, x, ext, ops, what=f"ops {ops} map {m}")


# --------------------------------------------------------------------------
# edge cases


@pytest.mark.parametrize("ext,ops", [
    ((1,), ("SUM",)), ((1,), ("NONE",)), ((37,), ("NONE",)), ((1, 1, 1), ("NONE", "SUM", "ARGMIN")),
    ((5, 1), ("NONE", "ARGMAX")), ((1, 100003), ("NONE", "SUM")), ((3, 1, 64), ("NONE", "MAX", "SUM")),
    ((2, 3, 1, 5, 7), ("NONE", "SUM", "MAX", "ARGMIN", "SUM")),
    ((2, 2, 2, 2, 2, 2, 2, 5), ("NONE",) + ("SUM", "MAX", "ARGMIN", "SUM", "MIN", "ARGMAX", "MAX")),
    ((1, 1 << 22), ("NONE", "SUM")), ((1, 1 << 22), ("NONE", "ARGMIN")),
])
def test_edge_shapes_int(ext, ops):
    say("case edge int", ext, ops)
    x = workloads.uniform_i32(70, ext, -(2**31), 2**31 - 1)
    got, _ = gpu_reduce(x, ext, ops)
    assert_match(got, x, ext, ops, what=f"{ext} {ops}")


@pytest.mark.parametrize("ext,ops", [
    ((1,), ("SUM",)), ((7, 3), ("NONE", "NONE")), ((1, 1 << 22), ("NONE", "SUM")), ((3, 1001), ("NONE", "SUM")),
    ((2, 3, 5, 7, 11), ("NONE", "SUM", "SUM", "SUM", "SUM")), ((1, 1 << 26), ("NONE", "SUM")),
])
def test_edge_shapes_float(ext, ops):
    say("case edge float", ext, ops)
    x = workloads.normal_f32(71, ext)
    got, _ = gpu_reduce(x, ext, ops)
    assert_match(got, x, ext, ops, what=f"{ext} {ops}")


@pytest.mark.parametrize("ext,ops,lo,hi", [
    ((20011, 1), ("NONE", "ARGMIN"), -5, 5), ((7001, 3, 5), ("NONE", "SUM", "ARGMIN"), 0, 3),
    ((6482, 2, 64), ("NONE", "MAX", "MAX"), -(2**31), 2**31 - 1), ((3, 999, 2, 3), ("NONE", "NONE", "MIN", "ARGMAX"), 0, 2),
    ((100003, 2), ("NONE", "SUM"), -(2**31), 2**31 - 1),
])
def test_packed_outputs_int(ext, ops, lo, hi):
    """Small blocks: the innermost output level shares the wave's lanes with the
    reduced block (several outputs per wave), with ragged strips and ARG ties."""
    say("case packed int", ext, ops)
    x = workloads.uniform_i32(75, ext, lo, hi)
    got, info = gpu_reduce(x, ext, ops)
    p = next(i for i, o in enumerate(ops) if o != "NONE")
    assert "V" in info["map"][p - 1], info["map"]
    assert_match(got, x, ext, ops, what=f"packed {ext} {ops}")


@pytest.mark.parametrize("ext", [(4097, 7), (9999, 3, 3), (50001, 12)])
def test_packed_outputs_float(ext):
    say("case packed float", ext)
    ops = ("NONE",) + ("SUM",) * (len(ext) - 1)
    x = workloads.normal_f32(76, ext)
    got, info = gpu_reduce(x, ext, ops)
    assert "V" in info["map"][0], info["map"]
    assert_match(got, x, ext, ops, what=f"packed {ext}")


def test_int_sum_of_int32_min_needs_64_bits():
    x = np.full((4, 4096), np.iinfo(np.int32).min, np.int32)
    got, _ = gpu_reduce(x, x.shape, ("NONE", "SUM"))
    np.testing.assert_array_equal(got, np.full(4, -(2**31) * 4096, np.int64))


def test_argmin_ties_first_occurrence():
    for ext in [(8, 64), (4, 1 << 20), (2, 3, 1000)]:
        x = workloads.uniform_i32(72, ext, 0, 1)
        ops = ("NONE",) * (len(ext) - 1) + ("ARGMIN",)
        got, _ = gpu_reduce(x, ext, ops)
        assert_match(got, x, ext, ops, what=f"ties {ext}")


@pytest.mark.parametrize("fill", ["max", "min"])
def test_arg_rows_of_extreme_values(fill):
    """Rows made only of the value a masked-out lane folds in (INT32_MAX under
    MIN / ARGMIN, INT32_MIN under MAX / ARGMAX), beside random rows, with ragged
    tails and chunk-internal ties: the first position of the row must still win."""
    v = np.iinfo(np.int32).max if fill == "max" else np.iinfo(np.int32).min
    op, argop = ("MIN", "ARGMIN") if fill == "max" else ("MAX", "ARGMAX")
    cases = [((5, 67), ("NONE", argop)), ((3, 1001), ("NONE", argop)), ((6, 4096), ("NONE", argop)),
             ((2, 3, 5, 131), ("NONE", "SUM", op, argop)), ((64, 7, 3, 13), ("NONE", "SUM", op, argop)),
             ((4, 9, 64, 64), ("NONE", "SUM", op, argop)), ((7, 33), ("NONE", op))]
    for ext, ops in cases:
        say("case extreme rows", fill, ext, ops)
        x = workloads.uniform_i32(77, ext, -3, 3)
        rows = x.reshape(-1, ext[-1])
        rows[::2] = v
        got, _ = gpu_reduce(x, ext, ops)
        assert_match(got, x, ext, ops, what=f"extreme {fill} {ext} {ops}")


def test_xcd_scope_maps():
    """Levels placed on the XCD scope give the oracle's results (bit-exact for
    integers, and the same bits as the automatic map), for an output level and
    for a reducing level on X."""
    import paper_2309_01906_amd as hp
    c3 = workloads.C3
    x = workloads.c3_input()
    dev = to_device(x)
    ops = c3.ops
    auto, _ = gpu_reduce(x, c3.extents, ops, dev=dev)
    m = ["X", ("GW", {"G": 16, "W": 8}), ("V", {"V": 16}), ("V", {"V": 4})]
    got, info = gpu_reduce(x, c3.extents, ops, m, dev=dev)
    say("case xcd c3", info["map"], info["grid"])
    assert info["map"][0] == "X"
    np.testing.assert_array_equal(got, auto)
    assert_match(got, x, c3.extents, ops, what="X map c3")
    n = 0
    for ext, ops, m in [((64, 64, 256), ("SUM", "SUM", "SUM"), ["X", ("GW", {"G": 4, "W": 4}), "V"]),
                        ((40, 64, 256), ("NONE", "SUM", "SUM"), [("XW", {"W": 2}), ("W", {"W": 4}), "V"]),
                        ((3, 1000, 100), ("NONE", "SUM", "SUM"), ["X", ("GW", {"G": 2, "W": 2}), "V"])]:
        xf = workloads.normal_f32(78, ext)
        got, info = gpu_reduce(xf, ext, ops, m)
        say("case xcd float", ext, info["map"], info["grid"])
        assert info["map"][0].startswith("X")
        assert_match(got, xf, ext, ops, what=f"X map {ext}")
        n += 1
    assert n == 3


def test_xcd_ids_follow_the_x_digit():
    """The XCD-aware numbering assumes the dispatcher deals workgroups round-robin to
    the 8 XCDs, so that workgroups b and b' share an XCD (and its L2) exactly when
    b = b' mod 8: the X digit of a plan then names one XCD's workgroups.  (Which XCD
    takes workgroup 0 depends on where the previous launch stopped, so the test
    checks the partition, not the index.)  The hardware's XCC_ID register of every
    workgroup, for the launch shapes of X-mapped plans, of the benchmarked nests and
    of large grids, must be (b + c) mod 8 for one c per launch."""
    import paper_2309_01906_amd as hp
    shapes = []
    for ext, ops, m in [(workloads.C3.extents, workloads.C3.ops,
                         ["X", ("GW", {"G": 16, "W": 8}), ("V", {"V": 16}), ("V", {"V": 4})]),
                        ((64, 64, 256), (1, 1, 1), ["X", ("GW", {"G": 4, "W": 4}), "V"]),
                        ((3, 1000, 100), (0, 1, 1), ["X", ("GW", {"G": 2, "W": 2}), "V"])]:
        inf = hp.inspect(ext, ops, hp.I32 if ext == workloads.C3.extents else hp.F32, m)
        shapes.append((inf["grid"], 64 * inf["waves"], inf["lds_bytes"]))
    for nest in (workloads.C2, workloads.C3):
        inf = hp.inspect(nest.extents, nest.ops, nest.dtype)
        shapes.append((inf["grid"], 64 * inf["waves"], inf["lds_bytes"]))
    shapes += [(8, 64, 0), (4096, 1024, 0), (65536, 256, 0)]
    for grid, threads, lds in shapes:
        ids = hp.xcd_ids(grid, threads, lds).cpu().numpy()
        torch.cuda.synchronize()
        want = (np.arange(grid) + ids[0]) % 8
        say("case xcd ids", grid, threads, lds, "workgroup 0 on XCD", int(ids[0]))
        np.testing.assert_array_equal(ids, want, err_msg=f"grid {grid} threads {threads}")


def test_flags_scalar_out_f32_noxcd_generic():
    import paper_2309_01906_amd as hp
    x = workloads.normal_f32(73, (256, 4096))
    for fl in [hp.FLAG_SCALAR, hp.FLAG_OUT_F32, hp.FLAG_NO_XCD, hp.FLAG_GENERIC]:
        got, info = gpu_reduce(x, x.shape, ("NONE", "SUM"), flags=fl)
        if fl == hp.FLAG_OUT_F32:
            assert got.dtype == np.float32
        assert_match(got.astype(np.float64), x, x.shape, ("NONE", "SUM"), what=f"flag {fl}")
    xi = workloads.uniform_i32(74, (256, 4096), -5, 5)
    got, _ = gpu_reduce(xi, xi.shape, ("NONE", "ARGMAX"), flags=hp.FLAG_SCALAR)
    assert_match(got, xi, xi.shape, ("NONE", "ARGMAX"), what="int scalar")


def test_bf16_nests():
    for ext in [(4, 64, 64), (64, 3, 64), (1, 2048, 64), (3, 5, 8), (2, 7)]:
        x = workloads.normal_bf16_bits(75, ext)
        ops = ("NONE",) + ("SUM",) * (len(ext) - 1)
        got, _ = gpu_reduce(x, ext, ops)
        assert_match(got, x, ext, ops, what=f"bf16 {ext}")


def test_grid_combine_nested_segments():
    # level 1 (ARGMAX) and level 2 (SUM) both span workgroups: partials folded per
    # output in nest order by the last workgroup
    ext = (3, 5, 4096)
    x = workloads.uniform_i32(76, ext, -100, 100)
    for ops, m in [(("NONE", "ARGMAX", "SUM"), ["G", "G", ("GWV", {"G": 4})]),
                   (("NONE", "MIN", "SUM"), ["G", ("G", {"G": 5}), ("GW", {"G": 8, "W": 2})]),
                   (("NONE", "SUM", "MAX"), ["G", ("G", {"G": 8}), ("GWV", {"G": 3, "W": 1})])]:
        got, info = gpu_reduce(x, ext, ops, m)
        assert info["gsplit"] > 1
        assert_match(got, x, ext, ops, what=f"nested {ops} {m}")


def test_sum_of_sums_collapsed_to_one_level():
    """A float nest whose automatic plan would iterate two levels in a thread is run
    as one level per output block: the result matches the oracle's nested sums, and
    the explicit nested map gives the general kernel on the same data."""
    import paper_2309_01906_amd as hp
    for ext, dt in [((64, 16, 1024), hp.F32), ((32, 4, 8, 1024), hp.F32), ((128, 4, 2048), hp.BF16),
                    ((48, 64, 512), hp.F32), ((5, 8, 8, 1024), hp.BF16), ((9, 4, 8, 512), hp.F32)]:
        ops = ("NONE",) + ("SUM",) * (len(ext) - 1)
        x = workloads.normal_f32(80, ext) if dt == hp.F32 else workloads.normal_bf16_bits(80, ext)
        got, info = gpu_reduce(x, ext, ops)
        assert info["depth"] == 2 and "lean" in info["kernel_name"], (ext, info["kernel_name"], info["map"])
        assert_match(got, x, ext, ops, what=f"collapsed {ext}")
        nested = ["G"] * (len(ext) - 2) + [("W", {"W": 2}), "V"]
        got2, info2 = gpu_reduce(x, ext, ops, nested)
        assert info2["depth"] == len(ext) and "lean" not in info2["kernel_name"]
        assert_match(got2, x, ext, ops, what=f"nested {ext}")
        say("collapsed", ext, info["kernel_name"], info["map"], "| nested", info2["kernel_name"])


def test_integer_grid_fold_on_lane_and_on_wave():
    """One grid-spanning integer segment folds its partials on one lane up to 16
    workgroups and on a whole wave beyond: both give the oracle's bits, ties of the
    ARG operators included (values from a range of 7 repeat millions of times)."""
    ext = (3, 1 << 21)
    x = workloads.uniform_i32(79, ext, -3, 3)
    dev = to_device(x)
    for op in ("SUM", "MIN", "MAX", "ARGMIN", "ARGMAX"):
        outs = []
        for g in (4, 16, 17, 64, 1024, 4096):
            got, info = gpu_reduce(x, ext, ("NONE", op), ["G", ("GWV", {"G": g, "W": 2})], dev=dev)
            assert info["gsplit"] == g
            assert_match(got, x, ext, ("NONE", op), what=f"{op} G={g}")
            outs.append(got)
        for o in outs[1:]:
            np.testing.assert_array_equal(o, outs[0])
        say("int fold", op, "bit-identical over G = 4 .. 4096")


def test_plan_reuse_and_determinism():
    import paper_2309_01906_amd as hp
    x1 = workloads.normal_f32(77, (4, 1 << 20))
    x2 = workloads.normal_f32(78, (4, 1 << 20))
    d1, d2 = to_device(x1), to_device(x2)
    with hp.Plan((4, 1 << 20), (0, 1), hp.F32) as p:
        assert p.info["gsplit"] > 1
        outs = []
        for d in (d1, d2, d1, d1):
            outs.append(p.run(d).cpu().numpy())
    assert_match(outs[0], x1, x1.shape, ("NONE", "SUM"), what="reuse 1")
    assert_match(outs[1], x2, x2.shape, ("NONE", "SUM"), what="reuse 2")
    np.testing.assert_array_equal(outs[0], outs[2])
    np.testing.assert_array_equal(outs[0], outs[3])


def test_run_rejects_bad_pointers():
    import ctypes

    import paper_2309_01906_amd as hp
    x = to_device(workloads.uniform_i32(79, (16, 64), 0, 9))
    with hp.Plan((16, 64), (0, 1), hp.I32) as p:
        out = p.empty_out(x.device)
        st = hp.lib().hp_run(p._h, ctypes.c_void_p(x.data_ptr() + 4), ctypes.c_void_p(out.data_ptr()), None)
        assert hp.STATUS[st] == "HP_EINVAL"
        st = hp.lib().hp_run(p._h, None, ctypes.c_void_p(out.data_ptr()), None)
        assert hp.STATUS[st] == "HP_EINVAL"
        st = hp.lib().hp_run(None, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
        assert hp.STATUS[st] == "HP_EINVAL"


@pytest.mark.parametrize("ext,op,kind", [
    ((4096, 65537), "SUM", "f32"), ((3, 1001), "SUM", "f32"), ((9, 2, 3, 5), "SUM", "f32"),
    ((1, 1000003), "SUM", "f32"), ((6482, 15), "SUM", "f32"), ((2, 3000017), "SUM", "f32"),
    ((100, 101), "MAX", "i32"), ((333, 77), "MIN", "i32"), ((77, 5, 13), "SUM", "i32"), ((3, 1 << 20 | 3), "MAX", "i32"),
    ((7, 3, 5, 7), "SUM", "bf16"), ((513, 1023), "SUM", "bf16"), ((2, 100003), "SUM", "bf16"), ((4099, 9), "SUM", "bf16"),
])
def test_flat_blocks(ext, op, kind):
    """Blocks that are not a multiple of the 16-byte vector, at every offset modulo the
    vector: the aligned interior streams with 16-byte loads and the elements around it
    are spread over the output's threads; results equal the oracle's."""
    import paper_2309_01906_amd as hp
    ops = ("NONE",) + (op,) * (len(ext) - 1) if ext[0] != 1 else (op,) * len(ext)
    if kind == "f32":
        x = workloads.normal_f32(81, ext)
    elif kind == "bf16":
        x = workloads.normal_bf16_bits(82, ext)
    else:
        x = workloads.uniform_i32(83, ext, -(2**31), 2**31 - 1)
    say("case flat", ext, op, kind)
    got, info = gpu_reduce(x, ext, ops)
    b = int(np.prod(ext[1:] if ops[0] == "NONE" else ext))
    c = 8 if kind == "bf16" else 4
    # a block shorter than 2c - 1 elements may hold no aligned vector: plain path
    assert info["flat_block"] == (b if b >= 2 * c - 1 else 0), info
    assert_match(got, x, ext, ops, what=f"flat {ext} {op} {kind}")


CHAIN_CASES = [
    # (extents, ops): chains of single-level segments that divide evenly
    ((64, 128, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN")),
    ((16, 32, 64, 64), ("NONE", "MIN", "ARGMAX", "MAX")),
    ((8, 16, 32, 128), ("NONE", "MAX", "SUM", "MIN")),
    ((32, 64, 256), ("NONE", "SUM", "ARGMIN")),
    ((32, 64, 256), ("NONE", "ARGMAX", "MIN")),
    ((128, 32, 64), ("NONE", "MIN", "SUM")),
    ((4, 64, 64, 64), ("NONE", "ARGMIN", "ARGMAX", "ARGMIN")),
    ((16, 64, 64), ("SUM", "MAX", "ARGMAX")),
]


@pytest.mark.parametrize("ext,ops", CHAIN_CASES)
@pytest.mark.parametrize("values", ["wide", "ties", "extreme"])
def test_chain_kernel(ext, ops, values):
    """The chain kernel (one operator per reducing level, every level divided evenly):
    every innermost operator, 2- and 3-level chains, random values over the full int32
    range, tie-heavy values in [0, 4) and rows of the extreme value a masked lane would
    fold in; bit-exact against the oracle."""
    import paper_2309_01906_amd as hp
    inf = hp.inspect(ext, [hp.OP_NAMES[o] for o in ops], hp.I32)
    assert inf["kernel"] == hp.KERNEL_INT_CHAIN, inf["kernel_name"]
    if values == "wide":
        x = workloads.uniform_i32(91, ext, -(2**31), 2**31 - 1)
    elif values == "ties":
        x = workloads.uniform_i32(92, ext, 0, 3)
    else:
        x = workloads.uniform_i32(93, ext, -3, 3)
        rows = x.reshape(-1, ext[-1])
        rows[::3] = np.iinfo(np.int32).max if ops[-1] in ("MIN", "ARGMIN") else np.iinfo(np.int32).min
    say("case chain", ext, ops, values, inf["kernel_name"], "gsplit", inf["gsplit"])
    got, _ = gpu_reduce(x, ext, ops)
    assert_match(got, x, ext, ops, what=f"chain {ext} {ops} {values}")
