"""Pins for the CPU oracle: closed forms, exactly rounded sums, numpy library
reductions, brute force on tiny nests and invariants.  None of these calls the
GPU library; each is chosen so that a plausible slip in the oracle (a dropped
term, a wrong index or stride, a wrong tie rule, a missing compensation branch,
an int32 accumulator) makes at least one of them fail."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

NONE, SUM, MIN, MAX, ARGMIN, ARGMAX = 0, 1, 2, 3, 4, 5
I32, F32, BF16 = 0, 1, 2


# ---------------------------------------------------------------------------
# library-based evaluator: reduce the last axis repeatedly with numpy.
# np.argmin/np.argmax return the first occurrence, which is the tie rule.

def numpy_eval(x, ops):
    v = np.asarray(x, dtype=np.int64)
    for op in reversed(ops):
        if op == NONE:
            break
        if op == SUM:
            v = v.sum(axis=-1, dtype=np.int64)
        elif op == MIN:
            v = v.min(axis=-1)
        elif op == MAX:
            v = v.max(axis=-1)
        elif op == ARGMIN:
            v = v.argmin(axis=-1).astype(np.int64)
        elif op == ARGMAX:
            v = v.argmax(axis=-1).astype(np.int64)
    return v.reshape(-1)


# ---------------------------------------------------------------------------
# integer SUM closed forms


def test_c1_arange_closed_form():
    i = np.arange(1024, dtype=np.int64)[:, None]
    j = np.arange(1024, dtype=np.int64)[None, :]
    a = (1024 * i + j).astype(np.int32)
    out = oracle.reduce(a, (1024, 1024), (NONE, SUM), I32)
    assert out.dtype == np.int64
    # sum_j (1024 i + j) = 1024*1024 i + 1023*1024/2
    np.testing.assert_array_equal(out, 1048576 * np.arange(1024, dtype=np.int64) + 523776)


@pytest.mark.parametrize("c", [0, 1, -1, 7, 2147483647])
def test_constant_fill(c):
    a = np.full((3, 1024), c, np.int32)
    out = oracle.reduce(a, (3, 1024), (NONE, SUM), I32)
    np.testing.assert_array_equal(out, np.full(3, 1024 * c, np.int64))


def test_int_min_fill_needs_64_bit_accumulator():
    a = np.full((2, 1024), np.iinfo(np.int32).min, np.int32)
    out = oracle.reduce(a, (2, 1024), (NONE, SUM), I32)
    np.testing.assert_array_equal(out, np.full(2, -(2**41), np.int64))


def test_c1_random_matches_numpy():
    a = workloads.c1_input()
    out = oracle.reduce(a, (1024, 1024), (NONE, SUM), I32, threads=4)
    np.testing.assert_array_equal(out, a.astype(np.int64).sum(axis=1))


# ---------------------------------------------------------------------------
# float SUM: closed forms, exact dyadic sums, exactly rounded sums


def test_constant_one_is_exact():
    a = np.ones((2, 256, 256), np.float32)
    out = oracle.reduce(a, (2, 256, 256), (NONE, SUM, SUM), F32)
    assert out.dtype == np.float64
    np.testing.assert_array_equal(out, [65536.0, 65536.0])


def test_index_fill_exact():
    # A[i,j,k] = 256 j + k: every value is an integer below 2^16 (exact in fp32);
    # sum over j,k = sum_{n<65536} n = 2147450880
    j = np.arange(256, dtype=np.float32)[:, None]
    k = np.arange(256, dtype=np.float32)[None, :]
    a = np.broadcast_to(256 * j + k, (3, 256, 256)).astype(np.float32).copy()
    out = oracle.reduce(a, (3, 256, 256), (NONE, SUM, SUM), F32)
    np.testing.assert_array_equal(out, np.full(3, 2147450880.0))


def test_dyadic_sums_are_exact():
    m = workloads.uniform_i32(11, (16, 4096), -(2**13) + 1, 2**13 - 1)
    a = (m.astype(np.float64) * 2.0**-10).astype(np.float32)
    out = oracle.reduce(a, (16, 64, 64), (NONE, SUM, SUM), F32)
    exact = m.astype(np.int64).sum(axis=1).astype(np.float64) * 2.0**-10
    np.testing.assert_array_equal(out, exact)


@pytest.mark.parametrize("vals", [[2.0**100, 1.0, -(2.0**100)], [1.0, 2.0**100, -(2.0**100)],
                                  [2.0**60, -1.0, 3.0, -(2.0**60), 0.5]])
def test_compensation_recovers_lost_terms(vals):
    # A plain double sum loses the small terms; both branches of the
    # compensation (|s| >= |x| and |s| < |x|) are exercised.
    a = np.array([vals], np.float32)
    out = oracle.reduce(a, a.shape, (NONE, SUM), F32)
    assert out[0] == float(sum(Fraction(v) for v in vals))


def test_normal_rows_match_exactly_rounded_sum():
    a = workloads.normal_f32(5, (8, 65536))
    out = oracle.reduce(a, (8, 256, 256), (NONE, SUM, SUM), F32)
    for r in range(8):
        ref = math.fsum(a[r].astype(np.float64).tolist())
        assert abs(out[r] - ref) <= 2 * 2.0**-53 * abs(ref) + 1e-300


def test_bf16_matches_exactly_rounded_sum():
    bits = workloads.normal_bf16_bits(6, (4, 4096))
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    out = oracle.reduce(bits, (4, 64, 64), (NONE, SUM, SUM), BF16)
    for r in range(4):
        ref = math.fsum(vals[r].tolist())
        assert abs(out[r] - ref) <= 2 * 2.0**-53 * abs(ref) + 1e-300


def test_abs_sum():
    a = workloads.normal_f32(7, (4, 1000))
    got = oracle.abs_sum(a, (4, 1000), (NONE, SUM), F32)
    for r in range(4):
        ref = math.fsum(np.abs(a[r].astype(np.float64)).tolist())
        assert abs(got[r] - ref) <= 2 * 2.0**-53 * ref


# ---------------------------------------------------------------------------
# MIN / MAX / ARG and mixed per-level ops


def test_c3_closed_forms_reduced_shape():
    e = (3, 8, 64, 64)
    ops = (NONE, SUM, MAX, ARGMIN)
    k = np.arange(64)[:, None]
    l = np.arange(64)[None, :]
    cases = {
        "l": (np.broadcast_to(l, e), 0),                  # argmin 0 everywhere
        "63-l": (np.broadcast_to(63 - l, e), 8 * 63),     # argmin 63 -> max 63 -> 8 * 63
        "const": (np.full(e, 5), 0),                      # ties: first occurrence
        "(l-k)%64": (np.broadcast_to((l - k) % 64, e), 8 * 63),  # argmin_l = k -> max_k 63
        "(k+l)%64": (np.broadcast_to((k + l) % 64, e), 8 * 63),  # argmin_l = (64-k)%64 -> max 63
    }
    for name, (a, want) in cases.items():
        a = np.ascontiguousarray(a, dtype=np.int32)
        out = oracle.reduce(a, e, ops, I32)
        assert out.dtype == np.int64, name
        np.testing.assert_array_equal(out, np.full(3, want, np.int64), err_msg=name)


def test_c3_random_and_tie_heavy_match_numpy():
    e = (4, 16, 64, 64)
    ops = (NONE, SUM, MAX, ARGMIN)
    for a in (workloads.uniform_i32(9, e, 0, (1 << 20) - 1), workloads.uniform_i32(10, e, 0, 3)):
        out = oracle.reduce(a, e, ops, I32, threads=3)
        np.testing.assert_array_equal(out, numpy_eval(a, ops))


@pytest.mark.parametrize("ops", [(NONE, MIN), (NONE, MAX), (NONE, ARGMIN), (NONE, ARGMAX),
                                 (NONE, ARGMAX, MIN), (NONE, MIN, SUM), (NONE, MAX, ARGMAX, SUM),
                                 (SUM, ARGMIN, MAX), (NONE, NONE, SUM, MIN)])
def test_mixed_ops_match_numpy(ops):
    e = (5, 7, 9, 11)[: len(ops)] if len(ops) <= 4 else None
    for lo, hi in ((-50, 50), (0, 2), (-(2**31), 2**31 - 1)):
        a = workloads.uniform_i32(12, e, lo, hi)
        out = oracle.reduce(a, e, ops, I32)
        np.testing.assert_array_equal(out.astype(np.int64), numpy_eval(a, ops))


def test_output_types():
    cases = [((NONE, SUM), I32, oracle.OUT_I64), ((NONE, MAX), I32, oracle.OUT_I32),
             ((NONE, ARGMIN), I32, oracle.OUT_I32), ((NONE, MAX, SUM), I32, oracle.OUT_I64),
             ((NONE, MAX, ARGMIN, SUM), I32, oracle.OUT_I32), ((NONE, SUM, SUM), F32, oracle.OUT_F64),
             ((NONE,), I32, oracle.OUT_I32), ((NONE, SUM), BF16, oracle.OUT_F64)]
    for ops, dt, kind in cases:
        assert oracle.out_kind((2,) * len(ops), ops, dt) == kind, (ops, dt)


@pytest.mark.parametrize("ops,dt", [((SUM, NONE), I32), ((NONE, MAX), F32), ((NONE, ARGMIN), BF16)])
def test_rejects_undefined_nests(ops, dt):
    with pytest.raises(ValueError):
        oracle.out_kind((2, 2), ops, dt)


def test_rejects_empty_extent():
    with pytest.raises(ValueError):
        oracle.out_kind((2, 0), (NONE, SUM), I32)


# ---------------------------------------------------------------------------
# brute force: exact rational recursion on tiny nests, every op combination


def _exact(a, ops, idx, m, as_float):
    if m == len(ops):
        v = a[tuple(idx)]
        return Fraction(float(v)) if as_float else int(v)
    vals = [_exact(a, ops, idx + [t], m + 1, as_float) for t in range(a.shape[m])]
    op = ops[m]
    if op == SUM:
        return sum(vals, Fraction(0) if as_float else 0)
    if op == MIN:
        return min(vals)
    if op == MAX:
        return max(vals)
    if op == ARGMIN:
        return vals.index(min(vals))
    return vals.index(max(vals))


def _brute(a, ops, as_float):
    p = next((m for m, o in enumerate(ops) if o != NONE), len(ops))
    outs = []
    for prefix in itertools.product(*[range(n) for n in a.shape[:p]]):
        outs.append(_exact(a, ops, list(prefix), p, as_float))
    return outs


def test_brute_force_all_integer_op_chains():
    red = [SUM, MIN, MAX, ARGMIN, ARGMAX]
    seed = 100
    for depth in (1, 2, 3):
        for p in range(0, depth):
            for chain in itertools.product(red, repeat=depth - p):
                ops = (NONE,) * p + chain
                ext = (2, 3, 4)[:depth]
                seed += 1
                a = workloads.uniform_i32(seed, ext, -3, 3)
                got = oracle.reduce(a, ext, ops, I32)
                want = _brute(a, ops, False)
                assert [int(v) for v in got] == want, (ops, ext)


def test_brute_force_float_sums_exact_within_bound():
    for depth, ext in ((1, (17,)), (2, (3, 17)), (3, (2, 3, 5)), (4, (2, 2, 3, 5))):
        for p in range(depth):
            ops = (NONE,) * p + (SUM,) * (depth - p)
            a = workloads.normal_f32(depth * 10 + p, ext) * np.float32(1e3)
            got = oracle.reduce(np.ascontiguousarray(a, np.float32), ext, ops, F32)
            want = _brute(a, ops, True)
            absb = _brute(np.abs(a), ops, True)
            for g, w, s in zip(got, want, absb):
                # per level the double Neumaier sum is within ~2u|s|; depth levels
                assert abs(Fraction(float(g)) - w) <= Fraction(4 * depth) * Fraction(2.0**-53) * s


# ---------------------------------------------------------------------------
# invariants and special cases


def test_copy_nest():
    a = workloads.uniform_i32(3, (37,), -9, 9)
    np.testing.assert_array_equal(oracle.reduce(a, (37,), (NONE,), I32), a)
    f = workloads.normal_f32(3, (5, 3))
    np.testing.assert_array_equal(oracle.reduce(f, (5, 3), (NONE, NONE), F32), f.reshape(-1).astype(np.float64))


def test_extent_one_levels_are_neutral():
    a = workloads.uniform_i32(4, (6, 40), -100, 100)
    for op in (SUM, MIN, MAX):
        base = oracle.reduce(a, (6, 40), (NONE, op), I32)
        more = oracle.reduce(a, (6, 1, 40), (NONE, op, op), I32)
        np.testing.assert_array_equal(base.astype(np.int64), more.astype(np.int64))


def test_adjacent_sum_levels_merge():
    a = workloads.uniform_i32(5, (6, 8, 5, 12), -(2**31), 2**31 - 1)
    one = oracle.reduce(a, (6, 480), (NONE, SUM), I32)
    three = oracle.reduce(a, (6, 8, 5, 12), (NONE, SUM, SUM, SUM), I32)
    np.testing.assert_array_equal(one, three)


def test_threads_do_not_change_results():
    a = workloads.c2_input((64, 32, 64))
    r1 = oracle.reduce(a, (64, 32, 64), (NONE, SUM, SUM), F32, threads=1)
    r7 = oracle.reduce(a, (64, 32, 64), (NONE, SUM, SUM), F32, threads=7)
    np.testing.assert_array_equal(r1, r7)


def test_output_range():
    a = workloads.c3_input((8, 4, 16, 16))
    ops = (NONE, SUM, MAX, ARGMIN)
    full = oracle.reduce(a, a.shape, ops, I32)
    np.testing.assert_array_equal(oracle.reduce(a, a.shape, ops, I32, o_begin=3, o_end=6), full[3:6])


# ---------------------------------------------------------------------------
# ordered (non-commutative) products: affine maps and 2x2 matrices modulo 2^64

M64 = (1 << 64) - 1
PROD, AFFINE, MAT2 = oracle.PROD, oracle.AFFINE, oracle.MAT2


def _py_affine_run(elems, x0):
    """Run the recurrence x <- a x + b over the elements in order (Python ints)."""
    x = x0
    for a, b in elems:
        x = (int(a) * x + int(b)) & M64
    return x


def _py_mat_prod(mats):
    r = [1, 0, 0, 1]
    for m in mats:
        m = [int(v) for v in m]
        r = [(r[0] * m[0] + r[1] * m[2]) & M64, (r[0] * m[1] + r[1] * m[3]) & M64,
             (r[2] * m[0] + r[3] * m[2]) & M64, (r[2] * m[1] + r[3] * m[3]) & M64]
    return r


def test_affine_closed_forms():
    x = np.zeros((3, 70, 2), np.uint64)
    x[..., 0] = 1
    x[..., 1] = 1
    np.testing.assert_array_equal(oracle.prod(x, (3, 70), (NONE, PROD), AFFINE), [[1, 70]] * 3)
    x[..., 0] = 2
    x[..., 1] = 0
    got = oracle.prod(x[:, :63].copy(), (3, 63), (NONE, PROD), AFFINE)
    np.testing.assert_array_equal(got, [[1 << 63, 0]] * 3)
    np.testing.assert_array_equal(oracle.prod(x, (3, 70), (NONE, PROD), AFFINE), [[0, 0]] * 3)


def test_affine_product_runs_the_recurrence():
    """(A, B) of the ordered product maps x0 to the recurrence's end value."""
    x = workloads.monoid_input(101, (4, 97), AFFINE)
    got = oracle.prod(x, (4, 97), (NONE, PROD), AFFINE)
    for o in range(4):
        for x0 in (0, 1, 12345, M64):
            want = _py_affine_run(x[o], x0)
            assert (int(got[o, 0]) * x0 + int(got[o, 1])) & M64 == want


def test_matrix_closed_forms():
    # Fibonacci: [[1,1],[1,0]]^n = [[F(n+1), F(n)], [F(n), F(n-1)]]
    n = 150
    f = [0, 1]
    for _ in range(n + 1):
        f.append(f[-1] + f[-2])
    x = np.tile(np.array([1, 1, 1, 0], np.uint64), (1, n, 1))
    got = oracle.prod(x, (1, n), (NONE, PROD), MAT2)[0]
    assert [int(v) for v in got] == [f[n + 1] & M64, f[n] & M64, f[n] & M64, f[n - 1] & M64]
    # shear: [[1,1],[0,1]]^n = [[1,n],[0,1]]
    s = np.tile(np.array([1, 1, 0, 1], np.uint64), (2, 1000, 1))
    np.testing.assert_array_equal(oracle.prod(s, (2, 1000), (NONE, PROD), MAT2), [[1, 1000, 0, 1]] * 2)


def test_matrix_product_is_ordered():
    """Brute force with Python integers, and the reversed order differs."""
    x = workloads.monoid_input(102, (5, 33), MAT2)
    got = oracle.prod(x, (5, 33), (NONE, PROD), MAT2)
    for o in range(5):
        assert [int(v) for v in got[o]] == _py_mat_prod(x[o])
        assert [int(v) for v in got[o]] != _py_mat_prod(x[o][::-1])
    y = workloads.monoid_input(103, (5, 33), AFFINE)
    fwd = oracle.prod(y, (5, 33), (NONE, PROD), AFFINE)
    rev = oracle.prod(y[:, ::-1].copy(), (5, 33), (NONE, PROD), AFFINE)
    assert np.any(fwd != rev)


@pytest.mark.parametrize("kind", [AFFINE, MAT2])
def test_nested_products_equal_flat_ones(kind):
    """Associativity: nested PROD levels equal one flat level over the block."""
    x = workloads.monoid_input(104, (3, 4, 6, 7), kind)
    flat = oracle.prod(x.reshape(3, 168, -1).copy(), (3, 168), (NONE, PROD), kind)
    nested = oracle.prod(x, (3, 4, 6, 7), (NONE, PROD, PROD, PROD), kind)
    np.testing.assert_array_equal(flat, nested)
    two = oracle.prod(x, (3, 4, 6, 7), (NONE, NONE, PROD, PROD), kind)
    # out[i] = prod over j of out2[i, j]: the outer level applied to the inner results
    again = oracle.prod(two.reshape(3, 4, -1).copy(), (3, 4), (NONE, PROD), kind)
    np.testing.assert_array_equal(again, flat)


def test_products_reject_mixed_operators_and_types():
    x = workloads.monoid_input(105, (2, 3), AFFINE)
    with pytest.raises(ValueError):
        oracle.prod(x, (2, 3), (NONE, SUM), AFFINE)
    with pytest.raises(ValueError):
        oracle.prod(x, (2, 3), (PROD, NONE), AFFINE)


def test_product_threads_and_ranges():
    x = workloads.monoid_input(106, (50, 20), MAT2)
    r1 = oracle.prod(x, (50, 20), (NONE, PROD), MAT2, threads=1)
    r5 = oracle.prod(x, (50, 20), (NONE, PROD), MAT2, threads=5)
    np.testing.assert_array_equal(r1, r5)
    np.testing.assert_array_equal(oracle.prod(x, (50, 20), (NONE, PROD), MAT2, o_begin=7, o_end=19), r1[7:19])


# ---------------------------------------------------------------------------
# stencils: five-point Jacobi sweeps with fixed boundary cells

def _np_jacobi(x, steps, c0, c1):
    """Independent numpy version (array slices, same association)."""
    a = x.astype(np.float64)
    for _ in range(steps):
        b = a.copy()
        b[1:-1, 1:-1] = c0 * a[1:-1, 1:-1] + c1 * ((a[:-2, 1:-1] + a[2:, 1:-1]) + (a[1:-1, :-2] + a[1:-1, 2:]))
        a = b
    return a


def test_stencil_linear_fields_are_fixed_points():
    i, j = np.mgrid[0:40, 0:56]
    x = (3 * i - 2 * j + 7).astype(np.float32)
    for steps in (1, 4, 9):
        np.testing.assert_array_equal(oracle.stencil(x, steps, 0.5, 0.125), x.astype(np.float64))


def test_stencil_quadratic_field_grows_by_the_laplacian():
    """A = i^2 + j^2 has Laplacian 4: each sweep adds 4 c1 wherever the sweep cone
    of the cell stays inside the interior."""
    i, j = np.mgrid[0:48, 0:48]
    x = (i * i + j * j).astype(np.float32)
    c0, c1, T = 0.5, 0.125, 5
    got = oracle.stencil(x, T, c0, c1)
    inner = (slice(T, 48 - T), slice(T, 48 - T))
    np.testing.assert_array_equal(got[inner], x[inner].astype(np.float64) + 4 * c1 * T)


def test_stencil_impulse_and_boundary():
    x = np.zeros((11, 13), np.float32)
    x[5, 6] = 1.0
    x[0, :] = 3.0  # boundary row: stays
    got = oracle.stencil(x, 1, 0.25, 0.1875)
    assert got[5, 6] == 0.25
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        assert got[5 + di, 6 + dj] == 0.1875
    np.testing.assert_array_equal(got[0, :], 3.0)
    assert got[1, 6] == 0.1875 * 3.0  # the boundary row feeds its interior neighbour
    np.testing.assert_array_equal(oracle.stencil(x, 0, 0.25, 0.1875), x.astype(np.float64))


def test_stencil_matches_an_independent_evaluation():
    x = workloads.normal_f32(120, (37, 61))
    for steps in (1, 3, 8):
        np.testing.assert_array_equal(oracle.stencil(x, steps, 0.6, 0.1), _np_jacobi(x, steps, 0.6, 0.1))
    tiny = workloads.normal_f32(121, (2, 9))  # no interior: unchanged
    np.testing.assert_array_equal(oracle.stencil(tiny, 4, 0.6, 0.1), tiny.astype(np.float64))


def test_verify_helper_flags_planted_mistakes():
    """oracle.verify (the many-nest checker of the GPU tests and the benchmark) passes
    the oracle's own results and catches a wrong integer and a float beyond 1e-6."""
    x = workloads.normal_f32(11, (8, 100))
    xi = workloads.uniform_i32(12, (4, 50), -5, 5)
    r = oracle.reduce(x, (8, 100), (0, 1), oracle.F32)
    ri = oracle.reduce(xi, (4, 50), (0, 1), oracle.I32)
    ok = oracle.verify([(x, (8, 100), (0, 1), oracle.F32, r), (xi, (4, 50), (0, 1), oracle.I32, ri)])
    assert ok["ok"] and ok["nests"] == 2 and ok["float_outputs"] == 8 and ok["max_rel_err"] == 0.0
    bad_i = ri.copy()
    bad_i[3] += 1
    v = oracle.verify([(xi, (4, 50), (0, 1), oracle.I32, bad_i)])
    assert not v["ok"] and v["int_nests_mismatched"] == 1 and v["failures"] == [0]
    bad_f = r.copy()
    bad_f[5] += 3e-6 * max(abs(bad_f[5]), 1.0)
    v = oracle.verify([(xi, (4, 50), (0, 1), oracle.I32, ri), (x, (8, 100), (0, 1), oracle.F32, bad_f)])
    assert not v["ok"] and not v["float_within"] and v["failures"] == [1]
    assert v["worst_condition_number"] >= 1.0
