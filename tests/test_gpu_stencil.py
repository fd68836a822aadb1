"""Stencil sweeps tiled through LDS against the fp64 oracle: partial tiles, arrays
without an interior, every step count one launch holds, more sweeps than that
(several launches), every plan variant (tile rows, sweeps per launch, XCD bands) bit
for bit against the others, and the benchmarked 8192 x 8192 array in full."""
import numpy as np
import pytest

import oracle
import paper_2309_01906_amd as hp
import workloads
from gpu_util import say

pytestmark = pytest.mark.gpu


def run(x, steps, c0, c1, **plan):
    import torch
    d = torch.from_numpy(x).cuda()
    with hp.Stencil(x.shape[0], x.shape[1], steps, c0, c1, **plan) as s:
        out = s.run(d)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def check_against_oracle(x, got, steps, c0, c1):
    ref = oracle.stencil(x, steps, c0, c1)
    tol = 8 * steps * 2.0**-24 * float(np.abs(x).max(initial=0.0))
    err = np.abs(got.astype(np.float64) - ref)
    assert float(err.max(initial=0.0)) <= tol, (x.shape, steps, float(err.max()), tol)
    # boundary cells are copied bit for bit
    np.testing.assert_array_equal(got[0, :], x[0, :])
    np.testing.assert_array_equal(got[-1, :], x[-1, :])
    np.testing.assert_array_equal(got[:, 0], x[:, 0])
    np.testing.assert_array_equal(got[:, -1], x[:, -1])


@pytest.mark.parametrize("shape", [(100, 150), (32, 64), (33, 65), (2, 9), (1, 1), (517, 1031), (3, 3)])
@pytest.mark.parametrize("steps", [1, 2, 5, 8])
def test_stencil_matches_the_oracle(shape, steps):
    say("case stencil", shape, steps)
    c0, c1 = 0.6, 0.1  # convex weights: the fp32 error stays below 6 T u max|A|
    x = workloads.normal_f32(130, shape)
    check_against_oracle(x, run(x, steps, c0, c1), steps, c0, c1)


@pytest.mark.parametrize("shape", [(100, 150), (33, 65), (517, 1031), (2, 9)])
@pytest.mark.parametrize("steps", [9, 12, 17])
def test_more_sweeps_than_one_launch(shape, steps):
    say("case stencil multi-launch", shape, steps)
    x = workloads.normal_f32(131, shape)
    with hp.Stencil(shape[0], shape[1], steps, 0.6, 0.1) as s:
        assert s.info["launches"] == -(-steps // 8)
    check_against_oracle(x, run(x, steps, 0.6, 0.1), steps, 0.6, 0.1)


def test_plan_variants_agree_bit_for_bit():
    """Every cell is the same fp32 function of its neighbours' previous values under
    any tiling, so tile rows, sweeps per launch and the XCD dealing of tiles change
    no bit of the result."""
    x = workloads.normal_f32(132, (517, 1031))
    steps = 12
    base = run(x, steps, 0.6, 0.1)
    check_against_oracle(x, base, steps, 0.6, 0.1)
    for th in (32, 64):
        for t in (1, 3, 8):
            for fl in (0, hp.STENCIL_NO_XCD):
                say("case stencil variant", th, t, fl)
                got = run(x, steps, 0.6, 0.1, tile_rows=th, sweeps_per_launch=t, flags=fl)
                np.testing.assert_array_equal(got, base, err_msg=f"tile_rows {th} sweeps {t} flags {fl}")


@pytest.mark.parametrize("steps", [1, 8, 12])
def test_full_size_8192(steps):
    """The benchmarked array (8192 x 8192 fp32, 256 MiB), every cell against the oracle."""
    say("case stencil full 8192x8192", steps)
    x = workloads.normal_f32(230901906 + 7, (8192, 8192))
    got = run(x, steps, 0.6, 0.1)
    check_against_oracle(x, got, steps, 0.6, 0.1)


def test_stencil_harmonic_field_is_exact():
    i, j = np.mgrid[0:300, 0:400]
    x = (2 * i - 3 * j + 5).astype(np.float32)
    np.testing.assert_array_equal(run(x, 8, 0.5, 0.125), x)
