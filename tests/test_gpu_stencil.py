"""Stencil sweeps tiled through LDS against the fp64 oracle: partial tiles, arrays
without an interior, every supported step count."""
import numpy as np
import pytest

import oracle
import paper_2309_01906_amd as hp
import workloads
from gpu_util import say

pytestmark = pytest.mark.gpu


def run(x, steps, c0, c1):
    import torch
    d = torch.from_numpy(x).cuda()
    with hp.Stencil(x.shape[0], x.shape[1], steps, c0, c1) as s:
        out = s.run(d)
        torch.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("shape", [(100, 150), (32, 64), (33, 65), (2, 9), (1, 1), (517, 1031), (3, 3)])
@pytest.mark.parametrize("steps", [1, 2, 5, 8])
def test_stencil_matches_the_oracle(shape, steps):
    say("case stencil", shape, steps)
    c0, c1 = 0.6, 0.1  # convex weights: the fp32 error stays below 6 T u max|A|
    x = workloads.normal_f32(130, shape)
    got = run(x, steps, c0, c1)
    ref = oracle.stencil(x, steps, c0, c1)
    tol = 8 * steps * 2.0**-24 * float(np.abs(x).max(initial=0.0))
    err = np.abs(got.astype(np.float64) - ref)
    assert float(err.max(initial=0.0)) <= tol, (shape, steps, float(err.max()), tol)
    # boundary cells are copied bit for bit
    np.testing.assert_array_equal(got[0, :], x[0, :])
    np.testing.assert_array_equal(got[:, -1], x[:, -1])


def test_stencil_harmonic_field_is_exact():
    i, j = np.mgrid[0:300, 0:400]
    x = (2 * i - 3 * j + 5).astype(np.float32)
    np.testing.assert_array_equal(run(x, 8, 0.5, 0.125), x)
