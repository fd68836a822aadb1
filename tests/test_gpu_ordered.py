"""Ordered (non-commutative) products on the GPU against the oracle, bit for bit:
affine maps and 2x2 matrices modulo 2^64, nested levels, ragged tiles, blocks
split over many waves and folded in order."""
import numpy as np
import pytest

import oracle
import paper_2309_01906_amd as hp
import workloads
from gpu_util import say

pytestmark = pytest.mark.gpu

KINDS = {"affine": (hp.AFFINE64, workloads.AFFINE), "mat2": (hp.MAT2X2_64, workloads.MAT2)}


def run_gpu(x, ext, ops, dtype):
    import torch
    d = torch.from_numpy(x.view(np.int64)).cuda()
    with hp.Plan(ext, ops, dtype) as p:
        out = p.run(d)
        torch.cuda.synchronize()
        return out.cpu().numpy().view(np.uint64), p.info


@pytest.mark.parametrize("kind", ["affine", "mat2"])
@pytest.mark.parametrize("ext,nprod", [
    ((64, 5000), 1), ((5, 3, 77, 13), 3), ((1000, 1), 1), ((1, 1 << 20), 1), ((1, 100003), 1),
    ((3, 2, 4097), 1), ((2, 3, 4), 0), ((7, 1, 1, 9), 2), ((3, 300007), 1),
])
def test_ordered_products_match_the_oracle(kind, ext, nprod):
    dt, ok = KINDS[kind]
    ops = ("NONE",) * (len(ext) - nprod) + ("PROD",) * nprod
    say("case ordered", kind, ext, ops)
    x = workloads.monoid_input(110, ext, ok)
    got, info = run_gpu(x, ext, [hp.OP_NAMES[o] for o in ops], dt)
    ref = oracle.prod(x, ext, [oracle.NONE if o == "NONE" else oracle.PROD for o in ops], ok, threads=8)
    assert got.shape == ref.shape
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, f"{kind} {ext}: {bad.size} outputs differ, first {bad[:5]}"


@pytest.mark.parametrize("kind", ["affine", "mat2"])
def test_ordered_product_order_matters_and_repeats(kind):
    dt, ok = KINDS[kind]
    ext = (4, 70001)
    x = workloads.monoid_input(111, ext, ok)
    a, info = run_gpu(x, ext, (hp.NONE, hp.PROD), dt)
    b, _ = run_gpu(x, ext, (hp.NONE, hp.PROD), dt)
    np.testing.assert_array_equal(a, b)
    r, _ = run_gpu(x[:, ::-1].copy(), ext, (hp.NONE, hp.PROD), dt)
    assert np.any(a != r)  # the reversed sequence has a different product
