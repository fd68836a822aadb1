"""hp_reduce_static, the entry point that allocates nothing (its plan and partials
live in the library's static scratch), against hp_run of a plan of the same nest:
the same kernels run, so outputs must be the same bits, and they must match the
oracle.  Two calls in a row share the scratch; the second is smaller, so stale
partials of the first must not leak into it."""
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


def _inputs(kind, ext, seed):
    if kind == "i32":
        return workloads.uniform_i32(seed, ext, 0, 1 << 20)
    return workloads.normal_f32(seed, ext)


CASES = [
    # grid-split integer nest with a different operator per level, then a smaller one
    ("i32", (8, 128, 64, 64), ("NONE", "SUM", "MAX", "ARGMIN"), (3, 64, 32, 64)),
    # grid-split float sum (fp32 pairs folded in fp64), then a smaller one
    ("f32", (4, 1 << 20), ("NONE", "SUM"), (2, 3 << 16)),
    # no grid split, ragged flat blocks
    ("f32", (300, 4099), ("NONE", "SUM"), (17, 1001)),
    ("i32", (64, 5000), ("NONE", "MIN"), (5, 77)),
    # one-output integer nest whose partials fold on a whole wave, then a smaller one
    ("i32", (1, 1 << 22), ("NONE", "MAX"), (3, 1 << 20)),
    # float sum of sums planned as one level, then a smaller one
    ("f32", (64, 16, 1024), ("NONE", "SUM", "SUM"), (5, 16, 1024)),
]


@pytest.mark.parametrize("kind,ext1,ops,ext2", CASES)
def test_static_entry_matches_hp_run_twice(kind, ext1, ops, ext2):
    import paper_2309_01906_amd as hp
    dt = hp.I32 if kind == "i32" else hp.F32
    opc = [hp.OP_NAMES[o] for o in ops]
    for call, ext in enumerate((ext1, ext2)):
        say("case static", kind, ext, ops, "call", call)
        x = _inputs(kind, ext, 500 + call)
        d = to_device(x)
        with hp.Plan(ext, opc, dt) as p:
            want = p.run(d)
            got = p.empty_out(d.device).fill_(-3)
            hp.reduce_static(d, got, ext, opc)
            torch.cuda.synchronize()
            info = p.info
        if call == 0 and ext[0] > 4:
            say("  gsplit", info["gsplit"], "workspace", info["workspace_bytes"])
        np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
        assert_match(got.cpu().numpy(), x, ext, ops, what=f"static {ext}")


def test_static_entry_grid_split_cases_exercise_the_scratch():
    import paper_2309_01906_amd as hp
    inf = hp.inspect((8, 128, 64, 64), (0, 1, 3, 4), hp.I32)
    assert inf["gsplit"] > 1 and inf["workspace_bytes"] > 0
    inf = hp.inspect((4, 1 << 20), (0, 1), hp.F32)
    assert inf["gsplit"] > 1 and inf["workspace_bytes"] > 0
