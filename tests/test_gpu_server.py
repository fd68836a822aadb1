"""GPU tests of the serving loop: requests that arrive while others run are
batched on the fly; every result matches the oracle and is the same bits as the
request served alone."""
import numpy as np
import pytest

import workloads
from gpu_util import assert_match, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_01906_amd as hp
    hp.lib()
    yield


def stream_and_pools(n, pool_elems, seed):
    st = workloads.c5_stream(duration_s=1.0, rate=20000.0, median_bytes=16 << 10, max_bytes=4 << 20,
                             pool_elems=pool_elems, seed=seed, max_requests=n)
    pi = st.pool_i32()
    pf = st.pool_f32()
    return st, pi, pf


def test_served_mix_equals_alone_and_oracle():
    import paper_2309_01906_amd as hp
    st, pi, pf = stream_and_pools(300, 1 << 22, 501)
    di, df = torch.from_numpy(pi).cuda(), torch.from_numpy(pf).cuda()
    reqs = st.requests
    say("case served mix", len(reqs), "requests")
    outs_mix, outs_alone = [], []
    for r in reqs:
        inf = hp.inspect(r.nest.extents, r.nest.ops, r.nest.dtype)
        dt = hp.torch_out_dtype(inf["out_dtype"])
        outs_mix.append(torch.full((inf["n_out"],), -7, dtype=dt, device="cuda"))
        outs_alone.append(torch.full((inf["n_out"],), -7, dtype=dt, device="cuda"))

    def ptr(r):
        base = di if r.pool == 0 else df
        return base.data_ptr() + r.offset * 4

    # mixed: open-loop arrivals at 20k/s on 3 slots
    with hp.Server(hbm_budget=1 << 30, slot_bytes=64 << 20, streams=3, max_batch=64, window_us=20) as s:
        t0 = s.now_us() + 2000.0
        arrivals = [t0 + (r.t_arrival_us - reqs[0].t_arrival_us) for r in reqs]
        tk = s.replay([(r.nest.extents, r.nest.ops, r.nest.dtype) for r in reqs], [ptr(r) for r in reqs],
                      [o.data_ptr() for o in outs_mix], arrivals)
        infos = [s.wait(t) for t in tk]
        stats = s.stats()
    assert all(i["status"] == 0 for i in infos)
    assert stats["batches"] < len(reqs)  # requests were actually batched together
    say("served stats", {k: round(v, 1) for k, v in stats.items()})
    # alone: one request at a time on an idle server
    with hp.Server(streams=1, max_batch=1, window_us=0) as s:
        for r, o in zip(reqs, outs_alone):
            s.wait(s.submit(r.nest.extents, r.nest.ops, r.nest.dtype, ptr(r), o.data_ptr()))
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        a, b = outs_mix[i].cpu().numpy(), outs_alone[i].cpu().numpy()
        np.testing.assert_array_equal(a, b, err_msg=f"request {i} {r.nest}")
        pool = pi if r.pool == 0 else pf
        x = np.ascontiguousarray(pool[r.offset:r.offset + r.nest.elems].reshape(r.nest.extents))
        assert_match(a, x, r.nest.extents, r.nest.ops, what=f"request {i} {r.nest}")
