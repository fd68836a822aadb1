"""Scheduler logic of the serving loop, on the host: a fake executor stands in for
the device (no GPU work; batches complete after a simulated delay).  Admission by
HBM budget, batching, failure handling and draining are checked here."""
import time

import pytest

import paper_2309_01906_amd as hp

NEST = ((4, 1024), ("NONE", "SUM"), hp.F32)  # 16 KiB in + 32 B out


def fake(**kw):
    kw.setdefault("flags", hp.SERVER_FAKE_DEVICE)
    return hp.Server(**kw)


def test_all_requests_complete_and_stats():
    with fake(streams=2, max_batch=8, window_us=50) as s:
        tickets = [s.submit(*NEST, 0, 0) for _ in range(100)]
        infos = [s.wait(t) for t in tickets]
        st = s.stats()
    assert all(i["status"] == 0 for i in infos)
    assert st["completed"] == 100 and st["failed"] == 0
    assert 1 <= st["batches"] <= 100
    assert st["p50_us"] <= st["p99_us"] <= st["max_us"]
    for i in infos:
        assert i["t_arrival_us"] <= i["t_admit_us"] <= i["t_launch_us"] <= i["t_done_us"]


def test_budget_limits_bytes_in_flight():
    req = 16384 + 32
    budget = 5 * req
    with fake(hbm_budget=budget, streams=4, max_batch=64) as s:
        tickets = [s.submit(*NEST, 0, 0) for _ in range(60)]
        for t in tickets:
            s.wait(t)
        st = s.stats()
    assert st["max_in_use_bytes"] <= budget
    assert st["in_use_bytes"] == 0
    assert st["completed"] == 60


def test_too_big_and_queue_full():
    with fake(hbm_budget=1000) as s:
        with pytest.raises(hp.HPError) as e:
            s.submit(*NEST, 0, 0)
        assert e.value.status_name == "HP_ETOOBIG"
    with fake(queue_cap=1, streams=1, window_us=1000000) as s:
        statuses = []
        for _ in range(200):
            try:
                s.submit(*NEST, 0, 0)
                statuses.append("ok")
            except hp.HPError as e:
                statuses.append(e.status_name)
        assert "HP_EAGAIN" in statuses


def test_failed_batches_release_budget_and_later_requests_proceed():
    with fake(streams=1, max_batch=1, fail_every_nth_batch=3) as s:
        tickets = [s.submit(*NEST, 0, 0) for _ in range(12)]
        infos = [s.wait(t) for t in tickets]
        st = s.stats()
    failed = [i for i in infos if i["status"] != 0]
    assert len(failed) == 4 and st["failed"] == 4 and st["completed"] == 8
    assert all(hp.STATUS[i["status"]] == "HP_EDEVICE" for i in failed)
    assert st["in_use_bytes"] == 0


def test_large_request_not_starved():
    big = ((1, 1 << 20), ("NONE", "SUM"), hp.F32)  # 4 MiB
    small = NEST
    budget = (4 << 20) + 64 + 8 * (16384 + 32)
    with fake(hbm_budget=budget, streams=4, max_batch=4, window_us=0) as s:
        ts = [s.submit(*small, 0, 0) for _ in range(20)]
        tb = s.submit(*big, 0, 0)
        ts += [s.submit(*small, 0, 0) for _ in range(200)]
        ib = s.wait(tb)
        for t in ts:
            s.wait(t)
    assert ib["status"] == 0


def test_destroy_drains_pending_work():
    s = fake(streams=1, max_batch=2, window_us=10)
    tickets = [s.submit(*NEST, 0, 0) for _ in range(30)]
    s.close()  # drains: every request completes before the scheduler stops


def test_replay_open_loop_timestamps():
    with fake(streams=2) as s:
        t0 = s.now_us() + 1000.0
        arrivals = [t0 + 50.0 * i for i in range(40)]
        tk = s.replay([NEST] * 40, [0] * 40, [0] * 40, arrivals)
        infos = [s.wait(t) for t in tk]
    assert [i["t_arrival_us"] for i in infos] == arrivals
    assert all(i["t_admit_us"] >= i["t_arrival_us"] for i in infos)


def test_replay_from_now_fixes_the_start_after_marshalling():
    """replay_from_now reads the start time only once the stream's arguments are
    marshalled, so a long stream's first requests are not submitted after their
    arrival times; arrivals are the start plus the offsets."""
    with fake(streams=2) as s:
        offsets = [25.0 * i for i in range(2000)]
        before = s.now_us()
        tk, t0 = s.replay_from_now([NEST] * 2000, [0] * 2000, [0] * 2000, offsets, lead_us=2000.0)
        infos = [s.wait(t) for t in tk]
    assert t0 >= before + 2000.0
    assert [i["t_arrival_us"] for i in infos] == [t0 + o for o in offsets]
    assert all(i["t_admit_us"] >= i["t_arrival_us"] for i in infos)


def test_invalid_config_and_nest():
    with pytest.raises(hp.HPError):
        hp.Server(streams=0, flags=hp.SERVER_FAKE_DEVICE)
    with fake() as s:
        with pytest.raises(hp.HPError) as e:
            s.submit((4, 0), ("NONE", "SUM"), hp.F32, 0, 0)
        assert e.value.status_name == "HP_EINVAL"


def _smallest_slot_for_one(nest=NEST):
    """The smallest slot arena (in 256-byte steps) in which one request of `nest` fits."""
    for slot in range(4096, 64 << 10, 256):
        with fake(slot_bytes=slot) as s:
            try:
                s.wait(s.submit(*nest, 0, 0))
                return slot
            except hp.HPError as e:
                assert e.status_name == "HP_ETOOBIG"
    raise AssertionError("no slot size fits one request")


def test_slot_arena_holds_one_request_not_two():
    """Packing charges each request's descriptors and workspace against the slot
    arena: with room for one request only, every request still completes, one per
    batch, instead of whole batches failing for how they were packed."""
    nest = ((1, 1 << 22), ("NONE", "SUM"), hp.F32)  # grid-split: plan, tasks, fold task and workspace
    slot = _smallest_slot_for_one(nest)
    assert slot > 4096 + 256
    with fake(slot_bytes=slot, streams=2, max_batch=16, window_us=1000) as s:
        tickets = [s.submit(*nest, 0, 0) for _ in range(40)]
        infos = [s.wait(t) for t in tickets]
        st = s.stats()
    assert all(i["status"] == 0 for i in infos)
    assert st["completed"] == 40 and st["failed"] == 0
    assert len({i["batch_id"] for i in infos}) == 40  # one request per batch
    # a request whose descriptors alone exceed the arena is refused at submission
    with fake(slot_bytes=slot - 256) as s:
        with pytest.raises(hp.HPError) as e:
            s.submit(*nest, 0, 0)
        assert e.value.status_name == "HP_ETOOBIG"
    # twice the room: batches of two or more form
    with fake(slot_bytes=2 * slot, streams=1, max_batch=16, window_us=100000) as s:
        s.wait(s.submit(*nest, 0, 0))
        tickets = [s.submit(*nest, 0, 0) for _ in range(30)]
        infos = [s.wait(t) for t in tickets]
    assert all(i["status"] == 0 for i in infos)
    assert len({i["batch_id"] for i in infos}) < 30


def test_mixed_sizes_share_slots_without_failures():
    """Requests of different kernel families and sizes packed under a small arena."""
    nests = [NEST, ((2, 3, 1000), ("NONE", "MAX", "ARGMIN"), hp.I32), ((1, 1 << 22), ("NONE", "SUM"), hp.F32),
             ((64, 5), ("NONE", "SUM"), hp.I32)]
    slot = max(_smallest_slot_for_one(n) for n in nests)
    with fake(slot_bytes=slot + 2048, streams=3, max_batch=64, window_us=200) as s:
        tickets = [s.submit(*nests[i % len(nests)], 0, 0) for i in range(200)]
        infos = [s.wait(t) for t in tickets]
        st = s.stats()
    assert all(i["status"] == 0 for i in infos) and st["failed"] == 0


def test_failure_after_enqueue_keeps_slot_until_drained():
    """A batch that fails after its descriptor upload was enqueued keeps its slot
    busy until the stream has drained (the fake executor takes at least 5 us), and
    only then fails its requests; the next batch on that slot starts after that."""
    with fake(streams=1, max_batch=1, fail_every_nth_batch=2, fail_step=1, window_us=0) as s:
        tickets = [s.submit(*NEST, 0, 0) for _ in range(10)]
        infos = [s.wait(t) for t in tickets]
        st = s.stats()
    failed = [k for k, i in enumerate(infos) if i["status"] != 0]
    assert len(failed) == 5 and st["failed"] == 5 and st["completed"] == 5
    assert all(hp.STATUS[infos[k]["status"]] == "HP_EDEVICE" for k in failed)
    for k in failed:
        i = infos[k]
        assert i["t_done_us"] - i["t_launch_us"] >= 5.0, i  # held until drained
        nxt = [j for j in infos if j["batch_id"] == i["batch_id"] + 1]
        for j in nxt:
            assert j["t_launch_us"] >= i["t_done_us"], (i, j)
    assert st["in_use_bytes"] == 0


def test_failure_before_enqueue_releases_at_once():
    with fake(streams=1, max_batch=1, fail_every_nth_batch=2, fail_step=0, window_us=0) as s:
        tickets = [s.submit(*NEST, 0, 0) for _ in range(6)]
        infos = [s.wait(t) for t in tickets]
    failed = [i for i in infos if i["status"] != 0]
    assert len(failed) == 3
    assert all(hp.STATUS[i["status"]] == "HP_EDEVICE" for i in failed)
