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


def test_invalid_config_and_nest():
    with pytest.raises(hp.HPError):
        hp.Server(streams=0, flags=hp.SERVER_FAKE_DEVICE)
    with fake() as s:
        with pytest.raises(hp.HPError) as e:
            s.submit((4, 0), ("NONE", "SUM"), hp.F32, 0, 0)
        assert e.value.status_name == "HP_EINVAL"
