"""Serving scheduler on the host: the server's simulated executor runs the
real admission, batching, completion and memory bookkeeping without any
device work, so these run on the CPU."""
import threading
import time

import pytest

from paper_2109_13504_amd import mgp

FAKE_W = 0x10000  # never dereferenced by the simulated executor


@pytest.fixture(scope="module", autouse=True)
def built():
    from paper_2109_13504_amd.csrc import build as b
    if b.needs_build():
        b.build()
    mgp.lib()


def footprint(n, d=0, b_max=1024, mego=True):
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    out = r(4 * n) + (r(4 * n * d) if d else 0)
    ws = r(4 * (2 * n + 2048)) + r(4 * b_max) if mego else 0
    return out + ws


def make(**kw):
    cfg = dict(variant="megopolis", d=0, hbm_budget=64 << 20, streams=2, max_batch=8, b_max=1024, simulate=True,
               sim_us_fixed=2000.0, sim_ns_per_particle=0.0)
    cfg.update(kw)
    return mgp.Server(**cfg)


def drain(srv, tickets):
    results = {}
    for t in tickets:
        results[t] = srv.wait(t, 20000.0)
        srv.release(t)
    return results


def test_all_requests_complete_and_memory_returns():
    srv = make()
    ts = [srv.submit(FAKE_W, n=10000 + 1000 * i, B=5, seed=i, stream_id=i) for i in range(30)]
    res = drain(srv, ts)
    assert all(r["state"] == mgp.MGP_REQ_DONE for r in res.values())
    st = srv.stats()
    assert st["completed"] == 30 and st["released"] == 30 and st["pool_in_use"] == 0 and st["in_flight"] == 0
    srv.close()


def test_admission_respects_budget_and_order():
    n = 200_000
    fp = footprint(n)
    budget = 4 * fp + fp // 2  # room for 4 requests at once
    srv = make(hbm_budget=budget, streams=4, max_batch=2, sim_us_fixed=3000.0)
    ts = [srv.submit(FAKE_W, n=n, B=5, seed=i) for i in range(16)]
    res = drain(srv, ts)
    st = srv.stats()
    assert st["pool_peak"] <= budget
    assert st["pool_peak"] >= 3 * fp  # the pool was actually used concurrently
    admits = [res[t]["t_admit"] for t in ts]
    assert admits == sorted(admits)  # first come, first admitted
    for r in res.values():
        assert r["t_submit"] <= r["t_admit"] <= r["t_dispatch"] <= r["t_done"]
        assert r["t_done"] - r["t_dispatch"] >= 2.5e-3  # the simulated batch time
    srv.close()


def test_requests_arriving_during_work_overlap_on_streams():
    srv = make(streams=3, max_batch=1, sim_us_fixed=20000.0)
    t1 = srv.submit(FAKE_W, n=1000, B=3)
    time.sleep(0.005)
    t2 = srv.submit(FAKE_W, n=1000, B=3)  # arrives while t1 runs
    r2 = srv.wait(t2, 20000.0)
    r1 = srv.poll(t1)
    assert r2["t_dispatch"] < r1["t_done"] or r1["state"] != mgp.MGP_REQ_DONE
    drain(srv, [t1, t2])
    assert srv.stats()["max_concurrent_batches"] >= 2
    srv.close()


def test_micro_batches_group_queued_requests():
    srv = make(streams=1, max_batch=8, sim_us_fixed=10000.0)
    first = srv.submit(FAKE_W, n=1000, B=3)
    time.sleep(0.002)
    rest = [srv.submit(FAKE_W, n=1000, B=3, seed=i) for i in range(16)]
    drain(srv, [first] + rest)
    st = srv.stats()
    # one batch for the first, then 16 queued ones in batches of at most 8
    assert st["micro_batches"] <= 4
    srv.close()


def test_cancel_queued_and_refuse_running():
    n = 100_000
    srv = make(hbm_budget=footprint(n) + 1024, streams=1, max_batch=1, sim_us_fixed=30000.0)
    t1 = srv.submit(FAKE_W, n=n, B=3)
    t2 = srv.submit(FAKE_W, n=n, B=3)  # cannot be admitted while t1 holds the pool
    time.sleep(0.005)
    srv.cancel(t2)
    assert srv.poll(t2)["state"] == mgp.MGP_REQ_CANCELLED
    with pytest.raises(mgp.MgpError) as e:
        srv.cancel(t1)
    assert e.value.code == mgp.MGP_EBUSY
    drain(srv, [t1, t2])
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1 and st["pool_in_use"] == 0
    srv.close()


def test_failures_are_isolated_and_memory_freed():
    srv = make(streams=2, max_batch=2, sim_us_fixed=500.0, sim_fail_every=3)
    ts = [srv.submit(FAKE_W, n=5000, B=3, seed=i) for i in range(24)]
    res = drain(srv, ts)
    states = [r["state"] for r in res.values()]
    assert states.count(mgp.MGP_REQ_FAILED) > 0 and states.count(mgp.MGP_REQ_DONE) > 0
    for r in res.values():
        if r["state"] == mgp.MGP_REQ_FAILED:
            assert r["ancestors_dev"] is None
    assert srv.stats()["pool_in_use"] == 0
    srv.close()


def test_outputs_held_until_release_block_admission():
    n = 100_000
    # after t1 completes only its ancestors (4n bytes) stay allocated, which
    # leaves less than one footprint free
    srv = make(hbm_budget=footprint(n) + 2 * n, streams=2, max_batch=1, sim_us_fixed=200.0)
    t1 = srv.submit(FAKE_W, n=n, B=3)
    srv.wait(t1, 5000.0)
    t2 = srv.submit(FAKE_W, n=n, B=3)
    time.sleep(0.02)
    # t1's outputs still occupy the pool: t2 waits
    assert srv.poll(t2)["state"] == mgp.MGP_REQ_QUEUED
    srv.release(t1)
    assert srv.wait(t2, 5000.0)["state"] == mgp.MGP_REQ_DONE
    srv.release(t2)
    srv.close()


def test_argument_errors():
    srv = make(hbm_budget=1 << 20)
    with pytest.raises(mgp.MgpError) as e:
        srv.submit(FAKE_W, n=1 << 20, B=3)  # can never fit a 1 MiB pool
    assert e.value.code == mgp.MGP_ENOMEM
    with pytest.raises(mgp.MgpError) as e:
        srv.submit(0, n=10, B=3)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        srv.submit(FAKE_W, n=10, B=0, epsilon=0.0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError):
        srv.poll(12345)
    srv.close()


def test_destroy_with_queued_requests_cancels_them():
    n = 100_000
    srv = make(hbm_budget=footprint(n) + 4096, streams=1, max_batch=1, sim_us_fixed=5000.0)
    for i in range(6):
        srv.submit(FAKE_W, n=n, B=3, seed=i)
    t0 = time.time()
    srv.close()  # must not wait for outputs nobody releases
    assert time.time() - t0 < 5.0


def test_submit_from_many_threads():
    srv = make(streams=4, max_batch=16, sim_us_fixed=300.0)
    tickets, lock = [], threading.Lock()

    def client(k):
        for i in range(25):
            t = srv.submit(FAKE_W, n=1000 + i, B=2, seed=k * 100 + i, stream_id=k)
            with lock:
                tickets.append(t)

    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(set(tickets)) == 150
    res = drain(srv, tickets)
    assert all(r["state"] == mgp.MGP_REQ_DONE for r in res.values())
    srv.close()
