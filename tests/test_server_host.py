"""Host-only tests of the serving layer (no GPU): the server's test mode runs
no device work, a request occupying its slot for a time proportional to n,
so admission by HBM footprint, slot limits, first-fit order with its
overtaking limit, cancellation and shutdown can be checked on the CPU."""
import time

import numpy as np
import pytest

import paper_2106_04727_amd as pc
from paper_2106_04727_amd import PCError

US_PER_KPT = 20000.0  # 20 ms per 1000 points


def fp(n):
    return pc.workspace_bytes(n, 2, "ward")


def pts(n, seed=0):
    return np.random.default_rng(seed).random((n, 2), dtype=np.float32)


def test_budget_and_slots_respected():
    sizes = [300, 900, 2000, 500, 1500, 700, 2500, 400, 1200, 800]
    budget = fp(2500) + fp(2000) + fp(300)
    with pc.Server(slots=3, hbm_budget_bytes=budget, fake_us_per_kpoint=US_PER_KPT) as srv:
        ts = [srv.submit(pts(n, i), "ward") for i, n in enumerate(sizes)]
        for t, n in zip(ts, sizes):
            Z, info = srv.result(t)
            assert Z.shape == (n - 1, 4) and info["state"] == "done" and info["footprint_bytes"] == fp(n)
        st = srv.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0 and st["queued"] == 0
    assert st["peak_bytes_in_use"] <= budget
    assert 2 <= st["peak_running"] <= 3
    # idle slots count only what their contexts keep, within their share
    assert st["bytes_in_use"] <= budget


def test_requests_overlap():
    # 8 equal requests on 4 slots take about two request times, not eight
    with pc.Server(slots=4, hbm_budget_bytes=1 << 40, fake_us_per_kpoint=US_PER_KPT) as srv:
        t0 = time.perf_counter()
        ts = [srv.submit(pts(2000, i), "average") for i in range(8)]
        infos = [srv.result(t)[1] for t in ts]
        wall = time.perf_counter() - t0
    assert wall < 0.04 * 8 * 0.75
    assert max(i["t_start_ms"] for i in infos[:4]) < min(i["t_done_ms"] for i in infos[:4])


def test_oversized_request_refused():
    with pc.Server(slots=2, hbm_budget_bytes=fp(1000), fake_us_per_kpoint=US_PER_KPT) as srv:
        with pytest.raises(PCError) as e:
            srv.submit(pts(5000), "ward")
        assert e.value.status == -3
        t = srv.submit(pts(1000), "ward")
        srv.result(t)
        assert srv.stats()["rejected"] == 1


def test_invalid_requests():
    with pc.Server(slots=1, hbm_budget_bytes=1 << 40, fake_us_per_kpoint=US_PER_KPT) as srv:
        with pytest.raises(PCError) as e:
            srv.submit(pts(100), 7)
        assert e.value.status == -1
        with pytest.raises(PCError):
            srv.submit(np.zeros((0, 2), np.float32), "ward")
        with pytest.raises(PCError):
            srv.poll(12345)


def test_first_fit_then_no_overtaking():
    """A waiting request that does not fit is overtaken by later ones that
    do, but only 16 times; after that they wait behind it."""
    big, small = 4000, 500
    budget = fp(big) + fp(small) + fp(small) // 2   # one big + one small fit together, not two bigs
    assert budget < 2 * fp(big)
    with pc.Server(slots=2, hbm_budget_bytes=budget, fake_us_per_kpoint=US_PER_KPT) as srv:
        ta = srv.submit(pts(big, 1), "ward")          # runs ~80 ms
        time.sleep(0.01)
        tb = srv.submit(pts(big, 2), "ward")          # waits for a
        smalls = [srv.submit(pts(small, 10 + i), "ward") for i in range(20)]  # ~10 ms each
        ib = srv.result(tb)[1]
        ia = srv.result(ta)[1]
        isx = [srv.result(t)[1] for t in smalls]
    starts = [i["t_start_ms"] for i in isx]
    assert ib["t_start_ms"] >= ia["t_done_ms"] - 1e-6
    # the first small requests overtook b ...
    assert sum(s < ib["t_start_ms"] for s in starts) >= 2
    # ... at most 16 of them
    assert sum(s < ib["t_start_ms"] for s in starts) <= 16


def test_growth_beyond_the_footprint_stays_within_budget():
    """Requests whose device need grows to 2.5x their initial footprint (as
    candidate records do): each stops at its reservation, goes back to the
    queue with twice the reservation and finishes; the bytes in use never
    exceed the budget, and none fails."""
    sizes = [800, 2000, 1200, 3000, 600, 1500, 2500, 1000]
    budget = int(2.6 * fp(3000)) + fp(2000)
    with pc.Server(slots=4, hbm_budget_bytes=budget, fake_us_per_kpoint=US_PER_KPT,
                   fake_growth=2.5) as srv:
        ts = [srv.submit(pts(n, i), "ward") for i, n in enumerate(sizes)]
        infos = [srv.result(t)[1] for t in ts]
        st = srv.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0
    assert st["requeued"] >= len(sizes)  # each needed one larger reservation
    assert st["peak_bytes_in_use"] <= budget
    for n, info in zip(sizes, infos):
        assert info["status"] == 0 and info["footprint_bytes"] >= 2.5 * fp(n)


def test_growth_beyond_the_budget_fails():
    with pc.Server(slots=2, hbm_budget_bytes=int(1.5 * fp(2000)), fake_us_per_kpoint=US_PER_KPT,
                   fake_growth=3.0) as srv:
        t = srv.submit(pts(2000), "ward")
        with pytest.raises(PCError) as e:
            srv.result(t)
        assert e.value.status == -3
        assert srv.stats()["failed"] == 1


def test_cancel_and_shutdown():
    srv = pc.Server(slots=1, hbm_budget_bytes=1 << 40, fake_us_per_kpoint=US_PER_KPT)
    ta = srv.submit(pts(5000), "complete")            # ~100 ms on the only slot
    time.sleep(0.02)
    tb = srv.submit(pts(100), "complete")
    tc = srv.submit(pts(100), "complete")
    with pytest.raises(PCError) as e:
        srv.cancel(ta)                                 # running
    assert e.value.status == -6
    srv.cancel(tb)
    info = srv.poll(tb)
    assert info["state"] == "cancelled" and info["status"] == -7
    with pytest.raises(PCError) as e:
        srv.wait(tc, timeout_ms=1.0)                   # still behind a
    assert e.value.status == -6
    srv.result(ta)
    srv.result(tc)
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 2
    # destroy with waiting requests: they are cancelled, the running one finishes
    srv.submit(pts(3000), "complete")
    for i in range(5):
        srv.submit(pts(3000), "complete")
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 1.0


def test_poll_reports_done_and_status():
    """pc_server_poll's form: (done, status) while a request waits, runs,
    finishes or is cancelled; pc_server_query keeps the full record."""
    with pc.Server(slots=1, hbm_budget_bytes=1 << 40, fake_us_per_kpoint=US_PER_KPT) as srv:
        a = srv.submit(pts(3000), "ward")  # 60 ms
        b = srv.submit(pts(100, 1), "ward")
        time.sleep(0.005)
        assert srv.done(a) == (False, -6)
        assert srv.done(b) == (False, -6)
        srv.cancel(b)
        assert srv.done(b) == (True, -7)
        srv.wait(a)
        assert srv.done(a) == (True, 0)
        assert srv.poll(a)["state"] == "done"
        with pytest.raises(PCError):
            srv.done(12345)
