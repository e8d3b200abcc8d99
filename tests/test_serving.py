"""Continuous-batching server (srv_* entry points).

CPU tests drive the host-only executor (device -1): requests are validated,
prepared, admitted by free slot and memory footprint in arrival order
(later requests may pass one that does not fit), advanced in chunks and
retired, with zero observables.  GPU tests check that a request's results
do not depend on what else runs and equal a plain single rollout."""
import numpy as np
import pytest

from paper_2603_25068_amd import workloads as W


def _srv(**kw):
    from paper_2603_25068_amd.sim import Server
    return Server(**kw)


def _reqs(n, seed=0, steps=120):
    """n small metro nowcast requests (the request generator's size mix, scaled down)."""
    return [W.metro(**spec) for _, spec in W.serving_requests(n, seed=seed, steps=steps, scale=0.02)]


def test_footprint_is_positive_and_grows_with_agents():
    from paper_2603_25068_amd.sim import footprint
    a = W.random_small(1, nx=4, ny=4, n_agents=200, steps=100)
    b = W.random_small(1, nx=4, ny=4, n_agents=20000, steps=100)
    fa, fb = footprint(a), footprint(b)
    assert 0 < fa < fb
    assert footprint(a, n_scenarios=4) > fa
    assert footprint(a, record=True) > fa


def test_host_executor_completes_all_requests():
    from paper_2603_25068_amd.sim import SRV_DONE
    ws = _reqs(12, seed=1)
    with _srv(device=-1, mem_budget_bytes=1 << 34, max_slots=4, chunk_steps=30) as s:
        tickets = [s.submit(w, steps=120) for w in ws]
        for t in tickets:
            assert s.wait(t, 60.0) == SRV_DONE
            counts, ttt, vs, lat = s.result(t)
            assert counts.shape[0] == 1 and lat > 0
        st = s.stats()
        assert st["completed"] == 12
        assert 1 <= st["max_running"] <= 4
        assert st["p50_s"] <= st["p99_s"]


def test_max_slots_bounds_concurrency():
    from paper_2603_25068_amd.sim import SRV_DONE
    ws = _reqs(10, seed=2)
    with _srv(device=-1, mem_budget_bytes=1 << 34, max_slots=2, chunk_steps=10) as s:
        ts = [s.submit(w, steps=100) for w in ws]
        assert all(s.wait(t, 60.0) == SRV_DONE for t in ts)
        assert s.stats()["max_running"] == 2


def test_memory_budget_bounds_concurrency():
    from paper_2603_25068_amd.sim import SRV_DONE, footprint
    w = W.random_small(4, nx=4, ny=4, n_agents=2000, steps=100)
    f = footprint(w, steps=100)
    with _srv(device=-1, mem_budget_bytes=int(2.5 * f), max_slots=8, chunk_steps=10) as s:
        ts = [s.submit(w, steps=100) for _ in range(6)]
        assert all(s.wait(t, 60.0) == SRV_DONE for t in ts)
        assert s.stats()["max_running"] == 2


def test_pool_ranges_are_reused_across_sizes():
    """Requests of two sizes share the server's pool: each takes a contiguous range of its
    footprint (first fit), freed ranges merge with their neighbours, so a large request waits for
    adjacent small ones to finish and then runs; every request completes and no more run at once
    than the pool holds."""
    from paper_2603_25068_amd.sim import SRV_DONE, footprint
    small = W.random_small(4, nx=4, ny=4, n_agents=1500, steps=100)
    big = W.random_small(5, nx=8, ny=8, n_agents=40000, steps=100)
    fs = (footprint(small, steps=100) + 255) // 256 * 256
    fb = (footprint(big, steps=100) + 255) // 256 * 256
    assert fb > 2 * fs
    budget = fb + fs
    order = [small, small, big, small, big, small, small, big]
    with _srv(device=-1, mem_budget_bytes=budget, max_slots=8, chunk_steps=10) as s:
        ts = [s.submit(w, steps=100) for w in order]
        assert all(s.wait(t, 60.0) == SRV_DONE for t in ts)
        st = s.stats()
        assert st["completed"] == len(order)
        assert 2 <= st["max_running"] <= budget // fs


def test_oversize_request_fails_alone():
    from paper_2603_25068_amd.sim import SRV_DONE, SRV_FAILED, SIM_ENOMEM, SimError, footprint
    small = W.random_small(5, nx=4, ny=4, n_agents=300, steps=100)
    big = W.random_small(5, nx=8, ny=8, n_agents=40000, steps=100)
    budget = 2 * footprint(small, steps=100)
    assert footprint(big, steps=100) > budget
    with _srv(device=-1, mem_budget_bytes=budget, max_slots=4, chunk_steps=20) as s:
        t0 = s.submit(small, steps=100)
        tb = s.submit(big, steps=100)
        t1 = s.submit(small, steps=100)
        assert s.wait(tb, 60.0) == SRV_FAILED
        assert "budget" in s.error(tb)
        with pytest.raises(SimError) as e:
            s.result(tb)
        assert e.value.code == SIM_ENOMEM
        assert s.wait(t0, 60.0) == SRV_DONE and s.wait(t1, 60.0) == SRV_DONE


def test_malformed_request_fails_without_disturbing_others():
    from paper_2603_25068_amd.sim import SRV_DONE, SRV_FAILED, SIM_EINVAL, SimError
    good = _reqs(3, seed=3)
    bad = W.random_small(6, nx=4, ny=4, n_agents=300, steps=100)
    bad.net.length = bad.net.length.copy()
    bad.net.length[0] = -5.0
    bad2 = W.random_small(7, nx=4, ny=4, n_agents=300, steps=100)
    bad2.dem.agent_dest = bad2.dem.agent_dest.copy()
    bad2.dem.agent_dest[3] = bad2.net.n_nodes + 7
    with _srv(device=-1, mem_budget_bytes=1 << 34, max_slots=2, chunk_steps=20) as s:
        tg = [s.submit(w, steps=100) for w in good]
        tb = [s.submit(bad, steps=100), s.submit(bad2, steps=100)]
        for t in tb:
            assert s.wait(t, 60.0) == SRV_FAILED
            with pytest.raises(SimError) as e:
                s.result(t)
            assert e.value.code == SIM_EINVAL
            assert s.error(t)
        assert all(s.wait(t, 60.0) == SRV_DONE for t in tg)


def test_cancel_and_unknown_ticket():
    from paper_2603_25068_amd.sim import SRV_CANCELLED, SRV_DONE, SIM_ESTATE, SimError
    ws = _reqs(6, seed=4)
    with _srv(device=-1, mem_budget_bytes=1 << 34, max_slots=1, chunk_steps=1) as s:
        ts = [s.submit(w, steps=2000) for w in ws]
        s.cancel(ts[-1])
        assert s.wait(ts[-1], 60.0) == SRV_CANCELLED
        with pytest.raises(SimError) as e:
            s.result(ts[-1])
        assert e.value.code == SIM_ESTATE
        for t in ts[:-1]:
            s.cancel(t)
        for t in ts[:-1]:
            assert s.wait(t, 60.0) in (SRV_CANCELLED, SRV_DONE)
        with pytest.raises(SimError):
            s.poll(10 ** 9)


def test_destroy_with_requests_in_flight():
    ws = _reqs(8, seed=5)
    s = _srv(device=-1, mem_budget_bytes=1 << 34, max_slots=2, chunk_steps=1)
    for w in ws:
        s.submit(w, steps=5000)
    s.close()


@pytest.mark.gpu
def test_results_do_not_depend_on_the_mix():
    """Each request alone equals the same request in a mix of 16, and both
    equal a plain single rollout through the simulator handle."""
    from paper_2603_25068_amd.sim import SRV_DONE, Simulator
    ws = _reqs(16, seed=7, steps=240)
    with _srv(device=0, mem_budget_bytes=8 << 30, max_slots=6, chunk_steps=45) as s:
        ts = [s.submit(w, steps=240) for w in ws]
        mix = []
        for t in ts:
            assert s.wait(t, 120.0) == SRV_DONE, s.error(t)
            mix.append(s.result(t))
        assert s.stats()["max_running"] > 1
    for i in (0, 5, 11):
        with _srv(device=0, mem_budget_bytes=8 << 30, max_slots=1, chunk_steps=240) as s:
            t = s.submit(ws[i], steps=240)
            assert s.wait(t, 120.0) == SRV_DONE, s.error(t)
            alone = s.result(t)
        sim = Simulator(ws[i], steps=240).rollout(240)
        c, T = sim.observables()
        for a, b in ((mix[i][0], alone[0]), (mix[i][0], c)):
            assert np.array_equal(a, b)
        assert mix[i][1][0] == alone[1][0] == T[0]
        assert mix[i][2][0] == alone[2][0] == int(sim.vehicle_steps()[0])
