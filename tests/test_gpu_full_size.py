"""HIP path against the oracle at the full sizes the benchmark runs, through
the C-ABI:

- the 1M-agent metro workload over its whole 1,800-step horizon in the
  benchmark's launch configuration, with the oracle adopting the library's
  near-tie log (at a near tie either outcome is correct; the oracle takes the
  library's decision only where its own margin is within rounding of a tie
  and only among its own candidates), state at 900 and 1,800 steps
  bit-exact, and the full-horizon gradient in every group within 1e-3;
- the batched-control workload at size (16 scenarios of 50k agents on the
  32x32 lattice, 3,600 steps, one launch per step): scenarios 0, 7 and 15
  against the oracle on state and on the capacity-multiplier gradient;
- served nowcast requests, one per size class, against the oracle;
- the state hand-off: a GPU run restored from a saved state and an oracle
  restored from its own saved state continue identically.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2603_25068_amd import workloads as W

pytestmark = pytest.mark.gpu

ALL_GROUPS = ("free_speed", "jam_density", "rates", "cap_mult", "beta", "cost", "alpha", "theta")


def _say(msg):
    print(f"[full-size] {msg}", flush=True)


def _compare(o, sg, lg, scen=0, ctx=""):
    """Oracle state against a library state (sim.state()) and link state (sim.link_state())."""
    so = o.state()
    assert np.array_equal(so["status"], sg["status"][scen]), f"{ctx}: status differs"
    on = so["status"] == oracle.ST_ON
    for k in ("link", "seq"):
        assert np.array_equal(so[k][on], sg[k][scen][on]), f"{ctx}: {k} differs"
    xo, xg = so["pos"][on].astype(np.float32), sg["pos"][scen][on]
    assert np.array_equal(xo, xg), f"{ctx}: positions differ, max {np.abs(xo - xg).max() if xo.size else 0}"
    co, cg = o.counters(), sg["counters"][scen]
    for k in ("released", "departed", "on_net", "exited", "transfers", "stuck", "order_viol"):
        assert co[k] == cg[k], f"{ctx}: counter {k}: oracle {co[k]} gpu {cg[k]}"
    lo = o.link_state()
    for k in ("E", "next_seq", "B"):
        assert np.array_equal(lo[k], lg[k][scen]), f"{ctx}: link {k} differs"
    return int(on.sum())


def _grad_close(go, gg, name, rtol=1e-3):
    go = np.asarray(go, np.float64).ravel()
    gg = np.asarray(gg, np.float64).ravel()
    scale = np.abs(go).max()
    if scale == 0:
        assert np.abs(gg).max() == 0, name
        return
    big = np.abs(go) > 1e-3 * scale
    rel = np.abs(gg[big] - go[big]) / np.abs(go[big])
    assert rel.max() <= rtol, f"{name}: component rel err {rel.max():.3g}"
    assert np.linalg.norm(gg - go) <= rtol * np.linalg.norm(go), f"{name}: norm rel err"


def test_metro_full_horizon_with_tie_adoption():
    from paper_2603_25068_amd.sim import Simulator
    w = W.metro()
    T, Th = w.cfg.steps, w.cfg.steps // 2
    t0 = time.perf_counter()
    s = Simulator(w, record=True, max_steps=T, tape_windows=T // w.cfg.ckpt_every)   # every window taped
    s.rollout()
    s.autotune(probe_steps=30)          # as the benchmark: tuned on the end-of-rollout state
    s.reset()
    s.step(Th)
    sg1, lg1 = s.state(), s.link_state()
    s.step(T - Th)
    sg2, lg2 = s.state(), s.link_state()
    cg, tg = s.observables()
    lib_log = s.tie_log()
    rng = np.random.default_rng(11)
    gQ = rng.normal(size=cg.shape[1:]).astype(np.float32)
    gg = s.backward(gQ=gQ[None], gT=[0.25], groups=ALL_GROUPS)
    _say(f"library pass done in {time.perf_counter() - t0:.1f} s; {len(lib_log)} near-tie records "
         f"{np.bincount(lib_log[:, 2], minlength=2).tolist() if len(lib_log) else []}")
    assert sg2["counters"][0]["ties"] == len(lib_log)
    o = Oracle(w, log=True, adopt=Oracle.tie_log_from_library(lib_log))
    o.run(Th)
    n1 = _compare(o, sg1, lg1, ctx=f"metro after {Th} steps")
    _say(f"oracle at step {Th}: {n1} agents on the network, bit-exact ({time.perf_counter() - t0:.1f} s)")
    o.run(T - Th)
    n2 = _compare(o, sg2, lg2, ctx=f"metro after {T} steps")
    co, to = o.counts()
    assert np.array_equal(co.astype(np.float32), cg[0]) and to == tg[0]
    st = o.tie_stats()
    _say(f"oracle at step {T}: {n2} on the network, counts and travel time equal; ties {st}")
    # the route-choice and merge near ties of both sides are the same events with the same
    # decisions (position thresholds are logged by the oracle only: both sides take them on the
    # same float positions)
    own = o.tie_log()
    own = own[own[:, 1] <= oracle.TIE_MERGE]
    lib = Oracle.tie_log_from_library(lib_log)
    assert sorted(map(tuple, own.tolist())) == sorted(map(tuple, lib.tolist()))
    assert st["flipped"] <= len(lib)
    go = o.backward(gQ=gQ.astype(np.float64), gT=0.25)
    for k in ALL_GROUPS:
        _grad_close(go[k], gg[k][0], f"metro full horizon {k}")
    _say(f"gradients within 1e-3 in every group ({time.perf_counter() - t0:.1f} s)")


def test_batched_control_at_size():
    """16 scenarios x 50k agents, 3,600 steps, one launch per step, autotuned as the benchmark
    runs it; scenarios 0, 7 and 15 against the oracle (each with its own multipliers and Philox
    key, seed + s): state and counts bit-exact, travel-time gradient in the multipliers within
    1e-3."""
    from paper_2603_25068_amd.sim import Simulator
    w = W.batched_control()
    S, T = int(w.extra["n_scenarios"]), w.cfg.steps
    m = w.extra["cap_mult"]
    t0 = time.perf_counter()
    s = Simulator(w, n_scenarios=S, record=True, max_steps=T, params={"cap_mult": m})
    s.rollout()
    s.autotune(probe_steps=20)
    s.reset()
    s.step(T)
    sg, lg = s.state(), s.link_state()
    cg, tg = s.observables()
    gg = s.backward(gT=np.ones(S), groups=("cap_mult",))["cap_mult"]
    _say(f"16 scenarios done in {time.perf_counter() - t0:.1f} s")
    for k in (0, 7, 15):
        o = Oracle(w, log=True, params={"cap_mult": m[k]}, seed=w.cfg.seed + k).run()
        _compare(o, sg, lg, scen=k, ctx=f"scenario {k}")
        co, to = o.counts()
        assert np.array_equal(co.astype(np.float32), cg[k]) and to == tg[k]
        go = o.backward(gT=1.0)["cap_mult"]
        assert np.count_nonzero(go) > 100
        _grad_close(go, gg[k], f"cap_mult scenario {k}")
        _say(f"scenario {k} equal to the oracle ({time.perf_counter() - t0:.1f} s)")


def test_served_requests_match_the_oracle():
    """A mix of nowcast requests through the continuous-batching server; the smallest request of
    each size class (agents below 50k, 50k-200k, 200k-1M) equals the oracle's rollout of it."""
    from paper_2603_25068_amd.sim import SRV_DONE, Server
    reqs = W.serving_requests(48, steps=3600)
    sizes = [spec["n_agents"] for _, spec in reqs]
    classes = [(0, 50_000), (50_000, 200_000), (200_000, 2_000_000)]
    picked = []
    for lo, hi in classes:
        inside = [i for i, n in enumerate(sizes) if lo <= n < hi]
        if inside:
            picked.append(min(inside, key=lambda i: sizes[i]))
    assert len(picked) == 3
    others = [i for i in range(len(reqs)) if i not in picked][:5]
    order = sorted(picked + others)
    ws = {i: W.metro(**reqs[i][1]) for i in order}
    t0 = time.perf_counter()
    with Server(device=0, mem_budget_bytes=32 << 30, max_slots=8, chunk_steps=60) as srv:
        tickets = {i: srv.submit(ws[i], steps=3600) for i in order}
        res = {}
        for i in order:
            assert srv.wait(tickets[i], 600.0) == SRV_DONE, srv.error(tickets[i])
            res[i] = srv.result(tickets[i])
        mr = srv.stats()["max_running"]
    _say(f"{len(order)} requests served in {time.perf_counter() - t0:.1f} s, up to {mr} at once")
    assert mr >= 2
    for i in picked:
        w = ws[i]
        o = Oracle(w, steps=3600).run(3600)
        co, to = o.counts()
        counts, ttt, vs, _ = res[i]
        assert np.array_equal(co.astype(np.float32), counts[0]), f"request {i}: counts differ"
        assert to == ttt[0], f"request {i}: travel time differs"
        _say(f"request {i} ({w.dem.n_agents} agents, {w.net.n_links} links) equals the oracle "
             f"({time.perf_counter() - t0:.1f} s)")


@pytest.mark.parametrize("mk,T0,T1", [(lambda: W.grid_rates(), 700, 1800),
                                      (lambda: W.random_small(12, nx=6, ny=6, n_agents=3000, rates=True,
                                                              steps=600), 233, 600)])
def test_nowcast_hand_off_against_the_oracle(mk, T0, T1):
    """A GPU run saved at T0 and restored into a fresh handle continues to T1; an oracle restored
    from its own saved state at T0 continues to T1; both equal (bit-exact) and equal the
    uninterrupted oracle run."""
    from paper_2603_25068_amd.sim import Simulator
    w = mk()
    a = Simulator(w)
    a.step(T0)
    blob = a.full_state()
    b = Simulator(w)
    b.set_full_state(blob)
    b.step(T1 - T0)
    o = Oracle(w)
    o.run(T0)
    ob = Oracle(w).import_state(o.export_state())
    ob.run(T1 - T0)
    o.run(T1 - T0)
    sg, lg = b.state(), b.link_state()
    n = _compare(ob, sg, lg, ctx="restored GPU vs restored oracle")
    _compare(o, sg, lg, ctx="restored GPU vs uninterrupted oracle")
    cg, tg = b.observables()
    co, to = ob.counts()
    assert np.array_equal(co.astype(np.float32), cg[0]) and to == tg[0]
    assert n > 0
