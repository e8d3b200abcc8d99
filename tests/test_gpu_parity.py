"""HIP path against the oracle, element by element, through the C-ABI.

Integer state (status, link, entry sequence, counters, cumulative outflow,
detector counts) must be bit-exact; positions too (both sides carry them in
float with the same operation order); token buckets and release
accumulators (double, same operation order) bit-exact; gradients within
1e-3 relative (GPU float adjoint vs oracle double adjoint on the same
trajectory).
"""
import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2603_25068_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, **kw):
    from paper_2603_25068_amd.sim import Simulator
    return Simulator(w, **kw)


def _compare_state(o, s, scen=0, ctx=""):
    so = o.state()
    sg = s.state()
    st_o, st_g = so["status"], sg["status"][scen]
    assert np.array_equal(st_o, st_g), f"{ctx}: status differs at agents {np.where(st_o != st_g)[0][:10]}"
    on = st_o == oracle.ST_ON
    assert np.array_equal(so["link"][on], sg["link"][scen][on]), f"{ctx}: link differs"
    assert np.array_equal(so["seq"][on], sg["seq"][scen][on]), f"{ctx}: seq differs"
    xo = so["pos"][on].astype(np.float32)
    xg = sg["pos"][scen][on]
    assert np.array_equal(xo, xg), f"{ctx}: positions differ, max {np.abs(xo - xg).max() if xo.size else 0}"
    co = o.counters()
    cg = sg["counters"][scen]
    for k in ("released", "departed", "exited", "transfers", "stuck", "order_viol"):
        assert co[k] == cg[k], f"{ctx}: counter {k}: oracle {co[k]} gpu {cg[k]}"
    assert co["on_net"] == cg["on_net"]
    lo, lg = o.link_state(), s.link_state()
    assert np.array_equal(lo["E"], lg["E"][scen]), f"{ctx}: cumulative outflow differs"
    assert np.array_equal(lo["next_seq"], lg["next_seq"][scen])
    assert np.array_equal(lo["B"], lg["B"][scen]), f"{ctx}: token buckets differ"


def test_philox_device_matches_host():
    w = W.tg_toy()
    s = _sim(w)
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(257, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(257, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    dev = s.philox(ctr, key)
    host = np.stack([oracle.philox(ctr[i], key[i]) for i in range(len(ctr))])
    assert np.array_equal(dev, host)
    assert [int(x) for x in dev[0]] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


def test_shortest_times_match_oracle_bitwise():
    w = W.random_small(5, nx=5, ny=4, n_agents=80)
    assert np.array_equal(_sim(w).dist_table(), Oracle(w).dist_table())


def test_tg_toy_gradient():
    w = W.tg_toy(2.0, 1.0)
    s = _sim(w, record=True, max_steps=10, ckpt_every=4)
    s.place([0], [0], [0.0])
    s.step(10)
    st = s.state()
    assert st["link"][0, 0] == 1 and st["pos"][0, 0] == 2.0
    g = s.backward(gx=np.array([[4.0]]), groups=("free_speed",))
    assert np.allclose(g["free_speed"][0], [32.0, 8.0])


@pytest.mark.parametrize("mk", [W.small_grid_fixed, lambda: W.diamond(300, lanes=2, capacity=0.3),
                                lambda: W.random_small(11, nx=4, ny=4, n_agents=400, rates=True, steps=300)])
def test_forward_parity_stepwise(mk):
    w = mk()
    o = Oracle(w)
    s = _sim(w)
    for t in range(w.cfg.steps):
        o.step()
        s.step()
        if t % 25 == 24 or t == w.cfg.steps - 1:
            _compare_state(o, s, ctx=f"{w.name} t={t}")
    co, to = o.counts()
    cg, tg = s.observables()
    assert np.array_equal(co.astype(np.float32), cg[0])
    assert to == tg[0]


@pytest.mark.parametrize("seed", [21, 22, 23, 24])
def test_forward_parity_random(seed):
    w = W.random_small(seed, nx=5, ny=5, n_agents=900, rates=bool(seed % 2), steps=400, lanes_max=3)
    o = Oracle(w).run()
    s = _sim(w).rollout()
    _compare_state(o, s, ctx=w.name)
    co, to = o.counts()
    cg, tg = s.observables()
    assert np.array_equal(co.astype(np.float32), cg[0]) and to == tg[0]


@pytest.mark.parametrize("seed", [5, 8])
def test_merge_ranks_on_double_keys_parity(seed):
    """Merge priorities near 600 put every merge key beyond the range of the
    kernel's single-precision fast pass (|key| < 512), so every node group
    with a chooser ranks its merge on double-precision keys; state and counts
    still equal the oracle's bit for bit."""
    w = W.random_small(seed, nx=5, ny=5, n_agents=900, rates=False, steps=400, lanes_max=3)
    alpha = np.random.default_rng(seed).uniform(600.0, 601.0, w.net.n_links).astype(np.float32)
    o = Oracle(w, params={"alpha": alpha}).run()
    s = _sim(w, params={"alpha": alpha}).rollout()
    _compare_state(o, s, ctx=f"{w.name} with alpha near 600")
    assert o.counters()["transfers"] > 100
    co, to = o.counts()
    cg, tg = s.observables()
    assert np.array_equal(co.astype(np.float32), cg[0]) and to == tg[0]


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


@pytest.mark.parametrize("seed", [2, 6, 31])
def test_gradient_parity(seed):
    w = W.random_small(seed, nx=4, ny=4, n_agents=500, rates=True, steps=300)
    o = Oracle(w, log=True).run()
    s = _sim(w, record=True, ckpt_every=37).rollout()
    _compare_state(o, s, ctx="trajectory")
    rng = np.random.default_rng(seed)
    cnt, _ = o.counts()
    gQ = rng.normal(size=cnt.shape).astype(np.float32)
    st = o.state()
    gx = (rng.normal(size=w.dem.n_agents) * (st["status"] == oracle.ST_ON)).astype(np.float32)
    gT = 0.25
    go = o.backward(gQ=gQ.astype(np.float64), gT=gT, gx=gx.astype(np.float64))
    gg = s.backward(gQ=gQ[None], gT=[gT], gx=gx[None])
    for k in ("free_speed", "jam_density", "rates"):
        _grad_close(go[k], gg[k][0], k)


def test_checkpoint_interval_does_not_change_gradients():
    w = W.random_small(8, nx=4, ny=4, n_agents=400, rates=True, steps=240)
    rng = np.random.default_rng(1)
    gQ = rng.normal(size=(1, w.net.n_detectors, 4)).astype(np.float32)
    out = []
    for ck in (1, 60, 240):
        s = _sim(w, record=True, ckpt_every=ck).rollout()
        out.append(s.backward(gQ=gQ, gT=[0.5]))
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]) and np.array_equal(out[0][k], out[2][k]), k


def test_scenario_batch_equals_single_runs():
    w = W.random_small(9, nx=4, ny=4, n_agents=500, rates=True, steps=240)
    S = 3
    rng = np.random.default_rng(3)
    u = np.stack([w.net.free_speed * rng.uniform(0.8, 1.2, w.net.n_links) for _ in range(S)]).astype(np.float32)
    m = rng.uniform(0.5, 1.0, (S, w.net.n_links)).astype(np.float32)
    seeds = [100 + s for s in range(S)]
    gQ = rng.normal(size=(S, w.net.n_detectors, 4)).astype(np.float32)
    b = _sim(w, n_scenarios=S, params={"free_speed": u, "cap_mult": m}, seeds=seeds, record=True).rollout()
    cb, tb = b.observables()
    gb = b.backward(gQ=gQ, gT=np.ones(S))
    stb = b.state()
    for s in range(S):
        a = _sim(w, params={"free_speed": u[s], "cap_mult": m[s]}, seeds=[seeds[s]], record=True).rollout()
        ca, ta = a.observables()
        assert np.array_equal(ca[0], cb[s]) and ta[0] == tb[s]
        sta = a.state()
        for k in ("status", "link", "pos", "seq"):
            assert np.array_equal(sta[k][0], stb[k][s]), (s, k)
        ga = a.backward(gQ=gQ[s:s + 1], gT=[1.0])
        for k in ga:
            assert np.array_equal(ga[k][0], gb[k][s]), (s, k)
        # and the oracle agrees with this scenario
        o = Oracle(w, params={"free_speed": u[s], "cap_mult": m[s]}, seed=seeds[s]).run()
        _compare_state(o, b, scen=s, ctx=f"scenario {s}")


def test_segsort_matches_lexsort():
    import torch
    w = W.tg_toy()
    s = _sim(w)
    rng = np.random.default_rng(4)
    n, nseg = 20000, 300
    seg = rng.integers(0, nseg, n).astype(np.int32)
    pos = rng.choice(np.float32([0.0, 1.5, 2.25, 100.0, 7.0]), n) + rng.integers(0, 3, n).astype(np.float32)
    seq = rng.integers(0, 50, n).astype(np.int32)
    dev = torch.device("cuda", 0)
    perm, off = s.segsort(torch.from_numpy(seg).to(dev), torch.from_numpy(pos).to(dev),
                          torch.from_numpy(seq).to(dev), nseg)
    ref = np.lexsort((np.arange(n), seq, -pos, seg))
    assert np.array_equal(perm.cpu().numpy(), ref)
    assert np.array_equal(off.cpu().numpy(), np.concatenate([[0], np.cumsum(np.bincount(seg, minlength=nseg))]))


def test_errors_are_reported():
    from paper_2603_25068_amd.sim import SimError, SIM_EINVAL, SIM_ESTATE
    w = W.tg_toy()
    w.net.length = np.float32([15.0, -1.0])
    with pytest.raises(SimError) as e:
        _sim(w)
    assert e.value.code == SIM_EINVAL
    w = W.tg_toy()
    s = _sim(w)
    with pytest.raises(SimError) as e:
        s.backward(gx=np.zeros((1, 1)))
    assert e.value.code == SIM_ESTATE
    s.step(3)
    with pytest.raises(SimError) as e:
        s.place([0], [0], [0.0])
    assert e.value.code == SIM_ESTATE


@pytest.mark.parametrize("sched", [(16, 64, 16), (32, 64, 32), (64, 64, 64), (16, 32, 64), (8, 16, 8)])
def test_schedules_give_identical_results(sched):
    w = W.random_small(12, nx=5, ny=5, n_agents=800, rates=True, steps=300, lanes_max=3)
    ref = _sim(w, record=True, ckpt_every=50).rollout()
    cr, tr = ref.observables()
    gr = ref.backward(gQ=np.ones((1,) + cr.shape[1:], np.float32), gT=[1.0])
    s = _sim(w, record=True, ckpt_every=50)
    need = s.schedule()[1]
    gl, gn, gv = sched
    s.set_schedule(gl, max(gn, need), gv)
    s.rollout()
    cs, ts = s.observables()
    assert np.array_equal(cr, cs) and np.array_equal(tr, ts)
    a, b = ref.state(), s.state()
    for k in ("status", "link", "pos", "seq"):
        assert np.array_equal(a[k], b[k]), k
    gs = s.backward(gQ=np.ones((1,) + cr.shape[1:], np.float32), gT=[1.0])
    for k in gr:
        assert np.array_equal(gr[k], gs[k]), k


@pytest.mark.parametrize("seed", [3, 9])
def test_capacity_multiplier_gradient_parity(seed):
    """Admission-time graft on the GPU against the oracle, with binding
    buckets and random multipliers; every other group on the same run too."""
    w = W.random_small(seed, nx=4, ny=4, n_agents=600, rates=True, steps=300)
    w.net.capacity = np.full(w.net.n_links, 0.12, np.float32)
    rng = np.random.default_rng(seed)
    m = rng.uniform(0.5, 1.0, w.net.n_links).astype(np.float32)
    o = Oracle(w, log=True, params={"cap_mult": m}).run()
    s = _sim(w, record=True, ckpt_every=45, params={"cap_mult": m}).rollout()
    _compare_state(o, s, ctx="trajectory")
    cnt, _ = o.counts()
    gQ = rng.normal(size=cnt.shape).astype(np.float32)
    gT = 0.7
    go = o.backward(gQ=gQ.astype(np.float64), gT=gT)
    gg = s.backward(gQ=gQ[None], gT=[gT], groups=("free_speed", "jam_density", "rates", "cap_mult"))
    assert np.count_nonzero(go["cap_mult"]) > 3
    for k in ("free_speed", "jam_density", "rates", "cap_mult"):
        _grad_close(go[k], gg[k][0], k)


def test_bottleneck_capacity_gradient_closed_form_gpu():
    N, q = 10, 0.5
    w = W.line(n_links=2, length=200.0, speed=13.9, lanes=1, capacity=q, n_agents=N, steps=60)
    m = np.float32([0.8, 1.0])
    s = _sim(w, record=True, max_steps=60, ckpt_every=7, params={"cap_mult": m})
    sp = 1.0 / float(np.float32(w.net.jam_density[0]))
    s.place(list(range(N)), [0] * N, [200.0 - k * sp for k in range(N)])
    s.step(60)
    g = s.backward(gT=[1.0], groups=("cap_mult",))["cap_mult"][0]
    mm = float(m[0])
    assert g[0] == pytest.approx(-sum(k / (mm * mm * q) for k in range(1, N + 1)), rel=1e-5)
    assert g[1] == 0.0


def test_batched_control_gradients_match_oracle():
    """Candidate control scenarios in one launch per step: each scenario's
    total-travel-time gradient in the capacity multipliers of the controlled
    links equals the oracle's for that scenario."""
    w = W.random_small(14, nx=4, ny=4, n_agents=700, rates=True, steps=300)
    w.net.capacity = np.full(w.net.n_links, 0.15, np.float32)
    S = 4
    ctrl, m = W.control_multipliers(w.net.n_links, w.net.n_links // 2, S, seed0=500)
    seeds = [200 + k for k in range(S)]
    s = _sim(w, n_scenarios=S, record=True, params={"cap_mult": m}, seeds=seeds).rollout()
    gg = s.backward(gT=np.ones(S), groups=("cap_mult",))["cap_mult"]
    for k in range(S):
        o = Oracle(w, log=True, params={"cap_mult": m[k]}, seed=seeds[k]).run()
        _compare_state(o, s, scen=k, ctx=f"scenario {k}")
        go = o.backward(gT=1.0)["cap_mult"]
        _grad_close(go, gg[k], f"cap_mult scenario {k}")


@pytest.mark.parametrize("seed", [4, 10, 23])
def test_straight_through_gradient_parity(seed):
    """beta, cost, alpha and theta through the straight-through node model
    (SI-B) on the GPU against the oracle, with every other group on the same
    run; two scenarios with their own seeds and utilities in one launch."""
    w = W.random_small(seed, nx=4, ny=4, n_agents=600, rates=True, steps=300)
    rng = np.random.default_rng(seed)
    L, S = w.net.n_links, 2
    prm = {"beta": rng.uniform(0.5, 2.0, (S, L)).astype(np.float32),
           "cost": rng.uniform(1.0, 3.0, (S, L)).astype(np.float32),
           "alpha": rng.uniform(0.5, 2.0, (S, L)).astype(np.float32)}
    seeds = [seed * 7 + k for k in range(S)]
    s = _sim(w, n_scenarios=S, record=True, ckpt_every=41, params=prm, seeds=seeds).rollout()
    groups = ("free_speed", "jam_density", "rates", "beta", "cost", "alpha", "theta")
    cg, _ = s.observables()
    gQ = rng.normal(size=cg.shape).astype(np.float32)
    gT = np.array([0.3, -0.2])
    gg = s.backward(gQ=gQ, gT=gT, groups=groups)
    for k in range(S):
        o = Oracle(w, log=True, params={n: prm[n][k] for n in prm}, seed=seeds[k]).run()
        _compare_state(o, s, scen=k, ctx=f"scenario {k}")
        go = o.backward(gQ=gQ[k].astype(np.float64), gT=float(gT[k]))
        for g in ("beta", "cost", "alpha", "theta"):
            assert np.abs(go[g]).max() > 0, g
        for g in groups:
            _grad_close(go[g], gg[g][k], f"{g} scenario {k}")


@pytest.mark.parametrize("alpha,seed", [((1.0, 1.0), 0), ((1.3, 0.6), 5), ((0.8, 1.1), 9)])
def test_merge_priority_gradient_closed_form_gpu(alpha, seed):
    """Two heads, one entry slot: dL/d alpha_w = -dL/d alpha_l =
    p'_w p'_l / tau (M adj_w + (M + L) adj_l) with p' the merge softmax of
    (alpha_from + g')/tau; one route candidate, so beta and cost get nothing."""
    w = W.merge_toy(alpha=alpha, seed=seed)
    length, tau, bigm = 100.0, w.cfg.gumbel_tau, w.cfg.big_m
    s = _sim(w, record=True, max_steps=1)
    s.place([0, 1], [0, 1], [length, length])
    s.step(1)
    st = s.state()
    win = int(np.where(st["link"][0] == 2)[0][0])
    lose = 1 - win
    assert st["link"][0][lose] == lose and st["pos"][0][lose] == length
    adj = np.float32([0.7, -1.3])
    g = s.backward(gx=adj[None], groups=("alpha", "beta", "cost", "theta"))
    keys = np.array([float(np.float32(alpha[a])) + oracle.gumbel(w.cfg.seed, a, 0, 1, 0) for a in (0, 1)])
    p = np.exp(keys / tau - (keys / tau).max())
    p /= p.sum()
    expect = p[win] * p[lose] / tau * (bigm * adj[win] + (bigm + length) * adj[lose])
    assert g["alpha"][0][win] == pytest.approx(expect, rel=1e-5)
    assert g["alpha"][0][lose] == pytest.approx(-expect, rel=1e-5)
    assert np.all(g["beta"] == 0.0) and np.all(g["cost"] == 0.0) and np.all(g["theta"] == 0.0)


@pytest.mark.parametrize("seed,alpha", [(3, (1.0, 1.0)), (5, (1.0, 1.0)), (10, (1.3, 0.6)), (19, (0.8, 1.1))])
def test_route_choice_straight_through_closed_form_gpu(seed, alpha):
    """The GPU's beta, cost, theta and alpha gradients through a contested
    route choice equal the hand derivation from SI-B's estimators (the
    oracle's own pin), so the kernel's relaxed route weight is checked
    independently of the oracle."""
    from closed_forms import route_merge_closed_form
    w = W.route_merge_toy(seed=seed, alpha=alpha)
    s = _sim(w, record=True, max_steps=1)
    s.place([0, 1], [0, 1], [100.0, 100.0])
    s.step(1)
    adj = np.float32([0.7, -1.3])
    expect, win = route_merge_closed_form(w, seed, adj.astype(np.float64))
    st = s.state()
    assert st["link"][0][win] == 2 and st["link"][0][1 - win] == 1 - win
    g = s.backward(gx=adj[None], groups=("alpha", "beta", "cost", "theta"))
    for k in ("beta", "cost", "alpha", "theta"):
        np.testing.assert_allclose(g[k][0], expect[k], rtol=1e-5, atol=1e-6 * np.abs(expect[k]).max(), err_msg=k)


def test_rollout_autograd_function_matches_backward():
    """The torch.autograd wrapper returns exactly what a direct backward call
    on the same recorded rollout returns, for every group it was given."""
    import torch
    from paper_2603_25068_amd.sim import make_rollout_function
    w = W.random_small(6, nx=4, ny=4, n_agents=500, rates=True, steps=200)
    s = _sim(w, record=True)
    dev = torch.device("cuda", 0)
    leaf = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev, requires_grad=True)
    u, k, r = leaf(w.net.free_speed), leaf(w.net.jam_density), leaf(w.dem.rates)
    beta, alpha = leaf(w.net.beta), leaf(w.net.alpha)
    counts, ttt = make_rollout_function().apply(s, 200, u, k, r, None, beta, None, alpha)
    wq = torch.randn(counts.shape, generator=torch.Generator().manual_seed(3)).to(dev)
    ((counts * wq).sum() + 0.1 * ttt.sum()).backward()
    g = s.backward(gQ=wq.cpu().numpy(), gT=[0.1], groups=("free_speed", "jam_density", "rates", "beta", "alpha"))
    for name, x in (("free_speed", u), ("jam_density", k), ("rates", r), ("beta", beta), ("alpha", alpha)):
        assert np.array_equal(x.grad.cpu().numpy().ravel(), g[name][0]), name
    assert np.abs(g["alpha"]).max() > 0


ALL_GROUPS = ("free_speed", "jam_density", "rates", "cap_mult", "beta", "cost", "alpha", "theta")


def _link_invariants(w, s, scen=0):
    """Properties that hold at any size: conservation, FIFO order, every agent
    on the network within its link, and per link the agents on it equal its
    entry sequence minus its cumulative outflow."""
    st = s.state()
    c = st["counters"][scen]
    assert c["departed"] == c["on_net"] + c["exited"]
    assert c["released"] >= c["departed"] and c["order_viol"] == 0
    on = st["status"][scen] == oracle.ST_ON
    assert int(on.sum()) == c["on_net"]
    lk, ps = st["link"][scen][on], st["pos"][scen][on]
    assert np.all(ps >= 0.0) and np.all(ps <= w.net.length[lk])
    ls = s.link_state()
    per_link = np.bincount(lk, minlength=w.net.n_links)
    assert np.array_equal(ls["next_seq"][scen] - ls["E"][scen], per_link)
    assert np.all(ls["B"][scen] <= 1.0 + 1e-12 + w.net.capacity * w.net.lanes * w.cfg.dt)


def test_metro_full_size_in_bench_configuration():
    """The 1M-agent metro workload (12k nodes, 35k links) at full size, in
    the launch configuration the benchmark times (checkpoints every 60, the
    autotuner's schedule chosen on the end-of-rollout state).  The full
    1,800-step rollout is checked by invariants; the first 300 steps are
    bit-exact against the oracle, and their gradients in every group match
    the oracle's."""
    w = W.metro()
    T = w.cfg.steps
    s = _sim(w, record=True, max_steps=T)
    s.rollout()
    _link_invariants(w, s)
    s.autotune(probe_steps=30)
    T0 = 300
    s.reset()
    s.step(T0)
    o = Oracle(w, log=True)
    o.run(T0)
    _compare_state(o, s, ctx=f"metro after {T0} steps")
    rng = np.random.default_rng(5)
    cnt, _ = o.counts()
    gQ = rng.normal(size=cnt.shape).astype(np.float32)
    go = o.backward(gQ=gQ.astype(np.float64), gT=0.5)
    gg = s.backward(gQ=gQ[None], gT=[0.5], groups=ALL_GROUPS)
    for k in ALL_GROUPS:
        _grad_close(go[k], gg[k][0], f"metro {k}")


def test_grid_full_size_rollout_and_calibration_gradient():
    """The 32x32 grid (3,968 links, 50k pool, 768 rate parameters, 400
    detectors) over its full 1,800 steps: final state bit-exact against the
    oracle and the gradient of the count loss against a ground truth drawn
    with other rates, in every group."""
    w = W.grid_rates()
    truth = Oracle(w).run()
    c_true, _ = truth.counts()
    rng = np.random.default_rng(8)
    rates = (w.dem.rates * rng.uniform(0.8, 1.25, w.dem.rates.shape)).astype(np.float32)
    o = Oracle(w, log=True, params={"rates": rates}).run()
    s = _sim(w, record=True, params={"rates": rates}).rollout()
    _compare_state(o, s, ctx="grid full rollout")
    _link_invariants(w, s)
    cnt, _ = o.counts()
    gQ = (2.0 * (cnt - c_true) / cnt.size).astype(np.float32)
    go = o.backward(gQ=gQ.astype(np.float64))
    gg = s.backward(gQ=gQ[None], groups=ALL_GROUPS)
    assert np.abs(go["rates"]).max() > 0
    for k in ALL_GROUPS:
        _grad_close(go[k], gg[k][0], f"grid {k}")


def test_kernel_limits_hub_parity():
    """Largest cases of the kernels: a node with 64 merge candidates (8 in-links
    of 8 lanes), rings far above 128 slots holding more agents than one
    staging piece, four detectors on one link.  Forward bit-exact every 100
    steps, then the gradients of the whole rollout in every group."""
    w = W.hub()
    o = Oracle(w)
    s = _sim(w)
    for t in range(100, w.cfg.steps + 1, 100):
        o.run(100)
        s.step(100)
        _compare_state(o, s, ctx=f"hub t={t}")
    _link_invariants(w, s)
    o = Oracle(w, log=True).run()
    r = _sim(w, record=True).rollout()
    cnt, _ = o.counts()
    gQ = np.random.default_rng(2).normal(size=cnt.shape).astype(np.float32)
    go = o.backward(gQ=gQ.astype(np.float64), gT=0.1)
    gg = r.backward(gQ=gQ[None], gT=[0.1], groups=ALL_GROUPS)
    for k in ALL_GROUPS:
        _grad_close(go[k], gg[k][0], f"hub {k}")


def test_zero_agents():
    """An empty demand: steps, observables and every gradient are zero."""
    w = W.line(n_links=3, n_agents=0, steps=40)
    s = _sim(w, record=True).rollout()
    c = s.state()["counters"][0]
    assert all(v == 0 for v in c.values())
    cnt, ttt = s.observables()
    assert np.all(cnt == 0) and np.all(ttt == 0)
    g = s.backward(gT=[1.0], groups=("free_speed", "jam_density", "cap_mult", "beta", "alpha", "theta"))
    assert all(np.all(v == 0) for v in g.values())


def test_closed_links_hold_their_queues():
    """Capacity multiplier 0 on a set of links: no token ever accrues, so no
    transfer leaves them (agents whose destination is the link's head still
    exit, which takes no token); state and every gradient match the oracle."""
    w = W.random_small(12, nx=4, ny=4, n_agents=600, rates=True, steps=300)
    rng = np.random.default_rng(12)
    m = np.where(rng.uniform(size=w.net.n_links) < 0.25, 0.0, 1.0).astype(np.float32)
    o = Oracle(w, log=True, params={"cap_mult": m}).run()
    s = _sim(w, record=True, params={"cap_mult": m}).rollout()
    _compare_state(o, s, ctx="closed links")
    assert np.all(s.link_state()["B"][0][m == 0] == 0.0)
    cnt, _ = o.counts()
    gQ = rng.normal(size=cnt.shape).astype(np.float32)
    go = o.backward(gQ=gQ.astype(np.float64), gT=0.2)
    gg = s.backward(gQ=gQ[None], gT=[0.2], groups=ALL_GROUPS)
    for k in ALL_GROUPS:
        _grad_close(go[k], gg[k][0], f"closed {k}")


@pytest.mark.parametrize("S", [1, 2])
def test_forward_tape_gives_the_replayed_gradients(S):
    """The recording forward writes the tape of its last windows, so the
    backward sweeps them without a replay (the final one partial here).  A
    second backward of the same rollout replays every window; a backward that
    also asks for capacity multipliers replays every window with the extra
    tape.  All three give bitwise the same gradients, for one scenario and for
    two scenarios with their own seeds in one handle."""
    w = W.random_small(7, nx=4, ny=4, n_agents=500, rates=True, steps=280)
    seeds = [70 + k for k in range(S)]
    s = _sim(w, n_scenarios=S, seeds=seeds, record=True, ckpt_every=30, tape_windows=4).rollout()
    cnt, _ = s.observables()
    gQ = np.random.default_rng(7).normal(size=cnt.shape).astype(np.float32)
    gT = [0.3, -0.1][:S]
    groups = ("free_speed", "jam_density", "rates")
    g1 = s.backward(gQ=gQ, gT=gT, groups=groups)
    g2 = s.backward(gQ=gQ, gT=gT, groups=groups)
    g3 = s.backward(gQ=gQ, gT=gT, groups=groups + ("cap_mult",))
    for k in groups:
        assert np.array_equal(g1[k], g2[k]) and np.array_equal(g1[k], g3[k]), k
    for sc in range(S):
        o = Oracle(w, log=True, seed=seeds[sc]).run()
        _compare_state(o, s, scen=sc, ctx=f"scenario {sc}")
        go = o.backward(gQ=gQ[sc].astype(np.float64), gT=gT[sc])
        for k in groups:
            _grad_close(go[k], g1[k][sc], f"{k} scenario {sc}")


def test_tape_windows_do_not_change_gradients():
    """Ten windows with 4, 5 or 7 tape sets: the last windows come from the
    forward's tape and the rest are replayed from their checkpoints (three at
    a time beside the sweep, or one at a time in timing mode).  Every mix
    gives bitwise the same gradients, and they match the oracle's."""
    w = W.random_small(11, nx=4, ny=4, n_agents=500, rates=True, steps=280)
    groups = ("free_speed", "jam_density", "rates")
    rng = np.random.default_rng(11)
    ref = None
    for tw, timing in ((4, False), (5, False), (7, False), (5, True)):
        s = _sim(w, record=True, ckpt_every=28, tape_windows=tw)
        if timing:
            s.set_timing(True)
        s.rollout()
        cnt, _ = s.observables()
        if ref is None:
            gQ = rng.normal(size=cnt.shape).astype(np.float32)
        g = s.backward(gQ=gQ, gT=[0.4], groups=groups)
        if ref is None:
            ref = g
            o = Oracle(w, log=True).run()
            go = o.backward(gQ=gQ[0].astype(np.float64), gT=0.4)
            for k in groups:
                _grad_close(go[k], g[k][0], k)
        else:
            for k in groups:
                assert np.array_equal(ref[k], g[k]), (tw, timing, k)


def test_straight_through_gradients_do_not_depend_on_recording_layout():
    """The straight-through groups replay every window (their tape is written
    only by replays): checkpoint interval and tape windows change nothing,
    bit for bit, in any group."""
    w = W.random_small(5, nx=4, ny=4, n_agents=500, rates=True, steps=240)
    groups = ("free_speed", "jam_density", "rates", "beta", "cost", "alpha", "theta")
    rng = np.random.default_rng(5)
    ref, gQ = None, None
    for ckpt, tw in ((24, 4), (40, 6), (17, 0)):
        s = _sim(w, record=True, ckpt_every=ckpt, tape_windows=tw).rollout()
        if gQ is None:
            cnt, _ = s.observables()
            gQ = rng.normal(size=cnt.shape).astype(np.float32)
        g = s.backward(gQ=gQ, gT=[0.2], groups=groups)
        if ref is None:
            ref = g
            assert np.abs(g["alpha"]).max() > 0 and np.abs(g["theta"]).max() > 0
        else:
            for k in groups:
                assert np.array_equal(ref[k], g[k]), (ckpt, tw, k)


def test_set_params_after_t0_ends_the_recording():
    """Parameters changed in the middle of a recorded rollout: the backward
    refuses (the replay would follow other parameters than the forward)."""
    from paper_2603_25068_amd.sim import SimError
    w = W.random_small(3, nx=3, ny=3, n_agents=100, rates=True, steps=120)
    s = _sim(w, record=True)
    s.step(50)
    s.set_params("free_speed", w.net.free_speed)
    s.step(10)
    with pytest.raises(SimError):
        s.backward(gT=[1.0])
    s.reset()
    s.step(60)
    s.backward(gT=[1.0])


def test_autotune_restores_state_and_caches(tmp_path):
    """The autotuner probes from the live state and puts it back: a rollout
    tuned half-way equals an untuned one (values and gradients), and a second
    handle of the same shape takes the cached choice without probing."""
    w = W.random_small(12, nx=5, ny=5, n_agents=800, rates=True, steps=300, lanes_max=3)
    gQ = np.ones((1, w.net.n_detectors, 4), np.float32)
    ref = _sim(w, record=True, ckpt_every=50).rollout()
    cr, tr = ref.observables()
    gr = ref.backward(gQ=gQ, gT=[1.0], groups=("free_speed", "jam_density", "rates", "cap_mult"))
    s = _sim(w, record=True, ckpt_every=50)
    s.step(150)
    before, lb = s.state(), s.link_state()
    path = tmp_path / "schedules.txt"
    sched = s.autotune(probe_steps=12, cache_path=str(path))
    assert s.t == 150 and tuple(s.schedule()) == tuple(sched)
    after, la = s.state(), s.link_state()
    for k in ("status", "link", "pos", "seq", "counters"):
        assert np.array_equal(before[k], after[k]), k
    for k in lb:
        assert np.array_equal(lb[k], la[k]), k
    s.step(150)
    cs, ts = s.observables()
    assert np.array_equal(cr, cs) and np.array_equal(tr, ts)
    gs = s.backward(gQ=gQ, gT=[1.0], groups=("free_speed", "jam_density", "rates", "cap_mult"))
    for k in gr:
        assert np.array_equal(gr[k], gs[k]), k
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:4] == [str(x) for x in sched]
    s2 = _sim(w, record=True, ckpt_every=50)
    s2.step(20)
    assert tuple(s2.autotune(probe_steps=12, cache_path=str(path))) == tuple(sched)
    assert len(path.read_text().splitlines()) == 1


def test_full_state_round_trip():
    """A run saved half-way and restored into a fresh handle continues
    exactly as the original; a blob of another network is rejected."""
    from paper_2603_25068_amd.sim import SimError, SIM_EINVAL
    w = W.random_small(15, nx=4, ny=4, n_agents=600, rates=True, steps=300)
    a = _sim(w)
    a.step(120)
    blob = a.full_state()
    b = _sim(w, record=True)
    b.set_full_state(blob)
    assert b.t == 120
    a.step(180)
    b.step(180)
    sa, sb = a.state(), b.state()
    for k in ("status", "link", "pos", "seq", "counters"):
        assert np.array_equal(sa[k], sb[k]), k
    la, lb = a.link_state(), b.link_state()
    for k in la:
        assert np.array_equal(la[k], lb[k]), k
    ca, ta = a.observables()
    cb, tb = b.observables()
    assert np.array_equal(ca, cb) and np.array_equal(ta, tb)
    with pytest.raises(SimError) as e:
        b.backward(gT=[1.0])
    other = _sim(W.random_small(16, nx=4, ny=5, n_agents=600, rates=True, steps=300))
    with pytest.raises(SimError) as e:
        other.set_full_state(blob)
    assert e.value.code == SIM_EINVAL
    # placed agents travel with the blob
    t = W.tg_toy(2.0, 1.0)
    p = _sim(t, max_steps=10)
    p.place([0], [0], [3.0])
    q = _sim(t, max_steps=10)
    q.set_full_state(p.full_state())
    p.step(6)
    q.step(6)
    assert np.array_equal(p.state()["pos"], q.state()["pos"])



@pytest.mark.parametrize("mk", [W.small_grid_fixed,
                                lambda: W.random_small(11, nx=4, ny=4, n_agents=400, rates=True, steps=300)])
def test_reset_after_placement_restores_the_origin_queues(mk):
    """A reset keeps the origin queues it built while no agent was placed and
    rebuilds them once a placement (sim_place, or a restored state carrying
    placed agents) has taken agents out of them: every rollout after a reset
    equals the oracle's rollout without placement."""
    w = mk()
    T = min(w.cfg.steps, 300)
    o = Oracle(w)
    for _ in range(T):
        o.step()
    s = _sim(w)
    s.step(T)
    _compare_state(o, s, ctx=f"{w.name} first rollout")
    for case in ("reset", "place", "reset", "restore", "reset"):
        if case == "place":
            s.reset()
            s.place([0, 1], [0, 1], [0.0, 0.0])
            s.step(20)
        elif case == "restore":
            p = _sim(w)
            p.place([0, 1], [0, 1], [0.0, 0.0])
            s.set_full_state(p.full_state())
            s.step(20)
        s.reset()
        s.step(T)
        _compare_state(o, s, ctx=f"{w.name} rollout after {case}")

def test_fast_gumbel_error_bound_exhaustive():
    """The single-precision Gumbel transform behind the fast decisions,
    against -log(-log U) in double for every one of the 2^24 values of
    U = (k + 1/2) 2^-24 it can take: the error stays below 1e-5, so a
    difference of two scores is off by less than 2e-5, five times below the
    1e-4 margin a fast decision must win by."""
    w = W.line(n_links=1, n_agents=1, steps=1)
    s = _sim(w)
    k = np.arange(1 << 24, dtype=np.uint64)
    words = ((k << np.uint64(8)) | np.uint64(0x5A)).astype(np.uint32)
    g32 = s.gumbel_fast(words).astype(np.float64)
    u = (k.astype(np.float64) + 0.5) * 2.0 ** -24
    g64 = -np.log(-np.log(u))
    err = np.abs(g32 - g64)
    assert np.all(np.isfinite(g32))
    assert err.max() < 1e-5, f"max error {err.max():.3g} at k={int(err.argmax())}"
