"""Platoon size dn > 1 (Methods, Newell's simplified car-following model: an
agent is a platoon of dn vehicles, the jam spacing is dn/kappa and the step
is dt = tau * dn; SI-E varies dn over 1, 2 and 4).

CPU: the oracle against closed forms at dn = 2 and 4 (jam spacing, lone
free-flow travel time, throughput of a link whose bucket counts agents at
capacity * lanes / dn per second) and its adjoint against central
differences of the frozen surrogate.  GPU: the HIP path against the oracle
at dn = 2 and 4, state bit-exact and gradients within 1e-3."""
import math

import numpy as np
import pytest

import oracle
from oracle import Oracle, ST_EXITED, ST_ON
from paper_2603_25068_amd import workloads as W


def _line_dn(dn, **kw):
    w = W.line(**kw)
    w.cfg.platoon = dn
    w.cfg.dt = float(dn)
    return w


@pytest.mark.parametrize("dn", [2, 4])
def test_platoon_jam_spacing(dn):
    """Agents behind a head that can never leave stand at L - k * dn/kappa."""
    w = _line_dn(dn, n_links=2, length=200.0, capacity=0.0, n_agents=12, steps=100)
    o = Oracle(w, variant="f64")
    o.run(100)
    st = o.state()
    on0 = np.sort(st["pos"][(st["status"] == ST_ON) & (st["link"] == 0)])[::-1]
    s = dn / float(np.float32(0.2))
    assert len(on0) == min(12, int(200.0 // s) + 1)
    assert np.allclose(on0, 200.0 - s * np.arange(len(on0)), atol=1e-9)


@pytest.mark.parametrize("dn", [2, 4])
@pytest.mark.parametrize("length,speed", [(200.0, 13.9), (333.0, 16.7)])
def test_platoon_lone_vehicle_travel_time(dn, length, speed):
    """With dt = dn a lone agent needs ceil((L - 0.01)/(u dt)) steps per link."""
    n = 3
    w = _line_dn(dn, n_links=n, length=length, speed=speed, steps=200)
    o = Oracle(w, variant="f64")
    k = math.ceil((float(np.float32(length)) - 0.01) / (float(np.float32(speed)) * dn))
    exit_step = None
    for t in range(200):
        o.step()
        if o.state()["status"][0] == ST_EXITED:
            exit_step = t
            break
    assert exit_step == n * k
    _, ttt = o.counts()
    assert ttt == n * k * float(dn)


@pytest.mark.parametrize("dn", [1, 2, 4])
def test_platoon_throughput_counts_agents(dn):
    """Saturated upstream, free downstream: the bucket accrues capacity *
    lanes * dt / dn agents per step, so at capacity 0.25 veh/s and dt = dn the
    cumulative outflow after the first departure at t0 is 1 + floor((k+1)/4),
    whatever dn."""
    q = 0.25   # veh/s: with dt = dn the bucket gains 0.25 * dn / dn = 0.25 agents per step
    w = _line_dn(dn, n_links=2, length=200.0, capacity=q, n_agents=60, steps=200)
    o = Oracle(w)
    E = []
    for t in range(200):
        o.step()
        E.append(int(o.link_state()["E"][0]))
    E = np.array(E)
    t0 = int(np.argmax(E > 0))
    k = np.arange(0, 200 - t0)
    expect = 1 + np.floor((k + 1) / 4)
    until = int(np.searchsorted(E, 60)) - t0
    assert until > 40
    assert np.array_equal(E[t0:t0 + until], expect[:until])


@pytest.mark.parametrize("dn", [2, 4])
def test_platoon_adjoint_matches_frozen_surrogate_fd(dn):
    """The adjoint at dn > 1 (jam term d(dn/kappa)/dkappa = -dn/kappa^2, token
    grafts at capacity/dn) equals central differences of the frozen surrogate."""
    w = W.with_platoon(W.random_small(6, nx=3, ny=3, n_agents=200, rates=True, steps=240), dn)
    w.net.capacity = np.full(w.net.n_links, 0.15, np.float32)
    rng = np.random.default_rng(dn)
    m = rng.uniform(0.6, 1.0, w.net.n_links).astype(np.float32)
    o = Oracle(w, variant="f64", log=True, params={"cap_mult": m})
    o.run()
    net = w.net
    base = {"u": net.free_speed.astype(np.float64), "kappa": net.jam_density.astype(np.float64),
            "rates": w.dem.rates.astype(np.float64), "cap_mult": m.astype(np.float64)}
    c0, t0, x0 = o.frozen(**base, record_base=True)
    cnt, ttt = o.counts()
    np.testing.assert_allclose(c0, cnt, atol=1e-9)
    gQ = rng.normal(size=c0.shape)
    gT = 0.3
    g = o.backward(gQ=gQ, gT=gT)
    for which, key in (("u", "free_speed"), ("kappa", "jam_density"), ("rates", "rates"),
                       ("cap_mult", "cap_mult")):
        d = rng.normal(size=base[which].shape)
        h = 1e-7 if which == "rates" else 1e-6 * max(1.0, float(np.abs(base[which]).max()))
        kw_p = {k: v.copy() for k, v in base.items()}
        kw_m = {k: v.copy() for k, v in base.items()}
        kw_p[which] = kw_p[which] + h * d
        kw_m[which] = kw_m[which] - h * d
        cp, tp, _ = o.frozen(**kw_p)
        cm, tm, _ = o.frozen(**kw_m)
        fd = (gQ * (cp - cm)).sum() / (2 * h) + gT * (tp - tm) / (2 * h)
        ad = (g[key] * d).sum()
        assert ad == pytest.approx(fd, rel=1e-6, abs=1e-8), which


@pytest.mark.gpu
@pytest.mark.parametrize("dn", [2, 4])
def test_platoon_parity_gpu(dn):
    """HIP path at dn = 2 and 4 against the oracle: every agent's status, link,
    entry sequence and position, the buckets and counts bit-exact; u, kappa,
    rates and capacity-multiplier gradients within 1e-3."""
    from paper_2603_25068_amd.sim import Simulator
    w = W.with_platoon(W.random_small(31, nx=5, ny=5, n_agents=900, rates=True, steps=400, lanes_max=3), dn)
    rng = np.random.default_rng(dn)
    m = rng.uniform(0.5, 1.0, w.net.n_links).astype(np.float32)
    o = Oracle(w, log=True, params={"cap_mult": m}).run()
    s = Simulator(w, record=True, params={"cap_mult": m}).rollout()
    so, sg = o.state(), s.state()
    assert np.array_equal(so["status"], sg["status"][0])
    on = so["status"] == ST_ON
    assert on.sum() > 20
    for k in ("link", "seq", "pos"):
        assert np.array_equal(so[k][on].astype(sg[k].dtype), sg[k][0][on]), k
    lo, lg = o.link_state(), s.link_state()
    assert np.array_equal(lo["B"], lg["B"][0]) and np.array_equal(lo["E"], lg["E"][0])
    co, to = o.counts()
    cg, tg = s.observables()
    assert np.array_equal(co.astype(np.float32), cg[0]) and to == tg[0]
    gQ = rng.normal(size=co.shape).astype(np.float32)
    go = o.backward(gQ=gQ.astype(np.float64), gT=0.5)
    gg = s.backward(gQ=gQ[None], gT=[0.5], groups=("free_speed", "jam_density", "rates", "cap_mult"))
    for k in ("free_speed", "jam_density", "rates", "cap_mult"):
        a, b = np.asarray(go[k], np.float64).ravel(), np.asarray(gg[k][0], np.float64).ravel()
        scale = np.abs(a).max()
        assert scale > 0, k
        big = np.abs(a) > 1e-3 * scale
        assert (np.abs(b[big] - a[big]) / np.abs(a[big])).max() <= 1e-3, k
        assert np.linalg.norm(b - a) <= 1e-3 * np.linalg.norm(a), k
