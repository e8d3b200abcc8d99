"""Gradient-based calibration and control (Methods, "Optimization"; Results,
"Gradient-based model calibration" and "Gradient-guided traffic control")
through sim_optimize, against the oracle:

- calibration of the paper's four per-link groups (u, kappa, beta, alpha) on
  a Sioux-Falls-sized synthetic network, observations from the oracle's run
  at the ground truth: the loop's first gradient equals the oracle's gradient
  of the same count loss within 1e-3; its second loss equals the oracle's
  loss at the parameters one AdamW step (written out below from Loshchilov
  and Hutter) takes from there; with speed, jam density and route weight the
  loss falls and the handle keeps the best parameters;
- calibration of departure rates on the 32x32 lattice (768 parameters);
- control through the link costs: the squared gap between one link's
  cumulative count and half its uncontrolled value, gradient through the
  route-choice straight-through estimator equal to the oracle's.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2603_25068_amd import workloads as W

pytestmark = pytest.mark.gpu

GROUPS = ("free_speed", "jam_density", "beta", "alpha")


def _grad_close(go, gg, name, rtol=1e-3):
    go = np.asarray(go, np.float64).ravel()
    gg = np.asarray(gg, np.float64).ravel()
    scale = np.abs(go).max()
    assert scale > 0, name
    big = np.abs(go) > 1e-3 * scale
    rel = np.abs(gg[big] - go[big]) / np.abs(go[big])
    assert rel.max() <= rtol, f"{name}: component rel err {rel.max():.3g}"
    assert np.linalg.norm(gg - go) <= rtol * np.linalg.norm(go), f"{name}: norm rel err"


def adamw_first_step(p, g, lr, wd, b1=0.9, b2=0.999, eps=1e-8, lo=-np.inf, hi=np.inf, normalized=False):
    """One AdamW update from zero moments (Kingma and Ba's Adam with the decoupled weight decay of
    Loshchilov and Hutter), in the coordinates x = (p - lo) / (hi - lo) when normalized, in double,
    with the library's operation order; returns float32 parameters.  Bounds are float32 values, as
    the library receives them."""
    lo, hi = float(np.float32(lo)), float(np.float32(hi))
    p = np.asarray(p, np.float32).astype(np.float64)
    x0, sc = (lo, hi - lo) if normalized else (0.0, 1.0)
    gx = np.asarray(g, np.float32).astype(np.float64) * sc
    m = b1 * 0.0 + (1.0 - b1) * gx
    v = b2 * 0.0 + (1.0 - b2) * gx * gx
    mh = m / (1.0 - b1 ** 1.0)
    vh = v / (1.0 - b2 ** 1.0)
    x = (p - x0) / sc
    x = x - lr * (mh / (np.sqrt(vh) + eps) + wd * x)
    y = x0 + sc * x
    return np.minimum(np.maximum(y, lo), hi).astype(np.float32)


def _mse(q, y):
    return float(np.mean((np.asarray(q, np.float64) - np.asarray(y, np.float64)) ** 2))


def _sioux_calibration():
    """The synthetic network at its starting parameters (middle of the paper's ranges) and counts
    observed from the ground truth on the same network (same route-choice time table)."""
    w = W.calibration_start(W.sioux_like())
    obs, _ = Oracle(w, params=W.sioux_like().extra["truth"]).run().counts()
    return w, obs.astype(np.float32)


def test_calibration_first_step_of_the_papers_per_link_groups():
    """All four per-link groups of the paper (u, kappa, beta, alpha) with its hyperparameters
    (learning rate 0.1 on each group's position in its range, weight decay 1e-5): the loop's first
    loss and gradient equal the oracle's, and its second loss is the oracle's at one AdamW step
    from the start along that gradient."""
    from paper_2603_25068_amd.sim import Simulator
    w, obs = _sioux_calibration()
    start = w.extra["start"]
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    s.set_params("jam_density", start["jam_density"])
    bounds = dict(W.PAPER_RANGES)
    res = s.optimize(GROUPS, observed=obs, lr=0.1, weight_decay=1e-5, max_iters=2, patience=20,
                     bounds=bounds, normalized=True)
    assert res["iterations"] == 2
    params0 = {g: start[g] for g in GROUPS}
    o = Oracle(w, log=True, params=params0).run()
    q0, _ = o.counts()
    assert res["first_loss"] == pytest.approx(_mse(q0, obs), rel=1e-12)
    gQ = 2.0 * (q0.astype(np.float32).astype(np.float64) - obs.astype(np.float64)) / obs.size
    go = o.backward(gQ=gQ.astype(np.float32).astype(np.float64))
    for g in GROUPS:
        _grad_close(go[g], res["first_grad"][g], f"first gradient {g}")
    p1 = {g: adamw_first_step(start[g], res["first_grad"][g], 0.1, 1e-5, lo=bounds[g][0], hi=bounds[g][1],
                              normalized=True) for g in GROUPS}
    p1["jam_density"] = np.minimum(p1["jam_density"], w.net.jam_density)
    q1, _ = Oracle(w, params=p1).run().counts()
    assert res["history"][1] == pytest.approx(_mse(q1, obs), rel=1e-12)


def test_calibration_descends_and_keeps_the_best():
    """Speed, jam density and route weight on the synthetic network (learning rate 0.01 on the
    positions in the paper's ranges): the loss falls, the handle keeps the parameters of the lowest
    loss, and a rollout from them reproduces it."""
    from paper_2603_25068_amd.sim import Simulator
    w, obs = _sioux_calibration()
    groups = ("free_speed", "jam_density", "beta")
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    s.set_params("jam_density", w.extra["start"]["jam_density"])
    bounds = {g: W.PAPER_RANGES[g] for g in groups}
    res = s.optimize(groups, observed=obs, lr=0.01, weight_decay=1e-5, max_iters=40, patience=20,
                     bounds=bounds, normalized=True)
    hist = res["history"]
    print(f"calibration: {res['iterations']} iterations in {res['seconds']:.2f} s, loss {res['first_loss']:.4g} -> "
          f"{res['best_loss']:.4g} (iteration {res['best_iter']})", flush=True)
    assert res["best_loss"] < 0.95 * res["first_loss"]
    assert res["best_loss"] == np.min(hist) and hist[res["best_iter"]] == res["best_loss"]
    for g in groups:
        v = s.get_params(g)[0]
        assert np.all(v >= np.float32(bounds[g][0])) and np.all(v <= np.float32(bounds[g][1])), g
    s.rollout(w.cfg.steps)
    qb, _ = s.observables()
    assert _mse(qb[0], obs) == pytest.approx(res["best_loss"], rel=1e-12)


def test_calibration_of_departure_rates_on_the_lattice():
    """768 departure rates of the 32x32 lattice against counts from the ground-truth rates; the
    loop's first gradient equals the oracle's and the loss falls."""
    from paper_2603_25068_amd.sim import Simulator
    w = W.grid_rates()
    truth = Oracle(w, params={"rates": w.extra["theta_true"]}).run()
    obs, _ = truth.counts()
    obs = obs.astype(np.float32)
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    res = s.optimize(("rates",), observed=obs, lr=0.01, weight_decay=1e-5, max_iters=30, patience=20,
                     bounds={"rates": (0.0, 0.25)}, normalized=True)
    print(f"rates: {res['iterations']} iterations in {res['seconds']:.2f} s, loss {res['first_loss']:.4g} -> "
          f"{res['best_loss']:.4g}", flush=True)
    o = Oracle(w, log=True).run()
    q0, _ = o.counts()
    assert res["first_loss"] == pytest.approx(_mse(q0, obs), rel=1e-12)
    gQ = (2.0 * (q0.astype(np.float32).astype(np.float64) - obs) / obs.size).astype(np.float32)
    _grad_close(o.backward(gQ=gQ.astype(np.float64))["rates"], res["first_grad"]["rates"], "rates")
    assert res["best_loss"] < 0.95 * res["first_loss"]


def test_control_through_link_costs():
    """The paper's control problem on the synthetic network: halve the cumulative count of the
    busiest road link by changing link costs (the utility is beta / c).  The loop's first gradient in
    the costs equals the oracle's straight-through gradient of the same loss, and the loss falls."""
    from paper_2603_25068_amd.sim import Simulator
    w = W.sioux_like()
    base, _ = Oracle(w).run().counts()
    tot = base.sum(1)
    roads = int(w.net.n_links - w.net.n_nodes // 2)          # the virtual links come last
    det = int(np.argmax(tot[:roads]))
    target = 0.5 * float(tot[det])
    s = Simulator(w, record=True, max_steps=w.cfg.steps)
    res = s.optimize(("cost",), loss="cumulative", target_detector=det, target=target, lr=0.1,
                     weight_decay=1e-5, max_iters=40, patience=20, bounds={"cost": (0.05, 20.0)})
    print(f"control: {res['iterations']} iterations in {res['seconds']:.2f} s, count {tot[det]:.0f} -> target "
          f"{target:.0f}; loss {res['first_loss']:.4g} -> {res['best_loss']:.4g}", flush=True)
    assert res["first_loss"] == pytest.approx((tot[det] - target) ** 2, rel=1e-12)
    gQ = np.zeros(base.shape)
    gQ[det, :] = 2.0 * (float(np.float32(tot[det])) - target)
    o = Oracle(w, log=True).run()
    go = o.backward(gQ=gQ.astype(np.float32).astype(np.float64))["cost"]
    _grad_close(go, res["first_grad"]["cost"], "cost")
    assert res["best_loss"] < res["first_loss"]
    c = s.get_params("cost")[0]
    assert np.all(c >= np.float32(0.05)) and np.all(c <= np.float32(20.0))
