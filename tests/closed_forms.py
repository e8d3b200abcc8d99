"""Closed forms derived by hand from the paper's equations, shared by the
oracle pins and the GPU tests (they use the oracle's Philox-Gumbel only for
the noise values, which are pinned by the generator's known answers)."""
import numpy as np

import oracle


def route_merge_closed_form(w, seed, adj):
    """dL/d(beta, cost, alpha, theta) of the route_merge_toy's first step,
    derived by hand from SI-B's estimators for the loss L = adj . x(1).

    Agent 0 chooses at node 2 between links 2 and 3 with utilities
    V_m = beta_m/c_m - theta r_m (r_m: free-flow time of m plus the time from
    its head to node 5) and noise g_m; its hard choice is link 2 (checked).
    Its relaxed weight of link 2 is l = onehot + pi - sg(pi) at
    pi = softmax((V + g)/tau), so dl/dV_m = pi_2 (delta_m2 - pi_m)/tau.
    Agent 1 has one admissible link (pi = 1).  The merge onto link 2 scores
    y_i = alpha_from(i) l_i + g'_i; with p' = softmax(y/tau) over the two
    heads, dL/dy_i = p'_0 p'_1 (G_i - G_other)/tau, G = M adj for the winner
    (it moved to position 0 of link 2) and -(M + L) adj for the loser (it
    stayed at the end L of its link).  Then dL/dalpha_from(i) = dL/dy_i,
    Gamma = alpha_0 dL/dy_0, and dL/dV_m = Gamma dl/dV_m."""
    f = lambda v: float(np.float32(v))
    net, tau, bigm, theta = w.net, w.cfg.gumbel_tau, w.cfg.big_m, w.cfg.dest_logit_coef
    r = {2: f(net.length[2]) / f(net.free_speed[2]) + f(net.length[4]) / f(net.free_speed[4]),
         3: f(net.length[3]) / f(net.free_speed[3]) + f(net.length[5]) / f(net.free_speed[5])}
    V = {m: f(net.beta[m]) / f(net.cost[m]) - theta * r[m] for m in (2, 3)}
    g = {m: oracle.gumbel(seed, 0, 0, 0, k) for k, m in enumerate((2, 3))}
    assert V[2] + g[2] > V[3] + g[3], "agent 0 must choose link 2"
    z = np.array([(V[m] + g[m]) / tau for m in (2, 3)])
    pi = np.exp(z - z.max())
    pi /= pi.sum()
    dl_dV = {m: pi[0] * ((m == 2) - pi[k]) / tau for k, m in enumerate((2, 3))}
    al = [f(net.alpha[0]), f(net.alpha[1])]
    y = np.array([al[i] + oracle.gumbel(seed, i, 0, 1, 0) for i in (0, 1)])
    win = int(np.argmax(y))
    length = f(net.length[0])
    G = [bigm * adj[i] if i == win else -(bigm + length) * adj[i] for i in (0, 1)]
    q = np.exp(y / tau - (y / tau).max())
    q /= q.sum()
    dy0 = q[0] * q[1] * (G[0] - G[1]) / tau
    gam = al[0] * dy0
    L = net.n_links
    out = {k: np.zeros(L) for k in ("beta", "cost", "alpha")}
    out["alpha"][0], out["alpha"][1] = dy0, -dy0
    th = 0.0
    for m in (2, 3):
        dV = gam * dl_dV[m]
        out["beta"][m] = dV / f(net.cost[m])
        out["cost"][m] = -f(net.beta[m]) / f(net.cost[m]) ** 2 * dV
        th += -r[m] * dV
    out["theta"] = np.array([th])
    return out, win
