"""One simulation step in a dense agent-by-link form, written from the
equations of the paper's supplementary sections SI-A and SI-B (not from its
listings), as an independent pin of the oracle's sparse per-agent form.

State: P [agents x links], the agent's position on the link it occupies and
NaN on every other link (the paper pads with -M; NaN keeps "absent" apart
from any position).  Values only: stop_gradient is the identity on values.

SI-A, Newell's car-following with sort-based headways: on each link, agents
ordered by position (front first); each agent's headway is the distance to
the one in front (none for the front agent).  The position increment is
min(u dt, max(headway - dn/kappa, 0)), and the trajectory-grafted cap keeps
the new position at most the link length (its value is min(x', L)).

SI-B, node model: an agent within 1e-2 m of the end of its link has
arrived; its candidate next links are the out-links of the link's head node,
scored V = beta/c (the text's utility; the destination term is left
out here); the sample is the argmax of log softmax(V) + Gumbel noise.  A
target link takes an entrant only if every agent on it is further than
dn/kappa from its start.  Among the arrived agents choosing one vacant
target, the merge picks the argmax of log softmax(alpha_from) + Gumbel
noise over those agents.  The winner's position becomes 0 on the target
(the transfer equation's value: x - (M + x) on the old link, -M + M + x - x
on the new one), everyone else keeps its place.

The sparse oracle must agree with this exactly when the two coincide: one
lane per link, outflow capacity not binding, no destination term, agents
placed on links at t = 0 (no departures).
"""
import numpy as np


def _log_softmax(z):
    z = z - z.max()
    return z - np.log(np.exp(z).sum())


def newell_dense(P, u, kappa, length, dt, dn):
    """SI-A on every link column: returns the capped positions x_hat."""
    out = np.full_like(P, np.nan)
    for j in range(P.shape[1]):
        who = np.flatnonzero(~np.isnan(P[:, j]))
        if who.size == 0:
            continue
        x = P[who, j]
        front_first = who[np.argsort(-x, kind="stable")]
        ahead = None
        for i in front_first:
            xi = P[i, j]
            step = u[j] * dt
            if ahead is not None:
                gap = P[ahead, j] - xi
                step = min(step, max(gap - dn / kappa[j], 0.0))
            out[i, j] = min(xi + step, length[j])
            ahead = i
    return out


def node_dense(P, tail, head, alpha, beta, cost, kappa, length, dn, noise_route, noise_merge):
    """SI-B.  noise_route [agents x links]: the route-choice Gumbel draw of
    agent i for link m; noise_merge [agents]: agent i's merge draw.  Returns
    the positions after the transfer."""
    n_ag, n_links = P.shape
    link_of = np.array([np.flatnonzero(~np.isnan(P[i]))[0] if np.any(~np.isnan(P[i])) else -1
                        for i in range(n_ag)])
    at_end = np.array([j >= 0 and P[i, j] >= length[j] - 1e-2 for i, j in enumerate(link_of)])
    # each arrived agent's sampled next link
    want = np.full(n_ag, -1)
    for i in range(n_ag):
        j = link_of[i]
        if j < 0 or not at_end[i]:
            continue
        cands = np.flatnonzero(tail == head[j])
        if cands.size == 0:
            continue
        score = _log_softmax(beta[cands] / cost[cands]) + noise_route[i, cands]
        want[i] = cands[int(np.argmax(score))]
    Q = P.copy()
    for m in range(n_links):
        occupants = P[:, m][~np.isnan(P[:, m])]
        if occupants.size and occupants.min() <= dn / kappa[m]:
            continue   # no vacancy at the start of m
        comers = np.flatnonzero(want == m)
        if comers.size == 0:
            continue
        score = _log_softmax(alpha[link_of[comers]]) + noise_merge[comers]
        w = comers[int(np.argmax(score))]
        Q[w, link_of[w]] = np.nan
        Q[w, m] = 0.0
    return Q
