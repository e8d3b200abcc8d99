"""The paper's dense tensor formulation of one simulation step, written from
its equations (SI-A: masked free-flow and congested increments, sort-based
headway, trajectory-grafted cap; SI-B: potential next links L* = I.A, link
utility, softmax + Gumbel + straight-through link choice, connectivity /
arrival / vacancy masks, merge priority and merge choice, grafted transfer).

Values only (stop_gradient is the identity on values).  Used by the tests
as an independent pin of the oracle's sparse per-agent form in the special
case where the two coincide: one lane, outflow capacity not binding, no
destination term in the utility, agents placed on links (no departures).

Where the paper's two listings disagree with the text (unsorted headway
differences in Alg. S1, `beta*cost` in Alg. S2, `sum` for the connectivity
mask) the equations of the text are followed.
"""
import numpy as np


def car_following(X, u, kappa, length, dt, dn, M):
    """SI-A, applied to every link column of X [agents x links]."""
    N, L = X.shape
    Xn = X.copy()
    for j in range(L):
        x = X[:, j]
        valid = x >= -1e-2
        dx_free = valid * u[j] * dt
        xt = np.where(valid, x, -M)
        sigma = np.argsort(-xt, kind="stable")
        hp = np.full(N, float(M))
        for k in range(1, N):
            hp[sigma[k]] = xt[sigma[k - 1]] - xt[sigma[k]]
        h = np.where(valid, hp, M)
        dx_cong = valid * np.maximum(h - dn / kappa[j], 0.0)
        xp = x + np.minimum(dx_free, dx_cong)
        x_limit = length[j]            # L + x' - sg(x') has the value L
        Xn[:, j] = np.minimum(xp, x_limit)
    return Xn


def node_model(X, A, alpha, beta, cost, kappa, length, dn, M, G, Gm):
    """SI-B.  G [agents x links]: Gumbel draws for link choice; Gm
    [links x agents]: Gumbel draws for merge choice.  Returns the new X."""
    N, L = X.shape
    I_xpos = (X >= -1e-2).astype(float)
    Lstar = I_xpos @ A
    V = (beta / cost)[None, :] * Lstar - M * (Lstar < 1)
    # log-softmax then Gumbel; the argmax of the tempered softmax is tau-free
    logz = V - V.max(1, keepdims=True)
    logz = logz - np.log(np.exp(logz).sum(1, keepdims=True))
    lprime = np.zeros_like(V)
    lprime[np.arange(N), np.argmax(logz + G, axis=1)] = 1.0
    I_connected = Lstar.max(1, keepdims=True) > 0
    I_arrived = (X >= length[None, :] - 1e-2).sum(1, keepdims=True) > 0
    Xmin = np.where(X >= -1e-2, X, M).min(0)
    I_vacant = Xmin > dn / kappa
    l = I_connected * I_arrived * I_vacant[None, :] * lprime
    p = ((I_xpos @ alpha)[:, None] * l).T                    # [links x agents]
    Vp = p - M * (p == 0)
    logzp = Vp - Vp.max(1, keepdims=True)
    logzp = logzp - np.log(np.exp(logzp).sum(1, keepdims=True))
    aprime = np.zeros_like(Vp)
    aprime[np.arange(L), np.argmax(logzp + Gm, axis=1)] = 1.0
    a = l.max(0)[:, None] * aprime
    I_remove = I_xpos * a.T.sum(1, keepdims=True)
    I_add = a.T
    x = X.max(1, keepdims=True)
    return X - (M + x) * I_remove + (M + x - x) * I_add
