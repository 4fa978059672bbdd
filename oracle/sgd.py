"""Reference for the constrained-SGD edge scaling of Alg. 1 (Sec. 3.3.4)
(TEST INFRASTRUCTURE ONLY; FP64, dense linear algebra, small graphs).

Setting (Sec. 3.3): G is the original graph and P a spectrally similar
subgraph on the same nodes (same node ids, a subset of G's edges) whose edge
weights w_P are scaled up to shrink the largest generalised eigenvalue
lambda_n of L_G u = lambda L_P u, while the smallest, estimated as
lambda_1 = min_p d_G(p) / d_P(p) (Courant-Fischer estimate, Sec. 3.3.4), may
not fall below lambda_1^(0) * Delta_bar.

Iteration k (the algorithm's steps in order):
  * h_t: t generalised power iterations h <- L_P^+ L_G h from a centred
    random h_0 (Sec. 3.3.3), normalised so h^T L_P h = 1;
  * lambda_n^(k) = h^T L_G h (the generalised Rayleigh quotient of h);
  * sensitivities s_pq = -lambda_n (h_p - h_q)^2 (Eq. of the weight
    sensitivity);
  * momentum step dw <- alpha dw - eta s;
  * degree caps: every node p may gain at most
    cap_p = d_G(p) / (lambda_1 Delta) - d_P(p) before its ratio
    d_G/d_P drops to lambda_1 Delta.
    Reading taken (the paper updates edges one by one): all edges are
    updated at once, and where the edges at p ask for more than cap_p in
    total, each edge's share is cut in proportion:
    dw_e <- max(0, min(dw_e, cap_p dw_e / S_p, cap_q dw_e / S_q)),
    S_p = sum of the (positive) proposals at p;
  * w += dw, d_P recomputed; eta <- (lambda_n^(k) / lambda_n^(0)) eta_max;
    lambda_1 <- min_p d_G(p) / d_P(p);
  * stop when (lambda_n^(k-1) - lambda_n^(k)) / lambda_n^(k) < eps, or after
    K_max iterations.
Readings for values the paper leaves open: Delta = Delta_bar^(1/K_max)
(Alg. 1's initialisation), eta_max = eta_scale * mean(w_P) / max|s^(1)| with
eta_scale = 0.1, h_0 from the test-vector generator (one column, centred).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import oracle as O


@dataclasses.dataclass
class SgdParams:
    alpha: float = 0.9
    eta_scale: float = 0.1
    eps: float = 1e-3
    k_max: int = 20
    delta_bar: float = 0.5
    t: int = 2
    seed: int = 1


@dataclasses.dataclass
class SgdResult:
    w_P: np.ndarray
    lambda_n: list
    lambda_1: list
    iterations: int


def _lap(n, eu, ev, w):
    L = np.zeros((n, n))
    np.add.at(L, (eu, ev), -w)
    np.add.at(L, (ev, eu), -w)
    L[np.arange(n), np.arange(n)] = -L.sum(axis=1)
    return L


def pinv_apply(Lp, b):
    """L_P^+ b for b orthogonal to 1 (connected P): solve (L_P + J/n) y = b."""
    n = Lp.shape[0]
    return np.linalg.solve(Lp + np.ones((n, n)) / n, b)


def power_vector(Lg, Lp, h0, t):
    h = h0 - h0.mean()
    for _ in range(t):
        h = pinv_apply(Lp, Lg @ h)
        h -= h.mean()
    return h / np.sqrt(h @ Lp @ h)


def sgd_scale(n, g_eu, g_ev, g_w, p_eu, p_ev, w_P, params: SgdParams):
    """Alg. 1 in the parallel reading above.  G and P as undirected edge
    lists (p_* a subset of g_*); returns the scaled w_P."""
    w0 = np.array(w_P, dtype=np.float64, copy=True)
    w = w0.copy()
    Lg = _lap(n, g_eu, g_ev, np.asarray(g_w, np.float64))
    d_G = np.diag(Lg).copy()
    h0 = O.init_vectors(n, 1, params.seed, centre=True)[:, 0]
    delta = params.delta_bar ** (1.0 / params.k_max)      # cap factor (Alg. 1 set-up)
    dw = np.zeros_like(w)                                 # momentum starts at zero
    d_P = np.bincount(p_eu, w, n) + np.bincount(p_ev, w, n)
    lam1 = float(np.min(d_G / d_P))
    lam_n_hist, lam_1_hist = [], [lam1]
    eta_max = eta = None
    lam_n0 = None
    k = 0
    while k < params.k_max:
        Lp = _lap(n, p_eu, p_ev, w)
        h = power_vector(Lg, Lp, h0, params.t)            # t power iterations
        lam_n = float(h @ Lg @ h)                         # h^T L_P h = 1
        if lam_n0 is None:
            lam_n0 = lam_n
        elif (lam_n_hist[-1] - lam_n) / lam_n < params.eps:  # stopping test
            lam_n_hist.append(lam_n)
            break
        lam_n_hist.append(lam_n)
        s = -lam_n * (h[p_eu] - h[p_ev]) ** 2             # edge sensitivities
        if eta_max is None:
            eta_max = params.eta_scale * float(np.mean(w0)) / float(np.max(np.abs(s)))
            eta = eta_max
        dw = params.alpha * dw - eta * s                  # momentum step
        prop = np.maximum(dw, 0.0)                        # endpoint caps (parallel reading)
        S = np.bincount(p_eu, prop, n) + np.bincount(p_ev, prop, n)
        cap = d_G / (lam1 * delta) - d_P
        safe = np.where(S > 0, S, 1.0)
        fac = np.where(S > 0, cap / safe, np.inf)
        lim = np.where(prop > 0, np.minimum(fac[p_eu], fac[p_ev]) * np.where(prop > 0, prop, 1.0), 0.0)
        dw = np.maximum(0.0, np.minimum(dw, lim))
        w = w + dw                                        # weights, then degrees
        d_P = np.bincount(p_eu, w, n) + np.bincount(p_ev, w, n)
        eta = (lam_n / lam_n0) * eta_max                  # step-size schedule
        lam1 = float(np.min(d_G / d_P))                   # lambda_1 from the degrees
        lam_1_hist.append(lam1)
        k += 1
    return SgdResult(w, lam_n_hist, lam_1_hist, k)
