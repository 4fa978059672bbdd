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
  * stop when (lambda_n^(k-1) - lambda_n^(k)) / lambda_n^(k) < eps (not
    tested at k = 1), or after K_max iterations;
  * sensitivities s_pq = -lambda_n (h_p - h_q)^2 (Eq. of the weight
    sensitivity);
  * momentum step dw <- alpha dw - eta s, per edge;
  * the lambda_1 guard: node p may gain at most
    cap_p = d_G(p) / (lambda_1 Delta) - d_P(p) before its ratio
    d_G/d_P drops to lambda_1 Delta;
  * w += dw and d_P(p), d_P(q) += dw, edge by edge in edge order;
  * eta <- (lambda_n^(k) / lambda_n^(0)) eta_max;
    lambda_1 <- min_p d_G(p) / d_P(p) (Courant-Fischer estimate).

Two modes of the per-edge loop of Alg. 1:
  * "sequential" is the paper's loop as written: edges one at a time in
    edge order (upper-triangle CSR order: p < q, by p then q), each testing
    the guard with the running d_P, i.e. after the earlier edges' updates,
    and, where it trips, taking dw := min(dw_p, dw_q) with
    dw_p = d_G(p)/(lambda_1 Delta) - d_P(p).  Reading: dw is also kept
    >= 0 (the method only scales weights up), so dw := max(0, min(...)).
  * "parallel" is the order-free reading that a GPU runs: every proposal
    and every cap come from the iteration-start d_P, and where the
    proposals at p exceed cap_p in total each is cut in proportion:
    dw_e <- max(0, min(dw_e, cap_p dw_e / S_p, cap_q dw_e / S_q)),
    S_p = sum of the positive proposals at p.  The updates are then
    applied edge by edge exactly as in the sequential mode.
Where no guard trips, both modes take the same dw and apply it in the same
order, so they agree bit for bit.  Where guards trip, the sequential mode
gives an edge's whole remaining cap to the first edge that reaches it and
none to the later ones; the parallel mode shares it.

Readings for values the paper leaves open: Delta = Delta_bar^(1/K_max)
(Alg. 1's initialisation), eta_max = eta_scale * mean(w_P) / max|s^(1)| with
eta_scale = 0.1, h_0 from the test-vector generator (one column, centred)
unless given.  lambda_n^(1) is lambda_n^(0): the first iteration's h_t is
computed from the input weights, so eta^(2) = eta_max.
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


def sgd_scale(n, g_eu, g_ev, g_w, p_eu, p_ev, w_P, params: SgdParams,
              mode: str = "parallel", h0=None):
    """Alg. 1 in the given mode ("parallel" or "sequential", see above).  G
    and P as undirected edge lists (p_* a subset of g_*, in edge order);
    h0 (optional, length n) replaces the generated start vector.  Returns
    the scaled w_P with the lambda_n and lambda_1 histories."""
    if mode not in ("parallel", "sequential"):
        raise ValueError(mode)
    p_eu = np.asarray(p_eu, np.int64)
    p_ev = np.asarray(p_ev, np.int64)
    w0 = np.array(w_P, dtype=np.float64, copy=True)
    w = w0.copy()
    Lg = _lap(n, g_eu, g_ev, np.asarray(g_w, np.float64))
    d_G = np.diag(Lg).copy()
    if h0 is None:
        h0 = O.init_vectors(n, 1, params.seed, centre=True)[:, 0]
    h0 = np.asarray(h0, np.float64)
    delta = params.delta_bar ** (1.0 / params.k_max)      # Delta_lambda1 (Alg. 1 set-up)
    dw = np.zeros_like(w)                                 # momentum starts at zero
    d_P = np.zeros(n)
    for e in range(w.size):                               # diagonal of L_P, edge order
        d_P[p_eu[e]] += w[e]
        d_P[p_ev[e]] += w[e]
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
        thr = lam1 * delta                                # the lambda_1 guard
        if mode == "parallel":
            prop = np.maximum(dw, 0.0)
            S = np.bincount(p_eu, prop, n) + np.bincount(p_ev, prop, n)
            cap = d_G / thr - d_P
            safe = np.where(S > 0, S, 1.0)
            fac = np.where(S > 0, cap / safe, np.inf)
            lim = np.where(prop > 0,
                           np.minimum(fac[p_eu], fac[p_ev]) * np.where(prop > 0, prop, 1.0), 0.0)
            dw = np.maximum(0.0, np.minimum(dw, lim))
            for e in range(w.size):                       # apply in edge order
                p, q = p_eu[e], p_ev[e]
                w[e] += dw[e]
                d_P[p] += dw[e]
                d_P[q] += dw[e]
        else:
            for e in range(w.size):                       # the paper's edge loop
                p, q = p_eu[e], p_ev[e]
                phi_p = d_G[p] / (d_P[p] + dw[e])
                phi_q = d_G[q] / (d_P[q] + dw[e])
                if min(phi_p, phi_q) <= thr:
                    dwp = d_G[p] / thr - d_P[p]
                    dwq = d_G[q] / thr - d_P[q]
                    dw[e] = max(0.0, min(dwp, dwq))
                w[e] += dw[e]
                d_P[p] += dw[e]
                d_P[q] += dw[e]
        eta = (lam_n / lam_n0) * eta_max                  # step-size schedule
        lam1 = float(np.min(d_G / d_P))                   # lambda_1 from the degrees
        lam_1_hist.append(lam1)
        k += 1
    return SgdResult(w, lam_n_hist, lam_1_hist, k)
