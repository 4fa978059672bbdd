"""Reference for Phase B, spectral graph sparsification (Sec. 3.3.2-3.3.3),
and for the flow of Alg. 2, which joins the two phases.

TEST INFRASTRUCTURE ONLY: plain FP64 NumPy/SciPy with dense solves, for
small graphs; the GPU library never imports it.

Phase B, in the paper's order:
  1. a spanning tree P of G (Sec. 3.3.2);
  2. h_t = (L_P^+ L_G)^t h_0 by t = 2 generalised power iterations from a
     random h_0 orthogonal to the all-one vector (Eq. formula_pwr_iter5),
     normalised so that h_t^T L_P h_t = 1; its quotient
     lambda_n = h_t^T L_G h_t estimates the largest generalised eigenvalue;
  3. the approximate spectral criticality of every edge of G outside P,
     c_pq = w_G(p, q) (h_p - h_q)^2 (Eq. formula_pwr_iter5new);
  4. incremental densification: the most critical of them join P, and the
     estimate is repeated until it is small enough (Sec. 3.3.3).
Alg. 2 then runs Phase A and Phase B in the order the density
gamma = |E_G| / |V| picks: Phase A first when gamma < gamma_max, else
Phase B (with the edge scaling of Alg. 1) first.

Readings (the paper does not fix these):
  * The tree is the maximum-weight spanning forest (Kruskal), edges by
    weight descending, ties by the smaller, then the larger endpoint: the
    paper cites low-stretch trees but gives no construction; heavy edges
    carry the most conductance.
  * h_0 is one column of the test-vector generator (seed given), the same
    start in every round.
  * Each round adds ceil(add_frac * n) edges (add_frac = 0.02), the most
    critical first, ties by edge order; the rounds stop after `rounds`
    (5) or once lambda_n <= lambda_target (0: never).  The k-dimensional
    embedding that filters similar edges is not used (k = 1).
  * |E_G| counts undirected edges; gamma_max = 40 (the paper's threshold).
  * In the sparse branch Phase B runs on R with R's edges; Alg. 1 scales
    the weights of the subgraph it selects (parallel mode).  In the dense
    branch Phase A runs on P with its scaled weights rounded to float32
    (the library's graph weights).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import oracle as O
from . import sgd as SG


# ---------------------------------------------------------------- the tree

def max_spanning_forest(n, eu, ev, w):
    """Boolean mask over the edges: Kruskal on the order (w desc, min id,
    max id) with union-find."""
    eu = np.asarray(eu, np.int64)
    ev = np.asarray(ev, np.int64)
    w = np.asarray(w, np.float64)
    order = np.lexsort((np.maximum(eu, ev), np.minimum(eu, ev), -w))
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    keep = np.zeros(eu.size, bool)
    for e in order:
        a, b = find(int(eu[e])), find(int(ev[e]))
        if a != b:
            parent[max(a, b)] = min(a, b)
            keep[e] = True
    return keep


# --------------------------------------------------------- criticality

def power_vector(n, g_eu, g_ev, g_w, in_P, h0, t):
    """h_t (normalised, h^T L_P h = 1) and lambda_n = h^T L_G h."""
    Lg = SG._lap(n, g_eu, g_ev, np.asarray(g_w, np.float64))
    Lp = SG._lap(n, np.asarray(g_eu)[in_P], np.asarray(g_ev)[in_P],
                 np.asarray(g_w, np.float64)[in_P])
    h = SG.power_vector(Lg, Lp, np.asarray(h0, np.float64), t)
    return h, float(h @ Lg @ h)


def criticality(g_eu, g_ev, g_w, in_P, h):
    """c_pq = w_G(p, q) (h_p - h_q)^2 for the edges outside P, 0 inside."""
    c = np.asarray(g_w, np.float64) * (h[np.asarray(g_eu)] - h[np.asarray(g_ev)]) ** 2
    return np.where(in_P, 0.0, c)


@dataclasses.dataclass
class SparsifyParams:
    t: int = 2
    rounds: int = 5
    add_frac: float = 0.02
    lambda_target: float = 0.0
    seed: int = 1


@dataclasses.dataclass
class SparsifyResult:
    in_P: np.ndarray          # bool [E]
    lambda_n: list            # estimate after the tree, then after each round
    rounds: int


def sparsify(n, g_eu, g_ev, g_w, prm: SparsifyParams) -> SparsifyResult:
    """Phase B's sparsifier: tree, then rounds of criticality-ranked edges."""
    in_P = max_spanning_forest(n, g_eu, g_ev, g_w)
    h0 = O.init_vectors(n, 1, prm.seed, centre=True)[:, 0]
    per = int(math.ceil(prm.add_frac * n))
    lam_hist = []
    rounds = 0
    while True:
        h, lam = power_vector(n, g_eu, g_ev, g_w, in_P, h0, prm.t)
        lam_hist.append(lam)
        if rounds >= prm.rounds or lam <= prm.lambda_target or in_P.all():
            break
        c = criticality(g_eu, g_ev, g_w, in_P, h)
        cand = np.flatnonzero(~in_P)
        order = cand[np.lexsort((cand, -c[cand]))]    # c desc, then edge order
        in_P = in_P.copy()
        in_P[order[:per]] = True
        rounds += 1
    return SparsifyResult(in_P, lam_hist, rounds)


# ----------------------------------------------------------------- Alg. 2

def csr_of_edges(n, eu, ev, w):
    """Symmetric CSR (columns ascending) of an undirected edge list."""
    eu = np.asarray(eu, np.int64)
    ev = np.asarray(ev, np.int64)
    r = np.concatenate([eu, ev])
    c = np.concatenate([ev, eu])
    ww = np.concatenate([w, w])
    o = np.lexsort((c, r))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp).astype(np.int32), c[o].astype(np.int32), np.asarray(ww)[o]


@dataclasses.dataclass
class FlowResult:
    dense: bool               # Phase B ran first
    agg: np.ndarray           # node -> node of S
    n_S: int
    row_ptr: np.ndarray       # S as CSR
    col: np.ndarray
    w: np.ndarray             # float64
    sparsify: SparsifyResult
    sgd: SG.SgdResult


def spectral_reduce(n, row_ptr, col, w, K, sweeps, ratio, vec_seed, colour_seed,
                    gamma_max=40.0, sp=SparsifyParams(), sgd=SG.SgdParams(),
                    largest_degree_first=False):
    """Alg. 2: density test, then Phase A and Phase B (sparsification and
    Alg. 1 edge scaling) in the order it selects."""
    eoe, eu, ev = O.edge_index(n, row_ptr, col)
    wE = np.zeros(eu.size)
    wE[eoe] = np.asarray(w, np.float64)
    gamma = eu.size / max(n, 1)
    if gamma < gamma_max:
        r = O.reduce(n, row_ptr, col, w, K, sweeps, ratio, vec_seed, colour_seed,
                     fp32_coarse=True, largest_degree_first=largest_degree_first)
        eo2, ru, rv = O.edge_index(r.n_coarse, r.row_ptr, r.col)
        rw = np.zeros(ru.size)
        rw[eo2] = r.w
        spr = sparsify(r.n_coarse, ru, rv, rw, sp)
        keep = spr.in_P
        sg = SG.sgd_scale(r.n_coarse, ru, rv, rw, ru[keep], rv[keep], rw[keep], sgd)
        rp, cl, ww = csr_of_edges(r.n_coarse, ru[keep], rv[keep], sg.w_P)
        return FlowResult(False, r.agg, r.n_coarse, rp, cl, ww, spr, sg)
    spr = sparsify(n, eu, ev, wE, sp)
    keep = spr.in_P
    sg = SG.sgd_scale(n, eu, ev, wE, eu[keep], ev[keep], wE[keep], sgd)
    w32 = sg.w_P.astype(np.float32).astype(np.float64)
    prp, pcl, pw = csr_of_edges(n, eu[keep], ev[keep], w32)
    r = O.reduce(n, prp, pcl, pw, K, sweeps, ratio, vec_seed, colour_seed, fp32_coarse=True,
                 largest_degree_first=largest_degree_first)
    return FlowResult(True, r.agg, r.n_coarse, r.row_ptr, r.col, r.w, spr, sg)
