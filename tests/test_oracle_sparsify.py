"""Pins of the oracle's Phase B (Sec. 3.3.2-3.3.3) and Alg. 2 flow: the
spanning forest against a library minimum spanning tree, the tie order by
hand, the cycle property; the criticality of the 5-cycle by hand and the
identity sum(c) = lambda_n - 1; densification lowering the dense largest
generalised eigenvalue; Alg. 2's branch choice."""
import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

from oracle import oracle as O
from oracle import sgd as SG
from oracle import sparsify as PB
from workloads import graphs as W


def _edges(g):
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    w = np.zeros(eu.size)
    w[eoe] = g.w
    return eu, ev, w


def test_forest_equals_library_tree_on_distinct_weights():
    rng = np.random.default_rng(1)
    for seed in range(3):
        g = W.random_weighted(120, 0.08, seed=seed)
        eu, ev, w = _edges(g)
        w = w + rng.uniform(0, 1e-3, w.size)        # distinct
        keep = PB.max_spanning_forest(g.n, eu, ev, w)
        M = sp.coo_matrix((-w, (eu, ev)), shape=(g.n, g.n))
        T = cg.minimum_spanning_tree(M).tocoo()
        lib = set(zip(np.minimum(T.row, T.col), np.maximum(T.row, T.col)))
        ours = set(zip(eu[keep].tolist(), ev[keep].tolist()))
        assert ours == lib and keep.sum() == g.n - 1


def test_forest_tie_order_by_hand():
    """The unit square 0-1, 1-2, 2-3, 0-3: ties go to the smaller endpoints,
    so (0,1), (0,3), (1,2) are kept and (2,3) closes the cycle."""
    eu = np.array([0, 0, 1, 2])
    ev = np.array([1, 3, 2, 3])
    keep = PB.max_spanning_forest(4, eu, ev, np.ones(4))
    assert keep.tolist() == [True, True, True, False]


def test_forest_cycle_property_and_components():
    g = W.disjoint_union(W.random_weighted(60, 0.1, seed=4), W.random_weighted(40, 0.15, seed=5))
    eu, ev, w = _edges(g)
    keep = PB.max_spanning_forest(g.n, eu, ev, w)
    ncomp = cg.connected_components(sp.csr_matrix((np.ones(eu.size), (eu, ev)),
                                                  shape=(g.n, g.n)), directed=False)[0]
    assert keep.sum() == g.n - ncomp
    T = sp.csr_matrix((w[keep], (eu[keep], ev[keep])), shape=(g.n, g.n))
    T = T + T.T
    for e in np.flatnonzero(~keep)[:40]:
        # the tree path between the endpoints has no lighter edge
        _, pred = cg.breadth_first_order(T, int(eu[e]), directed=False)
        v = int(ev[e])
        path_min = np.inf
        while pred[v] >= 0:
            path_min = min(path_min, T[v, pred[v]])
            v = pred[v]
        assert w[e] <= path_min


def test_criticality_by_hand_on_the_5_cycle():
    """P = the path of the 5-cycle, h_0 = (2, 1, 0, -1, -2): h_t = h_0 / 2,
    lambda_n = 5, and the one edge outside P, (0, 4), has
    c = 1 * (1 - (-1))^2 = 4 = lambda_n - 1."""
    eu = np.array([0, 0, 1, 2, 3])
    ev = np.array([1, 4, 2, 3, 4])
    w = np.ones(5)
    in_P = np.array([True, False, True, True, True])
    h, lam = PB.power_vector(5, eu, ev, w, in_P, np.array([2.0, 1, 0, -1, -2]), 2)
    assert abs(lam - 5.0) < 1e-12
    c = PB.criticality(eu, ev, w, in_P, h)
    assert np.allclose(c, [0, 4, 0, 0, 0], atol=1e-12)


def test_criticality_sums_to_lambda_minus_one():
    """sum over the edges outside P of w (e_pq^T h)^2 = h^T (L_G - L_P) h
    = lambda_n - 1 for h^T L_P h = 1 (Eq. formula_pwr_iter5new)."""
    g = W.random_weighted(90, 0.12, seed=7)
    eu, ev, w = _edges(g)
    in_P = PB.max_spanning_forest(g.n, eu, ev, w)
    h, lam = PB.power_vector(g.n, eu, ev, w, in_P, O.init_vectors(g.n, 1, 3)[:, 0], 2)
    c = PB.criticality(eu, ev, w, in_P, h)
    assert abs(c.sum() - (lam - 1.0)) <= 1e-10 * lam


def test_densification_lowers_the_largest_generalised_eigenvalue():
    """Each round adds ceil(add_frac n) edges of G to P with G's weights, so
    L_P grows in the Loewner order and the dense largest generalised
    eigenvalue of (L_G, L_P) can only fall, round after round; the edges
    added are the most critical ones outside P."""
    g = W.random_weighted(80, 0.15, seed=9)
    eu, ev, w = _edges(g)
    Lg = SG._lap(g.n, eu, ev, w)
    J = np.ones((g.n, g.n)) / g.n

    def lmax(m):
        return sl.eigh(Lg + J, SG._lap(g.n, eu[m], ev[m], w[m]) + J, eigvals_only=True)[-1]

    per = int(np.ceil(0.05 * g.n))
    prev = lmax(PB.max_spanning_forest(g.n, eu, ev, w))
    last = None
    for R in range(1, 5):
        r = PB.sparsify(g.n, eu, ev, w, PB.SparsifyParams(rounds=R, add_frac=0.05))
        assert r.rounds == R and r.in_P.sum() == g.n - 1 + R * per
        if last is not None:
            new_edges = r.in_P & ~last.in_P
            assert new_edges.sum() == per
            h, _ = PB.power_vector(g.n, eu, ev, w, last.in_P, O.init_vectors(g.n, 1, 1)[:, 0], 2)
            c = PB.criticality(eu, ev, w, last.in_P, h)
            assert c[new_edges].min() >= c[~r.in_P].max()
        cur = lmax(r.in_P)
        assert cur <= prev * (1 + 1e-12)
        prev, last = cur, r


def test_alg2_branches():
    """gamma = |E| / |V| below 40: Phase A first; at or above: Phase B first
    (K_100 has gamma = 49.5).  Either way S has the target size and positive
    weights."""
    g = W.grid2d(20, 20)
    r = PB.spectral_reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 8, 5, 8.0, 3, 4,
                           sgd=SG.SgdParams(k_max=5))
    assert not r.dense and r.n_S == O.target_size(g.n, 8.0) and np.all(r.w > 0)
    k100 = W.complete(100)
    k100.w = (k100.w * np.random.default_rng(2).uniform(0.5, 2.0, k100.w.size)).astype(np.float32)
    eoe, eu, ev = O.edge_index(k100.n, k100.row_ptr, k100.col)
    wsym = np.zeros(eu.size)
    wsym[eoe] = k100.w                      # one weight per edge, both directions
    rp, cl, ww = PB.csr_of_edges(k100.n, eu, ev, wsym.astype(np.float32).astype(np.float64))
    r = PB.spectral_reduce(k100.n, rp, cl, ww, 8, 5, 4.0, 3, 4, sgd=SG.SgdParams(k_max=5))
    assert r.dense and r.n_S >= O.target_size(k100.n, 4.0) and np.all(r.w > 0)
    assert r.sparsify.in_P.sum() < eu.size
