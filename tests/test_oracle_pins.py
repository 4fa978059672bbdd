"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, invariants, hand-worked cases, brute force on tiny graphs).

Each test names the property it relies on; none re-derives the oracle's own
loop.  CPU only.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import graphs as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    vals = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.extend(line.split())
    return vals


def zoo():
    return [
        G.path(7), G.cycle(8), G.cycle(9), G.star(6), G.complete(5),
        G.grid2d(4, 4), G.barbell(4),
        G.disjoint_union(G.path(4), G.cycle(5)),
        G.with_isolated(G.path(5), 2),
        G.random_weighted(12, 0.3, seed=1),
        G.random_weighted(10, 0.5, seed=2),
    ]


def wd(g):
    return g.w.astype(np.float64)


# ------------------------------------------------------------------ RNG

def test_splitmix64_published_sequence():
    want = [int(x) for x in _gold("splitmix64_seed1234567.txt")]
    got = [O.splitmix64(1234567, i) for i in range(5)]
    assert got == want


def test_init_vectors_exact_uniform_and_centred():
    n, K = 5000, 8
    raw = O.init_vectors(n, K, 99, centre=False)
    # (2m + 1 - 2^24) / 2^24 with integer m: odd integers over 2^24
    scaled = raw * 2.0**24
    assert np.all(scaled == np.round(scaled))
    assert np.all(np.abs(scaled.astype(np.int64)) % 2 == 1)
    assert np.all(np.abs(raw) < 1.0)
    assert np.all(raw.astype(np.float32).astype(np.float64) == raw)
    # uniform(-1,1): mean 0, variance 1/3 (5-sigma statistical bounds)
    assert abs(raw.mean()) < 5 * math.sqrt(1 / 3 / raw.size)
    assert abs(raw.var() - 1 / 3) < 5 * math.sqrt(4 / 45 / raw.size)
    X = O.init_vectors(n, K, 99, centre=True)
    # orthogonal to the all-one vector (Sec. 3.2.1), within the classical
    # bound of recursive summation: |error| <= 2 n u sum|x|
    bound = 2 * n * 2.0**-53 * np.abs(X).sum(axis=0)
    assert np.all(np.abs(X.sum(axis=0)) <= bound)
    # centring only shifts columns
    shift = raw - X
    assert np.allclose(shift, shift[0:1, :], atol=1e-15, rtol=0)
    # different seeds give different vectors
    assert not np.array_equal(O.init_vectors(50, 4, 1), O.init_vectors(50, 4, 2))


# ------------------------------------------------------------ colouring

@pytest.mark.parametrize("ldf", [False, True])
def test_greedy_colouring_is_valid_and_first_fit(ldf):
    for g in zoo() + [G.chung_lu(3000, mean_deg=20, seed=9)]:
        c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 77, ldf)
        assert O.validate_colouring(g.n, g.row_ptr, g.col, c, nc) == 0
        assert nc == (c.max() + 1 if g.n else 0)
        assert nc <= g.degrees().max() + 1
        # first-fit (Grundy) property of any greedy colouring: a node of
        # colour k sees every colour 0..k-1 among its neighbours
        for v in range(g.n):
            nb = set(c[g.col[g.row_ptr[v]:g.row_ptr[v + 1]]].tolist())
            assert set(range(c[v])) <= nb


def _priority_keys(g, seed, ldf):
    deg = g.degrees() if ldf else np.zeros(g.n, np.int64)
    return [(int(deg[v]), O.splitmix64(seed, v), v) for v in range(g.n)]


@pytest.mark.parametrize("ldf", [False, True])
def test_greedy_colouring_equals_jones_plassmann_rounds(ldf):
    """The colouring is first fit in decreasing priority.  Pinned two ways:
    (i) each node's colour is the smallest absent among its higher-priority
    neighbours' colours; (ii) an independent round-synchronous schedule
    (Jones-Plassmann: a node is coloured in the round after its last
    higher-priority neighbour) reproduces it exactly."""
    for g in zoo() + [G.chung_lu(1500, mean_deg=15, seed=4),
                      G.knn2d(800, 8, seed=2)]:
        c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 91, ldf)
        key = _priority_keys(g, 91, ldf)
        nbrs = [g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() for v in range(g.n)]
        for v in range(g.n):
            up = {int(c[u]) for u in nbrs[v] if key[u] > key[v]}
            mex = 0
            while mex in up:
                mex += 1
            assert c[v] == mex
        jp = [-1] * g.n
        left = set(range(g.n))
        rounds = 0
        while left:
            ready = [v for v in left
                     if all(jp[u] >= 0 for u in nbrs[v] if key[u] > key[v])]
            assert ready
            for v in ready:
                used = {jp[u] for u in nbrs[v] if jp[u] >= 0}
                k = 0
                while k in used:
                    k += 1
                jp[v] = k
            left -= set(ready)
            rounds += 1
        assert np.array_equal(np.array(jp, np.int32), c)


def test_colouring_special_cases():
    k6 = G.complete(6)
    c, nc = O.colour_greedy(6, k6.row_ptr, k6.col, 3)
    assert nc == 6
    s = G.star(9)
    c, nc = O.colour_greedy(s.n, s.row_ptr, s.col, 3)
    assert nc == 2
    # a planted monochromatic edge is rejected
    g = G.path(4)
    assert O.validate_colouring(4, g.row_ptr, g.col,
                                np.array([0, 0, 1, 0], np.int32), 2) != 0


# ------------------------------------------------------------ smoothing

def test_gs_one_sweep_by_hand():
    want = np.array([float(x) for x in _gold("gs_path4_by_hand.txt")])
    g = G.path(4, np.array([1.0, 2.0, 3.0], np.float32))
    colours = np.array([0, 1, 0, 1], np.int32)
    X = np.array([[1.0], [2.0], [3.0], [4.0]])
    Y = O.smooth(4, g.row_ptr, g.col, wd(g), colours, 2, X, 1)
    assert np.allclose(Y[:, 0], want, rtol=0, atol=1e-15)


def _colour(g, seed=5):
    if g.colours is not None:
        return g.colours, g.n_colours
    return O.colour_greedy(g.n, g.row_ptr, g.col, seed)


def test_gs_dense_colour_step_form():
    """A colour step is the matrix (I - E_c + E_c D^-1 A) applied to X,
    E_c the diagonal indicator of colour c (degree-0 rows kept)."""
    for g in zoo():
        c, nc = _colour(g)
        X0 = O.init_vectors(g.n, 3, 4)
        L = O.laplacian_dense(g.n, g.row_ptr, g.col, wd(g))
        A = -L + np.diag(np.diag(L))
        d = np.diag(L)
        Y = X0.copy()
        for _ in range(2):
            for col in range(nc):
                e = (c == col) & (d > 0)
                M = np.eye(g.n)
                M[e] = 0.0
                M[e] += A[e] / d[e][:, None]
                Y = M @ Y
        Z = O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc, X0, 2)
        assert np.allclose(Z, Y, rtol=0, atol=1e-13)


def test_gs_invariants():
    for g in zoo() + [G.grid2d(9, 7, "lognormal", 3)]:
        c, nc = _colour(g)
        L = O.laplacian_dense(g.n, g.row_ptr, g.col, wd(g))
        # constant vectors are fixed points (rows of D^-1 A sum to one)
        X = np.full((g.n, 2), 0.375)
        assert np.allclose(O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc, X, 3),
                           0.375, rtol=0, atol=1e-15)
        X = O.init_vectors(g.n, 4, 8)
        prev_e = np.trace(X.T @ L @ X)
        prev_m = np.abs(X).max(axis=0)
        for s in range(4):
            for col in range(nc):
                # one colour step at a time: coordinate minimisation of the
                # Laplacian energy never increases it
                X = _one_colour_step(g, c, col, X)
                e = np.trace(X.T @ L @ X)
                assert e <= prev_e * (1 + 1e-12) + 1e-15
                prev_e = e
            m = np.abs(X).max(axis=0)  # convex averages: max principle
            assert np.all(m <= prev_m * (1 + 1e-15))
            prev_m = m


def _one_colour_step(g, c, col, X):
    # one sweep over a single colour class: nodes of colour `col` become
    # colour 0 and all others colour 1, and only colour 0 is swept
    c2 = np.where(c == col, 0, 1).astype(np.int32)
    return O.smooth(g.n, g.row_ptr, g.col, wd(g), c2, 1, X, 1)


def test_gs_converges_to_constant_on_connected_graph():
    g = G.random_weighted(12, 0.3, seed=1)
    c, nc = _colour(g)
    X = O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc, O.init_vectors(12, 3, 1),
                 3000)
    assert np.all(X.max(axis=0) - X.min(axis=0) < 1e-10)


def test_gs_independent_of_order_within_colour():
    g = G.random_weighted(12, 0.4, seed=3)
    c, nc = _colour(g)
    X0 = O.init_vectors(12, 5, 2)
    Y = O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc, X0, 3)
    perm = np.random.default_rng(0).permutation(g.n)   # new id of old node
    inv = np.argsort(perm)
    u, v, w = G.edges_upper(g)
    h = G.csr_from_edges(g.n, np.minimum(perm[u], perm[v]),
                         np.maximum(perm[u], perm[v]), w)
    cp = np.empty_like(c)
    cp[perm] = c
    Xp = X0[inv]
    Yp = O.smooth(h.n, h.row_ptr, h.col, h.w.astype(np.float64), cp, nc, Xp, 3)
    assert np.allclose(Yp[perm], Y, rtol=0, atol=1e-14)


def test_gs_bf16_store_rounds_every_value():
    g = G.grid2d(6, 6, "lognormal", 1)
    X = O.smooth(g.n, g.row_ptr, g.col, wd(g), g.colours, 2,
                 O.init_vectors(g.n, 4, 3), 2, bf16=True)
    bits = X.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert O.round_bf16(1.0 + 2.0**-8) == 1.0           # tie -> even
    assert O.round_bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6  # tie -> even (up)
    assert O.round_bf16(1.0 + 2.0**-8 + 2.0**-12) == 1.0 + 2.0**-7


# ------------------------------------------------------------- affinity

def test_affinity_range_symmetry_and_closed_forms():
    for g in zoo():
        c, nc = _colour(g)
        X = O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc,
                     O.init_vectors(g.n, 6, 1), 2)
        a = O.affinity(g.n, g.row_ptr, g.col, X)
        assert np.all((a >= 0) & (a <= 1))
        # a_pq == a_qp bit for bit
        rows = np.repeat(np.arange(g.n), g.degrees())
        key = rows * g.n + g.col
        tkey = g.col.astype(np.int64) * g.n + rows
        order = np.argsort(key)
        pos = order[np.searchsorted(key[order], tkey)]
        assert np.array_equal(a, a[pos])
    # K = 1: any two nonzero scalars are parallel -> a = 1
    g = G.path(5)
    X = np.array([[1.0], [-2.0], [0.5], [3.0], [-7.0]])
    assert np.allclose(O.affinity(5, g.row_ptr, g.col, X), 1.0, atol=1e-15)
    # rows at angle theta: a = cos^2(theta); orthogonal rows: 0; zero row: 0
    th = np.array([0.0, 0.3, 1.1, 1.1 + math.pi / 2, 2.0])
    X = np.stack([np.cos(th), np.sin(th)], 1) * np.array([[1], [2], [0.5], [3],
                                                          [1]])
    a = O.affinity(5, g.row_ptr, g.col, X)
    want = np.cos(np.diff(th)) ** 2
    up = a[[0, 2, 4, 6]]   # entries (0,1), (1,2), (2,3), (3,4)
    assert np.allclose(up, want, atol=1e-14)
    X[2] = 0.0
    a = O.affinity(5, g.row_ptr, g.col, X)
    assert a[2] == 0.0 and a[3] == 0.0   # entries touching node 2
    # invariance to per-row scaling
    X = O.init_vectors(5, 3, 7)
    s = np.array([[2.0], [-0.25], [8.0], [1.5], [-3.0]])
    assert np.allclose(O.affinity(5, g.row_ptr, g.col, X * s),
                       O.affinity(5, g.row_ptr, g.col, X), atol=1e-14)


def test_algebraic_distance_grows_with_separation_on_path():
    """1 - a behaves like a squared distance on a path (Sec. 3.2.2): after
    smoothing, the affinity of the pair (p, p+k) falls as k grows."""
    n = 200
    g = G.path(n)
    c = (np.arange(n) % 2).astype(np.int32)
    X = O.smooth(n, g.row_ptr, g.col, wd(g), c, 2,
                 O.init_vectors(n, 16, 3), 30)
    p = 100
    d = []
    for k in (1, 2, 4, 8):
        num = (X[p] @ X[p + k]) ** 2
        d.append(1 - num / ((X[p] @ X[p]) * (X[p + k] @ X[p + k])))
    assert all(d[i] < d[i + 1] for i in range(3))


# ---------------------------------------------------------- aggregation

def test_aggregate_by_hand_path():
    # path 0-1-2-3-4-5 ; edge affinities (0,1)=.9 (1,2)=.5 (2,3)=.7
    # (3,4)=.7 (4,5)=.2
    g = G.path(6)
    ea = {(0, 1): .9, (1, 2): .5, (2, 3): .7, (3, 4): .7, (4, 5): .2}
    a = np.array([ea[(min(v, j), max(v, j))]
                  for v in range(6)
                  for j in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]])
    a = 1.0 - a    # decisions are taken on the algebraic distance d = 1 - a
    # best: 0->1, 1->0, 2->3, 3->2 (tie .7/.7 to the smaller index), 4->3,
    # 5->4.  Forest {0,1}, {2,3}, {3,4}, {4,5}: |F| = 4, n - |F| = 2
    r = O.aggregate(6, g.row_ptr, g.col, a, 1)
    assert r.best.tolist() == [1, 0, 3, 2, 3, 4]
    assert r.n_forest == 4 and r.n_coarse == 2
    assert r.agg.tolist() == [0, 0, 1, 1, 1, 1]
    # target 4: accept the top 2 forest edges: {0,1} (.9), then {2,3} (.7,
    # min 2) before {3,4} (.7, min 3)
    r = O.aggregate(6, g.row_ptr, g.col, a, 4)
    assert r.n_coarse == 4 and r.agg.tolist() == [0, 0, 1, 1, 2, 3]
    # target 3: {0,1}, {2,3}, {3,4}
    r = O.aggregate(6, g.row_ptr, g.col, a, 3)
    assert r.agg.tolist() == [0, 0, 1, 1, 1, 2]
    # all-equal affinities: every node points to its smaller neighbour
    r = O.aggregate(6, g.row_ptr, g.col, np.full(10, 0.5), 1)
    assert r.best.tolist() == [1, 0, 1, 2, 3, 4]
    assert r.n_coarse == 1


def test_aggregate_invariants():
    for g in zoo() + [G.chung_lu(2000, mean_deg=12, seed=4)]:
        c, nc = _colour(g)
        X = O.smooth(g.n, g.row_ptr, g.col, wd(g), c, nc,
                     O.init_vectors(g.n, 8, 2), 5)
        d = O.distance(g.n, g.row_ptr, g.col, X)
        for T in (1, max(1, g.n // 3), g.n):
            r = O.aggregate(g.n, g.row_ptr, g.col, d, T)
            assert r.n_coarse == max(T, g.n - r.n_forest)
            assert r.agg.min() == 0 and r.agg.max() == r.n_coarse - 1
            # ids in order of first appearance (smallest member)
            first = np.unique(r.agg, return_index=True)[1]
            assert np.all(np.diff(first) > 0)
            # each aggregate is connected in G
            for I in range(r.n_coarse):
                mem = np.nonzero(r.agg == I)[0]
                sub = set(mem.tolist())
                seen, stack = {mem[0]}, [mem[0]]
                while stack:
                    v = stack.pop()
                    for j in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
                        if j in sub and j not in seen:
                            seen.add(j)
                            stack.append(j)
                assert seen == sub


# -------------------------------------------------------------- Galerkin

def test_galerkin_matches_dense_and_laplacian_identities():
    rng = np.random.default_rng(0)
    for g in zoo():
        nc = max(1, g.n // 3)
        agg = np.concatenate([np.arange(nc), rng.integers(0, nc, g.n - nc)])
        rng.shuffle(agg)
        agg = agg.astype(np.int32)
        c_rp, c_col, c_w = O.galerkin(g.n, g.row_ptr, g.col, wd(g), agg, nc)
        P = O.prolongation_dense(agg, nc)
        L = O.laplacian_dense(g.n, g.row_ptr, g.col, wd(g))
        LR = O.laplacian_dense(nc, c_rp, c_col, c_w)
        # L_R = P^T L P  (Sec. 3.2.2): a Laplacian again, internal edges gone
        assert np.allclose(LR, P.T @ L @ P, atol=1e-12)
        assert np.allclose(LR.sum(axis=1), 0, atol=1e-12)
        assert np.allclose(LR, LR.T, atol=0)
        # Galerkin identity for random coarse vectors
        xr = rng.standard_normal(nc)
        assert np.isclose(xr @ LR @ xr, (P @ xr) @ L @ (P @ xr), rtol=1e-12)
        # weight conservation: cut weight + internal weight = total weight
        u, v, w = G.edges_upper(g)
        internal = w.astype(np.float64)[agg[u] == agg[v]].sum()
        assert np.isclose(c_w.sum() / 2 + internal, w.astype(np.float64).sum(),
                          rtol=1e-13)
        # structure: rows and columns ascending, no diagonal
        for I in range(nc):
            cc = c_col[c_rp[I]:c_rp[I + 1]]
            assert np.all(np.diff(cc) > 0) and I not in cc


def test_poincare_separation_after_reduction():
    """lambda_i(L_G) <= mu_i(L_R, P^T P): the reduced pencil's eigenvalues
    bound the fine ones from above (Poincare separation for the subspace
    range(P))."""
    import scipy.linalg as sl

    g = G.grid2d(16, 16, "lognormal", 2)
    r = O.reduce(g.n, g.row_ptr, g.col, wd(g), 8, 5, 4.0, 1, 2,
                 colours=g.colours, n_colours=2)
    lam = np.linalg.eigvalsh(O.laplacian_dense(g.n, g.row_ptr, g.col, wd(g)))
    LR = O.laplacian_dense(r.n_coarse, r.row_ptr, r.col, r.w)
    P = O.prolongation_dense(r.agg, r.n_coarse)
    mu = sl.eigh(LR, P.T @ P, eigvals_only=True)
    assert np.all(lam[:r.n_coarse] <= mu + 1e-10)


# ---------------------------------------------------------------- eigen

def test_grid64_eigenvalues_closed_form():
    want = np.array([float(x) for x in _gold("grid64_laplacian_eigs.txt")])
    g = G.grid2d(64, 64)
    lam = np.sort(np.linalg.eigvalsh(O.laplacian_dense(g.n, g.row_ptr, g.col,
                                                       wd(g))))[:11]
    assert np.allclose(lam, want, atol=6e-11)
    a = np.arange(64)
    cf = np.sort((4 * np.sin(np.pi * a / 128) ** 2)[:, None]
                 + (4 * np.sin(np.pi * a / 128) ** 2)[None, :], axis=None)
    assert np.allclose(lam, cf[:11], atol=1e-12)
    got = O.laplacian_eigs(g.n, g.row_ptr, g.col, wd(g), 10)
    assert np.allclose(got, want[1:], atol=6e-11)


def test_small_graph_spectra_closed_forms():
    n = 9
    lam = O.laplacian_eigs(n, *_rcw(G.cycle(n)), count=n - 1)
    k = np.arange(1, n)
    assert np.allclose(lam, np.sort(2 - 2 * np.cos(2 * np.pi * k / n)),
                       atol=1e-12)
    lam = O.laplacian_eigs(n, *_rcw(G.path(n)), count=n - 1)
    assert np.allclose(lam, 2 - 2 * np.cos(np.pi * np.arange(1, n) / n),
                       atol=1e-12)
    lam = O.laplacian_eigs(6, *_rcw(G.complete(6)), count=5)
    assert np.allclose(lam, 6.0, atol=1e-12)
    lam = O.laplacian_eigs(7, *_rcw(G.star(7)), count=6)
    assert np.allclose(lam, [1, 1, 1, 1, 1, 7], atol=1e-12)
    # disconnected: one zero skipped per component
    g = G.disjoint_union(G.complete(4), G.complete(3))
    lam = O.laplacian_eigs(g.n, *_rcw(g), count=5)
    assert np.allclose(lam, [3, 3, 4, 4, 4], atol=1e-12)


def _rcw(g):
    return g.row_ptr, g.col, wd(g)


# ------------------------------------------------------------ multilevel

def test_reduce_grid64_hits_target_and_bounds():
    g = G.grid2d(64, 64)
    r = O.reduce(g.n, g.row_ptr, g.col, wd(g), 8, 5, 4.0, 11, 21,
                 colours=g.colours, n_colours=2)
    assert r.n_coarse == 1024
    assert r.agg.max() == 1023
    assert O.n_components(r.n_coarse, r.row_ptr, r.col) == 1
    # multilevel: a larger ratio needs several levels and still lands on T
    r = O.reduce(g.n, g.row_ptr, g.col, wd(g), 8, 5, 64.0, 11, 21,
                 colours=g.colours, n_colours=2)
    assert r.n_coarse == 64 and len(r.levels) >= 2
    # composed ids agree with the final coarse graph: total cut weight
    u, v, w = G.edges_upper(g)
    cut = w.astype(np.float64)[r.agg[u] != r.agg[v]].sum()
    assert np.isclose(cut, r.w.sum() / 2, rtol=1e-12)


def test_reduce_degenerate_inputs():
    # edgeless graph: no level can shrink it
    g = G.csr_from_edges(5, np.zeros(0), np.zeros(0), np.zeros(0))
    r = O.reduce(5, g.row_ptr, g.col, wd(g), 4, 2, 2.0, 1, 1)
    assert r.no_progress and r.n_coarse == 5
    # ratio 1: nothing to do
    g = G.path(6)
    r = O.reduce(6, g.row_ptr, g.col, wd(g), 4, 2, 1.0, 1, 1)
    assert r.n_coarse == 6 and len(r.levels) == 0
    # isolated nodes stay singletons
    g = G.with_isolated(G.cycle(6), 2)
    r = O.reduce(g.n, g.row_ptr, g.col, wd(g), 4, 2, 100.0, 1, 1)
    assert r.agg[6] != r.agg[7] and np.sum(r.agg == r.agg[6]) == 1


# ----------------------------------------------------- derivative pins

def test_smooth_vjp_matches_finite_differences_and_adjoint_identity():
    g = G.random_weighted(9, 0.45, seed=5)
    c, nc = _colour(g)
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    E = eu.size
    rng = np.random.default_rng(1)
    wE = rng.uniform(0.5, 2.0, E)
    X0 = O.init_vectors(g.n, 3, 5)
    Gc = rng.standard_normal((g.n, 3))
    S = 3

    def f(w, X):
        wfull = w[eoe]
        return np.sum(Gc * O.smooth(g.n, g.row_ptr, g.col, wfull, c, nc, X, S))

    gw, gX = O.smooth_vjp(g.n, g.row_ptr, g.col, wE, c, nc, X0, Gc, S)
    for e in range(E):
        h = 1e-6 * wE[e]
        wp, wm = wE.copy(), wE.copy()
        wp[e] += h
        wm[e] -= h
        fd = (f(wp, X0) - f(wm, X0)) / (2 * h)
        assert abs(fd - gw[e]) <= 1e-6 * max(1.0, abs(fd))
    # the map is linear in X0: <G, J dX> = <J^T G, dX> exactly
    dX = rng.standard_normal(X0.shape)
    lhs = f(wE, X0 + dX) - f(wE, X0)
    assert np.isclose(lhs, np.sum(gX * dX), rtol=1e-10, atol=1e-12)


def test_rayleigh_gradient_hellmann_feynman():
    """At an eigenvector, dR_i/dw_e equals the derivative of the simple
    eigenvalue lambda_i (first-order perturbation, Sec. 3.3.3), checked by
    finite differences of dense eigenvalues."""
    g = G.random_weighted(10, 0.5, seed=6)
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    wE = np.random.default_rng(2).uniform(0.5, 2.0, eu.size)

    def eigs(w):
        L = O.laplacian_dense(g.n, g.row_ptr, g.col, w[eoe])
        return np.linalg.eigh(L)

    lam, U = eigs(wE)
    assert np.min(np.diff(lam[1:5])) > 1e-3   # simple eigenvalues
    Um = U[:, 1:5]
    R = O.rq_forward(eu, ev, wE, Um)
    assert np.allclose(R, lam[1:5], atol=1e-12)
    gR = np.array([1.0, -0.5, 0.25, 2.0])
    gw = O.rq_backward(eu, ev, wE, Um, gR)
    for e in range(eu.size):
        h = 1e-6
        wp, wm = wE.copy(), wE.copy()
        wp[e] += h
        wm[e] -= h
        fd = (eigs(wp)[0][1:5] - eigs(wm)[0][1:5]) / (2 * h) @ gR
        assert abs(fd - gw[e]) < 1e-6
    # normalized-cut quotient (B = D): its gradient against FD of R itself
    Rd = O.rq_forward(eu, ev, wE, Um, O.B_DEGREE)
    gwd = O.rq_backward(eu, ev, wE, Um, gR, O.B_DEGREE)
    for e in range(eu.size):
        h = 1e-6
        wp, wm = wE.copy(), wE.copy()
        wp[e] += h
        wm[e] -= h
        fd = (O.rq_forward(eu, ev, wp, Um, 1) - O.rq_forward(eu, ev, wm, Um, 1)) \
            / (2 * h) @ gR
        assert abs(fd - gwd[e]) < 1e-7
    assert Rd.shape == (4,)


# -------------------------------------------------- Alg. 1 edge scaling

def _sgd_setup(seed=3, n=60):
    g = G.random_weighted(n, 0.15, seed=seed)
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    w = np.zeros(eu.size)
    w[eoe] = g.w
    keep = G.spanning_sparsifier(g.n, eu, ev, w, 0.1)
    return g, eu, ev, w, keep


def test_sgd_constraint_monotone_weights_and_falling_lambda_n():
    """Alg. 1: weights only grow, lambda_1 (the degree-ratio estimate) stays
    above lambda_1^(0) * Delta_bar, and the dense generalised lambda_n of
    (L_G, L_P) falls."""
    import scipy.linalg as sl
    from oracle import sgd as S

    g, eu, ev, w, keep = _sgd_setup()
    p = S.SgdParams(k_max=15)
    r = S.sgd_scale(g.n, eu, ev, w, eu[keep], ev[keep], w[keep], p)
    assert r.iterations >= 2
    assert np.all(r.w_P >= w[keep] - 1e-15)
    lam1_0 = r.lambda_1[0]
    assert np.all(np.array(r.lambda_1) >= lam1_0 * p.delta_bar * (1 - 1e-12))

    def gen_lmax(wp):
        Lg = S._lap(g.n, eu, ev, w)
        Lp = S._lap(g.n, eu[keep], ev[keep], wp)
        J = np.ones((g.n, g.n)) / g.n
        return sl.eigh(Lg + J, Lp + J, eigvals_only=True)[-1]

    assert gen_lmax(r.w_P) < gen_lmax(w[keep])


def _cycle5_path():
    """G = the 5-cycle with unit weights, P = its path 0-1-2-3-4.  The
    vector u = (2, 1, 0, -1, -2) is the dominant generalised eigenvector of
    (L_G, L_P) whenever P's four weights are equal (L_P u = c (e_0 - e_4),
    L_G u = 5 (e_0 - e_4)), so h_t stays parallel to u and every quantity of
    Alg. 1 has a closed form."""
    g_eu = np.array([0, 0, 1, 2, 3], np.int32)
    g_ev = np.array([1, 4, 2, 3, 4], np.int32)
    p_eu = np.array([0, 1, 2, 3], np.int32)
    p_ev = np.array([1, 2, 3, 4], np.int32)
    u = np.array([2.0, 1.0, 0.0, -1.0, -2.0])
    return g_eu, g_ev, np.ones(5), p_eu, p_ev, np.ones(4), u


def test_sgd_hand_worked_momentum_and_step_schedule():
    """Three iterations of Alg. 1 worked by hand on the 5-cycle and its path
    (Delta_bar = 0.03, K_max = 3: no guard trips).  With equal path weights
    c: lambda_n = h^T L_G h = 5 / c (h = u / (2 sqrt c)), every path edge has
    s = -lambda_n / (4c) = -5 / (4 c^2), and lambda_1 = min d_G/d_P = 1/c.
      k = 1: eta_max = 0.1 * 1 / 1.25 = 0.08, dw = 0.08 * 1.25 = 0.1, c = 1.1
      k = 2: eta = eta_max (lambda_n^(1) = lambda_n^(0));
             dw = 0.9 * 0.1 + 0.08 * 5 / (4 * 1.1^2) = 0.09 + 0.1 / 1.21
      k = 3: eta = (lambda_n^(2) / lambda_n^(0)) eta_max = 0.08 / 1.1;
             dw = 0.9 dw_2 + (0.08 / 1.1) * 5 / (4 c_2^2)
    A dropped or sign-flipped momentum term changes k = 2; an inverted or
    missing step-size schedule changes k = 3.  Both modes agree bit for bit."""
    from oracle import sgd as S

    g_eu, g_ev, g_w, p_eu, p_ev, w0, u = _cycle5_path()
    prm = S.SgdParams(alpha=0.9, eta_scale=0.1, eps=1e-3, k_max=3, delta_bar=0.03, t=2)
    c1 = 1.1
    dw2 = 0.09 + 0.1 / 1.21
    c2 = c1 + dw2
    dw3 = 0.9 * dw2 + (0.08 / 1.1) * 5.0 / (4.0 * c2 * c2)
    c3 = c2 + dw3
    res = {}
    for mode in ("parallel", "sequential"):
        r = S.sgd_scale(5, g_eu, g_ev, g_w, p_eu, p_ev, w0, prm, mode=mode, h0=u)
        assert r.iterations == 3
        assert np.allclose(r.w_P, c3, rtol=1e-13, atol=0), (mode, r.w_P, c3)
        assert np.allclose(r.lambda_n, [5.0, 5.0 / c1, 5.0 / c2], rtol=1e-12, atol=0)
        assert np.allclose(r.lambda_1, [1.0, 1.0 / c1, 1.0 / c2, 1.0 / c3], rtol=1e-13, atol=0)
        res[mode] = r
    assert np.array_equal(res["parallel"].w_P, res["sequential"].w_P)
    assert res["parallel"].lambda_1 == res["sequential"].lambda_1


def test_sgd_hand_worked_guard_both_modes():
    """One iteration on the same pair with Delta_bar = 0.5, K_max = 20
    (Delta = 2^-0.05): every path edge proposes dw = 0.1, and the guard
    trips at the inner nodes, whose cap is 2/Delta - 2.
      parallel: node 1 (likewise 2, 3) shares its cap between its two edges,
        so every edge gets (2/Delta - 2)/2 and w = 1/Delta = 2^0.05;
      sequential (the paper's edge loop, running d_P): edge (0,1) takes
        min(2/Delta - 1, 2/Delta - 2) = 2/Delta - 2, which exhausts node 1,
        so edge (1,2) gets 0; edge (2,3) again gets 2/Delta - 2 and (3,4) 0.
    Either way lambda_1 lands exactly on lambda_1^(0) Delta = Delta."""
    from oracle import sgd as S

    g_eu, g_ev, g_w, p_eu, p_ev, w0, u = _cycle5_path()
    prm = S.SgdParams(alpha=0.9, eta_scale=0.1, eps=1.0, k_max=20, delta_bar=0.5, t=2)
    delta = 0.5 ** (1.0 / 20)
    par = S.sgd_scale(5, g_eu, g_ev, g_w, p_eu, p_ev, w0, prm, mode="parallel", h0=u)
    seq = S.sgd_scale(5, g_eu, g_ev, g_w, p_eu, p_ev, w0, prm, mode="sequential", h0=u)
    assert par.iterations == 1 and seq.iterations == 1
    assert np.allclose(par.w_P, 2.0 ** 0.05, rtol=1e-14, atol=0)
    full = 1.0 + (2.0 / delta - 2.0)
    assert np.allclose(seq.w_P, [full, 1.0, full, 1.0], rtol=0, atol=1e-14), seq.w_P
    assert abs(par.lambda_1[1] - delta) < 1e-14 and abs(seq.lambda_1[1] - delta) < 1e-14


def test_sgd_modes_agree_without_guard_and_keep_the_bound():
    """On a random graph and a spanning sparsifier: with a loose guard
    (Delta_bar small enough that it never trips) the two modes give equal
    bits; with the default guard both keep every lambda_1 estimate at or
    above lambda_1^(0) Delta_bar and both lower the dense generalised
    lambda_n."""
    import scipy.linalg as sl
    from oracle import sgd as S

    g, eu, ev, w, keep = _sgd_setup()
    loose = S.SgdParams(k_max=6, delta_bar=1e-9)
    a = S.sgd_scale(g.n, eu, ev, w, eu[keep], ev[keep], w[keep], loose, mode="parallel")
    b = S.sgd_scale(g.n, eu, ev, w, eu[keep], ev[keep], w[keep], loose, mode="sequential")
    assert a.iterations == b.iterations >= 2
    assert np.array_equal(a.w_P, b.w_P)

    def gen_lmax(wp):
        Lg = S._lap(g.n, eu, ev, w)
        Lp = S._lap(g.n, eu[keep], ev[keep], wp)
        J = np.ones((g.n, g.n)) / g.n
        return sl.eigh(Lg + J, Lp + J, eigvals_only=True)[-1]

    p = S.SgdParams(k_max=15)
    lam0 = gen_lmax(w[keep])
    for mode in ("parallel", "sequential"):
        r = S.sgd_scale(g.n, eu, ev, w, eu[keep], ev[keep], w[keep], p, mode=mode)
        assert np.all(np.array(r.lambda_1) >= r.lambda_1[0] * p.delta_bar * (1 - 1e-12))
        assert np.all(r.w_P >= w[keep])
        assert gen_lmax(r.w_P) < lam0


def test_sgd_power_vector_and_sensitivity_against_dense_eigen():
    """h_t approaches the dominant generalised eigenvector, and the
    sensitivity -lambda_n (e_pq^T u_n)^2 (u_n^T L_P u_n = 1) matches finite
    differences of the dense generalised lambda_n (Sec. 3.3.4)."""
    import scipy.linalg as sl
    from oracle import sgd as S

    g, eu, ev, w, keep = _sgd_setup(seed=5, n=40)
    pe, pv = eu[keep], ev[keep]
    Lg = S._lap(g.n, eu, ev, w)
    J = np.ones((g.n, g.n)) / g.n

    def gen(wp):
        return sl.eigh(Lg + J, S._lap(g.n, pe, pv, wp) + J)

    lam, U = gen(w[keep])
    u = U[:, -1] / np.sqrt(U[:, -1] @ S._lap(g.n, pe, pv, w[keep]) @ U[:, -1])
    h = S.power_vector(Lg, S._lap(g.n, pe, pv, w[keep]),
                       O.init_vectors(g.n, 1, 7)[:, 0], 60)
    assert abs(abs(h @ S._lap(g.n, pe, pv, w[keep]) @ u) - 1.0) < 1e-6
    sens = -lam[-1] * (u[pe] - u[pv]) ** 2
    for e in range(0, len(keep), max(1, len(keep) // 8)):
        hh = 1e-6 * w[keep][e]
        wp, wm = w[keep].copy(), w[keep].copy()
        wp[e] += hh
        wm[e] -= hh
        fd = (gen(wp)[0][-1] - gen(wm)[0][-1]) / (2 * hh)
        assert abs(fd - sens[e]) <= 1e-5 * max(1.0, abs(fd))


# -------------------------------------------------- data restriction (Alg. 6)

def test_restrict_mean_closed_forms():
    """F_R = H_G^R F as the averaging restriction: constant data stays
    constant, the identity aggregation returns F, indicator data gives the
    fraction of each aggregate's members in the set, and count-weighted rows
    of F_R add up to the column sums of F."""
    rng = np.random.default_rng(3)
    n, nc, d = 500, 37, 5
    agg = np.concatenate([np.arange(nc), rng.integers(0, nc, n - nc)]).astype(np.int32)
    rng.shuffle(agg)
    cnt = np.bincount(agg, minlength=nc)
    # constant columns (values exact in float32)
    F = np.tile(np.array([1.5, -2.0, 0.25, 3.0, 0.0], np.float32), (n, 1))
    assert np.array_equal(O.restrict_mean(agg, nc, F), F[:nc])
    # identity aggregation
    X = rng.standard_normal((n, d)).astype(np.float32)
    assert np.array_equal(O.restrict_mean(np.arange(n, dtype=np.int32), n, X), X)
    # indicator of a node set: the fraction of members inside it
    inset = rng.random(n) < 0.3
    frac = np.array([inset[agg == i].mean() for i in range(nc)])
    got = O.restrict_mean(agg, nc, inset.astype(np.float32)[:, None])[:, 0]
    assert np.allclose(got, frac, rtol=1e-7, atol=0)
    # sum preservation
    R = O.restrict_mean(agg, nc, X).astype(np.float64)
    assert np.allclose((R * cnt[:, None]).sum(axis=0), X.astype(np.float64).sum(axis=0),
                       rtol=1e-6, atol=1e-5)


def test_restrict_mean_hand_example():
    """Three nodes in aggregate 0 and one in aggregate 1, worked by hand."""
    agg = np.array([0, 1, 0, 0], np.int32)
    F = np.array([[1.0, 10.0], [7.0, -1.0], [2.0, 20.0], [6.0, 0.0]], np.float32)
    R = O.restrict_mean(agg, 2, F)
    assert np.array_equal(R, np.array([[3.0, 10.0], [7.0, -1.0]], np.float32))


# -------------------------------------------------- threaded oracle loops

def test_threaded_oracle_loops_are_bit_identical():
    """The smoothing and affinity node loops give the same bits on 1 and on
    several threads (each node's arithmetic is unchanged, and a colour class
    has no inner edges), in float64 and with bfloat16 rounding."""
    g = G.random_weighted(2000, 0.01, seed=11)
    cols, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 5)
    X = O.init_vectors(g.n, 16, 3)
    for bf16 in (False, True):
        a = O.smooth(g.n, g.row_ptr, g.col, g.w, cols, nc, X, 5, bf16=bf16)
        da = O.distance(g.n, g.row_ptr, g.col, a)
        with O.threads(4):
            b = O.smooth(g.n, g.row_ptr, g.col, g.w, cols, nc, X, 5, bf16=bf16)
            db = O.distance(g.n, g.row_ptr, g.col, b)
        assert np.array_equal(a, b) and np.array_equal(da, db)
