"""Pins of the oracle's solution refinement (Alg. 3, Sec. 3.5) and
multilevel Laplacian eigensolver (Alg. 5, Sec. 4.1): closed forms on the
cycle, fixed points at exact eigenvectors, the mass matrices induced by the
hierarchy, Poincare separation, the identity hierarchy, and Gram-Schmidt
against a library QR."""
import numpy as np
import pytest

from oracle import multilevel as M
from oracle import oracle as O
from workloads import graphs as W


def test_alg3_reading_reduces_to_the_written_step():
    """y - theta D^-1 (L - 0 B) y is Alg. 3's (1 - theta) y + theta D^-1 A y."""
    g = W.random_weighted(40, 0.2, seed=2)
    x = np.random.default_rng(1).standard_normal(g.n)
    a = M.jacobi_filter(g.row_ptr, g.col, g.w, x[:, None], theta=0.7, iters=1)[:, 0]
    b = M.alg3_step_by_definition(g.row_ptr, g.col, g.w, x, 0.7)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_filter_closed_form_on_the_cycle(lam):
    """On the n-cycle (degree 2) cos(2 pi m v / n) is an eigenvector with
    mu_m = 2 - 2 cos(2 pi m / n); one shifted step multiplies it by
    1 - theta (mu_m - lam) / 2 (B = I)."""
    n, theta, it = 48, 2.0 / 3.0, 5
    g = W.cycle(n)
    v = np.arange(n)
    y = np.stack([np.cos(2 * np.pi * 1 * v / n) + 0.5 * np.cos(2 * np.pi * 7 * v / n)], 1)
    out = M.jacobi_filter(g.row_ptr, g.col, g.w, y, theta, it, lam=[lam])[:, 0]
    f = lambda m: (1 - theta * ((2 - 2 * np.cos(2 * np.pi * m / n)) - lam) / 2) ** it
    expect = f(1) * np.cos(2 * np.pi * v / n) + 0.5 * f(7) * np.cos(2 * np.pi * 7 * v / n)
    assert np.allclose(out, expect, rtol=0, atol=1e-13)


def test_exact_generalized_eigenvectors_are_fixed_points():
    import scipy.linalg as sl

    g = W.random_weighted(30, 0.25, seed=4)
    b = np.random.default_rng(2).uniform(1.0, 3.0, g.n)
    L = O.laplacian_dense(g.n, g.row_ptr, g.col, g.w)
    lam, U = sl.eigh(L, np.diag(b))
    out = M.jacobi_filter(g.row_ptr, g.col, g.w, U[:, 1:5], 0.6, 7, lam=lam[1:5], bdiag=b)
    assert np.allclose(out, U[:, 1:5], rtol=0, atol=1e-11)


@pytest.mark.parametrize("cut", [M.RATIO_CUT, M.NORMALIZED_CUT])
def test_mass_hierarchy_matches_the_finest_quotient(cut):
    """x^T L_Y x / x^T B_Y x equals the finest quotient of the prolonged x
    (the Galerkin graphs and the induced B together)."""
    g = W.grid2d(24, 24)
    r = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 8, 5, 16.0, 3, 4,
                 colours=g.colours, n_colours=g.n_colours)
    assert len(r.maps) >= 2
    B = M.mass_hierarchy(g.n, g.row_ptr, g.w, r.maps, cut)
    x = np.random.default_rng(5).standard_normal(r.n_coarse)
    xf = x.copy()
    for agg in reversed(r.maps):
        xf = xf[agg]
    Lc = O.laplacian_dense(r.n_coarse, r.row_ptr, r.col, r.w)
    Lf = O.laplacian_dense(g.n, g.row_ptr, g.col, g.w)
    qc = (x @ Lc @ x) / (x @ (B[-1] * x))
    qf = (xf @ Lf @ xf) / (xf @ (B[0] * xf))
    assert abs(qc - qf) <= 1e-12 * qf
    if cut == M.RATIO_CUT:
        assert np.array_equal(B[-1], np.bincount(r.agg, minlength=r.n_coarse).astype(float))


def test_coarse_eigenvalues_bound_the_fine_ones():
    """Poincare separation: the i-th coarsest generalised eigenvalue is at
    least the i-th fine one."""
    g = W.knn2d(600, 8, seed=3)
    cols, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 5)
    r = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 8, 5, 6.0, 3, 4)
    B = M.mass_hierarchy(g.n, g.row_ptr, g.w, r.maps)
    lc, _ = M.generalized_eigpairs(r.n_coarse, r.row_ptr, r.col, r.w, B[-1], 10)
    lf = O.laplacian_eigs(g.n, g.row_ptr, g.col, g.w, 10)
    assert np.all(lc >= lf * (1 - 1e-12))


def test_identity_hierarchy_returns_exact_eigenvectors():
    """With no coarse level (psi = 1) Alg. 5 is the direct solve: exact
    eigenvectors, which the filter leaves alone."""
    g = W.random_weighted(50, 0.15, seed=8)
    res = M.multilevel_eigs(g.n, g.row_ptr, g.col, g.w, [], [], 6)
    lam, U = O.laplacian_eigpairs(g.n, g.row_ptr, g.col, g.w, 6)
    assert np.min(np.diff(lam)) > 1e-6           # distinct: unique up to sign
    assert np.allclose(np.abs(np.sum(res.U * U, axis=0)), 1.0, rtol=0, atol=1e-10)
    assert np.allclose(res.lam_coarse, lam, rtol=1e-12)


def test_gram_schmidt_against_library_qr():
    rng = np.random.default_rng(3)
    n, k = 200, 7
    U = rng.standard_normal((n, k))
    Q = M.gram_schmidt(U)
    R = np.linalg.qr(np.column_stack([np.ones(n), U]))[0][:, 1:]
    s = np.sign(np.sum(Q * R, axis=0))
    assert np.allclose(Q, R * s, rtol=0, atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(k), atol=1e-12)
    assert np.allclose(Q.sum(axis=0), 0.0, atol=1e-11)
    b = rng.uniform(0.5, 2.0, n)
    Qb = M.gram_schmidt(U, b)
    assert np.allclose(Qb.T @ (b[:, None] * Qb), np.eye(k), atol=1e-12)
    assert np.allclose(b @ Qb, 0.0, atol=1e-11)


def test_multilevel_vectors_approach_the_direct_ones():
    """On the 32 x 32 grid reduced 8x: the refined vectors' Ritz values lie
    above the exact eigenvalues (Courant-Fischer), and the filter lowers
    them compared with the bare prolongation."""
    g = W.grid2d(32, 32)
    r = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 8, 5, 8.0, 11, 21,
                 colours=g.colours, n_colours=g.n_colours)
    lam = O.laplacian_eigs(g.n, g.row_ptr, g.col, g.w, 8)
    L = O.laplacian_dense(g.n, g.row_ptr, g.col, g.w)

    def ritz(U):
        return np.linalg.eigvalsh(U.T @ L @ U)

    bare = M.multilevel_eigs(g.n, g.row_ptr, g.col, g.w, r.maps, r.graphs, 8, iters=0)
    ref = M.multilevel_eigs(g.n, g.row_ptr, g.col, g.w, r.maps, r.graphs, 8, iters=6)
    rb, rr = ritz(bare.U), ritz(ref.U)
    assert np.all(rr >= lam * (1 - 1e-10)) and np.all(rb >= lam * (1 - 1e-10))
    assert np.sum(rr) < np.sum(rb)
