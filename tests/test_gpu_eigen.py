"""GPU FP64 Laplacian eigenvalues (Chebyshev-filtered subspace iteration)
against closed forms (path, cycle, grids with repeated eigenvalues, complete
graph) and against the oracle's dense / shift-invert eigenvalues on reduced
graphs of the benchmark families."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import graphs as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RTOL = 1e-9


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _eigs(g, n_eig=10, **kw):
    from paper_1812_08942_amd import graphreduce as G
    say(f"eigs {g.name} n={g.n} nnz={g.nnz} n_eig={n_eig}")
    lam, rep = G.gr_laplacian_eigs(
        G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, _dev()), n_eig, **kw)
    say(f"  -> {rep}")
    return lam, rep


def _path_eigs(n):
    return 2.0 - 2.0 * np.cos(np.arange(n) * np.pi / n)


def test_path_and_cycle_closed_forms():
    n = 200
    lam, rep = _eigs(W.path(n))
    assert np.allclose(lam, _path_eigs(n)[1:11], rtol=RTOL, atol=0)
    assert rep["cholesky_warnings"] == 0
    n = 150
    lam, _ = _eigs(W.cycle(n))
    ref = np.sort(2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(1, n) / n))[:10]
    assert np.allclose(lam, ref, rtol=RTOL, atol=0)


@pytest.mark.parametrize("nx,ny", [(32, 32), (40, 30), (160, 150)])
def test_grid_closed_form_with_repeated_eigenvalues(nx, ny):
    lam, rep = _eigs(W.grid2d(nx, ny))
    ref = np.sort(np.add.outer(_path_eigs(ny), _path_eigs(nx)).ravel())[1:11]
    assert np.allclose(lam, ref, rtol=RTOL, atol=0)
    assert rep["cholesky_warnings"] == 0


def test_complete_graph_whole_complement():
    # n - 1 <= block width: the block spans the complement of the constant
    # vector, so every eigenvalue (n, with unit weights) comes out at once
    lam, rep = _eigs(W.complete(6), n_eig=8)
    assert np.allclose(lam[:5], 6.0, rtol=1e-12)
    assert np.all(np.isnan(lam[5:]))
    assert rep["block"] == 5


def test_disconnected_graph_reports_zero_eigenvalues():
    g = W.disjoint_union(W.cycle(40), W.path(30))
    lam, _ = _eigs(g, n_eig=6)
    dense = np.linalg.eigvalsh(O.laplacian_dense(g.n, g.row_ptr, g.col, g.w))
    assert abs(lam[0]) < 1e-10
    assert np.allclose(lam[1:], dense[2:7], rtol=RTOL, atol=0)


def _reduced(key, scale):
    wl = W.WORKLOADS[key]
    g = W.build_graph(key, scale)
    r = O.reduce(g.n, g.row_ptr, g.col, g.w, wl.K, wl.sweeps, wl.ratio,
                 wl.vec_seed, wl.colour_seed, fp32_coarse=True)
    return W.Graph(r.n_coarse, r.row_ptr.astype(np.int32),
                   r.col.astype(np.int32), r.w.astype(np.float32),
                   f"{key}@{scale}-reduced")


@pytest.mark.parametrize("key,scale", [("knn200k", 0.25), ("gmm70k", 0.25),
                                       ("chunglu434k", 0.05)])
def test_reduced_graphs_match_oracle(key, scale):
    g = _reduced(key, scale)
    lam, rep = _eigs(g)
    ref = O.laplacian_eigs(g.n, g.row_ptr, g.col, g.w, 10)
    assert O.n_components(g.n, g.row_ptr, g.col) == 1
    assert np.allclose(lam, ref, rtol=RTOL, atol=0), (lam, ref)
    assert rep["residual"] <= 1e-12 * rep["lambda_max_bound"]


@pytest.mark.parametrize("method", ["chebyshev", "lobpcg"])
def test_both_methods_match_oracle(method):
    for g in (W.grid2d(40, 30), W.knn2d(3000, 10, seed=4),
              W.chung_lu(5000, mean_deg=30.0, seed=3)):
        ref = O.laplacian_eigs(g.n, g.row_ptr, g.col, g.w, 10)
        lam, rep = _eigs(g, method=method)
        assert rep["method"] == method
        assert np.allclose(lam, ref, rtol=RTOL, atol=0), (g.name, lam, ref)


def test_auto_picks_lobpcg_on_hub_graphs():
    g = _reduced("chunglu434k", 0.05)
    d = np.bincount(np.repeat(np.arange(g.n), np.diff(g.row_ptr)),
                    g.w.astype(np.float64), g.n)
    assert d.max() > 16 * d.mean()
    _, rep = _eigs(g)
    assert rep["method"] == "lobpcg"
    _, rep = _eigs(W.grid2d(40, 30))
    assert rep["method"] == "chebyshev"


def test_seed_independent():
    g = W.knn2d(3000, 10, seed=9)
    a, _ = _eigs(g, seed=1)
    b, _ = _eigs(g, seed=2)
    assert np.allclose(a, b, rtol=RTOL, atol=0)


@pytest.mark.parametrize("method", ["chebyshev", "lobpcg"])
def test_eigenvectors_match_oracle(method):
    """The Ritz vectors returned with the eigenvalues: orthonormal,
    orthogonal to the all-one vector, L u = lambda u to the solve's
    tolerance, and (for eigenvalues separated from their neighbours) the
    dense oracle's eigenvector up to sign."""
    from paper_1812_08942_amd import graphreduce as G
    for g in (W.knn2d(3000, 10, seed=4), W.chung_lu(5000, mean_deg=30.0, seed=3)):
        say(f"eigpairs {g.name} {method}")
        lam, U, rep = G.gr_laplacian_eigpairs(
            G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, _dev()), 10, method=method)
        assert rep["method"] == method
        U = U.cpu().numpy()
        L = O.laplacian_dense(g.n, g.row_ptr, g.col, g.w)
        rlam, rU = O.laplacian_eigpairs(g.n, g.row_ptr, g.col, g.w, 10)
        assert np.allclose(lam, rlam, rtol=RTOL, atol=0)
        assert np.allclose(U.T @ U, np.eye(10), atol=1e-10)
        assert np.max(np.abs(U.sum(axis=0))) <= 1e-9 * np.sqrt(g.n)
        res = np.linalg.norm(L @ U - U * lam, axis=0)
        assert np.all(res <= 1e-6 * 2 * np.max(np.diag(L))), res
        gap = np.minimum(np.diff(np.r_[0.0, rlam]), np.diff(np.r_[rlam, np.inf]))
        for i in np.flatnonzero(gap > 1e-3 * rlam):
            assert abs(abs(U[:, i] @ rU[:, i]) - 1.0) <= 1e-8, (g.name, i)


def test_eigenvectors_of_a_one_node_graph_are_nan():
    from paper_1812_08942_amd import graphreduce as G
    say("eigpairs of a single node")
    g1 = G.DeviceGraph.from_numpy(np.zeros(2, np.int32), np.zeros(0, np.int32),
                                  np.zeros(0, np.float32), _dev())
    lam, U, _ = G.gr_laplacian_eigpairs(g1, 3)
    assert np.all(np.isnan(lam)) and U.shape == (1, 3) and bool(torch.isnan(U).all())
