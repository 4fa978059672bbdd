"""GPU parity of the edge-weight derivative kernels against the oracle:
edge numbering (bit-exact), FP64 Rayleigh quotients and their edge
gradients (1e-12 relative), the autograd.Function, gradcheck, and the
first-order eigenvalue sensitivity checked by finite differences of dense
eigenvalues."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import graphs as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _G():
    from paper_1812_08942_amd import graphreduce as G
    return G


def test_edge_list_bit_exact():
    dev = _dev()
    G = _G()
    for g in (W.grid2d(13, 7), W.knn2d(2000, 10, seed=5),
              W.with_isolated(W.random_weighted(30, 0.2, seed=4), 2),
              W.chung_lu(5000, mean_deg=30.0, seed=2)):
        say(f"edge list {g.name}")
        el = G.gr_edge_list(G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev))
        eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
        assert np.array_equal(el.eu.cpu().numpy(), eu)
        assert np.array_equal(el.ev.cpu().numpy(), ev)
        assert np.array_equal(el.edge_of_entry.cpu().numpy(), eoe)


@pytest.mark.parametrize("mode", [0, 1])
def test_rayleigh_forward_backward_match_oracle(mode):
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(7)
    for g in (W.knn2d(3000, 10, seed=3), W.chung_lu(4000, mean_deg=25.0, seed=8)):
        say(f"rq {g.name} mode {mode}")
        el = G.gr_edge_list(G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev))
        eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
        wE = rng.uniform(0.5, 2.0, eu.size)
        U = rng.standard_normal((g.n, 10))
        gR = rng.standard_normal(10)
        R, den = G.gr_rq_forward(el, torch.from_numpy(wE).to(dev),
                                 torch.from_numpy(U).to(dev), mode)
        Rr = O.rq_forward(eu, ev, wE, U, mode)
        assert np.allclose(R.cpu().numpy(), Rr, rtol=1e-12, atol=0)
        gw = G.gr_rq_backward(el, torch.from_numpy(U).to(dev), R, den,
                              torch.from_numpy(gR).to(dev), mode)
        gwr = O.rq_backward(eu, ev, wE, U, gR, mode)
        assert np.allclose(gw.cpu().numpy(), gwr, rtol=1e-11,
                           atol=1e-13 * np.max(np.abs(gwr)))


def test_autograd_function_and_gradcheck():
    dev = _dev()
    G = _G()
    from paper_1812_08942_amd.autograd import rayleigh_quotients

    g = W.random_weighted(25, 0.25, seed=11)
    el = G.gr_edge_list(G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev))
    rng = np.random.default_rng(3)
    U = torch.from_numpy(rng.standard_normal((g.n, 4))).to(dev)
    for mode in (0, 1):
        say(f"gradcheck mode {mode}")
        w = torch.from_numpy(rng.uniform(0.5, 2.0, el.E)).to(dev).requires_grad_(True)
        assert torch.autograd.gradcheck(
            lambda ww: rayleigh_quotients(ww, U, el, mode), (w,),
            eps=1e-6, atol=1e-8, rtol=1e-6)
        R = rayleigh_quotients(w, U, el, mode)
        gR = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device=dev)
        (R * gR).sum().backward()
        eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
        ref = O.rq_backward(eu, ev, w.detach().cpu().numpy(), U.cpu().numpy(),
                            gR.cpu().numpy(), mode)
        assert np.allclose(w.grad.cpu().numpy(), ref, rtol=1e-11, atol=1e-14)


def test_eigenvalue_sensitivity_matches_finite_differences():
    """At the Laplacian eigenvectors the GPU gradient of R_i is the
    derivative of the simple eigenvalue lambda_i (first-order perturbation,
    Sec. 3.3.3): checked against central differences of dense FP64
    eigenvalues, on a reduced graph of a Gaussian-mixture kNN graph."""
    dev = _dev()
    G = _G()
    g = W.gmm_knn(n_per=300, dim=784, n_comp=10, k=10, seed=4)
    say(f"sensitivity on reduced {g.name}")
    r = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 16, 5, 16.0,
                 14, 24)
    n = r.n_coarse
    eoe, eu, ev = O.edge_index(n, r.row_ptr, r.col)
    wE = np.zeros(eu.size)
    wE[eoe] = r.w
    lam, U = np.linalg.eigh(O.laplacian_dense(n, r.row_ptr, r.col, wE[eoe]))
    sel = [i for i in range(1, 12) if min(abs(lam[i] - lam[i - 1]),
                                          abs(lam[i + 1] - lam[i])) > 1e-6 * lam[-1]][:8]
    Um = np.ascontiguousarray(U[:, sel])
    dg = G.DeviceGraph.from_numpy(r.row_ptr, r.col, r.w.astype(np.float32), dev)
    el = G.gr_edge_list(dg)
    assert np.array_equal(el.eu.cpu().numpy(), eu)
    gR = np.linspace(1.0, 2.0, len(sel))
    R, den = G.gr_rq_forward(el, torch.from_numpy(wE).to(dev),
                             torch.from_numpy(Um).to(dev))
    assert np.allclose(R.cpu().numpy(), lam[sel], rtol=1e-10)
    gw = G.gr_rq_backward(el, torch.from_numpy(Um).to(dev), R, den,
                          torch.from_numpy(gR).to(dev)).cpu().numpy()
    for e in np.random.default_rng(0).choice(eu.size, 12, replace=False):
        h = 1e-6 * wE[e]
        wp, wm = wE.copy(), wE.copy()
        wp[e] += h
        wm[e] -= h
        lp = np.linalg.eigvalsh(O.laplacian_dense(n, r.row_ptr, r.col, wp[eoe]))
        lm = np.linalg.eigvalsh(O.laplacian_dense(n, r.row_ptr, r.col, wm[eoe]))
        fd = ((lp - lm)[sel] / (2 * h)) @ gR
        assert abs(fd - gw[e]) <= 1e-5 * max(1.0, abs(fd)), (e, fd, gw[e])


# --------------------------------------------------- reverse pass of the GS

def _vjp_case(g, K, dtype, store, seed=0):
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(seed)
    dg0 = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    el = G.gr_edge_list(dg0)
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    wE = rng.uniform(0.5, 2.0, eu.size).astype(np.float32)
    w_entries = G.gr_expand_edge_weights(el, torch.from_numpy(wE).to(dev))
    assert np.array_equal(w_entries.cpu().numpy(), wE[eoe])
    dg = G.DeviceGraph(dg0.row_ptr, dg0.col, w_entries)
    if g.colours is not None:
        c, nc = g.colours, g.n_colours
    else:
        c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 9)
    cd = torch.from_numpy(c).to(dev)
    X0 = O.init_vectors(g.n, K, 31)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    X0d = torch.from_numpy(X0).to(dev).to(tdt).contiguous()
    Gc = rng.standard_normal((g.n, K)).astype(np.float32)
    gw, gX = G.gr_smooth_vjp(dg, el, cd, nc, X0d, torch.from_numpy(Gc).to(dev),
                             5, store)
    rgw, rgX = O.smooth_vjp(g.n, g.row_ptr, g.col, wE.astype(np.float64), c,
                            nc, X0d.float().cpu().numpy().astype(np.float64),
                            Gc.astype(np.float64), 5)
    return gw.cpu().numpy(), gX.cpu().numpy(), rgw, rgX, (dg, el, cd, nc, X0d, Gc)


def _wheel(n):
    """A hub joined to every node of a cycle on n - 1 nodes (a plain star
    would be degenerate: one sweep copies the hub into every leaf, and the
    weight gradient is exactly zero)."""
    v = np.arange(1, n)
    u = np.concatenate([np.zeros(n - 1, np.int64), v])
    t = np.concatenate([v, np.roll(v, -1)])
    w = np.random.default_rng(4).uniform(0.5, 2.0, u.size).astype(np.float32)
    return W.csr_from_edges(n, u, t, w, f"wheel{n}")


def vjp_graphs():
    return {"er_30": W.random_weighted(30, 0.2, seed=3),
            "grid8_lognormal": W.grid2d(8, 8, "lognormal", 5),
            "knn_600": W.knn2d(600, 10, seed=6),
            "chunglu_3000": W.chung_lu(3000, mean_deg=40.0, seed=2),
            "grid3d_6": W.grid3d(6, seed=1),
            # one row of 2999 entries, spread over many workgroups
            "wheel_3000": _wheel(3000)}


@pytest.mark.parametrize("store", [True, False])
def test_smooth_vjp_matches_oracle_f32(store):
    """float32 states: gradients within 1e-4 of the largest FP64 component."""
    for name, g in vjp_graphs().items():
        say(f"vjp {name} f32 store={store}")
        gw, gX, rgw, rgX, _ = _vjp_case(g, 8, "f32", store)
        assert np.max(np.abs(gw - rgw)) <= 1e-4 * np.max(np.abs(rgw)), name
        assert np.max(np.abs(gX - rgX)) <= 1e-4 * np.max(np.abs(rgX)), name


def test_smooth_vjp_store_and_recompute_bitwise_equal():
    g = W.chung_lu(3000, mean_deg=40.0, seed=2)
    say("vjp store vs recompute")
    a = _vjp_case(g, 16, "f32", True)
    b = _vjp_case(g, 16, "f32", False)
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))


def test_smooth_vjp_bf16_states_report():
    """bfloat16 states (rounding treated as identity in the reverse pass):
    error against the FP64 oracle reported and bounded loosely."""
    g = W.grid3d(8, seed=2)
    say("vjp grid3d_8 bf16")
    gw, gX, rgw, rgX, _ = _vjp_case(g, 16, "bf16", False)
    ew = np.max(np.abs(gw - rgw)) / np.max(np.abs(rgw))
    ex = np.max(np.abs(gX - rgX)) / np.max(np.abs(rgX))
    print(f"[gpu-case] bf16 vjp max rel error: w {ew:.2e}, X0 {ex:.2e}")
    assert ew < 5e-2 and ex < 5e-2


def test_smooth_vjp_adjoint_identity_on_gpu():
    """The smoothing is linear in X0: <G, S(dX)> = <gX0, dX> with S the GPU
    forward itself."""
    G = _G()
    g = W.knn2d(800, 10, seed=8)
    say("vjp adjoint identity")
    gw, gX, _, _, (dg, el, cd, nc, X0d, Gc) = _vjp_case(g, 8, "f32", True)
    dX = np.random.default_rng(5).standard_normal(X0d.shape).astype(np.float32)
    Y = torch.from_numpy(dX).to(X0d.device).contiguous()
    G.gr_smooth(dg, cd, nc, Y, 5)
    lhs = float(np.sum(Gc.astype(np.float64) * Y.cpu().numpy()))
    rhs = float(np.sum(gX.astype(np.float64) * dX))
    assert abs(lhs - rhs) <= 1e-4 * (abs(lhs) + abs(rhs))


def test_smoothed_vectors_autograd():
    dev = _dev()
    G = _G()
    from paper_1812_08942_amd.autograd import smoothed_vectors

    g = W.knn2d(500, 10, seed=9)
    say("SmoothedVectors autograd")
    dg0 = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    el = G.gr_edge_list(dg0)
    c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 9)
    cd = torch.from_numpy(c).to(dev)
    rng = np.random.default_rng(2)
    wE = torch.from_numpy(rng.uniform(0.5, 2.0, el.E).astype(np.float32)).to(dev)
    wE.requires_grad_(True)
    X0 = torch.from_numpy(O.init_vectors(g.n, 8, 4).astype(np.float32)).to(dev)
    X0.requires_grad_(True)
    Gc = torch.from_numpy(rng.standard_normal((g.n, 8)).astype(np.float32)).to(dev)
    Y = smoothed_vectors(wE, X0, dg0, el, cd, nc, 5)
    (Y * Gc).sum().backward()
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    rgw, rgX = O.smooth_vjp(g.n, g.row_ptr, g.col,
                            wE.detach().cpu().numpy().astype(np.float64), c, nc,
                            X0.detach().cpu().numpy().astype(np.float64),
                            Gc.cpu().numpy().astype(np.float64), 5)
    assert np.max(np.abs(wE.grad.cpu().numpy() - rgw)) <= 1e-4 * np.max(np.abs(rgw))
    assert np.max(np.abs(X0.grad.cpu().numpy() - rgX)) <= 1e-4 * np.max(np.abs(rgX))


# ----------------------------------------------- Alg. 1 constrained SGD

@pytest.mark.parametrize("case", ["er_200", "gmm_reduced"])
def test_sgd_scale_matches_oracle(case):
    """Alg. 1 on the GPU (CG solves) against the FP64 oracle (dense solves):
    lambda_n and lambda_1 histories and the scaled weights agree to 1e-7."""
    from oracle import sgd as S

    dev = _dev()
    G = _G()
    if case == "er_200":
        g = W.random_weighted(200, 0.05, seed=12)
    else:
        big = W.gmm_knn(n_per=300, dim=784, n_comp=10, k=10, seed=4)
        r = O.reduce(big.n, big.row_ptr, big.col, big.w.astype(np.float64), 16,
                     5, 16.0, 14, 24, fp32_coarse=True)
        g = W.Graph(r.n_coarse, r.row_ptr, r.col, r.w.astype(np.float32), "gmm_red")
    say(f"sgd {case} n={g.n}")
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    w = np.zeros(eu.size)
    w[eoe] = g.w
    keep = W.spanning_sparsifier(g.n, eu, ev, w, 0.1)
    pg = W.csr_from_edges(g.n, eu[keep], ev[keep], w[keep])
    prm = S.SgdParams(k_max=12, eps=1e-4)
    ref = S.sgd_scale(g.n, eu, ev, w, eu[keep], ev[keep], w[keep], prm)
    dG = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    dP = G.DeviceGraph.from_numpy(pg.row_ptr, pg.col, pg.w, dev)
    pel = G.gr_edge_list(dP)
    assert np.array_equal(pel.eu.cpu().numpy(), eu[keep])
    wP = torch.from_numpy(w[keep].copy()).to(dev)
    rep = G.gr_sgd_scale(dG, dP, pel, wP, k_max=12, eps=1e-4, cg_tol=1e-14)
    print(f"[gpu-case] sgd {case}: iterations {rep['iterations']}, "
          f"lambda_n {rep['lambda_n'][0]:.6g} -> {rep['lambda_n'][-1]:.6g}, "
          f"cg max {rep['cg_iterations_max']}")
    assert rep["iterations"] == ref.iterations
    assert np.allclose(rep["lambda_n"], ref.lambda_n, rtol=1e-7)
    assert np.allclose(rep["lambda_1"], ref.lambda_1, rtol=1e-9)
    assert np.allclose(wP.cpu().numpy(), ref.w_P, rtol=1e-7)
    assert ref.lambda_n[-1] < ref.lambda_n[0]


def _wheel_with_isolated(n, n_iso):
    """The wheel of _wheel(n) followed by n_iso nodes without edges."""
    g = _wheel(n)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col > rows
    return W.csr_from_edges(n + n_iso, rows[up], g.col[up], g.w[up],
                            f"wheel{n}+{n_iso}")


@pytest.mark.parametrize("K,dtype,S", [(4, "f32", 1), (64, "f32", 2),
                                       (8, "bf16", 0), (32, "bf16", 3)])
def test_smooth_vjp_edge_cases(K, dtype, S):
    """One lane per row chunk (K = 4 float32, K = 8 bfloat16) up to a whole
    wave per row (K = 64 float32); no sweep (the cotangent passes through,
    the weight gradient is zero); a hub row of 599 entries cut into pieces;
    rows without neighbours, which keep their cotangent."""
    g = _wheel_with_isolated(600, 5)
    say(f"vjp edge case {g.name} K={K} {dtype} sweeps={S}")
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(K + S)
    dg0 = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    el = G.gr_edge_list(dg0)
    eoe, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
    wE = rng.uniform(0.5, 2.0, eu.size).astype(np.float32)
    dg = G.DeviceGraph(dg0.row_ptr, dg0.col,
                       G.gr_expand_edge_weights(el, torch.from_numpy(wE).to(dev)))
    c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, 9)
    X0 = O.init_vectors(g.n, K, 31)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    X0d = torch.from_numpy(X0).to(dev).to(tdt).contiguous()
    Gc = rng.standard_normal((g.n, K)).astype(np.float32)
    gw, gX = G.gr_smooth_vjp(dg, el, torch.from_numpy(c).to(dev), nc, X0d,
                             torch.from_numpy(Gc).to(dev), S, False)
    gw, gX = gw.cpu().numpy(), gX.cpu().numpy()
    rgw, rgX = O.smooth_vjp(g.n, g.row_ptr, g.col, wE.astype(np.float64), c, nc,
                            X0d.float().cpu().numpy().astype(np.float64),
                            Gc.astype(np.float64), S)
    iso = np.arange(600, g.n)
    assert np.array_equal(gX[iso], Gc[iso])
    if S == 0:
        assert np.array_equal(gX, Gc) and not np.any(gw)
        return
    tol = 1e-4 if dtype == "f32" else 5e-2
    assert np.max(np.abs(gw - rgw)) <= tol * np.max(np.abs(rgw))
    assert np.max(np.abs(gX - rgX)) <= tol * np.max(np.abs(rgX))


def test_smooth_vjp_without_edges():
    """A graph with no edges: every row keeps its cotangent, no gradient."""
    dev = _dev()
    G = _G()
    n, K = 37, 8
    say("vjp on an edgeless graph")
    dg = G.DeviceGraph.from_numpy(np.zeros(n + 1, np.int32), np.zeros(0, np.int32),
                                  np.zeros(0, np.float32), dev)
    el = G.gr_edge_list(dg)
    assert el.E == 0
    X0 = G.gr_init_vectors(n, K, 3, "f32", device=dev)
    Gc = torch.randn(n, K, device=dev)
    gw, gX = G.gr_smooth_vjp(dg, el, torch.zeros(n, dtype=torch.int32, device=dev), 1,
                             X0, Gc, 3, True)
    assert gw.numel() == 0 and torch.equal(gX, Gc)
