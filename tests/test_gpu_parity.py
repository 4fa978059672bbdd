"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Every case prints its name before touching the GPU.

Tolerances:
* test vectors: within one float32 rounding of the oracle's FP64 values;
* smoothed vectors (float32): |dX| <= 1e-5 * max(|X|, sum_j w|X_j| / d), the
  magnitude of the terms being averaged;
* affinities: |da| <= 1e-5 absolute (a lies in [0, 1]);
* colouring, aggregation ids, coarse structure: bit-exact;
* coarse weights: 1e-5 relative (sums of positive float32 terms).
"""
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


def _G():
    from paper_1812_08942_amd import graphreduce as G
    return G


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dgraph(g, dev):
    return _G().DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)


def small_graphs():
    return {
        "grid64": W.grid2d(64, 64),
        "grid2d_33x17_lognormal": W.grid2d(33, 17, "lognormal", 4),
        "knn2d_3000": W.knn2d(3000, 10, seed=2),
        "chunglu_20000": W.chung_lu(20000, mean_deg=40.0, seed=6),
        "grid3d_12": W.grid3d(12, seed=3),
        "er_40_isolated": W.with_isolated(W.random_weighted(40, 0.15, seed=9), 3),
    }


def _colour(g, seed=5, ldf=False):
    if g.colours is not None:
        return g.colours, g.n_colours
    return O.colour_greedy(g.n, g.row_ptr, g.col, seed, ldf)


def smooth_scale(g, X):
    """max(|X_vk|, sum_j w_vj |X_jk| / d_v) per element."""
    n = g.n
    rows = np.repeat(np.arange(n), g.degrees())
    w = g.w.astype(np.float64)
    absum = np.zeros_like(X)
    np.add.at(absum, rows, w[:, None] * np.abs(X[g.col]))
    d = np.bincount(rows, weights=w, minlength=n)
    d[d == 0] = 1.0
    return np.maximum(np.abs(X), absum / d[:, None])


# ------------------------------------------------------------------ tests

def test_validate_accepts_and_rejects():
    dev = _dev()
    G = _G()
    for name, g in small_graphs().items():
        say(f"validate {name}")
        G.gr_validate(dgraph(g, dev))
    # planted defects (prepared on the host; validation reads row_ptr first)
    g = W.path(6)
    bad = [
        ("asymmetric weight", g.row_ptr, g.col, np.where(np.arange(g.nnz) == 3, 2.0, 1.0)),
        ("self loop", g.row_ptr, np.where(np.arange(g.nnz) == 0, 0, g.col), g.w),
        ("column out of range", g.row_ptr, np.where(np.arange(g.nnz) == 2, 99, g.col), g.w),
        ("negative weight", g.row_ptr, g.col, -g.w),
        ("row_ptr not monotone", np.array([0, 1, 3, 2, 5, 9, 10]), g.col, g.w),
    ]
    # the same on a dense graph, whose rows are checked by several lanes each
    k = W.complete(40)
    swapped = k.col.copy()
    e0 = k.row_ptr[7] + 10
    swapped[e0], swapped[e0 + 1] = swapped[e0 + 1], swapped[e0]
    bad += [
        ("asymmetric weight (dense)", k.row_ptr, k.col,
         np.where(np.arange(k.nnz) == 777, 2.0, 1.0)),
        ("columns out of order (dense)", k.row_ptr, swapped, k.w),
    ]
    for what, rp, cl, w in bad:
        say(f"validate rejects {what}")
        with pytest.raises(G.GraphReduceError) as e:
            G.gr_validate(G.DeviceGraph.from_numpy(rp, cl, w, dev))
        assert e.value.code == -2, what
    say("validate accepts complete_40")
    G.gr_validate(dgraph(k, dev))


def test_init_vectors_match_oracle():
    """Bit for bit: every raw entry is an odd multiple of 2^-24 below 1 in
    magnitude, so both sides' FP64 column sums are exact (n < 2^29) whatever
    their order, the means are the same double, and each entry is one FP64
    subtraction rounded to the storage type."""
    dev = _dev()
    G = _G()
    for n, K, dt in ((5000, 8, "f32"), (1237, 16, "f32"), (999, 32, "bf16"),
                     (1, 4, "f32"), (300_001, 64, "bf16"), (70_001, 12, "f32")):
        say(f"init n={n} K={K} {dt}")
        X = G.gr_init_vectors(n, K, 1234 + n, dt, dev).float().cpu().numpy()
        ref = O.init_vectors(n, K, 1234 + n)
        if dt == "f32":
            assert np.array_equal(X, ref.astype(np.float32))
        else:
            f = ref.astype(np.float32).view(np.uint32).astype(np.uint64)
            u = (f + 0x7FFF + ((f >> 16) & 1)) & 0xFFFF0000
            want = u.astype(np.uint32).view(np.float32)
            assert np.array_equal(X, want)


def colouring_graphs():
    """The small graphs plus those that reach the colouring's other paths:
    a complete graph (every node waits on all earlier ones; colours above
    255 need the later colour windows), a power-law graph with hubs above
    degree 2048, and two graphs whose largest degree is far above the mean,
    which colour their first positions in one workgroup: a star, and K_300
    with disjoint edges (colours above 255 inside that workgroup, and the
    device-wide flow after it)."""
    gs = dict(small_graphs())
    gs["complete_300"] = W.complete(300)
    gs["chunglu_hubs_10000"] = W.chung_lu(10000, mean_deg=700.0, seed=7)
    gs["star_5000"] = W.star(5000)
    gs["clique_300_pairs"] = _clique_with_pairs(300, 5000)
    return gs


@pytest.mark.parametrize("ldf", [False, True])
def test_greedy_colouring_bit_exact(ldf):
    dev = _dev()
    G = _G()
    for name, g in colouring_graphs().items():
        say(f"colour {name} ldf={ldf}")
        c, nc = G.gr_colour_greedy(dgraph(g, dev), 777, ldf)
        rc, rnc = O.colour_greedy(g.n, g.row_ptr, g.col, 777, ldf)
        assert nc == rnc
        assert np.array_equal(c.cpu().numpy(), rc)


def test_greedy_colouring_exact_order_path(monkeypatch):
    """Largest-degree-first colouring through the exact two-key priority
    order (normally taken only when truncated sort keys tie)."""
    dev = _dev()
    G = _G()
    monkeypatch.setenv("GR_COLOUR_EXACT_ORDER", "1")
    for name, g in colouring_graphs().items():
        say(f"colour (exact order) {name}")
        c, nc = G.gr_colour_greedy(dgraph(g, dev), 4242, True)
        rc, rnc = O.colour_greedy(g.n, g.row_ptr, g.col, 4242, True)
        assert nc == rnc
        assert np.array_equal(c.cpu().numpy(), rc)


@pytest.mark.parametrize("ldf,bits", [(False, 8), (False, 13), (False, 20), (True, 13),
                                      (True, 20)])
def test_greedy_colouring_truncated_key_ties(ldf, bits, monkeypatch):
    """The priority orders sort a 32-bit key holding the degree (largest
    degree first) and the top bits of h(v), then put each run of equal keys
    in exact order; with the key cut to `bits` bits (runs of tens to
    hundreds of nodes) the colouring is still the oracle's, bit for bit."""
    dev = _dev()
    G = _G()
    monkeypatch.setenv("GR_COLOUR_KEY_BITS", str(bits))
    for name, g in colouring_graphs().items():
        say(f"colour (key of {bits} bits) {name} ldf={ldf}")
        c, nc = G.gr_colour_greedy(dgraph(g, dev), 2024, ldf)
        rc, rnc = O.colour_greedy(g.n, g.row_ptr, g.col, 2024, ldf)
        assert nc == rnc
        assert np.array_equal(c.cpu().numpy(), rc)


def test_greedy_colouring_plain_launch(monkeypatch):
    """GR_COLOUR_PLAIN_LAUNCH=1 (an ordinary launch of the waiting kernel, for
    profiling runs) colours exactly as the cooperative launch does."""
    dev = _dev()
    G = _G()
    monkeypatch.setenv("GR_COLOUR_PLAIN_LAUNCH", "1")
    for name, g in colouring_graphs().items():
        for ldf in (False, True):
            say(f"colour (plain launch) {name} ldf={ldf}")
            c, nc = G.gr_colour_greedy(dgraph(g, dev), 31, ldf)
            rc, rnc = O.colour_greedy(g.n, g.row_ptr, g.col, 31, ldf)
            assert nc == rnc
            assert np.array_equal(c.cpu().numpy(), rc)


def _clique_with_pairs(m, pairs):
    """K_m followed by `pairs` disjoint edges: the largest degree is far above
    the mean, so the colouring first runs its highest-priority positions (the
    clique, a dependence chain of m) in one workgroup."""
    iu, ju = np.triu_indices(m, 1)
    a = m + 2 * np.arange(pairs)
    u = np.concatenate([iu, a])
    v = np.concatenate([ju, a + 1])
    return W.csr_from_edges(m + 2 * pairs, u, v, np.ones(u.size, np.float32),
                            f"clique{m}+{pairs}pairs")


@pytest.mark.parametrize("which", ["complete_300", "clique_200_pairs"])
def test_colouring_wait_limit_fails_cleanly(monkeypatch, which):
    """A colouring whose waits run out reports the failure and leaves the
    device usable: GR_COLOUR_SPIN_LIMIT=1 cuts every wait to one poll (in a
    clique every node waits for the earlier ones: on the complete graph in
    the device-wide flow, on the clique with pairs in the single-workgroup
    core), then the same call without it colours as the oracle does."""
    dev = _dev()
    G = _G()
    g = W.complete(300) if which == "complete_300" else _clique_with_pairs(200, 5000)
    deg = g.degrees()
    assert (deg.max() * g.n > 16 * g.nnz) == (which != "complete_300")
    monkeypatch.setenv("GR_COLOUR_SPIN_LIMIT", "1")
    say(f"colour {which} with one poll per wait")
    with pytest.raises(G.GraphReduceError) as err:
        G.gr_colour_greedy(dgraph(g, dev), 5, True)
    assert "timed out" in str(err.value)
    monkeypatch.delenv("GR_COLOUR_SPIN_LIMIT")
    say(f"colour {which} again")
    c, nc = G.gr_colour_greedy(dgraph(g, dev), 5, True)
    rc, rnc = O.colour_greedy(g.n, g.row_ptr, g.col, 5, True)
    assert nc == rnc
    assert np.array_equal(c.cpu().numpy(), rc)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_smoothing_matches_oracle(dtype):
    dev = _dev()
    G = _G()
    graphs = dict(small_graphs())
    # hubs of degree above 2048: rows split across blocks
    graphs["chunglu_hubs_10000"] = W.chung_lu(10000, mean_deg=700.0, seed=7)
    assert graphs["chunglu_hubs_10000"].degrees().max() > 2048
    for name, g in graphs.items():
        for K in ((8, 16) if dtype == "f32" else (8, 32)):
            say(f"smooth {name} K={K} {dtype}")
            c, nc = _colour(g)
            X0 = O.init_vectors(g.n, K, 99)
            Xd = torch.from_numpy(X0).to(dev).to(
                torch.float32 if dtype == "f32" else torch.bfloat16).contiguous()
            X0q = Xd.float().cpu().numpy().astype(np.float64)
            G.gr_smooth(dgraph(g, dev), torch.from_numpy(c).to(dev), nc, Xd, 5)
            got = Xd.float().cpu().numpy()
            ref = O.smooth(g.n, g.row_ptr, g.col, g.w.astype(np.float64), c,
                           nc, X0q, 5, bf16=(dtype == "bf16"))
            scale = smooth_scale(g, ref)
            err = np.abs(got - ref)
            if dtype == "f32":
                assert np.all(err <= 1e-5 * scale + 1e-30), \
                    f"{name}: max rel {np.max(err / (scale + 1e-30))}"
            else:
                # bfloat16 storage: each stored value carries up to half an
                # ulp (2^-9 relative); allow a few ulps of the averaged terms
                assert np.all(err <= 2.0**-6 * scale + 1e-30), \
                    f"{name}: max rel {np.max(err / (scale + 1e-30))}"


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_smoothing_block_order_bit_identical(dtype, monkeypatch):
    """Colour steps with every other step's blocks in reverse order (the
    default) give the same bits as all steps in launch order: tiers of every
    width, split hub rows (kept at the front), isolated rows, odd block
    counts."""
    dev = _dev()
    G = _G()
    cases = {
        "grid3d_40": W.grid3d(40, seed=3),
        "chunglu_hubs_10000": W.chung_lu(10000, mean_deg=700.0, seed=7),
        "er_40_isolated": W.with_isolated(W.random_weighted(40, 0.15, seed=9), 3),
        "knn2d_3000": W.knn2d(3000, 10, seed=2),
    }
    for name, g in cases.items():
        c, nc = _colour(g)
        for K in ((8, 16) if dtype == "f32" else (8, 32)):
            X0 = torch.from_numpy(O.init_vectors(g.n, K, 17)).to(dev).to(
                torch.float32 if dtype == "f32" else torch.bfloat16).contiguous()
            out = {}
            for mode in ("0", "1"):
                say(f"smooth {name} K={K} {dtype} alternate={mode}")
                monkeypatch.setenv("GR_GS_ALTERNATE", mode)
                X = X0.clone()
                G.gr_smooth(dgraph(g, dev), torch.from_numpy(c).to(dev), nc, X, 3)
                torch.cuda.synchronize()
                out[mode] = X.view(torch.int16 if dtype == "bf16" else torch.int32).cpu().numpy()
            monkeypatch.delenv("GR_GS_ALTERNATE")
            assert np.array_equal(out["0"], out["1"]), name


def test_affinity_matches_oracle_and_is_symmetric():
    """a within 1e-5 absolute; the algebraic distance d = 1 - a within the
    error of its cancellation-free float32 evaluation: about 6 u / theta
    relative for rows at angle theta (u = 2^-24), i.e. |dd| <~ 4e-7 sqrt(d);
    both bit-symmetric."""
    dev = _dev()
    G = _G()
    for name, g in small_graphs().items():
        for K in (8, 16):
            say(f"affinity {name} K={K}")
            c, nc = _colour(g)
            X = O.smooth(g.n, g.row_ptr, g.col, g.w.astype(np.float64), c, nc,
                         O.init_vectors(g.n, K, 3), 5).astype(np.float32)
            a, d, best, dbest = G.gr_affinity(dgraph(g, dev),
                                              torch.from_numpy(X).to(dev))
            a = a.cpu().numpy()
            d = d.cpu().numpy()
            ra, rd = O.affinity(g.n, g.row_ptr, g.col, X.astype(np.float64),
                                with_distance=True)
            assert np.max(np.abs(a - ra)) <= 1e-5
            assert np.all(np.abs(d - rd) <= 2e-6 * np.sqrt(rd) + 1e-5 * rd + 1e-12), \
                f"{name}: worst {np.max(np.abs(d - rd) / (np.sqrt(rd) + 1e-30))}"
            rows = np.repeat(np.arange(g.n), g.degrees())
            key = rows * g.n + g.col
            pos = np.searchsorted(key, g.col.astype(np.int64) * g.n + rows)
            assert np.array_equal(a.view(np.uint32), a[pos].view(np.uint32))
            assert np.array_equal(d.view(np.uint32), d[pos].view(np.uint32))
            # best is the argmin of the GPU's own distances, ties to the
            # smaller index
            assert np.array_equal(best.cpu().numpy(),
                                  O.best(g.n, g.row_ptr, g.col, d))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_candidates_do_not_depend_on_requested_outputs(dtype):
    """best/dbest alone (the reduction's call) equal, bit for bit, those of
    the call that also returns a and d, over K of one to sixteen 16-byte
    chunks, workgroup-wide hub rows and isolated nodes (-1)."""
    dev = _dev()
    G = _G()
    graphs = dict(small_graphs())
    graphs["chunglu_hubs_10000"] = W.chung_lu(10000, mean_deg=700.0, seed=7)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    ks = (4, 16, 64) if dtype == "f32" else (8, 32, 64)
    for name, g in graphs.items():
        dg = dgraph(g, dev)
        c, nc = _colour(g)
        for K in ks:
            say(f"candidates {name} K={K} {dtype}")
            X = torch.from_numpy(O.init_vectors(g.n, K, 17)).to(dev).to(tdt).contiguous()
            G.gr_smooth(dg, torch.from_numpy(c).to(dev), nc, X, 2)
            _, d, b2, d2 = G.gr_affinity(dg, X, want_a=True, want_d=True)
            _, _, b1, d1 = G.gr_affinity(dg, X, want_a=False, want_d=False)
            assert torch.equal(b1, b2), name
            assert torch.equal(d1.view(torch.int32), d2.view(torch.int32)), name
            assert np.array_equal(b1.cpu().numpy(), O.best(g.n, g.row_ptr, g.col, d.cpu().numpy()))
            if name == "er_40_isolated":
                assert int((b1 < 0).sum()) >= 3


def test_affinity_block_order_bit_identical(monkeypatch):
    """The workgroup renumbering over the XCDs (GR_AFF_XCD_CHUNK: contiguous
    ranges, chunks of 16 and 3 blocks) changes only which XCD runs a row:
    a, d, best and dbest equal, bit for bit, those of the launch order, on
    a graph with workgroup-wide hub rows ahead of the renumbered blocks and
    on block counts that leave a ragged tail."""
    dev = _dev()
    G = _G()
    graphs = {"chunglu_hubs_10000": W.chung_lu(10000, mean_deg=700.0, seed=7),
              "grid2d_300x211": W.grid2d(300, 211, weights="lognormal", seed=5)}
    for name, g in graphs.items():
        dg = dgraph(g, dev)
        c, nc = _colour(g)
        for dtype, tdt, K in (("f32", torch.float32, 16), ("bf16", torch.bfloat16, 32)):
            say(f"affinity block order {name} {dtype}")
            X = torch.from_numpy(O.init_vectors(g.n, K, 29)).to(dev).to(tdt).contiguous()
            G.gr_smooth(dg, torch.from_numpy(c).to(dev), nc, X, 2)
            out = {}
            for chunk in ("0", "-1", "16", "3"):
                monkeypatch.setenv("GR_AFF_XCD_CHUNK", chunk)
                a, d, b, db = G.gr_affinity(dg, X, want_a=True, want_d=True)
                torch.cuda.synchronize()
                out[chunk] = [t.view(torch.int32).cpu().numpy() for t in (a, d, b, db)]
            monkeypatch.delenv("GR_AFF_XCD_CHUNK")
            for chunk in ("-1", "16", "3"):
                for ref, got in zip(out["0"], out[chunk]):
                    assert np.array_equal(ref, got), (name, dtype, chunk)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_affinity_extreme_angles(dtype):
    """Rows at angles where a rounds to 0 or 1 in float32: nearly parallel
    and nearly antiparallel pairs (d ~ 1e-8, where 1 - a would cancel),
    orthogonal pairs, a zero row, equal and opposite rows (d = 0 exactly).
    d stays within the bound of the main affinity test against the FP64
    oracle on the same stored rows, and is bit-symmetric."""
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(11)
    K = 32
    pairs = 8
    X = np.zeros((2 * pairs, K))
    for k in range(pairs):
        x = rng.standard_normal(K)
        X[2 * k] = x
        if k == 0:
            X[1] = x + 1e-4 * rng.standard_normal(K)
        elif k == 1:
            X[3] = -x + 1e-4 * rng.standard_normal(K)
        elif k == 2:
            y = rng.standard_normal(K)
            X[5] = y - (y @ x) / (x @ x) * x
        elif k == 3:
            X[7] = 0.0
        elif k == 4:
            X[9] = x
        elif k == 5:
            X[11] = -x
        elif k == 6:
            X[13] = 3.0 * x + 1e-3 * rng.standard_normal(K)
        else:
            X[15] = -0.5 * x + 1e-5 * rng.standard_normal(K)
    eu = np.arange(0, 2 * pairs, 2)
    g = W.csr_from_edges(2 * pairs, eu, eu + 1, np.ones(pairs))
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    Xd = torch.from_numpy(X).to(dev).to(tdt).contiguous()
    Xs = Xd.float().cpu().numpy().astype(np.float64)
    say(f"affinity extreme angles {dtype}")
    a, d, best, dbest = G.gr_affinity(dgraph(g, dev), Xd)
    d = d.cpu().numpy()
    ra, rd = O.affinity(g.n, g.row_ptr, g.col, Xs, with_distance=True)
    assert np.all(np.abs(d - rd) <= 2e-6 * np.sqrt(rd) + 1e-5 * rd + 1e-12), (d, rd)
    assert np.max(np.abs(a.cpu().numpy() - ra)) <= 1e-5
    assert np.array_equal(d[0::2].view(np.uint32), d[1::2].view(np.uint32))
    assert d[2 * 3] == 1.0 and a.cpu().numpy()[2 * 3] == 0.0      # zero row
    assert d[2 * 4] == 0.0 and d[2 * 5] == 0.0                     # equal, opposite
    if dtype == "f32":                                               # the cancelling cases
        assert 0 < rd[0] < 1e-6 and 0 < rd[2] < 1e-6


def test_aggregation_bit_exact_on_gpu_affinities():
    dev = _dev()
    G = _G()
    for name, g in small_graphs().items():
        say(f"aggregate {name}")
        c, nc = _colour(g)
        X = O.smooth(g.n, g.row_ptr, g.col, g.w.astype(np.float64), c, nc,
                     O.init_vectors(g.n, 8, 5), 5).astype(np.float32)
        dg = dgraph(g, dev)
        _, d, _, _ = G.gr_affinity(dg, torch.from_numpy(X).to(dev))
        dn = d.cpu().numpy()
        for T in (1, g.n // 5, g.n // 2, g.n - 1):
            T = max(1, T)
            agg, ncoarse = G.gr_aggregate(dg, d, T)
            r = O.aggregate(g.n, g.row_ptr, g.col, dn, T)
            assert ncoarse == r.n_coarse, (name, T)
            assert np.array_equal(agg.cpu().numpy(), r.agg), (name, T)


def test_aggregation_long_chain_bit_exact():
    """A path whose distances fall along it: every node's strongest neighbour
    is the next one, so the forest is one chain of 200k nodes (the pointer
    jumping runs several batches of launches)."""
    dev = _dev()
    G = _G()
    n = 200_000
    g = W.path(n)
    rows = np.repeat(np.arange(n), g.degrees())
    lo = np.minimum(rows, g.col)
    d = (1.0 - (lo + 1.0) / (n + 1.0)).astype(np.float32)   # edge {i, i+1}: decreasing in i
    dg = dgraph(g, dev)
    for T in (1, n // 3, n - 10):
        say(f"aggregate chain T={T}")
        agg, nc = G.gr_aggregate(dg, torch.from_numpy(d).to(dev), T)
        r = O.aggregate(g.n, g.row_ptr, g.col, d, T)
        assert nc == r.n_coarse and np.array_equal(agg.cpu().numpy(), r.agg), T


def test_aggregation_ties_bit_exact():
    """All-equal distances: every decision is a tie broken by index."""
    dev = _dev()
    G = _G()
    g = W.grid2d(20, 15)
    a = np.full(g.nnz, 0.5, np.float32)
    dg = dgraph(g, dev)
    for T in (1, 50, 150, 299):
        say(f"aggregate ties T={T}")
        agg, nc = G.gr_aggregate(dg, torch.from_numpy(a).to(dev), T)
        r = O.aggregate(g.n, g.row_ptr, g.col, a, T)
        assert nc == r.n_coarse and np.array_equal(agg.cpu().numpy(), r.agg)


def test_galerkin_matches_oracle():
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(3)
    for name, g in small_graphs().items():
        for nc in (1, max(1, g.n // 7), g.n):
            say(f"galerkin {name} n_c={nc}")
            agg = np.concatenate([np.arange(nc), rng.integers(0, nc, g.n - nc)])
            rng.shuffle(agg)
            agg = agg.astype(np.int32)
            cg = G.gr_galerkin(dgraph(g, dev), torch.from_numpy(agg).to(dev), nc)
            rp, cl, w = O.galerkin(g.n, g.row_ptr, g.col, g.w.astype(np.float64),
                                   agg, nc)
            assert np.array_equal(cg.row_ptr.cpu().numpy(), rp)
            assert np.array_equal(cg.col.cpu().numpy(), cl)
            assert np.allclose(cg.w.cpu().numpy(), w, rtol=1e-5, atol=0)
            assert_bitwise_symmetric(rp, cl, cg.w.cpu().numpy())


def test_galerkin_segment_classes():
    """Coarse rows of every size class of the collapse (lane groups of 16 and
    64, a workgroup in LDS, and hub rows above 2048 kept entries through the
    global sort, several of them at once), coarse ids without members, and
    a run twice: the same graph as the oracle's, bitwise-symmetric weights,
    bitwise-equal repeats."""
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(17)
    graphs = {"chunglu_20000": W.chung_lu(20000, mean_deg=40.0, seed=6),
              "grid2d_200x150": W.grid2d(200, 150, "lognormal", 8)}
    for name, g in graphs.items():
        n = g.n
        maps = {}
        # two hub aggregates (a quarter of the nodes each), the rest singletons
        a = np.arange(n, dtype=np.int64)
        perm = rng.permutation(n)
        a[perm[: n // 4]] = 0
        a[perm[n // 4: n // 2]] = 1
        rest = perm[n // 2:]
        a[rest] = 2 + np.arange(rest.size)
        maps["two_hubs"] = (a, 2 + rest.size)
        # aggregates of mixed sizes, 1 to 300 nodes, over unused ids too
        sizes = np.minimum(rng.geometric(0.05, n), 300)
        ids = np.repeat(np.arange(n), sizes)[:n]
        nc = int(ids.max()) + 1
        spread = rng.permutation(2 * nc)[:nc]          # ids with gaps
        maps["mixed_with_gaps"] = (spread[ids][rng.permutation(n)], 2 * nc)
        for mname, (agg, nc) in maps.items():
            agg = agg.astype(np.int32)
            say(f"galerkin classes {name} {mname} n_c={nc}")
            dg = dgraph(g, dev)
            da = torch.from_numpy(agg).to(dev)
            c1 = G.gr_galerkin(dg, da, nc)
            c2 = G.gr_galerkin(dg, da, nc)
            rp, cl, w = O.galerkin(g.n, g.row_ptr, g.col, g.w.astype(np.float64), agg, nc)
            assert np.array_equal(c1.row_ptr.cpu().numpy(), rp)
            assert np.array_equal(c1.col.cpu().numpy(), cl)
            assert np.allclose(c1.w.cpu().numpy(), w, rtol=1e-5, atol=0)
            assert_bitwise_symmetric(rp, cl, c1.w.cpu().numpy())
            assert torch.equal(c1.w.view(torch.int32), c2.w.view(torch.int32))


def test_galerkin_lane_counts(monkeypatch):
    """GR_GAL_LANES forces 1, 2, 4 or 8 lanes per fine row in the count and
    the placement (normally about the mean degree): every choice gives the
    oracle's coarse structure exactly, its weights within the float32 sum
    tolerance, and bitwise-symmetric weights; the placement positions do
    not depend on the lane count, so the weights agree bit for bit across
    the choices."""
    dev = _dev()
    G = _G()
    rng = np.random.default_rng(23)
    graphs = {"chunglu_20000": W.chung_lu(20000, mean_deg=40.0, seed=6),
              "grid2d_200x150": W.grid2d(200, 150, "lognormal", 8),
              "knn2d_3000": W.knn2d(3000, 10, seed=2)}
    for name, g in graphs.items():
        nc = max(1, g.n // 7)
        agg = np.concatenate([np.arange(nc), rng.integers(0, nc, g.n - nc)])
        rng.shuffle(agg)
        agg = agg.astype(np.int32)
        rp, cl, w = O.galerkin(g.n, g.row_ptr, g.col, g.w.astype(np.float64), agg, nc)
        dg = dgraph(g, dev)
        da = torch.from_numpy(agg).to(dev)
        first = None
        for lanes in ("1", "2", "4", "8"):
            say(f"galerkin lanes={lanes} {name} n_c={nc}")
            monkeypatch.setenv("GR_GAL_LANES", lanes)
            cg = G.gr_galerkin(dg, da, nc)
            torch.cuda.synchronize()
            assert np.array_equal(cg.row_ptr.cpu().numpy(), rp), (name, lanes)
            assert np.array_equal(cg.col.cpu().numpy(), cl), (name, lanes)
            cw = cg.w.cpu().numpy()
            assert np.allclose(cw, w, rtol=1e-5, atol=0), (name, lanes)
            assert_bitwise_symmetric(rp, cl, cw)
            if first is None:
                first = cw
            assert np.array_equal(cw.view(np.uint32), first.view(np.uint32)), (name, lanes)
        monkeypatch.delenv("GR_GAL_LANES")


def assert_bitwise_symmetric(rp, cl, w):
    """Both stored directions of every coarse edge carry the same bits."""
    n = rp.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    key = rows * n + cl
    assert np.all(np.diff(key) > 0)
    pos = np.searchsorted(key, cl.astype(np.int64) * n + rows)
    assert np.array_equal(key[pos], cl.astype(np.int64) * n + rows)
    assert np.array_equal(w.view(np.uint32), w[pos].view(np.uint32))


def _reduce_case(g, K, ratio, dtype="f32", ldf=False):
    dev = _dev()
    G = _G()
    dg = dgraph(g, dev)
    cols = torch.from_numpy(g.colours).to(dev) if g.colours is not None else None
    out = G.gr_reduce(dg, K, 5, ratio, 101, 202, dtype=dtype, colours=cols,
                      n_colours=g.n_colours, validate=True,
                      largest_degree_first=ldf)
    ref = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), K, 5, ratio,
                   101, 202, colours=g.colours, n_colours=g.n_colours,
                   bf16=(dtype == "bf16"), fp32_coarse=True,
                   largest_degree_first=ldf)
    return out, ref


def test_reduce_end_to_end_grid64():
    say("reduce grid64 K=8 ratio 4")
    g = W.grid2d(64, 64)
    out, ref = _reduce_case(g, 8, 4.0)
    assert out.coarse.n == ref.n_coarse == 1024
    agg = out.agg.cpu().numpy()
    assert np.array_equal(agg, ref.agg)
    assert np.array_equal(out.coarse.row_ptr.cpu().numpy(), ref.row_ptr)
    assert np.array_equal(out.coarse.col.cpu().numpy(), ref.col)
    w = out.coarse.w.cpu().numpy().astype(np.float64)
    eps_w = np.max(np.abs(w - ref.w) / ref.w)
    assert eps_w <= 1e-5
    # eigenvalue gate: identical structure, weights within eps_w relative, so
    # every Laplacian eigenvalue moves by at most eps_w relative (Loewner)
    lg = O.laplacian_eigs(out.coarse.n, ref.row_ptr, ref.col, w, 10)
    lr = O.laplacian_eigs(ref.n_coarse, ref.row_ptr, ref.col, ref.w, 10)
    assert np.all(np.abs(lg - lr) <= max(eps_w, 1e-9) * lr + 1e-12)


def partition_agreement(a, b):
    """Fraction of nodes whose aggregate, as a set of nodes, is the same in
    both labellings."""
    pairs = a.astype(np.int64) * (b.max() + 1) + b
    _, inv, cnt_pair = np.unique(pairs, return_inverse=True, return_counts=True)
    cnt_a = np.bincount(a)[a]
    cnt_b = np.bincount(b)[b]
    same = (cnt_pair[inv] == cnt_a) & (cnt_pair[inv] == cnt_b)
    return float(np.mean(same))


def check_valid_aggregation(g, agg, n_c):
    assert agg.min() == 0 and agg.max() == n_c - 1
    first = np.unique(agg, return_index=True)[1]
    assert np.all(np.diff(first) > 0)          # numbered by smallest member
    # each aggregate is connected in G
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    rows = np.repeat(np.arange(g.n), g.degrees())
    keep = agg[rows] == agg[g.col]
    A = sp.csr_matrix((np.ones(keep.sum()), (rows[keep], g.col[keep])),
                      shape=(g.n, g.n))
    ncomp = cg.connected_components(A, directed=False)[0]
    assert ncomp == n_c


@pytest.mark.parametrize("case,dtype", [("knn2d_3000", "f32"), ("chunglu_20000", "f32"),
                                        ("grid3d_12", "f32"), ("chunglu_20000", "bf16"),
                                        ("grid3d_12", "bf16")])
def test_reduce_end_to_end_multilevel(case, dtype):
    """Multilevel reduction, GPU against oracle.  Near-ties of the affinity
    argmax are decided by rounding (on the dense power-law graph nearly all
    affinities lie within 1e-4 of 1), so ids need not agree bit for bit end
    to end; the per-step decisions are pinned bit-exactly elsewhere (the
    oracle fed the GPU's affinities).  Here: the GPU result is a valid
    aggregation, its coarse graph is exactly P^T L P of its own map, and its
    first 10 nontrivial eigenvalues lambda_i agree with the oracle's (same
    seeds) within max(1e-4 lambda_i, half the range of the oracle's lambda_i
    over 5 vector seeds): where rounding flips near-ties, the GPU's
    reduction may differ from the oracle's by no more than changing the
    random test vectors does.  With bfloat16 vectors the oracle rounds every
    stored update the same way; the bfloat16 result is also reported
    against the float32 oracle's spread (the accuracy the storage format
    costs)."""
    g = small_graphs()[case]
    ratio = {"knn2d_3000": 32.0, "chunglu_20000": 33.4, "grid3d_12": 20.0}[case]
    say(f"reduce {case} ratio {ratio} {dtype}")
    out, ref = _reduce_case(g, 16, ratio, dtype)
    agg = out.agg.cpu().numpy()
    n_c = out.coarse.n
    T = O.target_size(g.n, ratio)
    assert n_c == ref.n_coarse == T or (n_c >= T and out.warnings)
    check_valid_aggregation(g, agg, n_c)
    # the coarse graph is the Galerkin product of the composed map
    rp, cl, w = O.galerkin(g.n, g.row_ptr, g.col, g.w.astype(np.float64), agg, n_c)
    assert np.array_equal(out.coarse.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(out.coarse.col.cpu().numpy(), cl)
    assert np.allclose(out.coarse.w.cpu().numpy(), w, rtol=1e-5, atol=0)
    assert_bitwise_symmetric(rp, cl, out.coarse.w.cpu().numpy())
    agree = partition_agreement(agg, ref.agg)
    print(f"[gpu-case] {case}: nodes whose aggregate equals the oracle's: {agree:.2%}")
    lam_gpu = O.laplacian_eigs(n_c, rp, cl, w, 10)
    lams = [O.laplacian_eigs(ref.n_coarse, ref.row_ptr, ref.col, ref.w, 10)]
    for s in range(1, 5):
        r = O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 16, 5, ratio,
                     101 + s, 202, colours=g.colours, n_colours=g.n_colours,
                     bf16=(dtype == "bf16"), fp32_coarse=True)
        lams.append(O.laplacian_eigs(r.n_coarse, r.row_ptr, r.col, r.w, 10))
    if dtype == "bf16":
        f32 = [O.reduce(g.n, g.row_ptr, g.col, g.w.astype(np.float64), 16, 5, ratio,
                        101 + s, 202, colours=g.colours, n_colours=g.n_colours,
                        fp32_coarse=True) for s in range(5)]
        l32 = np.array([O.laplacian_eigs(r.n_coarse, r.row_ptr, r.col, r.w, 10) for r in f32])
        dev32 = np.max(np.abs(lam_gpu - l32.mean(0)) / l32.std(0, ddof=1))
        print(f"[gpu-case] {case}: bf16 GPU eigenvalues vs the float32 oracle: "
              f"max |dlambda| = {dev32:.2f} seed standard deviations")
    lams = np.array(lams)
    spread = lams.max(0) - lams.min(0)
    gate = np.maximum(1e-4 * lams[0], 0.5 * spread)
    err = np.abs(lam_gpu - lams[0])
    print(f"[gpu-case] {case}: max |dlambda|/lambda {np.max(err / lams[0]):.3e}, "
          f"max seed range/lambda {np.max(spread / lams[0]):.3e}, "
          f"max |dlambda|/gate {np.max(err / gate):.3f}")
    assert np.all(err <= gate), (err / gate).round(3)
    if agree == 1.0:
        assert np.array_equal(agg, ref.agg)


@pytest.mark.parametrize("case", ["star_30000", "chunglu_hubs_10000"])
def test_reduce_hub_graphs(case):
    """Graphs whose hubs reach every wide path (split smoothing rows, a
    workgroup per long affinity and Galerkin row, wide colouring positions,
    one giant aggregate): the reduction is a valid aggregation, and its
    coarse graph is exactly the Galerkin product of its own map, stored
    with bitwise-symmetric weights."""
    dev = _dev()
    G = _G()
    if case == "star_30000":
        n = 30000
        rng = np.random.default_rng(3)
        g = W.csr_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n),
                             rng.uniform(0.5, 2.0, n - 1))
    else:
        g = W.chung_lu(10000, mean_deg=700.0, seed=7)
    for ldf in (False, True):
        say(f"reduce {case} ldf={ldf}")
        out = G.gr_reduce(dgraph(g, dev), 16, 5, 20.0, 31, 41, largest_degree_first=ldf)
        agg = out.agg.cpu().numpy()
        n_c = out.coarse.n
        assert n_c >= O.target_size(g.n, 20.0)
        check_valid_aggregation(g, agg, n_c)
        rp, cl, w = O.galerkin(g.n, g.row_ptr, g.col, g.w.astype(np.float64), agg, n_c)
        assert np.array_equal(out.coarse.row_ptr.cpu().numpy(), rp)
        assert np.array_equal(out.coarse.col.cpu().numpy(), cl)
        assert np.allclose(out.coarse.w.cpu().numpy(), w, rtol=1e-5, atol=0)
        assert_bitwise_symmetric(rp, cl, out.coarse.w.cpu().numpy())


def test_reduce_is_deterministic():
    dev = _dev()
    G = _G()
    g = W.chung_lu(20000, mean_deg=40.0, seed=6)
    say("reduce determinism chunglu_20000")
    dg = dgraph(g, dev)
    o1 = G.gr_reduce(dg, 16, 5, 33.4, 7, 8)
    a1 = o1.agg.clone(), o1.coarse.col.clone(), o1.coarse.w.clone()
    o2 = G.gr_reduce(dg, 16, 5, 33.4, 7, 8)
    assert torch.equal(a1[0], o2.agg)
    assert torch.equal(a1[1], o2.coarse.col)
    assert torch.equal(a1[2].view(torch.int32), o2.coarse.w.view(torch.int32))


def test_reduce_degenerate_inputs():
    dev = _dev()
    G = _G()
    say("reduce edgeless")
    g = W.csr_from_edges(7, np.zeros(0), np.zeros(0), np.zeros(0))
    out = G.gr_reduce(dgraph(g, dev), 8, 2, 2.0, 1, 1)
    assert out.warnings & G.GR_WNOPROGRESS and out.coarse.n == 7
    say("reduce ratio 1")
    g = W.path(9)
    out = G.gr_reduce(dgraph(g, dev), 8, 2, 1.0, 1, 1)
    assert out.levels == 0 and out.coarse.n == 9
    assert np.array_equal(out.agg.cpu().numpy(), np.arange(9))
    say("reduce with isolated nodes")
    g = W.with_isolated(W.cycle(10), 2)
    out = G.gr_reduce(dgraph(g, dev), 8, 2, 100.0, 1, 1)
    agg = out.agg.cpu().numpy()
    assert np.sum(agg == agg[10]) == 1 and np.sum(agg == agg[11]) == 1
    say("reduce single node")
    g = W.csr_from_edges(1, np.zeros(0), np.zeros(0), np.zeros(0))
    out = G.gr_reduce(dgraph(g, dev), 8, 2, 4.0, 1, 1)
    assert out.coarse.n == 1
