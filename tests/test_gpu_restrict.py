"""The data restriction of Alg. 6, F_R = H_G^R F (the mean of F over each
aggregate), on the GPU against the oracle: bit for bit where every
aggregate has at most 256 members (the same FP64 sums in node order),
within one float32 rounding where a large aggregate is summed in pieces,
plus the degenerate maps, the error paths, and the final maps of the
benchmark's reductions."""
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


def _run(agg, nc, F):
    dev = _dev()
    G = _G()
    R = G.gr_restrict_mean(torch.from_numpy(agg).to(dev), nc,
                           torch.from_numpy(F).to(dev).contiguous())
    return R.cpu().numpy()


def _ragged_map(n, nc, rng):
    agg = np.concatenate([np.arange(nc), rng.integers(0, nc, n - nc)]).astype(np.int32)
    rng.shuffle(agg)
    return agg


@pytest.mark.parametrize("n,nc,d", [(1, 1, 1), (5000, 300, 7), (20000, 4000, 33)])
def test_restrict_small_aggregates_bit_exact(n, nc, d):
    rng = np.random.default_rng(n + d)
    agg = _ragged_map(n, nc, rng)
    assert np.bincount(agg).max() <= 256
    F = rng.standard_normal((n, d)).astype(np.float32)
    say(f"restrict n={n} n_coarse={nc} d={d}")
    assert np.array_equal(_run(agg, nc, F), O.restrict_mean(agg, nc, F))


def test_restrict_large_aggregates_in_pieces():
    """An aggregate of 3000 members (12 pieces) and one of 257 (2 pieces)
    among small ones: within one float32 rounding of the oracle."""
    rng = np.random.default_rng(5)
    n, nc, d = 12000, 500, 64
    agg = _ragged_map(n - 3257, nc - 2, rng)
    agg = np.concatenate([agg, np.full(3000, nc - 2, np.int32), np.full(257, nc - 1, np.int32)])
    rng.shuffle(agg)
    F = (rng.standard_normal((n, d)) * 10.0).astype(np.float32)
    say(f"restrict with aggregates of 3000 and 257 members, d={d}")
    R, ref = _run(agg, nc, F), O.restrict_mean(agg, nc, F)
    assert np.all(np.abs(R - ref) <= np.spacing(np.abs(ref)))
    small = np.bincount(agg, minlength=nc) <= 256
    assert np.array_equal(R[small], ref[small])


def test_restrict_degenerate_maps():
    rng = np.random.default_rng(9)
    n, d = 100000, 3
    F = rng.standard_normal((n, d)).astype(np.float32)
    say("restrict with the identity map")
    assert np.array_equal(_run(np.arange(n, dtype=np.int32), n, F), F)
    say("restrict with one aggregate of 100000 members")
    R = _run(np.zeros(n, np.int32), 1, F)
    ref = O.restrict_mean(np.zeros(n, np.int32), 1, F)
    assert np.all(np.abs(R - ref) <= np.spacing(np.abs(ref)))


def test_restrict_rejects_bad_maps():
    G = _G()
    F = np.ones((10, 2), np.float32)
    say("restrict with an id out of range")
    with pytest.raises(G.GraphReduceError) as e:
        _run(np.array([0, 1, 2, 3, 4, 0, 1, 2, 3, 5], np.int32), 5, F)
    assert "outside" in str(e.value)
    say("restrict with an empty aggregate")
    with pytest.raises(G.GraphReduceError) as e:
        _run(np.array([0, 1, 2, 3, 0, 0, 1, 2, 3, 0], np.int32), 5, F)
    assert "no member" in str(e.value)


def test_restrict_with_the_map_of_a_reduction():
    """The composed map of a multilevel reduction (hub aggregates included)."""
    dev = _dev()
    G = _G()
    g = W.chung_lu(20000, mean_deg=30.0, seed=4)
    dg = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    say("reduce chunglu_20000 for its aggregate map")
    out = G.gr_reduce(dg, 8, 5, 20.0, 1, 2, largest_degree_first=True)
    agg, nc = out.agg.cpu().numpy(), out.coarse.n
    F = np.random.default_rng(2).standard_normal((g.n, 16)).astype(np.float32)
    say(f"restrict to {nc} aggregates (largest {np.bincount(agg).max()} members)")
    R, ref = _run(agg, nc, F), O.restrict_mean(agg, nc, F)
    assert np.all(np.abs(R - ref) <= np.spacing(np.abs(ref)))


def _sampled_reference(agg, F, ids):
    """The oracle on the members of aggregates `ids` only (node order kept)."""
    sel = np.isin(agg, ids)
    remap = np.full(agg.max() + 1, -1, np.int64)
    remap[ids] = np.arange(ids.size)
    return O.restrict_mean(remap[agg[sel]].astype(np.int32), ids.size, F[sel])


@pytest.mark.parametrize("key", ["chunglu434k", "grid256"])
def test_restrict_full_size_maps(key):
    """The final map of the benchmark's reduction of each workload (power
    law: 434,000 nodes into 13,000; grid: 16.8M nodes into 98,690), data of
    32 columns; the grid is checked on 2,000 sampled aggregates and the
    largest one."""
    dev = _dev()
    G = _G()
    wl = W.WORKLOADS[key]
    g = W.build_graph(key)
    dg = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    colours = torch.from_numpy(g.colours).to(dev) if g.colours is not None else None
    say(f"reduce {key} for its aggregate map")
    out = G.gr_reduce(dg, wl.K, wl.sweeps, wl.ratio, wl.vec_seed, wl.colour_seed,
                      dtype=G.vec_dtype_code(wl.dtype), colours=colours,
                      n_colours=g.n_colours if colours is not None else 0,
                      largest_degree_first=True)
    agg, nc = out.agg.cpu().numpy(), out.coarse.n
    del out, dg
    F = np.random.default_rng(7).standard_normal((g.n, 32)).astype(np.float32)
    say(f"restrict {key}: {g.n} nodes into {nc} aggregates")
    R = _run(agg, nc, F)
    if g.n <= 1_000_000:
        ref = O.restrict_mean(agg, nc, F)
        assert np.all(np.abs(R - ref) <= np.spacing(np.abs(ref)))
    else:
        cnt = np.bincount(agg, minlength=nc)
        ids = np.unique(np.concatenate([
            np.random.default_rng(3).choice(nc, 2000, replace=False), [cnt.argmax()]]))
        ref = _sampled_reference(agg, F, ids)
        assert np.all(np.abs(R[ids] - ref) <= np.spacing(np.abs(ref)))
