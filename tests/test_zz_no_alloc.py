"""The allocation-free Rayleigh-quotient entry point (gr_rq_forward_noalloc)
against the workspace entry point it mirrors (gr_rq_forward), through the
C ABI: equal bits on two calls in a row, the second smaller, in both
denominator modes; and the same values as the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import graphs as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_matches_workspace_entry_point(mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08942_amd import graphreduce as G

    dev = "cuda:0"
    rng = np.random.default_rng(21 + mode)
    # first call: 64 columns (the scratch's full width), then a smaller one
    for g, m in ((W.chung_lu(6000, mean_deg=30.0, seed=4), 64), (W.knn2d(1500, 10, seed=9), 7)):
        say(f"noalloc rq {g.name} m={m} mode={mode}")
        el = G.gr_edge_list(G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev))
        _, eu, ev = O.edge_index(g.n, g.row_ptr, g.col)
        wE = rng.uniform(0.5, 2.0, eu.size)
        U = rng.standard_normal((g.n, m))
        tw, tU = torch.from_numpy(wE).to(dev), torch.from_numpy(U).to(dev)
        R0, d0 = G.gr_rq_forward(el, tw, tU, mode)
        R = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
        den = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
        R1, d1 = G.gr_rq_forward_noalloc(el, tw, tU, mode, R=R, den=den)
        torch.cuda.synchronize()
        assert R1.data_ptr() == R.data_ptr()
        assert torch.equal(R0, R1) and torch.equal(d0, d1)
        assert np.allclose(R1.cpu().numpy(), O.rq_forward(eu, ev, wE, U, mode),
                           rtol=1e-12, atol=0)


def test_noalloc_limits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08942_amd import graphreduce as G

    assert G.gr_rq_forward_noalloc_scratch_bytes() == 3 * 512 * 64 * 8
    g = W.grid2d(6, 6)
    el = G.gr_edge_list(G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, "cuda:0"))
    U = torch.zeros((g.n, 65), dtype=torch.float64, device="cuda:0")
    w = torch.ones(el.E, dtype=torch.float64, device="cuda:0")
    with pytest.raises(RuntimeError, match="m must lie"):
        G.gr_rq_forward_noalloc(el, w, U)
