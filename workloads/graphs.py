"""Seeded synthetic graphs that stand in for the paper's workloads.

This module only builds inputs: symmetric CSR adjacency arrays (int32 row
pointers, int32 columns strictly increasing per row, float32 positive weights,
both directions stored with equal bits, no self-loops), plus the structured
colourings that a workload prescribes.  It holds none of the reduction
method's arithmetic, so the CPU oracle and the GPU library may both consume
it.

The paper's own graphs (DIMACS10 / SuiteSparse meshes and social networks,
and the USPS / MNIST data sets behind its kNN graphs) are not available; the
generators below reproduce their shapes and value distributions instead
(Section 5 lists the graph families).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    """Symmetric CSR adjacency; the Laplacian is D - A with D = row sums."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    w: np.ndarray        # float32 [nnz]
    name: str = ""
    colours: np.ndarray | None = None  # optional prescribed colouring, int32 [n]
    n_colours: int = 0

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _rng(seed: int, sub: int) -> np.random.Generator:
    return np.random.default_rng([int(seed) & 0xFFFFFFFF, int(sub)])


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray,
                   name: str = "") -> Graph:
    """Symmetric CSR from an undirected edge list with u != v and no
    duplicate pairs.  Each edge's float32 weight is stored in both
    directions."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float32)
    if u.size and (np.any(u == v) or u.min() < 0 or v.min() < 0
                   or max(u.max(), v.max()) >= n):
        raise ValueError("bad edge list")
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    ws = np.concatenate([w, w])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate edge")
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    ws = ws[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32")
    return Graph(n, row_ptr.astype(np.int32), cols, ws, name)


# ---------------------------------------------------------------- tiny zoo

def path(n: int, w: float | np.ndarray = 1.0) -> Graph:
    u = np.arange(n - 1)
    ws = np.broadcast_to(np.asarray(w, np.float32), (n - 1,))
    return csr_from_edges(n, u, u + 1, ws, f"path{n}")


def cycle(n: int, w: float = 1.0) -> Graph:
    u = np.arange(n)
    v = (u + 1) % n
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return csr_from_edges(n, lo, hi, np.full(n, w, np.float32), f"cycle{n}")


def star(n: int, w: float = 1.0) -> Graph:
    v = np.arange(1, n)
    return csr_from_edges(n, np.zeros(n - 1, np.int64), v,
                          np.full(n - 1, w, np.float32), f"star{n}")


def complete(n: int, w: float = 1.0) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju, np.full(iu.size, w, np.float32),
                          f"complete{n}")


def barbell(m: int, w: float = 1.0) -> Graph:
    """Two complete graphs K_m joined by one bridge edge."""
    iu, ju = np.triu_indices(m, 1)
    u = np.concatenate([iu, iu + m, [m - 1]])
    v = np.concatenate([ju, ju + m, [m]])
    return csr_from_edges(2 * m, u, v, np.full(u.size, w, np.float32),
                          f"barbell{m}")


def random_weighted(n: int, p: float, seed: int, connected: bool = True,
                    wlo: float = 0.5, whi: float = 2.0) -> Graph:
    """Erdos-Renyi G(n, p) with U[wlo, whi] weights; a random spanning path
    is added first when `connected`."""
    rng = _rng(seed, 7)
    adj = np.zeros((n, n), dtype=bool)
    if connected:
        perm = rng.permutation(n)
        a, b = perm[:-1], perm[1:]
        adj[np.minimum(a, b), np.maximum(a, b)] = True
    iu, ju = np.triu_indices(n, 1)
    adj[iu, ju] |= rng.random(iu.size) < p
    u, v = np.nonzero(np.triu(adj, 1))
    w = rng.uniform(wlo, whi, size=u.size).astype(np.float32)
    return csr_from_edges(n, u, v, w, f"er{n}")


def disjoint_union(a: Graph, b: Graph) -> Graph:
    ea = _edges(a)
    eb = _edges(b)
    u = np.concatenate([ea[0], eb[0] + a.n])
    v = np.concatenate([ea[1], eb[1] + a.n])
    w = np.concatenate([ea[2], eb[2]])
    return csr_from_edges(a.n + b.n, u, v, w, f"{a.name}+{b.name}")


def with_isolated(g: Graph, k: int = 1) -> Graph:
    """Appends k nodes with no edges."""
    u, v, w = _edges(g)
    return csr_from_edges(g.n + k, u, v, w, f"{g.name}+iso{k}")


def _edges(g: Graph):
    rows = np.repeat(np.arange(g.n), g.degrees())
    m = rows < g.col
    return rows[m], g.col[m].astype(np.int64), g.w[m]


def edges_upper(g: Graph):
    """(u, v, w) for each undirected edge once, u < v, in CSR order."""
    return _edges(g)


# ---------------------------------------------------------------- grids

def grid2d(nx: int, ny: int, weights: str = "unit", seed: int = 0) -> Graph:
    """4-neighbour grid, node v = x + nx*y.  Prescribed colouring is the
    checkerboard (x + y) mod 2."""
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    if weights == "unit":
        w = np.ones(u.size, np.float32)
    else:
        w = np.exp(_rng(seed, 0).standard_normal(u.size)).astype(np.float32)
    g = csr_from_edges(nx * ny, u, v, w, f"grid{nx}x{ny}")
    x = np.arange(nx * ny) % nx
    y = np.arange(nx * ny) // nx
    g.colours = ((x + y) % 2).astype(np.int32)
    g.n_colours = 2
    return g


# position of each parity triple (x&1, y&1, z&1), read as a 3-bit number
# b = 4*px + 2*py + pz, in the reflected Gray sequence 000 001 011 010 110
# 111 101 100.  Consecutive classes differ in one parity bit, so the class
# written by one colour step is a neighbour class of the next step.
GRAY_RANK = np.array([0, 1, 3, 2, 7, 6, 4, 5], dtype=np.int32)


def grid3d(n: int, seed: int = 5, weights: str = "lognormal") -> Graph:
    """n^3 grid, 7-point stencil, node v = x + n*y + n*n*z; per-edge weight
    exp(N(0,1)) (lognormal(0, 1)) stored as float32.  The prescribed
    colouring is the Gray rank of the parity triple (8 colours).

    Built directly in CSR order (neighbours -z, -y, -x, +x, +y, +z are in
    increasing id order), so it scales to 256^3 without an edge sort."""
    N = n * n * n
    rng = _rng(seed, 0)
    if weights == "lognormal":
        wx = np.exp(rng.standard_normal((n, n, n - 1))).astype(np.float32)
        wy = np.exp(rng.standard_normal((n, n - 1, n))).astype(np.float32)
        wz = np.exp(rng.standard_normal((n - 1, n, n))).astype(np.float32)
    else:
        wx = np.ones((n, n, n - 1), np.float32)
        wy = np.ones((n, n - 1, n), np.float32)
        wz = np.ones((n - 1, n, n), np.float32)
    col6 = np.full((n, n, n, 6), -1, dtype=np.int32)
    w6 = np.zeros((n, n, n, 6), dtype=np.float32)
    ids = np.arange(N, dtype=np.int32).reshape(n, n, n)  # [z, y, x]
    # -z
    col6[1:, :, :, 0] = ids[:-1]
    w6[1:, :, :, 0] = wz
    # -y
    col6[:, 1:, :, 1] = ids[:, :-1]
    w6[:, 1:, :, 1] = wy
    # -x
    col6[:, :, 1:, 2] = ids[:, :, :-1]
    w6[:, :, 1:, 2] = wx
    # +x
    col6[:, :, :-1, 3] = ids[:, :, 1:]
    w6[:, :, :-1, 3] = wx
    # +y
    col6[:, :-1, :, 4] = ids[:, 1:]
    w6[:, :-1, :, 4] = wy
    # +z
    col6[:-1, :, :, 5] = ids[1:]
    w6[:-1, :, :, 5] = wz
    del wx, wy, wz
    col6 = col6.reshape(N, 6)
    w6 = w6.reshape(N, 6)
    valid = col6 >= 0
    deg = valid.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = col6[valid]
    w = w6[valid]
    del col6, w6, valid
    g = Graph(N, row_ptr.astype(np.int32), col, w, f"grid3d_{n}")
    z, rem = np.divmod(np.arange(N, dtype=np.int64), n * n)
    y, x = np.divmod(rem, n)
    b = 4 * (x & 1) + 2 * (y & 1) + (z & 1)
    g.colours = GRAY_RANK[b]
    g.n_colours = 8
    return g


# ---------------------------------------------------------------- kNN graphs

def _knn_graph_from_points(pts: np.ndarray, k: int, nbr: np.ndarray,
                           dist: np.ndarray, name: str) -> Graph:
    """Union-symmetrised kNN graph with Gaussian weights exp(-d^2/sigma^2),
    sigma = mean of the N*k directed kNN distances."""
    n = pts.shape[0]
    sigma = float(dist.mean())
    i = np.repeat(np.arange(n, dtype=np.int64), k)
    j = nbr.reshape(-1).astype(np.int64)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo * n + hi)
    u, v = np.divmod(key, n)
    d2 = np.sum((pts[u] - pts[v]) ** 2, axis=1)
    w = np.exp(-d2 / (sigma * sigma)).astype(np.float32)
    # a weight that underflows float32 would break the positive-weight
    # contract; clamp to the smallest normal value (never hit at these sizes)
    w = np.maximum(w, np.float32(np.finfo(np.float32).tiny))
    return csr_from_edges(n, u, v, w, name)


def knn2d(n: int = 200_000, k: int = 10, seed: int = 1) -> Graph:
    """n points uniform in [0,1)^2 (float64), exact k-nearest neighbours."""
    from scipy.spatial import cKDTree

    pts = _rng(seed, 0).random((n, 2))
    tree = cKDTree(pts)
    dist, nbr = tree.query(pts, k=k + 1)
    # column 0 is the point itself (distinct random points, no ties at 0)
    return _knn_graph_from_points(pts, k, nbr[:, 1:], dist[:, 1:],
                                  f"knn2d_{n}")


def gmm_points(n_per: int = 7000, dim: int = 784, n_comp: int = 10,
               spread: float = 0.12, seed: int = 4) -> np.ndarray:
    """n_comp Gaussian components with identity covariance whose means are
    drawn from N(0, spread^2 I)."""
    rng = _rng(seed, 0)
    means = rng.standard_normal((n_comp, dim)) * spread
    pts = np.repeat(means, n_per, axis=0) + rng.standard_normal(
        (n_comp * n_per, dim))
    return pts


def gmm_knn(n_per: int = 7000, dim: int = 784, n_comp: int = 10,
            k: int = 10, spread: float = 0.12, seed: int = 4) -> Graph:
    """kNN graph of a Gaussian-mixture point cloud (MNIST-shaped: 70k points
    in 784 dimensions, 10 classes, at the default sizes).  Candidates come
    from float32 distances (on a GPU when one is present, else on the
    host); the k nearest are then re-ranked in float64 among the k + 8 best
    candidates, so the graph does not depend on where the candidates were
    found (float32 errors are far below the gap to the 18th candidate)."""
    import torch

    pts = gmm_points(n_per, dim, n_comp, spread, seed)
    n = pts.shape[0]
    dev = "cuda" if torch.cuda.is_available() else "cpu"
    p32 = torch.from_numpy(pts.astype(np.float32)).to(dev)
    sq = (p32 * p32).sum(1)
    kc = min(k + 8, n - 1)
    cand = np.empty((n, kc), dtype=np.int64)
    bs = 2048
    for s in range(0, n, bs):
        blk = p32[s:s + bs]
        d2 = sq[s:s + bs, None] + sq[None, :] - 2.0 * (blk @ p32.T)
        d2[torch.arange(blk.shape[0], device=dev),
           torch.arange(s, s + blk.shape[0], device=dev)] = float("inf")
        cand[s:s + bs] = torch.topk(d2, kc, dim=1, largest=False).indices.cpu().numpy()
    del p32, sq
    # exact float64 re-rank of the candidates (ties by index)
    dc = np.sqrt(np.sum((pts[:, None, :] - pts[cand]) ** 2, axis=2)) \
        if n * kc * dim < 2e8 else _rerank_blocks(pts, cand)
    order = np.lexsort((cand, dc), axis=1)[:, :k]
    nbr = np.take_along_axis(cand, order, axis=1)
    dist = np.take_along_axis(dc, order, axis=1)
    return _knn_graph_from_points(pts, k, nbr, dist, f"gmm_knn_{n}")


def _rerank_blocks(pts, cand):
    n, kc = cand.shape
    out = np.empty((n, kc))
    bs = 1024
    for s in range(0, n, bs):
        out[s:s + bs] = np.sqrt(np.sum(
            (pts[s:s + bs, None, :] - pts[cand[s:s + bs]]) ** 2, axis=2))
    return out


# ---------------------------------------------------------------- power law

def chung_lu(n: int = 434_000, mean_deg: float = 73.7, beta: float = 2.5,
             seed: int = 3, wlo: float = 0.5, whi: float = 2.0) -> Graph:
    """Chung-Lu expected-degree graph with a power-law degree tail of
    exponent beta: theta_i = c (i + i0)^(-1/(beta-1)), with c and i0 chosen
    so that mean(theta) = mean_deg and max(theta) = sqrt(sum(theta)).
    sum(theta)/2 endpoint pairs are drawn with probability proportional to
    theta; self-loops are dropped and duplicates merged.  Weights are
    U[wlo, whi] per undirected edge, float32."""
    g_exp = 1.0 / (beta - 1.0)
    total = n * mean_deg
    tmax = math.sqrt(total)
    i = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        t = (i + i0) ** (-g_exp)
        c = tmax / (i0 ** (-g_exp))
        return c * t.mean()

    lo, hi = 1e-3, 1e9  # mean_for decreases with i0 up to tmax... solve
    # mean_for(i0) is increasing in i0 (flatter profile); bisect in log space
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    c = tmax / (i0 ** (-g_exp))
    theta = c * (i + i0) ** (-g_exp)
    rng = _rng(seed, 0)
    m = int(round(theta.sum() / 2))
    cdf = np.cumsum(theta)
    cdf /= cdf[-1]
    a = np.searchsorted(cdf, rng.random(m), side="right")
    b = np.searchsorted(cdf, rng.random(m), side="right")
    np.minimum(a, n - 1, out=a)
    np.minimum(b, n - 1, out=b)
    keep = a != b
    a, b = a[keep], b[keep]
    key = np.unique(np.minimum(a, b).astype(np.int64) * n + np.maximum(a, b))
    u, v = np.divmod(key, n)
    w = _rng(seed, 1).uniform(wlo, whi, size=u.size).astype(np.float32)
    return csr_from_edges(n, u, v, w, f"chung_lu_{n}")


# ----------------------------------------------------- subgraph for Alg. 1

def spanning_sparsifier(n, eu, ev, w, frac=0.1):
    """A spectrally similar subgraph P for tests: the maximum-weight spanning
    forest (Kruskal, ties by edge index) plus the heaviest `frac` of the
    remaining edges.  Returns the indices of the chosen edges, ascending."""
    order = np.lexsort((np.arange(len(w)), -np.asarray(w)))
    par = np.arange(n)

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    tree = np.zeros(len(w), bool)
    for e in order:
        a, b = find(eu[e]), find(ev[e])
        if a != b:
            par[max(a, b)] = min(a, b)
            tree[e] = True
    rest = order[~tree[order]]
    extra = rest[:int(round(frac * len(rest)))]
    keep = np.zeros(len(w), bool)
    keep[tree] = True
    keep[extra] = True
    return np.nonzero(keep)[0]


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic configuration: graph recipe plus reduction parameters."""

    key: str
    description: str
    K: int
    sweeps: int
    ratio: float
    dtype: str          # "f32" or "bf16" storage of the test vectors
    vec_seed: int
    colour_seed: int
    ldf: bool = False   # greedy colouring in largest-degree-first order


WORKLOADS = {
    "grid64": Workload(
        "grid64", "2-D grid 64x64, 4-neighbour, unit weights, "
        "checkerboard colouring", 8, 5, 4.0, "f32", 11, 21),
    "knn200k": Workload(
        "knn200k", "kNN (k=10) graph of 200k uniform points in [0,1)^2, "
        "Gaussian weights", 16, 5, 32.0, "f32", 12, 22),
    "chunglu434k": Workload(
        "chunglu434k", "Chung-Lu power-law graph, 434k nodes, mean degree "
        "73.7, exponent 2.5, weights U[0.5,2]", 16, 5, 434000.0 / 13000.0,
        "f32", 13, 23, ldf=True),
    "gmm70k": Workload(
        "gmm70k", "kNN (k=10) graph of a 10-component Gaussian mixture, "
        "70k points in 784-d", 16, 5, 16.0, "f32", 14, 24),
    "grid256": Workload(
        "grid256", "3-D grid 256^3, 7-point stencil, lognormal(0,1) "
        "weights, 8-colour Gray parity colouring", 32, 5, 170.0, "bf16",
        15, 25),
}


def build_graph(key: str, scale: float = 1.0) -> Graph:
    """Graph of a workload; `scale` < 1 gives a smaller graph of the same
    family for tests."""
    if key == "grid64":
        return grid2d(64, 64)
    if key == "knn200k":
        return knn2d(max(64, int(200_000 * scale)), 10, seed=1)
    if key == "chunglu434k":
        nn = max(256, int(434_000 * scale))
        return chung_lu(nn, mean_deg=min(73.7, nn / 8), seed=3)
    if key == "gmm70k":
        per = max(20, int(7000 * scale))
        return gmm_knn(per, 784, 10, 10, seed=4)
    if key == "grid256":
        side = max(4, int(round(256 * scale ** (1 / 3))))
        return grid3d(side, seed=5)
    raise KeyError(key)
