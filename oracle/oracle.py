"""Python face of the reference oracle (TEST INFRASTRUCTURE ONLY).

The loops of Phase A live in oracle.c (FP64, single thread); this module
loads them through ctypes and adds the linear-algebra parts in NumPy/SciPy:
the multilevel driver, dense Laplacian eigenvalues, Rayleigh-quotient edge
gradients and the constrained-SGD edge scaling of Alg. 1.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may use it; the
GPU library never imports it and it imports nothing from the library.

Paper: Zhao, Wang & Feng, "Nearly-Linear Time Spectral Graph Reduction for
Scalable Graph Partitioning and Data Visualization" (arXiv 1812.08942).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

from . import build as _build

_LIB = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u64 = ctypes.c_uint64


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or \
                os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.or_splitmix64.restype = _u64
        L.or_splitmix64.argtypes = [_u64, _u64]
        L.or_validate_csr.restype = ctypes.c_int
        L.or_validate_csr.argtypes = [_i64, _i32p, _i32p, _f64p]
        L.or_colour_greedy.restype = ctypes.c_int
        L.or_colour_greedy.argtypes = [_i64, _i32p, _i32p, _u64, _i32, _i32p,
                                       ctypes.POINTER(_i32)]
        L.or_validate_colouring.restype = ctypes.c_int
        L.or_validate_colouring.argtypes = [_i64, _i32p, _i32p, _i32p, _i32]
        L.or_init_vectors.restype = None
        L.or_init_vectors.argtypes = [_i64, _i32, _u64, _f64p, _i32]
        L.or_round_bf16.restype = ctypes.c_double
        L.or_round_bf16.argtypes = [ctypes.c_double]
        L.or_smooth.restype = ctypes.c_int
        L.or_smooth.argtypes = [_i64, _i32p, _i32p, _f64p, _i32p, _i32, _i32,
                                _i32, _f64p, _i32]
        L.or_affinity.restype = None
        L.or_affinity.argtypes = [_i64, _i32p, _i32p, _i32, _f64p, _f64p,
                                  ctypes.c_void_p]
        L.or_best.restype = None
        L.or_best.argtypes = [_i64, _i32p, _i32p, _f64p, _i32p]
        L.or_aggregate.restype = ctypes.c_int
        L.or_aggregate.argtypes = [_i64, _i32p, _i32p, _f64p, _i64, _i32p,
                                   _i32p, ctypes.POINTER(_i64),
                                   ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.or_galerkin.restype = ctypes.c_int
        L.or_galerkin.argtypes = [_i64, _i32p, _i32p, _f64p, _i32p, _i64,
                                  _i32p, _i32p, _f64p, ctypes.POINTER(_i64)]
        L.or_edge_index.restype = _i64
        L.or_edge_index.argtypes = [_i64, _i32p, _i32p, _i32p, _i32p, _i32p]
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [_i32]
        L.or_get_threads.restype = _i32
        L.or_get_threads.argtypes = []
        L.or_smooth_vjp.restype = ctypes.c_int
        L.or_smooth_vjp.argtypes = [_i64, _i32p, _i32p, _i32p, _i64, _f64p,
                                    _i32p, _i32, _i32, _i32, _f64p, _f64p,
                                    _f64p, _f64p]
        _LIB = L
    return _LIB


def _ai32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _af64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


# ------------------------------------------------------------------ basics

def splitmix64(seed: int, i: int) -> int:
    """Output number i of SplitMix64 seeded with `seed`."""
    return int(lib().or_splitmix64(seed & (2**64 - 1), i & (2**64 - 1)))


def level_seed(seed: int, level: int) -> int:
    """Seed of level `level` of the multilevel driver."""
    return splitmix64(seed, level)


class threads:
    """Context manager: the smoothing and affinity node loops run on `t`
    OpenMP threads inside the block (bit-identical results for any t)."""

    def __init__(self, t: int):
        self.t = int(t)

    def __enter__(self):
        self.old = int(lib().or_get_threads())
        lib().or_set_threads(self.t)
        return self

    def __exit__(self, *exc):
        lib().or_set_threads(self.old)
        return False


def validate_csr(n, row_ptr, col, w) -> int:
    return int(lib().or_validate_csr(n, _ai32(row_ptr), _ai32(col), _af64(w)))


def colour_greedy(n, row_ptr, col, seed, largest_degree_first=False):
    """Sequential greedy (first-fit) colouring in decreasing priority
    (h(v), v), or (deg(v), h(v), v) largest-degree-first; h = splitmix64
    output v of `seed`."""
    colours = np.empty(n, np.int32)
    nc = ctypes.c_int32(0)
    _check(lib().or_colour_greedy(n, _ai32(row_ptr), _ai32(col),
                                  seed & (2**64 - 1),
                                  int(largest_degree_first), colours,
                                  ctypes.byref(nc)), "colour_greedy")
    return colours, int(nc.value)


def validate_colouring(n, row_ptr, col, colours, n_colours) -> int:
    return int(lib().or_validate_colouring(n, _ai32(row_ptr), _ai32(col),
                                           _ai32(colours), n_colours))


def init_vectors(n, K, seed, centre=True):
    X = np.empty(n * K, np.float64)
    lib().or_init_vectors(n, K, seed & (2**64 - 1), X, int(centre))
    return X.reshape(n, K)


def round_bf16(x: float) -> float:
    return float(lib().or_round_bf16(float(x)))


def smooth(n, row_ptr, col, w, colours, n_colours, X, sweeps, bf16=False):
    """Returns the smoothed copy of X (float64 [n, K])."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    K = X.shape[1]
    _check(lib().or_smooth(n, _ai32(row_ptr), _ai32(col), _af64(w),
                           _ai32(colours), n_colours, K, sweeps,
                           X.reshape(-1), int(bf16)), "smooth")
    return X


def affinity(n, row_ptr, col, X, with_distance=False):
    """Per-entry affinities a (and the algebraic distances d = 1 - a)."""
    X = _af64(X)
    a = np.empty(int(row_ptr[-1]), np.float64)
    d = np.empty(int(row_ptr[-1]), np.float64) if with_distance else None
    lib().or_affinity(n, _ai32(row_ptr), _ai32(col), X.shape[1], X.reshape(-1),
                      a, d.ctypes.data if d is not None else None)
    return (a, d) if with_distance else a


def distance(n, row_ptr, col, X):
    """Algebraic distances d = 1 - a per stored entry (Sec. 3.2.2)."""
    return affinity(n, row_ptr, col, X, with_distance=True)[1]


def best(n, row_ptr, col, d):
    """Strongest neighbour: argmin (d, j)."""
    b = np.empty(n, np.int32)
    lib().or_best(n, _ai32(row_ptr), _ai32(col), _af64(d), b)
    return b


@dataclasses.dataclass
class AggResult:
    agg: np.ndarray
    n_coarse: int
    best: np.ndarray
    n_forest: int
    n_accepted: int


def aggregate(n, row_ptr, col, d, target) -> AggResult:
    """Aggregation of one level from per-entry algebraic distances `d`
    (any float array; promoted exactly to float64)."""
    agg = np.empty(n, np.int32)
    b = np.empty(n, np.int32)
    nc, nf, na = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().or_aggregate(n, _ai32(row_ptr), _ai32(col), _af64(d),
                              int(target), b, agg, ctypes.byref(nc),
                              ctypes.byref(nf), ctypes.byref(na)),
           "aggregate")
    return AggResult(agg, int(nc.value), b, int(nf.value), int(na.value))


def galerkin(n, row_ptr, col, w, agg, n_coarse):
    nnz = int(row_ptr[-1])
    c_rp = np.empty(n_coarse + 1, np.int32)
    c_col = np.empty(max(nnz, 1), np.int32)
    c_w = np.empty(max(nnz, 1), np.float64)
    nnz_c = ctypes.c_int64(0)
    _check(lib().or_galerkin(n, _ai32(row_ptr), _ai32(col), _af64(w), _ai32(agg),
                             n_coarse, c_rp, c_col, c_w, ctypes.byref(nnz_c)),
           "galerkin")
    m = int(nnz_c.value)
    return c_rp, c_col[:m].copy(), c_w[:m].copy()


def edge_index(n, row_ptr, col):
    nnz = int(row_ptr[-1])
    eoe = np.empty(max(nnz, 1), np.int32)
    eu = np.empty(max(nnz // 2, 1), np.int32)
    ev = np.empty(max(nnz // 2, 1), np.int32)
    E = int(lib().or_edge_index(n, _ai32(row_ptr), _ai32(col), eoe, eu, ev))
    return eoe[:nnz].copy(), eu[:E].copy(), ev[:E].copy()


def smooth_vjp(n, row_ptr, col, w_E, colours, n_colours, X0, G, sweeps):
    """Gradients (gw_E, gX0) of <G, X_S> with respect to the edge weights and
    the initial vectors."""
    eoe, eu, ev = edge_index(n, row_ptr, col)
    E = eu.size
    X0 = _af64(X0)
    K = X0.shape[1]
    gw = np.empty(max(E, 1), np.float64)
    gX = np.empty(n * K, np.float64)
    _check(lib().or_smooth_vjp(n, _ai32(row_ptr), _ai32(col), eoe, E, _af64(w_E),
                               _ai32(colours), n_colours, K, sweeps,
                               X0.reshape(-1), _af64(G).reshape(-1), gw, gX),
           "smooth_vjp")
    return gw[:E], gX.reshape(n, K)


# ------------------------------------------------------------- multilevel

@dataclasses.dataclass
class Level:
    n: int
    nnz: int
    n_colours: int
    n_coarse: int
    n_forest: int
    n_accepted: int


@dataclasses.dataclass
class ReduceResult:
    agg: np.ndarray          # int32 [N0] final aggregate of each fine node
    n_coarse: int
    row_ptr: np.ndarray      # coarse CSR
    col: np.ndarray
    w: np.ndarray            # float64 coarse weights
    levels: list
    no_progress: bool
    # the hierarchy (Alg. 5 input): maps[l] sends level-l nodes to level
    # l+1 nodes (H_{l+1}^{l} = P_l), graphs[l] = level l+1's CSR
    maps: list = dataclasses.field(default_factory=list)
    graphs: list = dataclasses.field(default_factory=list)


def target_size(n0: int, ratio: float) -> int:
    """Target node count T = ceil(N0 / psi) for the reduction ratio psi
    (Alg. 2 input; Table 2 prints psi as e.g. "32X")."""
    return max(1, int(math.ceil(n0 / ratio)))


def reduce(n, row_ptr, col, w, K, sweeps, ratio, vec_seed, colour_seed,
           colours=None, n_colours=0, max_levels=32, bf16=False,
           fp32_coarse=False, largest_degree_first=False) -> ReduceResult:
    """Multilevel Phase A: per level, colour (prescribed at level 0 when
    given, greedy otherwise), draw fresh test vectors, smooth, compute
    affinities, aggregate toward T = ceil(N0/psi), collapse P^T L P, and
    compose the node-to-aggregate maps; stop at T nodes or when a level makes
    no progress."""
    T = target_size(n, ratio)
    total = np.arange(n, dtype=np.int32)
    rp, cl, ww = _ai32(row_ptr), _ai32(col), _af64(w)
    cur_n = n
    levels = []
    maps, graphs = [], []
    no_progress = False
    ell = 0
    while cur_n > T and ell < max_levels:
        if ell == 0 and colours is not None:
            cols_, nc_ = _ai32(colours), int(n_colours)
        else:
            cols_, nc_ = colour_greedy(cur_n, rp, cl,
                                       level_seed(colour_seed, ell),
                                       largest_degree_first)
        X = init_vectors(cur_n, K, level_seed(vec_seed, ell))
        X = smooth(cur_n, rp, cl, ww, cols_, nc_, X, sweeps, bf16=bf16)
        d = distance(cur_n, rp, cl, X)
        ag = aggregate(cur_n, rp, cl, d, T)
        c_rp, c_col, c_w = galerkin(cur_n, rp, cl, ww, ag.agg, ag.n_coarse)
        levels.append(Level(cur_n, int(rp[-1]), nc_, ag.n_coarse,
                            ag.n_forest, ag.n_accepted))
        total = ag.agg[total]
        if ag.n_coarse == cur_n:
            no_progress = True
            break
        if fp32_coarse:
            c_w = c_w.astype(np.float32).astype(np.float64)
        maps.append(ag.agg.copy())
        graphs.append((c_rp, c_col, c_w))
        rp, cl, ww, cur_n = c_rp, c_col, c_w, ag.n_coarse
        ell += 1
    return ReduceResult(total, cur_n, rp, cl, ww, levels, no_progress, maps, graphs)


# ------------------------------------------------------- dense linear algebra

def laplacian_dense(n, row_ptr, col, w):
    """L = D - A as a dense float64 matrix (Sec. 2.1)."""
    L = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, np.int64)))
    L[rows, np.asarray(col)] = -np.asarray(w, np.float64)
    L[np.arange(n), np.arange(n)] = -L.sum(axis=1)
    return L


def prolongation_dense(agg, n_coarse):
    """P (= H_R^G), the 0/1 node-to-aggregate matrix."""
    P = np.zeros((len(agg), n_coarse))
    P[np.arange(len(agg)), agg] = 1.0
    return P


def restrict_mean(agg, n_coarse, F):
    """The reduced data set of Alg. 6, F_R = H_G^R F, with H_G^R read as the
    averaging restriction for data (row I of F_R is the mean of the rows of
    F over the nodes of aggregate I).  FP64 sums in node order, then one
    rounding to float32, as the library returns it."""
    agg = np.asarray(agg, np.int64)
    F = np.asarray(F, np.float64)
    sums = np.zeros((n_coarse, F.shape[1]))
    for v in range(agg.size):          # node order, one row at a time
        sums[agg[v]] += F[v]
    cnt = np.bincount(agg, minlength=n_coarse).astype(np.float64)
    return (sums / cnt[:, None]).astype(np.float32)


def n_components(n, row_ptr, col) -> int:
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg

    A = sp.csr_matrix((np.ones(len(col)), np.asarray(col),
                       np.asarray(row_ptr)), shape=(n, n))
    return int(cg.connected_components(A, directed=False)[0])


def laplacian_eigs(n, row_ptr, col, w, count=10, dense_limit=20000):
    """The first `count` nontrivial Laplacian eigenvalues (ascending), after
    skipping one zero per connected component."""
    ncomp = n_components(n, row_ptr, col)
    want = ncomp + count
    if n <= dense_limit:
        import scipy.linalg as sl

        L = laplacian_dense(n, row_ptr, col, w)
        hi = min(n - 1, want - 1)
        lam = sl.eigh(L, eigvals_only=True, subset_by_index=(0, hi),
                      overwrite_a=True, check_finite=False)
    else:
        import scipy.sparse as sp
        import scipy.sparse.linalg as sla

        rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, np.int64)))
        A = sp.csr_matrix((np.asarray(w, np.float64), (rows, np.asarray(col))),
                          shape=(n, n))
        L = sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A
        lam = sla.eigsh(L.tocsc(), k=want, sigma=-1e-6, which="LM",
                        tol=1e-12, return_eigenvectors=False)
        lam = np.sort(lam)
    return np.sort(lam)[ncomp:want]


def laplacian_eigpairs(n, row_ptr, col, w, count=10):
    """Dense FP64 eigenpairs (lambda_2.., u_2..) of a connected graph."""
    lam, U = np.linalg.eigh(laplacian_dense(n, row_ptr, col, w))
    return lam[1:count + 1], U[:, 1:count + 1]


# ------------------------------------------------------ Rayleigh quotients

B_IDENTITY = 0
B_DEGREE = 1


def rq_forward(eu, ev, w_E, U, mode=B_IDENTITY):
    """R_i = u_i^T L(w) u_i / u_i^T B u_i for each column u_i of U, with
    u^T L(w) u = sum_e w_e (u_p - u_q)^2 (Laplacian quadratic form) and
    B = I or B = D(w) (Alg. 4: ratio cut or normalized cut)."""
    U = _af64(U)
    diff2 = (U[eu] - U[ev]) ** 2
    Q = w_E @ diff2
    if mode == B_IDENTITY:
        Dn = np.sum(U * U, axis=0)
    else:
        Dn = w_E @ (U[eu] ** 2 + U[ev] ** 2)
    return Q / Dn


def rq_backward(eu, ev, w_E, U, gR, mode=B_IDENTITY):
    """Edge-weight gradient of sum_i gR_i R_i.  With B = I,
    dR_i/dw_e = (u_ip - u_iq)^2 / u_i^T u_i; at an eigenvector this is
    d(lambda_i)/dw_e (first-order perturbation, Sec. 3.3.3).  With B = D(w)
    the quotient rule adds -R_i (u_ip^2 + u_iq^2) / u_i^T D u_i."""
    U = _af64(U)
    diff2 = (U[eu] - U[ev]) ** 2
    if mode == B_IDENTITY:
        Dn = np.sum(U * U, axis=0)
        return diff2 @ (np.asarray(gR) / Dn)
    sq = U[eu] ** 2 + U[ev] ** 2
    Dn = w_E @ sq
    R = (w_E @ diff2) / Dn
    return (diff2 - sq * R) @ (np.asarray(gR) / Dn)
