"""Python binding of libgraphreduce (the C ABI declared in
include/graphreduce.h).

Argument marshalling only: every step runs in the HIP library.  Device arrays
are torch tensors on a ROCm device; the current torch stream is passed as the
hipStream_t.  Functions keep the C names; the `reduce` helper wraps
gr_reduce with output allocation.  If the library is not built, importing
this module raises ImportError — there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphreduce.so")

GR_OK = 0
GR_ENOMEM = -4
GR_F32 = 0
GR_BF16 = 1
GR_VALIDATE = 1
GR_COLOUR_LDF = 2
GR_WNOPROGRESS = 1
GR_RQ_IDENTITY = 0
GR_RQ_DEGREE = 1


class gr_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class gr_params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("ratio", ctypes.c_double), ("vec_seed", ctypes.c_uint64),
                ("colour_seed", ctypes.c_uint64), ("vec_dtype", ctypes.c_int32),
                ("colours", ctypes.c_void_p), ("n_colours", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class gr_result(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_void_p), ("c_row_ptr", ctypes.c_void_p),
                ("c_col", ctypes.c_void_p), ("c_w", ctypes.c_void_p),
                ("n_coarse", ctypes.c_int64), ("nnz_coarse", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("warnings", ctypes.c_uint32),
                ("level_n", ctypes.c_int64 * 32),
                ("level_nnz", ctypes.c_int64 * 32),
                ("level_colours", ctypes.c_int32 * 32)]


class gr_profile(ctypes.Structure):
    _fields_ = [("phase_ms", ctypes.c_double * 8),
                ("phase_max_ms", ctypes.c_double * 8),
                ("phase_bytes", ctypes.c_double * 8),
                ("phase_launches", ctypes.c_int64 * 8),
                ("records", ctypes.c_int64)]


GR_SGD_MAX_ITER = 64


class gr_sgd_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("eta_scale", ctypes.c_double),
                ("eps", ctypes.c_double), ("delta_bar", ctypes.c_double),
                ("k_max", ctypes.c_int32), ("t", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("cg_max_iter", ctypes.c_int32),
                ("cg_tol", ctypes.c_double)]


class gr_eig_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("block", ctypes.c_int32),
                ("residual", ctypes.c_double),
                ("lambda_max_bound", ctypes.c_double),
                ("cholesky_warnings", ctypes.c_int32),
                ("method", ctypes.c_int32), ("restarts", ctypes.c_int32)]


GR_MAX_LEVELS = 32


class gr_hierarchy(ctypes.Structure):
    _fields_ = [("maps", ctypes.c_void_p), ("maps_cap", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("rp_cap", ctypes.c_int64),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("ent_cap", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("n", ctypes.c_int64 * (GR_MAX_LEVELS + 1)),
                ("nnz", ctypes.c_int64 * (GR_MAX_LEVELS + 1)),
                ("maps_off", ctypes.c_int64 * GR_MAX_LEVELS),
                ("rp_off", ctypes.c_int64 * GR_MAX_LEVELS),
                ("ent_off", ctypes.c_int64 * GR_MAX_LEVELS)]


class gr_sgd_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("n_lambda", ctypes.c_int32),
                ("cg_iterations_max", ctypes.c_int32),
                ("lambda_n", ctypes.c_double * GR_SGD_MAX_ITER),
                ("lambda_1", ctypes.c_double * (GR_SGD_MAX_ITER + 1))]


GR_SPARSIFY_MAX_ROUNDS = 64


class gr_sparsify_params(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("add_frac", ctypes.c_double), ("lambda_target", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("cg_max_iter", ctypes.c_int32),
                ("cg_tol", ctypes.c_double)]


class gr_sparsify_report(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("n_lambda", ctypes.c_int32),
                ("tree_edges", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("cg_iterations_max", ctypes.c_int32),
                ("lambda_n", ctypes.c_double * (GR_SPARSIFY_MAX_ROUNDS + 1))]


class gr_flow_params(ctypes.Structure):
    _fields_ = [("phase_a", gr_params), ("phase_b", gr_sparsify_params),
                ("scaling", gr_sgd_params), ("gamma_max", ctypes.c_double)]


class gr_flow_result(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_void_p), ("s_row_ptr", ctypes.c_void_p),
                ("s_col", ctypes.c_void_p), ("s_w", ctypes.c_void_p),
                ("n_s", ctypes.c_int64), ("nnz_s", ctypes.c_int64),
                ("dense", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("levels", ctypes.c_int32), ("warnings", ctypes.c_uint32),
                ("sparsify", gr_sparsify_report), ("scaling", gr_sgd_report)]


PHASES = ("colour", "relabel", "init", "smooth", "affinity", "aggregate",
          "galerkin", "other")


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_G = ctypes.POINTER(gr_graph)

_SIGNATURES = {
    "gr_version": ([], ctypes.c_int),
    "gr_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "gr_last_error": ([], ctypes.c_char_p),
    "gr_workspace_size": ([_I64, _I64, _I32, _I32, ctypes.POINTER(_SZ)],
                          ctypes.c_int),
    "gr_reduce": ([_G, ctypes.POINTER(gr_params), ctypes.POINTER(gr_result),
                   _P, _SZ, _P], ctypes.c_int),
    "gr_validate": ([_G, _P, _SZ, _P], ctypes.c_int),
    "gr_profile_start": ([], ctypes.c_int),
    "gr_profile_stop": ([ctypes.POINTER(gr_profile)], ctypes.c_int),
    "gr_colour_greedy": ([_G, _U64, _I32, _P, ctypes.POINTER(_I32), _P, _SZ,
                          _P], ctypes.c_int),
    "gr_init_vectors": ([_I64, _I32, _U64, _I32, _P, _P, _SZ, _P],
                        ctypes.c_int),
    "gr_smooth": ([_G, _P, _I32, _I32, _I32, _I32, _P, _P, _SZ, _P],
                  ctypes.c_int),
    "gr_affinity": ([_G, _I32, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P],
                    ctypes.c_int),
    "gr_aggregate": ([_G, _P, _I64, _P, ctypes.POINTER(_I64), _P, _SZ, _P],
                     ctypes.c_int),
    "gr_galerkin": ([_G, _P, _I64, _P, _P, _P, ctypes.POINTER(_I64), _P, _SZ,
                     _P], ctypes.c_int),
    "gr_restrict_workspace": ([_I64, _I64, _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_restrict_mean": ([_P, _I64, _I64, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "gr_edge_list": ([_G, _P, _P, _P, ctypes.POINTER(_I64), _P, _SZ, _P],
                     ctypes.c_int),
    "gr_rq_forward": ([_I64, _I64, _P, _P, _P, _P, _I32, _I32, _P, _P, _P,
                       _SZ, _P], ctypes.c_int),
    "gr_rq_backward": ([_I64, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _P],
                       ctypes.c_int),
    "gr_rq_forward_noalloc": ([_I64, _I64, _P, _P, _P, _P, _I32, _I32, _P, _P,
                               _P], ctypes.c_int),
    "gr_rq_forward_noalloc_scratch_bytes": ([], _SZ),
    "gr_eig_workspace": ([_I64, _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_reduce_hierarchy": ([_G, ctypes.POINTER(gr_params), ctypes.POINTER(gr_result),
                             ctypes.POINTER(gr_hierarchy), _P, _SZ, _P], ctypes.c_int),
    "gr_laplacian_geigpairs": ([_G, _P, _I32, _I32, ctypes.c_double, _I32, _I32, _U64,
                                ctypes.POINTER(ctypes.c_double), _P,
                                ctypes.POINTER(gr_eig_report), _P, _SZ, _P], ctypes.c_int),
    "gr_jacobi_workspace": ([_I64, _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_jacobi_filter": ([_G, _I32, _P, ctypes.POINTER(ctypes.c_double), _P,
                          ctypes.c_double, _I32, _P, _SZ, _P], ctypes.c_int),
    "gr_orthonormalize_workspace": ([_I64, _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_orthonormalize": ([_I64, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "gr_multilevel_workspace": ([_I64, _I64, _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_multilevel_eigs": ([_G, ctypes.POINTER(gr_hierarchy), _I32, _I32, ctypes.c_double,
                            _I32, ctypes.c_double, _I32, _U64,
                            ctypes.POINTER(ctypes.c_double), _P,
                            ctypes.POINTER(gr_eig_report), _P, _SZ, _P], ctypes.c_int),
    "gr_laplacian_eigs": ([_G, _I32, _I32, ctypes.c_double, _I32, _I32, _U64,
                           ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(gr_eig_report), _P, _SZ, _P],
                          ctypes.c_int),
    "gr_laplacian_eigpairs": ([_G, _I32, _I32, ctypes.c_double, _I32, _I32, _U64,
                               ctypes.POINTER(ctypes.c_double), _P,
                               ctypes.POINTER(gr_eig_report), _P, _SZ, _P],
                              ctypes.c_int),
    "gr_sgd_workspace": ([_I64, _I64, _I64, _I64, ctypes.POINTER(_SZ)],
                         ctypes.c_int),
    "gr_sgd_scale": ([_G, _G, _P, _I64, _P, _P, _P,
                      ctypes.POINTER(gr_sgd_params),
                      ctypes.POINTER(gr_sgd_report), _P, _SZ, _P], ctypes.c_int),
    "gr_expand_edge_weights": ([_P, _I64, _I64, _P, _P, _P], ctypes.c_int),
    "gr_sparsify_workspace": ([_I64, _I64, ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_spanning_forest": ([_G, _P, ctypes.POINTER(_I64), _P, _SZ, _P], ctypes.c_int),
    "gr_sparsify": ([_G, ctypes.POINTER(gr_sparsify_params), _P, _P,
                     ctypes.POINTER(gr_sparsify_report), _P, _SZ, _P], ctypes.c_int),
    "gr_subgraph": ([_G, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_I64),
                     ctypes.POINTER(_I64), _P, _SZ, _P], ctypes.c_int),
    "gr_spectral_reduce_workspace": ([_I64, _I64, _I32, _I32, ctypes.POINTER(_SZ)],
                                     ctypes.c_int),
    "gr_spectral_reduce": ([_G, ctypes.POINTER(gr_flow_params), ctypes.POINTER(gr_flow_result),
                            _P, _SZ, _P], ctypes.c_int),
    "gr_smooth_vjp_workspace": ([_I64, _I64, _I32, _I32, _I32, _I32,
                                 ctypes.POINTER(_SZ)], ctypes.c_int),
    "gr_smooth_vjp": ([_G, _P, _I64, _P, _I32, _I32, _I32, _I32, _P, _P, _P,
                       _P, _I32, _P, _SZ, _P], ctypes.c_int),
}

_lib = None


def load():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def exported_symbols():
    return sorted(_SIGNATURES)


class GraphReduceError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc):
    if rc != GR_OK:
        L = load()
        raise GraphReduceError(rc, (L.gr_last_error() or b"").decode()
                               or L.gr_status_string(rc).decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ graphs

@dataclasses.dataclass
class DeviceGraph:
    """Symmetric CSR adjacency on the device (int32 / int32 / float32)."""

    row_ptr: torch.Tensor
    col: torch.Tensor
    w: torch.Tensor

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col.numel()

    def c(self) -> gr_graph:
        for t, dt in ((self.row_ptr, torch.int32), (self.col, torch.int32),
                      (self.w, torch.float32)):
            if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("graph arrays must be contiguous device "
                                 "int32/int32/float32 tensors")
        return gr_graph(self.n, self.nnz, self.row_ptr.data_ptr(),
                        self.col.data_ptr() if self.nnz else None,
                        self.w.data_ptr() if self.nnz else None)

    @staticmethod
    def from_numpy(row_ptr, col, w, device="cuda"):
        import numpy as np

        return DeviceGraph(
            torch.from_numpy(np.ascontiguousarray(row_ptr, np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(device))


def vec_dtype_code(dtype) -> int:
    if dtype in (GR_F32, "f32", torch.float32):
        return GR_F32
    if dtype in (GR_BF16, "bf16", torch.bfloat16):
        return GR_BF16
    raise ValueError(f"unsupported vector dtype {dtype}")


def torch_dtype(code: int):
    return torch.bfloat16 if code == GR_BF16 else torch.float32


_ws_cache: dict = {}


def workspace(n, nnz, K=8, dtype=GR_F32, device="cuda") -> torch.Tensor:
    """Device workspace sized by gr_workspace_size (cached per device)."""
    nbytes = gr_workspace_size(n, nnz, K, dtype)
    key = str(torch.device(device))
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        _ws_cache.pop(key, None)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


# ------------------------------------------------------------ C functions

def gr_version() -> int:
    return load().gr_version()


def gr_status_string(code: int) -> str:
    return load().gr_status_string(code).decode()


def gr_last_error() -> str:
    return (load().gr_last_error() or b"").decode()


def gr_profile_start():
    _check(load().gr_profile_start())


def gr_profile_stop() -> dict:
    """Per-phase HIP-event totals recorded since gr_profile_start."""
    pr = gr_profile()
    _check(load().gr_profile_stop(ctypes.byref(pr)))
    return {name: {"ms": pr.phase_ms[i], "max_ms": pr.phase_max_ms[i],
                   "bytes": pr.phase_bytes[i],
                   "launches": int(pr.phase_launches[i])}
            for i, name in enumerate(PHASES)}


def gr_workspace_size(n, nnz, K, dtype=GR_F32) -> int:
    out = _SZ(0)
    _check(load().gr_workspace_size(n, nnz, K, vec_dtype_code(dtype),
                                    ctypes.byref(out)))
    return int(out.value)


def gr_validate(g: DeviceGraph, ws=None):
    ws = ws if ws is not None else workspace(g.n, g.nnz)
    cg = g.c()
    _check(load().gr_validate(ctypes.byref(cg), _ptr(ws), ws.numel(),
                              _stream()))


def gr_colour_greedy(g: DeviceGraph, seed: int, largest_degree_first=False,
                     ws=None):
    ws = ws if ws is not None else workspace(g.n, g.nnz)
    colours = torch.empty(max(g.n, 1), dtype=torch.int32,
                          device=g.row_ptr.device)
    nc = _I32(0)
    cg = g.c()
    _check(load().gr_colour_greedy(ctypes.byref(cg), seed & (2**64 - 1),
                                   int(bool(largest_degree_first)),
                                   _ptr(colours), ctypes.byref(nc), _ptr(ws),
                                   ws.numel(), _stream()))
    return colours[:g.n], int(nc.value)


def gr_init_vectors(n, K, seed, dtype=GR_F32, device="cuda", ws=None):
    code = vec_dtype_code(dtype)
    ws = ws if ws is not None else workspace(n, 0, K, code, device)
    X = torch.empty((max(n, 1), K), dtype=torch_dtype(code), device=device)
    _check(load().gr_init_vectors(n, K, seed & (2**64 - 1), code, _ptr(X),
                                  _ptr(ws), ws.numel(), _stream()))
    return X[:n]


def gr_smooth(g: DeviceGraph, colours, n_colours, X, sweeps, ws=None):
    """Smooths X ([n, K] float32 or bfloat16 device tensor) in place."""
    code = vec_dtype_code(X.dtype)
    K = X.shape[1]
    ws = ws if ws is not None else workspace(g.n, g.nnz, K, code)
    if not X.is_contiguous() or X.shape[0] != g.n:
        raise ValueError("X must be a contiguous [n, K] tensor")
    cg = g.c()
    _check(load().gr_smooth(ctypes.byref(cg), _ptr(colours), n_colours, K,
                            sweeps, code, _ptr(X), _ptr(ws), ws.numel(),
                            _stream()))
    return X


def gr_affinity(g: DeviceGraph, X, want_a=True, want_d=True, ws=None):
    """Returns (a, d, best, dbest): per-entry affinities and algebraic
    distances, the strongest neighbour of each node and its distance."""
    code = vec_dtype_code(X.dtype)
    dev = g.row_ptr.device
    a = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev) \
        if want_a else None
    d = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev) \
        if want_d else None
    best = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    dbest = torch.empty(max(g.n, 1), dtype=torch.float32, device=dev)
    if not X.is_contiguous() or X.shape[0] != g.n:
        raise ValueError("X must be a contiguous [n, K] tensor")
    ws = ws if ws is not None else workspace(g.n, g.nnz, X.shape[1], code)
    cg = g.c()
    _check(load().gr_affinity(ctypes.byref(cg), X.shape[1], code, _ptr(X),
                              _ptr(a), _ptr(d), _ptr(best), _ptr(dbest),
                              _ptr(ws), ws.numel(), _stream()))
    return ((a[:g.nnz] if a is not None else None),
            (d[:g.nnz] if d is not None else None), best[:g.n], dbest[:g.n])


def gr_aggregate(g: DeviceGraph, dist, target, ws=None):
    """Aggregation from per-entry algebraic distances `dist`."""
    ws = ws if ws is not None else workspace(g.n, g.nnz)
    agg = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.row_ptr.device)
    nc = _I64(0)
    cg = g.c()
    _check(load().gr_aggregate(ctypes.byref(cg), _ptr(dist), int(target),
                               _ptr(agg), ctypes.byref(nc), _ptr(ws),
                               ws.numel(), _stream()))
    return agg[:g.n], int(nc.value)


def gr_galerkin(g: DeviceGraph, agg, n_coarse, ws=None):
    ws = ws if ws is not None else workspace(g.n, g.nnz)
    dev = g.row_ptr.device
    c_rp = torch.empty(n_coarse + 1, dtype=torch.int32, device=dev)
    c_col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    c_w = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev)
    m = _I64(0)
    cg = g.c()
    _check(load().gr_galerkin(ctypes.byref(cg), _ptr(agg), int(n_coarse),
                              _ptr(c_rp), _ptr(c_col), _ptr(c_w),
                              ctypes.byref(m), _ptr(ws), ws.numel(),
                              _stream()))
    k = int(m.value)
    return DeviceGraph(c_rp, c_col[:k].clone(), c_w[:k].clone())


def gr_restrict_workspace(n, n_coarse, d) -> int:
    out = _SZ(0)
    _check(load().gr_restrict_workspace(int(n), int(n_coarse), int(d), ctypes.byref(out)))
    return int(out.value)


def gr_restrict_mean(agg, n_coarse, F):
    """F_R (float32 [n_coarse][d]): the mean of the rows of F (float32
    [n][d], device) over each aggregate of `agg` (int32 [n], device)."""
    if F.dtype != torch.float32 or F.dim() != 2 or not F.is_contiguous():
        raise ValueError("F must be a contiguous float32 [n][d] tensor")
    if agg.dtype != torch.int32 or agg.numel() != F.shape[0]:
        raise ValueError("agg must be int32 [n]")
    n, d = F.shape
    nbytes = gr_restrict_workspace(n, n_coarse, d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=F.device)
    FR = torch.empty((max(int(n_coarse), 1), d), dtype=torch.float32, device=F.device)
    _check(load().gr_restrict_mean(_ptr(agg), n, int(n_coarse), d, _ptr(F), _ptr(FR),
                                   _ptr(ws), nbytes, _stream()))
    return FR[:int(n_coarse)]


@dataclasses.dataclass
class ReduceOut:
    agg: torch.Tensor
    coarse: DeviceGraph
    levels: int
    warnings: int
    level_n: list
    level_nnz: list
    level_colours: list
    hierarchy: "Hierarchy | None" = None


class Hierarchy:
    """The levels Alg. 5 walks: device buffers plus the gr_hierarchy
    struct that describes them (filled by gr_reduce_hierarchy, or built
    from host arrays with from_numpy)."""

    def __init__(self, maps, row_ptr, col, w):
        self.maps, self.row_ptr, self.col, self.w = maps, row_ptr, col, w
        self.h = gr_hierarchy(maps.data_ptr(), maps.numel(), row_ptr.data_ptr(),
                              row_ptr.numel(), col.data_ptr(), w.data_ptr(), col.numel(), 0)

    @classmethod
    def empty(cls, n, maps_cap, rp_cap, ent_cap, device):
        return cls(torch.empty(maps_cap, dtype=torch.int32, device=device),
                   torch.empty(rp_cap, dtype=torch.int32, device=device),
                   torch.empty(ent_cap, dtype=torch.int32, device=device),
                   torch.empty(ent_cap, dtype=torch.float32, device=device))

    @classmethod
    def from_numpy(cls, n0, maps, graphs, device):
        """maps[l] (level l -> l+1) and graphs[l] = (row_ptr, col, w) of
        level l+1, as host arrays."""
        import numpy as np

        cat = lambda xs, dt: torch.from_numpy(  # noqa: E731
            np.concatenate([np.asarray(x, dt) for x in xs]) if xs else np.zeros(1, dt)).to(device)
        h = cls(cat(maps, np.int32), cat([gr[0] for gr in graphs], np.int32),
                cat([gr[1] for gr in graphs], np.int32), cat([gr[2] for gr in graphs], np.float32))
        h.h.levels = len(maps)
        h.h.n[0] = n0
        om = orp = oe = 0
        for l, (m, gr) in enumerate(zip(maps, graphs)):
            h.h.maps_off[l], h.h.rp_off[l], h.h.ent_off[l] = om, orp, oe
            h.h.n[l + 1] = len(gr[0]) - 1
            h.h.nnz[l + 1] = len(gr[1])
            om += len(m)
            orp += len(gr[0])
            oe += len(gr[1])
        return h

    @property
    def levels(self) -> int:
        return int(self.h.levels)

    @property
    def n(self) -> list:
        return [int(x) for x in self.h.n[:self.levels + 1]]

    def level(self, l):
        """(map of level l, (row_ptr, col, w) of level l + 1) as device views."""
        h = self.h
        n0, n1, m1 = int(h.n[l]), int(h.n[l + 1]), int(h.nnz[l + 1])
        mo, ro, eo = int(h.maps_off[l]), int(h.rp_off[l]), int(h.ent_off[l])
        return (self.maps[mo:mo + n0],
                (self.row_ptr[ro:ro + n1 + 1], self.col[eo:eo + m1], self.w[eo:eo + m1]))

    def graph(self, l) -> "DeviceGraph":
        """Level l >= 1 as a DeviceGraph."""
        _, (rp, col, w) = self.level(l - 1)
        return DeviceGraph(rp, col, w)


def gr_reduce(g: DeviceGraph, K, sweeps, ratio, vec_seed, colour_seed,
              dtype=GR_F32, colours=None, n_colours=0, max_levels=0,
              validate=False, largest_degree_first=False, ws=None,
              out=None, keep_hierarchy=False) -> ReduceOut:
    """graph_reduce(csr, K, sweeps, ratio) -> aggregate ids + coarse CSR;
    with keep_hierarchy, gr_reduce_hierarchy also keeps every level's map
    and graph (ReduceOut.hierarchy)."""
    code = vec_dtype_code(dtype)
    ws = ws if ws is not None else workspace(g.n, g.nnz, K, code)
    dev = g.row_ptr.device
    if out is None:
        out = (torch.empty(max(g.n, 1), dtype=torch.int32, device=dev),
               torch.empty(g.n + 1, dtype=torch.int32, device=dev),
               torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev),
               torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev))
    agg, c_rp, c_col, c_w = out
    p = gr_params(K, sweeps, float(ratio), vec_seed & (2**64 - 1),
                  colour_seed & (2**64 - 1), code,
                  colours.data_ptr() if colours is not None else None,
                  int(n_colours), int(max_levels),
                  (GR_VALIDATE if validate else 0)
                  | (GR_COLOUR_LDF if largest_degree_first else 0))
    r = gr_result(agg.data_ptr(), c_rp.data_ptr(), c_col.data_ptr(),
                  c_w.data_ptr())
    cg = g.c()
    hier = None
    if keep_hierarchy:
        caps = (2 * g.n + 64, 2 * g.n + 128, g.nnz + 1024)
        while True:
            hier = Hierarchy.empty(g.n, *caps, device=dev)
            rc = load().gr_reduce_hierarchy(ctypes.byref(cg), ctypes.byref(p), ctypes.byref(r),
                                            ctypes.byref(hier.h), _ptr(ws), ws.numel(),
                                            _stream())
            if rc != GR_ENOMEM or caps[0] > 64 * (g.n + 64):
                _check(rc)
                break
            caps = tuple(2 * c for c in caps)
        hier.h.n[0] = g.n
    else:
        _check(load().gr_reduce(ctypes.byref(cg), ctypes.byref(p), ctypes.byref(r),
                                _ptr(ws), ws.numel(), _stream()))
    nc, m = int(r.n_coarse), int(r.nnz_coarse)
    L = int(r.levels)
    return ReduceOut(agg[:g.n], DeviceGraph(c_rp[:nc + 1], c_col[:m], c_w[:m]),
                     L, int(r.warnings), list(r.level_n[:min(L, 32)]),
                     list(r.level_nnz[:min(L, 32)]),
                     list(r.level_colours[:min(L, 32)]), hier)


# ------------------------------------------------------- edge derivatives

@dataclasses.dataclass
class EdgeList:
    eu: torch.Tensor              # int32 [E]
    ev: torch.Tensor              # int32 [E]
    edge_of_entry: torch.Tensor   # int32 [nnz]
    n: int

    @property
    def E(self) -> int:
        return self.eu.numel()


def gr_edge_list(g: DeviceGraph, ws=None) -> EdgeList:
    ws = ws if ws is not None else workspace(g.n, g.nnz)
    dev = g.row_ptr.device
    E0 = max(g.nnz // 2, 1)
    eu = torch.empty(E0, dtype=torch.int32, device=dev)
    ev = torch.empty(E0, dtype=torch.int32, device=dev)
    eoe = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    ne = _I64(0)
    cg = g.c()
    _check(load().gr_edge_list(ctypes.byref(cg), _ptr(eu), _ptr(ev), _ptr(eoe),
                               ctypes.byref(ne), _ptr(ws), ws.numel(),
                               _stream()))
    E = int(ne.value)
    return EdgeList(eu[:E], ev[:E], eoe[:g.nnz], g.n)


def _f64c(t):
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous float64 device tensor")
    return t


def gr_rq_forward(edges: EdgeList, w_E, U, mode=GR_RQ_IDENTITY, ws=None):
    """(R, den): Rayleigh quotients of the columns of U ([n, m] float64)."""
    _f64c(w_E)
    _f64c(U)
    n, m = U.shape
    ws = ws if ws is not None else workspace(n, 0)
    R = torch.empty(m, dtype=torch.float64, device=U.device)
    den = torch.empty(m, dtype=torch.float64, device=U.device)
    _check(load().gr_rq_forward(n, edges.E, _ptr(edges.eu), _ptr(edges.ev),
                                _ptr(w_E), _ptr(U), m, int(mode), _ptr(R),
                                _ptr(den), _ptr(ws), ws.numel(), _stream()))
    return R, den


def gr_rq_forward_noalloc(edges: EdgeList, w_E, U, mode=GR_RQ_IDENTITY, R=None,
                          den=None):
    """(R, den) as gr_rq_forward, with the library's static scratch instead
    of a workspace.  R and den may be passed in (float64 [m], on U's device)
    so that the call itself allocates nothing."""
    _f64c(w_E)
    _f64c(U)
    n, m = U.shape
    if R is None:
        R = torch.empty(m, dtype=torch.float64, device=U.device)
    if den is None:
        den = torch.empty(m, dtype=torch.float64, device=U.device)
    _check(load().gr_rq_forward_noalloc(n, edges.E, _ptr(edges.eu), _ptr(edges.ev),
                                        _ptr(w_E), _ptr(U), m, int(mode), _ptr(R),
                                        _ptr(den), _stream()))
    return R, den


def gr_rq_forward_noalloc_scratch_bytes() -> int:
    """Bytes of the static device array that gr_rq_forward_noalloc uses."""
    return int(load().gr_rq_forward_noalloc_scratch_bytes())


def gr_rq_backward(edges: EdgeList, U, R, den, gR, mode=GR_RQ_IDENTITY):
    _f64c(U)
    gR = gR.contiguous().to(torch.float64)
    gw = torch.empty(max(edges.E, 1), dtype=torch.float64, device=U.device)
    _check(load().gr_rq_backward(edges.E, _ptr(edges.eu), _ptr(edges.ev),
                                 _ptr(U), U.shape[1], int(mode), _ptr(R),
                                 _ptr(den), _ptr(gR), _ptr(gw), _stream()))
    return gw[:edges.E]


def gr_smooth_vjp_workspace(n, nnz, K, dtype, sweeps, store_states) -> int:
    out = _SZ(0)
    _check(load().gr_smooth_vjp_workspace(n, nnz, K, vec_dtype_code(dtype),
                                          sweeps, int(store_states),
                                          ctypes.byref(out)))
    return int(out.value)


def gr_smooth_vjp(g: DeviceGraph, edges: EdgeList, colours, n_colours, X0, G,
                  sweeps, store_states=False):
    """(gw_E float32[E], gX0 float32[n, K]): gradients of <G, X_S> for the
    smoothing of X0 on g (whose entry weights are w_E[edge_of_entry])."""
    code = vec_dtype_code(X0.dtype)
    n, K = X0.shape
    if G.dtype != torch.float32 or not G.is_contiguous() or not X0.is_contiguous():
        raise ValueError("X0 and G must be contiguous; G float32")
    nbytes = gr_smooth_vjp_workspace(g.n, g.nnz, K, code, sweeps, store_states)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X0.device)
    gw = torch.empty(max(edges.E, 1), dtype=torch.float32, device=X0.device)
    gX = torch.empty((max(n, 1), K), dtype=torch.float32, device=X0.device)
    cg = g.c()
    _check(load().gr_smooth_vjp(ctypes.byref(cg), _ptr(edges.edge_of_entry),
                                edges.E, _ptr(colours), n_colours, K, sweeps,
                                code, _ptr(X0), _ptr(G), _ptr(gw), _ptr(gX),
                                int(store_states), _ptr(ws), nbytes,
                                _stream()))
    return gw[:edges.E], gX[:n]


def gr_expand_edge_weights(edges: EdgeList, w_E):
    """Entry weights float32[nnz] = w_E[edge_of_entry]."""
    w_E = w_E.contiguous().to(torch.float32)
    w = torch.empty(max(edges.edge_of_entry.numel(), 1), dtype=torch.float32,
                    device=w_E.device)
    _check(load().gr_expand_edge_weights(_ptr(edges.edge_of_entry),
                                         edges.edge_of_entry.numel(), edges.E,
                                         _ptr(w_E), _ptr(w), _stream()))
    return w[:edges.edge_of_entry.numel()]


def gr_sgd_workspace(n, nnz_g, nnz_p, p_edges) -> int:
    out = _SZ(0)
    _check(load().gr_sgd_workspace(n, nnz_g, nnz_p, p_edges, ctypes.byref(out)))
    return int(out.value)


def gr_sgd_scale(G_graph: DeviceGraph, P_graph: DeviceGraph, p_edges: EdgeList,
                 w_P, alpha=0.9, eta_scale=0.1, eps=1e-3, delta_bar=0.5,
                 k_max=20, t=2, seed=1, cg_max_iter=0, cg_tol=0.0):
    """Alg. 1 edge scaling: scales w_P (float64 [E_P], device) in place;
    returns the report as a dict."""
    _f64c(w_P)
    nbytes = gr_sgd_workspace(G_graph.n, G_graph.nnz, P_graph.nnz, p_edges.E)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=w_P.device)
    prm = gr_sgd_params(alpha, eta_scale, eps, delta_bar, k_max, t,
                        seed & (2**64 - 1), cg_max_iter, cg_tol)
    rep = gr_sgd_report()
    cgG, cgP = G_graph.c(), P_graph.c()
    _check(load().gr_sgd_scale(ctypes.byref(cgG), ctypes.byref(cgP),
                               _ptr(p_edges.edge_of_entry), p_edges.E,
                               _ptr(p_edges.eu), _ptr(p_edges.ev), _ptr(w_P),
                               ctypes.byref(prm), ctypes.byref(rep), _ptr(ws),
                               nbytes, _stream()))
    return {"iterations": int(rep.iterations),
            "lambda_n": list(rep.lambda_n[:rep.n_lambda]),
            "lambda_1": list(rep.lambda_1[:rep.iterations + 1]),
            "cg_iterations_max": int(rep.cg_iterations_max)}


# ------------------------------------------------------------ Phase B

def gr_sparsify_workspace(n, nnz) -> int:
    out = _SZ(0)
    _check(load().gr_sparsify_workspace(n, nnz, ctypes.byref(out)))
    return int(out.value)


def gr_spanning_forest(g: DeviceGraph):
    """(in_tree int32 [E] device, number of forest edges)."""
    dev = g.row_ptr.device
    nb = gr_sparsify_workspace(g.n, g.nnz)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    flags = torch.empty(max(g.nnz // 2, 1), dtype=torch.int32, device=dev)
    nt = _I64(0)
    cg = g.c()
    _check(load().gr_spanning_forest(ctypes.byref(cg), _ptr(flags), ctypes.byref(nt), _ptr(ws),
                                     nb, _stream()))
    return flags[:g.nnz // 2], int(nt.value)


def _sparsify_params(t=2, rounds=5, add_frac=0.02, lambda_target=0.0, seed=1,
                     cg_max_iter=0, cg_tol=0.0):
    return gr_sparsify_params(int(t), int(rounds), float(add_frac), float(lambda_target),
                              seed & (2**64 - 1), int(cg_max_iter), float(cg_tol))


def _sparsify_report(r):
    return {"rounds": int(r.rounds), "tree_edges": int(r.tree_edges), "edges": int(r.edges),
            "lambda_n": list(r.lambda_n[:r.n_lambda]),
            "cg_iterations_max": int(r.cg_iterations_max)}


def gr_sparsify(g: DeviceGraph, want_criticality=False, **kw):
    """Phase B's sparsifier: (in_P int32 [E], criticality float64 [E] or
    None, report dict)."""
    dev = g.row_ptr.device
    nb = gr_sparsify_workspace(g.n, g.nnz)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    E = g.nnz // 2
    flags = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    crit = torch.empty(max(E, 1), dtype=torch.float64, device=dev) if want_criticality else None
    prm = _sparsify_params(**kw)
    rep = gr_sparsify_report()
    cg = g.c()
    _check(load().gr_sparsify(ctypes.byref(cg), ctypes.byref(prm), _ptr(flags), _ptr(crit),
                              ctypes.byref(rep), _ptr(ws), nb, _stream()))
    return flags[:E], (crit[:E] if crit is not None else None), _sparsify_report(rep)


def gr_subgraph(g: DeviceGraph, keep):
    """(P as a DeviceGraph, P's EdgeList) for the edge flags keep."""
    dev = g.row_ptr.device
    nb = gr_sparsify_workspace(g.n, g.nnz)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    rp = torch.empty(g.n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    w = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev)
    eoe = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    eu = torch.empty(max(g.nnz // 2, 1), dtype=torch.int32, device=dev)
    ev = torch.empty(max(g.nnz // 2, 1), dtype=torch.int32, device=dev)
    m, E = _I64(0), _I64(0)
    cg = g.c()
    _check(load().gr_subgraph(ctypes.byref(cg), _ptr(keep), _ptr(rp), _ptr(col), _ptr(w),
                              _ptr(eoe), _ptr(eu), _ptr(ev), ctypes.byref(m), ctypes.byref(E),
                              _ptr(ws), nb, _stream()))
    m, E = int(m.value), int(E.value)
    return DeviceGraph(rp, col[:m], w[:m]), EdgeList(eu[:E], ev[:E], eoe[:m], g.n)


def gr_spectral_reduce_workspace(n, nnz, K, dtype=GR_F32) -> int:
    nb = _SZ(0)
    _check(load().gr_spectral_reduce_workspace(n, nnz, K, vec_dtype_code(dtype), ctypes.byref(nb)))
    return int(nb.value)


@dataclasses.dataclass
class FlowOut:
    agg: torch.Tensor
    S: DeviceGraph
    dense: bool
    gamma: float
    levels: int
    warnings: int
    sparsify: dict
    scaling: dict


def gr_spectral_reduce(g: DeviceGraph, K, sweeps, ratio, vec_seed, colour_seed, dtype=GR_F32,
                       colours=None, n_colours=0, largest_degree_first=False, gamma_max=40.0,
                       sparsify=None, scaling=None) -> FlowOut:
    """Alg. 2 (Phase A and Phase B in the order the density selects);
    sparsify/scaling: keyword dicts of gr_sparsify and gr_sgd_scale."""
    code = vec_dtype_code(dtype)
    dev = g.row_ptr.device
    nb = _SZ(gr_spectral_reduce_workspace(g.n, g.nnz, K, code))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    pa = gr_params(K, sweeps, float(ratio), vec_seed & (2**64 - 1), colour_seed & (2**64 - 1),
                   code, colours.data_ptr() if colours is not None else None, int(n_colours), 0,
                   GR_COLOUR_LDF if largest_degree_first else 0)
    sk = dict(alpha=0.9, eta_scale=0.1, eps=1e-3, delta_bar=0.5, k_max=20, t=2, seed=1,
              cg_max_iter=0, cg_tol=0.0)
    sk.update(scaling or {})
    ps = gr_sgd_params(sk["alpha"], sk["eta_scale"], sk["eps"], sk["delta_bar"], sk["k_max"],
                       sk["t"], sk["seed"] & (2**64 - 1), sk["cg_max_iter"], sk["cg_tol"])
    prm = gr_flow_params(pa, _sparsify_params(**(sparsify or {})), ps, float(gamma_max))
    agg = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    srp = torch.empty(g.n + 1, dtype=torch.int32, device=dev)
    scol = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    sw = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev)
    res = gr_flow_result(agg.data_ptr(), srp.data_ptr(), scol.data_ptr(), sw.data_ptr())
    cg = g.c()
    _check(load().gr_spectral_reduce(ctypes.byref(cg), ctypes.byref(prm), ctypes.byref(res),
                                     _ptr(ws), nb.value, _stream()))
    ns, ms = int(res.n_s), int(res.nnz_s)
    sc = res.scaling
    return FlowOut(agg[:g.n], DeviceGraph(srp[:ns + 1], scol[:ms], sw[:ms]), bool(res.dense),
                   float(res.gamma), int(res.levels), int(res.warnings),
                   _sparsify_report(res.sparsify),
                   {"iterations": int(sc.iterations), "lambda_n": list(sc.lambda_n[:sc.n_lambda]),
                    "lambda_1": list(sc.lambda_1[:sc.iterations + 1])})


def gr_eig_workspace(n, n_eig) -> int:
    out = _SZ(0)
    _check(load().gr_eig_workspace(n, n_eig, ctypes.byref(out)))
    return int(out.value)


GR_EIG_AUTO, GR_EIG_CHEBYSHEV, GR_EIG_LOBPCG = 0, 1, 2
EIG_METHODS = {"auto": GR_EIG_AUTO, "chebyshev": GR_EIG_CHEBYSHEV,
               "lobpcg": GR_EIG_LOBPCG}


def _eig_report(rep):
    names = {GR_EIG_CHEBYSHEV: "chebyshev", GR_EIG_LOBPCG: "lobpcg"}
    return {"iterations": int(rep.iterations), "block": int(rep.block),
            "residual": float(rep.residual),
            "lambda_max_bound": float(rep.lambda_max_bound),
            "cholesky_warnings": int(rep.cholesky_warnings),
            "method": names.get(int(rep.method), "none"),
            "restarts": int(rep.restarts)}


def gr_laplacian_eigpairs(g: DeviceGraph, n_eig=10, method="auto", tol=1e-12,
                          max_iter=1000, degree=80, seed=1):
    """As gr_laplacian_eigs, plus the eigenvectors: returns (numpy array of
    eigenvalues, float64 device tensor U [n][n_eig], report dict)."""
    import numpy as np

    nbytes = gr_eig_workspace(g.n, n_eig)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=g.row_ptr.device)
    U = torch.empty((max(g.n, 1), n_eig), dtype=torch.float64, device=g.row_ptr.device)
    out = (ctypes.c_double * n_eig)()
    rep = gr_eig_report()
    cg = g.c()
    _check(load().gr_laplacian_eigpairs(ctypes.byref(cg), n_eig, EIG_METHODS[method],
                                        float(tol), int(max_iter), int(degree),
                                        seed & (2**64 - 1), out, _ptr(U), ctypes.byref(rep),
                                        _ptr(ws), nbytes, _stream()))
    return np.array(out[:], dtype=np.float64), U[:g.n], _eig_report(rep)


def gr_laplacian_geigpairs(g: DeviceGraph, bdiag, n_eig=10, method="auto", tol=1e-12,
                           max_iter=1000, degree=80, seed=1):
    """Eigenpairs of L u = lambda B u, B = diag(bdiag) (float64 device
    tensor, or None for B = I): (numpy eigenvalues, U [n][n_eig], report)."""
    import numpy as np

    if bdiag is not None:
        _f64c(bdiag)
    nbytes = gr_eig_workspace(g.n, n_eig)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=g.row_ptr.device)
    U = torch.empty((max(g.n, 1), n_eig), dtype=torch.float64, device=g.row_ptr.device)
    out = (ctypes.c_double * n_eig)()
    rep = gr_eig_report()
    cg = g.c()
    _check(load().gr_laplacian_geigpairs(ctypes.byref(cg), _ptr(bdiag), n_eig,
                                         EIG_METHODS[method], float(tol), int(max_iter),
                                         int(degree), seed & (2**64 - 1), out, _ptr(U),
                                         ctypes.byref(rep), _ptr(ws), nbytes, _stream()))
    return np.array(out[:], dtype=np.float64), U[:g.n], _eig_report(rep)


def gr_jacobi_workspace(n, k) -> int:
    nb = _SZ(0)
    _check(load().gr_jacobi_workspace(n, k, ctypes.byref(nb)))
    return int(nb.value)


def gr_orthonormalize_workspace(n, k) -> int:
    nb = _SZ(0)
    _check(load().gr_orthonormalize_workspace(n, k, ctypes.byref(nb)))
    return int(nb.value)


def gr_multilevel_workspace(n, nnz, k) -> int:
    nb = _SZ(0)
    _check(load().gr_multilevel_workspace(n, nnz, k, ctypes.byref(nb)))
    return int(nb.value)


def gr_reduce_hierarchy(g: DeviceGraph, K, sweeps, ratio, vec_seed, colour_seed, **kw):
    """gr_reduce with the hierarchy kept (ReduceOut.hierarchy)."""
    return gr_reduce(g, K, sweeps, ratio, vec_seed, colour_seed, keep_hierarchy=True, **kw)


def gr_jacobi_filter(g: DeviceGraph, Y, lam=None, bdiag=None, theta=2.0 / 3.0, iters=4):
    """Weighted-Jacobi steps on the columns of Y (float64 [n, k], in place):
    Alg. 3 when lam is None, the shifted filter of Alg. 5 otherwise."""
    _f64c(Y)
    if bdiag is not None:
        _f64c(bdiag)
    n, k = Y.shape
    nb = _SZ(0)
    _check(load().gr_jacobi_workspace(n, k, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=Y.device)
    lam_c = (ctypes.c_double * k)(*[float(x) for x in lam]) if lam is not None else None
    cg = g.c()
    _check(load().gr_jacobi_filter(ctypes.byref(cg), k, _ptr(Y), lam_c, _ptr(bdiag),
                                   float(theta), int(iters), _ptr(ws), nb.value, _stream()))
    return Y


def gr_orthonormalize(U, bdiag=None):
    """Gram-Schmidt of [1, U] in the B inner product (U float64 [n, k], in
    place); returns U."""
    _f64c(U)
    if bdiag is not None:
        _f64c(bdiag)
    n, k = U.shape
    nb = _SZ(0)
    _check(load().gr_orthonormalize_workspace(n, k, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=U.device)
    _check(load().gr_orthonormalize(n, k, _ptr(U), _ptr(bdiag), _ptr(ws), nb.value, _stream()))
    return U


def gr_multilevel_eigs(g: DeviceGraph, hier: "Hierarchy", k=10, cut=GR_RQ_IDENTITY,
                       theta=2.0 / 3.0, iters=4, tol=1e-10, max_iter=2000, seed=1):
    """Alg. 5 on a kept hierarchy: (numpy coarsest eigenvalues, U float64
    [n, k] on the device, report dict)."""
    import numpy as np

    nb = _SZ(0)
    _check(load().gr_multilevel_workspace(g.n, g.nnz, k, ctypes.byref(nb)))
    dev = g.row_ptr.device
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    U = torch.empty((max(g.n, 1), k), dtype=torch.float64, device=dev)
    out = (ctypes.c_double * k)()
    rep = gr_eig_report()
    cg = g.c()
    _check(load().gr_multilevel_eigs(ctypes.byref(cg), ctypes.byref(hier.h), k, int(cut),
                                     float(theta), int(iters), float(tol), int(max_iter),
                                     seed & (2**64 - 1), out, _ptr(U), ctypes.byref(rep),
                                     _ptr(ws), nb.value, _stream()))
    return np.array(out[:], dtype=np.float64), U[:g.n], _eig_report(rep)


def gr_laplacian_eigs(g: DeviceGraph, n_eig=10, method="auto", tol=1e-12,
                      max_iter=1000, degree=80, seed=1):
    """The n_eig smallest Laplacian eigenvalues on the complement of the
    constant vector (FP64, GPU).  Returns (numpy array, report dict)."""
    import numpy as np

    nbytes = gr_eig_workspace(g.n, n_eig)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=g.row_ptr.device)
    out = (ctypes.c_double * n_eig)()
    rep = gr_eig_report()
    cg = g.c()
    _check(load().gr_laplacian_eigs(ctypes.byref(cg), n_eig, EIG_METHODS[method],
                                    float(tol), int(max_iter), int(degree),
                                    seed & (2**64 - 1), out, ctypes.byref(rep),
                                    _ptr(ws), nbytes, _stream()))
    return np.array(out[:], dtype=np.float64), _eig_report(rep)
