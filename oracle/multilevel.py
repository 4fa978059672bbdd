"""Reference for the solution refinement by weighted Jacobi (Alg. 3,
Sec. 3.5) and the multilevel Laplacian eigensolver (Alg. 5, Sec. 4.1).

TEST INFRASTRUCTURE ONLY: plain FP64 NumPy/SciPy, used to check the GPU
library; the library never imports it.

Alg. 3 (refinement): each approximate solution x is filtered N_iter times
by  x <- (1 - theta) x + theta D^-1 A x,  with L = D - A.

Alg. 5 (multilevel eigensolver), in the algorithm's order:
  1. the first k eigenpairs (lambda_i, u_i) of the coarsest problem
     L^Y u = lambda B^Y u;
  2. from level j = Y down to 2: U^{j-1} = H_j^{j-1} U^j, then every column
     y = U^{j-1}[:, i] is filtered by a few weighted-Jacobi steps on
     (L^{j-1} - lambda_i B^{j-1}) y = 0;
  3. the columns of U^1 are orthonormalised by Gram-Schmidt.

Readings (the paper fixes none of these):
  * The hierarchy is the multilevel Phase A: level 1 is G, level j+1 is
    P_j^T L_j P_j, and H_{j+1}^{j} = P_j, the 0/1 node-to-aggregate map
    (the Laplacian reading of H used throughout).
  * B on the coarse levels.  With a 0/1 prolongation the coarse Laplacians
    grow with the aggregate sizes, so a single set of lambda_i can only
    serve every level if each level's B is the one the prolongation
    induces: B^{j+1} = P_j^T B^j P_j, which is diagonal again (the sum of
    B^1 over the fine nodes of each aggregate).  Then a coarse vector's
    quotient x^T L^j x / x^T B^j x equals that of its prolongation to the
    finest level, and the coarsest lambda_i are upper bounds of the fine
    ones (Poincare separation).  B^1 = I for ratio cut (the fine B of
    Alg. 5), so B^j counts the fine nodes of each aggregate; B^1 = D_G for
    normalized cut.
  * "Weighted Jacobi on (L - lambda B) y = 0" keeps the Laplacian's own
    diagonal as the Jacobi diagonal:  y <- y - theta D^-1 (L - lambda B) y.
    With lambda = 0 this is Alg. 3's step exactly; unlike the diagonal of
    L - lambda B it never vanishes or changes sign.  Rows with d = 0
    (isolated nodes) are left unchanged.
  * theta = 2/3 (the classical damping for Laplacian smoothing) and 4
    iterations per level unless given.
  * The eigenpairs are the nontrivial ones (lambda_2 .. lambda_{k+1}); the
    Gram-Schmidt process runs over [1, u_1, .., u_k] in the B^1 inner
    product and drops the constant, so the result is B^1-orthonormal and
    B^1-orthogonal to the all-one vector, the convention of the GPU
    eigensolver.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import oracle as O

RATIO_CUT = 0
NORMALIZED_CUT = 1


def _rows(rp):
    rp = np.asarray(rp, np.int64)
    return np.repeat(np.arange(rp.size - 1), np.diff(rp))


def laplacian_apply(rp, col, w, Y):
    """L Y for L = D - A given as CSR adjacency (row by row, FP64)."""
    Y = np.asarray(Y, np.float64)
    rows = _rows(rp)
    w = np.asarray(w, np.float64)
    AY = np.zeros_like(Y)
    np.add.at(AY, rows, w[:, None] * Y[np.asarray(col)])
    d = np.bincount(rows, w, minlength=Y.shape[0])
    return d[:, None] * Y - AY


def degrees(rp, w, n):
    return np.bincount(_rows(rp), np.asarray(w, np.float64), minlength=n)


def jacobi_filter(rp, col, w, Y, theta=2.0 / 3.0, iters=4, lam=None, bdiag=None):
    """`iters` weighted-Jacobi steps y <- y - theta D^-1 (L - lam_i B) y on
    every column i of Y (n x k).  lam = None is Alg. 3 (lam = 0); bdiag is
    the diagonal of B (None = I)."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    n, k = Y.shape
    d = degrees(rp, w, n)
    safe = np.where(d > 0, d, 1.0)
    lamv = np.zeros(k) if lam is None else np.asarray(lam, np.float64)
    b = np.ones(n) if bdiag is None else np.asarray(bdiag, np.float64)
    for _ in range(iters):
        R = laplacian_apply(rp, col, w, Y) - (b[:, None] * Y) * lamv[None, :]
        Y = np.where(d[:, None] > 0, Y - theta * R / safe[:, None], Y)
    return Y


def alg3_step_by_definition(rp, col, w, x, theta):
    """One step of Alg. 3 exactly as written: (1 - theta) x + theta D^-1 A x."""
    x = np.asarray(x, np.float64)
    n = x.size
    rows = _rows(rp)
    Ax = np.bincount(rows, np.asarray(w, np.float64) * x[np.asarray(col)], minlength=n)
    d = degrees(rp, w, n)
    return (1.0 - theta) * x + theta * Ax / np.where(d > 0, d, 1.0)


def mass_hierarchy(n, rp, w, maps, cut=RATIO_CUT):
    """B^1 (I or D_G) and B^{j+1} = P_j^T B^j P_j for every level."""
    b = np.ones(n) if cut == RATIO_CUT else degrees(rp, w, n)
    out = [b]
    for agg in maps:
        nc = int(np.max(agg)) + 1 if len(agg) else 0
        out.append(np.bincount(np.asarray(agg), out[-1], minlength=nc))
    return out


def generalized_eigpairs(n, rp, col, w, bdiag, k):
    """The k smallest nontrivial eigenpairs of L u = lambda B u (B diagonal,
    positive) on a connected graph, dense FP64; u^T B u = 1."""
    import scipy.linalg as sl

    L = O.laplacian_dense(n, rp, col, w)
    lam, U = sl.eigh(L, np.diag(np.asarray(bdiag, np.float64)))
    return lam[1:k + 1], U[:, 1:k + 1]


def gram_schmidt(U, bdiag=None):
    """Modified Gram-Schmidt over [1, u_1, .., u_k] in the B inner product;
    returns the k columns after the constant (B-orthonormal, B-orthogonal to
    the all-one vector)."""
    U = np.asarray(U, np.float64)
    n, k = U.shape
    b = np.ones(n) if bdiag is None else np.asarray(bdiag, np.float64)
    Q = np.empty((n, k + 1))
    Q[:, 0] = 1.0
    Q[:, 1:] = U
    for i in range(k + 1):
        for j in range(i):
            Q[:, i] -= (Q[:, j] @ (b * Q[:, i])) * Q[:, j]
        Q[:, i] /= np.sqrt(Q[:, i] @ (b * Q[:, i]))
    return Q[:, 1:]


@dataclasses.dataclass
class MultilevelResult:
    U: np.ndarray          # n x k, the refined eigenvectors of the finest level
    lam_coarse: np.ndarray # lambda_i of the coarsest problem
    levels: int


def multilevel_eigs(n, rp, col, w, maps, graphs, k, theta=2.0 / 3.0, iters=4,
                    cut=RATIO_CUT):
    """Alg. 5 on a hierarchy given as the oracle's reduce() returns it:
    maps[j] (level j+1 -> j+2 in the paper's 1-based numbering) and
    graphs[j] = the CSR of level j+2.  With no coarse level the finest
    problem is solved directly."""
    levels = [(rp, col, w)] + list(graphs)
    sizes = [n] + [len(g[0]) - 1 for g in graphs]
    B = mass_hierarchy(n, rp, w, maps, cut)
    crp, ccol, cw = levels[-1]
    lam, U = generalized_eigpairs(sizes[-1], crp, ccol, cw, B[-1], k)
    for j in range(len(levels) - 1, 0, -1):
        U = U[np.asarray(maps[j - 1])]                  # U^{j-1} = H_j^{j-1} U^j
        frp, fcol, fw = levels[j - 1]
        U = jacobi_filter(frp, fcol, fw, U, theta, iters, lam=lam, bdiag=B[j - 1])
    return MultilevelResult(gram_schmidt(U, B[0]), lam, len(levels))
