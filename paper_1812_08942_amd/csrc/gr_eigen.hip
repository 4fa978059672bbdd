// FP64 evaluation of the first nontrivial Laplacian eigenvalues of a graph
// (the quality measure of a reduced graph: its first eigenvalues should
// follow the original's, Sec. 5, Fig. 5).  Two block eigensolvers on the
// complement of the all-one vector, both built from the same kernels
// (Laplacian times a row-major block, block Gram products, Cholesky QR,
// Rayleigh-Ritz by parallel Jacobi in one workgroup):
//
// * Chebyshev-filtered subspace iteration: X <- T_k(L) X with the Chebyshev
//   polynomial of the interval [a, b] (a = the largest Ritz value of the
//   block, b = 2 max degree >= lambda_max), which damps [a, b] and lifts the
//   eigenvalues below a.  Fast when the spectrum is not dominated by a few
//   huge degrees (grids, k-NN graphs).
// * LOBPCG (Knyazev, SIAM J. Sci. Comput. 2001) with the Jacobi
//   preconditioner D^{-1}: Rayleigh-Ritz over [X, D^{-1} R, P].  The
//   preconditioner absorbs the degree spread of hub-heavy (power-law and
//   aggregated) graphs, on which the polynomial filter stalls.
//
// Orthonormalisation is column-scaled Cholesky QR: a shifted pass (shift
// 11 (n p + p (p + 1)) u times the trace, Fukaya et al., SIAM J. Sci.
// Comput. 2020) and two plain passes.  A block m wider than the wanted count
// resolves repeated eigenvalues (grids have pairs).  Every reduction has a
// fixed shape, so results are reproducible bit for bit.
#include "gr_internal.hpp"

#include <math.h>

#include <vector>

namespace gr {

constexpr int kE = 256;
constexpr int kMaxP = 64;  // widest block (columns)
constexpr int kGramRows = 32;
constexpr int kRowBlocks = 128;
constexpr int kJacobiThreads = 1024;

// Y[:, 0:p] = L X[:, 0:p] for row-major blocks of stride ld.  Every row is
// cut into pieces of ep consecutive entries (ep >= the mean degree, so that
// there are at most 2n pieces, and a hub row spreads over many threads): the
// first kernel writes each piece's partial sums, `lanes` threads (a power of
// two >= p) per piece, one column each; the second adds a row's pieces in
// order and applies the diagonal.  Fixed order: deterministic.
__global__ void __launch_bounds__(kE) k_spmm_pieces(const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ w,
                                                    const int32_t* __restrict__ ppos,
                                                    const int32_t* __restrict__ prow, int64_t npieces,
                                                    int32_t ep, int p, int ld, int lanes,
                                                    const double* __restrict__ X,
                                                    const double* __restrict__ sc,
                                                    double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    const int64_t k = t / lanes;
    const int c = (int)(t % lanes);
    if (k >= npieces || c >= p) return;
    const int32_t v = prow[k];
    const int32_t e0 = rp[v] + (int32_t)(k - ppos[v]) * ep;
    const int32_t e1 = min(e0 + ep, rp[v + 1]);
    double s = 0.0;
    int32_t e = e0;
    for (; e + 4 <= e1; e += 4) {  // four gathers in flight, summed in entry order
        double xv[4], wv[4];
        int32_t j[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            wv[u] = (double)w[e + u];
            j[u] = col[e + u];
            xv[u] = X[(int64_t)j[u] * ld + c];
        }
        if (sc) {
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] *= sc[j[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s = fma(wv[u], xv[u], s);
    }
    for (; e < e1; ++e) {
        const int32_t j = col[e];
        const double x = sc ? X[(int64_t)j * ld + c] * sc[j] : X[(int64_t)j * ld + c];
        s = fma((double)w[e], x, s);
    }
    part[k * p + c] = s;
}

__global__ void __launch_bounds__(kE) k_spmm_rows(const int32_t* __restrict__ ppos,
                                                  const double* __restrict__ d, int64_t n, int p,
                                                  int ld, int lanes,
                                                  const double* __restrict__ part,
                                                  const double* __restrict__ X,
                                                  const double* __restrict__ sc,
                                                  double* __restrict__ Y) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    const int64_t v = t / lanes;
    const int c = (int)(t % lanes);
    if (v >= n || c >= p) return;
    double s = 0.0;
    for (int32_t k = ppos[v]; k < ppos[v + 1]; ++k) s += part[(int64_t)k * p + c];
    if (sc)  // S L S X with S = diag(sc)
        Y[v * ld + c] = sc[v] * (d[v] * (sc[v] * X[v * ld + c]) - s);
    else
        Y[v * ld + c] = d[v] * X[v * ld + c] - s;
}

// pieces of every row, and the row of every piece
__global__ void k_piece_counts_e(const int32_t* __restrict__ rp, int64_t n, int32_t ep,
                                 int32_t* __restrict__ cnt) {
    const int64_t v = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (v < n) cnt[v] = (rp[v + 1] - rp[v] + ep - 1) / ep;
}

__global__ void k_piece_rows(const int32_t* __restrict__ ppos, int64_t n, int32_t* __restrict__ prow) {
    const int64_t v = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (v >= n) return;
    for (int32_t k = ppos[v]; k < ppos[v + 1]; ++k) prow[k] = (int32_t)v;
}

// Chebyshev step on contiguous blocks: Z = (2/e) (L Y - c Y) - Z, or
// (1/e) (L Y - c Y) for the first step
__global__ void k_cheb(const double* __restrict__ LY, const double* __restrict__ Y,
                       double* __restrict__ Z, int64_t cnt, double c, double e, int first) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= cnt) return;
    double t = (LY[i] - c * Y[i]) / e;
    Z[i] = first ? t : 2.0 * t - Z[i];
}

// a wave per row (hub rows hold thousands of entries), fixed reduction tree
__global__ void __launch_bounds__(kE) k_degree_f64(const int32_t* __restrict__ rp,
                                                   const float* __restrict__ w, int64_t n,
                                                   double* __restrict__ d,
                                                   double* __restrict__ dinv) {
    const int64_t v = ((int64_t)blockIdx.x * kE + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    double s = 0.0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave) s += (double)w[e];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) s += __shfl_xor(s, off, kWave);
    if (l == 0) {
        d[v] = s;
        dinv[v] = s > 0.0 ? 1.0 / s : 1.0;
    }
}

// uniform (-1, 1) values from the counter RNG into columns [c0, c0 + p)
__device__ inline double block_rand(uint64_t seed, int64_t v, int c) {
    uint64_t r = splitmix64(seed, (uint64_t)v * kMaxP + (uint64_t)c);
    int64_t q = (int64_t)(r >> 40);
    return (double)(2 * q + 1 - (1ll << 24)) * (1.0 / 16777216.0);
}

__global__ void k_init_block(int64_t n, int p, int ld, uint64_t seed, double* __restrict__ X) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= n * p) return;
    int64_t v = i / p;
    int c = (int)(i - v * p);
    X[v * ld + c] = block_rand(seed, v, c);
}

// replace the columns whose squared norm (diagonal of G = X^T X) vanishes by
// fresh random columns: a block method must not carry a zero direction
__global__ void k_fix_zero_cols(const double* __restrict__ G, int64_t n, int p, int ld,
                                uint64_t seed, double* __restrict__ X) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= n * p) return;
    int64_t v = i / p;
    int c = (int)(i - v * p);
    double gmax = 0.0;
    for (int k = 0; k < p; ++k) gmax = fmax(gmax, G[k * p + k]);
    const double gc = G[c * p + c];
    if (!(gc > 1e-200 * gmax)) X[v * ld + c] = block_rand(seed, v, c);
}

// per-block partial column sums of X[:, 0:p] (stride ld), weighted by q
// when q is given (the products q^T X)
__global__ void __launch_bounds__(kE) k_colsum_part(const double* __restrict__ X, int64_t n, int p,
                                                    int ld, const double* __restrict__ q,
                                                    double* __restrict__ part) {
    const int64_t R = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * R, hi = min(n, lo + R);
    for (int c = threadIdx.x; c < p; c += kE) {
        double s = 0.0;
        if (q)
            for (int64_t v = lo; v < hi; ++v) s = fma(q[v], X[v * ld + c], s);
        else
            for (int64_t v = lo; v < hi; ++v) s += X[v * ld + c];
        part[(int64_t)blockIdx.x * p + c] = s;
    }
}

// s = sum over b of part[b * stride + idx], in b order, eight loads in flight
__device__ inline double strided_sum(const double* __restrict__ part, int nb, int64_t stride,
                                     int64_t idx) {
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u) * stride + idx];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nb; ++b) s += part[(int64_t)b * stride + idx];
    return s;
}

__global__ void k_colsum_final(const double* __restrict__ part, int nb, int p, double* __restrict__ out) {
    int c = threadIdx.x;
    if (c >= p) return;
    out[c] = strided_sum(part, nb, p, c);
}

// X <- X - 1 (1^T X) / n, or X - q (q^T X) / (q^T q) when q is given
__global__ void k_sub_colmean(double* __restrict__ X, int64_t n, int p, int ld,
                              const double* __restrict__ cs, const double* __restrict__ q,
                              const double* __restrict__ qq) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= n * p) return;
    int64_t v = i / p;
    int c = (int)(i - v * p);
    if (q)
        X[v * ld + c] -= q[v] * (cs[c] / *qq);
    else
        X[v * ld + c] -= cs[c] / (double)n;
}

// per-block partials of A[:, 0:pa]^T B[:, 0:pb] (both of stride ld), rows
// staged through LDS
__global__ void __launch_bounds__(kE) k_gram_part(const double* __restrict__ A,
                                                  const double* __restrict__ B, int64_t n, int pa,
                                                  int pb, int ld, double* __restrict__ part) {
    __shared__ double sa[kGramRows * kMaxP];
    __shared__ double sb[kGramRows * kMaxP];
    const int cnt = pa * pb;
    double acc[(kMaxP * kMaxP + kE - 1) / kE];
    const int per = (cnt + kE - 1) / kE;
    for (int k = 0; k < per; ++k) acc[k] = 0.0;
    const int64_t R = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * R, hi = min(n, lo + R);
    for (int64_t r0 = lo; r0 < hi; r0 += kGramRows) {
        const int rows = (int)min((int64_t)kGramRows, hi - r0);
        __syncthreads();
        for (int i = threadIdx.x; i < rows * pa; i += kE) sa[i] = A[(r0 + i / pa) * ld + i % pa];
        for (int i = threadIdx.x; i < rows * pb; i += kE) sb[i] = B[(r0 + i / pb) * ld + i % pb];
        __syncthreads();
        for (int k = 0; k < per; ++k) {
            int idx = threadIdx.x + k * kE;
            if (idx >= cnt) break;
            int i = idx / pb, j = idx % pb;
            double s = acc[k];
            for (int r = 0; r < rows; ++r) s = fma(sa[r * pa + i], sb[r * pb + j], s);
            acc[k] = s;
        }
    }
    for (int k = 0; k < per; ++k) {
        int idx = threadIdx.x + k * kE;
        if (idx < cnt) part[(int64_t)blockIdx.x * cnt + idx] = acc[k];
    }
}

__global__ void k_gram_final(const double* __restrict__ part, int nb, int cnt, double* __restrict__ out) {
    int idx = blockIdx.x * kE + threadIdx.x;
    if (idx >= cnt) return;
    out[idx] = strided_sum(part, nb, cnt, idx);
}

// Column-scaled Cholesky QR factor: with S = diag(G)^{-1/2}, factor
// S G S + shift p I = R^T R (upper R) and return M = S R^{-1}, so that
// X M has orthonormal columns.  One workgroup of kMaxP threads: rows of R
// by left-looking steps (thread i owns column i), then thread j solves
// column j of R^{-1}.  flag[0] = 1 if the matrix is not positive definite.
__global__ void __launch_bounds__(kMaxP) k_chol_inv(const double* __restrict__ G, int p,
                                                    double shift, double* __restrict__ M,
                                                    int* __restrict__ flag) {
    __shared__ double R[kMaxP * kMaxP];
    __shared__ double Gs[kMaxP * kMaxP];  // G, staged once (row stride p)
    __shared__ double Xs[kMaxP * kMaxP];  // column t of R^{-1} in Xs[.. * kMaxP + t]
    __shared__ double sc[kMaxP];
    __shared__ double tj[kMaxP];
    const int t = threadIdx.x;
    for (int i = t; i < p * p; i += kMaxP) Gs[i] = G[i];
    __syncthreads();
    if (t < p) {
        const double g = Gs[t * p + t];
        sc[t] = g > 0.0 ? 1.0 / sqrt(g) : 1.0;
    }
    __syncthreads();
    const double sh = shift * (double)p;
    for (int j = 0; j < p; ++j) {
        double s = 0.0;
        if (t >= j && t < p) {
            s = Gs[j * p + t] * sc[j] * sc[t] + (t == j ? sh : 0.0);
            for (int k = 0; k < j; ++k) s -= R[k * kMaxP + j] * R[k * kMaxP + t];
            tj[t] = s;
        }
        __syncthreads();
        double djj = tj[j];
        if (!(djj > 0.0)) {
            if (t == j) flag[0] = 1;
            djj = 1e-300;
        }
        const double rjj = sqrt(djj);
        if (t >= j && t < p) R[j * kMaxP + t] = (t == j) ? rjj : s / rjj;
        __syncthreads();
    }
    // column t of R^{-1} by back substitution, scaled rows into M
    if (t < p) {
        for (int i = t; i >= 0; --i) {
            double s = (i == t) ? 1.0 : 0.0;
            for (int k = i + 1; k <= t; ++k) s -= R[i * kMaxP + k] * Xs[k * kMaxP + t];
            Xs[i * kMaxP + t] = s / R[i * kMaxP + i];
        }
        for (int i = 0; i < p; ++i) M[i * p + t] = i <= t ? sc[i] * Xs[i * kMaxP + t] : 0.0;
    }
}

// Y[:, 0:q] = A[:, 0:k] M[0:k, 0:q] row by row (A of stride lda, M of stride
// ldm, Y of stride ldy); Y must not overlap A
__global__ void k_right_mul(const double* __restrict__ A, int lda, int k, const double* __restrict__ M,
                            int ldm, int q, int64_t n, double* __restrict__ Y, int ldy) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= n * q) return;
    int64_t v = i / q;
    int c = (int)(i - v * q);
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(A[v * lda + j], M[j * ldm + c], s);
    Y[v * ldy + c] = s;
}

// Eigen-decomposition of the symmetric p x p matrix (H + H^T)/2 by parallel
// cyclic Jacobi (round-robin ordering: each round rotates p/2 disjoint
// pairs at once), one workgroup.  Eigenvalues ascending into theta, the
// eigenvectors into the columns of Q (p x p); V is p x p scratch.
// row stride of the LDS matrices: one double of padding, so that the column
// updates (consecutive rows, one column) fall in different banks
constexpr int kJs = kMaxP + 1;

__global__ void __launch_bounds__(kJacobiThreads) k_jacobi(const double* __restrict__ H, int p,
                                                           int max_sweeps,
                                                           double* __restrict__ theta,
                                                           double* __restrict__ Q) {
    __shared__ double A[kJs * kMaxP];
    __shared__ double V[kJs * kMaxP];  // the rotations
    __shared__ double rc[kMaxP / 2], rs[kMaxP / 2];
    __shared__ int rl[kMaxP / 2], rh[kMaxP / 2];
    __shared__ double red_off[kJacobiThreads], red_tot[kJacobiThreads];
    __shared__ int order[kMaxP];
    const int t = threadIdx.x;
    for (int i = t; i < p * p; i += kJacobiThreads) {
        int r = i / p, c = i % p;
        A[r * kJs + c] = 0.5 * (H[r * p + c] + H[c * p + r]);
        V[r * kJs + c] = (r == c) ? 1.0 : 0.0;
    }
    const int p2 = p + (p & 1);
    const int npairs = p2 / 2;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps && p > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = t; i < p * p; i += kJacobiThreads) {
            int r = i / p, c = i % p;
            double a2 = A[r * kJs + c] * A[r * kJs + c];
            tot += a2;
            if (r != c) off += a2;
        }
        red_off[t] = off;
        red_tot[t] = tot;
        __syncthreads();
        for (int s = kJacobiThreads / 2; s > 0; s >>= 1) {
            if (t < s) {
                red_off[t] += red_off[t + s];
                red_tot[t] += red_tot[t + s];
            }
            __syncthreads();
        }
        const bool done = red_off[0] <= 1e-30 * red_tot[0];
        __syncthreads();
        if (done) break;
        for (int r = 0; r < p2 - 1; ++r) {
            if (t < npairs) {
                int a, b;
                if (t == 0) {
                    a = r;
                    b = p2 - 1;
                } else {
                    a = (r + t) % (p2 - 1);
                    b = (r - t + (p2 - 1)) % (p2 - 1);
                }
                const int lo = min(a, b), hi = max(a, b);
                double c = 1.0, s = 0.0;
                if (hi < p) {
                    const double apq = A[lo * kJs + hi];
                    if (apq != 0.0) {
                        const double tau = (A[hi * kJs + hi] - A[lo * kJs + lo]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                rl[t] = lo;
                rh[t] = hi;
                rc[t] = c;
                rs[t] = s;
            }
            __syncthreads();
            // rows lo, hi of every pair (disjoint rows)
            for (int i = t; i < npairs * p; i += kJacobiThreads) {
                const int k = i / p, j = i % p;
                const double s = rs[k];
                if (s == 0.0) continue;
                const double c = rc[k];
                const int lo = rl[k], hi = rh[k];
                const double ap = A[lo * kJs + j], aq = A[hi * kJs + j];
                A[lo * kJs + j] = c * ap - s * aq;
                A[hi * kJs + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns lo, hi of every pair, in A and in V (disjoint columns)
            for (int i = t; i < npairs * p; i += kJacobiThreads) {
                const int k = i / p, j = i % p;
                const double s = rs[k];
                if (s == 0.0) continue;
                const double c = rc[k];
                const int lo = rl[k], hi = rh[k];
                const double ap = A[j * kJs + lo], aq = A[j * kJs + hi];
                A[j * kJs + lo] = c * ap - s * aq;
                A[j * kJs + hi] = s * ap + c * aq;
                const double vp = V[j * kJs + lo], vq = V[j * kJs + hi];
                V[j * kJs + lo] = c * vp - s * vq;
                V[j * kJs + hi] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        // ascending order of the diagonal (stable: ties keep index order)
        for (int i = 0; i < p; ++i) order[i] = i;
        for (int i = 1; i < p; ++i) {
            int x = order[i], j = i - 1;
            while (j >= 0 && A[order[j] * kJs + order[j]] > A[x * kJs + x]) {
                order[j + 1] = order[j];
                --j;
            }
            order[j + 1] = x;
        }
    }
    __syncthreads();
    for (int i = t; i < p * p; i += kJacobiThreads) {
        const int r = i / p, c = i % p;
        Q[r * p + c] = V[r * kJs + order[c]];
    }
    for (int i = t; i < p; i += kJacobiThreads) theta[i] = A[order[i] * kJs + order[i]];
}

// residual R = L X - X diag(theta) of the first m columns: its per-block
// partial squared column norms, and (when W is given) the preconditioned
// block W = D^{-1} R written to columns [m, 2m) of the same row
__global__ void __launch_bounds__(kE) k_resid_part(const double* __restrict__ LX,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ theta, int64_t n,
                                                   int m, int ld, double* __restrict__ part) {
    const int64_t R = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * R, hi = min(n, lo + R);
    for (int c = threadIdx.x; c < m; c += kE) {
        double s = 0.0;
        for (int64_t v = lo; v < hi; ++v) {
            double r = LX[v * ld + c] - theta[c] * X[v * ld + c];
            s = fma(r, r, s);
        }
        part[(int64_t)blockIdx.x * m + c] = s;
    }
}

__global__ void k_precond_resid(const double* __restrict__ LX, double* __restrict__ S,
                                const double* __restrict__ theta, const double* __restrict__ dinv,
                                int64_t n, int m, int ld) {
    int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i >= n * m) return;
    int64_t v = i / m;
    int c = (int)(i - v * m);
    S[v * ld + m + c] = dinv[v] * (LX[v * ld + c] - theta[c] * S[v * ld + c]);
}

__global__ void __launch_bounds__(kE) k_deg_stats(const double* __restrict__ d, int64_t n,
                                                  double* __restrict__ out) {
    __shared__ double mx[kE], sm[kE];
    double m = 0.0, s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kE) {
        m = fmax(m, d[i]);
        s += d[i];
    }
    mx[threadIdx.x] = m;
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int k = kE / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + k]);
            sm[threadIdx.x] += sm[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = mx[0];
        out[1] = sm[0];
    }
}

// ------------------------------------------------------------------ driver

struct Eig {
    const gr_graph* g;
    int64_t n;
    int ld;
    hipStream_t st;
    uint64_t seed;
    int fix_round;
    double *d, *dinv, *S, *LS, *T, *U, *part, *G, *M, *theta, *cs, *res, *small;
    int* flag;
    int32_t *ppos, *prow;  // row pieces of the Laplacian product
    double* ppart;         // their partial sums [npieces][p]
    int64_t npieces;
    int32_t ep;            // entries per piece
    // generalised problem L u = lambda B u with B = diag(b) > 0: the solver
    // works on S L S (S = diag(b)^-1/2) in the complement of q = b^1/2,
    // its null vector; u = S v.  All three NULL for B = I.
    const double* sc = nullptr;  // b^-1/2
    const double* q = nullptr;   // b^1/2
    double* qq = nullptr;        // q^T q = sum of b (device scalar)

    static int lanes_for(int p) {
        int l = 1;
        while (l < p) l <<= 1;
        return l;
    }
    // B[:, 0:p] = L A[:, 0:p]
    int spmm(const double* A, double* B, int p) {
        const int lanes = lanes_for(p);
        if (npieces > 0) {
            hipLaunchKernelGGL(k_spmm_pieces, dim3(blocks_for(npieces * lanes, kE)), dim3(kE), 0, st,
                               g->row_ptr, g->col, g->w, (const int32_t*)ppos, (const int32_t*)prow,
                               npieces, ep, p, ld, lanes, A, sc, ppart);
            GR_LAUNCHED("spmm pieces");
        }
        hipLaunchKernelGGL(k_spmm_rows, dim3(blocks_for(n * lanes, kE)), dim3(kE), 0, st,
                           (const int32_t*)ppos, (const double*)d, n, p, ld, lanes,
                           (const double*)ppart, A, sc, B);
        GR_LAUNCHED("spmm rows");
        return GR_OK;
    }
    int project(double* A, int p) {
        hipLaunchKernelGGL(k_colsum_part, dim3(kRowBlocks), dim3(kE), 0, st, (const double*)A, n, p,
                           ld, q, part);
        GR_LAUNCHED("colsum");
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(kMaxP), 0, st, (const double*)part,
                           kRowBlocks, p, cs);
        GR_LAUNCHED("colsum final");
        hipLaunchKernelGGL(k_sub_colmean, dim3(blocks_for(n * p, kE)), dim3(kE), 0, st, A, n, p, ld,
                           (const double*)cs, q, (const double*)qq);
        GR_LAUNCHED("project");
        return GR_OK;
    }
    int gram(const double* A, const double* B, int pa, int pb, double* out) {
        hipLaunchKernelGGL(k_gram_part, dim3(kRowBlocks), dim3(kE), 0, st, A, B, n, pa, pb, ld, part);
        GR_LAUNCHED("gram");
        hipLaunchKernelGGL(k_gram_final, dim3(blocks_for(pa * pb, kE)), dim3(kE), 0, st,
                           (const double*)part, kRowBlocks, pa * pb, out);
        GR_LAUNCHED("gram final");
        return GR_OK;
    }
    // A[:, 0:p] <- A[:, 0:p] M with M from the column-scaled (shifted)
    // Cholesky factor of A^T A
    int cholqr(double* A, int p, double shift) {
        GR_TRY(gram(A, A, p, p, G));
        hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kMaxP), 0, st, (const double*)G, p, shift, M,
                           flag);
        GR_LAUNCHED("cholesky");
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * p, kE)), dim3(kE), 0, st,
                           (const double*)A, ld, p, (const double*)M, p, p, n, T, ld);
        GR_LAUNCHED("right mul");
        GR_HIP(hipMemcpyAsync(A, T, sizeof(double) * n * ld, hipMemcpyDeviceToDevice, st));
        return GR_OK;
    }
    // orthonormal columns, orthogonal to the all-one vector; zero columns
    // are first replaced by random ones
    int orthonormalise(double* A, int p) {
        GR_TRY(project(A, p));
        GR_TRY(gram(A, A, p, p, G));
        hipLaunchKernelGGL(k_fix_zero_cols, dim3(blocks_for(n * p, kE)), dim3(kE), 0, st,
                           (const double*)G, n, p, ld, splitmix64(seed, 1000 + fix_round++), A);
        GR_LAUNCHED("fix zero columns");
        GR_TRY(project(A, p));
        const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 0x1p-53;
        GR_TRY(cholqr(A, p, shift));
        GR_TRY(project(A, p));
        GR_TRY(cholqr(A, p, 0.0));
        GR_TRY(cholqr(A, p, 0.0));
        return GR_OK;
    }
    // Rayleigh-Ritz over the orthonormal A[:, 0:p] (LA = L A given):
    // theta[0:p] ascending and the p x p rotation in M
    int ritz_small(const double* A, const double* LA, int p) {
        GR_TRY(gram(A, LA, p, p, G));
        hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJacobiThreads), 0, st, (const double*)G, p, 40,
                           theta, M);
        GR_LAUNCHED("jacobi");
        return GR_OK;
    }
    // squared residual norms of the first m Ritz pairs into res (device)
    int residuals(const double* LX, const double* X, int m) {
        hipLaunchKernelGGL(k_resid_part, dim3(kRowBlocks), dim3(kE), 0, st, LX, X,
                           (const double*)theta, n, m, ld, part);
        GR_LAUNCHED("residual");
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(kMaxP), 0, st, (const double*)part,
                           kRowBlocks, m, res);
        GR_LAUNCHED("residual final");
        return GR_OK;
    }
};

static int lobpcg_block(int n_eig) { return n_eig + 8 < kMaxP / 3 ? n_eig + 8 : kMaxP / 3; }
static int cheb_block(int n_eig) {
    int m = n_eig + (n_eig > 8 ? n_eig : 8);
    return m > kMaxP ? kMaxP : m;
}

size_t eig_workspace(int64_t n, int32_t n_eig) {
    (void)n_eig;
    size_t blk = (size_t)(n + 1) * kMaxP * 8;
    // blocks, degrees, small matrices; row pieces (at most 2n: offsets, rows,
    // and partial sums of up to kMaxP columns each)
    size_t b = 4 * blk + 16 * (size_t)(n + 1) + 8 * (size_t)kRowBlocks * kMaxP * kMaxP +
               8 * 4 * kMaxP * kMaxP + 16 * (size_t)(n + 1) + 2 * blk +
               16 * (size_t)(n + 1);  // b^-1/2 and b^1/2 of a generalised problem
    return b + b / 16 + (1u << 20);
}

// Chebyshev-filtered subspace iteration; block m, ld = m
static int run_chebyshev(Eig& s, int n_eig, int m, double b, double tol, int max_iter, int degree,
                         std::vector<double>& th, double& worst, int& it) {
    const int64_t n = s.n;
    const int64_t cnt = n * m;
    hipStream_t st = s.st;
    hipLaunchKernelGGL(k_init_block, dim3(blocks_for(cnt, kE)), dim3(kE), 0, st, n, m, m, s.seed, s.S);
    GR_LAUNCHED("init block");
    std::vector<double> rs(m);
    worst = INFINITY;
    for (it = 0;; ++it) {
        GR_TRY(s.orthonormalise(s.S, m));
        GR_TRY(s.spmm(s.S, s.LS, m));
        GR_TRY(s.ritz_small(s.S, s.LS, m));
        // rotate X and L X by the Ritz vectors
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(cnt, kE)), dim3(kE), 0, st, (const double*)s.S,
                           m, m, (const double*)s.M, m, m, n, s.T, m);
        GR_LAUNCHED("rotate");
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(cnt, kE)), dim3(kE), 0, st,
                           (const double*)s.LS, m, m, (const double*)s.M, m, m, n, s.U, m);
        GR_LAUNCHED("rotate L");
        std::swap(s.S, s.T);
        std::swap(s.LS, s.U);
        GR_TRY(s.residuals(s.LS, s.S, m));
        GR_HIP(hipMemcpyAsync(th.data(), s.theta, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        GR_HIP(hipMemcpyAsync(rs.data(), s.res, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        worst = 0.0;
        for (int i = 0; i < n_eig && i < m; ++i) worst = fmax(worst, sqrt(fmax(rs[i], 0.0)));
        if (worst <= tol * b || m >= n - 1 || it >= max_iter) break;
        // filter on [a, b], a = the largest Ritz value:
        // Z_0 = X, Z_1 = (L X - c X)/e, Z_j = 2 (L Z_{j-1} - c Z_{j-1})/e - Z_{j-2}
        const double a = th[m - 1];
        const double c = 0.5 * (b + a), e = 0.5 * (b - a);
        if (!(e > 0.0)) break;  // the block already spans [0, b]
        // cap the degree so that the largest amplification (at lambda = 0,
        // T_k((b + a) / (b - a))) stays below 1e6: the filtered block then
        // has a condition number shifted Cholesky QR takes comfortably
        int deg = degree;
        const double per = acosh(fmax(c / e, 1.0));
        if (per > 0.0) deg = (int)fmin((double)degree, fmax(1.0, floor(acosh(1e6) / per)));
        double* Z0 = s.S;  // Z_{j-2}
        double* Z1 = s.T;  // Z_{j-1}
        hipLaunchKernelGGL(k_cheb, dim3(blocks_for(cnt, kE)), dim3(kE), 0, st, (const double*)s.LS,
                           (const double*)s.S, s.T, cnt, c, e, 1);
        GR_LAUNCHED("cheb 1");
        for (int j = 2; j <= deg; ++j) {
            GR_TRY(s.spmm(Z1, s.U, m));
            hipLaunchKernelGGL(k_cheb, dim3(blocks_for(cnt, kE)), dim3(kE), 0, st, (const double*)s.U,
                               (const double*)Z1, Z0, cnt, c, e, 0);
            GR_LAUNCHED("cheb");
            std::swap(Z0, Z1);
        }
        if (Z1 != s.S) std::swap(s.S, s.T);  // the filtered block into S
    }
    return GR_OK;
}

// LOBPCG with the Jacobi preconditioner; basis S = [X | W | P], ld = 3m
static int run_lobpcg(Eig& s, int n_eig, int m, double b, double tol, int max_iter,
                      std::vector<double>& th, double& worst, int& it, int& restarts) {
    const int64_t n = s.n;
    const int ld = s.ld;
    hipStream_t st = s.st;
    hipLaunchKernelGGL(k_init_block, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st, n, m, ld, s.seed, s.S);
    GR_LAUNCHED("init block");
    GR_TRY(s.orthonormalise(s.S, m));
    GR_TRY(s.spmm(s.S, s.LS, m));
    GR_TRY(s.ritz_small(s.S, s.LS, m));
    hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st, (const double*)s.S, ld,
                       m, (const double*)s.M, m, m, n, s.T, ld);
    GR_LAUNCHED("rotate X");
    hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st, (const double*)s.LS,
                       ld, m, (const double*)s.M, m, m, n, s.U, ld);
    GR_LAUNCHED("rotate LX");
    std::swap(s.S, s.T);
    std::swap(s.LS, s.U);  // LS[:, 0:m] = L X
    std::vector<double> rs(m);
    bool have_p = false;
    restarts = 0;
    worst = INFINITY;
    for (it = 0;; ++it) {
        GR_TRY(s.residuals(s.LS, s.S, m));
        GR_HIP(hipMemcpyAsync(th.data(), s.theta, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        GR_HIP(hipMemcpyAsync(rs.data(), s.res, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        worst = 0.0;
        for (int i = 0; i < n_eig; ++i) worst = fmax(worst, sqrt(fmax(rs[i], 0.0)));
        if (worst <= tol * b || it >= max_iter) break;
        // W = D^{-1} (L X - X Theta) into columns [m, 2m)
        hipLaunchKernelGGL(k_precond_resid, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st,
                           (const double*)s.LS, s.S, (const double*)s.theta, (const double*)s.dinv,
                           n, m, ld);
        GR_LAUNCHED("preconditioned residual");
        int p = have_p ? 3 * m : 2 * m;
        // keep [X W P] in U in case the basis with P is rank deficient
        if (have_p) GR_HIP(hipMemcpyAsync(s.U, s.S, sizeof(double) * n * ld, hipMemcpyDeviceToDevice, st));
        GR_HIP(hipMemsetAsync(s.flag, 0, sizeof(int), st));
        GR_TRY(s.orthonormalise(s.S, p));
        if (have_p) {
            int flag = 0;
            GR_HIP(hipMemcpyAsync(&flag, s.flag, sizeof(int), hipMemcpyDeviceToHost, st));
            GR_HIP(hipStreamSynchronize(st));
            if (flag) {  // drop P and start the basis again from [X W]
                ++restarts;
                std::swap(s.S, s.U);
                p = 2 * m;
                GR_HIP(hipMemsetAsync(s.flag, 0, sizeof(int), st));
                GR_TRY(s.orthonormalise(s.S, p));
            }
        }
        GR_TRY(s.spmm(s.S, s.LS, p));
        GR_TRY(s.ritz_small(s.S, s.LS, p));
        // X = S C[:, 0:m], P = S[:, m:p] C[m:p, 0:m], L X = (L S) C[:, 0:m]
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st, (const double*)s.S,
                           ld, p, (const double*)s.M, p, m, n, s.T, ld);
        GR_LAUNCHED("new X");
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st,
                           (const double*)(s.S + m), ld, p - m, (const double*)(s.M + (size_t)m * p), p,
                           m, n, s.T + 2 * m, ld);
        GR_LAUNCHED("new P");
        hipLaunchKernelGGL(k_right_mul, dim3(blocks_for(n * m, kE)), dim3(kE), 0, st, (const double*)s.LS,
                           ld, p, (const double*)s.M, p, m, n, s.U, ld);
        GR_LAUNCHED("new LX");
        std::swap(s.S, s.T);
        std::swap(s.LS, s.U);
        have_p = true;
    }
    return GR_OK;
}

// U[v][i] = the Ritz vector i (column i of the block, stride ld), NaN past
// m; times sc[v] for the generalised problem (u = S v)
__global__ void k_copy_vectors(const double* __restrict__ S, int ld, int m, int64_t n, int k,
                               const double* __restrict__ sc, double* __restrict__ U) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (t >= n * k) return;
    const int64_t v = t / k;
    const int i = (int)(t % k);
    U[t] = i < m ? (sc ? sc[v] * S[v * ld + i] : S[v * ld + i]) : __builtin_nan("");
}

// B = diag(b): sc = b^-1/2, q = b^1/2, and the Jacobi preconditioner of
// S L S, b / d (1 where d = 0); flag[1] = 1 if some b is not positive and
// finite
__global__ void k_b_setup(const double* __restrict__ b, const double* __restrict__ d, int64_t n,
                          double* __restrict__ sc, double* __restrict__ q, double* __restrict__ dinv,
                          int* flag) {
    const int64_t v = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (v >= n) return;
    const double bv = b[v];
    if (!(bv > 0.0) || !(bv < INFINITY)) {
        atomicOr(flag + 1, 1);
        sc[v] = q[v] = 1.0;
        return;
    }
    const double r = sqrt(bv);
    q[v] = r;
    sc[v] = 1.0 / r;
    dinv[v] = d[v] > 0.0 ? bv / d[v] : 1.0;
}

// Gershgorin bound of each row of S L S: sc_v (d_v sc_v + sum_j w_vj sc_j),
// a wave per row
__global__ void __launch_bounds__(kE) k_gersh_rows(const int32_t* __restrict__ rp,
                                                   const float* __restrict__ w,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ d,
                                                   const double* __restrict__ sc, int64_t n,
                                                   double* __restrict__ out) {
    const int64_t v = ((int64_t)blockIdx.x * kE + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    double s = 0.0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave) s = fma((double)w[e], sc[col[e]], s);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) s += __shfl_xor(s, off, kWave);
    if (l == 0) out[v] = sc[v] * (d[v] * sc[v] + s);
}

// degrees and row pieces of the Laplacian product of s.g for blocks of up
// to maxp columns (d, dinv, ppos, prow, ppart taken from ws)
static int setup_operator(Eig& s, int maxp, Arena& ws) {
    const gr_graph* g = s.g;
    const int64_t n = g->n;
    hipStream_t st = s.st;
    s.d = ws.take<double>(n + 1);
    s.dinv = ws.take<double>(n + 1);
    s.ppos = ws.take<int32_t>(n + 1);
    s.prow = ws.take<int32_t>(2 * (size_t)n + 1);
    s.ppart = ws.take<double>((2 * (size_t)n + 1) * maxp);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (Laplacian product)");
    hipLaunchKernelGGL(k_degree_f64, dim3(blocks_for(n * kWave, kE)), dim3(kE), 0, st, g->row_ptr,
                       g->w, n, s.d, s.dinv);
    GR_LAUNCHED("degrees");
    // row pieces of at least the mean degree: at most n + nnz / ep <= 2n
    s.ep = (int32_t)std::max<int64_t>(64, (g->nnz + n - 1) / (n > 0 ? n : 1));
    {
        const size_t mark = ws.used;
        int32_t* cnt = ws.take<int32_t>(n);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (eigen pieces)");
        hipLaunchKernelGGL(k_piece_counts_e, dim3(blocks_for(n, kE)), dim3(kE), 0, st, g->row_ptr, n,
                           s.ep, cnt);
        GR_LAUNCHED("piece counts");
        GR_TRY(scan_exclusive_i32(cnt, s.ppos, n, s.ppos + n, ws, st));
        ws.used = mark;
    }
    hipLaunchKernelGGL(k_piece_rows, dim3(blocks_for(n, kE)), dim3(kE), 0, st, (const int32_t*)s.ppos,
                       n, s.prow);
    GR_LAUNCHED("piece rows");
    int32_t np32 = 0;
    GR_HIP(hipMemcpyAsync(&np32, s.ppos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    s.npieces = np32;
    if (s.npieces > 2 * n) return set_error(GR_EINVAL, "row pieces exceed 2n");
    return GR_OK;
}

int laplacian_eigs(const gr_graph* g, const double* bdiag, int32_t n_eig, int32_t method,
                   double tol, int32_t max_iter, int32_t degree, uint64_t seed, double* eig_out,
                   double* vec_out, gr_eig_report* rep, Arena& ws, hipStream_t st) {
    Eig s{};
    s.g = g;
    s.n = g->n;
    s.st = st;
    s.seed = seed;
    const int64_t n = g->n;
    s.S = ws.take<double>((size_t)n * kMaxP + 1);
    s.LS = ws.take<double>((size_t)n * kMaxP + 1);
    s.T = ws.take<double>((size_t)n * kMaxP + 1);
    s.U = ws.take<double>((size_t)n * kMaxP + 1);
    s.part = ws.take<double>((size_t)kRowBlocks * kMaxP * kMaxP);
    s.G = ws.take<double>(kMaxP * kMaxP);
    s.M = ws.take<double>(kMaxP * kMaxP);
    s.theta = ws.take<double>(kMaxP);
    s.cs = ws.take<double>(kMaxP);
    s.res = ws.take<double>(kMaxP);
    s.small = ws.take<double>(8);
    s.flag = ws.take<int>(4);
    double* bsc = bdiag ? ws.take<double>(n + 1) : nullptr;
    double* bq = bdiag ? ws.take<double>(n + 1) : nullptr;
    double* bqq = bdiag ? ws.take<double>(8) : nullptr;
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (eigen)");
    GR_HIP(hipMemsetAsync(s.flag, 0, sizeof(int) * 4, st));
    GR_TRY(setup_operator(s, kMaxP, ws));
    hipLaunchKernelGGL(k_deg_stats, dim3(1), dim3(kE), 0, st, (const double*)s.d, n, s.small);
    GR_LAUNCHED("degree stats");
    double dstat[2] = {0.0, 0.0};
    GR_HIP(hipMemcpyAsync(dstat, s.small, sizeof(dstat), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    double b = 2.0 * dstat[0] * (1.0 + 1e-12) + 1e-300;  // lambda_max <= 2 max degree
    const double mean = dstat[1] / (double)n;
    if (bdiag) {  // the generalised problem: S L S in the complement of b^1/2
        hipLaunchKernelGGL(k_b_setup, dim3(blocks_for(n, kE)), dim3(kE), 0, st, bdiag,
                           (const double*)s.d, n, bsc, bq, s.dinv, s.flag);
        GR_LAUNCHED("generalised set-up");
        // q^T q = sum of b, in the fixed order of the column sums
        hipLaunchKernelGGL(k_colsum_part, dim3(kRowBlocks), dim3(kE), 0, st, bdiag, n, 1, 1,
                           (const double*)nullptr, s.part);
        GR_LAUNCHED("sum of b");
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(kMaxP), 0, st, (const double*)s.part,
                           kRowBlocks, 1, bqq);
        GR_LAUNCHED("sum of b final");
        // Gershgorin bound of lambda_max(S L S), rows into the T block
        hipLaunchKernelGGL(k_gersh_rows, dim3(blocks_for(n * kWave, kE)), dim3(kE), 0, st,
                           g->row_ptr, g->w, g->col, (const double*)s.d, (const double*)bsc, n, s.T);
        GR_LAUNCHED("gershgorin rows");
        hipLaunchKernelGGL(k_deg_stats, dim3(1), dim3(kE), 0, st, (const double*)s.T, n, s.small);
        GR_LAUNCHED("gershgorin bound");
        double gs[2] = {0.0, 0.0};
        int fl[2] = {0, 0};
        GR_HIP(hipMemcpyAsync(gs, s.small, sizeof(gs), hipMemcpyDeviceToHost, st));
        GR_HIP(hipMemcpyAsync(fl, s.flag, sizeof(fl), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        if (fl[1]) return set_error(GR_EINVAL, "the diagonal of B must be positive and finite");
        b = gs[0] * (1.0 + 1e-12) + 1e-300;
        s.sc = bsc;
        s.q = bq;
        s.qq = bqq;
    }
    // method choice: LOBPCG where a few hubs dominate the spectrum and the
    // block fits well inside the space; the filter otherwise
    const int ml = lobpcg_block(n_eig);
    const bool lobpcg_fits = n_eig + 2 <= ml && 3 * ml * 4 <= n;
    if (method == GR_EIG_LOBPCG && !lobpcg_fits)
        return set_error(GR_EUNSUP, "LOBPCG needs n_eig <= %d and n >= %d", kMaxP / 3 - 2, 12 * ml);
    const bool use_lobpcg =
        method == GR_EIG_LOBPCG || (method == GR_EIG_AUTO && lobpcg_fits && dstat[0] > 16.0 * mean);
    std::vector<double> th(kMaxP);
    double worst = INFINITY;
    int it = 0, restarts = 0, m;
    if (use_lobpcg) {
        m = ml;
        s.ld = 3 * m;
        GR_TRY(run_lobpcg(s, n_eig, m, b, tol, max_iter, th, worst, it, restarts));
    } else {
        m = cheb_block(n_eig);
        if (m > n - 1) m = (int)(n - 1);
        s.ld = m;
        GR_TRY(run_chebyshev(s, n_eig, m, b, tol, max_iter, degree, th, worst, it));
    }
    int flag = 0;
    GR_HIP(hipMemcpyAsync(&flag, s.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n_eig; ++i) eig_out[i] = i < m ? th[i] : NAN;
    if (vec_out) {  // the block holds the Ritz vectors of th, in ascending order
        hipLaunchKernelGGL(k_copy_vectors, dim3(blocks_for(n * n_eig, kE)), dim3(kE), 0, st,
                           (const double*)s.S, s.ld, m, n, n_eig, s.sc, vec_out);
        GR_LAUNCHED("copy vectors");
        GR_HIP(hipStreamSynchronize(st));
    }
    if (rep) {
        rep->iterations = it;
        rep->block = m;
        rep->residual = worst;
        rep->lambda_max_bound = b;
        rep->cholesky_warnings = flag;
        rep->method = use_lobpcg ? GR_EIG_LOBPCG : GR_EIG_CHEBYSHEV;
        rep->restarts = restarts;
    }
    return GR_OK;
}

// ------------------------------------- solution refinement and Alg. 5
// Alg. 3 filters approximate solutions by weighted Jacobi,
// x <- (1 - theta) x + theta D^-1 A x; Alg. 5 applies the same smoother to
// (L - lambda_i B) y = 0 on every level of the hierarchy.  The step used for
// both keeps the Laplacian's own diagonal: y <- y - theta D^-1 (L y - lambda_i B y),
// which is Alg. 3's step when lambda = 0 (rows with d = 0 stay).

// U[v][i] = Uc[agg[v]][i] (H = the 0/1 node-to-aggregate map)
__global__ void k_prolong(const int32_t* __restrict__ agg, int64_t n, int k,
                          const double* __restrict__ Uc, double* __restrict__ U) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (t >= n * k) return;
    const int64_t v = t / k;
    const int i = (int)(t - v * k);
    U[t] = Uc[(int64_t)agg[v] * k + i];
}

__global__ void k_jacobi_update(const double* __restrict__ LY, double* __restrict__ Y,
                                const double* __restrict__ d, const double* __restrict__ b,
                                const double* __restrict__ lam, int64_t n, int k, double theta) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (t >= n * k) return;
    const int64_t v = t / k;
    const int i = (int)(t - v * k);
    const double dv = d[v];
    if (!(dv > 0.0)) return;
    const double y = Y[t];
    double r = LY[t];
    if (lam) r -= ((b ? b[v] : 1.0) * y) * lam[i];
    Y[t] = y - (theta * r) / dv;
}

// X[v][i] *= f[v], or /= f[v]
__global__ void k_row_scale(double* __restrict__ X, const double* __restrict__ f, int64_t n, int k,
                            int divide) {
    const int64_t t = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (t >= n * k) return;
    const int64_t v = t / k;
    X[t] = divide ? X[t] / f[v] : X[t] * f[v];
}

__global__ void k_sqrt_vec(const double* __restrict__ b, int64_t n, double* __restrict__ r,
                           int* bad) {
    const int64_t v = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (v >= n) return;
    const double x = b[v];
    if (!(x > 0.0) || !(x < INFINITY)) {
        atomicOr(bad, 1);
        r[v] = 1.0;
    } else {
        r[v] = sqrt(x);
    }
}

size_t jacobi_workspace(int64_t n, int32_t k) {
    const size_t N = (size_t)n + 1;
    size_t b = 16 * N + 4 * N + 4 * (2 * N) + 8 * (2 * N) * (size_t)k   // operator
               + 8 * N * (size_t)k + 8 * 64 + 4 * N + (64u << 10);      // L Y, lambda, scan
    return b + b / 16 + (1u << 20);
}

int jacobi_filter(const gr_graph* g, int32_t k, double* Y, const double* lam_host,
                  const double* bdiag, double theta, int32_t iters, Arena& ws, hipStream_t st) {
    const int64_t n = g->n;
    if (n == 0 || iters == 0) return GR_OK;
    const size_t mark = ws.used;
    Eig s{};
    s.g = g;
    s.n = n;
    s.st = st;
    s.ld = k;
    GR_TRY(setup_operator(s, k, ws));
    double* LY = ws.take<double>((size_t)n * k + 1);
    double* lam = lam_host ? ws.take<double>(k) : nullptr;
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (Jacobi filter)");
    if (lam) GR_HIP(hipMemcpyAsync(lam, lam_host, sizeof(double) * k, hipMemcpyHostToDevice, st));
    for (int32_t it = 0; it < iters; ++it) {
        GR_TRY(s.spmm(Y, LY, k));
        hipLaunchKernelGGL(k_jacobi_update, dim3(blocks_for(n * k, kE)), dim3(kE), 0, st,
                           (const double*)LY, Y, (const double*)s.d, bdiag, (const double*)lam, n, k,
                           theta);
        GR_LAUNCHED("Jacobi update");
    }
    GR_HIP(hipStreamSynchronize(st));  // lam_host may be released on return
    ws.used = mark;
    return GR_OK;
}

size_t orthonormalize_workspace(int64_t n, int32_t k) {
    const size_t N = (size_t)n + 1;
    size_t b = 8 * N * (size_t)k + 8 * N + 8 * (size_t)kRowBlocks * kMaxP * kMaxP +
               8 * 4 * kMaxP * kMaxP + 8 * 64;
    return b + b / 16 + (1u << 20);
}

// Gram-Schmidt over [1, U] in the B inner product (B = diag(b), or I): with
// V = B^1/2 U and q = B^1/2 1 it is the plain process on [q, V], computed
// as a projection against q and Cholesky QR (the same Q: Gram-Schmidt and
// Cholesky QR both give the QR factor with a positive diagonal).
int orthonormalize(int64_t n, int32_t k, double* U, const double* bdiag, Arena& ws,
                   hipStream_t st) {
    if (n == 0) return GR_OK;
    if (k < 1 || k > kMaxP) return set_error(GR_EINVAL, "k must lie in [1, %d]", kMaxP);
    const size_t mark = ws.used;
    Eig s{};
    s.n = n;
    s.st = st;
    s.ld = k;
    s.seed = 0x9e3779b97f4a7c15ull;
    s.T = ws.take<double>((size_t)n * k + 1);
    s.part = ws.take<double>((size_t)kRowBlocks * kMaxP * kMaxP);
    s.G = ws.take<double>(kMaxP * kMaxP);
    s.M = ws.take<double>(kMaxP * kMaxP);
    s.cs = ws.take<double>(kMaxP);
    s.flag = ws.take<int>(4);
    double* q = bdiag ? ws.take<double>(n + 1) : nullptr;
    double* qq = bdiag ? ws.take<double>(8) : nullptr;
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (orthonormalisation)");
    GR_HIP(hipMemsetAsync(s.flag, 0, sizeof(int) * 4, st));
    if (bdiag) {
        hipLaunchKernelGGL(k_sqrt_vec, dim3(blocks_for(n, kE)), dim3(kE), 0, st, bdiag, n, q,
                           s.flag + 1);
        GR_LAUNCHED("B^1/2");
        hipLaunchKernelGGL(k_colsum_part, dim3(kRowBlocks), dim3(kE), 0, st, bdiag, n, 1, 1,
                           (const double*)nullptr, s.part);
        GR_LAUNCHED("sum of b");
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(kMaxP), 0, st, (const double*)s.part,
                           kRowBlocks, 1, qq);
        GR_LAUNCHED("sum of b final");
        hipLaunchKernelGGL(k_row_scale, dim3(blocks_for(n * k, kE)), dim3(kE), 0, st, U,
                           (const double*)q, n, k, 0);
        GR_LAUNCHED("B^1/2 U");
        s.q = q;
        s.qq = qq;
    }
    GR_TRY(s.orthonormalise(U, k));
    if (bdiag) {
        hipLaunchKernelGGL(k_row_scale, dim3(blocks_for(n * k, kE)), dim3(kE), 0, st, U,
                           (const double*)q, n, k, 1);
        GR_LAUNCHED("B^-1/2 V");
    }
    int fl[2] = {0, 0};
    GR_HIP(hipMemcpyAsync(fl, s.flag, sizeof(fl), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    ws.used = mark;
    if (fl[1]) return set_error(GR_EINVAL, "the diagonal of B must be positive and finite");
    if (fl[0]) return set_error(GR_EINVAL, "the columns are linearly dependent");
    return GR_OK;
}

__global__ void k_fill_f64(double* __restrict__ x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * kE + threadIdx.x;
    if (i < n) x[i] = v;
}

size_t multilevel_workspace(int64_t n, int64_t nnz, int32_t k) {
    (void)nnz;
    const size_t N = (size_t)n + 1;
    size_t b = eig_workspace(n, k) + 2 * 8 * N * (size_t)k + 2 * 8 * N + jacobi_workspace(n, k) +
               orthonormalize_workspace(n, k) + restrict_workspace(n, n, 1);
    return b + b / 16 + (1u << 20);
}

int multilevel_eigs(const gr_graph* g, const gr_hierarchy* h, int32_t k, int32_t cut, double theta,
                    int32_t iters, double tol, int32_t max_iter, uint64_t seed, double* lam_out,
                    double* U, gr_eig_report* rep, Arena& ws, hipStream_t st) {
    const int L = h->levels;
    const int64_t n0 = g->n;
    // level graphs: 0 = g, l >= 1 from the hierarchy
    std::vector<gr_graph> lv(L + 1);
    lv[0] = *g;
    for (int l = 1; l <= L; ++l) {
        lv[l].n = h->n[l];
        lv[l].nnz = h->nnz[l];
        lv[l].row_ptr = h->row_ptr + h->rp_off[l - 1];
        lv[l].col = h->col + h->ent_off[l - 1];
        lv[l].w = h->w + h->ent_off[l - 1];
    }
    // B on every level: B^1 = I (ratio cut) or D (normalized cut), then
    // B^{l+1} = P_l^T B^l P_l, the sums of B^l over each aggregate
    std::vector<double*> B(L + 1);
    for (int l = 0; l <= L; ++l) B[l] = ws.take<double>(lv[l].n + 1);
    double* Ua = ws.take<double>((size_t)n0 * k + 1);
    double* Ub = ws.take<double>((size_t)n0 * k + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (multilevel eigensolver)");
    if (cut == GR_RQ_IDENTITY) {
        hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n0, kE)), dim3(kE), 0, st, B[0], n0, 1.0);
        GR_LAUNCHED("B = I");
    } else {
        double* dinv = ws.take<double>(n0 + 1);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (multilevel eigensolver)");
        hipLaunchKernelGGL(k_degree_f64, dim3(blocks_for(n0 * kWave, kE)), dim3(kE), 0, st,
                           g->row_ptr, g->w, n0, B[0], dinv);
        GR_LAUNCHED("B = D");
    }
    for (int l = 0; l < L; ++l)
        GR_TRY(restrict_sum_f64(h->maps + h->maps_off[l], lv[l].n, lv[l + 1].n, B[l], B[l + 1], ws,
                                st));
    // the coarsest eigenpairs (lambda_i, u_i) of L^Y u = lambda B^Y u
    const bool plain = L == 0 && cut == GR_RQ_IDENTITY;
    {
        const size_t mark = ws.used;
        GR_TRY(laplacian_eigs(&lv[L], plain ? nullptr : B[L], k, GR_EIG_AUTO, tol, max_iter, 16,
                              seed, lam_out, Ua, rep, ws, st));
        ws.used = mark;
    }
    for (int i = 0; i < k; ++i)
        if (!(lam_out[i] == lam_out[i]))
            return set_error(GR_EINVAL, "the coarsest level has fewer than %d nontrivial eigenpairs", k);
    // down the hierarchy: prolong, then filter with the coarsest lambda_i
    double* cur = Ua;
    double* nxt = Ub;
    for (int l = L; l >= 1; --l) {
        const int64_t nf = lv[l - 1].n;
        hipLaunchKernelGGL(k_prolong, dim3(blocks_for(nf * k, kE)), dim3(kE), 0, st,
                           (const int32_t*)(h->maps + h->maps_off[l - 1]), nf, k, (const double*)cur,
                           nxt);
        GR_LAUNCHED("prolong");
        GR_TRY(jacobi_filter(&lv[l - 1], k, nxt, lam_out, B[l - 1], theta, iters, ws, st));
        std::swap(cur, nxt);
    }
    // Gram-Schmidt of the finest vectors (B^1 inner product, after 1)
    GR_TRY(orthonormalize(n0, k, cur, cut == GR_RQ_IDENTITY ? nullptr : B[0], ws, st));
    GR_HIP(hipMemcpyAsync(U, cur, sizeof(double) * n0 * k, hipMemcpyDeviceToDevice, st));
    GR_HIP(hipStreamSynchronize(st));
    return GR_OK;
}

}  // namespace gr
