// Constrained-SGD edge scaling (Alg. 1, Sec. 3.3.4) in FP64 on the GPU.
//
// G is the original graph, P a spectrally similar subgraph on the same
// nodes whose edge weights w_P (one per P-edge) are scaled up.  Per
// iteration: h_t from t generalised power iterations h <- L_P^+ L_G h
// (Sec. 3.3.3; the L_P solves by Jacobi-preconditioned conjugate gradients),
// normalised so h^T L_P h = 1; lambda_n = h^T L_G h; sensitivities
// s = -lambda_n (h_p - h_q)^2; momentum step dw <- alpha dw - eta s; degree
// caps cap_p = d_G(p) / (lambda_1 Delta) - d_P(p), shared in proportion
// where the edges at p ask for more (all edges updated at once); w += dw;
// eta <- (lambda_n / lambda_n^(0)) eta_max; lambda_1 = min_p d_G/d_P.
// All reductions have a fixed shape, so results are bit-reproducible.
#include "gr_internal.hpp"

#include <math.h>

#include <vector>

namespace gr {

constexpr int kS = 256;
constexpr int kRedBlocks = 256;

// scalar slots on the device
enum {
    SC_RZ = 0, SC_PQ, SC_RR, SC_BB, SC_TMP, SC_LAMN, SC_LAMN0, SC_ETA, SC_ETAMAX, SC_LAM1,
    SC_MAXS, SC_SUMW0, SC_HLH, SC_COUNT
};

__device__ inline double block_reduce_sum(double v, double* sh) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kS / kWave; ++w) t += sh[w];
    __syncthreads();
    return t;
}

__device__ inline double block_reduce_min(double v, double* sh) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = sh[0];
#pragma unroll
    for (int w = 1; w < kS / kWave; ++w) t = fmin(t, sh[w]);
    __syncthreads();
    return t;
}

// partials of sum_i x_i y_i (y == nullptr: sum_i x_i)
__global__ void __launch_bounds__(kS) k_dot_part(const double* __restrict__ x,
                                                 const double* __restrict__ y, int64_t n,
                                                 double* __restrict__ part) {
    __shared__ double sh[kS / kWave];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kS)
        s = y ? fma(x[i], y[i], s) : s + x[i];
    s = block_reduce_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kS) k_sum_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
    __shared__ double sh[kS / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kS) s += part[i];
    s = block_reduce_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// The row-walking kernels below take a wave per row, with kSpU loads in
// flight per lane, and reduce in a fixed tree: hub rows of reduced graphs
// hold thousands of entries, and fewer lanes would serialise them.
constexpr int kSpU = 4;

__device__ inline double wave_sum_f64(double s) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) s += __shfl_xor(s, off, kWave);
    return s;
}

// y_v = d_v x_v - sum_j w_vj x_j
__global__ void __launch_bounds__(kS) k_lap_spmv(const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ diag, int64_t n,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    const int32_t e1 = rp[v + 1];
    double s = 0.0;
    for (int32_t b = rp[v] + l; b < e1; b += kWave * kSpU) {
        double wv[kSpU], xv[kSpU];
#pragma unroll
        for (int u = 0; u < kSpU; ++u) {
            const int32_t e = b + u * kWave;
            const bool ok = e < e1;
            wv[u] = ok ? w[e] : 0.0;
            xv[u] = ok ? x[col[e]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSpU; ++u) s = fma(wv[u], xv[u], s);
    }
    s = wave_sum_f64(s);
    if (l == 0) y[v] = diag[v] * x[v] - s;
}

__global__ void __launch_bounds__(kS) k_row_sums(const int32_t* __restrict__ rp,
                                                 const double* __restrict__ w, int64_t n,
                                                 double* __restrict__ d) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    double s = 0.0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave) s += w[e];
    s = wave_sum_f64(s);
    if (l == 0) d[v] = s;
}

__global__ void k_promote(const float* __restrict__ a, int64_t n, double* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

__global__ void k_expand_f64(const int32_t* __restrict__ eoe, int64_t nnz, int64_t E,
                             const double* __restrict__ wE, double* __restrict__ w) {
    int64_t e = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (e >= nnz) return;
    int32_t k = eoe[e];
    w[e] = (k >= 0 && k < E) ? wE[k] : 0.0;
}

// x -= s[SC_TMP] / n  (centring; the sum was stored in SC_TMP)
__global__ void k_sub_mean(double* __restrict__ x, int64_t n, const double* __restrict__ sc) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i < n) x[i] -= sc[SC_TMP] / (double)n;
}

// x *= 1 / sqrt(s[SC_HLH])
__global__ void k_normalise(double* __restrict__ x, int64_t n, const double* __restrict__ sc) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i < n) x[i] /= sqrt(sc[SC_HLH]);
}

// h0: the test-vector generator for one column (x0 in (-1, 1) from the top 24
// bits of splitmix64 output v), centred afterwards
__global__ void k_init_h(int64_t n, uint64_t seed, double* __restrict__ h) {
    int64_t v = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (v >= n) return;
    uint64_t r = splitmix64(seed, (uint64_t)v);
    int64_t m = (int64_t)(r >> 40);
    h[v] = (double)(2 * m + 1 - (1ll << 24)) * (1.0 / 16777216.0);
}

// ------------------------------------------------------------------ CG
// conjugate gradients on L_P y = b (b orthogonal to 1), Jacobi preconditioner
__global__ void k_cg_init(const double* __restrict__ b, const double* __restrict__ d, int64_t n,
                          double* __restrict__ y, double* __restrict__ r, double* __restrict__ z,
                          double* __restrict__ p) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i >= n) return;
    y[i] = 0.0;
    r[i] = b[i];
    double zi = d[i] > 0.0 ? b[i] / d[i] : 0.0;
    z[i] = zi;
    p[i] = zi;
}

// alpha = rz / pq;  y += alpha p;  r -= alpha q;  z = r / d
__global__ void k_cg_step1(double* __restrict__ y, double* __restrict__ r, double* __restrict__ z,
                           const double* __restrict__ p, const double* __restrict__ q,
                           const double* __restrict__ d, int64_t n,
                           const double* __restrict__ sc) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i >= n) return;
    double pq = sc[SC_PQ];
    double alpha = pq != 0.0 ? sc[SC_RZ] / pq : 0.0;
    y[i] = fma(alpha, p[i], y[i]);
    double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    z[i] = d[i] > 0.0 ? ri / d[i] : 0.0;
}

// beta = rz_new / rz;  p = z + beta p;  rz <- rz_new
__global__ void k_cg_step2(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                           const double* __restrict__ sc) {
    int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i >= n) return;
    double beta = sc[SC_RZ] != 0.0 ? sc[SC_TMP] / sc[SC_RZ] : 0.0;
    p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_copy_scalar(double* __restrict__ sc, int from, int to) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc[to] = sc[from];
}

// ------------------------------------------------------------ Alg. 1 step
__global__ void k_sgd_propose(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                              const double* __restrict__ h, int64_t E, double alpha,
                              const double* __restrict__ sc, int first, double* __restrict__ s_out,
                              double* __restrict__ dw, double* __restrict__ prop) {
    int64_t e = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (e >= E) return;
    double df = h[eu[e]] - h[ev[e]];
    double s = -sc[SC_LAMN] * df * df;
    if (first) {
        s_out[e] = s;  // only needed for eta_max
        return;
    }
    double d = fma(alpha, dw[e], -sc[SC_ETA] * s);
    dw[e] = d;
    prop[e] = d > 0.0 ? d : 0.0;
}

__global__ void __launch_bounds__(kS) k_absmax_part(const double* __restrict__ x, int64_t n,
                                                    double* __restrict__ part) {
    __shared__ double sh[kS / kWave];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kS)
        m = fmax(m, fabs(x[i]));
    m = -block_reduce_min(-m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kS) k_max_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
    __shared__ double sh[kS / kWave];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += kS) m = fmax(m, part[i]);
    m = -block_reduce_min(-m, sh);
    if (threadIdx.x == 0) *out = m;
}

// eta_max = eta_scale * mean(w_P^(0)) / max |s^(1)|;  eta = eta_max
__global__ void k_set_eta(double* __restrict__ sc, double eta_scale, int64_t E) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double em = sc[SC_MAXS] > 0.0 ? eta_scale * (sc[SC_SUMW0] / (double)E) / sc[SC_MAXS] : 0.0;
    sc[SC_ETAMAX] = em;
    sc[SC_ETA] = em;
}

// S_v = sum of the proposals of the P-edges at v (gather over P's rows)
__global__ void __launch_bounds__(kS) k_node_sums(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ eoe,
                                                  const double* __restrict__ x, int64_t n,
                                                  int64_t E, double* __restrict__ S) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    double s = 0.0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave) {
        const int32_t k = eoe[e];
        if (k >= 0 && k < E) s += x[k];
    }
    s = wave_sum_f64(s);
    if (l == 0) S[v] = s;
}

// caps and update: dw = max(0, min(dw, min(f_p, f_q) * prop)), w += dw,
// f_p = cap_p / S_p with cap_p = d_G(p) / (lambda_1 Delta) - d_P(p)
__global__ void k_sgd_apply(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const double* __restrict__ dG, const double* __restrict__ dP,
                            const double* __restrict__ S, int64_t E, double delta,
                            const double* __restrict__ sc, double* __restrict__ dw,
                            const double* __restrict__ prop, double* __restrict__ w) {
    int64_t e = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (e >= E) return;
    const double lim = sc[SC_LAM1] * delta;
    double f = INFINITY;
    int32_t ends[2] = {eu[e], ev[e]};
    for (int k = 0; k < 2; ++k) {
        int32_t p = ends[k];
        if (S[p] > 0.0) f = fmin(f, (dG[p] / lim - dP[p]) / S[p]);
    }
    double d = fmin(dw[e], f * prop[e]);
    d = d > 0.0 ? d : 0.0;
    dw[e] = d;
    w[e] += d;
}

__global__ void __launch_bounds__(kS) k_ratio_min_part(const double* __restrict__ dG,
                                                       const double* __restrict__ dP, int64_t n,
                                                       double* __restrict__ part) {
    __shared__ double sh[kS / kWave];
    double m = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kS)
        if (dP[i] > 0.0) m = fmin(m, dG[i] / dP[i]);
    m = block_reduce_min(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kS) k_min_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
    __shared__ double sh[kS / kWave];
    double m = INFINITY;
    for (int i = threadIdx.x; i < nb; i += kS) m = fmin(m, part[i]);
    m = block_reduce_min(m, sh);
    if (threadIdx.x == 0) *out = m;
}

// eta <- (lambda_n / lambda_n^(0)) eta_max
__global__ void k_update_eta(double* __restrict__ sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        sc[SC_ETA] = sc[SC_LAMN0] != 0.0 ? (sc[SC_LAMN] / sc[SC_LAMN0]) * sc[SC_ETAMAX] : 0.0;
}

// ------------------------------------------------------------ host driver
struct Sgd {
    int64_t n, nnzG, nnzP, E;
    const int32_t *rpG, *colG, *rpP, *colP, *eoe, *eu, *ev;
    double *wG, *dG, *wPent, *dP, *w, *dw, *prop, *s1, *S, *h, *t1, *t2;
    double *y, *r, *z, *p, *q, *part, *sc;
    hipStream_t st;
    int cg_max;
    double cg_tol;
    int64_t cg_iters_max;

    int dot(const double* x, const double* yv, int64_t m, int slot) {
        hipLaunchKernelGGL(k_dot_part, dim3(kRedBlocks), dim3(kS), 0, st, x, yv, m, part);
        GR_LAUNCHED("dot");
        hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kS), 0, st, (const double*)part, kRedBlocks,
                           sc + slot);
        GR_LAUNCHED("dot final");
        return GR_OK;
    }
    int centre(double* x) {
        GR_TRY(dot(x, nullptr, n, SC_TMP));
        hipLaunchKernelGGL(k_sub_mean, dim3(blocks_for(n, kS)), dim3(kS), 0, st, x, n,
                           (const double*)sc);
        GR_LAUNCHED("centre");
        return GR_OK;
    }
    int lapG(const double* x, double* yv) {
        hipLaunchKernelGGL(k_lap_spmv, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, rpG, colG,
                           (const double*)wG, (const double*)dG, n, x, yv);
        GR_LAUNCHED("spmv G");
        return GR_OK;
    }
    int lapP(const double* x, double* yv) {
        hipLaunchKernelGGL(k_lap_spmv, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, rpP, colP,
                           (const double*)wPent, (const double*)dP, n, x, yv);
        GR_LAUNCHED("spmv P");
        return GR_OK;
    }
    double read(int slot) {
        double v = 0.0;
        if (hipMemcpyAsync(&v, sc + slot, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
            return NAN;
        if (hipStreamSynchronize(st) != hipSuccess) return NAN;
        return v;
    }
    // y = L_P^+ b by preconditioned CG, b orthogonal to 1
    int solve(const double* b, double* out) {
        const unsigned nb = blocks_for(n, kS);
        hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kS), 0, st, b, (const double*)dP, n, y, r, z, p);
        GR_LAUNCHED("cg init");
        GR_TRY(dot(r, z, n, SC_RZ));
        GR_TRY(dot(b, b, n, SC_BB));
        const double bb = read(SC_BB);
        if (!(bb > 0.0)) {
            GR_HIP(hipMemsetAsync(out, 0, sizeof(double) * n, st));
            return GR_OK;
        }
        int it = 0;
        for (; it < cg_max; ++it) {
            GR_TRY(lapP(p, q));
            GR_TRY(dot(p, q, n, SC_PQ));
            hipLaunchKernelGGL(k_cg_step1, dim3(nb), dim3(kS), 0, st, y, r, z, (const double*)p,
                               (const double*)q, (const double*)dP, n, (const double*)sc);
            GR_LAUNCHED("cg step1");
            GR_TRY(dot(r, z, n, SC_TMP));
            hipLaunchKernelGGL(k_cg_step2, dim3(nb), dim3(kS), 0, st, p, (const double*)z, n,
                               (const double*)sc);
            GR_LAUNCHED("cg step2");
            hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, st, sc, (int)SC_TMP, (int)SC_RZ);
            GR_LAUNCHED("cg scalar");
            if ((it & 7) == 7) {
                GR_TRY(dot(r, r, n, SC_RR));
                double rr = read(SC_RR);
                if (!(rr == rr)) return set_error(GR_EHIP, "CG diverged");
                if (rr <= cg_tol * cg_tol * bb) break;
            }
        }
        if (it > cg_iters_max) cg_iters_max = it;
        GR_HIP(hipMemcpyAsync(out, y, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        return centre(out);
    }
    // h_t: t generalised power iterations h <- L_P^+ L_G h from the centred
    // h_0, normalised to h^T L_P h = 1 (into h); lambda_n = h^T L_G h
    // (device slot SC_LAMN and *lam)
    int power_vector(uint64_t seed, int t_iters, double* lam) {
        const unsigned nb = blocks_for(n, kS);
        hipLaunchKernelGGL(k_init_h, dim3(nb), dim3(kS), 0, st, n, seed, h);
        GR_LAUNCHED("h0");
        GR_TRY(centre(h));
        for (int t = 0; t < t_iters; ++t) {
            GR_TRY(lapG(h, t1));
            GR_TRY(centre(t1));
            GR_TRY(solve(t1, h));
        }
        GR_TRY(lapP(h, t1));
        GR_TRY(dot(h, t1, n, SC_HLH));
        hipLaunchKernelGGL(k_normalise, dim3(nb), dim3(kS), 0, st, h, n, (const double*)sc);
        GR_LAUNCHED("normalise");
        GR_TRY(lapG(h, t1));
        GR_TRY(dot(h, t1, n, SC_LAMN));
        *lam = read(SC_LAMN);
        if (!(*lam == *lam)) return set_error(GR_EHIP, "lambda_n is not finite");
        return GR_OK;
    }
    int refresh_P() {
        hipLaunchKernelGGL(k_expand_f64, dim3(blocks_for(nnzP, kS)), dim3(kS), 0, st, eoe, nnzP, E,
                           (const double*)w, wPent);
        GR_LAUNCHED("expand P");
        hipLaunchKernelGGL(k_row_sums, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, rpP,
                           (const double*)wPent, n, dP);
        GR_LAUNCHED("d_P");
        return GR_OK;
    }
    int lambda1() {
        hipLaunchKernelGGL(k_ratio_min_part, dim3(kRedBlocks), dim3(kS), 0, st, (const double*)dG,
                           (const double*)dP, n, part);
        GR_LAUNCHED("ratio min");
        hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kS), 0, st, (const double*)part, kRedBlocks,
                           sc + SC_LAM1);
        GR_LAUNCHED("ratio min final");
        return GR_OK;
    }
};

size_t sgd_workspace(int64_t n, int64_t nnzG, int64_t nnzP, int64_t E) {
    size_t b = 8 * ((size_t)nnzG + (size_t)nnzP + 16 * (size_t)(n + 1) + 4 * (size_t)(E + 1)) +
               8 * (kRedBlocks + 64) + 32 * 256;
    return b + b / 16 + (1u << 20);
}

int sgd_scale(const gr_graph* G, const gr_graph* P, const int32_t* eoe, int64_t E,
              const int32_t* eu, const int32_t* ev, double* wP, const gr_sgd_params* prm,
              gr_sgd_report* rep, Arena& ws, hipStream_t st) {
    Sgd s{};
    s.n = G->n;
    s.nnzG = G->nnz;
    s.nnzP = P->nnz;
    s.E = E;
    s.rpG = G->row_ptr;
    s.colG = G->col;
    s.rpP = P->row_ptr;
    s.colP = P->col;
    s.eoe = eoe;
    s.eu = eu;
    s.ev = ev;
    s.w = wP;
    s.st = st;
    s.cg_max = prm->cg_max_iter > 0 ? prm->cg_max_iter : 20000;
    s.cg_tol = prm->cg_tol > 0.0 ? prm->cg_tol : 1e-13;
    const int64_t n = s.n;
    s.wG = ws.take<double>(s.nnzG + 1);
    s.dG = ws.take<double>(n + 1);
    s.wPent = ws.take<double>(s.nnzP + 1);
    s.dP = ws.take<double>(n + 1);
    s.dw = ws.take<double>(E + 1);
    s.prop = ws.take<double>(E + 1);
    s.s1 = ws.take<double>(E + 1);
    s.S = ws.take<double>(n + 1);
    s.h = ws.take<double>(n + 1);
    s.t1 = ws.take<double>(n + 1);
    s.t2 = ws.take<double>(n + 1);
    s.y = ws.take<double>(n + 1);
    s.r = ws.take<double>(n + 1);
    s.z = ws.take<double>(n + 1);
    s.p = ws.take<double>(n + 1);
    s.q = ws.take<double>(n + 1);
    s.part = ws.take<double>(kRedBlocks + 1);
    s.sc = ws.take<double>(32);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (sgd)");
    const unsigned eb = blocks_for(E, kS);
    GR_HIP(hipMemsetAsync(s.sc, 0, sizeof(double) * 32, st));
    GR_HIP(hipMemsetAsync(s.dw, 0, sizeof(double) * (E + 1), st));
    hipLaunchKernelGGL(k_promote, dim3(blocks_for(s.nnzG, kS)), dim3(kS), 0, st, G->w, s.nnzG, s.wG);
    GR_LAUNCHED("promote");
    hipLaunchKernelGGL(k_row_sums, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, G->row_ptr,
                       (const double*)s.wG, n, s.dG);
    GR_LAUNCHED("d_G");
    GR_TRY(s.refresh_P());
    GR_TRY(s.lambda1());
    GR_TRY(s.dot(s.w, nullptr, E, SC_SUMW0));
    const double delta = pow(prm->delta_bar, 1.0 / (double)prm->k_max);
    rep->iterations = 0;
    rep->lambda_1[0] = s.read(SC_LAM1);
    double lam_prev = 0.0;
    for (int k = 0; k < prm->k_max && k < GR_SGD_MAX_ITER; ++k) {
        double lam = 0.0;
        GR_TRY(s.power_vector(prm->seed, prm->t, &lam));
        rep->lambda_n[k] = lam;
        if (k == 0) {
            hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, st, s.sc, (int)SC_LAMN,
                               (int)SC_LAMN0);
            GR_LAUNCHED("lambda0");
            hipLaunchKernelGGL(k_sgd_propose, dim3(eb), dim3(kS), 0, st, eu, ev, (const double*)s.h,
                               E, prm->alpha, (const double*)s.sc, 1, s.s1, s.dw, s.prop);
            GR_LAUNCHED("first sensitivities");
            hipLaunchKernelGGL(k_absmax_part, dim3(kRedBlocks), dim3(kS), 0, st,
                               (const double*)s.s1, E, s.part);
            GR_LAUNCHED("max |s|");
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kS), 0, st, (const double*)s.part,
                               kRedBlocks, s.sc + SC_MAXS);
            GR_LAUNCHED("max final");
            hipLaunchKernelGGL(k_set_eta, dim3(1), dim3(1), 0, st, s.sc, prm->eta_scale, E);
            GR_LAUNCHED("eta");
        } else if ((lam_prev - lam) / lam < prm->eps) {
            rep->n_lambda = k + 1;
            break;
        }
        lam_prev = lam;
        rep->n_lambda = k + 1;
        hipLaunchKernelGGL(k_sgd_propose, dim3(eb), dim3(kS), 0, st, eu, ev, (const double*)s.h, E,
                           prm->alpha, (const double*)s.sc, 0, s.s1, s.dw, s.prop);
        GR_LAUNCHED("propose");
        hipLaunchKernelGGL(k_node_sums, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, s.rpP, eoe,
                           (const double*)s.prop, n, E, s.S);
        GR_LAUNCHED("node sums");
        hipLaunchKernelGGL(k_sgd_apply, dim3(eb), dim3(kS), 0, st, eu, ev, (const double*)s.dG,
                           (const double*)s.dP, (const double*)s.S, E, delta, (const double*)s.sc,
                           s.dw, (const double*)s.prop, s.w);
        GR_LAUNCHED("apply");
        GR_TRY(s.refresh_P());
        hipLaunchKernelGGL(k_update_eta, dim3(1), dim3(1), 0, st, s.sc);
        GR_LAUNCHED("eta update");
        GR_TRY(s.lambda1());
        rep->lambda_1[k + 1] = s.read(SC_LAM1);
        rep->iterations = k + 1;
    }
    rep->cg_iterations_max = (int32_t)s.cg_iters_max;
    return GR_OK;
}

// =====================================================================
// Phase B: spectral sparsification (Sec. 3.3.2-3.3.3).  A spanning tree of
// G, then rounds of densification: the approximate criticality
// c_pq = w_G(p, q) (h_p - h_q)^2 of every edge outside the subgraph P, from
// the same h_t as Alg. 1 (t generalised power iterations), ranks the edges,
// and the most critical join P.  The tree is the maximum-weight spanning
// forest, found by Boruvka rounds: every component takes its heaviest edge
// to another component (ties to the smaller edge number, i.e. the smaller
// endpoints), the components hook along those edges and are flattened by
// pointer jumping.  With the edges in a strict order that forest is unique,
// so the result equals sequential Kruskal on the same order bit for bit.
// =====================================================================

// heavier first, then the smaller edge number
__device__ inline uint64_t tree_key(float w, int32_t e) {
    return ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(~(uint32_t)e);
}

// per row (a wave): the best key of an entry leaving the row's component;
// one atomic maximum per row on the component's slot
__global__ void __launch_bounds__(kS) k_bv_best(const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ col,
                                                const float* __restrict__ w,
                                                const int32_t* __restrict__ eoe,
                                                const int32_t* __restrict__ comp, int64_t n,
                                                unsigned long long* __restrict__ best) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    const int32_t cv = comp[v];
    uint64_t m = 0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave)
        if (comp[col[e]] != cv) {
            const uint64_t k = tree_key(w[e], eoe[e]);
            m = k > m ? k : m;
        }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const uint64_t o = ((uint64_t)(uint32_t)__shfl_xor((int)(m >> 32), off, kWave) << 32) |
                           (uint32_t)__shfl_xor((int)(uint32_t)m, off, kWave);
        m = o > m ? o : m;
    }
    if (l == 0 && m) atomicMax(best + cv, (unsigned long long)m);
}

// every root takes its best edge: nxt[c] = the component across it, the
// edge joins the forest
__global__ void k_bv_hook(const unsigned long long* __restrict__ best,
                          const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                          const int32_t* __restrict__ comp, int64_t n, int32_t* __restrict__ nxt,
                          int32_t* __restrict__ in_tree, int32_t* changed) {
    const int64_t c = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (c >= n) return;
    nxt[c] = (int32_t)c;
    if (comp[c] != c || best[c] == 0) return;
    const int32_t e = (int32_t)(~(uint32_t)(best[c] & 0xffffffffull));
    const int32_t a = comp[eu[e]], b = comp[ev[e]];
    nxt[c] = a == (int32_t)c ? b : a;
    in_tree[e] = 1;
    *changed = 1;
}

// two components that took the same edge point at each other: the smaller
// id stays a root
__global__ void k_bv_pairs(int32_t* __restrict__ nxt, int64_t n) {
    const int64_t c = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (c >= n) return;
    const int32_t d = nxt[c];
    if (d != (int32_t)c && nxt[d] == (int32_t)c && (int32_t)c < d) nxt[c] = (int32_t)c;
}

__global__ void k_bv_jump(int32_t* __restrict__ nxt, int64_t n, int32_t* changed) {
    const int64_t c = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (c >= n) return;
    const int32_t x = nxt[c], y = nxt[x];
    if (x != y) {
        nxt[c] = y;
        *changed = 1;
    }
}

__global__ void k_bv_relabel(int32_t* __restrict__ comp, const int32_t* __restrict__ nxt,
                             int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (v < n) comp[v] = nxt[comp[v]];
}

__global__ void k_iota32(int32_t* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i < n) x[i] = (int32_t)i;
}

// number of nonzero flags (0/1 values) among E
static int count_flags(const int32_t* flags, int64_t E, int64_t* out, Arena& ws, hipStream_t st) {
    *out = 0;
    if (E <= 0) return GR_OK;
    const size_t mark = ws.used;
    int32_t* tmp = ws.take<int32_t>(E + 1);
    int32_t* tot = ws.take<int32_t>(4);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (count)");
    GR_TRY(scan_exclusive_i32(flags, tmp, E, tot, ws, st));
    int32_t h = 0;
    GR_HIP(hipMemcpyAsync(&h, tot, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    *out = h;
    ws.used = mark;
    return GR_OK;
}

int spanning_forest(const gr_graph* g, const int32_t* eu, const int32_t* ev, const int32_t* eoe,
                    int32_t* in_tree, int64_t E, int64_t* n_tree, Arena& ws, hipStream_t st) {
    const int64_t n = g->n;
    const size_t mark = ws.used;
    int32_t* comp = ws.take<int32_t>(n + 1);
    int32_t* nxt = ws.take<int32_t>(n + 1);
    unsigned long long* best = ws.take<unsigned long long>(n + 1);
    int32_t* flag = ws.take<int32_t>(4);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (spanning forest)");
    const unsigned nb = blocks_for(n, kS);
    GR_HIP(hipMemsetAsync(in_tree, 0, sizeof(int32_t) * (E > 0 ? E : 1), st));
    hipLaunchKernelGGL(k_iota32, dim3(nb), dim3(kS), 0, st, comp, n);
    GR_LAUNCHED("forest components");
    for (int round = 0; round < 64; ++round) {
        GR_HIP(hipMemsetAsync(best, 0, sizeof(unsigned long long) * n, st));
        GR_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_bv_best, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                           g->col, g->w, eoe, (const int32_t*)comp, n, best);
        GR_LAUNCHED("forest best edges");
        hipLaunchKernelGGL(k_bv_hook, dim3(nb), dim3(kS), 0, st, (const unsigned long long*)best, eu,
                           ev, (const int32_t*)comp, n, nxt, in_tree, flag);
        GR_LAUNCHED("forest hook");
        int32_t hooked = 0;
        GR_HIP(hipMemcpyAsync(&hooked, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        if (!hooked) break;
        hipLaunchKernelGGL(k_bv_pairs, dim3(nb), dim3(kS), 0, st, nxt, n);
        GR_LAUNCHED("forest pairs");
        for (;;) {  // flatten: four jumps per check
            GR_HIP(hipMemsetAsync(flag + 1, 0, sizeof(int32_t), st));
            for (int k = 0; k < 4; ++k) {
                hipLaunchKernelGGL(k_bv_jump, dim3(nb), dim3(kS), 0, st, nxt, n, flag + 1);
                GR_LAUNCHED("forest jump");
            }
            int32_t moved = 0;
            GR_HIP(hipMemcpyAsync(&moved, flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            GR_HIP(hipStreamSynchronize(st));
            if (!moved) break;
        }
        hipLaunchKernelGGL(k_bv_relabel, dim3(nb), dim3(kS), 0, st, comp, (const int32_t*)nxt, n);
        GR_LAUNCHED("forest relabel");
    }
    GR_TRY(count_flags(in_tree, E, n_tree, ws, st));
    ws.used = mark;
    return GR_OK;
}

// ------------------------------------------------- subgraph from edge flags
// rows of P: the entries of G whose edge is kept, in G's order (a wave per
// row; ballots keep the order)
__global__ void __launch_bounds__(kS) k_sub_count(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ eoe,
                                                  const int32_t* __restrict__ keep, int64_t n,
                                                  int32_t* __restrict__ cnt) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    int32_t c = 0;
    for (int32_t b = rp[v]; b < rp[v + 1]; b += kWave) {
        const int32_t e = b + l;
        c += __popcll(__ballot(e < rp[v + 1] && keep[eoe[e]]));
    }
    if (l == 0) cnt[v] = c;
}

__global__ void __launch_bounds__(kS) k_sub_fill(const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ w,
                                                 const int32_t* __restrict__ eoe,
                                                 const int32_t* __restrict__ keep,
                                                 const int32_t* __restrict__ prp,
                                                 const int32_t* __restrict__ pid, int64_t n,
                                                 int32_t* __restrict__ pcol, float* __restrict__ pw,
                                                 int32_t* __restrict__ peoe) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    int32_t o = prp[v];
    for (int32_t b = rp[v]; b < rp[v + 1]; b += kWave) {
        const int32_t e = b + l;
        const bool k = e < rp[v + 1] && keep[eoe[e]];
        const uint64_t m = __ballot(k);
        if (k) {
            const int32_t at = o + (int32_t)__popcll(m & ((1ull << l) - 1ull));
            pcol[at] = col[e];
            pw[at] = w[e];
            if (peoe) peoe[at] = pid[eoe[e]];
        }
        o += (int32_t)__popcll(m);
    }
}

// P's own edge list: the kept edges of G in G's edge order
__global__ void k_sub_edges(const int32_t* __restrict__ keep, const int32_t* __restrict__ pid,
                            const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            int64_t E, int32_t* __restrict__ peu, int32_t* __restrict__ pev) {
    const int64_t e = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (e >= E || !keep[e]) return;
    peu[pid[e]] = eu[e];
    pev[pid[e]] = ev[e];
}

int subgraph(const gr_graph* g, const int32_t* eoe, const int32_t* keep, int64_t E,
             const int32_t* eu, const int32_t* ev, int32_t* prp, int32_t* pcol, float* pw,
             int32_t* peoe, int32_t* peu, int32_t* pev, int64_t* p_nnz, int64_t* p_edges,
             Arena& ws, hipStream_t st) {
    const int64_t n = g->n;
    const size_t mark = ws.used;
    int32_t* cnt = ws.take<int32_t>(n + 1);
    int32_t* pid = ws.take<int32_t>(E + 1);
    int32_t* tot = ws.take<int32_t>(4);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (subgraph)");
    hipLaunchKernelGGL(k_sub_count, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                       eoe, keep, n, cnt);
    GR_LAUNCHED("subgraph counts");
    GR_TRY(scan_exclusive_i32(cnt, prp, n, prp + n, ws, st));
    GR_TRY(scan_exclusive_i32(keep, pid, E, tot, ws, st));
    hipLaunchKernelGGL(k_sub_fill, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                       g->col, g->w, eoe, keep, (const int32_t*)prp, (const int32_t*)pid, n, pcol,
                       pw, peoe);
    GR_LAUNCHED("subgraph fill");
    if (peu && pev && E > 0) {
        hipLaunchKernelGGL(k_sub_edges, dim3(blocks_for(E, kS)), dim3(kS), 0, st, keep,
                           (const int32_t*)pid, eu, ev, E, peu, pev);
        GR_LAUNCHED("subgraph edges");
    }
    int32_t h[2] = {0, 0};
    GR_HIP(hipMemcpyAsync(&h[0], prp + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipMemcpyAsync(&h[1], tot, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    *p_nnz = h[0];
    *p_edges = h[1];
    ws.used = mark;
    return GR_OK;
}

// --------------------------------------------------- criticality and rounds
// weight of every undirected edge from its upper entry
__global__ void __launch_bounds__(kS) k_edge_w(const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ col,
                                               const float* __restrict__ w,
                                               const int32_t* __restrict__ eoe, int64_t n,
                                               float* __restrict__ wE) {
    const int64_t v = ((int64_t)blockIdx.x * kS + threadIdx.x) / kWave;
    const int l = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += kWave)
        if (col[e] > v) wE[eoe[e]] = w[e];
}

int edge_weights(const gr_graph* g, const int32_t* eoe, float* wE, hipStream_t st) {
    if (g->n == 0) return GR_OK;
    hipLaunchKernelGGL(k_edge_w, dim3(blocks_for(g->n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                       g->col, g->w, eoe, g->n, wE);
    GR_LAUNCHED("edge weights");
    return GR_OK;
}

// c_e = w_e (h_p - h_q)^2 outside P; sort keys ascending = c descending
// (edges of P last)
__global__ void k_crit_keys(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const float* __restrict__ wE, const int32_t* __restrict__ keep,
                            const double* __restrict__ h, int64_t E, double* __restrict__ crit,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t e = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (e >= E) return;
    double c = 0.0;
    if (!keep[e]) {
        const double d = h[eu[e]] - h[ev[e]];
        c = (double)wE[e] * (d * d);
    }
    if (crit) crit[e] = c;
    keys[e] = keep[e] ? ~0ull : ~(uint64_t)__double_as_longlong(c);
    vals[e] = (uint32_t)e;
}

__global__ void k_mark_top(const uint32_t* __restrict__ vals, int64_t m, int32_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * kS + threadIdx.x;
    if (i < m) keep[vals[i]] = 1;
}

size_t sparsify_workspace(int64_t n, int64_t nnz) {
    const size_t N = (size_t)n + 1, M = (size_t)nnz + 1, E = M / 2 + 1;
    size_t b = 12 * E + 4 * M                       // edge list, entry -> edge
               + 4 * N + 8 * M                      // P's CSR
               + 4 * E                              // edge weights
               + 16 * M + 80 * N                    // Alg. 1 machinery (G, P, vectors)
               + 16 * N + 8 * E                     // forest state, counts
               + 8 * E + 2 * 12 * E                 // criticality, sort keys and values
               + 4 * N + 4 * E                      // subgraph counts and edge ranks
               + 2 * 256 * 4 * (M / 2048 + 1) + M / 32 + 512 * 1024 + 8 * 4096;
    return b + b / 8 + (2u << 20);
}

int sparsify(const gr_graph* g, const gr_sparsify_params* prm, int32_t* keep, double* crit_out,
             gr_sparsify_report* rep, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    const int64_t E0 = nnz / 2;
    const size_t mark = ws.used;
    int32_t* eu = ws.take<int32_t>(E0 + 1);
    int32_t* ev = ws.take<int32_t>(E0 + 1);
    int32_t* eoe = ws.take<int32_t>(nnz + 1);
    int32_t* prp = ws.take<int32_t>(n + 1);
    int32_t* pcol = ws.take<int32_t>(nnz + 1);
    float* pw = ws.take<float>(nnz + 1);
    float* wE = ws.take<float>(E0 + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (sparsify)");
    int64_t E = 0;
    GR_TRY(edge_list(g, eu, ev, eoe, &E, ws, st));
    hipLaunchKernelGGL(k_edge_w, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                       g->col, g->w, (const int32_t*)eoe, n, wE);
    GR_LAUNCHED("edge weights");
    int64_t ntree = 0;
    GR_TRY(spanning_forest(g, eu, ev, eoe, keep, E, &ntree, ws, st));
    rep->tree_edges = ntree;
    rep->edges = ntree;
    rep->rounds = 0;
    rep->n_lambda = 0;
    // the power-vector machinery of Alg. 1 on G and the current P
    Sgd s{};
    s.n = n;
    s.nnzG = nnz;
    s.rpG = g->row_ptr;
    s.colG = g->col;
    s.rpP = prp;
    s.colP = pcol;
    s.st = st;
    s.cg_max = prm->cg_max_iter > 0 ? prm->cg_max_iter : 20000;
    s.cg_tol = prm->cg_tol > 0.0 ? prm->cg_tol : 1e-12;
    s.wG = ws.take<double>(nnz + 1);
    s.dG = ws.take<double>(n + 1);
    s.wPent = ws.take<double>(nnz + 1);
    s.dP = ws.take<double>(n + 1);
    s.h = ws.take<double>(n + 1);
    s.t1 = ws.take<double>(n + 1);
    s.y = ws.take<double>(n + 1);
    s.r = ws.take<double>(n + 1);
    s.z = ws.take<double>(n + 1);
    s.p = ws.take<double>(n + 1);
    s.q = ws.take<double>(n + 1);
    s.part = ws.take<double>(kRedBlocks + 1);
    s.sc = ws.take<double>(32);
    double* crit = ws.take<double>(E + 1);
    uint64_t* k0 = ws.take<uint64_t>(E + 1);
    uint32_t* v0 = ws.take<uint32_t>(E + 1);
    uint64_t* k1 = ws.take<uint64_t>(E + 1);
    uint32_t* v1 = ws.take<uint32_t>(E + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (sparsify rounds)");
    GR_HIP(hipMemsetAsync(s.sc, 0, sizeof(double) * 32, st));
    hipLaunchKernelGGL(k_promote, dim3(blocks_for(nnz, kS)), dim3(kS), 0, st, g->w, nnz, s.wG);
    GR_LAUNCHED("promote");
    hipLaunchKernelGGL(k_row_sums, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, g->row_ptr,
                       (const double*)s.wG, n, s.dG);
    GR_LAUNCHED("d_G");
    const int64_t per = (int64_t)ceil(prm->add_frac * (double)n);
    for (int round = 0;; ++round) {
        int64_t pnnz = 0, pedges = 0;
        GR_TRY(subgraph(g, eoe, keep, E, nullptr, nullptr, prp, pcol, pw, nullptr, nullptr,
                        nullptr, &pnnz, &pedges, ws, st));
        s.nnzP = pnnz;
        hipLaunchKernelGGL(k_promote, dim3(blocks_for(pnnz, kS)), dim3(kS), 0, st, (const float*)pw,
                           pnnz, s.wPent);
        GR_LAUNCHED("promote P");
        hipLaunchKernelGGL(k_row_sums, dim3(blocks_for(n * kWave, kS)), dim3(kS), 0, st, prp,
                           (const double*)s.wPent, n, s.dP);
        GR_LAUNCHED("d_P");
        double lam = 0.0;
        GR_TRY(s.power_vector(prm->seed, prm->t, &lam));
        if (rep->n_lambda < GR_SPARSIFY_MAX_ROUNDS + 1) rep->lambda_n[rep->n_lambda++] = lam;
        rep->edges = pedges;
        const bool last = round >= prm->rounds || lam <= prm->lambda_target || pedges >= E;
        if (last && !crit_out) break;
        hipLaunchKernelGGL(k_crit_keys, dim3(blocks_for(E, kS)), dim3(kS), 0, st, (const int32_t*)eu,
                           (const int32_t*)ev, (const float*)wE, (const int32_t*)keep,
                           (const double*)s.h, E, crit, k0, v0);
        GR_LAUNCHED("criticality");
        if (last) {  // the criticality of the final P's outside edges
            GR_HIP(hipMemcpyAsync(crit_out, crit, sizeof(double) * E, hipMemcpyDeviceToDevice, st));
            break;
        }
        GR_TRY(radix_sort_pairs(k0, v0, k1, v1, E, 64, ws, st));
        const int64_t m = std::min<int64_t>(per, E - pedges);
        hipLaunchKernelGGL(k_mark_top, dim3(blocks_for(m, kS)), dim3(kS), 0, st, (const uint32_t*)v1,
                           m, keep);
        GR_LAUNCHED("densify");
        rep->rounds = round + 1;
    }
    rep->cg_iterations_max = (int32_t)s.cg_iters_max;
    GR_HIP(hipStreamSynchronize(st));
    ws.used = mark;
    return GR_OK;
}

}  // namespace gr
