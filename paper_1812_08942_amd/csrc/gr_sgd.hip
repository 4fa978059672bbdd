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
    const unsigned nb = blocks_for(n, kS), eb = blocks_for(E, kS);
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
        // h_t: t generalised power iterations from the centred h_0
        hipLaunchKernelGGL(k_init_h, dim3(nb), dim3(kS), 0, st, n, prm->seed, s.h);
        GR_LAUNCHED("h0");
        GR_TRY(s.centre(s.h));
        for (int t = 0; t < prm->t; ++t) {
            GR_TRY(s.lapG(s.h, s.t1));
            GR_TRY(s.centre(s.t1));
            GR_TRY(s.solve(s.t1, s.h));
        }
        GR_TRY(s.lapP(s.h, s.t1));
        GR_TRY(s.dot(s.h, s.t1, n, SC_HLH));
        hipLaunchKernelGGL(k_normalise, dim3(nb), dim3(kS), 0, st, s.h, n, (const double*)s.sc);
        GR_LAUNCHED("normalise");
        GR_TRY(s.lapG(s.h, s.t1));
        GR_TRY(s.dot(s.h, s.t1, n, SC_LAMN));
        const double lam = s.read(SC_LAMN);
        if (!(lam == lam)) return set_error(GR_EHIP, "lambda_n is not finite");
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

}  // namespace gr
