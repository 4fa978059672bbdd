// Edge-weight derivatives that serve the constrained-SGD edge scaling of
// Sec. 3.3.4 (Alg. 1): the undirected edge list of a CSR graph, FP64
// Rayleigh quotients R_i = u_i^T L(w) u_i / u_i^T B u_i with their
// edge-weight gradients (first-order eigenvalue perturbation, Sec. 3.3.3),
// and the reverse pass through the Gauss-Seidel smoothing.
#include "gr_internal.hpp"
#include "gr_device.hpp"

namespace gr {

constexpr int kA = 256;

// ------------------------------------------------------------- edge list
// Undirected edge e = (p, q), p < q, is numbered by the position of the upper
// entry (p, q) among all upper entries in CSR order; both stored entries map
// to it.
// a wave per row for both kernels: hub rows would serialise one thread
__global__ void k_upper_counts(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int64_t n, int32_t* __restrict__ flag) {
    const int64_t v = ((int64_t)blockIdx.x * kA + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    for (int32_t e = rp[v] + lane; e < rp[v + 1]; e += kWave) flag[e] = col[e] > v ? 1 : 0;
}

__global__ void k_edge_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ pos, int64_t n, int32_t* __restrict__ eu,
                            int32_t* __restrict__ ev, int32_t* __restrict__ eoe) {
    const int64_t v = ((int64_t)blockIdx.x * kA + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (v >= n) return;
    for (int32_t e = rp[v] + lane; e < rp[v + 1]; e += kWave) {
        int32_t j = col[e];
        if (j > v) {
            int32_t k = pos[e];
            eu[k] = (int32_t)v;
            ev[k] = j;
            if (eoe) eoe[e] = k;
        } else if (eoe) {
            // the partner entry (j, v) lies in row j; columns ascend there
            int32_t lo = rp[j], hi = rp[j + 1] - 1, f = -1;
            while (lo <= hi) {
                int32_t mid = lo + ((hi - lo) >> 1);
                int32_t c = col[mid];
                if (c == (int32_t)v) { f = mid; break; }
                if (c < (int32_t)v) lo = mid + 1; else hi = mid - 1;
            }
            eoe[e] = f >= 0 ? pos[f] : -1;
        }
    }
}

int edge_list(const gr_graph* g, int32_t* eu, int32_t* ev, int32_t* eoe, int64_t* n_edges, Arena& ws,
              hipStream_t st) {
    *n_edges = 0;
    if (g->nnz == 0) return GR_OK;
    size_t mark = ws.used;
    int32_t* flag = ws.take<int32_t>(g->nnz);
    int32_t* pos = ws.take<int32_t>(g->nnz + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (edge list)");
    const unsigned nb = blocks_for(g->n * kWave, kA);
    hipLaunchKernelGGL(k_upper_counts, dim3(nb), dim3(kA), 0, st, g->row_ptr, g->col, g->n, flag);
    GR_LAUNCHED("upper counts");
    GR_TRY(scan_exclusive_i32(flag, pos, g->nnz, pos + g->nnz, ws, st));
    hipLaunchKernelGGL(k_edge_fill, dim3(nb), dim3(kA), 0, st, g->row_ptr, g->col, pos, g->n, eu, ev,
                       eoe);
    GR_LAUNCHED("edge fill");
    int32_t E = 0;
    GR_HIP(hipMemcpyAsync(&E, pos + g->nnz, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    *n_edges = E;
    ws.used = mark;
    return GR_OK;
}

// set when a caller-supplied edge id lies outside [0, E); the offending
// entry is never dereferenced
__device__ int32_t g_bad_edge_id;

__global__ void k_expand_weights(const int32_t* __restrict__ eoe, int64_t nnz, int64_t E,
                                 const float* __restrict__ wE, float* __restrict__ w) {
    int64_t e = (int64_t)blockIdx.x * kA + threadIdx.x;
    if (e >= nnz) return;
    int32_t k = eoe[e];
    if (k >= 0 && k < E) {
        w[e] = wE[k];
    } else {
        w[e] = 0.0f;
        g_bad_edge_id = 1;
    }
}

static int reset_bad_edge_flag(hipStream_t st) {
    int32_t zero = 0;
    GR_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_bad_edge_id), &zero, sizeof(int32_t), 0,
                                  hipMemcpyHostToDevice, st));
    GR_HIP(hipStreamSynchronize(st));
    return GR_OK;
}

static int check_bad_edge_flag(hipStream_t st) {
    int32_t bad = 0;
    GR_HIP(hipMemcpyFromSymbolAsync(&bad, HIP_SYMBOL(g_bad_edge_id), sizeof(int32_t), 0,
                                    hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    if (bad) return set_error(GR_EINVAL, "edge_of_entry holds ids outside [0, n_edges)");
    return GR_OK;
}

int expand_weights(const int32_t* eoe, int64_t nnz, int64_t E, const float* wE, float* w,
                   hipStream_t st) {
    if (nnz == 0) return GR_OK;
    GR_TRY(reset_bad_edge_flag(st));
    hipLaunchKernelGGL(k_expand_weights, dim3(blocks_for(nnz, kA)), dim3(kA), 0, st, eoe, nnz, E, wE,
                       w);
    GR_LAUNCHED("expand weights");
    return check_bad_edge_flag(st);
}

// ------------------------------------------------------- Rayleigh quotients
constexpr int kRqBlocks = 512;

__device__ inline double block_sum_d(double v, double* sh) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kA / kWave; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// grid (kRqBlocks, m): partial sums over edges (grid-stride) of
//   num_i = sum_e w_e (u_pi - u_qi)^2   and, for B = D(w),
//   den_i = sum_e w_e (u_pi^2 + u_qi^2)  (= u_i^T D u_i).
__global__ void __launch_bounds__(kA) k_rq_edges(int64_t E, const int32_t* __restrict__ eu,
                                                 const int32_t* __restrict__ ev,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ U, int32_t m, int mode,
                                                 double* __restrict__ part_num,
                                                 double* __restrict__ part_den) {
    __shared__ double sh[kA / kWave];
    const int i = blockIdx.y;
    double num = 0.0, den = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kA + threadIdx.x; e < E; e += (int64_t)gridDim.x * kA) {
        double up = U[(int64_t)eu[e] * m + i], uq = U[(int64_t)ev[e] * m + i];
        double df = up - uq;
        num = fma(w[e] * df, df, num);
        if (mode == GR_RQ_DEGREE) den = fma(w[e], up * up + uq * uq, den);
    }
    num = block_sum_d(num, sh);
    den = block_sum_d(den, sh);
    if (threadIdx.x == 0) {
        part_num[(int64_t)i * gridDim.x + blockIdx.x] = num;
        part_den[(int64_t)i * gridDim.x + blockIdx.x] = den;
    }
}

// grid (kRqBlocks, m): partial sums of u_i^T u_i over nodes (B = I)
__global__ void __launch_bounds__(kA) k_rq_nodes(int64_t n, const double* __restrict__ U, int32_t m,
                                                 double* __restrict__ part_den) {
    __shared__ double sh[kA / kWave];
    const int i = blockIdx.y;
    double den = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * kA + threadIdx.x; v < n; v += (int64_t)gridDim.x * kA) {
        double u = U[v * m + i];
        den = fma(u, u, den);
    }
    den = block_sum_d(den, sh);
    if (threadIdx.x == 0) part_den[(int64_t)i * gridDim.x + blockIdx.x] = den;
}

__global__ void k_rq_final(const double* __restrict__ part_num, const double* __restrict__ part_den,
                           int nb, int32_t m, double* __restrict__ R, double* __restrict__ den_out) {
    int i = threadIdx.x;
    if (i >= m) return;
    double num = 0.0, den = 0.0;
    for (int b = 0; b < nb; ++b) {
        num += part_num[(int64_t)i * nb + b];
        den += part_den[(int64_t)i * nb + b];
    }
    R[i] = den != 0.0 ? num / den : 0.0;
    if (den_out) den_out[i] = den;
}

// gw_e = sum_i gR_i [ (u_pi - u_qi)^2 - (B = D: R_i (u_pi^2 + u_qi^2)) ] / den_i
__global__ void k_rq_backward(int64_t E, const int32_t* __restrict__ eu,
                              const int32_t* __restrict__ ev, const double* __restrict__ U,
                              int32_t m, int mode, const double* __restrict__ R,
                              const double* __restrict__ den, const double* __restrict__ gR,
                              double* __restrict__ gw) {
    int64_t e = (int64_t)blockIdx.x * kA + threadIdx.x;
    if (e >= E) return;
    const double* up = U + (int64_t)eu[e] * m;
    const double* uq = U + (int64_t)ev[e] * m;
    double g = 0.0;
    for (int i = 0; i < m; ++i) {
        if (den[i] == 0.0) continue;
        double df = up[i] - uq[i];
        double t = df * df;
        if (mode == GR_RQ_DEGREE) t -= R[i] * (up[i] * up[i] + uq[i] * uq[i]);
        g = fma(gR[i] / den[i], t, g);
    }
    gw[e] = g;
}

int rq_forward(int64_t n, int64_t E, const int32_t* eu, const int32_t* ev, const double* w,
               const double* U, int32_t m, int32_t mode, double* R, double* den, Arena& ws,
               hipStream_t st) {
    size_t mark = ws.used;
    double* pn = ws.take<double>((size_t)kRqBlocks * m);
    double* pd = ws.take<double>((size_t)kRqBlocks * m);
    double* pd2 = ws.take<double>((size_t)kRqBlocks * m);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (rq)");
    hipLaunchKernelGGL(k_rq_edges, dim3(kRqBlocks, m), dim3(kA), 0, st, E, eu, ev, w, U, m, mode, pn,
                       pd);
    GR_LAUNCHED("rq edges");
    if (mode == GR_RQ_IDENTITY) {
        hipLaunchKernelGGL(k_rq_nodes, dim3(kRqBlocks, m), dim3(kA), 0, st, n, U, m, pd2);
        GR_LAUNCHED("rq nodes");
        pd = pd2;
    }
    hipLaunchKernelGGL(k_rq_final, dim3(1), dim3(64), 0, st, (const double*)pn, (const double*)pd,
                       kRqBlocks, m, R, den);
    GR_LAUNCHED("rq final");
    ws.used = mark;
    return GR_OK;
}

int rq_backward(int64_t E, const int32_t* eu, const int32_t* ev, const double* U, int32_t m,
                int32_t mode, const double* R, const double* den, const double* gR, double* gw,
                hipStream_t st) {
    if (E == 0) return GR_OK;
    hipLaunchKernelGGL(k_rq_backward, dim3(blocks_for(E, kA)), dim3(kA), 0, st, E, eu, ev, U, m, mode,
                       R, den, gR, gw);
    GR_LAUNCHED("rq backward");
    return GR_OK;
}

}  // namespace gr

// ------------------------------------------- reverse pass of the smoothing
// A colour step maps row i of colour c (d_i > 0) to x_i' = sum_j w_ij x_j / d_i
// and leaves the other rows.  Its partial derivatives are
// dx_i'/dw_ij = (x_j - x_i') / d_i and dx_i'/dx_j = w_ij / d_i, and x_i' does
// not depend on the old x_i.  Undoing the steps in reverse order (sweeps
// S..1, colours C-1..0), with g = the adjoint of x_i':
//   wbar_ij += g . (x_j - x_i') / d_i          (kernel k_vjp_rows)
//   xbar_j  += (w_ij / d_i) g  for j in N(i)   (kernel k_vjp_segs, gather form:
//              each row j adds over its neighbours of colour c)
//   xbar_i   = 0.
// The state seen by step (s, c) is, in the colour-major order, rows of
// colour < c from X_s and rows of colour >= c from X_{s-1}; so the sweep
// boundary states X_0..X_S (stored, or recomputed from X_0) suffice.
namespace gr {

__global__ void k_perm_payload(const int32_t* __restrict__ rp, const uint32_t* __restrict__ perm,
                               const int32_t* __restrict__ nrp, int64_t n,
                               const int32_t* __restrict__ in, int32_t* __restrict__ out) {
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    int32_t v = (int32_t)perm[r];
    int32_t e0 = rp[v], e1 = rp[v + 1], o = nrp[r];
    for (int32_t e = e0 + lane; e < e1; e += kWave) out[o + (e - e0)] = in[e];
}

// keys (row, column) of the relabelled entries, to order each row by column
__global__ void k_row_col_keys(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int64_t n, int cb, uint64_t* __restrict__ keys,
                               uint32_t* __restrict__ vals) {
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += kWave) {
        keys[e] = ((uint64_t)r << cb) | (uint64_t)col[e];
        vals[e] = (uint32_t)e;
    }
}

__global__ void k_gather3(const uint32_t* __restrict__ order, int64_t m,
                          const int32_t* __restrict__ a, const float* __restrict__ b,
                          const int32_t* __restrict__ c, int32_t* __restrict__ a2,
                          float* __restrict__ b2, int32_t* __restrict__ c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint32_t o = order[i];
    a2[i] = a[o];
    b2[i] = b[o];
    c2[i] = c[o];
}

__device__ inline int32_t class_of(const int32_t* __restrict__ cp, int32_t C, int32_t j) {
    int32_t lo = 0, hi = C - 1;  // last c with cp[c] <= j
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (cp[mid] <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Segments: the maximal runs of one colour inside a column-sorted row. A row
// of colour-contiguous columns holds at most one run per colour, and the runs
// tile the entries in CSR order, so a run ends where the next one starts.
// A wave per row marks the first entry of every run.
__global__ void k_seg_heads(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            int64_t n, const int32_t* __restrict__ cp, int32_t C,
                            int32_t* __restrict__ head) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    const int32_t e0 = rp[r], e1 = rp[r + 1];
    for (int32_t e = e0 + lane; e < e1; e += kWave) {
        const int32_t c = class_of(cp, C, col[e]);
        head[e] = (e == e0 || col[e - 1] < cp[c]) ? 1 : 0;
    }
}

// the run starting at entry e goes to slot hpos[e], keyed by its colour
__global__ void k_seg_keys(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           int64_t n, const int32_t* __restrict__ cp, int32_t C,
                           const int32_t* __restrict__ head, const int32_t* __restrict__ hpos,
                           uint64_t* __restrict__ key, uint32_t* __restrict__ val,
                           int32_t* __restrict__ hrow, int32_t* __restrict__ hstart) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += kWave) {
        if (!head[e]) continue;
        const int32_t s = hpos[e];
        key[s] = (uint64_t)class_of(cp, C, col[e]);
        val[s] = (uint32_t)s;
        hrow[s] = (int32_t)r;
        hstart[s] = e;
    }
}

// record k = the k-th run in (colour, entry) order: (row, first, end)
__global__ void k_seg_records(const uint32_t* __restrict__ order, int64_t nh, int64_t nnz,
                              const int32_t* __restrict__ hrow, const int32_t* __restrict__ hstart,
                              int32_t* __restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nh) return;
    const uint32_t s = order[k];
    rec[3 * k] = hrow[s];
    rec[3 * k + 1] = hstart[s];
    rec[3 * k + 2] = (int64_t)s + 1 < nh ? hstart[s + 1] : (int32_t)nnz;
}

// segp[c] = first record of colour c (colour-sorted keys); k runs over [0, nh]
__global__ void k_seg_bounds(const uint64_t* __restrict__ skey, int64_t nh, int32_t C,
                             int32_t* __restrict__ segp) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nh) return;
    const int32_t lo = k == 0 ? -1 : (int32_t)skey[k - 1];
    const int32_t hi = k == nh ? C : (int32_t)skey[k];
    for (int32_t c = lo + 1; c <= hi; ++c) segp[c] = (int32_t)k;
}

template <int E>
__device__ inline void load_f32(const float* __restrict__ A, int64_t row, int K, int q, float* v) {
#pragma unroll
    for (int i = 0; i < E; i += 4) {
        float4 t = *reinterpret_cast<const float4*>(A + row * K + q * E + i);
        v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
    }
}
template <int E>
__device__ inline void store_f32(float* __restrict__ A, int64_t row, int K, int q, const float* v) {
#pragma unroll
    for (int i = 0; i < E; i += 4)
        *reinterpret_cast<float4*>(A + row * K + q * E + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
}

// rows [lo, hi) of colour c; L = Q*P lanes per row
template <int Q, int P, int DT>
__global__ void __launch_bounds__(256) k_vjp_rows(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const void* __restrict__ Xs,
                                                  const void* __restrict__ Xp, int32_t K, int64_t clo,
                                                  int64_t lo, int64_t hi, const float* __restrict__ dw,
                                                  float* __restrict__ xbar, float* __restrict__ H,
                                                  float* __restrict__ ge) {
    constexpr int L = Q * P;
    constexpr int RPW = kWave / L;
    constexpr int E = Chunk<DT>::E;
    const int lane = threadIdx.x & (kWave - 1);
    const int l = lane % L;
    const int p = l / Q, q = l % Q;
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    const int64_t r = lo + wave * RPW + lane / L;
    if (r >= hi) return;
    const int32_t e0 = rp[r], e1 = rp[r + 1];
    const float d = dw[r];
    if (!(d > 0.0f)) return;  // no equation: the step leaves this row alone
    float g[E], xi[E];
    load_f32<E>(xbar, r, K, q, g);
    Chunk<DT>::load(Xs, r, K, q, xi);
    const int32_t trips = (e1 - e0 + P - 1) / P;
    for (int32_t t = 0; t < trips; ++t) {
        int32_t e = e0 + p + t * P;
        bool ok = e < e1;
        int32_t j = ok ? col[e] : (int32_t)r;
        float xj[E];
        Chunk<DT>::load(j < clo ? Xs : Xp, j, K, q, xj);
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < E; ++i) s = __fmaf_rn(g[i], xj[i] - xi[i], s);
        s = qsum<Q>(s);
        if (ok && q == 0) ge[e] += s / d;
    }
    if (p == 0) {
        float h[E], z[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            h[i] = g[i] / d;
            z[i] = 0.0f;
        }
        store_f32<E>(H, r, K, q, h);
        store_f32<E>(xbar, r, K, q, z);
    }
}

// The rows of degree above kLongRow (the colour's first rows: its degree
// tiers come in decreasing order) take two launches, so that a hub row is
// spread over many workgroups: the first sets H_i = xbar_i / d_i and clears
// xbar_i, then every entry of those rows, Q lanes each, adds
// H_i . (x_j - x_i) to its gradient.  Weights are positive, so d_i > 0.
template <int Q, int DT>
__global__ void k_vjp_long_rows(const float* __restrict__ dw, int32_t K, int64_t lo, int64_t hi,
                                float* __restrict__ xbar, float* __restrict__ H) {
    constexpr int E = Chunk<DT>::E;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = lo + t / Q;
    const int q = (int)(t % Q);
    if (r >= hi) return;
    const float d = dw[r];
    float h[E], z[E];
    load_f32<E>(xbar, r, K, q, h);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        h[i] = h[i] / d;
        z[i] = 0.0f;
    }
    store_f32<E>(H, r, K, q, h);
    store_f32<E>(xbar, r, K, q, z);
}

// entries [rp[lo], rp[hi]) of the long rows [lo, hi)
template <int Q, int DT>
__global__ void __launch_bounds__(256) k_vjp_long_edges(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const void* __restrict__ Xs,
    const void* __restrict__ Xp, int32_t K, int64_t clo, int64_t lo, int64_t hi, int64_t ebeg,
    int64_t eend, const float* __restrict__ H, float* __restrict__ ge) {
    constexpr int E = Chunk<DT>::E;
    const int q = threadIdx.x % Q;
    const int64_t e = ebeg + ((int64_t)blockIdx.x * 256 + threadIdx.x) / Q;
    if (e >= eend) return;
    int64_t a = lo, b = hi - 1;  // the row holding e: last r with rp[r] <= e
    while (a < b) {
        const int64_t m = (a + b + 1) >> 1;
        if (rp[m] <= e) a = m; else b = m - 1;
    }
    const int64_t r = a;
    const int32_t j = col[e];
    float h[E], xi[E], xj[E];
    load_f32<E>(H, r, K, q, h);
    Chunk<DT>::load(Xs, r, K, q, xi);
    Chunk<DT>::load(j < clo ? Xs : Xp, j, K, q, xj);
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < E; ++i) s = __fmaf_rn(h[i], xj[i] - xi[i], s);
    s = qsum<Q>(s);
    if (q == 0) ge[e] += s;
}

// d_i = sum_j w_ij, a wave per row; constant over the sweeps
__global__ void k_row_weight(const int32_t* __restrict__ rp, const float* __restrict__ w, int64_t n,
                             float* __restrict__ dw) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    float d = 0.0f;
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += kWave) d += w[e];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) d += __shfl_xor(d, off, kWave);
    if (lane == 0) dw[r] = d;
}

// one row-group per segment (row j, entries [a, b) whose columns have colour c)
template <int Q, int P, int E>
__global__ void __launch_bounds__(256) k_vjp_segs(const int32_t* __restrict__ rec, int64_t nrec,
                                                  const int32_t* __restrict__ col,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ H, int32_t K,
                                                  float* __restrict__ xbar) {
    constexpr int L = Q * P;
    constexpr int RPW = kWave / L;
    const int lane = threadIdx.x & (kWave - 1);
    const int l = lane % L;
    const int p = l / Q, q = l % Q;
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    const int64_t k = wave * RPW + lane / L;
    if (k >= nrec) return;
    const int32_t row = rec[3 * k], a = rec[3 * k + 1], b = rec[3 * k + 2];
    float acc[E];
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = 0.0f;
    for (int32_t e = a + p; e < b; e += P) {
        float h[E];
        load_f32<E>(H, col[e], K, q, h);
        const float wt = w[e];
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] = __fmaf_rn(wt, h[i], acc[i]);
    }
#pragma unroll
    for (int off = Q; off < L; off <<= 1)
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] += __shfl_xor(acc[i], off, kWave);
    if (p == 0) {
        float x[E];
        load_f32<E>(xbar, row, K, q, x);
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] += acc[i];
        store_f32<E>(xbar, row, K, q, x);
    }
}

// the two relabelled entries of each undirected edge: slot 0 = the entry
// whose original row is the smaller endpoint
__global__ void k_edge_slots(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ eoe, const int32_t* __restrict__ perm,
                             int64_t n, int64_t E, int32_t* __restrict__ slots) {
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    int lane = threadIdx.x & (kWave - 1);
    if (r >= n) return;
    const int32_t orow = perm[r];
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += kWave) {
        int32_t k = eoe[e];
        if (k >= 0 && k < E) slots[2 * k + (orow < perm[col[e]] ? 0 : 1)] = e;
        else g_bad_edge_id = 1;
    }
}

__global__ void k_edge_grad(const int32_t* __restrict__ slots, const float* __restrict__ ge,
                            int64_t E, float* __restrict__ gw) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < E) gw[k] = ge[slots[2 * k]] + ge[slots[2 * k + 1]];
}

__global__ void k_zero_f32(float* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

static int pick_p_vjp(int Q, double mean_deg) {
    int P = 1;
    while (P * 2 <= mean_deg && Q * P * 2 <= kWave) P *= 2;
    return P;
}

template <int Q, int DT>
static int vjp_launch_rows(int P, const gr_graph* g, const void* Xs, const void* Xp, int K,
                           int64_t clo, int64_t lo, int64_t hi, const float* dw, float* xbar,
                           float* H, float* ge, hipStream_t st) {
    if (hi <= lo) return GR_OK;
    const int64_t waves = ((hi - lo) * Q * P + kWave - 1) / kWave;
    dim3 grid(blocks_for(waves * kWave, 256));
#define GR_VR(PP)                                                                                \
    case PP:                                                                                    \
        if constexpr (Q * PP <= kWave)                                                          \
            hipLaunchKernelGGL((k_vjp_rows<Q, PP, DT>), grid, dim3(256), 0, st, g->row_ptr, g->col, \
                               Xs, Xp, K, clo, lo, hi, dw, xbar, H, ge);                         \
        break;
    switch (P) {
        GR_VR(1) GR_VR(2) GR_VR(4) GR_VR(8) GR_VR(16) GR_VR(32) GR_VR(64)
        default: return set_error(GR_EINVAL, "bad lane split");
    }
#undef GR_VR
    GR_LAUNCHED("vjp rows");
    return GR_OK;
}

template <int Q, int E>
static int vjp_launch_segs(int P, const int32_t* rec, int64_t nrec, const gr_graph* g,
                           const float* H, int K, float* xbar, hipStream_t st) {
    if (nrec <= 0) return GR_OK;
    const int64_t waves = (nrec * Q * P + kWave - 1) / kWave;
    dim3 grid(blocks_for(waves * kWave, 256));
#define GR_VS(PP)                                                                                 \
    case PP:                                                                                     \
        if constexpr (Q * PP <= kWave)                                                           \
            hipLaunchKernelGGL((k_vjp_segs<Q, PP, E>), grid, dim3(256), 0, st, rec, nrec, g->col,  \
                               g->w, H, K, xbar);                                                 \
        break;
    switch (P) {
        GR_VS(1) GR_VS(2) GR_VS(4) GR_VS(8) GR_VS(16) GR_VS(32) GR_VS(64)
        default: return set_error(GR_EINVAL, "bad lane split");
    }
#undef GR_VS
    GR_LAUNCHED("vjp segments");
    return GR_OK;
}

size_t vjp_workspace(int64_t n, int64_t nnz, int32_t K, int32_t dtype, int32_t S, int32_t store) {
    const size_t N = (size_t)n + 1, M = (size_t)nnz + 1;
    const size_t xb = N * (size_t)K * (dtype == GR_BF16 ? 2 : 4) + 256;
    const size_t fb = N * (size_t)K * 4 + 256;
    size_t b = 4 * N * 3 + 8 * M          // relabelled graph
               + 12 * M                   // column-sorted col / w / eoe
               + 12 * M                   // segment records
               + 4 * M                    // per-entry gradients
               + 8 * (M / 2 + 1)          // edge slots
               + (size_t)(store ? S + 1 : 3) * xb + 2 * fb  // states, xbar, H
               + 4 * N                    // weighted degrees
               + 48 * M + 64 * N;         // sort / relabel / segment temporaries
    return b + b / 16 + (16u << 20);
}

template <int Q, int DT>
static int vjp_impl(const OrderedGraph* og, const int32_t* rec, const std::vector<int64_t>& seg_ptr,
                    int K, int S, int store, void* states, size_t xbytes, const float* dw, float* xbar,
                    float* H, float* ge, Arena& ws, hipStream_t st) {
    constexpr int E = Chunk<DT>::E;
    const int C = og->n_colours;
    std::vector<int> Prow(C), Pseg(C);
    for (int c = 0; c < C; ++c) {
        int64_t rows = og->class_ptr_h[c + 1] - og->class_ptr_h[c];
        Prow[c] = pick_p_vjp(Q, rows > 0 ? (double)og->class_nnz_h[c] / (double)rows : 1.0);
        int64_t ns = seg_ptr[c + 1] - seg_ptr[c];
        Pseg[c] = pick_p_vjp(Q, ns > 0 ? (double)og->class_nnz_h[c] / (double)ns : 1.0);
    }
    char* base = (char*)states;
    auto state = [&](int s) { return (void*)(base + (size_t)s * xbytes); };
    // states: store mode keeps X_0..X_S; recompute mode keeps X_0 in slot 0
    // and rebuilds X_{s-1} (slot 1) and X_s (slot 2) for every sweep s
    if (store) {
        for (int s = 1; s <= S; ++s) {
            GR_HIP(hipMemcpyAsync(state(s), state(s - 1), xbytes, hipMemcpyDeviceToDevice, st));
            GR_TRY(smooth_ordered(og, K, 1, DT, state(s), ws, st));
        }
    }
    for (int s = S; s >= 1; --s) {
        const void *Xs, *Xp;
        if (store) {
            Xs = state(s);
            Xp = state(s - 1);
        } else {
            GR_HIP(hipMemcpyAsync(state(1), state(0), xbytes, hipMemcpyDeviceToDevice, st));
            GR_TRY(smooth_ordered(og, K, s - 1, DT, state(1), ws, st));
            GR_HIP(hipMemcpyAsync(state(2), state(1), xbytes, hipMemcpyDeviceToDevice, st));
            GR_TRY(smooth_ordered(og, K, 1, DT, state(2), ws, st));
            Xs = state(2);
            Xp = state(1);
        }
        for (int c = C - 1; c >= 0; --c) {
            const int64_t clo = og->class_ptr_h[c], chi = og->class_ptr_h[c + 1];
            const int64_t mid = og->tier_ptr_h[(size_t)c * kNT + kLongTiers];  // end of long rows
            if (mid > clo) {
                hipLaunchKernelGGL((k_vjp_long_rows<Q, DT>), dim3(blocks_for((mid - clo) * Q, 256)),
                                   dim3(256), 0, st, dw, K, clo, mid, xbar, H);
                GR_LAUNCHED("vjp long rows");
                const int64_t ebeg = og->class_e_h[c], eend = ebeg + og->long_nnz_h[c];
                hipLaunchKernelGGL((k_vjp_long_edges<Q, DT>),
                                   dim3(blocks_for((eend - ebeg) * Q, 256)), dim3(256), 0, st,
                                   og->g.row_ptr, og->g.col, Xs, Xp, K, clo, clo, mid, ebeg, eend,
                                   (const float*)H, ge);
                GR_LAUNCHED("vjp long edges");
            }
            GR_TRY((vjp_launch_rows<Q, DT>(Prow[c], &og->g, Xs, Xp, K, clo, mid, chi, dw, xbar, H,
                                           ge, st)));
            GR_TRY((vjp_launch_segs<Q, E>(Pseg[c], rec + 3 * seg_ptr[c], seg_ptr[c + 1] - seg_ptr[c],
                                          &og->g, H, K, xbar, st)));
        }
    }
    return GR_OK;
}

int smooth_vjp(const gr_graph* g, const int32_t* eoe, int64_t E, const int32_t* colours, int32_t C,
               int32_t K, int32_t S, int32_t dtype, const void* X0, const float* Gc, float* gw,
               float* gX0, int32_t store, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    GR_TRY(validate_colouring(g, colours, C, ws, st));
    OrderedGraph og;
    GR_TRY(order_by_colour(g, colours, C, &og, ws, st));
    // per-entry edge ids in the relabelled order, then each row by column
    int32_t* eoe_r = ws.take<int32_t>(nnz + 1);
    int32_t* col_s = ws.take<int32_t>(nnz + 1);
    float* w_s = ws.take<float>(nnz + 1);
    int32_t* eoe_s = ws.take<int32_t>(nnz + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp)");
    if (nnz > 0) {
        size_t mark = ws.used;
        uint64_t* k0 = ws.take<uint64_t>(nnz);
        uint32_t* v0 = ws.take<uint32_t>(nnz);
        uint64_t* k1 = ws.take<uint64_t>(nnz);
        uint32_t* v1 = ws.take<uint32_t>(nnz);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp sort)");
        const unsigned wb = blocks_for(n * kWave, 256);
        hipLaunchKernelGGL(k_perm_payload, dim3(wb), dim3(256), 0, st, g->row_ptr,
                           (const uint32_t*)og.perm, og.g.row_ptr, n, eoe, eoe_r);
        GR_LAUNCHED("perm payload");
        const int cb = bits_for(n);
        hipLaunchKernelGGL(k_row_col_keys, dim3(wb), dim3(256), 0, st, og.g.row_ptr, og.g.col, n, cb,
                           k0, v0);
        GR_LAUNCHED("row col keys");
        GR_TRY(radix_sort_pairs(k0, v0, k1, v1, nnz, 2 * cb, ws, st));
        hipLaunchKernelGGL(k_gather3, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, (const uint32_t*)v1,
                           nnz, og.g.col, og.g.w, (const int32_t*)eoe_r, col_s, w_s, eoe_s);
        GR_LAUNCHED("gather sorted rows");
        ws.used = mark;
    }
    og.g.col = col_s;
    og.g.w = w_s;
    // colour segments of every row, grouped by colour
    std::vector<int32_t> cp32(C + 1);
    for (int c = 0; c <= C; ++c) cp32[c] = (int32_t)og.class_ptr_h[c];
    int32_t* cp = ws.take<int32_t>(C + 1);
    int32_t* segp = ws.take<int32_t>(C + 1);
    int32_t* rec = ws.take<int32_t>(3 * (nnz + 1));
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp segments)");
    GR_HIP(hipMemcpyAsync(cp, cp32.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice, st));
    std::vector<int64_t> seg_ptr(C + 1, 0);
    if (nnz > 0) {
        size_t mark = ws.used;
        int32_t* head = ws.take<int32_t>(nnz);
        int32_t* hpos = ws.take<int32_t>(nnz + 1);
        uint64_t* k0 = ws.take<uint64_t>(nnz);
        uint32_t* v0 = ws.take<uint32_t>(nnz);
        uint64_t* k1 = ws.take<uint64_t>(nnz);
        uint32_t* v1 = ws.take<uint32_t>(nnz);
        int32_t* hrow = ws.take<int32_t>(nnz);
        int32_t* hstart = ws.take<int32_t>(nnz);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp segments)");
        const unsigned wb = blocks_for(n * kWave, 256);
        hipLaunchKernelGGL(k_seg_heads, dim3(wb), dim3(256), 0, st, og.g.row_ptr, og.g.col, n,
                           (const int32_t*)cp, C, head);
        GR_LAUNCHED("segment heads");
        GR_TRY(scan_exclusive_i32(head, hpos, nnz, hpos + nnz, ws, st));
        int32_t nh32 = 0;
        GR_HIP(hipMemcpyAsync(&nh32, hpos + nnz, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        const int64_t nh = nh32;
        hipLaunchKernelGGL(k_seg_keys, dim3(wb), dim3(256), 0, st, og.g.row_ptr, og.g.col, n,
                           (const int32_t*)cp, C, (const int32_t*)head, (const int32_t*)hpos, k0, v0,
                           hrow, hstart);
        GR_LAUNCHED("segment keys");
        GR_TRY(radix_sort_pairs(k0, v0, k1, v1, nh, bits_for(C), ws, st));
        hipLaunchKernelGGL(k_seg_records, dim3(blocks_for(nh, 256)), dim3(256), 0, st,
                           (const uint32_t*)v1, nh, nnz, (const int32_t*)hrow,
                           (const int32_t*)hstart, rec);
        GR_LAUNCHED("segment records");
        hipLaunchKernelGGL(k_seg_bounds, dim3(blocks_for(nh + 1, 256)), dim3(256), 0, st,
                           (const uint64_t*)k1, nh, C, segp);
        GR_LAUNCHED("segment bounds");
        std::vector<int32_t> hs(C + 1);
        GR_HIP(hipMemcpyAsync(hs.data(), segp, sizeof(int32_t) * (C + 1), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        for (int c = 0; c <= C; ++c) seg_ptr[c] = hs[c];
        ws.used = mark;
    }
    // states, adjoints, per-entry gradients
    const size_t xbytes = (size_t)n * K * (dtype == GR_BF16 ? 2 : 4);
    void* states = ws.take<char>((size_t)(store ? S + 1 : 3) * ((xbytes + 255) & ~size_t(255)));
    float* xbar = ws.take<float>((size_t)n * K + 4);
    float* H = ws.take<float>((size_t)n * K + 4);
    float* dw = ws.take<float>(n + 1);
    float* ge = ws.take<float>(nnz + 1);
    int32_t* slots = ws.take<int32_t>(2 * (E + 1));
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp states)");
    const size_t xstride = (xbytes + 255) & ~size_t(255);
    GR_TRY(permute_rows(X0, states, og.perm, n, (size_t)K * (dtype == GR_BF16 ? 2 : 4), 0, st));
    GR_TRY(permute_rows(Gc, xbar, og.perm, n, (size_t)K * 4, 0, st));
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(nnz + 1, 256)), dim3(256), 0, st, ge, nnz + 1);
    GR_LAUNCHED("zero");
    if (n > 0) {
        hipLaunchKernelGGL(k_row_weight, dim3(blocks_for(n * kWave, 256)), dim3(256), 0, st,
                           og.g.row_ptr, og.g.w, n, dw);
        GR_LAUNCHED("row weights");
    }
    const int Q = K * (dtype == GR_BF16 ? 2 : 4) / 16;
#define GR_VJ(QQ, DD) \
    case QQ: GR_TRY((vjp_impl<QQ, DD>(&og, rec, seg_ptr, K, S, store, states, xstride, dw, xbar, H, ge, ws, st))); break;
    if (dtype == GR_BF16) {
        switch (Q) {
            GR_VJ(1, GR_BF16) GR_VJ(2, GR_BF16) GR_VJ(4, GR_BF16) GR_VJ(8, GR_BF16)
            default: return set_error(GR_EUNSUP, "unsupported K");
        }
    } else {
        switch (Q) {
            GR_VJ(1, GR_F32) GR_VJ(2, GR_F32) GR_VJ(4, GR_F32) GR_VJ(8, GR_F32) GR_VJ(16, GR_F32)
            default: return set_error(GR_EUNSUP, "unsupported K");
        }
    }
#undef GR_VJ
    GR_TRY(permute_rows(xbar, gX0, og.perm, n, (size_t)K * 4, 1, st));
    if (E > 0) {
        GR_TRY(fill_i32(slots, 0, 2 * E, st));  // unmatched slots read entry 0, never garbage
        GR_TRY(reset_bad_edge_flag(st));
        hipLaunchKernelGGL(k_edge_slots, dim3(blocks_for(n * kWave, 256)), dim3(256), 0, st,
                           og.g.row_ptr, og.g.col, (const int32_t*)eoe_s, og.perm, n, E, slots);
        GR_LAUNCHED("edge slots");
        GR_TRY(check_bad_edge_flag(st));
        hipLaunchKernelGGL(k_edge_grad, dim3(blocks_for(E, 256)), dim3(256), 0, st,
                           (const int32_t*)slots, (const float*)ge, E, gw);
        GR_LAUNCHED("edge grad");
    }
    GR_HIP(hipStreamSynchronize(st));  // host vectors above end here
    return GR_OK;
}

}  // namespace gr
