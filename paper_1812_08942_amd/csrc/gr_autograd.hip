// Edge-weight derivatives that serve the constrained-SGD edge scaling of
// Sec. 3.3.4 (Alg. 1): the undirected edge list of a CSR graph, FP64
// Rayleigh quotients R_i = u_i^T L(w) u_i / u_i^T B u_i with their
// edge-weight gradients (first-order eigenvalue perturbation, Sec. 3.3.3),
// and the reverse pass through the Gauss-Seidel smoothing.
#include "gr_internal.hpp"
#include "gr_device.hpp"

#include <mutex>

namespace gr {

constexpr int kA = 256;

// lanes per row for the row-walking kernels below: one below a mean degree
// of 8 (extra lanes only add waves there), else a power of two up to a
// wave, about half the mean degree (hub rows loop)
inline int lanes_per_row(int64_t n, int64_t nnz) {
    if (n <= 0 || nnz < 8 * n) return 1;
    int G = 4;
    while (G < kWave && G * 2 <= nnz / n) G *= 2;
    return G;
}

// ------------------------------------------------------------- edge list
// Undirected edge e = (p, q), p < q, is numbered by the position of the upper
// entry (p, q) among all upper entries in CSR order; both stored entries map
// to it.
// G lanes per row for both kernels (one thread would serialise a hub row)
__global__ void k_upper_counts(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int64_t n, int G, int32_t* __restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * kA + threadIdx.x;
    const int64_t v = t / G;
    const int lane = (int)(t % G);
    if (v >= n) return;
    for (int32_t e = rp[v] + lane; e < rp[v + 1]; e += G) flag[e] = col[e] > v ? 1 : 0;
}

__global__ void k_edge_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ pos, int64_t n, int G,
                            int32_t* __restrict__ eu, int32_t* __restrict__ ev,
                            int32_t* __restrict__ eoe) {
    const int64_t t = (int64_t)blockIdx.x * kA + threadIdx.x;
    const int64_t v = t / G;
    const int lane = (int)(t % G);
    if (v >= n) return;
    for (int32_t e = rp[v] + lane; e < rp[v + 1]; e += G) {
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
    const int G = lanes_per_row(g->n, g->nnz);
    const unsigned nb = blocks_for(g->n * G, kA);
    hipLaunchKernelGGL(k_upper_counts, dim3(nb), dim3(kA), 0, st, g->row_ptr, g->col, g->n, G, flag);
    GR_LAUNCHED("upper counts");
    GR_TRY(scan_exclusive_i32(flag, pos, g->nnz, pos + g->nnz, ws, st));
    hipLaunchKernelGGL(k_edge_fill, dim3(nb), dim3(kA), 0, st, g->row_ptr, g->col, pos, g->n, G, eu,
                       ev, eoe);
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

// ------------------------------------- Rayleigh quotients, no allocation
// The scratch of rq_forward (three per-block partial-sum arrays) for the
// widest block, m = 64, in a file-scope device array: one copy per GPU,
// held until the process ends.  Host code never passes the array's name to
// a kernel (in host code it is a stand-in, not a device address); it looks
// up the array's address on each device once, with that device current,
// and passes that pointer instead.
constexpr size_t kRqScratchPart = ((size_t)kRqBlocks * 64 * sizeof(double) + 255) & ~size_t(255);
constexpr size_t kRqScratchBytes = 3 * kRqScratchPart;
static __device__ __align__(256) unsigned char scratch[kRqScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_on_current_device(void** out) {
    int dev = 0;
    GR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(GR_EINVAL, "device %d: at most %d devices are supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(GR_EHIP, "no device address for the static scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GR_OK;
}

size_t rq_forward_scratch_bytes(int32_t m) {
    Arena sizing(nullptr, ~size_t(0));
    for (int i = 0; i < 3; ++i) sizing.take<double>((size_t)kRqBlocks * (size_t)(m > 0 ? m : 0));
    return sizing.used;
}

size_t rq_forward_scratch_capacity() { return kRqScratchBytes; }

int rq_forward_noalloc(int64_t n, int64_t E, const int32_t* eu, const int32_t* ev, const double* w,
                       const double* U, int32_t m, int32_t mode, double* R, double* den,
                       hipStream_t st) {
    const size_t need = rq_forward_scratch_bytes(m);
    if (need > kRqScratchBytes)
        return set_error(GR_EINVAL, "m = %d needs %zu scratch bytes; the static scratch holds %zu",
                         m, need, kRqScratchBytes);
    void* p = nullptr;
    GR_TRY(scratch_on_current_device(&p));
    Arena A(p, kRqScratchBytes);
    return rq_forward(n, E, eu, ev, w, U, m, mode, R, den, A, st);
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
// not depend on the old x_i.  The steps are undone in reverse order (sweeps
// S..1, colours C-1..0) in pull form.  Let g_i be the adjoint of the value
// x_i^s that step (s, c) gives row i, and h_i = g_i / d_i.  That value is
// read by the steps of sweep s with a larger colour and by the steps of
// sweep s+1 with a smaller one, so
//   g_i = [s = S] G_i + sum_{j in N(i)} w_ij h_j,
// with h_j from sweep s when colour(j) > c and from sweep s+1 when
// colour(j) < c.  One array H holds exactly that: in reverse order, step
// (s, c) runs after the larger colours of sweep s have rewritten their rows
// and before the smaller colours of sweep s replace their sweep-(s+1)
// values (H starts at zero: there is no sweep S+1).  Then
//   wbar_ij += h_i . (x_j - x_i')   for j in N(i),
// and, once sweep 1 is undone, x_j^0 has been read only by the sweep-1 steps
// of smaller colours:  gX0_j = sum_{i in N(j), colour(i) < colour(j)} w_ij h_i
// (a row without neighbours keeps G_j).  The state seen by step (s, c) is, in
// the colour-major order, rows of colour < c from X_s and rows of colour
// >= c from X_{s-1}; so the sweep-boundary states X_0..X_S (stored, or
// recomputed from X_0) suffice.  No value is accumulated by atomics and no
// array is written by two steps of one launch (a colour class has no inner
// edges).
namespace gr {

__global__ void k_perm_payload(const int32_t* __restrict__ rp, const uint32_t* __restrict__ perm,
                               const int32_t* __restrict__ nrp, int64_t n, int G,
                               const int32_t* __restrict__ in, int32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int lane = (int)(t % G);
    if (r >= n) return;
    int32_t v = (int32_t)perm[r];
    int32_t e0 = rp[v], e1 = rp[v + 1], o = nrp[r];
    for (int32_t e = e0 + lane; e < e1; e += G) out[o + (e - e0)] = in[e];
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

// d_i = sum_j w_ij, G lanes per row; constant over the sweeps
__global__ void k_row_weight(const int32_t* __restrict__ rp, const float* __restrict__ w, int64_t n,
                             int G, float* __restrict__ dw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int lane = (int)(t % G);
    if (r >= n) return;  // G divides the wave: a row's lanes leave together
    float d = 0.0f;
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += G) d += w[e];
    for (int off = 1; off < G; off <<= 1) d += __shfl_xor(d, off, kWave);
    if (lane == 0) dw[r] = d;
}

// trips (entries per lane) up to which a reverse step keeps the gathered
// state rows in registers instead of a second pass over the row: 32 values
// per lane (8 float32 or 4 bfloat16 chunks)
template <int DT>
constexpr int vjp_keep() { return 32 / Chunk<DT>::E; }

// Rows [lo, hi) of colour c with degree <= kLongRow, L = Q*P lanes per row.
// FINAL = 0: the reverse step (G = the cotangent in the last sweep, else
// null).  FINAL = 1: gX0 of those rows into out.
template <int Q, int P, int DT, int FINAL>
__global__ void __launch_bounds__(256) k_vjp_rows(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const float* __restrict__ w,
    const void* __restrict__ Xs, const void* __restrict__ Xp, int32_t K, int64_t clo, int64_t lo,
    int64_t hi, const float* __restrict__ dw, const float* __restrict__ G, float* __restrict__ H,
    float* __restrict__ ge, float* __restrict__ out) {
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
    if (!(d > 0.0f)) {  // no neighbours: no step changes this row
        if (FINAL && p == 0) {
            float gi[E];
            load_f32<E>(G, r, K, q, gi);
            store_f32<E>(out, r, K, q, gi);
        }
        return;
    }
    float acc[E];
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = 0.0f;
    const int32_t trips = (e1 - e0 + P - 1) / P;  // the same for every lane of the row
    if constexpr (!FINAL) {
        constexpr int kKeep = vjp_keep<DT>();
        if (trips <= kKeep) {
            // one pass: the state rows x_j are gathered with h_j and kept for
            // the gradient
            float xj[kKeep][E];
#pragma unroll
            for (int t = 0; t < kKeep; ++t) {
                if (t < trips) {
                    const int32_t e = e0 + p + t * P;
                    const bool ok = e < e1;
                    const int32_t j = ok ? col[e] : (int32_t)r;
                    Chunk<DT>::load(j < clo ? Xs : Xp, j, K, q, xj[t]);
                    if (ok) {
                        float hj[E];
                        load_f32<E>(H, j, K, q, hj);
                        const float wt = w[e];
#pragma unroll
                        for (int i = 0; i < E; ++i) acc[i] = __fmaf_rn(wt, hj[i], acc[i]);
                    }
                }
            }
#pragma unroll
            for (int off = Q; off < L; off <<= 1)
#pragma unroll
                for (int i = 0; i < E; ++i) acc[i] += __shfl_xor(acc[i], off, kWave);
            if (G) {
                float gi[E];
                load_f32<E>(G, r, K, q, gi);
#pragma unroll
                for (int i = 0; i < E; ++i) acc[i] += gi[i];
            }
            float h[E], xi[E];
#pragma unroll
            for (int i = 0; i < E; ++i) h[i] = acc[i] / d;
            if (p == 0) store_f32<E>(H, r, K, q, h);
            Chunk<DT>::load(Xs, r, K, q, xi);
#pragma unroll
            for (int t = 0; t < kKeep; ++t) {
                if (t < trips) {
                    const int32_t e = e0 + p + t * P;
                    float sdot = 0.0f;
#pragma unroll
                    for (int i = 0; i < E; ++i) sdot = __fmaf_rn(h[i], xj[t][i] - xi[i], sdot);
                    sdot = qsum<Q>(sdot);
                    if (e < e1 && q == 0) ge[e] += sdot;
                }
            }
            return;
        }
    }
    for (int32_t e = e0 + p; e < e1; e += P) {
        const int32_t j = col[e];
        if (FINAL && j >= clo) continue;
        float hj[E];
        load_f32<E>(H, j, K, q, hj);
        const float wt = w[e];
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] = __fmaf_rn(wt, hj[i], acc[i]);
    }
#pragma unroll
    for (int off = Q; off < L; off <<= 1)
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] += __shfl_xor(acc[i], off, kWave);
    if constexpr (FINAL) {
        if (p == 0) store_f32<E>(out, r, K, q, acc);
    } else {
        if (G) {
            float gi[E];
            load_f32<E>(G, r, K, q, gi);
#pragma unroll
            for (int i = 0; i < E; ++i) acc[i] += gi[i];
        }
        float h[E], xi[E];
#pragma unroll
        for (int i = 0; i < E; ++i) h[i] = acc[i] / d;
        if (p == 0) store_f32<E>(H, r, K, q, h);
        Chunk<DT>::load(Xs, r, K, q, xi);
        for (int32_t t = 0; t < trips; ++t) {
            const int32_t e = e0 + p + t * P;
            const bool ok = e < e1;
            const int32_t j = ok ? col[e] : (int32_t)r;
            float xj[E];
            Chunk<DT>::load(j < clo ? Xs : Xp, j, K, q, xj);
            float s = 0.0f;
#pragma unroll
            for (int i = 0; i < E; ++i) s = __fmaf_rn(h[i], xj[i] - xi[i], s);
            s = qsum<Q>(s);
            if (ok && q == 0) ge[e] += s;
        }
    }
}

// The rows of degree above kLongRow (the colour's first rows: its degree
// tiers come in decreasing order) are cut into pieces of kPiece entries, so
// that a hub row is spread over many workgroups.  Two launches: the partial
// sums of w_ij h_j of every piece, then a workgroup per piece that forms
// h_i = g_i / d_i and applies it to the piece's entries.  Weights are
// positive, so d_i > 0 on these rows.
constexpr int kPiece = 256;

__global__ void k_piece_counts(const int32_t* __restrict__ rp, int64_t n, int32_t* __restrict__ cnt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t deg = rp[r + 1] - rp[r];
    cnt[r] = deg > kLongRow ? (deg + kPiece - 1) / kPiece : 0;
}

__global__ void k_gather_i32(const int32_t* __restrict__ src, const int64_t* __restrict__ idx,
                             int64_t m, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = src[idx[i]];
}

// the row of piece k among the long rows [lo, hi): last r with ppos[r] <= k
__device__ inline int64_t piece_row(const int32_t* __restrict__ ppos, int64_t lo, int64_t hi,
                                    int64_t k) {
    int64_t a = lo, b = hi - 1;
    while (a < b) {
        const int64_t m = (a + b + 1) >> 1;
        if (ppos[m] <= k) a = m; else b = m - 1;
    }
    return a;
}

// pieces [pbeg, pbeg + gridDim.x) of the long rows [lo, hi); FINAL: only
// neighbours j < clo count
template <int Q, int DT, int FINAL>
__global__ void __launch_bounds__(256) k_vjp_pieces(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const float* __restrict__ w,
    const float* __restrict__ H, int32_t K, const int32_t* __restrict__ ppos, int64_t lo,
    int64_t hi, int64_t pbeg, int64_t clo, float* __restrict__ part) {
    constexpr int P = 256 / Q;
    constexpr int NW = 256 / kWave;
    constexpr int E = Chunk<DT>::E;
    __shared__ float red[NW * Q * E];
    const int tid = threadIdx.x;
    const int p = tid / Q, q = tid % Q;
    const int64_t k = pbeg + blockIdx.x;
    const int64_t r = piece_row(ppos, lo, hi, k);
    const int32_t e0 = rp[r] + (int32_t)(k - ppos[r]) * kPiece;
    const int32_t e1 = min(e0 + kPiece, rp[r + 1]);
    float acc[E];
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = 0.0f;
    for (int32_t e = e0 + p; e < e1; e += P) {
        const int32_t j = col[e];
        if (FINAL && j >= clo) continue;
        float hj[E];
        load_f32<E>(H, j, K, q, hj);
        const float wt = w[e];
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] = __fmaf_rn(wt, hj[i], acc[i]);
    }
#pragma unroll
    for (int off = Q; off < kWave; off <<= 1)
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] += __shfl_xor(acc[i], off, kWave);
    if ((tid & (kWave - 1)) < Q)
#pragma unroll
        for (int i = 0; i < E; ++i) red[(tid / kWave) * Q * E + q * E + i] = acc[i];
    __syncthreads();
    if (tid < Q) {
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] = red[q * E + i];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww)
#pragma unroll
            for (int i = 0; i < E; ++i) acc[i] += red[ww * Q * E + q * E + i];
        store_f32<E>(part, k, K, q, acc);
    }
}

// a workgroup per piece: h_i of its row from the row's pieces in order (plus
// G_i in the last sweep) over d_i, stored into H by the row's first piece;
// then every entry of the piece, Q lanes each, adds h_i . (x_j - x_i) to its
// gradient
template <int Q, int DT>
__global__ void __launch_bounds__(256) k_vjp_long_apply(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const void* __restrict__ Xs,
    const void* __restrict__ Xp, int32_t K, int64_t clo, const int32_t* __restrict__ ppos,
    int64_t lo, int64_t hi, int64_t pbeg, const float* __restrict__ dw,
    const float* __restrict__ G, const float* __restrict__ part, float* __restrict__ H,
    float* __restrict__ ge) {
    constexpr int P = 256 / Q;
    constexpr int E = Chunk<DT>::E;
    const int tid = threadIdx.x;
    const int p = tid / Q, q = tid % Q;
    const int64_t k = pbeg + blockIdx.x;
    const int64_t r = piece_row(ppos, lo, hi, k);
    const int32_t k0 = ppos[r], k1 = ppos[r + 1];
    float h[E];
#pragma unroll
    for (int i = 0; i < E; ++i) h[i] = 0.0f;
    for (int32_t kk = k0; kk < k1; ++kk) {
        float v[E];
        load_f32<E>(part, kk, K, q, v);
#pragma unroll
        for (int i = 0; i < E; ++i) h[i] += v[i];
    }
    if (G) {
        float gi[E];
        load_f32<E>(G, r, K, q, gi);
#pragma unroll
        for (int i = 0; i < E; ++i) h[i] += gi[i];
    }
    const float d = dw[r];
#pragma unroll
    for (int i = 0; i < E; ++i) h[i] = h[i] / d;
    if (k == k0 && p == 0) store_f32<E>(H, r, K, q, h);
    float xi[E];
    Chunk<DT>::load(Xs, r, K, q, xi);
    const int32_t e0 = rp[r] + (int32_t)(k - k0) * kPiece;
    const int32_t e1 = min(e0 + kPiece, rp[r + 1]);
#pragma unroll
    for (int t = 0; t < kPiece / P; ++t) {
        const int32_t e = e0 + p + t * P;
        const bool ok = e < e1;
        const int32_t j = ok ? col[e] : (int32_t)r;
        float xj[E];
        Chunk<DT>::load(j < clo ? Xs : Xp, j, K, q, xj);
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < E; ++i) s = __fmaf_rn(h[i], xj[i] - xi[i], s);
        s = qsum<Q>(s);
        if (ok && q == 0) ge[e] += s;
    }
}

// after the last reverse step: gX0_i of the long rows [lo, hi) from their
// pieces in order, a thread per (row, chunk)
template <int Q, int DT>
__global__ void k_vjp_long_final(const int32_t* __restrict__ ppos, const float* __restrict__ part,
                                 int32_t K, int64_t lo, int64_t hi, float* __restrict__ out) {
    constexpr int E = Chunk<DT>::E;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = lo + t / Q;
    const int q = (int)(t % Q);
    if (r >= hi) return;
    float g[E];
#pragma unroll
    for (int i = 0; i < E; ++i) g[i] = 0.0f;
    for (int32_t k = ppos[r]; k < ppos[r + 1]; ++k) {
        float v[E];
        load_f32<E>(part, k, K, q, v);
#pragma unroll
        for (int i = 0; i < E; ++i) g[i] += v[i];
    }
    store_f32<E>(out, r, K, q, g);
}

// the two relabelled entries of each undirected edge: slot 0 = the entry
// whose original row is the smaller endpoint
__global__ void k_edge_slots(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ eoe, const int32_t* __restrict__ perm,
                             int64_t n, int64_t E, int G, int32_t* __restrict__ slots) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int lane = (int)(t % G);
    if (r >= n) return;
    const int32_t orow = perm[r];
    for (int32_t e = rp[r] + lane; e < rp[r + 1]; e += G) {
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

// entry slots per row (a power of two, about a quarter of the mean degree):
// each lane then has a few gathers to overlap and a wave holds more rows
// (on the 256^3 grid, mean degree 6: one slot per row 34.0 ms, 2 slots
// 33.7, 4 slots 40.4, 8 slots 47.8 per backward call)
static int pick_p_vjp(int Q, double mean_deg) {
    int P = 1;
    while (P * 4 <= mean_deg && Q * P * 2 <= kWave) P *= 2;
    return P;
}

// What the launches of one colour need, fixed for the whole call.
struct VjpPlan {
    const OrderedGraph* og;
    const float* dw;
    const int32_t* ppos;
    std::vector<int64_t> pbeg, pend;  // the pieces of each colour's long rows
    std::vector<int> P;               // lanes per row (x Q) for its short rows
    float* part;
};

template <int Q, int DT, int FINAL>
static int vjp_colour(const VjpPlan& pl, int c, const void* Xs, const void* Xp, int K,
                      const float* G, float* H, float* ge, float* out, hipStream_t st) {
    const OrderedGraph* og = pl.og;
    const gr_graph* g = &og->g;
    const int64_t clo = og->class_ptr_h[c], chi = og->class_ptr_h[c + 1];
    const int64_t mid = og->long_end_h[c];
    if (mid > clo && pl.pend[c] > pl.pbeg[c]) {
        hipLaunchKernelGGL((k_vjp_pieces<Q, DT, FINAL>), dim3((unsigned)(pl.pend[c] - pl.pbeg[c])),
                           dim3(256), 0, st, g->row_ptr, g->col, g->w, (const float*)H, K, pl.ppos,
                           clo, mid, pl.pbeg[c], clo, pl.part);
        GR_LAUNCHED("vjp pieces");
        if constexpr (FINAL) {
            hipLaunchKernelGGL((k_vjp_long_final<Q, DT>), dim3(blocks_for((mid - clo) * Q, 256)),
                               dim3(256), 0, st, pl.ppos, (const float*)pl.part, K, clo, mid, out);
            GR_LAUNCHED("vjp long final");
        } else {
            hipLaunchKernelGGL((k_vjp_long_apply<Q, DT>), dim3((unsigned)(pl.pend[c] - pl.pbeg[c])),
                               dim3(256), 0, st, g->row_ptr, g->col, Xs, Xp, K, clo, pl.ppos, clo,
                               mid, pl.pbeg[c], pl.dw, G, (const float*)pl.part, H, ge);
            GR_LAUNCHED("vjp long apply");
        }
    }
    if (chi <= mid) return GR_OK;
    const int64_t waves = ((chi - mid) * Q * pl.P[c] + kWave - 1) / kWave;
    dim3 grid(blocks_for(waves * kWave, 256));
#define GR_VR(PP)                                                                                   \
    case PP:                                                                                       \
        if constexpr (Q * PP <= kWave)                                                             \
            hipLaunchKernelGGL((k_vjp_rows<Q, PP, DT, FINAL>), grid, dim3(256), 0, st, g->row_ptr,  \
                               g->col, g->w, Xs, Xp, K, clo, mid, chi, pl.dw, G, H, ge, out);      \
        break;
    switch (pl.P[c]) {
        GR_VR(1) GR_VR(2) GR_VR(4) GR_VR(8) GR_VR(16) GR_VR(32) GR_VR(64)
        default: return set_error(GR_EINVAL, "bad lane split");
    }
#undef GR_VR
    GR_LAUNCHED("vjp rows");
    return GR_OK;
}

size_t vjp_workspace(int64_t n, int64_t nnz, int32_t K, int32_t dtype, int32_t S, int32_t store) {
    const size_t N = (size_t)n + 1, M = (size_t)nnz + 1;
    const size_t xb = N * (size_t)K * (dtype == GR_BF16 ? 2 : 4) + 256;
    const size_t fb = N * (size_t)K * 4 + 256;
    const size_t pieces = M / kPiece + M / kLongRow + 1;
    size_t b = 4 * N * 3 + 8 * M          // relabelled graph
               + 4 * M                    // relabelled edge ids
               + 4 * M                    // per-entry gradients
               + 8 * (M / 2 + 1)          // edge slots
               + (size_t)(store ? S + 1 : 3) * xb + 3 * fb  // states, G, H, gX0
               + 12 * N                   // weighted degrees, piece offsets and counts
               + pieces * (size_t)K * 4   // piece sums
               + 48 * M + 64 * N;         // sort / relabel temporaries
    return b + b / 16 + (16u << 20);
}

template <int Q, int DT>
static int vjp_impl(const VjpPlan& pl, int K, int S, int store, void* states, size_t xbytes,
                    const float* Gp, float* H, float* ge, float* gx, Arena& ws, hipStream_t st) {
    const OrderedGraph* og = pl.og;
    const int C = og->n_colours;
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
        const float* G = s == S ? Gp : nullptr;
        for (int c = C - 1; c >= 0; --c)
            GR_TRY((vjp_colour<Q, DT, 0>(pl, c, Xs, Xp, K, G, H, ge, nullptr, st)));
    }
    if (S >= 1)
        for (int c = 0; c < C; ++c)
            GR_TRY((vjp_colour<Q, DT, 1>(pl, c, nullptr, nullptr, K, Gp, H, nullptr, gx, st)));
    return GR_OK;
}

int smooth_vjp(const gr_graph* g, const int32_t* eoe, int64_t E, const int32_t* colours, int32_t C,
               int32_t K, int32_t S, int32_t dtype, const void* X0, const float* Gc, float* gw,
               float* gX0, int32_t store, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    GR_TRY(validate_colouring(g, colours, C, ws, st));
    OrderedGraph og;
    GR_TRY(order_by_colour(g, colours, C, &og, ws, st));
    // edge ids of the relabelled entries, weighted degrees, long-row pieces
    const int G = lanes_per_row(n, nnz);
    int32_t* eoe_r = ws.take<int32_t>(nnz + 1);
    float* dw = ws.take<float>(n + 1);
    int32_t* ppos = ws.take<int32_t>(n + 1);
    int32_t* pbounds = ws.take<int32_t>(2 * (size_t)C + 1);
    int64_t* pidx = ws.take<int64_t>(2 * (size_t)C + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp)");
    if (nnz > 0) {
        hipLaunchKernelGGL(k_perm_payload, dim3(blocks_for(n * G, 256)), dim3(256), 0, st,
                           g->row_ptr, (const uint32_t*)og.perm, og.g.row_ptr, n, G, eoe, eoe_r);
        GR_LAUNCHED("perm payload");
    }
    hipLaunchKernelGGL(k_row_weight, dim3(blocks_for(n * G, 256)), dim3(256), 0, st, og.g.row_ptr,
                       og.g.w, n, G, dw);
    GR_LAUNCHED("row weights");
    {
        size_t mark = ws.used;
        int32_t* cnt = ws.take<int32_t>(n);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp pieces)");
        hipLaunchKernelGGL(k_piece_counts, dim3(blocks_for(n, 256)), dim3(256), 0, st, og.g.row_ptr,
                           n, cnt);
        GR_LAUNCHED("piece counts");
        GR_TRY(scan_exclusive_i32(cnt, ppos, n, ppos + n, ws, st));
        ws.used = mark;
    }
    // piece ranges of every colour's long rows [class start, long end), and the total
    std::vector<int64_t> hidx(2 * (size_t)C + 1);
    for (int c = 0; c < C; ++c) {
        hidx[2 * c] = og.class_ptr_h[c];
        hidx[2 * c + 1] = og.long_end_h[c];
    }
    hidx[2 * C] = n;
    std::vector<int32_t> hpb(2 * (size_t)C + 1);
    GR_HIP(hipMemcpyAsync(pidx, hidx.data(), sizeof(int64_t) * hidx.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gather_i32, dim3(blocks_for(2 * C + 1, 256)), dim3(256), 0, st,
                       (const int32_t*)ppos, (const int64_t*)pidx, (int64_t)(2 * C + 1), pbounds);
    GR_LAUNCHED("piece bounds");
    GR_HIP(hipMemcpyAsync(hpb.data(), pbounds, sizeof(int32_t) * hpb.size(), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    const int64_t n_pieces = hpb[2 * C];
    VjpPlan pl;
    pl.og = &og;
    pl.dw = dw;
    pl.ppos = ppos;
    pl.pbeg.resize(C);
    pl.pend.resize(C);
    pl.P.resize(C);
    const int Q = K * (dtype == GR_BF16 ? 2 : 4) / 16;
    for (int c = 0; c < C; ++c) {
        pl.pbeg[c] = hpb[2 * c];
        pl.pend[c] = hpb[2 * c + 1];
        const int64_t rows = og.class_ptr_h[c + 1] - og.long_end_h[c];
        const int64_t nz = og.class_nnz_h[c] - og.long_nnz_h[c];
        pl.P[c] = pick_p_vjp(Q, rows > 0 ? (double)nz / (double)rows : 1.0);
    }
    pl.part = ws.take<float>((size_t)(n_pieces + 1) * K);
    // states, cotangent, H, gX0 (relabelled), per-entry gradients
    const size_t xbytes = (size_t)n * K * (dtype == GR_BF16 ? 2 : 4);
    const size_t xstride = (xbytes + 255) & ~size_t(255);
    void* states = ws.take<char>((size_t)(store ? S + 1 : 3) * xstride);
    float* Gp = ws.take<float>((size_t)n * K + 4);
    float* H = ws.take<float>((size_t)n * K + 4);
    float* gx = ws.take<float>((size_t)n * K + 4);
    float* ge = ws.take<float>(nnz + 1);
    int32_t* slots = ws.take<int32_t>(2 * (E + 1));
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (vjp states)");
    GR_TRY(permute_rows(X0, states, og.perm, n, (size_t)K * (dtype == GR_BF16 ? 2 : 4), 0, st));
    GR_TRY(permute_rows(Gc, Gp, og.perm, n, (size_t)K * 4, 0, st));
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(n * K, 256)), dim3(256), 0, st, H, (int64_t)n * K);
    GR_LAUNCHED("zero");
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(nnz + 1, 256)), dim3(256), 0, st, ge, nnz + 1);
    GR_LAUNCHED("zero");
#define GR_VJ(QQ, DD) \
    case QQ: GR_TRY((vjp_impl<QQ, DD>(pl, K, S, store, states, xstride, Gp, H, ge, gx, ws, st))); break;
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
    // no sweep: X_S = X0 and the cotangent passes through
    GR_TRY(permute_rows(S >= 1 ? gx : Gp, gX0, og.perm, n, (size_t)K * 4, 1, st));
    if (E > 0) {
        GR_TRY(fill_i32(slots, 0, 2 * E, st));  // unmatched slots read entry 0, never garbage
        GR_TRY(reset_bad_edge_flag(st));
        hipLaunchKernelGGL(k_edge_slots, dim3(blocks_for(n * G, 256)), dim3(256), 0, st,
                           og.g.row_ptr, og.g.col, (const int32_t*)eoe_r, og.perm, n, E, G, slots);
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
