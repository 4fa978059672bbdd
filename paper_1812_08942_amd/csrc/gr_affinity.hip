// Spectral affinity of every stored edge (Eq. (eqn:agg) of Sec. 3.2.1) on
// the smoothed test vectors, and each row's closest neighbour by algebraic
// distance (the aggregation's candidate).
//
// Layout as in the smoothing: node-major rows of K values in 16-byte chunks;
// Q lanes hold one row, the P slots of a row-group walk the neighbours.
#include "gr_internal.hpp"
#include "gr_device.hpp"

namespace gr {

constexpr int kThreads = 256;
#ifndef GR_AFF_BLOCK
#define GR_AFF_BLOCK 512
#endif
// threads of an affinity block (measured: 512 beats 1024 by 0.3 ms per
// reduction on the power-law graph)
constexpr int kBig = GR_AFF_BLOCK;

// ---------------------------------------------------------------- affinity
// (d, id) ordering of candidates: smaller algebraic distance, then smaller id.
__device__ inline bool closer(float d1, int32_t id1, float d2, int32_t id2) {
    return d1 < d2 || (d1 == d2 && id1 < id2);
}

// Per row-group: a = (x_v . x_j)^2 / (|x_v|^2 |x_j|^2) and the algebraic
// distance d = 1 - a.  d is formed without cancellation as
// |u - w|^2 |u + w|^2 / 4 on the normalised rows u = x_v/|x_v|, w = x_j/|x_j|
// (equal to 1 - cos^2 in exact arithmetic), so that it keeps its relative
// accuracy where a itself rounds to 1 in float32.  Both quantities are
// computed by the same code for (v, j) and (j, v), hence bit-symmetric.
// Distance, affinity and the row-group's candidate for one entry (v, j):
// chunk q of the normalised rows, reduced over the Q lanes of the entry with
// a fixed tree, so (v, j) and (j, v) give identical bits.
template <int Q, int DT>
__device__ inline void entry_ad(const void* __restrict__ X, int32_t K, int q, const float* xv,
                                const float* uv, float nv, int32_t j, float* av, float* dv) {
    constexpr int E = Chunk<DT>::E;
    float xj[E];
    Chunk<DT>::load(X, j, K, q, xj);
    float c = qsum<Q>(chunk_dot<E>(xv, xj));
    float nj = qsum<Q>(chunk_dot<E>(xj, xj));
    const float rj = nj > 0.0f ? 1.0f / sqrtf(nj) : 0.0f;
    float dm = 0.0f, dp = 0.0f;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        float uj = xj[i] * rj;
        float m = uv[i] - uj, s2 = uv[i] + uj;
        dm = __fmaf_rn(m, m, dm);
        dp = __fmaf_rn(s2, s2, dp);
    }
    dm = qsum<Q>(dm);
    dp = qsum<Q>(dp);
    float den = nv * nj;
    *av = den == 0.0f ? 0.0f : fminf(1.0f, (c * c) / den);
    *dv = den == 0.0f ? 1.0f : fminf(1.0f, dm * dp * 0.25f);
}

template <int Q, int DT>
__device__ inline void row_prep(const void* __restrict__ X, int32_t K, int q, int64_t r, float* xv,
                                float* uv, float* nv_out) {
    constexpr int E = Chunk<DT>::E;
    Chunk<DT>::load(X, r, K, q, xv);
    const float nv = qsum<Q>(chunk_dot<E>(xv, xv));
    // the row is normalised by one correctly rounded reciprocal square root
    // (the same operations for every row, so (v, j) and (j, v) agree)
    const float rv = nv > 0.0f ? 1.0f / sqrtf(nv) : 0.0f;
#pragma unroll
    for (int i = 0; i < E; ++i) uv[i] = xv[i] * rv;
    *nv_out = nv;
}

// Rows with degree <= kLongRow: L = Q*P lanes per row.
template <int Q, int P, int DT>
__device__ inline void aff_normal(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  const void* __restrict__ X, int32_t K, int64_t n,
                                  const int32_t* __restrict__ ids, float* __restrict__ a,
                                  float* __restrict__ dist, int32_t* __restrict__ best,
                                  float* __restrict__ dbest, int64_t rblock) {
    constexpr int L = Q * P;
    constexpr int RPW = kWave / L;
    constexpr int E = Chunk<DT>::E;
    const int lane = threadIdx.x & (kWave - 1);
    const int l = lane % L;
    const int p = l / Q, q = l % Q;
    const int64_t wave = (rblock * kBig + threadIdx.x) / kWave;
    const int64_t r = wave * RPW + lane / L;
    if (r >= n) return;
    const int32_t e0 = rp[r], e1 = rp[r + 1];
    if (e1 - e0 > kLongRow) return;  // handled by a whole workgroup
    float xv[E], uv[E], nv;
    row_prep<Q, DT>(X, K, q, r, xv, uv, &nv);
    float bd = 2.0f;
    int32_t bj = -1, bid = 0x7fffffff;
    // every lane of the row-group runs the same trip count so the q-sums
    // (shuffles) stay converged; lanes past the end use a dummy column
    const int32_t trips = (e1 - e0 + P - 1) / P;
    for (int32_t t = 0; t < trips; ++t) {
        int32_t e = e0 + p + t * P;
        bool ok = e < e1;
        int32_t j = ok ? col[e] : (int32_t)r;
        float av, dv;
        entry_ad<Q, DT>(X, K, q, xv, uv, nv, j, &av, &dv);
        if (ok) {
            if (q == 0) {
                if (a) a[e] = av;
                if (dist) dist[e] = dv;
            }
            int32_t jid = ids ? ids[j] : j;
            if (closer(dv, jid, bd, bid)) { bd = dv; bj = j; bid = jid; }
        }
    }
#pragma unroll
    for (int off = Q; off < L; off <<= 1) {
        float od = __shfl_xor(bd, off, kWave);
        int32_t oj = __shfl_xor(bj, off, kWave);
        int32_t oid = __shfl_xor(bid, off, kWave);
        if (oj >= 0 && (bj < 0 || closer(od, oid, bd, bid))) { bd = od; bj = oj; bid = oid; }
    }
    if (l == 0) {
        best[r] = bj;
        if (dbest) dbest[r] = bj >= 0 ? bd : 1.0f;
    }
}

// A long row: the whole workgroup, P = kBig/Q entries at a time.
template <int Q, int DT>
__device__ inline void aff_long(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const void* __restrict__ X, int32_t K, int64_t r,
                                const int32_t* __restrict__ ids, float* __restrict__ a,
                                float* __restrict__ dist, int32_t* __restrict__ best,
                                float* __restrict__ dbest) {
    constexpr int E = Chunk<DT>::E;
    constexpr int P = kBig / Q;
    constexpr int NW = kBig / kWave;
    __shared__ float sbd[NW];
    __shared__ int32_t sbj[NW], sbid[NW];
    const int t = threadIdx.x;
    const int p = t / Q, q = t % Q;
    float xv[E], uv[E], nv;
    row_prep<Q, DT>(X, K, q, r, xv, uv, &nv);
    const int32_t e0 = rp[r], e1 = rp[r + 1];
    float bd = 2.0f;
    int32_t bj = -1, bid = 0x7fffffff;
    const int32_t trips = (e1 - e0 + P - 1) / P;
    for (int32_t it = 0; it < trips; ++it) {
        int32_t e = e0 + p + it * P;
        bool ok = e < e1;
        int32_t j = ok ? col[e] : (int32_t)r;
        float av, dv;
        entry_ad<Q, DT>(X, K, q, xv, uv, nv, j, &av, &dv);
        if (ok) {
            if (q == 0) {
                if (a) a[e] = av;
                if (dist) dist[e] = dv;
            }
            int32_t jid = ids ? ids[j] : j;
            if (closer(dv, jid, bd, bid)) { bd = dv; bj = j; bid = jid; }
        }
    }
#pragma unroll
    for (int off = Q; off < kWave; off <<= 1) {
        float od = __shfl_xor(bd, off, kWave);
        int32_t oj = __shfl_xor(bj, off, kWave);
        int32_t oid = __shfl_xor(bid, off, kWave);
        if (oj >= 0 && (bj < 0 || closer(od, oid, bd, bid))) { bd = od; bj = oj; bid = oid; }
    }
    const int wid = t / kWave, lane = t & (kWave - 1);
    if (lane == 0) {
        sbd[wid] = bd;
        sbj[wid] = bj;
        sbid[wid] = bid;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < NW; ++w)
            if (sbj[w] >= 0 && (bj < 0 || closer(sbd[w], sbid[w], bd, bid))) {
                bd = sbd[w];
                bj = sbj[w];
                bid = sbid[w];
            }
        best[r] = bj;
        if (dbest) dbest[r] = bj >= 0 ? bd : 1.0f;
    }
}

template <int Q, int P, int DT>
__global__ void __launch_bounds__(kBig) k_affinity(const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const void* __restrict__ X, int32_t K, int64_t n,
                                                   const int32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ long_rows,
                                                   int64_t n_long, float* __restrict__ a,
                                                   float* __restrict__ dist,
                                                   int32_t* __restrict__ best,
                                                   float* __restrict__ dbest) {
    const int64_t b = blockIdx.x;
    if (b < n_long) aff_long<Q, DT>(rp, col, X, K, long_rows[b], ids, a, dist, best, dbest);
    else aff_normal<Q, P, DT>(rp, col, X, K, n, ids, a, dist, best, dbest, b - n_long);
}

template <int Q, int DT>
static int launch_aff(const gr_graph* g, int K, const void* X, const int32_t* ids,
                      const int32_t* long_rows, int64_t n_long, float* a, float* dist,
                      int32_t* best, float* dbest, hipStream_t st) {
    // entry slots per row: a power of two, about a sixteenth of the mean
    // degree, so that a wave holds many rows (more independent gathers in
    // flight than more slots of one row give; 256^3 grid, mean degree 6:
    // 3.9 ms per reduction with one slot, 4.5 with 2, 5.7 with 4)
    double md = g->n > 0 ? (double)g->nnz / (double)g->n : 0.0;
    int P = 1;
    while (P * 16 <= md && Q * P * 2 <= kWave) P *= 2;
    const int64_t waves = (g->n * Q * P + kWave - 1) / kWave;
    const int64_t grid = n_long + (waves * kWave + kBig - 1) / kBig;
#define GR_AF(PP)                                                                                  \
    case PP:                                                                                      \
        if constexpr (Q * PP <= kWave)                                                            \
            hipLaunchKernelGGL((k_affinity<Q, PP, DT>), dim3((unsigned)grid), dim3(kBig), 0, st,    \
                               g->row_ptr, g->col, X, K, g->n, ids, long_rows, n_long, a, dist,    \
                               best, dbest);                                                      \
        break;
    switch (P) {
        GR_AF(1) GR_AF(2) GR_AF(4) GR_AF(8) GR_AF(16) GR_AF(32) GR_AF(64)
        default: return set_error(GR_EINVAL, "bad lane split");
    }
#undef GR_AF
    GR_LAUNCHED("affinity");
    return GR_OK;
}

__global__ void k_long_flags(const int32_t* __restrict__ rp, int64_t n, int32_t* __restrict__ flag) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = (rp[v + 1] - rp[v]) > kLongRow ? 1 : 0;
}

__global__ void k_long_scatter(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                               int64_t n, int32_t* __restrict__ out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && flag[v]) out[pos[v]] = (int32_t)v;
}

int find_long_rows(const gr_graph* g, int32_t** rows, int64_t* n_long, Arena& ws, hipStream_t st) {
    const int64_t n = g->n;
    *rows = nullptr;
    *n_long = 0;
    if (n == 0) return GR_OK;
    int32_t* flag = ws.take<int32_t>(n);
    int32_t* pos = ws.take<int32_t>(n + 1);
    int32_t* out = ws.take<int32_t>(n);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (long rows)");
    hipLaunchKernelGGL(k_long_flags, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st,
                       g->row_ptr, n, flag);
    GR_LAUNCHED("long flags");
    GR_TRY(scan_exclusive_i32(flag, pos, n, pos + n, ws, st));
    hipLaunchKernelGGL(k_long_scatter, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, flag,
                       pos, n, out);
    GR_LAUNCHED("long scatter");
    int32_t cnt = 0;
    GR_HIP(hipMemcpyAsync(&cnt, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    *rows = out;
    *n_long = cnt;
    return GR_OK;
}

int affinity(const gr_graph* g, int32_t K, int32_t dtype, const void* X, const int32_t* ids,
             const int32_t* long_rows, int64_t n_long, float* a, float* dist, int32_t* best,
             float* dbest, hipStream_t st) {
    if (g->n == 0) return GR_OK;
    int Q = K * (dtype == GR_BF16 ? 2 : 4) / 16;
#define GR_AFQ(QQ, DD) \
    case QQ: return launch_aff<QQ, DD>(g, K, X, ids, long_rows, n_long, a, dist, best, dbest, st);
    if (dtype == GR_BF16) {
        switch (Q) { GR_AFQ(1, GR_BF16) GR_AFQ(2, GR_BF16) GR_AFQ(4, GR_BF16) GR_AFQ(8, GR_BF16) }
    } else {
        switch (Q) {
            GR_AFQ(1, GR_F32) GR_AFQ(2, GR_F32) GR_AFQ(4, GR_F32) GR_AFQ(8, GR_F32)
            GR_AFQ(16, GR_F32)
        }
    }
#undef GR_AFQ
    return set_error(GR_EUNSUP, "unsupported K=%d for this dtype", K);
}

}  // namespace gr
