// Spectral affinity of every stored edge (Eq. (eqn:agg) of Sec. 3.2.1) on
// the smoothed test vectors, and each row's closest neighbour by algebraic
// distance (the aggregation's candidate).
//
// Layout as in the smoothing: node-major rows of K values in 16-byte chunks;
// Q lanes hold one row, the P slots of a row-group walk the neighbours.
#include <cstdlib>

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
// (d, id) ordering of candidates: smaller algebraic distance, then smaller
// original id.
__device__ inline bool closer(float d1, int32_t id1, float d2, int32_t id2) {
    return d1 < d2 || (d1 == d2 && id1 < id2);
}
__device__ inline int32_t idof(const int32_t* ids, int32_t j) { return ids ? ids[j] : j; }
// Candidate j (row index) beats the current best bj when its distance is
// smaller, or equal with a smaller id; the ids are read only for such exact
// ties.  (The search starts from bd = 2 above every distance, so a tie
// always has a best bj >= 0.)
__device__ inline bool beats(float d, int32_t j, float bd, int32_t bj, const int32_t* ids) {
    return d < bd || (d == bd && idof(ids, j) < idof(ids, bj));
}

// Per row-group: a = (x_v . x_j)^2 / (|x_v|^2 |x_j|^2) and the algebraic
// distance d = 1 - a.  On the normalised rows u = x_v/|x_v|, w = x_j/|x_j|,
// 1 - cos^2 = |u - w|^2 |u + w|^2 / 4, and the two factors add up to 4
// (|u|^2 + |w|^2 + ... = 4 for unit rows), so d = m (4 - m) / 4 with m the
// smaller factor: |u - w|^2 when x_v . x_j >= 0, else |u + w|^2.  m is the
// factor that would cancel if formed as 4 minus the other one, so d keeps its
// relative accuracy where a itself rounds to 1 in float32 (d ~ 0 at
// cos ~ +1 and at cos ~ -1); the other factor, in [2, 4], takes it from 4.
// A row is normalised by the hardware reciprocal square root of its squared
// norm (within an ulp or two; the unit rows need not be exact, only the
// same for every use of the row).  Everything is computed by the same
// operations for (v, j) and (j, v): the dot products commute, u - w and
// w - u differ in sign only, so both quantities are bit-symmetric.

// squared norm and reciprocal norm of a row chunk (reduced over the Q lanes)
template <int Q, int E>
__device__ inline float2 row_norm(const float* x) {
    const float nv = qsum<Q>(chunk_dot<E>(x, x));
    return make_float2(nv, nv > 0.0f ? rsqrtf(nv) : 0.0f);
}

// d (and a if wanted) of one entry from chunk q of both rows
template <int Q, int E>
__device__ inline float entry_d(const float* xv, const float* uv, float2 nrv, const float* xj,
                                float* av) {
    const float c = qsum<Q>(chunk_dot<E>(xv, xj));
    const float2 nrj = row_norm<Q, E>(xj);
    const float s = c >= 0.0f ? -1.0f : 1.0f;
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const float t = __fmaf_rn(s, xj[i] * nrj.y, uv[i]);  // u -+ w, rounded once
        m = __fmaf_rn(t, t, m);
    }
    m = qsum<Q>(m);
    if (av) {
        const float den = nrv.x * nrj.x;
        *av = den == 0.0f ? 0.0f : fminf(1.0f, (c * c) / den);
    }
    return (nrv.y == 0.0f || nrj.y == 0.0f) ? 1.0f : fminf(1.0f, m * (4.0f - m) * 0.25f);
}

// entries of a row taken per round by each lane: their columns, then their
// rows and ids, are all loaded before any is used, so that the gathers are
// in flight together
constexpr int kAU = 4;

// The row-group's part of one row: lanes (p, q) take entries p, p + P, ...
// (kAU at a time), chunk q.  Every lane of the row-group runs the same trip
// count so that the q-sums (shuffles) stay converged; lanes past the end
// use the row itself as a dummy neighbour.  Returns the lane's best (d, id).
template <int Q, int DT>
__device__ inline void row_entries(const int32_t* __restrict__ col, const void* __restrict__ X,
                                   int32_t K, const int32_t* __restrict__ ids, int64_t r,
                                   int32_t e0,
                                   int32_t e1, int p, int q, int P, float* __restrict__ a,
                                   float* __restrict__ dist, float& bd, int32_t& bj,
                                   int32_t& bid) {
    constexpr int E = Chunk<DT>::E;
    // with bfloat16 storage (8-bit mantissas) equal smoothed rows, and so
    // exact ties of d, are common: the ids then travel with the rows' loads
    // (a tie otherwise stops the loop for two dependent loads); with float32
    // they are read only on a tie, and the best one's at the end
    constexpr bool kEagerIds = DT == GR_BF16;
    float xv[E], uv[E];
    Chunk<DT>::load(X, r, K, q, xv);
    const float2 nrv = row_norm<Q, E>(xv);
#pragma unroll
    for (int i = 0; i < E; ++i) uv[i] = xv[i] * nrv.y;
    const int32_t trips = (e1 - e0 + P * kAU - 1) / (P * kAU);
    for (int32_t t = 0; t < trips; ++t) {
        int32_t e[kAU], j[kAU], jid[kAU];
#pragma unroll
        for (int u = 0; u < kAU; ++u) {
            e[u] = e0 + p + (t * kAU + u) * P;
            j[u] = e[u] < e1 ? col[e[u]] : (int32_t)r;
        }
        float xj[kAU][E];
#pragma unroll
        for (int u = 0; u < kAU; ++u) {
            Chunk<DT>::load(X, j[u], K, q, xj[u]);
            if constexpr (kEagerIds) jid[u] = idof(ids, j[u]);
        }
#pragma unroll
        for (int u = 0; u < kAU; ++u) {
            float av;
            const float dv = entry_d<Q, E>(xv, uv, nrv, xj[u], a ? &av : nullptr);
            if (e[u] < e1) {
                if (q == 0) {
                    if (a) a[e[u]] = av;
                    if (dist) dist[e[u]] = dv;
                }
                if constexpr (kEagerIds) {
                    if (closer(dv, jid[u], bd, bid)) {
                        bd = dv;
                        bj = j[u];
                        bid = jid[u];
                    }
                } else if (beats(dv, j[u], bd, bj, ids)) {
                    bd = dv;
                    bj = j[u];
                }
            }
        }
    }
    if constexpr (!kEagerIds) bid = bj >= 0 ? idof(ids, bj) : 0x7fffffff;
}

// Rows with degree <= kLongRow: L = Q*P lanes per row.
template <int Q, int P, int DT>
__device__ inline void aff_normal(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  const void* __restrict__ X, int32_t K, int64_t n,
                                  const int32_t* __restrict__ ids,
                                  float* __restrict__ a, float* __restrict__ dist,
                                  int32_t* __restrict__ best, float* __restrict__ dbest,
                                  int64_t rblock) {
    constexpr int L = Q * P;
    constexpr int RPW = kWave / L;
    const int lane = threadIdx.x & (kWave - 1);
    const int l = lane % L;
    const int p = l / Q, q = l % Q;
    const int64_t wave = (rblock * kBig + threadIdx.x) / kWave;
    const int64_t r = wave * RPW + lane / L;
    if (r >= n) return;
    const int32_t e0 = rp[r], e1 = rp[r + 1];
    if (e1 - e0 > kLongRow) return;  // handled by a whole workgroup
    float bd = 2.0f;
    int32_t bj = -1, bid = 0x7fffffff;
    row_entries<Q, DT>(col, X, K, ids, r, e0, e1, p, q, P, a, dist, bd, bj, bid);
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
                                const int32_t* __restrict__ ids,
                                float* __restrict__ a, float* __restrict__ dist,
                                int32_t* __restrict__ best, float* __restrict__ dbest) {
    constexpr int P = kBig / Q;
    constexpr int NW = kBig / kWave;
    __shared__ float sbd[NW];
    __shared__ int32_t sbj[NW], sbid[NW];
    const int t = threadIdx.x;
    const int p = t / Q, q = t % Q;
    float bd = 2.0f;
    int32_t bj = -1, bid = 0x7fffffff;
    row_entries<Q, DT>(col, X, K, ids, r, rp[r], rp[r + 1], p, q, P, a, dist, bd, bj, bid);
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

// Workgroups are handed to the 8 XCDs in turn (block b to XCD b mod 8),
// and each XCD has its own L2.  With chunk C > 0 the blocks are renumbered
// so that each XCD runs C consecutive row blocks of every 8C: neighbouring
// rows, whose gathered neighbour rows overlap, then share one L2.  The tail
// beyond the last whole group of 8C blocks keeps its order.  C = 0 keeps
// the launch order; C < 0 takes C = T / 8, one contiguous range per XCD.
// A bijection of [0, T) for any T; an offset o added to b and the result
// keeps the property (block o + b runs on XCD (o + b) mod 8).
__device__ inline int64_t xcd_block(int64_t b, int64_t T, int32_t C) {
    if (C < 0) C = (int32_t)(T >> 3);
    if (C <= 0) return b;
    const int64_t span = 8 * (int64_t)C;
    const int64_t s = b / span;
    if ((s + 1) * span > T) return b;
    const int64_t w = b - s * span;
    return s * span + (w & 7) * C + (w >> 3);
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
                                                   float* __restrict__ dbest, int32_t chunk) {
    // the workgroup-wide rows keep the launch order (spread over the XCDs)
    int64_t b = blockIdx.x;
    if (b >= n_long) b = n_long + xcd_block(b - n_long, (int64_t)gridDim.x - n_long, chunk);
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
    // Where the vectors exceed half the Infinity Cache, each XCD takes one
    // contiguous range of the row blocks (256^3 grid, bfloat16: level-0
    // affinity 1.80 -> 1.53 ms).  Vectors that stay on chip gain nothing
    // (the power-law graph's affinity, 27 MB of vectors, went 0.65 -> 0.74
    // ms with it).  GR_AFF_XCD_CHUNK sets the chunk instead (0 = launch
    // order, -1 = contiguous ranges, C > 0 = C blocks at a time).
    const double vbytes = (double)g->n * K * (DT == GR_BF16 ? 2 : 4);
    int32_t chunk = vbytes > 128.0 * 1024 * 1024 ? -1 : 0;
    if (const char* e = getenv("GR_AFF_XCD_CHUNK")) chunk = atoi(e);
#define GR_AF(PP)                                                                                  \
    case PP:                                                                                      \
        if constexpr (Q * PP <= kWave)                                                            \
            hipLaunchKernelGGL((k_affinity<Q, PP, DT>), dim3((unsigned)grid), dim3(kBig), 0, st,    \
                               g->row_ptr, g->col, X, K, g->n, ids, long_rows, n_long, a, dist,    \
                               best, dbest, chunk);                                               \
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
#define GR_AFQ(QQ, DD)                                                                            \
    case QQ:                                                                                      \
        return launch_aff<QQ, DD>(g, K, X, ids, long_rows, n_long, a, dist, best, dbest, st);
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
