// Strongest-affinity aggregation and the Galerkin collapse P^T L P
// (Sec. 3.2.2).  All integer work; the only floating-point arithmetic is the
// coarse weight sum, done once per unordered aggregate pair in a fixed
// (sorted, tiled) order.
#include "gr_internal.hpp"

namespace gr {

constexpr int kT = 256;

__device__ inline int32_t idof(const int32_t* ids, int32_t v) { return ids ? ids[v] : v; }

// own[v] = 1 when v owns the forest edge {v, best(v)}: always, except for the
// member of a mutual pair with the larger id.
__global__ void k_forest_own(const int32_t* __restrict__ best, const int32_t* __restrict__ ids,
                             int64_t n, int32_t* __restrict__ own) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    int32_t b = best[v];
    int32_t o = 0;
    if (b >= 0) o = !(best[b] == (int32_t)v && idof(ids, b) < idof(ids, (int32_t)v));
    own[v] = o;
}

// Truncation keys for the owned forest edges, compacted to slot pos[v]:
// k1 = bits(d) << idbits | min id   (smaller distance first, then smaller
//       min id; d in [0, 1] so its bits lie in [0, 0x3F800000] and ascend),
// k2 = max id (the last tie-break, sorted first in LSD order).
__global__ void k_forest_keys(const int32_t* __restrict__ best, const float* __restrict__ dbest,
                              const int32_t* __restrict__ ids, const int32_t* __restrict__ own,
                              const int32_t* __restrict__ pos, int64_t n, int idbits,
                              uint64_t* __restrict__ k1, uint64_t* __restrict__ k2,
                              uint32_t* __restrict__ slot, int32_t* __restrict__ owner) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n || !own[v]) return;
    int32_t b = best[v];
    int32_t iv = idof(ids, (int32_t)v), ib = idof(ids, b);
    uint64_t lo = (uint64_t)min(iv, ib), hi = (uint64_t)max(iv, ib);
    uint64_t d = (uint64_t)min(__float_as_uint(dbest[v]), 0x3F800000u);
    int32_t s = pos[v];
    k1[s] = (d << idbits) | lo;
    k2[s] = hi;
    slot[s] = (uint32_t)s;
    owner[s] = (int32_t)v;
}

__global__ void k_gather_keys(const uint64_t* __restrict__ src, const uint32_t* __restrict__ idx,
                              int64_t m, uint64_t* __restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) dst[i] = src[idx[i]];
}

__global__ void k_accept_first(const uint32_t* __restrict__ order, const int32_t* __restrict__ owner,
                               int64_t m, int32_t* __restrict__ acc) {
    int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) acc[owner[order[i]]] = 1;
}

__global__ void k_parent(const int32_t* __restrict__ best, const int32_t* __restrict__ ids,
                         const int32_t* __restrict__ acc, int64_t n, int32_t* __restrict__ par) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    int32_t b = best[v];
    int32_t p = (int32_t)v;
    if (b >= 0) {
        if (best[b] == (int32_t)v) {  // mutual pair: the smaller id is the root
            if (idof(ids, (int32_t)v) > idof(ids, b) && acc[b]) p = b;
        } else if (acc[v]) {
            p = b;
        }
    }
    par[v] = p;
}

// one pointer-jumping round; `changed` (when given) is raised by one lane
// per wave that moved a pointer (a benign same-value race)
__global__ void k_jump(const int32_t* __restrict__ pa, int64_t n, int32_t* __restrict__ pb,
                       int32_t* __restrict__ changed) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    bool ch = false;
    if (v < n) {
        const int32_t p = pa[v];
        const int32_t q = pa[p];
        pb[v] = q;
        ch = q != p;
    }
    if (changed && __ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) *changed = 1;
}

__global__ void k_min_member(const int32_t* __restrict__ root, const int32_t* __restrict__ ids,
                             int64_t n, int32_t* __restrict__ minid) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    // read first: once a small id has arrived, the larger ones of a big
    // aggregate skip the atomic (same-address atomics serialise); a stale
    // read only costs an atomic that changes nothing
    const int32_t r = root[v], id = idof(ids, (int32_t)v);
    if (id < minid[r]) atomicMin(&minid[r], id);
}

__global__ void k_leader_flags(const int32_t* __restrict__ root, const int32_t* __restrict__ ids,
                               const int32_t* __restrict__ minid, int64_t n,
                               int32_t* __restrict__ flag_by_id) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    int32_t id = idof(ids, (int32_t)v);
    flag_by_id[id] = (minid[root[v]] == id) ? 1 : 0;
}

__global__ void k_assign(const int32_t* __restrict__ root, const int32_t* __restrict__ minid,
                         const int32_t* __restrict__ rank_by_id, int64_t n,
                         int32_t* __restrict__ agg) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    agg[v] = rank_by_id[minid[root[v]]];
}

int aggregate(const gr_graph* g, const int32_t* best, const float* dbest, const int32_t* ids,
              int64_t target, int32_t* agg, int64_t* n_coarse, int64_t* n_forest, Arena& ws,
              hipStream_t st) {
    const int64_t n = g->n;
    *n_coarse = 0;
    if (n_forest) *n_forest = 0;
    if (n == 0) return GR_OK;
    if (target < 1) target = 1;
    size_t mark = ws.used;
    int32_t* own = ws.take<int32_t>(n);
    int32_t* pos = ws.take<int32_t>(n + 1);
    int32_t* acc = ws.take<int32_t>(n);
    int32_t* pa = ws.take<int32_t>(n);
    int32_t* pb = ws.take<int32_t>(n);
    int32_t* small = ws.take<int32_t>(4);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (aggregate)");
    const unsigned gb = blocks_for(n, kT);
    hipLaunchKernelGGL(k_forest_own, dim3(gb), dim3(kT), 0, st, best, ids, n, own);
    GR_LAUNCHED("forest own");
    GR_TRY(scan_exclusive_i32(own, pos, n, pos + n, ws, st));
    int32_t nf = 0;
    GR_HIP(hipMemcpyAsync(&nf, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    if (n_forest) *n_forest = nf;
    if (n - nf >= target) {
        GR_HIP(hipMemcpyAsync(acc, own, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    } else {
        // accept only the first m = n - target forest edges in the total order
        int64_t m = n - target;
        GR_HIP(hipMemsetAsync(acc, 0, sizeof(int32_t) * n, st));
        if (m > 0) {
            size_t mark2 = ws.used;
            uint64_t* k1 = ws.take<uint64_t>(nf);
            uint64_t* k2 = ws.take<uint64_t>(nf);
            uint64_t* ka = ws.take<uint64_t>(nf);
            uint64_t* kb = ws.take<uint64_t>(nf);
            uint32_t* sa = ws.take<uint32_t>(nf);
            uint32_t* sb = ws.take<uint32_t>(nf);
            int32_t* owner = ws.take<int32_t>(nf);
            if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (truncation)");
            const int idb = bits_for(n);
            hipLaunchKernelGGL(k_forest_keys, dim3(gb), dim3(kT), 0, st, best, dbest, ids, own, pos,
                               n, idb, k1, k2, sa, owner);
            GR_LAUNCHED("forest keys");
            // LSD order: stable by max id first, then stable by k1
            GR_TRY(radix_sort_pairs(k2, sa, ka, sb, nf, idb, ws, st));
            const unsigned fb = blocks_for(nf, kT);
            hipLaunchKernelGGL(k_gather_keys, dim3(fb), dim3(kT), 0, st, k1, sb, (int64_t)nf, kb);
            GR_LAUNCHED("gather keys");
            GR_TRY(radix_sort_pairs(kb, sb, ka, sa, nf, 30 + idb, ws, st));
            hipLaunchKernelGGL(k_accept_first, dim3(blocks_for(m, kT)), dim3(kT), 0, st, sa, owner,
                               m, acc);
            GR_LAUNCHED("accept");
            (void)k2;
            ws.used = mark2;
        }
    }
    hipLaunchKernelGGL(k_parent, dim3(gb), dim3(kT), 0, st, best, ids, acc, n, pa);
    GR_LAUNCHED("parent");
    // pointer jumping to the roots; the depth halves each round.  Rounds go
    // in batches of kJumpBatch with one host check: only the batch's last
    // round reports, and a round that moves nothing means every later one
    // moves nothing too (extra rounds on converged pointers are no-ops)
    constexpr int kJumpBatch = 4;
    for (int round = 0;; round += kJumpBatch) {
        if (round > 64) return set_error(GR_EHIP, "pointer jumping did not converge");
        GR_HIP(hipMemsetAsync(small, 0, sizeof(int32_t), st));
        for (int b = 0; b < kJumpBatch; ++b) {
            hipLaunchKernelGGL(k_jump, dim3(gb), dim3(kT), 0, st, pa, n, pb,
                               b == kJumpBatch - 1 ? small : (int32_t*)nullptr);
            GR_LAUNCHED("jump");
            int32_t* t = pa; pa = pb; pb = t;
        }
        int32_t ch = 0;
        GR_HIP(hipMemcpyAsync(&ch, small, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        if (!ch) break;
    }
    int32_t* root = pa;
    int32_t* minid = pb;  // reuse
    GR_TRY(fill_i32(minid, 0x7fffffff, n, st));
    hipLaunchKernelGGL(k_min_member, dim3(gb), dim3(kT), 0, st, root, ids, n, minid);
    GR_LAUNCHED("min member");
    int32_t* flag_by_id = own;   // reuse
    int32_t* rank_by_id = acc;   // reuse (acc no longer needed)
    hipLaunchKernelGGL(k_leader_flags, dim3(gb), dim3(kT), 0, st, root, ids, minid, n, flag_by_id);
    GR_LAUNCHED("leader flags");
    GR_TRY(scan_exclusive_i32(flag_by_id, rank_by_id, n, small + 1, ws, st));
    hipLaunchKernelGGL(k_assign, dim3(gb), dim3(kT), 0, st, root, minid, rank_by_id, n, agg);
    GR_LAUNCHED("assign");
    int32_t nc = 0;
    GR_HIP(hipMemcpyAsync(&nc, small + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    *n_coarse = nc;
    ws.used = mark;
    return GR_OK;
}

// ---------------------------------------------------------------- Galerkin
// The coarse weights are summed once per unordered aggregate pair: only
// stored entries (v, j) with agg(v) < agg(j) (each fine edge between two
// aggregates exactly once) enter the sort, and every summed (I, J) is then
// written to both (I, J) and (J, I), so both directions carry equal bits.

// 8 lanes per fine row: the number of the row's kept entries
__global__ void k_rap_count(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ agg, int64_t n, int32_t* __restrict__ cnt) {
    const int64_t v = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    if (v >= n || rp[v + 1] - rp[v] > kLongRow) return;  // the 8 lanes of a row leave together
    const int32_t I = agg[v];
    int32_t c = 0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += 8) c += agg[col[e]] > I ? 1 : 0;
    c += __shfl_xor(c, 1, kWave);
    c += __shfl_xor(c, 2, kWave);
    c += __shfl_xor(c, 4, kWave);
    if (l == 0) cnt[v] = c;
}

// the kept pairs of each fine row, in entry order, from the row's offset on
// (so the tuples come in (fine row, entry) order, as a scan of per-entry
// flags would place them)
__global__ void k_rap_scatter(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const float* __restrict__ w, const int32_t* __restrict__ agg,
                              const int32_t* __restrict__ roff, int64_t n, int jbits,
                              uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t v = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    const int grp = (threadIdx.x & (kWave - 1)) >> 3;
    if (v >= n || rp[v + 1] - rp[v] > kLongRow) return;
    const int32_t I = agg[v];
    const int32_t e1 = rp[v + 1];
    int64_t out = roff[v];
    for (int32_t e0 = rp[v]; e0 < e1; e0 += 8) {  // the same trip count for the row's lanes
        const int32_t e = e0 + l;
        const int32_t J = e < e1 ? agg[col[e]] : -1;
        const bool keep = J > I;
        const uint32_t bits = (uint32_t)(__ballot(keep) >> (8 * grp)) & 0xffu;
        if (keep) {
            const int64_t s = out + __popc(bits & ((1u << l) - 1u));
            keys[s] = ((uint64_t)I << jbits) | (uint64_t)J;
            vals[s] = __float_as_uint(w[e]);
        }
        out += __popc(bits);
    }
}

// the same two passes for the listed rows of degree above kLongRow, a
// workgroup each (a hub would serialise 8 lanes)
__global__ void __launch_bounds__(kT) k_rap_count_long(const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ agg,
                                                       const int32_t* __restrict__ long_rows,
                                                       int32_t* __restrict__ cnt) {
    __shared__ int32_t wc[kT / kWave];
    const int32_t v = long_rows[blockIdx.x];
    const int32_t I = agg[v];
    int32_t c = 0;
    for (int32_t e = rp[v] + threadIdx.x; e < rp[v + 1]; e += kT) c += agg[col[e]] > I ? 1 : 0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) wc[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kT / kWave; ++w) t += wc[w];
        cnt[v] = t;
    }
}

__global__ void __launch_bounds__(kT) k_rap_scatter_long(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const float* __restrict__ w,
    const int32_t* __restrict__ agg, const int32_t* __restrict__ roff,
    const int32_t* __restrict__ long_rows, int jbits, uint64_t* __restrict__ keys,
    uint32_t* __restrict__ vals) {
    __shared__ int32_t wc[kT / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int32_t v = long_rows[blockIdx.x];
    const int32_t I = agg[v];
    const int32_t e1 = rp[v + 1];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    int64_t out = roff[v];
    for (int32_t e0 = rp[v]; e0 < e1; e0 += kT) {  // the same trip count for the whole block
        const int32_t e = e0 + tid;
        const int32_t J = e < e1 ? agg[col[e]] : -1;
        const bool keep = J > I;
        const uint64_t m = __ballot(keep);
        if (lane == 0) wc[wid] = __popcll(m);
        __syncthreads();
        int32_t pre = 0, tot = 0;
#pragma unroll
        for (int ww = 0; ww < kT / kWave; ++ww) {
            pre += ww < wid ? wc[ww] : 0;
            tot += wc[ww];
        }
        if (keep) {
            const int64_t s = out + pre + __popcll(m & lt);
            keys[s] = ((uint64_t)I << jbits) | (uint64_t)J;
            vals[s] = __float_as_uint(w[e]);
        }
        out += tot;
        __syncthreads();
    }
}

__global__ void k_run_heads(const uint64_t* __restrict__ keys, int64_t m, int32_t* __restrict__ head) {
    int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_run_starts(const int32_t* __restrict__ head, const int32_t* __restrict__ ridx,
                             int64_t m, int32_t* __restrict__ start) {
    int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    if (head[i]) start[ridx[i]] = (int32_t)i;
}

// Segmented sums, pass 1: tiles of kSegTile sorted values.  Each thread owns
// kSegItems consecutive values; a block-wide segmented scan (fixed shape)
// gives every item its running sum within its run and the tile; the value
// at the last item of each run piece inside the tile is stored.
constexpr int kSegItems = 8;
constexpr int kSegTile = kT * kSegItems;

struct SegPair {
    int f;      // a run starts inside
    float s;    // sum since the last run start
};
__device__ inline SegPair seg_op(SegPair a, SegPair b) {
    return SegPair{a.f | b.f, b.f ? b.s : a.s + b.s};
}

__global__ void __launch_bounds__(kT) k_seg_tile(const uint32_t* __restrict__ vals,
                                                 const int32_t* __restrict__ head, int64_t m,
                                                 float* __restrict__ piece) {
    __shared__ SegPair wtot[kT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
    float v[kSegItems];
    int h[kSegItems];
    SegPair mine{0, 0.0f};
#pragma unroll
    for (int i = 0; i < kSegItems; ++i) {
        int64_t k = base + i;
        bool ok = k < m;
        v[i] = ok ? __uint_as_float(vals[k]) : 0.0f;
        h[i] = ok ? head[k] : 0;
        mine = seg_op(mine, SegPair{h[i], v[i]});
    }
    // inclusive scan of the thread aggregates across the wave, then waves
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    SegPair inc = mine;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int of = __shfl_up(inc.f, off, kWave);
        float os = __shfl_up(inc.s, off, kWave);
        if (lane >= off) inc = seg_op(SegPair{of, os}, inc);
    }
    if (lane == kWave - 1) wtot[wid] = inc;
    __syncthreads();
    SegPair carry{0, 0.0f};
    for (int w2 = 0; w2 < wid; ++w2) carry = seg_op(carry, wtot[w2]);
    // exclusive prefix of this thread = carry (+) inclusive of the previous lane
    int pf = __shfl_up(inc.f, 1, kWave);
    float ps = __shfl_up(inc.s, 1, kWave);
    SegPair excl = lane > 0 ? seg_op(carry, SegPair{pf, ps}) : carry;
    float run = excl.s;
#pragma unroll
    for (int i = 0; i < kSegItems; ++i) {
        int64_t k = base + i;
        if (k >= m) break;
        run = h[i] ? v[i] : run + v[i];
        bool tile_end = (i == kSegItems - 1 && threadIdx.x == kT - 1);
        bool piece_end = (k == m - 1) || tile_end || head[k + 1];
        if (piece_end) piece[k] = run;
    }
}

// pass 2: one thread per run adds the run's pieces in tile order; the run's
// key (I << jbits | J, I < J) and sum go to ukey / uw, and its column J with
// the run index to mkey / midx: the runs are ordered by I, so a stable sort
// by J alone orders the mirrored entries (J, I) by row and column
__global__ void k_seg_runs(const uint64_t* __restrict__ keys, const int32_t* __restrict__ start,
                           const float* __restrict__ piece, int64_t runs, int64_t m, int jbits,
                           uint64_t* __restrict__ ukey, float* __restrict__ uw,
                           uint64_t* __restrict__ mkey, uint32_t* __restrict__ midx) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= runs) return;
    int64_t s = start[r];
    int64_t e = (r + 1 < runs) ? start[r + 1] : m;  // one past the last item
    float acc = 0.0f;
    for (int64_t t = s / kSegTile; t * kSegTile < e; ++t) {
        int64_t pe = min(e, (t + 1) * (int64_t)kSegTile) - 1;
        acc += piece[pe];
    }
    const uint64_t k = keys[s];
    const uint64_t mask = (1ull << jbits) - 1;
    ukey[r] = k;
    uw[r] = acc;
    mkey[r] = k & mask;
    midx[r] = (uint32_t)r;
}

// first and one-past-last position of every row in a key array sorted by
// row (row = key >> shift)
__global__ void k_row_bounds(const uint64_t* __restrict__ keys, int64_t cnt, int shift,
                             int32_t* __restrict__ rfirst, int32_t* __restrict__ rend) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= cnt) return;
    uint64_t I = keys[r] >> shift;
    if (r == 0 || (keys[r - 1] >> shift) != I) rfirst[I] = (int32_t)r;
    if (r == cnt - 1 || (keys[r + 1] >> shift) != I) rend[I] = (int32_t)(r + 1);
}

// coarse row I = [lower part: mirrored entries (I, J < I)] ++ [upper part:
// summed runs (I, J > I)]; both parts already ascending in J
__global__ void k_row_counts(const int32_t* __restrict__ ufirst, const int32_t* __restrict__ uend,
                             const int32_t* __restrict__ lfirst, const int32_t* __restrict__ lend,
                             int64_t n_c, int32_t* __restrict__ cnt) {
    int64_t I = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (I >= n_c) return;
    cnt[I] = (ufirst[I] >= 0 ? uend[I] - ufirst[I] : 0) + (lfirst[I] >= 0 ? lend[I] - lfirst[I] : 0);
}

__global__ void k_place_upper(const uint64_t* __restrict__ ukey, const float* __restrict__ uw,
                              int64_t runs, int jbits, const int32_t* __restrict__ c_row_ptr,
                              const int32_t* __restrict__ ufirst, const int32_t* __restrict__ lfirst,
                              const int32_t* __restrict__ lend, int32_t* __restrict__ c_col,
                              float* __restrict__ c_w) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= runs) return;
    const uint64_t k = ukey[r];
    const int64_t I = (int64_t)(k >> jbits);
    const int32_t nlow = lfirst[I] >= 0 ? lend[I] - lfirst[I] : 0;
    const int64_t p = (int64_t)c_row_ptr[I] + nlow + (r - ufirst[I]);
    c_col[p] = (int32_t)(k & ((1ull << jbits) - 1));
    c_w[p] = uw[r];
}

__global__ void k_place_lower(const uint64_t* __restrict__ mkey, const uint32_t* __restrict__ midx,
                              const uint64_t* __restrict__ ukey, const float* __restrict__ uw,
                              int64_t runs, int jbits, const int32_t* __restrict__ c_row_ptr,
                              const int32_t* __restrict__ lfirst, int32_t* __restrict__ c_col,
                              float* __restrict__ c_w) {
    int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= runs) return;
    const int64_t J = (int64_t)mkey[t];
    const uint32_t r = midx[t];
    const int64_t p = (int64_t)c_row_ptr[J] + (t - lfirst[J]);
    c_col[p] = (int32_t)(ukey[r] >> jbits);
    c_w[p] = uw[r];
}

int galerkin(const gr_graph* g, const int32_t* agg, int64_t n_c, int32_t* c_row_ptr,
             int32_t* c_col, float* c_w, int64_t* nnz_coarse, const int32_t* long_rows,
             int64_t n_long, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    *nnz_coarse = 0;
    size_t mark = ws.used;
    int32_t* rcnt = ws.take<int32_t>(n + 1);
    int32_t* roff = ws.take<int32_t>(n + 1);
    int32_t* small = ws.take<int32_t>(4);
    int32_t* row_cnt = ws.take<int32_t>(n_c + 1);
    int32_t* ufirst = ws.take<int32_t>(n_c + 1);
    int32_t* uend = ws.take<int32_t>(n_c + 1);
    int32_t* lfirst = ws.take<int32_t>(n_c + 1);
    int32_t* lend = ws.take<int32_t>(n_c + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin)");
    int32_t m = 0;
    if (nnz > 0) {
        const unsigned rb = blocks_for(n * 8, kT);
        hipLaunchKernelGGL(k_rap_count, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, agg, n, rcnt);
        GR_LAUNCHED("rap count");
        if (n_long > 0) {
            hipLaunchKernelGGL(k_rap_count_long, dim3((unsigned)n_long), dim3(kT), 0, st, g->row_ptr,
                               g->col, agg, long_rows, rcnt);
            GR_LAUNCHED("rap count (long rows)");
        }
        GR_TRY(scan_exclusive_i32(rcnt, roff, n, small, ws, st));
        GR_HIP(hipMemcpyAsync(&m, small, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
    }
    int32_t runs = 0;
    GR_TRY(fill_i32(ufirst, -1, n_c + 1, st));
    GR_TRY(fill_i32(uend, -1, n_c + 1, st));
    GR_TRY(fill_i32(lfirst, -1, n_c + 1, st));
    GR_TRY(fill_i32(lend, -1, n_c + 1, st));
    if (m > 0) {
        const int jbits = bits_for(n_c);
        uint64_t* k0 = ws.take<uint64_t>(m);
        uint32_t* v0 = ws.take<uint32_t>(m);
        uint64_t* k1 = ws.take<uint64_t>(m);
        uint32_t* v1 = ws.take<uint32_t>(m);
        int32_t* head = ws.take<int32_t>(m);
        int32_t* ridx = ws.take<int32_t>(m);
        int32_t* start = ws.take<int32_t>(m);
        float* piece = ws.take<float>(m);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin sort)");
        const unsigned rb = blocks_for(n * 8, kT);
        hipLaunchKernelGGL(k_rap_scatter, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, g->w, agg,
                           (const int32_t*)roff, n, jbits, k0, v0);
        GR_LAUNCHED("rap scatter");
        if (n_long > 0) {
            hipLaunchKernelGGL(k_rap_scatter_long, dim3((unsigned)n_long), dim3(kT), 0, st,
                               g->row_ptr, g->col, g->w, agg, (const int32_t*)roff, long_rows,
                               jbits, k0, v0);
            GR_LAUNCHED("rap scatter (long rows)");
        }
        GR_TRY(radix_sort_pairs(k0, v0, k1, v1, m, 2 * jbits, ws, st));
        const unsigned mb = blocks_for(m, kT);
        hipLaunchKernelGGL(k_run_heads, dim3(mb), dim3(kT), 0, st, k1, (int64_t)m, head);
        GR_LAUNCHED("run heads");
        GR_TRY(scan_exclusive_i32(head, ridx, m, small + 1, ws, st));
        hipLaunchKernelGGL(k_run_starts, dim3(mb), dim3(kT), 0, st, head, ridx, (int64_t)m, start);
        GR_LAUNCHED("run starts");
        hipLaunchKernelGGL(k_seg_tile, dim3(blocks_for(m, kSegTile)), dim3(kT), 0, st, v1, head,
                           (int64_t)m, piece);
        GR_LAUNCHED("segment tiles");
        GR_HIP(hipMemcpyAsync(&runs, small + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        // the unsorted keys are no longer needed: the runs' keys reuse k0
        uint64_t* ukey = k0;
        uint64_t* mk0 = ws.take<uint64_t>(runs);
        uint32_t* mi0 = ws.take<uint32_t>(runs);
        uint64_t* mk1 = ws.take<uint64_t>(runs);
        uint32_t* mi1 = ws.take<uint32_t>(runs);
        float* uw = ws.take<float>(runs);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin mirror)");
        const unsigned nbr = blocks_for(runs, kT);
        hipLaunchKernelGGL(k_seg_runs, dim3(nbr), dim3(kT), 0, st, k1, start, piece, (int64_t)runs,
                           (int64_t)m, jbits, ukey, uw, mk0, mi0);
        GR_LAUNCHED("segment runs");
        GR_TRY(radix_sort_pairs(mk0, mi0, mk1, mi1, runs, jbits, ws, st));
        hipLaunchKernelGGL(k_row_bounds, dim3(nbr), dim3(kT), 0, st, ukey, (int64_t)runs, jbits,
                           ufirst, uend);
        GR_LAUNCHED("upper row bounds");
        hipLaunchKernelGGL(k_row_bounds, dim3(nbr), dim3(kT), 0, st, mk1, (int64_t)runs, 0,
                           lfirst, lend);
        GR_LAUNCHED("lower row bounds");
        if (n_c > 0) {
            hipLaunchKernelGGL(k_row_counts, dim3(blocks_for(n_c, kT)), dim3(kT), 0, st, ufirst,
                               uend, lfirst, lend, n_c, row_cnt);
            GR_LAUNCHED("row counts");
        }
        GR_TRY(scan_exclusive_i32(row_cnt, c_row_ptr, n_c, c_row_ptr + n_c, ws, st));
        hipLaunchKernelGGL(k_place_upper, dim3(nbr), dim3(kT), 0, st, ukey, uw, (int64_t)runs, jbits,
                           c_row_ptr, ufirst, lfirst, lend, c_col, c_w);
        GR_LAUNCHED("place upper");
        hipLaunchKernelGGL(k_place_lower, dim3(nbr), dim3(kT), 0, st, mk1, mi1,
                           (const uint64_t*)ukey, uw, (int64_t)runs, jbits, c_row_ptr, lfirst, c_col,
                           c_w);
        GR_LAUNCHED("place lower");
    } else {
        GR_TRY(fill_i32(c_row_ptr, 0, n_c + 1, st));
    }
    *nnz_coarse = 2 * (int64_t)runs;
    ws.used = mark;
    return GR_OK;
}

}  // namespace gr
