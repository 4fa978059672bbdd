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

template <class KT>
__global__ void k_gather_keys(const KT* __restrict__ src, const uint32_t* __restrict__ idx,
                              int64_t m, KT* __restrict__ dst) {
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

// Pointer jumping in place: each node follows up to kHops parent links and
// stores the farthest node reached.  Links that other threads shorten in the
// meantime are read as they are: every value ever stored is an ancestor, so
// any interleaving only moves a node closer to its root.  `changed` (when
// given) is raised by one lane per wave that moved a pointer (a benign
// same-value race); a launch that moves nothing leaves every node pointing
// at a root.
constexpr int kHops = 8;
__global__ void k_jump(int32_t* __restrict__ pa, int64_t n, int32_t* __restrict__ changed) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    bool ch = false;
    if (v < n) {
        const int32_t p0 = pa[v];
        int32_t x = p0;
        for (int h = 0; h < kHops; ++h) {
            const int32_t y = pa[x];
            if (y == x) break;
            x = y;
        }
        if (x != p0) {
            pa[v] = x;
            ch = true;
        }
    }
    if (changed && __ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) *changed = 1;
}

__global__ void k_min_member(const int32_t* __restrict__ root, const int32_t* __restrict__ ids,
                             int64_t n, int32_t* __restrict__ minid) {
    int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (!ids) {
        // ids are the rows: of a run of lanes with one root (members next to
        // each other) the first has the smallest id; the others stay out of
        // the atomics on that address
        const int32_t r = v < n ? root[v] : -1;
        const int32_t rp = __shfl_up(r, 1, kWave);
        if ((threadIdx.x & (kWave - 1)) > 0 && rp == r) return;
    }
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
    const int32_t* accepted = acc;  // the forest edges taken
    if (n - nf >= target) {
        accepted = own;  // all of them
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
            hipLaunchKernelGGL(k_gather_keys<uint64_t>, dim3(fb), dim3(kT), 0, st, k1, sb, (int64_t)nf, kb);
            GR_LAUNCHED("gather keys");
            GR_TRY(radix_sort_pairs(kb, sb, ka, sa, nf, 30 + idb, ws, st));
            hipLaunchKernelGGL(k_accept_first, dim3(blocks_for(m, kT)), dim3(kT), 0, st, sa, owner,
                               m, acc);
            GR_LAUNCHED("accept");
            (void)k2;
            ws.used = mark2;
        }
    }
    hipLaunchKernelGGL(k_parent, dim3(gb), dim3(kT), 0, st, best, ids, accepted, n, pa);
    GR_LAUNCHED("parent");
    // pointer jumping to the roots, in place, kHops links per node and
    // launch (a launch at least multiplies the distance covered by kHops).
    // Launches go in batches of kJumpBatch with one host check: only the
    // batch's last launch reports, and a launch that moves nothing means
    // every later one moves nothing too
    constexpr int kJumpBatch = 2;
    for (int round = 0;; round += kJumpBatch) {
        if (round > 32) return set_error(GR_EHIP, "pointer jumping did not converge");
        GR_HIP(hipMemsetAsync(small, 0, sizeof(int32_t), st));
        for (int b = 0; b < kJumpBatch; ++b) {
            hipLaunchKernelGGL(k_jump, dim3(gb), dim3(kT), 0, st, pa, n,
                               b == kJumpBatch - 1 ? small : (int32_t*)nullptr);
            GR_LAUNCHED("jump");
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
// stored entries (v, j) with I = agg(v) < J = agg(j) (each fine edge between
// two aggregates exactly once) are kept, and every summed (I, J) is then
// written to both (I, J) and (J, I), so both directions carry equal bits.
//
// The fine rows are first sorted by aggregate (stable, so by row inside
// one), which lays every coarse row's kept entries out as one segment in
// (fine row, entry) order.  A segment of at most kGalCap entries is then
// sorted by (J, position in the segment) -- in registers, a lane per entry,
// when it has at most 8, 16, 32 or 64 entries, else in LDS -- and each run of
// equal J is summed in that order.  Longer segments (hub aggregates) go
// through one stable radix sort by (segment, J) and tiled segmented sums.
// The runs of every coarse row are compacted into one list ordered by
// (I, J), and a stable sort of that list by J places the mirrored entries.
constexpr int kGalCap = 2048;
enum {
    kGalNone = 0, kGalG8, kGalG16, kGalG32, kGalG64, kGalLds, kGalBig, kGalClasses
};

// 8 lanes per fine row: the number of the row's kept entries
// G lanes per row (G a power of two up to 8, sized to the mean degree)
template <int G>
__global__ void k_rap_count(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ agg, int64_t n, int32_t* __restrict__ cnt) {
    const int64_t v = ((int64_t)blockIdx.x * kT + threadIdx.x) / G;
    const int l = threadIdx.x % G;
    if (v >= n || rp[v + 1] - rp[v] > kLongRow) return;  // the G lanes of a row leave together
    const int32_t I = agg[v];
    int32_t c = 0;
    for (int32_t e = rp[v] + l; e < rp[v + 1]; e += G) c += agg[col[e]] > I ? 1 : 0;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) c += __shfl_xor(c, off, kWave);
    if (l == 0) cnt[v] = c;
}

// the same count for the listed rows of degree above kLongRow, a workgroup
// each (a hub would serialise 8 lanes)
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

// sort keys of the fine rows: their aggregate
__global__ void k_agg_keys(const int32_t* __restrict__ agg, int64_t n, uint32_t* __restrict__ key,
                           uint32_t* __restrict__ val) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)agg[v];
    val[v] = (uint32_t)v;
}

// kept-entry counts in sorted row order, and each row's sorted position
__global__ void k_sorted_counts(const uint32_t* __restrict__ rows, const int32_t* __restrict__ rcnt,
                                int64_t n, int32_t* __restrict__ cnt_s, int32_t* __restrict__ tpos) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= n) return;
    const uint32_t v = rows[t];
    cnt_s[t] = rcnt[v];
    tpos[v] = (int32_t)t;
}

// each coarse row's first and one-past-last sorted fine row (-1 for a coarse
// row without members, which a map given from outside may have)
__global__ void k_agg_bounds(const uint32_t* __restrict__ skey, int64_t n,
                             int32_t* __restrict__ afirst, int32_t* __restrict__ aend) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= n) return;
    if (t == 0 || skey[t - 1] != skey[t]) afirst[skey[t]] = (int32_t)t;
    if (t == n - 1 || skey[t + 1] != skey[t]) aend[skey[t]] = (int32_t)(t + 1);
}

// segment of coarse row I: [uoff[I], uoff[I] + ucnt[I]), and its class
__global__ void k_agg_segments(const int32_t* __restrict__ afirst, const int32_t* __restrict__ aend,
                               const int32_t* __restrict__ pos_s, int64_t n_c,
                               int32_t* __restrict__ uoff, int32_t* __restrict__ ucnt,
                               int32_t* __restrict__ cls) {
    const int64_t I = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (I >= n_c) return;
    const int32_t t0 = afirst[I];
    const int32_t o = t0 >= 0 ? pos_s[t0] : 0;
    const int32_t c = t0 >= 0 ? pos_s[aend[I]] - o : 0;
    uoff[I] = o;
    ucnt[I] = c;
    cls[I] = c == 0 ? kGalNone : c <= 8 ? kGalG8 : c <= 16 ? kGalG16 : c <= 32 ? kGalG32
           : c <= 64 ? kGalG64 : c <= kGalCap ? kGalLds : kGalBig;
}

// The coarse rows of every class, each class in row order, the classes one
// after another (a stable partition): per block of kT rows the class counts,
// a scan over (class, block), then each row to its class's offset for its
// block plus its rank among the block's rows of that class.
__global__ void __launch_bounds__(kT) k_class_counts(const int32_t* __restrict__ cls, int64_t n_c,
                                                     int32_t nblk, int32_t* __restrict__ bcnt) {
    __shared__ int32_t c[kGalClasses];
    if (threadIdx.x < kGalClasses) c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t I = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (I < n_c) atomicAdd(&c[cls[I]], 1);
    __syncthreads();
    if (threadIdx.x < kGalClasses) bcnt[(int64_t)threadIdx.x * nblk + blockIdx.x] = c[threadIdx.x];
}

__global__ void __launch_bounds__(kT) k_class_scatter(const int32_t* __restrict__ cls, int64_t n_c,
                                                      int32_t nblk, const int32_t* __restrict__ boffs,
                                                      int32_t* __restrict__ list) {
    __shared__ int32_t wc[kT / kWave][kGalClasses];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t I = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int k = I < n_c ? cls[I] : -1;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    int rank = 0;
#pragma unroll
    for (int q = 0; q < kGalClasses; ++q) {
        const uint64_t m = __ballot(k == q);
        if (lane == 0) wc[wid][q] = __popcll(m);
        if (k == q) rank = __popcll(m & below);
    }
    __syncthreads();
    if (k >= 0) {
        for (int w = 0; w < wid; ++w) rank += wc[w][k];
        list[boffs[(int64_t)k * nblk + blockIdx.x] + rank] = (int32_t)I;
    }
}

// first list position and row count of every class (class k at start[k],
// start[kGalClasses] = n_c)
__global__ void k_class_starts(const int32_t* __restrict__ boffs, int32_t nblk, int64_t n_c,
                               int32_t* __restrict__ start) {
    const int k = threadIdx.x;
    if (k < kGalClasses) start[k] = boffs[(int64_t)k * nblk];
    if (k == kGalClasses) start[k] = (int32_t)n_c;
}

// Kept entries of the sorted rows at their segment positions: column
// aggregate J and weight.  G lanes per row (as in the count); rows above
// kLongRow are skipped (k_place_long takes them).
template <int G>
__global__ void k_place_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const float* __restrict__ w, const int32_t* __restrict__ agg,
                             const uint32_t* __restrict__ rows, const int32_t* __restrict__ pos_s,
                             int64_t n, int32_t* __restrict__ ej, float* __restrict__ ew) {
    const int64_t t = ((int64_t)blockIdx.x * kT + threadIdx.x) / G;
    const int l = threadIdx.x % G;
    const int grp = (threadIdx.x & (kWave - 1)) / G;
    if (t >= n) return;
    const int32_t v = (int32_t)rows[t];
    const int32_t e1 = rp[v + 1];
    if (e1 - rp[v] > kLongRow) return;  // the G lanes of a row leave together
    const int32_t I = agg[v];
    int64_t out = pos_s[t];
    constexpr uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    for (int32_t e0 = rp[v]; e0 < e1; e0 += G) {  // the same trip count for the row's lanes
        const int32_t e = e0 + l;
        const int32_t J = e < e1 ? agg[col[e]] : -1;
        const bool keep = J > I;
        const uint32_t bits = (uint32_t)((__ballot(keep) >> (G * grp)) & gmask);
        if (keep) {
            const int64_t s = out + __popc(bits & ((1u << l) - 1u));
            ej[s] = J;
            ew[s] = w[e];
        }
        out += __popc(bits);
    }
}

__global__ void __launch_bounds__(kT) k_place_long(const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ w,
                                                   const int32_t* __restrict__ agg,
                                                   const int32_t* __restrict__ long_rows,
                                                   const int32_t* __restrict__ tpos,
                                                   const int32_t* __restrict__ pos_s,
                                                   int32_t* __restrict__ ej, float* __restrict__ ew) {
    __shared__ int32_t wc[kT / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int32_t v = long_rows[blockIdx.x];
    const int32_t I = agg[v];
    const int32_t e1 = rp[v + 1];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    int64_t out = pos_s[tpos[v]];
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
            ej[s] = J;
            ew[s] = w[e];
        }
        out += tot;
        __syncthreads();
    }
}

// G lanes per coarse row (G = 8, 16, 32 or 64, a segment of at most G entries):
// bitonic sort of (J, position) across the lanes, then each run's first
// lane adds the run's weights in position order; the runs go to the front
// of the segment (J to rj, sums to rw) and their number to rc.
template <int G>
__global__ void __launch_bounds__(kT) k_seg_sort_lanes(const int32_t* __restrict__ list,
                                                       int32_t nlist,
                                                       const int32_t* __restrict__ uoff,
                                                       const int32_t* __restrict__ ucnt,
                                                       const int32_t* __restrict__ ej,
                                                       const float* __restrict__ ew,
                                                       int32_t* __restrict__ rj,
                                                       float* __restrict__ rw,
                                                       int32_t* __restrict__ rc) {
    const int64_t gidx = ((int64_t)blockIdx.x * kT + threadIdx.x) / G;
    const int i = threadIdx.x % G;
    const int lane = threadIdx.x & (kWave - 1);
    const int gbase = lane - i;  // first lane of the group
    if (gidx >= nlist) return;   // the G lanes of a group leave together
    const int32_t I = list[gidx];
    const int32_t o = uoff[I], c = ucnt[I];
    uint64_t key = ~0ull;
    float val = 0.0f;
    if (i < c) {
        key = ((uint64_t)(uint32_t)ej[o + i] << 32) | (uint32_t)i;
        val = ew[o + i];
    }
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t plo = __shfl_xor((uint32_t)key, j, kWave);
            const uint32_t phi = __shfl_xor((uint32_t)(key >> 32), j, kWave);
            const float pv = __shfl_xor(val, j, kWave);
            const uint64_t pk = ((uint64_t)phi << 32) | plo;
            const bool up = (i & k) == 0;
            const bool lower = (i & j) == 0;  // this lane is the pair's first
            const bool take = lower == up ? pk < key : pk > key;
            if (take) {
                key = pk;
                val = pv;
            }
        }
    }
    const int32_t J = (int32_t)(key >> 32);
    const int32_t Jprev = __shfl(J, gbase + (i > 0 ? i - 1 : 0), kWave);
    const bool valid = i < c;
    const bool head = valid && (i == 0 || Jprev != J);
    // the run sums, in position order (until no run of the wave is open)
    float acc = val;
    bool open = head;
    for (int m = 1; m < G; ++m) {
        const int src = gbase + (i + m < G ? i + m : G - 1);
        const int32_t Jm = __shfl(J, src, kWave);
        const float wm = __shfl(val, src, kWave);
        open = open && i + m < c && Jm == J;
        if (open) acc += wm;
        if (!__ballot(open)) break;  // the same for the whole wave
    }
    const uint64_t hm = __ballot(head);
    const uint64_t gmask = (G == kWave ? ~0ull : ((1ull << G) - 1ull)) << gbase;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    if (head) {
        const int r = __popcll(hm & gmask & below);
        rj[o + r] = J;
        rw[o + r] = acc;
    }
    if (i == 0) rc[I] = __popcll(hm & gmask);
}

// A workgroup per coarse row of 65..kGalCap entries: bitonic sort of
// (J, position) in LDS, run sums in position order by each run's first
// entry, runs to the front of the segment.
__global__ void __launch_bounds__(kT) k_seg_sort_lds(const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ uoff,
                                                     const int32_t* __restrict__ ucnt,
                                                     const int32_t* __restrict__ ej,
                                                     const float* __restrict__ ew,
                                                     int32_t* __restrict__ rj,
                                                     float* __restrict__ rw,
                                                     int32_t* __restrict__ rc) {
    __shared__ uint64_t sk[kGalCap];
    __shared__ float sv[kGalCap];
    __shared__ int32_t hs[kT / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int32_t I = list[blockIdx.x];
    const int32_t o = uoff[I], c = ucnt[I];
    int P = 128;
    while (P < c) P <<= 1;
    for (int i = tid; i < P; i += kT) {
        sk[i] = i < c ? (((uint64_t)(uint32_t)ej[o + i] << 32) | (uint32_t)i) : ~0ull;
        sv[i] = i < c ? ew[o + i] : 0.0f;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += kT) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = sk[i], b = sk[p];
                    if ((a > b) == up) {
                        sk[i] = b;
                        sk[p] = a;
                        const float t = sv[i];
                        sv[i] = sv[p];
                        sv[p] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    // runs: heads counted in chunk order, each head sums its run
    int32_t base = 0;
    for (int c0 = 0; c0 < c; c0 += kT) {
        const int i = c0 + tid;
        const int32_t J = i < c ? (int32_t)(sk[i] >> 32) : -1;
        const bool head = i < c && (i == 0 || (int32_t)(sk[i - 1] >> 32) != J);
        const uint64_t hm = __ballot(head);
        if (lane == 0) hs[wid] = __popcll(hm);
        __syncthreads();
        int32_t pre = 0, tot = 0;
        for (int ww = 0; ww < kT / kWave; ++ww) {
            pre += ww < wid ? hs[ww] : 0;
            tot += hs[ww];
        }
        if (head) {
            float acc = sv[i];
            for (int m = i + 1; m < c && (int32_t)(sk[m] >> 32) == J; ++m) acc += sv[m];
            const int r = base + pre + __popcll(hm & (lane == 0 ? 0ull : (~0ull >> (kWave - lane))));
            rj[o + r] = J;
            rw[o + r] = acc;
        }
        base += tot;
        __syncthreads();
    }
    if (tid == 0) rc[I] = base;
}

// position of t among the sorted offsets off[0..cnt): the last i with
// off[i] <= t
__device__ inline int32_t seg_of(const int32_t* __restrict__ off, int32_t cnt, int64_t t) {
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// the entries of the long segments, concatenated in list order: key
// (list rank << jbits | J), value the weight's bits; a thread per entry
template <class KT>
__global__ void k_big_gather(const int32_t* __restrict__ list, int32_t nbig,
                             const int32_t* __restrict__ boff, int64_t mb,
                             const int32_t* __restrict__ uoff, const int32_t* __restrict__ ej,
                             const float* __restrict__ ew, int jbits, KT* __restrict__ bk,
                             uint32_t* __restrict__ bv) {
    const int64_t d = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (d >= mb) return;
    const int32_t b = seg_of(boff, nbig, d);
    const int64_t src = (int64_t)uoff[list[b]] + (d - boff[b]);
    bk[d] = ((KT)(uint32_t)b << jbits) | (KT)(uint32_t)ej[src];
    bv[d] = __float_as_uint(ew[src]);
}

__global__ void k_big_sizes(const int32_t* __restrict__ list, int32_t nbig,
                            const int32_t* __restrict__ ucnt, int32_t* __restrict__ sz) {
    const int64_t b = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (b < nbig) sz[b] = ucnt[list[b]];
}

template <class KT>
__global__ void k_run_heads(const KT* __restrict__ keys, int64_t m, int32_t* __restrict__ head) {
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

// pass 2 for the long segments: one thread per run adds the run's pieces in
// tile order and writes (J, sum) at the run's rank inside its coarse row
template <class KT>
__global__ void k_big_runs(const KT* __restrict__ keys, const int32_t* __restrict__ start,
                           const float* __restrict__ piece, int64_t runs, int64_t m, int jbits,
                           const int32_t* __restrict__ list, const int32_t* __restrict__ uoff,
                           const int32_t* __restrict__ bfirst, int32_t* __restrict__ rj,
                           float* __restrict__ rw) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= runs) return;
    int64_t s = start[r];
    int64_t e = (r + 1 < runs) ? start[r + 1] : m;  // one past the last item
    float acc = 0.0f;
    for (int64_t t = s / kSegTile; t * kSegTile < e; ++t) {
        int64_t pe = min(e, (t + 1) * (int64_t)kSegTile) - 1;
        acc += piece[pe];
    }
    const uint64_t k = (uint64_t)keys[s];
    const int32_t b = (int32_t)(k >> jbits);
    const int32_t I = list[b];
    const int64_t pos = (int64_t)uoff[I] + (r - bfirst[b]);
    rj[pos] = (int32_t)(k & ((1ull << jbits) - 1));
    rw[pos] = acc;
}

// first and one-past-last position of every row in a key array sorted by
// row (row = key >> shift)
template <class KT>
__global__ void k_row_bounds(const KT* __restrict__ keys, int64_t cnt, int shift,
                             int32_t* __restrict__ rfirst, int32_t* __restrict__ rend) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= cnt) return;
    const KT I = keys[r] >> shift;
    if (r == 0 || (keys[r - 1] >> shift) != I) rfirst[I] = (int32_t)r;
    if (r == cnt - 1 || (keys[r + 1] >> shift) != I) rend[I] = (int32_t)(r + 1);
}

__global__ void k_big_counts(const int32_t* __restrict__ list, int32_t nbig,
                             const int32_t* __restrict__ bfirst, const int32_t* __restrict__ bend,
                             int32_t* __restrict__ rc) {
    const int64_t b = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (b < nbig) rc[list[b]] = bfirst[b] >= 0 ? bend[b] - bfirst[b] : 0;
}

// The runs of every coarse row into one list ordered by (I, J): ukey = (I <<
// jbits | J), uw the sum; the mirror sort's keys J and run indices.  8 lanes
// per coarse row.
__global__ void k_compact_runs(const int32_t* __restrict__ uoff, const int32_t* __restrict__ ucnt,
                               const int32_t* __restrict__ rc,
                               const int32_t* __restrict__ roff, int64_t n_c, int jbits,
                               const int32_t* __restrict__ rj, const float* __restrict__ rw,
                               uint64_t* __restrict__ ukey, float* __restrict__ uw,
                               uint32_t* __restrict__ mkey, uint32_t* __restrict__ midx) {
    const int64_t I = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    if (I >= n_c || ucnt[I] > 64) return;  // longer rows: k_compact_long
    const int32_t c = rc[I], o = uoff[I];
    const int64_t d = roff[I];
    for (int32_t k = l; k < c; k += 8) {
        const int32_t J = rj[o + k];
        ukey[d + k] = ((uint64_t)I << jbits) | (uint64_t)(uint32_t)J;
        uw[d + k] = rw[o + k];
        mkey[d + k] = (uint32_t)J;
        midx[d + k] = (uint32_t)(d + k);
    }
}

// the same for the coarse rows of more than 64 kept entries (a list of nh,
// their runs at hoff in list order): a thread per run
__global__ void k_compact_long(const int32_t* __restrict__ hlist, int32_t nh,
                               const int32_t* __restrict__ hoff, int64_t hr,
                               const int32_t* __restrict__ uoff, const int32_t* __restrict__ roff,
                               int jbits, const int32_t* __restrict__ rj,
                               const float* __restrict__ rw, uint64_t* __restrict__ ukey,
                               float* __restrict__ uw, uint32_t* __restrict__ mkey,
                               uint32_t* __restrict__ midx) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= hr) return;
    const int32_t h = seg_of(hoff, nh, t);
    const int32_t I = hlist[h];
    const int64_t k = t - hoff[h];
    const int64_t d = roff[I] + k;
    const int32_t J = rj[uoff[I] + k];
    ukey[d] = ((uint64_t)I << jbits) | (uint64_t)(uint32_t)J;
    uw[d] = rw[uoff[I] + k];
    mkey[d] = (uint32_t)J;
    midx[d] = (uint32_t)d;
}

__global__ void k_long_runs(const int32_t* __restrict__ hlist, int32_t nh,
                            const int32_t* __restrict__ rc, int32_t* __restrict__ hrc) {
    const int64_t h = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (h < nh) hrc[h] = rc[hlist[h]];
}

// coarse row I = [lower part: mirrored entries (I, J < I)] ++ [upper part:
// summed runs (I, J > I)]; both parts already ascending in J
__global__ void k_row_counts(const int32_t* __restrict__ rc, const int32_t* __restrict__ lfirst,
                             const int32_t* __restrict__ lend, int64_t n_c,
                             int32_t* __restrict__ cnt) {
    int64_t I = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (I >= n_c) return;
    cnt[I] = rc[I] + (lfirst[I] >= 0 ? lend[I] - lfirst[I] : 0);
}

__global__ void k_place_upper(const uint64_t* __restrict__ ukey, const float* __restrict__ uw,
                              int64_t runs, int jbits, const int32_t* __restrict__ c_row_ptr,
                              const int32_t* __restrict__ roff, const int32_t* __restrict__ lfirst,
                              const int32_t* __restrict__ lend, int32_t* __restrict__ c_col,
                              float* __restrict__ c_w) {
    int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= runs) return;
    const uint64_t k = ukey[r];
    const int64_t I = (int64_t)(k >> jbits);
    const int32_t nlow = lfirst[I] >= 0 ? lend[I] - lfirst[I] : 0;
    const int64_t p = (int64_t)c_row_ptr[I] + nlow + (r - roff[I]);
    c_col[p] = (int32_t)(k & ((1ull << jbits) - 1));
    c_w[p] = uw[r];
}

__global__ void k_place_lower(const uint32_t* __restrict__ mkey, const uint32_t* __restrict__ midx,
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

// the stable radix sort for either key width
static int sort_pairs(uint32_t* a, uint32_t* av, uint32_t* b, uint32_t* bv, int64_t n, int bits,
                      Arena& ws, hipStream_t st) {
    return radix_sort_pairs32(a, av, b, bv, n, bits, ws, st);
}
static int sort_pairs(uint64_t* a, uint32_t* av, uint64_t* b, uint32_t* bv, int64_t n, int bits,
                      Arena& ws, hipStream_t st) {
    return radix_sort_pairs(a, av, b, bv, n, bits, ws, st);
}

// The runs of the hub segments (more than kGalCap kept entries): their
// entries gathered in segment order, sorted by (segment rank, J) with the
// stable radix sort, summed by fixed tiles; keys of 32 bits where they fit.
template <class KT>
static int hub_runs(const int32_t* blist, int32_t nbig, const int32_t* boff, int32_t mb,
                    const int32_t* uoff, const int32_t* ej, const float* ew, int jbits, int bbits,
                    int32_t* small, int32_t* bfirst, int32_t* bend, int32_t* rj, float* rw,
                    int32_t* rc, Arena& ws, hipStream_t st) {
    KT* bk0 = ws.take<KT>(mb);
    uint32_t* bv0 = ws.take<uint32_t>(mb);
    KT* bk1 = ws.take<KT>(mb);
    uint32_t* bv1 = ws.take<uint32_t>(mb);
    int32_t* head = ws.take<int32_t>(mb);
    int32_t* ridx = ws.take<int32_t>(mb);
    int32_t* start = ws.take<int32_t>(mb);
    float* piece = ws.take<float>(mb);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin long rows)");
    hipLaunchKernelGGL(k_big_gather<KT>, dim3(blocks_for(mb, kT)), dim3(kT), 0, st, blist, nbig,
                       (const int32_t*)boff, (int64_t)mb, (const int32_t*)uoff,
                       (const int32_t*)ej, (const float*)ew, jbits, bk0, bv0);
    GR_LAUNCHED("long segments gather");
    GR_TRY(sort_pairs(bk0, bv0, bk1, bv1, mb, bbits + jbits, ws, st));
    const unsigned mbb = blocks_for(mb, kT);
    hipLaunchKernelGGL(k_run_heads<KT>, dim3(mbb), dim3(kT), 0, st, (const KT*)bk1, (int64_t)mb,
                       head);
    GR_LAUNCHED("run heads");
    GR_TRY(scan_exclusive_i32(head, ridx, mb, small + 9, ws, st));
    hipLaunchKernelGGL(k_run_starts, dim3(mbb), dim3(kT), 0, st, (const int32_t*)head,
                       (const int32_t*)ridx, (int64_t)mb, start);
    GR_LAUNCHED("run starts");
    hipLaunchKernelGGL(k_seg_tile, dim3(blocks_for(mb, kSegTile)), dim3(kT), 0, st,
                       (const uint32_t*)bv1, (const int32_t*)head, (int64_t)mb, piece);
    GR_LAUNCHED("segment tiles");
    int32_t bruns = 0;
    GR_HIP(hipMemcpyAsync(&bruns, small + 9, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    // each long segment's first run: the run keys' segment bits
    KT* rkey = bk0;  // free again
    hipLaunchKernelGGL(k_gather_keys<KT>, dim3(blocks_for(bruns, kT)), dim3(kT), 0, st,
                       (const KT*)bk1, (const uint32_t*)start, (int64_t)bruns, rkey);
    GR_LAUNCHED("run keys");
    GR_TRY(fill_i32(bfirst, -1, nbig, st));
    GR_TRY(fill_i32(bend, -1, nbig, st));
    hipLaunchKernelGGL(k_row_bounds<KT>, dim3(blocks_for(bruns, kT)), dim3(kT), 0, st,
                       (const KT*)rkey, (int64_t)bruns, jbits, bfirst, bend);
    GR_LAUNCHED("long segment run bounds");
    hipLaunchKernelGGL(k_big_runs<KT>, dim3(blocks_for(bruns, kT)), dim3(kT), 0, st,
                       (const KT*)bk1, (const int32_t*)start, (const float*)piece,
                       (int64_t)bruns, (int64_t)mb, jbits, blist, (const int32_t*)uoff,
                       (const int32_t*)bfirst, rj, rw);
    GR_LAUNCHED("long segment runs");
    hipLaunchKernelGGL(k_big_counts, dim3(blocks_for(nbig, kT)), dim3(kT), 0, st, blist, nbig,
                       (const int32_t*)bfirst, (const int32_t*)bend, rc);
    GR_LAUNCHED("long segment run counts");
    return GR_OK;
}

int galerkin(const gr_graph* g, const int32_t* agg, int64_t n_c, int32_t* c_row_ptr,
             int32_t* c_col, float* c_w, int64_t* nnz_coarse, const int32_t* long_rows,
             int64_t n_long, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    *nnz_coarse = 0;
    if (n == 0) return fill_i32(c_row_ptr, 0, n_c + 1, st);
    size_t mark = ws.used;
    int32_t* rcnt = ws.take<int32_t>(n + 1);
    int32_t* cnt_s = ws.take<int32_t>(n + 1);
    int32_t* pos_s = ws.take<int32_t>(n + 1);
    int32_t* tpos = ws.take<int32_t>(n + 1);
    uint32_t* akey = ws.take<uint32_t>(n);
    uint32_t* aval = ws.take<uint32_t>(n);
    uint32_t* skey = ws.take<uint32_t>(n);
    uint32_t* rows = ws.take<uint32_t>(n);
    int32_t* small = ws.take<int32_t>(16);
    int32_t* afirst = ws.take<int32_t>(n_c + 1);
    int32_t* aend = ws.take<int32_t>(n_c + 1);
    int32_t* uoff = ws.take<int32_t>(n_c + 1);
    int32_t* ucnt = ws.take<int32_t>(n_c + 1);
    int32_t* rc = ws.take<int32_t>(n_c + 1);
    int32_t* roff = ws.take<int32_t>(n_c + 1);
    int32_t* lists = ws.take<int32_t>(n_c + 1);
    int32_t* row_cnt = ws.take<int32_t>(n_c + 1);
    int32_t* lfirst = ws.take<int32_t>(n_c + 1);
    int32_t* lend = ws.take<int32_t>(n_c + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin)");
    const unsigned nb = blocks_for(n, kT);
    // lanes per fine row in the count and the placement: a power of two up
    // to 8, about the mean degree (GR_GAL_LANES=g forces g)
    int rl = 1;
    while (rl < 8 && rl * 2 <= (nnz + n - 1) / std::max<int64_t>(n, 1)) rl *= 2;
    if (const char* gl = getenv("GR_GAL_LANES")) {
        const int v = atoi(gl);
        if (v == 1 || v == 2 || v == 4 || v == 8) rl = v;
    }
    // kept entries per fine row, the rows in aggregate order, and each coarse
    // row's segment
    if (nnz > 0) {
        const unsigned rb = blocks_for(n * rl, kT);
        switch (rl) {
            case 1: hipLaunchKernelGGL(k_rap_count<1>, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, agg, n, rcnt); break;
            case 2: hipLaunchKernelGGL(k_rap_count<2>, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, agg, n, rcnt); break;
            case 4: hipLaunchKernelGGL(k_rap_count<4>, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, agg, n, rcnt); break;
            default: hipLaunchKernelGGL(k_rap_count<8>, dim3(rb), dim3(kT), 0, st, g->row_ptr, g->col, agg, n, rcnt); break;
        }
        GR_LAUNCHED("rap count");
        if (n_long > 0) {
            hipLaunchKernelGGL(k_rap_count_long, dim3((unsigned)n_long), dim3(kT), 0, st, g->row_ptr,
                               g->col, agg, long_rows, rcnt);
            GR_LAUNCHED("rap count (long rows)");
        }
    } else {
        GR_TRY(fill_i32(rcnt, 0, n, st));
    }
    hipLaunchKernelGGL(k_agg_keys, dim3(nb), dim3(kT), 0, st, agg, n, akey, aval);
    GR_LAUNCHED("aggregate keys");
    GR_TRY(radix_sort_pairs32(akey, aval, skey, rows, n, bits_for(n_c), ws, st));
    hipLaunchKernelGGL(k_sorted_counts, dim3(nb), dim3(kT), 0, st, (const uint32_t*)rows,
                       (const int32_t*)rcnt, n, cnt_s, tpos);
    GR_LAUNCHED("sorted counts");
    GR_TRY(scan_exclusive_i32(cnt_s, pos_s, n, pos_s + n, ws, st));
    GR_TRY(fill_i32(small, 0, 16, st));
    GR_TRY(fill_i32(afirst, -1, n_c, st));
    hipLaunchKernelGGL(k_agg_bounds, dim3(nb), dim3(kT), 0, st, (const uint32_t*)skey, n, afirst,
                       aend);
    GR_LAUNCHED("aggregate row bounds");
    // the class of every coarse row (rc holds it until the runs are counted)
    hipLaunchKernelGGL(k_agg_segments, dim3(blocks_for(n_c, kT)), dim3(kT), 0, st,
                       (const int32_t*)afirst, (const int32_t*)aend, (const int32_t*)pos_s, n_c, uoff,
                       ucnt, rc);
    GR_LAUNCHED("aggregate segments");
    // the rows of each class in row order, classes one after another
    {
        const int32_t nblk = (int32_t)blocks_for(n_c, kT);
        const size_t mk = ws.used;
        int32_t* bcnt = ws.take<int32_t>((size_t)kGalClasses * nblk + 1);
        int32_t* boffs = ws.take<int32_t>((size_t)kGalClasses * nblk + 1);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin classes)");
        hipLaunchKernelGGL(k_class_counts, dim3(nblk), dim3(kT), 0, st, (const int32_t*)rc, n_c, nblk,
                           bcnt);
        GR_LAUNCHED("class counts");
        GR_TRY(scan_exclusive_i32(bcnt, boffs, (int64_t)kGalClasses * nblk, nullptr, ws, st));
        hipLaunchKernelGGL(k_class_scatter, dim3(nblk), dim3(kT), 0, st, (const int32_t*)rc, n_c, nblk,
                           (const int32_t*)boffs, lists);
        GR_LAUNCHED("class lists");
        hipLaunchKernelGGL(k_class_starts, dim3(1), dim3(kWave), 0, st, (const int32_t*)boffs, nblk,
                           n_c, small);
        GR_LAUNCHED("class starts");
        ws.used = mk;  // stream order keeps them valid for the launches above
    }
    int32_t cs[kGalClasses + 1] = {0};  // class starts in the list
    GR_HIP(hipMemcpyAsync(cs, small, sizeof(int32_t) * (kGalClasses + 1), hipMemcpyDeviceToHost, st));
    int32_t m = 0;
    GR_HIP(hipMemcpyAsync(&m, pos_s + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    GR_TRY(fill_i32(lfirst, -1, n_c + 1, st));
    GR_TRY(fill_i32(lend, -1, n_c + 1, st));
    if (m == 0) {
        GR_TRY(fill_i32(c_row_ptr, 0, n_c + 1, st));
        ws.used = mark;
        return GR_OK;
    }
    const int jbits = bits_for(n_c);
    int32_t* ej = ws.take<int32_t>(m);
    float* ew = ws.take<float>(m);
    int32_t* rj = ws.take<int32_t>(m);
    float* rw = ws.take<float>(m);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin entries)");
    // the kept entries in segment order
#define GR_PLACE(GG)                                                                               \
    hipLaunchKernelGGL(k_place_rows<GG>, dim3(blocks_for(n * GG, kT)), dim3(kT), 0, st, g->row_ptr, \
                       g->col, g->w, agg, (const uint32_t*)rows, (const int32_t*)pos_s, n, ej, ew)
    switch (rl) {
        case 1: GR_PLACE(1); break;
        case 2: GR_PLACE(2); break;
        case 4: GR_PLACE(4); break;
        default: GR_PLACE(8); break;
    }
#undef GR_PLACE
    GR_LAUNCHED("place rows");
    if (n_long > 0) {
        hipLaunchKernelGGL(k_place_long, dim3((unsigned)n_long), dim3(kT), 0, st, g->row_ptr, g->col,
                           g->w, agg, long_rows, (const int32_t*)tpos, (const int32_t*)pos_s, ej, ew);
        GR_LAUNCHED("place rows (long)");
    }
    GR_TRY(fill_i32(rc, 0, n_c, st));
    // each segment collapsed into its runs
    auto cls_n = [&](int k) { return cs[k + 1] - cs[k]; };
    auto cls_list = [&](int k) { return (const int32_t*)(lists + cs[k]); };
    if (cls_n(kGalG8) > 0) {
        hipLaunchKernelGGL(k_seg_sort_lanes<8>, dim3(blocks_for((int64_t)cls_n(kGalG8) * 8, kT)),
                           dim3(kT), 0, st, cls_list(kGalG8), cls_n(kGalG8), (const int32_t*)uoff,
                           (const int32_t*)ucnt, (const int32_t*)ej, (const float*)ew, rj, rw, rc);
        GR_LAUNCHED("segments of <= 8");
    }
    if (cls_n(kGalG16) > 0) {
        hipLaunchKernelGGL(k_seg_sort_lanes<16>, dim3(blocks_for((int64_t)cls_n(kGalG16) * 16, kT)),
                           dim3(kT), 0, st, cls_list(kGalG16), cls_n(kGalG16), (const int32_t*)uoff,
                           (const int32_t*)ucnt, (const int32_t*)ej, (const float*)ew, rj, rw, rc);
        GR_LAUNCHED("segments of <= 16");
    }
    if (cls_n(kGalG32) > 0) {
        hipLaunchKernelGGL(k_seg_sort_lanes<32>, dim3(blocks_for((int64_t)cls_n(kGalG32) * 32, kT)),
                           dim3(kT), 0, st, cls_list(kGalG32), cls_n(kGalG32), (const int32_t*)uoff,
                           (const int32_t*)ucnt, (const int32_t*)ej, (const float*)ew, rj, rw, rc);
        GR_LAUNCHED("segments of <= 32");
    }
    if (cls_n(kGalG64) > 0) {
        hipLaunchKernelGGL(k_seg_sort_lanes<64>, dim3(blocks_for((int64_t)cls_n(kGalG64) * 64, kT)),
                           dim3(kT), 0, st, cls_list(kGalG64), cls_n(kGalG64), (const int32_t*)uoff,
                           (const int32_t*)ucnt, (const int32_t*)ej, (const float*)ew, rj, rw, rc);
        GR_LAUNCHED("segments of <= 64");
    }
    if (cls_n(kGalLds) > 0) {
        hipLaunchKernelGGL(k_seg_sort_lds, dim3((unsigned)cls_n(kGalLds)), dim3(kT), 0, st,
                           cls_list(kGalLds), (const int32_t*)uoff, (const int32_t*)ucnt,
                           (const int32_t*)ej, (const float*)ew, rj, rw, rc);
        GR_LAUNCHED("segments in LDS");
    }
    const int32_t nbig = cls_n(kGalBig);
    if (nbig > 0) {
        // long segments: one stable sort by (segment, J), tiled sums
        const size_t mk = ws.used;
        const int32_t* blist = cls_list(kGalBig);
        int32_t* bsz = ws.take<int32_t>(nbig + 1);
        int32_t* boff = ws.take<int32_t>(nbig + 1);
        int32_t* bfirst = ws.take<int32_t>(nbig + 1);
        int32_t* bend = ws.take<int32_t>(nbig + 1);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin long rows)");
        hipLaunchKernelGGL(k_big_sizes, dim3(blocks_for(nbig, kT)), dim3(kT), 0, st, blist, nbig,
                           (const int32_t*)ucnt, bsz);
        GR_LAUNCHED("long segment sizes");
        GR_TRY(scan_exclusive_i32(bsz, boff, nbig, small + 8, ws, st));
        int32_t mb = 0;
        GR_HIP(hipMemcpyAsync(&mb, small + 8, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        // keys (segment rank << jbits | J) of 32 bits where they fit
        const int bbits = bits_for(nbig);
        if (bbits + jbits <= 32)
            GR_TRY((hub_runs<uint32_t>(blist, nbig, boff, mb, uoff, ej, ew, jbits, bbits, small, bfirst,
                                       bend, rj, rw, rc, ws, st)));
        else
            GR_TRY((hub_runs<uint64_t>(blist, nbig, boff, mb, uoff, ej, ew, jbits, bbits, small, bfirst,
                                       bend, rj, rw, rc, ws, st)));
        ws.used = mk;
    }
    // all runs in (I, J) order, then the mirrored entries by a stable sort on J;
    // the rows of more than 64 kept entries (LDS and hub classes) compact
    // their runs a thread per run, at offsets of their own (one host read
    // brings both totals)
    GR_TRY(scan_exclusive_i32(rc, roff, n_c, small + 10, ws, st));
    const int32_t nh = cs[kGalClasses] - cs[kGalLds];
    int32_t* hoff = nullptr;
    if (nh > 0) {
        int32_t* hrc = ws.take<int32_t>(nh + 1);
        hoff = ws.take<int32_t>(nh + 1);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin long rows)");
        hipLaunchKernelGGL(k_long_runs, dim3(blocks_for(nh, kT)), dim3(kT), 0, st,
                           cls_list(kGalLds), nh, (const int32_t*)rc, hrc);
        GR_LAUNCHED("long row run counts");
        GR_TRY(scan_exclusive_i32(hrc, hoff, nh, small + 11, ws, st));
    }
    int32_t tot[2] = {0, 0};  // runs, runs of the long rows
    GR_HIP(hipMemcpyAsync(tot, small + 10, sizeof(tot), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    const int32_t runs = tot[0];
    const int32_t hr = nh > 0 ? tot[1] : 0;
    uint64_t* ukey = ws.take<uint64_t>(runs);
    float* uw = ws.take<float>(runs);
    uint32_t* mk0 = ws.take<uint32_t>(runs);
    uint32_t* mi0 = ws.take<uint32_t>(runs);
    uint32_t* mk1 = ws.take<uint32_t>(runs);
    uint32_t* mi1 = ws.take<uint32_t>(runs);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (galerkin mirror)");
    hipLaunchKernelGGL(k_compact_runs, dim3(blocks_for(n_c * 8, kT)), dim3(kT), 0, st,
                       (const int32_t*)uoff, (const int32_t*)ucnt, (const int32_t*)rc,
                       (const int32_t*)roff, n_c, jbits, (const int32_t*)rj, (const float*)rw, ukey,
                       uw, mk0, mi0);
    GR_LAUNCHED("compact runs");
    if (hr > 0) {
        hipLaunchKernelGGL(k_compact_long, dim3(blocks_for(hr, kT)), dim3(kT), 0, st,
                           cls_list(kGalLds), nh, (const int32_t*)hoff, (int64_t)hr,
                           (const int32_t*)uoff, (const int32_t*)roff, jbits, (const int32_t*)rj,
                           (const float*)rw, ukey, uw, mk0, mi0);
        GR_LAUNCHED("compact runs (long rows)");
    }
    GR_TRY(radix_sort_pairs32(mk0, mi0, mk1, mi1, runs, jbits, ws, st));
    const unsigned nbr = blocks_for(runs, kT);
    // row I's runs sit at [roff[I], roff[I] + rc[I]) of the upper list
    hipLaunchKernelGGL(k_row_bounds<uint32_t>, dim3(nbr), dim3(kT), 0, st, (const uint32_t*)mk1,
                       (int64_t)runs, 0, lfirst, lend);
    GR_LAUNCHED("lower row bounds");
    hipLaunchKernelGGL(k_row_counts, dim3(blocks_for(n_c, kT)), dim3(kT), 0, st,
                       (const int32_t*)rc, (const int32_t*)lfirst, (const int32_t*)lend, n_c,
                       row_cnt);
    GR_LAUNCHED("row counts");
    GR_TRY(scan_exclusive_i32(row_cnt, c_row_ptr, n_c, c_row_ptr + n_c, ws, st));
    hipLaunchKernelGGL(k_place_upper, dim3(nbr), dim3(kT), 0, st, (const uint64_t*)ukey,
                       (const float*)uw, (int64_t)runs, jbits, (const int32_t*)c_row_ptr,
                       (const int32_t*)roff, (const int32_t*)lfirst, (const int32_t*)lend, c_col,
                       c_w);
    GR_LAUNCHED("place upper");
    hipLaunchKernelGGL(k_place_lower, dim3(nbr), dim3(kT), 0, st, (const uint32_t*)mk1,
                       (const uint32_t*)mi1, (const uint64_t*)ukey, (const float*)uw, (int64_t)runs,
                       jbits, (const int32_t*)c_row_ptr, (const int32_t*)lfirst, c_col, c_w);
    GR_LAUNCHED("place lower");
    *nnz_coarse = 2 * (int64_t)runs;
    ws.used = mark;
    return GR_OK;
}

}  // namespace gr
