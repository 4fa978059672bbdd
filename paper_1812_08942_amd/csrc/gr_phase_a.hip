// Phase A of the spectral reduction (Sec. 3.2): graph checks, greedy
// colouring, colour-major relabel, random test vectors and multicolour
// Gauss-Seidel smoothing (the affinity is in gr_affinity.hip).
//
// Layout.  Test vectors are node-major rows of K values; a row is split into
// Q 16-byte chunks (4 float32 or 8 bfloat16 values).  A row-group of L = Q*P
// lanes handles one CSR row: lane (p, q) walks neighbours p, p+P, ... and
// accumulates chunk q, and the P partial sums are combined by a fixed xor
// shuffle tree.  Every reduction order is therefore a function of (Q, P)
// only, which keeps results bit-reproducible.
#include "gr_internal.hpp"
#include "gr_device.hpp"

namespace gr {

constexpr int kThreads = 256;

// ------------------------------------------------------------- validation
__global__ void k_check_rowptr(const int32_t* __restrict__ rp, int64_t n, int64_t nnz,
                               int32_t* __restrict__ bad) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    int32_t x = rp[v];
    bool ok = x >= 0 && x <= nnz;
    if (v == 0) ok = ok && x == 0;
    if (v == n) ok = ok && x == nnz;
    if (v < n) ok = ok && rp[v + 1] >= x;
    if (!ok) atomicOr(bad, 1);
}

// G lanes per row (one below a mean degree of 8, else about half the mean
// degree, at most a wave): every entry is checked on its own
__global__ void k_check_entries(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ w, int64_t n, int G,
                                int32_t* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = t / G;
    if (v >= n) return;
    const int32_t e0 = rp[v], e1 = rp[v + 1];
    int flags = 0;
    for (int32_t e = e0 + (int32_t)(t % G); e < e1; e += G) {
        int32_t j = col[e];
        float wv = w[e];
        if (j < 0 || j >= n || j == v) { flags |= 2; break; }
        if (e > e0 && col[e - 1] >= j) { flags |= 4; break; }
        if (!(wv > 0.0f) || !isfinite(wv)) { flags |= 8; break; }
        // partner entry (j, v) with bit-identical weight
        int32_t lo = rp[j], hi = rp[j + 1] - 1, f = -1;
        while (lo <= hi) {
            int32_t mid = lo + ((hi - lo) >> 1);
            int32_t c = col[mid];
            if (c == (int32_t)v) { f = mid; break; }
            if (c < (int32_t)v) lo = mid + 1; else hi = mid - 1;
        }
        if (f < 0 || __float_as_uint(w[f]) != __float_as_uint(wv)) { flags |= 16; break; }
    }
    if (flags) atomicOr(bad, flags);
}

int validate_graph(const gr_graph* g, Arena& ws, hipStream_t st) {
    int32_t* bad = ws.take<int32_t>(1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (validate)");
    GR_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_rowptr, dim3(blocks_for(g->n + 1, kThreads)), dim3(kThreads), 0, st,
                       g->row_ptr, g->n, g->nnz, bad);
    GR_LAUNCHED("check row_ptr");
    int32_t hb = 0;
    GR_HIP(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    if (hb) return set_error(GR_ECSR, "row_ptr is not a monotone offset array with row_ptr[0]=0, row_ptr[n]=nnz");
    if (g->n > 0) {
        int G = g->nnz < 8 * g->n ? 1 : 4;
        while (G > 1 && G < kWave && G * 2 <= g->nnz / g->n) G *= 2;
        hipLaunchKernelGGL(k_check_entries, dim3(blocks_for(g->n * G, kThreads)), dim3(kThreads), 0,
                           st, g->row_ptr, g->col, g->w, g->n, G, bad);
        GR_LAUNCHED("check entries");
        GR_HIP(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
    }
    if (hb & 2) return set_error(GR_ECSR, "column index out of range or self-loop");
    if (hb & 4) return set_error(GR_ECSR, "columns not strictly increasing within a row");
    if (hb & 8) return set_error(GR_ECSR, "weight not positive and finite");
    if (hb & 16) return set_error(GR_ECSR, "graph not symmetric (missing or unequal reverse entry)");
    return GR_OK;
}

// -------------------------------------------------------------- colouring
// The Gauss-Seidel smoothing of Sec. 3.2.1 runs in a multicolour order; the
// colouring is sequential greedy in decreasing priority: every node takes
// the smallest colour absent among its higher-priority neighbours.
// Priority: (h(v), v), h(v) = splitmix64 output v of the colour seed, or
// (deg(v), h(v), v) largest-degree-first.

__device__ inline uint64_t wave_or(uint64_t x) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, off, kWave);
        uint32_t hi = __shfl_xor((uint32_t)(x >> 32), off, kWave);
        x |= ((uint64_t)hi << 32) | lo;
    }
    return x;
}

__device__ inline int32_t first_free4(const uint64_t used[4], int32_t base) {
    for (int w = 0; w < 4; ++w)
        if (~used[w]) return base + w * 64 + __ffsll((unsigned long long)~used[w]) - 1;
    return -1;
}

__global__ void k_col_fill(int64_t n, int32_t* __restrict__ colours) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) colours[v] = -1;
}

// ------------------------------------------------ colouring as a dataflow
// The greedy colouring computed without rounds.  The nodes are sorted once into
// decreasing priority (position = rank); every node lists the ranks of its
// higher-priority neighbours (`uplist`, from the node's row offset on).  A
// cooperative launch holds as many waves as the device keeps resident; wave
// w takes the batches of kFlowBatch consecutive positions w, w + W, ... in
// order.  A position waits until each listed neighbour has a colour
// (device-coherent polling loads), takes the first colour absent among them
// and publishes it with a device-coherent store.  A batch whose positions
// all have few listed neighbours is coloured together, kFlowG lanes per
// position, each group publishing as soon as its own inputs are there;
// otherwise the whole wave takes the batch's positions one after another.
// A node waits only on earlier positions, so the earliest uncoloured
// position is always in a batch at the head of some wave, with all its
// inputs published: no deadlock while all waves are resident, which the
// cooperative launch guarantees.  The colour
// values are the only data passed between waves, so relaxed device-scope
// atomics suffice.  Every wait is bounded: past spin_limit polls a lane
// raises the abort flag, and every waiting lane leaves at its next check.
constexpr int kFlowThreads = 256;
constexpr int kFlowWaves = kFlowThreads / kWave;
constexpr int kFlowU = 4;                      // listed neighbours in flight per lane
constexpr unsigned kFlowSpinLimit = 1u << 21;  // polls of one neighbour at most
constexpr int kFlowG = 8;                      // lanes per position of a narrow batch
constexpr int kFlowBatch = kWave / kFlowG;     // positions of a batch
constexpr int32_t kFlowNarrow = 64;            // listed neighbours per position of a narrow batch
// resident workgroups per CU of the flow: more waves take more batches at
// once where the dependence chains are short (sparse graphs: grid colour
// phase 3.5 -> 3.07 ms with 8), fewer where long chains keep most waves
// polling (power law: 3.16 ms with 2, 3.66 with 8)
#ifndef GR_FLOW_BLOCKS_PER_CU
#define GR_FLOW_BLOCKS_PER_CU 2
#endif
#ifndef GR_FLOW_BLOCKS_PER_CU_SPARSE
#define GR_FLOW_BLOCKS_PER_CU_SPARSE 8
#endif
constexpr double kFlowSparseDegree = 32.0;  // mean degree up to which a graph counts as sparse
#ifndef GR_FLOW_SLEEP
#define GR_FLOW_SLEEP 2  // s_sleep units (64 cycles) between polls
#endif

__device__ inline int32_t ld_dev(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_max_degree(const int32_t* __restrict__ rp, int64_t n, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t m = 0;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) m = max(m, rp[i + 1] - rp[i]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

// bits of the largest degree (at least 1)
__device__ inline int degree_bits(int32_t maxdeg) {
    return maxdeg > 0 ? 32 - __clz(maxdeg) : 1;
}

// 32-bit sort keys whose ascending order is decreasing priority.  mode 0:
// the top hb bits of h(v), complemented; mode 1 (largest degree first): the
// degree above the top hl = max(hb - bd, 1) bits of h(v), bd the degree's
// bit width, complemented.  h is a bijection of v, so nodes tie only on the
// truncated h, and only with nodes of their own degree: k_order_ties puts
// each run of equal keys in decreasing full h after the sort.
__global__ void k_prio_keys(const int32_t* __restrict__ rp, int64_t n, uint64_t seed, int mode,
                            int hb, const int32_t* __restrict__ maxdeg,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint64_t h = splitmix64(seed, (uint64_t)v);
    uint64_t k;
    if (mode) {
        const int bd = degree_bits(*maxdeg);
        const int hl = hb - bd > 1 ? hb - bd : 1;
        k = ((uint64_t)(rp[v + 1] - rp[v]) << hl) | (h >> (64 - hl));
    } else {
        k = h >> (64 - hb);
    }
    keys[v] = ~(uint32_t)k;
    vals[v] = (uint32_t)v;
}

// after the sort: every run of equal truncated keys (a thread at the head of
// each run) in decreasing full h(v), by insertion sort (runs are short: a
// few nodes of one degree share the top bits of h)
__global__ void k_order_ties(const uint32_t* __restrict__ keys, uint32_t* __restrict__ order,
                             int64_t n, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= n || keys[i] != keys[i + 1] || (i > 0 && keys[i - 1] == keys[i])) return;
    int64_t j = i + 2;
    while (j < n && keys[j] == keys[i]) ++j;
    for (int64_t a = i + 1; a < j; ++a) {
        const uint32_t v = order[a];
        const uint64_t hv = splitmix64(seed, v);
        int64_t b = a - 1;
        while (b >= i && splitmix64(seed, order[b]) < hv) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
}

// second key of the exact largest-degree-first order: decreasing degree
// (a stable sort on it after a sort on h alone)
__global__ void k_degree_keys(const int32_t* __restrict__ rp, const uint32_t* __restrict__ order,
                              int64_t n, uint64_t* __restrict__ keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = order[i];
    keys[i] = ~(uint64_t)(uint32_t)(rp[v + 1] - rp[v]);
}

__global__ void k_rank_of(const uint32_t* __restrict__ order, int64_t n, int32_t* __restrict__ rank) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rank[order[i]] = (int32_t)i;
}

// up-lists of the nodes of degree <= kLongRow: 8 lanes per node, in node
// order (coalesced rows); the order inside a list is irrelevant to the
// colour.  Wider nodes are listed (by position) for k_flow_count_wide.
__global__ void __launch_bounds__(kThreads) k_flow_count(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ rank, int64_t n, int32_t* __restrict__ uplist,
    int32_t* __restrict__ pstart, int32_t* __restrict__ pcnt, int32_t* __restrict__ wide,
    int32_t* __restrict__ nwide) {
    const int64_t v = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    const int lane = threadIdx.x & (kWave - 1);
    const int grp = lane >> 3;
    if (v - (lane >> 3) >= n) return;  // whole waves leave together
    const bool in = v < n;
    const int32_t e0 = in ? rp[v] : 0, e1 = in ? rp[v + 1] : 0;
    const int32_t i = in ? rank[v] : 0;
    const bool wd = in && e1 - e0 > kLongRow;
    int32_t k = 0;
    const int32_t end = wd ? e0 : e1;  // wide rows: no trips here
    for (int32_t b = e0; b < end; b += 8) {  // the same trip count for the node's lanes
        const int32_t e = b + l;
        const int32_t r = e < end ? rank[col[e]] : 0x7fffffff;
        const bool up = r < i;
        const uint32_t bits = (uint32_t)(__ballot(up) >> (8 * grp)) & 0xffu;
        if (up) uplist[e0 + k + __popc(bits & ((1u << l) - 1u))] = r;
        k += __popc(bits);
    }
    if (in && !wd && l == 0) {
        pstart[i] = e0;
        pcnt[i] = k;
    }
    // the wide nodes: one append per wave (lane 0 of each group votes)
    const bool app = wd && l == 0;
    const uint64_t m = __ballot(app);
    if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(nwide, (int32_t)__popcll(m));
        base = __shfl(base, leader, kWave);
        if (app) wide[base + (int32_t)__popcll(m & ((1ull << lane) - 1))] = i;
    }
}

// up-lists of the listed wide nodes: a wave per node, grid-stride
__global__ void __launch_bounds__(kThreads) k_flow_count_wide(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const uint32_t* __restrict__ order, const int32_t* __restrict__ rank,
    const int32_t* __restrict__ wide, const int32_t* __restrict__ nwide,
    int32_t* __restrict__ uplist, int32_t* __restrict__ pstart, int32_t* __restrict__ pcnt) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (kThreads / kWave);
    const int32_t total = *nwide;
    for (int64_t t = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kWave; t < total; t += nw) {
        const int32_t i = wide[t];
        const int32_t v = (int32_t)order[i];
        const int32_t e0 = rp[v], e1 = rp[v + 1];
        int32_t k = 0;
        for (int32_t b = e0; b < e1; b += kWave) {
            const int32_t e = b + lane;
            const int32_t r = e < e1 ? rank[col[e]] : 0x7fffffff;
            const bool up = r < i;
            const uint64_t m = __ballot(up);
            if (up) uplist[e0 + k + (int32_t)__popcll(m & ((1ull << lane) - 1))] = r;
            k += (int32_t)__popcll(m);
        }
        if (lane == 0) {
            pstart[i] = e0;
            pcnt[i] = k;
        }
    }
}

// one position with the whole wave; false when the wave must leave (abort)
__device__ inline bool flow_wide(const int32_t* __restrict__ uplist, int32_t s, int32_t m,
                                 int64_t i, int32_t* cpos, int32_t* abort_flag,
                                 unsigned spin_limit) {
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t used[4] = {0, 0, 0, 0};
    int stop = 0;
    for (int32_t b = lane; b < m && !stop; b += kWave * kFlowU) {
        int32_t u[kFlowU], c[kFlowU];
#pragma unroll
        for (int k = 0; k < kFlowU; ++k) {
            const int32_t e = b + k * kWave;
            u[k] = e < m ? uplist[s + e] : -1;
        }
#pragma unroll
        for (int k = 0; k < kFlowU; ++k) c[k] = u[k] >= 0 ? ld_dev(cpos + u[k]) : -2;
#pragma unroll
        for (int k = 0; k < kFlowU; ++k) {
            unsigned spins = 0;
            while (c[k] == -1 && !stop) {
                __builtin_amdgcn_s_sleep(GR_FLOW_SLEEP);
                c[k] = ld_dev(cpos + u[k]);
                ++spins;
                if (spins >= spin_limit) {
                    atomicExch(abort_flag, 1);
                    stop = 1;
                } else if ((spins & 255u) == 0 && ld_dev(abort_flag)) {
                    stop = 1;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kFlowU; ++k)
            if (c[k] >= 0 && c[k] < 256) used[c[k] >> 6] |= 1ull << (c[k] & 63);
    }
    if (__ballot(stop)) return false;
#pragma unroll
    for (int w = 0; w < 4; ++w) used[w] = wave_or(used[w]);
    int32_t c = first_free4(used, 0);
    // colours 0..255 all taken: later windows (every listed neighbour is
    // coloured by now); colour <= m ends the search
    for (int32_t base = 256; c < 0; base += 256) {
        uint64_t wu[4] = {0, 0, 0, 0};
        for (int32_t e = lane; e < m; e += kWave) {
            const int32_t cj = ld_dev(cpos + uplist[s + e]);
            if (cj >= base && cj < base + 256) wu[(cj - base) >> 6] |= 1ull << ((cj - base) & 63);
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) wu[w] = wave_or(wu[w]);
        c = first_free4(wu, base);
    }
    if (lane == 0) st_dev(cpos + i, c);
    return true;
}

// or over the aligned group of kFlowG lanes (every lane of the wave calls it)
__device__ inline uint64_t group_or(uint64_t x) {
#pragma unroll
    for (int off = 1; off < kFlowG; off <<= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, off, kWave);
        uint32_t hi = __shfl_xor((uint32_t)(x >> 32), off, kWave);
        x |= ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// kFlowBatch positions together, kFlowG lanes each, every position with at
// most kFlowNarrow listed neighbours (so at most kFlowNarrow / kFlowG per lane,
// all loaded at once, and a colour <= kFlowNarrow < 128).  The loop is
// wave-uniform: a group publishes as soon as its own neighbours are all
// coloured, whatever the other groups of the wave still wait for.
__device__ inline bool flow_narrow(const int32_t* __restrict__ uplist, int32_t s, int32_t m,
                                   int64_t i, bool valid, int32_t* cpos, int32_t* abort_flag,
                                   unsigned spin_limit) {
    constexpr int U = kFlowNarrow / kFlowG;
    const int gl = threadIdx.x & (kFlowG - 1);
    int32_t u[U];
    uint32_t pend = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int32_t e = gl + k * kFlowG;
        u[k] = e < m ? uplist[s + e] : 0;
        if (e < m) pend |= 1u << k;
    }
    uint64_t used0 = 0, used1 = 0;
    bool pub = !valid;
    for (unsigned it = 0;; ++it) {
#pragma unroll
        for (int k = 0; k < U; ++k)
            if ((pend >> k) & 1u) {
                const int32_t c = ld_dev(cpos + u[k]);
                if (c >= 0) {
                    if (c < 64) used0 |= 1ull << c;
                    else if (c < 128) used1 |= 1ull << (c - 64);
                    pend &= ~(1u << k);
                }
            }
        const bool waiting = group_or(pend != 0 ? 1ull : 0ull) != 0;
        const uint64_t a0 = group_or(used0), a1 = group_or(used1);
        if (!pub && !waiting) {
            const int32_t c = ~a0 ? __ffsll((unsigned long long)~a0) - 1
                                  : 64 + __ffsll((unsigned long long)~a1) - 1;
            if (gl == 0) st_dev(cpos + i, c);
            pub = true;
        }
        if (__ballot(!pub) == 0) return true;
        __builtin_amdgcn_s_sleep(GR_FLOW_SLEEP);
        if (it >= spin_limit) {
            if ((threadIdx.x & (kWave - 1)) == 0) atomicExch(abort_flag, 1);
            return false;
        }
        if ((it & 255u) == 255u && ld_dev(abort_flag)) return false;
    }
}

// batches of the dataflow: aligned groups of kFlowBatch positions; a group
// whose positions all have at most kFlowNarrow listed neighbours is one
// (narrow) batch, any other group gives a batch per position.  A batch is
// coded as its first position, with kNarrowBatch set for a narrow one.
constexpr uint32_t kNarrowBatch = 0x80000000u;

__device__ inline bool flow_group_narrow(const int32_t* __restrict__ pcnt, int64_t i0, int c) {
    bool narrow = true;
    for (int j = 0; j < c; ++j) narrow = narrow && pcnt[i0 + j] <= kFlowNarrow;
    return narrow;
}

__global__ void k_flow_group_sizes(const int32_t* __restrict__ pcnt, int64_t n,
                                   int32_t* __restrict__ nbat) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = k * kFlowBatch;
    if (i0 >= n) return;
    const int c = (int)(n - i0 < kFlowBatch ? n - i0 : kFlowBatch);
    nbat[k] = flow_group_narrow(pcnt, i0, c) ? 1 : c;
}

__global__ void k_flow_batches(const int32_t* __restrict__ pcnt, int64_t n,
                               const int32_t* __restrict__ boff, uint32_t* __restrict__ batches) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = k * kFlowBatch;
    if (i0 >= n) return;
    const int c = (int)(n - i0 < kFlowBatch ? n - i0 : kFlowBatch);
    const int32_t b = boff[k];
    if (flow_group_narrow(pcnt, i0, c)) {
        batches[b] = (uint32_t)i0 | kNarrowBatch;
    } else {
        for (int j = 0; j < c; ++j) batches[b + j] = (uint32_t)(i0 + j);
    }
}

// The first positions (the highest priorities: on power-law graphs the dense
// core of hubs, where most of the dependence chain lies) are coloured first
// by one workgroup, the same dataflow with the colours in LDS: a link of the
// chain then costs an LDS poll instead of a device-coherent publish and poll
// across the chip.  Waves take positions w, w + 16, ... in order, a whole
// wave per position; the deadlock argument of the device-wide flow holds
// inside the workgroup, and every wait is bounded the same way.
#ifndef GR_FLOW_CORE
#define GR_FLOW_CORE 1024  // positions coloured by the single workgroup
#endif
constexpr int kCoreThreads = 1024;
constexpr int kCoreWaves = kCoreThreads / kWave;
static_assert(GR_FLOW_CORE % kFlowBatch == 0, "the core ends at a batch boundary");

__device__ inline int32_t ld_lds(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// It runs only on graphs with hubs (largest degree above kCoreHubRatio times
// the mean): elsewhere the chain is short and the core would only add its
// own serial time.  first_batch receives the flow's first batch either way.
constexpr int32_t kCoreHubRatio = 16;

__global__ void __launch_bounds__(kCoreThreads) k_jp_core(const int32_t* __restrict__ pstart,
                                                          const int32_t* __restrict__ pcnt,
                                                          const int32_t* __restrict__ uplist,
                                                          int64_t n, int64_t nnz,
                                                          const int32_t* __restrict__ maxdeg,
                                                          const int32_t* __restrict__ boff,
                                                          const int32_t* __restrict__ nbatches,
                                                          int32_t* first_batch, int32_t* cpos,
                                                          int32_t* abort_flag,
                                                          unsigned spin_limit) {
    __shared__ int32_t lc[GR_FLOW_CORE];
    const bool hubs = (int64_t)*maxdeg * n > (int64_t)kCoreHubRatio * nnz;
    const int32_t kc = hubs ? (int32_t)(n < GR_FLOW_CORE ? n : GR_FLOW_CORE) : 0;
    if (threadIdx.x == 0) *first_batch = kc == 0 ? 0 : (kc < n ? boff[kc / kFlowBatch] : *nbatches);
    if (kc == 0) return;
    for (int32_t i = threadIdx.x; i < kc; i += kCoreThreads) lc[i] = -1;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    for (int32_t i = threadIdx.x / kWave; i < kc; i += kCoreWaves) {
        const int32_t s = pstart[i], m = pcnt[i];
        uint64_t used[4] = {0, 0, 0, 0};
        int stop = 0;
        for (int32_t b = lane; b < m && !stop; b += kWave * kFlowU) {
            int32_t u[kFlowU], c[kFlowU];
#pragma unroll
            for (int k = 0; k < kFlowU; ++k) {
                const int32_t e = b + k * kWave;
                u[k] = e < m ? uplist[s + e] : -1;  // ranks below i < kc
            }
#pragma unroll
            for (int k = 0; k < kFlowU; ++k) c[k] = u[k] >= 0 ? ld_lds(lc + u[k]) : -2;
#pragma unroll
            for (int k = 0; k < kFlowU; ++k) {
                unsigned spins = 0;
                while (c[k] == -1 && !stop) {
                    __builtin_amdgcn_s_sleep(1);
                    c[k] = ld_lds(lc + u[k]);
                    ++spins;
                    if (spins >= spin_limit) {
                        atomicExch(abort_flag, 1);
                        stop = 1;
                    } else if ((spins & 255u) == 0 && ld_dev(abort_flag)) {
                        stop = 1;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kFlowU; ++k)
                if (c[k] >= 0 && c[k] < 256) used[c[k] >> 6] |= 1ull << (c[k] & 63);
        }
        if (__ballot(stop)) return;  // the other waves leave at their next check
#pragma unroll
        for (int w = 0; w < 4; ++w) used[w] = wave_or(used[w]);
        int32_t c = first_free4(used, 0);
        for (int32_t base = 256; c < 0; base += 256) {  // every listed colour is known
            uint64_t wu[4] = {0, 0, 0, 0};
            for (int32_t e = lane; e < m; e += kWave) {
                const int32_t cj = ld_lds(lc + uplist[s + e]);
                if (cj >= base && cj < base + 256) wu[(cj - base) >> 6] |= 1ull << ((cj - base) & 63);
            }
#pragma unroll
            for (int w = 0; w < 4; ++w) wu[w] = wave_or(wu[w]);
            c = first_free4(wu, base);
        }
        if (lane == 0) {
            __hip_atomic_store(lc + i, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            cpos[i] = c;  // read by the device-wide flow after this launch
        }
    }
}

__global__ void __launch_bounds__(kFlowThreads) k_jp_flow(const int32_t* __restrict__ pstart,
                                                          const int32_t* __restrict__ pcnt,
                                                          const int32_t* __restrict__ uplist,
                                                          const uint32_t* __restrict__ batches,
                                                          const int32_t* __restrict__ first_batch,
                                                          const int32_t* __restrict__ nbatches,
                                                          int64_t n, int32_t* cpos,
                                                          int32_t* abort_flag,
                                                          unsigned spin_limit) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * kFlowWaves;
    const int32_t nbt = *nbatches;
    if (ld_dev(abort_flag)) return;  // the core did not finish
    for (int64_t bt = *first_batch + (int64_t)blockIdx.x * kFlowWaves + threadIdx.x / kWave;
         bt < nbt; bt += nw) {
        const uint32_t code = batches[bt];
        if (code & kNarrowBatch) {
            const int64_t ig = (int64_t)(code & ~kNarrowBatch) + lane / kFlowG;
            const bool valid = ig < n;
            const int32_t s = valid ? pstart[ig] : 0, m = valid ? pcnt[ig] : 0;
            if (!flow_narrow(uplist, s, m, ig, valid, cpos, abort_flag, spin_limit)) return;
        } else {
            const int64_t i = code;
            if (!flow_wide(uplist, pstart[i], pcnt[i], i, cpos, abort_flag, spin_limit)) return;
        }
    }
}

// colours in node order (a gather through the ranks) and the largest one:
// grid-stride, one atomic per block (same-address atomics serialise)
constexpr int kGatherBlocks = 1024;
__global__ void __launch_bounds__(kThreads) k_flow_colours(const int32_t* __restrict__ rank,
                                                           const int32_t* __restrict__ cpos,
                                                           int64_t n, int32_t* __restrict__ colours,
                                                           int32_t* mx) {
    __shared__ int32_t wm[kThreads / kWave];
    int32_t m = -1;
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kThreads) {
        const int32_t c = cpos[rank[v]];
        colours[v] = c;
        m = max(m, c);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / kWave; ++w) m = max(m, wm[w]);
        atomicMax(mx, m);
    }
}

static int flow_blocks(int64_t n, int64_t nnz) {
    int dev = 0, cus = 0, per_cu = 0;
    GR_HIP(hipGetDevice(&dev));
    GR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_jp_flow,
                                                        kFlowThreads, 0));
    const bool sparse = n > 0 && (double)nnz <= kFlowSparseDegree * (double)n;
    per_cu = std::min(per_cu, sparse ? GR_FLOW_BLOCKS_PER_CU_SPARSE : GR_FLOW_BLOCKS_PER_CU);
    if (per_cu < 1 || cus < 1) return set_error(GR_EHIP, "colouring kernel does not fit a CU");
    const int64_t want = (n + kFlowWaves - 1) / kFlowWaves;
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * cus, want));
}

static int colour_flow(const gr_graph* g, uint64_t seed, int ldf, int32_t* colours,
                       int32_t* n_colours_host, Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    *n_colours_host = 0;
    if (n == 0) return GR_OK;
    const size_t mark = ws.used;
    uint64_t* ka = ws.take<uint64_t>(n);
    uint64_t* kb = ws.take<uint64_t>(n);
    uint32_t* va = ws.take<uint32_t>(n);
    uint32_t* order = ws.take<uint32_t>(n);
    int32_t* rank = ws.take<int32_t>(n);
    int32_t* pstart = ws.take<int32_t>(n);
    int32_t* pcnt = ws.take<int32_t>(n);
    int32_t* cpos = ws.take<int32_t>(n);
    int32_t* wide = ws.take<int32_t>(n);
    int32_t* uplist = ws.take<int32_t>(nnz + 1);
    const int64_t ngroups = (n + kFlowBatch - 1) / kFlowBatch;
    int32_t* nbat = ws.take<int32_t>(ngroups);
    int32_t* boff = ws.take<int32_t>(ngroups);
    // [0] largest degree, [1] unused, [2] wide count, [3] abort flag,
    // [4] largest colour, [5] batches, [6] first batch of the device-wide flow
    int32_t* small = ws.take<int32_t>(8);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (colouring)");
    const int nblk = flow_blocks(n, nnz);
    if (nblk < 0) return nblk;
    const unsigned nb = blocks_for(n, kThreads);
    // GR_COLOUR_EXACT_ORDER=1 builds the largest-degree-first order in two
    // sorts instead (by h, then stably by degree): a second route to the
    // same order, which tests check against the reference colouring
    const char* force = getenv("GR_COLOUR_EXACT_ORDER");
    const int exact = (ldf && force && force[0] == '1') ? 1 : 0;
    // GR_COLOUR_SPIN_LIMIT=k shortens every wait to k polls (tests of the
    // timed-out path: every wave then leaves early and the call fails)
    unsigned spin_limit = kFlowSpinLimit;
    if (const char* sl = getenv("GR_COLOUR_SPIN_LIMIT")) {
        const long v = atol(sl);
        if (v > 0 && v < (long)kFlowSpinLimit) spin_limit = (unsigned)v;
    }
    // GR_COLOUR_PLAIN_LAUNCH=1 launches the flow kernel as an ordinary
    // launch of the same grid (at most the blocks the device keeps resident,
    // so on an otherwise idle device all of them run at once; if they did
    // not, the bounded waits would end the call with GR_EHIP, never hang).
    // It exists for profiling: rocprofv3 faults in its own exit handlers
    // after a cooperative launch, once its results are written.
    // width of the priority sort key (32; the variable GR_COLOUR_KEY_BITS=b,
    // 8 <= b <= 32, keeps fewer bits of h, which makes ties of the truncated
    // keys frequent, for tests of their exact order)
    int hbits = 32;
    if (const char* kb_env = getenv("GR_COLOUR_KEY_BITS")) {
        const int b = atoi(kb_env);
        if (b >= 8 && b <= 32) hbits = b;
    }
    const char* plain_env = getenv("GR_COLOUR_PLAIN_LAUNCH");
    const bool plain = plain_env && plain_env[0] == '1';
    {
        GR_HIP(hipMemsetAsync(small, 0, sizeof(int32_t) * 8, st));
        GR_HIP(hipMemsetAsync(small + 4, 0xff, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_max_degree, dim3(256), dim3(kThreads), 0, st, g->row_ptr, n, small);
        GR_LAUNCHED("colour max degree");
        // the priority order
        const int mode = (ldf && !exact) ? 1 : 0;
        // (the 32-bit keys share the buffers of the 64-bit ones)
        uint32_t* ka32 = reinterpret_cast<uint32_t*>(ka);
        uint32_t* kb32 = reinterpret_cast<uint32_t*>(kb);
        hipLaunchKernelGGL(k_prio_keys, dim3(nb), dim3(kThreads), 0, st, g->row_ptr, n, seed, mode,
                           hbits, (const int32_t*)small, ka32, va);
        GR_LAUNCHED("colour keys");
        GR_TRY(radix_sort_pairs32(ka32, va, kb32, order, n, mode ? 32 : hbits, ws, st));
        hipLaunchKernelGGL(k_order_ties, dim3(nb), dim3(kThreads), 0, st, (const uint32_t*)kb32, order,
                           n, seed);
        GR_LAUNCHED("colour key ties (exact order)");
        if (ldf && exact) {
            hipLaunchKernelGGL(k_degree_keys, dim3(nb), dim3(kThreads), 0, st, g->row_ptr,
                               (const uint32_t*)order, n, ka);
            GR_LAUNCHED("colour degree keys");
            GR_HIP(hipMemcpyAsync(va, order, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
            GR_TRY(radix_sort_pairs(ka, va, kb, order, n, 32, ws, st));
        }
        hipLaunchKernelGGL(k_rank_of, dim3(nb), dim3(kThreads), 0, st, (const uint32_t*)order, n,
                           rank);
        GR_LAUNCHED("colour ranks");
        // the higher-priority neighbours of every position
        hipLaunchKernelGGL(k_flow_count, dim3(blocks_for(n * 8, kThreads)), dim3(kThreads), 0, st,
                           g->row_ptr, g->col, (const int32_t*)rank, n, uplist, pstart, pcnt, wide,
                           small + 2);
        GR_LAUNCHED("colour up-lists");
        hipLaunchKernelGGL(k_flow_count_wide, dim3(1024), dim3(kThreads), 0, st, g->row_ptr,
                           g->col, (const uint32_t*)order, (const int32_t*)rank,
                           (const int32_t*)wide, (const int32_t*)(small + 2), uplist, pstart,
                           pcnt);
        GR_LAUNCHED("colour up-lists (wide rows)");
        // the batches (the wide list is free again: it holds them)
        const unsigned ngb = blocks_for(ngroups, kThreads);
        hipLaunchKernelGGL(k_flow_group_sizes, dim3(ngb), dim3(kThreads), 0, st,
                           (const int32_t*)pcnt, n, nbat);
        GR_LAUNCHED("colour batch sizes");
        GR_TRY(scan_exclusive_i32(nbat, boff, ngroups, small + 5, ws, st));
        uint32_t* batches = (uint32_t*)wide;
        hipLaunchKernelGGL(k_flow_batches, dim3(ngb), dim3(kThreads), 0, st, (const int32_t*)pcnt,
                           n, (const int32_t*)boff, batches);
        GR_LAUNCHED("colour batches");
        hipLaunchKernelGGL(k_col_fill, dim3(nb), dim3(kThreads), 0, st, n, cpos);
        GR_LAUNCHED("colour fill");
        // on graphs with hubs the first positions in one workgroup; the flow
        // then starts at the batch the core kernel leaves in small[6]
        hipLaunchKernelGGL(k_jp_core, dim3(1), dim3(kCoreThreads), 0, st, (const int32_t*)pstart,
                           (const int32_t*)pcnt, (const int32_t*)uplist, n, nnz,
                           (const int32_t*)small, (const int32_t*)boff,
                           (const int32_t*)(small + 5), small + 6, cpos, small + 3, spin_limit);
        GR_LAUNCHED("colour core");
        const int32_t* fb = small + 6;
        const int32_t* ps = pstart;
        const int32_t* pc = pcnt;
        const int32_t* ul = uplist;
        const uint32_t* bl = batches;
        const int32_t* nbt = small + 5;
        int32_t* abort_flag = small + 3;
        int64_t nn = n;
        void* args[] = {(void*)&ps, (void*)&pc, (void*)&ul, (void*)&bl, (void*)&fb, (void*)&nbt,
                        (void*)&nn, (void*)&cpos, (void*)&abort_flag, (void*)&spin_limit};
        if (plain)
            GR_HIP(hipLaunchKernel((const void*)k_jp_flow, dim3(nblk), dim3(kFlowThreads), args, 0,
                                   st));
        else
            GR_HIP(hipLaunchCooperativeKernel((const void*)k_jp_flow, dim3(nblk),
                                              dim3(kFlowThreads), args, 0, st));
        hipLaunchKernelGGL(k_flow_colours, dim3(std::min<unsigned>(nb, kGatherBlocks)),
                           dim3(kThreads), 0, st, (const int32_t*)rank, (const int32_t*)cpos, n,
                           colours, small + 4);
        GR_LAUNCHED("colour gather");
        int32_t hs[8];
        GR_HIP(hipMemcpyAsync(hs, small, sizeof(hs), hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
        if (hs[3]) return set_error(GR_EHIP, "colouring wait timed out");
        if (hs[4] < 0) return set_error(GR_EHIP, "colouring left nodes uncoloured");
        *n_colours_host = hs[4] + 1;
    }
    ws.used = mark;
    return GR_OK;
}

int colour_greedy(const gr_graph* g, uint64_t seed, int ldf, int32_t* colours,
                  int32_t* n_colours_host, Arena& ws, hipStream_t st) {
    return colour_flow(g, seed, ldf, colours, n_colours_host, ws, st);
}

// G lanes per row (a power of two up to a wave, from the mean degree)
__global__ void k_check_colouring(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  const int32_t* __restrict__ colours, int64_t n, int32_t nc,
                                  int G, int32_t* bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = t / G;
    const int lane = (int)(t % G);
    if (v >= n) return;
    const int32_t c = colours[v];
    int f = 0;
    if (c < 0 || c >= nc) f = 1;
    else
        for (int32_t e = rp[v] + lane; e < rp[v + 1]; e += G)
            if (colours[col[e]] == c) { f = 2; break; }
    if (f) atomicOr(bad, f);
}

int validate_colouring(const gr_graph* g, const int32_t* colours, int32_t n_colours, Arena& ws,
                       hipStream_t st) {
    if (g->n == 0) return GR_OK;
    size_t mark = ws.used;
    int32_t* bad = ws.take<int32_t>(1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small");
    GR_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    // one lane per row below a mean degree of 8, else about half the mean degree
    int G = g->nnz < 8 * g->n ? 1 : 4;
    while (G > 1 && G < kWave && G * 2 <= g->nnz / g->n) G *= 2;
    hipLaunchKernelGGL(k_check_colouring, dim3(blocks_for(g->n * G, kThreads)), dim3(kThreads), 0, st,
                       g->row_ptr, g->col, colours, g->n, n_colours, G, bad);
    GR_LAUNCHED("check colouring");
    int32_t hb = 0;
    GR_HIP(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    ws.used = mark;
    if (hb & 1) return set_error(GR_ECOLOUR, "colour out of range [0, %d)", n_colours);
    if (hb & 2) return set_error(GR_ECOLOUR, "an edge joins two nodes of one colour");
    return GR_OK;
}

// ------------------------------------------------------- colour-major order
// Rows are relabelled by the key (colour, degree tier, old id): the rows of
// one colour become a contiguous range, in decreasing degree tiers, so that
// one smoothing launch can give every tier its own lanes-per-row.
__global__ void k_bucket_keys(const int32_t* __restrict__ rp, const int32_t* __restrict__ colours,
                              int64_t n, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t deg = rp[v + 1] - rp[v];
    uint32_t b = (uint32_t)colours[v] * kNT + (uint32_t)degree_tier(deg);
    keys[v] = b;
    vals[v] = (uint32_t)v;
}

// first and one-past-last row of every bucket present in the sorted keys
__global__ void k_bucket_bounds(const uint32_t* __restrict__ keys, int64_t n,
                                int32_t* __restrict__ bfirst, int32_t* __restrict__ bend) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) bfirst[k] = (int32_t)i;
    if (i == n - 1 || keys[i + 1] != k) bend[k] = (int32_t)(i + 1);
}

__global__ void k_perm_degrees(const int32_t* __restrict__ rp, const uint32_t* __restrict__ perm,
                               int64_t n, int32_t* __restrict__ iperm, int32_t* __restrict__ deg) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t v = (int32_t)perm[r];
    iperm[v] = (int32_t)r;
    deg[r] = rp[v + 1] - rp[v];
}

// G lanes per old row (G a power of two sized to the mean degree), in old
// order so that the old CSR streams in: copy the row's entries, columns
// relabelled, to its new row (each new row is written contiguously)
__global__ void k_perm_entries(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const float* __restrict__ w, const int32_t* __restrict__ iperm,
                               const int32_t* __restrict__ nrp, int64_t n, int G,
                               int32_t* __restrict__ ncol, float* __restrict__ nw) {
    const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int l = threadIdx.x % G;
    if (v >= n) return;
    const int32_t e0 = rp[v], e1 = rp[v + 1], o = nrp[iperm[v]];
    int32_t e = e0 + l;
    for (; e + 3 * G < e1; e += 4 * G) {  // four entries in flight per lane (hub rows)
        int32_t c[4];
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = iperm[col[e + u * G]];
            x[u] = w[e + u * G];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ncol[o + (e + u * G - e0)] = c[u];
            nw[o + (e + u * G - e0)] = x[u];
        }
    }
    for (; e < e1; e += G) {
        ncol[o + (e - e0)] = iperm[col[e]];
        nw[o + (e - e0)] = w[e];
    }
}

// per bucket: rows, and stored entries (from the relabelled row pointers)
__global__ void k_bucket_sizes(const int32_t* __restrict__ bfirst, const int32_t* __restrict__ bend,
                               const int32_t* __restrict__ nrp, int32_t nb,
                               int64_t* __restrict__ out) {
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int32_t f = bfirst[b], e = bend[b];
    out[2 * b] = f >= 0 ? (int64_t)(e - f) : 0;
    out[2 * b + 1] = f >= 0 ? (int64_t)(nrp[e] - nrp[f]) : 0;
}

// ids of the long rows, class by class: class c contributes the rows
// [cls[2c], cls[2c] + cls[2c+1]) at offset off[c]
__global__ void k_long_rows(const int64_t* __restrict__ cls, const int32_t* __restrict__ off,
                            int32_t n_colours, int32_t* __restrict__ out) {
    int32_t c = blockIdx.y;
    if (c >= n_colours) return;
    const int64_t first = cls[2 * c], cnt = cls[2 * c + 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x)
        out[off[c] + i] = (int32_t)(first + i);
}

int order_by_colour(const gr_graph* g, const int32_t* colours, int32_t n_colours, OrderedGraph* og,
                    Arena& ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    og->n_colours = n_colours;
    og->perm = ws.take<int32_t>(n);
    og->iperm = ws.take<int32_t>(n);
    int32_t* nrp = ws.take<int32_t>(n + 1);
    int32_t* ncol = ws.take<int32_t>(nnz);
    float* nw = ws.take<float>(nnz);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (relabel)");
    size_t mark = ws.used;
    const int32_t nb = kNT * n_colours;
    uint32_t* k0 = ws.take<uint32_t>(n);
    uint32_t* v0 = ws.take<uint32_t>(n);
    uint32_t* k1 = ws.take<uint32_t>(n);
    int32_t* bfirst = ws.take<int32_t>(nb + 1);
    int32_t* bend = ws.take<int32_t>(nb + 1);
    int64_t* sizes = ws.take<int64_t>(2 * (int64_t)nb + 2);
    int32_t* deg = ws.take<int32_t>(n + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (relabel)");
    GR_TRY(fill_i32(bfirst, -1, nb + 1, st));
    GR_TRY(fill_i32(bend, -1, nb + 1, st));
    if (n > 0) {
        hipLaunchKernelGGL(k_bucket_keys, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st,
                           g->row_ptr, colours, n, k0, v0);
        GR_LAUNCHED("bucket keys");
    }
    GR_TRY(radix_sort_pairs32(k0, v0, k1, (uint32_t*)og->perm, n, bits_for(nb), ws, st));
    if (n > 0) {
        hipLaunchKernelGGL(k_bucket_bounds, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st,
                           (const uint32_t*)k1, n, bfirst, bend);
        GR_LAUNCHED("bucket bounds");
        hipLaunchKernelGGL(k_perm_degrees, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st,
                           g->row_ptr, (const uint32_t*)og->perm, n, og->iperm, deg);
        GR_LAUNCHED("perm degrees");
    }
    GR_TRY(scan_exclusive_i32(deg, nrp, n, nrp + n, ws, st));
    if (n > 0) {
        int G = 4;
        while (G < kWave && G * 2 <= nnz / n) G *= 2;  // about half the mean degree
        hipLaunchKernelGGL(k_perm_entries, dim3(blocks_for(n * G, kThreads)), dim3(kThreads), 0,
                           st, g->row_ptr, g->col, g->w, og->iperm, nrp, n, G, ncol, nw);
        GR_LAUNCHED("perm entries");
    }
    // bucket sizes (rows, entries) on the host
    std::vector<int64_t> hs(2 * (size_t)nb);
    if (nb > 0) {
        hipLaunchKernelGGL(k_bucket_sizes, dim3(blocks_for(nb, kThreads)), dim3(kThreads), 0, st,
                           bfirst, bend, nrp, nb, sizes);
        GR_LAUNCHED("bucket sizes");
        GR_HIP(hipMemcpyAsync(hs.data(), sizes, sizeof(int64_t) * 2 * nb, hipMemcpyDeviceToHost, st));
        GR_HIP(hipStreamSynchronize(st));
    }
    og->class_ptr_h.assign((size_t)n_colours + 1, 0);
    og->tier_ptr_h.assign((size_t)nb + 1, 0);
    og->long_end_h.assign((size_t)n_colours, 0);
    og->class_nnz_h.assign((size_t)n_colours, 0);
    og->class_e_h.assign((size_t)n_colours + 1, 0);
    og->long_nnz_h.assign((size_t)n_colours, 0);
    std::vector<int64_t> cls(2 * (size_t)n_colours + 2, 0);
    std::vector<int32_t> long_off(n_colours + 1, 0);
    int64_t total = 0, nlong = 0;
    for (int c = 0; c < n_colours; ++c) {
        og->class_ptr_h[c] = total;
        int64_t nz = 0, lr = 0, lz = 0;
        for (int t = 0; t < kNT; ++t) {
            const int b = c * kNT + t;
            og->tier_ptr_h[b] = total;
            total += hs[2 * b];
            nz += hs[2 * b + 1];
            if (t < kLongTiers) {
                lr += hs[2 * b];
                lz += hs[2 * b + 1];
            }
        }
        og->class_nnz_h[c] = nz;
        og->class_e_h[c + 1] = og->class_e_h[c] + nz;
        og->long_nnz_h[c] = lz;
        og->long_end_h[c] = og->class_ptr_h[c] + lr;
        cls[2 * c] = og->class_ptr_h[c];
        cls[2 * c + 1] = lr;
        long_off[c] = (int32_t)nlong;
        nlong += lr;
    }
    long_off[n_colours] = (int32_t)nlong;
    og->class_ptr_h[n_colours] = total;
    og->tier_ptr_h[nb] = total;
    if (total != n) return set_error(GR_ECOLOUR, "colouring does not cover every node");
    ws.used = mark;
    // device list of the long rows (relabelled ids), class by class; it
    // stays at the front of the region released above
    og->n_long = nlong;
    og->long_rows = nullptr;
    if (nlong > 0) {
        og->long_rows = ws.take<int32_t>(nlong);
        const size_t keep = ws.used;
        int32_t* loff = ws.take<int32_t>(n_colours + 1);
        int64_t* dcls = ws.take<int64_t>(2 * (size_t)n_colours + 2);
        if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (long rows)");
        GR_HIP(hipMemcpyAsync(loff, long_off.data(), sizeof(int32_t) * (n_colours + 1),
                              hipMemcpyHostToDevice, st));
        GR_HIP(hipMemcpyAsync(dcls, cls.data(), sizeof(int64_t) * 2 * n_colours,
                              hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_long_rows, dim3(8, n_colours), dim3(kThreads), 0, st,
                           (const int64_t*)dcls, (const int32_t*)loff, n_colours, og->long_rows);
        GR_LAUNCHED("long rows");
        // the host vectors and the small tables are released below
        GR_HIP(hipStreamSynchronize(st));
        ws.used = keep;
    }
    og->g.n = n;
    og->g.nnz = nnz;
    og->g.row_ptr = nrp;
    og->g.col = ncol;
    og->g.w = nw;
    og->mean_deg = n > 0 ? (double)nnz / (double)n : 0.0;
    return GR_OK;
}

// ------------------------------------------------------------ row moves
__global__ void k_permute_rows(const uint4* __restrict__ src, uint4* __restrict__ dst,
                               const int32_t* __restrict__ perm, int64_t n, int64_t q, int inverse) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * q) return;
    int64_t r = i / q, c = i - r * q;
    int64_t o = perm[r];
    if (inverse) dst[o * q + c] = src[r * q + c];
    else dst[r * q + c] = src[o * q + c];
}

int permute_rows(const void* src, void* dst, const int32_t* perm, int64_t n, size_t row_bytes,
                 int inverse, hipStream_t st) {
    if (n == 0) return GR_OK;
    int64_t q = (int64_t)(row_bytes / 16);
    hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for(n * q, kThreads)), dim3(kThreads), 0, st,
                       (const uint4*)src, (uint4*)dst, perm, n, q, inverse);
    GR_LAUNCHED("permute rows");
    return GR_OK;
}

// ------------------------------------------------------------ test vectors
// Entry (v, k) of the raw vectors: t = 2m + 1 - 2^24 for m the top 24 bits of
// splitmix64 output id(v) * K + k, the value being t / 2^24.  The counter
// of splitmix64 advances by a fixed odd constant per output, so the E
// consecutive entries of a 16-byte chunk start from one product and add the
// constant; only the top 24 bits of the last multiplication are used.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

template <int E>
__device__ inline void rand_chunk(uint64_t seed, uint64_t first, int32_t* t) {
    uint64_t z = seed + (first + 1ull) * kGolden;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uint64_t y = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        y = (y ^ (y >> 27)) * 0x94D049BB133111EBull;
        // the final y ^ (y >> 31) leaves the top 24 bits as they are
        const int32_t m = (int32_t)(y >> 40);
        t[e] = 2 * m + 1 - (1 << 24);
        z += kGolden;
    }
}

constexpr int kInitBlocks = 2048;  // at most; a multiple of K / 4 in use
constexpr int kInitE = 4;  // entries per chunk in the column sums (K % 4 == 0)

// Column sums of the raw vectors.  Thread g takes the chunks g, g + G, ... of
// the n * K / 4 chunks (G a multiple of K / 4, so a thread keeps one chunk
// column q); the sums are of multiples of 2^-24 below n in magnitude, exact
// in FP64 for n < 2^29, so their order does not matter.  part[k * B + b]:
// block b's sum of column k.
__global__ void __launch_bounds__(kThreads) k_init_colsum(int64_t n, int32_t K, uint64_t seed,
                                                          const int32_t* __restrict__ ids,
                                                          double* __restrict__ part) {
    __shared__ double red[kThreads][kInitE];
    const int Qc = K / kInitE;
    const int tid = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * kThreads + tid;
    const int64_t G = (int64_t)gridDim.x * kThreads;
    const int q = (int)(g % Qc);
    double acc[kInitE];
#pragma unroll
    for (int e = 0; e < kInitE; ++e) acc[e] = 0.0;
    const int64_t items = n * Qc;
    const bool narrow = items <= 0xffffffffll;
    for (int64_t i = g; i < items; i += G) {
        const int64_t r = narrow ? (int64_t)((uint32_t)i / (uint32_t)Qc) : i / Qc;
        const int64_t id = ids ? ids[r] : r;
        int32_t t[kInitE];
        rand_chunk<kInitE>(seed, (uint64_t)id * (uint64_t)K + (uint64_t)(q * kInitE), t);
#pragma unroll
        for (int e = 0; e < kInitE; ++e) acc[e] += (double)t[e];
    }
#pragma unroll
    for (int e = 0; e < kInitE; ++e) red[tid][e] = acc[e];
    __syncthreads();
    // column k = q * 4 + e: the threads of chunk column q (tid = q mod Qc,
    // the block's first thread being of column blockIdx.x * kThreads mod Qc)
    for (int k = tid; k < K; k += kThreads) {
        const int qq = k / kInitE, e = k % kInitE;
        const int t0 = (int)(((int64_t)qq - (int64_t)blockIdx.x * kThreads) % Qc + Qc) % Qc;
        double sum = 0.0;
        for (int u = t0; u < kThreads; u += Qc) sum += red[u][e];
        part[(int64_t)k * gridDim.x + blockIdx.x] = sum * (1.0 / 16777216.0);
    }
}

// a block per column: the sum of its nb partial sums (exact, see above)
__global__ void __launch_bounds__(kThreads) k_init_mean(const double* __restrict__ part, int nb,
                                                        int64_t n, double* __restrict__ mean) {
    __shared__ double ws[kThreads / kWave];
    const int k = blockIdx.x;
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) t += part[(int64_t)k * nb + b];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) u += ws[w];
        mean[k] = u / (double)n;
    }
}

// one 16-byte chunk (4 float32 or 8 bfloat16 values) per thread, stored
// with one vector store: (value - column mean) in FP64, rounded once
template <int DT>
__global__ void k_init_write(int64_t n, int32_t K, uint64_t seed, const int32_t* __restrict__ ids,
                             const double* __restrict__ mean, void* __restrict__ X) {
    constexpr int E = Chunk<DT>::E;
    const int32_t Qc = K / E;  // chunks per row
    const int64_t total = n * Qc;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    int64_t r;
    if (total <= 0xffffffffll) r = (int64_t)((uint32_t)c / (uint32_t)Qc);
    else r = c / Qc;
    const int q = (int)(c - r * Qc);
    const int64_t id = ids ? ids[r] : r;
    int32_t t[E];
    rand_chunk<E>(seed, (uint64_t)id * (uint64_t)K + (uint64_t)(q * E), t);
    float v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = (float)((double)t[e] * (1.0 / 16777216.0) - mean[q * E + e]);
    Chunk<DT>::store(X, r, K, q, v);
}

int init_vectors(int64_t n, int32_t K, uint64_t seed, int32_t dtype, const int32_t* ids, void* X,
                 Arena& ws, hipStream_t st) {
    if (n == 0) return GR_OK;
    size_t mark = ws.used;
    double* part = ws.take<double>((size_t)(kInitBlocks + 64) * K);
    double* mean = ws.take<double>(K);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (init)");
    if (K % kInitE != 0) return set_error(GR_EUNSUP, "K=%d is not a multiple of 4", K);
    // a multiple of K / 4 blocks, so that every thread keeps one chunk column
    const int Qc = K / kInitE;
    const int64_t want = std::min<int64_t>(kInitBlocks, blocks_for(n * Qc, kThreads));
    const int nbk = (int)std::max<int64_t>(Qc, want / Qc * Qc);
    hipLaunchKernelGGL(k_init_colsum, dim3(nbk), dim3(kThreads), 0, st, n, K, seed, ids, part);
    GR_LAUNCHED("init colsum");
    hipLaunchKernelGGL(k_init_mean, dim3(K), dim3(kThreads), 0, st, (const double*)part, nbk, n,
                       mean);
    GR_LAUNCHED("init mean");
    const int E = dtype == GR_BF16 ? Chunk<GR_BF16>::E : Chunk<GR_F32>::E;
    if (K % E != 0) return set_error(GR_EUNSUP, "K=%d is not a whole number of 16-byte chunks", K);
    const unsigned wb = blocks_for(n * (K / E), kThreads);
    if (dtype == GR_BF16)
        hipLaunchKernelGGL(k_init_write<GR_BF16>, dim3(wb), dim3(kThreads), 0, st, n, K, seed, ids,
                           (const double*)mean, X);
    else
        hipLaunchKernelGGL(k_init_write<GR_F32>, dim3(wb), dim3(kThreads), 0, st, n, K, seed, ids,
                           (const double*)mean, X);
    GR_LAUNCHED("init write");
    ws.used = mark;
    return GR_OK;
}

// ----------------------------------------------------------- GS colour step
// One Gauss-Seidel colour step (Sec. 3.2.1): every node v of the colour with
// d_v > 0 becomes sum_j w_vj x_j / d_v.  One launch of kBig-thread blocks
// per step.  The rows of the colour come in degree tiers; tier t gets L_t
// lanes per row (a power of two from Q to kBig, about half the tier's
// largest degree times Q / kU, so that a row takes about two rounds of kU
// gathers per lane whatever its degree) and its own range of blocks, each
// block holding kBig / L_t rows.  Lane l of a row owns the 16-byte chunk
// l % Q of the vector rows and the neighbour slots l / Q, + L/Q, ...; the
// partial sums are combined by a fixed shuffle tree inside the wave and,
// for rows wider than a wave, across its waves in LDS.
constexpr int kU = 4;
// threads of a smoothing block (measured: 512 beats 1024 by 0.5 ms per
// reduction on the power-law graph; 256 loses 1.1 ms)
#ifndef GR_GS_BLOCK
#define GR_GS_BLOCK 512
#endif
constexpr int kBig = GR_GS_BLOCK;

// Rows of degree above 2048 (tier 0) are split: kSplit blocks each take a
// contiguous 1/kSplit of the row's entries and write a partial sum (K values
// and the weight sum) to `part`, release it to the device and count itself
// in the row's counter; the block that arrives last adds the kSplit partials
// in piece order, stores the row and clears the counter for the next use.
constexpr int kSplit = 8;

struct GsTiers {
    int32_t nt;                 // tiers present in this colour
    int32_t split;              // tier index 0 is the split tier 0
    int32_t lanes[kNT];         // lanes per row
    int64_t row0[kNT + 1];      // first row of each tier (and the end)
    int64_t blk0[kNT + 1];      // first block of each tier (and the total)
    int32_t reverse;            // blocks from blk0[split] on run in reverse order
};

template <int Q, int DT>
__device__ inline void gs_block(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ w, void* __restrict__ X, int32_t K,
                                const GsTiers& tt, int64_t b, float* __restrict__ part,
                                int32_t* __restrict__ splitcnt, float (*sacc)[Q][Chunk<DT>::E],
                                float* sd) {
    constexpr int E = Chunk<DT>::E;
    int t = 0;
    while (t + 1 < tt.nt && b >= tt.blk0[t + 1]) ++t;
    const int L = tt.lanes[t];
    const int P = L / Q;
    const int tid = threadIdx.x;
    const int l = tid % L;
    const int p = l / Q, q = l % Q;
    const bool split = tt.split && t == 0;  // block-uniform
    int64_t r, slot = 0;
    if (split) {
        r = tt.row0[0] + (b - tt.blk0[0]) / kSplit;
        slot = b - tt.blk0[0];  // (row in the tier) * kSplit + piece
    } else {
        r = tt.row0[t] + (b - tt.blk0[t]) * (kBig / L) + tid / L;
    }
    const bool valid = r < tt.row0[t + 1];
    int32_t e0 = 0, e1 = 0;
    if (valid) {
        e0 = rp[r];
        e1 = rp[r + 1];
        if (split) {
            const int32_t f = (int32_t)(slot % kSplit);
            const int32_t len = (e1 - e0 + kSplit - 1) / kSplit;
            e1 = min(e1, e0 + (f + 1) * len);
            e0 = min(e1, e0 + f * len);
        }
    }
    float acc[E];
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = 0.0f;
    float d = 0.0f;
    for (int32_t e = e0 + p; e < e1; e += kU * P) {
        int32_t j[kU];
        float wt[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int32_t eu = e + u * P;
            bool ok = eu < e1;
            j[u] = ok ? col[eu] : (int32_t)r;   // out of range: weight 0, own row
            wt[u] = ok ? w[eu] : 0.0f;
        }
        float x[kU][E];
#pragma unroll
        for (int u = 0; u < kU; ++u) Chunk<DT>::load(X, j[u], K, q, x[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
#pragma unroll
            for (int i = 0; i < E; ++i) acc[i] = __fmaf_rn(wt[u], x[u][i], acc[i]);
            d += wt[u];
        }
    }
    // combine the slots of the row inside the wave
    const int span = L < kWave ? L : kWave;
    for (int off = Q; off < span; off <<= 1) {
#pragma unroll
        for (int i = 0; i < E; ++i) acc[i] += __shfl_xor(acc[i], off, kWave);
        d += __shfl_xor(d, off, kWave);
    }
    if (L > kWave) {
        // rows wider than a wave: the waves of the row meet in LDS
        const int wid = tid / kWave, lane = tid & (kWave - 1);
        if (lane < Q) {
#pragma unroll
            for (int i = 0; i < E; ++i) sacc[wid][lane][i] = acc[i];
            if (lane == 0) sd[wid] = d;
        }
        __syncthreads();
        if (l < Q && valid) {
            const int w0 = (tid - l) / kWave, nw = L / kWave;
            float y[E];
            float dd = 0.0f;
#pragma unroll
            for (int i = 0; i < E; ++i) y[i] = 0.0f;
            for (int ww = w0; ww < w0 + nw; ++ww) {
#pragma unroll
                for (int i = 0; i < E; ++i) y[i] += sacc[ww][l][i];
                dd += sd[ww];
            }
            if (split) {
                float* pp = part + slot * (int64_t)(K + 1);
#pragma unroll
                for (int i = 0; i < E; ++i) pp[l * E + i] = y[i];
                if (l == 0) pp[K] = dd;
            } else if (dd > 0.0f) {
#pragma unroll
                for (int i = 0; i < E; ++i) y[i] = y[i] / dd;
                Chunk<DT>::store(X, r, K, l, y);
            }
        }
        if (split && tid < kWave) {
            // wave 0 wrote the partial: release it, count the piece; the
            // last piece of the row combines all of them
            const int64_t row = slot / kSplit;
            __threadfence();
            int last = 0;
            if (tid == 0) last = atomicAdd(splitcnt + row, 1) == kSplit - 1;
            last = __shfl(last, 0, kWave);
            if (last) {
                __threadfence();
                // lane (f0, q) adds partials f0, f0 + F, ... of chunk q; a
                // fixed xor tree over f0 combines them
                constexpr int F = kWave / Q < kSplit ? kWave / Q : kSplit;
                const int f0 = tid / Q, qq = tid % Q;
                float y[E];
                float dd = 0.0f;
#pragma unroll
                for (int i = 0; i < E; ++i) y[i] = 0.0f;
                if (f0 < F) {
#pragma unroll
                    for (int j = 0; j < kSplit / F; ++j) {
                        const float* pp = part + (row * kSplit + f0 + j * F) * (int64_t)(K + 1);
#pragma unroll
                        for (int i = 0; i < E; ++i) y[i] += pp[qq * E + i];
                        dd += pp[K];
                    }
                }
#pragma unroll
                for (int off = Q; off < Q * F; off <<= 1) {
#pragma unroll
                    for (int i = 0; i < E; ++i) y[i] += __shfl_xor(y[i], off, kWave);
                    dd += __shfl_xor(dd, off, kWave);
                }
                if (f0 == 0 && dd > 0.0f) {
#pragma unroll
                    for (int i = 0; i < E; ++i) y[i] = y[i] / dd;
                    Chunk<DT>::store(X, r, K, qq, y);
                }
                if (tid == 0) splitcnt[row] = 0;
            }
        }
        __syncthreads();  // the LDS slots are reused by the block's next rows
    } else if (p == 0 && valid && d > 0.0f) {
        float y[E];
#pragma unroll
        for (int i = 0; i < E; ++i) y[i] = acc[i] / d;
        Chunk<DT>::store(X, r, K, q, y);
    }
}

template <int Q, int DT>
__global__ void __launch_bounds__(kBig) k_gs_step(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const float* __restrict__ w,
                                                  void* __restrict__ X, int32_t K, GsTiers tt,
                                                  float* __restrict__ part,
                                                  int32_t* __restrict__ splitcnt) {
    __shared__ float sacc[kBig / kWave][Q][Chunk<DT>::E];
    __shared__ float sd[kBig / kWave];
    int64_t b = blockIdx.x;
    const int64_t b0 = tt.blk0[tt.split], nb = tt.blk0[tt.nt];
    if (tt.reverse && b >= b0) b = b0 + (nb - 1 - b);
    gs_block<Q, DT>(rp, col, w, X, K, tt, b, part, splitcnt, sacc, sd);
}

// lanes per row of tier t: about half the tier's largest degree times
// Q / kU (two rounds of kU gathers per lane), a power of two in [Q, kBig]
static int tier_lanes(int Q, int t) {
    const int64_t dmax = t == 0 ? 4096 : tier_max_degree(t);
    const int64_t want = (dmax * Q + 2 * kU - 1) / (2 * kU);
    int L = Q;
    while (L < want && L < kBig) L *= 2;
    return L;
}

static GsTiers plan_gs_step(const OrderedGraph* og, int Q, int c) {
    GsTiers tt{};
    int64_t blocks = 0;
    for (int t = 0; t < kNT; ++t) {
        const int64_t r0 = og->tier_ptr_h[(size_t)c * kNT + t];
        const int64_t r1 = og->tier_ptr_h[(size_t)c * kNT + t + 1];
        if (r1 == r0) continue;
        const int L = tier_lanes(Q, t);
        const int k = tt.nt++;
        tt.lanes[k] = L;
        tt.row0[k] = r0;
        tt.row0[k + 1] = r1;
        tt.blk0[k] = blocks;
        if (t == 0 && L == kBig) {
            tt.split = 1;  // k == 0 here: tier 0 comes first
            blocks += (r1 - r0) * kSplit;
        } else {
            blocks += ((r1 - r0) * L + kBig - 1) / kBig;
        }
        tt.blk0[k + 1] = blocks;
    }
    return tt;
}

template <int Q, int DT>
static int smooth_q(const OrderedGraph* og, int K, int sweeps, void* X, Arena& ws,
                    hipStream_t st) {
    const bool pr = prof::on();
    const int xs = DT == GR_BF16 ? 2 : 4;
    const int C = og->n_colours;
    std::vector<GsTiers> plan(C);
    int steps = 0;
    double sweep_bytes = 0.0;  // compulsory bytes of one sweep (see below)
    for (int c = 0; c < C; ++c) {
        plan[c] = plan_gs_step(og, Q, c);
        if (plan[c].nt == 0) continue;
        ++steps;
        // a colour step's CSR rows, plus one read and one write of each
        // updated vector row
        const double rows = (double)(og->class_ptr_h[c + 1] - og->class_ptr_h[c]);
        sweep_bytes += 4.0 * (rows + 1) + 8.0 * (double)og->class_nnz_h[c] + 2.0 * rows * K * xs;
    }
    if (steps == 0) return GR_OK;
    int64_t split_rows = 0;
    for (int c = 0; c < C; ++c)
        if (plan[c].split) split_rows = std::max<int64_t>(split_rows, plan[c].row0[1] - plan[c].row0[0]);
    const size_t mark = ws.used;
    float* part = ws.take<float>((size_t)std::max<int64_t>(split_rows, 1) * kSplit * (K + 1));
    int32_t* splitcnt = ws.take<int32_t>((size_t)std::max<int64_t>(split_rows, 1));
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (smoothing partials)");
    if (split_rows > 0) GR_TRY(fill_i32(splitcnt, 0, split_rows, st));
    // the profiler brackets all steps of the level at once (events between
    // the launches would stall the launch queue)
    if (pr) prof::begin(st);
    // where the vectors exceed half the Infinity Cache, every other step runs
    // its blocks in reverse, so that it starts on the rows whose neighbours
    // the step before touched last (still on chip; grid smoothing 13.4 ->
    // 13.25 ms per reduction; on smaller vectors, which stay on chip, it
    // only moved the widest tiers to the back).  GR_GS_ALTERNATE=0 / 1
    // turns it off / on at any size, for comparison and tests.
    const char* alt_env = getenv("GR_GS_ALTERNATE");
    const bool alternate = alt_env ? alt_env[0] == '1'
                                   : (double)og->g.n * K * xs > 128.0 * 1024 * 1024;
    int64_t launched = 0;
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < C; ++c) {
            GsTiers tt = plan[c];
            if (tt.nt == 0) continue;
            tt.reverse = alternate ? (int32_t)(launched & 1) : 0;
            ++launched;
            hipLaunchKernelGGL((k_gs_step<Q, DT>), dim3((unsigned)tt.blk0[tt.nt]), dim3(kBig), 0, st,
                               og->g.row_ptr, og->g.col, og->g.w, X, K, tt, part, splitcnt);
            GR_LAUNCHED("gs step");
        }
    if (pr) prof::end(st, prof::SMOOTH, sweep_bytes * sweeps, (int64_t)steps * sweeps);
    ws.used = mark;
    return GR_OK;
}

int smooth_ordered(const OrderedGraph* og, int32_t K, int32_t sweeps, int32_t dtype, void* X,
                   Arena& ws, hipStream_t st) {
    if (og->g.n == 0 || sweeps == 0) return GR_OK;
    int bytes = K * (dtype == GR_BF16 ? 2 : 4);
    int Q = bytes / 16;
    if (dtype == GR_BF16) {
        switch (Q) {
            case 1: return smooth_q<1, GR_BF16>(og, K, sweeps, X, ws, st);
            case 2: return smooth_q<2, GR_BF16>(og, K, sweeps, X, ws, st);
            case 4: return smooth_q<4, GR_BF16>(og, K, sweeps, X, ws, st);
            case 8: return smooth_q<8, GR_BF16>(og, K, sweeps, X, ws, st);
        }
    } else {
        switch (Q) {
            case 1: return smooth_q<1, GR_F32>(og, K, sweeps, X, ws, st);
            case 2: return smooth_q<2, GR_F32>(og, K, sweeps, X, ws, st);
            case 4: return smooth_q<4, GR_F32>(og, K, sweeps, X, ws, st);
            case 8: return smooth_q<8, GR_F32>(og, K, sweeps, X, ws, st);
            case 16: return smooth_q<16, GR_F32>(og, K, sweeps, X, ws, st);
        }
    }
    return set_error(GR_EUNSUP, "unsupported K=%d for this dtype", K);
}

}  // namespace gr
