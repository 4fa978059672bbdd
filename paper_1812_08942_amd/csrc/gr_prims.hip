// Deterministic device primitives for libgraphreduce: error state, prefix
// sums, a stable LSD radix sort and FP64 tree sums.  No floating-point
// atomics; every reduction order is fixed by the problem size alone.
#include "gr_internal.hpp"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

namespace gr {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return GR_OK;
    return set_error(GR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err; }
void clear_error() { g_err[0] = 0; }

// --------------------------------------------------------------- profiling
namespace prof {
struct Rec {
    int phase;
    hipEvent_t a, b;
    double bytes;
    int64_t launches;
};
static thread_local bool g_on = false;
static thread_local std::vector<Rec> g_recs;
static thread_local std::vector<hipEvent_t> g_pool;
static thread_local hipEvent_t g_open = nullptr;

static hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool on() { return g_on; }

void begin(hipStream_t st) {
    g_open = get_event();
    if (g_open) (void)hipEventRecord(g_open, st);
}

void end(hipStream_t st, int phase, double bytes, int64_t launches) {
    if (!g_open) return;
    hipEvent_t e = get_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_recs.push_back(Rec{phase, g_open, e, bytes, launches});
    g_open = nullptr;
}

// Every event is destroyed when a profile stops, so no HIP object of the
// profiler outlives a start/stop pair (nothing is left for the runtime to
// tear down at process exit).
static void release_all() {
    for (auto& r : g_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    if (g_open) (void)hipEventDestroy(g_open);
    g_open = nullptr;
}

void start() {
    g_on = true;
    release_all();
}

int stop(gr_profile* out) {
    g_on = false;
    memset(out, 0, sizeof(*out));
    for (auto& r : g_recs) {
        float ms = 0.0f;
        int rc = check_hip(hipEventSynchronize(r.b), "profile event");
        if (rc == GR_OK) rc = check_hip(hipEventElapsedTime(&ms, r.a, r.b), "profile event");
        if (rc != GR_OK) {
            release_all();
            return rc;
        }
        out->phase_ms[r.phase] += ms;
        out->phase_bytes[r.phase] += r.bytes;
        out->phase_launches[r.phase] += r.launches;
        if (ms > out->phase_max_ms[r.phase]) out->phase_max_ms[r.phase] = ms;
        out->records += 1;
    }
    release_all();
    return GR_OK;
}
}  // namespace prof

// ---------------------------------------------------------------- scans
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ inline T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and writes the block total to *total.
template <class T>
__device__ inline T block_exclusive_scan(T v, T* total) {
    __shared__ T wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// A thread's kScanItems consecutive values: 16-byte vector loads when the
// array is 16-byte aligned and the thread's items are all in range (each
// lane then moves whole 16-byte chunks), else one value at a time.
template <class T>
__device__ inline void scan_load(const T* __restrict__ in, int64_t base, int64_t n, bool vec,
                                 T* vals) {
    constexpr int V = 16 / sizeof(T);
    if (vec && base + kScanItems <= n) {
#pragma unroll
        for (int i = 0; i < kScanItems; i += V) {
            const uint4 u = *reinterpret_cast<const uint4*>(in + base + i);
            const T* t = reinterpret_cast<const T*>(&u);
#pragma unroll
            for (int k = 0; k < V; ++k) vals[i + k] = t[k];
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) vals[i] = (base + i < n) ? in[base + i] : T(0);
    }
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const T* __restrict__ in, int64_t n,
                                                            T* __restrict__ part, int vec) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T vals[kScanItems];
    scan_load<T>(in, base, n, vec != 0, vals);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) s += vals[i];
    T tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const T* __restrict__ in, T* __restrict__ out,
                                                            int64_t n, const T* __restrict__ part_off,
                                                            T* __restrict__ total, int vec) {
    constexpr int V = 16 / sizeof(T);
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T vals[kScanItems];
    scan_load<T>(in, base, n, vec != 0, vals);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) s += vals[i];
    T tot;
    T run = block_exclusive_scan(s, &tot) + (part_off ? part_off[blockIdx.x] : T(0));
    if (vec && base + kScanItems <= n) {
#pragma unroll
        for (int i = 0; i < kScanItems; i += V) {
            uint4 u;
            T* t = reinterpret_cast<T*>(&u);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                t[k] = run;
                run += vals[i + k];
            }
            *reinterpret_cast<uint4*>(out + base + i) = u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < n) out[base + i] = run;
            run += vals[i];
        }
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total = run;
}

template <class T>
static int scan_exclusive(const T* in, T* out, int64_t n, T* total, Arena& ws, hipStream_t st) {
    if (n <= 0) {
        if (total && !ws.sizing()) GR_HIP(hipMemsetAsync(total, 0, sizeof(T), st));
        return GR_OK;
    }
    unsigned nb = blocks_for(n, kScanTile);
    const int vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (nb == 1) {
        if (ws.sizing()) return GR_OK;
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kScanThreads), 0, st, in, out, n,
                           (const T*)nullptr, total, vec);
        GR_LAUNCHED("scan");
        return GR_OK;
    }
    size_t mark = ws.used;
    T* part = ws.take<T>(nb);
    T* part_off = ws.take<T>(nb);
    if (!ws.sizing() && ws.overflow) return set_error(GR_ENOMEM, "workspace too small (scan)");
    if (!ws.sizing()) {
        hipLaunchKernelGGL(k_tile_sums<T>, dim3(nb), dim3(kScanThreads), 0, st, in, n, part, vec);
        GR_LAUNCHED("scan partials");
    }
    GR_TRY(scan_exclusive<T>(part, part_off, nb, (T*)nullptr, ws, st));
    if (!ws.sizing()) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(nb), dim3(kScanThreads), 0, st, in, out, n,
                           (const T*)part_off, total, vec);
        GR_LAUNCHED("scan");
    }
    if (!ws.sizing()) ws.used = mark;  // scratch released (stream order keeps it valid)
    return GR_OK;
}

int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, Arena& ws,
                       hipStream_t st) {
    return scan_exclusive<int32_t>(in, out, n, total, ws, st);
}
int scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, Arena& ws,
                       hipStream_t st) {
    return scan_exclusive<int64_t>(in, out, n, total, ws, st);
}

// ----------------------------------------------------------- radix sort
#ifndef GR_SORT_ITERS
#define GR_SORT_ITERS 8
#endif
constexpr int kSortThreads = 256;
constexpr int kSortIters = GR_SORT_ITERS;
constexpr int kSortTile = kSortThreads * kSortIters;
constexpr int kRadix = 256;

template <class KT>
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const KT* __restrict__ keys,
                                                             int64_t n, int shift,
                                                             int32_t* __restrict__ hist,
                                                             int nblocks) {
    __shared__ int32_t cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        int64_t i = base + it * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xff], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// One pass of the stable LSD sort on digit (key >> shift) & 0xff (keys of 64
// or 32 bits; the narrow form moves a third fewer bytes).  Wave w of the
// block owns the kSortIters * 64 consecutive keys of its part of the tile
// and keeps them in registers.  It first counts its digits (a ballot match
// per round gives each digit's lanes; the lowest lane adds their number to
// the wave's own counter in LDS), the block then turns the counts into each
// wave's starting place per digit (digit-major, waves in order), and each
// wave walks its keys again in the same order, placing them at its running
// place plus their rank among the round's lanes of the same digit.  The
// order inside a digit is the input order (stable).  The tile is then
// written out digit by digit, each digit's keys as one contiguous run
// (coalesced stores) at the digit's global offset for this tile.
template <class KT>
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const KT* __restrict__ kin, const uint32_t* __restrict__ vin, KT* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, const int32_t* __restrict__ offs,
    int nblocks) {
    constexpr int kW = kSortThreads / kWave;
    __shared__ KT skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ int32_t gbase[kRadix];
    __shared__ int32_t lbase[kRadix];
    __shared__ int32_t wcnt[kW][kRadix];  // per wave: its count, then its place
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    for (int w = 0; w < kW; ++w) wcnt[w][tid] = 0;
    gbase[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tbase + (int64_t)wid * kSortIters * kWave;
    KT key[kSortIters];
    uint32_t val[kSortIters];
    int dig[kSortIters];
    uint64_t peer[kSortIters];
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        const int64_t i = wbase + it * kWave + lane;
        const bool valid = i < n;
        key[it] = valid ? kin[i] : KT(0);
        val[it] = valid ? vin[i] : 0u;
        // invalid lanes take digit 256: they match only each other
        dig[it] = valid ? (int)((key[it] >> shift) & 0xff) : kRadix;
    }
    __syncthreads();  // counters cleared
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        const int d = dig[it];
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        peer[it] = peers;
        if (d < kRadix && (peers & lt) == 0) wcnt[wid][d] += __popcll(peers);
    }
    __syncthreads();
    {
        // digit tid: the tile's count, its local base (exclusive scan over
        // digits), and each wave's place
        int32_t c = 0;
#pragma unroll
        for (int w = 0; w < kW; ++w) c += wcnt[w][tid];
        int32_t x = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        __shared__ int32_t wsum[kW];
        if (lane == kWave - 1) wsum[wid] = x;
        __syncthreads();
        int32_t pre = 0;
        for (int w = 0; w < wid; ++w) pre += wsum[w];
        int32_t place = pre + x - c;
        lbase[tid] = place;
#pragma unroll
        for (int w = 0; w < kW; ++w) {
            const int32_t cw = wcnt[w][tid];
            wcnt[w][tid] = place;
            place += cw;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortIters; ++it) {
        const int d = dig[it];
        if (d < kRadix) {
            const uint64_t peers = peer[it];
            const int lpos = wcnt[wid][d] + __popcll(peers & lt);
            skey[lpos] = key[it];
            sval[lpos] = val[it];
            // the digit's lowest lane moves the wave's place on, after every
            // lane of the digit has read it (a wave's LDS accesses are in order)
            if ((peers & lt) == 0) wcnt[wid][d] += __popcll(peers);
        }
    }
    __syncthreads();
    const int cnt = (int)(n - tbase < kSortTile ? n - tbase : kSortTile);
    for (int j = tid; j < cnt; j += kSortThreads) {
        const KT k = skey[j];
        const int d = (int)((k >> shift) & 0xff);
        const int64_t pos = (int64_t)gbase[d] + (j - lbase[d]);
        kout[pos] = k;
        vout[pos] = sval[j];
    }
}

template <class KT>
static int radix_sort(KT* keys_in, uint32_t* vals_in, KT* keys_out, uint32_t* vals_out, int64_t n,
                      int bits, Arena& ws, hipStream_t st) {
    int passes = (bits + 7) / 8;
    unsigned nb = blocks_for(n, kSortTile);
    size_t mark = ws.used;
    int32_t* hist = ws.take<int32_t>((size_t)kRadix * nb);
    int32_t* offs = ws.take<int32_t>((size_t)kRadix * nb);
    if (ws.sizing()) {
        GR_TRY(scan_exclusive_i32(nullptr, nullptr, (int64_t)kRadix * nb, nullptr, ws, st));
        return GR_OK;
    }
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (sort)");
    if (n <= 0) return GR_OK;
    KT* ks = keys_in;
    uint32_t* vs = vals_in;
    KT* kd = keys_out;
    uint32_t* vd = vals_out;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist<KT>, dim3(nb), dim3(kSortThreads), 0, st, ks, n, shift, hist,
                           (int)nb);
        GR_LAUNCHED("radix hist");
        GR_TRY(scan_exclusive_i32(hist, offs, (int64_t)kRadix * nb, nullptr, ws, st));
        hipLaunchKernelGGL(k_radix_scatter<KT>, dim3(nb), dim3(kSortThreads), 0, st, ks, vs, kd, vd,
                           n, shift, (const int32_t*)offs, (int)nb);
        GR_LAUNCHED("radix scatter");
        KT* tk = ks; ks = kd; kd = tk;
        uint32_t* tv = vs; vs = vd; vd = tv;
    }
    if (ks != keys_out) {
        GR_HIP(hipMemcpyAsync(keys_out, ks, sizeof(KT) * n, hipMemcpyDeviceToDevice, st));
        GR_HIP(hipMemcpyAsync(vals_out, vs, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
    }
    ws.used = mark;
    return GR_OK;
}

int radix_sort_pairs(uint64_t* keys_in, uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
                     int64_t n, int bits, Arena& ws, hipStream_t st) {
    return radix_sort<uint64_t>(keys_in, vals_in, keys_out, vals_out, n, bits, ws, st);
}

int radix_sort_pairs32(uint32_t* keys_in, uint32_t* vals_in, uint32_t* keys_out,
                       uint32_t* vals_out, int64_t n, int bits, Arena& ws, hipStream_t st) {
    if (bits > 32) return set_error(GR_EINVAL, "a 32-bit sort key has at most 32 bits");
    return radix_sort<uint32_t>(keys_in, vals_in, keys_out, vals_out, n, bits, ws, st);
}

// ------------------------------------------------------------ fp64 sum
constexpr int kSumThreads = 256;

__device__ inline double block_sum_f64(double v) {
    __shared__ double part[kSumThreads / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kSumThreads / kWave; ++w) t += part[w];
    __syncthreads();
    return t;
}

__global__ void __launch_bounds__(kSumThreads) k_sum_f64(const double* __restrict__ in, int64_t n,
                                                         int64_t per_block, double* __restrict__ out) {
    int64_t lo = (int64_t)blockIdx.x * per_block;
    int64_t hi = lo + per_block < n ? lo + per_block : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kSumThreads) s += in[i];
    s = block_sum_f64(s);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

int sum_f64(const double* in, int64_t n, double* out, Arena& ws, hipStream_t st) {
    const int64_t per = 8192;
    unsigned nb = blocks_for(n, (int)per);
    size_t mark = ws.used;
    double* part = ws.take<double>(nb);
    if (ws.sizing()) return GR_OK;
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (sum)");
    hipLaunchKernelGGL(k_sum_f64, dim3(nb), dim3(kSumThreads), 0, st, in, n, per, part);
    GR_LAUNCHED("sum_f64");
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kSumThreads), 0, st, (const double*)part,
                       (int64_t)nb, (int64_t)nb, out);
    GR_LAUNCHED("sum_f64 final");
    ws.used = mark;
    return GR_OK;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return GR_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
    GR_LAUNCHED("fill");
    return GR_OK;
}

}  // namespace gr
