// The reduced data set of the multilevel data visualisation (Alg. 6):
// F_R = H_G^R F, with H_G^R read as the averaging restriction for data, so
// that row I of F_R is the mean of the rows of F over the nodes of aggregate
// I.  The nodes are sorted by aggregate (stable, so members stay in node
// order); every aggregate is cut into pieces of kRPiece members whose FP64
// partial sums are added in order, so hub aggregates spread over many
// threads and the result does not depend on scheduling.
#include "gr_internal.hpp"
#include "gr_device.hpp"

namespace gr {

constexpr int kRT = 256;
constexpr int kRPiece = 256;  // members per piece

// flag bits: 1 = an aggregate id outside [0, n_coarse), 2 = an empty aggregate
__global__ void k_restrict_keys(const int32_t* __restrict__ agg, int64_t n, int64_t nc,
                                uint64_t* __restrict__ key, uint32_t* __restrict__ val,
                                int32_t* bad) {
    const int64_t v = (int64_t)blockIdx.x * kRT + threadIdx.x;
    if (v >= n) return;
    int32_t a = agg[v];
    if (a < 0 || a >= nc) {
        atomicOr(bad, 1);
        a = 0;
    }
    key[v] = (uint64_t)a;
    val[v] = (uint32_t)v;
}

// mstart[c] = the first sorted position whose aggregate is >= c; k over [0, n]
__global__ void k_member_bounds(const uint64_t* __restrict__ skey, int64_t n, int64_t nc,
                                int32_t* __restrict__ mstart) {
    const int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x;
    if (k > n) return;
    const int64_t lo = k == 0 ? -1 : (int64_t)skey[k - 1];
    const int64_t hi = k == n ? nc : (int64_t)skey[k];
    for (int64_t c = lo + 1; c <= hi; ++c) mstart[c] = (int32_t)k;
}

__global__ void k_restrict_piece_counts(const int32_t* __restrict__ mstart, int64_t nc,
                                        int32_t* __restrict__ cnt, int32_t* bad) {
    const int64_t c = (int64_t)blockIdx.x * kRT + threadIdx.x;
    if (c >= nc) return;
    const int32_t m = mstart[c + 1] - mstart[c];
    if (m == 0) atomicOr(bad, 2);
    cnt[c] = (m + kRPiece - 1) / kRPiece;
}

__global__ void k_restrict_piece_rows(const int32_t* __restrict__ ppos, int64_t nc,
                                      int32_t* __restrict__ prow) {
    const int64_t c = (int64_t)blockIdx.x * kRT + threadIdx.x;
    if (c >= nc) return;
    for (int32_t k = ppos[c]; k < ppos[c + 1]; ++k) prow[k] = (int32_t)c;
}

// a thread per (piece, column): the FP64 sum of the piece's members in order
template <class T>
__global__ void k_restrict_pieces(const uint32_t* __restrict__ members,
                                  const int32_t* __restrict__ mstart,
                                  const int32_t* __restrict__ ppos,
                                  const int32_t* __restrict__ prow, int64_t npieces, int32_t d,
                                  const T* __restrict__ F, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * kRT + threadIdx.x;
    const int64_t k = t / d;
    const int32_t col = (int32_t)(t % d);
    if (k >= npieces) return;
    const int32_t c = prow[k];
    const int32_t m0 = mstart[c] + (int32_t)(k - ppos[c]) * kRPiece;
    const int32_t m1 = min(m0 + kRPiece, mstart[c + 1]);
    double s = 0.0;
    int32_t m = m0;
    for (; m + 4 <= m1; m += 4) {  // four rows in flight, added in member order
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = F[(int64_t)members[m + u] * d + col];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += (double)x[u];
    }
    for (; m < m1; ++m) s += (double)F[(int64_t)members[m] * d + col];
    part[k * d + col] = s;
}

// a thread per (aggregate, column): its pieces in order, over the member
// count (the mean, float32) or not (the sum, FP64)
__global__ void k_restrict_final(const int32_t* __restrict__ mstart,
                                 const int32_t* __restrict__ ppos, int64_t nc, int32_t d,
                                 const double* __restrict__ part, float* __restrict__ FR) {
    const int64_t t = (int64_t)blockIdx.x * kRT + threadIdx.x;
    const int64_t c = t / d;
    const int32_t col = (int32_t)(t % d);
    if (c >= nc) return;
    double s = 0.0;
    for (int32_t k = ppos[c]; k < ppos[c + 1]; ++k) s += part[(int64_t)k * d + col];
    FR[c * d + col] = (float)(s / (double)(mstart[c + 1] - mstart[c]));
}

__global__ void k_restrict_final_sum(const int32_t* __restrict__ ppos, int64_t nc, int32_t d,
                                     const double* __restrict__ part, double* __restrict__ FR) {
    const int64_t t = (int64_t)blockIdx.x * kRT + threadIdx.x;
    const int64_t c = t / d;
    const int32_t col = (int32_t)(t % d);
    if (c >= nc) return;
    double s = 0.0;
    for (int32_t k = ppos[c]; k < ppos[c + 1]; ++k) s += part[(int64_t)k * d + col];
    FR[c * d + col] = s;
}

size_t restrict_workspace(int64_t n, int64_t nc, int32_t d) {
    const size_t N = (size_t)n + 1, C = (size_t)nc + 1;
    const size_t pieces = N / kRPiece + C;
    size_t b = 24 * N                          // keys and values, twice
               + 16 * C                        // member bounds, piece counts and offsets
               + 4 * pieces                    // piece aggregates
               + 8 * pieces * (size_t)d        // partial sums
               + 4 * N;                        // sort histograms and scans
    return b + b / 8 + (1u << 20);
}

// mean (FR32 != NULL) or FP64 sum (FR64 != NULL) of F's rows per aggregate
template <class T>
static int restrict_rows(const int32_t* agg, int64_t n, int64_t nc, int32_t d, const T* F,
                         float* FR32, double* FR64, Arena& ws, hipStream_t st) {
    const size_t mark = ws.used;
    uint64_t* k0 = ws.take<uint64_t>(n);
    uint32_t* v0 = ws.take<uint32_t>(n);
    uint64_t* k1 = ws.take<uint64_t>(n);
    uint32_t* v1 = ws.take<uint32_t>(n);
    int32_t* mstart = ws.take<int32_t>(nc + 1);
    int32_t* cnt = ws.take<int32_t>(nc);
    int32_t* ppos = ws.take<int32_t>(nc + 1);
    int32_t* bad = ws.take<int32_t>(4);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (restriction)");
    GR_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t) * 4, st));
    hipLaunchKernelGGL(k_restrict_keys, dim3(blocks_for(n, kRT)), dim3(kRT), 0, st, agg, n, nc, k0, v0,
                       bad);
    GR_LAUNCHED("restrict keys");
    GR_TRY(radix_sort_pairs(k0, v0, k1, v1, n, bits_for(nc), ws, st));
    hipLaunchKernelGGL(k_member_bounds, dim3(blocks_for(n + 1, kRT)), dim3(kRT), 0, st,
                       (const uint64_t*)k1, n, nc, mstart);
    GR_LAUNCHED("member bounds");
    hipLaunchKernelGGL(k_restrict_piece_counts, dim3(blocks_for(nc, kRT)), dim3(kRT), 0, st,
                       (const int32_t*)mstart, nc, cnt, bad);
    GR_LAUNCHED("piece counts");
    GR_TRY(scan_exclusive_i32(cnt, ppos, nc, ppos + nc, ws, st));
    int32_t hb[2] = {0, 0};
    GR_HIP(hipMemcpyAsync(&hb[0], bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipMemcpyAsync(&hb[1], ppos + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    if (hb[0] & 1) return set_error(GR_EINVAL, "an aggregate id lies outside [0, %lld)", (long long)nc);
    if (hb[0] & 2) return set_error(GR_EINVAL, "an aggregate has no member");
    const int64_t np = hb[1];
    int32_t* prow = ws.take<int32_t>(np + 1);
    double* part = ws.take<double>((size_t)np * d + 1);
    if (ws.overflow) return set_error(GR_ENOMEM, "workspace too small (restriction pieces)");
    hipLaunchKernelGGL(k_restrict_piece_rows, dim3(blocks_for(nc, kRT)), dim3(kRT), 0, st,
                       (const int32_t*)ppos, nc, prow);
    GR_LAUNCHED("piece rows");
    hipLaunchKernelGGL(k_restrict_pieces<T>, dim3(blocks_for(np * d, kRT)), dim3(kRT), 0, st,
                       (const uint32_t*)v1, (const int32_t*)mstart, (const int32_t*)ppos,
                       (const int32_t*)prow, np, d, F, part);
    GR_LAUNCHED("restrict pieces");
    if (FR32) {
        hipLaunchKernelGGL(k_restrict_final, dim3(blocks_for(nc * d, kRT)), dim3(kRT), 0, st,
                           (const int32_t*)mstart, (const int32_t*)ppos, nc, d, (const double*)part,
                           FR32);
    } else {
        hipLaunchKernelGGL(k_restrict_final_sum, dim3(blocks_for(nc * d, kRT)), dim3(kRT), 0, st,
                           (const int32_t*)ppos, nc, d, (const double*)part, FR64);
    }
    GR_LAUNCHED("restrict final");
    ws.used = mark;
    return GR_OK;
}

int restrict_mean(const int32_t* agg, int64_t n, int64_t nc, int32_t d, const float* F, float* FR,
                  Arena& ws, hipStream_t st) {
    return restrict_rows<float>(agg, n, nc, d, F, FR, nullptr, ws, st);
}

// B^{l+1} = P^T B^l P for a diagonal B: the FP64 sum of b over each
// aggregate's members, in node order (in fixed pieces of kRPiece)
int restrict_sum_f64(const int32_t* agg, int64_t n, int64_t nc, const double* b, double* bc,
                     Arena& ws, hipStream_t st) {
    if (n == 0) return GR_OK;
    return restrict_rows<double>(agg, n, nc, 1, b, nullptr, bc, ws, st);
}

}  // namespace gr
