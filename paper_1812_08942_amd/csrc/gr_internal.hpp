// Internal declarations shared by the HIP sources of libgraphreduce.
// gfx950 (CDNA4) only: wave64, 64 KiB+ LDS per workgroup, IEEE fp32 division.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "graphreduce.h"

namespace gr {

constexpr int kWave = 64;
// rows above this degree are listed (long_rows) and get a workgroup each
// in the per-row kernels that would otherwise serialise on them
constexpr int kLongRow = 128;

// ------------------------------------------------------------------ errors
int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);

#define GR_TRY(expr)                 \
    do {                             \
        int _rc = (expr);            \
        if (_rc != GR_OK) return _rc; \
    } while (0)

#define GR_HIP(expr) GR_TRY(::gr::check_hip((expr), #expr))
#define GR_LAUNCHED(what) GR_TRY(::gr::check_hip(hipGetLastError(), what))

// ------------------------------------------------------------- profiling
// Optional HIP-event timing of phases and kernels on the caller's stream
// (enabled by gr_profile_start on the calling thread; off by default).
namespace prof {
enum Phase { COLOUR = 0, RELABEL, INIT, SMOOTH, AFFINITY, AGGREGATE, GALERKIN, OTHER, NPHASE };
bool on();
void begin(hipStream_t st);
void end(hipStream_t st, int phase, double bytes, int64_t launches);
void start();
int stop(gr_profile* out);
}  // namespace prof

// ------------------------------------------------------------- workspace
// Bump allocator over a caller-provided device buffer.  Every carve is
// 256-byte aligned.  `base == nullptr` runs in sizing mode: nothing is
// dereferenced, only `used` grows, so the same code computes workspace sizes.
struct Arena {
    char* base;
    size_t cap;
    size_t used;
    bool overflow;
    Arena(void* b, size_t c) : base((char*)b), cap(c), used(0), overflow(false) {}
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        size_t bytes = count * sizeof(T);
        used = off + ((bytes + 255) & ~size_t(255));
        if (used > cap) overflow = true;
        if (!base || overflow) return nullptr;
        return reinterpret_cast<T*>(base + off);
    }
    bool sizing() const { return base == nullptr; }
};

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned blocks_for(int64_t n, int per_block) {
    int64_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

// ----------------------------------------------------------- device math
// SplitMix64 (Steele, Lea & Flood 2014): output i of the generator seeded
// with s is the variant-13 finaliser applied to s + (i + 1) * 0x9E3779B97F4A7C15.
__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// bfloat16 storage: round-to-nearest-even from binary32, NaN kept quiet.
__device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------- primitives
// Exclusive prefix sum of int32 values (deterministic).  Writes n outputs
// and, when `total` is non-null, the grand total to device memory.
int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                       Arena& ws, hipStream_t st);
// Same for int64.
int scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                       Arena& ws, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// Results land in keys_out/vals_out; the inputs are used as scratch.
int radix_sort_pairs(uint64_t* keys_in, uint32_t* vals_in, uint64_t* keys_out,
                     uint32_t* vals_out, int64_t n, int bits, Arena& ws, hipStream_t st);
// The same for keys of at most 32 bits.
int radix_sort_pairs32(uint32_t* keys_in, uint32_t* vals_in, uint32_t* keys_out,
                       uint32_t* vals_out, int64_t n, int bits, Arena& ws, hipStream_t st);

// Deterministic FP64 sum of n values into *out (device).
int sum_f64(const double* in, int64_t n, double* out, Arena& ws, hipStream_t st);

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);

inline int bits_for(int64_t n) {  // bits needed to hold values in [0, n)
    int b = 0;
    while (b < 63 && (int64_t(1) << b) < n) ++b;
    return b;
}

// --------------------------------------------------------------- phase A
int validate_graph(const gr_graph* g, Arena& ws, hipStream_t st);
int colour_greedy(const gr_graph* g, uint64_t seed, int ldf, int32_t* colours,
              int32_t* n_colours_host, Arena& ws, hipStream_t st);
int validate_colouring(const gr_graph* g, const int32_t* colours, int32_t n_colours,
                       Arena& ws, hipStream_t st);

// Colour-major relabel: new row r holds old node perm[r]; rows of colour c
// are [class_ptr[c], class_ptr[c+1]), and inside a class the rows come in
// decreasing degree tiers: tier 0 holds degrees above 2048, tier t in 1..8
// degrees in (4096 >> (t + 1), 4096 >> t], tier 9 degrees up to 8.  The
// long rows (degree above 128, tiers 0..4) thus come first:
// [class_ptr[c], long_end[c]).  Host copies of the boundaries are kept for
// launch planning.
constexpr int kNT = 10;
constexpr int kLongTiers = 5;
__host__ __device__ inline int degree_tier(int32_t deg) {
    int t = 0;
    for (int32_t hi = 2048; t < kNT - 1 && deg <= hi; hi >>= 1) ++t;
    return t;  // 0: > 2048, 1: (1024, 2048], ..., 9: <= 8
}
inline int32_t tier_max_degree(int t) { return t == 0 ? 0x7fffffff : (4096 >> t); }

struct OrderedGraph {
    gr_graph g;          // relabelled CSR (device pointers into the arena)
    int32_t* perm;       // [n] new -> old
    int32_t* iperm;      // [n] old -> new
    int32_t n_colours;
    std::vector<int64_t> class_ptr_h;   // host [C+1]
    std::vector<int64_t> tier_ptr_h;    // host [C*kNT+1]: row start of (class, tier)
    std::vector<int64_t> long_end_h;    // host [C]
    std::vector<int64_t> class_nnz_h;   // host [C]: stored entries per colour
    std::vector<int64_t> class_e_h;     // host [C+1]: first entry of each colour
    std::vector<int64_t> long_nnz_h;    // host [C]: entries of the colour's long rows
    int64_t n_long;      // long rows in all classes
    int32_t* long_rows;  // device [n_long]: their relabelled ids
    double mean_deg;
};
int order_by_colour(const gr_graph* g, const int32_t* colours, int32_t n_colours,
                    OrderedGraph* out, Arena& ws, hipStream_t st);

// dst[r] = src[perm[r]] (inverse = 0) or dst[perm[r]] = src[r] (inverse = 1),
// rows of row_bytes (a multiple of 16) bytes.
int permute_rows(const void* src, void* dst, const int32_t* perm, int64_t n, size_t row_bytes,
                 int inverse, hipStream_t st);

int init_vectors(int64_t n, int32_t K, uint64_t seed, int32_t dtype, const int32_t* ids,
                 void* X, Arena& ws, hipStream_t st);
int smooth_ordered(const OrderedGraph* og, int32_t K, int32_t sweeps, int32_t dtype,
                   void* X, Arena& ws, hipStream_t st);
// a (affinity) and dist (algebraic distance d = 1 - a) per entry are
// optional; best = argmin (d, id) per row, dbest its distance, id = ids[j]
// (ids NULL: j itself).  Rows of degree above the long-row threshold are
// listed in long_rows (n_long of them) and handled by a workgroup each.
int affinity(const gr_graph* g, int32_t K, int32_t dtype, const void* X, const int32_t* ids,
             const int32_t* long_rows, int64_t n_long, float* a, float* dist, int32_t* best,
             float* dbest, hipStream_t st);
// rows of degree above the long-row threshold, in increasing order
int find_long_rows(const gr_graph* g, int32_t** rows, int64_t* n_long, Arena& ws, hipStream_t st);

// ---------------------------------------------------- aggregation / RAP
int aggregate(const gr_graph* g, const int32_t* best, const float* dbest, const int32_t* ids,
              int64_t target, int32_t* agg, int64_t* n_coarse, int64_t* n_forest,
              Arena& ws, hipStream_t st);
int galerkin(const gr_graph* g, const int32_t* agg, int64_t n_coarse, int32_t* c_row_ptr,
             int32_t* c_col, float* c_w, int64_t* nnz_coarse, const int32_t* long_rows,
             int64_t n_long, Arena& ws, hipStream_t st);

// ------------------------------------------------ data restriction (Alg. 6)
size_t restrict_workspace(int64_t n, int64_t nc, int32_t d);
int restrict_mean(const int32_t* agg, int64_t n, int64_t nc, int32_t d, const float* F, float* FR,
                  Arena& ws, hipStream_t st);
int restrict_sum_f64(const int32_t* agg, int64_t n, int64_t nc, const double* b, double* bc,
                     Arena& ws, hipStream_t st);

// ------------------------------------------------------ edge derivatives
int edge_list(const gr_graph* g, int32_t* eu, int32_t* ev, int32_t* eoe, int64_t* n_edges,
              Arena& ws, hipStream_t st);
int rq_forward(int64_t n, int64_t E, const int32_t* eu, const int32_t* ev, const double* w,
               const double* U, int32_t m, int32_t mode, double* R, double* den, Arena& ws,
               hipStream_t st);
int expand_weights(const int32_t* eoe, int64_t nnz, int64_t E, const float* wE, float* w,
                   hipStream_t st);
size_t eig_workspace(int64_t n, int32_t n_eig);
int laplacian_eigs(const gr_graph* g, const double* bdiag, int32_t n_eig, int32_t method,
                   double tol, int32_t max_iter, int32_t degree, uint64_t seed, double* eig_out,
                   double* vec_out, gr_eig_report* rep, Arena& ws, hipStream_t st);
size_t jacobi_workspace(int64_t n, int32_t k);
int jacobi_filter(const gr_graph* g, int32_t k, double* Y, const double* lam_host,
                  const double* bdiag, double theta, int32_t iters, Arena& ws, hipStream_t st);
size_t orthonormalize_workspace(int64_t n, int32_t k);
int orthonormalize(int64_t n, int32_t k, double* U, const double* bdiag, Arena& ws,
                   hipStream_t st);
size_t multilevel_workspace(int64_t n, int64_t nnz, int32_t k);
int multilevel_eigs(const gr_graph* g, const gr_hierarchy* h, int32_t k, int32_t cut, double theta,
                    int32_t iters, double tol, int32_t max_iter, uint64_t seed, double* lam_out,
                    double* U, gr_eig_report* rep, Arena& ws, hipStream_t st);
size_t sparsify_workspace(int64_t n, int64_t nnz);
int edge_weights(const gr_graph* g, const int32_t* eoe, float* wE, hipStream_t st);
int spanning_forest(const gr_graph* g, const int32_t* eu, const int32_t* ev, const int32_t* eoe,
                    int32_t* in_tree, int64_t E, int64_t* n_tree, Arena& ws, hipStream_t st);
int subgraph(const gr_graph* g, const int32_t* eoe, const int32_t* keep, int64_t E,
             const int32_t* eu, const int32_t* ev, int32_t* prp, int32_t* pcol, float* pw,
             int32_t* peoe, int32_t* peu, int32_t* pev, int64_t* p_nnz, int64_t* p_edges,
             Arena& ws, hipStream_t st);
int sparsify(const gr_graph* g, const gr_sparsify_params* prm, int32_t* keep, double* crit_out,
             gr_sparsify_report* rep, Arena& ws, hipStream_t st);
size_t sgd_workspace(int64_t n, int64_t nnzG, int64_t nnzP, int64_t E);
int sgd_scale(const gr_graph* G, const gr_graph* P, const int32_t* eoe, int64_t E,
              const int32_t* eu, const int32_t* ev, double* wP, const gr_sgd_params* prm,
              gr_sgd_report* rep, Arena& ws, hipStream_t st);
size_t vjp_workspace(int64_t n, int64_t nnz, int32_t K, int32_t dtype, int32_t S, int32_t store);
int smooth_vjp(const gr_graph* g, const int32_t* eoe, int64_t E, const int32_t* colours, int32_t C,
               int32_t K, int32_t S, int32_t dtype, const void* X0, const float* Gc, float* gw,
               float* gX0, int32_t store, Arena& ws, hipStream_t st);
int rq_forward_noalloc(int64_t n, int64_t E, const int32_t* eu, const int32_t* ev, const double* w,
                       const double* U, int32_t m, int32_t mode, double* R, double* den,
                       hipStream_t st);
size_t rq_forward_scratch_bytes(int32_t m);
size_t rq_forward_scratch_capacity();
int rq_backward(int64_t E, const int32_t* eu, const int32_t* ev, const double* U, int32_t m,
                int32_t mode, const double* R, const double* den, const double* gR, double* gw,
                hipStream_t st);

}  // namespace gr
