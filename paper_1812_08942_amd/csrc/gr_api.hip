// extern "C" entry points of libgraphreduce and the multilevel driver of
// Phase A (Sec. 3.2; the reduction ratio psi of Alg. 2).  Argument checks
// happen here, on the host, before any kernel sees a pointer or a size.
#include "gr_internal.hpp"

#include <math.h>
#include <string.h>

namespace gr {
const char* last_error();
void clear_error();

static int check_graph_args(const gr_graph* g) {
    if (!g) return set_error(GR_EINVAL, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return set_error(GR_EINVAL, "negative n or nnz");
    if (g->n >= (int64_t(1) << 31) - 1 || g->nnz >= (int64_t(1) << 31) - 1)
        return set_error(GR_EINVAL, "n and nnz must be below 2^31 - 1");
    if (!g->row_ptr) return set_error(GR_EINVAL, "row_ptr is NULL");
    if (g->nnz > 0 && (!g->col || !g->w)) return set_error(GR_EINVAL, "col or w is NULL");
    return GR_OK;
}

static int check_vec_args(int32_t K, int32_t dtype) {
    if (dtype != GR_F32 && dtype != GR_BF16) return set_error(GR_EUNSUP, "unknown dtype %d", dtype);
    if (K < 1 || K > 64) return set_error(GR_EUNSUP, "K must lie in [1, 64]");
    int bytes = K * (dtype == GR_BF16 ? 2 : 4);
    if (bytes % 16) return set_error(GR_EUNSUP, "K=%d: rows must be a multiple of 16 bytes "
                                                "(K %% 4 == 0 for float32, K %% 8 == 0 for bfloat16)", K);
    return GR_OK;
}

static int check_aligned(const void* p, const char* what) {
    if (((uintptr_t)p) & 15) return set_error(GR_EINVAL, "%s must be 16-byte aligned", what);
    return GR_OK;
}

static size_t vec_bytes(int64_t n, int32_t K, int32_t dtype) {
    return (size_t)n * (size_t)K * (dtype == GR_BF16 ? 2 : 4);
}

// Upper bound of the workspace every entry point may carve (see each
// function's takes; 256-byte alignment slack included).
static size_t plan_bytes(int64_t n, int64_t nnz, int32_t K, int32_t dtype) {
    const size_t N = (size_t)n + 1, M = (size_t)nnz + 1;
    auto sort_scratch = [](size_t m) { return 2 * 256 * 4 * (m / 2048 + 1) + m / 64 + 256 * 1024; };
    size_t persistent = 4 * N                                  // colours
                        + 4 * N * 3 + 8 * M                    // relabelled graph
                        + vec_bytes(n, K, dtype) + 256         // X
                        + 4 * N * 4                            // best, abest, agg (two)
                        + 2 * (4 * N + 8 * M)                  // coarse ping-pong
                        + 4 * N;                               // long-row ids
    size_t relabel = 36 * N + 8 * 1024 + sort_scratch(N);
    // colouring: sort keys and values, ranks, positions, batches, up-lists
    size_t colour = 46 * N + 4 * M + sort_scratch(N) + 8192;
    size_t agg = 8 * N + 24 * N + 44 * N + sort_scratch(N);  // (+ best in own order)
    // per fine row: counts, positions, sort keys and values (twice);
    // per coarse row: bounds, segments, lists, runs, counts; per kept entry
    // (at most M/2): column, weight, run column, run sum, and for hub rows
    // the sort and segmented sums; per run (at most M/2): the mirror sort
    size_t gal = 64 * N + 64 * N + 24 * M + 36 * (M / 2) + 36 * (M / 2) + sort_scratch(M);
    size_t temp = relabel;
    if (colour > temp) temp = colour;
    if (agg > temp) temp = agg;
    if (gal > temp) temp = gal;
    size_t total = persistent + temp;
    return total + total / 16 + (17u << 20);
}

static void copy_params(const gr_params* p, gr_params* q) { memcpy(q, p, sizeof(*q)); }

__global__ void k_iota_i32(int32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// the strongest neighbour of relabelled row r, moved to the level's own
// order: entry perm[r] names perm[best[r]]
__global__ void k_best_own(const int32_t* __restrict__ best, const float* __restrict__ dbest,
                           const int32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ obest,
                           float* __restrict__ odbest) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t b = best[r], o = perm[r];
    obest[o] = b >= 0 ? perm[b] : -1;
    odbest[o] = dbest[r];
}

// agg_own[perm[r]] = aggp[r]
__global__ void k_unpermute(const int32_t* __restrict__ aggp, const int32_t* __restrict__ perm,
                            int64_t n, int32_t* __restrict__ agg) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) agg[perm[r]] = aggp[r];
}

// out[i] = perm[in[i]]: relabelled row ids back to the level's own
__global__ void k_map_ids(const int32_t* __restrict__ in, const int32_t* __restrict__ perm,
                          int64_t n, int32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = perm[in[i]];
}

// total[v] = lvl[total[v]]
__global__ void k_compose(const int32_t* __restrict__ lvl, int64_t n0, int32_t* __restrict__ total) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) total[v] = lvl[total[v]];
}

// strongest neighbour from per-entry algebraic distances: argmin (d, j),
// one thread per row
__global__ void k_best_from_d(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const float* __restrict__ d, int64_t n, int32_t* __restrict__ best,
                              float* __restrict__ dbest) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t b = -1;
    float bd = 1.0f;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
        if (b < 0 || d[e] < bd) { bd = d[e]; b = col[e]; }  // columns ascend: first min wins
    best[v] = b;
    dbest[v] = bd;
}

__global__ void k_f64_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_f32_to_f64(const float* __restrict__ a, int64_t n, double* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

}  // namespace gr

using namespace gr;

extern "C" {

int gr_version(void) { return 10000; }

const char* gr_status_string(int s) {
    switch (s) {
        case GR_OK: return "ok";
        case GR_EINVAL: return "invalid argument";
        case GR_ECSR: return "malformed CSR graph";
        case GR_ECOLOUR: return "invalid colouring";
        case GR_ENOMEM: return "workspace or output too small";
        case GR_EHIP: return "HIP runtime error";
        case GR_EUNSUP: return "unsupported K / dtype";
    }
    return "unknown status";
}

const char* gr_last_error(void) { return last_error(); }

int gr_profile_start(void) {
    clear_error();
    prof::start();
    return GR_OK;
}

int gr_profile_stop(gr_profile* out) {
    clear_error();
    if (!out) return set_error(GR_EINVAL, "out is NULL");
    return prof::stop(out);
}

int gr_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t vec_dtype, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz < 0) return set_error(GR_EINVAL, "negative size");
    GR_TRY(check_vec_args(K, vec_dtype));
    *bytes = plan_bytes(n, nnz, K, vec_dtype);
    return GR_OK;
}

int gr_validate(const gr_graph* g, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!ws) return set_error(GR_EINVAL, "workspace is NULL");
    Arena A(ws, ws_bytes);
    return validate_graph(g, A, S(stream));
}

int gr_colour_greedy(const gr_graph* g, uint64_t seed, int32_t ldf, int32_t* colours,
                     int32_t* n_colours, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!colours || !n_colours || !ws) return set_error(GR_EINVAL, "NULL output or workspace");
    Arena A(ws, ws_bytes);
    return colour_greedy(g, seed, ldf ? 1 : 0, colours, n_colours, A, S(stream));
}

int gr_init_vectors(int64_t n, int32_t K, uint64_t seed, int32_t dtype, void* X, void* ws,
                    size_t ws_bytes, void* stream) {
    clear_error();
    if (n < 0) return set_error(GR_EINVAL, "negative n");
    GR_TRY(check_vec_args(K, dtype));
    if (n > 0 && (!X || !ws)) return set_error(GR_EINVAL, "NULL X or workspace");
    Arena A(ws, ws_bytes);
    return init_vectors(n, K, seed, dtype, nullptr, X, A, S(stream));
}

int gr_smooth(const gr_graph* g, const int32_t* colours, int32_t n_colours, int32_t K,
              int32_t sweeps, int32_t dtype, void* X, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    GR_TRY(check_vec_args(K, dtype));
    if (sweeps < 0) return set_error(GR_EINVAL, "sweeps must be >= 0");
    if (n_colours < 0 || (g->n > 0 && n_colours < 1)) return set_error(GR_EINVAL, "bad n_colours");
    if (g->n == 0 || sweeps == 0) return GR_OK;
    if (!colours || !X || !ws) return set_error(GR_EINVAL, "NULL colours, X or workspace");
    GR_TRY(check_aligned(X, "X"));
    hipStream_t st = S(stream);
    Arena A(ws, ws_bytes);
    GR_TRY(validate_colouring(g, colours, n_colours, A, st));
    OrderedGraph og;
    GR_TRY(order_by_colour(g, colours, n_colours, &og, A, st));
    // permute X into colour-major rows, smooth, permute back
    size_t vb = vec_bytes(g->n, K, dtype);
    char* Xp = A.take<char>(vb);
    if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (smooth)");
    GR_TRY(permute_rows(X, Xp, og.perm, g->n, (size_t)K * (dtype == GR_BF16 ? 2 : 4), 0, st));
    GR_TRY(smooth_ordered(&og, K, sweeps, dtype, Xp, A, st));
    GR_TRY(permute_rows(Xp, X, og.perm, g->n, (size_t)K * (dtype == GR_BF16 ? 2 : 4), 1, st));
    return GR_OK;
}

int gr_affinity(const gr_graph* g, int32_t K, int32_t dtype, const void* X, float* a,
                float* dist, int32_t* best, float* dbest, void* ws, size_t ws_bytes,
                void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    GR_TRY(check_vec_args(K, dtype));
    if (g->n == 0) return GR_OK;
    if (!X || !best || !ws) return set_error(GR_EINVAL, "NULL X, best or workspace");
    GR_TRY(check_aligned(X, "X"));
    hipStream_t st = S(stream);
    Arena A(ws, ws_bytes);
    int32_t* long_rows = nullptr;
    int64_t n_long = 0;
    GR_TRY(find_long_rows(g, &long_rows, &n_long, A, st));
    return affinity(g, K, dtype, X, nullptr, long_rows, n_long, a, dist, best, dbest, st);
}

int gr_aggregate(const gr_graph* g, const float* dist, int64_t target, int32_t* agg,
                 int64_t* n_coarse, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!n_coarse) return set_error(GR_EINVAL, "n_coarse is NULL");
    *n_coarse = 0;
    if (g->n == 0) return GR_OK;
    if ((g->nnz > 0 && !dist) || !agg || !ws)
        return set_error(GR_EINVAL, "NULL dist, agg or workspace");
    hipStream_t st = S(stream);
    Arena A(ws, ws_bytes);
    int32_t* best = A.take<int32_t>(g->n);
    float* dbest = A.take<float>(g->n);
    if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (aggregate)");
    hipLaunchKernelGGL(k_best_from_d, dim3(blocks_for(g->n, 256)), dim3(256), 0, st, g->row_ptr,
                       g->col, dist, g->n, best, dbest);
    GR_LAUNCHED("best from d");
    return aggregate(g, best, dbest, nullptr, target, agg, n_coarse, nullptr, A, st);
}

int gr_galerkin(const gr_graph* g, const int32_t* agg, int64_t n_coarse, int32_t* c_row_ptr,
                int32_t* c_col, float* c_w, int64_t* nnz_coarse, void* ws, size_t ws_bytes,
                void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!nnz_coarse) return set_error(GR_EINVAL, "nnz_coarse is NULL");
    if (n_coarse < 0 || n_coarse > g->n || (g->n > 0 && n_coarse < 1))
        return set_error(GR_EINVAL, "n_coarse out of range");
    if (!c_row_ptr || !ws || (g->n > 0 && !agg) || (g->nnz > 0 && (!c_col || !c_w)))
        return set_error(GR_EINVAL, "NULL argument");
    Arena A(ws, ws_bytes);
    int32_t* long_rows = nullptr;
    int64_t n_long = 0;
    GR_TRY(find_long_rows(g, &long_rows, &n_long, A, S(stream)));
    return galerkin(g, agg, n_coarse, c_row_ptr, c_col, c_w, nnz_coarse, long_rows, n_long, A,
                    S(stream));
}

int gr_restrict_workspace(int64_t n, int64_t n_coarse, int32_t d, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || n_coarse < 0 || d < 1) return set_error(GR_EINVAL, "bad size");
    *bytes = restrict_workspace(n, n_coarse, d);
    return GR_OK;
}

int gr_restrict_mean(const int32_t* agg, int64_t n, int64_t n_coarse, int32_t d, const float* F,
                     float* F_R, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (n < 0 || d < 1) return set_error(GR_EINVAL, "bad size");
    if (n >= (int64_t(1) << 31)) return set_error(GR_EINVAL, "n must be below 2^31");
    if (n_coarse < 0 || n_coarse > n || (n > 0 && n_coarse < 1))
        return set_error(GR_EINVAL, "n_coarse out of range");
    if (n == 0) return GR_OK;
    if (!agg || !F || !F_R || !ws) return set_error(GR_EINVAL, "NULL argument");
    Arena A(ws, ws_bytes);
    return restrict_mean(agg, n, n_coarse, d, F, F_R, A, S(stream));
}

static int reduce_impl(const gr_graph* g, const gr_params* p_in, gr_result* res, gr_hierarchy* hier,
                       void* ws, size_t ws_bytes, void* stream) {
    GR_TRY(check_graph_args(g));
    if (!p_in || !res) return set_error(GR_EINVAL, "NULL params or result");
    gr_params p;
    copy_params(p_in, &p);
    GR_TRY(check_vec_args(p.K, p.vec_dtype));
    if (p.sweeps < 0) return set_error(GR_EINVAL, "sweeps must be >= 0");
    if (!(p.ratio >= 1.0) || !isfinite(p.ratio)) return set_error(GR_EINVAL, "ratio must be >= 1");
    if (p.max_levels < 0) return set_error(GR_EINVAL, "max_levels must be >= 0");
    if (p.colours && p.n_colours < 1) return set_error(GR_EINVAL, "n_colours must be >= 1");
    if (!res->agg || !res->c_row_ptr || (g->nnz > 0 && (!res->c_col || !res->c_w)) || !ws)
        return set_error(GR_EINVAL, "NULL output or workspace");
    res->n_coarse = 0;
    res->nnz_coarse = 0;
    res->levels = 0;
    res->warnings = 0;
    if (hier) {
        if (hier->maps_cap < 0 || hier->rp_cap < 0 || hier->ent_cap < 0)
            return set_error(GR_EINVAL, "negative hierarchy capacity");
        hier->levels = 0;
        for (int l = 0; l <= GR_MAX_LEVELS; ++l) hier->n[l] = hier->nnz[l] = 0;
        hier->n[0] = g->n;
        hier->nnz[0] = g->nnz;
    }
    int64_t h_maps = 0, h_rp = 0, h_ent = 0;  // hierarchy totals so far
    hipStream_t st = S(stream);
    Arena A(ws, ws_bytes);
    const int64_t n0 = g->n;
    if (p.flags & GR_VALIDATE) GR_TRY(validate_graph(g, A, st));
    A.used = 0;
    const int64_t target = (int64_t)ceil((double)n0 / p.ratio) < 1 ? 1
                                                                      : (int64_t)ceil((double)n0 / p.ratio);
    const int ldf = (p.flags & GR_COLOUR_LDF) ? 1 : 0;
    // persistent buffers sized for level 0
    int32_t* colours = A.take<int32_t>(n0 + 1);
    void* X = A.take<char>(vec_bytes(n0, p.K, p.vec_dtype) + 256);
    int32_t* best = A.take<int32_t>(n0 + 1);
    float* dbest = A.take<float>(n0 + 1);
    int32_t* aggl = A.take<int32_t>(n0 + 1);
    int32_t* gbuf_rp[2] = {A.take<int32_t>(n0 + 1), A.take<int32_t>(n0 + 1)};
    int32_t* gbuf_col[2] = {A.take<int32_t>(g->nnz + 1), A.take<int32_t>(g->nnz + 1)};
    float* gbuf_w[2] = {A.take<float>(g->nnz + 1), A.take<float>(g->nnz + 1)};
    if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (%zu bytes given)", ws_bytes);
    if (n0 > 0) {
        hipLaunchKernelGGL(k_iota_i32, dim3(blocks_for(n0, 256)), dim3(256), 0, st, res->agg, n0);
        GR_LAUNCHED("iota");
    }
    gr_graph cur = *g;
    int which = 0;
    int level = 0;
    const size_t level_mark = A.used;
    while (cur.n > target) {
        if (p.max_levels > 0 && level >= p.max_levels) break;
        A.used = level_mark;
        const uint64_t vseed = splitmix64(p.vec_seed, (uint64_t)level);
        const uint64_t cseed = splitmix64(p.colour_seed, (uint64_t)level);
        int32_t nc = 0;
        const int32_t* col_use = colours;
        const bool pr = prof::on();
        const double xs = p.vec_dtype == GR_BF16 ? 2.0 : 4.0;
        if (pr) prof::begin(st);
        if (level == 0 && p.colours) {
            GR_TRY(validate_colouring(&cur, p.colours, p.n_colours, A, st));
            col_use = p.colours;
            nc = p.n_colours;
        } else {
            GR_TRY(colour_greedy(&cur, cseed, ldf, colours, &nc, A, st));
        }
        if (pr) prof::end(st, prof::COLOUR, 0.0, 1);
        if (level < 32) {
            res->level_n[level] = cur.n;
            res->level_nnz[level] = cur.nnz;
            res->level_colours[level] = nc;
        }
        OrderedGraph og;
        if (pr) prof::begin(st);
        GR_TRY(order_by_colour(&cur, col_use, nc, &og, A, st));
        if (pr) prof::end(st, prof::RELABEL, 0.0, 1);
        if (pr) prof::begin(st);
        GR_TRY(init_vectors(cur.n, p.K, vseed, p.vec_dtype, og.perm, X, A, st));
        if (pr) prof::end(st, prof::INIT, (double)cur.n * p.K * xs + 4.0 * cur.n, 1);
        GR_TRY(smooth_ordered(&og, p.K, p.sweeps, p.vec_dtype, X, A, st));
        if (pr) prof::begin(st);
        GR_TRY(affinity(&og.g, p.K, p.vec_dtype, X, og.perm, og.long_rows, og.n_long, nullptr,
                        nullptr, best, dbest, st));
        // compulsory bytes: CSR columns, each vector row once, ids, best + abest
        if (pr)
            prof::end(st, prof::AFFINITY,
                      4.0 * (cur.n + 1) + 4.0 * cur.nnz + (double)cur.n * p.K * xs + 12.0 * cur.n,
                      1);
        int64_t ncoarse = 0, nforest = 0;
        if (pr) prof::begin(st);
        // on sparse levels the aggregation runs in the level's own order (a
        // node's strongest neighbour is near it there, and ids are the rows
        // themselves); on dense ones, without that locality, on the relabel
        const size_t mark_own = A.used;
        if (cur.nnz <= 32 * cur.n) {
            int32_t* obest = A.take<int32_t>(cur.n + 1);
            float* odbest = A.take<float>(cur.n + 1);
            if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (aggregation)");
            hipLaunchKernelGGL(k_best_own, dim3(blocks_for(cur.n, 256)), dim3(256), 0, st, best,
                               dbest, og.perm, cur.n, obest, odbest);
            GR_LAUNCHED("best, own order");
            GR_TRY(aggregate(&cur, obest, odbest, nullptr, target, aggl, &ncoarse, &nforest, A,
                             st));
        } else {
            int32_t* aggp = A.take<int32_t>(cur.n + 1);
            if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (aggregation)");
            GR_TRY(aggregate(&og.g, best, dbest, og.perm, target, aggp, &ncoarse, &nforest, A, st));
            hipLaunchKernelGGL(k_unpermute, dim3(blocks_for(cur.n, 256)), dim3(256), 0, st, aggp,
                               og.perm, cur.n, aggl);
            GR_LAUNCHED("unpermute");
        }
        A.used = mark_own;  // stream order keeps them valid for the launches above
        if (pr) prof::end(st, prof::AGGREGATE, 0.0, 1);
        gr_graph next;
        next.n = ncoarse;
        next.row_ptr = gbuf_rp[which];
        next.col = gbuf_col[which];
        next.w = gbuf_w[which];
        int64_t nnzc = 0;
        if (pr) prof::begin(st);
        // the collapse runs on the level's graph in its own order, where an
        // aggregate's members lie close together (in the colour-major order
        // they sit in different classes, far apart)
        int32_t* long_own = nullptr;
        if (og.n_long > 0) {
            long_own = A.take<int32_t>(og.n_long);
            if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (long rows)");
            hipLaunchKernelGGL(k_map_ids, dim3(blocks_for(og.n_long, 256)), dim3(256), 0, st,
                               og.long_rows, og.perm, og.n_long, long_own);
            GR_LAUNCHED("long rows, own order");
        }
        GR_TRY(galerkin(&cur, aggl, ncoarse, gbuf_rp[which], gbuf_col[which], gbuf_w[which], &nnzc,
                        long_own, og.n_long, A, st));
        if (pr) prof::end(st, prof::GALERKIN, 0.0, 1);
        next.nnz = nnzc;
        hipLaunchKernelGGL(k_compose, dim3(blocks_for(n0, 256)), dim3(256), 0, st, aggl, n0,
                           res->agg);
        GR_LAUNCHED("compose");
        bool stuck = ncoarse == cur.n;
        if (hier && !stuck) {  // keep this level's map and the graph it made
            const int l = hier->levels;
            if (l >= GR_MAX_LEVELS) return set_error(GR_ENOMEM, "more than %d levels", GR_MAX_LEVELS);
            if (h_maps + cur.n > hier->maps_cap || h_rp + ncoarse + 1 > hier->rp_cap ||
                h_ent + nnzc > hier->ent_cap || !hier->maps || !hier->row_ptr ||
                (nnzc > 0 && (!hier->col || !hier->w)))
                return set_error(GR_ENOMEM,
                                 "hierarchy buffers too small at level %d: need maps %lld, row "
                                 "pointers %lld, entries %lld so far",
                                 l, (long long)(h_maps + cur.n), (long long)(h_rp + ncoarse + 1),
                                 (long long)(h_ent + nnzc));
            hier->maps_off[l] = h_maps;
            hier->rp_off[l] = h_rp;
            hier->ent_off[l] = h_ent;
            GR_HIP(hipMemcpyAsync(hier->maps + h_maps, aggl, sizeof(int32_t) * cur.n,
                                  hipMemcpyDeviceToDevice, st));
            GR_HIP(hipMemcpyAsync(hier->row_ptr + h_rp, next.row_ptr,
                                  sizeof(int32_t) * (ncoarse + 1), hipMemcpyDeviceToDevice, st));
            if (nnzc > 0) {
                GR_HIP(hipMemcpyAsync(hier->col + h_ent, next.col, sizeof(int32_t) * nnzc,
                                      hipMemcpyDeviceToDevice, st));
                GR_HIP(hipMemcpyAsync(hier->w + h_ent, next.w, sizeof(float) * nnzc,
                                      hipMemcpyDeviceToDevice, st));
            }
            h_maps += cur.n;
            h_rp += ncoarse + 1;
            h_ent += nnzc;
            hier->levels = l + 1;
            hier->n[l + 1] = ncoarse;
            hier->nnz[l + 1] = nnzc;
        }
        ++level;
        cur = next;
        which ^= 1;
        if (stuck) {
            res->warnings |= GR_WNOPROGRESS;
            break;
        }
    }
    // final coarse graph into the caller's buffers
    GR_HIP(hipMemcpyAsync(res->c_row_ptr, cur.row_ptr, sizeof(int32_t) * (cur.n + 1),
                          hipMemcpyDeviceToDevice, st));
    if (cur.nnz > 0) {
        GR_HIP(hipMemcpyAsync(res->c_col, cur.col, sizeof(int32_t) * cur.nnz, hipMemcpyDeviceToDevice,
                              st));
        GR_HIP(hipMemcpyAsync(res->c_w, cur.w, sizeof(float) * cur.nnz, hipMemcpyDeviceToDevice, st));
    }
    res->n_coarse = cur.n;
    res->nnz_coarse = cur.nnz;
    res->levels = level;
    if (hier) GR_HIP(hipStreamSynchronize(st));
    return GR_OK;
}

int gr_reduce(const gr_graph* g, const gr_params* p, gr_result* res, void* ws, size_t ws_bytes,
              void* stream) {
    clear_error();
    return reduce_impl(g, p, res, nullptr, ws, ws_bytes, stream);
}

int gr_reduce_hierarchy(const gr_graph* g, const gr_params* p, gr_result* res, gr_hierarchy* h,
                        void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!h) return set_error(GR_EINVAL, "hierarchy is NULL");
    return reduce_impl(g, p, res, h, ws, ws_bytes, stream);
}

int gr_edge_list(const gr_graph* g, int32_t* eu, int32_t* ev, int32_t* edge_of_entry,
                 int64_t* n_edges, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!n_edges) return set_error(GR_EINVAL, "n_edges is NULL");
    *n_edges = 0;
    if (g->nnz == 0) return GR_OK;
    if (g->nnz % 2) return set_error(GR_ECSR, "odd nnz: graph not symmetric");
    if (!eu || !ev || !ws) return set_error(GR_EINVAL, "NULL eu, ev or workspace");
    Arena A(ws, ws_bytes);
    return edge_list(g, eu, ev, edge_of_entry, n_edges, A, S(stream));
}

static int check_rq_args(int64_t n, int64_t E, const int32_t* eu, const int32_t* ev,
                         const double* U, int32_t m, int32_t mode) {
    if (n < 0 || E < 0) return set_error(GR_EINVAL, "negative size");
    if (m < 1 || m > 64) return set_error(GR_EINVAL, "m must lie in [1, 64]");
    if (mode != GR_RQ_IDENTITY && mode != GR_RQ_DEGREE) return set_error(GR_EINVAL, "bad mode");
    if ((E > 0 && (!eu || !ev)) || (n > 0 && !U)) return set_error(GR_EINVAL, "NULL argument");
    return GR_OK;
}

int gr_rq_forward(int64_t n, int64_t n_edges, const int32_t* eu, const int32_t* ev,
                  const double* w_E, const double* U, int32_t m, int32_t mode, double* R,
                  double* den, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_rq_args(n, n_edges, eu, ev, U, m, mode));
    if (!R || !ws || (n_edges > 0 && !w_E)) return set_error(GR_EINVAL, "NULL argument");
    Arena A(ws, ws_bytes);
    return rq_forward(n, n_edges, eu, ev, w_E, U, m, mode, R, den, A, S(stream));
}

int gr_rq_forward_noalloc(int64_t n, int64_t n_edges, const int32_t* eu, const int32_t* ev,
                          const double* w_E, const double* U, int32_t m, int32_t mode, double* R,
                          double* den, void* stream) {
    clear_error();
    GR_TRY(check_rq_args(n, n_edges, eu, ev, U, m, mode));
    if (!R || (n_edges > 0 && !w_E)) return set_error(GR_EINVAL, "NULL argument");
    return rq_forward_noalloc(n, n_edges, eu, ev, w_E, U, m, mode, R, den, S(stream));
}

size_t gr_rq_forward_noalloc_scratch_bytes(void) { return rq_forward_scratch_capacity(); }

int gr_rq_backward(int64_t n_edges, const int32_t* eu, const int32_t* ev, const double* U,
                   int32_t m, int32_t mode, const double* R, const double* den, const double* gR,
                   double* gw_E, void* stream) {
    clear_error();
    GR_TRY(check_rq_args(0, n_edges, eu, ev, U, m, mode));
    if (n_edges > 0 && (!U || !R || !den || !gR || !gw_E)) return set_error(GR_EINVAL, "NULL argument");
    return rq_backward(n_edges, eu, ev, U, m, mode, R, den, gR, gw_E, S(stream));
}

int gr_expand_edge_weights(const int32_t* edge_of_entry, int64_t nnz, int64_t n_edges,
                           const float* w_E, float* w, void* stream) {
    clear_error();
    if (nnz < 0 || n_edges < 0) return set_error(GR_EINVAL, "negative size");
    if (nnz > 0 && (!edge_of_entry || !w_E || !w)) return set_error(GR_EINVAL, "NULL argument");
    return expand_weights(edge_of_entry, nnz, n_edges, w_E, w, S(stream));
}

int gr_smooth_vjp_workspace(int64_t n, int64_t nnz, int32_t K, int32_t dtype, int32_t sweeps,
                            int32_t store_states, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz < 0 || sweeps < 0) return set_error(GR_EINVAL, "negative size");
    GR_TRY(check_vec_args(K, dtype));
    *bytes = vjp_workspace(n, nnz, K, dtype, sweeps, store_states);
    return GR_OK;
}

int gr_smooth_vjp(const gr_graph* g, const int32_t* edge_of_entry, int64_t n_edges,
                  const int32_t* colours, int32_t n_colours, int32_t K, int32_t sweeps,
                  int32_t dtype, const void* X0, const float* G, float* gw_E, float* gX0,
                  int32_t store_states, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    GR_TRY(check_vec_args(K, dtype));
    if (sweeps < 0) return set_error(GR_EINVAL, "sweeps must be >= 0");
    if (n_edges != g->nnz / 2) return set_error(GR_EINVAL, "n_edges must be nnz / 2");
    if (g->n > 0 && (!colours || n_colours < 1)) return set_error(GR_EINVAL, "bad colouring");
    if (g->n > 0 && (!X0 || !G || !gX0 || !ws)) return set_error(GR_EINVAL, "NULL argument");
    if (g->nnz > 0 && (!edge_of_entry || !gw_E)) return set_error(GR_EINVAL, "NULL argument");
    GR_TRY(check_aligned(X0, "X0"));
    GR_TRY(check_aligned(G, "G"));
    GR_TRY(check_aligned(gX0, "gX0"));
    if (g->n == 0) return GR_OK;
    Arena A(ws, ws_bytes);
    return smooth_vjp(g, edge_of_entry, n_edges, colours, n_colours, K, sweeps, dtype, X0, G, gw_E,
                      gX0, store_states ? 1 : 0, A, S(stream));
}

int gr_eig_workspace(int64_t n, int32_t n_eig, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || n_eig < 1 || n_eig > 32) return set_error(GR_EINVAL, "bad size");
    *bytes = eig_workspace(n, n_eig);
    return GR_OK;
}

static int eigs_common(const gr_graph* g, const double* bdiag, int32_t n_eig, int32_t method, double tol,
                       int32_t max_iter, int32_t degree, uint64_t seed, double* eig, double* U,
                       gr_eig_report* report, void* ws, size_t ws_bytes, void* stream) {
    GR_TRY(check_graph_args(g));
    if (n_eig < 1 || n_eig > 32) return set_error(GR_EINVAL, "n_eig must lie in [1, 32]");
    if (method < GR_EIG_AUTO || method > GR_EIG_LOBPCG) return set_error(GR_EINVAL, "unknown method");
    if (!(tol > 0.0) || max_iter < 0 || degree < 1 || degree > 2000)
        return set_error(GR_EINVAL, "bad tol, max_iter or degree");
    if (!eig || !ws) return set_error(GR_EINVAL, "NULL argument");
    if (report) memset(report, 0, sizeof(*report));
    if (g->n < 2) {
        for (int i = 0; i < n_eig; ++i) eig[i] = NAN;
        if (U && g->n == 1) {  // all-ones bytes: NaN
            GR_HIP(hipMemsetAsync(U, 0xff, sizeof(double) * n_eig, S(stream)));
            GR_HIP(hipStreamSynchronize(S(stream)));
        }
        return GR_OK;
    }
    Arena A(ws, ws_bytes);
    return laplacian_eigs(g, bdiag, n_eig, method, tol, max_iter, degree, seed, eig, U, report, A,
                          S(stream));
}

int gr_laplacian_eigs(const gr_graph* g, int32_t n_eig, int32_t method, double tol,
                      int32_t max_iter, int32_t degree, uint64_t seed, double* eig,
                      gr_eig_report* report, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    return eigs_common(g, nullptr, n_eig, method, tol, max_iter, degree, seed, eig, nullptr, report,
                       ws, ws_bytes, stream);
}

int gr_laplacian_eigpairs(const gr_graph* g, int32_t n_eig, int32_t method, double tol,
                          int32_t max_iter, int32_t degree, uint64_t seed, double* eig, double* U,
                          gr_eig_report* report, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!U && g && g->n > 0) return set_error(GR_EINVAL, "U is NULL");
    return eigs_common(g, nullptr, n_eig, method, tol, max_iter, degree, seed, eig, U, report, ws,
                       ws_bytes, stream);
}

int gr_laplacian_geigpairs(const gr_graph* g, const double* bdiag, int32_t n_eig, int32_t method,
                           double tol, int32_t max_iter, int32_t degree, uint64_t seed,
                           double* eig, double* U, gr_eig_report* report, void* ws,
                           size_t ws_bytes, void* stream) {
    clear_error();
    if (!U && g && g->n > 0) return set_error(GR_EINVAL, "U is NULL");
    return eigs_common(g, bdiag, n_eig, method, tol, max_iter, degree, seed, eig, U, report, ws,
                       ws_bytes, stream);
}

int gr_jacobi_workspace(int64_t n, int32_t k, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || k < 1 || k > 64) return set_error(GR_EINVAL, "bad size");
    *bytes = jacobi_workspace(n, k);
    return GR_OK;
}

int gr_jacobi_filter(const gr_graph* g, int32_t k, double* Y, const double* lambda,
                     const double* bdiag, double theta, int32_t iters, void* ws, size_t ws_bytes,
                     void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (k < 1 || k > 64) return set_error(GR_EINVAL, "k must lie in [1, 64]");
    if (iters < 0 || !(theta > 0.0) || !isfinite(theta))
        return set_error(GR_EINVAL, "bad theta or iters");
    if (g->n == 0 || iters == 0) return GR_OK;
    if (!Y || !ws) return set_error(GR_EINVAL, "NULL Y or workspace");
    Arena A(ws, ws_bytes);
    return jacobi_filter(g, k, Y, lambda, bdiag, theta, iters, A, S(stream));
}

int gr_orthonormalize_workspace(int64_t n, int32_t k, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || k < 1 || k > 64) return set_error(GR_EINVAL, "bad size");
    *bytes = orthonormalize_workspace(n, k);
    return GR_OK;
}

int gr_orthonormalize(int64_t n, int32_t k, double* U, const double* bdiag, void* ws,
                      size_t ws_bytes, void* stream) {
    clear_error();
    if (n < 0 || k < 1 || k > 64) return set_error(GR_EINVAL, "bad size");
    if (n <= k) return set_error(GR_EINVAL, "need n > k (the constant takes one dimension)");
    if (!U || !ws) return set_error(GR_EINVAL, "NULL U or workspace");
    Arena A(ws, ws_bytes);
    return orthonormalize(n, k, U, bdiag, A, S(stream));
}

int gr_multilevel_workspace(int64_t n, int64_t nnz, int32_t k, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz < 0 || k < 1 || k > 32) return set_error(GR_EINVAL, "bad size");
    *bytes = multilevel_workspace(n, nnz, k);
    return GR_OK;
}

int gr_multilevel_eigs(const gr_graph* g, const gr_hierarchy* h, int32_t k, int32_t mode,
                       double theta, int32_t iters, double tol, int32_t max_iter, uint64_t seed,
                       double* eig, double* U, gr_eig_report* report, void* ws, size_t ws_bytes,
                       void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!h) return set_error(GR_EINVAL, "hierarchy is NULL");
    if (h->levels < 0 || h->levels > GR_MAX_LEVELS) return set_error(GR_EINVAL, "bad level count");
    if (h->n[0] != g->n) return set_error(GR_EINVAL, "h->n[0] must be the graph's node count");
    for (int l = 1; l <= h->levels; ++l) {
        if (h->n[l] < 1 || h->n[l] > h->n[l - 1] || h->nnz[l] < 0)
            return set_error(GR_EINVAL, "bad sizes at level %d", l);
        if (!h->maps || !h->row_ptr || (h->nnz[l] > 0 && (!h->col || !h->w)))
            return set_error(GR_EINVAL, "NULL hierarchy arrays");
    }
    if (k < 1 || k > 32) return set_error(GR_EINVAL, "k must lie in [1, 32]");
    if (mode != GR_RQ_IDENTITY && mode != GR_RQ_DEGREE) return set_error(GR_EINVAL, "bad mode");
    if (iters < 0 || !(theta > 0.0) || !isfinite(theta) || !(tol > 0.0) || max_iter < 0)
        return set_error(GR_EINVAL, "bad theta, iters, tol or max_iter");
    if (!eig || !U || !ws) return set_error(GR_EINVAL, "NULL argument");
    if (h->n[h->levels] <= k + 1)
        return set_error(GR_EINVAL, "the coarsest level needs more than k + 1 nodes");
    if (report) memset(report, 0, sizeof(*report));
    Arena A(ws, ws_bytes);
    return multilevel_eigs(g, h, k, mode, theta, iters, tol, max_iter, seed, eig, U, report, A,
                           S(stream));
}

static int check_sparsify_params(const gr_sparsify_params* p) {
    if (!p) return set_error(GR_EINVAL, "params is NULL");
    if (p->t < 1 || p->rounds < 0 || p->rounds > GR_SPARSIFY_MAX_ROUNDS || !(p->add_frac >= 0.0) ||
        !isfinite(p->add_frac) || !isfinite(p->lambda_target) || p->cg_max_iter < 0 ||
        !(p->cg_tol >= 0.0))
        return set_error(GR_EINVAL, "bad sparsification parameters");
    return GR_OK;
}

int gr_sparsify_workspace(int64_t n, int64_t nnz, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz < 0) return set_error(GR_EINVAL, "negative size");
    *bytes = sparsify_workspace(n, nnz);
    return GR_OK;
}

int gr_spanning_forest(const gr_graph* g, int32_t* in_tree, int64_t* n_tree, void* ws,
                       size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!n_tree) return set_error(GR_EINVAL, "n_tree is NULL");
    *n_tree = 0;
    if (g->nnz % 2) return set_error(GR_ECSR, "odd nnz: graph not symmetric");
    if (g->nnz == 0) return GR_OK;
    if (!in_tree || !ws) return set_error(GR_EINVAL, "NULL in_tree or workspace");
    hipStream_t st = S(stream);
    Arena A(ws, ws_bytes);
    const int64_t E0 = g->nnz / 2;
    int32_t* eu = A.take<int32_t>(E0 + 1);
    int32_t* ev = A.take<int32_t>(E0 + 1);
    int32_t* eoe = A.take<int32_t>(g->nnz + 1);
    if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (spanning forest)");
    int64_t E = 0;
    GR_TRY(edge_list(g, eu, ev, eoe, &E, A, st));
    return spanning_forest(g, eu, ev, eoe, in_tree, E, n_tree, A, st);
}

int gr_sparsify(const gr_graph* g, const gr_sparsify_params* p, int32_t* in_P, double* criticality,
                gr_sparsify_report* rep, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    GR_TRY(check_sparsify_params(p));
    if (!rep) return set_error(GR_EINVAL, "report is NULL");
    memset(rep, 0, sizeof(*rep));
    if (g->nnz % 2) return set_error(GR_ECSR, "odd nnz: graph not symmetric");
    if (g->nnz == 0) return GR_OK;
    if (!in_P || !ws) return set_error(GR_EINVAL, "NULL in_P or workspace");
    Arena A(ws, ws_bytes);
    return sparsify(g, p, in_P, criticality, rep, A, S(stream));
}

int gr_subgraph(const gr_graph* g, const int32_t* keep, int32_t* p_row_ptr, int32_t* p_col,
                float* p_w, int32_t* p_edge_of_entry, int32_t* p_eu, int32_t* p_ev, int64_t* p_nnz,
                int64_t* p_edges, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!p_nnz || !p_edges) return set_error(GR_EINVAL, "NULL size outputs");
    *p_nnz = *p_edges = 0;
    if (g->nnz % 2) return set_error(GR_ECSR, "odd nnz: graph not symmetric");
    if (!p_row_ptr || !ws || (g->nnz > 0 && (!keep || !p_col || !p_w)))
        return set_error(GR_EINVAL, "NULL argument");
    if ((p_eu == nullptr) != (p_ev == nullptr)) return set_error(GR_EINVAL, "p_eu and p_ev go together");
    hipStream_t st = S(stream);
    if (g->nnz == 0) {
        GR_TRY(fill_i32(p_row_ptr, 0, g->n + 1, st));
        return GR_OK;
    }
    Arena A(ws, ws_bytes);
    const int64_t E0 = g->nnz / 2;
    int32_t* eu = A.take<int32_t>(E0 + 1);
    int32_t* ev = A.take<int32_t>(E0 + 1);
    int32_t* eoe = A.take<int32_t>(g->nnz + 1);
    if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (subgraph)");
    int64_t E = 0;
    GR_TRY(edge_list(g, eu, ev, eoe, &E, A, st));
    return subgraph(g, eoe, keep, E, eu, ev, p_row_ptr, p_col, p_w, p_edge_of_entry, p_eu, p_ev,
                    p_nnz, p_edges, A, st);
}

// the flow's own buffers: one subgraph (CSR, edge list, entry -> edge),
// its flags and weights
static size_t flow_buffers(int64_t n, int64_t nnz) {
    const size_t N = (size_t)n + 1, M = (size_t)nnz + 1, E = M / 2 + 1;
    return 4 * N + 4 * M + 4 * M + 4 * M + 8 * E + 4 * E + 8 * E + 4 * E + 4 * N + 4 * M + 4 * M +
           32 * 256;
}

int gr_spectral_reduce_workspace(int64_t n, int64_t nnz, int32_t K, int32_t vec_dtype,
                                 size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz < 0) return set_error(GR_EINVAL, "negative size");
    GR_TRY(check_vec_args(K, vec_dtype));
    size_t inner = plan_bytes(n, nnz, K, vec_dtype);
    inner = std::max(inner, sparsify_workspace(n, nnz));
    inner = std::max(inner, sgd_workspace(n, nnz, nnz, nnz / 2));
    *bytes = flow_buffers(n, nnz) + inner + (4u << 20);
    return GR_OK;
}

int gr_spectral_reduce(const gr_graph* g, const gr_flow_params* p, gr_flow_result* res, void* ws,
                       size_t ws_bytes, void* stream) {
    clear_error();
    GR_TRY(check_graph_args(g));
    if (!p || !res || !ws) return set_error(GR_EINVAL, "NULL params, result or workspace");
    GR_TRY(check_sparsify_params(&p->phase_b));
    if (!(p->gamma_max > 0.0)) return set_error(GR_EINVAL, "gamma_max must be positive");
    const gr_sgd_params* sp = &p->scaling;
    if (sp->k_max < 1 || sp->k_max > GR_SGD_MAX_ITER || sp->t < 1 || !(sp->delta_bar > 0.0) ||
        !(sp->delta_bar <= 1.0))
        return set_error(GR_EINVAL, "bad scaling parameters");
    if (!res->agg || !res->s_row_ptr || (g->nnz > 0 && (!res->s_col || !res->s_w)))
        return set_error(GR_EINVAL, "NULL output");
    if (g->nnz % 2) return set_error(GR_ECSR, "odd nnz: graph not symmetric");
    memset(&res->sparsify, 0, sizeof(res->sparsify));
    memset(&res->scaling, 0, sizeof(res->scaling));
    res->n_s = res->nnz_s = 0;
    res->levels = 0;
    res->warnings = 0;
    hipStream_t st = S(stream);
    const int64_t n = g->n, nnz = g->nnz, E0 = nnz / 2;
    res->gamma = n > 0 ? (double)E0 / (double)n : 0.0;
    res->dense = res->gamma >= p->gamma_max ? 1 : 0;
    Arena F(ws, ws_bytes);
    // one subgraph's arrays, flags and weights; the rest is the inner workspace
    int32_t* Rrp = F.take<int32_t>(n + 1);   // R (sparse branch)
    int32_t* Rcol = F.take<int32_t>(nnz + 1);
    float* Rw = F.take<float>(nnz + 1);
    int32_t* keep = F.take<int32_t>(E0 + 1);
    int32_t* peu = F.take<int32_t>(E0 + 1);
    int32_t* pev = F.take<int32_t>(E0 + 1);
    int32_t* peoe = F.take<int32_t>(nnz + 1);
    double* wP = F.take<double>(E0 + 1);
    float* wPf = F.take<float>(E0 + 1);
    int32_t* Prp = F.take<int32_t>(n + 1);
    int32_t* Pcol = F.take<int32_t>(nnz + 1);
    float* Pw = F.take<float>(nnz + 1);
    if (F.overflow) return set_error(GR_ENOMEM, "workspace too small (flow buffers)");
    char* inner = (char*)ws + F.used;
    const size_t inner_bytes = ws_bytes - F.used;
    gr_params pa;
    copy_params(&p->phase_a, &pa);
    gr_result ra;
    memset(&ra, 0, sizeof(ra));
    // Phase B then Alg. 1 on graph h (g or R): the scaled sparsifier into
    // Prp/Pcol/Pw (float32 weights)
    auto phase_b = [&](const gr_graph* h, int64_t* pnnz_out) -> int {
        Arena A(inner, inner_bytes);
        GR_TRY(sparsify(h, &p->phase_b, keep, nullptr, &res->sparsify, A, st));
        int32_t* eu = A.take<int32_t>(h->nnz / 2 + 1);
        int32_t* ev = A.take<int32_t>(h->nnz / 2 + 1);
        int32_t* eoe = A.take<int32_t>(h->nnz + 1);
        if (A.overflow) return set_error(GR_ENOMEM, "workspace too small (flow sparsifier)");
        int64_t E = 0, pnnz = 0, pedges = 0;
        GR_TRY(edge_list(h, eu, ev, eoe, &E, A, st));
        GR_TRY(subgraph(h, eoe, keep, E, eu, ev, Prp, Pcol, Pw, peoe, peu, pev, &pnnz, &pedges, A,
                        st));
        gr_graph P{h->n, pnnz, Prp, Pcol, Pw};
        // w_P <- the subgraph's weights, one per P edge, then Alg. 1
        {
            Arena B(inner, inner_bytes);
            float* wEf = B.take<float>(pedges + 1);
            if (B.overflow) return set_error(GR_ENOMEM, "workspace too small (flow weights)");
            // the P edges' weights from their upper entries
            GR_TRY(edge_weights(&P, peoe, wEf, st));
            hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks_for(pedges, 256)), dim3(256), 0, st,
                               (const float*)wEf, pedges, wP);
            GR_LAUNCHED("flow weights f64");
        }
        {
            Arena B(inner, inner_bytes);
            GR_TRY(sgd_scale(h, &P, peoe, pedges, peu, pev, wP, &p->scaling, &res->scaling, B, st));
        }
        hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks_for(pedges, 256)), dim3(256), 0, st,
                           (const double*)wP, pedges, wPf);
        GR_LAUNCHED("flow scaled weights");
        GR_TRY(expand_weights(peoe, pnnz, pedges, wPf, Pw, st));
        *pnnz_out = pnnz;
        return GR_OK;
    };
    if (!res->dense) {
        // Phase A on g, into R; then Phase B and Alg. 1 on R
        ra.agg = res->agg;
        ra.c_row_ptr = Rrp;
        ra.c_col = Rcol;
        ra.c_w = Rw;
        GR_TRY(reduce_impl(g, &pa, &ra, nullptr, inner, inner_bytes, stream));
        gr_graph R{ra.n_coarse, ra.nnz_coarse, Rrp, Rcol, Rw};
        int64_t pnnz = 0;
        if (R.nnz > 0) {
            GR_TRY(phase_b(&R, &pnnz));
        } else {
            GR_TRY(fill_i32(Prp, 0, R.n + 1, st));
        }
        GR_HIP(hipMemcpyAsync(res->s_row_ptr, Prp, sizeof(int32_t) * (R.n + 1),
                              hipMemcpyDeviceToDevice, st));
        if (pnnz > 0) {
            GR_HIP(hipMemcpyAsync(res->s_col, Pcol, sizeof(int32_t) * pnnz, hipMemcpyDeviceToDevice, st));
            GR_HIP(hipMemcpyAsync(res->s_w, Pw, sizeof(float) * pnnz, hipMemcpyDeviceToDevice, st));
        }
        res->n_s = R.n;
        res->nnz_s = pnnz;
    } else {
        // Phase B and Alg. 1 on g, then Phase A on the scaled sparsifier
        int64_t pnnz = 0;
        GR_TRY(phase_b(g, &pnnz));
        gr_graph P{n, pnnz, Prp, Pcol, Pw};
        pa.colours = nullptr;  // a prescribed colouring belongs to g, not P
        pa.n_colours = 0;
        ra.agg = res->agg;
        ra.c_row_ptr = res->s_row_ptr;
        ra.c_col = res->s_col;
        ra.c_w = res->s_w;
        GR_TRY(reduce_impl(&P, &pa, &ra, nullptr, inner, inner_bytes, stream));
        res->n_s = ra.n_coarse;
        res->nnz_s = ra.nnz_coarse;
    }
    res->levels = ra.levels;
    res->warnings = ra.warnings;
    GR_HIP(hipStreamSynchronize(st));
    return GR_OK;
}

int gr_sgd_workspace(int64_t n, int64_t nnz_g, int64_t nnz_p, int64_t p_edges, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error(GR_EINVAL, "bytes is NULL");
    if (n < 0 || nnz_g < 0 || nnz_p < 0 || p_edges < 0) return set_error(GR_EINVAL, "negative size");
    *bytes = sgd_workspace(n, nnz_g, nnz_p, p_edges);
    return GR_OK;
}

int gr_sgd_scale(const gr_graph* G, const gr_graph* P, const int32_t* p_edge_of_entry,
                 int64_t p_edges, const int32_t* p_eu, const int32_t* p_ev, double* w_P,
                 const gr_sgd_params* params, gr_sgd_report* report, void* ws, size_t ws_bytes,
                 void* stream) {
    clear_error();
    GR_TRY(check_graph_args(G));
    if (!P) return set_error(GR_EINVAL, "P is NULL");
    if (P->n != G->n) return set_error(GR_EINVAL, "P must have the nodes of G");
    if (P->nnz < 0 || !P->row_ptr || (P->nnz > 0 && !P->col))
        return set_error(GR_EINVAL, "bad P arrays");
    if (!params || !report || !ws) return set_error(GR_EINVAL, "NULL argument");
    if (p_edges != P->nnz / 2) return set_error(GR_EINVAL, "p_edges must be nnz(P) / 2");
    if (p_edges > 0 && (!p_edge_of_entry || !p_eu || !p_ev || !w_P))
        return set_error(GR_EINVAL, "NULL P edge arrays");
    if (params->k_max < 1 || params->k_max > GR_SGD_MAX_ITER)
        return set_error(GR_EINVAL, "k_max must lie in [1, %d]", GR_SGD_MAX_ITER);
    if (params->t < 1) return set_error(GR_EINVAL, "t must be >= 1");
    if (!(params->delta_bar > 0.0 && params->delta_bar <= 1.0))
        return set_error(GR_EINVAL, "delta_bar must lie in (0, 1]");
    memset(report, 0, sizeof(*report));
    if (G->n == 0 || p_edges == 0) return GR_OK;
    Arena A(ws, ws_bytes);
    return sgd_scale(G, P, p_edge_of_entry, p_edges, p_eu, p_ev, w_P, params, report, A, S(stream));
}

}  // extern "C"
