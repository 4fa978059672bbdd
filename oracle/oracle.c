/*
 * Reference oracle for spectrum-preserving node aggregation (Phase A of
 * Zhao, Wang & Feng, "Nearly-Linear Time Spectral Graph Reduction for
 * Scalable Graph Partitioning and Data Visualization", Sec. 3.2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow FP64 restatement
 * of what the reduction computes, used to check the GPU library.  It runs
 * single-threaded by default; or_set_threads(t) lets the smoothing and the
 * affinity visit the nodes of one colour (resp. all nodes) on t OpenMP
 * threads.  Each node's arithmetic is the same sequence of operations in
 * either case and no node reads a value written in the same parallel loop
 * (a colour class has no inner edges), so the results are bit-identical
 * for every thread count.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or constant table
 * with the GPU library.
 *
 * Graph convention (Sec. 2.1, Eq. for A_G; Appendix A, Eq. for L_G): a
 * weighted undirected graph is stored as symmetric CSR adjacency, both
 * directions present with equal weights, columns strictly increasing per row,
 * no self-loops, weights positive and finite.  The Laplacian is L = D - A
 * with D(i,i) the weighted degree, so it is never stored.
 *
 * Every step follows the paper's order; where the paper is silent the
 * reading taken is stated at the step.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int g_threads = 1;

/* Threads of the node loops of or_smooth and or_affinity (default 1). */
void or_set_threads(int32_t t) { g_threads = t < 1 ? 1 : t; }
int32_t or_get_threads(void) { return g_threads; }

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ECSR -2
#define OR_ECOLOUR -3
#define OR_ENOMEM -4

/* ------------------------------------------------------------------ RNG */
/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the odd constant
 * 0x9E3779B97F4A7C15 and each output is the state passed through the
 * variant-13 64-bit finaliser (xor-shift 30, multiply, xor-shift 27,
 * multiply, xor-shift 31).  Output number i of the generator seeded with s
 * therefore depends on s + (i+1)*gamma only: a counter-based generator. */
uint64_t or_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ CSR */
/* Validates the adjacency convention above.  Returns OR_OK or OR_ECSR. */
int or_validate_csr(int64_t n, const int32_t *row_ptr, const int32_t *col,
                    const double *w)
{
    if (n < 0) return OR_EINVAL;
    if (row_ptr[0] != 0) return OR_ECSR;
    for (int64_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] < row_ptr[v]) return OR_ECSR;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t j = col[e];
            if (j < 0 || j >= n || j == v) return OR_ECSR;
            if (e > row_ptr[v] && col[e - 1] >= j) return OR_ECSR;
            if (!(w[e] > 0.0) || !isfinite(w[e])) return OR_ECSR;
        }
    }
    /* symmetry: entry (v,j) must have a partner (j,v) of equal weight */
    for (int64_t v = 0; v < n; ++v) {
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t j = col[e];
            int32_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1, f = -1;
            while (lo <= hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (col[mid] == v) { f = mid; break; }
                if (col[mid] < v) lo = mid + 1; else hi = mid - 1;
            }
            if (f < 0 || w[f] != w[e]) return OR_ECSR;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------ colouring */
/* Gauss-Seidel relaxation of L x = 0 (Sec. 3.2.1) needs an update order.
 * Reading taken: a multicolour order, colours 0..C-1 ascending in every
 * sweep, nodes of one colour mutually non-adjacent, so the result does not
 * depend on the order inside a colour.  When no colouring is prescribed the
 * colouring is sequential greedy (first fit) in decreasing priority: every
 * node takes the smallest colour absent among its neighbours of higher
 * priority, which are all coloured before it.  Priority is (h(v), v),
 * h(v) = splitmix64 output v for the colour seed, or (deg(v), h(v), v) in
 * largest-degree-first mode (the order of Welsh and Powell). */
typedef struct { uint64_t a, b, c; } or_prio;

static or_prio prio_of(const int32_t *row_ptr, int64_t v, uint64_t seed, int ldf)
{
    or_prio p;
    uint64_t h = or_splitmix64(seed, (uint64_t)v);
    p.a = ldf ? (uint64_t)(row_ptr[v + 1] - row_ptr[v]) : h;
    p.b = ldf ? h : 0;
    p.c = (uint64_t)v;
    return p;
}

static int prio_cmp_desc(const void *x, const void *y)
{
    const or_prio *p = (const or_prio *)x, *q = (const or_prio *)y;
    if (p->a != q->a) return p->a > q->a ? -1 : 1;
    if (p->b != q->b) return p->b > q->b ? -1 : 1;
    if (p->c != q->c) return p->c > q->c ? -1 : 1;
    return 0;
}

int or_colour_greedy(int64_t n, const int32_t *row_ptr, const int32_t *col,
                     uint64_t seed, int32_t largest_degree_first,
                     int32_t *colours, int32_t *n_colours)
{
    int32_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > maxdeg) maxdeg = row_ptr[v + 1] - row_ptr[v];
    or_prio *order = (or_prio *)malloc(sizeof(or_prio) * (size_t)(n > 0 ? n : 1));
    uint8_t *used = (uint8_t *)calloc((size_t)maxdeg + 2, 1);
    if (!order || !used) { free(order); free(used); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) {
        colours[v] = -1;
        order[v] = prio_of(row_ptr, v, seed, largest_degree_first);
    }
    qsort(order, (size_t)n, sizeof(or_prio), prio_cmp_desc);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = (int64_t)order[i].c;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t c = colours[col[e]];
            if (c >= 0 && c <= maxdeg) used[c] = 1;
        }
        int32_t c = 0;
        while (used[c]) ++c;
        colours[v] = c;
        if (c + 1 > nc) nc = c + 1;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t cc = colours[col[e]];
            if (cc >= 0 && cc <= maxdeg) used[cc] = 0;
        }
    }
    *n_colours = nc;
    free(order);
    free(used);
    return OR_OK;
}

/* A colouring is valid when every colour lies in [0, C) and no stored edge
 * joins two nodes of the same colour. */
int or_validate_colouring(int64_t n, const int32_t *row_ptr, const int32_t *col,
                          const int32_t *colours, int32_t n_colours)
{
    for (int64_t v = 0; v < n; ++v) {
        if (colours[v] < 0 || colours[v] >= n_colours) return OR_ECOLOUR;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (colours[col[e]] == colours[v]) return OR_ECOLOUR;
    }
    return OR_OK;
}

/* ------------------------------------------------------- test vectors */
/* K random test vectors orthogonal to the all-one vector (Sec. 3.2.1).
 * Entry (v,k) draws m = the top 24 bits of splitmix64 output v*K + k and
 * maps it to x0 = (2m + 1 - 2^24) / 2^24, a uniform value in (-1, 1) that is
 * exact in binary32.  Each column is then centred by subtracting its mean,
 * taken in FP64 in index order, which makes it orthogonal to 1. */
void or_init_vectors(int64_t n, int32_t K, uint64_t seed, double *X,
                     int32_t centre)
{
    for (int64_t v = 0; v < n; ++v)
        for (int32_t k = 0; k < K; ++k) {
            uint64_t r = or_splitmix64(seed, (uint64_t)v * (uint64_t)K + (uint64_t)k);
            int64_t m = (int64_t)(r >> 40);
            X[v * K + k] = (double)(2 * m + 1 - (1ll << 24)) / (double)(1ll << 24);
        }
    if (!centre || n == 0) return;
    for (int32_t k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t v = 0; v < n; ++v) s += X[v * K + k];
        double mean = s / (double)n;
        for (int64_t v = 0; v < n; ++v) X[v * K + k] -= mean;
    }
}

/* Round a double to the nearest bfloat16 value (ties to even), returned as a
 * double.  Used only to emulate bfloat16 storage of the test vectors. */
double or_round_bf16(double x)
{
    float f = (float)x; /* the stored value is first a binary32 result */
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* -------------------------------------------------------- smoothing */
/* Gauss-Seidel relaxation of L x = 0 for each of the K test vectors
 * (Sec. 3.2.1): visiting node v, the equation row
 *   d_v x_v - sum_j w_vj x_j = 0
 * is solved for x_v with the current neighbour values, i.e.
 *   x_v <- (sum_j w_vj x_j) / d_v.
 * One sweep visits colours 0..C-1 in order.  A node without edges (d_v = 0)
 * has no equation to relax and keeps its value.  When `bf16_store` is set
 * every stored value is rounded to bfloat16, the initial vectors included. */
int or_smooth(int64_t n, const int32_t *row_ptr, const int32_t *col,
              const double *w, const int32_t *colours, int32_t n_colours,
              int32_t K, int32_t sweeps, double *X, int32_t bf16_store)
{
    if (K <= 0 || sweeps < 0 || n_colours < 0) return OR_EINVAL;
    if (bf16_store)
        for (int64_t i = 0; i < n * K; ++i) X[i] = or_round_bf16(X[i]);
    int failed = 0;
    for (int32_t s = 0; s < sweeps; ++s)
        for (int32_t c = 0; c < n_colours; ++c) {
#pragma omp parallel num_threads(g_threads) reduction(|| : failed)
            {
                double *acc = (double *)malloc(sizeof(double) * (size_t)K);
                if (!acc) failed = 1;
#pragma omp for schedule(dynamic, 4096)
                for (int64_t v = 0; v < n; ++v) {
                    if (!acc || colours[v] != c) continue;
                    double d = 0.0;
                    for (int32_t k = 0; k < K; ++k) acc[k] = 0.0;
                    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                        d += w[e];
                        const double *xj = X + (int64_t)col[e] * K;
                        for (int32_t k = 0; k < K; ++k) acc[k] += w[e] * xj[k];
                    }
                    if (d > 0.0)
                        for (int32_t k = 0; k < K; ++k) {
                            double y = acc[k] / d;
                            X[v * K + k] = bf16_store ? or_round_bf16(y) : y;
                        }
                }
                free(acc);
            }
            if (failed) return OR_ENOMEM;
        }
    return OR_OK;
}

/* --------------------------------------------------------- affinity */
/* Spectral node affinity of neighbouring nodes p, q (Sec. 3.2.1, Eq. of
 * a_{p,q}):  a = (X_p, X_q)^2 / ((X_p, X_p)(X_q, X_q)) with
 * (X_p, X_q) = sum_k x_p^(k) x_q^(k).  The norm bars around the scalar
 * inner product are read as an absolute value.  A zero denominator gives 0,
 * and the value is clamped to at most 1 (Cauchy-Schwarz makes it <= 1 in
 * exact arithmetic).  One value per stored entry.  The algebraic distance
 * d = 1 - a (Sec. 3.2.2) is returned alongside when `d` is non-null. */
void or_affinity(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 int32_t K, const double *X, double *a, double *d)
{
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        const double *xv = X + v * K;
        double nv = 0.0;
        for (int32_t k = 0; k < K; ++k) nv += xv[k] * xv[k];
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const double *xj = X + (int64_t)col[e] * K;
            double nj = 0.0, c = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                nj += xj[k] * xj[k];
                c += xv[k] * xj[k];
            }
            double den = nv * nj;
            double r = den == 0.0 ? 0.0 : (c * c) / den;
            a[e] = r > 1.0 ? 1.0 : r;
            if (d) d[e] = 1.0 - a[e];
        }
    }
}

/* Strongest neighbour (Sec. 3.2.2: aggregation joins node pairs of high
 * affinity, i.e. of small algebraic distance).  best(v) minimises (d_vj, j)
 * over the neighbours of v, i.e. the smallest algebraic distance (largest
 * affinity) with ties to the smaller index; -1 without neighbours.  The
 * paper gives the criterion, not the rule that picks the partner: this rule
 * is a reading of it. */
void or_best(int64_t n, const int32_t *row_ptr, const int32_t *col,
             const double *d, int32_t *best)
{
    for (int64_t v = 0; v < n; ++v) {
        int32_t b = -1;
        double bd = 0.0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (b < 0 || d[e] < bd) { bd = d[e]; b = col[e]; } /* columns ascend: first min wins */
        best[v] = b;
    }
}

/* ------------------------------------------------------ aggregation */
/* Aggregation rule (reading of Sec. 3.2.2 with the reduction ratio of
 * Alg. 2), on algebraic distances d = 1 - a:
 *  1. F = the edges {v, best(v)}; a mutual pair is one edge.  F is a forest:
 *     around a pointer cycle of length >= 3 the edge keys would strictly
 *     decrease, which a total order forbids.
 *  2. Edges are ordered by the total order: smaller distance (larger
 *     affinity) first, then the smaller min(p,q), then the smaller max(p,q).
 *  3. If n - |F| >= target, every edge of F is accepted; otherwise only the
 *     first n - target edges in that order.  Each accepted forest edge
 *     joins two components, so exactly max(target, n - |F|) aggregates form.
 *  4. Aggregates are the connected components of the accepted edges,
 *     numbered 0, 1, ... in increasing order of their smallest member.
 * The distance of an edge is the value stored at entry (v, best(v)). */
typedef struct { double d; int32_t lo, hi; } or_fedge;

static int fedge_cmp(const void *x, const void *y)
{
    const or_fedge *p = (const or_fedge *)x, *q = (const or_fedge *)y;
    if (p->d != q->d) return p->d < q->d ? -1 : 1;
    if (p->lo != q->lo) return p->lo < q->lo ? -1 : 1;
    if (p->hi != q->hi) return p->hi < q->hi ? -1 : 1;
    return 0;
}

static int32_t uf_find(int32_t *par, int32_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

int or_aggregate(int64_t n, const int32_t *row_ptr, const int32_t *col,
                 const double *d, int64_t target, int32_t *best, int32_t *agg,
                 int64_t *n_coarse, int64_t *n_forest, int64_t *n_accepted)
{
    if (target < 1) target = 1;
    or_best(n, row_ptr, col, d, best);
    or_fedge *F = (or_fedge *)malloc(sizeof(or_fedge) * (size_t)(n > 0 ? n : 1));
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *minm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!F || !par || !minm) { free(F); free(par); free(minm); return OR_ENOMEM; }
    int64_t nf = 0;
    for (int64_t v = 0; v < n; ++v) {
        int32_t b = best[v];
        if (b < 0) continue;
        if (best[b] == v && b < v) continue; /* mutual pair: keep once */
        double dv = 2.0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col[e] == b) { dv = d[e]; break; }
        F[nf].d = dv;
        F[nf].lo = (int32_t)(v < b ? v : b);
        F[nf].hi = (int32_t)(v < b ? b : v);
        ++nf;
    }
    int64_t m = nf;
    if (n - nf < target) {
        m = n - target;
        if (m < 0) m = 0;
        qsort(F, (size_t)nf, sizeof(or_fedge), fedge_cmp);
    }
    for (int64_t v = 0; v < n; ++v) par[v] = (int32_t)v;
    for (int64_t t = 0; t < m; ++t) {
        int32_t x = uf_find(par, F[t].lo), y = uf_find(par, F[t].hi);
        if (x != y) par[x < y ? y : x] = x < y ? x : y;
    }
    /* components numbered by smallest member: scanning v upward, the first
     * member met of each component is its smallest */
    for (int64_t v = 0; v < n; ++v) minm[v] = -1;
    int64_t nc = 0;
    for (int64_t v = 0; v < n; ++v) {
        int32_t r = uf_find(par, (int32_t)v);
        if (minm[r] < 0) minm[r] = (int32_t)nc++;
        agg[v] = minm[r];
    }
    *n_coarse = nc;
    if (n_forest) *n_forest = nf;
    if (n_accepted) *n_accepted = m;
    free(F);
    free(par);
    free(minm);
    return OR_OK;
}

/* -------------------------------------------------------- Galerkin */
static int int_cmp(const void *x, const void *y)
{
    int32_t p = *(const int32_t *)x, q = *(const int32_t *)y;
    return (p > q) - (p < q);
}

/* Reduced Laplacian L_R = H_G^R L_G H_R^G (Sec. 3.2.2) with H_R^G = P, the
 * 0/1 node-to-aggregate matrix, and H_G^R = P^T.  For a Laplacian this is
 * again a Laplacian: its off-diagonal weights are
 *   W[I,J] = sum of w_vj over stored (v,j) with agg(v) = I, agg(j) = J, I != J,
 * while edges inside an aggregate cancel against the diagonal.  Output is
 * CSR with rows and columns ascending and FP64 weights, (I, J) and (J, I)
 * bitwise equal (each computed once, as the upper one).  `c_row_ptr` has
 * n_c + 1 entries; `c_col`/`c_w` must hold nnz entries (an upper bound). */
int or_galerkin(int64_t n, const int32_t *row_ptr, const int32_t *col,
                const double *w, const int32_t *agg, int64_t n_c,
                int32_t *c_row_ptr, int32_t *c_col, double *c_w,
                int64_t *nnz_c)
{
    int32_t *cnt = (int32_t *)calloc((size_t)n_c + 1, sizeof(int32_t));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)calloc((size_t)(n_c > 0 ? n_c : 1), sizeof(double));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
    if (!cnt || !members || !acc || !mark || !touched) {
        free(cnt); free(members); free(acc); free(mark); free(touched);
        return OR_ENOMEM;
    }
    for (int64_t v = 0; v < n; ++v) {
        if (agg[v] < 0 || agg[v] >= n_c) {
            free(cnt); free(members); free(acc); free(mark); free(touched);
            return OR_EINVAL;
        }
        cnt[agg[v] + 1]++;
    }
    for (int64_t I = 0; I < n_c; ++I) cnt[I + 1] += cnt[I];
    {
        int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
        if (!pos) { free(cnt); free(members); free(acc); free(mark); free(touched); return OR_ENOMEM; }
        for (int64_t I = 0; I < n_c; ++I) pos[I] = cnt[I];
        for (int64_t v = 0; v < n; ++v) members[pos[agg[v]]++] = (int32_t)v;
        free(pos);
    }
    for (int64_t I = 0; I < n_c; ++I) mark[I] = -1;
    int64_t out = 0;
    c_row_ptr[0] = 0;
    for (int64_t I = 0; I < n_c; ++I) {
        int32_t nt = 0;
        for (int32_t t = cnt[I]; t < cnt[I + 1]; ++t) {
            int32_t v = members[t];
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t J = agg[col[e]];
                if (J == I) continue;
                if (mark[J] != I) { mark[J] = (int32_t)I; acc[J] = 0.0; touched[nt++] = J; }
                acc[J] += w[e];
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), int_cmp); /* ascending columns */
        for (int32_t i = 0; i < nt; ++i) {
            c_col[out] = touched[i];
            c_w[out] = acc[touched[i]];
            ++out;
        }
        c_row_ptr[I + 1] = (int32_t)out;
    }
    /* L_R is symmetric: the weight of (I, J), I > J, is by definition the
     * same sum as that of (J, I); store the upper one's value in both so the
     * two directions carry identical bits */
    for (int64_t I = 0; I < n_c; ++I)
        for (int32_t t = c_row_ptr[I]; t < c_row_ptr[I + 1]; ++t) {
            int32_t J = c_col[t];
            if (J >= I) break;
            int32_t lo = c_row_ptr[J], hi = c_row_ptr[J + 1] - 1;
            while (lo <= hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (c_col[mid] == I) { c_w[t] = c_w[mid]; break; }
                if (c_col[mid] < I) lo = mid + 1; else hi = mid - 1;
            }
        }
    *nnz_c = out;
    free(cnt); free(members); free(acc); free(mark); free(touched);
    return OR_OK;
}

/* ------------------------------------------------------- edge numbering */
/* Undirected edge e = (p, q), p < q, is numbered by the position of the
 * upper entry (p, q) among all upper entries in CSR order.  Both stored
 * entries (p, q) and (q, p) map to e.  Returns the number of edges. */
int64_t or_edge_index(int64_t n, const int32_t *row_ptr, const int32_t *col,
                      int32_t *edge_of_entry, int32_t *eu, int32_t *ev)
{
    int64_t E = 0;
    for (int64_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col[e] > v) {
                edge_of_entry[e] = (int32_t)E;
                if (eu) eu[E] = (int32_t)v;
                if (ev) ev[E] = col[e];
                ++E;
            }
    for (int64_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col[e] < v) {
                int32_t j = col[e];
                for (int32_t f = row_ptr[j]; f < row_ptr[j + 1]; ++f)
                    if (col[f] == v) { edge_of_entry[e] = edge_of_entry[f]; break; }
            }
    return E;
}

/* -------------------------------------------- adjoint of the smoothing */
/* Reverse-mode derivative of the Gauss-Seidel smoothing with respect to the
 * undirected edge weights w_E and the initial vectors X0 (a differentiation
 * added on top of the paper's smoothing, which serves the edge-weight
 * scaling of Sec. 3.3.4).
 *
 * A colour step maps row i of colour c (d_i > 0) to x_i' = N_i / d_i with
 * N_i = sum_j w_ij x_j and d_i = sum_j w_ij; other rows are unchanged.  Its
 * partial derivatives are  dx_i'/dw_ij = (x_j - x_i') / d_i  and
 * dx_i'/dx_j = w_ij / d_i, while x_i' does not depend on the old x_i.  The
 * adjoint of one step therefore, with g = the adjoint of x_i':
 *   wbar_ij += sum_k g_k (x_jk - x'_ik) / d_i,
 *   xbar_j  += (w_ij / d_i) g   for each neighbour j,
 *   xbar_i   = 0.
 * Steps are undone in reverse: sweeps S..1, colours C-1..0.  States are
 * recomputed from stored sweep boundaries.  G is the cotangent of the final
 * vectors; gw_E and gX0 receive the gradients. */
int or_smooth_vjp(int64_t n, const int32_t *row_ptr, const int32_t *col,
                  const int32_t *edge_of_entry, int64_t E, const double *w_E,
                  const int32_t *colours, int32_t C, int32_t K, int32_t S,
                  const double *X0, const double *G, double *gw_E, double *gX0)
{
    size_t nk = (size_t)n * (size_t)K;
    double *bound = (double *)malloc(sizeof(double) * nk * (size_t)(S + 1));
    double *steps = (double *)malloc(sizeof(double) * nk * (size_t)(C > 0 ? C : 1));
    double *deg = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!bound || !steps || !deg) { free(bound); free(steps); free(deg); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) {
        double d = 0.0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) d += w_E[edge_of_entry[e]];
        deg[v] = d;
    }
    /* forward pass; one colour step applied to state Y in place */
#define OR_STEP(Y, c)                                                          \
    for (int64_t v = 0; v < n; ++v) {                                          \
        if (colours[v] != (c) || !(deg[v] > 0.0)) continue;                    \
        for (int32_t k = 0; k < K; ++k) {                                      \
            double acc = 0.0;                                                  \
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)              \
                acc += w_E[edge_of_entry[e]] * (Y)[(int64_t)col[e] * K + k];   \
            (Y)[v * K + k] = acc / deg[v];                                     \
        }                                                                      \
    }
    memcpy(bound, X0, sizeof(double) * nk);
    for (int32_t s = 0; s < S; ++s) {
        double *Y = bound + nk * (size_t)(s + 1);
        memcpy(Y, bound + nk * (size_t)s, sizeof(double) * nk);
        for (int32_t c = 0; c < C; ++c) { OR_STEP(Y, c) }
    }
    for (int64_t e = 0; e < E; ++e) gw_E[e] = 0.0;
    memcpy(gX0, G, sizeof(double) * nk); /* running adjoint of the state */
    for (int32_t s = S - 1; s >= 0; --s) {
        /* states after each colour step of sweep s */
        for (int32_t c = 0; c < C; ++c) {
            double *Y = steps + nk * (size_t)c;
            memcpy(Y, c == 0 ? bound + nk * (size_t)s : steps + nk * (size_t)(c - 1),
                   sizeof(double) * nk);
            OR_STEP(Y, c)
        }
        for (int32_t c = C - 1; c >= 0; --c) {
            const double *Y = steps + nk * (size_t)c;
            for (int64_t i = 0; i < n; ++i) {
                if (colours[i] != c || !(deg[i] > 0.0)) continue;
                double *g = gX0 + i * K;
                for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    int64_t j = col[e];
                    double dot = 0.0;
                    for (int32_t k = 0; k < K; ++k)
                        dot += g[k] * (Y[j * K + k] - Y[i * K + k]);
                    gw_E[edge_of_entry[e]] += dot / deg[i];
                    double f = w_E[edge_of_entry[e]] / deg[i];
                    for (int32_t k = 0; k < K; ++k) gX0[j * K + k] += f * g[k];
                }
                for (int32_t k = 0; k < K; ++k) g[k] = 0.0;
            }
        }
    }
#undef OR_STEP
    free(bound);
    free(steps);
    free(deg);
    return OR_OK;
}
