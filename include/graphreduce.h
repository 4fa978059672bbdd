/*
 * graphreduce.h — C ABI of libgraphreduce, an MI355X (gfx950) implementation
 * of the spectrum-preserving node aggregation of Zhao, Wang & Feng,
 * "Nearly-Linear Time Spectral Graph Reduction for Scalable Graph
 * Partitioning and Data Visualization" (arXiv 1812.08942), Phase A
 * (Sec. 3.2), with the edge-weight derivatives that serve the constrained
 * SGD edge scaling of Sec. 3.3.4 (Alg. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graphs.  A weighted undirected graph G = (V, E, w) is passed as symmetric
 *   CSR adjacency (the paper's A_G, Sec. 2.1): `row_ptr` int32[n+1] with
 *   row_ptr[0] = 0, `col` int32[nnz], `w` float32[nnz].  Both directions of
 *   every edge are stored with bit-identical weights; columns strictly
 *   increase within a row; no self-loops; weights are positive and finite;
 *   nnz < 2^31.  The Laplacian L = D - A (D = weighted degrees) is implicit.
 * Memory.  Every array argument is a DEVICE pointer owned by the caller
 *   unless it is documented as host.  The library never allocates device
 *   memory: scratch comes from the caller's workspace `ws` of `ws_bytes`
 *   bytes (size it with gr_workspace_size), except for the one fixed static
 *   array that gr_rq_forward_noalloc uses instead of a workspace.  Outputs
 *   have caller-allocated upper-bound sizes.
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Work is
 *   enqueued on it; an entry point returns only after the device-to-host
 *   size reads it documents, otherwise asynchronously.
 * Errors.  Every entry point returns GR_OK (0) or a negative GR_E* code and
 *   sets a thread-local message readable with gr_last_error().  On error,
 *   outputs are unspecified.  No C++ exception crosses the ABI.
 * Determinism.  Identical inputs, parameters and seeds give bit-identical
 *   outputs: no floating-point atomics are used anywhere.
 * Vector storage.  Test-vector matrices X are node-major [n][K]: float32
 *   (GR_F32, K a multiple of 4) or bfloat16 (GR_BF16, K a multiple of 8,
 *   round-to-nearest-even on store); arithmetic is float32 in both cases.
 *   1 <= K <= 64.
 */
#ifndef GRAPHREDUCE_H
#define GRAPHREDUCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GR_OK 0
#define GR_EINVAL (-1)   /* bad argument (null pointer, size, parameter)    */
#define GR_ECSR (-2)     /* graph violates the CSR convention above         */
#define GR_ECOLOUR (-3)  /* colouring invalid (edge inside one colour)      */
#define GR_ENOMEM (-4)   /* workspace or output buffer too small            */
#define GR_EHIP (-5)     /* a HIP runtime call failed (message has details) */
#define GR_EUNSUP (-6)   /* unsupported K / dtype combination               */

#define GR_F32 0
#define GR_BF16 1

/* gr_params.flags */
#define GR_VALIDATE 1u     /* check the CSR convention on the device first     */
#define GR_COLOUR_LDF 2u   /* greedy colouring in largest-degree-first order   */

/* gr_result.warnings */
#define GR_WNOPROGRESS 1u  /* a level could not shrink the graph; stopped early */

typedef struct gr_graph {
    int64_t n;              /* nodes                                */
    int64_t nnz;            /* stored entries = 2 |E|               */
    const int32_t* row_ptr; /* device int32[n+1]                    */
    const int32_t* col;     /* device int32[nnz]                    */
    const float* w;         /* device float32[nnz]                  */
} gr_graph;

typedef struct gr_params {
    int32_t K;              /* test vectors (Sec. 3.2.1: K random vectors)   */
    int32_t sweeps;         /* Gauss-Seidel sweeps ("a few", Sec. 3.2.1)     */
    double ratio;           /* reduction ratio psi = |V| / |V_S| >= 1 (Alg. 2) */
    uint64_t vec_seed;      /* seed of the test vectors; level l uses
                               splitmix64 output l of this seed             */
    uint64_t colour_seed;   /* seed of the greedy colouring priorities,
                               per level as above                           */
    int32_t vec_dtype;      /* GR_F32 or GR_BF16                              */
    const int32_t* colours; /* optional device int32[n] colouring of level 0;
                               NULL = greedy colouring                       */
    int32_t n_colours;      /* number of colours in `colours`               */
    int32_t max_levels;     /* 0 = no limit (stops at the target or when a
                               level makes no progress)                     */
    uint32_t flags;         /* GR_VALIDATE | GR_COLOUR_LDF                    */
} gr_params;

typedef struct gr_result {
    int32_t* agg;           /* device int32[n]: final aggregate of each node   */
    int32_t* c_row_ptr;     /* device int32[n+1] (upper bound): coarse CSR    */
    int32_t* c_col;         /* device int32[nnz] (upper bound)                */
    float* c_w;             /* device float32[nnz] (upper bound)              */
    int64_t n_coarse;       /* out: coarse nodes                              */
    int64_t nnz_coarse;     /* out: coarse stored entries                     */
    int32_t levels;         /* out: levels run                                */
    uint32_t warnings;      /* out: GR_W* bits                                */
    int64_t level_n[32];    /* out: node count entering each level           */
    int64_t level_nnz[32];  /* out: stored entries entering each level       */
    int32_t level_colours[32]; /* out: colours used on each level            */
} gr_result;

/* gr_rq_forward / gr_rq_backward: the quotient's denominator matrix B */
#define GR_RQ_IDENTITY 0   /* B = I      (ratio cut, Alg. 4)       */
#define GR_RQ_DEGREE 1     /* B = D(w)   (normalized cut, Alg. 4)  */

/* Phases reported by the profiler (indices into gr_profile arrays). */
#define GR_PHASE_COLOUR 0
#define GR_PHASE_RELABEL 1
#define GR_PHASE_INIT 2
#define GR_PHASE_SMOOTH 3    /* one record per level: its Gauss-Seidel steps */
#define GR_PHASE_AFFINITY 4
#define GR_PHASE_AGGREGATE 5
#define GR_PHASE_GALERKIN 6
#define GR_PHASE_OTHER 7

typedef struct gr_profile {
    double phase_ms[8];       /* summed HIP-event time of the phase's records  */
    double phase_max_ms[8];   /* longest single record                          */
    double phase_bytes[8];    /* algorithmic (compulsory) bytes of the records  */
    int64_t phase_launches[8];/* records (for SMOOTH: colour steps)            */
    int64_t records;
} gr_profile;

/* Library version (major*10000 + minor*100 + patch) and status strings. */
int gr_version(void);
const char* gr_status_string(int status);
/* Message of the last failing call on this thread ("" if none). */
const char* gr_last_error(void);

/*
 * gr_workspace_size — bytes of device workspace that every entry point of
 * this header needs for a graph of n nodes and nnz stored entries, K test
 * vectors of type `vec_dtype`.  Host outputs: *bytes.  GR_EINVAL for
 * negative sizes, GR_EUNSUP for an unsupported K/dtype.
 */
int gr_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t vec_dtype, size_t* bytes);

/*
 * gr_reduce — the whole Phase A node reduction (Sec. 3.2) run level by level
 * until at most T = ceil(n / ratio) nodes remain (the user-defined ratio psi
 * of Alg. 2) or a level cannot shrink the graph.  Each level: colouring
 * (prescribed on level 0 if given, else greedy), K centred random test
 * vectors, `sweeps` multicolour Gauss-Seidel sweeps on L x = 0, per-edge
 * affinity a_pq (Eq. of a_{p,q}), strongest-affinity aggregation, and the
 * coarse Laplacian L_R = H_G^R L_G H_R^G with H_R^G = P (0/1 node-to-
 * aggregate map) and H_G^R = P^T, formed by a sort and a segmented sum.
 * Aggregate ids are numbered by each aggregate's smallest fine node.
 * Outputs: res->agg (composed map), res->c_* (final coarse CSR, rows and
 * columns ascending), the counts in *res.  Synchronises with the host a few
 * times per level to read sizes.
 */
int gr_reduce(const gr_graph* g, const gr_params* p, gr_result* res, void* ws,
              size_t ws_bytes, void* stream);

/*
 * gr_profile_start / gr_profile_stop — measurement aid.  After start, calls
 * made on this thread record HIP events on their stream around each phase
 * of gr_reduce (the Gauss-Seidel colour steps of a level, in gr_reduce and
 * gr_smooth, as one bracket with their count), with the compulsory bytes
 * each one moves.  stop synchronises on the
 * recorded events, fills *out (HOST) and turns recording off.
 */
int gr_profile_start(void);
int gr_profile_stop(gr_profile* out);

/* ---------------------------------------------------------------------
 * Building blocks.  gr_reduce is made of these; they are exported for
 * testing and for callers that want one step.
 * ------------------------------------------------------------------- */

/* gr_validate — checks the CSR convention on the device (GR_ECSR if it is
 * violated).  Synchronises. */
int gr_validate(const gr_graph* g, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_colour_greedy — greedy colouring (the multicolour order that makes
 * Gauss-Seidel on L x = 0 reproducible, Sec. 3.2.1): the result of visiting
 * the nodes in decreasing priority and giving each the smallest colour
 * absent among its already coloured (higher-priority) neighbours.  Priority
 * is (h(v), v), h(v) = splitmix64 output v of `seed` — or (deg(v), h(v), v)
 * when `largest_degree_first`.  The device computes it without rounds: the
 * nodes are sorted by priority and each waits for its higher-priority
 * neighbours' colours (a bounded wait; GR_EHIP if it ever runs out).
 * Output: colours int32[n] (device), *n_colours (HOST).  Synchronises.
 * The waiting kernel is a cooperative launch (all its workgroups resident);
 * with the environment variable GR_COLOUR_PLAIN_LAUNCH=1 it is an ordinary
 * launch of the same grid instead, for profilers that fault on cooperative
 * launches (same result; on a busy device the bounded waits may then fail).
 */
int gr_colour_greedy(const gr_graph* g, uint64_t seed, int32_t largest_degree_first,
                     int32_t* colours, int32_t* n_colours, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * gr_init_vectors — K random test vectors orthogonal to the all-one vector
 * (Sec. 3.2.1).  Entry (v,k): m = top 24 bits of splitmix64 output v*K + k of
 * `seed`, x0 = (2m + 1 - 2^24) / 2^24 in (-1, 1); each column is then centred
 * by its FP64 mean and stored as `dtype`.  X: device [n][K].
 */
int gr_init_vectors(int64_t n, int32_t K, uint64_t seed, int32_t dtype, void* X,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * gr_smooth — `sweeps` Gauss-Seidel relaxations of L x = 0 applied to all K
 * columns of X in place (Sec. 3.2.1): within a sweep, colours 0..C-1 in
 * order; each node v of the current colour with d_v > 0 becomes
 * sum_j w_vj x_j / d_v.  `colours` is a valid colouring (device int32[n]);
 * GR_ECOLOUR if a colour is out of range.  X: device [n][K] of `dtype`.
 * Internally relabels the graph colour-major once per call.
 */
int gr_smooth(const gr_graph* g, const int32_t* colours, int32_t n_colours, int32_t K,
              int32_t sweeps, int32_t dtype, void* X, void* ws, size_t ws_bytes,
              void* stream);

/*
 * gr_affinity — spectral node affinity of every stored entry (Sec. 3.2.1,
 * Eq. of a_{p,q}): a = (X_p . X_q)^2 / ((X_p . X_p)(X_q . X_q)), 0 when the
 * denominator is 0, at most 1; and the algebraic distance d = 1 - a
 * (Sec. 3.2.2), evaluated without cancellation as |u-w|^2 |u+w|^2 / 4 on the
 * normalised rows u, w so that it stays accurate where a rounds to 1 in
 * float32.  Both are bit-symmetric: value(p,q) == value(q,p).  Outputs:
 * a float32[nnz] and dist float32[nnz] (either may be NULL), best int32[n]
 * = the neighbour minimising (d, index) — the largest affinity, ties to the
 * smaller index — or -1 without neighbours, dbest float32[n] its distance
 * (may be NULL).  Synchronises once (to size the list of long rows).
 */
int gr_affinity(const gr_graph* g, int32_t K, int32_t dtype, const void* X, float* a,
                float* dist, int32_t* best, float* dbest, void* ws, size_t ws_bytes,
                void* stream);

/*
 * gr_aggregate — strongest-affinity aggregation (Sec. 3.2.2: nodes with large
 * affinity, i.e. small algebraic distance, are aggregated).  From `dist`
 * (float32[nnz], symmetric) the forest F = {v, best(v)}, best(v) = argmin
 * (d, index), is formed; if n - |F| >= target all of F is accepted,
 * otherwise its first n - target edges in the order (smaller distance,
 * smaller min endpoint, smaller max endpoint).  Aggregates are connected
 * components of the accepted edges numbered by smallest member.  Outputs:
 * agg int32[n] (device), *n_coarse (HOST).  Synchronises.
 */
int gr_aggregate(const gr_graph* g, const float* dist, int64_t target, int32_t* agg,
                 int64_t* n_coarse, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_galerkin — coarse Laplacian L_R = P^T L_G P (Sec. 3.2.2) for the
 * aggregate map `agg` (int32[n], values in [0, n_coarse)).  Output CSR:
 * c_row_ptr int32[n_coarse+1], c_col int32[<= nnz], c_w float32[<= nnz]
 * with W[I,J] = sum of w_vj over stored (v,j), agg(v)=I != agg(j)=J, summed
 * in float32 in a fixed order.  *nnz_coarse is HOST.  Synchronises.
 */
int gr_galerkin(const gr_graph* g, const int32_t* agg, int64_t n_coarse, int32_t* c_row_ptr,
                int32_t* c_col, float* c_w, int64_t* nnz_coarse, void* ws, size_t ws_bytes,
                void* stream);

/*
 * gr_restrict_mean — the reduced data set of the multilevel data
 * visualisation (Alg. 6): F_R = H_G^R F, with the G-to-R mapping read as
 * the averaging restriction for data.  Row I of F_R is the mean of the rows
 * of F over the nodes v with agg[v] = I.
 *   agg  int32[n] (device): the aggregate of every node, in [0, n_coarse);
 *        every aggregate must have a member.
 *   F    float32[n][d] (device, row-major): one data point per node.
 *   F_R  float32[n_coarse][d] (device, caller-owned): the output.
 * Sums are taken in FP64, with the members of an aggregate in node order
 * and in fixed pieces of 256; each row is divided by the member count and
 * rounded once to float32.  Deterministic.  Errors: GR_EINVAL for bad
 * sizes, an id out of range or an empty aggregate (F_R is then
 * unspecified).  Workspace: gr_restrict_workspace.  Synchronises (reads
 * the validity flags and the piece count).
 */
int gr_restrict_workspace(int64_t n, int64_t n_coarse, int32_t d, size_t* bytes);
int gr_restrict_mean(const int32_t* agg, int64_t n, int64_t n_coarse, int32_t d, const float* F,
                     float* F_R, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Edge-weight derivatives (serving the SGD edge scaling of Sec. 3.3.4).
 * Edge weights are one FP64 value per undirected edge: edge e = (p, q),
 * p < q, numbered in CSR order of the upper entries.
 * ------------------------------------------------------------------- */

/*
 * gr_edge_list — the undirected edges of g: eu/ev int32[E] with eu < ev,
 * E = nnz / 2, and edge_of_entry int32[nnz] (may be NULL) mapping each
 * stored entry (both directions) to its edge.  *n_edges is HOST.
 * Synchronises.
 */
int gr_edge_list(const gr_graph* g, int32_t* eu, int32_t* ev, int32_t* edge_of_entry,
                 int64_t* n_edges, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_rq_forward — FP64 Rayleigh quotients of the m columns of U (node-major
 * double[n][m], 1 <= m <= 64) on the graph with edge weights w_E double[E]:
 *   R_i = u_i^T L(w) u_i / u_i^T B u_i,  u^T L(w) u = sum_e w_e (u_p - u_q)^2,
 * with B = I (GR_RQ_IDENTITY) or B = D(w) (GR_RQ_DEGREE) — the quotients of
 * the eigenproblems L u = lambda B u of Alg. 4/5, whose values at the
 * eigenvectors are the eigenvalues.  Outputs R double[m] and the
 * denominators den double[m] (needed by the backward), device.  Sums are
 * tree reductions of fixed shape (deterministic).
 */
int gr_rq_forward(int64_t n, int64_t n_edges, const int32_t* eu, const int32_t* ev,
                  const double* w_E, const double* U, int32_t m, int32_t mode, double* R,
                  double* den, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_rq_forward_noalloc — gr_rq_forward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same arguments minus ws/ws_bytes,
 * the same kernels and the same bits.  Its scratch (three arrays of 512
 * per-block partial sums per column) lives in a library-owned static
 * device array of gr_rq_forward_noalloc_scratch_bytes() = 786,432 bytes
 * per GPU (room for m = 64, so every valid m fits; GR_EINVAL if a call
 * ever needed more), held until the process ends.  Every call rewrites
 * what it reads of the array, so nothing carries over between calls, but
 * calls that overlap on one GPU (two streams, two threads) share it and
 * race: serialise them.  Allocates nothing; R and den as in gr_rq_forward.
 */
int gr_rq_forward_noalloc(int64_t n, int64_t n_edges, const int32_t* eu, const int32_t* ev,
                          const double* w_E, const double* U, int32_t m, int32_t mode, double* R,
                          double* den, void* stream);
size_t gr_rq_forward_noalloc_scratch_bytes(void);

/*
 * gr_rq_backward — edge-weight gradient of sum_i gR_i R_i:
 *   gw_e = sum_i gR_i [ (u_pi - u_qi)^2 - [B = D] R_i (u_pi^2 + u_qi^2) ] / den_i.
 * At an eigenvector u_i with B = I this is the first-order sensitivity
 * d(lambda_i)/dw_e = (e_pq^T u_i)^2 / u_i^T u_i of Sec. 3.3.3 (the paper's
 * formula for the generalised problem carries the factor -lambda_n instead,
 * for weights of the denominator Laplacian).  U is held fixed (at an
 * eigenvector the quotient is stationary in u).  Output gw_E double[E].
 */
int gr_rq_backward(int64_t n_edges, const int32_t* eu, const int32_t* ev, const double* U,
                   int32_t m, int32_t mode, const double* R, const double* den, const double* gR,
                   double* gw_E, void* stream);

/*
 * gr_expand_edge_weights — entry weights from edge weights:
 * w[e] = w_E[edge_of_entry[e]] for the nnz stored entries (float32, device).
 * GR_EINVAL if an id lies outside [0, n_edges) (such entries are never
 * dereferenced).  Synchronises.
 */
int gr_expand_edge_weights(const int32_t* edge_of_entry, int64_t nnz, int64_t n_edges,
                           const float* w_E, float* w, void* stream);

/*
 * gr_smooth_vjp — reverse-mode derivative of `sweeps` Gauss-Seidel sweeps
 * (the smoothing of Sec. 3.2.1 as computed by gr_smooth) with respect to the
 * undirected edge weights and the initial vectors.  The graph's entry
 * weights must be w_E[edge_of_entry[e]] (see gr_edge_list).  Inputs: X0
 * [n][K] of `dtype` (the initial vectors), G float32 [n][K] (the cotangent of
 * the smoothed vectors).  Outputs: gw_E float32[E] = d<G, X_S>/dw_E and
 * gX0 float32 [n][K] = d<G, X_S>/dX0.  With store_states != 0 the S+1
 * sweep-boundary states are kept; otherwise they are recomputed from X0
 * (S(S+1)/2 sweeps, three state buffers).  bfloat16 rounding of stored
 * states is treated as the identity in the reverse pass.  Deterministic
 * (gather form, no atomics on values).  Workspace: gr_smooth_vjp_workspace.
 */
int gr_smooth_vjp_workspace(int64_t n, int64_t nnz, int32_t K, int32_t dtype, int32_t sweeps,
                            int32_t store_states, size_t* bytes);
int gr_smooth_vjp(const gr_graph* g, const int32_t* edge_of_entry, int64_t n_edges,
                  const int32_t* colours, int32_t n_colours, int32_t K, int32_t sweeps,
                  int32_t dtype, const void* X0, const float* G, float* gw_E, float* gX0,
                  int32_t store_states, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * FP64 Laplacian eigenvalues (the spectrum a reduced graph should keep:
 * its first nontrivial eigenvalues, Sec. 5, Fig. 5).
 * ------------------------------------------------------------------- */
#define GR_EIG_AUTO 0      /* LOBPCG when max degree > 16 x mean degree   */
#define GR_EIG_CHEBYSHEV 1 /* Chebyshev-filtered subspace iteration       */
#define GR_EIG_LOBPCG 2    /* LOBPCG, Jacobi (D^-1) preconditioner        */

typedef struct gr_eig_report {
    int32_t iterations;        /* outer iterations                          */
    int32_t block;             /* block width m                             */
    double residual;           /* max ||L x_i - theta_i x_i|| of the wanted  */
    double lambda_max_bound;   /* b = 2 max degree >= lambda_max            */
    int32_t cholesky_warnings; /* 1 if an orthonormalisation lost rank      */
    int32_t method;            /* GR_EIG_CHEBYSHEV or GR_EIG_LOBPCG used    */
    int32_t restarts;          /* LOBPCG bases rebuilt without P            */
} gr_eig_report;

/*
 * gr_laplacian_eigs — the n_eig (1..32) smallest eigenvalues of L = D - A
 * restricted to the vectors orthogonal to the all-one vector (for a
 * connected graph lambda_2 .. lambda_{n_eig+1}; a graph with c components
 * reports c - 1 zeros first), in FP64.  Both methods keep a block of
 * m > n_eig orthonormal vectors and stop when every wanted Ritz pair has
 * residual <= tol * b (b = 2 max degree) or after max_iter iterations:
 *  - GR_EIG_CHEBYSHEV: m = n_eig + max(8, n_eig) (<= 64), each iteration
 *    applies the Chebyshev polynomial of [a, b] (a = the largest Ritz
 *    value) of degree <= `degree` (capped so no direction grows by more
 *    than 1e6), then Rayleigh-Ritz;
 *  - GR_EIG_LOBPCG: m = min(n_eig + 8, 21), Rayleigh-Ritz over
 *    [X, D^{-1} R, P]; needs n_eig <= 19 and n >= 12 m (GR_EUNSUP else).
 * Where n - 1 < m the block spans the whole complement and entries past
 * n - 1 are NaN.  Output eig double[n_eig] is HOST; report (may be NULL)
 * is HOST.  Synchronises once or twice per iteration.  Workspace:
 * gr_eig_workspace (about 32 n * 64 bytes).
 */
int gr_eig_workspace(int64_t n, int32_t n_eig, size_t* bytes);
int gr_laplacian_eigs(const gr_graph* g, int32_t n_eig, int32_t method, double tol,
                      int32_t max_iter, int32_t degree, uint64_t seed, double* eig,
                      gr_eig_report* report, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_laplacian_eigpairs — gr_laplacian_eigs with the eigenvectors: the same
 * solve (same arguments, same eig and report), and U double[n][n_eig]
 * (device, row-major, caller-owned) receives the Ritz vector of eig[i] in
 * column i: orthonormal, orthogonal to the all-one vector, each to within
 * the solve's residual (sign arbitrary; within a repeated eigenvalue any
 * orthonormal basis of its space).  Columns past the block are NaN, like
 * their eigenvalues.  Workspace: gr_eig_workspace.  Synchronises.
 */
int gr_laplacian_eigpairs(const gr_graph* g, int32_t n_eig, int32_t method, double tol,
                          int32_t max_iter, int32_t degree, uint64_t seed, double* eig, double* U,
                          gr_eig_report* report, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * The reduction hierarchy, the generalised eigenproblem L u = lambda B u,
 * the weighted-Jacobi solution refinement (Alg. 3, Sec. 3.5) and the
 * multilevel Laplacian eigensolver (Alg. 5, Sec. 4.1), all in FP64.
 * B is always diagonal, passed as its diagonal b (device double[n],
 * positive and finite), or NULL for B = I.
 * ------------------------------------------------------------------- */
#define GR_MAX_LEVELS 32

typedef struct gr_hierarchy {
    int32_t* maps;      /* device int32[maps_cap]: the node-to-aggregate map of
                           level l (H_{l+1}^{l} = P_l, values in [0, n[l+1])),
                           n[l] entries from maps_off[l]                      */
    int64_t maps_cap;
    int32_t* row_ptr;   /* device int32[rp_cap]: row pointers of level l+1,
                           n[l+1] + 1 entries from rp_off[l] (starting at 0)  */
    int64_t rp_cap;
    int32_t* col;       /* device int32[ent_cap]: columns of level l+1,
                           nnz[l+1] entries from ent_off[l]                   */
    float* w;           /* device float32[ent_cap]: weights, as col           */
    int64_t ent_cap;
    int32_t levels;     /* coarse levels held (level 0 is the input graph)    */
    int64_t n[GR_MAX_LEVELS + 1];    /* nodes of level l                      */
    int64_t nnz[GR_MAX_LEVELS + 1];  /* stored entries of level l             */
    int64_t maps_off[GR_MAX_LEVELS];
    int64_t rp_off[GR_MAX_LEVELS];
    int64_t ent_off[GR_MAX_LEVELS];
} gr_hierarchy;

/*
 * gr_reduce_hierarchy — gr_reduce (same arguments, same results) that also
 * keeps the hierarchy Alg. 5 walks (Sec. 4.1: every level's Laplacian and
 * its mapping operator): each level that shrank the graph appends its map
 * and the coarse graph it produced to *h (caller-allocated device arrays
 * with the capacities in *h; a level that made no progress is not kept).
 * Outputs: h->levels, h->n, h->nnz and the offsets.  GR_ENOMEM when a
 * capacity is too small (the message gives the totals needed so far); the
 * maps of a reduction total at most 2 n plus the isolated nodes once per
 * level, and its coarse graphs rarely more than nnz entries.
 */
int gr_reduce_hierarchy(const gr_graph* g, const gr_params* p, gr_result* res, gr_hierarchy* h,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * gr_laplacian_geigpairs — gr_laplacian_eigpairs for the generalised
 * problem L u = lambda B u with B = diag(b) (the B_G of Alg. 4 and 5):
 * the n_eig smallest eigenvalues with u B-orthogonal to the all-one vector
 * (its null vector), and U (device double[n][n_eig]) B-orthonormal.  The
 * solvers run on S L S, S = B^-1/2, in the complement of B^1/2 1 (same
 * methods, block sizes and stopping rule as gr_laplacian_eigs, with the
 * Gershgorin bound of S L S in place of 2 max degree).  b = NULL is the
 * plain problem.  GR_EINVAL if some b is not positive and finite.
 * Workspace: gr_eig_workspace.  Synchronises.
 */
int gr_laplacian_geigpairs(const gr_graph* g, const double* bdiag, int32_t n_eig, int32_t method,
                           double tol, int32_t max_iter, int32_t degree, uint64_t seed,
                           double* eig, double* U, gr_eig_report* report, void* ws,
                           size_t ws_bytes, void* stream);

/*
 * gr_jacobi_filter — `iters` weighted-Jacobi steps on every column i of Y
 * (device double[n][k], in place, 1 <= k <= 64):
 *     y <- y - theta D^-1 (L y - lambda_i B y),
 * D the weighted degrees of g.  With lambda = NULL this is the solution
 * refinement of Alg. 3, y <- (1 - theta) y + theta D^-1 A y; with the
 * eigenvalues lambda (HOST double[k]) and B = diag(bdiag) (or I) it is the
 * eigenvector filter of Alg. 5 on (L - lambda_i B) y = 0.  Rows with d = 0
 * are left unchanged.  Workspace: gr_jacobi_workspace.  Synchronises once
 * (to size the row pieces) and at the end.
 */
int gr_jacobi_workspace(int64_t n, int32_t k, size_t* bytes);
int gr_jacobi_filter(const gr_graph* g, int32_t k, double* Y, const double* lambda,
                     const double* bdiag, double theta, int32_t iters, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * gr_orthonormalize — Gram-Schmidt over [1, u_1, .., u_k] in the B inner
 * product (B = diag(bdiag), or I), keeping the k columns after the
 * constant: U (device double[n][k], in place) becomes B-orthonormal and
 * B-orthogonal to the all-one vector, each column in the span of the
 * constant and the columns before it (the final step of Alg. 5).
 * Computed as a projection and two Cholesky QR passes, which give the same
 * factor.  GR_EINVAL if the columns are linearly dependent (with the
 * constant).  Workspace: gr_orthonormalize_workspace.  Synchronises.
 */
int gr_orthonormalize_workspace(int64_t n, int32_t k, size_t* bytes);
int gr_orthonormalize(int64_t n, int32_t k, double* U, const double* bdiag, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * gr_multilevel_eigs — the multilevel Laplacian eigensolver (Alg. 5,
 * Sec. 4.1) on the hierarchy *h of graph g (as gr_reduce_hierarchy keeps
 * it; h->n[0] must be g->n):
 *  1. the first k nontrivial eigenpairs (lambda_i, u_i) of the coarsest
 *     problem L^Y u = lambda B^Y u (gr_laplacian_geigpairs, seed, tol,
 *     max_iter);
 *  2. for each level from the coarsest up: U <- H U (the level's 0/1 map),
 *     then `iters` steps of gr_jacobi_filter with the coarsest lambda_i and
 *     that level's B;
 *  3. gr_orthonormalize in the finest B.
 * B of the finest level is I (mode GR_RQ_IDENTITY, ratio cut) or D
 * (GR_RQ_DEGREE, normalized cut); each coarser level's B is the one the
 * prolongation induces, P^T B P (the sums of B over each aggregate), so a
 * coarse vector's quotient equals that of its prolongation.  Outputs:
 * eig HOST double[k] (the coarsest lambda_i), U device double[n][k].
 * 1 <= k <= 32, theta > 0.  Workspace: gr_multilevel_workspace.
 * Synchronises.
 */
int gr_multilevel_workspace(int64_t n, int64_t nnz, int32_t k, size_t* bytes);
int gr_multilevel_eigs(const gr_graph* g, const gr_hierarchy* h, int32_t k, int32_t mode,
                       double theta, int32_t iters, double tol, int32_t max_iter, uint64_t seed,
                       double* eig, double* U, gr_eig_report* report, void* ws, size_t ws_bytes,
                       void* stream);

/* ---------------------------------------------------------------------
 * Constrained-SGD edge scaling (Alg. 1, Sec. 3.3.4), FP64.
 * ------------------------------------------------------------------- */
#define GR_SGD_MAX_ITER 64

typedef struct gr_sgd_params {
    double alpha;       /* momentum coefficient                               */
    double eta_scale;   /* eta_max = eta_scale * mean(w_P) / max|s^(1)|        */
    double eps;         /* stop when (lambda_n^(k-1) - lambda_n^(k)) / lambda_n^(k) < eps */
    double delta_bar;   /* lambda_1 may fall at most to lambda_1^(0) * delta_bar */
    int32_t k_max;      /* iteration limit, <= GR_SGD_MAX_ITER                 */
    int32_t t;          /* generalised power iterations per h_t (the paper: 2) */
    uint64_t seed;      /* h_0 = one column of the test-vector generator       */
    int32_t cg_max_iter;/* 0 = 20000                                           */
    double cg_tol;      /* relative residual of the L_P solves; 0 = 1e-13      */
} gr_sgd_params;

typedef struct gr_sgd_report {
    int32_t iterations;              /* weight updates applied             */
    int32_t n_lambda;                /* entries of lambda_n                */
    int32_t cg_iterations_max;       /* longest L_P solve                  */
    double lambda_n[GR_SGD_MAX_ITER];     /* h_t^T L_G h_t per iteration  */
    double lambda_1[GR_SGD_MAX_ITER + 1]; /* min_p d_G(p)/d_P(p) after each */
} gr_sgd_report;

/*
 * gr_sgd_scale — Alg. 1 (Sec. 3.3.4) on the GPU in FP64.  G: the original
 * graph (float32 weights).  P: a subgraph on the same n nodes (CSR
 * structure; its weight array is ignored) with its edge list p_eu/p_ev
 * (E = p_edges, eu < ev) and p_edge_of_entry (see gr_edge_list).  w_P:
 * double[E] on the device, scaled in place.  Per iteration: h_t from t
 * generalised power iterations h <- L_P^+ L_G h (L_P solves by
 * Jacobi-preconditioned CG), normalised to h^T L_P h = 1;
 * lambda_n = h^T L_G h; s_e = -lambda_n (h_p - h_q)^2; dw <- alpha dw - eta s;
 * per-node caps cap_p = d_G(p)/(lambda_1 Delta) - d_P(p),
 * Delta = delta_bar^(1/k_max), shared in proportion where the edges at p ask
 * for more (all edges are updated at once: the parallel reading of the
 * paper's edge-by-edge lines); w += dw; eta <- (lambda_n/lambda_n^(0)) eta_max;
 * lambda_1 = min_p d_G(p)/d_P(p).  *report is HOST.  Synchronises every CG
 * check and iteration.  Workspace: gr_sgd_workspace.
 */
int gr_sgd_workspace(int64_t n, int64_t nnz_g, int64_t nnz_p, int64_t p_edges, size_t* bytes);
int gr_sgd_scale(const gr_graph* G, const gr_graph* P, const int32_t* p_edge_of_entry,
                 int64_t p_edges, const int32_t* p_eu, const int32_t* p_ev, double* w_P,
                 const gr_sgd_params* params, gr_sgd_report* report, void* ws, size_t ws_bytes,
                 void* stream);

/* ---------------------------------------------------------------------
 * Phase B, spectral sparsification (Sec. 3.3.2-3.3.3), and the flow of
 * Alg. 2.  Edge flags and edge values are indexed by the undirected edge
 * numbering of gr_edge_list (upper entries in CSR order).
 * ------------------------------------------------------------------- */
#define GR_SPARSIFY_MAX_ROUNDS 64

typedef struct gr_sparsify_params {
    int32_t t;             /* generalised power iterations per estimate (the paper: 2) */
    int32_t rounds;        /* densification rounds at most (<= GR_SPARSIFY_MAX_ROUNDS) */
    double add_frac;       /* edges added per round: ceil(add_frac * n)          */
    double lambda_target;  /* stop once the estimate of lambda_n is at most this */
    uint64_t seed;         /* h_0: one column of the test-vector generator       */
    int32_t cg_max_iter;   /* 0 = 20000                                          */
    double cg_tol;         /* relative residual of the L_P solves; 0 = 1e-12     */
} gr_sparsify_params;

typedef struct gr_sparsify_report {
    int32_t rounds;          /* densification rounds run                       */
    int32_t n_lambda;        /* entries of lambda_n                            */
    int64_t tree_edges;      /* edges of the spanning forest                   */
    int64_t edges;           /* edges of the sparsifier at the end             */
    int32_t cg_iterations_max;
    double lambda_n[GR_SPARSIFY_MAX_ROUNDS + 1]; /* h_t^T L_G h_t after the tree
                                                    and after each round       */
} gr_sparsify_report;

/*
 * gr_spanning_forest — the spanning tree that Phase B starts from
 * (Sec. 3.3.2), read as the maximum-weight spanning forest: edges ordered by
 * weight descending, ties by the smaller, then the larger endpoint, taken
 * greedily (the unique forest of that order, found by Boruvka rounds).
 * Output: in_tree int32[nnz/2] (device, 1 = in the forest), *n_tree HOST.
 * Workspace: gr_sparsify_workspace.  Synchronises every round.
 */
int gr_spanning_forest(const gr_graph* g, int32_t* in_tree, int64_t* n_tree, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * gr_sparsify — Phase B's sparsifier P of g (Sec. 3.3.2-3.3.3): the
 * spanning forest above, then rounds of densification.  Each round forms
 * h_t (t generalised power iterations h <- L_P^+ L_G h from h_0, L_P solves
 * by Jacobi-preconditioned CG, normalised to h^T L_P h = 1), records
 * lambda_n = h^T L_G h, and adds the ceil(add_frac n) edges outside P of
 * largest criticality w_G(p,q) (h_p - h_q)^2 (ties to the smaller edge
 * number); it stops after `rounds` rounds or once lambda_n <= lambda_target.
 * Outputs: in_P int32[nnz/2] (device, 1 = in P); criticality double[nnz/2]
 * (device, may be NULL): the final P's criticalities (0 on P's edges);
 * *rep HOST.  Workspace: gr_sparsify_workspace.  Synchronises.
 */
int gr_sparsify_workspace(int64_t n, int64_t nnz, size_t* bytes);
int gr_sparsify(const gr_graph* g, const gr_sparsify_params* p, int32_t* in_P, double* criticality,
                gr_sparsify_report* rep, void* ws, size_t ws_bytes, void* stream);

/*
 * gr_subgraph — the subgraph of g on the edges flagged in keep (int32[nnz/2],
 * device): CSR p_row_ptr int32[n+1], p_col int32[<= nnz], p_w float32[<= nnz]
 * with g's weights, entries in g's order; optionally (non-NULL) its edge list
 * p_eu/p_ev int32[<= nnz/2] (the kept edges in g's edge order) and
 * p_edge_of_entry int32[<= nnz] (P's edge of each P entry).  *p_nnz and
 * *p_edges HOST.  Workspace: gr_sparsify_workspace.  Synchronises.
 */
int gr_subgraph(const gr_graph* g, const int32_t* keep, int32_t* p_row_ptr, int32_t* p_col,
                float* p_w, int32_t* p_edge_of_entry, int32_t* p_eu, int32_t* p_ev, int64_t* p_nnz,
                int64_t* p_edges, void* ws, size_t ws_bytes, void* stream);

typedef struct gr_flow_params {
    gr_params phase_a;           /* the node reduction (Phase A)                 */
    gr_sparsify_params phase_b;  /* the sparsification (Phase B)                 */
    gr_sgd_params scaling;       /* Alg. 1 on the sparsifier                     */
    double gamma_max;            /* density threshold of Alg. 2 (the paper: 40)   */
} gr_flow_params;

typedef struct gr_flow_result {
    int32_t* agg;           /* device int32[n]: the node of S of every node of g  */
    int32_t* s_row_ptr;     /* device int32[n+1] (upper bound): S as CSR           */
    int32_t* s_col;         /* device int32[nnz] (upper bound)                     */
    float* s_w;             /* device float32[nnz] (upper bound)                   */
    int64_t n_s;            /* out */
    int64_t nnz_s;          /* out */
    int32_t dense;          /* out: 1 when Phase B ran first (gamma >= gamma_max)  */
    double gamma;           /* out: |E_G| / |V|, undirected edges                  */
    int32_t levels;         /* out: Phase A levels                                 */
    uint32_t warnings;      /* out: Phase A's GR_W* bits                           */
    gr_sparsify_report sparsify;  /* out */
    gr_sgd_report scaling;        /* out */
} gr_flow_result;

/*
 * gr_spectral_reduce — Alg. 2: gamma = |E_G| / |V|; below gamma_max,
 * Phase A reduces g to R, then Phase B sparsifies R and Alg. 1 scales the
 * sparsifier's weights, giving S; otherwise Phase B and Alg. 1 first give P
 * (g's nodes, scaled weights rounded to float32) and Phase A reduces P to
 * S.  Phase A is gr_reduce with p->phase_a (a prescribed colouring is used
 * only when Phase A runs on g itself), Phase B gr_sparsify, Alg. 1
 * gr_sgd_scale.  Outputs in *res (device arrays caller-allocated, sizes as
 * gr_reduce's).  Workspace: gr_spectral_reduce_workspace.  Synchronises.
 */
int gr_spectral_reduce_workspace(int64_t n, int64_t nnz, int32_t K, int32_t vec_dtype,
                                 size_t* bytes);
int gr_spectral_reduce(const gr_graph* g, const gr_flow_params* p, gr_flow_result* res, void* ws,
                       size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHREDUCE_H */
