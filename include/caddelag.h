/*
 * caddelag.h - C ABI of the MI355X (gfx950) commute-time anomaly-detection
 * library (libcaddelag.so).
 *
 * The calls follow the problem statements of the paper's algorithms:
 *   cdl_build_graph      - the fully connected Gaussian-kernel graph of one
 *                          snapshot (Section "Climate Data"; Background:
 *                          symmetric A, no self-edges, volume V_G).
 *   cdl_graph_from_weights - the same, for a caller-supplied weight matrix.
 *   cdl_build_chain      - ChainProduct of Algorithm 2: the normalised
 *                          matrix S = D^{-1/2} A D^{-1/2} and its repeated
 *                          squares (eq. inverse-chain).
 *   cdl_solve_embedding  - CommuteTimeEmbedding of Algorithm 3: k random
 *                          right-hand sides y = B^T W^{1/2} q (Algorithm 1),
 *                          each solved with the chain as preconditioner
 *                          (EstimateSolution of Algorithm 2, batched over the
 *                          k columns) to an FP64 residual tolerance.
 *   cdl_anomaly_scores   - Algorithm 4: commute times c = V_G ||z_i - z_j||^2
 *                          (eq. 1) of two snapshots, node scores
 *                          F_i = sum_j omega_ij |c_t(i,j) - c_{t+1}(i,j)| and
 *                          the top-K nodes.
 *   cdl_solve_embedding_pair - the same for both snapshots of a pair on one
 *                          node set, their right-hand sides made together.
 *   cdl_anomaly_edges    - the K largest edge scores of a pair (the CAD edge
 *                          score of the Background section).
 *   cdl_chain_densify    - Algorithm 2's dense product of the chain.
 *   cdl_score_sequence   - Algorithm 4 over consecutive pairs of a sequence
 *                          of snapshots with uneven node sets.
 *   cdl_stream_embedding - graph and embedding of one snapshot without storing
 *                          any n x n matrix (weights recomputed per sweep).
 *
 * Conventions
 * -----------
 * Memory.  Pointers documented as "device" point to GPU memory owned by the
 *   caller; "host" pointers point to CPU memory.  The library never allocates
 *   or frees device memory: every scratch buffer is a caller-supplied
 *   workspace whose size is returned by cdl_workspace_bytes().  Workspaces
 *   must be 256-byte aligned.  A context keeps one pinned host buffer for the
 *   values that calls read back (norms, statistics, flags), grown on demand
 *   and freed by cdl_ctx_destroy.
 * Layout.  n x n matrices (weights W, chain levels) use the library's padded
 *   square layout: cdl_ld(n) rows of cdl_ld(n) elements, row-major, with
 *   cdl_ld(n) = n rounded up to a multiple of 256; entries in padding rows and
 *   columns are zero (the library writes them so).  Node series X, the
 *   embedding Z and the scores F use plain row-major layouts described per
 *   call.
 * Streams.  Every call enqueues its GPU work on the context's stream (set at
 *   creation or with cdl_ctx_set_stream) in stream order.  A call that returns
 *   host values (marked "syncs") synchronises that stream before returning.
 * Errors.  Every call returns a cdl_status; no exception or abort crosses the
 *   boundary.  cdl_last_error() returns a message for the last failing call on
 *   the context.  On an error, output buffers hold unspecified values, except
 *   CDL_E_NOCONV, which leaves the last iterate in Z and fills the info struct.
 * Threads.  A context must not be used by two host threads at once.
 */
#ifndef CADDELAG_H
#define CADDELAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cdl_ctx cdl_ctx;

typedef enum {
    CDL_OK = 0,
    CDL_E_ARG = 1,          /* invalid argument: size, pointer, alignment, enum */
    CDL_E_WORKSPACE = 2,    /* workspace smaller than cdl_workspace_bytes() */
    CDL_E_NONFINITE = 3,    /* NaN or Inf in an input or an intermediate */
    CDL_E_GRAPH = 4,        /* invalid graph: node of zero degree, negative or
                               asymmetric weights, fewer than two nodes */
    CDL_E_DIVERGED = 5,     /* chain does not contract (spectral radius of the
                               normalised, deflated matrix is >= 1) */
    CDL_E_NOCONV = 6,       /* solve did not reach tol within max_iter */
    CDL_E_HIP = 7,          /* HIP runtime error */
    CDL_E_UNSUPPORTED = 8   /* valid request the library does not implement */
} cdl_status;

typedef enum { CDL_FP64 = 0, CDL_FP32 = 1, CDL_BF16 = 2, CDL_FP16 = 3 } cdl_prec;
typedef enum { CDL_RICHARDSON = 0, CDL_PCG = 1 } cdl_solver;
typedef enum {
    CDL_SCORE_UNWEIGHTED = 0,  /* omega_ij = 1 */
    CDL_SCORE_DELTA_A = 1      /* omega_ij = |A_{t+1}(i,j) - A_t(i,j)| (CAD edge score) */
} cdl_score_mode;

#define CDL_MAX_DEPTH 14
#define CDL_MAX_TOPK 256
#define CDL_GRAPH_STATS 4      /* device doubles: vol, sigma, deg_min, deg_max */

typedef struct {
    int depth;                 /* number of stored levels S~, S~^2, ..., S~^{2^(depth-1)} */
    int lazy;                  /* 1: levels are of (I + S)/2 (lazy walk) */
    cdl_prec prec;             /* element type of the stored levels */
    double rho_hat;            /* fro(S~_{d-1})^(1/2^(d-1)): upper estimate of rho(S~) */
    double rho_bound;          /* ||S~||_F of the unrounded FP64 S~: rigorous bound on rho */
    double fro[CDL_MAX_DEPTH + 1]; /* Frobenius norm of each stored level */
    int dense_levels;          /* 0: a chain of levels; m > 0: after cdl_chain_densify, the
                                  one stored matrix is prod_{l<m} (I + S~^{2^l}) - I (depth 1) */
} cdl_chain_info;

typedef struct {
    int iterations;            /* preconditioner applications performed */
    int converged;             /* 1 if the stopping test passed */
    double rel_residual;       /* final max_r ||y_r - L z_r|| / ||y_r|| (FP64) */
    double kappa;              /* deg_max (1 + rho_bound) / (deg_min (1 - rho_bound)) */
    double certified_error;    /* kappa * rel_residual: bound on ||Z - L^+ Y||_F / ||L^+ Y||_F */
    double history[64];        /* max relative residual after each iteration */
    int depth_used[64];        /* chain depth (stored + applied-by-repetition) per iteration */
} cdl_solve_info;

/* One snapshot of a sequence, for cdl_score_sequence. */
typedef struct {
    const double *X;           /* device, n x T row-major node series (row stride ldx) */
    int64_t n, T, ldx;
    const int32_t *gid;        /* device, n strictly increasing global node ids < 2^20 */
    const int32_t *gid_host;   /* host copy of gid (used to plan common-node maps) */
} cdl_snapshot;

typedef struct {
    int64_t k;                 /* random projections per snapshot */
    uint64_t seed;             /* projection seed (same for every snapshot) */
    double sigma;              /* > 0: fixed kernel bandwidth; <= 0: per-snapshot median rule */
    cdl_prec prec;             /* chain element type */
    int depth;                 /* > 0: fixed chain depth; 0: adaptive */
    int depth_max;
    double chain_eps;          /* adaptive-depth truncation target (<= 0: default per prec) */
    cdl_solver solver;
    double tol;                /* relative FP64 residual target of each solve */
    int max_iter;
    cdl_score_mode mode;
    int32_t top_k;
    int32_t flags;             /* 0, or CDL_SEQ_ASYNC with CDL_SEQ_GRAPH and/or CDL_SEQ_BATCHED */
} cdl_seq_params;

/* cdl_seq_params.flags.  CDL_SEQ_ASYNC: enqueue the whole sequence with no
 * host reads between kernels (fixed depth, Richardson with exactly max_iter
 * iterations, every pair's common-node map uploaded first), alternate
 * snapshots on the context's stream and a second stream of the context
 * (consecutive snapshots overlap; a pair is scored once both are done); one
 * read-back at the end checks every graph and residual.
 * CDL_SEQ_GRAPH (with CDL_SEQ_ASYNC): a call whose buffers, sizes,
 * parameters and global ids equal the previous graph call on the context is
 * captured into a HIP graph (both streams), later such calls replay it with
 * one launch. */
#define CDL_SEQ_ASYNC 1
#define CDL_SEQ_GRAPH 2
/* CDL_SEQ_BATCHED (with CDL_SEQ_ASYNC; FP32, BF16 or FP16 levels): one pass
 * over the whole sequence with every snapshot resident (the workspace grows
 * with the sum of the snapshots' sizes): grouped launches over all
 * snapshots for the graphs and level-0 chains, the right-hand sides per
 * snapshot on four streams of the context, then grouped launches over
 * all snapshots for each chain squaring, each step of the refinement (the
 * applications level by level, the FP64 residual product and reduction, the
 * norms) and the embeddings, and over all pairs for the scores.  Convergence
 * is tested on the device after every iteration: a snapshot whose relative
 * residual reaches tol (> 0) stops (its workgroups of later iterations
 * return at once), so max_iter is only an upper bound; tol = 0 runs exactly
 * max_iter iterations.  info->max_iterations is the largest iteration count
 * used; CDL_E_NOCONV if a snapshot ends above tol.  The split-K counts of the
 * grouped level applications and FP64 residual products are chosen for the
 * whole group (the smallest that gives two workgroups per CU), so the
 * results equal the per-snapshot path's to rounding; with the "apply" and
 * "residual" choices pinned on the context (cdl_ctx_force_choice) each
 * snapshot keeps its own counts and the results are bit for bit the same. */
#define CDL_SEQ_BATCHED 4

typedef struct {
    int32_t pairs;             /* number of scored pairs (n_snap - 1) */
    int32_t max_iterations;    /* largest iteration count over the solves */
    double max_rel_residual;   /* largest final residual over the solves */
    int32_t graph_launches;    /* CDL_SEQ_GRAPH: 1 if the call ran as a HIP graph */
} cdl_seq_info;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device` using HIP stream `stream` (a
 * hipStream_t; NULL = the default stream).  Allocates no device memory; takes
 * a 4 KiB pinned host buffer for read-backs, and on the first context of a
 * device resolves that device's address of the fixed scratch array of
 * cdl_anomaly_scores_noalloc (with the device made current for the call,
 * the caller's current device restored). */
cdl_status cdl_ctx_create(int device, void *stream, cdl_ctx **out);
cdl_status cdl_ctx_destroy(cdl_ctx *ctx);
cdl_status cdl_ctx_set_stream(cdl_ctx *ctx, void *stream);
const char *cdl_status_string(cdl_status s);
const char *cdl_last_error(const cdl_ctx *ctx);
/* Library version string, e.g. "caddelag-gfx950 1.0". */
const char *cdl_version(void);

/* depth > 0: every later solve iteration on this context applies the chain
 * at total depth `depth` (stored levels first, deeper ones by repeated
 * application of the last stored level) instead of the autotuned depth;
 * 0 restores autotuning.  CDL_E_ARG outside [0, 16]. */
cdl_status cdl_ctx_set_solve_depth(cdl_ctx *ctx, int depth);

/* Median-rule bandwidth selection of later cdl_build_graph and
 * cdl_stream_embedding calls on this context.  0 (default): a sorted sample
 * of pair distances (4096; 16384 computed from the series when streamed)
 * brackets the target rank, one pass over the matrix (streamed: one sweep
 * over the recomputed upper panels) counts the keys below the bracket and
 * collects those inside, and the radix passes run over the collected keys
 * (over the matrix, or one sweep per 12-bit digit, when the rank falls
 * outside the bracket).  1: radix passes over the matrix (digit sweeps) only.
 * Both are exact and give the same sigma.  CDL_E_ARG for other values. */
cdl_status cdl_ctx_set_select(cdl_ctx *ctx, int mode);

/* ---- per-kernel timing ------------------------------------------------- */

/* enable != 0: every kernel launch of later calls on this context is
 * bracketed by HIP events recorded on the context's stream (about ten
 * microseconds of stream time per timed launch); totals accumulate per kernel name
 * ("gram_dist", "select_median", "exp_degree", "normalize", "square",
 * "apply", "rhs", "residual", "score", "topk", ...). */
cdl_status cdl_ctx_set_timing(cdl_ctx *ctx, int enable);
/* Restricts the timing to the named kernels: `names` is a comma-separated
 * list of the names above ("rhs_pair,residual"; spaces ignored), copied;
 * NULL or "" times every kernel again.  Each timed launch adds two event
 * records to the stream, so timing only the kernel of interest keeps the
 * others' launches back to back.  CDL_E_ARG for a null context only. */
cdl_status cdl_ctx_set_timing_only(cdl_ctx *ctx, const char *names);
/* Syncs.  Entry idx (0-based, in first-seen order) of the totals: kernel
 * name (valid until the next reset), launches and summed milliseconds.
 * CDL_E_ARG past the last entry. */
cdl_status cdl_timing_read(cdl_ctx *ctx, int32_t idx, const char **name, int64_t *launches,
                           double *total_ms);
/* Syncs.  Clears the totals. */
cdl_status cdl_timing_reset(cdl_ctx *ctx);

/* ---- launch-configuration tuning ---------------------------------------- */

/* Three kernel families have several correct launch configurations, which
 * give the same results up to the rounding order of their sums:
 *   "square"    16-bit levels (cdl_build_chain, cdl_chain_densify): 256 x 256
 *               tiles on 8 waves with 32 x 32 x 16 MFMAs (choices 0, 1), 4
 *               waves with 32 x 32 x 16 (2, 3) or 8 waves with 16 x 16 x 32
 *               (4, 5); the last partial round of workgroups split over the
 *               reduction (even choices) or not (odd); other level types:
 *               one choice;
 *   "apply"     the chain application (cdl_solve_embedding*), BF16/FP16/FP32
 *               levels: the split-K count, the default (0), half (1) or
 *               twice (2) it; FP64 levels: one choice;
 *   "residual"  the FP64 residual product W X of the solves: split-K count,
 *               choices as for "apply".
 * A table per process keeps, per GPU architecture name, family, element
 * type and padded shape (cdl_ld(n), and the padded k for apply/residual),
 * the measured milliseconds of every candidate and the fastest one's index;
 * calls use the table's choice, else choice 0.  The environment variable
 * CDL_AUTOTUNE_CACHE names a JSON file that is merged into the table on first
 * use and rewritten after every new entry.  The chain-depth cost model of
 * cdl_build_chain and of the solves uses the measured times of the chosen
 * configurations when the table holds the shape. */

/* mode 1: later calls on this context time every candidate of a family the
 * first time they meet a shape the table does not hold (on the call's own
 * data; every candidate leaves a complete result; syncs once per candidate)
 * and record them; 0 (default): use the table only.  Calls of
 * cdl_score_sequence never tune.  CDL_E_ARG for other modes. */
cdl_status cdl_ctx_set_autotune(cdl_ctx *ctx, int mode);
/* Pins family ("square", "apply", "residual") to candidate `choice` on this
 * context (choice < 0 releases it; a choice beyond the family's candidates
 * for some shape falls back to the table there).  CDL_E_ARG for an unknown
 * family. */
cdl_status cdl_ctx_force_choice(cdl_ctx *ctx, const char *family, int choice);
/* The table's entry for family, element type and shape (n nodes, k columns;
 * k is ignored for "square") on device `device`'s architecture (device < 0:
 * the architecture name "none").  choice, candidates, ms (the chosen
 * candidate's time) may be NULL.  CDL_E_UNSUPPORTED: no entry;
 * CDL_E_ARG: invalid arguments. */
cdl_status cdl_autotune_lookup(int device, const char *family, cdl_prec prec, int64_t n,
                               int64_t k, int *choice, int *candidates, double *ms);
/* Merge a JSON table file into the table / write the whole table / empty it
 * (also forgetting CDL_AUTOTUNE_CACHE's file for the rest of the process).
 * CDL_E_ARG for an unreadable or malformed file or an unwritable path.
 * File format: {"format": "caddelag-autotune-1", "entries": [{"arch": name,
 * "key": "square/bf16/ld16384", "choice": i, "ms": [t0, t1, ...]}, ...]}. */
cdl_status cdl_autotune_load(const char *path);
cdl_status cdl_autotune_save(const char *path);
cdl_status cdl_autotune_clear(void);
/* Number of entries in the table. */
int32_t cdl_autotune_entries(void);

/* ---- sizes ------------------------------------------------------------- */

/* Padded leading dimension (and row count) of the library's n x n layout. */
int64_t cdl_ld(int64_t n);
/* Number of random projections k_RP = ceil(ln(n / eps_rp)) that Algorithm 1
 * and Algorithm 3 take for n nodes and accuracy eps_rp (the paper leaves the
 * logarithm's base open; the natural log is used).  This is the k that
 * cdl_solve_embedding uses when it is called with k <= 0.
 *   k       host output.
 * Errors: CDL_E_ARG for n < 2, eps_rp outside (0, 1) or a NULL k. */
cdl_status cdl_k_rp(int64_t n, double eps_rp, int64_t *k);
/* Storage scale of chain levels of type prec for n nodes: FP16 levels hold
 * scale * S~ with scale = 2^floor(log2 n), so that entries of order 1/n stay
 * in FP16's normal range; 1 for the other types.  Divide a level read back
 * through cdl_chain_level_offset by it.
 *   scale   host output.
 * Errors: CDL_E_ARG for n < 1, an invalid prec or a NULL scale. */
cdl_status cdl_level_scale(int64_t n, cdl_prec prec, double *scale);
/* Plain device-to-device copy on the context's stream (one 16-byte
 * nontemporal load and store per lane over a grid that covers the buffer):
 * the reference stream against which the hot kernels' HBM traffic and
 * bandwidth are read.  Not part of the method.
 *   src, dst  device buffers of `bytes` bytes, 16-byte aligned, disjoint;
 *             the caller owns both.
 *   bytes     a multiple of 16 (0: nothing to do).
 * Errors: CDL_E_ARG for a NULL ctx or buffer, misalignment, a size that is
 * not a multiple of 16 or overlapping buffers; CDL_E_HIP if the launch fails. */
cdl_status cdl_device_copy(cdl_ctx *ctx, const void *src, void *dst, size_t bytes);
/* Bytes of an n x n matrix of `prec` elements in the padded layout. */
size_t cdl_matrix_bytes(int64_t n, cdl_prec prec);
/* Byte offset of level 0 inside a chain buffer; level l starts at
 * offset + l * cdl_matrix_bytes(n, prec) (padded layout; FP16 levels hold
 * 2^floor(log2 n) * S~).  0 for invalid arguments. */
size_t cdl_chain_level_offset(int64_t n, cdl_prec prec);
/* Workspace sizes for one snapshot of n nodes with series of length T, k
 * projections and at most depth_max chain levels of element type prec:
 *   graph: for cdl_build_graph / cdl_graph_from_weights;
 *   chain: storage of the chain levels (kept between build_chain and every
 *          solve that uses it);
 *   solve: for cdl_solve_embedding;
 *   score: for cdl_anomaly_scores with up to n common nodes.
 * Any output pointer may be NULL. */
cdl_status cdl_workspace_bytes(int64_t n, int64_t T, int64_t k, int depth_max,
                               cdl_prec prec, size_t *graph, size_t *chain,
                               size_t *solve, size_t *score);

/* ---- graph --------------------------------------------------------------- */

/* Gaussian-kernel graph of one snapshot (Section "Climate Data"; Background).
 *   X       device, n x T FP64 node series, row i at X + i*ldx (ldx >= T).
 *   sigma   > 0: kernel bandwidth to use; <= 0: the lower median of the
 *           n(n-1)/2 pair distances ||x_i - x_j|| (element of 0-based rank
 *           floor((N-1)/2) of the sorted distances).
 *   W       device output, padded n x n FP64: W_ij = exp(-||x_i-x_j||^2 / sigma^2)
 *           for i != j, W_ii = 0.
 *   deg     device output, n FP64 degrees deg_i = sum_j W_ij.
 *   stats   device output, CDL_GRAPH_STATS FP64: vol = sum_i deg_i, sigma used,
 *           min and max degree.
 *   ws      device workspace of ws_bytes >= graph size from cdl_workspace_bytes.
 * Async.  Errors: CDL_E_ARG (n < 2, T < 1, ldx < T, NULL), CDL_E_WORKSPACE.
 * Non-finite X or a zero degree are reported by cdl_check_graph(). */
cdl_status cdl_build_graph(cdl_ctx *ctx, const double *X, int64_t n, int64_t T,
                           int64_t ldx, double sigma, double *W, double *deg,
                           double *stats, void *ws, size_t ws_bytes);

/* Copy a caller weight matrix into the padded layout and compute degrees.
 *   Win     device, n x n FP64 symmetric weights, row stride ldw (>= n); the
 *           diagonal is ignored (no self-edges).
 *   W, deg, stats, ws as for cdl_build_graph (stats[1] = 0).
 * Syncs: validates symmetry (exact), non-negativity, finiteness and positive
 * degrees; CDL_E_GRAPH / CDL_E_NONFINITE on failure. */
cdl_status cdl_graph_from_weights(cdl_ctx *ctx, const double *Win, int64_t n,
                                  int64_t ldw, double *W, double *deg,
                                  double *stats, void *ws, size_t ws_bytes);

/* Syncs.  Checks a built graph: CDL_E_NONFINITE if any weight or degree is
 * not finite, CDL_E_GRAPH if the minimum degree is not positive.  Optionally
 * returns stats to the host (host_stats may be NULL). */
cdl_status cdl_check_graph(cdl_ctx *ctx, const double *deg, const double *stats,
                           int64_t n, double *host_stats);

/* ---- chain (Algorithm 2, ChainProduct) ------------------------------------ */

/* Levels S~_0 = S - u u^T (S = D^{-1/2} W D^{-1/2}, u = D^{1/2} 1 / sqrt(vol);
 * lazy: S = (I + D^{-1/2} W D^{-1/2}) / 2) and S~_{l+1} = S~_l^2, stored in
 * element type prec (FP32 accumulation; FP64 for CDL_FP64).
 *   W, deg, stats  from cdl_build_graph / cdl_graph_from_weights.
 *   depth   > 0: exactly this many levels (<= depth_max); 0: adaptive.
 *   chain_eps  adaptive rule.  > 0: square until the truncation bound
 *           fro(S~_l)^2 / (1 - rho_hat) <= chain_eps (then depth = l+1) or
 *           depth_max levels are stored.  <= 0: autotune - before each
 *           squaring, compare the modelled time of one more squaring plus the
 *           refinement iterations it saves against stopping now (model: MFMA
 *           and HBM rates of the level type, a 1e-8 residual target, k = 256
 *           columns, contraction max(truncation bound, rounding floor of the
 *           level type)) and square only while that is cheaper.
 *   chain   device buffer of chain_bytes >= chain size from cdl_workspace_bytes.
 *   info    host output.
 * Syncs (reads back the level norms).  Errors: CDL_E_ARG, CDL_E_WORKSPACE,
 * CDL_E_DIVERGED (a level with fro >= 0.999 that did not shrink - an
 * eigenvalue of modulus one, e.g. a bipartite graph without lazy - or, in
 * adaptive mode, rho_hat >= 1 after all of depth_max >= 3 levels),
 * CDL_E_NONFINITE.  On CDL_E_DIVERGED info holds the levels built so far. */
cdl_status cdl_build_chain(cdl_ctx *ctx, const double *W, const double *deg,
                           const double *stats, int64_t n, cdl_prec prec,
                           int depth, int depth_max, double chain_eps, int lazy,
                           void *chain, size_t chain_bytes, cdl_chain_info *info);

/* The dense schedule of Algorithm 2 (the factor P of ChainProduct formed
 * once, then one product per Richardson step): replaces the info->depth
 * stored levels by the single matrix Q = prod_{l<d} (I + S~^{2^l}) - I, in
 * the level type and storage scale, built by d - 1 products
 * Q <- Q + L + Q L (symmetric MFMA GEMMs, upper tiles mirrored; the factors
 * commute).  The identity stays out of Q, so the solve applies
 * P = I + Q as it applies a one-level chain (the identity term in FP64).
 * On return info->depth = 1 and info->dense_levels = d; later solves apply P
 * once per iteration (no repeated levels).
 *   n      nodes of the chain's graph.
 *   chain  the buffer cdl_build_chain filled; for d >= 2 it must hold d + 1
 *          levels (the last as scratch): cdl_workspace_bytes with
 *          depth_max >= d + 1.
 * Errors: CDL_E_ARG (bad info, already dense), CDL_E_WORKSPACE. */
cdl_status cdl_chain_densify(cdl_ctx *ctx, int64_t n, void *chain, size_t chain_bytes,
                             cdl_chain_info *info);

/* ---- embedding (Algorithm 3 with Algorithm 1's right-hand sides) ---------- */

/* Z = L^+ Y for the k columns y_r = (1/sqrt(k)) B^T W^{1/2} q_r (L = D - W;
 * B the signed edge-node incidence with each edge's head at the endpoint of
 * lower global id; q_r(edge) = +-1 from the counter-based generator below).
 *   gid     device, n int32 global node ids < 2^20 (NULL = 0..n-1).  Signs
 *           depend only on (seed, r, global ids), so snapshots of a sequence
 *           share random numbers on common edges.
 *   k       number of projections (k <= 0: ceil(ln(n / eps_rp)), Algorithm 1).
 *   seed    sign word of edge {lo, hi} (global ids, lo < hi) and block
 *           beta = r / 64 is mix(mix(seed) ^ (beta << 40 | lo << 20 | hi)),
 *           mix = the SplitMix64 output function; bit (r mod 64) set = -1.
 *   solver  CDL_RICHARDSON: x <- x + P1 (y - L x) (EstimateSolution with
 *           P2 y = P1 L y); CDL_PCG: conjugate gradients preconditioned by
 *           the same P1, one recurrence per column (flexible beta =
 *           z_{j+1} . (r_{j+1} - r_j) / z_j . r_j), x0 = 0; the residual is
 *           the recursively updated one.  Residuals and inner products in
 *           FP64.  An iteration is one application of P1 followed by one
 *           product with L.
 *   tol     > 0: stop when max_r ||y_r - L x_r|| / ||y_r|| <= tol;
 *           < 0: stop when the certified embedding error kappa * max_r rel_r
 *           <= |tol| (kappa from the degree range and rho_bound: the nonzero
 *           spectrum of L lies in [deg_min (1 - rho), deg_max (1 + rho)]);
 *           == 0: run exactly max_iter preconditioner applications.
 *   Depth   each iteration applies the stored levels and, when the model says
 *           it pays, further levels S~^{2^l} (l >= depth) as 2^(l-depth+1)
 *           repeated applications of the last stored level; a cost model
 *           (FP64 residual vs. level applications, rounding floor of the
 *           level type) picks the depth per iteration (info->depth_used).
 *   Z       device output, n x k FP64 row-major (row i = z_i), columns
 *           centred (1^T z_r = 0).
 *   info    host output (may be NULL).
 * Syncs once per iteration (residual norms).  Errors: CDL_E_ARG,
 * CDL_E_WORKSPACE, CDL_E_NOCONV (Z holds the last iterate), CDL_E_NONFINITE. */
cdl_status cdl_solve_embedding(cdl_ctx *ctx, const double *W, const double *deg,
                               const double *stats, const int32_t *gid, int64_t n,
                               const void *chain, const cdl_chain_info *chain_info,
                               int64_t k, double eps_rp, uint64_t seed,
                               cdl_solver solver, double tol, int max_iter,
                               double *Z, void *ws, size_t ws_bytes,
                               cdl_solve_info *info);

/* Both snapshots of a pair on one node set (the same n and global ids):
 * cdl_solve_embedding for each, with the right-hand sides of both made in
 * one sweep over W0 and W1.  The two graphs share the projection on every
 * edge (the same seed and ids give the same signs), so each edge's sign word
 * is hashed once for both (Algorithm 4 over Algorithm 3's embeddings of G1
 * and G2).  Results equal two cdl_solve_embedding calls up to the rounding of
 * the right-hand sides' FP64 sums (< 1e-15 relative).
 *   W0, deg0, stats0, chain0, chain_info0   snapshot 0 as for
 *           cdl_solve_embedding (likewise for snapshot 1; the chains may
 *           differ in type and depth).
 *   gid, n, k, seed, solver, tol, max_iter   shared; k >= 1.
 *   Z0, Z1  device outputs, n x k FP64 each.
 *   ws0, ws1  two solve workspaces of at least ws_bytes each (the size of
 *           cdl_workspace_bytes for that chain type).
 *   info0, info1  host outputs (may be NULL).
 * Snapshot 0 is solved first; if it fails, its status is returned and Z1 is
 * unspecified.  Errors as for cdl_solve_embedding. */
cdl_status cdl_solve_embedding_pair(cdl_ctx *ctx, const double *W0, const double *deg0,
                                    const double *stats0, const void *chain0,
                                    const cdl_chain_info *chain_info0, const double *W1,
                                    const double *deg1, const double *stats1,
                                    const void *chain1, const cdl_chain_info *chain_info1,
                                    const int32_t *gid, int64_t n, int64_t k, uint64_t seed,
                                    cdl_solver solver, double tol, int max_iter, double *Z0,
                                    double *Z1, void *ws0, void *ws1, size_t ws_bytes,
                                    cdl_solve_info *info0, cdl_solve_info *info1);

/* ---- right-hand sides alone ------------------------------------------------ */

/* The k right-hand sides of Algorithm 1 for one graph, or for two graphs on
 * one node set, as cdl_solve_embedding and cdl_solve_embedding_pair make
 * them: y_i = (1/sqrt(k)) sum_j B(e_ij, i) q(e_ij) sqrt(W_ij), the sign of
 * edge {i, j} in column r the bit r mod 64 of the SplitMix64 word of
 * (seed, r / 64, the two global ids), negated at the edge's tail (the end
 * with the higher id).  The signed sums are exact int8 matrix products of
 * the sign bits with base-256 digits of the weights' square roots scaled by a
 * power of two per 1024 neighbours; the only rounding is that scaling (at
 * most 2^-55 of the largest |sqrt(W_ij)| of those neighbours per term) and
 * the FP64 sums.
 *   W0      device, padded n x n FP64 weights (non-negative; a non-finite
 *           weight makes its row of Y non-finite).
 *   W1      device, a second padded n x n FP64 weight matrix on the same node
 *           set (the same ids, so the same signs), or NULL.
 *   gid     device, n global node ids < 2^20, or NULL for ids 0..n-1.
 *   n, k, seed  2 <= n <= 2^20, 1 <= k <= 2^20; seed as for
 *           cdl_solve_embedding.
 *   Y0, Y1  device outputs, n x k FP64 row-major (row i = y_i); Y1 NULL
 *           exactly when W1 is NULL.
 *   ws      device workspace of ws_bytes >= cdl_rhs_workspace_bytes (pair =
 *           W1 != NULL).
 * Async.  Errors: CDL_E_ARG, CDL_E_WORKSPACE. */
cdl_status cdl_rhs_workspace_bytes(int64_t n, int64_t k, int pair, size_t *bytes);
cdl_status cdl_rhs(cdl_ctx *ctx, const double *W0, const double *W1, const int32_t *gid,
                   int64_t n, int64_t k, uint64_t seed, double *Y0, double *Y1, void *ws,
                   size_t ws_bytes);

/* ---- streamed snapshots (graphs larger than device memory) ---------------- */

/* One snapshot end to end - bandwidth, weights, degrees, right-hand sides and
 * the solve of cdl_solve_embedding - without storing any n x n matrix
 * (Algorithm 3 with the graph of the "Climate Data" section).  Every sweep
 * over the weights recomputes them row panel by row panel from X (the
 * distance Gram of cdl_build_graph, then W = exp(-D2 / sigma^2) with
 * W_ii = 0); each panel value equals the stored matrix's bit for bit.  The
 * device memory needed grows as n (T + 5 k + panel_rows) instead of n^2:
 * the complexity section's recomputation/communication trade made on one
 * device, where memory capacity rather than arithmetic limits n.
 *   X, n, T, ldx, sigma   as for cdl_build_graph (sigma <= 0: the exact
 *           lower median rule: one sweep over the upper row panels gathers
 *           the keys inside a sampled bracket (about 2.3 % of them, into the
 *           workspace), or, when the bracket misses, one sweep per 12-bit
 *           digit of the key; see cdl_ctx_set_select).
 *   gid, k, seed          as for cdl_solve_embedding (k >= 1).
 *   tol, max_iter         as for cdl_solve_embedding.  The preconditioner is
 *           the chain of depth 1, P1 = D^{-1/2} (I + S) D^{-1/2} (Algorithm 2
 *           with d = 1: no squaring needs a stored matrix), in Richardson's
 *           iteration x <- x + P1 (y - L x); each iteration is two sweeps
 *           (one product with W for P1, one for the residual), the residual
 *           contracting by rho(S~)^2 per iteration.  kappa (for tol < 0) uses
 *           rho_bound = ||S~||_F from the first sweep.
 *   panel_rows            rows of W recomputed per panel (rounded up to a
 *           multiple of 256, at most ld; 0: 32768).  Results do not depend on
 *           it.
 *   level_prec, chain, chain_bytes, chain_info   level_prec = -1: as above,
 *           no n x n storage at all (chain and chain_info may be NULL).
 *           level_prec = a cdl_prec: level 0 of the chain, S~ in that type
 *           (n^2 x 2 bytes in FP16: 128 GiB at n = 262144, where the FP64 W
 *           would take 512 GiB), is stored in the caller's chain buffer
 *           (cdl_workspace_bytes with depth_max = 1) by one more sweep, and
 *           the solve is cdl_solve_embedding's (solver CDL_RICHARDSON, the
 *           cost model's depth with deeper levels applied by repetition),
 *           its FP64 residual's product W X taken by a streamed sweep.  The
 *           level is exactly symmetric and equals cdl_build_chain's up to the
 *           rounding of the degrees (summed in another order).  chain_info
 *           (host, may be NULL) receives the level's description (depth 1).
 *   deg, stats            device outputs as for cdl_build_graph.
 *   Z, info               as for cdl_solve_embedding (depth_used = 1).
 *   ws, ws_bytes          device workspace of cdl_stream_workspace_bytes.
 * Scores of two streamed snapshots come from cdl_anomaly_scores in the
 * unweighted mode (W0 = W1 = NULL).  Syncs once per digit of the median and
 * once per iteration.  Errors: CDL_E_ARG, CDL_E_WORKSPACE, CDL_E_NONFINITE
 * (non-finite series, degrees or residuals), CDL_E_GRAPH (zero degree),
 * CDL_E_NOCONV (Z holds the last iterate). */
cdl_status cdl_stream_workspace_bytes(int64_t n, int64_t T, int64_t k, int64_t panel_rows,
                                      int level_prec, size_t *bytes);
cdl_status cdl_stream_embedding(cdl_ctx *ctx, const double *X, int64_t n, int64_t T,
                                int64_t ldx, double sigma, const int32_t *gid, int64_t k,
                                uint64_t seed, double tol, int max_iter, int64_t panel_rows,
                                int level_prec, void *chain, size_t chain_bytes,
                                cdl_chain_info *chain_info, double *deg, double *stats,
                                double *Z, void *ws, size_t ws_bytes, cdl_solve_info *info);

/* ---- scores (Algorithm 4) -------------------------------------------------- */

/* F_c = sum_{c'} omega |c_0(a,b) - c_1(a',b')| over the m common nodes, where
 * common node c is row map0[c] of snapshot 0 and row map1[c] of snapshot 1,
 * c_t = vol_t ||z_i - z_j||^2, omega = 1 or |W1(a',b') - W0(a,b)|.
 *   Z0, Z1      device, n0 x k and n1 x k FP64 row-major embeddings.
 *   W0, W1      device, padded weight matrices (only read for DELTA_A; may be
 *               NULL for UNWEIGHTED).
 *   stats0/1    device graph stats (vol read from element 0).
 *   map0, map1  device, m int32 row indices (NULL = identity; then m = n0 = n1).
 *   F           device output, m FP64.
 *   top_k       number of top nodes (0..CDL_MAX_TOPK, <= m).
 *   top_idx     device output, top_k int32 common-node indices sorted by
 *               descending F, ties by ascending index.
 * Async.  Errors: CDL_E_ARG, CDL_E_WORKSPACE. */
cdl_status cdl_anomaly_scores(cdl_ctx *ctx, const double *Z0, const double *W0,
                              const double *stats0, int64_t n0,
                              const double *Z1, const double *W1,
                              const double *stats1, int64_t n1, int64_t k,
                              const int32_t *map0, const int32_t *map1, int64_t m,
                              cdl_score_mode mode, double *F, int32_t top_k,
                              int32_t *top_idx, void *ws, size_t ws_bytes);

/* cdl_anomaly_scores without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Arguments, results and errors as for
 * cdl_anomaly_scores; the workspace is a fixed 160 MiB array in device memory
 * that the library holds on every device it runs on until the process ends
 * (enough for m = 16384 common nodes at k = 256; the bytes needed are
 * cdl_workspace_bytes' score size plus 256).  Larger m, k: CDL_E_WORKSPACE,
 * nothing enqueued.  The call allocates and frees nothing (device or pinned
 * memory, events) and does not time its kernels.  Every byte the kernels
 * read is written earlier in the same call, so the array's contents from an
 * earlier call do not matter; but all calls on one device share the array,
 * so calls that overlap on a device (other host threads, other streams not
 * ordered with this one) race and give undefined results.  With maps, their
 * entries are checked on the device and the stream is synchronised once
 * (CDL_E_ARG for an entry out of range); without maps the call is
 * asynchronous.  CDL_E_HIP if the device's scratch address could not be
 * resolved when its first context was created. */
cdl_status cdl_anomaly_scores_noalloc(cdl_ctx *ctx, const double *Z0, const double *W0,
                                      const double *stats0, int64_t n0,
                                      const double *Z1, const double *W1,
                                      const double *stats1, int64_t n1, int64_t k,
                                      const int32_t *map0, const int32_t *map1, int64_t m,
                                      cdl_score_mode mode, double *F, int32_t top_k,
                                      int32_t *top_idx);

/* Edge-level anomalies (Background: the CAD edge score
 * dE_ab = omega_ab |c_0(a,b) - c_1(a,b)|, whose row sums are the node
 * scores of Algorithm 4): the top_k edges a < b over the m common nodes.
 *   Inputs as for cdl_anomaly_scores; F (device, m FP64) receives the node
 *   scores as a by-product.
 *   top_k       1..CDL_MAX_TOPK, at most m(m-1)/2.
 *   edge_a, edge_b  device outputs, top_k int32 common-node indices (a < b),
 *               sorted by descending score, ties by ascending (a, b).
 *   edge_val    device output, top_k FP64 scores.
 *   ws          device workspace of cdl_edges_workspace_bytes(m, k, top_k).
 * Exact: the per-tile maxima of the fused score give a lower bound on the
 * K-th largest edge score (the K-th largest tile maximum); only tiles reaching
 * it are recomputed and their edges at or above it sorted.  Syncs once.
 * Errors: CDL_E_ARG, CDL_E_WORKSPACE, CDL_E_UNSUPPORTED when more than
 * max(16384 top_k, 2^22) edges reach that bound (massive exact ties). */
cdl_status cdl_edges_workspace_bytes(int64_t m, int64_t k, int32_t top_k, size_t *bytes);
cdl_status cdl_anomaly_edges(cdl_ctx *ctx, const double *Z0, const double *W0,
                             const double *stats0, int64_t n0,
                             const double *Z1, const double *W1,
                             const double *stats1, int64_t n1, int64_t k,
                             const int32_t *map0, const int32_t *map1, int64_t m,
                             cdl_score_mode mode, double *F, int32_t top_k,
                             int32_t *edge_a, int32_t *edge_b, double *edge_val,
                             void *ws, size_t ws_bytes);

/* Whole sequence: for every snapshot, graph + chain + embedding; for every
 * consecutive pair (t, t+1), scores over the common global ids.
 *   F[t]        device output for pair t: m_t FP64, m_t = |V_t ∩ V_{t+1}|, in
 *               ascending global-id order.
 *   top_idx[t]  device output for pair t: top_k int32 indices into F[t].
 *   ws          device workspace of cdl_sequence_workspace_bytes().
 * Syncs.  Errors as for the per-snapshot calls.  With CDL_SEQ_ASYNC: needs
 * depth > 0, CDL_RICHARDSON and tol >= 0 (CDL_E_ARG otherwise); the results
 * equal the synchronous call with tol = 0 and the same depth and max_iter;
 * tol > 0 turns a final residual above tol into CDL_E_NOCONV, after the
 * outputs are written.  A graph replay reuses the call's device pointers: the
 * snapshot series and outputs are read and written where they were when the
 * graph was captured.  Concurrent calls on one context race. */
cdl_status cdl_sequence_workspace_bytes(int32_t n_snap, const cdl_snapshot *snaps,
                                        const cdl_seq_params *p, size_t *bytes);
cdl_status cdl_score_sequence(cdl_ctx *ctx, int32_t n_snap, const cdl_snapshot *snaps,
                              const cdl_seq_params *p, double *const *F,
                              int32_t *const *top_idx, void *ws, size_t ws_bytes,
                              cdl_seq_info *info);

#ifdef __cplusplus
}
#endif

#endif /* CADDELAG_H */
