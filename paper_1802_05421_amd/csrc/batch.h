// Grouped launches over the snapshots (and pairs) of a sequence: one launch
// of a kernel family covers the tiles of every snapshot, found through a
// prefix table of per-snapshot workgroup counts; snapshots whose solve has
// converged (a device-side flag) skip their workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdl {

// Everything the grouped chain and solve kernels need of one snapshot.
struct BatchSnap {
    int64_t n, ld;
    const double *W, *deg;
    char *levels;              // chain levels (level l at levels + l * level_bytes)
    int64_t level_bytes;
    const double *dm;          // chain's (cD)^{-1/2}
    double *fro;               // squaring's per-tile norm partials
    float inv_scale;           // 1 / storage scale of the levels
    double *Yt, *Xt, *Rt, *V64;
    void *Vlo[2];              // rounded operand ping-pong
    float *Pap;                // split-K partials of the application
    double *Pres;              // split-K partials of the residual product
    double *npart, *mpart, *scal;
    int ap_splits, res_splits;
};

struct SelectState;

// Everything the grouped graph build (padding, distance Gram, median
// selection, weights, degrees, statistics) and the level-0 chain of one
// snapshot need.
struct GraphSnap {
    const double *X;           // series, n x T, row pitch ldx
    int64_t n, T, ldx, Tp, ld;
    double *Xp, *sqn;          // padded series (ld x Tp) and squared row norms
    int *flags;                // non-finite input flag
    double *W, *deg, *stats;   // distances, then weights in place; degrees; statistics
    SelectState *sel;
    unsigned long long *buf;   // bracket buffer of the selection
    int64_t cap;               // its capacity (keys)
    int bracket;               // the selection starts with a sampled bracket
    double *dpart;             // degree partials
    // level 0 of the chain
    double *dmn, *dm, *u;
    void *level0;
    double *fro, *fro64;
    double scale;              // storage scale of the level
};

// Prefix tables of the grouped graph build (one per workgroup count):
enum GraphTable {
    kGtRows,      // padded rows: ld
    kGtOne,       // one workgroup per snapshot
    kGtGram,      // upper-triangle 256 x 128 tiles
    kGtSample,    // one per snapshot whose selection starts with a sampled bracket
    kGtKeys,      // 16 per such snapshot (its sample's keys from the series)
    kGtPass,      // min(n, 2048) per snapshot
    kGtSym,       // upper 64 x 64 tiles
    kGtNodes64,   // ceil(n / 64)
    kGtPrep,      // ceil(ld / 256)
    kGraphTables
};
// Workgroup counts of table `tb` for a snapshot (bracket: its selection
// starts with the sampled bracket).
int graph_table_count(int tb, int64_t n, int64_t ld, bool bracket);
// Whether the stored selection of n keys' matrix starts with a sampled
// bracket (the bracket must fit the buffer).
bool select_uses_bracket(int64_t n, bool allowed);

// The graph of every snapshot: padding, Gram (with the key bounds when
// selecting), the exact lower median (sigma <= 0) or the given sigma,
// weights, degrees and statistics.  tables: kGraphTables x (P + 1) prefix
// tables in device memory; totals: their last entries (host).
hipError_t launch_graph_grouped(const GraphSnap *snaps, const int *tables, const int *totals,
                                int P, double sigma, hipStream_t s);
// Level 0 of every snapshot's chain: (cD)^{-1/2}, u and the normalised,
// deflated, rounded level with its norm partials.
hipError_t launch_chain_level0_grouped(int prec, const GraphSnap *snaps, const int *tables,
                                       const int *totals, int P, hipStream_t s);

// One pair of consecutive snapshots for the grouped score kernels.
struct BatchPair {
    int64_t m, mpad;
    const double *Z0, *Z1;
    const int32_t *map0, *map1;
    const double *stats0, *stats1;
    const double *W0, *W1;     // weighted mode only
    int64_t ld0, ld1;
    double *Zh, *Zhe, *sq, *part;
    double *F;
};

// Problem index of workgroup b: prefix[p] <= b < prefix[p + 1] (P problems).
__device__ inline int group_find(const int *prefix, int P, int b) {
    int p = 0;
    while (p + 1 < P && b >= prefix[p + 1]) ++p;
    return p;
}

// ---- host launchers (grouped kernels; every pointer table in device memory) --

// One squaring of level `level` into level + 1 for every snapshot; prefix over
// each snapshot's upper-tile count (square_tiles).  Stream-ordered.
hipError_t launch_square_grouped(int prec, const BatchSnap *snaps, const int *prefix, int P,
                                 int total, int level, hipStream_t s);
// The chain application of one level for every unconverged snapshot: the
// split-K product (prefix over mt * nt * ap_splits) then the update of
// V64 / Vlo[out] / X (prefix over the reduction's workgroups, last level
// when `last`).
hipError_t launch_apply_grouped(int prec, const BatchSnap *snaps, const int *prefix_gemm,
                                int total_gemm, const int *prefix_red, int total_red, int P,
                                int64_t kpad, int level, int in, int accumulate, int last,
                                const int *done, hipStream_t s);
// Workgroups of one snapshot's share of the application's update (also the
// FP16 operand preparation's), at most `cap`; the kernels stride over them.
int apply_reduce_blocks(int64_t ld, int64_t kpad, int cap = 2048);
int apply_gemm_tiles(int64_t ld, int64_t kpad, int nsplit);
int residual_gemm_tiles(int64_t ld, int64_t kpad, int S);
// Split-K counts S clamped to what a snapshot of n nodes allows (a grouped
// launch picks one S for all snapshots from the tiles of the whole group).
int apply_splits_fixed(int prec, int64_t n, int S);
int residual_splits_fixed(int64_t n, int S);
// R = Y - deg X + W X, V = dm R (rounded copy into Vlo[0]) and the norm
// partials, for every unconverged snapshot; skip_gemm: R = Y (initial).
hipError_t launch_residual_grouped(int prec, const BatchSnap *snaps, const int *prefix_gemm,
                                   int total_gemm, const int *prefix_red, int total_red, int P,
                                   int64_t kpad, int64_t k, int skip_gemm, const int *done,
                                   hipStream_t s);
// Column norms (and the FP16 operand scale) of every unconverged snapshot,
// then per snapshot: rel = max_r ||R_r|| / ||Y_r|| (ynorm: P x kpad), and
// done[p] = rel <= tol (tol > 0), iters[p] += 1 when it was not done before.
// init: ynorm = the norms (no convergence test).
hipError_t launch_norms_grouped(const BatchSnap *snaps, int P, int64_t kpad, int64_t k,
                                int scaled, double tol, int init, double *ynorm,
                                double *rel_out, int *done, int *iters, hipStream_t s);
// FP16 operand: V = scale * dm R and its rounded copy, unconverged snapshots.
hipError_t launch_prep_grouped(int prec, const BatchSnap *snaps, const int *prefix, int total,
                               int P, int64_t kpad, const int *done, hipStream_t s);
// Scores of every pair: signature embeddings, the FP64 Gram tiles over the
// upper triangles and the row sums.
hipError_t launch_score_grouped(const BatchPair *pairs, const int *prefix_zhat, int total_zhat,
                                const int *prefix_score, int total_score,
                                const int *prefix_red, int total_red, int P, int64_t k,
                                int64_t kpad, int weighted, hipStream_t s);

}  // namespace cdl
