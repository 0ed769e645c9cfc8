// Host-side launchers of the gfx950 kernels (one per kernel family).  All
// take the HIP stream to enqueue on and return hipSuccess or the launch error.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdl {

// Layout constants of the library (see common.h for the device side).
int64_t pad_n(int64_t n);           // padded n x n leading dimension
int64_t pad_k(int64_t k);           // padded number of projection columns
int64_t pad_t(int64_t T);           // padded series length (multiple of 16)

// ---- graph ------------------------------------------------------------------
constexpr int kSelCap = 4096;       // candidates sorted in the last selection step
struct SelectState {                // device scratch of the exact median selection
    unsigned long long prefix;      // selected high bits so far
    unsigned long long rank;        // rank still to skip inside the prefix
    unsigned long long kmin, kmax;  // smallest / largest key (from the Gram epilogue)
    int bits;                       // number of resolved high bits
    int mode;                       // 0 histogram, 1 collect, 2 done
    unsigned int count;             // collected candidates
    int src;                        // keys read from 0: the matrix, 1: the bracket buffer
    unsigned long long lo, hi;      // sampled bracket [lo, hi] around the target rank
    unsigned long long below;       // keys < lo
    unsigned long long nbuf;        // keys in [lo, hi] (appended to the bracket buffer)
    unsigned long long hist[4096];  // 64-bit: a bin can exceed 2^32 keys for n > 92681
    unsigned long long cand[kSelCap];
};
// Keys the bracket buffer of the selection holds for n nodes.
int64_t select_buffer_keys(int64_t n);

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// dst = src (bytes a multiple of 16, both 16-byte aligned, no overlap).
hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_pad_series(const double *X, int64_t n, int64_t T, int64_t ldx,
                             double *Xp, int64_t rows, int64_t Tp, double *sqn,
                             int *flags, hipStream_t s);
// st != nullptr: also record min/max upper-triangle keys for the selection
// (st must have been reset with launch_select_reset); brbuf != nullptr (with
// st, after launch_select_presample): also count the upper-triangle keys
// below the bracket and gather those inside it into brbuf (brcap keys).
hipError_t launch_gram_dist(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                            int64_t ld, double *D2, SelectState *st, unsigned long long *brbuf,
                            int64_t brcap, hipStream_t s);
// Row panel [row0, row0 + rows) of the same tiles (row0 and rows multiples of
// 256): the upper-triangle cover only (full = false) or every tile of the
// rows (full = true), row i stored at D2p + (i - row0) ld.  wstats != nullptr
// (full panels only): store the weights exp(-D2 / sigma^2) with the zero
// diagonal instead, sigma = wstats[1] (the same bits as launch_exp_rows).
hipError_t launch_gram_panel(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                             int64_t ld, int64_t row0, int64_t rows, bool full, double *D2p,
                             const double *wstats, hipStream_t s);
int64_t gram_panel_tiles(int64_t ld, int64_t row0, int64_t rows, bool full);
hipError_t launch_select_reset(SelectState *st, hipStream_t s);
// Streamed median: start at the top bit; per digit one launch_select_panel
// per row panel of D2 (rows [row0, row1) at D2p) and one launch_select_pick.
// st->mode == 2 once stats[1] holds the bandwidth.
hipError_t launch_select_start_top(SelectState *st, int64_t n, hipStream_t s);
hipError_t launch_select_panel(const double *D2p, int64_t ld, int64_t n, int64_t row0,
                               int64_t row1, SelectState *st, hipStream_t s);
hipError_t launch_select_pick(SelectState *st, double *stats, hipStream_t s);
// Streamed bracket: a sample of distances computed from the series brackets
// the median rank; one sweep of launch_select_bracket_panel over the upper
// panels counts keys below the bracket and gathers those inside into buf (at
// most cap = select_stream_keys(n)); launch_select_check moves the radix to
// the buffer (st->src = 1) when the rank lies inside and nothing overflowed;
// then launch_select_buffer_pass (one radix pass and pick) until st->mode = 2.
int64_t select_stream_keys(int64_t n);
hipError_t launch_select_sample_x(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                                  SelectState *st, hipStream_t s);
hipError_t launch_select_bracket_panel(const double *D2p, int64_t ld, int64_t n, int64_t row0,
                                       int64_t row1, SelectState *st, unsigned long long *buf,
                                       int64_t cap, hipStream_t s);
hipError_t launch_select_check(SelectState *st, int64_t cap, double *stats, hipStream_t s);
hipError_t launch_select_buffer_pass(SelectState *st, const unsigned long long *buf, int64_t cap,
                                     double *stats, hipStream_t s);
// Weights of a row panel in place from its squared distances (bit-identical
// to the stored matrix); optional row sums into deg[row0 + q] and, with
// dinv = D^{-1/2}, per-row squared Frobenius norms of S into fro[q].
hipError_t launch_exp_rows(double *Wp, int64_t ld, int64_t n, int64_t row0, int64_t rows,
                           const double *stats, double *deg, const double *dinv, double *fro,
                           hipStream_t s);
// The bracket of the median selection from a sample of pair distances taken
// from the padded series (buf: select_buffer_keys(n) words of scratch, its
// first 4096 words used); call before launch_gram_dist with brbuf = buf.
hipError_t launch_select_presample(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                                   SelectState *st, unsigned long long *buf, hipStream_t s);
// The exact lower median after the Gram: gathered = the Gram gathered the
// bracket into buf (radix passes over it when it holds the target rank),
// else radix passes over the matrix only.
hipError_t launch_select_median(const double *D2, int64_t ld, int64_t n,
                                SelectState *st, unsigned long long *buf, bool gathered,
                                double *stats, hipStream_t s);
hipError_t launch_set_sigma(double sigma, double *stats, hipStream_t s);
// part: (ld / 64) x ld doubles of degree partials.
int sym_tiles64(int64_t ld);   // upper 64 x 64 tiles of an ld x ld matrix
hipError_t launch_exp_degree(double *W, int64_t ld, int64_t n, const double *stats,
                             double *deg, double *part, hipStream_t s);
hipError_t launch_graph_stats(const double *deg, int64_t n, double *stats, hipStream_t s);
hipError_t launch_import_weights(const double *Win, int64_t ldw, int64_t n, double *W,
                                 int64_t ld, double *deg, int *flags, hipStream_t s);

// ---- chain ------------------------------------------------------------------
// prec: 0 fp64, 1 fp32, 2 bf16, 3 fp16 (matches cdl_prec)
hipError_t launch_chain_prep(const double *deg, const double *stats, int64_t n, int64_t ld,
                             int lazy, double *dmn, double *dm, double *u, hipStream_t s);
float level_scale(int prec, int64_t n);   // storage scale of FP16 levels (1 otherwise)
// Reads the upper 64 x 64 tiles of W only and writes S0 with its mirror.
// fro_part / fro64_part: one squared Frobenius sum of the stored (rounded)
// and of the unrounded FP64 level per upper tile (doubled off the diagonal),
// sym_tiles64(ld) entries each.
hipError_t launch_normalize(int prec, const double *W, int64_t ld, int64_t n,
                            const double *dmn, const double *u, int lazy, void *S0,
                            double *fro_part, double *fro64_part, hipStream_t s);
int square_tiles(int prec, int64_t ld);   // number of partial norms written
// Level 0 from a row panel of W (rows [row0, row0 + rows), full rows): the
// values of launch_normalize; per-row sums of squares (rounded, exact) into
// fro_part[q], fro64_part[q].
hipError_t launch_normalize_rows(int prec, const double *Wp, int64_t ld, int64_t n, int64_t row0,
                                 int64_t rows, const double *dmn, const double *u, int lazy,
                                 void *S0, double *fro_part, double *fro64_part, hipStream_t s);
// Bytes of the FP32 partial tiles that a 16-bit squaring of an n-node level
// uses for its last, partial round of workgroups (split over k); 0 if none.
size_t square_tail_bytes(int prec, int64_t ld, int64_t n);
// tail: square_tail_bytes() of scratch (nullptr: no split).
// variant < square_variants(prec): for 16-bit levels bit 0 set = no k-split
// of the last round, bit 1 set = the 4-wave tile core.
int square_variants(int prec);
hipError_t launch_square(int prec, const void *S, void *S2, int64_t ld, int64_t n,
                         double *fro_part, float *tail, int variant, hipStream_t s);
// C = Q + L + Q L for commuting symmetric Q, L (levels' storage scale).
hipError_t launch_chain_product(int prec, const void *Q, const void *L, void *C, int64_t ld,
                                int64_t n, double *fro_part, float *tail, int variant,
                                hipStream_t s);
// accumulate: V64 += S~ Vin (else V64 = S~ Vin); Vout = V64 rounded.
// inv_vs != nullptr marks the last level: X += dm * V * (*inv_vs).  P is the
// split-K partial buffer (nsplit x kpad x ld floats; unused for FP64).
hipError_t launch_apply(int prec, const void *Vin, const void *S, void *Vout, double *V64,
                        int64_t ld, int64_t n, int64_t kpad, double *Xt, const double *dm,
                        const double *inv_vs, float *P, int accumulate, int nsplit,
                        hipStream_t s);
// The split-K product of one application alone (partials into P), for timing.
hipError_t launch_apply_gemm(int prec, const void *Vin, const void *S, int64_t ld, int64_t n,
                             int64_t kpad, int nsplit, float *P, hipStream_t s);
// V64 += T64, Vout = V64 rounded, last level: X += dm * V64 * (*inv_vs).
hipError_t launch_axpy_v(int prec, const double *T64, int64_t ld, int64_t kpad, double *V64,
                         void *Vout, double *Xt, const double *dm, const double *inv_vs,
                         hipStream_t s);
// Split-K count of the chain application (choices as for residual_splits).
int apply_splits(int prec, int64_t ld, int64_t kpad, int64_t n, int choice);

// ---- solve ------------------------------------------------------------------
hipError_t launch_rhs(const double *W, int64_t ld, int64_t n, const int32_t *gid, int64_t k,
                      int64_t kpad, uint64_t seed, double *Yt, hipStream_t s);
// Y0 and Y1 of two snapshots on one node set (the same ids, so the same
// sign words) in one sweep over W0 and W1.
hipError_t launch_rhs_pair(const double *W0, const double *W1, int64_t ld, int64_t n,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Y0t, double *Y1t, hipStream_t s);
// Rows [row0, row1) of Y from a row panel of W (row i at Wp + (i - row0) ld).
hipError_t launch_rhs_rows(const double *Wp, int64_t ld, int64_t n, int64_t row0, int64_t row1,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Yt, hipStream_t s);
// Prod[r][row0 + q] = sum_j Vt[r][j] Wp[q][j] for the rows of a panel
// (rows a multiple of 128; one FP64 MFMA pass, no split).
hipError_t launch_panel_product(const double *Vt, const double *Wp, int64_t ld, int64_t n,
                                int64_t kpad, int64_t row0, int64_t rows, double *Prod,
                                hipStream_t s);
// The residual reduction with S explicit split partials (S = 1: P is W X);
// dm (ld entries) scales the maxima written to mpart.
hipError_t launch_residual_reduce(const double *P, int S, const double *Yt, const double *Xt,
                                  const double *deg, const double *dm, int64_t ld, int64_t n,
                                  int64_t kpad, int64_t k, double *Rt, double *npart,
                                  double *mpart, hipStream_t s);
// Streamed solve steps: dinv = D^{-1/2}, rdeg = D^{-1}; Ut = rdeg * Rt;
// Xt += Ut + rdeg * Prod (Xt += P1 r for the one-level chain).
hipError_t launch_stream_prep(const double *deg, int64_t n, int64_t ld, double *dinv,
                              double *rdeg, hipStream_t s);
hipError_t launch_stream_scale(const double *Rt, const double *rdeg, int64_t ld, int64_t kpad,
                               double *Ut, hipStream_t s);
hipError_t launch_stream_update(const double *Ut, const double *Prod, const double *rdeg,
                                int64_t ld, int64_t kpad, double *Xt, hipStream_t s);
// R = Y - deg * X + W X (skip_gemm: R = Y - deg * X).  P: residual_splits()
// x kpad x ld doubles of split-K partials.  For prec 0..2 the reduction also
// writes V = dm * R (V64) and its rounded copy (Vlo); prec 3 leaves V alone.
hipError_t launch_residual_k(int prec, const double *Xt, const double *W, const double *Yt,
                             const double *deg, const double *dm, int64_t ld, int64_t n,
                             int64_t kpad, int64_t k, int skip_gemm, double *P, double *Rt,
                             double *V64, void *Vlo, double *npart, double *mpart,
                             hipStream_t s);
// Split-K count of the residual product: choice 0 the default, 1 half of
// it, 2 twice it (the candidates of the tuner; workspaces hold choice 2).
int residual_splits(int64_t ld, int64_t kpad, int64_t n, int choice);
// The two halves of launch_residual_k: the split-K product W X into S
// partials of P, and the reduction over S partials (S = 0: none,
// R = Y - deg X) that forms R, the operand V and the norm partials.
hipError_t launch_residual_gemm(const double *Xt, const double *W, int64_t ld, int64_t n,
                                int64_t kpad, int S, double *P, hipStream_t s);
hipError_t launch_residual_reduce_k(int prec, const double *P, int S, const double *Yt,
                                    const double *Xt, const double *deg, const double *dm,
                                    int64_t ld, int64_t n, int64_t kpad, int64_t k, double *Rt,
                                    double *V64, void *Vlo, double *npart, double *mpart,
                                    hipStream_t s);
int residual_parts(int64_t ld);               // column-norm partials per column
int residual_tiles(int64_t ld, int64_t kpad); // maxima written
hipError_t launch_col_norms2(const double *npart, int nparts, int64_t kpad, const double *mpart,
                             int ntiles, int scaled, double *out, hipStream_t s);
hipError_t launch_prep_v2(int prec, const double *Rt, const double *dm, int64_t ld, int64_t kpad,
                          const double *scal, double *V64, void *Vlo, hipStream_t s);
// Z[i][r] = Xt[r][i] for i < n, r < k (Z n x k row-major).
hipError_t launch_transpose(const double *Xt, int64_t ld, int64_t n, int64_t k, double *Z,
                            hipStream_t s);
hipError_t launch_finalize_z2(const double *Xt, int64_t ld, int64_t n, int64_t kpad, int64_t k,
                              double *mean, double *Z, hipStream_t s);

// ---- scores -------------------------------------------------------------------
hipError_t launch_build_zhat(const double *Z0, const double *Z1, const int32_t *map0,
                             const int32_t *map1, int64_t m, int64_t mpad, int64_t k,
                             int64_t kpad, const double *stats0, const double *stats1,
                             double *Zh, double *Zhe, double *sq, hipStream_t s);
// Partial-sum slots of mpad entries each (mpad / 128 + mpad / 256).
int score_tiles_1d(int64_t mpad);
// *flag = 1 if an entry of map0 (map1) is outside [0, n0) ([0, n1)), else 0.
hipError_t launch_check_maps(const int32_t *map0, const int32_t *map1, int64_t m, int64_t n0,
                             int64_t n1, int *flag, hipStream_t s);
// Score tiles: 256 x 128 over the upper triangle (rect_upper_tiles).
// tmax: per-tile maximum edge score (a < b), score_tiles_2d(mpad) entries,
// or nullptr.
hipError_t launch_score(const double *Zh, const double *Zhe, int64_t kpad, const double *sq,
                        int64_t m, int64_t mpad, const double *W0, int64_t ld0,
                        const double *W1, int64_t ld1, const int32_t *map0,
                        const int32_t *map1, int weighted, double *part, double *tmax,
                        hipStream_t s);
int score_tiles_2d(int64_t mpad);
// tile_order: tile indices by descending maximum (first K used); sets tau
// and clears *count, then appends the edges with score >= tau to
// (cval, cidx) through *count (at most cap stored).
hipError_t launch_edge_collect(const double *Zh, const double *Zhe, int64_t kpad,
                               const double *sq, int64_t m, int64_t mpad, const double *W0,
                               int64_t ld0, const double *W1, int64_t ld1,
                               const int32_t *map0, const int32_t *map1, int weighted,
                               const double *tmax, const int32_t *tile_order, int K,
                               double *tau, int64_t cap, unsigned int *count, double *cval,
                               int64_t *cidx, hipStream_t s);
hipError_t launch_edge_split(const int64_t *idx, int64_t m, int K, int32_t *a, int32_t *b,
                             hipStream_t s);
hipError_t launch_topk64(const double *val, const int64_t *idx, int64_t cap,
                         const unsigned int *dcount, int K, void *scratch, double *val_out,
                         int64_t *idx_out, hipStream_t s);
hipError_t launch_score_reduce(const double *part, int nparts, int64_t m, int64_t mpad,
                               double *F, hipStream_t s);
// Top-K by (descending value, ascending index); scratch holds 2 * cand_cap
// doubles + 2 * cand_cap ints, cand_cap = topk_scratch_elems(m, K).
int64_t topk_scratch_elems(int64_t m, int K);
hipError_t launch_topk(const double *F, int64_t m, int K, void *scratch, int32_t *out,
                       hipStream_t s);

// Preconditioned conjugate gradients (per column, FP64).
hipError_t launch_col_dots(const double *A0, const double *B0, const double *A1,
                           const double *B1, int64_t ld, int64_t kpad, double *part,
                           hipStream_t s);
hipError_t launch_pcg_scalars(const double *part, int64_t ld, int64_t kpad, int mode, int first,
                              double *sc, hipStream_t s);
hipError_t launch_pcg_dir(const double *Zt, double *Pt, const double *beta, int64_t ld,
                          int64_t kpad, int first, hipStream_t s);
hipError_t launch_pcg_update(int prec, const double *Pt, const double *Qt, const double *alpha,
                             const double *dm, int64_t ld, int64_t kpad, double *Xt, double *Rt,
                             double *V64, void *Vlo, double *npart, double *mpart, hipStream_t s);

} // namespace cdl
