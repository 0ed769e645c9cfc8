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
struct SelectState {                // device scratch of the radix selection
    unsigned long long prefix;      // selected high bits so far
    unsigned long long rank;        // rank still to skip inside the prefix
    unsigned int hist[4096];
};

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_pad_series(const double *X, int64_t n, int64_t T, int64_t ldx,
                             double *Xp, int64_t rows, int64_t Tp, double *sqn,
                             int *flags, hipStream_t s);
hipError_t launch_gram_dist(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                            int64_t ld, double *D2, hipStream_t s);
hipError_t launch_select_median(const double *D2, int64_t ld, int64_t n,
                                SelectState *st, double *stats, hipStream_t s);
hipError_t launch_set_sigma(double sigma, double *stats, hipStream_t s);
hipError_t launch_exp_degree(double *W, int64_t ld, int64_t n, const double *stats,
                             double *deg, hipStream_t s);
hipError_t launch_graph_stats(const double *deg, int64_t n, double *stats, hipStream_t s);
hipError_t launch_import_weights(const double *Win, int64_t ldw, int64_t n, double *W,
                                 int64_t ld, double *deg, int *flags, hipStream_t s);

// ---- chain ------------------------------------------------------------------
// prec: 0 fp64, 1 fp32, 2 bf16, 3 fp16 (matches cdl_prec)
hipError_t launch_chain_prep(const double *deg, const double *stats, int64_t n, int64_t ld,
                             int lazy, double *dmn, double *dm, double *u, hipStream_t s);
float level_scale(int prec, int64_t n);   // storage scale of FP16 levels (1 otherwise)
hipError_t launch_normalize(int prec, const double *W, int64_t ld, int64_t n,
                            const double *dmn, const double *u, int lazy, void *S0,
                            double *fro_part, hipStream_t s);
int square_tiles(int prec, int64_t ld);   // number of partial norms written
hipError_t launch_square(int prec, const void *S, void *S2, int64_t ld, int64_t n,
                         double *fro_part, hipStream_t s);
// inv_vs != nullptr marks the last level: X += dm * V * (*inv_vs).
hipError_t launch_apply(int prec, const void *Vin, const void *S, void *Vout, double *V64,
                        int64_t ld, int64_t n, int64_t kpad, double *Xt, const double *dm,
                        const double *inv_vs, hipStream_t s);

// ---- solve ------------------------------------------------------------------
hipError_t launch_rhs(const double *W, int64_t ld, int64_t n, const int32_t *gid, int64_t k,
                      int64_t kpad, uint64_t seed, double *Yt, hipStream_t s);
hipError_t launch_residual_k(const double *Xt, const double *W, const double *Yt,
                             const double *deg, const double *dm, int64_t ld, int64_t n,
                             int64_t kpad, int64_t k, int skip_gemm, double *Rt, double *npart,
                             double *mpart, hipStream_t s);
int residual_parts(int64_t ld);               // column-norm partials per column
int residual_tiles(int64_t ld, int64_t kpad); // tile maxima written
hipError_t launch_col_norms2(const double *npart, int nparts, int64_t kpad, const double *mpart,
                             int ntiles, double *out, hipStream_t s);
hipError_t launch_prep_v2(int prec, const double *Rt, const double *dm, int64_t ld, int64_t kpad,
                          const double *scal, double *V64, void *Vlo, hipStream_t s);
hipError_t launch_finalize_z2(const double *Xt, int64_t ld, int64_t n, int64_t kpad, int64_t k,
                              double *mean, double *Z, hipStream_t s);

// ---- scores -------------------------------------------------------------------
hipError_t launch_build_zhat(const double *Z0, const double *Z1, const int32_t *map0,
                             const int32_t *map1, int64_t m, int64_t mpad, int64_t k,
                             int64_t kpad, const double *stats0, const double *stats1,
                             double *Zh, double *Zhe, double *sq, hipStream_t s);
int score_tiles_1d(int64_t mpad);
hipError_t launch_score(const double *Zh, const double *Zhe, int64_t kpad, const double *sq,
                        int64_t m, int64_t mpad, const double *W0, int64_t ld0,
                        const double *W1, int64_t ld1, const int32_t *map0,
                        const int32_t *map1, int weighted, double *part, hipStream_t s);
hipError_t launch_score_reduce(const double *part, int nparts, int64_t m, int64_t mpad,
                               double *F, hipStream_t s);
// Top-K by (descending value, ascending index); scratch holds 2 * cand_cap
// doubles + 2 * cand_cap ints, cand_cap = topk_scratch_elems(m, K).
int64_t topk_scratch_elems(int64_t m, int K);
hipError_t launch_topk(const double *F, int64_t m, int K, void *scratch, int32_t *out,
                       hipStream_t s);

} // namespace cdl
