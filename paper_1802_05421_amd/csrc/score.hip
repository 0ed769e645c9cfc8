// Node anomaly scores (Algorithm 4 with the CAD edge score of the Background
// section), without materialising any n x n commute-time matrix.
//
//   build_zhat  Zh = [sqrt(vol0) Z0 | sqrt(vol1) Z1] over the common nodes,
//               Zhe = Zh with the second half negated, sq_c = Zh_c . Zhe_c
//   score       G = Zh Zhe^T on FP64 MFMA over 256 x 128 tiles covering the
//               upper triangle; per pair a < b, dc_ab = sq_a + sq_b - 2 G_ab
//               = c_0(a,b) - c_1(a,b) (eq. 1 in embedding form), weighted by
//               |W1 - W0| on request; |dc| is summed per row into one
//               partial per (column block, node) and per column into one
//               partial per (row block, node)
//   reduce      F_a = sum of exactly the written partials (fixed order)
//   topk        bitonic sort of chunks in LDS, keep the best K per chunk,
//               repeat on the candidates (order: value desc, index asc)
//   edges       the K largest edge scores (a < b) exactly: per-tile maxima
//               from k_score, threshold = K-th largest tile maximum, only
//               tiles reaching it recomputed and their edges collected
#include "batch.h"
#include "caddelag.h"
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace cdl {

// Row c of the signature embeddings (one wave).
__device__ inline void build_zhat_row(const double *Z0, const double *Z1, const int32_t *map0,
                                      const int32_t *map1, int64_t m, int64_t k, int64_t kpad,
                                      const double *stats0, const double *stats1, double *Zh,
                                      double *Zhe, double *sq, int64_t c) {
    const int lane = threadIdx.x;
    const double s0 = sqrt(stats0[0]), s1 = sqrt(stats1[0]);
    const int64_t ldz = 2 * kpad;
    double acc = 0.0;
    int64_t a = -1, b = -1;
    if (c < m) {
        a = map0 ? map0[c] : c;
        b = map1 ? map1[c] : c;
    }
    for (int64_t r = lane; r < kpad; r += 64) {
        double x0 = 0.0, x1 = 0.0;
        if (c < m && r < k) {
            x0 = s0 * Z0[a * k + r];
            x1 = s1 * Z1[b * k + r];
        }
        Zh[c * ldz + r] = x0;
        Zh[c * ldz + kpad + r] = x1;
        Zhe[c * ldz + r] = x0;
        Zhe[c * ldz + kpad + r] = -x1;
        acc += x0 * x0 - x1 * x1;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) sq[c] = acc;
}

// One wave per common node.
__global__ void k_build_zhat(const double *Z0, const double *Z1, const int32_t *map0,
                             const int32_t *map1, int64_t m, int64_t k, int64_t kpad,
                             const double *stats0, const double *stats1, double *Zh,
                             double *Zhe, double *sq) {
    build_zhat_row(Z0, Z1, map0, map1, m, k, kpad, stats0, stats1, Zh, Zhe, sq, blockIdx.x);
}

hipError_t launch_build_zhat(const double *Z0, const double *Z1, const int32_t *map0,
                             const int32_t *map1, int64_t m, int64_t mpad, int64_t k,
                             int64_t kpad, const double *stats0, const double *stats1,
                             double *Zh, double *Zhe, double *sq, hipStream_t s) {
    hipLaunchKernelGGL(k_build_zhat, dim3((unsigned)mpad), dim3(64), 0, s, Z0, Z1, map0, map1,
                       m, k, kpad, stats0, stats1, Zh, Zhe, sq);
    return hipGetLastError();
}

// 256 x 128 tiles covering the upper triangle (upper_band_tile); each wave
// 64 x 64.  Only pairs a < b count: a tile straddling the diagonal also holds
// pairs a > b, whose mirror images another tile covers.
using ScoreCore = GemmCore<MfmaF64, 256, 128, 16, 4, 2>;
constexpr int kScoreWM = 4, kScoreWN = 2;

// Edge score omega_ab |c_0(a,b) - c_1(a,b)| of common nodes a != b from the
// signature Gram entry G_ab (shared by the node and the edge kernels, so
// both see bit-identical values).
__device__ inline double edge_score(int64_t ga, int64_t gb, double G, double sqa, double sqb,
                                    const double *W0, int64_t ld0, const double *W1,
                                    int64_t ld1, const int32_t *map0, const int32_t *map1,
                                    int weighted) {
    double v = fabs(sqa + sqb - 2.0 * G);
    if (weighted) {
        const int64_t a0 = map0 ? map0[ga] : ga, b0 = map0 ? map0[gb] : gb;
        const int64_t a1 = map1 ? map1[ga] : ga, b1 = map1 ? map1[gb] : gb;
        v *= fabs(W1[a1 * ld1 + b1] - W0[a0 * ld0 + b0]);
    }
    return v;
}

// Partial sums: row a's sum over the columns of tile (I, J) goes to
// part[J][a], column b's sum over the rows of the tile to part[ncol + I][b];
// each slot has exactly one writer.  tmax != nullptr: also the largest edge
// score of the tile over a < b, at the tile's logical index.
struct ScoreShared {
    double srow[kScoreWN][256], scol[kScoreWM][128], smax[8];
};

// Upper-triangle tile `id` of the score Gram with its partial sums (one
// workgroup).
__device__ __forceinline__ void score_tile(const double *Zh, const double *Zhe, int64_t ldz,
                                  const double *sq, int64_t m, int64_t mpad, const double *W0,
                                  int64_t ld0, const double *W1, int64_t ld1,
                                  const int32_t *map0, const int32_t *map1, int weighted,
                                  int ncol, double *part, double *tmax, int id, char *smem_raw,
                                  ScoreShared &sh) {
    double *smem = (double *)smem_raw;
    auto &srow = sh.srow;
    auto &scol = sh.scol;
    auto &smax = sh.smax;
    int I, J;
    upper_band_tile<4>(id, 0, ncol / 2, ncol, I, J);
    const int64_t m0 = (int64_t)I * 256, n0 = (int64_t)J * 128;
    ScoreCore g;
    g.run(Zh, ldz, Zhe, ldz, m0, n0, ldz, smem);

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid % kScoreWM, wn = wid / kScoreWM;
    double cs[ScoreCore::WTN], vmax = -1.0, sqb[ScoreCore::WTN];
#pragma unroll
    for (int b = 0; b < ScoreCore::WTN; ++b) {
        cs[b] = 0.0;
        sqb[b] = sq[n0 + ScoreCore::col_of(b)];
    }
#pragma unroll
    for (int a = 0; a < ScoreCore::WTM; ++a)
#pragma unroll
        for (int rr = 0; rr < MfmaF64::R; ++rr) {
            const int lr = ScoreCore::row_of(a, rr);
            const int64_t ga = m0 + lr;
            const double sqa = sq[ga];
            double rs = 0.0;
#pragma unroll
            for (int b = 0; b < ScoreCore::WTN; ++b) {
                const int64_t gb = n0 + ScoreCore::col_of(b);
                double v = 0.0;
                if (ga < gb && gb < m) {
                    v = edge_score(ga, gb, g.acc[a][b][rr], sqa, sqb[b], W0, ld0, W1, ld1, map0,
                                   map1, weighted);
                    vmax = fmax(vmax, v);
                }
                rs += v;
                cs[b] += v;
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) rs += __shfl_xor(rs, off);
            if ((lane & 15) == 0) srow[wn][lr] = rs;
        }
#pragma unroll
    for (int b = 0; b < ScoreCore::WTN; ++b) {
        double v = cs[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lane < 16) scol[wm][ScoreCore::col_of(b)] = v;
    }
    if (tmax) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
        if (lane == 0) smax[wid] = vmax;
    }
    __syncthreads();
    if (tmax && threadIdx.x == 0) {
        double mx = smax[0];
        for (int q = 1; q < ScoreCore::NT / 64; ++q) mx = fmax(mx, smax[q]);
        tmax[id] = mx;
    }
    for (int t = threadIdx.x; t < 256; t += ScoreCore::NT) {
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < kScoreWN; ++q) rs += srow[q][t];
        part[(int64_t)J * mpad + m0 + t] = rs;
    }
    for (int t = threadIdx.x; t < 128; t += ScoreCore::NT) {
        double cs2 = 0.0;
#pragma unroll
        for (int q = 0; q < kScoreWM; ++q) cs2 += scol[q][t];
        part[(int64_t)(ncol + I) * mpad + n0 + t] = cs2;
    }
}

__global__ __launch_bounds__(512) void k_score(const double *Zh, const double *Zhe,
                                               int64_t ldz, const double *sq, int64_t m,
                                               int64_t mpad, const double *W0, int64_t ld0,
                                               const double *W1, int64_t ld1,
                                               const int32_t *map0, const int32_t *map1,
                                               int weighted, int ncol, double *part,
                                               double *tmax) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    __shared__ ScoreShared sh;
    const int id = xcd_remap(blockIdx.x, rect_upper_tiles(mpad));
    score_tile(Zh, Zhe, ldz, sq, m, mpad, W0, ld0, W1, ld1, map0, map1, weighted, ncol, part, tmax,
               id, smem_raw, sh);
}

int score_tiles_1d(int64_t mpad) { return (int)(mpad / 128 + mpad / 256); }

hipError_t launch_score(const double *Zh, const double *Zhe, int64_t kpad, const double *sq,
                        int64_t m, int64_t mpad, const double *W0, int64_t ld0,
                        const double *W1, int64_t ld1, const int32_t *map0,
                        const int32_t *map1, int weighted, double *part, double *tmax,
                        hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_score,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ScoreCore::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ncol = (int)(mpad / 128);
    const int total = rect_upper_tiles(mpad);
    hipLaunchKernelGGL(k_score, dim3(total), dim3(ScoreCore::NT), ScoreCore::SMEM, s, Zh, Zhe, 2 * kpad,
                       sq, m, mpad, W0, ld0, W1, ld1, map0, map1, weighted, ncol, part, tmax);
    return hipGetLastError();
}

int score_tiles_2d(int64_t mpad) { return rect_upper_tiles(mpad); }

// ---------------------------------------------------------------------------
// Top edges.  The K largest tile maxima are K distinct edges, so the K-th
// largest edge score is at least tau = the K-th largest tile maximum (when
// there are fewer than K tiles, tau = -1 and every edge is collected).  Only tiles whose maximum reaches tau are
// recomputed (same core, same epilogue arithmetic as k_score); their edges
// a < b with score >= tau are appended to the candidate list.

__global__ void k_edge_threshold(const double *tmax, const int32_t *tile_order, int K,
                                 int ntiles, double *tau, unsigned int *count) {
    if (threadIdx.x != 0) return;
    *tau = ntiles >= K ? tmax[tile_order[K - 1]] : -1.0;
    *count = 0;
}

__global__ __launch_bounds__(512) void k_edge_collect(
    const double *Zh, const double *Zhe, int64_t ldz, const double *sq, int64_t m,
    const double *W0, int64_t ld0, const double *W1, int64_t ld1, const int32_t *map0,
    const int32_t *map1, int weighted, int ncol, int64_t mpad, const double *tmax,
    const double *tau, int64_t cap, unsigned int *count, double *cval, int64_t *cidx) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    double *smem = (double *)smem_raw;
    const int total = rect_upper_tiles(mpad);
    const int id = xcd_remap(blockIdx.x, total);
    const double th = *tau;
    if (tmax[id] < th) return;   // uniform over the workgroup
    int I, J;
    upper_band_tile<4>(id, 0, ncol / 2, ncol, I, J);
    const int64_t m0 = (int64_t)I * 256, n0 = (int64_t)J * 128;
    ScoreCore g;
    g.run(Zh, ldz, Zhe, ldz, m0, n0, ldz, smem);
#pragma unroll
    for (int a = 0; a < ScoreCore::WTM; ++a)
#pragma unroll
        for (int rr = 0; rr < MfmaF64::R; ++rr) {
            const int64_t ga = m0 + ScoreCore::row_of(a, rr);
#pragma unroll
            for (int b = 0; b < ScoreCore::WTN; ++b) {
                const int64_t gb = n0 + ScoreCore::col_of(b);
                if (ga < m && gb < m && ga < gb) {
                    const double v = edge_score(ga, gb, g.acc[a][b][rr], sq[ga], sq[gb], W0, ld0,
                                                W1, ld1, map0, map1, weighted);
                    if (v >= th) {
                        const unsigned int q = atomicAdd(count, 1u);
                        if ((int64_t)q < cap) {
                            cval[q] = v;
                            cidx[q] = ga * m + gb;
                        }
                    }
                }
            }
        }
}

hipError_t launch_edge_collect(const double *Zh, const double *Zhe, int64_t kpad,
                               const double *sq, int64_t m, int64_t mpad, const double *W0,
                               int64_t ld0, const double *W1, int64_t ld1,
                               const int32_t *map0, const int32_t *map1, int weighted,
                               const double *tmax, const int32_t *tile_order, int K,
                               double *tau, int64_t cap, unsigned int *count, double *cval,
                               int64_t *cidx, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_edge_collect,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ScoreCore::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ncol = (int)(mpad / 128);
    const int total = rect_upper_tiles(mpad);
    hipLaunchKernelGGL(k_edge_threshold, dim3(1), dim3(64), 0, s, tmax, tile_order, K, total, tau,
                       count);
    hipLaunchKernelGGL(k_edge_collect, dim3(total), dim3(ScoreCore::NT), ScoreCore::SMEM, s, Zh,
                       Zhe, 2 * kpad, sq, m, W0, ld0, W1, ld1, map0, map1, weighted, ncol, mpad,
                       tmax, tau, cap, count, cval, cidx);
    return hipGetLastError();
}

// flag = 1 if some entry of map0 lies outside [0, n0) or of map1 outside
// [0, n1), else 0.  One workgroup; the flag needs no initial value.
__global__ __launch_bounds__(256) void k_check_maps(const int32_t *map0, const int32_t *map1,
                                                    int64_t m, int64_t n0, int64_t n1,
                                                    int *flag) {
    int bad = 0;
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        const int32_t a = map0[c], b = map1[c];
        bad |= (a < 0 || a >= n0 || b < 0 || b >= n1);
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *flag = bad ? 1 : 0;
}

hipError_t launch_check_maps(const int32_t *map0, const int32_t *map1, int64_t m, int64_t n0,
                             int64_t n1, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_maps, dim3(1), dim3(256), 0, s, map0, map1, m, n0, n1, flag);
    return hipGetLastError();
}

// F_a = its row partials over the column blocks J >= 2 (a / 256), then its
// column partials over the row blocks I <= (a / 128) / 2: exactly the slots
// the score tiles wrote, summed in a fixed order.
__device__ inline void score_reduce_node(const double *part, int ncol, int64_t m, int64_t mpad,
                                         double *F, int64_t a) {
    if (a >= m) return;
    const int J0 = (int)(a / 256) * 2;
    double s = J0 < ncol ? ordered_sum(part + (int64_t)J0 * mpad + a, mpad, ncol - J0, 0.0) : 0.0;
    const int Imax = (int)(a / 128) / 2;
    s = ordered_sum(part + (int64_t)ncol * mpad + a, mpad, Imax + 1, s);
    F[a] = s;
}

__global__ void k_score_reduce(const double *part, int ncol, int64_t m, int64_t mpad,
                               double *F) {
    score_reduce_node(part, ncol, m, mpad, F, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---- grouped over the pairs of a sequence ------------------------------------

__global__ void k_build_zhat_grouped(const BatchPair *pairs, const int *prefix, int P, int64_t k,
                                     int64_t kpad) {
    const int p = group_find(prefix, P, blockIdx.x);
    const BatchPair &q = pairs[p];
    build_zhat_row(q.Z0, q.Z1, q.map0, q.map1, q.m, k, kpad, q.stats0, q.stats1, q.Zh, q.Zhe, q.sq,
                   blockIdx.x - prefix[p]);
}

__global__ __launch_bounds__(512) void k_score_grouped(const BatchPair *pairs, const int *prefix, int P,
                                                       int64_t kpad, int weighted) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    __shared__ ScoreShared sh;
    const int p = group_find(prefix, P, blockIdx.x);
    const BatchPair &q = pairs[p];
    const int id = xcd_remap(blockIdx.x - prefix[p], prefix[p + 1] - prefix[p]);
    score_tile(q.Zh, q.Zhe, 2 * kpad, q.sq, q.m, q.mpad, q.W0, q.ld0, q.W1, q.ld1, q.map0, q.map1,
               weighted, (int)(q.mpad / 128), q.part, nullptr, id, smem_raw, sh);
}

__global__ void k_score_reduce_grouped(const BatchPair *pairs, const int *prefix, int P) {
    const int p = group_find(prefix, P, blockIdx.x);
    const BatchPair &q = pairs[p];
    score_reduce_node(q.part, (int)(q.mpad / 128), q.m, q.mpad, q.F,
                      (int64_t)(blockIdx.x - prefix[p]) * blockDim.x + threadIdx.x);
}

hipError_t launch_score_grouped(const BatchPair *pairs, const int *prefix_zhat, int total_zhat,
                                const int *prefix_score, int total_score,
                                const int *prefix_red, int total_red, int P, int64_t k,
                                int64_t kpad, int weighted, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_score_grouped,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ScoreCore::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_build_zhat_grouped, dim3(total_zhat), dim3(64), 0, s, pairs, prefix_zhat, P,
                       k, kpad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_score_grouped, dim3(total_score), dim3(ScoreCore::NT), ScoreCore::SMEM, s,
                       pairs, prefix_score, P, kpad, weighted);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_score_reduce_grouped, dim3(total_red), dim3(64), 0, s, pairs, prefix_red, P);
    return hipGetLastError();
}

hipError_t launch_score_reduce(const double *part, int nparts, int64_t m, int64_t mpad,
                               double *F, hipStream_t s) {
    (void)nparts;   // the slot layout follows from mpad
    hipLaunchKernelGGL(k_score_reduce, dim3((unsigned)cdiv(m, 64)), dim3(64), 0, s, part,
                       (int)(mpad / 128), m, mpad, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top-K.

// Chunks of 512 (one compare-exchange per thread and stage, 45 stages):
// twice the largest K, so every round at least halves the candidates, and
// small enough that the first round spreads over many workgroups.
constexpr int kChunk = 512;
static_assert(kChunk >= 2 * CDL_MAX_TOPK, "every round must shrink the candidates");

__device__ inline bool before(double va, int ia, double vb, int ib) {
    return va > vb || (va == vb && ia < ib);
}

// Sort chunk blockIdx.x of (val, idx) pairs; idx_in == nullptr means idx is
// the position.  Writes the first K of each chunk.
__global__ __launch_bounds__(256) void k_topk_chunk(const double *val_in, const int32_t *idx_in,
                                                    int64_t count, int K, double *val_out,
                                                    int32_t *idx_out) {
    __shared__ double sv[kChunk];
    __shared__ int32_t si[kChunk];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int t = threadIdx.x; t < kChunk; t += 256) {
        const int64_t p = base + t;
        if (p < count) {
            sv[t] = val_in[p];
            si[t] = idx_in ? idx_in[p] : (int32_t)p;
        } else {
            sv[t] = -INFINITY;
            si[t] = 0x7fffffff;
        }
    }
    __syncthreads();
    for (int size = 2; size <= kChunk; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kChunk / 2; t += 256) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;   // first half of each run: best first
                const bool swap = desc ? before(sv[hi], si[hi], sv[lo], si[lo])
                                       : before(sv[lo], si[lo], sv[hi], si[hi]);
                if (swap) {
                    double tv = sv[lo]; sv[lo] = sv[hi]; sv[hi] = tv;
                    int32_t ti = si[lo]; si[lo] = si[hi]; si[hi] = ti;
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < K; t += 256) {
        val_out[(int64_t)blockIdx.x * K + t] = sv[t];
        idx_out[(int64_t)blockIdx.x * K + t] = si[t];
    }
}

int64_t topk_scratch_elems(int64_t m, int K) { return cdiv(m, kChunk) * (int64_t)K; }

__global__ void k_edge_split(const int64_t *idx, int64_t m, int K, int32_t *a, int32_t *b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K) return;
    const int64_t v = idx[t];
    a[t] = (int32_t)(v / m);
    b[t] = (int32_t)(v % m);
}

hipError_t launch_edge_split(const int64_t *idx, int64_t m, int K, int32_t *a, int32_t *b,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_edge_split, dim3((unsigned)cdiv(K, 256)), dim3(256), 0, s, idx, m, K, a, b);
    return hipGetLastError();
}

// As k_topk_chunk for (value, int64 index) pairs; entries at positions >=
// *dcount (when given) are empty.  Order: value descending, index ascending.
__device__ inline bool before64(double va, int64_t ia, double vb, int64_t ib) {
    return va > vb || (va == vb && ia < ib);
}

__global__ __launch_bounds__(256) void k_topk64_chunk(const double *val_in, const int64_t *idx_in,
                                                      int64_t count, const unsigned int *dcount,
                                                      int K, double *val_out, int64_t *idx_out) {
    __shared__ double sv[kChunk];
    __shared__ int64_t si[kChunk];
    const int64_t lim = dcount ? ((int64_t)*dcount < count ? (int64_t)*dcount : count) : count;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int t = threadIdx.x; t < kChunk; t += 256) {
        const int64_t p = base + t;
        if (p < lim) {
            sv[t] = val_in[p];
            si[t] = idx_in[p];
        } else {
            sv[t] = -INFINITY;
            si[t] = INT64_MAX;
        }
    }
    __syncthreads();
    for (int size = 2; size <= kChunk; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kChunk / 2; t += 256) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const bool swap = desc ? before64(sv[hi], si[hi], sv[lo], si[lo])
                                       : before64(sv[lo], si[lo], sv[hi], si[hi]);
                if (swap) {
                    double tv = sv[lo]; sv[lo] = sv[hi]; sv[hi] = tv;
                    int64_t ti = si[lo]; si[lo] = si[hi]; si[hi] = ti;
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < K; t += 256) {
        val_out[(int64_t)blockIdx.x * K + t] = sv[t];
        idx_out[(int64_t)blockIdx.x * K + t] = si[t];
    }
}

// Best K of `cap` candidates (count on the device); scratch holds
// 2 * topk_scratch_elems(cap, K) doubles and as many int64.  Writes the K
// values and indices to val_out / idx_out.
hipError_t launch_topk64(const double *val, const int64_t *idx, int64_t cap,
                         const unsigned int *dcount, int K, void *scratch, double *val_out,
                         int64_t *idx_out, hipStream_t s) {
    const int64_t sc = topk_scratch_elems(cap, K);
    double *v[2] = {(double *)scratch, (double *)scratch + sc};
    int64_t *ix[2] = {(int64_t *)((double *)scratch + 2 * sc), (int64_t *)((double *)scratch + 2 * sc) + sc};
    const double *vin = val;
    const int64_t *iin = idx;
    const unsigned int *dc = dcount;
    int64_t count = cap;
    int side = 0;
    while (true) {
        const int64_t blocks = cdiv(count, kChunk);
        hipLaunchKernelGGL(k_topk64_chunk, dim3((unsigned)blocks), dim3(256), 0, s, vin, iin, count,
                           dc, K, v[side], ix[side]);
        if (blocks == 1) break;
        vin = v[side];
        iin = ix[side];
        dc = nullptr;
        count = blocks * K;
        side ^= 1;
    }
    hipError_t e = hipMemcpyAsync(val_out, v[side], sizeof(double) * K, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(idx_out, ix[side], sizeof(int64_t) * K, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_topk(const double *F, int64_t m, int K, void *scratch, int32_t *out,
                       hipStream_t s) {
    if (K <= 0) return hipSuccess;
    const int64_t cap = topk_scratch_elems(m, K);
    double *v[2] = {(double *)scratch, (double *)scratch + cap};
    int32_t *ix[2] = {(int32_t *)((double *)scratch + 2 * cap), (int32_t *)((double *)scratch + 2 * cap) + cap};
    const double *vin = F;
    const int32_t *iin = nullptr;
    int64_t count = m;
    int side = 0;
    while (true) {
        const int64_t blocks = cdiv(count, kChunk);
        hipLaunchKernelGGL(k_topk_chunk, dim3((unsigned)blocks), dim3(256), 0, s, vin, iin, count,
                           K, v[side], ix[side]);
        if (blocks == 1) break;
        vin = v[side];
        iin = ix[side];
        count = blocks * K;
        side ^= 1;
    }
    hipError_t e = hipMemcpyAsync(out, ix[side], sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

} // namespace cdl
