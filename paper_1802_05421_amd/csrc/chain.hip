// Inverse chain (eq. inverse-chain; Algorithm 2, ChainProduct) on MFMA.
//
//   chain_prep  dmn = D^{-1/2}, dm = (cD)^{-1/2} (c = 2 for the lazy walk),
//               u = D^{1/2} 1 / sqrt(vol)
//   normalize   S~_0 = D^{-1/2} W D^{-1/2} - u u^T  (lazy: (I + S)/2 - u u^T),
//               computed in FP64 from the upper 64 x 64 tiles of W, rounded
//               to the storage type and written with the mirror; removing the
//               eigenvalue-1 mode u makes every power decay (the chain only
//               ever multiplies vectors orthogonal to u, where S~ = S)
//   square      S~_{l+1} = S~_l S~_l^T (= S~_l^2, S~ symmetric): upper
//               triangular output tiles with mirrored stores, FP32
//               accumulation (FP64 for FP64 levels), per-tile Frobenius sums
//   apply       V <- V + S~_l V for the k columns at once (one level of
//               P1 = D^{-1/2} prod_l (I + S~^{2^l}) D^{-1/2}); V kept in FP64,
//               the MFMA operand is V rounded to the storage type; on the
//               last level X += dm * V.
//
// FP16 levels hold scale * S~ (scale = a power of two near n) so entries of
// order 1/n stay in FP16's normal range; the squaring and the application
// divide the scale back out.
#include <type_traits>

#include "batch.h"
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace cdl {

__device__ inline double block_sum256c(double v, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

float level_scale(int prec, int64_t n) {
    if (prec != 3) return 1.0f;
    float s = 1.0f;
    while (s * 2.0f <= (float)n) s *= 2.0f;
    return s;
}

__device__ __forceinline__ void chain_prep_elem(const double *deg, const double *stats, int64_t n,
                                                int64_t ld, int lazy, double *dmn, double *dm,
                                                double *u, int64_t i) {
    if (i >= ld) return;
    if (i < n) {
        const double d = deg[i], vol = stats[0];
        dmn[i] = 1.0 / sqrt(d);
        dm[i] = 1.0 / sqrt(lazy ? 2.0 * d : d);
        u[i] = sqrt(d / vol);
    } else {
        dmn[i] = dm[i] = u[i] = 0.0;
    }
}

__global__ void k_chain_prep(const double *deg, const double *stats, int64_t n, int64_t ld,
                             int lazy, double *dmn, double *dm, double *u) {
    chain_prep_elem(deg, stats, n, ld, lazy, dmn, dm, u,
                    (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_chain_prep(const double *deg, const double *stats, int64_t n, int64_t ld,
                             int lazy, double *dmn, double *dm, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_chain_prep, dim3((unsigned)cdiv(ld, 256)), dim3(256), 0, s, deg,
                       stats, n, ld, lazy, dmn, dm, u);
    return hipGetLastError();
}

// One upper 64 x 64 tile per workgroup.  A lane takes two adjacent columns
// of every other row: 16-byte loads of W and two-element stores of the
// level, so a wave access covers two contiguous row segments.  The mirror is
// written from the LDS copy of the rounded tile, two adjacent rows per lane.
// Every element is the expression of k_normalize_rows.
// Upper tile `id` (after the XCD remap) of the sym_tile<8> order.
template <typename T>
__device__ __forceinline__ void normalize_tile(const double *W, int64_t ld, int64_t n,
                                               const double *dmn, const double *u, int lazy,
                                               double scale, int nt, T *S0, double *fro_part,
                                               double *fro64_part, int id) {
    struct alignas(2 * sizeof(T)) T2 { T a, b; };
    struct alignas(16) D2 { double x, y; };
    // row pitch: a whole number of T2 pairs; 2-byte types get an odd word
    // count, so the mirror's column reads spread over the banks
    constexpr int PAD = sizeof(T) == 2 ? 2 : 16 / (int)sizeof(T);
    __shared__ T t[64][64 + PAD];
    __shared__ double red[4];
    int I, J;
    sym_tile<8>(id, nt, I, J);
    const int64_t i0 = (int64_t)I * 64, j0 = (int64_t)J * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cp = lane & 31, h = lane >> 5;
    const int64_t ja = j0 + 2 * cp;   // this lane's columns ja, ja + 1
    double dj[2], uj[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        dj[e] = ja + e < n ? dmn[ja + e] : 0.0;
        uj[e] = ja + e < n ? u[ja + e] : 0.0;
    }
    const double inv_scale = 1.0 / scale;   // scale is a power of two: exact
    double s = 0.0, s64 = 0.0;
    // all row loads (W pairs and the rows' factors) in flight before the
    // first use: the rows of a wave differ between its halves, so the
    // factors are vector loads
    D2 wl[8];
    double di[8], ui[8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        const int64_t i = i0 + wv * 16 + 2 * rr + h;
        wl[rr] = *(const D2 *)(W + i * ld + ja);
        di[rr] = i < n ? dmn[i] : 0.0;
        ui[rr] = i < n ? u[i] : 0.0;
    }
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        const int r = wv * 16 + 2 * rr + h;
        const int64_t i = i0 + r;
        T tv[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t j = ja + e;
            double v = 0.0;
            if (i < n && j < n) {
                v = (e ? wl[rr].y : wl[rr].x) * (di[rr] * dj[e]);
                if (lazy) v = 0.5 * ((i == j ? 1.0 : 0.0) + v);
                v -= ui[rr] * uj[e];
            }
            tv[e] = cvtd<T>(v * scale);
            const double back = tod<T>(tv[e]) * inv_scale;
            s += back * back;
            s64 += v * v;
        }
        const T2 pk{tv[0], tv[1]};
        *(T2 *)&t[r][2 * cp] = pk;
        *(T2 *)(S0 + i * ld + ja) = pk;
    }
    if (I != J) {
        __syncthreads();
#pragma unroll 4
        for (int cc = 0; cc < 8; ++cc) {
            const int c = wv * 16 + 2 * cc + h;
            const T2 pk{t[2 * cp][c], t[2 * cp + 1][c]};
            *(T2 *)(S0 + (j0 + c) * ld + i0 + 2 * cp) = pk;
        }
    }
    const double w = I != J ? 2.0 : 1.0;
    s = block_sum256c(s, red);
    if (threadIdx.x == 0) fro_part[id] = w * s;
    s64 = block_sum256c(s64, red);
    if (threadIdx.x == 0) fro64_part[id] = w * s64;
}

template <typename T>
__global__ __launch_bounds__(256) void k_normalize(const double *W, int64_t ld, int64_t n,
                                                   const double *dmn, const double *u, int lazy,
                                                   double scale, int nt, T *S0,
                                                   double *fro_part, double *fro64_part) {
    normalize_tile<T>(W, ld, n, dmn, u, lazy, scale, nt, S0, fro_part, fro64_part,
                      xcd_remap(blockIdx.x, nt * (nt + 1) / 2));
}

hipError_t launch_normalize(int prec, const double *W, int64_t ld, int64_t n,
                            const double *dmn, const double *u, int lazy, void *S0,
                            double *fro_part, double *fro64_part, hipStream_t s) {
    const double sc = level_scale(prec, n);
    const int nt = (int)(ld / 64);
    dim3 g((unsigned)sym_tiles64(ld)), b(256);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_normalize<double>, g, b, 0, s, W, ld, n, dmn, u, lazy, sc, nt, (double *)S0, fro_part, fro64_part); break;
    case 1: hipLaunchKernelGGL(k_normalize<float>, g, b, 0, s, W, ld, n, dmn, u, lazy, sc, nt, (float *)S0, fro_part, fro64_part); break;
    case 2: hipLaunchKernelGGL(k_normalize<__bf16>, g, b, 0, s, W, ld, n, dmn, u, lazy, sc, nt, (__bf16 *)S0, fro_part, fro64_part); break;
    case 3: hipLaunchKernelGGL(k_normalize<_Float16>, g, b, 0, s, W, ld, n, dmn, u, lazy, sc, nt, (_Float16 *)S0, fro_part, fro64_part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The same level from a row panel of W (panel row q = node row0 + q, full
// rows): one workgroup per row, the expression of k_normalize, so the same
// weights and degrees give the same bits in both triangles.  fro_part[q] and
// fro64_part[q] get the row's sums of squares (rounded and exact).
template <typename T>
__global__ __launch_bounds__(256) void k_normalize_rows(const double *Wp, int64_t ld, int64_t n,
                                                        int64_t row0, const double *dmn,
                                                        const double *u, int lazy, double scale,
                                                        T *S0, double *fro_part,
                                                        double *fro64_part) {
    __shared__ double red[4];
    const int64_t q = blockIdx.x, i = row0 + q;
    const double *row = Wp + q * ld;
    T *out = S0 + i * ld;
    const bool live = i < n;
    const double di = live ? dmn[i] : 0.0, ui = live ? u[i] : 0.0;
    const double inv_scale = 1.0 / scale;   // scale is a power of two: exact
    double s = 0.0, s64 = 0.0;
    for (int64_t j0 = threadIdx.x; j0 < ld; j0 += 4 * 256) {
        double wl[4];   // four loads in flight
#pragma unroll
        for (int c = 0; c < 4; ++c) wl[c] = j0 + 256 * c < ld ? row[j0 + 256 * c] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = j0 + 256 * c;
            if (j >= ld) break;
            double v = 0.0;
            if (live && j < n) {
                v = wl[c] * (di * dmn[j]);
                if (lazy) v = 0.5 * ((i == j ? 1.0 : 0.0) + v);
                v -= ui * u[j];
            }
            const T tv = cvtd<T>(v * scale);
            out[j] = tv;
            const double back = tod<T>(tv) * inv_scale;
            s += back * back;
            s64 += v * v;
        }
    }
    s = block_sum256c(s, red);
    if (threadIdx.x == 0) fro_part[q] = s;
    s64 = block_sum256c(s64, red);
    if (threadIdx.x == 0) fro64_part[q] = s64;
}

hipError_t launch_normalize_rows(int prec, const double *Wp, int64_t ld, int64_t n, int64_t row0,
                                 int64_t rows, const double *dmn, const double *u, int lazy,
                                 void *S0, double *fro_part, double *fro64_part, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const double sc = level_scale(prec, n);
    dim3 g((unsigned)rows), b(256);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_normalize_rows<double>, g, b, 0, s, Wp, ld, n, row0, dmn, u, lazy, sc, (double *)S0, fro_part, fro64_part); break;
    case 1: hipLaunchKernelGGL(k_normalize_rows<float>, g, b, 0, s, Wp, ld, n, row0, dmn, u, lazy, sc, (float *)S0, fro_part, fro64_part); break;
    case 2: hipLaunchKernelGGL(k_normalize_rows<__bf16>, g, b, 0, s, Wp, ld, n, row0, dmn, u, lazy, sc, (__bf16 *)S0, fro_part, fro64_part); break;
    case 3: hipLaunchKernelGGL(k_normalize_rows<_Float16>, g, b, 0, s, Wp, ld, n, row0, dmn, u, lazy, sc, (_Float16 *)S0, fro_part, fro64_part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric squaring.

// 16-bit levels: 256 x 256 tiles on NW = 8 waves (2 x 4 of 128 x 64) or
// NW = 4 waves (2 x 2 of 128 x 128); FP32/FP64 levels: one configuration.
// SH: the MFMA shape of the 16-bit cores (32: 32 x 32 x 16, 16: 16 x 16 x 32).
template <typename T, int NW, int SH = 32> struct SqCfg;
template <int NW, int SH> struct SqCfg<__bf16, NW, SH> {
    using Core = DmaCore<std::conditional_t<SH == 16, MfmaBF16x32, MfmaBF16>, 256, 256, 2, NW / 2>;
    static constexpr int TILE = 256;
};
template <int NW, int SH> struct SqCfg<_Float16, NW, SH> {
    using Core = DmaCore<std::conditional_t<SH == 16, MfmaF16x32, MfmaF16>, 256, 256, 2, NW / 2>;
    static constexpr int TILE = 256;
};
template <int NW, int SH> struct SqCfg<float, NW, SH> { using Core = GemmCore<MfmaF32, 128, 128, 32, 2, 2>; static constexpr int TILE = 128; };
template <int NW, int SH> struct SqCfg<double, NW, SH> { using Core = GemmCore<MfmaF64, 128, 128, 16, 2, 2>; static constexpr int TILE = 128; };

template <typename T, int NW, int SH = 32> constexpr size_t sq_smem() {
    using C = typename SqCfg<T, NW, SH>::Core;
    constexpr int TL = SqCfg<T, NW, SH>::TILE;
    constexpr size_t stage = (size_t)TL * (TL + 16 / sizeof(T)) * sizeof(T);
    return C::SMEM > stage ? C::SMEM : stage;
}

// Epilogue of one output tile of C = A B (tile rows m0.., columns n0..):
// scale back by inv_scale, with add != 0 also add A + B (the next factor of
// the dense chain product, below), round to T, store the tile and (off the
// diagonal) its mirror, and write the squared Frobenius norm of the stored
// values (doubled off the diagonal) to *fro_out.  A and B are polynomials in
// the same symmetric matrix, so they commute and C is symmetric.
template <typename T, class Core>
__device__ inline void square_epilogue(Core &g, const T *A, const T *B, T *S2, int64_t ld,
                                       int64_t m0, int64_t n0, bool mirror, float inv_scale,
                                       int add, double *fro_out, T *smem, double *red) {
    using Acc = typename Core::MF::Acc;
    double fro = 0.0;
    auto f = [&](int r, int c, Acc acc) -> T {
        Acc v = acc * (Acc)inv_scale;
        if (add) {
            const int64_t o = (m0 + r) * ld + n0 + c;
            v += (Acc)tod<T>(A[o]) + (Acc)tod<T>(B[o]);
        }
        T t = (T)v;
        double tv = tod<T>(t) * (double)inv_scale;
        fro += tv * tv;
        return t;
    };
    stage_and_store(g, smem, f, S2, ld, m0, n0, mirror);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) fro += __shfl_xor(fro, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = fro;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < Core::NT / 64; ++q) t += red[q];
        *fro_out = (mirror ? 2.0 : 1.0) * t;
    }
}

// C = A B over the upper tiles with logical ids [0, count) (count = all
// tiles, or the full rounds of 256 workgroups when the last round is split
// over k below).  The squaring is A = B = S, add = 0.
// Upper tile `id` of C = A B and its epilogue (one workgroup).
template <typename T, int NW, int SH = 32>
__device__ __forceinline__ void square_tile(const T *A, const T *B, T *S2, int64_t ld, int64_t kend, int nt,
                                   int id, float inv_scale, int add, double *fro_part,
                                   char *smem_raw, double *red) {
    using Core = typename SqCfg<T, NW, SH>::Core;
    constexpr int TL = SqCfg<T, NW, SH>::TILE;
    int I, J;
    sym_tile<8>(id, nt, I, J);
    const int64_t m0 = (int64_t)I * TL, n0 = (int64_t)J * TL;
    Core g;
    g.run(A, ld, B, ld, m0, n0, kend, (T *)smem_raw);
    square_epilogue<T>(g, A, B, S2, ld, m0, n0, I != J, inv_scale, add, fro_part + id,
                       (T *)smem_raw, red);
}

template <typename T, int NW, int SH>
__global__ __launch_bounds__((SqCfg<T, NW, SH>::Core::NT)) void k_square(const T *A, const T *B, T *S2, int64_t ld,
                                                int64_t kend, int nt, int count, float inv_scale,
                                                int add, double *fro_part) {
    using Core = typename SqCfg<T, NW, SH>::Core;
    constexpr int TL = SqCfg<T, NW, SH>::TILE;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    __shared__ double red[Core::NT / 64];
    const int id = TL == 256 ? round_remap(blockIdx.x, count) : xcd_remap(blockIdx.x, count);
    square_tile<T, NW, SH>(A, B, S2, ld, kend, nt, id, inv_scale, add, fro_part, smem_raw, red);
}

// Level `level` squared into level + 1 for every snapshot of a sequence:
// workgroup b is upper tile b - prefix[p] of snapshot p.
template <typename T>
__global__ __launch_bounds__((SqCfg<T, 8>::Core::NT)) void k_square_grouped(const BatchSnap *snaps,
                                                                           const int *prefix, int P,
                                                                           int level) {
    using Core = typename SqCfg<T, 8>::Core;
    constexpr int TL = SqCfg<T, 8>::TILE;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    __shared__ double red[Core::NT / 64];
    const int p = group_find(prefix, P, blockIdx.x);
    const BatchSnap &d = snaps[p];
    const T *A = (const T *)(d.levels + d.level_bytes * level);
    T *C = (T *)(d.levels + d.level_bytes * (level + 1));
    square_tile<T, 8>(A, A, C, d.ld, (d.n + 63) / 64 * 64, (int)(d.ld / TL), blockIdx.x - prefix[p],
                      d.inv_scale, 0, d.fro, smem_raw, red);
}

// The tiles of the last, partial round of workgroups (logical ids
// first + b / splits), each split into `splits` k-ranges of ks elements:
// workgroup b multiplies its range and stores the FP32 accumulators as a
// partial tile (element e of thread t at P[b * TL^2 + e * NT + t]).
template <typename T, int NW, int SH>
__global__ __launch_bounds__((SqCfg<T, NW, SH>::Core::NT)) void k_square_part(const T *A, const T *B, int64_t ld,
                                                     int64_t kend, int64_t ks, int nt, int first,
                                                     int splits, float *P) {
    using Core = typename SqCfg<T, NW, SH>::Core;
    constexpr int TL = SqCfg<T, NW, SH>::TILE;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int b = blockIdx.x, sp = b % splits;
    int I, J;
    sym_tile<8>(first + b / splits, nt, I, J);
    const int64_t k0 = (int64_t)sp * ks;
    const int64_t kk = kend - k0 < ks ? kend - k0 : ks;
    Core g;
    g.run(A + k0, ld, B + k0, ld, (int64_t)I * TL, (int64_t)J * TL, kk, (T *)smem_raw);
    float *Pb = P + (size_t)b * TL * TL;
    int e = 0;
#pragma unroll
    for (int i = 0; i < Core::WTM; ++i)
#pragma unroll
        for (int j = 0; j < Core::WTN; ++j)
#pragma unroll
            for (int r = 0; r < Core::MF::R; ++r, ++e) Pb[(size_t)e * Core::NT + threadIdx.x] = g.acc[i][j][r];
}

// One workgroup per tile of the split round: the partial tiles summed in
// split order into the accumulator layout of the core, then the epilogue.
// Loads go out sixteen elements by four splits at a time, so a thread has
// 64 in flight instead of one round trip per element and split.
template <typename T, int NW, int SH>
__global__ __launch_bounds__((SqCfg<T, NW, SH>::Core::NT)) void k_square_tail(const T *A, const T *B, T *S2,
                                                     int64_t ld, int nt, int first, int splits,
                                                     const float *P, float inv_scale, int add,
                                                     double *fro_part) {
    using Core = typename SqCfg<T, NW, SH>::Core;
    constexpr int TL = SqCfg<T, NW, SH>::TILE;
    constexpr int R = Core::MF::R, E = Core::WTM * Core::WTN * R;
    constexpr int G = 16, SB = 4;   // elements per group, splits per batch
    static_assert(E % G == 0, "accumulator count");
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    __shared__ double red[Core::NT / 64];
    const int id = first + blockIdx.x;
    int I, J;
    sym_tile<8>(id, nt, I, J);
    Core g;
    const float *Pt = P + (size_t)blockIdx.x * splits * TL * TL + threadIdx.x;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += G) {
        float v[G];
#pragma unroll
        for (int q = 0; q < G; ++q) v[q] = 0.f;
        for (int sp0 = 0; sp0 < splits; sp0 += SB) {
            float w[SB][G];
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (sp0 + u < splits)
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        w[u][q] = Pt[(size_t)(sp0 + u) * TL * TL + (size_t)(e0 + q) * Core::NT];
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (sp0 + u < splits)
#pragma unroll
                    for (int q = 0; q < G; ++q) v[q] += w[u][q];
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int e = e0 + q, r = e % R, ij = e / R;
            g.acc[ij / Core::WTN][ij % Core::WTN][r] = v[q];
        }
    }
    square_epilogue<T>(g, A, B, S2, ld, (int64_t)I * TL, (int64_t)J * TL, I != J, inv_scale, add,
                       fro_part + id, (T *)smem_raw, red);
}

int square_tiles(int prec, int64_t ld) {
    int TL = (prec == 2 || prec == 3) ? 256 : 128;
    int nt = (int)(ld / TL);
    return nt * (nt + 1) / 2;
}

// Work split of one 16-bit squaring: the upper tiles fill `full` rounds of
// one workgroup per CU; when a last round of at most half the CUs remains,
// its `rem` tiles are split over k into `splits` ranges of ks elements, so
// that the last round occupies the whole chip.
struct SqPlan {
    int total, full, rem, splits;
    int64_t kend, ks;
};
static SqPlan square_plan(int prec, int64_t ld, int64_t n) {
    SqPlan p;
    p.total = square_tiles(prec, ld);
    p.kend = (n + 63) / 64 * 64;   // multiple of every BK used (64/32/16)
    p.full = p.total;
    p.rem = 0;
    p.splits = 0;
    p.ks = 0;
    const bool dma = prec == 2 || prec == 3;
    const int rem = p.total % kNumCu;
    if (!dma || p.total < kNumCu || rem == 0 || rem > kNumCu / 2) return p;
    const int64_t nk = p.kend / 64;
    int s = kNumCu / rem;
    if (s > nk / 2) s = (int)(nk / 2);
    if (s < 2) return p;
    p.ks = cdiv(nk, s) * 64;
    p.splits = (int)cdiv(p.kend, p.ks);
    if (p.splits < 2) return p;
    p.full = p.total - rem;
    p.rem = rem;
    return p;
}

size_t square_tail_bytes(int prec, int64_t ld, int64_t n) {
    const SqPlan p = square_plan(prec, ld, n);
    return (size_t)p.rem * p.splits * 256 * 256 * sizeof(float);
}

template <typename T, int NW, int SH = 32>
static hipError_t sq_launch(const void *A, const void *B, void *S2, int64_t ld, int64_t n,
                            float inv_scale, int add, double *fro_part, float *tail, hipStream_t s) {
    using Cfg = SqCfg<T, NW, SH>;
    constexpr int TL = Cfg::TILE;
    constexpr size_t smem = sq_smem<T, NW, SH>();
    static bool attr = false;
    if (!attr) {
        for (const void *fn : {(const void *)k_square<T, NW, SH>, (const void *)k_square_part<T, NW, SH>,
                               (const void *)k_square_tail<T, NW, SH>}) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            if (e != hipSuccess) return e;
        }
        attr = true;
    }
    const int nt = (int)(ld / TL);
    const int prec = std::is_same<T, double>::value ? 0 : std::is_same<T, float>::value ? 1 :
                     std::is_same<T, __bf16>::value ? 2 : 3;
    SqPlan p = square_plan(prec, ld, n);
    if (!tail) p = SqPlan{p.total, p.total, 0, 0, p.kend, 0};
    constexpr int NT = Cfg::Core::NT;
    hipLaunchKernelGGL((k_square<T, NW, SH>), dim3(p.full), dim3(NT), smem, s, (const T *)A,
                       (const T *)B, (T *)S2, ld, p.kend, nt, p.full, inv_scale, add, fro_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.rem == 0) return e;
    hipLaunchKernelGGL((k_square_part<T, NW, SH>), dim3(p.rem * p.splits), dim3(NT), smem, s,
                       (const T *)A, (const T *)B, ld, p.kend, p.ks, nt, p.full, p.splits, tail);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_square_tail<T, NW, SH>), dim3(p.rem), dim3(NT), smem, s, (const T *)A,
                       (const T *)B, (T *)S2, ld, nt, p.full, p.splits, (const float *)tail,
                       inv_scale, add, fro_part);
    return hipGetLastError();
}

int square_variants(int prec) { return prec == 2 || prec == 3 ? 6 : 1; }

// (the 4-wave core with 16 x 16 x 32 MFMAs needs more than its 512
// registers and is not a candidate)
template <typename T>
static hipError_t sq_dispatch16(const void *A, const void *B, void *C, int64_t ld, int64_t n,
                                float inv, int add, double *fro_part, float *t, int variant,
                                hipStream_t s) {
    switch (variant >> 1) {
    case 0: return sq_launch<T, 8, 32>(A, B, C, ld, n, inv, add, fro_part, t, s);
    case 1: return sq_launch<T, 4, 32>(A, B, C, ld, n, inv, add, fro_part, t, s);
    default: return sq_launch<T, 8, 16>(A, B, C, ld, n, inv, add, fro_part, t, s);
    }
}

// variant (16-bit levels, 0..5): bit 0 set = no k-split of the last round;
// variant >> 1 = 0: 8-wave core, 32 x 32 x 16 MFMAs; 1: 4-wave core, 32 x 32
// x 16; 2: 8-wave core, 16 x 16 x 32.  Other types have one variant.
static hipError_t sq_dispatch(int prec, const void *A, const void *B, void *C, int64_t ld, int64_t n,
                              int add, double *fro_part, float *tail, int variant, hipStream_t s) {
    const float inv = 1.0f / level_scale(prec, n);
    float *t = (variant & 1) ? nullptr : tail;
    switch (prec) {
    case 0: return sq_launch<double, 8>(A, B, C, ld, n, inv, add, fro_part, nullptr, s);
    case 1: return sq_launch<float, 8>(A, B, C, ld, n, inv, add, fro_part, nullptr, s);
    case 2: return sq_dispatch16<__bf16>(A, B, C, ld, n, inv, add, fro_part, t, variant, s);
    case 3: return sq_dispatch16<_Float16>(A, B, C, ld, n, inv, add, fro_part, t, variant, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_square(int prec, const void *S, void *S2, int64_t ld, int64_t n,
                         double *fro_part, float *tail, int variant, hipStream_t s) {
    return sq_dispatch(prec, S, S, S2, ld, n, 0, fro_part, tail, variant, s);
}

// Inside a diagonal tile both triangles come out of the GEMM, and for A != B
// C_ij and C_ji are sums in different orders: copy the upper triangle of each
// diagonal tile onto its lower one so the stored product is exactly
// symmetric.  One workgroup per diagonal tile.
template <typename T>
__global__ __launch_bounds__(256) void k_sym_diag(T *C, int64_t ld, int TL) {
    const int64_t t0 = (int64_t)blockIdx.x * TL;
    for (int64_t q = threadIdx.x; q < (int64_t)TL * TL; q += 256) {
        const int r = (int)(q / TL), c = (int)(q % TL);
        if (r > c) C[(t0 + r) * ld + t0 + c] = C[(t0 + c) * ld + t0 + r];
    }
}

template <typename T>
static hipError_t sym_diag_launch(void *C, int64_t ld, hipStream_t s) {
    const int TL = SqCfg<T, 8>::TILE;
    hipLaunchKernelGGL(k_sym_diag<T>, dim3((unsigned)(ld / TL)), dim3(256), 0, s, (T *)C, ld, TL);
    return hipGetLastError();
}

hipError_t launch_chain_product(int prec, const void *Q, const void *L, void *C, int64_t ld,
                                int64_t n, double *fro_part, float *tail, int variant,
                                hipStream_t s) {
    hipError_t e = sq_dispatch(prec, Q, L, C, ld, n, 1, fro_part, tail, variant, s);
    if (e != hipSuccess) return e;
    switch (prec) {
    case 0: return sym_diag_launch<double>(C, ld, s);
    case 1: return sym_diag_launch<float>(C, ld, s);
    case 2: return sym_diag_launch<__bf16>(C, ld, s);
    case 3: return sym_diag_launch<_Float16>(C, ld, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Chain application: C[r][i] = sum_j Vin[r][j] S~[i][j]  (= (S~ V)_{i r}).
// BF16/FP16/FP32 levels: split-K MFMA GEMM over 256 x 256 output tiles (8
// waves) writing FP32 partials, then a reduction that updates V (FP64), its
// rounded copy and, on the last level, X.  FP64 levels: one 64-wide tile
// per workgroup, updating in the epilogue.

template <typename T> struct ApBK { static constexpr int v = 64 * 2 / (int)sizeof(T) < 16 ? 16 : 64 * 2 / (int)sizeof(T); };

// 16-bit levels stream through the direct-to-LDS core, FP32 levels through
// the register-staged one.
template <typename T, int BM> struct ApCfg {
    static constexpr int WM = BM / 128 > 0 ? BM / 128 : 1;
    static constexpr int WN = 8 / WM;
    using Mf = typename MfmaOf<T>::type;
    using Core = std::conditional_t<sizeof(T) == 2, DmaCore<Mf, BM, 256, WM, WN>,
                                    GemmCore<Mf, BM, 256, ApBK<T>::v, WM, WN>>;
};

// Split-K product tile `id` of the chain application (one workgroup).
template <typename T, int BM>
__device__ __forceinline__ void apply_gemm_tile(const T *Vin, const T *S, int64_t ld, int64_t kend,
                                       int64_t ks, int mt, int nt, float *P, int64_t kpad, int id,
                                       char *smem_raw) {
    using Core = typename ApCfg<T, BM>::Core;
    T *smem = (T *)smem_raw;
    const int split = id / (mt * nt);
    int I, J;
    rect_tile<4>(id % (mt * nt), mt, nt, I, J);
    const int64_t m0 = (int64_t)I * BM, n0 = (int64_t)J * 256;
    const int64_t k0 = (int64_t)split * ks;
    const int64_t kk = k0 < kend ? (kend - k0 < ks ? kend - k0 : ks) : 0;
    Core g;
    g.run(Vin + k0, ld, S + k0, ld, m0, n0, kk, smem);
    float *Ps = P + (int64_t)split * kpad * ld;
#pragma unroll
    for (int a = 0; a < Core::WTM; ++a)
#pragma unroll
        for (int b = 0; b < Core::WTN; ++b)
#pragma unroll
            for (int r = 0; r < Core::MF::R; ++r)
                Ps[(m0 + Core::row_of(a, r)) * ld + n0 + Core::col_of(b)] = g.acc[a][b][r];
}

template <typename T, int BM>
__global__ __launch_bounds__(512) void k_apply_gemm(const T *Vin, const T *S, int64_t ld,
                                                    int64_t kend, int64_t ks, int mt, int nt,
                                                    int nsplit, float *P, int64_t kpad) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int id = xcd_remap(blockIdx.x, mt * nt * nsplit);
    apply_gemm_tile<T, BM>(Vin, S, ld, kend, ks, mt, nt, P, kpad, id, smem_raw);
}

static int ap_bm(int64_t kpad) { return kpad % 256 == 0 ? 256 : (kpad % 128 == 0 ? 128 : 64); }

// k-range of one split of an application's product (64-element multiples).
__host__ __device__ inline int64_t apply_split_len(int64_t n, int nsplit) {
    const int64_t kend = (n + 63) / 64 * 64;
    return (cdiv(kend, nsplit) + 63) / 64 * 64;
}

// Split-K count of the chain application: choice 0 aims at >= 256
// workgroups, 1 halves that count, 2 doubles it (at least two 64-wide
// k-tiles per split either way); FP64 levels are not split.
int apply_splits(int prec, int64_t ld, int64_t kpad, int64_t n, int choice) {
    if (prec == 0) return 1;
    const int64_t base = (kpad / ap_bm(kpad)) * (ld / 256);
    const int64_t kend = (n + 63) / 64 * 64;
    int64_t S = (256 + base - 1) / base;
    if (choice == 1) S = S / 2;
    if (choice == 2) S = 2 * S;
    const int64_t smax = kend / 128 > 0 ? kend / 128 : 1;   // >= 2 k-tiles per split
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    return (int)S;
}

// Elements first, first + step, ... (< total) of the application's update.
template <typename T>
__device__ inline void apply_reduce_range(const float *P, int nsplit, int64_t total, int64_t ld,
                                          int64_t kpad, float inv_scale, int accumulate,
                                          double *V64, T *Vout, double *Xt, const double *dm,
                                          const double *inv_vs, int64_t first, int64_t step) {
    const double ivs = inv_vs ? *inv_vs : 0.0;
    for (int64_t o = first; o < total; o += step) {
        float acc = 0.f;
        for (int q = 0; q < nsplit; ++q) acc += P[(int64_t)q * kpad * ld + o];
        const double v = (accumulate ? V64[o] : 0.0) + (double)acc * (double)inv_scale;
        V64[o] = v;
        Vout[o] = cvtd<T>(v);
        if (inv_vs) Xt[o] += dm[o % ld] * v * ivs;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_reduce(const float *P, int nsplit, int64_t total,
                                                      int64_t ld, int64_t kpad, float inv_scale,
                                                      int accumulate, double *V64, T *Vout,
                                                      double *Xt, const double *dm,
                                                      const double *inv_vs) {
    apply_reduce_range<T>(P, nsplit, total, ld, kpad, inv_scale, accumulate, V64, Vout, Xt, dm,
                          inv_vs, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                          (int64_t)gridDim.x * blockDim.x);
}

template <typename T, int BM>
static hipError_t apg_launch(const void *Vin, const void *S, int64_t ld, int64_t n,
                             int64_t kpad, int nsplit, float *P, hipStream_t s) {
    using Core = typename ApCfg<T, BM>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_apply_gemm<T, BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(ld / 256);
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t ks = (cdiv(kend, nsplit) + 63) / 64 * 64;
    hipLaunchKernelGGL((k_apply_gemm<T, BM>), dim3(mt * nt * nsplit), dim3(512), Core::SMEM, s,
                       (const T *)Vin, (const T *)S, ld, kend, ks, mt, nt, nsplit, P, kpad);
    return hipGetLastError();
}

template <typename T>
static hipError_t ap_gemm_launch(const void *Vin, const void *S, int64_t ld, int64_t n,
                                 int64_t kpad, int ns, float *P, hipStream_t s) {
    switch (ap_bm(kpad)) {
    case 256: return apg_launch<T, 256>(Vin, S, ld, n, kpad, ns, P, s);
    case 128: return apg_launch<T, 128>(Vin, S, ld, n, kpad, ns, P, s);
    default: return apg_launch<T, 64>(Vin, S, ld, n, kpad, ns, P, s);
    }
}

template <typename T>
static hipError_t ap_split_launch(const void *Vin, const void *S, void *Vout, double *V64,
                                  int64_t ld, int64_t n, int64_t kpad, float inv_scale,
                                  double *Xt, const double *dm, const double *inv_vs, float *P,
                                  int accumulate, int ns, hipStream_t s) {
    hipError_t e = ap_gemm_launch<T>(Vin, S, ld, n, kpad, ns, P, s);
    if (e != hipSuccess) return e;
    const int64_t total = kpad * ld;
    const int grid = (int)(cdiv(total, 256) < 16384 ? cdiv(total, 256) : 16384);
    hipLaunchKernelGGL(k_apply_reduce<T>, dim3(grid), dim3(256), 0, s, P, ns, total, ld, kpad,
                       inv_scale, accumulate, V64, (T *)Vout, Xt, dm, inv_vs);
    return hipGetLastError();
}

// ---- grouped over the snapshots of a sequence ----------------------------

template <typename T, int BM>
__global__ __launch_bounds__(512) void k_apply_gemm_grouped(const BatchSnap *snaps, const int *prefix,
                                                            int P, int64_t kpad, int level, int in,
                                                            const int *done) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int p = group_find(prefix, P, blockIdx.x);
    if (done[p]) return;
    const BatchSnap &d = snaps[p];
    const int mt = (int)(kpad / BM), nt = (int)(d.ld / 256);
    const int count = prefix[p + 1] - prefix[p];
    const int id = xcd_remap(blockIdx.x - prefix[p], count);
    apply_gemm_tile<T, BM>((const T *)d.Vlo[in], (const T *)(d.levels + d.level_bytes * level), d.ld,
                           (d.n + 63) / 64 * 64, apply_split_len(d.n, d.ap_splits), mt, nt, d.Pap,
                           kpad, id, smem_raw);
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_reduce_grouped(const BatchSnap *snaps, const int *prefix,
                                                              int P, int64_t kpad, int in,
                                                              int accumulate, int last,
                                                              const int *done) {
    const int p = group_find(prefix, P, blockIdx.x);
    if (done[p]) return;
    const BatchSnap &d = snaps[p];
    const int64_t nb = prefix[p + 1] - prefix[p];
    apply_reduce_range<T>(d.Pap, d.ap_splits, kpad * d.ld, d.ld, kpad, d.inv_scale, accumulate,
                          d.V64, (T *)d.Vlo[in ^ 1], d.Xt, d.dm, last ? d.scal + kpad + 1 : nullptr,
                          (int64_t)(blockIdx.x - prefix[p]) * 256 + threadIdx.x, nb * 256);
}

int apply_gemm_tiles(int64_t ld, int64_t kpad, int nsplit) {
    return (int)(kpad / ap_bm(kpad) * (ld / 256)) * nsplit;
}

int apply_reduce_blocks(int64_t ld, int64_t kpad, int cap) {
    const int64_t b = cdiv(kpad * ld, 256);
    return (int)(b < cap ? b : cap);
}

int apply_splits_fixed(int prec, int64_t n, int S) {
    if (prec == 0) return 1;
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t smax = kend / 128 > 0 ? kend / 128 : 1;   // >= 2 k-tiles per split
    return (int)(S < 1 ? 1 : S > smax ? smax : S);
}

template <typename T, int BM>
static hipError_t apply_grouped_launch(const BatchSnap *snaps, const int *prefix_gemm, int total_gemm,
                                       const int *prefix_red, int total_red, int P, int64_t kpad,
                                       int level, int in, int accumulate, int last, const int *done,
                                       hipStream_t s) {
    using Core = typename ApCfg<T, BM>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_apply_gemm_grouped<T, BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_apply_gemm_grouped<T, BM>), dim3(total_gemm), dim3(512), Core::SMEM, s, snaps,
                       prefix_gemm, P, kpad, level, in, done);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply_reduce_grouped<T>, dim3(total_red), dim3(256), 0, s, snaps, prefix_red,
                       P, kpad, in, accumulate, last, done);
    return hipGetLastError();
}

template <typename T>
static hipError_t apply_grouped_bm(const BatchSnap *snaps, const int *pg, int tg, const int *pr,
                                   int tr, int P, int64_t kpad, int level, int in, int accumulate,
                                   int last, const int *done, hipStream_t s) {
    switch (ap_bm(kpad)) {
    case 256: return apply_grouped_launch<T, 256>(snaps, pg, tg, pr, tr, P, kpad, level, in, accumulate, last, done, s);
    case 128: return apply_grouped_launch<T, 128>(snaps, pg, tg, pr, tr, P, kpad, level, in, accumulate, last, done, s);
    default: return apply_grouped_launch<T, 64>(snaps, pg, tg, pr, tr, P, kpad, level, in, accumulate, last, done, s);
    }
}

hipError_t launch_apply_grouped(int prec, const BatchSnap *snaps, const int *prefix_gemm,
                                int total_gemm, const int *prefix_red, int total_red, int P,
                                int64_t kpad, int level, int in, int accumulate, int last,
                                const int *done, hipStream_t s) {
    switch (prec) {
    case 1: return apply_grouped_bm<float>(snaps, prefix_gemm, total_gemm, prefix_red, total_red, P, kpad, level, in, accumulate, last, done, s);
    case 2: return apply_grouped_bm<__bf16>(snaps, prefix_gemm, total_gemm, prefix_red, total_red, P, kpad, level, in, accumulate, last, done, s);
    case 3: return apply_grouped_bm<_Float16>(snaps, prefix_gemm, total_gemm, prefix_red, total_red, P, kpad, level, in, accumulate, last, done, s);
    default: return hipErrorInvalidValue;   // FP64 chains are not grouped
    }
}

template <typename T>
static hipError_t square_grouped_launch(const BatchSnap *snaps, const int *prefix, int P, int total,
                                        int level, hipStream_t s) {
    constexpr size_t smem = sq_smem<T, 8>();
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_square_grouped<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_square_grouped<T>, dim3(total), dim3(SqCfg<T, 8>::Core::NT), smem, s, snaps,
                       prefix, P, level);
    return hipGetLastError();
}

hipError_t launch_square_grouped(int prec, const BatchSnap *snaps, const int *prefix, int P,
                                 int total, int level, hipStream_t s) {
    switch (prec) {
    case 1: return square_grouped_launch<float>(snaps, prefix, P, total, level, s);
    case 2: return square_grouped_launch<__bf16>(snaps, prefix, P, total, level, s);
    case 3: return square_grouped_launch<_Float16>(snaps, prefix, P, total, level, s);
    default: return hipErrorInvalidValue;
    }
}

// FP64 levels: in-epilogue update (small n only in practice).
template <int BM>
__global__ __launch_bounds__(BM) void k_apply_f64(const double *Vin, const double *S, double *Vout,
                                                  double *V64, int64_t ld, int64_t kend, int mt,
                                                  int nt, double *Xt, const double *dm,
                                                  const double *inv_vs, int accumulate) {
    using Core = GemmCore<MfmaF64, BM, 64, 16, BM / 64, 1>;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    double *smem = (double *)smem_raw;
    int I, J;
    rect_tile<4>(xcd_remap(blockIdx.x, mt * nt), mt, nt, I, J);
    const int64_t m0 = (int64_t)I * BM, n0 = (int64_t)J * 64;
    Core g;
    g.run(Vin, ld, S, ld, m0, n0, kend, smem);
    const double ivs = inv_vs ? *inv_vs : 0.0;
#pragma unroll
    for (int a = 0; a < Core::WTM; ++a)
#pragma unroll
        for (int b = 0; b < Core::WTN; ++b)
#pragma unroll
            for (int r = 0; r < MfmaF64::R; ++r) {
                const int64_t row = m0 + Core::row_of(a, r), col = n0 + Core::col_of(b);
                const int64_t o = row * ld + col;
                const double v = (accumulate ? V64[o] : 0.0) + g.acc[a][b][r];
                V64[o] = v;
                Vout[o] = v;
                if (inv_vs) Xt[o] += dm[col] * v * ivs;
            }
}

template <int BM>
static hipError_t apf64_launch(const void *Vin, const void *S, void *Vout, double *V64,
                               int64_t ld, int64_t n, int64_t kpad, double *Xt, const double *dm,
                               const double *inv_vs, int accumulate, hipStream_t s) {
    using Core = GemmCore<MfmaF64, BM, 64, 16, BM / 64, 1>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_apply_f64<BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(ld / 64);
    const int64_t kend = (n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_apply_f64<BM>, dim3(mt * nt), dim3(BM), Core::SMEM, s,
                       (const double *)Vin, (const double *)S, (double *)Vout, V64, ld, kend, mt,
                       nt, Xt, dm, inv_vs, accumulate);
    return hipGetLastError();
}

hipError_t launch_apply(int prec, const void *Vin, const void *S, void *Vout, double *V64,
                        int64_t ld, int64_t n, int64_t kpad, double *Xt, const double *dm,
                        const double *inv_vs, float *P, int accumulate, int nsplit, hipStream_t s) {
    const float inv = 1.0f / level_scale(prec, n);
    const int ns = nsplit;
    switch (prec) {
    case 0:
        if (kpad % 256 == 0) return apf64_launch<256>(Vin, S, Vout, V64, ld, n, kpad, Xt, dm, inv_vs, accumulate, s);
        if (kpad % 128 == 0) return apf64_launch<128>(Vin, S, Vout, V64, ld, n, kpad, Xt, dm, inv_vs, accumulate, s);
        return apf64_launch<64>(Vin, S, Vout, V64, ld, n, kpad, Xt, dm, inv_vs, accumulate, s);
    case 1: return ap_split_launch<float>(Vin, S, Vout, V64, ld, n, kpad, inv, Xt, dm, inv_vs, P, accumulate, ns, s);
    case 2: return ap_split_launch<__bf16>(Vin, S, Vout, V64, ld, n, kpad, inv, Xt, dm, inv_vs, P, accumulate, ns, s);
    case 3: return ap_split_launch<_Float16>(Vin, S, Vout, V64, ld, n, kpad, inv, Xt, dm, inv_vs, P, accumulate, ns, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_apply_gemm(int prec, const void *Vin, const void *S, int64_t ld, int64_t n,
                             int64_t kpad, int nsplit, float *P, hipStream_t s) {
    switch (prec) {
    case 1: return ap_gemm_launch<float>(Vin, S, ld, n, kpad, nsplit, P, s);
    case 2: return ap_gemm_launch<__bf16>(Vin, S, ld, n, kpad, nsplit, P, s);
    case 3: return ap_gemm_launch<_Float16>(Vin, S, ld, n, kpad, nsplit, P, s);
    default: return hipErrorInvalidValue;
    }
}

// V += T (FP64), Vout = V rounded; on the last level X += dm * V * (*inv_vs).
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_v(const double *T64, int64_t total, int64_t ld,
                                                double *V64, T *Vout, double *Xt,
                                                const double *dm, const double *inv_vs) {
    const double ivs = inv_vs ? *inv_vs : 0.0;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * blockDim.x) {
        const double v = V64[o] + T64[o];
        V64[o] = v;
        Vout[o] = cvtd<T>(v);
        if (inv_vs) Xt[o] += dm[o % ld] * v * ivs;
    }
}

hipError_t launch_axpy_v(int prec, const double *T64, int64_t ld, int64_t kpad, double *V64,
                         void *Vout, double *Xt, const double *dm, const double *inv_vs,
                         hipStream_t s) {
    const int64_t total = kpad * ld;
    const int grid = (int)(cdiv(total, 256) < 16384 ? cdiv(total, 256) : 16384);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_axpy_v<double>, dim3(grid), dim3(256), 0, s, T64, total, ld, V64, (double *)Vout, Xt, dm, inv_vs); break;
    case 1: hipLaunchKernelGGL(k_axpy_v<float>, dim3(grid), dim3(256), 0, s, T64, total, ld, V64, (float *)Vout, Xt, dm, inv_vs); break;
    case 2: hipLaunchKernelGGL(k_axpy_v<__bf16>, dim3(grid), dim3(256), 0, s, T64, total, ld, V64, (__bf16 *)Vout, Xt, dm, inv_vs); break;
    case 3: hipLaunchKernelGGL(k_axpy_v<_Float16>, dim3(grid), dim3(256), 0, s, T64, total, ld, V64, (_Float16 *)Vout, Xt, dm, inv_vs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Level 0 of many snapshots' chains in grouped launches (the per-snapshot
// kernels' workgroups, found through prefix tables: the same bits).

__global__ __launch_bounds__(256) void k_chain_prep_grouped(const GraphSnap *snaps, const int *prefix,
                                                            int P) {
    const int p = group_find(prefix, P, blockIdx.x);
    const GraphSnap &d = snaps[p];
    chain_prep_elem(d.deg, d.stats, d.n, d.ld, 0, d.dmn, d.dm, d.u,
                    (int64_t)(blockIdx.x - prefix[p]) * 256 + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_normalize_grouped(const GraphSnap *snaps, const int *prefix,
                                                           int P) {
    const int p = group_find(prefix, P, blockIdx.x);
    const GraphSnap &d = snaps[p];
    const int nt = (int)(d.ld / 64);
    normalize_tile<T>(d.W, d.ld, d.n, d.dmn, d.u, 0, d.scale, nt, (T *)d.level0, d.fro, d.fro64,
                      xcd_remap(blockIdx.x - prefix[p], prefix[p + 1] - prefix[p]));
}

hipError_t launch_chain_level0_grouped(int prec, const GraphSnap *snaps, const int *tables,
                                       const int *totals, int P, hipStream_t s) {
    auto tb = [&](int t) { return tables + (size_t)t * (P + 1); };
    hipLaunchKernelGGL(k_chain_prep_grouped, dim3(totals[kGtPrep]), dim3(256), 0, s, snaps, tb(kGtPrep), P);
    const dim3 g((unsigned)totals[kGtSym]), b(256);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_normalize_grouped<double>, g, b, 0, s, snaps, tb(kGtSym), P); break;
    case 1: hipLaunchKernelGGL(k_normalize_grouped<float>, g, b, 0, s, snaps, tb(kGtSym), P); break;
    case 2: hipLaunchKernelGGL(k_normalize_grouped<__bf16>, g, b, 0, s, snaps, tb(kGtSym), P); break;
    case 3: hipLaunchKernelGGL(k_normalize_grouped<_Float16>, g, b, 0, s, snaps, tb(kGtSym), P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace cdl
