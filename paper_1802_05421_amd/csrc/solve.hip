// Embedding solve (Algorithm 3 with Algorithm 1's right-hand sides; the
// refinement is EstimateSolution of Algorithm 2 with P2 y = P1 L y, batched
// over the k columns).
//
//   rhs         Y = B^T W^{1/2} Q^T / sqrt(k) with counter-based SplitMix64
//               signs: per row, the signed sums as an exact int8 MFMA
//               product of the sign bits with base-256 digits of the scaled
//               weights; the pair form serves two snapshots on one node set
//               with each sign word
//   streamed    the products with W of the streamed solve, one row panel of
//               W at a time, and the one-level chain's vector steps
//   residual    R = Y - (deg * X - W X) on FP64 MFMA, per-column partial
//               sums of R^2 and the tile maximum of |D^{-1/2} R|
//   col_norms   ||R_r|| (fixed-order sums) and a power-of-two scale for the
//               next preconditioner operand
//   prep_v      V = scale * D^{-1/2} R in FP64 and rounded to the chain type
//   finalize_z  centre the columns of X and transpose it into Z (n x k)
//
// Vectors of k columns are stored transposed: row r of a kpad x ld panel
// holds column r over all (padded) nodes.
#include "batch.h"
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace cdl {

// Right-hand sides on the int8 matrix cores.
//
// Column r of row i is y_i[r] = (T - 2 M_r) / sqrt(k): v_j = c_j sqrt(W_ij)
// (c_j = -1 when i is the tail of edge {i, j}, the end with the higher global
// id), T = sum_j v_j and M_r = sum_j b_jr v_j, where b_jr is bit r mod 64 of
// the SplitMix64 sign word of the edge for projection block r / 64 (a set bit
// negates the sign; Steele, Lea & Flood, OOPSLA 2014, for the mixer).  For a
// row, M is a (columns x neighbours) 0/1 matrix times the vector v, summed
// here exactly on v_mfma_i32_16x16x64_i8:
//   * per chunk of 1024 neighbours and snapshot, v is scaled by a power of two
//     2^e chosen from the chunk's largest |v| so that V = rint(2^e v) has
//     |V| <= 2^54, and V is split into seven balanced base-256 digits d_s in
//     [-128, 127] (V = sum_s d_s 256^s: the bytes of V + 0x80808080808080,
//     each XOR 0x80);
//   * the sign bits enter as bytes holding one bit, 2^p with p in 0..7 (p = 7
//     reads as -128 in int8): bit plane b of a 64-bit word is its byte b, and
//     MFMA c (c = 0..3) takes for its row m the bit 4 m + c, found in byte
//     m / 2 at position p = 4 (m & 1) + c, by one AND per four neighbours;
//   * one MFMA multiplies 16 columns by 16 digit slots (seven digits of each
//     snapshot and a zero slot) over 64 neighbours; the int32 sums are
//     exact (|sum| <= 2^22 per chunk and wave) and are scaled into FP64
//     accumulators (times 256^s 2^-e / 2^p, all powers of two) whenever e
//     changes and every 256 chunks.
// So the only rounding is V = rint(2^e v) (at most 2^-55 of the chunk's
// largest |v| per term) and the FP64 sums; T is summed in FP64 from v itself,
// which also carries non-finite weights into y.
//
// A workgroup is one row and NB projection blocks of 64 columns: 4 NB waves,
// wave (beta, kq) multiplying its block over every fourth 64-neighbour step
// of a chunk.  Staging, per chunk: thread (beta, q) hashes the sign words of
// neighbours q + 256 e (e = 0..3) and stores them as 8 bit planes of 4
// bytes; the digit threads (one per snapshot and q) take the square roots,
// the chunk maxima and the digits, stored as 7 rows of 4 bytes.  A neighbour
// sits at the same byte position in the planes and in the digit rows, which
// is all the contraction needs.  The sign words and digits of chunk c are
// staged while the MFMAs of chunk c - 1 run from the other LDS buffer; the
// loads and square roots of chunk c + 1 follow; one barrier per chunk.

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kRhsChunk = 1024;
constexpr int kRhsPitch = kRhsChunk + 64;   // bytes per LDS row (spreads the banks)

static uint64_t splitmix64_mix_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rhs_sign_word(uint64_t mseed, uint64_t key) {
    uint64_t z = mseed ^ key;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// out[b] = byte b of a0, a1, a2, a3 (in that order from the low byte): a
// 4 x 4 byte transpose in eight v_perm_b32 (perm(x, y, s) takes result byte
// t from byte s_t of the 64-bit value x:y, y in the low half).
__device__ __forceinline__ void rhs_bytes4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                                           uint32_t out[4]) {
    const uint32_t l01 = __builtin_amdgcn_perm(a1, a0, 0x05010400u);   // a0.0 a1.0 a0.1 a1.1
    const uint32_t l23 = __builtin_amdgcn_perm(a3, a2, 0x05010400u);
    const uint32_t h01 = __builtin_amdgcn_perm(a1, a0, 0x07030602u);   // a0.2 a1.2 a0.3 a1.3
    const uint32_t h23 = __builtin_amdgcn_perm(a3, a2, 0x07030602u);
    out[0] = __builtin_amdgcn_perm(l23, l01, 0x05040100u);
    out[1] = __builtin_amdgcn_perm(l23, l01, 0x07060302u);
    out[2] = __builtin_amdgcn_perm(h23, h01, 0x05040100u);
    out[3] = __builtin_amdgcn_perm(h23, h01, 0x07060302u);
}

// 2^e for -1022 <= e <= 1023.
__device__ __forceinline__ double rhs_pow2(int e) { return __hiloint2double((e + 1023) << 20, 0); }

// Scale exponent of a chunk whose largest |v| has high word h: 2^q |v| < 2^54.
__device__ __forceinline__ int rhs_qexp(uint32_t h) {
    const int q = 1076 - (int)(h >> 20);
    return q < -1000 ? -1000 : (q > 1000 ? 1000 : q);
}

template <int NB, int S>
__global__ __launch_bounds__(256 * NB) void k_rhs(const double *W0, const double *W1, int64_t ld,
                                                  int64_t n, int64_t row0, int64_t row1,
                                                  const int32_t *gid, int64_t k, uint64_t mseed,
                                                  double inv_sqrt_k, int nb, double *Y0t,
                                                  double *Y1t) {
    constexpr int NT = 256 * NB;
    constexpr int DG = (S * 256 + NT - 1) / NT;       // digit groups per thread
    constexpr int PL = 2 * NB * 8 * kRhsPitch;         // bit planes, two buffers
    constexpr int DB = 2 * 16 * kRhsPitch;             // digit rows, two buffers
    static_assert(NB * 4 * S * 64 * 8 <= PL, "reduction buffer must fit the planes");
    __shared__ __align__(16) unsigned char smem[PL + DB];
    __shared__ uint32_t wmax[2][S * 4];
    __shared__ double tred[S][4];
    unsigned char *const planes = smem, *const digs = smem + PL;

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int nbg = (nb + NB - 1) / NB;
    // The projection groups of one row take ids kNumXcd apart (one XCD).
    const int w = blockIdx.x, per = kNumXcd * nbg, l = w % per;
    const int64_t i = row0 + (int64_t)(w / per) * kNumXcd + l % kNumXcd;
    const int bgrp = l / kNumXcd;
    if (i >= row1) return;
    const uint32_t gi = gid ? (uint32_t)gid[i] : (uint32_t)i;
    const int64_t wrow = (i - row0) * ld;

    // roles
    const int q = t & 255, bw = t >> 8;                        // sign words
    const bool word_on = bgrp * NB + bw < nb;
    const uint64_t kbeta = (uint64_t)(bgrp * NB + bw) << 40;
    const int mb = wv >> 2, kq = wv & 3, m16 = lane & 15, g4 = lane >> 4;   // MFMAs
    const bool mfma_on = bgrp * NB + mb < nb;
    const int sn = S == 2 ? (m16 >> 3) : 0;                     // snapshot of this lane's slot
    uint32_t mask[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) mask[c] = 0x01010101u << (4 * (m16 & 1) + c);

    // zero the digit rows once (the unused slots stay zero)
    for (int o = t * 16; o < DB; o += NT * 16) *(uint4 *)(digs + o) = make_uint4(0, 0, 0, 0);

    uint32_t gn[4];            // global ids of the next chunk's neighbours
    double vn[DG][4];          // its signed square roots
    double tp[DG];             // running sums of v
#pragma unroll
    for (int d = 0; d < DG; ++d) tp[d] = 0.0;

    // (indices clamped into the row, so that the loads need no branches)
    auto load_ids = [&](int64_t j0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + q + 256 * e, jc = j < n ? j : n - 1;
            const uint32_t g = gid ? (uint32_t)gid[jc] : (uint32_t)jc;
            gn[e] = j < n ? g : 0u;
        }
    };
    auto load_w = [&](int64_t j0) {
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            const int gx = t + d * NT;
            if (gx >= S * 256) continue;
            const double *Ws = (S == 2 && (gx >> 8)) ? W1 : W0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = j0 + q + 256 * e, jc = j < n ? j : n - 1;
                const double x = Ws[wrow + jc];
                vn[d][e] = j < n ? x : 0.0;
            }
        }
    };
    // square roots (correctly rounded), signs, running sums and the chunk
    // maxima of the loaded weights, into slot `slot`
    auto roots = [&](int slot) {
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            const int gx = t + d * NT;
            if (gx >= S * 256) continue;
            uint32_t h = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double r = sqrt(vn[d][e]);
                vn[d][e] = gi > gn[e] ? -r : r;
                tp[d] += vn[d][e];
                const uint32_t hv = (uint32_t)__double2hiint(r) & 0x7fffffffu;
                h = h > hv ? h : hv;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const uint32_t x = (uint32_t)__shfl_xor((int)h, o);
                h = h > x ? h : x;
            }
            if (lane == 0) wmax[slot][gx >> 6] = h;
        }
    };

    i32x4 acc[4];
    double acc64[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        acc[c] = i32x4{0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[c][r] = 0.0;
    }
    // The integer sums are scaled into FP64 when the scale exponent of this
    // lane's snapshot changes (in any lane of the wave) and every 256 chunks
    // (|sum| < 2^30).
    int qacc = 0, held = 0;
    auto flush = [&]() {
        const int sl = m16 & 7;
        const double f = sl < 7 ? rhs_pow2(8 * sl - qacc) : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[c][r] = fma((double)acc[c][r], f, acc64[c][r]);
            acc[c] = i32x4{0, 0, 0, 0};
        }
        held = 0;
    };
    // the MFMAs of the chunk in buffer pb (qx: its scale exponent for this
    // lane's snapshot)
    auto multiply = [&](int pb, int qx) {
        if (!mfma_on) return;
        if (held == 0) {
            qacc = qx;
        } else if (__any(qx != qacc) || held == 256) {
            flush();
            qacc = qx;
        }
        ++held;
        const unsigned char *pa = planes + ((pb * NB + mb) * 8 + (m16 >> 1)) * kRhsPitch + 16 * g4;
        const unsigned char *pd = digs + (pb * 16 + m16) * kRhsPitch + 16 * g4;
#pragma unroll
        for (int kk = 0; kk < kRhsChunk / 256; ++kk) {
            const int off = (kk * 4 + kq) * 64;
            const uint4 a = *(const uint4 *)(pa + off);
            const i32x4 b = *(const i32x4 *)(pd + off);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const i32x4 ac = i32x4{(int)(a.x & mask[c]), (int)(a.y & mask[c]),
                                       (int)(a.z & mask[c]), (int)(a.w & mask[c])};
                acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ac, b, acc[c], 0, 0, 0);
            }
        }
    };

    const int64_t nch = cdiv(n, kRhsChunk);
    load_ids(0);
    load_w(0);
    roots(0);
    __syncthreads();
    int qprev = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        const int buf = (int)(ch & 1), slot = buf;
        int qs[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            uint32_t h = wmax[slot][4 * s];
#pragma unroll
            for (int u = 1; u < 4; ++u) h = h > wmax[slot][4 * s + u] ? h : wmax[slot][4 * s + u];
            qs[s] = rhs_qexp(h);
        }
        // digits of this chunk
#pragma unroll
        for (int d = 0; d < DG; ++d) {
            const int gx = t + d * NT;
            if (gx >= S * 256) continue;
            const int s = gx >> 8;
            const double Q = rhs_pow2(S == 2 && s ? qs[S - 1] : qs[0]);
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // (clamped, so that non-finite weights convert without
                // overflow; T carries them)
                const double x = fmin(fmax(rint(vn[d][e] * Q), -0x1p54), 0x1p54);
                const double xh = floor(x * 0x1p-32);
                const double xl = fma(xh, -0x1p32, x);
                const uint64_t u = (((uint64_t)(uint32_t)(int)xh << 32) | (uint32_t)xl) +
                                   0x80808080808080ull;
                lo[e] = (uint32_t)u ^ 0x80808080u;
                hi[e] = (uint32_t)(u >> 32) ^ 0x808080u;
            }
            uint32_t o[4];
            unsigned char *pd = digs + (buf * 16 + 8 * s) * kRhsPitch + 4 * q;
            rhs_bytes4(lo[0], lo[1], lo[2], lo[3], o);
#pragma unroll
            for (int b = 0; b < 4; ++b) *(uint32_t *)(pd + b * kRhsPitch) = o[b];
            rhs_bytes4(hi[0], hi[1], hi[2], hi[3], o);
#pragma unroll
            for (int b = 0; b < 3; ++b) *(uint32_t *)(pd + (4 + b) * kRhsPitch) = o[b];
        }
        // sign words of this chunk
        if (word_on) {
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t a = gi < gn[e] ? gi : gn[e], b = gi < gn[e] ? gn[e] : gi;
                const uint64_t wd = rhs_sign_word(mseed, kbeta | ((uint64_t)a << 20) | b);
                lo[e] = (uint32_t)wd;
                hi[e] = (uint32_t)(wd >> 32);
            }
            uint32_t o[4];
            unsigned char *pp = planes + (buf * NB + bw) * 8 * kRhsPitch + 4 * q;
            rhs_bytes4(lo[0], lo[1], lo[2], lo[3], o);
#pragma unroll
            for (int b = 0; b < 4; ++b) *(uint32_t *)(pp + b * kRhsPitch) = o[b];
            rhs_bytes4(hi[0], hi[1], hi[2], hi[3], o);
#pragma unroll
            for (int b = 0; b < 4; ++b) *(uint32_t *)(pp + (4 + b) * kRhsPitch) = o[b];
        }
        const bool more = ch + 1 < nch;
        if (more) {
            load_ids((ch + 1) * kRhsChunk);
            load_w((ch + 1) * kRhsChunk);
        }
        if (ch > 0) multiply(buf ^ 1, qprev);
        qprev = S == 2 && sn ? qs[S - 1] : qs[0];
        if (more) roots(slot ^ 1);
        __syncthreads();
    }
    multiply((int)((nch - 1) & 1), qprev);
    if (mfma_on) flush();
    __syncthreads();   // the planes now hold the reduction buffer

    // sum each snapshot's seven digit slots (lanes m16 & 7 = 0..6) and undo
    // the bit scale 2^p, p = 4 (row & 1) + c for accumulator row 4 g4 + r
    double *red = (double *)smem;   // [NB][4][S][64]
    if (mfma_on) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double x = acc64[c][r];
                x += __shfl_xor(x, 1);
                x += __shfl_xor(x, 2);
                x += __shfl_xor(x, 4);
                const int p = 4 * (r & 1) + c;
                const double inv = p == 7 ? -0x1p-7 : rhs_pow2(-p);
                if ((m16 & 7) == 0 && (m16 >> 3) < S)
                    red[((mb * 4 + kq) * S + sn) * 64 + 16 * g4 + 4 * r + c] = x * inv;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        const int gx = t + d * NT;
        if (gx >= S * 256) continue;
        double x = tp[d];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) tred[gx >> 8][(gx >> 6) & 3] = x;
    }
    __syncthreads();
    if (t < NB * S * 64) {
        const int b = t / (S * 64), s = (t / 64) % S, r = t & 63;
        const int beta = bgrp * NB + b;
        if (beta < nb) {
            const double *rb = red + (b * 4 * S + s) * 64 + r;
            const double M = ((rb[0] + rb[S * 64]) + rb[2 * S * 64]) + rb[3 * S * 64];
            const double T = ((tred[s][0] + tred[s][1]) + tred[s][2]) + tred[s][3];
            const int64_t col = (int64_t)beta * 64 + r;
            double *Y = s == 0 ? Y0t : Y1t;
            Y[col * ld + i] = col < k ? (T - 2.0 * M) * inv_sqrt_k : 0.0;
        }
    }
}

template <int S>
static hipError_t launch_rhs_k(const double *W0, const double *W1, int64_t ld, int64_t n,
                               int64_t row0, int64_t row1, const int32_t *gid, int64_t k,
                               int64_t kpad, uint64_t seed, double *Y0t, double *Y1t,
                               hipStream_t s) {
    if (row0 < 0 || row1 > n) return hipErrorInvalidValue;
    if (row1 <= row0) return hipSuccess;
    const uint64_t mseed = splitmix64_mix_host(seed);
    const int nb = (int)(kpad / 64);
    const int NB = nb >= 3 ? 4 : nb;
    const int nbg = (nb + NB - 1) / NB;
    const int64_t rows = cdiv(row1 - row0, kNumXcd) * kNumXcd;
    const dim3 grid((unsigned)(rows * nbg));
    const double isk = 1.0 / sqrt((double)k);
    switch (NB) {
    case 4: hipLaunchKernelGGL((k_rhs<4, S>), grid, dim3(1024), 0, s, W0, W1, ld, n, row0, row1, gid, k, mseed, isk, nb, Y0t, Y1t); break;
    case 2: hipLaunchKernelGGL((k_rhs<2, S>), grid, dim3(512), 0, s, W0, W1, ld, n, row0, row1, gid, k, mseed, isk, nb, Y0t, Y1t); break;
    default: hipLaunchKernelGGL((k_rhs<1, S>), grid, dim3(256), 0, s, W0, W1, ld, n, row0, row1, gid, k, mseed, isk, nb, Y0t, Y1t); break;
    }
    return hipGetLastError();
}

hipError_t launch_rhs_pair(const double *W0, const double *W1, int64_t ld, int64_t n,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Y0t, double *Y1t, hipStream_t s) {
    return launch_rhs_k<2>(W0, W1, ld, n, 0, n, gid, k, kpad, seed, Y0t, Y1t, s);
}

hipError_t launch_rhs_rows(const double *W, int64_t ld, int64_t n, int64_t row0, int64_t row1,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Yt, hipStream_t s) {
    return launch_rhs_k<1>(W, nullptr, ld, n, row0, row1, gid, k, kpad, seed, Yt, nullptr, s);
}

hipError_t launch_rhs(const double *W, int64_t ld, int64_t n, const int32_t *gid, int64_t k,
                      int64_t kpad, uint64_t seed, double *Yt, hipStream_t s) {
    return launch_rhs_rows(W, ld, n, 0, n, gid, k, kpad, seed, Yt, s);
}

// ---------------------------------------------------------------------------
// FP64 residual R = Y - deg * X + W X, as a split-K MFMA GEMM
// P[s][r][i] = sum_{j in split s} Xt[r][j] W[i][j] followed by a reduction
// that forms R, the next preconditioner operand and the column-norm partials.

// BT: W is the whole symmetric matrix, read along its rows as W^T (k-tiles of
// 16 rows x 128 contiguous columns); row panels are read as they are.
template <int BM, bool BT = false> struct ResCfg {
    static constexpr int WM = BM / 64, WN = 8 / (BM / 64);
    using Core = GemmCore<MfmaF64, BM, 128, 16, WM, WN, BT>;
};

// W may be a row panel: its row q holds node row0 + q, whose products land in
// column row0 + q of the partials (row0 = 0 for the whole matrix).
template <int BM, bool BT>
__device__ __forceinline__ void residual_gemm_tile(const double *Xt, const double *W, int64_t ld,
                                          int64_t kend, int64_t ks, int mt, int nt, double *P,
                                          int64_t kpad, int64_t row0, int id, char *smem_raw) {
    using Core = typename ResCfg<BM, BT>::Core;
    double *smem = (double *)smem_raw;
    // split-major order: the WGs of one split stream the same K range
    const int split = id / (mt * nt);
    int I, J;
    rect_tile<4>(id % (mt * nt), mt, nt, I, J);
    const int64_t m0 = (int64_t)I * BM, n0 = (int64_t)J * 128;
    const int64_t k0 = (int64_t)split * ks;
    const int64_t kk = k0 < kend ? (kend - k0 < ks ? kend - k0 : ks) : 0;
    Core g;
    g.run(Xt + k0, ld, BT ? W + k0 * ld : W + k0, ld, m0, n0, kk, smem);
    double *Ps = P + (int64_t)split * kpad * ld + row0;
#pragma unroll
    for (int a = 0; a < Core::WTM; ++a)
#pragma unroll
        for (int b = 0; b < Core::WTN; ++b)
#pragma unroll
            for (int rr = 0; rr < MfmaF64::R; ++rr)
                Ps[(m0 + Core::row_of(a, rr)) * ld + n0 + Core::col_of(b)] = g.acc[a][b][rr];
}

template <int BM, bool BT>
__global__ __launch_bounds__(512) void k_residual_gemm(const double *Xt, const double *W,
                                                       int64_t ld, int64_t kend, int64_t ks,
                                                       int mt, int nt, int S, double *P,
                                                       int64_t kpad, int64_t row0) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int id = xcd_remap(blockIdx.x, mt * nt * S);
    residual_gemm_tile<BM, BT>(Xt, W, ld, kend, ks, mt, nt, P, kpad, row0, id, smem_raw);
}

static int res_bm(int64_t kpad) { return kpad % 256 == 0 ? 256 : (kpad % 128 == 0 ? 128 : 64); }

// k-range of one split of the residual product (16-element multiples).
__host__ __device__ inline int64_t residual_split_len(int64_t n, int S) {
    const int64_t kend = (n + 63) / 64 * 64;
    return (cdiv(kend, S) + 15) / 16 * 16;
}

// Split-K count of the FP64 residual product: choice 0 aims at >= 256
// workgroups, 1 halves that count, 2 doubles it (at least four 16-wide
// k-tiles per split either way).
int residual_splits_fixed(int64_t n, int S) {
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t smax = kend / 64 > 0 ? kend / 64 : 1;   // >= 4 k-tiles per split
    return (int)(S < 1 ? 1 : S > smax ? smax : S);
}

int residual_splits(int64_t ld, int64_t kpad, int64_t n, int choice) {
    const int64_t base = (kpad / res_bm(kpad)) * (ld / 128);
    const int64_t kend = (n + 63) / 64 * 64;
    int64_t S = (256 + base - 1) / base;          // aim at >= 256 workgroups
    if (choice == 1) S = S / 2;
    if (choice == 2) S = 2 * S;
    const int64_t smax = kend / 64 > 0 ? kend / 64 : 1;   // >= 4 k-tiles per split
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    return (int)S;
}

template <int BM>
static hipError_t resg_launch(const double *Xt, const double *W, int64_t ld, int64_t n,
                              int64_t kpad, int S, double *P, hipStream_t s) {
    using Core = typename ResCfg<BM, true>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_residual_gemm<BM, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(ld / 128);
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t ks = (cdiv(kend, S) + 15) / 16 * 16;
    hipLaunchKernelGGL((k_residual_gemm<BM, true>), dim3(mt * nt * S), dim3(512), Core::SMEM, s, Xt, W,
                       ld, kend, ks, mt, nt, S, P, kpad, (int64_t)0);
    return hipGetLastError();
}

template <int BM>
static hipError_t panel_launch(const double *Vt, const double *Wp, int64_t ld, int64_t n,
                               int64_t kpad, int64_t row0, int64_t rows, double *Prod,
                               hipStream_t s) {
    using Core = typename ResCfg<BM, false>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_residual_gemm<BM, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(rows / 128);
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t ks = (kend + 15) / 16 * 16;
    hipLaunchKernelGGL((k_residual_gemm<BM, false>), dim3(mt * nt), dim3(512), Core::SMEM, s, Vt, Wp, ld,
                       kend, ks, mt, nt, 1, Prod, kpad, row0);
    return hipGetLastError();
}

hipError_t launch_panel_product(const double *Vt, const double *Wp, int64_t ld, int64_t n,
                                int64_t kpad, int64_t row0, int64_t rows, double *Prod,
                                hipStream_t s) {
    if (rows <= 0 || rows % 128 || row0 < 0 || row0 + rows > ld || kpad % 64)
        return hipErrorInvalidValue;
    switch (res_bm(kpad)) {
    case 256: return panel_launch<256>(Vt, Wp, ld, n, kpad, row0, rows, Prod, s);
    case 128: return panel_launch<128>(Vt, Wp, ld, n, kpad, row0, rows, Prod, s);
    default: return panel_launch<64>(Vt, Wp, ld, n, kpad, row0, rows, Prod, s);
    }
}

// R[r][i] = Y - deg X + sum_s P[s] (zero outside r < k, i < n; Y = NULL
// reads as zero, giving -L X); optional
// V = dm R (FP64) and V rounded to the chain type; per (256-node block, r)
// partial sums of R^2 and per-block maxima of |dm R|.
// Node block bx, column r of the residual's reduction (one workgroup).
template <typename T>
__device__ inline void residual_reduce_block(
    const double *P, int S, const double *Yt, const double *Xt, const double *deg,
    const double *dm, int64_t ld, int64_t n, int64_t k, int64_t kpad, int skip_gemm,
    double *Rt, double *V64, T *Vlo, double *npart, double *mpart, int64_t bx, int64_t r,
    double *red, double *redm) {
    const int64_t i = bx * 256 + threadIdx.x;
    const int64_t o = r * ld + i;
    double R = 0.0;
    if (r < k && i < n) {
        double acc = 0.0;
        if (!skip_gemm)
            for (int q = 0; q < S; ++q) acc += P[(int64_t)q * kpad * ld + o];
        R = (Yt ? Yt[o] : 0.0) - deg[i] * Xt[o] + acc;
    }
    Rt[o] = R;
    const double v = dm[i] * R;
    if (Vlo) {
        V64[o] = v;
        Vlo[o] = cvtd<T>(v);
    }
    double ss = R * R, mx = fabs(v);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ss += __shfl_xor(ss, off);
        mx = fmax(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = ss;
        redm[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        npart[bx * kpad + r] = (red[0] + red[1]) + (red[2] + red[3]);
        mpart[bx * kpad + r] = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_residual_reduce(
    const double *P, int S, const double *Yt, const double *Xt, const double *deg,
    const double *dm, int64_t ld, int64_t n, int64_t k, int64_t kpad, int skip_gemm,
    double *Rt, double *V64, T *Vlo, double *npart, double *mpart) {
    __shared__ double red[4], redm[4];
    residual_reduce_block<T>(P, S, Yt, Xt, deg, dm, ld, n, k, kpad, skip_gemm, Rt, V64, Vlo, npart,
                             mpart, blockIdx.x, blockIdx.y, red, redm);
}

hipError_t launch_residual_reduce(const double *P, int S, const double *Yt, const double *Xt,
                                  const double *deg, const double *dm, int64_t ld, int64_t n,
                                  int64_t kpad, int64_t k, double *Rt, double *npart,
                                  double *mpart, hipStream_t s) {
    dim3 grid((unsigned)(ld / 256), (unsigned)kpad), blk(256);
    hipLaunchKernelGGL(k_residual_reduce<double>, grid, blk, 0, s, P, S, Yt, Xt, deg, dm, ld, n,
                       k, kpad, 0, Rt, (double *)nullptr, (double *)nullptr, npart, mpart);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streamed solve (the weights recomputed panel by panel): the one-level
// chain P1 = D^{-1/2} (I + S) D^{-1/2} = D^{-1} + D^{-1} W D^{-1} (Algorithm
// 2 with d = 1).  Its apply is Xt += U + D^{-1} (W U), U = D^{-1} R.

__global__ void k_stream_prep(const double *deg, int64_t n, int64_t ld, double *dinv,
                              double *rdeg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    const double d = i < n ? deg[i] : 0.0;
    dinv[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    rdeg[i] = d > 0.0 ? 1.0 / d : 0.0;
}

hipError_t launch_stream_prep(const double *deg, int64_t n, int64_t ld, double *dinv,
                              double *rdeg, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_prep, dim3((unsigned)cdiv(ld, 256)), dim3(256), 0, s, deg, n, ld,
                       dinv, rdeg);
    return hipGetLastError();
}

// One thread per element of the kpad x ld panels (zero rows and columns stay zero:
// rdeg is zero beyond n and R is zero beyond k).
__global__ void k_stream_scale(const double *Rt, const double *rdeg, int64_t ld, int64_t total,
                               double *Ut) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    Ut[o] = Rt[o] * rdeg[o % ld];
}

hipError_t launch_stream_scale(const double *Rt, const double *rdeg, int64_t ld, int64_t kpad,
                               double *Ut, hipStream_t s) {
    const int64_t total = ld * kpad;
    hipLaunchKernelGGL(k_stream_scale, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, Rt,
                       rdeg, ld, total, Ut);
    return hipGetLastError();
}

__global__ void k_stream_update(const double *Ut, const double *Prod, const double *rdeg,
                                int64_t ld, int64_t total, double *Xt) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    Xt[o] += Ut[o] + rdeg[o % ld] * Prod[o];
}

hipError_t launch_stream_update(const double *Ut, const double *Prod, const double *rdeg,
                                int64_t ld, int64_t kpad, double *Xt, hipStream_t s) {
    const int64_t total = ld * kpad;
    hipLaunchKernelGGL(k_stream_update, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, Ut,
                       Prod, rdeg, ld, total, Xt);
    return hipGetLastError();
}

hipError_t launch_residual_gemm(const double *Xt, const double *W, int64_t ld, int64_t n,
                                int64_t kpad, int S, double *P, hipStream_t s) {
    switch (res_bm(kpad)) {
    case 256: return resg_launch<256>(Xt, W, ld, n, kpad, S, P, s);
    case 128: return resg_launch<128>(Xt, W, ld, n, kpad, S, P, s);
    default: return resg_launch<64>(Xt, W, ld, n, kpad, S, P, s);
    }
}

hipError_t launch_residual_reduce_k(int prec, const double *P, int S, const double *Yt,
                                    const double *Xt, const double *deg, const double *dm,
                                    int64_t ld, int64_t n, int64_t kpad, int64_t k, double *Rt,
                                    double *V64, void *Vlo, double *npart, double *mpart,
                                    hipStream_t s) {
    const int skip = S == 0;
    dim3 grid((unsigned)(ld / 256), (unsigned)kpad), blk(256);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_residual_reduce<double>, grid, blk, 0, s, P, S, Yt, Xt, deg, dm, ld, n, k, kpad, skip, Rt, V64, (double *)Vlo, npart, mpart); break;
    case 1: hipLaunchKernelGGL(k_residual_reduce<float>, grid, blk, 0, s, P, S, Yt, Xt, deg, dm, ld, n, k, kpad, skip, Rt, V64, (float *)Vlo, npart, mpart); break;
    case 2: hipLaunchKernelGGL(k_residual_reduce<__bf16>, grid, blk, 0, s, P, S, Yt, Xt, deg, dm, ld, n, k, kpad, skip, Rt, V64, (__bf16 *)Vlo, npart, mpart); break;
    default: hipLaunchKernelGGL(k_residual_reduce<_Float16>, grid, blk, 0, s, P, S, Yt, Xt, deg, dm, ld, n, k, kpad, skip, Rt, V64, (_Float16 *)nullptr, npart, mpart); break;
    }
    return hipGetLastError();
}

// prec < 0: no fused operand (FP16 chains scale it separately).
hipError_t launch_residual_k(int prec, const double *Xt, const double *W, const double *Yt,
                             const double *deg, const double *dm, int64_t ld, int64_t n,
                             int64_t kpad, int64_t k, int skip_gemm, double *P, double *Rt,
                             double *V64, void *Vlo, double *npart, double *mpart,
                             hipStream_t s) {
    const int S = residual_splits(ld, kpad, n, 0);
    if (!skip_gemm) {
        hipError_t e = launch_residual_gemm(Xt, W, ld, n, kpad, S, P, s);
        if (e != hipSuccess) return e;
    }
    return launch_residual_reduce_k(prec, P, skip_gemm ? 0 : S, Yt,
                                    Xt, deg, dm, ld, n, kpad, k, Rt, V64, Vlo, npart, mpart, s);
}

int residual_parts(int64_t ld) { return (int)(ld / 256); }

int residual_tiles(int64_t ld, int64_t kpad) { return (int)(ld / 256 * kpad); }

// out[r] = ||R_r|| (fixed-order sum of the partials), r < kpad; block kpad
// writes out[kpad] = scale, out[kpad+1] = 1/scale: a power of two bringing
// max |D^{-1/2} R| into [0.5, 1) when `scaled`, else 1.
__device__ inline void col_norms_block(const double *npart, int nparts, int64_t kpad,
                                       const double *mpart, int ntiles, int scaled, double *out,
                                       int64_t r, double *red) {
    if (r < kpad) {
        double s = 0.0;
        for (int p = threadIdx.x; p < nparts; p += 256) s += npart[(int64_t)p * kpad + r];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) out[r] = sqrt((red[0] + red[1]) + (red[2] + red[3]));
        return;
    }
    double m = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 256) m = fmax(m, mpart[t]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        double sc = 1.0;
        if (scaled && m > 0.0 && isfinite(m)) sc = ldexp(1.0, -ilogb(m) - 1);
        out[kpad] = sc;
        out[kpad + 1] = 1.0 / sc;
    }
}

__global__ __launch_bounds__(256) void k_col_norms(const double *npart, int nparts,
                                                   int64_t kpad, const double *mpart,
                                                   int ntiles, int scaled, double *out) {
    __shared__ double red[4];
    col_norms_block(npart, nparts, kpad, mpart, ntiles, scaled, out, blockIdx.x, red);
}

hipError_t launch_col_norms2(const double *npart, int nparts, int64_t kpad, const double *mpart,
                             int ntiles, int scaled, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_col_norms, dim3((unsigned)kpad + 1), dim3(256), 0, s, npart, nparts, kpad,
                       mpart, ntiles, scaled, out);
    return hipGetLastError();
}

template <typename T>
__device__ inline void prep_v_range(const double *Rt, const double *dm, int64_t ld, int64_t total,
                                    const double *scal, double scale_lo, double *V64, T *Vlo,
                                    int64_t first, int64_t step) {
    const double sc = *scal;
    for (int64_t o = first; o < total; o += step) {
        const int64_t col = o % ld;
        const double v = sc * dm[col] * Rt[o];
        V64[o] = v;
        Vlo[o] = cvtd<T>(v * scale_lo);
    }
}

template <typename T>
__global__ void k_prep_v(const double *Rt, const double *dm, int64_t ld, int64_t total,
                         const double *scal, double scale_lo, double *V64, T *Vlo) {
    prep_v_range<T>(Rt, dm, ld, total, scal, scale_lo, V64, Vlo,
                    (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

hipError_t launch_prep_v2(int prec, const double *Rt, const double *dm, int64_t ld, int64_t kpad,
                          const double *scal, double *V64, void *Vlo, hipStream_t s) {
    const int64_t total = kpad * ld;
    const int grid = (int)(cdiv(total, 256) < 16384 ? cdiv(total, 256) : 16384);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_prep_v<double>, dim3(grid), dim3(256), 0, s, Rt, dm, ld, total, scal, 1.0, V64, (double *)Vlo); break;
    case 1: hipLaunchKernelGGL(k_prep_v<float>, dim3(grid), dim3(256), 0, s, Rt, dm, ld, total, scal, 1.0, V64, (float *)Vlo); break;
    case 2: hipLaunchKernelGGL(k_prep_v<__bf16>, dim3(grid), dim3(256), 0, s, Rt, dm, ld, total, scal, 1.0, V64, (__bf16 *)Vlo); break;
    case 3: hipLaunchKernelGGL(k_prep_v<_Float16>, dim3(grid), dim3(256), 0, s, Rt, dm, ld, total, scal, 1.0, V64, (_Float16 *)Vlo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped over the snapshots of a sequence (one launch for all of them;
// converged snapshots skip their workgroups).

template <int BM>
__global__ __launch_bounds__(512) void k_residual_gemm_grouped(const BatchSnap *snaps, const int *prefix,
                                                               int P, int64_t kpad, const int *done) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int p = group_find(prefix, P, blockIdx.x);
    if (done[p]) return;
    const BatchSnap &d = snaps[p];
    const int mt = (int)(kpad / BM), nt = (int)(d.ld / 128);
    const int id = xcd_remap(blockIdx.x - prefix[p], prefix[p + 1] - prefix[p]);
    residual_gemm_tile<BM, true>(d.Xt, d.W, d.ld, (d.n + 63) / 64 * 64, residual_split_len(d.n, d.res_splits),
                           mt, nt, d.Pres, kpad, 0, id, smem_raw);
}

template <typename T>
__global__ __launch_bounds__(256) void k_residual_reduce_grouped(const BatchSnap *snaps, const int *prefix,
                                                                 int P, int64_t kpad, int64_t k,
                                                                 int skip_gemm, int fused,
                                                                 const int *done) {
    __shared__ double red[4], redm[4];
    const int p = group_find(prefix, P, blockIdx.x);
    if (done[p]) return;
    const BatchSnap &d = snaps[p];
    // the snapshot's (node block, column) items, strided over its workgroups
    const int64_t nb = d.ld / 256, items = nb * kpad, step = prefix[p + 1] - prefix[p];
    for (int64_t lb = blockIdx.x - prefix[p]; lb < items; lb += step) {
        residual_reduce_block<T>(d.Pres, d.res_splits, d.Yt, d.Xt, d.deg, d.dm, d.ld, d.n, k, kpad,
                                 skip_gemm, d.Rt, d.V64, fused ? (T *)d.Vlo[0] : (T *)nullptr,
                                 d.npart, d.mpart, lb % nb, lb / nb, red, redm);
        __syncthreads();   // red / redm are rewritten by the next item
    }
}

template <int BM>
static hipError_t resg_grouped_launch(const BatchSnap *snaps, const int *prefix, int total, int P,
                                      int64_t kpad, const int *done, hipStream_t s) {
    using Core = typename ResCfg<BM, true>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_residual_gemm_grouped<BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_residual_gemm_grouped<BM>, dim3(total), dim3(512), Core::SMEM, s, snaps,
                       prefix, P, kpad, done);
    return hipGetLastError();
}

int residual_gemm_tiles(int64_t ld, int64_t kpad, int S) {
    return (int)(kpad / res_bm(kpad) * (ld / 128)) * S;
}

hipError_t launch_residual_grouped(int prec, const BatchSnap *snaps, const int *prefix_gemm,
                                   int total_gemm, const int *prefix_red, int total_red, int P,
                                   int64_t kpad, int64_t k, int skip_gemm, const int *done,
                                   hipStream_t s) {
    if (!skip_gemm) {
        hipError_t e;
        switch (res_bm(kpad)) {
        case 256: e = resg_grouped_launch<256>(snaps, prefix_gemm, total_gemm, P, kpad, done, s); break;
        case 128: e = resg_grouped_launch<128>(snaps, prefix_gemm, total_gemm, P, kpad, done, s); break;
        default: e = resg_grouped_launch<64>(snaps, prefix_gemm, total_gemm, P, kpad, done, s); break;
        }
        if (e != hipSuccess) return e;
    }
    // FP16 operands get their power-of-two scale from the norms first (prep)
    const int fused = prec != 3;
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_residual_reduce_grouped<double>, dim3(total_red), dim3(256), 0, s, snaps, prefix_red, P, kpad, k, skip_gemm, fused, done); break;
    case 1: hipLaunchKernelGGL(k_residual_reduce_grouped<float>, dim3(total_red), dim3(256), 0, s, snaps, prefix_red, P, kpad, k, skip_gemm, fused, done); break;
    case 2: hipLaunchKernelGGL(k_residual_reduce_grouped<__bf16>, dim3(total_red), dim3(256), 0, s, snaps, prefix_red, P, kpad, k, skip_gemm, fused, done); break;
    case 3: hipLaunchKernelGGL(k_residual_reduce_grouped<_Float16>, dim3(total_red), dim3(256), 0, s, snaps, prefix_red, P, kpad, k, skip_gemm, fused, done); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Block b: snapshot b / (kpad + 1), column norm (or operand scale) b % (kpad + 1).
__global__ __launch_bounds__(256) void k_col_norms_grouped(const BatchSnap *snaps, int P, int64_t kpad,
                                                           int scaled, const int *done) {
    __shared__ double red[4];
    const int p = (int)(blockIdx.x / (kpad + 1));
    if (p >= P || done[p]) return;
    const BatchSnap &d = snaps[p];
    const int nparts = (int)(d.ld / 256);
    col_norms_block(d.npart, nparts, kpad, d.mpart, nparts * (int)kpad, scaled, d.scal,
                    blockIdx.x % (kpad + 1), red);
}

// One workgroup per snapshot: rel = max over the k columns of ||R_r|| / ||Y_r||;
// init: ||Y_r|| is taken from these norms.  An unconverged snapshot counts
// the iteration and is marked done once rel <= tol (tol > 0).
__global__ __launch_bounds__(256) void k_converge(const BatchSnap *snaps, int P, int64_t kpad,
                                                  int64_t k, double tol, int init, double *ynorm,
                                                  double *rel_out, int *done, int *iters) {
    __shared__ double red[4];
    const int p = blockIdx.x;
    if (p >= P || done[p]) return;
    const double *nr = snaps[p].scal;
    double *yn = ynorm + (int64_t)p * kpad;
    double rel = 0.0;
    for (int64_t r = threadIdx.x; r < k; r += 256) {
        if (init) yn[r] = nr[r];
        const double y = yn[r];
        const double q = y > 0.0 ? nr[r] / y : 0.0;
        rel = (q > rel || q != q) ? q : rel;   // NaN propagates
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double v = __shfl_xor(rel, o);
        rel = (v > rel || v != v) ? v : rel;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rel;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < 4; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
        if (init) {
            rel_out[p] = 1.0;
            return;
        }
        rel_out[p] = m;
        iters[p] += 1;
        if (tol > 0.0 && m <= tol) done[p] = 1;
    }
}

hipError_t launch_norms_grouped(const BatchSnap *snaps, int P, int64_t kpad, int64_t k,
                                int scaled, double tol, int init, double *ynorm,
                                double *rel_out, int *done, int *iters, hipStream_t s) {
    hipLaunchKernelGGL(k_col_norms_grouped, dim3((unsigned)(P * (kpad + 1))), dim3(256), 0, s, snaps,
                       P, kpad, scaled, done);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_converge, dim3((unsigned)P), dim3(256), 0, s, snaps, P, kpad, k, tol, init,
                       ynorm, rel_out, done, iters);
    return hipGetLastError();
}

template <typename T>
__global__ void k_prep_grouped(const BatchSnap *snaps, const int *prefix, int P, int64_t kpad,
                               const int *done) {
    const int p = group_find(prefix, P, blockIdx.x);
    if (done[p]) return;
    const BatchSnap &d = snaps[p];
    const int64_t nb = prefix[p + 1] - prefix[p];
    prep_v_range<T>(d.Rt, d.dm, d.ld, kpad * d.ld, d.scal + kpad, 1.0, d.V64, (T *)d.Vlo[0],
                    (int64_t)(blockIdx.x - prefix[p]) * 256 + threadIdx.x, nb * 256);
}

hipError_t launch_prep_grouped(int prec, const BatchSnap *snaps, const int *prefix, int total,
                               int P, int64_t kpad, const int *done, hipStream_t s) {
    switch (prec) {
    case 3: hipLaunchKernelGGL(k_prep_grouped<_Float16>, dim3(total), dim3(256), 0, s, snaps, prefix, P, kpad, done); break;
    default: return hipErrorInvalidValue;   // only FP16 operands are prepared separately
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_col_mean(const double *Xt, int64_t ld, int64_t n,
                                                  double *mean) {
    __shared__ double red[4];
    const int64_t r = blockIdx.x;
    // a thread's entries in increasing order, 32 loads in flight
    const int64_t cnt = n > threadIdx.x ? (n - threadIdx.x + 255) / 256 : 0;
    double s = ordered_sum(Xt + r * ld + threadIdx.x, 256, (int)cnt, 0.0);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) mean[r] = ((red[0] + red[1]) + (red[2] + red[3])) / (double)n;
}

// Z[i][r] = Xt[r][i] - mean[r] (mean NULL: no shift) through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_transpose_z(const double *Xt, int64_t ld, int64_t n,
                                                     int64_t k, const double *mean, double *Z) {
    __shared__ double t[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, i = i0 + tx;
        t[q][tx] = (r < k && i < n) ? Xt[r * ld + i] - (mean ? mean[r] : 0.0) : 0.0;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t i = i0 + q, r = r0 + tx;
        if (i < n && r < k) Z[i * k + r] = t[tx][q];
    }
}

hipError_t launch_transpose(const double *Xt, int64_t ld, int64_t n, int64_t k, double *Z,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_z, dim3((unsigned)cdiv(n, 32), (unsigned)cdiv(k, 32)),
                       dim3(256), 0, s, Xt, ld, n, k, (const double *)nullptr, Z);
    return hipGetLastError();
}

hipError_t launch_finalize_z2(const double *Xt, int64_t ld, int64_t n, int64_t kpad, int64_t k,
                              double *mean, double *Z, hipStream_t s) {
    hipLaunchKernelGGL(k_col_mean, dim3((unsigned)kpad), dim3(256), 0, s, Xt, ld, n, mean);
    hipLaunchKernelGGL(k_transpose_z, dim3((unsigned)cdiv(n, 32), (unsigned)cdiv(k, 32)),
                       dim3(256), 0, s, Xt, ld, n, k, mean, Z);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Preconditioned conjugate gradients, one independent recurrence per column
// (flexible form: beta from z_{j+1} . (r_{j+1} - r_j)), all in FP64:
//   q' = -L p (residual kernels with Y = 0); alpha = rho / (p . L p);
//   x += alpha p; r -= alpha L p;  z = P1 r (chain);  beta; p = z + beta p.

// part[j][b][r] = sum over the 256 nodes of block b of A_j[r][.] * B_j[r][.]
// for the pairs j < 2 (pair 1 skipped when A1 is NULL).
__global__ __launch_bounds__(256) void k_col_dots(const double *A0, const double *B0,
                                                  const double *A1, const double *B1,
                                                  int64_t ld, int64_t kpad, int64_t nblk,
                                                  double *part) {
    __shared__ double red[2][4];
    const int64_t r = blockIdx.y, i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t o = r * ld + i;
    double s0 = A0[o] * B0[o], s1 = A1 ? A1[o] * B1[o] : 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * kpad + r] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        part[(nblk + blockIdx.x) * kpad + r] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Per-column scalars sc = [rho | alpha | beta] (kpad each) from the block
// partials of k_col_dots, summed in block order.
//   mode 0 (after z = P1 r): rho' = z . r, zq = z . q' (q' = -L p), beta =
//          alpha zq / rho (0 on the first direction or when rho = 0); rho = rho'
//   mode 1 (after q' = -L p): alpha = -rho / (p . q') (0 when p . q' = 0)
__global__ void k_pcg_scalars(const double *part, int64_t nblk, int64_t kpad, int mode,
                              int first, double *sc) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= kpad) return;
    double d0 = 0.0, d1 = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
        d0 += part[b * kpad + r];
        d1 += part[(nblk + b) * kpad + r];
    }
    double *rho = sc, *alpha = sc + kpad, *beta = sc + 2 * kpad;
    if (mode == 0) {
        beta[r] = (first || rho[r] == 0.0) ? 0.0 : alpha[r] * d1 / rho[r];
        rho[r] = d0;
    } else {
        alpha[r] = d0 != 0.0 ? -rho[r] / d0 : 0.0;
    }
}

// p = z + beta p (p = z on the first direction).
__global__ void k_pcg_dir(const double *Zt, double *Pt, const double *beta, int64_t ld,
                          int64_t total, int first) {
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * blockDim.x)
        Pt[o] = first ? Zt[o] : Zt[o] + beta[o / ld] * Pt[o];
}

// x += alpha p, r += alpha q' (q' = -L p); V = D^{-1/2} r for the next
// preconditioner operand (unless FP16, which scales it separately) and the
// same per-block partials as the residual reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update(const double *Pt, const double *Qt,
                                                    const double *alpha, const double *dm,
                                                    int64_t ld, int64_t kpad, double *Xt,
                                                    double *Rt, double *V64, T *Vlo,
                                                    double *npart, double *mpart) {
    __shared__ double red[4], redm[4];
    const int64_t r = blockIdx.y, i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t o = r * ld + i;
    const double a = alpha[r];
    Xt[o] += a * Pt[o];
    const double R = Rt[o] + a * Qt[o];
    Rt[o] = R;
    const double v = dm[i] * R;
    if (Vlo) {
        V64[o] = v;
        Vlo[o] = cvtd<T>(v);
    }
    double ss = R * R, mx = fabs(v);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ss += __shfl_xor(ss, off);
        mx = fmax(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = ss;
        redm[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        npart[(int64_t)blockIdx.x * kpad + r] = (red[0] + red[1]) + (red[2] + red[3]);
        mpart[(int64_t)blockIdx.x * kpad + r] = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
    }
}

hipError_t launch_col_dots(const double *A0, const double *B0, const double *A1,
                           const double *B1, int64_t ld, int64_t kpad, double *part,
                           hipStream_t s) {
    const int64_t nblk = ld / 256;
    hipLaunchKernelGGL(k_col_dots, dim3((unsigned)nblk, (unsigned)kpad), dim3(256), 0, s, A0, B0,
                       A1, B1, ld, kpad, nblk, part);
    return hipGetLastError();
}

hipError_t launch_pcg_scalars(const double *part, int64_t ld, int64_t kpad, int mode, int first,
                              double *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_scalars, dim3((unsigned)cdiv(kpad, 64)), dim3(64), 0, s, part,
                       ld / 256, kpad, mode, first, sc);
    return hipGetLastError();
}

hipError_t launch_pcg_dir(const double *Zt, double *Pt, const double *beta, int64_t ld,
                          int64_t kpad, int first, hipStream_t s) {
    const int64_t total = kpad * ld;
    const int grid = (int)(cdiv(total, 256) < 16384 ? cdiv(total, 256) : 16384);
    hipLaunchKernelGGL(k_pcg_dir, dim3(grid), dim3(256), 0, s, Zt, Pt, beta, ld, total, first);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int prec, const double *Pt, const double *Qt, const double *alpha,
                             const double *dm, int64_t ld, int64_t kpad, double *Xt, double *Rt,
                             double *V64, void *Vlo, double *npart, double *mpart, hipStream_t s) {
    dim3 grid((unsigned)(ld / 256), (unsigned)kpad), blk(256);
    switch (prec) {
    case 0: hipLaunchKernelGGL(k_pcg_update<double>, grid, blk, 0, s, Pt, Qt, alpha, dm, ld, kpad, Xt, Rt, V64, (double *)Vlo, npart, mpart); break;
    case 1: hipLaunchKernelGGL(k_pcg_update<float>, grid, blk, 0, s, Pt, Qt, alpha, dm, ld, kpad, Xt, Rt, V64, (float *)Vlo, npart, mpart); break;
    case 2: hipLaunchKernelGGL(k_pcg_update<__bf16>, grid, blk, 0, s, Pt, Qt, alpha, dm, ld, kpad, Xt, Rt, V64, (__bf16 *)Vlo, npart, mpart); break;
    default: hipLaunchKernelGGL(k_pcg_update<_Float16>, grid, blk, 0, s, Pt, Qt, alpha, dm, ld, kpad, Xt, Rt, V64, (_Float16 *)nullptr, npart, mpart); break;
    }
    return hipGetLastError();
}

} // namespace cdl
