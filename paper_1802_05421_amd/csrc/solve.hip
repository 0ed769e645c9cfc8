// Embedding solve (Algorithm 3 with Algorithm 1's right-hand sides; the
// refinement is EstimateSolution of Algorithm 2 with P2 y = P1 L y, batched
// over the k columns).
//
//   rhs         Y = B^T W^{1/2} Q^T / sqrt(k) with counter-based SplitMix64
//               signs, one row of Y per wave (lane = neighbour j), FP64
//               accumulation of EXEC-masked adds, deterministic butterfly
//               reduction; rhs_pair does the same for two snapshots on one
//               node set, each sign word and lane mask serving both
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

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014), split after
// its first step z ^ (z >> 30): that step is linear over GF(2), so it can be
// applied to the parts of a key separately and the results XORed.
__device__ inline uint64_t xorshift30(uint64_t z) { return z ^ (z >> 30); }
__device__ inline uint64_t splitmix64_mix_tail(uint64_t z) {
    z = z * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static uint64_t splitmix64_mix_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// acc_q += w on the lanes whose next bit of h (most significant first) is
// set, for eight bits; h is shifted left by eight.  Doubling h moves its top
// bit into the carry mask of that lane; the FP64 add then runs with EXEC
// restricted to the carry mask: two VALU instructions per column instead of
// the three a per-lane sign insertion needs.  EXEC is saved and restored
// inside the block, so inactive lanes (loop tails) stay inactive.
__device__ __forceinline__ void masked_add8(uint32_t &h, double w, double &a0, double &a1,
                                            double &a2, double &a3, double &a4, double &a5,
                                            double &a6, double &a7) {
    uint64_t sv, m0, m1, m2, m3, m4, m5, m6, m7;
    asm volatile(
        "s_mov_b64 %[sv], exec\n\t"
        "v_add_co_u32 %[h], %[m0], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m1], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m2], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m3], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m4], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m5], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m6], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m7], %[h], %[h]\n\t"
        "s_and_b64 exec, %[sv], %[m0]\n\t"
        "v_add_f64 %[a0], %[a0], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m1]\n\t"
        "v_add_f64 %[a1], %[a1], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m2]\n\t"
        "v_add_f64 %[a2], %[a2], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m3]\n\t"
        "v_add_f64 %[a3], %[a3], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m4]\n\t"
        "v_add_f64 %[a4], %[a4], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m5]\n\t"
        "v_add_f64 %[a5], %[a5], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m6]\n\t"
        "v_add_f64 %[a6], %[a6], %[w]\n\t"
        "s_and_b64 exec, %[sv], %[m7]\n\t"
        "v_add_f64 %[a7], %[a7], %[w]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [h] "+v"(h), [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3),
          [a4] "+v"(a4), [a5] "+v"(a5), [a6] "+v"(a6), [a7] "+v"(a7), [sv] "=&s"(sv),
          [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2), [m3] "=&s"(m3), [m4] "=&s"(m4),
          [m5] "=&s"(m5), [m6] "=&s"(m6), [m7] "=&s"(m7)
        : [w] "v"(w)
        : "scc");
}

// Row i of Y for one projection block beta (64 columns).  The sign of edge
// {i, j} in column r is B(e, i) * q_r(e) = c (1 - 2 b), b = bit r of the sign
// word, c = 1 when i is the head (lower global id) and -1 when it is the
// tail.  So sum_j s_j w_j = T - 2 M_r with v_j = c_j w_j, T = sum_j v_j and
// M_r the sum of v_j over the j whose bit is set, all in FP64; the sums'
// rounding errors stay below 1e-15 sum_j w_j, far below |y| here.
//
// A workgroup is 4 waves: 4/P rows, P projection blocks per row.  The P
// waves of a row share sqrt(W_ij) and the global ids through LDS: per
// iteration each computes them for its own 64 neighbours, then all P waves
// sweep the P * 64 neighbours with their own sign words.
//
// Rows [row0, row1): row i is read at W + (i - row0) ld (the whole matrix with
// row0 = 0, row1 = n, or one row panel of it).
template <int P>
__global__ __launch_bounds__(256) void k_rhs(const double *W, int64_t ld, int64_t n,
                                             int64_t row0, int64_t row1,
                                             const int32_t *gid, int64_t k, uint64_t mseed,
                                             double inv_sqrt_k, int nb, double *Yt) {
    constexpr int R = 4 / P;
    __shared__ double sw[R][P * 64];   // c_j sqrt(W_ij)
    __shared__ uint2 sz[R][P * 64];    // xorshift30 of the key of {i, j} (beta = 0) XOR the mixed seed
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int rs = wv / P, q = wv % P;
    // Workgroups are dispatched round-robin over the XCDs: the projection
    // groups of one row group get ids 8 apart, so they run together on one
    // XCD and read those rows of W through its L2 once.
    const int nbg = (nb + P - 1) / P;
    const int w = blockIdx.x, per = kNumXcd * nbg, l = w % per;
    const int64_t group = (int64_t)(w / per) * kNumXcd + l % kNumXcd;
    const int beta_i = (l / kNumXcd) * P + q;
    const uint64_t beta = (uint64_t)beta_i;
    const int64_t i = row0 + group * R + rs;
    const bool row_ok = i < row1, active = row_ok && beta_i < nb;
    const uint32_t gi = !row_ok ? 0u : (gid ? (uint32_t)gid[i] : (uint32_t)i);
    // The key beta << 40 | lo << 20 | hi of a pair (ids < 2^20) XOR the mixed
    // seed in 32-bit halves: low = lo << 20 | hi, high = beta << 8 | lo >> 12
    // (disjoint bits, so the ORs are XORs and beta enters last).
    const uint32_t seed_lo = (uint32_t)mseed, seed_hi = (uint32_t)(mseed >> 32);
    const uint64_t fbeta = xorshift30((uint64_t)((uint32_t)beta_i << 8) << 32);
    double acc[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) acc[r] = 0.0;
    double tsum = 0.0;
    const double *row = W + (row_ok ? i - row0 : 0) * ld;
    for (int64_t j0 = 0; j0 < n; j0 += P * 64) {
        {   // per neighbour, once for the P projection blocks: the correctly
            // rounded sqrt(W) (the bare hardware instruction is only an
            // approximation in FP64), negated when row i is the edge's tail
            // (gi > gj: every sign flips, so T and M both take -w), and the
            // key halves; zero beyond n (no contribution whatever the sign)
            const int64_t j = j0 + q * 64 + lane;
            double v = 0.0;
            uint2 z = make_uint2(0u, 0u);
            if (row_ok && j < n) {
                const uint32_t gj = gid ? (uint32_t)gid[j] : (uint32_t)j;
                const double wj = sqrt(row[j]);
                const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
                const uint64_t f = xorshift30(((uint64_t)((lo >> 12) ^ seed_hi) << 32) |
                                              (((lo << 20) | hi) ^ seed_lo));
                z = make_uint2((uint32_t)f, (uint32_t)(f >> 32));
                v = gi > gj ? -wj : wj;
            }
            sw[rs][q * 64 + lane] = v;
            sz[rs][q * 64 + lane] = z;
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int sub = 0; sub < P; ++sub) {
                const double ws = sw[rs][sub * 64 + lane];
                const uint2 z = sz[rs][sub * 64 + lane];
                const uint64_t h = splitmix64_mix_tail((((uint64_t)z.y << 32) | z.x) ^ fbeta);
                tsum += ws;
                uint32_t hh = (uint32_t)(h >> 32), hl = (uint32_t)h;
                masked_add8(hh, ws, acc[63], acc[62], acc[61], acc[60], acc[59], acc[58], acc[57], acc[56]);
                masked_add8(hh, ws, acc[55], acc[54], acc[53], acc[52], acc[51], acc[50], acc[49], acc[48]);
                masked_add8(hh, ws, acc[47], acc[46], acc[45], acc[44], acc[43], acc[42], acc[41], acc[40]);
                masked_add8(hh, ws, acc[39], acc[38], acc[37], acc[36], acc[35], acc[34], acc[33], acc[32]);
                masked_add8(hl, ws, acc[31], acc[30], acc[29], acc[28], acc[27], acc[26], acc[25], acc[24]);
                masked_add8(hl, ws, acc[23], acc[22], acc[21], acc[20], acc[19], acc[18], acc[17], acc[16]);
                masked_add8(hl, ws, acc[15], acc[14], acc[13], acc[12], acc[11], acc[10], acc[9], acc[8]);
                masked_add8(hl, ws, acc[7], acc[6], acc[5], acc[4], acc[3], acc[2], acc[1], acc[0]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tsum += __shfl_xor(tsum, o);
    // Butterfly transpose-reduction: afterwards lane l holds column l summed
    // over all 64 lanes.
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const bool up = (lane & s) != 0;
#pragma unroll
        for (int q2 = 0; q2 < s; ++q2) {
            const double send = up ? acc[q2] : acc[q2 + s];
            const double keep = up ? acc[q2 + s] : acc[q2];
            acc[q2] = keep + __shfl_xor(send, s);
        }
    }
    const int64_t r = (int64_t)beta * 64 + lane;
    Yt[r * ld + i] = r < k ? (tsum - 2.0 * acc[0]) * inv_sqrt_k : 0.0;
}

// masked_add8 for two sums with the same signs: one lane mask per column
// serves acc_a (+= wa) and acc_b (+= wb).
__device__ __forceinline__ void masked_add8x2(uint32_t &h, double wa, double wb, double &a0,
                                              double &a1, double &a2, double &a3, double &a4,
                                              double &a5, double &a6, double &a7, double &b0,
                                              double &b1, double &b2, double &b3, double &b4,
                                              double &b5, double &b6, double &b7) {
    uint64_t sv, m0, m1, m2, m3, m4, m5, m6, m7;
    asm volatile(
        "s_mov_b64 %[sv], exec\n\t"
        "v_add_co_u32 %[h], %[m0], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m1], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m2], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m3], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m4], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m5], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m6], %[h], %[h]\n\t"
        "v_add_co_u32 %[h], %[m7], %[h], %[h]\n\t"
        "s_and_b64 exec, %[sv], %[m0]\n\t"
        "v_add_f64 %[a0], %[a0], %[wa]\n\t"
        "v_add_f64 %[b0], %[b0], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m1]\n\t"
        "v_add_f64 %[a1], %[a1], %[wa]\n\t"
        "v_add_f64 %[b1], %[b1], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m2]\n\t"
        "v_add_f64 %[a2], %[a2], %[wa]\n\t"
        "v_add_f64 %[b2], %[b2], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m3]\n\t"
        "v_add_f64 %[a3], %[a3], %[wa]\n\t"
        "v_add_f64 %[b3], %[b3], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m4]\n\t"
        "v_add_f64 %[a4], %[a4], %[wa]\n\t"
        "v_add_f64 %[b4], %[b4], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m5]\n\t"
        "v_add_f64 %[a5], %[a5], %[wa]\n\t"
        "v_add_f64 %[b5], %[b5], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m6]\n\t"
        "v_add_f64 %[a6], %[a6], %[wa]\n\t"
        "v_add_f64 %[b6], %[b6], %[wb]\n\t"
        "s_and_b64 exec, %[sv], %[m7]\n\t"
        "v_add_f64 %[a7], %[a7], %[wa]\n\t"
        "v_add_f64 %[b7], %[b7], %[wb]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [h] "+v"(h), [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3),
          [a4] "+v"(a4), [a5] "+v"(a5), [a6] "+v"(a6), [a7] "+v"(a7), [b0] "+v"(b0),
          [b1] "+v"(b1), [b2] "+v"(b2), [b3] "+v"(b3), [b4] "+v"(b4), [b5] "+v"(b5),
          [b6] "+v"(b6), [b7] "+v"(b7), [sv] "=&s"(sv), [m0] "=&s"(m0), [m1] "=&s"(m1),
          [m2] "=&s"(m2), [m3] "=&s"(m3), [m4] "=&s"(m4), [m5] "=&s"(m5), [m6] "=&s"(m6),
          [m7] "=&s"(m7)
        : [wa] "v"(wa), [wb] "v"(wb)
        : "scc");
}

// Rows of Y for two snapshots on one node set (the same global ids, so the
// same sign words on every edge): Y0 from W0 and Y1 from W1 in one sweep,
// each word and each lane mask serving both.  A workgroup is one row and 16
// waves: projection block beta = 4 g + wave / 4 (g the block group), the
// wave's quarter of it the 16 columns [64 beta + 16 c, 64 beta + 16 c + 16),
// so that 32 accumulators per lane leave room for four waves per SIMD.
// Neighbours come in chunks of 512; every thread stages two sign words and
// one signed square root of the chunk (the stage is the same work for every
// wave, so the one barrier per chunk finds them together), into one of two
// LDS buffers, and issues the next chunk's loads before summing this one.
__global__ __launch_bounds__(1024) void k_rhs_pair(const double *W0, const double *W1, int64_t ld,
                                                   int64_t n, const int32_t *gid, int64_t k,
                                                   uint64_t mseed, double inv_sqrt_k, int nb,
                                                   double *Y0t, double *Y1t) {
    constexpr int C = 512;
    __shared__ uint64_t sh[2][4][C];
    __shared__ double sw[2][2][C];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int bq = wv >> 2, quarter = wv & 3;
    const int nbg = (nb + 3) / 4;
    const int w = blockIdx.x, per = kNumXcd * nbg, l = w % per;
    const int64_t i = (int64_t)(w / per) * kNumXcd + l % kNumXcd;
    const int bgrp = l / kNumXcd;
    const bool row_ok = i < n, active = row_ok && bgrp * 4 + bq < nb;
    const uint32_t gi = !row_ok ? 0u : (gid ? (uint32_t)gid[i] : (uint32_t)i);
    // stage roles: neighbour jj = t % C; the words of blocks 4 g + 2 s and
    // 4 g + 2 s + 1, and the root of snapshot s, s = t / C
    const int jj = t & (C - 1), sr = t / C;
    const uint64_t kb0 = (uint64_t)(bgrp * 4 + 2 * sr) << 40, kb1 = kb0 + (1ull << 40);
    const double *wrow = (sr == 0 ? W0 : W1) + (row_ok ? i : 0) * ld;
    double acc0[16], acc1[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc0[q] = acc1[q] = 0.0;
    double t0 = 0.0, t1 = 0.0;
    auto load = [&](int64_t j0, uint32_t &g, double &v) {
        const int64_t j = j0 + jj;
        g = 0u;
        v = 0.0;
        if (row_ok && j < n) {
            g = gid ? (uint32_t)gid[j] : (uint32_t)j;
            v = wrow[j];
        }
    };
    auto word = [&](uint64_t key) -> uint64_t {
        uint64_t z = mseed ^ key;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    uint32_t gj;
    double wv0;
    load(0, gj, wv0);
    int buf = 0;
    for (int64_t j0 = 0; j0 < n; j0 += C, buf ^= 1) {
        {   // stage this chunk: zero beyond n (no contribution whatever the sign)
            const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
            const uint64_t key = ((uint64_t)lo << 20) | (uint64_t)hi;
            sh[buf][2 * sr][jj] = word(kb0 | key);
            sh[buf][2 * sr + 1][jj] = word(kb1 | key);
            const double r = sqrt(wv0);   // correctly rounded
            sw[buf][sr][jj] = gi > gj ? -r : r;
        }
        load(j0 + C, gj, wv0);   // in flight while this chunk is summed
        __syncthreads();
        if (active) {
#pragma unroll 2
            for (int sub = 0; sub < C / 64; ++sub) {
                const int q = sub * 64 + lane;
                const uint64_t hw = sh[buf][bq][q];
                const double a = sw[buf][0][q], b = sw[buf][1][q];
                // the quarter's 16 bits, most significant first
                uint32_t h = (uint32_t)(hw >> (16 * quarter)) << 16;
                t0 += a;
                t1 += b;
                masked_add8x2(h, a, b, acc0[15], acc0[14], acc0[13], acc0[12], acc0[11], acc0[10],
                              acc0[9], acc0[8], acc1[15], acc1[14], acc1[13], acc1[12], acc1[11],
                              acc1[10], acc1[9], acc1[8]);
                masked_add8x2(h, a, b, acc0[7], acc0[6], acc0[5], acc0[4], acc0[3], acc0[2],
                              acc0[1], acc0[0], acc1[7], acc1[6], acc1[5], acc1[4], acc1[3],
                              acc1[2], acc1[1], acc1[0]);
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        t0 += __shfl_xor(t0, o);
        t1 += __shfl_xor(t1, o);
    }
    // Butterfly transpose-reduction over each 16-lane group, then across the
    // groups: lane l ends with column l % 16 summed over all 64 lanes.
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) {
        const bool up = (lane & s) != 0;
#pragma unroll
        for (int q2 = 0; q2 < s; ++q2) {
            const double s0 = up ? acc0[q2] : acc0[q2 + s], k0 = up ? acc0[q2 + s] : acc0[q2];
            const double s1 = up ? acc1[q2] : acc1[q2 + s], k1 = up ? acc1[q2 + s] : acc1[q2];
            acc0[q2] = k0 + __shfl_xor(s0, s);
            acc1[q2] = k1 + __shfl_xor(s1, s);
        }
    }
    acc0[0] += __shfl_xor(acc0[0], 16);
    acc1[0] += __shfl_xor(acc1[0], 16);
    acc0[0] += __shfl_xor(acc0[0], 32);
    acc1[0] += __shfl_xor(acc1[0], 32);
    if (lane < 16) {
        const int64_t r = (int64_t)(bgrp * 4 + bq) * 64 + quarter * 16 + lane;
        Y0t[r * ld + i] = r < k ? (t0 - 2.0 * acc0[0]) * inv_sqrt_k : 0.0;
        Y1t[r * ld + i] = r < k ? (t1 - 2.0 * acc1[0]) * inv_sqrt_k : 0.0;
    }
}

hipError_t launch_rhs_pair(const double *W0, const double *W1, int64_t ld, int64_t n,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Y0t, double *Y1t, hipStream_t s) {
    const uint64_t mseed = splitmix64_mix_host(seed);
    const int nb = (int)(kpad / 64);
    const int nbg = (nb + 3) / 4;
    const int64_t rows = cdiv(n, kNumXcd) * kNumXcd;
    hipLaunchKernelGGL(k_rhs_pair, dim3((unsigned)(rows * nbg)), dim3(1024), 0, s, W0, W1, ld, n,
                       gid, k, mseed, 1.0 / sqrt((double)k), nb, Y0t, Y1t);
    return hipGetLastError();
}

hipError_t launch_rhs_rows(const double *W, int64_t ld, int64_t n, int64_t row0, int64_t row1,
                           const int32_t *gid, int64_t k, int64_t kpad, uint64_t seed,
                           double *Yt, hipStream_t s) {
    if (row0 < 0 || row1 > n) return hipErrorInvalidValue;
    if (row1 <= row0) return hipSuccess;
    const uint64_t mseed = splitmix64_mix_host(seed);
    const int nb = (int)(kpad / 64);
    const int P = nb >= 4 ? 4 : (nb >= 2 ? 2 : 1);
    const int nbg = (nb + P - 1) / P;
    const int64_t groups = cdiv(cdiv(row1 - row0, 4 / P), kNumXcd) * kNumXcd;
    const dim3 grid((unsigned)(groups * nbg)), blk(256);
    const double isk = 1.0 / sqrt((double)k);
    switch (P) {
    case 4: hipLaunchKernelGGL(k_rhs<4>, grid, blk, 0, s, W, ld, n, row0, row1, gid, k, mseed, isk, nb, Yt); break;
    case 2: hipLaunchKernelGGL(k_rhs<2>, grid, blk, 0, s, W, ld, n, row0, row1, gid, k, mseed, isk, nb, Yt); break;
    default: hipLaunchKernelGGL(k_rhs<1>, grid, blk, 0, s, W, ld, n, row0, row1, gid, k, mseed, isk, nb, Yt); break;
    }
    return hipGetLastError();
}

hipError_t launch_rhs(const double *W, int64_t ld, int64_t n, const int32_t *gid, int64_t k,
                      int64_t kpad, uint64_t seed, double *Yt, hipStream_t s) {
    return launch_rhs_rows(W, ld, n, 0, n, gid, k, kpad, seed, Yt, s);
}

// ---------------------------------------------------------------------------
// FP64 residual R = Y - deg * X + W X, as a split-K MFMA GEMM
// P[s][r][i] = sum_{j in split s} Xt[r][j] W[i][j] followed by a reduction
// that forms R, the next preconditioner operand and the column-norm partials.

template <int BM> struct ResCfg {
    static constexpr int WM = BM / 64, WN = 8 / (BM / 64);
    using Core = GemmCore<MfmaF64, BM, 128, 16, WM, WN>;
};

// W may be a row panel: its row q holds node row0 + q, whose products land in
// column row0 + q of the partials (row0 = 0 for the whole matrix).
template <int BM>
__device__ __forceinline__ void residual_gemm_tile(const double *Xt, const double *W, int64_t ld,
                                          int64_t kend, int64_t ks, int mt, int nt, double *P,
                                          int64_t kpad, int64_t row0, int id, char *smem_raw) {
    using Core = typename ResCfg<BM>::Core;
    double *smem = (double *)smem_raw;
    // split-major order: the WGs of one split stream the same K range
    const int split = id / (mt * nt);
    int I, J;
    rect_tile<4>(id % (mt * nt), mt, nt, I, J);
    const int64_t m0 = (int64_t)I * BM, n0 = (int64_t)J * 128;
    const int64_t k0 = (int64_t)split * ks;
    const int64_t kk = k0 < kend ? (kend - k0 < ks ? kend - k0 : ks) : 0;
    Core g;
    g.run(Xt + k0, ld, W + k0, ld, m0, n0, kk, smem);
    double *Ps = P + (int64_t)split * kpad * ld + row0;
#pragma unroll
    for (int a = 0; a < Core::WTM; ++a)
#pragma unroll
        for (int b = 0; b < Core::WTN; ++b)
#pragma unroll
            for (int rr = 0; rr < MfmaF64::R; ++rr)
                Ps[(m0 + Core::row_of(a, rr)) * ld + n0 + Core::col_of(b)] = g.acc[a][b][rr];
}

template <int BM>
__global__ __launch_bounds__(512) void k_residual_gemm(const double *Xt, const double *W,
                                                       int64_t ld, int64_t kend, int64_t ks,
                                                       int mt, int nt, int S, double *P,
                                                       int64_t kpad, int64_t row0) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const int id = xcd_remap(blockIdx.x, mt * nt * S);
    residual_gemm_tile<BM>(Xt, W, ld, kend, ks, mt, nt, P, kpad, row0, id, smem_raw);
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
    using Core = typename ResCfg<BM>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_residual_gemm<BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(ld / 128);
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t ks = (cdiv(kend, S) + 15) / 16 * 16;
    hipLaunchKernelGGL(k_residual_gemm<BM>, dim3(mt * nt * S), dim3(512), Core::SMEM, s, Xt, W,
                       ld, kend, ks, mt, nt, S, P, kpad, (int64_t)0);
    return hipGetLastError();
}

template <int BM>
static hipError_t panel_launch(const double *Vt, const double *Wp, int64_t ld, int64_t n,
                               int64_t kpad, int64_t row0, int64_t rows, double *Prod,
                               hipStream_t s) {
    using Core = typename ResCfg<BM>::Core;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_residual_gemm<BM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Core::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int mt = (int)(kpad / BM), nt = (int)(rows / 128);
    const int64_t kend = (n + 63) / 64 * 64;
    const int64_t ks = (kend + 15) / 16 * 16;
    hipLaunchKernelGGL(k_residual_gemm<BM>, dim3(mt * nt), dim3(512), Core::SMEM, s, Vt, Wp, ld,
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
    residual_gemm_tile<BM>(d.Xt, d.W, d.ld, (d.n + 63) / 64 * 64, residual_split_len(d.n, d.res_splits),
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
    using Core = typename ResCfg<BM>::Core;
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

// Z[i][r] = Xt[r][i] - mean[r] through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_transpose_z(const double *Xt, int64_t ld, int64_t n,
                                                     int64_t k, const double *mean, double *Z) {
    __shared__ double t[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, i = i0 + tx;
        t[q][tx] = (r < k && i < n) ? Xt[r * ld + i] - mean[r] : 0.0;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t i = i0 + q, r = r0 + tx;
        if (i < n && r < k) Z[i * k + r] = t[tx][q];
    }
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
