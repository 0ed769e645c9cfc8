// Generic LDS-tiled MFMA core for C = A * B^T (both operands row-major along
// the reduction index k), used by every dense contraction of the path:
// kernel-distance Gram, chain squarings, chain application, FP64 residual
// and the score Gram.  Callers supply padded operands (K a multiple of BK,
// tile rows inside the allocation), so the core has no bounds checks.
#pragma once

#include "common.h"

namespace cdl {

template <class Mf, int BM, int BN, int BK, int WM, int WN>
struct GemmCore {
    using T = typename Mf::T;
    using Frag = typename Mf::Frag;
    using AccV = typename Mf::AccV;
    using MF = Mf;
    static constexpr int TBM = BM, TBN = BN;
    static constexpr int NT = WM * WN * 64;
    static constexpr int CE = 16 / (int)sizeof(T);     // elements per 16-byte chunk
    static constexpr int LDSK = BK + CE;                // padded LDS row (elements)
    static constexpr int CPR = BK / CE;                 // chunks per tile row
    static constexpr int A_CH = BM * CPR / NT;
    static constexpr int B_CH = BN * CPR / NT;
    static constexpr int WTM = BM / WM / Mf::M;
    static constexpr int WTN = BN / WN / Mf::M;
    static constexpr int STAGE = (BM + BN) * LDSK;      // elements per LDS stage
    static constexpr size_t SMEM = 2 * (size_t)STAGE * sizeof(T);
    static_assert(BM * CPR % NT == 0 && BN * CPR % NT == 0, "tile/thread mismatch");
    static_assert(WTM >= 1 && WTN >= 1, "wave tile too small");
    static_assert(BK % Mf::KI == 0 && BK % CE == 0, "bad BK");

    AccV acc[WTM][WTN];
    uint4 ra[A_CH], rb[B_CH];

    __device__ inline void zero() {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
#pragma unroll
                for (int r = 0; r < Mf::R; ++r) acc[i][j][r] = 0;
    }

    __device__ inline void load_global(const T *A, int64_t lda, const T *B, int64_t ldb,
                                       int64_t m0, int64_t n0, int64_t k0) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int c = 0; c < A_CH; ++c) {
            int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
            ra[c] = *(const uint4 *)(A + (m0 + row) * lda + k0 + kc * CE);
        }
#pragma unroll
        for (int c = 0; c < B_CH; ++c) {
            int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
            rb[c] = *(const uint4 *)(B + (n0 + row) * ldb + k0 + kc * CE);
        }
    }

    __device__ inline void store_lds(T *s) {
        const int tid = threadIdx.x;
        T *sA = s, *sB = s + BM * LDSK;
#pragma unroll
        for (int c = 0; c < A_CH; ++c) {
            int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
            *(uint4 *)(sA + row * LDSK + kc * CE) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < B_CH; ++c) {
            int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
            *(uint4 *)(sB + row * LDSK + kc * CE) = rb[c];
        }
    }

    __device__ inline void compute(const T *s) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int wm = wid % WM, wn = wid / WM;
        const T *sA = s + (wm * WTM * Mf::M) * LDSK;
        const T *sB = s + BM * LDSK + (wn * WTN * Mf::M) * LDSK;
        const int fr = lane % Mf::M, fk = Mf::E * (lane / Mf::M);
#pragma unroll
        for (int kk = 0; kk < BK; kk += Mf::KI) {
            Frag a[WTM], b[WTN];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
                a[i] = *(const Frag *)(sA + (i * Mf::M + fr) * LDSK + kk + fk);
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                b[j] = *(const Frag *)(sB + (j * Mf::M + fr) * LDSK + kk + fk);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j] = Mf::mma(a[i], b[j], acc[i][j]);
        }
    }

    // Full K loop with a two-stage LDS ring; K is a multiple of BK.
    __device__ inline void run(const T *A, int64_t lda, const T *B, int64_t ldb,
                               int64_t m0, int64_t n0, int64_t K, T *smem) {
        zero();
        const int nk = (int)(K / BK);
        if (nk == 0) return;
        load_global(A, lda, B, ldb, m0, n0, 0);
        store_lds(smem);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            T *cur = smem + (kt & 1) * STAGE;
            T *nxt = smem + ((kt + 1) & 1) * STAGE;
            if (kt + 1 < nk) load_global(A, lda, B, ldb, m0, n0, (int64_t)(kt + 1) * BK);
            compute(cur);
            if (kt + 1 < nk) store_lds(nxt);
            __syncthreads();
        }
    }

    // Tile-local coordinates of accumulator element (i, j, r) of this lane.
    __device__ static inline int row_of(int i, int r) {
        const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) % WM;
        return wm * WTM * Mf::M + i * Mf::M + Mf::crow(lane, r);
    }
    __device__ static inline int col_of(int j) {
        const int lane = threadIdx.x & 63, wn = (threadIdx.x >> 6) / WM;
        return wn * WTN * Mf::M + j * Mf::M + Mf::ccol(lane);
    }
};

// Stage the BM x BN tile of values f(row, col, acc) (tile-local row, col) of
// type O in LDS (row stride BN + 16/sizeof(O)), then copy it to global
// memory as rows C + (m0 + r) * ldc + n0 and, if `mirror`, as its transpose
// C + (n0 + c) * ldc + m0.  `sC` must hold BM * (BN + 16/sizeof(O)) elements
// and may alias the core's operand stages (a barrier separates the uses).
// Every thread of the workgroup must call this.
template <class Core, typename O, class F>
__device__ inline void stage_and_store(Core &g, O *sC, F f, O *C, int64_t ldc,
                                       int64_t m0, int64_t n0, bool mirror) {
    constexpr int BM = Core::TBM, BN = Core::TBN, NT = Core::NT;
    constexpr int CEo = 16 / (int)sizeof(O);
    constexpr int LDC = BN + CEo;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Core::WTM; ++i)
#pragma unroll
        for (int j = 0; j < Core::WTN; ++j)
#pragma unroll
            for (int r = 0; r < Core::MF::R; ++r) {
                int row = Core::row_of(i, r), col = Core::col_of(j);
                sC[row * LDC + col] = f(row, col, g.acc[i][j][r]);
            }
    __syncthreads();
    constexpr int CPR = BN / CEo;
    for (int ch = threadIdx.x; ch < BM * CPR; ch += NT) {
        int r = ch / CPR, c = ch % CPR;
        *(uint4 *)(C + (m0 + r) * ldc + n0 + c * CEo) = *(const uint4 *)(sC + r * LDC + c * CEo);
    }
    if (mirror) {
        constexpr int QPR = BM / CEo;
        for (int ch = threadIdx.x; ch < BN * QPR; ch += NT) {
            int c = ch % BN, q = ch / BN;
            union { uint4 v; O e[CEo]; } u;
#pragma unroll
            for (int e = 0; e < CEo; ++e) u.e[e] = sC[(q * CEo + e) * LDC + c];
            *(uint4 *)(C + (n0 + c) * ldc + m0 + q * CEo) = u.v;
        }
    }
}

// As stage_and_store, staging RC rows of the tile at a time so that the
// staging buffer (RC * (BN + 16/sizeof(O)) elements) stays small.
template <int RC, class Core, typename O, class F>
__device__ inline void stage_and_store_rows(Core &g, O *sC, F f, O *C, int64_t ldc, int64_t m0,
                                            int64_t n0, bool mirror) {
    constexpr int BM = Core::TBM, BN = Core::TBN, NT = Core::NT;
    constexpr int CEo = 16 / (int)sizeof(O);
    constexpr int LDC = BN + CEo;
    static_assert(BM % RC == 0 && RC % CEo == 0, "bad row chunk");
#pragma unroll 1
    for (int r0 = 0; r0 < BM; r0 += RC) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Core::WTM; ++i)
#pragma unroll
            for (int j = 0; j < Core::WTN; ++j)
#pragma unroll
                for (int r = 0; r < Core::MF::R; ++r) {
                    const int row = Core::row_of(i, r), col = Core::col_of(j);
                    if (row >= r0 && row < r0 + RC) sC[(row - r0) * LDC + col] = f(row, col, g.acc[i][j][r]);
                }
        __syncthreads();
        constexpr int CPR = BN / CEo;
        for (int ch = threadIdx.x; ch < RC * CPR; ch += NT) {
            const int r = ch / CPR, c = ch % CPR;
            *(uint4 *)(C + (m0 + r0 + r) * ldc + n0 + c * CEo) = *(const uint4 *)(sC + r * LDC + c * CEo);
        }
        if (mirror) {
            constexpr int QPR = RC / CEo;
            for (int ch = threadIdx.x; ch < BN * QPR; ch += NT) {
                const int c = ch % BN, q = ch / BN;
                union { uint4 v; O e[CEo]; } u;
#pragma unroll
                for (int e = 0; e < CEo; ++e) u.e[e] = sC[(q * CEo + e) * LDC + c];
                *(uint4 *)(C + (n0 + c) * ldc + m0 + r0 + q * CEo) = u.v;
            }
        }
    }
}

} // namespace cdl
