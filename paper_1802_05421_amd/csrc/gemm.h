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

// ---------------------------------------------------------------------------
// 16-bit operand core fed by direct global->LDS loads (gfx950
// global_load_lds_dwordx4): each wave instruction moves 64 x 16 bytes into
// 1 KB of LDS at M0 + 16 * lane, so operands never pass through VGPRs.  LDS
// rows are BK = 64 elements (128 B) with the 16-byte chunks XOR-swizzled by
// (row >> 1) & 7, which keeps the 16 lanes that an ds_read_b128 serves per
// cycle on distinct banks for the 32-row MFMA fragments.  Two stages: the
// loads of k-tile t+1 are issued before the MFMAs of tile t; the fragments
// of the next 16-wide k-step are read while the current ones are consumed.
// The loads are issued from inline assembly because the compiler cannot tell
// the target stage from the one being read and would otherwise wait for
// every outstanding load before each LDS read.

typedef __attribute__((address_space(3))) char lds_char;

__device__ inline uint32_t lds_offset(const void *p) {
    return (uint32_t)(uintptr_t)(const lds_char *)p;
}

// 16 bytes per lane from src into LDS at m0base + 16 * lane.  M0 is set in
// the same statement (one wait state before the load, as the ISA requires).
__device__ inline void lds_dma16(const void *src, uint32_t m0base) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(__builtin_amdgcn_readfirstlane(m0base))
                 : "memory", "m0");
}

__device__ inline void wait_vmem_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <class Mf, int BM, int BN, int WM, int WN>
struct DmaCore {
    using T = typename Mf::T;
    using Frag = typename Mf::Frag;
    using AccV = typename Mf::AccV;
    using MF = Mf;
    static_assert(sizeof(T) == 2, "16-bit operands");
    static constexpr int BK = 64;
    static constexpr int TBM = BM, TBN = BN;
    static constexpr int NW = WM * WN, NT = NW * 64;
    static constexpr int CE = 8;                  // elements per 16-byte chunk
    static constexpr int CPR = BK / CE;           // 8 chunks per LDS row
    static constexpr int RPI = 64 / CPR;          // rows per wave instruction
    static constexpr int ROWB = BK * 2;           // bytes per LDS row
    static constexpr int STAGE = (BM + BN) * ROWB;
    static constexpr size_t SMEM = 2 * (size_t)STAGE;
    static constexpr int WTM = BM / WM / Mf::M, WTN = BN / WN / Mf::M;
    static constexpr int AI = BM / RPI / NW, BI = BN / RPI / NW;
    static constexpr int NKK = BK / Mf::KI;
    static_assert(AI * RPI * NW == BM && BI * RPI * NW == BN, "rows per wave");

    AccV acc[WTM][WTN];

    __device__ static inline int swz(int c, int row) { return c ^ ((row >> 1) & 7); }

    __device__ inline void issue(uint32_t stage, const T *A, int64_t lda, const T *B, int64_t ldb,
                                 int64_t m0, int64_t n0, int64_t k0) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int rl = lane / CPR, sl = lane % CPR;
#pragma unroll
        for (int q = 0; q < AI; ++q) {
            const int row0 = (w * AI + q) * RPI, row = row0 + rl;
            lds_dma16(A + (m0 + row) * lda + k0 + swz(sl, row) * CE, stage + row0 * ROWB);
        }
#pragma unroll
        for (int q = 0; q < BI; ++q) {
            const int row0 = (w * BI + q) * RPI, row = row0 + rl;
            lds_dma16(B + (n0 + row) * ldb + k0 + swz(sl, row) * CE, stage + (BM + row0) * ROWB);
        }
    }

    __device__ inline void load_frags(const char *sA, const char *sB, int kk, Frag *a, Frag *b) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int wm = wid % WM, wn = wid / WM;
        const int ch = (kk + Mf::E * (lane / Mf::M)) / CE;
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
            const int row = wm * WTM * Mf::M + i * Mf::M + lane % Mf::M;
            a[i] = *(const Frag *)(sA + row * ROWB + 16 * swz(ch, row));
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int row = wn * WTN * Mf::M + j * Mf::M + lane % Mf::M;
            b[j] = *(const Frag *)(sB + row * ROWB + 16 * swz(ch, row));
        }
    }

    __device__ inline void compute(const char *s) {
        const char *sA = s, *sB = s + BM * ROWB;
        Frag a[2][WTM], b[2][WTN];
        load_frags(sA, sB, 0, a[0], b[0]);
#pragma unroll
        for (int q = 0; q < NKK; ++q) {
            if (q + 1 < NKK) load_frags(sA, sB, (q + 1) * Mf::KI, a[(q + 1) & 1], b[(q + 1) & 1]);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    acc[i][j] = Mf::mma(a[q & 1][i], b[q & 1][j], acc[i][j]);
        }
    }

    // Full K loop (K a multiple of 64; rows m0.. and n0.. inside the
    // allocations).  smem holds SMEM bytes.
    __device__ inline void run(const T *A, int64_t lda, const T *B, int64_t ldb, int64_t m0,
                               int64_t n0, int64_t K, void *smem_v) {
        char *smem = (char *)smem_v;
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
#pragma unroll
                for (int r = 0; r < Mf::R; ++r) acc[i][j][r] = 0;
        const int nk = (int)(K / BK);
        if (nk == 0) return;
        const uint32_t s0 = lds_offset(smem);
        issue(s0, A, lda, B, ldb, m0, n0, 0);
        wait_vmem_all();
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk)
                issue(s0 + ((kt + 1) & 1) * STAGE, A, lda, B, ldb, m0, n0, (int64_t)(kt + 1) * BK);
            compute(smem + (kt & 1) * STAGE);
            wait_vmem_all();
            __syncthreads();
        }
    }

    __device__ static inline int row_of(int i, int r) {
        const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) % WM;
        return wm * WTM * Mf::M + i * Mf::M + Mf::crow(lane, r);
    }
    __device__ static inline int col_of(int j) {
        const int lane = threadIdx.x & 63, wn = (threadIdx.x >> 6) / WM;
        return wn * WTN * Mf::M + j * Mf::M + Mf::ccol(lane);
    }
};

} // namespace cdl
