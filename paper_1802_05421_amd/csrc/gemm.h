// Generic LDS-tiled MFMA core for C = A * B^T (A row-major along the
// reduction index k; B row-major along k, or with BT = true row-major along
// n, i.e. element (n, k) at B[k * ldb + n]), used by every dense contraction
// of the path: kernel-distance Gram, chain squarings, chain application,
// FP64 residual and the score Gram.  BT reads a k-tile of B as BK rows of BN
// contiguous elements (1 KB segments for 128 doubles) instead of BN rows of
// BK; for a symmetric B both forms multiply the same values in the same
// order.  Callers supply padded operands (K a multiple of BK, tile rows
// inside the allocation), so the core has no bounds checks.
#pragma once

#include "common.h"

namespace cdl {

template <class Mf, int BM, int BN, int BK, int WM, int WN, bool BT = false>
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
    // BT: B's k-tile as BK rows of BN (+ pad: consecutive k rows start 32
    // banks apart, so the two k rows that one half-wave of a fragment read
    // takes, 16 consecutive doubles each, cover the 64 banks once)
    static constexpr int LDSN = BN + 16;
    static constexpr int CPN = BN / CE;                 // chunks per B^T tile row
    static constexpr int STAGE = BM * LDSK + (BT ? BK * LDSN : BN * LDSK);   // elements per stage
    static constexpr size_t SMEM = 2 * (size_t)STAGE * sizeof(T);
    static_assert(BM * CPR % NT == 0 && BN * CPR % NT == 0, "tile/thread mismatch");
    static_assert(!BT || (Mf::E == 1 && BN % CE == 0), "B^T tiles need one k per fragment");
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
            if (BT) {
                int ch = tid + c * NT, row = ch / CPN, nc = ch % CPN;
                rb[c] = *(const uint4 *)(B + (k0 + row) * ldb + n0 + nc * CE);
            } else {
                int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
                rb[c] = *(const uint4 *)(B + (n0 + row) * ldb + k0 + kc * CE);
            }
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
            if (BT) {
                int ch = tid + c * NT, row = ch / CPN, nc = ch % CPN;
                *(uint4 *)(sB + row * LDSN + nc * CE) = rb[c];
            } else {
                int ch = tid + c * NT, row = ch / CPR, kc = ch % CPR;
                *(uint4 *)(sB + row * LDSK + kc * CE) = rb[c];
            }
        }
    }

    __device__ inline void compute(const T *s) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int wm = wid % WM, wn = wid / WM;
        const T *sA = s + (wm * WTM * Mf::M) * LDSK;
        const T *sB = s + BM * LDSK + (wn * WTN * Mf::M) * (BT ? 1 : LDSK);
        const int fr = lane % Mf::M, fk = Mf::E * (lane / Mf::M);
#pragma unroll
        for (int kk = 0; kk < BK; kk += Mf::KI) {
            Frag a[WTM], b[WTN];
#pragma unroll
            for (int i = 0; i < WTM; ++i)
                a[i] = *(const Frag *)(sA + (i * Mf::M + fr) * LDSK + kk + fk);
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                b[j] = BT ? *(const Frag *)(sB + (kk + fk) * LDSN + j * Mf::M + fr)
                          : *(const Frag *)(sB + (j * Mf::M + fr) * LDSK + kk + fk);
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
// buffer_load_dwordx4 ... lds): each wave instruction moves 64 x 16 bytes
// into 1 KB of LDS, so operands never pass through VGPRs.  The two operand
// panels are addressed through buffer resources (base = first row of the
// panel, in SGPRs); per instruction the wave-uniform part of the offset (row
// block, k-slice) is a scalar offset and the per-lane part one of two VGPR
// offsets, so the loads need no 64-bit address arithmetic.  LDS rows are
// BK = 64 elements (128 B) with the 16-byte chunks XOR-swizzled by
// (row >> 1) & 7, which keeps the 16 lanes that an ds_read_b128 serves per
// cycle on distinct banks for the 32-row MFMA fragments.
//
// Pipeline (two LDS stages): the fragments of k-step q + 1 are read while
// the MFMAs of k-step q run (sched_group_barrier interleaves one LDS read
// with the MFMAs that fit beside it); before the last k-step of a stage
// every wave waits for the next stage's loads and meets the others at a
// barrier, then reads the next stage's first fragments beside the last
// k-step's MFMAs and issues the loads of the stage after next into the buffer
// just released.  The loop body is uniform; the last stage is peeled.

typedef __attribute__((address_space(3))) void lds_void;

template <int N> __device__ inline void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier without a memory fence (the loads into LDS are waited
// for explicitly); the empty asm statements keep the compiler from moving
// memory accesses across it.
__device__ inline void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

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
    static constexpr int NF = WTM + WTN;          // fragment reads per k-step
    static constexpr int NM = WTM * WTN;          // MFMAs per k-step
    static_assert(AI * RPI * NW == BM && BI * RPI * NW == BN, "rows per wave");
    static_assert(NKK >= 2 && NKK % 2 == 0, "an even number of k-steps per stage");

    AccV acc[WTM][WTN];

    __device__ static inline int swz(int c, int row) { return c ^ ((row >> 1) & 7); }

    // Loads of one 64-wide k-slice (element offset k0) of both panels into
    // the LDS stage at byte offset `stage`.  Row r of a panel lies at byte
    // r * ld * 2 of its resource; rows of one instruction start at a multiple
    // of 8, so their swizzle depends only on the parity of the row block.
    __device__ inline void issue(uint32_t stage, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb,
                                 int64_t lda, int64_t ldb, int64_t k0, int w, const uint32_t *voa,
                                 const uint32_t *vob) {
#pragma unroll
        for (int q = 0; q < AI; ++q) {
            const int blk = w * AI + q, row0 = blk * RPI;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                ra, (lds_void *)(uintptr_t)(stage + row0 * ROWB), 16, voa[blk & 1],
                (uint32_t)((int64_t)row0 * lda * 2 + k0 * 2), 0, 0);
        }
#pragma unroll
        for (int q = 0; q < BI; ++q) {
            const int blk = w * BI + q, row0 = blk * RPI;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rb, (lds_void *)(uintptr_t)(stage + (BM + row0) * ROWB), 16, vob[blk & 1],
                (uint32_t)((int64_t)row0 * ldb * 2 + k0 * 2), 0, 0);
        }
    }

    __device__ inline void load_frags(const char *s, int kk, Frag *f) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int wm = wid % WM, wn = wid / WM;
        const int ch = (kk + Mf::E * (lane / Mf::M)) / CE;
        const char *sA = s, *sB = s + BM * ROWB;
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
            const int row = wm * WTM * Mf::M + i * Mf::M + lane % Mf::M;
            f[i] = *(const Frag *)(sA + row * ROWB + 16 * swz(ch, row));
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int row = wn * WTN * Mf::M + j * Mf::M + lane % Mf::M;
            f[WTM + j] = *(const Frag *)(sB + row * ROWB + 16 * swz(ch, row));
        }
    }

    __device__ inline void mmas(const Frag *f) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) acc[i][j] = Mf::mma(f[i], f[WTM + j], acc[i][j]);
    }

    // Scheduling order of one k-step: the NF fragment reads spread evenly
    // between its NM MFMAs.
    template <int I = 0> __device__ static inline void interleave() {
        constexpr int G = NF > NM ? NF : NM;
        constexpr int nd = (I + 1) * NF / G - I * NF / G;
        constexpr int nm = (I + 1) * NM / G - I * NM / G;
        if constexpr (nd > 0) __builtin_amdgcn_sched_group_barrier(0x100, nd, 0);
        if constexpr (nm > 0) __builtin_amdgcn_sched_group_barrier(0x008, nm, 0);
        if constexpr (I + 1 < G) interleave<I + 1>();
    }

    // Full K loop (K a multiple of 64; rows m0.. and n0.. of the operands
    // inside the allocations).  smem holds SMEM bytes.
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
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const uint32_t s0 = (uint32_t)(uintptr_t)(lds_void *)smem;
        __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + m0 * lda), 0, (int)(BM * lda * 2), 0x00020000);
        __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B + n0 * ldb), 0, (int)(BN * ldb * 2), 0x00020000);
        uint32_t voa[2], vob[2];
        {
            const int lane = threadIdx.x & 63, rl = lane / CPR, sl = lane % CPR;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int c = 16 * (sl ^ (((rl >> 1) + 4 * p) & 7));
                voa[p] = (uint32_t)(rl * lda * 2 + c);
                vob[p] = (uint32_t)(rl * ldb * 2 + c);
            }
        }
        issue(s0, ra, rb, lda, ldb, 0, w, voa, vob);
        if (nk > 1) {
            issue(s0 + STAGE, ra, rb, lda, ldb, BK, w, voa, vob);
            wait_vmcnt<AI + BI>();
        } else {
            wait_vmcnt<0>();
        }
        lds_barrier();
        Frag f[2][NF];
        load_frags(smem, 0, f[0]);
        for (int kt = 0; kt < nk - 1; ++kt) {
            const char *cur = smem + (kt & 1) * STAGE;
#pragma unroll
            for (int q = 0; q < NKK - 1; ++q) {
                load_frags(cur, (q + 1) * Mf::KI, f[(q + 1) & 1]);
                mmas(f[q & 1]);
                interleave();
            }
            wait_vmcnt<0>();      // stage kt + 1, issued one stage ago, has landed
            lds_barrier();        // ... for every wave, and nobody reads stage kt any more
            load_frags(smem + ((kt + 1) & 1) * STAGE, 0, f[0]);
            mmas(f[1]);
            interleave();
            if (kt + 2 < nk) issue(s0 + (kt & 1) * STAGE, ra, rb, lda, ldb, (int64_t)(kt + 2) * BK, w, voa, vob);
        }
        const char *cur = smem + ((nk - 1) & 1) * STAGE;
#pragma unroll
        for (int q = 0; q < NKK - 1; ++q) {
            load_frags(cur, (q + 1) * Mf::KI, f[(q + 1) & 1]);
            mmas(f[q & 1]);
            interleave();
        }
        mmas(f[1]);
        lds_barrier();
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
