// Shared definitions for the gfx950 kernels of libcaddelag.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

namespace cdl {

// n x n matrices are stored with ld = n rounded up to kPadN rows and columns.
constexpr int kPadN = 256;
// Vectors of k projections are padded to a multiple of kPadK columns.
constexpr int kPadK = 64;
constexpr int kNumXcd = 8;

inline int64_t ld_of(int64_t n) { return (n + kPadN - 1) / kPadN * kPadN; }
inline int64_t kpad_of(int64_t k) { return (k + kPadK - 1) / kPadK * kPadK; }

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// MFMA families.  Operand layout (checked on gfx950 hardware): for an
// instruction computing an M x M tile over KI reduction steps, lane l holds
// E consecutive reduction elements k = E*(l / M) .. +E-1 of row (l % M) of
// both operands (A row-major along k; B given as its transpose, also
// row-major along k).  Accumulator element r of lane l is (crow, ccol).

struct MfmaBF16 {
    using T = __bf16;
    using Frag = bf16x8;
    using Acc = float;
    using AccV = f32x16;
    static constexpr int M = 32, KI = 16, E = 8, R = 16;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ static inline int ccol(int lane) { return lane & 31; }
};

struct MfmaF16 {
    using T = _Float16;
    using Frag = f16x8;
    using Acc = float;
    using AccV = f32x16;
    static constexpr int M = 32, KI = 16, E = 8, R = 16;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ static inline int ccol(int lane) { return lane & 31; }
};

// The 16 x 16 x 32 forms: half the work and latency of the 32 x 32 x 16
// instruction, the same per-lane operand layout (8 consecutive reduction
// elements of one row), four accumulators per lane.
struct MfmaBF16x32 {
    using T = __bf16;
    using Frag = bf16x8;
    using Acc = float;
    using AccV = f32x4;
    static constexpr int M = 16, KI = 32, E = 8, R = 4;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static inline int ccol(int lane) { return lane & 15; }
};

struct MfmaF16x32 {
    using T = _Float16;
    using Frag = f16x8;
    using Acc = float;
    using AccV = f32x4;
    static constexpr int M = 16, KI = 32, E = 8, R = 4;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static inline int ccol(int lane) { return lane & 15; }
};

struct MfmaF32 {
    using T = float;
    using Frag = float;
    using Acc = float;
    using AccV = f32x16;
    static constexpr int M = 32, KI = 2, E = 1, R = 16;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ static inline int ccol(int lane) { return lane & 31; }
};

struct MfmaF64 {
    using T = double;
    using Frag = double;
    using Acc = double;
    using AccV = f64x4;
    static constexpr int M = 16, KI = 4, E = 1, R = 4;
    __device__ static inline AccV mma(const Frag &a, const Frag &b, const AccV &c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int crow(int lane, int r) { return (lane >> 4) + 4 * r; }
    __device__ static inline int ccol(int lane) { return lane & 15; }
};

template <typename T> struct MfmaOf;
template <> struct MfmaOf<__bf16> { using type = MfmaBF16; };
template <> struct MfmaOf<_Float16> { using type = MfmaF16; };
template <> struct MfmaOf<float> { using type = MfmaF32; };
template <> struct MfmaOf<double> { using type = MfmaF64; };

// Conversions from float/double accumulators to storage types (round to
// nearest even).
template <typename T> __device__ inline T cvt(float x);
template <> __device__ inline __bf16 cvt<__bf16>(float x) { return (__bf16)x; }
template <> __device__ inline _Float16 cvt<_Float16>(float x) { return (_Float16)x; }
template <> __device__ inline float cvt<float>(float x) { return x; }
template <> __device__ inline double cvt<double>(float x) { return (double)x; }

template <typename T> __device__ inline T cvtd(double x);
template <> __device__ inline __bf16 cvtd<__bf16>(double x) { return (__bf16)(float)x; }
template <> __device__ inline _Float16 cvtd<_Float16>(double x) { return (_Float16)(float)x; }
template <> __device__ inline float cvtd<float>(double x) { return (float)x; }
template <> __device__ inline double cvtd<double>(double x) { return x; }

template <typename T> __device__ inline double tod(T x) { return (double)(float)x; }
template <> __device__ inline double tod<double>(double x) { return x; }

// ---------------------------------------------------------------------------
// Workgroup -> tile maps.  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; remapping so that consecutive logical tiles
// land on the same XCD lets neighbouring tiles share operand panels in L2.

// Upper-triangle cover by 256 x 128 tiles of an ld x ld matrix (ncol =
// ld / 128 column blocks, nrow = ld / 256 row blocks): row block I takes the
// column blocks J = 2I .. ncol - 1; rect_upper_tiles(ld) = nrow ncol -
// nrow (nrow - 1) tiles in all.
// The tiles of the cover in the row panel [I0, I0 + nrows) (I0 = 0, nrows = ld / 256:
// the whole matrix), enumerated in bands of G tile rows: within a band column
// by column, so that consecutive ids (which one XCD runs side by side) share
// their 128-column operand block across up to G row blocks.  A band starting
// at row r0 with h rows holds h (h + 1) tiles in columns 2 r0 .. 2 (r0 + h) - 1
// (column pair p has p + 1 rows) and h tiles in each later column.
template <int G>
__host__ __device__ inline void upper_band_tile(int id, int I0, int nrows, int ncol, int &I,
                                                int &J) {
    int r0 = I0;
    while (true) {
        const int h = I0 + nrows - r0 < G ? I0 + nrows - r0 : G;
        const int cnt = h * (h + 1) + (ncol - 2 * r0 - 2 * h) * h;
        if (id < cnt || r0 + h >= I0 + nrows) {
            if (id < h * (h + 1)) {
                int p = (int)((sqrt(4.0 * (double)id + 1.0) - 1.0) * 0.5);
                while (p > 0 && p * (p + 1) > id) --p;
                while ((p + 1) * (p + 2) <= id) ++p;
                const int r = id - p * (p + 1);
                J = 2 * r0 + 2 * p + r / (p + 1);
                I = r0 + r % (p + 1);
            } else {
                const int q = id - h * (h + 1);
                J = 2 * r0 + 2 * h + q / h;
                I = r0 + q % h;
            }
            return;
        }
        id -= cnt;
        r0 += h;
    }
}
__host__ __device__ inline int rect_upper_tiles(int64_t ld) {
    const int ncol = (int)(ld / 128), nrow = (int)(ld / 256);
    return nrow * ncol - nrow * (nrow - 1);
}

__device__ inline int xcd_remap(int w, int total) {
    int x = w % kNumXcd, j = w / kNumXcd;
    int base = total / kNumXcd, rem = total % kNumXcd;
    return x * base + (x < rem ? x : rem) + j;
}

// For one-workgroup-per-CU kernels: workgroups run in rounds of kNumCu (one
// per CU); within a full round XCD x takes the CPX = kNumCu / kNumXcd
// consecutive logical tiles [CPX x, CPX x + CPX).  Each round thus covers a
// compact run of logical tiles chip-wide (operand panels shared across XCDs
// through the memory-attached cache) and each XCD a compact sub-run (shared
// in its L2).  The last, partial round keeps the dispatch order.
constexpr int kNumCu = 256;
__device__ inline int round_remap(int w, int total) {
    constexpr int cpx = kNumCu / kNumXcd;
    const int r = w / kNumCu, x = w % kNumXcd, j = (w / kNumXcd) % cpx;
    return (r + 1) * kNumCu <= total ? r * kNumCu + x * cpx + j : w;
}

// Upper-triangular tile (I <= J) of an nt x nt tile grid, grouped in bands
// of G tile rows: band g enumerates the G x G diagonal triangle column by
// column, then the rectangular part column by column, so that a run of
// consecutive ids covers a compact G-row block.
template <int G>
__device__ inline void sym_tile(int id, int nt, int &I, int &J) {
    int g0 = 0;
    while (true) {
        int h = nt - g0 < G ? nt - g0 : G;
        int tri = h * (h + 1) / 2;
        int cnt = tri + (nt - g0 - h) * h;
        if (id < cnt) {
            if (id < tri) {
                int c = 0;
                while ((c + 1) * (c + 2) / 2 <= id) ++c;
                J = g0 + c;
                I = g0 + (id - c * (c + 1) / 2);
            } else {
                int q = id - tri;
                J = g0 + h + q / h;
                I = g0 + q % h;
            }
            return;
        }
        id -= cnt;
        g0 += G;
    }
}

// Rectangular mt x nt tile grid in column bands of G tile columns.
template <int G>
__device__ inline void rect_tile(int id, int mt, int nt, int &I, int &J) {
    int band = id / (G * mt);
    int j0 = band * G;
    int w = nt - j0 < G ? nt - j0 : G;
    int q = id - band * G * mt;
    I = q / w;
    J = j0 + q % w;
}

// acc + p[0] + p[stride] + ... + p[(cnt - 1) stride], added in index order
// (the same rounding as a plain loop), with 32 loads in flight at a time.
__device__ inline double ordered_sum(const double *p, int64_t stride, int cnt, double acc) {
    int b = 0;
    for (; b + 32 <= cnt; b += 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = p[(int64_t)(b + u) * stride];
#pragma unroll
        for (int u = 0; u < 32; ++u) acc += v[u];
    }
    for (; b < cnt; ++b) acc += p[(int64_t)b * stride];
    return acc;
}

} // namespace cdl
