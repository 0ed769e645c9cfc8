// Graph construction for one snapshot (Section "Climate Data": fully
// connected graph with Gaussian-kernel weights of the distance between node
// series; Background: symmetric A, no self-edges, volume V_G = sum_i D(i,i)).
//
//   pad_series   copy X into a zero-padded FP64 panel, row norms ||x_i||^2
//   gram_dist    D2_ij = ||x_i||^2 + ||x_j||^2 - 2 x_i.x_j on FP64 MFMA,
//                256 x 128 tiles covering the upper triangle (the strictly
//                lower tiles are never computed or read), stored from the
//                accumulators
//   select       exact lower median of D2 over i < j: a sampled bracket
//                around the median rank, the keys inside it gathered into a
//                buffer and ranked by radix passes over their IEEE-754 bit
//                patterns (order-preserving for D2 >= 0); the same radix
//                passes over the whole upper triangle when the bracket
//                misses the rank or overflows the buffer
//   exp_sym      per upper 64 x 64 tile: W = exp(-D2 / sigma^2) in place,
//                W_ii = 0, written with its mirror; row and column sums
//                into one partial per (tile column, node)
//   degree       deg = sum of the partials in tile order
//   graph_stats  vol = sum deg, min and max degree (fixed-order reductions)
//
// Streamed snapshots (no n x n matrix stored) use the same tiles on row
// panels: gram_dist over the panel's upper tiles (median sweeps) or all of
// its tiles, optionally with the weights formed in the epilogue; select by
// radix digits from the top bit, one sweep over the upper panels per digit;
// exp_rows for the weights, degrees and Frobenius rows of a panel.
#include "batch.h"
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace cdl {

int64_t pad_n(int64_t n) { return ld_of(n); }
int64_t pad_k(int64_t k) { return kpad_of(k); }
int64_t pad_t(int64_t T) { return (T + 15) / 16 * 16; }

// Deterministic sum over a 64-lane wave (xor butterfly, same order everywhere).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Deterministic sum over a 256-thread block; result valid in every thread.
__device__ inline double block_sum256(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------

__global__ void k_fill_zero(uint4 *p, size_t n16) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 16 || ((uintptr_t)p) % 16) return hipErrorInvalidValue;
    size_t n16 = bytes / 16;
    int grid = (int)(n16 / 256 + 1 < 8192 ? n16 / 256 + 1 : 8192);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s, (uint4 *)p, n16);
    return hipGetLastError();
}

// Plain device copy: one 16-byte element per lane, a grid covering the whole
// buffer (consecutive workgroups stream consecutive memory), nontemporal
// loads and stores (the data is touched once).  The reference stream for HBM
// bandwidth and for the byte counters; measured on gfx950 at 1 GiB it moves
// about 1.5x the bytes per second of a grid-stride loop over the same data.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const u32x4 *__restrict__ src,
                                                u32x4 *__restrict__ dst, size_t n16) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 16 || ((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16, grid = (n16 + 255) / 256;
    if (grid > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(256), 0, s, (const u32x4 *)src,
                       (u32x4 *)dst, n16);
    return hipGetLastError();
}

// One wave per (padded) row.
// Padded row i of the series and its squared norm (one wave).
__device__ __forceinline__ void pad_row(const double *X, int64_t n, int64_t T, int64_t ldx,
                                        double *Xp, int64_t Tp, double *sqn, int *flags,
                                        int64_t i) {
    const int lane = threadIdx.x;
    double s = 0.0;
    int bad = 0;
    for (int64_t t = lane; t < Tp; t += 64) {
        double v = (i < n && t < T) ? X[i * ldx + t] : 0.0;
        if (!isfinite(v)) bad = 1;
        Xp[i * Tp + t] = v;
        s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) sqn[i] = s;
    if (bad) atomicOr(flags, 1);
}

__global__ void k_pad_series(const double *X, int64_t n, int64_t T, int64_t ldx,
                             double *Xp, int64_t Tp, double *sqn, int *flags) {
    pad_row(X, n, T, ldx, Xp, Tp, sqn, flags, blockIdx.x);
}

hipError_t launch_pad_series(const double *X, int64_t n, int64_t T, int64_t ldx,
                             double *Xp, int64_t rows, int64_t Tp, double *sqn,
                             int *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_series, dim3((unsigned)rows), dim3(64), 0, s, X, n, T, ldx, Xp,
                       Tp, sqn, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Squared distances from the Gram matrix of the series (FP64 MFMA).

// The cover is made of 256 x 128 tiles; each is computed as two 128 x 128
// halves by two workgroups of four waves (each wave 64 x 64: 16 MFMAs per 8
// fragment reads), BK 16.  A half takes 74 KB of LDS, so two workgroups fit
// on a CU and one's epilogue (distances, median bracket, stores) runs beside
// the other's MFMAs.
using GramCore = GemmCore<MfmaF64, 128, 128, 16, 2, 2>;
constexpr int kGramWgPerTile = 2;
constexpr size_t kGramSmem = GramCore::SMEM;



// Tiles of row blocks [I0, I0 + pb): those of the upper-triangle cover
// (full = 0; I0 = 0 and pb = ld / 256 give the whole cover) or all ncol of
// each row block (full = 1).  Row i is stored at D2 + (i - 256 I0) ld, so a
// row panel needs a buffer of 256 pb rows only.
// st != nullptr: also fold the smallest and largest upper-triangle key
// (i < j) into st->kmin / st->kmax (the median selection starts below their
// common bit prefix); with brbuf as well, the bracket pass of the selection
// on the tile's upper-triangle keys: count those below st->lo into st->below
// and append those in [lo, hi] to brbuf (capacity brcap) through an LDS
// stage in the GEMM's staging memory, one segment per wave filled at ballot
// positions (a wave with more of them than its segment holds marks the
// buffer full, which sends the selection to its passes over the matrix:
// exact either way).  kExp: store the
// weights exp(-D2 / sigma^2) instead (zero on the diagonal and outside n;
// sigma = wstats[1]), the expression of the separate exponential kernels, so
// the values are the same bits.
template <bool kExp>
__device__ __forceinline__ void gram_tile(const double *Xp, int64_t Tp, const double *sqn,
                                          int64_t n, int64_t ld, double *D2, int ncol, int I0,
                                          int pb, int full, int id, SelectState *st,
                                          const double *wstats, double *smem,
                                          unsigned long long *brbuf = nullptr,
                                          int64_t brcap = 0) {
    // workgroup id: half id & 1 (rows 128 (id & 1) ..) of tile id >> 1
    const int tile = id >> 1, half = id & 1;
    int I, J;
    if (full) {
        rect_tile<4>(tile, pb, ncol, I, J);
        I += I0;
    } else {
        upper_band_tile<4>(tile, I0, pb, ncol, I, J);
    }
    const int64_t m0 = (int64_t)I * 256 + 128 * half, n0 = (int64_t)J * 128;
    double *const out = D2 - (int64_t)I0 * 256 * ld;
    GramCore g;
    g.run(Xp, Tp, Xp, Tp, m0, n0, Tp, smem);
    unsigned long long kmin = ~0ull, kmax = 0ull;
    // bracket stage: the GEMM's LDS, free once every wave is past its last
    // fragment read; each wave appends to its own segment of it
    constexpr unsigned int kSeg = (unsigned int)(GramCore::SMEM / 8 / (GramCore::NT / 64));
    __shared__ unsigned long long sbel[GramCore::NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned long long *const seg = (unsigned long long *)smem + wid * kSeg;
    const unsigned long long ltmask = (1ull << lane) - 1ull;
    unsigned long long blo = 0ull, bhi = 0ull;
    unsigned int below = 0, wcount = 0;   // wcount: the wave's bracket keys so far (every lane)
    if (brbuf) {
        blo = st->lo;
        bhi = st->hi;
        __syncthreads();
    }
    // the squared norms of this lane's rows and columns, loaded once (the
    // stores below may alias sqn as far as the compiler knows)
    double sa[GramCore::WTM][MfmaF64::R], sb[GramCore::WTN];
#pragma unroll
    for (int a = 0; a < GramCore::WTM; ++a)
#pragma unroll
        for (int rr = 0; rr < MfmaF64::R; ++rr) sa[a][rr] = sqn[m0 + GramCore::row_of(a, rr)];
#pragma unroll
    for (int b = 0; b < GramCore::WTN; ++b) sb[b] = sqn[n0 + GramCore::col_of(b)];
    // D2 of element (r, c) (zero outside n and on the diagonal); upper: an
    // upper-triangle pair inside n, whose key is set
    auto f = [&](int r, int c, double acc, double sqa, double sqb, bool &upper,
                 unsigned long long &key) -> double {
        const int64_t a = m0 + r, b = n0 + c;
        upper = false;
        key = 0ull;
        if (a >= n || b >= n || a == b) return 0.0;
        double d = sqa + sqb - 2.0 * acc;
        d = d < 0.0 ? 0.0 : d;
        if (a < b) {
            key = (unsigned long long)__double_as_longlong(d);
            kmin = key < kmin ? key : kmin;
            kmax = key > kmax ? key : kmax;
            upper = true;
        }
        return d;
    };
    double s2 = 0.0;
    if (kExp) {
        const double sigma = wstats[1];
        s2 = sigma * sigma;
    }
    // direct stores: 16 lanes cover 16 consecutive columns of one row
#pragma unroll
    for (int a = 0; a < GramCore::WTM; ++a)
#pragma unroll
        for (int b = 0; b < GramCore::WTN; ++b)
#pragma unroll
            for (int rr = 0; rr < MfmaF64::R; ++rr) {
                const int r = GramCore::row_of(a, rr), c = GramCore::col_of(b);
                bool upper;
                unsigned long long key;
                double v = f(r, c, g.acc[a][b][rr], sa[a][rr], sb[b], upper, key);
                if (brbuf) {   // count below; append inside at the wave's ballot positions
                    below += upper && key < blo ? 1u : 0u;
                    const bool in = upper && key >= blo && key <= bhi;
                    const unsigned long long m = __ballot(in);
                    const unsigned int pos = wcount + (unsigned int)__popcll(m & ltmask);
                    if (in && pos < kSeg) seg[pos] = key;
                    wcount += (unsigned int)__popcll(m);
                }
                if (kExp) {
                    const int64_t ia = m0 + r, ib = n0 + c;
                    v = (ia < n && ib < n && ia != ib) ? exp(-v / s2) : 0.0;
                }
                out[(m0 + r) * ld + n0 + c] = v;
            }
    if (brbuf) {
        // each wave's segment behind one global atomic (a full segment marks
        // the buffer full: the passes then take the matrix); the count below
        // behind one atomic per tile
        unsigned long long base = 0ull;
        if (lane == 0 && wcount > 0)
            base = atomicAdd(&st->nbuf, wcount > kSeg ? (unsigned long long)brcap + 1ull
                                                      : (unsigned long long)wcount);
        base = __shfl(base, 0);
        if (wcount <= kSeg)
            for (unsigned int q = lane; q < wcount; q += 64)
                if (base + q < (unsigned long long)brcap) brbuf[base + q] = seg[q];
        unsigned long long bw = below;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) bw += __shfl_xor(bw, o);
        if (lane == 0) sbel[wid] = bw;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long bl = 0ull;
#pragma unroll
            for (int w = 0; w < GramCore::NT / 64; ++w) bl += sbel[w];
            if (bl) atomicAdd(&st->below, bl);
        }
    }
    if (st) {
        // the tile's smallest and largest key: waves, then the workgroup, then
        // one pair of atomics per tile (all tiles update the same two words)
        __shared__ unsigned long long wmin[GramCore::NT / 64], wmax[GramCore::NT / 64];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long a = __shfl_xor(kmin, o), b = __shfl_xor(kmax, o);
            kmin = a < kmin ? a : kmin;
            kmax = b > kmax ? b : kmax;
        }
        if ((threadIdx.x & 63) == 0) {
            wmin[threadIdx.x >> 6] = kmin;
            wmax[threadIdx.x >> 6] = kmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 1; w < GramCore::NT / 64; ++w) {
                kmin = wmin[w] < kmin ? wmin[w] : kmin;
                kmax = wmax[w] > kmax ? wmax[w] : kmax;
            }
            if (kmin != ~0ull) atomicMin(&st->kmin, kmin);
            if (kmax != 0ull) atomicMax(&st->kmax, kmax);
        }
    }
}

template <bool kExp>
__global__ __launch_bounds__(GramCore::NT, 2) void k_gram_dist(const double *Xp, int64_t Tp,
                                                   const double *sqn, int64_t n, int64_t ld,
                                                   double *D2, int ncol, int I0, int pb,
                                                   int full, int total, SelectState *st,
                                                   const double *wstats,
                                                   unsigned long long *brbuf, int64_t brcap) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    gram_tile<kExp>(Xp, Tp, sqn, n, ld, D2, ncol, I0, pb, full, xcd_remap(blockIdx.x, total), st,
                    wstats, (double *)smem_raw, brbuf, brcap);
}

static hipError_t gram_attr() {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_gram_dist<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kGramSmem);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_gram_dist<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGramSmem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    return hipSuccess;
}

hipError_t launch_gram_dist(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                            int64_t ld, double *D2, SelectState *st, unsigned long long *brbuf,
                            int64_t brcap, hipStream_t s) {
    if (brbuf && !st) return hipErrorInvalidValue;
    hipError_t e = gram_attr();
    if (e != hipSuccess) return e;
    const int ncol = (int)(ld / 128);
    const int total = kGramWgPerTile * rect_upper_tiles(ld);
    hipLaunchKernelGGL(k_gram_dist<false>, dim3(total), dim3(GramCore::NT), kGramSmem, s, Xp, Tp, sqn, n,
                       ld, D2, ncol, 0, (int)(ld / 256), 0, total, st, (const double *)nullptr,
                       brbuf, brcap);
    return hipGetLastError();
}

int64_t gram_panel_tiles(int64_t ld, int64_t row0, int64_t rows, bool full) {
    const int64_t ncol = ld / 128, I0 = row0 / 256, pb = rows / 256;
    return full ? pb * ncol : pb * ncol - 2 * (I0 * pb + pb * (pb - 1) / 2);
}

hipError_t launch_gram_panel(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                             int64_t ld, int64_t row0, int64_t rows, bool full, double *D2p,
                             const double *wstats, hipStream_t s) {
    if (row0 % 256 || rows % 256 || rows <= 0 || row0 + rows > ld) return hipErrorInvalidValue;
    if (wstats && !full) return hipErrorInvalidValue;
    hipError_t e = gram_attr();
    if (e != hipSuccess) return e;
    const int64_t total = kGramWgPerTile * gram_panel_tiles(ld, row0, rows, full);
    if (total <= 0 || total > INT32_MAX) return hipErrorInvalidValue;
    const int ncol = (int)(ld / 128), I0 = (int)(row0 / 256), pb = (int)(rows / 256);
    if (wstats)
        hipLaunchKernelGGL(k_gram_dist<true>, dim3((unsigned)total), dim3(GramCore::NT), kGramSmem, s, Xp,
                           Tp, sqn, n, ld, D2p, ncol, I0, pb, 1, (int)total,
                           (SelectState *)nullptr, wstats, (unsigned long long *)nullptr,
                           (int64_t)0);
    else
        hipLaunchKernelGGL(k_gram_dist<false>, dim3((unsigned)total), dim3(GramCore::NT), kGramSmem, s, Xp,
                           Tp, sqn, n, ld, D2p, ncol, I0, pb, full ? 1 : 0, (int)total,
                           (SelectState *)nullptr, (const double *)nullptr,
                           (unsigned long long *)nullptr, (int64_t)0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact selection of the element of rank floor((N-1)/2), N = n(n-1)/2, among
// D2_ij (i < j).  D2 >= 0, so its IEEE bit pattern orders like its value.
// First a bracket: a sorted sample of kSelSample keys gives [lo, hi] around
// the target quantile (three standard deviations of the sample quantile on
// each side), the sample's keys taken from the series before the Gram; the
// keys below lo are counted and those in [lo, hi] appended to a buffer, by
// the Gram's epilogue for stored snapshots, by one sweep over the recomputed
// upper panels for streamed ones.  If the target rank falls inside the bracket
// the radix passes below run over the buffer, else over the matrix (the
// result is exact either way).  Radix passes of 12-bit digits start below the
// common prefix of the bracket (or of the smallest and largest key); as soon
// as the selected bin holds at most kSelCap keys, one pass collects them and
// a single workgroup sorts them.  Every pass kernel reads the state's mode,
// so the fixed launch sequence turns into no-ops once the answer is known.

__device__ __forceinline__ void select_reset_body(SelectState *st) {
    for (int b = threadIdx.x; b < 4096; b += blockDim.x) st->hist[b] = 0;
    if (threadIdx.x == 0) {
        st->kmin = ~0ull;
        st->kmax = 0ull;
        st->count = 0;
        st->mode = 0;
        st->src = 0;
        st->below = 0;
        st->nbuf = 0;
    }
}

__global__ void k_select_reset(SelectState *st) { select_reset_body(st); }

constexpr int kSelSample = 4096;
constexpr int kSelMargin = 96;    // 3 sqrt(kSelSample / 4): misses in ~0.3% of calls

int64_t select_buffer_keys(int64_t n) {
    const int64_t N = n * (n - 1) / 2;
    const int64_t cap = N / 8 + 65536;
    return cap < ((int64_t)1 << 27) ? cap : ((int64_t)1 << 27);
}

__device__ inline unsigned long long sel_mix(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Sample pair u of the bracket: a pseudo-random pair i != j.
__device__ inline void sel_pair(unsigned long long u, int64_t n, int64_t &a, int64_t &b) {
    const unsigned long long h = sel_mix(0x5851f42d4c957f2dull + u);
    const int64_t i = (int64_t)((h & 0xffffffffull) % (unsigned long long)n);
    int64_t j = (int64_t)((h >> 32) % (unsigned long long)(n - 1));
    if (j >= i) ++j;   // j != i
    a = i < j ? i : j;
    b = i < j ? j : i;
}

// Sort the kSelSample keys in sk (LDS, 1024 threads) and set the bracket
// [lo, hi] of kSelMargin sample ranks on each side of the target rank.
__device__ __forceinline__ void select_sort_bracket(int64_t n, SelectState *st,
                                                    unsigned long long *sk) {
    const int t = threadIdx.x;
    for (int size = 2; size <= kSelSample; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = t; q < kSelSample / 2; q += 1024) {
                const int lo = 2 * q - (q & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned long long a = sk[lo], b = sk[hi];
                if ((a > b) == up) { sk[lo] = b; sk[hi] = a; }
            }
            __syncthreads();
        }
    if (t == 0) {
        const unsigned long long N = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
        const double rho = (double)((N - 1ull) / 2ull) / (double)N;
        const int q = (int)(rho * kSelSample);
        st->lo = q - kSelMargin <= 0 ? 0ull : sk[q - kSelMargin];
        st->hi = q + kSelMargin >= kSelSample - 1 ? ~0ull : sk[q + kSelMargin];
        st->below = 0;
        st->nbuf = 0;
    }
}

// The same sample pairs' keys from the padded series, before the Gram: one
// wave per pair, D2 = sq_a + sq_b - 2 x_a.x_b with the dot product summed
// over the lanes (another order than the Gram's: an estimate of the quantile,
// which is all the bracket needs; the counts against it are exact).
__device__ __forceinline__ void select_sample_keys_body(const double *Xp, int64_t Tp,
                                                        const double *sqn, int64_t n,
                                                        unsigned long long *keys, int wave,
                                                        int nwave) {
    const int lane = threadIdx.x & 63;
    for (int u = wave; u < kSelSample; u += nwave) {
        int64_t a, b;
        sel_pair((unsigned long long)u, n, a, b);
        const double *xa = Xp + a * Tp, *xb = Xp + b * Tp;
        double dot = 0.0;
        for (int64_t q = lane; q < Tp; q += 64) dot += xa[q] * xb[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) dot += __shfl_xor(dot, o);
        if (lane == 0) {
            double d = sqn[a] + sqn[b] - 2.0 * dot;
            d = d < 0.0 ? 0.0 : d;
            keys[u] = (unsigned long long)__double_as_longlong(d);
        }
    }
}

__global__ __launch_bounds__(256) void k_select_sample_keys(const double *Xp, int64_t Tp,
                                                            const double *sqn, int64_t n,
                                                            unsigned long long *keys) {
    select_sample_keys_body(Xp, Tp, sqn, n, keys, blockIdx.x * 4 + (threadIdx.x >> 6),
                            gridDim.x * 4);
}

__device__ __forceinline__ void select_sort_keys(const unsigned long long *keys, int64_t n,
                                                 SelectState *st, unsigned long long *sk) {
    for (int u = threadIdx.x; u < kSelSample; u += 1024) sk[u] = keys[u];
    __syncthreads();
    select_sort_bracket(n, st, sk);
}

__global__ __launch_bounds__(1024) void k_select_sort_bracket(const unsigned long long *keys,
                                                              int64_t n, SelectState *st) {
    extern __shared__ unsigned long long sk[];
    select_sort_keys(keys, n, st, sk);
}

// The bracket pass for very many keys (streamed panels: billions of keys,
// tens of thousands inside the bracket per workgroup): the workgroup's rows
// go in rounds of 2048 keys with a barrier after each, and whenever the LDS
// stage holds 2048 or more keys it is copied out behind one global atomic,
// so the global counter sees one atomic per ~2048 keys instead of one each.
__global__ __launch_bounds__(256) void k_select_bracket_flush(const double *D2, int64_t ld,
                                                              int64_t n, int64_t row0,
                                                              int64_t row1, SelectState *st,
                                                              unsigned long long *buf,
                                                              int64_t cap) {
    constexpr unsigned int kStage = 4096, kRound = 8 * 256;
    __shared__ unsigned long long sb[kStage];
    __shared__ unsigned int scnt;
    __shared__ unsigned long long sbase, spart[4];
    if (st->mode == 2) return;
    const unsigned long long lo = st->lo, hi = st->hi;
    const int t = threadIdx.x;
    if (t == 0) scnt = 0;
    __syncthreads();
    unsigned long long below = 0;
    auto flush = [&]() {   // every thread, after a barrier
        const unsigned int c = scnt;
        if (t == 0 && c > 0) sbase = atomicAdd(&st->nbuf, (unsigned long long)c);
        __syncthreads();
        const unsigned long long base = sbase;
        for (unsigned int q = t; q < c; q += 256)
            if (base + q < (unsigned long long)cap) buf[base + q] = sb[q];
        __syncthreads();
        if (t == 0) scnt = 0;
        __syncthreads();
    };
    for (int64_t i = row0 + blockIdx.x; i < row1; i += gridDim.x) {
        const unsigned long long *row = (const unsigned long long *)(D2 + (i - row0) * ld);
        for (int64_t jb = i + 1; jb < n; jb += kRound) {   // the same trip count in every thread
            unsigned long long key[8];   // eight independent loads in flight
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t j = jb + t + 256 * u;
                key[u] = j < n ? row[j] : ~0ull;   // ~0: above every bracket
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (key[u] < lo) {
                    ++below;
                } else if (key[u] <= hi && key[u] != ~0ull) {
                    const unsigned int q = atomicAdd(&scnt, 1u);   // < kStage: at most kRound per round
                    sb[q] = key[u];
                }
            }
            __syncthreads();
            const unsigned int c = scnt;
            __syncthreads();   // read by every thread before the next round appends
            if (c >= kStage - kRound) flush();
        }
    }
    __syncthreads();
    flush();
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) below += __shfl_xor(below, o);
    if ((t & 63) == 0) spart[t >> 6] = below;
    __syncthreads();
    if (t == 0) {
        const unsigned long long b = spart[0] + spart[1] + spart[2] + spart[3];
        if (b) atomicAdd(&st->below, b);
    }
}

// Switch the radix passes to the buffer when the target lies in the bracket.
__device__ __forceinline__ void select_check_body(SelectState *st, int64_t cap, double *stats) {
    if (threadIdx.x != 0 || st->mode == 2) return;
    const unsigned long long below = st->below, nb = st->nbuf, rank = st->rank;
    if (nb > (unsigned long long)cap || rank < below || rank >= below + nb) return;   // stay on the matrix
    st->src = 1;
    st->rank = rank - below;
    const unsigned long long x = st->lo ^ st->hi;
    if (x == 0ull) {   // every bracket key equals lo
        st->prefix = st->lo;
        st->bits = 64;
        st->mode = 2;
        stats[1] = sqrt(__longlong_as_double((long long)st->lo));
        return;
    }
    const int L = __clzll((long long)x);
    if (L > st->bits) {
        st->bits = L;
        st->prefix = st->lo & ~((1ull << (64 - L)) - 1ull);
    }
    st->mode = nb <= (unsigned long long)kSelCap ? 1 : 0;
    st->count = 0;
}

__global__ void k_select_check(SelectState *st, int64_t cap, double *stats) {
    select_check_body(st, cap, stats);
}

__device__ __forceinline__ void select_setup_body(SelectState *st, int64_t n, double *stats) {
    if (threadIdx.x != 0) return;
    const unsigned long long N = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
    st->rank = (N - 1ull) / 2ull;
    const unsigned long long x = st->kmin ^ st->kmax;
    if (x == 0ull) {   // every pair distance is the same value
        st->prefix = st->kmin;
        st->bits = 64;
        st->mode = 2;
        stats[1] = sqrt(__longlong_as_double((long long)st->kmin));
        return;
    }
    const int L = __clzll((long long)x);
    st->bits = L;
    st->prefix = L == 0 ? 0ull : (st->kmin & ~((1ull << (64 - L)) - 1ull));
    st->mode = 0;
}

__global__ void k_select_setup(SelectState *st, int64_t n, double *stats) {
    select_setup_body(st, n, stats);
}

__device__ inline void sel_digit(const SelectState *st, int &shift, int &width,
                                 unsigned long long &hi_mask) {
    const int bits = st->bits;
    width = 64 - bits < 12 ? 64 - bits : 12;
    shift = 64 - bits - width;
    hi_mask = bits == 0 ? 0ull : ~((1ull << (64 - bits)) - 1ull);
}

// Keys of rows [row0, row1): row i at D2 + (i - row0) ld (a row panel, or
// the whole matrix with row0 = 0, row1 = n).
// Workgroup b of nb.
__device__ __forceinline__ void select_pass_body(const double *D2, int64_t ld, int64_t n,
                                                 int64_t row0, int64_t row1, SelectState *st,
                                                 const unsigned long long *buf, int64_t b,
                                                 int64_t nb) {
    __shared__ unsigned int h[4096];
    const int mode = st->mode;
    if (mode == 2) return;
    // Up to 2^24 buffered keys go to at most kBufBlocks workgroups, each
    // flushing its histogram once for many keys: the flush is global atomics
    // on the same 4096 bins, and thousands of workgroups flushing them
    // contend.  Larger buffers keep the whole grid for bandwidth.
    constexpr int kBufBlocks = 256;
    const bool from_buf = st->src == 1;
    const bool few = from_buf && st->nbuf <= (1ull << 24);
    if (few && b >= kBufBlocks) return;
    int shift, width;
    unsigned long long hi_mask;
    sel_digit(st, shift, width, hi_mask);
    const unsigned long long prefix = st->prefix;
    if (mode == 0) {
        for (int b = threadIdx.x; b < 4096; b += 256) h[b] = 0;
        __syncthreads();
    }
    const unsigned long long dmask = (1ull << width) - 1ull;
    auto take = [&](unsigned long long key) {
        if ((key & hi_mask) != prefix) return;
        if (mode == 0) {
            atomicAdd(&h[(key >> shift) & dmask], 1u);
        } else {
            const unsigned int q = atomicAdd(&st->count, 1u);
            if (q < kSelCap) st->cand[q] = key;
        }
    };
    // eight independent loads in flight per thread
    if (from_buf) {
        const int64_t gb = few && nb > kBufBlocks ? (int64_t)kBufBlocks : nb;
        const int64_t nk = (int64_t)st->nbuf, stride = gb * 256;
        for (int64_t q0 = b * 256 + threadIdx.x; q0 < nk; q0 += 8 * stride) {
            unsigned long long key[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) key[u] = q0 + u * stride < nk ? buf[q0 + u * stride] : 0ull;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u * stride < nk) take(key[u]);
        }
    } else {
        for (int64_t i = row0 + b; i < row1; i += nb) {
            const unsigned long long *row = (const unsigned long long *)(D2 + (i - row0) * ld);
            for (int64_t j0 = i + 1 + threadIdx.x; j0 < n; j0 += 8 * 256) {
                unsigned long long key[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) key[u] = j0 + 256 * u < n ? row[j0 + 256 * u] : 0ull;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + 256 * u < n) take(key[u]);
            }
        }
    }
    if (mode == 0) {
        __syncthreads();
        for (int q = threadIdx.x; q < 4096; q += 256)
            if (h[q]) atomicAdd(&st->hist[q], (unsigned long long)h[q]);
    }
}

__global__ __launch_bounds__(256) void k_select_pass(const double *D2, int64_t ld, int64_t n,
                                                     int64_t row0, int64_t row1,
                                                     SelectState *st,
                                                     const unsigned long long *buf) {
    select_pass_body(D2, ld, n, row0, row1, st, buf, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void select_pick_body(SelectState *st, double *stats) {
    constexpr int NT = 1024, BPT = 4096 / NT;
    __shared__ unsigned long long part[NT / 64];
    __shared__ unsigned long long keys[kSelCap];
    const int t = threadIdx.x;
    const int mode = st->mode;
    if (mode == 2) return;
    if (mode == 1) {
        // sort the collected candidates (count <= kSelCap) and take the rank
        const unsigned int cnt = st->count;
        for (int q = t; q < kSelCap; q += NT) keys[q] = q < (int)cnt ? st->cand[q] : ~0ull;
        __syncthreads();
        for (int size = 2; size <= kSelCap; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int q = t; q < kSelCap / 2; q += NT) {
                    const int lo = 2 * q - (q & (stride - 1)), hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const unsigned long long a = keys[lo], b = keys[hi];
                    if ((a > b) == up) { keys[lo] = b; keys[hi] = a; }
                }
                __syncthreads();
            }
        if (t == 0) {
            const unsigned long long key = keys[st->rank];
            st->prefix = key;
            st->bits = 64;
            st->mode = 2;
            stats[1] = sqrt(__longlong_as_double((long long)key));
        }
        return;
    }
    int shift, width;
    unsigned long long hi_mask;
    sel_digit(st, shift, width, hi_mask);
    unsigned long long c[BPT], sum = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        c[q] = st->hist[t * BPT + q];
        sum += c[q];
    }
    // exclusive prefix of the per-thread bin sums: within each wave by
    // shuffles, then across the waves
    unsigned long long incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(incl, o);
        if ((t & 63) >= o) incl += y;
    }
    if ((t & 63) == 63) part[t >> 6] = incl;
    __syncthreads();
    unsigned long long before = incl - sum;
    for (int w = 0; w < (t >> 6); ++w) before += part[w];
    const unsigned long long rank = st->rank;
    int bin = -1;
    unsigned long long newrank = 0, cnt = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        if (bin < 0 && rank >= before && rank < before + c[q]) {
            bin = t * BPT + q;
            newrank = rank - before;
            cnt = c[q];
        }
        before += c[q];
    }
    __syncthreads();
    if (bin >= 0) {
        const unsigned long long p = st->prefix | ((unsigned long long)bin << shift);
        st->prefix = p;
        st->bits += width;
        st->rank = newrank;
        if (st->bits >= 64) {
            st->mode = 2;
            stats[1] = sqrt(__longlong_as_double((long long)p));
        } else if (cnt <= (unsigned long long)kSelCap) {
            st->mode = 1;
            st->count = 0;
        }
    }
    __syncthreads();
    for (int b = t; b < 4096; b += NT) st->hist[b] = 0;
}

__global__ __launch_bounds__(1024) void k_select_pick(SelectState *st, double *stats) {
    select_pick_body(st, stats);
}

hipError_t launch_select_reset(SelectState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_select_reset, dim3(1), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_select_presample(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                                   SelectState *st, unsigned long long *buf, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_select_sort_bracket,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kSelSample * 8);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (select_buffer_keys(n) < kSelSample) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select_sample_keys, dim3(64), dim3(256), 0, s, Xp, Tp, sqn, n, buf);
    hipLaunchKernelGGL(k_select_sort_bracket, dim3(1), dim3(1024), kSelSample * 8, s, buf, n, st);
    return hipGetLastError();
}

hipError_t launch_select_median(const double *D2, int64_t ld, int64_t n, SelectState *st,
                                unsigned long long *buf, bool gathered, double *stats,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_select_setup, dim3(1), dim3(64), 0, s, st, n, stats);
    const int grid = (int)(n < 2048 ? n : 2048);
    const int64_t cap = select_buffer_keys(n);
    if (gathered)   // the Gram's epilogue counted and gathered the bracket
        hipLaunchKernelGGL(k_select_check, dim3(1), dim3(64), 0, s, st, cap, stats);
    // at most 6 digit passes resolve 64 bits; the collect pass is one more
    for (int p = 0; p < 7; ++p) {
        hipLaunchKernelGGL(k_select_pass, dim3(grid), dim3(256), 0, s, D2, ld, n, (int64_t)0, n,
                           st, buf);
        hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(1024), 0, s, st, stats);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streamed selection (no stored matrix): radix digits from the top bit, each
// digit one k_select_pass per recomputed row panel of the upper triangle and
// one pick; the collect pass and the final sort are those of the stored path.

__global__ void k_select_start_top(SelectState *st, int64_t n) {
    if (threadIdx.x != 0) return;
    const unsigned long long N = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
    st->rank = (N - 1ull) / 2ull;
    st->prefix = 0ull;
    st->bits = 0;
    st->mode = 0;
    st->src = 0;
    st->count = 0;
}

hipError_t launch_select_start_top(SelectState *st, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_select_reset, dim3(1), dim3(256), 0, s, st);
    hipLaunchKernelGGL(k_select_start_top, dim3(1), dim3(64), 0, s, st, n);
    return hipGetLastError();
}

hipError_t launch_select_panel(const double *D2p, int64_t ld, int64_t n, int64_t row0,
                               int64_t row1, SelectState *st, hipStream_t s) {
    if (row1 <= row0) return hipSuccess;
    const int64_t rows = row1 - row0;
    const int grid = (int)(rows < 2048 ? rows : 2048);
    hipLaunchKernelGGL(k_select_pass, dim3(grid), dim3(256), 0, s, D2p, ld, n, row0, row1, st,
                       (const unsigned long long *)nullptr);
    return hipGetLastError();
}

hipError_t launch_select_pick(SelectState *st, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(1024), 0, s, st, stats);
    return hipGetLastError();
}

// The streamed bracket: kStreamSample distances of pseudo-random pairs
// computed directly from the padded series (sq_a + sq_b - 2 x_a.x_b in
// sequential FP64, an estimate of the quantile only: the bracket is checked
// against exact counts), sorted in LDS, bracket of kStreamMargin sample ranks
// on each side of the target; then one sweep over the upper panels counts the
// keys below the bracket and gathers those inside it, and the radix passes run
// over the gathered keys.  The larger sample keeps the bracket to about 2.3 %
// of the keys.
constexpr int kStreamSample = 16384;
constexpr int kStreamMargin = 192;   // 3 sqrt(kStreamSample / 4)

int64_t select_stream_keys(int64_t n) {
    const int64_t N = n * (n - 1) / 2;
    return N / 100 * 3 + 65536;
}

__global__ __launch_bounds__(1024) void k_select_sample_x(const double *Xp, int64_t Tp,
                                                          const double *sqn, int64_t n,
                                                          SelectState *st) {
    extern __shared__ unsigned long long sk[];
    const int t = threadIdx.x;
    for (int u = 0; u < kStreamSample / 1024; ++u) {
        int64_t i, j;
        sel_pair((unsigned long long)(t + 1024 * u), n, i, j);
        const double *xa = Xp + i * Tp, *xb = Xp + j * Tp;
        double dot = 0.0;
        for (int64_t q = 0; q < Tp; ++q) dot += xa[q] * xb[q];
        double d = sqn[i] + sqn[j] - 2.0 * dot;
        d = d < 0.0 ? 0.0 : d;
        sk[t + 1024 * u] = (unsigned long long)__double_as_longlong(d);
    }
    __syncthreads();
    for (int size = 2; size <= kStreamSample; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = t; q < kStreamSample / 2; q += 1024) {
                const int lo = 2 * q - (q & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned long long a = sk[lo], b = sk[hi];
                if ((a > b) == up) { sk[lo] = b; sk[hi] = a; }
            }
            __syncthreads();
        }
    if (t == 0) {
        const unsigned long long N = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
        const double rho = (double)((N - 1ull) / 2ull) / (double)N;
        const int q = (int)(rho * kStreamSample);
        st->lo = q - kStreamMargin <= 0 ? 0ull : sk[q - kStreamMargin];
        st->hi = q + kStreamMargin >= kStreamSample - 1 ? ~0ull : sk[q + kStreamMargin];
        st->below = 0;
        st->nbuf = 0;
    }
}

hipError_t launch_select_sample_x(const double *Xp, int64_t Tp, const double *sqn, int64_t n,
                                  SelectState *st, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_select_sample_x,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kStreamSample * 8);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_select_sample_x, dim3(1), dim3(1024), kStreamSample * 8, s, Xp, Tp, sqn,
                       n, st);
    return hipGetLastError();
}

hipError_t launch_select_bracket_panel(const double *D2p, int64_t ld, int64_t n, int64_t row0,
                                       int64_t row1, SelectState *st, unsigned long long *buf,
                                       int64_t cap, hipStream_t s) {
    if (row1 <= row0) return hipSuccess;
    const int64_t rows = row1 - row0;
    const int grid = (int)(rows < 2048 ? rows : 2048);
    hipLaunchKernelGGL(k_select_bracket_flush, dim3(grid), dim3(256), 0, s, D2p, ld, n, row0, row1,
                       st, buf, cap);
    return hipGetLastError();
}

hipError_t launch_select_check(SelectState *st, int64_t cap, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_select_check, dim3(1), dim3(64), 0, s, st, cap, stats);
    return hipGetLastError();
}

hipError_t launch_select_buffer_pass(SelectState *st, const unsigned long long *buf, int64_t cap,
                                     double *stats, hipStream_t s) {
    const int grid = (int)(cap / 2048 + 1 < 2048 ? cap / 2048 + 1 : 2048);
    hipLaunchKernelGGL(k_select_pass, dim3(grid), dim3(256), 0, s, (const double *)nullptr,
                       (int64_t)0, (int64_t)0, (int64_t)0, (int64_t)0, st, buf);
    hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(1024), 0, s, st, stats);
    return hipGetLastError();
}

// Row panel of the weights from its squared distances, in place: W_ij =
// exp(-D2_ij / sigma^2) for i != j (both < n), else 0 - the expression of
// k_exp_sym, so each value equals the stored matrix's bit for bit.  Panel row
// q is node row0 + q.  deg != nullptr: deg_i = sum_j W_ij (fixed order).
// dinv != nullptr: fro[q] = sum_j (W_ij dinv_i dinv_j)^2 with dinv = D^{-1/2},
// a row of the squared Frobenius norm of S = D^{-1/2} W D^{-1/2}.
__global__ __launch_bounds__(256) void k_exp_rows(double *Wp, int64_t ld, int64_t n,
                                                  int64_t row0, const double *stats,
                                                  double *deg, const double *dinv,
                                                  double *fro) {
    __shared__ double red[4];
    const int64_t i = row0 + blockIdx.x;
    double *row = Wp + (int64_t)blockIdx.x * ld;
    const double sigma = stats[1];
    const double s2 = sigma * sigma;
    const bool live = i < n;
    const double di = (dinv && live) ? dinv[i] : 0.0;
    double acc = 0.0, f = 0.0;
    for (int64_t j0 = threadIdx.x; j0 < ld; j0 += 4 * 256) {
        double d2[4];   // four loads in flight before the first exp
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + 256 * u;
            d2[u] = j < ld ? row[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + 256 * u;
            if (j >= ld) break;
            const double v = (live && j < n && i != j) ? exp(-d2[u] / s2) : 0.0;
            row[j] = v;
            acc += v;
            if (dinv && v != 0.0) {
                const double sv = v * di * dinv[j];
                f += sv * sv;
            }
        }
    }
    acc = block_sum256(acc, red);
    if (deg && live && threadIdx.x == 0) deg[i] = acc;
    if (fro) {
        f = block_sum256(f, red);
        if (threadIdx.x == 0) fro[blockIdx.x] = f;
    }
}

hipError_t launch_exp_rows(double *Wp, int64_t ld, int64_t n, int64_t row0, int64_t rows,
                           const double *stats, double *deg, const double *dinv, double *fro,
                           hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exp_rows, dim3((unsigned)rows), dim3(256), 0, s, Wp, ld, n, row0, stats,
                       deg, dinv, fro);
    return hipGetLastError();
}

__global__ void k_set_sigma(double sigma, double *stats) { stats[1] = sigma; }

hipError_t launch_set_sigma(double sigma, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_set_sigma, dim3(1), dim3(1), 0, s, sigma, stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

int sym_tiles64(int64_t ld) {
    const int nt = (int)(ld / 64);
    return nt * (nt + 1) / 2;
}

// One 64 x 64 tile (I <= J) per workgroup.  part[J][i] receives the sum of
// row i over the tile's columns and, for I < J, part[I][j] the sum of column
// j: every (tile column, node) slot is written by exactly one tile.  A lane
// takes two adjacent columns of every other row (16-byte loads and stores),
// so a wave access covers two contiguous 512-byte row segments; the four
// waves take 16 rows each.  The mirror is written from the LDS copy, two
// adjacent rows per lane.
// Upper tile `id` (after the XCD remap) of the sym_tile<8> order.
__device__ __forceinline__ void exp_sym_tile(double *W, int64_t ld, int64_t n,
                                             const double *stats, int nt, double *part, int id) {
    struct alignas(16) D2 { double x, y; };
    __shared__ double t[64][66];   // even pitch: 16-byte rows of pairs
    __shared__ double cs[4][64];
    int I, J;
    sym_tile<8>(id, nt, I, J);
    const double sigma = stats[1];
    const double s2 = sigma * sigma;
    const int64_t i0 = (int64_t)I * 64, j0 = (int64_t)J * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cp = lane & 31, h = lane >> 5;
    const int64_t ja = j0 + 2 * cp;   // this lane's columns ja, ja + 1
    double c0 = 0.0, c1 = 0.0;
    D2 d2[8];   // all eight row loads in flight before the first exp
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) d2[rr] = *(const D2 *)(W + (i0 + wv * 16 + 2 * rr + h) * ld + ja);
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
        const int r = wv * 16 + 2 * rr + h;
        const int64_t i = i0 + r;
        D2 v;
        v.x = (i < n && ja < n && i != ja) ? exp(-d2[rr].x / s2) : 0.0;
        v.y = (i < n && ja + 1 < n && i != ja + 1) ? exp(-d2[rr].y / s2) : 0.0;
        *(D2 *)(W + i * ld + ja) = v;
        *(D2 *)&t[r][2 * cp] = v;
        c0 += v.x;
        c1 += v.y;
    }
    // this wave's column sums: the two halves hold the even and odd rows
    c0 += __shfl_xor(c0, 32);
    c1 += __shfl_xor(c1, 32);
    if (h == 0) {
        cs[wv][2 * cp] = c0;
        cs[wv][2 * cp + 1] = c1;
    }
    __syncthreads();
    {   // row sums: thread (row r, quarter q) over 16 columns
        const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
        double rs = 0.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) rs += t[r][16 * q + c];
        rs += __shfl_xor(rs, 1);
        rs += __shfl_xor(rs, 2);
        if (q == 0) part[(int64_t)J * ld + i0 + r] = rs;
    }
    if (I == J) return;
    if (threadIdx.x < 64)
        part[(int64_t)I * ld + j0 + threadIdx.x] =
            (cs[0][threadIdx.x] + cs[1][threadIdx.x]) + (cs[2][threadIdx.x] + cs[3][threadIdx.x]);
#pragma unroll 4
    for (int cc = 0; cc < 8; ++cc) {   // mirror: row j0 + c gets column c of the tile
        const int c = wv * 16 + 2 * cc + h;
        const D2 m{t[2 * cp][c], t[2 * cp + 1][c]};
        *(D2 *)(W + (j0 + c) * ld + i0 + 2 * cp) = m;
    }
}

__global__ __launch_bounds__(256) void k_exp_sym(double *W, int64_t ld, int64_t n,
                                                 const double *stats, int nt, double *part) {
    exp_sym_tile(W, ld, n, stats, nt, part, xcd_remap(blockIdx.x, nt * (nt + 1) / 2));
}

__global__ void k_degree_reduce(const double *part, int nt, int64_t ld, int64_t n, double *deg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    deg[i] = ordered_sum(part + i, ld, nt, 0.0);
}

hipError_t launch_exp_degree(double *W, int64_t ld, int64_t n, const double *stats,
                             double *deg, double *part, hipStream_t s) {
    const int nt = (int)(ld / 64);
    hipLaunchKernelGGL(k_exp_sym, dim3((unsigned)sym_tiles64(ld)), dim3(256), 0, s, W, ld, n,
                       stats, nt, part);
    // one wave per workgroup: the n threads spread over every CU
    hipLaunchKernelGGL(k_degree_reduce, dim3((unsigned)cdiv(n, 64)), dim3(64), 0, s, part, nt,
                       ld, n, deg);
    return hipGetLastError();
}

__device__ __forceinline__ void graph_stats_body(const double *deg, int64_t n, double *stats) {
    __shared__ double red[4];
    __shared__ double rmin[256], rmax[256];
    double s = 0.0, lo = INFINITY, hi = -INFINITY;
    // a thread's nodes in increasing order, sixteen loads in flight
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += 16 * 256) {
        double dv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) dv[u] = i0 + 256 * u < n ? deg[i0 + 256 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (i0 + 256 * u >= n) break;
            const double d = dv[u];
            s += d;
            lo = fmin(lo, d);
            hi = fmax(hi, d);
            if (isnan(d)) lo = hi = d;
        }
    }
    rmin[threadIdx.x] = lo;
    rmax[threadIdx.x] = hi;
    s = block_sum256(s, red);
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = rmin[0], b = rmax[0];
        for (int q = 1; q < 256; ++q) {
            a = (isnan(rmin[q]) || isnan(a)) ? NAN : fmin(a, rmin[q]);
            b = (isnan(rmax[q]) || isnan(b)) ? NAN : fmax(b, rmax[q]);
        }
        stats[0] = s;
        stats[2] = a;
        stats[3] = b;
    }
}

__global__ __launch_bounds__(256) void k_graph_stats(const double *deg, int64_t n,
                                                     double *stats) {
    graph_stats_body(deg, n, stats);
}

hipError_t launch_graph_stats(const double *deg, int64_t n, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_graph_stats, dim3(1), dim3(256), 0, s, deg, n, stats);
    return hipGetLastError();
}

// Caller-supplied weights: copy into the padded layout, zero the diagonal,
// row sums, and flag non-finite (1), negative (2) or asymmetric (4) input.
__global__ __launch_bounds__(256) void k_import_weights(const double *Win, int64_t ldw,
                                                        int64_t n, double *W, int64_t ld,
                                                        double *deg, int *flags) {
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    double s = 0.0;
    int f = 0;
    for (int64_t j = threadIdx.x; j < ld; j += 256) {
        double v = 0.0;
        if (i < n && j < n && i != j) {
            v = Win[i * ldw + j];
            if (!isfinite(v)) f |= 1;
            if (v < 0.0) f |= 2;
            if (v != Win[j * ldw + i]) f |= 4;
        }
        W[i * ld + j] = v;
        s += v;
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0 && i < n) deg[i] = s;
    if (f) atomicOr(flags, f);
}

hipError_t launch_import_weights(const double *Win, int64_t ldw, int64_t n, double *W,
                                 int64_t ld, double *deg, int *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_import_weights, dim3((unsigned)ld), dim3(256), 0, s, Win, ldw, n, W,
                       ld, deg, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The graph build of many snapshots in grouped launches: each kernel below
// runs, for workgroup blockIdx.x, the per-snapshot kernel's workgroup
// blockIdx.x - prefix[p] of snapshot p (found through the kernel's prefix
// table), with that snapshot's arguments, so the results are the
// per-snapshot kernels' bit for bit.

bool select_uses_bracket(int64_t n, bool allowed) {
    const double N = (double)n * (double)(n - 1) / 2.0;
    return allowed && N * 2.0 * kSelMargin / kSelSample <= 0.8 * (double)select_buffer_keys(n);
}

int graph_table_count(int tb, int64_t n, int64_t ld, bool bracket) {
    const int grid = (int)(n < 2048 ? n : 2048);
    switch (tb) {
    case kGtRows: return (int)ld;
    case kGtOne: return 1;
    case kGtGram: return kGramWgPerTile * rect_upper_tiles(ld);
    case kGtSample: return bracket ? 1 : 0;
    case kGtKeys: return bracket ? 16 : 0;
    case kGtPass: return grid;
    case kGtSym: return sym_tiles64(ld);
    case kGtNodes64: return (int)cdiv(n, 64);
    case kGtPrep: return (int)cdiv(ld, 256);
    default: return 0;
    }
}

struct GroupSlot {
    int p;
    int64_t b, nb;
};
__device__ __forceinline__ GroupSlot group_slot(const int *prefix, int P) {
    GroupSlot g;
    g.p = group_find(prefix, P, blockIdx.x);
    g.b = blockIdx.x - prefix[g.p];
    g.nb = prefix[g.p + 1] - prefix[g.p];
    return g;
}

__global__ __launch_bounds__(256) void k_graph_init_grouped(const GraphSnap *snaps, const int *prefix,
                                                            int P, int select) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    if (threadIdx.x < 64) d.flags[threadIdx.x] = 0;
    if (select) select_reset_body(d.sel);
}

__global__ __launch_bounds__(64) void k_pad_grouped(const GraphSnap *snaps, const int *prefix, int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    pad_row(d.X, d.n, d.T, d.ldx, d.Xp, d.Tp, d.sqn, d.flags, g.b);
}

__global__ __launch_bounds__(256) void k_select_keys_grouped(const GraphSnap *snaps, const int *prefix,
                                                             int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    select_sample_keys_body(d.Xp, d.Tp, d.sqn, d.n, d.buf, (int)g.b * 4 + (threadIdx.x >> 6),
                            (int)g.nb * 4);
}

__global__ __launch_bounds__(1024) void k_select_sort_grouped(const GraphSnap *snaps, const int *prefix,
                                                              int P) {
    extern __shared__ unsigned long long sk[];
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    select_sort_keys(d.buf, d.n, d.sel, sk);
}

__global__ __launch_bounds__(GramCore::NT, 2) void k_gram_grouped(const GraphSnap *snaps, const int *prefix, int P,
                                                      int select) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    gram_tile<false>(d.Xp, d.Tp, d.sqn, d.n, d.ld, d.W, (int)(d.ld / 128), 0, (int)(d.ld / 256), 0,
                     xcd_remap((int)g.b, (int)g.nb), select ? d.sel : nullptr,
                     (const double *)nullptr, (double *)smem_raw,
                     select && d.bracket ? d.buf : nullptr, d.cap);
}

__global__ __launch_bounds__(64) void k_select_setup_grouped(const GraphSnap *snaps, const int *prefix,
                                                             int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    select_setup_body(d.sel, d.n, d.stats);
}

__global__ __launch_bounds__(64) void k_select_check_grouped(const GraphSnap *snaps, const int *prefix,
                                                             int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    select_check_body(d.sel, d.cap, d.stats);
}

__global__ __launch_bounds__(256) void k_select_pass_grouped(const GraphSnap *snaps, const int *prefix,
                                                             int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    select_pass_body(d.W, d.ld, d.n, 0, d.n, d.sel, d.buf, g.b, g.nb);
}

__global__ __launch_bounds__(1024) void k_select_pick_grouped(const GraphSnap *snaps, const int *prefix,
                                                              int P) {
    const GroupSlot g = group_slot(prefix, P);
    select_pick_body(snaps[g.p].sel, snaps[g.p].stats);
}

__global__ void k_set_sigma_grouped(const GraphSnap *snaps, const int *prefix, int P, double sigma) {
    const GroupSlot g = group_slot(prefix, P);
    if (threadIdx.x == 0) snaps[g.p].stats[1] = sigma;
}

__global__ __launch_bounds__(256) void k_exp_sym_grouped(const GraphSnap *snaps, const int *prefix, int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    const int nt = (int)(d.ld / 64);
    exp_sym_tile(d.W, d.ld, d.n, d.stats, nt, d.dpart, xcd_remap((int)g.b, (int)g.nb));
}

__global__ __launch_bounds__(64) void k_degree_grouped(const GraphSnap *snaps, const int *prefix, int P) {
    const GroupSlot g = group_slot(prefix, P);
    const GraphSnap &d = snaps[g.p];
    const int64_t i = g.b * 64 + threadIdx.x;
    if (i < d.n) d.deg[i] = ordered_sum(d.dpart + i, d.ld, (int)(d.ld / 64), 0.0);
}

__global__ __launch_bounds__(256) void k_graph_stats_grouped(const GraphSnap *snaps, const int *prefix,
                                                             int P) {
    const GroupSlot g = group_slot(prefix, P);
    graph_stats_body(snaps[g.p].deg, snaps[g.p].n, snaps[g.p].stats);
}

hipError_t launch_graph_grouped(const GraphSnap *snaps, const int *tables, const int *totals,
                                int P, double sigma, hipStream_t s) {
    auto tb = [&](int t) { return tables + (size_t)t * (P + 1); };
    hipError_t e = gram_attr();
    if (e != hipSuccess) return e;
    static bool attr = false;
    if (!attr) {
        e = hipFuncSetAttribute((const void *)k_gram_grouped,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGramSmem);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_select_sort_grouped,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kSelSample * 8);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const bool select = sigma <= 0.0;
    hipLaunchKernelGGL(k_graph_init_grouped, dim3(totals[kGtOne]), dim3(256), 0, s, snaps, tb(kGtOne), P,
                       select ? 1 : 0);
    hipLaunchKernelGGL(k_pad_grouped, dim3(totals[kGtRows]), dim3(64), 0, s, snaps, tb(kGtRows), P);
    // the brackets from samples of the series; the Gram counts and gathers them
    if (select && totals[kGtSample] > 0) {
        hipLaunchKernelGGL(k_select_keys_grouped, dim3(totals[kGtKeys]), dim3(256), 0, s, snaps,
                           tb(kGtKeys), P);
        hipLaunchKernelGGL(k_select_sort_grouped, dim3(totals[kGtSample]), dim3(1024), kSelSample * 8, s,
                           snaps, tb(kGtSample), P);
    }
    hipLaunchKernelGGL(k_gram_grouped, dim3(totals[kGtGram]), dim3(GramCore::NT), kGramSmem, s, snaps,
                       tb(kGtGram), P, select ? 1 : 0);
    if (select) {
        hipLaunchKernelGGL(k_select_setup_grouped, dim3(totals[kGtOne]), dim3(64), 0, s, snaps, tb(kGtOne), P);
        if (totals[kGtSample] > 0)
            hipLaunchKernelGGL(k_select_check_grouped, dim3(totals[kGtSample]), dim3(64), 0, s, snaps,
                               tb(kGtSample), P);
        // as in the per-snapshot selection: at most 6 digit passes and the
        // collect pass, each followed by the pick
        for (int q = 0; q < 7; ++q) {
            hipLaunchKernelGGL(k_select_pass_grouped, dim3(totals[kGtPass]), dim3(256), 0, s, snaps,
                               tb(kGtPass), P);
            hipLaunchKernelGGL(k_select_pick_grouped, dim3(totals[kGtOne]), dim3(1024), 0, s, snaps,
                               tb(kGtOne), P);
        }
    } else {
        hipLaunchKernelGGL(k_set_sigma_grouped, dim3(totals[kGtOne]), dim3(64), 0, s, snaps, tb(kGtOne), P,
                           sigma);
    }
    hipLaunchKernelGGL(k_exp_sym_grouped, dim3(totals[kGtSym]), dim3(256), 0, s, snaps, tb(kGtSym), P);
    hipLaunchKernelGGL(k_degree_grouped, dim3(totals[kGtNodes64]), dim3(64), 0, s, snaps, tb(kGtNodes64), P);
    hipLaunchKernelGGL(k_graph_stats_grouped, dim3(totals[kGtOne]), dim3(256), 0, s, snaps, tb(kGtOne), P);
    return hipGetLastError();
}

} // namespace cdl
