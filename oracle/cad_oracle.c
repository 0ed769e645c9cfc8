/*
 * Plain CPU FP64 oracle helpers for commute-time anomaly detection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists so that the tests, the smoke check and the CPU
 * baseline can compute reference results.  It shares no code, headers or
 * constants-generators with the GPU library.
 *
 * Every loop is the plain definition, in FP64, with a fixed summation order
 * (ascending index), parallelised over independent output rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* SplitMix64 output function (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014; the 64-bit finaliser with the
 * constants of the public-domain reference generator). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Sign word for edge {lo, hi} (global ids, lo < hi < 2^20) and projection
 * block beta = r / 64 (< 2^24): bit (r mod 64) set means sign -1. */
uint64_t orc_sign_word(uint64_t seed, uint64_t beta, uint64_t lo, uint64_t hi)
{
    uint64_t key = orc_mix64(seed) ^ ((beta << 40) | (lo << 20) | hi);
    return orc_mix64(key);
}

/*
 * Right-hand sides of Algorithm 1 (random vector q over the edges, mapped to
 * node space by the transposed signed incidence matrix):
 *   Y[v, r] = (1/sqrt(k)) * sum over edges e containing v of
 *             B(e, v) * sqrt(W_e) * q_r(e),
 * with B(e, v) = +1 if v is e's head (the endpoint with the lower global id)
 * and -1 if v is its tail, and q_r(e) = +-1 from the sign word.
 * W: n x n row-major (only off-diagonal entries are read), Y: n x k row-major.
 */
void orc_rhs(const double *W, int64_t n, const int32_t *gid, int64_t k,
             uint64_t seed, double *Y)
{
    const double scale = 1.0 / sqrt((double)k);
    const int64_t nb = (k + 63) / 64;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t v = 0; v < n; ++v) {
        double *y = Y + v * k;
        for (int64_t r = 0; r < k; ++r) y[r] = 0.0;
        uint64_t gv = gid ? (uint64_t)gid[v] : (uint64_t)v;
        for (int64_t u = 0; u < n; ++u) {
            if (u == v) continue;
            uint64_t gu = gid ? (uint64_t)gid[u] : (uint64_t)u;
            double w = sqrt(W[v * n + u]) * scale;
            /* incidence sign of v on edge {u, v} */
            double inc = (gv < gu) ? 1.0 : -1.0;
            uint64_t lo = gv < gu ? gv : gu, hi = gv < gu ? gu : gv;
            for (int64_t b = 0; b < nb; ++b) {
                uint64_t h = orc_sign_word(seed, (uint64_t)b, lo, hi);
                int64_t r1 = (b + 1) * 64 < k ? (b + 1) * 64 : k;
                for (int64_t r = b * 64; r < r1; ++r) {
                    double q = ((h >> (r & 63)) & 1ULL) ? -1.0 : 1.0;
                    y[r] += inc * q * w;
                }
            }
        }
    }
}

/* Same as orc_rhs for a subset of rows: Y is nrows x k for rows[0..nrows). */
void orc_rhs_rows(const double *W, int64_t n, const int32_t *gid, int64_t k,
                  uint64_t seed, const int64_t *rows, int64_t nrows, double *Y)
{
    const double scale = 1.0 / sqrt((double)k);
    const int64_t nb = (k + 63) / 64;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t v = rows[t];
        double *y = Y + t * k;
        for (int64_t r = 0; r < k; ++r) y[r] = 0.0;
        uint64_t gv = gid ? (uint64_t)gid[v] : (uint64_t)v;
        for (int64_t u = 0; u < n; ++u) {
            if (u == v) continue;
            uint64_t gu = gid ? (uint64_t)gid[u] : (uint64_t)u;
            double w = sqrt(W[t * n + u]) * scale;   /* W holds the sampled rows */
            double inc = (gv < gu) ? 1.0 : -1.0;
            uint64_t lo = gv < gu ? gv : gu, hi = gv < gu ? gu : gv;
            for (int64_t b = 0; b < nb; ++b) {
                uint64_t h = orc_sign_word(seed, (uint64_t)b, lo, hi);
                int64_t r1 = (b + 1) * 64 < k ? (b + 1) * 64 : k;
                for (int64_t r = b * 64; r < r1; ++r) {
                    double q = ((h >> (r & 63)) & 1ULL) ? -1.0 : 1.0;
                    y[r] += inc * q * w;
                }
            }
        }
    }
}

/* Squared Euclidean distances by direct differences for rows[0..nrows):
 * out[t, j] = sum_tau (X[rows[t], tau] - X[j, tau])^2.  X: n x T row-major. */
void orc_sq_distances_rows(const double *X, int64_t n, int64_t T,
                           const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        const double *xi = X + rows[t] * T;
        for (int64_t j = 0; j < n; ++j) {
            const double *xj = X + j * T;
            double s = 0.0;
            for (int64_t c = 0; c < T; ++c) {
                double d = xi[c] - xj[c];
                s += d * d;
            }
            out[t * n + j] = s;
        }
    }
}

/*
 * Node anomaly scores (Algorithm 4 with the CAD edge score):
 *   F[i] = sum_j  omega_ij * | c0(i,j) - c1(i,j) |,
 *   c_t(i,j) = vol_t * || z^t_i - z^t_j ||^2   (by direct differences),
 * over the m common nodes: Z0, Z1 are m x k row-major (already restricted to
 * the common nodes, same order).  omega = |A1 - A0| if A0 and A1 are given
 * (their rows rows[0..nrows), each m long: nrows x m row-major), else 1.
 * Only rows[0..nrows) of F are computed.
 */
void orc_scores_rows(const double *Z0, double vol0, const double *Z1, double vol1,
                     int64_t m, int64_t k, const double *A0, const double *A1,
                     const int64_t *rows, int64_t nrows, double *F)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double s0 = 0.0, s1 = 0.0;
            for (int64_t r = 0; r < k; ++r) {
                double d0 = Z0[i * k + r] - Z0[j * k + r];
                double d1 = Z1[i * k + r] - Z1[j * k + r];
                s0 += d0 * d0;
                s1 += d1 * d1;
            }
            double dc = fabs(vol0 * s0 - vol1 * s1);
            if (A0 && A1) dc *= fabs(A1[t * m + j] - A0[t * m + j]);
            acc += dc;
        }
        F[t] = acc;
    }
}
