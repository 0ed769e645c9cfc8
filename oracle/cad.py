"""CPU FP64 oracle: the plain definitions, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Citations name the
paper's sections, equations and algorithms:

* Background section: the graph model (symmetric A_t, no self-edges), the
  incidence factorisation L = B^T W B, commute time eq. (1)
  c(i,j) = V_G (l+_ii + l+_jj - 2 l+_ij) with V_G = sum_i D(i,i), and the
  CAD edge score Delta E_t = |A_{t+1} - A_t| * |c_{t+1} - c_t|.
* Algorithm 1 (commute time distance): random vector q over the edges,
  y = B^T W^{1/2} q (the printed W^{1/2} B q does not type-check; the
  transposed incidence is the only reading that yields an n-vector), solve
  L z = y, accumulate (z_i - z_j)^2.
* Section "Solving SDD Linear Systems", eq. (inverse chain):
  (I - A)^{-1} = prod_k (I + A^{2^k}) + eps for ||A|| < 1.
* Algorithm 2 (SDD solver): ChainProduct with S = D^{-1/2} A D^{-1/2},
  P = (I+S)(I+S^2)...(I+S^{2^{d-1}}) C, P1 = D^{-1/2} P, P2 = D^{-1/2} P L;
  EstimateSolution: chi = P1 b, y_1 = 0, y_{k+1} = y_k - P2 y_k + chi.
* Algorithm 3 (CommuteTimeEmbedding) and Algorithm 4 (CADDeLaG): Z from the
  k_RP solves; node scores F_i = sum_j Delta E_{i,j}; top anomalies by F.
* Section "Climate Data": fully connected graph with Gaussian-kernel weights
  of the distance between node series.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg

__all__ = [
    "mix64", "sign_words", "projection_signs",
    "sq_distances", "sq_distances_rows", "bandwidth", "gaussian_weights",
    "degrees", "laplacian", "build_graph",
    "rhs", "rhs_rows", "rhs_numpy",
    "solve_embedding", "solve_embedding_eigh", "pinv_laplacian",
    "commute_times", "exact_commute_times", "scores", "scores_rows", "top_k",
    "edge_scores", "top_edges",
    "normalized_deflated", "chain_levels", "chain_product", "chain_apply", "estimate_solution",
    "spectral_radius", "pair_pipeline", "lib",
]

# ---------------------------------------------------------------------------
# The oracle's own C helpers (plain loops, FP64), compiled with gcc.

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cad_oracle.c")
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile oracle/cad_oracle.c into oracle/_build/liboracle.so."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_SO), exist_ok=True)
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build_lib()
        L = ctypes.CDLL(_SO)
        d, i64, u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64
        P = ctypes.c_void_p
        L.orc_mix64.argtypes = [u64]
        L.orc_mix64.restype = u64
        L.orc_sign_word.argtypes = [u64, u64, u64, u64]
        L.orc_sign_word.restype = u64
        L.orc_rhs.argtypes = [P, i64, P, i64, u64, P]
        L.orc_rhs_rows.argtypes = [P, i64, P, i64, u64, P, i64, P]
        L.orc_sq_distances_rows.argtypes = [P, i64, i64, P, i64, P]
        L.orc_scores_rows.argtypes = [P, d, P, d, i64, i64, P, P, P, i64, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Counter-based Rademacher signs (the paper does not say how q is drawn).
#
# mix64 is the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
# The sign word of edge {lo, hi} (global ids, lo < hi) and projection block
# beta = r // 64 is  mix64( mix64(seed) XOR (beta << 40 | lo << 20 | hi) );
# its bit (r mod 64) set means q_r(edge) = -1, clear means +1.

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def sign_words(seed: int, beta, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.uint64)
    hi = np.asarray(hi, dtype=np.uint64)
    if np.any(hi >= (1 << 20)) or np.any(lo >= hi):
        raise ValueError("edge ids must satisfy lo < hi < 2^20")
    beta = np.asarray(beta, dtype=np.uint64)
    key = mix64(np.uint64(seed)) ^ ((beta << np.uint64(40)) | (lo << np.uint64(20)) | hi)
    return mix64(key)


def projection_signs(seed: int, k: int, lo: int, hi: int) -> np.ndarray:
    """q_r(edge {lo,hi}) for r = 0..k-1, as +-1.0."""
    out = np.empty(k)
    for b in range((k + 63) // 64):
        h = int(sign_words(seed, b, lo, hi))
        for r in range(b * 64, min(k, b * 64 + 64)):
            out[r] = -1.0 if (h >> (r % 64)) & 1 else 1.0
    return out


# ---------------------------------------------------------------------------
# Graph construction (Background section; Section "Climate Data").

def sq_distances_rows(X: np.ndarray, rows: Sequence[int]) -> np.ndarray:
    """||x_i - x_j||^2 by direct differences, for i in rows, all j."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), X.shape[0]))
    lib().orc_sq_distances_rows(_ptr(X), X.shape[0], X.shape[1], _ptr(rows),
                                len(rows), _ptr(out))
    return out


def sq_distances(X: np.ndarray) -> np.ndarray:
    """Full n x n matrix of squared Euclidean distances (direct differences)."""
    D2 = sq_distances_rows(X, np.arange(X.shape[0]))
    np.fill_diagonal(D2, 0.0)
    return D2


def bandwidth(D2: np.ndarray) -> float:
    """Lower median of the pair distances sqrt(D2_ij) over i < j.

    The element of 0-based rank floor((N-1)/2) among the N = n(n-1)/2 sorted
    distances.  (The paper fixes sigma by hand for its climate graph; the
    median-distance rule is the reading taken here for synthetic inputs.)
    """
    n = D2.shape[0]
    if n < 2:
        raise ValueError("need at least two nodes")
    iu = np.triu_indices(n, 1)
    vals = np.sqrt(D2[iu])
    r = (vals.size - 1) // 2
    return float(np.partition(vals, r)[r])


def gaussian_weights(D2: np.ndarray, sigma: float) -> np.ndarray:
    """W_ij = exp(-D2_ij / sigma^2) for i != j; W_ii = 0 (no self-edges)."""
    W = np.exp(-D2 / (sigma * sigma))
    np.fill_diagonal(W, 0.0)
    return W


def degrees(W: np.ndarray):
    """deg = W 1 and the volume V_G = sum_i D(i,i) (Background, eq. 1)."""
    deg = W.sum(axis=1)
    if np.any(deg <= 0):
        raise ValueError("graph has a node of zero degree")
    return deg, float(deg.sum())


def laplacian(W: np.ndarray, deg: Optional[np.ndarray] = None) -> np.ndarray:
    """L = D - A (Algorithm 1, first step; Algorithm 2, ChainProduct)."""
    if deg is None:
        deg = W.sum(axis=1)
    return np.diag(deg) - W


def build_graph(X: np.ndarray, sigma: Optional[float] = None):
    """Distances, bandwidth, weights, degrees and volume for one snapshot."""
    D2 = sq_distances(X)
    s = bandwidth(D2) if sigma is None or sigma <= 0 else float(sigma)
    W = gaussian_weights(D2, s)
    deg, vol = degrees(W)
    return dict(D2=D2, sigma=s, W=W, deg=deg, vol=vol)


# ---------------------------------------------------------------------------
# Right-hand sides: y = B^T W^{1/2} q / sqrt(k)  (Algorithm 1; Algorithm 3).
# Edge {a,b} is oriented with its head at the lower global id; the k random
# vectors are the columns r = 0..k-1 of Y, scaled by 1/sqrt(k).

def rhs_numpy(W: np.ndarray, k: int, seed: int, gid=None) -> np.ndarray:
    """Pure-numpy right-hand sides, one row at a time (small n only)."""
    n = W.shape[0]
    gid = np.arange(n, dtype=np.int64) if gid is None else np.asarray(gid, np.int64)
    Y = np.zeros((n, k))
    scale = 1.0 / math.sqrt(k)
    r = np.arange(64, dtype=np.uint64)
    for v in range(n):
        others = np.array([u for u in range(n) if u != v], dtype=np.int64)
        gv, gu = gid[v], gid[others]
        lo, hi = np.minimum(gv, gu), np.maximum(gv, gu)
        inc = np.where(gv < gu, 1.0, -1.0)
        w = np.sqrt(W[v, others]) * scale * inc
        for b in range((k + 63) // 64):
            h = sign_words(seed, b, lo, hi)
            bits = (h[:, None] >> r[None, :]) & np.uint64(1)
            q = 1.0 - 2.0 * bits.astype(np.float64)
            cols = min(64, k - 64 * b)
            Y[v, 64 * b:64 * b + cols] = (w[:, None] * q[:, :cols]).sum(axis=0)
    return Y


def rhs(W: np.ndarray, k: int, seed: int, gid=None) -> np.ndarray:
    """Right-hand sides by the oracle's C loops (same definition)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    n = W.shape[0]
    g = None if gid is None else np.ascontiguousarray(gid, dtype=np.int32)
    if (g is not None and g.max() >= (1 << 20)) or n > (1 << 20):
        raise ValueError("global ids must be below 2^20")
    Y = np.empty((n, k))
    lib().orc_rhs(_ptr(W), n, _ptr(g), k, seed, _ptr(Y))
    return Y


def rhs_rows(W_rows: np.ndarray, rows, k: int, seed: int, gid=None) -> np.ndarray:
    """Rows `rows` of Y, given those rows of W (len(rows) x n)."""
    W_rows = np.ascontiguousarray(W_rows, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = W_rows.shape[1]
    g = None if gid is None else np.ascontiguousarray(gid, dtype=np.int32)
    Y = np.empty((len(rows), k))
    lib().orc_rhs_rows(_ptr(W_rows), n, _ptr(g), k, seed, _ptr(rows), len(rows), _ptr(Y))
    return Y


# ---------------------------------------------------------------------------
# The embedding Z = L^+ Y, directly (what Algorithms 2 and 3 approximate).

def solve_embedding(W: np.ndarray, Y: np.ndarray, deg=None) -> np.ndarray:
    """Z = L^+ Y by Cholesky of L + 1 1^T / n, then column centering.

    For a connected graph L + J/n is positive definite and its inverse is
    L^+ + J/n, so (L + J/n)^{-1} Y = L^+ Y + 1 (1^T Y)/n; removing each
    column's mean leaves L^+ Y, the solution of L z = y orthogonal to 1.
    """
    n = W.shape[0]
    L = laplacian(W, deg)
    L += 1.0 / n
    c = scipy.linalg.cho_factor(L, lower=True, overwrite_a=True, check_finite=False)
    Z = scipy.linalg.cho_solve(c, Y, check_finite=False)
    return Z - Z.mean(axis=0, keepdims=True)


def pinv_laplacian(L: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Moore-Penrose pseudoinverse of L by symmetric eigendecomposition."""
    lam, V = np.linalg.eigh(L)
    keep = lam > rtol * lam[-1]
    return (V[:, keep] / lam[keep]) @ V[:, keep].T


def solve_embedding_eigh(W: np.ndarray, Y: np.ndarray) -> np.ndarray:
    return pinv_laplacian(laplacian(W)) @ Y


# ---------------------------------------------------------------------------
# Commute times and scores (eq. 1; Algorithm 1, last step; Algorithm 4).

def commute_times(Z: np.ndarray, vol: float) -> np.ndarray:
    """c(i,j) = V_G ||z_i - z_j||^2 by direct differences (small n)."""
    diff = Z[:, None, :] - Z[None, :, :]
    return vol * np.einsum("ijk,ijk->ij", diff, diff)


def exact_commute_times(W: np.ndarray) -> np.ndarray:
    """eq. (1): c(i,j) = V_G (l+_ii + l+_jj - 2 l+_ij)."""
    deg = W.sum(axis=1)
    Lp = pinv_laplacian(np.diag(deg) - W)
    d = np.diag(Lp)
    return deg.sum() * (d[:, None] + d[None, :] - 2.0 * Lp)


def scores_rows(Z0, vol0, Z1, vol1, rows, A0_rows=None, A1_rows=None) -> np.ndarray:
    """F_i for i in rows; Z0, Z1 are the m x k embeddings of the common nodes."""
    Z0 = np.ascontiguousarray(Z0, dtype=np.float64)
    Z1 = np.ascontiguousarray(Z1, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m, k = Z0.shape
    if Z1.shape != (m, k):
        raise ValueError("embeddings must cover the same nodes")
    A0r = None if A0_rows is None else np.ascontiguousarray(A0_rows, dtype=np.float64)
    A1r = None if A1_rows is None else np.ascontiguousarray(A1_rows, dtype=np.float64)
    F = np.empty(len(rows))
    lib().orc_scores_rows(_ptr(Z0), vol0, _ptr(Z1), vol1, m, k, _ptr(A0r), _ptr(A1r),
                          _ptr(rows), len(rows), _ptr(F))
    return F


def scores(Z0, vol0, Z1, vol1, W0=None, W1=None, map0=None, map1=None) -> np.ndarray:
    """Node scores F_i = sum_j omega_ij |c0(i,j) - c1(i,j)| (Algorithm 4).

    map0/map1 select the common nodes (row indices into Z0/Z1, same length);
    omega = |A1 - A0| on those nodes when W0 and W1 are given, else 1.
    """
    if map0 is not None:
        Z0 = Z0[map0]
        Z1 = Z1[map1]
        if W0 is not None:
            W0 = W0[np.ix_(map0, map0)]
            W1 = W1[np.ix_(map1, map1)]
    m = Z0.shape[0]
    return scores_rows(Z0, vol0, Z1, vol1, np.arange(m), W0, W1)


def edge_scores(Z0, vol0, Z1, vol1, W0=None, W1=None, map0=None, map1=None,
                block: int = 64) -> np.ndarray:
    """The m x m matrix of CAD edge scores omega_ab |c_0(a,b) - c_1(a,b)|.

    c_t(a,b) = vol_t ||z_a - z_b||^2 by direct differences (Background, the
    edge score whose row sums are Algorithm 4's node scores); omega = 1, or
    |A1 - A0| on the common nodes when W0 and W1 are given.  Diagonal 0.
    """
    if map0 is not None:
        Z0, Z1 = Z0[map0], Z1[map1]
        if W0 is not None:
            W0 = W0[np.ix_(map0, map0)]
            W1 = W1[np.ix_(map1, map1)]
    m = Z0.shape[0]
    E = np.empty((m, m))
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        c0 = vol0 * ((Z0[r0:r1, None, :] - Z0[None, :, :]) ** 2).sum(axis=2)
        c1 = vol1 * ((Z1[r0:r1, None, :] - Z1[None, :, :]) ** 2).sum(axis=2)
        e = np.abs(c0 - c1)
        if W0 is not None:
            e *= np.abs(W1[r0:r1] - W0[r0:r1])
        E[r0:r1] = e
    np.fill_diagonal(E, 0.0)
    return E


def top_edges(E: np.ndarray, K: int):
    """The K largest entries of the upper triangle (a < b) of E, ordered by
    value descending, then a, then b.  Returns (a, b, value)."""
    a, b = np.triu_indices(E.shape[0], 1)
    v = E[a, b]
    order = np.lexsort((b, a, -v))[:K]
    return a[order].astype(np.int32), b[order].astype(np.int32), v[order]


def top_k(F: np.ndarray, K: int) -> np.ndarray:
    """Indices of the K largest scores, ties broken by the lower index."""
    order = np.lexsort((np.arange(F.size), -F))
    return order[:min(K, F.size)].astype(np.int32)


# ---------------------------------------------------------------------------
# Inverse chain (eq. inverse-chain; Algorithm 2), for checking GPU levels.
# Readings: the undefined factor C in P is D^{-1/2}; the eigenvalue-1 mode of
# S (eigenvector u = D^{1/2} 1 / sqrt(V_G)) is removed before squaring (the
# chain only acts on vectors orthogonal to u); d counts stored levels
# S, S^2, ..., S^{2^{d-1}}.

def normalized_deflated(W: np.ndarray, deg: np.ndarray, vol: float,
                        lazy: bool = False) -> np.ndarray:
    """S~ = D^{-1/2} A D^{-1/2} - u u^T  (lazy: (I + S)/2 - u u^T)."""
    s = 1.0 / np.sqrt(deg)
    S = s[:, None] * W * s[None, :]
    if lazy:
        S = 0.5 * (np.eye(W.shape[0]) + S)
    u = np.sqrt(deg / vol)
    return S - np.outer(u, u)


def chain_levels(St: np.ndarray, d: int) -> List[np.ndarray]:
    """[S~, S~^2, S~^4, ..., S~^{2^{d-1}}] by repeated squaring."""
    levels = [St]
    for _ in range(d - 1):
        levels.append(levels[-1] @ levels[-1])
    return levels


def chain_product(levels: List[np.ndarray]) -> np.ndarray:
    """P = prod_l (I + S~_l), the dense factor of ChainProduct (Algorithm 2)
    before the outer D^{-1/2} factors, multiplied in level order."""
    n = levels[0].shape[0]
    P = np.eye(n)
    for S in levels:
        P = P @ (np.eye(n) + S)
    return P


def chain_apply(levels: List[np.ndarray], deg: np.ndarray, R: np.ndarray,
                lazy: bool = False) -> np.ndarray:
    """P1 R = D^{-1/2} prod_l (I + S~_l) D^{-1/2} R  (lazy: 2D for D)."""
    dm = 1.0 / np.sqrt((2.0 if lazy else 1.0) * deg)
    V = dm[:, None] * R
    for S in levels:
        V = V + S @ V
    return dm[:, None] * V


def estimate_solution(W: np.ndarray, deg: np.ndarray, Y: np.ndarray,
                      levels: List[np.ndarray], q: int, lazy: bool = False) -> np.ndarray:
    """EstimateSolution: y_1 = 0; y_{k+1} = y_k - P2 y_k + chi, k = 1..q-1,

    with chi = P1 b and P2 = P1 L applied as y + P1 (b - L y) (P2 is never
    formed).  Returns y_q.
    """
    L = laplacian(W, deg)
    y = np.zeros_like(Y)
    for _ in range(q - 1):
        y = y + chain_apply(levels, deg, Y - L @ y, lazy)
    return y


def spectral_radius(St: np.ndarray) -> float:
    lam = np.linalg.eigvalsh(St)
    return float(max(abs(lam[0]), abs(lam[-1])))


# ---------------------------------------------------------------------------

def pair_pipeline(X0: np.ndarray, X1: np.ndarray, k: int, seed: int,
                  sigma: Optional[float] = None, weighted: bool = False,
                  top: int = 50):
    """The whole path for one graph pair, by the oracle's definitions."""
    out = {}
    for t, X in ((0, X0), (1, X1)):
        g = build_graph(X, sigma)
        Y = rhs(g["W"], k, seed)
        Z = solve_embedding(g["W"], Y, g["deg"])
        out[t] = dict(g, Y=Y, Z=Z)
    F = scores(out[0]["Z"], out[0]["vol"], out[1]["Z"], out[1]["vol"],
               out[0]["W"] if weighted else None, out[1]["W"] if weighted else None)
    out["F"] = F
    out["top"] = top_k(F, top)
    return out
