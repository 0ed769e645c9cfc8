"""Pins for the CPU oracle: closed forms, invariants, brute force and library
routines that fix what the oracle must compute (no GPU needed).

Each test names the fact it checks.  A plausible slip in the oracle (a dropped
term, a flipped sign or orientation, a wrong scale, a transposed operand)
fails at least one of them.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.spatial.distance as ssd

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_dense_graph(n, seed, lo=0.05, hi=1.0):
    rng = np.random.default_rng(seed)
    A = rng.uniform(lo, hi, size=(n, n))
    A = np.triu(A, 1)
    return A + A.T


def edge_embedding(W, gid=None):
    """Full edge-space embedding Z = L^+ B^T W^{1/2} (k = m, q = identity)."""
    n = W.shape[0]
    gid = np.arange(n) if gid is None else np.asarray(gid)
    edges = [(a, b) for a in range(n) for b in range(a + 1, n)]
    B = np.zeros((len(edges), n))
    for e, (a, b) in enumerate(edges):
        head, tail = (a, b) if gid[a] < gid[b] else (b, a)
        B[e, head] = 1.0
        B[e, tail] = -1.0
    w = np.array([W[a, b] for (a, b) in edges])
    Lp = oracle.pinv_laplacian(oracle.laplacian(W))
    return Lp @ (B.T * np.sqrt(w)[None, :]), B, w, edges


# --------------------------------------------------------------- signs / RNG

def test_splitmix64_published_outputs():
    vals = [int(line, 16) for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if line.strip() and not line.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    got = [int(oracle.mix64(np.uint64((gamma * (i + 1)) % 2**64))) for i in range(len(vals))]
    assert got == vals
    assert [oracle.lib().orc_mix64((gamma * (i + 1)) % 2**64) for i in range(len(vals))] == vals


def test_sign_words_match_between_numpy_and_c():
    L = oracle.lib()
    rng = np.random.default_rng(0)
    for _ in range(200):
        lo, hi = sorted(rng.choice(1 << 20, size=2, replace=False).tolist())
        beta = int(rng.integers(0, 1 << 24))
        seed = int(rng.integers(0, 2**63))
        assert int(oracle.sign_words(seed, beta, lo, hi)) == L.orc_sign_word(seed, beta, lo, hi)


def test_sign_statistics():
    # Rademacher signs: each bit is a fair coin, bits of one word and words of
    # neighbouring edges are uncorrelated.
    n = 256
    a, b = np.triu_indices(n, 1)
    h = oracle.sign_words(7, 0, a, b)
    bits = ((h[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(float)
    N = bits.shape[0]
    p = bits.mean(axis=0)
    assert np.all(np.abs(p - 0.5) < 5 * 0.5 / math.sqrt(N))
    q = 1 - 2 * bits
    C = (q.T @ q) / N
    off = C[~np.eye(64, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / math.sqrt(N)
    h1 = oracle.sign_words(7, 1, a, b)
    bits1 = ((h1[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(float)
    cross = ((1 - 2 * bits1).T @ q) / N
    assert np.max(np.abs(cross)) < 5 / math.sqrt(N)


def test_sign_words_reject_bad_edges():
    with pytest.raises(ValueError):
        oracle.sign_words(1, 0, 5, 5)
    with pytest.raises(ValueError):
        oracle.sign_words(1, 0, 3, 1 << 20)


# ------------------------------------------------- commute times, closed forms

@pytest.mark.parametrize("n", [3, 5, 16, 64])
def test_complete_graph(n):
    W = np.ones((n, n)) - np.eye(n)
    C = oracle.exact_commute_times(W)
    off = ~np.eye(n, dtype=bool)
    # K_n: effective resistance 2/n, volume n(n-1), commute time 2(n-1)
    np.testing.assert_allclose(C[off], 2.0 * (n - 1), rtol=1e-12)
    np.testing.assert_allclose(np.diag(C), 0.0, atol=1e-9)
    if n <= 16:
        Z, *_ = edge_embedding(W)
        D = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
        np.testing.assert_allclose(D[off], 2.0 / n, rtol=1e-12)


def test_weighted_path():
    w = np.array([0.5, 2.0, 1.25, 4.0, 0.1])
    n = len(w) + 1
    W = np.zeros((n, n))
    for i, wi in enumerate(w):
        W[i, i + 1] = W[i + 1, i] = wi
    R = oracle.exact_commute_times(W) / (2 * w.sum())
    for i in range(n):
        for j in range(i + 1, n):
            np.testing.assert_allclose(R[i, j], np.sum(1.0 / w[i:j]), rtol=1e-11)


def test_cycle():
    n = 9
    W = np.zeros((n, n))
    for i in range(n):
        W[i, (i + 1) % n] = W[(i + 1) % n, i] = 1.0
    R = oracle.exact_commute_times(W) / (2 * n)
    for i in range(n):
        for j in range(n):
            l = (j - i) % n
            np.testing.assert_allclose(R[i, j], l * (n - l) / n, atol=1e-12)


def test_foster_theorem():
    n = 12
    W = random_dense_graph(n, 3)
    C = oracle.exact_commute_times(W)
    R = C / W.sum()
    iu = np.triu_indices(n, 1)
    np.testing.assert_allclose((W[iu] * R[iu]).sum(), n - 1, rtol=1e-12)


def _det_fraction(M):
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for cc in range(c, n):
                M[r][cc] -= f * M[c][cc]
    return det


@pytest.mark.parametrize("n,seed", [(3, 0), (4, 1), (5, 2), (6, 3)])
def test_matrix_tree_resistance_exact(n, seed):
    # Kirchhoff: R_ij = det L_{-i-j} / det L_{-i}, in exact rationals.
    rng = np.random.default_rng(seed)
    Wi = np.triu(rng.integers(1, 6, size=(n, n)), 1)
    Wi = Wi + Wi.T
    Lf = [[Fraction(int(-Wi[r, c])) if r != c else Fraction(int(Wi[r].sum()))
           for c in range(n)] for r in range(n)]
    C = oracle.exact_commute_times(Wi.astype(float))
    vol = Wi.sum()
    for i in range(n):
        keep_i = [r for r in range(n) if r != i]
        den = _det_fraction([[Lf[r][c] for c in keep_i] for r in keep_i])
        for j in range(n):
            if j == i:
                continue
            keep = [r for r in range(n) if r not in (i, j)]
            num = _det_fraction([[Lf[r][c] for c in keep] for r in keep]) if keep else Fraction(1)
            assert abs(C[i, j] - float(vol * num / den)) <= 1e-11 * abs(C[i, j])


def test_hitting_times():
    # commute time = H(i,j) + H(j,i) for the random walk P = D^-1 A.
    n = 7
    W = random_dense_graph(n, 5)
    P = W / W.sum(axis=1, keepdims=True)
    H = np.zeros((n, n))
    for j in range(n):
        idx = [i for i in range(n) if i != j]
        M = np.eye(n - 1) - P[np.ix_(idx, idx)]
        H[idx, j] = np.linalg.solve(M, np.ones(n - 1))
    C = oracle.exact_commute_times(W)
    np.testing.assert_allclose(C, H + H.T, rtol=1e-10, atol=1e-10)


def test_commute_time_scale_invariance_and_metric():
    W = random_dense_graph(10, 8)
    C = oracle.exact_commute_times(W)
    np.testing.assert_allclose(oracle.exact_commute_times(3.7 * W), C, rtol=1e-11)
    np.testing.assert_allclose(C, C.T, atol=1e-9)
    R = C / W.sum()
    assert np.all(R[~np.eye(10, dtype=bool)] > 0)
    # effective resistance is a metric
    for i in range(10):
        for j in range(10):
            assert np.all(R[i, j] <= R[i, :] + R[:, j] + 1e-12)


def test_cholesky_and_eigh_routes_agree():
    n = 40
    W = random_dense_graph(n, 9)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((n, 5))
    Y -= Y.mean(axis=0)
    Z1 = oracle.solve_embedding(W, Y)
    Z2 = oracle.solve_embedding_eigh(W, Y)
    np.testing.assert_allclose(Z1, Z2, rtol=0, atol=1e-12 * np.abs(Z2).max())
    # residual certificate and gauge
    L = oracle.laplacian(W)
    assert np.abs(L @ Z1 - Y).max() < 1e-12 * np.abs(Y).max()
    np.testing.assert_allclose(Z1.sum(axis=0), 0, atol=1e-12)


def test_complete_graph_embedding_closed_form():
    # K_n: L^+ = (I - J/n)/n, so Z = (Y - mean)/n.
    n = 30
    W = np.ones((n, n)) - np.eye(n)
    Y = oracle.rhs(W, 16, 3)
    Z = oracle.solve_embedding(W, Y)
    np.testing.assert_allclose(Z, (Y - Y.mean(axis=0)) / n, atol=1e-15)


# ----------------------------------------------------------- right-hand sides

@pytest.mark.parametrize("n,k,perm", [(5, 3, False), (9, 70, True), (12, 64, True)])
def test_rhs_equals_literal_incidence_form(n, k, perm):
    # y = B^T W^{1/2} q / sqrt(k) with explicit m x n incidence B (head = lower
    # global id), diagonal W over the edges and k random edge vectors.
    W = random_dense_graph(n, n)
    rng = np.random.default_rng(k)
    gid = rng.permutation(50)[:n].astype(np.int32) if perm else np.arange(n, dtype=np.int32)
    _, B, w, edges = edge_embedding(W, gid)
    Q = np.stack([oracle.projection_signs(11, k, min(gid[a], gid[b]), max(gid[a], gid[b]))
                  for (a, b) in edges])                       # m x k
    Y_lit = B.T @ (np.sqrt(w)[:, None] * Q) / math.sqrt(k)
    np.testing.assert_allclose(oracle.rhs(W, k, 11, gid), Y_lit, rtol=0, atol=1e-14)
    np.testing.assert_allclose(oracle.rhs_numpy(W, k, 11, gid), Y_lit, rtol=0, atol=1e-14)
    # every column sums to zero (each edge adds +s and -s)
    np.testing.assert_allclose(Y_lit.sum(axis=0), 0, atol=1e-13)
    rows = np.array([n - 1, 0, n // 2])
    np.testing.assert_allclose(oracle.rhs_rows(W[rows], rows, k, 11, gid), Y_lit[rows],
                               rtol=0, atol=1e-14)


def test_rhs_unbiased_effective_resistance():
    # E ||z_i - z_j||^2 = R_ij  (Algorithm 1 estimates resistances).
    n, k, S = 8, 64, 300
    W = random_dense_graph(n, 21)
    C = oracle.exact_commute_times(W)
    R = C / W.sum()
    acc = np.zeros((S, n, n))
    for s in range(S):
        Z = oracle.solve_embedding(W, oracle.rhs(W, k, 1000 + s))
        acc[s] = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    mean = acc.mean(axis=0)
    se = acc.std(axis=0) / math.sqrt(S)
    off = ~np.eye(n, dtype=bool)
    assert np.all(np.abs(mean[off] - R[off]) < 4.5 * se[off])
    # the spread matches the Rademacher projection variance ~ 2 R^2 / k
    rel_sd = (acc.std(axis=0)[off] / R[off]).mean()
    assert 0.5 * math.sqrt(2 / k) < rel_sd < 1.5 * math.sqrt(2 / k)


# ----------------------------------------------------------------- the graph

def test_sq_distances_match_library_and_brute_force():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((37, 13))
    D2 = oracle.sq_distances(X)
    np.testing.assert_allclose(D2, ssd.squareform(ssd.pdist(X, "sqeuclidean")), rtol=1e-13, atol=1e-13)
    i, j = 3, 30
    assert abs(D2[i, j] - sum((X[i, t] - X[j, t]) ** 2 for t in range(13))) < 1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 17, 50])
def test_bandwidth_is_lower_median(n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 6))
    D2 = oracle.sq_distances(X)
    s = oracle.bandwidth(D2)
    vals = np.sort(ssd.pdist(X))
    assert s == pytest.approx(vals[(len(vals) - 1) // 2], rel=1e-14)
    W = oracle.gaussian_weights(D2, s)
    # the median pair's weight is exp(-1) by construction
    iu = np.triu_indices(n, 1)
    wv = np.sort(W[iu])[::-1]
    assert wv[(len(wv) - 1) // 2] == pytest.approx(math.exp(-1), rel=1e-12)


def test_weights_properties():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((30, 20))
    g = oracle.build_graph(X)
    W = g["W"]
    assert np.all(np.diag(W) == 0)
    np.testing.assert_array_equal(W, W.T)
    off = W[~np.eye(30, dtype=bool)]
    assert np.all((off > 0) & (off <= 1))
    np.testing.assert_allclose(g["deg"], W.sum(1), rtol=1e-15)
    assert g["vol"] == pytest.approx(W.sum(), rel=1e-14)
    with pytest.raises(ValueError):
        oracle.degrees(np.zeros((3, 3)))


# -------------------------------------------------------------------- scores

def test_scores_zero_for_identical_snapshots():
    W = random_dense_graph(20, 1)
    Z = oracle.solve_embedding(W, oracle.rhs(W, 8, 1))
    F = oracle.scores(Z, 5.0, Z, 5.0)
    assert np.all(F == 0)


def test_scores_with_exact_embeddings_equal_eq1():
    # With the full edge-space embedding, ||z_i - z_j||^2 = R_ij exactly, so the
    # scores built from Z equal those built from eq. (1)'s commute times.
    n = 9
    W0 = random_dense_graph(n, 30)
    W1 = random_dense_graph(n, 31)
    Z0, *_ = edge_embedding(W0)
    Z1, *_ = edge_embedding(W1)
    C0, C1 = oracle.exact_commute_times(W0), oracle.exact_commute_times(W1)
    F = oracle.scores(Z0, W0.sum(), Z1, W1.sum())
    np.testing.assert_allclose(F, np.abs(C0 - C1).sum(axis=1), rtol=1e-11)
    Fw = oracle.scores(Z0, W0.sum(), Z1, W1.sum(), W0, W1)
    np.testing.assert_allclose(Fw, (np.abs(W1 - W0) * np.abs(C0 - C1)).sum(axis=1), rtol=1e-11)


def test_embedding_commute_times_equal_eq1():
    # Algorithm 1's embedding form vol * ||z_i - z_j||^2 with the full
    # edge-space embedding (||z_i - z_j||^2 = R_ij exactly) against eq. (1)
    # and, on K_n, against the closed form c = 2 (n - 1).
    W = random_dense_graph(8, 40)
    Z, *_ = edge_embedding(W)
    C = oracle.commute_times(Z, W.sum())
    np.testing.assert_allclose(C, oracle.exact_commute_times(W), rtol=1e-11, atol=1e-11)
    assert np.all(np.diag(C) == 0.0)
    n = 7
    Kn = np.ones((n, n)) - np.eye(n)
    Zk, *_ = edge_embedding(Kn)
    Ck = oracle.commute_times(Zk, Kn.sum())
    off = ~np.eye(n, dtype=bool)
    np.testing.assert_allclose(Ck[off], 2.0 * (n - 1), rtol=1e-12)


def test_edge_scores_sum_to_node_scores():
    # Algorithm 4's node score is the row sum of the edge scores; the two are
    # computed independently (direct differences here, the C row loops for
    # the node scores).
    n = 40
    W0 = random_dense_graph(n, 50)
    W1 = random_dense_graph(n, 51)
    Z0 = oracle.solve_embedding(W0, oracle.rhs(W0, 12, 4))
    Z1 = oracle.solve_embedding(W1, oracle.rhs(W1, 12, 4))
    E = oracle.edge_scores(Z0, W0.sum(), Z1, W1.sum())
    np.testing.assert_allclose(E, E.T, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(E.sum(axis=1), oracle.scores(Z0, W0.sum(), Z1, W1.sum()), rtol=1e-12)
    Ew = oracle.edge_scores(Z0, W0.sum(), Z1, W1.sum(), W0, W1)
    np.testing.assert_allclose(Ew.sum(axis=1), oracle.scores(Z0, W0.sum(), Z1, W1.sum(), W0, W1), rtol=1e-12)
    perm = np.random.default_rng(1).permutation(n)[:25]
    Em = oracle.edge_scores(Z0, W0.sum(), Z1, W1.sum(), map0=perm, map1=perm)
    np.testing.assert_allclose(Em, E[np.ix_(perm, perm)], rtol=1e-13, atol=1e-12)


def test_edge_scores_with_exact_embeddings_equal_eq1():
    n = 9
    W0 = random_dense_graph(n, 60)
    W1 = random_dense_graph(n, 61)
    Z0, *_ = edge_embedding(W0)
    Z1, *_ = edge_embedding(W1)
    C0, C1 = oracle.exact_commute_times(W0), oracle.exact_commute_times(W1)
    E = oracle.edge_scores(Z0, W0.sum(), Z1, W1.sum())
    np.testing.assert_allclose(E, np.abs(C0 - C1), rtol=1e-10, atol=1e-10)


def test_top_edges_order_and_ties():
    E = np.zeros((5, 5))
    E[1, 3] = E[3, 1] = 2.0
    E[0, 4] = E[4, 0] = 2.0
    E[2, 3] = E[3, 2] = 5.0
    a, b, v = oracle.top_edges(E, 4)
    assert list(zip(a.tolist(), b.tolist())) == [(2, 3), (0, 4), (1, 3), (0, 1)]
    assert v.tolist() == [5.0, 2.0, 2.0, 0.0]


def test_weighted_scores_single_changed_edge():
    # Only one edge changes weight: only its two end nodes score, equally.
    n = 10
    W0 = random_dense_graph(n, 40)
    W1 = W0.copy()
    W1[2, 7] = W1[7, 2] = W0[2, 7] + 0.8
    Z0 = oracle.solve_embedding(W0, oracle.rhs(W0, 16, 3))
    Z1 = oracle.solve_embedding(W1, oracle.rhs(W1, 16, 3))
    F = oracle.scores(Z0, W0.sum(), Z1, W1.sum(), W0, W1)
    nz = np.flatnonzero(F)
    assert set(nz.tolist()) == {2, 7}
    c0 = W0.sum() * ((Z0[2] - Z0[7]) ** 2).sum()
    c1 = W1.sum() * ((Z1[2] - Z1[7]) ** 2).sum()
    assert F[2] == pytest.approx(0.8 * abs(c0 - c1), rel=1e-12)
    assert F[7] == pytest.approx(F[2], rel=1e-12)


def test_scores_permutation_equivariant_and_maps():
    n = 15
    W0, W1 = random_dense_graph(n, 50), random_dense_graph(n, 51)
    Z0 = oracle.solve_embedding(W0, oracle.rhs(W0, 8, 2))
    Z1 = oracle.solve_embedding(W1, oracle.rhs(W1, 8, 2))
    F = oracle.scores(Z0, 3.0, Z1, 4.0)
    p = np.random.default_rng(0).permutation(n)
    np.testing.assert_allclose(oracle.scores(Z0[p], 3.0, Z1[p], 4.0), F[p], rtol=1e-13)
    # maps pick common nodes: identity maps reproduce the plain scores
    np.testing.assert_allclose(oracle.scores(Z0, 3.0, Z1, 4.0, map0=np.arange(n), map1=np.arange(n)), F)
    sub = np.array([1, 4, 9])
    Fs = oracle.scores(Z0, 3.0, Z1, 4.0, map0=sub, map1=sub)
    np.testing.assert_allclose(Fs, oracle.scores(Z0[sub], 3.0, Z1[sub], 4.0))


def test_top_k_tie_break():
    F = np.array([1.0, 3.0, 3.0, 2.0, 3.0, 0.5])
    np.testing.assert_array_equal(oracle.top_k(F, 4), [1, 2, 4, 3])
    np.testing.assert_array_equal(oracle.top_k(F, 10), [1, 2, 4, 3, 0, 5])


# --------------------------------------------------------------- inverse chain

def test_chain_complete_graph_closed_form():
    n = 12
    W = np.ones((n, n)) - np.eye(n)
    deg, vol = oracle.degrees(W)
    St = oracle.normalized_deflated(W, deg, vol)
    Pi = np.eye(n) - 1.0 / n
    np.testing.assert_allclose(St, -Pi / (n - 1), atol=1e-16)
    lev = oracle.chain_levels(St, 4)
    for l in range(1, 4):
        np.testing.assert_allclose(lev[l], Pi / (n - 1) ** (2 ** l), atol=1e-16)


def test_chain_product_telescopes():
    # prod_{l<d} (I + S^{2^l}) = sum_{j < 2^d} S^j = V diag((1-lam^{2^d})/(1-lam)) V^T
    n, d = 20, 3
    W = random_dense_graph(n, 60)
    deg, vol = oracle.degrees(W)
    St = oracle.normalized_deflated(W, deg, vol)
    lev = oracle.chain_levels(St, d)
    P = oracle.chain_product(lev)
    lam, V = np.linalg.eigh(St)
    np.testing.assert_allclose(P, (V * ((1 - lam ** (2 ** d)) / (1 - lam))) @ V.T, atol=1e-13)
    u = np.sqrt(deg / vol)
    np.testing.assert_allclose(St @ u, 0, atol=1e-15)
    assert oracle.spectral_radius(St) < 1


@pytest.mark.parametrize("lazy", [False, True])
def test_chain_preconditioner_converges_to_pseudoinverse(lazy):
    n = 30
    W = random_dense_graph(n, 70)
    deg, vol = oracle.degrees(W)
    St = oracle.normalized_deflated(W, deg, vol, lazy=lazy)
    Y = oracle.rhs(W, 6, 4)
    Zx = oracle.solve_embedding(W, Y)
    X = oracle.chain_apply(oracle.chain_levels(St, 10), deg, Y, lazy=lazy)
    # the chain solves in the gauge deg^T x = 0; centring gives L^+ Y
    np.testing.assert_allclose(deg @ X, 0, atol=1e-12)
    np.testing.assert_allclose(X - X.mean(axis=0), Zx, atol=1e-13)
    # Richardson from a short chain reaches the same solution
    Z10 = oracle.estimate_solution(W, deg, Y, oracle.chain_levels(St, 2), q=12, lazy=lazy)
    np.testing.assert_allclose(Z10 - Z10.mean(axis=0), Zx, atol=1e-12)


def test_lazy_chain_handles_bipartite_graph():
    # path graph: eigenvalue -1 of S makes the plain chain useless; lazy works
    n = 6
    W = np.zeros((n, n))
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1.0
    deg, vol = oracle.degrees(W)
    assert oracle.spectral_radius(oracle.normalized_deflated(W, deg, vol)) == pytest.approx(1.0)
    St = oracle.normalized_deflated(W, deg, vol, lazy=True)
    assert oracle.spectral_radius(St) < 1
    Y = oracle.rhs(W + 0.0, 4, 1)
    Zx = oracle.solve_embedding(W, Y)
    Z = oracle.estimate_solution(W, deg, Y, oracle.chain_levels(St, 6), q=40, lazy=True)
    np.testing.assert_allclose(Z - Z.mean(axis=0), Zx, atol=1e-10)
