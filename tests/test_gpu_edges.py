"""Edge-level anomalies (the CAD edge score of the Background section): the
top-K edges a < b by omega |c_0(a,b) - c_1(a,b)|, against the oracle's full
edge-score matrix on the same seeded inputs."""

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def series(n, T, seed):
    return np.random.default_rng(seed).standard_normal((n, T)) * 1.3 + 0.2


def embed(cdl, X, k, seed=3):
    g = cdl.build_graph(dev(X))
    ch = cdl.build_chain(g, prec="fp64", depth=0, depth_max=6)
    Z, _ = cdl.solve_embedding(g, ch, k, seed, tol=1e-12, max_iter=40)
    o = oracle.build_graph(X)
    Zo = oracle.solve_embedding(o["W"], oracle.rhs(o["W"], k, seed), o["deg"])
    return g, Z, o, Zo


def check(a, b, v, want, K):
    wa, wb, wv = want
    np.testing.assert_allclose(v, wv, rtol=1e-8, atol=1e-12 * max(1.0, abs(wv[0])))
    # the pairs must agree wherever the oracle's values are not near-ties
    for q in range(K):
        close = np.abs(wv - wv[q]) <= 1e-8 * abs(wv[0]) + 1e-14
        if close.sum() == 1:
            assert (a[q], b[q]) == (wa[q], wb[q]), q
    assert np.all(a < b) and np.all(np.diff(v) <= 0)


@pytest.mark.parametrize("mode", ["unweighted", "delta_a"])
@pytest.mark.parametrize("K", [1, 7, 50, 256])
def test_top_edges_match_oracle(cdl, mode, K):
    n, k = 300, 32
    X0, X1 = series(n, 30, 11), series(n, 30, 12)
    g0, Z0, o0, Zo0 = embed(cdl, X0, k)
    g1, Z1, o1, Zo1 = embed(cdl, X1, k)
    print("edges n=%d K=%d mode=%s" % (n, K, mode), flush=True)
    F, a, b, v = cdl.anomaly_edges(Z0, g0, Z1, g1, top_k=K, mode=mode)
    w = mode == "delta_a"
    E = oracle.edge_scores(Zo0, o0["vol"], Zo1, o1["vol"], o0["W"] if w else None, o1["W"] if w else None)
    check(host(a), host(b), host(v), oracle.top_edges(E, K), K)
    # the node scores are the row sums of the edge scores
    Fn, _ = cdl.anomaly_scores(Z0, g0, Z1, g1, mode=mode, top_k=0)
    np.testing.assert_array_equal(host(F), host(Fn))
    np.testing.assert_allclose(host(F), E.sum(axis=1), rtol=1e-8)


def test_top_edges_with_maps(cdl):
    k = 24
    X0, X1 = series(260, 20, 21), series(280, 20, 22)
    g0, Z0, o0, Zo0 = embed(cdl, X0, k)
    g1, Z1, o1, Zo1 = embed(cdl, X1, k)
    rng = np.random.default_rng(5)
    m0 = rng.choice(260, 150, replace=False).astype(np.int32)
    m1 = rng.choice(280, 150, replace=False).astype(np.int32)
    F, a, b, v = cdl.anomaly_edges(Z0, g0, Z1, g1, top_k=40, map0=dev(m0), map1=dev(m1))
    E = oracle.edge_scores(Zo0, o0["vol"], Zo1, o1["vol"], map0=m0, map1=m1)
    check(host(a), host(b), host(v), oracle.top_edges(E, 40), 40)


def test_all_ties_give_the_first_pairs(cdl):
    # Weighted mode with equal weight matrices: every edge score is exactly 0,
    # so the top edges are the lexicographically first pairs.
    n, k = 200, 16
    X = series(n, 20, 31)
    g, Z, _, _ = embed(cdl, X, k)
    F, a, b, v = cdl.anomaly_edges(Z, g, Z, g, top_k=20, mode="delta_a")
    assert np.all(host(v) == 0.0)
    want = [(0, j) for j in range(1, 21)]
    assert list(zip(host(a).tolist(), host(b).tolist())) == want


def test_top_edges_many_tiles(cdl):
    # 2000 nodes: 16 x 16 tiles of 128, 136 upper tiles; K = 256 > tiles in
    # a row band, so the threshold comes from many tiles.
    k = 16
    p = gen.make_pair(G=45, T=60, patches=2, patch_size=3)
    X0, X1 = p.X0[:2000], p.X1[:2000]
    g0, Z0, o0, Zo0 = embed(cdl, X0, k)
    g1, Z1, o1, Zo1 = embed(cdl, X1, k)
    F, a, b, v = cdl.anomaly_edges(Z0, g0, Z1, g1, top_k=256)
    E = oracle.edge_scores(Zo0, o0["vol"], Zo1, o1["vol"])
    check(host(a), host(b), host(v), oracle.top_edges(E, 256), 256)
