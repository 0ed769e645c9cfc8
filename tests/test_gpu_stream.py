"""Streamed snapshots (cdl_stream_embedding): no n x n matrix is ever stored;
the weights are recomputed from the series, row panel by row panel, on every
sweep.

Checked against the oracle over the whole snapshot (ragged sizes, several
panels), against the stored path on the GPU (the same bandwidth bits, the
same degrees and embeddings to rounding), and for independence of the panel
size (bit-identical results).
"""

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

SEED = gen.grid.PROJ_SEED


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def series(n, T, seed):
    return np.random.default_rng(seed).standard_normal((n, T)) * 1.3 + 0.2


@pytest.mark.parametrize("n,T,k,panel", [(300, 37, 5, 0), (513, 240, 70, 256),
                                         (1100, 50, 130, 512)])
def test_stream_matches_oracle(cdl, n, T, k, panel):
    X = series(n, T, n + 7 * T)
    print("stream case n=%d T=%d k=%d panel=%d" % (n, T, k, panel), flush=True)
    g, Z, info = cdl.stream_embedding(dev(X), k, SEED, tol=1e-11, max_iter=30, panel_rows=panel)
    o = oracle.build_graph(X)
    s = g.host_stats()
    assert s["sigma"] == pytest.approx(o["sigma"], rel=1e-12)
    np.testing.assert_allclose(host(g.deg), o["deg"], rtol=1e-12)
    assert s["vol"] == pytest.approx(o["vol"], rel=1e-12)
    assert s["deg_min"] == pytest.approx(o["deg"].min(), rel=1e-12)
    Y = oracle.rhs(o["W"], k, SEED)
    Zo = oracle.solve_embedding(o["W"], Y, o["deg"])
    e = rel(host(Z), Zo)
    print("  iterations %d residual %.2e e_Z %.2e" % (info.iterations, info.rel_residual, e))
    assert info.converged and info.rel_residual <= 1e-11
    assert all(info.depth_used[i] == 1 for i in range(info.iterations))
    assert e <= 1e-9


@pytest.mark.parametrize("perm", [False, True])
def test_stream_global_ids(cdl, perm):
    n, T, k = 600, 24, 70
    X = series(n, T, 5 + perm)
    rng = np.random.default_rng(n + perm)
    gid = (rng.permutation(9000)[:n] if perm else np.sort(rng.choice(9000, n, replace=False)))
    gid = gid.astype(np.int32)
    g, Z, info = cdl.stream_embedding(dev(X), k, 1234, gid=dev(gid), tol=1e-11, panel_rows=256)
    o = oracle.build_graph(X)
    Zo = oracle.solve_embedding(o["W"], oracle.rhs(o["W"], k, 1234, gid))
    Zg = host(Z)
    e = rel(Zg, Zo)
    print("  perm=%s iterations %d e_Z %.2e" % (perm, info.iterations, e))
    assert info.converged and e <= 1e-9
    np.testing.assert_allclose(Zg.sum(axis=0), 0, atol=1e-12 * np.abs(Zg).max() * n)


def test_stream_given_sigma_and_certified_tolerance(cdl):
    n, T, k = 700, 19, 64
    X = series(n, T, 3)
    o = oracle.build_graph(X)
    sigma = 0.8 * o["sigma"]
    g, Z, info = cdl.stream_embedding(dev(X), k, SEED, sigma=sigma, tol=-1e-7, panel_rows=256)
    assert g.host_stats()["sigma"] == sigma
    ob = oracle.build_graph(X, sigma=sigma)
    np.testing.assert_allclose(host(g.deg), ob["deg"], rtol=1e-12)
    Zo = oracle.solve_embedding(ob["W"], oracle.rhs(ob["W"], k, SEED), ob["deg"])
    e = rel(host(Z), Zo)
    print("  certified %.2e (kappa %.3f) e_Z %.2e" % (info.certified_error, info.kappa, e))
    assert info.converged and np.isfinite(info.kappa)
    assert info.certified_error <= 1.01e-7
    assert e <= info.certified_error


def test_stream_median_bracket_and_digit_sweeps_agree(cdl):
    # the sampled bracket (default) and the digit sweeps from the top bit
    # (select mode 1) are both exact: the same bandwidth bits
    X = dev(series(2100, 33, 21))
    try:
        cdl.set_select(1)
        g1, _, _ = cdl.stream_embedding(X, 8, SEED, tol=1e-6, panel_rows=512)
    finally:
        cdl.set_select(0)
    g0, _, _ = cdl.stream_embedding(X, 8, SEED, tol=1e-6, panel_rows=512)
    gs = cdl.build_graph(X)
    print("  sigma %.17g / %.17g / %.17g" % (g0.host_stats()["sigma"], g1.host_stats()["sigma"],
                                            gs.host_stats()["sigma"]))
    assert g0.host_stats()["sigma"] == g1.host_stats()["sigma"] == gs.host_stats()["sigma"]


def test_panel_size_does_not_change_results(cdl):
    n, T, k = 1300, 61, 64
    X = dev(series(n, T, 11))
    runs = [cdl.stream_embedding(X, k, SEED, tol=1e-10, panel_rows=p) for p in (0, 256, 768)]
    g0, Z0, i0 = runs[0]
    for g, Z, info in runs[1:]:
        assert torch.equal(g.stats, g0.stats)
        assert torch.equal(g.deg, g0.deg)
        assert torch.equal(Z, Z0)
        assert info.iterations == i0.iterations


def test_stream_equals_stored_path_on_grid_pair(cdl):
    """The C2 grid pair (n = 4096, T = 240, k = 128): streamed vs stored graph,
    embedding and scores."""
    cfg = gen.CONFIGS["C2"]
    pair = gen.make_pair(cfg["G"], cfg["T"], cfg["patches"], cfg["patch_size"])
    k = cfg["k"]
    out = {"stored": [], "stream": []}
    for X in (pair.X0, pair.X1):
        Xd = dev(X)
        g = cdl.build_graph(Xd)
        ch = cdl.build_chain(g, prec="fp32", depth=0, depth_max=6)
        Z, info = cdl.solve_embedding(g, ch, k, SEED, tol=1e-11, max_iter=30)
        out["stored"].append((g, Z))
        gs, Zs, infs = cdl.stream_embedding(Xd, k, SEED, tol=1e-11, panel_rows=1024)
        out["stream"].append((gs, Zs))
        a, b = g.host_stats(), gs.host_stats()
        print("  sigma %.17g / %.17g, iterations %d / %d" % (a["sigma"], b["sigma"],
                                                            info.iterations, infs.iterations))
        assert a["sigma"] == b["sigma"]          # the same distance keys, bit for bit
        np.testing.assert_allclose(host(gs.deg), host(g.deg), rtol=1e-14)
        assert b["vol"] == pytest.approx(a["vol"], rel=1e-14)
        assert rel(host(Zs), host(Z)) <= 1e-9
    F, top = cdl.anomaly_scores(out["stored"][0][1], out["stored"][0][0],
                                out["stored"][1][1], out["stored"][1][0], top_k=50)
    Fs, tops = cdl.anomaly_scores(out["stream"][0][1], out["stream"][0][0],
                                  out["stream"][1][1], out["stream"][1][0], top_k=50)
    assert rel(host(Fs), host(F)) <= 1e-8
    assert set(host(tops).tolist()) == set(host(top).tolist())


@pytest.mark.parametrize("prec,u", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8), ("fp32", 2.0 ** -24)])
def test_stream_stored_level_equals_stored_chain(cdl, prec, u):
    # the level normalised from the recomputed panels is the stored path's
    # level 0 up to the degrees' rounding (the two paths sum the rows in other
    # orders): a few entries at most one unit of the level type apart; the
    # solves agree to their tolerance
    cfg = gen.CONFIGS["C2"]
    X = dev(gen.make_pair(cfg["G"], cfg["T"], cfg["patches"], cfg["patch_size"]).X0)
    k = 128
    g = cdl.build_graph(X)
    ch = cdl.build_chain(g, prec=prec, depth=1, depth_max=1)
    Z, info = cdl.solve_embedding(g, ch, k, SEED, tol=1e-11, max_iter=30)
    gs, Zs, infs = cdl.stream_embedding(X, k, SEED, tol=1e-11, panel_rows=1024, level=prec)
    print("  %s: iterations %d / %d, fro %.15g / %.15g" % (
        prec, info.iterations, infs.iterations, ch.info.fro[0], gs.chain.info.fro[0]))
    assert gs.chain.info.depth == 1 and gs.chain.info.prec == ch.info.prec
    A, B = cdl.level(ch, 0).double(), cdl.level(gs.chain, 0).double()
    d = A != B
    print("  %s: %d of %d level entries differ" % (prec, int(d.sum()), d.numel()))
    assert float(d.double().mean()) <= 1e-6
    assert bool(((A - B).abs() <= 2 * u * A.abs()).all())
    assert torch.equal(B, B.T)
    assert gs.chain.info.fro[0] == pytest.approx(ch.info.fro[0], rel=1e-13)
    assert gs.chain.info.rho_bound == pytest.approx(ch.info.rho_bound, rel=1e-13)
    assert infs.converged and infs.rel_residual <= 1e-11
    assert rel(host(Zs), host(Z)) <= 1e-9


@pytest.mark.parametrize("n,T,k,panel", [(513, 40, 70, 256), (1100, 50, 130, 0)])
def test_stream_stored_level_matches_oracle(cdl, n, T, k, panel):
    X = series(n, T, 3 * n + T)
    gs, Z, info = cdl.stream_embedding(dev(X), k, SEED, tol=1e-11, panel_rows=panel, level="fp16")
    o = oracle.build_graph(X)
    Zo = oracle.solve_embedding(o["W"], oracle.rhs(o["W"], k, SEED), o["deg"])
    e = rel(host(Z), Zo)
    print("  n=%d: iterations %d e_Z %.2e depth used %s" % (
        n, info.iterations, e, [info.depth_used[i] for i in range(info.iterations)]))
    assert info.converged and e <= 1e-9


@pytest.mark.parametrize("n,T,k", [(3, 1, 1), (4, 6, 1), (5, 3, 65)])
def test_stream_tiny_snapshots(cdl, n, T, k):
    # the smallest graphs the one-level chain converges on (two nodes form a
    # bipartite graph, eigenvalue -1 of S: the stored path's lazy chain is
    # the tool for that); rho(S~) = 0.79, 0.46, 0.60 here, so the residual
    # contracts by rho^2 per iteration; ragged k
    X = series(n, T, 100 + n)
    g, Z, info = cdl.stream_embedding(dev(X), k, SEED, tol=1e-10, max_iter=64)
    o = oracle.build_graph(X)
    assert g.host_stats()["sigma"] == pytest.approx(o["sigma"], rel=1e-12)
    np.testing.assert_allclose(host(g.deg), o["deg"], rtol=1e-12)
    Zo = oracle.solve_embedding(o["W"], oracle.rhs(o["W"], k, SEED), o["deg"])
    assert info.converged
    np.testing.assert_allclose(host(Z), Zo, rtol=0, atol=1e-8 * np.abs(Zo).max() + 1e-300)


def test_stream_rejects_bad_arguments(cdl):
    X = dev(series(100, 5, 1))
    with pytest.raises(cdl.CdlError):
        cdl.stream_embedding(X, 0, SEED)
    with pytest.raises(cdl.CdlError):
        cdl.stream_embedding(X, 8, SEED, max_iter=0)
    with pytest.raises(cdl.CdlError):
        cdl.stream_embedding(X, 8, SEED, panel_rows=-1)
    bad = series(100, 5, 1)
    bad[17, 3] = np.nan
    with pytest.raises(cdl.CdlError):
        cdl.stream_embedding(dev(bad), 8, SEED)
