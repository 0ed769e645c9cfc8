"""One-pass sequences (CDL_SEQ_BATCHED): grouped launches over all snapshots
for the chain squarings and every refinement step, over all pairs for the
scores, and convergence tested on the device.

* With tol = 0 (exactly max_iter iterations) the grouped kernels compute the
  same tiles in the same order as the per-snapshot path, so the scores and
  top-K equal the synchronous call's bit for bit, also as HIP-graph replays.
* With tol > 0 each snapshot stops on its own once its FP64 relative
  residual reaches tol; the scores match the oracle.
* The full 24-snapshot sequence (96 x 96 grid, n_t in [1024, 8192], T = 120,
  k = 128, FP16 chains) against the oracle run on every snapshot: node
  scores of all 23 pairs within 1e-5 (||.||_inf relative) and the same top-50
  wherever the oracle's 50th/51st gap exceeds 2 e_F.
"""

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

E_ARG, E_NONFINITE, E_GRAPH, E_NOCONV = 1, 3, 4, 6


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small_sequence():
    return gen.make_sequence(G=40, T=60, n_snap=4, stride=20, n_min=450, n_max=1100,
                             patch_size=3, onsets=(2,))


@pytest.mark.parametrize("prec,mode,depth", [("fp32", "delta_a", 3), ("fp16", "unweighted", 5),
                                             ("bf16", "unweighted", 2)])
def test_batched_equals_per_snapshot_path_and_graph_replays(cdl, prec, mode, depth):
    seq = small_sequence()
    k, seed = 40, gen.grid.PROJ_SEED
    Xs = [dev(X) for X in seq.X]
    gdev = [torch.from_numpy(g).cuda() for g in seq.gid]
    base = dict(k=k, seed=seed, prec=prec, depth=depth, tol=0.0, max_iter=6, mode=mode, top_k=50)
    print("batched sequence", prec, mode, depth, [len(g) for g in seq.gid], flush=True)
    # the group's own split counts: the per-snapshot path's results to rounding
    wF, wT, wi = cdl.score_sequence(Xs, gdev, cdl.SeqParams(**base))
    wF, wT = [host(f) for f in wF], [host(t) for t in wT]
    pb = cdl.SeqParams(**base, asynchronous=True, batched=True)
    Fb, Tb, ib = cdl.score_sequence(Xs, gdev, pb)
    assert ib.max_iterations == 6 and ib.pairs == len(Xs) - 1
    for t in range(len(wF)):
        compare(host(Fb[t]), host(Tb[t]), wF[t], wT[t], 1e-9)
    # pinned choices: every snapshot keeps its own split counts, and the
    # grouped launches compute the per-snapshot path's tiles bit for bit
    cdl.force_choice("apply", 0)
    cdl.force_choice("residual", 0)
    try:
        wF, wT, wi = cdl.score_sequence(Xs, gdev, cdl.SeqParams(**base))
        wF, wT = [host(f) for f in wF], [host(t) for t in wT]
        Fb, Tb, ib = cdl.score_sequence(Xs, gdev, pb)
        for t in range(len(wF)):
            np.testing.assert_array_equal(host(Fb[t]), wF[t])
            np.testing.assert_array_equal(host(Tb[t]), wT[t])
    finally:
        cdl.force_choice("apply", -1)
        cdl.force_choice("residual", -1)
    # graph replays of the group's own counts equal its eager call
    eF, eT, _ = cdl.score_sequence(Xs, gdev, pb)
    eF, eT = [host(f) for f in eF], [host(t) for t in eT]
    sF0 = host(cdl.score_sequence(Xs[:2], gdev[:2], cdl.SeqParams(**base))[0][0])
    pg = cdl.SeqParams(**base, asynchronous=True, batched=True, graph=True)
    ws = torch.empty(cdl.sequence_workspace_bytes(Xs, gdev, pg), dtype=torch.uint8, device="cuda")
    Fs, tops, info = cdl.score_sequence(Xs, gdev, pg, ws=ws)
    launches = []
    for r in range(3):
        for f in Fs:
            f.fill_(-1.0)
        F2, T2, info = cdl.score_sequence(Xs, gdev, pg, ws=ws, out=(Fs, tops))
        launches.append(info.graph_launches)
        for t in range(len(eF)):
            np.testing.assert_array_equal(host(F2[t]), eF[t])
            np.testing.assert_array_equal(host(T2[t]), eT[t])
        # eager work on the same stream between replays
        Fx, _, _ = cdl.score_sequence(Xs[:2], gdev[:2], cdl.SeqParams(**base))
        np.testing.assert_array_equal(host(Fx[0]), sF0)
    assert launches == [1, 1, 1]


@pytest.mark.parametrize("case", ["given_sigma", "matrix_select"])
def test_batched_graph_build_variants_equal_per_snapshot_path(cdl, case):
    """The grouped graph build with a caller's bandwidth (no selection) and
    with the selection forced onto the matrix (no sampled bracket): the
    per-snapshot path's results bit for bit (choices pinned)."""
    seq = small_sequence()
    Xs = [dev(X) for X in seq.X]
    gdev = [torch.from_numpy(g).cuda() for g in seq.gid]
    base = dict(k=24, seed=gen.grid.PROJ_SEED, prec="fp16", depth=2, tol=0.0, max_iter=3,
                top_k=50, sigma=8.0 if case == "given_sigma" else 0.0)
    print("batched graph build", case, flush=True)
    cdl.force_choice("apply", 0)
    cdl.force_choice("residual", 0)
    if case == "matrix_select":
        cdl.set_select(1)
    try:
        wF, wT, _ = cdl.score_sequence(Xs, gdev, cdl.SeqParams(**base))
        Fb, Tb, _ = cdl.score_sequence(Xs, gdev, cdl.SeqParams(**base, asynchronous=True,
                                                               batched=True))
        for t in range(len(wF)):
            np.testing.assert_array_equal(host(Fb[t]), host(wF[t]))
            np.testing.assert_array_equal(host(Tb[t]), host(wT[t]))
    finally:
        cdl.set_select(0)
        cdl.force_choice("apply", -1)
        cdl.force_choice("residual", -1)


def seq_oracle(seq, k, seed, idx=None):
    out = {}
    for t in (range(len(seq.X)) if idx is None else idx):
        g = oracle.build_graph(seq.X[t])
        Z = oracle.solve_embedding(g["W"], oracle.rhs(g["W"], k, seed, seq.gid[t]), g["deg"])
        out[t] = (g["vol"], Z)
    return out


def pair_oracle(seq, snaps, t):
    common, i0, i1 = np.intersect1d(seq.gid[t], seq.gid[t + 1], assume_unique=True,
                                    return_indices=True)
    (v0, Z0), (v1, Z1) = snaps[t], snaps[t + 1]
    F = oracle.scores(Z0, v0, Z1, v1, map0=i0, map1=i1)
    return F, oracle.top_k(F, 50)


def compare(F, top, Fo, to, tol):
    ef = np.abs(F - Fo).max() / np.abs(Fo).max()
    srt = np.sort(Fo)[::-1]
    gap = (srt[49] - srt[50]) / np.abs(Fo).max() if Fo.size > 50 else 1.0
    assert ef <= tol
    assert np.all(np.diff(F[top]) <= 0)
    if gap > 2 * ef:
        assert set(top.tolist()) == set(to.tolist())
    return ef, gap


def test_batched_device_convergence_matches_oracle(cdl):
    seq = small_sequence()
    k, seed = 40, gen.grid.PROJ_SEED
    Xs = [dev(X) for X in seq.X]
    gdev = [torch.from_numpy(g).cuda() for g in seq.gid]
    p = cdl.SeqParams(k=k, seed=seed, prec="fp16", depth=2, tol=1e-11, max_iter=40, top_k=50,
                      asynchronous=True, batched=True)
    Fs, tops, info = cdl.score_sequence(Xs, gdev, p)
    print("device convergence: max iterations %d, residual %.2e" % (info.max_iterations,
                                                                      info.max_rel_residual))
    assert 1 <= info.max_iterations < 40 and info.max_rel_residual <= 1e-11
    snaps = seq_oracle(seq, k, seed)
    for t in range(len(Xs) - 1):
        Fo, to = pair_oracle(seq, snaps, t)
        ef, gap = compare(host(Fs[t]), host(tops[t]), Fo, to, 1e-8)
        print("  pair %d: e_F %.2e gap %.2e" % (t, ef, gap))
    # an unreachable tolerance within max_iter: the call reports it
    p.tol, p.max_iter = 1e-30, 2
    with pytest.raises(cdl.CdlError) as e:
        cdl.score_sequence(Xs, gdev, p)
    assert e.value.status == 6


# ---- the 24-snapshot sequence --------------------------------------------------

C4K = 128


@pytest.fixture(scope="module")
def c4(cdl):
    cfg = gen.CONFIGS["C4"]
    seq = gen.make_sequence(G=cfg["G"], T=cfg["T"], n_snap=cfg["n_snap"], stride=cfg["stride"],
                            n_min=cfg["n_min"], n_max=cfg["n_max"], patch_size=cfg["patch_size"],
                            onsets=cfg["onsets"])
    Xs = [dev(X) for X in seq.X]
    gdev = [torch.from_numpy(g).cuda() for g in seq.gid]
    p = cdl.SeqParams(k=C4K, seed=gen.grid.PROJ_SEED, prec="fp16", depth=2, tol=1e-9,
                      max_iter=20, top_k=50, asynchronous=True, batched=True)
    print("C4 batched: sizes", [len(g) for g in seq.gid], flush=True)
    Fs, tops, info = cdl.score_sequence(Xs, gdev, p)
    out = dict(seq=seq, F=[host(f) for f in Fs], top=[host(t) for t in tops], info=info)
    del Xs, gdev, Fs, tops
    torch.cuda.empty_cache()
    return out


_c4_oracle = {}


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("chunk", [0, 1, 2])
def test_c4_oracle_snapshots(c4, chunk):
    # the oracle's embeddings, eight snapshots per test (cached)
    seq = c4["seq"]
    idx = range(8 * chunk, min(8 * chunk + 8, len(seq.X)))
    print("oracle snapshots", list(idx), flush=True)
    _c4_oracle.update(seq_oracle(seq, C4K, gen.grid.PROJ_SEED, idx))
    info = c4["info"]
    assert info.pairs == len(seq.X) - 1 and info.max_rel_residual <= 1e-9


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_c4_scores_and_top50_match_oracle(c4):
    seq = c4["seq"]
    missing = [t for t in range(len(seq.X)) if t not in _c4_oracle]
    _c4_oracle.update(seq_oracle(seq, C4K, gen.grid.PROJ_SEED, missing))
    worst = 0.0
    for t in range(len(seq.X) - 1):
        Fo, to = pair_oracle(seq, _c4_oracle, t)
        ef, gap = compare(c4["F"][t], c4["top"][t], Fo, to, 1e-5)
        worst = max(worst, ef)
        print("  pair %2d: m=%d e_F %.2e gap %.2e" % (t, Fo.size, ef, gap))
    print("C4: %d pairs, worst e_F %.2e, iterations %d" % (len(seq.X) - 1, worst,
                                                           c4["info"].max_iterations))


def test_batched_errors(cdl):
    """Failure handling of the one-pass mode, every case decided on the host
    (argument checks before any launch, or the final read-back of graph
    statistics and residuals), so every kernel exits normally."""
    seq = small_sequence()
    Xs = [dev(X) for X in seq.X]
    gdev = [torch.from_numpy(g).cuda() for g in seq.gid]
    base = dict(k=16, seed=gen.grid.PROJ_SEED, prec="fp16", depth=2, tol=0.0, max_iter=3,
                asynchronous=True, batched=True)
    # arguments: FP64 levels, and the one-pass flag without the asynchronous one
    for bad in (dict(prec="fp64"), dict(asynchronous=False)):
        q = dict(base)
        q.update(bad)
        with pytest.raises(cdl.CdlError) as e:
            cdl.score_sequence(Xs, gdev, cdl.SeqParams(**q))
        assert e.value.status == E_ARG
    # a non-finite value in one snapshot's series
    Xn = [x.clone() for x in Xs]
    Xn[2][5, 3] = float("nan")
    print("batched errors: non-finite series", flush=True)
    with pytest.raises(cdl.CdlError) as e:
        cdl.score_sequence(Xn, gdev, cdl.SeqParams(**base))
    assert e.value.status == E_NONFINITE
    # a bandwidth so small that every weight underflows: zero degrees
    print("batched errors: underflowing weights", flush=True)
    with pytest.raises(cdl.CdlError) as e:
        cdl.score_sequence(Xs, gdev, cdl.SeqParams(**dict(base, sigma=1e-3)))
    assert e.value.status in (E_GRAPH, E_NONFINITE)
    # a residual target the iteration bound cannot reach
    print("batched errors: no convergence", flush=True)
    with pytest.raises(cdl.CdlError) as e:
        cdl.score_sequence(Xs, gdev, cdl.SeqParams(**dict(base, tol=1e-15, max_iter=1)))
    assert e.value.status == E_NOCONV
    # the context still works afterwards
    F, T, info = cdl.score_sequence(Xs, gdev, cdl.SeqParams(**base))
    assert info.max_iterations == 3 and all(np.isfinite(host(f)).all() for f in F)
