"""The measured launch-configuration tuner: a tuning context times every
candidate of the squaring (6 tile variants), the chain application and the
FP64 residual product (3 split-K counts each) on first use of a shape, and
keeps the fastest; every candidate must give the oracle's results within the
tolerances of the untuned path (the squared level within its rounding bound,
the embedding within 1e-9)."""

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

U = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    cdl.autotune_clear()
    yield cdl
    cdl.set_autotune(False)
    for fam in ("square", "apply", "residual"):
        cdl.force_choice(fam, -1)
    cdl.autotune_clear()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def square_case():
    # 78 x 78 grid (n = 6084: 300 upper tiles, a full round and a split tail),
    # kernel bandwidth 0.3 x the oracle's median rule
    X = gen.make_pair(78, 240, 4, 4).X0
    D2 = oracle.sq_distances(X)
    sigma = 0.3 * oracle.bandwidth(D2)
    W = oracle.gaussian_weights(D2, sigma)
    del D2
    deg, vol = oracle.degrees(W)
    St = oracle.normalized_deflated(W, deg, vol)
    A = np.abs(St)
    v = np.sqrt(deg / vol)
    a = A @ v
    return dict(X=X, sigma=sigma, C1=St @ St, A2=A @ A, r=A.sum(axis=1), v=v, a=a)


def level1(cdl, case, prec):
    g = cdl.build_graph(dev(case["X"]), sigma=case["sigma"])
    ch = cdl.build_chain(g, prec=prec, depth=2, depth_max=2)
    n = case["X"].shape[0]
    L1 = host(cdl.level(ch, 1).double())[:n, :n] / cdl.level_scale(ch)
    del ch, g
    return L1


def check_level1(case, L1, prec, n):
    # first-order rounding bound of one squaring of the rounded level (the
    # derivation is in tests/test_gpu_square_fullsize.py)
    u, nu = U[prec], n * 2.0 ** -24
    e = 2.0 ** -25 / 4096.0 if prec == "fp16" else 0.0
    r, v, a = case["r"], case["v"], case["a"]
    bound = ((2 * u + nu) * case["A2"] + u * np.abs(case["C1"]) + e * (1 + r[:, None] + r[None, :])
             + 2 * 2e-11 * (case["A2"] + np.outer(a, v) + np.outer(v, a)))
    ratio = float((np.abs(L1 - case["C1"]) / bound).max())
    return ratio


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_squaring_tuned_and_every_variant_within_bound(cdl, square_case, prec):
    n = square_case["X"].shape[0]
    assert cdl.autotune_lookup("square", prec, n) is None
    cdl.set_autotune(True)
    try:
        L1 = level1(cdl, square_case, prec)
    finally:
        cdl.set_autotune(False)
    entry = cdl.autotune_lookup("square", prec, n)
    assert entry is not None
    choice, ncand, ms = entry
    print("square %s n=%d: choice %d of %d, %.3f ms" % (prec, n, choice, ncand, ms), flush=True)
    assert ncand == 6 and 0 <= choice < 6 and ms > 0
    assert check_level1(square_case, L1, prec, n) <= 1.0
    for v in range(6):
        cdl.force_choice("square", v)
        try:
            ratio = check_level1(square_case, level1(cdl, square_case, prec), prec, n)
        finally:
            cdl.force_choice("square", -1)
        print("  variant %d: max error / bound %.3f" % (v, ratio), flush=True)
        assert ratio <= 1.0


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_solve_tuned_and_every_split_matches_oracle(cdl, prec):
    n, k = 700, 70
    X = np.random.default_rng(9).standard_normal((n, 24))
    o = oracle.build_graph(X)
    Zo = oracle.solve_embedding(o["W"], oracle.rhs(o["W"], k, 5))
    g = cdl.build_graph(dev(X))
    ch = cdl.build_chain(g, prec=prec, depth=0, depth_max=4)
    cdl.set_autotune(True)
    try:
        Z, info = cdl.solve_embedding(g, ch, k, 5, tol=1e-11, max_iter=40)
    finally:
        cdl.set_autotune(False)
    for fam in ("apply", "residual"):
        entry = cdl.autotune_lookup(fam, prec if fam == "apply" else "fp64", n, k)
        assert entry is not None and entry[1] == 3 and entry[2] > 0, (fam, entry)
        print("%s %s: choice %d, %.3f ms" % (fam, prec, entry[0], entry[2]), flush=True)
    e = np.linalg.norm(host(Z) - Zo) / np.linalg.norm(Zo)
    assert info.converged and e <= 1e-9
    for fam in ("apply", "residual"):
        for c in range(3):
            cdl.force_choice(fam, c)
            try:
                Z, info = cdl.solve_embedding(g, ch, k, 5, tol=1e-11, max_iter=40)
            finally:
                cdl.force_choice(fam, -1)
            e = np.linalg.norm(host(Z) - Zo) / np.linalg.norm(Zo)
            print("  %s choice %d: e_Z %.2e, %d iterations" % (fam, c, e, info.iterations))
            assert info.converged and e <= 1e-9


def test_table_save_and_load(cdl, tmp_path):
    assert cdl.autotune_entries() >= 1
    path = str(tmp_path / "tune.json")
    cdl.autotune_save(path)
    before = cdl.autotune_lookup("square", "bf16", 6084)
    cdl.autotune_clear()
    assert cdl.autotune_entries() == 0
    cdl.autotune_load(path)
    assert cdl.autotune_lookup("square", "bf16", 6084) == before
