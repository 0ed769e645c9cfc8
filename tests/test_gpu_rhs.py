"""Right-hand sides of Algorithm 1 alone (cdl_rhs) against the oracle's
definition, element by element.

The GPU sums the signed square roots of a row as an exact int8 product of the
sign bits with base-256 digits of the roots scaled by a power of two per
chunk of 1024 neighbours, so its only rounding is that scaling and the FP64
sums.  Two kinds of cases:

* exact: weights W_ij = (m_ij 2^-(27+s))^2 with integer m < 2^26 and a scale
  exponent s per chunk of columns: every root, digit, integer sum and FP64
  sum is exact on both sides, and with k = 64 or 256 (1/sqrt(k) a power of
  two) so is the final scaling, so Y must equal the oracle's bit for bit.  A
  wrong digit, bit, byte position, sign or chunk scale shows up here;
* general: Gaussian-kernel and wide-range weights, ids permuted, k from 1 to
  300 (one to five blocks of 64 projections, every workgroup shape), within
  a bound derived from the two sides' rounding.
"""

import ctypes as C
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

SEED = 2024


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def graph(cdl, W):
    """A Graph holding W in the padded layout (only W and n are read)."""
    n = W.shape[0]
    m = cdl.ld(n)
    Wp = np.zeros((m, m))
    Wp[:n, :n] = W
    t = torch.from_numpy(Wp).cuda()
    return cdl.Graph(W=t, deg=torch.zeros(n, dtype=torch.float64, device="cuda"),
                     stats=torch.zeros(4, dtype=torch.float64, device="cuda"), n=n)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ids(n, perm, seed):
    if not perm:
        return None
    rng = np.random.default_rng(seed)
    return rng.choice(1 << 20, size=n, replace=False).astype(np.int32)


def gpu_ids(g):
    return None if g is None else torch.from_numpy(g).cuda()


def dyadic(n, seed, scales=(0, 4, 9)):
    """W_ij = (m 2^-(27+s))^2, m in [1, 2^26), s by column chunk of 1024."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 1 << 26, size=(n, n)).astype(np.float64)
    s = np.array([scales[(j // 1024) % len(scales)] for j in range(n)], dtype=np.float64)
    v = m * np.exp2(-(27.0 + s))[None, :]
    W = v * v
    np.fill_diagonal(W, 0.0)
    assert np.array_equal(np.sqrt(W), np.where(np.eye(n, dtype=bool), 0.0, v))
    return W


def kernel_weights(n, seed):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((n, 6))
    D2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    W = np.exp(-D2 / np.median(D2))
    np.fill_diagonal(W, 0.0)
    return W


def bound(W, k):
    """Per-row bound on |Y_gpu - Y_oracle|: the GPU's scaling errs by at most
    2^-55 of a chunk's largest root per term (n 2^-55 max_j |v_ij| in all),
    and both sides' FP64 sums of signed terms by about sqrt(n) u
    sum_j |v_ij| (random signs; (n + 2) u in the worst case).  2e-14
    sum_j |v_ij| / sqrt(k) is about ten times what either gives at n = 3000."""
    return 2e-14 * np.sqrt(W).sum(axis=1, keepdims=True) / math.sqrt(k) + 1e-300


@pytest.mark.parametrize("n,k,perm", [(333, 64, False), (333, 256, True), (2500, 64, True),
                                      (2500, 256, False)])
def test_rhs_exact_on_dyadic_weights(cdl, n, k, perm):
    print("exact rhs case n=%d k=%d perm=%d" % (n, k, perm), flush=True)
    W = dyadic(n, n + k)
    gid = ids(n, perm, 7)
    Y = host(cdl.rhs(graph(cdl, W), k, SEED, gid=gpu_ids(gid)))
    Yo = oracle.rhs(W, k, SEED, gid)
    assert np.array_equal(Y, Yo), np.abs(Y - Yo).max()


@pytest.mark.parametrize("n,k,perm", [(2, 1, False), (333, 70, True), (1025, 128, False),
                                      (1500, 130, True), (2049, 300, True), (3000, 256, True)])
def test_rhs_matches_oracle(cdl, n, k, perm):
    print("rhs case n=%d k=%d perm=%d" % (n, k, perm), flush=True)
    W = kernel_weights(n, n + k)
    gid = ids(n, perm, n)
    Y = host(cdl.rhs(graph(cdl, W), k, SEED, gid=gpu_ids(gid)))
    Yo = oracle.rhs(W, k, SEED, gid)
    err = np.abs(Y - Yo)
    b = bound(W, k)
    print("  max |dY| / bound %.2e, max |dY| / |Y| %.2e" % ((err / b).max(),
                                                            err.max() / np.abs(Yo).max()))
    assert (err <= b).all()


def test_rhs_wide_range_rows(cdl):
    """Weights over 300 decades, rows of uniformly tiny weights, a row with one
    nonzero weight: each chunk's own scale keeps every row's relative accuracy."""
    n, k = 2300, 256
    rng = np.random.default_rng(11)
    W = 10.0 ** rng.uniform(-150.0, 150.0, size=(n, n))
    W[3] = 1e-290 * rng.uniform(0.5, 1.0, size=n)
    W[4] = 0.0
    W[4, 2000] = 1e-200
    W[5, :1024] *= 1e-250   # one chunk far below the others
    np.fill_diagonal(W, 0.0)
    Y = host(cdl.rhs(graph(cdl, W), k, SEED))
    Yo = oracle.rhs(W, k, SEED)
    err = np.abs(Y - Yo)
    b = bound(W, k)
    print("  max |dY| / bound %.2e" % (err / b).max())
    assert (err <= b).all()
    assert np.abs(Y[4]).max() > 0 and np.allclose(Y[4], Yo[4], rtol=1e-15, atol=0)


def test_rhs_pair_matches_single_and_oracle(cdl):
    n, k = 3000, 256
    W0, W1 = kernel_weights(n, 1), dyadic(n, 2)
    gid = ids(n, True, 3)
    g0, g1 = graph(cdl, W0), graph(cdl, W1)
    Y0, Y1 = cdl.rhs(g0, k, SEED, gid=gpu_ids(gid), g1=g1)
    Y0, Y1 = host(Y0), host(Y1)
    S0 = host(cdl.rhs(g0, k, SEED, gid=gpu_ids(gid)))
    S1 = host(cdl.rhs(g1, k, SEED, gid=gpu_ids(gid)))
    # the pair scales its integer sums into FP64 at chunk boundaries where
    # either snapshot's exponent changes, the single form where its own does
    assert (np.abs(Y0 - S0) <= 1e-15 * np.sqrt(W0).sum(axis=1, keepdims=True) / 16).all()
    assert np.array_equal(Y1, S1)   # dyadic: every sum exact in both forms
    assert (np.abs(Y0 - oracle.rhs(W0, k, SEED, gid)) <= bound(W0, k)).all()
    assert np.array_equal(Y1, oracle.rhs(W1, k, SEED, gid))


def test_rhs_nonfinite_weights_reach_their_rows(cdl):
    n, k = 600, 64
    W = kernel_weights(n, 5)
    W[5, 7] = np.nan
    W[11, 300] = np.inf
    Y = host(cdl.rhs(graph(cdl, W), k, SEED))
    bad = ~np.isfinite(Y).all(axis=1)
    assert bad[5] and bad[11] and bad.sum() == 2
    Wc = W.copy()
    Wc[5, 7] = Wc[11, 300] = 0.0
    ok = ~bad
    Yo = oracle.rhs(Wc, k, SEED)
    assert (np.abs(Y[ok] - Yo[ok]) <= bound(Wc, k)[ok]).all()


def test_rhs_argument_errors(cdl):
    from paper_1802_05421_amd import _lib
    L = _lib.load()
    sz = C.c_size_t()
    assert L.cdl_rhs_workspace_bytes(1, 8, 0, C.byref(sz)) != 0
    assert L.cdl_rhs_workspace_bytes(100, 0, 0, C.byref(sz)) != 0
    assert L.cdl_rhs_workspace_bytes(100, 8, 0, C.byref(sz)) == 0
    one = sz.value
    assert L.cdl_rhs_workspace_bytes(100, 8, 1, C.byref(sz)) == 0 and sz.value >= 2 * one - 256
    from paper_1802_05421_amd.api import context
    ctx = context(0)
    W = torch.zeros((256, 256), dtype=torch.float64, device="cuda")
    Y = torch.zeros((100, 8), dtype=torch.float64, device="cuda")
    ws = torch.zeros(one, dtype=torch.uint8, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    E_ARG, E_WS = 1, 2
    assert L.cdl_rhs(ctx.h, p(W), None, None, 100, 8, 1, p(Y), None, p(ws), one) == 0
    assert L.cdl_rhs(ctx.h, p(W), p(W), None, 100, 8, 1, p(Y), None, p(ws), one) == E_ARG
    assert L.cdl_rhs(ctx.h, p(W), None, None, 100, 0, 1, p(Y), None, p(ws), one) == E_ARG
    assert L.cdl_rhs(ctx.h, p(W), None, None, 100, 8, 1, p(Y), None, p(ws), one - 8) == E_WS
    torch.cuda.synchronize()
