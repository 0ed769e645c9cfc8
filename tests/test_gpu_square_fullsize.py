"""Chain squarings (Algorithm 2, ChainProduct; eq. inverse-chain) at
production sizes, against the oracle's FP64 levels.

The GPU's level l+1 is its level l squared on MFMA with FP32 accumulation and
rounded to the level type; the oracle's levels are exact FP64 powers of its own
S~ (from its own weights).  Both sides take the same kernel bandwidth (0.3 x
the oracle's median rule, which pushes rho(S~) to about 0.75 so that the
squared levels stay large).  Every compared entry must lie within a
first-order rounding bound derived from the level type's unit roundoff u,
FP32 accumulation over n terms and, for FP16, its subnormal spacing eta
(scaled levels):

  level 0:  |dS|  <= u |S| + eta
  level 1:  |dC1| <= (2u + n u32) (|S||S|) + u |C1| + eta (1 + r_i + r_j)
  level 2:  |dC2| <= (6u + 3 n u32) |S|^4 + u |C2|
                     + eta (1 + r2_i + r2_j + r3_i + r3_j + r2_i r_j + r_i r2_j)

with r = |S| 1, r2 = |S|^2 1, r3 = |S|^3 1 (level 2 bounds |C1| and the level-1
error by |S|^2, so only rows of |S|-powers are needed).  The FP64 values that
the two sides round differ too (degrees summed in other orders, distances by a
Gram against direct differences): by at most delta (|S| + 2 v v^T) with
v = D^{1/2} 1 / sqrt(vol) and delta = 2e-11, which matters where S~ = S - v v^T
cancels; its terms are carried through both squarings
(a = |S| v, c = |S|^2 v, b = |S|^3 v):

  level 0:  + delta (|S| + 2 v v^T)
  level 1:  + 2 delta (|S|^2 + a v^T + v a^T)
  level 2:  + delta (4 |S|^4 + 2 (b v^T + v b^T) + 2 (c a^T + a c^T))

A 256 x 256 tile
computed from the wrong panels, or left unwritten, exceeds these bounds by
orders of magnitude.

* n = 6084 (78 x 78 grid): 300 upper 256 x 256 tiles, more than one round of
  256 workgroups, so the full-round branch of the tile order runs; levels 1
  and 2 compared in full.
* n = 16384 (the 128 x 128 benchmark grid): 40 sampled rows of levels 1 and
  2 (the oracle's rows of S~^2 and S~^4 by repeated vector-matrix products).
"""

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(600)]

U = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp32": 2.0 ** -24}
U32 = 2.0 ** -24
DELTA = 2e-11


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def eta(prec, n, cdl):
    # half the smallest subnormal spacing of the stored (scaled) level
    if prec != "fp16":
        return 0.0
    return 2.0 ** -25 / cdl.level_scale_for(n, prec)


def grid_snapshot(G):
    p = gen.make_pair(G, 240, 4, 4)
    return p.X0


def oracle_st(X):
    D2 = oracle.sq_distances(X)
    sigma = 0.3 * oracle.bandwidth(D2)
    W = oracle.gaussian_weights(D2, sigma)
    del D2
    deg, vol = oracle.degrees(W)
    St = oracle.normalized_deflated(W, deg, vol)
    return sigma, St, np.sqrt(deg / vol)


def gpu_levels(cdl, X, sigma, prec, rows=None):
    n = X.shape[0]
    g = cdl.build_graph(dev(X), sigma=sigma)
    ch = cdl.build_chain(g, prec=prec, depth=3, depth_max=3)
    assert ch.depth == 3
    sc = cdl.level_scale(ch)
    out = []
    for l in range(3):
        lev = cdl.level(ch, l)
        if rows is None:
            L = host(lev.double()) / sc
            np.testing.assert_array_equal(L, L.T)           # mirrored tiles
            assert np.all(L[n:, :] == 0) and np.all(L[:, n:] == 0)
            out.append(L[:n, :n])
        else:
            out.append(host(lev[dev(rows).long(), :n].double()) / sc)
    del ch, g
    torch.cuda.empty_cache()
    return out


def check(name, got, want, bound):
    err = np.abs(got - want)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    relf = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print("  %s: rel Frobenius error %.2e, max error / bound %.3f" % (name, relf, ratio), flush=True)
    assert np.all(err <= bound), name


@pytest.fixture(scope="module")
def mid():
    X = grid_snapshot(78)
    sigma, St, v = oracle_st(X)
    A = np.abs(St)
    A2 = A @ A
    C1 = St @ St
    C2 = C1 @ C1
    A4 = A2 @ A2
    r = A.sum(axis=1)
    r2 = A2.sum(axis=1)
    r3 = A @ r2
    a = A @ v
    c = A @ a
    b = A @ c
    return dict(X=X, sigma=sigma, St=St, A=A, A2=A2, A4=A4, C1=C1, C2=C2, r=r, r2=r2, r3=r3,
                v=v, a=a, b=b, c=c)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_square_full_matrix_more_than_one_round(cdl, mid, prec):
    n = mid["X"].shape[0]
    assert (cdl.ld(n) // 256) * (cdl.ld(n) // 256 + 1) // 2 > 256
    print("squaring parity n=%d prec=%s sigma=%.4f" % (n, prec, mid["sigma"]), flush=True)
    L0, L1, L2 = gpu_levels(cdl, mid["X"], mid["sigma"], prec)
    u, e = U[prec], eta(prec, n, cdl)
    nu = n * U32
    r, r2, r3 = mid["r"], mid["r2"], mid["r3"]
    v, a, b, c = mid["v"], mid["a"], mid["b"], mid["c"]
    b0 = u * mid["A"] + e + DELTA * (mid["A"] + 2 * np.outer(v, v))
    check("level 0", L0, mid["St"], 1.01 * b0)
    b1 = ((2 * u + nu) * mid["A2"] + u * np.abs(mid["C1"]) + e * (1 + r[:, None] + r[None, :])
          + 2 * DELTA * (mid["A2"] + np.outer(a, v) + np.outer(v, a)))
    check("level 1", L1, mid["C1"], 1.01 * b1)
    b2 = ((6 * u + 3 * nu) * mid["A4"] + u * np.abs(mid["C2"])
          + e * (1 + r2[:, None] + r2[None, :] + r3[:, None] + r3[None, :]
                 + np.outer(r2, r) + np.outer(r, r2))
          + DELTA * (4 * mid["A4"] + 2 * (np.outer(b, v) + np.outer(v, b))
                     + 2 * (np.outer(c, a) + np.outer(a, c))))
    check("level 2", L2, mid["C2"], 1.01 * b2)


@pytest.fixture(scope="module")
def big():
    X = grid_snapshot(128)
    sigma, St, v = oracle_st(X)
    n = X.shape[0]
    rows = np.sort(np.concatenate([np.random.default_rng(23).choice(n, 38, replace=False), [0, n - 1]]))
    A = np.abs(St)
    r = A.sum(axis=1)
    r2 = A @ r
    r3 = A @ r2
    a = A @ v
    c = A @ a
    b = A @ c
    Sr = St[rows]
    C1r = Sr @ St                  # rows of S~^2
    C2r = ((C1r @ St) @ St)        # rows of S~^4
    Ar = A[rows]
    A2r = Ar @ A                   # rows of |S|^2
    A4r = ((A2r @ A) @ A)          # rows of |S|^4
    del A, St
    return dict(X=X, sigma=sigma, rows=rows, S0r=Sr, C1r=C1r, C2r=C2r, A0r=Ar, A2r=A2r, A4r=A4r,
                r=r, r2=r2, r3=r3, v=v, a=a, b=b, c=c)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_square_sampled_rows_n16384(cdl, big, prec):
    n, rows = big["X"].shape[0], big["rows"]
    print("squaring parity n=%d prec=%s, %d sampled rows" % (n, prec, rows.size), flush=True)
    L0, L1, L2 = gpu_levels(cdl, big["X"], big["sigma"], prec, rows)
    u, e = U[prec], eta(prec, n, cdl)
    nu = n * U32
    r, r2, r3 = big["r"], big["r2"], big["r3"]
    ri, r2i, r3i = r[rows][:, None], r2[rows][:, None], r3[rows][:, None]
    v, a, b, c = big["v"], big["a"], big["b"], big["c"]
    vi, ai, bi, ci = v[rows][:, None], a[rows][:, None], b[rows][:, None], c[rows][:, None]
    b0 = u * big["A0r"] + e + DELTA * (big["A0r"] + 2 * vi * v[None, :])
    check("level 0 rows", L0, big["S0r"], 1.01 * b0)
    b1 = ((2 * u + nu) * big["A2r"] + u * np.abs(big["C1r"]) + e * (1 + ri + r[None, :])
          + 2 * DELTA * (big["A2r"] + ai * v[None, :] + vi * a[None, :]))
    check("level 1 rows", L1, big["C1r"], 1.01 * b1)
    b2 = ((6 * u + 3 * nu) * big["A4r"] + u * np.abs(big["C2r"])
          + e * (1 + r2i + r2[None, :] + r3i + r3[None, :] + r2i * r[None, :] + ri * r2[None, :])
          + DELTA * (4 * big["A4r"] + 2 * (bi * v[None, :] + vi * b[None, :])
                     + 2 * (ci * a[None, :] + ai * c[None, :])))
    check("level 2 rows", L2, big["C2r"], 1.01 * b2)
