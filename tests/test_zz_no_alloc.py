"""The allocation-free score entry point (cdl_anomaly_scores_noalloc), called
through the C ABI, against cdl_anomaly_scores on the same inputs: the same
kernels over the same workspace layout, so node scores and top-K must agree
bit for bit.  Two calls in a row, the second on a smaller input (the fixed
device scratch keeps the first call's contents), then the documented errors:
a size beyond the fixed scratch and a map entry out of range."""

import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cdl():
    import paper_1802_05421_amd as cdl
    return cdl


def series(n, T, seed):
    return torch.from_numpy(np.random.default_rng(seed).standard_normal((n, T))).cuda()


def ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def noalloc(cdl, Z0, g0, Z1, g1, mode, top_k, map0=None, map1=None, m=None):
    from paper_1802_05421_amd import _lib
    L = _lib.load()
    from paper_1802_05421_amd.api import context
    ctx = context(Z0.device.index)
    m = m if m is not None else (map0.numel() if map0 is not None else g0.n)
    F = torch.full((m,), float("nan"), dtype=torch.float64, device=Z0.device)
    top = torch.full((max(top_k, 1),), -7, dtype=torch.int32, device=Z0.device)
    weighted = mode == "delta_a"
    st = L.cdl_anomaly_scores_noalloc(ctx.h, ptr(Z0), ptr(g0.W) if weighted else None, ptr(g0.stats),
                                      g0.n, ptr(Z1), ptr(g1.W) if weighted else None, ptr(g1.stats),
                                      g1.n, Z0.shape[1], ptr(map0), ptr(map1), m, _lib.MODE[mode],
                                      ptr(F), top_k, ptr(top))
    return st, F, top[:top_k], L.cdl_last_error(ctx.h).decode()


def test_noalloc_scores_equal_workspace_entry_point(cdl):
    # call 1: maps onto two snapshots of different sizes, weighted scores
    n0, n1, m, k = 2100, 2230, 2000, 40
    g0, g1 = cdl.build_graph(series(n0, 24, 1)), cdl.build_graph(series(n1, 24, 2))
    rng = np.random.default_rng(3)
    Z0 = torch.from_numpy(rng.standard_normal((n0, k)) * 1e-2).cuda()
    Z1 = torch.from_numpy(rng.standard_normal((n1, k)) * 1e-2).cuda()
    map0 = torch.from_numpy(np.sort(rng.choice(n0, m, replace=False)).astype(np.int32)).cuda()
    map1 = torch.from_numpy(np.sort(rng.choice(n1, m, replace=False)).astype(np.int32)).cuda()
    print("no-alloc call 1: m=%d k=%d delta_a with maps" % (m, k), flush=True)
    st, F, top, msg = noalloc(cdl, Z0, g0, Z1, g1, "delta_a", 50, map0, map1)
    assert st == 0, msg
    Fw, topw = cdl.anomaly_scores(Z0, g0, Z1, g1, mode="delta_a", top_k=50, map0=map0, map1=map1)
    torch.cuda.synchronize()
    assert torch.equal(F, Fw)
    assert torch.equal(top, topw)
    # call 2: smaller, identity maps, unweighted
    n, k2 = 700, 16
    h0, h1 = cdl.build_graph(series(n, 12, 4)), cdl.build_graph(series(n, 12, 5))
    Y0 = torch.from_numpy(rng.standard_normal((n, k2))).cuda()
    Y1 = torch.from_numpy(rng.standard_normal((n, k2))).cuda()
    print("no-alloc call 2: m=%d k=%d unweighted, identity" % (n, k2), flush=True)
    st, F2, top2, msg = noalloc(cdl, Y0, h0, Y1, h1, "unweighted", 20)
    assert st == 0, msg
    F2w, top2w = cdl.anomaly_scores(Y0, h0, Y1, h1, top_k=20)
    torch.cuda.synchronize()
    assert torch.equal(F2, F2w)
    assert torch.equal(top2, top2w)
    assert torch.isfinite(F2).all()


def test_noalloc_rejects_oversize_and_bad_maps(cdl):
    n, k = 300, 8
    g = cdl.build_graph(series(n, 6, 7))
    Z = torch.zeros((n, k), dtype=torch.float64, device="cuda")
    # m = 16384 at k = 320 needs more than the fixed scratch: rejected before
    # any kernel reads the (deliberately small) inputs
    from paper_1802_05421_amd import _lib
    L = _lib.load()
    from paper_1802_05421_amd.api import context
    ctx = context(0)
    F = torch.empty(16, dtype=torch.float64, device="cuda")
    Zb = torch.zeros((16, 320), dtype=torch.float64, device="cuda")
    st = L.cdl_anomaly_scores_noalloc(ctx.h, ptr(Zb), None, ptr(g.stats), 16384, ptr(Zb), None,
                                      ptr(g.stats), 16384, 320, None, None, 16384, 0, ptr(F), 0,
                                      None)
    assert st == 2, L.cdl_last_error(ctx.h).decode()       # CDL_E_WORKSPACE
    assert "scratch" in L.cdl_last_error(ctx.h).decode()
    # a map entry out of range: checked on the device, nothing scored
    bad = torch.arange(100, dtype=torch.int32, device="cuda")
    bad[37] = n
    good = torch.arange(100, dtype=torch.int32, device="cuda")
    st, _, _, msg = noalloc(cdl, Z, g, Z, g, "unweighted", 5, bad, good)
    assert st == 1 and "map" in msg                          # CDL_E_ARG
    st, _, _, msg = noalloc(cdl, Z, g, Z, g, "unweighted", 5, good, bad)
    assert st == 1
    # and a valid call afterwards still works
    st, F3, _, msg = noalloc(cdl, Z, g, Z, g, "unweighted", 5, good, good)
    assert st == 0, msg
    torch.cuda.synchronize()
    assert torch.all(F3 == 0)
