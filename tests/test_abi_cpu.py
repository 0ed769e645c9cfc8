"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and its host-side logic (sizes, layouts, argument checks, status
strings) behaves as documented."""

import ctypes as C
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "caddelag.h")


@pytest.fixture(scope="module")
def L():
    from paper_1802_05421_amd import _build, _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(L):
    from paper_1802_05421_amd import _lib
    names = _lib.declared_symbols(HEADER)
    assert len(names) >= 20
    lib = C.CDLL(os.path.join(ROOT, "paper_1802_05421_amd", "libcaddelag.so"))
    missing = [s for s in names if not hasattr(lib, s)]
    assert missing == []


def test_version_and_status_strings(L):
    assert L.cdl_version().decode().startswith("caddelag-gfx950")
    for code in range(9):
        assert L.cdl_status_string(code).decode() not in ("", "unknown status")
    assert L.cdl_status_string(99).decode() == "unknown status"
    assert L.cdl_last_error(None).decode() == "null context"


@pytest.mark.parametrize("n,ld", [(2, 256), (256, 256), (257, 512), (16384, 16384), (65536, 65536)])
def test_padded_layout(L, n, ld):
    assert L.cdl_ld(n) == ld
    assert L.cdl_matrix_bytes(n, 2) == ld * ld * 2
    assert L.cdl_matrix_bytes(n, 0) == ld * ld * 8
    assert L.cdl_matrix_bytes(n, 7) == 0


def sizes(L, n, T, k, dmax, prec):
    out = [C.c_size_t() for _ in range(4)]
    st = L.cdl_workspace_bytes(n, T, k, dmax, prec, *[C.byref(o) for o in out])
    return st, [o.value for o in out]


def test_workspace_sizes_and_validation(L):
    st, (g, c, s, sc) = sizes(L, 16384, 240, 256, 6, 2)
    assert st == 0
    ld = 16384
    assert g >= ld * 240 * 8                       # padded series panel
    assert c >= 6 * ld * ld * 2                    # six BF16 levels
    assert s >= 4 * 256 * ld * 8                   # Y, X, R, V panels
    assert sc >= 2 * ld * 512 * 8                  # two 2k-wide embedding panels
    assert all(v % 256 == 0 for v in (g, c, s, sc))
    # chain buffer = level offset + levels
    off = L.cdl_chain_level_offset(16384, 2)
    assert off > 0 and off % 256 == 0
    assert c == off + 6 * L.cdl_matrix_bytes(16384, 2)
    for bad in [(1, 240, 256, 6, 2), (16384, 0, 256, 6, 2), (16384, 240, 0, 6, 2),
                (16384, 240, 256, 0, 2), (16384, 240, 256, 15, 2), (16384, 240, 256, 6, 9),
                ((1 << 20) + 1, 240, 256, 6, 2)]:
        assert sizes(L, *bad)[0] == 1            # CDL_E_ARG
    # NULL outputs are allowed
    assert L.cdl_workspace_bytes(300, 10, 5, 2, 1, None, None, None, None) == 0


def test_stream_workspace_grows_linearly_in_n(L):
    def size(n, T, k, p, lev=-1):
        out = C.c_size_t()
        st = L.cdl_stream_workspace_bytes(n, T, k, p, lev, C.byref(out))
        return st, out.value
    # n = 2^18 with 8192-row panels: series, one panel and five k-wide panels;
    # the full weight matrix (512 GiB) is never part of it
    st, b = size(262144, 240, 256, 8192)
    ld = 262144
    assert st == 0 and b % 256 == 0
    assert b >= ld * 240 * 8 + 8192 * ld * 8 + 5 * 256 * ld * 8
    assert b < 2 * (ld * 240 * 8 + 8192 * ld * 8 + 5 * 256 * ld * 8)
    # panel rows: rounded up to 256, at most ld; 0 = default
    assert size(1000, 10, 4, 300)[1] == size(1000, 10, 4, 512)[1]
    assert size(1000, 10, 4, 10 ** 6)[1] == size(1000, 10, 4, 1024)[1]
    assert size(1000, 10, 4, 0)[1] == size(1000, 10, 4, 1024)[1]
    for bad in [(1, 10, 4, 0), (1000, 0, 4, 0), (1000, 10, 0, 0), (1000, 10, 4, -1),
                ((1 << 20) + 1, 10, 4, 0), (1000, 10, 4, 0, 4), (1000, 10, 4, 0, -2)]:
        assert size(*bad)[0] == 1
    assert L.cdl_stream_workspace_bytes(1000, 10, 4, 0, -1, None) == 1
    # with a stored FP16 level: the stored path's solve panels instead
    st, b16 = size(262144, 240, 256, 8192, 3)
    assert st == 0 and b16 >= ld * 240 * 8 + 8192 * ld * 8 + 8 * 256 * ld * 8


def test_calls_reject_a_null_context(L):
    # every entry point checks its context before touching a device
    assert L.cdl_build_graph(None, None, 10, 5, 5, 0.0, None, None, None, None, 0) == 1
    assert L.cdl_check_graph(None, None, None, 10, None) == 1
    assert L.cdl_graph_from_weights(None, None, 10, 10, None, None, None, None, 0) == 1
    assert L.cdl_build_chain(None, None, None, None, 10, 2, 0, 4, 0.0, 0, None, 0, None) == 1
    assert L.cdl_solve_embedding(None, None, None, None, None, 10, None, None, 4, 0.0, 1, 0,
                                 1e-8, 5, None, None, 0, None) == 1
    assert L.cdl_anomaly_scores(None, None, None, None, 10, None, None, None, 10, 4, None,
                                None, 10, 0, None, 5, None, None, 0) == 1
    assert L.cdl_ctx_set_stream(None, None) == 1
    assert L.cdl_ctx_set_timing(None, 1) == 1
    assert L.cdl_ctx_set_timing_only(None, b"rhs") == 1
    assert L.cdl_ctx_set_solve_depth(None, 2) == 1
    assert L.cdl_ctx_set_select(None, 0) == 1
    assert L.cdl_chain_densify(None, 100, None, 0, None) == 1
    assert L.cdl_solve_embedding_pair(None, None, None, None, None, None, None, None, None, None,
                                      None, None, 10, 4, 1, 0, 1e-8, 5, None, None, None, None, 0,
                                      None, None) == 1
    assert L.cdl_stream_embedding(None, None, 10, 5, 5, 0.0, None, 4, 1, 1e-8, 5, 0, -1, None, 0,
                                  None, None, None, None, None, 0, None) == 1
    assert L.cdl_timing_reset(None) == 1
    assert L.cdl_ctx_destroy(None) == 0


def test_context_creation_without_a_device_fails_cleanly(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert L.cdl_ctx_create(0, None, C.byref(h)) == 1
    assert L.cdl_ctx_create(0, None, None) == 1


def test_sequence_workspace_validation(L):
    from paper_1802_05421_amd import _lib
    snaps = (_lib.Snapshot * 2)()
    for t in range(2):
        snaps[t].n, snaps[t].T, snaps[t].ldx = 1000 + 500 * t, 120, 120
    p = _lib.SeqParams(k=128, seed=7, sigma=0.0, prec=2, depth=0, depth_max=6, chain_eps=0.0,
                       solver=0, tol=-1e-6, max_iter=20, mode=0, top_k=50)
    nb = C.c_size_t()
    assert L.cdl_sequence_workspace_bytes(2, snaps, C.byref(p), C.byref(nb)) == 0
    st, (g, c, s, sc) = sizes(L, 1500, 120, 128, 6, 2)
    assert nb.value >= g + c + s + sc + 2 * L.cdl_matrix_bytes(1500, 0)
    assert L.cdl_sequence_workspace_bytes(1, snaps, C.byref(p), C.byref(nb)) == 1
    snaps[1].n = 1
    assert L.cdl_sequence_workspace_bytes(2, snaps, C.byref(p), C.byref(nb)) == 1


def test_package_import_fails_loudly_without_library(tmp_path):
    # The binding refuses to run without the native library (no fallback).
    import subprocess
    import sys
    code = ("import sys, os; sys.path.insert(0, %r)\n"
            "import paper_1802_05421_amd._build as b\n"
            "b.LIB = %r\n"
            "import paper_1802_05421_amd._lib as l\n"
            "l.LIB = %r\n"
            "l._lib = None\n"
            "try:\n    l.load()\nexcept ImportError as e:\n    print('refused', e)\n") % (
        ROOT, str(tmp_path / "missing.so"), str(tmp_path / "missing.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "refused" in out.stdout


def test_k_rp_and_level_scale_queries(L):
    import math
    k = C.c_int64()
    assert L.cdl_k_rp(16384, 1e-2, C.byref(k)) == 0
    assert k.value == math.ceil(math.log(16384 / 1e-2)) == 15
    for n, eps in [(1, 0.1), (100, 0.0), (100, 1.0), (100, -0.5), (100, float("nan"))]:
        assert L.cdl_k_rp(n, eps, C.byref(k)) == 1          # CDL_E_ARG
    assert L.cdl_k_rp(100, 0.1, None) == 1
    s = C.c_double()
    for n, want in [(1, 1.0), (2, 2.0), (300, 256.0), (16384, 16384.0), (16385, 16384.0)]:
        assert L.cdl_level_scale(n, 3, C.byref(s)) == 0 and s.value == want
        for p in (0, 1, 2):
            assert L.cdl_level_scale(n, p, C.byref(s)) == 0 and s.value == 1.0
    assert L.cdl_level_scale(0, 3, C.byref(s)) == 1
    assert L.cdl_level_scale(10, 4, C.byref(s)) == 1
    assert L.cdl_level_scale(10, 3, None) == 1


def test_autotune_table_json_round_trip(L, tmp_path):
    # without a GPU the table's architecture is "none" (device < 0)
    assert L.cdl_autotune_clear() == 0
    src = tmp_path / "tune.json"
    src.write_text(
        '{"format": "caddelag-autotune-1", "entries": ['
        '{"arch": "none", "key": "square/bf16/ld16384", "choice": 1, "ms": [4.8, 4.3, 5.3, 5.0]},'
        '{"arch": "none", "key": "apply/fp16/ld16384/k256", "choice": 2, "ms": [0.20, 0.24, 0.18]},'
        '{"arch": "gfx950:sramecc+:xnack-", "key": "residual/fp64/ld16384/k256", "choice": 0,'
        ' "ms": [2.2, 2.4, 2.3]}]}')
    assert L.cdl_autotune_load(str(src).encode()) == 0
    assert L.cdl_autotune_entries() == 3
    ch, nc, ms = C.c_int(), C.c_int(), C.c_double()

    def look(fam, prec, n, k):
        return L.cdl_autotune_lookup(-1, fam, prec, n, k, C.byref(ch), C.byref(nc), C.byref(ms))

    assert look(b"square", 2, 16384, 0) == 0 and (ch.value, nc.value, ms.value) == (1, 4, 4.3)
    assert look(b"square", 2, 16300, 0) == 0            # same padded shape (ld 16384)
    assert look(b"apply", 3, 16384, 250) == 0 and (ch.value, ms.value) == (2, 0.18)   # k pads to 256
    assert look(b"residual", 0, 16384, 256) == 8         # another architecture's entry
    assert look(b"square", 3, 16384, 0) == 8             # no FP16 squaring entry
    assert look(b"nonsense", 2, 16384, 0) == 1
    assert look(b"apply", 2, 16384, 0) == 1               # apply needs k
    out = tmp_path / "out.json"
    assert L.cdl_autotune_save(str(out).encode()) == 0
    assert L.cdl_autotune_clear() == 0 and L.cdl_autotune_entries() == 0
    assert L.cdl_autotune_load(str(out).encode()) == 0 and L.cdl_autotune_entries() == 3
    assert look(b"apply", 3, 16384, 256) == 0 and (ch.value, nc.value) == (2, 3)
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "something else", "entries": []}')
    assert L.cdl_autotune_load(str(bad).encode()) == 1
    bad.write_text('{"format": "caddelag-autotune-1", "entries": [')
    assert L.cdl_autotune_load(str(bad).encode()) == 1
    assert L.cdl_autotune_load(str(tmp_path / "missing.json").encode()) == 1
    assert L.cdl_autotune_clear() == 0


def test_sequence_id_cache_follows_the_tensors():
    """The binding's cached host/device copies of global ids: reused while the
    tensor is unchanged, refreshed after an in-place write, dropped when the
    tensor is freed (so a new tensor at a reused address never sees them)."""
    import gc

    import torch

    from paper_1802_05421_amd import api
    cpu = torch.device("cpu")
    g = torch.arange(16, dtype=torch.int64)
    h, d = api._gid_copies(g, cpu)
    assert h.dtype == torch.int32 and api._gid_copies(g, cpu)[0] is h
    g[3] = 99
    h2, _ = api._gid_copies(g, cpu)
    assert h2 is not h and int(h2[3]) == 99
    n = len(api._gid_cache)
    del g, h, d, h2, _
    gc.collect()
    assert len(api._gid_cache) == n - 1
