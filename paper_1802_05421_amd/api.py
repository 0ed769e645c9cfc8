"""Thin torch-facing binding of libcaddelag (same call names as the C ABI).

Every step runs in the library's HIP kernels; this module only allocates
device buffers with torch, passes raw pointers and the current HIP stream,
and turns status codes into exceptions.  There is no CPU or PyTorch compute
fallback: if the library is missing, importing the package fails.
"""

from __future__ import annotations

import ctypes as C
import weakref
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _lib as L

_ctx_cache = {}


def _lib():
    return L.load()


def _check(status: int, ctx=None):
    if status != 0:
        msg = _lib().cdl_last_error(ctx).decode() if ctx else ""
        raise L.CdlError(status, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        h = C.c_void_p()
        _check(_lib().cdl_ctx_create(device, C.c_void_p(s.cuda_stream), C.byref(h)))
        self.h = h

    def sync_stream(self):
        """Follow torch's current stream of the device."""
        s = torch.cuda.current_stream(self.device)
        if s.cuda_stream != self._stream.cuda_stream:
            _check(_lib().cdl_ctx_set_stream(self.h, C.c_void_p(s.cuda_stream)), self.h)
            self._stream = s

    def __del__(self):
        try:
            if getattr(self, "h", None) and L._lib is not None:
                L._lib.cdl_ctx_destroy(self.h)
        except Exception:
            pass


def set_solve_depth(depth: int, device: int = 0):
    """Force the total chain depth of every solve iteration (0 = autotune)."""
    ctx = context(device)
    _check(_lib().cdl_ctx_set_solve_depth(ctx.h, int(depth)), ctx.h)


def set_select(mode: int, device: int = 0):
    """Median selection of later graph builds: 0 bracketed (default), 1 radix over the matrix."""
    ctx = context(device)
    _check(_lib().cdl_ctx_set_select(ctx.h, int(mode)), ctx.h)


def set_timing(enable: bool, device: int = 0, only=None):
    """Per-kernel HIP-event timing on the context's stream (see include/caddelag.h);
    `only`: kernel names to time (None: every kernel)."""
    ctx = context(device)
    names = None if only is None else ",".join(only).encode()
    _check(_lib().cdl_ctx_set_timing_only(ctx.h, names), ctx.h)
    _check(_lib().cdl_ctx_set_timing(ctx.h, int(enable)), ctx.h)


def timing(device: int = 0, reset: bool = False) -> dict:
    """{kernel name: (launches, total ms)} accumulated since the last reset."""
    ctx = context(device)
    out, i = {}, 0
    nm, cnt, ms = C.c_char_p(), C.c_int64(), C.c_double()
    while _lib().cdl_timing_read(ctx.h, i, C.byref(nm), C.byref(cnt), C.byref(ms)) == 0:
        out[nm.value.decode()] = (cnt.value, ms.value)
        i += 1
    if reset:
        _check(_lib().cdl_timing_reset(ctx.h), ctx.h)
    return out


def set_autotune(enable: bool, device: int = 0):
    """Time every launch candidate of a tuned kernel family on first use of a
    shape (cdl_ctx_set_autotune)."""
    ctx = context(device)
    _check(_lib().cdl_ctx_set_autotune(ctx.h, 1 if enable else 0), ctx.h)


def force_choice(family: str, choice: int, device: int = 0):
    """Pin a tuned kernel family to one candidate on this stream's context (-1 releases)."""
    ctx = context(device)
    _check(_lib().cdl_ctx_force_choice(ctx.h, family.encode(), int(choice)), ctx.h)


def autotune_lookup(family: str, prec: str, n: int, k: int = 0, device: int = 0):
    """(choice, candidates, ms) of the tuning table's entry, or None."""
    ch, nc, ms = C.c_int(), C.c_int(), C.c_double()
    st = _lib().cdl_autotune_lookup(device, family.encode(), L.PREC[prec], int(n), int(k),
                                    C.byref(ch), C.byref(nc), C.byref(ms))
    if st == 8:
        return None
    _check(st)
    return ch.value, nc.value, ms.value


def autotune_save(path: str):
    _check(_lib().cdl_autotune_save(path.encode()))


def autotune_load(path: str):
    _check(_lib().cdl_autotune_load(path.encode()))


def autotune_clear():
    _check(_lib().cdl_autotune_clear())


def autotune_entries() -> int:
    return int(_lib().cdl_autotune_entries())


def context(device: int = 0) -> Context:
    """The library context for torch's current stream on `device`.

    One context per (device, stream): calls made from different host threads
    on different streams never share a context.
    """
    s = torch.cuda.current_stream(device)
    key = (device, s.cuda_stream)
    c = _ctx_cache.get(key)
    if c is None:
        c = Context(device, s)
        _ctx_cache[key] = c
    return c


def ld(n: int) -> int:
    return int(_lib().cdl_ld(n))


def workspace_bytes(n: int, T: int, k: int, depth_max: int = 14, prec: str = "bf16"):
    g, c, s, sc = C.c_size_t(), C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(_lib().cdl_workspace_bytes(n, T, k, depth_max, L.PREC[prec], C.byref(g), C.byref(c),
                                      C.byref(s), C.byref(sc)))
    return dict(graph=g.value, chain=c.value, solve=s.value, score=sc.value)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


@dataclass
class Graph:
    W: Optional[torch.Tensor]  # (ld, ld) float64, padded (None for streamed snapshots)
    deg: torch.Tensor        # (n,) float64
    stats: torch.Tensor      # (4,) float64: vol, sigma, deg_min, deg_max
    n: int
    chain: Optional["Chain"] = None   # streamed snapshots with a stored level

    def host_stats(self):
        s = self.stats.cpu().tolist()
        return dict(vol=s[0], sigma=s[1], deg_min=s[2], deg_max=s[3])


@dataclass
class Chain:
    buf: torch.Tensor
    info: L.ChainInfo
    n: int

    @property
    def depth(self) -> int:
        return self.info.depth

    @property
    def fro(self) -> List[float]:
        return [self.info.fro[i] for i in range(self.info.depth)]

    @property
    def dense_levels(self) -> int:
        return self.info.dense_levels


def build_graph(X: torch.Tensor, sigma: Optional[float] = None, ws: Optional[torch.Tensor] = None,
                out: Optional[Graph] = None, check: bool = True) -> Graph:
    """Gaussian-kernel graph of one snapshot; X is (n, T) float64 on the GPU."""
    if X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a CUDA float64 matrix with unit column stride")
    ctx = context(X.device.index)
    n, T = X.shape
    m = ld(n)
    if out is None:
        out = Graph(W=torch.empty((m, m), dtype=torch.float64, device=X.device),
                    deg=torch.empty(n, dtype=torch.float64, device=X.device),
                    stats=torch.empty(L.CDL_GRAPH_STATS, dtype=torch.float64, device=X.device), n=n)
    need = workspace_bytes(n, T, 1, 1, "fp64")["graph"]
    if ws is None or ws.numel() < need:
        ws = _ws(need, X.device)
    _check(_lib().cdl_build_graph(ctx.h, _ptr(X), n, T, X.stride(0),
                                  float(sigma) if sigma else 0.0, _ptr(out.W), _ptr(out.deg),
                                  _ptr(out.stats), _ptr(ws), ws.numel()), ctx.h)
    if check:
        check_graph(out)
    return out


def check_graph(g: Graph) -> dict:
    ctx = context(g.W.device.index)
    h = (C.c_double * L.CDL_GRAPH_STATS)()
    _check(_lib().cdl_check_graph(ctx.h, _ptr(g.deg), _ptr(g.stats), g.n, h), ctx.h)
    return dict(vol=h[0], sigma=h[1], deg_min=h[2], deg_max=h[3])


def graph_from_weights(Win: torch.Tensor) -> Graph:
    if Win.dtype != torch.float64 or not Win.is_cuda or Win.dim() != 2 or Win.stride(1) != 1:
        raise ValueError("weights must be a CUDA float64 matrix with unit column stride")
    ctx = context(Win.device.index)
    n = Win.shape[0]
    m = ld(n)
    g = Graph(W=torch.empty((m, m), dtype=torch.float64, device=Win.device),
              deg=torch.empty(n, dtype=torch.float64, device=Win.device),
              stats=torch.empty(L.CDL_GRAPH_STATS, dtype=torch.float64, device=Win.device), n=n)
    ws = _ws(256, Win.device)
    _check(_lib().cdl_graph_from_weights(ctx.h, _ptr(Win), n, Win.stride(0), _ptr(g.W),
                                         _ptr(g.deg), _ptr(g.stats), _ptr(ws), ws.numel()), ctx.h)
    return g


def build_chain(g: Graph, prec: str = "bf16", depth: int = 0, depth_max: int = 14,
                chain_eps: float = 0.0, lazy: bool = False,
                buf: Optional[torch.Tensor] = None) -> Chain:
    ctx = context(g.W.device.index)
    need = workspace_bytes(g.n, 1, 1, depth_max, prec)["chain"]
    if buf is None or buf.numel() < need:
        buf = _ws(need, g.W.device)
    info = L.ChainInfo()
    _check(_lib().cdl_build_chain(ctx.h, _ptr(g.W), _ptr(g.deg), _ptr(g.stats), g.n,
                                  L.PREC[prec], depth, depth_max, chain_eps, int(lazy),
                                  _ptr(buf), buf.numel(), C.byref(info)), ctx.h)
    return Chain(buf=buf, info=info, n=g.n)


def chain_densify(chain: Chain) -> Chain:
    """Replace the levels by Q = prod_l (I + S~^{2^l}) - I (Algorithm 2's
    dense schedule; see cdl_chain_densify).  Grows the buffer when it has no
    scratch level."""
    ctx = context(chain.buf.device.index)
    d = chain.info.depth
    need = workspace_bytes(chain.n, 1, 1, d + 1 if d >= 2 else 1, L.PREC_NAME[chain.info.prec])["chain"]
    if chain.buf.numel() < need:
        buf = _ws(need, chain.buf.device)
        buf[:chain.buf.numel()].copy_(chain.buf)
        chain.buf = buf
    _check(_lib().cdl_chain_densify(ctx.h, chain.n, _ptr(chain.buf), chain.buf.numel(),
                                    C.byref(chain.info)), ctx.h)
    return chain


def level(chain: Chain, l: int) -> torch.Tensor:
    """View of stored chain level l as an (ld, ld) tensor (for inspection)."""
    prec = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float16}[chain.info.prec]
    m = ld(chain.n)
    off = int(_lib().cdl_chain_level_offset(chain.n, chain.info.prec))
    lb = int(_lib().cdl_matrix_bytes(chain.n, chain.info.prec))
    raw = chain.buf[off + l * lb: off + (l + 1) * lb]
    return raw.view(prec).view(m, m)


def device_copy(src: torch.Tensor, dst: torch.Tensor):
    """dst <- src bytewise on the current stream with the library's plain copy
    kernel (cdl_device_copy): the bandwidth and byte-counter reference."""
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("device_copy: contiguous tensors only")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("device_copy: sizes differ")
    ctx = context(src.device.index or 0)
    _check(_lib().cdl_device_copy(ctx.h, _ptr(src), _ptr(dst), nb), ctx.h)


def level_scale(chain: Chain) -> float:
    """Storage scale of the chain's levels (cdl_level_scale)."""
    out = C.c_double()
    _check(_lib().cdl_level_scale(chain.n, chain.info.prec, C.byref(out)))
    return out.value


def level_scale_for(n: int, prec: str) -> float:
    """Storage scale of chain levels of type `prec` for n nodes (cdl_level_scale)."""
    out = C.c_double()
    _check(_lib().cdl_level_scale(int(n), L.PREC[prec], C.byref(out)))
    return out.value


def k_rp(n: int, eps_rp: float) -> int:
    """Algorithm 1's number of projections for n nodes and accuracy eps_rp (cdl_k_rp)."""
    out = C.c_int64()
    _check(_lib().cdl_k_rp(int(n), float(eps_rp), C.byref(out)))
    return out.value


def solve_embedding(g: Graph, chain: Chain, k: int, seed: int, tol: float = 1e-8,
                    max_iter: int = 30, gid: Optional[torch.Tensor] = None,
                    solver: str = "richardson", eps_rp: float = 0.0,
                    ws: Optional[torch.Tensor] = None, Z: Optional[torch.Tensor] = None,
                    raise_noconv: bool = True):
    """Embedding Z (n, k) float64 with L Z = Y to relative residual tol."""
    ctx = context(g.W.device.index)
    kk = k if k > 0 else k_rp(g.n, eps_rp)
    need = workspace_bytes(g.n, 1, kk, max(chain.info.depth, 1), L.PREC_NAME[chain.info.prec])["solve"]
    if ws is None or ws.numel() < need:
        ws = _ws(need, g.W.device)
    if Z is None:
        Z = torch.empty((g.n, kk), dtype=torch.float64, device=g.W.device)
    if gid is not None and (gid.dtype != torch.int32 or not gid.is_cuda):
        raise ValueError("gid must be a CUDA int32 vector")
    info = L.SolveInfo()
    st = _lib().cdl_solve_embedding(ctx.h, _ptr(g.W), _ptr(g.deg), _ptr(g.stats), _ptr(gid), g.n,
                                    _ptr(chain.buf), C.byref(chain.info), kk, float(eps_rp),
                                    C.c_uint64(seed), L.SOLVER[solver], float(tol), max_iter,
                                    _ptr(Z), _ptr(ws), ws.numel(), C.byref(info))
    if st != 0 and not (st == 6 and not raise_noconv):
        _check(st, ctx.h)
    return Z, info


def solve_embedding_pair(g0: Graph, chain0: Chain, g1: Graph, chain1: Chain, k: int, seed: int,
                         tol: float = 1e-8, max_iter: int = 30,
                         gid: Optional[torch.Tensor] = None, solver: str = "richardson",
                         ws: Optional[tuple] = None, Z: Optional[tuple] = None,
                         raise_noconv: bool = True):
    """Embeddings of both snapshots of a pair on one node set, their
    right-hand sides made in one sweep (cdl_solve_embedding_pair).
    Returns (Z0, Z1, info0, info1)."""
    if g0.n != g1.n:
        raise ValueError("the two snapshots need the same node set")
    dev = g0.W.device
    ctx = context(dev.index)
    need = max(workspace_bytes(g0.n, 1, k, max(c.info.depth, 1), L.PREC_NAME[c.info.prec])["solve"]
               for c in (chain0, chain1))
    if ws is None or min(w.numel() for w in ws) < need:
        ws = (_ws(need, dev), _ws(need, dev))
    if Z is None:
        Z = (torch.empty((g0.n, k), dtype=torch.float64, device=dev),
             torch.empty((g0.n, k), dtype=torch.float64, device=dev))
    if gid is not None and (gid.dtype != torch.int32 or not gid.is_cuda):
        raise ValueError("gid must be a CUDA int32 vector")
    i0, i1 = L.SolveInfo(), L.SolveInfo()
    st = _lib().cdl_solve_embedding_pair(
        ctx.h, _ptr(g0.W), _ptr(g0.deg), _ptr(g0.stats), _ptr(chain0.buf), C.byref(chain0.info),
        _ptr(g1.W), _ptr(g1.deg), _ptr(g1.stats), _ptr(chain1.buf), C.byref(chain1.info),
        _ptr(gid), g0.n, k, C.c_uint64(seed), L.SOLVER[solver], float(tol), max_iter,
        _ptr(Z[0]), _ptr(Z[1]), _ptr(ws[0]), _ptr(ws[1]), min(w.numel() for w in ws),
        C.byref(i0), C.byref(i1))
    if st != 0 and not (st == 6 and not raise_noconv):
        _check(st, ctx.h)
    return Z[0], Z[1], i0, i1


def rhs(g: Graph, k: int, seed: int, gid: Optional[torch.Tensor] = None,
        g1: Optional[Graph] = None):
    """Algorithm 1's right-hand sides Y (n, k) float64 of g, as the solves make
    them (cdl_rhs); with g1 (the same node set) the pair (Y0, Y1) in one sweep."""
    dev = g.W.device
    if g1 is not None and g1.n != g.n:
        raise ValueError("the two graphs need the same node set")
    if gid is not None and (gid.dtype != torch.int32 or not gid.is_cuda):
        raise ValueError("gid must be a CUDA int32 vector")
    ctx = context(dev.index)
    need = C.c_size_t()
    _check(_lib().cdl_rhs_workspace_bytes(g.n, k, int(g1 is not None), C.byref(need)))
    ws = _ws(need.value, dev)
    Y0 = torch.empty((g.n, k), dtype=torch.float64, device=dev)
    Y1 = None if g1 is None else torch.empty((g.n, k), dtype=torch.float64, device=dev)
    _check(_lib().cdl_rhs(ctx.h, _ptr(g.W), None if g1 is None else _ptr(g1.W), _ptr(gid), g.n, k,
                          C.c_uint64(seed), _ptr(Y0), _ptr(Y1), _ptr(ws), ws.numel()), ctx.h)
    return Y0 if g1 is None else (Y0, Y1)


def stream_workspace_bytes(n: int, T: int, k: int, panel_rows: int = 0,
                           level: Optional[str] = None) -> int:
    out = C.c_size_t()
    _check(_lib().cdl_stream_workspace_bytes(n, T, k, panel_rows,
                                             -1 if level is None else L.PREC[level], C.byref(out)))
    return out.value


def stream_embedding(X: torch.Tensor, k: int, seed: int, sigma: Optional[float] = None,
                     gid: Optional[torch.Tensor] = None, tol: float = 1e-8, max_iter: int = 30,
                     panel_rows: int = 0, level: Optional[str] = None,
                     ws: Optional[torch.Tensor] = None, chain_buf: Optional[torch.Tensor] = None,
                     Z: Optional[torch.Tensor] = None, raise_noconv: bool = True):
    """Graph and embedding of one snapshot with no n x n FP64 matrix in
    memory: the weights are recomputed from X row panel by row panel on every
    sweep (cdl_stream_embedding).  level (e.g. "fp16") stores chain level 0 in
    that type and solves as solve_embedding does.  Returns (Graph with W =
    None and, with a level, .chain set; Z; info); the graph serves
    anomaly_scores in the unweighted mode."""
    if X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a CUDA float64 matrix with unit column stride")
    if gid is not None and (gid.dtype != torch.int32 or not gid.is_cuda):
        raise ValueError("gid must be a CUDA int32 vector")
    ctx = context(X.device.index)
    n, T = X.shape
    need = stream_workspace_bytes(n, T, k, panel_rows, level)
    if ws is None or ws.numel() < need:
        ws = _ws(need, X.device)
    chain = None
    cinfo = L.ChainInfo()
    if level is not None:
        cneed = workspace_bytes(n, 1, 1, 1, level)["chain"]
        if chain_buf is None or chain_buf.numel() < cneed:
            chain_buf = _ws(cneed, X.device)
        chain = Chain(buf=chain_buf, info=cinfo, n=n)
    if Z is None:
        Z = torch.empty((n, k), dtype=torch.float64, device=X.device)
    g = Graph(W=None, deg=torch.empty(n, dtype=torch.float64, device=X.device),
              stats=torch.empty(L.CDL_GRAPH_STATS, dtype=torch.float64, device=X.device), n=n,
              chain=chain)
    info = L.SolveInfo()
    st = _lib().cdl_stream_embedding(ctx.h, _ptr(X), n, T, X.stride(0),
                                     float(sigma) if sigma else 0.0, _ptr(gid), k,
                                     C.c_uint64(seed), float(tol), max_iter, panel_rows,
                                     -1 if level is None else L.PREC[level],
                                     _ptr(chain_buf) if level is not None else None,
                                     chain_buf.numel() if level is not None else 0,
                                     C.byref(cinfo), _ptr(g.deg), _ptr(g.stats), _ptr(Z),
                                     _ptr(ws), ws.numel(), C.byref(info))
    if st != 0 and not (st == 6 and not raise_noconv):
        _check(st, ctx.h)
    return g, Z, info


def anomaly_scores(Z0: torch.Tensor, g0: Graph, Z1: torch.Tensor, g1: Graph,
                   mode: str = "unweighted", top_k: int = 50,
                   map0: Optional[torch.Tensor] = None, map1: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, F: Optional[torch.Tensor] = None,
                   top: Optional[torch.Tensor] = None):
    ctx = context(Z0.device.index)
    k = Z0.shape[1]
    m = map0.numel() if map0 is not None else g0.n
    need = workspace_bytes(max(m, 2), 1, k, 1, "fp64")["score"]
    if ws is None or ws.numel() < need:
        ws = _ws(need, Z0.device)
    if F is None:
        F = torch.empty(m, dtype=torch.float64, device=Z0.device)
    if top is None:
        top = torch.empty(max(top_k, 1), dtype=torch.int32, device=Z0.device)
    weighted = mode == "delta_a"
    _check(_lib().cdl_anomaly_scores(ctx.h, _ptr(Z0), _ptr(g0.W) if weighted else None,
                                     _ptr(g0.stats), g0.n, _ptr(Z1),
                                     _ptr(g1.W) if weighted else None, _ptr(g1.stats), g1.n, k,
                                     _ptr(map0), _ptr(map1), m, L.MODE[mode], _ptr(F), top_k,
                                     _ptr(top), _ptr(ws), ws.numel()), ctx.h)
    return F, top[:top_k]


def anomaly_edges(Z0: torch.Tensor, g0: Graph, Z1: torch.Tensor, g1: Graph,
                  top_k: int = 50, mode: str = "unweighted",
                  map0: Optional[torch.Tensor] = None, map1: Optional[torch.Tensor] = None,
                  ws: Optional[torch.Tensor] = None):
    """Node scores and the top_k edges (a < b) by omega |c_0(a,b) - c_1(a,b)|.

    Returns (F, a, b, value): F over the m common nodes, and the edges as
    common-node index pairs sorted by descending score, ties by (a, b).
    """
    ctx = context(Z0.device.index)
    k = Z0.shape[1]
    m = map0.numel() if map0 is not None else g0.n
    nb = C.c_size_t()
    _check(_lib().cdl_edges_workspace_bytes(m, k, top_k, C.byref(nb)))
    if ws is None or ws.numel() < nb.value:
        ws = _ws(nb.value, Z0.device)
    F = torch.empty(m, dtype=torch.float64, device=Z0.device)
    ea = torch.empty(top_k, dtype=torch.int32, device=Z0.device)
    eb = torch.empty(top_k, dtype=torch.int32, device=Z0.device)
    ev = torch.empty(top_k, dtype=torch.float64, device=Z0.device)
    weighted = mode == "delta_a"
    _check(_lib().cdl_anomaly_edges(ctx.h, _ptr(Z0), _ptr(g0.W) if weighted else None,
                                    _ptr(g0.stats), g0.n, _ptr(Z1),
                                    _ptr(g1.W) if weighted else None, _ptr(g1.stats), g1.n, k,
                                    _ptr(map0), _ptr(map1), m, L.MODE[mode], _ptr(F), top_k,
                                    _ptr(ea), _ptr(eb), _ptr(ev), _ptr(ws), ws.numel()), ctx.h)
    return F, ea, eb, ev


@dataclass
class SeqParams:
    k: int = 128
    seed: int = 7
    sigma: float = 0.0
    prec: str = "bf16"
    depth: int = 0
    depth_max: int = 14
    chain_eps: float = 0.0
    solver: str = "richardson"
    tol: float = 1e-8
    max_iter: int = 30
    mode: str = "unweighted"
    top_k: int = 50
    # No host reads inside the sequence (fixed depth, exactly max_iter
    # Richardson steps), snapshots alternating over two streams.
    asynchronous: bool = False
    # With asynchronous: a repeat of the previous call replays a HIP graph.
    graph: bool = False
    # With asynchronous: one pass with grouped launches over all snapshots
    # and pairs, convergence tested on the device (max_iter an upper bound).
    batched: bool = False


# Host and device int32 copies of global-id tensors, so that repeated calls
# on the same ids copy nothing.  An entry is keyed by the tensor object (a
# weak reference: the entry goes when the tensor does, so a later tensor at
# the same address never meets it) and holds its version counter (an
# in-place write bumps it and invalidates the entry).
_gid_cache: dict = {}


def _gid_copies(g: torch.Tensor, dev):
    key = id(g)
    hit = _gid_cache.get(key)
    if hit is not None and hit[0]() is g and hit[1] == g._version and hit[2] == dev:
        return (g if hit[3] is None else hit[3]), (g if hit[4] is None else hit[4])
    host = g.cpu().to(torch.int32).contiguous()
    devc = g.to(device=dev, dtype=torch.int32).contiguous()
    ref = weakref.ref(g, lambda _r, k=key: _gid_cache.pop(k, None))
    # a copy that is the tensor itself is not held (that would keep it alive)
    _gid_cache[key] = (ref, g._version, dev, None if host is g else host, None if devc is g else devc)
    return host, devc


def _seq_args(Xs, gids, p: SeqParams):
    dev = Xs[0].device
    n_snap = len(Xs)
    pairs = [_gid_copies(g, dev) for g in gids]
    gid_host = [h for h, _ in pairs]
    gid_dev = [d for _, d in pairs]
    snaps = (L.Snapshot * n_snap)()
    for t, X in enumerate(Xs):
        snaps[t].X = X.data_ptr()
        snaps[t].n, snaps[t].T = X.shape
        snaps[t].ldx = X.stride(0)
        snaps[t].gid = gid_dev[t].data_ptr()
        snaps[t].gid_host = gid_host[t].data_ptr()
    q = L.SeqParams(k=p.k, seed=p.seed, sigma=p.sigma, prec=L.PREC[p.prec], depth=p.depth,
                    depth_max=p.depth_max, chain_eps=p.chain_eps, solver=L.SOLVER[p.solver],
                    tol=p.tol, max_iter=p.max_iter, mode=L.MODE[p.mode], top_k=p.top_k,
                    flags=(1 if p.asynchronous else 0) | (2 if p.graph else 0) |
                    (4 if p.batched else 0))
    return snaps, q, gid_host, gid_dev


def sequence_workspace_bytes(Xs: Sequence[torch.Tensor], gids: Sequence[torch.Tensor],
                             p: SeqParams) -> int:
    snaps, q, _, _ = _seq_args(Xs, gids, p)
    nb = C.c_size_t()
    _check(_lib().cdl_sequence_workspace_bytes(len(Xs), snaps, C.byref(q), C.byref(nb)))
    return nb.value


def score_sequence(Xs: Sequence[torch.Tensor], gids: Sequence[torch.Tensor], p: SeqParams,
                   ws: Optional[torch.Tensor] = None, out=None):
    """Scores of every consecutive pair of snapshots (common global ids).

    out: (Fs, tops) from an earlier call with the same snapshots, written in
    place (an asynchronous repeat then replays its graph)."""
    dev = Xs[0].device
    ctx = context(dev.index)
    n_snap = len(Xs)
    snaps, q, gid_host, gid_dev = _seq_args(Xs, gids, p)
    nb = C.c_size_t()
    _check(_lib().cdl_sequence_workspace_bytes(n_snap, snaps, C.byref(q), C.byref(nb)))
    if ws is None or ws.numel() < nb.value:
        ws = _ws(nb.value, dev)
    if out is not None:
        Fs, tops = out
        tops = [t._base if t._base is not None else t for t in tops]
    else:
        Fs, tops = [], []
        for t in range(n_snap - 1):
            a = set(gid_host[t].tolist())
            m = sum(1 for v in gid_host[t + 1].tolist() if v in a)
            Fs.append(torch.empty(m, dtype=torch.float64, device=dev))
            tops.append(torch.empty(max(1, min(p.top_k, m)), dtype=torch.int32, device=dev))
    Fp = (C.c_void_p * (n_snap - 1))(*[f.data_ptr() for f in Fs])
    Tp = (C.c_void_p * (n_snap - 1))(*[t.data_ptr() for t in tops])
    info = L.SeqInfo()
    _check(_lib().cdl_score_sequence(ctx.h, n_snap, snaps, C.byref(q), Fp, Tp, _ptr(ws),
                                     ws.numel(), C.byref(info)), ctx.h)
    return Fs, [t[:min(p.top_k, f.numel())] for t, f in zip(tops, Fs)], info
