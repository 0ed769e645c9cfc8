"""MI355X (gfx950) commute-time anomaly detection for dense graph sequences.

The hot path - Gaussian-kernel graph, inverse-chain squarings, chain-
preconditioned FP64-refined multi-RHS Laplacian solve, fused all-pairs node
scores - runs in hand-written HIP kernels behind the C ABI of
include/caddelag.h (libcaddelag.so, built in-tree).  This package is the thin
torch binding: it allocates device buffers and passes pointers and streams.
Importing it loads the library and fails if it has not been built.
"""

from . import _lib

_lib.load()

from .api import (  # noqa: E402,F401
    Chain,
    Context,
    Graph,
    SeqParams,
    anomaly_edges,
    autotune_clear,
    autotune_entries,
    autotune_load,
    autotune_lookup,
    autotune_save,
    anomaly_scores,
    build_chain,
    chain_densify,
    device_copy,
    force_choice,
    build_graph,
    check_graph,
    graph_from_weights,
    ld,
    level,
    k_rp,
    level_scale,
    level_scale_for,
    rhs,
    score_sequence,
    sequence_workspace_bytes,
    set_autotune,
    set_select,
    set_solve_depth,
    set_timing,
    timing,
    solve_embedding,
    solve_embedding_pair,
    stream_embedding,
    stream_workspace_bytes,
    workspace_bytes,
)
from ._lib import CdlError  # noqa: E402,F401
