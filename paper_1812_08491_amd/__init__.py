"""MI355X (gfx950) PC-stable skeleton: HIP kernels behind the C ABI of include/pc.h.

The compute path is libpc.so; this package only marshals arguments (see _lib.py) and offers a
convenience wrapper, :func:`skeleton`, that allocates the buffers with torch and decodes results.
"""
from __future__ import annotations

from ._lib import (PC_MAX_LEVEL, PC_MLP_PARAMS, PCError, Context, bits_to_dense, decode_sepsets,
                   default_options, dense_to_bits, lib, pc_comb_unrank, pc_run_stats, pc_threshold,
                   pc_tuning, pc_workspace_bytes, status_str)

__all__ = ["PC_MAX_LEVEL", "PC_MLP_PARAMS", "PCError", "Context", "bits_to_dense", "decode_sepsets",
           "default_options", "dense_to_bits", "lib", "pc_comb_unrank", "pc_run_stats",
           "pc_threshold", "pc_tuning", "pc_workspace_bytes", "status_str", "skeleton"]


def skeleton(X, alpha: float, max_level: int = -1, precision: str = "fp32", **options):
    """Runs pc_skeleton on data X (m x n, numpy or torch FP64). Returns (adjacency n x n uint8,
    SepSets dict, stats dict, status)."""
    import numpy as np
    import torch

    Xt = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64)).cuda() \
        if not torch.is_tensor(X) else X.to(device="cuda", dtype=torch.float64).contiguous()
    m, n = Xt.shape
    ctx = Context(precision=precision, **options)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc_run_stats()
    status = ctx.pc_skeleton(Xt, alpha, adj, recs, count, ws, max_level=max_level, stats=st)
    torch.cuda.synchronize()
    k = int(count.item())
    G = bits_to_dense(adj.cpu().numpy(), n)
    seps = decode_sepsets(recs[:k].cpu().numpy(), k)
    ctx.close()
    return G, seps, st.as_dict(), status
