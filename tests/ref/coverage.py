"""Evaluation reference for the learned level-1 order (used by the training tool and by tests, never by
the library): the edge coverage of a per-node candidate ranking, recomputed in FP64 torch from the FP32
C and the snapshot G'.

An edge (i, j) of G' is level-1-separable when some k adjacent to i or j gives |rho_ij.k| <= tanh(tau_1)
(Eq. 3-6 at l = 1). The coverage at T is the fraction of those edges that a set {k} of the T best-ranked
candidates of i, or of j, separates: what the shared-set order's first pass can remove.
"""
from __future__ import annotations

import math


def _torch():
    import torch
    return torch


def edge_coverage(scores, node, cand, C, adj_dense, alpha: float, m: int, tops=(1, 2, 4, 8)) -> dict:
    """For one dataset: the fraction of level-1-separable edges (i, j) of G' (some k in N_i or N_j
    gives |rho_ij.k| <= tanh(tau_1)) that a set {k} of the T best-scored candidates of i or of j
    separates, for each T in tops."""
    torch = _torch()
    from paper_1812_08491_amd._lib import pc_threshold
    n = C.shape[0]
    th = math.tanh(pc_threshold(alpha, m, 1))
    G = adj_dense
    Cd = C.double()
    # independence of (i, j) given k for all triples with k adjacent to i or j
    ii, jj = torch.nonzero(torch.triu(G, 1), as_tuple=True)
    if ii.numel() == 0:
        return {T: float("nan") for T in tops}
    cij, cik, cjk = Cd[ii, jj].unsqueeze(1), Cd[ii], Cd[jj]
    den = ((1 - cik ** 2) * (1 - cjk ** 2)).clamp_min(0)
    indep = ((cij - cik * cjk).abs() <= th * den.sqrt()) & (den > 0)
    kmask = (G[ii] | G[jj])
    kmask[torch.arange(ii.numel()), ii] = False
    kmask[torch.arange(ii.numel()), jj] = False
    sep = (indep & kmask).any(1)
    # rank of each candidate within its node by score (ties: lower candidate id first)
    rank = torch.full((n, n), 1 << 30, dtype=torch.long, device="cuda")
    order = torch.argsort(cand.double() - scores.double() * 1e6, stable=True)   # score desc, then id
    order = order[torch.argsort(node[order], stable=True)]
    nd = node[order]
    start = torch.ones_like(nd, dtype=torch.bool)
    start[1:] = nd[1:] != nd[:-1]
    seg = torch.cumsum(start.long(), 0) - 1
    first = torch.nonzero(start).squeeze(1)
    rank[nd, cand[order]] = torch.arange(nd.numel(), device="cuda") - first[seg]
    out = {}
    for T in tops:
        topk = (rank < T)
        cover = indep & ((topk[ii] & G[ii]) | (topk[jj] & G[jj]))
        cover[torch.arange(ii.numel()), ii] = False
        cover[torch.arange(ii.numel()), jj] = False
        out[T] = float((cover.any(1) & sep).sum().item() / max(int(sep.sum().item()), 1))
    return out
