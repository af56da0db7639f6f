"""Learned conditioning-set ordering: training rows from the plain method, training, evaluation.

Everything runs on the GPU through the library's entry points: pc_corr / pc_level produce the
plain method's levels and SepSets, pc_features the candidate features of a level's snapshot G',
and pc_mlp_forward / pc_mlp_bce / pc_mlp_backward / pc_mlp_adam train the scorer. torch only holds
buffers and does index bookkeeping on them.

Labels. At level l >= 1 a direction (i, j) is the edge (i, j) seen from row i, with candidates
k in N'_i minus {j} (N'_i: neighbours of i in the snapshot G' the level draws its conditioning
sets from, Sec. 2.4). If the plain level removes the edge and its recorded SepSet S lies inside
that candidate list, each candidate k gives one row labelled [k in S]. Directions of edges that
survive the level carry no label: every order tests all of their subsets, so the order cannot
matter for them. The scorer therefore learns which candidates tend to separate an edge, which is
what lets the probe pass (top-scored subsets first) remove edges with fewer tests; PC-stable's
result does not depend on the order (Sec. 2.4), so the skeleton stays the same.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from ._lib import (PC_MAX_LEVEL, PC_MLP_HID, PC_MLP_IN, PC_MLP_PARAMS, Context, pc_run_stats)

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "order_mlp_n200.npy")
ROW_WEIGHTS = os.path.join(WEIGHTS_DIR, "order_row_mlp_n200.npy")
PROBE_MAX_LEVEL = 8     # the probe pass runs for levels 1 .. 8
ROW_SHORT = 8           # the row model scores the 8 candidates of largest |C_ik| of a node


def _torch():
    import torch
    return torch


def init_params(rng: np.random.Generator) -> np.ndarray:
    """He-normal weights, zero biases, in the library's flat layout: W1[64][8], b1[64],
    W2[64][64], b2[64], W3[64], b3."""
    p = np.zeros(PC_MLP_PARAMS, np.float32)
    o = 0
    p[o:o + PC_MLP_HID * PC_MLP_IN] = rng.normal(0, math.sqrt(2.0 / PC_MLP_IN), PC_MLP_HID * PC_MLP_IN)
    o += PC_MLP_HID * PC_MLP_IN + PC_MLP_HID
    p[o:o + PC_MLP_HID * PC_MLP_HID] = rng.normal(0, math.sqrt(2.0 / PC_MLP_HID), PC_MLP_HID * PC_MLP_HID)
    o += PC_MLP_HID * PC_MLP_HID + PC_MLP_HID
    p[o:o + PC_MLP_HID] = rng.normal(0, math.sqrt(2.0 / PC_MLP_HID), PC_MLP_HID)
    return p


def load_weights(path: str = DEFAULT_WEIGHTS):
    """Trained scorer parameters as a device FP32 tensor."""
    torch = _torch()
    w = np.load(path, allow_pickle=False).astype(np.float32)
    if w.shape != (PC_MLP_PARAMS,):
        raise ValueError(f"{path}: expected {PC_MLP_PARAMS} parameters, got {w.shape}")
    return torch.from_numpy(w).cuda()


def _dense(adj, n: int):
    """Device bit matrix (n x W int64) -> n x n bool."""
    torch = _torch()
    shifts = torch.arange(64, device=adj.device, dtype=torch.int64)
    bits = (adj.unsqueeze(-1) >> shifts) & 1
    return bits.reshape(n, -1)[:, :n].bool()


class RowCollector:
    """Runs the plain method level by level on one problem size and returns labelled rows."""

    def __init__(self, n: int, m: int, precision: str = "fp32", max_level: int = PROBE_MAX_LEVEL):
        torch = _torch()
        self.n, self.m, self.max_level = n, m, max_level
        self.ctx = Context(precision=precision)
        self.ws = self.ctx.workspace(n, m)
        self.adj = self.ctx.adjacency(n)
        self.recs, self.count = self.ctx.sepsets(n * (n - 1) // 2)
        self.cap = 1 << 20
        self.feats = torch.empty((self.cap, PC_MLP_IN), dtype=torch.float32, device="cuda")
        self.meta = torch.empty((self.cap, 3), dtype=torch.int32, device="cuda")

    def _features(self, level: int, alpha: float) -> int:
        torch = _torch()
        while True:
            rows = self.ctx.pc_features(level, self.n, self.m, alpha, self.adj, self.feats, self.meta, self.ws)
            if rows >= 0:
                return rows
            self.cap = max(-rows, 2 * self.cap)
            self.feats = torch.empty((self.cap, PC_MLP_IN), dtype=torch.float32, device="cuda")
            self.meta = torch.empty((self.cap, 3), dtype=torch.int32, device="cuda")

    def run(self, X, alpha: float, cap_per_level: int | None, gen=None, whole_directions: bool = False):
        """Plain levels 1 .. max_level on data X (m x n, numpy or device FP64). Returns a list of
        (level, feats [r, 8], labels [r], direction id [r]) per level with labelled rows; with
        cap_per_level, a random subset of at most that many rows per level."""
        torch = _torch()
        n = self.n
        Xd = X if torch.is_tensor(X) else torch.from_numpy(np.ascontiguousarray(X)).cuda()
        self.count.zero_()
        self.ctx.pc_corr(Xd, alpha, self.ws, adj_out=self.adj)
        out = []
        for level in range(1, self.max_level + 1):
            Gp = _dense(self.adj, n)
            deg = Gp.sum(1)
            if int(deg.max().item()) - 1 < level or self.m - level - 3 <= 0:
                break
            rows = self._features(level, alpha)
            c0 = int(self.count.item())
            self.ctx.pc_level(level, n, self.m, alpha, self.adj, self.recs, self.count, self.ws)
            c1 = int(self.count.item())
            if rows == 0 or c1 == c0:
                continue
            rec = self.recs[c0:c1].long()
            ii, jj, S = rec[:, 0], rec[:, 1], rec[:, 3:3 + level]
            lab = torch.zeros(n * n * n, dtype=torch.bool, device="cuda")
            lab[((ii * n + jj) * n).unsqueeze(1).add(S).flatten()] = True
            lab[((jj * n + ii) * n).unsqueeze(1).add(S).flatten()] = True
            lab = lab.view(n, n, n)
            removed = torch.zeros((n, n), dtype=torch.bool, device="cuda")
            removed[ii, jj] = True
            removed[jj, ii] = True
            # the direction can hold the SepSet only if every member is a candidate of row i
            valid = removed & ~(lab & ~Gp.unsqueeze(1)).any(-1)
            mi, mj, mk = self.meta[:rows].long().unbind(1)
            keep = valid[mi, mj].nonzero().squeeze(1)
            if keep.numel() == 0:
                continue
            if cap_per_level is not None and keep.numel() > cap_per_level and not whole_directions:
                pick = torch.randperm(keep.numel(), device="cuda", generator=gen)[:cap_per_level]
                keep = keep[pick.sort().values]
            out.append((level, self.feats[keep].clone(), lab[mi[keep], mj[keep], mk[keep]].float(),
                        mi[keep] * n + mj[keep]))
        return out

    def close(self):
        self.ctx.close()


class Trainer:
    """Minibatch Adam on the weighted binary cross-entropy, all on the library's MLP kernels."""

    def __init__(self, params=None, seed: int = 0, batch: int = 65536, lr: float = 2e-3):
        torch = _torch()
        self.ctx = Context(precision="fp32")
        self.params = (params.clone() if params is not None
                       else torch.from_numpy(init_params(np.random.default_rng(seed))).cuda())
        self.batch, self.lr, self.step = batch, lr, 0
        self.m1 = torch.zeros(PC_MLP_PARAMS, device="cuda")
        self.m2 = torch.zeros(PC_MLP_PARAMS, device="cuda")
        self.grads = torch.empty(PC_MLP_PARAMS, device="cuda")
        self.scores = torch.empty(batch, device="cuda")
        self.act = torch.empty((batch, 2 * PC_MLP_HID), device="cuda")
        self.dscore = torch.empty(batch, device="cuda")
        self.partial = torch.empty(((batch + 63) // 64, PC_MLP_PARAMS), device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)

    def epoch(self, X, y, pos_weight: float) -> float:
        torch = _torch()
        N = X.shape[0]
        perm = torch.randperm(N, device="cuda", generator=self.gen)
        total, seen = 0.0, 0
        for b0 in range(0, N, self.batch):
            idx = perm[b0:b0 + self.batch]
            r = idx.numel()
            Xb, yb = X[idx].contiguous(), y[idx].contiguous()
            self.step += 1
            self.ctx.pc_mlp_forward(self.params, Xb, self.scores[:r], self.act[:r])
            self.ctx.pc_mlp_bce(self.scores[:r], yb, pos_weight, self.dscore[:r], self.loss)
            self.ctx.pc_mlp_backward(self.params, Xb, self.act[:r], self.dscore[:r], self.grads,
                                     self.partial[:(r + 63) // 64])
            self.ctx.pc_mlp_adam(self.params, self.grads, self.m1, self.m2, self.step, lr=self.lr)
            total += float(self.loss.item()) * r
            seen += r
        return total / max(seen, 1)

    def scores_of(self, X):
        torch = _torch()
        out = torch.empty(X.shape[0], device="cuda")
        if X.shape[0]:
            self.ctx.pc_mlp_forward(self.params, X.contiguous(), out)
        return out

    def close(self):
        self.ctx.close()


def bce_loss(trainer: Trainer, X, y, pos_weight: float) -> float:
    torch = _torch()
    s = trainer.scores_of(X)
    ds = torch.empty_like(s)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    trainer.ctx.pc_mlp_bce(s, y.contiguous(), pos_weight, ds, loss)
    return float(loss.item())


def topq_recall(scores, labels, direction, q: int) -> float:
    """Fraction of labelled directions whose whole SepSet lies within their q best-scored
    candidates (the probe then removes the edge with its first C(q, l) subsets)."""
    torch = _torch()
    if direction.numel() == 0:
        return float("nan")
    # rank of each row inside its direction, by descending score (ties: lower row first)
    order = torch.argsort(scores, descending=True, stable=True)
    order = order[torch.argsort(direction[order], stable=True)]
    d_sorted = direction[order]
    start = torch.ones_like(d_sorted, dtype=torch.bool)
    start[1:] = d_sorted[1:] != d_sorted[:-1]
    seg = torch.cumsum(start.long(), 0) - 1
    first = torch.nonzero(start).squeeze(1)
    rank = torch.arange(d_sorted.numel(), device=scores.device) - first[seg]
    pos = labels[order] > 0.5
    worst = torch.zeros(first.numel(), dtype=torch.long, device=scores.device)
    worst.scatter_reduce_(0, seg[pos], rank[pos], reduce="amax")
    return float((worst < q).float().mean().item())


def collect(datasets, n: int, m: int, cap_per_level: int, seed: int = 0, log=None):
    """Rows of many datasets of one shape: (feats, labels) concatenated on the device."""
    torch = _torch()
    coll = RowCollector(n, m)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    feats, labels = [], []
    t0 = time.time()
    for k, (X, alpha) in enumerate(datasets):
        for level, f, y, _ in coll.run(X, alpha, cap_per_level, gen):
            feats.append(f)
            labels.append(y)
        if log and (k + 1) % 100 == 0:
            log(f"collected {k + 1} datasets, {sum(x.shape[0] for x in feats)} rows, {time.time() - t0:.1f} s")
    coll.close()
    if not feats:
        return (torch.empty((0, PC_MLP_IN), device="cuda"), torch.empty(0, device="cuda"))
    return torch.cat(feats), torch.cat(labels)


class NodeRowCollector:
    """Level-1 training rows of the shared-set order (one per candidate k of node i) for datasets
    of one shape: level 0 through pc_corr, then pc_row_features on its G'."""

    def __init__(self, n: int, m: int, precision: str = "fp32"):
        torch = _torch()
        self.n, self.m = n, m
        self.ctx = Context(precision=precision)
        self.ws = self.ctx.workspace(n, m)
        self.adj = self.ctx.adjacency(n)
        self.cap = 1 << 16
        self._alloc()

    def _alloc(self):
        torch = _torch()
        self.feats = torch.empty((self.cap, PC_MLP_IN), dtype=torch.float32, device="cuda")
        self.labels = torch.empty(self.cap, dtype=torch.float32, device="cuda")
        self.meta = torch.empty((self.cap, 2), dtype=torch.int32, device="cuda")

    def run(self, X, alpha: float):
        """(feats [r, 8], labels [r], node i [r], candidate k [r], C) of dataset X."""
        torch = _torch()
        Xd = X if torch.is_tensor(X) else torch.from_numpy(np.ascontiguousarray(X)).cuda()
        C = torch.empty((self.n, self.n), dtype=torch.float32, device="cuda")
        self.ctx.pc_corr(Xd, alpha, self.ws, C_out=C, adj_out=self.adj)
        while True:
            rows = self.ctx.pc_row_features(1, self.n, self.m, alpha, self.adj, self.feats, self.labels, self.meta,
                                            self.ws)
            if rows >= 0:
                break
            self.cap = max(-rows, 2 * self.cap)
            self._alloc()
        mi, mk = self.meta[:rows].long().unbind(1)
        return self.feats[:rows].clone(), self.labels[:rows].clone(), mi, mk, C

    def plain_level1_records(self, X, alpha: float):
        """(i, j, k) of every edge the plain skeleton removes at level 1 on X, with its SepSet {k}."""
        torch = _torch()
        n = self.n
        Xd = X if torch.is_tensor(X) else torch.from_numpy(np.ascontiguousarray(X)).cuda()
        adj = self.ctx.adjacency(n)
        recs, count = self.ctx.sepsets(n * (n - 1) // 2)
        self.ctx.pc_skeleton(Xd, alpha, adj, recs, count, self.ws, max_level=1)
        r = recs[:int(count.item())].long()
        r = r[r[:, 2] == 1]
        return r[:, [0, 1, 3]]

    def sepset_labels(self, X, alpha: float, mi, mk, records=None):
        """Labels from the SepSets the plain method finds: for row (i, k), the fraction of the level-1
        removals of edges at i whose recorded SepSet is {k} (records: plain_level1_records of X, run
        here when not given)."""
        torch = _torch()
        n = self.n
        r = self.plain_level1_records(X, alpha) if records is None else records
        i, j, s = r[:, 0], r[:, 1], r[:, 2]
        hits = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        hits.index_put_((torch.cat([i, j]), torch.cat([s, s])), torch.ones(2 * i.numel(), device="cuda"),
                        accumulate=True)
        per_node = hits.sum(1)
        return hits[mi, mk] / per_node[mi].clamp(min=1.0)

    def close(self):
        self.ctx.close()


def compare_orders(X, alpha: float, params, precision: str = "fp32", min_level: int = 2, top: int = 4,
                   repeats: int = 3, max_level: int = 0, row_params=None, row_top: int = 0):
    """Plain vs learned-order skeleton on the same data: identical adjacency is required; returns
    per-run tests and wall times (median over repeats after one warm-up of each, the two orders
    alternating so that both see the same device state)."""
    torch = _torch()
    Xd = X if torch.is_tensor(X) else torch.from_numpy(np.ascontiguousarray(X)).cuda()
    m, n = Xd.shape
    runs = {}
    for mode in ("plain", "learned"):
        ctx = Context(precision=precision)
        adj = ctx.adjacency(n)
        recs, count = ctx.sepsets(n * (n - 1) // 2)
        order = None
        if mode == "plain":
            ws = ctx.workspace(n, m)
        else:
            order = ctx.order(params, min_level=min_level, top=top, max_level=max_level, row_params=row_params,
                              row_top=row_top)
            ws = ctx.ordered_workspace(n, m, order)
        runs[mode] = dict(ctx=ctx, adj=adj, recs=recs, count=count, ws=ws, order=order, walls=[], st=None)

    def once(mode):
        r = runs[mode]
        st = pc_run_stats()
        torch.cuda.synchronize()
        if mode == "plain":
            r["ctx"].pc_skeleton(Xd, alpha, r["adj"], r["recs"], r["count"], r["ws"], stats=st)
        else:
            r["ctx"].pc_skeleton_ordered(Xd, alpha, r["adj"], r["recs"], r["count"], r["ws"], r["order"], stats=st)
        torch.cuda.synchronize()
        r["st"] = st
        return st.wall_ms

    for rep in range(repeats + 1):
        for mode in ("plain", "learned"):
            w = once(mode)
            if rep > 0:
                runs[mode]["walls"].append(w)
    res = {}
    for mode, r in runs.items():
        d = r["st"].as_dict()
        res[mode] = {"adj": r["adj"].cpu().numpy(), "wall_ms": float(np.median(r["walls"])), "tests": d["tests"],
                     "probe_tests": d["probe_tests"], "probe_removed": d["probe_removed"],
                     "levels_run": d["levels_run"]}
        r["ctx"].close()
    same = bool(np.array_equal(res["plain"].pop("adj"), res["learned"].pop("adj")))
    return {"same_skeleton": same, **res}


def short_list_mask(absc, node, K: int):
    """Rows (grouped by node, ascending candidate position within a node) whose |C_ik| (absc) is
    among the K largest of their node, ties to the lower position: the candidates the row model
    scores when pc_order.row_short = K."""
    torch = _torch()
    order = torch.argsort(-absc.double(), stable=True)
    order = order[torch.argsort(node[order], stable=True)]
    nd = node[order]
    start = torch.ones_like(nd, dtype=torch.bool)
    start[1:] = nd[1:] != nd[:-1]
    seg = torch.cumsum(start.long(), 0) - 1
    first = torch.nonzero(start).squeeze(1)
    rank = torch.empty_like(order)
    rank[order] = torch.arange(nd.numel(), device=nd.device) - first[seg]
    return rank < K


def train_rows(args, log) -> None:
    """Shared-set (row) model: level-1 rows of generated n = 200 SEMs, restricted to each node's
    short list (the ROW_SHORT candidates of largest |C_ik|), soft-label cross-entropy, Adam. Labels
    (--labels): by default the SepSets the plain method records at level 1 (the fraction of node i's
    level-1 removals whose SepSet is {k}); or the fraction of i's edges {k} separates (k*) or
    separates and k* does not (the others). With
    --eval, the edge coverage of its top-T candidates per node is reported against the |C_ik| order
    and a random order on held-out SEMs (tests/ref/coverage.py; run from the repository root)."""
    torch = _torch()
    import semgen
    from ._lib import bits_to_dense
    K = args.short
    t0 = time.time()
    coll = NodeRowCollector(200, 1000)
    feats, labels = [], []
    for k, (X, _, a) in enumerate(semgen.training_sems(args.sems, instance=0)):
        f, y, mi, mk, _ = coll.run(X, a)
        if args.labels == "sepsets":
            y = coll.sepset_labels(X, a, mi, mk)
        keep = short_list_mask(f[:, 0], mi, K)
        feats.append(f[keep])
        labels.append(y[keep])
        if (k + 1) % 200 == 0:
            log(f"collected {k + 1} datasets, {sum(x.shape[0] for x in feats)} rows, {time.time() - t0:.1f} s")
    X = torch.cat(feats)
    y = torch.cat(labels)
    t_collect = time.time() - t0
    pos = float(y.sum().item())
    pos_weight = 1.0   # soft labels (fractions of the row's edges separated): plain cross-entropy
    log(f"{X.shape[0]} training rows (short lists of {K}), mean label {pos / max(y.numel(), 1):.3f}")
    val = []
    for Xv, _, a in semgen.training_sems(args.val_sems, instance=1):
        f, yv, mi, mk, C = coll.run(Xv, a)
        if args.labels == "sepsets":
            yv = coll.sepset_labels(Xv, a, mi, mk)
        G = torch.from_numpy(bits_to_dense(coll.adj.cpu().numpy(), 200).astype(bool)).cuda()
        val.append((f, yv, mi, mk, C, G, a, short_list_mask(f[:, 0], mi, K)))
    trainer = Trainer(seed=args.seed, lr=args.lr)

    def coverage(score_fn):
        from tests.ref.coverage import edge_coverage
        acc = {T: [] for T in (1, 2, 4, 8)}
        for f, yv, mi, mk, C, G, a, sl in val:
            cov = edge_coverage(score_fn(f, sl), mi, mk, C, G, a, 1000)
            for T in acc:
                if cov[T] == cov[T]:
                    acc[T].append(cov[T])
        return {T: float(np.mean(v)) if v else float("nan") for T, v in acc.items()}

    def learned(f, sl):
        sc = trainer.scores_of(f)
        return torch.where(sl, sc, torch.full_like(sc, -1e30))

    base_abs = base_rand = None
    if args.eval:
        base_abs = coverage(lambda f, sl: f[:, 0].contiguous())
        base_rand = coverage(lambda f, sl: torch.rand(f.shape[0], device="cuda"))
        log(f"|C_ik| order coverage@1/2/4/8: {base_abs[1]:.3f} {base_abs[2]:.3f} {base_abs[4]:.3f} {base_abs[8]:.3f}")
        log(f"random order coverage@1/2/4/8: {base_rand[1]:.3f} {base_rand[2]:.3f} {base_rand[4]:.3f} "
            f"{base_rand[8]:.3f}")
    vX = torch.cat([v[0][v[7]] for v in val])
    vy = torch.cat([v[1][v[7]] for v in val])
    history = []
    t1 = time.time()
    for ep in range(args.epochs):
        tl = trainer.epoch(X, y, pos_weight)
        vl = bce_loss(trainer, vX, vy, pos_weight)
        h = {"epoch": ep + 1, "train_loss": tl, "val_loss": vl}
        msg = f"epoch {ep + 1}: train {tl:.4f} val {vl:.4f}"
        if args.eval:
            cov = coverage(learned)
            h["coverage"] = cov
            msg += f" coverage@1/2/4/8 {cov[1]:.3f} {cov[2]:.3f} {cov[4]:.3f} {cov[8]:.3f}"
        history.append(h)
        log(msg)
    t_train = time.time() - t1
    coll.close()
    out = args.out or ROW_WEIGHTS
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.save(out, trainer.params.cpu().numpy().astype(np.float32), allow_pickle=False)
    meta = {"model": "row", "sems": args.sems, "n": 200, "m": 1000, "degree": "U[2,10]", "alpha": 0.01,
            "row_short": K,
            "label": ("fraction of the row's level-1 removals whose SepSet (plain method) is {k}"
                      if args.labels == "sepsets" else
                      "k*: fraction of the row's edges it separates; others: fraction they separate and k* does not"),
            "features": ["|C_ik|", "|C_ik|/max_q|C_iq|", "min(n|N_i&N_k|/(d_i d_k), 8)/8", "d_k/(d_i+d_k)",
                         "|C_kk*|", "|rho_ik.k*|", "mean_j|C_ij|/max_q|C_iq|", "|N_i&N_k|/d_i"],
            "order": "k* (largest |C_ik|) first; the model picks the next from the row_short candidates of "
                     "largest |C_ik|",
            "rows": int(X.shape[0]), "mean_label": pos / max(y.numel(), 1), "pos_weight": pos_weight,
            "epochs": args.epochs, "lr": args.lr, "batch": trainer.batch, "collect_s": t_collect, "train_s": t_train,
            "abs_corr_coverage": base_abs, "random_coverage": base_rand, "history": history}
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"saved {out} (collect {t_collect:.1f} s, train {t_train:.1f} s)")
    trainer.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the conditioning-set scorer on generated SEMs.")
    ap.add_argument("--model", choices=("edge", "row"), default="edge",
                    help="edge: the probe pass's per-edge scorer; row: the level-1 shared-set order")
    ap.add_argument("--sems", type=int, default=2000)
    ap.add_argument("--val-sems", type=int, default=100)
    ap.add_argument("--cap", type=int, default=2048, help="labelled rows kept per level and SEM")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--short", type=int, default=ROW_SHORT, help="row model: candidates per node it scores")
    ap.add_argument("--eval", action="store_true", help="row model: report held-out edge coverage")
    ap.add_argument("--labels", choices=("separated", "sepsets"), default="sepsets",
                    help="row model labels: the fraction of the row's edges a candidate separates (and k* "
                         "does not), or the fraction of the row's removals whose plain-method SepSet it is")
    args = ap.parse_args(argv)
    import semgen  # the project's seeded SEM generator (repository root)
    torch = _torch()

    def log(msg):
        print(f"[learn] {msg}", flush=True)

    if args.model == "row":
        train_rows(args, log)
        return
    args.out = args.out or DEFAULT_WEIGHTS

    train_sets = ((X, a) for X, _, a in semgen.training_sems(args.sems, instance=0))
    t0 = time.time()
    X, y = collect(train_sets, 200, 1000, args.cap, seed=args.seed, log=log)
    t_collect = time.time() - t0
    pos = float(y.sum().item())
    pos_weight = float(min(50.0, max(1.0, (y.numel() - pos) / max(pos, 1.0))))
    log(f"{X.shape[0]} training rows, {pos / max(y.numel(), 1):.3f} positive, pos_weight {pos_weight:.2f}")
    val = list((Xv, a) for Xv, _, a in semgen.training_sems(args.val_sems, instance=1))
    coll = RowCollector(200, 1000)
    vrows = [r for Xv, a in val for r in coll.run(Xv, a, None, whole_directions=True)]
    coll.close()
    vX = torch.cat([r[1] for r in vrows])
    vy = torch.cat([r[2] for r in vrows])
    vdir = torch.cat([r[3] + (k << 32) for k, r in enumerate(vrows)])
    trainer = Trainer(seed=args.seed, lr=args.lr)
    base = {q: topq_recall(torch.rand(vX.shape[0], device="cuda"), vy, vdir, q) for q in (2, 4, 8)}
    log(f"random-order recall@2/4/8: {base[2]:.3f} {base[4]:.3f} {base[8]:.3f}")
    history = []
    t1 = time.time()
    for ep in range(args.epochs):
        tl = trainer.epoch(X, y, pos_weight)
        vl = bce_loss(trainer, vX, vy, pos_weight)
        s = trainer.scores_of(vX)
        rec = {q: topq_recall(s, vy, vdir, q) for q in (2, 4, 8)}
        history.append({"epoch": ep + 1, "train_loss": tl, "val_loss": vl, "recall": rec})
        log(f"epoch {ep + 1}: train {tl:.4f} val {vl:.4f} recall@2/4/8 {rec[2]:.3f} {rec[4]:.3f} {rec[8]:.3f}")
    t_train = time.time() - t1
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, trainer.params.cpu().numpy().astype(np.float32), allow_pickle=False)
    meta = {"sems": args.sems, "n": 200, "m": 1000, "degree": "U[2,10]", "alpha": 0.01, "rows": int(X.shape[0]),
            "positive_fraction": pos / max(y.numel(), 1), "pos_weight": pos_weight, "epochs": args.epochs,
            "lr": args.lr, "batch": trainer.batch, "collect_s": t_collect, "train_s": t_train,
            "random_recall": base, "history": history}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"saved {args.out} (collect {t_collect:.1f} s, train {t_train:.1f} s)")
    trainer.close()


if __name__ == "__main__":
    main()
