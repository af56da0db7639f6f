"""Benchmark: PC-stable skeleton on one MI355X through the C ABI.

Headline workload: a linear-Gaussian SEM with n = 2000 variables, expected degree 10 and m = 1000
samples, alpha = 0.01. CI tests run in FP32 and borderline tests are re-done in FP64. Level 1 uses
the learned conditioning-set order: a row model trained on 2000 generated n = 200 SEMs picks each
node's best candidates k, and their sets {k} are tested first.

One step is one whole skeleton: standardization, the correlation GEMM with level 0, and every
level with its re-checks, captured once as a hipGraph (pc_batch_capture_ordered) and replayed. The
data is resident in HBM. `ms_per_step` is the host wall time of back-to-back replays per replay.

`value` is CI tests per second: the tests that the sequential PC-stable enumeration performs on this
input (canonical order, first success ends an edge), divided by the time per step. The CPU oracle
counts them on the same input.

The same skeleton is also run with plain lexicographic enumeration and with candidates ranked by
|C_ik| alone, and timed the same way. All three skeletons must equal the oracle's; if one does not,
`value` is null.

`roofline` prices the level-1 pass of a step (k_row_order + k_window + k_level<float,1>) on the
canonical level-1 work. Each CI test reads 8 bytes (C_ij and C_jk) and each conditioning set
{k} of a row reads 8 bytes (C_ik, C_kk). The pass is timed with HIP events on the same stream, in
eager runs of the same skeleton right after the timed replays (a captured graph holds no events).

Further legs (skipped with --no-extras):
* the n = 1000, degree 4, m = 500 skeleton as a captured hipGraph;
* the n = 8000, degree 6, m = 2000 skeleton with the BF16x3 GEMM, levels 1-3;
* 256 uneven datasets in one graph;
* orientation of the n = 1000 skeleton;
* the paper's scalability grid (n = 1000-4000, m = 2000-10000, d = 0.1-0.5).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
                    [--headline-only] [--copy-calibration MiB] [--write-traffic ...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HEADLINE = "n2000_d10_m1000_apply"
C2_WORKLOAD = "n1000_d4_m500_fp32"
C3_WORKLOAD = "n8000_d6_m2000_bf16x3"
C3_GOLDEN = os.path.join(ROOT, "tests", "golden", "n8000_d6_m2000_levels3.npz")
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E
# Level-1 orders compared on the headline workload (each the fastest of a sweep over its
# parameters on this workload): candidates tested first per node (row_top), the remaining sets
# enumerated by descending |C_ik| (row_sort) and run in two passes split at rank row_split.
LEARNED_ORDER = dict(row_top=2, row_sort=True, row_split=32)   # + row_short = learn.ROW_SHORT
ABS_ORDER = dict(row_top=1, row_sort=True, row_split=8)
TAIL_TESTS = 2048     # c2 graph: levels with more CI tests than this run as level kernels
TAIL_MAX_LEVEL = 8    # deepest level the tail kernel runs
TRAFFIC = {
    "headline": os.path.join(ROOT, "profiles", "traffic_level1_n2000_d10_m1000.json"),
}
LEVEL1_KERNELS = {"headline": ["k_row_order<float>", "k_window", "k_level<float, 1>"]}
LEVEL_SOURCES = ["paper_1812_08491_amd/csrc/pc_level.h", "paper_1812_08491_amd/csrc/pc_level_f32.hip",
                 "paper_1812_08491_amd/csrc/pc_level.hip", "paper_1812_08491_amd/csrc/pc_citest.h",
                 "paper_1812_08491_amd/csrc/pc_dev.h", "paper_1812_08491_amd/csrc/pc_comb.h",
                 "paper_1812_08491_amd/csrc/pc_mlp.hip"]


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def level_source_hash() -> str:
    h = hashlib.sha256()
    for p in LEVEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(leg: str):
    """HBM bytes per level-1 pass from the committed PMC summary, or None when a level-1 source
    changed after the counters were taken."""
    try:
        with open(TRAFFIC[leg]) as f:
            t = json.load(f)
    except (KeyError, OSError, ValueError):
        return None
    if t.get("source_hash") != level_source_hash():
        return None
    return float(t["bytes_per_pass"])


def level1_bytes(ref, n: int) -> float:
    """Canonical level-1 bytes: 8 B per CI test the sequential enumeration performs (C_ij and C_jk)
    and 8 B per conditioning set {k} of a row of G' (C_ik, C_kk), i.e. two per edge of G after
    level 0."""
    edges_after_0 = n * (n - 1) // 2 - int(ref.removed[0])
    return 8.0 * (int(ref.tests[1]) + 2 * edges_after_0)


def copy_calibration(mib: int, reps: int = 5) -> None:
    """Device-to-device copies of a known size, for scaling the PMC byte counters."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": mib << 20, "reps": reps}))


def write_traffic(leg: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str,
                  copy_bytes: int) -> None:
    """Per-dispatch HBM bytes of the level-1 kernels of a leg from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for
    a device copy of copy_bytes; written with the hash of the level-1 sources."""
    import csv

    def per_dispatch(path, kernel):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Kernel_Name"].startswith("void pcg::" + kernel) or r["Kernel_Name"].startswith("pcg::" + kernel)
                or r["Kernel_Name"].startswith(kernel)]
        return (float(np.mean(vals)) if vals else 0.0), len(vals)

    cf, _ = per_dispatch(copy_fetch_csv, "__amd_rocclr_copyBuffer")
    cw, _ = per_dispatch(copy_write_csv, "__amd_rocclr_copyBuffer")
    f_fetch, f_write = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    kernels, total = {}, 0.0
    # a level-1 pass dispatches the first kernel of the list once (and k_level once per pass of a
    # split order): per-pass bytes = all dispatches' bytes / the first kernel's dispatches
    _, passes = per_dispatch(fetch_csv, LEVEL1_KERNELS[leg][0])
    for k in LEVEL1_KERNELS[leg]:
        fetch, nf = per_dispatch(fetch_csv, k)
        write, nw = per_dispatch(write_csv, k)
        b = (fetch * f_fetch + write * f_write) * 1024.0
        kernels[k] = {"fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
                      "bytes_per_launch": b, "launches_per_pass": nf / max(passes, 1)}
        total += b * nf / max(passes, 1)
    out = {"leg": leg, "kernels": kernels, "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_fetch, "write_scale": f_write, "bytes_per_pass": total,
           "source_hash": level_source_hash()}
    with open(TRAFFIC[leg], "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def oracle_timed(X, alpha, threads: int, max_level: int = -1):
    """The FP64 oracle as it stands on `threads` threads: (result, seconds)."""
    import oracle
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        ref = oracle.skeleton(X, alpha, max_level=max_level)
        return ref, time.perf_counter() - t0
    finally:
        oracle.set_threads(1)


def host_threads() -> int:
    """Threads for the multi-threaded oracle run: this process's CPU share (OMP_NUM_THREADS when
    the host sets it), at most the CPUs present."""
    cpus = os.cpu_count() or 1
    try:
        cpus = min(cpus, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        pass
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(cpus, int(env))) if env.isdigit() and int(env) > 0 else cpus


# ---------------------------------------------------------------------------------------------
# Headline: learned order vs |C_ik| vs plain, n = 2000, degree 10, m = 1000
# ---------------------------------------------------------------------------------------------
def headline(args, torch, pc, semgen, out):
    from paper_1812_08491_amd import learn
    progress("headline: n=2000 learned / |C_ik| / plain")
    X, _, alpha = semgen.workload(HEADLINE)
    m, n = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    row_w = learn.load_weights(learn.ROW_WEIGHTS)
    # The levels the skeleton needs, from one eager run: every graph records all of them, so no
    # replay needs the stream continuation of pc_graph_results.
    ectx = pc.Context(precision="fp32")
    eadj = ectx.adjacency(n)
    erecs, ecount = ectx.sepsets(n * (n - 1) // 2)
    est = pc.pc_run_stats()
    eorder = ectx.order(None, row_params=row_w, row_short=learn.ROW_SHORT, **LEARNED_ORDER)
    assert ectx.pc_skeleton_ordered(Xd, alpha, eadj, erecs, ecount, ectx.workspace(n, m), eorder, stats=est) == 0
    graph_levels = max(1, est.levels_run - 1)
    stream = torch.cuda.Stream()
    modes = {}
    with torch.cuda.stream(stream):
        for mode in ("learned", "abs", "plain"):
            ctx = pc.Context(stream=stream, precision="fp32", graph_levels=graph_levels)
            order = None
            if mode == "learned":
                order = ctx.order(None, row_params=row_w, row_short=learn.ROW_SHORT, **LEARNED_ORDER)
            elif mode == "abs":
                order = ctx.order(None, row_rank="abs", **ABS_ORDER)
            adj = ctx.adjacency(n)
            recs, count = ctx.sepsets(n * (n - 1) // 2)
            probs = ctx.problems([(Xd, alpha, -1, adj, recs, count)])
            ws = ctx.batch_workspace(probs)
            # Per-level launch shapes tuned on this workload and order, then recorded in the graph.
            t0 = time.perf_counter()
            if args.load_tuning:
                # shapes a previous run tuned (profiling runs time exactly that configuration)
                with open(args.load_tuning) as f:
                    tuning = pc.pc_tuning.from_dict(json.load(f)[mode])
                ctx.pc_set_tuning(tuning)
            else:
                progress(f"headline: tuning {mode}")
                tuning = ctx.pc_tune(probs, ws, order)
            tune_s = time.perf_counter() - t0
            graph = ctx.pc_batch_capture(probs, ws, order)
            modes[mode] = dict(ctx=ctx, order=order, adj=adj, recs=recs, count=count, graph=graph, ws=ws,
                               probs=probs, tuning=tuning, tune_s=tune_s)

    def results(mode):
        st = (pc.pc_run_stats * 1)()
        r, status = modes[mode]["graph"].pc_graph_results(st)
        assert r == 0 and status[0] == 0, (mode, r, status)
        d = st[0].as_dict()
        assert d["levels_run"] - 1 <= graph_levels, "a replay needed levels beyond the recorded ones"
        return d

    names = ("learned",) if args.headline_only else ("learned", "abs", "plain")
    res = {}
    with torch.cuda.stream(stream):
        for mode in names:
            g = modes[mode]["graph"]
            for _ in range(max(1, args.warmup)):
                g.pc_graph_launch()
                results(mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.pc_graph_launch()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / args.steps
            last = results(mode)
            # The level-1 pass (the same kernels on the same stream), timed with HIP events around
            # it in eager runs of the same skeleton (a captured graph holds no timing events).
            tctx = pc.Context(stream=stream, precision="fp32", timing=32)
            tctx.pc_set_tuning(modes[mode]["tuning"])
            tadj = tctx.adjacency(n)
            trecs, tcount = tctx.sepsets(n * (n - 1) // 2)
            tws = tctx.workspace(n, m)
            torder = modes[mode]["order"]
            l1 = []
            for _ in range(10):
                st = pc.pc_run_stats()
                if torder is None:
                    tctx.pc_skeleton(Xd, alpha, tadj, trecs, tcount, tws, stats=st)
                else:
                    tctx.pc_skeleton_ordered(Xd, alpha, tadj, trecs, tcount, tws, torder, stats=st)
                l1.append(st.level_ms[1])
            del tws, trecs
            td = modes[mode]["tuning"].as_dict()
            res[mode] = {"ms_per_step": sec * 1e3, "tests": last["tests"], "probe_tests": last["probe_tests"],
                         "rechecks": last["rechecks"], "levels_run": last["levels_run"],
                         "level1_pass_ms": float(np.mean(l1)), "adj": modes[mode]["adj"].cpu().numpy(),
                         "tuning": {"tests_per_lane": td["tests_per_lane"], "ranks_per_lane": td["ranks_per_lane"],
                                    "lds_budget": td["lds_budget"], "grid": td["grid"],
                                    "recheck_grid": td["recheck_grid"], "set_lanes": td["set_lanes"][:3],
                                    "runs": td["runs"],
                                    "seconds": modes[mode]["tune_s"],
                                    "level_ms_tuned": [round(x, 4) for x in td["level_ms"]],
                                    "level_ms_default": [round(x, 4) for x in td["default_ms"]]}}
    if args.save_tuning:
        with open(args.save_tuning, "w") as f:
            json.dump({mode: modes[mode]["tuning"].as_dict() for mode in modes}, f)
    G = {mode: pc.bits_to_dense(res[mode].pop("adj"), n) for mode in names}
    sec = res["learned"]["ms_per_step"] * 1e-3
    out.update({
        "ms_per_step": res["learned"]["ms_per_step"],
        "config": {"workload": "pc_stable_skeleton_n2000_deg10_m1000_alpha0.01_fp32_recheck_learned_order",
                   "n": n, "m": m, "expected_degree": 10, "alpha": alpha,
                   "precision": "fp32 CI tests + fp64 re-check of borderline tests",
                   "order": {"form": "shared-set (row) model at level 1", **LEARNED_ORDER,
                             "row_short": learn.ROW_SHORT, "abs_order": ABS_ORDER,
                             "weights": "paper_1812_08491_amd/weights/order_row_mlp_n200.npy",
                             "trained_on": "2000 generated SEMs, n=200, degree~U[2,10], m=1000"},
                   "step": "one replay of the whole skeleton captured as a hipGraph (pc_batch_capture_ordered)",
                   "launch_shapes": "per level, autotuned on this workload before capture (pc_tune)",
                   "graph_levels": graph_levels},
        "gpu_tests_per_step": int(sum(res["learned"]["tests"])),
        "orders": {mode: {k: v for k, v in r.items()} for mode, r in res.items()},
    })
    if "plain" in G:
        out["orders_same_skeleton"] = bool(np.array_equal(G["learned"], G["plain"]) and
                                           np.array_equal(G["abs"], G["plain"]))
        out["learned_vs_plain_speedup"] = res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"]
        out["learned_vs_abs_speedup"] = res["abs"]["ms_per_step"] / res["learned"]["ms_per_step"]
    if args.no_cpu_baseline:
        out["value"] = None
        out["note"] = "no oracle run: value needs the oracle's canonical test count"
        return
    progress("headline: GPU steps done; oracle at 1 thread")
    ref1, t1 = oracle_timed(X, alpha, 1)
    threads = host_threads()
    progress(f"headline: oracle at {threads} threads")
    refN, tN = oracle_timed(X, alpha, threads)
    assert np.array_equal(ref1.G, refN.G) and ref1.tests == refN.tests
    canonical = int(sum(ref1.tests))
    equal = {mode: bool(np.array_equal(G[mode], ref1.G)) for mode in names}
    out["canonical_tests_per_step"] = canonical
    out["canonical_tests_per_level"] = list(ref1.tests)
    out["skeleton_equal_to_oracle"] = equal
    ok = all(equal.values()) and out.get("orders_same_skeleton", True)
    out["value"] = canonical / sec if ok else None
    for mode in names:
        out["orders"][mode]["canonical_tests_per_s"] = canonical / (res[mode]["ms_per_step"] * 1e-3)
    lb = level1_bytes(ref1, n)
    l1_ms = res["learned"]["level1_pass_ms"]
    ach = lb / (l1_ms * 1e-3) / 1e9
    out["roofline"] = {"kernel": "level-1 pass: k_row_order + k_window + k_level<float,1>", "bound": "hbm",
                       "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                       "traffic": measured_traffic("headline"), "algorithmic_bytes": lb,
                       "algorithmic_units": {"canonical_level1_tests": int(ref1.tests[1]),
                                             "level1_sets": 2 * (n * (n - 1) // 2 - int(ref1.removed[0]))},
                       "launch_ms": l1_ms}
    if "plain" in res:
        pl = res["plain"]["level1_pass_ms"]
        out["roofline_plain_level1"] = {"kernel": "k_level<float,1> (plain order)", "achieved": lb / (pl * 1e-3) / 1e9,
                                        "frac": lb / (pl * 1e-3) / 1e9 / PEAK_HBM_GBS, "launch_ms": pl,
                                        "executed_over_canonical": res["plain"]["tests"][1] / ref1.tests[1]}
    out["cpu_baseline"] = {"value": canonical / t1, "unit": "CI tests/s", "cores": 1, "kind": "oracle",
                           "sample": f"whole workload (same input), one run, {t1:.2f} s",
                           "wall_s_per_skeleton": t1,
                           "threaded": {"value": canonical / tN, "cores": threads, "wall_s_per_skeleton": tN},
                           "build": "gcc -O3 -march=native -fopenmp (edges of a level in parallel)"}


# ---------------------------------------------------------------------------------------------
# n = 1000, degree 4, m = 500: the whole skeleton as one captured graph
# ---------------------------------------------------------------------------------------------
def leg_c2_graph(args, torch, pc, semgen, out):
    progress("c2: n=1000 graph")
    X, sem, alpha = semgen.workload(C2_WORKLOAD)
    m, n = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    ctx = pc.Context(precision="fp32", timing=1 | 2)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    # launch shapes autotuned on this workload (applied to the eager runs and the graph below)
    tprobs = ctx.problems([(Xd, alpha, -1, adj, recs, count)])
    tws = ctx.batch_workspace(tprobs)
    tuning = ctx.pc_tune(tprobs, tws)
    del tws
    sts = []
    for _ in range(max(3, args.warmup)):
        st = pc.pc_run_stats()
        assert ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, stats=st) == 0
        sts.append(st.as_dict())
    last = sts[-1]
    L = last["levels_run"]
    big = [l for l in range(1, L) if last["tests"][l] > TAIL_TESTS]
    graph_levels = max([1] + big)
    if L - 1 > TAIL_MAX_LEVEL:
        graph_levels = max(graph_levels, L - 1)
    gstream = torch.cuda.Stream()
    with torch.cuda.stream(gstream):
        gctx = pc.Context(stream=gstream, precision="fp32", graph_levels=graph_levels, tail_tests=1 << 30)
        gctx.pc_set_tuning(tuning)
        gadj = gctx.adjacency(n)
        grecs, gcount = gctx.sepsets(n * (n - 1) // 2)
        probs = gctx.problems([(Xd, alpha, -1, gadj, grecs, gcount)])
        gws = gctx.batch_workspace(probs)
        graph = gctx.pc_batch_capture(probs, gws)
        for _ in range(args.warmup):
            graph.pc_graph_launch()
        torch.cuda.synchronize()
        reps = max(20, args.steps)
        g0 = time.perf_counter()
        for _ in range(reps):
            graph.pc_graph_launch()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - g0) / reps
        gst = (pc.pc_run_stats * 1)()
        r, gstatus = graph.pc_graph_results(gst)
        graph.close()
    assert r == 0 and gstatus[0] == 0, (r, gstatus)
    gd = gst[0].as_dict()
    assert gd["levels_run"] - 1 <= max(graph_levels, TAIL_MAX_LEVEL), "the graph did not cover every level"
    G = pc.bits_to_dense(gadj.cpu().numpy(), n)
    td = tuning.as_dict()
    leg = {"workload": "n=1000, degree 4, m=500, alpha 0.01, fp32 + fp64 re-check; one hipGraph replay",
           "launch_shapes": {"tests_per_lane": td["tests_per_lane"], "ranks_per_lane": td["ranks_per_lane"],
                             "lds_budget": td["lds_budget"], "set_lanes": td["set_lanes"][:3]},
           "ms_per_skeleton": sec * 1e3, "graph_levels": graph_levels, "levels_run": gd["levels_run"],
           "gpu_tests": int(sum(gd["tests"])), "edges": int(G.sum()) // 2,
           "level1_ms_events": float(np.mean([s["level_ms"][1] for s in sts[1:]])),
           "corr_ms_events": float(np.mean([s["corr_ms"] for s in sts[1:]]))}
    fl = float(m) * n * (n - 1) / (leg["corr_ms_events"] * 1e-3) / 1e12
    leg["roofline_corr"] = {"kernel": "k_corr<fp32> (SYRK + level-0 test)", "bound": "mfma", "achieved": fl,
                            "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": fl / PEAK_FP32_MFMA_TFLOPS}
    if not args.no_cpu_baseline:
        ref, t1 = oracle_timed(X, alpha, 1)
        canonical = int(sum(ref.tests))
        leg["skeleton_equal_to_oracle"] = bool(np.array_equal(G, ref.G))
        leg["canonical_tests"] = canonical
        leg["canonical_tests_per_s"] = canonical / sec if leg["skeleton_equal_to_oracle"] else None
        lb = level1_bytes(ref, n)
        ach = lb / (leg["level1_ms_events"] * 1e-3) / 1e9
        leg["roofline_level1"] = {"kernel": "k_level<float,1>", "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                                  "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": None,
                                  "algorithmic_bytes": lb,
                                  "executed_over_canonical": last["tests"][1] / max(1, ref.tests[1])}
        leg["cpu_oracle_s"] = t1
    out["c2_graph"] = leg
    return gctx, gadj, grecs, gcount, G, n


# ---------------------------------------------------------------------------------------------
# n = 8000, degree 6, m = 2000: BF16x3 correlation GEMM, levels 1-3
# ---------------------------------------------------------------------------------------------
def leg_c3(args, torch, pc, semgen, out):
    progress("c3: n=8000 levels 0-3")
    X, sem, alpha = semgen.workload(C3_WORKLOAD)
    m, n = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    leg = {"workload": "n=8000, degree 6, m=2000, alpha 0.05, bf16x3 GEMM + fp32 tests + fp64 re-check, levels 0-3"}
    for prec in ("bf16x3", "fp32"):
        progress(f"c3: {prec}")
        ctx = pc.Context(precision=prec, timing=1 | 2 | 8)
        adj = ctx.adjacency(n)
        recs, count = ctx.sepsets(4 * n * n // 8)
        # launch shapes autotuned on this workload, levels 1-3
        tprobs = ctx.problems([(Xd, alpha, 3, adj, recs, count)])
        ws = ctx.batch_workspace(tprobs)
        t0 = time.perf_counter()
        tuning = ctx.pc_tune(tprobs, ws).as_dict()
        tune_s = time.perf_counter() - t0
        walls, sts = [], []
        for r in range(3):
            st = pc.pc_run_stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            assert ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, max_level=3, stats=st) == 0
            torch.cuda.synchronize()
            if r:
                walls.append(time.perf_counter() - t0)
                sts.append(st.as_dict())
        G = pc.bits_to_dense(adj.cpu().numpy(), n)
        d = sts[-1]
        corr_ms = float(np.mean([s["corr_ms"] for s in sts]))
        e = {"ms_per_skeleton": float(np.median(walls)) * 1e3, "corr_ms": corr_ms,
             "level_ms": [float(np.mean([s["level_ms"][l] for s in sts])) for l in range(4)],
             "recheck_ms": [float(np.mean([s["recheck_ms"][l] for s in sts])) for l in range(4)],
             "gpu_tests": d["tests"], "rechecks": d["rechecks"], "edges": int(G.sum()) // 2,
             "launch_shapes": {"tests_per_lane": tuning["tests_per_lane"][:4],
                               "ranks_per_lane": tuning["ranks_per_lane"][:4],
                               "lds_budget": tuning["lds_budget"][:4], "set_lanes": tuning["set_lanes"][:3],
                               "tune_s": tune_s, "level_ms_untuned": [round(x, 4) for x in tuning["default_ms"][:4]]}}
        flops = float(m) * n * (n - 1)
        if prec == "bf16x3":
            ach = 3 * flops / (corr_ms * 1e-3) / 1e12
            e["roofline_corr"] = {"kernel": "k_corr<bf16x3>", "bound": "mfma", "achieved": ach,
                                  "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s (3 BF16 products)",
                                  "frac": ach / PEAK_BF16_MFMA_TFLOPS}
        else:
            ach = flops / (corr_ms * 1e-3) / 1e12
            e["roofline_corr"] = {"kernel": "k_corr<fp32>", "bound": "mfma", "achieved": ach,
                                  "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA_TFLOPS}
        if os.path.exists(C3_GOLDEN):
            # the oracle's stored result for this input (tests/golden/make_oracle_skeletons.py)
            g = np.load(C3_GOLDEN, allow_pickle=False)
            digest = hashlib.sha256(np.ascontiguousarray(X, dtype=np.float64).tobytes()).hexdigest()
            if str(g["digest"]) == digest:
                ref_edges = g["edges_after_3"]
                Gr = np.zeros((n, n), bool)
                Gr[ref_edges[:, 0], ref_edges[:, 1]] = True
                Gr |= Gr.T
                e["skeleton_equal_to_oracle"] = bool(np.array_equal(G.astype(bool), Gr))
                canonical = int(g["tests"].sum())
                e["canonical_tests"] = canonical
                e["canonical_tests_per_s"] = canonical / (e["ms_per_skeleton"] * 1e-3)
                lb = 8.0 * (int(g["tests"][1]) + 2 * (n * (n - 1) // 2 - int(g["removed"][0])))
                a1 = lb / (e["level_ms"][1] * 1e-3) / 1e9
                e["roofline_level1"] = {"kernel": "k_level<float,1>", "bound": "hbm", "achieved": a1,
                                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": a1 / PEAK_HBM_GBS,
                                        "algorithmic_bytes": lb,
                                        "executed_over_canonical": d["tests"][1] / int(g["tests"][1])}
        leg[prec] = e
        del ws, tprobs
    out["c3_n8000"] = leg


def leg_batch(args, torch, pc, semgen, out):
    progress("batch: 256 datasets")
    batch = semgen.batch_problems(256)
    bstream = torch.cuda.Stream()
    with torch.cuda.stream(bstream):
        bctx = pc.Context(stream=bstream, precision="fp32")
        items = []
        for Xb, _, ab in batch:
            mb, nb = Xb.shape
            rb, cb = bctx.sepsets(nb * (nb - 1) // 2)
            items.append((torch.from_numpy(np.ascontiguousarray(Xb)).cuda(), ab, -1, bctx.adjacency(nb), rb, cb))
        bprobs = bctx.problems(items)
        bws = bctx.batch_workspace(bprobs)
        bst = (pc.pc_run_stats * len(items))()

        def timed_graph():
            bgraph = bctx.pc_batch_capture(bprobs, bws)
            for _ in range(2):
                bgraph.pc_graph_launch()
                bgraph.pc_graph_results(bst)
            torch.cuda.synchronize()
            reps = max(3, args.steps // 5)
            b0 = time.perf_counter()
            for _ in range(reps):
                # a replay and its results: levels some datasets need beyond the recorded ones run
                # inside pc_graph_results, so both are timed
                bgraph.pc_graph_launch()
                br, bstatus = bgraph.pc_graph_results(bst)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - b0) / reps * 1e3
            bgraph.close()
            assert br == 0 and all(s == 0 for s in bstatus), (br, bstatus)
            return bms

        ms_default = timed_graph()
        progress("batch: tuning")
        t0 = time.perf_counter()
        tuning = bctx.pc_tune(bprobs, bws).as_dict()
        tune_s = time.perf_counter() - t0
        bms = timed_graph()
    tests = int(sum(sum(s.as_dict()["tests"]) for s in bst))
    out["batch256_graph"] = {"workload": "256 datasets, n~U[20,400], degree~U[2,8], m~U[200,5000], alpha 0.01, fp32",
                             "ms_per_batch": bms, "ms_per_batch_untuned": ms_default, "status": 0,
                             "gpu_tests": tests, "gpu_tests_per_s": tests / (bms * 1e-3),
                             "launch_shapes": {"tests_per_lane": tuning["tests_per_lane"],
                                               "ranks_per_lane": tuning["ranks_per_lane"],
                                               "lds_budget": tuning["lds_budget"],
                                               "set_lanes": tuning["set_lanes"][:3], "tune_s": tune_s,
                                               "runs": tuning["runs"]}}


def leg_orient(args, torch, pc, out, c2):
    progress("orientation")
    gctx, gadj, grecs, gcount, G, n = c2
    nrec = int(gcount.item())
    arrows = gctx.adjacency(n)
    ows = gctx.orient_workspace(n)
    rounds = gctx.pc_orient(n, gadj, grecs, nrec, arrows, ows)
    torch.cuda.synchronize()
    o0 = time.perf_counter()
    oreps = 20
    for _ in range(oreps):
        gctx.pc_orient(n, gadj, grecs, nrec, arrows, ows)
    torch.cuda.synchronize()
    orient_ms = (time.perf_counter() - o0) / oreps * 1e3
    Hg = pc.bits_to_dense(arrows.cpu().numpy(), n).astype(bool)
    leg = {"workload": "CPDAG of the n=1000 skeleton (colliders + Meek R1-R3)", "ms": orient_ms, "rounds": rounds,
           "directed": int((Hg & ~Hg.T).sum()), "bidirected": int((Hg & Hg.T).sum()) // 2,
           "undirected": int(G.sum()) // 2 - int((Hg & ~Hg.T).sum()) - int((Hg & Hg.T).sum()) // 2}
    if not args.no_cpu_baseline:
        from oracle import orient as orient_ref
        seps = pc.decode_sepsets(grecs[:max(nrec, 1)].cpu().numpy(), nrec)
        c0 = time.perf_counter()
        H_ref, rounds_ref = orient_ref.orient(G.astype(bool), orient_ref.sepset_lookup(seps))
        leg["cpu_reference_s"] = time.perf_counter() - c0
        leg["same_as_reference"] = bool(np.array_equal(H_ref, Hg) and rounds_ref == rounds)
    out["orientation"] = leg


def leg_scalability(args, torch, pc, semgen, out):
    """The paper's scalability grid (Sec. 5.6, Fig. 10): n = 1000-4000 at d = 0.1, m = 2000-10000 at
    n = 1000, d = 0.1-0.5 at n = 1000; one graph per point, FP64 tests. FP32 tests at two points
    (nearly every FP32 test lies in the error band there: the re-check queue overflows and the run
    is completed in FP64 from that level)."""
    progress("paper scalability grid")
    points = []
    fp32_at = {(1000, 0.1, 10000), (1000, 0.3, 10000)}
    for n, p, m in semgen.SCALABILITY_GRID:
        X, _, alpha = semgen.scalability(n, p, m)
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        del X
        point = {"n": n, "d": p, "m": m}
        for prec in ("fp64", "fp32") if (n, p, m) in fp32_at else ("fp64",):
            progress(f"paper scalability n={n} d={p} m={m}: {prec}")
            sctx = pc.Context(precision=prec)
            sadj = sctx.adjacency(n)
            srecs, scount = sctx.sepsets(n * (n - 1) // 2)
            sprobs = sctx.problems([(Xd, alpha, -1, sadj, srecs, scount)])
            sws = sctx.batch_workspace(sprobs)
            sst = (pc.pc_run_stats * 1)()

            def wall_ms():
                walls = []
                for r in range(3):
                    torch.cuda.synchronize()
                    s0 = time.perf_counter()
                    sr, sstatus = sctx.pc_batch_skeleton(sprobs, sws, sst)
                    torch.cuda.synchronize()
                    assert sr == 0 and sstatus == [0], (n, p, m, prec, sr, sstatus)
                    if r:
                        walls.append(time.perf_counter() - s0)
                return float(np.median(walls)) * 1e3

            ms = wall_ms()
            sd = sst[0].as_dict()
            point[prec] = {"ms": ms, "status": 0, "levels_run": sd["levels_run"],
                           "gpu_tests": int(sum(sd["tests"])), "rechecks": int(sum(sd["rechecks"])),
                           "fp64_from": sd["fp64_from"],
                           "edges": int(pc.bits_to_dense(sadj.cpu().numpy(), n).sum()) // 2}
            if prec == "fp64":
                # the same skeleton with launch shapes autotuned on it
                t0 = time.perf_counter()
                tuning = sctx.pc_tune(sprobs, sws).as_dict()
                point[prec]["tune_s"] = time.perf_counter() - t0
                point[prec]["ms_tuned"] = wall_ms()
                point[prec]["tests_per_lane"] = tuning["tests_per_lane"]
            del sws, sadj, srecs, scount, sprobs
            sctx.close()
        points.append(point)
        del Xd
        torch.cuda.empty_cache()
    out["paper_scalability"] = {
        "workload": "paper's family: edge probability d per pair, positive weights U[0.1, 1], alpha 0.01",
        "points": points}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the learned-order steps of the headline (for profiling; no value)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--leg", choices=["c2", "c3", "batch", "scalability"],
                    help="run only this leg (for profiling; no headline value)")
    ap.add_argument("--save-tuning", metavar="JSON", help="write the headline's tuned launch shapes")
    ap.add_argument("--load-tuning", metavar="JSON", help="use these launch shapes instead of tuning")
    ap.add_argument("--write-traffic", nargs=5, metavar=("LEG", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV"))
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, copy_bytes=256 << 20)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path.", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return 0
    if args.headline_only:
        args.no_extras = True
        args.no_cpu_baseline = True

    import torch

    import paper_1812_08491_amd as pc
    import semgen

    progress("torch imported")
    torch.cuda.set_device(0)
    out = {
        "metric": "CI tests/sec and skeleton wall time (learned-order vs plain, identical skeleton)",
        "value": None, "unit": "CI tests/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic linear-Gaussian SEM (seeded), resident in HBM",
    }
    if args.leg:
        {"c2": leg_c2_graph, "c3": leg_c3, "batch": leg_batch, "scalability": leg_scalability}[args.leg](
            args, torch, pc, semgen, out)
        print(json.dumps(out))
        return 0
    headline(args, torch, pc, semgen, out)
    if not args.no_extras:
        c2 = leg_c2_graph(args, torch, pc, semgen, out)
        leg_orient(args, torch, pc, out, c2)
        leg_c3(args, torch, pc, semgen, out)
        leg_batch(args, torch, pc, semgen, out)
        leg_scalability(args, torch, pc, semgen, out)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
