"""Benchmark of the box-code volume potential V + grad V on one MI355X.

One step = one bx_volume_eval_grad over the whole tree (P2M, M2M, M2L, X, L2L,
leaf far field, near tables) with f, V, G, tables and lists resident on the
GPU.  Prints one JSON line.  The default workload is the adaptive 20-Gaussian
source (seed 0, tail tolerance 1e-10, depth <= 14, 8x8 nodes, p = 30); by
default the mixed-precision path (near tables as exact int8 slice products,
slice tolerance 1e-11) is the headline value and the plain FP64 path runs
beside it on the same inputs, with the split result's deviation from FP64 and
both results' errors against the oracle on the CPU-baseline sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "leaf-points/sec for V+\u2207V at 1e-10 rel err, mixed vs plain FP64 (1 MI355X)"
PEAK_FP64 = 78.6e12          # MI355X dense FP64 (vector and matrix), FLOP/s
PEAK_HBM = 8.0e12            # B/s
PEAK_I8 = 5.0e15             # MI355X dense int8 MFMA, OP/s
# how each phase's kernel is bound, and by what
BOUND = {"leaf": ("mfma", PEAK_FP64), "m2l": ("mfma", PEAK_FP64), "p2m": ("mfma", PEAK_FP64),
         "p2l": ("alu", PEAK_FP64), "m2m": ("alu", PEAK_FP64), "l2l": ("alu", PEAK_FP64)}
KERNEL_OF = {"leaf": "leaf_mfma_kernel", "m2l": "m2l_mfma_kernel", "p2m": "p2m_mfma_kernel",
             "p2l": "p2l_mfma_kernel", "m2m": "m2m_mfma_kernel", "l2l": "l2l_mfma_kernel"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(tree, f, target_s=15.0, seed=0):
    """The oracle on a seeded, level-stratified sample of leaves (all their nodes)."""
    import oracle
    rng = np.random.default_rng(seed)
    levels = np.unique(tree.level)
    order = []
    pools = {l: list(rng.permutation(np.flatnonzero(tree.level == l))) for l in levels}
    while any(pools.values()):
        for l in levels:
            if pools[l]:
                order.append(pools[l].pop())
    n = f.shape[-1]
    t0 = time.perf_counter()
    oracle.volume_at_nodes(tree.level, tree.ix, tree.iy, f, leaves=np.array(order[:2]))
    t_probe = max(time.perf_counter() - t0, 1e-3)
    k = int(min(len(order), max(2, 2 * target_s / t_probe)))
    sel = np.array(order[:k])
    t0 = time.perf_counter()
    vals = oracle.volume_at_nodes(tree.level, tree.ix, tree.iy, f, leaves=sel)
    dt = time.perf_counter() - t0
    pts = k * n * n
    return ({"value": pts / dt, "unit": "leaf-points/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": f"{k} leaves ({pts} nodes, seeded, stratified by level) of the same tree, "
                       f"{dt:.1f} s"}, sel, vals)


def kernel_source_hash():
    """Hash of the kernel sources: counter summaries taken on other sources do not apply."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1610_00823_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None when it was taken on other kernel sources or another workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    e = d.get("kernels", {}).get(f"{kernel}|{workload}|{precision}")
    return None if e is None else e.get("bytes_per_launch")


def run_precision(args, precision, tree, f_host):
    """Build a context, upload the tree and time K graph-replayed steps (region 1),
    then K steps launched phase by phase with HIP events (region 2)."""
    import torch
    from paper_1610_00823_amd import boxfmm as B
    flags = B.BX_FP64 if precision == "fp64" else B.BX_SPLIT_INT8
    t0 = time.perf_counter()
    ctx = B.Context(args.n, args.p, flags)
    t_tables = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    tr = B.Tree.forest(ctx, tree.trees, stream) if isinstance(tree, Forest) else B.Tree.from_inputs(ctx, tree, stream)
    f = torch.from_numpy(f_host).cuda()
    if f.dim() == 3:
        f = f.unsqueeze(0)
    V = torch.empty_like(f)
    G = torch.empty((f.shape[0], tree.n_leaves, 2, args.n, args.n), dtype=torch.float64, device=f.device)
    log(f"{precision}: tables {t_tables:.1f} s, tree upload {tr.query('upload_ms'):.0f} ms")
    tuning = None
    if args.autotune:                    # untimed set-up, like the tables and the upload
        t0 = time.perf_counter()
        _, _, tuning = B.autotune(ctx, tr, f, V, G, reps=3, stream=stream)
        log(f"{precision}: autotune {time.perf_counter() - t0:.1f} s: heavy {tuning[0]}, fp64 weight "
            f"{tuning[1]}, m2l blocks {tuning[2]}, two-level threshold {tuning[3]}, {tuning[4]:.4f} ms")
    for _ in range(args.warmup):
        B.volume_eval_grad(ctx, tr, f, V, G, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.volume_eval_grad(ctx, tr, f, V, G, stream)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.volume_eval_grad(ctx, tr, f, V, G, stream)
    torch.cuda.synchronize()
    ms_prof = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.profile(False)
    phase_ms, nev = ctx.profile_read()
    per_eval = {k: v / max(nev, 1) for k, v in phase_ms.items()}
    nr = int(f.shape[0])
    phases = {}
    for k, v in per_eval.items():
        a, _ = tr.phase_cost(k)
        phases[k] = {"ms": round(v, 4), "tflops": round(nr * a / (v / 1e3) / 1e12, 3) if v > 0 else None}
    npts = f_host.size
    return {"nrhs": nr, "ctx": ctx, "tree": tr, "V": V, "G": G, "ms_step": ms_step, "ms_prof": ms_prof,
            "value": npts / (ms_step / 1e3), "per_eval": per_eval, "tuning": tr.tuning(), "phases": phases, "t_tables": t_tables,
            "split_products": tr.query("split_products") if precision == "split" else None}


def roofline_of(res, args, precision):
    per_eval = res["per_eval"]
    dom = max(per_eval, key=per_eval.get)
    fl, by = res["tree"].phase_cost(dom)
    fl, by = fl * res["nrhs"], by * res["nrhs"]
    bound, peak = BOUND[dom]
    t_dom = per_eval[dom] / 1e3
    if bound == "hbm":
        ach, unit, pk = by / t_dom / 1e9, "GB/s", peak / 1e9
    else:
        ach, unit, pk = fl / t_dom / 1e12, "TFLOP/s", peak / 1e12
    kernel = KERNEL_OF[dom]
    out = {"bound": bound, "achieved": ach, "peak": pk, "unit": unit, "frac": ach / pk}
    if dom == "leaf" and precision == "split":
        # the mixed near field is an int8 contraction: its algorithmic ops are the
        # FP64 near-table flops times the mean slice products per table entry;
        # the FP64-equivalent rate of the whole leaf phase is given beside it
        kernel = "leaf_near_i8_kernel"
        i8 = res["tree"].query("near_flops") * res["nrhs"] * res["split_products"]
        a8 = i8 / t_dom / 1e12
        out = {"bound": "mfma", "achieved": a8, "peak": PEAK_I8 / 1e12, "unit": "TOP/s", "frac": a8 / (PEAK_I8 / 1e12),
               "algorithmic_int8_ops": i8,
               "fp64_equivalent": {"achieved": ach, "peak": pk, "unit": unit, "frac": ach / pk}}
    out.update({"traffic": measured_traffic(kernel, args.workload, precision), "kernel": kernel, "phase": dom,
                "launch_ms": per_eval[dom], "algorithmic_flops": fl, "algorithmic_bytes": by})
    return out


class Forest:
    """Several trees evaluated as one (the leaves tree after tree)."""

    def __init__(self, trees):
        self.trees = trees
        self.n_leaves = sum(t.n_leaves for t in trees)


def learned_forest(count, n, cap=9):
    """Train the refinement network on the plain criterion's decisions (with the
    seed rule) for seeded sums of 1-40 and of 20 Gaussians and the kink source,
    then build trees for `count` fresh sums of 1-8 Gaussians (seeds 10000 + i)
    with the network proposing and the plain tail criterion checking."""
    from paper_1610_00823_amd import inputs as I
    from paper_1610_00823_amd import refine as RF
    t0 = time.perf_counter()
    jobs = (RF.source_jobs(range(300, 348), kinds=("gaussK",), n=n, cap=cap)
            + RF.source_jobs(range(400, 412), kinds=("gauss20",), n=n, cap=cap)
            + RF.source_jobs([0], kinds=("kink",), n=n, cap=cap))
    s, lv, y = RF.labelled_boxes(jobs, workers=16)   # host processes, before the GPU is touched
    t_labels = time.perf_counter() - t0
    import torch
    ref = RF.LearnedRefiner(seed=0)
    x = ref.features(s, lv)
    del s
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = ref.train(x, y, epochs=8, batch=1024, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    live = lv < cap
    acc = float((ref.predict(x)[live] == (y[live] > 0.5)).mean())
    del x
    funs = [I.random_gaussians(10000 + i, int(np.random.default_rng([10000 + i, 7]).integers(1, 9)))
            for i in range(count)]
    trees, st = ref.build(funs, n=n, cap=cap)
    plain, plain_ev = RF.plain_trees(funs[:32], n=n, cap=cap)
    e_l = [RF.resolution_error(t, f, n, points=f.c) for t, f in zip(trees[:32], funs[:32])]
    e_p = [RF.resolution_error(t, f, n, points=f.c) for t, f in zip(plain, funs[:32])]
    missed = [i for i in range(len(plain)) if e_p[i] > 1e-3]
    info = {"training_boxes": int(len(y)), "labels_s": round(t_labels, 1), "train_s": round(t_train, 2),
            "final_loss": round(losses[-1], 4), "accuracy_below_cap": round(acc, 4), "cap": cap,
            "net_boxes": st.net_boxes, "proposed_leaves": st.proposed_leaves, "fallback_leaves": st.failed_leaves,
            "f_evals": st.f_evals, "build_s": {k: round(v, 2) for k, v in st.seconds.items()},
            "first32": {"plain_missed_bump": len(missed), "learned_resolved": sum(e_l[i] < 1e-3 for i in missed),
                        "leaves_learned": sum(t.n_leaves for t in trees[:32]),
                        "leaves_plain": sum(t.n_leaves for t in plain), "f_evals_plain": plain_ev}}
    log(f"learned refinement: {info}")
    return trees, funs, info


def rel_err(a, b):
    return float((a - b).abs().max() / b.abs().max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gauss20_s0")
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--p", type=int, default=30)
    ap.add_argument("--precision", choices=["both", "fp64", "split"], default="both",
                    help="both: the mixed (int8-split near tables) path is the headline, with the plain FP64 "
                         "path beside it")
    ap.add_argument("--nrhs", type=int, default=1, help="right-hand sides on the same tree (seeded sources)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time candidate schedules of each tree before the timed region and keep the fastest "
                         "(results are bitwise the same; the default schedules are the measured best of each "
                         "precision on the 20-Gaussian workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized FP64 buffer on the GPU 5 times (a plain copy kernel "
                         "of known traffic, to scale the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8,
                          "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU sharding is a design, not code.", file=sys.stderr)
        sys.exit(2)

    from paper_1610_00823_amd import inputs as I

    t0 = time.perf_counter()
    learned = None
    if args.workload.startswith("learned"):          # trees proposed by the trained network
        tree, src, learned = learned_forest(int(args.workload[7:] or 256), args.n)
    elif args.workload.startswith("forest"):         # trees and their samples from one process pool
        body = args.workload[len("forest"):]
        count, seed = (int(body.split("_s")[0]), int(body.split("_s")[1])) if "_s" in body else (int(body), 0)
        tree, src, fs = I.forest(count, seed, args.n, samples=True)
    else:
        tree, src = I.workload(args.workload, args.n)
    if isinstance(tree, list):                       # a forest: one upload, one evaluation
        f_host = (np.concatenate(fs) if args.workload.startswith("forest")
                  else np.concatenate([I.sample(t, s_, args.n) for t, s_ in zip(tree, src)]))
        tree = Forest(tree)
    elif args.nrhs > 1:                              # the same tree, n_rhs seeded sources
        f_host = np.stack([I.sample(tree, I.random_gaussians(1000 + r, 20), args.n) for r in range(args.nrhs)])
    else:
        f_host = I.sample(tree, src, args.n)
    log(f"inputs: {args.workload}: {tree.n_leaves} leaves, {f_host.size} points, {time.perf_counter() - t0:.1f} s")
    npts = f_host.size
    precs = ["split", "fp64"] if args.precision == "both" else [args.precision]
    res = {p: run_precision(args, p, tree, f_host) for p in precs}
    head = precs[0]                      # the mixed path when both run
    r = res[head]
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "leaf-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "ms_per_step_profiled": r["ms_prof"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "i8-split+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "precision": head, "n_leaves": tree.n_leaves, "points": npts,
                   "n_rhs": int(f_host.shape[0]) if f_host.ndim == 4 else 1,
                   "trees": len(tree.trees) if isinstance(tree, Forest) else 1,
                   "nodes": args.n, "order": args.p, "levels": int(r["tree"].query("n_levels")),
                   "tree_upload_ms": r["tree"].query("upload_ms"), "table_build_s": r["t_tables"],
                   "schedule": dict(zip(["heavy", "fp64_weight", "m2l_blocks", "two_level_max"], r["tuning"])),
                   "autotuned": bool(args.autotune)},
        "roofline": roofline_of(r, args, head),
        "phases": r["phases"],
    }
    if learned is not None:
        out["config"]["learned_refinement"] = learned
    if "split" in res:
        out["config"]["split_tolerance"] = 1e-11
        out["config"]["split_mean_slice_products"] = res["split"]["split_products"]
    if len(res) == 2:
        p = res["fp64"]
        out["plain_fp64"] = {"value": p["value"], "ms_per_step": p["ms_step"], "ms_per_step_profiled": p["ms_prof"],
                             "schedule": dict(zip(["heavy", "fp64_weight", "m2l_blocks", "two_level_max"], p["tuning"])),
                             "roofline": roofline_of(p, args, "fp64"), "phases": p["phases"]}
        out["mixed_vs_plain"] = r["value"] / p["value"]
        # the split result against the FP64 result over every node (the FP64 path
        # itself meets the oracle to 1e-12: see cpu_baseline.oracle_check)
        s_, d_ = res["split"], res["fp64"]
        out["split_vs_fp64"] = {"E_V": rel_err(s_["V"], d_["V"]), "E_dV_dx1": rel_err(s_["G"][:, :, 0], d_["G"][:, :, 0]),
                                "E_dV_dx2": rel_err(s_["G"][:, :, 1], d_["G"][:, :, 1])}
    if not args.no_cpu_baseline and (isinstance(tree, Forest) or f_host.ndim == 4):
        log("cpu baseline: single-tree, single-RHS workloads only")
    elif not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, sel, vals = cpu_baseline(tree, f_host)
        check = {}
        for k, rr in res.items():
            Vg = rr["V"][0].cpu().numpy()
            Gg = rr["G"][0].cpu().numpy()
            Vo, Gxo, Gyo = vals
            check[k] = {"E_V": float(np.abs(Vg[sel] - Vo).max() / np.abs(Vg).max()),
                        "E_dV_dx1": float(np.abs(Gg[sel, 0] - Gxo).max() / np.abs(Gg[:, 0]).max()),
                        "E_dV_dx2": float(np.abs(Gg[sel, 1] - Gyo).max() / np.abs(Gg[:, 1]).max())}
        cb["oracle_check"] = check
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
