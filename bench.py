"""Benchmark of the flow-shop bounding path on one MI355X.

Default workload (the headline): one decomposition step = pfsp_bound_children
with the full two-machine bound LB2 (all 190 machine pairs) over 1,048,576
random bidirectional partial schedules of one n=20 x m=20 instance with
p ~ U[1,99], including the MinMin branching decision and the prune flags.
The metric is children bounded per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
    python bench.py --workload search|multi|learned [...]

Prints one JSON line.  Other workloads (not the headline): `search` = the
device depth-first B&B on n=20 x m=10 instances (seeds 1..8, NEH incumbent)
to proven optimality; `multi` = 64 instances of mixed (n, m) bounded in one
persistent graph launch, autotuned shape vs default; `learned` = full LB2
vs learned-pair LB2 searches to the same proven optimum (by default the
20 x 20-trained selector in its int8 form, top-32 pairs; --float-selector,
--topk and --selector select the other variants).  The dominant kernel's
roofline entry divides the
kernel's algorithmic integer operations (formula in alg_ops_lb2) by its mean
duration measured with HIP events on the library stream over the timed
steps.  The CPU baseline is the plain oracle on a bounded sample of the same
pool, on the host cores available to this process (at most 16).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "children bounded/sec (LB2) on 1 MI355X + time-to-optimal; learned-pair vs full LB2"
# MI355X: 256 CUs x 4 SIMD16 = 64 int32 lanes per CU per clock at 2.4 GHz
PEAK_INT32_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8e12


def alg_ops_lb2(n, m, d1, d2):
    """Algorithmic int32 operations of full LB2 for the given parents.

    The O(1)-per-child reformulation of the two-machine bound run over the
    parent's r = n - d unscheduled jobs only (the jobs' Johnson positions in
    each pair's order), counting the operations the method cannot avoid:
      per machine pair and unscheduled job: forward scan 3 (term, prefix
      maximum, running sum), backward scan 4 (suffix maximum, X_a = max(PM -
      (b - a), SM), X_b = X_a + b - a), children 4 (an add and a max for
      each direction);
      per child (2r of them) and machine: 4 for its start times and LB1.
    So 11 r P + 8 r m per parent (a parent with one job left needs LB1 only:
    8 m).  Every kernel issues at least this many lane operations per parent,
    so achieved / peak stays at most 1 at every depth.
    """
    P = m * (m - 1) // 2
    r = n - d1.astype(np.int64) - d2.astype(np.int64)
    ops = np.where(r >= 2, 11 * r * P + 8 * r * m, 8 * m)
    return int(ops.sum())


def yardstick_ops_lb2(n, m, d1, d2):
    """The count fixed before any kernel was written, P (n + 32 (n - d)) per
    parent: one pass over all n Johnson positions per pair plus 16 operations
    per child, pair and direction.  It over-counts the children and
    under-counts the scans (its fraction exceeds 1 at the root), so it is
    reported only as a yardstick next to the algorithmic count."""
    P = m * (m - 1) // 2
    r = n - d1.astype(np.int64) - d2.astype(np.int64)
    return int((P * (n + 32 * r)).sum())


def bytes_lb2(n, m, count):
    """Algorithmic HBM bytes of k_lb2: node records and parent costs in,
    bounds, prune flags and directions out."""
    per = (n + 2) + 3 * m * 4 + 2 * n * 4 + 2 * n + 1
    return per * count


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE scaled by a probe copy of known size), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_lb2q_20x20_1M.md")
    try:
        text = open(path).read()
        rec = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for f in ("bound.hip", "wave.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2012_09511_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if rec.get("source_sha256") != h.hexdigest() or not rec["kernel"].startswith(kernel):
        return None
    return rec


def host_cpu():
    """Cores this process may use, the machine's logical CPU count and model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), os.cpu_count(), model


def cpu_baseline(p, perm, d1, d2, kind, target_s=12.0, threads=None):
    import oracle
    cores, nproc, model = host_cpu()
    if threads is None:
        threads = cores
    # calibrate on samples growing until one takes 0.5 s (thread start-up
    # dominates tiny ones), then run ~target_s of work
    k = 64
    while True:
        t = time.perf_counter()
        oracle.bound_children(p, perm[:k], d1[:k], d2[:k], kind, threads=threads)
        dt = max(time.perf_counter() - t, 1e-3)
        if dt >= 0.5 or k >= len(perm):
            break
        k = min(len(perm), k * 4)
    k2 = int(min(len(perm), max(k, k * target_s / dt)))
    t = time.perf_counter()
    oracle.bound_children(p, perm[:k2], d1[:k2], d2[:k2], kind, threads=threads)
    dt = time.perf_counter() - t
    n = p.shape[0]
    children = int((2 * (n - d1[:k2].astype(np.int64) - d2[:k2].astype(np.int64))).sum())
    return dict(value=children / dt, unit="children/s", cores=threads, kind="oracle",
                sample=f"first {k2} parents of the same pool ({children} children), "
                       f"{dt:.1f} s" + (", OpenMP over parents" if threads > 1 else ""),
                nproc=nproc, cpu_model=model)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--parents", type=int, default=1 << 20)
    ap.add_argument("--kind", default="LB2_FULL", choices=["LB1", "LB2_FULL"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the fixed-depth sweep (profiles of the headline launch alone)")
    ap.add_argument("--headline-only", action="store_true",
                    help="bound workload without the search and learned summaries")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", default="bound", choices=["bound", "search", "multi", "learned"])
    ap.add_argument("--selector", default=os.path.join(ROOT, "paper_2012_09511_amd", "data",
                                                       "selector_n20m20.npy"),
                    help="learned workload: trained weights (selector_n50m20.npy: the 50 x 20 "
                         "training set)")
    ap.add_argument("--topk", type=int, default=32, help="pairs kept by the learned selector")
    ap.add_argument("--float-selector", action="store_true",
                    help="learned workload: rank pairs with the float model instead of its "
                         "int8 form")
    ap.add_argument("--pool-batch", type=int, default=0,
                    help="learned workload: nodes popped per search step (0 = 262144, the "
                         "fastest of 2^16 .. 2^20 for both the full and the learned search)")
    ap.add_argument("--no-graph", action="store_true",
                    help="search steps as plain launches (profilers see graph replays as one)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the bounding path has no multi-GPU mode in this "
              "build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2012_09511_amd import binding, inputs

    if args.workload == "search":
        return bench_search(args)
    if args.workload == "multi":
        return bench_multi(args)
    if args.workload == "learned":
        return bench_learned(args)
    n, m, N = 20, 20, args.parents
    p = inputs.instance(n, m, 2012)
    perm, d1, d2 = inputs.random_pool(n, N, 9511)
    ctx = binding.Context(0)
    ctx.load_instance(p)
    ub, _ = ctx.neh()
    kind = getattr(binding, args.kind)
    dev = [torch.from_numpy(a).cuda() for a in (perm, d1, d2)]
    out_lb = torch.empty((N, 2, n), dtype=torch.int32, device="cuda")
    out_pr = torch.empty((N, 2, n), dtype=torch.uint8, device="cuda")
    out_dir = torch.empty(N, dtype=torch.uint8, device="cuda")
    children = int((2 * (n - d1.astype(np.int64) - d2.astype(np.int64))).sum())

    if args.copy_probe:
        _copy_probe(torch)
    for _ in range(args.warmup):
        ctx.bound_children(*dev, kind=kind, ub=ub, out_lb=out_lb, out_prune=out_pr,
                           dir_out=out_dir)
    torch.cuda.synchronize()
    ctx.check()
    ctx.set_option("timing", 1)
    ctx.kernel_time("k_lb2", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.bound_children(*dev, kind=kind, ub=ub, out_lb=out_lb, out_prune=out_pr,
                           dir_out=out_dir)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    kt = {k: ctx.kernel_time(k) for k in ("k_costs", "k_lb1", "k_lb2", "k_lb2d")}
    ctx.kernel_time("k_lb2", reset=True)   # (reset clears every kernel's total)
    ctx.set_option("timing", 0)
    per_launch = {k: ms / l for k, (ms, l) in kt.items() if l > 0}
    elapsed = t1 - t0
    value = children * args.steps / elapsed
    if kind != binding.LB1:
        roof = lb2_roofline(n, m, d1, d2, per_launch, ctx.get_option("deep_r"))
    else:
        b = bytes_lb2(n, m, N)
        dom_ms = per_launch["k_lb1"]
        achieved = b / (dom_ms * 1e-3)
        roof = dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=achieved / PEAK_HBM, traffic=None, kernel="k_lb1", kernel_ms=dom_ms)
    out = dict(metric=METRIC, value=value, unit="children/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=elapsed / args.steps * 1e3,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="int32",
               data="synthetic",
               config=dict(workload=f"{args.kind} decomposition of {N} random bidirectional "
                                    f"partial schedules, one n=20 x m=20 instance, p~U[1,99]",
                           n=n, m=m, parents=N, children=children, lb_kind=args.kind, ub=ub,
                           instance_seed=2012, pool_seed=9511,
                           deep_r=ctx.get_option("deep_r")),
               roofline=roof, kernels_ms=per_launch)
    if kind != binding.LB1 and not args.no_sweep:
        out["depth_sweep"] = depth_sweep(ctx, torch, binding, inputs, n, m, ub)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, perm, d1, d2, kind)
        out["cpu_baseline_1core"] = cpu_baseline(p, perm, d1, d2, kind, target_s=8.0, threads=1)
    ctx.close()
    if not args.headline_only:
        out["search"] = search_summary(args, with_cpu=not args.no_cpu)
        out["learned"] = learned_summary(args)
    print(json.dumps(out))


def lb2_roofline(n, m, d1, d2, per_launch, deep_r):
    """Roofline entry of the LB2 stage: each kernel's algorithmic operations
    (alg_ops_lb2 over the parents it bounds) over its mean launch time."""
    r = n - d1.astype(np.int64) - d2.astype(np.int64)
    deep = (r <= deep_r) if deep_r else np.zeros_like(r, dtype=bool)
    parts = {"k_lb2": ~deep, "k_lb2d": deep}
    ker = {}
    for k, sel in parts.items():
        if k in per_launch and sel.any():
            ops = alg_ops_lb2(n, m, d1[sel], d2[sel])
            ker[k] = dict(parents=int(sel.sum()), alg_ops=ops, ms=per_launch[k],
                          frac=ops / (per_launch[k] * 1e-3) / PEAK_INT32_OPS)
    dom = max(ker, key=lambda k: ker[k]["ms"])
    ops_all = alg_ops_lb2(n, m, d1, d2)
    ms_all = sum(v["ms"] for v in ker.values())
    prof = profiled_traffic("pfsp::k_lb2q<20, false, true>")
    return dict(bound="alu", achieved=ker[dom]["alg_ops"] / (ker[dom]["ms"] * 1e-3) / 1e12,
                peak=PEAK_INT32_OPS / 1e12, unit="TOP/s", frac=ker[dom]["frac"],
                traffic=prof["traffic_bytes"] if prof and dom == "k_lb2" else None,
                kernel=dom, kernel_ms=ker[dom]["ms"], alg_ops_per_launch=ker[dom]["alg_ops"],
                op_count="11 r P + 8 r m per parent (members-only O(1)-per-child LB2, r jobs "
                         "left, P pairs): alg_ops_lb2",
                valu_issue_frac=prof["valu_issue_frac"] if prof and dom == "k_lb2" else None,
                kernels=ker,
                lb2_stage=dict(ms=ms_all, frac=ops_all / (ms_all * 1e-3) / PEAK_INT32_OPS),
                yardstick_frac=yardstick_ops_lb2(n, m, d1, d2) / (ms_all * 1e-3) /
                PEAK_INT32_OPS)


def depth_sweep(ctx, torch, binding, inputs, n, m, ub, depths=(0, 5, 10, 12, 15, 18),
                N=1 << 18):
    """LB2 stage time (whichever of k_lb2 / k_lb2d bounds the pool) and
    roofline fraction on pools of one fixed depth d (d1 ~ U{0..d})."""
    res = {}
    for d in depths:
        perm, d1, d2 = inputs.random_pool(n, N, 9600 + d, depth=d)
        dev = [torch.from_numpy(a).cuda() for a in (perm, d1, d2)]
        ctx.bound_children(*dev, kind=binding.LB2_FULL, ub=ub)
        torch.cuda.synchronize()
        ctx.set_option("timing", 1)
        ctx.kernel_time("k_lb2", reset=True)
        for _ in range(5):
            ctx.bound_children(*dev, kind=binding.LB2_FULL, ub=ub)
        torch.cuda.synchronize()
        ms = {k: ctx.kernel_time(k)[0] / 5 for k in ("k_lb2", "k_lb2d")}
        ctx.kernel_time("k_lb2", reset=True)
        ctx.set_option("timing", 0)
        t = ms["k_lb2"] + ms["k_lb2d"]
        children = 2 * (n - d) * N
        res[str(d)] = dict(parents=N, kernel="k_lb2d" if ms["k_lb2d"] > ms["k_lb2"] else "k_lb2",
                           ms=round(t, 4), children_per_s=children / (t * 1e-3),
                           frac=alg_ops_lb2(n, m, d1, d2) / (t * 1e-3) / PEAK_INT32_OPS)
    return res


def _copy_probe(torch):
    src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
    junk = torch.empty(1 << 29, dtype=torch.int32, device="cuda")
    junk.fill_(1)                      # evicts src from the caches
    del junk
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def search_summary(args, with_cpu=True):
    """Time to proven optimality of the device B&B on n=20 x m=10, p~U[1,99],
    seeds 1..8 from NEH + 1, with LB1 and with full LB2 (65,536 nodes per step),
    each optimum asserted equal to the CPU oracle's.  CPU baselines: the
    oracle's depth-first search on one core (LB1) and its OpenMP-task search
    on every usable core (LB1 and LB2)."""
    import oracle
    from paper_2012_09511_amd import binding, inputs
    ctx = binding.Context(0)
    cores, nproc, model = host_cpu()
    ref = {}
    for seed in range(1, 9):
        p = inputs.instance(20, 10, seed)
        ub0, _ = oracle.neh(p)
        r = oracle.search(p, ub0 + 1, oracle.LB1, threads=cores)
        assert r["proven"] and r["found"]
        ref[seed] = r["best"]
    rows, tot = [], {}
    for kind_name in ("LB1", "LB2_FULL"):
        kind = getattr(binding, kind_name)
        t_all = nodes = ch = 0
        for seed in range(1, 9):
            p = inputs.instance(20, 10, seed)
            ctx.load_instance(p)
            ub0, _ = ctx.neh()
            ctx.search(ub0 + 1, 0, kind)          # warm-up: graph build, allocation
            t = time.perf_counter()
            r = ctx.search(ub0 + 1, 0, kind)
            dt = time.perf_counter() - t
            assert r["proven"] and r["found"] and r["best"] == ref[seed], (kind_name, seed)
            assert oracle.makespan(p, r["perm"]) == r["best"]
            rows.append(dict(kind=kind_name, seed=seed, best=r["best"], nodes=r["nodes"],
                             seconds=round(dt, 5)))
            t_all += dt
            nodes += r["nodes"]
            ch += r["children"]
        tot[kind_name] = dict(seconds=t_all, nodes=nodes, nodes_per_s=nodes / t_all,
                              children_per_s=ch / t_all)
    ctx.close()
    out = dict(workload="depth-first B&B to proven optimality, n=20 x m=10, p~U[1,99], "
                        "seeds 1..8, incumbent NEH+1, 65536 nodes per step; optima equal "
                        "the oracle's", lb1=tot["LB1"], lb2=tot["LB2_FULL"], instances=rows)
    if with_cpu:
        cpu = {}
        for name, kind, threads in (("lb1_1core", oracle.LB1, 1), ("lb1_all", oracle.LB1, cores),
                                    ("lb2_all", oracle.LB2_FULL, cores)):
            t = time.perf_counter()
            for seed in range(1, 9):
                p = inputs.instance(20, 10, seed)
                ub0, _ = oracle.neh(p)
                r = oracle.search(p, ub0 + 1, kind, threads=threads)
                assert r["best"] == ref[seed]
            cpu[name] = dict(seconds=time.perf_counter() - t, cores=threads)
        out["cpu_baseline"] = dict(kind="oracle", nproc=nproc, cpu_model=model,
                                   sample="the same 8 instances to the same optima: "
                                          "recursive DFS (1 core), OpenMP-task DFS with a "
                                          "shared incumbent (all usable cores)", **cpu)
    return out


def bench_search(args):
    """The search workload alone, as its own JSON line."""
    s = search_summary(args, with_cpu=not args.no_cpu)
    out = dict(metric="time to proven optimum, 8 instances (device B&B)",
               value=s["lb2"]["seconds"], unit="s", n_gpus=1, steps=1, warmup=1,
               ms_per_step=s["lb2"]["seconds"] * 1e3, higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="int32", data="synthetic",
               config=dict(workload=s["workload"], lb_kind="LB2_FULL"), **{
                   k: v for k, v in s.items() if k != "workload"})
    print(json.dumps(out))


def bench_multi(args):
    """64 instances, (n, m) round-robin over {20,50,100} x {5,10,20}, 25% job-correlated,
    16,384 random parents each, LB2 in one persistent graph launch."""
    import torch
    from paper_2012_09511_amd import binding, inputs
    ctx = binding.Context(0)
    insts = inputs.mixed_instances(64, 4000)
    stride = max(n for n, _, _ in insts)
    per = 16384
    perms, d1s, d2s, seg = [], [], [], [0]
    children = 0
    for k, (n, m, p) in enumerate(insts):
        perm, d1, d2 = inputs.random_pool(n, per, 5000 + k)
        pad = np.zeros((per, stride), dtype=np.uint8)
        pad[:, :n] = perm
        perms.append(pad)
        d1s.append(d1)
        d2s.append(d2)
        seg.append(seg[-1] + per)
        children += int((2 * (n - d1.astype(np.int64) - d2.astype(np.int64))).sum())
    perm = torch.from_numpy(np.concatenate(perms)).cuda()
    d1 = torch.from_numpy(np.concatenate(d1s)).cuda()
    d2 = torch.from_numpy(np.concatenate(d2s)).cuda()
    seg = np.array(seg)
    ub = np.full(64, binding.INT32_MAX, dtype=np.int32)
    mt = binding.Multi(ctx, [p for _, _, p in insts])
    out_bufs = mt.outputs(perm.shape[0], stride)

    def run(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            mt.bound(perm, d1, d2, seg, ub, binding.LB2_FULL, out=out_bufs)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / k

    run(args.warmup)
    default_s = run(args.steps)
    rep = mt.autotune(perm, d1, d2, seg, ub, binding.LB2_FULL, out=out_bufs, reps=2)
    run(args.warmup)
    tuned_s = run(args.steps)
    d1h, d2h = d1.cpu().numpy(), d2.cpu().numpy()
    ops = sum(alg_ops_lb2(n, m, d1h[seg[k]:seg[k + 1]], d2h[seg[k]:seg[k + 1]])
              for k, (n, m, _) in enumerate(insts))
    roof = dict(bound="alu", achieved=ops / tuned_s / 1e12, peak=PEAK_INT32_OPS / 1e12,
                unit="TOP/s", frac=ops / tuned_s / PEAK_INT32_OPS, traffic=None,
                kernel="whole graph launch (costs + every class kernel)",
                alg_ops_per_launch=ops, op_count="P*(n+32(n-d)) per parent, summed")
    out = dict(metric="children bounded/sec (LB2), 64 mixed instances, one graph launch",
               value=children / tuned_s, unit="children/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=tuned_s * 1e3, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="int32", data="synthetic",
               config=dict(workload="64 instances (n,m) in {20,50,100}x{5,10,20}, 25% "
                                    "job-correlated, 16384 random parents each, LB2_FULL",
                           parents=int(perm.shape[0]), children=children),
               roofline=roof,
               default_shape=dict(ms=default_s * 1e3, children_per_s=children / default_s),
               autotuned=rep)
    mt.close()
    ctx.close()
    print(json.dumps(out))


def bench_learned(args):
    """Full LB2 vs learned-pair LB2 (top-k) searches to the same proven optimum."""
    import torch
    from paper_2012_09511_amd import binding, inputs, selector_quant
    ctx = binding.Context(0)
    params = np.load(args.selector, allow_pickle=False)
    ctx.selector_set(params)
    ctx.set_option("learned_topk", args.topk)
    ctx.set_option("pool_batch", args.pool_batch or 1 << 18)
    if args.no_graph:
        ctx.set_option("use_graph", 0)
    rows = []
    modes = (("full", binding.LB2_FULL), ("learned", binding.LB2_LEARNED))
    for seed in range(600, 608):
        p = inputs.instance(20, 20, seed)
        ctx.load_instance(p)
        if not args.float_selector:   # int8 form, calibrated on random nodes of this instance
            ctx.selector_set_quant(selector_quant.quantize(
                params, selector_quant.calibration_features(ctx, 20, 4096, seed)))
        ub0, _ = ctx.neh()
        for _, kind in modes:   # untimed: workspaces and graph capture for this instance
            ctx.search(ub0 + 1, 1, kind)
        res = {}
        for name, kind in modes:
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ctx.search(ub0 + 1, 0, kind)
            res[name] = dict(best=r["best"], proven=r["proven"], nodes=r["nodes"],
                             children=r["children"], seconds=time.perf_counter() - t)
        assert res["full"]["best"] == res["learned"]["best"]
        assert res["full"]["proven"] and res["learned"]["proven"]
        res["prune_rate_loss"] = prune_rate_loss(ctx, torch, binding, inputs, res["full"]["best"],
                                                 seed)
        rows.append(dict(seed=seed, **res))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    tf = sum(x["full"]["seconds"] for x in rows)
    tl = sum(x["learned"]["seconds"] for x in rows)
    nf = sum(x["full"]["nodes"] for x in rows)
    nl = sum(x["learned"]["nodes"] for x in rows)
    out = dict(metric="time to the same proven optimum, learned-pair vs full LB2",
               value=tf / tl, unit="speedup", n_gpus=1, steps=1, warmup=0,
               ms_per_step=tl * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="int32", data="synthetic",
               config=dict(workload="depth-first B&B, n=20 x m=20, seeds 600..607, NEH+1, "
                                    f"{ctx.get_option('pool_batch')} nodes per step, "
                                    f"learned top-{args.topk} of 190 pairs, "
                                    + ("float" if args.float_selector else "int8") + " selector "
                                    + os.path.basename(args.selector)),
               full_seconds=tf, learned_seconds=tl, node_ratio=nl / nf,
               prune_rate_loss=float(np.mean([x["prune_rate_loss"] for x in rows])),
               instances=rows)
    ctx.close()
    print(json.dumps(out))


def prune_rate_loss(ctx, torch, binding, inputs, opt, seed, N=1 << 16):
    """Share of the children that full LB2 prunes at the optimum (LB >= opt)
    and the learned bound does not, over those full LB2 prunes, on N random
    nodes of the loaded instance (same children for both bounds)."""
    n = 20
    perm, d1, d2 = inputs.random_pool(n, N, 9900 + seed)
    dev = [torch.from_numpy(a).cuda() for a in (perm, d1, d2)]
    lf, pf, _, _ = ctx.bound_children(*dev, kind=binding.LB2_FULL, ub=opt)
    pl = ctx.bound_children(*dev, kind=binding.LB2_LEARNED, ub=opt)[1]
    torch.cuda.synchronize()
    live = lf < binding.INT32_MAX
    full_pr = (pf.bool() & live).sum().item()
    lost = (pf.bool() & ~pl.bool() & live).sum().item()
    return lost / max(full_pr, 1)


if __name__ == "__main__":
    main()
