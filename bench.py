"""Benchmark: walker-steps/s of Node2Vec walks on R-MAT scale 22 on one MI355X.

A "step" of this benchmark is one whole walk job: one walker per vertex of the
scale-22 R-MAT graph (4.19M walkers), Node2Vec p=0.5 q=2.0 weighted, 80 steps each,
strategies chosen per step by the cost model.  The graph and the start vertices are
resident in HBM before the timed region.  Prints one JSON line on stdout; details go
to stderr.
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

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2512_00705_amd/csrc/fw_kernels.hip", "paper_2512_00705_amd/csrc/fw_device.h",
                  "paper_2512_00705_amd/csrc/fw_internal.h")
TRAFFIC_FILE = "profiles/traffic_walk_kernel_node2vec_rmat22.txt"


PLAN_FIELDS = ("rho", "d_lo", "lds_cap", "bound", "proposal", "rjs_cap", "grid", "hub_deg", "hub_lanes", "rvs_share")


def parse_plan(text: str):
    """A plan from ``rho,d_lo,lds_cap[,bound[,proposal[,rjs_cap[,grid[,hub_deg,hub_lanes[,rvs_share]]]]]]]``;
    omitted fields take fw_plan_default's values."""
    import paper_2512_00705_amd as fw
    f = text.split(",")
    names = PLAN_FIELDS
    if not 3 <= len(f) <= len(names):
        raise SystemExit(f"--plan: expected 3..{len(names)} comma-separated fields, got {len(f)}")
    kw = {n: (float(v) if n == "rho" else int(v)) for n, v in zip(names, f)}
    return fw.fw_plan_default(**kw)


def plan_arg(plan) -> str:
    """The --plan text that reproduces ``plan`` (float rho in full precision)."""
    return ",".join([repr(float(plan.rho))] + [str(int(getattr(plan, n))) for n in
                     PLAN_FIELDS[1:]])


def plan_dict(plan) -> dict:
    return {n: (float(getattr(plan, n)) if n == "rho" else int(getattr(plan, n))) for n in
            PLAN_FIELDS}


def one_off_share(prep_ms, profile_ms, index_ms, alias_ms, tune_ms, job_ms) -> dict:
    """One-off costs beside one walk job.  The paper reports profiling plus preprocessing at
    0.46-3.98 % of total runtime; here the same two (profiling kernels, h_MAX/h_SUM pass)
    and all one-off work (adding the edge index, the proposal records and the autotuner's
    sample walks) are given as a share of themselves plus one job, with the number of jobs
    on a resident graph after which the share falls below 3.98 %."""
    paper_like = prep_ms + profile_ms
    everything = prep_ms + index_ms + alias_ms + tune_ms
    return {"paper_like_ms": paper_like, "all_ms": everything,
            "paper_like_share_one_job": paper_like / (paper_like + job_ms),
            "all_share_one_job": everything / (everything + job_ms),
            "jobs_for_all_below_3.98pct": int(np.ceil(everything * (1 - 0.0398) / (0.0398 * job_ms))),
            "paper_range": "0.46-3.98 % (profile + preprocess, of total)"}


def host_cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_STATS = ("steps", "rjs_steps", "rvs_steps", "rjs_fallbacks", "rjs_trials", "rvs_triggers")


def measured_traffic(plan, st: dict) -> dict | None:
    """HBM traffic of one launch from the committed counter summary, or None unless it was
    taken on this kernel source and on a launch that made the same decisions (the same
    step, trial and fall-back counts, and the same LDS cap when eRVS ran).  Reads are the
    size-resolved TCC->memory read requests (32/64/128 B), writes WRITE_SIZE."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
            return None
        rec = dict(x.split("=") for x in kv["stats"].split(","))
        if any(int(rec[k]) != int(st[k]) for k in TRAFFIC_STATS):
            return None
        if int(st["rvs_steps"]) + int(st["rjs_fallbacks"]) > 0 and int(kv["lds_cap"]) != plan.lds_cap:
            return None
        return {"bytes": 1024.0 * (float(kv["read_kib_per_launch"]) + float(kv["write_kib_per_launch"])),
                "read_requests": float(kv["read_requests_per_launch"])}
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--graph", default="rmat22_labels")
    ap.add_argument("--L", type=int, default=None, help="walk length (default 80; 40 for metapath)")
    ap.add_argument("--p", type=float, default=0.5)
    ap.add_argument("--q", type=float, default=2.0)
    ap.add_argument("--logic", default="node2vec", choices=["node2vec", "secondpr", "metapath"],
                    help="walk logic of the scale-22 job (node2vec p, q; second-order PageRank gamma; MetaPath "
                         "schema 0,1,2,3,4 repeated from 2^20 uniform starts)")
    ap.add_argument("--gamma", type=float, default=0.2)
    ap.add_argument("--weights", default="f32", choices=["f32", "q8"],
                    help="edge property weights as float32, or as 8-bit codes (scale 10/255) of the same weights")
    ap.add_argument("--strategy", default="auto", choices=["auto", "rvs", "rjs"])
    ap.add_argument("--modes", type=int, default=1, help="also time the single-kernel modes")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=0, help="walkers for the CPU baseline (0: sized to ~15 s)")
    ap.add_argument("--workload", default="node2vec", choices=["node2vec", "batched", "served", "skew"],
                    help="node2vec: the headline scale-22 job; batched: 4096 queries on skewed scale 24; "
                         "served: Poisson request stream against a resident scale-25 graph")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-scale", type=int, default=25)
    ap.add_argument("--tick-steps", type=int, default=64)
    ap.add_argument("--skew-scale", type=int, default=20, help="skew: R-MAT scale of the topology")
    ap.add_argument("--skew-L", type=int, default=20, help="skew: walk length")
    ap.add_argument("--plan", default="",
                    help="rho,d_lo,lds_cap[,bound[,proposal[,rjs_cap[,grid[,hub_deg,hub_lanes[,rvs_share]]]]]]]: use this plan "
                         "instead of autotuning (the plan_arg of a bench line)")
    ap.add_argument("--per-query", type=int, default=1, help="batched: also time one launch per query")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB: only run a plain device-to-device copy of this size 3 times (counter calibration)")
    ap.add_argument("--calibrate-random", type=int, default=0,
                    help="MiB: only gather 2^25 random float32 from an array of this size 3 times (counter "
                         "calibration for random reads) and print the gather rate")
    args = ap.parse_args()
    if args.calibrate_random:
        import torch
        dev = torch.device("cuda:0")
        a = torch.ones((args.calibrate_random << 20) // 4, dtype=torch.float32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        idx = torch.randint(0, a.numel(), (1 << 25,), device=dev, generator=g)
        out = torch.empty(1 << 25, dtype=torch.float32, device=dev)
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch.index_select(a, 0, idx, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        print(json.dumps({"random_reads": 1 << 25, "array_bytes": a.numel() * 4, "launches": 3, "ms": ms,
                          "random_reads_per_s": (1 << 25) / (min(ms) / 1e3)}))
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): walkers are independent, so a "
              "multi-GPU run is this job on each GPU's share of the walkers with no exchange", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2512_00705_amd as fw
    import synth

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "skew":
        return bench_skew(args)
    t0 = time.time()
    g = synth.cached(args.graph)
    log(f"graph {args.graph}: nv={g['nv']} ne={g['ne']} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    if args.weights == "q8":  # the same weights stored as 8-bit codes
        g = dict(g)
        g["h8"], g["h_scale"] = synth.quantize_u8(g["h"])
        g["h"] = None
    keys = ("row_ptr", "col", "h", "h8") + (("label",) if args.logic == "metapath" else ())
    t = {k: torch.from_numpy(g[k]).to(dev) for k in keys if g.get(k) is not None}
    gh = fw.fw_graph_create(g["nv"], g["ne"], t["row_ptr"], t["col"], t.get("h"), t.get("label"), on_device=True,
                            h8=t.get("h8"), h_scale=float(g.get("h_scale", 0.0)))
    del t
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fw.fw_graph_preprocess(gh)
    e1.record()
    torch.cuda.synchronize()
    prep_ms = e0.elapsed_time(e1)
    e0.record()
    fw.fw_graph_build_index(gh)
    e1.record()
    torch.cuda.synchronize()
    index_ms = e0.elapsed_time(e1)
    a0 = time.perf_counter()
    fw.fw_graph_build_alias(gh)
    alias_ms = (time.perf_counter() - a0) * 1e3
    label_ms = 0.0
    if args.logic == "metapath":  # label groups for label-conditioned proposals
        a0 = time.perf_counter()
        fw.fw_graph_build_label_alias(gh)
        label_ms = (time.perf_counter() - a0) * 1e3
    if args.logic == "secondpr":
        logic = fw.fw_logic_second_pr(args.gamma, True)
        logic_text = f"second-order PageRank gamma={args.gamma}"
    elif args.logic == "metapath":
        logic = fw.fw_logic_metapath([0, 1, 2, 3, 4], True)
        logic_text = "MetaPath schema (0,1,2,3,4) repeated, labels U{0..4}"
    else:
        logic = fw.fw_logic_node2vec(args.p, args.q, True)
        logic_text = f"node2vec p={args.p} q={args.q}"
    # the paper's one-off costs are its profiling kernels and the preprocessing pass; the
    # profiling kernels alone (fw_plan_profile, which the autotuner also runs) are timed here
    p0 = time.perf_counter()
    fw.fw_plan_profile(gh, logic)
    torch.cuda.synchronize()
    profile_ms = (time.perf_counter() - p0) * 1e3
    t1 = time.time()
    if args.plan:
        plan = parse_plan(args.plan)
    else:
        plan = fw.fw_plan_autotune(gh, logic)
    tune_ms = (time.time() - t1) * 1e3
    log(f"preprocess {prep_ms:.2f} ms, autotune {tune_ms:.1f} ms, plan {plan_arg(plan)}")

    nv, seed = g["nv"], 42
    L = args.L if args.L is not None else (40 if args.logic == "metapath" else 80)
    # walkers: one per vertex, or 2^20 uniform starts for MetaPath
    starts_np = (synth.uniform_starts(nv, 1 << 20, 42) if args.logic == "metapath"
                 else np.arange(nv, dtype=np.int32))
    n = len(starts_np)
    starts = torch.from_numpy(starts_np).to(dev)
    paths = torch.empty((n, L + 1), dtype=torch.int32, device=dev)
    lengths = torch.empty(n, dtype=torch.int32, device=dev)
    stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=dev)
    strat = {"auto": fw.FW_AUTO, "rvs": fw.FW_RVS_ONLY, "rjs": fw.FW_RJS_ONLY}

    def run(mode: str, steps: int, warmup: int, plan=plan, paths=paths, lengths=lengths):
        # one launch with the device counters (steps, trials, algorithmic bytes); the walks
        # are a fixed function of (seed, walker, step), so every launch below takes the
        # same steps; the timed launches run without counters, as a caller would
        stats.zero_()
        fw.fw_walk(gh, logic, plan, strat[mode], starts, n, L, seed, paths, lengths, stats)
        for _ in range(warmup):
            fw.fw_walk(gh, logic, plan, strat[mode], starts, n, L, seed, paths, lengths, None)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in evs:
            a.record()
            fw.fw_walk(gh, logic, plan, strat[mode], starts, n, L, seed, paths, lengths, None)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        fw.fw_graph_check(gh)
        ms = [a.elapsed_time(b) for a, b in evs]
        st = dict(zip(fw.STAT_NAMES, stats.cpu().numpy().tolist()))
        return ms, wall, st

    ms, wall, st = run(args.strategy, args.steps, args.warmup)
    rng = np.random.default_rng(7)
    avg_ms = float(np.mean(ms))
    steps_per_walk = st["steps"]
    value = steps_per_walk / (avg_ms / 1e3)
    achieved = st["alg_bytes"] / (avg_ms / 1e3) / 1e9
    log(f"{args.strategy}: per-walk ms {['%.2f' % x for x in ms]}, wall {wall:.3f}s, stats {st}")

    modes = {}
    if args.modes:
        # own output buffers: the timed job's walks stay for the CPU comparison below
        m_paths, m_lengths = torch.empty_like(paths), torch.empty_like(lengths)
        # the single-kernel modes, and the same job under the other eRJS bounds the logic
        # and graph allow (Node2Vec's split bound and member board need a symmetric graph)
        sym = fw.fw_graph_info(gh)[3]
        cases = [(m + "_only", m, plan) for m in ("rvs", "rjs") if m != args.strategy]
        bounds = ([0, 1, 2] if (args.logic == "node2vec" and sym) else [0] if args.logic in ("node2vec", "metapath")
                  else [0, 2])
        for b in bounds:
            if b != plan.bound:
                other = fw.fw_plan_default(rho=plan.rho, d_lo=plan.d_lo, lds_cap=plan.lds_cap, bound=b,
                                           proposal=plan.proposal)
                cases.append((("paper_bound", "split_bound", "member_board")[b], args.strategy, other))
        names = {0: "uniform_proposals", 1: "h_proposals", 2: "label_proposals"}
        for pr in ([0, 1, 2] if args.logic == "metapath" else [0, 1]):
            if pr != plan.proposal:
                other = fw.fw_plan_default(rho=plan.rho, d_lo=plan.d_lo, lds_cap=plan.lds_cap, bound=plan.bound,
                                           proposal=pr)
                cases.append((names[pr], args.strategy, other))
        paper = fw.fw_plan_default(rho=plan.rho, d_lo=plan.d_lo, lds_cap=plan.lds_cap)
        cases.append(("paper_eRJS", args.strategy, paper))  # uniform proposals, bound max(w) * h_MAX
        for name, m, pl in cases:
            mms, _, mst = run(m, 2, 1, plan=pl, paths=m_paths, lengths=m_lengths)
            a = float(np.mean(mms))
            modes[name] = {"ms": round(a, 3), "walker_steps_per_s": mst["steps"] / (a / 1e3),
                           "alg_GBps": mst["alg_bytes"] / (a / 1e3) / 1e9, "bound": pl.bound,
                           "rjs_steps": mst["rjs_steps"], "rvs_steps": mst["rvs_steps"],
                           "trials_per_rjs_step": mst["rjs_trials"] / max(1, mst["rjs_steps"] + mst["rjs_fallbacks"])}
            log(f"{name}: ms {mms}, stats {mst}")
        del m_paths, m_lengths

    cpu = None
    if args.cpu_baseline:
        import oracle
        og = oracle.Graph(g)
        og.aux()
        lg = (oracle.Logic(kind=oracle.SECOND_PR, weighted=True, gamma=args.gamma) if args.logic == "secondpr"
              else oracle.Logic(kind=oracle.METAPATH, weighted=True, schema=(0, 1, 2, 3, 4))
              if args.logic == "metapath"
              else oracle.Logic(kind=oracle.NODE2VEC, weighted=True, p=args.p, q=args.q))
        pl = oracle.Plan(rho=plan.rho, d_lo=plan.d_lo, rjs_cap=plan.rjs_cap, bound=plan.bound, proposal=plan.proposal,
                         hub_deg=plan.hub_deg, hub_lanes=plan.hub_lanes, rvs_share=bool(plan.rvs_share))
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        smode = {"auto": 0, "rvs": 1, "rjs": 2}[args.strategy]
        k = args.cpu_sample or 2048
        while True:  # grow a seeded walker sample until the oracle works for ~10-30 s
            sample = np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)
            c0 = time.perf_counter()
            r = oracle.walk(og, lg, pl, smode, starts_np[sample], L, seed, walker_ids=sample,
                            diagnostics=False, nthreads=cores)
            cs = time.perf_counter() - c0
            if args.cpu_sample or cs >= 10.0 or k >= n:
                break
            k = int(min(n, k * max(2.0, 15.0 / max(cs, 1e-3))))
        # the GPU run covered these walkers too: compare the sample
        gp = paths[torch.from_numpy(sample).to(dev)].cpu().numpy()
        same = float((gp == r.paths).all(axis=1).mean())
        # a plain CPU sampler beside it: inverse transform sampling over every step's exact
        # weights (cumulative sum, binary search) on the same walkers, same cores
        # (every step reads the whole row: a smaller sample, grown until ~5-15 s of work)
        ki = 64
        while True:
            isub = sample[:ki]
            i0 = time.perf_counter()
            ri = oracle.walk(og, lg, pl, oracle.ITS, starts_np[isub], L, seed, walker_ids=isub,
                             diagnostics=False, nthreads=cores)
            its_s = time.perf_counter() - i0
            if its_s >= 5.0 or ki >= len(sample):
                break
            ki = int(min(len(sample), ki * max(2.0, 8.0 / max(its_s, 1e-3))))
        cpu = {"value": r.counters["steps"] / cs, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(sample)} of {n} walkers (seeded), full {L}-step walks, {cs:.1f}s; "
                         f"{same * 100:.3f}% identical to the GPU walks",
               "cpu": host_cpu_model(), "nproc": os.cpu_count(),
               "its": {"value": ri.counters["steps"] / its_s, "unit": "walker-steps/s", "cores": cores,
                       "sample": f"the first {len(isub)} walkers of that sample, full {L}-step walks, "
                                 f"{its_s:.1f}s"}}
        log(f"cpu oracle: {cpu}")

    fw.fw_graph_destroy(gh)
    # the recorded counters cover the float32-weight Node2Vec job only
    traffic = measured_traffic(plan, st) if (args.weights == "f32" and args.logic == "node2vec") else None
    ceiling = fw.fw_calibrate_random_reads(4 << 30)  # random 8-byte reads/s, 128 B moved each
    random_access = {"ceiling_reads_per_s": ceiling,
                     "achieved_reads_per_s": None if traffic is None else traffic["read_requests"] / (avg_ms / 1e3),
                     "frac": None if traffic is None else traffic["read_requests"] / (avg_ms / 1e3) / ceiling}
    out = {
        "metric": ("walker-steps/sec + achieved HBM GB/s, node2vec R-MAT s22; p99 latency served"
                   if args.logic == "node2vec" else f"walker-steps/sec + achieved HBM GB/s, {args.logic} R-MAT s22"),
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": avg_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{logic_text} weighted h~U(1,10)"
                               + (" stored as 8-bit codes (h = (10/255)*code)" if args.weights == "q8" else "")
                               + ", R-MAT scale 22 "
                               f"(a=0.57,b=0.19,c=0.19, edge factor 16, {g['ne']} CSR entries), "
                               + (f"{n} uniform start vertices (seed 42)" if args.logic == "metapath"
                                  else f"one walker per vertex ({nv})")
                               + f", L={L}, strategy={args.strategy}",
                   "walker_steps_per_walk_job": steps_per_walk, "preprocess_ms": prep_ms,
                   "edge_index_ms": index_ms, "alias_build_ms": alias_ms, "label_groups_build_ms": label_ms,
                   "autotune_ms": tune_ms, "profile_ms": profile_ms,
                   "one_off_share": one_off_share(prep_ms, profile_ms, index_ms, alias_ms + label_ms, tune_ms, avg_ms),
                   "plan": plan_dict(plan), "plan_arg": plan_arg(plan),
                   "stats": st, "modes": modes,
                   "hbm_traffic_GBps": None if traffic is None else traffic["bytes"] / (avg_ms / 1e3) / 1e9,
                   "random_access": random_access},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None if traffic is None else traffic["bytes"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_skew(args):
    """Property-weight skew and selection policy (the paper's power-law / degree-based
    weight study and its selection-strategy comparison): one R-MAT topology, weights
    uniform U(1,10), Pareto(alpha) as numpy.random.pareto draws them for alpha in
    {1, 1.5, 2, 3, 4}, and h(v,u) = d(u); Node2Vec p=0.5 q=2, one walker per vertex.  Each
    setting is autotuned, then timed under the cost model (AUTO), the fair-coin and the
    degree-threshold (1K) selection policies, and the two single-kernel modes."""
    import torch
    import paper_2512_00705_amd as fw
    import synth

    dev = torch.device("cuda:0")
    s = args.skew_scale
    topo = synth.rmat(s, 16 << s, seed=1, weighted=False)
    rp, col = topo["row_ptr"], topo["col"]
    settings = [("uniform", None)] + [(f"pareto{a:g}", a) for a in (1.0, 1.5, 2.0, 3.0, 4.0)] + [("degree", "deg")]
    L, seed, nv = args.skew_L, 42, topo["nv"]
    logic = fw.fw_logic_node2vec(0.5, 2.0, True)
    starts = torch.arange(nv, dtype=torch.int32, device=dev)
    paths = torch.empty((nv, L + 1), dtype=torch.int32, device=dev)
    lengths = torch.empty(nv, dtype=torch.int32, device=dev)
    stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=dev)
    rows = []
    t_rp, t_col = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    for name, a in settings:
        if a is None:
            h, _ = synth.edge_props(rp, col, 1)
        elif a == "deg":
            h = synth.degree_weights(rp, col)
        else:
            h = synth.pareto_weights(rp, col, a, 7)
        t_h = torch.from_numpy(h).to(dev)
        gh = fw.fw_graph_create(nv, topo["ne"], t_rp, t_col, t_h, None, on_device=True)
        fw.fw_graph_preprocess(gh)
        fw.fw_graph_build_index(gh)
        fw.fw_graph_build_alias(gh)
        plan = fw.fw_plan_autotune(gh, logic)
        uni = fw.fw_plan_default(rho=plan.rho, d_lo=plan.d_lo, lds_cap=plan.lds_cap, bound=plan.bound)
        modes = {"auto": (fw.FW_AUTO, plan),
                 "auto_uniform_proposals": (fw.FW_AUTO, uni),
                 "random": (fw.FW_RANDOM_SELECT, plan),
                 "degree": (fw.FW_DEGREE_SELECT, fw.fw_plan_default(d_lo=1000, bound=plan.bound,
                                                                   proposal=plan.proposal, lds_cap=plan.lds_cap)),
                 "rjs_only": (fw.FW_RJS_ONLY, plan),
                 "rvs_only": (fw.FW_RVS_ONLY, plan)}
        row = {"weights": name, "h_max": float(h.max()), "h_median": float(np.median(h)), "plan_rho": plan.rho,
               "plan_bound": plan.bound, "plan_proposal": plan.proposal}
        for m, (strat, pl) in modes.items():
            stats.zero_()  # warm-up launch with the counters; the timed one runs without
            fw.fw_walk(gh, logic, pl, strat, starts, nv, L, seed, paths, lengths, stats)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fw.fw_walk(gh, logic, pl, strat, starts, nv, L, seed, paths, lengths, None)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            st = dict(zip(fw.STAT_NAMES, stats.cpu().numpy().tolist()))
            row[m] = {"ms": round(ms, 3), "steps_per_s": st["steps"] / (ms / 1e3),
                      "rjs_share": (st["rjs_steps"] + st["rjs_fallbacks"]) / max(1, st["steps"]),
                      "trials_per_rjs_step": st["rjs_trials"] / max(1, st["rjs_steps"] + st["rjs_fallbacks"])}
        fw.fw_graph_check(gh)
        fw.fw_graph_destroy(gh)
        del t_h
        for m in ("random", "degree", "rjs_only", "rvs_only"):
            row["auto_speedup_vs_" + m] = row[m]["ms"] / row["auto"]["ms"]
        log(f"{name}: " + ", ".join(f"{m} {row[m]['ms']:.2f} ms" for m in modes) +
            f", auto eRJS share {row['auto']['rjs_share']:.3f}")
        rows.append(row)
    gm = lambda key: float(np.exp(np.mean([np.log(r[key]) for r in rows])))
    steps_auto = [r["auto"]["steps_per_s"] for r in rows]
    print(json.dumps({
        "metric": "walker-steps/sec under property-weight skew (geometric mean over weight settings), AUTO",
        "value": float(np.exp(np.mean(np.log(steps_auto)))), "unit": "walker-steps/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"node2vec p=0.5 q=2 on R-MAT scale {s} (edge factor 16, {topo['ne']} CSR entries), "
                               f"one walker per vertex, L={L}; weights uniform U(1,10), numpy-style Pareto "
                               f"alpha in {{1,1.5,2,3,4}}, and h(v,u)=d(u)",
                   "geomean_auto_speedup_vs_random": gm("auto_speedup_vs_random"),
                   "geomean_auto_speedup_vs_degree": gm("auto_speedup_vs_degree"),
                   "rows": rows}}), flush=True)


def bench_batched(args):
    """4096 Node2Vec queries (per-query p, q, start set, L, seed) on the skewed scale-24
    R-MAT: one captured HIP-graph launch for all of them against one launch per query."""
    import torch
    import paper_2512_00705_amd as fw
    import synth

    t0 = time.time()
    g = synth.cached("rmat24_skew")
    log(f"graph rmat24_skew: nv={g['nv']} ne={g['ne']} max_deg={int(np.diff(g['row_ptr']).max())} "
        f"({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(g[k]).to(dev) for k in ("row_ptr", "col", "h")}
    gh = fw.fw_graph_create(g["nv"], g["ne"], t["row_ptr"], t["col"], t["h"], None, on_device=True)
    del t
    fw.fw_graph_preprocess(gh)
    fw.fw_graph_build_index(gh)
    fw.fw_graph_build_alias(gh)
    qd = synth.batch_queries(g["nv"], 4096, 7)
    # one plan for the batch: tuned over the distinct logics its queries use
    mix = sorted({(float(p), float(q)) for p, q in zip(qd["p"], qd["q"])})
    t0 = time.perf_counter()
    plan = fw.fw_plan_autotune_mix(gh, [fw.fw_logic_node2vec(p, q, True) for p, q in mix])
    tune_ms = (time.perf_counter() - t0) * 1e3
    log(f"autotune over {len(mix)} logics {tune_ms:.0f} ms: rho={plan.rho:.3f} d_lo={plan.d_lo} "
        f"lds_cap={plan.lds_cap} bound={plan.bound} proposal={plan.proposal}")
    starts = torch.from_numpy(qd["starts"]).to(dev)
    paths = torch.empty((qd["total_paths"],), dtype=torch.int32, device=dev)
    lengths = torch.empty((int(qd["n"].sum()),), dtype=torch.int32, device=dev)
    stats = torch.zeros(fw.FW_NSTATS, dtype=torch.int64, device=dev)
    qs, lgs = [], []
    for i in range(4096):
        q = fw.fw_query()
        q.logic = fw.fw_logic_node2vec(float(qd["p"][i]), float(qd["q"][i]), True)
        q.n, q.L, q.seed = int(qd["n"][i]), int(qd["L"][i]), int(qd["seed"][i])
        q.start_off, q.out_off, q.len_off = int(qd["start_off"][i]), int(qd["out_off"][i]), int(qd["len_off"][i])
        qs.append(q)
        lgs.append(q.logic)
    b = fw.fw_batch_create(gh, qs, plan, fw.FW_AUTO, starts, paths, lengths)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # one launch with the device counters, then the captured launch without them
        fw.fw_batch_launch(b, stats, stream)
        for _ in range(args.warmup):
            fw.fw_batch_launch(b, None, stream)
        fw.fw_batch_capture(b, None, stream)
        stream.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e_a, e_b in evs:
            e_a.record(stream)
            fw.fw_batch_replay(b, stream)
            e_b.record(stream)
        stream.synchronize()
    fw.fw_graph_check(gh)
    ms = [e_a.elapsed_time(e_b) for e_a, e_b in evs]
    st = dict(zip(fw.STAT_NAMES, stats.cpu().numpy().tolist()))
    avg = float(np.mean(ms))
    log(f"batched graph replay ms {['%.2f' % x for x in ms]}, stats {st}")
    per_q = None
    if args.per_query:
        e_a, e_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e_a.record()
        for i in range(4096):
            n, L = int(qd["n"][i]), int(qd["L"][i])
            fw.fw_walk(gh, lgs[i], plan, fw.FW_AUTO, starts.data_ptr() + 4 * int(qd["start_off"][i]), n, L,
                       int(qd["seed"][i]), paths.data_ptr() + 4 * int(qd["out_off"][i]),
                       lengths.data_ptr() + 4 * int(qd["len_off"][i]), None)
        e_b.record()
        torch.cuda.synchronize()
        per_q = e_a.elapsed_time(e_b)
        log(f"one launch per query: {per_q:.2f} ms")
    fw.fw_batch_destroy(b)
    fw.fw_graph_destroy(gh)
    out = {
        "metric": "walker-steps/sec, batched node2vec queries on R-MAT scale 24 (a=0.6)",
        "value": st["steps"] / (avg / 1e3),
        "unit": "walker-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": avg,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"4096 node2vec queries, p,q in {{0.25,0.5,1,2,4}}, start sets log-uniform 1..65536 "
                               f"({int(qd['n'].sum())} walkers), L in 5..200, one captured HIP-graph launch, "
                               f"R-MAT scale 24 (0.6,0.175,0.175), {g['ne']} CSR entries",
                   "stats": st, "rho": plan.rho, "d_lo": plan.d_lo,
                   "plan": plan_dict(plan), "autotune_ms": tune_ms,
                   "per_query_launches_ms": per_q,
                   "per_query_walker_steps_per_s": (st["steps"] / (per_q / 1e3)) if per_q else None},
        "roofline": {"bound": "hbm", "achieved": st["alg_bytes"] / (avg / 1e3) / 1e9, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": st["alg_bytes"] / (avg / 1e3) / 1e9 / PEAK_HBM_GBS, "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Poisson arrivals of mixed Node2Vec / MetaPath requests against a resident R-MAT
    graph with labels, served by continuous batching; p50/p99 latency and walker-steps/s."""
    import threading

    import torch
    import paper_2512_00705_amd as fw
    import synth

    t0 = time.time()
    s = args.serve_scale
    g = synth.rmat(s, 16 << s, seed=1, nlabels=5)
    log(f"graph rmat{s}_labels: nv={g['nv']} ne={g['ne']} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(g[k]).to(dev) for k in ("row_ptr", "col", "h", "label")}
    gh = fw.fw_graph_create(g["nv"], g["ne"], t["row_ptr"], t["col"], t["h"], t["label"], on_device=True)
    del t
    nv = g["nv"]
    del g
    fw.fw_graph_preprocess(gh)
    fw.fw_graph_build_index(gh)
    fw.fw_graph_build_alias(gh)
    fw.fw_graph_build_label_alias(gh)
    # one plan for the server: tuned over every logic the requests may carry
    pq = np.array([0.25, 0.5, 1.0, 2.0, 4.0], np.float32)
    mix = [fw.fw_logic_node2vec(float(p), float(q), True) for p in pq for q in pq]
    mix.append(fw.fw_logic_metapath([0, 1, 2, 3, 4], True))
    plan = fw.fw_plan_autotune_mix(gh, mix)
    log(f"plan: rho={plan.rho:.3f} d_lo={plan.d_lo} lds_cap={plan.lds_cap} bound={plan.bound} "
        f"proposal={plan.proposal}")
    budget = 32 << 30
    srv = fw.fw_server_create(gh, plan, fw.FW_AUTO, budget, tick_steps=args.tick_steps, max_active=8192,
                              max_pending=1 << 16)
    rng = np.random.default_rng(11)
    T, lam = args.serve_seconds, args.serve_rate
    arrivals = np.cumsum(rng.exponential(1.0 / lam, int(lam * T * 1.2) + 16))
    arrivals = arrivals[arrivals < T]
    reqs = []
    for i in range(len(arrivals)):
        n = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(65536)))), 1, 65536))
        L = int(rng.integers(10, 101))
        if i % 2 == 0:
            lg = fw.fw_logic_node2vec(float(rng.choice(pq)), float(rng.choice(pq)), True)
        else:
            lg = fw.fw_logic_metapath([0, 1, 2, 3, 4], True)
        reqs.append((lg, n, L, 1000 + i))
    offered_steps = sum(n * L for _, n, L, _ in reqs)
    log(f"{len(reqs)} requests over {T}s, offered {offered_steps / T / 1e6:.1f} M walker-steps/s")
    busy = [0]
    meta = {}
    start = time.perf_counter()

    def submit():
        for i, (lg, n, L, seed) in enumerate(reqs):
            wait = start + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            starts = rng_s.integers(0, nv, n, dtype=np.int64).astype(np.int32)
            while True:
                try:
                    rid = fw.fw_server_submit(srv, lg, starts, L, seed)
                    break
                except fw.FlexiWalkError as e:
                    if e.code != fw.FW_E_BUSY:
                        raise
                    busy[0] += 1
                    time.sleep(0.001)
            meta[rid] = (n, L)

    rng_s = np.random.default_rng(12)
    th = threading.Thread(target=submit)
    th.start()
    lat, done_steps, t_last = [], 0, start
    deadline = start + T + 120
    while len(lat) < len(reqs) and time.perf_counter() < deadline:
        rid = fw.fw_server_next_done(srv, 200)
        if not rid:
            continue
        while rid not in meta:
            time.sleep(0.0005)
        n, L = meta[rid]
        p, ln, l_s = fw.fw_server_result(srv, rid, n, L)
        lat.append(l_s)
        done_steps += int(ln.sum())
        t_last = time.perf_counter()
    th.join()
    st = fw.fw_server_stats(srv)
    fw.fw_server_destroy(srv)
    fw.fw_graph_destroy(gh)
    wall = t_last - start
    lat_ms = np.array(lat) * 1e3
    p50, p99 = float(np.percentile(lat_ms, 50)), float(np.percentile(lat_ms, 99))
    sustained = len(lat) == len(reqs) and wall < T * 1.1 + 1.0
    log(f"served {len(lat)}/{len(reqs)} in {wall:.2f}s, p50 {p50:.2f} ms, p99 {p99:.2f} ms, stats {st}, "
        f"busy retries {busy[0]}")
    out = {
        "metric": "walker-steps/sec + p50/p99 latency served, mixed node2vec/metapath requests",
        "value": done_steps / wall, "unit": "walker-steps/s", "n_gpus": 1, "steps": len(lat), "warmup": 0,
        "ms_per_step": p50, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Poisson arrivals {lam:.0f} req/s for {T:.0f}s, half node2vec (p,q in "
                               f"{{0.25..4}}), half metapath schema (0,1,2,3,4) repeated, start sets log-uniform "
                               f"1..65536, L in 10..100, resident R-MAT scale {s} with labels, continuous "
                               f"batching (tick {args.tick_steps} steps), budget {budget >> 30} GiB",
                   "p50_ms": p50, "p99_ms": p99, "requests": len(reqs), "completed": len(lat),
                   "sustained": sustained, "offered_walker_steps_per_s": offered_steps / T, "server": st,
                   "plan": plan_dict(plan),
                   "busy_retries": busy[0], "rho": plan.rho},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
