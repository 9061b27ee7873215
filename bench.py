#!/usr/bin/env python3
"""Benchmark of the MI355X branch-MPC hot path (one JSON line on stdout).

Default workload: the tree-Riccati microbenchmark, nx=12, nu=4, horizon 40,
binary branching at stages 0, 4, ..., 36 (1024 scenarios, 8,185 nodes), FP64.
One step = one tree-LQR solve through the C ABI (level-parallel backward
Riccati + path forward rollout, costates included) on inputs already
resident in HBM.  Steps rotate over 12 independent instances (about 0.5 GB)
so that the 256 MB Infinity Cache cannot hold the working set.

Also reported: per-kernel HIP-event times measured inside the timed region,
the roofline of the dominant kernel, branch-MPC solve figures when the
solver is built, and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
METRIC = "BMPC solves/sec & tree-Riccati nodes/sec at KKT 1e-6, 1 GPU; warm vs cold iters"


def progress(msg):
    """One progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lqr_algorithmic(parent, nx, nu):
    """Algorithmic bytes and FLOPs of one backward and one forward launch.

    Backward: every input read once (A, B, c per edge; Q, R, M, q, r per
    control node; Q, q per leaf) and K, k, P, p written once per node.
    Forward: K, k, A, B, c, P, p read once, x, u, lam written once per node.
    FLOPs (dense): per edge 4n^3 + 4n^2 m + 2n m^2 + 4n^2 + 2nm, per control
    node m^3/3 + 2m^2 n + 2m n^2 + 2m^2 + 2mn (backward); per edge
    4n^2 + 2nm + 2n plus 2n^2 for the costate (forward)."""
    N = len(parent)
    nch = np.bincount(parent[1:], minlength=N)
    ctrl = int((nch > 0).sum())
    leaves = N - ctrl
    edges = N - 1
    n, m = nx, nu
    d = 8
    bwd_bytes = d * (edges * (n * n + n * m + n) + ctrl * (n * n + m * m + m * n + n + m)
                     + leaves * (n * n + n) + N * (m * n + m + n * n + n))
    fwd_bytes = d * (ctrl * (m * n + m) + edges * (n * n + n * m + n) + N * (n * n + n)
                     + N * (n + m + n))
    bwd_flops = edges * (4 * n ** 3 + 4 * n * n * m + 2 * n * m * m + 4 * n * n + 2 * n * m) + \
        ctrl * (m ** 3 / 3 + 2 * m * m * n + 2 * m * n * n + 2 * m * m + 2 * m * n)
    fwd_flops = edges * (4 * n * n + 2 * n * m + 2 * n) + N * 2 * n * n
    return {"bwd_bytes": bwd_bytes, "fwd_bytes": fwd_bytes, "bwd_flops": bwd_flops,
            "fwd_flops": fwd_flops}


def lqr_solve_algorithmic_bytes(parent, nx, nu):
    """Algorithmic bytes of one tree-LQR solve with no intermediate stored:
    every input read once (A, B, c per edge; Q, R, q, r per control node;
    Q_f, q_f per leaf) and x, u, lam written once.  Returns (bytes read by
    the backward pass, bytes of the whole solve).  For nx = 12, nu = 4 that
    is 1,632 B per edge, 1,408 B per control node and 1,248 B per leaf read,
    24.7 MB and 26.5 MB for the 8,185-node tree."""
    N = len(parent)
    nch = np.bincount(parent[1:], minlength=N)
    ctrl = int((nch > 0).sum())
    leaves = N - ctrl
    n, m, d = nx, nu, 8
    reads = d * ((N - 1) * (n * n + n * m + n) + ctrl * (n * n + m * m + n + m) + leaves * (n * n + n))
    writes = d * (N * 2 * n + ctrl * m)
    return reads, reads + writes


def host_info():
    """Host cores, CPU model and clock, as the kernel reports them."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "cpu_mhz": mhz}


def baseline_cores():
    """Worker count for the CPU baselines: every host core, at most 16 (the
    host share of one GPU)."""
    return max(1, min(16, os.cpu_count() or 1))


SOLVER_SRCS = ["paper_2506_13624_amd/csrc/bmpc_solver.hip", "paper_2506_13624_amd/csrc/bmpc_device.hpp",
               "paper_2506_13624_amd/csrc/lqr_device.hpp", "paper_2506_13624_amd/csrc/cvf_device.hpp"]


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, srcs):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    e = tab.get(kernel)
    if not e or e.get("source_digest") != source_digest(srcs):
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline_lqr(inst, budget_s=10.0):
    """The oracle's serial tree Riccati (built -O3 -march=native for this
    host), independent solves of the same tree on every host core (one per
    thread; the C oracle runs outside the interpreter lock), for about
    budget_s seconds."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.use_native_build()
    cores = baseline_cores()
    oracle.tree_lqr_inst(inst)  # warm
    t1 = time.perf_counter()
    oracle.tree_lqr_inst(inst)
    one_core = time.perf_counter() - t1

    def worker(_):
        k = 0
        while time.perf_counter() - t0 < budget_s:
            oracle.tree_lqr_inst(inst)
            k += 1
        return k
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        n = sum(ex.map(worker, range(cores)))
    el = time.perf_counter() - t0
    N = len(inst.parent)
    return {"value": N * n / el, "unit": "tree-Riccati nodes/s", "cores": cores, "kind": "oracle",
            "one_core_nodes_per_s": round(N / one_core, 1), "build": "gcc -O3 -march=native",
            "host": host_info(),
            "sample": f"{n} serial tree-Riccati solves (backward + forward) of the nx=12, nu=4, "
                      f"8,185-node tree in {el:.1f} s, one solve per thread on {cores} host cores"}


def _stages(parent):
    st = np.zeros(len(parent), dtype=np.int64)
    for i in range(1, len(parent)):
        st[i] = st[parent[i]] + 1
    return st


def critical_path_floor(torch, L, par, nx, nu, layout, bwd_name, full_us, steps, warmup, seed=77):
    """Dependency floor of a level-parallel backward kernel: the same kernel
    on the tree's critical path alone, one root-to-leaf path of the same
    depth with a leaf stub on each of its branch nodes (so every merge on the
    path is still done), timed like the full tree.  Its time is what the
    depth costs with no width."""
    import bmpc_synth as S
    from paper_2506_13624_amd.layout import empty, to_device

    N = len(par)
    stages = _stages(par)
    depth = int(stages.max())
    branch_stages = sorted({int(v) for v in stages[np.bincount(par[1:], minlength=N) > 1]})
    # deepest leaf's path in any order: node k at stage k, then the stubs
    cat = list(range(-1, depth)) + branch_stages
    _, cat_par = L.bmpc_tree_order(np.array(cat, dtype=np.int32))
    cinst = S.lqr_on(cat_par, nx, nu, seed=seed)
    ctree = L.bmpc_tree_create(cat_par)
    cplan = L.bmpc_lqr_plan_create(ctree, nx, nu, layout)
    Nc = len(cat_par)
    cd = {k: to_device(getattr(cinst, k), layout) for k in "ABcQRMqr"}
    cx0 = to_device(cinst.x0, layout)
    couts = [empty((Nc, nx)), empty((Nc, nu)), empty((Nc, nx))]

    def cstep():
        L.bmpc_lqr_solve(cplan, cd["A"], cd["B"], cd["c"], cd["Q"], cd["R"], cd["M"], cd["q"], cd["r"],
                         cx0, *couts, variant=L.RICCATI_LEVEL)
    for _ in range(max(1, warmup)):
        cstep()
    torch.cuda.synchronize()
    L.bmpc_profile_only(bwd_name)
    L.bmpc_profile_enable(True)
    for _ in range(steps):
        cstep()
    torch.cuda.synchronize()
    cprof = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    L.bmpc_profile_only(None)
    cst, cbad = L.bmpc_lqr_check(cplan)
    L.bmpc_lqr_plan_destroy(cplan)
    L.bmpc_tree_destroy(ctree)
    if cst != 0:
        raise RuntimeError(f"critical-path LQR solve failed (status {cst}, node {cbad})")
    c_ms, c_n = cprof[bwd_name]
    c_us = c_ms / c_n * 1e3
    return {"tree": f"one root-to-leaf path of {depth + 1} nodes with a leaf stub on each of its "
                    f"{len(branch_stages)} branch nodes ({Nc} nodes)",
            "kernel": bwd_name, "backward_us": round(c_us, 2), "per_stage_us": round(c_us / (depth + 1), 3),
            "full_tree_backward_us": round(full_us, 2), "full_tree_over_floor": round(full_us / c_us, 3)}


def run_lqr(args, torch, L):
    from paper_2506_13624_amd.layout import empty, to_device
    import bmpc_synth as S

    n_inst = 12
    insts = [S.lqr_microbench(i) for i in range(n_inst)]
    par = insts[0].parent
    N = len(par)
    nx, nu = 12, 4
    layout = L.LAYOUT_NODE_MAJOR
    tree = L.bmpc_tree_create(par)
    plan = L.bmpc_lqr_plan_create(tree, nx, nu, layout)
    dev = []
    for inst in insts:
        d = {k: to_device(getattr(inst, k), layout) for k in "ABcQRMqr"}
        d["x0"] = to_device(inst.x0, layout)
        d["x"] = empty((N, nx))
        d["u"] = empty((N, nu))
        d["lam"] = empty((N, nx))
        d["K"] = empty((N, nu, nx))
        d["k"] = empty((N, nu))
        d["P"] = empty((N, nx, nx))
        d["p"] = empty((N, nx))
        dev.append(d)

    def step(i):
        d = dev[i % n_inst]
        L.bmpc_lqr_solve(plan, d["A"], d["B"], d["c"], d["Q"], d["R"], d["M"], d["q"], d["r"],
                         d["x0"], d["x"], d["u"], d["lam"], d["K"], d["k"], d["P"], d["p"],
                         variant=L.RICCATI_LEVEL)

    if args.calib_copy:
        # plain copy of known size, for scaling rocprofv3 FETCH/WRITE counters
        nbytes = 512 * 2 ** 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    st, bad = L.bmpc_lqr_check(plan)
    if st != 0:
        raise RuntimeError(f"LQR solve failed (status {st}, node {bad})")

    # the backward kernel this plan dispatches (one untimed solve, every
    # kernel named)
    L.bmpc_profile_enable(True)
    step(0)
    torch.cuda.synchronize()
    bwd_name = next(k for k in L.bmpc_profile_read() if k.startswith("lqr_backward"))
    L.bmpc_profile_enable(False)
    # timed region: HIP event pairs around the backward kernel only (the
    # kernel the roofline is quoted for), recorded on its launch stream
    L.bmpc_profile_only(bwd_name)
    L.bmpc_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        step(i)
    ev1.record()
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    prof = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    L.bmpc_profile_only(None)

    # untimed passes, reported beside `value`: every kernel timed, and no
    # event pairs at all
    L.bmpc_profile_enable(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    prof_all = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        step(i)
    ev1.record()
    torch.cuda.synchronize()
    clean_ms = ev0.elapsed_time(ev1)

    alg = lqr_algorithmic(par, nx, nu)
    bwd_ms, bwd_n = prof.get(bwd_name, (float("nan"), 1))
    fwd_ms, fwd_n = prof_all.get("lqr_forward_paths", (float("nan"), 1))
    bwd_avg_s = bwd_ms / bwd_n / 1e3
    fwd_avg_s = fwd_ms / fwd_n / 1e3
    srcs = ["paper_2506_13624_amd/csrc/lqr.hip", "paper_2506_13624_amd/csrc/lqr_device.hpp",
            "paper_2506_13624_amd/csrc/cvf_device.hpp"]
    bwd_reads, solve_bytes = lqr_solve_algorithmic_bytes(par, nx, nu)
    achieved = bwd_reads / bwd_avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(bwd_name, srcs),
                "kernel": bwd_name, "avg_launch_us": round(bwd_avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": bwd_reads,
                "bytes_with_stored_gains_per_launch": alg["bwd_bytes"],
                "frac_with_stored_gains": round(alg["bwd_bytes"] / bwd_avg_s / 1e9 / HBM_PEAK_GBS, 5),
                "fp64_tflops": round(alg["bwd_flops"] / bwd_avg_s / 1e12, 4),
                "fp64_frac": round(alg["bwd_flops"] / bwd_avg_s / 1e12 / FP64_PEAK_TFLOPS, 5)}
    kernels = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]} for k, v in prof_all.items()}
    ms_step = elapsed_ms / args.steps

    dependency_floor = critical_path_floor(torch, L, par, nx, nu, layout, bwd_name, bwd_avg_s * 1e6,
                                           args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": round(N / (ms_step / 1e3), 1),
        "unit": "tree-Riccati nodes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tree-Riccati microbenchmark: nx=12, nu=4, horizon 40, binary "
                               "branching every 4 stages, 1024 scenarios, 8185 nodes, FP64",
                   "num_nodes": N, "nx": nx, "nu": nu, "instances_rotated": n_inst,
                   "riccati_variant": "level", "layout": "node-major"},
        "ms_per_step_without_event_pairs": round(clean_ms / args.steps, 5),
        "kernels": kernels,
        "forward_GBps": round(alg["fwd_bytes"] / fwd_avg_s / 1e9, 2),
        "solve_algorithmic_bytes": solve_bytes,
        "solve_GBps": round(solve_bytes / (ms_step * 1e-3) / 1e9, 2),
        "roofline": roofline,
        "dependency_floor": dependency_floor,
    }
    L.bmpc_lqr_plan_destroy(plan)

    # Independent solves on several streams at once (reported beside
    # `value`, which is the one-solve-at-a-time rate): one solve of this tree
    # is bound by its dependency depth and leaves most of the GPU idle.
    conc = {}
    for n_str in (() if args.no_concurrent else (2, 4, 8)):
        plans = [L.bmpc_lqr_plan_create(tree, nx, nu, layout) for _ in range(n_str)]
        streams = [torch.cuda.Stream() for _ in range(n_str)]
        # each stream has its own output arrays
        outs = [[empty((N, nx)), empty((N, nu)), empty((N, nx)), empty((N, nu, nx)), empty((N, nu)),
                 empty((N, nx, nx)), empty((N, nx))] for _ in range(n_str)]

        def cstep(i):
            k = i % n_str
            d = dev[i % n_inst]
            L.bmpc_lqr_solve(plans[k], d["A"], d["B"], d["c"], d["Q"], d["R"], d["M"], d["q"], d["r"],
                             d["x0"], *outs[k], variant=L.RICCATI_LEVEL, stream=streams[k])
        for i in range(args.warmup):
            cstep(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            cstep(i)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        for k in range(n_str):
            st, bad = L.bmpc_lqr_check(plans[k], stream=streams[k])
            if st != 0:
                raise RuntimeError(f"concurrent LQR solve failed (status {st}, node {bad})")
            L.bmpc_lqr_plan_destroy(plans[k])
        conc[f"{n_str}_streams"] = {"solves": args.steps, "seconds": round(el, 5),
                                    "nodes_per_s": round(N * args.steps / el, 1),
                                    "backward_bytes_GBps": round(alg["bwd_bytes"] * args.steps / el / 1e9, 2)}
    if conc:
        out["concurrent_independent_solves"] = conc

    # The same solves from host arrays (bmpc_lqr_solve_host: pinned staging,
    # one transfer each way, blocking): the PCIe-inclusive rate, reported
    # beside `value`, which has its inputs resident in HBM.
    if not args.no_concurrent:
        hplan = L.bmpc_lqr_plan_create(tree, nx, nu, layout)
        host = [[d[k].cpu().numpy() for k in "ABcQRMqr"] + [d["x0"].cpu().numpy()] for d in dev]
        for i in range(max(1, args.warmup)):
            L.bmpc_lqr_solve_host(hplan, *host[i % n_inst], variant=L.RICCATI_LEVEL)
        n_host = max(5, args.steps // 2)
        t0 = time.perf_counter()
        for i in range(n_host):
            L.bmpc_lqr_solve_host(hplan, *host[i % n_inst], variant=L.RICCATI_LEVEL)
        el = time.perf_counter() - t0
        st, bad = L.bmpc_lqr_check(hplan)
        if st != 0:
            raise RuntimeError(f"host-array LQR solve failed (status {st}, node {bad})")
        L.bmpc_lqr_plan_destroy(hplan)
        in_bytes = 8 * sum(a.size for a in host[0])
        out["host_arrays_pcie_inclusive"] = {
            "solves": n_host, "ms_per_solve": round(el / n_host * 1e3, 4),
            "nodes_per_s": round(N * n_host / el, 1),
            "bytes_in": in_bytes, "bytes_out": 8 * N * (2 * nx + nu)}
    L.bmpc_tree_destroy(tree)
    return out, insts[0]


def _oracle_batch_solve(args):
    import bmpc_synth as S
    import oracle
    i = args
    inst = _BATCH_CACHE[i]
    t0 = time.perf_counter()
    _, st, _ = oracle.solve(oracle.problem_from_instance(inst))
    return st["status"], st["inner_it"], time.perf_counter() - t0


_BATCH_CACHE = None


def cpu_baseline_bmpc(insts, budget_s=10.0):
    """Oracle solves of the batched workload spread over the host cores (one
    instance per process), for about budget_s seconds."""
    global _BATCH_CACHE
    import multiprocessing as mp
    import oracle
    oracle.use_native_build()
    _BATCH_CACHE = insts
    cores = baseline_cores()
    ctx = mp.get_context("fork")
    done = 0
    conv = 0
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        idx = 0
        while time.perf_counter() - t0 < budget_s and idx < len(insts):
            chunk = list(range(idx, min(len(insts), idx + cores)))
            idx += len(chunk)
            for stt, it, dt in pool.map(_oracle_batch_solve, chunk):
                done += 1
                conv += stt == 0
    el = time.perf_counter() - t0
    return {"value": conv / el, "unit": "BMPC solves/s (KKT <= 1e-6)", "cores": cores, "kind": "oracle",
            "build": "gcc -O3 -march=native", "host": host_info(),
            "sample": f"{done} cold oracle solves of the first {done} batched instances "
                      f"({conv} converged) in {el:.1f} s, one instance per process on {cores} cores"}


def phase_us_per_iteration(stats):
    """Device time per inner iteration of each solver phase (from the
    solver's own phase clock), summed over the given solves."""
    its = max(1, sum(x["inner_it"] for x in stats))
    return {k: round(sum(x["time_ms"][k] for x in stats) * 1e3 / its, 2) for k in stats[0]["time_ms"]}


def slowest(stats, insts):
    i = int(np.argmax([x["inner_it"] for x in stats]))
    return {"instance": i, "nodes": int(insts[i].num_nodes), "inner_it": int(stats[i]["inner_it"]),
            "status": int(stats[i]["status"]), "phase_us_per_iteration": phase_us_per_iteration([stats[i]])}


def not_converged(stats):
    out = {}
    for x in stats:
        if x["status"] != 0:
            out[str(x["status"])] = out.get(str(x["status"]), 0) + 1
    return out


def run_bmpc(args, torch, L):
    import bmpc_synth as S
    from paper_2506_13624_amd.bicycle import Problem

    out = {}
    st = L.bmpc_settings_default()
    # single branch-MPC problem (53 nodes): solve latency
    single = [Problem(S.single_bmpc(i)) for i in range(8)]
    b1 = [L.bmpc_batch_create([p.handle]) for p in single]
    for b in b1:
        L.bmpc_batch_launch(b, st)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    ev0.record()
    for _ in range(reps):
        for b in b1:
            L.bmpc_batch_launch(b, st)
    ev1.record()
    torch.cuda.synchronize()
    ms_single = ev0.elapsed_time(ev1) / (reps * len(b1))
    st1 = [L.bmpc_batch_stats(b, 1)[0] for b in b1]
    # the same solves with the exact Hessian and eigenvalue modification
    st_ex = L.bmpc_settings_default(hessian=L.HESSIAN_EXACT)
    for b in b1:
        L.bmpc_batch_launch(b, st_ex)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        for b in b1:
            L.bmpc_batch_launch(b, st_ex)
    ev1.record()
    torch.cuda.synchronize()
    ms_single_ex = ev0.elapsed_time(ev1) / (reps * len(b1))
    st1_ex = [L.bmpc_batch_stats(b, 1)[0] for b in b1]
    out["bmpc_single"] = {
        "workload": "single branch-MPC tree: bicycle, horizon 20, trunk 5 stages then 3 branches, "
                    "53 nodes, seeds 0-7, cold start",
        "ms_per_solve": round(ms_single, 4), "solves_per_s": round(1e3 / ms_single, 1),
        "converged": sum(s["status"] == 0 for s in st1), "of": len(st1),
        "mean_inner_it": float(np.mean([s["inner_it"] for s in st1])),
        "phase_us_per_iteration": phase_us_per_iteration(st1),
        "exact_hessian": {"ms_per_solve": round(ms_single_ex, 4), "solves_per_s": round(1e3 / ms_single_ex, 1),
                          "converged": sum(s["status"] == 0 for s in st1_ex), "of": len(st1_ex),
                          "mean_inner_it": float(np.mean([s["inner_it"] for s in st1_ex])),
                          "phase_us_per_iteration": phase_us_per_iteration(st1_ex)}}
    for b in b1:
        L.bmpc_batch_destroy(b)
    for p in single:
        p.close()

    # batched: 512 instances of uneven size in one launch
    insts = S.batched_instances(512)
    pbs = [Problem(i) for i in insts]
    b = L.bmpc_batch_create([p.handle for p in pbs])
    L.bmpc_batch_launch(b, st)  # warm-up (also compiles nothing; first launch)
    torch.cuda.synchronize()
    L.bmpc_profile_enable(True)
    ev0.record()
    L.bmpc_batch_launch(b, st)
    ev1.record()
    torch.cuda.synchronize()
    ms_cold = ev0.elapsed_time(ev1)
    s_cold = L.bmpc_batch_stats(b, len(insts))
    # the same cold batch with the log-depth (segment-scan) backward pass
    st_seg = L.bmpc_settings_default(riccati_variant=L.RICCATI_SEGSCAN)
    ev0.record()
    L.bmpc_batch_launch(b, st_seg)
    ev1.record()
    torch.cuda.synchronize()
    ms_cold_seg = ev0.elapsed_time(ev1)
    s_cold_seg = L.bmpc_batch_stats(b, len(insts))
    # autotuner: every (backward variant, threads per problem) pair timed on this batch
    progress("autotuning the batched solver")
    tv, tb, cand = L.bmpc_batch_tune(b, st, warm=0, reps=1)
    ev0.record()
    L.bmpc_batch_launch(b, st)  # AUTO: the tuned pair
    ev1.record()
    torch.cuda.synchronize()
    ms_tuned = ev0.elapsed_time(ev1)
    s_tuned = L.bmpc_batch_stats(b, len(insts))
    # the same tuned cold launch captured once into a HIP graph and replayed
    # (a cold start reads only the problem data, so every replay repeats the
    # eager launch's solves: same statuses and iteration counts)
    gs = torch.cuda.Stream()
    L.bmpc_graph_begin(gs)
    L.bmpc_batch_launch(b, st, warm=0, stream=gs)
    cold_graph = L.bmpc_graph_end(gs)
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    cold_graph_ms, cold_graph_same = [], []
    for _ in range(3):
        g0.record(gs)
        L.bmpc_graph_launch(cold_graph, gs)
        g1.record(gs)
        ss = L.bmpc_batch_stats(b, len(insts), stream=gs)
        cold_graph_ms.append(g0.elapsed_time(g1))
        cold_graph_same.append(all(x["status"] == y["status"] and x["inner_it"] == y["inner_it"]
                                   for x, y in zip(ss, s_tuned)))
    L.bmpc_graph_destroy(cold_graph)
    s_cold_graph = ss
    # the same with a cap of 200 inner iterations per problem
    st_cap = L.bmpc_settings_default(max_iter_total=200)
    ev0.record()
    L.bmpc_batch_launch(b, st_cap)
    ev1.record()
    torch.cuda.synchronize()
    ms_cap = ev0.elapsed_time(ev1)
    s_cap = L.bmpc_batch_stats(b, len(insts))
    # cold, exact Hessian with eigenvalue modification (tuned pair)
    ev0.record()
    L.bmpc_batch_launch(b, st_ex)
    ev1.record()
    torch.cuda.synchronize()
    ms_ex = ev0.elapsed_time(ev1)
    s_ex = L.bmpc_batch_stats(b, len(insts))
    # receding-horizon step, then warm and cold solves of the same shifted problems
    L.bmpc_batch_launch(b, st)  # back to the solution at t
    torch.cuda.synchronize()
    L.bmpc_batch_shift(b)
    ev0.record()
    L.bmpc_batch_launch(b, st, warm=7)
    ev1.record()
    torch.cuda.synchronize()
    ms_warm = ev0.elapsed_time(ev1)
    s_warm = L.bmpc_batch_stats(b, len(insts))
    ev0.record()
    L.bmpc_batch_launch(b, st, warm=0)
    ev1.record()
    torch.cuda.synchronize()
    ms_cold2 = ev0.elapsed_time(ev1)
    s_cold2 = L.bmpc_batch_stats(b, len(insts))
    # closed loop: [shift, warm solve] captured once in a HIP graph, replayed
    L.bmpc_batch_launch(b, st, warm=7)  # solution of the shifted problems
    torch.cuda.synchronize()
    L.bmpc_graph_begin(gs)
    L.bmpc_batch_shift(b, stream=gs)
    L.bmpc_batch_launch(b, st, warm=7, stream=gs)
    graph = L.bmpc_graph_end(gs)
    loop_ms, loop_conv = [], []
    for _ in range(5):
        g0.record(gs)
        L.bmpc_graph_launch(graph, gs)
        g1.record(gs)
        ss = L.bmpc_batch_stats(b, len(insts), stream=gs)
        loop_ms.append(g0.elapsed_time(g1))
        loop_conv.append(int(sum(x["status"] == 0 for x in ss)))
    L.bmpc_graph_destroy(graph)
    prof = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    nodes = sum(i.num_nodes for i in insts)

    def conv(ss):
        return int(sum(x["status"] == 0 for x in ss))

    def mean_it(ss):
        v = [x["inner_it"] for x in ss if x["status"] == 0]
        return float(np.mean(v)) if v else None

    out["bmpc_batched"] = {
        "workload": "512 bicycle branch-MPC instances in one launch: branches U{2..8} at stage U{0..5}, "
                    f"horizon U{{20..60}}, {nodes} nodes in total",
        "cold": {"ms": round(ms_cold, 3), "converged": conv(s_cold), "mean_inner_it": mean_it(s_cold),
                 "solves_per_s": round(conv(s_cold) / (ms_cold / 1e3), 1)},
        "cold_segment_scan": {"ms": round(ms_cold_seg, 3), "converged": conv(s_cold_seg),
                              "mean_inner_it": mean_it(s_cold_seg),
                              "solves_per_s": round(conv(s_cold_seg) / (ms_cold_seg / 1e3), 1)},
        "shifted_warm": {"ms": round(ms_warm, 3), "converged": conv(s_warm), "mean_inner_it": mean_it(s_warm),
                         "solves_per_s": round(conv(s_warm) / (ms_warm / 1e3), 1)},
        "cold_same_shifted_problems": {"ms": round(ms_cold2, 3), "converged": conv(s_cold2),
                                       "mean_inner_it": mean_it(s_cold2),
                                       "solves_per_s": round(conv(s_cold2) / (ms_cold2 / 1e3), 1)},
        "autotuner": {"chosen": {"variant": "segment_scan" if tv == L.RICCATI_SEGSCAN else "level",
                                 "threads_per_problem": tb},
                      "criterion": "launch time per inner iteration summed over the batch",
                      "candidates_us_per_iteration": {
                          f"{'segment_scan' if v == L.RICCATI_SEGSCAN else 'level'}/{blk}": round(t * 1e3, 3)
                          for (v, blk), t in cand.items()}},
        "cold_tuned": {"ms": round(ms_tuned, 3), "converged": conv(s_tuned), "mean_inner_it": mean_it(s_tuned),
                       "solves_per_s": round(conv(s_tuned) / (ms_tuned / 1e3), 1),
                       # the launch ends with its longest-running problem
                       "most_iterations": slowest(s_tuned, insts),
                       "not_converged_by_status": not_converged(s_tuned)},
        "cold_tuned_graph_replay": {"captured": "tuned cold launch", "replays": len(cold_graph_ms),
                                    "ms_per_replay": [round(v, 3) for v in cold_graph_ms],
                                    "converged": conv(s_cold_graph),
                                    "solves_per_s": round(conv(s_cold_graph) / (min(cold_graph_ms) / 1e3), 1),
                                    "same_statuses_and_iterations_as_eager": all(cold_graph_same)},
        "cold_tuned_cap_200_iterations": {"ms": round(ms_cap, 3), "converged": conv(s_cap),
                                          "mean_inner_it": mean_it(s_cap),
                                          "solves_per_s": round(conv(s_cap) / (ms_cap / 1e3), 1)},
        "cold_tuned_exact_hessian": {"ms": round(ms_ex, 3), "converged": conv(s_ex), "mean_inner_it": mean_it(s_ex),
                                     "solves_per_s": round(conv(s_ex) / (ms_ex / 1e3), 1),
                                     "most_iterations": slowest(s_ex, insts),
                                     "not_converged_by_status": not_converged(s_ex),
                                     "phase_us_per_iteration": phase_us_per_iteration(s_ex)},
        "closed_loop_graph_replay": {"captured": "shift + shifted-warm solve", "steps": len(loop_ms),
                                     "ms_per_step": [round(v, 3) for v in loop_ms], "converged": loop_conv},
        "kernels": {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]} for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        out["bmpc_batched"]["cpu_baseline"] = cpu_baseline_bmpc(insts, args.cpu_budget)
    L.bmpc_batch_destroy(b)
    for p in pbs:
        p.close()
    return out


def mlp_flops_per_sample(widths):
    """Dense multiply-adds x 2 of one training sample: forward Z = A W, weight
    gradient A^T dZ and input gradient dZ W^T (not for the first layer)."""
    fwd = sum(widths[l] * widths[l + 1] for l in range(len(widths) - 1))
    dinp = sum(widths[l] * widths[l + 1] for l in range(1, len(widths) - 1))
    return 2 * fwd, 2 * (2 * fwd + dinp)


def run_warmstart(args, torch, L):
    import bmpc_synth as S
    from paper_2506_13624_amd import warmstart as W
    from paper_2506_13624_amd.bicycle import ProblemPool

    out = {}
    n_train, n_val, n_test = args.ws_train, 1024, args.ws_test
    t0 = time.perf_counter()
    gen_settings = L.bmpc_settings_default(max_iter_total=300)
    Xtr, Ttr, oktr, ittr = W.generate((S.learned_topology_instance(i) for i in range(n_train)), pool_size=2048,
                                      settings=gen_settings,
                                      progress=lambda d, n: progress(f"generated {d}/{n}") if d % 16384 == 0 else None)
    gen_s = time.perf_counter() - t0
    Xva, Tva, okva, _ = W.generate((S.learned_topology_instance(500_000 + i) for i in range(n_val)),
                                   settings=gen_settings)
    starter = W.WarmStarter(Ttr.shape[1], max_batch=1024, seed=0)
    log, train_s, rate = starter.fit(Xtr[oktr], Ttr[oktr], steps=args.ws_steps, batch=1024, lr=2e-3,
                                     log_every=max(args.ws_steps // 8, 1))
    progress(f"trained {args.ws_steps} steps")
    val_loss = starter.loss(Xva[okva], Tva[okva])
    # per-kernel times of training steps (event pairs around every launch)
    xb = torch.from_numpy(((Xtr[:1024] - starter.x_mean) / starter.x_std).astype(np.float32)).cuda()
    tb = torch.from_numpy(((Ttr[:1024] - starter.t_mean) / starter.t_std).astype(np.float32)).cuda()
    prof_steps = 200
    L.bmpc_profile_enable(True)
    for _ in range(prof_steps):
        L.bmpc_mlp_train_step(starter.train_net, xb, tb, 1e-6, want_loss=False)
    prof = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    fwd_f, train_f = mlp_flops_per_sample(starter.widths)
    gemm_ms = sum(v[0] for k, v in prof.items() if k.startswith("mlp_gemm"))
    step_flops = train_f * 1024
    gemm_tflops = step_flops * prof_steps / (gemm_ms / 1e3) / 1e12 if gemm_ms > 0 else None

    test = [S.learned_topology_instance(1_000_000 + i) for i in range(n_test)]
    pool = ProblemPool(test[0].parent, n_test, first_inst=test[0])
    st = L.bmpc_settings_default(max_iter_total=args.ws_cap)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed_launch(warm):
        torch.cuda.synchronize()
        ev[0].record()
        L.bmpc_batch_launch(pool.batch, st, warm=warm)
        ev[1].record()
        ss = L.bmpc_batch_stats(pool.batch, n_test)
        torch.cuda.synchronize()
        return ss, ev[0].elapsed_time(ev[1])

    def summary(ss, ms, extra=None):
        conv = [x for x in ss if x["status"] == 0]
        d = {"ms": round(ms, 3), "converged": len(conv), "of": len(ss),
             "mean_inner_it": round(float(np.mean([x["inner_it"] for x in conv])), 2) if conv else None,
             "total_inner_it": int(sum(x["inner_it"] for x in ss)),
             "solves_per_s": round(len(conv) / (ms / 1e3), 1)}
        if extra:
            d.update(extra)
        return d

    progress("learned warm start: evaluation")
    pool.load(test)
    L.bmpc_batch_launch(pool.batch, st)  # warm-up
    s_cold, ms_cold = timed_launch(0)
    feats = np.array([W.features(i) for i in test])
    s_net, t_net = W.solve_with_network(pool, None, starter, st, feats=feats)
    s_netu, t_netu = W.solve_with_network(pool, None, starter, st, guarded=False, feats=feats)
    s_neto, t_neto = W.solve_with_network(pool, None, starter, st, guarded=False, feats=feats,
                                          with_multipliers=False)
    # one receding-horizon step: shifted warm start vs cold vs network on the
    # same shifted problems
    L.bmpc_batch_launch(pool.batch, st)
    L.bmpc_batch_shift(pool.batch)
    torch.cuda.synchronize()
    F_shift = W.shifted_features(pool, test)
    s_shift, ms_shift = timed_launch(7)
    s_cold2, ms_cold2 = timed_launch(0)
    s_net2, t_net2 = W.solve_with_network(pool, test, starter, st, feats=F_shift)
    s_net2u, t_net2u = W.solve_with_network(pool, test, starter, st, guarded=False, feats=F_shift)
    pool.close()
    starter.close()

    def net_summary(ss, t):
        return summary(ss, t["network_ms"] + t["solve_ms"],
                       {"network_ms": round(t["network_ms"], 4), "network_start_kept": int(sum(x["start"] for x in ss))})

    out["learned_warm_start"] = {
        "workload": f"bicycle branch-MPC, horizon 30, 4 branches at stage 4 (109 nodes); network 44-256-256-256-734 "
                    f"GELU, BF16 weights/activations, FP32 accumulate; trained on {int(oktr.sum())} converged cold "
                    f"solves of {n_train} seeded instances, validated on {int(okva.sum())}, tested on {n_test}",
        "data_generation": {"instances": n_train, "converged": int(oktr.sum()), "seconds": round(gen_s, 2),
                            "iteration_cap": 300,
                            "mean_inner_it": round(float(ittr[oktr].mean()), 2)},
        "training": {"steps": args.ws_steps, "batch": 1024, "samples_per_s": round(rate, 0),
                     "loss_log": [(int(a), round(float(b), 5)) for a, b in log],
                     "validation_loss": round(float(val_loss), 5),
                     "kernels": {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]} for k, v in prof.items()},
                     "mfma_bf16": {"flops_per_step": step_flops, "gemm_tflops": round(gemm_tflops, 3) if gemm_tflops else None,
                                   "peak_tflops": 2500.0,
                                   "frac": round(gemm_tflops / 2500.0, 5) if gemm_tflops else None}},
        "evaluation": f"{n_test} test problems per launch (persistent queue), at most {args.ws_cap} inner "
                      "iterations per problem; solves/s counts converged problems over the launch time "
                      "(network inference included for network starts)",
        "fresh_problems": {"cold": summary(s_cold, ms_cold), "network_guarded": net_summary(s_net, t_net),
                           "network_unguarded": net_summary(s_netu, t_netu),
                           "network_inputs_only": net_summary(s_neto, t_neto)},
        "after_one_shift": {"shifted_warm": summary(s_shift, ms_shift), "cold": summary(s_cold2, ms_cold2),
                            "network_guarded": net_summary(s_net2, t_net2),
                            "network_unguarded": net_summary(s_net2u, t_net2u)},
    }
    return out


def run_solver_profile(args, torch, L):
    """Only the branch-MPC solver on one workload, for per-kernel profiles:
    'single' = the 53-node tree, seeds 0-7, each solved args.steps times;
    'batched' = the 512-instance batch with a cap of 200 inner iterations
    per problem, args.steps launches."""
    import bmpc_synth as S
    from paper_2506_13624_amd.bicycle import Problem
    if args.only_solver == "single":
        insts = [S.single_bmpc(i) for i in range(8)]
        st = L.bmpc_settings_default()
        pbs = [Problem(i) for i in insts]
        bs = [L.bmpc_batch_create([p.handle]) for p in pbs]
    else:
        insts = S.batched_instances(512)
        st = L.bmpc_settings_default(max_iter_total=200)
        pbs = [Problem(i) for i in insts]
        bs = [L.bmpc_batch_create([p.handle for p in pbs])]
    for b in bs:
        L.bmpc_batch_launch(b, st)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        for b in bs:
            L.bmpc_batch_launch(b, st)
    ev1.record()
    torch.cuda.synchronize()
    stats = [x for b in bs for x in L.bmpc_batch_stats(b, 1 if len(bs) > 1 else len(insts))]
    out = {"workload": args.only_solver, "launches": args.steps * len(bs),
           "ms_per_launch": round(ev0.elapsed_time(ev1) / (args.steps * len(bs)), 4),
           "converged": int(sum(x["status"] == 0 for x in stats)), "of": len(stats),
           "inner_it": int(sum(x["inner_it"] for x in stats)),
           "phase_us_per_iteration": phase_us_per_iteration(stats)}
    for b in bs:
        L.bmpc_batch_destroy(b)
    for p in pbs:
        p.close()
    return {"solver_profile": out}


def run_mass_spring(args, torch, L):
    """Tree LQR of the mass-spring chain (15 masses: nx = 30, nu = 14), two
    sampled spring constants, robust horizon 10 (1,024 scenarios), horizon
    40: 32,767 nodes, FP64, node-major, inputs resident in HBM."""
    import bmpc_synth as S
    from paper_2506_13624_amd.layout import empty, to_device
    inst = S.mass_spring_tree()
    par = inst.parent
    N = len(par)
    nx, nu = inst.nx, inst.nu
    tree = L.bmpc_tree_create(par)
    plan = L.bmpc_lqr_plan_create(tree, nx, nu, L.LAYOUT_NODE_MAJOR)
    d = {k: to_device(getattr(inst, k), L.LAYOUT_NODE_MAJOR) for k in "ABcQRMqr"}
    x0 = to_device(inst.x0, L.LAYOUT_NODE_MAJOR)
    outs = [empty((N, nx)), empty((N, nu)), empty((N, nx)), empty((N, nu, nx)), empty((N, nu)), empty((N, nx, nx)),
            empty((N, nx))]

    def step():
        L.bmpc_lqr_solve(plan, d["A"], d["B"], d["c"], d["Q"], d["R"], d["M"], d["q"], d["r"], x0, *outs)
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    st, bad = L.bmpc_lqr_check(plan)
    if st != 0:
        raise RuntimeError(f"mass-spring LQR failed (status {st}, node {bad})")
    steps = max(20, args.steps // 10)
    L.bmpc_profile_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    prof = L.bmpc_profile_read()
    L.bmpc_profile_enable(False)
    ms = ev0.elapsed_time(ev1) / steps
    L.bmpc_lqr_plan_destroy(plan)
    L.bmpc_tree_destroy(tree)
    kern = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]} for k, v in prof.items()}
    bwd_us = kern["lqr_backward_level_mfma"]["avg_us"]
    reads, solve_bytes = lqr_solve_algorithmic_bytes(par, nx, nu)
    alg = lqr_algorithmic(par, nx, nu)
    tflops = alg["bwd_flops"] / (bwd_us * 1e-6) / 1e12
    return {"mass_spring_tree": {
        "workload": "mass-spring chain tree LQR: 15 masses (nx=30, nu=14), 2 sampled spring constants, robust "
                    f"horizon 10 (1024 scenarios), horizon 40, {N} nodes, FP64",
        "ms_per_solve": round(ms, 4), "nodes_per_s": round(N / (ms * 1e-3), 1), "kernels": kern,
        "backward_algorithmic_bytes": reads, "backward_flops": alg["bwd_flops"],
        "backward_GBps": round(reads / (bwd_us * 1e-6) / 1e9, 2),
        "backward_fp64_tflops": round(tflops, 3),
        "roofline_backward": {"bound": "mfma", "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(tflops / FP64_PEAK_TFLOPS, 5),
                              "hbm_frac": round(reads / (bwd_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5),
                              "traffic": measured_traffic("lqr_backward_level_mfma_mass_spring",
                                                          ["paper_2506_13624_amd/csrc/lqr.hip",
                                                           "paper_2506_13624_amd/csrc/lqr_device.hpp",
                                                           "paper_2506_13624_amd/csrc/cvf_device.hpp"])},
    }}


def run_large_tree(args, torch, L):
    """Tree LQR on the 4096-scenario bicycle tree (122,871 nodes): the Gauss-
    Newton LQR subproblem at the cold start, level-parallel vs segment-scan
    backward; plus the time per AL inner iteration of the whole-grid solver
    on this tree, with its measured HBM traffic per iteration when the
    committed counter summary matches the solver sources."""
    import bmpc_synth as S
    from paper_2506_13624_amd.bicycle import Problem

    inst = S.large_tree(0)
    par = inst.parent
    N = len(par)
    pb = Problem(inst)
    st0 = L.bmpc_settings_default(max_outer=0)
    x = torch.zeros(N * 4, dtype=torch.float64, device="cuda")
    u = torch.zeros(N * 2, dtype=torch.float64, device="cuda")
    lam = torch.zeros(N * 4, dtype=torch.float64, device="cuda")
    ye = torch.zeros(N * 5, dtype=torch.float64, device="cuda")
    L.bmpc_solve(pb.handle, st0, 0, x, u, lam, ye)  # cold start only (rollout + adjoint)
    A, B, c, Q, R, q, r = (torch.zeros(N * k, dtype=torch.float64, device="cuda") for k in (16, 8, 4, 16, 4, 4, 2))
    L.bmpc_linearize(pb.handle, x, u, lam, ye, 100.0, A, B, c, Q, R, q, r)
    # the LQR takes the step Jacobians on the edge into each child
    pidx = torch.from_numpy(np.maximum(par, 0).astype(np.int64)).cuda()
    Ae = A.view(N, 16)[pidx].contiguous().view(-1)
    Be = B.view(N, 8)[pidx].contiguous().view(-1)
    M = torch.zeros(N * 8, dtype=torch.float64, device="cuda")
    x0 = torch.zeros(4, dtype=torch.float64, device="cuda")
    tree = L.bmpc_tree_create(par)
    plan = L.bmpc_lqr_plan_create(tree, 4, 2, L.LAYOUT_NODE_MAJOR)
    outs = [torch.empty(N * k, dtype=torch.float64, device="cuda") for k in (4, 2, 4, 8, 2, 16, 4)]
    alg = lqr_algorithmic(par, 4, 2)
    res = {}
    steps = max(20, args.steps // 10)
    for name, variant, kname in (("level", L.RICCATI_LEVEL, "lqr_backward_level"),
                                 ("segment_scan", L.RICCATI_SEGSCAN, "lqr_backward_segscan")):
        def step():
            L.bmpc_lqr_solve(plan, Ae, Be, c, Q, R, M, q, r, x0, *outs, variant=variant)
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        status, bad = L.bmpc_lqr_check(plan)
        L.bmpc_profile_enable(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        prof = L.bmpc_profile_read()
        L.bmpc_profile_enable(False)
        # the backward kernel that ran (its name carries the variant)
        kname = next(k for k in prof if k.startswith(kname))
        bwd_us = prof[kname][0] / prof[kname][1] * 1e3
        tot_us = sum(v[0] for v in prof.values()) / steps * 1e3
        res[name] = {"backward_us": round(bwd_us, 2), "lqr_solve_us": round(tot_us, 2), "status": int(status),
                     "backward_GBps": round(alg["bwd_bytes"] / (bwd_us * 1e-6) / 1e9, 2),
                     "backward_hbm_frac": round(alg["bwd_bytes"] / (bwd_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5),
                     "backward_fp64_TFLOPs": round(alg["bwd_flops"] / (bwd_us * 1e-6) / 1e12, 4),
                     "backward_fp64_frac": round(alg["bwd_flops"] / (bwd_us * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 6),
                     "kernels": {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]}
                                 for k, v in prof.items()}}
    lvl_kernel = next(k for k in res["level"]["kernels"] if k.startswith("lqr_backward_level"))
    res["level"]["dependency_floor"] = critical_path_floor(torch, L, par, 4, 2, L.LAYOUT_NODE_MAJOR, lvl_kernel,
                                                           res["level"]["backward_us"], steps, 5)
    # the same subproblem in FP32, and in mixed precision (FP32 sweeps, FP64
    # residuals, refinement steps added until the FP64 residual floor)
    L.bmpc_lqr_solve(plan, Ae, Be, c, Q, R, M, q, r, x0, *outs, variant=L.RICCATI_LEVEL)
    ref = [o.clone() for o in outs[:3]]
    f32_in = [t.float() for t in (Ae, Be, c, Q, R, M, q, r, x0)]
    f32_out = [o.float() for o in outs]

    def timed(fn, kernels):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        L.bmpc_profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        prof = L.bmpc_profile_read()
        L.bmpc_profile_enable(False)
        return e0.elapsed_time(e1) / steps * 1e3, {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1]}
                                                  for k, v in prof.items() if k in kernels}

    fp32_k = ("lqr_backward_level_quad_f32", "lqr_backward_level_lane_f32", "lqr_forward_paths_f32",
              "lqr_costate_f32")
    us32, k32 = timed(lambda: L.bmpc_lqr_solve_f32(plan, *f32_in, *f32_out), fp32_k)
    rel = lambda a, b: float((a.double() - b).abs().max() / b.abs().max())
    mixed = {"fp32_solve_us": round(us32, 2), "fp32_kernels": k32,
             "fp32_rel_error_x": rel(f32_out[0], ref[0]), "refinement": {}}
    for rs in (1, 2, 3):
        # timed without the residual norms (a diagnostic), which are then
        # read from one more call
        norms = torch.zeros(rs + 2, dtype=torch.float64, device="cuda")
        mo = [torch.zeros_like(o) for o in outs[:3]]
        usm, km = timed(lambda: L.bmpc_lqr_solve_mixed(plan, Ae, Be, c, Q, R, M, q, r, x0, *mo, rs),
                        fp32_k + ("lqr_residual_f64", "lqr_refine_update", "lqr_matrices_to_f32"))
        L.bmpc_lqr_solve_mixed(plan, Ae, Be, c, Q, R, M, q, r, x0, *mo, rs, norms)
        mixed["refinement"][f"{rs}_steps"] = {
            "solve_us": round(usm, 2), "residual_norms": [float(v) for v in norms.cpu()],
            "rel_diff_to_fp64_solve": {k: rel(a, b) for k, a, b in zip(("x", "u", "lam"), mo, ref)},
            "kernels": km}
    res["mixed_precision"] = mixed
    L.bmpc_lqr_plan_destroy(plan)
    L.bmpc_tree_destroy(tree)
    # AL iterations on this tree (a single large problem: the whole grid);
    # the launch that only builds the cold start is timed again here, after
    # the first launch of the kernel above
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev0[0].record()
    L.bmpc_solve(pb.handle, st0, 0, x, u, lam, ye)
    ev0[1].record()
    torch.cuda.synchronize()
    start_ms = ev0[0].elapsed_time(ev0[1])
    st = L.bmpc_settings_default(max_outer=1, max_inner=5)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    s = L.bmpc_solve(pb.handle, st, 0, x, u, lam, ye)
    ev[1].record()
    torch.cuda.synchronize()
    pb.close()
    n_it = max(s["inner_it"], 1)
    ms_all = ev[0].elapsed_time(ev[1])
    # per inner iteration: the launch with five inner iterations less the
    # launch that only builds the cold start
    ms_it = (ms_all - start_ms) / n_it
    al = {"inner_iterations": s["inner_it"], "ms_launch": round(ms_all, 3), "ms_start_only_launch": round(start_ms, 3),
          "ms_per_inner_iteration": round(ms_it, 3), "phase_us_per_iteration": phase_us_per_iteration([s])}
    # measured HBM traffic of the same two launches (rocprofv3 FETCH_SIZE +
    # WRITE_SIZE, profiles/), while the solver sources are unchanged
    tb = measured_traffic("bmpc_solve_grid_5_inner", SOLVER_SRCS)
    t0 = measured_traffic("bmpc_solve_grid_start_only", SOLVER_SRCS)
    if tb is not None and t0 is not None and s["inner_it"] == 5:
        per_it = (tb - t0) / 5
        gbps = per_it / (ms_it * 1e-3) / 1e9
        al.update({"hbm_bytes_per_inner_iteration": round(per_it), "hbm_GBps": round(gbps, 2),
                   "hbm_frac": round(gbps / HBM_PEAK_GBS, 5)})
    return {"large_tree": {
        "workload": "bicycle tree, horizon 80, binary branching every 5 stages to stage 55 (4096 scenarios, "
                    f"{N} nodes, 8191 segments); tree LQR of the Gauss-Newton subproblem at the cold start, nx=4, nu=2",
        "algorithmic_bytes_backward": alg["bwd_bytes"], "flops_backward": alg["bwd_flops"],
        "lqr": res,
        "al_solver_whole_grid": al,
    }}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="launch one 512 MiB copy first (rocprofv3 counter calibration)")
    ap.add_argument("--skip-bmpc", action="store_true")
    ap.add_argument("--skip-warmstart", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the independent solves on several streams (for per-kernel profiles)")
    ap.add_argument("--only-solver", choices=("single", "batched"), default=None,
                    help="only the branch-MPC solver on one workload, printed on its own (for profiles)")
    ap.add_argument("--only-mass-spring", action="store_true",
                    help="only the mass-spring tree LQR, printed on its own (for profiles)")
    ap.add_argument("--only-large", action="store_true",
                    help="only the 4096-scenario tree section, printed on its own (for counter runs)")
    ap.add_argument("--ws-train", type=int, default=200000, help="training instances of the learned warm start")
    ap.add_argument("--ws-steps", type=int, default=3000, help="training steps (batch 1024)")
    ap.add_argument("--ws-test", type=int, default=8192, help="test problems of the learned warm start")
    ap.add_argument("--ws-cap", type=int, default=300, help="inner-iteration cap in the warm-start evaluation")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}))
        sys.exit(1)
    from paper_2506_13624_amd import _lib as L

    if args.only_solver:
        if args.calib_copy:
            nbytes = 512 * 2 ** 20
            src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        progress(f"solver profile: {args.only_solver}")
        print(json.dumps(run_solver_profile(args, torch, L)), flush=True)
        return

    if args.only_mass_spring:
        if args.calib_copy:
            nbytes = 512 * 2 ** 20
            src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        progress("mass-spring tree LQR")
        print(json.dumps(run_mass_spring(args, torch, L)), flush=True)
        return

    if args.only_large:
        if args.calib_copy:
            nbytes = 512 * 2 ** 20
            src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        progress("large tree")
        print(json.dumps(run_large_tree(args, torch, L)), flush=True)
        return

    progress("tree-Riccati microbenchmark")
    out, inst = run_lqr(args, torch, L)
    if not args.skip_bmpc:
        progress("branch-MPC single and batched solves")
        out.update(run_bmpc(args, torch, L))
    if not args.skip_bmpc and not args.skip_warmstart:
        progress("learned warm start")
        out.update(run_warmstart(args, torch, L))
    if not args.skip_bmpc and not args.skip_large:
        progress("large tree")
        out.update(run_large_tree(args, torch, L))
    progress("mass-spring tree LQR")
    out.update(run_mass_spring(args, torch, L))
    if not args.no_cpu_baseline:
        progress("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline_lqr(inst, args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
