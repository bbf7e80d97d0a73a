#!/usr/bin/env python3
"""Benchmark of the FEM hot path on one MI355X.

Default workload (batch512): 512 MaxCut instances of uneven size (N
log-uniform in [1000, 50000], even b random 3-regular, odd b G(n, 5n), +/-1
weights), R = 32 replicas each, linear beta 0.01 -> 5, Adam lr 0.1.  One
"step" is one pass of the whole hot path over the block-diagonal union of all
512 instances in one launch: sparse field product, gradient, Adam, new
bfloat16 marginal copy (float32 fields, accumulation and Adam state),
per-replica energies U, S, F, and the anytime read-out with integer
evaluation every 25 steps.

Metric: replica-edge updates per second = nnz * R * K / seconds over K
steps in one captured HIP graph, inputs resident in HBM (nnz = 2 x edges,
summed over instances).  The same line carries the time to a best cut within
0.1% of plain FEM (per-instance float32 solvers) for batched float32,
batched bfloat16 and batched bfloat16 with the learned warm start, and the
FP64 C oracle timed on the host as a baseline.  Prints one JSON line.

Other workloads (--workload): maxcut1e5 (N = 10^5, 3*10^5 +/-1 edges,
R = 256; --dtype, --gradient manipulated), bmincut1e6 (3-D RGG, N = 10^6,
q = 8, R = 16), max3sat1e5 (N = 10^5, M = 8*10^5, R = 64), er800 (G(800,
19176), R = 16), k2000dense (complete graph K_2000, the dense matrix-core
path, R = 1000), copy (a plain device copy that calibrates the HBM counters).

roofline.achieved is the algorithmic bytes of one step-kernel launch (each
array touched once: h, m1, m2 read and written, the marginal copy read once
and written once, the graph as 4-byte row offsets and 4-byte entries) over
the kernel's average duration from HIP events on the solver's stream.
roofline.traffic is the HBM traffic of one launch measured with the
FETCH_SIZE and WRITE_SIZE counters (scaled by a plain copy of known size),
read from the committed counter summary of the workload; it is null when the
kernel sources, launch shape or marginal type differ from the ones the
counters were taken with.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6
MFMA_I8_PEAK_TOPS = 5000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def step_kernel_bytes(n, R, nnz, mbytes):
    """Algorithmic bytes of one MaxCut step launch: h, m1, m2 read and written
    (24 B per replica-node), the marginal copy read once and written once
    (2 b per replica-node), the graph as 4-byte row offsets and 4-byte entries
    (a column with the sign of a +/-1 weight)."""
    return n * R * (24 + 2 * mbytes) + 4 * (n + 1) + 4 * nnz


def manip_kernel_bytes(n, R, nnz):
    """Algorithmic bytes of one manipulated-gradient MaxCut launch: h, m1, m2
    read and written, the sign bits (ceil(R/32) words per row) read once and
    written once, the graph (4-byte offsets and entries) and the per-node
    normaliser (4 B)."""
    rw = (R + 31) // 32
    return n * R * 24 + 2 * 4 * n * rw + 4 * (n + 1) + 4 * nnz + 4 * n


KERNEL_SOURCES = {
    "explicit": ["fem_kernels.hip", "fem_device.h", "fem_internal.h"],
    "manipulated": ["fem_manip.hip", "fem_device.h", "fem_internal.h"],
    "dense": ["fem_dense.hip", "fem_dense.h", "fem_device.h", "fem_internal.h"],
}


def kernel_sources_sha(gradient):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[gradient]:
        with open(os.path.join(ROOT, "paper_2412_09285_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, gradient, tile, marginals, layout="interleaved"):
    """Bytes per launch from a committed counter summary, or None when the
    summary is missing or was taken with other kernel sources / launch shape."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        m = re.search(r"^counters-json: (\{.*\})\s*$", f.read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sources_sha256") != kernel_sources_sha(gradient) or list(rec.get("tile", [])) != list(tile) \
            or rec.get("marginals") != marginals or rec.get("state_layout", "separate") != layout:
        return None
    return int(rec["traffic_bytes_per_launch"])


def _oracle_setup(kind, key, R):
    import oracle as O
    from paper_2412_09285_amd import workloads as W

    if kind == "batch":
        g = W.batch_instance(key)
        h0 = W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"])
        T = 1000
    else:
        g = W.config_graph(key)
        h0 = W.initial_fields(g.n, R, seed=100 + key)
        T = 2000
    return g.nnz * R, O.maxcut_run(g, O.Params(R=R, T=T), h0)


def _oracle_maxcut_task(task):
    """One oracle run (FP64 C, one thread): `steps` steps of an instance;
    (updates, seconds of the run alone)."""
    kind, key, R, steps = task
    upd, run = _oracle_setup(kind, key, R)
    t0 = time.perf_counter()
    run.step(steps)
    return upd * steps, time.perf_counter() - t0


def _oracle_worker(tasks, barrier, results):
    """Builds its oracle runs, waits at the barrier, runs them all, reports."""
    runs = [(_oracle_setup(kind, key, R), steps) for (kind, key, R, steps) in tasks]
    barrier.wait()
    upd = 0
    for (u, run), steps in runs:
        run.step(steps)
        upd += u * steps
    results.put(upd)


def host_threads():
    """Threads the CPU baseline uses: the cores this process may run on,
    at most 16 (one GPU's share of a shared host)."""
    return min(len(os.sched_getaffinity(0)), 16)


def oracle_parallel(tasks, threads):
    """Runs the tasks on `threads` processes (task k on process k mod
    threads); every process builds its inputs first, then all start
    together.  Returns (updates, wall seconds of the runs)."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(threads + 1)
    results = ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(tasks[k::threads], barrier, results)) for k in range(threads)]
    for p in procs:
        p.start()
    barrier.wait()
    t0 = time.perf_counter()
    upd = sum(results.get() for _ in procs)
    wall = time.perf_counter() - t0
    for p in procs:
        p.join()
    return upd, wall


def cpu_baseline_batch(n_inst, R, steps, one_thread_instances):
    """The oracle on the batch: every instance for `steps` steps with one
    process per host thread (all cores), then a sample of instances in one
    thread.  Rate = summed nnz * R * steps / wall time of the runs."""
    import numpy as np

    threads = host_threads()
    upd, wall = oracle_parallel([("batch", b, R, steps) for b in range(n_inst)], threads)
    sample = [int(b) for b in np.random.default_rng(7).permutation(n_inst)[:one_thread_instances]]
    one = [_oracle_maxcut_task(("batch", b, R, steps)) for b in sample]
    upd1, t1 = sum(r[0] for r in one), sum(r[1] for r in one)
    return {
        "value": upd / wall,
        "unit": "replica-edge updates/s",
        "cores": threads,
        "kind": "oracle",
        "nproc": os.cpu_count(),
        "affinity_cores": len(os.sched_getaffinity(0)),
        "sample": f"all {n_inst} instances, R = {R}, the first {steps} steps of each, FP64 C oracle, one process "
                  f"per thread on {threads} threads (instances dealt round-robin): {wall:.1f} s wall",
        "one_thread": {"value": upd1 / t1, "cores": 1,
                       "sample": f"{one_thread_instances} instances (seeded sample), the first {steps} steps, "
                                 f"one thread: {t1:.1f} s"},
    }


def cpu_baseline_graph(cfg, R_sample, steps_sample):
    """The oracle on one graph workload: one process per host thread, each
    running R_sample replicas of it, and one thread alone."""
    threads = host_threads()
    upd1, t1 = _oracle_maxcut_task(("config", cfg, R_sample, steps_sample))
    upd, wall = oracle_parallel([("config", cfg, R_sample, steps_sample)] * threads, threads)
    return {
        "value": upd / wall,
        "unit": "replica-edge updates/s",
        "cores": threads,
        "kind": "oracle",
        "nproc": os.cpu_count(),
        "affinity_cores": len(os.sched_getaffinity(0)),
        "sample": f"same graph, {threads} processes of {R_sample} replicas each, the first {steps_sample} steps, "
                  f"FP64 C oracle: {wall:.1f} s wall",
        "one_thread": {"value": upd1 / t1, "cores": 1,
                       "sample": f"{R_sample} replicas, the first {steps_sample} steps, one thread: {t1:.1f} s"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps K (one anneal of K steps; default: the workload's anneal length)")
    ap.add_argument("--warmup", type=int, default=50, help="untimed warm-up steps W")
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--gradient", choices=["explicit", "manipulated"], default="explicit")
    ap.add_argument("--state-layout", choices=["separate", "interleaved"], default="interleaved",
                    help="device layout of h and the Adam moments (no effect on results)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--retune", action="store_true", help="time every launch shape even if one is cached")
    ap.add_argument("--cpu-replicas", type=int, default=8,
                    help="single-graph workloads: replicas per oracle process in the CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU baseline (default: 10 for batch512, 100 for maxcut1e5)")
    ap.add_argument("--cpu-one-thread", type=int, default=32,
                    help="batch512: instances in the one-thread CPU baseline sample")
    ap.add_argument("--workload", choices=["batch512", "maxcut1e5", "bmincut1e6", "max3sat1e5", "k2000dense", "er800",
                                           "infer512", "copy"],
                    default="batch512",
                    help="batch512 (default): 512 uneven MaxCut instances, R = 32, in one launch per step, with time "
                         "to target; maxcut1e5: N = 10^5, R = 256; bmincut1e6 / max3sat1e5: the Potts and Max-3-SAT "
                         "kernels at full size; er800: a G-set-sized instance (800 nodes, R = 16), launch-bound; "
                         "k2000dense: the dense-W (matrix-core) path on a complete 2000-node graph; "
                         "infer512: the warm-start network's proposal for every replica of the 512-instance batch "
                         "(--steps calls, timed on the device); "
                         "copy: a plain device copy (calibrates HBM counters)")
    ap.add_argument("--order", choices=["draw", "rcm"], default="rcm",
                    help="bmincut1e6: node order of the graph (rcm: relabelled by fem_graph_order before the "
                         "problem is built; draw: as generated)")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--no-ttt", action="store_true", help="batch512: skip the time-to-target runs")
    ap.add_argument("--plain-steps", type=int, default=1000)
    ap.add_argument("--early-steps", type=int, default=100, help="batch512: plain steps before the proposal")
    ap.add_argument("--warm-steps", type=int, default=300, help="batch512: length of the continued anneal")
    ap.add_argument("--beta-start", type=float, default=0.3, help="batch512: beta at the start of the continuation")
    ap.add_argument("--alpha", type=float, default=1.0, help="batch512: scale of the network's proposal")
    ap.add_argument("--eval-every", type=int, default=25)
    ap.add_argument("--params", default=os.path.join(ROOT, "paper_2412_09285_amd", "data", "mpnn_maxcut.bin"))
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicas would shard across GPUs with no per-step communication). "
              f"Requested --gpus {args.gpus} (WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_09285_amd import fem
    from paper_2412_09285_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "copy":
        n = 1 << 28   # 1 GiB of float32
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"workload": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                          "copies": 6, "ms_per_copy": ms, "read_plus_write_GBps": 8 * n / (ms * 1e-3) / 1e9}))
        return
    if args.workload == "batch512":
        batch_headline(args)
        return
    if args.workload == "infer512":
        infer_batch(args)
        return
    throughput(args)


def infer_batch(args):
    """The warm-start network's proposal for all 32 replicas of the
    512-instance union (inputs on the device), queued on one stream; one
    JSON line with the time per call."""
    import numpy as np
    import torch

    from paper_2412_09285_amd import batchbench as BB
    from paper_2412_09285_amd import fem

    b = BB.Batch(BB.instances(args.instances))
    net = fem.MPNN(np.zeros(fem.N_MPNN_PARAMS, dtype=np.float32))
    net.load(args.params)
    stream = torch.cuda.Stream()
    out = torch.empty_like(b.h0)
    K = args.steps if args.steps else 10
    for _ in range(2):
        net.infer(b.union, b.h0, seed=5, alpha=1.0, out=out, stream=stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        net.infer(b.union, b.h0, seed=5, alpha=1.0, out=out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / K
    print(json.dumps({"workload": "infer512", "instances": len(b.graphs), "n": b.n, "nnz": b.nnz, "replicas": b.R,
                      "calls": K, "ms_per_call": ms, "data": "synthetic (the batch512 instances and fields h0)"}))


def batch_headline(args):
    """The default line: throughput of the batched step over the 512-instance
    union, its roofline, the CPU oracle baseline, and the time to target."""
    import torch

    from paper_2412_09285_amd import batchbench as BB
    from paper_2412_09285_amd import fem

    K = args.steps if args.steps else 200
    Wm = args.warmup
    R = BB.R_BATCH
    t0 = time.perf_counter()
    graphs = BB.instances(args.instances)
    b = BB.Batch(graphs, R)
    log(f"{len(graphs)} instances, {b.n} nodes, nnz {b.nnz}, R = {R} ({time.perf_counter() - t0:.1f} s to build)")
    stream = torch.cuda.Stream()
    thr = BB.throughput(b, K, Wm, stream, dtype=fem.BF16, eval_every=args.eval_every, tune=not args.no_tune)
    log(f"timed {K} steps in {thr['seconds'] * 1e3:.1f} ms: {thr['updates_per_s']:.3e} updates/s; step kernel "
        f"{thr['kernel_ms'] * 1e3:.1f} us (launch shape {thr['tile']})")
    alg = step_kernel_bytes(b.n, R, b.nnz, 2)
    achieved = alg / (thr["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(os.path.join(ROOT, "profiles", "maxcut_batch512_R32_bf16_hbm_counters.md"),
                               "explicit", thr["tile"], "bf16")
    out = {
        "metric": "replica-edge updates/s (nnz*R*steps/s) + time to best cut within 0.1% of plain",
        "value": thr["updates_per_s"],
        "unit": "replica-edge updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": thr["seconds"] * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16-marginals",
        "data": "synthetic (seeded generator: 512 MaxCut instances, N log-uniform in [1000, 50000], random "
                "3-regular and G(n, 5n), +/-1 weights)",
        "config": {"workload": "maxcut_batch512_uneven_R32", "instances": len(graphs), "n": b.n, "nnz": b.nnz,
                   "replicas": R, "marginals": "bf16", "energies": "every step", "eval_every": min(args.eval_every, K),
                   "schedule": "linear beta 0.01->5, Adam lr 0.1", "tile": list(thr["tile"]),
                   "parallelism": "single GPU, one launch per step over the block-diagonal union"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "maxcut_step_kernel", "kernel_avg_ms": round(thr["kernel_ms"], 5),
                     "kernel_launches": thr["kernel_launches"], "alg_bytes_per_launch": int(alg),
                     "alg_bytes_model": "28 B per replica-node (h, m1, m2 read and written, bf16 copy read and "
                                        "written) + 4 B per row offset + 4 B per adjacency entry",
                     "kernel_sources_sha256": kernel_sources_sha("explicit")},
        "result": {"U_mean": thr["U_mean"], "anytime_best_cut_sum": thr["best_sum"]},
    }
    if not args.no_ttt:
        log("time to target ...")
        out["time_to_target"] = BB.time_to_target(b, stream, plain_steps=args.plain_steps, K=args.eval_every,
                                                  early_steps=args.early_steps, warm_steps=args.warm_steps,
                                                  beta_start=args.beta_start, alpha=args.alpha, params=args.params)
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline_batch(args.instances, R, args.cpu_steps or 10, args.cpu_one_thread)
    print(json.dumps(out), flush=True)


# The single-GPU throughput workloads: the default line (MaxCut, N = 10^5,
# R = 256) and the Potts / Max-3-SAT kernels at their full workload sizes.
WORKLOADS = {
    "maxcut1e5": dict(kind="maxcut", recipe=2, R=256, seed=102, T=2000,
                      name="maxcut_sparse_n100000_e300000_pm1", counters="maxcut_n1e5_R256",
                      data="random sparse graph, uniform endpoints, +/-1 weights"),
    "bmincut1e6": dict(kind="bmincut", recipe=3, R=16, q=8, lam=1.0, seed=103, T=3000,
                       name="bmincut_rgg3d_n1000000_deg14_q8", counters="bmincut_rgg1e6_q8_R16",
                       data="3-D random geometric graph, mean degree 14, unit weights"),
    "max3sat1e5": dict(kind="maxsat", recipe=4, R=64, seed=104, T=2000,
                       name="max3sat_n100000_m800000", counters="max3sat_1e5_R64",
                       data="random 3-SAT, distinct variables, fair signs, ratio 8"),
    "er800": dict(kind="maxcut", recipe=1, R=16, seed=101, T=500,
                  name="maxcut_er_n800_e19176", counters="maxcut_er800_R16",
                  data="Erdos-Renyi G(800, 19176), unit weights"),
    "k2000dense": dict(kind="maxcut_dense", n=2000, R=1000, seed=105, T=1000,
                       name="maxcut_complete_n2000_pm1_dense", counters="maxcut_dense_k2000_R1000",
                       data="complete graph K_2000, +/-1 weights"),
}

# the paper's K2000 optimiser: RMSprop (alpha 0.56, momentum 0.63, weight
# decay 0.013, lr 0.03), inverse-proportional schedule T 1.16 -> 6e-5
K2000_PARAMS = dict(optimizer=1, rms_alpha=0.56, momentum=0.63, weight_decay=0.013, lr=0.03, schedule=2,
                    beta_min=1 / 1.16, beta_max=1 / 6e-5)


def dense_kernel_bytes(n, R, w_bytes):
    """Algorithmic bytes of one dense step launch: W once (w_bytes per entry:
    4 float, 1 int8), the marginal copy read and written (4 B per value as
    float or as four int8 digits), h, m1, m2 read and written."""
    return w_bytes * n * n + n * R * (24 + 8)


def potts_kernel_bytes(n, R, q, nnz, mbytes):
    """Algorithmic bytes of one bMinCut launch: h, m1, m2 read and written and
    the marginal copy read once and written once (24 + 2 b per replica-node-
    state) and the graph (4-byte row offsets and entries; unit weights)."""
    return n * R * q * (24 + 2 * mbytes) + 4 * (n + 1) + 4 * nnz


def sat_kernel_bytes(n, R, nnz, mbytes, rec_bytes=8):
    """Algorithmic bytes of one Max-k-SAT launch: h, m1, m2 and the marginal
    copy as for MaxCut, one record per literal incidence (the other two
    literals of a 3-SAT clause, 4 B each) and 4-byte row offsets."""
    return n * R * (24 + 2 * mbytes) + 4 * (n + 1) + rec_bytes * nnz


def throughput(args):
    import numpy as np
    import torch

    from paper_2412_09285_amd import fem
    from paper_2412_09285_amd import workloads as W

    wl = WORKLOADS[args.workload]
    K, Wm = args.steps if args.steps else wl["T"], args.warmup
    R = wl["R"]
    kind = wl["kind"]
    manip = args.gradient == "manipulated"
    if manip and kind != "maxcut":
        raise SystemExit("--gradient manipulated is measured on the MaxCut workload")
    log("generating the workload ...")
    order_s = None
    dense_i8 = False
    if kind == "maxcut_dense":
        g = W.complete_pm1(wl["n"], seed=wl["seed"])
        n, nnz, q = g.n, g.nnz, 1
        Wd = W.dense_matrix(g)
        dense_i8 = bool(np.all(Wd == np.rint(Wd)) and np.abs(Wd).max() <= 127)
        prob = fem.Problem.maxcut_dense(Wd, device=0)
        h0 = W.initial_fields(n, R, seed=wl["seed"])
    elif kind == "maxsat":
        cnf = W.config_cnf(wl["recipe"])
        n, nnz, q = cnf.n_vars, int(cnf.clause_off[-1]), 1
        prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits, device=0)
        h0 = W.initial_fields(n, R, seed=wl["seed"])
    else:
        g = W.config_graph(wl["recipe"])
        n, nnz = g.n, g.nnz
        q = wl.get("q", 1)
        if kind == "bmincut" and args.order == "rcm":
            t_o = time.perf_counter()
            order = fem.graph_order(g.n, g.u, g.v)
            g.u, g.v = fem.relabel(order, g.u, g.v)
            order_s = time.perf_counter() - t_o
            log(f"relabelled in reverse Cuthill-McKee order ({order_s:.1f} s)")
        if kind == "bmincut":
            prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q, device=0)
            h0 = W.initial_fields(n, R, seed=wl["seed"], q=q)
        else:
            prob = fem.Problem.maxcut(g.n, g.u, g.v, g.w, device=0)
            h0 = W.initial_fields(n, R, seed=wl["seed"])
    dtype = fem.BF16 if args.dtype == "bf16" else fem.F32
    stream = torch.cuda.Stream()
    T = max(K, Wm, 1)
    extra = dict(gradient=fem.GRAD_MANIPULATED, energy_every=0) if manip else dict(energy_every=1)
    extra["state_layout"] = fem.STATE_INTERLEAVED if args.state_layout == "interleaved" else fem.STATE_SEPARATE
    if kind == "bmincut":
        extra["lam"] = wl["lam"]
    if kind == "maxcut_dense":
        extra.update(K2000_PARAMS)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, marginal_dtype=dtype, **extra), stream=stream)
    s.set_fields(h0)
    tile = s.tile()
    if not args.no_tune:
        tile = s.tune(trial_steps=10, use_cache=not args.retune)
    log(f"launch shape (vec, waves, rows, nt, lanes) = {tile}")
    # warm-up: W eager steps, then capture the K-step graph
    s.set_fields(h0)
    s.step(min(Wm, T))
    s.sync()
    s.set_fields(h0)
    s.capture(K)
    s.sync()
    # timed region: one graph launch of all K steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_until(K)
    s.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    U = s.energies()[0] if not manip else None
    rep, val, _ = s.best()
    ints = prob.eval_int(s.round())[0]
    updates = nnz * R * K
    value = updates / dt
    log(f"timed {K} steps in {dt * 1e3:.1f} ms: {value:.3e} updates/s; best {val[0]} (replica {rep[0]})")

    # dominant kernel: the fused step kernel, timed with HIP events on the
    # solver's stream around every launch (eager pass over the same steps)
    s.set_fields(h0)
    s.profile(True)
    s.step(min(K, 200))
    kern_ms, n_k = s.profile_result()
    s.profile(False)
    mbytes = 2 if dtype == fem.BF16 else 4
    if manip:
        alg_bytes = manip_kernel_bytes(n, R, nnz)
        kname, counters = "maxcut_manip_kernel", "maxcut_manip_n1e5_R256_hbm_counters.md"
    elif kind == "maxcut_dense":
        alg_bytes = dense_kernel_bytes(n, R, 1 if dense_i8 else 4)
        kname = "maxcut_dense_i8_step_kernel" if dense_i8 else "maxcut_dense_step_kernel"
        counters = f"{wl['counters']}_{'i8' if dense_i8 else 'f64'}_hbm_counters.md"
    elif kind == "maxcut":
        alg_bytes = step_kernel_bytes(n, R, nnz, mbytes)
        kname, counters = "maxcut_step_kernel", f"{wl['counters']}_{args.dtype}_hbm_counters.md"
    elif kind == "bmincut":
        alg_bytes = potts_kernel_bytes(n, R, q, nnz, mbytes)
        rcm = "_rcm" if args.order == "rcm" else ""
        kname, counters = "potts_step_kernel", f"{wl['counters']}{rcm}_{args.dtype}_hbm_counters.md"
    else:
        alg_bytes = sat_kernel_bytes(n, R, nnz, mbytes)
        kname, counters = "sat_step_kernel", f"{wl['counters']}_{args.dtype}_hbm_counters.md"
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    if args.state_layout != "interleaved":
        counters = counters.replace("_hbm_counters", f"_{args.state_layout}_hbm_counters")
    src = "dense" if kind == "maxcut_dense" else args.gradient
    traffic = measured_traffic(os.path.join(ROOT, "profiles", counters), src, tile, args.dtype,
                               args.state_layout)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kname, "kernel_avg_ms": round(kern_ms, 5), "kernel_launches": n_k,
            "alg_bytes_per_launch": int(alg_bytes), "kernel_sources_sha256": kernel_sources_sha(src)}
    if kind == "maxcut_dense":
        # a dense contraction: the matrix-core peak of the type it runs in
        # bounds it (int8: four digit-plane products per step; FP64: one);
        # the HBM figures stay alongside
        flops = (4.0 if dense_i8 else 1.0) * 2.0 * n * n * R
        peak = MFMA_I8_PEAK_TOPS if dense_i8 else MFMA_F64_PEAK_TFLOPS
        tfs = flops / (kern_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": peak, "unit": "TOP/s" if dense_i8 else "TFLOP/s",
                "frac": round(tfs / peak, 4), "traffic": traffic, "ops_per_launch": flops,
                "hbm_achieved_GBps": round(achieved, 1), "kernel": kname, "kernel_avg_ms": round(kern_ms, 5),
                "kernel_launches": n_k, "alg_bytes_per_launch": int(alg_bytes),
                "kernel_sources_sha256": kernel_sources_sha(src)}
    label = {"maxcut": "cut", "maxcut_dense": "cut", "bmincut": "2 cut + lambda sum |Pi|(|Pi|-1)",
             "maxsat": "unsatisfied clauses"}[kind]
    out = {
        "metric": "replica-edge updates/s (nnz*R*steps/s)",
        "value": value,
        "unit": "replica-edge updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": dt * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32+sign-bit-readouts" if manip
                  else ("f32 state, exact int8 x fixed-point field product" if dense_i8 else
                        "f32 state, f64 field product") if kind == "maxcut_dense"
                  else "f32" if dtype == fem.F32 else "f32+bf16-marginals"),
        "data": f"synthetic (seeded generator: {wl['data']})",
        "config": {"workload": wl["name"] + ("_rcm" if kind == "bmincut" and args.order == "rcm" else ""),
                   "n": n, "nnz": nnz, "q": q if kind == "bmincut" else 2,
                   "replicas": R, "anneal_steps": K, "marginals": args.dtype, "gradient": args.gradient,
                   "state_layout": args.state_layout,
                   "schedule": ("inverse-proportional T 1.16->6e-5, RMSprop lr 0.03 alpha 0.56 momentum 0.63 "
                                "weight decay 0.013" if kind == "maxcut_dense" else "linear beta 0.01->5, Adam lr 0.1"),
                   "tile": list(tile),
                   "parallelism": "single GPU",
                   "node_order": args.order if kind == "bmincut" else "as generated",
                   "order_seconds": order_s if kind == "bmincut" else None},
        "result": {"best": float(val[0]), "best_is": label, "mean_integer": float(np.mean(ints)),
                   "U_mean_final": float(np.mean(U)) if U is not None else None},
        "roofline": roof,
    }
    if kind == "maxcut" and not args.no_cpu and not manip:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline_graph(wl["recipe"], args.cpu_replicas,
                                                 args.cpu_steps or (100 if n > 10_000 else 500))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
