#!/usr/bin/env python3
"""Throughput benchmark of the FEM hot path on one MI355X.

Workload (default): MaxCut on a random sparse graph, N = 100,000 nodes,
300,000 edges with uniform endpoints and +/-1 weights, R = 256 replicas,
a 2,000-step anneal (linear beta 0.01 -> 5, Adam lr 0.1), float32 fields and
Adam state, float32 (or --dtype bf16) marginal copy.  One "step" is one pass
of the whole hot path: sparse field product, gradient, Adam, new marginals,
and per-replica energies U, S, F; the read-out runs at the end of the anneal.

Metric: replica-edge updates per second = nnz * R * steps / seconds, with
nnz = 2 x edges, timed over one captured HIP graph of all K steps with the
inputs resident in HBM.  Prints one JSON line.

--gradient manipulated runs the same workload with the paper's manipulated
gradients (one-hot neighbour read-outs, 1/sum|W| normalisation): the gather
then reads sign bits, and no energies are formed.

--workload k2000dense is the dense-W path: MaxCut on a complete graph of
2,000 nodes with +/-1 weights (the shape of the paper's K2000 benchmark),
R = 1,000, RMSprop with the paper's K2000 settings.  With integral weights the
field product is formed exactly from int8 digit planes of the fixed-point
marginals on the int8 matrix cores (four int8 products per step), so its
roofline is the int8 MFMA peak; other weights run on the FP64 matrix cores.

roofline.traffic is the HBM traffic of one step-kernel launch measured with
the FETCH_SIZE and WRITE_SIZE counters (scaled by a plain copy of known
size), read from the committed counter summary of this workload; it is null
when the kernel sources, launch shape or marginal type differ from the ones
the counters were taken with.
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


def step_kernel_bytes(n, R, nnz, mbytes, n_tiles, NE=2):
    """Algorithmic bytes of one step-kernel launch (MaxCut): h, m1, m2 read and
    written (24 B per replica-node), the marginal copy read once and written
    once, the CSR (int64 row offsets, 8-byte {col, weight} entries) and the
    per-tile energy partials."""
    state = n * R * (24 + 2 * mbytes)
    csr = 8 * (n + 1) + 8 * nnz
    parts = 8 * NE * R * n_tiles
    return state + csr + parts


def manip_kernel_bytes(n, R, nnz):
    """Algorithmic bytes of one manipulated-gradient MaxCut launch: h, m1, m2
    read and written, the sign bits (ceil(R/32) words per row) read once and
    written once, the CSR and the per-node normaliser (8 B)."""
    rw = (R + 31) // 32
    return n * R * 24 + 2 * 4 * n * rw + 8 * (n + 1) + 8 * nnz + 8 * n


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


def cpu_baseline(graph, R_sample, steps_sample):
    import oracle as O
    from paper_2412_09285_amd import workloads as W

    h0 = W.initial_fields(graph.n, R_sample, seed=102)
    run = O.maxcut_run(graph, O.Params(R=R_sample, T=2000), h0)
    t0 = time.perf_counter()
    run.step(steps_sample)
    dt = time.perf_counter() - t0
    return {
        "value": graph.nnz * R_sample * steps_sample / dt,
        "unit": "replica-edge updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"same graph (N={graph.n}, nnz={graph.nnz}), {R_sample} of the replicas, first "
                  f"{steps_sample} steps, FP64 single-threaded C oracle, {dt:.1f} s",
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
    ap.add_argument("--cpu-replicas", type=int, default=8)
    ap.add_argument("--cpu-steps", type=int, default=400,
                    help="oracle steps of the CPU baseline sample (8 replicas by default): 10-20 s of CPU work")
    ap.add_argument("--workload", choices=["maxcut1e5", "bmincut1e6", "max3sat1e5", "k2000dense", "er800", "batch512",
                                           "copy"],
                    default="maxcut1e5",
                    help="maxcut1e5: the throughput line; bmincut1e6 / max3sat1e5: the Potts and Max-3-SAT "
                         "kernels at full size; er800: a G-set-sized instance (800 nodes, R = 16), launch-bound; "
                         "k2000dense: the dense-W (matrix-core) path on a complete "
                         "2000-node graph; batch512: time to target on 512 uneven MaxCut instances; "
                         "copy: a plain device copy (calibrates HBM counters)")
    ap.add_argument("--order", choices=["draw", "rcm"], default="rcm",
                    help="bmincut1e6: node order of the graph (rcm: relabelled by fem_graph_order before the "
                         "problem is built; draw: as generated)")
    ap.add_argument("--instances", type=int, default=512)
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
              "(replicas would shard with no communication; see the design notes). "
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
        from paper_2412_09285_amd import batchbench

        res = batchbench.main_batch(args, torch.cuda.Stream())
        plain = res["plain_per_instance_s"]
        best = res.get("batched_bf16_warm", {}).get("time_to_target_s") or \
            res["batched_bf16"]["time_to_target_s"]
        print(json.dumps({"metric": "time to best cut within 0.1% of plain FEM", "value": best, "unit": "s",
                          "higher_is_better": False, "n_gpus": 1, "vs_baseline": None,
                          "dtype": "f32 fields/Adam + bf16 marginals", "data": "synthetic",
                          "config": dict(workload="batch512_maxcut", **res["config"]), "result": res}))
        return
    throughput(args)


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
    float or as four int8 digits), h, m1, m2 read and written, the energy
    partials."""
    return w_bytes * n * n + n * R * (24 + 8) + 16 * R * (-(-n // 64))


def potts_kernel_bytes(n, R, q, nnz, mbytes, n_tiles):
    """Algorithmic bytes of one bMinCut launch: h, m1, m2 read and written and
    the marginal copy read once and written once (24 + 2 b per replica-node-
    state), the CSR, the weighted degree (4 B per node), and per tile the
    centred column sums read, the column-sum partials and the three energy
    partials written (8 B each per replica and state / replica)."""
    return n * R * q * (24 + 2 * mbytes) + 8 * (n + 1) + 8 * nnz + 4 * n + 8 * R * (2 * q + 3) * n_tiles


def sat_kernel_bytes(n, R, nnz, mbytes, n_tiles, rec_bytes=8):
    """Algorithmic bytes of one Max-k-SAT launch: h, m1, m2 and the marginal
    copy as for MaxCut, the incidence records (8 B each for 3-SAT), the row
    offsets and the per-tile energy partials."""
    return n * R * (24 + 2 * mbytes) + 8 * (n + 1) + rec_bytes * nnz + 16 * R * n_tiles


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
    vec, waves, rows, nt, lanes = tile
    per_lane = vec if kind != "bmincut" else 1
    lanes = min(lanes, 64)
    n_tiles = -(-n // (waves * (64 // lanes) * rows))
    mbytes = 2 if dtype == fem.BF16 else 4
    if manip:
        alg_bytes = manip_kernel_bytes(n, R, nnz)
        kname, counters = "maxcut_manip_kernel", "maxcut_manip_n1e5_R256_hbm_counters.md"
    elif kind == "maxcut_dense":
        alg_bytes = dense_kernel_bytes(n, R, 1 if dense_i8 else 4)
        kname = "maxcut_dense_i8_step_kernel" if dense_i8 else "maxcut_dense_step_kernel"
        counters = f"{wl['counters']}_{'i8' if dense_i8 else 'f64'}_hbm_counters.md"
    elif kind == "maxcut":
        alg_bytes = step_kernel_bytes(n, R, nnz, mbytes, n_tiles)
        kname, counters = "maxcut_step_kernel", f"{wl['counters']}_{args.dtype}_hbm_counters.md"
    elif kind == "bmincut":
        alg_bytes = potts_kernel_bytes(n, R, q, nnz, mbytes, n_tiles)
        rcm = "_rcm" if args.order == "rcm" else ""
        kname, counters = "potts_step_kernel", f"{wl['counters']}{rcm}_{args.dtype}_hbm_counters.md"
    else:
        alg_bytes = sat_kernel_bytes(n, R, nnz, mbytes, n_tiles)
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
    if kind in ("maxcut", "maxcut_dense") and not args.no_cpu and not manip:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_replicas, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
