"""Benchmark of the hierarchical Russian-roulette hot path on one MI355X.

Default workload (one "step" = one pass of the whole hot path over a frame):
1920x1080 eye vertices against 2^20 light vertices drawn from one seeded
64-Gaussian mixture (sigma 0.02) in the unit cube, fp32 positions, 64x64
dither tile, s = 1e-4, Morton hierarchy with leaf size 1 (built once,
before timing), one persistent launch per step: per-eye shift, rotated
radical inverse, range minimum per node (the paper's sweep), node bound,
cull/descend, exact leaf test and pair emission.  Inputs and the output
buffer are resident in HBM before timing starts.

Prints ONE JSON line.  Metric: eye-vertex traversals per second (the pair
rate is reported beside it).  Other workloads (--workload rangemin | batched
| served) are for the design notes, not the headline line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# non-packed 32-bit VALU issue: 256 CU x 64 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic 32-bit VALU lane-operations per unit of traversal work, counted
# from the arithmetic each unit needs as gfx950 executes it (the breakdown
# follows):
#   visit : one internal node popped, both children bounded -- inherited
#           minimum selection 5; per child 34 (box distance 9, squares and sum
#           5, IEEE division 10, margin and min 3, fixed-point keep test 5,
#           rotated value 2); survivor/leaf decisions 8; ballot compaction 8
#   rmq   : one range minimum with the default method (case test, bit-parallel
#           flip-position selection, seed and about two refinement steps)
#   leaf  : one exact test of a light inside a multi-light leaf
#   pair  : one emitted pair (compaction, position, store address)
OPS_VISIT = 5 + 2 * 34 + 8 + 8
OPS_RMQ = 40
OPS_LEAF = 30
OPS_PAIR = 6
BYTES_PER_QUERY = 20   # range minimum: a, b, r in; argmin, min out


def _sync_all():
    import torch
    torch.cuda.synchronize()


def frame_workload(args):
    import numpy as np
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    fr = synth.frame()
    ctx = hrr.Context(fr["tile"], device=0)
    t0 = time.time()
    h = ctx.build_hierarchy(fr["lights"], leaf_size=fr["leaf"])
    build_s = time.time() - t0
    eyes = torch.from_numpy(fr["eyes"]).to("cuda:0")
    n_eyes = fr["eyes"].shape[0]
    method = hrr.RMQ_DIRECT if args.rmq == "direct" else hrr.RMQ_PAPER
    kw = dict(rmq_method=method, eyes_per_wave=args.epw, stack_entries=args.stack)
    n = ctx.count(h, eyes, fr["s"], fr["width"], **kw)
    pairs = torch.empty((max(n, 1), 2), dtype=torch.int32, device="cuda:0")
    # one untimed launch with counters on: units of work for the roofline
    _, _, st = ctx.traverse(h, eyes, fr["s"], fr["width"], pairs=pairs, stats=True, **kw)
    for _ in range(args.warmup):
        ctx.traverse(h, eyes, fr["s"], fr["width"], pairs=pairs, **kw)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    _sync_all()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        _, got, _ = ctx.traverse(h, eyes, fr["s"], fr["width"], pairs=pairs, **kw)
        assert got == n
    e1.record(stream)
    _sync_all()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    gpu_ms = e0.elapsed_time(e1) / args.steps

    multi_leaf_tests = max(st["leaf_tests"] - 2 * st["node_visits"], 0)
    ops = (st["node_visits"] * OPS_VISIT + st["rmq_calls"] * OPS_RMQ + multi_leaf_tests * OPS_LEAF
           + n * OPS_PAIR)
    achieved = ops / (gpu_ms * 1e-3) / 1e12
    line = {
        "metric": "eye-vertex traversals/s",
        "value": n_eyes / (ms * 1e-3),
        "unit": "eyes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "frame: 1920x1080 eyes x 2^20 lights, 64-Gaussian mixture "
                               "sigma 0.02, s=1e-4, leaf 1, one launch",
                   "n_eyes": n_eyes, "n_lights": int(fr["lights"].shape[0]),
                   "rmq": args.rmq, "parallelism": "1 GPU"},
        "pairs_per_s": n / (ms * 1e-3),
        "accepted_pairs": n,
        "kernel_ms": gpu_ms,
        "hierarchy_build_s": build_s,
        "units": {"node_visits": st["node_visits"], "rmq_calls": st["rmq_calls"],
                  "leaf_tests": st["leaf_tests"], "pairs": n},
        "algorithmic_lane_ops": ops,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": (None if args.traffic_kib is None
                                 else (args.traffic_kib[0] + args.traffic_kib[1]) * 1024.0)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_frame(fr, h.permutation(), n_eyes, args)
    h.free()
    ctx.close()
    return line


def cpu_baseline_frame(fr, perm, n_eyes, args):
    import numpy as np
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    ls = fr["lights"][perm]
    sel = np.linspace(0, n_eyes - 1, args.cpu_eyes).astype(np.uint32)
    t0 = time.perf_counter()
    oracle.accept_eyes(fr["eyes"], sel, fr["width"], 0, fr["tile"], ls, fr["s"], threads=threads)
    dt = time.perf_counter() - t0
    return {"value": sel.size / dt, "unit": "eyes/s", "cores": threads, "kind": "oracle",
            "sample": "%d eyes evenly spaced over the frame, all-pairs test against all %d "
                      "lights (%.1f s)" % (sel.size, ls.shape[0], dt)}


def rangemin_workload(args):
    import numpy as np
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    a, b, r = synth.rangemin_queries()
    ctx = hrr.Context(synth.dither_tile(100), device=0)
    dev = "cuda:0"
    ta, tb, tr = (hrr.u32_tensor(x, dev) for x in (a, b, r))
    k = torch.empty_like(ta)
    v = torch.empty_like(ta)
    method = hrr.RMQ_DIRECT if args.rmq == "direct" else hrr.RMQ_PAPER
    for _ in range(args.warmup):
        ctx.range_min(ta, tb, tr, method=method, out_k=k, out_v=v)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    _sync_all()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.range_min(ta, tb, tr, method=method, out_k=k, out_v=v)
    e1.record(stream)
    _sync_all()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    gpu_ms = e0.elapsed_time(e1) / args.steps
    nq = a.size
    gbs = nq * BYTES_PER_QUERY / (gpu_ms * 1e-3) / 1e9
    line = {
        "metric": "range-min queries/s", "value": nq / (ms * 1e-3), "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "rangemin: 2^28 queries, a<b uniform u32, r uniform u32",
                   "rmq": args.rmq},
        "kernel_ms": gpu_ms,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        a2, b2, r2 = synth.rangemin_check_queries()
        t0 = time.perf_counter()
        oracle.rmq_scan(a2[:8192], b2[:8192], r2[:8192], threads=threads)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 8192 / dt, "unit": "queries/s", "cores": threads,
                                "kind": "oracle",
                                "sample": "8192 queries with b-a <= 2^16 by scanning (%.1f s)"
                                          % dt}
    ctx.close()
    return line


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="frame", choices=["frame", "rangemin"])
    p.add_argument("--rmq", default="paper", choices=["paper", "direct"])
    p.add_argument("--epw", type=int, default=1)
    p.add_argument("--stack", type=int, default=512)
    p.add_argument("--traffic-kib", type=float, nargs=2, default=None,
                   metavar=("FETCH", "WRITE"),
                   help="FETCH_SIZE and WRITE_SIZE (KiB per launch) of the traversal kernel "
                        "from rocprofv3 --pmc runs, already scaled by the copy-kernel factors")
    p.add_argument("--cpu-eyes", type=int, default=256)
    p.add_argument("--no-cpu-baseline", action="store_true")
    args = p.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sharded design is documented, not built)", file=sys.stderr)
        sys.exit(2)
    fn = frame_workload if args.workload == "frame" else rangemin_workload
    line = fn(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
