"""Benchmark of the hierarchical Russian-roulette hot path on one MI355X.

Default run (``python bench.py``): every measurement of the hot path, printed
as ONE JSON line whose headline is the frame:

* frame (headline; one "step" = one pass of the whole hot path over a frame):
  1920x1080 eye vertices against 2^20 light vertices drawn from one seeded
  64-Gaussian mixture (sigma 0.02) in the unit cube, fp32 positions, 64x64
  dither tile, s = 1e-4, Morton hierarchy with leaf size 1 (built once, before
  timing), one persistent launch per step: per-eye shift, rotated radical
  inverse, range minimum per node (the paper's method), node bound,
  cull/descend, exact leaf test and pair emission.  Inputs and the output
  buffer are resident in HBM before timing starts.  The headline uses the
  hierarchy with power-of-two splits; ``frame_other_split`` is the same frame
  on the radix (highest differing Morton bit) hierarchy;
* ``range_min``: 2^28 range-minimum queries (a < b uniform u32, uniform shift);
* ``batched``: 256 caches in one call against 256 plain launches;
* ``served``: the serving loop at 0.3 / 0.6 / 0.9 of its saturation rate,
  against plain single launches served one at a time.

``--workload frame|tiny|rangemin|batched|served`` runs one of them alone.

Rooflines price the work with fixed per-unit figures (lane-operations or
bytes per unit of work, see OPS_* below) times the units the kernel's
statistics launch counts, divided by the kernel's own duration (HIP events
around that kernel on the call's stream).
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
# 32-bit VALU lane-operations: 256 CU x 4 SIMD x 32 lanes x 2.4 GHz = 78.6 T/s,
# the rate behind the published fp32 vector peak (157.3 TFLOP/s = 78.6 T FMA/s).
# (Plain 32-bit integer instructions issue at half that rate on gfx950; the
# higher denominator is the conservative one.)
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

# Algorithmic work per unit (32-bit lane-operations), the hot path's own
# per-unit figures:
#   bound : one child's node bound -- box distance, acceptance bound and the
#           comparison with the child's minimum (~15 fp32/int operations)
#   rmq   : one range minimum with the paper's sweeps, ~15 sweep steps of ~10
#           integer operations each on node-like ranges
#   pair  : one accepted pair: its exact test and its emission (~15)
#   leaf  : one exact test of a light inside a leaf of several lights (~15)
#   query : one query of the range-minimum microbenchmark: ~3 sweep steps of
#           ~10 operations plus ~15 fixed
OPS_BOUND = 15
OPS_RMQ = 150
OPS_PAIR = 15
OPS_LEAF = 15
OPS_QUERY = 3 * 10 + 15
BYTES_PER_QUERY = 20   # range minimum: a, b, r in; argmin, min out
RMQ_METHODS = {"paper": 0, "direct": 1, "paper_full": 2, "paper_loop": 3, "dyadic": 4,
               "paper_no_reuse": 5}
# Section 3's extra rotation of sample n: psi(n) = s0 + n alpha (mod 1), s0 fixed here
PSI_S0 = 0x6A09E667


def _sync_all():
    import torch
    torch.cuda.synchronize()


def _free_gpu():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def lane_ops(st, n_pairs):
    """Algorithmic lane-operations of a traversal from its statistics: each
    node visit bounds both children."""
    return (2 * st["node_visits"] * OPS_BOUND + st["rmq_calls"] * OPS_RMQ
            + n_pairs * OPS_PAIR + st["leaf_tests"] * OPS_LEAF)


def alu_roofline(ops, kernel_ms, traffic=None):
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic}


def host_cpu():
    """Threads this process may run on, the machine's CPU count and model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, usable), os.cpu_count() or 1, model


def timed_launches(fn, steps, warmup):
    """Run fn warmup + steps times; wall ms per step and GPU ms per step
    (torch events on the current stream around the timed steps)."""
    import torch
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    _sync_all()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    _sync_all()
    return (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps


# ---------------------------------------------------------------------------
# frame
# ---------------------------------------------------------------------------

def frame_workload(args, split=None, cpu=True, steps=None, warmup=None):
    import numpy as np
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    split = split or args.split
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    tiny = args.workload == "tiny"
    fr = synth.tiny() if tiny else synth.frame()
    ns = 1 if tiny else max(1, args.samples)
    if ns > 1:
        # several samples per eye (Section 3): the first 1080 / N pixel rows,
        # so that eyes x samples stays at about one frame of virtual eyes
        rows = max(1, 1080 // ns)
        fr = dict(fr, eyes=np.ascontiguousarray(fr["eyes"][:rows * fr["width"]]))
    ctx = hrr.Context(fr["tile"], device=0)
    t0 = time.time()
    h = ctx.build_hierarchy(fr["lights"], leaf_size=fr["leaf"], split=split)
    build_s = time.time() - t0
    lights_dev = torch.from_numpy(fr["lights"]).to("cuda:0")
    hd = ctx.build_hierarchy_device(lights_dev, leaf_size=fr["leaf"], split=split)   # warm-up
    hd.free()
    _sync_all()
    t0 = time.perf_counter()
    hd = ctx.build_hierarchy_device(lights_dev, leaf_size=fr["leaf"], split=split)
    build_dev_s = time.perf_counter() - t0
    hd.free()
    eyes = torch.from_numpy(fr["eyes"]).to("cuda:0")
    n_eyes = fr["eyes"].shape[0] * ns           # virtual eyes (eye x sample)
    method = RMQ_METHODS[args.rmq]
    kw = dict(rmq_method=method, eyes_per_wave=args.epw, stack_entries=args.stack)
    if ns > 1:
        kw.update(n_samples=ns, psi_s0=PSI_S0)
    n = ctx.count(h, eyes, fr["s"], fr["width"], **kw)
    pairs = torch.empty((max(n, 1), 2), dtype=torch.int32, device="cuda:0")
    weights = torch.empty((max(n, 1),), dtype=torch.float32, device="cuda:0") if args.weights else None
    kw["weights"] = weights
    # one untimed launch with counters on: units of work for the roofline
    st = ctx.traverse(h, eyes, fr["s"], fr["width"], pairs=pairs, stats=True, **kw)[2]
    kernel_ms = []

    def step():
        # timing=True: the library brackets the traversal kernel with HIP
        # events on this same stream
        _, got, stt = ctx.traverse(h, eyes, fr["s"], fr["width"], pairs=pairs, timing=True, **kw)[:3]
        assert got == n
        kernel_ms.append(stt["kernel_ms"])

    ms, step_gpu_ms = timed_launches(step, steps, warmup)
    gpu_ms = sum(kernel_ms[warmup:]) / max(len(kernel_ms) - warmup, 1)
    ops = lane_ops(st, n)
    traffic = (_traffic_bytes(args, split=split)
               if (ns == 1 and not args.weights and not tiny and method == 0) else None)
    line = {
        "metric": "eye-vertex traversals/s",
        "value": n_eyes / (ms * 1e-3),
        "unit": "eyes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": _frame_name(ns, args.weights, tiny, split),
                   "n_eyes": n_eyes, "n_lights": int(fr["lights"].shape[0]), "split": split,
                   "rmq": args.rmq, "parallelism": "1 GPU"},
        "pairs_per_s": n / (ms * 1e-3),
        "accepted_pairs": n,
        "kernel_ms": gpu_ms,
        "step_gpu_ms": step_gpu_ms,
        "hierarchy_build_s": build_s,
        "hierarchy_build_device_s": build_dev_s,
        "units": {"node_visits": st["node_visits"], "child_bounds": 2 * st["node_visits"],
                  "rmq_calls": st["rmq_calls"], "leaf_tests": st["leaf_tests"], "pairs": n,
                  "stack_spills": st["spills"], "max_stack": st["max_stack"]},
        "algorithmic_lane_ops": ops,
        "roofline": alu_roofline(ops, gpu_ms, traffic),
    }
    if ns > 1:
        line["config"]["samples_per_eye"] = ns
        line["config"]["psi_s0"] = PSI_S0
    if traffic is not None:
        # everything that leaves the L2s (Infinity Cache hits included),
        # beside the ALU roofline (from the recorded counter runs)
        line["memory_side"] = {"bytes": traffic, "TB_per_s": traffic / (gpu_ms * 1e-3) / 1e12,
                               "frac_of_hbm_peak": traffic / (gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "source": "profiles/traverse_frame_traffic.json"}
    if cpu and not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_frame(fr, fr["eyes"].shape[0], args, ns)
    del pairs, weights, eyes, lights_dev
    h.free()
    ctx.close()
    _free_gpu()
    return line


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traverse_frame_traffic.json")
RMQ_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "range_min_traffic.json")
# Everything that shapes the counted launches: the kernels and their headers,
# the launch layout (eye order, queues) and the host build's record layout.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1907_12343_amd", "csrc", f)
                  for f in ("hrr_kernels.hip", "hrr_rmq.hpp", "hrr_types.hpp", "hrr_compact.hpp",
                            "hrr_scan.hpp", "hrr_layout.hpp", "hrr_launch.cpp", "hrr_build.cpp")]


def kernel_source_digest():
    """SHA-256 of the kernel sources with comments and blank space removed, so
    that only a change of the code itself invalidates recorded counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def _traffic_bytes(args, path=TRAFFIC_FILE, split=None):
    """HBM bytes of one timed launch of the dominant kernel: FETCH_SIZE +
    WRITE_SIZE from rocprofv3 --pmc runs, scaled by the copy-kernel
    calibration, as recorded in profiles/ together with the digest of the
    kernel sources they were taken on; None when the kernel has changed since
    (or --traffic-kib overrides)."""
    if args.traffic_kib is not None:
        return (args.traffic_kib[0] + args.traffic_kib[1]) * 1024.0
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != kernel_source_digest():
        return None
    if split is not None and rec.get("split", "radix") != split:
        return None   # counters taken on the other hierarchy
    return (rec["fetch_kib_scaled"] + rec["write_kib_scaled"]) * 1024.0


def _frame_name(ns, weights, tiny=False, split="radix"):
    name = "frame: 1920x1080 eyes x 2^20 lights, 64-Gaussian mixture sigma 0.02, s=1e-4, leaf 1"
    if tiny:
        # the small parity case: launch-latency bound, reported for completeness
        name = "tiny: 4096 uniform eyes (64 wide) x 1024 uniform lights, s=1e-3, leaf 1"
    elif ns > 1:
        name = ("frame rows 0..%d (1920x%d eyes) x %d samples per eye x 2^20 lights, "
                "64-Gaussian mixture sigma 0.02, s=1e-4, leaf 1" % (1080 // ns - 1, 1080 // ns, ns))
    name += ", power-of-two splits" if split == "pow2" else ", radix splits"
    if weights:
        name += ", 1/p weights"
    return name + ", one launch"


def cpu_baseline_frame(fr, n_eyes, args, ns=1):
    import numpy as np
    import oracle
    threads, cpu_count, model = host_cpu()
    ls = fr["lights"][oracle.morton_order(fr["lights"])]   # the oracle's own light order
    sel = np.linspace(0, n_eyes - 1, max(1, args.cpu_eyes // ns)).astype(np.uint32)
    t0 = time.perf_counter()
    oracle.accept_eyes(fr["eyes"], sel, fr["width"], 0, fr["tile"], ls, fr["s"], n_samples=ns,
                       psi_s0=PSI_S0 if ns > 1 else 0, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": sel.size * ns / dt, "unit": "eyes/s", "cores": threads, "kind": "oracle",
            "sample": "%d eyes%s evenly spaced over the eye set, all-pairs test against all %d "
                      "lights (%.1f s)" % (sel.size, " x %d samples" % ns if ns > 1 else "",
                                           ls.shape[0], dt),
            "host_cpu_count": cpu_count, "cpu_model": model}


# ---------------------------------------------------------------------------
# range minimum
# ---------------------------------------------------------------------------

def rangemin_workload(args, steps=None, warmup=None):
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    if args.rmq == "paper_no_reuse":
        sys.exit("--rmq paper_no_reuse changes the traversal only; range_min has no parent minimum")
    a, b, r = synth.rangemin_queries()
    ctx = hrr.Context(synth.dither_tile(100), device=0)
    dev = "cuda:0"
    ta, tb, tr = (hrr.u32_tensor(x, dev) for x in (a, b, r))
    k = torch.empty_like(ta)
    v = torch.empty_like(ta)
    method = RMQ_METHODS[args.rmq]
    ms, gpu_ms = timed_launches(lambda: ctx.range_min(ta, tb, tr, method=method, out_k=k, out_v=v),
                                steps, warmup)
    nq = a.size
    gbs = nq * BYTES_PER_QUERY / (gpu_ms * 1e-3) / 1e9
    line = {
        "metric": "range-min queries/s", "value": nq / (ms * 1e-3), "unit": "queries/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "rangemin: 2^28 queries, a<b uniform u32, r uniform u32",
                   "rmq": args.rmq},
        "kernel_ms": gpu_ms,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic_bytes(args, RMQ_TRAFFIC_FILE)},
        # the integer work beside it
        "valu": {"lane_ops": nq * OPS_QUERY, "unit": "Tlane-op/s",
                 "achieved": nq * OPS_QUERY / (gpu_ms * 1e-3) / 1e12,
                 "frac": nq * OPS_QUERY / (gpu_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads, cpu_count, model = host_cpu()
        a2, b2, r2 = synth.rangemin_check_queries()
        m = min(args.cpu_queries, a2.size)
        t0 = time.perf_counter()
        oracle.rmq_scan(a2[:m], b2[:m], r2[:m], threads=threads)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": m / dt, "unit": "queries/s", "cores": threads,
                                "kind": "oracle",
                                "sample": "%d queries with b-a <= 2^16 by scanning (%.1f s)"
                                          % (m, dt),
                                "host_cpu_count": cpu_count, "cpu_model": model}
    del ta, tb, tr, k, v
    ctx.close()
    _free_gpu()
    return line


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

def batched_workload(args, steps=None, warmup=None):
    """256 independent caches (own mixture, 2^U[10,20] lights, 2^U[10,16]
    eyes, s = 1e-4) in ONE call -- one persistent launch per eyes-per-wave
    group of the items -- against 256 plain launches of the same items on the
    same GPU.  Before timing, the batched autotuner runs once per light
    class (log2 of the light count) on all caches of the class together, over
    leaf sizes 1, 2, 4, 8 and the launch shapes; every cache is built with
    its class's leaf size, and the call groups the items by their classes'
    eyes per wave.  Every group's own ALU fraction is measured with a call of
    that group alone."""
    import numpy as np
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    ctx = hrr.Context(synth.dither_tile(100), device=0)
    caches = [synth.batched_cache(c) for c in range(256)]
    sizes = np.array([d["lights"].shape[0] for d in caches])
    lclass = np.array([int(n).bit_length() - 1 for n in sizes])
    t0 = time.time()
    eyes = [torch.from_numpy(d["eyes"]).to("cuda:0") for d in caches]
    tuned = {}
    for c in sorted(set(lclass.tolist())):
        ks = np.flatnonzero(lclass == c)
        sets = []
        for L in (1, 2, 4, 8):
            sets.append([dict(h=ctx.build_hierarchy(caches[k]["lights"], leaf_size=L, split=args.split),
                              eyes=eyes[k], s=caches[k]["s"], width=caches[k]["width"]) for k in ks])
        tuned[c] = ctx.autotune_batched(sets)
        for st_ in sets:
            for it in st_:
                it["h"].free()
    leaves = [tuned[int(c)]["leaf_size"] for c in lclass]
    hs = [ctx.build_hierarchy(d["lights"], leaf_size=L, split=args.split) for d, L in zip(caches, leaves)]
    setup_s = time.time() - t0
    counts = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    total = int(offs[-1])
    pairs = torch.empty((max(total, 1), 2), dtype=torch.int32, device="cuda:0")
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(counts[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    n_eyes = int(sum(d["eyes"].shape[0] for d in caches))
    got, st = ctx.traverse_batched(items, pairs, stats=True)
    assert [int(x) for x in got] == counts

    kms = []

    def batched():
        _, stt = ctx.traverse_batched(items, pairs, timing=True)
        kms.append(stt["kernel_ms"])

    ms, step_gpu_ms = timed_launches(batched, steps, warmup)
    gpu_ms = sum(kms[warmup:]) / max(len(kms) - warmup, 1)

    def plain():
        for k, (h, e, d) in enumerate(zip(hs, eyes, caches)):
            ctx.traverse(h, e, d["s"], d["width"], pairs=pairs[offs[k]:offs[k] + max(counts[k], 1)],
                         capacity=counts[k])

    ms_plain, _ = timed_launches(plain, max(1, steps // 4), 1)
    ops = lane_ops(st, total)

    # the groups alone (the call's grouping: the eyes per wave tuned for the class)
    groups = {}
    for k in range(len(caches)):
        e = tuned[int(lclass[k])]["eyes_per_wave"]
        groups.setdefault("%d eye%s/wave" % (e, "" if e == 1 else "s"), []).append(k)
    per_group = {}
    for g, ks in groups.items():
        sub = [items[k] for k in ks]
        _, sst = ctx.traverse_batched(sub, pairs, stats=True)
        gk = []

        def run_sub():
            _, stt = ctx.traverse_batched(sub, pairs, timing=True)
            gk.append(stt["kernel_ms"])

        timed_launches(run_sub, steps, warmup)
        g_ms = sum(gk[warmup:]) / max(len(gk) - warmup, 1)
        g_pairs = int(sum(counts[k] for k in ks))
        per_group[g] = {"items": len(ks), "eyes": int(sum(caches[k]["eyes"].shape[0] for k in ks)),
                        "light_classes": sorted({int(lclass[k]) for k in ks}),
                        "pairs": g_pairs, "kernel_ms": g_ms,
                        "alu_frac": alu_roofline(lane_ops(sst, g_pairs), g_ms)["frac"]}
    line = {
        "metric": "eye-vertex traversals/s", "value": n_eyes / (ms * 1e-3), "unit": "eyes/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "batched: 256 caches, own 64-Gaussian mixture each, 2^U[10,20] "
                               "lights, 2^U[10,16] eyes, s=1e-4, one call (a launch per "
                               "eyes-per-wave group)",
                   "n_eyes": n_eyes, "n_lights": int(sizes.sum()), "split": args.split,
                   "tuned_per_light_class": {"2^%d" % c: v for c, v in sorted(tuned.items())},
                   "parallelism": "1 GPU"},
        "pairs_per_s": total / (ms * 1e-3), "accepted_pairs": total, "kernel_ms": gpu_ms,
        "step_gpu_ms": step_gpu_ms, "setup_s": setup_s,
        "plain_launches": {"ms_per_step": ms_plain, "eyes_per_s": n_eyes / (ms_plain * 1e-3),
                           "speedup_of_batched": ms_plain / ms},
        "units": {"node_visits": st["node_visits"], "child_bounds": 2 * st["node_visits"],
                  "rmq_calls": st["rmq_calls"], "leaf_tests": st["leaf_tests"], "pairs": total},
        "algorithmic_lane_ops": ops,
        "roofline": alu_roofline(ops, gpu_ms),
        "groups": per_group,
    }
    del pairs, eyes
    for h in hs:
        h.free()
    ctx.close()
    _free_gpu()
    return line


# ---------------------------------------------------------------------------
# served
# ---------------------------------------------------------------------------

def served_workload(args):
    """Serving loop: 16 resident hierarchies of 2^(16+6h/15) lights, requests
    of 2^U[8,18] eyes (each with its own shift offset, s = 1e-4) arriving as
    a Poisson stream at 0.3, 0.6 and 0.9 of the measured saturation rate.
    Reports latency percentiles per load, the same at 0.9 with strict FIFO
    admission, and plain single launches served one at a time (FIFO queue
    replayed over the measured per-request service times of the plain path)."""
    import threading
    import numpy as np
    import torch
    import paper_1907_12343_amd as hrr
    import synth

    ctx = hrr.Context(synth.dither_tile(100), device=0)
    t0 = time.time()
    scenes = [synth.served_hierarchy(k) for k in range(16)]
    hs = [ctx.build_hierarchy(sc["lights"], split=args.split) for sc in scenes]
    n_req = args.requests
    base = synth.served_requests(n_req, 1.0)
    req_eyes = [synth.request_eyes(scenes[int(base["hier"][q])]["centers"], int(base["size"][q]),
                                   int(base["eye_seed"][q])) for q in range(n_req)]
    setup_s = time.time() - t0
    s_val = 1e-4

    def submit(q):
        return ctx.submit(hs[int(base["hier"][q])], req_eyes[q], 64, int(base["offset"][q]), s_val)

    def start(overtake_ms):
        ctx.server_start(hbm_budget_bytes=int(args.budget_gib * (1 << 30)), max_inflight=args.inflight,
                         max_batch_eyes=args.batch_eyes, max_batch_items=64, pairs_per_eye_guess=2000.0,
                         overtake_ms=overtake_ms)

    def drain(tickets, out):
        for t in tickets:
            while not ctx.wait(t, 60000):
                pass
            _, n, info = ctx.poll(t)
            out.append((info["done_s"] - info["submit_s"], n, info["launches"]))
            ctx.release(t)

    start(args.overtake_ms)
    # warm-up and saturation: everything submitted at once
    warm = min(16, n_req)
    res = []
    drain([submit(q) for q in range(warm)], res)
    t_sat = time.perf_counter()
    res = []
    drain([submit(q) for q in range(n_req)], res)
    sat_s = time.perf_counter() - t_sat
    sat_rate = n_req / sat_s
    sat_eyes = float(base["size"].sum()) / sat_s
    sat_pairs = sum(r[1] for r in res) / sat_s

    # per load: about args.load_seconds of arrivals, at least 100 requests
    def n_at(rate):
        return int(min(n_req, max(100, rate * args.load_seconds)))

    def offered(load):
        rate = load * sat_rate
        m = n_at(rate)
        arr = synth.served_requests(n_req, rate)["t"][:m]
        tickets = [None] * m
        ready = threading.Semaphore(0)
        out = []

        def waiter():
            for q in range(m):
                ready.acquire()
                drain([tickets[q]], out)

        th = threading.Thread(target=waiter)
        th.start()
        t_start = time.perf_counter()
        for q in range(m):
            delay = t_start + arr[q] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[q] = submit(q)
            ready.release()
        th.join()
        wall = time.perf_counter() - t_start
        lat = np.array([r[0] for r in out]) * 1e3
        return {"offered_req_per_s": rate, "requests": m, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "pairs_per_s": sum(r[1] for r in out) / wall,
                "eyes_per_s": float(base["size"][:m].sum()) / wall,
                "retried": int(sum(1 for r in out if r[2] > 1))}

    loads = {"%.1f" % load: offered(load) for load in (0.3, 0.6, 0.9)}
    stats = ctx.server_stats()
    ctx.server_stop()
    # the same 0.9 load with strict FIFO admission (a request that does not
    # fit holds up everything behind it)
    start(0.0)
    drain([submit(q) for q in range(warm)], [])
    fifo_09 = offered(0.9)
    ctx.server_stop()

    # plain single launches: upload, count, traverse, one request at a time
    service = np.zeros(n_req)
    for q in range(n_req):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e = torch.from_numpy(req_eyes[q]).to("cuda:0")
        ctx.traverse_all(hs[int(base["hier"][q])], e, s_val, 64, shift_offset=int(base["offset"][q]))
        torch.cuda.synchronize()
        service[q] = time.perf_counter() - t1
    plain = {"req_per_s": n_req / service.sum(), "eyes_per_s": float(base["size"].sum()) / service.sum()}
    for load in (0.3, 0.6, 0.9):
        m = n_at(load * sat_rate)
        arr = synth.served_requests(n_req, load * sat_rate)["t"][:m]
        free_at, lat = 0.0, []
        for q in range(m):
            begin = max(arr[q], free_at)
            free_at = begin + service[q]
            lat.append((free_at - arr[q]) * 1e3)
        lat = np.array(lat)
        plain["load_%.1f" % load] = {"p50_ms": float(np.percentile(lat, 50)),
                                     "p99_ms": float(np.percentile(lat, 99)),
                                     "stable": bool(service[:m].sum() < arr[-1] + service[m - 1])}
    line = {
        "metric": "eye-vertex traversals/s", "value": loads["0.9"]["eyes_per_s"], "unit": "eyes/s",
        "n_gpus": 1, "steps": n_req, "warmup": warm, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "served: 16 resident hierarchies 2^(16+6h/15) lights, Poisson "
                               "requests of 2^U[8,18] eyes, own shift offset, s=1e-4",
                   "requests": n_req, "budget_gib": args.budget_gib, "split": args.split,
                   "overtake_ms": args.overtake_ms, "workers": args.inflight,
                   "max_batch_eyes": args.batch_eyes, "parallelism": "1 GPU"},
        "saturation": {"req_per_s": sat_rate, "eyes_per_s": sat_eyes, "pairs_per_s": sat_pairs},
        "loads": loads, "strict_fifo_admission_0.9": fifo_09, "plain_single_launches": plain,
        "server_stats": stats, "setup_s": setup_s, "roofline": None,
    }
    for h in hs:
        h.free()
    ctx.close()
    _free_gpu()
    return line


# ---------------------------------------------------------------------------
# everything
# ---------------------------------------------------------------------------

def _brief(line, keys):
    return {k: line[k] for k in keys if k in line}


def all_workloads(args):
    """The frame as the headline line, and every other measurement beside it."""
    head = frame_workload(args)
    other = "radix" if args.split == "pow2" else "pow2"
    fo = frame_workload(args, split=other, cpu=False, steps=max(3, args.steps // 2),
                        warmup=min(args.warmup, 3))
    head["frame_other_split"] = dict(
        _brief(fo, ("value", "unit", "ms_per_step", "pairs_per_s", "kernel_ms", "units",
                    "algorithmic_lane_ops", "roofline")),
        workload=fo["config"]["workload"], split=other)
    rm = rangemin_workload(args, steps=max(5, args.steps), warmup=max(2, args.warmup))
    head["range_min"] = dict(_brief(rm, ("value", "unit", "ms_per_step", "kernel_ms", "roofline",
                                         "valu", "cpu_baseline")),
                             workload=rm["config"]["workload"])
    bt = batched_workload(args, steps=max(3, args.steps // 2), warmup=min(args.warmup, 2))
    head["batched"] = dict(_brief(bt, ("value", "unit", "ms_per_step", "kernel_ms", "pairs_per_s",
                                       "plain_launches", "units", "algorithmic_lane_ops",
                                       "roofline", "groups")),
                           workload=bt["config"]["workload"],
                           tuned_per_light_class=bt["config"]["tuned_per_light_class"])
    sv = served_workload(args)
    head["served"] = dict(_brief(sv, ("value", "unit", "saturation", "loads",
                                      "strict_fifo_admission_0.9", "plain_single_launches")),
                          workload=sv["config"]["workload"], overtake_ms=args.overtake_ms,
                          workers=args.inflight, max_batch_eyes=args.batch_eyes)
    return head


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="all",
                   choices=["all", "frame", "tiny", "rangemin", "batched", "served"])
    p.add_argument("--requests", type=int, default=300, help="served: requests per load")
    p.add_argument("--budget-gib", type=float, default=64.0, help="served: device arena")
    p.add_argument("--load-seconds", type=float, default=8.0,
                   help="served: seconds of arrivals per offered load")
    p.add_argument("--inflight", type=int, default=2, help="served: worker threads (launches in flight)")
    p.add_argument("--batch-eyes", type=int, default=1 << 16,
                   help="served: eyes per batch at most (a larger request runs alone)")
    p.add_argument("--overtake-ms", type=float, default=100.0,
                   help="served: a queued request that does not fit is passed over by later "
                        "ones until it has waited this long (0 = strict FIFO admission)")
    p.add_argument("--rmq", default="paper", choices=list(RMQ_METHODS),
                   help="range-minimum method: paper (bit-parallel flip-position selection, "
                        "default), direct, paper_full (sweeps as loops), paper_loop (pruned loops), "
                        "dyadic (aligned blocks, not the paper's), paper_no_reuse (frame only: "
                        "no inheritance of the parent's argmin)")
    p.add_argument("--split", default="pow2", choices=["radix", "pow2"],
                   help="hierarchy split rule of the headline (the default run also measures "
                        "the other): pow2 (left child = largest power of two below the length) "
                        "or radix (highest differing Morton bit, the library's default)")
    p.add_argument("--samples", type=int, default=1,
                   help="frame: samples per eye (rotation psi(n) per sample; fewer pixel rows)")
    p.add_argument("--weights", action="store_true", help="frame: also write 1/p per pair")
    p.add_argument("--epw", type=int, default=0,
                   help="eyes per wave: 0 = the library's choice by hierarchy size (1 for the "
                        "frame's 2^20 lights, 8 for the small case), else 1, 2, 4 or 8")
    p.add_argument("--stack", type=int, default=0,
                   help="LDS stack entries per wave: 0 = the library's choice (192 for one eye per wave)")
    p.add_argument("--traffic-kib", type=float, nargs=2, default=None,
                   metavar=("FETCH", "WRITE"),
                   help="FETCH_SIZE and WRITE_SIZE (KiB per launch) of the traversal kernel "
                        "from rocprofv3 --pmc runs, already scaled by the copy-kernel factors")
    p.add_argument("--cpu-eyes", type=int, default=3072,
                   help="frame: eyes in the oracle's timed sample (about 10 s on 16 threads)")
    p.add_argument("--cpu-queries", type=int, default=65536,
                   help="rangemin: queries in the oracle's timed sample (about 6 s on 16 threads)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    args = p.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sharded design is documented, not built)", file=sys.stderr)
        sys.exit(2)
    fn = {"all": all_workloads, "frame": frame_workload, "tiny": frame_workload,
          "rangemin": rangemin_workload, "batched": batched_workload,
          "served": served_workload}[args.workload]
    line = fn(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
