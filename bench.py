#!/usr/bin/env python3
"""Benchmark: windowed out-of-order kernel scheduling on one MI355X.

Headline workload (one "step" = one batched run): 256 independent synthetic
rigid-body RL scenes of uneven size (16-512 spheres, log-uniform, constant
density), advanced 20 physics steps together through one persistent launch
of the device-resident scheduler.  Each physics step of a scene is an
input-dependent kernel graph (predict, broadphase, islands, permute, then 8
Jacobi iterations x one kernel per multi-body island, then integrate); the
island lists are read back per group of scenes.  The window size, window
groups, workgroups per task, where the dependency checks run and the input
queue depth are picked by the autotuner before the timed region.  Inputs are
seeded and synthetic: they stand in for the paper's Brax environments, which
are not available here.

`value` is kernels/s of the tuned device path on that workload; beside it the
in-order single stream on the same scenes (`speedup_vs_inorder`), the roofline
of the persistent kernel's launch, the oracle on the host cores (one core and
all cores) and further sections: the 64-sphere episode on every path
(`rl64`), per-kernel overhead probes, the dynamic and the static network, a
window-size sweep, the host dependency-check cost table and serving.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one persistent-kernel launch of the headline workload, from
# two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) scaled
# by the same counters' reading on a device-to-device copy of known size
# (--copy-calibration), one entry per tuned configuration that was measured.
# Valid only for the kernel sources whose digest is recorded and for the same
# workload and configuration: any change makes the figure stale (null).
def _cfg_key(qd, hc=64):
    return (256, 20, json.dumps({"W": 64, "n_groups": 1, "wg_per_task": 1, "queue_depth": qd,
                                 "host_check_depth": hc, "window_check": 0}, sort_keys=True))


TRAFFIC = {
    "digest": "65488b41e62ec398",
    "copy_bytes": 268435456, "copy_fetch_kib": 131085.2917, "copy_write_kib": 262144.0,
    "runs": [{"workload": _cfg_key(256), "fetch_kib": 318555.75, "write_kib": 587168.3125},
             {"workload": _cfg_key(1024), "fetch_kib": 320026.9375, "write_kib": 586719.25},
             {"workload": _cfg_key(256, 128), "fetch_kib": 323091.25, "write_kib": 587344.28125},
             {"workload": _cfg_key(1024, 128), "fetch_kib": 323495.75, "write_kib": 586999.78125}],
}
KERNEL_SOURCES = ["kernels.hip", "persistent.hpp", "bodies.hpp", "dev_shared.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2401_12377_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_calibration(torch):
    """Device-to-device copies of a known size, for scaling the PMC byte counters."""
    n = 64 << 20                                   # 64 Mi floats = 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copies": 3, "digest": kernel_digest()}), flush=True)


def open_window(acs, path, W, **kw):
    """`device_windowcheck`: the device path with the dependency checks made
    by the window wave; `device_hostcheck` is the device path with them on
    the host (a scheduled list of the last W kernels) instead of the window wave."""
    if path == "device_hostcheck":
        return acs.Window(W, path="device", host_check_depth=W, **kw)
    if path == "device_windowcheck":
        return acs.Window(W, path="device", window_check=1, **kw)
    return acs.Window(W, path=path, **kw)


def overhead_probe(acs, path, n, chain):
    w = open_window(acs, path, 32)
    ns = acs.nop_run(w, n, chain)
    w.destroy()
    return ns / n / 1000.0


def dnn_section(acs, inputs, torch, args):
    """Dynamic DNN, batch 1: per-inference latency on each path, and
    throughput with many inferences in one window."""
    import numpy as np
    wts = inputs.dnn_weights()
    seeds = list(range(args.dnn_inputs))
    out = {}
    for path in ("device", "device_windowcheck", "device_hostcheck", "inorder", "events"):
        nets = [acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES) for _ in range(8)]
        lat = []
        kernels = 0
        with open_window(acs, path, 16) as w:
            for i, sd in enumerate(seeds):
                inp = inputs.dnn_input(sd)
                net = nets[i % len(nets)]
                net.set_input(inp.x)
                t0 = time.perf_counter()
                kernels += acs.dnn_submit(w, net, inp.logits)
                w.sync()
                lat.append(time.perf_counter() - t0)
            # throughput: inferences submitted back to back, 8 at a time in flight
            for net in nets:
                net.set_input(inputs.dnn_input(0).x)
            t0 = time.perf_counter()
            k2 = 0
            for i, sd in enumerate(seeds):
                k2 += acs.dnn_submit(w, nets[i % len(nets)], inputs.dnn_input(sd).logits)
                if i % len(nets) == len(nets) - 1:
                    w.sync()
            w.sync()
            dt = time.perf_counter() - t0
        lat = np.array(lat[2:]) * 1e3
        out[path] = {"latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                     "kernels_per_s": k2 / dt, "inferences_per_s": len(seeds) / dt}
        log(f"[bench] dnn {path}: p50 {out[path]['latency_ms']['p50']:.3f} ms, {len(seeds) / dt:.0f} inferences/s")
    # The graph rebuilt for every input is not measured here: the rebuild
    # loop's process has ended with a host-side segmentation fault (see the
    # --paths option) and no cause has been found in this code.
    out["graph_per_input"] = None
    # steady state: the network with every branch on (a static graph),
    # recorded once and replayed as a HIP graph, against the window paths
    import numpy as np
    static = np.ones((len(inputs.DNN_CELLS), 2), np.float32)
    steady = {}
    net = acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    net.set_input(inputs.dnn_input(0).x)
    with acs.Window(16, path="inorder") as w:
        w.graph_begin()
        acs.dnn_submit(w, net, static)
        g = w.graph_end()
    with g:
        g.launch()
        g.sync()
        lat = []
        for _ in seeds:
            t0 = time.perf_counter()
            g.launch()
            g.sync()
            lat.append(time.perf_counter() - t0)
        lat = np.array(lat) * 1e3
        steady["graph"] = {"latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                           "edges": g.info()["edges"], "kernels": g.info()["kernels"]}
    for path in ("device", "inorder"):
        with acs.Window(16, path=path) as w:
            acs.dnn_submit(w, net, static)
            w.sync()
            lat = []
            for _ in seeds:
                t0 = time.perf_counter()
                acs.dnn_submit(w, net, static)
                w.sync()
                lat.append(time.perf_counter() - t0)
        lat = np.array(lat) * 1e3
        steady[path] = {"latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}
    log(f"[bench] dnn steady state p50: graph {steady['graph']['latency_ms']['p50']:.3f} ms, device "
        f"{steady['device']['latency_ms']['p50']:.3f} ms, inorder {steady['inorder']['latency_ms']['p50']:.3f} ms")
    return {"workload": f"gated 12-cell conv network, batch 1, {len(seeds)} inputs, W=16",
            "steady_state": dict(steady, workload="every branch on (static graph), replayed"),
            "by_path": out, "device": out["device"], "inorder": out["inorder"],
            "latency_speedup_p50": out["inorder"]["latency_ms"]["p50"] / out["device"]["latency_ms"]["p50"],
            "throughput_speedup": out["device"]["inferences_per_s"] / out["inorder"]["inferences_per_s"]}


def serve_section(acs, inputs, torch, args):
    """Serving: an open-loop Poisson stream of mixed requests (RL scene steps,
    DNN inferences) at several arrival rates through one open window per
    run; latency = completion seen by the host minus arrival."""
    import numpy as np
    rates = [float(r) for r in args.serve_rates.split(",")]
    n = args.serve_requests
    specs0 = inputs.serve_requests(seed=4, rate_per_s=rates[0], n_requests=n)
    rl = {s.seed: inputs.rl_scene(seed=s.seed, n=s.n) for s in specs0 if s.kind == inputs.SERVE_RL}
    dnn = {s.seed: inputs.dnn_input(s.seed) for s in specs0 if s.kind == inputs.SERVE_DNN}
    net = acs.DNNGPU(inputs.dnn_weights(), inputs.DNN_CELLS, inputs.DNN_CLASSES)
    pool = torch.empty(args.serve_pool_mib << 20, dtype=torch.uint8, device="cuda")
    host = acs.serve_host(args.serve_resident)
    # (path, W, groups, host-check depth, window wave checks)
    configs = [("device", 32, 1, 0, 0), ("device", 32, 1, 0, 1), ("device", 32, 1, 32, 0), ("device", 16, 4, 0, 0),
               ("device", 8, 8, 0, 0), ("inorder", 8, 1, 0, 0)]
    table = {}
    outputs = {}
    for path, W, G, hc, wc in configs:
        key = (f"{path}_W{W}_G{G}" + ("_hostcheck" if hc else "") + ("_windowcheck" if wc else "")
               if path == "device" else path)
        rows = []
        for lam in rates:
            specs = inputs.serve_requests(seed=4, rate_per_s=lam, n_requests=n)
            sset = acs.ServeSet(specs, rl, dnn, inputs.DNN_CLASSES)
            with acs.Window(W, path=path, n_groups=G, host_check_depth=hc, window_check=wc) as w:
                res, st = acs.serve_run(w, sset, pool, host, max_resident=args.serve_resident, model=net,
                                        stall_ns=60 * 10 ** 9)
            lat = np.array([r["done_ns"] - s.arrival_ns for r, s in zip(res, specs)]) / 1e6
            kinds = np.array([s.kind for s in specs])
            row = {"rate_per_s": lam, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "mean_ms": float(lat.mean()),
                   "p50_ms_rl": float(np.percentile(lat[kinds == inputs.SERVE_RL], 50)),
                   "p50_ms_dnn": float(np.percentile(lat[kinds == inputs.SERVE_DNN], 50)),
                   "requests_per_s": n / (st["wall_ns"] * 1e-9), "kernels_per_s": st["kernels"] / (st["wall_ns"] * 1e-9),
                   "kernels": st["kernels"], "peak_resident": st["peak_resident"],
                   "peak_pool_mib": st["peak_pool_bytes"] / 2 ** 20, "waited_memory": st["waited_memory"],
                   "waited_resident": st["waited_resident"]}
            rows.append(row)
            if lam == rates[len(rates) // 2]:
                outputs[key] = sset.outputs()
            log(f"[bench] serve {key} rate {lam:.0f}/s: p50 {row['p50_ms']:.3f} ms, p99 {row['p99_ms']:.3f} ms, "
                f"{row['requests_per_s']:.0f} req/s")
            del sset
        table[key] = rows

    def same(a, b):
        for x, y in zip(a, b):
            xs = x if isinstance(x, tuple) else (x,)
            ys = y if isinstance(y, tuple) else (y,)
            if not all(np.array_equal(u.view(np.uint32), v.view(np.uint32)) for u, v in zip(xs, ys)):
                return False
        return True
    ref = outputs["inorder"]
    return {"workload": f"{n} requests per rate, Poisson arrivals, half RL scene steps (16-512 bodies log-uniform) "
                        f"and half DNN inferences, pool {args.serve_pool_mib} MiB, at most {args.serve_resident} "
                        "in flight",
            "by_config": table,
            "results_equal_inorder": {k: same(v, ref) for k, v in outputs.items() if k != "inorder"}}


def dag_section(acs, inputs, torch, args):
    """Static irregular network (randomly wired, 32 nodes, batch 1): latency
    per inference on every path, the graph captured once and replayed, and
    the graph rebuilt for every input."""
    import numpy as np
    graph = inputs.dag_graph()
    wts = inputs.dag_weights(graph)
    xs = [inputs.dag_input(graph, s) for s in range(args.dag_inputs)]
    res = {}

    def summary(lat):
        lat = np.array(lat[2:]) * 1e3
        return {"latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}
    ref_out = None
    for path in ("device", "device_windowcheck", "device_hostcheck", "inorder", "events", "plain"):
        net = acs.DAGGPU(graph, wts)
        lat = []
        with open_window(acs, path, 16, n_streams=args.streams) as w:
            for x in xs:
                net.set_input(x)
                t0 = time.perf_counter()
                n = acs.dag_submit(w, net)
                w.sync()
                lat.append(time.perf_counter() - t0)
        res[path] = summary(lat)
        out = net.out.cpu().numpy()
        if ref_out is None:
            ref_out = out
        res[path]["last_output_equals_device"] = bool(np.array_equal(out.view(np.uint32), ref_out.view(np.uint32)))
        log(f"[bench] dag {path}: p50 {res[path]['latency_ms']['p50']:.3f} ms")
    # graph captured once, replayed per input
    net = acs.DAGGPU(graph, wts)
    with acs.Window(16, path="inorder") as w:
        w.graph_begin()
        acs.dag_submit(w, net)
        g = w.graph_end()
    with g:
        lat = []
        for x in xs:
            net.set_input(x)
            t0 = time.perf_counter()
            g.launch()
            g.sync()
            lat.append(time.perf_counter() - t0)
        res["graph_replay"] = summary(lat)
        res["graph_replay"]["edges"] = g.info()["edges"]
    log(f"[bench] dag graph_replay: p50 {res['graph_replay']['latency_ms']['p50']:.3f} ms")
    # The graph rebuilt for every input is not measured on this network: its
    # host process once ended with a segmentation fault inside that loop (no
    # GPU fault reported) and no cause has been found in this code; it is
    # measured on the RL episode and the dynamic network.
    res["graph_per_input"] = None
    base = res["inorder"]["latency_ms"]["p50"]
    return {"workload": f"randomly wired network, {len(graph.preds)} nodes (3x3 conv 32x32x32 each), batch 1, "
                        f"{n} kernels, {len(xs)} inputs, W=16",
            "by_path": res,
            "speedup_p50_vs_inorder": {k: base / v["latency_ms"]["p50"] for k, v in res.items() if v is not None}}



def traffic_bytes(workload_key):
    """Calibrated HBM bytes per launch, or None when not measured for these
    sources or for this workload and configuration."""
    if TRAFFIC is None or TRAFFIC["digest"] != kernel_digest():
        return None
    run = next((r for r in TRAFFIC["runs"] if r["workload"] == workload_key), None)
    if run is None:
        return None
    # bytes per counter unit, from the copy that moved copy_bytes each way
    bf = TRAFFIC["copy_bytes"] / TRAFFIC["copy_fetch_kib"]
    bw = TRAFFIC["copy_bytes"] / TRAFFIC["copy_write_kib"]
    return int(run["fetch_kib"] * bf + run["write_kib"] * bw)


def algorithmic_bytes(counts: dict, sizes, steps: int) -> int:
    """Bytes each kernel must move at least once (inputs read, outputs written),
    summed over every scene and physics step.  Per scene step with n bodies,
    E directed contact edges, I islands and m multi-body islands:
      predict 48n, broadphase 24n+4+4E, islands 20n+24+8E+4(I+1)+16m,
      permute 36n, integrate 84n;
    per Jacobi kernel over an island of b bodies and e edges: 36b+4+4e."""
    fixed = steps * sum(212 * int(n) + 28 for n in sizes) + 12 * counts["edges"] \
        + 4 * (counts["islands"] + counts["steps"]) + 16 * counts["multi_islands"]
    jac = 36 * counts["jacobi_bodies"] + 4 * counts["jacobi_kernels"] + 4 * counts["jacobi_edges"]
    return int(fixed + jac)


def open_batched(acs, cfg, path="device"):
    return acs.Window(cfg["W"], path=path, n_groups=cfg["n_groups"], wg_per_task=cfg["wg_per_task"],
                      queue_depth=cfg["queue_depth"], host_check_depth=cfg.get("host_check_depth", 0),
                      window_check=cfg.get("window_check", 0))


def headline(acs, inputs, torch, args):
    """The batched workload: autotune (untimed), then `warmup` + `steps`
    batched runs of the tuned device path, each a fresh copy of the scenes in
    its own persistent launch; then the in-order stream on the same scenes."""
    import numpy as np
    from paper_2401_12377_amd import tune
    scenes = inputs.batched_scenes(3, args.batch_scenes)
    sizes = [sc.n for sc in scenes]
    if args.config:
        best, table = json.loads(args.config), []
    else:
        log(f"[bench] headline: autotuning over {args.batch_scenes} scenes")
        best, table = tune.autotune(scenes, steps=1, log=log, wg=(1, 2))
    log(f"[bench] headline: tuned {best}")
    runs = []
    final = None
    for i in range(args.warmup + args.steps):
        gpu = [acs.RLSceneGPU(sc) for sc in scenes]
        torch.cuda.synchronize()
        w = open_batched(acs, best)
        t0 = time.perf_counter()
        counts, step_ns = acs.rl_run_batch(w, gpu, args.batch_steps, n_groups=best["n_groups"])
        dt = time.perf_counter() - t0
        w.stop()
        st = w.stats()
        w.destroy()
        if i >= args.warmup:
            runs.append((dt, counts, st["kernel_ns"], np.array(step_ns)))
        final = [g.get(acs.RL_X) for g in gpu]
        log(f"[bench] headline run {i}: {dt * 1e3:.1f} ms, {counts['kernels'] / dt / 1e3:.0f}k kernels/s")
    # the single-stream baseline on the same scenes
    ino = []
    same = None
    if not args.no_inorder:
        gpu = [acs.RLSceneGPU(sc) for sc in scenes]
        torch.cuda.synchronize()
        with acs.Window(8, path="inorder") as w:
            t0 = time.perf_counter()
            c_in, _ = acs.rl_run_batch(w, gpu, args.batch_steps)
            ino.append((time.perf_counter() - t0, c_in))
        same = all(np.array_equal(a.view(np.uint32), g.get(acs.RL_X).view(np.uint32)) for a, g in zip(final, gpu))
        log(f"[bench] headline in-order: {c_in['kernels'] / ino[0][0] / 1e3:.0f}k kernels/s")
    return {"scenes": scenes, "sizes": sizes, "tuned": best, "candidates": len(table), "runs": runs,
            "inorder": ino, "device_equals_inorder": None if same is None else bool(same)}


def run_path(acs, inputs, torch, path, args, n_episodes, collect):
    """64-sphere episodes on one path; returns (seconds, kernels, step_ns
    list, kernel_ns list, counts, overlap tests per kernel)."""
    scenes = [acs.RLSceneGPU(inputs.rl_scene(seed=args.seed, n=args.bodies)) for _ in range(n_episodes)]
    torch.cuda.synchronize()
    kernels = 0
    step_ns, kern_ns, counts = [], [], None
    tests = 0
    t0 = time.perf_counter()
    for g in scenes:
        w = open_window(acs, path, args.window, n_streams=args.streams, wg_per_task=1)
        c, ns = acs.rl_run(w, g, args.physics_steps)
        w.stop()
        st = w.stats()
        w.destroy()
        kernels += c["kernels"]
        tests += st["overlap_tests"]
        if collect:
            step_ns.extend(ns.tolist())
            kern_ns.append(st["kernel_ns"])
        counts = c
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, kernels, step_ns, kern_ns, counts, tests / max(1, kernels)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(inputs, args):
    """The oracle (program order, one kernel after the other) on the
    headline's scenes and physics steps, repeated for about cpu_seconds:
    once on one thread, once with the scenes spread over every host core
    (each scene's kernels still in program order on one thread)."""
    import concurrent.futures as cf
    from oracle import oracle as O
    scenes = inputs.batched_scenes(3, args.batch_scenes)

    def one(sc):
        s = O.Scene.from_inputs(sc)
        k = 0
        for _ in range(args.batch_steps):
            s.step()
            k += 5 + s.c.iters * s.n_multi
        return k

    res = {}
    threads = os.cpu_count() or 1
    for label, nt in (("single", 1), ("all", threads)):
        kernels, reps = 0, 0
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(nt) as ex:
            while time.perf_counter() - t0 < args.cpu_seconds / 2 or reps == 0:
                kernels += sum(ex.map(one, scenes)) if nt > 1 else sum(map(one, scenes))
                reps += 1
        dt = time.perf_counter() - t0
        res[label] = (kernels / dt, kernels, dt, reps, nt)
    v1, k1, d1, r1, _ = res["single"]
    va, ka, da, ra, nt = res["all"]
    host = f"{threads} logical CPUs visible, {cpu_model()}"
    sample = (f"the headline workload ({args.batch_scenes} scenes x {args.batch_steps} physics steps) run {ra} times "
              f"({ka} kernels, {da:.1f} s); scenes spread over {nt} threads, each scene in program order")
    return {"value": va, "unit": "kernels/s", "cores": nt, "kind": "oracle", "sample": sample, "host": host,
            "single_core": {"value": v1, "unit": "kernels/s", "cores": 1, "kind": "oracle",
                            "sample": f"same workload run {r1} times ({k1} kernels, {d1:.1f} s), one thread"}}


def window_sweep(acs, inputs, torch, args):
    """Window size W in {8, 16, 32, 64} (Section VI-D) on the tiny random stream
    (latency of one 64-kernel stream), the 64-sphere episode (kernels/s) and
    the dynamic network (latency of one inference), device path."""
    import numpy as np
    out = {}
    st = inputs.tiny_stream(0)
    for W in (8, 16, 32, 64):
        arena = torch.from_numpy(st.init.copy()).cuda()
        torch.cuda.synchronize()
        lat = []
        with acs.Window(W, path="device") as w:
            for r in range(22):
                arena.copy_(torch.from_numpy(st.init))
                torch.cuda.current_stream().synchronize()
                t0 = time.perf_counter()
                acs.submit_tiny_stream(w, st, arena.data_ptr())
                w.sync()
                lat.append(time.perf_counter() - t0)
        lat = np.array(lat[2:]) * 1e3
        out.setdefault("tiny_stream_latency_ms_p50", {})[W] = float(np.percentile(lat, 50))
        g = acs.RLSceneGPU(inputs.rl_scene(seed=args.seed, n=args.bodies))
        torch.cuda.synchronize()
        with acs.Window(W, path="device") as w:
            t0 = time.perf_counter()
            c, _ = acs.rl_run(w, g, args.physics_steps)
            dt = time.perf_counter() - t0
        out.setdefault("rl64_kernels_per_s", {})[W] = c["kernels"] / dt
        wts = inputs.dnn_weights()
        net = acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES)
        lat = []
        with acs.Window(W, path="device") as w:
            for sd in range(24):
                inp = inputs.dnn_input(sd)
                net.set_input(inp.x)
                t0 = time.perf_counter()
                acs.dnn_submit(w, net, inp.logits)
                w.sync()
                lat.append(time.perf_counter() - t0)
        lat = np.array(lat[4:]) * 1e3
        out.setdefault("dnn_latency_ms_p50", {})[W] = float(np.percentile(lat, 50))
        log(f"[bench] window sweep W={W}: tiny {out['tiny_stream_latency_ms_p50'][W]:.3f} ms, "
            f"rl64 {out['rl64_kernels_per_s'][W] / 1e3:.0f}k kernels/s, dnn {out['dnn_latency_ms_p50'][W]:.3f} ms")
    return out


def profile_case(acs, inputs, torch, args):
    """A short fixed run of one small workload on the device path (one
    persistent launch) and then on the in-order stream, for counter runs:
    the tiny random stream (64 kernels, W=8) 20 times, or the gated network
    (W=16) on 8 inputs."""
    for path in ("device", "inorder"):
        if args.profile_case == "tiny":
            st = inputs.tiny_stream(0)
            arena = torch.from_numpy(st.init.copy()).cuda()
            torch.cuda.synchronize()
            with acs.Window(8, path=path) as w:
                for _ in range(20):
                    acs.submit_tiny_stream(w, st, arena.data_ptr())
                    w.sync()
        else:
            net = acs.DNNGPU(inputs.dnn_weights(), inputs.DNN_CELLS, inputs.DNN_CLASSES)
            with acs.Window(16, path=path) as w:
                for sd in range(8):
                    inp = inputs.dnn_input(sd)
                    net.set_input(inp.x)
                    acs.dnn_submit(w, net, inp.logits)
                    w.sync()
        torch.cuda.synchronize()
        log(f"[bench] profile case {args.profile_case}: {path} done")


def check_cost(acs):
    """The host's dependency check per insert at W in {16, 32} and 6 or 10
    read/write segments (the overhead table of Section IV-D), and the device
    path's cost per independent kernel with that many segments (checks in the
    check waves, or on the host against the last W kernels)."""
    import ctypes as C
    L = acs.lib()
    L.acs_check_probe.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    L.acs_check_probe.restype = C.c_int
    host = {}
    for W in (16, 32):
        for S in (6, 10):
            a, b, t = C.c_double(), C.c_double(), C.c_double()
            rc = L.acs_check_probe(W, S, 100000, C.byref(a), C.byref(b), C.byref(t))
            if rc != 0:
                raise RuntimeError(f"acs_check_probe: {rc}")
            host[f"W{W}_segs{S}"] = {"check_ns": a.value - b.value, "insert_ns": a.value, "pair_tests": t.value}
    device = {}
    for W in (16, 32):
        for S in (6, 8):
            for mode, kw in (("check_wave", {}), ("host_check", {"host_check_depth": W})):
                w = acs.Window(W, path="device", **kw)
                ns = acs.nop_segs_run(w, 20000, S)
                w.destroy()
                device.setdefault(f"W{W}_segs{S}", {})[mode + "_us_per_kernel"] = ns / 20000 / 1e3
    return {"host": host, "device_independent_kernels": device,
            "note": "10 segments are merged to the 8 positions a kernel keeps (conservatively)"}

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed batched runs of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-scenes", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--config", default=None, help="tuned configuration as JSON (skips the autotuner)")
    ap.add_argument("--only-headline", action="store_true", help="the headline workload only (profiling runs)")
    ap.add_argument("--no-inorder", action="store_true",
                    help="skip the headline's in-order comparison (counter runs, where every dispatch is serialised)")
    ap.add_argument("--profile-case", choices=("tiny", "dnn"), default=None,
                    help="only run the tiny random stream or the gated network on the device and in-order paths "
                         "(occupancy runs)")
    ap.add_argument("--episodes", type=int, default=3, help="64-sphere episodes timed per path")
    ap.add_argument("--physics-steps", type=int, default=200)
    ap.add_argument("--bodies", type=int, default=64)
    ap.add_argument("--window", type=int, default=32)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rl64", action="store_true", help="skip the 64-sphere episode section")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--paths", default="device,device_windowcheck,device_hostcheck,inorder,plain,events")
    ap.add_argument("--no-dnn", action="store_true", help="skip the dynamic-DNN section")
    ap.add_argument("--dnn-inputs", type=int, default=64)
    ap.add_argument("--no-dag", action="store_true", help="skip the static-network section")
    ap.add_argument("--dag-inputs", type=int, default=32)
    ap.add_argument("--no-sweep", action="store_true", help="skip the window-size sweep")
    ap.add_argument("--no-check-cost", action="store_true", help="skip the dependency-check cost table")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000")
    ap.add_argument("--serve-pool-mib", type=int, default=256)
    ap.add_argument("--serve-resident", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device copies of known size (for PMC byte-counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the scheduler runs on a single MI355X; "
              "independent scenes would shard across GPUs with no communication", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2401_12377_amd import acs, inputs
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    acs.lib()
    if args.profile_case:
        profile_case(acs, inputs, torch, args)
        return
    paths = args.paths.split(",")
    if "graph_per_input" in paths:
        # Its host process has ended with a segmentation fault inside the
        # rebuild loop; the host code of that loop runs clean under the
        # address and undefined-behaviour sanitizers on the CPU (thousands of
        # steps with changing plans, tests/test_host_sanitize.py), so no cause
        # has been shown in this code and the case stays off the GPU.
        print("graph_per_input is switched off: its rebuild loop ended the process with a host-side "
              "segmentation fault and no cause has been found in this code", file=sys.stderr)
        sys.exit(2)

    # ---- headline: the batched scenes, tuned device path vs in-order stream
    hl = headline(acs, inputs, torch, args)
    runs = hl["runs"]
    dt = sum(r[0] for r in runs)
    kernels = sum(r[1]["kernels"] for r in runs)
    value = kernels / dt
    counts = runs[-1][1]
    kns = float(np.mean([r[2] for r in runs]))
    ino_rate = hl["inorder"][0][1]["kernels"] / hl["inorder"][0][0] if hl["inorder"] else None
    step_ms = np.concatenate([r[3] for r in runs]) / 1e6
    best = hl["tuned"]
    out = {
        "metric": "kernels/sec and end-to-end speedup vs in-order stream; p50/p99 graph latency",
        "value": value,
        "unit": "kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "speedup_vs_inorder": value / ino_rate if ino_rate else None,
        "inorder_kernels_per_s": ino_rate,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.batch_scenes} independent rigid-body RL scenes (16-512 spheres, log-uniform, "
                               f"constant density) x {args.batch_steps} physics steps, one persistent launch per step "
                               "of the benchmark, autotuned",
                   "scenes": args.batch_scenes, "physics_steps": args.batch_steps,
                   "bodies_total": int(sum(hl["sizes"])), "kernels_per_step": counts["kernels"],
                   "tuned": best, "candidates": hl["candidates"], "parallelism": "single GPU"},
        "graph_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                             "graph": f"one physics step of all {args.batch_scenes} scenes"},
        "device_equals_inorder": hl["device_equals_inorder"],
    }
    bytes_per_launch = algorithmic_bytes(counts, hl["sizes"], args.batch_steps)
    achieved = bytes_per_launch / kns   # bytes per ns = GB/s
    wkey = (args.batch_scenes, args.batch_steps, json.dumps(best, sort_keys=True))
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(wkey),
                       "kernel": f"k_persistent<{1 if best['n_groups'] <= 1 else (2 if best['n_groups'] <= 2 else (4 if best['n_groups'] <= 4 else 8))}>",
                       "launch_ms": kns / 1e6, "bytes_per_launch": bytes_per_launch, "kernel_digest": kernel_digest()}
    log(f"[bench] headline: {value / 1e3:.0f}k kernels/s, {out['speedup_vs_inorder'] or 0:.2f}x in-order, "
        f"launch {kns / 1e6:.1f} ms, {achieved:.3f} GB/s algorithmic")
    if args.only_headline:
        print(json.dumps(out), flush=True)
        return

    # ---- the 64-sphere episode on every path
    if not args.no_rl64:
        res = {}
        for path in paths:
            log(f"[bench] rl64 {path}: warmup")
            run_path(acs, inputs, torch, path, args, 1, False)
            res[path] = run_path(acs, inputs, torch, path, args, args.episodes, True)
            log(f"[bench] rl64 {path}: {res[path][1] / res[path][0] / 1e3:.0f}k kernels/s")
        rl = {"workload": f"rigid-body RL step, {args.bodies} spheres x {args.physics_steps} steps, W={args.window}",
              "kernels_per_episode": res[paths[0]][4]["kernels"], "by_path": {}}
        for p, r in res.items():
            sp = np.array(r[2]) / 1e6
            rl["by_path"][p] = {"kernels_per_s": r[1] / r[0], "step_ms": {"p50": float(np.percentile(sp, 50)),
                                                                          "p99": float(np.percentile(sp, 99))}}
            if p == "device_hostcheck":
                rl["by_path"][p]["host_overlap_tests_per_kernel"] = r[5]
        if "inorder" in res:
            base = res["inorder"][1] / res["inorder"][0]
            rl["speedup_vs_inorder"] = {p: v["kernels_per_s"] / base for p, v in rl["by_path"].items()}
        if "device" in res:
            d = res["device"]
            ab = algorithmic_bytes(d[4], [args.bodies], args.physics_steps)
            kn = float(np.mean(d[3]))
            rl["device_roofline"] = {"launch_ms": kn / 1e6, "bytes_per_launch": ab, "achieved_GBps": ab / kn,
                                     "frac": ab / kn / HBM_PEAK_GBS}
        out["rl64"] = rl
    if not args.no_probe:
        log("[bench] overhead probes")
        probes = {}
        for p in paths:
            probes[p] = {"independent_us_per_kernel": overhead_probe(acs, p, 20000 if p.startswith("device") else 4000,
                                                                     False),
                         "chain_us_per_kernel": overhead_probe(acs, p, 2000, True)}
        out["overhead_us_per_kernel"] = probes
    if not args.no_check_cost:
        log("[bench] dependency-check cost table")
        out["check_cost"] = check_cost(acs)
    if not args.no_sweep:
        out["window_sweep"] = window_sweep(acs, inputs, torch, args)
    if not args.no_dnn:
        out["dnn"] = dnn_section(acs, inputs, torch, args)
    if not args.no_dag:
        out["static_dag"] = dag_section(acs, inputs, torch, args)
    if not args.no_serve:
        out["serving"] = serve_section(acs, inputs, torch, args)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (about {args.cpu_seconds:.0f} s of oracle)")
        out["cpu_baseline"] = cpu_baseline(inputs, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
