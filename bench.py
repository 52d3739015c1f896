#!/usr/bin/env python3
"""Benchmark: windowed out-of-order kernel scheduling on one MI355X.

Workload (one "step" of this benchmark = one episode): a synthetic rigid-body
RL scene of 64 spheres advanced 200 physics steps.  Each physics step is an
input-dependent kernel graph (predict, broadphase, islands, permute, then
8 Jacobi iterations x one kernel per multi-body island, then integrate),
about 85 kernels; the island list is read back from the device every step.
Inputs are seeded and synthetic (they stand in for the paper's Brax
environments, which are not available here).

Paths timed on the same episodes:
  device              the persistent scheduler kernel (headline `value`); the
                      dependency checks run in a wave ahead of the window,
                      against the last 64 kernels (the host/device split made
                      inside the device), the window wave only filtering
  device_windowcheck  the same kernel with the checks made by the window wave
                      at insert
  device_hostcheck    the same kernel with the checks made on the host
                      against its list of the last W kernels
  inorder           every kernel launched into one HIP stream (the baseline)
  plain             host-side window + pool of HIP streams

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

# HBM traffic of one persistent-kernel launch (one episode of the default
# workload), from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per
# dispatch) scaled by the same counters' reading on a device-to-device copy of
# known size (--copy-calibration).  Valid only for the kernel sources whose
# digest is recorded: any change to them makes the figure stale (null).
TRAFFIC = {"digest": "15e0b3568c656847", "workload": (64, 200, 32, 1),
           "fetch_kib": 10562.0625, "write_kib": 9951.34375,
           "copy_bytes": 268435456, "copy_fetch_kib": 131085.16666666666, "copy_write_kib": 262144.0}
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


def traffic_bytes(args):
    """Calibrated HBM bytes per launch, or None when not measured for these
    sources or for this workload (bodies, physics steps, window, seed)."""
    if TRAFFIC is None or TRAFFIC["digest"] != kernel_digest():
        return None
    if TRAFFIC["workload"] != (args.bodies, args.physics_steps, args.window, args.seed):
        return None
    # bytes per counter unit, from the copy that moved copy_bytes each way
    bf = TRAFFIC["copy_bytes"] / TRAFFIC["copy_fetch_kib"]
    bw = TRAFFIC["copy_bytes"] / TRAFFIC["copy_write_kib"]
    return int(TRAFFIC["fetch_kib"] * bf + TRAFFIC["write_kib"] * bw)


def copy_calibration(torch):
    """Device-to-device copies of a known size, for scaling the PMC byte counters."""
    n = 64 << 20                                   # 64 Mi floats = 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copies": 3, "digest": kernel_digest()}), flush=True)


def algorithmic_bytes(counts: dict, n: int) -> int:
    """Bytes each kernel must move at least once (inputs read, outputs written),
    summed over an episode.  Per physics step with E directed contact edges,
    I islands and m multi-body islands:
      predict 48n, broadphase 24n+4+4E, islands 20n+24+8E+4(I+1)+16m,
      permute 36n, integrate 84n;
    per Jacobi kernel over an island of b bodies and e edges: 36b+4+4e."""
    steps = counts["steps"]
    fixed = steps * (212 * n + 28) + 12 * counts["edges"] + 4 * (counts["islands"] + steps) \
        + 16 * counts["multi_islands"]
    jac = 36 * counts["jacobi_bodies"] + 4 * counts["jacobi_kernels"] + 4 * counts["jacobi_edges"]
    return int(fixed + jac)


def open_window(acs, path, W, **kw):
    """`device_windowcheck`: the device path with the dependency checks made
    by the window wave; `device_hostcheck` is the device path with them on
    the host (a scheduled list of the last W kernels) instead of the window wave."""
    if path == "device_hostcheck":
        return acs.Window(W, path="device", host_check_depth=W, **kw)
    if path == "device_windowcheck":
        return acs.Window(W, path="device", window_check=1, **kw)
    return acs.Window(W, path=path, **kw)


def run_path(acs, inputs, torch, path, args, n_episodes, collect):
    """Runs n_episodes fresh episodes; returns (seconds, kernels, step_ns list,
    kernel_ns list, counts, overlap tests per kernel)."""
    scenes = [acs.RLSceneGPU(inputs.rl_scene(seed=args.seed, n=args.bodies)) for _ in range(n_episodes)]
    torch.cuda.synchronize()
    kernels = 0
    step_ns, kern_ns, counts = [], [], None
    tests = 0
    if path == "graph_per_input":
        build = 0.0
        t0 = time.perf_counter()
        for g in scenes:
            c, ns, b = acs.rl_run_graphs(g, args.physics_steps)
            kernels += c["kernels"]
            build += b
            if collect:
                step_ns.extend(ns.tolist())
            counts = c
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, kernels, step_ns, [build * 1e-9 / dt], counts, 0.0
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


def overhead_probe(acs, path, n, chain):
    w = open_window(acs, path, 32)
    ns = acs.nop_run(w, n, chain)
    w.destroy()
    return ns / n / 1000.0


def cpu_baseline(inputs, args):
    from oracle import oracle as O
    sc = inputs.rl_scene(seed=args.seed, n=args.bodies)
    kernels, episodes = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < args.cpu_seconds:
        s = O.Scene.from_inputs(sc)
        for _ in range(args.physics_steps):
            s.step()
            kernels += 5 + s.c.iters * s.n_multi
        episodes += 1
    dt = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": kernels / dt, "unit": "kernels/s", "cores": 1, "kind": "oracle",
            "host": f"{os.cpu_count()} logical CPUs visible, {model}",
            "sample": f"{episodes} episodes of {args.physics_steps} steps x {args.bodies} spheres "
                      f"({kernels} kernels, {dt:.1f} s, single thread, program order)"}


def batched_section(acs, inputs, torch, args):
    """Batched scenes: autotune, then time the tuned device path and the
    in-order stream on fresh copies of the same scenes."""
    import numpy as np
    from paper_2401_12377_amd import tune
    scenes = inputs.batched_scenes(3, args.batch_scenes)
    log(f"[bench] batched: autotuning over {args.batch_scenes} scenes")
    best, table = tune.autotune(scenes, steps=1, log=log, wg=(1, 2))
    res = {}
    finals = {}
    for path, cfg in (("device", best), ("inorder", {"W": 8, "n_groups": 1, "wg_per_task": 1, "queue_depth": 4096})):
        gpu = [acs.RLSceneGPU(sc) for sc in scenes]
        torch.cuda.synchronize()
        with acs.Window(cfg["W"], path=path, n_groups=cfg["n_groups"], wg_per_task=cfg["wg_per_task"],
                        queue_depth=cfg["queue_depth"], host_check_depth=cfg.get("host_check_depth", 0),
                        window_check=cfg.get("window_check", 0)) as w:
            t0 = time.perf_counter()
            counts, step_ns = acs.rl_run_batch(w, gpu, args.batch_steps, n_groups=cfg["n_groups"])
            dt = time.perf_counter() - t0
        res[path] = (counts["kernels"] / dt, np.array(step_ns) / 1e6, counts)
        finals[path] = [g.get(acs.RL_X) for g in gpu]
        log(f"[bench] batched {path}: {counts['kernels'] / dt / 1e3:.0f}k kernels/s")
    same = all(np.array_equal(a.view(np.uint32), b.view(np.uint32)) for a, b in zip(finals["device"], finals["inorder"]))
    dev, ino = res["device"], res["inorder"]
    return {"workload": f"{args.batch_scenes} independent scenes, 16-512 bodies log-uniform, {args.batch_steps} steps, "
                        "one persistent launch",
            "kernels": dev[2]["kernels"], "kernels_per_s": dev[0], "inorder_kernels_per_s": ino[0],
            "speedup_vs_inorder": dev[0] / ino[0],
            "batched_step_ms": {"p50": float(np.percentile(dev[1], 50)), "p99": float(np.percentile(dev[1], 99))},
            "inorder_batched_step_ms": {"p50": float(np.percentile(ino[1], 50)), "p99": float(np.percentile(ino[1], 99))},
            "tuned": best, "candidates": len(table), "device_equals_inorder": bool(same)}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed episodes per path")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--physics-steps", type=int, default=200)
    ap.add_argument("--bodies", type=int, default=64)
    ap.add_argument("--window", type=int, default=32)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    # graph_per_input (each step's graph rebuilt, run and destroyed) is not in
    # the default set: its process has ended with a host-side segmentation
    # fault inside that loop in two runs (no GPU fault reported; other runs of
    # the same loop completed) and no cause has been found in this code
    ap.add_argument("--paths", default="device,device_windowcheck,device_hostcheck,inorder,plain,events")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-scenes section")
    ap.add_argument("--batch-scenes", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-dnn", action="store_true", help="skip the dynamic-DNN section")
    ap.add_argument("--dnn-inputs", type=int, default=64)
    ap.add_argument("--no-dag", action="store_true", help="skip the static-network section")
    ap.add_argument("--dag-inputs", type=int, default=32)
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
    res = {}
    for path in paths:
        log(f"[bench] {path}: warmup {args.warmup} episodes")
        run_path(acs, inputs, torch, path, args, args.warmup, False)
        log(f"[bench] {path}: timing {args.steps} episodes")
        res[path] = run_path(acs, inputs, torch, path, args, args.steps, True)
        dt, k = res[path][0], res[path][1]
        log(f"[bench] {path}: {dt * 1e3 / args.steps:.2f} ms/episode, {k / dt:.0f} kernels/s")

    dev = res["device"]
    dt, kernels, step_ns, kern_ns, counts, _ = dev
    value = kernels / dt
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rigid-body RL step, {args.bodies} spheres x {args.physics_steps} steps, "
                               f"W={args.window}, device-resident path",
                   "bodies": args.bodies, "physics_steps": args.physics_steps, "window": args.window,
                   "kernels_per_episode": counts["kernels"], "parallelism": "single GPU",
                   "dependency_checks": "check waves ahead of the window (default for one window)"},
    }
    if "inorder" in res:
        out["speedup_vs_inorder"] = res["inorder"][0] / dt
        out["inorder_kernels_per_s"] = res["inorder"][1] / res["inorder"][0]
    if "device_windowcheck" in res:
        wc = res["device_windowcheck"]
        out["window_wave_checks"] = {"kernels_per_s": wc[1] / wc[0], "vs_check_wave": dt / wc[0]}
    if "device_hostcheck" in res:
        hc = res["device_hostcheck"]
        out["host_check_split"] = {"kernels_per_s": hc[1] / hc[0], "vs_device_checks": dt / hc[0],
                                   "host_overlap_tests_per_kernel": hc[5]}
    if "events" in res:
        out["events_kernels_per_s"] = res["events"][1] / res["events"][0]
    if "graph_per_input" in res:
        gp = res["graph_per_input"]
        out["graph_per_input"] = {"kernels_per_s": gp[1] / gp[0], "build_fraction": gp[3][0]}
    if "plain" in res:
        out["plain_kernels_per_s"] = res["plain"][1] / res["plain"][0]
        out["plain_speedup_vs_inorder"] = res["inorder"][0] / res["plain"][0] if "inorder" in res else None
    sn = np.array(step_ns) / 1e6
    out["graph_latency_ms"] = {"p50": float(np.percentile(sn, 50)), "p99": float(np.percentile(sn, 99)),
                               "graph": "one physics step"}
    for p in res:
        sp = np.array(res[p][2]) / 1e6
        out.setdefault("graph_latency_ms_by_path", {})[p] = {"p50": float(np.percentile(sp, 50)),
                                                             "p99": float(np.percentile(sp, 99))}
    # roofline of the dominant (only) kernel of the device path: the persistent kernel
    kns = float(np.mean(kern_ns))
    bytes_per_launch = algorithmic_bytes(counts, args.bodies)
    achieved = bytes_per_launch / kns   # bytes per ns = GB/s
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(args),
                       "kernel": "k_persistent", "launch_ms": kns / 1e6, "bytes_per_launch": bytes_per_launch,
                       "kernel_digest": kernel_digest()}
    if not args.no_probe:
        log("[bench] overhead probes")
        probes = {}
        for p in paths:
            if p == "graph_per_input":
                continue
            probes[p] = {"independent_us_per_kernel": overhead_probe(acs, p, 20000 if p.startswith("device") else 4000,
                                                                     False),
                         "chain_us_per_kernel": overhead_probe(acs, p, 2000, True)}
        out["overhead_us_per_kernel"] = probes
    if not args.no_batch:
        out["batched"] = batched_section(acs, inputs, torch, args)
    if not args.no_dnn:
        out["dnn"] = dnn_section(acs, inputs, torch, args)
    if not args.no_dag:
        out["static_dag"] = dag_section(acs, inputs, torch, args)
    if not args.no_serve:
        out["serving"] = serve_section(acs, inputs, torch, args)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline ({args.cpu_seconds:.0f} s of oracle)")
        out["cpu_baseline"] = cpu_baseline(inputs, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
