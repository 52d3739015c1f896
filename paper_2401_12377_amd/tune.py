"""Autotuner for batched task graphs: picks the window size W, the number
of window groups, the workgroups per splittable task and the input queue
depth for a set of independent scenes by timing short runs of each
candidate on the device path.

Each candidate runs on its own copy of the scenes (the tuning steps do not
advance the caller's scenes).  The search is exhaustive over (W, groups,
workgroups per task, where the dependency checks run) with W in {8, 16, 32,
48, 64} and groups * pow2(W) <= 64, then over the queue depth for the best
of those.  Windows wider than the 32 the paper evaluates are included
because a wider window exposes more independent kernels (Section VI-D).
Rates within 2% of the fastest count as equal, and the cheapest of those is
taken.  With one group the checks may run in the check wave ahead of the
window (the default), on the host against the last W kernels or the last 2W
(at most 128: a long kernel then holds back only the kernels more than 2W
after it), or in the window wave; with more groups always in the window
wave.
"""
from __future__ import annotations

import itertools
import time

from . import acs


def _pow2(x: int) -> int:
    p = 1
    while p < x:
        p <<= 1
    return p


CHECK_SITES = ("wave", "host", "host2", "window")


def _host_depth(W: int, site: str) -> int:
    if site == "host":
        return W
    if site == "host2":
        return min(2 * W, acs.HOST_CHECK_MAX)
    return 0


def candidates(windows=(8, 16, 32, 48, 64), groups=(1, 2, 4, 8), wg=(1, 2, 4), sites=CHECK_SITES):
    for W, G, g, site in itertools.product(windows, groups, wg, sites):
        if G * _pow2(W) > acs.W_MAX:
            continue
        if G > 1 and site != sites[0]:
            continue   # more than one group: the window wave checks, whatever is asked
        yield {"W": W, "n_groups": G, "wg_per_task": g, "queue_depth": 4096,
               "host_check_depth": _host_depth(W, site) if G == 1 else 0,
               "window_check": 1 if (G == 1 and site == "window") else 0}


def open_window(cfg: dict):
    return acs.Window(cfg["W"], path="device", n_groups=cfg["n_groups"], wg_per_task=cfg["wg_per_task"],
                      queue_depth=cfg["queue_depth"], host_check_depth=cfg.get("host_check_depth", 0),
                      window_check=cfg.get("window_check", 0))


def time_config(scenes, cfg: dict, steps: int = 2, warmup: int = 1) -> float:
    """kernels/s of `steps` batched steps of fresh copies of `scenes` (RLScene
    inputs) under cfg, after `warmup` untimed steps."""
    import torch
    gpu = [acs.RLSceneGPU(sc) for sc in scenes]
    torch.cuda.synchronize()
    with open_window(cfg) as w:
        if warmup:
            acs.rl_run_batch(w, gpu, warmup, n_groups=cfg["n_groups"])
        t0 = time.perf_counter()
        counts, _ = acs.rl_run_batch(w, gpu, steps, n_groups=cfg["n_groups"])
        dt = time.perf_counter() - t0
    return counts["kernels"] / dt


def pick(table, tie: float = 0.0) -> dict:
    """The fastest configuration of `table`; among those within a fraction
    `tie` of it (timing noise), the one with the fewest workgroups per task,
    then groups, then the shortest input queue, then the fastest."""
    top = max(v for _, v in table)
    close = [(c, v) for c, v in table if v >= (1.0 - tie) * top]
    return dict(min(close, key=lambda t: (t[0]["wg_per_task"], t[0]["n_groups"], t[0]["queue_depth"], -t[1]))[0])


def autotune(scenes, steps: int = 2, log=None, timer=None, tie: float = 0.02, **space):
    """Returns (best config, table of (config, kernels/s)).  `timer(scenes,
    cfg, steps)` measures one candidate (time_config unless given); `tie` is
    the relative difference below which two rates count as equal (see pick)."""
    timer = timer or time_config
    table = []
    for cfg in candidates(**space):
        v = timer(scenes, cfg, steps)
        table.append((cfg, v))
        if log:
            log(f"[tune] {cfg}: {v / 1e3:.0f}k kernels/s")
    best = pick(table, tie)
    for qd in (256, 1024):
        cfg = dict(best, queue_depth=qd)
        v = timer(scenes, cfg, steps)
        table.append((cfg, v))
        if log:
            log(f"[tune] {cfg}: {v / 1e3:.0f}k kernels/s")
    best = pick([(c, v) for c, v in table if all(c[k] == best[k] for k in best if k != "queue_depth")], tie)
    return best, table
