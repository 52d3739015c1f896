"""Python binding of libacs (include/acs.h, acs_tasks.h, acs_workloads.h).

Argument marshalling only: every step of the scheduling path and every task
body runs inside libacs.so.  PyTorch is used for device memory.  Importing
works without a GPU; creating a GPU window needs the built library and a
device, and fails loudly otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libacs.so")

# ---------------------------------------------------------------------------
# constants mirrored from the headers
# ---------------------------------------------------------------------------
OK, EINVAL, ENOMEM, EAGAIN, EDEVICE, ETIMEDOUT, EKERNEL, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
PENDING, READY, EXECUTING = 0, 1, 2
PATH_INORDER, PATH_PLAIN, PATH_DEVICE, PATH_MANUAL, PATH_EVENTS = 0, 1, 2, 3, 4
PATHS = {"inorder": PATH_INORDER, "plain": PATH_PLAIN, "device": PATH_DEVICE, "manual": PATH_MANUAL,
         "events": PATH_EVENTS}
W_MAX, K_MAX, ARGS_MAX = 64, 8, 64
HOST_CHECK_MAX = 128   # longest host check list (acs_config.host_check_depth)
SEG_ALL = (0, (1 << 64) - 1)

K_NOP, K_SCALE, K_AXPY, K_SUM = 0, 1, 2, 3
K_RL_PREDICT, K_RL_BROADPHASE, K_RL_ISLANDS, K_RL_PERMUTE, K_RL_JACOBI, K_RL_INTEGRATE = 10, 11, 12, 13, 14, 15
K_CONV, K_JOIN, K_AVGPOOL, K_FC = 20, 21, 22, 23
K_COPY, K_SIGNAL = 24, 25
SERVE_RL, SERVE_DNN = 0, 1
DNN_MAX_CELLS = 16

RL_X, RL_V, RL_P, RL_Q0, RL_Q1, RL_DEG, RL_ADJ_OFF, RL_ADJ, RL_LABEL, RL_PERM, RL_INV_PERM, RL_ISL_OFF, \
    RL_PADJ_OFF, RL_PADJ, RL_END = range(15)
RL_NREGIONS = 15


class AcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"acs error {code}: {msg}")
        self.code = code


class Seg(C.Structure):
    _fields_ = [("start", C.c_uint64), ("size", C.c_uint64)]


class Config(C.Structure):
    _fields_ = [("path", C.c_int32), ("n_streams", C.c_int32), ("wg_per_task", C.c_int32), ("n_workers", C.c_int32),
                ("queue_depth", C.c_int32), ("nonblocking", C.c_int32), ("trace", C.c_int32),
                ("trace_capacity", C.c_int32), ("device", C.c_int32), ("n_groups", C.c_int32),
                ("host_check_depth", C.c_int32), ("window_check", C.c_int32), ("reserved", C.c_int32 * 4)]


class Entry(C.Structure):
    _fields_ = [("seq", C.c_uint64), ("kernel_id", C.c_int32), ("state", C.c_int32), ("upstream_mask", C.c_uint64),
                ("slot", C.c_int32), ("reserved", C.c_int32)]


TRACE_DTYPE = np.dtype([("seq", np.int64), ("slot", np.int64), ("kid", np.int64),
                        ("ev_insert", np.int64), ("ev_dispatch", np.int64), ("ev_retire", np.int64),
                        ("valid_mask", np.uint64), ("up_mask", np.uint64),
                        ("t_start", np.int64), ("t_end", np.int64),
                        ("t_dispatch", np.int64), ("t_retire", np.int64)])


class Stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("retired", C.c_uint64), ("dispatched", C.c_uint64),
                ("coalesced", C.c_uint64), ("overlap_tests", C.c_uint64), ("poisoned", C.c_uint64),
                ("path", C.c_int32), ("W", C.c_int32), ("n_workers", C.c_int32), ("n_streams", C.c_int32),
                ("kernel_ns", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# task argument structs (acs_tasks.h)
class ArgsNop(C.Structure):
    _fields_ = [("spin_ns", C.c_uint64)]


class ArgsScale(C.Structure):
    _fields_ = [("out", C.c_uint64), ("x", C.c_uint64), ("a", C.c_float), ("n", C.c_uint32)]


class ArgsAxpy(C.Structure):
    _fields_ = [("out", C.c_uint64), ("x", C.c_uint64), ("y", C.c_uint64), ("a", C.c_float), ("n", C.c_uint32)]


class ArgsSum(C.Structure):
    _fields_ = [("out", C.c_uint64), ("ins", C.c_uint64 * 3), ("len", C.c_uint32 * 3), ("nin", C.c_uint32)]


class ArgsConv(C.Structure):
    _fields_ = [("inp", C.c_uint64), ("w", C.c_uint64), ("bias", C.c_uint64), ("out", C.c_uint64),
                ("hin", C.c_int32), ("cin", C.c_int32), ("cout", C.c_int32), ("k", C.c_int32), ("stride", C.c_int32)]


class ArgsJoin(C.Structure):
    _fields_ = [("out", C.c_uint64), ("a", C.c_uint64), ("b", C.c_uint64), ("n", C.c_uint32)]


class ArgsAvgpool(C.Structure):
    _fields_ = [("out", C.c_uint64), ("inp", C.c_uint64), ("hw", C.c_int32), ("c", C.c_int32)]


class ArgsFC(C.Structure):
    _fields_ = [("out", C.c_uint64), ("inp", C.c_uint64), ("w", C.c_uint64), ("bias", C.c_uint64),
                ("cin", C.c_int32), ("cout", C.c_int32)]


class DNNCellC(C.Structure):
    _fields_ = [("hin", C.c_int32), ("cin", C.c_int32), ("cout", C.c_int32), ("stride", C.c_int32),
                ("w3", C.c_uint64), ("b3", C.c_uint64), ("w1", C.c_uint64), ("b1", C.c_uint64),
                ("t3", C.c_uint64), ("t1", C.c_uint64), ("y", C.c_uint64)]


class DNNGraphC(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("classes", C.c_int32), ("x", C.c_uint64),
                ("cell", DNNCellC * DNN_MAX_CELLS), ("pool", C.c_uint64), ("fc_w", C.c_uint64),
                ("fc_b", C.c_uint64), ("out", C.c_uint64)]


class ArgsCopy(C.Structure):
    _fields_ = [("dst", C.c_uint64), ("src", C.c_uint64), ("bytes", C.c_uint64)]


class ArgsSignal(C.Structure):
    _fields_ = [("addr", C.c_uint64), ("value", C.c_uint64)]


class ServeRequestC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("iters", C.c_int32), ("r", C.c_float), ("dt", C.c_float),
                ("pad", C.c_int32), ("arrival_ns", C.c_double), ("input", C.c_uint64), ("output", C.c_uint64),
                ("logits", C.c_void_p)]


class ServeResultC(C.Structure):
    _fields_ = [("admit_ns", C.c_double), ("done_ns", C.c_double), ("kernels", C.c_uint64),
                ("footprint", C.c_uint64), ("group", C.c_int32), ("multi_islands", C.c_int32)]


class ServeConfigC(C.Structure):
    _fields_ = [("pool", C.c_uint64), ("pool_bytes", C.c_uint64), ("host", C.c_void_p), ("host_bytes", C.c_uint64),
                ("max_resident", C.c_int32), ("pad", C.c_int32),
                ("model", C.c_void_p), ("stall_ns", C.c_uint64)]


class ServeStatsC(C.Structure):
    _fields_ = [("wall_ns", C.c_double)] + [(f, C.c_uint64) for f in ("kernels", "peak_resident", "peak_pool_bytes",
                                                                       "waited_memory", "waited_resident")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


DAG_MAX_NODES, DAG_MAX_IN = 64, 8


class DAGNodeC(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("inp", C.c_int32 * DAG_MAX_IN), ("w", C.c_uint64), ("b", C.c_uint64),
                ("agg", C.c_uint64), ("y", C.c_uint64)]


class DAGGraphC(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("h", C.c_int32), ("c", C.c_int32), ("classes", C.c_int32),
                ("x", C.c_uint64), ("node", DAGNodeC * DAG_MAX_NODES), ("sink", C.c_uint64), ("pool", C.c_uint64),
                ("fc_w", C.c_uint64), ("fc_b", C.c_uint64), ("out", C.c_uint64)]


class ArgsRL(C.Structure):
    _fields_ = [("base", C.c_uint64), ("plan", C.c_uint64), ("n", C.c_int32), ("r", C.c_float), ("dt", C.c_float),
                ("iter", C.c_int32), ("b0", C.c_int32), ("b1", C.c_int32)]


class DeviceInfo(C.Structure):
    _fields_ = [("compute_units", C.c_int32), ("wall_clock_khz", C.c_int32), ("persistent_wg_per_cu", C.c_int32),
                ("runtime_version", C.c_int32), ("lds_bytes_per_wg", C.c_int32), ("reserved", C.c_int32 * 3)]


class RLCounts(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in ("kernels", "steps", "islands", "multi_islands", "edges", "jacobi_kernels",
                                          "jacobi_bodies", "jacobi_edges")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RLSceneC(C.Structure):
    _fields_ = [("n", C.c_int32), ("iters", C.c_int32), ("r", C.c_float), ("dt", C.c_float),
                ("arena", C.c_uint64), ("plan", C.c_void_p)]


_lib = None


def lib():
    """The loaded libacs.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_12377_amd.build`")
        # One HIP runtime per process: torch ships its own copy, which binds
        # libacs's reference (same soname) only if torch is loaded first.
        # Loaded the other way round, torch adds a second runtime, and the
        # one initialised second finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.acs_config_default.argtypes = [P(Config)]
        L.acs_config_default.restype = None
        L.acs_window_create.argtypes = [C.c_int32]
        L.acs_window_create.restype = C.c_void_p
        L.acs_window_configure.argtypes = [C.c_void_p, P(Config)]
        L.acs_window_configure_noalloc.argtypes = [C.c_void_p, P(Config), C.c_void_p, C.c_uint64, C.c_void_p]
        L.acs_submit.argtypes = [C.c_void_p, C.c_int32, P(Seg), C.c_int32, P(Seg), C.c_int32, C.c_void_p, C.c_size_t,
                                 P(C.c_uint64)]
        L.acs_sync.argtypes = [C.c_void_p]
        L.acs_sync_timeout.argtypes = [C.c_void_p, C.c_uint64]
        L.acs_scheduled_list.argtypes = [C.c_void_p, P(Entry), C.c_int32, P(C.c_int32)]
        L.acs_trace_read.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.acs_stats_get.argtypes = [C.c_void_p, P(Stats)]
        L.acs_window_destroy.argtypes = [C.c_void_p]
        L.acs_window_stop.argtypes = [C.c_void_p]
        L.acs_manual_take_ready.argtypes = [C.c_void_p, P(C.c_uint64), C.c_int32, P(C.c_int32)]
        L.acs_manual_complete.argtypes = [C.c_void_p, C.c_uint64, C.c_int32]
        L.acs_last_error.argtypes = []
        L.acs_strerror.argtypes = [C.c_int]
        L.acs_strerror.restype = C.c_char_p
        L.acs_rl_layout.argtypes = [C.c_int32, P(C.c_uint64)]
        L.acs_device_query.argtypes = [C.c_int32, P(DeviceInfo)]
        L.acs_device_query.restype = C.c_int
        L.acs_host_alloc.argtypes = [C.c_size_t]
        L.acs_host_alloc.restype = C.c_void_p
        L.acs_host_free.argtypes = [C.c_void_p]
        L.acs_rl_run.argtypes = [C.c_void_p, P(RLSceneC), C.c_int32, P(C.c_double), P(RLCounts)]
        L.acs_nop_run.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, P(C.c_double)]
        L.acs_nop_segs_run.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double)]
        L.acs_check_probe.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double)]
        L.acs_dnn_submit.argtypes = [C.c_void_p, P(DNNGraphC), C.c_void_p, P(C.c_uint64)]
        L.acs_graph_begin.argtypes = [C.c_void_p]
        L.acs_graph_end.argtypes = [C.c_void_p, P(C.c_void_p)]
        L.acs_graph_launch.argtypes = [C.c_void_p]
        L.acs_graph_sync.argtypes = [C.c_void_p]
        L.acs_graph_info.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int64)]
        L.acs_graph_destroy.argtypes = [C.c_void_p]
        L.acs_submit_group.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(Seg), C.c_int32, P(Seg), C.c_int32,
                                       C.c_void_p, C.c_size_t, P(C.c_uint64)]
        L.acs_sync_group.argtypes = [C.c_void_p, C.c_int32, C.c_uint64]
        L.acs_rl_run_batch.argtypes = [C.c_void_p, P(RLSceneC), C.c_int32, C.c_int32, C.c_int32, P(C.c_double),
                                       P(RLCounts)]
        L.acs_poll.argtypes = [C.c_void_p]
        L.acs_dag_submit.argtypes = [C.c_void_p, P(DAGGraphC), P(C.c_uint64)]
        L.acs_rl_run_graphs.argtypes = [P(RLSceneC), C.c_int32, C.c_int32, P(C.c_double), P(RLCounts),
                                        P(C.c_double)]
        L.acs_pool_create.argtypes = [C.c_uint64, C.c_uint64]
        L.acs_pool_create.restype = C.c_void_p
        L.acs_pool_alloc.argtypes = [C.c_void_p, C.c_uint64, P(C.c_uint64)]
        L.acs_pool_free.argtypes = [C.c_void_p, C.c_uint64]
        L.acs_pool_info.argtypes = [C.c_void_p, P(C.c_uint64), P(C.c_uint64), P(C.c_int64)]
        L.acs_pool_destroy.argtypes = [C.c_void_p]
        L.acs_pool_destroy.restype = None
        L.acs_serve_host_bytes.argtypes = [C.c_int32]
        L.acs_serve_host_bytes.restype = C.c_uint64
        L.acs_serve_run.argtypes = [C.c_void_p, P(ServeConfigC), P(ServeRequestC), C.c_int32, P(ServeResultC),
                                    P(ServeStatsC)]
        for f in ("acs_nop_segs_run", "acs_check_probe", "acs_dag_submit", "acs_rl_run_graphs", "acs_poll", "acs_pool_alloc", "acs_pool_free", "acs_pool_info", "acs_serve_run",
                  "acs_window_configure", "acs_submit", "acs_sync", "acs_sync_timeout", "acs_scheduled_list",
                  "acs_trace_read", "acs_stats_get", "acs_window_destroy", "acs_window_stop", "acs_manual_take_ready",
                  "acs_manual_complete", "acs_last_error", "acs_rl_layout", "acs_host_free", "acs_rl_run",
                  "acs_nop_run", "acs_dnn_submit", "acs_submit_group", "acs_sync_group", "acs_rl_run_batch",
                  "acs_graph_begin", "acs_graph_end", "acs_graph_launch", "acs_graph_sync", "acs_graph_info",
                  "acs_graph_destroy"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class Graph:
    """A recorded task graph (acs_graph_*): replayed as one HIP graph."""

    def __init__(self, handle):
        self._h = handle

    def launch(self):
        _check(lib().acs_graph_launch(self._h))

    def sync(self):
        _check(lib().acs_graph_sync(self._h))

    def info(self):
        k, e = C.c_int64(), C.c_int64()
        _check(lib().acs_graph_info(self._h, C.byref(k), C.byref(e)))
        return {"kernels": k.value, "edges": e.value}

    def destroy(self):
        if self._h:
            lib().acs_graph_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _check(rc):
    if rc < 0:
        raise AcsError(rc, lib().acs_strerror(rc).decode())
    return rc


def _segs(lst):
    n = len(lst)
    arr = (Seg * max(1, n))()
    for i, (s, z) in enumerate(lst):
        arr[i].start, arr[i].size = int(s), int(z)
    return arr, n


_live = weakref.WeakSet()


class Window:
    """One scheduling window (acs_window_create + acs_window_configure).
    The keyword arguments are the fields of acs_config (include/acs.h); on
    the device path with one group the dependency checks run in the check
    waves ahead of the window unless host_check_depth > 0 (on the host) or
    window_check = 1 (in the window wave at insert).  noalloc = (host
    pointer, host bytes, HIP stream handle) configures the device path
    through acs_window_configure_noalloc instead."""

    def __init__(self, W: int, path: str = "device", n_streams: int = 4, wg_per_task: int = 1, n_workers: int = 0,
                 queue_depth: int = 4096, nonblocking: bool = False, trace: bool = False,
                 trace_capacity: int = 1 << 16, device: int = 0, n_groups: int = 1, host_check_depth: int = 0,
                 window_check: int = 0, noalloc: tuple | None = None):
        L = lib()
        h = L.acs_window_create(W)
        if not h:
            code = L.acs_last_error()
            raise AcsError(code, L.acs_strerror(code).decode())
        self._h = h
        self.W = W
        self.path = path
        cfg = Config()
        L.acs_config_default(C.byref(cfg))
        cfg.path = PATHS[path]
        cfg.n_streams, cfg.wg_per_task, cfg.n_workers = n_streams, wg_per_task, n_workers
        cfg.queue_depth, cfg.nonblocking, cfg.trace = queue_depth, int(nonblocking), int(trace)
        cfg.trace_capacity, cfg.device, cfg.n_groups = trace_capacity, device, n_groups
        cfg.host_check_depth = host_check_depth
        cfg.window_check = window_check
        self.n_groups = n_groups
        if noalloc is None:
            rc = L.acs_window_configure(h, C.byref(cfg))
        else:
            host_ptr, host_bytes, stream = noalloc
            rc = L.acs_window_configure_noalloc(h, C.byref(cfg), host_ptr, host_bytes, stream)
        if rc < 0:
            msg = L.acs_strerror(rc).decode()
            L.acs_window_destroy(h)
            self._h = None
            raise AcsError(rc, msg)
        _live.add(self)

    @property
    def handle(self):
        if self._h is None:
            raise AcsError(ESTATE, "window destroyed")
        return self._h

    def submit(self, kid: int, reads, writes, args) -> int:
        r, nr = _segs(reads)
        w, nw = _segs(writes)
        seq = C.c_uint64()
        _check(lib().acs_submit(self.handle, kid, r, nr, w, nw, C.byref(args) if args is not None else None,
                                C.sizeof(args) if args is not None else 0, C.byref(seq)))
        return seq.value

    def submit_group(self, group: int, kid: int, reads, writes, args) -> int:
        r, nr = _segs(reads)
        w, nw = _segs(writes)
        seq = C.c_uint64()
        _check(lib().acs_submit_group(self.handle, group, kid, r, nr, w, nw,
                                      C.byref(args) if args is not None else None,
                                      C.sizeof(args) if args is not None else 0, C.byref(seq)))
        return seq.value

    def sync_group(self, group: int, timeout_ns: int = 0) -> int:
        return _check(lib().acs_sync_group(self.handle, group, timeout_ns))

    def graph_begin(self):
        """Subsequent submits are recorded instead of run (see acs_graph_begin)."""
        _check(lib().acs_graph_begin(self.handle))

    def graph_end(self) -> "Graph":
        h = C.c_void_p()
        _check(lib().acs_graph_end(self.handle, C.byref(h)))
        return Graph(h.value)

    def submit_raw(self, kid, reads, writes, args_bytes: bytes):
        """Like submit, with the argument block given as bytes (for tests)."""
        r, nr = _segs(reads)
        w, nw = _segs(writes)
        buf = C.create_string_buffer(args_bytes, len(args_bytes)) if args_bytes else None
        seq = C.c_uint64()
        rc = lib().acs_submit(self.handle, kid, r, nr, w, nw, buf, len(args_bytes), C.byref(seq))
        return rc, seq.value

    def sync(self, timeout_ns: int | None = None) -> int:
        if timeout_ns is None:
            return _check(lib().acs_sync(self.handle))
        return _check(lib().acs_sync_timeout(self.handle, timeout_ns))

    def sync_rc(self, timeout_ns: int | None = None) -> int:
        """Status code of a sync, without raising."""
        if timeout_ns is None:
            return lib().acs_sync(self.handle)
        return lib().acs_sync_timeout(self.handle, timeout_ns)

    def scheduled_list(self):
        arr = (Entry * W_MAX)()
        n = C.c_int32()
        _check(lib().acs_scheduled_list(self.handle, arr, W_MAX, C.byref(n)))
        return [(arr[i].seq, arr[i].kernel_id, arr[i].state, arr[i].upstream_mask, arr[i].slot)
                for i in range(n.value)]

    def trace(self, cap: int | None = None) -> np.ndarray:
        st = self.stats()
        cap = int(st["submitted"]) if cap is None else cap
        out = np.zeros(max(1, cap), dtype=TRACE_DTYPE)
        n = C.c_int64()
        _check(lib().acs_trace_read(self.handle, out.ctypes.data, cap, C.byref(n)))
        return out[:n.value]

    def stats(self) -> dict:
        s = Stats()
        _check(lib().acs_stats_get(self.handle, C.byref(s)))
        return s.as_dict()

    def take_ready(self):
        arr = (C.c_uint64 * W_MAX)()
        n = C.c_int32()
        _check(lib().acs_manual_take_ready(self.handle, arr, W_MAX, C.byref(n)))
        return [arr[i] for i in range(n.value)]

    def complete(self, seq: int, status: int = 0):
        _check(lib().acs_manual_complete(self.handle, seq, status))

    def stop(self) -> int:
        """Drains and releases the execution resources; stats and trace stay readable."""
        return _check(lib().acs_window_stop(self.handle))

    def destroy(self) -> int:
        if self._h is None:
            return OK
        rc = lib().acs_window_destroy(self._h)
        self._h = None
        _flush_host_frees()
        return rc

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


@atexit.register
def _destroy_live_windows():
    # a device window left alive would keep its persistent kernel running
    for w in list(_live):
        try:
            w.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# range helpers (the get_addresses of each task type, Section IV-A)
# ---------------------------------------------------------------------------
def tensor_seg(t, elem_offset: int = 0, n_elems: int | None = None):
    """Byte range of n_elems elements of tensor t starting at elem_offset."""
    es = t.element_size()
    n = t.numel() - elem_offset if n_elems is None else n_elems
    return (t.data_ptr() + es * elem_offset, es * n)


def gemm_segments(a_ptr: int, b_ptr: int, c_ptr: int, m: int, n: int, k: int, elem_size: int):
    """Read and write ranges of C[m,k] = A[m,n] @ B[n,k] (the paper's
    get_addresses example for matrix multiply, Section IV-A)."""
    return [(a_ptr, m * n * elem_size), (b_ptr, n * k * elem_size)], [(c_ptr, m * k * elem_size)]


def tiny_kernel_task(stream, k, base: int):
    """(kernel_id, reads, writes, args) of one tiny-stream kernel whose buffers
    live in an arena starting at device address `base`."""
    from .inputs import OP_SCALE, OP_AXPY
    addr = [base + 4 * int(o) for o in stream.offsets]
    L = [int(x) for x in stream.lengths]
    if k.op in (OP_SCALE, OP_AXPY):
        n = min([L[k.out]] + [L[b] for b in k.ins])
        reads = [(addr[b], 4 * n) for b in k.ins]
        writes = [(addr[k.out], 4 * n)]
        if k.op == OP_SCALE:
            return K_SCALE, reads, writes, ArgsScale(addr[k.out], addr[k.ins[0]], k.a, n)
        return K_AXPY, reads, writes, ArgsAxpy(addr[k.out], addr[k.ins[0]], addr[k.ins[1]], k.a, n)
    reads = [(addr[b], 4 * L[b]) for b in k.ins]
    out = addr[k.out] + 4 * k.j
    a = ArgsSum()
    a.out = out
    for t, b in enumerate(k.ins):
        a.ins[t] = addr[b]
        a.len[t] = L[b]
    a.nin = len(k.ins)
    return K_SUM, reads, [(out, 4)], a


def submit_tiny_stream(win: Window, stream, base: int):
    return [win.submit(*tiny_kernel_task(stream, k, base)) for k in stream.kernels]


# ---------------------------------------------------------------------------
# RL scene
# ---------------------------------------------------------------------------
def device_query(device: int = 0) -> dict:
    d = DeviceInfo()
    _check(lib().acs_device_query(device, C.byref(d)))
    return {f: getattr(d, f) for f, _ in DeviceInfo._fields_ if f != "reserved"}


def rl_layout(n: int) -> np.ndarray:
    off = (C.c_uint64 * RL_NREGIONS)()
    _check(lib().acs_rl_layout(n, off))
    return np.array(off[:], dtype=np.int64)


def rl_plan_ints(n: int) -> int:
    return 4 + 4 * (n // 2)


_deferred_host_frees = []


def _device_window_open() -> bool:
    return any(w._h is not None and w.path == "device" for w in list(_live))


def _flush_host_frees():
    """Frees host buffers released while a device window was open (the HIP
    host allocator synchronises the whole device, which would wait forever
    on a resident scheduler kernel)."""
    if _deferred_host_frees and not _device_window_open():
        while _deferred_host_frees:
            lib().acs_host_free(_deferred_host_frees.pop())


class HostBuffer:
    """Pinned, coherent host memory from acs_host_alloc, viewed as numpy.
    Allocate it before opening a device-path window; a free while one is
    open is deferred until the last one closes."""

    def __init__(self, nbytes: int):
        if _device_window_open():
            raise AcsError(ESTATE, "allocate host buffers before opening a device window "
                                   "(the host allocator synchronises the device)")
        p = lib().acs_host_alloc(nbytes)
        if not p:
            raise AcsError(ENOMEM, "acs_host_alloc failed: " + lib().acs_strerror(lib().acs_last_error()).decode())
        self.ptr = p
        self.nbytes = nbytes

    def view(self, dtype=np.int32):
        buf = (C.c_uint8 * self.nbytes).from_address(self.ptr)
        return np.frombuffer(buf, dtype=dtype)

    def free(self):
        if self.ptr:
            _deferred_host_frees.append(self.ptr)
            self.ptr = None
            _flush_host_frees()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class RLSceneGPU:
    """Device arena and host plan buffer of one RL scene (torch for memory)."""

    def __init__(self, scene, device="cuda"):
        import torch
        self.n = scene.n
        self.r = float(scene.radius)
        self.dt = float(scene.dt)
        self.iters = scene.iters
        self.off = rl_layout(self.n)
        self.arena = torch.zeros(int(self.off[RL_END]), dtype=torch.uint8, device=device)
        self.plan_buf = HostBuffer(4 * rl_plan_ints(self.n))
        self.plan_buf.view()[:] = 0
        self.set_state(scene.x, scene.v)

    def region(self, r: int, dtype, count: int):
        import torch
        o = int(self.off[r])
        es = torch.tensor([], dtype=dtype).element_size()
        return self.arena[o:o + es * count].view(dtype)

    def set_state(self, x, v):
        import torch
        self.region(RL_X, torch.float32, 4 * self.n).copy_(torch.as_tensor(np.ascontiguousarray(x, np.float32)).reshape(-1))
        self.region(RL_V, torch.float32, 4 * self.n).copy_(torch.as_tensor(np.ascontiguousarray(v, np.float32)).reshape(-1))
        # the library's streams do not wait for torch's; a stream-level wait
        # (not a device-wide one, which would wait for a resident persistent
        # kernel that only stops when its window is closed)
        torch.cuda.current_stream().synchronize()

    def get(self, r: int):
        import torch
        n = self.n
        if r in (RL_X, RL_V, RL_P, RL_Q0, RL_Q1):
            return self.region(r, torch.float32, 4 * n).cpu().numpy().reshape(n, 4)
        counts = {RL_DEG: n, RL_ADJ_OFF: n + 1, RL_ADJ: n * (n - 1), RL_LABEL: n, RL_PERM: n, RL_INV_PERM: n,
                  RL_ISL_OFF: n + 1, RL_PADJ_OFF: n + 1, RL_PADJ: n * (n - 1)}
        return self.region(r, torch.int32, counts[r]).cpu().numpy()

    def plan(self) -> np.ndarray:
        return self.plan_buf.view().copy()

    def c_struct(self) -> RLSceneC:
        s = RLSceneC()
        s.n, s.iters, s.r, s.dt = self.n, self.iters, self.r, self.dt
        s.arena = self.arena.data_ptr()
        s.plan = self.plan_buf.ptr
        return s


def rl_run(win: Window, scene_gpu: RLSceneGPU, steps: int):
    """Runs `steps` RL steps through the window; returns (counts dict, per-step ns)."""
    sc = scene_gpu.c_struct()
    step_ns = (C.c_double * max(1, steps))()
    k = RLCounts()
    _check(lib().acs_rl_run(win.handle, C.byref(sc), steps, step_ns, C.byref(k)))
    return k.as_dict(), np.array(step_ns[:steps])


def rl_run_batch(win: Window, scenes_gpu, steps: int, n_groups: int = 1):
    """Runs `steps` batched steps of independent scenes (scene i in group
    i % n_groups); returns (counts dict, per-batched-step ns)."""
    arr = (RLSceneC * len(scenes_gpu))()
    for i, g in enumerate(scenes_gpu):
        arr[i] = g.c_struct()
    step_ns = (C.c_double * max(1, steps))()
    k = RLCounts()
    _check(lib().acs_rl_run_batch(win.handle, arr, len(scenes_gpu), n_groups, steps, step_ns, C.byref(k)))
    return k.as_dict(), np.array(step_ns[:steps])


def rl_run_graphs(scene_gpu: RLSceneGPU, steps: int, device: int = 0):
    """The graph-per-input baseline: each step's halves recorded, built into a
    HIP graph, run and destroyed; returns (counts, per-step ns, build ns)."""
    sc = scene_gpu.c_struct()
    step_ns = (C.c_double * max(1, steps))()
    k = RLCounts()
    b = C.c_double()
    _check(lib().acs_rl_run_graphs(C.byref(sc), steps, device, step_ns, C.byref(k), C.byref(b)))
    return k.as_dict(), np.array(step_ns[:steps]), b.value


def nop_run(win: Window, n: int, chain: bool, spin_ns: int = 0) -> float:
    t = C.c_double()
    _check(lib().acs_nop_run(win.handle, n, int(chain), spin_ns, C.byref(t)))
    return t.value


def nop_segs_run(win: Window, n: int, nsegs: int) -> float:
    """n independent no-op kernels of nsegs disjoint segments each; wall ns."""
    t = C.c_double()
    _check(lib().acs_nop_segs_run(win.handle, n, nsegs, C.byref(t)))
    return t.value


# ---------------------------------------------------------------------------
# dynamic DNN (batch 1, NHWC)
# ---------------------------------------------------------------------------
def conv_task(x, w, b, out, k: int, stride: int):
    """(kernel_id, reads, writes, args) of one convolution over torch tensors
    x[h][h][cin], w[k][k][cin][cout] (or [cin][cout]), b[cout], out[ho][ho][cout]."""
    h, cin, cout = x.shape[0], x.shape[2], b.shape[0]
    a = ArgsConv(x.data_ptr(), w.data_ptr(), b.data_ptr(), out.data_ptr(), h, cin, cout, k, stride)
    return K_CONV, [tensor_seg(x), tensor_seg(w), tensor_seg(b)], [tensor_seg(out)], a


def join_task(out, a, b=None):
    args = ArgsJoin(out.data_ptr(), a.data_ptr(), b.data_ptr() if b is not None else 0, out.numel())
    reads = [tensor_seg(a)] + ([tensor_seg(b)] if b is not None else [])
    return K_JOIN, reads, [tensor_seg(out)], args


class DNNGPU:
    """Device weights and the per-inference activation buffers of the gated
    network (torch tensors for memory; every kernel runs in libacs)."""

    def __init__(self, weights, cells, classes: int, device="cuda"):
        import torch
        self.cells = cells
        self.classes = classes
        dev = torch.device(device)

        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dev)
        self.w3 = [t(a) for a in weights.w3]
        self.b3 = [t(a) for a in weights.b3]
        self.w1 = [t(a) for a in weights.w1]
        self.b1 = [t(a) for a in weights.b1]
        self.fc_w, self.fc_b = t(weights.fc_w), t(weights.fc_b)
        h0, c0 = cells[0][0], cells[0][1]
        self.x = torch.zeros((h0, h0, c0), dtype=torch.float32, device=dev)
        self.t3, self.t1, self.y = [], [], []
        for (h, cin, cout, st) in cells:
            ho = h // st
            for lst in (self.t3, self.t1, self.y):
                lst.append(torch.full((ho, ho, cout), float("nan"), dtype=torch.float32, device=dev))
        self.pool = torch.zeros(cells[-1][2], dtype=torch.float32, device=dev)
        self.out = torch.zeros(classes, dtype=torch.float32, device=dev)
        torch.cuda.current_stream().synchronize()

    def set_input(self, x):
        import torch
        self.x.copy_(torch.as_tensor(np.ascontiguousarray(x, np.float32)))
        # the library's streams do not wait for torch's; a stream-level wait
        # (not a device-wide one, which would wait for a resident persistent
        # kernel that only stops when its window is closed)
        torch.cuda.current_stream().synchronize()

    def c_struct(self) -> DNNGraphC:
        g = DNNGraphC()
        g.n_cells, g.classes = len(self.cells), self.classes
        g.x = self.x.data_ptr()
        for c, (h, cin, cout, st) in enumerate(self.cells):
            L = g.cell[c]
            L.hin, L.cin, L.cout, L.stride = h, cin, cout, st
            L.w3, L.b3, L.w1, L.b1 = (self.w3[c].data_ptr(), self.b3[c].data_ptr(), self.w1[c].data_ptr(),
                                      self.b1[c].data_ptr())
            L.t3, L.t1, L.y = self.t3[c].data_ptr(), self.t1[c].data_ptr(), self.y[c].data_ptr()
        g.pool, g.fc_w, g.fc_b, g.out = (self.pool.data_ptr(), self.fc_w.data_ptr(), self.fc_b.data_ptr(),
                                         self.out.data_ptr())
        return g


def dnn_submit(win: Window, net: DNNGPU, logits) -> int:
    """Submits one inference (no drain); returns the number of kernels."""
    g = net.c_struct()
    lg = np.ascontiguousarray(logits, np.float32).reshape(-1)
    n = C.c_uint64()
    _check(lib().acs_dnn_submit(win.handle, C.byref(g), lg.ctypes.data, C.byref(n)))
    return n.value


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class Pool:
    """Host-side allocator over a device address range (acs_pool_*)."""

    def __init__(self, base: int, nbytes: int):
        self.h = lib().acs_pool_create(base, nbytes)
        if not self.h:
            raise AcsError(EINVAL, "acs_pool_create: base must be 256-byte aligned and the range at least 256 bytes")

    def alloc(self, nbytes: int):
        """Block address, or None when no free block is large enough."""
        a = C.c_uint64()
        rc = lib().acs_pool_alloc(self.h, nbytes, C.byref(a))
        if rc == ENOMEM:
            return None
        _check(rc)
        return a.value

    def free(self, addr: int):
        _check(lib().acs_pool_free(self.h, addr))

    def info(self) -> dict:
        u, f, n = C.c_uint64(), C.c_uint64(), C.c_int64()
        _check(lib().acs_pool_info(self.h, C.byref(u), C.byref(f), C.byref(n)))
        return {"used": u.value, "largest_free": f.value, "blocks": n.value}

    def destroy(self):
        if self.h:
            lib().acs_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _align(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


class ServeSet:
    """Device-resident inputs and outputs of a list of serving requests
    (inputs.ServeSpec), and the request array acs_serve_run takes."""

    def __init__(self, specs, rl_scenes: dict, dnn_inputs: dict, classes: int, device="cuda"):
        import torch
        self.specs = specs
        self.classes = classes
        in_off, out_off, self.out_bytes = [], [], []
        ip = op = 0
        for sp in specs:
            if sp.kind == SERVE_RL:
                off = rl_layout(sp.n)
                nb = int(off[RL_V]) + 16 * sp.n
            else:
                nb = int(np.prod(dnn_inputs[sp.seed].x.shape)) * 4
            ob = nb if sp.kind == SERVE_RL else 4 * classes
            in_off.append(ip)
            out_off.append(op)
            self.out_bytes.append(ob)
            ip += _align(nb)
            op += _align(ob)
        host_in = np.zeros(max(ip, 256), np.uint8)
        for sp, o in zip(specs, in_off):
            if sp.kind == SERVE_RL:
                sc = rl_scenes[sp.seed]
                off = rl_layout(sp.n)
                host_in[o:o + 16 * sp.n] = np.ascontiguousarray(sc.x, np.float32).view(np.uint8).reshape(-1)
                v0 = o + int(off[RL_V])
                host_in[v0:v0 + 16 * sp.n] = np.ascontiguousarray(sc.v, np.float32).view(np.uint8).reshape(-1)
            else:
                x = np.ascontiguousarray(dnn_inputs[sp.seed].x, np.float32).view(np.uint8).reshape(-1)
                host_in[o:o + x.size] = x
        self.inp = torch.from_numpy(host_in).to(device)
        self.out = torch.zeros(max(op, 256), dtype=torch.uint8, device=device)
        self.out_off = out_off
        self.logits = [np.ascontiguousarray(dnn_inputs[sp.seed].logits, np.float32).reshape(-1)
                       if sp.kind == SERVE_DNN else None for sp in specs]
        self.req = (ServeRequestC * max(1, len(specs)))()
        for i, sp in enumerate(specs):
            q = self.req[i]
            q.kind = sp.kind
            q.arrival_ns = sp.arrival_ns
            q.input = self.inp.data_ptr() + in_off[i]
            q.output = self.out.data_ptr() + out_off[i]
            if sp.kind == SERVE_RL:
                sc = rl_scenes[sp.seed]
                q.n, q.iters, q.r, q.dt = sp.n, sc.iters, float(sc.radius), float(sc.dt)
            else:
                q.logits = self.logits[i].ctypes.data
        torch.cuda.current_stream().synchronize()

    def clear_outputs(self):
        import torch
        self.out.fill_(0xFF)
        torch.cuda.current_stream().synchronize()

    def outputs(self):
        """Per request: (X, V) float32[n, 4] for an RL step, logits for a DNN inference."""
        host = self.out.cpu().numpy()
        res = []
        for sp, o, nb in zip(self.specs, self.out_off, self.out_bytes):
            if sp.kind == SERVE_RL:
                off = rl_layout(sp.n)
                x = host[o:o + 16 * sp.n].view(np.float32).reshape(sp.n, 4).copy()
                v0 = o + int(off[RL_V])
                v = host[v0:v0 + 16 * sp.n].view(np.float32).reshape(sp.n, 4).copy()
                res.append((x, v))
            else:
                res.append(host[o:o + nb].view(np.float32).copy())
        return res


def serve_footprint_rl(n: int) -> int:
    return int(rl_layout(n)[RL_END])


def serve_host(max_resident: int = 256) -> HostBuffer:
    """Host signal and plan memory for serve_run (allocate before opening the window)."""
    return HostBuffer(int(lib().acs_serve_host_bytes(max_resident)))


def serve_run(win: Window, sset: ServeSet, pool, host: HostBuffer, pool_bytes: int | None = None,
              max_resident: int = 256, model: "DNNGPU | None" = None, stall_ns: int = 0):
    """Runs the requests of `sset` through `win` (acs_serve_run) with working
    memory from the device tensor `pool` and host memory from serve_host();
    returns (results, stats) with one dict per request (admit_ns, done_ns,
    kernels, footprint, group, multi_islands)."""
    cfg = ServeConfigC()
    cfg.host, cfg.host_bytes = host.ptr, host.nbytes
    cfg.pool = pool.data_ptr()
    cfg.pool_bytes = pool.numel() * pool.element_size() if pool_bytes is None else pool_bytes
    cfg.max_resident = max_resident
    g = model.c_struct() if model is not None else None
    cfg.model = C.cast(C.pointer(g), C.c_void_p) if g is not None else None
    cfg.stall_ns = stall_ns
    n = len(sset.specs)
    res = (ServeResultC * max(1, n))()
    st = ServeStatsC()
    _check(lib().acs_serve_run(win.handle, C.byref(cfg), sset.req, n, res, C.byref(st)))
    out = [{f: getattr(res[i], f) for f, _ in ServeResultC._fields_} for i in range(n)]
    return out, st.as_dict()


# ---------------------------------------------------------------------------
# static irregular network (randomly wired, batch 1)
# ---------------------------------------------------------------------------
class DAGGPU:
    """Device weights and activation buffers of the randomly wired network
    (torch tensors for memory; every kernel runs in libacs)."""

    def __init__(self, graph, weights, device="cuda"):
        import torch
        self.graph = graph
        dev = torch.device(device)

        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dev)
        h, c = graph.h, graph.c
        self.w = [t(a) for a in weights.w]
        self.b = [t(a) for a in weights.b]
        self.fc_w, self.fc_b = t(weights.fc_w), t(weights.fc_b)
        self.x = torch.zeros((h, h, c), dtype=torch.float32, device=dev)
        self.agg = [torch.full((h, h, c), float("nan"), dtype=torch.float32, device=dev) for _ in graph.preds]
        self.y = [torch.full((h, h, c), float("nan"), dtype=torch.float32, device=dev) for _ in graph.preds]
        self.sink = torch.zeros((h, h, c), dtype=torch.float32, device=dev)
        self.pool = torch.zeros(c, dtype=torch.float32, device=dev)
        self.out = torch.zeros(graph.classes, dtype=torch.float32, device=dev)
        torch.cuda.current_stream().synchronize()

    def set_input(self, x):
        import torch
        self.x.copy_(torch.as_tensor(np.ascontiguousarray(x, np.float32)))
        torch.cuda.current_stream().synchronize()

    def c_struct(self) -> DAGGraphC:
        g = DAGGraphC()
        g.n_nodes, g.h, g.c, g.classes = len(self.graph.preds), self.graph.h, self.graph.c, self.graph.classes
        g.x = self.x.data_ptr()
        for i, ps in enumerate(self.graph.preds):
            nd = g.node[i]
            nd.n_in = len(ps)
            for q, p in enumerate(ps):
                nd.inp[q] = p
            nd.w, nd.b = self.w[i].data_ptr(), self.b[i].data_ptr()
            nd.agg, nd.y = self.agg[i].data_ptr(), self.y[i].data_ptr()
        g.sink, g.pool = self.sink.data_ptr(), self.pool.data_ptr()
        g.fc_w, g.fc_b, g.out = self.fc_w.data_ptr(), self.fc_b.data_ptr(), self.out.data_ptr()
        return g


def dag_submit(win: Window, net: DAGGPU) -> int:
    """Submits one inference of the randomly wired network (no drain); returns the kernel count."""
    g = net.c_struct()
    n = C.c_uint64()
    _check(lib().acs_dag_submit(win.handle, C.byref(g), C.byref(n)))
    return n.value

