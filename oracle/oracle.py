"""ctypes wrapper around the CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: the library's product path never imports this
module.  Only tests/, the smoke check and the benchmark's CPU-baseline leg do.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KMAX = 16


class Seg(C.Structure):
    _fields_ = [("start", C.c_uint64), ("size", C.c_uint64)]


class Access(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_w", C.c_int32), ("r", Seg * KMAX), ("w", Seg * KMAX)]

    def reads(self):
        return [(self.r[i].start, self.r[i].size) for i in range(self.n_r)]

    def writes(self):
        return [(self.w[i].start, self.w[i].size) for i in range(self.n_w)]


TRACE_DTYPE = np.dtype([("seq", np.int64), ("slot", np.int64), ("kid", np.int64),
                        ("ev_insert", np.int64), ("ev_dispatch", np.int64), ("ev_retire", np.int64),
                        ("valid_mask", np.uint64), ("up_mask", np.uint64),
                        ("t_start", np.int64), ("t_end", np.int64),
                        ("t_dispatch", np.int64), ("t_retire", np.int64)])


class TinyKernelC(C.Structure):
    _fields_ = [("op", C.c_int32), ("out", C.c_int32), ("nin", C.c_int32), ("ins", C.c_int32 * 3),
                ("j", C.c_int32), ("a", C.c_float)]


class SceneC(C.Structure):
    _fields_ = [("n", C.c_int32), ("iters", C.c_int32), ("r", C.c_float), ("dt", C.c_float)] + \
               [(f, C.c_void_p) for f in ("X", "V", "P", "Q0", "Q1", "deg", "adj_off", "adj", "label",
                                          "perm", "inv_perm", "isl_off", "padj_off", "padj", "meta", "plan")]


class RLKernelC(C.Structure):
    _fields_ = [("op", C.c_int32), ("island", C.c_int32), ("iter", C.c_int32)]


RL_PREDICT, RL_BROADPHASE, RL_ISLANDS, RL_PERMUTE, RL_JACOBI, RL_INTEGRATE = range(6)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(path)
        L.or_overlap.argtypes = [C.c_uint64] * 4
        L.or_overlap.restype = C.c_int
        L.or_conflict.argtypes = [C.POINTER(Access), C.POINTER(Access)]
        L.or_conflict.restype = C.c_int
        L.or_conflict_literal.argtypes = [C.POINTER(Access), C.POINTER(Access)]
        L.or_conflict_literal.restype = C.c_int
        L.or_dag.argtypes = [C.c_int32, C.POINTER(Access), C.c_int32, C.c_void_p]
        L.or_dag.restype = None
        L.or_check_trace.argtypes = [C.c_int32, C.POINTER(Access), C.c_int32, C.c_void_p, C.c_int32,
                                     C.c_int32, C.c_char_p, C.c_int32]
        L.or_check_trace.restype = C.c_int32
        L.or_tiny_access.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(TinyKernelC),
                                     C.POINTER(Access)]
        L.or_tiny_access.restype = None
        L.or_tiny_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(TinyKernelC),
                                  C.c_void_p]
        L.or_tiny_run.restype = None
        L.or_tree_sum.argtypes = [C.c_void_p, C.c_int64]
        L.or_tree_sum.restype = C.c_float
        L.or_rl_run_kernel.argtypes = [C.POINTER(SceneC), C.POINTER(RLKernelC)]
        L.or_rl_run_kernel.restype = None
        L.or_rl_access.argtypes = [C.POINTER(SceneC), C.POINTER(RLKernelC), C.POINTER(Access)]
        L.or_rl_access.restype = None
        L.or_rl_step_kernels.argtypes = [C.POINTER(SceneC), C.POINTER(RLKernelC), C.c_int32]
        L.or_rl_step_kernels.restype = C.c_int32
        L.or_rl_step.argtypes = [C.POINTER(SceneC)]
        L.or_rl_step.restype = None
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# predicate, DAG, trace checker
# ---------------------------------------------------------------------------

def make_access(reads, writes) -> Access:
    a = Access()
    a.n_r, a.n_w = len(reads), len(writes)
    for i, (s, z) in enumerate(reads):
        a.r[i].start, a.r[i].size = s, z
    for i, (s, z) in enumerate(writes):
        a.w[i].start, a.w[i].size = s, z
    return a


def overlap(s1, z1, s2, z2) -> bool:
    return bool(lib().or_overlap(s1, z1, s2, z2))


def conflict(older: Access, newer: Access, literal: bool = False) -> bool:
    f = lib().or_conflict_literal if literal else lib().or_conflict
    return bool(f(C.byref(older), C.byref(newer)))


def access_array(accs):
    arr = (Access * max(1, len(accs)))()
    for i, a in enumerate(accs):
        arr[i] = a
    return arr


def dag(accs, literal: bool = False) -> np.ndarray:
    n = len(accs)
    adj = np.zeros((n, n), dtype=np.uint8)
    if n:
        lib().or_dag(n, access_array(accs), int(literal), adj.ctypes.data)
    return adj


def check_trace(accs, W: int, trace: np.ndarray, check_times: bool = False, early: bool = False):
    """Returns (code, message); code 0 means the trace is a valid schedule.
    early=True: kernels may be handed out before their upstream kernels retire
    (they must be handed out after them and must start after they end)."""
    trace = np.ascontiguousarray(trace, dtype=TRACE_DTYPE)
    buf = C.create_string_buffer(512)
    code = lib().or_check_trace(len(accs), access_array(accs), W, trace.ctypes.data,
                                int(check_times), int(early), buf, 512)
    return int(code), buf.value.decode()


def random_topological_order(adj: np.ndarray, rng: np.random.Generator) -> list:
    n = adj.shape[0]
    indeg = adj.sum(axis=0).astype(np.int64)
    ready = [i for i in range(n) if indeg[i] == 0]
    order = []
    while ready:
        k = int(rng.integers(len(ready)))
        i = ready.pop(k)
        order.append(i)
        for j in np.nonzero(adj[i])[0]:
            indeg[j] -= 1
            if indeg[j] == 0:
                ready.append(int(j))
    assert len(order) == n
    return order


# ---------------------------------------------------------------------------
# tiny random stream
# ---------------------------------------------------------------------------

def _tiny_kernels(stream):
    ks = (TinyKernelC * len(stream.kernels))()
    for i, k in enumerate(stream.kernels):
        ks[i].op, ks[i].out, ks[i].nin = k.op, k.out, len(k.ins)
        for t, b in enumerate(k.ins):
            ks[i].ins[t] = b
        ks[i].j, ks[i].a = k.j, k.a
    return ks


def tiny_accesses(stream, base: int = 0):
    offs = np.ascontiguousarray(stream.offsets, dtype=np.int64)
    lens = np.ascontiguousarray(stream.lengths, dtype=np.int64)
    ks = _tiny_kernels(stream)
    out = []
    for i in range(len(stream.kernels)):
        a = Access()
        lib().or_tiny_access(offs.ctypes.data, lens.ctypes.data, base, C.byref(ks[i]), C.byref(a))
        out.append(a)
    return out


def tiny_run(stream, order=None, arena=None) -> np.ndarray:
    """Executes the stream on a copy of its initial arena (program order by default)."""
    a = np.array(stream.init if arena is None else arena, dtype=np.float32, copy=True)
    offs = np.ascontiguousarray(stream.offsets, dtype=np.int64)
    lens = np.ascontiguousarray(stream.lengths, dtype=np.int64)
    ks = _tiny_kernels(stream)
    o = None
    if order is not None:
        o = np.ascontiguousarray(order, dtype=np.int32)
    lib().or_tiny_run(a.ctypes.data, offs.ctypes.data, lens.ctypes.data, len(stream.kernels), ks,
                      None if o is None else o.ctypes.data)
    return a


def tree_sum(v: np.ndarray) -> np.float32:
    v = np.ascontiguousarray(v, dtype=np.float32)
    return np.float32(lib().or_tree_sum(v.ctypes.data, len(v)))


# ---------------------------------------------------------------------------
# rigid-body RL scene
# ---------------------------------------------------------------------------

class Scene:
    """Host arrays for one RL scene plus the C view of them."""

    INT_FIELDS = ("deg", "adj_off", "adj", "label", "perm", "inv_perm", "isl_off", "padj_off",
                  "padj", "meta", "plan")

    def __init__(self, n: int, r: float, dt: float, iters: int, x: np.ndarray, v: np.ndarray):
        self.n = n
        e = max(1, n * (n - 1))
        self.X = np.array(x, dtype=np.float32).reshape(n, 4).copy()
        self.V = np.array(v, dtype=np.float32).reshape(n, 4).copy()
        self.P = np.zeros((n, 4), np.float32)
        self.Q0 = np.zeros((n, 4), np.float32)
        self.Q1 = np.zeros((n, 4), np.float32)
        self.deg = np.zeros(n, np.int32)
        self.adj_off = np.zeros(n + 1, np.int32)
        self.adj = np.zeros(e, np.int32)
        self.label = np.zeros(n, np.int32)
        self.perm = np.zeros(n, np.int32)
        self.inv_perm = np.zeros(n, np.int32)
        self.isl_off = np.zeros(n + 1, np.int32)
        self.padj_off = np.zeros(n + 1, np.int32)
        self.padj = np.zeros(e, np.int32)
        self.meta = np.zeros(3, np.int32)
        self.plan = np.zeros(4 * max(1, n // 2), np.int32)
        self.c = SceneC()
        self.c.n, self.c.iters, self.c.r, self.c.dt = n, iters, r, dt
        for f in ("X", "V", "P", "Q0", "Q1") + self.INT_FIELDS:
            setattr(self.c, f, getattr(self, f).ctypes.data)

    @classmethod
    def from_inputs(cls, sc):
        return cls(sc.n, float(sc.radius), float(sc.dt), sc.iters, sc.x, sc.v)

    def step(self):
        lib().or_rl_step(C.byref(self.c))

    def run_kernel(self, op, island=0, it=0):
        k = RLKernelC(op, island, it)
        lib().or_rl_run_kernel(C.byref(self.c), C.byref(k))

    def step_kernels(self):
        cap = 16 + self.c.iters * self.n
        arr = (RLKernelC * cap)()
        m = lib().or_rl_step_kernels(C.byref(self.c), arr, cap)
        return [(arr[i].op, arr[i].island, arr[i].iter) for i in range(m)]

    def access(self, op, island=0, it=0) -> Access:
        k = RLKernelC(op, island, it)
        a = Access()
        lib().or_rl_access(C.byref(self.c), C.byref(k), C.byref(a))
        return a

    @property
    def n_islands(self):
        return int(self.meta[0])

    @property
    def n_multi(self):
        return int(self.meta[1])

    def plan_rows(self):
        return self.plan[:4 * self.n_multi].reshape(-1, 4)
