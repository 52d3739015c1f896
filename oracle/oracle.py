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
    """The oracle library, built on first use."""
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        _lib = load(path)
    return _lib


def load(path: str):
    """Loads an oracle library from `path` with its signatures declared (the
    built oracle, or a copy built elsewhere by a test)."""
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
    L.or_conv_hout.argtypes = [C.c_int32] * 3
    L.or_conv_hout.restype = C.c_int32
    L.or_conv_f32.argtypes = [C.c_void_p] * 4 + [C.c_int32] * 5
    L.or_conv_f32.restype = None
    L.or_conv_f64.argtypes = [C.c_void_p] * 5 + [C.c_int32] * 5
    L.or_conv_f64.restype = None
    L.or_relu.argtypes = [C.c_float]
    L.or_relu.restype = C.c_float
    L.or_join.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
    L.or_join.restype = None
    L.or_avgpool.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]
    L.or_avgpool.restype = None
    L.or_fc.argtypes = [C.c_void_p] * 4 + [C.c_int32] * 2
    L.or_fc.restype = None
    return L


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

    def __init__(self, n: int, r: float, dt: float, iters: int, x: np.ndarray, v: np.ndarray, L=None):
        # Jacobi sweeps alternate Q0 -> Q1 -> Q0 and the integrator reads Q0,
        # so a step is defined for an even number of sweeps only
        if iters < 0 or iters % 2:
            raise ValueError("the number of Jacobi iterations must be even and non-negative")
        self._L = L if L is not None else lib()
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
    def from_inputs(cls, sc, L=None):
        return cls(sc.n, float(sc.radius), float(sc.dt), sc.iters, sc.x, sc.v, L=L)

    def step(self):
        self._L.or_rl_step(C.byref(self.c))

    def run_kernel(self, op, island=0, it=0):
        k = RLKernelC(op, island, it)
        self._L.or_rl_run_kernel(C.byref(self.c), C.byref(k))

    def step_kernels(self):
        cap = 16 + self.c.iters * self.n
        arr = (RLKernelC * cap)()
        m = self._L.or_rl_step_kernels(C.byref(self.c), arr, cap)
        return [(arr[i].op, arr[i].island, arr[i].iter) for i in range(m)]

    def access(self, op, island=0, it=0) -> Access:
        k = RLKernelC(op, island, it)
        a = Access()
        self._L.or_rl_access(C.byref(self.c), C.byref(k), C.byref(a))
        return a

    @property
    def n_islands(self):
        return int(self.meta[0])

    @property
    def n_multi(self):
        return int(self.meta[1])

    def plan_rows(self):
        return self.plan[:4 * self.n_multi].reshape(-1, 4)


# ---------------------------------------------------------------------------
# dynamic DNN, batch 1 (Section II-C)
# ---------------------------------------------------------------------------

def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def conv_f32(x, w, b, k, s):
    """FP32 convolution in the defined order (see or_conv_f32).  x: [h, h, cin]."""
    x, w, b = _f32(x), _f32(w), _f32(b)
    h, cin = x.shape[0], x.shape[2]
    cout = b.shape[0]
    ho = lib().or_conv_hout(h, k, s)
    out = np.zeros((ho, ho, cout), np.float32)
    lib().or_conv_f32(x.ctypes.data, w.ctypes.data, b.ctypes.data, out.ctypes.data, h, cin, cout, k, s)
    return out


def conv_f64(x, w, b, k, s):
    """The same convolution in double, and the sum of |terms| per output."""
    x, w, b = _f32(x), _f32(w), _f32(b)
    h, cin = x.shape[0], x.shape[2]
    cout = b.shape[0]
    ho = lib().or_conv_hout(h, k, s)
    out = np.zeros((ho, ho, cout), np.float64)
    mag = np.zeros((ho, ho, cout), np.float64)
    lib().or_conv_f64(x.ctypes.data, w.ctypes.data, b.ctypes.data, out.ctypes.data, mag.ctypes.data,
                      h, cin, cout, k, s)
    return out, mag


def join(a, b=None):
    a = _f32(a)
    out = np.zeros_like(a)
    bb = _f32(b) if b is not None else None
    lib().or_join(out.ctypes.data, a.ctypes.data, bb.ctypes.data if bb is not None else None, a.size)
    return out


def avgpool(x):
    x = _f32(x)
    hw, c = x.shape[0] * x.shape[1], x.shape[2]
    out = np.zeros(c, np.float32)
    lib().or_avgpool(out.ctypes.data, x.ctypes.data, hw, c)
    return out


def fc(x, w, b):
    x, w, b = _f32(x), _f32(w), _f32(b)
    out = np.zeros(b.shape[0], np.float32)
    lib().or_fc(out.ctypes.data, x.ctypes.data, w.ctypes.data, b.ctypes.data, w.shape[0], w.shape[1])
    return out


DNN_CONV3, DNN_CONV1, DNN_JOIN, DNN_POOL, DNN_FC = range(5)


class DNN:
    """One inference of the gated network, run strictly in program order.

    Cell c reads the current activation; its 3x3 branch runs when logit[c][0]
    > 0, its 1x1 branch when logit[c][1] > 0 or the cell changes resolution
    (stride 2, so that the cell always produces an output); the join is
    relu(t3 + t1), relu(t3) or relu(t1).  A cell with neither branch is the
    identity.  The head is an average pool and a fully connected layer.

    Tensors get abstract, disjoint address ranges (tensor index << 40), so the
    kernels' read/write sets give the dataflow dependencies."""

    def __init__(self, weights, inp, cells):
        self.wts, self.inp, self.cells = weights, inp, cells
        self.g3 = [bool(inp.logits[c, 0] > 0) for c in range(len(cells))]
        self.g1 = [bool(inp.logits[c, 1] > 0) or cells[c][3] == 2 for c in range(len(cells))]
        self.t3, self.t1, self.y = {}, {}, {}
        self.pool = self.out = None

    # tensor ids: 0 input; per cell 1 + 7c + {0 w3, 1 b3, 2 w1, 3 b1, 4 t3, 5 t1, 6 y}; then pool, fc_w, fc_b, out
    def _tid(self, c, part):
        return 1 + 7 * c + part

    def _tensor_bytes(self, tid):
        n = len(self.cells)
        if tid == 0:
            return self.inp.x.nbytes
        if tid < 1 + 7 * n:
            c, part = divmod(tid - 1, 7)
            h, cin, cout, st = self.cells[c]
            ho = h // st
            return 4 * [9 * cin * cout, cout, cin * cout, cout, ho * ho * cout, ho * ho * cout, ho * ho * cout][part]
        extra = tid - (1 + 7 * n)
        cl = self.cells[-1][2]
        return 4 * [cl, cl * self.wts.fc_w.shape[1], self.wts.fc_b.shape[0], self.wts.fc_b.shape[0]][extra]

    def kernels(self):
        """Program-order kernel list: (op, cell, reads, writes) with reads and
        writes as tensor ids."""
        ks = []
        cur = 0
        for c in range(len(self.cells)):
            ins = []
            if self.g3[c]:
                ks.append((DNN_CONV3, c, [cur, self._tid(c, 0), self._tid(c, 1)], [self._tid(c, 4)]))
                ins.append(self._tid(c, 4))
            if self.g1[c]:
                ks.append((DNN_CONV1, c, [cur, self._tid(c, 2), self._tid(c, 3)], [self._tid(c, 5)]))
                ins.append(self._tid(c, 5))
            if ins:
                ks.append((DNN_JOIN, c, ins, [self._tid(c, 6)]))
                cur = self._tid(c, 6)
        n = len(self.cells)
        pool, fcw, fcb, out = 1 + 7 * n, 2 + 7 * n, 3 + 7 * n, 4 + 7 * n
        ks.append((DNN_POOL, -1, [cur], [pool]))
        ks.append((DNN_FC, -1, [pool, fcw, fcb], [out]))
        return ks

    def accesses(self):
        def seg(t):
            return (t << 40, self._tensor_bytes(t))
        return [make_access([seg(t) for t in r], [seg(t) for t in w]) for (_, _, r, w) in self.kernels()]

    def run(self, order=None):
        """Executes the kernels (program order, or the given permutation of the
        kernel list, which must respect the dependencies)."""
        ks = self.kernels()
        vals = {0: self.inp.x}
        idx = order if order is not None else range(len(ks))
        for i in idx:
            op, c, r, w = ks[i]
            if op in (DNN_CONV3, DNN_CONV1):
                h, cin, cout, st = self.cells[c]
                if op == DNN_CONV3:
                    vals[w[0]] = conv_f32(vals[r[0]], self.wts.w3[c], self.wts.b3[c], 3, st)
                else:
                    vals[w[0]] = conv_f32(vals[r[0]], self.wts.w1[c], self.wts.b1[c], 1, st)
            elif op == DNN_JOIN:
                vals[w[0]] = join(vals[r[0]], vals[r[1]] if len(r) > 1 else None)
            elif op == DNN_POOL:
                vals[w[0]] = avgpool(vals[r[0]])
            else:
                vals[w[0]] = fc(vals[r[0]], self.wts.fc_w, self.wts.fc_b)
        for c in range(len(self.cells)):
            for part, dst in ((4, self.t3), (5, self.t1), (6, self.y)):
                if self._tid(c, part) in vals:
                    dst[c] = vals[self._tid(c, part)]
        n = len(self.cells)
        self.pool = vals[1 + 7 * n]
        self.out = vals[4 + 7 * n]
        return self.out

    def cell_input(self, c):
        """The activation cell c reads (after run())."""
        for cc in range(c - 1, -1, -1):
            if cc in self.y:
                return self.y[cc]
        return self.inp.x


DAG_CONV, DAG_JOIN, DAG_POOL, DAG_FC = range(4)


class StaticDAG:
    """One inference of the randomly wired network, run strictly in program
    order (the static-network workload of Section VI-C).

    Node i with no predecessor convolves the input; otherwise it first
    aggregates its predecessors p0, p1, ...: agg = relu(y[p0] (+ y[p1])), then
    agg = relu(agg + y[pq]) for q >= 2, and convolves agg.  Every convolution
    is 3x3, stride 1, with bias.  The nodes nobody reads are aggregated the
    same way into `sink`, followed by an average pool and the head.  Tensors
    get abstract, disjoint address ranges (tensor index << 40)."""

    def __init__(self, graph, weights, x):
        self.g, self.wts, self.x = graph, weights, x
        self.n = len(graph.preds)
        self.y, self.agg = {}, {}
        self.sink = self.pool = self.out = None

    # tensor ids: 0 input; node i: 1 + 4i + {0 w, 1 b, 2 agg, 3 y}; then sink, pool, fc_w, fc_b, out
    def _tid(self, i, part):
        return 1 + 4 * i + part

    def _tensor_bytes(self, tid):
        h, c, k = self.g.h, self.g.c, self.g.classes
        act = 4 * h * h * c
        if tid == 0:
            return act
        if tid < 1 + 4 * self.n:
            return [4 * 9 * c * c, 4 * c, act, act][(tid - 1) % 4]
        return [act, 4 * c, 4 * c * k, 4 * k, 4 * k][tid - 1 - 4 * self.n]

    def _chain(self, node, srcs, dst):
        ks = [(DAG_JOIN, node, srcs[:2], [dst])]
        for s in srcs[2:]:
            ks.append((DAG_JOIN, node, [dst, s], [dst]))
        return ks

    def kernels(self):
        """Program-order kernel list: (op, node, reads, writes), tensor ids."""
        ks = []
        for i, ps in enumerate(self.g.preds):
            if ps:
                ks += self._chain(i, [self._tid(p, 3) for p in ps], self._tid(i, 2))
                src = self._tid(i, 2)
            else:
                src = 0
            ks.append((DAG_CONV, i, [src, self._tid(i, 0), self._tid(i, 1)], [self._tid(i, 3)]))
        n = self.n
        sink, pool, fcw, fcb, out = 1 + 4 * n, 2 + 4 * n, 3 + 4 * n, 4 + 4 * n, 5 + 4 * n
        ks += self._chain(-1, [self._tid(s, 3) for s in self.g.sinks], sink)
        ks.append((DAG_POOL, -1, [sink], [pool]))
        ks.append((DAG_FC, -1, [pool, fcw, fcb], [out]))
        return ks

    def accesses(self):
        def seg(t):
            return (t << 40, self._tensor_bytes(t))
        return [make_access([seg(t) for t in r], [seg(t) for t in w]) for (_, _, r, w) in self.kernels()]

    def run(self, order=None):
        ks = self.kernels()
        vals = {0: self.x}
        for i in (order if order is not None else range(len(ks))):
            op, node, r, w = ks[i]
            if op == DAG_CONV:
                vals[w[0]] = conv_f32(vals[r[0]], self.wts.w[node], self.wts.b[node], 3, 1)
            elif op == DAG_JOIN:
                vals[w[0]] = join(vals[r[0]], vals[r[1]] if len(r) > 1 else None)
            elif op == DAG_POOL:
                vals[w[0]] = avgpool(vals[r[0]])
            else:
                vals[w[0]] = fc(vals[r[0]], self.wts.fc_w, self.wts.fc_b)
        for i in range(self.n):
            self.y[i] = vals[self._tid(i, 3)]
            if self._tid(i, 2) in vals:
                self.agg[i] = vals[self._tid(i, 2)]
        n = self.n
        self.sink, self.pool, self.out = vals[1 + 4 * n], vals[2 + 4 * n], vals[5 + 4 * n]
        return self.out

    def node_input(self, i):
        """The activation node i convolves (after run())."""
        return self.agg[i] if self.g.preds[i] else self.x
