"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers and lays out buffers.  It holds none of
the scheduler's logic (segments, overlap tests, window state) and none of the
task-body arithmetic: both sides receive the same arrays and kernel lists from
here and compute everything else on their own.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: draw k of stream s is mix(s + (k + 1) * GAMMA).

Workloads (the paper's own suites are not available, so these synthetic ones
stand in for them, shaped like the paper's evaluation workloads):

* tiny random stream: 16 FP32 buffers of 256..4096 elements, 64 kernels drawn
  from {scale, axpy, sum_reduce}, each reading 1..3 distinct buffers and
  writing one buffer;
* rigid-body RL step: N spheres in the unit box with random velocities, the
  per-step kernel list of which depends on the contacts found at run time
  (the paper's physics-engine case study, Section II-B);
* batched scenes: many RL scenes of log-uniform size;
* dynamic DNN, batch 1: 12 cells of two gated parallel branches (3x3 and 1x1
  convolutions), 32x32x32 -> 8x8x128 NHWC, average pool and a 128 -> 10 fully
  connected head; which branches run depends on seeded per-input logits (the
  paper's dynamic-network case study, Section II-C);
* serving: an open-loop request stream with Poisson arrivals mixing RL scene
  steps (log-uniform size) and DNN inferences.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

OP_SCALE, OP_AXPY, OP_SUM = 0, 1, 2
OP_NAMES = {OP_SCALE: "scale", OP_AXPY: "axpy", OP_SUM: "sum_reduce"}


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream (scalar draws)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        return _mix(self.state)

    def below(self, n: int) -> int:
        """Integer in [0, n) (plain modulo; the bias is part of the definition)."""
        return self.next() % n

    def uniform_pm1(self) -> np.float32:
        return np.float32(((self.next() >> 40) * 2.0 ** -23) - 1.0)


def splitmix64_array(seed: int, n: int) -> np.ndarray:
    """Draws 0..n-1 of the stream seeded with `seed`, vectorised."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + k * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(bits: np.ndarray) -> np.ndarray:
    """U[-1, 1) in FP32 from the top 24 bits; every value is exact in FP32."""
    return ((bits >> np.uint64(40)).astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)


def uniform_01(bits: np.ndarray) -> np.ndarray:
    """U[0, 1) in float64 from the top 24 bits."""
    return (bits >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


# ---------------------------------------------------------------------------
# Tiny random stream
# ---------------------------------------------------------------------------

@dataclass
class TinyKernel:
    op: int               # OP_SCALE / OP_AXPY / OP_SUM
    out: int              # buffer written
    ins: tuple            # buffers read (distinct), 1 for scale, 2 for axpy, 1..3 for sum
    a: float              # scalar for scale / axpy
    j: int                # element of `out` written by sum_reduce


@dataclass
class TinyStream:
    seed: int
    lengths: np.ndarray          # int64[n_buffers], elements
    offsets: np.ndarray          # int64[n_buffers], elements from the arena start (256-B aligned)
    arena_elems: int
    init: np.ndarray             # float32[arena_elems], initial arena contents
    kernels: list = field(default_factory=list)

    @property
    def n_buffers(self) -> int:
        return len(self.lengths)


def tiny_stream(seed: int = 0, n_kernels: int = 64, n_buffers: int = 16,
                min_len: int = 256, max_len: int = 4096) -> TinyStream:
    rng = SplitMix64(seed)
    lengths = np.array([min_len + rng.below(max_len - min_len + 1) for _ in range(n_buffers)],
                       dtype=np.int64)
    offsets = np.zeros(n_buffers, dtype=np.int64)
    pos = 0
    for b in range(n_buffers):
        offsets[b] = pos
        pos += int(lengths[b])
        pos = (pos + 63) // 64 * 64          # 64 floats = 256 bytes
    arena = np.zeros(pos, dtype=np.float32)
    data_seed = rng.next()
    vals = uniform_pm1(splitmix64_array(data_seed, int(lengths.sum())))
    k = 0
    for b in range(n_buffers):
        L = int(lengths[b])
        arena[offsets[b]:offsets[b] + L] = vals[k:k + L]
        k += L
    kernels = []
    for _ in range(n_kernels):
        op = rng.below(3)
        a = float(rng.uniform_pm1())
        out = rng.below(n_buffers)
        if op == OP_SCALE:
            ins = (rng.below(n_buffers),)
        elif op == OP_AXPY:
            x = rng.below(n_buffers)
            y = rng.below(n_buffers - 1)
            if y >= x:
                y += 1
            ins = (x, y)
        else:
            nin = 1 + rng.below(3)
            chosen: list = []
            while len(chosen) < nin:
                c = rng.below(n_buffers)
                if c not in chosen:
                    chosen.append(c)
            ins = tuple(chosen)
        j = rng.below(int(lengths[out]))
        kernels.append(TinyKernel(op=op, out=out, ins=ins, a=a, j=j))
    return TinyStream(seed=seed, lengths=lengths, offsets=offsets, arena_elems=pos,
                      init=arena, kernels=kernels)


# ---------------------------------------------------------------------------
# Rigid-body RL scene
# ---------------------------------------------------------------------------

RL_DT = np.float32(1.0 / 120.0)
RL_RADIUS_64 = 0.10
RL_ITERS = 8


@dataclass
class RLScene:
    seed: int
    n: int
    radius: np.float32
    dt: np.float32
    iters: int
    x: np.ndarray     # float32[n, 4]  (x, y, z, 0)
    v: np.ndarray     # float32[n, 4]  (vx, vy, vz, 0)


def rl_scene(seed: int = 1, n: int = 64, radius: float | None = None) -> RLScene:
    """Spheres uniform in [r, 1-r]^3 with velocities uniform in [-1, 1)^3.

    The radius defaults to 0.10 * (64 / n)^(1/3), which keeps the body density
    (and so the expected contact degree) the same for every scene size.  At
    this density a 64-sphere scene keeps about 7-9 multi-body islands per step
    (about 75 kernels per step) once the initial overlaps are resolved; a
    radius of 0.06 decays to under 2 islands per step.
    """
    if radius is None:
        radius = RL_RADIUS_64 * (64.0 / n) ** (1.0 / 3.0)
    r = np.float32(radius)
    bits = splitmix64_array(seed, 6 * n)
    u = uniform_01(bits[:3 * n]).reshape(n, 3)
    x = np.zeros((n, 4), dtype=np.float32)
    x[:, :3] = (float(r) + (1.0 - 2.0 * float(r)) * u).astype(np.float32)
    v = np.zeros((n, 4), dtype=np.float32)
    v[:, :3] = uniform_pm1(bits[3 * n:]).reshape(n, 3)
    return RLScene(seed=seed, n=n, radius=r, dt=RL_DT, iters=RL_ITERS, x=x, v=v)


def batched_scene_sizes(seed: int = 3, n_scenes: int = 256, lo: int = 16, hi: int = 512) -> np.ndarray:
    """Scene sizes log-uniform in [lo, hi]."""
    u = uniform_01(splitmix64_array(seed, n_scenes))
    n = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    return np.clip(n, lo, hi)


def batched_scenes(seed: int = 3, n_scenes: int = 256) -> list:
    sizes = batched_scene_sizes(seed, n_scenes)
    return [rl_scene(seed=(seed * 1_000_003 + i) & MASK64, n=int(s)) for i, s in enumerate(sizes)]


# ---------------------------------------------------------------------------
# Dynamic DNN (batch 1)
# ---------------------------------------------------------------------------

# (input height = width, input channels, output channels, stride) per cell.
# Cells 4 and 8 halve the resolution and double the channels.
DNN_CELLS = ([(32, 32, 32, 1)] * 4 + [(32, 32, 64, 2)] + [(16, 64, 64, 1)] * 3 +
             [(16, 64, 128, 2)] + [(8, 128, 128, 1)] * 3)
DNN_CLASSES = 10
DNN_INPUT = (32, 32, 32)   # H, W, C (NHWC, batch 1)


@dataclass
class DNNWeights:
    w3: list      # per cell float32[3, 3, cin, cout]
    b3: list      # per cell float32[cout]
    w1: list      # per cell float32[cin, cout]
    b1: list      # per cell float32[cout]
    fc_w: np.ndarray   # float32[128, 10]
    fc_b: np.ndarray   # float32[10]


def _uniform_sym(seed: int, n: int, bound: float) -> np.ndarray:
    """U[-bound, bound) in FP32 (bound times an exact U[-1, 1) draw, rounded once)."""
    return (uniform_pm1(splitmix64_array(seed, n)).astype(np.float64) * bound).astype(np.float32)


def dnn_weights(seed: int = 2) -> DNNWeights:
    """He-uniform weights (bound sqrt(6 / fan_in)) and biases U[-1/sqrt(fan_in), ...)."""
    w3, b3, w1, b1 = [], [], [], []
    for c, (h, cin, cout, st) in enumerate(DNN_CELLS):
        base = (seed * 1_000_003 + 97 * c) & MASK64
        f3, f1 = 9 * cin, cin
        w3.append(_uniform_sym(base + 1, 9 * cin * cout, math.sqrt(6.0 / f3)).reshape(3, 3, cin, cout))
        b3.append(_uniform_sym(base + 2, cout, 1.0 / math.sqrt(f3)))
        w1.append(_uniform_sym(base + 3, cin * cout, math.sqrt(6.0 / f1)).reshape(cin, cout))
        b1.append(_uniform_sym(base + 4, cout, 1.0 / math.sqrt(f1)))
    cl = DNN_CELLS[-1][2]
    base = (seed * 1_000_003 + 97 * len(DNN_CELLS)) & MASK64
    fc_w = _uniform_sym(base + 1, cl * DNN_CLASSES, math.sqrt(6.0 / cl)).reshape(cl, DNN_CLASSES)
    fc_b = _uniform_sym(base + 2, DNN_CLASSES, 1.0 / math.sqrt(cl))
    return DNNWeights(w3, b3, w1, b1, fc_w, fc_b)


@dataclass
class DNNInput:
    seed: int
    x: np.ndarray        # float32[32, 32, 32] NHWC
    logits: np.ndarray   # float32[12, 2]: gate logits of the 3x3 and 1x1 branch of each cell


def dnn_input(seed: int = 0) -> DNNInput:
    """Input image U[-1, 1) and one gate logit U[-1, 1) per branch; a branch
    runs when its logit is positive (only the sign is used)."""
    h, w, c = DNN_INPUT
    bits = splitmix64_array((0xD22 << 32) ^ seed, h * w * c + 2 * len(DNN_CELLS))
    x = uniform_pm1(bits[:h * w * c]).reshape(h, w, c)
    logits = uniform_pm1(bits[h * w * c:]).reshape(len(DNN_CELLS), 2)
    return DNNInput(seed=seed, x=x, logits=logits)


# ---------------------------------------------------------------------------
# Serving: Poisson arrivals of mixed requests
# ---------------------------------------------------------------------------

SERVE_RL, SERVE_DNN = 0, 1


@dataclass
class ServeSpec:
    kind: int             # SERVE_RL or SERVE_DNN
    arrival_ns: float     # after the start of the run
    seed: int             # scene or input seed
    n: int = 0            # RL bodies


def serve_requests(seed: int = 4, rate_per_s: float = 5000.0, n_requests: int = 2000, rl_fraction: float = 0.5,
                   lo: int = 16, hi: int = 512) -> list:
    """Poisson arrivals at rate_per_s (exponential gaps by inversion of
    U[0, 1)); each request is an RL step of a scene of log-uniform size in
    [lo, hi] with probability rl_fraction, else a DNN inference."""
    u = uniform_01(splitmix64_array((0x5E27E << 32) ^ seed, 3 * n_requests)).reshape(n_requests, 3)
    gaps = -np.log1p(-u[:, 0]) / rate_per_s * 1e9
    t = np.cumsum(gaps)
    sizes = np.clip(np.rint(np.exp(math.log(lo) + u[:, 2] * (math.log(hi) - math.log(lo)))), lo, hi).astype(np.int64)
    out = []
    for i in range(n_requests):
        req_seed = (seed * 1_000_003 + 7919 * i) & MASK64
        if u[i, 1] < rl_fraction:
            out.append(ServeSpec(SERVE_RL, float(t[i]), req_seed, int(sizes[i])))
        else:
            out.append(ServeSpec(SERVE_DNN, float(t[i]), req_seed))
    return out



# ---------------------------------------------------------------------------
# Static irregular DAG network (randomly wired, batch 1)
# ---------------------------------------------------------------------------

DAG_MAX_IN = 8
DAG_H, DAG_C = 32, 32      # every node's activation is DAG_H x DAG_H x DAG_C (NHWC)


@dataclass
class DAGGraph:
    preds: list            # per node: sorted earlier nodes it reads (empty: reads the input)
    h: int
    c: int
    classes: int

    @property
    def sinks(self):
        used = {p for ps in self.preds for p in ps}
        return [i for i in range(len(self.preds)) if i not in used]


def dag_graph(seed: int = 5, nodes: int = 32, k: int = 4, p: float = 0.75) -> DAGGraph:
    """A randomly wired network in the style of the randomly wired NAS
    networks: a Watts-Strogatz small-world graph (ring lattice where each
    node links to its k / 2 next neighbours, each link rewired with
    probability p to a uniformly drawn node that is neither itself nor
    already linked), made acyclic by directing every link from the lower to
    the higher node index.  At most DAG_MAX_IN inputs per node (the lowest
    indices are kept)."""
    rng = SplitMix64((0xDA6 << 40) ^ seed)
    adj = [set() for _ in range(nodes)]
    for i in range(nodes):
        for j in range(1, k // 2 + 1):
            adj[i].add((i + j) % nodes)
            adj[(i + j) % nodes].add(i)
    for j in range(1, k // 2 + 1):
        for i in range(nodes):
            t = (i + j) % nodes
            u = rng.next() >> 11
            if u * 2.0 ** -53 < p and t in adj[i]:
                cands = [v for v in range(nodes) if v != i and v not in adj[i]]
                if cands:
                    v = cands[rng.below(len(cands))]
                    adj[i].discard(t)
                    adj[t].discard(i)
                    adj[i].add(v)
                    adj[v].add(i)
    preds = [sorted(v for v in adj[i] if v < i)[:DAG_MAX_IN] for i in range(nodes)]
    return DAGGraph(preds=preds, h=DAG_H, c=DAG_C, classes=DNN_CLASSES)


@dataclass
class DAGWeights:
    w: list                # per node float32[3, 3, c, c]
    b: list                # per node float32[c]
    fc_w: np.ndarray       # float32[c, classes]
    fc_b: np.ndarray


def dag_weights(graph: DAGGraph, seed: int = 6) -> DAGWeights:
    c = graph.c
    w, b = [], []
    for i in range(len(graph.preds)):
        base = (seed * 1_000_003 + 131 * i) & MASK64
        w.append(_uniform_sym(base + 1, 9 * c * c, math.sqrt(6.0 / (9 * c))).reshape(3, 3, c, c))
        b.append(_uniform_sym(base + 2, c, 1.0 / math.sqrt(9 * c)))
    base = (seed * 1_000_003 + 131 * len(graph.preds)) & MASK64
    fc_w = _uniform_sym(base + 1, c * graph.classes, math.sqrt(6.0 / c)).reshape(c, graph.classes)
    fc_b = _uniform_sym(base + 2, graph.classes, 1.0 / math.sqrt(c))
    return DAGWeights(w, b, fc_w, fc_b)


def dag_input(graph: DAGGraph, seed: int = 0) -> np.ndarray:
    """Input image U[-1, 1), h x h x c."""
    n = graph.h * graph.h * graph.c
    return uniform_pm1(splitmix64_array((0xDA7 << 32) ^ seed, n)).reshape(graph.h, graph.h, graph.c)
