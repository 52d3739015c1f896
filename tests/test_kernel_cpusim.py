"""The persistent scheduler kernel's own source, built for the CPU.

tests/cpusim/sim.cpp compiles the window wave, the FIFO wave, the check waves and the worker
loop (persistent.hpp, bodies.hpp) against a host emulation of the HIP
built-ins they use, one OS thread per GPU thread.  These tests push the tiny
random stream through that build and compare with the oracle: the arena must
be bit-identical to in-order execution (Section III: reordering only among
proven-independent kernels leaves the result unchanged) and the trace must be
a valid windowed schedule of the stream's dependency DAG (Section III-C,
Algorithm 1), with execution intervals of dependent kernels disjoint.

The emulation's atomics are sequentially consistent, so these runs check the
scheduling logic (admission, upstream masks, early dispatch, completion
targets, ring back-pressure, drain), not the GPU memory model; the GPU
parity tests cover the latter.
"""
from __future__ import annotations

import ctypes as C
import time
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import acs, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM_DIR = os.path.join(ROOT, "tests", "cpusim")
OUT = os.path.join(ROOT, "_build", "cpusim", "libsim.so")


class SimDesc(C.Structure):
    _fields_ = [("kid", C.c_int32), ("npieces", C.c_uint32), ("nseg", C.c_uint32), ("wbits", C.c_uint32),
                ("s", C.c_uint64 * 8), ("e", C.c_uint64 * 8), ("args", C.c_uint8 * 64)]


@pytest.fixture(scope="module")
def sim():
    cxx = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
    if not os.path.exists(cxx):
        pytest.skip("clang++ (for the vector types of the kernel source) not available")
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    # built under a private name and moved into place, so that parallel test
    # processes never load a half-written library
    tmp = f"{OUT}.{os.getpid()}"
    cmd = [cxx, "-std=c++20", "-O1", "-pthread", "-fPIC", "-shared",
           "-I", SIM_DIR, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2401_12377_amd", "csrc"),
           os.path.join(SIM_DIR, "sim.cpp"), "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    os.replace(tmp, OUT)
    lib = C.CDLL(OUT)
    lib.sim_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_uint32, C.c_void_p,
                            C.c_double, C.POINTER(C.c_uint64)]
    lib.sim_run.restype = C.c_int
    return lib


def _descs(st, base):
    descs = (SimDesc * len(st.kernels))()
    for i, k in enumerate(st.kernels):
        kid, r, w, a = acs.tiny_kernel_task(st, k, base)
        d = descs[i]
        d.kid = kid
        # elementwise bodies split over two workgroups, the reduction runs in one
        d.npieces = 2 if k.op in (inputs.OP_SCALE, inputs.OP_AXPY) else 1
        segs = [(s, s + z) for s, z in r] + [(s, s + z) for s, z in w]
        d.nseg = len(segs)
        d.wbits = sum(1 << (len(r) + j) for j in range(len(w)))
        for j, (s0, e0) in enumerate(segs):
            d.s[j] = s0
            d.e[j] = e0
        b = bytes(a)
        C.memmove(d.args, b, len(b))
    return descs


# a deadlock in the emulated kernel would block inside the C call: the thread
# method ends the run instead of hanging it
@pytest.mark.timeout(180, method="thread")
@pytest.mark.parametrize("seed,W,workers,ring", [
    (0, 8, 2, 64),
    (1, 4, 1, 64),
    (2, 64, 3, 64),
    (3, 16, 2, 4),      # ring smaller than the stream: host back-pressure
    (4, 1, 2, 64),      # window of one: strictly in order
    (5, 32, 2, 64),     # two lanes per slot
    (6, 3, 2, 64),      # window not a power of two
    (7, 20, 3, 16),
])
def test_tiny_stream_through_kernel_source(sim, seed, W, workers, ring):
    st = inputs.tiny_stream(seed)
    arena = st.init.copy()
    descs = _descs(st, arena.ctypes.data)
    tr = np.zeros(len(st.kernels), dtype=acs.TRACE_DTYPE)
    retired = C.c_uint64()
    rc = sim.sim_run(W, workers, len(st.kernels), descs, ring, tr.ctypes.data, 60.0, C.byref(retired))
    assert rc == 0 and retired.value == len(st.kernels)
    ref = O.tiny_run(st)
    assert np.array_equal(arena.view(np.uint32), ref.view(np.uint32))
    code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
    assert code == 0, msg
    if W == 1:
        # with one slot every kernel is inserted only after its predecessor retired
        assert np.all(tr["up_mask"] == 0)
        assert np.all(np.diff(tr["t_start"]) > 0)


@pytest.mark.timeout(180, method="thread")
@pytest.mark.parametrize("h,cin,cout,k,s", [(8, 32, 32, 3, 1), (16, 64, 32, 1, 2), (16, 32, 64, 3, 2),
                                            (12, 32, 32, 3, 1), (4, 128, 64, 3, 1), (8, 64, 32, 1, 1)])
def test_conv_tile_through_kernel_source(sim, h, cin, cout, k, s):
    """The convolution body's tiling, K split between waves and partial-tile
    sum, on the emulated 16x16x4 matrix step, against the oracle's float64
    convolution."""
    g = np.random.default_rng(h + cin + k)
    x = g.uniform(-1, 1, (h, h, cin)).astype(np.float32)
    w = g.uniform(-1, 1, (k, k, cin, cout) if k == 3 else (cin, cout)).astype(np.float32)
    b = g.uniform(-1, 1, cout).astype(np.float32)
    exact, mag = O.conv_f64(x, w, b, k, s)
    out = np.full(exact.shape, np.nan, np.float32)
    a = acs.ArgsConv(x.ctypes.data, w.ctypes.data, b.ctypes.data, out.ctypes.data, h, cin, cout, k, s)
    descs = (SimDesc * 1)()
    d = descs[0]
    d.kid = acs.K_CONV
    d.npieces = max(1, (exact.shape[0] * exact.shape[1] // 16) * (cout // 32))
    d.nseg = 1
    d.wbits = 1
    d.s[0], d.e[0] = out.ctypes.data, out.ctypes.data + out.nbytes
    C.memmove(d.args, bytes(a), C.sizeof(a))
    retired = C.c_uint64()
    assert sim.sim_run(4, 2, 1, descs, 4, None, 60.0, C.byref(retired)) == 0
    assert retired.value == 1
    assert np.all(np.abs(out.astype(np.float64) - exact) <= 1e-5 * np.maximum(np.abs(exact), mag))


@pytest.mark.timeout(180, method="thread")
@pytest.mark.parametrize("n,radius", [(8, None), (33, None), (64, None), (80, None),
                                      (2, 0.01), (2, 0.3), (64, 0.01), (64, 0.3), (65, 0.3),
                                      (137, None), (300, None), (257, 0.12), (700, 0.6), (1024, None)])
def test_rl_prefix_through_kernel_source(sim, n, radius):
    """One RL step through the kernel source: predict, broadphase, islands
    and permute (the one-wave paths for at most 64 bodies, the workgroup
    paths above), then the plan's Jacobi kernels and integrate, against the
    oracle's step: integer buffers and positions and velocities bit-exact.
    The edge scenes: the smallest scene, two bodies apart and touching, no
    contacts at all (every body an island of its own), one island of every
    body on either side of the one-wave limit, and scenes above 128 bodies
    (the cell grid, the sorted positions) including one dense enough for
    long islands, one whose radius makes a single cell, and the largest
    scene, whose lists do not fit in LDS (the all-pairs walk)."""
    sc = inputs.rl_scene(seed=11, n=n, radius=radius)
    off = acs.rl_layout(n)
    arena = np.zeros(int(off[acs.RL_END]), np.uint8)
    plan = np.zeros(acs.rl_plan_ints(n), np.int32)

    def region(r, dtype, count):
        return arena[int(off[r]):int(off[r]) + np.dtype(dtype).itemsize * count].view(dtype)
    region(acs.RL_X, np.float32, 4 * n)[:] = sc.x.reshape(-1)
    region(acs.RL_V, np.float32, 4 * n)[:] = sc.v.reshape(-1)
    kids = [acs.K_RL_PREDICT, acs.K_RL_BROADPHASE, acs.K_RL_ISLANDS, acs.K_RL_PERMUTE]
    descs = (SimDesc * len(kids))()
    for i, kid in enumerate(kids):
        a = acs.ArgsRL()
        a.base, a.plan, a.n, a.r, a.dt = arena.ctypes.data, plan.ctypes.data, n, float(sc.radius), float(sc.dt)
        d = descs[i]
        d.kid, d.npieces, d.nseg, d.wbits = kid, 1, 1, 1
        d.s[0], d.e[0] = arena.ctypes.data, arena.ctypes.data + arena.nbytes   # one chain
        C.memmove(d.args, bytes(a), C.sizeof(a))
    retired = C.c_uint64()
    assert sim.sim_run(4, 2, len(kids), descs, 8, None, 120.0, C.byref(retired)) == 0
    ref = O.Scene.from_inputs(sc)
    for op in (O.RL_PREDICT, O.RL_BROADPHASE, O.RL_ISLANDS, O.RL_PERMUTE):
        ref.run_kernel(op)
    assert np.array_equal(region(acs.RL_P, np.uint32, 4 * n), ref.P.view(np.uint32).reshape(-1))
    for r, name, cnt in ((acs.RL_DEG, "deg", n), (acs.RL_ADJ_OFF, "adj_off", n + 1), (acs.RL_LABEL, "label", n),
                         (acs.RL_PERM, "perm", n), (acs.RL_INV_PERM, "inv_perm", n),
                         (acs.RL_PADJ_OFF, "padj_off", n + 1)):
        assert np.array_equal(region(r, np.int32, cnt), getattr(ref, name)[:cnt]), name
    e = int(ref.adj_off[n])
    assert np.array_equal(region(acs.RL_ADJ, np.int32, e), ref.adj[:e])
    assert np.array_equal(region(acs.RL_PADJ, np.int32, e), ref.padj[:e])
    k = int(ref.meta[0])
    assert np.array_equal(region(acs.RL_ISL_OFF, np.int32, k + 1), ref.isl_off[:k + 1])
    m = int(ref.meta[1])
    if radius is not None:   # the edge scene is the one named
        assert (k, m) == ((n, 0) if radius < 0.05 else (1, 1))
    assert plan[0] == ref.meta[0] and plan[1] == ref.meta[1] and plan[2] == ref.meta[2]
    assert np.array_equal(plan[4:4 + 4 * m], ref.plan[:4 * m])
    assert np.array_equal(region(acs.RL_Q0, np.uint32, 4 * n), ref.Q0.view(np.uint32).reshape(-1))
    # the rest of the step from the plan just written: the Jacobi kernels
    # (iteration-major) and integrate, against the oracle's whole step
    tail = []
    for it in range(sc.iters):
        for q in range(m):
            tail.append((acs.K_RL_JACOBI, it, int(plan[4 + 4 * q]), int(plan[5 + 4 * q])))
    tail.append((acs.K_RL_INTEGRATE, 0, 0, 0))
    descs = (SimDesc * len(tail))()
    for i, (kid, it, b0, b1) in enumerate(tail):
        a = acs.ArgsRL()
        a.base, a.plan, a.n, a.r, a.dt = arena.ctypes.data, plan.ctypes.data, n, float(sc.radius), float(sc.dt)
        a.iter, a.b0, a.b1 = it, b0, b1
        d = descs[i]
        d.kid, d.npieces, d.nseg, d.wbits = kid, 1, 1, 1
        d.s[0], d.e[0] = arena.ctypes.data, arena.ctypes.data + arena.nbytes
        C.memmove(d.args, bytes(a), C.sizeof(a))
    assert sim.sim_run(4, 2, len(tail), descs, 8, None, 120.0, C.byref(retired)) == 0
    full = O.Scene.from_inputs(sc)
    full.step()
    assert np.array_equal(region(acs.RL_X, np.uint32, 4 * n), full.X.view(np.uint32).reshape(-1))
    assert np.array_equal(region(acs.RL_V, np.uint32, 4 * n), full.V.view(np.uint32).reshape(-1))


def group_trace(tr, ids, g, Wp):
    """The records of the kernels `ids` (global sequence numbers, in their
    group's program order) as a single-window trace of group g."""
    sub = tr[ids].copy()
    sub["seq"] = np.arange(len(ids))
    assert np.all(sub["slot"] // Wp == g)
    sub["slot"] = sub["slot"] % Wp
    m = np.uint64((1 << Wp) - 1)
    sub["valid_mask"] = (sub["valid_mask"] >> np.uint64(g * Wp)) & m
    sub["up_mask"] = (sub["up_mask"] >> np.uint64(g * Wp)) & m
    return sub


@pytest.mark.timeout(300, method="thread")
@pytest.mark.parametrize("G,W,workers", [(2, 8, 2), (4, 16, 3), (8, 8, 3), (3, 5, 2)])
def test_window_groups_through_kernel_source(sim, G, W, workers):
    """Independent tiny streams in the groups of one window wave: each
    stream's buffers bit-identical to its in-order run, each group's trace a
    valid windowed schedule of its own stream."""
    streams = [inputs.tiny_stream(100 + s, n_kernels=24) for s in range(G + 1)]   # one group gets two streams
    arenas = [st.init.copy() for st in streams]
    per = [(_descs(st, ar.ctypes.data), st) for st, ar in zip(streams, arenas)]
    group_of_stream = [s % G for s in range(len(streams))]
    # interleave the streams' kernels round robin; a group's streams stay in order
    order, pos = [], [0] * len(streams)
    while any(pos[s] < len(streams[s].kernels) for s in range(len(streams))):
        for s in range(len(streams)):
            if pos[s] < len(streams[s].kernels):
                order.append((s, pos[s]))
                pos[s] += 1
    n = len(order)
    descs = (SimDesc * n)()
    groups = np.zeros(n, np.int32)
    for i, (s, k) in enumerate(order):
        C.memmove(C.addressof(descs[i]), C.addressof(per[s][0][k]), C.sizeof(SimDesc))
        groups[i] = group_of_stream[s]
    tr = np.zeros(n, dtype=acs.TRACE_DTYPE)
    retired = C.c_uint64()
    sim.sim_run_groups.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint32,
                                   C.c_void_p, C.c_double, C.POINTER(C.c_uint64)]
    rc = sim.sim_run_groups(W, G, workers, n, descs, groups.ctypes.data, 16, tr.ctypes.data, 120.0, C.byref(retired))
    assert rc == 0 and retired.value == n
    for st, ar in zip(streams, arenas):
        assert np.array_equal(ar.view(np.uint32), O.tiny_run(st).view(np.uint32))
    Wp = 1 << (W - 1).bit_length()
    for g in range(G):
        ids = [i for i, (s, k) in enumerate(order) if group_of_stream[s] == g]
        accs = []
        for i in ids:
            s, k = order[i]
            accs.append(O.tiny_accesses(streams[s], base=(s + 1) << 40)[k])
        code, msg = O.check_trace(accs, W, group_trace(tr, ids, g, Wp), check_times=True, early=True)
        assert code == 0, (g, msg)


def host_lists(accs, M):
    """The host side of host-check mode, from the oracle's conflict test:
    bit d of entry j set when kernel j - 1 - d (d < M) conflicts with j."""
    out = np.zeros(len(accs), np.uint64)
    for j in range(len(accs)):
        for d in range(min(M, j)):
            if O.conflict(accs[j - 1 - d], accs[j]):
                out[j] |= np.uint64(1 << d)
    return out


def _run_hostcheck(sim, W, M, workers, descs, up, n, ring=64):
    sim.sim_run_hostcheck.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint32,
                                      C.c_void_p, C.c_double, C.POINTER(C.c_uint64)]
    tr = np.zeros(n, dtype=acs.TRACE_DTYPE)
    retired = C.c_uint64()
    rc = sim.sim_run_hostcheck(W, M, workers, n, descs, up.ctypes.data, ring, tr.ctypes.data, 120.0, C.byref(retired))
    assert rc == 0 and retired.value == n
    return tr


@pytest.mark.timeout(300, method="thread")
@pytest.mark.parametrize("seed,W,M,workers", [(0, 8, 8, 2), (1, 16, 4, 3), (2, 32, 64, 2), (3, 8, 1, 2),
                                              (4, 5, 12, 3)])
def test_host_check_mode_through_kernel_source(sim, seed, W, M, workers):
    """The host/device split: upstream lists computed on the host over the
    M previous kernels, filtered and gated in the window wave.  Same bits as
    in-order execution, and the trace passes the same checker as the device
    check (the upstream set at each insert is every conflicting kernel in the
    window, none missed)."""
    st = inputs.tiny_stream(seed)
    arena = st.init.copy()
    descs = _descs(st, arena.ctypes.data)
    accs = O.tiny_accesses(st, base=arena.ctypes.data)
    up = host_lists(accs, M)
    tr = _run_hostcheck(sim, W, M, workers, descs, up, len(st.kernels))
    assert np.array_equal(arena.view(np.uint32), O.tiny_run(st).view(np.uint32))
    code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
    assert code == 0, msg


def host_lists2(accs, M):
    """host_lists for M up to 128: bit d of lo[j] is the kernel j - 1 - d,
    bit d of hi[j] the kernel j - 65 - d."""
    lo = np.zeros(len(accs), np.uint64)
    hi = np.zeros(len(accs), np.uint64)
    for j in range(len(accs)):
        for d in range(min(M, j)):
            if O.conflict(accs[j - 1 - d], accs[j]):
                if d < 64:
                    lo[j] |= np.uint64(1 << d)
                else:
                    hi[j] |= np.uint64(1 << (d - 64))
    return lo, hi


@pytest.mark.timeout(300, method="thread")
@pytest.mark.parametrize("seed,W,M,workers", [(7, 16, 100, 3), (8, 64, 128, 2), (9, 8, 128, 2)])
def test_host_lists_longer_than_64_through_kernel_source(sim, seed, W, M, workers):
    """Host lists over up to 128 kernels (two words per list) on streams of
    200 kernels: same bits as in-order execution, and the trace passes the
    checker (every conflicting kernel in the window at insert is an
    upstream, including those 65 or more places back)."""
    st = inputs.tiny_stream(seed, n_kernels=200)
    arena = st.init.copy()
    descs = _descs(st, arena.ctypes.data)
    accs = O.tiny_accesses(st, base=arena.ctypes.data)
    lo, hi = host_lists2(accs, M)
    assert np.any(hi != 0)
    n = len(st.kernels)
    sim.sim_run_hostcheck2.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_uint32, C.c_void_p, C.c_double, C.POINTER(C.c_uint64)]
    tr = np.zeros(n, dtype=acs.TRACE_DTYPE)
    retired = C.c_uint64()
    rc = sim.sim_run_hostcheck2(W, M, workers, n, descs, lo.ctypes.data, hi.ctypes.data, 64, tr.ctypes.data, 120.0,
                                C.byref(retired))
    assert rc == 0 and retired.value == n
    assert np.array_equal(arena.view(np.uint32), O.tiny_run(st).view(np.uint32))
    code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
    assert code == 0, msg


@pytest.mark.timeout(300, method="thread")
def test_host_check_gate_holds_back_past_a_long_kernel(sim):
    """A long kernel writes byte 0, twenty short independent kernels follow,
    then one reads byte 0.  The host's list (M = 4) cannot see the long
    kernel from the reader; the gate keeps every kernel more than M younger
    out of the window until the long one is done, so the reader still waits."""
    buf = np.zeros(4096, np.uint8)
    base = buf.ctypes.data
    specs = [([], [(base, 1)], 3_000_000)] + [([], [(base + 64 * (i + 1), 1)], 0) for i in range(20)] + \
        [([(base, 1)], [(base + 2048, 1)], 0)]
    n = len(specs)
    descs = (SimDesc * n)()
    accs = []
    for i, (r, w, spin) in enumerate(specs):
        d = descs[i]
        d.kid, d.npieces = acs.K_NOP, 1
        segs = [(s, s + z) for s, z in r] + [(s, s + z) for s, z in w]
        d.nseg = len(segs)
        d.wbits = sum(1 << (len(r) + j) for j in range(len(w)))
        for j, (s0, e0) in enumerate(segs):
            d.s[j], d.e[j] = s0, e0
        a = bytes(acs.ArgsNop(spin))
        C.memmove(d.args, a, len(a))
        accs.append(O.make_access(r, w))
    M = 4
    up = host_lists(accs, M)
    assert up[n - 1] == 0                      # the reader's list misses the writer
    tr = _run_hostcheck(sim, 8, M, 3, descs, up, n)
    code, msg = O.check_trace(accs, 8, tr, check_times=True, early=True)
    assert code == 0, msg
    assert tr["t_start"][n - 1] >= tr["t_end"][0]
    # kernels M + 1 places after the long one were inserted only once it had left
    assert np.all(tr["ev_insert"][M + 1:] > tr["ev_retire"][0])


def _run_checkwave(sim, W, workers, descs, n, ring=64):
    sim.sim_run_checkwave.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_double,
                                      C.POINTER(C.c_uint64)]
    tr = np.zeros(n, dtype=acs.TRACE_DTYPE)
    retired = C.c_uint64()
    rc = sim.sim_run_checkwave(W, workers, n, descs, ring, tr.ctypes.data, 120.0, C.byref(retired))
    assert rc == 0 and retired.value == n
    return tr


@pytest.mark.timeout(300, method="thread")
@pytest.mark.parametrize("seed,W,workers,ring", [(0, 8, 2, 64), (1, 16, 3, 16), (2, 32, 2, 64), (5, 64, 3, 128),
                                                 (6, 3, 2, 8)])
def test_check_wave_mode_through_kernel_source(sim, seed, W, workers, ring):
    """The split made inside the device: the check wave tests each staged
    kernel against the 64 submitted before it, the window wave keeps the
    ones still in the window.  Same bits as in-order execution, and the
    trace passes the checker (every conflicting kernel in the window is an
    upstream kernel at insert, none missed, none extra)."""
    st = inputs.tiny_stream(seed, n_kernels=160)
    arena = st.init.copy()
    descs = _descs(st, arena.ctypes.data)
    tr = _run_checkwave(sim, W, workers, descs, len(st.kernels), ring)
    assert np.array_equal(arena.view(np.uint32), O.tiny_run(st).view(np.uint32))
    code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
    assert code == 0, msg


def random_nop_descs(seed, n, base):
    """n no-op kernels with 0-3 writes and 0-4 reads (at least one range)
    over a small address range, so that reads meet reads, writes and
    partial overlaps; returns the descriptors and the oracle's accesses."""
    g = np.random.default_rng(seed)
    descs = (SimDesc * n)()
    accs = []
    for i in range(n):
        nw, nr = int(g.integers(0, 4)), int(g.integers(0, 5))
        if nw + nr == 0:
            nw = 1
        rng = [(base + int(g.integers(0, 4000)), int(g.integers(1, 300))) for _ in range(nw + nr)]
        r, w = rng[:nr], rng[nr:]
        d = descs[i]
        d.kid, d.npieces = acs.K_NOP, 1
        segs = [(s0, s0 + z) for s0, z in r] + [(s0, s0 + z) for s0, z in w]
        d.nseg = len(segs)
        d.wbits = sum(1 << (nr + j) for j in range(nw))
        for j, (s0, e0) in enumerate(segs):
            d.s[j], d.e[j] = s0, e0
        a = bytes(acs.ArgsNop(0))
        C.memmove(d.args, a, len(a))
        accs.append(O.make_access(r, w))
    return descs, accs


@pytest.mark.timeout(300, method="thread")
@pytest.mark.parametrize("seed,W,n,ring", [(0, 16, 300, 64), (1, 64, 300, 64), (2, 5, 300, 64), (3, 64, 700, 16)])
def test_check_wave_mixed_write_counts(sim, seed, W, n, ring):
    """Kernels with different numbers of writes (so that a kernel's first
    positions are writes for some and reads for others): the upstream mask
    recorded at every insert is exactly the window's conflicting kernels.
    700 kernels wrap the staging ring several times while the two check
    waves alternate."""
    buf = np.zeros(4096 + 512, np.uint8)
    descs, accs = random_nop_descs(seed, n, buf.ctypes.data)
    tr = _run_checkwave(sim, W, 3, descs, len(accs), ring)
    code, msg = O.check_trace(accs, W, tr, check_times=True, early=True)
    assert code == 0, msg


@pytest.mark.timeout(300, method="thread")
def test_check_wave_gate_holds_back_past_a_long_kernel(sim):
    """A long kernel writes byte 0, seventy independent kernels follow, then
    one reads byte 0: seventy-one places back, out of the check wave's reach.
    The gate keeps every kernel more than 64 younger than the long one out
    of the window until it is done, so the reader still waits for it."""
    buf = np.zeros(8192, np.uint8)
    base = buf.ctypes.data
    specs = [([], [(base, 1)], 3_000_000)] + [([], [(base + 64 * (i + 1), 1)], 0) for i in range(70)] + \
        [([(base, 1)], [(base + 6000, 1)], 0)]
    n = len(specs)
    descs = (SimDesc * n)()
    accs = []
    for i, (r, w, spin) in enumerate(specs):
        d = descs[i]
        d.kid, d.npieces = acs.K_NOP, 1
        segs = [(s0, s0 + z) for s0, z in r] + [(s0, s0 + z) for s0, z in w]
        d.nseg = len(segs)
        d.wbits = sum(1 << (len(r) + j) for j in range(len(w)))
        for j, (s0, e0) in enumerate(segs):
            d.s[j], d.e[j] = s0, e0
        a = bytes(acs.ArgsNop(spin))
        C.memmove(d.args, a, len(a))
        accs.append(O.make_access(r, w))
    tr = _run_checkwave(sim, 16, 3, descs, n)
    code, msg = O.check_trace(accs, 16, tr, check_times=True, early=True)
    assert code == 0, msg
    assert tr["t_start"][n - 1] >= tr["t_end"][0]
    assert np.all(tr["ev_insert"][65:] > tr["ev_retire"][0])


@pytest.mark.timeout(120, method="thread")
def test_check_wave_mode_abort_releases_every_wave(sim):
    """An abort while kernels are still queued behind a long one: the host
    gives up after 0.3 s and sets the abort flag; the window, FIFO and check
    waves and every worker leave (the call returns), with the long kernel's
    followers not retired."""
    buf = np.zeros(8192, np.uint8)
    base = buf.ctypes.data
    n = 120
    descs = (SimDesc * n)()
    for i in range(n):
        d = descs[i]
        d.kid, d.npieces, d.nseg, d.wbits = acs.K_NOP, 1, 1, 1
        d.s[0], d.e[0] = (base, base + 1) if i % 3 == 0 else (base + 64 * i, base + 64 * i + 1)
        a = bytes(acs.ArgsNop(1_500_000_000 if i == 0 else 0))
        C.memmove(d.args, a, len(a))
    sim.sim_run_checkwave.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_uint32, C.c_void_p, C.c_double,
                                      C.POINTER(C.c_uint64)]
    retired = C.c_uint64()
    t0 = time.perf_counter()
    rc = sim.sim_run_checkwave(8, 2, n, descs, 16, None, 0.3, C.byref(retired))
    assert rc == -5
    assert retired.value < n
    assert time.perf_counter() - t0 < 30


@pytest.mark.timeout(300, method="thread")
def test_join_pool_fc_bodies_through_kernel_source(sim):
    """The elementwise join (vector and scalar tails, several pieces), the
    average pool and the head with lengths that are not multiples of their
    16-wide load blocks: bit-identical to the oracle."""
    g = np.random.default_rng(3)
    n = 2048 * 3 + 7
    a, b = g.uniform(-1, 1, n).astype(np.float32), g.uniform(-1, 1, n).astype(np.float32)
    o1, o2 = np.full(n, np.nan, np.float32), np.full(n, np.nan, np.float32)
    hw, c = 20, 40
    x = g.uniform(-1, 1, (hw, c)).astype(np.float32)
    pool = np.full(c, np.nan, np.float32)
    w, bias = g.uniform(-1, 1, (c, 10)).astype(np.float32), g.uniform(-1, 1, 10).astype(np.float32)
    out = np.full(10, np.nan, np.float32)
    specs = [(acs.K_JOIN, acs.ArgsJoin(o1.ctypes.data, a.ctypes.data, b.ctypes.data, n), 4, [o1]),
             (acs.K_JOIN, acs.ArgsJoin(o2.ctypes.data, a.ctypes.data, 0, n), 4, [o2]),
             (acs.K_AVGPOOL, acs.ArgsAvgpool(pool.ctypes.data, x.ctypes.data, hw, c), 1, [pool]),
             (acs.K_FC, acs.ArgsFC(out.ctypes.data, pool.ctypes.data, w.ctypes.data, bias.ctypes.data, c, 10), 1,
              [out])]
    descs = (SimDesc * len(specs))()
    for i, (kid, args, np_, writes) in enumerate(specs):
        d = descs[i]
        d.kid, d.npieces = kid, np_
        # the head reads the pool: give both the pool's range so they stay ordered
        rng = [(int(pool.ctypes.data), int(pool.ctypes.data) + pool.nbytes)] if kid in (acs.K_AVGPOOL, acs.K_FC) else []
        segs = rng + [(int(t.ctypes.data), int(t.ctypes.data) + t.nbytes) for t in writes]
        d.nseg = len(segs)
        d.wbits = (1 << len(segs)) - 1
        for j, (s0, e0) in enumerate(segs):
            d.s[j], d.e[j] = s0, e0
        C.memmove(d.args, bytes(args), C.sizeof(args))
    retired = C.c_uint64()
    assert sim.sim_run(4, 2, len(specs), descs, 8, None, 120.0, C.byref(retired)) == 0
    assert retired.value == len(specs)
    assert np.array_equal(o1.view(np.uint32), O.join(a, b).view(np.uint32))
    assert np.array_equal(o2.view(np.uint32), O.join(a).view(np.uint32))
    assert np.array_equal(pool.view(np.uint32), O.avgpool(x.reshape(hw, 1, c)).view(np.uint32))
    assert np.array_equal(out.view(np.uint32), O.fc(O.avgpool(x.reshape(hw, 1, c)), w, bias).view(np.uint32))
