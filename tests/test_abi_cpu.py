"""CPU tests of libacs: exports, argument checks, submission normalisation,
range helpers, and the host window through the manual path (no GPU).

The window's decisions are checked against the oracle: its DAG gives the
reference ready sets and its trace checker validates every schedule.
"""
import itertools
import json
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import acs, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(acs.LIB_PATH):
        from paper_2401_12377_amd import build
        build.build()
    return acs.lib()


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(acs_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 19
    out = subprocess.run(["nm", "-D", "--defined-only", acs.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = names - exported
    assert not missing, missing


def manual(W, **kw):
    return acs.Window(W, path="manual", **kw)


NOP = acs.ArgsNop(0)


def sub(win, reads, writes):
    return win.submit(acs.K_NOP, reads, writes, NOP)


def test_window_size_limits():
    for bad in (0, -1, 65):
        with pytest.raises(acs.AcsError) as e:
            acs.Window(bad, path="manual")
        assert e.value.code == acs.EINVAL
    for ok in (1, 64):
        manual(ok).destroy()


def test_submit_argument_checks():
    w = manual(4)
    rc, _ = w.submit_raw(99, [], [(0, 4)], bytes(8))
    assert rc == acs.EINVAL                         # unknown kernel id
    rc, _ = w.submit_raw(acs.K_NOP, [], [(0, 4)], bytes(12))
    assert rc == acs.EINVAL                         # args size mismatch
    rc, _ = w.submit_raw(acs.K_NOP, [], [(2 ** 64 - 8, 16)], bytes(8))
    assert rc == acs.EINVAL                         # range wraps
    rc, _ = w.submit_raw(acs.K_NOP, [], [acs.SEG_ALL], bytes(8))
    assert rc == acs.OK                             # the all-memory range is allowed
    s = acs.ArgsSum()
    s.nin = 0
    rc, _ = w.submit_raw(acs.K_SUM, [], [(0, 4)], bytes(s))
    assert rc == acs.EINVAL                         # sum needs 1..3 inputs
    r = acs.ArgsRL()
    r.n = 5000
    rc, _ = w.submit_raw(acs.K_RL_PREDICT, [], [(0, 4)], bytes(r))
    assert rc == acs.EINVAL                         # scene too large
    w.destroy()


def test_configure_rejects_bad_values():
    for kw in (dict(n_streams=0), dict(wg_per_task=0), dict(wg_per_task=300), dict(queue_depth=0),
               dict(trace=True, trace_capacity=0)):
        with pytest.raises(acs.AcsError) as e:
            acs.Window(4, path="manual", **kw)
        assert e.value.code == acs.EINVAL


def test_window_of_one_is_serial():
    w = manual(1)
    seqs = [sub(w, [], [(100 * i, 8)]) for i in range(5)]      # all independent
    order = []
    for _ in range(5):
        r = w.take_ready()
        assert len(r) == 1
        order.append(r[0])
        w.complete(r[0])
    assert order == seqs
    assert w.sync() == 0
    w.destroy()


def test_disjoint_kernels_all_ready():
    w = manual(8, queue_depth=64)
    for i in range(8):
        sub(w, [(1000 + 16 * i, 16)], [(16 * i, 16)])
    assert sorted(w.take_ready()) == list(range(8))
    w.destroy()


def test_raw_chain_is_serial():
    w = manual(8)
    for i in range(6):
        sub(w, [(8 * i, 8)], [(8 * (i + 1), 8)])   # k_i reads what k_{i-1} wrote
    for i in range(6):
        r = w.take_ready()
        assert r == [i]
        w.complete(i)
    w.destroy()


def test_all_memory_kernel_is_a_barrier():
    w = manual(16, queue_depth=64)
    for i in range(3):
        sub(w, [], [(64 * i, 8)])
    sub(w, [acs.SEG_ALL], [acs.SEG_ALL])
    for i in range(3):
        sub(w, [], [(64 * i + 4096, 8)])
    assert sorted(w.take_ready()) == [0, 1, 2]
    for s in (0, 1, 2):
        w.complete(s)
    assert w.take_ready() == [3]
    w.complete(3)
    assert sorted(w.take_ready()) == [4, 5, 6]
    w.destroy()


def test_read_after_write_is_a_dependency():
    """The case Algorithm 1 as printed misses: the newer kernel only reads
    what the older one writes."""
    w = manual(4)
    sub(w, [], [(0, 64)])
    sub(w, [(0, 64)], [(64, 64)])
    assert w.take_ready() == [0]
    w.complete(0)
    assert w.take_ready() == [1]
    w.destroy()


def test_scheduled_list_states():
    w = manual(4, queue_depth=16)
    sub(w, [], [(0, 8)])
    sub(w, [(0, 8)], [(8, 8)])
    sub(w, [], [(100, 8)])
    lst = w.scheduled_list()
    assert [e[0] for e in lst] == [0, 1, 2]
    st = {e[0]: e[2] for e in lst}
    assert st == {0: acs.READY, 1: acs.PENDING, 2: acs.READY}
    up = {e[0]: e[3] for e in lst}
    slot = {e[0]: e[4] for e in lst}
    assert up[1] == 1 << slot[0]
    w.take_ready()
    st = {e[0]: e[2] for e in w.scheduled_list()}
    assert st == {0: acs.EXECUTING, 1: acs.PENDING, 2: acs.EXECUTING}
    w.destroy()


def reference_ready(adj, window, executing):
    """Ready set from the oracle's DAG: in the window, not executing, no older
    conflicting kernel still in the window."""
    return sorted(j for j in window if j not in executing and not any(adj[i, j] for i in window if i < j))


def drive(accs, W, pick, fifo=4096):
    """Runs a manual window; pick(ready_running) chooses which kernel completes."""
    adj = O.dag(accs)
    w = manual(W, trace=True, queue_depth=fifo)
    for a in accs:
        w.submit(acs.K_NOP, a.reads(), a.writes(), NOP)
    n = len(accs)
    window, running, done = [], set(), set()
    nxt = 0
    while len(done) < n:
        while nxt < n and len(window) < W:
            window.append(nxt)
            nxt += 1
        want = reference_ready(adj, window, running)
        got = sorted(w.take_ready())
        assert got == want
        running |= set(got)
        j = pick(sorted(running))
        w.complete(j)
        running.discard(j)
        window.remove(j)
        done.add(j)
    assert w.sync() == 0
    tr = w.trace()
    code, msg = O.check_trace(accs, W, tr)
    w.destroy()
    assert code == 0, msg
    return tr


@pytest.mark.parametrize("W", [1, 2, 3, 8, 64])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_completion_orders_match_oracle(W, seed):
    st = inputs.tiny_stream(seed)
    accs = O.tiny_accesses(st, base=1 << 32)
    rng = np.random.default_rng(seed * 100 + W)
    drive(accs, W, lambda run: run[int(rng.integers(len(run)))])


def test_every_completion_order_small_stream():
    st = inputs.tiny_stream(4, n_kernels=6)
    accs = O.tiny_accesses(st)
    for W in (2, 3, 6):
        # enumerate completion choices by index into the running list
        for choice in itertools.product(range(3), repeat=6):
            it = iter(choice)
            drive(accs, W, lambda run: run[next(it) % len(run)])


def test_fifo_backpressure_in_manual_mode():
    w = manual(2, queue_depth=2)
    for i in range(4):
        sub(w, [], [(0, 8)])                      # a chain through one range
    rc, _ = w.submit_raw(acs.K_NOP, [], [(0, 8)], bytes(NOP))
    assert rc == acs.EAGAIN
    assert w.sync_rc() == acs.ETIMEDOUT          # nothing completes by itself in manual mode
    for i in range(4):
        r = w.take_ready()
        assert r == [i]
        w.complete(i)
    assert w.sync() == 0
    w.destroy()


def test_failed_kernel_poisons_dependents_only():
    w = manual(8, queue_depth=64)
    a = sub(w, [], [(0, 8)])            # will fail
    b = sub(w, [(0, 8)], [(8, 8)])      # reads a's output: poisoned
    c = sub(w, [], [(100, 8)])          # independent
    d = sub(w, [(8, 8)], [(200, 8)])    # depends on b: poisoned transitively
    assert sorted(w.take_ready()) == [a, c]
    w.complete(a, status=-6)
    w.complete(c)
    assert w.take_ready() == []         # b and d retire without running
    e = sub(w, [(0, 4)], [(300, 8)])    # admitted after a retired: still sees the failure
    f = sub(w, [], [(400, 8)])
    assert w.take_ready() == [f]
    w.complete(f)
    assert w.sync_rc() == acs.EKERNEL
    s = w.stats()
    assert s["poisoned"] == 3 and s["retired"] == 6
    w.destroy()


def test_coalescing_is_conservative():
    rng = np.random.default_rng(3)
    for _ in range(200):
        nr, nw = int(rng.integers(0, 12)), int(rng.integers(0, 12))
        reads = [(int(rng.integers(0, 4000)), int(rng.integers(1, 50))) for _ in range(nr)]
        writes = [(int(rng.integers(0, 4000)), int(rng.integers(1, 50))) for _ in range(nw)]
        probe_r = [(int(rng.integers(0, 4000)), int(rng.integers(1, 50)))]
        probe_w = [(int(rng.integers(0, 4000)), int(rng.integers(1, 50)))]
        w = manual(2)
        sub(w, reads, writes)
        sub(w, probe_r, probe_w)
        lst = w.scheduled_list()
        got = lst[1][3] != 0
        want = O.conflict(O.make_access(reads, writes), O.make_access(probe_r, probe_w))
        if want:
            assert got
        if nr + nw <= acs.K_MAX:
            assert got == want
        w.destroy()


def test_lossy_merge_of_one_kind_is_counted():
    """Ten disjoint reads and no write do not fit ACS_K_MAX positions: the
    merge adds bytes, which is recorded, and stays conservative."""
    w = manual(2)
    reads = [(1000 * i, 10) for i in range(10)]
    sub(w, reads, [])
    assert w.stats()["coalesced"] == 1
    sub(w, [], [(1500, 1)])                 # a write into a gap the merge covered
    assert w.scheduled_list()[1][3] != 0
    w.destroy()
    w = manual(2)
    sub(w, [(1000 * i, 10) for i in range(8)], [])   # eight fit: exact
    assert w.stats()["coalesced"] == 0
    w.destroy()


def test_more_than_sixty_four_ranges():
    """Lists longer than the on-stack capacity spill to the heap (twice for
    100 and 200 ranges) and still give a conservative, counted merge."""
    rng = np.random.default_rng(11)
    for n in (33, 65, 100, 200):
        reads = [(int(s), 7) for s in rng.choice(1 << 20, size=n, replace=False) * 16]
        writes = [(int(s), 5) for s in rng.choice(1 << 20, size=n // 2, replace=False) * 16 + (1 << 25)]
        w = manual(2)
        sub(w, reads, writes)
        assert w.stats()["coalesced"] == 1
        for r in reads[:10] + [(reads[-1][0] + 3, 1)]:
            sub(w, [], [r])
            lst = w.scheduled_list()
            assert lst[-1][3] != 0, (n, r)
            w.destroy()
            w = manual(2)
            sub(w, reads, writes)
        w.destroy()


def test_rl_driver_rejects_odd_sweep_counts():
    """Sweeps alternate between the two position buffers and integrate reads
    the first: an odd count is refused before anything is submitted."""
    import ctypes as C
    plan = (C.c_int32 * 64)()
    for iters, want in ((1, acs.EINVAL), (7, acs.EINVAL), (-2, acs.EINVAL)):
        sc = acs.RLSceneC(16, iters, 0.1, 1.0 / 120, 1 << 30, C.cast(plan, C.c_void_p))
        w = manual(8)
        steps = (C.c_double * 1)()
        cnt = acs.RLCounts()
        assert acs.lib().acs_rl_run(w.handle, C.byref(sc), 1, steps, C.byref(cnt)) == want
        assert w.stats()["submitted"] == 0
        w.destroy()


def test_package_tiny_ranges_equal_oracle_ranges():
    st = inputs.tiny_stream(7)
    base = 1 << 36
    ours = [acs.tiny_kernel_task(st, k, base) for k in st.kernels]
    theirs = O.tiny_accesses(st, base=base)
    for (kid, r, w, _), a in zip(ours, theirs):
        assert sorted(r) == sorted(a.reads())
        assert sorted(w) == sorted(a.writes())


def test_gemm_ranges_match_the_paper_example():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "get_addresses_matmul.json")))
    for c in g["cases"]:
        r, w = acs.gemm_segments(c["a"], c["b"], c["c"], c["m"], c["n"], c["k"], g["elem_size"])
        assert [list(x) for x in r] == c["reads"]
        assert [list(x) for x in w] == c["writes"]


def test_rl_layout_is_contiguous_and_aligned():
    for n in (2, 16, 64, 511, 1024):
        off = acs.rl_layout(n)
        assert np.all(off % 256 == 0) and np.all(np.diff(off) >= 0)
        assert off[acs.RL_ADJ_OFF] - off[acs.RL_DEG] >= 4 * n
        assert off[acs.RL_END] - off[acs.RL_PADJ] >= 4 * n * (n - 1)
    with pytest.raises(acs.AcsError):
        acs.rl_layout(1)
    with pytest.raises(acs.AcsError):
        acs.rl_layout(2000)


# ---------------------------------------------------------------------------
# the native DNN driver's ranges, on the manual path (no GPU, no memory touched)
# ---------------------------------------------------------------------------
def fake_dnn_graph(cells, classes):
    """A graph whose tensors are disjoint fake address ranges."""
    nxt = [1 << 40]

    def alloc(nbytes):
        p = nxt[0]
        nxt[0] += (nbytes + 4095) // 4096 * 4096 + 4096
        return p
    g = acs.DNNGraphC()
    g.n_cells, g.classes = len(cells), classes
    h0, c0 = cells[0][0], cells[0][1]
    g.x = alloc(4 * h0 * h0 * c0)
    for c, (h, cin, cout, st) in enumerate(cells):
        L = g.cell[c]
        L.hin, L.cin, L.cout, L.stride = h, cin, cout, st
        L.w3, L.b3 = alloc(36 * cin * cout), alloc(4 * cout)
        L.w1, L.b1 = alloc(4 * cin * cout), alloc(4 * cout)
        ho = h // st
        L.t3, L.t1, L.y = (alloc(4 * ho * ho * cout) for _ in range(3))
    g.pool = alloc(4 * cells[-1][2])
    g.fc_w, g.fc_b, g.out = alloc(4 * cells[-1][2] * classes), alloc(4 * classes), alloc(4 * classes)
    return g


@pytest.mark.parametrize("seed", [0, 1, 2, 5])
def test_dnn_driver_dependencies_match_oracle_dataflow(seed):
    inp = inputs.dnn_input(seed)
    net = O.DNN(inputs.dnn_weights(), inp, inputs.DNN_CELLS)
    adj = O.dag(net.accesses())
    n = len(net.kernels())
    W = 16
    w = manual(W, trace=True, queue_depth=4096)
    g = fake_dnn_graph(inputs.DNN_CELLS, inputs.DNN_CLASSES)
    lg = np.ascontiguousarray(inp.logits, np.float32).reshape(-1)
    cnt = acs.C.c_uint64()
    assert acs.lib().acs_dnn_submit(w.handle, acs.C.byref(g), lg.ctypes.data, acs.C.byref(cnt)) == 0
    assert cnt.value == n
    rng = np.random.default_rng(seed)
    window, running, done, nxt = [], set(), set(), 0
    while len(done) < n:
        while nxt < n and len(window) < W:
            window.append(nxt)
            nxt += 1
        got = sorted(w.take_ready())
        assert got == reference_ready(adj, window, running)
        running |= set(got)
        j = sorted(running)[int(rng.integers(len(running)))]
        w.complete(j)
        running.discard(j)
        window.remove(j)
        done.add(j)
    assert w.sync() == 0
    code, msg = O.check_trace(net.accesses(), W, w.trace())
    w.destroy()
    assert code == 0, msg


def test_conv_argument_checks():
    w = manual(4)
    good = acs.ArgsConv(1 << 20, 2 << 20, 3 << 20, 4 << 20, 8, 32, 32, 3, 1)
    rc, _ = w.submit_raw(acs.K_CONV, [], [(4 << 20, 4)], bytes(good))
    assert rc == acs.OK
    for field, val in (("k", 2), ("stride", 3), ("cin", 16), ("cout", 48), ("hin", 6)):
        a = acs.ArgsConv(1 << 20, 2 << 20, 3 << 20, 4 << 20, 8, 32, 32, 3, 1)
        setattr(a, field, val)
        rc, _ = w.submit_raw(acs.K_CONV, [], [(4 << 20, 4)], bytes(a))
        assert rc == acs.EINVAL, field
    w.destroy()


def test_graph_recording_states():
    w = manual(4)
    with pytest.raises(acs.AcsError) as e:
        w.graph_end()
    assert e.value.code == acs.ESTATE                 # not recording
    w.graph_begin()
    with pytest.raises(acs.AcsError) as e:
        w.graph_begin()
    assert e.value.code == acs.ESTATE                 # already recording
    with pytest.raises(acs.AcsError) as e:
        w.graph_end()
    assert e.value.code == acs.EINVAL                 # nothing recorded
    # recorded kernels do not reach the window
    w.graph_begin()
    s0 = sub(w, [], [(0, 8)])
    s1 = sub(w, [(0, 8)], [(8, 8)])
    assert (s0, s1) == (0, 1)
    assert w.take_ready() == []
    w.destroy()


def test_host_check_depth_validation():
    for kw in ({"host_check_depth": 129}, {"host_check_depth": -1}, {"host_check_depth": 4, "n_groups": 2}):
        with pytest.raises(acs.AcsError) as e:
            acs.Window(8, path="device", **kw)
        assert e.value.code == acs.EINVAL
    # the host's list may be longer than the window (up to 128 kernels); the
    # range is checked on every path
    with pytest.raises(acs.AcsError):
        acs.Window(8, path="manual", host_check_depth=129)
    acs.Window(8, path="manual", host_check_depth=128).destroy()
    # other paths accept and ignore it
    with acs.Window(8, path="manual", host_check_depth=4) as w:
        w.submit(acs.K_NOP, [], [(0, 1)], acs.ArgsNop(0))


def test_window_check_validation():
    for v in (2, -1):
        with pytest.raises(acs.AcsError) as e:
            acs.Window(8, path="device", window_check=v)
        assert e.value.code == acs.EINVAL
    with pytest.raises(acs.AcsError):
        acs.Window(8, path="manual", window_check=3)
    # other paths accept and ignore it
    with acs.Window(8, path="manual", window_check=1) as w:
        w.submit(acs.K_NOP, [], [(0, 1)], acs.ArgsNop(0))


def fake_dag_graph(graph):
    nxt = [1 << 40]

    def alloc(nbytes):
        p = nxt[0]
        nxt[0] += (nbytes + 4095) // 4096 * 4096 + 4096
        return p
    h, c, k = graph.h, graph.c, graph.classes
    g = acs.DAGGraphC()
    g.n_nodes, g.h, g.c, g.classes = len(graph.preds), h, c, k
    g.x = alloc(4 * h * h * c)
    for i, ps in enumerate(graph.preds):
        nd = g.node[i]
        nd.n_in = len(ps)
        for q, p in enumerate(ps):
            nd.inp[q] = p
        nd.w, nd.b, nd.agg, nd.y = alloc(36 * c * c), alloc(4 * c), alloc(4 * h * h * c), alloc(4 * h * h * c)
    g.sink, g.pool = alloc(4 * h * h * c), alloc(4 * c)
    g.fc_w, g.fc_b, g.out = alloc(4 * c * k), alloc(4 * k), alloc(4 * k)
    return g


@pytest.mark.parametrize("seed", [5, 7])
def test_dag_driver_dependencies_match_oracle_dataflow(seed):
    graph = inputs.dag_graph(seed=seed)
    net = O.StaticDAG(graph, None, None)
    adj = O.dag(net.accesses())
    n = len(net.kernels())
    W = 16
    w = manual(W, trace=True, queue_depth=4096)
    cnt = acs.C.c_uint64()
    assert acs.lib().acs_dag_submit(w.handle, acs.C.byref(fake_dag_graph(graph)), acs.C.byref(cnt)) == 0
    assert cnt.value == n
    rng = np.random.default_rng(seed)
    window, running, done, nxt = [], set(), set(), 0
    while len(done) < n:
        while nxt < n and len(window) < W:
            window.append(nxt)
            nxt += 1
        got = sorted(w.take_ready())
        assert got == reference_ready(adj, window, running)
        running |= set(got)
        j = sorted(running)[int(rng.integers(len(running)))]
        w.complete(j)
        running.discard(j)
        window.remove(j)
        done.add(j)
    assert w.sync() == 0
    code, msg = O.check_trace(net.accesses(), W, w.trace())
    w.destroy()
    assert code == 0, msg


def test_dag_driver_rejects_malformed_graphs():
    graph = inputs.dag_graph(nodes=8)
    for mutate in ("forward_edge", "too_many_inputs", "bad_shape"):
        g = fake_dag_graph(graph)
        if mutate == "forward_edge":
            g.node[3].n_in, g.node[3].inp[0] = 1, 5
        elif mutate == "too_many_inputs":
            g.node[3].n_in = 9
        else:
            g.c = 48
        w = manual(16)
        assert acs.lib().acs_dag_submit(w.handle, acs.C.byref(g), None) == acs.EINVAL, mutate
        assert w.stats()["submitted"] == 0, mutate           # nothing went in before the check
        w.destroy()


def test_check_probe_counts_every_segment_pair():
    """The host check-cost probe (the overhead table of Section IV-D): with
    W - 1 resident kernels of S segments (S/2 reads, the rest writes, all
    disjoint), each check tests the new kernel's writes against every range
    and its reads against the writes of every resident kernel."""
    import ctypes as C
    L = acs.lib()
    for W, S in ((16, 6), (32, 6), (4, 2)):
        a, b, t = C.c_double(), C.c_double(), C.c_double()
        assert L.acs_check_probe(W, S, 2000, C.byref(a), C.byref(b), C.byref(t)) == 0
        nr = S // 2
        nw = S - nr
        assert t.value == (W - 1) * (nw * S + nr * nw)
        assert a.value > 0 and b.value > 0
    assert L.acs_check_probe(1, 6, 10, C.byref(a), C.byref(b), None) == acs.EINVAL
