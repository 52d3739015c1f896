"""Pins for the oracle's trace checker.

A tiny test-side simulator produces schedules by hand (it picks which running
kernel completes next at random); the checker must accept every such schedule
and reject each planted mistake: a dropped or extra upstream bit, a dispatch
before an upstream retires, an admission out of program order, an
over-full window and overlapping execution of conflicting kernels.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import inputs


def simulate(accs, W, rng, adj):
    """A hand-written window schedule (test helper, not a reference model)."""
    n = len(accs)
    tr = np.zeros(n, dtype=O.TRACE_DTYPE)
    tr["seq"] = np.arange(n)
    tr["t_start"] = -1
    tr["t_end"] = -1
    tr["t_dispatch"] = -1
    tr["t_retire"] = -1
    ev = 0
    window = {}          # slot -> seq
    running = set()
    dispatched = set()
    nxt = 0
    clock = 0
    while nxt < n or window:
        # admit in program order while a slot is free
        while nxt < n and len(window) < W:
            slot = min(set(range(W)) - set(window))
            valid = 0
            up = 0
            for s, i in window.items():
                valid |= 1 << s
                if adj[i, nxt]:
                    up |= 1 << s
            tr[nxt]["slot"] = slot
            tr[nxt]["valid_mask"] = valid
            tr[nxt]["up_mask"] = up
            tr[nxt]["ev_insert"] = ev
            ev += 1
            window[slot] = nxt
            nxt += 1
        # dispatch every ready kernel
        for s, j in sorted(window.items(), key=lambda t: t[1]):
            if j in dispatched:
                continue
            if all(not adj[i, j] for i in window.values() if i < j):
                tr[j]["ev_dispatch"] = ev
                ev += 1
                clock += 1
                tr[j]["t_start"] = clock
                dispatched.add(j)
                running.add(j)
        # complete one running kernel, chosen at random
        j = sorted(running)[int(rng.integers(len(running)))]
        running.remove(j)
        clock += 1
        tr[j]["t_end"] = clock
        tr[j]["ev_retire"] = ev
        ev += 1
        del window[int(tr[j]["slot"])]
    return tr


@pytest.fixture(params=[1, 2, 8, 64])
def setup(request):
    W = request.param
    st = inputs.tiny_stream(request.param + 100)
    accs = O.tiny_accesses(st)
    adj = O.dag(accs)
    tr = simulate(accs, W, np.random.default_rng(W), adj)
    return W, accs, adj, tr


def test_valid_schedules_pass(setup):
    W, accs, adj, tr = setup
    code, msg = O.check_trace(accs, W, tr, check_times=True)
    assert code == 0, msg


def test_dropped_upstream_bit_is_caught(setup):
    W, accs, adj, tr = setup
    cand = [j for j in range(len(tr)) if tr[j]["up_mask"]]
    if not cand:
        pytest.skip("no kernel had an upstream kernel in the window")
    j = cand[0]
    m = int(tr[j]["up_mask"])
    tr[j]["up_mask"] = m & (m - 1)
    code, msg = O.check_trace(accs, W, tr)
    assert code == 16, msg


def test_extra_upstream_bit_is_caught(setup):
    W, accs, adj, tr = setup
    cand = [j for j in range(len(tr)) if int(tr[j]["valid_mask"]) & ~int(tr[j]["up_mask"])]
    if not cand:
        pytest.skip("no independent kernel shared the window")
    j = cand[0]
    extra = int(tr[j]["valid_mask"]) & ~int(tr[j]["up_mask"])
    tr[j]["up_mask"] = int(tr[j]["up_mask"]) | (extra & -extra)
    code, msg = O.check_trace(accs, W, tr)
    assert code == 16, msg


def test_early_dispatch_is_caught(setup):
    W, accs, adj, tr = setup
    pairs = [(i, j) for i in range(len(tr)) for j in range(i + 1, len(tr)) if adj[i, j]]
    i, j = pairs[0]
    tr[j]["ev_dispatch"] = tr[i]["ev_retire"] - 1
    if tr[j]["ev_dispatch"] <= tr[j]["ev_insert"]:
        tr[j]["ev_insert"] = tr[j]["ev_dispatch"] - 1
    code, msg = O.check_trace(accs, W, tr)
    assert code != 0, msg


def test_out_of_order_admission_is_caught(setup):
    W, accs, adj, tr = setup
    tr[3]["ev_insert"], tr[4]["ev_insert"] = tr[4]["ev_insert"], tr[3]["ev_insert"]
    code, msg = O.check_trace(accs, W, tr)
    assert code != 0, msg


def test_window_overflow_is_caught():
    st = inputs.tiny_stream(5)
    accs = O.tiny_accesses(st)
    adj = O.dag(accs)
    tr = simulate(accs, 8, np.random.default_rng(0), adj)
    code, msg = O.check_trace(accs, 4, tr)      # schedule made with W=8 checked against W=4
    assert code != 0, msg


def test_overlapping_conflicting_execution_is_caught(setup):
    W, accs, adj, tr = setup
    pairs = [(i, j) for i in range(len(tr)) for j in range(i + 1, len(tr)) if adj[i, j]]
    i, j = pairs[-1]
    tr[i]["t_end"] = tr[j]["t_start"] + 1
    code, msg = O.check_trace(accs, W, tr, check_times=True)
    assert code == 21, msg


def test_serial_schedule_is_valid_for_any_window():
    st = inputs.tiny_stream(9)
    accs = O.tiny_accesses(st)
    n = len(accs)
    tr = np.zeros(n, dtype=O.TRACE_DTYPE)
    tr["seq"] = np.arange(n)
    tr["slot"] = 0
    tr["ev_insert"] = 3 * np.arange(n)
    tr["ev_dispatch"] = 3 * np.arange(n) + 1
    tr["ev_retire"] = 3 * np.arange(n) + 2
    tr["t_start"] = 2 * np.arange(n)
    tr["t_end"] = 2 * np.arange(n) + 1
    for W in (1, 8, 64):
        code, msg = O.check_trace(accs, W, tr, check_times=True)
        assert code == 0, msg


def test_early_dispatch_mode():
    """Handing a kernel out before its upstream kernels retire is accepted in
    early mode only if they were handed out first and the execution intervals
    stay ordered; both mistakes are caught."""
    st = inputs.tiny_stream(12)
    accs = O.tiny_accesses(st)
    adj = O.dag(accs)
    tr = simulate(accs, 8, np.random.default_rng(1), adj)
    pairs = [(i, j) for i in range(len(tr)) for j in range(i + 1, len(tr)) if adj[i, j]]
    i, j = pairs[0]
    code, msg = O.check_trace(accs, 8, tr, early=True)
    assert code == 0, msg
    # handed out before the upstream kernel: caught
    bad = tr.copy()
    bad[j]["ev_dispatch"] = bad[i]["ev_dispatch"] - 1
    bad[j]["ev_insert"] = min(bad[j]["ev_insert"], bad[j]["ev_dispatch"] - 1)
    code, msg = O.check_trace(accs, 8, bad, early=True)
    assert code != 0
    # execution overlap: caught (times are required in early mode)
    ov = tr.copy()
    ov[i]["t_end"] = ov[j]["t_start"] + 1
    code, msg = O.check_trace(accs, 8, ov, early=True)
    assert code == 21, msg
