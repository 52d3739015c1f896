"""GPU parity for the host/device split of the dependency check (Section
IV-C): the host checks each kernel against the kernels of the M sequence
numbers before it; the window wave drops upstream kernels that already
completed and holds a kernel back while one more than M older is still in
the window.

Bars: the same bits as in-order execution (the oracle's); the trace passes
the oracle's checker (every conflicting kernel in the window at insert is an
upstream, conflicting kernels never overlap in time); a dependency the
host's list cannot see is still honoured through the gate.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import acs, inputs

pytestmark = pytest.mark.gpu

SYNC_NS = 30 * 10 ** 9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    acs.lib()
    return t


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("W,M", [(8, 8), (16, 4), (32, 64), (8, 1)])
def test_tiny_stream_host_check(torch, W, M):
    for seed in range(3):
        say(f"host check tiny seed={seed} W={W} M={M}")
        st = inputs.tiny_stream(seed + 30)
        arena = torch.from_numpy(st.init.copy()).cuda()
        torch.cuda.current_stream().synchronize()
        with acs.Window(W, path="device", trace=True, host_check_depth=M) as w:
            acs.submit_tiny_stream(w, st, arena.data_ptr())
            assert w.sync_rc(SYNC_NS) == 0
            tr = w.trace()
            stats = w.stats()
        assert np.array_equal(bits(arena.cpu().numpy()), bits(O.tiny_run(st)))
        code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
        assert code == 0, msg
        # the host made the segment-pair tests, at most M predecessors per kernel
        assert 0 < stats["overlap_tests"] <= len(st.kernels) * M * acs.K_MAX * acs.K_MAX


@pytest.mark.parametrize("W,M", [(32, 32), (64, 128), (16, 100)])
def test_rl_steps_host_check(torch, W, M):
    """Six physics steps (about 450 kernels): with M above 64 the host's
    lists use their second word (a step's islands kernel reads what the next
    step's broadphase writes, some 75 kernels later)."""
    sc = inputs.rl_scene(seed=1, n=64)
    g = acs.RLSceneGPU(sc)
    ref = O.Scene.from_inputs(sc)
    accs = []
    with acs.Window(W, path="device", trace=True, host_check_depth=M, trace_capacity=1 << 16) as w:
        for step in range(6):
            say(f"host check rl step={step} W={W} M={M}")
            acs.rl_run(w, g, 1)
            ref.step()
            accs += [ref.access(*k) for k in ref.step_kernels()]
            assert np.array_equal(bits(g.get(acs.RL_X)), bits(ref.X))
            assert np.array_equal(bits(g.get(acs.RL_V)), bits(ref.V))
        tr = w.trace()
    code, msg = O.check_trace(accs, W, tr, check_times=True, early=True)
    assert code == 0, msg


def test_second_word_orders_a_dependency_inside_the_gate(torch):
    """A 2 ms kernel writes byte 0, a hundred short independent kernels
    follow, then one reads byte 0, 101 places after the writer.  With M = 128
    the host's list holds the writer: the reader is admitted while the writer
    still runs (the gate does not hold it), and its workers wait for the
    writer through the second word of its upstream list."""
    buf = torch.zeros(8192, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    torch.cuda.current_stream().synchronize()
    say("host check second word")
    with acs.Window(8, path="device", trace=True, host_check_depth=128) as w:
        w.submit(acs.K_NOP, [], [(base, 1)], acs.ArgsNop(2_000_000))
        for i in range(100):
            w.submit(acs.K_NOP, [], [(base + 64 * (i + 1), 1)], acs.ArgsNop(0))
        w.submit(acs.K_NOP, [(base, 1)], [(base + 7000, 1)], acs.ArgsNop(0))
        assert w.sync_rc(SYNC_NS) == 0
        tr = w.trace()
    assert tr["t_start"][101] >= tr["t_end"][0]
    assert tr["ev_insert"][101] < tr["ev_retire"][0]
    assert tr["up_mask"][101] == 1 << int(tr["slot"][0])


def test_gate_orders_a_dependency_outside_the_host_list(torch):
    """A 2 ms kernel writes byte 0 of a buffer, twenty short independent
    kernels follow, then one reads byte 0.  With M = 4 the host's list of the
    reader misses the writer; the gate still makes the reader wait for it."""
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    torch.cuda.current_stream().synchronize()
    say("host check gate")
    with acs.Window(8, path="device", trace=True, host_check_depth=4) as w:
        w.submit(acs.K_NOP, [], [(base, 1)], acs.ArgsNop(2_000_000))
        for i in range(20):
            w.submit(acs.K_NOP, [], [(base + 64 * (i + 1), 1)], acs.ArgsNop(0))
        w.submit(acs.K_NOP, [(base, 1)], [(base + 2048, 1)], acs.ArgsNop(0))
        assert w.sync_rc(SYNC_NS) == 0
        tr = w.trace()
    assert tr["t_start"][21] >= tr["t_end"][0]
    assert np.all(tr["ev_insert"][5:] > tr["ev_retire"][0])


def test_host_check_paths_agree_on_an_episode(torch):
    sc = inputs.rl_scene(seed=2, n=64)
    finals = []
    for M in (0, 32, 8, 128):
        say(f"host check episode M={M}")
        g = acs.RLSceneGPU(sc)
        with acs.Window(32, path="device", host_check_depth=M) as w:
            acs.rl_run(w, g, 40)
        finals.append((g.get(acs.RL_X), g.get(acs.RL_V)))
    for x, v in finals[1:]:
        assert np.array_equal(bits(x), bits(finals[0][0])) and np.array_equal(bits(v), bits(finals[0][1]))
