"""GPU parity for the dependency checks made by the check wave, the default
for one window (the host/device split of Section IV-C with the host's part
inside the device): each kernel is tested, as it is staged, against the 64
submitted before it; the window wave drops upstream kernels that already
completed and holds a kernel back while one more than 64 older is still in
the window.

Bars: the same bits as in-order execution (the oracle's); the trace passes
the oracle's checker (every conflicting kernel in the window at insert is an
upstream, conflicting kernels never overlap in time); a dependency farther
back than 64 kernels is still honoured through the gate.
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


@pytest.mark.parametrize("W", [8, 16, 32, 64, 5])
def test_tiny_stream_check_wave(torch, W):
    for seed in range(3):
        say(f"check wave tiny seed={seed} W={W}")
        st = inputs.tiny_stream(seed + 50, n_kernels=200)
        arena = torch.from_numpy(st.init.copy()).cuda()
        torch.cuda.current_stream().synchronize()
        with acs.Window(W, path="device", trace=True) as w:
            acs.submit_tiny_stream(w, st, arena.data_ptr())
            assert w.sync_rc(SYNC_NS) == 0
            w.stop()   # the device's test counts are published when its waves leave
            tr = w.trace()
            stats = w.stats()
        assert np.array_equal(bits(arena.cpu().numpy()), bits(O.tiny_run(st)))
        code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
        assert code == 0, msg
        # the check wave made the pair tests: at most 64 predecessors per kernel
        assert 0 < stats["overlap_tests"] <= len(st.kernels) * 64 * acs.K_MAX * acs.K_MAX


def test_rl_steps_check_wave(torch):
    sc = inputs.rl_scene(seed=4, n=64)
    g = acs.RLSceneGPU(sc)
    ref = O.Scene.from_inputs(sc)
    accs = []
    with acs.Window(32, path="device", trace=True, trace_capacity=1 << 16) as w:
        for step in range(6):
            say(f"check wave rl step={step}")
            acs.rl_run(w, g, 1)
            ref.step()
            accs += [ref.access(*k) for k in ref.step_kernels()]
            assert np.array_equal(bits(g.get(acs.RL_X)), bits(ref.X))
            assert np.array_equal(bits(g.get(acs.RL_V)), bits(ref.V))
        tr = w.trace()
    code, msg = O.check_trace(accs, 32, tr, check_times=True, early=True)
    assert code == 0, msg


def test_gate_orders_a_dependency_beyond_the_history(torch):
    """A 2 ms kernel writes byte 0 of a buffer, seventy short independent
    kernels follow, then one reads byte 0, seventy-one places later: out of
    the check wave's reach; the gate still makes the reader wait for it."""
    buf = torch.zeros(8192, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    torch.cuda.current_stream().synchronize()
    say("check wave gate")
    with acs.Window(16, path="device", trace=True) as w:
        w.submit(acs.K_NOP, [], [(base, 1)], acs.ArgsNop(2_000_000))
        for i in range(70):
            w.submit(acs.K_NOP, [], [(base + 64 * (i + 1), 1)], acs.ArgsNop(0))
        w.submit(acs.K_NOP, [(base, 1)], [(base + 6000, 1)], acs.ArgsNop(0))
        assert w.sync_rc(SYNC_NS) == 0
        tr = w.trace()
    assert tr["t_start"][71] >= tr["t_end"][0]
    assert np.all(tr["ev_insert"][65:] > tr["ev_retire"][0])


def test_check_sites_agree_on_an_episode_and_a_network(torch):
    sc = inputs.rl_scene(seed=2, n=64)
    finals = []
    for wc in (0, 1):
        say(f"check sites episode window_check={wc}")
        g = acs.RLSceneGPU(sc)
        with acs.Window(32, path="device", window_check=wc) as w:
            acs.rl_run(w, g, 40)
        finals.append((g.get(acs.RL_X), g.get(acs.RL_V)))
    assert np.array_equal(bits(finals[1][0]), bits(finals[0][0]))
    assert np.array_equal(bits(finals[1][1]), bits(finals[0][1]))
    wts = inputs.dnn_weights()
    outs = []
    for path in ("inorder", "device"):
        say(f"check wave dnn {path}")
        net = acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES)
        res = []
        for sd in range(4):
            inp = inputs.dnn_input(sd)
            net.set_input(inp.x)
            with acs.Window(16, path=path) as w:
                acs.dnn_submit(w, net, inp.logits)
                assert w.sync_rc(SYNC_NS) == 0
            res.append(net.out.cpu().numpy().copy())
        outs.append(res)
    for a, b in zip(*outs):
        assert np.array_equal(bits(a), bits(b))
