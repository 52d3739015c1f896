"""GPU parity for the graph-captured steady state (acs_graph_*).

A recorded task graph replays as one HIP graph with the conflict edges of
its kernels.  Bars: every replay gives the bits of in-order execution (the
oracle's for the tiny stream, the in-order path's for the network), with
other GPU work and host synchronisation between replays; the graph keeps
only edges the conflict relation implies.
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


@pytest.mark.parametrize("seed", [0, 5])
def test_tiny_stream_graph_replays(torch, seed):
    st = inputs.tiny_stream(seed)
    ref = O.tiny_run(st)
    arena = torch.from_numpy(st.init.copy()).cuda()
    init = torch.from_numpy(st.init.copy()).cuda()
    torch.cuda.current_stream().synchronize()
    say(f"graph tiny seed={seed}")
    with acs.Window(8, path="inorder") as w:
        w.graph_begin()
        acs.submit_tiny_stream(w, st, arena.data_ptr())
        g = w.graph_end()
    with g:
        info = g.info()
        assert info["kernels"] == len(st.kernels)
        adj = O.dag(O.tiny_accesses(st))
        assert 0 < info["edges"] <= int(adj.sum())
        for rep in range(3):
            arena.copy_(init)
            (arena[:16] * 2).sum().item()          # other GPU work between replays
            torch.cuda.current_stream().synchronize()
            g.launch()
            g.sync()
            assert np.array_equal(bits(arena.cpu().numpy()), bits(ref)), rep


def test_dnn_graph_replays_match_inorder(torch):
    wts = inputs.dnn_weights()
    gates = inputs.dnn_input(11).logits            # one gate pattern for every replay
    xs = [inputs.dnn_input(s).x for s in (21, 22, 23)]
    # the in-order path on each input (same gates)
    want = []
    for x in xs:
        net = acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES)
        net.set_input(x)
        with acs.Window(16, path="inorder") as w:
            acs.dnn_submit(w, net, gates)
            w.sync()
        want.append(net.out.cpu().numpy())
    net = acs.DNNGPU(wts, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    say("graph dnn record")
    with acs.Window(16, path="inorder") as w:
        w.graph_begin()
        n = acs.dnn_submit(w, net, gates)
        g = w.graph_end()
    with g:
        assert g.info()["kernels"] == n
        for rep, (x, ref) in enumerate(zip(xs, want)):
            net.set_input(x)
            g.launch()
            g.sync()
            assert np.array_equal(bits(net.out.cpu().numpy()), bits(ref)), rep
