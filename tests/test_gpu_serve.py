"""GPU parity for the serving loop (acs_serve_run): requests with Poisson
arrivals mixing RL scene steps and DNN inferences, admitted by working-memory
footprint, run concurrently through one open window.

Bars: every request's result in the mix equals its result alone, bit for bit
(an RL step: the oracle's program-order step of that scene, which the RL
bodies reproduce exactly; a DNN inference: the in-order path's inference on
that input, and the oracle's FP32 network to the propagation level); the
plan read mid-request gives the oracle's island count; admission keeps the
pool and the resident cap; every request is admitted after it arrives and
completes after it is admitted.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import acs, inputs

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def model():
    return inputs.dnn_weights()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def build(specs):
    rl = {s.seed: inputs.rl_scene(seed=s.seed, n=s.n) for s in specs if s.kind == inputs.SERVE_RL}
    dnn = {s.seed: inputs.dnn_input(s.seed) for s in specs if s.kind == inputs.SERVE_DNN}
    return rl, dnn


@pytest.fixture(scope="module")
def mix():
    specs = inputs.serve_requests(seed=4, rate_per_s=20000.0, n_requests=40)
    rl, dnn = build(specs)
    return specs, rl, dnn


@pytest.fixture(scope="module")
def expected(torch, model, mix):
    """Each request alone: the oracle's RL step, the in-order path's inference."""
    specs, rl, dnn = mix
    want = {}
    net = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    for s in specs:
        if s.kind == inputs.SERVE_RL:
            ref = O.Scene.from_inputs(rl[s.seed])
            ref.step()
            want[s.seed] = (ref.X.copy(), ref.V.copy(), ref.n_multi)
        else:
            net.set_input(dnn[s.seed].x)
            with acs.Window(16, path="inorder") as w:
                acs.dnn_submit(w, net, dnn[s.seed].logits)
                assert w.sync_rc(30 * 10 ** 9) == 0
            want[s.seed] = net.out.cpu().numpy().copy()
    return want


def check(specs, outs, res, want, model, dnn):
    for i, (s, o, r) in enumerate(zip(specs, outs, res)):
        assert r["admit_ns"] >= s.arrival_ns and r["done_ns"] > r["admit_ns"], i
        if s.kind == inputs.SERVE_RL:
            x, v, nm = want[s.seed]
            assert np.array_equal(bits(o[0]), bits(x)), ("rl X", i, s.n)
            assert np.array_equal(bits(o[1]), bits(v)), ("rl V", i, s.n)
            assert r["multi_islands"] == nm, i
        else:
            assert np.array_equal(bits(o), bits(want[s.seed])), ("dnn", i)
            assert r["multi_islands"] == -1


@pytest.mark.parametrize("path,W,G,pool_mib,resident,hc", [("device", 32, 1, 64, 16, 0), ("device", 16, 4, 64, 32, 0),
                                                           ("device", 8, 8, 6, 64, 0), ("device", 32, 1, 64, 16, 32),
                                                           ("plain", 32, 1, 64, 16, 0), ("inorder", 8, 1, 64, 8, 0)])
def test_mix_matches_solo(torch, model, mix, expected, path, W, G, pool_mib, resident, hc):
    specs, rl, dnn = mix
    sset = acs.ServeSet(specs, rl, dnn, inputs.DNN_CLASSES)
    sset.clear_outputs()
    net = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    pool = torch.empty(pool_mib << 20, dtype=torch.uint8, device="cuda")
    host = acs.serve_host(resident)
    torch.cuda.current_stream().synchronize()
    say(f"serve path={path} W={W} G={G} pool={pool_mib}MiB resident={resident} host_check={hc}")
    with acs.Window(W, path=path, n_groups=G, host_check_depth=hc) as w:
        res, st = acs.serve_run(w, sset, pool, host, max_resident=resident, model=net, stall_ns=30 * 10 ** 9)
    say(f"  stats {st}")
    check(specs, sset.outputs(), res, expected, model, dnn)
    assert st["peak_pool_bytes"] <= pool_mib << 20
    assert 1 <= st["peak_resident"] <= resident
    assert st["kernels"] == sum(r["kernels"] for r in res)
    assert all(0 <= r["group"] < G for r in res)
    if pool_mib == 6:
        # a 6 MiB pool holds two inferences' activations: admission had to wait
        assert st["waited_memory"] > 0
        assert st["peak_pool_bytes"] > 4 << 20


def test_dnn_results_match_oracle_network(torch, model, mix, expected):
    specs, _, dnn = mix
    seen = 0
    for s in specs:
        if s.kind != inputs.SERVE_DNN or seen >= 3:
            continue
        seen += 1
        ref = O.DNN(model, dnn[s.seed], inputs.DNN_CELLS)
        ref.run()
        out = expected[s.seed].astype(np.float64)
        assert np.abs(out.astype(np.float64) - ref.out).max() <= 1e-5 * np.abs(ref.out).max()
    assert seen == 3


def test_repeated_runs_reuse_memory(torch, model):
    """Two runs on one pool and one host area: the second run's requests
    reuse blocks the first run's kernels used, with the same results."""
    specs = inputs.serve_requests(seed=9, rate_per_s=50000.0, n_requests=12)
    rl, dnn = build(specs)
    sset = acs.ServeSet(specs, rl, dnn, inputs.DNN_CLASSES)
    net = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    pool = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    host = acs.serve_host(8)
    torch.cuda.current_stream().synchronize()
    outs = []
    say("serve repeated runs")
    for rep in range(2):
        sset.clear_outputs()
        with acs.Window(32, path="device") as w:
            res, st = acs.serve_run(w, sset, pool, host, max_resident=8, model=net, stall_ns=30 * 10 ** 9)
        outs.append(sset.outputs())
    for a, b in zip(*outs):
        if isinstance(a, tuple):
            assert np.array_equal(bits(a[0]), bits(b[0])) and np.array_equal(bits(a[1]), bits(b[1]))
        else:
            assert np.array_equal(bits(a), bits(b))


def test_larger_mix_device_equals_inorder(torch, model):
    """300 requests at 10k/s (over capacity of the in-order path): the device
    path with four window groups gives every request the in-order path's bits,
    and a sample of the RL requests the oracle's."""
    specs = inputs.serve_requests(seed=12, rate_per_s=10000.0, n_requests=300)
    rl, dnn = build(specs)
    sset = acs.ServeSet(specs, rl, dnn, inputs.DNN_CLASSES)
    net = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
    pool = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    host = acs.serve_host(256)
    torch.cuda.current_stream().synchronize()
    outs = {}
    for path, W, G in (("inorder", 8, 1), ("device", 16, 4)):
        sset.clear_outputs()
        say(f"serve 300 requests path={path}")
        with acs.Window(W, path=path, n_groups=G) as w:
            res, st = acs.serve_run(w, sset, pool, host, max_resident=256, model=net, stall_ns=60 * 10 ** 9)
        assert st["kernels"] == sum(r["kernels"] for r in res)
        outs[path] = sset.outputs()
    for i, (a, b) in enumerate(zip(outs["device"], outs["inorder"])):
        if isinstance(a, tuple):
            assert np.array_equal(bits(a[0]), bits(b[0])) and np.array_equal(bits(a[1]), bits(b[1])), i
        else:
            assert np.array_equal(bits(a), bits(b)), i
    rl_ids = [i for i, s in enumerate(specs) if s.kind == inputs.SERVE_RL][:20]
    for i in rl_ids:
        ref = O.Scene.from_inputs(rl[specs[i].seed])
        ref.step()
        assert np.array_equal(bits(outs["device"][i][0]), bits(ref.X)), i
