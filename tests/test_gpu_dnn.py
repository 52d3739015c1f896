"""GPU parity for the dynamic-DNN workload (gated convolution cells).

Bars:
* every convolution, teacher-forced with the oracle's FP32 input of that
  layer: |gpu - exact| <= 1e-5 * max(|exact|, sum of |terms|) against the
  oracle's float64 sum (the matrix unit accumulates in its own order);
* join, average pool and the head, teacher-forced: bit-exact against the
  oracle (same FP32 operations in the same order);
* whole inferences: bit-identical across the in-order, plain and device
  paths; the device and plain schedules pass the oracle's trace checker with
  the oracle's own dataflow ranges; the logits within 1e-5 of the largest
  logit of the oracle's FP32 network.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import acs, inputs

pytestmark = pytest.mark.gpu

SYNC_NS = 30 * 10 ** 9
TOL = 1e-5


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


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()


def run_tasks(torch, tasks, path="device", W=16):
    torch.cuda.synchronize()
    with acs.Window(W, path=path) as w:
        for t in tasks:
            w.submit(*t)
        rc = w.sync_rc(SYNC_NS)
        assert rc == 0, acs.lib().acs_strerror(rc)


def layer_shapes():
    """Every distinct convolution of the network: (cell, k)."""
    seen, out = set(), []
    for c, (h, cin, cout, st) in enumerate(inputs.DNN_CELLS):
        for k in (3, 1):
            if (h, cin, cout, st, k) not in seen:
                seen.add((h, cin, cout, st, k))
                out.append((c, k))
    return out


@pytest.mark.parametrize("c,k", layer_shapes())
def test_conv_teacher_forced(torch, model, c, k):
    h, cin, cout, st = inputs.DNN_CELLS[c]
    # the oracle's own activation entering cell c (all branches on for seed 5's run, else its input)
    net = O.DNN(model, inputs.dnn_input(5), inputs.DNN_CELLS)
    net.run()
    x = net.cell_input(c)
    assert x.shape == (h, h, cin)
    w = model.w3[c] if k == 3 else model.w1[c]
    b = model.b3[c] if k == 3 else model.b1[c]
    exact, mag = O.conv_f64(x, w, b, k, st)
    outs = {}
    for path in ("inorder", "device"):
        say(f"conv cell={c} k={k} path={path}")
        xd, wd, bd = dev(torch, x), dev(torch, w), dev(torch, b)
        od = torch.full(exact.shape, float("nan"), dtype=torch.float32, device="cuda")
        run_tasks(torch, [acs.conv_task(xd, wd, bd, od, k, st)], path)
        outs[path] = od.cpu().numpy()
    g = outs["device"].astype(np.float64)
    assert np.all(np.isfinite(g))
    assert np.all(np.abs(g - exact) <= TOL * np.maximum(np.abs(exact), mag))
    assert np.array_equal(bits(outs["device"]), bits(outs["inorder"]))


def test_join_pool_fc_teacher_forced(torch, model):
    net = O.DNN(model, inputs.dnn_input(5), inputs.DNN_CELLS)
    net.run()
    tasks, checks = [], []
    for c in sorted(net.y):
        a = net.t3.get(c)
        b = net.t1.get(c)
        parts = [p for p in (a, b) if p is not None]
        out = torch.zeros(net.y[c].shape, dtype=torch.float32, device="cuda")
        ta = [dev(torch, p) for p in parts]
        tasks.append(acs.join_task(out, ta[0], ta[1] if len(ta) > 1 else None))
        checks.append((out, net.y[c], ta))
    last = net.y[max(net.y)]
    xin = dev(torch, last)
    pool = torch.zeros(last.shape[2], dtype=torch.float32, device="cuda")
    hw = last.shape[0] * last.shape[1]
    tasks.append((acs.K_AVGPOOL, [acs.tensor_seg(xin)], [acs.tensor_seg(pool)],
                  acs.ArgsAvgpool(pool.data_ptr(), xin.data_ptr(), hw, last.shape[2])))
    pin = dev(torch, net.pool)
    fw, fb = dev(torch, model.fc_w), dev(torch, model.fc_b)
    logits = torch.zeros(inputs.DNN_CLASSES, dtype=torch.float32, device="cuda")
    tasks.append((acs.K_FC, [acs.tensor_seg(pin), acs.tensor_seg(fw), acs.tensor_seg(fb)], [acs.tensor_seg(logits)],
                  acs.ArgsFC(logits.data_ptr(), pin.data_ptr(), fw.data_ptr(), fb.data_ptr(),
                             model.fc_w.shape[0], model.fc_w.shape[1])))
    say("join / pool / fc teacher-forced")
    run_tasks(torch, tasks)
    for out, ref, _ in checks:
        assert np.array_equal(bits(out.cpu().numpy()), bits(ref))
    assert np.array_equal(bits(pool.cpu().numpy()), bits(net.pool))
    assert np.array_equal(bits(logits.cpu().numpy()), bits(net.out))


def run_inference(torch, gnet, inp, path, W=16, trace=False):
    gnet.set_input(inp.x)
    with acs.Window(W, path=path, trace=trace) as w:
        n = acs.dnn_submit(w, gnet, inp.logits)
        rc = w.sync_rc(SYNC_NS)
        assert rc == 0, acs.lib().acs_strerror(rc)
        tr = w.trace() if trace else None
    bufs = {"out": gnet.out.cpu().numpy(), "pool": gnet.pool.cpu().numpy()}
    for c in range(len(gnet.cells)):
        bufs[f"y{c}"] = gnet.y[c].cpu().numpy()
        bufs[f"t3_{c}"] = gnet.t3[c].cpu().numpy()
        bufs[f"t1_{c}"] = gnet.t1[c].cpu().numpy()
    return n, bufs, tr


@pytest.mark.parametrize("seed", [0, 1, 2, 7])
def test_inference_paths_agree_and_schedules_valid(torch, model, seed):
    inp = inputs.dnn_input(seed)
    ref = O.DNN(model, inp, inputs.DNN_CELLS)
    ref.run()
    accs = ref.accesses()
    results = {}
    for path in ("inorder", "plain", "device"):
        say(f"dnn inference seed={seed} path={path}")
        gnet = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
        n, bufs, tr = run_inference(torch, gnet, inp, path, trace=(path != "inorder"))
        assert n == len(ref.kernels())
        results[path] = bufs
        if tr is not None:
            code, msg = O.check_trace(accs, 16, tr, check_times=True, early=True)
            assert code == 0, msg
    for path in ("plain", "device"):
        for key, v in results["inorder"].items():
            assert np.array_equal(bits(results[path][key]), bits(v)), (path, key)
    # branches that did not run were never written
    for c in range(len(inputs.DNN_CELLS)):
        if not ref.g3[c]:
            assert np.all(np.isnan(results["device"][f"t3_{c}"]))
    out = results["device"]["out"].astype(np.float64)
    err = np.abs(out - ref.out).max() / np.abs(ref.out).max()
    say(f"dnn logits seed={seed}: max |gpu - oracle| / max |oracle| = {err:.3e}")
    assert err <= 1e-5


def test_many_inferences_one_window(torch, model):
    """Several inferences submitted back to back into one device window: each
    result equals its solo run bit for bit."""
    seeds = [3, 4, 5, 6]
    solo = {}
    for s in seeds:
        gnet = acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES)
        _, bufs, _ = run_inference(torch, gnet, inputs.dnn_input(s), "device")
        solo[s] = bufs["out"]
    nets = {s: acs.DNNGPU(model, inputs.DNN_CELLS, inputs.DNN_CLASSES) for s in seeds}
    for s in seeds:
        nets[s].set_input(inputs.dnn_input(s).x)
    say("dnn 4 inferences in one window")
    with acs.Window(16, path="device") as w:
        for s in seeds:
            acs.dnn_submit(w, nets[s], inputs.dnn_input(s).logits)
        assert w.sync_rc(SYNC_NS) == 0
    for s in seeds:
        assert np.array_equal(bits(nets[s].out.cpu().numpy()), bits(solo[s]))
