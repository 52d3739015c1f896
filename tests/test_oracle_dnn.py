"""Pins of the oracle's dynamic-DNN pieces (Section II-C workload).

The convolution is pinned to PyTorch's CPU conv2d in float64 (a library
routine), its FP32 defined-order version to the float64 result within the
error bound of K + 1 roundings, the head and the join to their closed forms,
and the whole gated network to an independent float64 PyTorch rendition of
the same architecture.  The kernel list's read/write sets are validated by
running the network in random topological orders of its dependency DAG.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2401_12377_amd import inputs

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


def torch_conv64(x, w, b, k, s):
    xt = torch.from_numpy(x.astype(np.float64)).permute(2, 0, 1)[None]
    wt = torch.from_numpy(w.astype(np.float64).reshape(k, k, w.shape[-2], w.shape[-1])).permute(3, 2, 0, 1)
    bt = torch.from_numpy(b.astype(np.float64))
    y = torch.nn.functional.conv2d(xt, wt, bt, stride=s, padding=(k - 1) // 2)
    return y[0].permute(1, 2, 0).numpy()


def rnd(seed, shape, scale=1.0):
    return (np.random.default_rng(seed).uniform(-1, 1, size=shape) * scale).astype(np.float32)


@pytest.mark.parametrize("h,cin,cout,k,s", [(8, 4, 6, 3, 1), (8, 4, 6, 3, 2), (7, 3, 5, 3, 2), (8, 4, 6, 1, 1),
                                            (8, 4, 6, 1, 2), (6, 32, 8, 3, 1), (4, 128, 16, 1, 1)])
def test_conv_f64_matches_torch(h, cin, cout, k, s):
    x = rnd(1, (h, h, cin))
    w = rnd(2, (k, k, cin, cout) if k == 3 else (cin, cout))
    b = rnd(3, (cout,))
    out, mag = O.conv_f64(x, w, b, k, s)
    ref = torch_conv64(x, w, b, k, s)
    assert out.shape == ref.shape
    assert np.all(np.abs(out - ref) <= 1e-13 * mag + 1e-300)


@pytest.mark.parametrize("h,cin,cout,k,s", [(8, 32, 8, 3, 1), (8, 32, 8, 3, 2), (8, 64, 8, 1, 1), (4, 128, 4, 3, 1)])
def test_conv_f32_within_rounding_bound(h, cin, cout, k, s):
    x = rnd(4, (h, h, cin))
    w = rnd(5, (k, k, cin, cout) if k == 3 else (cin, cout))
    b = rnd(6, (cout,))
    f32 = O.conv_f32(x, w, b, k, s)
    f64, mag = O.conv_f64(x, w, b, k, s)
    K = k * k * cin
    assert np.all(np.abs(f32.astype(np.float64) - f64) <= gamma(K + 1) * mag)
    # and it is not exact in general: the check above is not vacuous
    assert np.any(f32.astype(np.float64) != f64)


def test_conv_exact_on_small_integers():
    # every partial sum is an integer below 2^24: the FP32 result is exact
    g = np.random.default_rng(7)
    x = g.integers(-4, 5, size=(6, 6, 16)).astype(np.float32)
    w = g.integers(-4, 5, size=(3, 3, 16, 8)).astype(np.float32)
    b = g.integers(-4, 5, size=(8,)).astype(np.float32)
    for s in (1, 2):
        f32 = O.conv_f32(x, w, b, 3, s)
        assert np.array_equal(f32.astype(np.float64), torch_conv64(x, w, b, 3, s))


def test_relu_and_join():
    assert O.lib().or_relu(-0.0) == 0.0 and np.signbit(np.float32(O.lib().or_relu(-0.0))) == False  # noqa: E712
    assert O.lib().or_relu(float("nan")) == 0.0
    assert O.lib().or_relu(2.5) == 2.5 and O.lib().or_relu(-2.5) == 0.0
    a, b = rnd(8, (1000,)), rnd(9, (1000,))
    s = (a.astype(np.float64) + b.astype(np.float64)).astype(np.float32)   # one rounding, as FP32 addition
    assert np.array_equal(O.join(a, b), np.where(s > 0, s, np.float32(0)))
    assert np.array_equal(O.join(a), np.where(a > 0, a, np.float32(0)))


def test_avgpool_and_fc_bounds():
    x = rnd(10, (8, 8, 128))
    p = O.avgpool(x)
    ref = x.astype(np.float64).reshape(64, 128).mean(axis=0)
    mag = np.abs(x.astype(np.float64)).reshape(64, 128).sum(axis=0) / 64
    assert np.all(np.abs(p - ref) <= gamma(63) * mag)
    xi = np.random.default_rng(11).integers(-100, 100, size=(8, 8, 16)).astype(np.float32)
    assert np.array_equal(O.avgpool(xi).astype(np.float64), xi.astype(np.float64).reshape(64, 16).sum(0) / 64)
    v, w, b = rnd(12, (128,)), rnd(13, (128, 10)), rnd(14, (10,))
    out = O.fc(v, w, b)
    ref = b.astype(np.float64) + v.astype(np.float64) @ w.astype(np.float64)
    mag = np.abs(b.astype(np.float64)) + np.abs(v.astype(np.float64)) @ np.abs(w.astype(np.float64))
    assert np.all(np.abs(out - ref) <= gamma(128) * mag)


def _torch_net64(wts, inp, cells):
    """Independent float64 rendition of the gated network (same architecture)."""
    F = torch.nn.functional
    x = torch.from_numpy(inp.x.astype(np.float64)).permute(2, 0, 1)[None]
    for c, (h, cin, cout, st) in enumerate(cells):
        g3 = inp.logits[c, 0] > 0
        g1 = inp.logits[c, 1] > 0 or st == 2
        parts = []
        if g3:
            w = torch.from_numpy(wts.w3[c].astype(np.float64)).permute(3, 2, 0, 1)
            parts.append(F.conv2d(x, w, torch.from_numpy(wts.b3[c].astype(np.float64)), stride=st, padding=1))
        if g1:
            w = torch.from_numpy(wts.w1[c].astype(np.float64)).T[:, :, None, None]
            parts.append(F.conv2d(x, w, torch.from_numpy(wts.b1[c].astype(np.float64)), stride=st))
        if parts:
            x = torch.relu(sum(parts))
    pooled = x.mean(dim=(2, 3))[0]
    return (pooled @ torch.from_numpy(wts.fc_w.astype(np.float64)) + torch.from_numpy(wts.fc_b.astype(np.float64))).numpy()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_network_matches_float64_rendition(seed):
    wts = inputs.dnn_weights()
    inp = inputs.dnn_input(seed)
    net = O.DNN(wts, inp, inputs.DNN_CELLS)
    out = net.run()
    ref = _torch_net64(wts, inp, inputs.DNN_CELLS)
    # FP32 rounding through 12 cells: relative agreement at the 1e-4 level
    assert np.allclose(out, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_gating_structure():
    wts = inputs.dnn_weights()
    for seed in range(20):
        inp = inputs.dnn_input(seed)
        net = O.DNN(wts, inp, inputs.DNN_CELLS)
        ks = net.kernels()
        n3 = sum(inp.logits[c, 0] > 0 for c in range(12))
        n1 = sum((inp.logits[c, 1] > 0) or inputs.DNN_CELLS[c][3] == 2 for c in range(12))
        nj = sum((inp.logits[c, 0] > 0) or (inp.logits[c, 1] > 0) or inputs.DNN_CELLS[c][3] == 2 for c in range(12))
        assert len(ks) == n3 + n1 + nj + 2
        assert sum(1 for k in ks if k[0] == O.DNN_CONV3) == n3
        # transition cells always produce an output
        for c in (4, 8):
            assert any(k[0] == O.DNN_JOIN and k[1] == c for k in ks)


@pytest.mark.parametrize("seed", [0, 3])
def test_network_topological_order_invariance(seed):
    wts = inputs.dnn_weights()
    inp = inputs.dnn_input(seed)
    ref = O.DNN(wts, inp, inputs.DNN_CELLS)
    out0 = ref.run()
    adj = O.dag(ref.accesses())
    g = np.random.default_rng(seed)
    for _ in range(5):
        order = O.random_topological_order(adj, g)
        net = O.DNN(wts, inp, inputs.DNN_CELLS)
        assert np.array_equal(net.run(order).view(np.uint32), out0.view(np.uint32))
        for c in ref.y:
            assert np.array_equal(net.y[c].view(np.uint32), ref.y[c].view(np.uint32))
    # the two branches of a cell are independent, the join depends on both
    ks = ref.kernels()
    for i, (op, c, _, _) in enumerate(ks):
        if op == O.DNN_CONV3 and i + 1 < len(ks) and ks[i + 1][0] == O.DNN_CONV1:
            assert adj[i, i + 1] == 0 and adj[i, i + 2] == 1 and adj[i + 1, i + 2] == 1
