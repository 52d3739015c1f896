"""Pins of the oracle's static irregular network (randomly wired, the
static-network workload of Section VI-C).

The generator is pinned to the Watts-Strogatz construction's invariants
(ring lattice when nothing is rewired, the link count kept by rewiring,
links directed forward), the network to an independent float64 PyTorch
rendition of the same architecture, and the kernel list's read/write sets by
running it in random topological orders of its dependency DAG.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2401_12377_amd import inputs


def test_ring_lattice_when_nothing_is_rewired():
    n, k = 16, 4
    g = inputs.dag_graph(seed=1, nodes=n, k=k, p=0.0)
    for i in range(n):
        nb = {(i + j) % n for j in range(1, k // 2 + 1)} | {(i - j) % n for j in range(1, k // 2 + 1)}
        assert g.preds[i] == sorted(v for v in nb if v < i)


@pytest.mark.parametrize("seed", range(5))
def test_rewiring_keeps_the_link_count_and_order(seed):
    n, k = 32, 4
    g = inputs.dag_graph(seed=seed, nodes=n, k=k, p=0.75)
    assert all(all(p < i for p in ps) for i, ps in enumerate(g.preds))
    assert all(ps == sorted(set(ps)) for ps in g.preds)
    assert sum(len(ps) for ps in g.preds) == n * k // 2       # no degree above the cap here
    assert g.preds[0] == [] and len(g.sinks) >= 1 and (n - 1) in g.sinks
    # rewiring happened: not the lattice
    assert g.preds != inputs.dag_graph(seed=seed, nodes=n, k=k, p=0.0).preds
    assert inputs.dag_graph(seed=seed).preds == g.preds       # deterministic


def _torch_dag64(g, wts, x):
    F = torch.nn.functional

    def t(a):
        return torch.from_numpy(np.asarray(a, np.float64))

    def conv(v, i):
        w = t(wts.w[i]).permute(3, 2, 0, 1)
        return F.conv2d(v, w, t(wts.b[i]), padding=1)

    def agg(vs):
        a = torch.relu(vs[0] + vs[1]) if len(vs) > 1 else torch.relu(vs[0])
        for v in vs[2:]:
            a = torch.relu(a + v)
        return a
    xin = t(x).permute(2, 0, 1)[None]
    y = {}
    for i, ps in enumerate(g.preds):
        y[i] = conv(agg([y[p] for p in ps]) if ps else xin, i)
    s = agg([y[i] for i in g.sinks])
    pooled = s.mean(dim=(2, 3))[0]
    return (pooled @ t(wts.fc_w) + t(wts.fc_b)).numpy()


@pytest.mark.parametrize("seed", [0, 1])
def test_network_matches_float64_rendition(seed):
    g = inputs.dag_graph(nodes=16)
    wts = inputs.dag_weights(g)
    x = inputs.dag_input(g, seed)
    out = O.StaticDAG(g, wts, x).run()
    ref = _torch_dag64(g, wts, x)
    assert np.allclose(out, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_kernel_count():
    g = inputs.dag_graph()
    net = O.StaticDAG(g, inputs.dag_weights(g), inputs.dag_input(g))
    ks = net.kernels()
    joins = sum(max(1, len(ps) - 1) for ps in g.preds if ps) + max(1, len(g.sinks) - 1)
    assert len(ks) == len(g.preds) + joins + 2
    assert sum(1 for k in ks if k[0] == O.DAG_CONV) == len(g.preds)


def test_topological_order_invariance():
    g = inputs.dag_graph(nodes=12)
    wts = inputs.dag_weights(g)
    x = inputs.dag_input(g, 3)
    ref = O.StaticDAG(g, wts, x)
    out0 = ref.run()
    adj = O.dag(ref.accesses())
    rng = np.random.default_rng(0)
    for _ in range(4):
        order = O.random_topological_order(adj, rng)
        net = O.StaticDAG(g, wts, x)
        assert np.array_equal(net.run(order).view(np.uint32), out0.view(np.uint32))
    # nodes with no path between them are independent in the DAG
    ks = ref.kernels()
    conv_of = {k[1]: i for i, k in enumerate(ks) if k[0] == O.DAG_CONV}
    reach = adj.copy().astype(bool)
    for m in range(len(ks)):
        reach |= reach[:, [m]] & reach[[m], :]
    assert not all(reach[conv_of[a], conv_of[b]] or reach[conv_of[b], conv_of[a]]
                   for a in range(12) for b in range(a + 1, 12))
