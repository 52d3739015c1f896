"""Pins for the oracle's tiny-random-stream bodies and its in-order executor.

* scale / axpy against exact rational arithmetic rounded to FP32;
* the pairwise tree sum against closed forms and Higham's error bound;
* program-order execution against every / many topological orders of the
  dependency DAG (any schedule the window may produce must give identical
  buffers), which also shows that the declared segments cover what the bodies
  touch;
* the printed one-directional check of Algorithm 1 fails that invariance.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_12377_amd import inputs


def round_fp32(v: Fraction) -> np.float32:
    """Round an exact rational to the nearest FP32 value (ties to even)."""
    f = np.float32(float(v))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        err = abs(Fraction(float(c)) - v)
        key = (err, int(np.frombuffer(np.float32(c).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return np.float32(best[1])


def _one_kernel_stream(op, ins, out, a, j=0, lens=(1000, 700, 1200, 300)):
    offs, pos = [], 0
    for L in lens:
        offs.append(pos)
        pos = (pos + L + 63) // 64 * 64
    rng = np.random.default_rng(3)
    init = np.zeros(pos, np.float32)
    for o, L in zip(offs, lens):
        init[o:o + L] = rng.uniform(-1, 1, L).astype(np.float32)
    st = inputs.TinyStream(seed=0, lengths=np.array(lens, np.int64), offsets=np.array(offs, np.int64),
                           arena_elems=pos, init=init,
                           kernels=[inputs.TinyKernel(op=op, out=out, ins=tuple(ins), a=a, j=j)])
    return st


def test_scale_is_correctly_rounded_product():
    a = np.float32(-0.3711)
    st = _one_kernel_stream(inputs.OP_SCALE, [1], 0, float(a))
    out = O.tiny_run(st)
    x = st.init[st.offsets[1]:st.offsets[1] + 700]
    got = out[st.offsets[0]:st.offsets[0] + 700]
    for i in range(0, 700, 7):
        assert got[i] == round_fp32(Fraction(float(a)) * Fraction(float(x[i])))
    # elements past n = min(len) are untouched
    assert np.array_equal(out[st.offsets[0] + 700:st.offsets[0] + 1000],
                          st.init[st.offsets[0] + 700:st.offsets[0] + 1000])


def test_axpy_is_single_rounding_fma():
    a = np.float32(0.8125)
    st = _one_kernel_stream(inputs.OP_AXPY, [0, 2], 1, float(a))
    out = O.tiny_run(st)
    x = st.init[st.offsets[0]:]
    y = st.init[st.offsets[2]:]
    got = out[st.offsets[1]:]
    for i in range(0, 700, 5):
        exact = Fraction(float(a)) * Fraction(float(x[i])) + Fraction(float(y[i]))
        assert got[i] == round_fp32(exact), i


def test_axpy_in_place():
    a = np.float32(1.5)
    st = _one_kernel_stream(inputs.OP_AXPY, [0, 1], 1, float(a))
    out = O.tiny_run(st)
    x, y = st.init[st.offsets[0]:], st.init[st.offsets[1]:]
    got = out[st.offsets[1]:]
    for i in range(0, 700, 3):
        assert got[i] == round_fp32(Fraction(1.5) * Fraction(float(x[i])) + Fraction(float(y[i])))


@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 4096, 12288])
def test_tree_sum_exact_on_integers(n):
    v = np.arange(1, n + 1, dtype=np.float32) % 64   # partial sums stay below 2^24: exact
    assert O.tree_sum(v) == np.float32(sum(int(t) for t in v))


def test_tree_sum_error_bound():
    rng = np.random.default_rng(5)
    for n in (300, 1000, 4096, 5000, 12288):
        v = rng.uniform(-1, 1, n).astype(np.float32)
        P = 1 << (n - 1).bit_length()
        levels = int(math.log2(P))
        u = 2.0 ** -24
        gamma = levels * u / (1 - levels * u)
        exact = math.fsum(float(t) for t in v)
        bound = gamma * math.fsum(abs(float(t)) for t in v)
        assert abs(float(O.tree_sum(v)) - exact) <= bound


def test_tree_sum_order_is_the_pairwise_one():
    # 1 + 2^-24 + ... : sequential left-to-right summation loses the small
    # terms, the pairwise tree pairs element i with i + P/2 first.
    v = np.array([1.0, 2.0 ** -24, 2.0 ** -24, 2.0 ** -24], dtype=np.float32)
    # level 1: [1 + 2^-24, 2^-24 + 2^-24] = [1, 2^-23]; level 2: 1 + 2^-23
    assert O.tree_sum(v) == np.float32(1.0 + 2.0 ** -23)


def test_sum_reduce_writes_one_element_and_reads_output_first():
    st = _one_kernel_stream(inputs.OP_SUM, [0, 3], 0, 0.0, j=17)
    out = O.tiny_run(st)
    cat = np.concatenate([st.init[st.offsets[0]:st.offsets[0] + 1000], st.init[st.offsets[3]:st.offsets[3] + 300]])
    exact = math.fsum(float(t) for t in cat)
    assert abs(float(out[st.offsets[0] + 17]) - exact) <= 11 * 2.0 ** -24 * math.fsum(abs(float(t)) for t in cat)
    changed = np.nonzero(out != st.init)[0]
    assert set(changed.tolist()) <= {int(st.offsets[0]) + 17}


def test_generator_shape():
    st = inputs.tiny_stream(0)
    assert st.n_buffers == 16 and len(st.kernels) == 64
    assert np.all((st.lengths >= 256) & (st.lengths <= 4096))
    assert np.all(st.offsets % 64 == 0)
    for k in st.kernels:
        assert len(set(k.ins)) == len(k.ins)
        assert 1 <= len(k.ins) <= 3 and 0 <= k.out < 16
        if k.op == inputs.OP_SCALE:
            assert len(k.ins) == 1
        if k.op == inputs.OP_AXPY:
            assert len(k.ins) == 2
        assert 0 <= k.j < st.lengths[k.out]
    # every initial value is exact in FP32 and inside [-1, 1)
    vals = np.concatenate([st.init[o:o + L] for o, L in zip(st.offsets, st.lengths)])
    assert vals.min() >= -1.0 and vals.max() < 1.0


@pytest.mark.parametrize("seed", list(range(12)))
def test_topological_order_invariance(seed):
    st = inputs.tiny_stream(seed)
    accs = O.tiny_accesses(st)
    adj = O.dag(accs)
    ref = O.tiny_run(st)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        order = O.random_topological_order(adj, rng)
        assert np.array_equal(O.tiny_run(st, order=order).view(np.uint32), ref.view(np.uint32))


def test_all_topological_orders_small_stream():
    st = inputs.tiny_stream(3, n_kernels=7)
    accs = O.tiny_accesses(st)
    adj = O.dag(accs)
    ref = O.tiny_run(st)
    n = len(accs)
    count = 0

    def rec(prefix, indeg):
        nonlocal count
        if len(prefix) == n:
            count += 1
            assert np.array_equal(O.tiny_run(st, order=prefix).view(np.uint32), ref.view(np.uint32))
            return
        for i in range(n):
            if i not in prefix and indeg[i] == 0:
                d = indeg.copy()
                for j in np.nonzero(adj[i])[0]:
                    d[j] -= 1
                rec(prefix + [i], d)

    rec([], adj.sum(axis=0).astype(int))
    assert count >= 1


def test_literal_check_breaks_invariance():
    """With the printed one-directional check a reader can be moved before
    the writer it depends on, and the result changes."""
    lens = (512, 512, 512)
    offs = np.array([0, 512, 1024], np.int64)
    init = np.zeros(1536, np.float32)
    init[:512] = 1.0
    init[512:1024] = 2.0
    ks = [inputs.TinyKernel(op=inputs.OP_SCALE, out=0, ins=(2,), a=3.0, j=0),   # writes A (buffer 0)
          inputs.TinyKernel(op=inputs.OP_SCALE, out=1, ins=(0,), a=5.0, j=0)]   # reads A, writes B
    st = inputs.TinyStream(seed=0, lengths=np.array(lens, np.int64), offsets=offs, arena_elems=1536,
                           init=init, kernels=ks)
    accs = O.tiny_accesses(st)
    assert O.dag(accs)[0, 1] == 1
    assert O.dag(accs, literal=True)[0, 1] == 0
    ref = O.tiny_run(st)
    swapped = O.tiny_run(st, order=[1, 0])        # allowed by the literal DAG only
    assert not np.array_equal(ref, swapped)


def test_literal_check_breaks_invariance_on_generated_streams():
    broken = 0
    for seed in range(10):
        st = inputs.tiny_stream(seed)
        accs = O.tiny_accesses(st)
        adj_lit = O.dag(accs, literal=True)
        ref = O.tiny_run(st)
        rng = np.random.default_rng(seed)
        for _ in range(10):
            order = O.random_topological_order(adj_lit, rng)
            if not np.array_equal(O.tiny_run(st, order=order), ref):
                broken += 1
                break
    assert broken > 0
