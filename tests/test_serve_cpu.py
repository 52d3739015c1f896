"""CPU tests of the serving loop's host logic: the working-memory pool
against a brute-force model of the address range, the request generator,
the copy and signal task argument checks, and the serving entry point's
argument validation (everything that runs before a GPU is touched).
"""
import ctypes as C
import math
import os

import numpy as np
import pytest

from paper_2401_12377_amd import acs, inputs


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(acs.LIB_PATH):
        from paper_2401_12377_amd import build
        build.build()
    return acs.lib()


BASE = 1 << 40


def test_pool_create_checks():
    with pytest.raises(acs.AcsError):
        acs.Pool(BASE + 16, 1 << 20)         # unaligned base
    with pytest.raises(acs.AcsError):
        acs.Pool(BASE, 100)                  # smaller than one block
    p = acs.Pool(BASE, 1 << 20)
    assert p.info() == {"used": 0, "largest_free": 1 << 20, "blocks": 0}
    with pytest.raises(acs.AcsError):
        p.alloc(0)
    assert p.alloc((1 << 20) + 1) is None
    with pytest.raises(acs.AcsError):
        p.free(BASE + 256)                   # not a live block
    a = p.alloc(1)
    assert a == BASE and p.info()["used"] == 256
    with pytest.raises(acs.AcsError):
        p.free(a + 256)
    p.free(a)
    with pytest.raises(acs.AcsError):
        p.free(a)                            # double free


@pytest.mark.parametrize("seed", range(6))
def test_pool_random_against_bitmap(seed):
    """Random allocs and frees: blocks stay inside the range, 256-aligned,
    pairwise disjoint; used bytes and the largest free run equal a byte map's;
    an allocation fails only when no free run of that size exists (best fit
    never misses a fitting hole); everything freed merges back to one run."""
    g = np.random.default_rng(seed)
    units = 512                                   # 256-byte units
    p = acs.Pool(BASE, units * 256)
    used = np.zeros(units, bool)
    live = {}
    for step in range(3000):
        if live and (g.random() < 0.45 or len(live) > 60):
            a = list(live)[g.integers(len(live))]
            p.free(a)
            u0, nu = (a - BASE) // 256, live.pop(a)
            assert used[u0:u0 + nu].all()
            used[u0:u0 + nu] = False
        else:
            want = int(g.integers(1, 40 * 256))
            nu = math.ceil(want / 256)
            a = p.alloc(want)
            runs, cur = [], 0
            for u in used:
                cur = 0 if u else cur + 1
                runs.append(cur)
            fits = max(runs) >= nu
            if a is None:
                assert not fits
                continue
            assert fits
            assert (a - BASE) % 256 == 0 and BASE <= a and a + nu * 256 <= BASE + units * 256
            u0 = (a - BASE) // 256
            assert not used[u0:u0 + nu].any()
            used[u0:u0 + nu] = True
            live[a] = nu
        info = p.info()
        assert info["used"] == int(used.sum()) * 256
        assert info["blocks"] == len(live)
        best = cur = 0
        for u in used:
            cur = 0 if u else cur + 1
            best = max(best, cur)
        assert info["largest_free"] == best * 256
    for a in list(live):
        p.free(a)
    assert p.info() == {"used": 0, "largest_free": units * 256, "blocks": 0}


def test_pool_best_fit_takes_the_smallest_hole():
    p = acs.Pool(BASE, 64 * 256)
    a = [p.alloc(4 * 256) for _ in range(16)]     # fills the range
    assert p.alloc(1) is None
    p.free(a[1])                                  # hole of 4 units
    p.free(a[5])
    p.free(a[6])                                  # hole of 8 units
    b = p.alloc(3 * 256)
    assert b == a[1]                              # the smaller hole
    c = p.alloc(8 * 256)
    assert c == a[5]
    assert p.alloc(256) == a[1] + 3 * 256


def test_serve_requests_generator():
    lam = 5000.0
    r = inputs.serve_requests(4, lam, 4000)
    t = np.array([q.arrival_ns for q in r])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t])) * 1e-9
    # exponential gaps: mean 1/lam, coefficient of variation 1 (within sampling error)
    assert abs(gaps.mean() * lam - 1) < 0.05
    assert abs(gaps.std() / gaps.mean() - 1) < 0.06
    kinds = np.array([q.kind for q in r])
    assert abs(kinds.mean() - 0.5) < 0.03
    n = np.array([q.n for q in r if q.kind == inputs.SERVE_RL])
    assert n.min() >= 16 and n.max() <= 512
    assert abs(np.log(n).mean() - 0.5 * (np.log(16) + np.log(512))) < 0.06
    assert len({q.seed for q in r}) == len(r)
    assert [q.seed for q in inputs.serve_requests(4, lam, 10)] == [q.seed for q in r[:10]]
    assert all(q.n == 0 for q in r if q.kind == inputs.SERVE_DNN)


def test_copy_and_signal_argument_checks():
    buf = np.zeros(1024, np.uint8)
    base = (buf.ctypes.data + 255) // 256 * 256
    with acs.Window(4, path="manual") as w:
        good = acs.ArgsCopy(base, base + 256, 128)
        w.submit(acs.K_COPY, [(base + 256, 128)], [(base, 128)], good)
        for bad in (acs.ArgsCopy(base + 8, base + 256, 128),     # unaligned
                    acs.ArgsCopy(base, base + 256, 100),         # not a multiple of 16
                    acs.ArgsCopy(base, base + 64, 128),          # overlapping
                    acs.ArgsCopy(0, base, 16)):                  # null
            with pytest.raises(acs.AcsError):
                w.submit(acs.K_COPY, [], [], bad)
        w.submit(acs.K_SIGNAL, [], [(base, 8)], acs.ArgsSignal(base, 7))
        with pytest.raises(acs.AcsError):
            w.submit(acs.K_SIGNAL, [], [], acs.ArgsSignal(base + 4, 7))
        with pytest.raises(acs.AcsError):
            w.submit(acs.K_SIGNAL, [], [], acs.ArgsSignal(0, 7))


_HOST = np.zeros(1 << 24, np.uint8)             # stands in for pinned host memory (never touched)
_HOST_PTR = (_HOST.ctypes.data + 255) // 256 * 256


def _serve_rc(specs, pool_bytes=1 << 26, max_resident=16, model=False, host=_HOST_PTR, host_bytes=None):
    reqs = (acs.ServeRequestC * max(1, len(specs)))()
    lg = np.zeros(24, np.float32)
    for i, (kind, t, n) in enumerate(specs):
        q = reqs[i]
        q.kind, q.arrival_ns, q.n, q.iters, q.r, q.dt = kind, t, n, 8, 0.05, 1 / 120
        q.input, q.output, q.logits = 1 << 20, 2 << 20, lg.ctypes.data
    cfg = acs.ServeConfigC()
    cfg.pool, cfg.pool_bytes, cfg.max_resident = 1 << 30, pool_bytes, max_resident
    cfg.host = host
    cfg.host_bytes = (1 << 24) - 256 if host_bytes is None else host_bytes
    graph = acs.DNNGraphC()
    graph.n_cells, graph.classes = len(inputs.DNN_CELLS), inputs.DNN_CLASSES
    for c, (h, cin, cout, st) in enumerate(inputs.DNN_CELLS):
        graph.cell[c].hin, graph.cell[c].cin, graph.cell[c].cout, graph.cell[c].stride = h, cin, cout, st
    cfg.model = C.cast(C.pointer(graph), C.c_void_p) if model else None
    with acs.Window(8, path="manual") as w:
        return acs.lib().acs_serve_run(w.handle, C.byref(cfg), reqs, len(specs), None, None)


def test_serve_argument_validation():
    RL, DNN = acs.SERVE_RL, acs.SERVE_DNN
    assert _serve_rc([(RL, 10.0, 64), (RL, 5.0, 64)]) == acs.EINVAL          # arrivals out of order
    assert _serve_rc([(RL, 0.0, 1)]) == acs.EINVAL                            # too few bodies
    assert _serve_rc([(RL, 0.0, 2000)]) == acs.EINVAL                         # too many bodies
    assert _serve_rc([(7, 0.0, 64)]) == acs.EINVAL                            # unknown kind
    assert _serve_rc([(DNN, 0.0, 0)]) == acs.EINVAL                           # no model
    assert _serve_rc([(RL, 0.0, 512)], pool_bytes=1 << 20) == acs.EINVAL      # larger than the whole pool
    assert _serve_rc([(RL, 0.0, 64)], max_resident=0) == acs.EINVAL
    assert _serve_rc([(RL, 0.0, 64)], max_resident=5000) == acs.EINVAL
    assert _serve_rc([(RL, 0.0, 64)], host=None) == acs.EINVAL                # no host memory
    assert _serve_rc([(RL, 0.0, 64)], host=_HOST_PTR + 16) == acs.EINVAL      # unaligned
    need = acs.lib().acs_serve_host_bytes(16)
    assert _serve_rc([(RL, 0.0, 64)], host_bytes=need - 1) == acs.EINVAL      # too small
    # host memory: at least one signal word and one island plan of the largest scene per slot
    assert need >= 16 * (8 + 4 * (4 + 4 * 512))
    assert acs.lib().acs_serve_host_bytes(0) == 0
    # a DNN request's working memory: three tensors per cell and the pooled vector
    act = sum(3 * (-(-4 * (h // st) ** 2 * cout // 256) * 256) for h, _, cout, st in inputs.DNN_CELLS) + 512
    assert _serve_rc([(DNN, 0.0, 0)], pool_bytes=act - 256, model=True) == acs.EINVAL
