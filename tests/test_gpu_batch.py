"""GPU parity for batched scenes: many independent RL scenes of uneven size
in one persistent launch, split over the groups of one window wave.

Bars: every scene's state after the run is bit-identical to the oracle's
program-order run of that scene alone; each group's schedule passes the
oracle's trace checker against the group's own kernel stream; the in-order
and plain paths give the same bits.
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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def scenes(n_scenes, seed=3):
    sizes = inputs.batched_scene_sizes(seed, n_scenes)
    return [inputs.rl_scene(seed=1000 + i, n=int(s)) for i, s in enumerate(sizes)]


def shifted(acc, off):
    """The same access with every range moved by off bytes (scenes get
    disjoint abstract address spaces in the oracle)."""
    return O.make_access([(s + off, z) for s, z in acc.reads()], [(s + off, z) for s, z in acc.writes()])


@pytest.mark.parametrize("path,G,W,hc", [("device", 4, 16, 0), ("device", 8, 8, 0), ("device", 2, 32, 0),
                                         ("device", 1, 16, 16), ("inorder", 1, 8, 0), ("plain", 1, 32, 0)])
def test_batch_matches_solo_oracle(torch, path, G, W, hc):
    scs = scenes(12)
    steps = 4
    gpu = [acs.RLSceneGPU(sc) for sc in scs]
    trace = path == "device"
    say(f"batch path={path} G={G} W={W} host_check={hc}")
    with acs.Window(W, path=path, n_groups=G, trace=trace, trace_capacity=1 << 16, host_check_depth=hc) as w:
        counts, step_ns = acs.rl_run_batch(w, gpu, steps, n_groups=G)
        tr = w.trace() if trace else None
    assert counts["steps"] == steps * len(scs)
    refs = [O.Scene.from_inputs(sc) for sc in scs]
    # the oracle's kernel streams, in the order the driver submits them
    streams = {g: [] for g in range(G)}
    def put(i, k):
        refs[i].run_kernel(*k)
        streams[i % G].append(shifted(refs[i].access(*k), (i + 1) << 46))

    for step in range(steps):
        # stage by stage across the scenes
        for k in [(O.RL_PREDICT, 0, 0), (O.RL_BROADPHASE, 0, 0), (O.RL_ISLANDS, 0, 0), (O.RL_PERMUTE, 0, 0)]:
            for i in range(len(refs)):
                put(i, k)
        tails = [ref.step_kernels()[4:] for ref in refs]
        # per group: Jacobi iteration by iteration, island by island across
        # its scenes, then integrate
        for g in range(G):
            mine = range(g, len(refs), G)
            for it in range(max(refs[i].c.iters for i in mine)):
                js = {i: [k for k in tails[i] if k[0] == O.RL_JACOBI and k[2] == it] for i in mine}
                for kk in range(max(len(v) for v in js.values())):
                    for i in mine:
                        if kk < len(js[i]):
                            put(i, js[i][kk])
            for i in mine:
                for k in tails[i]:
                    if k[0] != O.RL_JACOBI:
                        put(i, k)
    for i, (g_, ref) in enumerate(zip(gpu, refs)):
        assert np.array_equal(bits(g_.get(acs.RL_X)), bits(ref.X)), i
        assert np.array_equal(bits(g_.get(acs.RL_V)), bits(ref.V)), i
    assert counts["kernels"] == sum(len(v) for v in streams.values())
    if tr is not None:
        Wp = 1 << (W - 1).bit_length()
        grp = tr["slot"] // Wp
        for g in range(G):
            ids = np.nonzero(grp == g)[0]
            assert len(ids) == len(streams[g])
            sub = tr[ids].copy()
            sub["seq"] = np.arange(len(ids))
            sub["slot"] = sub["slot"] % Wp
            m = np.uint64((1 << Wp) - 1)
            sub["valid_mask"] = (sub["valid_mask"] >> np.uint64(g * Wp)) & m
            sub["up_mask"] = (sub["up_mask"] >> np.uint64(g * Wp)) & m
            code, msg = O.check_trace(streams[g], W, sub, check_times=True, early=True)
            assert code == 0, (g, msg)


def test_group_sync_and_validation(torch):
    with pytest.raises(acs.AcsError):
        acs.Window(32, path="device", n_groups=4)          # 4 x 32 lanes do not fit one wave
    sc = scenes(4)
    gpu = [acs.RLSceneGPU(s) for s in sc]
    with acs.Window(16, path="device", n_groups=4) as w:
        with pytest.raises(acs.AcsError):
            w.sync_group(4)
        counts, _ = acs.rl_run_batch(w, gpu, 2, n_groups=4)
        for g in range(4):
            assert w.sync_group(g) == 0
        assert w.stats()["retired"] == counts["kernels"]


@pytest.mark.parametrize("G,W,wg,hc,qd", [(1, 16, 2, 0, 4096), (4, 16, 1, 0, 4096),
                                          (1, 32, 1, 32, 256), (1, 48, 1, 48, 1024),   # the autotuner's picks
                                          (1, 64, 1, 64, 1024), (1, 64, 1, 64, 256), (1, 64, 1, 128, 256),
                                          (1, 32, 1, 0, 1024)])
def test_full_size_batch_matches_oracle(torch, G, W, wg, hc, qd):
    """The batched workload at full size (256 scenes of 16-512 bodies, 20
    steps, one persistent launch): every scene's final state bit-identical to
    the oracle's program-order run of that scene alone."""
    scs = inputs.batched_scenes(3, 256)
    gpu = [acs.RLSceneGPU(sc) for sc in scs]
    say(f"full batch G={G} W={W} wg={wg} host_check={hc} queue={qd}")
    with acs.Window(W, path="device", n_groups=G, wg_per_task=wg, host_check_depth=hc, queue_depth=qd) as w:
        counts, _ = acs.rl_run_batch(w, gpu, 20, n_groups=G)
    assert counts["steps"] == 20 * 256
    for i, (g, sc) in enumerate(zip(gpu, scs)):
        ref = O.Scene.from_inputs(sc)
        for _ in range(20):
            ref.step()
        assert np.array_equal(bits(g.get(acs.RL_X)), bits(ref.X)), (i, sc.n)
        assert np.array_equal(bits(g.get(acs.RL_V)), bits(ref.V)), (i, sc.n)
