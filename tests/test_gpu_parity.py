"""GPU parity: every path's results against the CPU oracle, every schedule
against the oracle's trace checker.  Runs only on an MI355X with libacs built.

Bars:
* tiny random stream and RL step: bit-exact against the oracle on every
  buffer (both sides run the same FP32 operations in the same order), so
  also bit-exact across paths;
* schedules: the window decisions, admission order, dispatch order and (where
  recorded) execution intervals pass the oracle's checker.
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


# ---------------------------------------------------------------------------
# tiny random stream
# ---------------------------------------------------------------------------
def window(W, path, **kw):
    """`device_window`: the device path with the dependency checks made by
    the window wave itself (for one window the default makes them in a wave
    ahead of it)."""
    if path == "device_window":
        return acs.Window(W, path="device", window_check=1, **kw)
    return acs.Window(W, path=path, **kw)


def run_tiny(torch, st, path, W, **kw):
    arena = torch.from_numpy(st.init.copy()).cuda()
    torch.cuda.synchronize()
    with window(W, path, trace=True, **kw) as w:
        acs.submit_tiny_stream(w, st, arena.data_ptr())
        rc = w.sync_rc(SYNC_NS)
        assert rc == 0, acs.lib().acs_strerror(rc)
        tr = w.trace()
        stats = w.stats()
    return arena.cpu().numpy(), tr, stats


@pytest.mark.parametrize("path", ["inorder", "plain", "device", "device_window"])
def test_tiny_stream_matches_oracle(torch, path):
    for seed in range(4):
        say(f"tiny seed={seed} path={path}")
        st = inputs.tiny_stream(seed)
        got, tr, stats = run_tiny(torch, st, path, 8)
        ref = O.tiny_run(st)
        assert np.array_equal(bits(got), bits(ref)), f"seed {seed}: {np.count_nonzero(bits(got) != bits(ref))} words differ"
        assert stats["retired"] == len(st.kernels)


@pytest.mark.parametrize("path,W", [("plain", 8), ("device", 8), ("device", 1), ("device", 64), ("plain", 2),
                                    ("device_window", 8), ("device_window", 1), ("device_window", 64)])
def test_tiny_stream_schedule_is_valid(torch, path, W):
    for seed in range(3):
        say(f"tiny schedule seed={seed} path={path} W={W}")
        st = inputs.tiny_stream(seed + 10)
        got, tr, _ = run_tiny(torch, st, path, W)
        assert np.array_equal(bits(got), bits(O.tiny_run(st)))
        # the oracle's ranges on the same addresses as the run (any base works:
        # conflicts only depend on relative placement)
        accs = O.tiny_accesses(st, base=0)
        code, msg = O.check_trace(accs, W, tr, check_times=True, early=True)
        assert code == 0, msg


def test_inorder_trace_is_serial(torch):
    st = inputs.tiny_stream(21)
    got, tr, _ = run_tiny(torch, st, "inorder", 8)
    code, msg = O.check_trace(O.tiny_accesses(st), 1, tr, check_times=True)
    assert code == 0, msg


@pytest.mark.parametrize("wg", [1, 3, 16])
def test_tiny_stream_pieces_do_not_change_bits(torch, wg):
    st = inputs.tiny_stream(5)
    say(f"tiny pieces wg={wg}")
    got, _, _ = run_tiny(torch, st, "device", 8, wg_per_task=wg)
    assert np.array_equal(bits(got), bits(O.tiny_run(st)))


@pytest.mark.parametrize("path,W", [("device", 16), ("device", 64), ("device_window", 64)])
def test_tiny_stream_long_streams_device(torch, path, W):
    """Streams of 1000 kernels (the check waves' 64-kernel history and the
    staging ring wrap many times): bits equal to the oracle's, and every
    schedule valid with the exact upstream masks."""
    for seed in range(200, 206):
        say(f"tiny long seed={seed} path={path} W={W}")
        st = inputs.tiny_stream(seed, n_kernels=1000)
        got, tr, _ = run_tiny(torch, st, path, W, trace_capacity=4096)
        assert np.array_equal(bits(got), bits(O.tiny_run(st))), seed
        code, msg = O.check_trace(O.tiny_accesses(st), W, tr, check_times=True, early=True)
        assert code == 0, (seed, msg)


def test_tiny_stream_many_seeds_device(torch):
    for seed in range(100, 140):
        st = inputs.tiny_stream(seed)
        got, _, _ = run_tiny(torch, st, "device", 8)
        assert np.array_equal(bits(got), bits(O.tiny_run(st))), seed


# ---------------------------------------------------------------------------
# rigid-body RL step
# ---------------------------------------------------------------------------
INT_REGIONS = [("deg", acs.RL_DEG), ("adj_off", acs.RL_ADJ_OFF), ("label", acs.RL_LABEL), ("perm", acs.RL_PERM),
               ("inv_perm", acs.RL_INV_PERM), ("padj_off", acs.RL_PADJ_OFF)]


def compare_step(g, ref, step):
    n = ref.n
    for name, r in (("X", acs.RL_X), ("V", acs.RL_V), ("P", acs.RL_P), ("Q0", acs.RL_Q0)):
        got = g.get(r)
        want = getattr(ref, name)
        assert np.array_equal(bits(got), bits(want)), f"step {step}: {name} differs at {np.argwhere(bits(got) != bits(want))[:5]}"
    for name, r in INT_REGIONS:
        assert np.array_equal(g.get(r), getattr(ref, name)), f"step {step}: {name} differs"
    E = int(ref.meta[2])
    assert np.array_equal(g.get(acs.RL_ADJ)[:E], ref.adj[:E]), f"step {step}: adj differs"
    assert np.array_equal(g.get(acs.RL_PADJ)[:E], ref.padj[:E]), f"step {step}: padj differs"
    nisl = int(ref.meta[0])
    assert np.array_equal(g.get(acs.RL_ISL_OFF)[:nisl + 1], ref.isl_off[:nisl + 1]), f"step {step}: isl_off differs"
    plan = g.plan()
    assert list(plan[:3]) == list(ref.meta[:3]), f"step {step}: plan header differs"
    m = int(ref.meta[1])
    assert np.array_equal(plan[4:4 + 4 * m], ref.plan[:4 * m]), f"step {step}: plan rows differ"


@pytest.mark.parametrize("path,n,W,wg", [("inorder", 64, 32, 1), ("plain", 64, 32, 1), ("device", 64, 32, 1),
                                          ("device", 16, 8, 1), ("device", 300, 16, 2), ("plain", 300, 16, 2),
                                          ("device", 1024, 32, 4), ("device_window", 64, 32, 1),
                                          ("device_window", 300, 16, 2)])
def test_rl_steps_match_oracle(torch, path, n, W, wg):
    steps = 6 if n <= 300 else 2
    sc = inputs.rl_scene(seed=1, n=n)
    g = acs.RLSceneGPU(sc)
    ref = O.Scene.from_inputs(sc)
    accs = []
    with window(W, path, trace=True, wg_per_task=wg, trace_capacity=1 << 16) as w:
        for step in range(steps):
            say(f"rl path={path} n={n} W={W} step={step}")
            counts, _ = acs.rl_run(w, g, 1)
            ref.step()
            kl = ref.step_kernels()
            assert counts["kernels"] == len(kl)
            accs += [ref.access(*k) for k in kl]
            compare_step(g, ref, step)
        tr = w.trace()
    if path != "inorder":
        code, msg = O.check_trace(accs, W, tr, check_times=True, early=True)
        assert code == 0, msg


@pytest.mark.parametrize("path", ["inorder", "device"])
@pytest.mark.parametrize("n,radius", [(2, 0.01), (2, 0.3), (64, 0.01), (64, 0.3), (65, 0.3)])
def test_rl_edge_scenes_match_oracle(torch, path, n, radius):
    """The degenerate contact structures: the smallest scene apart and
    touching, no contacts at all, and one island of every body on either
    side of the one-wave limit; three steps against the oracle."""
    sc = inputs.rl_scene(seed=11, n=n, radius=radius)
    g = acs.RLSceneGPU(sc)
    ref = O.Scene.from_inputs(sc)
    with window(16, path) as w:
        for step in range(3):
            say(f"rl edge path={path} n={n} radius={radius} step={step}")
            counts, _ = acs.rl_run(w, g, 1)
            ref.step()
            assert counts["kernels"] == len(ref.step_kernels())
            compare_step(g, ref, step)


def test_rl_full_episode_device(torch):
    """The timed workload: 64 spheres, 200 steps, W = 32, device path."""
    sc = inputs.rl_scene(seed=1, n=64)
    g = acs.RLSceneGPU(sc)
    ref = O.Scene.from_inputs(sc)
    say("rl episode 200 steps device")
    with acs.Window(32, path="device") as w:
        counts, step_ns = acs.rl_run(w, g, 200)
    for _ in range(200):
        ref.step()
    assert np.array_equal(bits(g.get(acs.RL_X)), bits(ref.X))
    assert np.array_equal(bits(g.get(acs.RL_V)), bits(ref.V))
    assert counts["steps"] == 200 and counts["kernels"] > 200 * 5
    assert np.all(step_ns > 0)


def test_rl_episode_paths_agree(torch):
    sc = inputs.rl_scene(seed=2, n=64)
    finals = {}
    for path in ("inorder", "plain", "device"):
        say(f"rl episode 40 steps {path}")
        g = acs.RLSceneGPU(sc)
        with acs.Window(32, path=path) as w:
            acs.rl_run(w, g, 40)
        finals[path] = (g.get(acs.RL_X), g.get(acs.RL_V))
    for p in ("plain", "device"):
        assert np.array_equal(bits(finals[p][0]), bits(finals["inorder"][0]))
        assert np.array_equal(bits(finals[p][1]), bits(finals["inorder"][1]))


# ---------------------------------------------------------------------------
# device path: liveness, snapshots, stop
# ---------------------------------------------------------------------------
def test_device_many_nops_and_chains(torch):
    say("nop independent 20000")
    with acs.Window(32, path="device") as w:
        acs.nop_run(w, 20000, chain=False)
        assert w.stats()["retired"] == 20000
    say("nop chain 2000")
    with acs.Window(32, path="device", trace=True) as w:
        acs.nop_run(w, 2000, chain=True)
        tr = w.trace()
    # a chain: every kernel waits for its predecessor
    assert np.all(tr["t_start"][1:] >= tr["t_end"][:-1])


def test_device_scheduled_list_snapshot(torch):
    say("scheduled list")
    with acs.Window(8, path="device") as w:
        for _ in range(6):
            w.submit(acs.K_NOP, [(0, 1)], [(0, 1)], acs.ArgsNop(2_000_000))   # 2 ms each, a chain
        lst = w.scheduled_list()
        assert 1 <= len(lst) <= 8
        seqs = [e[0] for e in lst]
        assert seqs == sorted(seqs)
        states = [e[2] for e in lst]
        assert states.count(acs.EXECUTING) <= 1
        w.sync(SYNC_NS)
        assert w.scheduled_list() == []


def test_device_stop_reports_kernel_time(torch):
    with acs.Window(16, path="device") as w:
        acs.nop_run(w, 100, chain=False)
        w.stop()
        s = w.stats()
        assert s["kernel_ns"] > 0
        with pytest.raises(acs.AcsError) as e:
            w.submit(acs.K_NOP, [], [(0, 1)], acs.ArgsNop(0))
        assert e.value.code == acs.ESTATE


def test_empty_windows(torch):
    for path in ("inorder", "plain", "device"):
        with acs.Window(4, path=path) as w:
            assert w.sync(SYNC_NS) == 0
