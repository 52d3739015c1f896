"""CPU tests of the batched-scene autotuner's search (no GPU: candidates are
scored by a stand-in timer)."""
import itertools

from paper_2401_12377_amd import acs, tune


def pow2(x):
    p = 1
    while p < x:
        p <<= 1
    return p


def test_candidates_cover_the_documented_space():
    got = list(tune.candidates())
    keys = {(c["W"], c["n_groups"], c["wg_per_task"], c["host_check_depth"], c["window_check"]) for c in got}
    assert len(keys) == len(got), "duplicate candidates"
    want = set()
    for W, G, g in itertools.product((8, 16, 32, 48, 64), (1, 2, 4, 8), (1, 2, 4)):
        if G * pow2(W) > acs.W_MAX:
            continue
        if G == 1:
            # check wave, host against W and against 2W (at most 128), window wave
            want |= {(W, 1, g, 0, 0), (W, 1, g, W, 0), (W, 1, g, min(2 * W, 128), 0), (W, 1, g, 0, 1)}
        else:
            want.add((W, G, g, 0, 0))
    assert keys == want
    for c in got:
        assert c["queue_depth"] == 4096
        assert c["n_groups"] * pow2(c["W"]) <= acs.W_MAX
        assert c["n_groups"] == 1 or (c["host_check_depth"] == 0 and c["window_check"] == 0)


def test_candidates_respect_a_restricted_space():
    got = list(tune.candidates(windows=(32,), groups=(1, 2, 4), wg=(2,), sites=("wave",)))
    assert [(c["W"], c["n_groups"], c["wg_per_task"]) for c in got] == [(32, 1, 2), (32, 2, 2)]


def test_autotune_picks_the_fastest_then_refines_queue_depth():
    calls = []

    def timer(scenes, cfg, steps):
        calls.append(dict(cfg))
        v = 1000.0 * cfg["W"] - 10 * cfg["n_groups"] + cfg["wg_per_task"] + (5 if cfg["window_check"] else 0)
        return v + (50 if cfg["queue_depth"] == 1024 else 0)

    best, table = tune.autotune(None, steps=1, timer=timer, tie=0.0)
    n = len(list(tune.candidates()))
    assert len(calls) == n + 2 and len(table) == n + 2
    assert best["W"] == 64 and best["n_groups"] == 1 and best["wg_per_task"] == 4 and best["window_check"] == 1
    assert best["queue_depth"] == 1024
    assert [c["queue_depth"] for c in calls[-2:]] == [256, 1024]
    assert all(calls[-1][k] == best[k] for k in best)


def test_near_ties_go_to_the_cheapest_configuration():
    # 32/host with one or two workgroups per task 0.4% apart, queue depths
    # 0.8% apart: the cheaper of each pair is taken; a 5% gap is not a tie
    rates = {(32, 1, "host"): 2098.0, (32, 2, "host"): 2089.0, (16, 1, "host"): 1812.0}

    def timer(scenes, cfg, steps):
        site = ("host2" if cfg["host_check_depth"] > cfg["W"] else "host") if cfg["host_check_depth"] else \
            ("window" if cfg["window_check"] else "wave")
        v = rates.get((cfg["W"], cfg["wg_per_task"], site), 1000.0)
        return v - (16.0 if cfg["queue_depth"] == 1024 else 0.0) + (2.0 if cfg["queue_depth"] == 4096 else 0.0)

    best, _ = tune.autotune(None, steps=1, timer=timer)
    assert best == {"W": 32, "n_groups": 1, "wg_per_task": 1, "queue_depth": 256, "host_check_depth": 32,
                    "window_check": 0}
    far = tune.pick([({"W": 8, "n_groups": 1, "wg_per_task": 1, "queue_depth": 256}, 95.0),
                     ({"W": 32, "n_groups": 1, "wg_per_task": 2, "queue_depth": 4096}, 100.0)], tie=0.02)
    assert far["W"] == 32
