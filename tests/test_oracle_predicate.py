"""Pins for the oracle's overlap test, conflict relation and DAG.

Everything here is checked against brute-force set intersection over small
address spaces, not against the formula itself (Algorithm 1; Section III-C).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O

U64 = (1 << 64) - 1


def byteset(s, z):
    return set(range(s, s + z))


def test_overlap_exhaustive_small_space():
    space = 7
    segs = [(s, z) for s in range(space) for z in range(space - s + 1)]
    for (s1, z1), (s2, z2) in itertools.product(segs, segs):
        want = bool(byteset(s1, z1) & byteset(s2, z2))
        assert O.overlap(s1, z1, s2, z2) == want, (s1, z1, s2, z2)


def test_overlap_special_cases():
    assert not O.overlap(0, 8, 8, 8)          # adjacent ranges do not overlap
    assert not O.overlap(8, 8, 0, 8)
    assert O.overlap(0, 9, 8, 8)
    assert not O.overlap(4, 0, 0, 16)         # a zero-size range never overlaps
    assert O.overlap(3, 2, 3, 2)              # identical
    assert O.overlap(0, 100, 40, 2)           # contained
    # the "whole memory" range overlaps any non-empty range, at any address
    for s in (0, 1, 1 << 40, U64 - 1):
        assert O.overlap(0, U64, s, 1)
    # saturation: a range whose end would wrap past 2^64 still overlaps
    assert O.overlap(U64 - 10, 100, U64 - 5, 1)
    assert not O.overlap(U64 - 10, 5, U64 - 5, 1)


def _rand_access(rng, space=24, kmax=3):
    nr = int(rng.integers(0, kmax + 1))
    nw = int(rng.integers(0, kmax + 1))
    def seg():
        s = int(rng.integers(0, space))
        z = int(rng.integers(0, 5))
        return (s, z)
    return [seg() for _ in range(nr)], [seg() for _ in range(nw)]


def _bytes(segs):
    out = set()
    for s, z in segs:
        out |= byteset(s, z)
    return out


def test_conflict_matches_hazard_definition():
    """conflict(i<j) <=> RAW or WAR or WAW on at least one byte."""
    rng = np.random.default_rng(7)
    for _ in range(3000):
        ro, wo = _rand_access(rng)
        rn, wn = _rand_access(rng)
        R0, W0, R1, W1 = _bytes(ro), _bytes(wo), _bytes(rn), _bytes(wn)
        raw = bool(R1 & W0)
        war = bool(W1 & R0)
        waw = bool(W1 & W0)
        a0, a1 = O.make_access(ro, wo), O.make_access(rn, wn)
        assert O.conflict(a0, a1) == (raw or war or waw)
        # Algorithm 1 as printed sees WAR and WAW but not RAW
        assert O.conflict(a0, a1, literal=True) == (war or waw)
        # read-read sharing never creates a dependency
        if not (raw or war or waw):
            assert not O.conflict(a0, a1)


def test_literal_algorithm_misses_read_after_write():
    """k0 writes A; k1 reads A and writes B.  The printed check finds no
    dependency, the symmetric reading does."""
    A, B = (0, 64), (64, 64)
    k0 = O.make_access([], [A])
    k1 = O.make_access([A], [B])
    assert not O.conflict(k0, k1, literal=True)
    assert O.conflict(k0, k1)


def test_dag_matches_pairwise_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(20):
        n = int(rng.integers(1, 12))
        accs_py = [_rand_access(rng) for _ in range(n)]
        accs = [O.make_access(r, w) for r, w in accs_py]
        adj = O.dag(accs)
        for i in range(n):
            for j in range(n):
                if i >= j:
                    assert adj[i, j] == 0
                    continue
                Ri, Wi = _bytes(accs_py[i][0]), _bytes(accs_py[i][1])
                Rj, Wj = _bytes(accs_py[j][0]), _bytes(accs_py[j][1])
                want = bool((Rj & Wi) | (Wj & Ri) | (Wj & Wi))
                assert bool(adj[i, j]) == want


@pytest.mark.parametrize("n", [1, 5, 16])
def test_whole_memory_kernel_is_a_barrier(n):
    rng = np.random.default_rng(n)
    accs = [O.make_access(*_rand_access(rng, space=1000)) for _ in range(n)]
    barrier = O.make_access([(0, U64)], [(0, U64)])
    accs = accs + [barrier] + accs
    adj = O.dag(accs)
    b = n
    for i in range(len(accs)):
        if i < b:
            assert adj[i, b] == (1 if (accs[i].n_r or accs[i].n_w) and
                                 any(z for _, z in accs[i].reads() + accs[i].writes()) else 0)
        elif i > b:
            assert adj[b, i] == (1 if any(z for _, z in accs[i].reads() + accs[i].writes()) else 0)
