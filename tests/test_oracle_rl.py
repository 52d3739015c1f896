"""Pins for the oracle's rigid-body RL step.

* broadphase against float64 all-pairs distances (decisions agree away from
  the contact threshold);
* islands against scipy's connected components and the canonical ordering;
* the Jacobi contact kernel against the closed form for an isolated pair and
  the centroid invariant of an island;
* free flight and wall reflection in the integrator;
* the body permutation: permute gathers the positions grouped by island
  (order fixed independently of the oracle's own perm array), and integrate
  puts every body back in its own place (no Jacobi sweeps: each body ends at
  its wall-clamped predicted position; a full step: every body without
  contacts flies free);
* the step's kernel list in any topological order of its dependency DAG gives
  the same state as program order.

The permutation pins are functions of a scene so that
tests/test_oracle_mutants.py can run them against copies of the oracle with
planted mistakes and show that they fail there.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from oracle import oracle as O
from paper_2401_12377_amd import inputs


def scene(seed=1, n=64, L=None):
    return O.Scene.from_inputs(inputs.rl_scene(seed=seed, n=n), L=L)


def run_prefix(s):
    for op in (O.RL_PREDICT, O.RL_BROADPHASE, O.RL_ISLANDS, O.RL_PERMUTE):
        s.run_kernel(op)


@pytest.mark.parametrize("seed,n", [(1, 64), (2, 64), (3, 200), (4, 16)])
def test_broadphase_against_float64(seed, n):
    s = scene(seed, n)
    s.run_kernel(O.RL_PREDICT)
    s.run_kernel(O.RL_BROADPHASE)
    P = s.P[:, :3].astype(np.float64)
    d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    thr = (2.0 * float(s.c.r)) ** 2
    for i in range(n):
        nb = set(s.adj[s.adj_off[i]:s.adj_off[i + 1]].tolist())
        assert s.deg[i] == len(nb) == s.adj_off[i + 1] - s.adj_off[i]
        assert list(s.adj[s.adj_off[i]:s.adj_off[i + 1]]) == sorted(nb)
        for j in range(n):
            if i == j:
                assert j not in nb
                continue
            if abs(d2[i, j] - thr) > 1e-5:
                assert (j in nb) == (d2[i, j] < thr), (i, j)
    # symmetric
    A = np.zeros((n, n), bool)
    for i in range(n):
        A[i, s.adj[s.adj_off[i]:s.adj_off[i + 1]]] = True
    assert np.array_equal(A, A.T)


@pytest.mark.parametrize("seed,n", [(1, 64), (5, 64), (6, 300)])
def test_islands_match_connected_components(seed, n):
    s = scene(seed, n)
    s.run_kernel(O.RL_PREDICT)
    s.run_kernel(O.RL_BROADPHASE)
    s.run_kernel(O.RL_ISLANDS)
    E = s.adj_off[n]
    rows = np.repeat(np.arange(n), s.deg)
    G = csr_matrix((np.ones(E), (rows, s.adj[:E])), shape=(n, n))
    ncomp, lab = connected_components(G, directed=False)
    assert s.n_islands == ncomp
    # same partition, labelled by the smallest member
    for c in range(ncomp):
        members = np.nonzero(lab == c)[0]
        assert np.all(s.label[members] == members.min())
    # permutation groups islands by smallest member, members ascending
    assert sorted(s.perm.tolist()) == list(range(n))
    assert np.array_equal(s.inv_perm[s.perm], np.arange(n))
    keys = [(int(s.label[b]), int(b)) for b in s.perm]
    assert keys == sorted(keys)
    sizes = np.diff(s.isl_off[:ncomp + 1])
    assert sizes.sum() == n and np.all(sizes >= 1)
    # plan = multi-body islands in order
    rows_ = s.plan_rows()
    assert len(rows_) == int((sizes >= 2).sum())
    for (b0, b1, e0, e1) in rows_:
        assert b1 - b0 >= 2 and e0 == s.padj_off[b0] and e1 == s.padj_off[b1]
        island = set(s.perm[b0:b1].tolist())
        for p in range(b0, b1):
            nbr = s.padj[s.padj_off[p]:s.padj_off[p + 1]]
            assert sorted(nbr.tolist()) == nbr.tolist()
            assert all(b0 <= q < b1 for q in nbr)
            assert {int(s.perm[q]) for q in nbr} == set(s.adj[s.adj_off[s.perm[p]]:s.adj_off[s.perm[p] + 1]].tolist())
            assert int(s.perm[p]) in island


def two_sphere_scene(d, r=0.06, axis=0):
    x = np.zeros((2, 4), np.float32)
    x[:, :] = 0.5
    x[:, 3] = 0
    x[0, axis] = 0.5 - d / 2
    x[1, axis] = 0.5 + d / 2
    v = np.zeros((2, 4), np.float32)
    return O.Scene(2, r, np.float32(1 / 120), 8, x, v)


@pytest.mark.parametrize("d", [0.05, 0.1, 0.119])
def test_jacobi_isolated_pair_reaches_contact_distance(d):
    s = two_sphere_scene(d)
    run_prefix(s)
    assert s.n_multi == 1
    s.run_kernel(O.RL_JACOBI, 0, 0)
    gap = float(np.linalg.norm(s.Q1[1, :3].astype(np.float64) - s.Q1[0, :3]))
    assert abs(gap - 2 * 0.06) < 4e-7
    # the pair moves symmetrically about its midpoint
    mid0 = (s.Q0[0, :3].astype(np.float64) + s.Q0[1, :3]) / 2
    mid1 = (s.Q1[0, :3].astype(np.float64) + s.Q1[1, :3]) / 2
    assert np.allclose(mid0, mid1, atol=1e-7)


def test_jacobi_coincident_pair_uses_fixed_normal():
    s = two_sphere_scene(0.0)
    run_prefix(s)
    s.run_kernel(O.RL_JACOBI, 0, 0)
    # the lower position is pushed along +x, the other along -x, by r each
    assert np.isclose(s.Q1[0, 0] - s.Q1[1, 0], 0.12, atol=1e-7)
    assert np.isclose(s.Q1[0, 0], 0.56, atol=1e-7)
    assert s.Q1[0, 1] == s.Q1[1, 1] and s.Q1[0, 2] == s.Q1[1, 2]


def test_jacobi_keeps_island_centroid():
    s = scene(1, 64)
    run_prefix(s)
    assert s.n_multi > 0
    Q_before = s.Q0.astype(np.float64).copy()
    for t in range(8):
        for k in range(s.n_multi):
            s.run_kernel(O.RL_JACOBI, k, t)
    for (b0, b1, e0, e1) in s.plan_rows():
        deg = np.diff(s.padj_off[b0:b1 + 1])
        if np.all(deg == deg[0]):   # equal weights: pair forces cancel in the sum
            c0 = Q_before[b0:b1, :3].mean(0)
            c1 = s.Q0[b0:b1, :3].astype(np.float64).mean(0)
            assert np.allclose(c0, c1, atol=1e-6)


def test_free_flight_and_walls():
    x = np.array([[0.5, 0.5, 0.5, 0], [0.2, 0.8, 0.5, 0], [0.061, 0.5, 0.938, 0]], np.float32)
    v = np.array([[0.3, -0.2, 0.1, 0], [1.0, 0.0, -1.0, 0], [-1.0, 0.5, 1.0, 0]], np.float32)
    s = O.Scene(3, np.float32(0.06), np.float32(1 / 120), 8, x, v)
    s.step()
    dt = np.float32(1 / 120)
    # free bodies: x' = fma(dt, v, x), v' = v exactly
    for i in (0, 1):
        for c in range(3):
            assert s.X[i, c] == np.float32(np.float64(dt) * np.float64(v[i, c]) + np.float64(x[i, c]))
            assert s.V[i, c] == v[i, c]
    # body 2 crosses the lower x wall and the upper z wall
    assert s.X[2, 0] == np.float32(0.06) and s.V[2, 0] == np.float32(1.0)
    assert s.X[2, 2] == np.float32(1.0) - np.float32(0.06) and s.V[2, 2] == np.float32(-1.0)


@pytest.mark.parametrize("seed,n", [(1, 64), (7, 64), (8, 150)])
def test_step_topological_order_invariance(seed, n):
    base = scene(seed, n)
    for _ in range(3):                       # advance a few steps to get a generic state
        base.step()
    ref = O.Scene(n, float(base.c.r), float(base.c.dt), 8, base.X, base.V)
    ref.step()
    s = O.Scene(n, float(base.c.r), float(base.c.dt), 8, base.X, base.V)
    run_prefix(s)
    kl = s.step_kernels()[4:]
    accs = [s.access(*k) for k in kl]
    adj = O.dag(accs)
    rng = np.random.default_rng(seed)
    snap = {f: getattr(s, f).copy() for f in ("X", "V", "P", "Q0", "Q1")}
    for _ in range(10):
        for f, a in snap.items():
            getattr(s, f)[...] = a
        for q in O.random_topological_order(adj, rng):
            s.run_kernel(*kl[q])
        assert np.array_equal(s.X.view(np.uint32), ref.X.view(np.uint32))
        assert np.array_equal(s.V.view(np.uint32), ref.V.view(np.uint32))


def test_step_kernel_list_shape():
    s = scene(1, 64)
    run_prefix(s)
    kl = s.step_kernels()
    m = s.n_multi
    assert len(kl) == 5 + 8 * m
    # iteration-major order of the Jacobi kernels
    jac = kl[4:-1]
    assert jac == [(O.RL_JACOBI, k, t) for t in range(8) for k in range(m)]
    # different islands never conflict; consecutive iterations of one island do
    accs = {k: s.access(*k) for k in jac}
    for t in range(7):
        for a in range(m):
            assert O.conflict(accs[(O.RL_JACOBI, a, t)], accs[(O.RL_JACOBI, a, t + 1)])
            for b in range(m):
                if a != b:
                    assert not O.conflict(accs[(O.RL_JACOBI, a, t)], accs[(O.RL_JACOBI, b, t + 1)])


def test_scene_statistics_match_the_workload_shape():
    """64 spheres at the default density keep several multi-body islands (and
    so several independent Jacobi chains) per step after the start-up overlaps
    are resolved."""
    multis, contacts = [], []
    for seed in range(1, 4):
        s = scene(seed, 64)
        for step in range(80):
            s.step()
            if step >= 40:
                multis.append(s.n_multi)
                contacts.append(s.meta[2] // 2)
    assert 4 <= np.mean(multis) <= 20
    assert 5 <= np.mean(contacts) <= 60


# ---------------------------------------------------------------------------
# body permutation (islands kernel's perm / inv_perm, permute, integrate)
# ---------------------------------------------------------------------------

def clamp_reflect(p, v, r):
    """Integrator semantics for a body whose corrected position equals its
    prediction p: clamp to [r, 1 - r], the velocity's sign set by the wall."""
    x, v = p.copy(), v.copy()
    lo, hi = np.float32(r), np.float32(1.0) - np.float32(r)
    for c in range(3):
        if x[c] < lo:
            x[c], v[c] = lo, abs(v[c])
        elif x[c] > hi:
            x[c], v[c] = hi, -abs(v[c])
    return x, v


def non_involutive_scene(L=None, seeds=range(1, 40), n=64):
    """A seeded scene (prefix run) whose body permutation is not its own
    inverse, so that perm and inv_perm cannot be told apart by accident."""
    for seed in seeds:
        s = scene(seed, n, L=L)
        for _ in range(2):
            s.step()
        t = O.Scene(n, float(s.c.r), float(s.c.dt), 8, s.X, s.V, L=L)
        run_prefix(t)
        if not np.array_equal(t.perm[t.perm], np.arange(n)):
            return t
    raise AssertionError("no scene with a non-involutive permutation")


def pin_permute_groups_islands(L=None):
    """Permute's output, row p, is the predicted state of the body at place p
    when bodies are ordered by (island label, body index), the order that
    groups every island into a contiguous range.  The order is rebuilt here
    from the labels alone (themselves pinned against scipy's components)."""
    s = non_involutive_scene(L)
    order = np.lexsort((np.arange(s.n), s.label))
    assert np.array_equal(s.Q0.view(np.uint32), s.P[order].view(np.uint32)), "permute: wrong gather"
    assert np.array_equal(s.perm, order)
    assert np.array_equal(s.inv_perm[order], np.arange(s.n))


def pin_integrate_unpermutes_without_sweeps(L=None):
    """With no Jacobi sweep the corrected positions are the predicted ones, so
    after a step every body i sits at its own wall-clamped prediction
    fma(dt, v, x) and keeps its velocity (up to the wall's sign flip)."""
    base = non_involutive_scene(L)
    n = base.n
    s = O.Scene(n, float(base.c.r), float(base.c.dt), 0, base.X, base.V, L=L)
    x0, v0 = base.X.copy(), base.V.copy()
    s.step()
    assert s.n_multi > 0 and not np.array_equal(s.perm[s.perm], np.arange(n))
    dt = np.float32(base.c.dt)
    for i in range(n):
        p = (np.float64(dt) * v0[i].astype(np.float64) + x0[i].astype(np.float64)).astype(np.float32)
        p[3] = x0[i, 3]
        xe, ve = clamp_reflect(p, v0[i], base.c.r)
        assert np.array_equal(s.X[i, :3].view(np.uint32), xe[:3].view(np.uint32)), f"body {i}: position"
        assert np.array_equal(s.V[i, :3].view(np.uint32), ve[:3].view(np.uint32)), f"body {i}: velocity"


def pin_free_bodies_fly_free_in_a_full_step(L=None):
    """In a full step (8 sweeps) on a scene with contacts, a body with no
    contact moves by exactly fma(dt, v, x) and keeps v, whatever happens to
    the other bodies."""
    base = non_involutive_scene(L)
    n = base.n
    s = O.Scene(n, float(base.c.r), float(base.c.dt), 8, base.X, base.V, L=L)
    x0, v0 = base.X.copy(), base.V.copy()
    s.step()
    dt = np.float64(np.float32(base.c.dt))
    lo, hi = np.float32(base.c.r), np.float32(1.0) - np.float32(base.c.r)
    free = 0
    for i in range(n):
        if s.deg[i] != 0:
            continue
        p = (dt * v0[i, :3].astype(np.float64) + x0[i, :3].astype(np.float64)).astype(np.float32)
        if np.any(p < lo) or np.any(p > hi):
            continue
        free += 1
        assert np.array_equal(s.X[i, :3].view(np.uint32), p.view(np.uint32)), f"free body {i} moved wrongly"
        assert np.array_equal(s.V[i, :3].view(np.uint32), v0[i, :3].view(np.uint32)), f"free body {i} velocity"
    assert free >= 4 and s.n_multi > 0


def pin_pair_velocity_from_correction(L=None):
    """Closed form of a full step for an isolated resting pair at distance
    d < 2r along x: the first sweep separates the pair to exactly 2r, so each
    body moves by (2r - d) / 2 along the pair's axis and the integrator turns
    that correction into the velocity (2r - d) / (2 dt), outwards."""
    d, r = 0.1, 0.06
    x = np.full((2, 4), 0.5, np.float32)
    x[:, 3] = 0
    x[0, 0], x[1, 0] = 0.5 - d / 2, 0.5 + d / 2
    v = np.zeros((2, 4), np.float32)
    dt = np.float32(1 / 120)
    s = O.Scene(2, r, dt, 8, x, v, L=L)
    s.step()
    h = (2 * r - float(x[1, 0] - x[0, 0])) / 2
    assert abs(float(s.X[0, 0]) - (float(x[0, 0]) - h)) < 1e-6 and abs(float(s.X[1, 0]) - (float(x[1, 0]) + h)) < 1e-6
    assert abs(float(s.V[0, 0]) + h / float(dt)) < 1e-3 and abs(float(s.V[1, 0]) - h / float(dt)) < 1e-3
    assert np.all(s.V[:, 1:3] == 0) and np.all(s.X[:, 1:3] == np.float32(0.5))


def test_pair_velocity_from_correction():
    pin_pair_velocity_from_correction()


def test_permute_groups_bodies_by_island():
    pin_permute_groups_islands()


def test_integrate_unpermutes_without_sweeps():
    pin_integrate_unpermutes_without_sweeps()


def test_free_bodies_fly_free_in_a_full_step():
    pin_free_bodies_fly_free_in_a_full_step()


def test_odd_sweep_count_is_rejected():
    """Sweeps alternate between the two position buffers and the integrator
    reads the first, so an odd count would drop the last sweep."""
    sc = inputs.rl_scene(seed=1, n=16)
    with pytest.raises(ValueError):
        O.Scene(sc.n, float(sc.radius), float(sc.dt), 1, sc.x, sc.v)
