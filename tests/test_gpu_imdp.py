"""GPU: robust value iteration for interval MDPs (imdp_vi.h) against the oracle
(oracle/imdp.py, sequential O-maximization in the paper's order).

Tolerance: one iteration forms each value as a sum of at most m + 2 products
of numbers in [0, max|V|] (lower-bound part, gap part, threshold remainder),
in a different order on each side, so the two differ by at most about
(m + 2) u max|V| per iteration (u = 2^-53); value iteration is
non-expansive in the max norm, so after K iterations the bound is
K (m + 2) u max|V|, doubled for safety.  Policies: where two actions' values
differ by less than that bound either choice is correct, so the GPU's choice
is checked to be optimal within the bound at every state and time step.
"""
import numpy as np
import pytest

from oracle import imdp as O
from paper_2401_04068_amd import workloads as wl

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _tol(K, m_max, vmax=1.0):
    return 2.0 * K * (m_max + 2) * U * max(vmax, 1.0)


def _oracle_model(m):
    return O.IMDP(m.n_states, m.stateptr, m.colptr, m.rowval, m.lower, m.upper)


def _solver(m):
    from paper_2401_04068_amd import binding

    return binding.IMDPSolver(m.n_states, m.stateptr, m.colptr, m.rowval, m.lower, m.upper)


def _run_both(m, spec_kw, gpu_kw):
    from paper_2401_04068_amd import binding

    om = _oracle_model(m)
    spec = O.Spec(**spec_kw)
    with _solver(m) as sol:
        got = sol.run(**gpu_kw)
    return om, spec, got


def _policy_is_optimal(om, spec, pol, tol):
    """Replays the oracle's iterations and checks that the GPU's action at
    every (state, time) is optimal within tol."""
    v = O.initial_values(om, spec)
    K = spec.horizon
    held = np.zeros(om.n_states, dtype=bool)  # goal / avoid states: any action
    if spec.kind != O.REWARD:
        held[np.asarray(spec.targets, dtype=np.int64)] = True
        if spec.kind == O.REACH_AVOID:
            held[np.asarray(spec.avoid, dtype=np.int64)] = True
    for k in range(1, K + 1):
        nv, act, q = O.bellman(v, om, spec)
        t = K - k
        for s in range(om.n_states):
            a0, a1 = int(om.stateptr[s]), int(om.stateptr[s + 1])
            if a1 <= a0 or held[s]:
                continue
            qs = q[a0:a1]
            best = qs.max() if spec.maximize else qs.min()
            chosen = qs[pol[s, t]]
            assert abs(chosen - best) <= tol, (s, t, pol[s, t], qs)
        v = nv


def _three_state_arrays():
    lower = [np.array([[0.0, 0.5], [0.1, 0.3], [0.2, 0.1]]),
             np.array([[0.1, 0.2], [0.2, 0.3], [0.3, 0.4]]),
             np.array([[0.0], [0.0], [1.0]])]
    upper = [np.array([[0.5, 0.7], [0.6, 0.5], [0.7, 0.3]]),
             np.array([[0.6, 0.6], [0.5, 0.5], [0.4, 0.4]]),
             np.array([[0.0], [0.0], [1.0]])]
    stateptr, colptr, rows, lo, up = [0], [0], [], [], []
    for s in range(3):
        for a in range(lower[s].shape[1]):
            rows.extend(range(3))
            lo.extend(lower[s][:, a])
            up.extend(upper[s][:, a])
            colptr.append(len(rows))
        stateptr.append(len(colptr) - 1)
    return wl.IMDPModel(3, np.array(stateptr, dtype=np.int32), np.array(colptr), np.array(rows, dtype=np.int32),
                        np.array(lo), np.array(up), np.array([2], dtype=np.int32), 0)


@pytest.mark.parametrize("case", [
    ("reach_pess_max", 1, [0.2, 0.4, 1.0], dict(pessimistic=True, maximize=True)),
    ("reach_pess_max", 2, [0.42, 0.58, 1.0], dict(pessimistic=True, maximize=True)),
    ("reach_opt_max", 1, [0.7, 0.4, 1.0], dict(pessimistic=False, maximize=True)),
    ("reach_pess_min", 1, [0.1, 0.3, 1.0], dict(pessimistic=True, maximize=False)),
], ids=lambda c: f"{c[0]}-k{c[1]}")
def test_three_state_example_hand_values(case):
    """The hand-derived values of tests/golden/imdp_three_state.txt."""
    name, k, want, kw = case
    m = _three_state_arrays()
    with _solver(m) as sol:
        V, it, _, pol, _ = sol.run(horizon=k, targets=[2], **kw)
    assert it == k
    np.testing.assert_allclose(V, want, rtol=0, atol=1e-14)


def test_three_state_reward_and_reach_avoid():
    from paper_2401_04068_amd import binding

    m = _three_state_arrays()
    with _solver(m) as sol:
        V, _, _, _, _ = sol.run(prop=binding.IMDP_REWARD, horizon=1, reward=[1.0, 2.0, 3.0], discount=0.9)
        np.testing.assert_allclose(V, [2.53, 3.89, 5.7], rtol=0, atol=1e-14)
        V, _, _, _, _ = sol.run(prop=binding.IMDP_REACH_AVOID, horizon=2, targets=[2], avoid=[1])
        np.testing.assert_allclose(V, [0.24, 0.0, 1.0], rtol=0, atol=1e-14)
        # infinite horizon: the fixed point is 1 everywhere (the oracle pin)
        V, it, res, pol, _ = sol.run(horizon=0, eps=1e-12, targets=[2])
        assert res < 1e-12 and it > 10
        np.testing.assert_allclose(V, 1.0, atol=1e-10)
        assert list(pol) == [0, 1, 0]


# (n_states, n_actions, window): columns of 1 .. 2000+ destinations cover every
# register class and the streaming path
SHAPES = [(40, 2, 3), (64, 3, 30), (120, 2, 100), (150, 2, 160), (300, 1, 250), (350, 1, 300), (400, 2, 500),
          (700, 1, 600), (900, 1, 1000), (2600, 1, 2200)]


MODES = [(True, True), (False, True), (True, False), (False, False)]
# the largest shapes in one mode only (the oracle is slow there)
CASES = [(s, pm) for s in SHAPES for pm in (MODES if s[0] * s[2] <= 300_000 else MODES[:1])]


@pytest.mark.parametrize("shape,pess,maxi", [(s, p, x) for s, (p, x) in CASES],
                         ids=[f"S{s[0]}A{s[1]}w{s[2]}-{p}-{x}" for s, (p, x) in CASES])
def test_random_models_match_oracle(shape, pess, maxi):
    S, A, w = shape
    m = wl.imdp_synthetic(S, A, w, seed=7000 + S + w)
    K = 12 if S * w <= 300_000 else 3
    print(f"case imdp S={S} A={A} w={w} pess={pess} max={maxi}", flush=True)
    om, spec, got = _run_both(m, dict(kind=O.REACH, horizon=K, targets=m.targets, pessimistic=pess, maximize=maxi),
                              dict(horizon=K, targets=m.targets, pessimistic=pess, maximize=maxi))
    V, it, res, pol, _ = got
    Vo, ko, reso, _ = O.value_iteration(om, spec)
    tol = _tol(K, w + 1)
    assert it == K
    assert np.max(np.abs(V - Vo)) <= tol, np.max(np.abs(V - Vo))
    assert abs(res - reso) <= 2 * tol
    if S * w <= 60_000:
        _policy_is_optimal(om, spec, pol, tol)


def test_reward_and_reach_avoid_match_oracle():
    from paper_2401_04068_amd import binding

    m = wl.imdp_synthetic(150, 3, 40, seed=7301)
    rng = np.random.default_rng(7302)
    r = rng.uniform(-1, 3, m.n_states)
    om = _oracle_model(m)
    K = 20
    with _solver(m) as sol:
        V, _, _, pol, _ = sol.run(prop=binding.IMDP_REWARD, horizon=K, reward=r, discount=0.95, pessimistic=True,
                                  maximize=True)
        spec = O.Spec(kind=O.REWARD, horizon=K, reward=r, discount=0.95, pessimistic=True, maximize=True)
        Vo = O.value_iteration(om, spec)[0]
        tol = _tol(K, 41, np.max(np.abs(Vo)))
        assert np.max(np.abs(V - Vo)) <= tol
        _policy_is_optimal(om, spec, pol, tol)
        avoid = np.arange(10, 30)
        V, _, _, _, _ = sol.run(prop=binding.IMDP_REACH_AVOID, horizon=K, targets=m.targets, avoid=avoid,
                                pessimistic=False, maximize=False)
        Vo = O.value_iteration(om, O.Spec(kind=O.REACH_AVOID, horizon=K, targets=m.targets, avoid=avoid,
                                          pessimistic=False, maximize=False))[0]
        assert np.max(np.abs(V - Vo)) <= _tol(K, 41)
        assert np.all(V[avoid] == 0.0)


def test_infinite_horizon_matches_oracle():
    m = wl.imdp_synthetic(200, 2, 20, seed=7401)
    om = _oracle_model(m)
    with _solver(m) as sol:
        V, it, res, pol, _ = sol.run(horizon=0, eps=1e-9, targets=m.targets)
    Vo, ko, reso, polo = O.value_iteration(om, O.Spec(horizon=0, eps=1e-9, targets=m.targets))
    assert res < 1e-9
    assert abs(it - ko) <= 1  # the stopping test sits on a rounding-level residual difference at most
    assert np.max(np.abs(V - Vo)) <= max(_tol(ko, 21), 2e-9)


def test_edge_columns():
    """A state with no action, one-destination columns, lower bounds that sum
    to 1 (nothing left to hand out), upper bounds that sum to less than 1 (every
    gap handed out), and all-equal values (one tie group)."""
    stateptr = np.array([0, 0, 1, 2, 3, 4, 5], dtype=np.int32)  # state 0: no column
    cols = [
        ([1], [1.0], [1.0]),                       # state 1: stays
        ([0, 2, 3], [0.2, 0.3, 0.5], [0.2, 0.3, 0.5]),  # state 2: sum lower = 1
        ([1, 4], [0.1, 0.2], [0.3, 0.4]),          # state 3: sum upper = 0.7 < 1
        ([2, 3, 4, 5], [0.0] * 4, [0.5] * 4),      # state 4: ties when V is flat
        ([5], [1.0], [1.0]),                       # state 5: target, stays
    ]
    colptr, rows, lo, up = [0], [], [], []
    for d, l, u in cols:
        rows.extend(d)
        lo.extend(l)
        up.extend(u)
        colptr.append(len(rows))
    m = wl.IMDPModel(6, stateptr, np.array(colptr), np.array(rows, dtype=np.int32), np.array(lo), np.array(up),
                     np.array([5], dtype=np.int32), 0)
    om = _oracle_model(m)
    for pess in (True, False):
        for K in (1, 3, 7):
            with _solver(m) as sol:
                V, _, _, _, _ = sol.run(horizon=K, targets=[5], pessimistic=pess)
            Vo = O.value_iteration(om, O.Spec(horizon=K, targets=np.array([5]), pessimistic=pess))[0]
            np.testing.assert_allclose(V, Vo, rtol=0, atol=1e-15)


def test_pimdp2_shape_sampled_steps():
    """The largest benchmark shape (42,634 states x 3 actions, 48.1 M
    transitions): the GPU's V_{k-1} and V_k (k = 1, 2, 50) and the oracle's
    one step from that V_{k-1} at 300 sampled states (all their actions)."""
    m = wl.imdp_pimdp2_shape()
    om = _oracle_model(m)
    rng = np.random.default_rng(7501)
    sample = np.unique(np.concatenate([rng.choice(m.n_states, 300, replace=False), m.targets[:3],
                                       [m.n_states - 1]]))
    spec = O.Spec(kind=O.REACH, horizon=1, targets=m.targets)
    fixed = np.zeros(m.n_states, dtype=bool)
    fixed[m.targets] = True
    with _solver(m) as sol:
        for k in (1, 2, 50):
            print(f"case pimdp2 k={k}", flush=True)
            Vprev = O.initial_values(om, spec) if k == 1 else sol.run(horizon=k - 1, targets=m.targets,
                                                                      want_policy=False)[0]
            V, _, _, pol, _ = sol.run(horizon=k, targets=m.targets)
            for s in sample:
                if fixed[s]:
                    assert V[s] == 1.0
                    continue
                a0, a1 = int(om.stateptr[s]), int(om.stateptr[s + 1])
                q = np.array([O.column_value(Vprev, om, j, True) for j in range(a0, a1)])
                assert abs(V[s] - q.max()) <= _tol(1, 377), (s, V[s], q)
                assert abs(q[pol[s, 0]] - q.max()) <= _tol(1, 377)
            assert np.all((V >= 0) & (V <= 1))
            assert np.all(V >= Vprev - 1e-15)  # reachability values grow with k
