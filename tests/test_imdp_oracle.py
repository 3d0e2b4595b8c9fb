"""CPU: pins of the IMDP value-iteration oracle (oracle/imdp.py).

* hand-derived values of the paper's three-state example
  (tests/golden/imdp_three_state.txt);
* O-maximization against a linear program (the inner problem of the paper's
  Eq. 3 is an LP over the box lower <= p <= upper with sum p = 1), solved by
  scipy's HiGHS;
* the sequential and cumulative-sum forms of O-maximization agree;
* lower == upper reduces to ordinary MDP value iteration (matrix products);
* one action per state: an interval Markov chain, policy 0 everywhere;
* reachability values stay in [0, 1], grow with k, and pessimistic <=
  optimistic.
"""
import os

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import imdp as O

HERE = os.path.dirname(os.path.abspath(__file__))


def three_state():
    lower = [np.array([[0.0, 0.5], [0.1, 0.3], [0.2, 0.1]]),
             np.array([[0.1, 0.2], [0.2, 0.3], [0.3, 0.4]]),
             np.array([[0.0], [0.0], [1.0]])]
    upper = [np.array([[0.5, 0.7], [0.6, 0.5], [0.7, 0.3]]),
             np.array([[0.6, 0.6], [0.5, 0.5], [0.4, 0.4]]),
             np.array([[0.0], [0.0], [1.0]])]
    # keep every destination (the paper's dense form), zero bounds included
    n = 3
    stateptr, colptr, rows, lo, up = [0], [0], [], [], []
    for s in range(n):
        for a in range(lower[s].shape[1]):
            rows.extend(range(n))
            lo.extend(lower[s][:, a])
            up.extend(upper[s][:, a])
            colptr.append(len(rows))
        stateptr.append(len(colptr) - 1)
    return O.IMDP(n, np.array(stateptr), np.array(colptr), np.array(rows), np.array(lo), np.array(up))


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "imdp_three_state.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((t[0], int(t[1]), np.array([float(x) for x in t[2:5]]), [int(x) for x in t[5:8]]))
    return rows


SPECS = {
    "reach_pess_max": dict(kind=O.REACH, pessimistic=True, maximize=True),
    "reach_opt_max": dict(kind=O.REACH, pessimistic=False, maximize=True),
    "reach_pess_min": dict(kind=O.REACH, pessimistic=True, maximize=False),
    "reach_avoid_pess_max": dict(kind=O.REACH_AVOID, pessimistic=True, maximize=True, avoid=np.array([1])),
    "reward_pess_max": dict(kind=O.REWARD, pessimistic=True, maximize=True, reward=np.array([1.0, 2.0, 3.0]),
                            discount=0.9),
}


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}-k{r[1]}")
def test_three_state_example_hand_values(row):
    name, k, want, pol = row
    spec = O.Spec(horizon=k, targets=np.array([2]), **SPECS[name])
    V, iters, _, policy = O.value_iteration(three_state(), spec)
    assert iters == k
    np.testing.assert_allclose(V, want, rtol=0, atol=1e-14)
    # the action taken at time 0 is the maximiser of the last iteration
    for s in range(3):
        if pol[s] >= 0:
            assert policy[s, 0] == pol[s]


def _random_column(rng, m):
    lo = rng.uniform(0, 1, m)
    lo *= rng.uniform(0.2, 0.95) / lo.sum()
    up = lo + rng.uniform(0, 1, m) * rng.uniform(0.05, 0.6)
    if up.sum() < 1.0:
        up *= 1.0 / up.sum() * rng.uniform(1.0, 1.3)
        up = np.maximum(up, lo)
    return lo, np.minimum(up, 1.0)


@pytest.mark.parametrize("pessimistic", [True, False])
def test_omaximization_solves_the_linear_program(pessimistic):
    rng = np.random.default_rng(31)
    for trial in range(200):
        m = int(rng.integers(1, 40))
        lo, up = _random_column(rng, m)
        if up.sum() < 1.0 - 1e-12:
            continue
        values = rng.uniform(0, 1, 60)
        if trial % 3 == 0:  # ties
            values = np.round(values * 4) / 4
        dest = np.sort(rng.choice(60, m, replace=False))
        v = values[dest]
        c = v if pessimistic else -v
        lp = linprog(c, A_eq=np.ones((1, m)), b_eq=[1.0], bounds=list(zip(lo, up)), method="highs")
        assert lp.status == 0
        want = float(np.dot(lp.x, v))
        p = O.omax_sequential(values, dest, lo, up, pessimistic)
        assert np.all(p >= lo - 1e-15) and np.all(p <= up + 1e-15)
        assert abs(p.sum() - 1.0) <= 1e-12
        assert abs(float(np.dot(p, v)) - want) <= 1e-9


def test_sequential_and_cumulative_sum_forms_agree():
    rng = np.random.default_rng(32)
    for trial in range(300):
        m = int(rng.integers(1, 70))
        lo, up = _random_column(rng, m)
        values = rng.uniform(0, 1, 100)
        if trial % 4 == 0:
            values = np.round(values * 3) / 3
        dest = np.sort(rng.choice(100, m, replace=False))
        for pess in (True, False):
            a = O.omax_sequential(values, dest, lo, up, pess)
            b = O.omax_cumsum(values, dest, lo, up, pess)
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def _random_imdp(rng, n, acts, m, exact=False):
    stateptr, colptr, rows, lo, up = [0], [0], [], [], []
    for s in range(n):
        for a in range(acts):
            mm = min(n, m)
            dest = np.sort(rng.choice(n, mm, replace=False))
            if exact:
                p = rng.uniform(0.1, 1, mm)
                l = u = p / p.sum()
            else:
                l, u = _random_column(rng, mm)
            rows.extend(dest.tolist())
            lo.extend(l)
            up.extend(u)
            colptr.append(len(rows))
        stateptr.append(len(colptr) - 1)
    return O.IMDP(n, np.array(stateptr), np.array(colptr), np.array(rows), np.array(lo), np.array(up))


def test_point_intervals_reduce_to_mdp_value_iteration():
    rng = np.random.default_rng(33)
    n, acts = 12, 3
    M = _random_imdp(rng, n, acts, 5, exact=True)
    P = np.zeros((n, acts, n))
    for s in range(n):
        for a in range(acts):
            d, l, _ = M.column(M.stateptr[s] + a)
            P[s, a, d] = l
    goal = np.array([0, 5])
    spec = O.Spec(kind=O.REACH, horizon=15, targets=goal, pessimistic=True, maximize=True)
    V, _, _, _ = O.value_iteration(M, spec)
    v = np.zeros(n)
    v[goal] = 1.0
    for _ in range(15):
        v = np.max(P @ v, axis=1)
        v[goal] = 1.0
    np.testing.assert_allclose(V, v, rtol=0, atol=1e-13)
    spec_opt = O.Spec(kind=O.REACH, horizon=15, targets=goal, pessimistic=False, maximize=True)
    np.testing.assert_allclose(O.value_iteration(M, spec_opt)[0], v, rtol=0, atol=1e-13)


def test_single_action_chain_and_value_properties():
    rng = np.random.default_rng(34)
    M = _random_imdp(rng, 20, 1, 6)
    goal = np.array([3])
    prev = None
    for k in (1, 2, 5, 10):
        pess = O.value_iteration(M, O.Spec(horizon=k, targets=goal, pessimistic=True))
        opt = O.value_iteration(M, O.Spec(horizon=k, targets=goal, pessimistic=False))
        assert np.all(pess[3] == 0)  # one action: policy 0
        assert np.all((pess[0] >= 0) & (pess[0] <= 1 + 1e-15))
        assert np.all(pess[0] <= opt[0] + 1e-15)
        if prev is not None:
            assert np.all(pess[0] >= prev - 1e-15)
        prev = pess[0]


def test_infinite_horizon_converges_on_three_state_example():
    # pessimistic-max fixed point: with x = V(0), y = V(1) and action 0 / 1
    # as in the golden file, x = 0.5 x + 0.3 y + 0.2, y = 0.3 x + 0.3 y + 0.4,
    # whose solution is x = y = 1.
    spec = O.Spec(horizon=0, eps=1e-12, targets=np.array([2]))
    V, k, res, pol = O.value_iteration(three_state(), spec)
    assert res < 1e-12 and k > 10
    np.testing.assert_allclose(V, [1.0, 1.0, 1.0], atol=1e-10)
    assert list(pol) == [0, 1, 0]
