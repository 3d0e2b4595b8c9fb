"""Robust value iteration for interval Markov decision processes (IMDPs) --
TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's problem statement (section 2, "Robust Value Iteration for
IMDPs": the IMDP tuple, feasible distributions Gamma_{s,a}, the objective of
Eq. 1 and the recursion of Eq. 2), its specification options (section 3.2:
finite- and infinite-horizon reachability, discounted reward, pessimistic or
optimistic adversary, maximising or minimising strategy, time-dependent or
stationary policies), and the inner problem of Eq. 3 solved by
O-maximization (section 4), in both the sequential form and the form built
on an ordered cumulative sum of the gaps.

Model layout (compressed sparse columns, one column per state-action pair):
the columns of state s are stateptr[s] .. stateptr[s+1]-1; column j holds the
destinations rowval[colptr[j] .. colptr[j+1]-1] with probability bounds
lower[.] and upper[.].  Everything is plain Python / numpy in float64.

Readings where the paper is silent (each also listed in the design notes):

* ties in the ordering by value are broken by destination index (a stable
  sort): the value is the same for any tie order, the distribution is not;
* ties between actions go to the lowest action index;
* discounted reward: V_0 = r and V_k = r + gamma * opt_a opt_p sum p V_{k-1}
  (the paper names the property but does not write its recursion);
* reach-avoid: avoid states are held at 0 (a state in both sets counts as a
  goal);
* a finite-horizon policy is returned as policy[s, t], t = 0 .. K-1, the
  action to take at time t, i.e. the maximiser of iteration K - t (with K - t
  steps to go);
* infinite horizon: iterate until max_s |V_k - V_{k-1}| < eps; the returned
  policy is the maximiser of the last iteration;
* O-maximization when the upper bounds cannot absorb the remaining mass
  (sum of upper < 1, an infeasible interval set) assigns every gap and leaves
  the rest unassigned, which is what the sequential procedure does.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

REACH = 0
REACH_AVOID = 1
REWARD = 2


@dataclass
class IMDP:
    """An IMDP in compressed sparse columns (one column per (s, a))."""
    n_states: int
    stateptr: np.ndarray   # int, n_states + 1
    colptr: np.ndarray     # int, n_columns + 1
    rowval: np.ndarray     # int, nnz (destination states)
    lower: np.ndarray      # float64, nnz
    upper: np.ndarray      # float64, nnz

    @property
    def n_columns(self) -> int:
        return len(self.colptr) - 1

    def column(self, j: int):
        a, b = int(self.colptr[j]), int(self.colptr[j + 1])
        return self.rowval[a:b], self.lower[a:b], self.upper[a:b]


@dataclass
class Spec:
    """Property and modes (section 3.2)."""
    kind: int = REACH
    horizon: int = 100            # > 0: finite horizon K; 0: infinite
    eps: float = 1e-6             # infinite horizon: stop when residual < eps
    targets: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    avoid: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    reward: Optional[np.ndarray] = None
    discount: float = 1.0
    pessimistic: bool = True      # adversary minimises (else maximises)
    maximize: bool = True         # strategy maximises (else minimises)
    max_iterations: int = 100000  # infinite horizon safety bound


# ------------------------------------------------------------ O-maximization

def ordering(values: np.ndarray, dest: np.ndarray, pessimistic: bool) -> np.ndarray:
    """Positions of a column's destinations in the order mass is handed out
    (section 4): lowest value first when the adversary minimises, highest
    first when it maximises; ties by destination index."""
    v = values[dest]
    key = v if pessimistic else -v
    return np.lexsort((dest, key))


def omax_sequential(values, dest, lower, upper, pessimistic: bool = True) -> np.ndarray:
    """The feasible distribution that optimises sum p V for the adversary,
    built as the sequential procedure of section 4 describes: start from the
    lower bounds, then walk the ordering and give each destination as much of
    the remaining mass as its gap allows."""
    p = np.array(lower, dtype=np.float64, copy=True)
    rem = 1.0 - float(np.sum(lower))
    gap = np.asarray(upper, dtype=np.float64) - np.asarray(lower, dtype=np.float64)
    for o in ordering(values, dest, pessimistic):
        if gap[o] < rem:
            p[o] += gap[o]
            rem -= gap[o]
        else:
            p[o] += rem
            break
    return p


def omax_cumsum(values, dest, lower, upper, pessimistic: bool = True) -> np.ndarray:
    """The same distribution from an ordered cumulative sum of the gaps
    (section 4): the mass left for the i-th destination in the ordering is
    rem minus the gaps of the destinations before it, clipped to [0, gap]."""
    lower = np.asarray(lower, dtype=np.float64)
    gap = np.asarray(upper, dtype=np.float64) - lower
    rem = 1.0 - float(np.sum(lower))
    order = ordering(values, dest, pessimistic)
    cum = np.cumsum(gap[order])
    p = lower.copy()
    for i, o in enumerate(order):
        before = cum[i] - gap[o]
        p[o] += min(gap[o], max(rem - before, 0.0))
    return p


def column_value(values, imdp: IMDP, j: int, pessimistic: bool) -> float:
    """opt_{p in Gamma_{s,a}} sum_s' p(s') V(s') for column j (Eq. 3's inner
    problem)."""
    dest, lo, up = imdp.column(j)
    if len(dest) == 0:
        return 0.0
    p = omax_sequential(values, dest, lo, up, pessimistic)
    return float(np.dot(p, values[dest]))


# ------------------------------------------------------------ value iteration

def _fixed(spec: Spec, n: int):
    """(mask, value) of states whose value the recursion does not update."""
    fixed = np.zeros(n, dtype=bool)
    val = np.zeros(n)
    if spec.kind in (REACH, REACH_AVOID):
        if spec.kind == REACH_AVOID and len(spec.avoid):
            fixed[np.asarray(spec.avoid)] = True
            val[np.asarray(spec.avoid)] = 0.0
        fixed[np.asarray(spec.targets, dtype=np.int64)] = True
        val[np.asarray(spec.targets, dtype=np.int64)] = 1.0
    return fixed, val


def initial_values(imdp: IMDP, spec: Spec) -> np.ndarray:
    """V_0 of Eq. 2: the goal indicator (reachability), r (reward)."""
    n = imdp.n_states
    if spec.kind == REWARD:
        return np.asarray(spec.reward, dtype=np.float64).copy()
    fixed, val = _fixed(spec, n)
    v = np.zeros(n)
    v[fixed] = val[fixed]
    return v


def bellman(values: np.ndarray, imdp: IMDP, spec: Spec):
    """One step of Eq. 2: returns (V_k, argopt action index per state, the
    per-column values).  Action indices count from 0 within each state."""
    n = imdp.n_states
    q = np.array([column_value(values, imdp, j, spec.pessimistic) for j in range(imdp.n_columns)])
    newv = np.empty(n)
    act = np.zeros(n, dtype=np.int64)
    for s in range(n):
        a0, a1 = int(imdp.stateptr[s]), int(imdp.stateptr[s + 1])
        qs = q[a0:a1]
        if len(qs) == 0:
            best, arg = 0.0, 0
        else:
            arg = int(np.argmax(qs) if spec.maximize else np.argmin(qs))  # first on ties
            best = float(qs[arg])
        act[s] = arg
        if spec.kind == REWARD:
            newv[s] = spec.reward[s] + spec.discount * best
        else:
            newv[s] = best
    if spec.kind != REWARD:
        fixed, val = _fixed(spec, n)
        newv[fixed] = val[fixed]
    return newv, act, q


def value_iteration(imdp: IMDP, spec: Spec):
    """Eq. 2 iterated: finite horizon K steps, or until the Bellman residual
    max_s |V_k - V_{k-1}| drops below eps.  Returns (V, k, residual,
    policy) with policy (n_states, K) for a finite horizon and (n_states,)
    for an infinite one."""
    v = initial_values(imdp, spec)
    n = imdp.n_states
    if spec.horizon > 0:
        K = spec.horizon
        pol = np.zeros((n, K), dtype=np.int64)
        res = 0.0
        for k in range(1, K + 1):
            nv, act, _ = bellman(v, imdp, spec)
            res = float(np.max(np.abs(nv - v))) if n else 0.0
            pol[:, K - k] = act
            v = nv
        return v, K, res, pol
    k = 0
    act = np.zeros(n, dtype=np.int64)
    res = np.inf
    while k < spec.max_iterations:
        nv, act, _ = bellman(v, imdp, spec)
        k += 1
        res = float(np.max(np.abs(nv - v))) if n else 0.0
        v = nv
        if res < spec.eps:
            break
    return v, k, res, act


# ------------------------------------------------------------ helpers

def from_dense(lower_cols, upper_cols):
    """Build an IMDP from per-state lists of dense (n_states x n_actions)
    bound matrices (columns are actions, rows destinations), keeping the
    destinations whose upper bound is nonzero."""
    n = len(lower_cols)
    stateptr = [0]
    colptr = [0]
    rows, lo, up = [], [], []
    for s in range(n):
        L = np.atleast_2d(np.asarray(lower_cols[s], dtype=np.float64).T).T
        U = np.atleast_2d(np.asarray(upper_cols[s], dtype=np.float64).T).T
        for a in range(L.shape[1]):
            nz = np.flatnonzero(U[:, a] > 0)
            rows.extend(nz.tolist())
            lo.extend(L[nz, a].tolist())
            up.extend(U[nz, a].tolist())
            colptr.append(len(rows))
        stateptr.append(len(colptr) - 1)
    return IMDP(n, np.array(stateptr), np.array(colptr), np.array(rows, dtype=np.int64),
                np.array(lo), np.array(up))
