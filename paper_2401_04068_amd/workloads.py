"""Seeded synthetic workloads for frequency-response evaluation.

This module only *builds inputs*: state-space models (A, B, C, D) with a
prescribed pole set and frequency grids.  It contains none of the arithmetic
that evaluates G(jw) = C (jw I - A)^{-1} B + D, so both the CPU oracle and the
GPU library can be fed from it without sharing any of the method.

Every model is built the same way:

* a block-diagonal pole matrix Lambda holding real poles and 2x2 blocks
  [[sigma, omega_d], [-omega_d, sigma]] (eigenvalues sigma +/- j omega_d);
* a Haar-random orthogonal Q (QR of a standard normal matrix with the columns
  of Q multiplied by sign(diag R), Mezzadri 2007);
* A = Q Lambda Q^T, so A is normal and its eigenvalues are exactly the
  generated poles (up to rounding of the two products);
* B, C, D with independent standard normal entries.

Draw order inside one model's generator is fixed: real poles, then the pair
parameters, then the n x n normal matrix for Q, then B, C, D.

The five workloads:

* ``siso8``    n=8,   m=p=1,  200 log-spaced w in [1e-2, 1e2], seed 1
* ``mimo64``   n=64,  m=p=4,  2000 log-spaced w in [1e-3, 1e3], seed 2
* ``serving``  4096 requests, Poisson arrivals at 2000 req/s (seed 3);
  request r from seed 3_000_000 + r with n ~ U{4..128}, m, p ~ U{1..8},
  K ~ U{256..4096}, logspace(-3, 3, K)
* ``large1024`` n=1024, m=p=16, 10,000 log-spaced w in [1e-4, 1e4],
  models from seeds 4000..4007; ten queries, the last two repeat models 0
  and 3 on a grid shifted by half a log-step
* ``damped256`` 512 models, n=256, m=p=4, all poles complex with damping
  ratio zeta = 10^U(-5,-2) and natural frequency U(1,100); 3072 log-spaced
  w in [1e-3, 1e3] followed by 1024 points each within +/-1 % of the damped
  frequency of a uniformly chosen mode; model j from seed 5_000_000 + j
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Model",
    "haar_orthogonal",
    "pole_matrix",
    "mixed_pole_model",
    "damped_pole_model",
    "resonant_model",
    "logspace_grid",
    "siso8",
    "mimo64",
    "serving_requests",
    "serving_arrivals",
    "large1024_models",
    "large1024_queries",
    "damped256_model",
    "damped256",
    "WORKLOADS",
]


@dataclass
class Model:
    """One continuous-time state-space model and the grid it is evaluated on."""

    A: np.ndarray  # (n, n) float64, row-major
    B: np.ndarray  # (n, m)
    C: np.ndarray  # (p, n)
    D: np.ndarray  # (p, m)
    omega: np.ndarray  # (K,) rad/s
    poles: np.ndarray = field(default=None)  # (n,) complex, eigenvalues of A
    Q: np.ndarray = field(default=None)  # orthogonal factor, A = Q Lambda Q^T
    Lam: np.ndarray = field(default=None)  # block-diagonal pole matrix
    seed: int = -1
    E: np.ndarray = field(default=None)  # descriptor systems: E x' = A x + B u

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def m(self) -> int:
        return self.B.shape[1]

    @property
    def p(self) -> int:
        return self.C.shape[0]

    @property
    def K(self) -> int:
        return self.omega.shape[0]


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix (Mezzadri 2007, sec. 5)."""
    Z = rng.standard_normal((n, n))
    Qm, Rm = np.linalg.qr(Z)
    d = np.sign(np.diag(Rm))
    d[d == 0] = 1.0
    return Qm * d[None, :]


def pole_matrix(real_poles: np.ndarray, sigma: np.ndarray, omega_d: np.ndarray):
    """Block-diagonal Lambda: real poles first, then 2x2 rotation-scaling blocks.

    Returns (Lambda, poles) with poles listed in block order (each pair as
    sigma + j omega_d, sigma - j omega_d).
    """
    n_real = len(real_poles)
    n_pairs = len(sigma)
    n = n_real + 2 * n_pairs
    Lam = np.zeros((n, n))
    poles = np.empty(n, dtype=np.complex128)
    for i, lam in enumerate(real_poles):
        Lam[i, i] = lam
        poles[i] = lam
    for q in range(n_pairs):
        i = n_real + 2 * q
        Lam[i, i] = sigma[q]
        Lam[i + 1, i + 1] = sigma[q]
        Lam[i, i + 1] = omega_d[q]
        Lam[i + 1, i] = -omega_d[q]
        poles[i] = complex(sigma[q], omega_d[q])
        poles[i + 1] = complex(sigma[q], -omega_d[q])
    return Lam, poles


def _finish_model(rng, Lam, poles, m, p, omega, seed) -> Model:
    n = Lam.shape[0]
    Q = haar_orthogonal(rng, n)
    A = Q @ Lam @ Q.T
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    D = rng.standard_normal((p, m))
    return Model(
        A=np.ascontiguousarray(A),
        B=np.ascontiguousarray(B),
        C=np.ascontiguousarray(C),
        D=np.ascontiguousarray(D),
        omega=np.ascontiguousarray(omega, dtype=np.float64),
        poles=poles,
        Q=Q,
        Lam=Lam,
        seed=seed,
    )


def mixed_pole_model(rng, n: int, m: int, p: int, omega, seed: int = -1) -> Model:
    """Real poles -U(0.1, 2) and pairs with sigma = -U(0.05, 1), omega_d = U(0.5, 10).

    floor(n/4) pairs and n - 2 floor(n/4) real poles.
    """
    n_pairs = n // 4
    n_real = n - 2 * n_pairs
    real_poles = -rng.uniform(0.1, 2.0, n_real)
    sigma = -rng.uniform(0.05, 1.0, n_pairs)
    omega_d = rng.uniform(0.5, 10.0, n_pairs)
    Lam, poles = pole_matrix(real_poles, sigma, omega_d)
    return _finish_model(rng, Lam, poles, m, p, omega, seed)


def damped_pole_model(rng, n: int, m: int, p: int, seed: int = -1):
    """All poles complex: zeta = 10^U(-5,-2), w_n = U(1,100),
    sigma = -zeta w_n, omega_d = w_n sqrt(1 - zeta^2).

    Returns (model without grid, omega_d) so a caller can cluster points.
    """
    n_pairs = n // 2
    zeta = 10.0 ** rng.uniform(-5.0, -2.0, n_pairs)
    w_n = rng.uniform(1.0, 100.0, n_pairs)
    sigma = -zeta * w_n
    omega_d = w_n * np.sqrt(1.0 - zeta * zeta)
    Lam, poles = pole_matrix(np.zeros(0), sigma, omega_d)
    mdl = _finish_model(rng, Lam, poles, m, p, np.zeros(0), seed)
    return mdl, omega_d


def resonant_model(n: int, m: int, p: int, zeta: float, wn: float, seed: int,
                   offsets=(0.0, 1e-8, -1e-8, 1e-7, -1e-7, 1e-6, 1e-5)) -> Model:
    """Mixed poles (as ``mixed_pole_model``, n - 2 states) plus one pair with
    damping ratio ``zeta`` and natural frequency ``wn``; the grid holds 24
    log-spaced points in [1e-2, 1e2] and the points omega_d (1 + offset) next
    to that pair's damped frequency (kappa(jw I - A) ~ max|pole| / (zeta wn)
    there)."""
    rng = np.random.default_rng(seed)
    n_pairs = (n - 2) // 4
    n_real = (n - 2) - 2 * n_pairs
    real_poles = -rng.uniform(0.1, 2.0, n_real)
    sigma = np.concatenate([[-zeta * wn], -rng.uniform(0.05, 1.0, n_pairs)])
    omega_d = np.concatenate([[wn * np.sqrt(1.0 - zeta * zeta)], rng.uniform(0.5, 10.0, n_pairs)])
    Lam, poles = pole_matrix(real_poles, sigma, omega_d)
    w = np.concatenate([logspace_grid(1e-2, 1e2, 24), omega_d[0] * (1.0 + np.asarray(offsets))])
    return _finish_model(rng, Lam, poles, m, p, w, seed)


def logspace_grid(lo: float, hi: float, K: int) -> np.ndarray:
    """K log-spaced points in [lo, hi], both endpoints included."""
    return np.logspace(np.log10(lo), np.log10(hi), K)


# ---------------------------------------------------------------- workloads

def siso8(seed: int = 1) -> Model:
    rng = np.random.default_rng(seed)
    return mixed_pole_model(rng, 8, 1, 1, logspace_grid(1e-2, 1e2, 200), seed)


def mimo64(seed: int = 2, K: int = 2000) -> Model:
    rng = np.random.default_rng(seed)
    return mixed_pole_model(rng, 64, 4, 4, logspace_grid(1e-3, 1e3, K), seed)


SERVING_N_REQUESTS = 4096
SERVING_RATE_HZ = 2000.0


def serving_arrivals(n_requests: int = SERVING_N_REQUESTS, rate_hz: float = SERVING_RATE_HZ,
                     seed: int = 3) -> np.ndarray:
    """Arrival times in seconds of a Poisson stream (exponential gaps)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    return np.cumsum(gaps)


def serving_request(r: int) -> Model:
    """Request r of the serving mix: dims drawn first, then the model."""
    seed = 3_000_000 + r
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 129))
    m = int(rng.integers(1, 9))
    p = int(rng.integers(1, 9))
    K = int(rng.integers(256, 4097))
    return mixed_pole_model(rng, n, m, p, logspace_grid(1e-3, 1e3, K), seed)


def serving_requests(count: int = SERVING_N_REQUESTS, start: int = 0):
    return [serving_request(r) for r in range(start, start + count)]


LARGE_SEEDS = tuple(range(4000, 4008))


def large1024_models(n: int = 1024, m: int = 16, p: int = 16, K: int = 10_000,
                     seeds=LARGE_SEEDS):
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        out.append(mixed_pole_model(rng, n, m, p, logspace_grid(1e-4, 1e4, K), s))
    return out


def large1024_queries(models):
    """Ten queries: models 0..7, then models 0 and 3 again on a grid shifted by
    half a log-step (the repeats reuse the resident reduction)."""
    q = [(i, mdl.omega) for i, mdl in enumerate(models)]
    for i in (0, 3):
        w = models[i].omega
        step = np.log10(w[1]) - np.log10(w[0])
        q.append((i, w * 10.0 ** (0.5 * step)))
    return q


def damped256_model(j: int, n: int = 256, m: int = 4, p: int = 4,
                    n_log: int = 3072, n_clustered: int = 1024) -> Model:
    seed = 5_000_000 + j
    rng = np.random.default_rng(seed)
    mdl, omega_d = damped_pole_model(rng, n, m, p, seed)
    base = logspace_grid(1e-3, 1e3, n_log)
    modes = rng.integers(0, len(omega_d), n_clustered)
    rel = rng.uniform(-0.01, 0.01, n_clustered)
    clustered = omega_d[modes] * (1.0 + rel)
    mdl.omega = np.ascontiguousarray(np.concatenate([base, clustered]))
    return mdl


def damped256(count: int = 512, **kw):
    return [damped256_model(j, **kw) for j in range(count)]


WORKLOADS = {
    "siso8": "n=8, m=p=1, K=200 over [1e-2,1e2], seed 1 (plain FP64 path)",
    "mimo64": "n=64, m=p=4, K=2000 over [1e-3,1e3], seed 2 (plain FP64 path)",
    "serving": "4096 Poisson requests at 2000 req/s, n~U{4..128}, m,p~U{1..8}, "
               "K~U{256..4096} over [1e-3,1e3] (refined FP32 path)",
    "large1024": "n=1024, m=p=16, K=10000 over [1e-4,1e4], 8 models + 2 repeats",
    "damped256": "512 models n=256, m=p=4, zeta in [1e-5,1e-2], 4096 points, "
                 "25% clustered at resonances",
}


# ---------------------------------------------------------------- interval MDPs
#
# Stand-ins for the abstraction models of the paper's benchmark table (its
# appendix "Benchmarking models": grid abstractions of linear and non-linear
# systems, up to 42,634 states x 3 actions and 48.1 M transitions).  Those
# model files are not available here, so each synthetic model has the
# table's shape: n_states states (the last one an absorbing sink), n_actions
# actions per state, and per state-action pair a window of w consecutive
# destination states around a drifted centre plus the sink (w + 1
# transitions).  Nominal probabilities follow a discretised Gaussian over the
# window with a small sink mass; the interval is [p (1 - a), p (1 + b)] with
# a, b ~ U(0, spread), clipped to [0, 1], so sum lower <= 1 <= sum upper.
# Targets: a band of states at the top of the grid.


@dataclass
class IMDPModel:
    n_states: int
    stateptr: np.ndarray
    colptr: np.ndarray
    rowval: np.ndarray
    lower: np.ndarray
    upper: np.ndarray
    targets: np.ndarray
    seed: int

    @property
    def n_columns(self) -> int:
        return len(self.colptr) - 1

    @property
    def nnz(self) -> int:
        return len(self.rowval)


def imdp_synthetic(n_states: int, n_actions: int, window: int, seed: int, spread: float = 0.2,
                   target_frac: float = 0.05) -> IMDPModel:
    rng = np.random.default_rng(seed)
    S, A = int(n_states), int(n_actions)
    grid = S - 1  # the last state is the sink
    w = int(min(window, grid))
    C = S * A
    # the sink has one self-loop column per action
    cols = np.arange(C)
    state = cols // A
    shift = rng.integers(-max(1, w // 2), max(2, w // 2 + 1), size=C)
    centre = (state + shift) % max(grid, 1)
    off = np.arange(w) - w // 2
    dest = (centre[:, None] + off[None, :]) % max(grid, 1)  # (C, w)
    sigma = rng.uniform(0.15, 0.4, size=C)[:, None] * w
    p = np.exp(-0.5 * (off[None, :] / sigma) ** 2)
    sink_mass = rng.uniform(0.0, 0.02, size=C)
    p *= ((1.0 - sink_mass) / p.sum(axis=1))[:, None]
    a = rng.uniform(0.0, spread, size=p.shape)
    b = rng.uniform(0.0, spread, size=p.shape)
    lo = p * (1.0 - a)
    up = np.minimum(1.0, p * (1.0 + b))
    slo = sink_mass * (1.0 - rng.uniform(0.0, spread, size=C))
    sup = np.minimum(1.0, sink_mass * (1.0 + rng.uniform(0.0, spread, size=C)))
    # destinations sorted within each column (window wrap-around reorders)
    order = np.argsort(dest, axis=1, kind="stable")
    dest = np.take_along_axis(dest, order, axis=1)
    lo = np.take_along_axis(lo, order, axis=1)
    up = np.take_along_axis(up, order, axis=1)
    rowval = np.concatenate([dest, np.full((C, 1), S - 1)], axis=1)
    lower = np.concatenate([lo, slo[:, None]], axis=1)
    upper = np.concatenate([up, sup[:, None]], axis=1)
    # sink columns: stay with probability 1
    sink = state == S - 1
    rowval[sink] = S - 1
    lower[sink] = 0.0
    upper[sink] = 0.0
    lower[sink, -1] = 1.0
    upper[sink, -1] = 1.0
    m = w + 1
    colptr = np.arange(C + 1, dtype=np.int64) * m
    stateptr = np.arange(S + 1, dtype=np.int64) * A
    nt = max(1, int(target_frac * grid))
    targets = np.arange(grid - nt, grid)
    return IMDPModel(S, stateptr.astype(np.int32), colptr.astype(np.int64), rowval.reshape(-1).astype(np.int32),
                     lower.reshape(-1), upper.reshape(-1), targets.astype(np.int32), seed)


def imdp_pimdp2_shape(seed: int = 6000) -> IMDPModel:
    """The largest model of the paper's table: 42,634 states x 3 actions,
    375 window destinations + sink per column (48.0 M transitions)."""
    return imdp_synthetic(42634, 3, 375, seed)


# ---------------------------------------------------------------- descriptor systems


def descriptor_model(n: int, m: int, p: int, n_alg: int, seed: int, omega=None) -> Model:
    """A descriptor system E x' = A x + B u, y = C x + D u with n - n_alg
    finite poles (the mixed pole recipe: real -U(0.1, 2), pairs with
    sigma = -U(0.05, 1), omega_d = U(0.5, 10)) and n_alg algebraic states
    (E singular when n_alg > 0): in Weierstrass-like form
    E0 = diag(I, 0), A0 = diag(Lambda, I), then E = P E0 R, A = P A0 R with
    P, R Haar orthogonal times diagonals U(0.5, 2) (well conditioned).  The
    finite poles are Lambda's; the algebraic block adds a constant part to G.
    omega: default 300 log-spaced points in [1e-2, 1e2]."""
    rng = np.random.default_rng(seed)
    nd = n - n_alg
    n_pairs = nd // 4
    n_real = nd - 2 * n_pairs
    real_poles = -rng.uniform(0.1, 2.0, n_real)
    sigma = -rng.uniform(0.05, 1.0, n_pairs)
    omega_d = rng.uniform(0.5, 10.0, n_pairs)
    Lam, poles = pole_matrix(real_poles, sigma, omega_d)
    E0 = np.zeros((n, n))
    E0[:nd, :nd] = np.eye(nd)
    A0 = np.zeros((n, n))
    A0[:nd, :nd] = Lam
    A0[nd:, nd:] = np.eye(n_alg)
    P = haar_orthogonal(rng, n) * rng.uniform(0.5, 2.0, n)[None, :]
    R = haar_orthogonal(rng, n) * rng.uniform(0.5, 2.0, n)[None, :]
    E = P @ E0 @ R
    A = P @ A0 @ R
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    D = rng.standard_normal((p, m))
    w = logspace_grid(1e-2, 1e2, 300) if omega is None else np.asarray(omega, dtype=np.float64)
    return Model(A=np.ascontiguousarray(A), B=B, C=C, D=D, omega=np.ascontiguousarray(w), poles=poles,
                 seed=seed, E=np.ascontiguousarray(E))
