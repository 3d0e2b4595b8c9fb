"""Householder reduction to upper Hessenberg form (oracle, test only).

Restates Golub & Van Loan, *Matrix Computations*, 4th ed., Algorithm 7.4.2:
for k = 1..n-2 a Householder reflector P_k = I - tau v v^T, acting on rows
k+1..n, annihilates A(k+2:n, k); A <- P_k A P_k.  Here the reflector follows
the LAPACK dlarfg convention (v(1) = 1, P x = beta e_1 with
beta = -sign(x_1) ||x||), and the same reflectors are applied to B from the
left and to C from the right, so that with Q = P_1 P_2 ... P_{n-2}

    H = Q^T A Q,   Bt = Q^T B,   Ct = C Q,

and (H, Bt, Ct, D) has the same transfer function as (A, B, C, D).
Unblocked and in float64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["house", "hessenberg", "normalize_signs"]


def house(x):
    """(v, tau, beta) with (I - tau v v^T) x = beta e_1 and v[0] = 1."""
    x = np.asarray(x, dtype=np.float64)
    alpha = x[0]
    sigma = np.linalg.norm(x[1:])
    v = np.zeros_like(x)
    v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, alpha
    norm = np.hypot(alpha, sigma)
    beta = -norm if alpha >= 0 else norm
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def hessenberg(A, B=None, C=None, want_q: bool = False):
    """Return (H, Bt, Ct[, Q]) with H = Q^T A Q upper Hessenberg."""
    H = np.array(A, dtype=np.float64, copy=True)
    n = H.shape[0]
    Bt = None if B is None else np.array(B, dtype=np.float64, copy=True)
    Ct = None if C is None else np.array(C, dtype=np.float64, copy=True)
    Q = np.eye(n) if want_q else None
    for k in range(n - 2):
        v, tau, beta = house(H[k + 1:, k])
        if tau == 0.0:
            continue
        # left: rows k+1..n-1 of A (columns k..n-1) and of B
        w = v @ H[k + 1:, k:]
        H[k + 1:, k:] -= tau * np.outer(v, w)
        H[k + 2:, k] = 0.0
        H[k + 1, k] = beta
        if Bt is not None:
            wb = v @ Bt[k + 1:, :]
            Bt[k + 1:, :] -= tau * np.outer(v, wb)
        # right: columns k+1..n-1 of A (all rows) and of C
        z = H[:, k + 1:] @ v
        H[:, k + 1:] -= tau * np.outer(z, v)
        if Ct is not None:
            zc = Ct[:, k + 1:] @ v
            Ct[:, k + 1:] -= tau * np.outer(zc, v)
        if Q is not None:
            zq = Q[:, k + 1:] @ v
            Q[:, k + 1:] -= tau * np.outer(zq, v)
    # exact zeros below the first subdiagonal
    H[np.tril_indices(n, -2)] = 0.0
    out = (H, Bt, Ct)
    if want_q:
        out = out + (Q,)
    return out


def normalize_signs(H, Bt=None, Ct=None):
    """Fix the sign freedom of Q (Q -> Q S with S = diag(+-1), S[0,0] = 1) so
    that every subdiagonal entry of H is >= 0.  Two reductions of the same A
    with Q e_1 = e_1 and unreduced H agree after this (implicit-Q theorem,
    Golub & Van Loan Theorem 7.4.2)."""
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    s = np.ones(n)
    for i in range(n - 1):
        sub = H[i + 1, i] * s[i]
        s[i + 1] = -1.0 if sub < 0 else 1.0
    Hn = s[:, None] * H * s[None, :]
    Bn = None if Bt is None else s[:, None] * np.asarray(Bt)
    Cn = None if Ct is None else np.asarray(Ct) * s[None, :]
    return Hn, Bn, Cn
