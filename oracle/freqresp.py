"""Frequency response by the definition -- oracle (test infrastructure only).

G(jw_k) = C (jw_k I - A)^{-1} B + D  for every w_k.

Each frequency is one dense complex solve with partial pivoting (LAPACK
zgesv through ``numpy.linalg.solve``), exactly the textbook definition: form
M = jw I - A, solve M X = B, return C X + D.  No Hessenberg form, no shared
factorisation between frequencies, no reordering.

``freqresp_extended`` adds classical iterative refinement (Wilkinson 1963;
Higham, *Accuracy and Stability of Numerical Algorithms*, 2nd ed., ch. 12):
the correction equation is solved with the float64 LU, while the residual
r = B - M X and the iterate X are held in extended precision
(``np.clongdouble``, 64-bit significand, unit roundoff 2^-64).  The limiting
forward error is then about kappa(M) * 2^-64 instead of kappa(M) * 2^-53.
"""
from __future__ import annotations

import numpy as np

__all__ = ["freqresp", "freqresp_extended", "freqresp_at", "freqresp_at_extended", "derivative_at", "derivative_at_extended", "cond2",
           "rel_err", "rel_err_max", "freqresp_descriptor", "freqresp_descriptor_extended"]


def _check(A, B, C, D, omega):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    m = B.shape[1]
    p = C.shape[0]
    if B.shape != (n, m) or C.shape != (p, n):
        raise ValueError("B must be n x m and C p x n")
    D = np.zeros((p, m)) if D is None else np.asarray(D, dtype=np.float64)
    if D.shape != (p, m):
        raise ValueError("D must be p x m")
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    return A, B, C, D, omega


def freqresp(A, B, C, D, omega, chunk: int = 256) -> np.ndarray:
    """G[k] = C (j omega[k] I - A)^{-1} B + D, shape (K, p, m), complex128.

    Frequencies are stacked ``chunk`` at a time into one batched
    ``numpy.linalg.solve`` call; each matrix in the stack is still factored on
    its own with partial pivoting.
    """
    A, B, C, D, omega = _check(A, B, C, D, omega)
    n = A.shape[0]
    K = omega.shape[0]
    G = np.empty((K, C.shape[0], B.shape[1]), dtype=np.complex128)
    eye = np.eye(n)
    Bc = B.astype(np.complex128)
    for k0 in range(0, K, chunk):
        w = omega[k0:k0 + chunk]
        M = 1j * w[:, None, None] * eye[None, :, :] - A[None, :, :]
        X = np.linalg.solve(M, np.broadcast_to(Bc, (len(w),) + Bc.shape))
        G[k0:k0 + chunk] = C[None, :, :] @ X + D[None, :, :]
    return G


def freqresp_extended(A, B, C, D, omega, iters: int = 3, return_longdouble: bool = False):
    """Oracle of record: float64 LU plus ``iters`` refinement steps with the
    residual and the iterate in extended precision.

    M = jw I - A is exact in clongdouble (its entries are float64 values).
    Each step: r = B - M X (extended), d = LU \\ r (float64 solve of the
    rounded residual), X = X + d (extended).  G = C X + D is formed in
    extended precision and rounded once at the end.
    """
    A, B, C, D, omega = _check(A, B, C, D, omega)
    n = A.shape[0]
    K = omega.shape[0]
    ld = np.clongdouble
    A_ld = A.astype(ld)
    B_ld = B.astype(ld)
    C_ld = C.astype(ld)
    D_ld = D.astype(ld)
    eye = np.eye(n)
    out = np.empty((K, C.shape[0], B.shape[1]), dtype=ld if return_longdouble else np.complex128)
    for k, w in enumerate(omega):
        M64 = 1j * w * eye - A
        M_ld = (1j * np.longdouble(w)) * np.eye(n, dtype=ld) - A_ld
        X = np.linalg.solve(M64, B.astype(np.complex128)).astype(ld)
        for _ in range(iters):
            r = B_ld - M_ld @ X
            d = np.linalg.solve(M64, r.astype(np.complex128))
            X = X + d.astype(ld)
        G = C_ld @ X + D_ld
        out[k] = G if return_longdouble else G.astype(np.complex128)
    return out


def freqresp_at(A, B, C, D, s, chunk: int = 256) -> np.ndarray:
    """G(s_k) = C (s_k I - A)^{-1} B + D at arbitrary complex points s_k,
    shape (K, p, m): the transfer matrix of the model off the imaginary axis
    (continuous time, s = sigma + j w), or of a discrete-time model
    x[t+1] = A x[t] + B u[t], y = C x + D u at z = s (z = exp(j theta) on the
    unit circle gives its frequency response; any linear-systems text, e.g.
    Kailath 1980, ch. 2).  One dense LU with partial pivoting per point."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    n = A.shape[0]
    K = s.shape[0]
    G = np.empty((K, C.shape[0], B.shape[1]), dtype=np.complex128)
    eye = np.eye(n)
    Bc = B.astype(np.complex128)
    for k0 in range(0, K, chunk):
        sk = s[k0:k0 + chunk]
        M = sk[:, None, None] * eye[None, :, :] - A[None, :, :]
        X = np.linalg.solve(M, np.broadcast_to(Bc, (len(sk),) + Bc.shape))
        G[k0:k0 + chunk] = C[None, :, :] @ X + D[None, :, :]
    return G


def freqresp_at_extended(A, B, C, D, s, iters: int = 3) -> np.ndarray:
    """``freqresp_at`` followed by the extended-precision refinement of
    ``freqresp_extended`` (residual and iterate in x87 extended precision);
    s_k is rounded to float64 real and imaginary parts first, and those are
    the points evaluated exactly."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    n = A.shape[0]
    ld = np.clongdouble
    A_ld, B_ld, C_ld, D_ld = A.astype(ld), B.astype(ld), C.astype(ld), D.astype(ld)
    eye = np.eye(n)
    out = np.empty((len(s), C.shape[0], B.shape[1]), dtype=np.complex128)
    for k, sk in enumerate(s):
        M64 = sk * eye - A
        s_ld = np.longdouble(sk.real) + 1j * np.longdouble(sk.imag)
        M_ld = s_ld * np.eye(n, dtype=ld) - A_ld
        X = np.linalg.solve(M64, B.astype(np.complex128)).astype(ld)
        for _ in range(iters):
            r = B_ld - M_ld @ X
            d = np.linalg.solve(M64, r.astype(np.complex128))
            X = X + d.astype(ld)
        out[k] = (C_ld @ X + D_ld).astype(np.complex128)
    return out


def derivative_at(A, B, C, D, s) -> np.ndarray:
    """dG/ds = -C (s I - A)^{-2} B at complex points s_k, shape (K, p, m): the
    derivative of G(s) = C (s I - A)^{-1} B + D (from d/ds M^{-1} =
    -M^{-1} (dM/ds) M^{-1} with dM/ds = I).  Two dense LU solves per point:
    X = M^{-1} B, then Y = M^{-1} X, dG/ds = -C Y.  On the imaginary axis
    dG/dw = j dG/ds."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    n = A.shape[0]
    out = np.empty((len(s), C.shape[0], B.shape[1]), dtype=np.complex128)
    Bc = B.astype(np.complex128)
    for k, sk in enumerate(s):
        M = sk * np.eye(n) - A
        X = np.linalg.solve(M, Bc)
        Y = np.linalg.solve(M, X)
        out[k] = -(C @ Y)
    return out


def _refined_solve_ld(M64, M_ld, rhs_ld, iters):
    X = np.linalg.solve(M64, rhs_ld.astype(np.complex128)).astype(np.clongdouble)
    for _ in range(iters):
        r = rhs_ld - M_ld @ X
        X = X + np.linalg.solve(M64, r.astype(np.complex128)).astype(np.clongdouble)
    return X


def derivative_at_extended(A, B, C, D, s, iters: int = 3) -> np.ndarray:
    """``derivative_at`` with both solves refined in extended precision (the
    residual and iterate in x87 clongdouble, as in ``freqresp_extended``)."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    n = A.shape[0]
    ld = np.clongdouble
    A_ld, B_ld, C_ld = A.astype(ld), B.astype(ld), C.astype(ld)
    out = np.empty((len(s), C.shape[0], B.shape[1]), dtype=np.complex128)
    for k, sk in enumerate(s):
        M64 = sk * np.eye(n) - A
        s_ld = np.longdouble(sk.real) + 1j * np.longdouble(sk.imag)
        M_ld = s_ld * np.eye(n, dtype=ld) - A_ld
        X = _refined_solve_ld(M64, M_ld, B_ld, iters)
        Y = _refined_solve_ld(M64, M_ld, X, iters)
        out[k] = (-(C_ld @ Y)).astype(np.complex128)
    return out


def cond2(A, omega) -> np.ndarray:
    """kappa_2(jw I - A) = sigma_max / sigma_min per frequency (SVD)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    out = np.empty(len(omega))
    for k, w in enumerate(omega):
        s = np.linalg.svd(1j * w * np.eye(n) - A, compute_uv=False)
        out[k] = np.inf if s[-1] == 0 else s[0] / s[-1]
    return out


def rel_err(G, G_ref, floor: float = 1e-300) -> np.ndarray:
    """err_k = ||G_k - G_ref,k||_F / max(||G_ref,k||_F, floor), shape (K,)."""
    G = np.asarray(G)
    G_ref = np.asarray(G_ref)
    K = G_ref.shape[0]
    num = np.linalg.norm((G - G_ref).reshape(K, -1).astype(np.complex128), axis=1)
    den = np.linalg.norm(G_ref.reshape(K, -1).astype(np.complex128), axis=1)
    return num / np.maximum(den, floor)


def rel_err_max(G, G_ref) -> float:
    e = rel_err(G, G_ref)
    return float(e.max()) if e.size else 0.0


def freqresp_descriptor(A, B, C, D, E, s) -> np.ndarray:
    """G(s_k) = C (s_k E - A)^{-1} B + D for a descriptor system
    E x' = A x + B u, y = C x + D u (E may be singular: a differential-
    algebraic system; G is then defined wherever s E - A is nonsingular, and
    may be improper).  Any text on descriptor systems, e.g. Dai, *Singular
    Control Systems* (1989), ch. 1.  One dense LU with partial pivoting per
    point, shape (K, p, m)."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    E = np.asarray(E, dtype=np.float64)
    if E.shape != A.shape:
        raise ValueError("E must be n x n")
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    G = np.empty((len(s), C.shape[0], B.shape[1]), dtype=np.complex128)
    Bc = B.astype(np.complex128)
    for k, sk in enumerate(s):
        X = np.linalg.solve(sk * E - A, Bc)
        G[k] = C @ X + D
    return G


def freqresp_descriptor_extended(A, B, C, D, E, s, iters: int = 3) -> np.ndarray:
    """``freqresp_descriptor`` followed by the extended-precision refinement
    of ``freqresp_extended``: residual B - (s E - A) X and iterate in x87
    extended precision, corrections from the float64 LU."""
    A, B, C, D, _ = _check(A, B, C, D, [0.0])
    E = np.asarray(E, dtype=np.float64)
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    ld = np.clongdouble
    A_ld, B_ld, C_ld, D_ld, E_ld = A.astype(ld), B.astype(ld), C.astype(ld), D.astype(ld), E.astype(ld)
    out = np.empty((len(s), C.shape[0], B.shape[1]), dtype=np.complex128)
    for k, sk in enumerate(s):
        M64 = sk * E - A
        s_ld = np.longdouble(sk.real) + 1j * np.longdouble(sk.imag)
        M_ld = s_ld * E_ld - A_ld
        X = np.linalg.solve(M64, B.astype(np.complex128)).astype(ld)
        for _ in range(iters):
            r = B_ld - M_ld @ X
            X = X + np.linalg.solve(M64, r.astype(np.complex128)).astype(ld)
        out[k] = (C_ld @ X + D_ld).astype(np.complex128)
    return out
