"""Resonance peaks and H-infinity norm by brute force (oracle, test only).

sigma(w) = sigma_max(G(j w)) (numpy.linalg.svd of the oracle's G) on a dense
logarithmic grid; every interior local maximum of the grid is then refined
by golden-section search on sigma alone (Kiefer 1953), inside the bracket of
its two grid neighbours.  ||G||_inf = sup_w sigma(w) is estimated as the
largest of the refined maxima, the grid values and sigma_max(D) (w -> inf)
(e.g. Zhou, Doyle & Glover, Robust and Optimal Control, 1996, ch. 4).
Derivative-free on purpose: the library refines with derivatives.
"""
from __future__ import annotations

import numpy as np

from .freqresp import freqresp

__all__ = ["sigma_max", "peaks_bruteforce"]

_GOLD = (np.sqrt(5.0) - 1.0) / 2.0


def sigma_max(A, B, C, D, omega) -> np.ndarray:
    G = freqresp(A, B, C, D, omega)
    return np.linalg.svd(G, compute_uv=False)[:, 0]


def _golden(f, a, b, tol):
    c = b - _GOLD * (b - a)
    d = a + _GOLD * (b - a)
    fc, fd = f(c), f(d)
    while b - a > tol * max(abs(c), 1e-300):
        if fc >= fd:
            b, d, fd = d, c, fc
            c = b - _GOLD * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + _GOLD * (b - a)
            fd = f(d)
    return (c, fc) if fc >= fd else (d, fd)


def peaks_bruteforce(A, B, C, D, lo: float, hi: float, n: int = 4000, max_peaks: int = 8, tol: float = 1e-12):
    """Returns (hinf, w_hinf, [(w, gain), ...] largest first)."""
    w = np.logspace(np.log10(lo), np.log10(hi), n)
    s = sigma_max(A, B, C, D, w)
    f = lambda x: float(sigma_max(A, B, C, D, [x])[0])  # noqa: E731
    loc = [k for k in range(1, n - 1) if s[k] >= s[k - 1] and s[k] >= s[k + 1]]
    loc = sorted(loc, key=lambda k: -s[k])[:max_peaks]
    peaks = sorted((_golden(f, w[k - 1], w[k + 1], tol) for k in loc), key=lambda t: -t[1])
    cands = [(float(s.max()), float(w[int(s.argmax())]))]
    cands += [(g, x) for x, g in peaks]
    if D is not None:
        cands.append((float(np.linalg.svd(np.asarray(D, dtype=float), compute_uv=False)[0]), np.inf))
    hinf, wh = max(cands)
    return hinf, wh, peaks
