"""Exact rational frequency response for tiny systems (oracle, test only).

With A, B, C, D rational and w rational, every entry of
G(jw) = C (jw I - A)^{-1} B + D lies in Q(j).  This module carries complex
rationals as pairs of ``fractions.Fraction`` and solves M X = B by Gaussian
elimination over Q(j) (any pivot that is exactly nonzero is admissible, since
there is no rounding).  It is brute force, meant for n <= 4.
"""
from __future__ import annotations

from fractions import Fraction

__all__ = ["QJ", "freqresp_exact", "derivative_exact", "to_complex"]


class QJ:
    """a + j b with a, b rational."""

    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    def __add__(self, o):
        o = _lift(o)
        return QJ(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _lift(o)
        return QJ(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _lift(o) - self

    def __neg__(self):
        return QJ(-self.re, -self.im)

    def __mul__(self, o):
        o = _lift(o)
        return QJ(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = _lift(o)
        den = o.re * o.re + o.im * o.im
        if den == 0:
            raise ZeroDivisionError("division by exact zero in Q(j)")
        num = self * QJ(o.re, -o.im)
        return QJ(num.re / den, num.im / den)

    def is_zero(self) -> bool:
        return self.re == 0 and self.im == 0

    def __eq__(self, o):
        o = _lift(o)
        return self.re == o.re and self.im == o.im

    def __repr__(self):
        return f"QJ({self.re}, {self.im})"


def _lift(x) -> QJ:
    if isinstance(x, QJ):
        return x
    if isinstance(x, complex):
        return QJ(Fraction(x.real), Fraction(x.imag))
    return QJ(Fraction(x), 0)


def to_complex(z: QJ) -> complex:
    return complex(float(z.re), float(z.im))


def _solve(M, Bcols):
    """Gauss-Jordan over Q(j); M is n x n (lists of QJ), Bcols n x m."""
    n = len(M)
    m = len(Bcols[0])
    aug = [list(M[i]) + list(Bcols[i]) for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if not aug[r][col].is_zero()), None)
        if piv is None:
            raise ZeroDivisionError("jw I - A is exactly singular")
        aug[col], aug[piv] = aug[piv], aug[col]
        inv = QJ(1) / aug[col][col]
        aug[col] = [v * inv for v in aug[col]]
        for r in range(n):
            if r != col and not aug[r][col].is_zero():
                f = aug[r][col]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[col])]
    return [[aug[i][n + j] for j in range(m)] for i in range(n)]


def freqresp_exact(A, B, C, D, w, sigma=0, E=None):
    """Exact G(s) = C (s E - A)^{-1} B + D for rational inputs at the point
    s = sigma + j w (sigma = 0: the frequency response at w); E = None means
    the identity (a standard state-space model).

    A, E: n x n, B: n x m, C: p x n, D: p x m (nested sequences of ints,
    Fractions or floats -- floats are taken at their exact binary value),
    w, sigma: rational.  Returns a p x m nested list of QJ.
    """
    n = len(A)
    m = len(B[0])
    p = len(C)
    w = Fraction(w)
    sigma = Fraction(sigma)
    if E is None:
        E = [[1 if i == k else 0 for k in range(n)] for i in range(n)]
    M = [[QJ(sigma * Fraction(E[i][k]) - Fraction(A[i][k]), w * Fraction(E[i][k])) for k in range(n)]
         for i in range(n)]
    Bq = [[QJ(Fraction(B[i][j])) for j in range(m)] for i in range(n)]
    X = _solve(M, Bq)
    G = []
    for i in range(p):
        row = []
        for j in range(m):
            acc = QJ(Fraction(D[i][j]))
            for k in range(n):
                acc = acc + X[k][j] * Fraction(C[i][k])
            row.append(acc)
        G.append(row)
    return G


def derivative_exact(A, B, C, D, w, sigma=0):
    """Exact dG/ds = -C (s I - A)^{-2} B at s = sigma + j w (rational inputs):
    two exact solves over Q(j).  Returns a p x m nested list of QJ."""
    n = len(A)
    m = len(B[0])
    p = len(C)
    w = Fraction(w)
    sigma = Fraction(sigma)
    M = [[QJ(sigma - Fraction(A[i][k]) if i == k else -Fraction(A[i][k]), w if i == k else 0) for k in range(n)]
         for i in range(n)]
    Bq = [[QJ(Fraction(B[i][j])) for j in range(m)] for i in range(n)]
    Y = _solve(M, _solve(M, Bq))
    out = []
    for i in range(p):
        row = []
        for j in range(m):
            acc = QJ(0)
            for k in range(n):
                acc = acc - Y[k][j] * Fraction(C[i][k])
            row.append(acc)
        out.append(row)
    return out
