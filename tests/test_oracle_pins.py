"""Pins for the CPU oracle: each checks it against something other than itself.

Every pin is chosen so that a plausible slip in the oracle fails at least one:
a wrong sign of jw (first-order imaginary part), a dropped D (first order with
d != 0, brute force), A used transposed (companion form, brute force with a
non-symmetric A), a wrong index or operand order (MIMO brute force,
superposition), a broken refinement (ill-conditioned exact cases).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact, hessenberg
from paper_2401_04068_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def _first_order(a, b, c, d):
    return (np.array([[-a]]), np.array([[b]]), np.array([[c]]), np.array([[d]]))


def _second_order(wn, zeta):
    A = np.array([[0.0, 1.0], [-wn * wn, -2.0 * zeta * wn]])
    B = np.array([[0.0], [1.0]])
    C = np.array([[wn * wn, 0.0]])
    D = np.zeros((1, 1))
    return A, B, C, D


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, *vals = line.split()
            rows.append((kind, [float(v) for v in vals]))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}-{r[1]}")
def test_golden_closed_forms(row):
    kind, (x1, x2, c, d, w, re, im) = row
    sys_ = _first_order(x1, x2, c, d) if kind == "first" else _second_order(x1, x2)
    G = oracle.freqresp(*sys_, [w])[0, 0, 0]
    ref = complex(re, im)
    assert abs(G - ref) <= 1e-14 * max(abs(ref), 1e-300) + 1e-300, (G, ref)


def test_first_order_closed_form_grid():
    a, b, c, d = 0.7, -1.3, 2.1, 0.4
    w = np.concatenate([-np.logspace(-3, 3, 50), [0.0], np.logspace(-3, 3, 50)])
    G = oracle.freqresp(*_first_order(a, b, c, d), w)[:, 0, 0]
    ref = c * b * (a - 1j * w) / (a * a + w * w) + d
    assert np.max(np.abs(G - ref) / np.abs(ref)) < 1e-14


def test_second_order_textbook():
    for wn, zeta in [(1.0, 0.1), (7.0, 1e-3), (50.0, 0.7)]:
        w = np.logspace(-2, 3, 80) * wn / 10
        G = oracle.freqresp(*_second_order(wn, zeta), w)[:, 0, 0]
        ref = wn * wn / (wn * wn - w * w + 2j * zeta * wn * w)
        assert np.max(np.abs(G - ref) / np.abs(ref)) < 1e-12
        g = oracle.freqresp(*_second_order(wn, zeta), [wn])[0, 0, 0]
        assert abs(abs(g) - 1.0 / (2.0 * zeta)) <= 1e-12 / zeta
        assert abs(np.angle(g, deg=True) + 90.0) < 1e-9


def _rand_small_int_system(rng, n, m, p):
    A = rng.integers(-4, 5, (n, n)).astype(float)
    B = rng.integers(-3, 4, (n, m)).astype(float)
    C = rng.integers(-3, 4, (p, n)).astype(float)
    D = rng.integers(-2, 3, (p, m)).astype(float)
    return A, B, C, D


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_exact_rational(seed):
    rng = np.random.default_rng(100 + seed)
    n = 1 + seed % 4
    m = 1 + (seed % 3)
    p = 1 + ((seed + 1) % 3)
    A, B, C, D = _rand_small_int_system(rng, n, m, p)
    for w in [Fraction(0), Fraction(3, 8), Fraction(-5, 4), Fraction(7, 2), Fraction(33, 16)]:
        try:
            Gx = exact.freqresp_exact(A.tolist(), B.tolist(), C.tolist(), D.tolist(), w)
        except ZeroDivisionError:
            continue
        Gref = np.array([[exact.to_complex(z) for z in row] for row in Gx])
        G = oracle.freqresp(A, B, C, D, [float(w)])[0]
        kappa = oracle.cond2(A, [float(w)])[0]
        err = np.linalg.norm(G - Gref) / max(np.linalg.norm(Gref), 1e-300)
        assert err <= 1e-15 * max(kappa, 1.0) * 10, (seed, w, err, kappa)


def test_brute_force_catches_transpose():
    """Sanity of the pin itself: A^T in place of A gives a different answer."""
    rng = np.random.default_rng(7)
    A, B, C, D = _rand_small_int_system(rng, 3, 2, 2)
    w = Fraction(1, 2)
    Gx = exact.freqresp_exact(A.T.tolist(), B.tolist(), C.tolist(), D.tolist(), w)
    Gwrong = np.array([[exact.to_complex(z) for z in row] for row in Gx])
    G = oracle.freqresp(A, B, C, D, [0.5])[0]
    assert np.linalg.norm(G - Gwrong) > 1e-3 * np.linalg.norm(G)


def test_conjugate_symmetry():
    mdl = wl.mimo64(K=64)
    G = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    Gm = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, -mdl.omega)
    assert np.max(oracle.rel_err(Gm, np.conj(G))) < 1e-13


def test_dc_gain():
    mdl = wl.mimo64(K=4)
    G0 = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, [0.0])[0]
    dc = mdl.D - mdl.C @ np.linalg.solve(mdl.A, mdl.B)
    assert np.max(np.abs(G0.imag)) == 0.0 or np.max(np.abs(G0.imag)) < 1e-14 * np.abs(dc).max()
    assert np.linalg.norm(G0.real - dc) / np.linalg.norm(dc) < 1e-13


def test_similarity_invariance():
    mdl = wl.siso8()
    rng = np.random.default_rng(11)
    n = mdl.n
    # T with kappa(T) about 10: orthogonal times a graded diagonal
    U = wl.haar_orthogonal(rng, n)
    T = U @ np.diag(np.logspace(0, 1, n))
    Ti = np.linalg.inv(T)
    G1 = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    G2 = oracle.freqresp(T @ mdl.A @ Ti, T @ mdl.B, mdl.C @ Ti, mdl.D, mdl.omega)
    kappa = oracle.cond2(mdl.A, mdl.omega).max()
    assert np.max(oracle.rel_err(G2, G1)) < 10 * kappa * 1e-15 * 10


def _modal_freqresp(mdl, omega):
    """D + (C Q)(jw I - Lambda)^{-1}(Q^T B) with closed-form block inverses:
    scalar blocks 1/(jw - lam); 2x2 blocks [[x, y], [-y, x]] with
    x = jw - sigma, y = -omega_d have inverse [[x, -y], [y, x]] / (x^2 + y^2)."""
    Lam = mdl.Lam
    n = mdl.n
    CQ = mdl.C @ mdl.Q
    QB = mdl.Q.T @ mdl.B
    out = np.empty((len(omega), mdl.p, mdl.m), dtype=complex)
    for k, w in enumerate(omega):
        Y = np.zeros((n, mdl.m), dtype=complex)
        i = 0
        while i < n:
            if i + 1 < n and Lam[i, i + 1] != 0.0:
                x = 1j * w - Lam[i, i]
                y = -Lam[i, i + 1]
                det = x * x + y * y
                Y[i] = (x * QB[i] - y * QB[i + 1]) / det
                Y[i + 1] = (y * QB[i] + x * QB[i + 1]) / det
                i += 2
            else:
                Y[i] = QB[i] / (1j * w - Lam[i, i])
                i += 1
        out[k] = CQ @ Y + mdl.D
    return out


@pytest.mark.parametrize("which", ["siso8", "mimo64"])
def test_modal_form(which):
    mdl = wl.siso8() if which == "siso8" else wl.mimo64(K=200)
    G = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    Gm = _modal_freqresp(mdl, mdl.omega)
    assert np.max(oracle.rel_err(G, Gm)) < 1e-12


def test_high_frequency_asymptote():
    mdl = wl.mimo64(K=4)
    normA = np.linalg.norm(mdl.A, 2)
    for w in [1e6, 1e8]:
        G = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, [w])[0]
        approx = mdl.C @ mdl.B / (1j * w)
        rel = np.linalg.norm((G - mdl.D) - approx) / np.linalg.norm(approx)
        assert rel < 3 * normA / w


def test_mimo_superposition():
    mdl = wl.mimo64(K=50)
    G = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    for j in range(mdl.m):
        Gj = oracle.freqresp(mdl.A, mdl.B[:, j:j + 1], mdl.C, mdl.D[:, j:j + 1], mdl.omega)
        assert np.max(np.abs(Gj[:, :, 0] - G[:, :, j])) < 1e-13 * np.abs(G).max()


def test_cond2_normal_closed_form():
    mdl = wl.mimo64(K=100)
    kap = oracle.cond2(mdl.A, mdl.omega)
    d = np.abs(1j * mdl.omega[:, None] - mdl.poles[None, :])
    ref = d.max(axis=1) / d.min(axis=1)
    assert np.max(np.abs(kap - ref) / ref) < 1e-10


def _exact_matrix(A, B, C, D, w):
    Gx = exact.freqresp_exact(A.tolist(), B.tolist(), C.tolist(), D.tolist(), Fraction(w))
    return np.array([[exact.to_complex(z) for z in row] for row in Gx])


@pytest.mark.parametrize("case", ["rotation", "marginal"])
def test_extended_oracle_ill_conditioned(case):
    """Refinement with an extended-precision residual recovers the exact answer
    where kappa * u64 is large."""
    if case == "rotation":
        eps = 2.0 ** -24
        w0 = 1.5
        A = np.array([[-eps, w0, 0.0], [-w0, -eps, 1.0], [0.0, 0.0, -2.0]])
        w = w0
    else:
        A = np.array([[0.0, 3.0, 1.0], [-3.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
        w = 3.0 + 2.0 ** -22
    B = np.array([[1.0, 0.0], [0.5, -1.0], [2.0, 1.0]])
    C = np.array([[1.0, -2.0, 0.25], [0.0, 1.0, 3.0]])
    D = np.array([[0.5, 0.0], [-1.0, 2.0]])
    kappa = oracle.cond2(A, [w])[0]
    assert kappa > 1e6
    Gx = _exact_matrix(A, B, C, D, w)
    Ge = oracle.freqresp_extended(A, B, C, D, [w])[0]
    G64 = oracle.freqresp(A, B, C, D, [w])[0]
    e_ext = np.linalg.norm(Ge - Gx) / np.linalg.norm(Gx)
    e_64 = np.linalg.norm(G64 - Gx) / np.linalg.norm(Gx)
    # limiting accuracy of refinement with an extended residual: about
    # kappa * u_ext (Higham, ch. 12); the plain float64 solve sits near kappa * u64
    u_ext = float(np.finfo(np.longdouble).eps)
    assert u_ext < 2e-19
    assert e_ext < kappa * u_ext + 4e-16, (e_ext, e_64, kappa)
    assert e_ext < e_64 / 100, (e_ext, e_64)
    assert e_64 < 1e-15 * kappa * 10


def test_extended_matches_plain_when_well_conditioned():
    mdl = wl.siso8()
    Ge = oracle.freqresp_extended(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega[::10])
    G = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega[::10])
    assert np.max(oracle.rel_err(G, Ge)) < 1e-14


def test_rel_err_metric():
    G = np.ones((3, 2, 2), dtype=complex)
    H = G.copy()
    H[1, 0, 0] += 1e-3j
    e = oracle.rel_err(H, G)
    assert e[0] == 0 and e[2] == 0
    assert abs(e[1] - 1e-3 / 2.0) < 1e-15


# ------------------------------------------------------------ Hessenberg oracle

@pytest.mark.parametrize("n", [3, 8, 33, 64])
def test_hessenberg_invariants(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, 3))
    C = rng.standard_normal((2, n))
    H, Bt, Ct, Q = hessenberg.hessenberg(A, B, C, want_q=True)
    u = np.finfo(float).eps
    assert np.all(H[np.tril_indices(n, -2)] == 0.0)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 10 * n * u
    assert np.linalg.norm(A @ Q - Q @ H) / np.linalg.norm(A) < 10 * n * u
    assert np.allclose(Q[:, 0], np.eye(n)[:, 0])
    assert np.linalg.norm(Bt - Q.T @ B) < 10 * n * u * np.linalg.norm(B)
    assert np.linalg.norm(Ct - C @ Q) < 10 * n * u * np.linalg.norm(C)


@pytest.mark.parametrize("n", [5, 16, 64])
def test_hessenberg_matches_lapack(n):
    """Implicit-Q theorem: same H up to a diagonal +-1 similarity."""
    import scipy.linalg

    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n))
    H, _, _ = hessenberg.hessenberg(A)
    Hl = scipy.linalg.hessenberg(A)
    Hn, _, _ = hessenberg.normalize_signs(H)
    Hln, _, _ = hessenberg.normalize_signs(Hl)
    assert np.max(np.abs(Hn - Hln)) < 1e-12 * np.abs(A).max() * n


def test_hessenberg_preserves_transfer_function():
    mdl = wl.mimo64(K=100)
    H, Bt, Ct = hessenberg.hessenberg(mdl.A, mdl.B, mdl.C)
    G1 = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    G2 = oracle.freqresp(H, Bt, Ct, mdl.D, mdl.omega)
    assert np.max(oracle.rel_err(G2, G1)) < 1e-12
    ev = np.sort_complex(np.linalg.eigvals(H))
    assert np.max(np.abs(ev - np.sort_complex(mdl.poles))) < 1e-11


# ---------------------------------------------------------------- complex points

GOLDEN_S = os.path.join(os.path.dirname(__file__), "golden", "closed_forms_s.txt")


def _golden_s_rows():
    rows = []
    with open(GOLDEN_S) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, *vals = line.split()
            rows.append((kind, [float(v) for v in vals]))
    return rows


@pytest.mark.parametrize("row", _golden_s_rows(), ids=lambda r: f"{r[0]}-{r[1]}")
def test_golden_closed_forms_complex_points(row):
    """Hand-derived first-order values at s off the imaginary axis
    (continuous time) and at z = exp(j theta) (discrete time)."""
    kind, (a, b, c, d, x, y, re, im) = row
    if kind == "cs":
        sys_ = (np.array([[-a]]), np.array([[b]]), np.array([[c]]), np.array([[d]]))
        s = complex(x, y)
    else:
        sys_ = (np.array([[a]]), np.array([[b]]), np.array([[c]]), np.array([[d]]))
        s = np.exp(1j * x)
    ref = complex(re, im)
    for fn in (oracle.freqresp_at, oracle.freqresp_at_extended):
        G = fn(*sys_, [s])[0, 0, 0]
        assert abs(G - ref) <= 1e-14 * abs(ref), (fn.__name__, G, ref)


@pytest.mark.parametrize("seed", range(6))
def test_complex_points_exact_rational(seed):
    """Brute force over Q(j) at rational s = sigma + j w: a dropped or
    sign-flipped real part of s, or a transposed A, fails this."""
    rng = np.random.default_rng(300 + seed)
    n = 1 + seed % 4
    m, p = 1 + seed % 2, 1 + (seed + 1) % 3
    A, B, C, D = _rand_small_int_system(rng, n, m, p)
    for sig, w in [(Fraction(1, 2), Fraction(3, 8)), (Fraction(-7, 4), Fraction(-5, 4)), (Fraction(9, 2), Fraction(0)),
                   (Fraction(-1, 8), Fraction(33, 16))]:
        try:
            Gx = exact.freqresp_exact(A.tolist(), B.tolist(), C.tolist(), D.tolist(), w, sigma=sig)
        except ZeroDivisionError:
            continue
        Gref = np.array([[exact.to_complex(z) for z in row] for row in Gx])
        s = complex(float(sig), float(w))
        M = s * np.eye(n) - A
        kappa = np.linalg.cond(M)
        for fn, u in ((oracle.freqresp_at, 1e-15), (oracle.freqresp_at_extended, 1e-18)):
            G = fn(A, B, C, D, [s])[0]
            err = np.linalg.norm(G - Gref) / max(np.linalg.norm(Gref), 1e-300)
            assert err <= max(u * kappa * 10, 1e-15), (fn.__name__, seed, s, err, kappa)


def test_discrete_time_impulse_response_series():
    """For |z| > rho(A): G(z) = D + sum_k C A^k B z^-(k+1) (the z-transform of
    the impulse response).  A stable discrete model (rho(A) = 0.8), on the
    unit circle, summed to 400 terms (0.8^400 ~ 1e-39)."""
    rng = np.random.default_rng(17)
    n, m, p = 6, 2, 3
    A = rng.standard_normal((n, n))
    A *= 0.8 / np.max(np.abs(np.linalg.eigvals(A)))
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    D = rng.standard_normal((p, m))
    theta = np.linspace(-np.pi, np.pi, 17)
    z = np.exp(1j * theta)
    G = oracle.freqresp_at(A, B, C, D, z)
    Ak_B = B.astype(np.complex128)
    series = np.broadcast_to(D.astype(np.complex128), (len(z), p, m)).copy()
    zinv = 1.0 / z
    zpow = zinv.copy()
    for _ in range(400):
        series += (C @ Ak_B)[None, :, :] * zpow[:, None, None]
        Ak_B = A @ Ak_B
        zpow = zpow * zinv
    assert np.max(oracle.rel_err(G, series)) < 1e-12


def test_complex_points_on_the_axis_agree_with_frequency_grid():
    """s = j w gives the frequency response (two separate code paths)."""
    mdl = wl.mimo64(K=40)
    G1 = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    G2 = oracle.freqresp_at(mdl.A, mdl.B, mdl.C, mdl.D, 1j * mdl.omega)
    assert np.max(oracle.rel_err(G2, G1)) < 1e-14


# ---------------------------------------------------------------- derivative

def test_derivative_closed_forms():
    """First order: d/ds [c b / (s + a) + d] = -c b / (s + a)^2.  Second order
    (companion form): d/ds [wn^2 / (s^2 + 2 zeta wn s + wn^2)] =
    -wn^2 (2 s + 2 zeta wn) / (s^2 + 2 zeta wn s + wn^2)^2."""
    a, b, c, d = 0.7, -1.3, 2.1, 0.4
    s = np.array([0.3j, -0.2 + 1.5j, 2.0 + 0j, -1.0 - 4.0j])
    dG = oracle.derivative_at(*_first_order(a, b, c, d), s)[:, 0, 0]
    ref = -c * b / (s + a) ** 2
    assert np.max(np.abs(dG - ref) / np.abs(ref)) < 1e-14
    for wn, zeta in [(1.0, 0.1), (7.0, 1e-3)]:
        s = 1j * wn * np.array([0.3, 0.999, 1.0, 2.0]) + 0.01
        dG = oracle.derivative_at(*_second_order(wn, zeta), s)[:, 0, 0]
        den = s * s + 2 * zeta * wn * s + wn * wn
        ref = -wn * wn * (2 * s + 2 * zeta * wn) / den ** 2
        assert np.max(np.abs(dG - ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_derivative_exact_rational(seed):
    rng = np.random.default_rng(500 + seed)
    n = 1 + seed % 4
    A, B, C, D = _rand_small_int_system(rng, n, 2, 2)
    for sig, w in [(Fraction(1, 2), Fraction(3, 8)), (Fraction(-7, 4), Fraction(5, 4)), (Fraction(0), Fraction(9, 4))]:
        try:
            Gx = exact.derivative_exact(A.tolist(), B.tolist(), C.tolist(), D.tolist(), w, sigma=sig)
        except ZeroDivisionError:
            continue
        ref = np.array([[exact.to_complex(z) for z in row] for row in Gx])
        s = complex(float(sig), float(w))
        kappa = np.linalg.cond(s * np.eye(n) - A)
        dG = oracle.derivative_at(A, B, C, D, [s])[0]
        assert np.linalg.norm(dG - ref) <= 1e-14 * kappa ** 2 * max(np.linalg.norm(ref), 1e-300), (seed, s)


def test_derivative_matches_central_difference():
    """(G(s + h) - G(s - h)) / 2h = dG/ds + O(h^2) along the imaginary axis."""
    mdl = wl.mimo64(K=16)
    s = 1j * mdl.omega
    h = 1e-5
    fd = (oracle.freqresp_at(mdl.A, mdl.B, mdl.C, mdl.D, s + 1j * h)
          - oracle.freqresp_at(mdl.A, mdl.B, mdl.C, mdl.D, s - 1j * h)) / (2j * h)
    dG = oracle.derivative_at(mdl.A, mdl.B, mdl.C, mdl.D, s)
    assert np.max(oracle.rel_err(fd, dG)) < 1e-6


def test_derivative_extended_exact_ill_conditioned():
    """Near an eigenvalue (kappa ~ 1e7) the extended derivative stays within
    kappa^2 u_ext of the exact rational value, where the float64 one cannot."""
    A = [[0, 1], [-1, Fraction(-2e-7)]]  # zeta = 1e-7, wn = 1 (the float's exact value)
    B = [[0], [1]]
    C = [[1, 0]]
    D = [[0]]
    w = Fraction(1)
    Gx = exact.derivative_exact(A, B, C, D, w)
    ref = exact.to_complex(Gx[0][0])
    Af = np.array([[0.0, 1.0], [-1.0, -2e-7]])
    dG = oracle.derivative_at_extended(Af, np.array(B, float), np.array(C, float), np.zeros((1, 1)), [1j])[0, 0, 0]
    assert abs(dG - ref) <= 1e-8 * abs(ref), (dG, ref)


# ---------------------------------------------------------------- peaks

@pytest.mark.parametrize("wn,zeta", [(1.0, 0.05), (7.0, 1e-3), (30.0, 0.3)])
def test_peak_bruteforce_second_order_closed_form(wn, zeta):
    """|wn^2 / (wn^2 - w^2 + 2 j zeta wn w)| peaks at w_r = wn sqrt(1 - 2 zeta^2)
    with value 1 / (2 zeta sqrt(1 - zeta^2)) (zeta < 1/sqrt 2)."""
    from oracle import peaks

    hinf, wh, pk = peaks.peaks_bruteforce(*_second_order(wn, zeta), wn / 100, wn * 100, n=2000)
    wr = wn * np.sqrt(1 - 2 * zeta * zeta)
    gr = 1.0 / (2 * zeta * np.sqrt(1 - zeta * zeta))
    assert abs(pk[0][0] - wr) <= 1e-6 * wr
    assert abs(pk[0][1] - gr) <= 1e-12 * gr
    assert abs(hinf - gr) <= 1e-12 * gr


def test_peak_bruteforce_monotone_first_order():
    """c b / (jw + a) + d decreases in |.| when d = 0: sup at w -> 0, no
    interior peak."""
    from oracle import peaks

    hinf, wh, pk = peaks.peaks_bruteforce(*_first_order(2.0, 1.0, 3.0, 0.0), 1e-4, 1e4, n=500)
    assert pk == []
    assert abs(hinf - 1.5) <= 1e-8 * 1.5


# ---------------------------------------------------------------- descriptor systems

GOLDEN_E = os.path.join(os.path.dirname(__file__), "golden", "closed_forms_descriptor.txt")


def _golden_e_rows():
    rows = []
    with open(GOLDEN_E) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, *vals = line.split()
            rows.append((kind, [float(v) for v in vals]))
    return rows


def _descriptor_case(kind, a, e, b, c, d):
    if kind == "e1":
        return np.array([[-a]]), np.array([[b]]), np.array([[c]]), np.array([[d]]), np.array([[e]])
    if kind == "alg":
        return (np.array([[-a, 0.0], [0.0, 1.0]]), np.array([[1.0], [-1.0]]), np.array([[1.0, 1.0]]),
                np.array([[d]]), np.diag([1.0, 0.0]))
    return (np.eye(2), np.array([[0.0], [1.0]]), np.array([[1.0, 0.0]]), np.array([[d]]),
            np.array([[0.0, 1.0], [0.0, 0.0]]))


@pytest.mark.parametrize("row", _golden_e_rows(), ids=lambda r: f"{r[0]}-{r[1]}")
def test_golden_descriptor_closed_forms(row):
    """Hand-derived values: first order with e != 1, a differential-algebraic
    system (singular E: the algebraic state adds a constant), and a nilpotent
    E (G(s) = -s + d, improper)."""
    kind, (a, e, b, c, d, sr, si, re, im) = row
    sys_ = _descriptor_case(kind, a, e, b, c, d)
    ref = complex(re, im)
    for fn in (oracle.freqresp_descriptor, oracle.freqresp_descriptor_extended):
        G = fn(*sys_, [complex(sr, si)])[0, 0, 0]
        assert abs(G - ref) <= 1e-14 * max(abs(ref), 1.0), (fn.__name__, G, ref)


def test_descriptor_identity_E_is_the_standard_system():
    rng = np.random.default_rng(81)
    n, m, p = 9, 2, 3
    A = rng.standard_normal((n, n)) - 3 * np.eye(n)
    B, C, D = rng.standard_normal((n, m)), rng.standard_normal((p, n)), rng.standard_normal((p, m))
    s = np.array([0.3j, 1 + 2j, -0.5 + 0.1j, 7j])
    np.testing.assert_allclose(oracle.freqresp_descriptor(A, B, C, D, np.eye(n), s),
                               oracle.freqresp_at(A, B, C, D, s), rtol=0, atol=1e-13)


def test_descriptor_invertible_E_equals_E_inverse_system_and_equivalence():
    """E invertible: G = C (s I - E^-1 A)^-1 E^-1 B + D.  Restricted system
    equivalence (P E R, P A R, P B, C R, D) with invertible P, R leaves G
    unchanged."""
    rng = np.random.default_rng(82)
    n, m, p = 7, 2, 2
    A = rng.standard_normal((n, n)) - 2 * np.eye(n)
    E = rng.standard_normal((n, n)) + 3 * np.eye(n)
    B, C, D = rng.standard_normal((n, m)), rng.standard_normal((p, n)), rng.standard_normal((p, m))
    s = np.array([0.2j, 2 + 1j, 5j])
    G = oracle.freqresp_descriptor(A, B, C, D, E, s)
    Ei = np.linalg.inv(E)
    np.testing.assert_allclose(G, oracle.freqresp_at(Ei @ A, Ei @ B, C, D, s), rtol=1e-11, atol=1e-11)
    P = rng.standard_normal((n, n)) + 2 * np.eye(n)
    R = rng.standard_normal((n, n)) + 2 * np.eye(n)
    G2 = oracle.freqresp_descriptor(P @ A @ R, P @ B, C @ R, D, P @ E @ R, s)
    np.testing.assert_allclose(G2, G, rtol=1e-10, atol=1e-10)


def test_descriptor_exact_rational_agreement():
    """Random small integer systems with a singular E against exact
    arithmetic over Q(j)."""
    rng = np.random.default_rng(83)
    for trial in range(12):
        n, m, p = int(rng.integers(2, 5)), int(rng.integers(1, 3)), int(rng.integers(1, 3))
        A = rng.integers(-4, 5, (n, n)).astype(float)
        E = rng.integers(-2, 3, (n, n)).astype(float)
        E[-1] = 0.0  # singular E
        B = rng.integers(-3, 4, (n, m)).astype(float)
        C = rng.integers(-3, 4, (p, n)).astype(float)
        D = rng.integers(-2, 3, (p, m)).astype(float)
        w = float(rng.integers(1, 9)) / 4
        sig = float(rng.integers(-3, 4)) / 2
        try:
            ex = exact.freqresp_exact(A.tolist(), B.tolist(), C.tolist(), D.tolist(), w, sig, E=E.tolist())
        except ZeroDivisionError:
            continue
        ref = np.array([[exact.to_complex(z) for z in row] for row in ex])
        G = oracle.freqresp_descriptor(A, B, C, D, E, [complex(sig, w)])[0]
        assert np.max(np.abs(G - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), (trial, G, ref)
