"""The seeded input generators: determinism, shapes and the pole structure."""
import numpy as np
import pytest

from paper_2401_04068_amd import workloads as wl


def test_siso8_shape_and_determinism():
    a = wl.siso8()
    b = wl.siso8()
    assert (a.n, a.m, a.p, a.K) == (8, 1, 1, 200)
    for x, y in [(a.A, b.A), (a.B, b.B), (a.C, b.C), (a.D, b.D), (a.omega, b.omega)]:
        assert np.array_equal(x, y)
    assert a.omega[0] == pytest.approx(1e-2) and a.omega[-1] == pytest.approx(1e2)
    # 4 real poles and 2 pairs
    assert np.sum(a.poles.imag == 0) == 4


def test_mimo64_pole_structure():
    mdl = wl.mimo64()
    assert (mdl.n, mdl.m, mdl.p, mdl.K) == (64, 4, 4, 2000)
    ev = np.sort_complex(np.linalg.eigvals(mdl.A))
    assert np.max(np.abs(ev - np.sort_complex(mdl.poles))) < 1e-12
    real = mdl.poles[mdl.poles.imag == 0].real
    assert np.all((real <= -0.1) & (real >= -2.0))
    cplx = mdl.poles[mdl.poles.imag != 0]
    assert np.all((cplx.real <= -0.05) & (cplx.real >= -1.0))
    assert np.all((np.abs(cplx.imag) >= 0.5) & (np.abs(cplx.imag) <= 10.0))
    # A is normal by construction
    A = mdl.A
    assert np.linalg.norm(A @ A.T - A.T @ A) < 1e-13 * np.linalg.norm(A) ** 2
    # Q is orthogonal
    assert np.linalg.norm(mdl.Q.T @ mdl.Q - np.eye(64)) < 1e-13


def test_serving_requests_ranges():
    reqs = wl.serving_requests(64)
    for r in reqs:
        assert 4 <= r.n <= 128 and 1 <= r.m <= 8 and 1 <= r.p <= 8
        assert 256 <= r.K <= 4096
        assert r.omega[0] == pytest.approx(1e-3) and r.omega[-1] == pytest.approx(1e3)
    again = wl.serving_request(17)
    assert np.array_equal(again.A, reqs[17].A)
    t = wl.serving_arrivals()
    assert len(t) == 4096 and np.all(np.diff(t) > 0)
    # mean rate about 2000 req/s
    assert 1700 < len(t) / t[-1] < 2300


def test_damped256_model():
    mdl = wl.damped256_model(3)
    assert (mdl.n, mdl.m, mdl.p, mdl.K) == (256, 4, 4, 4096)
    assert np.all(mdl.poles.imag != 0)
    wn = np.abs(mdl.poles)
    zeta = -mdl.poles.real / wn
    assert np.all((zeta >= 1e-5 * 0.999) & (zeta <= 1e-2 * 1.001))
    assert np.all((wn >= 1.0) & (wn <= 100.0))
    wd = np.abs(mdl.poles.imag)
    clustered = mdl.omega[3072:]
    rel = np.min(np.abs(clustered[:, None] / wd[None, :] - 1.0), axis=1)
    assert np.all(rel <= 0.01 + 1e-12)


def test_large1024_queries_repeat_shifted():
    models = wl.large1024_models(n=32, m=2, p=2, K=100)
    q = wl.large1024_queries(models)
    assert len(q) == 10
    assert q[8][0] == 0 and q[9][0] == 3
    w0 = models[0].omega
    ratio = q[8][1] / w0
    assert np.allclose(ratio, ratio[0]) and ratio[0] > 1.0
