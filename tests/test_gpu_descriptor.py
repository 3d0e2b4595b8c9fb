"""GPU: descriptor systems G(s) = C (s E - A)^{-1} B + D through the
Hessenberg-triangular reduction and the s T - H sweep, against the oracle
(dense LU of s E - A per point) and hand-derived closed forms.

Tolerance: 1e-10 relative Frobenius error per point (the float64 path's
bar); every model here has kappa(s E - A) <= ~1e3 on its grid, where a
backward-stable float64 solve is within ~kappa * n * u ~ 1e-11.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2401_04068_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def eng():
    from paper_2401_04068_amd import binding

    e = binding.Engine(arena_bytes=1 << 30)
    yield e
    e.close()


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "closed_forms_descriptor.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                kind, *vals = line.split()
                rows.append((kind, [float(v) for v in vals]))
    return rows


def _case(kind, a, e, b, c, d):
    if kind == "e1":
        return np.array([[-a]]), np.array([[b]]), np.array([[c]]), np.array([[d]]), np.array([[e]])
    if kind == "alg":
        return (np.array([[-a, 0.0], [0.0, 1.0]]), np.array([[1.0], [-1.0]]), np.array([[1.0, 1.0]]),
                np.array([[d]]), np.diag([1.0, 0.0]))
    return (np.eye(2), np.array([[0.0], [1.0]]), np.array([[1.0, 0.0]]), np.array([[d]]),
            np.array([[0.0, 1.0], [0.0, 0.0]]))


def test_closed_forms(eng):
    """First order with e != 1, a differential-algebraic system, and the
    nilpotent E whose G(s) = -s + d is improper (tests/golden)."""
    from paper_2401_04068_amd import binding

    for kind, (a, e, b, c, d, sr, si, re, im) in _golden():
        A, B, C, D, E = _case(kind, a, e, b, c, d)
        h = eng.submit(A, B, C, D, [complex(sr, si)], points=binding.POINTS_S, E=E)
        assert eng.poll(h, -1)
        ref = complex(re, im)
        assert abs(h.G[0, 0, 0] - ref) <= 1e-13 * max(1.0, abs(ref)), (kind, h.G[0, 0, 0], ref)
        assert h.info["path"][0] == binding.PATH_FP64


@pytest.mark.parametrize("n", [1, 2, 7, 31, 64, 65, 100, 128, 129, 200, 256])
def test_identity_E_equals_standard_path(eng, n):
    from paper_2401_04068_amd import binding

    rng = np.random.default_rng(9100 + n)
    mdl = wl.mixed_pole_model(rng, n, 3, 2, wl.logspace_grid(1e-2, 1e2, 150), 9100 + n)
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    h = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=np.eye(n))
    assert eng.poll(h, -1)
    assert oracle.rel_err(h.G, ref).max() <= TOL
    assert np.all(h.info["path"] == binding.PATH_FP64)


SHAPES = [(2, 1, 1, 1), (5, 2, 3, 1), (16, 1, 4, 0), (40, 4, 4, 6), (64, 3, 2, 8), (65, 2, 5, 9), (100, 6, 6, 10),
          (128, 8, 1, 16), (150, 2, 9, 0), (200, 4, 4, 20), (256, 3, 3, 32)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n{}m{}p{}alg{}".format(*s))
def test_random_descriptor_systems(eng, shape):
    """Well-conditioned pencils with n_alg algebraic states (singular E), on
    the imaginary axis and at complex points, including p < m (transposed
    system)."""
    from paper_2401_04068_amd import binding

    n, m, p, na = shape
    mdl = wl.descriptor_model(n, m, p, na, seed=9200 + n)
    print(f"case descriptor n={n} m={m} p={p} alg={na}", flush=True)
    ref = oracle.freqresp_descriptor(mdl.A, mdl.B, mdl.C, mdl.D, mdl.E, 1j * mdl.omega)
    h = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=mdl.E)
    assert eng.poll(h, -1)
    err = oracle.rel_err(h.G, ref)
    assert err.max() <= TOL, (err.max(), int(err.argmax()))
    s = np.array([0.5 + 1j, -0.3 + 0.2j, 2.0 + 0j, 0.1 + 30j])
    ref_s = oracle.freqresp_descriptor(mdl.A, mdl.B, mdl.C, mdl.D, mdl.E, s)
    h = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, s, points=binding.POINTS_S, E=mdl.E)
    assert eng.poll(h, -1)
    assert oracle.rel_err(h.G, ref_s).max() <= TOL


def test_refined_request_runs_float64_and_repeat_reuses(eng):
    from paper_2401_04068_amd import binding

    mdl = wl.descriptor_model(48, 3, 3, 5, seed=9301)
    ref = oracle.freqresp_descriptor(mdl.A, mdl.B, mdl.C, mdl.D, mdl.E, 1j * mdl.omega)
    h1 = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=mdl.E, precision=binding.PREC_REFINED,
                    model_key=77)
    assert eng.poll(h1, -1)
    assert np.all(h1.info["path"] == binding.PATH_FP64)
    assert oracle.rel_err(h1.G, ref).max() <= TOL
    h2 = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=mdl.E, model_key=77)
    assert eng.poll(h2, -1)
    assert h2.result["reduction_reused"] == 1
    np.testing.assert_array_equal(h2.G, h1.G)
    # the same key without E is another model
    h3 = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, model_key=77)
    assert eng.poll(h3, -1)
    assert h3.result["reduction_reused"] == 0


def test_descriptor_and_standard_requests_in_flight_together(eng):
    """Continuous batching across both kinds: each result equals the one
    computed alone."""
    mdls = [wl.descriptor_model(30 + 17 * i, 2, 3, i, seed=9400 + i) for i in range(4)]
    rng = np.random.default_rng(9410)
    std = [wl.mixed_pole_model(rng, 20 + 30 * i, 3, 2, wl.logspace_grid(1e-2, 1e2, 200), 9410 + i)
           for i in range(4)]
    alone = []
    for d in mdls:
        h = eng.submit(d.A, d.B, d.C, d.D, d.omega, E=d.E)
        assert eng.poll(h, -1)
        alone.append(h.G)
    hs = []
    for d, s_ in zip(mdls, std):
        hs.append(eng.submit(d.A, d.B, d.C, d.D, d.omega, E=d.E))
        hs.append(eng.submit(s_.A, s_.B, s_.C, s_.D, s_.omega))
    for h in hs:
        assert eng.poll(h, -1)
    for i, d in enumerate(mdls):
        np.testing.assert_array_equal(hs[2 * i].G, alone[i])
        s_ = std[i]
        assert oracle.rel_err(hs[2 * i + 1].G, oracle.freqresp(s_.A, s_.B, s_.C, s_.D, s_.omega)).max() <= TOL


def test_device_memory_descriptor_request(eng):
    import torch

    mdl = wl.descriptor_model(70, 2, 2, 7, seed=9501)
    ref = oracle.freqresp_descriptor(mdl.A, mdl.B, mdl.C, mdl.D, mdl.E, 1j * mdl.omega)
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(mdl, k))).to(dev) for k in ("A", "B", "C", "D", "E", "omega")}
    G = torch.empty(mdl.K * 2 * 2 * 2, dtype=torch.float64, device=dev)
    h = eng.submit_device(t["A"], t["B"], t["C"], t["D"], t["omega"], G, E=t["E"])
    assert eng.poll(h, -1)
    Gh = G.cpu().numpy().view(np.complex128).reshape(mdl.K, 2, 2)
    assert oracle.rel_err(Gh, ref).max() <= TOL


def test_descriptor_errors(eng):
    from paper_2401_04068_amd import binding

    mdl = wl.descriptor_model(8, 1, 1, 1, seed=9601)
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=mdl.E, want_derivative=True)
    assert ei.value.code == binding.LTI_EUNSUPPORTED
    E = mdl.E.copy()
    E[0, 0] = np.nan
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, E=E)
    assert ei.value.code == binding.LTI_EINVAL
    big = np.eye(300)
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(-big, np.ones((300, 1)), np.ones((1, 300)), None, [1.0], E=big)
    assert ei.value.code == binding.LTI_EUNSUPPORTED
