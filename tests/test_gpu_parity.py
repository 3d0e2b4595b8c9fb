"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (relative Frobenius error per frequency, see oracle.rel_err):
float64 path <= 1e-10, refined float32 path <= 1e-9; both are taken at
points where the float64 oracle itself is accurate to far better than that
(kappa(jwI - A) <= 1e3 here, so kappa * u64 <= 1e-13).
"""
import numpy as np
import pytest

import oracle
from oracle import hessenberg
from paper_2401_04068_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_REFINED = 1e-9


@pytest.fixture(scope="module")
def eng():
    from paper_2401_04068_amd import binding

    e = binding.Engine(arena_bytes=2 << 30)
    yield e
    e.close()


def _run(eng, mdl_or_tuple, precision, key=0, omega=None):
    from paper_2401_04068_amd import binding

    if isinstance(mdl_or_tuple, wl.Model):
        A, B, C, D, w = mdl_or_tuple.A, mdl_or_tuple.B, mdl_or_tuple.C, mdl_or_tuple.D, mdl_or_tuple.omega
    else:
        A, B, C, D, w = mdl_or_tuple
    if omega is not None:
        w = omega
    h = eng.submit(A, B, C, D, w, precision=precision, model_key=key)
    assert eng.poll(h, -1)
    assert h.result["status"] == binding.LTI_OK
    return h


def _prec(name):
    from paper_2401_04068_amd import binding

    return binding.PREC_FP64 if name == "fp64" else binding.PREC_REFINED


def _tol(name):
    return TOL_FP64 if name == "fp64" else TOL_REFINED


def test_siso8_fp64(eng):
    mdl = wl.siso8()
    print("case siso8 fp64", flush=True)
    h = _run(eng, mdl, _prec("fp64"))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    err = oracle.rel_err(h.G, ref)
    assert err.max() <= TOL_FP64, err.max()
    assert np.all(h.info["path"] == 0)


@pytest.mark.parametrize("prec", ["fp64", "refined"])
def test_mimo64_full_grid(eng, prec):
    """The 64-state, 4x4, 2000-point workload exactly as the benchmark runs it."""
    mdl = wl.mimo64()
    print(f"case mimo64 {prec}", flush=True)
    h = _run(eng, mdl, _prec(prec))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    err = oracle.rel_err(h.G, ref)
    assert err.max() <= _tol(prec), (err.max(), int(err.argmax()))
    if prec == "refined":
        assert np.all(h.info["path"] == 1)
        assert np.all(h.info["iters"] >= 2)
        # the stopping rule targets 1e-10; check it delivered that here
        assert err.max() <= 1e-10


@pytest.mark.parametrize("n,m,p", [(64, 4, 4), (100, 8, 8), (200, 3, 2), (300, 5, 4), (520, 16, 16)])
def test_reduced_model_matches_oracle(eng, n, m, p):
    """The reduced model of each reduction kernel (registers n <= 128, one
    workgroup n <= 256, blocked beyond) against the oracle's Householder
    reduction, after fixing the reflectors' signs (implicit-Q theorem)."""
    if (n, m, p) == (64, 4, 4):
        mdl = wl.mimo64(K=16)
    else:
        rng = np.random.default_rng(8100 + n)
        mdl = wl.mixed_pole_model(rng, n, m, p, wl.logspace_grid(1e-2, 1e2, 16))
    key = 0xA11CE + n
    print(f"case reduced n={n} m={m} p={p}", flush=True)
    _run(eng, mdl, _prec("fp64"), key=key)
    H, Bt, Ct = eng.get_reduced(key, n, m, p)
    if p < m:
        # reduced through the transposed system (A^T, C^T, B^T): H is the
        # transpose of that system's Hessenberg form
        assert np.all(np.triu(H, 2) == 0.0)
        Ho, Bo, Co = hessenberg.hessenberg(mdl.A.T, mdl.C.T, mdl.B.T)
        Hn, Cn_t, Bn_t = hessenberg.normalize_signs(H.T, Ct.T, Bt.T)
        Bn, Cn = Bn_t.T, Cn_t.T
        Hn = Hn.T
        Hon, Con_t, Bon_t = hessenberg.normalize_signs(Ho, Bo, Co)
        Hon, Bon, Con = Hon.T, Bon_t.T, Con_t.T
    else:
        assert np.all(np.tril(H, -2) == 0.0)
        Ho, Bo, Co = hessenberg.hessenberg(mdl.A, mdl.B, mdl.C)
        Hn, Bn, Cn = hessenberg.normalize_signs(H, Bt, Ct)
        Hon, Bon, Con = hessenberg.normalize_signs(Ho, Bo, Co)
    tol = 1e-12 * max(n, 64)
    assert np.abs(Hn - Hon).max() <= tol * np.abs(mdl.A).max()
    assert np.abs(Bn - Bon).max() <= tol * np.abs(mdl.B).max()
    assert np.abs(Cn - Con).max() <= tol * np.abs(mdl.C).max()
    G1 = oracle.freqresp(H, Bt, Ct, mdl.D, mdl.omega)
    G0 = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    assert oracle.rel_err(G1, G0).max() <= 1e-11


_SIZES = [1, 2, 3, 5, 31, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256]


@pytest.mark.parametrize("prec", ["fp64", "refined"])
@pytest.mark.parametrize("n", _SIZES)
def test_state_dimensions_and_ragged_tails(eng, n, prec):
    rng = np.random.default_rng(7000 + n)
    m, p = 2, 3
    w = np.concatenate([[0.0, -0.7], wl.logspace_grid(1e-2, 1e2, 35)])
    mdl = wl.mixed_pole_model(rng, n, m, p, w)
    print(f"case n={n} {prec}", flush=True)
    h = _run(eng, mdl, _prec(prec))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    err = oracle.rel_err(h.G, ref)
    assert err.max() <= _tol(prec), (n, err.max(), int(err.argmax()))


@pytest.mark.parametrize("mp", [(1, 8), (8, 1), (3, 5), (16, 16), (16, 3), (5, 16), (7, 7)])
@pytest.mark.parametrize("n", [40, 100])
def test_io_shapes(eng, n, mp):
    m, p = mp
    rng = np.random.default_rng(100 * m + p + n)
    mdl = wl.mixed_pole_model(rng, n, m, p, wl.logspace_grid(1e-3, 1e3, 50))
    print(f"case n={n} m={m} p={p}", flush=True)
    for prec in ("fp64", "refined"):
        h = _run(eng, mdl, _prec(prec))
        ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
        err = oracle.rel_err(h.G, ref)
        assert err.max() <= _tol(prec), (prec, err.max())


def test_conjugate_symmetry(eng):
    mdl = wl.mimo64(K=100)
    h1 = _run(eng, mdl, _prec("fp64"))
    h2 = _run(eng, mdl, _prec("fp64"), omega=-mdl.omega)
    assert oracle.rel_err(h2.G, np.conj(h1.G)).max() <= 1e-12


def test_singular_point_flagged(eng):
    from paper_2401_04068_amd import binding

    A = np.zeros((1, 1))
    B = np.ones((1, 1))
    C = np.ones((1, 1))
    D = np.zeros((1, 1))
    h = _run(eng, (A, B, C, D, np.array([0.0, 2.0])), _prec("fp64"))
    assert h.info["path"][0] == binding.PATH_SINGULAR
    assert h.info["path"][1] == binding.PATH_FP64
    assert abs(h.G[1, 0, 0] - 1.0 / 2.0j) < 1e-15
    assert h.result["n_singular"] == 1


def test_no_d_matrix(eng):
    mdl = wl.siso8()
    h = _run(eng, (mdl.A, mdl.B, mdl.C, None, mdl.omega), _prec("fp64"))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, None, mdl.omega)
    assert oracle.rel_err(h.G, ref).max() <= TOL_FP64


def test_device_memory_request_equals_host(eng):
    import torch

    mdl = wl.mimo64(K=500)
    dev = "cuda:0"
    t = {k: torch.from_numpy(getattr(mdl, k)).to(dev) for k in ("A", "B", "C", "D", "omega")}
    G = torch.empty((mdl.K, mdl.p, mdl.m, 2), dtype=torch.float64, device=dev)
    h = eng.submit_device(t["A"], t["B"], t["C"], t["D"], t["omega"], G)
    assert eng.poll(h, -1)
    torch.cuda.synchronize()
    Gd = G.cpu().numpy()
    Gd = Gd[..., 0] + 1j * Gd[..., 1]
    hh = _run(eng, mdl, _prec("fp64"))
    assert np.array_equal(Gd, hh.G)


def test_caller_result_buffers(eng):
    """Results written into arrays the caller passes (and reuses): the same
    as in freshly allocated arrays (to rounding: the column split of the
    tiles follows the engine's load), every entry overwritten."""
    from paper_2401_04068_amd import binding

    mdl = wl.mimo64(K=300)
    ref = _run(eng, mdl, _prec("refined"))
    G = np.full((mdl.K, mdl.p, mdl.m), np.nan + 1j * np.nan)
    info = np.empty(mdl.K, dtype=binding.POINT_INFO_DTYPE)
    info.view(np.uint8).fill(0xff)
    for _ in range(2):
        h = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, precision=_prec("refined"), out=(G, info))
        assert eng.poll(h, -1)
        assert h.G is G and h.info is info
        assert oracle.rel_err(G, ref.G).max() <= 1e-12
        assert np.array_equal(info["path"], ref.info["path"])
        G[:] = np.nan
    with pytest.raises(ValueError):
        eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, out=(G[:, :, :1], info))


def test_repeat_query_reuses_reduction(eng):
    mdl = wl.mimo64(K=300)
    s0 = eng.stats()
    h1 = _run(eng, mdl, _prec("refined"), key=77)
    h2 = _run(eng, mdl, _prec("refined"), key=77)
    s1 = eng.stats()
    assert h1.result["reduction_reused"] == 0 and h2.result["reduction_reused"] == 1
    assert s1["reductions"] - s0["reductions"] == 1
    assert s1["reduction_cache_hits"] - s0["reduction_cache_hits"] == 1
    assert np.array_equal(h1.G, h2.G)
    # a different model under the same key is not confused with it
    other = wl.mimo64(seed=99, K=300)
    h3 = _run(eng, other, _prec("refined"), key=77)
    assert h3.result["reduction_reused"] == 0
    ref = oracle.freqresp(other.A, other.B, other.C, other.D, other.omega)
    assert oracle.rel_err(h3.G, ref).max() <= TOL_REFINED


def test_repeats_and_new_models_in_flight_together(eng):
    """Repeat queries of one model, submitted while its first query (and the
    reductions of new models between them) are still in flight, wait for that
    reduction and all match the oracle."""
    base = wl.mimo64(K=300)
    others = wl.serving_requests(6, start=80)
    p64 = _prec("fp64")
    hs = [eng.submit(base.A, base.B, base.C, base.D, base.omega, precision=p64, model_key=501)]
    reqs = [base]
    for i, r in enumerate(others):
        hs.append(eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=p64, model_key=600 + i))
        hs.append(eng.submit(base.A, base.B, base.C, base.D, base.omega, precision=p64, model_key=501))
        reqs += [r, base]
    for h in hs:
        assert eng.poll(h, -1)
    sub = slice(None, None, 7)
    for r, h in zip(reqs, hs):
        ref = oracle.freqresp(r.A, r.B, r.C, r.D, r.omega[sub])
        assert oracle.rel_err(h.G[sub], ref).max() <= TOL_FP64, (r.n, r.m, r.p, r.K)
    assert sum(h.result["reduction_reused"] for h in hs[2::2]) == len(others)


def _mix_vs_alone(eng, reqs):
    alone = [_run(eng, r, _prec("refined")).G for r in reqs]
    handles = [eng.submit(r.A, r.B, r.C, r.D, r.omega, precision=_prec("refined")) for r in reqs]
    for h in handles:
        assert eng.poll(h, -1)
    return alone, [h.G for h in handles]


def test_serving_mix_equals_alone(eng):
    """Requests of uneven (n, m, p, K) in flight together give the same G as
    when each runs alone, within the refined tolerance, and match the oracle.
    (Under load the engine splits right-hand-side columns over fewer tiles,
    which changes the order of some sums.)"""
    reqs = wl.serving_requests(12, start=40)
    alone, mixed = _mix_vs_alone(eng, reqs)
    for r, g, ga in zip(reqs, mixed, alone):
        assert oracle.rel_err(g, ga).max() <= TOL_REFINED, (r.n, r.m, r.p, r.K)
        sub = slice(None, None, 17)
        ref = oracle.freqresp(r.A, r.B, r.C, r.D, r.omega[sub])
        assert oracle.rel_err(g[sub], ref).max() <= TOL_REFINED


def test_serving_mix_bitwise_with_fixed_tiling(monkeypatch):
    """With the column split fixed, the tiling no longer depends on the load
    and the mix reproduces each request's result alone bit for bit."""
    from paper_2401_04068_amd import binding

    monkeypatch.setenv("LTI_FREQRESP_RHS_SPLIT", "1")
    reqs = wl.serving_requests(12, start=40)
    with binding.Engine(arena_bytes=2 << 30) as e2:
        alone, mixed = _mix_vs_alone(e2, reqs)
    for r, g, ga in zip(reqs, mixed, alone):
        assert np.array_equal(g, ga), (r.n, r.m, r.p, r.K)


def test_error_codes(eng):
    from paper_2401_04068_amd import binding

    mdl = wl.siso8()
    A = mdl.A.copy()
    A[0, 0] = np.nan
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(A, mdl.B, mdl.C, mdl.D, mdl.omega)
    assert ei.value.code == binding.LTI_EINVAL
    big = np.eye(1025)
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(-big, np.ones((1025, 1)), np.ones((1, 1025)), None, [1.0])
    assert ei.value.code == binding.LTI_EUNSUPPORTED
    # 16 x 16 outputs: 4 KiB of G per frequency, 600k frequencies > the 2 GiB arena
    with pytest.raises(binding.LtiError) as ei:
        eng.submit(-np.eye(4), np.ones((4, 16)), np.ones((16, 4)), None, np.linspace(0, 1, 600_000))
    assert ei.value.code == binding.LTI_ENOSPC
    bogus = binding.Handle(987654321, None, None)
    with pytest.raises(binding.LtiError) as ei:
        eng.poll(bogus, 0)
    assert ei.value.code == binding.LTI_ENOENT


@pytest.mark.parametrize("split", ["1", "2", "3"])
def test_rhs_split_policies_agree(split, monkeypatch):
    """Splitting a request's right-hand-side columns over several tiles (a
    scheduling choice that depends only on the request) changes the order of
    the final lane reduction, not the result beyond rounding."""
    from paper_2401_04068_amd import binding

    mdl = wl.mixed_pole_model(np.random.default_rng(5), 70, 5, 3, wl.logspace_grid(1e-2, 1e2, 300))
    outs = {}
    for knob in ("1", split):
        monkeypatch.setenv("LTI_FREQRESP_RHS_SPLIT", knob)
        with binding.Engine(arena_bytes=256 << 20) as e:
            for prec in ("fp64", "refined"):
                h = e.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, precision=_prec(prec))
                assert e.poll(h, -1)
                outs[(knob, prec)] = h.G
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    assert oracle.rel_err(outs[(split, "fp64")], outs[("1", "fp64")]).max() <= 1e-14
    for knob in ("1", split):
        assert oracle.rel_err(outs[(knob, "fp64")], ref).max() <= TOL_FP64
        assert oracle.rel_err(outs[(knob, "refined")], ref).max() <= TOL_REFINED


@pytest.mark.parametrize("n", [1, 2, 7, 16, 17, 31, 33, 48, 63, 64])
def test_four_frequency_kernel_matches_single(n, monkeypatch):
    """The four-frequencies-per-wavefront float64 kernel (models up to 64
    states) against the one-frequency-per-wavefront kernel and the oracle;
    grid sizes that leave partly filled groups of four."""
    from paper_2401_04068_amd import binding

    rng = np.random.default_rng(9000 + n)
    w = np.concatenate([[0.0, -1.25], wl.logspace_grid(1e-2, 1e2, 27)])  # 29 points
    mdl = wl.mixed_pole_model(rng, n, 3, 2, w)
    outs = {}
    for knob in ("0", "1"):
        monkeypatch.setenv("LTI_FREQRESP_SWEEP16", knob)
        with binding.Engine(arena_bytes=256 << 20) as e:
            h = e.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
            assert e.poll(h, -1)
            outs[knob] = (h.G, h.info.copy())
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    assert oracle.rel_err(outs["1"][0], ref).max() <= TOL_FP64
    assert oracle.rel_err(outs["1"][0], outs["0"][0]).max() <= 1e-13
    assert np.array_equal(outs["1"][1]["path"], outs["0"][1]["path"])


@pytest.mark.parametrize("n,m,p", [(65, 3, 2), (66, 1, 1), (80, 2, 5), (95, 4, 4), (96, 3, 3), (97, 2, 1),
                                   (100, 4, 6), (113, 1, 3), (127, 2, 2), (128, 4, 4)])
def test_two_frequency_kernel_matches_single(n, m, p, monkeypatch):
    """The two-frequencies-per-wavefront kernels (65 to 128 states, at most
    four columns) against the one-frequency-per-wavefront kernels and the
    oracle, both precisions; 29 grid points leave one pair half filled."""
    from paper_2401_04068_amd import binding

    rng = np.random.default_rng(9050 + n)
    w = np.concatenate([[0.0, -1.25], wl.logspace_grid(1e-2, 1e2, 27)])
    mdl = wl.mixed_pole_model(rng, n, m, p, w)
    outs = {}
    for knob in ("0", "1"):
        monkeypatch.setenv("LTI_FREQRESP_SWEEP32", knob)
        with binding.Engine(arena_bytes=256 << 20) as e:
            for prec in ("fp64", "refined"):
                print(f"case two-frequency n={n} m={m} p={p} knob={knob} {prec}", flush=True)
                h = e.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, precision=_prec(prec))
                assert e.poll(h, -1)
                outs[(knob, prec)] = (h.G, h.info.copy())
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    assert oracle.rel_err(outs[("1", "fp64")][0], ref).max() <= TOL_FP64
    assert oracle.rel_err(outs[("1", "fp64")][0], outs[("0", "fp64")][0]).max() <= 1e-13
    assert np.array_equal(outs[("1", "fp64")][1]["path"], outs[("0", "fp64")][1]["path"])
    assert oracle.rel_err(outs[("1", "refined")][0], ref).max() <= TOL_REFINED
    assert np.all(outs[("1", "refined")][1]["path"] == binding.PATH_REFINED)


@pytest.mark.parametrize("split,m", [("2", 4), ("0", 7), ("0", 16)])
def test_two_frequency_kernel_column_groups(split, m, monkeypatch):
    """Columns over several tiles of the two-frequency kernels: a forced
    split of four columns into two groups, and 7 and 16 columns in groups of
    four (merged point records)."""
    from paper_2401_04068_amd import binding

    rng = np.random.default_rng(9070 + m)
    mdl = wl.mixed_pole_model(rng, 110, m, 16, wl.logspace_grid(1e-2, 1e2, 41))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    monkeypatch.setenv("LTI_FREQRESP_RHS_SPLIT", split)
    with binding.Engine(arena_bytes=256 << 20) as e:
        for prec in ("fp64", "refined"):
            print(f"case two-frequency columns split={split} m={m} {prec}", flush=True)
            h = e.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, precision=_prec(prec))
            assert e.poll(h, -1)
            tol = TOL_FP64 if prec == "fp64" else TOL_REFINED
            assert oracle.rel_err(h.G, ref).max() <= tol
            want = binding.PATH_FP64 if prec == "fp64" else binding.PATH_REFINED
            assert np.all(h.info["path"] == want)
            assert np.all(h.info["iters"] >= 1)


@pytest.mark.parametrize("n,m,p", [(257, 3, 2), (300, 5, 4), (512, 2, 3), (1024, 16, 16)])
def test_large_state_dimensions(eng, n, m, p):
    """Models above 256 states (one workgroup per frequency), float64 path."""
    rng = np.random.default_rng(12000 + n)
    w = np.concatenate([[0.0, -3.0], wl.logspace_grid(1e-2, 1e2, 7)])
    mdl = wl.mixed_pole_model(rng, n, m, p, w)
    print(f"case large n={n} m={m} p={p}", flush=True)
    h = _run(eng, mdl, _prec("fp64"))
    ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
    err = oracle.rel_err(h.G, ref)
    assert err.max() <= TOL_FP64, (n, err.max(), int(err.argmax()))
    assert np.all(h.info["path"] == 0)
