"""The 1024-state, 16x16 workload at full size: 10,000 frequencies of one
model, then a repeat query on a shifted grid that must reuse the resident
reduction; both the float64 path and the refined path (complex-float32
workgroup sweeps with float64 residuals).  Sampled points against the
float64 oracle (kappa is small for these mixed-pole models, so the float64
oracle is accurate to ~1e-13)."""
import numpy as np
import pytest

import oracle
from paper_2401_04068_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "refined"])
def test_large1024_full_grid_and_repeat(prec):
    from paper_2401_04068_amd import binding

    precision = binding.PREC_FP64 if prec == "fp64" else binding.PREC_REFINED
    tol = 1e-10 if prec == "fp64" else 1e-9
    models = wl.large1024_models(seeds=(4000,))
    mdl = models[0]
    queries = wl.large1024_queries(models * 8)  # query 8 repeats model 0, shifted
    w_repeat = queries[8][1]
    with binding.Engine(arena_bytes=4 << 30) as eng:
        print(f"case large1024 {prec} first query", flush=True)
        h1 = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega, model_key=4000, precision=precision)
        assert eng.poll(h1, -1)
        print(f"case large1024 {prec} repeat query", flush=True)
        h2 = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, w_repeat, model_key=4000, precision=precision)
        assert eng.poll(h2, -1)
        st = eng.stats()
    assert h1.result["reduction_reused"] == 0 and h2.result["reduction_reused"] == 1
    assert st["reductions"] == 1
    idx = np.unique(np.concatenate([np.arange(0, 10_000, 1111), [9999]]))
    for h, w in ((h1, mdl.omega), (h2, w_repeat)):
        ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, w[idx])
        err = oracle.rel_err(h.G[idx], ref)
        assert err.max() <= tol, err.max()
        if prec == "refined":
            assert h.result["n_refined"] + h.result["n_fallback"] == 10_000
            assert h.result["n_refined"] >= 9_990
            assert np.all(h.info["iters"][h.info["path"] == binding.PATH_REFINED] >= 2)


def test_blocked_reductions_of_one_pass_side_by_side(monkeypatch):
    """Models above 256 states of different sizes admitted together share the
    blocked reduction's launches (one model per blockIdx.z, the column loop
    of the largest): each result equals the one computed alone, bitwise (the
    column split of the sweep tiles is pinned, as it decides the order of the
    output sums), and matches the oracle."""
    from paper_2401_04068_amd import binding

    monkeypatch.setenv("LTI_FREQRESP_RHS_SPLIT", "1")
    rng = np.random.default_rng(4700)
    w = np.concatenate([[0.0, -2.0], wl.logspace_grid(1e-2, 1e2, 9)])
    shapes = [(257, 3, 2), (300, 1, 4), (384, 5, 5), (520, 2, 3), (290, 4, 1), (333, 2, 2)]
    mdls = [wl.mixed_pole_model(rng, n, m, p, w) for n, m, p in shapes]
    alone = []
    with binding.Engine(arena_bytes=2 << 30) as eng:
        for (n, m, p), mdl in zip(shapes, mdls):
            print(f"case blocked alone n={n}", flush=True)
            h = eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
            assert eng.poll(h, -1)
            alone.append(h.G)
    with binding.Engine(arena_bytes=2 << 30) as eng:
        print("case blocked together", flush=True)
        hs = [eng.submit(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega) for mdl in mdls]
        for h in hs:
            assert eng.poll(h, -1)
    for (n, m, p), mdl, h, g in zip(shapes, mdls, hs, alone):
        np.testing.assert_array_equal(h.G, g)
        ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
        assert oracle.rel_err(h.G, ref).max() <= 1e-10, (n, m, p)
