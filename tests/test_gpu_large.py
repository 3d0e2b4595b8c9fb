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
