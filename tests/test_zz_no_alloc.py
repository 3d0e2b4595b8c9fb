"""GPU: lti_freqresp_eval_noalloc (the entry point that allocates nothing)
against the context path (submit + poll of the same device-memory request)
and against the oracle, on two calls in a row, the second smaller, so that
the second call runs on scratch memory the first one left behind."""
import numpy as np
import pytest

import oracle
from paper_2401_04068_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _model(n, m, p, K, seed):
    rng = np.random.default_rng(seed)
    return wl.mixed_pole_model(rng, n, m, p, wl.logspace_grid(1e-3, 1e3, K), seed)


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def _run_noalloc(mdl, precision, torch, binding):
    K, p, m = len(mdl.omega), mdl.C.shape[0], mdl.B.shape[1]
    args = [_dev(v, torch) for v in (mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)]
    G = torch.full((K * p * m * 2,), float("nan"), dtype=torch.float64, device="cuda:0")
    info = torch.full((K * 8,), 0xFF, dtype=torch.uint8, device="cuda:0")
    binding.eval_noalloc(*args, G, info=info, precision=precision)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().view(np.complex128).reshape(K, p, m)
    ih = info.cpu().numpy().view(binding.POINT_INFO_DTYPE)
    return Gh, ih


def _run_context(eng, mdl, precision, torch, binding):
    K, p, m = len(mdl.omega), mdl.C.shape[0], mdl.B.shape[1]
    args = [_dev(v, torch) for v in (mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)]
    G = torch.zeros(K * p * m * 2, dtype=torch.float64, device="cuda:0")
    info = torch.zeros(K * 8, dtype=torch.uint8, device="cuda:0")
    h = eng.submit_device(*args, G, info=info, precision=precision)
    assert eng.poll(h, -1)
    torch.cuda.synchronize()
    return (G.cpu().numpy().view(np.complex128).reshape(K, p, m),
            info.cpu().numpy().view(binding.POINT_INFO_DTYPE))


# (n, m, p, K): first call, then a smaller one
CASES = [
    ((64, 4, 4, 2000), (40, 3, 2, 700)),
    ((200, 5, 3, 1500), (100, 2, 6, 301)),
    ((7, 1, 1, 400), (3, 2, 2, 5)),
]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_context_path_twice(case, precision):
    import torch

    from paper_2401_04068_amd import binding

    tol = 1e-10 if precision == binding.PREC_FP64 else 1e-9
    with binding.Engine(arena_bytes=512 << 20, device=0) as eng:
        for call, (n, m, p, K) in enumerate(CASES[case]):
            mdl = _model(n, m, p, K, seed=7100 + 10 * case + call)
            print(f"case noalloc n={n} m={m} p={p} K={K} precision={precision} call={call}", flush=True)
            Gn, infn = _run_noalloc(mdl, precision, torch, binding)
            Gc, infc = _run_context(eng, mdl, precision, torch, binding)
            ref = oracle.freqresp(mdl.A, mdl.B, mdl.C, mdl.D, mdl.omega)
            assert np.all(np.isfinite(Gn.view(np.float64)))
            assert oracle.rel_err(Gn, ref).max() <= tol
            # same kernels, same tiling as a context running the request alone
            np.testing.assert_array_equal(Gn.view(np.float64), Gc.view(np.float64))
            np.testing.assert_array_equal(infn["path"], infc["path"])
            np.testing.assert_array_equal(infn["iters"], infc["iters"])


def test_noalloc_rejects_beyond_its_limits():
    import torch

    from paper_2401_04068_amd import binding

    t = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    A = torch.zeros(300 * 300, dtype=torch.float64, device="cuda:0").view(300, 300)
    B = torch.zeros(300, 1, dtype=torch.float64, device="cuda:0")
    C = torch.zeros(1, 300, dtype=torch.float64, device="cuda:0")
    with pytest.raises(binding.LtiError) as ei:
        binding.eval_noalloc(A, B, C, None, t, t, precision=0)
    assert ei.value.code == binding.LTI_EUNSUPPORTED
    A2 = torch.zeros(4, 4, dtype=torch.float64, device="cuda:0")
    B2 = torch.zeros(4, 1, dtype=torch.float64, device="cuda:0")
    C2 = torch.zeros(1, 4, dtype=torch.float64, device="cuda:0")
    w = torch.zeros((1 << 18) + 1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(binding.LtiError) as ei:
        binding.eval_noalloc(A2, B2, C2, None, w, w, precision=0)
    assert ei.value.code == binding.LTI_EUNSUPPORTED
