"""design_greedy_noalloc against design_greedy through the C ABI: the same
order and curve bit for bit, on two calls in a row (the second smaller, so
it reuses the scratch the first left behind), for a uniform and a Gaussian
prior; oversize requests are refused before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


def _hessians(rng, S, C):
    G = rng.standard_normal((S, C, 7, 4))
    scale = (0.2 + (np.arange(C) * 7 % C) / C) ** 2
    return np.einsum("scik,scjk->scij", G, G) * scale[None, :, None, None] + \
        1e-2 * np.eye(7)[None, None]


@pytest.mark.parametrize("gaussian", [False, True])
def test_noalloc_greedy_equals_design_greedy(gaussian):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context, make_prior
    rng = np.random.default_rng(7 + gaussian)
    lo, hi = -np.ones(7), np.ones(7)
    prior = (make_prior(mean=np.zeros(7), cov=np.diag(np.linspace(0.5, 2.0, 7)))
             if gaussian else make_prior(lo, hi))
    with Context(0, 1 << 30) as ctx:
        for S, C, K in ((97, 41, 12), (23, 9, 5)):   # the second call is smaller
            _say(f"design_greedy_noalloc S={S} C={C} K={K} gaussian={gaussian}")
            H = torch.as_tensor(_hessians(rng, S, C), device="cuda")
            X = rng.uniform(-1, 1, (S, 7))
            W = rng.uniform(0.5, 1.5, S)
            W /= W.sum()
            o_ref = torch.empty(K, dtype=torch.int32, device="cuda")
            c_ref = torch.empty(K, dtype=torch.float64, device="cuda")
            ctx.design_greedy(H, prior, W, K, o_ref, c_ref, theta=X)
            o = torch.full((K,), -7, dtype=torch.int32, device="cuda")
            c = torch.full((K,), -7.0, dtype=torch.float64, device="cuda")
            ctx.design_greedy_noalloc(H, prior, torch.as_tensor(W, device="cuda"), K, o, c,
                                      theta=torch.as_tensor(X, device="cuda") if gaussian
                                      else None)
            torch.cuda.synchronize()
            assert torch.equal(o, o_ref), (o.cpu(), o_ref.cpu())
            assert torch.equal(c, c_ref), (c.cpu(), c_ref.cpu())
            assert len(set(o.cpu().tolist())) == K


def test_noalloc_greedy_refuses_oversize_requests():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context, eigseis, make_prior
    prior = make_prior(-np.ones(7), np.ones(7))
    small = torch.zeros(64, dtype=torch.float64, device="cuda")
    order = torch.zeros(4, dtype=torch.int32, device="cuda")
    with Context(0, 1 << 30) as ctx:
        # 100000 samples x 100 candidates need ~118 MiB of scratch: refused
        # before any launch reads the (too small) arrays
        rc = eigseis._lib.design_greedy_noalloc(
            ctx._h, 100000, 100, small.data_ptr(), ctypes.byref(prior), None,
            small.data_ptr(), 4, order.data_ptr(), small.data_ptr(), None)
        assert rc == eigseis.EIG_EBUDGET
        assert b"MiB scratch" in eigseis._lib.eig_last_error()
        torch.cuda.synchronize()
