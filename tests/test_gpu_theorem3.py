"""Theorem-3 estimator on the GPU vs the oracle, through the C ABI.

H_2 from one dual (time-reversed) solve against the oracle's 22 direct
second-derivative solves; the MAP point, H_1 and the integrand against the
oracle's Gauss-Newton.  Tolerances: H entries relative to sqrt(H1_ii H1_jj)
<= 1e-3, MAP within 1e-2 posterior standard deviations, integrands within
1e-3 nats.
"""
import numpy as np
import pytest

import synthetic
from oracle import elastic, laplace, theorem3

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAT_TOL = 1e-3


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


def _case(kind, nsample, seed):
    rng = np.random.default_rng(seed)
    nx, nz, h = 48, 44, 16.0
    if kind == "nodal":
        med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=80.0)
    else:
        med = synthetic.random_layers_medium(rng, nz, h, 3, vp_lo=2500.0, vp_hi=3500.0)
    grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), 260)
    lo, hi = synthetic.prior_box(grid)
    th = synthetic.draw_uniform(rng, lo, hi, nsample)
    rec = synthetic.equispaced_receivers(nx, 7)
    peak = np.abs(elastic.forward(grid, med, 0.5 * (lo + hi), rec)).max()
    sigma = 0.02 * peak
    noise = rng.standard_normal((nsample, grid.nsteps + 1, len(rec), 2)).astype(np.float32)
    return grid, med, rec, lo, hi, th, sigma, noise


def _run(ctx_opts, grid, med, rec, th, sigma, noise, prior, iters):
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    S = len(th)
    dm = device_medium(med.kind, med.rho, med.lam, med.mu)
    nz = [torch.as_tensor(noise[s], device="cuda") for s in range(S)]
    H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
    H2 = torch.empty_like(H1)
    val = torch.empty(S, dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(S, dtype=torch.int32, device="cuda")
    with Context(0, 8 << 30) as ctx:
        for k, v in ctx_opts.items():
            ctx.set_option(k, v)
        th_hat = ctx.theorem3_eig([grid_tuple(grid)] * S, [dm] * S, th, [rec] * S, nz, sigma,
                                  prior, np.full(S, 1.0 / S), H1, H2, val, eig, st,
                                  iters=iters)
        torch.cuda.synchronize()
    return (th_hat, H1.cpu().numpy(), H2.cpu().numpy(), val.cpu().numpy(),
            float(eig.cpu()[0]), st.cpu().numpy())


@pytest.mark.parametrize("kind,opts", [("layered", {}), ("layered", {"stencil_variant": 0}),
                                       ("nodal", {"stencil_variant": 6}),
                                       ("nodal", {"stencil_variant": 17})])
def test_h2_from_dual_solve_matches_direct_second_derivatives(kind, opts):
    # iters = 0: theta^ = theta*, so only the dual solve and its contraction
    # are compared (two-nodes-per-lane, one-node-per-lane and both nodal kernels)
    from paper_1502_07873_amd import make_prior
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _say(f"H2 dual vs direct ({kind}, {opts})")
    grid, med, rec, lo, hi, th, sigma, noise = _case(kind, 2, 3)
    th_hat, H1, H2, _, _, st = _run(opts, grid, med, rec, th, sigma, noise,
                                    make_prior(lo, hi), 0)
    assert np.array_equal(th_hat, th)
    for s in range(len(th)):
        g = elastic.forward(grid, med, th[s], rec)
        y = g + sigma * noise[s].astype(np.float64)
        H2r = theorem3.hessian_h2(grid, med, th[s], rec, y, sigma)
        _, J = elastic.jacobian_sensitivity(grid, med, th[s], rec)
        H1r = laplace.hessian_h1(J, sigma)
        d = np.sqrt(np.diag(H1r))
        sc = np.outer(d, d)
        # away from the MAP point H_1 + H_2 need not be definite (the noise
        # term of H_2); the status must say what the oracle's matrix is
        pd = np.linalg.eigvalsh((H1r + H2r) / sc).min() > 0
        assert (st[s] == 0) == pd, (s, st[s], pd)
        assert np.max(np.abs(H2r / sc)) > 1e-3          # H_2 is resolved
        assert np.max(np.abs((H1[s] - H1r) / sc)) < 1e-4
        assert np.max(np.abs((H2[s] - H2r) / sc)) < 1e-3, np.max(np.abs((H2[s] - H2r) / sc))


@pytest.mark.parametrize("prior_kind", ["uniform", "gaussian"])
def test_theorem3_estimator_matches_oracle(prior_kind):
    from paper_1502_07873_amd import make_prior
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _say(f"theorem3 estimator ({prior_kind})")
    grid, med, rec, lo, hi, th, sigma, noise = _case("layered", 3, 5)
    if prior_kind == "uniform":
        prior_o = laplace.uniform_prior(lo, hi)
        prior_g = make_prior(lo, hi)
    else:
        mean = 0.5 * (lo + hi)
        cov = np.diag(((hi - lo) / 4) ** 2)
        prior_o = {"kind": "gaussian", "mean": mean, "cov": cov}
        prior_g = make_prior(mean=mean, cov=cov)
    th_hat, H1, H2, val, eig, st = _run({}, grid, med, rec, th, sigma, noise, prior_g, 5)
    assert np.all(st == 0)
    want = []
    for s in range(len(th)):
        ref = theorem3.sample_terms(grid, med, rec, th[s], noise[s], sigma, prior_o, iters=6)
        d = np.sqrt(np.diag(ref["H1"]))
        sc = np.outer(d, d)
        assert np.max(np.abs((th_hat[s] - ref["theta_hat"]) * d)) < 1e-2
        assert np.max(np.abs((H1[s] - ref["H1"]) / sc)) < 1e-3
        assert np.max(np.abs((H2[s] - ref["H2"]) / sc)) < 1e-3
        assert abs(val[s] - ref["value"]) <= NAT_TOL, (s, val[s], ref["value"])
        want.append(ref["value"])
    assert abs(eig - np.mean(want)) <= NAT_TOL


def test_theorem3_rejects_absorbing_edges():
    from paper_1502_07873_amd import Context, eigseis, make_prior
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    wl = synthetic.loh_workload(1)
    dm = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    nz = [torch.zeros((wl.grid.nsteps + 1, len(wl.receivers), 2), device="cuda")]
    H = torch.empty((1, 7, 7), dtype=torch.float64, device="cuda")
    v = torch.empty(1, dtype=torch.float64, device="cuda")
    with Context(0, 1 << 30) as ctx:
        with pytest.raises(eigseis.EigError) as ei:
            ctx.theorem3_eig([grid_tuple(wl.grid)], [dm], wl.theta[:1], [wl.receivers], nz,
                             0.01, make_prior(wl.lo, wl.hi), [1.0], H, H.clone(), v)
    assert ei.value.code == eigseis.EIG_EUNSUPPORTED
