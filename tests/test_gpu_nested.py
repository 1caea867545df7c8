"""Nested Monte Carlo EIG and reduced-parameter Laplace on the GPU vs the
oracle, through the C ABI.  Log ratios and their mean within 1e-3 nats
(both sides take the same FP32 inputs and compute in FP64)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import elastic, laplace, nested

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAT_TOL = 1e-3


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    c = Context(0, 16 << 30)
    yield c
    c.close()


def _run(ctx, go, noise, gi, sigma):
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")  # noqa: E731
    lr = torch.empty(go.shape[0], dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.nested_mc_eig(t(go), t(noise), t(gi), sigma, lr, eig)
    torch.cuda.synchronize()
    return lr.cpu().numpy(), float(eig.cpu()[0])


@pytest.mark.parametrize("N,M,K", [(77, 130, 37), (300, 500, 204), (1, 1, 1), (65, 64, 17)])
def test_nested_kernel_matches_oracle(ctx, N, M, K):
    # ragged tile tails in rows, columns and observations; signal-to-noise
    # like the seismic traces (|g| up to ~100 sigma)
    _say(f"nested kernel N={N} M={M} K={K}")
    rng = np.random.default_rng(N * 7 + M)
    sigma = 0.01
    A = rng.standard_normal((K, 3)) * 0.3
    th_o, th_i = rng.standard_normal((N, 3)), rng.standard_normal((M, 3))
    go = (th_o @ A.T).astype(np.float32)
    gi = (th_i @ A.T).astype(np.float32)
    noise = rng.standard_normal((N, K)).astype(np.float32)
    lr, eig = _run(ctx, go, noise, gi, sigma)
    ref = nested.log_ratios(go.astype(np.float64), noise.astype(np.float64),
                            gi.astype(np.float64), sigma)
    assert np.max(np.abs(lr - ref)) <= NAT_TOL, np.max(np.abs(lr - ref))
    assert abs(eig - ref.mean()) <= NAT_TOL


def test_nested_inner_splits_with_empty_tail_match_oracle(ctx):
    # 130 outer rows (a full and a 2-row block), 4100 inner samples over 16
    # inner-range splits of 384 whose last five hold no columns, 45
    # observations (two full k chunks and a ragged one)
    _say("nested kernel N=130 M=4100 K=45 (splits, empty tail)")
    rng = np.random.default_rng(41)
    sigma = 0.02
    A = rng.standard_normal((45, 4)) * 0.2
    go = (rng.standard_normal((130, 4)) @ A.T).astype(np.float32)
    gi = (rng.standard_normal((4100, 4)) @ A.T).astype(np.float32)
    noise = rng.standard_normal((130, 45)).astype(np.float32)
    lr, eig = _run(ctx, go, noise, gi, sigma)
    ref = nested.log_ratios(go.astype(np.float64), noise.astype(np.float64),
                            gi.astype(np.float64), sigma)
    assert np.max(np.abs(lr - ref)) <= NAT_TOL, np.max(np.abs(lr - ref))
    assert abs(eig - ref.mean()) <= NAT_TOL


def test_nested_large_amplitude_within_gram_rounding(ctx):
    # traces of up to ~3e4 sigma: the squared distances, formed as |y|^2 +
    # |g|^2 - 2<y, g>, round to ~K 2^-53 (|y|^2 + |g|^2) / (2 sigma^2), here
    # ~3e-5 nats at most
    _say("nested kernel N=257 M=700 K=37 at up to ~3e4 sigma")
    rng = np.random.default_rng(77)
    sigma = 0.01
    A = rng.standard_normal((37, 3)) * 30.0
    go = (rng.standard_normal((257, 3)) @ A.T).astype(np.float32)
    gi = (rng.standard_normal((700, 3)) @ A.T).astype(np.float32)
    noise = rng.standard_normal((257, 37)).astype(np.float32)
    assert np.abs(go).max() / sigma > 1000
    lr, _ = _run(ctx, go, noise, gi, sigma)
    ref = nested.log_ratios(go.astype(np.float64), noise.astype(np.float64),
                            gi.astype(np.float64), sigma)
    y = go.astype(np.float64) + sigma * noise.astype(np.float64)
    bound = 37 * 2.0 ** -53 * (np.sum(y ** 2, axis=1).max() + np.sum(gi.astype(np.float64) ** 2, axis=1).max()) \
        / (2 * sigma ** 2)
    assert np.max(np.abs(lr - ref)) <= max(4 * bound, 1e-5), (np.max(np.abs(lr - ref)), bound)


def test_nested_reuse_bound_and_single_sample(ctx):
    rng = np.random.default_rng(5)
    g = rng.standard_normal((200, 50)).astype(np.float32)
    noise = rng.standard_normal((200, 50)).astype(np.float32)
    lr, _ = _run(ctx, g, noise, g, 0.05)
    assert np.all(lr <= math.log(200) + 1e-9)
    lr1, _ = _run(ctx, g[:1], noise[:1], g[:1], 0.05)
    assert abs(lr1[0]) < 1e-9


def test_model_problem_nested_and_reduced_laplace(ctx):
    # Section 4.4 setup at a small size: forward solves, nested MC with the
    # outer samples reused as inner ones, and Theorem 4 on the three inferred
    # parameters (prior active mask) for the same samples
    from paper_1502_07873_amd import make_prior
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    _say("model problem nested MC + reduced Laplace")
    grid, med, rec, lo, hi, _ = synthetic.loh_nested_setup()
    rng = np.random.default_rng(9)
    th = synthetic.loh_nested_draws(rng, 96)
    N = len(th)
    K = (grid.nsteps + 1) * len(rec) * 2
    g = torch.empty((N, K), dtype=torch.float32, device="cuda")
    dm = device_medium(med.kind, med.rho, med.lam, med.mu)
    ctx.forward_solve_batch([grid_tuple(grid)] * N, [dm] * N, th, [rec] * N, list(g),
                            stf="gauss")
    noise = rng.standard_normal((N, K)).astype(np.float32)
    nz = torch.as_tensor(noise, device="cuda")
    lr = torch.empty(N, dtype=torch.float64, device="cuda")
    ctx.nested_mc_eig(g, nz, g, 0.01, lr)
    gref = np.stack([elastic.forward(grid, med, x, rec, "gauss").ravel() for x in th])
    torch.cuda.synchronize()
    assert np.max(np.abs(g.cpu().numpy() - gref)) <= 1e-5 * np.abs(gref).max()
    ref = nested.log_ratios(g.cpu().numpy().astype(np.float64), noise.astype(np.float64),
                            g.cpu().numpy().astype(np.float64), 0.01)
    assert np.max(np.abs(lr.cpu().numpy() - ref)) <= NAT_TOL
    # reduced Laplace on 8 of the samples
    S = 8
    act = list(synthetic.LOH_NESTED_ACTIVE)
    H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
    ctx.jacobian_fd([grid_tuple(grid)] * S, [dm] * S, th[:S], [rec] * S, 0.01, H1, stf="gauss")
    dkl = torch.empty(S, dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.laplace_eig(H1, make_prior(lo, hi, active=act), np.full(S, 1.0 / S), dkl, eig,
                    theta=th[:S])
    torch.cuda.synchronize()
    pr = laplace.uniform_prior(lo[act], hi[act])
    want = []
    for s in range(S):
        J = elastic.jacobian_literal(grid, med, th[s], rec, 1e-4, "gauss")[1]
        Hs = laplace.hessian_h1(J, 0.01)[np.ix_(act, act)]
        want.append(laplace.dkl_hat(Hs, th[s][act], pr)[0])
    assert np.max(np.abs(dkl.cpu().numpy() - np.array(want))) <= NAT_TOL
    assert abs(float(eig.cpu()[0]) - np.mean(want)) <= NAT_TOL


def test_active_mask_gaussian_prior_marginal(ctx):
    # Gaussian prior restricted to a subset: the marginal (sub-mean,
    # sub-covariance) enters h; H_1 sub-block as for the uniform prior
    from paper_1502_07873_amd import make_prior
    rng = np.random.default_rng(3)
    S = 5
    B = rng.standard_normal((S, 7, 7))
    H = np.einsum("sij,skj->sik", B, B) + 7 * np.eye(7)
    Ct = rng.standard_normal((7, 7))
    cov = Ct @ Ct.T + 7 * np.eye(7)
    mean = rng.standard_normal(7)
    th = rng.standard_normal((S, 7))
    act = [0, 2, 5]
    Hd = torch.as_tensor(H, device="cuda")
    dkl = torch.empty(S, dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.laplace_eig(Hd, make_prior(mean=mean, cov=cov, active=act), np.full(S, 0.2), dkl, eig,
                    theta=th)
    torch.cuda.synchronize()
    pr = {"kind": "gaussian", "mean": mean[act], "cov": cov[np.ix_(act, act)]}
    want = [laplace.dkl_hat(H[s][np.ix_(act, act)], th[s][act], pr)[0] for s in range(S)]
    assert np.max(np.abs(dkl.cpu().numpy() - want)) < 1e-9


def test_nested_full_size_sampled_rows(ctx):
    # Section 4.4 size: N = M = 4e5 outer samples reused as the inner ones,
    # K = 204 observations (51 levels x 2 receivers x 2 components), traces of
    # up to ~16 sigma, so log ratios of 6-10 nats, below log M: many inner
    # samples contribute to each evidence.  Every log ratio is at most log M
    # (reuse); sampled rows, the first and last blocks' edges included,
    # against the oracle
    N, K, sigma = 400_000, 204, 0.01
    _say(f"nested full size N=M={N} K={K}")
    rng = np.random.default_rng(2024)
    A = (rng.standard_normal((K, 3)) * 0.03).astype(np.float32)
    th = rng.uniform(-1.0, 1.0, (N, 3)).astype(np.float32)
    g = th @ A.T
    noise = rng.standard_normal((N, K), dtype=np.float32)
    gd = torch.as_tensor(g, device="cuda")
    nd = torch.as_tensor(noise, device="cuda")
    lr = torch.empty(N, dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.nested_mc_eig(gd, nd, gd, sigma, lr, eig)
    torch.cuda.synchronize()
    lr = lr.cpu().numpy()
    assert np.all(np.isfinite(lr))
    assert np.all(lr <= math.log(N) + 1e-6)
    assert abs(float(eig.cpu()[0]) - lr.mean()) < 1e-9 * max(1.0, abs(lr.mean()))
    rows = np.unique(np.concatenate([[0, 127, 128, N - 129, N - 1],
                                     rng.integers(0, N, 11)]))
    g64 = g.astype(np.float64)
    ref = nested.log_ratios(g64[rows], noise[rows].astype(np.float64), g64, sigma)
    assert np.max(np.abs(lr[rows] - ref)) <= NAT_TOL, np.max(np.abs(lr[rows] - ref))
