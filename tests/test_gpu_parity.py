"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances (stated by the method's precision split: FP32 wavefields, FP64
Jacobian/Hessian/log-det): receiver traces relative L2 <= 1e-5 per solve,
Jacobian columns relative L2 <= 1e-3, D^_KL and EIG absolute <= 1e-3 nats.
"""
import numpy as np
import pytest

import synthetic
from _compare import check_greedy, check_jacobian, check_receivers, scaled_hessian_err
from oracle import elastic, laplace, pipeline as opipe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-5
JAC_TOL = 1e-3
NAT_TOL = 1e-3


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    c = Context(0, 48 << 30)
    yield c
    c.close()


def _dev_medium(med):
    from paper_1502_07873_amd.query import device_medium
    return device_medium(med.kind, med.rho, med.lam, med.mu)


def _forward(ctx, grid, medium, thetas, receivers, dev_param=None, dev_step=None,
             stf="gauss_deriv"):
    from paper_1502_07873_amd.query import grid_tuple
    n = len(thetas)
    g = grid_tuple(grid)
    dm = _dev_medium(medium)
    tr = [torch.empty((grid.nsteps + 1, len(receivers), 2), dtype=torch.float32,
                      device="cuda") for _ in range(n)]
    ctx.forward_solve_batch([g] * n, [dm] * n, np.asarray(thetas), [receivers] * n, tr,
                            dev_param=dev_param, dev_step=dev_step, stf=stf)
    torch.cuda.synchronize()
    return [t.cpu().numpy().astype(np.float64) for t in tr]


def test_forward_traces_c1(ctx):
    wl = synthetic.config("c1")[0]
    _say(f"forward c1 {wl.grid}")
    out = _forward(ctx, wl.grid, wl.medium, wl.theta, wl.receivers)
    for s, th in enumerate(wl.theta):
        ref = elastic.forward(wl.grid, wl.medium, th, wl.receivers)
        assert np.all(out[s][0] == 0)
        check_receivers(out[s], ref, TRACE_TOL, what=f"c1 solve {s}")


@pytest.mark.parametrize("case", ["ragged_layered", "ragged_nodal", "gauss_stf"])
def test_forward_traces_ragged(ctx, case):
    # grids that are not multiples of the 64x32 tile, receivers on the first
    # and last free columns, sources at the prior-box margins
    rng = np.random.default_rng(11)
    nx, nz, h = 133, 71, 12.0
    if case == "ragged_nodal":
        med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=60.0)
    else:
        med = synthetic.random_layers_medium(rng, nz, h, 4)
    grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), 333)
    lo, hi = synthetic.prior_box(grid)
    thetas = synthetic.draw_uniform(rng, lo, hi, 5)
    thetas[0, 0], thetas[0, 1] = lo[0], hi[1]
    thetas[1, 0], thetas[1, 1] = hi[0] - 1e-9, lo[1]
    rec = np.array([1, 2, 40, 63, 64, 65, 100, nx - 2], dtype=np.int32)
    stf = "gauss" if case == "gauss_stf" else "gauss_deriv"
    if stf == "gauss":
        thetas[:, 3] = rng.uniform(20, 40, len(thetas))
    _say(f"forward {case} {grid}")
    out = _forward(ctx, grid, med, thetas, rec, stf=stf)
    for s, th in enumerate(thetas):
        ref = elastic.forward(grid, med, th, rec, stf)
        check_receivers(out[s], ref, TRACE_TOL, what=f"{case} solve {s}")


def test_deviation_solves_match_literal_differences(ctx):
    wl = synthetic.config("c1", nsample=2)[0]
    th = wl.theta[0]
    d = elastic.fd_steps(th, 1e-4)
    _say("deviation solves c1")
    params = np.repeat(np.arange(7), 2).astype(np.int32)
    steps = np.array([d[j] * s for j in range(7) for s in (1, -1)])
    out = _forward(ctx, wl.grid, wl.medium, [th] * 14, wl.receivers, params, steps)
    for q in range(14):
        j = params[q]
        tp = th.copy()
        tp[j] += steps[q]
        ref = (elastic.forward(wl.grid, wl.medium, tp, wl.receivers)
               - elastic.forward(wl.grid, wl.medium, th, wl.receivers))
        check_receivers(out[q], ref, 1e-4, what=f"deviation solve {q}")


def test_jacobian_hessian_eig_c1(ctx):
    from paper_1502_07873_amd.query import grid_tuple, run_query
    wl = synthetic.config("c1")[0]
    _say("jacobian/H1/eig c1")
    ref = opipe.query(wl, keep_J=True)
    out = run_query(ctx, grid_tuple(wl.grid), _dev_medium(wl.medium), wl.receivers,
                    wl.lo, wl.hi, wl.theta, wl.weights, sigma=ref["sigma"],
                    keep_nominal=True, keep_J=True)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    for s in range(len(wl.theta)):
        check_receivers(out["nominal"][s].cpu().numpy(), ref["nominal"][s], TRACE_TOL,
                        what=f"nominal {s}")
        check_jacobian(out["J"][s].cpu().numpy(), ref["J"][s], JAC_TOL, what=f"sample {s}")
    # |dH_ij| <= (2 eps + eps^2) sqrt(H_ii H_jj) for columns within eps
    assert scaled_hessian_err(out["H1"].cpu().numpy(), ref["H1"]) <= 2 * JAC_TOL
    dkl = out["dkl"].cpu().numpy()
    assert np.max(np.abs(dkl - ref["dkl"])) <= NAT_TOL, np.abs(dkl - ref["dkl"])
    assert abs(float(out["eig"].cpu()[0]) - ref["eig"]) <= NAT_TOL


SENS_TOL = 1e-4   # one FP32 solve per column, no difference taken


def test_sensitivity_jacobian_hessian_eig_c1(ctx):
    # Algorithm 1's sensitivity solves on the GPU vs the oracle's
    from paper_1502_07873_amd.query import grid_tuple, run_query
    wl = synthetic.config("c1")[0]
    _say("sensitivity jacobian/H1/eig c1")
    ref = opipe.query(wl, keep_J=True, jacobian="sensitivity")
    out = run_query(ctx, grid_tuple(wl.grid), _dev_medium(wl.medium), wl.receivers,
                    wl.lo, wl.hi, wl.theta, wl.weights, sigma=ref["sigma"],
                    keep_nominal=True, keep_J=True, jacobian="sensitivity")
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    worst = 0.0
    for s in range(len(wl.theta)):
        check_receivers(out["nominal"][s].cpu().numpy(), ref["nominal"][s], TRACE_TOL,
                        what=f"nominal {s}")
        worst = max(worst, check_jacobian(out["J"][s].cpu().numpy(), ref["J"][s], SENS_TOL,
                                          what=f"sample {s}"))
    _say(f"  worst column rel err {worst:.3e}")
    H = out["H1"].cpu().numpy()
    relH = np.max(np.abs(H - ref["H1"]) / np.sqrt(np.abs(np.einsum("sii,sjj->sij",
                                                                   ref["H1"], ref["H1"]))))
    assert relH < 1e-4
    dkl = out["dkl"].cpu().numpy()
    assert np.max(np.abs(dkl - ref["dkl"])) <= NAT_TOL, np.abs(dkl - ref["dkl"])
    assert abs(float(out["eig"].cpu()[0]) - ref["eig"]) <= NAT_TOL


@pytest.mark.parametrize("case", ["nodal_gauss", "layered_per_receiver"])
def test_sensitivity_ragged(ctx, case):
    # uneven grids in one call, zero moment entries (allowed here), sources on
    # cell boundaries; per-receiver Hessians sum to the full one
    from paper_1502_07873_amd.query import grid_tuple
    _say(f"sensitivity ragged {case}")
    rng = np.random.default_rng(11)
    shapes = [(70, 45, 16.0, 260), (53, 61, 12.0, 311)]
    grids, meds, dmeds, recs, thetas = [], [], [], [], []
    for k, (nx, nz, h, nt) in enumerate(shapes):
        if case == "nodal_gauss":
            med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=60.0)
        else:
            med = synthetic.random_layers_medium(rng, nz, h, 3)
        grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), nt)
        x = (nx // 2 + (0.0 if k == 0 else 0.37)) * h
        z = (nz - 9) * h if k == 0 else 15 * h
        theta = np.array([x, z, 0.06, 12.0, 2e13, 0.0 if k == 0 else -1e13, 3e13])
        grids.append(grid)
        meds.append(med)
        dmeds.append(_dev_medium(med))
        recs.append(synthetic.equispaced_receivers(nx, 6))
        thetas.append(theta)
    stf = "gauss" if case == "nodal_gauss" else "gauss_deriv"
    if stf == "gauss":
        for th in thetas:
            th[3] = 60.0   # angular frequency of the Gaussian
    per = case == "layered_per_receiver"
    S = len(grids)
    R = len(recs[0])
    sigma = 0.05
    H1 = torch.empty((S, R, 7, 7) if per else (S, 7, 7), dtype=torch.float64, device="cuda")
    J = [torch.empty((g.nsteps + 1, R, 2, 7), dtype=torch.float64, device="cuda")
         for g in grids]
    status = torch.empty(S, dtype=torch.int32, device="cuda")
    ctx.jacobian_sensitivity([grid_tuple(g) for g in grids], dmeds, np.stack(thetas), recs,
                             sigma, H1, stf=stf, per_receiver=per, J=J, status=status)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    for s in range(S):
        _, Jr = elastic.jacobian_sensitivity(grids[s], meds[s], thetas[s], recs[s], stf)
        assert np.max(np.abs(Jr)) > 0
        check_jacobian(J[s].cpu().numpy(), Jr, SENS_TOL, what=f"{case} sample {s}")
        Hr = (laplace.hessian_h1_per_receiver(Jr, sigma) if per
              else laplace.hessian_h1(Jr, sigma))
        Hg = H1[s].cpu().numpy()
        d = np.sqrt(np.abs(np.diagonal(Hr.sum(0) if per else Hr)))
        assert np.max(np.abs(Hg - Hr)) <= 1e-4 * np.max(np.outer(d, d))


def test_sensitivity_agrees_with_central_differences(ctx):
    # both GPU Jacobians of one sample: equal up to the O(d^2) truncation of
    # the central differences and FP32 rounding of the deviation traces
    from paper_1502_07873_amd.query import grid_tuple, run_query
    wl = synthetic.config("c1", nsample=2)[0]
    _say("sensitivity vs central differences (GPU)")
    kw = dict(sigma=0.01, keep_J=True)
    g = grid_tuple(wl.grid)
    dm = _dev_medium(wl.medium)
    a = run_query(ctx, g, dm, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                  jacobian="sensitivity", **kw)
    # at rel_step 1e-4 the oracle's own truncation gap is <= 1.1e-5 on these
    # samples (1e-3 on the z column at rel_step 1e-3)
    b = run_query(ctx, g, dm, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                  rel_step=1e-4, jacobian="fd", **kw)
    torch.cuda.synchronize()
    for s in range(2):
        check_jacobian(b["J"][s].cpu().numpy(), a["J"][s].cpu().numpy(), JAC_TOL,
                       what=f"sample {s}")
    assert np.max(np.abs(a["dkl"].cpu().numpy() - b["dkl"].cpu().numpy())) <= NAT_TOL


def test_noise_sigma_peak_c1(ctx):
    from paper_1502_07873_amd.query import grid_tuple
    wl = synthetic.config("c1")[0]
    _say("noise sigma c1")
    s_gpu = ctx.noise_sigma_peak(grid_tuple(wl.grid), _dev_medium(wl.medium), wl.theta_bar)
    s_ref = elastic.noise_sigma(wl.grid, wl.medium, wl.theta_bar)
    assert abs(s_gpu - s_ref) <= 1e-5 * s_ref


def test_sigma_nominal_peak_mode(ctx):
    from paper_1502_07873_amd import eigseis
    from paper_1502_07873_amd.query import grid_tuple
    wl = synthetic.config("c1", nsample=3)[0]
    _say("sigma nominal-peak mode")
    g = grid_tuple(wl.grid)
    dm = _dev_medium(wl.medium)
    S = len(wl.theta)
    H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
    ctx.jacobian_fd([g] * S, [dm] * S, wl.theta, [wl.receivers] * S, 1e-3, H1,
                    sigma_mode=eigseis.SIGMA_NOMINAL_PEAK)
    torch.cuda.synchronize()
    for s in range(S):
        nominal, J = elastic.jacobian_literal(wl.grid, wl.medium, wl.theta[s], wl.receivers)
        sig = 1e-3 * np.max(np.abs(nominal))
        Href = laplace.hessian_h1(J, sig)
        ld_g = laplace.logdet_scaled(H1[s].cpu().numpy())[0]
        ld_r = laplace.logdet_scaled(Href)[0]
        assert abs(ld_g - ld_r) < 2e-3


def test_per_receiver_design_eval_and_greedy(ctx):
    from paper_1502_07873_amd import eigseis, make_prior
    from paper_1502_07873_amd.query import grid_tuple, run_query
    wl = synthetic.config("c1", nsample=4)[0]
    rec = np.array([3, 9, 17, 25, 32, 40, 47, 55, 60], dtype=np.int32)
    _say("per-receiver H1, design_eval, greedy")
    # oracle per-receiver Hessians on the candidate set
    H1r_ref = np.stack([opipe.sample_terms(
        synthetic.Workload("c1", wl.grid, wl.medium, rec, wl.lo, wl.hi, None, None),
        th, 0.5, per_receiver=True)[2] for th in wl.theta])
    out = run_query(ctx, grid_tuple(wl.grid), _dev_medium(wl.medium), rec, wl.lo, wl.hi,
                    wl.theta, wl.weights, sigma=0.5, per_receiver=True)
    torch.cuda.synchronize()
    H1r = out["H1"]
    Hg = H1r.cpu().numpy()
    scale = np.sqrt(np.abs(np.einsum("scii,scjj->scij", H1r_ref, H1r_ref)))
    assert np.max(np.abs(Hg - H1r_ref) / scale) < 1e-3
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    rng = np.random.default_rng(5)
    masks = (rng.random((6, len(rec))) < 0.5).astype(np.uint8)
    masks[0] = 1
    masks[1] = 0
    masks[1, 4] = 1
    eig_ref = laplace.design_eval(H1r_ref, masks, wl.theta, wl.weights, prior)
    eig_g = torch.empty(len(masks), dtype=torch.float64, device="cuda")
    ctx.design_eval(H1r, torch.as_tensor(masks, device="cuda"), make_prior(wl.lo, wl.hi),
                    wl.weights, eig_g, theta=wl.theta)
    torch.cuda.synchronize()
    eg = eig_g.cpu().numpy()
    ok = ~np.isnan(eig_ref)
    assert np.array_equal(ok, ~np.isnan(eg))
    assert np.max(np.abs(eg[ok] - eig_ref[ok])) <= NAT_TOL
    K = 5
    order = torch.empty(K, dtype=torch.int32, device="cuda")
    curve = torch.empty(K, dtype=torch.float64, device="cuda")
    ctx.design_greedy(H1r, make_prior(wl.lo, wl.hi), wl.weights, K, order, curve,
                      theta=wl.theta)
    torch.cuda.synchronize()
    og, cg = order.cpu().numpy(), curve.cpu().numpy()
    # every step: the pick is the argmax of the oracle's I on the same FP64
    # Hessians and the run's own prefix (ties only within 1e-9 relative), and
    # the oracle's own argmax on its Hessians wherever its best two
    # candidates are more than 2 NAT_TOL apart
    check_greedy(og, cg, Hg, wl.theta, wl.weights, prior, ref_H1r=H1r_ref,
                 ref_gap=2 * NAT_TOL)
    # the value of each chosen design on the oracle's Hessians
    masks = np.zeros((K, len(rec)), dtype=np.uint8)
    for k in range(K):
        masks[k, og[:k + 1]] = 1
    ref_curve = laplace.design_eval(H1r_ref, masks, wl.theta, wl.weights, prior)
    assert np.max(np.abs(cg - ref_curve)) <= NAT_TOL
    del eigseis


def test_alone_equals_in_batch(ctx):
    from paper_1502_07873_amd.query import grid_tuple, run_query
    wl = synthetic.config("c1", nsample=6)[0]
    _say("alone vs batch")
    g = grid_tuple(wl.grid)
    dm = _dev_medium(wl.medium)
    full = run_query(ctx, g, dm, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights, sigma=0.7)
    one = run_query(ctx, g, dm, wl.receivers, wl.lo, wl.hi, wl.theta[3:4], [1.0], sigma=0.7)
    torch.cuda.synchronize()
    assert torch.equal(full["H1"][3], one["H1"][0])
    assert float(full["dkl"][3]) == float(one["dkl"][0])


def test_edge_cases(ctx):
    from paper_1502_07873_amd import EigError
    from paper_1502_07873_amd.query import grid_tuple
    wl = synthetic.config("c1", nsample=1, grid_override=(40, 40, 0))[0]
    _say("edge cases")
    # zero steps: a single recorded level, all zero
    out = _forward(ctx, wl.grid, wl.medium, wl.theta, wl.receivers)
    assert out[0].shape == (1, len(wl.receivers), 2) and np.all(out[0] == 0)
    g1 = synthetic.Grid(40, 40, wl.grid.h, wl.grid.dt, 1)
    out = _forward(ctx, g1, wl.medium, wl.theta, wl.receivers)
    ref = elastic.forward(g1, wl.medium, wl.theta[0], wl.receivers)
    assert np.allclose(out[0], ref, rtol=1e-5, atol=0)
    dm = _dev_medium(wl.medium)
    g = grid_tuple(g1)
    tr = [torch.empty((2, 2, 2), dtype=torch.float32, device="cuda")]
    bad = wl.theta.copy()
    bad[0, 0] = wl.grid.h * 2.5     # stencil reaches the rigid left edge
    with pytest.raises(EigError):
        ctx.forward_solve_batch([g], [dm], bad, [np.array([3, 5], np.int32)], tr)
    with pytest.raises(EigError):   # repeated receiver
        ctx.forward_solve_batch([g], [dm], wl.theta, [np.array([3, 3], np.int32)], tr)
    with pytest.raises(EigError):   # receiver on the rigid corner
        ctx.forward_solve_batch([g], [dm], wl.theta, [np.array([0, 5], np.int32)], tr)
    H1 = torch.empty((1, 7, 7), dtype=torch.float64, device="cuda")
    th0 = wl.theta.copy()
    th0[0, 5] = 0.0                 # zero parameter: relative FD step undefined
    with pytest.raises(EigError):
        ctx.jacobian_fd([g], [dm], th0, [wl.receivers], 1.0, H1)
    # a singular Hessian is flagged, not factored
    from paper_1502_07873_amd import make_prior
    Hs = torch.zeros((2, 7, 7), dtype=torch.float64, device="cuda")
    Hs[0] = torch.eye(7, dtype=torch.float64)
    dkl = torch.empty(2, dtype=torch.float64, device="cuda")
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(2, dtype=torch.int32, device="cuda")
    ctx.laplace_eig(Hs, make_prior(wl.lo, wl.hi), [0.5, 0.5], dkl, eig, status=st)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, -4]
    assert np.isnan(float(eig.cpu()[0]))


def test_empty_batches(ctx):
    """Zero solves or zero samples: forward_solve_batch and jacobian_fd return
    without work; laplace_eig and the nested estimator, which average over
    samples, refuse an empty set."""
    from paper_1502_07873_amd import EigError, make_prior
    _say("empty batches")
    ctx.forward_solve_batch([], [], np.zeros((0, 7)), [], [])
    H1 = torch.empty((0, 7, 7), dtype=torch.float64, device="cuda")
    ctx.jacobian_fd([], [], np.zeros((0, 7)), [], 1.0, H1)
    torch.cuda.synchronize()
    prior = make_prior(-np.ones(7), np.ones(7))
    eig = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(EigError):
        ctx.laplace_eig(H1, prior, np.zeros(0), torch.empty(0, dtype=torch.float64,
                                                             device="cuda"), eig)
    g0 = torch.empty((0, 6), dtype=torch.float32, device="cuda")
    g = torch.zeros((5, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(EigError):
        ctx.nested_mc_eig(g0, g0, g, 0.1, torch.empty(0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("nsteps", [1, 2, 400, 9000, 13200])
def test_hessian_and_peak_for_any_element_count(ctx, nsteps):
    """A sample's (level, receiver) elements are summed in ranges of at least
    4096, at most 16 ranges: 10, 15 and 2005 elements make one range, 45005
    ten uneven ones, 66005 sixteen.  H1 in nominal-peak mode must equal
    sum J^T J / sigma^2 in FP64 over the Jacobian the same call returns, with
    sigma = rel x the exact maximum of its nominal traces (a source two nodes
    deep moves the surface in one step)."""
    from paper_1502_07873_amd import eigseis
    from paper_1502_07873_amd.query import grid_tuple
    wl = synthetic.config("c1", nsample=3, grid_override=(40, 40, nsteps))[0]
    _say(f"H1 reduction, {nsteps} steps")
    th = wl.theta.copy()
    th[:, 0] = [400.0, 410.0, 300.0]
    th[:, 1] = [41.0, 45.0, 55.0]
    th[:, 2] = [0.01, 0.012, 0.02]
    S, R = len(th), len(wl.receivers)
    g = grid_tuple(wl.grid)
    dm = _dev_medium(wl.medium)
    H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
    nominal = [torch.empty((nsteps + 1, R, 2), dtype=torch.float32, device="cuda")
               for _ in range(S)]
    J = [torch.empty((nsteps + 1, R, 2, 7), dtype=torch.float64, device="cuda")
         for _ in range(S)]
    status = torch.empty(S, dtype=torch.int32, device="cuda")
    rel = 1e-3
    ctx.jacobian_fd([g] * S, [dm] * S, th, [wl.receivers] * S, rel, H1, nominal=nominal, J=J,
                    status=status, sigma_mode=eigseis.SIGMA_NOMINAL_PEAK)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * S
    for s in range(S):
        peak = float(np.max(np.abs(nominal[s].cpu().numpy())))
        assert peak > 0.0
        sig = rel * peak
        Js = J[s].cpu().numpy().reshape(-1, 7)
        Href = (Js.T @ Js) / (sig * sig)
        Hg = H1[s].cpu().numpy()
        scale = np.sqrt(np.outer(np.diag(Href), np.diag(Href))) + 1e-300
        assert np.max(np.abs(Hg - Href) / scale) < 1e-12, (s, nsteps)
        assert np.array_equal(Hg, Hg.T)


@pytest.mark.parametrize("nsteps", [700, 333])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 23])
def test_stencil_variants_bitwise_identical(variant, nsteps, monkeypatch):
    # every layered-medium stencil variant computes the same arithmetic per
    # node, so the traces must agree bit for bit (and with the oracle)
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    rng = np.random.default_rng(21)
    nx, nz, h = 201, 83, 10.0
    med = synthetic.random_layers_medium(rng, nz, h, 4)
    grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), nsteps)
    lo, hi = synthetic.prior_box(grid)
    thetas = synthetic.draw_uniform(rng, lo, hi, 3)
    thetas[:, 2] = 0.1      # early wavelets: the signal reaches the surface in time
    rec = np.array([1, 50, 63, 64, 127, 128, 129, nx - 2], dtype=np.int32)
    _say(f"stencil variant {variant}, {nsteps} steps")
    outs = {}
    for v in (0, variant):
        monkeypatch.setenv("EIG_STENCIL_VARIANT", str(v))
        c = Context(0, 4 << 30)
        outs[v] = _forward(c, grid, med, thetas, rec)
        c.close()
    for s in range(len(thetas)):
        assert np.array_equal(outs[0][s], outs[variant][s]), s
        ref = elastic.forward(grid, med, thetas[s], rec)
        assert np.max(np.abs(ref)) > 1.0  # the wavefield has reached the receivers
        if nsteps % 2:
            assert np.max(np.abs(ref[-1])) > 0
        check_receivers(outs[variant][s], ref, TRACE_TOL, what=f"variant {variant} solve {s}")


@pytest.mark.parametrize("variant,nsteps", [(17, 333), (18, 333), (19, 333), (19, 334),
                                            (20, 333), (20, 334), (24, 333), (24, 334),
                                            (24, 335), (24, 336), (25, 333), (25, 336)])
def test_nodal_variants_bitwise_identical(variant, nsteps, monkeypatch):
    # the two-nodes-per-lane nodal kernels (one step per launch: 17, 18; two
    # steps: 19, 20, with odd and even step counts) and the four-step kernels
    # with the tile in LDS (24, 25: every step count mod 4) hand the per-node
    # update the same operands as the one-node kernel (variant 6): bit-for-bit
    # equal traces, across strip and tile boundaries, a ragged last strip, and the oracle's
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    rng = np.random.default_rng(23)
    nx, nz, h = 300, 97, 10.0
    med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=4, corr_len=80.0)
    grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), nsteps)
    lo, hi = synthetic.prior_box(grid)
    thetas = synthetic.draw_uniform(rng, lo, hi, 3)
    thetas[:, 2] = 0.1
    thetas[0, 0] = 126.5 * h    # source window across the first strip boundary
    rec = np.array([1, 2, 63, 64, 127, 128, 129, 255, 256, nx - 2], dtype=np.int32)
    _say(f"nodal stencil variant {variant}, {nsteps} steps")
    outs = {}
    for v in (6, variant):
        monkeypatch.setenv("EIG_STENCIL_VARIANT", str(v))
        c = Context(0, 4 << 30)
        outs[v] = _forward(c, grid, med, thetas, rec)
        assert c.get_option("last_variant") == v
        c.close()
    for s in range(len(thetas)):
        assert np.array_equal(outs[6][s], outs[variant][s]), s
        ref = elastic.forward(grid, med, thetas[s], rec)
        assert np.max(np.abs(ref)) > 1.0
        check_receivers(outs[variant][s], ref, TRACE_TOL, what=f"variant {variant} solve {s}")


@pytest.mark.parametrize("kind,nx,nz", [("layered", 65, 20), ("layered", 257, 113),
                                         ("nodal", 65, 26), ("nodal", 193, 50)])
def test_four_step_kernels_on_ragged_grids(kind, nx, nz, monkeypatch):
    # the four-step kernels (tile and halo in LDS) on grids that are not
    # multiples of their tiles: a last strip one column wide (nx = 65, 257,
    # 193), fewer free rows than a tile (nz = 20, 26) and a ragged last row
    # band; sources at the corners of the source box (near the sides and the
    # bottom), receivers on tile edges; every step count mod 4; bitwise equal
    # to the one-step kernel and the oracle's traces
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    rng = np.random.default_rng(nx * 1000 + nz)
    h = 10.0
    if kind == "nodal":
        med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=2, corr_len=40.0)
        fours, one = (24, 25), 6
    else:
        med = synthetic.random_layers_medium(rng, nz, h, 2)
        fours, one = (23,), 0
    rec = np.unique(np.r_[1, 56, 63, 64, 65, 127, 128, nx - 2])
    rec = rec[rec <= nx - 2].astype(np.int32)
    for nsteps in (201, 202, 203, 204):
        grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = synthetic.prior_box(grid)
        th = synthetic.draw_uniform(rng, lo, hi, 4)
        th[:, 0] = [lo[0], hi[0], lo[0], hi[0]]   # both sides
        th[:, 1] = [lo[1], hi[1], hi[1], lo[1]]   # mid-depth and the bottom
        th[:, 2] = 0.08
        _say(f"four-step kernels {fours} on {kind} {nx}x{nz}x{nsteps}")
        outs = {}
        for v in (one,) + fours:
            monkeypatch.setenv("EIG_STENCIL_VARIANT", str(v))
            c = Context(0, 1 << 30)
            outs[v] = _forward(c, grid, med, th, rec)
            assert c.get_option("last_variant") == v
            c.close()
        for v in fours:
            for s in range(len(th)):
                assert np.array_equal(outs[one][s], outs[v][s]), (v, nsteps, s)
        if nsteps == 203:
            for s in (1, 2):
                ref = elastic.forward(grid, med, th[s], rec)
                assert np.max(np.abs(ref)) > 0
                check_receivers(outs[fours[0]][s], ref, TRACE_TOL,
                                what=f"{kind} {nx}x{nz} solve {s}")


@pytest.mark.parametrize("variant", [20, 18, 24])
def test_nodal_tile_interleave_is_bitwise_neutral(variant, monkeypatch):
    # tiles of consecutive solves on one nodal medium run position-major in
    # sets of coef_interleave; the sets here are ragged (5 solves of one
    # length split 3 + 2, then 2 shorter ones, then 3 on a second medium and
    # grid), and every solve's traces equal the solve-major order's bit for
    # bit, and the oracle's
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import grid_tuple
    rng = np.random.default_rng(29)
    h = 10.0
    mA = synthetic.nodal_perturbed_medium(rng, 97, 300, h, nlayers=4, corr_len=80.0)
    mB = synthetic.nodal_perturbed_medium(rng, 70, 200, h, nlayers=3, corr_len=60.0)
    dt = synthetic.cfl_dt(h, max(mA.vp_max(), mB.vp_max()))
    gA1 = synthetic.Grid(300, 97, h, dt, 301)
    gA2 = synthetic.Grid(300, 97, h, dt, 250)
    gB = synthetic.Grid(200, 70, h, dt, 288)
    spec = [(gA1, mA)] * 5 + [(gA2, mA)] * 2 + [(gB, mB)] * 3
    thetas = np.concatenate([synthetic.draw_uniform(rng, *synthetic.prior_box(g), 1)
                             for g, _ in spec])
    thetas[:, 2] = 0.1
    rec = {id(gA1): np.array([1, 64, 128, 200, 298], dtype=np.int32),
           id(gB): np.array([1, 63, 64, 128, 198], dtype=np.int32)}
    rec[id(gA2)] = rec[id(gA1)]
    dmA, dmB = _dev_medium(mA), _dev_medium(mB)
    dms = [dmA if m is mA else dmB for _, m in spec]
    _say(f"nodal tile interleave, variant {variant}, 10 solves on two media")
    outs = {}
    monkeypatch.setenv("EIG_STENCIL_VARIANT", str(variant))
    for G in (1, 3):
        c = Context(0, 4 << 30)
        c.set_option("coef_interleave", G)
        tr = [torch.empty((g.nsteps + 1, len(rec[id(g)]), 2), dtype=torch.float32,
                          device="cuda") for g, _ in spec]
        c.forward_solve_batch([grid_tuple(g) for g, _ in spec], dms, thetas,
                              [rec[id(g)] for g, _ in spec], tr)
        torch.cuda.synchronize()
        assert c.get_option("last_variant") == variant
        c.close()
        outs[G] = [t.cpu().numpy().astype(np.float64) for t in tr]
    for s, (g, m) in enumerate(spec):
        assert np.array_equal(outs[1][s], outs[3][s]), s
    for s in (0, 4, 6, 9):
        g, m = spec[s]
        ref = elastic.forward(g, m, thetas[s], rec[id(g)])
        check_receivers(outs[3][s], ref, TRACE_TOL, what=f"interleaved solve {s}")


@pytest.mark.parametrize("tb,kind", [(3, "layered"), (4, "layered"), (4, "nodal")])
def test_multi_step_family_with_mixed_lengths_matches_one_step(tb, kind):
    # temporal_blocking = 3 or 4 through the normal (tuned) path: solves of
    # different lengths in one wave (running prefixes of tiles and halo
    # tiles), tails of every shorter length; bitwise equal to one step per
    # launch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import grid_tuple
    rng = np.random.default_rng(33)
    nx, nz, h = 300, 141, 10.0
    if kind == "nodal":
        med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=70.0)
    else:
        med = synthetic.random_layers_medium(rng, nz, h, 3)
    dt = synthetic.cfl_dt(h, med.vp_max())
    lens = [600, 431, 302, 601]
    grids = [synthetic.Grid(nx, nz, h, dt, n) for n in lens]
    lo, hi = synthetic.prior_box(grids[0])
    th = synthetic.draw_uniform(rng, lo, hi, len(lens))
    th[:, 2] = 0.08
    rec = np.array([1, 127, 128, 129, 255, 256, nx - 2], dtype=np.int32)
    _say(f"{tb}-step family, mixed lengths ({kind})")
    dm = _dev_medium(med)
    outs = []
    for t in (tb, 0):
        with Context(0, 4 << 30) as c:
            c.set_option("temporal_blocking", t)
            tr = [torch.empty((n + 1, len(rec), 2), dtype=torch.float32, device="cuda")
                  for n in lens]
            c.forward_solve_batch([grid_tuple(g) for g in grids], [dm] * len(lens), th,
                                  [rec] * len(lens), tr)
            torch.cuda.synchronize()
            outs.append([t.cpu().numpy() for t in tr])
            assert c.get_option("temporal_blocking") == (tb if t == tb else 1)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    assert np.max(np.abs(outs[0][2])) > 0


def test_graph_replays_match_direct_launches():
    # the time loop captured once and replayed: every replay, with eager work
    # and synchronisations in between, equals the direct-launch result
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import grid_tuple
    wl = synthetic.config("c1", nsample=4)[0]
    _say("graph capture and replays")
    g = grid_tuple(wl.grid)
    dm = _dev_medium(wl.medium)
    S = len(wl.theta)

    # the same destinations every time: they are part of the replayed launches
    tr = [torch.empty((wl.grid.nsteps + 1, len(wl.receivers), 2), dtype=torch.float32,
                      device="cuda") for _ in range(S)]

    def run(c):
        for t in tr:
            t.fill_(-1.0)
        c.forward_solve_batch([g] * S, [dm] * S, wl.theta, [wl.receivers] * S, tr)
        return tr

    with Context(0, 2 << 30) as c:
        c.set_option("graphs", 0)
        c.set_option("autotune", 0)
        ref = [t.cpu().numpy() for t in run(c)]
    with Context(0, 2 << 30) as c:
        c.set_option("autotune", 0)
        outs = []
        for rep in range(4):
            run(c)
            junk = torch.randn(1 << 20, device="cuda")   # eager work between replays
            junk.mul_(2.0).sum()
            torch.cuda.synchronize()
            outs.append([t.cpu().numpy() for t in tr])
        assert c.get_option("graph_captures") == 1
        assert c.get_option("graph_replays") == 3
    for o in outs:
        for a, b in zip(o, ref):
            assert np.array_equal(a, b)


def test_cache_sized_wave_chunks_match_one_wave():
    # a wave whose live fields exceed wave_cache_bytes runs as consecutive
    # chunks (more launches); every solve's traces are bitwise those of the
    # unsplit wave.  Mixed grids, lengths, media kinds and edge conditions.
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import grid_tuple
    rng = np.random.default_rng(41)
    cases = []
    medA = synthetic.random_layers_medium(rng, 141, 10.0, 3)
    dtA = synthetic.cfl_dt(10.0, medA.vp_max())
    for n in (400, 352, 400, 290, 401, 400, 333, 400, 398, 400):
        cases.append((synthetic.Grid(300, 141, 10.0, dtA, n), medA))
    medB = synthetic.random_layers_medium(rng, 70, 15.0, 2)
    dtB = synthetic.cfl_dt(15.0, medB.vp_max())
    for n in (260, 261, 199, 260, 260, 230, 260, 260, 261, 199, 260, 260, 230, 260):
        cases.append((synthetic.Grid(90, 70, 15.0, dtB, n), medB))
    medC = synthetic.random_layers_medium(rng, 80, 15.0, 2)
    dtC = synthetic.cfl_dt(15.0, medC.vp_max())
    for n in (240, 240, 211, 240, 240, 240, 211, 240):
        cases.append((synthetic.Grid(120, 80, 15.0, dtC, n, bc="absorbing"), medC))
    medN = synthetic.nodal_perturbed_medium(rng, 70, 90, 15.0)
    dtN = synthetic.cfl_dt(15.0, medN.vp_max())
    for n in (250, 250, 180, 250, 250, 250, 180, 250):
        cases.append((synthetic.Grid(90, 70, 15.0, dtN, n), medN))
    th = []
    for g, _ in cases:
        lo, hi = synthetic.prior_box(g)
        th.append(synthetic.draw_uniform(rng, lo, hi, 1)[0])
    th = np.stack(th)
    recs = [synthetic.random_receivers(rng, g.nx, 9) for g, _ in cases]
    dms = {id(m): _dev_medium(m) for _, m in cases}
    _say("cache-sized wave chunks vs one wave (40 mixed solves)")
    outs, launches = [], []
    # ~24 MB of live fields, mean 0.6 MB: a 10 MiB limit fits 16 solves,
    # giving three chunks (solves regrouped by kind, grid and length); two
    # steps per launch (four-step solves are never split for the cache)
    for lim in (0, 10 << 20):
        with Context(0, 2 << 30) as c:
            c.set_option("temporal_blocking", 2)
            c.set_option("wave_cache_bytes", lim)
            assert c.get_option("wave_cache_bytes") == lim
            tr = [torch.empty((g.nsteps + 1, len(r), 2), dtype=torch.float32, device="cuda")
                  for (g, _), r in zip(cases, recs)]
            c.stencil_stats(reset=True)
            c.forward_solve_batch([grid_tuple(g) for g, _ in cases],
                                  [dms[id(m)] for _, m in cases], th, recs, tr)
            torch.cuda.synchronize()
            launches.append(c.stencil_stats(reset=True)["launches"])
            outs.append([t.cpu().numpy() for t in tr])
    assert launches[1] > launches[0]
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
        assert np.isfinite(a).all()
    assert max(np.max(np.abs(a)) for a in outs[0]) > 0


@pytest.mark.parametrize("cache_bytes,tb", [(0, 4), (3 << 20, 4), (192 << 20, 4),
                                           (0, 2), (3 << 20, 2), (192 << 20, 2)])
def test_server_alone_equals_mix_and_matches_jacobian_path(ctx, cache_bytes, tb):
    # cache_bytes > 0: admission limited to that many live field bytes
    # (groups shrink to fit, queries wait for room) for kinds that take one
    # or two steps per launch (tb 2); tb 4: both kinds take four steps per
    # launch and are admitted by memory alone - the same results
    from paper_1502_07873_amd import eigseis, make_prior
    from paper_1502_07873_amd.query import grid_tuple, run_query
    _say(f"serving engine: alone vs mix (serve_cache_bytes {cache_bytes}, "
         f"temporal_blocking {tb})")
    default_cache = ctx.get_option("serve_cache_bytes")
    default_tb = ctx.get_option("temporal_blocking")
    ctx.set_option("serve_cache_bytes", cache_bytes)
    ctx.set_option("temporal_blocking", tb)
    wlA = synthetic.config("c1", nsample=5)[0]
    rng = np.random.default_rng(3)
    medB = synthetic.random_layers_medium(rng, 70, 15.0, 3)
    gB = synthetic.Grid(90, 70, 15.0, synthetic.cfl_dt(15.0, medB.vp_max()), 260)
    loB, hiB = synthetic.prior_box(gB)
    thB = synthetic.draw_uniform(rng, loB, hiB, 7)
    recB = synthetic.random_receivers(rng, 90, 11)
    dA, dB = _dev_medium(wlA.medium), _dev_medium(medB)
    medN = synthetic.nodal_perturbed_medium(rng, 60, 150, 15.0, nlayers=3, corr_len=80.0)
    gN = synthetic.Grid(150, 60, 15.0, synthetic.cfl_dt(15.0, medN.vp_max()), 240)
    loN, hiN = synthetic.prior_box(gN)
    thN = synthetic.draw_uniform(rng, loN, hiN, 3)
    recN = synthetic.random_receivers(rng, 150, 9)
    dN = _dev_medium(medN)

    def run(queries, stagger):
        srv = eigseis.Server(ctx, 2 << 30, group_samples=2)
        outs = []
        for k, (g, med, th, rec, lo, hi) in enumerate(queries):
            S = len(th)
            o = {"H1": torch.empty((S, 7, 7), dtype=torch.float64, device="cuda"),
                 "dkl": torch.empty(S, dtype=torch.float64, device="cuda"),
                 "eig": torch.empty(1, dtype=torch.float64, device="cuda")}
            o["id"] = srv.submit(grid_tuple(g), med, th, rec, make_prior(lo, hi),
                                 np.full(S, 1.0 / S), o["H1"], o["dkl"], o["eig"], 0.9)
            outs.append(o)
            srv.step(stagger)      # later queries join while earlier ones run
        left = list(outs)
        for _ in range(100000):
            if not left:
                break
            srv.step(64)
            torch.cuda.synchronize()
            left = [o for o in left if not srv.poll(o["id"])]
        assert not left
        srv.close()
        return outs

    qA = (wlA.grid, dA, wlA.theta, wlA.receivers, wlA.lo, wlA.hi)
    qB = (gB, dB, thB, recB, loB, hiB)
    qN = (gN, dN, thN, recN, loN, hiN)
    alone = run([qA], 0)
    mix = run([qB, qA, qB, qN], 37)
    assert torch.equal(alone[0]["H1"], mix[1]["H1"])
    assert torch.equal(alone[0]["dkl"], mix[1]["dkl"])
    assert torch.equal(alone[0]["eig"], mix[1]["eig"])
    assert torch.equal(mix[0]["H1"], mix[2]["H1"])
    ref = run_query(ctx, grid_tuple(wlA.grid), dA, wlA.receivers, wlA.lo, wlA.hi, wlA.theta,
                    np.full(5, 0.2), sigma=0.9)
    torch.cuda.synchronize()
    assert torch.equal(ref["H1"], alone[0]["H1"])
    assert torch.equal(ref["dkl"], alone[0]["dkl"])
    # a nodal-medium query in the mix (the server's four-step or two-node
    # nodal kernel)
    refN = run_query(ctx, grid_tuple(gN), dN, recN, loN, hiN, thN, np.full(3, 1.0 / 3),
                     sigma=0.9)
    torch.cuda.synchronize()
    assert torch.equal(refN["H1"], mix[3]["H1"])
    assert torch.equal(refN["dkl"], mix[3]["dkl"])
    ctx.set_option("serve_cache_bytes", default_cache)
    ctx.set_option("temporal_blocking", default_tb)


def test_sparse_quadrature_greedy_pipeline_c5_shape(ctx):
    # the c5 pipeline at a size the oracle finishes quickly: nodal random-
    # field medium, Gauss-Legendre sparse grid over the 7 parameters, one H_1
    # per candidate receiver, greedy selection; weights may be negative
    import paper_1502_07873_amd as pkg
    from paper_1502_07873_amd import make_prior
    from paper_1502_07873_amd.query import grid_tuple, run_query
    from oracle import smolyak
    wl = synthetic.config("c5", grid_override=(96, 64, 240))[0]
    cand = synthetic.candidate_receivers(wl.grid.nx, 21)
    nodes, w = pkg.sparse_grid_gl(7, 1, wl.lo, wl.hi)
    X, W = smolyak.sparse_grid(7, 1, wl.lo, wl.hi)
    assert np.allclose(nodes, X, rtol=0, atol=1e-9) and np.allclose(w, W, rtol=0, atol=1e-12)
    _say(f"c5-shaped pipeline: {len(w)} sparse-grid nodes, {len(cand)} candidates")
    sigma = 2.0
    out = run_query(ctx, grid_tuple(wl.grid), _dev_medium(wl.medium), cand, wl.lo, wl.hi,
                    nodes, w, sigma=sigma, per_receiver=True)
    torch.cuda.synchronize()
    H1r = out["H1"]
    wl_c = synthetic.Workload("c5", wl.grid, wl.medium, cand, wl.lo, wl.hi, None, None)
    H1r_ref = np.stack([opipe.sample_terms(wl_c, th, sigma, per_receiver=True)[2]
                        for th in X])
    scale = np.sqrt(np.abs(np.einsum("scii,scjj->scij", H1r_ref, H1r_ref)))
    assert np.max(np.abs(H1r.cpu().numpy() - H1r_ref) / scale) < 1e-3
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    K = 6
    order = torch.empty(K, dtype=torch.int32, device="cuda")
    curve = torch.empty(K, dtype=torch.float64, device="cuda")
    ctx.design_greedy(H1r, make_prior(wl.lo, wl.hi), w, K, order, curve, theta=nodes)
    torch.cuda.synchronize()
    og, cg = order.cpu().numpy(), curve.cpu().numpy()
    # I = sum_s w_s D_s with sparse-grid weights of both signs: a per-sample
    # error bound of NAT_TOL carries over as NAT_TOL * sum |w_s| (= 13 here)
    wtol = NAT_TOL * np.sum(np.abs(W))
    check_greedy(og, cg, H1r.cpu().numpy(), X, W, prior, ref_H1r=H1r_ref, ref_gap=2 * wtol)
    masks = np.zeros((K, len(cand)), dtype=np.uint8)
    for k in range(K):
        masks[k, og[:k + 1]] = 1
    assert np.max(np.abs(cg - laplace.design_eval(H1r_ref, masks, X, W, prior))) <= wtol
