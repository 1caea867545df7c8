"""Parity at the workloads' full sizes, through the C ABI in their launch
configurations:
  - the c2 Monte Carlo query (256 prior samples x 15 solves of 512x512 x
    2000 steps, 24-solve chunks in the last-level cache): one sample whose
    solves straddle a chunk boundary recomputed by the oracle, properties on
    all 256;
  - the whole c3 batch (61440 solves): two samples recomputed by the oracle;
  - one c5 sparse-grid node (2048 x 1024 x 4000, nodal medium, 201
    candidates) and one sample of the largest serving query (1024^2 x 4000,
    101 receivers) served by the engine, against the oracle's stored values
    (tests/golden/make_fullsize_golden.py: its 15 solves take minutes);
  - the c5 design search (589 nodes x 201 candidates x 40 greedy steps).
Traces and Jacobian columns are compared per receiver.  Tolerances: traces
relative L2 <= 1e-5, Jacobian columns <= 1e-3, scaled H_1 <= 2e-3 (what the
column bound implies), D^_KL <= 1e-3 nats; identical FP64 inputs 1e-9
relative.
"""
import importlib.util
import os

import numpy as np
import pytest

import synthetic
from _compare import check_greedy, check_jacobian, check_receivers, scaled_hessian_err
from oracle import laplace, pipeline as opipe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-5
JAC_TOL = 1e-3
NAT_TOL = 1e-3


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name, wl):
    """The oracle's stored values for a full-size case (written by
    tests/golden/make_fullsize_golden.py, which calls only the oracle), after
    checking that they were made from exactly these inputs."""
    spec = importlib.util.spec_from_file_location(
        "make_fullsize_golden", os.path.join(GOLDEN, "make_fullsize_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    d = np.load(os.path.join(GOLDEN, name))
    assert str(d["input_sha256"]) == mk.medium_digest(wl), "inputs changed since the golden"
    return {k: d[k] for k in d.files}


def test_c2_full_query_sampled_against_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query
    wl = synthetic.config("c2")[0]
    S = len(wl.theta)
    assert S == 256
    g = grid_tuple(wl.grid)
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    _say("c2 full query: 3840 solves of 512x512x2000 in the default launch configuration")
    with Context(0, 200 << 30) as ctx:
        sig = ctx.noise_sigma_peak(g, med, 0.5 * (wl.lo + wl.hi), wl.noise_rel)
        ctx.stencil_stats(reset=True)
        out = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                        sigma=sig, keep_nominal=True, keep_J=True)
        torch.cuda.synchronize()
        st = ctx.stencil_stats(reset=True)
        v = ctx.get_option("last_variant")
        steps = {15: 3, 16: 3, 23: 4}.get(v, 2)
        solves_per_launch = st["updates"] / st["launches"] / (512 * 512 * steps)
        # four steps per launch: the whole wave in every launch; two: 24-solve
        # chunks in the last-level cache
        assert solves_per_launch == pytest.approx(3840.0 if steps == 4 else 24.0)
        k = 137   # solves 2055..2069 (in 24-solve chunks, cut by the boundary at 2064)
        gpu = {"nominal": out["nominal"][k].cpu().numpy().astype(np.float64),
               "J": out["J"][k].cpu().numpy(), "H1": out["H1"].cpu().numpy(),
               "dkl": out["dkl"].cpu().numpy(), "eig": float(out["eig"].cpu()[0]),
               "status": out["status"].cpu().numpy(),
               "chol": out["chol_status"].cpu().numpy()}
        del out
        # the forward-sensitivity Jacobian (1 + 7 solves per sample, 2048
        # solves in cache chunks) gives the same D^_KL up to the central
        # differences' O(d^2) truncation, for every sample
        _say("c2 full query, forward-sensitivity Jacobian")
        outs = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                         sigma=sig, jacobian="sensitivity")
        torch.cuda.synchronize()
        assert int(outs["status"].abs().sum()) == 0
        dkl_sens = outs["dkl"].cpu().numpy()
    # properties of every sample
    assert (gpu["status"] == 0).all() and (gpu["chol"] == 0).all()
    assert np.isfinite(gpu["dkl"]).all()
    H = gpu["H1"]
    assert np.allclose(H, np.transpose(H, (0, 2, 1)), rtol=1e-12, atol=0)
    assert (np.diagonal(H, axis1=1, axis2=2) > 0).all()
    assert gpu["eig"] == pytest.approx(float(np.dot(wl.weights, gpu["dkl"])), rel=1e-12)
    assert np.max(np.abs(dkl_sens - gpu["dkl"])) <= NAT_TOL
    # the sampled sample against the oracle (same sigma)
    _say(f"oracle: sample {k} of the c2 query (15 solves)")
    ref = opipe.query(wl, theta=wl.theta[k:k + 1], weights=[1.0], sigma=sig, keep_J=True)
    check_receivers(gpu["nominal"], ref["nominal"][0], TRACE_TOL, what="c2 nominal")
    check_jacobian(gpu["J"], ref["J"][0], JAC_TOL, what="c2")
    assert abs(float(gpu["dkl"][k]) - float(ref["dkl"][0])) <= NAT_TOL
    assert scaled_hessian_err(H[k], ref["H1"][0]) <= 2 * JAC_TOL


def test_c3_full_batch_sampled_against_oracle():
    # the whole uneven batch (4096 samples x 15 solves of {256,384,512}^2 x
    # {1000,1500,2000} steps, per-sample media) in one jacobian_fd call, in
    # the default launch configuration (four steps per launch, one wave per
    # grid and length; with two steps, uniform cache chunks); two samples of
    # different grids recomputed by the oracle, properties on all
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wls = synthetic.config("c3")
    S = len(wls)
    assert S == 4096
    # candidates for the oracle check: 256^2 x 1000 and 384^2 x 1500 samples
    cands = [[40, 50, 60], [3, 9, 17]]
    assert all((wls[k].grid.nx, wls[k].grid.nsteps) == (256, 1000) for k in cands[0])
    assert all((wls[k].grid.nx, wls[k].grid.nsteps) == (384, 1500) for k in cands[1])
    grids = [grid_tuple(w.grid) for w in wls]
    media = [device_medium(w.medium.kind, w.medium.rho, w.medium.lam, w.medium.mu)
             for w in wls]
    theta = np.concatenate([w.theta for w in wls])
    recs = [w.receivers for w in wls]
    nominal = [None] * S
    J = [None] * S
    for k in cands[0] + cands[1]:
        g = wls[k].grid
        nominal[k] = torch.empty((g.nsteps + 1, len(recs[k]), 2), dtype=torch.float32,
                                 device="cuda")
        J[k] = torch.empty((g.nsteps + 1, len(recs[k]), 2, 7), dtype=torch.float64,
                           device="cuda")
    H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
    status = torch.empty(S, dtype=torch.int32, device="cuda")
    _say("c3 full batch: 61440 solves in one jacobian_fd call")
    with Context(0, 200 << 30) as ctx:
        ctx.stencil_stats(reset=True)
        ctx.jacobian_fd(grids, media, theta, recs, 1.0, H1, nominal=nominal, J=J,
                        status=status)
        torch.cuda.synchronize()
        launches = ctx.stencil_stats()["launches"]
        if ctx.get_option("last_variant") == 23:
            # nine grid and length classes (in one or two waves), at most
            # 2000 / 4 launches each per wave
            assert launches < 20000
        else:
            # cache chunks: unsplit, the waves would take ~1000 launches each
            assert launches > 100000
    st = status.cpu().numpy()
    Hg = H1.cpu().numpy()
    assert (st == 0).all()
    assert np.isfinite(Hg).all()
    assert np.allclose(Hg, np.transpose(Hg, (0, 2, 1)), rtol=1e-12, atol=0)
    diag = np.diagonal(Hg, axis1=1, axis2=2)
    assert (diag >= 0).all()
    # a deep source with the shortest record may never reach the surface:
    # its Jacobian and H_1 are exactly zero; most samples record signal
    seen = (diag > 0).all(axis=1)
    assert seen.mean() > 0.5
    _say(f"c3: {int(seen.sum())} of {S} samples record signal within their duration")
    picks = [next(k for k in group if seen[k]) for group in cands]
    for k in picks:
        _say(f"oracle: c3 sample {k} ({wls[k].grid.nx}^2 x {wls[k].grid.nsteps})")
        ref = opipe.query(wls[k], sigma=1.0, keep_J=True)
        check_receivers(nominal[k].cpu().numpy(), ref["nominal"][0], TRACE_TOL,
                        what=f"c3 sample {k} nominal")
        check_jacobian(J[k].cpu().numpy(), ref["J"][0], JAC_TOL, what=f"c3 sample {k}")
        assert scaled_hessian_err(Hg[k], ref["H1"][0]) <= 2 * JAC_TOL


def test_c5_full_size_node_against_oracle():
    # 2048 x 1024 x 4000 on the nodal random-field medium, the centre node of
    # the level-3 sparse grid, all 201 candidate receivers, in the launch
    # configuration of the workload (one 15-solve wave, two-node nodal
    # kernel): noise level, nominal traces and Jacobian columns per receiver
    # at sampled candidates, H_1 of every candidate and D^_KL of the whole
    # array against the oracle's stored values; then properties that hold at
    # any size (per-candidate H_1 sum to the whole-array H_1, the sensitivity
    # path, all nodal kernels bit for bit)
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wl = synthetic.config("c5")[0]
    gold = _golden("c5_node_fullsize.npz", wl)
    th = gold["theta"][None, :]
    sig = float(gold["sigma"])
    g = grid_tuple(wl.grid)
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    R = len(wl.receivers)
    nt = wl.grid.nsteps + 1
    _say("c5 full size: noise level, per-candidate H1 with traces and J vs the oracle")
    Hr = torch.empty((1, R, 7, 7), dtype=torch.float64, device="cuda")
    Ha = torch.empty((1, 7, 7), dtype=torch.float64, device="cuda")
    Hs = torch.empty((1, 7, 7), dtype=torch.float64, device="cuda")
    nom = torch.empty((nt, R, 2), dtype=torch.float32, device="cuda")
    J = torch.empty((nt, R, 2, 7), dtype=torch.float64, device="cuda")
    with Context(0, 64 << 30) as ctx:
        sig_gpu = ctx.noise_sigma_peak(g, med, wl.theta_bar, wl.noise_rel)
        ctx.jacobian_fd([g], [med], th, [wl.receivers], sig, Hr, per_receiver=True,
                        nominal=[nom], J=[J])
        ctx.jacobian_fd([g], [med], th, [wl.receivers], sig, Ha)
        ctx.jacobian_sensitivity([g], [med], th, [wl.receivers], sig, Hs)
        torch.cuda.synchronize()
    assert abs(sig_gpu - sig) <= TRACE_TOL * sig
    e_tr = check_receivers(nom.cpu().numpy()[:, gold["trace_cands"]], gold["nominal"],
                           TRACE_TOL, what="c5 nominal")
    e_j = check_jacobian(J.cpu().numpy()[:, gold["jac_cands"]], gold["J"], JAC_TOL, what="c5")
    Hr, Ha, Hs = Hr.cpu().numpy()[0], Ha.cpu().numpy()[0], Hs.cpu().numpy()[0]
    e_hr = max(scaled_hessian_err(Hr[r], gold["H1r"][r]) for r in range(R))
    assert e_hr <= 2 * JAC_TOL
    assert scaled_hessian_err(Ha, gold["H1"]) <= 2 * JAC_TOL
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    dkl, ok = laplace.dkl_hat(Ha, th[0], prior)
    assert ok
    _say(f"c5 full size: trace {e_tr:.2e}, J {e_j:.2e}, per-candidate H1 {e_hr:.2e}, "
         f"D_KL {abs(dkl - float(gold['dkl'])):.2e} nats")
    # D^_KL from the GPU's H_1 through the library's own laplace kernel
    from paper_1502_07873_amd import make_prior
    with Context(0, 1 << 30) as ctx:
        Hd = torch.as_tensor(Ha[None], device="cuda")
        dk = torch.empty(1, dtype=torch.float64, device="cuda")
        eg = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.laplace_eig(Hd, make_prior(wl.lo, wl.hi), [1.0], dk, eg, theta=th)
        torch.cuda.synchronize()
        assert abs(float(dk.cpu()[0]) - float(gold["dkl"])) <= NAT_TOL
    d = np.sqrt(np.diag(Ha))
    sc = np.outer(d, d)
    assert np.max(np.abs((Hr.sum(axis=0) - Ha) / sc)) <= 1e-12
    assert np.linalg.eigvalsh(Ha / sc).min() > 0
    assert np.max(np.abs((Hs - Ha) / sc)) <= 1e-3
    _say("c5 full size: nodal kernels 6, 17, 18, 19, 20, 24, 25 on one solve")
    outs = []
    for v in (6, 17, 18, 19, 20, 24, 25):
        tr = [torch.empty((wl.grid.nsteps + 1, R, 2), dtype=torch.float32, device="cuda")]
        with Context(0, 16 << 30) as ctx:
            ctx.set_option("stencil_variant", v)
            ctx.forward_solve_batch([g], [med], th, [wl.receivers], tr)
            torch.cuda.synchronize()
            assert ctx.get_option("last_variant") == v
        outs.append(tr[0].cpu().numpy())
    assert np.abs(outs[0]).max() > 0
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    assert np.array_equal(outs[0], nom.cpu().numpy())


def test_c4_largest_query_through_the_server_equals_jacobian_path():
    # the largest serving query shape (1024^2 grid, 4000 steps, 101 random
    # receivers, 64 samples = 960 solves): the engine's H_1, D^_KL and EIG
    # equal the jacobian_fd + laplace_eig path bit for bit (its samples are
    # larger than the cache limit, so memory alone admits them)
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context, eigseis, make_prior
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query
    wl = synthetic.c4_largest_query()
    grid, med, th, rec, lo, hi = wl.grid, wl.medium, wl.theta, wl.receivers, wl.lo, wl.hi
    gold = _golden("c4_sample_fullsize.npz", wl)
    k = int(gold["sample"])
    assert np.array_equal(th[k], gold["theta"])
    g = grid_tuple(grid)
    dm = device_medium(med.kind, med.rho, med.lam, med.mu)
    S = len(th)
    w = np.full(S, 1.0 / S)
    _say("c4 largest query: 960 solves of 1024^2 x 4000 through the server")
    with Context(0, 200 << 30) as ctx:
        srv = eigseis.Server(ctx, 120 << 30, group_samples=16)
        o = {"H1": torch.empty((S, 7, 7), dtype=torch.float64, device="cuda"),
             "dkl": torch.empty(S, dtype=torch.float64, device="cuda"),
             "eig": torch.empty(1, dtype=torch.float64, device="cuda")}
        qid = srv.submit(g, dm, th, rec, make_prior(lo, hi), w, o["H1"], o["dkl"], o["eig"], 0.5)
        for _ in range(100000):
            srv.step(400)
            torch.cuda.synchronize()
            if srv.poll(qid):
                break
        else:
            raise AssertionError("query did not complete")
        srv.close()
        _say("c4 largest query: jacobian_fd + laplace_eig")
        ref = run_query(ctx, g, dm, rec, lo, hi, th, w, sigma=0.5)
        torch.cuda.synchronize()
        assert torch.equal(ref["H1"], o["H1"])
        assert torch.equal(ref["dkl"], o["dkl"])
        assert torch.equal(ref["eig"], o["eig"])
        assert int(ref["status"].abs().sum()) == 0
        # one served sample against the oracle: H_1 and D^_KL as the server
        # returned them, and per receiver through jacobian_fd (the same
        # kernels; bitwise equal above)
        _say(f"c4 largest query: served sample {k} vs the oracle")
        assert float(gold["sigma"]) == 0.5
        assert scaled_hessian_err(o["H1"][k].cpu().numpy(), gold["H1"]) <= 2 * JAC_TOL
        assert abs(float(o["dkl"][k].cpu()) - float(gold["dkl"])) <= NAT_TOL
        nt = grid.nsteps + 1
        Hr = torch.empty((1, len(rec), 7, 7), dtype=torch.float64, device="cuda")
        nom = torch.empty((nt, len(rec), 2), dtype=torch.float32, device="cuda")
        J = torch.empty((nt, len(rec), 2, 7), dtype=torch.float64, device="cuda")
        ctx.jacobian_fd([g], [dm], th[k:k + 1], [rec], 0.5, Hr, per_receiver=True,
                        nominal=[nom], J=[J])
        torch.cuda.synchronize()
    e_tr = check_receivers(nom.cpu().numpy()[:, gold["trace_recs"]], gold["nominal"],
                           TRACE_TOL, what="c4 nominal")
    e_j = check_jacobian(J.cpu().numpy()[:, gold["jac_recs"]], gold["J"], JAC_TOL, what="c4")
    Hr = Hr.cpu().numpy()[0]
    e_hr = max(scaled_hessian_err(Hr[r], gold["H1r"][r]) for r in range(len(rec)))
    assert e_hr <= 2 * JAC_TOL
    assert np.array_equal(Hr.sum(axis=0) > 0, gold["H1"] > 0)
    _say(f"c4 served sample: trace {e_tr:.2e}, J {e_j:.2e}, per-receiver H1 {e_hr:.2e}")


def test_c5_greedy_design_at_full_size_against_oracle():
    # the c5 design search at its full size: 589 sparse-grid nodes (7
    # parameters, level 3, weights of both signs) x 201 candidate receivers,
    # 40 greedy steps.  The per-candidate Hessians are drawn on the host
    # (SPD, rank 4 plus a small ridge, candidate-dependent scale) and given
    # to both sides, so the FP64 arithmetic is all that differs: at every one
    # of the 40 steps the GPU's pick is the argmax of the oracle's I over all
    # remaining candidates on the GPU's prefix (ties only within 1e-9
    # relative), each reported value is that I within 1e-9 relative, and
    # design_eval on the 40 designs gives the oracle's I within 1e-9 relative
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context, make_prior
    from oracle import smolyak
    lo, hi = -np.ones(7), np.ones(7)
    X, W = smolyak.sparse_grid(7, 3, lo, hi)
    S, C, K = len(W), 201, 40
    assert S == 589
    _say(f"c5 greedy at full size: {S} nodes x {C} candidates, {K} steps")
    rng = np.random.default_rng(589)
    G = rng.standard_normal((S, C, 7, 4))
    scale = (0.2 + (np.arange(C) * 37 % C) / C) ** 2
    H1r = np.einsum("scik,scjk->scij", G, G) * scale[None, :, None, None] + \
        1e-2 * np.eye(7)[None, None]
    prior = laplace.uniform_prior(lo, hi)
    with Context(0, 16 << 30) as ctx:
        Hd = torch.as_tensor(H1r, device="cuda")
        order = torch.empty(K, dtype=torch.int32, device="cuda")
        curve = torch.empty(K, dtype=torch.float64, device="cuda")
        ctx.design_greedy(Hd, make_prior(lo, hi), W, K, order, curve, theta=X)
        torch.cuda.synchronize()
        order = order.cpu().numpy().astype(np.int64)
        curve = curve.cpu().numpy()
        # design_eval on the 40 designs the greedy search went through
        masks = np.zeros((K, C), dtype=np.uint8)
        for k in range(K):
            masks[k, order[:k + 1]] = 1
        ev = torch.empty(K, dtype=torch.float64, device="cuda")
        ctx.design_eval(Hd, torch.as_tensor(masks, device="cuda"), make_prior(lo, hi), W, ev,
                        theta=X)
        torch.cuda.synchronize()
        ev = ev.cpu().numpy()
    assert len(set(order.tolist())) == K and order.min() >= 0 and order.max() < C
    check_greedy(order, curve, H1r, X, W, prior, rel_tie=1e-9)
    ref = laplace.design_eval(H1r, masks, X, W, prior)
    assert np.all(np.abs(ev - ref) <= 1e-9 * np.abs(ref)), np.max(np.abs(ev - ref))
    assert np.all(np.abs(curve - ref) <= 1e-9 * np.abs(ref)), np.max(np.abs(curve - ref))
