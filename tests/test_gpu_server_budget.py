"""The serving engine under a small HBM budget: a query whose full sample
group does not fit is still admitted (groups shrink on an idle server), the
arena never holds more than its budget, results equal the jacobian_fd +
laplace_eig path bit for bit, and requests that cannot fit or that step the
source out of its forcing window are refused at submit."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


def _dev_medium(m):
    from paper_1502_07873_amd.query import device_medium
    return device_medium(m.kind, m.rho, m.lam, m.mu)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    c = Context(0, 4 << 30)
    yield c
    c.close()


def _query(seed=11, n=128, nsteps=300, nsample=20):
    rng = np.random.default_rng(seed)
    med = synthetic.random_layers_medium(rng, n, 10.0, 3)
    g = synthetic.Grid(n, n, 10.0, synthetic.cfl_dt(10.0, med.vp_max()), nsteps)
    lo, hi = synthetic.prior_box(g)
    th = synthetic.draw_uniform(rng, lo, hi, nsample)
    rec = synthetic.random_receivers(rng, n, 7)
    return g, med, th, rec, lo, hi


def test_small_budget_admits_shrunk_groups_within_the_arena(ctx):
    from paper_1502_07873_amd import eigseis, make_prior
    from paper_1502_07873_amd.query import grid_tuple, run_query
    g, med, th, rec, lo, hi = _query()
    dm = _dev_medium(med)
    S = len(th)
    budget = 64 << 20
    # a 16-sample group of this query needs ~130 MB: more than the arena
    srv = eigseis.Server(ctx, budget, group_samples=16)
    o = {"H1": torch.empty((S, 7, 7), dtype=torch.float64, device="cuda"),
         "dkl": torch.empty(S, dtype=torch.float64, device="cuda"),
         "eig": torch.empty(1, dtype=torch.float64, device="cuda")}
    _say(f"server with a {budget >> 20} MiB arena: {S} samples of {g.nx}^2 x {g.nsteps}")
    qid = srv.submit(grid_tuple(g), dm, th, rec, make_prior(lo, hi), np.full(S, 1.0 / S),
                     o["H1"], o["dkl"], o["eig"], 0.7)
    peak_seen = 0
    for _ in range(10000):
        srv.step(50)
        mem = srv.memory()
        assert mem["budget"] == budget
        assert mem["in_use"] <= budget
        peak_seen = max(peak_seen, mem["in_use"])
        torch.cuda.synchronize()
        if srv.poll(qid):
            break
    else:
        raise AssertionError("query never completed")
    mem = srv.memory()
    assert mem["in_use"] == 0
    assert peak_seen <= mem["peak"] <= budget
    assert mem["peak"] > budget // 2    # groups were as large as the arena allows
    srv.close()
    ref = run_query(ctx, grid_tuple(g), dm, rec, lo, hi, th, np.full(S, 1.0 / S), sigma=0.7)
    torch.cuda.synchronize()
    assert torch.equal(ref["H1"], o["H1"])
    assert torch.equal(ref["dkl"], o["dkl"])
    assert torch.equal(ref["eig"], o["eig"])


def test_short_query_behind_a_long_one_runs_first(ctx):
    # a long query (8 samples of 512^2 x 3000 steps: 31 million grid points
    # per launch, above the size at which one launch fills the device) is
    # running when a short one (4 samples of 128^2 x 400) arrives: the short
    # one runs at once and alone, finishing within its own launch count plus
    # one segment while the long one waits; both equal their runs alone
    from paper_1502_07873_amd import eigseis, make_prior
    from paper_1502_07873_amd.query import grid_tuple, run_query
    gL, mL, thL, rL, loL, hiL = _query(seed=21, n=512, nsteps=3000, nsample=8)
    gS, mS, thS, rS, loS, hiS = _query(seed=22, n=128, nsteps=400, nsample=4)
    dL, dS = _dev_medium(mL), _dev_medium(mS)

    def outputs(S):
        return {"H1": torch.empty((S, 7, 7), dtype=torch.float64, device="cuda"),
                "dkl": torch.empty(S, dtype=torch.float64, device="cuda"),
                "eig": torch.empty(1, dtype=torch.float64, device="cuda")}

    srv = eigseis.Server(ctx, 8 << 30, group_samples=8)
    oL, oS = outputs(8), outputs(4)
    _say("serving: a short query arriving behind a long one")
    qL = srv.submit(grid_tuple(gL), dL, thL, rL, make_prior(loL, hiL), np.full(8, 1 / 8),
                    oL["H1"], oL["dkl"], oL["eig"], 0.7)
    srv.step(100)
    qS = srv.submit(grid_tuple(gS), dS, thS, rS, make_prior(loS, hiS), np.full(4, 1 / 4),
                    oS["H1"], oS["dkl"], oS["eig"], 0.7)
    short_launches = (gS.nsteps + 1) // 2     # two steps per launch (depth-only media)
    used = 0
    while not srv.poll(qS):
        srv.step(20)
        torch.cuda.synchronize()
        used += 20
        assert used <= short_launches + 40, "the short query waited behind the long one"
    assert not srv.poll(qL)
    for _ in range(1000):
        srv.step(200)
        torch.cuda.synchronize()
        if srv.poll(qL):
            break
    else:
        raise AssertionError("long query never completed")
    srv.close()
    for g, dm, th, rec, lo, hi, o in ((gL, dL, thL, rL, loL, hiL, oL),
                                      (gS, dS, thS, rS, loS, hiS, oS)):
        ref = run_query(ctx, grid_tuple(g), dm, rec, lo, hi, th, np.full(len(th), 1 / len(th)),
                        sigma=0.7)
        torch.cuda.synchronize()
        assert torch.equal(ref["H1"], o["H1"])
        assert torch.equal(ref["dkl"], o["dkl"])


def test_submit_refuses_what_cannot_fit_or_leaves_the_window(ctx):
    from paper_1502_07873_amd import eigseis, make_prior
    from paper_1502_07873_amd.query import grid_tuple
    srv = eigseis.Server(ctx, 64 << 20, group_samples=4)
    out = (torch.empty((2, 7, 7), dtype=torch.float64, device="cuda"),
           torch.empty(2, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"))
    # one 1024^2 sample holds ~0.5 GB of fields: EIG_EBUDGET at submit
    g, med, th, rec, lo, hi = _query(n=1024, nsteps=10, nsample=2)
    _say("server submit: one sample larger than the arena")
    with pytest.raises(eigseis.EigError) as e:
        srv.submit(grid_tuple(g), _dev_medium(med), th, rec, make_prior(lo, hi),
                   np.full(2, 0.5), *out, 0.7)
    assert e.value.code == eigseis.EIG_EBUDGET
    # a relative step that moves the source by more than one cell (x_s =
    # 1280 m, rel_step 0.02: 25.6 m, two to three cells of 10 m; every
    # perturbed stencil stays inside the grid)
    g, med, th, rec, lo, hi = _query(n=256, nsteps=10, nsample=2)
    th[:, 0] = 1280.0
    th[:, 1] = 1800.0
    _say("server submit: deviation step beyond the forcing window")
    with pytest.raises(eigseis.EigError) as e:
        srv.submit(grid_tuple(g), _dev_medium(med), th, rec, make_prior(lo, hi),
                   np.full(2, 0.5), *out, 0.7, rel_step=0.02)
    assert e.value.code == eigseis.EIG_EINVAL
    assert "more than one cell" in str(e.value)
    assert srv.pending() == (0, 0)
    assert srv.memory()["peak"] == 0
    srv.close()
