"""Resident solves (grids whose two field levels fit one workgroup's LDS,
advanced through their whole time loop by one launch) against the tiled
kernels and the oracle: bit-for-bit equal traces and Hessians for
depth-only and nodal media, rigid and absorbing edges, forward, deviation,
sensitivity and dual solves, in waves that mix resident and tiled grids,
and at the LDS limit (160 KiB) and one column past it."""
import numpy as np
import pytest

import synthetic
from oracle import elastic
from _compare import check_receivers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-4


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


def _dev_medium(m):
    from paper_1502_07873_amd.query import device_medium
    return device_medium(m.kind, m.rho, m.lam, m.mu)


def _ctx(resident):
    from paper_1502_07873_amd import Context
    c = Context(0, 4 << 30)
    c.set_option("resident", 1 if resident else 0)
    return c


def _mixed_wave(seed=31):
    """(grid, medium, receivers) per solve: resident-sized depth-only and
    nodal grids with rigid and absorbing edges, ragged lengths, and one grid
    too large for LDS in the same wave."""
    rng = np.random.default_rng(seed)
    h = 10.0
    L1 = synthetic.random_layers_medium(rng, 64, h, 3)
    L2 = synthetic.random_layers_medium(rng, 76, h, 4)
    L3 = synthetic.random_layers_medium(rng, 97, h, 4)
    L4 = synthetic.random_layers_medium(rng, 25, h, 2)
    N1 = synthetic.nodal_perturbed_medium(rng, 50, 100, h, nlayers=3, corr_len=60.0)
    N2 = synthetic.nodal_perturbed_medium(rng, 60, 90, h, nlayers=3, corr_len=60.0)
    N3 = synthetic.nodal_perturbed_medium(rng, 20, 34, h, nlayers=2, corr_len=40.0)
    vmax = max(m.vp_max() for m in (L1, L2, L3, L4, N1, N2, N3))
    dt = synthetic.cfl_dt(h, vmax)
    out = []
    # 40 x 25 and 34 x 20: more row bands (1024 // (nx - 2)) than free rows,
    # so some bands are empty and the surface row is not in the first band
    for nx, nz, med, n, bc in ((64, 64, L1, 333, 0), (101, 76, L2, 320, 1), (300, 97, L3, 301, 0),
                               (100, 50, N1, 290, 0), (90, 60, N2, 311, 1), (40, 25, L4, 342, 1),
                               (34, 20, N3, 287, 0)):
        g = synthetic.Grid(nx, nz, h, dt, n, bc="absorbing" if bc else "rigid")
        rec = np.unique(np.r_[1, 2, 63, 64, 65, nx // 2, nx - 2])
        rec = rec[rec <= nx - 2].astype(np.int32)
        out.append((g, med, rec))
    return out


def _forward(ctx, spec, thetas):
    from paper_1502_07873_amd.query import grid_tuple
    tr = [torch.empty((g.nsteps + 1, len(r), 2), dtype=torch.float32, device="cuda")
          for g, _, r in spec]
    ctx.forward_solve_batch([grid_tuple(g) for g, _, _ in spec],
                            [_dev_medium(m) for _, m, _ in spec], thetas,
                            [r for _, _, r in spec], tr)
    torch.cuda.synchronize()
    return [t.cpu().numpy().astype(np.float64) for t in tr]


def _thetas(spec, seed):
    rng = np.random.default_rng(seed)
    th = np.concatenate([synthetic.draw_uniform(rng, *synthetic.prior_box(g), 1)
                         for g, _, _ in spec])
    # at most 20 rows deep (within each prior box): the wave reaches the
    # surface in time
    th[:, 1] = [min(20 * g.h, synthetic.prior_box(g)[1][1]) for g, _, _ in spec]
    th[:, 2] = 0.1
    return th


def test_forward_resident_equals_tiled_in_a_mixed_wave():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    spec = _mixed_wave()
    th = _thetas(spec, 5)
    _say("resident vs tiled: mixed wave of 7 grids (6 resident-sized)")
    outs = {}
    launches = {}
    for res in (True, False):
        c = _ctx(res)
        c.stencil_stats(reset=True)
        outs[res] = _forward(c, spec, th)
        launches[res] = c.stencil_stats(reset=True)["launches"]
        c.close()
    # resident: one launch per resident group plus the tiled grid's launches
    assert launches[True] < launches[False]
    for s, (g, m, rec) in enumerate(spec):
        assert np.array_equal(outs[True][s], outs[False][s]), s
        ref = elastic.forward(g, m, th[s], rec)
        assert np.max(np.abs(ref)) > 1.0
        check_receivers(outs[True][s], ref, TRACE_TOL, what=f"resident solve {s}")


@pytest.mark.parametrize("kind", ["layered", "nodal"])
def test_jacobians_resident_equal_tiled(kind):
    # deviation solves (jacobian_fd) and sensitivity solves
    # (jacobian_sensitivity), per receiver, on absorbing grids of the model
    # problem's size: H_1 bit for bit
    from paper_1502_07873_amd.query import grid_tuple
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    rng = np.random.default_rng(37)
    nx, nz, h = 101, 76, 10.0
    if kind == "nodal":
        med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=60.0)
    else:
        med = synthetic.random_layers_medium(rng, nz, h, 3)
    g = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), 240, bc="absorbing")
    lo, hi = synthetic.prior_box(g)
    th = synthetic.draw_uniform(rng, lo, hi, 3)
    th[:, 1] = 20 * h
    th[:, 2] = 0.08
    rec = np.array([1, 20, 50, 64, 99], dtype=np.int32)
    dm = _dev_medium(med)
    S, R = len(th), len(rec)
    _say(f"resident vs tiled jacobians ({kind}, absorbing {nx}x{nz}x{g.nsteps})")
    got = {}
    for res in (True, False):
        c = _ctx(res)
        for fn in ("jacobian_fd", "jacobian_sensitivity"):
            H = torch.empty((S, R, 7, 7), dtype=torch.float64, device="cuda")
            getattr(c, fn)([grid_tuple(g)] * S, [dm] * S, th, [rec] * S, 1.0, H,
                           per_receiver=True, stf="gauss")
            torch.cuda.synchronize()
            got[(res, fn)] = H.cpu().numpy()
        c.close()
    for fn in ("jacobian_fd", "jacobian_sensitivity"):
        assert np.all(np.isfinite(got[(True, fn)]))
        assert np.min(np.abs(got[(True, fn)][..., np.arange(7), np.arange(7)])) > 0
        assert np.array_equal(got[(True, fn)], got[(False, fn)]), fn


def test_theorem3_dual_solves_resident_equal_tiled():
    # the Theorem-3 estimator's dual solves inject receiver forces and record
    # the source window: every output bit for bit
    from paper_1502_07873_amd import make_prior
    from paper_1502_07873_amd.query import grid_tuple
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    rng = np.random.default_rng(41)
    nx, nz, h = 48, 44, 16.0
    med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=80.0)
    g = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), 260)
    lo, hi = synthetic.prior_box(g)
    th = synthetic.draw_uniform(rng, lo, hi, 2)
    rec = synthetic.equispaced_receivers(nx, 7)
    S = len(th)
    noise = rng.standard_normal((S, g.nsteps + 1, len(rec), 2)).astype(np.float32)
    dm = _dev_medium(med)
    _say("resident vs tiled: theorem-3 dual solves (nodal 48x44x260)")
    got = {}
    for res in (True, False):
        c = _ctx(res)
        nz_t = [torch.as_tensor(noise[s], device="cuda") for s in range(S)]
        H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
        H2 = torch.empty_like(H1)
        val = torch.empty(S, dtype=torch.float64, device="cuda")
        eig = torch.empty(1, dtype=torch.float64, device="cuda")
        st = torch.empty(S, dtype=torch.int32, device="cuda")
        th_hat = c.theorem3_eig([grid_tuple(g)] * S, [dm] * S, th, [rec] * S, nz_t, 0.05,
                                make_prior(lo, hi), np.full(S, 1.0 / S), H1, H2, val, eig, st,
                                iters=2)
        torch.cuda.synchronize()
        got[res] = (np.asarray(th_hat), H1.cpu().numpy(), H2.cpu().numpy(), val.cpu().numpy())
        c.close()
    for a, b in zip(got[True], got[False]):
        assert np.array_equal(a, b)


def test_resident_at_the_lds_limit_and_past_it():
    # depth-only 123 x 80: 2 levels x 8 B x 9840 nodes + 80 coefficient rows
    # of 64 B + 512 B of window weights = 163072 B of the 163840 B of LDS,
    # resident; 124 x 80 (164352 B) runs tiled; both equal the tiled kernels
    # and the oracle
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    rng = np.random.default_rng(43)
    h = 10.0
    med = synthetic.random_layers_medium(rng, 80, h, 3)
    dt = synthetic.cfl_dt(h, med.vp_max())
    for nx, want_res in ((123, True), (124, False)):
        g = synthetic.Grid(nx, 80, h, dt, 257, bc="absorbing")
        rec = np.array([1, 64, nx - 2], dtype=np.int32)
        spec = [(g, med, rec)] * 2
        th = _thetas(spec, 7)
        _say(f"resident limit: {nx}x80x257 absorbing")
        outs = {}
        for res in (True, False):
            c = _ctx(res)
            c.stencil_stats(reset=True)
            outs[res] = _forward(c, spec, th)
            st = c.stencil_stats(reset=True)
            if res:
                assert (st["launches"] == 1) == want_res, st
                assert (c.get_option("last_variant") == 21) == want_res
            c.close()
        for s in range(2):
            assert np.array_equal(outs[True][s], outs[False][s]), (nx, s)
        ref = elastic.forward(g, med, th[0], rec)
        check_receivers(outs[True][0], ref, TRACE_TOL, what=f"{nx}x80")
