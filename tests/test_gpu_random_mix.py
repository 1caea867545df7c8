"""Seeded random mixes of solves through one forward_solve_batch call, against
the oracle solve by solve: grid sizes on and off the 128-column strips,
depth-only and nodal media, rigid and absorbing edges, different lengths,
sources across strip boundaries and near the bottom, and a small
wave_cache_bytes so that the wave runs as many chunks (tuned variants, edge
waves, both nodal kernels).  Traces: relative L2 <= 1e-5 per solve.
"""
import numpy as np
import pytest

import synthetic
from _compare import check_receivers
from oracle import elastic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-5


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)


def _mix(seed, n):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        nx = int(rng.choice([40, 127, 128, 129, 200, 257]))
        nz = int(rng.integers(24, 90))
        h = float(rng.choice([10.0, 15.0]))
        if rng.random() < 0.35:
            med = synthetic.nodal_perturbed_medium(rng, nz, nx, h, nlayers=3, corr_len=60.0)
        else:
            med = synthetic.random_layers_medium(rng, nz, h, int(rng.integers(1, 4)))
        bc = "absorbing" if rng.random() < 0.4 else "rigid"
        nt = int(rng.integers(120, 400))
        grid = synthetic.Grid(nx, nz, h, synthetic.cfl_dt(h, med.vp_max()), nt, bc=bc)
        lo, hi = synthetic.prior_box(grid)
        th = synthetic.draw_uniform(rng, lo, hi, 1)[0]
        th[2] = 0.05
        if nx > 130 and rng.random() < 0.5:
            th[0] = (126.0 + rng.random() * 4.0) * h     # window across x = 128
        if rng.random() < 0.3:
            th[1] = (nz - 5.0 - rng.random()) * h        # window down to row nz-2
        rec = np.unique(np.concatenate([[1, nx - 2], rng.integers(1, nx - 1, 5)])).astype(np.int32)
        cases.append((grid, med, th, rec))
    return cases


@pytest.mark.parametrize("seed,tb", [(101, 2), (202, 2), (303, 4)])
def test_random_mix_in_small_chunks_matches_oracle(seed, tb):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    cases = _mix(seed, 48)
    _say(f"random mix seed {seed}: {[(g.nx, g.nz, g.nsteps, g.bc, m.kind) for g, m, _, _ in cases]}")
    dms = [device_medium(m.kind, m.rho, m.lam, m.mu) for _, m, _, _ in cases]
    tr = [torch.empty((g.nsteps + 1, len(r), 2), dtype=torch.float32, device="cuda")
          for g, _, _, r in cases]
    # live field bytes as the library counts them; a limit that 16.5 mean
    # solves fit splits the wave into three chunks
    live = [(4 if (g.bc == "rigid" and m.kind == "layered") else 2) * g.nz *
            (-(-g.nx // 128) * 128) * 8 for g, m, _, _ in cases]
    lim = int(16.5 * np.mean(live))
    assert sum(live) > 2 * lim
    with Context(0, 2 << 30) as c:
        # two steps per launch: every rigid solve counts towards the limit;
        # four (the default): rigid solves run unsplit, the rest in chunks
        c.set_option("temporal_blocking", tb)
        c.set_option("wave_cache_bytes", lim)
        c.stencil_stats(reset=True)
        c.forward_solve_batch([grid_tuple(g) for g, _, _, _ in cases], dms,
                              np.stack([t for _, _, t, _ in cases]), [r for _, _, _, r in cases],
                              tr)
        torch.cuda.synchronize()
        if tb == 2:
            assert c.stencil_stats()["launches"] > max(g.nsteps for g, _, _, _ in cases)
    for s, (g, m, th, r) in enumerate(cases):
        ref = elastic.forward(g, m, th, r)
        out = tr[s].cpu().numpy().astype(np.float64)
        assert np.abs(ref).max() > 0, s
        check_receivers(out, ref, TRACE_TOL, what=f"solve {s} {g.nx}x{g.nz} {g.bc} {m.kind}")
