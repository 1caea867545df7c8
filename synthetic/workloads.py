"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper (Section 4.1) studies a layered 2-D elastic half-space with a point
moment-tensor source, surface receivers and a uniform prior on the seven
source parameters.  No dataset is involved; every input here is drawn from
numpy's PCG64 generator with a fixed seed.

Coordinates: x runs from the left edge (node i at x = i*h) and z is depth
(node k at z = k*h, k = 0 is the free surface).  Parameter order follows the
paper's theta = (x_s, z_s, t_s, omega_s, m_xx, m_xz, m_zz) (Section 2.1); for
the Gaussian-derivative wavelet the frequency slot holds f in Hz.

Media are described by nodal density and Lame parameters (lambda, mu), the
quantities in the paper's stress law (Section 2.1); velocities are only the
way the workloads are specified.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PARAM_NAMES = ("x", "z", "t0", "f", "Mxx", "Mxz", "Mzz")
CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


@dataclasses.dataclass
class Grid:
    nx: int
    nz: int
    h: float
    dt: float
    nsteps: int
    bc: str = "rigid"   # left/right/bottom edges: "rigid" or "absorbing"

    @property
    def lx(self) -> float:
        return (self.nx - 1) * self.h

    @property
    def lz(self) -> float:
        return (self.nz - 1) * self.h

    @property
    def nt(self) -> int:
        """Recorded time levels t_m = m*dt, m = 0..nsteps."""
        return self.nsteps + 1


@dataclasses.dataclass
class Medium:
    """Nodal density and Lame parameters.

    kind == "layered": arrays of shape [nz] (properties vary with depth only).
    kind == "nodal":   arrays of shape [nz, nx].
    """
    kind: str
    rho: np.ndarray
    lam: np.ndarray
    mu: np.ndarray

    def nodal(self, nx: int):
        if self.kind == "nodal":
            return self.rho, self.lam, self.mu
        rep = lambda a: np.repeat(a[:, None], nx, axis=1)  # noqa: E731
        return rep(self.rho), rep(self.lam), rep(self.mu)

    def vp_max(self) -> float:
        return float(np.max(np.sqrt((self.lam + 2 * self.mu) / self.rho)))


@dataclasses.dataclass
class Workload:
    """One design query: a grid, a medium, receivers, a prior box, samples."""
    name: str
    grid: Grid
    medium: Medium
    receivers: np.ndarray          # int32 surface node indices (x index)
    lo: np.ndarray                 # prior box, paper parameter order
    hi: np.ndarray
    theta: Optional[np.ndarray]    # [S, 7] prior draws (None: quadrature)
    weights: Optional[np.ndarray]  # [S] Monte Carlo weights 1/S
    stf: str = "gauss_deriv"
    rel_step: float = 1e-4
    noise_rel: float = 1e-3
    smolyak_level: Optional[int] = None
    greedy_kmax: Optional[int] = None
    sigma: Optional[float] = None  # fixed noise std (else noise_rel x peak)

    @property
    def theta_bar(self) -> np.ndarray:
        return 0.5 * (self.lo + self.hi)


def cfl_dt(h: float, vp_max: float, cfl: float = 0.5) -> float:
    return cfl * h / vp_max


def _lame(rho, vp, vs):
    rho = np.asarray(rho, dtype=np.float64)
    vp = np.asarray(vp, dtype=np.float64)
    vs = np.asarray(vs, dtype=np.float64)
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu


def homogeneous_medium(nz: int, rho: float, vp: float, vs: float) -> Medium:
    lam, mu = _lame(rho, vp, vs)
    one = np.ones(nz)
    return Medium("layered", rho * one, lam * one, mu * one)


def layered_medium(nz: int, h: float, interfaces, rho, vp, vs) -> Medium:
    """Layer j holds nodes whose depth z = k*h satisfies
    interfaces[j-1] <= z < interfaces[j]; interfaces sit on nodes."""
    z = np.arange(nz) * h
    layer = np.searchsorted(np.asarray(interfaces, dtype=np.float64), z,
                            side="right")
    rho_n = np.asarray(rho, dtype=np.float64)[layer]
    lam_l, mu_l = _lame(rho, vp, vs)
    return Medium("layered", rho_n, np.asarray(lam_l)[layer],
                  np.asarray(mu_l)[layer])


def random_layers_medium(rng: np.random.Generator, nz: int, h: float,
                         nlayers: int, vp_lo=1500.0, vp_hi=4500.0,
                         rho=2500.0) -> Medium:
    lz = (nz - 1) * h
    interfaces = np.sort(rng.uniform(0.0, lz, nlayers - 1))
    vp = rng.uniform(vp_lo, vp_hi, nlayers)
    vs = vp / math.sqrt(3.0)
    return layered_medium(nz, h, interfaces, np.full(nlayers, rho), vp, vs)


def _gaussian_random_field(rng, nz, nx, h, corr_len):
    """Stationary field with squared-exponential covariance exp(-r^2/(2 l^2)),
    made by filtering white noise with a Gaussian kernel in Fourier space."""
    noise = rng.standard_normal((nz, nx))
    kz = np.fft.fftfreq(nz, d=h) * 2 * np.pi
    kx = np.fft.fftfreq(nx, d=h) * 2 * np.pi
    k2 = kz[:, None] ** 2 + kx[None, :] ** 2
    # kernel std s = l/sqrt(2) gives covariance exp(-r^2 / (2 l^2)).
    s = corr_len / math.sqrt(2.0)
    filt = np.exp(-0.5 * k2 * s * s)
    g = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    return g / np.max(np.abs(g))


def nodal_perturbed_medium(rng: np.random.Generator, nz: int, nx: int,
                           h: float, nlayers: int = 6, amp: float = 0.05,
                           corr_len: float = 200.0, rho: float = 2500.0,
                           ) -> Medium:
    """Random layers whose velocities are scaled by (1 + amp*g(x, z)),
    g a Gaussian random field normalised to max|g| = 1."""
    lz = (nz - 1) * h
    interfaces = np.sort(rng.uniform(0.0, lz, nlayers - 1))
    vp_l = rng.uniform(1500.0, 4500.0, nlayers)
    z = np.arange(nz) * h
    layer = np.searchsorted(interfaces, z, side="right")
    vp = vp_l[layer][:, None] * np.ones((1, nx))
    g = _gaussian_random_field(rng, nz, nx, h, corr_len)
    vp = vp * (1.0 + amp * g)
    vs = vp / math.sqrt(3.0)
    rho_n = np.full((nz, nx), rho)
    lam, mu = _lame(rho_n, vp, vs)
    return Medium("nodal", rho_n, lam, mu)


def prior_box(grid: Grid, t0=(0.1, 0.3), f=(5.0, 10.0), m=(1e13, 1e14)):
    """Uniform prior: source in the lower half of the box and at least 4
    cells away from the rigid sides and bottom."""
    h = grid.h
    lo = np.array([4 * h, 0.5 * grid.lz, t0[0], f[0], m[0], m[0], m[0]])
    hi = np.array([grid.lx - 4 * h, grid.lz - 4 * h, t0[1], f[1],
                   m[1], m[1], m[1]])
    return lo, hi


def draw_uniform(rng: np.random.Generator, lo, hi, n: int) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, lo.size))


def equispaced_receivers(nx: int, nr: int) -> np.ndarray:
    r = np.arange(nr)
    return np.floor((r + 1) * (nx - 1) / (nr + 1) + 0.5).astype(np.int32)


def candidate_receivers(nx: int, nc: int = 201) -> np.ndarray:
    c = np.arange(nc)
    return (4 + np.floor(c * (nx - 9) / (nc - 1) + 0.5)).astype(np.int32)


def random_receivers(rng: np.random.Generator, nx: int, nr: int) -> np.ndarray:
    """nr distinct non-corner surface nodes, sorted."""
    pick = rng.choice(np.arange(1, nx - 1), size=nr, replace=False)
    return np.sort(pick).astype(np.int32)


def _mc(theta):
    return np.full(theta.shape[0], 1.0 / theta.shape[0])


def config(name: str, nsample: Optional[int] = None, seed: Optional[int] = None,
           grid_override: Optional[tuple] = None) -> List[Workload]:
    """The five workloads, as lists of design queries.

    c1: 64^2, h=20, 400 steps, homogeneous, 5 receivers, 8 samples.
    c2: 512^2, h=10, 2000 steps, two layers, 21 receivers, 256 samples.
    c3: 4096 single-sample queries on grids {256,384,512}^2 with
        {1000,1500,2000} steps and random 4-layer media.
    c4: a stream of design queries (grid 256..1024, 500..4000 steps,
        5..101 random receivers, 64..512 samples); see serving_queries().
    c5: 2048x1024, 4000 steps, nodal 6-layer medium with a 5 % Gaussian
        random-field perturbation, 201 candidate receivers, sparse grid
        level 3, greedy to 40 receivers.
    grid_override = (nx, nz, nsteps) shrinks a config for tests.
    """
    idx = CONFIG_NAMES.index(name)
    rng = np.random.Generator(np.random.PCG64(idx if seed is None else seed))
    if name == "c1":
        nx, nz, nsteps, h = 64, 64, 400, 20.0
        if grid_override:
            nx, nz, nsteps = grid_override
        med = homogeneous_medium(nz, 2500.0, 3000.0, 1730.0)
        grid = Grid(nx, nz, h, cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = prior_box(grid)
        theta = draw_uniform(rng, lo, hi, nsample or 8)
        return [Workload("c1", grid, med, equispaced_receivers(nx, 5), lo, hi,
                         theta, _mc(theta))]
    if name == "c2":
        nx, nz, nsteps, h = 512, 512, 2000, 10.0
        if grid_override:
            nx, nz, nsteps = grid_override
        lz = (nz - 1) * h
        zint = rng.uniform(0.15, 0.45) * lz
        med = layered_medium(nz, h, [zint], [2500.0, 2500.0], [2000.0, 3500.0],
                             [1150.0, 2000.0])
        grid = Grid(nx, nz, h, cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = prior_box(grid)
        theta = draw_uniform(rng, lo, hi, nsample or 256)
        return [Workload("c2", grid, med, equispaced_receivers(nx, 21), lo, hi,
                         theta, _mc(theta))]
    if name == "c3":
        out = []
        for _ in range(nsample or 4096):
            n = int(rng.choice([256, 384, 512]))
            nsteps = int(rng.choice([1000, 1500, 2000]))
            nx = nz = n
            if grid_override:
                nx, nz, nsteps = grid_override
            h = 10.0
            med = random_layers_medium(rng, nz, h, 4)
            grid = Grid(nx, nz, h, cfl_dt(h, med.vp_max()), nsteps)
            lo, hi = prior_box(grid)
            theta = draw_uniform(rng, lo, hi, 1)
            out.append(Workload("c3", grid, med, equispaced_receivers(nx, 21),
                                lo, hi, theta, _mc(theta)))
        return out
    if name == "c4":
        return serving_queries(rng, nsample or 128, grid_override)
    if name == "c5":
        nx, nz, nsteps, h = 2048, 1024, 4000, 10.0
        if grid_override:
            nx, nz, nsteps = grid_override
        med = nodal_perturbed_medium(rng, nz, nx, h)
        grid = Grid(nx, nz, h, cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = prior_box(grid)
        return [Workload("c5", grid, med, candidate_receivers(nx, 201), lo, hi,
                         None, None, smolyak_level=3, greedy_kmax=40)]
    raise ValueError(name)


# The paper's model problem (Section 4.1): a layer over a half-space in the
# box [-10 km, 10 km] x [-15 km, 0], h = 200 m, dt = 0.025 s, T = 8 s,
# stress-free top and first-order absorbing sides and bottom, the Gaussian
# wavelet with frequency omega_s, C_eps = 1e-4 I.  Build frame: x = x_1 +
# 10 km, depth z = -x_2, so m_xz = -m_{x1 x2}.
LOH_NX, LOH_NZ, LOH_H, LOH_DT, LOH_NSTEPS = 101, 76, 200.0, 0.025, 320
LOH_X0 = 10000.0   # build x of the paper's x_1 = 0


def loh_medium(nz: int = LOH_NZ, h: float = LOH_H) -> Medium:
    # top layer: depth <= 1000 m (nodes down to the interface node included)
    return layered_medium(nz, h, [1000.0 + 0.5 * h], [2600.0, 2700.0],
                          [4000.0, 6000.0], [2000.0, 3464.0])


def loh_prior():
    """The paper's uniform prior, in the build frame and parameter order."""
    lo = np.array([LOH_X0 - 1000.0, 1000.0, 0.5, 3.0, 1e13, -1e15, 1e13])
    hi = np.array([LOH_X0 + 1000.0, 3000.0, 1.5, 5.0, 1e15, -1e13, 1e15])
    return lo, hi


def loh_prior_mean_paper() -> np.ndarray:
    """E[theta] of the paper's conditioning example, in the build frame."""
    return np.array([LOH_X0, 2000.0, 1.0, 4.0, 1e14, -1e14, 1e14])


def loh_receivers(x1) -> np.ndarray:
    """Surface node indices of receivers at paper coordinates x_1 (metres)."""
    return np.rint((np.asarray(x1, dtype=np.float64) + LOH_X0) / LOH_H).astype(np.int32)


def loh_scenarios():
    """Receiver arrays of the three scenarios (Section 4.5), as
    {scenario: [(label, node indices), ...]}."""
    out = {"I": [], "II": [], "III": []}
    for nr in (3, 5, 9, 17, 41, 81):                 # fixed span [-8 km, 8 km]
        d = 16000.0 / (nr - 1)
        out["I"].append((f"NR={nr},dR={d:g}", loh_receivers(-8000.0 + d * np.arange(nr))))
    for nr in range(1, 20, 2):                       # d_R = 1 km, symmetric
        out["II"].append((f"NR={nr}", loh_receivers(1000.0 * (np.arange(nr) - (nr - 1) / 2))))
    for d in range(200, 4001, 200):                  # 5 receivers, symmetric
        out["III"].append((f"dR={d}", loh_receivers(float(d) * (np.arange(5) - 2))))
    return out


def loh_candidates() -> np.ndarray:
    """Every surface node a scenario uses (x_1 in [-9 km, 9 km])."""
    return loh_receivers(np.arange(-9000.0, 9000.1, LOH_H))


def loh_workload(nsample: int = 256, seed: int = 5, nsteps: int = LOH_NSTEPS) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = Grid(LOH_NX, LOH_NZ, LOH_H, LOH_DT, nsteps, bc="absorbing")
    lo, hi = loh_prior()
    theta = draw_uniform(rng, lo, hi, nsample)
    return Workload("loh2d", grid, loh_medium(), loh_candidates(), lo, hi, theta, _mc(theta),
                    stf="gauss", sigma=0.01)


# Section 4.4: the Laplace method against the nested Monte Carlo estimator
# on the model problem with T = 1.25 s, two receivers at x_1 = -9 km and
# 1 km, x_1 = -1 km, t_s = 1 s, m_{x1x2} = m_{x2x2} = 1e14 known, and the
# depth, omega_s and m_{x1x1} inferred (the priors of Section 4.3).
LOH_NESTED_ACTIVE = (1, 3, 4)


def loh_nested_setup(nsteps: int = 50):
    """(grid, medium, receivers, lo, hi, template theta) of the comparison."""
    grid = Grid(LOH_NX, LOH_NZ, LOH_H, LOH_DT, nsteps, bc="absorbing")
    lo, hi = loh_prior()
    template = np.array([LOH_X0 - 1000.0, 2000.0, 1.0, 4.0, 1e14, -1e14, 1e14])
    return grid, loh_medium(), loh_receivers([-9000.0, 1000.0]), lo, hi, template


def loh_nested_draws(rng: np.random.Generator, n: int) -> np.ndarray:
    """n prior draws of the three inferred parameters, the rest fixed."""
    _, _, _, lo, hi, template = loh_nested_setup()
    th = np.repeat(template[None, :], n, axis=0)
    for j in LOH_NESTED_ACTIVE:
        th[:, j] = rng.uniform(lo[j], hi[j], n)
    return th


def serving_queries(rng: np.random.Generator, nquery: int,
                    grid_override: Optional[tuple] = None) -> List[Workload]:
    out = []
    for _ in range(nquery):
        n = int(rng.integers(256 // 64, 1024 // 64 + 1)) * 64
        nsteps = int(rng.integers(500, 4001))
        nr = int(rng.integers(5, 102))
        ns = int(rng.integers(64, 513))
        nx = nz = n
        if grid_override:
            nx, nz, nsteps = grid_override
            ns = max(1, ns // 64)
            nr = min(nr, nx - 2)
        h = 10.0
        med = random_layers_medium(rng, nz, h, 4)
        grid = Grid(nx, nz, h, cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = prior_box(grid)
        theta = draw_uniform(rng, lo, hi, ns)
        out.append(Workload("c4", grid, med, random_receivers(rng, nx, nr),
                            lo, hi, theta, _mc(theta)))
    return out


def c4_largest_query(seed: int = 44, nsample: int = 64) -> Workload:
    """A design query at the largest serving shape: 1024^2 grid (h = 10 m),
    4000 steps, random 4-layer medium, 101 random surface receivers,
    `nsample` prior draws."""
    rng = np.random.default_rng(seed)
    n, nt, h = 1024, 4000, 10.0
    med = random_layers_medium(rng, n, h, 4)
    grid = Grid(n, n, h, cfl_dt(h, med.vp_max()), nt)
    lo, hi = prior_box(grid)
    theta = draw_uniform(rng, lo, hi, nsample)
    rec = random_receivers(rng, n, 101)
    return Workload("c4", grid, med, rec, lo, hi, theta, _mc(theta))


def serving_stream(rng: np.random.Generator, nquery: int, n_range=(256, 512),
                   steps_range=(500, 2000), rec_range=(5, 101), sample_range=(16, 64),
                   h: float = 10.0, cover_travel: bool = True) -> List[Workload]:
    """A design-query stream shaped like c4 (random grid size, duration,
    receiver count and positions, sample count; random 4-layer media) with
    adjustable ranges, so a serving run can be sized to minutes.

    With cover_travel, a drawn duration is raised where needed to 1.5 x the
    vertical P travel time from the deepest prior source plus the latest
    wavelet: otherwise no wave reaches the surface, every H_1 is singular and
    the whole query only returns flags."""
    out = []
    for _ in range(nquery):
        n = int(rng.integers(n_range[0] // 64, n_range[1] // 64 + 1)) * 64
        nsteps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        nr = int(rng.integers(rec_range[0], rec_range[1] + 1))
        ns = int(rng.integers(sample_range[0], sample_range[1] + 1))
        med = random_layers_medium(rng, n, h, 4)
        grid = Grid(n, n, h, cfl_dt(h, med.vp_max()), nsteps)
        lo, hi = prior_box(grid)
        if cover_travel:
            vp = np.sqrt((med.lam + 2 * med.mu) / med.rho)
            travel = float(np.sum(h / vp[: int(hi[1] / h) + 1]))
            need = int(math.ceil((1.5 * travel + hi[2] + 2.0 / lo[3]) / grid.dt))
            grid.nsteps = max(nsteps, need)
        theta = draw_uniform(rng, lo, hi, ns)
        out.append(Workload("c4", grid, med, random_receivers(rng, n, min(nr, n - 2)),
                            lo, hi, theta, _mc(theta)))
    return out


def serving_head_of_line(seed: int = 9, nshort: int = 8, gap: float = 0.5):
    """A head-of-line stream at the serving workload's sizes: one long query
    (1024^2 grid, 4000 steps, 101 random receivers, 64 samples) arriving at
    t = 0 and `nshort` short ones (256^2 grid, 500..1000 steps raised where
    needed to cover the P travel time, 5..101 receivers, 64 samples)
    arriving `gap` seconds apart from t = gap.  Returns (workloads, arrival
    times)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lng = serving_stream(rng, 1, n_range=(1024, 1024), steps_range=(4000, 4000),
                         rec_range=(101, 101), sample_range=(64, 64), cover_travel=False)
    short = serving_stream(rng, nshort, n_range=(256, 256), steps_range=(500, 1000),
                           sample_range=(64, 64))
    arrivals = np.concatenate([[0.0], gap * (1 + np.arange(nshort))])
    return lng + short, arrivals


def poisson_arrivals(rng: np.random.Generator, n: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, n))
