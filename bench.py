#!/usr/bin/env python
"""Throughput of the Laplace-EIG hot path on one MI355X.

One step = one whole design query of the paper-shaped Monte Carlo workload:
512 x 512 grid (h = 10 m), 2000 leapfrog steps, two-layer medium, 21 surface
receivers, 256 prior samples -> noise level from the nominal solve at the
prior mean, 256 x (1 + 2*7) forward solves, central-difference Jacobians,
H_1, scaled Cholesky log-dets, D^_KL and the Monte Carlo EIG.  Inputs are
resident on the device before the timed region.

value = sample-EIG evaluations per second (D^_KL(theta_s) values, each from
15 solves + H_1 + log-det).  The stencil launches are timed live with HIP
events by the library (eig_ctx_stencil_stats) for the roofline figure.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("EIG evals/s and grid-pt updates/s (HBM GB/s % peak) at ≤1e-3 nat err; "
          "p50/p99")
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_FLOPS = 78.6e12   # published dense FP64 matrix rate
FP32_VECTOR_PEAK_FLOPS = 157.3e12  # published FP32 vector rate (packed FMA)
# vector issue: 256 CUs x 4 SIMDs x 16 lanes per clock at 2.4 GHz (a wave64
# instruction occupies a SIMD for 4 clocks), in lane-instructions per second
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
# FP32 operations of one depth-only grid-point update: the row sums and
# differences (4), 15 per component for the operator, 3 per component for
# the leapfrog combination
LAYERED_FLOPS_PER_UPDATE = 40
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "stencil_layered_c2_traffic.json")
NODAL_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "stencil_nodal_c5_traffic.json")
RESIDENT_RECORD = os.path.join(ROOT, "profiles", "stencil_resident_model_problem.json")
CSRC = os.path.join(ROOT, "paper_1502_07873_amd", "csrc")
# the kernel sources each counter record was taken on
LAYERED_SOURCES = ("stencil.hip", "node_update.h", "tile.h")
NODAL_SOURCES = ("nodal.hip", "node_update.h", "tile.h")
BLOCKED_SOURCES = ("blocked.hip", "node_update.h", "tile.h")   # variants 23, 24, 25
RESIDENT_SOURCES = ("resident.hip", "node_update.h", "ce.h")


def _sources_sha(*names):
    """sha256 over the named kernel sources, in order."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(CSRC, n), "rb").read())
    return h.hexdigest()


def _counter_record(path, sources, **want):
    """A committed rocprofv3 counter record, only if it was taken on these
    kernel sources and matches every `want` field."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != _sources_sha(*sources):
        return None
    for k, v in want.items():
        if rec.get(k) != v:
            return None
    return rec


def _measured_traffic(solves_per_launch, wave_cache_bytes, variant):
    """Bytes per stencil launch past the L2 caches (served by the last-level
    cache or HBM) from the committed rocprofv3 counter record, only if it was
    taken on these kernel sources, workload and wave size."""
    rec = _counter_record(TRAFFIC_RECORD, _kernel_sources(variant, LAYERED_SOURCES),
                          solves_per_launch=solves_per_launch, variant=variant,
                          wave_cache_bytes=wave_cache_bytes)
    return rec["traffic_bytes_per_launch"] if rec else None


# fields a four-step launch must move per update: each node's two levels
# read once and written once per four steps (the tiles' halos, which
# neighbouring tiles share, come mostly from L2)
BLOCKED_FLOOR_B = 32.0 / 4


def _kernel_sources(variant, tiled):
    """The sources of a stencil variant's kernel: `tiled` unless it is one of
    the four-step kernels with the tile in LDS."""
    return BLOCKED_SOURCES if variant in (23, 24, 25) else tiled


def _steps_per_launch(variant):
    """Leapfrog steps one launch of a stencil variant takes."""
    if variant in (15, 16):
        return 3
    if variant in (23, 24, 25):
        return 4
    return 2 if (9 <= variant <= 14 or variant in (19, 20)) else 1


CPU_SHARE = 16   # host cores a one-GPU machine grants a process


def _cpu_baseline(wl, theta_s, gpu):
    """The oracle, untuned, on one prior sample: its noise solve at the
    prior mean and its 15 Jacobian solves, 16 single-threaded solves spread
    over the host's CPU share (16 cores per GPU), then H_1 and D^_KL.  Also
    the error set against the GPU's outputs for that sample (gpu: nominal
    traces, J, H1, dkl of the same sample and sigma)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from oracle import elastic, laplace
    nproc = os.cpu_count() or 1
    threads = min(CPU_SHARE, nproc)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        fut = pool.submit(elastic.noise_sigma, wl.grid, wl.medium, wl.theta_bar, wl.noise_rel,
                          wl.stf)
        nominal, J = elastic.jacobian_literal(wl.grid, wl.medium, theta_s, wl.receivers,
                                              wl.rel_step, wl.stf, pool=pool)
        sigma = fut.result()
    H1 = laplace.hessian_h1(J, sigma)
    dkl, _ = laplace.dkl_hat(H1, theta_s, laplace.uniform_prior(wl.lo, wl.hi))
    t = time.perf_counter() - t0
    upd = 16.0 * wl.grid.nx * wl.grid.nz * wl.grid.nsteps
    Jg = gpu["J"]
    d = np.sqrt(np.abs(np.diag(H1)))

    def per_rec(a, b):
        ax = tuple(k for k in range(b.ndim) if k != 1)
        return float(np.max(np.sqrt(np.sum((a - b) ** 2, axis=ax)) /
                            np.sqrt(np.sum(b * b, axis=ax))))
    errors = {
        "trace_rel_l2": float(np.linalg.norm(gpu["nominal"] - nominal) / np.linalg.norm(nominal)),
        "trace_rel_l2_worst_receiver": per_rec(gpu["nominal"], nominal),
        "jacobian_col_rel_l2_max": float(max(np.linalg.norm(Jg[..., j] - J[..., j]) /
                                             np.linalg.norm(J[..., j]) for j in range(7))),
        "jacobian_col_rel_l2_worst_receiver": max(per_rec(Jg[..., j], J[..., j])
                                                  for j in range(7)),
        "scaled_hessian_max_abs": float(np.max(np.abs((gpu["H1"] - H1) / np.outer(d, d)))),
        "dkl_abs": abs(float(dkl) - float(gpu["dkl"])),
        "eig_abs": abs(float(dkl) - float(gpu["dkl"])),
        "sigma_rel": abs(gpu["sigma"] - sigma) / sigma,
        "sample": "prior sample 0 of the timed query (the oracle with its own sigma)"}
    return ({"value": 1.0 / t, "unit": "sample-EIG evals/s", "cores": threads,
             "host_nproc": nproc, "kind": "oracle", "updates_per_s": upd / t,
             "updates_per_s_per_core": upd / t / threads,
             "sample": f"1 prior sample of the timed workload: its noise solve and 15 Jacobian "
                       f"solves (512x512x2000, FP64), one thread each on {threads} threads "
                       f"(the box's CPU share of {CPU_SHARE} cores per GPU; the host shows "
                       f"{nproc}), then H_1 and D^_KL; {t:.1f} s wall"}, errors)


def _copy_rate(nbytes=4 << 30, reps=5):
    """GB/s (read + write) of a plain device-to-device copy of nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()   # later legs need the HBM back
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def _graph_gain(reps=20):
    """A launch-bound query (c1: 8 samples x 15 solves of 64^2 x 400 steps)
    repeated with the time loop replayed from a captured HIP graph and with
    direct launches; sample-EIG evals/s of each."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query
    wl = synthetic.config("c1")[0]
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    g = grid_tuple(wl.grid)
    out = {}
    for graphs in (1, 0):
        with Context(0, 4 << 30) as ctx:
            ctx.set_option("graphs", graphs)
            sig = ctx.noise_sigma_peak(g, med, wl.theta_bar, wl.noise_rel)
            for _ in range(3):   # tune, capture, replay once
                run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                          sigma=sig)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                              sigma=sig)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            out["graphs" if graphs else "direct"] = {
                "sample_eig_evals_per_s": reps * len(wl.theta) / t,
                "ms_per_query": 1e3 * t / reps,
                "graph_replays": ctx.get_option("graph_replays"),
                "eig": float(r["eig"].cpu()[0])}
    out["speedup"] = (out["graphs"]["sample_eig_evals_per_s"] /
                      out["direct"]["sample_eig_evals_per_s"])
    out["workload"] = "c1 query: 8 samples x 15 solves, 64x64 grid, 400 steps (launch-bound)"
    return out


def _copy_calibration(nbytes=4 << 30, reps=4):
    """A plain device-to-device copy of nbytes, reps times: the HBM counters
    of these dispatches should read nbytes fetched and nbytes written."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


SERVE_BUDGET = 250 << 30   # the serving workload's HBM budget


def _run_stream(ctx, wls, arrivals, overlap, budget=SERVE_BUDGET, group_samples=16,
                progress=False):
    """Serves design queries (synthetic workloads) arriving at the given
    offsets; sigma = 1e-3 x each sample's nominal peak.  Returns the queries
    with their times; progress prints a line as each query is submitted and
    done."""
    from paper_1502_07873_amd import eigseis
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    from paper_1502_07873_amd.serve import Query, serve
    qs = []
    for w, t in zip(wls, arrivals):
        med = device_medium(w.medium.kind, w.medium.rho, w.medium.lam, w.medium.mu)
        qs.append(Query(grid_tuple(w.grid), med, w.theta, w.receivers, w.lo, w.hi, w.weights,
                        w.noise_rel, eigseis.SIGMA_NOMINAL_PEAK, arrival=float(t)))
    srv = eigseis.Server(ctx, budget, group_samples=group_samples)
    index = {id(q): k for k, q in enumerate(qs)}

    def report(kind, q, t):
        print(f"[bench] serving: query {index[id(q)]} ({q.grid[0]}^2 x {q.grid[4]}, "
              f"{len(q.theta)} samples) {kind} at {t:.1f} s", flush=True)

    serve(srv, qs, launches_per_step=20, overlap=overlap,
          on_event=report if progress else None)
    mem = srv.memory()
    srv.close()
    return qs, mem


def _stream_stats(qs, mem, work):
    import numpy as np

    from paper_1502_07873_amd.serve import latency_stats
    st = latency_stats(qs)
    span = max(q.t_done for q in qs) - min(q.t_submit for q in qs)
    nsamp = sum(len(q.theta) for q in qs)
    flagged = sum(int((q.status != 0).sum()) + int((q.chol_status != 0).sum()) for q in qs)
    return {"queries": len(qs), "latency_p50_s": st["p50_s"], "latency_p99_s": st["p99_s"],
            "latency_mean_s": st["mean_s"], "span_s": span,
            "design_eig_evals_per_s": len(qs) / span, "sample_eig_evals_per_s": nsamp / span,
            "grid_pt_updates": float(np.sum(work)),
            "grid_pt_updates_per_s": float(np.sum(work)) / span, "samples": nsamp,
            "flagged_samples": flagged, "arena_budget_GB": mem["budget"] / 1e9,
            "arena_peak_GB": mem["peak"] / 1e9}


def _serving_head_of_line(ctx):
    """One long query (1024^2 x 4000, 64 samples: 4.0e12 updates) arriving
    first and eight short ones (256^2, ~1000-2000 steps, 64 samples) arriving
    every 0.5 s behind it, under both disciplines: continuous batching admits
    the short queries beside the long one; queue-only makes them wait."""
    import numpy as np

    import synthetic
    from paper_1502_07873_amd.serve import latency_stats
    wls, arr = synthetic.serving_head_of_line()
    work = np.array([15 * len(w.theta) * w.grid.nx * w.grid.nz * w.grid.nsteps for w in wls])
    out = {"workload": "head-of-line: 1 query of 1024^2 x 4000 steps, 101 receivers, 64 "
                       "samples at t=0, then 8 queries of 256^2 x 1249..1952 steps, 7..91 "
                       "receivers, 64 samples, every 0.5 s; 250 GB arena"}
    for overlap in (True, False):
        print(f"[bench] serving head-of-line ({'continuous' if overlap else 'queue-only'})",
              flush=True)
        qs, mem = _run_stream(ctx, wls, arr, overlap)
        d = _stream_stats(qs, mem, work)
        short = latency_stats(qs[1:])
        d.update({"short_latency_p50_s": short["p50_s"], "short_latency_p99_s": short["p99_s"],
                  "long_latency_s": qs[0].t_done - qs[0].arrival})
        out["continuous_batching" if overlap else "queue_only"] = d
    cb, qo = out["continuous_batching"], out["queue_only"]
    out["short_p50_speedup"] = qo["short_latency_p50_s"] / cb["short_latency_p50_s"]
    out["short_p99_speedup"] = qo["short_latency_p99_s"] / cb["short_latency_p99_s"]
    return out


def _serving_c4(ctx, updates_per_s, max_updates=1.2e13, load=0.8, seed=3, overlap=True,
                nquery=None):
    """Design queries drawn from the serving workload's full ranges (grids
    256..1024^2, 500..4000 steps, 5..101 random receivers, 64..512 samples,
    random 4-layer media, 250 GB arena), Poisson arrivals at `load` x the
    capacity implied by updates_per_s; the first queries of the stream up to
    max_updates grid-point updates (or nquery of them)."""
    import numpy as np

    import synthetic
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = synthetic.serving_queries(rng, 128)
    work = np.array([15 * len(w.theta) * w.grid.nx * w.grid.nz * w.grid.nsteps for w in pool])
    n = nquery or max(2, int(np.searchsorted(np.cumsum(work), max_updates, side="right")))
    wls, work = pool[:n], work[:n]
    rate = load * updates_per_s / work.mean()
    arr = synthetic.poisson_arrivals(rng, n, rate)
    print(f"[bench] serving stream at the serving workload's ranges: {n} queries, "
          f"{work.sum():.3g} updates ({'continuous' if overlap else 'queue-only'})", flush=True)
    qs, mem = _run_stream(ctx, wls, arr, overlap, progress=True)
    d = _stream_stats(qs, mem, work)
    d.update({"discipline": "continuous batching" if overlap else "queue only",
              "offered_load": load, "arrival_rate_per_s": rate,
              "workload": "serving ranges: N ~ U{256..1024 step 64}^2, steps ~ U{500..4000}, "
                          "N_R ~ U{5..101} random surface receivers, samples ~ U{64..512}, "
                          "random 4-layer media, 250 GB arena; sigma = 1e-3 x each sample's "
                          "nominal peak (samples whose wave never reaches the surface within "
                          "the record are flagged)",
              "grids": [int(w.grid.nx) for w in wls], "steps": [int(w.grid.nsteps) for w in wls],
              "samples_per_query": [len(w.theta) for w in wls]})
    return d


def _leg_roofline(st, bytes_note, bound="hbm"):
    """Stencil figures of one leg from the library's timing (eig_ctx_stencil_stats)."""
    ms = max(st["ms"], 1e-9)
    achieved = st["bytes"] / (ms * 1e-3) / 1e9
    return {"stencil_ms": st["ms"], "launches": st["launches"],
            "avg_launch_ms": st["ms"] / max(st["launches"], 1),
            "grid_pt_updates_per_s_stencil": st["updates"] / (ms * 1e-3),
            "roofline": {"bound": bound, "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "note": bytes_note}}


def _bench_c3(nsample=4096, oracle_check=True):
    """Uneven batching: nsample single-sample queries with grids from
    {256,384,512}^2 and 1000/1500/2000 steps, each with its own 4-layer
    medium, all 15*nsample solves in one jacobian_fd call, in its own
    context (the batch's workspace is ~214 GB).  One 256^2 x 1000 sample is
    recomputed by the oracle for the error fields."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import Context, eigseis
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wls = synthetic.config("c3", nsample=nsample)
    grids = [grid_tuple(w.grid) for w in wls]
    media = [device_medium(w.medium.kind, w.medium.rho, w.medium.lam, w.medium.mu) for w in wls]
    theta = np.concatenate([w.theta for w in wls])
    recs = [w.receivers for w in wls]
    # the sample the oracle checks: the first 256^2 x 1000 one whose wave
    # reaches the surface (the first of 40, 50, 60)
    picks = [k for k in (40, 50, 60) if k < nsample]
    nominal, J = [None] * nsample, [None] * nsample
    for k in picks:
        g = wls[k].grid
        nominal[k] = torch.empty((g.nsteps + 1, len(recs[k]), 2), dtype=torch.float32,
                                 device="cuda")
        J[k] = torch.empty((g.nsteps + 1, len(recs[k]), 2, 7), dtype=torch.float64,
                           device="cuda")
    H1 = torch.empty((nsample, 7, 7), dtype=torch.float64, device="cuda")
    status = torch.empty(nsample, dtype=torch.int32, device="cuda")
    updates = float(sum(15 * g[0] * g[1] * g[4] for g in grids))
    with Context(0, 230 << 30) as ctx:
        ctx.stencil_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.jacobian_fd(grids, media, theta, recs, 1.0, H1, nominal=nominal, J=J,
                        status=status)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = ctx.stencil_stats(reset=True)
        ws = ctx.workspace_bytes
        variant = ctx.get_option("last_variant")
    out = {"workload": f"uneven batch: {nsample} samples x 15 solves, grids "
                       "{256,384,512}^2, 1000/1500/2000 steps, per-sample 4-layer media",
           "solves": 15 * nsample, "seconds": t, "sample_eig_evals_per_s": nsample / t,
           "grid_pt_updates_per_s": updates / t, "variant_last": variant,
           "workspace_GB": ws / 1e9, "flagged": int((status != 0).sum())}
    four = _steps_per_launch(variant) == 4
    out.update(_leg_roofline(
        st, "24 B per grid-point update (read u^m, u^{m-1}, write u^{m+1}) over the stencil "
            "launch time, against the 8 TB/s HBM peak; " +
            ("four steps per launch with the tile in LDS, one wave per grid and length "
             "through HBM: the kernel moves about 8 B per update, so achieved can pass "
             "the peak" if four else
             "the waves run as cache-sized chunks, so the launches read and write the "
             "256 MB last-level cache (bound 'llc') and achieved may approach or pass the "
             "HBM figure"), bound="hbm" if four else "llc"))
    Hg = H1.cpu().numpy()
    seen = [k for k in picks if (np.diag(Hg[k]) > 0).all()]
    if oracle_check and seen:
        from oracle import pipeline as opipe
        k = seen[0]
        print(f"[bench] c3: oracle on sample {k} ({wls[k].grid.nx}^2 x {wls[k].grid.nsteps})",
              flush=True)
        ref = opipe.query(wls[k], sigma=1.0, keep_J=True, threads=CPU_SHARE)
        Jg, Jr = J[k].cpu().numpy(), ref["J"][0]
        d = np.sqrt(np.diag(ref["H1"][0]))
        out["errors"] = {
            "sample": k,
            "trace_rel_l2": float(np.linalg.norm(nominal[k].cpu().numpy() - ref["nominal"][0]) /
                                  np.linalg.norm(ref["nominal"][0])),
            "jacobian_col_rel_l2_max": float(max(np.linalg.norm(Jg[..., j] - Jr[..., j]) /
                                                 np.linalg.norm(Jr[..., j]) for j in range(7))),
            "scaled_hessian_max_abs": float(np.max(np.abs((Hg[k] - ref["H1"][0]) /
                                                          np.outer(d, d)))),
            "dkl_abs": None}
        dk_ref = float(ref["dkl"][0])
        # the GPU's own D^_KL of that sample through laplace_eig
        with Context(0, 1 << 30) as c2:
            dk = torch.empty(1, dtype=torch.float64, device="cuda")
            eg = torch.empty(1, dtype=torch.float64, device="cuda")
            c2.laplace_eig(H1[k:k + 1].contiguous(), eigseis.make_prior(wls[k].lo, wls[k].hi),
                           [1.0], dk, eg, theta=wls[k].theta)
            torch.cuda.synchronize()
            out["errors"]["dkl_abs"] = abs(float(dk.cpu()[0]) - dk_ref)
    del nominal, J, H1
    torch.cuda.empty_cache()
    return out


def _bench_c5(reduced_grid=(512, 256, 1000), full_nodes=2, kmax=40, pipeline=True,
              coef_interleave=None):
    """Sparse quadrature + greedy design: (a) the full 2048x1024x4000 nodal
    problem on `full_nodes` sparse-grid nodes, the first being the centre
    node whose oracle values are stored with the tests (throughput, roofline,
    errors); (b) the whole pipeline (589 level-3 nodes, 201 candidates,
    greedy to kmax) on a reduced grid, with the EIG-vs-count curve."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import Context, make_prior, sparse_grid_gl
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query
    out = {}
    wl = synthetic.config("c5")[0]
    nodes, w = sparse_grid_gl(7, 3, wl.lo, wl.hi)
    centre = 0.5 * (wl.lo + wl.hi)
    k0 = int(np.argmin(np.max(np.abs(nodes - centre) / (wl.hi - wl.lo), axis=1)))
    order = [k0] + [k for k in range(len(w)) if k != k0][:full_nodes - 1]
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    g = grid_tuple(wl.grid)
    gold_path = os.path.join(ROOT, "tests", "golden", "c5_node_fullsize.npz")
    gold = np.load(gold_path) if os.path.exists(gold_path) else None
    sigma = float(gold["sigma"]) if gold is not None else 1.0
    with Context(0, 64 << 30) as ctx:
        if coef_interleave:
            ctx.set_option("coef_interleave", coef_interleave)
        # warm: tune and grow the workspace on one node
        run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, nodes[order[:1]], [1.0],
                  sigma=sigma, per_receiver=True)
        torch.cuda.synchronize()
        ctx.stencil_stats(reset=True)
        t0 = time.perf_counter()
        r = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, nodes[order],
                      w[order], sigma=sigma, per_receiver=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = ctx.stencil_stats(reset=True)
        variant = ctx.get_option("last_variant")
        coef_interleave = ctx.get_option("coef_interleave")
        Hr = r["H1"].cpu().numpy()
        del r
        rk = None
        if gold is not None:
            # untimed: the centre node's 4000-step traces and Jacobian at the
            # receivers the oracle's stored values cover
            rk = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, nodes[order[:1]], [1.0],
                           sigma=sigma, per_receiver=True, keep_nominal=True, keep_J=True)
            torch.cuda.synchronize()
            nom0 = rk["nominal"][0].cpu().numpy()[:, gold["trace_cands"]].astype(np.float64)
            jac0 = rk["J"][0].cpu().numpy()[:, gold["jac_cands"]]
            del rk
    upd = 15 * full_nodes * wl.grid.nx * wl.grid.nz * wl.grid.nsteps
    pts = wl.grid.nx * wl.grid.nz
    shared = (24.0 * st["updates"] + 12.0 * pts * st["launches"]) / max(st["ms"], 1e-9) * 1e-6
    fs = {"grid": [wl.grid.nx, wl.grid.nz, wl.grid.nsteps],
          "sparse_grid_nodes_total": len(w), "nodes_run": full_nodes,
          "candidates": len(wl.receivers), "seconds": t, "variant_last": variant,
          "grid_pt_updates_per_s": upd / t, "sample_eig_evals_per_s": full_nodes / t,
          "projected_full_query_minutes": len(w) * t / full_nodes / 60}
    leg = _leg_roofline(st, "")
    avg_ms = leg["avg_launch_ms"]
    solves_per_launch = round(st["updates"] / max(st["launches"], 1) /
                              (pts * _steps_per_launch(variant)))
    rec = _counter_record(NODAL_TRAFFIC_RECORD, _kernel_sources(variant, NODAL_SOURCES),
                          variant=variant, solves_per_launch=solves_per_launch,
                          coef_interleave=coef_interleave)
    traffic = rec["traffic_bytes_per_launch"] if rec else None
    trate = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
    copy_gbs = _copy_rate()
    leg["roofline"] = {
        "bound": "hbm", "achieved": shared, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": shared / HBM_PEAK_GBS, "traffic": traffic, "traffic_rate_GBs": trate,
        "copy_GBs_measured": copy_gbs,
        "frac_of_copy": trate / copy_gbs if trate else None,
        "achieved_36B_per_update_GBs": 36.0 * st["updates"] / (max(st["ms"], 1e-9) * 1e-3) / 1e9,
        "note": "achieved: 24 B of fields per grid-point update plus the medium's 12 B of "
                "nodal lambda, mu, dt^2/(rho h^2) per grid point once per launch (the "
                f"{solves_per_launch} solves of a launch share one medium); the 36 B-per-"
                "update unit (achieved_36B_per_update_GBs) counts those coefficients once "
                "per solve and so overstates the bytes.  traffic: bytes per launch past L2 "
                "(FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the counter record; "
                "frac_of_copy: that rate over a plain 4 GiB copy measured here"}
    fs.update(leg)
    if gold is not None:
        from oracle import laplace
        H = Hr[0].sum(axis=0)
        Hgold = gold["H1"]
        d = np.sqrt(np.diag(Hgold))
        dk, _ = laplace.dkl_hat(H, nodes[k0], laplace.uniform_prior(wl.lo, wl.hi))
        dr = np.sqrt(np.abs(np.einsum("rii->ri", gold["H1r"])))
        def per_rec(a, b):
            # per-receiver relative L2 over levels (and components, columns)
            ax = tuple(k for k in range(b.ndim) if k != 1)
            nb = np.sqrt(np.sum(b * b, axis=ax))
            nd = np.sqrt(np.sum((a - b) ** 2, axis=ax))
            keep = nb >= 1e-2 * nb.max()
            return float(np.max(nd[keep] / nb[keep]))
        fs["errors"] = {
            "node": "centre of the level-3 sparse grid (all parameters at their prior mean)",
            "trace_rel_l2_per_receiver_max": per_rec(nom0, gold["nominal"]),
            "jacobian_rel_l2_per_receiver_max": max(
                per_rec(jac0[..., j].astype(np.float64), gold["J"][..., j].astype(np.float64))
                for j in range(7)),
            "trace_levels": int(gold["nominal"].shape[0]),
            "scaled_hessian_max_abs": float(np.max(np.abs((H - Hgold) / np.outer(d, d)))),
            "per_candidate_scaled_hessian_max_abs": float(np.max(
                np.abs(Hr[0] - gold["H1r"]) / (dr[:, :, None] * dr[:, None, :]))),
            "dkl_abs": abs(dk - float(gold["dkl"])),
            "reference": "oracle values stored by tests/golden/make_fullsize_golden.py"}
    out["full_size"] = fs
    if not pipeline:
        return out
    wr = synthetic.config("c5", grid_override=reduced_grid)[0]
    nodes, w = sparse_grid_gl(7, 3, wr.lo, wr.hi)
    medr = device_medium(wr.medium.kind, wr.medium.rho, wr.medium.lam, wr.medium.mu)
    gr = grid_tuple(wr.grid)
    with Context(0, 64 << 30) as ctx:
        sigma = ctx.noise_sigma_peak(gr, medr, wr.theta_bar, wr.noise_rel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = run_query(ctx, gr, medr, wr.receivers, wr.lo, wr.hi, nodes, w, sigma=sigma,
                      per_receiver=True)
        order = torch.empty(kmax, dtype=torch.int32, device="cuda")
        curve = torch.empty(kmax, dtype=torch.float64, device="cuda")
        ctx.design_greedy(r["H1"], make_prior(wr.lo, wr.hi), w, kmax, order, curve, theta=nodes)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    cv = curve.cpu().numpy()
    ks = np.arange(1, kmax + 1)
    ok = np.isfinite(cv)
    slope = float(np.polyfit(np.log(ks[ok][4:]), cv[ok][4:], 1)[0]) if ok.sum() > 6 else None
    out["reduced_pipeline"] = {"grid": list(reduced_grid), "sparse_grid_nodes": len(w),
                               "solves": 15 * len(w), "candidates": len(wr.receivers),
                               "greedy_kmax": kmax, "seconds": t,
                               "order": order.cpu().numpy().tolist(),
                               "eig_curve": [float(x) for x in cv],
                               "slope_d_eig_d_log_k": slope,
                               "note": "Laplace EIG grows ~ (N_theta/2) log k for large "
                                       "k when H1 grows in proportion to receiver count"}
    return out


def _bench_c5_full_query(batch=30, kmax=40):
    """The whole c5 query at full size: per-candidate H_1 on all 589 level-3
    sparse-grid nodes of the 2048 x 1024 x 4000 nodal problem (8835 solves,
    in batches of `batch` nodes, progress printed per batch), then greedy
    design over the 201 candidates to kmax receivers."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import Context, make_prior, sparse_grid_gl
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query
    wl = synthetic.config("c5")[0]
    nodes, w = sparse_grid_gl(7, 3, wl.lo, wl.hi)
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    g = grid_tuple(wl.grid)
    R, S = len(wl.receivers), len(w)
    H = torch.empty((S, R, 7, 7), dtype=torch.float64, device="cuda")
    flagged = 0
    with Context(0, 64 << 30) as ctx:
        t0 = time.perf_counter()
        sigma = ctx.noise_sigma_peak(g, med, wl.theta_bar, wl.noise_rel)
        for a in range(0, S, batch):
            b = min(S, a + batch)
            r = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, nodes[a:b], w[a:b],
                          sigma=sigma, per_receiver=True)
            H[a:b] = r["H1"]
            flagged += int(r["status"].ne(0).sum())
            torch.cuda.synchronize()
            print(f"[bench] c5 full query: nodes {b}/{S}, {time.perf_counter() - t0:.1f} s",
                  flush=True)
        t_solve = time.perf_counter() - t0
        order = torch.empty(kmax, dtype=torch.int32, device="cuda")
        curve = torch.empty(kmax, dtype=torch.float64, device="cuda")
        t1 = time.perf_counter()
        ctx.design_greedy(H, make_prior(wl.lo, wl.hi), w, kmax, order, curve, theta=nodes)
        torch.cuda.synchronize()
        t_greedy = time.perf_counter() - t1
        st = ctx.stencil_stats(reset=True)
    upd = 15.0 * S * wl.grid.nx * wl.grid.nz * wl.grid.nsteps
    cv = curve.cpu().numpy()
    return {"workload": "c5 at full size: 2048x1024x4000 nodal medium, level-3 sparse grid "
                        "(589 nodes, 8835 solves), per-candidate H_1 over 201 receivers, "
                        f"greedy to {kmax}",
            "seconds_solves_and_h1": t_solve, "seconds_greedy": t_greedy,
            "grid_pt_updates_per_s": upd / t_solve, "sigma": sigma,
            "flagged_nodes": flagged, "stencil_launches": st["launches"],
            "order": order.cpu().numpy().tolist(), "eig_curve": [float(x) for x in cv],
            "eig_first_last": [float(cv[0]), float(cv[-1])]}


def _bench_model(nmc=10000, ncheck=2):
    """The paper's model problem (Section 4.1, absorbing edges, 91 candidate
    receivers): per-receiver H_1 for nmc Monte Carlo samples by central
    differences (15 solves each) and by forward sensitivities (8 solves),
    every Section 4.5 scenario design's EIG from them, and the oracle's
    per-receiver H_1 and D_KL on ncheck samples.  The 101 x 76 grid fits one
    workgroup's LDS, so each solve runs resident (fields never in HBM): the
    roofline is the FP32 vector rate."""
    import numpy as np
    import torch

    import synthetic
    from oracle import laplace
    from oracle import pipeline as opipe
    from paper_1502_07873_amd import Context, make_prior
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wl = synthetic.loh_workload(nmc)
    g = grid_tuple(wl.grid)
    R = len(wl.receivers)
    pos = {int(ix): c for c, ix in enumerate(wl.receivers)}
    designs = [(scen, lab, idx) for scen, ds in synthetic.loh_scenarios().items()
               for lab, idx in ds]
    masks = np.zeros((len(designs), R), dtype=np.uint8)
    for q, (_, _, idx) in enumerate(designs):
        masks[q, [pos[int(i)] for i in idx]] = 1
    prior = make_prior(wl.lo, wl.hi)
    out = {"grid": [wl.grid.nx, wl.grid.nz, wl.grid.nsteps],
           "edges": "absorbing (first-order Clayton-Engquist)", "samples": nmc,
           "candidates": R, "designs": len(designs)}
    with Context(0, 64 << 30) as ctx:
        med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
        dmask = torch.as_tensor(masks, device="cuda")
        H = torch.empty((nmc, R, 7, 7), dtype=torch.float64, device="cuda")
        st_ = torch.empty(nmc, dtype=torch.int32, device="cuda")
        e = torch.empty(len(designs), dtype=torch.float64, device="cuda")
        for jac in ("fd", "sensitivity"):
            fn = ctx.jacobian_fd if jac == "fd" else ctx.jacobian_sensitivity
            fn([g] * 64, [med] * 64, wl.theta[:64], [wl.receivers] * 64, wl.sigma, H[:64],
               stf="gauss", per_receiver=True, status=st_[:64])
            torch.cuda.synchronize()
            ctx.stencil_stats(reset=True)
            t0 = time.perf_counter()
            fn([g] * nmc, [med] * nmc, wl.theta, [wl.receivers] * nmc, wl.sigma, H,
               stf="gauss", per_receiver=True, status=st_)
            ctx.design_eval(H, dmask, prior, wl.weights, e, theta=wl.theta)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st = ctx.stencil_stats(reset=True)
            variant = ctx.get_option("last_variant")
            nsol = 15 if jac == "fd" else 8
            upd_s = st["updates"] / (max(st["ms"], 1e-9) * 1e-3)
            r = {"seconds": t, "sample_eig_evals_per_s": nmc / t, "solves": nsol * nmc,
                 "grid_pt_updates_per_s": nsol * nmc * wl.grid.nx * wl.grid.nz *
                 wl.grid.nsteps / t,
                 "grid_pt_updates_per_s_stencil": upd_s, "stencil_ms": st["ms"],
                 "launches": st["launches"], "variant": variant,
                 "flagged_samples": int(st_.ne(0).sum())}
            ev = e.cpu().numpy()
            qb = int(np.argmax(ev))
            r["best_design"] = {"scenario": designs[qb][0], "design": designs[qb][1],
                                "eig_nats": float(ev[qb])}
            if jac == "fd":
                rec = _counter_record(RESIDENT_RECORD, RESIDENT_SOURCES, variant=variant)
                issue = (upd_s * rec["valu_lane_instr_per_update"] / VALU_ISSUE_PEAK
                         if rec else None)
                r["roofline"] = {
                    "bound": "alu", "achieved": upd_s * LAYERED_FLOPS_PER_UPDATE / 1e12,
                    "peak": FP32_VECTOR_PEAK_FLOPS / 1e12, "unit": "TFLOP/s",
                    "frac": upd_s * LAYERED_FLOPS_PER_UPDATE / FP32_VECTOR_PEAK_FLOPS,
                    "traffic": (rec["traffic_bytes_per_update"] * st["updates"] /
                                max(st["launches"], 1)) if rec else None,
                    "valu_issue_frac": issue,
                    "valu_lane_instr_per_update":
                        rec["valu_lane_instr_per_update"] if rec else None,
                    "update_equivalent_GBs_24B": upd_s * 24 / 1e9,
                    "note": f"{LAYERED_FLOPS_PER_UPDATE} FP32 operations per grid-point "
                            "update over the kernel time, against the published 157.3 "
                            "TFLOP/s (packed FP32 FMA, which this build does not emit: "
                            "adds and multiplies each take a full issue slot); "
                            "valu_issue_frac: vector lane-instructions per update "
                            "(SQ_INSTS_VALU x 64 from the counter record) times the "
                            "update rate over the 3.93e13/s issue limit.  The fields stay "
                            "in LDS: traffic is the whole launch's bytes past L2"}
            out[jac] = r
        # oracle on ncheck samples
        idx = [0, nmc // 2][:ncheck]
        Hc = torch.empty((len(idx), R, 7, 7), dtype=torch.float64, device="cuda")
        ctx.jacobian_fd([g] * len(idx), [med] * len(idx), wl.theta[idx], [wl.receivers] * len(idx),
           wl.sigma, Hc, stf="gauss", per_receiver=True)
        torch.cuda.synchronize()
        Hg = Hc.cpu().numpy()
    ref = opipe.query(wl, theta=wl.theta[idx], weights=np.full(len(idx), 1 / len(idx)),
                      per_receiver=True)
    Hr = ref["H1"]
    d = np.sqrt(np.abs(np.einsum("srii->sri", Hr)))
    pr = laplace.uniform_prior(wl.lo, wl.hi)
    dk = np.array([laplace.dkl_hat(Hg[s].sum(axis=0), wl.theta[idx][s], pr)[0]
                   for s in range(len(idx))])
    out["errors"] = {
        "samples": idx,
        "per_receiver_scaled_hessian_max_abs": float(np.max(
            np.abs(Hg - Hr) / (d[..., :, None] * d[..., None, :] + 1e-300))),
        "dkl_all_receivers_abs": float(np.max(np.abs(dk - ref["dkl"]))),
        "reference": "oracle (oracle/pipeline.py) on the same samples"}
    return out


def _bench_loh2d(ctx, nmc=10000, level=5, nbatch=10):
    """The paper's model problem (Section 4.1) and its scenarios (Section 4.5):
    per-receiver H_1 over the 91 candidate surface nodes for M = nmc Monte
    Carlo samples and for the level-`level` sparse grid (8583 nodes at level
    5), every scenario design's EIG from the same solves, a 68 % interval
    from batch means, and the conditioning of H_1 at the prior mean."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import make_prior, sparse_grid_gl
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wl = synthetic.loh_workload(nmc)
    g = grid_tuple(wl.grid)
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    R = len(wl.receivers)
    pos = {int(ix): c for c, ix in enumerate(wl.receivers)}
    designs = [(scen, lab, idx) for scen, ds in synthetic.loh_scenarios().items()
               for lab, idx in ds]
    masks = np.zeros((len(designs), R), dtype=np.uint8)
    for q, (_, _, idx) in enumerate(designs):
        masks[q, [pos[int(i)] for i in idx]] = 1
    dmask = torch.as_tensor(masks, device="cuda")
    prior = make_prior(wl.lo, wl.hi)

    def per_receiver_h1(theta, jacobian):
        S = len(theta)
        H = torch.empty((S, R, 7, 7), dtype=torch.float64, device="cuda")
        st = torch.empty(S, dtype=torch.int32, device="cuda")
        fn = ctx.jacobian_fd if jacobian == "fd" else ctx.jacobian_sensitivity
        fn([g] * S, [med] * S, theta, [wl.receivers] * S, wl.sigma, H, stf="gauss",
           per_receiver=True, status=st)
        return H, st

    def design_eigs(H, theta, w):
        e = torch.empty(len(designs), dtype=torch.float64, device="cuda")
        ctx.design_eval(H, dmask, prior, w, e, theta=theta)
        return e.cpu().numpy()

    out = {"grid": [wl.grid.nx, wl.grid.nz, wl.grid.nsteps], "h": wl.grid.h,
           "dt": wl.grid.dt, "edges": "absorbing (first-order Clayton-Engquist)",
           "candidates": R, "designs": len(designs)}
    # warm-up and tuning on a few samples, then once at full size (the
    # workspace grows to its final size outside the timed runs)
    per_receiver_h1(wl.theta[:64], "fd")
    per_receiver_h1(wl.theta, "fd")
    torch.cuda.synchronize()
    runs = {}
    for jac in ("fd", "sensitivity"):
        ctx.stencil_stats(reset=True)
        t0 = time.perf_counter()
        H, st = per_receiver_h1(wl.theta, jac)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        sst = ctx.stencil_stats(reset=True)
        nsol = 15 if jac == "fd" else 8
        upd = nsol * nmc * wl.grid.nx * wl.grid.nz * wl.grid.nsteps
        eig = design_eigs(H, wl.theta, wl.weights)
        bm = []
        b = nmc // nbatch
        for k in range(nbatch):
            bm.append(design_eigs(H[k * b:(k + 1) * b].contiguous(), wl.theta[k * b:(k + 1) * b],
                                  np.full(b, 1.0 / b)))
        ci = np.std(np.stack(bm), axis=0, ddof=1) / np.sqrt(nbatch)
        runs[jac] = {"seconds": t, "sample_eig_evals_per_s": nmc / t,
                     "grid_pt_updates_per_s": upd / t, "solves": nsol * nmc,
                     "stencil_avg_launch_ms": sst["ms"] / max(sst["launches"], 1),
                     "stencil_launches": sst["launches"],
                     "flagged_samples": int(st.abs().gt(0).sum())}
        runs[jac]["eig"] = eig
        runs[jac]["ci68"] = ci
        del H
    out["mc"] = {"samples": nmc, "batches_for_ci": nbatch,
                 **{jac: {k: v for k, v in r.items() if k not in ("eig", "ci68")}
                    for jac, r in runs.items()}}
    # sparse quadrature
    nodes, w = sparse_grid_gl(7, level, wl.lo, wl.hi)
    t0 = time.perf_counter()
    H, st = per_receiver_h1(nodes, "fd")
    eig_sg = design_eigs(H, nodes, w)
    torch.cuda.synchronize()
    out["sparse"] = {"level": level, "nodes": len(w), "seconds": time.perf_counter() - t0,
                     "flagged_nodes": int(st.abs().gt(0).sum())}
    del H
    curves = {}
    for q, (scen, lab, _) in enumerate(designs):
        curves.setdefault(scen, []).append(
            {"design": lab, "eig_mc": float(runs["fd"]["eig"][q]),
             "ci68_mc": float(runs["fd"]["ci68"][q]),
             "eig_mc_sensitivity": float(runs["sensitivity"]["eig"][q]),
             "eig_sparse": float(eig_sg[q])})
    out["scenarios"] = curves
    c3 = curves["III"]
    out["scenario_III_best_dR"] = c3[int(np.argmax([c["eig_mc"] for c in c3]))]["design"]
    c1 = [c["eig_mc"] for c in curves["I"]]
    out["scenario_I_gain_3_to_17_vs_17_to_81"] = [c1[3] - c1[0], c1[5] - c1[3]]
    # conditioning of H_1 at the prior mean (one array per scenario family)
    th = synthetic.loh_prior_mean_paper()[None, :]
    H, _ = per_receiver_h1(th, "fd")
    Hr = H.cpu().numpy()[0]
    conds = {}
    for scen, lab in (("I", "NR=17,dR=1000"), ("III", "dR=1000"), ("I", "NR=81,dR=200")):
        idx = next(i for s_, l_, i in designs if s_ == scen and l_ == lab)
        H1 = Hr[[pos[int(i)] for i in idx]].sum(axis=0)
        d = np.sqrt(np.diag(H1))
        conds[f"{scen}:{lab}"] = {"cond_H1": float(np.linalg.cond(H1)),
                                  "cond_scaled": float(np.linalg.cond(H1 / np.outer(d, d)))}
    out["conditioning_at_prior_mean"] = conds
    return out


def _bench_nested(ctx, sizes=(1000, 10000, 100000, 400000), nlaplace=10000, sg_level=4):
    """Section 4.4: the Laplace method (Theorem 4 on the three inferred
    parameters, Monte Carlo and sparse quadrature) against the nested Monte
    Carlo estimator with the outer samples reused as inner ones, on the
    model problem with T = 1.25 s and two receivers.  Also times the
    nested kernel (the distances in Gram form make the (n, m, k) work one
    FP64 multiply-add of a dense product on the matrix cores: 2 flops per
    pair-element, mfma_frac against the published dense FP64 matrix rate)."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import make_prior, sparse_grid_gl
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    grid, med, rec, lo, hi, tpl = synthetic.loh_nested_setup()
    dm = device_medium(med.kind, med.rho, med.lam, med.mu)
    g = grid_tuple(grid)
    act = list(synthetic.LOH_NESTED_ACTIVE)
    sigma = 0.01
    K = (grid.nsteps + 1) * len(rec) * 2
    rng = np.random.default_rng(44)
    out = {"grid": [grid.nx, grid.nz, grid.nsteps], "receivers_x1": [-9000, 1000],
           "inferred": ["depth", "omega_s", "m_xx"], "nobs": K, "sigma": sigma}
    # Laplace, Monte Carlo
    prior = make_prior(lo, hi, active=act)

    def laplace(theta, w):
        S = len(theta)
        H1 = torch.empty((S, 7, 7), dtype=torch.float64, device="cuda")
        ctx.jacobian_fd([g] * S, [dm] * S, theta, [rec] * S, sigma, H1, stf="gauss")
        dkl = torch.empty(S, dtype=torch.float64, device="cuda")
        eig = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.laplace_eig(H1, prior, w, dkl, eig, theta=theta)
        return float(eig.cpu()[0]), dkl.cpu().numpy()

    th = synthetic.loh_nested_draws(rng, nlaplace)
    t0 = time.perf_counter()
    e_mc, dk = laplace(th, np.full(nlaplace, 1.0 / nlaplace))
    out["laplace_mc"] = {"samples": nlaplace, "eig": e_mc,
                         "ci68": float(np.std(dk, ddof=1) / np.sqrt(nlaplace)),
                         "seconds": time.perf_counter() - t0}
    # Laplace, sparse quadrature over the three inferred parameters
    nodes3, w3 = sparse_grid_gl(3, sg_level, lo[act], hi[act])
    thq = np.repeat(tpl[None, :], len(w3), axis=0)
    thq[:, act] = nodes3
    e_sg, _ = laplace(thq, w3)
    out["laplace_sparse"] = {"level": sg_level, "nodes": len(w3), "eig": e_sg}
    # nested Monte Carlo, reuse
    res = []
    for N in sizes:
        th = synthetic.loh_nested_draws(rng, N)
        gtr = torch.empty((N, K), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.forward_solve_batch([g] * N, [dm] * N, th, [rec] * N, list(gtr), stf="gauss")
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        noise = torch.randn((N, K), generator=torch.Generator(device="cuda").manual_seed(N),
                            device="cuda", dtype=torch.float32)
        lr = torch.empty(N, dtype=torch.float64, device="cuda")
        eig = torch.empty(1, dtype=torch.float64, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.nested_mc_eig(gtr, noise, gtr, sigma, lr, eig)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pairs = float(N) * N * K
        v = float(eig.cpu()[0])
        res.append({"N=M": N, "eig": v, "log_M": float(np.log(N)),
                    "ci68": float(lr.std().item() / np.sqrt(N)),
                    "rel_diff_vs_laplace_mc": (v - e_mc) / e_mc,
                    "forward_seconds": t_fwd, "kernel_ms": ms,
                    "pair_elements_per_s": pairs / (ms * 1e-3),
                    "fp64_TFLOPs": 2 * pairs / (ms * 1e-3) / 1e12,
                    "mfma_frac": 2 * pairs / (ms * 1e-3) / FP64_MFMA_PEAK_FLOPS})
        print(f"[bench] nested N=M={N}: {v:.4f} nats, kernel {ms:.1f} ms", flush=True)
        del gtr, noise
    out["nested_reuse"] = res
    out["note"] = ("with reuse each log ratio is at most log M, so the nested estimate "
                   "approaches the Laplace value from below as M grows past exp(EIG)")
    return out


def _bench_estimators(ctx, sig_rels=(0.3, 0.6, 1.0), n_outer=4000, n_inner=200000,
                      n_lap=2000, iters=5):
    """Theorem 4 (O(1/N)), Theorem 3 (O(1/N^2)) and the nested double loop
    with independent inner samples, on one low-information problem: the
    64x64x400 homogeneous grid with rigid edges, two receivers, depth,
    frequency and m_xx inferred under a Gaussian prior (width 1/10 of the
    c1 box, draws clipped to the box), at several noise levels."""
    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import make_prior
    from paper_1502_07873_amd.query import device_medium, grid_tuple
    wl = synthetic.config("c1")[0]
    grid, med = wl.grid, wl.medium
    g = grid_tuple(grid)
    dm = device_medium(med.kind, med.rho, med.lam, med.mu)
    rec = np.array([16, 48], dtype=np.int32)
    act = [1, 3, 4]
    tpl = 0.5 * (wl.lo + wl.hi)
    std = (wl.hi - wl.lo) / 10
    cov = np.diag(std ** 2)
    prior = make_prior(mean=tpl, cov=cov, active=act)
    rng = np.random.default_rng(12)

    def draws(n):
        th = np.repeat(tpl[None, :], n, axis=0)
        for j in act:
            th[:, j] = np.clip(tpl[j] + std[j] * rng.standard_normal(n), wl.lo[j], wl.hi[j])
        return th

    K = (grid.nsteps + 1) * len(rec) * 2

    def forward(th):
        out = torch.empty((len(th), K), dtype=torch.float32, device="cuda")
        ctx.forward_solve_batch([g] * len(th), [dm] * len(th), th, [rec] * len(th), list(out))
        return out

    peak = float(forward(tpl[None, :]).abs().max())
    th_out, th_in, th_lap = draws(n_outer), draws(n_inner), draws(n_lap)
    noise = torch.randn((n_outer, K), generator=torch.Generator(device="cuda").manual_seed(3),
                        device="cuda", dtype=torch.float32)
    t0 = time.perf_counter()
    g_out, g_in = forward(th_out), forward(th_in)
    torch.cuda.synchronize()
    out = {"grid": [grid.nx, grid.nz, grid.nsteps], "receivers": rec.tolist(),
           "inferred": ["depth", "f", "m_xx"], "prior": "gaussian, std = c1 box / 10",
           "n_outer": n_outer, "n_inner": n_inner, "n_laplace": n_lap,
           "forward_seconds": time.perf_counter() - t0, "levels": []}
    for rel in sig_rels:
        sigma = rel * peak
        row = {"sigma_rel_peak": rel}
        # Theorem 4
        H1 = torch.empty((n_lap, 7, 7), dtype=torch.float64, device="cuda")
        ctx.jacobian_fd([g] * n_lap, [dm] * n_lap, th_lap, [rec] * n_lap, sigma, H1)
        dkl = torch.empty(n_lap, dtype=torch.float64, device="cuda")
        e4 = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.laplace_eig(H1, prior, np.full(n_lap, 1.0 / n_lap), dkl, e4, theta=th_lap)
        d4 = dkl.cpu().numpy()
        row["theorem4"] = {"eig": float(e4.cpu()[0]),
                           "ci68": float(d4.std(ddof=1) / np.sqrt(n_lap))}
        # Theorem 3 on the first n_lap outer samples and their noise
        n3 = n_lap
        H1t = torch.empty((n3, 7, 7), dtype=torch.float64, device="cuda")
        H2t = torch.empty_like(H1t)
        v3 = torch.empty(n3, dtype=torch.float64, device="cuda")
        e3 = torch.empty(1, dtype=torch.float64, device="cuda")
        st = torch.empty(n3, dtype=torch.int32, device="cuda")
        t0 = time.perf_counter()
        ctx.theorem3_eig([g] * n3, [dm] * n3, th_out[:n3], [rec] * n3, list(noise[:n3]), sigma,
                         prior, np.full(n3, 1.0 / n3), H1t, H2t, v3, e3, st, iters=iters)
        torch.cuda.synchronize()
        v3n = v3.cpu().numpy()
        ok = st.cpu().numpy() == 0
        row["theorem3"] = {"eig": float(e3.cpu()[0]), "eig_ok_samples": float(v3n[ok].mean()),
                           "ci68": float(v3n[ok].std(ddof=1) / np.sqrt(ok.sum())),
                           "not_pd": int((~ok).sum()), "seconds": time.perf_counter() - t0}
        # nested double loop, independent inner samples
        lr = torch.empty(n_outer, dtype=torch.float64, device="cuda")
        en = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.nested_mc_eig(g_out, noise, g_in, sigma, lr, en)
        lrn = lr.cpu().numpy()
        row["nested"] = {"eig": float(en.cpu()[0]), "ci68": float(lrn.std(ddof=1) / np.sqrt(n_outer)),
                         "eig_same_outer_as_theorem3": float(lrn[:n3][ok].mean())}
        out["levels"].append(row)
        print(f"[bench] sigma={rel} peak: thm4 {row['theorem4']['eig']:.3f} "
              f"thm3 {row['theorem3']['eig_ok_samples']:.3f} nested {row['nested']['eig']:.3f}",
              flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="leave out the uneven-batch leg")
    ap.add_argument("--no-c5", action="store_true", help="leave out the design-sweep leg")
    ap.add_argument("--c5-full-only", action="store_true",
                    help="--workload c5: only the full-size nodes (for counter runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed query: no other leg (for counter runs)")
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c3", "c5", "c5-full", "model", "loh2d", "nested",
                             "estimators", "serving"],
                    help="c2: the headline query and every leg (default); c3/c5: those legs "
                         "alone; c5-full: the whole 589-node c5 query at full size and its "
                         "greedy design; model: the model-problem leg alone; loh2d: the paper's "
                         "model problem with sparse quadrature and scenarios; serving: "
                         "the serving streams with both disciplines")
    ap.add_argument("--serving-rate", type=float, default=3.2e11,
                    help="grid-point updates/s that sets the arrival rate of --workload "
                         "serving (default: about the headline's update rate)")
    ap.add_argument("--serving-queries", type=int, default=0,
                    help="--workload serving: queries of the full-range stream (0: up to "
                         "1.2e13 updates)")
    ap.add_argument("--wave-cache-mib", type=int, default=192,
                    help="live field MiB per wave chunk (0: whole waves through HBM)")
    ap.add_argument("--coef-interleave", type=int, default=None,
                    help="c5 leg: solves of one nodal medium whose tiles run interleaved "
                         "by position (library default 8; 1: solve-major)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter scale)")
    args = ap.parse_args()
    if args.copy_calibration:
        _copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(samples would shard across GPUs with one all-reduce of the "
              "per-design sums).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic
    from paper_1502_07873_amd import Context
    from paper_1502_07873_amd.query import device_medium, grid_tuple, run_query

    if args.workload in ("c3", "c5", "model", "c5-full"):
        if args.workload == "c5-full":
            res = _bench_c5_full_query()
        elif args.workload == "c3":
            res = _bench_c3(args.samples if args.samples != 256 else 4096)
        elif args.workload == "c5":
            res = _bench_c5(pipeline=not args.c5_full_only,
                            coef_interleave=args.coef_interleave)
        else:
            res = _bench_model(args.samples if args.samples != 256 else 10000)
        print(json.dumps({"workload": args.workload, **res}), flush=True)
        return
    if args.workload != "c2":
        ctx = Context(0, 200 << 30)
        ctx.set_option("wave_cache_bytes", args.wave_cache_mib << 20)
        if args.workload == "loh2d":
            res = _bench_loh2d(ctx, args.samples if args.samples != 256 else 10000)
        elif args.workload == "nested":
            res = _bench_nested(ctx)
        elif args.workload == "estimators":
            res = _bench_estimators(ctx)
        else:
            res = {"load_basis_updates_per_s": args.serving_rate,
                   "serving_head_of_line": _serving_head_of_line(ctx)}
            for overlap in (True, False):
                key = "serving_c4" + ("" if overlap else "_queue_only")
                res[key] = _serving_c4(ctx, args.serving_rate, overlap=overlap,
                                       nquery=args.serving_queries or None)
        print(json.dumps({"workload": args.workload, **res}), flush=True)
        ctx.close()
        return
    wl = synthetic.config("c2", nsample=args.samples)[0]
    g = grid_tuple(wl.grid)
    dev = torch.device("cuda", 0)
    med = device_medium(wl.medium.kind, wl.medium.rho, wl.medium.lam, wl.medium.mu)
    ctx = Context(0, 200 << 30)
    ctx.set_option("wave_cache_bytes", args.wave_cache_mib << 20)
    stream = torch.cuda.current_stream(dev)

    theta_bar = 0.5 * (wl.lo + wl.hi)
    jac_stats = {"ms": 0.0, "launches": 0, "updates": 0.0, "bytes": 0.0}

    def one_step(record=False):
        # the noise level comes from one nominal solve at the prior mean; its
        # 1-solve launches are kept out of the stencil roofline figures
        sigma = ctx.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
        ctx.stencil_stats(reset=True)
        out = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                        sigma=sigma)
        if record:
            st = ctx.stencil_stats(reset=True)
            for k in jac_stats:
                jac_stats[k] += st[k]
        return out

    print(f"[bench] workload c2 S={len(wl.theta)} grid={g} warmup={args.warmup} "
          f"steps={args.steps}", flush=True)
    for w in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} done", flush=True)
    ctx.stencil_stats(reset=True)
    torch.cuda.synchronize()
    lat = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    t0 = time.perf_counter()
    out = None
    for k in range(args.steps):
        out = one_step(record=True)
        ev[k + 1].record(stream)
        torch.cuda.synchronize()
        lat.append(ev[k].elapsed_time(ev[k + 1]))
        print(f"[bench] step {k} {lat[-1]:.1f} ms", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev[0].elapsed_time(ev[-1])
    st = jac_stats
    variant = ctx.get_option("last_variant")
    steps_per_launch = _steps_per_launch(variant)
    S = len(wl.theta)
    value = S * args.steps / (total_ms / 1e3)
    avg_launch_ms = st["ms"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    dkl = out["dkl"].cpu().numpy()
    eig = float(out["eig"].cpu()[0])
    copy_gbs = _copy_rate()
    llc_copy_gbs = _copy_rate(96 << 20, reps=200)
    solves_per_launch = st["updates"] / max(st["launches"], 1) / (
        wl.grid.nx * wl.grid.nz * steps_per_launch)
    traffic = _measured_traffic(round(solves_per_launch), ctx.get_option("wave_cache_bytes"),
                                variant)
    traffic_rate = traffic / (avg_launch_ms * 1e-3) / 1e9 if traffic else None
    in_cache = steps_per_launch < 4   # two or three steps: cache-sized chunks
    floor_b = {1: 24.0, 2: 16.0, 3: 32.0 / 3.0, 4: BLOCKED_FLOOR_B}[steps_per_launch]
    status_ok = int(out["status"].abs().sum()) == 0 and int(out["chol_status"].abs().sum()) == 0
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "sample-EIG evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "precision": "f32 wavefields; f64 forcing differences, Jacobian, H_1, scaling, "
                     "Cholesky, log-det, averages",
        "data": "synthetic",
        "config": {"workload": "c2 Monte Carlo query: 512x512 grid, h=10 m, 2000 steps, "
                               "two-layer medium, 21 receivers, "
                               f"{S} prior samples x 15 solves (+1 sigma solve)",
                   "samples": S, "solves_per_step": 15 * S + 1,
                   "grid": [wl.grid.nx, wl.grid.nz], "nsteps": wl.grid.nsteps},
        "eig_nats": eig,
        "status_ok": status_ok,
        "grid_pt_updates_per_s": st["updates"] / (total_ms / 1e3),
        "stencil": {"launches": st["launches"], "avg_launch_ms": avg_launch_ms,
                    "variant": variant, "steps_per_launch": steps_per_launch,
                    "bytes_per_launch": bytes_per_launch,
                    "kernel_floor_bytes_per_update": floor_b,
                    "achieved_at_kernel_floor_GBs": achieved * floor_b / 24,
                    "time_frac_of_step": st["ms"] / total_ms,
                    "solves_per_launch": solves_per_launch,
                    "note": ("launches of the 15*S-solve jacobian_fd wave, every solve in "
                             "every launch (four steps per launch with each 58x58 tile and "
                             "its 4-node halo in LDS: the fields stream through HBM)"
                             if not in_cache else
                             "launches of the 15*S-solve jacobian_fd wave, run as chunks "
                             "whose fields (4 buffers per solve) fit wave_cache_bytes, so "
                             "they stay in the 256 MB last-level cache between launches") +
                            "; bytes_per_launch and roofline.achieved count 24 B per "
                            "grid-point update (read u^m, u^{m-1}, write u^{m+1}); "
                            "kernel_floor_bytes_per_update: what the kernel itself must "
                            "move per update (achieved_at_kernel_floor_GBs)"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "llc" if in_cache else "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_rate_GBs": traffic_rate,
                     "llc_copy_GBs_measured": llc_copy_gbs,
                     "frac_of_llc_copy": (traffic_rate / llc_copy_gbs
                                          if traffic_rate and in_cache else None),
                     "copy_GBs_measured": copy_gbs,
                     "frac_of_copy": (traffic_rate / copy_gbs
                                      if traffic_rate and not in_cache else None),
                     "wave_cache_bytes": ctx.get_option("wave_cache_bytes"),
                     "note": "achieved: 24 B per update (algorithmic: read u^m, u^{m-1}, "
                             "write u^{m+1}) over the launch time; frac: achieved / the "
                             "8 TB/s HBM peak. " + (
                                 "The kernel takes four steps per launch with the tile in "
                                 "LDS, so it moves about 8 B per update, not 24: "
                                 "achieved can pass the peak. traffic: bytes per launch "
                                 "past L2 from the counter record; frac_of_copy: that "
                                 "traffic rate over a plain 2 x 4 GiB copy measured in "
                                 "this run (copy_GBs_measured). two_step_llc: the same "
                                 "query with two steps per launch in cache-sized chunks"
                                 if not in_cache else
                                 "The launches work in the 256 MB last-level cache "
                                 "(cache-sized chunks), so the bound is that cache; "
                                 "traffic: bytes per launch past L2 from the counter record; "
                                 "frac_of_llc_copy: that rate over a plain 96 MiB copy "
                                 "measured in this run")},
        "wall_s": wall,
    }
    if args.headline_only:
        print(json.dumps(line), flush=True)
        ctx.close()
        return
    # the same query with the other temporal-blocking family: two steps per
    # launch in cache-sized chunks (or four steps, if two ran above)
    other_tb = 2 if not in_cache else 4
    print(f"[bench] same query, temporal_blocking {other_tb}", flush=True)
    tb0 = ctx.get_option("temporal_blocking")
    ctx.set_option("temporal_blocking", other_tb)
    one_step()
    torch.cuda.synchronize()
    ctx.stencil_stats(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ou = one_step()
    e1.record(stream)
    torch.cuda.synchronize()
    stu = ctx.stencil_stats(reset=True)
    tu = e0.elapsed_time(e1) / 1e3
    vu = ctx.get_option("last_variant")
    ctx.set_option("temporal_blocking", tb0)
    ach_u = stu["bytes"] / (stu["ms"] * 1e-3) / 1e9
    line["two_step_llc" if other_tb == 2 else "four_step_hbm"] = {
        "value": S / tu, "unit": "sample-EIG evals/s", "variant": vu,
        "steps_per_launch": _steps_per_launch(vu),
        "avg_launch_ms": stu["ms"] / max(stu["launches"], 1),
        "launches": stu["launches"],
        "grid_pt_updates_per_s_stencil": stu["updates"] / (stu["ms"] * 1e-3),
        "achieved_GBs": ach_u, "frac": ach_u / HBM_PEAK_GBS,
        "headline_speedup": value / (S / tu),
        "dkl_match": bool(np.array_equal(ou["dkl"].cpu().numpy(), dkl))}
    # the plain GPU path: the same kernels, one solve per launch
    print("[bench] one-solve-per-launch GPU baseline (2 samples)", flush=True)
    ctx1 = Context(0, 8 << 30)
    ctx1.set_option("max_wave_solves", 1)
    sig1 = ctx1.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
    run_query(ctx1, g, med, wl.receivers, wl.lo, wl.hi, wl.theta[:1], [1.0], sigma=sig1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sig1 = ctx1.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
    o1 = run_query(ctx1, g, med, wl.receivers, wl.lo, wl.hi, wl.theta[:2], [0.5, 0.5],
                   sigma=sig1)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = e0.elapsed_time(e1) / 1e3
    line["baseline_one_solve_per_launch"] = {
        "value": 2 / t1, "unit": "sample-EIG evals/s", "samples": 2,
        "speedup_of_batched": value / (2 / t1),
        "dkl_match": bool(np.allclose(o1["dkl"].cpu().numpy(), dkl[:2], rtol=0, atol=0))}
    ctx1.close()
    print("[bench] launch-bound query with and without graph replay", flush=True)
    line["graph_replay"] = _graph_gain()
    # the forward-sensitivity Jacobian (1 + 7 solves per sample) on the same query
    print("[bench] forward-sensitivity Jacobian path (same samples)", flush=True)
    sig = ctx.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
    run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta[:8], np.full(8, 1 / 8),
              sigma=sig, jacobian="sensitivity")   # tunes the 8*S-solve bucket
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sig = ctx.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
    os_ = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta, wl.weights,
                    sigma=sig, jacobian="sensitivity")
    e1.record(stream)
    torch.cuda.synchronize()
    ts = e0.elapsed_time(e1) / 1e3
    line["sensitivity_path"] = {
        "value": S / ts, "unit": "sample-EIG evals/s", "samples": S,
        "solves_per_step": 8 * S + 1, "ms_per_step": ts * 1e3,
        "speedup_over_central_differences": (S / ts) / value,
        "eig_nats": float(os_["eig"].cpu()[0]),
        "max_abs_dkl_diff_vs_central_differences":
            float(np.max(np.abs(os_["dkl"].cpu().numpy() - dkl))),
        "status_ok": int(os_["status"].abs().sum()) == 0}
    # the CPU baseline's GPU side of the sample (before the other legs)
    gpu0 = None
    if not args.no_cpu_baseline:
        sig = ctx.noise_sigma_peak(g, med, theta_bar, wl.noise_rel)
        o0 = run_query(ctx, g, med, wl.receivers, wl.lo, wl.hi, wl.theta[:1], [1.0], sigma=sig,
                       keep_nominal=True, keep_J=True)
        torch.cuda.synchronize()
        gpu0 = {"nominal": o0["nominal"][0].cpu().numpy().astype(np.float64),
                "J": o0["J"][0].cpu().numpy(), "H1": o0["H1"][0].cpu().numpy(),
                "dkl": float(o0["dkl"].cpu()[0]), "sigma": sig}
        del o0
    # the remaining legs bring their own contexts: the headline's workspace
    # goes back to the device first (c3 needs ~214 GB, serving a 250 GB arena)
    ctx.close()
    del out, ou, o1, os_
    torch.cuda.empty_cache()
    if not args.no_c5:
        print("[bench] c5: full-size sparse-grid nodes and the reduced design pipeline",
              flush=True)
        line["c5"] = _bench_c5()
    print("[bench] the paper's model problem (absorbing edges, resident solves)", flush=True)
    line["model_problem"] = _bench_model()
    if not args.no_c3:
        print("[bench] c3: the 61440-solve uneven batch", flush=True)
        line["c3"] = _bench_c3()
    if not args.no_serving:
        rate = line["grid_pt_updates_per_s"]
        sctx = Context(0, 2 << 30)
        line["serving_head_of_line"] = _serving_head_of_line(sctx)
        line["serving_c4"] = _serving_c4(sctx, rate)
        sctx.close()
        hol = line["serving_head_of_line"]["continuous_batching"]
        line["latency_ms"]["serving_p50"] = line["serving_c4"]["latency_p50_s"] * 1e3
        line["latency_ms"]["serving_p99"] = line["serving_c4"]["latency_p99_s"] * 1e3
        line["latency_ms"]["serving_hol_short_p50"] = hol["short_latency_p50_s"] * 1e3
        line["latency_ms"]["serving_hol_short_p99"] = hol["short_latency_p99_s"] * 1e3
    if gpu0 is not None:
        print("[bench] cpu baseline (oracle, 1 sample)", flush=True)
        cb, errs = _cpu_baseline(wl, wl.theta[0], gpu0)
        line["cpu_baseline"] = cb
        line["errors"] = errs
        line["sampled_err_nats"] = errs["dkl_abs"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
