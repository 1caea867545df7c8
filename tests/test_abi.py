"""The C-ABI library loads and exports every entry point include/eigseis.h
declares; host-only entry points match the oracle (CPU, no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import smolyak

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eigseis.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "defined")))


def test_library_exports_every_declared_symbol():
    from paper_1502_07873_amd import eigseis
    lib = ctypes.CDLL(eigseis.LIB_PATH)
    declared = _declared()
    assert "jacobian_fd" in declared and "forward_solve_batch" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(eigseis.EXPORTED)


@pytest.mark.parametrize("d,w", [(1, 0), (2, 5), (3, 5), (3, 6), (7, 3), (7, 5)])
def test_sparse_grid_matches_oracle(d, w):
    import paper_1502_07873_amd as p
    lo = np.linspace(1.0, 2.0, d)
    hi = lo + np.linspace(0.5, 3.0, d)
    X, W = smolyak.sparse_grid(d, w, lo, hi)
    n, wt = p.sparse_grid_gl(d, w, lo, hi)
    assert n.shape == X.shape
    assert np.max(np.abs(n - X)) < 1e-12
    assert np.max(np.abs(wt - W)) < 1e-11


def test_sparse_grid_rejects_bad_arguments():
    import paper_1502_07873_amd as p
    with pytest.raises(p.EigError):
        p.sparse_grid_gl(0, 3)
    with pytest.raises(p.EigError):
        p.sparse_grid_gl(3, -1)


def test_binding_refuses_media_it_cannot_pass_on():
    # the library reads nz (layered) or nz*nx (nodal) float64 device values
    # per medium array; the binding refuses anything else before a launch
    torch = pytest.importorskip("torch")
    from paper_1502_07873_amd import eigseis
    g = (40, 30, 10.0, 1e-3, 10, 0)
    short = torch.zeros(29, dtype=torch.float64)
    with pytest.raises(eigseis.EigError):
        eigseis.Context._media([(eigseis.MEDIUM_LAYERED, short, short, short)], [g])
    with pytest.raises(eigseis.EigError):
        eigseis.Context._media([(eigseis.MEDIUM_LAYERED,) + (short,) * 3] * 2, [g])


def test_library_binds_to_torchs_hip_runtime():
    # one HIP runtime per process: the binding imports torch before loading
    # the library, so the library's HIP calls resolve into torch's runtime
    # whatever the caller imported first (checked in a fresh process)
    import subprocess
    import sys
    pytest.importorskip("torch")
    code = ("import sys; sys.path.insert(0, %r); "
            "from paper_1502_07873_amd import eigseis" % ROOT)
    env = dict(os.environ, LD_DEBUG="bindings")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines()
             if "libeigseis.so" in ln and "`hipLaunchKernel'" in ln]
    assert lines, "no binding of hipLaunchKernel reported"
    import torch
    torch_lib = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), "lib"))
    assert all(torch_lib in ln for ln in lines), lines


def test_binding_argument_checks_refuse_before_any_call():
    # device arrays must be contiguous GPU tensors of the right dtype and at
    # least the size the library will touch; host rows must match exactly
    torch = pytest.importorskip("torch")
    from paper_1502_07873_amd import eigseis
    cpu = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(eigseis.EigError, match="dkl"):
        eigseis._dev(cpu, "dkl", torch.float64, 8)
    with pytest.raises(eigseis.EigError, match="required"):
        eigseis._dev(None, "H1", torch.float64, 49)
    eigseis._dev(None, "status", torch.int32, 8, optional=True)
    with pytest.raises(eigseis.EigError, match="expected 3 tensors"):
        eigseis._dev_list([cpu, cpu], "traces", torch.float32, [1, 1, 1])
    eigseis._dev_list(None, "nominal", torch.float32, [1], optional=True)
    eigseis._dev_list([None, None], "nominal", torch.float32, [1, 1], entries_optional=True)
    with pytest.raises(eigseis.EigError, match=r"noise\[0\]"):
        eigseis._dev_list([None, None], "noise", torch.float32, [1, 1])
    with pytest.raises(eigseis.EigError, match="at least 5"):
        eigseis._host([1.0, 2.0], "w", 5)
    assert eigseis._host([1.0, 2.0, 3.0], "w", 3).dtype == np.float64
    with pytest.raises(eigseis.EigError, match="2 x 7"):
        eigseis._theta(np.zeros(13), "theta", 2)
    assert eigseis._theta(np.zeros(14), "theta", 2).shape == (2, 7)
    # entry points check their arrays before reaching the library: a context
    # without a device handle never gets that far
    ctx = object.__new__(eigseis.Context)
    f32 = torch.zeros((4, 3), dtype=torch.float32)
    with pytest.raises(eigseis.EigError, match="g_outer"):
        ctx.nested_mc_eig(f32, f32, f32, 0.1, torch.zeros(4, dtype=torch.float64))
    with pytest.raises(eigseis.EigError, match="shape mismatch"):
        ctx.nested_mc_eig(f32, f32[:3], f32, 0.1, torch.zeros(4, dtype=torch.float64))
    H = torch.zeros((2, 7, 7), dtype=torch.float64)
    with pytest.raises(eigseis.EigError, match="H1"):
        ctx.laplace_eig(H, eigseis.make_prior(-np.ones(7), np.ones(7)), [0.5, 0.5],
                        torch.zeros(2, dtype=torch.float64), torch.zeros(1, dtype=torch.float64))
    g = (40, 30, 10.0, 1e-3, 10, 0)
    with pytest.raises(eigseis.EigError, match="traces"):
        ctx.forward_solve_batch([g], [None], np.zeros(7), [np.array([3, 5])],
                                [torch.zeros(10, dtype=torch.float32)])
    with pytest.raises(eigseis.EigError, match="one receiver array per grid"):
        ctx.forward_solve_batch([g, g], [None, None], np.zeros(14), [np.array([3])], [None, None])


def _raw_args():
    """Host structs for raw C-ABI calls whose argument checks fail before
    the (NULL) context or any device pointer is used."""
    from paper_1502_07873_amd import eigseis
    g = eigseis.Grid(2048, 256, 10.0, 1e-3, 10, eigseis.BC_RIGID)
    med = eigseis.Medium(eigseis.MEDIUM_LAYERED, 256, 256, 256)   # never read
    rec = np.array([100, 200], dtype=np.int32)
    R = eigseis.Receivers(2, rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return eigseis, g, med, rec, R


@pytest.mark.parametrize("rel_step,moves", [(1e-4, False), (6e-4, False), (0.01, True),
                                            (0.0015, True)])
def test_jacobian_refuses_deviation_steps_beyond_the_forcing_window(rel_step, moves):
    # x_s = 15005 m, h = 10 m: a step of rel_step * x_s leaves the source
    # cell by more than one cell at rel_step >= 0.0015 (22.5 m); the 7-node
    # forcing window then no longer holds both 6x6 stencils and the call is
    # refused; smaller steps pass every argument check and stop at the NULL
    # context
    eigseis, g, med, rec, R = _raw_args()
    theta = np.array([15005.0, 1205.0, 0.2, 7.0, 5e13, 5e13, 5e13])
    sigma = np.ones(1)
    rc = eigseis._lib.jacobian_fd(
        None, 1, ctypes.byref(g), ctypes.byref(med), theta.ctypes.data_as(ctypes.c_void_p),
        rel_step, eigseis.STF_GAUSS_DERIV, ctypes.byref(R), eigseis.SIGMA_GIVEN,
        sigma.ctypes.data_as(ctypes.c_void_p), 0, None, None, 256, None, None)
    msg = eigseis._lib.eig_last_error().decode()
    assert rc == eigseis.EIG_EINVAL
    assert ("more than one cell" in msg) == moves, msg
    assert ("ctx is NULL" in msg) == (not moves), msg


def test_forward_solve_refuses_a_deviation_step_of_two_cells():
    eigseis, g, med, rec, R = _raw_args()
    theta = np.array([10005.0, 1205.0, 0.2, 7.0, 5e13, 5e13, 5e13])
    tr = (ctypes.c_void_p * 1)(256)
    for param, step, moves in ((0, 12.0, False), (0, 20.0, True), (1, -25.0, True),
                               (1, 9.9, False), (3, 100.0, False)):
        dp = np.array([param], dtype=np.int32)
        ds = np.array([step])
        rc = eigseis._lib.forward_solve_batch(
            None, 1, ctypes.byref(g), ctypes.byref(med), theta.ctypes.data_as(ctypes.c_void_p),
            dp.ctypes.data_as(ctypes.c_void_p), ds.ctypes.data_as(ctypes.c_void_p),
            eigseis.STF_GAUSS_DERIV, ctypes.byref(R), tr, None)
        msg = eigseis._lib.eig_last_error().decode()
        assert rc == eigseis.EIG_EINVAL
        assert ("more than one cell" in msg) == moves, (param, step, msg)
