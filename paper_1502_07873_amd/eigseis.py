"""Thin ctypes binding of libeigseis.so (include/eigseis.h).

Argument marshalling only: every step of the Laplace-EIG path runs in the
library's HIP kernels.  Device arrays are torch tensors on the HIP device;
host arrays are numpy arrays.  The library is loaded from this package's
directory; if it is missing the import fails (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeigseis.so")

NTHETA = 7
EIG_OK = 0
EIG_EINVAL = -1
EIG_ENOMEM = -2
EIG_EBUDGET = -3
EIG_ENOTPD = -4
EIG_ENONFINITE = -5
EIG_EHIP = -6
EIG_EUNSUPPORTED = -7
EIG_EUNSTABLE = -8
STF_GAUSS = 0
STF_GAUSS_DERIV = 1
MEDIUM_LAYERED = 0
MEDIUM_NODAL = 1
BC_RIGID = 0
BC_ABSORBING = 1
BC_CODES = {"rigid": BC_RIGID, "absorbing": BC_ABSORBING}
PRIOR_UNIFORM = 0
PRIOR_GAUSSIAN = 1
SIGMA_GIVEN = 0
SIGMA_NOMINAL_PEAK = 1

STF_KINDS = {"gauss": STF_GAUSS, "gauss_deriv": STF_GAUSS_DERIV}


class EigError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"eigseis error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("h", ctypes.c_double),
                ("dt", ctypes.c_double), ("nsteps", ctypes.c_int32), ("bc", ctypes.c_int32)]


class Medium(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rho", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("mu", ctypes.c_void_p)]


class Receivers(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ix", ctypes.POINTER(ctypes.c_int32))]


class Prior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lo", ctypes.c_double * NTHETA),
                ("hi", ctypes.c_double * NTHETA), ("mean", ctypes.c_double * NTHETA),
                ("cov", ctypes.c_double * (NTHETA * NTHETA)), ("active", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch ships its own HIP runtime and puts it in the global symbol
    # scope; importing it first makes the library bind to that same runtime,
    # so device memory, streams and ordering are shared with torch.  Loaded
    # the other way round, the library would start the system runtime and a
    # second one would come up beside it.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "eig_ctx_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)], ctypes.c_int),
        "eig_ctx_destroy": ([vp], None),
        "eig_last_error": ([], ctypes.c_char_p),
        "eig_ctx_workspace_bytes": ([vp], ctypes.c_size_t),
        "eig_ctx_stencil_stats": ([vp, i32, vp, vp, vp, vp], ctypes.c_int),
        "eig_ctx_set_option": ([vp, ctypes.c_char_p, ctypes.c_int64], ctypes.c_int),
        "eig_ctx_get_option": ([vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)],
                               ctypes.c_int),
        "forward_solve_batch": ([vp, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "jacobian_fd": ([vp, i32, vp, vp, vp, dbl, i32, vp, i32, vp, i32, vp, vp, vp, vp, vp],
                        ctypes.c_int),
        "jacobian_sensitivity": ([vp, i32, vp, vp, vp, i32, vp, i32, vp, i32, vp, vp, vp,
                                  vp, vp], ctypes.c_int),
        "nested_mc_eig": ([vp, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "theorem3_eig": ([vp, i32, vp, vp, vp, i32, vp, vp, dbl, vp, vp, i32, vp, vp, vp, vp,
                          vp, vp, vp], ctypes.c_int),
        "laplace_eig": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "design_eval": ([vp, i32, i32, vp, i32, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "design_greedy": ([vp, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "design_greedy_noalloc": ([vp, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp],
                                  ctypes.c_int),
        "noise_sigma_peak": ([vp, vp, vp, vp, i32, dbl, vp, vp], ctypes.c_int),
        "sparse_grid_gl": ([i32, i32, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "eig_server_create": ([vp, ctypes.c_size_t, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "eig_server_destroy": ([vp], None),
        "eig_server_submit": ([vp, vp, vp, i32, vp, dbl, i32, vp, i32, dbl, vp, vp, vp, vp, vp,
                               vp, vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "eig_server_step": ([vp, i32, vp, ctypes.POINTER(i32)], ctypes.c_int),
        "eig_server_poll": ([vp, ctypes.c_int64, ctypes.POINTER(i32)], ctypes.c_int),
        "eig_server_pending": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "eig_server_memory": ([vp, ctypes.POINTER(ctypes.c_size_t),
                               ctypes.POINTER(ctypes.c_size_t),
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()
EXPORTED = ("eig_ctx_create", "eig_ctx_destroy", "eig_last_error", "eig_ctx_workspace_bytes",
            "eig_ctx_stencil_stats", "eig_ctx_set_option", "eig_ctx_get_option",
            "forward_solve_batch", "jacobian_fd", "jacobian_sensitivity", "nested_mc_eig",
            "theorem3_eig", "laplace_eig",
            "design_eval", "design_greedy", "design_greedy_noalloc", "noise_sigma_peak", "sparse_grid_gl", "eig_server_create",
            "eig_server_destroy", "eig_server_submit", "eig_server_step", "eig_server_poll",
            "eig_server_pending", "eig_server_memory")


def _check(rc: int):
    if rc != EIG_OK:
        raise EigError(rc, _lib.eig_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return t.data_ptr()


def _dev(t, name, dtype, count, optional=False):
    """A device array the library reads or writes through a raw pointer is
    refused here, before any launch, unless it is a contiguous GPU tensor of
    `dtype` holding at least `count` values (None where it is optional)."""
    import torch
    if t is None:
        if optional:
            return
        raise EigError(EIG_EINVAL, f"{name}: a device tensor is required")
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype
            or not t.is_contiguous() or t.numel() < count):
        raise EigError(EIG_EINVAL, f"{name}: expected a contiguous {dtype} device tensor "
                                   f"of at least {count} values")


def _dev_list(ts, name, dtype, counts, optional=False, entries_optional=False):
    """One device array per solve or sample (see _dev); with
    entries_optional, single entries may be None (nothing kept for them)."""
    if ts is None:
        if optional:
            return
        raise EigError(EIG_EINVAL, f"{name}: a list of device tensors is required")
    if len(ts) != len(counts):
        raise EigError(EIG_EINVAL, f"{name}: expected {len(counts)} tensors, got {len(ts)}")
    for i, (t, c) in enumerate(zip(ts, counts)):
        _dev(t, f"{name}[{i}]", dtype, c, optional=entries_optional)


def _host(a, name, count, dtype=np.float64):
    """A host array the library reads `count` values of."""
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.size < count:
        raise EigError(EIG_EINVAL, f"{name}: expected at least {count} values, got {arr.size}")
    return arr


def _theta(a, name, n):
    """Host [n][7] parameter rows."""
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.size != n * NTHETA:
        raise EigError(EIG_EINVAL, f"{name}: expected {n} x {NTHETA} values, got {arr.size}")
    return arr.reshape(n, NTHETA)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr_array(tensors):
    if tensors is None:
        return None
    arr = (ctypes.c_void_p * len(tensors))(*[None if t is None else t.data_ptr()
                                            for t in tensors])
    return arr


def make_prior(lo=None, hi=None, mean=None, cov=None, active=None) -> Prior:
    """active: indices of the inferred parameters (None: all seven)."""
    p = Prior()
    p.active = 0 if active is None else sum(1 << int(j) for j in active)
    if mean is not None:
        p.kind = PRIOR_GAUSSIAN
        p.mean[:] = list(np.asarray(mean, dtype=np.float64))
        p.cov[:] = list(np.asarray(cov, dtype=np.float64).ravel())
    else:
        p.kind = PRIOR_UNIFORM
    if lo is not None:
        p.lo[:] = list(np.asarray(lo, dtype=np.float64))
        p.hi[:] = list(np.asarray(hi, dtype=np.float64))
    return p


def sparse_grid_gl(dim: int, level: int, lo=None, hi=None):
    """Nodes [eta][dim] and weights [eta] of the Gauss-Legendre total-degree
    sparse grid (host computation in the library)."""
    count = ctypes.c_int32(0)
    lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
    hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
    rc = _lib.sparse_grid_gl(dim, level, None if lo_a is None else _np_ptr(lo_a),
                             None if hi_a is None else _np_ptr(hi_a), 0, None, None,
                             ctypes.byref(count))
    n = count.value
    if rc != EIG_OK and n <= 0:
        _check(rc)
    nodes = np.empty((n, dim))
    w = np.empty(n)
    _check(_lib.sparse_grid_gl(dim, level, None if lo_a is None else _np_ptr(lo_a),
                               None if hi_a is None else _np_ptr(hi_a), n, _np_ptr(nodes),
                               _np_ptr(w), ctypes.byref(count)))
    return nodes, w


class Context:
    """An eig_ctx on one HIP device with a workspace budget in bytes."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30):
        h = ctypes.c_void_p()
        _check(_lib.eig_ctx_create(device, budget_bytes, ctypes.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _lib.eig_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def workspace_bytes(self) -> int:
        return _lib.eig_ctx_workspace_bytes(self._h)

    def set_option(self, name: str, value: int):
        _check(_lib.eig_ctx_set_option(self._h, name.encode(), int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        _check(_lib.eig_ctx_get_option(self._h, name.encode(), ctypes.byref(v)))
        return v.value

    def stencil_stats(self, reset: bool = False) -> dict:
        """Device time (ms) from first to last stencil launch of each wave,
        launch count, grid-point updates and algorithmic HBM bytes."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        upd = ctypes.c_double()
        by = ctypes.c_double()
        _check(_lib.eig_ctx_stencil_stats(self._h, 1 if reset else 0, ctypes.byref(ms),
                                          ctypes.byref(n), ctypes.byref(upd),
                                          ctypes.byref(by)))
        return {"ms": ms.value, "launches": n.value, "updates": upd.value,
                "bytes": by.value}

    # -- marshalling helpers ------------------------------------------------
    @staticmethod
    def _grids(grids):
        arr = (Grid * len(grids))()
        for k, g in enumerate(grids):
            arr[k] = Grid(int(g[0]), int(g[1]), float(g[2]), float(g[3]), int(g[4]),
                          int(g[5]) if len(g) > 5 else BC_RIGID)
        return arr

    @staticmethod
    def _media(media, grids):
        """The library reads nz (layered) or nz*nx (nodal) float64 values from
        each device array; shorter or non-contiguous arrays are refused here."""
        import torch
        if len(media) != len(grids):
            raise EigError(EIG_EINVAL, "one medium per grid expected")
        arr = (Medium * len(media))()
        for k, ((kind, rho, lam, mu), g) in enumerate(zip(media, grids)):
            need = g[1] if kind == MEDIUM_LAYERED else g[0] * g[1]
            for a in (rho, lam, mu):
                if (a is None or a.dtype != torch.float64 or not a.is_cuda
                        or not a.is_contiguous() or a.numel() < need):
                    raise EigError(EIG_EINVAL, f"medium {k}: expected contiguous float64 "
                                               f"device arrays of at least {need} values")
            arr[k] = Medium(kind, _ptr(rho), _ptr(lam), _ptr(mu))
        return arr

    @staticmethod
    def _receivers(recs):
        keep = [np.ascontiguousarray(r, dtype=np.int32) for r in recs]
        arr = (Receivers * len(keep))()
        for k, r in enumerate(keep):
            arr[k] = Receivers(r.size, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return arr, keep

    @staticmethod
    def _jacobian_outputs(grids, receivers, per_receiver, H1, nominal, J, status):
        """Device outputs of jacobian_fd / jacobian_sensitivity (see _dev)."""
        import torch
        n = len(grids)
        if len(receivers) != n:
            raise EigError(EIG_EINVAL, "one receiver array per grid expected")
        groups = len(receivers[0]) if (per_receiver and n) else 1
        _dev(H1, "H1", torch.float64, n * groups * NTHETA * NTHETA)
        _dev(status, "status", torch.int32, n, optional=True)
        levels = [(int(g[4]) + 1) * len(r) * 2 for g, r in zip(grids, receivers)]
        _dev_list(nominal, "nominal", torch.float32, levels, optional=True,
                  entries_optional=True)
        _dev_list(J, "J", torch.float64, [c * NTHETA for c in levels], optional=True,
                  entries_optional=True)

    # -- entry points --------------------------------------------------------
    def forward_solve_batch(self, grids, media, theta, receivers, traces,
                            dev_param=None, dev_step=None, stf="gauss_deriv",
                            stream=None):
        """grids: [(nx, nz, h, dt, nsteps)]; media: [(kind, rho, lam, mu)]
        with device float64 tensors; theta: [n][7]; receivers: [int arrays];
        traces: [float32 device tensors [nsteps+1][nrec][2]]."""
        import torch
        n = len(grids)
        if len(receivers) != n:
            raise EigError(EIG_EINVAL, "one receiver array per grid expected")
        _dev_list(traces, "traces", torch.float32,
                  [(int(g[4]) + 1) * len(r) * 2 for g, r in zip(grids, receivers)])
        th = _theta(theta, "theta", n)
        recs, keep = self._receivers(receivers)
        dp = None if dev_param is None else _host(dev_param, "dev_param", n, np.int32)
        ds = None if dev_step is None else _host(dev_step, "dev_step", n)
        _check(_lib.forward_solve_batch(
            self._h, n, self._grids(grids), self._media(media, grids), _np_ptr(th),
            None if dp is None else _np_ptr(dp), None if ds is None else _np_ptr(ds),
            STF_KINDS[stf], recs, _ptr_array(traces), _stream(stream)))
        del keep

    def jacobian_fd(self, grids, media, theta, receivers, sigma, H1,
                    rel_step=1e-4, stf="gauss_deriv", sigma_mode=SIGMA_GIVEN,
                    per_receiver=False, nominal=None, J=None, status=None,
                    stream=None):
        n = len(grids)
        self._jacobian_outputs(grids, receivers, per_receiver, H1, nominal, J, status)
        th = _theta(theta, "theta", n)
        sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (n,)))
        recs, keep = self._receivers(receivers)
        _check(_lib.jacobian_fd(
            self._h, n, self._grids(grids), self._media(media, grids), _np_ptr(th),
            float(rel_step), STF_KINDS[stf], recs, int(sigma_mode), _np_ptr(sg),
            1 if per_receiver else 0, _ptr_array(nominal), _ptr_array(J), _ptr(H1),
            _ptr(status), _stream(stream)))
        del keep

    def jacobian_sensitivity(self, grids, media, theta, receivers, sigma, H1,
                             stf="gauss_deriv", sigma_mode=SIGMA_GIVEN, per_receiver=False,
                             nominal=None, J=None, status=None, stream=None):
        n = len(grids)
        self._jacobian_outputs(grids, receivers, per_receiver, H1, nominal, J, status)
        th = _theta(theta, "theta", n)
        sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (n,)))
        recs, keep = self._receivers(receivers)
        _check(_lib.jacobian_sensitivity(
            self._h, n, self._grids(grids), self._media(media, grids), _np_ptr(th),
            STF_KINDS[stf], recs, int(sigma_mode), _np_ptr(sg), 1 if per_receiver else 0,
            _ptr_array(nominal), _ptr_array(J), _ptr(H1), _ptr(status), _stream(stream)))
        del keep

    def nested_mc_eig(self, g_outer, noise, g_inner, sigma, logratio, eig=None, stream=None):
        """g_outer/noise [N][K], g_inner [M][K] device float32 (contiguous);
        logratio [N] and eig [1] (or None) device float64."""
        import torch
        if g_outer.dim() != 2 or g_inner.dim() != 2:
            raise EigError(EIG_EINVAL, "nested_mc_eig: g_outer and g_inner are [rows][K]")
        n, k = int(g_outer.shape[0]), int(g_outer.shape[1])
        m = int(g_inner.shape[0])
        if tuple(noise.shape) != (n, k) or int(g_inner.shape[1]) != k:
            raise EigError(EIG_EINVAL, "nested_mc_eig: shape mismatch")
        _dev(g_outer, "g_outer", torch.float32, n * k)
        _dev(noise, "noise", torch.float32, n * k)
        _dev(g_inner, "g_inner", torch.float32, m * k)
        _dev(logratio, "logratio", torch.float64, n)
        _dev(eig, "eig", torch.float64, 1, optional=True)
        _check(_lib.nested_mc_eig(self._h, n, m, k, _ptr(g_outer), _ptr(noise), _ptr(g_inner),
                                  float(sigma), _ptr(logratio), _ptr(eig), _stream(stream)))

    def theorem3_eig(self, grids, media, theta_star, receivers, noise, sigma, prior: Prior, w,
                     H1, H2, val, eig=None, status=None, iters=5, stf="gauss_deriv",
                     stream=None):
        """Returns theta_hat [n][7] (numpy); H1/H2/val/eig/status are device
        tensors filled asynchronously."""
        import torch
        n = len(grids)
        if len(receivers) != n:
            raise EigError(EIG_EINVAL, "one receiver array per grid expected")
        _dev_list(noise, "noise", torch.float32,
                  [(int(g[4]) + 1) * len(r) * 2 for g, r in zip(grids, receivers)])
        _dev(H1, "H1", torch.float64, n * NTHETA * NTHETA)
        _dev(H2, "H2", torch.float64, n * NTHETA * NTHETA)
        _dev(val, "val", torch.float64, n)
        _dev(eig, "eig", torch.float64, 1, optional=True)
        _dev(status, "status", torch.int32, n, optional=True)
        th = _theta(theta_star, "theta_star", n)
        wa = np.ascontiguousarray(np.broadcast_to(np.asarray(w, dtype=np.float64), (n,)))
        out = np.zeros((n, NTHETA))
        recs, keep = self._receivers(receivers)
        _check(_lib.theorem3_eig(self._h, n, self._grids(grids), self._media(media, grids), _np_ptr(th),
                                 STF_KINDS[stf], recs, _ptr_array(noise), float(sigma),
                                 ctypes.byref(prior), _np_ptr(wa), int(iters), _np_ptr(out),
                                 _ptr(H1), _ptr(H2), _ptr(val), _ptr(eig), _ptr(status),
                                 _stream(stream)))
        del keep
        return out

    def laplace_eig(self, H1, prior: Prior, w, dkl, eig, theta=None, logdet=None,
                    status=None, stream=None):
        import torch
        n = int(H1.shape[0])
        _dev(H1, "H1", torch.float64, n * NTHETA * NTHETA)
        _dev(dkl, "dkl", torch.float64, n)
        _dev(eig, "eig", torch.float64, 1)
        _dev(logdet, "logdet", torch.float64, n, optional=True)
        _dev(status, "status", torch.int32, n, optional=True)
        wa = _host(w, "w", n)
        th = None if theta is None else _host(theta, "theta", n * NTHETA)
        _check(_lib.laplace_eig(self._h, n, _ptr(H1), ctypes.byref(prior),
                                None if th is None else _np_ptr(th), _np_ptr(wa),
                                _ptr(dkl), _ptr(logdet), _ptr(eig), _ptr(status),
                                _stream(stream)))

    def design_eval(self, H1r, mask, prior: Prior, w, eig, theta=None, stream=None):
        import torch
        ns, nc = int(H1r.shape[0]), int(H1r.shape[1])
        nd = int(mask.shape[0])
        _dev(H1r, "H1r", torch.float64, ns * nc * NTHETA * NTHETA)
        _dev(mask, "mask", torch.uint8, nd * nc)
        _dev(eig, "eig", torch.float64, nd)
        wa = _host(w, "w", ns)
        th = None if theta is None else _host(theta, "theta", ns * NTHETA)
        _check(_lib.design_eval(self._h, ns, nc, _ptr(H1r), nd, _ptr(mask),
                                ctypes.byref(prior), None if th is None else _np_ptr(th),
                                _np_ptr(wa), _ptr(eig), _stream(stream)))

    def design_greedy(self, H1r, prior: Prior, w, kmax, order, curve, theta=None,
                      stream=None):
        import torch
        ns, nc = int(H1r.shape[0]), int(H1r.shape[1])
        _dev(H1r, "H1r", torch.float64, ns * nc * NTHETA * NTHETA)
        _dev(order, "order", torch.int32, max(int(kmax), 0))
        _dev(curve, "curve", torch.float64, max(int(kmax), 0))
        wa = _host(w, "w", ns)
        th = None if theta is None else _host(theta, "theta", ns * NTHETA)
        _check(_lib.design_greedy(self._h, ns, nc, _ptr(H1r), ctypes.byref(prior),
                                  None if th is None else _np_ptr(th), _np_ptr(wa),
                                  int(kmax), _ptr(order), _ptr(curve), _stream(stream)))

    def design_greedy_noalloc(self, H1r, prior: Prior, w, kmax, order, curve, theta=None,
                              stream=None):
        """design_greedy without device allocation: w [nsample] and theta
        [nsample][7] (or None for a uniform prior) are device float64
        tensors."""
        import torch
        ns, nc = int(H1r.shape[0]), int(H1r.shape[1])
        _dev(H1r, "H1r", torch.float64, ns * nc * NTHETA * NTHETA)
        _dev(w, "w", torch.float64, ns)
        _dev(theta, "theta", torch.float64, ns * NTHETA, optional=True)
        _dev(order, "order", torch.int32, max(int(kmax), 0))
        _dev(curve, "curve", torch.float64, max(int(kmax), 0))
        _check(_lib.design_greedy_noalloc(self._h, ns, nc, _ptr(H1r), ctypes.byref(prior),
                                          _ptr(theta), _ptr(w), int(kmax), _ptr(order),
                                          _ptr(curve), _stream(stream)))

    def noise_sigma_peak(self, grid, medium, theta, rel=1e-3, stf="gauss_deriv",
                         stream=None) -> float:
        out = ctypes.c_double(0.0)
        th = _theta(theta, "theta", 1)
        _check(_lib.noise_sigma_peak(self._h, self._grids([grid]), self._media([medium], [grid]),
                                     _np_ptr(th), STF_KINDS[stf], float(rel),
                                     ctypes.byref(out), _stream(stream)))
        return out.value


class Server:
    """Continuous-batching serving engine (eig_server_*) on a Context."""

    def __init__(self, ctx: "Context", budget_bytes: int, group_samples: int = 16):
        h = ctypes.c_void_p()
        _check(_lib.eig_server_create(ctx._h, budget_bytes, group_samples, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        # per query: the device tensors the engine reads (medium) or writes
        # (outputs) after submit returns, held until poll reports it done
        self._held = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.eig_server_destroy(self._h)   # waits for the device
            self._h = None
        self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, grid, medium, theta, receivers, prior: Prior, w, H1, dkl, eig,
               sigma, sigma_mode=SIGMA_GIVEN, rel_step=1e-4, stf="gauss_deriv",
               status=None, chol_status=None) -> int:
        import torch
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, NTHETA)
        n = th.shape[0]
        _dev(H1, "H1", torch.float64, n * NTHETA * NTHETA)
        _dev(dkl, "dkl", torch.float64, n)
        _dev(eig, "eig", torch.float64, 1)
        _dev(status, "status", torch.int32, n, optional=True)
        _dev(chol_status, "chol_status", torch.int32, n, optional=True)
        wa = _host(w, "w", n)
        recs, keep = Context._receivers([receivers])
        qid = ctypes.c_int64()
        _check(_lib.eig_server_submit(
            self._h, Context._grids([grid]), Context._media([medium], [grid]), n, _np_ptr(th),
            float(rel_step), STF_KINDS[stf], recs, int(sigma_mode), float(sigma),
            ctypes.byref(prior), _np_ptr(wa), _ptr(H1), _ptr(dkl), _ptr(eig), _ptr(status),
            _ptr(chol_status), ctypes.byref(qid)))
        del keep
        self._held[qid.value] = (tuple(medium), H1, dkl, eig, status, chol_status)
        return qid.value

    def step(self, max_launches: int, stream=None) -> int:
        running = ctypes.c_int32()
        _check(_lib.eig_server_step(self._h, int(max_launches), _stream(stream),
                                    ctypes.byref(running)))
        return running.value

    def poll(self, qid: int) -> bool:
        done = ctypes.c_int32()
        _check(_lib.eig_server_poll(self._h, int(qid), ctypes.byref(done)))
        if done.value:
            self._held.pop(int(qid), None)
        return bool(done.value)

    def memory(self) -> dict:
        """Arena budget, bytes in use now and the most ever in use."""
        b, u, p = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.eig_server_memory(self._h, ctypes.byref(b), ctypes.byref(u),
                                      ctypes.byref(p)))
        return {"budget": b.value, "in_use": u.value, "peak": p.value}

    def pending(self):
        q, r = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.eig_server_pending(self._h, ctypes.byref(q), ctypes.byref(r)))
        return q.value, r.value
