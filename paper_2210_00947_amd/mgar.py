"""Thin ctypes binding of libmgar.so (include/mgar.h).

Argument marshalling only: every numerical step runs in the HIP library. The
functions keep the C names. Tensors are torch CUDA (HIP) tensors, FP64 and
contiguous; work is enqueued on torch's current stream unless the handle was
given another one. There is no fallback: if the library is missing, or a
tensor is not on the GPU, a call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgar.so")

MGAR_OK = 0
MGAR_W_NOT_CONVERGED = 1
MGAR_E_ARG = -1
MGAR_E_DIMS = -2
MGAR_E_SINGULAR = -3
MGAR_E_HIP = -4
MGAR_E_NOT_SPD = -5
MGAR_E_PRECISION = -6
MGAR_E_STATE = -7
PATH_MGCG, PATH_ACCEPT, PATH_FALLBACK = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

EXPORTS = [
    "mgar_default_params", "mgar_setup", "mgar_destroy", "mgar_set_stream", "mgar_set_timing", "mgar_strerror",
    "mgar_sizes", "mgar_load_vector", "mgar_density_filter", "mgcg_solve", "mgar_solve",
    "sens_filter", "oc_update", "mgar_sens_oc", "mgar_reset", "mgar_op_apply", "mgar_op_jacobi",
    "mgar_op_restrict", "mgar_op_prolong", "mgar_op_coarsen", "mgar_build_hierarchy",
    "mgar_vcycle", "mgar_op_dk", "mgar_op_bf16", "mgar_autotune", "mgar_tune_get",
    "mgar_tune_set", "mgar_set_graphs", "mgar_residual", "mgar_net_create", "mgar_net_destroy", "mgar_net_sizes",
    "mgar_net_set_params", "mgar_net_get_params", "mgar_net_set_source", "mgar_net_infer", "mgar_net_output",
    "mgar_net_grad",
    "mgar_net_train_step", "mgar_batch_setup", "mgar_batch_destroy", "mgar_batch_layout",
    "mgar_batch_set_graph", "mgar_batch_set_block", "mgar_batch_get_block", "mgar_batch_autotune",
    "mgar_batch_load_vector", "mgcg_batch_solve", "mgar_batch_solve",
    "mgar_profile", "mgar_profile_read", "mgar_residual_noalloc", "mgar_set_filter_radius",
    "mgar_smooth_boundary",
]


class mgar_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nelx", ctypes.c_int), ("nely", ctypes.c_int),
        ("nelz", ctypes.c_int), ("levels", ctypes.c_int),
        ("fix_lo", ctypes.c_int * 3), ("fix_hi", ctypes.c_int * 3),
        ("k0", ctypes.c_double), ("kmin", ctypes.c_double), ("penal", ctypes.c_double),
        ("omega", ctypes.c_double), ("n_basis", ctypes.c_int), ("eps_accept", ctypes.c_double),
        ("cg_max", ctypes.c_int), ("basis_x0_zero", ctypes.c_int), ("precision", ctypes.c_int),
        ("filter_r", ctypes.c_double), ("inner_tol", ctypes.c_double),
    ]


class mgar_stats(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int), ("cg_iters", ctypes.c_int), ("vcycles", ctypes.c_int),
        ("refinements", ctypes.c_int), ("res_ca", ctypes.c_double),
        ("res_final", ctypes.c_double), ("ms", ctypes.c_float),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MgarError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib():
    """Load libmgar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2210_00947_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, VP = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        LL = ctypes.c_longlong
        L.mgar_default_params.argtypes = [ctypes.POINTER(mgar_params)]
        L.mgar_default_params.restype = None
        L.mgar_setup.argtypes = [ctypes.POINTER(mgar_params), VP, ctypes.POINTER(P)]
        L.mgar_destroy.argtypes = [P]
        L.mgar_destroy.restype = None
        L.mgar_set_stream.argtypes = [P, VP]
        L.mgar_set_timing.argtypes = [P, I]
        L.mgar_strerror.argtypes = [I]
        L.mgar_strerror.restype = ctypes.c_char_p
        L.mgar_sizes.argtypes = [P, I, ctypes.POINTER(LL), ctypes.POINTER(LL)]
        L.mgar_load_vector.argtypes = [P, VP, VP]
        L.mgar_density_filter.argtypes = [P, VP, VP]
        for f in ("mgcg_solve", "mgar_solve"):
            getattr(L, f).argtypes = [P, VP, VP, VP, D, VP, ctypes.POINTER(mgar_stats)]
        L.sens_filter.argtypes = [P, VP, VP, VP, VP, VP, ctypes.POINTER(D)]
        L.oc_update.argtypes = [P, VP, VP, VP, D, D, VP, ctypes.POINTER(D)]
        L.mgar_sens_oc.argtypes = [P, VP, VP, VP, VP, D, D, VP, VP, VP, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.mgar_reset.argtypes = [P]
        L.mgar_op_apply.argtypes = [P, I, VP, VP, VP]
        L.mgar_op_jacobi.argtypes = [P, I, VP, VP, VP, VP]
        L.mgar_op_restrict.argtypes = [P, I, VP, VP]
        L.mgar_op_prolong.argtypes = [P, I, VP, VP]
        L.mgar_op_coarsen.argtypes = [P, I, VP, VP]
        L.mgar_build_hierarchy.argtypes = [P, VP]
        L.mgar_vcycle.argtypes = [P, VP, VP, VP]
        L.mgar_op_dk.argtypes = [P, VP, VP, VP]
        L.mgar_op_bf16.argtypes = [P, VP, VP]
        L.mgar_profile.argtypes = [P, ctypes.c_uint]
        L.mgar_profile_read.argtypes = [P, ctypes.POINTER(LL), ctypes.POINTER(D), ctypes.POINTER(D)]
        L.mgar_set_filter_radius.argtypes = [P, D]
        L.mgar_smooth_boundary.argtypes = [P, VP, D, D, I, VP, VP, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.mgar_residual_noalloc.argtypes = [ctypes.POINTER(mgar_params), VP, VP, VP, VP, VP]
        for f in EXPORTS:
            if f not in ("mgar_default_params", "mgar_destroy", "mgar_strerror", "mgar_batch_destroy",
                         "mgar_net_destroy"):
                getattr(L, f).restype = I
        _lib = L
    return _lib


def mgar_residual_noalloc(params: mgar_params, xphys, q, T, relres, stream=None):
    """||q - K(xphys) T|| / ||q|| into relres (a one-entry FP64 GPU tensor), enqueued on
    `stream` (default: torch's current stream) without a host synchronisation and
    without any device allocation (the library's static partial-sum array)."""
    import torch
    ne = params.nelx * params.nely * (params.nelz if params.dim == 3 else 1)
    nn = (params.nelx + 1) * (params.nely + 1) * ((params.nelz + 1) if params.dim == 3 else 1)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().mgar_residual_noalloc(ctypes.byref(params), _ptr(xphys, ne, "xphys"), _ptr(q, nn, "q"),
                                       _ptr(T, nn, "T"), _ptr(relres, 1, "relres"), ctypes.c_void_p(stream)),
           "mgar_residual_noalloc")


def strerror(code: int) -> str:
    return lib().mgar_strerror(int(code)).decode()


def _ptr(t, n=None, name="tensor"):
    """Device pointer of an FP64 contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    import torch
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _check(rc, where, warn_ok=True):
    if rc < 0 or (rc > 0 and not warn_ok):
        raise MgarError(rc, where)
    return rc


def params_for(prob, n_basis=2, eps_accept=None, cg_max=200, omega=0.8, basis_x0_zero=False,
               precision=PREC_FP64, inner_tol=None):
    """mgar_params from a workloads.Problem description."""
    p = mgar_params()
    lib().mgar_default_params(ctypes.byref(p))
    p.dim, p.nelx, p.nely = prob.dim, prob.nelx, prob.nely
    p.nelz = prob.nelz if prob.dim == 3 else 0
    p.levels = prob.levels
    for a in range(3):
        p.fix_lo[a] = prob.fix_lo[a]
        p.fix_hi[a] = prob.fix_hi[a]
    p.k0, p.kmin, p.penal = prob.k0, prob.kmin, prob.penal
    p.omega = omega
    p.n_basis = n_basis
    p.eps_accept = prob.tol if eps_accept is None else eps_accept
    p.cg_max = cg_max
    p.basis_x0_zero = int(bool(basis_x0_zero))
    p.precision = precision
    p.filter_r = prob.filter_r
    if inner_tol is not None:
        p.inner_tol = inner_tol
    return p


class Handle:
    """Owns one mgar_handle. Methods keep the names of the C entry points."""

    def __init__(self, params: mgar_params, stream=None):
        import torch
        self._L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(self._L.mgar_setup(ctypes.byref(params), ctypes.c_void_p(stream), ctypes.byref(h)),
               "mgar_setup", warn_ok=False)
        self.h = h
        self.params = params
        nn, ne = ctypes.c_longlong(), ctypes.c_longlong()
        self._L.mgar_sizes(h, 0, ctypes.byref(nn), ctypes.byref(ne))
        self.N, self.E = nn.value, ne.value

    def close(self):
        if getattr(self, "h", None):
            self._L.mgar_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self, level):
        nn, ne = ctypes.c_longlong(), ctypes.c_longlong()
        _check(self._L.mgar_sizes(self.h, level, ctypes.byref(nn), ctypes.byref(ne)), "mgar_sizes")
        return nn.value, ne.value

    def set_stream(self, stream):
        _check(self._L.mgar_set_stream(self.h, ctypes.c_void_p(stream)), "mgar_set_stream")

    def mgar_set_timing(self, on):
        _check(self._L.mgar_set_timing(self.h, int(bool(on))), "mgar_set_timing")

    def mgar_load_vector(self, Qe, q):
        _check(self._L.mgar_load_vector(self.h, _ptr(Qe, self.E, "Qe"), _ptr(q, self.N, "q")),
               "mgar_load_vector")

    def mgar_density_filter(self, x, xphys):
        _check(self._L.mgar_density_filter(self.h, _ptr(x, self.E, "x"), _ptr(xphys, self.E, "xphys")),
               "mgar_density_filter")

    def _solve(self, fn, xphys, q, T0, tol, T):
        st = mgar_stats()
        rc = fn(self.h, _ptr(xphys, self.E, "xphys"), _ptr(q, self.N, "q"),
                _ptr(T0, self.N, "T0"), float(tol), _ptr(T, self.N, "T"), ctypes.byref(st))
        _check(rc, fn.__name__)
        d = st.as_dict()
        d["rc"] = rc
        return d

    def mgcg_solve(self, xphys, q, T0, tol, T):
        return self._solve(self._L.mgcg_solve, xphys, q, T0, tol, T)

    def mgar_solve(self, xphys, q, T0, tol, T):
        return self._solve(self._L.mgar_solve, xphys, q, T0, tol, T)

    def sens_filter(self, xphys, T, q, dc, dv):
        c = ctypes.c_double()
        _check(self._L.sens_filter(self.h, _ptr(xphys, self.E, "xphys"), _ptr(T, self.N, "T"),
                                   _ptr(q, self.N, "q"), _ptr(dc, self.E, "dc"),
                                   _ptr(dv, self.E, "dv"), ctypes.byref(c)), "sens_filter")
        return c.value

    def oc_update(self, x, dc, dv, volfrac, move, x_new):
        lam = ctypes.c_double()
        _check(self._L.oc_update(self.h, _ptr(x, self.E, "x"), _ptr(dc, self.E, "dc"),
                                 _ptr(dv, self.E, "dv"), float(volfrac), float(move),
                                 _ptr(x_new, self.E, "x_new"), ctypes.byref(lam)), "oc_update")
        return lam.value

    def mgar_sens_oc(self, xphys, T, q, x, volfrac, move, dc, dv, x_new):
        """sens_filter then oc_update with one host synchronisation; returns
        (compliance, lambda)."""
        c, lam = ctypes.c_double(), ctypes.c_double()
        _check(self._L.mgar_sens_oc(self.h, _ptr(xphys, self.E, "xphys"), _ptr(T, self.N, "T"),
                                    _ptr(q, self.N, "q"), _ptr(x, self.E, "x"), float(volfrac), float(move),
                                    _ptr(dc, self.E, "dc"), _ptr(dv, self.E, "dv"),
                                    _ptr(x_new, self.E, "x_new"), ctypes.byref(c), ctypes.byref(lam)),
               "mgar_sens_oc")
        return c.value, lam.value

    def mgar_reset(self):
        _check(self._L.mgar_reset(self.h), "mgar_reset")

    def mgar_op_apply(self, level, k, x, y):
        nn, ne = self.sizes(level)
        _check(self._L.mgar_op_apply(self.h, level, _ptr(k, ne, "k"), _ptr(x, nn, "x"),
                                     _ptr(y, nn, "y")), "mgar_op_apply")

    def mgar_op_jacobi(self, level, k, b, x, out):
        nn, ne = self.sizes(level)
        _check(self._L.mgar_op_jacobi(self.h, level, _ptr(k, ne, "k"), _ptr(b, nn, "b"),
                                      _ptr(x, nn, "x"), _ptr(out, nn, "out")), "mgar_op_jacobi")

    def mgar_op_restrict(self, level, rf, rc):
        nf, _ = self.sizes(level)
        nc, _ = self.sizes(level + 1)
        _check(self._L.mgar_op_restrict(self.h, level, _ptr(rf, nf, "rf"), _ptr(rc, nc, "rc")),
               "mgar_op_restrict")

    def mgar_op_prolong(self, level, xc, xf):
        nf, _ = self.sizes(level)
        nc, _ = self.sizes(level + 1)
        _check(self._L.mgar_op_prolong(self.h, level, _ptr(xc, nc, "xc"), _ptr(xf, nf, "xf")),
               "mgar_op_prolong")

    def mgar_op_coarsen(self, level, kf, kc):
        _, ef = self.sizes(level)
        _, ec = self.sizes(level + 1)
        _check(self._L.mgar_op_coarsen(self.h, level, _ptr(kf, ef, "kf"), _ptr(kc, ec, "kc")),
               "mgar_op_coarsen")

    def mgar_build_hierarchy(self, xphys):
        _check(self._L.mgar_build_hierarchy(self.h, _ptr(xphys, self.E, "xphys")),
               "mgar_build_hierarchy", warn_ok=False)

    def mgar_vcycle(self, b, x0, x):
        _check(self._L.mgar_vcycle(self.h, _ptr(b, self.N, "b"), _ptr(x0, self.N, "x0"),
                                   _ptr(x, self.N, "x")), "mgar_vcycle")

    def mgar_op_dk(self, xphys, r, b):
        _check(self._L.mgar_op_dk(self.h, _ptr(xphys, self.E, "xphys"), _ptr(r, self.N, "r"),
                                  _ptr(b, self.N, "b")), "mgar_op_dk")


    def mgar_op_bf16(self, x, out):
        """out: int16 GPU tensor with E entries (the BF16 bit patterns)."""
        import torch
        if out.dtype != torch.int16 or not out.is_cuda or out.numel() != self.E:
            raise ValueError("out must be an int16 GPU tensor with E entries")
        _check(self._L.mgar_op_bf16(self.h, _ptr(x, self.E, "x"), ctypes.c_void_p(out.data_ptr())),
               "mgar_op_bf16")

    def mgar_smooth_boundary(self, dc, volfrac, r, rho, ns=None, nsub=4):
        """Eq 24-27 post-process of the design whose sensitivities are dc; returns (level, volume)."""
        lv, vol = ctypes.c_double(), ctypes.c_double()
        _check(self._L.mgar_smooth_boundary(self.h, _ptr(dc, self.E, "dc"), float(volfrac), float(r), int(nsub),
                                            _ptr(rho, self.E, "rho"), _ptr(ns, self.N, "ns"), ctypes.byref(lv),
                                            ctypes.byref(vol)), "mgar_smooth_boundary")
        return lv.value, vol.value

    def mgar_set_filter_radius(self, r):
        _check(self._L.mgar_set_filter_radius(self.h, float(r)), "mgar_set_filter_radius")

    def mgar_set_graphs(self, on):
        _check(self._L.mgar_set_graphs(self.h, int(bool(on))), "mgar_set_graphs")

    def mgar_residual(self, xphys, q, T):
        r = ctypes.c_double()
        _check(self._L.mgar_residual(self.h, _ptr(xphys, self.E), _ptr(q, self.N), _ptr(T, self.N),
                                     ctypes.byref(r)), "mgar_residual")
        return r.value

    def mgar_autotune(self, reps=20):
        """Time the candidate launch shapes and install the fastest; returns the
        winning times (microseconds) as a list indexed [cls][level][mode]."""
        L = self.params.levels
        buf = (ctypes.c_double * (2 * L * 7))()
        _check(self._L.mgar_autotune(self.h, int(reps), buf), "mgar_autotune")
        return [[[buf[(c * L + l) * 7 + m] for m in range(7)] for l in range(L)] for c in range(2)]

    def mgar_tune_get(self, cls, level, mode):
        s = (ctypes.c_int * 4)()
        _check(self._L.mgar_tune_get(self.h, int(cls), int(level), int(mode), s), "mgar_tune_get")
        return list(s)

    def mgar_tune_set(self, cls, level, mode, shape):
        s = (ctypes.c_int * 4)(*[int(v) for v in shape])
        _check(self._L.mgar_tune_set(self.h, int(cls), int(level), int(mode), s), "mgar_tune_set")

    def mgar_profile(self, mode_mask):
        _check(self._L.mgar_profile(self.h, ctypes.c_uint(mode_mask)), "mgar_profile")

    def mgar_profile_read(self):
        n, ms, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        _check(self._L.mgar_profile_read(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)),
               "mgar_profile_read")
        return n.value, ms.value, by.value


def n_on(maxit: int) -> int:
    """Activation parameter of the loop: MGCG while the cycle is below 2/15 of maxit."""
    return (2 * maxit) // 15


class Batch:
    """Owns one mgar_batch (many designs solved together). Methods keep the
    names of the C entry points; vectors are concatenations over designs
    (offsets in self.node_off / self.elem_off)."""

    def __init__(self, params_list, stream=None):
        import torch
        self._L = lib()
        n = len(params_list)
        arr = (mgar_params * n)(*params_list)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        b = ctypes.c_void_p()
        _check(self._L.mgar_batch_setup(arr, n, ctypes.c_void_p(stream), ctypes.byref(b)),
               "mgar_batch_setup")
        self.b = b
        self.n = n
        no = (ctypes.c_longlong * (n + 1))()
        eo = (ctypes.c_longlong * (n + 1))()
        _check(self._L.mgar_batch_layout(self.b, no, eo), "mgar_batch_layout")
        self.node_off = list(no)
        self.elem_off = list(eo)
        self.N = self.node_off[-1]
        self.E = self.elem_off[-1]

    def close(self):
        if getattr(self, "b", None):
            self._L.mgar_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mgar_batch_set_graph(self, use_graph):
        _check(self._L.mgar_batch_set_graph(self.b, int(bool(use_graph))), "mgar_batch_set_graph")

    def mgar_batch_set_block(self, bs):
        _check(self._L.mgar_batch_set_block(self.b, int(bs)), "mgar_batch_set_block")

    def mgar_batch_get_block(self):
        v = ctypes.c_int()
        _check(self._L.mgar_batch_get_block(self.b, ctypes.byref(v)), "mgar_batch_get_block")
        return v.value

    def mgar_batch_autotune(self, xphys, q, tol, reps=3):
        """Times the candidate block sizes (256, 128, 64) on batched MGCG solves
        of (xphys, q) and keeps the fastest; returns (block size, {size: us})."""
        bs = ctypes.c_int()
        us = (ctypes.c_float * 3)()
        _check(self._L.mgar_batch_autotune(self.b, _ptr(xphys, self.E), _ptr(q, self.N), ctypes.c_double(tol),
                                           int(reps), ctypes.byref(bs), us), "mgar_batch_autotune")
        return bs.value, {256: us[0], 128: us[1], 64: us[2]}

    def mgar_batch_load_vector(self, Qe, q):
        _check(self._L.mgar_batch_load_vector(self.b, _ptr(Qe, self.E), _ptr(q, self.N)),
               "mgar_batch_load_vector")

    def _solve(self, fn, name, xphys, q, T0, tol, T):
        stats = (mgar_stats * self.n)()
        rc = fn(self.b, _ptr(xphys, self.E), _ptr(q, self.N),
                _ptr(T0, self.N) if T0 is not None else None, ctypes.c_double(tol), _ptr(T, self.N), stats)
        if rc < 0:
            raise MgarError(rc, name)
        out = [s.as_dict() for s in stats]
        for s in out:
            s["rc"] = rc
        return out

    def mgcg_batch_solve(self, xphys, q, T0, tol, T):
        return self._solve(self._L.mgcg_batch_solve, "mgcg_batch_solve", xphys, q, T0, tol, T)

    def mgar_batch_solve(self, xphys, q, T0, tol, T):
        return self._solve(self._L.mgar_batch_solve, "mgar_batch_solve", xphys, q, T0, tol, T)


class Net:
    """Owns one mgar_net (the learned initial guess on the element grid);
    methods keep the C names."""

    def __init__(self, params: mgar_params, channels=(16, 32, 64, 64), stream=None):
        import torch
        self._L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        ch = (ctypes.c_int * len(channels))(*[int(c) for c in channels])
        n = ctypes.c_void_p()
        _check(self._L.mgar_net_create(ctypes.byref(params), len(channels), ch, ctypes.c_void_p(stream),
                                       ctypes.byref(n)), "mgar_net_create")
        self.n = n
        npar = ctypes.c_longlong()
        _check(self._L.mgar_net_sizes(self.n, ctypes.byref(npar)), "mgar_net_sizes")
        self.nparams = npar.value
        self.channels = tuple(int(c) for c in channels)
        self.E = params.nelx * params.nely * params.nelz
        self.N = (params.nelx + 1) * (params.nely + 1) * (params.nelz + 1)
        self.cells = (params.nelz, params.nely, params.nelx)

    def close(self):
        if getattr(self, "n", None):
            self._L.mgar_net_destroy(self.n)
            self.n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mgar_net_set_source(self, qe):
        _check(self._L.mgar_net_set_source(self.n, _ptr(qe, self.E)), "mgar_net_set_source")

    def mgar_net_set_params(self, theta):
        import numpy as np
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.nparams
        _check(self._L.mgar_net_set_params(self.n, a.ctypes.data_as(ctypes.c_void_p)), "mgar_net_set_params")

    def mgar_net_get_params(self):
        import numpy as np
        a = np.empty(self.nparams, dtype=np.float32)
        _check(self._L.mgar_net_get_params(self.n, a.ctypes.data_as(ctypes.c_void_p)), "mgar_net_get_params")
        return a

    def mgar_net_infer(self, xphys, scale, T):
        _check(self._L.mgar_net_infer(self.n, _ptr(xphys, self.E), ctypes.c_double(scale), _ptr(T, self.N)),
               "mgar_net_infer")

    def mgar_net_output(self):
        import numpy as np
        a = np.empty(self.cells, dtype=np.float32)
        _check(self._L.mgar_net_output(self.n, a.ctypes.data_as(ctypes.c_void_p)), "mgar_net_output")
        return a

    def mgar_net_grad(self, xphys, T, scale):
        import numpy as np
        g = np.empty(self.nparams, dtype=np.float64)
        loss = ctypes.c_double()
        _check(self._L.mgar_net_grad(self.n, _ptr(xphys, self.E), _ptr(T, self.N), ctypes.c_double(scale),
                                     g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)), "mgar_net_grad")
        return loss.value, g

    def mgar_net_train_step(self, xphys, T, scale, lr, want_loss=True):
        """One Adam step; returns the loss (a host synchronisation on the
        network's stream) or, with want_loss=False, None without waiting."""
        loss = ctypes.c_double()
        _check(self._L.mgar_net_train_step(self.n, _ptr(xphys, self.E), _ptr(T, self.N), ctypes.c_double(scale),
                                           ctypes.c_double(lr), ctypes.byref(loss) if want_loss else None),
               "mgar_net_train_step")
        return loss.value if want_loss else None
