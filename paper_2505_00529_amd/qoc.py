"""Thin Python binding of the C ABI in include/qoc.h (argument marshalling only).

Every computation runs in the HIP library ``libqoc.so`` built in-tree for gfx950
(``python -m paper_2505_00529_amd.build``).  There is no fallback: if the library is
missing or the device is unavailable, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqoc.so")

QOC_OK = 0
QOC_ERR_INVALID_ARG = -1
QOC_ERR_NOT_SYMMETRIC = -2
QOC_ERR_STATE = -3
QOC_ERR_UNSUPPORTED = -4
QOC_ERR_NOCONV = -5
QOC_ERR_DEVICE = -6
QOC_ERR_OOM = -7
QOC_ERR_NOT_CONVERGED = -8

QOC_BASIS_FOURIER = 0
QOC_BASIS_IDENTITY = 1
QOC_BASIS_DENSE = 2
QOC_TR_SUBPROBLEM_DEFAULT = 0
QOC_TR_SUBPROBLEM_CG = 1

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_st = ctypes.c_int32

# name -> (restype, argtypes)
SIGNATURES = {
    "qoc_create": (_st, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "qoc_destroy": (None, [_vp]),
    "qoc_set_stream": (_st, [_vp, _vp]),
    "qoc_set_system": (_st, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "qoc_set_target": (_st, [_vp, _dp]),
    "qoc_set_control_basis": (_st, [_vp, ctypes.c_int, _i32, ctypes.c_double, _i32, _dp]),
    "qoc_set_weights": (_st, [_vp, ctypes.c_double, ctypes.c_double]),
    "qoc_get_num_params": (_st, [_vp, ctypes.POINTER(_i32)]),
    "qoc_cost": (_st, [_vp, _dp, _dp]),
    "qoc_grad": (_st, [_vp, _dp, _dp, _dp]),
    "qoc_hess": (_st, [_vp, _dp, _dp, _dp, _dp]),
    "qoc_hvp": (_st, [_vp, _dp, _dp, _dp, _dp]),
    "qoc_hess_many": (_st, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "qoc_grad_many": (_st, [_vp, _i32, _dp, _dp, _dp]),
    "qoc_cost_dev": (_st, [_vp, _vp, _vp]),
    "qoc_grad_dev": (_st, [_vp, _vp, _vp, _vp]),
    "qoc_hess_dev": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "qoc_hvp_dev": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "qoc_hess_many_dev": (_st, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "qoc_hess_many_dev_noalloc": (_st, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "qoc_sync": (_st, [_vp]),
    "qoc_step_propagators": (_st, [_vp, _dp, _i32, _dp, _dp, _dp]),
    "qoc_set_checkpoint_interval": (_st, [_vp, _i32]),
    "qoc_set_jacobi_sweep_cap": (_st, [_vp, _i32]),
    "qoc_set_jacobi_tolerance": (_st, [_vp, ctypes.c_double]),
    "qoc_memory_usage": (_st, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "qoc_tr_solve": (_st, [_vp, _dp, ctypes.c_double, _i32, _dp, _dp, ctypes.POINTER(_i32)]),
    "qoc_tr_solve_many": (_st, [_vp, _i32, _dp, _dp, ctypes.c_double, _i32, _dp, _dp, ctypes.POINTER(_i32),
                                ctypes.POINTER(_i32)]),
    "qoc_hess_many_targets": (_st, [_vp, _i32, _dp, _dp, _dp, _dp, _dp]),
    "qoc_control_coords": (_st, [_vp, _i32, _dp, _dp, ctypes.POINTER(_i32)]),
    "qoc_tr_gradient_norms": (_st, [_vp, _i32, _dp, _dp, _dp]),
    "qoc_set_tr_step_tolerance": (_st, [_vp, ctypes.c_double]),
    "qoc_set_tr_subproblem": (_st, [_vp, _i32]),
    "qoc_set_system_hermitian": (_st, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "qoc_set_system_multi": (_st, [_vp, _i32, _i32, _dp, _dp, _dp, _dp]),
    "qoc_eval_controls": (_st, [_vp, _dp, _dp, _dp, _dp, _dp]),
    "qoc_set_eig_chunk": (_st, [_vp, _i32]),
    "qoc_tr_solve_bfgs_many": (_st, [_vp, _i32, _dp, _dp, ctypes.c_double, _i32, _dp, _dp, ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32)]),
    "qoc_bfgs_update": (_st, [_i32, _dp, _dp, _dp, _dp, _i32]),
    "qoc_params_from_coords": (_st, [_vp, _i32, _dp, _dp]),
    "qoc_batch_create": (_st, [ctypes.c_int, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "qoc_batch_destroy": (None, [_vp]),
    "qoc_batch_hess": (_st, [_vp, ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                             ctypes.POINTER(_dp)]),
    "qoc_batch_hess_unbatched": (_st, [_vp, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                       ctypes.POINTER(_dp), ctypes.POINTER(_dp)]),
    "qoc_batch_last_error": (ctypes.c_char_p, [_vp]),
    "qoc_batch_autotune": (_st, [_vp, ctypes.POINTER(_dp)]),
    "qoc_batch_get_config": (_st, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "qoc_batch_set_config": (_st, [_vp, _i32, _i32, _i32]),
    "qoc_batch_last_ms": (_st, [_vp, _dp]),
    "qoc_batch_memory": (_st, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "qoc_profile_enable": (_st, [_vp, _i32]),
    "qoc_profile_kernel_ms": (_st, [_vp, ctypes.c_char_p, _dp, ctypes.POINTER(_i32)]),
    "qoc_jacobi_stats": (_st, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), _i32]),
    "qoc_mlp_create": (_st, [ctypes.c_int, _vp, _i32, _i32, _i32, _i32, ctypes.POINTER(_vp)]),
    "qoc_mlp_destroy": (None, [_vp]),
    "qoc_mlp_num_params": (ctypes.c_int64, [_vp]),
    "qoc_mlp_set_params": (_st, [_vp, _fp]),
    "qoc_mlp_get_params": (_st, [_vp, _fp]),
    "qoc_mlp_get_grads": (_st, [_vp, _fp]),
    "qoc_mlp_forward": (_st, [_vp, _i32, _vp, _vp]),
    "qoc_mlp_loss_grad": (_st, [_vp, _i32, _vp, _vp, _vp]),
    "qoc_mlp_train_step": (_st, [_vp, _i32, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, _vp]),
    "qoc_mlp_sync": (_st, [_vp]),
    "qoc_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "qoc_status_string": (ctypes.c_char_p, [_st]),
    "qoc_last_error": (ctypes.c_char_p, [_vp]),
}


class QocError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"qoc status {status}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libqoc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2505_00529_amd.build`")
        handle = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    return lib().qoc_status_string(status).decode()


def _f64(x, size=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if size is not None and a.size != size:
        raise ValueError(f"expected {size} values, got {a.size}")
    return a


def _cplx(x, n) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(n))
    return a.view(np.float64)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


class Problem:
    """Handle over one system + control basis (``qoc_problem``)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self._h = _vp()
        st = lib().qoc_create(device, _vp(stream) if stream else None, ctypes.byref(self._h))
        if st != QOC_OK:
            raise QocError(st, status_string(st))
        self.n = 0
        self.P = 0

    # -- lifecycle
    def close(self):
        if self._h:
            lib().qoc_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _check(self, st: int):
        if st != QOC_OK:
            raise QocError(st, lib().qoc_last_error(self._h).decode())

    # -- configuration
    def set_stream(self, stream: Optional[int]):
        """Enqueue later calls on this hipStream_t handle; 0 / None is the null stream."""
        self._check(lib().qoc_set_stream(self._h, _vp(stream) if stream else None))

    def set_system(self, h0, m, psi0, psi_target):
        h0 = _f64(h0)
        n = h0.shape[0]
        m = _f64(m, n * n)
        self._check(lib().qoc_set_system(self._h, n, _ptr(h0), _ptr(m), _ptr(_cplx(psi0, n)),
                                         _ptr(_cplx(psi_target, n))))
        self.n = n

    def eval_controls(self, f, hessian: bool = True):
        """(cost, J^T dC/df, J^T d2C/df2 J or None, dC/df) at control samples f, with the model's
        Jacobian J set as a DENSE basis."""
        fv = _f64(f, self.nt)
        c = np.zeros(1)
        g = np.zeros(self.P)
        h = np.zeros((self.P, self.P)) if hessian else None
        w = np.zeros(self.nt)
        self._check(lib().qoc_eval_controls(self._h, _ptr(fv), _ptr(c), _ptr(g), _ptr(h), _ptr(w)))
        return float(c[0]), g, h, w

    def set_system_multi(self, h0, ms, psi0, psi_target):
        """Real symmetric H0 and K = len(ms) control operators M_k (K <= 3); the control basis is
        set afterwards (one nt x P matrix per direction)."""
        h0 = _f64(h0)
        n = int(np.asarray(h0).shape[0])
        mv = np.ascontiguousarray(np.asarray(ms, dtype=np.float64).reshape(-1, n, n))
        self._check(lib().qoc_set_system_multi(self._h, n, mv.shape[0], _ptr(h0), _ptr(mv), _ptr(_cplx(psi0, n)),
                                               _ptr(_cplx(psi_target, n))))
        self.n = n
        self.ndir = mv.shape[0]

    def set_system_hermitian(self, h0, m, psi0, psi_target):
        """Complex Hermitian H0, M (n x n complex); evaluated through the exact real embedding."""
        h0 = np.ascontiguousarray(np.asarray(h0, dtype=np.complex128))
        n = h0.shape[0]
        m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(n, n))
        hv, mv = h0.view(np.float64), m.view(np.float64)
        self._check(lib().qoc_set_system_hermitian(self._h, n, _ptr(hv), _ptr(mv), _ptr(_cplx(psi0, n)),
                                                   _ptr(_cplx(psi_target, n))))
        self.n = n

    def set_target(self, psi_target):
        self._check(lib().qoc_set_target(self._h, _ptr(_cplx(psi_target, self.n))))

    def set_control_basis(self, kind: int, nt: int, dt: float, k_or_p: int = 0, b=None):
        bb = None if b is None else _f64(b)
        self._check(lib().qoc_set_control_basis(self._h, kind, nt, dt, k_or_p, _ptr(bb)))
        p = _i32()
        self._check(lib().qoc_get_num_params(self._h, ctypes.byref(p)))
        self.P = p.value
        self.nt = nt

    def set_weights(self, gamma: float, rho: float):
        self._check(lib().qoc_set_weights(self._h, gamma, rho))

    def set_eig_chunk(self, steps: int):
        """Length of the warm-started eigen chains (0: automatic, 1..32: fixed)."""
        self._check(lib().qoc_set_eig_chunk(self._h, int(steps)))

    def set_checkpoint_interval(self, steps: int):
        self._check(lib().qoc_set_checkpoint_interval(self._h, steps))

    def set_jacobi_sweep_cap(self, max_sweeps: int):
        self._check(lib().qoc_set_jacobi_sweep_cap(self._h, max_sweeps))

    def set_jacobi_tolerance(self, tol_rel: float):
        self._check(lib().qoc_set_jacobi_tolerance(self._h, tol_rel))

    def memory_usage(self) -> Tuple[int, int]:
        c = ctypes.c_int64()
        pk = ctypes.c_int64()
        self._check(lib().qoc_memory_usage(self._h, ctypes.byref(c), ctypes.byref(pk)))
        return c.value, pk.value

    # -- evaluation (host arrays)
    def cost(self, theta) -> float:
        th = _f64(theta, self.P)
        c = np.zeros(1)
        self._check(lib().qoc_cost(self._h, _ptr(th), _ptr(c)))
        return float(c[0])

    def grad(self, theta):
        th = _f64(theta, self.P)
        c = np.zeros(1)
        g = np.zeros(self.P)
        self._check(lib().qoc_grad(self._h, _ptr(th), _ptr(c), _ptr(g)))
        return float(c[0]), g

    def hess(self, theta):
        th = _f64(theta, self.P)
        c = np.zeros(1)
        g = np.zeros(self.P)
        h = np.zeros((self.P, self.P))
        self._check(lib().qoc_hess(self._h, _ptr(th), _ptr(c), _ptr(g), _ptr(h)))
        return float(c[0]), g, h

    def hvp(self, theta, v, with_grad: bool = False):
        th = _f64(theta, self.P)
        vv = _f64(v, self.P)
        hv = np.zeros(self.P)
        g = np.zeros(self.P) if with_grad else None
        self._check(lib().qoc_hvp(self._h, _ptr(th), _ptr(vv), _ptr(hv), _ptr(g)))
        return (hv, g) if with_grad else hv

    def hess_many(self, thetas):
        th = _f64(thetas)
        count = th.size // self.P
        th = th.reshape(count, self.P)
        c = np.zeros(count)
        g = np.zeros((count, self.P))
        h = np.zeros((count, self.P, self.P))
        self._check(lib().qoc_hess_many(self._h, count, _ptr(th), _ptr(c), _ptr(g), _ptr(h)))
        return c, g, h

    def grad_many(self, thetas):
        th = _f64(thetas)
        count = th.size // self.P
        th = th.reshape(count, self.P)
        c = np.zeros(count)
        g = np.zeros((count, self.P))
        self._check(lib().qoc_grad_many(self._h, count, _ptr(th), _ptr(c), _ptr(g)))
        return c, g

    # -- evaluation (device pointers, enqueue only)
    def cost_dev(self, theta_ptr: int, cost_ptr: int):
        self._check(lib().qoc_cost_dev(self._h, _vp(theta_ptr), _vp(cost_ptr)))

    def grad_dev(self, theta_ptr: int, cost_ptr: Optional[int], grad_ptr: int):
        self._check(lib().qoc_grad_dev(self._h, _vp(theta_ptr), _vp(cost_ptr) if cost_ptr else None,
                                       _vp(grad_ptr)))

    def hess_dev(self, theta_ptr, cost_ptr, grad_ptr, hess_ptr):
        self._check(lib().qoc_hess_dev(self._h, _vp(theta_ptr), _vp(cost_ptr) if cost_ptr else None,
                                       _vp(grad_ptr) if grad_ptr else None, _vp(hess_ptr)))

    def hvp_dev(self, theta_ptr, v_ptr, hv_ptr, grad_ptr=None):
        self._check(lib().qoc_hvp_dev(self._h, _vp(theta_ptr), _vp(v_ptr), _vp(hv_ptr),
                                      _vp(grad_ptr) if grad_ptr else None))

    def hess_many_dev(self, count, thetas_ptr, costs_ptr, grads_ptr, hess_ptr):
        self._check(lib().qoc_hess_many_dev(self._h, count, _vp(thetas_ptr),
                                            _vp(costs_ptr) if costs_ptr else None,
                                            _vp(grads_ptr) if grads_ptr else None,
                                            _vp(hess_ptr) if hess_ptr else None))

    def hess_many_dev_noalloc(self, count, thetas_ptr, costs_ptr, grads_ptr, hess_ptr):
        self._check(lib().qoc_hess_many_dev_noalloc(self._h, count, _vp(thetas_ptr),
                                                    _vp(costs_ptr) if costs_ptr else None,
                                                    _vp(grads_ptr) if grads_ptr else None,
                                                    _vp(hess_ptr) if hess_ptr else None))

    def sync(self):
        self._check(lib().qoc_sync(self._h))

    # -- profiling
    def profile_enable(self, on: bool = True):
        self._check(lib().qoc_profile_enable(self._h, 1 if on else 0))

    def profile_kernel_ms(self, kernel: str):
        ms = np.zeros(1)
        n = _i32()
        self._check(lib().qoc_profile_kernel_ms(self._h, kernel.encode(), _ptr(ms), ctypes.byref(n)))
        return float(ms[0]), int(n.value)

    def jacobi_stats(self, reset: bool = True):
        st = ctypes.c_int64()
        sw = ctypes.c_int64()
        self._check(lib().qoc_jacobi_stats(self._h, ctypes.byref(st), ctypes.byref(sw), 1 if reset else 0))
        return int(st.value), int(sw.value)

    # -- inspection and solvers
    def step_propagators(self, theta, j: int):
        th = _f64(theta, self.P)
        n = self.n
        u = np.zeros((n, n), np.complex128)
        u1 = np.zeros((n, n), np.complex128)
        u2 = np.zeros((n, n), np.complex128)
        self._check(lib().qoc_step_propagators(self._h, _ptr(th), j, _ptr(u.view(np.float64)),
                                               _ptr(u1.view(np.float64)), _ptr(u2.view(np.float64))))
        return u, u1, u2

    def hess_many_targets(self, thetas, targets):
        th = _f64(thetas)
        count = th.size // self.P
        tg = np.ascontiguousarray(np.asarray(targets, dtype=np.complex128).reshape(count, self.n)).view(np.float64)
        c = np.zeros(count)
        g = np.zeros((count, self.P))
        h = np.zeros((count, self.P, self.P))
        self._check(lib().qoc_hess_many_targets(self._h, count, _ptr(th), _ptr(tg), _ptr(c), _ptr(g), _ptr(h)))
        return c, g, h

    def tr_solve_many(self, theta0s, targets=None, gtol: float = 1e-8, max_iter: int = 10000):
        th = _f64(theta0s)
        count = th.size // self.P
        th = th.reshape(count, self.P)
        tg = None
        if targets is not None:
            tg = np.ascontiguousarray(np.asarray(targets, dtype=np.complex128).reshape(count, self.n)).view(np.float64)
        out = np.zeros((count, self.P))
        c = np.zeros(count)
        its = np.zeros(count, dtype=np.int32)
        conv = np.zeros(count, dtype=np.int32)
        self._check(lib().qoc_tr_solve_many(self._h, count, _ptr(th), _ptr(tg), gtol, max_iter, _ptr(out), _ptr(c),
                                            its.ctypes.data_as(ctypes.POINTER(_i32)),
                                            conv.ctypes.data_as(ctypes.POINTER(_i32))))
        return out, c, its, conv.astype(bool)

    def gradient_norms(self, grads):
        """(||g||_2, ||V_r^T g||_2) per row of grads (count x P)."""
        g = _f64(grads)
        count = g.size // self.P
        gn = np.zeros(count)
        pn = np.zeros(count)
        self._check(lib().qoc_tr_gradient_norms(self._h, count, _ptr(g), _ptr(gn), _ptr(pn)))
        return gn, pn

    def set_tr_subproblem(self, kind: int):
        """QOC_TR_SUBPROBLEM_DEFAULT (eigen-exact / dogleg) or QOC_TR_SUBPROBLEM_CG (Steihaug CG)."""
        self._check(lib().qoc_set_tr_subproblem(self._h, int(kind)))

    def set_tr_step_tolerance(self, xtol: float):
        """Stop trust-region solves once a step or the radius is shorter than xtol (0: off)."""
        self._check(lib().qoc_set_tr_step_tolerance(self._h, float(xtol)))

    def tr_solve_bfgs_many(self, theta0s, targets=None, gtol: float = 1e-8, max_iter: int = 10000):
        """BFGS trust-region solves (gradient evaluations only): (theta, cost, iters, converged)."""
        th = _f64(theta0s)
        count = th.size // self.P
        th = th.reshape(count, self.P)
        tg = None
        if targets is not None:
            tg = np.ascontiguousarray(np.asarray(targets, dtype=np.complex128).reshape(count, self.n)).view(np.float64)
        out = np.zeros((count, self.P))
        c = np.zeros(count)
        its = np.zeros(count, dtype=np.int32)
        conv = np.zeros(count, dtype=np.int32)
        self._check(lib().qoc_tr_solve_bfgs_many(self._h, count, _ptr(th), _ptr(tg), gtol, max_iter, _ptr(out),
                                                 _ptr(c), its.ctypes.data_as(ctypes.POINTER(_i32)),
                                                 conv.ctypes.data_as(ctypes.POINTER(_i32))))
        return out, c, its, conv.astype(bool)

    def control_coords(self, thetas):
        """(coords (count x P), rank): c = diag(sigma_r) V_r^T theta of the trust-region metric."""
        th = _f64(thetas)
        count = th.size // self.P
        out = np.zeros((count, self.P))
        r = _i32()
        self._check(lib().qoc_control_coords(self._h, count, _ptr(th), _ptr(out), ctypes.byref(r)))
        return out, int(r.value)

    def params_from_coords(self, coords):
        c = _f64(coords)
        count = c.size // self.P
        out = np.zeros((count, self.P))
        self._check(lib().qoc_params_from_coords(self._h, count, _ptr(c), _ptr(out)))
        return out

    def tr_solve(self, theta0, gtol: float = 1e-8, max_iter: int = 10000):
        th = _f64(theta0, self.P)
        out = np.zeros(self.P)
        c = np.zeros(1)
        it = _i32()
        st = lib().qoc_tr_solve(self._h, _ptr(th), gtol, max_iter, _ptr(out), _ptr(c), ctypes.byref(it))
        if st not in (QOC_OK, QOC_ERR_NOT_CONVERGED):
            self._check(st)
        return out, float(c[0]), int(it.value), st == QOC_OK


class Mlp:
    """Handle over the warm-start network (``qoc_mlp``).  Batches are device pointers of FP32
    row-major arrays, enqueued on the handle's stream (``stream`` = 0 / None: the null stream,
    which is torch's default stream)."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, max_batch: int, device: int = 0,
                 stream: Optional[int] = None):
        self._h = _vp()
        st = lib().qoc_mlp_create(device, _vp(stream) if stream else None, n_in, n_hidden, n_out, max_batch,
                                  ctypes.byref(self._h))
        if st != QOC_OK:
            raise QocError(st, status_string(st))
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        self.num_params = int(lib().qoc_mlp_num_params(self._h))

    def close(self):
        if self._h:
            lib().qoc_mlp_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != QOC_OK:
            raise QocError(st, lib().qoc_mlp_last_error(self._h).decode())

    def set_params(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if a.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {a.size}")
        self._check(lib().qoc_mlp_set_params(self._h, a.ctypes.data_as(_fp)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.num_params, np.float32)
        self._check(lib().qoc_mlp_get_params(self._h, a.ctypes.data_as(_fp)))
        return a

    def get_grads(self) -> np.ndarray:
        a = np.zeros(self.num_params, np.float32)
        self._check(lib().qoc_mlp_get_grads(self._h, a.ctypes.data_as(_fp)))
        return a

    def forward(self, batch: int, x_ptr: int, y_ptr: int):
        self._check(lib().qoc_mlp_forward(self._h, batch, _vp(x_ptr), _vp(y_ptr)))

    def loss_grad(self, batch: int, x_ptr: int, t_ptr: int, loss_ptr: Optional[int] = None):
        self._check(lib().qoc_mlp_loss_grad(self._h, batch, _vp(x_ptr), _vp(t_ptr),
                                            _vp(loss_ptr) if loss_ptr else None))

    def train_step(self, batch: int, x_ptr: int, t_ptr: int, lr: float, beta1: float = 0.9,
                   beta2: float = 0.999, eps: float = 1e-8, loss_ptr: Optional[int] = None):
        self._check(lib().qoc_mlp_train_step(self._h, batch, _vp(x_ptr), _vp(t_ptr), lr, beta1, beta2, eps,
                                             _vp(loss_ptr) if loss_ptr else None))

    def sync(self):
        self._check(lib().qoc_mlp_sync(self._h))


class Batch:
    """Handle over many independent problems evaluated together (``qoc_batch``)."""

    def __init__(self, problems, device: int = 0):
        self.problems = list(problems)
        self.P = [p.P for p in self.problems]
        self._h = _vp()
        arr = (_vp * len(self.problems))(*[p.handle for p in self.problems])
        st = lib().qoc_batch_create(device, len(self.problems), arr, ctypes.byref(self._h))
        if st != QOC_OK:
            raise QocError(st, status_string(st))

    def close(self):
        if self._h:
            lib().qoc_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != QOC_OK:
            raise QocError(st, lib().qoc_batch_last_error(self._h).decode())

    def _thetas(self, thetas):
        th = [_f64(t, P) for t, P in zip(thetas, self.P)]
        if len(th) != len(self.P):
            raise ValueError("one theta per problem")
        return th, (_dp * len(th))(*[_ptr(t) for t in th])

    def _run(self, fn, thetas, with_hessian=True):
        th, tp = self._thetas(thetas)
        c = [np.zeros(1) for _ in self.P]
        g = [np.zeros(P) for P in self.P]
        h = [np.zeros((P, P)) for P in self.P] if with_hessian else None
        cp = (_dp * len(c))(*[_ptr(x) for x in c])
        gp = (_dp * len(g))(*[_ptr(x) for x in g])
        hp = (_dp * len(h))(*[_ptr(x) for x in h]) if with_hessian else None
        self._check(fn(self._h, tp, cp, gp, hp))
        return np.array([x[0] for x in c]), g, h

    def hess(self, thetas, with_hessian: bool = True):
        """Batched launch (graph replay): (costs, [grad_i], [hess_i])."""
        return self._run(lib().qoc_batch_hess, thetas, with_hessian)

    def hess_unbatched(self, thetas, with_hessian: bool = True):
        """Same results from one launch sequence per problem."""
        return self._run(lib().qoc_batch_hess_unbatched, thetas, with_hessian)

    def autotune(self, thetas):
        th, tp = self._thetas(thetas)
        self._check(lib().qoc_batch_autotune(self._h, tp))

    def config(self, i: int):
        pg = _i32()
        ch = _i32()
        self._check(lib().qoc_batch_get_config(self._h, i, ctypes.byref(pg), ctypes.byref(ch)))
        return int(pg.value), int(ch.value)

    def set_config(self, i: int, pg: int, chunk: int):
        self._check(lib().qoc_batch_set_config(self._h, i, pg, chunk))

    def last_ms(self) -> float:
        ms = np.zeros(1)
        self._check(lib().qoc_batch_last_ms(self._h, _ptr(ms)))
        return float(ms[0])

    def memory(self) -> int:
        b = ctypes.c_int64()
        self._check(lib().qoc_batch_memory(self._h, ctypes.byref(b)))
        return int(b.value)


def bfgs_update(b, h, s, y, rescale: bool = False):
    """In-place BFGS update of (b, h = b^-1) from step s and gradient change y (qoc_bfgs_update)."""
    r = len(s)
    for a in (b, h):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous and a.size == r * r):
            raise ValueError("b and h must be C-contiguous float64 arrays of r x r")
    sv, yv = _f64(s, r), _f64(y, r)   # held for the duration of the call
    st = lib().qoc_bfgs_update(r, _ptr(b), _ptr(h), _ptr(sv), _ptr(yv), 1 if rescale else 0)
    if st != QOC_OK:
        raise QocError(st, status_string(st))


def problem_from_workload(w, device: int = 0) -> Problem:
    """Configure a handle from a paper_2505_00529_amd.inputs.Workload (Fourier model)."""
    p = Problem(device)
    s = w.system
    p.set_system(s.h0, s.m, s.psi0, s.psi_target)
    p.set_control_basis(QOC_BASIS_FOURIER, w.nt, w.dt, w.k)
    p.set_weights(w.gamma, w.rho)
    return p
