"""ctypes binding of the hrx C-ABI (include/hrx.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libhrx.so``.  Device buffers are
torch tensors on a ROCm device (PyTorch supplies memory and streams); the binding
passes their raw pointers and the current HIP stream.  A missing library is an
error: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrx.so")

GAS_CPG, GAS_AIR5 = 0, 1
FD_EXPLICIT, FD_COMPACT = 0, 1
WALL_ADIABATIC, WALL_ISOTHERMAL = 0, 1
RK3_2N, RK45_2N, SSPRK3 = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
THERMO_PLAIN, THERMO_SURROGATE = 0, 1
MLP_NPARAM = 9352

HRX_OK = 0
# per-point failures reported by hrx_get_counters (not raised by counters())
HRX_ENEWTON, HRX_EDOMAIN, HRX_ENONFINITE = -5, -6, -7
HRX_ETOOBIG = -8
NOALLOC_MAX_BYTES = 64 << 20     # HRX_NOALLOC_MAX_BYTES


class HrxError(RuntimeError):
    """A call returned a negative hrx_status (in .code)."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


class _Config(C.Structure):
    _fields_ = [
        ("gas", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
        ("fd_order", C.c_int), ("rk_scheme", C.c_int), ("precision", C.c_int), ("ad_on", C.c_int),
        ("ad_coef", C.c_double * 5),
        ("gamma", C.c_double), ("Pr", C.c_double), ("mach", C.c_double), ("T_inf", C.c_double),
        ("p_inf", C.c_double), ("Re", C.c_double), ("L_ref", C.c_double),
        ("Y_inf", C.c_double * 5),
        ("wall", C.c_int), ("T_wall", C.c_double),
        ("sponge_in", C.c_int), ("sponge_out", C.c_int), ("sponge_top", C.c_int),
        ("sigma_max", C.c_double),
        ("hold", C.POINTER(C.c_int64)), ("n_hold", C.c_int64),
        ("newton_max_iter", C.c_int), ("newton_rtol", C.c_double),
        ("diffusion", C.c_int), ("fd_scheme", C.c_int),
    ]


class Reference(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "gamma", "Re", "Pr", "Ec", "T_ref", "rho_inf", "c_inf", "mu_inf", "kappa_inf", "R_inf",
        "L_ref")]


class Counters(C.Structure):
    _fields_ = [("newton_nonconverged", C.c_int64), ("energy_below_min", C.c_int64),
                ("surrogate_fallbacks", C.c_int64), ("nonfinite", C.c_int64),
                ("negative_density", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhrx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HrxError(f"{path} not found: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, dp, i64 = C.c_void_p, C.c_void_p, C.c_int64
    lib.hrx_create.argtypes = [C.POINTER(_Config), C.POINTER(vp)]
    lib.hrx_create.restype = C.c_int
    lib.hrx_destroy.argtypes = [vp]
    lib.hrx_destroy.restype = None
    lib.hrx_get_reference.argtypes = [vp, C.POINTER(Reference)]
    lib.hrx_get_reference.restype = C.c_int
    lib.hrx_rhs_eval.argtypes = [vp, dp, dp, dp, vp]
    lib.hrx_rhs_eval.restype = C.c_int
    lib.hrx_rhs_eval_noalloc.argtypes = [vp, dp, dp, dp, vp]
    lib.hrx_rhs_eval_noalloc.restype = C.c_int
    lib.hrx_rk_stage.argtypes = [vp, C.c_int, C.c_double, dp, dp, dp, dp, vp]
    lib.hrx_rk_stage.restype = C.c_int
    lib.hrx_thermo_eval.argtypes = [vp, i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, vp]
    lib.hrx_thermo_eval.restype = C.c_int
    lib.hrx_chem_source.argtypes = [vp, i64, dp, dp, dp, vp]
    lib.hrx_chem_source.restype = C.c_int
    lib.hrx_equilibrium.argtypes = [vp, i64, dp, dp, dp, dp, dp, vp]
    lib.hrx_equilibrium.restype = C.c_int
    lib.hrx_get_counters.argtypes = [vp, C.POINTER(Counters), C.c_int]
    lib.hrx_get_counters.restype = C.c_int
    lib.hrx_timing_enable.argtypes = [vp, C.c_int]
    lib.hrx_timing_enable.restype = C.c_int
    lib.hrx_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.hrx_timing_read.restype = C.c_int
    f32 = C.c_float
    lib.hrx_mlp_init.argtypes = [vp, i64]
    lib.hrx_mlp_set_params.argtypes = [vp, dp, vp]
    lib.hrx_mlp_get_params.argtypes = [vp, dp, vp]
    lib.hrx_mlp_set_norm.argtypes = [vp, C.POINTER(f32), C.POINTER(f32), C.POINTER(f32),
                                     C.POINTER(f32), C.POINTER(f32), C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_double, C.c_double]
    lib.hrx_set_thermo_mode.argtypes = [vp, C.c_int]
    lib.hrx_mlp_features.argtypes = [vp, i64, dp, dp, dp, dp, vp]
    lib.hrx_mlp_dataset.argtypes = [vp, i64, dp, dp, dp, dp, dp, dp, vp]
    lib.hrx_mlp_fit.argtypes = [vp, i64, dp, dp, dp, dp] + [C.c_double] * 6 + \
        [C.POINTER(C.c_double), vp]
    lib.hrx_mlp_forward.argtypes = [vp, i64, dp, dp, vp]
    lib.hrx_mlp_backward.argtypes = [vp, i64, dp, dp, dp, vp]
    lib.hrx_adam_step.argtypes = [vp, dp, f32, C.c_int, vp]
    lib.hrx_mlp_train_step.argtypes = [vp, i64, dp, dp, dp, f32, C.c_int, dp, vp]
    for fn in ("hrx_mlp_init", "hrx_mlp_set_params", "hrx_mlp_get_params", "hrx_mlp_set_norm",
               "hrx_mlp_features", "hrx_mlp_dataset", "hrx_mlp_fit",
               "hrx_set_thermo_mode", "hrx_mlp_forward", "hrx_mlp_backward", "hrx_adam_step",
               "hrx_mlp_train_step"):
        getattr(lib, fn).restype = C.c_int
    lib.hrx_strerror.argtypes = [C.c_int]
    lib.hrx_strerror.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != HRX_OK:
        raise HrxError(f"hrx error {rc}: {_lib.hrx_strerror(rc).decode()}", rc)


def _ptr(t):
    """Raw device pointer of a tensor; the C-ABI takes dense row-major arrays only."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise HrxError("hrx arrays must be contiguous (row-major) tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """Owns one hrx_ctx.  Built from a workload description (fields.FlowConfig)."""

    def __init__(self, cfg, x, y, z=None, hold=None, precision=PREC_FP64, newton_max_iter=0):
        lib = load()
        self._keep = []
        c = _Config()
        c.gas = cfg.gas
        c.nx, c.ny, c.nz = cfg.nx, cfg.ny, cfg.nz

        def arr(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self._keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_double))

        c.x, c.y = arr(x), arr(y)
        c.z = arr(z) if (z is not None and cfg.nz > 1) else None
        c.fd_order, c.rk_scheme, c.precision = cfg.fd_order, cfg.rk, precision
        c.ad_on = 1 if cfg.ad else 0
        c.ad_coef[:] = list(cfg.ad_coef)
        c.gamma, c.Pr, c.mach, c.T_inf = cfg.gamma, cfg.Pr, cfg.mach, cfg.T_inf
        c.p_inf, c.Re, c.L_ref = cfg.p_inf, cfg.Re, cfg.L_ref
        c.Y_inf[:] = list(cfg.Y_inf)
        c.wall, c.T_wall = cfg.wall, cfg.T_wall
        c.sponge_in, c.sponge_out, c.sponge_top = cfg.sponge_in, cfg.sponge_out, cfg.sponge_top
        c.sigma_max = cfg.sigma_max
        if hold is not None and len(hold):
            h = np.ascontiguousarray(hold, dtype=np.int64)
            self._keep.append(h)
            c.hold = h.ctypes.data_as(C.POINTER(C.c_int64))
            c.n_hold = len(h)
        else:
            c.hold, c.n_hold = None, 0
        c.newton_max_iter, c.newton_rtol = int(newton_max_iter), 0.0
        c.diffusion = getattr(cfg, "diffusion", 0)
        c.fd_scheme = getattr(cfg, "fd_scheme", 0)
        h = C.c_void_p()
        _check(lib.hrx_create(C.byref(c), C.byref(h)))
        self._h = h
        self.cfg = cfg
        self.nvar = cfg.nvar
        self.N = cfg.npts

    def close(self):
        if getattr(self, "_h", None):
            _lib.hrx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reference(self):
        r = Reference()
        _check(_lib.hrx_get_reference(self._h, C.byref(r)))
        return {n: getattr(r, n) for n, _ in Reference._fields_}

    def counters(self, reset=False):
        """Counter values, plus 'status': the failure code hrx_get_counters returned
        (HRX_OK, HRX_ENEWTON, HRX_EDOMAIN or HRX_ENONFINITE)."""
        c = Counters()
        rc = _lib.hrx_get_counters(self._h, C.byref(c), 1 if reset else 0)
        if rc not in (HRX_OK, HRX_ENEWTON, HRX_EDOMAIN, HRX_ENONFINITE):
            _check(rc)
        out = {n: getattr(c, n) for n, _ in Counters._fields_}
        out["status"] = rc
        return out


KERNEL_NAMES = ("prim", "ad_src", "ad_d4", "ad_filter_x", "ad_filter_y", "ad_filter_z", "flux",
                "div", "bc", "thermo_eval", "chem_source", "cderiv", "fin", "equilibrium")


def timing_enable(ctx, on=True):
    _check(_lib.hrx_timing_enable(ctx._h, 1 if on else 0))


def timing_read(ctx):
    """{kernel: (total ms, launches)} since timing was enabled (synchronises)."""
    n = len(KERNEL_NAMES)
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(_lib.hrx_timing_read(ctx._h, ms, cnt))
    return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(n)}


def rhs_eval(ctx, Q, Q_ref, R, stream=None):
    _check(_lib.hrx_rhs_eval(ctx._h, _ptr(Q), _ptr(Q_ref), _ptr(R), _stream(stream)))


def rhs_eval_noalloc(ctx, Q, Q_ref, R, stream=None):
    """hrx_rhs_eval_noalloc: the right-hand side with the library's static workspace."""
    _check(_lib.hrx_rhs_eval_noalloc(ctx._h, _ptr(Q), _ptr(Q_ref), _ptr(R), _stream(stream)))


def rk_stage(ctx, stage, dt, Q, dQ, Q_ref, stream=None, R=None):
    """One RK stage; R (optional) is a precomputed right-hand side (unfused stage)."""
    _check(_lib.hrx_rk_stage(ctx._h, int(stage), float(dt), _ptr(Q), _ptr(dQ), _ptr(Q_ref),
                             _ptr(R), _stream(stream)))


def thermo_eval(ctx, n, rho, e, Y, T, p=None, h=None, mu=None, kappa=None, D=None, status=None,
                stream=None):
    _check(_lib.hrx_thermo_eval(ctx._h, int(n), _ptr(rho), _ptr(e), _ptr(Y), _ptr(T), _ptr(p),
                                _ptr(h), _ptr(mu), _ptr(kappa), _ptr(D), _ptr(status),
                                _stream(stream)))


def chem_source(ctx, n, rho_s, T, wdot, stream=None):
    _check(_lib.hrx_chem_source(ctx._h, int(n), _ptr(rho_s), _ptr(T), _ptr(wdot), _stream(stream)))


def equilibrium(ctx, n, rho, T, Y, xiN=None, status=None, stream=None):
    """LTE compositions Y [5][n] at (rho, T, xiN) (hrx_equilibrium)."""
    _check(_lib.hrx_equilibrium(ctx._h, int(n), _ptr(rho), _ptr(T), _ptr(xiN), _ptr(Y),
                                _ptr(status), _stream(stream)))


# ---------------------------------------------------------------- surrogate network
def mlp_init(ctx, max_batch):
    _check(_lib.hrx_mlp_init(ctx._h, int(max_batch)))


def mlp_set_params(ctx, theta, stream=None):
    _check(_lib.hrx_mlp_set_params(ctx._h, _ptr(theta), _stream(stream)))


def mlp_get_params(ctx, theta_out, stream=None):
    _check(_lib.hrx_mlp_get_params(ctx._h, _ptr(theta_out), _stream(stream)))


def mlp_set_norm(ctx, in_mean, in_std, out_mean, out_std, log10rho_range, T_range,
                 out_lin=None, xiN_range=(0.0, 1.0)):
    """Feature standardisation, output composition (out_lin: [8][8] or None) and the
    training hull of the surrogate (hrx_mlp_set_norm)."""
    def f(a, shape):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.shape != shape:
            raise HrxError(f"expected shape {shape}, got {a.shape}")
        return a
    arrs = [f(in_mean, (7,)), f(in_std, (7,)), f(out_mean, (8,)), f(out_std, (8,))]
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_float)) for a in arrs]
    lin = None if out_lin is None else f(out_lin, (8, 8))
    lptr = None if lin is None else lin.ctypes.data_as(C.POINTER(C.c_float))
    _check(_lib.hrx_mlp_set_norm(ctx._h, *ptrs, lptr, float(log10rho_range[0]),
                                 float(log10rho_range[1]), float(T_range[0]), float(T_range[1]),
                                 float(xiN_range[0]), float(xiN_range[1])))


def mlp_features(ctx, n, rho, e, Y, f, stream=None):
    """Raw surrogate features f [n][7] (FP32) of SI states (hrx_mlp_features)."""
    _check(_lib.hrx_mlp_features(ctx._h, int(n), _ptr(rho), _ptr(e), _ptr(Y), _ptr(f),
                                 _stream(stream)))


def mlp_dataset(ctx, n, rho, e, Y, F, T, status=None, stream=None):
    """Raw features F [n][7] and targets T [n][8] (FP64) of SI states (hrx_mlp_dataset)."""
    _check(_lib.hrx_mlp_dataset(ctx._h, int(n), _ptr(rho), _ptr(e), _ptr(Y), _ptr(F), _ptr(T),
                                _ptr(status), _stream(stream)))


def mlp_fit(ctx, n, F, T, Xs, Ys, log10rho_range, T_range, xiN_range, stream=None):
    """Composition statistics of a training set, installed, and its standardised rows
    (hrx_mlp_fit); returns the statistics (m, s, rm, rs, L) as numpy arrays."""
    st = (C.c_double * 94)()
    _check(_lib.hrx_mlp_fit(ctx._h, int(n), _ptr(F), _ptr(T), _ptr(Xs), _ptr(Ys),
                            float(log10rho_range[0]), float(log10rho_range[1]),
                            float(T_range[0]), float(T_range[1]), float(xiN_range[0]),
                            float(xiN_range[1]), st, _stream(stream)))
    a = np.array(st[:])
    return dict(xm=a[0:7], xs=a[7:14], ym=a[14:22], ys=a[22:30], L=a[30:94].reshape(8, 8))


def set_thermo_mode(ctx, mode):
    _check(_lib.hrx_set_thermo_mode(ctx._h, int(mode)))


def mlp_forward(ctx, n, X, Y, stream=None):
    _check(_lib.hrx_mlp_forward(ctx._h, int(n), _ptr(X), _ptr(Y), _stream(stream)))


def mlp_backward(ctx, n, X, dLdY, grad, stream=None):
    _check(_lib.hrx_mlp_backward(ctx._h, int(n), _ptr(X), _ptr(dLdY), _ptr(grad), _stream(stream)))


def adam_step(ctx, grad, lr, t, stream=None):
    _check(_lib.hrx_adam_step(ctx._h, _ptr(grad), float(lr), int(t), _stream(stream)))


def mlp_train_step(ctx, n, idx, X, Yt, lr, t, loss=None, stream=None):
    _check(_lib.hrx_mlp_train_step(ctx._h, int(n), _ptr(idx), _ptr(X), _ptr(Yt), float(lr), int(t),
                                   _ptr(loss), _stream(stream)))
