"""Parallel state-space GP regression on MI355X: Python binding of libpssgp.so.

Temporal Gaussian-process regression in logarithmic span (Corenflos, Zhao,
Sarkka): the GP is written as a linear SDE, discretised per time step, and
the Kalman filter and RTS smoother run as parallel prefix scans over their
associative elements; test points are missing measurements on the merged
time grid. Every step of the computation runs in the HIP kernels of
``libpssgp.so``; this module only marshals torch tensors (device memory and
the current stream) into the C ABI of ``include/pssgp.h``. Importing works
without a GPU; the calls need a HIP device and raise otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpssgp.so")

MATERN12, MATERN32, MATERN52, RBF, QUASIPERIODIC = 1, 2, 3, 4, 5
F32, F64 = 0, 1
STATIC_SCRATCH_BYTES = 64 << 20  # PSSGP_STATIC_SCRATCH_BYTES: the scratch behind pssgp_loglik_static
OP_FILTER, OP_SMOOTH, OP_LOGLIK, OP_LOGLIK_GRAD, OP_DISCRETIZE, OP_PLAIN, OP_PREDICT = 1, 2, 3, 4, 5, 6, 7
STATUS_UNSORTED, STATUS_NONFINITE, STATUS_BAD_S, STATUS_CHOLESKY = 1, 2, 4, 8

_ERRORS = {-1: "EINVAL", -2: "EUNSUPPORTED", -3: "EWORKSPACE", -4: "EDEVICE", -5: "ENODEVICE",
           -6: "EMODEL"}


class PssgpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRORS.get(code, "?"), code, msg))
        self.code = code


class Component(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32),
                ("lengthscale", ctypes.c_double), ("variance", ctypes.c_double),
                ("period", ctypes.c_double), ("lengthscale2", ctypes.c_double)]


class Model(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("comp", Component * 4), ("noise_var", ctypes.c_double)]


class BatchGroup(ctypes.Structure):
    _fields_ = [("kind", Component), ("series_begin", ctypes.c_int64), ("series_end", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("deterministic", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 6), ("pass_events", ctypes.c_void_p * 8)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_VP, _I64, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
_MP = ctypes.POINTER(Model)
_OP = ctypes.POINTER(Options)
SIGNATURES = [
    ("pssgp_version", ctypes.c_int, []),
    ("pssgp_last_error", ctypes.c_char_p, []),
    ("pssgp_state_dim", ctypes.c_int, [_MP]),
    ("pssgp_state_basis", ctypes.c_int, [_MP, _VP]),
    ("pssgp_model_matrices", ctypes.c_int, [_MP, _VP, _VP, _VP]),
    ("pssgp_workspace_bytes", _SZ, [_MP, _I64, ctypes.c_int, ctypes.c_int, _OP]),
    ("pssgp_discretize", ctypes.c_int, [_MP, _VP, _I64, _VP, _VP, _VP, _SZ, _VP]),
    ("pssgp_filter", ctypes.c_int, [_MP, _VP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _VP,
                                    _SZ, _OP, _VP]),
    ("pssgp_smooth", ctypes.c_int, [_MP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _VP, _VP,
                                    _SZ, _OP, _VP]),
    ("pssgp_loglik", ctypes.c_int, [_MP, _VP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _SZ, _OP,
                                    _VP]),
    ("pssgp_loglik_grad", ctypes.c_int, [_MP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _SZ,
                                         _OP, _VP]),
    ("pssgp_loglik_grad_noise", ctypes.c_int, [_MP, _VP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _SZ,
                                               _OP, _VP]),
    ("pssgp_batched_workspace_bytes", _SZ, [ctypes.c_void_p, ctypes.c_int, _I64, _VP, ctypes.c_int, ctypes.c_int,
                                            _OP]),
    ("pssgp_batched_filter", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _I64, _VP, _VP, _VP, _VP, _VP, _VP,
                                            ctypes.c_int, _VP, _VP, _VP, _VP, _SZ, _OP, _VP]),
    ("pssgp_batched_smooth", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _I64, _VP, _VP, _VP, _VP, _VP, _VP,
                                            ctypes.c_int, _VP, _VP, _VP, _SZ, _OP, _VP]),
    ("pssgp_batched_loglik", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _I64, _VP, _VP, _VP, _VP, _VP, _VP,
                                            ctypes.c_int, _VP, _VP, _SZ, _OP, _VP]),
    ("pssgp_batched_predict", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _I64, _VP, _VP, _VP, _VP, _VP, _VP,
                                             ctypes.c_int, _VP, _VP, _VP, _VP, _SZ, _OP, _VP]),
    ("pssgp_status", ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_uint32)]),
    ("pssgp_predict", ctypes.c_int, [_MP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _VP, _SZ, _OP, _VP]),
    ("pssgp_plain_predict", ctypes.c_int, [_MP, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("pssgp_merge_times", ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, _I64, ctypes.c_int, _VP, _VP, _VP, _VP, _VP]),
    ("pssgp_loglik_static", ctypes.c_int, [_MP, _VP, _VP, _VP, _VP, _I64, ctypes.c_int, _VP, _OP, _VP]),
    ("pssgp_plan_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, _MP, _VP, _VP, _VP, _I64,
                                         ctypes.c_int, _VP, _VP, _VP, _VP, _SZ, _OP]),
    ("pssgp_plan_launch", ctypes.c_int, [_VP, _VP]),
    ("pssgp_plan_destroy", ctypes.c_int, [_VP]),
]


def lib() -> ctypes.CDLL:
    """Load libpssgp.so (built by ``build()``); fails loudly when absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpssgp.so is not built (run paper_2102_09964_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)  # AttributeError: the library misses an entry point
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def build():
    from .build import build as _b
    return _b()


def _check(rc):
    if rc != 0:
        raise PssgpError(rc, lib().pssgp_last_error().decode())


def make_model(components, noise_var) -> Model:
    """components: list of (kind, order, lengthscale, variance) or, for a
    quasi-periodic component, (QUASIPERIODIC, J, ell_p, variance, period,
    ell_matern)."""
    m = Model()
    m.n_comp = len(components)
    if not 1 <= m.n_comp <= 4:
        raise ValueError("1 to 4 components")
    for i, comp in enumerate(components):
        kind, order, ell, var = comp[:4]
        m.comp[i].kind = int(kind)
        m.comp[i].order = int(order)
        m.comp[i].lengthscale = float(ell)
        m.comp[i].variance = float(var)
        if len(comp) > 4:
            m.comp[i].period = float(comp[4])
            m.comp[i].lengthscale2 = float(comp[5])
    m.noise_var = float(noise_var)
    return m


def _as_model(model):
    if isinstance(model, Model):
        return model
    if isinstance(model, dict):
        return make_model(model["components"], model["noise_var"])
    raise TypeError("model must be a Model or a dict with 'components' and 'noise_var'")


def make_options(chunk=0, deterministic=False) -> Options:
    o = Options()
    o.chunk = int(chunk)
    o.deterministic = 1 if deterministic else 0
    return o


def event_handle(ev) -> int:
    """Raw hipEvent_t of a torch.cuda.Event (recorded once if not yet created)."""
    if not ev.cuda_event:
        ev.record()
    return int(ev.cuda_event)


def _with_events(options, events) -> Options:
    o = Options()
    if options is not None:
        ctypes.memmove(ctypes.byref(o), ctypes.byref(options), ctypes.sizeof(Options))
    for i, ev in enumerate(events):
        o.pass_events[i] = event_handle(ev) if ev is not None else None
    return o


def state_dim(model) -> int:
    d = lib().pssgp_state_dim(ctypes.byref(_as_model(model)))
    if d < 0:
        _check(d)
    return d


def state_basis(model) -> np.ndarray:
    """Diagonal T with x_canonical = diag(T) z for the library's state z."""
    m = _as_model(model)
    d = state_dim(m)
    out = np.empty(d)
    _check(lib().pssgp_state_basis(ctypes.byref(m), out.ctypes.data))
    return out


def model_matrices(model):
    """(G, Pinf, H) of the continuous model in the library's coordinates."""
    m = _as_model(model)
    d = state_dim(m)
    G, P, H = np.empty((d, d)), np.empty((d, d)), np.empty(d)
    _check(lib().pssgp_model_matrices(ctypes.byref(m), G.ctypes.data, P.ctypes.data, H.ctypes.data))
    return G, P, H


def workspace_bytes(model, n, dtype, op, options=None) -> int:
    return int(lib().pssgp_workspace_bytes(ctypes.byref(_as_model(model)), int(n), int(dtype), int(op),
                                           ctypes.byref(options) if options is not None else None))


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


def _dt(dtype):
    torch = _torch()
    if dtype in (F32, torch.float32, "f32", "float32"):
        return F32, torch.float32
    if dtype in (F64, torch.float64, "f64", "float64"):
        return F64, torch.float64
    raise ValueError("dtype must be float32 or float64")


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(x, dtype, device):
    torch = _torch()
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


def _require_gpu():
    torch = _torch()
    if not torch.cuda.is_available():
        raise PssgpError(-5, "no HIP device: the pssgp kernels need an MI355X")


def alloc_workspace(model, n, dtype, op, options=None, device="cuda"):
    torch = _torch()
    nb = workspace_bytes(model, n, dtype, op, options)
    if nb == 0:
        _check(-1)
    return torch.empty(nb, dtype=torch.uint8, device=device)


def status(ws) -> int:
    """Device status bits of the last call that used workspace ws (syncs)."""
    bits = ctypes.c_uint32(0)
    _check(lib().pssgp_status(_p(ws), _stream(), ctypes.byref(bits)))
    return bits.value


def discretize(model, t, device="cuda"):
    """F: (n, d, d) float64, Q: (NS, n) float64 packed upper (library basis)."""
    _require_gpu()
    torch = _torch()
    m = _as_model(model)
    d = state_dim(m)
    t = _dev(t, torch.float64, device)
    n = t.shape[0]
    F = torch.empty((n, d, d), dtype=torch.float64, device=device)
    Q = torch.empty((d * (d + 1) // 2, n), dtype=torch.float64, device=device)
    ws = alloc_workspace(m, n, F64, OP_DISCRETIZE, device=device)
    _check(lib().pssgp_discretize(ctypes.byref(m), _p(t), n, _p(F), _p(Q), _p(ws), ws.numel(), _stream()))
    return F, Q


def filter(model, t, y, mask=None, noise_k=None, dtype="float32", moments=True, options=None,
           ws=None, device="cuda"):
    """Parallel Kalman filter. Returns dict with 'loglik' (float64 tensor [1])
    and, if moments, 'm' (d, n) and 'P' (NS, n) packed upper, entry-major."""
    _require_gpu()
    torch = _torch()
    m = _as_model(model)
    code, tdt = _dt(dtype)
    d = state_dim(m)
    t = _dev(t, torch.float64, device)
    n = t.shape[0]
    y = _dev(y, tdt, device)
    mask = _dev(mask, torch.uint8, device)
    noise_k = _dev(noise_k, torch.float64, device)
    op = OP_FILTER if moments else OP_LOGLIK
    if ws is None:
        ws = alloc_workspace(m, n, code, op, options, device)
    out = {"loglik": torch.empty(1, dtype=torch.float64, device=device), "ws": ws}
    if moments:
        out["m"] = torch.empty((d, n), dtype=tdt, device=device)
        out["P"] = torch.empty((d * (d + 1) // 2, n), dtype=tdt, device=device)
        rc = lib().pssgp_filter(ctypes.byref(m), _p(t), _p(y), _p(mask), _p(noise_k), n, code,
                                _p(out["m"]), _p(out["P"]), _p(out["loglik"]), _p(ws), ws.numel(),
                                ctypes.byref(options) if options is not None else None, _stream())
    else:
        rc = lib().pssgp_loglik(ctypes.byref(m), _p(t), _p(y), _p(mask), _p(noise_k), n, code,
                                _p(out["loglik"]), _p(ws), ws.numel(),
                                ctypes.byref(options) if options is not None else None, _stream())
    _check(rc)
    return out


def smooth(model, t, m_f, P_f, dtype="float32", full_state=False, options=None, ws=None, device="cuda"):
    """Parallel RTS smoother from filter moments. Returns dict with 'f_mean',
    'f_var' (n,) and, if full_state, 'ms' (d, n), 'Ps' (NS, n)."""
    _require_gpu()
    torch = _torch()
    mdl = _as_model(model)
    code, tdt = _dt(dtype)
    d = state_dim(mdl)
    t = _dev(t, torch.float64, device)
    n = t.shape[0]
    m_f = _dev(m_f, tdt, device)
    P_f = _dev(P_f, tdt, device)
    if ws is None:
        ws = alloc_workspace(mdl, n, code, OP_SMOOTH, options, device)
    out = {"f_mean": torch.empty(n, dtype=tdt, device=device),
           "f_var": torch.empty(n, dtype=tdt, device=device), "ws": ws}
    ms = Ps = None
    if full_state:
        ms = out["ms"] = torch.empty((d, n), dtype=tdt, device=device)
        Ps = out["Ps"] = torch.empty((d * (d + 1) // 2, n), dtype=tdt, device=device)
    _check(lib().pssgp_smooth(ctypes.byref(mdl), _p(t), _p(m_f), _p(P_f), n, code, _p(out["f_mean"]),
                              _p(out["f_var"]), _p(ms), _p(Ps), _p(ws), ws.numel(),
                              ctypes.byref(options) if options is not None else None, _stream()))
    return out


def predict(model, t, y, mask=None, dtype="float32", options=None, device="cuda", fused=True):
    """Filter + smoother on a merged grid (test points: mask 0). Returns
    dict with 'f_mean', 'f_var', 'loglik' (and the filter moments 'm', 'P'
    when fused=False)."""
    if fused:
        _require_gpu()
        torch = _torch()
        m = _as_model(model)
        code, tdt = _dt(dtype)
        t = _dev(t, torch.float64, device)
        n = t.shape[0]
        y = _dev(y, tdt, device)
        mask = _dev(mask, torch.uint8, device)
        ws = alloc_workspace(m, n, code, OP_PREDICT, options, device)
        fm = torch.empty(n, dtype=tdt, device=device)
        fv = torch.empty(n, dtype=tdt, device=device)
        ll = torch.empty(1, dtype=torch.float64, device=device)
        _check(lib().pssgp_predict(ctypes.byref(m), _p(t), _p(y), _p(mask), n, code, _p(fm), _p(fv), _p(ll), _p(ws),
                                   ws.numel(), ctypes.byref(options) if options is not None else None, _stream()))
        return {"f_mean": fm, "f_var": fv, "loglik": ll, "ws": ws}
    f = filter(model, t, y, mask, dtype=dtype, options=options, device=device)
    s = smooth(model, t, f["m"], f["P"], dtype=dtype, options=options, device=device)
    return {"f_mean": s["f_mean"], "f_var": s["f_var"], "loglik": f["loglik"], "m": f["m"], "P": f["P"]}


def merge_times(t_train, y_train, t_test, mask_train=None, dtype="float32", device="cuda"):
    """Merged time grid of a prediction (pssgp_merge_times): returns
    (t, y, mask, test_pos) with t float64 [n + m], y dtype [n + m] (0 at test
    steps; None when y_train is None), mask uint8 [n + m] (0 at test steps)
    and test_pos int64 [m], the merged index of every test time."""
    _require_gpu()
    torch = _torch()
    code, tdt = _dt(dtype)
    t_train = _dev(t_train, torch.float64, device)
    t_test = _dev(t_test, torch.float64, device)
    y_train = _dev(y_train, tdt, device)
    mask_train = _dev(mask_train, torch.uint8, device)
    n, m = t_train.shape[0], t_test.shape[0]
    t = torch.empty(n + m, dtype=torch.float64, device=device)
    y = torch.empty(n + m, dtype=tdt, device=device) if y_train is not None else None
    mask = torch.empty(n + m, dtype=torch.uint8, device=device)
    pos = torch.empty(m, dtype=torch.int64, device=device)
    _check(lib().pssgp_merge_times(_p(t_train), _p(y_train), _p(mask_train), n, _p(t_test), m, code, _p(t),
                                   _p(y), _p(mask), _p(pos), _stream()))
    return t, y, mask, pos


def plain_predict(model, t, y, mask=None, ws=None, device="cuda"):
    """Filter, log-likelihood and smoother through the plain FP64 scan
    (materialised elements, one launch per scan level). Same outputs as
    ``predict`` in FP64."""
    _require_gpu()
    torch = _torch()
    m = _as_model(model)
    t = _dev(t, torch.float64, device)
    n = t.shape[0]
    y = _dev(y, torch.float64, device)
    mask = _dev(mask, torch.uint8, device)
    d = state_dim(m)
    if ws is None:
        ws = alloc_workspace(m, n, F64, OP_PLAIN, None, device)
    mm = torch.empty((d, n), dtype=torch.float64, device=device)
    PP = torch.empty((d * (d + 1) // 2, n), dtype=torch.float64, device=device)
    fm = torch.empty(n, dtype=torch.float64, device=device)
    fv = torch.empty(n, dtype=torch.float64, device=device)
    ll = torch.empty(1, dtype=torch.float64, device=device)
    _check(lib().pssgp_plain_predict(ctypes.byref(m), _p(t), _p(y), _p(mask), n, _p(mm), _p(PP), _p(fm), _p(fv),
                                     _p(ll), _p(ws), ws.numel(), _stream()))
    return {"f_mean": fm, "f_var": fv, "loglik": ll, "m": mm, "P": PP}


def loglik(model, t, y, mask=None, noise_k=None, dtype="float32", options=None, device="cuda"):
    return filter(model, t, y, mask, noise_k, dtype, moments=False, options=options, device=device)["loglik"]


def loglik_static(model, t, y, mask=None, noise_k=None, dtype="float32", options=None, out=None, device="cuda"):
    """Log-likelihood through pssgp_loglik_static: no workspace, the library's
    per-device static scratch instead (nothing is allocated by the library;
    out, a device float64[1] tensor, may be given so that the call allocates
    nothing at all). Calls that overlap on one device race on that scratch."""
    _require_gpu()
    torch = _torch()
    m = _as_model(model)
    code, tdt = _dt(dtype)
    t = _dev(t, torch.float64, device)
    y = _dev(y, tdt, device)
    mask = _dev(mask, torch.uint8, device)
    noise_k = _dev(noise_k, torch.float64, device)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=device)
    rc = lib().pssgp_loglik_static(ctypes.byref(m), _p(t), _p(y), _p(mask), _p(noise_k), t.shape[0], code, _p(out),
                                   ctypes.byref(options) if options is not None else None, _stream())
    _check(rc)
    return out


def loglik_grad(model, t, y, mask=None, dtype="float32", options=None, ws=None, device="cuda", noise_k=None):
    """Log-likelihood and its gradient with respect to
    (ell_0, var_0, ell_1, var_1, ..., noise_var). With noise_k (per-step
    noise variances, fixed data) the model's noise_var is unused and the
    last gradient entry is 0."""
    _require_gpu()
    torch = _torch()
    m = _as_model(model)
    code, tdt = _dt(dtype)
    t = _dev(t, torch.float64, device)
    n = t.shape[0]
    y = _dev(y, tdt, device)
    mask = _dev(mask, torch.uint8, device)
    if ws is None:
        ws = alloc_workspace(m, n, code, OP_LOGLIK_GRAD, options, device)
    ll = torch.empty(1, dtype=torch.float64, device=device)
    g = torch.empty(2 * m.n_comp + 1, dtype=torch.float64, device=device)
    opt = ctypes.byref(options) if options is not None else None
    if noise_k is None:
        _check(lib().pssgp_loglik_grad(ctypes.byref(m), _p(t), _p(y), _p(mask), n, code, _p(ll), _p(g), _p(ws),
                                       ws.numel(), opt, _stream()))
    else:
        nk = _dev(noise_k, torch.float64, device)
        _check(lib().pssgp_loglik_grad_noise(ctypes.byref(m), _p(t), _p(y), _p(mask), _p(nk), n, code, _p(ll),
                                             _p(g), _p(ws), ws.numel(), opt, _stream()))
    return ll, g


def unpack_sym(Pp, d):
    """(NS, n) packed upper entry-major -> (n, d, d) symmetric (torch or numpy)."""
    iu = [(i, j) for i in range(d) for j in range(i, d)]
    if hasattr(Pp, "detach"):
        torch = _torch()
        n = Pp.shape[1]
        out = torch.empty((n, d, d), dtype=Pp.dtype, device=Pp.device)
        for e, (i, j) in enumerate(iu):
            out[:, i, j] = Pp[e]
            out[:, j, i] = Pp[e]
        return out
    n = Pp.shape[1]
    out = np.empty((n, d, d), dtype=Pp.dtype)
    for e, (i, j) in enumerate(iu):
        out[:, i, j] = Pp[e]
        out[:, j, i] = Pp[e]
    return out


def _theta_of(model):
    th = []
    for c in range(model.n_comp):
        th += [model.comp[c].lengthscale, model.comp[c].variance]
    return th + [model.noise_var]


def _model_with_theta(model, theta):
    comps = [(model.comp[c].kind, model.comp[c].order, float(theta[2 * c]), float(theta[2 * c + 1]))
             for c in range(model.n_comp)]
    return make_model(comps, float(theta[-1]))


def _make_autograd():
    torch = _torch()

    class LogLikelihood(torch.autograd.Function):
        """loglik(theta) with the hand-written adjoint as its backward.

        theta: float64 tensor (ell_0, var_0, ..., noise_var); the remaining
        arguments are fixed data. Forward runs the filter scan (which
        stores the per-step forward quantities) and the reverse adjoint scan
        together; backward scales the
        stored gradient by the incoming gradient."""

        @staticmethod
        def forward(ctx, theta, kinds_orders, t, y, mask, dtype):
            th = theta.detach().cpu().double().numpy()
            comps = [(k, o, th[2 * i], th[2 * i + 1]) for i, (k, o) in enumerate(kinds_orders)]
            ll, g = loglik_grad(make_model(comps, th[-1]), t, y, mask, dtype=dtype, device=t.device)
            ctx.save_for_backward(g.to(theta.device))
            return ll.to(theta.device).reshape(())

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return gout * g, None, None, None, None, None

    return LogLikelihood


_autograd_cls = None


def loglik_autograd(theta, kinds_orders, t, y, mask=None, dtype="float32"):
    """Differentiable log-likelihood: theta -> loglik (torch.autograd)."""
    global _autograd_cls
    if _autograd_cls is None:
        _autograd_cls = _make_autograd()
    return _autograd_cls.apply(theta, kinds_orders, t, y, mask, dtype)


class Plan:
    """pssgp_plan: one pssgp_predict (or pssgp_loglik) call recorded into a
    HIP graph by the library, with device buffers bound at creation;
    ``launch()`` replays it on the current stream. Refill ``t``, ``y``,
    ``mask`` in place between launches to process new data of the same
    size."""

    def __init__(self, model, n, dtype="float32", options=None, loglik_only=False, device="cuda"):
        _require_gpu()
        torch = _torch()
        self.model = _as_model(model)
        self.code, self.tdt = _dt(dtype)
        self.n = int(n)
        op = OP_LOGLIK if loglik_only else OP_PREDICT
        self.ws = alloc_workspace(self.model, self.n, self.code, op, options, device)
        self.t = torch.zeros(self.n, dtype=torch.float64, device=device)
        self.y = torch.zeros(self.n, dtype=self.tdt, device=device)
        self.mask = torch.ones(self.n, dtype=torch.uint8, device=device)
        self.f_mean = None if loglik_only else torch.empty(self.n, dtype=self.tdt, device=device)
        self.f_var = None if loglik_only else torch.empty(self.n, dtype=self.tdt, device=device)
        self.loglik = torch.empty(1, dtype=torch.float64, device=device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(lib().pssgp_plan_create(ctypes.byref(h), op, ctypes.byref(self.model), _p(self.t), _p(self.y),
                                       _p(self.mask), self.n, self.code, _p(self.f_mean), _p(self.f_var),
                                       _p(self.loglik), _p(self.ws), self.ws.numel(),
                                       ctypes.byref(options) if options is not None else None))
        self.handle = h

    def launch(self):
        _check(lib().pssgp_plan_launch(self.handle, _stream()))
        return self.f_mean, self.f_var, self.loglik

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().pssgp_plan_destroy(h)
            self.handle = None


class Pipeline:
    """Preallocated filter + smoother (+ log-likelihood) for a fixed model,
    length and dtype: workspaces and outputs are allocated once, so that
    ``run()`` only launches kernels (stream-ordered, no synchronisation).

    By default both scans run in one ``pssgp_predict`` call, which hands the
    filter moments to the smoother inside its workspace; with
    ``full_state`` (smoothed state moments wanted) or ``fused=False`` the
    filter moments are written to ``m``, ``P`` and read back by
    ``pssgp_smooth``.
    """

    def __init__(self, model, n, dtype="float32", options=None, full_state=False, fused=True, device="cuda"):
        _require_gpu()
        torch = _torch()
        self.model = _as_model(model)
        self.code, self.tdt = _dt(dtype)
        self.n = int(n)
        self.d = state_dim(self.model)
        self.options = options
        self.fused = fused and not full_state
        ns = self.d * (self.d + 1) // 2
        if self.fused:
            self.ws_p = alloc_workspace(self.model, n, self.code, OP_PREDICT, options, device)
            self.ws_f = self.ws_s = self.ws_p
            self.m = self.P = None
        else:
            self.ws_f = alloc_workspace(self.model, n, self.code, OP_FILTER, options, device)
            self.ws_s = alloc_workspace(self.model, n, self.code, OP_SMOOTH, options, device)
            self.m = torch.empty((self.d, n), dtype=self.tdt, device=device)
            self.P = torch.empty((ns, n), dtype=self.tdt, device=device)
        self.loglik = torch.empty(1, dtype=torch.float64, device=device)
        self.f_mean = torch.empty(n, dtype=self.tdt, device=device)
        self.f_var = torch.empty(n, dtype=self.tdt, device=device)
        self.ms = torch.empty((self.d, n), dtype=self.tdt, device=device) if full_state else None
        self.Ps = torch.empty((ns, n), dtype=self.tdt, device=device) if full_state else None
        self.device = device

    def run(self, t, y, mask=None, events=None, pass_events=None):
        """events: optional list of 3 torch.cuda.Event recorded before the
        filter, between filter and smoother, and after the smoother.
        pass_events: optional (filter, smoother) pair of lists of 4 recorded
        torch.cuda.Event (see pssgp_options.pass_events), for the duration
        of every pass."""
        L = lib()
        mp = ctypes.byref(self.model)
        st = _stream()
        op = ctypes.byref(self.options) if self.options is not None else None
        if self.fused:
            if pass_events is not None:
                op = ctypes.byref(_with_events(self.options, list(pass_events[0]) + list(pass_events[1])))
            if events:
                events[0].record()
            _check(L.pssgp_predict(mp, _p(t), _p(y), _p(mask), self.n, self.code, _p(self.f_mean), _p(self.f_var),
                                   _p(self.loglik), _p(self.ws_p), self.ws_p.numel(), op, st))
            if events:
                events[1].record()
                events[2].record()
            return self.f_mean, self.f_var, self.loglik
        op_f = op_s = op
        if pass_events is not None:
            op_f = ctypes.byref(_with_events(self.options, pass_events[0]))
            op_s = ctypes.byref(_with_events(self.options, pass_events[1]))
        if events:
            events[0].record()
        _check(L.pssgp_filter(mp, _p(t), _p(y), _p(mask), None, self.n, self.code, _p(self.m), _p(self.P),
                              _p(self.loglik), _p(self.ws_f), self.ws_f.numel(), op_f, st))
        if events:
            events[1].record()
        _check(L.pssgp_smooth(mp, _p(t), _p(self.m), _p(self.P), self.n, self.code, _p(self.f_mean),
                              _p(self.f_var), _p(self.ms), _p(self.Ps), _p(self.ws_s), self.ws_s.numel(), op_s,
                              st))
        if events:
            events[2].record()
        return self.f_mean, self.f_var, self.loglik


_STATE_DIM = {MATERN12: 1, MATERN32: 2, MATERN52: 3}


def batch_groups(kinds):
    """Groups of consecutive series with the same (Matern) kind; kinds must be
    sorted by state size. Returns a ctypes array of BatchGroup."""
    kinds = [int(k) for k in kinds]
    groups = []
    start = 0
    for i in range(1, len(kinds) + 1):
        if i == len(kinds) or kinds[i] != kinds[start]:
            groups.append((kinds[start], start, i))
            start = i
    arr = (BatchGroup * len(groups))()
    for g, (k, a, b) in enumerate(groups):
        arr[g].kind.kind = k
        arr[g].series_begin = a
        arr[g].series_end = b
    return arr


def batched_loglik(kinds, offsets, params, t, y, mask=None, dtype="float32", options=None, device="cuda"):
    """Per-series log-likelihoods of a batch (pssgp_batched_loglik); kinds,
    offsets, params as for BatchedPipeline. Returns a float64 tensor
    [n_series]."""
    _require_gpu()
    torch = _torch()
    groups = batch_groups(kinds)
    off_h = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    ns = off_h.shape[0] - 1
    code, tdt = _dt(dtype)
    L = lib()
    op = ctypes.byref(options) if options is not None else None
    nb = L.pssgp_batched_workspace_bytes(groups, len(groups), ns, off_h.ctypes.data, code, OP_LOGLIK, op)
    if nb == 0:
        raise PssgpError(-1, L.pssgp_last_error().decode())
    ws = torch.empty(nb, dtype=torch.uint8, device=device)
    off_d = torch.as_tensor(off_h, device=device)
    prm = _dev(np.asarray(params, dtype=np.float64).reshape(ns, 3), torch.float64, device)
    t = _dev(t, torch.float64, device)
    y = _dev(y, tdt, device)
    mask = _dev(mask, torch.uint8, device) if mask is not None else None
    ll = torch.empty(ns, dtype=torch.float64, device=device)
    _check(L.pssgp_batched_loglik(groups, len(groups), ns, _p(off_d), off_h.ctypes.data, _p(prm), _p(t), _p(y),
                                  _p(mask), code, _p(ll), _p(ws), ws.numel(), op, _stream()))
    return ll


class BatchedPipeline:
    """Preallocated batched filter + smoother over concatenated series.

    kinds: per-series Matern kind (sorted by state size, at most two kinds);
    offsets: int64 [n_series + 1]; params: float64 [n_series, 3] with
    (lengthscale, variance, noise_var) per series. fused=True runs both scans
    in one pssgp_batched_predict call (smoother elements handed over in the
    workspace, no filter moments in memory); fused=False runs
    pssgp_batched_filter, keeps m and P, then pssgp_batched_smooth.
    """

    def __init__(self, kinds, offsets, params, dtype="float32", options=None, device="cuda", fused=True):
        _require_gpu()
        torch = _torch()
        self.groups = batch_groups(kinds)
        self.ng = len(self.groups)
        self.offsets_host = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.ns = self.offsets_host.shape[0] - 1
        self.n = int(self.offsets_host[-1])
        self.offsets = torch.as_tensor(self.offsets_host, device=device)
        self.params = _dev(np.asarray(params, dtype=np.float64).reshape(self.ns, 3), torch.float64, device)
        self.code, self.tdt = _dt(dtype)
        self.options = options
        dmax = max(_STATE_DIM[int(k)] for k in kinds)
        self.dmax = dmax
        L = lib()
        op = ctypes.byref(options) if options is not None else None
        self.fused = bool(fused)
        ops = (OP_PREDICT,) if self.fused else (OP_FILTER, OP_SMOOTH)
        nbs = [L.pssgp_batched_workspace_bytes(self.groups, self.ng, self.ns, self.offsets_host.ctypes.data,
                                               self.code, o, op) for o in ops]
        if min(nbs) == 0:
            raise PssgpError(-1, L.pssgp_last_error().decode())
        if self.fused:
            self.ws_p = torch.empty(nbs[0], dtype=torch.uint8, device=device)
            self.ws_f = self.ws_s = self.ws_p
            self.m = self.P = None
        else:
            self.ws_f = torch.empty(nbs[0], dtype=torch.uint8, device=device)
            self.ws_s = torch.empty(nbs[1], dtype=torch.uint8, device=device)
            self.m = torch.empty((dmax, self.n), dtype=self.tdt, device=device)
            self.P = torch.empty((dmax * (dmax + 1) // 2, self.n), dtype=self.tdt, device=device)
        self.loglik = torch.empty(self.ns, dtype=torch.float64, device=device)
        self.f_mean = torch.empty(self.n, dtype=self.tdt, device=device)
        self.f_var = torch.empty(self.n, dtype=self.tdt, device=device)

    def run(self, t, y, mask=None, events=None, pass_events=None):
        """events: optional 3 torch.cuda.Event (before, between, after the
        two scans; the middle one coincides with the last when fused);
        pass_events: optional (filter, smoother) pair of lists of 4 events."""
        L = lib()
        op = ctypes.byref(self.options) if self.options is not None else None
        st = _stream()
        oh = self.offsets_host.ctypes.data
        if self.fused:
            if pass_events is not None:
                op = ctypes.byref(_with_events(self.options, list(pass_events[0]) + list(pass_events[1])))
            if events:
                events[0].record()
            _check(L.pssgp_batched_predict(self.groups, self.ng, self.ns, _p(self.offsets), oh, _p(self.params),
                                           _p(t), _p(y), _p(mask), self.code, _p(self.f_mean), _p(self.f_var),
                                           _p(self.loglik), _p(self.ws_p), self.ws_p.numel(), op, st))
            if events:
                events[1].record()
                events[2].record()
            return self.f_mean, self.f_var, self.loglik
        op_f = op_s = op
        if pass_events is not None:
            op_f = ctypes.byref(_with_events(self.options, pass_events[0]))
            op_s = ctypes.byref(_with_events(self.options, pass_events[1]))
        if events:
            events[0].record()
        _check(L.pssgp_batched_filter(self.groups, self.ng, self.ns, _p(self.offsets), oh, _p(self.params), _p(t),
                                      _p(y), _p(mask), self.code, _p(self.m), _p(self.P), _p(self.loglik),
                                      _p(self.ws_f), self.ws_f.numel(), op_f, st))
        if events:
            events[1].record()
        _check(L.pssgp_batched_smooth(self.groups, self.ng, self.ns, _p(self.offsets), oh, _p(self.params), _p(t),
                                      _p(self.m), _p(self.P), self.code, _p(self.f_mean), _p(self.f_var),
                                      _p(self.ws_s), self.ws_s.numel(), op_s, st))
        if events:
            events[2].record()
        return self.f_mean, self.f_var, self.loglik
