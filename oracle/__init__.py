"""Oracle for the parallel state-space GP path: a plain, slow, obviously
correct sequential CPU implementation in FP64.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here.
The GPU library never imports it and shares no code with it; the only module
both sides use is ``workloads`` (seeded input generators, no arithmetic of
the method).

Pieces:
* ``model.py``  -- continuous model construction (Matern-1/2, 3/2, 5/2,
  RBF Taylor approximation, sums), Lyapunov equation, Osborne balancing,
  complex-step parameter derivatives (numpy).
* ``ssgp_seq.c`` -- sequential Kalman filter, RTS smoother, log-likelihood
  and forward-mode gradient with Van Loan discretisation (C, FP64). Built
  into ``liboracle.so`` by :func:`build`.

State outputs are returned in the canonical companion coordinates of
``model.model_ssm`` (the oracle balances internally, section 4.2, and undoes
the scaling on output).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .model import MATERN12, MATERN32, MATERN52, RBF, OracleModel  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssgp_seq.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C core (gcc -O2, plain scalar code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-D_DEFAULT_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("G", ctypes.c_void_p), ("W", ctypes.c_void_p), ("Pinf", ctypes.c_void_p),
        ("H", ctypes.c_void_p), ("R", ctypes.c_double), ("np", ctypes.c_int),
        ("dG", ctypes.c_void_p), ("dW", ctypes.c_void_p), ("dPinf", ctypes.c_void_p),
        ("dR", ctypes.c_void_p),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            lib.ssgp_run.restype = ctypes.c_int
            lib.ssgp_run.argtypes = [ctypes.POINTER(_Model), ctypes.c_int64] + [ctypes.c_void_p] * 12
            lib.ssgp_loglik_terms.restype = ctypes.c_int
            lib.ssgp_loglik_terms.argtypes = [ctypes.POINTER(_Model), ctypes.c_int64] + [ctypes.c_void_p] * 5
            lib.ssgp_discretize.restype = ctypes.c_int
            lib.ssgp_discretize.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
            lib.ssgp_expm.restype = ctypes.c_int
            lib.ssgp_expm.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def expm(a: np.ndarray) -> np.ndarray:
    """The oracle's own matrix exponential (Pade-13 scaling and squaring)."""
    a = _c(a)
    out = np.empty_like(a)
    rc = _load().ssgp_expm(a.shape[0], _ptr(a), _ptr(out))
    if rc:
        raise RuntimeError("ssgp_expm failed: %d" % rc)
    return out


def discretize(model: OracleModel, dt: float):
    """(F, Q) for a step of length dt, in canonical coordinates."""
    d = model.d
    F = np.empty((d, d))
    Q = np.empty((d, d))
    Gb, Wb = _c(model.Gb), _c(model.Wb)
    rc = _load().ssgp_discretize(d, _ptr(Gb), _ptr(Wb), float(dt), _ptr(F), _ptr(Q))
    if rc:
        raise RuntimeError("ssgp_discretize failed: %d" % rc)
    D = model.D
    return D[:, None] * F / D[None, :], D[:, None] * Q * D[None, :]


def run(model: OracleModel, t, y, mask=None, noise_k=None, filter_moments=True,
        smoother=True, gradient=False):
    """Sequential filter / smoother / log-likelihood / gradient.

    Returns a dict with 'loglik' and, as requested, 'mf', 'Pf' (filter),
    'ms', 'Ps' (smoother), 'f_mean', 'f_var', 'grad' (order: ell_0, var_0,
    ..., noise_var). State moments are in canonical coordinates.
    """
    lib = _load()
    t = _c(t)
    y = _c(y)
    n = t.shape[0]
    d = model.d
    mask_a = None if mask is None else _c(mask, np.uint8)
    nk = _c(noise_k)
    keep = []
    Gb, Wb, Pb, Hb = _c(model.Gb), _c(model.Wb), _c(model.Pinfb), _c(model.Hb)
    keep += [Gb, Wb, Pb, Hb]
    cm = _Model(d, _ptr(Gb), _ptr(Wb), _ptr(Pb), _ptr(Hb), model.noise_var, 0, None, None, None, None)
    grad = None
    if gradient:
        if model.dGb is None:
            raise ValueError("model was built without derivatives")
        dG, dW, dP, dR = _c(model.dGb), _c(model.dWb), _c(model.dPinfb), _c(model.dR)
        keep += [dG, dW, dP, dR]
        cm.np = model.n_params
        cm.dG, cm.dW, cm.dPinf, cm.dR = _ptr(dG), _ptr(dW), _ptr(dP), _ptr(dR)
        grad = np.zeros(model.n_params)
    mf = np.empty((n, d)) if filter_moments else None
    Pf = np.empty((n, d, d)) if filter_moments else None
    ms = np.empty((n, d)) if smoother else None
    Ps = np.empty((n, d, d)) if smoother else None
    fmean = np.empty(n) if smoother else None
    fvar = np.empty(n) if smoother else None
    ll = np.zeros(1)
    rc = lib.ssgp_run(ctypes.byref(cm), n, _ptr(t), _ptr(y), _ptr(mask_a), _ptr(nk),
                      _ptr(mf), _ptr(Pf), _ptr(ms), _ptr(Ps), _ptr(fmean), _ptr(fvar),
                      _ptr(ll), _ptr(grad))
    if rc:
        raise RuntimeError("ssgp_run failed: %d" % rc)
    D = model.D
    out = {"loglik": float(ll[0])}
    if filter_moments:
        out["mf"] = mf * D[None, :]
        out["Pf"] = Pf * D[None, :, None] * D[None, None, :]
    if smoother:
        out["ms"] = ms * D[None, :]
        out["Ps"] = Ps * D[None, :, None] * D[None, None, :]
        out["f_mean"] = fmean
        out["f_var"] = fvar
    if gradient:
        out["grad"] = grad
    return out


def loglik_terms(model: OracleModel, t, y, mask=None, noise_k=None) -> np.ndarray:
    """Per-step log-likelihood terms of the sequential filter (0 at missing
    steps); their sum is run()'s loglik, their absolute sum the condition
    number of that sum."""
    lib = _load()
    t = _c(t)
    y = _c(y)
    n = t.shape[0]
    mask_a = None if mask is None else _c(mask, np.uint8)
    nk = _c(noise_k)
    Gb, Wb, Pb, Hb = _c(model.Gb), _c(model.Wb), _c(model.Pinfb), _c(model.Hb)
    cm = _Model(model.d, _ptr(Gb), _ptr(Wb), _ptr(Pb), _ptr(Hb), model.noise_var, 0, None, None, None, None)
    out = np.empty(max(n, 1))
    rc = lib.ssgp_loglik_terms(ctypes.byref(cm), n, _ptr(t), _ptr(y), _ptr(mask_a), _ptr(nk), _ptr(out))
    if rc:
        raise RuntimeError("ssgp_loglik_terms failed: %d" % rc)
    return out[:n]


def run_batched(models, offsets, t, y, mask=None, threads=None, smoother=True, abs_terms=False):
    """Independent series (CSR offsets) spread over host threads; returns
    per-series loglik and concatenated f_mean / f_var (abs_terms: also the
    per-series sum of absolute log-likelihood terms)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    ns = offsets.shape[0] - 1
    total = int(offsets[-1])
    f_mean = np.empty(total) if smoother else None
    f_var = np.empty(total) if smoother else None
    ll = np.empty(ns)
    lla = np.empty(ns) if abs_terms else None

    def one(s):
        a, b = int(offsets[s]), int(offsets[s + 1])
        r = run(models[s], t[a:b], y[a:b], None if mask is None else mask[a:b],
                filter_moments=False, smoother=smoother)
        ll[s] = r["loglik"]
        if abs_terms:
            lla[s] = float(np.sum(np.abs(loglik_terms(models[s], t[a:b], y[a:b],
                                                       None if mask is None else mask[a:b]))))
        if smoother:
            f_mean[a:b] = r["f_mean"]
            f_var[a:b] = r["f_var"]

    threads = threads or os.cpu_count() or 1
    if threads <= 1:
        for s in range(ns):
            one(s)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(ns)))
    out = {"loglik": ll, "f_mean": f_mean, "f_var": f_var}
    if abs_terms:
        out["loglik_abs_terms"] = lla
    return out
