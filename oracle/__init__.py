"""FP64 CPU oracle for MPL / batch-mode MPL (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU library neither imports nor links it, and it imports nothing
from the GPU package.  The arithmetic lives in ``mpl_oracle.c`` (plain C,
float64, OpenMP over signals); this file marshals numpy arrays through ctypes.

Status bits returned per signal: 1 converged (natural stop, Eq. (9)),
2 iteration cap, 4 active-set cap, 8 non-finite input, 32 a restricted solve
could not be verified exact, 64 an early stop (Eq. (10) or Eq. (13)).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmpl_oracle.so")
_lib = None

ST_CONVERGED, ST_CAP_ITERS, ST_CAP_ACTIVE, ST_NONFINITE, ST_INEXACT, ST_EARLY = 1, 2, 4, 8, 32, 64

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "mpl_oracle.c")):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.mpl_oracle_solve.restype = ctypes.c_int
    lib.mpl_oracle_solve.argtypes = [_fp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _fp, ctypes.c_int64,
                                     ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int64, _ip, _dp, _dp, _dp, _dp, _ip,
                                     _ip]
    lib.mpl_oracle_trace.restype = ctypes.c_int
    lib.mpl_oracle_trace.argtypes = [_fp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _fp, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, _dp, _ip, _dp, _dp, _dp, _dp, _ip, _ip, _dp, _ip, _dp, _ip]
    lib.mpl_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def max_threads() -> int:
    return int(_load().mpl_oracle_max_threads())


def solve(At: np.ndarray, Bt: np.ndarray, lam, rho: int, max_outer: int | None = None,
          max_active: int | None = None, nthreads: int = 0, omega: int = 1, eps_early: float = 0.0,
          r_inf_rel: float = 0.0, r2_rel: float = 0.0) -> dict:
    """Solve every row of Bt; returns dense X (p, m) float64 and per-signal arrays.
    omega > 1 runs subspace exploratory matching (Algorithm 2, SMPL) with omega * rho candidates;
    eps_early > 0 adds the objective-decrease stop of Eq. (13); r_inf_rel / r2_rel > 0 add the stops of
    Eq. (10) with r_inf = r_inf_rel ||A^T b||_inf and r_2 = r2_rel ||b||."""
    lib = _load()
    At = np.ascontiguousarray(At, dtype=np.float32)
    Bt = np.ascontiguousarray(np.atleast_2d(Bt), dtype=np.float32)
    m, n = At.shape
    p = Bt.shape[0]
    lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (p,)))
    if max_outer is None:
        max_outer = -(-m // rho)
    if max_active is None:
        max_active = min(m, 2 * n)
    X = np.zeros((p, m), dtype=np.float64)
    it = np.zeros(p, np.int32)
    kkt, obj, mar, gap = (np.zeros(p) for _ in range(4))
    st = np.zeros(p, np.int32)
    sl = np.zeros(p, np.int32)
    rc = lib.mpl_oracle_solve(_ptr(At, _fp), n, n, m, _ptr(Bt, _fp), n, p, _ptr(lam, _dp), rho, omega,
                              float(eps_early), float(r_inf_rel), float(r2_rel), max_outer, max_active, nthreads, _ptr(X, _dp), m, _ptr(it, _ip), _ptr(kkt, _dp),
                              _ptr(obj, _dp), _ptr(mar, _dp), _ptr(gap, _dp), _ptr(st, _ip), _ptr(sl, _ip))
    if rc != 0:
        raise ValueError("mpl_oracle_solve rejected its arguments")
    return {"X": X, "iters": it, "kkt": kkt, "objective": obj, "margin": mar, "gap": gap,
            "status": st, "supp_len": sl, "lambda": lam}


def trace(At: np.ndarray, b: np.ndarray, lam: float, rho: int, max_outer: int | None = None,
          max_active: int | None = None, omega: int = 1, eps_early: float = 0.0, r_inf_rel: float = 0.0,
          r2_rel: float = 0.0) -> dict:
    """One signal, with the objective after every outer iteration and the atoms added."""
    lib = _load()
    At = np.ascontiguousarray(At, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    m, n = At.shape
    if max_outer is None:
        max_outer = -(-m // rho)
    if max_active is None:
        max_active = min(m, 2 * n)
    x = np.zeros(m)
    it = np.zeros(1, np.int32)
    kkt, obj, mar, gap = (np.zeros(1) for _ in range(4))
    st = np.zeros(1, np.int32)
    sl = np.zeros(1, np.int32)
    ot = np.zeros(max_outer + 1)
    added = np.full(max(1, max_outer * rho), -1, np.int32)
    gsel = np.zeros(max(1, max_outer * rho))
    nadd = np.zeros(max(1, max_outer), np.int32)
    rc = lib.mpl_oracle_trace(_ptr(At, _fp), n, n, m, _ptr(b, _fp), float(lam), rho, omega, float(eps_early),
                              float(r_inf_rel), float(r2_rel), max_outer, max_active,
                              _ptr(x, _dp), _ptr(it, _ip), _ptr(kkt, _dp), _ptr(obj, _dp), _ptr(mar, _dp),
                              _ptr(gap, _dp), _ptr(st, _ip), _ptr(sl, _ip), _ptr(ot, _dp), _ptr(added, _ip),
                              _ptr(gsel, _dp), _ptr(nadd, _ip))
    if rc != 0:
        raise ValueError("mpl_oracle_trace rejected its arguments")
    T = int(it[0])
    steps = []
    for t in range(T):
        q = int(nadd[t])
        steps.append((added[t * rho:t * rho + q].copy(), gsel[t * rho:t * rho + q].copy()))
    return {"x": x, "iters": T, "kkt": float(kkt[0]), "objective": float(obj[0]), "margin": float(mar[0]),
            "gap": float(gap[0]), "status": int(st[0]), "supp_len": int(sl[0]), "obj_trace": ot[:T + 1].copy(),
            "steps": steps}
