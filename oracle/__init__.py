"""FP64 CPU oracle for the explicit Grunwald-Letnikov fractional
reaction-diffusion scheme (Sprouse, MacDonald & Silva, arXiv:1004.5128).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library and its Python binding never do, and the two share no code.

This module is argument marshalling (numpy <-> C) around ``gl_oracle.c``,
where every computation lives and where each function cites the passage of
the paper it follows.  Problems and memory settings are plain dicts, the
form the seeded workload generators emit:

  problem = {"ndim", "nx", "ny", "nz", "dx", "dt", "gamma", "alpha", "rxn", "rate"}
            ("ny" and "nz" may be left out below 2D and 3D)
            rxn in {"none", "linear", "fisher"}
  memory  = {"mode", "L", "a", "rule"}
            mode in {"full", "short", "adaptive"},
            rule in {"partition", "literal", "unit_stride"}
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODES = {"full": 0, "short": 1, "adaptive": 2}
RULES = {"partition": 0, "literal": 1, "unit_stride": 2}
RXNS = {"none": 0, "linear": 1, "fisher": 2}


class _Problem(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("gamma", C.c_double),
                ("alpha", C.c_double), ("rxn", C.c_int32), ("rate", C.c_double)]


class _Memory(C.Structure):
    _fields_ = [("mode", C.c_int32), ("rule", C.c_int32), ("L", C.c_int64), ("a", C.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    lp = C.POINTER(C.c_int64)
    fp = C.POINTER(C.c_float)
    lib.orc_psi.argtypes = [C.c_double, C.c_int64, dp]
    lib.orc_psi.restype = None
    lib.orc_dpsi.argtypes = [C.c_double, C.c_int64, dp]
    lib.orc_dpsi.restype = None
    lib.orc_schedule.argtypes = [C.POINTER(_Memory), C.c_int64, lp, dp, C.c_int64]
    lib.orc_schedule.restype = C.c_int64
    lib.orc_r.argtypes = [C.POINTER(_Problem)]
    lib.orc_r.restype = C.c_double
    lib.orc_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Memory), dp, C.c_int64, dp, C.c_int]
    lib.orc_run.restype = C.c_int
    lib.orc_mode_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Memory), C.c_int32, C.c_int32,
                                 C.c_int32, C.c_double, C.c_int64, dp]
    lib.orc_mode_run.restype = C.c_int
    lib.orc_history_sum.argtypes = [C.c_double, C.POINTER(_Memory), C.c_int64, fp, C.c_int64,
                                    C.c_int64, dp]
    lib.orc_history_sum.restype = None
    lib.orc_adjoint.argtypes = [C.POINTER(_Problem), C.POINTER(_Memory), dp, C.c_int64, dp, dp,
                                dp, dp]
    lib.orc_adjoint.restype = C.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _problem(p):
    return _Problem(int(p["ndim"]), int(p["nx"]), int(p.get("ny", 1)), int(p.get("nz", 1)),
                    float(p["dx"]),
                    float(p["dt"]), float(p["gamma"]), float(p["alpha"]),
                    RXNS[p.get("rxn", "none")], float(p.get("rate", 0.0)))


def _memory(m):
    m = m or {"mode": "full"}
    return _Memory(MODES[m["mode"]], RULES[m.get("rule", "partition")], int(m.get("L", 0)),
                   int(m.get("a", 2)))


def npoints(p):
    nd = int(p["ndim"])
    return (int(p["nx"]) * (int(p.get("ny", 1)) if nd >= 2 else 1) *
            (int(p.get("nz", 1)) if nd == 3 else 1))


def psi(gamma, n):
    """psi(gamma, m), m = 0..n (Sec. 2.1, eqs. 11-12)."""
    out = np.empty(n + 1, np.float64)
    _load().orc_psi(float(gamma), int(n), _dptr(out))
    return out


def dpsi(gamma, n):
    """d psi(gamma, m) / d gamma, m = 0..n (derivative of the recurrence, eq. 11)."""
    out = np.empty(n + 1, np.float64)
    _load().orc_dpsi(float(gamma), int(n), _dptr(out))
    return out


def schedule(memory, k):
    """(offsets m, multiplicities c) summed at step k (eqs. 21, 22, 24)."""
    mem = _memory(memory)
    lib = _load()
    cap = k + 1
    while True:
        ms = np.empty(cap, np.int64)
        cs = np.empty(cap, np.float64)
        n = lib.orc_schedule(C.byref(mem), int(k), ms.ctypes.data_as(C.POINTER(C.c_int64)),
                             _dptr(cs), cap)
        if n <= cap:
            return ms[:n].copy(), cs[:n].copy()
        cap = n


def r_of(problem):
    """r = alpha dt^gamma / dx^2."""
    return _load().orc_r(C.byref(_problem(problem)))


def run(problem, memory, u0, nsteps, store_all=False):
    """u[nsteps] (or u[0..nsteps] if store_all) of the scheme of eq. (21)."""
    P = npoints(problem)
    u0 = np.ascontiguousarray(u0, np.float64).reshape(-1)
    assert u0.size == P
    out = np.empty(((nsteps + 1) * P) if store_all else P, np.float64)
    rc = _load().orc_run(C.byref(_problem(problem)), C.byref(_memory(memory)), _dptr(u0),
                         int(nsteps), _dptr(out), 1 if store_all else 0)
    if rc != 0:
        raise MemoryError("oracle run: out of memory")
    return out.reshape(nsteps + 1, P) if store_all else out


def mode_run(problem, memory, p, q, v0, n, s=1):
    """Amplitude v[0..n] of the discrete sine mode (p, q[, s]) under the scheme (linear f)."""
    out = np.empty(n + 1, np.float64)
    rc = _load().orc_mode_run(C.byref(_problem(problem)), C.byref(_memory(memory)), int(p),
                              int(q), int(s), float(v0), int(n), _dptr(out))
    if rc != 0:
        raise ValueError("oracle mode_run: nonlinear reaction or out of memory")
    return out


def history_sum(gamma, memory, k, H):
    """S[p] = sum over the schedule at step k of c psi(m) H[k-m, p], FP64, H float32 [rows, P]."""
    H = np.ascontiguousarray(H, np.float32)
    assert H.ndim == 2 and H.shape[0] >= k + 1
    S = np.empty(H.shape[1], np.float64)
    _load().orc_history_sum(float(gamma), C.byref(_memory(memory)), int(k),
                            H.ctypes.data_as(C.POINTER(C.c_float)), H.shape[1], H.shape[1],
                            _dptr(S))
    return S


def adjoint(problem, memory, u0, n, target):
    """(loss, dL/du0, [dL/dalpha, dL/dgamma, dL/drate]) for 0.5||u[n]-target||^2."""
    P = npoints(problem)
    u0 = np.ascontiguousarray(u0, np.float64).reshape(-1)
    target = np.ascontiguousarray(target, np.float64).reshape(-1)
    du0 = np.empty(P, np.float64)
    dpar = np.empty(3, np.float64)
    loss = np.empty(1, np.float64)
    rc = _load().orc_adjoint(C.byref(_problem(problem)), C.byref(_memory(memory)), _dptr(u0),
                             int(n), _dptr(target), _dptr(loss), _dptr(du0), _dptr(dpar))
    if rc != 0:
        raise MemoryError("oracle adjoint: out of memory")
    return float(loss[0]), du0, dpar


def num_threads():
    return int(_load().orc_num_threads())
