"""FP64 CPU oracle of the PDR method (arXiv 2108.07549) -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It never serves the product path and shares no code with it.

``pdr_oracle.c`` holds the arithmetic (Algorithms 1-4, the capacity-enforcing
edge step for Section 6's formulation and the definitions of Sections 3-5, in
FP64); this module builds it with gcc and wraps it with ctypes.
Flows are m x K arrays in the caller's CSR arc order.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ESO, AGD, GDM, CAP = 0, 1, 2, 3
VERDICT = {0: "undecided", 1: "feasible", 2: "infeasible"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _AgdParams(C.Structure):
    _fields_ = [("beta_init", C.c_double), ("beta_min", C.c_double), ("beta_max", C.c_double),
                ("alpha_inc", C.c_double), ("alpha_dec", C.c_double), ("inc_period", C.c_int32),
                ("gamma", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_degrees.argtypes = [i32, i32, P, P, P]
        L.orc_excess.argtypes = [i32, i32, P, P, i32, P, P, P, P, P, P]
        L.orc_congestion.argtypes = [i32, i32, P, P, P, P]
        L.orc_objective.argtypes = [i32, i32, P, i32, P, P, P]
        L.orc_objective_edge_form.argtypes = [i32, i32, P, P, i32, P, P]
        L.orc_objective_edge_form.restype = dbl
        L.orc_eso_edge.argtypes = [i32, P, P, P, dbl, P, P, P, P]
        L.orc_eso_edge.restype = C.c_int
        L.orc_cap_edge.argtypes = [i32, P, P, P, dbl, P, P, P]
        L.orc_cap_edge.restype = C.c_int
        L.orc_agd_edge.argtypes = [i32, P, P, P, dbl, dbl, dbl, i64, P, dbl, dbl, dbl, dbl, i32,
                                   P, P]
        L.orc_agd_edge.restype = C.c_int
        L.orc_gdm_edge.argtypes = [i32, P, P, P, P, dbl, dbl, dbl, i64, P, dbl, dbl, dbl, dbl,
                                   i32, dbl, P, P, P]
        L.orc_gdm_edge.restype = C.c_int
        L.orc_run.argtypes = [i32, i32, P, P, P, i32, P, P, P, i32, C.POINTER(_AgdParams), i64,
                              dbl, dbl, P, P, P, P, P, P, P]
        L.orc_run.restype = i64
        L.orc_eso_tangent.argtypes = [i32, i32, P, P, P, i32, P, P, P, P, P, i64, P, P, P, P]
        L.orc_eso_tangent.restype = None
        L.orc_report.argtypes = [i32, i32, P, P, P, i32, P, P, P, P, dbl, P]
        L.orc_report.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(nt: int) -> None:
    """Threads of later oracle calls (for timing; results do not depend on it)."""
    lib().orc_set_num_threads(int(nt))


def degrees(inst) -> np.ndarray:
    deg = np.zeros(inst.n, np.int32)
    rp, col = _c(inst.row_ptr, np.int64), _c(inst.col, np.int32)
    lib().orc_degrees(inst.n, inst.m, _p(rp), _p(col), _p(deg))
    return deg


def excess(inst, f):
    """(Delta, h) as n x K arrays for flows f (m x K)."""
    n, m, K = inst.n, inst.m, inst.K
    Delta = np.zeros((n, K))
    h = np.zeros((n, K))
    args = [_c(inst.row_ptr, np.int64), _c(inst.col, np.int32), _c(inst.s, np.int32),
            _c(inst.t, np.int32), _c(inst.d, np.float64), _c(f, np.float64).reshape(m, K)]
    lib().orc_excess(n, m, _p(args[0]), _p(args[1]), K, _p(args[2]), _p(args[3]), _p(args[4]),
                     _p(args[5]), _p(Delta), _p(h))
    return Delta, h


def congestion(inst, f):
    """(F, psi): arc flow totals and congestion."""
    m, K = inst.m, inst.K
    F = np.zeros(m)
    psi = np.zeros(m)
    fc = _c(f, np.float64).reshape(m, K)
    u = _c(inst.u, np.float64)
    lib().orc_congestion(m, K, _p(fc), _p(u), _p(F), _p(psi))
    return F, psi


def objective(inst, h, psi):
    """(z, z_psi, z_h) as Algorithm 1 computes z."""
    deg = degrees(inst)
    out = np.zeros(3)
    hc = _c(h, np.float64)
    pc = _c(psi, np.float64)
    lib().orc_objective(inst.n, inst.m, _p(deg), inst.K, _p(hc), _p(pc), _p(out))
    return tuple(out.tolist())


def objective_edge_form(inst, h, psi) -> float:
    hc, pc = _c(h, np.float64), _c(psi, np.float64)
    rp, col = _c(inst.row_ptr, np.int64), _c(inst.col, np.int32)
    return float(lib().orc_objective_edge_form(inst.n, inst.m, _p(rp), _p(col), inst.K,
                                               _p(hc), _p(pc)))


def eso_edge(hi, hj, fe, u):
    """Algorithm 2 on one arc: returns (f_new, psi, r, congested)."""
    hi, hj, fe = (_c(x, np.float64) for x in (hi, hj, fe))
    K = hi.shape[0]
    out = np.zeros(K)
    work = np.zeros(max(K, 1))
    psi = np.zeros(1)
    r = np.zeros(1)
    cg = lib().orc_eso_edge(K, _p(hi), _p(hj), _p(fe), float(u), _p(out), _p(work), _p(psi), _p(r))
    return out, float(psi[0]), float(r[0]), bool(cg)


def cap_edge(hi, hj, fe, u):
    """Capacity-enforcing edge step (Section 6's formulation): returns
    (f_new, lambda, binds)."""
    hi, hj, fe = (_c(x, np.float64) for x in (hi, hj, fe))
    K = hi.shape[0]
    out = np.zeros(K)
    work = np.zeros(max(K, 1))
    lam = np.zeros(1)
    b = lib().orc_cap_edge(K, _p(hi), _p(hj), _p(fe), float(u), _p(out), _p(work), _p(lam))
    return out, float(lam[0]), bool(b)


def gdm_edge(hi, hj, fe, ve, u, t, beta, params=None):
    """One GDM arc step: returns (f_new, v_new, beta_new, accepted, dz)."""
    hi, hj, fe, ve = (_c(x, np.float64) for x in (hi, hj, fe, ve))
    K = hi.shape[0]
    p = default_gdm_params(K) if params is None else params
    F = 0.0
    for x in fe.tolist():
        F += x
    psi = max(0.0, F - u)
    b = np.array([beta], np.float64)
    fo = np.zeros(K)
    vo = np.zeros(K)
    dz = np.zeros(1)
    a = lib().orc_gdm_edge(K, _p(hi), _p(hj), _p(fe), _p(ve), F, float(u), psi, int(t), _p(b),
                           p["beta_min"], p["beta_max"], p["alpha_inc"], p["alpha_dec"],
                           int(p["inc_period"]), p["gamma"], _p(fo), _p(vo), _p(dz))
    return fo, vo, float(b[0]), bool(a), float(dz[0])


def agd_edge(hi, hj, fe, u, t, beta, params=None):
    """One AGD arc step: returns (f_new, beta_new, accepted, dz)."""
    hi, hj, fe = (_c(x, np.float64) for x in (hi, hj, fe))
    K = hi.shape[0]
    p = default_agd_params(K) if params is None else params
    F = float(np.sum(fe)) if K else 0.0
    acc = 0.0
    for x in fe.tolist():
        acc += x
    F = acc
    psi = max(0.0, F - u)
    b = np.array([beta], np.float64)
    out = np.zeros(K)
    dz = np.zeros(1)
    a = lib().orc_agd_edge(K, _p(hi), _p(hj), _p(fe), F, float(u), psi, int(t), _p(b),
                           p["beta_min"], p["beta_max"], p["alpha_inc"], p["alpha_dec"],
                           int(p["inc_period"]), _p(out), _p(dz))
    return out, float(b[0]), bool(a), float(dz[0])


def default_agd_params(K: int) -> dict:
    """AGD parameters of the paper's experiments (Section 7.2)."""
    return dict(beta_init=0.25, beta_min=1.0 / K, beta_max=0.5, alpha_inc=2.0, alpha_dec=0.5,
                inc_period=10, gamma=0.0)


def default_gdm_params(K: int) -> dict:
    """GDM parameters of the paper's experiments (Section 7.2)."""
    return dict(beta_init=0.1, beta_min=1.0 / K, beta_max=0.2, alpha_inc=2.0, alpha_dec=0.5,
                inc_period=10, gamma=0.9)


def default_params(method: int, K: int) -> dict:
    return default_gdm_params(K) if method == GDM else default_agd_params(K)


class State:
    """Resumable oracle run state: flows, AGD/GDM rates, GDM velocities, iteration
    counter, z_prev."""

    def __init__(self, inst, method=ESO, params=None):
        self.inst = inst
        self.method = method
        self.params = default_params(method, inst.K) if params is None else dict(params)
        self.params.setdefault("gamma", 0.0)
        self.f = np.zeros((inst.m, inst.K))
        self.v = np.zeros((inst.m, inst.K))
        self.beta = np.full(inst.m, self.params["beta_init"])
        self.t = 0
        self.z_prev = math.inf
        self.stopped = False

    def run(self, max_iter, eps_obj=0.0, z_target=0.0, record=True):
        """Run up to max_iter passes of Algorithm 1/3; returns the recorded z values."""
        inst = self.inst
        n, m, K = inst.n, inst.m, inst.K
        args = [_c(inst.row_ptr, np.int64), _c(inst.col, np.int32), _c(inst.u, np.float64),
                _c(inst.s, np.int32), _c(inst.t, np.int32), _c(inst.d, np.float64)]
        prm = _AgdParams(**self.params)
        zh = np.full(max(int(max_iter), 1), np.nan) if record else None
        t = np.array([self.t], np.int64)
        zp = np.array([self.z_prev], np.float64)
        st = np.zeros(1, np.int32)
        done = lib().orc_run(n, m, _p(args[0]), _p(args[1]), _p(args[2]), K, _p(args[3]),
                             _p(args[4]), _p(args[5]), int(self.method), C.byref(prm),
                             int(max_iter), float(eps_obj), float(z_target), _p(self.f),
                             _p(self.beta), _p(self.v), _p(t), _p(zp),
                             _p(zh) if record else None, _p(st))
        self.t = int(t[0])
        self.z_prev = float(zp[0])
        self.stopped = bool(st[0])
        if not record:
            return None
        npass = int(done) + (1 if self.stopped else 0)
        return zh[:npass]


def run(inst, method=ESO, T=1, eps_obj=0.0, z_target=0.0, params=None):
    """Run T passes from f = 0; returns (State, z history)."""
    st = State(inst, method, params)
    zs = st.run(T, eps_obj, z_target)
    return st, zs


def eso_tangent(inst, T, du, dd, f0=None):
    """T PDR-ESO sweeps from f0 (default 0) with the forward-mode tangent along
    (du, dd): returns (f^T, fdot^T, z(f^T), dz along (du, dd))."""
    m, K = inst.m, inst.K
    f = np.zeros((m, K)) if f0 is None else np.array(f0, np.float64).reshape(m, K)
    fdot = np.zeros((m, K))
    z = np.zeros(1)
    zd = np.zeros(1)
    args = [_c(inst.row_ptr, np.int64), _c(inst.col, np.int32), _c(inst.u, np.float64),
            _c(inst.s, np.int32), _c(inst.t, np.int32), _c(inst.d, np.float64),
            _c(du, np.float64), _c(dd, np.float64)]
    lib().orc_eso_tangent(inst.n, m, _p(args[0]), _p(args[1]), _p(args[2]), K, _p(args[3]),
                          _p(args[4]), _p(args[5]), _p(args[6]), _p(args[7]), int(T), _p(f),
                          _p(fdot), _p(z), _p(zd))
    return f, fdot, float(z[0]), float(zd[0])


def eso_gradient(inst, T, f0=None):
    """Gradient of z(f^T) after T PDR-ESO sweeps with respect to every
    capacity and demand, one forward-mode run per coordinate: (z, dz/du, dz/dd)."""
    m, K = inst.m, inst.K
    gu, gd = np.zeros(m), np.zeros(K)
    z = None
    for j in range(m + K):
        du, dd = np.zeros(m), np.zeros(K)
        if j < m:
            du[j] = 1.0
        else:
            dd[j - m] = 1.0
        _, _, z, zd = eso_tangent(inst, T, du, dd, f0)
        if j < m:
            gu[j] = zd
        else:
            gd[j - m] = zd
    return z, gu, gd


def report(inst, f, z_feasible_tol=1e-8) -> dict:
    out = np.zeros(8)
    args = [_c(inst.row_ptr, np.int64), _c(inst.col, np.int32), _c(inst.u, np.float64),
            _c(inst.s, np.int32), _c(inst.t, np.int32), _c(inst.d, np.float64),
            _c(f, np.float64).reshape(inst.m, inst.K)]
    v = lib().orc_report(inst.n, inst.m, *[_p(a) for a in args[:3]], inst.K,
                         *[_p(a) for a in args[3:]], float(z_feasible_tol), _p(out))
    keys = ["z", "z_psi", "z_h", "kkt_sq", "max_abs_excess", "max_congestion", "farkas_gap",
            "farkas_tol"]
    r = dict(zip(keys, out.tolist()))
    r["verdict"] = VERDICT[int(v)]
    return r
