"""CPU oracle of the convection scheme -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded FP64 C++ implementation (``conv_oracle.cpp``) of the deep
(Zhang-McFarlane-style) and shallow (UW bulk-plume-style) schemes whose loop skeletons the paper
gives (arXiv:1711.00289, Algorithms 2 and 3), in the written reading's steps C0-C1, D1-D10 and
S1-S9 stated in that source, wrapped with ctypes for numpy arrays.  ``mlp_ref`` is the numpy
reference of the surrogate network.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library and never imports it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py`` against what the
mathematics fixes independently of the code: closed forms (the vapour-pressure constant at 0 C,
Clausius-Clapeyron, the dry-adiabat CAPE that telescopes, isothermal buoyancy, the Gaussian-tail
closure), an independent empirical formula (Goff-Gratch), roots checked by their residuals,
conservation of column energy and water, exit paths that must give exact zeros, and central finite
differences (closure F, forward-mode tangents, the network's gradients).  Fidelity to CAM5's own
ZM/UW code is "parity unpinned": no such code or reference output exists for this work.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "conv_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

PARAM_FIELDS = (
    "cape_threshold", "tau", "eps_deep", "alpha_dd", "evap_max_frac", "p_launch_min", "p_top_min",
    "eps_sh", "delta_sh", "qlcrit_sh", "cin_max", "a_buoy", "b_drag", "c_tke", "p_lcl_min",
    "p_sh_top_min", "eps_cape",
)

# Parameter defaults of the scheme reading (SI units).
DEFAULT_PARAMS = dict(
    cape_threshold=70.0, tau=3600.0, eps_deep=1.0e-4, alpha_dd=0.2, evap_max_frac=0.9,
    p_launch_min=60000.0, p_top_min=4000.0, eps_sh=1.0e-3, delta_sh=1.0e-3, qlcrit_sh=1.0e-3,
    cin_max=100.0, a_buoy=1.0, b_drag=1.0, c_tke=1.0, p_lcl_min=60000.0, p_sh_top_min=40000.0,
    eps_cape=0.0,
)


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in PARAM_FIELDS]


class State(C.Structure):
    _fields_ = [("T", C.c_void_p), ("q", C.c_void_p), ("p_mid", C.c_void_p), ("z", C.c_void_p),
                ("p_int", C.c_void_p), ("phis", C.c_void_p), ("pblh", C.c_void_p),
                ("tke", C.c_void_p), ("ld", C.c_int64), ("dt", C.c_double)]


class DeepOut(C.Structure):
    _fields_ = [("dTdt", C.c_void_p), ("dqdt", C.c_void_p), ("mu", C.c_void_p), ("md", C.c_void_p),
                ("prec", C.c_void_p), ("cape", C.c_void_p), ("klaunch", C.c_void_p),
                ("ktop", C.c_void_p), ("trig", C.c_void_p), ("status", C.c_void_p)]


class ShallowOut(C.Structure):
    _fields_ = [("dTdt", C.c_void_p), ("dqdt", C.c_void_p), ("mu", C.c_void_p),
                ("prec", C.c_void_p), ("cin", C.c_void_p), ("kbase", C.c_void_p),
                ("ktop", C.c_void_p), ("status", C.c_void_p)]


class DeepDiag(C.Structure):
    _fields_ = [("kb", C.c_int32), ("kt", C.c_int32), ("kd", C.c_int32), ("klim", C.c_int32),
                ("status", C.c_int32)] + [(n, C.c_double) for n in
                                          ("cape", "F", "Mc", "Mlim", "Mb", "alpha", "C1", "E1", "P1")]


class ShallowDiag(C.Structure):
    _fields_ = [("ks", C.c_int32), ("klcl", C.c_int32), ("klfc", C.c_int32), ("kt", C.c_int32),
                ("status", C.c_int32)] + [(n, C.c_double) for n in
                                          ("hs", "qs", "cin", "rho_s", "sigw2", "Mclos", "Mlim",
                                           "Mb", "P1")]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (-O2, no FMA contraction, OpenMP for the CPU baseline)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_es.restype = C.c_double
        L.oracle_es.argtypes = [C.c_double]
        L.oracle_qs.restype = C.c_double
        L.oracle_qs.argtypes = [C.c_double, C.c_double]
        L.oracle_dqsdT.restype = C.c_double
        L.oracle_dqsdT.argtypes = [C.c_double, C.c_double]
        L.oracle_tsat.restype = C.c_double
        L.oracle_tsat.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]
        for name in ("oracle_deep", "oracle_shallow"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                         C.c_void_p]
        L.oracle_step.restype = C.c_int
        L.oracle_step.argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                  C.POINTER(DeepOut), C.POINTER(ShallowOut)]
        L.oracle_step_omp.restype = C.c_int
        L.oracle_step_omp.argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                      C.POINTER(DeepOut), C.POINTER(ShallowOut), C.c_int, C.c_int]
        L.oracle_step_ops.restype = C.c_int
        L.oracle_step_ops.argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                      C.c_void_p]
        L.oracle_deep_column.restype = C.c_int
        L.oracle_deep_column.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 +
                                         [C.c_double, C.c_double] + [dp] * 5 +
                                         [C.POINTER(DeepDiag), dp, dp])
        L.oracle_shallow_column.restype = C.c_int
        L.oracle_shallow_column.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 +
                                            [C.c_double] * 4 + [dp] * 4 + [C.POINTER(ShallowDiag)])
        L.oracle_deep_parcel.restype = C.c_int
        L.oracle_deep_parcel.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 + [C.c_double] +
                                         [dp, C.POINTER(C.c_int32), dp, dp])
        L.oracle_deep_column_jvp.restype = C.c_int
        L.oracle_deep_column_jvp.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 +
                                             [C.c_double, C.c_double, dp, dp, C.c_double,
                                              C.c_double, dp, dp, dp])
        L.oracle_tracers.restype = C.c_int
        L.oracle_tracers.argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                     C.c_int, dp, dp, dp]
        L.oracle_momentum.restype = C.c_int
        L.oracle_momentum.argtypes = [C.c_int64, C.c_int, C.POINTER(Params), C.POINTER(State),
                                      dp, C.c_double, dp, dp]
        L.oracle_shallow_column_jvp.restype = C.c_int
        L.oracle_shallow_column_jvp.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 +
                                                [C.c_double] * 4 + [dp, dp, C.c_double,
                                                                    C.c_double, dp, dp, dp])
        L.oracle_step_column_jvp.restype = C.c_int
        L.oracle_step_column_jvp.argtypes = ([C.c_int, C.POINTER(Params)] + [dp] * 5 +
                                             [C.c_double] * 4 + [dp] * 5 +
                                             [C.POINTER(C.c_int32)])
        _lib = L
    return _lib


def make_params(**over) -> Params:
    d = dict(DEFAULT_PARAMS)
    for k, v in over.items():
        if k not in d:
            raise KeyError(k)
        d[k] = float(v)
    return Params(*[d[n] for n in PARAM_FIELDS])


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _state(st: dict, keep: list) -> State:
    arrs = {}
    for k in ("T", "q", "p_mid", "z", "p_int", "phis", "pblh", "tke"):
        a = _c64(st[k])
        keep.append(a)
        arrs[k] = a.ctypes.data
    ld = st["T"].shape[1]
    return State(arrs["T"], arrs["q"], arrs["p_mid"], arrs["z"], arrs["p_int"], arrs["phis"],
                 arrs["pblh"], arrs["tke"], ld, float(st["dt"]))


def _deep_out(L, n, keep):
    o = dict(dTdt=np.zeros((L, n)), dqdt=np.zeros((L, n)), mu=np.zeros((L + 1, n)),
             md=np.zeros((L + 1, n)), prec=np.zeros(n), cape=np.zeros(n),
             klaunch=np.zeros(n, np.int32), ktop=np.zeros(n, np.int32),
             trig=np.zeros(n, np.int32), status=np.zeros(n, np.int32))
    keep.append(o)
    return o, DeepOut(*[o[f].ctypes.data for f, _ in DeepOut._fields_])


def _shallow_out(L, n, keep):
    o = dict(dTdt=np.zeros((L, n)), dqdt=np.zeros((L, n)), mu=np.zeros((L + 1, n)),
             prec=np.zeros(n), cin=np.zeros(n), kbase=np.zeros(n, np.int32),
             ktop=np.zeros(n, np.int32), status=np.zeros(n, np.int32))
    keep.append(o)
    return o, ShallowOut(*[o[f].ctypes.data for f, _ in ShallowOut._fields_])


def _dims(st):
    L, n = st["T"].shape
    return L, n


def deep(st: dict, params: Params | None = None) -> dict:
    """Deep scheme over every column of a level-major state dict (arrays [nlev][ncol])."""
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    o, oc = _deep_out(L, n, keep)
    rc = lib().oracle_deep(n, L, C.byref(params), C.byref(s), C.cast(C.pointer(oc), C.c_void_p))
    if rc != 0:
        raise ValueError("oracle_deep: bad arguments")
    return o


def shallow(st: dict, params: Params | None = None) -> dict:
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    o, oc = _shallow_out(L, n, keep)
    rc = lib().oracle_shallow(n, L, C.byref(params), C.byref(s), C.cast(C.pointer(oc), C.c_void_p))
    if rc != 0:
        raise ValueError("oracle_shallow: bad arguments")
    return o


def step(st: dict, params: Params | None = None, threads: int = 0, chunk: int = 0):
    """Deep -> state update -> shallow (Algorithm 1 order).  threads>0 uses the OpenMP driver
    (dynamic schedule, ``chunk`` columns per grab) for the CPU baseline."""
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    od, odc = _deep_out(L, n, keep)
    os_, osc = _shallow_out(L, n, keep)
    if threads > 0:
        rc = lib().oracle_step_omp(n, L, C.byref(params), C.byref(s), C.byref(odc), C.byref(osc),
                                   max(1, chunk), threads)
    else:
        rc = lib().oracle_step(n, L, C.byref(params), C.byref(s), C.byref(odc), C.byref(osc))
    if rc != 0:
        raise ValueError("oracle_step: bad arguments")
    return od, os_


def step_ops(st: dict, params: Params | None = None):
    """Algorithmic operation count of the step per column (float64 [ncol]): +, -, *, /, sqrt,
    exp and log count 1 each (see oracle_step_ops)."""
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    ops = np.zeros(n)
    if lib().oracle_step_ops(n, L, C.byref(params), C.byref(s), ops.ctypes.data) != 0:
        raise ValueError("oracle_step_ops: bad arguments")
    return ops


def column(st: dict, c: int) -> dict:
    """Column c of a level-major state as contiguous 1-D arrays."""
    return dict(T=_c64(st["T"][:, c]), q=_c64(st["q"][:, c]), p_mid=_c64(st["p_mid"][:, c]),
                p_int=_c64(st["p_int"][:, c]), z=_c64(st["z"][:, c]),
                phis=float(st["phis"][c]), pblh=float(st["pblh"][c]), tke=float(st["tke"][c]),
                dt=float(st["dt"]))


def deep_column(col: dict, params: Params | None = None):
    """One deep column with diagnostics and plume profiles."""
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    out = dict(dTdt=np.zeros(L), dqdt=np.zeros(L), mu=np.zeros(L + 1), md=np.zeros(L + 1),
               eta=np.zeros(L + 1), eta_d=np.zeros(L + 1))
    prec = C.c_double(0.0)
    diag = DeepDiag()
    lib().oracle_deep_column(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi), _ptr(z),
                             col.get("phis", 0.0), col.get("dt", 1800.0), _ptr(out["dTdt"]),
                             _ptr(out["dqdt"]), _ptr(out["mu"]), _ptr(out["md"]), C.byref(prec),
                             C.byref(diag), _ptr(out["eta"]), _ptr(out["eta_d"]))
    out["prec"] = prec.value
    out["diag"] = {f: getattr(diag, f) for f, _ in DeepDiag._fields_}
    return out


def shallow_column(col: dict, params: Params | None = None):
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    out = dict(dTdt=np.zeros(L), dqdt=np.zeros(L), mu=np.zeros(L + 1))
    prec = C.c_double(0.0)
    diag = ShallowDiag()
    lib().oracle_shallow_column(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi), _ptr(z),
                                col.get("phis", 0.0), col["pblh"], col["tke"],
                                col.get("dt", 1800.0), _ptr(out["dTdt"]), _ptr(out["dqdt"]),
                                _ptr(out["mu"]), C.byref(prec), C.byref(diag))
    out["prec"] = prec.value
    out["diag"] = {f: getattr(diag, f) for f, _ in ShallowDiag._fields_}
    return out


def deep_parcel(col: dict, params: Params | None = None):
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    B, Tp, qp = np.zeros(L), np.zeros(L), np.zeros(L)
    sat = np.zeros(L, np.int32)
    lib().oracle_deep_parcel(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi), _ptr(z),
                             col.get("phis", 0.0), _ptr(B),
                             sat.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(Tp), _ptr(qp))
    return dict(B=B, sat=sat.astype(bool), Tp=Tp, qp=qp)


def deep_column_jvp(col: dict, dT, dq, dtau=0.0, deps=0.0, params: Params | None = None):
    """Forward-mode tangent of (dTdt, dqdt, prec) along (dT, dq, dtau, deps), branches fixed."""
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    dT, dq = _c64(dT), _c64(dq)
    tT, tq = np.zeros(L), np.zeros(L)
    tp = C.c_double(0.0)
    st = lib().oracle_deep_column_jvp(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi),
                                      _ptr(z), col.get("phis", 0.0), col.get("dt", 1800.0),
                                      _ptr(dT), _ptr(dq), float(dtau), float(deps), _ptr(tT),
                                      _ptr(tq), C.byref(tp))
    return dict(dTdt=tT, dqdt=tq, prec=tp.value, status=st)


def tracers(st: dict, tr, params: Params | None = None):
    """Convective transport of passive tracers tr [ntr][nlev][ncol] by one step: returns
    (tend, deep_tend), each [ntr][nlev][ncol]; tend = deep + shallow tendency."""
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    tr = np.ascontiguousarray(tr, dtype=np.float64)
    ntr = tr.shape[0]
    tend, deep = np.zeros_like(tr), np.zeros_like(tr)
    rc = lib().oracle_tracers(n, L, C.byref(params), C.byref(s), ntr, _ptr(tr), _ptr(tend),
                              _ptr(deep))
    if rc != 0:
        raise ValueError("oracle_tracers: bad arguments")
    return tend, deep


CPGF_DEFAULT = 0.7  # Gregory, Kershaw & Inness (1997)


def momentum(st: dict, wind, cpgf: float = CPGF_DEFAULT, params: Params | None = None):
    """Convective momentum transport by one step: wind [2][nlev][ncol] (u, v) -> (tend,
    deep_tend), each [2][nlev][ncol] in m s^-2; cpgf is the pressure-gradient coefficient."""
    params = params or make_params()
    L, n = _dims(st)
    keep = []
    s = _state(st, keep)
    wind = np.ascontiguousarray(wind, dtype=np.float64)
    if wind.shape != (2, L, n):
        raise ValueError("wind must be [2][nlev][ncol]")
    tend, deep = np.zeros_like(wind), np.zeros_like(wind)
    rc = lib().oracle_momentum(n, L, C.byref(params), C.byref(s), _ptr(wind), float(cpgf),
                               _ptr(tend), _ptr(deep))
    if rc != 0:
        raise ValueError("oracle_momentum: bad arguments")
    return tend, deep


def shallow_column_jvp(col: dict, dT, dq, deps_sh=0.0, ddelta_sh=0.0,
                       params: Params | None = None):
    """Forward-mode tangent of the shallow scheme's (dTdt, dqdt, prec) along (dT, dq, d eps_sh,
    d delta_sh), every integer decision of the run held fixed."""
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    dT, dq = _c64(dT), _c64(dq)
    tT, tq = np.zeros(L), np.zeros(L)
    tp = C.c_double(0.0)
    st = lib().oracle_shallow_column_jvp(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi),
                                         _ptr(z), col.get("phis", 0.0), col.get("pblh", 800.0),
                                         col.get("tke", 1.0), col.get("dt", 1800.0), _ptr(dT),
                                         _ptr(dq), float(deps_sh), float(ddelta_sh), _ptr(tT),
                                         _ptr(tq), C.byref(tp))
    return dict(dTdt=tT, dqdt=tq, prec=tp.value, status=st)


def step_column_jvp(col: dict, dT, dq, dpar=(0.0, 0.0, 0.0, 0.0), params: Params | None = None):
    """Forward-mode tangent of one column of the step (deep, state update, shallow) along
    (dT, dq) and the parameter tangents dpar = (d tau, d eps_deep, d eps_sh, d delta_sh).
    Returns {"deep": {dTdt, dqdt, prec}, "shallow": {...}, "status": (deep, shallow)}."""
    params = params or make_params()
    L = len(col["T"])
    T, q, pm, pi, z = (_c64(col[k]) for k in ("T", "q", "p_mid", "p_int", "z"))
    dT, dq, dp_ = _c64(dT), _c64(dq), _c64(dpar)
    td, ts = np.zeros(2 * L + 1), np.zeros(2 * L + 1)
    status = np.zeros(2, dtype=np.int32)
    rc = lib().oracle_step_column_jvp(L, C.byref(params), _ptr(T), _ptr(q), _ptr(pm), _ptr(pi),
                                      _ptr(z), col.get("phis", 0.0), col.get("pblh", 800.0),
                                      col.get("tke", 1.0), col.get("dt", 1800.0), _ptr(dT),
                                      _ptr(dq), _ptr(dp_), _ptr(td), _ptr(ts),
                                      status.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != 0:
        raise ValueError("oracle_step_column_jvp: bad arguments")
    split = lambda t: dict(dTdt=t[:L], dqdt=t[L:2 * L], prec=float(t[2 * L]))
    return dict(deep=split(td), shallow=split(ts), status=(int(status[0]), int(status[1])))


def es(T: float) -> float:
    return lib().oracle_es(T)


def qs(T: float, p: float) -> float:
    return lib().oracle_qs(T, p)


def dqsdT(T: float, p: float) -> float:
    return lib().oracle_dqsdT(T, p)


def tsat(H: float, p: float, T_guess: float | None = None):
    it = C.c_int(0)
    g = H / 1004.64 if T_guess is None else T_guess
    T = lib().oracle_tsat(H, p, g, C.byref(it))
    return T, it.value
