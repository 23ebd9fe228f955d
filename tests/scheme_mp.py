"""Independent high-precision evaluation of the scheme's decisions on single columns (test helper).

Written from the scheme's statement (grid C0, thermodynamics C1, deep steps D1-D6, shallow steps
S1-S7), not from the oracle's source: every quantity is an mpmath number at 50 significant digits,
saturation temperatures are found by plain bisection (no Newton, no initial guess), and sums run
in exact-enough arithmetic that their rounding cannot matter at the tolerances the pins use.  It
shares no code with the oracle or with the HIP library.

Each decision also reports its *margin* (the distance of the deciding quantity from its
threshold), so a pin can skip the rare column whose decision is within rounding of a tie.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50

CP = mp.mpf("1004.64")
RD = mp.mpf("287.04")
RV = mp.mpf("461.5")
LV = mp.mpf("2.501e6")
G = mp.mpf("9.80616")
EPS = RD / RV
CV = 1 / EPS - 1
T_CUT = mp.mpf(40)


def F(x) -> mp.mpf:
    """An input double as an exact mpmath number."""
    return mp.mpf(float(x))


def es(T):
    """Bolton (1980) saturation vapour pressure over liquid, Pa; 0 at or below 40 K."""
    if T <= T_CUT:
        return mp.mpf(0)
    return mp.mpf("611.2") * mp.exp(mp.mpf("17.67") * (T - mp.mpf("273.15")) / (T - mp.mpf("29.65")))


def qs(T, p):
    """Saturation specific humidity; 1 where the vapour pressure reaches the pressure."""
    e = es(T)
    if e >= p:
        return mp.mpf(1)
    return EPS * e / (p - (1 - EPS) * e)


def tsat(H, p):
    """The temperature T with cp*T + Lv*qs(T, p) = H, by bisection on [40 K, H/cp]."""
    hi = H / CP
    if hi <= T_CUT:
        return hi
    lo = T_CUT
    for _ in range(200):
        mid = (lo + hi) / 2
        if CP * mid + LV * qs(mid, p) - H > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo < mp.mpf("1e-45") * hi:
            break
    return (lo + hi) / 2


def tv(T, q):
    return T * (1 + CV * q)


def lift(H, qt, p):
    """A parcel of energy H (= h - g z - phis) and total water qt at pressure p: (T, q_v, sat,
    margin), margin = |qt - qs(T_dry)| relative to qt."""
    Tdry = (H - LV * qt) / CP
    qsd = qs(Tdry, p)
    margin = abs(qt - qsd) / max(qt, mp.mpf("1e-30"))
    if qt <= qsd:
        return Tdry, qt, False, margin
    T = tsat(H, p)
    return T, qs(T, p), True, margin


def grid(col):
    """Interface heights, layer thicknesses (m and Pa) and log-pressure widths (C0)."""
    z = [F(v) for v in col["z"]]
    pi = [F(v) for v in col["p_int"]]
    L = len(z)
    zi = [mp.mpf(0)] * (L + 1)
    for i in range(1, L):
        zi[i] = (z[i - 1] + z[i]) / 2
    zi[0] = 2 * z[0] - zi[1]
    dz = [zi[k] - zi[k + 1] for k in range(L)]
    dp = [pi[k + 1] - pi[k] for k in range(L)]
    lam = [mp.log(pi[k + 1] / pi[k]) for k in range(L)]
    return dict(z=z, pi=pi, zi=zi, dz=dz, dp=dp, lam=lam)


def _mse(col, k):
    return CP * F(col["T"][k]) + G * F(col["z"][k]) + F(col.get("phis", 0.0)) + LV * F(col["q"][k])


def _gap(ordered, scale):
    """Relative gap between the best and the second-best of an ordered list (inf if only one)."""
    if len(ordered) < 2:
        return mp.inf
    return abs(ordered[0] - ordered[1]) / abs(scale)


def deep(col, P):
    """Deep decisions D1-D4 and the downdraft start D6 of one column: kb, klim, kt, CAPE, trig,
    kd, and the smallest relative margin among the buoyancy signs and saturation tests that
    decided them."""
    L = len(col["T"])
    g = grid(col)
    pm = [F(v) for v in col["p_mid"]]
    phis = F(col.get("phis", 0.0))
    h = [_mse(col, k) for k in range(L)]
    cand = [k for k in range(L) if pm[k] >= P["p_launch_min"]]
    r = dict(kb=-1, klim=-1, kt=-1, kd=-1, cape=mp.mpf(0), trig=0, margin=mp.inf)
    if not cand:
        return r
    hmax = max(h[k] for k in cand)
    kb = max(k for k in cand if h[k] == hmax)  # a tie goes to the lower layer
    r["margin"] = _gap(sorted((h[k] for k in cand), reverse=True), hmax)
    klim = min((k for k in range(L) if pm[k] >= P["p_top_min"]), default=-1)
    r.update(kb=kb, klim=klim)
    if klim < 0:
        return r
    qkb = F(col["q"][kb])
    B = {}
    for k in range(klim, kb):
        T, qv, _, m = lift(h[kb] - G * g["z"][k] - phis, qkb, pm[k])
        B[k] = tv(T, qv) - tv(F(col["T"][k]), F(col["q"][k]))
        r["margin"] = min(r["margin"], m, abs(B[k]) / tv(F(col["T"][k]), 0))
    pos = [k for k in range(klim, kb) if B[k] > 0]
    if not pos:
        return r
    kt = min(pos)
    cape = sum(RD * B[k] * g["lam"][k] for k in range(kt, kb))
    r.update(kt=kt, cape=max(cape, mp.mpf(0)), B=B)
    r["trig"] = int(r["cape"] > P["cape_threshold"])
    if r["trig"] and kb - kt >= 2:
        inner = range(kt + 1, kb)
        hmin = min(h[k] for k in inner)
        r["kd"] = min(k for k in inner if h[k] == hmin)  # a tie goes to the upper layer
        r["margin"] = min(r["margin"], _gap(sorted(h[k] for k in inner), hmin))
    return r


def shallow(col, P, loading=True):
    """Shallow decisions S1-S7 of one column: source layer ks and source means, LCL, LFC, CIN,
    the exits 1-5, and the plume top kt from the vertical-velocity equation.  `loading=False`
    drops the condensate term from the density temperature (to show which top it decides)."""
    L = len(col["T"])
    g = grid(col)
    pm = [F(v) for v in col["p_mid"]]
    phis = F(col.get("phis", 0.0))
    pblh = F(col["pblh"])
    T = [F(v) for v in col["T"]]
    q = [F(v) for v in col["q"]]
    h = [_mse(col, k) for k in range(L)]
    r = dict(ks=-1, klcl=-1, klfc=-1, kt=-1, cin=mp.mpf(0), status=-1, margin=mp.inf)
    # S1: the contiguous run of layers from the bottom with z <= pblh (the lowest always in).
    ks = L - 1
    while ks > 0 and g["z"][ks - 1] <= pblh:
        ks -= 1
    r["margin"] = min(abs(g["z"][k] - pblh) / pblh for k in range(L))
    w = sum(g["dp"][k] for k in range(ks, L))
    hs = sum(g["dp"][k] * h[k] for k in range(ks, L)) / w
    qsrc = sum(g["dp"][k] * q[k] for k in range(ks, L)) / w
    r.update(ks=ks, hs=hs, qs=qsrc)
    # S2: the undilute parcel from the source at every layer above it.
    B, sat = {}, {}
    for k in range(ks - 1, -1, -1):
        Tp, qv, s, m = lift(hs - G * g["z"][k] - phis, qsrc, pm[k])
        B[k] = tv(Tp, qv) - tv(T[k], q[k])
        sat[k] = s
        r["margin"] = min(r["margin"], m, abs(B[k]) / tv(T[k], 0))
    # S3: the lifting condensation level: the first saturated layer going up; none, or one above
    # p_lcl_min, ends the scheme (status 1).
    sats = [k for k in sat if sat[k]]
    if not sats or pm[max(sats)] < P["p_lcl_min"]:
        r["status"] = 1
        return r
    klcl = max(sats)
    r["klcl"] = klcl
    # S4: the level of free convection: the first layer at or above the LCL with positive
    # buoyancy, not above p_sh_top_min (status 2 if none).
    lfc = [k for k in range(0, klcl + 1) if B[k] > 0 and pm[k] >= P["p_sh_top_min"]]
    if not lfc:
        r["status"] = 2
        return r
    klfc = max(lfc)
    r["klfc"] = klfc
    # S5: CIN over the layers between the source and the LFC.
    cin = sum(RD * max(-B[k], mp.mpf(0)) * g["lam"][k] for k in range(klfc + 1, ks))
    r["cin"] = cin
    if cin > P["cin_max"]:
        r["status"] = 3
        return r
    sig2 = F(P["c_tke"]) * F(col["tke"])
    if not sig2 > 0:
        r["status"] = 4
        return r
    # S7: the entraining-detraining plume from interface ks with its vertical-velocity equation.
    a, b = F(P["a_buoy"]), F(P["b_drag"])
    eps, dlt, qlc = F(P["eps_sh"]), F(P["delta_sh"]), F(P["qlcrit_sh"])
    Tb, qv, _, _ = lift(hs - G * g["zi"][ks] - phis, qsrc, g["pi"][ks])
    rain = max(qsrc - qv - qlc, mp.mpf(0))
    eta, hu, qtu = mp.mpf(1), hs, qsrc - rain
    w2 = sig2 + 2 * a * cin
    wmargin = mp.inf
    kt = -1
    for k in range(ks - 1, -1, -1):
        E, D = eps * eta * g["dz"][k], dlt * eta * g["dz"][k]
        en = eta + E - D
        if g["pi"][k] < P["p_sh_top_min"] or k == 0 or not en > 0:
            kt = k
            break
        hm = ((eta - D) * hu + E * h[k]) / en
        qm = ((eta - D) * qtu + E * q[k]) / en
        Tu, qv, _, _ = lift(hm - G * g["zi"][k] - phis, qm, g["pi"][k])
        ql = qm - qv
        rain = max(ql - qlc, mp.mpf(0))
        Trho = Tu * (1 + CV * qv - ((ql - rain) if loading else 0))
        Tve = tv(T[k], q[k])
        Bk = G * (Trho - Tve) / Tve
        w2n = w2 + 2 * g["dz"][k] * (a * Bk - b * eps * w2)
        wmargin = min(wmargin, abs(w2n) / w2)
        if not w2n > 0:
            kt = k
            break
        eta, hu, qtu, w2 = en, hm, qm - rain, w2n
    r.update(kt=kt, wmargin=wmargin, status=5 if kt == ks - 1 else 0)
    return r
