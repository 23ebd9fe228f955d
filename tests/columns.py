"""Hand-built single columns for the oracle pins (host-side test helpers, numpy only)."""
import math

import numpy as np

RD, G, CP, LV = 287.04, 9.80616, 1004.64, 2.501e6


def pressure_grid(nlev, p_top=300.0, p_s=1.0e5):
    i = np.arange(nlev + 1, dtype=np.float64)
    p_int = p_top * (p_s / p_top) ** (1.0 - (1.0 - i / nlev) ** 2)
    return p_int, 0.5 * (p_int[:-1] + p_int[1:])


def linear_grid(nlev, p_top, p_s):
    p_int = np.linspace(p_top, p_s, nlev + 1)
    return p_int, 0.5 * (p_int[:-1] + p_int[1:])


def heights(T, q, p_int, p_mid):
    """Hydrostatic mid-layer heights above the surface for a given column."""
    nlev = len(T)
    z = np.empty(nlev)
    zi = 0.0
    for k in range(nlev - 1, -1, -1):
        hs = RD * T[k] * (1.0 + 0.608 * q[k]) / G
        z[k] = zi + hs * math.log(p_int[k + 1] / p_mid[k])
        zi = zi + hs * math.log(p_int[k + 1] / p_int[k])
    return z


def column(T, q, p_int, p_mid, z=None, pblh=800.0, tke=1.0, dt=1800.0):
    T = np.asarray(T, float)
    q = np.asarray(q, float)
    if z is None:
        z = heights(T, q, p_int, p_mid)
    return dict(T=T, q=q, p_int=np.asarray(p_int, float), p_mid=np.asarray(p_mid, float),
                z=np.asarray(z, float), phis=0.0, pblh=float(pblh), tke=float(tke), dt=float(dt))


def to_state(cols):
    """Stack single columns into a level-major state dict."""
    st = {k: np.stack([c[k] for c in cols], axis=1) for k in ("T", "q", "p_int", "p_mid", "z")}
    for k in ("phis", "pblh", "tke"):
        st[k] = np.array([c[k] for c in cols], float)
    st["dt"] = cols[0]["dt"]
    st["ncol"], st["nlev"] = len(cols), len(cols[0]["T"])
    return st


def z_interfaces(z):
    """Interface heights of the scheme's grid: surface 0, means of neighbouring mids, top
    extrapolated."""
    L = len(z)
    zi = np.zeros(L + 1)
    for i in range(1, L):
        zi[i] = 0.5 * (z[i - 1] + z[i])
    zi[0] = 2.0 * z[0] - zi[1]
    return zi
