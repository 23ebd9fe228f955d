"""Seeded synthetic atmospheric soundings in the level-major layout of the library.

This module only builds inputs.  It holds none of the convection scheme's arithmetic: the humidity
is set from relative humidity with its own Tetens-form saturation curve and the heights come from a
plain hydrostatic integration, both part of the input recipe, not of the scheme.  The oracle and
the HIP path both consume what it returns.

Recipe (the paper's workloads are CESM/CAM5 FC5 model states at 30 levels and the resolutions of
its Table "Details of Resolutions": R1 13,824, R2 221,184, R3 884,736 columns; those states are not
available, so these soundings stand in for them at the same shapes):

* levels: ``p_int[i] = p_top * (p_s/p_top) ** (1 - (1 - i/L)**2)``, p_top = 300 Pa, p_s = 1e5 Pa,
  ``p_mid`` the mean of the two interfaces (30 layers from 3.7 to 996.8 hPa);
* temperature: ``T_s * (max(p, 200 hPa)/p_s) ** (Rd*0.0065/g)`` (6.5 K/km to a 200 hPa tropopause,
  isothermal above) plus N(0, 0.5 K) noise per level;
* relative humidity linear in p from RH_s at the surface to 0.1 at 300 hPa, 0.1 above;
* warm columns: T_s ~ U(280, 305) K, RH_s ~ U(0.6, 0.95); cold columns: T_s ~ U(250, 285) K,
  RH_s ~ U(0.3, 0.7); on a lat-lon grid the rows with |lat| below the tropical half-width are warm;
* pblh ~ U(300, 1500) m, tke ~ U(0.1, 2) m^2 s^-2, phis = 0.

Random numbers are counter based: every draw is splitmix64 of a key made from (seed, field, column,
level), so a value never depends on draw order, chunking or device.
"""
from __future__ import annotations

import math

import numpy as np

P_TOP = 300.0
P_SURF = 1.0e5
_RD = 287.04
_G = 9.80616

_K_SEED = np.uint64(0x9E3779B97F4A7C15)
_K_FIELD = np.uint64(0xC2B2AE3D27D4EB4F)
_K_COL = np.uint64(0x165667B19E3779F9)
_K_LEV = np.uint64(0xD6E8FEB86659FD93)

F_TS, F_RH, F_PBLH, F_TKE, F_N1, F_N2 = range(6)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function (Steele, Lea, Flood 2014) on a uint64 array."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, field: int, col: np.ndarray, lev: np.ndarray | int = 0) -> np.ndarray:
    """U(0,1) (open interval) draw for each (column, level): 53-bit mantissa of splitmix64."""
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) * _K_SEED + np.uint64(field) * _K_FIELD +
               np.asarray(col, dtype=np.uint64) * _K_COL + np.asarray(lev, dtype=np.uint64) * _K_LEV)
    bits = splitmix64(key) >> np.uint64(11)
    return (bits.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normal(seed: int, col: np.ndarray, lev: np.ndarray) -> np.ndarray:
    """N(0,1) by Box-Muller from two uniforms with distinct field tags."""
    u1 = uniform(seed, F_N1, col, lev)
    u2 = uniform(seed, F_N2, col, lev)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def levels(nlev: int):
    i = np.arange(nlev + 1, dtype=np.float64)
    p_int = P_TOP * (P_SURF / P_TOP) ** (1.0 - (1.0 - i / nlev) ** 2)
    p_mid = 0.5 * (p_int[:-1] + p_int[1:])
    return p_int, p_mid


def _qsat_recipe(T, p):
    # Tetens-form saturation curve of the input recipe (not the scheme's own formula).
    e = 610.78 * np.exp(17.27 * (T - 273.15) / (T - 35.86))
    return 0.622 * e / (p - 0.378 * e)


def make_state(ncol: int, nlev: int = 30, seed: int = 101, warm=None, dt: float = 1800.0,
               ld: int | None = None, col_offset: int = 0) -> dict:
    """Level-major state dict: T, q, p_mid, z [nlev][ld]; p_int [nlev+1][ld]; phis, pblh, tke [ld].

    ``warm``: boolean array [ncol] (True = warm distribution) or None for all warm.
    ``ld`` >= ncol pads the column dimension (padding columns hold a copy of column 0).
    ``col_offset`` shifts the counter so a chunk of a larger grid reproduces its columns exactly.
    """
    ld = ncol if ld is None else ld
    if ld < ncol:
        raise ValueError("ld must be >= ncol")
    cols = np.arange(ncol, dtype=np.uint64) + np.uint64(col_offset)
    warm = np.ones(ncol, bool) if warm is None else np.asarray(warm, bool)
    u_ts = uniform(seed, F_TS, cols)
    u_rh = uniform(seed, F_RH, cols)
    Ts = np.where(warm, 280.0 + 25.0 * u_ts, 250.0 + 35.0 * u_ts)
    RHs = np.where(warm, 0.6 + 0.35 * u_rh, 0.3 + 0.4 * u_rh)
    pblh = 300.0 + 1200.0 * uniform(seed, F_PBLH, cols)
    tke = 0.1 + 1.9 * uniform(seed, F_TKE, cols)

    p_int1, p_mid1 = levels(nlev)
    lev = np.arange(nlev, dtype=np.uint64)[:, None]
    noise = 0.5 * normal(seed, cols[None, :], lev)
    pm = p_mid1[:, None]
    T = Ts[None, :] * (np.maximum(pm, 2.0e4) / P_SURF) ** (_RD * 0.0065 / _G) + noise
    rh = np.where(pm >= 3.0e4, RHs[None, :] + (0.1 - RHs[None, :]) * (P_SURF - pm) / (P_SURF - 3.0e4),
                  0.1)
    q = rh * _qsat_recipe(T, pm)
    tv = T * (1.0 + 0.608 * q)
    z = np.empty((nlev, ncol))
    zi = np.zeros(ncol)
    for k in range(nlev - 1, -1, -1):
        hscale = _RD * tv[k] / _G
        z[k] = zi + hscale * math.log(p_int1[k + 1] / p_mid1[k])
        zi = zi + hscale * math.log(p_int1[k + 1] / p_int1[k])

    def pad2(a):
        out = np.empty((a.shape[0], ld))
        out[:, :ncol] = a
        if ld > ncol:
            out[:, ncol:] = a[:, :1]
        return out

    def pad1(a):
        out = np.empty(ld)
        out[:ncol] = a
        if ld > ncol:
            out[ncol:] = a[0]
        return out

    return dict(
        T=pad2(T), q=pad2(q), p_mid=pad2(np.repeat(pm, ncol, axis=1)), z=pad2(z),
        p_int=pad2(np.repeat(p_int1[:, None], ncol, axis=1)), phis=pad1(np.zeros(ncol)),
        pblh=pad1(pblh), tke=pad1(tke), dt=float(dt), ncol=int(ncol), nlev=int(nlev),
    )


def latlon_warm_mask(nlon: int, nlat: int, halfwidth_deg: float = 20.0) -> np.ndarray:
    """Columns ordered lat-major (col = j*nlon + i); True where |lat_j| < halfwidth."""
    lat = -90.0 + (np.arange(nlat) + 0.5) * 180.0 / nlat
    return np.repeat(np.abs(lat) < halfwidth_deg, nlon)


# Workloads (seeds fixed per workload).
def small_warm(nlev: int = 30) -> dict:
    """256 warm columns x 30 levels: the deep-only case the oracle finishes in well under a second."""
    return make_state(256, nlev, seed=101)


def grid_1deg(nlev: int = 30) -> dict:
    """288 x 192 = 55,296 columns, latitude-clustered convection."""
    return make_state(288 * 192, nlev, seed=102, warm=latlon_warm_mask(288, 192))


def grid_quarter_deg(nlev: int = 30) -> dict:
    """1152 x 768 = 884,736 columns (the paper's R3 column count), latitude-clustered."""
    return make_state(1152 * 768, nlev, seed=103, warm=latlon_warm_mask(1152, 768))


ENSEMBLE_NLEV = (30, 46, 72)
ENSEMBLE_TAU = (1800.0, 3600.0, 7200.0)


def ensemble_member_spec(m: int) -> dict:
    """Member m of the uneven ensemble: 55,296 columns, nlev in {30, 46, 72}, tau in
    {1800, 3600, 7200} s, tropical half-width 20 deg (m < 8) or 30 deg (m >= 8)."""
    return dict(nlev=ENSEMBLE_NLEV[m % 3], tau=ENSEMBLE_TAU[(m // 3) % 3],
                halfwidth=20.0 if m < 8 else 30.0, seed=103 * 1000 + m, ncol=288 * 192)


def ensemble_member(m: int, ncol: int | None = None) -> dict:
    spec = ensemble_member_spec(m)
    n = spec["ncol"] if ncol is None else ncol
    warm = latlon_warm_mask(288, 192, spec["halfwidth"])[:n]
    st = make_state(n, spec["nlev"], seed=spec["seed"], warm=warm)
    st["tau"] = spec["tau"]
    return st


def subset(st: dict, cols) -> dict:
    """A new state holding the given columns (fancy-indexed copy)."""
    cols = np.asarray(cols)
    out = {k: (v[:, cols] if isinstance(v, np.ndarray) and v.ndim == 2 else
               v[cols] if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    out["ncol"] = len(cols)
    return out
