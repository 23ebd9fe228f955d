"""Pins of the oracle's convective momentum transport: the wind carried by the plumes of the step
as a tracer is, plus the pressure-gradient term of Gregory, Kershaw & Inness (1997), coefficient
cpgf (scheme reading 35; the paper's convection moves heat and water, and its runtime includes
other work around the two loops it optimises, Experiments, Table "All optimizations").

Independent fixes:
* cpgf = 0 is passive tracer transport of each component (bit for bit against the pinned tracer
  transport);
* a uniform wind gets no tendency, and adding a uniform wind changes no tendency (Galilean
  invariance), for any cpgf;
* the column momentum (tendency weighted by dp/g) is conserved;
* closed forms without entrainment: a deep updraft with cpgf = 1 follows the environment's wind
  exactly (u_u at interface i = u of layer i), with cpgf = 0 it keeps the launch layer's wind; a
  downdraft with cpgf = 1 carries the wind of the layer above each interface and so adds no flux;
  a shallow plume without mixing keeps its source offset u_u - u = S - u[k_s] with cpgf = 1 and
  the source mean S with cpgf = 0.  The tendency is then the divergence of those fluxes.
"""
import numpy as np
import pytest

import oracle
from columns import G, z_interfaces
from paper_1711_00289_amd import soundings as S


def _wind(L, n, seed):
    rng = np.random.default_rng(seed)
    # a sheared profile plus noise, different for u and v
    base = np.linspace(20.0, -5.0, L)[:, None]
    return np.stack([base + rng.normal(0.0, 3.0, (L, n)), -0.5 * base + rng.normal(0.0, 3.0, (L, n))])


@pytest.fixture(scope="module")
def grid():
    # the 1-degree grid's tropical rows and some extratropical ones: deep, shallow and quiet columns
    st = S.subset(S.grid_1deg(), np.r_[np.arange(288 * 78, 288 * 84), np.arange(288 * 20, 288 * 21)])
    return st, oracle.step(st)


def test_zero_coefficient_is_passive_tracer_transport(grid):
    st, _ = grid
    w = _wind(30, st["ncol"], 1)
    tm, dm = oracle.momentum(st, w, cpgf=0.0)
    tt, dt = oracle.tracers(st, w)
    assert np.array_equal(tm, tt) and np.array_equal(dm, dt)
    # with the pressure-gradient term the tendencies differ where a plume crosses shear
    t7, _ = oracle.momentum(st, w, cpgf=0.7)
    assert np.abs(t7 - tm).max() > 1e-3 * np.abs(tm).max()


@pytest.mark.parametrize("cpgf", [0.0, 0.7, 1.0])
def test_uniform_wind_invariance_and_conservation(grid, cpgf):
    st, (od, osh) = grid
    L, n = st["T"].shape
    w = _wind(L, n, 2)
    t, d = oracle.momentum(st, w, cpgf=cpgf)
    scale = np.abs(t).max()
    act = (od["status"] == 0) | (osh["status"] == 0)
    assert act.sum() > 100 and scale > 0
    # a uniform wind is not transported
    u0 = np.broadcast_to(np.array([7.0, -3.0])[:, None, None], w.shape)
    t0, _ = oracle.momentum(st, np.ascontiguousarray(u0), cpgf=cpgf)
    assert np.abs(t0).max() <= 1e-12 * scale
    # adding one changes nothing (Galilean invariance)
    t1, _ = oracle.momentum(st, w + u0, cpgf=cpgf)
    assert np.abs(t1 - t).max() <= 1e-10 * scale
    # column momentum is conserved by the deep part and by the whole step
    dp = np.diff(st["p_int"], axis=0)
    for x in (t, d):
        col = (x * dp / G).sum(1)
        mag = (np.abs(x) * dp / G).sum(1) + 1e-300
        assert (np.abs(col) / mag).max() < 1e-12
    # quiet columns get exact zeros
    assert (t[:, :, ~act] == 0).all()


def _deep_closed_form(col, d, u, cpgf):
    """Deep tendency of one component with eps_deep = 0 (eta = 1, |eta_d| = 1)."""
    kb, kt, kd, a, Mb = d["kb"], d["kt"], d["kd"], d["alpha"], d["Mb"]
    L = len(u)
    F = np.zeros(L + 1)
    for i in range(kt + 1, kb + 1):
        cu = u[i] if cpgf == 1.0 else u[kb]                 # updraft wind at interface i
        m = 1.0 - (a if (kd >= 0 and i >= kd + 1) else 0.0)
        up = u[i - 1] if m >= 0.0 else u[i]
        F[i] = cu - up
        if kd >= 0 and i >= kd + 1:
            cd = u[i - 1] if cpgf == 1.0 else u[kd]         # downdraft wind at interface i
            F[i] += -a * (cd - up)
    dp = np.diff(col["p_int"])
    out = np.zeros(L)
    for k in range(kt, kb + 1):
        out[k] = Mb * (F[k + 1] - F[k]) * G / dp[k]
    return out


@pytest.mark.parametrize("cpgf,alpha_dd", [(1.0, 0.0), (0.0, 0.0), (1.0, 0.2), (0.0, 0.2)])
def test_deep_closed_forms_without_entrainment(grid, cpgf, alpha_dd):
    st, _ = grid
    prm = oracle.make_params(eps_deep=0.0, alpha_dd=alpha_dd)
    od, _ = oracle.step(st, prm)
    L, n = st["T"].shape
    w = _wind(L, n, 3)
    _, dm = oracle.momentum(st, w, cpgf=cpgf, params=prm)
    checked = 0
    for c in np.nonzero(od["status"] == 0)[0][:60]:
        col = oracle.column(st, int(c))
        d = oracle.deep_column(col, prm)["diag"]
        for comp in range(2):
            want = _deep_closed_form(col, d, w[comp, :, c], cpgf)
            got = dm[comp, :, c]
            assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), (c, comp)
        checked += 1
    assert checked >= 30
    if alpha_dd > 0:
        # with cpgf = 1 the downdraft adds no flux: the same tendencies as without it
        if cpgf == 1.0:
            prm0 = oracle.make_params(eps_deep=0.0, alpha_dd=0.0)
            _, d0 = oracle.momentum(st, w, cpgf=1.0, params=prm0)
            same = od["status"] == 0
            od0, _ = oracle.step(st, prm0)
            same &= od0["status"] == 0
            # the base mass flux differs (the downdraft changes the closure); compare per unit Mb
            for c in np.nonzero(same)[0][:20]:
                col = oracle.column(st, int(c))
                m1 = oracle.deep_column(col, prm)["diag"]["Mb"]
                m0 = oracle.deep_column(col, prm0)["diag"]["Mb"]
                np.testing.assert_allclose(dm[:, :, c] / m1, d0[:, :, c] / m0, rtol=1e-11,
                                           atol=1e-11 * np.abs(d0[:, :, c] / m0).max())


@pytest.mark.parametrize("cpgf", [1.0, 0.0])
def test_shallow_closed_form_without_mixing(grid, cpgf):
    """Shallow plumes with eps_sh = delta_sh = 0 on columns the deep scheme leaves alone (so the
    shallow scheme sees the input wind)."""
    st, _ = grid
    prm = oracle.make_params(eps_sh=0.0, delta_sh=0.0)
    od, osh = oracle.step(st, prm)
    L, n = st["T"].shape
    w = _wind(L, n, 4)
    t, d = oracle.momentum(st, w, cpgf=cpgf, params=prm)
    sel = np.nonzero((osh["status"] == 0) & (od["status"] != 0))[0]
    assert len(sel) >= 5
    dp = np.diff(st["p_int"], axis=0)
    for c in sel[:30]:
        col = oracle.column(st, int(c))
        sd = oracle.shallow_column(col, prm)["diag"]
        ks, kt, Mb = sd["ks"], sd["kt"], sd["Mb"]
        for comp in range(2):
            u = w[comp, :, c]
            src = (dp[ks:, c] * u[ks:]).sum() / dp[ks:, c].sum()
            F = np.zeros(L + 1)
            for i in range(kt + 1, ks + 1):
                cu = u[i] + (src - u[ks]) if cpgf == 1.0 else src
                F[i] = cu - u[i - 1]
            want = np.zeros(L)
            for k in range(kt, ks + 1):
                want[k] = Mb * (F[k + 1] - F[k]) * G / dp[k, c]
            got = t[comp, :, c] - d[comp, :, c]
            assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), (c, comp)
