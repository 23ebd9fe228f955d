"""Pins of the oracle's convective tracer transport (passive tracers carried by the deep and shallow
plumes of one step, in flux form with the schemes' own mixing and upwind rules).

What fixes it, independently of the transport code:
* moist static energy h = cp T + g z + phis + Lv q is mixed by both plumes exactly like a passive
  tracer and its flux divergence is the schemes' energy tendency (the precipitation terms of the
  temperature and humidity tendencies cancel in h), so the tracer C = h must give
  cp dTdt + Lv dqdt of each scheme as the oracle's step computes them, to rounding;
* a uniform tracer has zero tendency (every plume and environment value equals it);
* the flux form conserves the column burden: sum_k tend_k dp_k = 0;
* the transport is linear in the tracer, and quiet columns get exact zeros.
"""
import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S

CP, LV, GRAV = 1004.64, 2.501e6, 9.80616


@pytest.fixture(scope="module")
def cols():
    """Columns of the 1-degree grid where both schemes act, only the deep one acts, and neither."""
    st = S.grid_1deg()
    od, osh = oracle.step(st, threads=8, chunk=16)
    rng = np.random.default_rng(3)
    deep = np.nonzero(od["status"] == 0)[0]
    shallow = np.nonzero(osh["status"] == 0)[0]
    quiet = np.nonzero((od["status"] != 0) & (osh["status"] != 0))[0]
    pick = np.unique(np.concatenate([shallow, rng.choice(deep, 600, replace=False),
                                     rng.choice(quiet, 200, replace=False)]))
    sub = S.subset(st, pick)
    od, osh = oracle.step(sub)
    return sub, od, osh


def _h(st):
    return CP * st["T"] + GRAV * st["z"] + st["phis"][None, :] + LV * st["q"]


def test_moist_static_energy_tracer_gives_the_energy_tendencies(cols):
    st, od, osh = cols
    tend, deep = oracle.tracers(st, _h(st)[None])
    want_d = CP * od["dTdt"] + LV * od["dqdt"]
    want_s = CP * osh["dTdt"] + LV * osh["dqdt"]
    act_d, act_s = od["status"] == 0, osh["status"] == 0
    assert act_d.sum() > 500 and act_s.sum() > 100
    scale_d = np.abs(want_d).max(axis=0)
    scale_s = np.abs(want_s).max(axis=0)
    assert np.all(np.abs(deep[0] - want_d).max(axis=0) <= 1e-9 * np.maximum(scale_d, 1e-300))
    shallow = tend[0] - deep[0]
    err = np.abs(shallow - want_s).max(axis=0)
    assert np.all(err[act_s] <= 1e-9 * scale_s[act_s] + 1e-12 * scale_d[act_s])
    assert np.all(shallow[:, ~act_s] == 0.0)


def test_uniform_tracer_has_no_tendency(cols):
    st, _, _ = cols
    L, n = st["T"].shape
    rng = np.random.default_rng(4)
    ref, _ = oracle.tracers(st, rng.standard_normal((1, L, n)))
    tend, _ = oracle.tracers(st, np.full((1, L, n), 3.7))
    assert np.abs(tend).max() <= 1e-12 * np.abs(ref).max()


def test_column_burden_is_conserved(cols):
    st, _, _ = cols
    L, n = st["T"].shape
    rng = np.random.default_rng(5)
    tr = np.exp(rng.standard_normal((2, L, n)))
    tend, deep = oracle.tracers(st, tr)
    dp = np.diff(st["p_int"], axis=0)
    for t in (tend, deep):
        burden = (t * dp[None]).sum(axis=1)
        scale = np.abs(t * dp[None]).sum(axis=1)
        assert np.all(np.abs(burden) <= 1e-12 * np.maximum(scale, 1e-300))


def test_transport_is_linear_and_quiet_columns_are_zero(cols):
    st, od, osh = cols
    L, n = st["T"].shape
    rng = np.random.default_rng(6)
    a, b = rng.standard_normal((L, n)), rng.standard_normal((L, n))
    t, _ = oracle.tracers(st, np.stack([a, b, 2.0 * a - 3.0 * b]))
    assert np.allclose(t[2], 2.0 * t[0] - 3.0 * t[1], rtol=0.0, atol=1e-12 * np.abs(t[2]).max())
    quiet = (od["status"] != 0) & (osh["status"] != 0)
    assert quiet.sum() > 100 and np.all(t[:, :, quiet] == 0.0)
