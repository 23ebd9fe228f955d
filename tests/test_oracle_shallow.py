"""Pins of the oracle's shallow scheme (steps S1-S9 of the scheme reading; the paper's shallow
convection, Background and Algorithm 3: repeated thermodynamic checks that send a column to an exit
that zeroes its outputs).

Independent fixes: every exit status is reached by a constructed or drawn column and zeroes the
outputs exactly; column energy and water budgets close to rounding; with equal entrainment and
detrainment the mass flux is constant; the cloud-base closure has the Gaussian-tail closed form in
TKE and CIN; q stays non-negative after the step; without rain-out nothing precipitates."""
import math

import numpy as np
import pytest

import oracle
from columns import CP, G, LV, RD
from paper_1711_00289_amd import soundings as S


@pytest.fixture(scope="module")
def grid():
    st = S.subset(S.grid_1deg(), np.arange(0, 288 * 192, 7))
    return st, oracle.shallow(st)


def _budgets(st, o):
    dp = np.diff(st["p_int"], axis=0)
    e = (CP * o["dTdt"] * dp / G).sum(0) - LV * o["prec"]
    es = (np.abs(CP * o["dTdt"]) * dp / G).sum(0) + LV * np.abs(o["prec"]) + 1e-300
    w = (o["dqdt"] * dp / G).sum(0) + o["prec"]
    ws = (np.abs(o["dqdt"]) * dp / G).sum(0) + np.abs(o["prec"]) + 1e-300
    return np.abs(e) / es, np.abs(w) / ws


def test_exit_statuses_zero_outputs(grid):
    st, o = grid
    seen = set(np.unique(o["status"]).tolist())
    assert {0, 2, 3, 5} <= seen
    inact = o["status"] != 0
    for f in ("dTdt", "dqdt", "mu"):
        assert (o[f][:, inact] == 0).all() and not np.signbit(o[f][:, inact]).any()
    assert (o["prec"][inact] == 0).all()
    # ktop only where the plume ran; cin only where it was completed
    assert (o["ktop"][~np.isin(o["status"], (0, 5))] == -1).all()
    assert (o["cin"][np.isin(o["status"], (1, 2))] == 0).all()


def test_constructed_exits():
    st = S.subset(S.grid_1deg(), np.arange(288 * 96, 288 * 96 + 288))
    o = oracle.shallow(st)
    c = int(np.nonzero(o["status"] == 0)[0][0])
    col = oracle.column(st, c)
    base = oracle.shallow_column(col)["diag"]
    assert base["status"] == 0
    dry = dict(col, q=col["q"] * 1e-3)                     # no saturation below 600 hPa
    assert oracle.shallow_column(dry)["diag"]["status"] == 1
    calm = dict(col, tke=0.0)                               # no boundary-layer turbulence
    assert oracle.shallow_column(calm)["diag"]["status"] == 4
    drag = oracle.shallow_column(col, oracle.make_params(b_drag=1.0e3))  # plume dies at once
    assert drag["diag"]["status"] == 5 and drag["prec"] == 0.0
    bad = dict(col, T=col["T"].copy())
    bad["T"][4] = np.inf
    assert oracle.shallow_column(bad)["diag"]["status"] == 6
    tight = oracle.shallow_column(col, oracle.make_params(cin_max=0.5 * base["cin"]))
    if base["cin"] > 0:
        assert tight["diag"]["status"] == 3


def test_conservation_and_signs(grid):
    st, o = grid
    act = o["status"] == 0
    assert act.sum() >= 5
    e, w = _budgets(st, o)
    assert e[act].max() < 1e-13 and w[act].max() < 1e-13
    assert (o["mu"] >= 0).all() and (o["prec"] >= 0).all()
    qn = st["q"] + st["dt"] * o["dqdt"]
    assert qn.min() >= -1e-15


def test_source_is_boundary_layer_mean(grid):
    st, o = grid
    for c in np.nonzero(o["status"] == 0)[0][:10]:
        col = oracle.column(st, int(c))
        d = oracle.shallow_column(col)["diag"]
        ks = d["ks"]
        assert col["z"][ks] <= col["pblh"] or ks == len(col["z"]) - 1
        assert ks == 0 or col["z"][ks - 1] > col["pblh"]
        h = CP * col["T"] + G * col["z"] + LV * col["q"]
        assert h[ks:].min() - 1e-9 <= d["hs"] <= h[ks:].max() + 1e-9


def test_equal_entrainment_detrainment_keeps_unit_mass_flux(grid):
    st, o = grid
    for c in np.nonzero(o["status"] == 0)[0][:10]:
        col = oracle.column(st, int(c))
        r = oracle.shallow_column(col)
        d = r["diag"]
        nz = r["mu"] != 0
        assert nz.sum() == d["ks"] - d["kt"]
        np.testing.assert_allclose(r["mu"][nz], d["Mb"], rtol=1e-15, atol=0)


def test_closure_gaussian_tail_in_tke_and_cin(grid):
    st, o = grid
    n = 0
    for c in np.nonzero(o["status"] == 0)[0][:10]:
        col = oracle.column(st, int(c))
        d1 = oracle.shallow_column(col)["diag"]
        col2 = dict(col, tke=2.0 * col["tke"])
        d2 = oracle.shallow_column(col2)["diag"]
        if d2["status"] != 0:
            continue
        a = oracle.DEFAULT_PARAMS["a_buoy"]
        ratio = math.sqrt(2.0) * math.exp(-a * d1["cin"] * (1 / col2["tke"] - 1 / col["tke"]))
        assert abs(d2["Mclos"] / d1["Mclos"] / ratio - 1.0) < 1e-13
        # Without the CIN factor the flux is rho_s * sigma_w / sqrt(2*pi).
        d0 = oracle.shallow_column(col, oracle.make_params(a_buoy=0.0))["diag"]
        ks = d0["ks"]
        tv = col["T"][ks] * (1.0 + (461.5 / RD - 1.0) * col["q"][ks])
        rho = col["p_int"][ks] / (RD * tv)
        assert abs(d0["Mclos"] / (rho * math.sqrt(col["tke"]) / math.sqrt(2 * math.pi)) - 1) < 1e-14
        n += 1
    assert n >= 3


def test_no_rainout_means_no_precipitation(grid):
    st, o = grid
    o2 = oracle.shallow(st, oracle.make_params(qlcrit_sh=1.0))
    act = o2["status"] == 0
    assert act.sum() >= 5 and (o2["prec"] == 0).all()
    e, w = _budgets(st, o2)
    assert e[act].max() < 1e-13 and w[act].max() < 1e-13
