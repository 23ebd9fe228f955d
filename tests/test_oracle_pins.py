"""Independent pins of the oracle's level decisions, downdraft, CIN and shallow plume top.

Budgets of energy and water close for any downdraft evaporation, any downdraft start and any CIN,
so they cannot catch a mistake there.  These checks fix those parts from outside the oracle:

* brute force on tiny columns (4-6 levels): the launch layer kb and cloud top kt (D1-D3), the
  downdraft start k_d (D6), the source layer, LCL, LFC and plume top (S1-S4, S7), each recomputed
  by enumerating the candidates of its definition in 50-digit arithmetic (``scheme_mp``), with CAPE
  and CIN (D4, S5) compared to 1e-12;
* exact ties, built bit for bit in double precision: the launch layer goes to the lower layer, the
  downdraft start to the upper one;
* the downdraft without entrainment (eps_deep = 0): |eta_d| stays 1, so the evaporation telescopes
  to E1 = q_d[kb] - q[k_d], with q_d[kb] the saturation humidity of the unmixed downdraft air
  brought to the base (a root found here by 50-digit bisection); the updraft's condensation
  telescopes to C1 = q[kb] - q_u[kt+1]; then alpha (both branches of the evaporation cap) and
  P1 = C1 - alpha*E1, so P1 = (1 - beta)*C1 whenever the cap binds;
* the CIN test is strict: status 3 appears exactly when cin_max drops below the reported CIN;
* without buoyancy forcing (a_buoy = 0) the vertical-velocity equation is a pure decay
  w2[k] = w2[k+1]*(1 - 2*b_drag*eps_sh*dz_k), whose first non-positive factor fixes the plume top
  and the status-5 boundary in closed form;
* a plume whose top is decided by the condensate term of the density temperature: the top with
  that term differs from the top without it, and the oracle's is the one with it.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import scheme_mp as X
from columns import CP, G, LV, column, heights, linear_grid, pressure_grid, z_interfaces
from paper_1711_00289_amd import soundings as S

TOL = 1e-12
MARGIN = 1e-9  # decisions closer than this (relative) to a tie are not compared


def _params(**over):
    d = dict(oracle.DEFAULT_PARAMS)
    d.update(over)
    return d


def _tiny_columns(n, seed):
    """Random tiny columns on a linear pressure grid (tall or shallow): warm or cool surface, lapse
    rate between moist and dry adiabatic, per-level temperature noise and relative humidity."""
    rng = np.random.default_rng(seed)
    cols = []
    for _ in range(n):
        L = int(rng.integers(4, 7))
        # tall columns (tops at 100-300 hPa) and shallow ones (tops at 800-900 hPa, thin layers)
        tall = rng.uniform() < 0.5
        top = rng.uniform(1.0e4, 3.0e4) if tall else rng.uniform(8.0e4, 9.0e4)
        p_int, p_mid = linear_grid(L, float(top), 1.0e5)
        Ts = rng.uniform(280.0, 308.0)
        gam = rng.uniform(4.0e-3, 9.0e-3) if tall else rng.uniform(7.0e-3, 1.1e-2)
        z0 = heights(np.full(L, Ts - 20.0), np.zeros(L), p_int, p_mid)
        T = Ts - gam * z0 + rng.normal(0.0, 2.0, L)
        rh = rng.uniform(0.3, 1.05, L) * (rng.uniform(0.1, 1.0) if tall else rng.uniform(0.5, 1.0))
        q = np.array([min(r * float(X.qs(X.F(t), X.F(p))), 0.05) for r, t, p in zip(rh, T, p_mid)])
        z = heights(T, q, p_int, p_mid)
        cols.append(column(T, q, p_int, p_mid, z=z, pblh=float(rng.uniform(100.0, 3000.0) if tall else rng.uniform(50.0, 700.0)),
                           tke=float(rng.uniform(0.1, 2.0) if tall else rng.uniform(1.0, 40.0))))
    return cols


# Thresholds scaled to columns of 4-6 layers so that every decision has several candidates.
TINY = dict(p_launch_min=5.0e4, p_top_min=5.0e3, p_lcl_min=4.0e4, p_sh_top_min=2.5e4,
            cape_threshold=10.0, cin_max=30.0, b_drag=0.1)


@pytest.fixture(scope="module")
def tiny():
    cols = _tiny_columns(240, seed=11)
    P = _params(**TINY)
    prm = oracle.make_params(**TINY)
    out = []
    for c in cols:
        out.append((c, oracle.deep_column(c, prm)["diag"], oracle.shallow_column(c, prm)["diag"],
                    X.deep(c, P), X.shallow(c, P)))
    return out


def test_deep_levels_brute_force_on_tiny_columns(tiny):
    compared, skipped, kinds = 0, 0, set()
    for c, d, _, m, _ in tiny:
        if m["margin"] < MARGIN:
            skipped += 1
            continue
        assert (d["kb"], d["klim"]) == (m["kb"], m["klim"])
        assert d["kt"] == m["kt"]
        if m["kt"] >= 0:
            scale = sum(abs(X.RD * m["B"][k] * X.grid(c)["lam"][k]) for k in range(m["kt"], m["kb"]))
            assert abs(d["cape"] - float(m["cape"])) <= TOL * float(scale)
        trig = int(d["status"] in (0, 2))
        assert trig == m["trig"]
        if trig:
            assert d["kd"] == m["kd"]
            kinds.add("kd" if m["kd"] >= 0 else "no_kd")
        kinds.add(("trig", trig))
        kinds.add(("kt", m["kt"] >= 0))
        compared += 1
    assert skipped <= 0.05 * len(tiny)
    assert {("trig", 0), ("trig", 1), ("kt", True), ("kt", False), "kd", "no_kd"} <= kinds


def test_shallow_levels_brute_force_on_tiny_columns(tiny):
    statuses = set()
    skipped = 0
    for c, _, d, _, m in tiny:
        if m["margin"] < MARGIN or m.get("wmargin", mp.inf) < MARGIN:
            skipped += 1
            continue
        assert d["ks"] == m["ks"]
        assert abs(d["hs"] - float(m["hs"])) <= TOL * abs(float(m["hs"]))
        assert abs(d["qs"] - float(m["qs"])) <= TOL * abs(float(m["qs"]))
        assert d["status"] == m["status"], (d, m)
        if m["status"] >= 2 or m["status"] == 0:
            assert d["klcl"] == m["klcl"]
        if m["status"] in (0, 3, 4, 5):
            assert d["klfc"] == m["klfc"]
            assert abs(d["cin"] - float(m["cin"])) <= TOL * max(float(m["cin"]), 1e-3)
        if m["status"] in (0, 5):
            assert d["kt"] == m["kt"]
        statuses.add(m["status"])
    assert skipped <= 0.05 * len(tiny)
    assert {0, 1, 2, 3, 5} <= statuses, statuses


def _tie_value(make_h, target):
    """A double x with make_h(x) == target exactly, searched among neighbours of the linear
    solution; None if no neighbour hits it."""
    x0 = make_h(None)
    for k in range(0, 64):
        for s in (1.0, -1.0):
            x = x0
            for _ in range(k):
                x = np.nextafter(x, s * np.inf)
            if make_h(x) == target:
                return x
    return None


def _h(T, z, q, phis=0.0):
    s = CP * T + G * z + phis
    return s + LV * q


def test_launch_layer_exact_tie_goes_to_the_lower_layer():
    p_int, p_mid = linear_grid(6, 2.0e4, 1.0e5)
    z = heights(np.full(6, 280.0), np.zeros(6), p_int, p_mid)
    T = 300.0 - 0.0098 * z
    q = np.zeros(6)
    T[4] += 2.0  # layers 4 and 5 above every other layer of the launch region
    target = _h(T[4], z[4], q[4])
    t5 = _tie_value(lambda x: (target - G * z[5]) / CP if x is None else _h(x, z[5], q[5]), target)
    assert t5 is not None
    T[5] = t5
    col = column(T, q, p_int, p_mid, z=z)
    assert _h(T[4], z[4], q[4]) == _h(T[5], z[5], q[5])
    d = oracle.deep_column(col, oracle.make_params(p_launch_min=5.0e4))["diag"]
    assert d["kb"] == 5
    # Break the tie by one unit in the last place either way: the larger h wins.
    for dlt, kb in ((np.inf, 5), (-np.inf, 4)):
        c2 = dict(col, T=col["T"].copy())
        c2["T"][5] = np.nextafter(np.nextafter(t5, dlt), dlt)
        assert oracle.deep_column(c2, oracle.make_params(p_launch_min=5.0e4))["diag"]["kb"] == kb


@pytest.fixture(scope="module")
def warm_active():
    st = S.small_warm()
    o = oracle.deep(st)
    return st, np.nonzero(o["status"] == 0)[0]


def test_downdraft_start_exact_tie_goes_to_the_upper_layer(warm_active):
    st, act = warm_active
    done = 0
    for c in act:
        col = oracle.column(st, int(c))
        d = oracle.deep_column(col)["diag"]
        kb, kt = d["kb"], d["kt"]
        if kb - kt < 4:
            continue
        i, j = kt + 1, kt + 3  # make layers i (upper) and j tie below every other cloud layer
        T = col["T"].copy()
        h = _h(T, col["z"], col["q"])
        target = float(np.min(h[kt + 1:kb])) - 50.0
        ti = _tie_value(lambda x: (target - LV * col["q"][i] - G * col["z"][i]) / CP if x is None
                        else _h(x, col["z"][i], col["q"][i]), target)
        tj = _tie_value(lambda x: (target - LV * col["q"][j] - G * col["z"][j]) / CP if x is None
                        else _h(x, col["z"][j], col["q"][j]), target)
        if ti is None or tj is None:
            continue
        T[i], T[j] = ti, tj
        c2 = dict(col, T=T)
        d2 = oracle.deep_column(c2)["diag"]
        if (d2["kb"], d2["kt"], d2["status"]) != (kb, kt, 0):
            continue  # the colder layers moved the cloud top or the trigger: not this pin
        hh = _h(T, col["z"], col["q"])
        assert hh[i] == hh[j] == hh[kt + 1:kb].min()
        assert d2["kd"] == i
        # Lower the lower layer by one ulp of its temperature: it becomes the start.
        c3 = dict(c2, T=T.copy())
        c3["T"][j] = np.nextafter(np.nextafter(tj, -np.inf), -np.inf)
        assert oracle.deep_column(c3)["diag"]["kd"] == j
        done += 1
        if done >= 5:
            break
    assert done >= 3


def _downdraft_closed_form(col, d, P):
    """C1, E1 of a column run with eps_deep = 0, from their telescoped forms."""
    kb, kt, kd = d["kb"], d["kt"], d["kd"]
    zi = [X.F(v) for v in z_interfaces(col["z"])]
    h = [X._mse(col, k) for k in range(len(col["T"]))]
    # Updraft: eta = 1, no mixing, so the condensation sums to q[kb] minus the vapour the undilute
    # updraft air holds at the highest interface it reaches (kt + 1).
    _, qv_top, _, _ = X.lift(h[kb] - X.G * zi[kt + 1], X.F(col["q"][kb]), X.F(col["p_int"][kt + 1]))
    C1 = X.F(col["q"][kb]) - qv_top
    # Downdraft: |eta_d| = 1, h_d = h[kd] all the way, saturated: at the base it holds
    # qs(T*, p_int[kb]) with cp T* + Lv qs(T*, p_int[kb]) = h[kd] - g z_int[kb].
    pb = X.F(col["p_int"][kb])
    Tstar = X.tsat(h[kd] - X.G * zi[kb], pb)
    E1 = X.qs(Tstar, pb) - X.F(col["q"][kd])
    return float(C1), float(E1)


@pytest.mark.parametrize("beta", [0.9, 0.05])
def test_downdraft_evaporation_and_precipitation_telescope_without_entrainment(warm_active, beta):
    st, act = warm_active
    prm = oracle.make_params(eps_deep=0.0, evap_max_frac=beta)
    branches = set()
    n = 0
    for c in act[:60]:
        col = oracle.column(st, int(c))
        r = oracle.deep_column(col, prm)
        d = r["diag"]
        if d["status"] != 0 or d["kd"] < 0:
            continue
        C1, E1 = _downdraft_closed_form(col, d, None)
        assert abs(d["C1"] - C1) <= TOL * abs(C1)
        assert abs(d["E1"] - E1) <= TOL * max(abs(E1), abs(C1))
        capped = 0.2 * E1 > beta * C1
        alpha = beta * C1 / E1 if capped else 0.2
        assert abs(d["alpha"] - alpha) <= TOL * alpha
        P1 = (1.0 - beta) * C1 if capped else C1 - 0.2 * E1
        assert abs(d["P1"] - P1) <= TOL * abs(C1)
        assert abs(r["prec"] - d["Mb"] * P1) <= 1e-11 * abs(d["Mb"] * C1)
        # The downdraft mass flux is alpha times the base flux at every interface it crosses.
        kd, kb = d["kd"], d["kb"]
        np.testing.assert_allclose(r["md"][kd + 1:kb + 1], -d["Mb"] * alpha, rtol=1e-12, atol=0)
        assert (r["md"][:kd + 1] == 0).all() and (r["md"][kb + 1:] == 0).all()
        branches.add(capped)
        n += 1
    assert n >= 10
    assert branches == ({False} if beta == 0.9 else {True})


@pytest.fixture(scope="module")
def shallow_active():
    st = S.subset(S.grid_1deg(), np.arange(0, 288 * 192, 5))
    o = oracle.shallow(st)
    return st, np.nonzero(o["status"] == 0)[0]


def test_cin_brute_force_and_strict_threshold(shallow_active):
    st, act = shallow_active
    P = _params()
    flipped = 0
    for c in act[:40]:
        col = oracle.column(st, int(c))
        d = oracle.shallow_column(col)["diag"]
        m = X.shallow(col, P)
        if m["margin"] < MARGIN:
            continue
        assert (d["ks"], d["klcl"], d["klfc"]) == (m["ks"], m["klcl"], m["klfc"])
        assert abs(d["cin"] - float(m["cin"])) <= TOL * max(float(m["cin"]), 1e-3)
        if d["cin"] > 0.0:
            at = oracle.shallow_column(col, oracle.make_params(cin_max=d["cin"]))["diag"]
            below = oracle.shallow_column(
                col, oracle.make_params(cin_max=float(np.nextafter(d["cin"], 0.0))))["diag"]
            assert at["status"] == 0 and below["status"] == 3
            assert below["cin"] == d["cin"]
            flipped += 1
    assert flipped >= 5


def _closed_form_top(col, ks, P):
    """Plume top with a_buoy = 0 and eps_sh = delta_sh: w2 only decays, so the plume stops at the
    first layer whose factor 1 - 2*b*eps*dz is not positive (or at p_sh_top_min / the model top).
    Returns (kt, smallest relative distance of a factor from zero)."""
    zi = z_interfaces(col["z"])
    dz = zi[:-1] - zi[1:]
    dist = math.inf
    for k in range(ks - 1, -1, -1):
        if col["p_int"][k] < P["p_sh_top_min"] or k == 0:
            return k, dist
        f = 1.0 - 2.0 * P["b_drag"] * P["eps_sh"] * dz[k]
        dist = min(dist, abs(f))
        if f <= 0.0:
            return k, dist
    return -1, dist


def test_plume_top_closed_form_without_buoyancy(shallow_active):
    st, act = shallow_active
    seen_tops, status5 = set(), 0
    for c in act[:30]:
        col = oracle.column(st, int(c))
        ks = oracle.shallow_column(col)["diag"]["ks"]
        zi = z_interfaces(col["z"])
        dz = zi[:-1] - zi[1:]
        # b_drag values putting the first non-positive factor at each layer above the source,
        # just past (1 + 1e-6) and just short of (1 - 1e-6) the closed-form boundary.
        for k in range(ks - 1, max(ks - 6, 0), -1):
            for f in (1.0 + 1e-6, 1.0 - 1e-6):
                b = f / (2.0 * 1e-3 * dz[k])
                P = _params(a_buoy=0.0, b_drag=b)
                kt, dist = _closed_form_top(col, ks, P)
                if dist < 1e-9:
                    continue
                d = oracle.shallow_column(col, oracle.make_params(a_buoy=0.0, b_drag=b))["diag"]
                assert d["status"] in (0, 5)
                assert d["kt"] == kt, (c, k, f, d["kt"], kt)
                assert (d["status"] == 5) == (kt == ks - 1)
                seen_tops.add(ks - kt)
                status5 += d["status"] == 5
    assert status5 > 0 and len(seen_tops) >= 4


def test_plume_tops_match_brute_force(shallow_active):
    st, act = shallow_active
    P = _params(qlcrit_sh=5.0e-3)
    prm = oracle.make_params(qlcrit_sh=5.0e-3)
    agree = 0
    for c in act[:60]:
        col = oracle.column(st, int(c))
        d = oracle.shallow_column(col, prm)["diag"]
        m = X.shallow(col, P)
        if m["margin"] < MARGIN or m.get("wmargin", mp.inf) < MARGIN or m["status"] not in (0, 5):
            continue
        assert d["kt"] == m["kt"] and d["status"] == m["status"]
        agree += 1
    assert agree >= 10


@pytest.mark.parametrize("tke,kt_loaded,kt_unloaded", [(20.0, 26, 24), (40.0, 25, 24)])
def test_condensate_loading_decides_a_plume_top(tke, kt_loaded, kt_unloaded):
    # A moist, steeply lapsed sounding whose saturated plume carries up to 10 g/kg of liquid
    # (q_lcrit = 1e-2): the density temperature's condensate term is what stops it.  At the
    # smaller boundary-layer turbulence the loaded plume dies in its first layer (status 5) while
    # an unloaded one would rise two layers.
    L = 30
    p_int, p_mid = pressure_grid(L)
    z0 = heights(np.full(L, 270.0), np.zeros(L), p_int, p_mid)
    T = np.maximum(303.0 - 0.0095 * z0, 200.0)
    rh = np.clip(0.97 - (1.0e5 - p_mid) / 7.0e4 * 0.5, 0.1, 1.0)
    q = np.array([r * float(X.qs(X.F(t), X.F(p))) for r, t, p in zip(rh, T, p_mid)])
    col = column(T, q, p_int, p_mid, z=heights(T, q, p_int, p_mid), pblh=500.0, tke=tke)
    P = _params(qlcrit_sh=1.0e-2)
    m, m0 = X.shallow(col, P), X.shallow(col, P, loading=False)
    assert m["margin"] > MARGIN and m["wmargin"] > MARGIN and m0["wmargin"] > MARGIN
    assert (m["kt"], m0["kt"]) == (kt_loaded, kt_unloaded)
    d = oracle.shallow_column(col, oracle.make_params(qlcrit_sh=1.0e-2))["diag"]
    assert d["kt"] == kt_loaded and d["ks"] == m["ks"]
    assert d["status"] == (5 if kt_loaded == d["ks"] - 1 else 0)
