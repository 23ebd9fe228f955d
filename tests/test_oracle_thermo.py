"""Pins of the oracle's thermodynamics (scheme step C1: es, qs, dqs/dT, the saturated inversion
tsat that stands in for the paper's iterative `ientropy`, Algorithm 2).

Each check compares with something the oracle does not compute itself: an independent saturation
curve (Goff-Gratch), the mixing-ratio route to specific humidity, the Clausius-Clapeyron slope,
finite differences of the oracle's own qs, and the root property of tsat."""
import math

import numpy as np
import pytest

import oracle

CP, LV, RD, RV = 1004.64, 2.501e6, 287.04, 461.5
EPS = RD / RV


def goff_gratch_hpa(T):
    """Saturation vapour pressure over liquid water (Goff-Gratch 1946, WMO form), hPa."""
    Ts = 373.15
    lg = (-7.90298 * (Ts / T - 1.0) + 5.02808 * math.log10(Ts / T)
          - 1.3816e-7 * (10.0 ** (11.344 * (1.0 - T / Ts)) - 1.0)
          + 8.1328e-3 * (10.0 ** (-3.49149 * (Ts / T - 1.0)) - 1.0) + math.log10(1013.25))
    return 10.0 ** lg


def test_es_at_melting_point_is_the_formula_constant():
    # Bolton's curve passes through 6.112 hPa at 0 C exactly (exp(0) = 1).
    assert oracle.es(273.15) == 611.2


@pytest.mark.parametrize("Tc", [-30.0, -20.0, -10.0, 0.0, 10.0, 20.0, 30.0, 35.0])
def test_es_matches_goff_gratch(Tc):
    # Bolton's fit stays within about 0.35 % of the Goff-Gratch curve over -30..35 C; allow 0.4 %.
    # A wrong constant (e.g. 35.86 instead of 29.65 in the denominator) is off by about 3 %.
    T = 273.15 + Tc
    ref = 100.0 * goff_gratch_hpa(T)
    assert abs(oracle.es(T) / ref - 1.0) < 4e-3


@pytest.mark.parametrize("T", [250.0, 273.15, 300.0])
def test_es_follows_clausius_clapeyron(T):
    h = 1e-3
    slope = (math.log(oracle.es(T + h)) - math.log(oracle.es(T - h))) / (2 * h)
    assert abs(slope / (LV / (RV * T * T)) - 1.0) < 0.05


def test_es_cut_below_minimum_temperature():
    assert oracle.es(40.0) == 0.0 and oracle.es(35.0) == 0.0
    assert oracle.es(40.5) > 0.0


@pytest.mark.parametrize("T,p", [(300.0, 1.0e5), (280.0, 8.0e4), (250.0, 5.0e4), (220.0, 2.0e4),
                                 (200.0, 4.0e3), (310.0, 3.0e4)])
def test_qs_equals_mixing_ratio_route(T, p):
    # Specific humidity from the saturation mixing ratio r = eps*e/(p - e), q = r/(1 + r).
    e = oracle.es(T)
    r = EPS * e / (p - e)
    assert abs(oracle.qs(T, p) - r / (1.0 + r)) <= 4e-16 * (r / (1.0 + r))


def test_qs_capped_where_vapour_pressure_reaches_pressure():
    p = 3000.0  # es reaches 30 hPa near 297 K
    assert oracle.qs(305.0, p) == 1.0
    assert oracle.qs(290.0, p) < 1.0


@pytest.mark.parametrize("T,p", [(300.0, 1.0e5), (280.0, 8.0e4), (250.0, 5.0e4), (220.0, 2.0e4),
                                 (190.0, 1.0e4)])
def test_dqsdT_matches_central_difference_of_qs(T, p):
    h = 1e-6 * T
    fd = (oracle.qs(T + h, p) - oracle.qs(T - h, p)) / (2 * h)
    assert abs(oracle.dqsdT(T, p) / fd - 1.0) < 1e-7


CASES = [(3.40e5, 9.5e4), (3.30e5, 8.0e4), (3.10e5, 6.0e4), (2.90e5, 4.0e4), (2.60e5, 2.0e4),
         (2.30e5, 1.0e4), (1.40e5, 4.0e3), (3.60e5, 1.0e5), (3.00e5, 3.0e3)]


@pytest.mark.parametrize("H,p", CASES)
def test_tsat_is_the_root_of_G(H, p):
    T, it = oracle.tsat(H, p)
    G = lambda x: CP * x + LV * oracle.qs(x, p) - H  # noqa: E731
    assert abs(G(T)) <= 1e-14 * H
    d = 1e-12 * T
    assert G(T - d) < 0.0 < G(T + d)
    assert 0 < it < 60


@pytest.mark.parametrize("H,p", CASES)
def test_tsat_independent_of_initial_guess(H, p):
    T0, _ = oracle.tsat(H, p)
    for g in (45.0, 150.0, 200.0, 250.0, 280.0, 300.0, H / CP):
        T, _ = oracle.tsat(H, p, g)
        assert abs(T - T0) <= 4e-15 * T0


def test_tsat_dry_limit_and_cold_cut():
    # At very low temperature qs underflows and the root is H/cp; below the es cut it is H/cp.
    for H in (30.0 * CP, 45.0 * CP, 60.0 * CP):
        T, _ = oracle.tsat(H, 5.0e4)
        assert abs(T - H / CP) <= 1e-15 * H / CP


def test_tsat_moist_adiabat_relation():
    # Along the root, cp*dT + Lv*dqs = dH: the slope dT/dH equals 1/(cp + Lv*qs'(T)).
    p, H, h = 7.0e4, 3.3e5, 1.0
    Tp, _ = oracle.tsat(H + h, p)
    Tm, _ = oracle.tsat(H - h, p)
    T0, _ = oracle.tsat(H, p)
    assert abs((Tp - Tm) / (2 * h) * (CP + LV * oracle.dqsdT(T0, p)) - 1.0) < 1e-6
