"""Pins of the deep closure and of the dilute (entraining) CAPE parcel in the oracle.

What fixes them, independently of the closure code:
* F is defined as minus the derivative of CAPE along the unit tendencies with the launch level,
  top and saturation flags fixed: a central difference of the oracle's own CAPE, recomputed from
  the state moved along (dT1, dq1) = (dTdt, dqdt) / M_b, must give F, for the undilute parcel (the
  default) and for a dilute one, whose F also carries the entrained air's change;
* the dilute parcel is continuous in its entrainment rate and equals the undilute one at 0;
* mixing environmental air (whose moist static energy is below the launch layer's, which is the
  largest of the launch region) into the parcel lowers CAPE on the tropical soundings.
"""
import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S


def _cape_and_ints(col, T, q, p):
    c = dict(col)
    c["T"], c["q"] = T, q
    d = oracle.deep_column(c, p)["diag"]
    return d["cape"], (d["kb"], d["kt"], d["status"])


@pytest.mark.parametrize("eps_cape", [0.0, 1e-4, 3e-4])
def test_closure_is_minus_the_derivative_of_cape(eps_cape):
    st = S.small_warm()
    p = oracle.make_params(eps_cape=eps_cape)
    od = oracle.deep(st, p)
    act = np.nonzero(od["status"] == 0)[0]
    assert len(act) > 20
    checked = 0
    for c in act[:40]:
        col = oracle.column(st, int(c))
        r = oracle.deep_column(col, p)
        d = r["diag"]
        dT1, dq1 = r["dTdt"] / d["Mb"], r["dqdt"] / d["Mb"]
        h = 1e-4 / np.abs(dT1).max()  # moves T by at most 1e-4 K
        c0, i0 = _cape_and_ints(col, col["T"], col["q"], p)
        cp_, ip = _cape_and_ints(col, col["T"] + h * dT1, col["q"] + h * dq1, p)
        cm, im = _cape_and_ints(col, col["T"] - h * dT1, col["q"] - h * dq1, p)
        fd = -(cp_ - cm) / (2 * h)
        if not (ip == i0 == im) or abs((cp_ - c0) - (c0 - cm)) > 1e-3 * abs(cp_ - cm):
            continue  # a saturation flag or an index changes across the step
        assert abs(fd - d["F"]) <= 1e-6 * abs(d["F"]), (int(c), fd, d["F"])
        checked += 1
    assert checked >= 15


def test_dilute_parcel_is_continuous_at_zero_entrainment():
    st = S.small_warm()
    base = oracle.deep(st)
    tiny = oracle.deep(st, oracle.make_params(eps_cape=1e-12))
    zero = oracle.deep(st, oracle.make_params(eps_cape=0.0))
    for k in ("dTdt", "dqdt", "prec", "cape"):
        assert np.array_equal(zero[k], base[k])
    same = tiny["status"] == base["status"]
    assert same.mean() > 0.99
    rel = np.abs(tiny["cape"] - base["cape"])[same] / np.maximum(base["cape"][same], 1.0)
    assert rel.max() < 1e-6


def test_dilution_lowers_cape_on_tropical_soundings():
    st = S.small_warm()
    und = oracle.deep(st)
    dil = oracle.deep(st, oracle.make_params(eps_cape=1e-4))
    both = (und["status"] != 3) & (und["cape"] > 0)
    assert both.sum() > 100
    assert np.median(dil["cape"][both] - und["cape"][both]) < 0.0
    assert (dil["trig"] == 1).sum() < (und["trig"] == 1).sum()
