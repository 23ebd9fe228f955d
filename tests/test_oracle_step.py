"""Pins of the oracle's step: deep scheme, then the state update, then the shallow scheme on the
updated state (the paper's Algorithm 1 calls deep_convection before shallow_convection in every
chunk of every time step)."""
import numpy as np

import oracle
from columns import CP, G, LV
from paper_1711_00289_amd import soundings as S


def test_step_is_deep_then_shallow_on_updated_state():
    st = S.subset(S.grid_1deg(), np.arange(288 * 80, 288 * 80 + 1500))
    od, osh = oracle.step(st)
    od2 = oracle.deep(st)
    for f in od:
        assert np.array_equal(od[f], od2[f])
    st2 = dict(st, T=st["T"] + st["dt"] * od["dTdt"], q=st["q"] + st["dt"] * od["dqdt"])
    # The standalone shallow call re-validates its input; clip rounding-level negative humidity
    # (where the deep limiter binds) so the comparison is about the scheme, not the check.
    st2["q"] = np.where(np.abs(st2["q"]) < 1e-15, np.abs(st2["q"]), st2["q"])
    os2 = oracle.shallow(st2)
    for f in osh:
        assert np.array_equal(osh[f], os2[f])


def test_step_does_not_revalidate_updated_state():
    # With no downdraft the deep limiter often drives q' to zero within rounding; the shallow
    # scheme of the step still treats the (valid) input column as valid.
    st = S.subset(S.grid_1deg(), np.arange(288 * 70, 288 * 70 + 4000))
    od, osh = oracle.step(st, oracle.make_params(alpha_dd=0.0))
    assert not (osh["status"][od["status"] != 3] == 6).any()


def test_openmp_driver_matches_serial():
    st = S.subset(S.grid_1deg(), np.arange(288 * 80, 288 * 80 + 800))
    a = oracle.step(st)
    b = oracle.step(st, threads=4, chunk=3)
    for x, y in zip(a, b):
        for f in x:
            assert np.array_equal(x[f], y[f])


def test_total_budget_closes():
    st = S.subset(S.grid_1deg(), np.arange(288 * 80, 288 * 80 + 1500))
    od, osh = oracle.step(st)
    dp = np.diff(st["p_int"], axis=0)
    for o in (od, osh):
        act = o["status"] == 0
        e = (CP * o["dTdt"] * dp / G).sum(0) - LV * o["prec"]
        s = (np.abs(CP * o["dTdt"]) * dp / G).sum(0) + LV * o["prec"] + 1e-300
        assert (np.abs(e[act]) / s[act]).max() < 1e-13
