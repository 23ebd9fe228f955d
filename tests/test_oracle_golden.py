"""The oracle's step reproduces its stored regression fixture (tests/golden/oracle_step_6x30.json,
written by tests/golden/make_oracle_step_fixture.py, which calls only the oracle): integer outputs
exactly, floating-point outputs to 1e-12 relative per column (the host's libm may differ by an
ulp).  A change to the oracle's arithmetic shows up here and must name the passage of the paper,
or the reading of it, that justifies it."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "oracle_step_6x30.json")


def _arr(hexes, shape):
    return np.array([float.fromhex(h) for h in hexes], dtype=np.float64).reshape(shape)


def test_oracle_step_matches_the_stored_fixture():
    fx = json.load(open(FIXTURE))
    n, L = fx["ncol"], fx["nlev"]
    st = {"ncol": n, "nlev": L, "dt": float.fromhex(fx["dt"])}
    for k in ("T", "q", "p_mid", "z"):
        st[k] = _arr(fx["inputs"][k], (L, n))
    st["p_int"] = _arr(fx["inputs"]["p_int"], (L + 1, n))
    for k in ("phis", "pblh", "tke"):
        st[k] = _arr(fx["inputs"][k], (n,))
    d, s = oracle.step(st)
    for got, want in ((d, fx["deep"]), (s, fx["shallow"])):
        assert set(got) == set(want)
        for k, v in want.items():
            g = got[k]
            if g.dtype.kind == "i":
                assert g.ravel().tolist() == v, k
            else:
                w = _arr(v, g.shape)
                err = np.abs(g - w).reshape(-1, n).max(axis=0)
                scale = np.abs(w).reshape(-1, n).max(axis=0)
                assert (err <= 1e-12 * scale + 1e-300).all(), (k, err, scale)
    # the fixture exercises both schemes' plumes and quiet columns
    assert (d["status"] == 0).sum() >= 2 and (s["status"] == 0).sum() >= 2
    assert (d["status"] != 0).any() and (s["status"] != 0).any()
