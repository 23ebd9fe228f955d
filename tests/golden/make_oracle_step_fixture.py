"""Writes oracle_step_6x30.json: a regression fixture of the CPU oracle's step (deep, state update,
shallow) on six columns of the 288 x 192 synthetic grid, picked from the oracle's own statuses:
deep-active columns (on this grid one also has an active shallow plume on the deep-updated state,
one a shallow plume that dies in its first layer), a shallow-only column and quiet columns.
Inputs and outputs are stored as hexadecimal floats, so the fixture does not depend on the
sounding generator staying unchanged.

The paper prints no physics values for a worked example (its tables are timings), so this fixture
pins the oracle against unintended change, not against the paper; it is written by the oracle
alone.  Run from the repository root: python tests/golden/make_oracle_step_fixture.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1711_00289_amd import soundings as S  # noqa: E402

STATE_2D = ("T", "q", "p_mid", "z", "p_int")
STATE_1D = ("phis", "pblh", "tke")


def pick_columns(st):
    d, s = oracle.step(st)
    deep = np.nonzero(d["status"] == 0)[0]
    shallow = np.nonzero(s["status"] == 0)[0]
    quiet1 = np.nonzero((d["status"] == 1) & (s["status"] != 0))[0]
    other = np.nonzero((d["status"] != 0) & (d["status"] != 1))[0]
    if other.size == 0:
        other = np.nonzero((d["status"] == 1) & (s["status"] == 2))[0]
    return [int(c) for c in (deep[0], deep[deep.size // 2], shallow[0], shallow[-1],
                             quiet1[quiet1.size // 3], other[0])]


def hexes(a):
    return [float(x).hex() for x in np.asarray(a, dtype=np.float64).ravel()]


def main():
    grid = S.grid_1deg(30)
    cols = pick_columns(grid)
    st = S.subset(grid, cols)
    d, s = oracle.step(st)
    out = {
        "what": "oracle.step on six columns of the 288x192 x 30-level synthetic grid (seed 102)",
        "columns_of_grid": cols,
        "ncol": st["ncol"], "nlev": st["nlev"], "dt": float(st["dt"]).hex(),
        "inputs": {k: hexes(st[k]) for k in STATE_2D + STATE_1D},
        "deep": {k: (v.astype(int).ravel().tolist() if v.dtype.kind == "i" else hexes(v))
                 for k, v in d.items()},
        "shallow": {k: (v.astype(int).ravel().tolist() if v.dtype.kind == "i" else hexes(v))
                    for k, v in s.items()},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_step_6x30.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(path, cols)


if __name__ == "__main__":
    main()
