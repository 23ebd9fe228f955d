"""The dilute (entraining) CAPE parcel on the GPU (conv_params_t.eps_cape > 0) against the oracle's
(pinned on the CPU by central differences of CAPE along the unit tendencies and by continuity at
zero entrainment): element-wise parity of the whole step at two entrainment rates on warm
soundings and on the 1-degree grid, the same columns in an ensemble member, and the adjoints'
refusal of a dilute context."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S
from parity import compare_deep, compare_shallow, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _B():
    from paper_1711_00289_amd import binding

    return binding


def _step(st, eps_cape):
    B = _B()
    dev = B.to_device(st)
    conv = B.Conv(st["ncol"], st["nlev"], B.make_params(eps_cape=eps_cape))
    d, s = conv.step(dev)
    return conv, dev, to_np(d), to_np(s)


@pytest.mark.parametrize("eps_cape", [1e-4, 3e-4])
def test_step_parity_on_warm_soundings(torch, eps_cape):
    st = S.small_warm()
    _, _, d, s = _step(st, eps_cape)
    od, osh = oracle.step(st, oracle.make_params(eps_cape=eps_cape))
    compare_deep(d, od, st["ncol"])
    compare_shallow(s, osh, st["ncol"])
    assert (d["status"] == 0).sum() > 50


def test_step_parity_on_the_1deg_grid(torch):
    st = S.grid_1deg()
    _, _, d, s = _step(st, 1e-4)
    od, osh = oracle.step(st, oracle.make_params(eps_cape=1e-4), threads=8, chunk=16)
    compare_deep(d, od, st["ncol"])
    compare_shallow(s, osh, st["ncol"])
    und = oracle.deep(st)
    assert 0 < (d["status"] == 0).sum() < (und["status"] == 0).sum()


def test_dilute_member_in_an_ensemble(torch):
    B = _B()
    a, b = S.small_warm(), S.subset(S.grid_1deg(), np.arange(20000, 21000))
    members = [dict(state=B.to_device(a), nlev=a["nlev"], params=B.make_params(eps_cape=2e-4)),
               dict(state=B.to_device(b), nlev=b["nlev"])]
    ens = B.Ensemble(members)
    ens.step()
    torch.cuda.synchronize()
    for m, st, e in zip(ens.members, (a, b), (2e-4, 0.0)):
        od, osh = oracle.step(st, oracle.make_params(eps_cape=e))
        compare_deep(to_np(m["deep"]), od, st["ncol"])
        compare_shallow(to_np(m["shallow"]), osh, st["ncol"])


def test_adjoints_refuse_a_dilute_context(torch):
    B = _B()
    st = S.subset(S.small_warm(), np.arange(64))
    conv, dev, _, _ = _step(st, 1e-4)
    d, s = conv.step(dev)
    with pytest.raises(RuntimeError, match="conv_deep_backward"):
        conv.deep_backward(dev, d)
    with pytest.raises(RuntimeError, match="conv_step_backward"):
        conv.step_backward(dev, d, s)
