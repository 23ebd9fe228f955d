"""The batched ensemble (conv_ensemble_*, through the C ABI): members with different column
counts, level counts (30/46/72) and parameters stepped by the same launches give, column for
column, bit-identical results to conv_step on each member alone, and the oracle's results on
sampled columns, also with a seeded draw of every parameter per member; a captured HIP graph
replays to the same bits with eager work between replays; every persistent-grid shape and the
autotuner's choice give the same bits; the 884,736-column grid plus 16 members of 55,296 columns
runs as one ensemble."""
import os

import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S
from parity import compare_deep, compare_shallow, to_np

pytestmark = pytest.mark.gpu

DEEP_F = ("dTdt", "dqdt", "mu", "md", "prec", "cape", "klaunch", "ktop", "trig", "status")
SHALLOW_F = ("dTdt", "dqdt", "mu", "prec", "cin", "kbase", "ktop", "status")


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _B():
    from paper_1711_00289_amd import binding

    return binding


def small_members():
    """Uneven members: level counts 30/46/72, adjustment times 1800/3600/7200 s, a one-column and
    an empty member, ragged column counts."""
    specs = [(3000, 30, 3600.0, 501), (1, 46, 1800.0, 502), (0, 30, 3600.0, 503),
             (777, 72, 7200.0, 504), (2049, 46, 3600.0, 505), (300, 30, 1800.0, 506)]
    out = []
    for n, L, tau, seed in specs:
        if n == 0:
            st = S.make_state(1, L, seed=seed, warm=np.ones(1, dtype=bool))
            st = S.subset(st, np.arange(0))
        else:
            warm = np.random.default_rng(seed).random(n) < 0.5
            st = S.make_state(n, L, seed=seed, warm=warm)
        out.append((st, L, tau))
    return out


def _members(torch, specs):
    B = _B()
    ms = []
    for st, L, tau in specs:
        dev = B.to_device(st) if st["ncol"] > 0 else _empty_dev(torch, L, st)
        ms.append(dict(state=dev, nlev=L, ncol=st["ncol"], params=B.make_params(tau=tau)))
    return ms


def _empty_dev(torch, L, st):
    z = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
    return dict(T=z(L, 0), q=z(L, 0), p_mid=z(L, 0), z=z(L, 0), p_int=z(L + 1, 0), phis=z(0),
                pblh=z(0), tke=z(0), dt=float(st["dt"]), ncol=0)


def _snapshot(m):
    return ({f: m["deep"][f].clone() for f in DEEP_F}, {f: m["shallow"][f].clone() for f in SHALLOW_F})


def _equal(a, b):
    """Bit-for-bit equality of two dicts of device arrays (float64 compared as int64 bits)."""
    import torch

    for k in a:
        x, y = a[k], b[k]
        assert x.shape == y.shape, k
        if x.dtype == torch.float64:
            x, y = x.view(torch.int64), y.view(torch.int64)
        assert bool((x == y).all()), k


def _separate(torch, m):
    B = _B()
    c = B.Conv(m["ncol"], m["nlev"], m["params"])
    d, s = c.step(m["state"])
    torch.cuda.synchronize()
    return d, s


def test_ensemble_matches_separate_steps_bit_for_bit(torch):
    B = _B()
    ms = _members(torch, small_members())
    ens = B.Ensemble(ms)
    ens.step()
    torch.cuda.synchronize()
    for m in ens.members:
        if m["ncol"] == 0:
            continue
        d, s = _separate(torch, m)
        _equal({f: m["deep"][f] for f in DEEP_F}, {f: d[f] for f in DEEP_F})
        _equal({f: m["shallow"][f] for f in SHALLOW_F}, {f: s[f] for f in SHALLOW_F})
    st0 = ens.members[0]["deep"]["status"]
    assert int((st0 == 0).sum()) > 100


def test_ensemble_matches_oracle_on_sampled_columns(torch):
    B = _B()
    specs = small_members()
    ens = B.Ensemble(_members(torch, specs))
    ens.step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(61)
    for (st, L, tau), m in zip(specs, ens.members):
        n = st["ncol"]
        if n == 0:
            continue
        idx = np.sort(rng.choice(n, min(n, 150), replace=False))
        sub = S.subset(st, idx)
        od, osh = oracle.step(sub, oracle.make_params(tau=tau))
        gd = {k: v[..., idx] for k, v in to_np(m["deep"]).items()}
        gs = {k: v[..., idx] for k, v in to_np(m["shallow"]).items()}
        compare_deep(gd, od, len(idx))
        compare_shallow(gs, osh, len(idx))


def test_members_with_their_own_random_parameter_sets(torch):
    """Each member carries its own seeded draw of all seventeen parameters (dilute CAPE in some,
    undilute in others): every kernel must read each lane's parameters from that lane's member.
    Every column of every member against the oracle under that member's parameters, and bit for
    bit against conv_step on the member alone."""
    from parity import random_params

    B = _B()
    specs = small_members()
    draws = [random_params(20 + i) for i in range(len(specs))]
    ms = []
    for (st, L, _), over in zip(specs, draws):
        dev = B.to_device(st) if st["ncol"] > 0 else _empty_dev(torch, L, st)
        ms.append(dict(state=dev, nlev=L, ncol=st["ncol"], params=B.make_params(**over)))
    ens = B.Ensemble(ms)
    ens.step()
    torch.cuda.synchronize()
    active = 0
    for (st, L, _), over, m in zip(specs, draws, ens.members):
        n = st["ncol"]
        if n == 0:
            continue
        print(f"member {n} x {L}: {over}", flush=True)
        od, osh = oracle.step(st, oracle.make_params(**over))
        gd, gs = to_np(m["deep"]), to_np(m["shallow"])
        compare_deep(gd, od, n, label=f"deep {n} x {L}")
        compare_shallow(gs, osh, n, label=f"shallow {n} x {L}")
        d, s = _separate(torch, m)
        _equal({f: m["deep"][f] for f in DEEP_F}, {f: d[f] for f in DEEP_F})
        _equal({f: m["shallow"][f] for f in SHALLOW_F}, {f: s[f] for f in SHALLOW_F})
        active += int((gd["status"] == 0).sum()) + int((gs["status"] == 0).sum())
    assert active > 500


def test_graph_replays_reproduce_eager_step(torch):
    B = _B()
    ens = B.Ensemble(_members(torch, small_members()))
    ens.step()
    torch.cuda.synchronize()
    ref = [_snapshot(m) for m in ens.members]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ens.capture(side)
    side.synchronize()
    x = torch.randn(512, 512, device="cuda")
    for rep in range(4):
        for m in ens.members:  # eager work between replays: poison every output
            for o in (m["deep"], m["shallow"]):
                for v in o.values():
                    v.fill_(-7)
        y = x @ x
        torch.cuda.synchronize()
        ens.replay(side)
        side.synchronize()
        for r, m in zip(ref, ens.members):
            _equal(r[0], {f: m["deep"][f] for f in DEEP_F})
            _equal(r[1], {f: m["shallow"][f] for f in SHALLOW_F})
        assert float(y.abs().sum()) > 0
    ens.step()  # eager again after replays
    torch.cuda.synchronize()
    for r, m in zip(ref, ens.members):
        _equal(r[0], {f: m["deep"][f] for f in DEEP_F})


def test_every_launch_shape_and_the_autotuner_give_the_same_bits(torch):
    B = _B()
    ens = B.Ensemble(_members(torch, small_members()))
    ens.step()
    torch.cuda.synchronize()
    ref = [_snapshot(m) for m in ens.members]
    for f, s in ((1, 1), (5, 16), (12, 32), (32, 4), (24, 8), (3, 7)):
        ens.set_launch(f, s)
        assert ens.get_launch() == (f, s)
        ens.step()
        torch.cuda.synchronize()
        for r, m in zip(ref, ens.members):
            _equal(r[0], {k: m["deep"][k] for k in DEEP_F})
            _equal(r[1], {k: m["shallow"][k] for k in SHALLOW_F})
    f, s, ms = ens.autotune(reps=3, force=True)
    assert f in (4, 5, 6, 8) and s == 32 and ms > 0
    assert ens.get_launch() == (f, s)
    assert ens.autotune(reps=3) == (f, s, ms)  # cached
    ens.step()
    torch.cuda.synchronize()
    for r, m in zip(ref, ens.members):
        _equal(r[0], {k: m["deep"][k] for k in DEEP_F})
        _equal(r[1], {k: m["shallow"][k] for k in SHALLOW_F})
    with pytest.raises(RuntimeError):
        ens.set_launch(0, 1)
    with pytest.raises(RuntimeError):
        ens.set_launch(33, 4)


def test_single_context_autotune_keeps_results(torch):
    B = _B()
    st = S.subset(S.grid_1deg(30), np.arange(20000))
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], 30)
    d, s = c.step(dev)
    torch.cuda.synchronize()
    ref = ({k: d[k].clone() for k in DEEP_F}, {k: s[k].clone() for k in SHALLOW_F})
    f, sh, ms = c.autotune(dev, d, s, reps=3, force=True)
    assert c.get_launch() == (f, sh) and ms > 0
    c.step(dev, d, s)
    torch.cuda.synchronize()
    _equal(ref[0], {k: d[k] for k in DEEP_F})
    _equal(ref[1], {k: s[k] for k in SHALLOW_F})


def test_replay_without_capture_and_capture_on_null_stream_are_rejected(torch):
    B = _B()
    ens = B.Ensemble(_members(torch, small_members()[:2]))
    side = torch.cuda.Stream()
    with pytest.raises(RuntimeError):
        ens.replay(side)
    import ctypes as C

    assert B.lib().conv_ensemble_capture(ens.h, None) == B.CONV_EINVAL
    ens.capture(side)
    ens.set_launch(2, 2)  # drops the graph
    with pytest.raises(RuntimeError):
        ens.replay(side)


def test_full_ensemble_grid_plus_sixteen_members(torch):
    """884,736 x 30 plus 16 members of 55,296 columns (30/46/72 levels, tau 1800/3600/7200 s):
    bit-identical to separate steps of each member, and every column of every member against the
    oracle (its OpenMP driver over the host's cores)."""
    B = _B()
    specs = [(S.grid_quarter_deg(30), 30, 3600.0)]
    for m in range(16):
        sp = S.ensemble_member_spec(m)
        specs.append((S.ensemble_member(m), sp["nlev"], sp["tau"]))
    ens = B.Ensemble(_members(torch, specs))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ens.capture(side)
    ens.replay(side)
    side.synchronize()
    threads = min(16, len(os.sched_getaffinity(0)))
    for i, ((st, L, tau), m) in enumerate(zip(specs, ens.members)):
        print(f"member {i}: {st['ncol']} columns x {L} levels, tau {tau}", flush=True)
        d, s = _separate(torch, m)
        _equal({f: m["deep"][f] for f in DEEP_F}, {f: d[f] for f in DEEP_F})
        _equal({f: m["shallow"][f] for f in SHALLOW_F}, {f: s[f] for f in SHALLOW_F})
        del d, s
        od, osh = oracle.step(st, oracle.make_params(tau=tau), threads=threads, chunk=16)
        compare_deep(to_np(m["deep"]), od, st["ncol"], label=f"member {i} deep")
        compare_shallow(to_np(m["shallow"]), osh, st["ncol"], label=f"member {i} shallow")
