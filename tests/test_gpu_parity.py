"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element on the same
seeded inputs: deep scheme D1-D10, shallow scheme S1-S9 and the full step (deep, state update,
shallow; the paper's Algorithm 1 order), at sizes that span many tiles with ragged tails, at the
full 884,736-column grid on sampled columns, and on the edge cases (one column, padding, invalid
columns, nothing convecting, other level counts, parameter extremes)."""
import os

import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S
from parity import compare_deep, compare_shallow, exact_positive_zero, random_params, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bind():
    from paper_1711_00289_amd import binding

    return binding


def run_gpu(st, mode, params=None, ld=None):
    B = _bind()
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], st["nlev"], params)
    if mode == "deep":
        r = (to_np(c.deep_forward(dev)), None)
    elif mode == "shallow":
        r = (None, to_np(c.shallow_forward(dev)))
    else:
        d, s = c.step(dev)
        r = (to_np(d), to_np(s))
    import torch

    torch.cuda.synchronize()
    return r


def oracle_params(**kw):
    return oracle.make_params(**kw)


def gpu_params(**kw):
    return _bind().make_params(**kw)


def test_small_warm_deep(torch):
    st = S.small_warm()
    d, _ = run_gpu(st, "deep")
    compare_deep(d, oracle.deep(st), st["ncol"])
    assert (d["status"] == 0).sum() > 100


@pytest.mark.parametrize("ncol", [1, 63, 257, 1000])
def test_ragged_sizes_step(torch, ncol):
    st = S.subset(S.grid_1deg(), np.arange(288 * 80, 288 * 80 + ncol))
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st)
    compare_deep(d, od, ncol)
    compare_shallow(s, osh, ncol)


def test_grid_1deg_step_all_columns(torch):
    st = S.grid_1deg()
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st)
    compare_deep(d, od, st["ncol"])
    compare_shallow(s, osh, st["ncol"])
    print("deep active", (d["status"] == 0).mean(), "shallow active", (s["status"] == 0).mean())
    exact_positive_zero(d, ("dTdt", "dqdt", "mu", "md"), np.nonzero(d["status"] != 0)[0])
    exact_positive_zero(s, ("dTdt", "dqdt", "mu"), np.nonzero(s["status"] != 0)[0])


def test_grid_1deg_deep_and_shallow_alone(torch):
    st = S.grid_1deg()
    d, _ = run_gpu(st, "deep")
    compare_deep(d, oracle.deep(st), st["ncol"])
    _, s = run_gpu(st, "shallow")
    compare_shallow(s, oracle.shallow(st), st["ncol"])


def test_quarter_degree_grid_every_column(torch):
    """The 1152 x 768 = 884,736-column grid in one launch, every column against the oracle (its
    OpenMP driver over the host's cores: the same per-column oracle, scheduled in parallel)."""
    st = S.grid_quarter_deg()
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st, threads=min(16, len(os.sched_getaffinity(0))), chunk=16)
    compare_deep(d, od, st["ncol"])
    compare_shallow(s, osh, st["ncol"])
    # properties at every column
    dp = np.diff(st["p_int"], axis=0)
    for o in (d, s):
        a = o["status"] == 0
        e = (1004.64 * o["dTdt"] * dp / 9.80616).sum(0) - 2.501e6 * o["prec"]
        sc = (np.abs(1004.64 * o["dTdt"]) * dp / 9.80616).sum(0) + 2.501e6 * o["prec"] + 1e-300
        assert (np.abs(e[a]) / sc[a]).max() < 1e-12
    assert (d["mu"] >= 0).all() and (d["md"] <= 0).all() and (s["mu"] >= 0).all()


def test_quarter_degree_grid_at_the_benchmarked_launch_shapes(torch):
    """The 884,736-column step at the launch shape the benchmark's autotuner picks, and at the
    extreme shapes it may pick, gives the same bits at every column as the default shape (whose
    sampled columns the previous test checks against the oracle)."""
    B = _bind()
    st = S.grid_quarter_deg()
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], st["nlev"])
    d, s = c.step(dev)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in (d, s)]
    f, sh, _ = c.autotune(dev, d, s, reps=3, force=True)
    shapes = [(f, sh), (1, 1), (4, 4), (32, 32)]
    for shape in shapes:
        c.set_launch(*shape)
        for o in (d, s):
            for v in o.values():
                v.fill_(-7)
        c.step(dev, d, s)
        torch.cuda.synchronize()
        for r, o in zip(ref, (d, s)):
            for k in r:
                assert torch.equal(r[k], o[k]), (shape, k)


def test_padding_ld_greater_than_ncol(torch):
    base = S.make_state(777, 30, seed=31, warm=np.arange(777) % 3 != 0, ld=1024)
    d, s = run_gpu(base, "step")
    od, osh = oracle.step(S.make_state(777, 30, seed=31, warm=np.arange(777) % 3 != 0))
    compare_deep(d, od, 777)
    compare_shallow(s, osh, 777)


def test_invalid_and_quiet_columns(torch):
    st = S.subset(S.small_warm(), np.arange(128))
    st["T"][3, 1] = np.nan
    st["q"][10, 2] = -1e-3
    st["p_mid"][5, 3] = st["p_int"][5, 3]
    st["z"][20, 4] = st["z"][21, 4]
    st["pblh"][5] = np.inf
    st["T"][:, 6] = 250.0 + 0.002 * st["z"][:, 6]
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st)
    compare_deep(d, od, 128)
    compare_shallow(s, osh, 128)
    assert list(d["status"][1:5]) == [3, 3, 3, 3] and list(s["status"][1:6]) == [6] * 5


@pytest.mark.parametrize("nlev", [2, 3, 46, 72, 256])
def test_other_level_counts(torch, nlev):
    """From the fewest levels the context accepts (nothing can trigger) to the most (256)."""
    st = S.make_state(3000, nlev, seed=77, warm=np.arange(3000) < 1500)
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st)
    compare_deep(d, od, 3000)
    compare_shallow(s, osh, 3000)
    if nlev >= 46:
        assert (d["status"] == 0).sum() > 500 and (s["status"] == 0).sum() > 100


@pytest.mark.parametrize("over", [dict(alpha_dd=0.0), dict(eps_deep=0.0), dict(eps_deep=5e-4),
                                  dict(cape_threshold=0.0), dict(tau=600.0),
                                  dict(eps_sh=2e-3, delta_sh=5e-4), dict(qlcrit_sh=0.0),
                                  dict(cin_max=1e9, p_sh_top_min=20000.0),
                                  # the evaporation cap on alpha (D6): every active column, and
                                  # about one in eight (a wavefront's lanes on both branches)
                                  dict(evap_max_frac=0.05), dict(evap_max_frac=0.15)])
def test_parameter_variants(torch, over):
    st = S.subset(S.grid_1deg(), np.arange(288 * 70, 288 * 70 + 4000))
    B = _bind()
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], st["nlev"], B.make_params(**over))
    d, s = c.step(dev)
    d, s = to_np(d), to_np(s)
    od, osh = oracle.step(st, oracle.make_params(**over))
    compare_deep(d, od, st["ncol"], label=f"deep {over}")
    compare_shallow(s, osh, st["ncol"], label=f"shallow {over}")


@pytest.mark.parametrize("seed", range(6))
def test_random_parameter_sets(torch, seed):
    """Six seeded draws of the whole parameter set on 4,000 columns of the convecting band of the
    1-degree grid: the step's outputs element by element against the oracle."""
    over = random_params(seed)
    st = S.subset(S.grid_1deg(), np.arange(288 * 70, 288 * 70 + 4000))
    B = _bind()
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], st["nlev"], B.make_params(**over))
    d, s = c.step(dev)
    d, s = to_np(d), to_np(s)
    od, osh = oracle.step(st, oracle.make_params(**over))
    compare_deep(d, od, st["ncol"], label=f"deep seed {seed}")
    compare_shallow(s, osh, st["ncol"], label=f"shallow seed {seed}")


def test_limiter_binding_long_step(torch):
    st = S.subset(S.small_warm(), np.arange(256))
    st["dt"] = 2.0e5
    d, s = run_gpu(st, "step")
    od, osh = oracle.step(st)
    compare_deep(d, od, 256)
    compare_shallow(s, osh, 256)
    qn = st["q"] + st["dt"] * d["dqdt"]
    assert qn.min() > -1e-15


def test_repeatable_and_permutation_equivariant(torch):
    st = S.subset(S.grid_1deg(), np.arange(288 * 75, 288 * 75 + 5000))
    d1, s1 = run_gpu(st, "step")
    d2, s2 = run_gpu(st, "step")
    for a, b in ((d1, d2), (s1, s2)):
        for f in a:
            assert np.array_equal(a[f], b[f], equal_nan=True), f
    perm = np.random.default_rng(3).permutation(5000)
    dp_, sp_ = run_gpu(S.subset(st, perm), "step")
    for a, b in ((d1, dp_), (s1, sp_)):
        for f in a:
            assert np.array_equal(a[f][..., perm], b[f]), f


def test_invalid_arguments_rejected(torch):
    B = _bind()
    st = S.subset(S.small_warm(), np.arange(64))
    dev = B.to_device(st)
    c = B.Conv(64, 30)
    bad = dict(dev)
    bad["dt"] = 0.0
    with pytest.raises(RuntimeError, match="invalid argument"):
        c.step(bad)
    with pytest.raises(ValueError):
        c.step(dict(dev, T=dev["T"][:, :32].contiguous()))
