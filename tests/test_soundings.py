"""The seeded input generator: counter-based draws (published SplitMix64 outputs), independence of
chunking, and the shape/monotonicity the scheme's validity check requires."""
import numpy as np

from paper_1711_00289_amd import soundings as S

GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_reference_outputs():
    # SplitMix64 (Steele, Lea, Flood 2014): state 0 -> 0xE220A8397B1DCDAF; state seeded 1234567
    # -> 6457827717110365317, 3203168211198807973, 9817491932198370423.
    assert int(S.splitmix64(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF
    seq = [int(S.splitmix64(np.array([(1234567 + i * GOLDEN_GAMMA) % 2 ** 64], np.uint64))[0])
           for i in range(3)]
    assert seq == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_uniform_range_and_moments():
    u = S.uniform(5, 1, np.arange(200000))
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    n = S.normal(5, np.arange(200000), 3)
    assert abs(n.mean()) < 0.01 and abs(n.std() - 1) < 0.01


def test_chunks_reproduce_the_full_grid():
    full = S.make_state(1000, 30, seed=9)
    part = S.make_state(300, 30, seed=9, col_offset=500)
    for k in ("T", "q", "z", "pblh", "tke"):
        assert np.array_equal(full[k][..., 500:800], part[k])


def test_padding_copies_and_layout():
    st = S.make_state(100, 30, seed=3, ld=128)
    assert st["T"].shape == (30, 128) and st["p_int"].shape == (31, 128)
    assert np.array_equal(st["T"][:, 100:], np.repeat(st["T"][:, :1], 28, axis=1))


def test_profiles_are_valid_columns():
    st = S.grid_1deg()
    assert (np.diff(st["p_int"], axis=0) > 0).all()
    assert (st["p_int"][:-1] < st["p_mid"]).all() and (st["p_mid"] < st["p_int"][1:]).all()
    assert (np.diff(st["z"], axis=0) < 0).all() and (st["z"][-1] > 0).all()
    assert st["T"].min() > 150 and st["T"].max() < 320 and st["q"].min() > 0
    warm = S.latlon_warm_mask(288, 192)
    assert abs(warm.mean() - 42 / 192) < 1e-12
