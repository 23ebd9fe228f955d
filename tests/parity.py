"""Element-by-element comparison of HIP outputs with the oracle (host-side test helpers).

Bar: integer and index outputs bit-exact; FP64 arrays within 1e-9 normwise per column
(max_k |g - o| <= 1e-9 * max_k |o| + 1e-300); FP64 per-column scalars within 1e-9 relative (same
floor).  Any index mismatch is reported with the column and values so its decision margin can be
inspected."""
import numpy as np

RTOL = 1e-9
FLOOR = 1e-300
# Absolute floors (on top of RTOL) for scalars that are sums of buoyancy terms: each term carries
# the absolute rounding of a difference of two virtual temperatures near 300 K (the saturated
# parcel's root is exact only to its last bit), about 1e-12 J/kg per layer whatever the sum's
# size, so a sum near zero cannot meet a relative bar.  CAPE (D4) gets the floor only where the
# column does not trigger (triggered columns, CAPE above the threshold, keep the pure relative
# bar); CIN (S5) gets it everywhere (its decision is made at cin_max = 100 J/kg, far above).
ABS_FLOOR = {"cape": 1e-9, "cin": 1e-9}
ABS_FLOOR_ONLY_UNTRIGGERED = ("cape",)

DEEP_INT = ("klaunch", "ktop", "trig", "status")
DEEP_ARR = ("dTdt", "dqdt", "mu", "md")
DEEP_SCAL = ("prec", "cape")
SH_INT = ("kbase", "ktop", "status")
SH_ARR = ("dTdt", "dqdt", "mu")
SH_SCAL = ("prec", "cin")


def to_np(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}


def compare(gpu: dict, ora: dict, ints, arrs, scals, ncol, cols=None, label=""):
    """Raise AssertionError with details on the first failing output."""
    idx = np.arange(ncol) if cols is None else np.asarray(cols)
    for f in ints:
        g, o = gpu[f][..., :ncol][..., idx], ora[f]
        bad = np.nonzero(g != o)[0]
        assert bad.size == 0, (f"{label} {f}: {bad.size} mismatches, first cols "
                               f"{idx[bad[:5]].tolist()} gpu={g[bad[:5]].tolist()} "
                               f"oracle={o[bad[:5]].tolist()}")
    for f in arrs:
        g, o = gpu[f][:, :ncol][:, idx], ora[f]
        err = np.abs(g - o).max(axis=0)
        scale = np.abs(o).max(axis=0)
        bad = np.nonzero(~(err <= RTOL * scale + FLOOR))[0]
        assert bad.size == 0, (f"{label} {f}: {bad.size} columns beyond tolerance, first "
                               f"{idx[bad[:5]].tolist()} rel={(err[bad[:5]] / (scale[bad[:5]] + FLOOR)).tolist()}")
    for f in scals:
        g, o = gpu[f][:ncol][idx], ora[f]
        floor = np.full(o.shape, ABS_FLOOR.get(f, FLOOR))
        if f in ABS_FLOOR_ONLY_UNTRIGGERED and "trig" in ora:
            floor[ora["trig"] != 0] = FLOOR
        bad = np.nonzero(~(np.abs(g - o) <= RTOL * np.abs(o) + floor))[0]
        assert bad.size == 0, (f"{label} {f}: {bad.size} mismatches, first cols "
                               f"{idx[bad[:5]].tolist()} gpu={g[bad[:5]].tolist()} "
                               f"oracle={o[bad[:5]].tolist()}")


def compare_deep(gpu, ora, ncol, cols=None, label="deep"):
    compare(gpu, ora, DEEP_INT, DEEP_ARR, DEEP_SCAL, ncol, cols, label)


def compare_shallow(gpu, ora, ncol, cols=None, label="shallow"):
    compare(gpu, ora, SH_INT, SH_ARR, SH_SCAL, ncol, cols, label)


def exact_positive_zero(d: dict, fields, cols):
    for f in fields:
        a = d[f][..., cols]
        assert (a == 0).all() and not np.signbit(a).any(), f


def random_params(seed):
    """Every parameter drawn at once around its default (rates log-uniform, thresholds and
    pressures uniform), odd seeds with a dilute CAPE: combinations that variants of one parameter
    at a time do not reach."""
    rng = np.random.default_rng(seed)
    lu = lambda lo, hi: float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    return dict(cape_threshold=rng.uniform(0.0, 300.0), tau=lu(600.0, 14400.0),
                eps_deep=lu(1e-5, 1e-3), alpha_dd=rng.uniform(0.0, 0.5),
                evap_max_frac=rng.uniform(0.02, 1.0), p_launch_min=rng.uniform(5e4, 8e4),
                p_top_min=rng.uniform(1e3, 2e4), eps_sh=lu(2e-4, 3e-3), delta_sh=lu(2e-4, 3e-3),
                qlcrit_sh=lu(1e-4, 3e-3), cin_max=rng.uniform(10.0, 400.0),
                a_buoy=rng.uniform(0.0, 2.0), b_drag=rng.uniform(0.2, 3.0),
                c_tke=rng.uniform(0.3, 3.0), p_lcl_min=rng.uniform(5e4, 8e4),
                p_sh_top_min=rng.uniform(2e4, 6e4),
                eps_cape=lu(1e-5, 3e-4) if seed % 2 else 0.0)
