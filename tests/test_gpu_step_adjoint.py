"""The HIP adjoints of the shallow scheme (conv_shallow_backward) and of the whole step
(conv_step_backward: deep, the state update, shallow on the updated state), through the C ABI,
against the oracle's forward-mode derivatives (dual numbers, decisions held fixed; pinned to central
differences of the oracle's forward scheme on the CPU) and against central differences of the HIP
forward itself.

* dot-product identity per column: <g, v> = <cotangents, J v> for random v and cotangents, 1e-9
  of the sum of absolute terms;
* full gradients (all 2L entries) from 2L unit tangents of the oracle, 1e-9 normwise;
* the parameter gradients (eps_sh, delta_sh; for the step also tau, eps_deep) against the oracle's
  tangents along each parameter summed over the columns, 1e-9;
* central differences of the HIP forward on the 55,296-column grid, per column and per scheme,
  columns whose integer outputs change across the step excluded;
* quiet columns get exactly zero (shallow) or pass-through (step) gradients; the autograd Function;
  bit-reproducibility; argument errors.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _B():
    from paper_1711_00289_amd import binding

    return binding


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(x):
    return x.detach().cpu().numpy()


def _cotangents(rng, L, ld):
    return (rng.standard_normal((L, ld)), rng.standard_normal((L, ld)) * 1e3,
            rng.standard_normal(ld) * 1e3)


def _dot(cot, c, j):
    cT, cq, cP = cot
    terms = np.concatenate([cT[:, c] * j["dTdt"], cq[:, c] * j["dqdt"], [cP[c] * j["prec"]]])
    return terms.sum(), np.abs(terms).sum()


@pytest.fixture(scope="module")
def grid1(torch):
    """The 288 x 192 = 55,296-column grid: the shallow scheme alone and the step on the GPU, with
    random cotangents on every output."""
    B = _B()
    st = S.grid_1deg(30)
    n, L = st["ncol"], st["nlev"]
    dev = B.to_device(st)
    conv = B.Conv(n, L)
    rng = np.random.default_rng(41)
    sh = conv.shallow_forward(dev)
    scot = _cotangents(rng, L, n)
    gs = conv.shallow_backward(dev, sh, *(_t(torch, a) for a in scot))
    deep, shs = conv.step(dev)
    dcot2 = _cotangents(rng, L, n)
    scot2 = _cotangents(rng, L, n)
    gstep = conv.step_backward(dev, deep, shs, tuple(_t(torch, a) for a in dcot2),
                               tuple(_t(torch, a) for a in scot2))
    torch.cuda.synchronize()
    return dict(st=st, dev=dev, conv=conv, sh={k: _np(v) for k, v in sh.items()}, scot=scot,
                gs={k: _np(v) for k, v in gs.items()},
                deep={k: _np(v) for k, v in deep.items()},
                shs={k: _np(v) for k, v in shs.items()}, dcot2=dcot2, scot2=scot2,
                gstep={k: _np(v) for k, v in gstep.items()}, deep_t=deep, shs_t=shs)


# ------------------------------------------------------------------ the shallow scheme alone
def test_shallow_dot_product_identity(grid1):
    st, g, scot = grid1["st"], grid1["gs"], grid1["scot"]
    L = st["nlev"]
    status = grid1["sh"]["status"]
    act = np.nonzero(status == 0)[0]
    assert len(act) > 60
    rng = np.random.default_rng(42)
    for c in act:
        col = oracle.column(st, int(c))
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        j = oracle.shallow_column_jvp(col, dT, dq)
        assert j["status"] == 0
        rhs, rscale = _dot(scot, c, j)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), int(c)
    quiet = status != 0
    assert np.all(g["g_T"][:, quiet] == 0.0) and np.all(g["g_q"][:, quiet] == 0.0)


def _oracle_grad(jvp, L, cot, c):
    g = np.zeros(2 * L)
    for i in range(2 * L):
        e = np.zeros(2 * L)
        e[i] = 1.0
        g[i] = sum(_dot(ct, c, j)[0] for ct, j in zip(cot, jvp(e[:L], e[L:])))
    return g[:L], g[L:]


def test_shallow_full_gradient_from_unit_tangents(grid1):
    st, g = grid1["st"], grid1["gs"]
    L = st["nlev"]
    act = np.nonzero(grid1["sh"]["status"] == 0)[0]
    for c in act[:: max(1, len(act) // 8)]:
        col = oracle.column(st, int(c))
        gT, gq = _oracle_grad(lambda a, b: [oracle.shallow_column_jvp(col, a, b)], L,
                              [grid1["scot"]], int(c))
        for got, want in ((g["g_T"][:, c], gT), (g["g_q"][:, c], gq)):
            assert np.abs(got - want).max() <= TOL * np.abs(want).max(), int(c)


def test_shallow_parameter_gradients(grid1):
    st, g, scot = grid1["st"], grid1["gs"], grid1["scot"]
    L = st["nlev"]
    want, scale = np.zeros(2), np.zeros(2)
    for c in np.nonzero(grid1["sh"]["status"] == 0)[0]:
        col = oracle.column(st, int(c))
        for i, (de, dd) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            j = oracle.shallow_column_jvp(col, np.zeros(L), np.zeros(L), de, dd)
            s, a = _dot(scot, int(c), j)
            want[i] += s
            scale[i] += a
    assert scale[0] > 0.0 and scale[1] > 0.0
    assert abs(g["g_eps_sh"] - want[0]) <= TOL * scale[0]
    assert abs(g["g_delta_sh"] - want[1]) <= TOL * scale[1]


# ------------------------------------------------------------------ the whole step
def _step_jvp(col, dT, dq, dpar=(0.0, 0.0, 0.0, 0.0)):
    r = oracle.step_column_jvp(col, dT, dq, dpar)
    return r, [r["deep"], r["shallow"]]


def _sample(grid1, rng):
    """Columns with both schemes active, the deep scheme only, and neither."""
    ds, ss = grid1["deep"]["status"], grid1["shs"]["status"]
    both = np.nonzero((ds == 0) & (ss == 0))[0]
    shallow = np.nonzero((ds != 0) & (ss == 0))[0]
    deep = np.nonzero((ds == 0) & (ss != 0))[0]
    quiet = np.nonzero((ds != 0) & (ss != 0))[0]
    pick = lambda a, k: a if len(a) <= k else np.sort(rng.choice(a, k, replace=False))
    return both, shallow, np.concatenate([pick(both, 48), pick(shallow, 48), pick(deep, 48),
                                          pick(quiet, 16)])


def test_step_dot_product_identity(grid1):
    st, g = grid1["st"], grid1["gstep"]
    L = st["nlev"]
    rng = np.random.default_rng(43)
    both, shallow, cols = _sample(grid1, rng)
    assert len(both) + len(shallow) > 60
    cot = [grid1["dcot2"], grid1["scot2"]]
    for c in cols:
        col = oracle.column(st, int(c))
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        r, js = _step_jvp(col, dT, dq)
        assert r["status"] == (int(grid1["deep"]["status"][c]), int(grid1["shs"]["status"][c]))
        parts = [_dot(ct, int(c), j) for ct, j in zip(cot, js)]
        rhs, rscale = sum(p[0] for p in parts), sum(p[1] for p in parts)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), int(c)


def test_step_full_gradient_from_unit_tangents(grid1):
    st, g = grid1["st"], grid1["gstep"]
    L = st["nlev"]
    rng = np.random.default_rng(44)
    both, shallow, _ = _sample(grid1, rng)
    cot = [grid1["dcot2"], grid1["scot2"]]
    for c in list(both[:4]) + list(shallow[:4]):
        col = oracle.column(st, int(c))
        gT, gq = _oracle_grad(lambda a, b: _step_jvp(col, a, b)[1], L, cot, int(c))
        for got, want in ((g["g_T"][:, c], gT), (g["g_q"][:, c], gq)):
            assert np.abs(got - want).max() <= TOL * np.abs(want).max(), int(c)


def test_step_parameter_gradients(grid1):
    st, g = grid1["st"], grid1["gstep"]
    L = st["nlev"]
    cot = [grid1["dcot2"], grid1["scot2"]]
    active = np.nonzero((grid1["deep"]["status"] == 0) | (grid1["shs"]["status"] == 0))[0]
    want, scale = np.zeros(4), np.zeros(4)
    for c in active:
        col = oracle.column(st, int(c))
        for i in range(4):
            e = np.zeros(4)
            e[i] = 1.0
            _, js = _step_jvp(col, np.zeros(L), np.zeros(L), e)
            for ct, j in zip(cot, js):
                s, a = _dot(ct, int(c), j)
                want[i] += s
                scale[i] += a
    got = [g["g_tau"], g["g_eps"], g["g_eps_sh"], g["g_delta_sh"]]
    for i in range(4):
        assert scale[i] > 0.0
        assert abs(got[i] - want[i]) <= TOL * scale[i], i


@pytest.mark.parametrize("seed", [2, 4])
def test_step_adjoint_under_random_parameters(torch, seed):
    """A seeded draw of the whole parameter set (undilute CAPE: the adjoints refuse a dilute one)
    on 4,000 columns of the 1-degree grid's convecting band: the step's adjoint through the
    dot-product identity on every column where a scheme acts, and the four parameter gradients
    summed over the columns, against the oracle's tangents."""
    from parity import random_params

    B = _B()
    over = random_params(seed)
    assert over["eps_cape"] == 0.0
    st = S.subset(S.grid_1deg(), np.arange(288 * 70, 288 * 70 + 4000))
    n, L = st["ncol"], st["nlev"]
    print(f"step adjoint, seed {seed}, {over}", flush=True)
    dev = B.to_device(st)
    conv = B.Conv(n, L, B.make_params(**over))
    deep, shs = conv.step(dev)
    rng = np.random.default_rng(60 + seed)
    cot = [_cotangents(rng, L, n), _cotangents(rng, L, n)]
    g = conv.step_backward(dev, deep, shs, tuple(_t(torch, a) for a in cot[0]),
                           tuple(_t(torch, a) for a in cot[1]))
    torch.cuda.synchronize()
    g = {k: _np(v) for k, v in g.items()}
    ds, ss = _np(deep["status"]), _np(shs["status"])
    active = np.nonzero((ds == 0) | (ss == 0))[0]
    assert (ds == 0).sum() > 100 and (ss == 0).sum() > 50
    op = oracle.make_params(**over)
    want, scale = np.zeros(4), np.zeros(4)
    for c in active:
        col = oracle.column(st, int(c))
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        r = oracle.step_column_jvp(col, dT, dq, params=op)
        assert r["status"] == (int(ds[c]), int(ss[c])), int(c)
        parts = [_dot(ct, int(c), j) for ct, j in zip(cot, (r["deep"], r["shallow"]))]
        rhs, rscale = sum(p[0] for p in parts), sum(p[1] for p in parts)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), int(c)
        for i in range(4):
            e = np.zeros(4)
            e[i] = 1.0
            rp = oracle.step_column_jvp(col, np.zeros(L), np.zeros(L), e, params=op)
            for ct, j in zip(cot, (rp["deep"], rp["shallow"])):
                s, a = _dot(ct, int(c), j)
                want[i] += s
                scale[i] += a
    got = [g["g_tau"], g["g_eps"], g["g_eps_sh"], g["g_delta_sh"]]
    for i in range(4):
        assert abs(got[i] - want[i]) <= TOL * scale[i], (i, got[i], want[i])


def test_step_quiet_columns_pass_the_shallow_gradient_through(grid1):
    """Where the deep scheme is inactive the update is the identity: the step's gradient is the
    shallow adjoint's at the (unchanged) state; where neither is active it is zero."""
    g = grid1["gstep"]
    ds, ss = grid1["deep"]["status"], grid1["shs"]["status"]
    quiet = (ds != 0) & (ss != 0)
    assert np.all(g["g_T"][:, quiet] == 0.0) and np.all(g["g_q"][:, quiet] == 0.0)


@pytest.mark.parametrize("which", ["deep", "shallow"])
def test_step_against_central_differences_of_the_hip_forward(torch, grid1, which):
    """Per column and per scheme: the loss <cotangent, outputs of one scheme> differenced along a
    random direction in (T, q) restricted to sampled columns, against the adjoint with only that
    scheme's cotangents.  h = 1e-5 with the shallow scheme's curvature filter and bound (the same
    reasoning as the oracle's pin): 2e-6 of the sum of the absolute terms of <g, v>."""
    st, dev, conv = grid1["st"], grid1["dev"], grid1["conv"]
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(45 if which == "deep" else 46)
    both, shallow, cols = _sample(grid1, rng)
    ds = grid1["deep"]["status"]
    cols = np.unique(np.concatenate([both, shallow])) if which == "shallow" else cols[ds[cols] == 0]
    mask = np.zeros(n, dtype=bool)
    mask[cols] = True
    cot = grid1["dcot2"] if which == "deep" else grid1["scot2"]
    cot = tuple(np.where(mask, a, 0.0) for a in cot)
    zero = (None, None, None)
    tc = tuple(_t(torch, a) for a in cot)
    g = conv.step_backward(dev, grid1["deep_t"], grid1["shs_t"], tc if which == "deep" else zero,
                           tc if which == "shallow" else zero)
    gT, gq = _np(g["g_T"]), _np(g["g_q"])
    T0, q0 = _np(dev["T"]), _np(dev["q"])
    vT = np.where(mask, rng.standard_normal((L, n)), 0.0)
    vq = np.where(mask, rng.standard_normal((L, n)) * 1e-3 * q0, 0.0)
    h = 1e-5

    def fwd(sign):
        d = dict(dev)
        d["T"], d["q"] = _t(torch, T0 + sign * h * vT), _t(torch, q0 + sign * h * vq)
        o = conv.step(d)
        torch.cuda.synchronize()
        return [{k: _np(v) for k, v in x.items()} for x in o]

    outs = [fwd(+1.0), [grid1["deep"], grid1["shs"]], fwd(-1.0)]
    blk = 0 if which == "deep" else 1
    cT, cq, cP = cot

    def loss(o):
        o = o[blk]
        return (cT * o["dTdt"]).sum(0) + (cq * o["dqdt"]).sum(0) + cP * o["prec"]

    Lp, L0, Lm = (loss(o) for o in outs)
    keys = (("status", "klaunch", "ktop"), ("status", "kbase", "ktop"))
    ints = [np.stack([o[b][k] for b in (0, 1) for k in keys[b]]) for o in outs]
    same = np.all(ints[0] == ints[1], axis=0) & np.all(ints[2] == ints[1], axis=0)
    an = (gT * vT).sum(0) + (gq * vq).sum(0)
    # Scale: the sum of the absolute terms of <g, v> (a random cotangent can make <g, v> itself
    # small by cancellation, which would inflate a relative error without any real mismatch).
    scale = np.abs(gT * vT).sum(0) + np.abs(gq * vq).sum(0)
    fd = (Lp - Lm) / (2 * h)
    smooth = np.abs((Lp - L0) - (L0 - Lm)) / h <= 1e-3 * scale
    ok = mask & same & smooth & (scale > 0.0)
    assert ok.sum() >= (40 if which == "deep" else 30), ok.sum()
    rel = np.abs(fd - an)[ok] / scale[ok]
    assert rel.max() <= 2e-6, (rel.max(), np.nonzero(ok)[0][np.argmax(rel)])


def test_step_autograd_function_matches_the_abi(torch, grid1):
    B = _B()
    st, dev = grid1["st"], grid1["dev"]
    L, n = st["nlev"], st["ncol"]
    conv = B.Conv(n, L)
    p = conv.params
    p4 = torch.tensor([p.tau, p.eps_deep, p.eps_sh, p.delta_sh], dtype=torch.float64,
                      requires_grad=True)
    T = dev["T"].clone().requires_grad_(True)
    q = dev["q"].clone().requires_grad_(True)
    outs = B.step_conv(conv, dev, T, q, p4)
    cots = [_t(torch, a) for a in (*grid1["dcot2"], *grid1["scot2"])]
    loss = sum((o * c).sum() for o, c in zip(outs, cots))
    loss.backward()
    g = grid1["gstep"]
    assert np.array_equal(_np(T.grad), g["g_T"]) and np.array_equal(_np(q.grad), g["g_q"])
    want = np.array([g["g_tau"], g["g_eps"], g["g_eps_sh"], g["g_delta_sh"]])
    assert np.array_equal(_np(p4.grad), want)


def test_backward_is_bit_reproducible(torch, grid1):
    conv, dev = grid1["conv"], grid1["dev"]
    tc = lambda a: tuple(_t(torch, x) for x in a)
    g1 = conv.step_backward(dev, grid1["deep_t"], grid1["shs_t"], tc(grid1["dcot2"]),
                            tc(grid1["scot2"]))
    g2 = conv.step_backward(dev, grid1["deep_t"], grid1["shs_t"], tc(grid1["dcot2"]),
                            tc(grid1["scot2"]))
    for k in g1:
        assert np.array_equal(_np(g1[k]), _np(g2[k])), k


def test_shallow_cotangents_may_be_omitted(torch, grid1):
    conv, dev = grid1["conv"], grid1["dev"]
    sh = conv.shallow_forward(dev)
    g = conv.shallow_backward(dev, sh)
    assert float(_np(g["g_T"]).__abs__().max()) == 0.0 and float(g["g_eps_sh"]) == 0.0


def test_argument_errors(torch, grid1):
    B = _B()
    L = B.lib()
    conv, dev = grid1["conv"], grid1["dev"]
    st = conv._state(dev)
    sh = B.Conv._shallow_struct(grid1["shs_t"])
    d = B.Conv._deep_struct(grid1["deep_t"])
    cot = B.DeepCot(None, None, None)
    gT = torch.empty(conv.nlev, st.ld, dtype=torch.float64, device="cuda")
    gp = torch.empty(4, dtype=torch.float64, device="cuda")
    g = B.DeepGrad(gT.data_ptr(), gT.data_ptr(), gp.data_ptr())
    nbytes = L.conv_backward_workspace_bytes(conv.ncol, conv.nlev, st.ld)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    wptr = C.c_void_p((ws.data_ptr() + 255) & ~255)
    s0 = B._stream(torch)
    EINVAL = -1
    assert L.conv_shallow_backward(conv.h, C.byref(st), None, C.byref(cot), C.byref(g), wptr,
                                   nbytes, s0) == EINVAL
    assert L.conv_shallow_backward(conv.h, C.byref(st), C.byref(sh), C.byref(cot), C.byref(g),
                                   wptr, 16, s0) == EINVAL
    assert L.conv_step_backward(conv.h, C.byref(st), C.byref(d), C.byref(sh), C.byref(cot),
                                C.byref(cot), C.byref(g), C.c_void_p(wptr.value + 8), nbytes,
                                s0) == EINVAL
    assert L.conv_step_backward(conv.h, C.byref(st), C.byref(d), None, C.byref(cot), C.byref(cot),
                                C.byref(g), wptr, nbytes, s0) == EINVAL
