"""The HIP adjoint of the deep scheme (conv_deep_backward, through the C ABI) against the oracle's
forward-mode derivative (dual numbers, branches held fixed; pinned to central differences on the
CPU) and against central finite differences of the HIP forward itself.

* dot-product identity per column: <g, v> = <cotangent, J v> for random v and cotangents, 1e-9;
* full gradients (all 2L entries) from 2L unit tangents of the oracle, 1e-9 normwise per column;
* dL/dtau and dL/deps_deep against the oracle's tangents along tau and eps, 1e-9;
* the 55,296-column x 30-level workload with the loss sum(a*dTdt^2 + b*(Lv/cp*dqdt)^2), a, b ~
  N(0,1): 64 sampled active columns (none within 1 J/kg of the trigger threshold) against the
  oracle (1e-9) and against central differences of the HIP forward with a 1e-6 relative step
  (1e-6), columns whose branches change across the step excluded;
* the torch.autograd.Function, bit-reproducibility, inactive and padded columns, edge sizes and
  argument errors.
"""
import numpy as np
import pytest

import oracle
from paper_1711_00289_amd import soundings as S
from parity import to_np

pytestmark = pytest.mark.gpu

LV_CP = 2.501e6 / 1004.64
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


def _run(torch, st, cT, cq, cP, params=None):
    B = _B()
    dev = B.to_device(st)
    c = B.Conv(st["ncol"], st["nlev"], params)
    out = c.deep_forward(dev)
    g = c.deep_backward(dev, out, None if cT is None else _t(torch, cT),
                        None if cq is None else _t(torch, cq), None if cP is None else _t(torch, cP))
    torch.cuda.synchronize()
    return c, dev, out, {k: _np(v) for k, v in g.items()}


def _cot_dot(cT, cq, cP, c, j):
    terms = np.concatenate([cT[:, c] * j["dTdt"], cq[:, c] * j["dqdt"], [cP[c] * j["prec"]]])
    return terms.sum(), np.abs(terms).sum()


def _oracle_grad(st, c, cT, cq, cP, params=None):
    """Full gradient of <cot, outputs> for one column from 2L unit tangents of the oracle."""
    col = oracle.column(st, c)
    L = len(col["T"])
    g = np.zeros(2 * L)
    for i in range(2 * L):
        e = np.zeros(2 * L)
        e[i] = 1.0
        j = oracle.deep_column_jvp(col, e[:L], e[L:], params=params)
        g[i] = _cot_dot(cT, cq, cP, c, j)[0]
    return g[:L], g[L:]


def _cotangents(rng, L, ld):
    return (rng.standard_normal((L, ld)), rng.standard_normal((L, ld)) * 1e3,
            rng.standard_normal(ld) * 1e3)


def test_dot_product_identity_per_column(torch):
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(21)
    cT, cq, cP = _cotangents(rng, L, n)
    _, _, out, g = _run(torch, st, cT, cq, cP)
    status = _np(out["status"])
    act = np.nonzero(status == 0)[0]
    assert len(act) > 100
    for c in act:
        col = oracle.column(st, int(c))
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        j = oracle.deep_column_jvp(col, dT, dq)
        assert j["status"] == 0
        rhs, rscale = _cot_dot(cT, cq, cP, c, j)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), int(c)
    quiet = status != 0
    assert np.all(g["g_T"][:, quiet] == 0.0) and np.all(g["g_q"][:, quiet] == 0.0)


@pytest.mark.parametrize("kw,branch", [(dict(tau=20.0), "limited"),
                                       (dict(evap_max_frac=0.05), "capped")])
def test_dot_product_identity_on_the_other_branches(torch, kw, branch):
    """Every active column with the humidity limiter setting the base flux (D9), or with the
    downdraft strength capped by the evaporation limit (D6): the state gradient through those
    branches, per column."""
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(26)
    cT, cq, cP = _cotangents(rng, L, n)
    op = oracle.make_params(**kw)
    _, _, out, g = _run(torch, st, cT, cq, cP, _B().make_params(**kw))
    act = np.nonzero(_np(out["status"]) == 0)[0]
    assert len(act) > 100
    hit = 0
    for c in act:
        col = oracle.column(st, int(c))
        d = oracle.deep_column(col, op)["diag"]
        hit += int(d["Mb"] < d["Mc"] if branch == "limited" else d["alpha"] < op.alpha_dd)
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        j = oracle.deep_column_jvp(col, dT, dq, params=op)
        rhs, rscale = _cot_dot(cT, cq, cP, c, j)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), int(c)
    assert hit > len(act) // 2


def test_full_gradient_from_unit_tangents(torch):
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(22)
    cT, cq, cP = _cotangents(rng, L, n)
    _, _, out, g = _run(torch, st, cT, cq, cP)
    act = np.nonzero(_np(out["status"]) == 0)[0]
    for c in act[:: max(1, len(act) // 10)]:
        gT, gq = _oracle_grad(st, int(c), cT, cq, cP)
        for got, want in ((g["g_T"][:, c], gT), (g["g_q"][:, c], gq)):
            assert np.abs(got - want).max() <= TOL * np.abs(want).max(), int(c)


@pytest.mark.parametrize("only", ["dTdt", "dqdt", "prec"])
def test_each_cotangent_alone(torch, only):
    st = S.subset(S.small_warm(), np.arange(64))
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(23)
    cT, cq, cP = _cotangents(rng, L, n)
    z = dict(dTdt=(cT, np.zeros_like(cq), np.zeros_like(cP)),
             dqdt=(np.zeros_like(cT), cq, np.zeros_like(cP)),
             prec=(np.zeros_like(cT), np.zeros_like(cq), cP))[only]
    args = dict(dTdt=(cT, None, None), dqdt=(None, cq, None), prec=(None, None, cP))[only]
    _, _, out, g = _run(torch, st, *args)
    act = np.nonzero(_np(out["status"]) == 0)[0]
    assert len(act) > 10
    for c in act[:6]:
        gT, gq = _oracle_grad(st, int(c), *z)
        assert np.abs(g["g_T"][:, c] - gT).max() <= TOL * np.abs(gT).max()
        assert np.abs(g["g_q"][:, c] - gq).max() <= TOL * np.abs(gq).max()


@pytest.mark.parametrize("kw", [dict(), dict(tau=20.0), dict(alpha_dd=1.0),
                                dict(eps_deep=5e-4, alpha_dd=0.5), dict(evap_max_frac=0.05)])
def test_parameter_gradients(torch, kw):
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(24)
    cT, cq, cP = _cotangents(rng, L, n)
    _, _, out, g = _run(torch, st, cT, cq, cP, _B().make_params(**kw))
    op = oracle.make_params(**kw)
    act = np.nonzero(_np(out["status"]) == 0)[0]
    want = np.zeros(2)
    scale = np.zeros(2)
    for c in act:
        col = oracle.column(st, int(c))
        for i, (dtau, deps) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            j = oracle.deep_column_jvp(col, np.zeros(L), np.zeros(L), dtau, deps, params=op)
            s, a = _cot_dot(cT, cq, cP, c, j)
            want[i] += s
            scale[i] += a
    assert abs(g["g_tau"] - want[0]) <= TOL * scale[0]
    assert abs(g["g_eps"] - want[1]) <= TOL * scale[1]
    # and the state gradients under these parameters
    for c in act[:3]:
        gT, gq = _oracle_grad(st, int(c), cT, cq, cP, params=op)
        assert np.abs(g["g_T"][:, c] - gT).max() <= TOL * np.abs(gT).max()
        assert np.abs(g["g_q"][:, c] - gq).max() <= TOL * np.abs(gq).max()


@pytest.mark.parametrize("seed", range(3))
def test_random_deep_parameter_sets(torch, seed):
    """Seeded draws of all the deep scheme's parameters at once: the state gradient of every
    active column through the per-column dot-product identity, and dL/dtau, dL/deps summed over
    the columns, against the oracle's tangents."""
    prng = np.random.default_rng(700 + seed)
    lu = lambda lo, hi: float(np.exp(prng.uniform(np.log(lo), np.log(hi))))
    kw = dict(cape_threshold=prng.uniform(0.0, 300.0), tau=lu(300.0, 14400.0),
              eps_deep=lu(1e-5, 1e-3), alpha_dd=prng.uniform(0.0, 1.0),
              evap_max_frac=prng.uniform(0.02, 1.0), p_launch_min=prng.uniform(5e4, 8e4),
              p_top_min=prng.uniform(1e3, 2e4))
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(30 + seed)
    cT, cq, cP = _cotangents(rng, L, n)
    op = oracle.make_params(**kw)
    _, _, out, g = _run(torch, st, cT, cq, cP, _B().make_params(**kw))
    act = np.nonzero(_np(out["status"]) == 0)[0]
    assert len(act) > 10, kw
    want = np.zeros(2)
    scale = np.zeros(2)
    for c in act:
        col = oracle.column(st, int(c))
        dT = rng.standard_normal(L)
        dq = rng.standard_normal(L) * 1e-3 * col["q"]
        j = oracle.deep_column_jvp(col, dT, dq, params=op)
        rhs, rscale = _cot_dot(cT, cq, cP, c, j)
        lterms = np.concatenate([g["g_T"][:, c] * dT, g["g_q"][:, c] * dq])
        assert abs(lterms.sum() - rhs) <= TOL * max(rscale, np.abs(lterms).sum()), (int(c), kw)
        for i, (dtau, deps) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            jp = oracle.deep_column_jvp(col, np.zeros(L), np.zeros(L), dtau, deps, params=op)
            s, a = _cot_dot(cT, cq, cP, c, jp)
            want[i] += s
            scale[i] += a
    assert abs(g["g_tau"] - want[0]) <= TOL * scale[0], kw
    assert abs(g["g_eps"] - want[1]) <= TOL * scale[1], kw


@pytest.fixture(scope="module")
def grid(torch):
    """The 288 x 192 = 55,296-column x 30-level workload with the squared-tendency loss."""
    B = _B()
    st = S.grid_1deg(30)
    n, L = st["ncol"], st["nlev"]
    rng = np.random.default_rng(25)
    a = rng.standard_normal((L, n))
    b = rng.standard_normal((L, n))
    dev = B.to_device(st)
    c = B.Conv(n, L)
    out = c.deep_forward(dev)
    dT, dq = _np(out["dTdt"]), _np(out["dqdt"])
    cT = 2.0 * a * dT
    cq = 2.0 * b * LV_CP ** 2 * dq
    g = c.deep_backward(dev, out, _t(torch, cT), _t(torch, cq), None)
    g = {k: _np(v) for k, v in g.items()}
    status, cape = _np(out["status"]), _np(out["cape"])
    cand = np.nonzero((status == 0) & (np.abs(cape - 70.0) > 1.0))[0]
    sample = np.sort(rng.choice(cand, 64, replace=False))
    return dict(st=st, dev=dev, conv=c, out=out, a=a, b=b, cT=cT, cq=cq, g=g, sample=sample)


def _loss_cols(out, a, b, cols):
    dT, dq = _np(out["dTdt"])[:, cols], _np(out["dqdt"])[:, cols]
    return (a[:, cols] * dT ** 2 + b[:, cols] * (LV_CP * dq) ** 2).sum(0)


def test_grid_sampled_columns_against_oracle(grid):
    cT, cq = grid["cT"], grid["cq"]
    cP = np.zeros(grid["st"]["ncol"])
    for c in grid["sample"]:
        gT, gq = _oracle_grad(grid["st"], int(c), cT, cq, cP)
        assert np.abs(grid["g"]["g_T"][:, c] - gT).max() <= TOL * np.abs(gT).max(), int(c)
        assert np.abs(grid["g"]["g_q"][:, c] - gq).max() <= TOL * np.abs(gq).max(), int(c)


def test_grid_sampled_columns_against_central_differences(torch, grid):
    B = _B()
    st, dev, conv, out = grid["st"], grid["dev"], grid["conv"], grid["out"]
    cols = grid["sample"]
    rng = np.random.default_rng(26)
    vT = rng.standard_normal(dev["T"].shape)
    vq = rng.standard_normal(dev["q"].shape)
    h = 1e-6
    T0, q0 = _np(dev["T"]), _np(dev["q"])
    dT, dq = T0 * vT, q0 * vq  # relative direction: x -> x (1 + h v)

    def fwd(sign):
        d = dict(dev)
        d["T"] = _t(torch, T0 + sign * h * dT)
        d["q"] = _t(torch, q0 + sign * h * dq)
        o = conv.deep_forward(d)
        torch.cuda.synchronize()
        return o

    op, om = fwd(+1.0), fwd(-1.0)
    Lp, Lm = _loss_cols(op, grid["a"], grid["b"], cols), _loss_cols(om, grid["a"], grid["b"], cols)
    L0 = _loss_cols(out, grid["a"], grid["b"], cols)
    ints = [np.stack([_np(o[k])[cols] for k in ("status", "klaunch", "ktop")]) for o in (op, out, om)]
    same = np.all(ints[0] == ints[1], axis=0) & np.all(ints[2] == ints[1], axis=0)
    fd = (Lp - Lm) / (2 * h)
    an = (grid["g"]["g_T"][:, cols] * dT[:, cols]).sum(0) + (grid["g"]["g_q"][:, cols] * dq[:, cols]).sum(0)
    kink = np.abs((Lp - L0) - (L0 - Lm)) / h > 1e-3 * np.abs(an)
    ok = same & ~kink
    assert ok.sum() >= 48, ok.sum()
    rel = np.abs(fd - an)[ok] / np.abs(an)[ok]
    assert rel.max() <= 1e-6, (rel.max(), cols[ok][np.argmax(rel)])


def test_grid_parameter_gradients_on_sampled_columns(torch, grid):
    """Cotangents restricted to the sampled columns: dL/dtau, dL/deps against the oracle's tangents
    (1e-9) and against central differences of the HIP forward in tau and eps (1e-6)."""
    B = _B()
    st, dev, conv, out = grid["st"], grid["dev"], grid["conv"], grid["out"]
    cols = grid["sample"]
    mask = np.zeros(st["ncol"], dtype=bool)
    mask[cols] = True
    cT = np.where(mask, grid["cT"], 0.0)
    cq = np.where(mask, grid["cq"], 0.0)
    g = conv.deep_backward(dev, out, _t(torch, cT), _t(torch, cq), None)
    gtau, geps = float(g["g_tau"]), float(g["g_eps"])
    L = st["nlev"]
    cP = np.zeros(st["ncol"])
    want, scale = np.zeros(2), np.zeros(2)
    for c in cols:
        col = oracle.column(st, int(c))
        for i, (dtau, deps) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            j = oracle.deep_column_jvp(col, np.zeros(L), np.zeros(L), dtau, deps)
            s, a = _cot_dot(cT, cq, cP, int(c), j)
            want[i] += s
            scale[i] += a
    assert abs(gtau - want[0]) <= TOL * scale[0]
    assert abs(geps - want[1]) <= TOL * scale[1]
    p0 = B.make_params()
    h = 1e-6
    for name, got in (("tau", gtau), ("eps_deep", geps)):
        v = getattr(p0, name)
        Ls = []
        for sgn in (+1.0, -1.0):
            conv.set_params(B.make_params(**{name: v * (1 + sgn * h)}))
            o = conv.deep_forward(dev)
            torch.cuda.synchronize()
            assert np.array_equal(_np(o["status"])[cols], _np(out["status"])[cols])
            Ls.append(_loss_cols(o, grid["a"], grid["b"], cols).sum())
        conv.set_params(p0)
        fd = (Ls[0] - Ls[1]) / (2 * h * v)
        assert abs(fd - got) <= 1e-6 * abs(got), (name, fd, got)


def test_autograd_function_matches_direct_call(torch):
    B = _B()
    st = S.subset(S.small_warm(), np.arange(128))
    dev = B.to_device(st)
    conv = B.Conv(st["ncol"], st["nlev"])
    rng = np.random.default_rng(27)
    a = _t(torch, rng.standard_normal(dev["T"].shape))
    T = dev["T"].clone().requires_grad_(True)
    q = dev["q"].clone().requires_grad_(True)
    tau = torch.tensor(3600.0, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(1e-4, dtype=torch.float64, device="cuda", requires_grad=True)
    dTdt, dqdt, prec = B.deep_conv(conv, dev, T, q, tau, eps)
    loss = (a * dTdt ** 2).sum() + (LV_CP * dqdt).pow(2).sum() + 1e3 * prec.sum()
    loss.backward()
    out = conv.deep_forward(dev)
    cT = 2.0 * a * out["dTdt"]
    cq = 2.0 * LV_CP ** 2 * out["dqdt"]
    cP = torch.full_like(out["prec"], 1e3)
    g = conv.deep_backward(dev, out, cT, cq, cP)
    torch.cuda.synchronize()
    assert torch.equal(T.grad, g["g_T"]) and torch.equal(q.grad, g["g_q"])
    assert float(tau.grad) == float(g["g_tau"]) and float(eps.grad) == float(g["g_eps"])
    assert float(T.grad.abs().max()) > 0.0


def test_bit_reproducible_and_padding(torch):
    B = _B()
    st = S.small_warm()
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(28)
    cT, cq, cP = _cotangents(rng, L, n)
    _, dev, out, g1 = _run(torch, st, cT, cq, cP)
    _, _, _, g2 = _run(torch, st, cT, cq, cP)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k
    # the same columns at leading dimension 1000 give the same gradients; pad columns untouched
    ld = 1000
    pad = {k: np.full((v.shape[0], ld) if v.ndim == 2 else (ld,), np.nan) for k, v in st.items()
           if isinstance(v, np.ndarray)}
    for k in pad:
        if st[k].ndim == 2:
            pad[k][:, :n] = st[k]
            pad[k][:, n:] = st[k][:, :1]
        else:
            pad[k][:n] = st[k]
            pad[k][n:] = st[k][0]
    stp = dict(st)
    stp.update(pad)
    devp = B.to_device(stp)
    c = B.Conv(n, L)
    o = c.deep_forward(devp)

    def widen(x):
        w = np.zeros((x.shape[0], ld) if x.ndim == 2 else (ld,))
        w[..., :n] = x
        return _t(torch, w)

    g = c.deep_backward(devp, o, widen(cT), widen(cq), widen(cP))
    torch.cuda.synchronize()
    assert np.array_equal(_np(g["g_T"])[:, :n], g1["g_T"])
    assert np.array_equal(_np(g["g_q"])[:, :n], g1["g_q"])
    assert float(g["g_tau"]) == float(g1["g_tau"])


@pytest.mark.parametrize("n", [1, 63, 257])
def test_ragged_sizes(torch, n):
    base = S.small_warm()
    od = oracle.deep(base)
    act = np.nonzero(od["status"] == 0)[0]
    idx = np.concatenate([act, np.arange(base["ncol"])])[:n] if n > 1 else act[:1]
    idx = np.resize(idx, n)
    st = S.subset(base, idx)
    L = st["nlev"]
    rng = np.random.default_rng(29 + n)
    cT, cq, cP = _cotangents(rng, L, n)
    _, _, out, g = _run(torch, st, cT, cq, cP)
    for c in [0, n - 1]:
        if _np(out["status"])[c] != 0:
            continue
        gT, gq = _oracle_grad(st, c, cT, cq, cP)
        assert np.abs(g["g_T"][:, c] - gT).max() <= TOL * np.abs(gT).max()


@pytest.mark.parametrize("nlev", [46, 256])
def test_other_level_count(torch, nlev):
    st = S.make_state(300, nlev, seed=404, warm=np.ones(300, dtype=bool))
    L, n = st["nlev"], st["ncol"]
    rng = np.random.default_rng(31)
    cT, cq, cP = _cotangents(rng, L, n)
    _, _, out, g = _run(torch, st, cT, cq, cP)
    act = np.nonzero(_np(out["status"]) == 0)[0]
    assert len(act) > 50
    for c in act[:5]:
        gT, gq = _oracle_grad(st, int(c), cT, cq, cP)
        assert np.abs(g["g_T"][:, c] - gT).max() <= TOL * np.abs(gT).max()
        assert np.abs(g["g_q"][:, c] - gq).max() <= TOL * np.abs(gq).max()


def test_invalid_arguments(torch):
    import ctypes as C

    B = _B()
    st = S.subset(S.small_warm(), np.arange(64))
    dev = B.to_device(st)
    conv = B.Conv(64, st["nlev"])
    out = conv.deep_forward(dev)
    L = B.lib()
    nbytes = L.conv_backward_workspace_bytes(64, st["nlev"], 64)
    assert nbytes > 0 and L.conv_backward_workspace_bytes(64, st["nlev"], 10) == 0
    ws = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) & ~255
    gT = torch.empty_like(dev["T"])
    gq = torch.empty_like(dev["T"])
    gp = torch.empty(2, dtype=torch.float64, device="cuda")
    s = conv._state(dev)
    o = conv._deep_struct(out)
    cot = B.DeepCot(None, None, None)
    good = B.DeepGrad(gT.data_ptr(), gq.data_ptr(), gp.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    call = lambda g, w, nb: L.conv_deep_backward(conv.h, C.byref(s), C.byref(o), C.byref(cot),
                                                 C.byref(g), C.c_void_p(w), nb, stream)
    assert call(good, base, nbytes) == B.CONV_OK
    torch.cuda.synchronize()
    assert float(gp.abs().sum()) == 0.0  # zero cotangents give zero gradients
    assert call(B.DeepGrad(None, gq.data_ptr(), gp.data_ptr()), base, nbytes) == B.CONV_EINVAL
    assert call(good, base + 8, nbytes) == B.CONV_EINVAL
    assert call(good, base, nbytes - 4096) == B.CONV_EINVAL
