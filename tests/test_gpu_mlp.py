"""The surrogate network's HIP kernels (BF16 MFMA GEMM with fused epilogues, MSE, backward, Adam;
through the C ABI) against the numpy reference (oracle/mlp_ref.py, pinned on the CPU), with BF16
rounding emulated where the GPU rounds.

Tolerances.  FP32 outputs of one GEMM: |gpu - ref| <= 3e-5 * (|A| |B|^T) elementwise (the bound on
float32 accumulation error, K * 2^-24 * sum|a b|, for K <= 512).  BF16 outputs: at most one unit in
the last place (2^-7 relative) where the float32 value lies within rounding error of a tie, and
bit-equal on at least 99.9 % of elements.  Whole-network quantities pass through several BF16
roundings.  Each can flip one BF16 ulp where GPU and reference differ in the last float32 bits
(float32 accumulation over K = 512 differs by ~1e-6 relative, so ~5e-4 of activations sit close
enough to a rounding tie to flip: about one flip per 2048 activations of a row over four layers).
A flip moves a downstream value by ~2^-8 |a w|.  Whole-network outputs and gradients are therefore
compared normwise at 5e-3, the size of a few flips in one row."""
import numpy as np
import pytest

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu

WIDTHS = [96, 512, 512, 512, 512, 64]


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _B():
    from paper_1711_00289_amd import binding

    return binding


def bf16_dev(torch, x):
    bits = R.bf16_bits(np.asarray(x, np.float32))
    return torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)


def host_bf16(t):
    import torch

    return R.from_bits(t.contiguous().view(torch.int16).cpu().numpy().view(np.uint16)).astype(np.float64)


@pytest.mark.parametrize("M,N,K", [(1000, 512, 96), (300, 64, 512), (128, 128, 32), (1, 64, 8),
                                   (4097, 128, 512), (77, 64, 40)])
def test_gemm_fp32_epilogue(torch, M, N, K):
    rng = np.random.default_rng(M + N + K)
    A = R.bf16(rng.standard_normal((M, K)).astype(np.float32)).astype(np.float64)
    Bm = R.bf16(rng.standard_normal((N, K)).astype(np.float32)).astype(np.float64)
    bias = rng.standard_normal(N).astype(np.float32)
    c = _B().gemm_nt(bf16_dev(torch, A), bf16_dev(torch, Bm), torch.from_numpy(bias).cuda(), mode=0)
    got = c.cpu().numpy().astype(np.float64)
    ref = A @ Bm.T + bias
    bound = 3e-5 * (np.abs(A) @ np.abs(Bm).T + np.abs(bias)) + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= bound), float((err / bound).max())


@pytest.mark.parametrize("M,N,K", [(999, 512, 96), (256, 64, 512)])
def test_gemm_gelu_epilogue(torch, M, N, K):
    rng = np.random.default_rng(M * 7 + K)
    A = R.bf16(rng.standard_normal((M, K)).astype(np.float32)).astype(np.float64)
    Bm = R.bf16((rng.standard_normal((N, K)) / np.sqrt(K)).astype(np.float32)).astype(np.float64)
    bias = (0.1 * rng.standard_normal(N)).astype(np.float32)
    act, z = _B().gemm_nt(bf16_dev(torch, A), bf16_dev(torch, Bm), torch.from_numpy(bias).cuda(),
                          mode=1, z=True)
    zref = A @ Bm.T + bias
    bound = 3e-5 * (np.abs(A) @ np.abs(Bm).T + np.abs(bias)) + 1e-30
    zg = z.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(zg - zref) <= bound)
    ag = host_bf16(act)
    aref = R.bf16(R.gelu(zg.astype(np.float32)).astype(np.float32)).astype(np.float64)
    eq = ag == aref
    assert eq.mean() >= 0.999, eq.mean()
    assert np.all(np.abs(ag - aref) <= 2.0 ** -7 * np.abs(aref) + 1e-30)


@pytest.fixture(scope="module", params=[96, 512])
def full_size_product(request):
    """Operands of the full-size product on the 256 x 256 tile (M = 131,137, N = 512, K = 96 or
    512) with its float64 reference and FP32-accumulation bound (computed once per K)."""
    K = request.param
    M, N = 131_137, 512
    rng = np.random.default_rng(K + 5)
    A = R.bf16(rng.standard_normal((M, K)).astype(np.float32)).astype(np.float64)
    Bm = R.bf16((rng.standard_normal((N, K)) / np.sqrt(K)).astype(np.float32)).astype(np.float64)
    bias = (0.1 * rng.standard_normal(N)).astype(np.float32)
    ref = A @ Bm.T + bias
    bound = 3e-5 * (np.abs(A) @ np.abs(Bm).T + np.abs(bias)) + 1e-30
    return A, Bm, bias, ref, bound


@pytest.mark.parametrize("mode", [0, 1])
def test_gemm_full_size_on_the_large_tile(torch, full_size_product, mode):
    """The 256 x 256 tile (eight wavefronts, operands loaded straight into swizzled LDS rows) runs
    every hidden layer of the one-chunk inference: it is chosen when the product has at least
    1,024 tiles (M >= 131,072 at N = 512).  M = 131,137 adds a ragged 65-row tail; K = 96 is the
    input layer (one direct K tile and a zero-filled K tail), K = 512 a hidden layer.  Every
    element against the float64 product: mode 0 (FP32 + bias) and mode 1's FP32 pre-activation at
    the accumulation bound, mode 1's BF16 GELU output bit-equal on >= 99.9 % of the elements and
    within one BF16 unit everywhere."""
    A, Bm, bias, ref, bound = full_size_product
    print(f"gemm {A.shape[0]} x {Bm.shape[0]} x {A.shape[1]} mode {mode}", flush=True)
    a, b, bb = bf16_dev(torch, A), bf16_dev(torch, Bm), torch.from_numpy(bias).cuda()
    if mode == 0:
        c = _B().gemm_nt(a, b, bb, mode=0)
        err = np.abs(c.cpu().numpy().astype(np.float64) - ref)
        assert np.all(err <= bound), float((err / bound).max())
        return
    act, z = _B().gemm_nt(a, b, bb, mode=1, z=True)
    zg = z.cpu().numpy().astype(np.float64)
    err = np.abs(zg - ref)
    assert np.all(err <= bound), float((err / bound).max())
    ag = host_bf16(act)
    aref = R.bf16(R.gelu(zg.astype(np.float32)).astype(np.float32)).astype(np.float64)
    assert (ag == aref).mean() >= 0.999
    assert np.all(np.abs(ag - aref) <= 2.0 ** -7 * np.abs(aref) + 1e-30)


def _net(torch, batch, seed, widths=WIDTHS):
    B = _B()
    net = B.MLP(widths, max_batch=max(batch, 64))
    params = R.init_params(widths, seed)
    rng = np.random.default_rng(seed + 1)
    params = [(W, (0.05 * rng.standard_normal(len(b))).astype(np.float32)) for W, b in params]
    net.set_params(torch.from_numpy(R.flatten(params)).cuda())
    x = R.bf16(rng.standard_normal((batch, widths[0])).astype(np.float32)).astype(np.float64)
    t = rng.standard_normal((batch, widths[-1])).astype(np.float32)
    return net, params, x, t


def _rel(a, b):
    return float(np.abs(a - b).max() / (np.abs(b).max() + 1e-30))


@pytest.mark.parametrize("batch", [1, 333, 2048])
def test_forward_loss_backward_against_reference(torch, batch):
    net, params, x, t = _net(torch, batch, 11)
    xd = bf16_dev(torch, x)
    y = net.forward(xd, keep=True)
    loss = net.mse(y, torch.from_numpy(t).cuda(), 61)
    net.backward(batch)
    grads = R.unflatten(net.get_grads().cpu().numpy(), WIDTHS)
    torch.cuda.synchronize()
    yr, acts, zs = R.forward(params, x, emulate=True)
    assert _rel(y.cpu().numpy(), yr) <= 5e-3
    lr, dy = R.mse(yr, t, 61, emulate=True)
    assert abs(float(loss.item()) - lr) <= 5e-3 * lr
    gref = R.backward(params, acts, zs, dy, emulate=True)
    for i, ((gW, gb), (rW, rb)) in enumerate(zip(grads, gref)):
        assert _rel(gW, rW) <= 5e-3, (i, "W", _rel(gW, rW))
        assert _rel(gb, rb) <= 5e-3, (i, "b", _rel(gb, rb))


@pytest.mark.parametrize("widths,batch", [((64, 32, 96, 32), 333), ((32, 64, 64, 32), 1),
                                          ((96, 160, 32, 64), 777)])
def test_other_widths_forward_backward(torch, widths, batch):
    """Narrow layers (the 128 x 64 tile, also for the transposed copies of the training
    products), a width that is not a multiple of the 128-column tile, ragged batches."""
    widths = list(widths)
    net, params, x, t = _net(torch, batch, 21, widths)
    y = net.forward(bf16_dev(torch, x), keep=True)
    loss = net.mse(y, torch.from_numpy(t).cuda(), widths[-1])
    net.backward(batch)
    grads = R.unflatten(net.get_grads().cpu().numpy(), widths)
    torch.cuda.synchronize()
    yr, acts, zs = R.forward(params, x, emulate=True)
    assert _rel(y.cpu().numpy(), yr) <= 5e-3
    lr, dy = R.mse(yr, t, widths[-1], emulate=True)
    assert abs(float(loss.item()) - lr) <= 5e-3 * lr
    gref = R.backward(params, acts, zs, dy, emulate=True)
    for i, ((gW, gb), (rW, rb)) in enumerate(zip(grads, gref)):
        assert _rel(gW, rW) <= 5e-3, (i, "W", _rel(gW, rW))
        assert _rel(gb, rb) <= 5e-3, (i, "b", _rel(gb, rb))


def test_separate_training_batch_limit(torch):
    """A context whose training limit is below its inference limit gives the same bits as one
    sized for training at the full batch: inference over the full batch, a training forward,
    loss and backward at the training limit; a training forward above the limit is rejected."""
    B = _B()
    net, params, x, t = _net(torch, 1000, 31)
    small = B.MLP(WIDTHS, max_batch=3000, max_train_batch=1000)
    small.set_params(torch.from_numpy(R.flatten(params)).cuda())
    big = B.MLP(WIDTHS, max_batch=3000)
    big.set_params(torch.from_numpy(R.flatten(params)).cuda())
    rng = np.random.default_rng(32)
    xi = bf16_dev(torch, rng.standard_normal((3000, WIDTHS[0])).astype(np.float32))
    assert torch.equal(small.forward(xi), big.forward(xi))
    xd, td = bf16_dev(torch, x), torch.from_numpy(t).cuda()
    for m in (small, big):
        y = m.forward(xd, keep=True)
        m.mse(y, td, 61)
        m.backward(1000)
    torch.cuda.synchronize()
    assert torch.equal(small.get_grads(), big.get_grads())
    with pytest.raises(RuntimeError):
        small.forward(xi[:1001], keep=True)


def test_gradients_reproducible_bit_for_bit(torch):
    net, params, x, t = _net(torch, 1500, 12)
    xd, td = bf16_dev(torch, x), torch.from_numpy(t).cuda()
    out = []
    for _ in range(2):
        y = net.forward(xd, keep=True)
        net.mse(y, td, 61)
        net.backward(1500)
        out.append(net.get_grads().cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_train_step_equals_the_separate_calls(torch):
    net1, params, x, t = _net(torch, 777, 16)
    net2, _, _, _ = _net(torch, 777, 16)
    xd, td = bf16_dev(torch, x), torch.from_numpy(t).cuda()
    for step in range(3):
        y1 = net1.forward(xd, keep=True)
        l1 = net1.mse(y1, td, 61).clone()
        net1.backward(777)
        net1.adam_step(1e-3)
        y2, l2 = net2.train_step(xd, td, 61, 1e-3)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2) and torch.equal(l1, l2)
    assert torch.equal(net1.get_params(), net2.get_params())


def test_adam_step_against_reference(torch):
    net, params, x, t = _net(torch, 512, 13)
    xd, td = bf16_dev(torch, x), torch.from_numpy(t).cuda()
    p0 = net.get_params().cpu().numpy()
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0
    for step in range(1, 4):
        y = net.forward(xd, keep=True)
        net.mse(y, td, 61)
        net.backward(512)
        g = net.get_grads().cpu().numpy()
        net.adam_step(1e-3, 0.9, 0.999, 1e-8)
        p, m, v = R.adam(p, g, m, v, step, 1e-3, 0.9, 0.999, 1e-8)
        got = net.get_params().cpu().numpy()
        # float32 rounding of the update (a few ulp of p) plus 1e-4 of one step (lr); a wrong moment
        # or bias correction moves parameters by a sizeable fraction of lr
        err = np.abs(got - p)
        assert np.all(err <= 4 * np.spacing(np.abs(p)) + 1e-7), (step, float(err.max()))


def test_training_reduces_the_loss_on_a_teacher_network(torch):
    """A student trained by the kernels fits a random GELU teacher: the loss falls tenfold."""
    widths = [64, 128, 128, 32]
    rng = np.random.default_rng(14)
    teacher = R.init_params(widths, 99)
    X = R.bf16(rng.standard_normal((8192, 64)).astype(np.float32)).astype(np.float64)
    Y, _, _ = R.forward(teacher, X, emulate=False)
    net, _, _, _ = _net(torch, 8192, 15, widths)
    xd, yd = bf16_dev(torch, X), torch.from_numpy(Y.astype(np.float32)).cuda()
    y = net.forward(xd, keep=False)
    first = float(net.mse(y, yd, 32).item())
    curve = []
    for step in range(1200):
        sl = slice((step % 8) * 1024, (step % 8 + 1) * 1024)
        y = net.forward(xd[sl], keep=True)
        net.mse(y, yd[sl], 32)
        net.backward(1024)
        net.adam_step(2e-3)
        if step % 200 == 199:
            y = net.forward(xd, keep=False)
            curve.append(float(net.mse(y, yd, 32).item()))
    print("teacher-student loss", first, curve)
    assert all(b < a for a, b in zip(curve, curve[1:])), curve
    assert curve[-1] < 0.2 * first, (first, curve)


def test_invalid_arguments(torch):
    import ctypes as C

    B = _B()
    L = B.lib()
    bad = (C.c_int32 * 3)(96, 100, 64)  # not a multiple of 32
    assert L.mlp_workspace_bytes(bad, 2, 1024) == 0
    ok = (C.c_int32 * 3)(96, 128, 64)
    assert L.mlp_workspace_bytes(ok, 2, 0) == 0
    h = C.c_void_p()
    assert L.mlp_create(ok, 2, 1024, C.c_void_p(257), 1 << 30, C.byref(h)) == B.CONV_EINVAL
    net = B.MLP([96, 128, 64], 64)
    with pytest.raises(RuntimeError):
        net.backward(64)  # no forward with keep yet
    x = torch.zeros(65, 96, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(RuntimeError):
        net.forward(x)  # batch above max_batch
