"""Pins of the numpy reference of the surrogate network (oracle/mlp_ref.py), independently of its
own arithmetic:

* bfloat16 rounding: exact bit patterns of representable values, ties to even, one-ulp steps;
* GELU: GELU(0) = 0, GELU'(0) = 1/2, GELU(z) -> z and -> 0 in the tails, the derivative against a
  central difference, and the closed form at z = 1 (Phi(1) = 0.841344746...);
* the float64 backward pass against central finite differences of the loss on a tiny network (the
  definition of the gradient: a dropped term, wrong sign or transposed operand fails it);
* the float64 MSE and its gradient against their definitions on a 2x3 example worked by hand;
* one Adam step against the algorithm worked by hand on a scalar (first step moves by lr).
"""
import math

import numpy as np
import pytest

from oracle import mlp_ref as R


def test_bf16_rounding_bit_patterns():
    assert R.bf16_bits(np.float32([1.0]))[0] == 0x3F80
    assert R.bf16_bits(np.float32([-2.0]))[0] == 0xC000
    one_ulp = np.float32(2.0 ** -7)
    # halfway between 1 and 1 + 2^-7 rounds to even (1.0); just above rounds up
    assert R.bf16(np.float32([1.0 + 2.0 ** -8]))[0] == np.float32(1.0)
    assert R.bf16(np.float32([1.0 + 2.0 ** -8 + 2.0 ** -20]))[0] == np.float32(1.0) + one_ulp
    # halfway between 1 + 2^-7 and 1 + 2^-6 rounds to even (1 + 2^-6)
    assert R.bf16(np.float32([1.0 + 3 * 2.0 ** -8]))[0] == np.float32(1.0 + 2.0 ** -6)
    x = np.float32(np.random.default_rng(0).standard_normal(10000))
    r = R.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-7))
    assert np.array_equal(R.from_bits(R.bf16_bits(x)), r)


def test_gelu_special_values_and_derivative():
    assert R.gelu(0.0) == 0.0 and R.gelu_grad(0.0) == 0.5
    assert abs(R.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(R.gelu(8.0) - 8.0) < 1e-12 and abs(R.gelu(-8.0)) < 1e-12
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    assert np.allclose(R.gelu_grad(z), fd, rtol=0, atol=1e-9)


def test_mse_by_hand():
    y = np.array([[1.0, 2.0, 5.0], [0.0, -1.0, 7.0]])
    t = np.array([[0.0, 2.0, 0.0], [1.0, 1.0, 0.0]])
    loss, dy = R.mse(y, t, 2, emulate=False)
    assert loss == pytest.approx((1 + 0 + 1 + 4) / 4.0, abs=0)
    assert np.array_equal(dy, np.array([[0.5, 0.0, 0.0], [-0.5, -1.0, 0.0]]))


def test_backward_matches_central_differences():
    widths = [8, 16, 16, 5]
    params = R.init_params(widths, 3)
    params = [(W.astype(np.float64), np.random.default_rng(4).standard_normal(len(b)) * 0.1)
              for W, b in params]
    rng = np.random.default_rng(5)
    x = rng.standard_normal((7, 8))
    t = rng.standard_normal((7, 5))

    def loss_of(ps):
        y, _, _ = R.forward(ps, x, emulate=False)
        return R.mse(y, t, 4, emulate=False)[0]

    y, acts, zs = R.forward(params, x, emulate=False)
    _, dy = R.mse(y, t, 4, emulate=False)
    grads = R.backward(params, acts, zs, dy, emulate=False)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 17)):
                old = flat[idx]
                flat[idx] = old + h
                lp = loss_of(params)
                flat[idx] = old - h
                lm = loss_of(params)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (li, idx)


def test_emulated_forward_rounds_where_the_gpu_stores():
    widths = [32, 64, 32]
    params = R.init_params(widths, 6)
    x = R.bf16(np.random.default_rng(7).standard_normal((5, 32)).astype(np.float32)).astype(np.float64)
    y, acts, zs = R.forward(params, x, emulate=True)
    assert np.array_equal(acts[1], R.bf16(acts[1].astype(np.float32)).astype(np.float64))
    assert np.array_equal(zs[1], zs[1].astype(np.float32).astype(np.float64))
    y64, _, _ = R.forward(params, x, emulate=False)
    assert np.allclose(y, y64, rtol=0.05, atol=0.05)  # bf16 weights: a few per cent at most


def test_adam_first_step_by_hand():
    p, m, v = R.adam(np.float32([1.0]), np.float32([0.3]), np.float32([0.0]), np.float32([0.0]),
                     1, 1e-3, 0.9, 0.999, 1e-8)
    # m_hat = g, v_hat = g^2: the first step is lr * g / (|g| + eps)
    assert abs(p[0] - (1.0 - 1e-3 * 0.3 / (0.3 + 1e-8))) < 1e-7
    # float32 arithmetic: 1 - 0.999 carries a relative error of about 1e-5
    assert abs(m[0] - 0.03) < 1e-8 and abs(v[0] - 0.001 * 0.09) < 2e-5 * 0.001 * 0.09
