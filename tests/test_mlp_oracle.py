"""Pins of the MLP oracle: backpropagation against central finite
differences of the loss, and GELU against its definition by quadrature."""
import numpy as np
from scipy import integrate

from oracle import mlp_oracle as mo
import synth


def test_gelu_matches_definition():
    for z in (-3.0, -0.7, 0.0, 0.4, 2.5):
        cdf = integrate.quad(lambda u: np.exp(-0.5 * u * u) / np.sqrt(2 * np.pi), -np.inf, z)[0]
        assert abs(mo.gelu(z) - z * cdf) < 1e-12
        h = 1e-6
        fd = (mo.gelu(z + h) - mo.gelu(z - h)) / (2 * h)
        assert abs(mo.gelu_grad(z) - fd) < 1e-8


def test_backprop_matches_finite_differences():
    nin, width, depth = 7, 12, 3
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.1)
              for W, b in synth.mlp.unflatten(synth.mlp.init_params(nin, width, depth, seed=9), nin, width, depth)]
    rng = np.random.default_rng(3)
    x = rng.standard_normal((10, nin))
    t = rng.standard_normal(10)
    loss, grads = mo.loss_and_grads(params, x, t)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = mo.loss_and_grads(params, x, t)
                flat[idx] = old - h
                lm, _ = mo.loss_and_grads(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)


def test_adam_first_step_is_lr_times_sign():
    params = [(np.ones((2, 3)), np.zeros(3))]
    grads = [(np.full((2, 3), 0.5), np.array([-2.0, 0.0, 3.0]))]
    m = [(np.zeros((2, 3)), np.zeros(3))]
    v = [(np.zeros((2, 3)), np.zeros(3))]
    p, _, _ = mo.adam_step(params, grads, m, v, 1, 0.01, eps=1e-12)
    assert np.allclose(p[0][0], 1.0 - 0.01)
    assert np.allclose(p[0][1], [0.01, 0.0, -0.01])


def test_bf16_round_grid_and_ties():
    grid = np.array([1.0, 1.0078125, -2.5, 3.0e-3, 0.0], np.float32)
    grid = synth.mlp.bf16_round(grid)
    assert np.array_equal(synth.mlp.bf16_round(grid), grid)
    # halfway between 1 and 1 + 2^-7 goes to the even mantissa (1.0);
    # halfway between 1 + 2^-7 and 1 + 2^-6 goes to 1 + 2^-6
    assert synth.mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert synth.mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    assert np.max(np.abs(synth.mlp.bf16_round(x) - x) / np.abs(x)) <= 2.0 ** -8
