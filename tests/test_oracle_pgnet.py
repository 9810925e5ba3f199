"""Pins of the learned-guess conv net reference: library correlation, finite differences,
BF16 rounding, Adam's first step."""
import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import pgnet as N


def test_bf16_round_matches_torch_bit_exactly():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10 ** rng.uniform(-8, 8, 10000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.005859375, -2.5, 3.0e38])])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(N.bf16_round(x), ref)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 6, 5))
    W = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    out = N.conv3d(x, W, b)
    for o in range(3):
        ref = np.full(x.shape[1:], b[o])
        for c in range(2):
            k = np.zeros((3, 3, 3))
            for t, (dx, dy, dz) in enumerate(N.TAPS):
                k[dx + 1, dy + 1, dz + 1] = W[t, c, o]
            ref += ndimage.correlate(x[c], k, mode="constant", cval=0.0)
        np.testing.assert_allclose(out[o], ref, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    params = N.init_weights(seed=3, hidden=4)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in params]   # nonzero biases
    x = rng.normal(size=(3, 5, 5, 5))
    t = rng.normal(size=(5, 5, 5))
    mask = rng.random((5, 5, 5)) > 0.3

    def L(ps):
        y, _ = N.forward(ps, x, bf16=False)
        return N.loss_and_grad(y, t, mask)[0]

    y, cache = N.forward(params, x, bf16=False)
    _, dy = N.loss_and_grad(y, t, mask)
    grads = N.backward(params, cache, dy, bf16=False)
    h = 1e-6
    for k in range(6):
        flat = params[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[k].reshape(-1)[idx] += h
            pm[k].reshape(-1)[idx] -= h
            fd = (L(pp) - L(pm)) / (2 * h)
            assert grads[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_loss_is_gauge_invariant():
    rng = np.random.default_rng(4)
    y = rng.normal(size=(4, 4, 4))
    t = rng.normal(size=(4, 4, 4))
    m = np.ones((4, 4, 4), bool)
    assert N.loss_and_grad(y, t, m)[0] == pytest.approx(N.loss_and_grad(y + 3.0, t, m)[0], abs=1e-12)
    assert abs(N.loss_and_grad(y, t, m)[1].sum()) < 1e-12


def test_adam_first_step_is_signed_lr():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 0.0])]
    out = N.adam(p, g, {}, lr=1e-3)
    np.testing.assert_allclose(out[0], [1.0 - 1e-3, -2.0 + 1e-3, 3.0], atol=1e-9)


def test_features_are_normalised():
    rng = np.random.default_rng(5)
    p1 = rng.normal(size=(6, 6, 6)) * 3 + 7
    act = rng.random((6, 6, 6)) > 0.2
    f, mu, s = N.features(p1, p1 * 0.5, p1 * 0.1, 0.25, act)
    assert abs(f[0][act].mean()) < 1e-12
    assert np.sqrt(np.mean(f[0][act] ** 2)) == pytest.approx(1.0)
    assert np.all(f[:, ~act] == 0)
