"""Pins of the seed-network oracle (CPU): convolution against SciPy's
correlate, gradients against central finite differences, adjoint pairs,
interpolation exactness on linear fields, Adam's first step."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import workloads as W
from oracle import nets


def rand_theta(c1, c2, seed):
    _, n = nets.param_layout(c1, c2)
    return np.random.default_rng(seed).normal(0.0, 0.3, n)


def test_conv3d_is_zero_padded_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 5, 4, 6))
    w = rng.normal(size=(2, 3, 3, 3, 3))
    b = rng.normal(size=2)
    out = nets.conv3d(x, w, b)
    for o in range(2):
        ref = b[o] + sum(ndi.correlate(x[c], w[o, c], mode="constant", cval=0.0) for c in range(3))
        assert np.allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 6, 8))
    y = rng.normal(size=(2, 2, 3, 4))
    assert np.isclose(np.sum(nets.pool2(x) * y), np.sum(x * nets.pool2_backward(y)))
    assert np.isclose(np.sum(nets.up2(y) * x), np.sum(y * nets.up2_backward(x)))
    assert np.allclose(nets.pool2(nets.up2(y)), y)


def test_gradients_match_central_differences():
    c1, c2 = 3, 4
    rng = np.random.default_rng(3)
    theta = rand_theta(c1, c2, 4)
    inp = rng.uniform(0, 1, size=(2, 4, 4, 4))
    y = rng.normal(size=(4, 4, 4))
    loss, g = nets.loss_and_grad(theta, inp, y, c1, c2)
    lay, n = nets.param_layout(c1, c2)
    idx = list(rng.choice(n, 60, replace=False))
    for _name, wo, wl, bo, co, ci in lay:
        idx += list(range(bo, bo + co))           # every bias
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nets.loss_and_grad(tp, inp, y, c1, c2)[0] - nets.loss_and_grad(tm, inp, y, c1, c2)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, i


def test_loss_is_mse_of_forward():
    c1, c2 = 2, 2
    theta = rand_theta(c1, c2, 5)
    inp = np.random.default_rng(6).uniform(size=(2, 2, 2, 4))
    y = np.zeros((2, 2, 4))
    u, _ = nets.forward(theta, inp, c1, c2)
    loss, _ = nets.loss_and_grad(theta, inp, y, c1, c2)
    assert np.isclose(loss, np.mean(u ** 2))


def test_interpolation_exact_for_linear_fields():
    prob = W.tiny_3d(16, 16, 16, 3)
    f = 4
    D = H = Wd = 4
    cz, cy, cx = np.meshgrid(np.arange(D), np.arange(H), np.arange(Wd), indexing="ij")
    u = 0.3 + 0.1 * cx - 0.2 * cy + 0.05 * cz          # linear in centre coordinates
    t = nets.net_to_nodes(prob, u, f, scale=2.0).reshape(17, 17, 17)
    # node n sits at centre coordinate (n - f/2)/f; exact inside the centres' span
    for (k, j, i) in [(2, 2, 2), (6, 10, 14), (14, 14, 2), (9, 5, 7)]:
        want = 2.0 * (0.3 + 0.1 * (i - 2) / 4 - 0.2 * (j - 2) / 4 + 0.05 * (k - 2) / 4)
        if prob.fix_lo[2] <= k <= prob.fix_hi[2] and prob.fix_lo[1] <= j <= prob.fix_hi[1] \
                and prob.fix_lo[0] <= i <= prob.fix_hi[0]:
            want = 0.0
        assert np.isclose(t[k, j, i], want, rtol=1e-13, atol=1e-13)
    # clamping: nodes outside the centres take the nearest centre's value
    assert np.isclose(t[16, 16, 16], 2.0 * u[3, 3, 3])


def test_target_takes_centre_nodes_and_input_channels():
    prob = W.tiny_3d(16, 16, 16, 3)
    f = 4
    T = np.arange(prob.nnodes, dtype=float)
    y = nets.net_target(prob, T, f, scale=10.0)
    assert y.shape == (4, 4, 4)
    assert y[1, 2, 3] == (14 + 17 * (10 + 17 * 6)) / 10.0
    x = np.full(prob.nelem, 0.4)
    inp = nets.net_input(prob, x, f)
    assert np.allclose(inp[0], 0.4)
    assert inp[1].max() > 0 and inp[1].min() == 0.0
    assert inp[1][1:].max() == 0.0                       # only the z = 0 layer touches the patch


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = nets.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(t1, theta - 0.01 * np.sign(g), rtol=0, atol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
