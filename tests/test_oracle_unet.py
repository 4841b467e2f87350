"""Pins of the seed-network oracle (CPU): convolution against SciPy's
correlate, pooling and upsampling against PyTorch's CPU routines, adjoint
identities of every linear operator, gradients against central differences,
node averaging exact on linear fields, BF16 rounding against PyTorch's
bfloat16 conversion, Adam's first step."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import workloads as W
from oracle import unet


def rand_theta(C, seed, s=0.3):
    _, n = unet.param_layout(C)
    return np.random.default_rng(seed).normal(0.0, s, n)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        # exact ties between two BF16 neighbours (low 16 bits = 0x8000)
                        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(float),
                        [0.0, -0.0, 1.0, -3.5, 65504.0]])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16r(x), want)


def test_conv3d_is_zero_padded_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 5, 4, 6))
    w = rng.normal(size=(2, 3, 3, 3, 3))
    b = rng.normal(size=2)
    out = unet.conv3d(x, w, b)
    for o in range(2):
        ref = b[o] + sum(ndi.correlate(x[c], w[o, c], mode="constant", cval=0.0) for c in range(3))
        assert np.allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(4, 3, 5, 4))
    w = rng.normal(size=(5, 4, 3, 3, 3))
    g = rng.normal(size=(5, 3, 5, 4))
    zero = np.zeros(5)
    lhs = np.sum(unet.conv3d(x, w, zero) * g)
    assert np.isclose(lhs, np.sum(x * unet.conv3d_input_grad(w, g)), rtol=1e-12)
    gw, gb = unet.conv3d_weight_grad(x, g)
    assert np.isclose(lhs, np.sum(w * gw), rtol=1e-12)
    assert np.allclose(gb, g.sum(axis=(1, 2, 3)))


def test_pool_and_upsampling_match_torch():
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, 4, 6, 8))
    want = F.avg_pool3d(torch.tensor(x)[None], 2)[0].numpy()
    assert np.allclose(unet.pool2(x), want, rtol=1e-14, atol=1e-14)
    y = rng.normal(size=(3, 2, 3, 5))
    want = F.interpolate(torch.tensor(y)[None], scale_factor=2, mode="trilinear", align_corners=False)[0].numpy()
    assert np.allclose(unet.up2(y), want, rtol=1e-13, atol=1e-13)


def test_pool_and_upsampling_adjoints():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, 4, 6, 8))
    y = rng.normal(size=(2, 2, 3, 4))
    assert np.isclose(np.sum(unet.pool2(x) * y), np.sum(x * unet.pool2_adjoint(y)))
    assert np.isclose(np.sum(unet.up2(y) * x), np.sum(y * unet.up2_adjoint(x)))
    # a constant field stays constant through both
    c = np.full((1, 2, 2, 2), 0.7)
    assert np.allclose(unet.up2(c), 0.7) and np.allclose(unet.pool2(unet.up2(c)), 0.7)


def test_layer_list_and_parameter_count():
    C = (16, 32, 64, 64)
    names = [n for n, *_ in unet.layer_list(C)]
    assert names == ["e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b",
                     "d2a", "d2b", "d1a", "d1b", "d0a", "d0b", "head"]
    ci = {n: c for n, _, c, _ in unet.layer_list(C)}
    assert (ci["e0a"], ci["d2a"], ci["d1a"], ci["d0a"]) == (3, 128, 96, 48)
    # 27 (3*16 + 16*16 + 16*32 + 32*32 + 32*64 + 3*64*64 + 128*64 + 64*64 + 96*32 + 32*32
    #     + 48*16 + 16*16) + biases + head
    w27 = 3 * 16 + 16 * 16 + 16 * 32 + 32 * 32 + 32 * 64 + 3 * 64 * 64 + 128 * 64 + 64 * 64 \
        + 96 * 32 + 32 * 32 + 48 * 16 + 16 * 16
    biases = 2 * 16 + 2 * 32 + 2 * 64 + 2 * 64 + 2 * 64 + 2 * 32 + 2 * 16 + 1
    assert unet.param_layout(C)[1] == 27 * w27 + biases + 16


@pytest.mark.parametrize("bf16", [False, True])
def test_network_gradient_matches_central_differences(bf16):
    """FP64 mode: every bias and a sample of weights against central
    differences of the loss. BF16 mode is not differentiable (rounding), so
    there it is checked against the FP64 gradient to the BF16 precision."""
    prob = W.tiny_3d(8, 8, 8, 3)
    C = (3, 4, 4)
    rng = np.random.default_rng(5)
    theta = rand_theta(C, 6)
    x = rng.uniform(0.05, 1.0, prob.nelem)
    qe = W.element_source(prob)
    T = rng.uniform(0.0, 1.0, prob.nnodes)
    loss, g = unet.loss_and_grad(prob, theta, x, qe, T, 1.0, C, bf16=bf16)
    if bf16:
        _, g64 = unet.loss_and_grad(prob, theta, x, qe, T, 1.0, C)
        assert np.linalg.norm(g - g64) <= 3e-2 * np.linalg.norm(g64)
        return
    lay, n = unet.param_layout(C)
    idx = list(rng.choice(n, 50, replace=False))
    for _name, wo, wl, bo, co, ci, k in lay:
        idx += list(range(bo, bo + co))
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (unet.loss_and_grad(prob, tp, x, qe, T, 1.0, C)[0] -
              unet.loss_and_grad(prob, tm, x, qe, T, 1.0, C)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_output_gradient_matches_central_differences():
    prob = W.tiny_3d(4, 6, 4, 2)
    rng = np.random.default_rng(7)
    u = rng.normal(size=(4, 6, 4))
    T = rng.normal(size=prob.nnodes)
    loss, du = unet.loss_and_output_grad(prob, u, T, 2.0)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (3, 5, 3), (2, 0, 1)]:
        up, um = u.copy(), u.copy()
        up[idx] += h
        um[idx] -= h
        fd = (unet.loss_and_output_grad(prob, up, T, 2.0)[0] - unet.loss_and_output_grad(prob, um, T, 2.0)[0]) / (2 * h)
        assert np.isclose(fd, du[idx], rtol=1e-6, atol=1e-10)


def test_node_average_exact_for_linear_fields():
    prob = W.tiny_3d(8, 8, 8, 3)
    cz, cy, cx = np.meshgrid(np.arange(8) + 0.5, np.arange(8) + 0.5, np.arange(8) + 0.5, indexing="ij")
    u = 0.3 + 0.1 * cx - 0.2 * cy + 0.05 * cz          # linear in element-centre coordinates
    t = unet.to_nodes(prob, u, 2.0).reshape(9, 9, 9)
    fixed = unet.fixed_nodes(prob)
    for (k, j, i) in [(1, 1, 1), (4, 6, 2), (7, 7, 7), (3, 5, 6)]:      # interior nodes
        want = 0.0 if fixed[k, j, i] else 2.0 * (0.3 + 0.1 * i - 0.2 * j + 0.05 * k)
        assert np.isclose(t[k, j, i], want, rtol=1e-13, atol=1e-13)
    assert np.all(t[fixed] == 0.0) and fixed.any()
    # a corner node touches one element
    assert np.isclose(t[8, 8, 8], 2.0 * u[7, 7, 7])
    assert np.array_equal(unet.node_counts(prob)[[0, 4, 8], 4, 4], [4.0, 8.0, 4.0])


def test_input_channels():
    prob = W.tiny_3d(8, 8, 8, 3)
    x = np.full(prob.nelem, 0.4)
    qe = W.quadrant_source(prob) if prob.dim == 2 else W.element_source(prob)
    inp = unet.net_input(prob, x, qe)
    assert inp.shape == (3, 8, 8, 8)
    assert np.allclose(inp[0], 0.4) and np.allclose(inp[2], 1.0)
    # fraction of Dirichlet corners, counted by brute force
    lo, hi = prob.fix_lo, prob.fix_hi
    for (k, j, i) in [(0, 3, 3), (0, 0, 0), (1, 3, 3), (0, 4, 4)]:
        cnt = sum(lo[0] <= i + bx <= hi[0] and lo[1] <= j + by <= hi[1] and lo[2] <= k + bz <= hi[2]
                  for bx in (0, 1) for by in (0, 1) for bz in (0, 1))
        assert inp[1, k, j, i] == cnt / 8.0
    assert inp[1, 1:].max() == 0.0 and inp[1].max() > 0.0
    assert np.all(unet.net_input(prob, x, np.zeros(prob.nelem))[2] == 0.0)


def test_bf16_forward_is_close_to_fp64():
    prob = W.tiny_3d(8, 8, 8, 3)
    C = (16, 16, 16)
    theta = W.unet_init(C, seed=1)
    x = W.random_density(prob.nelem, 2, 0.0, 1.0)
    inp = unet.net_input(prob, x, W.element_source(prob))
    u64, _ = unet.forward(theta, inp, C)
    u16, _ = unet.forward(theta, inp, C, bf16=True)
    assert np.linalg.norm(u16 - u64) <= 2e-2 * np.linalg.norm(u64)
    assert not np.array_equal(u16, u64)


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = unet.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(t1, theta - 0.01 * np.sign(g), rtol=0, atol=1e-6)
    assert np.allclose(m, 0.1 * g, rtol=1e-7) and np.allclose(v, 0.001 * g * g, rtol=1e-7)
