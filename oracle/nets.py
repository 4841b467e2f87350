"""Oracle for the learned initial guess: a small 3D convolutional network.

Test infrastructure only (see the package docstring). The paper has no
learned component; this module fixes, in plain FP64 NumPy, what the GPU's
seed network computes, so that its forward pass, its gradients and its Adam
step can be checked element by element.

Network ("seed net"), on a coarse cell grid of D x H x W cells, each cell a
block of f^3 finest elements (f = pool factor):

  input   2 channels: mean physical density of the block; fraction of the
          block's 8 corner nodes (finest-grid nodes f*i, f*(i+1), ...) that
          are Dirichlet nodes
  c1      conv 3x3x3 (2 -> C1) + ReLU
  c2      conv 3x3x3 (C1 -> C1) + ReLU                 -> skip s
  pool    2x2x2 average                                  (D/2 x H/2 x W/2)
  c3      conv 3x3x3 (C1 -> C2) + ReLU
  c4      conv 3x3x3 (C2 -> C2) + ReLU
  up      2x nearest-neighbour upsampling
  cat     [up, s]                                       (C2 + C1 channels)
  c5      conv 3x3x3 (C2 + C1 -> C1) + ReLU
  c6      conv 3x3x3 (C1 -> 1)                          -> u (D x H x W)

Convolutions are cross-correlations with zero padding 1, weights indexed
w[co, ci, dz, dy, dx] and one bias per output channel. Arrays are
[channel, z, y, x].

Prediction on the finest nodes: T(node) = scale * trilinear interpolation of
u between coarse cell centres, which sit on the finest nodes f*i + f/2 (node
units), clamped to the outermost centres; Dirichlet nodes get 0. Training
target: y[c] = T(centre node of c) / scale; loss = mean over cells of
(u - y)^2. The scale is the max-norm of the pair's previous temperature.
Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps)
with bias corrections mhat = m / (1 - b1^t), vhat = v / (1 - b2^t).
"""
from __future__ import annotations

import numpy as np

LAYERS = ("c1", "c2", "c3", "c4", "c5", "c6")


def layer_shapes(c1: int, c2: int):
    """(co, ci) of every convolution."""
    return {"c1": (c1, 2), "c2": (c1, c1), "c3": (c2, c1), "c4": (c2, c2), "c5": (c1, c2 + c1),
            "c6": (1, c1)}


def param_layout(c1: int, c2: int):
    """Flat parameter vector: per layer, weights (co*ci*27, [co][ci][dz][dy][dx])
    then biases (co), layers in order c1..c6. Returns [(name, w_off, w_len, b_off, co, ci)]."""
    out, off = [], 0
    for name in LAYERS:
        co, ci = layer_shapes(c1, c2)[name]
        out.append((name, off, co * ci * 27, off + co * ci * 27, co, ci))
        off += co * ci * 27 + co
    return out, off


def unpack(theta, c1, c2):
    lay, _ = param_layout(c1, c2)
    P = {}
    for name, wo, wl, bo, co, ci in lay:
        P[name] = (theta[wo:wo + wl].reshape(co, ci, 3, 3, 3), theta[bo:bo + co])
    return P


def pack_grads(G, c1, c2):
    lay, n = param_layout(c1, c2)
    g = np.zeros(n)
    for name, wo, wl, bo, co, ci in lay:
        gw, gb = G[name]
        g[wo:wo + wl] = gw.ravel()
        g[bo:bo + co] = gb
    return g


def conv3d(x, w, b):
    """Zero-padded 3x3x3 cross-correlation: out[o] = b[o] + sum_{c,d} w[o,c,d] x[c, . + d - 1]."""
    C, D, H, W = x.shape
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], D, H, W))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx], xp[:, dz:dz + D, dy:dy + H, dx:dx + W])
    return out + b[:, None, None, None]


def conv3d_backward(x, w, gout):
    """Gradients of conv3d wrt its input, weights and bias, from the output gradient."""
    C, D, H, W = x.shape
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = (slice(None), slice(dz, dz + D), slice(dy, dy + H), slice(dx, dx + W))
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gout, xp[sl])
                gxp[sl] += np.einsum("oc,ozyx->czyx", w[:, :, dz, dy, dx], gout)
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gout.sum(axis=(1, 2, 3))


def pool2(x):
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool2_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(g):
    C, D, H, W = g.shape
    return g.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


def forward(theta, inp, c1, c2):
    """Network output u (D, H, W) and the activations needed by backward."""
    P = unpack(theta, c1, c2)
    a = {"in": inp}
    a["c1"] = np.maximum(conv3d(inp, *P["c1"]), 0.0)
    a["c2"] = np.maximum(conv3d(a["c1"], *P["c2"]), 0.0)
    a["pool"] = pool2(a["c2"])
    a["c3"] = np.maximum(conv3d(a["pool"], *P["c3"]), 0.0)
    a["c4"] = np.maximum(conv3d(a["c3"], *P["c4"]), 0.0)
    a["cat"] = np.concatenate([up2(a["c4"]), a["c2"]], axis=0)
    a["c5"] = np.maximum(conv3d(a["cat"], *P["c5"]), 0.0)
    a["u"] = conv3d(a["c5"], *P["c6"])[0]
    return a["u"], a


def loss_and_grad(theta, inp, y, c1, c2):
    """MSE loss of the output against y and its gradient wrt the flat parameters."""
    P = unpack(theta, c1, c2)
    u, a = forward(theta, inp, c1, c2)
    n = u.size
    loss = float(np.sum((u - y) ** 2) / n)
    g = (2.0 / n) * (u - y)[None]
    G = {}
    g, G["c6"] = _bw(a["c5"], P["c6"], g, relu_out=None)
    g = g * (a["c5"] > 0)
    g, G["c5"] = _bw(a["cat"], P["c5"], g, relu_out=None)
    gup, gskip = g[:c2], g[c2:]
    g = up2_backward(gup) * (a["c4"] > 0)
    g, G["c4"] = _bw(a["c3"], P["c4"], g, relu_out=None)
    g = g * (a["c3"] > 0)
    g, G["c3"] = _bw(a["pool"], P["c3"], g, relu_out=None)
    g = pool2_backward(g) + gskip
    g = g * (a["c2"] > 0)
    g, G["c2"] = _bw(a["c1"], P["c2"], g, relu_out=None)
    g = g * (a["c1"] > 0)
    _, G["c1"] = _bw(a["in"], P["c1"], g, relu_out=None)
    return loss, pack_grads(G, c1, c2)


def _bw(x, wb, gout, relu_out=None):
    gx, gw, gb = conv3d_backward(x, wb[0], gout)
    return gx, (gw, gb)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- grid <-> network

def net_input(prob, xphys, f):
    """The two input channels on the coarse cell grid of pool factor f."""
    nx, ny, nz = prob.nelx, prob.nely, prob.nelz
    W, H, D = nx // f, ny // f, nz // f
    rho = np.asarray(xphys, float).reshape(nz, ny, nx)
    ch0 = rho.reshape(D, f, H, f, W, f).mean(axis=(1, 3, 5))
    lo, hi = prob.fix_lo, prob.fix_hi
    ch1 = np.zeros((D, H, W))
    for k in range(D):
        for j in range(H):
            for i in range(W):
                cnt = 0
                for c in range(8):
                    ni, nj, nk = f * (i + (c & 1)), f * (j + ((c >> 1) & 1)), f * (k + ((c >> 2) & 1))
                    cnt += (lo[0] <= ni <= hi[0]) and (lo[1] <= nj <= hi[1]) and (lo[2] <= nk <= hi[2])
                ch1[k, j, i] = cnt / 8.0
    return np.stack([ch0, ch1])


def net_target(prob, t_full, f, scale):
    """y[c] = T at the centre node of coarse cell c, divided by scale."""
    nnx, nny = prob.nelx + 1, prob.nely + 1
    W, H, D = prob.nelx // f, prob.nely // f, prob.nelz // f
    T = np.asarray(t_full, float).reshape(prob.nelz + 1, nny, nnx)
    h = f // 2
    return T[h::f, h::f, h::f][:D, :H, :W] / scale


def net_to_nodes(prob, u, f, scale):
    """Finest-node field from the coarse output: trilinear between cell
    centres (node f*i + f/2), clamped at the outermost centres, Dirichlet 0."""
    D, H, W = u.shape
    axes = []
    for n_nodes, ncell in ((prob.nelz + 1, D), (prob.nely + 1, H), (prob.nelx + 1, W)):
        pos = (np.arange(n_nodes) - f / 2.0) / f          # position in cell-centre units
        pos = np.clip(pos, 0.0, ncell - 1.0)
        i0 = np.minimum(np.floor(pos).astype(int), ncell - 1)
        i1 = np.minimum(i0 + 1, ncell - 1)
        axes.append((i0, i1, pos - i0))
    (z0, z1, wz), (y0, y1, wy), (x0, x1, wx) = axes
    out = np.zeros((prob.nelz + 1, prob.nely + 1, prob.nelx + 1))
    for a, za, wa in ((0, z0, 1 - wz), (1, z1, wz)):
        for b, yb, wb in ((0, y0, 1 - wy), (1, y1, wy)):
            for c, xc, wc in ((0, x0, 1 - wx), (1, x1, wx)):
                out += (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) * \
                    u[za[:, None, None], yb[None, :, None], xc[None, None, :]]
    out *= scale
    lo, hi = prob.fix_lo, prob.fix_hi
    out[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = 0.0
    return out.ravel()
