"""Oracle for the learned initial guess: a 3D convolutional U-Net on the element grid.

TEST INFRASTRUCTURE ONLY (see the package docstring). The paper has no learned
component; this module fixes, in plain NumPy, what the GPU's seed network
computes, so that its forward pass, gradients and Adam step can be checked
element by element. Everything is FP64 unless ``bf16=True``, in which case
the values the GPU stores in BF16 are rounded to BF16 at the same points
(``bf16r``); the arithmetic between those points stays FP64.

Network on the element grid (nz, ny, nx), L levels with channels C[0..L-1]
(arrays are [channel, z, y, x]; level l has n / 2^l elements per axis):

  input  3 channels per element: physical density; fraction of the
         element's 8 corner nodes that are Dirichlet nodes; element heat
         source divided by the largest |source| (0 for a zero source)
  encoder, level l = 0 .. L-1:
         e_l = relu(conv(x_l)), s_l = relu(conv(e_l))      (x_0 = input,
         x_l = pool(s_(l-1)) for l >= 1); s_(L-1) is the bottom
  decoder, level l = L-2 .. 0:
         cat = [up(d_(l+1)), s_l]  (up channels first; d_(L-1) = s_(L-1))
         d_l = relu(conv(relu(conv(cat))))
  head   u = w . d_0 + b (1x1x1 convolution to one channel, linear)

conv: 3x3x3 zero-padded cross-correlation with one bias per output channel,
weights w[co, ci, dz, dy, dx]. pool: mean over 2x2x2 children. up: trilinear
2x upsampling of cell-centred values (fine cell f sits at coarse coordinate
(f + 1/2)/2 - 1/2 on each axis, coordinates clamped to the coarse range),
which is PyTorch's trilinear interpolation with align_corners=False.

Prediction on the finest nodes: T(node) = scale * mean of u over the
elements that touch the node; 0 on Dirichlet nodes. Training pair (xphys, T,
scale): y = T / scale, loss = mean over the free nodes of (T/scale - y)^2
with T the prediction. The scale is the max-norm of the pair's previous
temperature (the temperature the loop had before this design's solve).

BF16 rounding points of the GPU (bf16=True): the input channels; every
convolution weight; every stored activation (after ReLU, after pooling, after
upsampling); the gradient of every stored activation (after each
transposed convolution, after the upsampling adjoint, after adding the
pooling adjoint into a skip gradient, and the head's data gradient). Sums
inside a convolution are FP32 on the GPU (FP64 here); the head, the node
averaging, the loss and the weight-gradient reductions are not rounded.

Adam (per parameter, step t >= 1, on FP32-stored parameters and moments):
m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps),
mhat = m / (1 - b1^t), vhat = v / (1 - b2^t), evaluated in FP64 and stored
as FP32.
"""
from __future__ import annotations

import numpy as np

CIN = 3


def bf16r(x):
    """Round to BF16 (nearest even) through FP32, returned as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- layout

def layer_list(C):
    """(name, co, ci, k) of every layer in parameter order: encoder convs,
    decoder convs, head (k = kernel edge)."""
    L = len(C)
    out = []
    for l in range(L):
        out.append((f"e{l}a", C[l], CIN if l == 0 else C[l - 1], 3))
        out.append((f"e{l}b", C[l], C[l], 3))
    for l in range(L - 2, -1, -1):
        out.append((f"d{l}a", C[l], C[l + 1] + C[l], 3))
        out.append((f"d{l}b", C[l], C[l], 3))
    out.append(("head", 1, C[0], 1))
    return out


def param_layout(C):
    """Flat parameter vector: per layer its weights ([co][ci][k][k][k]) then
    its co biases, layers in layer_list order. Returns ([(name, w_off, w_len,
    b_off, co, ci, k)], total)."""
    out, off = [], 0
    for name, co, ci, k in layer_list(C):
        wl = co * ci * k ** 3
        out.append((name, off, wl, off + wl, co, ci, k))
        off += wl + co
    return out, off


def unpack(theta, C):
    lay, _ = param_layout(C)
    P = {}
    for name, wo, wl, bo, co, ci, k in lay:
        P[name] = (np.asarray(theta[wo:wo + wl], float).reshape(co, ci, k, k, k),
                   np.asarray(theta[bo:bo + co], float))
    return P


def pack(G, C):
    lay, n = param_layout(C)
    g = np.zeros(n)
    for name, wo, wl, bo, co, ci, k in lay:
        gw, gb = G[name]
        g[wo:wo + wl] = gw.ravel()
        g[bo:bo + co] = gb
    return g


# ---------------------------------------------------------------- operators

def conv3d(x, w, b):
    """Zero-padded 3x3x3 correlation: out[o] = b[o] + sum_{c,d} w[o,c,d] x[c, . + d - 1]."""
    C, D, H, W = x.shape
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], D, H, W))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx], xp[:, dz:dz + D, dy:dy + H, dx:dx + W])
    return out + b[:, None, None, None]


def conv3d_input_grad(w, gout):
    """Gradient of conv3d with respect to its input."""
    Co, D, H, W = gout.shape
    gxp = np.zeros((w.shape[1], D + 2, H + 2, W + 2))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                gxp[:, dz:dz + D, dy:dy + H, dx:dx + W] += np.einsum("oc,ozyx->czyx", w[:, :, dz, dy, dx], gout)
    return gxp[:, 1:-1, 1:-1, 1:-1]


def conv3d_weight_grad(x, gout):
    """Gradients of conv3d with respect to its weights and biases."""
    C, D, H, W = x.shape
    xp = np.zeros((C, D + 2, H + 2, W + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gw = np.zeros((gout.shape[0], C, 3, 3, 3))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gout, xp[:, dz:dz + D, dy:dy + H, dx:dx + W])
    return gw, gout.sum(axis=(1, 2, 3))


def pool2(x):
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool2_adjoint(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up_matrix(n):
    """(2n x n) matrix of 1D linear 2x upsampling of cell-centred values:
    fine cell f at coarse coordinate (f + 1/2)/2 - 1/2, clamped to [0, n-1]."""
    U = np.zeros((2 * n, n))
    for f in range(2 * n):
        c = min(max((f + 0.5) / 2.0 - 0.5, 0.0), n - 1.0)
        i0 = int(np.floor(c))
        i1 = min(i0 + 1, n - 1)
        t = c - i0
        U[f, i0] += 1.0 - t
        U[f, i1] += t
    return U


def up2(x):
    C, D, H, W = x.shape
    Uz, Uy, Ux = up_matrix(D), up_matrix(H), up_matrix(W)
    return np.einsum("Zz,Yy,Xx,czyx->cZYX", Uz, Uy, Ux, x)


def up2_adjoint(g):
    C, D2, H2, W2 = g.shape
    Uz, Uy, Ux = up_matrix(D2 // 2), up_matrix(H2 // 2), up_matrix(W2 // 2)
    return np.einsum("Zz,Yy,Xx,cZYX->czyx", Uz, Uy, Ux, g)


# ---------------------------------------------------------------- network

def forward(theta, inp, C, bf16=False):
    """Output u (nz, ny, nx) and the stored activations."""
    R = bf16r if bf16 else (lambda v: v)
    P = unpack(theta, C)
    L = len(C)
    a = {"in": R(inp)}

    def conv_relu(name, x):
        w, b = P[name]
        return R(np.maximum(conv3d(x, R(w), b), 0.0))

    x = a["in"]
    for l in range(L):
        if l > 0:
            x = a[f"p{l}"] = R(pool2(a[f"s{l - 1}"]))
        a[f"e{l}"] = conv_relu(f"e{l}a", x)
        a[f"s{l}"] = conv_relu(f"e{l}b", a[f"e{l}"])
    a[f"d{L - 1}"] = a[f"s{L - 1}"]
    for l in range(L - 2, -1, -1):
        a[f"u{l}"] = R(up2(a[f"d{l + 1}"]))
        a[f"cat{l}"] = np.concatenate([a[f"u{l}"], a[f"s{l}"]], axis=0)
        a[f"h{l}"] = conv_relu(f"d{l}a", a[f"cat{l}"])
        a[f"d{l}"] = conv_relu(f"d{l}b", a[f"h{l}"])
    wh, bh = P["head"]
    u = np.einsum("c,czyx->zyx", wh[0, :, 0, 0, 0], a["d0"]) + bh[0]
    return u, a


def backward(theta, a, du, C, bf16=False):
    """Gradient of the flat parameters from the output gradient du."""
    R = bf16r if bf16 else (lambda v: v)
    P = unpack(theta, C)
    L = len(C)
    G = {}
    wh, _ = P["head"]
    G["head"] = (np.einsum("zyx,czyx->c", du, a["d0"])[None, :, None, None, None], np.array([du.sum()]))
    g = R(wh[0, :, 0, 0, 0][:, None, None, None] * du[None])

    def conv_back(name, x_in, out, g_out, need_input=True):
        w, _ = P[name]
        gz = g_out * (out > 0)
        G[name] = conv3d_weight_grad(x_in, gz)
        return R(conv3d_input_grad(R(w), gz)) if need_input else None

    gskip = {}
    for l in range(L - 1):
        g = conv_back(f"d{l}b", a[f"h{l}"], a[f"d{l}"], g)
        gcat = conv_back(f"d{l}a", a[f"cat{l}"], a[f"h{l}"], g)
        cu = a[f"u{l}"].shape[0]
        gskip[l] = gcat[cu:]
        g = R(up2_adjoint(gcat[:cu]))
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            g = R(gskip[l] + g)
        g = conv_back(f"e{l}b", a[f"e{l}"], a[f"s{l}"], g)
        if l == 0:
            conv_back("e0a", a["in"], a["e0"], g, need_input=False)
        else:
            g = conv_back(f"e{l}a", a[f"p{l}"], a[f"e{l}"], g)
            g = pool2_adjoint(g)
    return pack(G, C)


# ---------------------------------------------------------------- grid <-> network

def net_input(prob, xphys, qe):
    """The three input channels on the element grid: density, fraction of
    Dirichlet corner nodes, source over its max-norm."""
    nx, ny, nz = prob.nelx, prob.nely, prob.nelz
    rho = np.asarray(xphys, float).reshape(nz, ny, nx)
    lo, hi = prob.fix_lo, prob.fix_hi
    fix = np.zeros((nz, ny, nx))
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        i = np.arange(nx) + bx
        j = np.arange(ny) + by
        k = np.arange(nz) + bz
        fi = (lo[0] <= i) & (i <= hi[0])
        fj = (lo[1] <= j) & (j <= hi[1])
        fk = (lo[2] <= k) & (k <= hi[2])
        fix += fk[:, None, None] & fj[None, :, None] & fi[None, None, :]
    q = np.asarray(qe, float).reshape(nz, ny, nx)
    qm = np.abs(q).max()
    src = q / qm if qm > 0 else np.zeros_like(q)
    return np.stack([rho, fix / 8.0, src])


def node_counts(prob):
    """Number of elements touching each node (nz+1, ny+1, nx+1)."""
    cnt = np.zeros((prob.nelz + 1, prob.nely + 1, prob.nelx + 1))
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cnt[bz:bz + prob.nelz, by:by + prob.nely, bx:bx + prob.nelx] += 1.0
    return cnt


def fixed_nodes(prob):
    lo, hi = prob.fix_lo, prob.fix_hi
    f = np.zeros((prob.nelz + 1, prob.nely + 1, prob.nelx + 1), bool)
    f[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    return f


def to_nodes(prob, u, scale):
    """Node field scale * (mean of u over the touching elements), 0 on Dirichlet nodes."""
    s = np.zeros((prob.nelz + 1, prob.nely + 1, prob.nelx + 1))
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        s[bz:bz + prob.nelz, by:by + prob.nely, bx:bx + prob.nelx] += u
    t = scale * s / node_counts(prob)
    t[fixed_nodes(prob)] = 0.0
    return t.ravel()


def loss_and_output_grad(prob, u, T, scale):
    """Loss (mean over free nodes of (prediction/scale - T/scale)^2) and its
    gradient with respect to u."""
    cnt = node_counts(prob)
    free = ~fixed_nodes(prob)
    nf = float(free.sum())
    yhat = to_nodes(prob, u, 1.0).reshape(cnt.shape)
    y = np.asarray(T, float).reshape(cnt.shape) / scale
    r = np.where(free, yhat - y, 0.0)
    loss = float(np.sum(r * r) / nf)
    gn = 2.0 * r / nf / cnt
    du = np.zeros_like(u)
    for c in range(8):
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        du += gn[bz:bz + prob.nelz, by:by + prob.nely, bx:bx + prob.nelx]
    return loss, du


def loss_and_grad(prob, theta, xphys, qe, T, scale, C, bf16=False):
    """Loss of one training pair and its gradient with respect to the flat parameters."""
    inp = net_input(prob, xphys, qe)
    u, a = forward(theta, inp, C, bf16)
    loss, du = loss_and_output_grad(prob, u, T, scale)
    if bf16:
        du = du.astype(np.float32).astype(np.float64)
    return loss, backward(theta, a, du, C, bf16)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1) on FP32-stored parameters and moments."""
    f32 = lambda z: np.asarray(z, np.float64).astype(np.float32).astype(np.float64)
    m = f32(b1 * np.asarray(m, float) + (1.0 - b1) * g)
    v = f32(b2 * np.asarray(v, float) + (1.0 - b2) * g * g)
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return f32(np.asarray(theta, float) - lr * mh / (np.sqrt(vh) + eps)), m, v
