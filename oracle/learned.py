"""Learned coarse correction: the small 3D convolutional network, its gradient, Adam, and the
guarded correction step it provides inside the velocity V-cycle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper has no learned component; everything below is a reading, stated in the design notes:

* level: the velocity multigrid level Q1 on N/2 elements per direction, M = N/2 + 1 nodes per
  direction, fields stored [component][z][y][x] (x fastest), like the velocity vectors;
* input x[b] with 4 channels on the M^3 node grid: channel 0 = (log10 mu)/5 with mu the mean of
  log10 over the Gauss points of each element, averaged over the elements that share the node;
  channels 1-3 = r / rho, rho = root mean square of the residual vector r over all 3 M^3 entries;
* network: 3x3x3 convolutions with zero padding, 4 -> H -> H -> H -> 3 channels, leaky ReLU
  (slope 0.1) after the first three; output o[b] with 3 channels;
* correction: delta = rho * o / d with d the Jacobi diagonal of the level operator (zero on
  Dirichlet nodes), then x <- x + alpha delta with alpha = (r, A delta) / (A delta, A delta)
  clipped to [0, 2]: the residual norm cannot grow, and alpha = 0 is the plain V-cycle;
* training pairs: e = (I - V A) e0 for random e0 (the error one plain V-cycle leaves), r = A e;
  target t = d e / rho (so that o ~ t), weight w = rho^2 / (d sum_j d_j e_j^2) (zero on
  Dirichlet nodes): sum_i w_i (o_i - t_i)^2 is the relative error of delta in the diagonally
  weighted norm;
* loss over a batch of B pairs: (1/B) sum_b sum_i w_i (o_i - t_i)^2; Adam (Kingma and Ba 2015)
  with bias correction.

Parameter blob (flat FP32), per layer l in order: W_l [Cout][Cin][27] then b_l [Cout]; tap
index t = dx + 3 dy + 9 dz (dx, dy, dz in {0, 1, 2}) multiplies the input at node offset
(dx - 1, dy - 1, dz - 1).

Parity status: conv3d pinned against a nested-loop sum and the adjoint identity; the backward
pass pinned by central finite differences; Adam pinned by its first step in closed form
(-lr * sign(g)); the node feature pinned on constant and two-valued fields.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.1


def layer_shapes(H: int):
    return [(4, H), (H, H), (H, H), (H, 3)]


def n_params(H: int) -> int:
    return sum(co * ci * 27 + co for ci, co in layer_shapes(H))


def unpack(params: np.ndarray, H: int):
    out, o = [], 0
    for ci, co in layer_shapes(H):
        W = params[o:o + co * ci * 27].reshape(co, ci, 27)
        o += co * ci * 27
        b = params[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(H: int, seed: int) -> np.ndarray:
    """He-style uniform initialization (used by tests only; the library draws its own)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in layer_shapes(H):
        lim = np.sqrt(6.0 / (ci * 27))
        parts.append(rng.uniform(-lim, lim, co * ci * 27))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def _taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield dx + 3 * dy + 9 * dz, dx, dy, dz


def conv3d(x, W, b):
    """y[b, o, z, y, x] = b[o] + sum_{c, taps} W[o, c, t] x[b, c, z+dz-1, y+dy-1, x+dx-1]
    (zero outside the grid)."""
    B, C, M = x.shape[0], x.shape[1], x.shape[2]
    xp = np.zeros((B, C, M + 2, M + 2, M + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    y = np.broadcast_to(b[None, :, None, None, None], (B, W.shape[0], M, M, M)).copy()
    for t, dx, dy, dz in _taps():
        xs = xp[:, :, dz:dz + M, dy:dy + M, dx:dx + M]
        y += np.einsum("oc,bczyx->bozyx", W[:, :, t], xs)
    return y


def conv3d_adjoint(gy, W):
    """Adjoint of conv3d in its input: gx[b, c, n] = sum_{o, t} W[o, c, t] gy[b, o, n - offset_t]."""
    B, M = gy.shape[0], gy.shape[2]
    C = W.shape[1]
    gp = np.zeros((B, W.shape[0], M + 2, M + 2, M + 2))
    gp[:, :, 1:-1, 1:-1, 1:-1] = gy
    gx = np.zeros((B, C, M, M, M))
    for t, dx, dy, dz in _taps():
        # input node n receives from output node n - (d - 1)
        gs = gp[:, :, 2 - dz:2 - dz + M, 2 - dy:2 - dy + M, 2 - dx:2 - dx + M]
        gx += np.einsum("oc,bozyx->bczyx", W[:, :, t], gs)
    return gx


def conv3d_wgrad(x, gy):
    """dW[o, c, t] = sum_{b, n} gy[b, o, n] x[b, c, n + offset_t]; db[o] = sum_{b, n} gy[b, o, n]."""
    B, C, M = x.shape[0], x.shape[1], x.shape[2]
    xp = np.zeros((B, C, M + 2, M + 2, M + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    dW = np.zeros((gy.shape[1], C, 27))
    for t, dx, dy, dz in _taps():
        xs = xp[:, :, dz:dz + M, dy:dy + M, dx:dx + M]
        dW[:, :, t] = np.einsum("bozyx,bczyx->oc", gy, xs)
    return dW, gy.sum(axis=(0, 2, 3, 4))


def leaky(z):
    return np.where(z > 0, z, SLOPE * z)


def forward(params, x, H, cache=False):
    layers = unpack(params, H)
    a, zs, acts = x, [], [x]
    for li, (W, b) in enumerate(layers):
        z = conv3d(a, W, b)
        zs.append(z)
        a = leaky(z) if li + 1 < len(layers) else z
        acts.append(a)
    return (a, zs, acts) if cache else a


def loss_and_grad(params, x, t, w, H):
    """Loss (1/B) sum w (o - t)^2 and its gradient with respect to the flat parameters."""
    B = x.shape[0]
    o, zs, acts = forward(params, x, H, cache=True)
    diff = o - t
    loss = float((w * diff * diff).sum() / B)
    g = 2.0 * w * diff / B
    layers = unpack(params, H)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        if li + 1 < len(layers):
            g = g * np.where(zs[li] > 0, 1.0, SLOPE)
        dW, db = conv3d_wgrad(acts[li], g)
        grads[li] = (dW, db)
        if li > 0:
            g = conv3d_adjoint(g, layers[li][0])
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new params, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def node_log_mu(coef_q: np.ndarray, N: int) -> np.ndarray:
    """Channel 0 of the input on a Q1 level with N elements per direction: the element mean of
    log10(coef) over its Gauss points, averaged over the elements sharing each node, / 5.
    coef_q: [E][8] with e = ex + N (ey + N ez)."""
    M = N + 1
    em = np.log10(coef_q).mean(axis=1).reshape(N, N, N)     # [ez][ey][ex]
    s = np.zeros((M, M, M))
    c = np.zeros((M, M, M))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                s[dz:dz + N, dy:dy + N, dx:dx + N] += em
                c[dz:dz + N, dy:dy + N, dx:dx + N] += 1
    return (s / c / 5.0).reshape(-1)


def net_input(feat: np.ndarray, r: np.ndarray, M: int):
    """x [1][4][M][M][M] and rho from the node feature [M^3] and the residual [3][M^3]."""
    rho = float(np.sqrt(np.mean(r * r)))
    x = np.empty((1, 4, M, M, M))
    x[0, 0] = feat.reshape(M, M, M)
    x[0, 1:] = (r / rho).reshape(3, M, M, M) if rho > 0 else 0.0
    return x, rho


def guarded_correction(A, d, feat, r, params, H, M):
    """delta = rho o / d (zero where d = 0), alpha = clip((r, A delta)/(A delta, A delta), 0, 2).
    A acts on the full [3 M^3] vector (Dirichlet rows and columns zero)."""
    x, rho = net_input(feat, r, M)
    if rho == 0.0:
        return np.zeros_like(r), 0.0
    o = forward(params, x, H)[0].reshape(-1)
    delta = np.where(d > 0, rho * o / np.where(d > 0, d, 1.0), 0.0)
    Ad = A @ delta
    den = float(Ad @ Ad)
    alpha = 0.0 if den <= 0 else min(max(float(r @ Ad) / den, 0.0), 2.0)
    return delta, alpha
