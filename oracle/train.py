"""Per-timestep BCE loss, its gradient by manual reverse mode, and Adam (oracle).

Test infrastructure only (see the package docstring).

The paper trains each member as a per-timestep binary classifier ("AI ensemble
construction": every time step is labelled "waveform" or "noise") with random
weight initialisation. Reading for the training form here: label 1 within
+/-0.1 s of the injected coalescence time, else 0; loss = mean over all
windows and time steps of the binary cross-entropy on logits,
    softplus(z) - y z,
whose derivative is (sigmoid(z) - y) / N. Adam (Kingma & Ba) with bias
correction, no weight decay, no clipping.

The gradient is written out layer by layer from the forward definitions in
`oracle.forward` (chain rule, in reverse order), not by automatic differentiation.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .arch import Arch, layout, pack, two_branch_as_trunk, two_branch_blocks, unpack
from .forward import causal_conv, gated_layer, input_projection, relu, shift_right, sigmoid


def bce_logits(z: np.ndarray, y: np.ndarray) -> float:
    """Mean of softplus(z) - y z over every element."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    softplus = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(softplus - y * z))


def bce_grad(z: np.ndarray, y: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    return (sigmoid(z) - np.asarray(y, dtype=np.float64)) / z.size


def _conv_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray, d: int):
    """Reverse of y[t] = b + sum_j W[:, :, j] x[t - (k-1-j) d].

    Returns (dx, dW, db) with dx[t] = sum_j dy[t + (k-1-j) d] W[:, :, j].
    """
    k = W.shape[2]
    T = x.shape[-2]
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    flat_dy = dy.reshape(-1, dy.shape[-1])
    for j in range(k):
        s = (k - 1 - j) * d
        xs = shift_right(x, s)
        dW[:, :, j] = flat_dy.T @ xs.reshape(-1, xs.shape[-1])
        # dy shifted left by s: dy_l[t] = dy[t + s], zero past the end
        dyl = np.zeros_like(dy)
        if s < T:
            dyl[..., :T - s, :] = dy[..., s:, :]
        dx += dyl @ np.ascontiguousarray(W[:, :, j])
    db = flat_dy.sum(axis=0)
    return dx, dW, db


def loss_and_grad(a: Arch, blob: np.ndarray, u: np.ndarray, y: np.ndarray
                  ) -> Tuple[float, np.ndarray, np.ndarray]:
    """(loss, d loss / d blob [n_params], d loss / d u) for windows u [B, T, 2] and labels y [B, T]."""
    if a.kind == 2:
        # the member equals its block-diagonal trunk, whose weights are a linear (selection) image of
        # the branch tensors: the branch gradient is the trunk gradient read back at those positions
        p2 = unpack(a, blob)
        t, q = two_branch_as_trunk(a, p2)
        loss, gt, du = loss_and_grad(t, pack(t, q), u, y)
        gq = unpack(t, gt)
        gb = {n: np.zeros(s) for n, s, _ in layout(a)}
        for bn, bi, tn, ti in two_branch_blocks(a):
            gb[bn][bi] = gq[tn][ti]
        return loss, pack(a, gb), du
    p = unpack(a, blob)
    u = np.asarray(u, dtype=np.float64)
    g: Dict[str, np.ndarray] = {}

    def rows(v):
        return v.reshape(-1, v.shape[-1])

    if a.kind == 0:
        ys = [u]
        for i in range(a.n_layers):
            ys.append(relu(causal_conv(ys[-1], p[f"conv{i}.W"], p[f"conv{i}.b"], a.dilation(i))))
        z = (ys[-1] @ p["out.W"].T + p["out.b"])[..., 0]
        loss = bce_logits(z, y)
        dz = bce_grad(z, y)[..., None]
        g["out.W"] = rows(dz).T @ rows(ys[-1])
        g["out.b"] = rows(dz).sum(axis=0)
        dy = dz @ p["out.W"]
        for i in reversed(range(a.n_layers)):
            dpre = dy * (ys[i + 1] > 0)
            dy, g[f"conv{i}.W"], g[f"conv{i}.b"] = _conv_backward(ys[i], p[f"conv{i}.W"], dpre, a.dilation(i))
        du = dy
    else:
        C = a.channels
        x = input_projection(a, p, u)
        xs, pres, gs = [], [], []
        skip = np.zeros(x.shape[:-1] + (a.skip_channels,))
        for l in range(a.n_layers):
            xs.append(x)
            pre, gl, x, skip = gated_layer(a, p, l, x, skip)
            pres.append(pre)
            gs.append(gl)
        r = relu(skip)
        h = r @ p["h1.W"].T + p["h1.b"]
        hh = relu(h) if a.head_mid_relu else h
        z = (hh @ p["h2.W"].T + p["h2.b"])[..., 0]
        loss = bce_logits(z, y)
        dz = bce_grad(z, y)[..., None]
        g["h2.W"] = rows(dz).T @ rows(hh)
        g["h2.b"] = rows(dz).sum(axis=0)
        dh = dz @ p["h2.W"]
        if a.head_mid_relu:
            dh = dh * (h > 0)
        g["h1.W"] = rows(dh).T @ rows(r)
        g["h1.b"] = rows(dh).sum(axis=0)
        dskip = (dh @ p["h1.W"]) * (skip > 0)
        dx_next = np.zeros_like(x)          # the head does not read the residual stream
        for l in reversed(range(a.n_layers)):
            gl, pre = gs[l], pres[l]
            dg = dskip @ p[f"skip{l}.W"]
            g[f"skip{l}.W"] = rows(dskip).T @ rows(gl)
            g[f"skip{l}.b"] = rows(dskip).sum(axis=0)
            if l < a.n_layers - 1:
                dg = dg + dx_next @ p[f"res{l}.W"]
                g[f"res{l}.W"] = rows(dx_next).T @ rows(gl)
                g[f"res{l}.b"] = rows(dx_next).sum(axis=0)
            th = np.tanh(pre[..., :C])
            sg = sigmoid(pre[..., C:])
            dpre = np.concatenate([dg * sg * (1.0 - th * th), dg * th * sg * (1.0 - sg)], axis=-1)
            dxc, g[f"dil{l}.W"], g[f"dil{l}.b"] = _conv_backward(xs[l], p[f"dil{l}.W"], dpre, a.dilation(l))
            # residual identity path: x_{l+1} = x_l + ...; for the last layer x_{l+1} = x_l too
            dx_next = dx_next + dxc
        dx0 = dx_next
        if a.input_kernel == 1:
            g["in.W"] = rows(dx0).T @ rows(u)
            g["in.b"] = rows(dx0).sum(axis=0)
            du = dx0 @ p["in.W"]
        else:
            du, g["in.W"], g["in.b"] = _conv_backward(u, p["in.W"], dx0, 1)
    grad = np.concatenate([g[name].reshape(-1) for name, _, _ in layout(a)])
    return loss, grad, du


def loss_only(a: Arch, blob: np.ndarray, u: np.ndarray, y: np.ndarray) -> float:
    from .forward import forward_window
    return bce_logits(forward_window(a, unpack(a, blob), u), y)


def adam_step(w: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, step: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update at 1-based step `step`; returns (w, m, v) as new arrays."""
    grad = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    w = np.asarray(w, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return w, m, v
