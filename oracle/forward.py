"""Forward pass of one classifier member, float64 (oracle).

Test infrastructure only (see the package docstring).

Follows the paper's classifier description (Materials and Methods, "AI
architecture", Fig. 1: a WaveNet-style stack of dilated causal convolutions that
maps two-detector strain to one classification probability per time step) with
the concrete members and readings stated in `oracle.arch`.

Every window is an independent input with zero left context: the paper's
inference engine takes a batch of (1024, 4096, 2) windows and returns
(1024, 4096, 1) per-timestep outputs ("Optimization with TensorRT").
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from .arch import Arch, branch_arch


def sigmoid(z: np.ndarray) -> np.ndarray:
    """Logistic function 1 / (1 + exp(-z))."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def relu(v: np.ndarray) -> np.ndarray:
    return np.maximum(v, 0.0)


def shift_right(x: np.ndarray, d: int) -> np.ndarray:
    """Return y with y[..., t, :] = x[..., t - d, :] and zeros for t < d (causal delay along time)."""
    y = np.zeros_like(x)
    if d < x.shape[-2]:
        y[..., d:, :] = x[..., :x.shape[-2] - d, :]
    return y


def causal_conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, d: int) -> np.ndarray:
    """Dilated causal convolution along time.

    x: [..., T, Cin]; W: [Cout, Cin, k]; b: [Cout].
    y[t] = b + sum_j W[:, :, j] . x[t - (k-1-j) d], with x[tau < 0] = 0, so tap
    k-1 is the current sample and tap 0 the oldest.
    """
    k = W.shape[2]
    y = np.broadcast_to(b, x.shape[:-1] + (W.shape[0],)).astype(np.float64).copy()
    for j in range(k):
        # contiguous copy of the tap so the product goes through BLAS (a strided view would not)
        y += shift_right(x, (k - 1 - j) * d) @ np.ascontiguousarray(W[:, :, j]).T
    return y


def input_projection(a: Arch, p: Dict[str, np.ndarray], u: np.ndarray) -> np.ndarray:
    """x0 = W_in u + b_in (1x1 input layer), or a kernel-2 causal conv when input_kernel = 2."""
    if a.input_kernel == 1:
        return u @ p["in.W"].T + p["in.b"]
    return causal_conv(u, p["in.W"], p["in.b"], 1)


def gated_layer(a: Arch, p: Dict[str, np.ndarray], l: int, x: np.ndarray, skip: np.ndarray):
    """One gated residual layer l of the kind-1 member.

    Returns (pre, g, x_next, skip_next):
      pre    = dilated causal conv of x, [.., T, 2C]   (pre-activation)
      g      = tanh(pre[:, :C]) * sigmoid(pre[:, C:])  [.., T, C]
      skip_next = skip + W_s g + b_s
      x_next    = x + W_r g + b_r   (x unchanged for the last layer, which has no residual 1x1)
    """
    C = a.channels
    pre = causal_conv(x, p[f"dil{l}.W"], p[f"dil{l}.b"], a.dilation(l))
    g = np.tanh(pre[..., :C]) * sigmoid(pre[..., C:])
    skip_next = skip + g @ p[f"skip{l}.W"].T + p[f"skip{l}.b"]
    if l < a.n_layers - 1:
        x_next = x + g @ p[f"res{l}.W"].T + p[f"res{l}.b"]
    else:
        x_next = x
    return pre, g, x_next, skip_next


def head(a: Arch, p: Dict[str, np.ndarray], skip: np.ndarray) -> np.ndarray:
    """Logit per timestep: w_h2 . act(W_h1 ReLU(skip) + b_h1) + b_h2, act = ReLU or identity."""
    h = relu(skip) @ p["h1.W"].T + p["h1.b"]
    if a.head_mid_relu:
        h = relu(h)
    return (h @ p["h2.W"].T + p["h2.b"])[..., 0]


def forward_window(a: Arch, p: Dict[str, np.ndarray], u: np.ndarray,
                   capture: Optional[List[dict]] = None) -> np.ndarray:
    """Per-timestep logits z of one member for windows u.

    u: [..., T, 2] float (any leading batch dims); returns z: [..., T].
    The probability is sigmoid(z). If `capture` is a list, per-layer
    intermediates are appended to it (used for layer-local comparisons).
    """
    u = np.asarray(u, dtype=np.float64)
    if a.kind == 0:
        y = u
        for i in range(a.n_layers):
            y = relu(causal_conv(y, p[f"conv{i}.W"], p[f"conv{i}.b"], a.dilation(i)))
            if capture is not None:
                capture.append({"y": y})
        return (y @ p["out.W"].T + p["out.b"])[..., 0]
    if a.kind == 2:
        return forward_two_branch(a, p, u, capture)
    x = input_projection(a, p, u)
    skip = np.zeros(x.shape[:-1] + (a.skip_channels,))
    for l in range(a.n_layers):
        x_in = x
        pre, g, x, skip = gated_layer(a, p, l, x, skip)
        if capture is not None:
            capture.append({"x_in": x_in, "pre": pre, "g": g, "x_out": x, "skip": skip})
    return head(a, p, skip)


def branch_skip(a: Arch, p: Dict[str, np.ndarray], u: np.ndarray, br: int,
                capture: Optional[List[dict]] = None) -> np.ndarray:
    """Skip sum [..., T, S] of branch br of a kind-2 member, which reads detector channel br only."""
    ab = branch_arch(a)
    pre = f"b{br}."
    pb = {k[len(pre):]: v for k, v in p.items() if k.startswith(pre)}
    x = input_projection(ab, pb, u[..., br:br + 1])
    skip = np.zeros(x.shape[:-1] + (ab.skip_channels,))
    for l in range(ab.n_layers):
        x_in = x
        pre_act, g, x, skip = gated_layer(ab, pb, l, x, skip)
        if capture is not None:
            capture.append({"branch": br, "x_in": x_in, "pre": pre_act, "g": g, "x_out": x, "skip": skip})
    return skip


def forward_two_branch(a: Arch, p: Dict[str, np.ndarray], u: np.ndarray,
                       capture: Optional[List[dict]] = None) -> np.ndarray:
    """Kind-2 member: each detector through its own branch, the two skip sums concatenated
    (Hanford first), then the head."""
    s = np.concatenate([branch_skip(a, p, u, br, capture) for br in range(2)], axis=-1)
    return head(a, p, s)


def forward_stream(a: Arch, p: Dict[str, np.ndarray], u_stream: np.ndarray) -> np.ndarray:
    """One causal pass over a whole zero-left-padded stream u_stream [L, 2] -> z [L].

    Because every output depends only on the previous receptive-field samples,
    this equals the owner-window stitched output whenever RF - 1 <= W - S.
    """
    return forward_window(a, p, u_stream)
