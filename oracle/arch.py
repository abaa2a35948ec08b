"""Architecture descriptors and the canonical flat weight-blob layout (FP64 oracle).

Test infrastructure only (see the package docstring).

The paper describes its classifier as a modified WaveNet that reads the two
detector strains sampled at 4096 Hz and emits a classification probability per
time step (Materials and Methods, "AI architecture"; Fig. 1). It gives no
widths, depths or kernel sizes, so this package fixes two concrete members:

kind 0, "plain stack": four causal convolutions, kernel 2, dilations 1, 2, 4, 8,
    16 channels, ReLU after each, then a 1x1 convolution to one channel; the
    per-timestep probability is the sigmoid of that logit.
kind 1, "gated residual WaveNet": a 1x1 input projection 2 -> C, then
    n_stacks x layers_per_stack gated residual layers (kernel 2, dilation
    2**(l mod layers_per_stack)), each with a tanh*sigmoid gate and residual
    and skip 1x1 convolutions; the skip sum goes through ReLU, a 1x1 to H
    channels, an optional ReLU, a 1x1 to one channel, then the sigmoid.

kind 2, "two-branch" (the paper's Fig. 1): one gated residual WaveNet per
    detector (Hanford, Livingston), each reading its own channel through a
    1x1 input projection 1 -> C, with its own n_stacks x layers_per_stack
    gated layers and its own skip sum of S channels; the two skip sums are
    concatenated (2S channels, Hanford first) and go through the same head as
    kind 1 (ReLU, 1x1 to H, optional ReLU, 1x1 to one channel).

Readings where the paper is silent (all listed in the design notes):
  * the input layer is a 1x1 convolution with bias (input_kernel=1), so the
    receptive field is 1 + (kernel-1) * sum of dilations;
  * the last gated layer has no residual 1x1 (its output would be unused);
  * kernel taps: W[..., 0] multiplies x[t - d], W[..., 1] multiplies x[t];
  * gate split: channels [0, C) feed tanh, [C, 2C) feed the sigmoid;
  * head_mid_relu=0: no nonlinearity between the two head 1x1s (the literal
    configuration); 1 inserts a ReLU there (the usual WaveNet head).

Blob layout (per member, float, in this order):
  kind 0: for i = 1..4: conv_i.W[16][Cin][2], conv_i.b[16]  (Cin = 2, then 16)
          out.W[1][16], out.b[1]
  kind 1: in.W[C][2] (or [C][2][2] when input_kernel=2), in.b[C]
          for l = 0..L-1: dil.W[2C][C][2], dil.b[2C],
                          res.W[C][C], res.b[C]      (absent for l = L-1)
                          skip.W[S][C], skip.b[S]
          h1.W[H][S], h1.b[H], h2.W[1][H], h2.b[1]
  kind 2: for branch b = 0 (Hanford), 1 (Livingston): the kind-1 tensors from
          in.W[C][1] through the last skip.b[S], prefixed "b<b>."
          h1.W[H][2S], h1.b[H], h2.W[1][H], h2.b[1]
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class Arch:
    kind: int = 1                 # 0 plain ReLU stack, 1 gated residual WaveNet, 2 two-branch
    in_channels: int = 2          # Hanford, Livingston
    channels: int = 128           # residual channels (kind 1) / conv channels (kind 0)
    skip_channels: int = 128
    head_channels: int = 128
    n_stacks: int = 3
    layers_per_stack: int = 10
    kernel_size: int = 2
    input_kernel: int = 1
    head_mid_relu: int = 0

    @property
    def n_layers(self) -> int:
        return self.n_stacks * self.layers_per_stack

    def dilation(self, l: int) -> int:
        return 2 ** (l % self.layers_per_stack)


# The two members used throughout: the small parity model and the full-size member.
TINY = Arch(kind=0, in_channels=2, channels=16, skip_channels=0, head_channels=0,
            n_stacks=1, layers_per_stack=4, kernel_size=2, input_kernel=1, head_mid_relu=0)
FULL = Arch()
# The paper's two-branch topology at the same total width: two 64-channel branches whose skip sums
# concatenate to the 128 channels the head reads.
TWO_BRANCH = Arch(kind=2, in_channels=2, channels=64, skip_channels=64, head_channels=128)


def branch_arch(a: Arch) -> Arch:
    """The single-detector gated member one branch of a kind-2 member is."""
    return Arch(kind=1, in_channels=1, channels=a.channels, skip_channels=a.skip_channels,
                head_channels=a.head_channels, n_stacks=a.n_stacks, layers_per_stack=a.layers_per_stack,
                kernel_size=a.kernel_size, input_kernel=a.input_kernel, head_mid_relu=a.head_mid_relu)


def layout(a: Arch) -> List[Tuple[str, Tuple[int, ...], int]]:
    """Ordered list of (name, shape, fan_in) for every tensor of the blob.

    fan_in is the He-normal fan-in (C_in * kernel) for weights and 0 for biases.
    """
    out: List[Tuple[str, Tuple[int, ...], int]] = []
    k = a.kernel_size
    if a.kind == 0:
        cin = a.in_channels
        for i in range(a.n_layers):
            out.append((f"conv{i}.W", (a.channels, cin, k), cin * k))
            out.append((f"conv{i}.b", (a.channels,), 0))
            cin = a.channels
        out.append(("out.W", (1, a.channels), a.channels))
        out.append(("out.b", (1,), 0))
        return out
    if a.kind == 2:
        trunk = [t for t in layout(branch_arch(a)) if not t[0].startswith("h")]
        for br in range(2):
            out += [(f"b{br}.{name}", shape, fan) for name, shape, fan in trunk]
        S2, H = 2 * a.skip_channels, a.head_channels
        return out + [("h1.W", (H, S2), S2), ("h1.b", (H,), 0), ("h2.W", (1, H), H), ("h2.b", (1,), 0)]
    C, S, H = a.channels, a.skip_channels, a.head_channels
    if a.input_kernel == 1:
        out.append(("in.W", (C, a.in_channels), a.in_channels))
    else:
        out.append(("in.W", (C, a.in_channels, a.input_kernel), a.in_channels * a.input_kernel))
    out.append(("in.b", (C,), 0))
    for l in range(a.n_layers):
        out.append((f"dil{l}.W", (2 * C, C, k), C * k))
        out.append((f"dil{l}.b", (2 * C,), 0))
        if l < a.n_layers - 1:
            out.append((f"res{l}.W", (C, C), C))
            out.append((f"res{l}.b", (C,), 0))
        out.append((f"skip{l}.W", (S, C), C))
        out.append((f"skip{l}.b", (S,), 0))
    out.append(("h1.W", (H, S), S))
    out.append(("h1.b", (H,), 0))
    out.append(("h2.W", (1, H), H))
    out.append(("h2.b", (1,), 0))
    return out


def num_params(a: Arch) -> int:
    return int(sum(int(np.prod(s)) for _, s, _ in layout(a)))


def receptive_field(a: Arch) -> int:
    """Number of input samples that influence one output sample (causal)."""
    rf = 1 + (a.kernel_size - 1) * sum(a.dilation(l) for l in range(a.n_layers))
    if a.kind in (1, 2):
        rf += a.input_kernel - 1
    return rf


def unpack(a: Arch, blob: np.ndarray) -> Dict[str, np.ndarray]:
    """Split one member's flat blob into named float64 arrays (copies)."""
    blob = np.asarray(blob, dtype=np.float64).reshape(-1)
    n = num_params(a)
    if blob.size != n:
        raise ValueError(f"blob has {blob.size} values, architecture needs {n}")
    p: Dict[str, np.ndarray] = {}
    off = 0
    for name, shape, _ in layout(a):
        cnt = int(np.prod(shape))
        p[name] = blob[off:off + cnt].reshape(shape).copy()
        off += cnt
    return p


def pack(a: Arch, params: Dict[str, np.ndarray]) -> np.ndarray:
    """Inverse of unpack: named arrays -> flat float64 blob in canonical order."""
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1)
                           for name, _, _ in layout(a)])


def two_branch_blocks(a: Arch):
    """(branch tensor name, its index, trunk tensor name, trunk index) for every tensor of a kind-2
    member: where it sits in the single trunk of twice the width that the member equals when that
    trunk's weights are block-diagonal (branch b owns residual and skip channels [bC, (b+1)C), the
    same slice of each half of the dilated output, and input channel b). The head is shared."""
    C, S = a.channels, a.skip_channels
    out = []
    for b in range(2):
        r, sk = slice(b * C, (b + 1) * C), slice(b * S, (b + 1) * S)
        out.append((f"b{b}.in.W", (slice(None), 0), "in.W", (r, b)))
        out.append((f"b{b}.in.b", (slice(None),), "in.b", (r,)))
        for l in range(a.n_layers):
            for half in range(2):
                hs = slice(half * C, (half + 1) * C)
                o = slice(half * 2 * C + b * C, half * 2 * C + (b + 1) * C)
                out.append((f"b{b}.dil{l}.W", (hs,), f"dil{l}.W", (o, r)))
                out.append((f"b{b}.dil{l}.b", (hs,), f"dil{l}.b", (o,)))
            if l < a.n_layers - 1:
                out.append((f"b{b}.res{l}.W", (slice(None),), f"res{l}.W", (r, r)))
                out.append((f"b{b}.res{l}.b", (slice(None),), f"res{l}.b", (r,)))
            out.append((f"b{b}.skip{l}.W", (slice(None),), f"skip{l}.W", (sk, r)))
            out.append((f"b{b}.skip{l}.b", (slice(None),), f"skip{l}.b", (sk,)))
    for n in ("h1.W", "h1.b", "h2.W", "h2.b"):
        out.append((n, (slice(None),), n, (slice(None),)))
    return out


def two_branch_trunk_arch(a: Arch) -> Arch:
    return Arch(kind=1, in_channels=2, channels=2 * a.channels, skip_channels=2 * a.skip_channels,
                head_channels=a.head_channels, n_stacks=a.n_stacks, layers_per_stack=a.layers_per_stack,
                kernel_size=a.kernel_size, input_kernel=a.input_kernel, head_mid_relu=a.head_mid_relu)


def two_branch_as_trunk(a: Arch, p: Dict[str, np.ndarray]):
    """(trunk arch, trunk params) of the block-diagonal trunk a kind-2 member equals."""
    t = two_branch_trunk_arch(a)
    q = {n: np.zeros(s) for n, s, _ in layout(t)}
    for bn, bi, tn, ti in two_branch_blocks(a):
        q[tn][ti] = p[bn][bi]
    return t, q

