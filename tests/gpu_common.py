"""Helpers for the GPU parity tests (inputs come from the seeded generator, expectations from the oracle)."""
import math

import numpy as np

U32 = 2.0 ** -24      # fp32 unit roundoff
FP32_P_TOL = 1e-5     # per-timestep probability tolerance for the FP32 path


def sigmoid64(z):
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fragile_keys(e64, offsets, p_thr=0.9, wc=4096, margin=1e-4):
    """Samples whose trigger decision is within `margin` (logit) of flipping in the oracle's scores:
    near the threshold, or with an in-window competitor within margin."""
    from scipy.ndimage import maximum_filter1d
    thr = math.log(p_thr / (1 - p_thr))
    out = set()
    for s in range(len(offsets) - 1):
        seg = np.asarray(e64[offsets[s]:offsets[s + 1]], dtype=np.float64)
        n = seg.size
        if n == 0:
            continue
        near_thr = np.abs(seg - thr) < margin
        pad = np.concatenate([np.full(wc, -np.inf), seg, np.full(wc, -np.inf)])
        # max over [a - wc, a + wc] excluding a itself is at least the 2nd order statistic; use the
        # window max of everything but a: compare a's value with the max of its two half-windows
        fm = maximum_filter1d(pad, size=wc, origin=-(wc // 2), mode="constant", cval=-np.inf)
        left = fm[0:n]
        right = fm[wc + 1:wc + 1 + n]
        comp = np.maximum(left, right)
        close = np.abs(seg - comp) < margin
        for a in np.nonzero(near_thr | close)[0]:
            out.add((s, int(a)))
    return out
