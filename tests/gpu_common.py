"""Helpers for the GPU parity tests (inputs come from the seeded generator, expectations from the oracle)."""
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
    """Samples whose trigger decision is within `margin` (logit) of flipping in the oracle's scores."""
    from oracle.triggers import fragile_decisions
    return fragile_decisions(e64, offsets, p_thr, wc, margin)
