"""Python binding of libgwd (ctypes): argument marshalling only.

Every step of the hot path runs in the HIP kernels of libgwd.so; this module
only converts torch tensors (device memory, streams) to the C ABI declared in
include/gwd.h. There is no fallback: if the library is missing, importing the
binding raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwd.so")

OK = 0
ERR_ARG = -1
ERR_SHAPE = -2
ERR_CAPACITY = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5
ERR_NONFINITE = -6
ERR_NO_DEVICE = -7

FP32, BF16, FP8_E4M3, FP64 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3, "fp64": FP64}


class GwdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgwd error {code}: {msg}")
        self.code = code


class Arch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("kind", "in_channels", "channels", "skip_channels", "head_channels",
                 "n_stacks", "layers_per_stack", "kernel_size", "input_kernel", "head_mid_relu")]


class Stream(ctypes.Structure):
    _fields_ = [("ch", ctypes.c_void_p * 2), ("elem_stride", ctypes.c_int64), ("length", ctypes.c_int64)]


class Trigger(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_int32), ("_pad", ctypes.c_int32), ("sample", ctypes.c_int64),
                ("logit", ctypes.c_float), ("prob", ctypes.c_float)]


def tiny_arch() -> Arch:
    return Arch(0, 2, 16, 0, 0, 1, 4, 2, 1, 0)


def full_arch(head_mid_relu: int = 0) -> Arch:
    return Arch(1, 2, 128, 128, 128, 3, 10, 2, 1, head_mid_relu)


def two_branch_arch(head_mid_relu: int = 0) -> Arch:
    """One 64-channel gated branch per detector, skip sums concatenated into a 128-channel head."""
    return Arch(2, 2, 64, 64, 128, 3, 10, 2, 1, head_mid_relu)


def _load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "or python paper_2201_11133_amd/build.py")
    # torch carries its own HIP runtime (soname libamdhip64.so.7, loaded by file name). Importing it
    # first makes libgwd's dependency resolve to that same runtime, so device pointers and streams
    # from torch are valid in libgwd; opened the other way round the process would hold two HIP
    # runtimes and torch would find no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64, F32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    sig = {
        "gwd_num_params": (I64, [ctypes.POINTER(Arch)]),
        "gwd_receptive_field": (I32, [ctypes.POINTER(Arch)]),
        "gwd_load_weights": (I32, [ctypes.POINTER(Arch), I32, P, I64, I32, ctypes.POINTER(P)]),
        "gwd_free": (None, [P]),
        "gwd_forward": (I32, [P, ctypes.POINTER(Stream), I32, I32, I32, I32, P, I64, P]),
        "gwd_forward_out_floats": (I64, [P, ctypes.POINTER(Stream), I32, I32, I32, I32]),
        "gwd_triggers": (I32, [P, P, I32, D, I32, ctypes.POINTER(Trigger), I64, ctypes.POINTER(I64), P]),
        "gwd_triggers_noalloc": (I32, [P, P, I32, D, I32, ctypes.POINTER(Trigger), I64, ctypes.POINTER(I64), P]),
        "gwd_triggers_noalloc_scratch_bytes": (I64, [P, I32, I32]),
        "gwd_time_slide": (I32, [ctypes.POINTER(Stream), P, I32, P, P]),
        "gwd_far_curve": (I32, [ctypes.POINTER(Trigger), I64, P, I32, D, P, P]),
        "gwd_prob64": (I32, [P, I64, P, P]),
        "gwd_find_peaks": (I32, [P, I64, D, D, P, P, I64, ctypes.POINTER(I64), P]),
        "gwd_coincidence": (I32, [P, P, I32, I64, P, I64, ctypes.POINTER(I64)]),
        "gwd_welch_psd": (I32, [ctypes.POINTER(Stream), I32, D, P, P]),
        "gwd_whiten": (I32, [ctypes.POINTER(Stream), P, I32, D, I32, P, P]),
        "gwd_saved_bytes": (I64, [P, I32, I32]),
        "gwd_forward_train": (I32, [P, I32, P, I32, I32, P, P, P]),
        "gwd_backward": (I32, [P, I32, P, I32, I32, P, P, P, P, P]),
        "gwd_adam_step": (I32, [P, I32, P, P, P, P, I64, F32, F32, F32, F32, P, P]),
        "gwd_last_error": (ctypes.c_char_p, []),
        "gwd_debug_layer": (I32, [P, I32, I32, P, I32, I32, P, P, P, P]),
        "gwd_bce_logits": (I32, [P, P, I64, P, P, P]),
        "gwd_debug_time_layer": (I32, [P, I32, I32, I32, ctypes.POINTER(F32), ctypes.POINTER(I32),
                                       ctypes.POINTER(I32), P]),
        "gwd_plan_create": (I32, [P, ctypes.POINTER(Stream), I32, I32, I32, I32, P, I64, ctypes.POINTER(P)]),
        "gwd_plan_launch": (I32, [P, P]),
        "gwd_plan_completion_us": (I32, [P, P, I32, ctypes.POINTER(D)]),
        "gwd_plan_free": (None, [P]),
        "gwd_set_tiling": (I32, [P, I32, I32, I32, I32]),
        "gwd_set_fused_blocks": (I32, [P, I32]),
        "gwd_set_persistent": (I32, [P, I32]),
        "gwd_autotune": (I32, [P, ctypes.POINTER(Stream), I32, I32, I32, P, I64, ctypes.POINTER(I32),
                               ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                               ctypes.POINTER(I32), P]),
        "gwd_debug_export_weights": (I32, [P, I32, P, I64]),
        "gwd_debug_capture_backward": (I32, [P, I32, P, P, P, P, P, P, P, P]),
        "gwd_debug_fused": (I32, [P, I32, I32, P, I32, I32, P, P, P, P, ctypes.POINTER(I32), P]),
        "gwd_debug_mfma": (I32, [I32, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.gwd_last_error().decode()


def check(code: int) -> None:
    if code != OK:
        raise GwdError(code, last_error())


def num_params(arch: Arch) -> int:
    return int(lib.gwd_num_params(ctypes.byref(arch)))


def receptive_field(arch: Arch) -> int:
    return int(lib.gwd_receptive_field(ctypes.byref(arch)))


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_streams(tensors: Sequence) -> Tuple[ctypes.Array, List[int]]:
    """gwd_stream array for device tensors of shape [L, 2] (interleaved) or pairs (ch0, ch1) of [L]."""
    arr = (Stream * len(tensors))()
    lengths = []
    for i, t in enumerate(tensors):
        if isinstance(t, (tuple, list)):
            c0, c1 = t
            assert c0.dtype == c1.dtype and c0.shape == c1.shape and c0.dim() == 1
            assert c0.stride(0) == c1.stride(0)
            arr[i].ch[0], arr[i].ch[1] = c0.data_ptr(), c1.data_ptr()
            arr[i].elem_stride = c0.stride(0)
            arr[i].length = c0.shape[0]
        else:
            assert t.dim() == 2 and t.shape[1] == 2 and t.stride(1) == 1
            arr[i].ch[0] = t.data_ptr()
            arr[i].ch[1] = t.data_ptr() + 4
            arr[i].elem_stride = t.stride(0)
            arr[i].length = t.shape[0]
        lengths.append(int(arr[i].length))
    return arr, lengths


class Model:
    """Opaque libgwd model handle: n_members members of one architecture at one precision."""

    def __init__(self, arch: Arch, blobs: np.ndarray, precision: str = "fp32"):
        blobs = np.ascontiguousarray(np.asarray(blobs, dtype=np.float32))
        if blobs.ndim == 1:
            blobs = blobs[None]
        self.arch = arch
        self.n_members = blobs.shape[0]
        self.n_params = blobs.shape[1]
        # a two-branch model runs (and exports) as the block-diagonal trunk of twice the width
        self.export_params = self.n_params if arch.kind != 2 else num_params(
            Arch(1, 2, 2 * arch.channels, 2 * arch.skip_channels, arch.head_channels, arch.n_stacks,
                 arch.layers_per_stack, arch.kernel_size, arch.input_kernel, arch.head_mid_relu))
        self.precision = precision
        h = ctypes.c_void_p()
        check(lib.gwd_load_weights(ctypes.byref(arch), self.n_members, blobs.ctypes.data, self.n_params,
                                   PRECISIONS[precision], ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib.gwd_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def out_floats(self, streams, window: int, stride: int, out_mode: int) -> int:
        arr, _ = make_streams(streams)
        n = lib.gwd_forward_out_floats(self.h, arr, len(streams), window, stride, out_mode)
        if n < 0:
            raise GwdError(ERR_ARG, last_error())
        return int(n)

    def forward(self, streams, window: int = 4096, stride: int = 256, out_mode: int = 0, out=None, stream=None):
        """Run gwd_forward; returns the float32 device output tensor (layout per out_mode)."""
        import torch
        arr, _ = make_streams(streams)
        n = lib.gwd_forward_out_floats(self.h, arr, len(streams), window, stride, out_mode)
        if n < 0:   # invalid arguments: let gwd_forward report its own status code
            check(lib.gwd_forward(self.h, arr, len(streams), window, stride, out_mode, None, 0,
                                  _stream_handle(stream)))
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        check(lib.gwd_forward(self.h, arr, len(streams), window, stride, out_mode, _ptr(out), out.numel(),
                              _stream_handle(stream)))
        return out[:n]

    def time_layer(self, member: int = 0, layer: int = 15, reps: int = 10, stream=None):
        """(ms per launch, windows per launch, layers per launch) of the forward's launch at a middle
        layer (a fused triple covers three layers, a sextet six)."""
        ms, nw, nl = ctypes.c_float(0), ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib.gwd_debug_time_layer(self.h, member, layer, reps, ctypes.byref(ms), ctypes.byref(nw),
                                       ctypes.byref(nl), _stream_handle(stream)))
        return float(ms.value), int(nw.value), int(nl.value)

    def set_tiling(self, tile_rows: int = 0, waves: int = 0, batch_windows: int = 512, layers_per_launch: int = 0):
        check(lib.gwd_set_tiling(self.h, tile_rows, waves, layers_per_launch, batch_windows))

    def set_fused_blocks(self, blocks: int = 0):
        """gwd_set_fused_blocks: the number of blocks a fused launch aims at (0 = the default, 512)."""
        check(lib.gwd_set_fused_blocks(self.h, blocks))

    def set_persistent(self, on: bool = True):
        """gwd_set_persistent: run the forward (and plans created afterwards) as one persistent launch."""
        check(lib.gwd_set_persistent(self.h, 1 if on else 0))

    def autotune(self, streams, window: int = 4096, stride: int = 256, out=None, stream=None):
        """Pick the fastest schedule for this request; returns (tile_rows, waves, layers_per_launch,
        batch_windows, fused_blocks, persistent)."""
        import torch
        arr, _ = make_streams(streams)
        n = self.out_floats(streams, window, stride, 0)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        rw, w, fu, b, fb, pe = (ctypes.c_int32(0) for _ in range(6))
        check(lib.gwd_autotune(self.h, arr, len(streams), window, stride, _ptr(out), out.numel(), ctypes.byref(rw),
                               ctypes.byref(w), ctypes.byref(fu), ctypes.byref(b), ctypes.byref(fb),
                               ctypes.byref(pe), _stream_handle(stream)))
        return int(rw.value), int(w.value), int(fu.value), int(b.value), int(fb.value), int(pe.value)

    def plan(self, streams, window: int = 4096, stride: int = 256, out_mode: int = 0, out=None):
        """Capture the whole forward for this request into a replayable graph (see Plan)."""
        return Plan(self, streams, window, stride, out_mode, out)

    def export_weights(self, member: int = 0) -> np.ndarray:
        out = np.zeros(self.export_params, dtype=np.float32)
        check(lib.gwd_debug_export_weights(self.h, member, out.ctypes.data, self.export_params))
        return out

    def fused_layers(self, layer: int, window: int) -> int:
        """Layers of the fused launch that starts at `layer` for this window length (0 if none)."""
        nl = ctypes.c_int32(0)
        code = lib.gwd_debug_fused(self.h, 0, layer, None, 1, window, None, None, None, None, ctypes.byref(nl), None)
        return int(nl.value) if code == OK else 0

    def debug_fused(self, member: int, layer: int, x_in, n_windows: int, window: int, skip, stream=None):
        """gwd_debug_fused: (pre [nl][rows][2C], x_out [nl][rows][C], skip_out [nl][rows][C]) fp32 device
        tensors of the fused launch at `layer`; skip (fp32 [rows][C]) is updated in place."""
        import torch
        nl = self.fused_layers(layer, window)
        if nl == 0:
            raise GwdError(ERR_ARG, f"no fused launch starts at layer {layer}")
        rows = n_windows * window
        pre = torch.empty((nl, rows, 256), dtype=torch.float32, device="cuda")
        xo = torch.zeros((nl, rows, 128), dtype=torch.float32, device="cuda")
        so = torch.empty((nl, rows, 128), dtype=torch.float32, device="cuda")
        n = ctypes.c_int32(0)
        check(lib.gwd_debug_fused(self.h, member, layer, _ptr(x_in), n_windows, window, _ptr(skip), _ptr(pre),
                                  _ptr(xo), _ptr(so), ctypes.byref(n), _stream_handle(stream)))
        return pre, xo, so

    def capture_backward(self, layer: int, bufs=None):
        """gwd_debug_capture_backward: the next backward copies gated layer `layer`'s operands and
        results into bufs (dict of fp32 device tensors x_in, pre, dskip, dx_in, dg, g, dpre, dx_out);
        layer -1 turns it off."""
        names = ("x_in", "pre", "dskip", "dx_in", "dg", "g", "dpre", "dx_out")
        ptrs = [_ptr(bufs[k]) if bufs else 0 for k in names]
        check(lib.gwd_debug_capture_backward(self.h, layer, *ptrs))

    def debug_layer(self, member: int, layer: int, x_in, n_windows: int, window: int, pre_out, x_out, skip,
                    stream=None):
        check(lib.gwd_debug_layer(self.h, member, layer, _ptr(x_in), n_windows, window, _ptr(pre_out),
                                  _ptr(x_out), _ptr(skip), _stream_handle(stream)))


def debug_mfma(kind: int, a, b, c, stream=None):
    """gwd_debug_mfma: D = A B + C by one matrix-core instruction (kind 0: bf16 [32][16] x [16][32],
    kind 1: E4M3 [32][64] x [64][32]); a and b are uint8/int16 device tensors of the operand bits,
    c a [32][32] fp32 device tensor. Returns D."""
    import torch
    K = 16 if kind == 0 else 64
    eb = 2 if kind == 0 else 1
    assert a.is_contiguous() and a.numel() * a.element_size() == 32 * K * eb
    assert b.is_contiguous() and b.numel() * b.element_size() == 32 * K * eb
    assert c.dtype == torch.float32 and c.is_contiguous() and c.numel() == 1024
    d = torch.empty((32, 32), dtype=torch.float32, device=c.device)
    check(lib.gwd_debug_mfma(kind, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _stream_handle(stream)))
    return d


def _member_function():
    import torch

    class MemberFunction(torch.autograd.Function):
        """Per-timestep logits of one member over a batch of windows [B, T, 2], differentiable through
        the library's hand-written backward (gwd_forward_train keeps the per-stack checkpoints,
        gwd_backward recomputes each stack and returns the weight and input gradients).

        `weights` is the member's fp32 (fp64 for FP64 models) master blob the model currently holds
        (the one it was loaded from or gwd_adam_step last wrote); it is an argument so that autograd
        routes the weight gradient to it. The forward itself uses the model's packed copy."""

        @staticmethod
        def forward(ctx, windows, weights, model, member):
            B, T = windows.shape[0], windows.shape[1]
            dt = torch.float64 if model.precision == "fp64" else torch.float32
            logits = torch.empty((B, T), dtype=dt, device=windows.device)
            saved = torch.empty(int(lib.gwd_saved_bytes(model.h, B, T)), dtype=torch.uint8, device=windows.device)
            windows = windows.contiguous()
            check(lib.gwd_forward_train(model.h, member, windows.data_ptr(), B, T, logits.data_ptr(),
                                        saved.data_ptr(), _stream_handle(None)))
            ctx.save_for_backward(windows)
            ctx.saved_buf, ctx.model, ctx.member, ctx.wshape = saved, model, member, weights.shape
            return logits

        @staticmethod
        def backward(ctx, grad_logits):
            (windows,) = ctx.saved_tensors
            B, T = windows.shape[0], windows.shape[1]
            dz = grad_logits.contiguous()
            grad = torch.empty(ctx.wshape, dtype=dz.dtype, device=dz.device)
            du = torch.empty_like(windows) if ctx.needs_input_grad[0] else None
            check(lib.gwd_backward(ctx.model.h, ctx.member, windows.data_ptr(), B, T, ctx.saved_buf.data_ptr(),
                                   dz.data_ptr(), grad.data_ptr(), du.data_ptr() if du is not None else None,
                                   _stream_handle(None)))
            return du, grad, None, None

    return MemberFunction


_MEMBER_FN = None


def member_logits(model: "Model", weights, windows, member: int = 0):
    """Differentiable logits of one member (see MemberFunction)."""
    global _MEMBER_FN
    if _MEMBER_FN is None:
        _MEMBER_FN = _member_function()
    return _MEMBER_FN.apply(windows, weights, model, member)


class Trainer:
    """Buffers and calls of one training step of member `member` (forward with checkpoints, BCE,
    backward, Adam) through the C ABI; master weights, moments and gradients live on the device."""

    def __init__(self, model: "Model", blob: np.ndarray, B: int, T: int, member: int = 0):
        import torch
        self.m, self.B, self.T, self.member = model, B, T, member
        self.master = torch.from_numpy(np.ascontiguousarray(blob, dtype=np.float32)).cuda()
        self.mom = torch.zeros_like(self.master)
        self.vel = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.logits = torch.empty((B, T), dtype=torch.float32, device="cuda")
        self.dz = torch.empty_like(self.logits)
        self.saved = torch.empty(int(lib.gwd_saved_bytes(model.h, B, T)), dtype=torch.uint8, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.norm = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.step_no = 0

    def step(self, windows, labels, lr: float = 1e-3, stream=None):
        s = _stream_handle(stream)
        check(lib.gwd_forward_train(self.m.h, self.member, windows.data_ptr(), self.B, self.T,
                                    self.logits.data_ptr(), self.saved.data_ptr(), s))
        check(lib.gwd_bce_logits(self.logits.data_ptr(), labels.data_ptr(), self.B * self.T, self.dz.data_ptr(),
                                 self.loss.data_ptr(), s))
        check(lib.gwd_backward(self.m.h, self.member, windows.data_ptr(), self.B, self.T, self.saved.data_ptr(),
                               self.dz.data_ptr(), self.grad.data_ptr(), None, s))
        self.step_no += 1
        check(lib.gwd_adam_step(self.m.h, self.member, self.master.data_ptr(), self.grad.data_ptr(),
                                self.mom.data_ptr(), self.vel.data_ptr(), self.step_no, lr, 0.9, 0.999, 1e-8,
                                self.norm.data_ptr(), s))
        return self.loss, self.norm

    # ---- checkpoint and resume: master weights, Adam moments and the step count
    def save(self, path: str) -> None:
        """Write a checkpoint (safetensors): fp32 master weights and Adam moments of this member,
        the step count, and the architecture, precision and batch shape."""
        import json
        import torch
        from safetensors.torch import save_file
        torch.cuda.synchronize()
        arch = {n: int(getattr(self.m.arch, n)) for n, _ in Arch._fields_}
        meta = {"step": str(self.step_no), "member": str(self.member), "B": str(self.B), "T": str(self.T),
                "precision": self.m.precision, "arch": json.dumps(arch)}
        save_file({"master": self.master.cpu(), "mom": self.mom.cpu(), "vel": self.vel.cpu()}, path, metadata=meta)

    @classmethod
    def resume(cls, path: str) -> "Trainer":
        """A trainer (and its one-member model, trainer.m) continuing from a checkpoint written by
        save(): the model's working weights are packed from the saved master weights, and the next
        step is step_no + 1 with the saved moments, so training continues as if uninterrupted."""
        import json
        import torch
        from safetensors import safe_open
        with safe_open(path, framework="pt") as f:
            meta = f.metadata()
            t = {k: f.get_tensor(k) for k in ("master", "mom", "vel")}
        arch = Arch(**json.loads(meta["arch"]))
        master = t["master"].numpy()
        model = Model(arch, master, meta["precision"])
        tr = cls(model, master, int(meta["B"]), int(meta["T"]), member=0)
        tr.mom.copy_(t["mom"].to(tr.mom.device))
        tr.vel.copy_(t["vel"].to(tr.vel.device))
        tr.step_no = int(meta["step"])
        torch.cuda.synchronize()
        return tr


class Plan:
    """A captured forward: one graph launch per call, bound to the given stream buffers and output."""

    def __init__(self, model: "Model", streams, window: int, stride: int, out_mode: int, out=None):
        import torch
        self.model = model
        self.arr, self.lengths = make_streams(streams)
        self.n_streams = len(streams)
        n = model.out_floats(streams, window, stride, out_mode)
        self.out = out if out is not None else torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        h = ctypes.c_void_p()
        check(lib.gwd_plan_create(model.h, self.arr, self.n_streams, window, stride, out_mode, _ptr(self.out),
                                  self.out.numel(), ctypes.byref(h)))
        self.h = h
        self.n_out = n

    def launch(self, stream=None):
        check(lib.gwd_plan_launch(self.h, _stream_handle(stream)))
        return self.out[: self.n_out]

    def completion_us(self):
        """(per-stream completion times, total) in microseconds for the last launch."""
        per = np.zeros(self.n_streams, dtype=np.float64)
        tot = ctypes.c_double(0)
        check(lib.gwd_plan_completion_us(self.h, per.ctypes.data, self.n_streams, ctypes.byref(tot)))
        return per, float(tot.value)

    def close(self):
        if getattr(self, "h", None):
            lib.gwd_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def triggers(e, offsets: Sequence[int], threshold_prob: float = 0.9, cluster_window: int = 4096,
             capacity: Optional[int] = None, stream=None) -> List[Tuple[int, int, float, float]]:
    """gwd_triggers on a device score tensor e; returns (stream, sample, logit, prob) records."""
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n_streams = offs.size - 1
    if capacity is None:
        capacity = int(sum(-(-(int(offs[i + 1] - offs[i])) // cluster_window) for i in range(n_streams)))
    buf = (Trigger * max(capacity, 1))()
    nf = ctypes.c_int64(0)
    check(lib.gwd_triggers(_ptr(e), offs.ctypes.data, n_streams, threshold_prob, cluster_window, buf, capacity,
                           ctypes.byref(nf), _stream_handle(stream)))
    return [(buf[i].stream, buf[i].sample, buf[i].logit, buf[i].prob) for i in range(min(nf.value, capacity))]


def triggers_noalloc(e, offsets: Sequence[int], threshold_prob: float = 0.9, cluster_window: int = 4096,
                     capacity: Optional[int] = None, stream=None) -> List[Tuple[int, int, float, float]]:
    """gwd_triggers_noalloc (the allocation-free form, static device scratch) on a device score
    tensor e; returns (stream, sample, logit, prob) records."""
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n_streams = offs.size - 1
    if capacity is None:
        capacity = int(sum(-(-(int(offs[i + 1] - offs[i])) // cluster_window) for i in range(n_streams)))
    buf = (Trigger * max(capacity, 1))()
    nf = ctypes.c_int64(0)
    check(lib.gwd_triggers_noalloc(_ptr(e), offs.ctypes.data, n_streams, threshold_prob, cluster_window, buf,
                                   capacity, ctypes.byref(nf), _stream_handle(stream)))
    return [(buf[i].stream, buf[i].sample, buf[i].logit, buf[i].prob) for i in range(min(nf.value, capacity))]


def time_slide(src, shifts: Sequence[int], out=None, stream=None):
    """gwd_time_slide: slid copies of one device stream ([L, 2] tensor or (ch0, ch1) pair) as a
    [len(shifts), L, 2] float32 device tensor; channel 1 of copy k is read shifts[k] samples later,
    circularly."""
    import torch
    arr, lengths = make_streams([src])
    L = lengths[0]
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.int64))
    if out is None:
        dev = src[0].device if isinstance(src, (tuple, list)) else src.device
        out = torch.empty((sh.size, L, 2), dtype=torch.float32, device=dev)
    assert out.dtype == torch.float32 and out.is_contiguous() and tuple(out.shape) == (sh.size, L, 2)
    check(lib.gwd_time_slide(arr, sh.ctypes.data, int(sh.size), _ptr(out), _stream_handle(stream)))
    return out


def far_curve(records: Sequence[Tuple[int, int, float, float]], logit_thresholds: Sequence[float],
              livetime_s: float) -> Tuple[np.ndarray, np.ndarray]:
    """gwd_far_curve on (stream, sample, logit, prob) trigger records: (counts, false alarms per second)."""
    n = len(records)
    buf = (Trigger * max(n, 1))()
    for i, (st, a, z, pr) in enumerate(records):
        buf[i].stream, buf[i].sample, buf[i].logit, buf[i].prob = int(st), int(a), float(z), float(pr)
    thr = np.ascontiguousarray(np.asarray(logit_thresholds, dtype=np.float64))
    counts = np.zeros(thr.size, dtype=np.int64)
    far = np.zeros(thr.size, dtype=np.float64)
    check(lib.gwd_far_curve(buf, n, thr.ctypes.data, int(thr.size), float(livetime_s), counts.ctypes.data,
                            far.ctypes.data))
    return counts, far


def prob64(z, out=None, stream=None):
    """gwd_prob64: float64 probabilities 1 / (1 + e^-z) of a float32 device logit tensor."""
    import torch
    z = z.contiguous()
    if out is None:
        out = torch.empty(z.shape, dtype=torch.float64, device=z.device)
    check(lib.gwd_prob64(_ptr(z), z.numel(), _ptr(out), _stream_handle(stream)))
    return out


def find_peaks(x, height: float, min_width: float, capacity: Optional[int] = None, stream=None):
    """gwd_find_peaks on a float64 device signal: (peak indices int64, widths float64) as numpy arrays."""
    n = x.numel()
    cap = (n // 2 + 1) if capacity is None else int(capacity)
    peaks = np.empty(max(cap, 1), dtype=np.int64)
    widths = np.empty(max(cap, 1), dtype=np.float64)
    nf = ctypes.c_int64(0)
    check(lib.gwd_find_peaks(_ptr(x), n, float(height), float(min_width), peaks.ctypes.data, widths.ctypes.data, cap,
                             ctypes.byref(nf), _stream_handle(stream)))
    return peaks[:nf.value].copy(), widths[:nf.value].copy()


def coincidence(peak_lists: Sequence, window: int) -> List[int]:
    """gwd_coincidence: peaks of member 0 matched by every other member within +/- window samples."""
    arrs = [np.ascontiguousarray(np.asarray(p, dtype=np.int64)) for p in peak_lists]
    ptrs = (ctypes.c_void_p * max(len(arrs), 1))(*[a.ctypes.data for a in arrs])
    counts = np.array([a.size for a in arrs], dtype=np.int64)
    cap = int(arrs[0].size) if arrs else 0
    ev = np.empty(max(cap, 1), dtype=np.int64)
    nf = ctypes.c_int64(0)
    check(lib.gwd_coincidence(ptrs, counts.ctypes.data, len(arrs), int(window), ev.ctypes.data, cap, ctypes.byref(nf)))
    return [int(v) for v in ev[:nf.value]]


def welch_psd(src, nperseg: int = 16384, fs: float = 4096.0, out=None, stream=None):
    """gwd_welch_psd: one-sided Welch PSD of both channels of one device stream ([L, 2] tensor or
    (ch0, ch1) pair) as a float64 device tensor [2, nperseg // 2 + 1]."""
    import torch
    arr, _ = make_streams([src])
    if out is None:
        dev = src[0].device if isinstance(src, (tuple, list)) else src.device
        out = torch.empty((2, nperseg // 2 + 1), dtype=torch.float64, device=dev)
    assert out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == (2, nperseg // 2 + 1)
    check(lib.gwd_welch_psd(arr, int(nperseg), float(fs), _ptr(out), _stream_handle(stream)))
    return out


def whiten(src, psd, nperseg: int = 16384, fs: float = 4096.0, normalize: bool = True, out=None, stream=None):
    """gwd_whiten: the stream whitened by psd (float64 device [2, nperseg // 2 + 1]) and, if normalize,
    scaled to unit deviation per channel, as a float32 device tensor [L, 2]."""
    import torch
    arr, lengths = make_streams([src])
    if out is None:
        dev = src[0].device if isinstance(src, (tuple, list)) else src.device
        out = torch.empty((lengths[0], 2), dtype=torch.float32, device=dev)
    assert out.dtype == torch.float32 and out.is_contiguous() and tuple(out.shape) == (lengths[0], 2)
    assert psd.dtype == torch.float64 and psd.is_contiguous() and tuple(psd.shape) == (2, nperseg // 2 + 1)
    check(lib.gwd_whiten(arr, _ptr(psd), int(nperseg), float(fs), int(bool(normalize)), _ptr(out),
                         _stream_handle(stream)))
    return out
