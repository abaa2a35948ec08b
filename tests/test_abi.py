"""C ABI host paths on a machine without a GPU: the library loads, exports every function the
header declares, and rejects bad arguments with the documented codes before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwd.h")


@pytest.fixture(scope="module")
def g():
    from paper_2201_11133_amd import gwd
    return gwd


def host_has_gpu() -> bool:
    # counting devices does not initialise the GPU runtime
    import torch
    return torch.cuda.device_count() > 0


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gwd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["gwd_load_weights", "gwd_forward", "gwd_triggers", "gwd_backward", "gwd_adam_step",
              "gwd_forward_train", "gwd_num_params", "gwd_receptive_field", "gwd_free", "gwd_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(g):
    lib = ctypes.CDLL(g.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_counts(g):
    assert g.num_params(g.tiny_arch()) == 1681
    assert g.num_params(g.full_arch()) == 2964993
    assert g.num_params(g.full_arch(1)) == 2964993
    assert g.receptive_field(g.tiny_arch()) == 16
    assert g.receptive_field(g.full_arch()) == 3070
    a = g.full_arch()
    a.input_kernel = 2
    assert g.receptive_field(a) == 3071
    assert g.num_params(a) == 2964993 + 256
    bad = g.full_arch()
    bad.kind = 7
    assert g.num_params(bad) == -1 and g.receptive_field(bad) == -1


def test_counts_match_oracle(g):
    from oracle.arch import FULL, TINY, Arch, num_params, receptive_field
    for ours, theirs in [(g.tiny_arch(), TINY), (g.full_arch(), FULL)]:
        assert g.num_params(ours) == num_params(theirs)
        assert g.receptive_field(ours) == receptive_field(theirs)
    for ls, ns in [(2, 3), (5, 2), (10, 1)]:
        a = g.full_arch()
        a.layers_per_stack, a.n_stacks = ls, ns
        o = Arch(n_stacks=ns, layers_per_stack=ls)
        assert g.num_params(a) == num_params(o) and g.receptive_field(a) == receptive_field(o)


def load(g, arch, blob, n_members, n_params, prec):
    h = ctypes.c_void_p()
    code = g.lib.gwd_load_weights(ctypes.byref(arch), n_members, blob.ctypes.data if blob is not None else None,
                                  n_params, prec, ctypes.byref(h))
    return code, h


def test_load_weights_argument_errors(g):
    a = g.full_arch()
    n = g.num_params(a)
    blob = np.zeros(n, np.float32)
    assert load(g, a, blob, 1, n - 1, g.FP32)[0] == g.ERR_ARG          # wrong parameter count
    assert load(g, a, None, 1, n, g.FP32)[0] == g.ERR_ARG               # null blob
    assert load(g, a, blob, 0, n, g.FP32)[0] == g.ERR_ARG               # no members
    assert load(g, a, blob, 1, n, 9)[0] == g.ERR_ARG                    # unknown precision
    bad = g.full_arch()
    bad.kernel_size = 3
    assert load(g, bad, blob, 1, g.num_params(bad), g.FP32)[0] == g.ERR_ARG
    unsup = g.full_arch()
    unsup.channels = 64
    assert load(g, unsup, np.zeros(g.num_params(unsup), np.float32), 1, g.num_params(unsup), g.FP32)[0] == g.ERR_UNSUPPORTED
    if not host_has_gpu():
        # the plain member loads in every precision (its BF16/FP8 forms pass the argument checks)
        for prec in (g.BF16, g.FP8_E4M3):
            assert load(g, g.tiny_arch(), np.zeros(1681, np.float32), 1, 1681, prec)[0] == g.ERR_NO_DEVICE
        code, h = load(g, a, blob, 1, n, g.FP32)
        assert code == g.ERR_NO_DEVICE and not h.value      # valid arguments, but this host has no GPU
        assert g.last_error() != ""


def test_forward_and_debug_argument_errors(g):
    arr = (g.Stream * 1)()
    assert g.lib.gwd_forward(None, arr, 1, 4096, 256, 0, None, 0, None) == g.ERR_ARG
    assert g.lib.gwd_forward_out_floats(None, arr, 1, 4096, 256, 0) == -1
    assert g.lib.gwd_debug_layer(None, 0, 0, None, 1, 4096, None, None, None, None) == g.ERR_ARG
    out = np.zeros(10, np.float32)
    assert g.lib.gwd_debug_export_weights(None, 0, out.ctypes.data, 10) == g.ERR_ARG
    assert g.lib.gwd_set_persistent(None, 1) == g.ERR_ARG
    assert g.lib.gwd_set_fused_blocks(None, 0) == g.ERR_ARG
    g.lib.gwd_free(None)    # ignored


def trig(g, offs, p=0.9, wc=4096, cap=4, e_ptr=8):
    offs = np.asarray(offs, np.int64)
    nf = ctypes.c_int64(-1)
    buf = (g.Trigger * 4)()
    code = g.lib.gwd_triggers(e_ptr, offs.ctypes.data, len(offs) - 1, p, wc, buf, cap, ctypes.byref(nf), None)
    return code, nf.value


def test_trigger_argument_errors(g):
    assert trig(g, [0, 10], p=0.0)[0] == g.ERR_ARG
    assert trig(g, [0, 10], p=1.0)[0] == g.ERR_ARG
    assert trig(g, [0, 10], wc=0)[0] == g.ERR_ARG
    assert trig(g, [0, 10], wc=70000)[0] == g.ERR_ARG
    assert trig(g, [0, 10], cap=-1)[0] == g.ERR_ARG
    assert trig(g, [1, 10])[0] == g.ERR_ARG              # offsets must start at 0
    assert trig(g, [0, 10, 5])[0] == g.ERR_ARG           # and not decrease
    assert trig(g, [0, 10], e_ptr=None)[0] == g.ERR_ARG  # scores needed when samples exist
    assert trig(g, [0, 10], e_ptr=6)[0] == g.ERR_ARG     # misaligned
    assert trig(g, [0, 0, 0]) == (g.OK, 0)               # nothing to scan: no device needed
    if not host_has_gpu():                               # (the score pointer is not a real buffer)
        assert trig(g, [0, 10])[0] == g.ERR_NO_DEVICE


def test_training_argument_errors(g):
    assert g.lib.gwd_saved_bytes(None, 1, 4096) == -1
    assert g.lib.gwd_forward_train(None, 0, None, 1, 4096, None, None, None) in (g.ERR_ARG, g.ERR_UNSUPPORTED)
    assert g.lib.gwd_backward(None, 0, None, 1, 4096, None, None, None, None, None) in (g.ERR_ARG, g.ERR_UNSUPPORTED)
    assert g.lib.gwd_adam_step(None, 0, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None, None) in (g.ERR_ARG, g.ERR_UNSUPPORTED)


def test_one_hip_runtime_in_process():
    """libgwd shares torch's HIP runtime: a second copy would leave torch without devices."""
    import subprocess
    import sys
    code = ("import paper_2201_11133_amd.gwd\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__)))).stdout
    assert out.count("libamdhip64") == 1, out


def slide(g, length=10, stride=2, shifts=(1,), dst=8, ch0=16, ch1=20):
    src = g.Stream()
    src.ch[0], src.ch[1], src.elem_stride, src.length = ch0, ch1, stride, length
    sh = np.asarray(shifts, np.int64)
    return g.lib.gwd_time_slide(ctypes.byref(src), sh.ctypes.data, sh.size, dst, None)


def test_time_slide_argument_errors(g):
    assert g.lib.gwd_time_slide(None, None, 1, 8, None) == g.ERR_ARG
    assert slide(g, shifts=()) == g.ERR_ARG               # no shift
    assert slide(g, length=-1) == g.ERR_ARG
    assert slide(g, stride=0) == g.ERR_ARG
    assert slide(g, dst=None) == g.ERR_ARG
    assert slide(g, ch1=None) == g.ERR_ARG
    assert slide(g, dst=12) == g.ERR_ARG                  # output moves as 8-byte words
    assert slide(g, ch0=18) == g.ERR_ARG                  # misaligned input
    assert slide(g, length=0) == g.OK                     # nothing to copy: no device needed
    if not host_has_gpu():                                # (the pointers are not real buffers)
        assert slide(g) == g.ERR_NO_DEVICE


def test_far_curve_matches_oracle(g):
    from oracle.background import far_curve
    rng = np.random.default_rng(5)
    z = rng.normal(2.5, 3.0, 700).astype(np.float32)
    recs = [(int(i % 3), int(i * 5000), float(v), 0.0) for i, v in enumerate(z)]
    thr = np.array([-2.0, 0.0, np.log(9.0), 3.0, float(z[17]), 7.5, 20.0])
    counts, far = g.far_curve(recs, thr, 7200.0)
    c_o, f_o = far_curve(z.astype(np.float64), thr, 7200.0)
    assert np.array_equal(counts, c_o)
    assert np.array_equal(far, f_o)
    assert g.far_curve([], [1.0], 10.0)[0].tolist() == [0]
    for bad in [dict(livetime_s=0.0), dict(livetime_s=-1.0)]:
        with pytest.raises(g.GwdError):
            g.far_curve(recs, thr, **bad)
    assert g.lib.gwd_far_curve(None, 3, thr.ctypes.data, 1, 1.0, np.zeros(1, np.int64).ctypes.data,
                               np.zeros(1).ctypes.data) == g.ERR_ARG


def test_coincidence_matches_oracle(g):
    from oracle.postproc import coincident_events
    rng = np.random.default_rng(8)
    for _ in range(40):
        lists = [np.sort(rng.choice(50000, int(rng.integers(0, 40)), replace=False)) for _ in range(int(rng.integers(1, 5)))]
        wnd = int(rng.integers(0, 4000))
        assert g.coincidence(lists, wnd) == coincident_events(lists, wnd)


def test_postproc_argument_errors(g):
    nf = ctypes.c_int64(-1)
    out = np.zeros(4, np.int64)
    assert g.lib.gwd_coincidence(None, None, 1, 10, None, 0, ctypes.byref(nf)) == g.ERR_ARG
    cnt = np.array([1], np.int64)
    lst = (ctypes.c_void_p * 1)(out.ctypes.data)
    assert g.lib.gwd_coincidence(lst, cnt.ctypes.data, 1, -1, out.ctypes.data, 4, ctypes.byref(nf)) == g.ERR_ARG
    assert g.lib.gwd_coincidence(lst, cnt.ctypes.data, 0, 10, out.ctypes.data, 4, ctypes.byref(nf)) == g.ERR_ARG
    pk, wd = np.zeros(4, np.int64), np.zeros(4)
    assert g.lib.gwd_find_peaks(8, 2, 0.5, 1.0, pk.ctypes.data, wd.ctypes.data, 4, ctypes.byref(nf), None) == g.OK
    assert nf.value == 0                                  # fewer than 3 samples: nothing, no device needed
    assert g.lib.gwd_find_peaks(8, 100, float("nan"), 1.0, pk.ctypes.data, wd.ctypes.data, 4, ctypes.byref(nf), None) == g.ERR_ARG
    assert g.lib.gwd_find_peaks(12, 100, 0.5, 1.0, pk.ctypes.data, wd.ctypes.data, 4, ctypes.byref(nf), None) == g.ERR_ARG  # misaligned
    assert g.lib.gwd_find_peaks(8, 100, 0.5, 1.0, None, None, 4, ctypes.byref(nf), None) == g.ERR_ARG
    assert g.lib.gwd_prob64(None, 10, None, None) == g.ERR_ARG
    assert g.lib.gwd_prob64(None, 0, None, None) == g.OK


def whiten_call(g, length=4096, stride=2, n=256, fs=4096.0, normalize=1, psd=8, dst=8, ch0=16, ch1=20):
    src = g.Stream()
    src.ch[0], src.ch[1], src.elem_stride, src.length = ch0, ch1, stride, length
    return g.lib.gwd_whiten(ctypes.byref(src), psd, n, fs, normalize, dst, None)


def welch_call(g, length=4096, stride=2, n=256, fs=4096.0, psd=8, ch0=16, ch1=20):
    src = g.Stream()
    src.ch[0], src.ch[1], src.elem_stride, src.length = ch0, ch1, stride, length
    return g.lib.gwd_welch_psd(ctypes.byref(src), n, fs, psd, None)


def test_whitening_argument_errors(g):
    assert g.lib.gwd_whiten(None, 8, 256, 4096.0, 1, 8, None) == g.ERR_ARG
    assert g.lib.gwd_welch_psd(None, 256, 4096.0, 8, None) == g.ERR_ARG
    for f in (whiten_call, welch_call):
        assert f(g, n=100) == g.ERR_ARG                   # not a power of two
        assert f(g, n=8) == g.ERR_ARG                     # below 16
        assert f(g, n=32768) == g.ERR_ARG                 # above 16384
        assert f(g, fs=0.0) == g.ERR_ARG
        assert f(g, fs=float("inf")) == g.ERR_ARG
        assert f(g, psd=None) == g.ERR_ARG
        assert f(g, psd=12) == g.ERR_ARG                  # float64 PSD, misaligned
        assert f(g, ch0=18) == g.ERR_ARG
        assert f(g, ch1=None) == g.ERR_ARG
        assert f(g, stride=0) == g.ERR_ARG
    assert whiten_call(g, dst=12) == g.ERR_ARG
    assert whiten_call(g, normalize=2) == g.ERR_ARG
    assert whiten_call(g, length=5000) == g.ERR_SHAPE     # whole-stream transform: a power of two
    assert whiten_call(g, length=8) == g.ERR_SHAPE
    assert whiten_call(g, length=1 << 29) == g.ERR_SHAPE
    assert whiten_call(g, length=128, n=256) == g.ERR_SHAPE
    assert welch_call(g, length=255, n=256) == g.ERR_SHAPE
    if not host_has_gpu():                                # (the pointers are not real buffers)
        assert whiten_call(g) == g.ERR_NO_DEVICE
        assert welch_call(g, length=5000) == g.ERR_NO_DEVICE


def test_two_branch_counts_and_load_errors(g):
    from oracle.arch import TWO_BRANCH, num_params, receptive_field
    a = g.two_branch_arch()
    assert g.num_params(a) == num_params(TWO_BRANCH) == 1_498_497
    assert g.receptive_field(a) == receptive_field(TWO_BRANCH) == 3070
    bad = g.two_branch_arch()
    bad.in_channels = 3                                   # one branch per detector: exactly 2
    assert g.num_params(bad) == -1
    blob = np.zeros(g.num_params(a), np.float32)
    h = ctypes.c_void_p()
    assert g.lib.gwd_load_weights(ctypes.byref(a), 1, blob.ctypes.data, blob.size, g.FP64, ctypes.byref(h)) == g.ERR_UNSUPPORTED
    wide = g.two_branch_arch()
    wide.channels = wide.skip_channels = 128              # valid, but not what the kernels take
    wb = np.zeros(g.num_params(wide), np.float32)
    assert g.lib.gwd_load_weights(ctypes.byref(wide), 1, wb.ctypes.data, wb.size, g.FP32, ctypes.byref(h)) == g.ERR_UNSUPPORTED
    if not host_has_gpu():
        assert g.lib.gwd_load_weights(ctypes.byref(a), 1, blob.ctypes.data, blob.size, g.BF16, ctypes.byref(h)) == g.ERR_NO_DEVICE


def test_debug_entries_reject_bad_arguments(g):
    """The test-support entries check their arguments on the host."""
    assert g.lib.gwd_debug_capture_backward(None, 0, None, None, None, None, None, None, None, None) == g.ERR_ARG
    nl = ctypes.c_int32(7)
    assert g.lib.gwd_debug_fused(None, 0, 0, None, 1, 4096, None, None, None, None, ctypes.byref(nl), None) == g.ERR_ARG
    buf = (ctypes.c_float * 1024)()
    assert g.lib.gwd_debug_mfma(2, buf, buf, buf, buf, None) == g.ERR_ARG
    assert g.lib.gwd_debug_mfma(0, None, buf, buf, buf, None) == g.ERR_ARG
    if not host_has_gpu():
        assert g.lib.gwd_debug_mfma(1, buf, buf, buf, buf, None) == g.ERR_NO_DEVICE


def test_noalloc_triggers_scratch_limit(g):
    """The allocation-free trigger entry: same argument checks as gwd_triggers, and a request whose
    scratch need exceeds the static 16 MiB array is refused on the host, before any device work."""
    def nz(offs, wc=4096, cap=4, e_ptr=8, p=0.9):
        offs = np.asarray(offs, np.int64)
        nf = ctypes.c_int64(-1)
        buf = (g.Trigger * 4)()
        code = g.lib.gwd_triggers_noalloc(e_ptr, offs.ctypes.data, len(offs) - 1, p, wc, buf, cap,
                                          ctypes.byref(nf), None)
        return code, nf.value

    def need(offs, wc):
        offs = np.asarray(offs, np.int64)
        return g.lib.gwd_triggers_noalloc_scratch_bytes(offs.ctypes.data, len(offs) - 1, wc)

    r256 = lambda b: (b + 255) // 256 * 256
    assert need([0, 600_000], 1) == r256(32) + r256(8 * 600_000) + r256(24 * 600_000) + 256
    assert need([0, 0, 0], 64) == 0
    assert need([1, 5], 64) == -1 and need([0, 5, 4], 64) == -1 and need([0, 5], 0) == -1
    # the largest single stream that fits at cluster window 1 is accepted by the size check; one more tile is not
    n_fit = (16 << 20) - 256 - 256 - 512
    n_fit = n_fit // 32
    while need([0, n_fit + 1], 1) <= 16 << 20:
        n_fit += 1
    while need([0, n_fit], 1) > 16 << 20:
        n_fit -= 1
    assert need([0, n_fit], 1) <= 16 << 20 < need([0, n_fit + 1], 1)
    assert nz([0, n_fit + 1], wc=1) == (g.ERR_CAPACITY, 0)
    assert nz([0, 600_000], wc=1) == (g.ERR_CAPACITY, 0)
    assert "static maximum" in g.last_error()
    assert nz([0, 10], p=0.0)[0] == g.ERR_ARG
    assert nz([0, 10], wc=70000)[0] == g.ERR_ARG
    assert nz([0, 10], cap=-1)[0] == g.ERR_ARG
    assert nz([1, 10])[0] == g.ERR_ARG
    assert nz([0, 10, 5])[0] == g.ERR_ARG
    assert nz([0, 10], e_ptr=None)[0] == g.ERR_ARG
    assert nz([0, 10], e_ptr=6)[0] == g.ERR_ARG
    assert nz([0, 0, 0]) == (g.OK, 0)
