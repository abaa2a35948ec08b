"""Benchmark of the ensemble gravitational-wave search hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic two-detector strain:
window gather + input projection, 30 gated dilated-conv layers, head, owner-window stitch,
ensemble minimum over the members, threshold + clustering into triggers.

Default workload: an ensemble of 4 members (3 stacks x 10 gated layers, 128 residual/skip
channels, independent He-normal weights), BF16 operands with fp32 accumulation, over a
3,600 s two-channel white-noise stream at 4096 Hz carrying leading-order chirps (200 per
86,400 s day, network SNR 8-20), window 4096, stride 256. Throughput does not depend on the
stream length at this scale (the stream is cut into batches of 512 windows). Inputs are
generated on the device before timing (HBM-resident when the timed region starts).

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FS = 4096
W, S = 4096, 256
FLOP_LAYERS_T = 5865984                   # flop per window time step per member: input conv + 30 gated layers
FLOP_HEAD_T = 33024                       # flop per owned (output) sample per member: 128x128 + 128 -> 1
FLOP_PER_LAYER_T = 196608                 # flop per time step of one gated layer (conv + res/skip)
# the two-branch member's own work per window time step: two 64-channel branches (input 1x1, 30 gated
# layers with 64 -> 128 dilated convs and 64 x 64 res/skip), i.e. the nonzero blocks of the trunk image
FLOP_LAYERS_T_2B = 2 * (64 * 2 + 30 * 2 * 128 * 64 * 2 + 29 * 2 * 64 * 64 + 30 * 2 * 64 * 64)
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
# End-to-end accuracy of each precision against the FP64 oracle, on a member trained by this package
# (300 BF16 steps; measured by tests/test_gpu_trained_member.py, not in this run): the target is
# max |dp| <= 2e-2 per sample.
ACCURACY = {
    "fp32": "max |dp| 4.6e-7 vs the FP64 oracle on a trained member: meets the 2e-2 target",
    "bf16": "max |dp| 0.0113 vs the FP64 oracle on a trained member: meets the 2e-2 target (gated)",
    "fp8": "max |dp| 0.098 vs the FP64 oracle on a trained member: misses the 2e-2 target (stated, not gated)",
}
# HBM bytes per launch of the dominant BF16 kernel, the middle stack's sextet (512 windows x 6 layers),
# from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a 1 GiB copy; valid only for the
# kernel source they were taken on (profiles/fused_sextet_bf16_counters_64s.md).
MEASURED_TRAFFIC = {"bf16": {"source_sha256_16": "6f025f4101bb5838", "bytes": 3306783521, "windows": 512, "layers": 6}}


def kernel_traffic(prec: str, windows: int, layers: int):
    import hashlib
    t = MEASURED_TRAFFIC.get(prec)
    if not t or t["windows"] != windows or t.get("layers", 1) != layers:
        return None
    h = hashlib.sha256()
    for f in ("fwd_lowp.hip", "fused_bf16_body.inc", "fused_fp8_body.inc", "layer_common.h"):   # the kernel source
        h.update(open(os.path.join(ROOT, "paper_2201_11133_amd", "csrc", f), "rb").read())
    sig = h.hexdigest()[:16]
    return t["bytes"] if sig == t["source_sha256_16"] else None


def make_stream_gpu(seconds: float, seed: int, chirps_per_day: float = 200.0):
    """Device stream [L, 2]: N(0,1) noise from a seeded torch generator plus seeded chirps."""
    import torch
    from paper_2201_11133_amd import synth
    L = int(round(seconds * FS))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    x = torch.randn((L, 2), dtype=torch.float32, device="cuda", generator=gen)
    rng = np.random.default_rng(seed)
    n = int(round(chirps_per_day * seconds / 86400.0))
    injs = [synth.draw_injection(rng, tc) for tc in synth.place_times(rng, n, seconds, 4.0, 10.0)]
    for inj in injs:
        lo = max(0, int(math.floor((inj.tc - inj.tau20 - 0.02) * FS)))
        hi = min(L, int(math.ceil((inj.tc + 0.02) * FS)) + 1)
        sig = synth.injection_signal(inj, lo / FS, hi - lo).astype(np.float32)
        x[lo:hi] += torch.from_numpy(sig).cuda()
    torch.cuda.synchronize()
    return x, injs


def n_windows(L: int) -> int:
    return 1 if L <= W else -(-(L - W) // S) + 1


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(fn, steps: int, warmup: int, label: str = "", warm_fn=None):
    import torch
    for i in range(warmup):
        t = time.perf_counter()
        (warm_fn or fn)()
        torch.cuda.synchronize()
        progress(f"{label} warmup {i + 1}/{warmup}: {time.perf_counter() - t:.2f} s")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, (time.perf_counter() - t0) * 1e3 / steps


def layer_kernel_timing(model, prec: str, reps: int = 10):
    """Average duration of the dominant kernel in the forward's own launch configuration, timed by
    the library with HIP events on the stream it launches on. The middle stack's launches are timed
    one by one (BF16 by default: a sextet, dilations 1-32, and a quad, 64-512; triples and a quad
    with three layers per launch); the kernel with the most time per stack is the dominant one, and
    the others are reported beside it. With one layer per launch: the single-layer kernel at a
    middle layer."""
    timed, l = [], 10
    while l < 20:
        t = model.time_layer(0, l, reps)
        if t[2] == 1:
            timed = [model.time_layer(0, 15, reps)]
            break
        timed.append(t)
        l += t[2]
    groups = {}
    for t in timed:
        groups.setdefault(t[2], []).append(t)
    nl = max(groups, key=lambda k: sum(x[0] for x in groups[k]))
    launches = groups[nl]
    ms = sum(x[0] for x in launches) / len(launches)
    nb = launches[0][1]
    flop = nb * W * FLOP_PER_LAYER_T * nl
    achieved = flop / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    traffic = kernel_traffic(prec, nb, nl)
    names = {1: "gated layer", 3: "fused gated layer triple", 4: "fused gated layer quad", 6: "fused gated layer sextet"}
    kernel = f"{names.get(nl, f'fused {nl}-layer launch')} ({prec})"
    out = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kernel,
           "ms_per_launch": round(ms, 4), "ms_per_launch_each": [round(x[0], 4) for x in launches],
           "windows_per_launch": nb, "layers_per_launch": nl, "flop_per_launch": flop}
    if traffic:
        out["hbm_GBps"] = round(traffic / (ms * 1e-3) / 1e9, 1)
    for k in sorted(groups):
        if k == nl:
            continue
        kms = sum(x[0] for x in groups[k]) / len(groups[k])
        kflop = groups[k][0][1] * W * FLOP_PER_LAYER_T * k
        out[names.get(k, f"{k}-layer").split()[-1]] = {
            "ms_per_launch": round(kms, 4), "layers_per_launch": k, "flop_per_launch": kflop,
            "achieved": round(kflop / (kms * 1e-3) / 1e12, 2)}
    return out


def streaming_line(gwd, blobs, x, out, ref_scores, args):
    """A separate line, not the metric: the same stitched ensemble scores from windows of 2^20
    samples with stride 2^20 - 3072. Owned rows only need their 3070-sample receptive field inside
    the window, so this reproduces the 4096/256 windowed scores bit for bit (checked here) with
    about 1/16 of the layer work; its own flop count is reported."""
    import torch
    Wl = 1 << 20
    Sl = Wl - 3072
    m = gwd.Model(gwd.full_arch(), blobs, args.precision)
    L = x.shape[0]

    def step(xx=x):
        m.forward([xx], Wl, Sl, out_mode=0, out=out)

    ms_ev, ms_wall = time_steps(step, args.steps, args.warmup, "streaming", step)  # full stream: sizes the workspace
    same = bool(torch.equal(out[:L], ref_scores[:L]))
    nw = 1 if L <= Wl else -(-(L - Wl) // Sl) + 1
    flop = args.members * (nw * Wl * FLOP_LAYERS_T + L * FLOP_HEAD_T)
    res = {"window": Wl, "stride": Sl, "strain_s_per_s": round(L / FS / (ms_wall / 1e3), 2),
           "ms_per_step": round(ms_wall, 3), "tflop_per_step": round(flop / 1e12, 2),
           "tflops": round(flop / (ms_wall * 1e-3) / 1e12, 2), "scores_identical_to_windowed": same,
           "precision": args.precision}
    if args.stream_day:
        # the same ensemble over a full day of strain (86400 s, 200 chirps): one pass, then triggers
        progress("streaming variant over 86400 s")
        xd, _ = make_stream_gpu(86400.0, 102)
        od = torch.empty(xd.shape[0], dtype=torch.float32, device="cuda")
        n_trig = [0]

        def day():
            m.forward([xd], Wl, Sl, out_mode=0, out=od)
            n_trig[0] = len(gwd.triggers(od, [0, xd.shape[0]], 0.9, 4096))

        _, ms_day = time_steps(day, 1, 1, "streaming day", lambda: m.forward([xd[: 64 * FS]], Wl, Sl, out_mode=0,
                                                                            out=od))
        res["day"] = {"stream_s": 86400.0, "s_per_day": round(ms_day / 1e3, 2),
                      "strain_s_per_s": round(86400.0 / (ms_day / 1e3), 2), "triggers": n_trig[0],
                      "scores_finite": bool(torch.isfinite(od).all().item())}
        del xd, od
    m.close()
    return res


def ragged_workload(gwd, blobs, prec: str):
    """32 concurrent streams, lengths log-uniform in 8-4096 s, each with 0-5 chirps (>= 2.5 s apart),
    all members and streams in one captured graph launch; tiling chosen by the autotuner on a
    64 s sample of the first stream."""
    import torch
    from paper_2201_11133_amd import synth
    lens = synth.ragged_lengths(103, 32)
    rng = np.random.default_rng(103)
    bufs = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(103)
    for L in lens:
        x = torch.randn((L, 2), dtype=torch.float32, device="cuda", generator=gen)
        secs = L / FS
        for inj in [synth.draw_injection(rng, tc) for tc in
                    synth.place_times(rng, int(rng.integers(0, 6)), secs, 1.25, 2.5)]:
            lo = max(0, int(math.floor((inj.tc - inj.tau20 - 0.02) * FS)))
            hi = min(L, int(math.ceil((inj.tc + 0.02) * FS)) + 1)
            if hi > lo:
                x[lo:hi] += torch.from_numpy(synth.injection_signal(inj, lo / FS, hi - lo).astype(np.float32)).cuda()
        bufs.append(x)
    m = gwd.Model(gwd.full_arch(), blobs, prec)
    rows, waves, fuse, batch, blocks, persistent = m.autotune([bufs[0][: 64 * FS]])
    offs = np.concatenate([[0], np.cumsum(lens)])
    total_s = sum(lens) / FS

    def timed_plan():
        plan = m.plan(bufs, W, S, out_mode=0)
        plan.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.launch()
        n_trig = len(gwd.triggers(out, offs, 0.9, 4096))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per, tot = plan.completion_us()
        plan.close()
        return wall, per, tot, n_trig, out.clone()

    wall, per, tot, n_trig, out_a = timed_plan()
    res = {"streams": 32, "stream_seconds_total": round(total_s, 1), "strain_s_per_s": round(total_s / wall, 2),
           "completion_s_p50": round(float(np.percentile(per, 50)) / 1e6, 3),
           "completion_s_p99": round(float(np.percentile(per, 99)) / 1e6, 3),
           "graph_total_s": round(tot / 1e6, 3), "autotune": {"tile_rows": rows, "waves": waves, "layers_per_launch": fuse,
                                                          "batch_windows": batch, "fused_blocks": blocks,
                                                          "persistent": persistent},
           "triggers": n_trig, "precision": prec}
    # the other form of the same request: the persistent launch (in the default fused grouping) if the
    # autotuner chose the launch sequence, else the launch sequence
    m.set_persistent(not persistent)
    if not persistent:
        m.set_tiling(64, 4, 512, 0)
        m.set_fused_blocks(0)
    wall2, per2, tot2, n_trig2, out_b = timed_plan()
    res["persistent_launch" if not persistent else "launch_sequence"] = {
        "strain_s_per_s": round(total_s / wall2, 2),
        "completion_s_p50": round(float(np.percentile(per2, 50)) / 1e6, 3),
        "completion_s_p99": round(float(np.percentile(per2, 99)) / 1e6, 3),
        "graph_total_s": round(tot2 / 1e6, 3), "triggers": n_trig2,
        "scores_identical": bool(torch.equal(out_a, out_b))}
    m.close()
    return res


def background_workload(gwd, blobs, x, prec: str, seconds: float = 900.0, n_slides: int = 4,
                        step_s: float = 64.0):
    """Time-slide background ("Statistical Analysis"): n_slides copies of a stream slice with channel 1
    shifted by k * step_s seconds (circularly), scored in one forward call as ragged streams; the
    false-alarm curve of their triggers."""
    import torch
    xs = x[: int(round(seconds * FS))]
    L = xs.shape[0]
    shifts = [k * int(step_s * FS) for k in range(1, n_slides + 1)]
    m = gwd.Model(gwd.full_arch(), blobs, prec)
    warm = gwd.time_slide(xs[: 64 * FS], shifts)
    m.forward([warm[k] for k in range(n_slides)], W, S, out_mode=0)
    del warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slid = gwd.time_slide(xs, shifts)
    e = m.forward([slid[k] for k in range(n_slides)], W, S, out_mode=0)
    recs = gwd.triggers(e, [k * L for k in range(n_slides + 1)], 0.9, 4096)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.close()
    live = n_slides * L / FS
    probs = [0.9, 0.99, 0.999, 0.9998]
    counts, far = gwd.far_curve(recs, [math.log(p / (1 - p)) for p in probs], live)
    return {"slides": n_slides, "slide_step_s": step_s, "slice_s": round(L / FS, 1), "background_s": round(live, 1),
            "strain_s_per_s": round(live / wall, 2), "triggers": len(recs),
            "false_alarms_per_hour": {str(p): round(float(f) * 3600.0, 2) for p, f in zip(probs, far)},
            "counts": {str(p): int(c) for p, c in zip(probs, counts)}, "precision": prec,
            "note": "random-weight members: the rates show the mechanism, not a trained model's background"}


def postproc_workload(gwd, blobs, x, prec: str, seconds: float = 900.0, height: float = 0.9,
                      width_s: float = 0.5):
    """The paper's post-processing: each member's stitched logits (one forward call, out_mode 1) to
    float64 probabilities, peaks of height >= 0.9 and width >= 0.5 s per member, and the events all
    members report within 0.5 s. Timed apart from the forward."""
    import torch
    xs = x[: int(round(seconds * FS))]
    L = xs.shape[0]
    M = blobs.shape[0]
    m = gwd.Model(gwd.full_arch(), blobs, prec)
    out = m.forward([xs], W, S, out_mode=1)
    torch.cuda.synchronize()
    p = torch.empty(L, dtype=torch.float64, device="cuda")
    gwd.find_peaks(gwd.prob64(out[L: 2 * L], out=p), height, width_s * FS)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lists = []
    for k in range(M):
        gwd.prob64(out[(k + 1) * L: (k + 2) * L], out=p)
        lists.append(gwd.find_peaks(p, height, width_s * FS)[0])
    events = gwd.coincidence(lists, int(width_s * FS))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # context, untimed: member 0's peaks above the height at any width (random-weight members give
    # narrow peaks, so few or none reach 0.5 s)
    any_width = len(gwd.find_peaks(gwd.prob64(out[L: 2 * L], out=p), height, 0.0)[0])
    m.close()
    return {"slice_s": round(L / FS, 1), "members": M, "height": height, "min_width_s": width_s,
            "peaks_per_member": [int(len(q)) for q in lists], "member0_peaks_any_width": any_width,
            "coincident_events": len(events),
            "postproc_s": round(wall, 4), "strain_s_per_s": round(L / FS / wall, 1), "precision": prec}


def two_branch_workload(gwd, x, prec: str, seconds: float = 256.0, members: int = 4):
    """The paper's two-branch topology (Fig. 1: one gated branch of 64 channels per detector, skip sums
    concatenated into the 128-channel head): a 4-member ensemble scored and thresholded like the main
    line. It runs as the block-diagonal 128-channel trunk on the same fused kernels, whose waves take
    only their own branch's k-steps (the zero blocks are skipped), so the MFMA work done is the
    two-branch member's own: half the trunk's."""
    import torch
    from paper_2201_11133_amd import synth
    xs = x[: int(round(seconds * FS))]
    L = xs.shape[0]
    blobs = np.stack([synth.two_branch_weights(21 + i) for i in range(members)])
    m = gwd.Model(gwd.two_branch_arch(), blobs, prec)
    out = torch.empty(L, dtype=torch.float32, device="cuda")
    m.forward([xs[: 64 * FS]], W, S, out_mode=0, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.forward([xs], W, S, out_mode=0, out=out)
    n_trig = len(gwd.triggers(out, [0, L], 0.9, 4096))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.close()
    nw = n_windows(L)
    own = members * (nw * W * FLOP_LAYERS_T_2B + L * FLOP_HEAD_T) / wall / 1e12
    return {"slice_s": round(L / FS, 1), "members": members, "precision": prec, "triggers": n_trig,
            "strain_s_per_s": round(L / FS / wall, 2), "tflops": round(own, 1),
            "flop_per_window_step": FLOP_LAYERS_T_2B,
            "note": "block-diagonal image on the trunk's fused kernels with the zero blocks skipped "
                    "(bit-identical to the dense run)"}


def whitening_workload(gwd, seconds: float = 4096.0, nperseg: int = 16384, reps: int = 5):
    """The front end before the networks ("Data preparation"): the Welch PSD of a coloured
    two-channel stream (4 s Hann segments, half overlap) and the whitening of the whole stream by it,
    scaled to unit deviation. The paper's data segments are 4096 s at 4096 Hz: 2^24 samples per
    detector. Algorithmic HBM bytes per time step: 8 read by the PSD, 8 read and 8 written by the
    whitening (both channels, fp32), 24 in all."""
    import torch
    from paper_2201_11133_amd import synth
    L = int(round(seconds * FS))
    x = torch.from_numpy(synth.coloured_stream(2024, L)).cuda()
    psd = torch.empty((2, nperseg // 2 + 1), dtype=torch.float64, device="cuda")
    y = torch.empty((L, 2), dtype=torch.float32, device="cuda")
    gwd.whiten(x, gwd.welch_psd(x, nperseg, FS, out=psd), nperseg, FS, True, out=y)   # warm-up (workspace)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_psd, t_wh = [], []
    t0 = time.perf_counter()
    for _ in range(reps):
        ev[0].record()
        gwd.welch_psd(x, nperseg, FS, out=psd)
        ev[1].record()
        gwd.whiten(x, psd, nperseg, FS, True, out=y)
        ev[2].record()
        ev[2].synchronize()
        t_psd.append(ev[0].elapsed_time(ev[1]))
        t_wh.append(ev[1].elapsed_time(ev[2]))
    wall = (time.perf_counter() - t0) / reps
    ms_psd, ms_wh = float(np.median(t_psd)), float(np.median(t_wh))
    gbs = 24.0 * L / ((ms_psd + ms_wh) * 1e-3) / 1e9
    sd = [round(float(v), 6) for v in torch.std(y, dim=0, unbiased=False).tolist()]
    del x, y
    return {"stream_s": seconds, "samples_per_channel": L, "nperseg": nperseg,
            "ms_psd": round(ms_psd, 3), "ms_whiten": round(ms_wh, 3), "ms_wall": round(wall * 1e3, 3),
            "strain_s_per_s": round(seconds / wall, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(gbs / 8000.0, 4), "algorithmic_bytes_per_step": 24},
            "output_std": sd}


def train_workload(gwd, steps: int = 2, B: int = 256, curve_steps: int = 60):
    """Training of one full-size member: BF16 forward with per-stack checkpoints, BCE on logits,
    hand-written backward (bf16-operand row and weight-gradient GEMMs, fp32 accumulation), Adam on fp32 master
    weights; batches of 256 windows of 2 x 4096,
    half of them chirped (SNR 8-20), labels 1 within 0.1 s of the coalescence time. Then the loss
    curve of a fresh member over curve_steps steps on fresh seeded batches."""
    import torch
    from paper_2201_11133_amd import synth
    blob = synth.full_weights(4)
    m = gwd.Model(gwd.full_arch(), blob, "bf16")
    tr = gwd.Trainer(m, blob, B, W)
    x, injs = synth.make_windows(104, B, B // 2)
    y = np.zeros((B, W), np.float32)
    for i, inj in injs:
        y[i] = synth.box_labels(W, inj.tc)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    tr.step(xd, yd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss, norm = tr.step(xd, yd)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    m.close()
    # loss curve: a fresh member trained on fresh batches (seeded), the mean loss of every 10 steps
    m = gwd.Model(gwd.full_arch(), blob, "bf16")
    tr = gwd.Trainer(m, blob, B, W)
    curve, acc = [], []
    for step in range(curve_steps):
        xb, ib = synth.make_windows(5000 + step, B, B // 2)
        yb = np.zeros((B, W), np.float32)
        for i, inj in ib:
            yb[i] = synth.box_labels(W, inj.tc)
        acc.append(float(tr.step(torch.from_numpy(xb).cuda(), torch.from_numpy(yb).cuda())[0].item()))
        if len(acc) == 10:
            curve.append(round(float(np.mean(acc)), 4))
            acc = []
    m.close()
    return {"train_windows_per_s": round(B / dt, 1), "s_per_step": round(dt, 3), "batch": B,
            "loss": round(float(loss.item()), 5), "grad_norm": round(float(norm.item()), 5),
            "loss_curve": {"steps": curve_steps, "mean_loss_per_10_steps": curve,
                           "data": "fresh seeded batches of 256 windows per step, half chirped"},
            "precision": "bf16 forward and recompute, bf16-operand row and weight-gradient GEMMs in the "
                         "backward (fp32 accumulation), fp32 master weights and Adam"}


def cpu_baseline(n_members: int, n_windows_sample: int = 3):
    """The FP64 oracle, windowed (the same algorithm and work as the GPU path), on a bounded sample:
    n_windows_sample consecutive windows for every member; the strain they add is S samples each."""
    import torch  # noqa: F401  (thread count report only)
    from oracle.arch import FULL, unpack
    from oracle.forward import forward_window
    from oracle.stream import gather_windows
    from paper_2201_11133_amd import synth
    x, _ = synth.make_stream(102, (W + (n_windows_sample - 1) * S) / FS, 0)
    win = gather_windows(x.astype(np.float64), W, S)[:n_windows_sample]
    ps = [unpack(FULL, synth.full_weights(11 + i).astype(np.float64)) for i in range(n_members)]
    t0 = time.perf_counter()
    for p in ps:
        forward_window(FULL, p, win)
    dt = time.perf_counter() - t0
    strain_s = n_windows_sample * S / FS
    cores = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max((i.get("num_threads", 0) for i in info), default=cores) or cores
    except Exception:
        pass
    # the same oracle held to one BLAS thread, on one window of one member, scaled to the ensemble
    single = None
    try:
        import threadpoolctl
        with threadpoolctl.threadpool_limits(1):
            t1 = time.perf_counter()
            forward_window(FULL, ps[0], win[:1])
            d1 = time.perf_counter() - t1
        single = {"value": round(S / FS / (d1 * n_members), 6), "unit": "strain-s/s", "cores": 1,
                  "sample": f"1 window x 1 member ({d1:.1f} s), scaled to {n_members} members"}
    except Exception:
        pass
    # the oracle's streaming form: one causal pass over a whole stream gives the same stitched scores
    # with 1/16 of the windowed work (a separate line, like the GPU's streaming variant)
    from oracle.forward import forward_stream
    xs, _ = synth.make_stream(102, 8.0, 0)
    t2 = time.perf_counter()
    forward_stream(FULL, ps[0], xs.astype(np.float64))
    d2 = time.perf_counter() - t2
    streaming = {"value": round(8.0 / (d2 * n_members), 6), "unit": "strain-s/s", "cores": int(cores),
                 "sample": f"8 s x 1 member, streaming form ({d2:.1f} s), scaled to {n_members} members"}
    return {"value": round(strain_s / dt, 6), "unit": "strain-s/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_windows_sample} windows x {n_members} members, windowed FP64 NumPy ({dt:.1f} s)",
            "single_thread": single, "streaming_form": streaming}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--seconds", type=float, default=3600.0)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32/FP8 comparison lines")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ragged", action="store_true", help="skip the 32-stream ragged graph workload")
    ap.add_argument("--no-train", action="store_true", help="skip the training-throughput measurement")
    ap.add_argument("--no-streaming", action="store_true", help="skip the long-window (streaming) line")
    ap.add_argument("--no-background", action="store_true", help="skip the time-slide background line")
    ap.add_argument("--no-postproc", action="store_true", help="skip the peak-finding post-processing line")
    ap.add_argument("--no-whiten", action="store_true", help="skip the whitening front-end line")
    ap.add_argument("--no-two-branch", action="store_true", help="skip the two-branch topology line")
    ap.add_argument("--stream-day", action=argparse.BooleanOptionalAction, default=True,
                    help="also run the streaming line over a full day (86400 s) of strain")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(windows shard by time with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_11133_amd import gwd, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        progress("calibration copy of 1 GiB done")
    progress(f"generating a {args.seconds:.0f} s stream on the device")
    x, injs = make_stream_gpu(args.seconds, 102)
    L = x.shape[0]
    blobs = np.stack([synth.full_weights(11 + i) for i in range(args.members)])
    out = torch.empty(L, dtype=torch.float32, device="cuda")
    result = {}

    def run(prec, seconds=None):
        xs = x if seconds is None else x[: int(round(seconds * FS))]
        m = gwd.Model(gwd.full_arch(), blobs, prec)
        n_trig = [0]

        def step(xx=xs):
            m.forward([xx], W, S, out_mode=0, out=out)
            n_trig[0] = len(gwd.triggers(out[: xx.shape[0]], [0, xx.shape[0]], 0.9, 4096))

        # warm-up passes run the same code on a 64 s prefix (kernels, workspace, caches)
        ms_ev, ms_wall = time_steps(step, args.steps, args.warmup, prec, lambda: step(xs[: 64 * FS]))
        progress(f"{prec}: {ms_wall / 1e3:.2f} s per step")
        secs = xs.shape[0] / FS
        return m, {"strain_s_per_s": secs / (ms_wall / 1e3), "ms_per_step": ms_wall, "ms_events": ms_ev,
                   "stream_s": secs, "triggers": n_trig[0],
                   "tflops": args.members * (n_windows(xs.shape[0]) * W * FLOP_LAYERS_T + xs.shape[0] * FLOP_HEAD_T)
                   / (ms_wall * 1e-3) / 1e12}

    model, main_r = run(args.precision)
    ref_scores = out.clone()
    progress("dominant-kernel timing")
    roof = layer_kernel_timing(model, args.precision)
    model.close()
    streaming = None
    if not args.no_streaming:
        streaming = streaming_line(gwd, blobs, x, out, ref_scores, args)
        progress(f"streaming variant: {streaming['strain_s_per_s']} strain-s/s")
    del ref_scores
    extra = {}
    if not args.no_extra:
        for prec, secs in (("fp8", None), ("fp32", min(args.seconds, 256.0))):
            if prec == args.precision:
                continue
            m2, r2 = run(prec, secs)
            m2.close()
            extra[prec] = {k: round(v, 3) if isinstance(v, float) else v for k, v in r2.items()}
        extra[args.precision] = {k: round(v, 3) if isinstance(v, float) else v for k, v in main_r.items()}
        for prec in extra:
            extra[prec]["accuracy"] = ACCURACY[prec]
    ragged = None
    if not args.no_ragged:
        progress("ragged workload: 32 streams, one graph launch")
        ragged = ragged_workload(gwd, blobs, args.precision)
        progress(f"ragged: {ragged['strain_s_per_s']} strain-s/s over {ragged['stream_seconds_total']} s")
    background = None
    if not args.no_background:
        progress("time-slide background")
        background = background_workload(gwd, blobs, x, args.precision, min(900.0, args.seconds))
        progress(f"background: {background['strain_s_per_s']} strain-s/s over {background['background_s']} s")
    postproc = None
    if not args.no_postproc:
        progress("post-processing: peaks and coincidence")
        postproc = postproc_workload(gwd, blobs, x, args.precision, min(900.0, args.seconds))
        progress(f"post-processing: {postproc['strain_s_per_s']} strain-s/s")
    two_branch = None
    if not args.no_two_branch:
        progress("two-branch topology: 4 members")
        two_branch = two_branch_workload(gwd, x, args.precision, min(256.0, args.seconds))
        progress(f"two-branch: {two_branch['strain_s_per_s']} strain-s/s")
    whitening = None
    if not args.no_whiten:
        progress("whitening front end: Welch PSD and whitening of a 4096 s stream")
        whitening = whitening_workload(gwd)
        progress(f"whitening: {whitening['strain_s_per_s']} strain-s/s")
    train = None
    if not args.no_train:
        progress("training throughput")
        train = train_workload(gwd)
        progress(f"training: {train['train_windows_per_s']} windows/s")
    progress("CPU oracle baseline")
    cpu = None if args.no_cpu else cpu_baseline(args.members)
    value = main_r["strain_s_per_s"]
    line = {
        "metric": "2-detector strain-sec/s per GPU, 4-model ensemble, FP32 vs BF16/FP8; train win/s",
        "value": round(value, 3), "unit": "strain-s/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main_r["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": (f"ensemble of {args.members} gated dilated-conv members (3x10 layers, 128 "
                                f"channels), {args.precision} operands / fp32 accumulation, "
                                f"{args.seconds:.0f} s two-channel 4096 Hz stream slice (white noise + "
                                f"chirps), window 4096 stride 256, ensemble min + triggers (p>=0.9, +/-4096)"),
                   "members": args.members, "stream_seconds": args.seconds, "window": W, "stride": S,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": {"triggers": main_r["triggers"], "tflops_step": round(main_r["tflops"], 2),
                   "ms_events": round(main_r["ms_events"], 3), "precisions": extra,
                   "ragged_streams": ragged, "time_slide_background": background, "postprocessing": postproc,
                   "whitening_front_end": whitening, "two_branch": two_branch, "training": train,
                   "streaming_variant": streaming},
    }
    print(json.dumps(line), flush=True)



if __name__ == "__main__":
    main()
