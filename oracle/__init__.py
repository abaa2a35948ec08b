"""Plain FP64 CPU oracle for the ensemble gravitational-wave search hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import or call it. The product path
(the HIP library and its Python binding) never imports it and shares no code
with it: every function here is written from the paper and from the plain
mathematical definition of each step, in float64 NumPy, with no blocking,
fusion or reordering beyond what the definition states.

Paper: "Inference-optimized AI and high performance computing for
gravitational wave detection at scale" (arXiv 2201.11133).

Modules
  arch      architecture descriptors, parameter counts, receptive field,
            canonical flat weight-blob layout
  forward   per-window forward pass, per-layer forward, streaming forward
  stream    sliding windows over a stream, owner-window stitching, ensemble
  triggers  threshold + non-maximum-suppression trigger rule (+ brute force)
  train     per-timestep BCE loss, manual reverse-mode gradient, Adam
  quant     bfloat16 and FP8-E4M3 quantisers written from the formats
  background  time-slid copies of a two-channel stream and the false-alarm
            count per threshold ("Statistical Analysis")
  postproc  the paper's peak finding (SciPy find_peaks: height, width >= 0.5 s)
            and all-member coincidence within 0.5 s
  whiten    the front end ("Data preparation"): Welch PSD, whitening of the
            stream by it, unit standard deviation
"""
