/*
 * gwd.h — C ABI of libgwd, the MI355X (gfx950) hot path of an ensemble
 * gravitational-wave search over two-detector strain.
 *
 * Paper: "Inference-optimized AI and high performance computing for
 * gravitational wave detection at scale" (arXiv 2201.11133).
 *
 * What the library computes (each entry point below names its passage):
 *   - an ensemble of dilated causal 1-D convolutional classifiers (a modified
 *     WaveNet, Materials and Methods "AI architecture", Fig. 1) applied to
 *     sliding windows of two-channel (Hanford, Livingston) strain sampled at
 *     4096 Hz, one logit per time step and window ("Optimization with
 *     TensorRT": the engine maps (batch, 4096, 2) windows to (batch, 4096, 1));
 *   - the per-sample ensemble score (minimum over members: a sample passes
 *     the threshold only if every member passes it, Results "Event Detection");
 *   - threshold + clustering of that score into a trigger list;
 *   - a hand-written backward pass and Adam step for training one member
 *     ("AI ensemble construction": per-timestep labels, random initialisation).
 *
 * Conventions
 *   - Every function returns gwd_status (0 = OK, negative = error) unless its
 *     return type says otherwise; gwd_last_error() gives a thread-local text.
 *   - No C++ exception and no abort crosses this ABI.
 *   - All argument checks run on the host before any HIP call, so invalid
 *     arguments are reported even on a machine without a GPU.
 *   - Device pointers are owned by the caller (for example torch CUDA/ROCm
 *     tensors) and must stay valid until the enqueued work completes.
 *   - The library owns only the opaque model handle: packed weights, scales,
 *     workspace and launch plans. A model lives on the device that was current
 *     when gwd_load_weights was called; call it with that device current.
 *   - Every enqueueing call takes `hip_stream` (a hipStream_t; NULL = the
 *     default stream) and is asynchronous with respect to the host, except
 *     where stated (gwd_load_weights, gwd_triggers).
 *   - Calls that share one model handle must not overlap in time (they share
 *     its workspace); use one handle per host thread for concurrency.
 */
#ifndef GWD_H
#define GWD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gwd_model gwd_model; /* opaque, library-owned */

typedef enum {
    GWD_FP32 = 0,     /* fp32 storage and operands; the dilated-conv GEMM accumulates in fp64,
                         the res/skip GEMM in fp32                                          */
    GWD_BF16 = 1,     /* bf16 operands (RNE), fp32 accumulation, bf16 residual stream
                         between layers, fp32 skip sum                                      */
    GWD_FP8_E4M3 = 2, /* OCP E4M3FN operands, per-output-channel weight scales            */
    GWD_FP64 = 3      /* plain member only, training entry points only: everything in fp64
                         (device finite-difference gradient checks)                         */
} gwd_precision;

typedef enum {
    GWD_OK = 0,
    GWD_ERR_ARG = -1,         /* null/misaligned pointer, value out of range      */
    GWD_ERR_SHAPE = -2,       /* window shorter than the receptive field, ...     */
    GWD_ERR_CAPACITY = -3,    /* caller buffer too small (true size is reported)  */
    GWD_ERR_HIP = -4,         /* a HIP runtime call failed                         */
    GWD_ERR_UNSUPPORTED = -5, /* valid but not implemented combination            */
    GWD_ERR_NONFINITE = -6,   /* NaN/Inf in a score stream                          */
    GWD_ERR_NO_DEVICE = -7    /* no HIP device visible                              */
} gwd_status;

/* Architecture of one ensemble member (all members of a model share it).
 * kind 0: plain stack — n_stacks*layers_per_stack causal convolutions of
 *         `channels` channels, kernel `kernel_size`, dilation
 *         2^(l mod layers_per_stack), ReLU after each, then a 1x1 to one logit.
 * kind 1: gated residual WaveNet — 1x1 input projection in_channels ->
 *         channels, then n_stacks*layers_per_stack layers
 *           a = dilated causal conv (kernel 2) of x, 2*channels outputs
 *           g = tanh(a[0:C]) * sigmoid(a[C:2C])
 *           skip += W_s g + b_s ;  x += W_r g + b_r  (no residual in the last layer)
 *         then logit = w_h2 . act(W_h1 ReLU(skip) + b_h1) + b_h2 with
 *         act = identity (head_mid_relu = 0) or ReLU (head_mid_relu = 1).
 * kind 2: two-branch (the paper's Fig. 1) — one kind-1 trunk per detector,
 *         each reading its own input channel (in_channels must be 2: branch b
 *         reads channel b) with `channels` residual and `skip_channels` skip
 *         channels; the two skip sums are concatenated (detector 0 first) and
 *         go through the kind-1 head with W_h1 of [head_channels][2 *
 *         skip_channels]. Blob: branch 0's trunk tensors (in.W[C][1] .. the
 *         last skip.b), branch 1's, then h1.W, h1.b, h2.W, h2.b.
 * The paper (Fig. 1) does not give widths or depths; these are the build's
 * members. Supported by the GPU path: kind 0 with channels 16, in_channels 2,
 * kernel 2; kind 1 with channels = skip_channels = head_channels = 128,
 * in_channels 2, kernel 2, input_kernel 1; kind 2 with channels =
 * skip_channels = 64, head_channels = 128, kernel 2, input_kernel 1, which
 * gwd_load_weights expands into the block-diagonal kind-1 member of 128
 * channels and runs on the same kernels; its BF16 fused kernels skip the
 * zero blocks. Training (FP32 and BF16 models) takes and returns the kind-2
 * blob layout: gwd_backward writes dL/dparams of the branch blob (the trunk
 * image's gradient read back at each branch parameter's place) and
 * gwd_adam_step updates the branch blob, then re-expands the working weights.
 * gwd_debug_export_weights returns the expanded kind-1 blob. */
typedef struct {
    int32_t kind;
    int32_t in_channels;
    int32_t channels;
    int32_t skip_channels;
    int32_t head_channels;
    int32_t n_stacks;
    int32_t layers_per_stack;
    int32_t kernel_size;
    int32_t input_kernel;
    int32_t head_mid_relu;
} gwd_arch;

/* One two-channel strain stream in device memory: sample t of channel c is
 * ch[c][t * elem_stride], t in [0, length). Planar (elem_stride 1, two
 * pointers) and interleaved (elem_stride 2, ch[1] = ch[0] + 1) both work
 * without a copy. */
typedef struct {
    const float* ch[2];
    int64_t elem_stride;
    int64_t length;
} gwd_stream;

/* One trigger: stream index, sample index within that stream, ensemble logit
 * and its sigmoid. */
typedef struct {
    int32_t stream;
    int32_t _pad;
    int64_t sample;
    float logit;
    float prob;
} gwd_trigger;

/* Number of float parameters of one member in the canonical flat blob (the
 * paper's members are the gated dilated-convolution networks of "AI
 * architecture", Fig. 1; their widths and depths are this library's reading)
 * (kind 0 with 16 channels: 1,681; kind 1 with 128 channels, 3x10 layers:
 * 2,964,993; kind 2 with two 64-channel branches and a 128-channel head:
 * 1,498,497), or -1 for an invalid descriptor.
 * Blob order (float32):
 *   kind 0: for each layer i: W[channels][c_in][kernel], b[channels]
 *           (c_in = in_channels for i = 0, else channels); out.W[1][channels], out.b[1]
 *   kind 1: in.W[C][in_channels], in.b[C];
 *           for layer l: dil.W[2C][C][2], dil.b[2C],
 *                        res.W[C][C], res.b[C]   (absent in the last layer),
 *                        skip.W[S][C], skip.b[S];
 *           h1.W[H][S], h1.b[H], h2.W[1][H], h2.b[1]
 *   kind 2: for branch b = 0, 1: the kind-1 tensors from in.W[C][1] to the
 *           last skip.b[S]; then h1.W[H][2S], h1.b[H], h2.W[1][H], h2.b[1]
 *   Kernel tap 0 multiplies x[t - d], tap 1 multiplies x[t]. */
int64_t gwd_num_params(const gwd_arch* arch);

/* Input samples that influence one output sample ("AI architecture": stacks
 * of causal convolutions with doubling dilations): 1 + (kernel-1) * sum of
 * dilations (16 for the plain member, 3070 for the gated and two-branch
 * members), or -1 if invalid. */
int32_t gwd_receptive_field(const gwd_arch* arch);

/* Build the inference engine of an ensemble once ("Optimization with
 * TensorRT": one engine per model, half precision where it can be used):
 * copy, pack and (for BF16 / FP8) quantise the weights of n_members members
 * onto the current device. host_blob holds n_members consecutive blobs of
 * n_params floats each (host memory, read during the call only). BF16 rounds
 * to nearest even; FP8 E4M3 uses one scale per output channel of every
 * weight matrix (max |w| over the channel / 448) and saturates at +/-448.
 * precision is one of the gwd_precision values (passed as int32_t, so any
 * other value is an argument error rather than an invalid enumeration).
 * Synchronous. On success *out owns device memory until gwd_free. */
gwd_status gwd_load_weights(const gwd_arch* arch, int32_t n_members, const float* host_blob,
                            int64_t n_params, int32_t precision, gwd_model** out);

/* Release a model (waits for the device; NULL is ignored). */
void gwd_free(gwd_model* model);

/* Forward pass of every member over every window of every stream
 * (windows: "Data preparation" — 1 s at 4096 Hz; the engine batch —
 * "Optimization with TensorRT").
 *
 * Window k of a stream covers samples [k*stride, k*stride + window); samples
 * at or past the stream length read as 0; each window starts from zero
 * context. A stream of length L has n_win = 1 if L <= window, else
 * ceil((L - window) / stride) + 1 windows. Each sample a is scored by its
 * owner window: window 0 for a < window - stride, else
 * k = floor((a - window + stride) / stride) at position a - k*stride.
 * Ensemble score e[a] = minimum over members of the owner-window logits.
 *
 * out_mode and the layout of `out` (device, float32):
 *   0: e for every stream, streams back to back:          [sum L]
 *   1: as 0, followed by each member's stitched logits:   [sum L] + [M][sum L]
 *   2: every member's full per-window logits:             [M][sum n_win][window]
 * out_capacity_floats must be >= gwd_forward_out_floats(...).
 * Requirements: 1 <= n_streams <= 65536, window a multiple of 128 (256 for
 * the plain member) and
 * >= receptive field (else GWD_ERR_SHAPE), 0 < stride <= window,
 * window - stride >= receptive field - 1 (so owner positions never see the
 * zero left context of a later window, else GWD_ERR_SHAPE), stream pointers
 * 4-byte aligned. Streams with length 0 are allowed and produce nothing.
 * Asynchronous on hip_stream. */
gwd_status gwd_forward(gwd_model* model, const gwd_stream* streams, int32_t n_streams,
                       int32_t window, int32_t stride, int32_t out_mode,
                       float* out, int64_t out_capacity_floats, void* hip_stream);

/* Number of floats gwd_forward writes for these arguments (or -1 if invalid). */
int64_t gwd_forward_out_floats(const gwd_model* model, const gwd_stream* streams, int32_t n_streams,
                               int32_t window, int32_t stride, int32_t out_mode);

/* Threshold + clustering of ensemble scores into triggers (the paper's
 * post-processing keeps a candidate only if all members flag it, Results
 * "Event Detection", and locates each merger with a peak search, "AI ensemble
 * construction"). Rule, per stream (samples never interact across streams):
 *   sample a triggers iff  e[a] >= ln(p / (1 - p))   (p = threshold_prob), and
 *   e[a] >  e[b] for all b in [a - cluster_window, a), and
 *   e[a] >= e[b] for all b in (a, a + cluster_window]
 * i.e. non-maximum suppression over +/-cluster_window, ties to the earliest.
 * The comparison with the threshold is done in double precision.
 * ens_logit: device [stream_offsets[n_streams]] floats; stream s is
 * ens_logit[stream_offsets[s] .. stream_offsets[s+1]) (host offsets,
 * non-decreasing, starting at 0). Records are written to host memory `out`
 * sorted by (stream, sample); *n_found receives the true count. If it
 * exceeds `capacity`, the first `capacity` records are written and
 * GWD_ERR_CAPACITY is returned. Any NaN or Inf in the scanned scores gives
 * GWD_ERR_NONFINITE (and no records). 0 < threshold_prob < 1,
 * 1 <= cluster_window <= 65536. Synchronises hip_stream before returning. */
gwd_status gwd_triggers(const float* ens_logit, const int64_t* stream_offsets, int32_t n_streams,
                        double threshold_prob, int32_t cluster_window, gwd_trigger* out,
                        int64_t capacity, int64_t* n_found, void* hip_stream);

/* Allocation-free form of gwd_triggers, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc). Same rule,
 * arguments, records and errors as gwd_triggers, and the same kernels, but the
 * per-tile candidates, the stream table, the records and the counters live in
 * a fixed device array of 16 MiB (16,777,216 bytes) that the library holds on
 * each device it runs on until the process ends; the call allocates nothing.
 * A request needing more scratch than that gives GWD_ERR_CAPACITY before any
 * device work (*n_found stays 0); the need is
 *   256-aligned(32 n_streams) + 256-aligned(8 n_tiles) + 256-aligned(24 n_tiles) + 256
 * bytes, n_tiles = sum over streams of ceil(length / cluster_window), and
 * gwd_triggers_noalloc_scratch_bytes reports it (-1 for invalid offsets or
 * sizes). Calls on one device share its array: the library serialises them
 * (a process-wide lock held until the call has synchronised hip_stream), and
 * the array keeps the last call's contents, which no call reads. */
gwd_status gwd_triggers_noalloc(const float* ens_logit, const int64_t* stream_offsets, int32_t n_streams,
                                double threshold_prob, int32_t cluster_window, gwd_trigger* out,
                                int64_t capacity, int64_t* n_found, void* hip_stream);
int64_t gwd_triggers_noalloc_scratch_bytes(const int64_t* stream_offsets, int32_t n_streams,
                                           int32_t cluster_window);

/* ---- time-slide background ("Statistical Analysis") -------------------------
 * The paper measures how often the ensemble fires on noise with years of
 * background built from one month of two-detector data by time slides: one
 * detector's strain is shifted against the other's by far more than the
 * light travel time between the sites, so no astrophysical coincidence
 * survives and every trigger in slid data is a false positive.
 *
 * gwd_time_slide writes, for each shift k, the slid copy of `src` as an
 * interleaved device stream at dst + 2 * length * k (feed it to gwd_forward
 * with elem_stride 2):
 *   dst[k][t][0] = ch0[t],   dst[k][t][1] = ch1[(t + shifts[k]) mod length]
 * for t in [0, length): channel 0 stays, channel 1 is read shifts[k] samples
 * later, circularly over the stream. shifts: host array of n_shifts values of
 * any sign and size (taken modulo length). The copies are plain fp32 moves.
 * dst: device, 2 * length * n_shifts floats, 8-byte aligned, not overlapping
 * the source. length 0 writes nothing. GWD_ERR_ARG for NULL pointers, n_shifts
 * < 1, elem_stride < 1, length < 0 or misaligned pointers. Asynchronous on
 * hip_stream. */
gwd_status gwd_time_slide(const gwd_stream* src, const int64_t* shifts, int32_t n_shifts, float* dst,
                          void* hip_stream);

/* False-alarm counts of a background trigger list (host memory, no device
 * work): counts[i] = number of records with logit >= thresholds[i] (compared in
 * double), far_per_s[i] = counts[i] / livetime_s. The clustering rule of
 * gwd_triggers does not involve the threshold, so the records found at the
 * lowest threshold give the whole curve above it; thresholds below that one
 * are undercounted. GWD_ERR_ARG for NULL pointers (n > 0 needs trig), n < 0,
 * n_thr < 1 or livetime_s <= 0. */
gwd_status gwd_far_curve(const gwd_trigger* trig, int64_t n, const double* thresholds, int32_t n_thr,
                         double livetime_s, int64_t* counts, double* far_per_s);

/* ---- the paper's post-processing ("AI ensemble construction", "Statistical Analysis",
 * "Event Detection") ---------------------------------------------------------
 * The paper locates mergers with SciPy's find_peaks on each model's output,
 * keeps peaks at least 0.5 s wide above a height threshold, and flags an event
 * when all models report it within 0.5 s.
 *
 * gwd_prob64 writes p[i] = 1 / (1 + e^-z[i]) in float64 for float32 logits z
 * (device arrays of n elements); asynchronous on hip_stream.
 *
 * gwd_find_peaks finds the peaks of a float64 device signal x[0, n) with the
 * semantics of scipy.signal.find_peaks(x, height=height, width=min_width):
 *   - a peak is a sample, or the middle (rounded down) of a run of equal
 *     samples, with a strictly lower neighbour on each side; the first and
 *     last samples are never peaks; x[peak] >= height;
 *   - prominence: the peak's height above the higher of the lowest points
 *     reached walking left and right up to a strictly higher sample (or the
 *     end), which are also the bases;
 *   - width: between the crossings of the level x[peak] - prominence / 2
 *     inside the bases, linearly interpolated, in samples; kept if >= min_width.
 * Peak indices (ascending) and widths go to host arrays `peaks` and `widths`;
 * *n_found receives the true count, and if it exceeds `capacity` the first
 * `capacity` are written and GWD_ERR_CAPACITY is returned. NaN or Inf in x
 * gives GWD_ERR_NONFINITE. n < 3 finds nothing (no device work). The
 * prominence and width arithmetic is float64 in the order above, so results
 * equal SciPy's exactly. Synchronises hip_stream before returning.
 *
 * gwd_coincidence (host memory, no device work): peak_lists[m] holds counts[m]
 * ascending peak indices of member m; a peak t of member 0 is an event when
 * every other member has a peak within |t' - t| <= window. Events (ascending)
 * go to `events`, up to `capacity` (GWD_ERR_CAPACITY beyond, *n_events gets the
 * true count). GWD_ERR_ARG for NULL pointers, n_members < 1, negative counts
 * or window. */
gwd_status gwd_prob64(const float* z, int64_t n, double* p, void* hip_stream);
gwd_status gwd_find_peaks(const double* x, int64_t n, double height, double min_width, int64_t* peaks,
                          double* widths, int64_t capacity, int64_t* n_found, void* hip_stream);
gwd_status gwd_coincidence(const int64_t* const* peak_lists, const int64_t* counts, int32_t n_members,
                           int64_t window, int64_t* events, int64_t capacity, int64_t* n_events);

/* ---- whitening front end ("Data preparation") -------------------------------
 * Before the networks see strain, the paper estimates the detector noise's
 * power spectral density (PSD), whitens the strain with it and scales the
 * network input to unit standard deviation. Both functions take one
 * two-channel device stream (gwd_stream above) and treat the channels alike.
 *
 * gwd_welch_psd writes the one-sided Welch PSD of each channel to
 * psd[c * (nperseg/2 + 1) + k] (device, float64, k = 0 .. nperseg/2, bin k at
 * k fs / nperseg Hz): segments of nperseg samples at step nperseg/2 (only
 * full segments, K = (length - nperseg) / (nperseg/2) + 1), periodic Hann
 * window w[j] = 1/2 - 1/2 cos(2 pi j / nperseg), no detrending, mean of
 * |FFT|^2 over the segments, scaled by c_k / (K fs sum w^2) with c_k = 1 at
 * k = 0 and nperseg/2 and 2 elsewhere (scipy.signal.welch with window "hann",
 * noverlap nperseg/2, detrend False). The transforms run in float32; the
 * squared magnitudes and the mean in float64.
 *
 * gwd_whiten writes the whitened stream, interleaved, to dst[t * 2 + c]
 * (device float32 [length][2], 8-byte aligned; dst may be the source's own
 * interleaved buffer): X = DFT of the whole channel (length L), divided bin by
 * bin by sqrt(P(f) fs / 2) with P linearly interpolated at f = m fs / L from
 * the psd grid (same layout as above), inverse DFT; white noise of variance
 * s^2 thus comes out with unit variance. With normalize = 1 each channel is
 * then divided by its population standard deviation (mean not removed). The
 * transforms are float32 (both channels in one complex transform); the
 * coefficients and the deviation float64. The psd must be positive: a zero
 * bin gives non-finite output, as the definition does.
 *
 * Limits and errors: nperseg a power of two in [16, 16384]; fs > 0 and
 * finite; gwd_whiten needs length a power of two in [16, 2^28] and
 * nperseg <= length (GWD_ERR_SHAPE otherwise; a 4096 s segment at 4096 Hz is
 * 2^24 samples); gwd_welch_psd needs length >= nperseg (GWD_ERR_SHAPE).
 * GWD_ERR_ARG for NULL or misaligned pointers, elem_stride < 1 or normalize
 * not 0 or 1. Both use a library-owned workspace (2 L complex float32 for
 * gwd_whiten, 2 G (nperseg/2 + 1) float64 for gwd_welch_psd, G = min(K, 256)
 * for nperseg > 4096, else min(K, 1024)) that grows on
 * demand and is shared by the calls of the process: calls must not overlap
 * in time. Asynchronous on hip_stream (except when the workspace grows). */
gwd_status gwd_welch_psd(const gwd_stream* src, int32_t nperseg, double fs, double* psd, void* hip_stream);
gwd_status gwd_whiten(const gwd_stream* src, const double* psd, int32_t nperseg, double fs, int32_t normalize,
                      float* dst, void* hip_stream);

/* ---- training (one member; "AI ensemble construction") ---------------------
 * windows: device [B][W][2] float32 (interleaved channels). Element type T of
 * logits, grad_logit, grad_params and grad_input is float, or double for a
 * model loaded with GWD_FP64.
 * gwd_forward_train runs member `member` forward over the B windows (each with
 * zero context), writes the logits [B][W] (T) and keeps what the backward pass
 * needs in `saved` (device, caller-owned, gwd_saved_bytes(model, B, W) bytes):
 * for the gated member the input of each stack of layers_per_stack layers and
 * the final skip sum (everything else is recomputed one stack at a time); for
 * the plain member every layer output.
 * gwd_backward takes dL/dlogit [B][W] (T) and the same windows and `saved`,
 * and writes dL/dparams (device T [n_params], overwritten, canonical blob
 * order) and, if grad_input is not NULL, dL/dwindows [B][W][2] (T).
 * The gated member's forward and its per-stack recompute use the model's
 * precision (FP32 or BF16 kernels). For BF16 members the backward's row and
 * weight-gradient GEMMs take bf16 operands (fp32 accumulation); the gradient
 * is fp32, against the fp32 master weights. FP8
 * models are inference only (GWD_ERR_UNSUPPORTED). The gated member needs W a
 * multiple of 128. Calls with one model must not overlap (shared workspace). */
int64_t gwd_saved_bytes(const gwd_model* model, int32_t B, int32_t W);
gwd_status gwd_forward_train(gwd_model* model, int32_t member, const float* windows, int32_t B, int32_t W,
                             void* logits, void* saved, void* hip_stream);
gwd_status gwd_backward(gwd_model* model, int32_t member, const float* windows, int32_t B, int32_t W,
                        const void* saved, const void* grad_logit, void* grad_params,
                        void* grad_input, void* hip_stream);

/* Per-timestep binary cross-entropy on logits (labels 0/1, "AI ensemble
 * construction"): grad[i] = (sigmoid(z_i) - y_i) / n (float32 device), and the
 * mean loss accumulated in double into *loss (device double). */
gwd_status gwd_bce_logits(const float* logits, const float* labels, int64_t n, float* grad, double* loss,
                          void* hip_stream);

/* Adam (Kingma & Ba) with bias correction on float32 master weights
 * (device [n_params], canonical order), gradient, first and second moments
 * (updated in place); step is 1-based. Writes the global gradient 2-norm,
 * accumulated in double, to *grad_norm_out (device, may be NULL), then
 * refreshes member `member`'s working weights (packed operands for the
 * forward kernels and the backward's copy) from the new master weights.
 * No weight decay, no clipping. FP32 and BF16 models. Synchronises
 * hip_stream (the working weights are repacked on the host). */
gwd_status gwd_adam_step(gwd_model* model, int32_t member, float* master, const float* grad, float* m, float* v,
                         int64_t step, float lr, float beta1, float beta2, float eps,
                         double* grad_norm_out, void* hip_stream);

/* ---- captured plans and tuning -------------------------------------------------
 * A plan binds one request (streams, window, stride, out_mode, output buffer —
 * exactly as for gwd_forward) to a hipGraph holding every kernel of the forward:
 * all batches of windows packed across the (ragged) streams, all members, all
 * layers, head, stitch and ensemble minimum, plus a device wall-clock stamp
 * after every batch. gwd_plan_launch replays it with one graph launch; new data
 * written into the same stream buffers is processed by the next launch. The
 * plan owns its own workspace; free plans before their model. Creating a plan
 * synchronises the device. (The paper serialises its engine once and replays
 * it, "Optimization with TensorRT".)
 * gwd_plan_completion_us (after a launch; synchronises the device) gives, per
 * stream, the time from the plan's start to the end of the batch holding the
 * stream's last window (persistent forward: to the end of the stream's last
 * window to finish), and the total, in microseconds. */
typedef struct gwd_plan gwd_plan;
gwd_status gwd_plan_create(gwd_model* model, const gwd_stream* streams, int32_t n_streams, int32_t window,
                           int32_t stride, int32_t out_mode, float* out, int64_t out_capacity_floats,
                           gwd_plan** plan);
gwd_status gwd_plan_launch(gwd_plan* plan, void* hip_stream);
gwd_status gwd_plan_completion_us(gwd_plan* plan, double* per_stream_us, int32_t n_streams, double* total_us);
void gwd_plan_free(gwd_plan* plan);

/* Layer-kernel schedule of a model:
 *   tile_rows, waves: tiling of the single-layer BF16/FP8 kernel, (64, 4),
 *     (64, 8) or (128, 4); (0, 0) = default per precision (BF16 (64, 4), FP8
 *     (64, 8)); FP32 models have one tiling and accept only (0, 0);
 *   layers_per_launch: BF16 and FP8, 3 = fused launches: the layers with
 *     dilations d, 2d, 4d of a stack run as one launch, and the triple at
 *     stack position 6 also takes the stack's last layer (four layers) when
 *     the sub-sequences at its dilation fit one 64-row chunk (window <= 64 x
 *     that dilation, e.g. 4096 at 64); 6 (stacks of ten layers) = sextets:
 *     stack positions 0-5 (dilations 1-32) in one launch, then 6-9 in another
 *     at any window length; 1 = one launch per layer; 0 = default (6 where
 *     sextets apply, else 3); FP32 models accept 0 or 1;
 *   batch_windows: windows per batch of layer launches (1..8192, default 512;
 *     gwd_forward lowers it for a call whose activations would not fit in 60 %
 *     of the free device memory, e.g. windows of 2^20 samples).
 * Results do not depend on any of them. GWD_ERR_ARG for other values. */
gwd_status gwd_set_tiling(gwd_model* model, int32_t tile_rows, int32_t waves, int32_t layers_per_launch,
                          int32_t batch_windows);

/* Shape of the fused launches (BF16/FP8 gated models): the number of blocks a
 * launch aims at. Each interleaved sub-sequence of a window is split into
 * enough segments (each after the first starting with one warm-up chunk that
 * rebuilds its history rows) for windows x sub-sequences x segments to reach
 * `blocks`; 0 restores the default, 512 (two blocks per compute unit). The
 * profiling-based kernel choice of the paper's engine ("Optimization with
 * TensorRT") is gwd_autotune's, which tries 512, 1024 and 2048. Results do not
 * depend on it. GWD_ERR_ARG unless blocks is 0 or in [256, 16384];
 * GWD_ERR_UNSUPPORTED for other models. */
gwd_status gwd_set_fused_blocks(gwd_model* model, int32_t blocks);

/* Persistent forward (BF16/FP8 gated models, on = 1; 0 restores the launch
 * sequence): gwd_forward and plans created afterwards run the whole request as
 * one kernel launch over all members and all windows of all streams. Each
 * block owns a window at a time (windows b, b + grid, ..., grid = two blocks
 * per compute unit, at most one per window) and runs every member's layers
 * (the fused launches' arithmetic over each whole interleaved sub-sequence, in
 * buffers of the block's own) and head on it, the members in order; no block
 * waits for another. Results are bit for bit those of the launch sequence.
 * (The paper's engine is built once and replayed for every batch,
 * "Optimization with TensorRT"; here the whole ragged request is one launch.)
 * It runs the fused grouping set by gwd_set_tiling (sextets and quads, or
 * triples and quads) and needs a fused schedule and windows of up to 4096
 * samples; gwd_forward returns GWD_ERR_UNSUPPORTED otherwise. It leaves the workspace without the batch layout that
 * gwd_debug_time_layer reads. GWD_ERR_ARG unless on is 0 or 1;
 * GWD_ERR_UNSUPPORTED for other models (FP32, small member, two-branch). */
gwd_status gwd_set_persistent(gwd_model* model, int32_t on);

/* Autotuner (the engine's kernel choice by profiling, "Optimization with
 * TensorRT"): times gwd_forward (out_mode 0) on the given request for every
 * schedule candidate (BF16/FP8: fused launches aiming at 512, 1024 and 2048
 * blocks, with stacks of ten layers also sextets aiming at 512 and 1024,
 * and the three tilings one layer per launch; all: batch 256, 512,
 * 1024 windows; BF16/FP8 gated models where the window allows it: the
 * persistent forward), keeps the fastest on the model and reports it
 * (*fused_blocks is 0 for schedules without fused launches, *persistent 1 for
 * the persistent forward; either pointer may be NULL). If the environment
 * variable GWD_AUTOTUNE_CACHE names a file, a cached choice for the same
 * (architecture, precision, members, window, stride) is used instead of
 * timing, and new choices are appended to it. Synchronises hip_stream. */
gwd_status gwd_autotune(gwd_model* model, const gwd_stream* streams, int32_t n_streams, int32_t window,
                        int32_t stride, float* out, int64_t out_capacity_floats, int32_t* tile_rows,
                        int32_t* waves, int32_t* layers_per_launch, int32_t* batch_windows,
                        int32_t* fused_blocks, int32_t* persistent, void* hip_stream);

/* Last error message of the calling thread ("" if none). */
const char* gwd_last_error(void);

/* ---- test support ------------------------------------------------------------
 * gwd_debug_layer runs gated layer `layer` of member `member` (kind 1) with
 * the model's single-layer kernel (the one the forward uses with one layer
 * per launch; the default forward fuses three or four layers per launch, see
 * gwd_debug_fused, and computes every output with the same operations in the
 * same order), on M = n_windows * window rows of
 * device input x_in [n_windows][window][C] (each window zero-context), and
 * writes the pre-activation a [M][2C] (may be NULL), x_out [M][C] (ignored in
 * the last layer) and updates skip [M][S] in place (skip_inout; it is
 * overwritten rather than accumulated when `layer` is 0).
 * gwd_debug_export_weights copies the operands exactly as the kernels see
 * them, unpacked to row-major float32: for every weight matrix of member
 * `member` in blob order, the de-quantised values (bf16 / e4m3 value times
 * scale), into host `out` of n_params floats (biases copied as stored). */
gwd_status gwd_debug_layer(gwd_model* model, int32_t member, int32_t layer, const float* x_in,
                           int32_t n_windows, int32_t window, float* pre_out, float* x_out,
                           float* skip_inout, void* hip_stream);
gwd_status gwd_debug_export_weights(const gwd_model* model, int32_t member, float* out, int64_t n_params);

/* Per-layer outputs of a fused launch (test support for layer-local parity of the timed kernels).
 * Runs the fused BF16/FP8 launch that gwd_forward issues at gated layer `layer` for windows of
 * length `window` (three consecutive layers of a stack, or four in a BF16 quad; see
 * gwd_set_tiling), on n_windows windows of caller-provided input x_in [n_windows][window][C] (device
 * fp32, rounded to bf16 as the residual stream of these paths is; each window zero-context), with
 * skip_inout [n_windows window][C] the skip sum before the launch (ignored when `layer` is 0) and
 * updated in place, and writes, for every layer j of the launch, its pre-activation
 * pre_out[j][row][2C] (fp32), its residual output x_out[j][row][C] (the bf16 values, as fp32; not
 * written for the network's last layer) and the running skip sum skip_out[j][row][C]
 * (row = window index * window + t). The arithmetic is that of the launch gwd_forward makes.
 * *layers_out receives the number of layers of the launch; with all buffers NULL the call only
 * reports it. GWD_ERR_ARG if no fused launch starts at `layer` for this window length, for bad
 * indices or misaligned (16-byte) buffers; GWD_ERR_UNSUPPORTED for FP32 or two-branch models. */
gwd_status gwd_debug_fused(gwd_model* model, int32_t member, int32_t layer, const float* x_in, int32_t n_windows,
                           int32_t window, float* skip_inout, float* pre_out, float* x_out, float* skip_out,
                           int32_t* layers_out, void* hip_stream);

/* One matrix-core instruction on one wave (test support: the accumulation rounding of the
 * instructions the reduced-precision kernels use). D = A B + C for A [32][K] and B [K][32]
 * (row-major device arrays of bf16 bit patterns for kind 0, K = 16, v_mfma_f32_32x32x16_bf16; of
 * E4M3 (OCP) bytes for kind 1, K = 64, v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales) and
 * C, D [32][32] fp32 row-major. GWD_ERR_ARG for another kind or NULL/misaligned pointers,
 * GWD_ERR_NO_DEVICE without a GPU. Asynchronous on hip_stream. */
gwd_status gwd_debug_mfma(int32_t kind, const void* a, const void* b, const float* c, float* d, void* hip_stream);

/* Backward operands of one gated layer (test support for layer-local parity of the hand-written
 * backward, "AI ensemble construction"). After this call, every gwd_backward on the model copies,
 * for gated layer `layer` (of the member it is called for), the operands and results of that layer's
 * backward step into the caller's device fp32 buffers, each [B W][C] with C = 128 unless noted:
 *   x_in   the layer input as the recompute produced it (bf16 values for BF16 models),
 *   pre    its pre-activation [B W][2C],
 *   dskip  dL/dskip (the same for every layer),
 *   dx_in  dL/d(layer output x'), zero for the last layer,
 *   dg     dL/dg = dskip W_s + dx_in W_r,
 *   g      the gate output as the weight-gradient GEMMs read it (bf16 values for BF16 models),
 *   dpre   dL/dpre [B W][2C] as the GEMMs read it (bf16 values for BF16 models),
 *   dx_out dL/dx = dx_in + dpre[t] W_tap1 + dpre[t + d] W_tap0.
 * The buffers must hold B W rows for the batch of the next gwd_backward and stay valid until it
 * completes. layer = -1 turns the copies off (the pointers may then be NULL). GWD_ERR_UNSUPPORTED
 * for other than kind-1 gated models; GWD_ERR_ARG for a layer out of range or NULL/misaligned
 * buffers. No device work; the copies add work to gwd_backward only while enabled. */
gwd_status gwd_debug_capture_backward(gwd_model* model, int32_t layer, float* x_in, float* pre, float* dskip,
                                      float* dx_in, float* dg, float* g, float* dpre, float* dx_out);

/* Measurement support: issues the launch that gwd_forward makes at middle gated
 * layer `layer` of member `member` (the single-layer kernel, or the fused
 * kernel when a fused launch starts there; every layer it covers must be a
 * middle one) reps + 1 times, with the forward's grid over its batch
 * of windows, on the activations the last gwd_forward left in the model's
 * workspace, and times the last `reps` launches between two HIP events
 * recorded on hip_stream. Writes the average milliseconds per launch, the
 * windows per launch and the layers per launch (1, 3, 4 or 6). Requires a prior
 * gwd_forward on the model; synchronises hip_stream. The workspace contents
 * are overwritten. */
gwd_status gwd_debug_time_layer(gwd_model* model, int32_t member, int32_t layer, int32_t reps,
                                float* ms_per_launch, int32_t* windows_per_launch, int32_t* layers_per_launch,
                                void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* GWD_H */
