// Internal declarations shared by the libgwd translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gwd.h"

namespace gwd {

// Residual / skip / head width of the full-size member; the FP32/BF16/FP8 layer kernels are
// specialised for it.
constexpr int kC = 128;
// Rows (time steps) of one layer-kernel tile.
constexpr int kBM = 64;
// Plain member (kind 0, four 16-channel layers and a 1x1 to one logit): per-output-channel weight
// scales follow its packed blob, 16 per conv layer then 1 for the output layer (1 unless FP8).
constexpr int kTinyScales = 4 * 16 + 1;
__host__ __device__ inline int tiny_scale_index(int layer, int out_channel) { return 16 * layer + out_channel; }

// One stream as the kernels see it; win_begin / sample_begin are prefix sums over streams.
struct StreamDesc {
    const float* ch0;
    const float* ch1;
    int64_t stride;
    int64_t length;
    int64_t win_begin;     // global index of this stream's first window
    int64_t sample_begin;  // offset of this stream's first sample in the stitched output
    int64_t n_win;
    int64_t _pad;
};

// Device binary search: stream that owns global window gw (streams with no windows are skipped).
__device__ inline int find_stream(const StreamDesc* s, int n, int64_t gw) {
    int lo = 0, hi = n;  // first index with win_begin > gw
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[mid].win_begin <= gw) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

// Blocks of a 1-D grid are dealt round-robin to the 8 XCDs of an MI355X. Renumber them so that
// consecutive work items (tiles of one window, which share dilation halos) run on one XCD and
// share its L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
    const int nx = 8;
    int per = nblocks / nx, rem = nblocks % nx;
    int x = bid % nx, i = bid / nx;
    // XCD x gets items [start(x), start(x) + per + (x < rem))
    int start = x * per + (x < rem ? x : rem);
    return start + i;
}

// Per-member packed weights (device), offsets in floats (or bytes for FP8) into one buffer.
struct LayerOffsets {
    int64_t wc, bc;    // conv weights (packed for the MFMA fragments), conv bias [2C]
    int64_t wrs, brs;  // res|skip weights (packed), res|skip bias [2C] (skip only in the last layer: [C])
    int64_t sc, srs;   // FP8 per-output-channel scales of conv [2C] and res|skip [2C] (floats)
};

struct MemberWeights {
    void* base = nullptr;   // device buffer
    int64_t bytes = 0;
    std::vector<LayerOffsets> layers;
    int64_t w_in = 0, b_in = 0, h1w = 0, h1b = 0, h2w = 0, h2b = 0;  // fp32 offsets (floats)
    // kind 0 (tiny member): plain fp32 copy of the blob
    int64_t blob = 0;
};

struct Workspace {
    void* base = nullptr;
    int64_t bytes = 0;
};

// Offsets (floats) of every tensor of a gated-member (kind 1) blob, in blob order.
struct BlobOffsets {
    int64_t in_w, in_b, h1w, h1b, h2w, h2b;
    std::vector<int64_t> dil_w, dil_b, res_w, res_b, skip_w, skip_b;
};
BlobOffsets blob_offsets(const gwd_arch& a);

}  // namespace gwd

struct gwd_model {
    gwd_arch arch;
    gwd_precision prec;
    int32_t n_members;
    int64_t n_params;
    int device;
    std::vector<float> host_blob;              // canonical fp32 weights as loaded (the source of the first packing)
    std::vector<gwd::MemberWeights> members;
    gwd::Workspace ws;
    gwd::Workspace tws;                        // training workspace
    std::vector<void*> canon;                  // device copy of each member's canonical blob (fp32; fp64 for GWD_FP64)
    int32_t batch_windows;                     // windows per layer-kernel batch
    int32_t last_nb = 0, last_T = 0;           // batch shape of the last gwd_forward (workspace contents)
    int64_t ws_tab_bytes = 0;                  // bytes reserved for the stream table at the workspace start
    std::vector<int64_t> host_firsts;          // host copy of FwdBatch::firsts for the current request
    int32_t lp_rows = 0;                       // BF16/FP8 layer tiling: rows per tile (0 = default per precision)
    int32_t lp_waves = 0;                      // and waves per block
    int32_t lp_fuse = 3;                       // BF16/FP8: layers per launch (3 = fused triples and quads, 6 = sextets and quads, 1 = one per launch)
    int32_t fused_blocks = 0;                  // blocks a fused launch aims at (segments per sub-sequence); 0 = 512
    bool two_branch = false;                   // loaded as kind 2 and expanded to the block-diagonal kind-1 image
    gwd_arch branch_arch{};                    // kind 2: the architecture as loaded
    int64_t branch_params = 0;                 // kind 2: parameters of one member in its own (branch) blob
    int64_t* branch_map = nullptr;             // kind 2: device [branch_params], trunk index of each branch parameter
    float* dense_grad = nullptr;               // kind 2: device [n_params], the trunk gradient before read-back
    void* repack_tab = nullptr;                // device per-layer offsets of the on-device weight refresh (gwd_adam_step)
    bool persistent = false;                   // BF16/FP8: the forward as one persistent launch (gwd_set_persistent)
    int32_t persist_grid = 0, persist_R = 1;   // its blocks and windows per block at a time, and its tables'
                                               // offset in the workspace (forward_prepare)
    int64_t persist_tab_off = 0;
    // test support (gwd_debug_capture_backward): gated layer whose backward operands and results the
    // next gwd_backward copies out as fp32 [M][C] ([M][2C] for pre and dpre); -1 = off
    int32_t cap_layer = -1;
    float* cap_buf[8] = {};                    // x_in, pre, dskip, dx_in, dg, g, dpre, dx_out
};

namespace gwd {
// The trunk blob (kind-1 order) of one kind-2 member: its block-diagonal image.
void expand_two_branch(const gwd_arch* a, const float* src, std::vector<float>& dst);
}

namespace gwd {

void set_error(const char* fmt, ...);
gwd_status hip_fail(hipError_t e, const char* what);

// Packing (pack.cpp): build the device image of one member from its canonical blob.
gwd_status pack_member(gwd_model* m, int member, const float* blob);
gwd_status export_member(const gwd_model* m, int member, float* out);

// Launchers (kernel translation units). All enqueue on `st`.
struct FwdBatch {
    const StreamDesc* streams;  // device
    int n_streams;
    int64_t win_base;   // global index of the batch's first window
    int nb;             // windows in the batch
    int T;              // window length
    int S;              // stride
    int out_mode;
    int member;
    int n_members;
    float* out;
    int64_t sum_L;      // total samples (stitched layout)
    int64_t total_win;  // total windows (mode 2 layout)
    const int64_t* firsts;  // device: global index of each stream's first window (streams with windows)
    int64_t first_idx;      // first entry of `firsts` inside this batch
    int n_first;            // entries of `firsts` inside this batch
    unsigned long long* done;  // persistent forward (optional): per stream, the wall clock at completion
};

hipError_t launch_tiny_forward(const gwd_model* m, const FwdBatch& fb, hipStream_t st);
hipError_t launch_wavenet_forward(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                                  hipStream_t st);
hipError_t launch_layer_debug(gwd_model* m, int member, int layer, const float* x_in, int nb, int T,
                              float* pre_out, float* x_out, float* skip, hipStream_t st);
// BF16/FP8 members: one layer on bf16 activations (training; skip may be null: no skip sum; pre16, if
// set, receives the pre-activations rounded to bf16 [nb T][256]), and an fp32 -> bf16 rounding copy.
hipError_t launch_layer_train_bf16io(gwd_model* m, int member, int l, const uint16_t* x_in, int nb, int T,
                                     uint16_t* pre16, uint16_t* x_out, float* skip, hipStream_t st);
hipError_t launch_f32_to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st);
hipError_t launch_bf16_to_f32(const uint16_t* x, int64_t n, float* y, hipStream_t st);
int train_layers_per_launch(const gwd_model* m, int l, int T);
// Test support: layers of the fused BF16/FP8 launch that starts at layer l (0 if none), and that
// launch with per-layer outputs.
int fused_layers_at(const gwd_model* m, int l, int T);
int default_layers_per_launch(const gwd_model* m);
hipError_t launch_mfma_probe(int kind, const void* A, const void* B, const float* C, float* D, hipStream_t st);
hipError_t launch_fused_debug(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* skip,
                              float* pre_out, float* x_out, float* skip_out, hipStream_t st);
hipError_t launch_fused_train(gwd_model* m, int member, int l, int nl, const uint16_t* x_in, uint16_t* x_out,
                              float* skip, int nb, int T, hipStream_t st);
hipError_t launch_fused_recompute(gwd_model* m, int member, int l, int nl, const uint16_t* x_in, uint16_t* x_out,
                                  uint16_t* pre, int64_t pre_stride, uint16_t* xs, int64_t xs_stride, int nb, int T,
                                  hipStream_t st);

// Layers covered by the launch that starts at layer l (3, 4 or 6 for a fused launch, else 1).
int layers_per_launch(const gwd_model* m, int l);
// One production launch of a middle layer on the workspace buffers (timing support).
hipError_t launch_layer_production(gwd_model* m, int member, int layer, void* x_in, void* x_out, float* skip, int nb,
                                   int T, hipStream_t st);

// Forward sequencing shared by gwd_forward and the captured plans (api.cpp).
gwd_status check_forward(const gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window,
                         int32_t stride, int32_t out_mode, std::vector<int64_t>& nwin, int64_t& sum_L,
                         int64_t& total_win, int64_t& out_floats);
gwd_status ensure_workspace(gwd_model* m, int64_t bytes, hipStream_t st);
gwd_status forward_prepare(gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window, int32_t stride,
                           int32_t out_mode, float* out, int64_t out_capacity_floats, hipStream_t st, bool sync_table,
                           FwdBatch& fb, int64_t& total_win, int& nb_max, std::vector<int64_t>* nwin_out);
hipError_t forward_enqueue(gwd_model* m, FwdBatch fb, int64_t total_win, int nb_max, hipStream_t st,
                           hipError_t (*after_batch)(void*, int64_t, hipStream_t), void* ctx);
hipError_t launch_stamp(unsigned long long* slot, hipStream_t st);

// Persistent forward (fwd_lowp.hip): whether a model runs it at window length T, the size of its
// launch tables and per-block buffers, the tables of a request (host bytes for the device address
// they are uploaded to), and the launch.
constexpr int kPersistWindows = 16;  // at most this many windows a persistent block holds at a time
bool persistent_supported(const gwd_model* m, int T);
int64_t persistent_table_bytes(const gwd_model* m, int T);
int64_t persistent_block_bytes(int T);
void persistent_tables(gwd_model* m, const FwdBatch& fb, std::vector<char>& host);
hipError_t launch_persistent(gwd_model* m, const FwdBatch& fb, const void* d_tables, void* act, int grid, int R,
                             unsigned long long* done, hipStream_t st);

// Triggers (triggers.hip)
struct TrigWork;
gwd_status run_triggers(const float* e, const int64_t* offs, int n_streams, double thr, int wc,
                        gwd_trigger* out, int64_t capacity, int64_t* n_found, hipStream_t st);
// The allocation-free form runs on a fixed 16 MiB device array per device.
constexpr int64_t kTrigScratchBytes = 16ll << 20;
int64_t trig_scratch_need(const int64_t* offs, int n_streams, int wc);   // bytes of scratch (0: nothing to scan)
gwd_status run_triggers_noalloc(const float* e, const int64_t* offs, int n_streams, double thr, int wc,
                                gwd_trigger* out, int64_t capacity, int64_t* n_found, hipStream_t st);

}  // namespace gwd
