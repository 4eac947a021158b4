// Internal declarations of the PVFinder HIP library: arena plan, engine state
// and kernel launchers.  Not part of the C ABI (see include/pvf.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pvf.h"

namespace pvf {

constexpr int kFeat = PVF_N_FEATURES;
constexpr int kHidden = 20;       // width of the per-track hidden layers
constexpr int kMaxHiddenLayers = 16;
constexpr int kTaps = 5;          // UNet conv kernel size
constexpr int kGuard = 2;         // zero rows before and after each event
constexpr int kMaxLevels = 6;
constexpr size_t kAlign = 256;
constexpr int kXcds = 8;          // MI355X: workgroups go round-robin over 8 XCDs

// Activation layout: channels-last, one block of R = L + 2*kGuard rows per
// event, rows [kGuard, kGuard + L) hold positions 0..L-1 and the guard rows
// stay zero for the life of the engine, so a 5-tap window never reaches into
// a neighbouring event and needs no branch.
struct Level {
    int L;      // positions
    int R;      // rows per event (L + 2*kGuard)
    int C;      // channels of this level
};

// Offsets (bytes from the arena base) of every buffer.  Activations a, cat,
// pool, d hold the compute dtype (4 or 2 bytes per element).
struct Plan {
    int n_levels = 0;
    int c0 = 0;
    int max_events = 0;
    int units = 1;                 // UNet sequences per event (1, or the interval count)
    Level lv[kMaxLevels];
    size_t weights = 0, weights_bytes = 0;
    size_t weights_lp = 0;         // 16-bit conv weights (BF16/FP16 engines)
    size_t mlp_lp = 0;             // track network packed for the matrix cores (BF16/FP16/FP8 engines)
    // E below is the number of UNet sequences (events x units)
    size_t x0 = 0;                 // [E][R0][1]      scaled histogram (always FP32)
    size_t a[kMaxLevels] = {};     // [E][Rl][Cl]     conv1 outputs (enc, then dec)
    size_t cat[kMaxLevels] = {};   // [E][Rl][2Cl]    skip | upsampled  (l < n-1)
    size_t pool[kMaxLevels] = {};  // [E][Rl][C(l-1)] pooled input of level l (l >= 1)
    size_t d[kMaxLevels] = {};     // [E][Rl][Cl]     decoder conv2 out (1 <= l <= n-2), deepest conv2 (l = n-1)
    size_t prob = 0;               // [events][n_bins] float
    size_t flags = 0;              // [E] int32 track-stage status
    size_t order = 0;              // [E] int32 event order of the track work queue
    size_t scales = 0;             // FP8: per-launch column and output scales
    size_t queue = 0;              // int32 ticket counter of the track work queue
    size_t zero_begin = 0, zero_end = 0;   // region cleared at init
    size_t total = 0;
};

// Packed weights, as element offsets (floats) from the weight region.
struct WeightLayout {
    size_t mlp = 0, mlp_count = 0;          // MLP tensors as in the blob
    size_t first_w = 0, first_b = 0;        // enc0.c1: [C0][5], [C0]
    struct Conv { size_t w = 0, b = 0; int cin = 0, cout = 0, taps = 0; };
    Conv enc[kMaxLevels][2];                // [l][0] conv1 (l > 0), [l][1] conv2
    Conv up[kMaxLevels];                    // up[l]: from level l+1 into level l
    Conv dec[kMaxLevels][2];
    size_t head_w = 0, head_b = 0;
    size_t total = 0;
};

// EPI_UP: a decoder conv whose output is consumed only by the transposed
// conv that follows it; the epilogue runs that transposed conv on its own
// output tile (which then never goes to HBM) and stores the upsampled rows.
enum Epi { EPI_STORE = 0, EPI_POOL = 1, EPI_CONVT = 2, EPI_HEAD = 3, EPI_UP = 4 };

// Row m0 + t of a channels-last batch with R rows per event -> (event, row
// within the event), for the rows of one output tile (t < 2^20).  The tile's
// first event is found once; the rest is a 32-bit divide by R done with a
// float estimate (off by at most one for quotients below 2^23) and one
// correction, instead of a 64-bit integer division per row.
struct RowMap {
    int64_t e0;
    int loc0, R;
    float inv;
    __device__ RowMap(int64_t m0, int rows_per_event)
        : e0(m0 / rows_per_event), loc0((int)(m0 - m0 / rows_per_event * rows_per_event)), R(rows_per_event),
          inv(1.f / (float)rows_per_event)
    {
    }
    __device__ __forceinline__ void at(int t, int64_t& e, int& loc) const
    {
        const int x = loc0 + t;
        int q = (int)((float)x * inv);
        int rem = x - q * R;
        if (rem >= R) { rem -= R; ++q; }
        else if (rem < 0) { rem += R; --q; }
        e = e0 + q;
        loc = rem;
    }
};

// One output channel of the first convolution (one input channel, five
// taps) at one row: bias, then the taps in order as fused multiply-adds, then
// the LeakyReLU.  The standalone first-convolution kernel and the conv kernels
// that fuse it into their staging share this, so both give the same bits.
__device__ __forceinline__ float first_conv_at(const float* w5, float b, const float* x5, float slope)
{
    float s = b;
#pragma unroll
    for (int j = 0; j < kTaps; ++j) s = fmaf(w5[j], x5[j], s);
    return s >= 0.f ? s : slope * s;
}

// OCP e4m3 code of x, saturated at +-448 (the hardware conversion would give
// NaN beyond).
__device__ __forceinline__ uint8_t e4m3_sat(float x)
{
    x = fminf(fmaxf(x, -448.f), 448.f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

struct ConvArgs {
    const void* in;      // input rows, channels-last (element type = compute dtype)
    int ld_in;           // floats per input row
    int cin;             // channels read (multiple of 16)
    int m_rows;          // total input rows (= events * R_in)
    int r_in;            // rows per event of the input level
    const void* w;       // packed [N][taps][cin] (element type = compute dtype)
    const float* bias;   // [Cout]
    int n;               // GEMM N (Cout, or 2*Cout for the transposed conv)
    float slope;         // LeakyReLU slope
    void* out;           // output base (row 0, channel 0 of the destination)
    int ld_out;          // floats per output row
    int r_out;           // rows per event of the output level
    int cout;            // output channels (transposed conv: n / 2)
    void* pool_out;      // EPI_POOL: pooled destination
    int ld_pool;
    int r_pool;
    const float* head_w; // EPI_HEAD: [C0] head weights
    float head_b;
    float* prob;         // EPI_HEAD: [E][L0]
    int l_out;           // positions per event of the output (EPI_HEAD)
    const float* col_scale;     // FP8: per GEMM column, dequantises the accumulator
    const float* out_inv_scale; // FP8: per output channel, 1 / scale of the stored tensor
    const float* fold_scale;    // FP8 stored outputs: per GEMM column, col_scale / output scale (16-byte aligned)
    const float* fold_bias;     // FP8 stored outputs: per GEMM column, bias / output scale (16-byte aligned)
    // First convolution fused into the staging of enc0.c2 (launch_conv_first
    // only): the input rows are then computed from the histogram rows instead
    // of read from `in`
    const float* first_x0;      // [m_rows] histogram rows, the input level's row layout
    const float* first_w;       // [cin][taps]
    const float* first_b;       // [cin]
    const float* first_inv_scale;   // FP8: [cin], 1 / scale of the first convolution's stored output
    // EPI_UP: the transposed conv applied to this launch's output tile
    const void* up_w;           // packed [2 up_cout][n] (compute dtype), as a transposed-conv launch reads it
    const float* up_b;          // [up_cout] (16-bit engines; FP8 folds it into up_fold_bias)
    void* up_out;               // its destination: row 0, channel 0 of the upsampled half
    int up_ld;                  // elements per destination row
    int up_r_out;               // destination rows per event
    int up_cout;                // transposed-conv output channels
    const float* up_fold_scale; // FP8: the transposed conv's folded column scales (16-byte aligned)
    const float* up_fold_bias;  // FP8: its folded bias (16-byte aligned)
};

struct TrackArgs {
    const int32_t* offsets;
    const float* feat[kFeat];
    int64_t n_tracks_total;
    int max_tracks;
    const float* mlp;        // MLP tensors in blob order
    int n_hidden;
    int n_out;               // bins per interval
    int n_intervals;
    double z_min;
    double interval_mm;
    float shift[kFeat];
    float scale[kFeat];
    float slope;
    float s_in;
    double boundary_mm;      // > 0: boundary tracks also feed the neighbouring interval
    float* x0;               // [E * units][R0]
    int r0;
    int unit_bins;           // bins per UNet sequence (n_bins, or bins per interval)
    int32_t* flags;          // [E]
    int32_t* order;          // [E] queue order (persistent form), or null
    int32_t* queue_counter;  // ticket counter (persistent form), or null
    // network arithmetic: FP32 on the vector ALUs, or BF16/FP16/FP8 on the
    // matrix cores with FP32 accumulation
    int mlp_dtype;
    const void* mlp_lp;      // packed weights: per layer [NP][32] (NP = 32, or 112 for the output layer)
    const float* mlp_in_inv; // FP8: per layer [32], 1 / scale of each input channel
    const float* mlp_col;    // FP8: per layer [NP], column scales
    float* mlp_calib;        // calibration only: |max| of every layer's input channels
};

// Low-precision network layout: every layer as a K = 32 GEMM (inputs zero-
// padded from 9 or 20), hidden layers 32 columns wide (20 used), the output
// layer 112 (100 used).
constexpr int kMlpK = 32;
constexpr int kMlpHiddenN = 32;
constexpr int kMlpOutN = 112;
inline int mlp_layer_cols(int layer, int n_hidden) { return layer < n_hidden ? kMlpHiddenN : kMlpOutN; }
inline size_t mlp_lp_elems(int n_hidden) { return ((size_t)n_hidden * kMlpHiddenN + kMlpOutN) * kMlpK; }
inline int mlp_calib_channels(int n_hidden) { return kFeat + n_hidden * kHidden; }

struct FirstConvArgs {
    const float* x0;         // [E][R0]
    int m_rows;
    int r0;
    const float* w;          // [C0][5]
    const float* b;          // [C0]
    int c0;
    float slope;
    void* out;               // [E][R0][C0], element type = compute dtype
    const float* out_inv_scale;   // FP8: per channel, 1 / scale of the stored tensor
};

struct PeakArgs {
    const float* prob;       // [E][L]
    int L;
    const int32_t* flags;    // [E] track-stage status
    double z_min, bw, p_min, s_min;
    int hw;
    int max_peaks;
    int32_t* n_vertices;
    double* z;
    float* peak_prob;
    double* integral;
    int32_t* status;
    int32_t* bin;            // may be null
};

struct GatherArgs {          // debug copy of an internal activation
    const void* src;
    int src_bytes;           // 4 = float, 2 = 16-bit compute dtype (see dtype)
    int dtype;
    int ld, r, guard, L, C, ch_off;
    float* dst;              // [E][C][L]
    int64_t count;
    const float* ch_scale;   // FP8 source: per channel dequantisation scale
};

// Per-channel absolute maximum of a channels-last activation (calibration):
// out[c] = max(out[c], max over rows |src[row][ch_off + c]|).
struct AmaxArgs {
    const void* src;
    int elem_bytes, dtype;
    int64_t rows;
    int ld, C, ch_off;
    float* out;
};
hipError_t launch_amax(const AmaxArgs& a, hipStream_t s);

// persistent_blocks > 0: the work-queue form (order kernel + persistent
// blocks, a.order and a.queue_counter set).  Otherwise one block per event.
hipError_t launch_track(const TrackArgs& a, int n_events, int persistent_blocks, hipStream_t s);
// Blocks of the track stage's work-queue form for this engine: as many as fit
// on the device at once.
int track_queue_blocks(int dtype, int n_intervals, int n_out, int cu_count);
// Name of the track-stage kernel an engine launches.
std::string track_kernel_name(int dtype, bool persistent, int n_intervals, int n_out);
hipError_t launch_first_conv(const FirstConvArgs& a, int dtype, hipStream_t s);
// Conv launches run one of several tile-shape variants of the kernel for
// the compute dtype; all variants of a dtype give identical bits.
hipError_t launch_conv(int dtype, const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s);
// enc0.c2 (5 taps, max-pool epilogue) with the first convolution computed in
// its staging (a.first_* set); conv_first_ok tells which variants do this
// (none in FP8: its 16-channel halo chunks need about 200 registers for the
// first convolution's weights, and the launch ran slower than the two it
// replaces).
hipError_t launch_conv_first(int dtype, const ConvArgs& a, int variant, hipStream_t s);
bool conv_first_ok(int dtype, int variant);
std::string conv_first_kernel_name(int dtype, int variant);
int conv_variant_count(int dtype);
bool conv_variant_ok(int dtype, int variant, int n, int cin, int taps, Epi epi);
int conv_default_variant(int dtype, int n, int cin, int taps, Epi epi);
// Default tile variant of a 5-tap launch that runs the transposed conv after
// it in its epilogue (EPI_UP), or -1 where no variant of the dtype can.
int conv_default_up_variant(int dtype, int n, int cin);
// Default variant of the head launch that also computes dec0.c1 (the 8-wave
// fused kernel for BF16/FP16), or -1 for dtypes without one.
int conv_default_dec0_variant(int dtype);
std::string conv_kernel_name(int dtype, int variant, int cin, int taps, Epi epi);

// per-precision implementations behind the functions above
hipError_t launch_conv_f32(const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s);
int f32_variant_count();
bool f32_variant_ok(int variant, int n, int taps, Epi epi);
int f32_default_variant(int n, int cin, int taps, Epi epi);
std::string f32_kernel_name(int variant, int taps, Epi epi);
hipError_t launch_conv_f32_first(const ConvArgs& a, int variant, hipStream_t s);
bool f32_first_ok(int variant);
std::string f32_first_kernel_name(int variant);
hipError_t launch_conv_lp(int dtype, const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s);
int lp_variant_count();
bool lp_variant_ok(int variant, int n, int cin, int taps, Epi epi);
int lp_default_variant(int n, int cin, int taps, Epi epi);
std::string lp_kernel_name(int dtype, int variant, int taps, Epi epi);
hipError_t launch_conv_lp_first(int dtype, const ConvArgs& a, int variant, hipStream_t s);
bool lp_first_ok(int variant);
int lp_default_up_variant(int n, int cin);
// Head-launch variants that also compute dec0.c1 (32-channel network): the
// 32-channel tensor between the two convs stays in LDS.  c1: dec0.c1's
// arguments, c2: dec0.c2 + head's.
bool lp_dec0_ok(int variant);
hipError_t launch_conv_lp_dec0(int dtype, const ConvArgs& c1, const ConvArgs& c2, int variant, hipStream_t s);
bool fp8_dec0_ok(int variant);
// enc0.c2 with the first convolution fused into its staging (FP8)
hipError_t launch_conv_fp8_first(const ConvArgs& a, int variant, hipStream_t s);
bool fp8_first_ok(int variant);
std::string fp8_first_kernel_name(int variant);
hipError_t launch_conv_fp8_dec0(const ConvArgs& c1, const ConvArgs& c2, int variant, hipStream_t s);
// dec0.c1 computed inside the head launch (16-bit and FP8 engines)
bool conv_dec0_ok(int dtype, int variant);
hipError_t launch_conv_dec0(int dtype, const ConvArgs& c1, const ConvArgs& c2, int variant, hipStream_t s);
int fp8_default_up_variant(int n, int cin);
std::string lp_first_kernel_name(int dtype, int variant);

hipError_t launch_conv_fp8(const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s);
int fp8_variant_count();
bool fp8_variant_ok(int variant, int n, int cin, int taps, Epi epi);
int fp8_default_variant(int n, int cin, int taps, Epi epi);
std::string fp8_kernel_name(int variant, int cin, int taps, Epi epi);

inline int act_bytes(int dtype) { return dtype == PVF_FP32 ? 4 : (dtype == PVF_FP8_E4M3 ? 1 : 2); }

hipError_t launch_peaks(const PeakArgs& a, int n_events, hipStream_t s);

// The library's fixed per-device scratch (pvf_execute_scratch).
constexpr size_t kScratchBytes = PVF_SCRATCH_BYTES;
constexpr int kMaxGuardRegions = 1 + 4 * kMaxLevels;
struct GuardRegion {
    char* base;          // first row of the region's first sequence
    int row_bytes;       // bytes per row (a multiple of 4)
    int rows_per_seq;    // R = L + 2 kGuard
};
struct GuardZeroArgs {
    GuardRegion r[kMaxGuardRegions];
    int n;               // regions
    int64_t n_seq;       // sequences per region
};
// Device address of the scratch on `device` (which must be current): looked
// up once per device and cached; nullptr if the lookup failed.
char* scratch_base(int device);
// Clear the kGuard rows at both ends of every sequence of every region.
hipError_t launch_zero_guard_rows(const GuardZeroArgs& a, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);

}  // namespace pvf
