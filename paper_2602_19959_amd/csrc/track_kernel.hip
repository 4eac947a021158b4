// FC stage: per-track network and histogram, one workgroup per event.
//
// Section 2 of arXiv:2602.19959: nine features per track go through six FC
// layers, and every track's outputs are combined into the event's histogram
// over 40 intervals of 100 bins; Section 3: a track feeds the interval that
// holds it, and an event is processed by one block reading SoA buffers.
//
// Boundary tracks (Section 3 variant): a track closer than boundary_mm to an
// edge its interval shares with another one also feeds that neighbour, its
// features taken in the neighbour's frame.  After a chunk's own items are
// accumulated, its boundary tracks are compacted into a staging list (track
// order) and go through the network and the accumulation once more.
//
// Two forms, both deterministic, atomic-free and dependent only on the
// event's own tracks; the block writes the scaled histogram once, straight
// into the UNet's input rows.
//
// track_stage_mma (every engine, histograms of at most 48 intervals and 112
// bins per interval): per chunk of 256 tracks (one per thread, coalesced SoA
// loads) each thread bins its track (exact comparison with the interval
// edges in double) and builds its features; each wave runs its 64 tracks
// through the hidden layers on the matrix cores (FP32, or BF16/FP16/FP8 with
// FP32 accumulation); each wave then computes two of the seven 16-column
// tiles of the output layer for every track of the chunk and adds them to
// the histogram, which it holds in registers, as a one-hot GEMM on the
// matrix cores (the output fragment is the GEMM's B operand as it stands).
//
// track_stage / track_stage_queue (longer histograms): the hidden layers in
// registers (FP32 on the vector ALUs, weights through the scalar cache), or
// on the matrix cores; per sub-chunk of 64 tracks the outputs go to LDS, the
// sub-chunk's tracks are grouped by interval (wave ballots, track order kept
// inside a group), and each (group, output column) pair is summed in track
// order in a register by one thread and added to its LDS bin, so every bin
// is a fixed sequence of sums in ascending track order.
#include <cfloat>
#include <cmath>

#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int NT = 256;   // tracks per chunk, one per thread
constexpr int SUB = 64;   // tracks per output/scatter sub-chunk (one per lane)
constexpr int HP = kHidden + 1;   // LDS pitch of the hidden activations (one row per thread)
// LDS pitch of the FP32 layer rows of the matrix-core form: with 64 banks,
// 20 makes both of its access patterns conflict-free (fragment reads: 16
// rows x 4 consecutive k; writes: 4 row groups x 16 consecutive channels)
constexpr int HPM = kHidden;

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

// softplus(x) = max(x, 0) + log1p(exp(-|x|)), in about 20 instructions:
//   * t = exp(-|x|) = 2^(-|x| log2 e) on the hardware exp2, with the product
//     split into hi + lo (the FMA gives the rounding error of hi exactly) and
//     2^lo applied to first order; below 2^-120 the library exp2f keeps the
//     subnormal result;
//   * log1p(t) = 2 atanh(s), s = t / (2 + t) in (0, 1/3], from the atanh
//     series s + s^3/3 + ... + s^17/17 (truncation below 2e-9 relative).
// Relative error about 1e-6 (4e-6 at |x| = 80), against FP32 network
// errors of the same order and the histogram's 1e-4 bound.
__device__ __forceinline__ float softplus(float x)
{
    constexpr float kLog2e = 1.44269504f, kLog2eLo = 1.92596303e-8f, kLn2 = 0.693147181f;
    const float a = -fabsf(x);
    const float hi = a * kLog2e;
    const float lo = fmaf(a, kLog2eLo, fmaf(a, kLog2e, -hi));
    const float t0 = hi < -120.f ? exp2f(hi) : __builtin_amdgcn_exp2f(hi);
    const float t = fmaf(t0, lo * kLn2, t0);
    const float s = t * __builtin_amdgcn_rcpf(2.f + t);
    const float z = s * s;
    float p = 1.f / 17.f;
    p = fmaf(p, z, 1.f / 15.f);
    p = fmaf(p, z, 1.f / 13.f);
    p = fmaf(p, z, 1.f / 11.f);
    p = fmaf(p, z, 1.f / 9.f);
    p = fmaf(p, z, 1.f / 7.f);
    p = fmaf(p, z, 1.f / 5.f);
    p = fmaf(p, z, 1.f / 3.f);
    p = fmaf(p, z, 1.f);
    return fmaxf(x, 0.f) + 2.f * s * p;
}

// Softplus of the matrix-core engines, whose outputs come from a network
// with 16-bit or 8-bit inputs: the same method with the exponent argument
// rounded once (relative error of t below 6e-6 for |x| < 88; t flushes to
// zero where the hardware exp2 does, near x = -87) and the atanh series to
// s^11 / 11 (truncation below 2e-7 relative), about half the instructions.
__device__ __forceinline__ float softplus_lp(float x)
{
    const float t = __builtin_amdgcn_exp2f(-fabsf(x) * 1.44269504f);
    const float s = t * __builtin_amdgcn_rcpf(2.f + t);
    const float z = s * s;
    float p = 1.f / 11.f;
    p = fmaf(p, z, 1.f / 9.f);
    p = fmaf(p, z, 1.f / 7.f);
    p = fmaf(p, z, 1.f / 5.f);
    p = fmaf(p, z, 1.f / 3.f);
    p = fmaf(p, z, 1.f);
    return fmaxf(x, 0.f) + 2.f * s * p;
}

// Exact (uncontracted) lower edge of interval i, as the binning takes it.
__device__ __forceinline__ double edge(const TrackArgs& a, int i)
{
    return __dadd_rn(a.z_min, __dmul_rn(a.interval_mm, (double)i));
}

// Network inputs of one track in the frame of interval itv: the z offset
// mapped to [-1, 1) inside that interval, the other features standardised.
__device__ __forceinline__ void features(const TrackArgs& a, const float* f, double zd, int itv, float* g)
{
    g[0] = (float)((zd - edge(a, itv)) / (a.interval_mm * 0.5) - 1.0);
#pragma unroll
    for (int k = 1; k < kFeat; ++k) g[k] = (f[k] - a.shift[k]) * a.scale[k];
}

// Item t of an event (t < end): its interval (-1 when it is dropped: outside
// the window or not finite), its network inputs g in that interval's frame,
// and the neighbouring interval it also feeds (-1 if none); the binning
// compares with the exact interval edges in double.  A dropped item sets
// *dropped (a benign race: every writer stores 1).
__device__ __forceinline__ void bin_track(const TrackArgs& a, int64_t t, double z_max, bool two, int& itv, int& nb,
                                          float* g, int* dropped)
{
    float f[kFeat];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) {
        f[k] = a.feat[k][t];
        finite = finite && isfinite(f[k]);
    }
    const double zd = (double)f[0];
    if (finite && zd >= a.z_min && zd < z_max) {
        int i = (int)floor((zd - a.z_min) / a.interval_mm);
        i = i < 0 ? 0 : (i >= a.n_intervals ? a.n_intervals - 1 : i);
        if (zd < edge(a, i)) --i;
        else if (zd >= edge(a, i + 1)) ++i;
        if (i >= 0 && i < a.n_intervals) itv = i;
    }
    if (itv < 0) {
        *dropped = 1;
    } else {
        features(a, f, zd, itv, g);
        // boundary item: closer than boundary_mm to an edge shared with
        // another interval (distances in double, exact edges)
        if (two) {
            if (zd - edge(a, itv) < a.boundary_mm && itv > 0) nb = itv - 1;
            else if (edge(a, itv + 1) - zd < a.boundary_mm && itv < a.n_intervals - 1) nb = itv + 1;
        }
    }
}

// Calibration: the largest |v| over the wave, per channel, merged into the
// table (float bits compare like unsigned integers for v >= 0).
__device__ __forceinline__ void wave_amax(float* dst, float v)
{
    v = fabsf(v);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int*>(dst), __float_as_uint(v));
}

// Calibration table offset of the inputs of network layer l.
__device__ __forceinline__ int calib_off(int l) { return l == 0 ? 0 : kFeat + (l - 1) * kHidden; }

// FP32 hidden layers on the vector ALUs, for every lane (lanes without a
// track carry zeros and their results are never used), so that the
// calibration reductions see a whole wave.
__device__ __forceinline__ void hidden_layers_f32(const TrackArgs& a, const float* g, bool valid, float* h)
{
    const float* W1 = a.mlp;                               // [kHidden][kFeat]
    const float* b1 = W1 + kHidden * kFeat;
    const float* Wh = b1 + kHidden;                        // hidden layers 2.. : [W 20x20, b 20]
    if (a.mlp_calib)
#pragma unroll
        for (int k = 0; k < kFeat; ++k) wave_amax(a.mlp_calib + calib_off(0) + k, valid ? g[k] : 0.f);
#pragma unroll
    for (int j = 0; j < kHidden; ++j) {
        float s = b1[j];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) s = fmaf(W1[j * kFeat + k], g[k], s);
        h[j] = lrelu(s, a.slope);
    }
    for (int l = 1; l < a.n_hidden; ++l) {
        if (a.mlp_calib)
            for (int j = 0; j < kHidden; ++j) wave_amax(a.mlp_calib + calib_off(l) + j, valid ? h[j] : 0.f);
        const float* W = Wh + (size_t)(l - 1) * (kHidden * kHidden + kHidden);
        const float* bb = W + kHidden * kHidden;
        float hn[kHidden];
#pragma unroll
        for (int j = 0; j < kHidden; ++j) {
            float s = bb[j];
#pragma unroll
            for (int k = 0; k < kHidden; ++k) s = fmaf(W[j * kHidden + k], h[k], s);
            hn[j] = lrelu(s, a.slope);
        }
#pragma unroll
        for (int j = 0; j < kHidden; ++j) h[j] = hn[j];
    }
    if (a.mlp_calib)
        for (int j = 0; j < kHidden; ++j) wave_amax(a.mlp_calib + calib_off(a.n_hidden) + j, valid ? h[j] : 0.f);
}

// ---------------------------------------------------------------- matrix-core network
//
// BF16/FP16/FP8 engines run the network as GEMMs on the matrix cores: each
// wave takes its 64 items (4 tiles of 16 rows); every layer is a K = 32 GEMM
// (inputs zero-padded), the hidden layers 2 column tiles wide and the output
// layer 7, accumulated in FP32; bias, LeakyReLU / softplus in FP32; the
// hidden activations go back to LDS in the compute type for the next layer.
// FP8 (OCP e4m3) uses per-channel scales as the convolutions do: each layer
// input holds v / a_c, the weights carry a_c and a column scale s_n.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint8_t to_e4m3(float x)
{
    x = fminf(fmaxf(x, -448.f), 448.f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

template <class E> struct Net;
template <> struct Net<__bf16> {
    using V = bf16x8;
    static constexpr int KP = 40;              // LDS row pitch (elements)
    __device__ static f32x4 mfma(V x, V w, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, w, c, 0, 0, 0); }
    __device__ static __bf16 cvt(float v, float) { return (__bf16)v; }
};
template <> struct Net<_Float16> {
    using V = f16x8;
    static constexpr int KP = 40;
    __device__ static f32x4 mfma(V x, V w, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, w, c, 0, 0, 0); }
    __device__ static _Float16 cvt(float v, float) { return (_Float16)v; }
};
template <> struct Net<uint8_t> {
    using V = long;
    static constexpr int KP = 48;
    __device__ static f32x4 mfma(V x, V w, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x, w, c, 0, 0, 0); }
    __device__ static uint8_t cvt(float v, float inv) { return to_e4m3(v * inv); }
};

// Layer l's bias (FP32, from the blob layout) and packed weights.
__device__ __forceinline__ const float* layer_bias(const TrackArgs& a, int l)
{
    const float* b1 = a.mlp + kHidden * kFeat;
    if (l == 0) return b1;
    const float* Wh = b1 + kHidden;
    if (l < a.n_hidden) return Wh + (size_t)(l - 1) * (kHidden * kHidden + kHidden) + kHidden * kHidden;
    const float* Wo = Wh + (size_t)(a.n_hidden - 1) * (kHidden * kHidden + kHidden);
    return Wo + (size_t)a.n_out * kHidden;
}

// Row i of the wave's input tile: the features of item i, quantised.
template <class E>
__device__ __forceinline__ void store_inputs(const TrackArgs& a, E* xa, int row, const float* g)
{
    E* r = xa + row * Net<E>::KP;
#pragma unroll
    for (int k = 0; k < kMlpK; ++k) {
        const float inv = (sizeof(E) == 1 && k < kFeat) ? a.mlp_in_inv[k] : 1.f;
        r[k] = Net<E>::cvt(k < kFeat ? g[k] : 0.f, inv);
    }
}

// Hidden layers of the wave's 64 rows, in place in xa.
template <class E>
__device__ void hidden_layers_mma(const TrackArgs& a, E* xa, const int* iv, int wave, int lane)
{
    using V = typename Net<E>::V;
    constexpr int KP = Net<E>::KP;
    const int li = lane & 15, lg = lane >> 4;
    const E* wp = static_cast<const E*>(a.mlp_lp);
    E* rows = xa + (size_t)wave * 64 * KP;
    const int* kept = iv + wave * 64 + 4 * lg;   // kept[16 i + v] >= 0: row 16 i + 4 lg + v is a kept item
    for (int l = 0; l < a.n_hidden; ++l) {
        const E* W = wp + (size_t)l * kMlpHiddenN * kMlpK;
        const float* b = layer_bias(a, l);
        V x[4], w[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = *reinterpret_cast<const V*>(rows + (16 * i + li) * KP + 8 * lg);
#pragma unroll
        for (int j = 0; j < 2; ++j) w[j] = *reinterpret_cast<const V*>(W + (16 * j + li) * kMlpK + 8 * lg);
        f32x4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Net<E>::mfma(x[i], w[j], f32x4{0.f, 0.f, 0.f, 0.f});
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = 16 * j + li;                        // output channel of this lane
            const bool used = n < kHidden;
            const float cs = (sizeof(E) == 1 && used) ? a.mlp_col[l * kMlpHiddenN + n] : 1.f;
            const float bn = used ? b[n] : 0.f;
            const float inv = (sizeof(E) == 1 && used) ? a.mlp_in_inv[(l + 1) * kMlpK + n] : 1.f;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float y = used ? lrelu(acc[i][j][v] * cs + bn, a.slope) : 0.f;
                    rows[(16 * i + 4 * lg + v) * KP + n] = Net<E>::cvt(y, inv);
                }
            if (a.mlp_calib) {
                // the largest |output| over the wave's kept items
                float m = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (kept[16 * i + v] >= 0) m = fmaxf(m, fabsf(used ? lrelu(acc[i][j][v] * cs + bn, a.slope) : 0.f));
                m = fmaxf(m, __shfl_xor(m, 16));
                m = fmaxf(m, __shfl_xor(m, 32));
                if (lg == 0 && used)
                    atomicMax(reinterpret_cast<unsigned int*>(a.mlp_calib + calib_off(l + 1) + n), __float_as_uint(m));
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Output layer of the 64 rows that wave `owner` computed: every wave takes
// every fourth 16-column tile; softplus outputs into ob [64][n_out + 1].
template <class E>
__device__ void outputs_mma(const TrackArgs& a, const E* xa, int owner, int wave, int lane, float* ob)
{
    using V = typename Net<E>::V;
    constexpr int KP = Net<E>::KP;
    const int li = lane & 15, lg = lane >> 4;
    const int op = a.n_out + 1;
    const E* W = static_cast<const E*>(a.mlp_lp) + (size_t)a.n_hidden * kMlpHiddenN * kMlpK;
    const float* b = layer_bias(a, a.n_hidden);
    const E* rows = xa + (size_t)owner * 64 * KP;
    V x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = *reinterpret_cast<const V*>(rows + (16 * i + li) * KP + 8 * lg);
    for (int jt = wave; jt < kMlpOutN / 16; jt += NT / 64) {
        const int n = 16 * jt + li;
        const V w = *reinterpret_cast<const V*>(W + (size_t)n * kMlpK + 8 * lg);
        const bool used = n < a.n_out;
        const float cs = (sizeof(E) == 1 && used) ? a.mlp_col[a.n_hidden * kMlpHiddenN + n] : 1.f;
        const float bn = used ? b[n] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const f32x4 acc = Net<E>::mfma(x[i], w, f32x4{0.f, 0.f, 0.f, 0.f});
            if (used)
#pragma unroll
                for (int v = 0; v < 4; ++v) ob[(16 * i + 4 * lg + v) * op + n] = softplus(acc[v] * cs + bn);
        }
    }
}

// ---------------------------------------------------------------- one event

// E = float: the FP32 network on the vector ALUs; otherwise the matrix-core
// network in E.  Everything else (binning, staging, ordered accumulation) is
// shared.
template <class E>
__device__ void track_event(const TrackArgs& a, int e, float* smem)
{
    constexpr bool kF32 = sizeof(E) == 4;
    const int n_bins = a.n_out * a.n_intervals;
    float* H = smem;                                  // [n_bins]
    float* hb = H + n_bins;                           // FP32: [NT][HP] hidden activations
    E* xa = reinterpret_cast<E*>(hb);                 // matrix cores: [NT][KP] layer inputs
    float* ob = hb + NT * HP;                         // [SUB][n_out + 1]
    int* iv = reinterpret_cast<int*>(ob + SUB * (a.n_out + 1));   // [NT] interval of each item
    int* nbv = iv + NT;                               // [NT] neighbour interval of each track, or -1
    // a sub-chunk's items grouped by interval: lst [SUB] rows of ob (offsets),
    // group g = lst[gbeg[g] .. gbeg[g+1]) of interval giv[g]
    int* lst = nbv + NT;
    int* giv = lst + SUB;
    int* gbeg = giv + SUB;                            // [SUB + 1]
    __shared__ int n_groups;
    // staging list of the chunk's boundary tracks; it shares ob's space: it is
    // written after the own items' last use of ob and read before ob's next
    int* st = reinterpret_cast<int*>(ob);
    __shared__ int dropped_any;
    __shared__ int wave_count[NT / 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int op = a.n_out + 1;

    for (int b = tid; b < n_bins; b += NT) H[b] = 0.f;
    if (tid == 0) dropped_any = 0;

    const int64_t beg = a.offsets[e];
    const int64_t end = a.offsets[e + 1];
    int status = 0;
    if (beg < 0 || end < beg || end > a.n_tracks_total) status = PVF_EV_BAD_INPUT;
    else if (end - beg > a.max_tracks) status = PVF_EV_TOO_MANY_TRACKS;
    __syncthreads();

    const float* Wo = a.mlp + kHidden * kFeat + kHidden +
                      (size_t)(a.n_hidden - 1) * (kHidden * kHidden + kHidden);   // [n_out][kHidden]
    const float* bo = Wo + (size_t)a.n_out * kHidden;
    const double z_max = edge(a, a.n_intervals);
    const bool two = a.boundary_mm > 0.0;

    // A for one item per thread: the hidden layers (FP32 in registers, then
    // to hb; or the matrix-core layers in xa)
    auto network_hidden = [&](const float* g, bool valid) {
        // a wave without a single kept item skips the network (its rows are
        // never accumulated, and it adds nothing to a calibration maximum)
        const bool any = __ballot(valid) != 0;
        if constexpr (kF32) {
            float h[kHidden];
            if (any) hidden_layers_f32(a, g, valid, h);
#pragma unroll
            for (int j = 0; j < kHidden; ++j) hb[tid * HP + j] = (any && valid) ? h[j] : 0.f;
        } else {
            float z[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) z[k] = valid ? g[k] : 0.f;
            if (a.mlp_calib)
#pragma unroll
                for (int k = 0; k < kFeat; ++k) wave_amax(a.mlp_calib + calib_off(0) + k, z[k]);
            store_inputs<E>(a, xa, tid, z);
            __builtin_amdgcn_wave_barrier();
            if (any) hidden_layers_mma<E>(a, xa, iv, wave, lane);
        }
    };

    // B + C over the first n items: outputs, then the ordered accumulation
    // (thread j owns column j, items in list order)
    auto outputs_and_accumulate = [&](int n) {
        for (int sub = 0; sub < n; sub += SUB) {
            // ---- B: the sub-chunk's outputs into ob
            if constexpr (kF32) {
                // wave q computes outputs q, q+4, ... for the 64 items
                const int tt = sub + lane;
                if (tt < n && iv[tt] >= 0) {
                    float hl[kHidden];
#pragma unroll
                    for (int k = 0; k < kHidden; ++k) hl[k] = hb[tt * HP + k];
                    for (int j = wave; j < a.n_out; j += NT / 64) {
                        float s = bo[j];
#pragma unroll
                        for (int k = 0; k < kHidden; ++k) s = fmaf(Wo[j * kHidden + k], hl[k], s);
                        ob[lane * op + j] = softplus(s);
                    }
                }
            } else {
                // all waves share the output layer of these 64 rows
                outputs_mma<E>(a, xa, sub / SUB, wave, lane, ob);
            }
            __syncthreads();
            // ---- C: accumulation.  Wave 0 groups the sub-chunk's kept items by
            // interval (one ballot round per distinct interval, earliest item
            // first; track order inside a group); then every thread takes
            // (group, column) pairs, sums the group's outputs in track order in
            // a register and adds that to the bin once.
            const int lim = (n - sub) < SUB ? (n - sub) : SUB;
            if (wave == 0) {
                const int itv = lane < lim ? iv[sub + lane] : -1;
                bool pending = itv >= 0;
                uint64_t rem = __ballot(pending);
                int ng = 0, pos = 0;
                while (rem) {
                    const int v = __shfl(itv, __ffsll((unsigned long long)rem) - 1);
                    const bool mine = pending && itv == v;
                    const uint64_t m = __ballot(mine);
                    if (mine) {
                        lst[pos + __popcll(m & ((1ull << lane) - 1ull))] = lane * op;   // row offset in ob
                        pending = false;
                    }
                    if (lane == 0) {
                        giv[ng] = v;
                        gbeg[ng] = pos;
                    }
                    pos += __popcll(m);
                    ++ng;
                    rem &= ~m;
                }
                if (lane == 0) {
                    gbeg[ng] = pos;
                    n_groups = ng;
                }
            }
            __syncthreads();
            const int ng = n_groups;
            for (int q = tid; q < ng * a.n_out; q += NT) {
                const int g = q / a.n_out, j = q - g * a.n_out;
                const int ue = gbeg[g + 1];
                int u = gbeg[g];
                float sum = 0.f;
                // four items at a time: their LDS reads overlap, the sums stay in order
                for (; u + 4 <= ue; u += 4) {
                    const int r0 = lst[u], r1 = lst[u + 1], r2 = lst[u + 2], r3 = lst[u + 3];
                    const float o0 = ob[r0 + j], o1 = ob[r1 + j], o2 = ob[r2 + j], o3 = ob[r3 + j];
                    sum += o0;
                    sum += o1;
                    sum += o2;
                    sum += o3;
                }
                for (; u < ue; ++u) sum += ob[lst[u] + j];
                H[giv[g] * a.n_out + j] += sum;
            }
            __syncthreads();
        }
    };

    if (status == 0) {
        for (int64_t base = beg; base < end; base += NT) {
            // ---- A: bin, features, hidden layers (own interval)
            const int64_t t = base + tid;
            int itv = -1, nb = -1;
            float g[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) g[k] = 0.f;
            if (t < end) bin_track(a, t, z_max, two, itv, nb, g, &dropped_any);
            iv[tid] = itv;   // read by the hidden layers' calibration
            network_hidden(g, itv >= 0);
            nbv[tid] = nb;
            __syncthreads();

            const int n_chunk = (int)((end - base) < NT ? (end - base) : NT);
            outputs_and_accumulate(n_chunk);

            if (two) {
                // ---- staging: the chunk's boundary tracks, in track order
                const bool is_b = nbv[tid] >= 0;
                const uint64_t m = __ballot(is_b);
                if (lane == 0) wave_count[wave] = __popcll(m);
                __syncthreads();
                int off = 0, n_st = 0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) {
                    off += w < wave ? wave_count[w] : 0;
                    n_st += wave_count[w];
                }
                if (is_b) st[off + __popcll(m & ((1ull << lane) - 1ull))] = tid;
                __syncthreads();
                if (n_st > 0) {
                    // ---- A again for the staged items, in the neighbour's frame
                    int inb = -1;
                    float gs[kFeat];
#pragma unroll
                    for (int k = 0; k < kFeat; ++k) gs[k] = 0.f;
                    if (tid < n_st) {
                        const int src = st[tid];
                        inb = nbv[src];
                        float fs[kFeat];
#pragma unroll
                        for (int k = 0; k < kFeat; ++k) fs[k] = a.feat[k][base + src];
                        features(a, fs, (double)fs[0], inb, gs);
                    }
                    __syncthreads();    // every read of nbv / st above is done
                    iv[tid] = inb;
                    network_hidden(gs, tid < n_st);
                    __syncthreads();
                    outputs_and_accumulate(n_st);
                }
            }
        }
    }
    __syncthreads();
    // scaled histogram into the UNet's input rows: one sequence per event, or
    // one per interval (unit_bins bins each), two guard rows on each side
    const int U = n_bins / a.unit_bins;
    float* x0 = a.x0 + (int64_t)e * U * a.r0 + kGuard;
    for (int b = tid; b < n_bins; b += NT) {
        const int u = b / a.unit_bins;
        x0[(int64_t)u * a.r0 + (b - u * a.unit_bins)] = a.s_in * H[b];
    }
    if (tid == 0) a.flags[e] = status | (dropped_any ? PVF_EV_TRACKS_DROPPED : 0);
    __syncthreads();   // the block's LDS is reused by its next event
}

// One block per event.
template <class E>
__global__ __launch_bounds__(NT) void track_stage(TrackArgs a)
{
    extern __shared__ float smem[];
    track_event<E>(a, blockIdx.x, smem);
}

// Persistent form for uneven track counts: a fixed grid of blocks takes
// tickets from a device counter; ticket k is the k-th event in descending
// track count (largest first, so the long events do not end the launch
// alone).  Every event's result is the same whichever block computes it.
template <class E>
__global__ __launch_bounds__(NT) void track_stage_queue(TrackArgs a, int n_events)
{
    extern __shared__ float smem[];
    __shared__ int ticket;
    for (;;) {
        if (threadIdx.x == 0) ticket = atomicAdd(a.queue_counter, 1);
        __syncthreads();
        const int k = ticket;
        __syncthreads();
        if (k >= n_events) break;
        track_event<E>(a, a.order[k], smem);
    }
}

// ---------------------------------------------------------------- histogram on the matrix cores
//
// Every engine keeps an event's histogram in registers when it has at most
// kRegIntervals intervals, and accumulates it on the matrix cores: per
// sub-chunk of 64 items, H[i][j] += sum_t S[i][t] Y[t][j], with S the one-hot
// item-to-interval matrix (a dropped item has a zero column) and Y the items'
// softplus outputs.  Each wave owns two of the seven output column tiles (16
// columns each) over every interval tile, and computes those outputs for all
// of the chunk's sub-chunks itself; the output layer's MFMA fragment already
// is the B operand of the accumulation: in K step s, element u of lane group
// lg is item 16 (2 s + u / 4) + 4 lg + u % 4, the row that lane holds.  Y
// enters as two BF16 terms in the 16-bit and 8-bit engines, y = t0 + t1 + r
// with t0 = bf16(y) and t1 = bf16(y - t0), so |r| <= 2^-16 |y| (below the
// network's own rounding), and as itself in the FP32 engine (FP32 MFMA); the
// products with the one-hot operand are exact, and the sums are FP32 in the
// matrix core's fixed order: deterministic, no atomics, depending only on
// the event's own items.  Outputs are capped at the largest finite value of
// the operand type, so a non-finite output cannot reach other intervals
// through 0 x inf.  The event's histogram leaves the registers once, scaled,
// into the UNet's input rows.
constexpr int kRegMT = 3;                   // interval tiles of 16
constexpr int kRegIntervals = 16 * kRegMT;
constexpr float kBf16Max = 0x1.fcp127f;     // largest finite BF16

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One-hot A operand of interval m for K step s: element u is 1 when the
// lane's item (2 s + u / 4, u % 4) lies in interval m.
__device__ __forceinline__ bf16x8 onehot(const int (&itv)[4][4], int s, int m)
{
    u32x4 r;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int u0 = 2 * p, u1 = 2 * p + 1;
        const bool e0 = itv[2 * s + u0 / 4][u0 % 4] == m;
        const bool e1 = itv[2 * s + u1 / 4][u1 % 4] == m;
        r[p] = (e0 ? 0x3F80u : 0u) | (e1 ? 0x3F800000u : 0u);
    }
    return __builtin_bit_cast(bf16x8, r);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 x, bf16x8 w, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, w, c, 0, 0, 0);
}

// Column tiles of wave `wave` in block `blk`: q and q + 4, q = (wave + blk) % 4
// (the tile count is odd, so the rotation spreads the lighter wave over the
// SIMDs of a CU).
__device__ __forceinline__ int hist_tile(int wave, int blk, int jl) { return ((wave + blk) & 3) + 4 * jl; }

// Outputs of items [0, n) of the chunk for the wave's column tiles, added to
// the wave's histogram tiles h[column tile][interval tile].
template <class E>
__device__ void outputs_to_hist(const TrackArgs& a, const E* xa, const int* iv, int n, int wave, int lane,
                                f32x4 (&h)[2][kRegMT])
{
    using V = typename Net<E>::V;
    constexpr int KP = Net<E>::KP;
    const int li = lane & 15, lg = lane >> 4;
    const E* W = static_cast<const E*>(a.mlp_lp) + (size_t)a.n_hidden * kMlpHiddenN * kMlpK;
    const float* b = layer_bias(a, a.n_hidden);
    bool on[2];
    V w[2];
    float cs[2], bn[2];
#pragma unroll
    for (int jl = 0; jl < 2; ++jl) {
        const int jt = hist_tile(wave, blockIdx.x, jl);
        on[jl] = jt < kMlpOutN / 16 && 16 * jt < a.n_out;
        const int c = on[jl] ? 16 * jt + li : li;
        w[jl] = *reinterpret_cast<const V*>(W + (size_t)c * kMlpK + 8 * lg);
        const bool used = on[jl] && c < a.n_out;
        cs[jl] = (sizeof(E) == 1 && used) ? a.mlp_col[a.n_hidden * kMlpHiddenN + c] : 1.f;
        bn[jl] = used ? b[c] : 0.f;
    }
#pragma unroll 1
    for (int sub = 0; sub < n; sub += SUB) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            // the lane's items 16 i + 4 lg + v, i = 2 s, 2 s + 1: intervals,
            // layer inputs, and the one-hot operand of each interval tile
            int itv[4][4];
            V x[2];
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int i = 2 * s + ii;
                x[ii] = *reinterpret_cast<const V*>(xa + (size_t)(sub + 16 * i + li) * KP + 8 * lg);
                const int4 q = *reinterpret_cast<const int4*>(iv + sub + 16 * i + 4 * lg);
                itv[i][0] = q.x;
                itv[i][1] = q.y;
                itv[i][2] = q.z;
                itv[i][3] = q.w;
            }
            bf16x8 oh[kRegMT];
#pragma unroll
            for (int mt = 0; mt < kRegMT; ++mt) oh[mt] = onehot(itv, s, 16 * mt + li);
#pragma unroll
            for (int jl = 0; jl < 2; ++jl) {
                if (!on[jl]) continue;
                // y = t0 + t1 + r with t0 = bf16(y), t1 = bf16(y - t0), |r| <= 2^-16 |y|
                bf16x8 t0, t1;
#pragma unroll
                for (int ii = 0; ii < 2; ++ii) {
                    const f32x4 acc = Net<E>::mfma(x[ii], w[jl], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float y = fminf(softplus_lp(acc[v] * cs[jl] + bn[jl]), kBf16Max);
                        const __bf16 y0 = (__bf16)y;
                        t0[4 * ii + v] = y0;
                        t1[4 * ii + v] = (__bf16)(y - (float)y0);
                    }
                }
#pragma unroll
                for (int mt = 0; mt < kRegMT; ++mt) {
                    if (16 * mt >= a.n_intervals) break;
                    h[jl][mt] = mfma_bf16(oh[mt], t0, h[jl][mt]);
                    h[jl][mt] = mfma_bf16(oh[mt], t1, h[jl][mt]);
                }
            }
        }
    }
}

// FP32 hidden layers on the matrix cores (v_mfma_f32_16x16x4_f32) for the
// wave's 64 rows of hb, in place: K step s of row tile i gives lane (lg, li)
// element k = 4 s + lg of row 16 i + li (zero past the layer's inputs) and
// of channel 16 j + li's weights; bias and LeakyReLU in FP32 on the way back.
// Calibration: each layer's per-channel output maximum over the wave's kept
// rows (iv >= 0), the quantity the vector-ALU form measures.
__device__ void hidden_layers_f32_mma(const TrackArgs& a, float* hb, const int* iv, int wave, int lane)
{
    const int li = lane & 15, lg = lane >> 4;
    float* rows = hb + (size_t)wave * 64 * HPM;
    const float* Wh = a.mlp + kHidden * kFeat + kHidden;   // hidden layers 2.. : [W 20x20, b 20]
    constexpr int KS = kHidden / 4;
    const int* kept = iv + wave * 64 + 4 * lg;   // kept[16 i + v] >= 0: row 16 i + 4 lg + v is a kept item
    for (int l = 0; l < a.n_hidden; ++l) {
        const int K = l == 0 ? kFeat : kHidden;
        const float* W = l == 0 ? a.mlp : Wh + (size_t)(l - 1) * (kHidden * kHidden + kHidden);   // [20][K]
        const float* b = W + kHidden * K;
        float w[2][KS], bn[2], m[2] = {0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = 16 * j + li;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + lg;
                w[j][ks] = (c < kHidden && k < K) ? W[c * K + k] : 0.f;
            }
            bn[j] = c < kHidden ? b[c] : 0.f;
        }
        // one row tile at a time: its outputs replace its inputs (the tile's
        // reads come first in the wave's program order), so only that tile's
        // accumulators are live
#pragma unroll 1
        for (int i = 0; i < 4; ++i) {
            f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (4 * ks >= K) break;
                const int k = 4 * ks + lg;
                const float x = k < K ? rows[(16 * i + li) * HPM + k] : 0.f;
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, w[j][ks], acc[j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = 16 * j + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float y = lrelu(acc[j][v] + bn[j], a.slope);
                    if (c < kHidden) rows[(16 * i + 4 * lg + v) * HPM + c] = y;
                    if (a.mlp_calib && kept[16 * i + v] >= 0) m[j] = fmaxf(m[j], fabsf(y));
                }
            }
        }
        if (a.mlp_calib) {
            // the largest |output| over the wave's kept items
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                float mm = fmaxf(m[j], __shfl_xor(m[j], 16));
                mm = fmaxf(mm, __shfl_xor(mm, 32));
                const int c = 16 * j + li;
                if (lg == 0 && c < kHidden)
                    atomicMax(reinterpret_cast<unsigned int*>(a.mlp_calib + calib_off(l + 1) + c), __float_as_uint(mm));
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// FP32 engines: the output layer and the histogram on the matrix cores in
// FP32 (v_mfma_f32_16x16x4_f32), from the last hidden activations in hb.  Output layer: K step s of
// row tile i gives lane (lg, li) element k = 4 s + lg of item 16 i + li and
// of column li's weights (K = 20, five steps).  Histogram: K step (i, v)
// gives item 16 i + 4 lg + v, whose output the lane holds in acc[v] (the B
// operand as it stands) and whose one-hot entry for interval 16 mt + li is
// the A operand; every product is exact and the sums are FP32.
__device__ void outputs_to_hist_f32(const TrackArgs& a, const float* hb, const int* iv, int n, int wave, int lane,
                                    f32x4 (&h)[2][kRegMT])
{
    const int li = lane & 15, lg = lane >> 4;
    const float* Wo = a.mlp + kHidden * kFeat + kHidden +
                      (size_t)(a.n_hidden - 1) * (kHidden * kHidden + kHidden);   // [n_out][kHidden]
    const float* bo = Wo + (size_t)a.n_out * kHidden;
    constexpr int KS = kHidden / 4;
#pragma unroll
    for (int jl = 0; jl < 2; ++jl) {
        const int jt = hist_tile(wave, blockIdx.x, jl);
        if (jt >= kMlpOutN / 16 || 16 * jt >= a.n_out) continue;
        const int c = 16 * jt + li;
        const bool used = c < a.n_out;
        float w[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) w[ks] = used ? Wo[(size_t)c * kHidden + 4 * ks + lg] : 0.f;
        const float bn = used ? bo[c] : 0.f;
#pragma unroll 1
        for (int sub = 0; sub < n; sub += SUB) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int4 q = *reinterpret_cast<const int4*>(iv + sub + 16 * i + 4 * lg);
                const int itv[4] = {q.x, q.y, q.z, q.w};
                const float* x = hb + (size_t)(sub + 16 * i + li) * HPM + lg;
                f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[4 * ks], w[ks], acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float y = fminf(softplus(acc[v] + bn), FLT_MAX);
#pragma unroll
                    for (int mt = 0; mt < kRegMT; ++mt) {
                        if (16 * mt >= a.n_intervals) break;
                        const float oh = itv[v] == 16 * mt + li ? 1.f : 0.f;
                        h[jl][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(oh, y, h[jl][mt], 0, 0, 0);
                    }
                }
            }
        }
    }
}

// Bytes of the layer-input rows: FP32 hidden activations [NT][HPM], or the
// matrix-core network's inputs [NT][KP] in E.
template <class E>
constexpr size_t row_tile_bytes()
{
    if constexpr (sizeof(E) == 4) return (size_t)NT * HPM * sizeof(float);
    else return (size_t)NT * Net<E>::KP * sizeof(E);
}

template <class E>
__device__ void track_event_mma(const TrackArgs& a, int e, char* smem)
{
    constexpr bool kF32 = sizeof(E) == 4;
    E* xa = reinterpret_cast<E*>(smem);            // [NT][KP] layer inputs (matrix-core network)
    float* hb = reinterpret_cast<float*>(smem);    // [NT][HPM] layer rows (FP32 network)
    int* iv = reinterpret_cast<int*>(smem + row_tile_bytes<E>());    // [NT] interval of each item
    int* nbv = iv + NT;                                               // [NT] neighbour interval, or -1
    int* st = nbv + NT;                                               // [NT] staged boundary items
    __shared__ int dropped_any;
    __shared__ int wave_count[NT / 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    f32x4 h[2][kRegMT];
#pragma unroll
    for (int jl = 0; jl < 2; ++jl)
#pragma unroll
        for (int mt = 0; mt < kRegMT; ++mt) h[jl][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (tid == 0) dropped_any = 0;
    const int64_t beg = a.offsets[e];
    const int64_t end = a.offsets[e + 1];
    int status = 0;
    if (beg < 0 || end < beg || end > a.n_tracks_total) status = PVF_EV_BAD_INPUT;
    else if (end - beg > a.max_tracks) status = PVF_EV_TOO_MANY_TRACKS;
    __syncthreads();

    const double z_max = edge(a, a.n_intervals);
    const bool two = a.boundary_mm > 0.0;

    // hidden layers of one item per thread, into hb (FP32) or xa; a wave
    // without a single kept item skips the network (its rows are never
    // accumulated, and it adds nothing to a calibration maximum)
    auto network_hidden = [&](const float* g, bool valid) {
        const bool any = __ballot(valid) != 0;
        if constexpr (kF32) {
#pragma unroll
            for (int k = 0; k < kFeat; ++k) hb[tid * HPM + k] = valid ? g[k] : 0.f;
            if (a.mlp_calib)
#pragma unroll
                for (int k = 0; k < kFeat; ++k) wave_amax(a.mlp_calib + calib_off(0) + k, valid ? g[k] : 0.f);
            __builtin_amdgcn_wave_barrier();
            if (any) hidden_layers_f32_mma(a, hb, iv, wave, lane);
        } else {
            float z[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) z[k] = valid ? g[k] : 0.f;
            if (a.mlp_calib)
#pragma unroll
                for (int k = 0; k < kFeat; ++k) wave_amax(a.mlp_calib + calib_off(0) + k, z[k]);
            store_inputs<E>(a, xa, tid, z);
            __builtin_amdgcn_wave_barrier();
            if (any) hidden_layers_mma<E>(a, xa, iv, wave, lane);
        }
    };
    auto outputs = [&](int n) {
        if constexpr (kF32) outputs_to_hist_f32(a, hb, iv, n, wave, lane, h);
        else outputs_to_hist<E>(a, xa, iv, n, wave, lane, h);
    };

    if (status == 0) {
        for (int64_t base = beg; base < end; base += NT) {
            const int64_t t = base + tid;
            int itv = -1, nb = -1;
            float g[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) g[k] = 0.f;
            if (t < end) bin_track(a, t, z_max, two, itv, nb, g, &dropped_any);
            iv[tid] = itv;   // read by the hidden layers' calibration
            network_hidden(g, itv >= 0);
            nbv[tid] = nb;
            __syncthreads();
            const int n_chunk = (int)((end - base) < NT ? (end - base) : NT);
            outputs(n_chunk);
            if (two) {
                // the chunk's boundary items, in item order, once more in the
                // neighbour's frame (the barrier below also ends every wave's
                // reads of xa and iv above)
                const bool is_b = nbv[tid] >= 0;
                const uint64_t m = __ballot(is_b);
                if (lane == 0) wave_count[wave] = __popcll(m);
                __syncthreads();
                int off = 0, n_st = 0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) {
                    off += w < wave ? wave_count[w] : 0;
                    n_st += wave_count[w];
                }
                if (is_b) st[off + __popcll(m & ((1ull << lane) - 1ull))] = tid;
                __syncthreads();
                if (n_st > 0) {
                    int inb = -1;
                    float gs[kFeat];
#pragma unroll
                    for (int k = 0; k < kFeat; ++k) gs[k] = 0.f;
                    if (tid < n_st) {
                        const int src = st[tid];
                        inb = nbv[src];
                        float fs[kFeat];
#pragma unroll
                        for (int k = 0; k < kFeat; ++k) fs[k] = a.feat[k][base + src];
                        features(a, fs, (double)fs[0], inb, gs);
                    }
                    __syncthreads();    // every read of nbv / st above is done
                    iv[tid] = inb;
                    network_hidden(gs, tid < n_st);
                    __syncthreads();
                    outputs(n_st);
                }
            }
            __syncthreads();   // xa and iv are rewritten by the next chunk
        }
    }
    // scaled histogram into the UNet's input rows (one sequence per event, or
    // one per interval of unit_bins bins, two guard rows on each side); the
    // lane holds intervals 16 mt + 4 lg + v of column 16 jt + li
    const int n_bins = a.n_out * a.n_intervals;
    const int U = n_bins / a.unit_bins;
    float* x0 = a.x0 + (int64_t)e * U * a.r0 + kGuard;
    // the store addresses are formed here, not held in registers (or spilled)
    // through the event
    int lo = lane;
    asm volatile("" : "+v"(lo));
    const int li = lo & 15, lg = lo >> 4;
#pragma unroll
    for (int jl = 0; jl < 2; ++jl) {
        const int jt = hist_tile(wave, blockIdx.x, jl);
        const int c = 16 * jt + li;
        if (jt >= kMlpOutN / 16 || c >= a.n_out) continue;
#pragma unroll
        for (int mt = 0; mt < kRegMT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int iw = 16 * mt + 4 * lg + v;
                if (iw >= a.n_intervals) continue;
                const int bb = iw * a.n_out + c;
                const int u = bb / a.unit_bins;
                x0[(int64_t)u * a.r0 + (bb - u * a.unit_bins)] = a.s_in * h[jl][mt][v];
            }
    }
    if (tid == 0) a.flags[e] = status | (dropped_any ? PVF_EV_TRACKS_DROPPED : 0);
    __syncthreads();   // the block's LDS is reused by its next event
}

// One block per event (queued == 0, grid = events), or the work-queue form
// of track_stage_queue (queued == 1) when the events outnumber the blocks
// that fit on the device at once.
template <class E>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void track_stage_mma(TrackArgs a, int n_events,
                                                                                         int queued)
{
    extern __shared__ __attribute__((aligned(16))) char smem_mma[];
    __shared__ int ticket;
    // one call site of the event body, for both forms
    for (int k = blockIdx.x;;) {
        if (queued) {
            if (threadIdx.x == 0) ticket = atomicAdd(a.queue_counter, 1);
            __syncthreads();
            k = ticket;
            __syncthreads();
        }
        if (k >= n_events) break;
        track_event_mma<E>(a, queued ? a.order[k] : k, smem_mma);
        if (!queued) break;
    }
}

// Queue order: a counting sort of the events by descending track count
// (counts clamped to [0, min(max_tracks, kOrderBuckets - 2) + 1]; malformed
// offsets count 0), in one block, with the count histogram and the scatter
// in LDS.  Events of equal (clamped) count may come out in any order: the
// order only schedules work, it never changes a result.  The kernel also
// resets the queue counter for the launch that follows, so no memset is
// needed (safe under graph capture).
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 4096;
__global__ __launch_bounds__(kOrderThreads) void track_order(TrackArgs a, int n_events)
{
    __shared__ int hist[kOrderBuckets];
    __shared__ int part[kOrderThreads];
    const int tid = threadIdx.x;
    const int cap = a.max_tracks < kOrderBuckets - 2 ? a.max_tracks : kOrderBuckets - 2;
    const int nb = cap + 2;
    auto bucket = [&](int e) {           // descending count -> ascending bucket
        const int64_t beg = a.offsets[e], end = a.offsets[e + 1];
        const int64_t t = (beg < 0 || end < beg || end > a.n_tracks_total) ? 0 : end - beg;
        return nb - 1 - (int)(t > cap ? cap + 1 : t);
    };
    for (int b = tid; b < nb; b += kOrderThreads) hist[b] = 0;
    __syncthreads();
    for (int e = tid; e < n_events; e += kOrderThreads) atomicAdd(&hist[bucket(e)], 1);
    __syncthreads();
    // exclusive scan of hist: each thread sums a run of buckets, the runs are
    // scanned in LDS, then each thread rewrites its run
    const int per = (nb + kOrderThreads - 1) / kOrderThreads;
    const int b0 = tid * per < nb ? tid * per : nb;
    const int b1 = b0 + per < nb ? b0 + per : nb;
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += hist[b];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kOrderThreads; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - sum;
    for (int b = b0; b < b1; ++b) {
        const int c = hist[b];
        hist[b] = run;
        run += c;
    }
    if (tid == 0) *a.queue_counter = 0;
    __syncthreads();
    for (int e = tid; e < n_events; e += kOrderThreads) a.order[atomicAdd(&hist[bucket(e)], 1)] = e;
}

}  // namespace

static_assert(NT * HP * sizeof(float) >= NT * Net<__bf16>::KP * 2 && NT * HP * sizeof(float) >= NT * Net<uint8_t>::KP,
              "the layer-input tile fits the FP32 hidden-activation space");
static size_t track_stage_lds_bytes(int n_out, int n_intervals)
{
    return sizeof(float) * ((size_t)n_out * n_intervals + NT * HP + SUB * (n_out + 1)) +
           sizeof(int) * (2 * NT + 3 * SUB + 1);
}

// Whether the event's histogram fits the registers of the matrix-core form.
static bool track_mma_ok(int n_intervals, int n_out) { return n_intervals <= kRegIntervals && n_out <= kMlpOutN; }

template <class E>
static size_t track_mma_lds_bytes()
{
    return row_tile_bytes<E>() + 3 * NT * sizeof(int);
}

template <class E>
hipError_t launch_track_typed(const TrackArgs& a, int n_events, int persistent_blocks, hipStream_t s)
{
    if (a.n_out < 1 || a.n_out > NT) return hipErrorInvalidValue;   // one thread per output column
    {
        if (track_mma_ok(a.n_intervals, a.n_out)) {
            // the queue (and its ordering pass) only when the events do not all
            // fit on the device at once
            const int queued = persistent_blocks > 0 && n_events > persistent_blocks && a.order && a.queue_counter;
            if (queued) {
                hipLaunchKernelGGL(track_order, dim3(1), dim3(kOrderThreads), 0, s, a, n_events);
                const hipError_t err = hipGetLastError();
                if (err != hipSuccess) return err;
            }
            hipLaunchKernelGGL(track_stage_mma<E>, dim3(queued ? persistent_blocks : n_events), dim3(NT),
                               track_mma_lds_bytes<E>(), s, a, n_events, queued);
            return hipGetLastError();
        }
    }
    const size_t lds = track_stage_lds_bytes(a.n_out, a.n_intervals);
    if (lds > 64 * 1024) {
        hipError_t err = hipFuncSetAttribute((const void*)track_stage<E>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err == hipSuccess)
            err = hipFuncSetAttribute((const void*)track_stage_queue<E>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
        if (err != hipSuccess) return err;
    }
    if (persistent_blocks <= 0 || !a.order || !a.queue_counter) {
        hipLaunchKernelGGL(track_stage<E>, dim3(n_events), dim3(NT), lds, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(track_order, dim3(1), dim3(kOrderThreads), 0, s, a, n_events);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int blocks = persistent_blocks < n_events ? persistent_blocks : n_events;
    hipLaunchKernelGGL(track_stage_queue<E>, dim3(blocks), dim3(NT), lds, s, a, n_events);
    return hipGetLastError();
}

hipError_t launch_track(const TrackArgs& a, int n_events, int persistent_blocks, hipStream_t s)
{
    if (a.mlp_dtype != PVF_FP32 && (!a.mlp_lp || a.n_out > kMlpOutN ||
                                    (a.mlp_dtype == PVF_FP8_E4M3 && (!a.mlp_in_inv || !a.mlp_col))))
        return hipErrorInvalidValue;
    switch (a.mlp_dtype) {
    case PVF_FP32: return launch_track_typed<float>(a, n_events, persistent_blocks, s);
    case PVF_BF16: return launch_track_typed<__bf16>(a, n_events, persistent_blocks, s);
    case PVF_FP16: return launch_track_typed<_Float16>(a, n_events, persistent_blocks, s);
    case PVF_FP8_E4M3: return launch_track_typed<uint8_t>(a, n_events, persistent_blocks, s);
    default: return hipErrorInvalidValue;
    }
}

int track_queue_blocks(int dtype, int n_intervals, int n_out, int cu_count)
{
    if (!track_mma_ok(n_intervals, n_out)) return 2 * cu_count;   // two 64 KB-LDS blocks per CU
    int per_cu = 0;
    hipError_t err = hipErrorInvalidValue;
    switch (dtype) {
    case PVF_FP32:
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, track_stage_mma<float>, NT,
                                                           track_mma_lds_bytes<float>());
        break;
    case PVF_BF16:
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, track_stage_mma<__bf16>, NT,
                                                           track_mma_lds_bytes<__bf16>());
        break;
    case PVF_FP16:
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, track_stage_mma<_Float16>, NT,
                                                           track_mma_lds_bytes<_Float16>());
        break;
    case PVF_FP8_E4M3:
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, track_stage_mma<uint8_t>, NT,
                                                           track_mma_lds_bytes<uint8_t>());
        break;
    default: break;
    }
    return (err == hipSuccess && per_cu > 0 ? per_cu : 1) * cu_count;
}

std::string track_kernel_name(int dtype, bool persistent, int n_intervals, int n_out)
{
    static const char* const kType[] = {"float", "__bf16", "_Float16", "unsigned char"};
    if (track_mma_ok(n_intervals, n_out)) return std::string("track_stage_mma<") + kType[dtype] + ">";
    return std::string(persistent ? "track_stage_queue<" : "track_stage<") + kType[dtype] + ">";
}

}  // namespace pvf
