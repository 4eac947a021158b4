// Host side of the C ABI declared in include/pvf.h: spec validation, the
// arena plan, weight unpacking and packing, and the launch sequence.
//
// Section 3 of arXiv:2602.19959 shapes this file: the specification is frozen
// and checked once (Prepare), all memory is a caller-provided arena bound at
// init, every launch goes to the one stream given at init (Execute), and the
// outputs stay on the device where the consumers read them (Extract).  Only
// pvf_init synchronises; pvf_execute enqueues and returns.
#include <cmath>
#include <cstring>
#include <new>

#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int kMaxBins = 16384;
constexpr size_t kMaxScaleFloats = 1 << 16;   // FP8 column / output / tensor scales
constexpr int kMaxBinsPerInterval = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ spec

pvf_status validate_spec(const pvf_spec* s)
{
    if (s->abi_version != PVF_ABI_VERSION) return PVF_ERR_INVALID_ARGUMENT;
    if (s->max_events < 1 || s->max_tracks_per_event < 0 || s->max_peaks_per_event < 1 ||
        s->max_tracks_total < 0 || s->max_tracks_total > INT32_MAX)
        return PVF_ERR_INVALID_ARGUMENT;
    if (s->compute_dtype < PVF_FP32 || s->compute_dtype > PVF_FP8_E4M3) return PVF_ERR_INVALID_ARGUMENT;
    if (!(std::isfinite(s->z_min_mm) && std::isfinite(s->bin_width_mm) && s->bin_width_mm > 0 &&
          std::isfinite(s->peak_min) && std::isfinite(s->integral_min)))
        return PVF_ERR_INVALID_ARGUMENT;
    if (s->half_window < 0) return PVF_ERR_INVALID_ARGUMENT;
    if (s->unet_layout != PVF_LAYOUT_EVENT && s->unet_layout != PVF_LAYOUT_INTERVAL) return PVF_ERR_INVALID_ARGUMENT;
    if (s->reserved != 0) return PVF_ERR_INVALID_ARGUMENT;
    if (s->n_levels < 2 || s->n_levels > kMaxLevels) return PVF_ERR_SHAPE;
    // the head epilogue holds all level-0 channels in one 32- or 64-wide tile
    if (s->base_channels != 32 && s->base_channels != 64) return PVF_ERR_SHAPE;
    if (s->n_bins < 4 || s->n_bins > kMaxBins) return PVF_ERR_SHAPE;
    if (s->bins_per_interval < 1 || s->bins_per_interval > kMaxBinsPerInterval ||
        s->n_bins % s->bins_per_interval != 0)
        return PVF_ERR_SHAPE;
    const int seq = s->unet_layout == PVF_LAYOUT_INTERVAL ? s->bins_per_interval : s->n_bins;
    if (seq < 4 || seq % (1 << (s->n_levels - 1)) != 0) return PVF_ERR_SHAPE;
    const double interval_mm = s->bin_width_mm * s->bins_per_interval;
    if (!std::isfinite(s->boundary_mm) || s->boundary_mm < 0 || s->boundary_mm > 0.5 * interval_mm)
        return PVF_ERR_INVALID_ARGUMENT;
    if (s->max_peaks_per_event > s->n_bins) return PVF_ERR_SHAPE;
    return PVF_OK;
}

// Per-batch working regions (histogram rows, activations, probabilities,
// flags, the track work queue) for `events` events, laid out from byte
// offset `off`; returns the end.  The level geometry must already be set.
size_t layout_work(const pvf_spec* s, int events, size_t off, Plan* p)
{
    const size_t eb = (size_t)act_bytes(s->compute_dtype);
    const size_t E = (size_t)events * p->units;           // UNet sequences
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    p->zero_begin = off;
    p->x0 = take(E * p->lv[0].R * sizeof(float));
    const int n = s->n_levels;
    for (int l = 0; l < n; ++l) {
        const size_t rows = E * p->lv[l].R;
        p->a[l] = take(rows * p->lv[l].C * eb);
        if (l < n - 1) p->cat[l] = take(rows * 2 * p->lv[l].C * eb);
        if (l >= 1) p->pool[l] = take(rows * p->lv[l - 1].C * eb);
        if (l >= 1) p->d[l] = take(rows * p->lv[l].C * eb);
    }
    p->zero_end = off;
    p->prob = take((size_t)events * s->n_bins * sizeof(float));
    p->flags = take((size_t)events * sizeof(int32_t));
    p->order = take((size_t)events * sizeof(int32_t));
    p->queue = take(sizeof(int32_t));
    return off;
}

void make_plan(const pvf_spec* s, size_t weight_floats, Plan* p)
{
    p->n_levels = s->n_levels;
    p->c0 = s->base_channels;
    p->max_events = s->max_events;
    // UNet sequences: one per event, or one per interval
    p->units = s->unet_layout == PVF_LAYOUT_INTERVAL ? s->n_bins / s->bins_per_interval : 1;
    const int seq = s->n_bins / p->units;
    for (int l = 0; l < s->n_levels; ++l) {
        p->lv[l].L = seq >> l;
        p->lv[l].R = p->lv[l].L + 2 * kGuard;
        p->lv[l].C = s->base_channels << l;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    // weights and constants first, then the per-batch regions
    p->weights_bytes = weight_floats * sizeof(float);
    p->weights = take(p->weights_bytes);
    // 16-bit copy of the conv weights, same element offsets as the FP32 layout
    p->weights_lp = s->compute_dtype == PVF_FP32 ? 0 : take(weight_floats * 2);
    p->mlp_lp = s->compute_dtype == PVF_FP32 ? 0 : take(mlp_lp_elems(kMaxHiddenLayers) * 2);
    p->scales = s->compute_dtype == PVF_FP8_E4M3 ? take(kMaxScaleFloats * sizeof(float)) : 0;
    p->total = layout_work(s, s->max_events, off, p);
}

// ------------------------------------------------------------------ weights

struct NetShape {
    int n_feat, hidden, n_hidden, n_out, n_levels, c0, ksize;
};

// Expected element counts of the blob's tensors, in blob (forward) order.
std::vector<int64_t> blob_tensor_sizes(const NetShape& n)
{
    std::vector<int64_t> v;
    int in = n.n_feat;
    for (int l = 0; l < n.n_hidden; ++l) {
        v.push_back((int64_t)n.hidden * in);
        v.push_back(n.hidden);
        in = n.hidden;
    }
    v.push_back((int64_t)n.n_out * n.hidden);
    v.push_back(n.n_out);
    int cin = 1;
    for (int l = 0; l < n.n_levels; ++l) {
        const int c = n.c0 << l;
        v.push_back((int64_t)c * cin * n.ksize); v.push_back(c);
        v.push_back((int64_t)c * c * n.ksize);   v.push_back(c);
        cin = c;
    }
    for (int l = n.n_levels - 2; l >= 0; --l) {
        const int c = n.c0 << l, cu = n.c0 << (l + 1);
        v.push_back((int64_t)cu * c * 2);        v.push_back(c);
        v.push_back((int64_t)c * 2 * c * n.ksize); v.push_back(c);
        v.push_back((int64_t)c * c * n.ksize);   v.push_back(c);
    }
    v.push_back(n.c0);
    v.push_back(1);
    return v;
}

struct Blob {
    NetShape shape;
    float leaky, s_in;
    float shift[kFeat], scale[kFeat];
    std::vector<const float*> t;      // tensor pointers into `store`
    std::vector<std::vector<float>> store;
};

template <class T>
bool rd(const uint8_t*& p, const uint8_t* end, T* out)
{
    if ((size_t)(end - p) < sizeof(T)) return false;
    std::memcpy(out, p, sizeof(T));
    p += sizeof(T);
    return true;
}

pvf_status parse_blob(const void* data, size_t bytes, const pvf_spec* s, Blob* b)
{
    const uint8_t* p = static_cast<const uint8_t*>(data);
    const uint8_t* end = p + bytes;
    uint32_t version;
    if (bytes < 4 || std::memcmp(p, "PVFW", 4) != 0) return PVF_ERR_WEIGHTS;
    p += 4;
    if (!rd(p, end, &version) || version != 1) return PVF_ERR_WEIGHTS;
    int32_t sh[7];
    for (int i = 0; i < 7; ++i)
        if (!rd(p, end, &sh[i])) return PVF_ERR_WEIGHTS;
    b->shape = NetShape{sh[0], sh[1], sh[2], sh[3], sh[4], sh[5], sh[6]};
    const NetShape& n = b->shape;
    if (n.n_feat != kFeat || n.hidden != kHidden || n.n_hidden < 1 || n.n_hidden > kMaxHiddenLayers ||
        n.ksize != kTaps)
        return PVF_ERR_WEIGHTS;
    if (n.n_out != s->bins_per_interval || n.n_levels != s->n_levels || n.c0 != s->base_channels)
        return PVF_ERR_WEIGHTS;
    if (!rd(p, end, &b->leaky) || !rd(p, end, &b->s_in)) return PVF_ERR_WEIGHTS;
    for (int k = 0; k < kFeat; ++k)
        if (!rd(p, end, &b->shift[k])) return PVF_ERR_WEIGHTS;
    for (int k = 0; k < kFeat; ++k)
        if (!rd(p, end, &b->scale[k])) return PVF_ERR_WEIGHTS;
    int32_t nt;
    if (!rd(p, end, &nt)) return PVF_ERR_WEIGHTS;
    const std::vector<int64_t> want = blob_tensor_sizes(n);
    if (nt != (int32_t)want.size()) return PVF_ERR_WEIGHTS;
    for (int i = 0; i < nt; ++i) {
        int32_t c;
        if (!rd(p, end, &c) || c != want[i]) return PVF_ERR_WEIGHTS;
    }
    b->store.resize(nt);
    for (int i = 0; i < nt; ++i) {
        const size_t nb = (size_t)want[i] * sizeof(float);
        if ((size_t)(end - p) < nb) return PVF_ERR_WEIGHTS;
        b->store[i].resize(want[i]);
        std::memcpy(b->store[i].data(), p, nb);
        p += nb;
        for (float v : b->store[i])
            if (!std::isfinite(v)) return PVF_ERR_WEIGHTS;
    }
    if (p != end) return PVF_ERR_WEIGHTS;
    b->t.resize(nt);
    for (int i = 0; i < nt; ++i) b->t[i] = b->store[i].data();
    return PVF_OK;
}

size_t weight_layout(const NetShape& n, WeightLayout* w)
{
    size_t off = 0;
    auto take = [&](size_t floats) { size_t o = off; off += (floats + 63) / 64 * 64; return o; };
    size_t mlp = (size_t)n.hidden * n.n_feat + n.hidden +
                 (size_t)(n.n_hidden - 1) * (n.hidden * n.hidden + n.hidden) + (size_t)n.n_out * n.hidden + n.n_out;
    w->mlp_count = mlp;
    w->mlp = take(mlp);
    w->first_w = take((size_t)n.c0 * n.ksize);
    w->first_b = take(n.c0);
    for (int l = 0; l < n.n_levels; ++l) {
        const int c = n.c0 << l, cin = l == 0 ? 1 : (n.c0 << (l - 1));
        if (l > 0) {
            w->enc[l][0] = {take((size_t)c * n.ksize * cin), take(c), cin, c, n.ksize};
        }
        w->enc[l][1] = {take((size_t)c * n.ksize * c), take(c), c, c, n.ksize};
    }
    for (int l = n.n_levels - 2; l >= 0; --l) {
        const int c = n.c0 << l, cu = n.c0 << (l + 1);
        w->up[l] = {take((size_t)2 * c * cu), take(c), cu, c, 1};
        w->dec[l][0] = {take((size_t)c * n.ksize * 2 * c), take(c), 2 * c, c, n.ksize};
        w->dec[l][1] = {take((size_t)c * n.ksize * c), take(c), c, c, n.ksize};
    }
    w->head_w = take(n.c0);
    w->head_b = take(1);
    w->total = off;
    return off;
}

// [Cout][Cin][k] -> [Cout][k][Cin]
void pack_conv(const float* src, int cout, int cin, int k, float* dst)
{
    for (int o = 0; o < cout; ++o)
        for (int j = 0; j < k; ++j)
            for (int c = 0; c < cin; ++c)
                dst[((size_t)o * k + j) * cin + c] = src[((size_t)o * cin + c) * k + j];
}

// transposed conv [Cin][Cout][2] -> GEMM rows n = j*Cout + o over k = Cin
void pack_convT(const float* src, int cin, int cout, float* dst)
{
    for (int j = 0; j < 2; ++j)
        for (int o = 0; o < cout; ++o)
            for (int c = 0; c < cin; ++c)
                dst[((size_t)j * cout + o) * cin + c] = src[((size_t)c * cout + o) * 2 + j];
}

void pack_weights(const Blob& b, const WeightLayout& w, std::vector<float>& out)
{
    const NetShape& n = b.shape;
    out.assign(w.total, 0.f);
    size_t ti = 0;
    // MLP: blob order, contiguous
    size_t pos = w.mlp;
    for (int l = 0; l <= n.n_hidden; ++l) {
        for (int q = 0; q < 2; ++q) {
            const size_t cnt = b.store[ti].size();
            std::memcpy(&out[pos], b.t[ti], cnt * sizeof(float));
            pos += cnt;
            ++ti;
        }
    }
    for (int l = 0; l < n.n_levels; ++l) {
        const int c = n.c0 << l, cin = l == 0 ? 1 : (n.c0 << (l - 1));
        if (l == 0) {
            std::memcpy(&out[w.first_w], b.t[ti], sizeof(float) * c * n.ksize);
            std::memcpy(&out[w.first_b], b.t[ti + 1], sizeof(float) * c);
        } else {
            pack_conv(b.t[ti], c, cin, n.ksize, &out[w.enc[l][0].w]);
            std::memcpy(&out[w.enc[l][0].b], b.t[ti + 1], sizeof(float) * c);
        }
        ti += 2;
        pack_conv(b.t[ti], c, c, n.ksize, &out[w.enc[l][1].w]);
        std::memcpy(&out[w.enc[l][1].b], b.t[ti + 1], sizeof(float) * c);
        ti += 2;
    }
    for (int l = n.n_levels - 2; l >= 0; --l) {
        const int c = n.c0 << l, cu = n.c0 << (l + 1);
        pack_convT(b.t[ti], cu, c, &out[w.up[l].w]);
        std::memcpy(&out[w.up[l].b], b.t[ti + 1], sizeof(float) * c);
        ti += 2;
        pack_conv(b.t[ti], c, 2 * c, n.ksize, &out[w.dec[l][0].w]);
        std::memcpy(&out[w.dec[l][0].b], b.t[ti + 1], sizeof(float) * c);
        ti += 2;
        pack_conv(b.t[ti], c, c, n.ksize, &out[w.dec[l][1].w]);
        std::memcpy(&out[w.dec[l][1].b], b.t[ti + 1], sizeof(float) * c);
        ti += 2;
    }
    std::memcpy(&out[w.head_w], b.t[ti], sizeof(float) * n.c0);
    std::memcpy(&out[w.head_b], b.t[ti + 1], sizeof(float));
}

// float -> bfloat16, round to nearest even (NaN kept quiet)
uint16_t to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

uint16_t to_f16(float f)
{
    _Float16 h = (_Float16)f;      // IEEE round to nearest even
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

// float -> OCP e4m3 (finite range +-448, saturated), round to nearest even:
// the nearest of the 127 non-negative finite codes, ties to the even code.
uint8_t to_e4m3_host(float f)
{
    static float tab[127];
    static bool init = false;
    if (!init) {
        for (int b = 0; b < 127; ++b) {
            const int e = b >> 3, m = b & 7;
            tab[b] = e ? std::ldexp(1.f + m / 8.f, e - 7) : std::ldexp(m / 8.f, -6);
        }
        init = true;
    }
    const bool neg = std::signbit(f);
    float a = std::fabs(f);
    if (!(a < 448.f)) a = 448.f;                     // saturate (NaN never reaches here)
    int lo = 0, hi = 126;                            // largest code with tab <= a
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tab[mid] <= a) lo = mid; else hi = mid - 1;
    }
    int b = lo;
    if (lo < 126) {
        const float d0 = a - tab[lo], d1 = tab[lo + 1] - a;
        if (d1 < d0 || (d1 == d0 && ((lo + 1) & 1) == 0)) b = lo + 1;
    }
    return (uint8_t)(b | (neg ? 0x80 : 0));
}

// 16-bit copy of every conv weight tensor the matrix-core kernels read
void pack_weights_lp(const WeightLayout& w, const NetShape& n, const std::vector<float>& f32, int dtype,
                     std::vector<uint16_t>& out)
{
    out.assign(w.total, 0);
    auto conv = [&](const WeightLayout::Conv& c) {
        const size_t cnt = (size_t)c.cout * (c.taps == 1 ? 2 : c.taps) * c.cin;
        for (size_t i = 0; i < cnt; ++i)
            out[c.w + i] = dtype == PVF_BF16 ? to_bf16(f32[c.w + i]) : to_f16(f32[c.w + i]);
    };
    for (int l = 0; l < n.n_levels; ++l) {
        if (l > 0) conv(w.enc[l][0]);
        conv(w.enc[l][1]);
    }
    for (int l = n.n_levels - 2; l >= 0; --l) {
        conv(w.up[l]);
        conv(w.dec[l][0]);
        conv(w.dec[l][1]);
    }
}

size_t weight_floats_for(const pvf_spec* s)
{
    NetShape n{kFeat, kHidden, 6, s->bins_per_interval, s->n_levels, s->base_channels, kTaps};
    // the MLP depth is read from the blob; reserve for the deepest supported
    n.n_hidden = kMaxHiddenLayers;
    WeightLayout w;
    return weight_layout(n, &w);
}

}  // namespace
}  // namespace pvf

using namespace pvf;

struct pvf_engine {
    pvf_spec spec;
    Plan plan;
    WeightLayout wl;
    int n_hidden = 0;
    float leaky = 0.f, s_in = 0.f, head_b = 0.f;
    float shift[kFeat] = {}, scale[kFeat] = {};
    char* arena = nullptr;
    char* scratch = nullptr;             // the library's scratch on this engine's device
    hipStream_t stream = nullptr;
    std::vector<std::string> names;      // one per launch of pvf_execute
    std::vector<std::string> kernels;    // kernel instance of each launch
    struct ConvLaunch {
        int n = 0, cin = 0, taps = 0, cout = 0;
        Epi epi = EPI_STORE;
        int variant = -1;
        const WeightLayout::Conv* w = nullptr;
        std::vector<int> in_src;      // launches whose stored outputs form this input, in channel order
        size_t col = 0;               // FP8: offsets (floats) into the scales region
        size_t fold = 0;              // FP8 stored outputs: [n] s_n / a_out, then [n] bias / a_out
        bool first = false;           // enc0.c2: may compute the first convolution (the launch before it) itself
        bool up = false;              // dec(l+1).c2: may run the transposed conv (the launch after it) in its epilogue
        bool dec0 = false;            // dec0.c2+head: may compute dec0.c1 (the launch before it) in the same kernel
    };
    std::vector<int> out_channels;       // channels of the tensor launch i stores (0: none)
    std::vector<size_t> outinv_off, a_off;   // FP8: 1/a and a of launch i's stored tensor
    std::vector<size_t> calib_off;       // offset of launch i's channels in the calibration table
    size_t calib_total = 0;
    size_t calib_mlp_off = 0;            // the track network's layer inputs, after the UNet tensors
    size_t mlp_in_inv_off = 0, mlp_col_off = 0;   // FP8: network scales in the scales region
    float* calib_table = nullptr;        // set only during pvf_calibrate
    std::vector<ConvLaunch> conv;        // per launch; variant -1 = not a conv launch
    std::vector<hipEvent_t> events;      // launch boundaries when profiling
    bool profiling = false;
    int track_blocks = 0;                // > 0: persistent work-queue track stage
    int cu_count = 0;
    hipGraph_t graph = nullptr;          // pvf_graph_capture
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

template <class T>
T* at(pvf_engine* e, size_t off) { return reinterpret_cast<T*>(e->arena + off); }

// Whether launch i (enc0.c2) computes the first convolution in its staging:
// its tile variant can, and no calibration is running (the calibration reads
// the first convolution's stored output).
bool fuses_first(const pvf_engine* e, int i)
{
    return e->conv[i].first && !e->calib_table && conv_first_ok(e->spec.compute_dtype, e->conv[i].variant);
}

// Whether launch i (a decoder conv2 below the deepest level) runs the
// transposed conv that follows it in its epilogue: 16-bit and FP8 engines,
// a tile variant whose tile holds all its output channels, and no
// calibration running (the calibration reads the stored output).
bool fuses_up(const pvf_engine* e, int i)
{
    const auto& c = e->conv[i];
    const int dt = e->spec.compute_dtype;
    return c.up && !e->calib_table && dt != PVF_FP32 && conv_variant_ok(dt, c.variant, c.n, c.cin, c.taps, EPI_UP);
}

// Whether launch i (dec0.c2 + head) computes dec0.c1 in the same kernel:
// 16-bit and FP8 engines, a variant that does, and no calibration running
// (the calibration reads dec0.c1's stored output).
bool fuses_dec0(const pvf_engine* e, int i)
{
    return e->conv[i].dec0 && !e->calib_table && conv_dec0_ok(e->spec.compute_dtype, e->conv[i].variant);
}

// Kernel names of dec0.c1 and dec0.c2 + head for the head's current variant.
void name_dec0(pvf_engine* e)
{
    const int dt = e->spec.compute_dtype;
    for (size_t i = 1; i < e->conv.size(); ++i) {
        const auto& c = e->conv[i];
        if (!c.dec0) continue;
        const auto& p = e->conv[i - 1];
        const bool f = fuses_dec0(e, (int)i);
        e->kernels[i] = conv_kernel_name(dt, c.variant, c.cin, c.taps, c.epi);
        e->kernels[i - 1] = f ? "conv (in " + e->names[i] + ")" : conv_kernel_name(dt, p.variant, p.cin, p.taps, p.epi);
    }
}

// Kernel names of the launches a fused transposed conv involves.
void name_up(pvf_engine* e)
{
    const int dt = e->spec.compute_dtype;
    for (size_t i = 0; i + 1 < e->conv.size(); ++i) {
        const auto& c = e->conv[i];
        if (!c.up) continue;
        const auto& u = e->conv[i + 1];
        const bool f = fuses_up(e, (int)i);
        e->kernels[i] = conv_kernel_name(dt, c.variant, c.cin, c.taps, f ? EPI_UP : c.epi);
        e->kernels[i + 1] = f ? "transposed conv (in " + e->names[i] + ")"
                              : conv_kernel_name(dt, u.variant, u.cin, u.taps, u.epi);
    }
}

// Kernel names of enc0.c1 and enc0.c2 for enc0.c2's current variant.
void name_first(pvf_engine* e)
{
    for (size_t i = 1; i < e->conv.size(); ++i) {
        const auto& c = e->conv[i];
        if (!c.first) continue;
        const bool f = conv_first_ok(e->spec.compute_dtype, c.variant);
        e->kernels[i] = f ? conv_first_kernel_name(e->spec.compute_dtype, c.variant)
                          : conv_kernel_name(e->spec.compute_dtype, c.variant, c.cin, c.taps, c.epi);
        e->kernels[i - 1] = f ? "first_conv (in enc0.c2)" : "first_conv";
    }
}

void build_names(pvf_engine* e)
{
    const int n = e->spec.n_levels;
    const int c0 = e->spec.base_channels;
    const WeightLayout& W = e->wl;
    e->names.clear();
    e->kernels.clear();
    e->conv.clear();
    e->out_channels.clear();
    auto find = [&](const std::string& name) {
        for (size_t i = 0; i < e->names.size(); ++i)
            if (e->names[i] == name) return (int)i;
        return -1;
    };
    auto plain = [&](const std::string& name, const std::string& kernel, int stored_channels) {
        e->names.push_back(name);
        e->kernels.push_back(kernel);
        e->conv.push_back({});
        e->out_channels.push_back(stored_channels);
    };
    auto conv = [&](const std::string& name, int gemm_n, int cout, int cin, int taps, Epi epi,
                    const WeightLayout::Conv* w, std::vector<int> src) {
        pvf_engine::ConvLaunch c;
        c.n = gemm_n;
        c.cout = cout;
        c.cin = cin;
        c.taps = taps;
        c.epi = epi;
        c.w = w;
        c.in_src = std::move(src);
        c.variant = conv_default_variant(e->spec.compute_dtype, gemm_n, cin, taps, epi);
        e->names.push_back(name);
        e->kernels.push_back(conv_kernel_name(e->spec.compute_dtype, c.variant, cin, taps, epi));
        e->conv.push_back(c);
        e->out_channels.push_back(epi == EPI_HEAD ? 0 : cout);
    };
    plain("track", track_kernel_name(e->spec.compute_dtype, e->track_blocks > 0,
                                    e->spec.n_bins / e->spec.bins_per_interval, e->spec.bins_per_interval), 0);
    for (int l = 0; l < n; ++l) {
        const std::string L = std::to_string(l);
        const int C = c0 << l;
        if (l == 0) plain("enc0.c1", "first_conv", C);
        else conv("enc" + L + ".c1", C, C, C / 2, kTaps, EPI_STORE, &W.enc[l][0],
                  {find("enc" + std::to_string(l - 1) + ".c2")});
        conv("enc" + L + ".c2", C, C, C, kTaps, l < n - 1 ? EPI_POOL : EPI_STORE, &W.enc[l][1],
             {find("enc" + L + ".c1")});
    }
    for (int l = n - 2; l >= 0; --l) {
        const std::string L = std::to_string(l);
        const int C = c0 << l;
        conv("up" + L, 2 * C, C, 2 * C, 1, EPI_CONVT, &W.up[l],
             {find(l == n - 2 ? "enc" + std::to_string(n - 1) + ".c2" : "dec" + std::to_string(l + 1) + ".c2")});
        conv("dec" + L + ".c1", C, C, 2 * C, kTaps, EPI_STORE, &W.dec[l][0], {find("enc" + L + ".c2"), find("up" + L)});
        conv(l == 0 ? "dec0.c2+head" : "dec" + L + ".c2", C, C, C, kTaps, l == 0 ? EPI_HEAD : EPI_STORE,
             &W.dec[l][1], {find("dec" + L + ".c1")});
    }
    plain("peaks", "peak_finder", 0);
    // enc0.c2 (launch 2, after the track stage and enc0.c1) can take the first
    // convolution into its staging when it has the max-pool epilogue
    if (n > 1) e->conv[2].first = true;
    name_first(e);
    // dec(l+1).c2 feeds only up(l) (l + 1 <= n - 2): it may run it itself, and
    // takes a tile variant that can when there is one
    for (int l = n - 3; l >= 0; --l) {
        const int p = find("dec" + std::to_string(l + 1) + ".c2");
        if (p < 0 || find("up" + std::to_string(l)) != p + 1) continue;
        auto& c = e->conv[p];
        c.up = true;
        const int v = conv_default_up_variant(e->spec.compute_dtype, c.n, c.cin);
        if (v >= 0) c.variant = v;
    }
    name_up(e);
    // dec0.c2 + head may compute dec0.c1 (the launch before it) itself
    {
        const int h = find("dec0.c2+head");
        if (h > 0 && find("dec0.c1") == h - 1) {
            auto& c = e->conv[h];
            c.dec0 = true;
            const int v = conv_default_dec0_variant(e->spec.compute_dtype);
            if (v >= 0 && conv_variant_ok(e->spec.compute_dtype, v, c.n, c.cin, c.taps, c.epi)) c.variant = v;
        }
    }
    name_dec0(e);
    // calibration table: the stored tensors' channels, in launch order
    e->calib_off.assign(e->names.size(), 0);
    e->calib_total = 0;
    for (size_t i = 0; i < e->names.size(); ++i) {
        e->calib_off[i] = e->calib_total;
        e->calib_total += e->out_channels[i];
    }
    e->calib_mlp_off = e->calib_total;
    e->calib_total += mlp_calib_channels(e->n_hidden);
}

bool misaligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; }


// The track network's layers inside the packed FP32 weights (blob order):
// W [N][K] row-major, then b [N].
struct MlpLayer { size_t w, b; int k, n; };
std::vector<MlpLayer> mlp_layers(const pvf_engine* e)
{
    std::vector<MlpLayer> v;
    size_t off = e->wl.mlp;
    int k = kFeat;
    for (int l = 0; l <= e->n_hidden; ++l) {
        const int n = l < e->n_hidden ? kHidden : e->spec.bins_per_interval;
        v.push_back({off, off + (size_t)n * k, k, n});
        off += (size_t)n * k + n;
        k = n;
    }
    return v;
}

// Matrix-core copy of the network, [layer][cols][32] zero-padded, through
// `put(layer, n, k, w)` -> element.
template <class T, class Put>
void pack_mlp(const pvf_engine* e, const std::vector<float>& f32, std::vector<T>& out, Put put)
{
    out.assign(mlp_lp_elems(e->n_hidden), T{});
    size_t base = 0;
    const auto layers = mlp_layers(e);
    for (int l = 0; l <= e->n_hidden; ++l) {
        const MlpLayer& L = layers[l];
        for (int n = 0; n < L.n; ++n)
            for (int k = 0; k < L.k; ++k) out[base + (size_t)n * kMlpK + k] = put(l, n, k, f32[L.w + (size_t)n * L.k + k]);
        base += (size_t)mlp_layer_cols(l, e->n_hidden) * kMlpK;
    }
}

// FP8 engine set-up from a calibration table (per-channel absolute maxima of
// every stored tensor, layout of pvf_calibrate):
//   a_c   = amax_c / 448 (1 for a channel that never left zero);
//   W'    = W * a_c of the input channel, s_n = max|W'[n]| / 448 per column,
//   Wq    = e4m3(W' / s_n);
// the kernels then compute acc * s_n (+ bias) and store y / a of their output.
pvf_status setup_fp8(pvf_engine* e, const std::vector<float>& f32, const float* amax, size_t n_amax,
                     std::vector<uint8_t>& wq, std::vector<float>& sc, std::vector<uint8_t>& mlp_fp8)
{
    if (!amax || n_amax != e->calib_total) return PVF_ERR_INVALID_ARGUMENT;
    const size_t nl = e->names.size();
    std::vector<std::vector<float>> a(nl);
    for (size_t i = 0; i < nl; ++i)
        for (int c = 0; c < e->out_channels[i]; ++c) {
            const float m = amax[e->calib_off[i] + c];
            if (!std::isfinite(m) || m < 0.f) return PVF_ERR_INVALID_ARGUMENT;
            a[i].push_back(m > 0.f ? m / 448.f : 1.f);
        }
    sc.clear();
    e->outinv_off.assign(nl, 0);
    e->a_off.assign(nl, 0);
    for (size_t i = 0; i < nl; ++i) {
        if (e->out_channels[i] == 0) continue;
        e->outinv_off[i] = sc.size();
        for (float x : a[i]) sc.push_back(1.f / x);
        e->a_off[i] = sc.size();
        for (float x : a[i]) sc.push_back(x);
    }
    wq.assign(e->wl.total, 0);
    for (size_t i = 0; i < nl; ++i) {
        auto& c = e->conv[i];
        if (c.variant < 0) continue;
        std::vector<float> ain;                 // scale of every input channel
        for (int src : c.in_src) ain.insert(ain.end(), a[src].begin(), a[src].end());
        if ((int)ain.size() != c.cin) return PVF_ERR_INVALID_ARGUMENT;
        c.col = sc.size();
        const int per_n = c.taps * c.cin;       // packed row: [tap][cin]
        for (int n = 0; n < c.n; ++n) {
            const float* row = &f32[c.w->w + (size_t)n * per_n];
            float m = 0.f;
            for (int t = 0; t < c.taps; ++t)
                for (int ch = 0; ch < c.cin; ++ch) m = std::max(m, std::fabs(row[t * c.cin + ch] * ain[ch]));
            const float sn = m > 0.f ? m / 448.f : 1.f;
            sc.push_back(sn);
            for (int t = 0; t < c.taps; ++t)
                for (int ch = 0; ch < c.cin; ++ch)
                    wq[c.w->w + (size_t)n * per_n + t * c.cin + ch] = to_e4m3_host(row[t * c.cin + ch] * ain[ch] / sn);
        }
        // stored outputs: the column scale and the bias divided by the output
        // channel's scale (a positive factor, which LeakyReLU commutes with),
        // 16-byte aligned so a lane reads its four columns with one load each
        if (c.epi != EPI_HEAD) {
            if ((int)a[i].size() != c.cout) return PVF_ERR_INVALID_ARGUMENT;
            while (sc.size() % 4) sc.push_back(0.f);
            c.fold = sc.size();
            for (int n = 0; n < c.n; ++n) sc.push_back(sc[c.col + n] / a[i][n % c.cout]);
            for (int n = 0; n < c.n; ++n) sc.push_back(f32[c.w->b + n % c.cout] / a[i][n % c.cout]);
        }
    }
    // the track network: per layer input-channel scales from the calibration,
    // folded into the weights, and one scale per column
    const auto layers = mlp_layers(e);
    std::vector<std::vector<float>> am(layers.size());
    size_t coff = e->calib_mlp_off;
    for (size_t l = 0; l < layers.size(); ++l)
        for (int k = 0; k < layers[l].k; ++k) {
            const float m = amax[coff++];
            if (!std::isfinite(m) || m < 0.f) return PVF_ERR_INVALID_ARGUMENT;
            am[l].push_back(m > 0.f ? m / 448.f : 1.f);
        }
    e->mlp_in_inv_off = sc.size();
    for (size_t l = 0; l < layers.size(); ++l)
        for (int k = 0; k < kMlpK; ++k) sc.push_back(k < layers[l].k ? 1.f / am[l][k] : 1.f);
    e->mlp_col_off = sc.size();
    std::vector<std::vector<float>> col(layers.size());
    for (size_t l = 0; l < layers.size(); ++l) {
        const MlpLayer& L = layers[l];
        for (int n = 0; n < mlp_layer_cols((int)l, e->n_hidden); ++n) {
            float m = 0.f;
            for (int k = 0; n < L.n && k < L.k; ++k) m = std::max(m, std::fabs(f32[L.w + (size_t)n * L.k + k] * am[l][k]));
            col[l].push_back(m > 0.f ? m / 448.f : 1.f);
            sc.push_back(col[l].back());
        }
    }
    pack_mlp<uint8_t>(e, f32, mlp_fp8, [&](int l, int n, int k, float w) { return to_e4m3_host(w * am[l][k] / col[l][n]); });
    if (sc.size() > kMaxScaleFloats) return PVF_ERR_SHAPE;
    return PVF_OK;
}

ConvArgs conv_args(pvf_engine* eng, const WeightLayout::Conv& c, const void* in, int ld_in, int rows_per_event,
                   int n_events, void* out, int ld_out)
{
    ConvArgs a{};
    const float* wbase = at<float>(eng, eng->plan.weights);
    a.in = in;
    a.ld_in = ld_in;
    a.cin = c.cin;
    a.m_rows = n_events * rows_per_event;
    a.r_in = rows_per_event;
    if (eng->spec.compute_dtype == PVF_FP32) a.w = wbase + c.w;
    else if (eng->spec.compute_dtype == PVF_FP8_E4M3) a.w = at<uint8_t>(eng, eng->plan.weights_lp) + c.w;
    else a.w = at<uint16_t>(eng, eng->plan.weights_lp) + c.w;
    a.bias = wbase + c.b;
    a.n = c.cout;
    a.slope = eng->leaky;
    a.out = out;
    a.ld_out = ld_out;
    a.r_out = rows_per_event;
    a.cout = c.cout;
    return a;
}

// Enqueue the whole path.  Weights and constants come from the engine's
// arena (eng->plan); the per-batch regions of plan P start at `work` (the
// arena itself, or the library's static scratch).
pvf_status enqueue(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out, hipStream_t s, const Plan& P,
                   char* work)
{
    const int E = tr->n_events;
    const int EU = E * eng->plan.units;          // UNet sequences
    const int dt = eng->spec.compute_dtype;
    const size_t eb = (size_t)act_bytes(dt);
    auto act = [&](size_t off) { return work + off; };
    auto wk = [&](size_t off) { return work + off; };
    const WeightLayout& W = eng->wl;
    const int n = P.n_levels;
    const float* wbase = at<float>(eng, eng->plan.weights);
    float* prob = out->d_prob_hist ? out->d_prob_hist : reinterpret_cast<float*>(wk(P.prob));
    int32_t* flags = reinterpret_cast<int32_t*>(wk(P.flags));
    int li = 0;                       // index of the launch about to be enqueued
    hipError_t err = hipSuccess;
    if (eng->profiling) err = hipEventRecord(eng->events[0], s);
    auto check = [&](hipError_t e) {
        if (err == hipSuccess) err = e;
        if (eng->profiling && err == hipSuccess) err = hipEventRecord(eng->events[li + 1], s);
        ++li;
    };
    auto var = [&]() { return eng->conv[li].variant; };

    // ---- FC stage: tracks -> scaled histogram rows of level 0
    TrackArgs ta{};
    ta.offsets = tr->d_event_offsets;
    static const float kDummy[1] = {0.f};
    for (int k = 0; k < kFeat; ++k) ta.feat[k] = tr->d_feat[k] ? tr->d_feat[k] : kDummy;
    ta.n_tracks_total = tr->n_tracks_total;
    ta.max_tracks = eng->spec.max_tracks_per_event;
    ta.mlp = wbase + W.mlp;
    ta.n_hidden = eng->n_hidden;
    ta.n_out = eng->spec.bins_per_interval;
    ta.n_intervals = eng->spec.n_bins / eng->spec.bins_per_interval;
    ta.z_min = eng->spec.z_min_mm;
    ta.interval_mm = eng->spec.bin_width_mm * eng->spec.bins_per_interval;
    for (int k = 0; k < kFeat; ++k) { ta.shift[k] = eng->shift[k]; ta.scale[k] = eng->scale[k]; }
    ta.slope = eng->leaky;
    ta.s_in = eng->s_in;
    ta.x0 = reinterpret_cast<float*>(wk(P.x0));
    ta.r0 = P.lv[0].R;
    ta.unit_bins = P.lv[0].L;
    ta.boundary_mm = eng->spec.boundary_mm;
    ta.mlp_dtype = dt;
    ta.mlp_lp = dt == PVF_FP32 ? nullptr : eng->arena + eng->plan.mlp_lp;
    if (dt == PVF_FP8_E4M3) {
        ta.mlp_in_inv = at<float>(eng, eng->plan.scales) + eng->mlp_in_inv_off;
        ta.mlp_col = at<float>(eng, eng->plan.scales) + eng->mlp_col_off;
    }
    ta.mlp_calib = eng->calib_table ? eng->calib_table + eng->calib_mlp_off : nullptr;
    ta.flags = flags;
    ta.order = reinterpret_cast<int32_t*>(wk(P.order));
    ta.queue_counter = reinterpret_cast<int32_t*>(wk(P.queue));
    check(launch_track(ta, E, eng->track_blocks, s));

    // Calibration (pvf_calibrate only): per-channel absolute maximum of the
    // tensor the launch just enqueued stored.
    auto calib = [&](const char* base, int ld, int level, int C, int ch_off) {
        if (!eng->calib_table || err != hipSuccess) return;
        AmaxArgs m{};
        m.src = base;
        m.elem_bytes = (int)eb;
        m.dtype = dt;
        m.rows = (int64_t)EU * P.lv[level].R;
        m.ld = ld;
        m.C = C;
        m.ch_off = ch_off;
        m.out = eng->calib_table + eng->calib_off[li - 1];
        err = launch_amax(m, s);
    };
    float* scales = dt == PVF_FP8_E4M3 ? at<float>(eng, eng->plan.scales) : nullptr;
    // one UNet convolution: FP8 scales of this launch, launch, then calibration
    auto conv = [&](ConvArgs a, int taps, Epi epi, int store_level, int store_ld, int store_ch_off) {
        if (scales) {
            a.col_scale = scales + eng->conv[li].col;
            a.out_inv_scale = epi == EPI_HEAD ? nullptr : scales + eng->outinv_off[li];
            a.fold_scale = epi == EPI_HEAD ? nullptr : scales + eng->conv[li].fold;
            a.fold_bias = epi == EPI_HEAD ? nullptr : scales + eng->conv[li].fold + eng->conv[li].n;
        }
        const int C = eng->conv[li].cout;
        if (a.first_x0)
            check(launch_conv_first(dt, a, var(), s));
        else
            check(launch_conv(dt, a, taps, epi, var(), s));
        if (epi != EPI_HEAD) {
            // a.out points at the tensor's first channel; the calibration reads
            // whole rows from the buffer start with the channel offset
            const char* base = static_cast<const char*>(a.out) - (size_t)store_ch_off * eb;
            calib(base, store_ld, store_level, C, store_ch_off);
        }
    };

    // ---- encoder
    const int first_li = li;          // enc0.c1
    const bool fused = fuses_first(eng, first_li + 1);
    if (fused) {
        check(hipSuccess);            // enc0.c2 computes it in its staging
    } else {
        FirstConvArgs fa{};
        fa.x0 = reinterpret_cast<float*>(wk(P.x0));
        fa.m_rows = EU * P.lv[0].R;
        fa.r0 = P.lv[0].R;
        fa.w = wbase + W.first_w;
        fa.b = wbase + W.first_b;
        fa.c0 = P.lv[0].C;
        fa.slope = eng->leaky;
        fa.out = act(P.a[0]);
        fa.out_inv_scale = scales ? scales + eng->outinv_off[li] : nullptr;
        check(launch_first_conv(fa, dt, s));
        calib(act(P.a[0]), P.lv[0].C, 0, P.lv[0].C, 0);
    }

    for (int l = 0; l < n; ++l) {
        const Level& lv = P.lv[l];
        if (l > 0) {
            const Level& up = P.lv[l - 1];
            conv(conv_args(eng, W.enc[l][0], act(P.pool[l]), up.C, lv.R, EU, act(P.a[l]), lv.C), kTaps, EPI_STORE,
                 l, lv.C, 0);
        }
        if (l < n - 1) {
            ConvArgs a = conv_args(eng, W.enc[l][1], act(P.a[l]), lv.C, lv.R, EU, act(P.cat[l]), 2 * lv.C);
            a.pool_out = act(P.pool[l + 1]);
            a.ld_pool = lv.C;
            a.r_pool = P.lv[l + 1].R;
            if (l == 0 && fused) {
                a.first_x0 = reinterpret_cast<float*>(wk(P.x0));
                a.first_w = wbase + W.first_w;
                a.first_b = wbase + W.first_b;
                a.first_inv_scale = scales ? scales + eng->outinv_off[first_li] : nullptr;
            }
            conv(a, kTaps, EPI_POOL, l, 2 * lv.C, 0);
        } else {
            conv(conv_args(eng, W.enc[l][1], act(P.a[l]), lv.C, lv.R, EU, act(P.d[l]), lv.C), kTaps, EPI_STORE, l,
                 lv.C, 0);
        }
    }
    // ---- decoder
    bool up_done = false;             // the previous launch ran this level's transposed conv
    for (int l = n - 2; l >= 0; --l) {
        const Level& lv = P.lv[l];
        const Level& lo = P.lv[l + 1];
        if (up_done) {
            check(hipSuccess);        // it ran in dec(l+1).c2's epilogue
        } else {
            ConvArgs u = conv_args(eng, W.up[l], act(P.d[l + 1]), lo.C, lo.R, EU,
                                   act(P.cat[l]) + (size_t)lv.C * eb, 2 * lv.C);
            u.n = 2 * lv.C;
            u.cout = lv.C;
            u.r_out = lv.R;
            conv(u, 1, EPI_CONVT, l, 2 * lv.C, lv.C);
        }
        const ConvArgs c1 = conv_args(eng, W.dec[l][0], act(P.cat[l]), 2 * lv.C, lv.R, EU, act(P.a[l]), lv.C);
        const bool dec0 = l == 0 && fuses_dec0(eng, li + 1);
        if (dec0) check(hipSuccess);  // computed inside the head launch
        else conv(c1, kTaps, EPI_STORE, l, lv.C, 0);
        if (l > 0) {
            ConvArgs c2 = conv_args(eng, W.dec[l][1], act(P.a[l]), lv.C, lv.R, EU, act(P.d[l]), lv.C);
            up_done = fuses_up(eng, li);
            if (up_done) {
                // up(l - 1) on this launch's output tiles: its weights, bias
                // and destination (the upsampled half of level l - 1's concat)
                const Level& lu = P.lv[l - 1];
                const WeightLayout::Conv& wu = W.up[l - 1];
                if (dt == PVF_FP8_E4M3) {
                    c2.up_w = at<uint8_t>(eng, eng->plan.weights_lp) + wu.w;
                    c2.up_fold_scale = scales + eng->conv[li + 1].fold;
                    c2.up_fold_bias = scales + eng->conv[li + 1].fold + eng->conv[li + 1].n;
                } else {
                    c2.up_w = at<uint16_t>(eng, eng->plan.weights_lp) + wu.w;
                }
                c2.up_b = wbase + wu.b;
                c2.up_out = act(P.cat[l - 1]) + (size_t)lu.C * eb;
                c2.up_ld = 2 * lu.C;
                c2.up_r_out = lu.R;
                c2.up_cout = lu.C;
                conv(c2, kTaps, EPI_UP, l, lv.C, 0);
            } else {
                conv(c2, kTaps, EPI_STORE, l, lv.C, 0);
            }
        } else {
            ConvArgs b = conv_args(eng, W.dec[0][1], act(P.a[0]), lv.C, lv.R, EU, nullptr, 0);
            b.head_w = wbase + W.head_w;
            b.head_b = eng->head_b;
            b.prob = prob;
            b.l_out = lv.L;
            if (dec0) {
                ConvArgs d1 = c1;
                if (scales) {        // FP8: dec0.c1's (launch li - 1) stored-output factors, the head's column scales
                    d1.col_scale = scales + eng->conv[li - 1].col;
                    d1.fold_scale = scales + eng->conv[li - 1].fold;
                    d1.fold_bias = scales + eng->conv[li - 1].fold + eng->conv[li - 1].n;
                    b.col_scale = scales + eng->conv[li].col;
                }
                check(launch_conv_dec0(dt, d1, b, var(), s));
            } else if (eng->conv[li].dec0 && conv_dec0_ok(dt, var())) {
                // a fused variant while calibrating: dec0.c1 ran on its own,
                // and the head takes the default tile
                check(launch_conv(dt, b, kTaps, EPI_HEAD, conv_default_variant(dt, b.n, b.cin, kTaps, EPI_HEAD), s));
            } else {
                conv(b, kTaps, EPI_HEAD, 0, 0, 0);
            }
        }
    }
    // ---- peaks
    PeakArgs pa{};
    pa.prob = prob;
    pa.L = eng->spec.n_bins;
    pa.flags = flags;
    pa.z_min = eng->spec.z_min_mm;
    pa.bw = eng->spec.bin_width_mm;
    pa.p_min = eng->spec.peak_min;
    pa.s_min = eng->spec.integral_min;
    pa.hw = eng->spec.half_window;
    pa.max_peaks = eng->spec.max_peaks_per_event;
    pa.n_vertices = out->d_n_vertices;
    pa.z = out->d_z;
    pa.peak_prob = out->d_peak_prob;
    pa.integral = out->d_integral;
    pa.status = out->d_event_status;
    pa.bin = out->d_bin;
    check(launch_peaks(pa, E, s));
    return err == hipSuccess ? PVF_OK : PVF_ERR_DEVICE;
}

}  // namespace

extern "C" {

void pvf_spec_default(pvf_spec* s)
{
    if (!s) return;
    std::memset(s, 0, sizeof(*s));
    s->abi_version = PVF_ABI_VERSION;
    s->max_events = 1000;
    s->max_tracks_per_event = 1500;
    s->max_peaks_per_event = 2000;
    s->max_tracks_total = 1500 * 1000;
    s->compute_dtype = PVF_FP32;
    s->n_levels = 4;
    s->base_channels = 32;
    s->n_bins = 4000;
    s->bins_per_interval = 100;
    s->half_window = 5;
    s->z_min_mm = -100.0;
    s->bin_width_mm = 0.1;
    s->peak_min = 0.01;
    s->integral_min = 0.2;
}

pvf_status pvf_arena_bytes(const pvf_spec* spec, size_t* out_bytes)
{
    if (!spec || !out_bytes) return PVF_ERR_INVALID_ARGUMENT;
    pvf_status st = validate_spec(spec);
    if (st != PVF_OK) return st;
    Plan p;
    make_plan(spec, weight_floats_for(spec), &p);
    *out_bytes = p.total;
    return PVF_OK;
}

static pvf_status init_impl(const pvf_spec* spec, const void* blob, size_t blob_bytes, const float* amax,
                            size_t n_amax, void* d_arena, size_t arena_bytes, void* stream, pvf_engine** out)
{
    if (out) *out = nullptr;
    if (!spec || !blob || !d_arena || !stream || !out) return PVF_ERR_INVALID_ARGUMENT;
    if (misaligned(d_arena, kAlign)) return PVF_ERR_ALIGNMENT;
    pvf_status st = validate_spec(spec);
    if (st != PVF_OK) return st;
    const bool fp8 = spec->compute_dtype == PVF_FP8_E4M3;
    if (fp8 != (amax != nullptr)) return PVF_ERR_INVALID_ARGUMENT;
    Plan plan;
    make_plan(spec, weight_floats_for(spec), &plan);
    if (arena_bytes < plan.total) return PVF_ERR_ARENA_TOO_SMALL;
    Blob b;
    st = parse_blob(blob, blob_bytes, spec, &b);
    if (st != PVF_OK) return st;

    pvf_engine* e = new (std::nothrow) pvf_engine();
    if (!e) return PVF_ERR_INVALID_ARGUMENT;
    e->spec = *spec;
    e->plan = plan;
    weight_layout(b.shape, &e->wl);
    e->n_hidden = b.shape.n_hidden;
    e->leaky = b.leaky;
    e->s_in = b.s_in;
    e->head_b = b.store.back()[0];
    for (int k = 0; k < kFeat; ++k) { e->shift[k] = b.shift[k]; e->scale[k] = b.scale[k]; }
    e->arena = static_cast<char*>(d_arena);
    e->stream = static_cast<hipStream_t>(stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&e->cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete e;
        return PVF_ERR_DEVICE;
    }
    e->track_blocks = track_queue_blocks(e->spec.compute_dtype, e->spec.n_bins / e->spec.bins_per_interval,
                                         e->spec.bins_per_interval, e->cu_count);
    e->scratch = scratch_base(dev);      // set-up of pvf_execute_scratch, once per device
    build_names(e);

    std::vector<float> packed;
    pack_weights(b, e->wl, packed);
    std::vector<uint16_t> packed_lp;
    std::vector<uint8_t> packed_fp8, mlp_fp8;
    std::vector<uint16_t> mlp_lp;
    std::vector<float> fp8_scales;
    if (fp8) {
        st = setup_fp8(e, packed, amax, n_amax, packed_fp8, fp8_scales, mlp_fp8);
        if (st != PVF_OK) {
            delete e;
            return st;
        }
    }
    hipError_t err = hipMemcpyAsync(e->arena + plan.weights, packed.data(), packed.size() * sizeof(float),
                                    hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess && fp8) {
        err = hipMemcpyAsync(e->arena + plan.weights_lp, packed_fp8.data(), packed_fp8.size(), hipMemcpyHostToDevice,
                             e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(e->arena + plan.scales, fp8_scales.data(), fp8_scales.size() * sizeof(float),
                                 hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(e->arena + plan.mlp_lp, mlp_fp8.data(), mlp_fp8.size(), hipMemcpyHostToDevice,
                                 e->stream);
    } else if (err == hipSuccess && spec->compute_dtype != PVF_FP32) {
        pack_weights_lp(e->wl, b.shape, packed, spec->compute_dtype, packed_lp);
        const int dt = spec->compute_dtype;
        pack_mlp<uint16_t>(e, packed, mlp_lp,
                           [dt](int, int, int, float w) { return dt == PVF_BF16 ? to_bf16(w) : to_f16(w); });
        err = hipMemcpyAsync(e->arena + plan.weights_lp, packed_lp.data(), packed_lp.size() * sizeof(uint16_t),
                             hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(e->arena + plan.mlp_lp, mlp_lp.data(), mlp_lp.size() * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, e->stream);
    }
    if (err == hipSuccess)
        err = hipMemsetAsync(e->arena + plan.zero_begin, 0, plan.zero_end - plan.zero_begin, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) {
        delete e;
        return PVF_ERR_DEVICE;
    }
    *out = e;
    return PVF_OK;
}

pvf_status pvf_init(const pvf_spec* spec, const void* blob, size_t blob_bytes, void* d_arena, size_t arena_bytes,
                    void* stream, pvf_engine** out)
{
    return init_impl(spec, blob, blob_bytes, nullptr, 0, d_arena, arena_bytes, stream, out);
}

pvf_status pvf_init_fp8(const pvf_spec* spec, const void* blob, size_t blob_bytes, const float* amax, size_t n_amax,
                        void* d_arena, size_t arena_bytes, void* stream, pvf_engine** out)
{
    if (!amax) return PVF_ERR_INVALID_ARGUMENT;
    return init_impl(spec, blob, blob_bytes, amax, n_amax, d_arena, arena_bytes, stream, out);
}

static pvf_status check_call(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out)
{
    if (!eng || !tr || !out) return PVF_ERR_INVALID_ARGUMENT;
    if (tr->n_events < 0 || tr->n_tracks_total < 0) return PVF_ERR_INVALID_ARGUMENT;
    if (tr->n_events > eng->spec.max_events || tr->n_tracks_total > eng->spec.max_tracks_total)
        return PVF_ERR_CAPACITY;
    if (tr->n_events == 0) return PVF_OK;
    if (!tr->d_event_offsets) return PVF_ERR_INVALID_ARGUMENT;
    if (misaligned(tr->d_event_offsets, 4)) return PVF_ERR_ALIGNMENT;
    for (int k = 0; k < kFeat; ++k) {
        if (tr->n_tracks_total > 0 && !tr->d_feat[k]) return PVF_ERR_INVALID_ARGUMENT;
        if (tr->d_feat[k] && misaligned(tr->d_feat[k], 4)) return PVF_ERR_ALIGNMENT;
    }
    if (!out->d_n_vertices || !out->d_z || !out->d_peak_prob || !out->d_integral || !out->d_event_status)
        return PVF_ERR_INVALID_ARGUMENT;
    if (misaligned(out->d_n_vertices, 4) || misaligned(out->d_z, 8) || misaligned(out->d_peak_prob, 4) ||
        misaligned(out->d_integral, 8) || misaligned(out->d_event_status, 4) ||
        (out->d_prob_hist && misaligned(out->d_prob_hist, 4)) || (out->d_bin && misaligned(out->d_bin, 4)))
        return PVF_ERR_ALIGNMENT;
    return PVF_OK;
}

pvf_status pvf_execute(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out)
{
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK || tr->n_events == 0) return st;
    return enqueue(eng, tr, out, eng->stream, eng->plan, eng->arena);
}

pvf_status pvf_execute_on(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out, void* stream)
{
    if (!stream) return PVF_ERR_INVALID_ARGUMENT;
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK || tr->n_events == 0) return st;
    return enqueue(eng, tr, out, static_cast<hipStream_t>(stream), eng->plan, eng->arena);
}

pvf_status pvf_execute_scratch(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out)
{
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK || tr->n_events == 0) return st;
    if (!eng->scratch) return PVF_ERR_DEVICE;
    // the per-batch regions laid out for this batch alone, from the scratch's start
    Plan P = eng->plan;
    P.total = layout_work(&eng->spec, tr->n_events, 0, &P);
    if (P.total > kScratchBytes) return PVF_ERR_SCRATCH_TOO_SMALL;
    // zero padding: the guard rows of every activation tensor
    const size_t eb = (size_t)act_bytes(eng->spec.compute_dtype);
    GuardZeroArgs g{};
    g.n_seq = (int64_t)tr->n_events * P.units;
    auto region = [&](size_t off, int level, size_t row_bytes) {
        g.r[g.n].base = eng->scratch + off;
        g.r[g.n].row_bytes = (int)row_bytes;
        g.r[g.n].rows_per_seq = P.lv[level].R;
        ++g.n;
    };
    region(P.x0, 0, sizeof(float));
    for (int l = 0; l < P.n_levels; ++l) {
        region(P.a[l], l, P.lv[l].C * eb);
        if (l < P.n_levels - 1) region(P.cat[l], l, 2 * P.lv[l].C * eb);
        if (l >= 1) region(P.pool[l], l, P.lv[l - 1].C * eb);
        if (l >= 1) region(P.d[l], l, P.lv[l].C * eb);
    }
    if (launch_zero_guard_rows(g, eng->stream) != hipSuccess) return PVF_ERR_DEVICE;
    return enqueue(eng, tr, out, eng->stream, P, eng->scratch);
}

pvf_status pvf_destroy(pvf_engine* eng)
{
    if (!eng) return PVF_ERR_INVALID_ARGUMENT;
    if (eng->graph_exec) (void)hipGraphExecDestroy(eng->graph_exec);
    if (eng->graph) (void)hipGraphDestroy(eng->graph);
    for (hipEvent_t ev : eng->events) (void)hipEventDestroy(ev);
    delete eng;
    return PVF_OK;
}

const char* pvf_status_string(pvf_status s)
{
    switch (s) {
    case PVF_OK: return "ok";
    case PVF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PVF_ERR_SHAPE: return "unsupported shape";
    case PVF_ERR_CAPACITY: return "batch exceeds the frozen capacity";
    case PVF_ERR_ARENA_TOO_SMALL: return "arena too small";
    case PVF_ERR_WEIGHTS: return "malformed weight blob or shape mismatch";
    case PVF_ERR_UNSUPPORTED_DTYPE: return "compute dtype not supported";
    case PVF_ERR_DEVICE: return "HIP runtime error";
    case PVF_ERR_ALIGNMENT: return "misaligned buffer";
    case PVF_ERR_SCRATCH_TOO_SMALL:
        return "batch too large for the library's fixed scratch (PVF_SCRATCH_BYTES = 64 MiB per device)";
    }
    return "unknown status";
}

int pvf_launch_count(const pvf_engine* eng) { return eng ? (int)eng->names.size() : 0; }

const char* pvf_launch_name(const pvf_engine* eng, int i)
{
    if (!eng || i < 0 || i >= (int)eng->names.size()) return nullptr;
    return eng->names[i].c_str();
}

const char* pvf_launch_kernel(const pvf_engine* eng, int i)
{
    if (!eng || i < 0 || i >= (int)eng->kernels.size()) return nullptr;
    return eng->kernels[i].c_str();
}

int pvf_launch_variant_count(const pvf_engine* eng, int i)
{
    if (!eng || i < 0 || i >= (int)eng->conv.size() || eng->conv[i].variant < 0) return 0;
    return conv_variant_count(eng->spec.compute_dtype);
}

int pvf_launch_variant(const pvf_engine* eng, int i)
{
    if (!eng || i < 0 || i >= (int)eng->conv.size()) return -1;
    return eng->conv[i].variant;
}

pvf_status pvf_set_launch_variant(pvf_engine* eng, int i, int v)
{
    if (!eng || i < 0 || i >= (int)eng->conv.size() || eng->conv[i].variant < 0) return PVF_ERR_INVALID_ARGUMENT;
    auto& c = eng->conv[i];
    if (!conv_variant_ok(eng->spec.compute_dtype, v, c.n, c.cin, c.taps, c.epi)) return PVF_ERR_INVALID_ARGUMENT;
    c.variant = v;
    eng->kernels[i] = conv_kernel_name(eng->spec.compute_dtype, v, c.cin, c.taps, c.epi);
    name_first(eng);
    name_up(eng);
    name_dec0(eng);
    return PVF_OK;
}

pvf_status pvf_autotune(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out, int reps)
{
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK) return st;
    if (tr->n_events == 0 || reps < 1) return PVF_ERR_INVALID_ARGUMENT;
    const bool was = eng->profiling;
    if (!was && (st = pvf_profile_enable(eng, 1)) != PVF_OK) return st;
    const int nl = (int)eng->names.size();
    std::vector<float> best(nl, 1e30f), ms(nl);
    std::vector<int> pick(nl, -1);
    for (int i = 0; i < nl; ++i) pick[i] = eng->conv[i].variant;
    const std::vector<pvf_engine::ConvLaunch> saved = eng->conv;
    for (int v = 0; v < conv_variant_count(eng->spec.compute_dtype) && st == PVF_OK; ++v) {
        // try variant v on every conv launch that accepts it, all in one pass
        bool any = false;
        for (int i = 0; i < nl; ++i) {
            auto& c = eng->conv[i];
            if (c.variant < 0) continue;
            if (conv_variant_ok(eng->spec.compute_dtype, v, c.n, c.cin, c.taps, c.epi)) { c.variant = v; any = true; }
            else c.variant = saved[i].variant;
        }
        if (!any) continue;
        for (int r = 0; r < reps + 1 && st == PVF_OK; ++r) {       // first pass warms up
            st = enqueue(eng, tr, out, eng->stream, eng->plan, eng->arena);
            if (st == PVF_OK && hipStreamSynchronize(eng->stream) != hipSuccess) st = PVF_ERR_DEVICE;
            if (st == PVF_OK && r > 0) st = pvf_profile_read(eng, ms.data(), nl);
            if (st != PVF_OK || r == 0) continue;
            for (int i = 0; i < nl; ++i) {
                // enc0.c2 is charged the first convolution too: it runs either
                // inside it or as the launch before it; a decoder conv2 that can
                // run the next transposed conv is charged that launch too, and
                // a transposed conv is not timed in a pass where it ran inside
                // the launch before it
                if (i > 0 && eng->conv[i - 1].up && fuses_up(eng, i - 1)) continue;
                if (i + 1 < nl && eng->conv[i + 1].dec0 && fuses_dec0(eng, i + 1)) continue;
                const float t = ms[i] + (eng->conv[i].first || eng->conv[i].dec0 ? ms[i - 1] : 0.f) +
                                (eng->conv[i].up ? ms[i + 1] : 0.f);
                if (eng->conv[i].variant == v && t < best[i]) { best[i] = t; pick[i] = v; }
            }
        }
    }
    for (int i = 0; i < nl; ++i) {
        eng->conv[i] = saved[i];
        if (saved[i].variant >= 0 && st == PVF_OK) pvf_set_launch_variant(eng, i, pick[i]);
    }
    if (!was) pvf_profile_enable(eng, 0);
    return st;
}

pvf_status pvf_set_track_schedule(pvf_engine* eng, int persistent)
{
    if (!eng || (persistent != 0 && persistent != 1)) return PVF_ERR_INVALID_ARGUMENT;
    const int n_intervals = eng->spec.n_bins / eng->spec.bins_per_interval;
    const int n_out = eng->spec.bins_per_interval;
    eng->track_blocks =
        persistent ? track_queue_blocks(eng->spec.compute_dtype, n_intervals, n_out, eng->cu_count) : 0;
    eng->kernels[0] = track_kernel_name(eng->spec.compute_dtype, persistent, n_intervals, n_out);
    return PVF_OK;
}

pvf_status pvf_graph_capture(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out)
{
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK) return st;
    if (tr->n_events == 0) return PVF_ERR_INVALID_ARGUMENT;
    if (eng->graph_exec) { (void)hipGraphExecDestroy(eng->graph_exec); eng->graph_exec = nullptr; }
    if (eng->graph) { (void)hipGraphDestroy(eng->graph); eng->graph = nullptr; }
    const bool was = eng->profiling;
    eng->profiling = false;                   // no event records inside the graph
    if (hipStreamBeginCapture(eng->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        eng->profiling = was;
        return PVF_ERR_DEVICE;
    }
    st = enqueue(eng, tr, out, eng->stream, eng->plan, eng->arena);
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(eng->stream, &g);
    eng->profiling = was;
    if (st != PVF_OK || end != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != PVF_OK ? st : PVF_ERR_DEVICE;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return PVF_ERR_DEVICE;
    }
    eng->graph = g;
    eng->graph_exec = x;
    return PVF_OK;
}

pvf_status pvf_graph_launch(pvf_engine* eng)
{
    if (!eng || !eng->graph_exec) return PVF_ERR_INVALID_ARGUMENT;
    return hipGraphLaunch(eng->graph_exec, eng->stream) == hipSuccess ? PVF_OK : PVF_ERR_DEVICE;
}

int64_t pvf_calibration_size(const pvf_engine* eng) { return eng ? (int64_t)eng->calib_total : -1; }

pvf_status pvf_calibrate(pvf_engine* eng, const pvf_tracks* tr, const pvf_vertices* out, float* d_amax, int64_t n)
{
    pvf_status st = check_call(eng, tr, out);
    if (st != PVF_OK) return st;
    if (!d_amax || n != (int64_t)eng->calib_total || tr->n_events == 0) return PVF_ERR_INVALID_ARGUMENT;
    if (eng->spec.compute_dtype == PVF_FP8_E4M3) return PVF_ERR_UNSUPPORTED_DTYPE;
    if (misaligned(d_amax, 4)) return PVF_ERR_ALIGNMENT;
    if (hipMemsetAsync(d_amax, 0, (size_t)n * sizeof(float), eng->stream) != hipSuccess) return PVF_ERR_DEVICE;
    eng->calib_table = d_amax;
    st = enqueue(eng, tr, out, eng->stream, eng->plan, eng->arena);
    eng->calib_table = nullptr;
    return st;
}

pvf_status pvf_profile_enable(pvf_engine* eng, int on)
{
    if (!eng) return PVF_ERR_INVALID_ARGUMENT;
    if (on && !eng->profiling) {
        eng->events.assign(eng->names.size() + 1, nullptr);
        for (auto& ev : eng->events)
            if (hipEventCreate(&ev) != hipSuccess) return PVF_ERR_DEVICE;
        eng->profiling = true;
    } else if (!on && eng->profiling) {
        for (hipEvent_t ev : eng->events) (void)hipEventDestroy(ev);
        eng->events.clear();
        eng->profiling = false;
    }
    return PVF_OK;
}

pvf_status pvf_profile_read(pvf_engine* eng, float* ms, int n)
{
    if (!eng || !ms || !eng->profiling || n > (int)eng->names.size() || n < 0) return PVF_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < n; ++i)
        if (hipEventElapsedTime(&ms[i], eng->events[i], eng->events[i + 1]) != hipSuccess) return PVF_ERR_DEVICE;
    return PVF_OK;
}

pvf_status pvf_debug_tensor(pvf_engine* eng, const char* name, int32_t n_events, float* d_dst, int64_t* out_count)
{
    if (!eng || !name || !out_count || n_events < 0 || n_events > eng->spec.max_events)
        return PVF_ERR_INVALID_ARGUMENT;
    const Plan& P = eng->plan;
    const int n = P.n_levels;
    GatherArgs g{};
    bool found = false;
    const int eb = act_bytes(eng->spec.compute_dtype);
    g.dtype = eng->spec.compute_dtype;
    auto launch_of = [&](const std::string& nm) {
        for (size_t i = 0; i < eng->names.size(); ++i)
            if (eng->names[i] == nm) return (int)i;
        return -1;
    };
    int producer = -1;     // launch whose stored tensor the name refers to
    auto set = [&](size_t off, int ld, int l, int C, int ch_off, int bytes) {
        g.src = eng->arena + off;
        g.src_bytes = bytes;
        g.ld = ld;
        g.r = P.lv[l].R;
        g.guard = kGuard;
        g.L = P.lv[l].L;
        g.C = C;
        g.ch_off = ch_off;
        found = true;
    };
    const std::string s(name);
    producer = launch_of(s.rfind("pool", 0) == 0 ? "enc" + s.substr(4) + ".c2" : s);
    if (s == "hist") set(P.x0, 1, 0, 1, 0, 4);
    if (s == "prob") {
        g.src = at<float>(eng, P.prob);
        g.src_bytes = 4;
        g.ld = 1; g.r = P.lv[0].L; g.guard = 0; g.L = P.lv[0].L; g.C = 1; g.ch_off = 0;
        found = true;
    }
    for (int l = 0; l < n; ++l) {
        const std::string L = std::to_string(l);
        const int C = P.lv[l].C;
        if (l < n - 1 && s == "enc" + L + ".c2") set(P.cat[l], 2 * C, l, C, 0, eb);
        if (l == n - 1 && s == "enc" + L + ".c2") set(P.d[l], C, l, C, 0, eb);
        if (l == n - 1 && s == "enc" + L + ".c1") set(P.a[l], C, l, C, 0, eb);
        if (l < n - 1 && s == "pool" + L) set(P.pool[l + 1], C, l + 1, C, 0, eb);
        if (l < n - 1 && s == "up" + L) set(P.cat[l], 2 * C, l, C, C, eb);
        if (l < n - 1 && s == "dec" + L + ".c1") set(P.a[l], C, l, C, 0, eb);
        if (l >= 1 && l < n - 1 && s == "dec" + L + ".c2") set(P.d[l], C, l, C, 0, eb);
    }
    if (!found) return PVF_ERR_INVALID_ARGUMENT;
    // a decoder conv2 that ran its transposed conv in the epilogue never
    // stores its own output
    if (producer >= 0 && s.rfind("dec", 0) == 0 && fuses_up(eng, producer)) return PVF_ERR_INVALID_ARGUMENT;
    if (producer >= 0 && producer + 1 < (int)eng->conv.size() && fuses_dec0(eng, producer + 1))
        return PVF_ERR_INVALID_ARGUMENT;
    if (g.src_bytes == 1) {
        if (producer < 0) return PVF_ERR_INVALID_ARGUMENT;
        g.ch_scale = at<float>(eng, P.scales) + eng->a_off[producer];
    }
    g.count = (int64_t)n_events * P.units * g.C * g.L;
    *out_count = g.count;
    if (!d_dst) return PVF_OK;
    g.dst = d_dst;
    return launch_gather(g, eng->stream) == hipSuccess ? PVF_OK : PVF_ERR_DEVICE;
}

}  // extern "C"
