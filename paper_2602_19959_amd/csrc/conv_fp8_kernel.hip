// UNet convolutions in FP8 (OCP e4m3) on the matrix cores, accumulated in
// FP32: the low-precision step of the mixed-precision roadmap in Section 5 of
// arXiv:2602.19959 taken one format further.
//
// Scaling (exact algebra, so only the FP8 roundings are approximations):
//   * every stored activation tensor has one scale per channel, a_c, from a
//     calibration run (absolute maximum / 448); it holds x / a_c in FP8;
//   * the consumer folds a_c into its weights, W'[n][c] = W[n][c] * a_c, and
//     quantises each GEMM column with its own scale s_n = max|W'[n]| / 448;
//   * so the accumulator times s_n is the conv output; the epilogue adds the
//     bias (+ LeakyReLU) in FP32 and stores y / a_out saturated to +-448.
// Max-pool of stored FP8 values equals the FP8 of the max (one scale per
// channel), and the head and sigmoid work on the FP32 dequantised values.
//
// MFMA: v_mfma_f32_16x16x32_fp8_fp8.  One stage = 32 input channels (32 bytes
// per row); each lane reads 8 consecutive channels (8 bytes) of its row (A)
// and of its column (B); the 32 lanes an LDS pass serves read 512 consecutive
// bytes, so rows need no padding or swizzle.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;            // input channels (bytes) per stage and row

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

// FP32 -> OCP e4m3, saturated to +-448 (the conversion itself turns values
// beyond the range into NaN), round to nearest even.
__device__ __forceinline__ uint8_t to_e4m3(float x)
{
    x = fminf(fmaxf(x, -448.f), 448.f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

__device__ __forceinline__ float e4m3_to_f32(uint8_t b)
{
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e ? ldexpf(1.f + m / 8.f, e - 7) : ldexpf(m / 8.f, -6);
    return (b & 0x80) ? -v : v;
}

template <int A, int B> struct Max { static constexpr int v = A > B ? A : B; };

template <int WM, int WN, int TMW, int TNW, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) void conv_mfma_fp8(ConvArgs a)
{
    constexpr int NT = WM * WN * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int XROWS = BM + TAPS - 1;
    constexpr int NCH = KC / 16;                 // 16-byte chunks per row
    constexpr int XV = XROWS * NCH;
    constexpr int WV = BN * TAPS * NCH;
    constexpr int OP = BN + 16;                  // epilogue tile pitch (bytes)
    constexpr int STAGE = XROWS * KC + BN * TAPS * KC;
    constexpr int SMEM = Max<STAGE, (EPI == EPI_HEAD ? 0 : BM * OP)>::v;

    __shared__ __attribute__((aligned(16))) uint8_t smem[SMEM];
    uint8_t* xs = smem;
    uint8_t* ws = smem + XROWS * KC;

    const uint8_t* in = static_cast<const uint8_t*>(a.in);
    const uint8_t* wt = static_cast<const uint8_t*>(a.w);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int li = lane & 15;
    const int lg = lane >> 4;
    // XCD-aware tile order (block b runs on XCD b % 8): every N tile of an M
    // tile runs back to back on one XCD, sharing its L2.
    const int n_tiles = (a.n + BN - 1) / BN;
    const int m_tiles = (int)((a.m_rows + BM - 1) / BM);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = (slot / n_tiles) * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BM;
    const int n0 = (slot % n_tiles) * BN;
    const int kw = TAPS * a.cin;

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c0 = 0; c0 < a.cin; c0 += KC) {
        for (int idx = tid; idx < XV; idx += NT) {
            const int row = idx / NCH, q = idx % NCH;
            const int64_t g = m0 - RAD + row;
            uint4 v = {0u, 0u, 0u, 0u};
            if (g >= 0 && g < a.m_rows) v = *reinterpret_cast<const uint4*>(in + g * a.ld_in + c0 + 16 * q);
            *reinterpret_cast<uint4*>(xs + row * KC + 16 * q) = v;
        }
        for (int idx = tid; idx < WV; idx += NT) {
            const int q = idx % NCH, rest = idx / NCH;
            const int tap = rest % TAPS, nn = rest / TAPS;
            uint4 v = {0u, 0u, 0u, 0u};
            if (n0 + nn < a.n)
                v = *reinterpret_cast<const uint4*>(wt + (int64_t)(n0 + nn) * kw + tap * a.cin + c0 + 16 * q);
            *reinterpret_cast<uint4*>(ws + rest * KC + 16 * q) = v;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            long av[TMW], bv[TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[i] = *reinterpret_cast<const long*>(xs + (wm * TMW * 16 + i * 16 + li + tap) * KC + 8 * lg);
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[j] = *reinterpret_cast<const long*>(ws + ((wn * TNW * 16 + j * 16 + li) * TAPS + tap) * KC + 8 * lg);
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    const int rw = wm * TMW * 16;
    const int cw = wn * TNW * 16;
    if constexpr (EPI == EPI_HEAD) {
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < TNW; ++j) {
                    const int col = n0 + cw + j * 16 + li;
                    s += lrelu(acc[i][j][v] * a.col_scale[col] + a.bias[col], a.slope) * a.head_w[col];
                }
                s += __shfl_xor(s, 8);
                s += __shfl_xor(s, 4);
                s += __shfl_xor(s, 2);
                s += __shfl_xor(s, 1);
                const int64_t r = m0 + rw + i * 16 + 4 * lg + v;
                if (li == 0 && r < a.m_rows) {
                    const int64_t e = r / a.r_in;
                    const int loc = (int)(r - e * a.r_in);
                    if (loc >= kGuard && loc < a.r_in - kGuard)
                        a.prob[e * a.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(s + a.head_b)));
                }
            }
        }
        return;
    } else {
        uint8_t* ot = smem;   // [BM][OP] bytes, reuses the stage buffers
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int col = cw + j * 16 + li;
            const int n = n0 + col;
            const int oc = EPI == EPI_CONVT ? n % a.cout : n;      // output channel
            const float cs = n < a.n ? a.col_scale[n] : 0.f;
            const float b = n < a.n ? a.bias[oc] : 0.f;
            const float inv = n < a.n ? a.out_inv_scale[oc] : 0.f;
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float y = acc[i][j][v] * cs + b;
                    if (EPI != EPI_CONVT) y = lrelu(y, a.slope);
                    ot[(rw + i * 16 + 4 * lg + v) * OP + col] = to_e4m3(y * inv);
                }
        }
        __syncthreads();
        uint8_t* out = static_cast<uint8_t*>(a.out);
        constexpr int CH = BN / 16;                 // 16-byte chunks per tile row
        const int n_valid = a.n - n0 < BN ? a.n - n0 : BN;
        for (int idx = tid; idx < BM * CH; idx += NT) {
            const int row = idx / CH, q = idx % CH;
            const int64_t r = m0 + row;
            if (16 * q >= n_valid || r >= a.m_rows) continue;
            const int64_t e = r / a.r_in;
            const int loc = (int)(r - e * a.r_in);
            if (loc < kGuard || loc >= a.r_in - kGuard) continue;
            const uint4 v = *reinterpret_cast<const uint4*>(ot + row * OP + 16 * q);
            if constexpr (EPI == EPI_CONVT) {
                const int n = n0 + 16 * q;
                const int tj = n / a.cout, o = n - tj * a.cout;
                const int64_t ro = e * a.r_out + kGuard + 2 * (loc - kGuard) + tj;
                *reinterpret_cast<uint4*>(out + ro * a.ld_out + o) = v;
            } else {
                *reinterpret_cast<uint4*>(out + r * a.ld_out + n0 + 16 * q) = v;
            }
        }
        if constexpr (EPI == EPI_POOL) {
            uint8_t* pout = static_cast<uint8_t*>(a.pool_out);
            for (int idx = tid; idx < (BM / 2) * CH; idx += NT) {
                const int pr = idx / CH, q = idx % CH;
                const int64_t r = m0 + 2 * pr;
                if (16 * q >= n_valid || r >= a.m_rows) continue;
                const int64_t e = r / a.r_in;
                const int loc = (int)(r - e * a.r_in);
                if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                const uint8_t* x0 = ot + (2 * pr) * OP + 16 * q;
                const uint8_t* x1 = x0 + OP;
                uint8_t y[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) y[u] = e4m3_to_f32(x0[u]) >= e4m3_to_f32(x1[u]) ? x0[u] : x1[u];
                const int64_t rp = e * a.r_pool + kGuard + (loc - kGuard) / 2;
                *reinterpret_cast<uint4*>(pout + rp * a.ld_pool + n0 + 16 * q) = *reinterpret_cast<const uint4*>(y);
            }
        }
    }
}

template <int WM, int WN, int TMW, int TNW, int TAPS, int EPI>
hipError_t run(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    hipLaunchKernelGGL((conv_mfma_fp8<WM, WN, TMW, TNW, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

struct Variant { int wm, wn, tmw, tnw; };
constexpr Variant kVariants[] = {
    {4, 1, 4, 2},   // 256 x 32
    {4, 1, 4, 4},   // 256 x 64
    {2, 2, 4, 4},   // 128 x 128
    {4, 2, 4, 4},   // 256 x 128 (512 threads)
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define PVF_FP8_CASE(V) \
    case V: return run<kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw, TAPS, EPI>(a, s);

template <int TAPS, int EPI>
hipError_t dispatch(int v, const ConvArgs& a, hipStream_t s)
{
    if constexpr (EPI == EPI_HEAD) {
        switch (v) {
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (v) {
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(2)
            PVF_FP8_CASE(3)
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int fp8_variant_count() { return kNumVariants; }

bool fp8_variant_ok(int v, int n, int taps, Epi epi)
{
    if (v < 0 || v >= kNumVariants) return false;
    (void)taps;
    const int bn = kVariants[v].wn * kVariants[v].tnw * 16;
    if (epi == EPI_HEAD) return (v == 0 || v == 1) && bn == n;
    return bn <= (n < 32 ? 32 : n);
}

// picks of variant sweeps over 1000 events (ties within noise go to the
// smaller tile)
int fp8_default_variant(int n, int taps, Epi epi)
{
    if (epi == EPI_HEAD) return n == 64 ? 1 : 0;
    if (n <= 32) return 0;
    if (epi == EPI_CONVT && taps == 1) return n >= 128 ? 3 : 0;
    if (epi == EPI_POOL) return 1;
    return n <= 64 ? 1 : 3;
}

std::string fp8_kernel_name(int v, int taps, Epi epi)
{
    const Variant& x = kVariants[v];
    return "conv_mfma_fp8<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) +
           ", " + std::to_string(x.tnw) + ", " + std::to_string(taps) + ", " + std::to_string((int)epi) + ">";
}

hipError_t launch_conv_fp8(const ConvArgs& a, int taps, Epi epi, int v, hipStream_t s)
{
    if (a.cin % KC != 0 || a.m_rows <= 0 || !fp8_variant_ok(v, a.n, taps, epi) || !a.col_scale) return hipErrorInvalidValue;
    if (epi != EPI_HEAD && !a.out_inv_scale) return hipErrorInvalidValue;
    if (epi == EPI_CONVT && a.cout % 16 != 0) return hipErrorInvalidValue;
    if (taps == 5) {
        switch (epi) {
        case EPI_STORE: return dispatch<5, EPI_STORE>(v, a, s);
        case EPI_POOL: return dispatch<5, EPI_POOL>(v, a, s);
        case EPI_HEAD: return dispatch<5, EPI_HEAD>(v, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (taps == 1 && epi == EPI_CONVT) return dispatch<1, EPI_CONVT>(v, a, s);
    return hipErrorInvalidValue;
}

}  // namespace pvf
