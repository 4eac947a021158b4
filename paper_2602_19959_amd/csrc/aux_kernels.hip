// Small kernels around the UNet: the first convolution (one input channel,
// five taps: too thin for the matrix cores) and the debug gather that copies
// an internal activation out in channels-first order.
#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int NT = 256;
constexpr int kMaxC0 = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// OCP e4m3 decoding
__device__ __forceinline__ float e4m3_to_f32(uint8_t b)
{
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e ? ldexpf(1.f + m / 8.f, e - 7) : ldexpf(m / 8.f, -6);
    return (b & 0x80) ? -v : v;
}

// enc0.c1: y[c] = LeakyReLU(b[c] + sum_j w[c][j] x[t + j - 2]).  Thread i
// computes the 16-byte chunk i % CPR of row i / CPR (CPR chunks per row), so
// the lanes of a wave store consecutive chunks: one contiguous 1 KB per wave
// store.  Guard rows are not written (they stay zero).
template <class T>
__global__ __launch_bounds__(NT) void first_conv(FirstConvArgs a)
{
    constexpr int CH = 16 / (int)sizeof(T);       // channels per 16-byte chunk
    __shared__ float w[kMaxC0 * kTaps];
    __shared__ float b[kMaxC0];
    for (int i = threadIdx.x; i < a.c0 * kTaps; i += NT) w[i] = a.w[i];
    for (int i = threadIdx.x; i < a.c0; i += NT) b[i] = a.b[i];
    __syncthreads();
    const int lg_cpr = 31 - __clz(a.c0 / CH);     // chunks per row: a power of two
    const unsigned i = blockIdx.x * NT + threadIdx.x;    // rows * chunks < 2^31 (checked)
    const unsigned r = i >> lg_cpr;
    if (r >= (unsigned)a.m_rows) return;
    const int c = (int)(i & ((1u << lg_cpr) - 1u)) * CH;   // first channel of the chunk
    const unsigned e = r / (unsigned)a.r0;
    const int loc = (int)(r - e * (unsigned)a.r0);
    if (loc < kGuard || loc >= a.r0 - kGuard) return;
    float x[kTaps];
#pragma unroll
    for (int j = 0; j < kTaps; ++j) x[j] = a.x0[(int64_t)r + j - kGuard];
    T y[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const float act = first_conv_at(w + (c + u) * kTaps, b[c + u], x, a.slope);
        if constexpr (sizeof(T) == 1) y[u] = e4m3_sat(act * a.out_inv_scale[c + u]);
        else y[u] = (T)act;
    }
    *reinterpret_cast<uint4*>(static_cast<T*>(a.out) + (int64_t)r * a.c0 + c) = *reinterpret_cast<const uint4*>(y);
}

template <class T>
__global__ __launch_bounds__(NT) void gather_channels_first(GatherArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= a.count) return;
    const int64_t per_event = (int64_t)a.C * a.L;
    const int64_t e = i / per_event;
    const int64_t rem = i - e * per_event;
    const int c = (int)(rem / a.L);
    const int t = (int)(rem - (int64_t)c * a.L);
    const T v = static_cast<const T*>(a.src)[(e * a.r + a.guard + t) * a.ld + a.ch_off + c];
    if constexpr (sizeof(T) == 1) a.dst[i] = e4m3_to_f32(v) * a.ch_scale[c];
    else a.dst[i] = (float)v;
}

template <class T>
__global__ __launch_bounds__(NT) void amax_channels(AmaxArgs a)
{
    // block: 256 threads = row lanes x channel lanes, 64 rows per row lane;
    // C <= 256: 256 / C row lanes of C channels; C > 256: one row lane and
    // C / 256 channels per thread
    const int cl = a.C < NT ? a.C : NT;
    const int per = NT / cl;
    const int c0 = threadIdx.x % cl, lr = threadIdx.x / cl;
    const int64_t r0 = ((int64_t)blockIdx.x * per + lr) * 64;
    for (int c = c0; c < a.C; c += NT) {
        float m = 0.f;
        for (int64_t r = r0; r < r0 + 64 && r < a.rows; ++r)
            m = fmaxf(m, fabsf((float)static_cast<const T*>(a.src)[r * a.ld + a.ch_off + c]));
        atomicMax(reinterpret_cast<unsigned int*>(a.out + c), __float_as_uint(m));
    }
}

}  // namespace

hipError_t launch_first_conv(const FirstConvArgs& a, int dtype, hipStream_t s)
{
    const int bytes = dtype == PVF_FP32 ? 4 : (dtype == PVF_FP8_E4M3 ? 1 : 2);
    const int cpr = a.c0 * bytes / 16;
    if (a.c0 > kMaxC0 || (a.c0 * bytes) % 16 != 0 || (cpr & (cpr - 1)) != 0) return hipErrorInvalidValue;
    const int64_t threads = (int64_t)a.m_rows * cpr;
    if (threads >= (1ll << 31)) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((threads + NT - 1) / NT);
    if (dtype == PVF_FP32) hipLaunchKernelGGL(first_conv<float>, dim3(blocks), dim3(NT), 0, s, a);
    else if (dtype == PVF_BF16) hipLaunchKernelGGL(first_conv<__bf16>, dim3(blocks), dim3(NT), 0, s, a);
    else if (dtype == PVF_FP16) hipLaunchKernelGGL(first_conv<_Float16>, dim3(blocks), dim3(NT), 0, s, a);
    else if (dtype == PVF_FP8_E4M3 && a.out_inv_scale) hipLaunchKernelGGL(first_conv<uint8_t>, dim3(blocks), dim3(NT), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.count + NT - 1) / NT);
    if (a.src_bytes == 4) hipLaunchKernelGGL(gather_channels_first<float>, dim3(blocks), dim3(NT), 0, s, a);
    else if (a.src_bytes == 1) {
        if (!a.ch_scale) return hipErrorInvalidValue;
        hipLaunchKernelGGL(gather_channels_first<uint8_t>, dim3(blocks), dim3(NT), 0, s, a);
    }
    else if (a.dtype == PVF_BF16) hipLaunchKernelGGL(gather_channels_first<__bf16>, dim3(blocks), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL(gather_channels_first<_Float16>, dim3(blocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_amax(const AmaxArgs& a, hipStream_t s)
{
    if (a.C <= 0 || a.rows <= 0 || (a.C <= NT ? NT % a.C : a.C % NT) != 0) return hipErrorInvalidValue;
    const int per = a.C < NT ? NT / a.C : 1;
    const unsigned blocks = (unsigned)((a.rows + (int64_t)per * 64 - 1) / ((int64_t)per * 64));
    if (a.elem_bytes == 4) hipLaunchKernelGGL(amax_channels<float>, dim3(blocks), dim3(NT), 0, s, a);
    else if (a.dtype == PVF_BF16) hipLaunchKernelGGL(amax_channels<__bf16>, dim3(blocks), dim3(NT), 0, s, a);
    else if (a.dtype == PVF_FP16) hipLaunchKernelGGL(amax_channels<_Float16>, dim3(blocks), dim3(NT), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace pvf
