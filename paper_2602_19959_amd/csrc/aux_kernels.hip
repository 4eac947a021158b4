// Small kernels around the UNet: the first convolution (one input channel,
// five taps: too thin for the matrix cores) and the debug gather that copies
// an internal activation out in channels-first order.
#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int NT = 256;
constexpr int kMaxC0 = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// enc0.c1: y[c] = LeakyReLU(b[c] + sum_j w[c][j] x[t + j - 2]), one row per
// thread, all C0 channels written as one contiguous run of float4 stores.
template <class T>
__global__ __launch_bounds__(NT) void first_conv(FirstConvArgs a)
{
    __shared__ float w[kMaxC0 * kTaps];
    __shared__ float b[kMaxC0];
    for (int i = threadIdx.x; i < a.c0 * kTaps; i += NT) w[i] = a.w[i];
    for (int i = threadIdx.x; i < a.c0; i += NT) b[i] = a.b[i];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (r >= a.m_rows) return;
    const int64_t e = r / a.r0;
    const int loc = (int)(r - e * a.r0);
    if (loc < kGuard || loc >= a.r0 - kGuard) return;
    float x[kTaps];
#pragma unroll
    for (int j = 0; j < kTaps; ++j) x[j] = a.x0[r + j - kGuard];
    T* o = static_cast<T*>(a.out) + r * a.c0;
    for (int c = 0; c < a.c0; c += 8) {
        T y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float s = b[c + u];
#pragma unroll
            for (int j = 0; j < kTaps; ++j) s = fmaf(w[(c + u) * kTaps + j], x[j], s);
            y[u] = (T)(s >= 0.f ? s : a.slope * s);
        }
        // 8 channels = 32 B (float) or 16 B (16-bit): whole-vector stores
        if constexpr (sizeof(T) == 4) {
            reinterpret_cast<f32x4*>(o + c)[0] = *reinterpret_cast<const f32x4*>(y);
            reinterpret_cast<f32x4*>(o + c)[1] = *reinterpret_cast<const f32x4*>(y + 4);
        } else {
            *reinterpret_cast<uint4*>(o + c) = *reinterpret_cast<const uint4*>(y);
        }
    }
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
    a.dst[i] = (float)static_cast<const T*>(a.src)[(e * a.r + a.guard + t) * a.ld + a.ch_off + c];
}

}  // namespace

hipError_t launch_first_conv(const FirstConvArgs& a, int dtype, hipStream_t s)
{
    if (a.c0 > kMaxC0 || a.c0 % 8 != 0) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((a.m_rows + NT - 1) / NT);
    if (dtype == PVF_FP32) hipLaunchKernelGGL(first_conv<float>, dim3(blocks), dim3(NT), 0, s, a);
    else if (dtype == PVF_BF16) hipLaunchKernelGGL(first_conv<__bf16>, dim3(blocks), dim3(NT), 0, s, a);
    else if (dtype == PVF_FP16) hipLaunchKernelGGL(first_conv<_Float16>, dim3(blocks), dim3(NT), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.count + NT - 1) / NT);
    if (a.src_bytes == 4) hipLaunchKernelGGL(gather_channels_first<float>, dim3(blocks), dim3(NT), 0, s, a);
    else if (a.dtype == PVF_BF16) hipLaunchKernelGGL(gather_channels_first<__bf16>, dim3(blocks), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL(gather_channels_first<_Float16>, dim3(blocks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace pvf
