// Precision dispatch for the UNet convolution launches.
#include "pvf_internal.h"

namespace pvf {

hipError_t launch_conv(int dtype, const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s)
{
    if (dtype == PVF_FP32) return launch_conv_f32(a, taps, epi, variant, s);
    if (dtype == PVF_FP8_E4M3) return launch_conv_fp8(a, taps, epi, variant, s);
    return launch_conv_lp(dtype, a, taps, epi, variant, s);
}

hipError_t launch_conv_first(int dtype, const ConvArgs& a, int variant, hipStream_t s)
{
    if (!a.first_x0 || !a.first_w || !a.first_b) return hipErrorInvalidValue;
    if (dtype == PVF_FP32) return launch_conv_f32_first(a, variant, s);
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return launch_conv_lp_first(dtype, a, variant, s);
    if (dtype == PVF_FP8_E4M3) return launch_conv_fp8_first(a, variant, s);
    return hipErrorInvalidValue;
}

bool conv_first_ok(int dtype, int variant)
{
    if (dtype == PVF_FP32) return f32_first_ok(variant);
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return lp_first_ok(variant);
    if (dtype == PVF_FP8_E4M3) return fp8_first_ok(variant);
    return false;
}

std::string conv_first_kernel_name(int dtype, int variant)
{
    if (dtype == PVF_FP32) return f32_first_kernel_name(variant);
    if (dtype == PVF_FP8_E4M3) return fp8_first_kernel_name(variant);
    return lp_first_kernel_name(dtype, variant);
}

int conv_variant_count(int dtype)
{
    return dtype == PVF_FP32 ? f32_variant_count() : dtype == PVF_FP8_E4M3 ? fp8_variant_count() : lp_variant_count();
}

bool conv_variant_ok(int dtype, int variant, int n, int cin, int taps, Epi epi)
{
    if (dtype == PVF_FP32) return f32_variant_ok(variant, n, taps, epi);
    if (dtype == PVF_FP8_E4M3) return fp8_variant_ok(variant, n, cin, taps, epi);
    return lp_variant_ok(variant, n, cin, taps, epi);
}

int conv_default_variant(int dtype, int n, int cin, int taps, Epi epi)
{
    if (dtype == PVF_FP32) return f32_default_variant(n, cin, taps, epi);
    if (dtype == PVF_FP8_E4M3) return fp8_default_variant(n, cin, taps, epi);
    return lp_default_variant(n, cin, taps, epi);
}

int conv_default_up_variant(int dtype, int n, int cin)
{
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return lp_default_up_variant(n, cin);
    if (dtype == PVF_FP8_E4M3) return fp8_default_up_variant(n, cin);
    return -1;
}

int conv_default_dec0_variant(int dtype)
{
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return 32;   // the autotuner's pick at 1000 events
    return dtype == PVF_FP8_E4M3 ? 20 : -1;
}

bool conv_dec0_ok(int dtype, int variant)
{
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return lp_dec0_ok(variant);
    return dtype == PVF_FP8_E4M3 && fp8_dec0_ok(variant);
}

hipError_t launch_conv_dec0(int dtype, const ConvArgs& c1, const ConvArgs& c2, int variant, hipStream_t s)
{
    if (dtype == PVF_BF16 || dtype == PVF_FP16) return launch_conv_lp_dec0(dtype, c1, c2, variant, s);
    if (dtype == PVF_FP8_E4M3) return launch_conv_fp8_dec0(c1, c2, variant, s);
    return hipErrorInvalidValue;
}

std::string conv_kernel_name(int dtype, int variant, int cin, int taps, Epi epi)
{
    if (dtype == PVF_FP32) return f32_kernel_name(variant, taps, epi);
    if (dtype == PVF_FP8_E4M3) return fp8_kernel_name(variant, cin, taps, epi);
    return lp_kernel_name(dtype, variant, taps, epi);
}

}  // namespace pvf
