// Peak finding on the per-bin probability, one workgroup per event.
//
// Section 2 of arXiv:2602.19959: the last stage applies local-maximum
// detection with thresholds to the CNN output; Section 3: it reads the CNN
// output in place.  A vertex is a strict local maximum p[t-1] < p[t] > p[t+1]
// (1 <= t <= L-2) with p[t] > p_min whose window sum S over [t-hw, t+hw]
// (clipped to the histogram) exceeds s_min; its z is the p-weighted mean of
// the window's bin centres.  Window sums and centroids are accumulated in
// double, in ascending bin order.
//
// The row is staged in LDS; thread k owns a contiguous run of bins, counts
// its vertices, a block-wide exclusive scan gives each thread its first
// output slot, and the vertices are written in ascending bin order.
#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int NT = 256;

struct Vertex {
    bool ok;
    double S, M;
};

__device__ __forceinline__ Vertex test_bin(const float* ps, int t, int L, const PeakArgs& a)
{
    Vertex v{false, 0.0, 0.0};
    const float c = ps[t];
    if (!(ps[t - 1] < c && c > ps[t + 1])) return v;
    if (!((double)c > a.p_min)) return v;
    const int lo = t - a.hw < 0 ? 0 : t - a.hw;
    const int hi = t + a.hw > L - 1 ? L - 1 : t + a.hw;
    double S = 0.0, M = 0.0;
    for (int j = lo; j <= hi; ++j) {
        const double pj = (double)ps[j];
        S += pj;
        M += pj * (a.z_min + a.bw * (j + 0.5));
    }
    v.ok = S > a.s_min;
    v.S = S;
    v.M = M;
    return v;
}

__global__ __launch_bounds__(NT) void peak_finder(PeakArgs a)
{
    extern __shared__ float ps[];                 // [L]
    __shared__ int scan[NT];

    const int tid = threadIdx.x;
    const int e = blockIdx.x;
    const int L = a.L;
    const float* p = a.prob + (int64_t)e * L;
    for (int t = tid; t < L; t += NT) ps[t] = p[t];
    const int flags = a.flags[e];
    const bool bypass = (flags & (PVF_EV_TOO_MANY_TRACKS | PVF_EV_BAD_INPUT)) != 0;
    __syncthreads();

    const int chunk = (L + NT - 1) / NT;
    const int t0 = tid * chunk < 1 ? 1 : tid * chunk;
    const int t1 = (tid + 1) * chunk > L - 1 ? L - 1 : (tid + 1) * chunk;
    int n = 0;
    if (!bypass)
        for (int t = t0; t < t1; ++t) n += test_bin(ps, t, L, a).ok ? 1 : 0;

    // inclusive Hillis-Steele scan of the per-thread counts
    scan[tid] = n;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int v = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    const int total = scan[NT - 1];
    int k = scan[tid] - n;

    double* zo = a.z + (int64_t)e * a.max_peaks;
    float* po = a.peak_prob + (int64_t)e * a.max_peaks;
    double* so = a.integral + (int64_t)e * a.max_peaks;
    int32_t* bo = a.bin ? a.bin + (int64_t)e * a.max_peaks : nullptr;
    if (!bypass && n > 0) {
        for (int t = t0; t < t1 && k < a.max_peaks; ++t) {
            const Vertex v = test_bin(ps, t, L, a);
            if (!v.ok) continue;
            zo[k] = v.M / v.S;
            po[k] = ps[t];
            so[k] = v.S;
            if (bo) bo[k] = t;
            ++k;
        }
    }
    if (tid == 0) {
        a.n_vertices[e] = total < a.max_peaks ? total : a.max_peaks;
        a.status[e] = flags | (total > a.max_peaks ? PVF_EV_PEAKS_TRUNCATED : 0);
    }
}

}  // namespace

hipError_t launch_peaks(const PeakArgs& a, int n_events, hipStream_t s)
{
    hipLaunchKernelGGL(peak_finder, dim3(n_events), dim3(NT), sizeof(float) * a.L, s, a);
    return hipGetLastError();
}

}  // namespace pvf
