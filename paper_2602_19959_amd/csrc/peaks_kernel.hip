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
// The row is staged in LDS.  Round k tests bins k * NT + tid (consecutive
// lanes read consecutive bins, so the LDS reads are conflict-free); a ballot
// per wave and round counts the vertices, and after one barrier every thread
// knows how many vertices precede its own in ascending bin order (earlier
// rounds, then earlier waves, then lower lanes of its round), so they are
// written in that order.
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

constexpr int kMaxRounds = 64;   // bins per event <= NT * kMaxRounds (one bit per round)

__global__ __launch_bounds__(NT) void peak_finder(PeakArgs a)
{
    extern __shared__ float ps[];                 // [L]
    __shared__ int wcount[NT / 64][kMaxRounds];   // vertices per wave and round

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e = blockIdx.x;
    const int L = a.L;
    const float* p = a.prob + (int64_t)e * L;
    for (int t = tid; t < L; t += NT) ps[t] = p[t];
    const int flags = a.flags[e];
    const bool bypass = (flags & (PVF_EV_TOO_MANY_TRACKS | PVF_EV_BAD_INPUT)) != 0;
    __syncthreads();

    const int rounds = (L + NT - 1) / NT;
    uint64_t mine = 0;                            // bit k: bin k * NT + tid is a vertex
    for (int k = 0; k < rounds; ++k) {
        const int t = k * NT + tid;
        const bool ok = !bypass && t >= 1 && t <= L - 2 && test_bin(ps, t, L, a).ok;
        const uint64_t m = __ballot(ok);
        if (lane == 0) wcount[wave][k] = __popcll(m);
        mine |= (uint64_t)ok << k;
    }
    __syncthreads();

    double* zo = a.z + (int64_t)e * a.max_peaks;
    float* po = a.peak_prob + (int64_t)e * a.max_peaks;
    double* so = a.integral + (int64_t)e * a.max_peaks;
    int32_t* bo = a.bin ? a.bin + (int64_t)e * a.max_peaks : nullptr;
    const uint64_t below = (1ull << lane) - 1ull;
    int base = 0;                                 // vertices in earlier rounds
    for (int k = 0; k < rounds; ++k) {
        int before = 0, in_round = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            const int c = wcount[w][k];
            in_round += c;
            before += w < wave ? c : 0;
        }
        const bool ok = (mine >> k) & 1ull;
        const uint64_t m = __ballot(ok);
        const int slot = base + before + __popcll(m & below);
        if (ok && slot < a.max_peaks) {
            const int t = k * NT + tid;
            const Vertex v = test_bin(ps, t, L, a);
            zo[slot] = v.M / v.S;
            po[slot] = ps[t];
            so[slot] = v.S;
            if (bo) bo[slot] = t;
        }
        base += in_round;
    }
    if (tid == 0) {
        a.n_vertices[e] = base < a.max_peaks ? base : a.max_peaks;
        a.status[e] = flags | (base > a.max_peaks ? PVF_EV_PEAKS_TRUNCATED : 0);
    }
}

}  // namespace

hipError_t launch_peaks(const PeakArgs& a, int n_events, hipStream_t s)
{
    if (a.L < 3 || a.L > NT * kMaxRounds) return hipErrorInvalidValue;
    hipLaunchKernelGGL(peak_finder, dim3(n_events), dim3(NT), sizeof(float) * a.L, s, a);
    return hipGetLastError();
}

}  // namespace pvf
