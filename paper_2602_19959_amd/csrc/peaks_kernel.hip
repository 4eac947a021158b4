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
// The row is staged in LDS and the work is split in three passes so that
// every lane is busy in each of them (about one bin in three is a local
// maximum, so testing the window inside the bin loop would leave two thirds
// of the lanes idle during the window sums):
//   1. round k gives thread tid the four bins 4 (k * NT + tid) + s; it reads
//      them and their two outer neighbours at once and flags the strict local
//      maxima above p_min.  Ballots per wave, round and s count the flags;
//      after one barrier each candidate knows its rank in ascending bin order
//      (earlier rounds, earlier waves, lower lanes, lower s) and writes its
//      bin to a list in LDS;
//   2. the list is dealt out NT candidates per round; each lane sums its
//      candidate's window in double (ascending bin order) and tests S > s_min,
//      again with per-wave ballot counts;
//   3. each vertex takes its rank among the vertices (ascending bin order),
//      recomputes its window sums and writes its row of the output.
// Global loads of the row are issued four per thread before any LDS store,
// so a row costs one memory round trip.
#include "pvf_internal.h"

namespace pvf {
namespace {

constexpr int NT = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kQ = 4;            // bins per thread and round in the candidate pass
constexpr int kMaxRounds = 16;   // bins per event <= kQ * NT * kMaxRounds (kQ bits per round)
constexpr int kMaxList = 32;     // rounds of the candidate list (at most half the bins)

// S = sum of p over the window [t - hw, t + hw] clipped to the row, M = sum
// of p times the bin centre, both accumulated in double in ascending bin
// order.  HW > 0: the half-width is a compile-time constant and the window is
// read as 2 HW + 1 bins at once, clipped bins contributing an exact zero
// (which leaves both sums unchanged).  HW < 0: any half-width, a plain loop.
template <int HW>
__device__ __forceinline__ void window(const float* ps, int t, int L, const PeakArgs& a, double& S, double& M)
{
    S = 0.0;
    M = 0.0;
    if constexpr (HW > 0) {
        float pv[2 * HW + 1];
#pragma unroll
        for (int d = -HW; d <= HW; ++d) {
            const int j = t + d;
            pv[d + HW] = ps[j < 0 ? 0 : (j > L - 1 ? L - 1 : j)];
        }
#pragma unroll
        for (int d = -HW; d <= HW; ++d) {
            const int j = t + d;
            const double pj = (j >= 0 && j <= L - 1) ? (double)pv[d + HW] : 0.0;
            S += pj;
            M += pj * (a.z_min + a.bw * (j + 0.5));
        }
    } else {
        const int lo = t - a.hw < 0 ? 0 : t - a.hw;
        const int hi = t + a.hw > L - 1 ? L - 1 : t + a.hw;
        for (int j = lo; j <= hi; ++j) {
            const double pj = (double)ps[j];
            S += pj;
            M += pj * (a.z_min + a.bw * (j + 0.5));
        }
    }
}

// Sum of the per-wave counts of round k over all waves, and over the waves
// before this one.
template <int R>
__device__ __forceinline__ void round_counts(const int (*cnt)[R], int k, int wave, int& before, int& all)
{
    before = 0;
    all = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int c = cnt[w][k];
        all += c;
        before += w < wave ? c : 0;
    }
}

template <int HW>
__global__ __launch_bounds__(NT) void peak_finder(PeakArgs a)
{
    extern __shared__ __attribute__((aligned(16))) float ps[];   // [L] row, then the candidate list
    __shared__ int ccount[NT / 64][kMaxRounds];   // candidates per wave and round
    __shared__ int vcount[NT / 64][kMaxList];     // vertices per wave and list round

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e = blockIdx.x;
    const int L = a.L;
    uint16_t* cl = reinterpret_cast<uint16_t*>(ps + L);   // [L / 2] candidate bins, ascending
    const float* p = a.prob + (int64_t)e * L;
    if ((L & 3) == 0) {
        // indices past the row are clamped for the load (so all four are
        // issued unconditionally) and skipped for the store
        const int n4 = L / 4;
        const f32x4* p4 = reinterpret_cast<const f32x4*>(p);
        f32x4* s4 = reinterpret_cast<f32x4*>(ps);
        for (int b = 0; b < n4; b += 4 * NT) {
            f32x4 r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = p4[min(b + u * NT + tid, n4 - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (b + u * NT + tid < n4) s4[b + u * NT + tid] = r[u];
        }
    } else {
        for (int t = tid; t < L; t += NT) ps[t] = p[t];
    }
    const int flags = a.flags[e];
    const bool bypass = (flags & (PVF_EV_TOO_MANY_TRACKS | PVF_EV_BAD_INPUT)) != 0;
    const uint64_t below = (1ull << lane) - 1ull;
    __syncthreads();

    // 1. candidates: strict local maxima above p_min
    const int rounds = (L + kQ * NT - 1) / (kQ * NT);
    uint64_t mine = 0;                            // bit kQ k + s: bin kQ (k NT + tid) + s is a candidate
    for (int k = 0; k < rounds; ++k) {
        const int t0 = kQ * (k * NT + tid);
        float v[kQ + 2];                          // bins t0 - 1 .. t0 + kQ (clamped reads)
#pragma unroll
        for (int s = 0; s < kQ + 2; ++s) {
            const int j = t0 - 1 + s;
            v[s] = ps[j < 0 ? 0 : (j > L - 1 ? L - 1 : j)];
        }
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < kQ; ++s) {
            const int t = t0 + s;
            const float c = v[s + 1];
            const bool ok = !bypass && t >= 1 && t <= L - 2 && v[s] < c && c > v[s + 2] && (double)c > a.p_min;
            cnt += __popcll(__ballot(ok));
            mine |= (uint64_t)ok << (kQ * k + s);
        }
        if (lane == 0) ccount[wave][k] = cnt;
    }
    __syncthreads();
    int nc = 0;
    for (int k = 0; k < rounds; ++k) {
        int before, all;
        round_counts<kMaxRounds>(ccount, k, wave, before, all);
        const unsigned bits = (unsigned)(mine >> (kQ * k)) & ((1u << kQ) - 1u);
        int rank = nc + before;                   // candidates before this thread's first one
#pragma unroll
        for (int s = 0; s < kQ; ++s) rank += __popcll(__ballot((bits >> s) & 1u) & below);
#pragma unroll
        for (int s = 0; s < kQ; ++s)
            if ((bits >> s) & 1u) cl[rank++] = (uint16_t)(kQ * (k * NT + tid) + s);
        nc += all;
    }
    __syncthreads();

    // 2. window test, candidates dealt out in list order
    const int crounds = (nc + NT - 1) / NT;
    uint64_t vmine = 0;
    for (int r = 0; r < crounds; ++r) {
        const int i = r * NT + tid;
        bool ok = false;
        if (i < nc) {
            double S, M;
            window<HW>(ps, cl[i], L, a, S, M);
            ok = S > a.s_min;
        }
        const uint64_t m = __ballot(ok);
        if (lane == 0) vcount[wave][r] = __popcll(m);
        vmine |= (uint64_t)ok << r;
    }
    __syncthreads();

    // 3. output rows in ascending bin order
    double* zo = a.z + (int64_t)e * a.max_peaks;
    float* po = a.peak_prob + (int64_t)e * a.max_peaks;
    double* so = a.integral + (int64_t)e * a.max_peaks;
    int32_t* bo = a.bin ? a.bin + (int64_t)e * a.max_peaks : nullptr;
    int nv = 0;
    for (int r = 0; r < crounds; ++r) {
        int before, all;
        round_counts<kMaxList>(vcount, r, wave, before, all);
        const bool ok = (vmine >> r) & 1ull;
        const uint64_t m = __ballot(ok);
        const int slot = nv + before + __popcll(m & below);
        if (ok && slot < a.max_peaks) {
            const int t = cl[r * NT + tid];
            double S, M;
            window<HW>(ps, t, L, a, S, M);
            zo[slot] = M / S;
            po[slot] = ps[t];
            so[slot] = S;
            if (bo) bo[slot] = t;
        }
        nv += all;
    }
    if (tid == 0) {
        a.n_vertices[e] = nv < a.max_peaks ? nv : a.max_peaks;
        a.status[e] = flags | (nv > a.max_peaks ? PVF_EV_PEAKS_TRUNCATED : 0);
    }
}

}  // namespace

hipError_t launch_peaks(const PeakArgs& a, int n_events, hipStream_t s)
{
    // strict local maxima are never adjacent: at most L / 2 candidates
    if (a.L < 3 || a.L > kQ * NT * kMaxRounds || a.hw < 0) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * a.L + sizeof(uint16_t) * (a.L / 2 + 1);
    if (a.hw == 5)
        hipLaunchKernelGGL(peak_finder<5>, dim3(n_events), dim3(NT), lds, s, a);
    else
        hipLaunchKernelGGL(peak_finder<-1>, dim3(n_events), dim3(NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace pvf
