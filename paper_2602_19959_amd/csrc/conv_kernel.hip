// UNet convolutions as implicit GEMM on the CDNA4 matrix cores (FP32).
//
// The UNet of Section 2 (arXiv:2602.19959) is a stack of 1D convolutions.
// Each is a GEMM  D[m][n] = sum_k A[m][k] B[k][n]  with
//   m = (event, position)  rows of the channels-last activation,
//   n = output channel     (transposed conv: (tap, output channel)),
//   k = (tap, input channel).
// A is never materialised: a block stages the (BM + 4) x 16 halo tile of input
// rows once per 16-channel chunk in LDS and all five taps read it with a row
// shift.  LDS tiles are unpadded and XOR-swizzled per 16-byte chunk.  The packed weights are [N][taps][Cin], so one 16-byte LDS read gives
// a lane four consecutive k of its column.
//
// MFMA: v_mfma_f32_16x16x4_f32.  For one 16-wide k chunk, lane group g = lane/16
// supplies k = 4g+s to the s-th of four MFMAs; A and B use the same order, so
// the four MFMAs add up the whole chunk.  The k order of every output is fixed
// by the kernel alone (chunk, tap, s), never by the tile's position, so results
// are bitwise independent of the batch size and of where an event sits in it.
//
// Epilogues (fused, nothing re-read from HBM):
//   EPI_STORE  bias + LeakyReLU
//   EPI_POOL   bias + LeakyReLU, plus the width-2 max-pool of row pairs into
//              the next level's input
//   EPI_CONVT  stride-2 2-tap transposed conv: row t of the coarse level goes
//              to rows 2t and 2t+1 of the fine level, bias, no activation
//   EPI_HEAD   bias + LeakyReLU, then the 1x1 head over all channels and the
//              sigmoid, writing the per-bin probability
// Guard rows (the two zero rows before and after each event) are never written.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 16;         // input channels per LDS stage = 4 chunks of 16 B

// LDS rows are KC floats (4 chunks of 16 B) with no padding; chunk q of row r
// is stored at position q ^ swz(r), swz(r) = 2 * bit 3 of r.  Read-pattern
// probes on gfx950 show that bits 1..2 of r would make every fragment read
// conflict-free (with this one only the halo reads of tap 0 are), yet the
// dominant FP32 layer ran 6% slower with it in repeated A/B runs (same
// instruction stream apart from the address arithmetic; cause not pinned down).
__device__ __forceinline__ int swz(int r) { return (r >> 2) & 2; }
__device__ __forceinline__ int lds_at(int r, int q) { return (r * 4 + (q ^ swz(r))) * 4; }   // in floats

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

// Occupancy target handed to the register allocator: as many waves per SIMD
// as the block's LDS allows on one CU (160 KB), at most 4 (128 registers);
// none for the register-prefetch variants, which need the registers.
constexpr int occupancy_target(int lds_bytes, int waves_per_block)
{
    const int blocks = lds_bytes > 0 ? 163840 / lds_bytes : 8;
    const int w = blocks * waves_per_block / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// Epilogue shared by the FP32 kernels, straight from the accumulators.
// Output D layout of the 16x16 MFMA: lane holds rows 4*lg + v (v = 0..3) of
// column li.
template <int WM, int TMW, int TNW, int EPI>
__device__ __forceinline__ void f32_epilogue(const f32x4 (&acc)[TMW][TNW], const ConvArgs& a, int64_t m0, int n0,
                                             int tid)
{
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t rbase = m0 + (wave % WM) * TMW * 16;
    const int cbase = n0 + (wave / WM) * TNW * 16;
    float* out = static_cast<float*>(a.out);
    float* pout = static_cast<float*>(a.pool_out);

    if constexpr (EPI == EPI_HEAD) {
        // the block holds every channel of its rows (BN == n, one wave in N)
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < TNW; ++j) {
                    const int col = cbase + j * 16 + li;
                    s += lrelu(acc[i][j][v] + a.bias[col], a.slope) * a.head_w[col];
                }
                s += __shfl_xor(s, 8);
                s += __shfl_xor(s, 4);
                s += __shfl_xor(s, 2);
                s += __shfl_xor(s, 1);
                const int64_t r = rbase + i * 16 + 4 * lg + v;
                if (li == 0 && r < a.m_rows) {
                    const int64_t e = r / a.r_in;
                    const int loc = (int)(r - e * a.r_in);
                    if (loc >= kGuard && loc < a.r_in - kGuard) {
                        const float logit = s + a.head_b;
                        a.prob[e * a.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-logit));
                    }
                }
            }
        }
        return;
    }

#pragma unroll
    for (int j = 0; j < TNW; ++j) {
        const int col = cbase + j * 16 + li;
        if (col >= a.n) continue;
        if constexpr (EPI == EPI_CONVT) {
            const int tj = col / a.cout;           // which of the two output rows
            const int o = col - tj * a.cout;
            const float b = a.bias[o];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t r = rbase + i * 16 + 4 * lg + v;
                    if (r >= a.m_rows) continue;
                    const int64_t e = r / a.r_in;
                    const int loc = (int)(r - e * a.r_in);
                    if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                    const int64_t ro = e * a.r_out + kGuard + 2 * (loc - kGuard) + tj;
                    out[ro * a.ld_out + o] = acc[i][j][v] + b;
                }
        } else {
            const float b = a.bias[col];
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                float y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) y[v] = lrelu(acc[i][j][v] + b, a.slope);
                const int64_t r0 = rbase + i * 16 + 4 * lg;   // multiple of 4
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t r = r0 + v;
                    if (r >= a.m_rows) continue;
                    const int64_t e = r / a.r_in;
                    const int loc = (int)(r - e * a.r_in);
                    if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                    out[r * a.ld_out + col] = y[v];
                }
                if constexpr (EPI == EPI_POOL) {
                    // rows per event and the guard are even, so an even row is
                    // the first of a pooling pair
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const int64_t r = r0 + 2 * p;
                        if (r >= a.m_rows) continue;
                        const int64_t e = r / a.r_in;
                        const int loc = (int)(r - e * a.r_in);
                        if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                        const int64_t rp = e * a.r_pool + kGuard + (loc - kGuard) / 2;
                        pout[rp * a.ld_pool + col] = fmaxf(y[2 * p], y[2 * p + 1]);
                    }
                }
            }
        }
    }
}

// (register estimate: 4 per accumulator tile and per fragment, about 56
// others, 40 more for the 4 x 4-tile waves; the target never asks for fewer)
template <int TMW, int TNW> struct F32Regs {
    static constexpr int v = 4 * TMW * TNW + 4 * (TMW + TNW) + 56 + (TMW * TNW >= 16 ? 40 : 0);
};
template <int WM, int WN, int TMW, int TNW, int PF, int TAPS>
struct F32Occ {
    static constexpr int lds = occupancy_target(4 * KC * (WM * TMW * 16 + TAPS - 1 + WN * TNW * 16 * TAPS), WM * WN);
    static constexpr int regs = 512 / F32Regs<TMW, TNW>::v;
    static constexpr int v = PF ? 1 : (lds < regs ? lds : regs);
};
template <int WM, int WN, int TMW, int TNW, int PF, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(F32Occ<WM, WN, TMW, TNW, PF, TAPS>::v)))
void conv_mfma_f32(ConvArgs a)
{
    constexpr int NT = WM * WN * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int XROWS = BM + TAPS - 1;
    constexpr int XV = XROWS * (KC / 4);          // float4 per stage of the halo tile
    constexpr int WV = BN * TAPS * (KC / 4);      // float4 per stage of the weight tile
    constexpr int XPT = (XV + NT - 1) / NT;
    constexpr int WPT = (WV + NT - 1) / NT;

    __shared__ float xs[XROWS * KC];
    __shared__ float ws[BN * TAPS * KC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int li = lane & 15;
    const int lg = lane >> 4;

    // XCD-aware tile order: block b runs on XCD b % 8; every N tile of one M
    // tile goes to the same XCD back to back, so the halo rows (and the
    // weights) are served from that XCD's L2 instead of HBM.
    const int n_tiles = (a.n + BN - 1) / BN;
    const int m_tiles = (int)((a.m_rows + BM - 1) / BM);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = (slot / n_tiles) * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BM;
    const int n0 = (slot % n_tiles) * BN;
    const int kw = TAPS * a.cin;
    const float* in = static_cast<const float*>(a.in);
    const float* wt = static_cast<const float*>(a.w);

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // PF = 1: software pipeline, the next chunk's tiles are fetched into
    // registers while the current chunk's MFMAs run from LDS.  PF = 0: fetch,
    // stage and compute in turn (fewer registers, more blocks per CU).
    f32x4 xr[XPT], wr[WPT];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int idx = tid + u * NT;
            xr[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (idx < XV) {
                const int row = idx / (KC / 4), q = idx % (KC / 4);
                const int64_t g = m0 - RAD + row;
                if (g >= 0 && g < a.m_rows)
                    xr[u] = *reinterpret_cast<const f32x4*>(in + g * a.ld_in + c0 + 4 * q);
            }
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int idx = tid + u * NT;
            wr[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (idx < WV) {
                const int q = idx % (KC / 4);
                const int rest = idx / (KC / 4);
                const int tap = rest % TAPS, nn = rest / TAPS;
                if (n0 + nn < a.n)
                    wr[u] = *reinterpret_cast<const f32x4*>(wt + (int64_t)(n0 + nn) * kw + tap * a.cin + c0 + 4 * q);
            }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int idx = tid + u * NT;
            if (idx < XV) {
                const int row = idx / (KC / 4), q = idx % (KC / 4);
                *reinterpret_cast<f32x4*>(xs + lds_at(row, q)) = xr[u];
            }
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int idx = tid + u * NT;
            if (idx < WV) {
                const int q = idx % (KC / 4);
                const int rest = idx / (KC / 4);
                *reinterpret_cast<f32x4*>(ws + lds_at(rest, q)) = wr[u];
            }
        }
    };

    fetch(0);
    stage();
    __syncthreads();
    for (int c0 = 0; c0 < a.cin; c0 += KC) {
        const bool more = c0 + KC < a.cin;
        if (PF && more) fetch(c0 + KC);
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            f32x4 av[TMW], bv[TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[i] = *reinterpret_cast<const f32x4*>(xs + lds_at(wm * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[j] = *reinterpret_cast<const f32x4*>(ws + lds_at((wn * TNW * 16 + j * 16 + li) * TAPS + tap, lg));
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            if (!PF) fetch(c0 + KC);
            stage();
            __syncthreads();
        }
    }

    f32_epilogue<WM, TMW, TNW, EPI>(acc, a, m0, n0, tid);
}


// PF = 2, double-buffered: the next 16-channel stage streams from global
// memory straight into the second LDS buffer (global_load_lds_dwordx4: lane L
// fills 16-byte slot L of a 1 KB block = 16 rows of 64 bytes) while the
// current stage is on the matrix cores, and the fragments of the next tap are
// read during the current tap's MFMAs.  Rows beyond the batch and columns
// beyond n are clamped to valid addresses: they only feed outputs the
// epilogue discards.  Same k order (16-channel chunk, tap, MFMA step).
template <int WM, int WN, int TMW, int TNW, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) void conv_mfma_f32_db(ConvArgs a)
{
    constexpr int NW = WM * WN;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int ROWB = KC * 4;                     // 64 bytes per LDS row
    constexpr int XR = (BM + TAPS - 1 + 15) / 16 * 16;
    constexpr int WRW = BN * TAPS;
    static_assert(WRW % 16 == 0, "weight rows fill whole 1 KB loads");
    constexpr int XI = XR / 16, WI = WRW / 16;
    constexpr int STAGE = (XR + WRW) * KC;           // floats
    __shared__ __attribute__((aligned(16))) float smem[2 * STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int li = lane & 15;
    const int lg = lane >> 4;
    const int n_tiles = (a.n + BN - 1) / BN;
    const int m_tiles = (int)((a.m_rows + BM - 1) / BM);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = (slot / n_tiles) * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BM;
    const int n0 = (slot % n_tiles) * BN;
    const int kw = TAPS * a.cin;
    const float* in = static_cast<const float*>(a.in);
    const float* wt = static_cast<const float*>(a.w);

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int lrow = lane >> 2, lpos = lane & 3;
    auto issue = [&](int buf, int c0) {
        float* base = smem + buf * STAGE;
        for (int j = wave; j < XI + WI; j += NW) {
            const bool xj = j < XI;
            const int row = 16 * (xj ? j : j - XI) + lrow;
            const int c = lpos ^ swz(row);
            const float* g;
            if (xj) {
                int64_t gr = m0 - RAD + row;
                gr = gr < 0 ? 0 : (gr >= a.m_rows ? a.m_rows - 1 : gr);
                g = in + gr * a.ld_in + c0 + 4 * c;
            } else {
                const int nn = row / TAPS, tap = row - nn * TAPS;
                const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
                g = wt + (int64_t)n * kw + tap * a.cin + c0 + 4 * c;
            }
            float* dst = base + (xj ? 16 * j * KC : XR * KC + 16 * (j - XI) * KC);
            __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        }
    };
    (void)ROWB;

    const int nk = a.cin / KC;
    issue(0, 0);
    for (int k = 0; k < nk; ++k) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (k + 1 < nk) issue((k + 1) & 1, (k + 1) * KC);
        const float* xs = smem + (k & 1) * STAGE;
        const float* ws = xs + XR * KC;
        f32x4 av[2][TMW], bv[2][TNW];
        auto frag = [&](int tap, int f) {
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[f][i] = *reinterpret_cast<const f32x4*>(xs + lds_at(wm * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[f][j] = *reinterpret_cast<const f32x4*>(ws + lds_at((wn * TNW * 16 + j * 16 + li) * TAPS + tap, lg));
        };
        frag(0, 0);
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            if (tap + 1 < TAPS) frag(tap + 1, (tap + 1) & 1);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[tap & 1][i][s], bv[tap & 1][j][s], acc[i][j],
                                                                          0, 0, 0);
        }
    }
    f32_epilogue<WM, TMW, TNW, EPI>(acc, a, m0, n0, tid);
}

template <int WM, int WN, int TMW, int TNW, int PF, int TAPS, int EPI>
hipError_t run(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    if constexpr (PF == 2)
        hipLaunchKernelGGL((conv_mfma_f32_db<WM, WN, TMW, TNW, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    else
        hipLaunchKernelGGL((conv_mfma_f32<WM, WN, TMW, TNW, PF, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

// Tile-shape variants.  Every variant accumulates each output's k terms in
// the same order (16-channel chunk, tap, MFMA step), so all of them give
// bitwise-identical results; they differ only in speed.
struct Variant { int wm, wn, tmw, tnw, pf; };
constexpr Variant kVariants[] = {
    {4, 1, 4, 2, 0}, {4, 1, 4, 2, 1}, {2, 1, 4, 2, 0},
    {4, 1, 4, 4, 0}, {4, 1, 4, 4, 1}, {4, 1, 2, 4, 0},
    {2, 2, 4, 4, 0}, {2, 2, 4, 4, 1}, {4, 2, 4, 4, 0}, {4, 2, 4, 4, 1},
    {2, 4, 4, 4, 0},
    {4, 1, 4, 2, 2}, {4, 1, 4, 4, 2}, {4, 2, 4, 4, 2}, {2, 1, 4, 2, 2},   // 11-14: double-buffered
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define PVF_VARIANT_CASE(V, TAPS, EPI)                                                                  \
    case V:                                                                                             \
        return run<kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw, kVariants[V].pf, \
                   TAPS, EPI>(a, s);

template <int TAPS, int EPI>
hipError_t dispatch(int v, const ConvArgs& a, hipStream_t s)
{
    if constexpr (EPI == EPI_HEAD) {
        switch (v) {
            PVF_VARIANT_CASE(0, TAPS, EPI)
            PVF_VARIANT_CASE(1, TAPS, EPI)
            PVF_VARIANT_CASE(2, TAPS, EPI)
            PVF_VARIANT_CASE(3, TAPS, EPI)
            PVF_VARIANT_CASE(5, TAPS, EPI)
            PVF_VARIANT_CASE(11, TAPS, EPI)
            PVF_VARIANT_CASE(12, TAPS, EPI)
            PVF_VARIANT_CASE(14, TAPS, EPI)
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (v) {
            PVF_VARIANT_CASE(0, TAPS, EPI)
            PVF_VARIANT_CASE(1, TAPS, EPI)
            PVF_VARIANT_CASE(2, TAPS, EPI)
            PVF_VARIANT_CASE(3, TAPS, EPI)
            PVF_VARIANT_CASE(4, TAPS, EPI)
            PVF_VARIANT_CASE(5, TAPS, EPI)
            PVF_VARIANT_CASE(6, TAPS, EPI)
            PVF_VARIANT_CASE(7, TAPS, EPI)
            PVF_VARIANT_CASE(8, TAPS, EPI)
            PVF_VARIANT_CASE(9, TAPS, EPI)
            PVF_VARIANT_CASE(10, TAPS, EPI)
            PVF_VARIANT_CASE(11, TAPS, EPI)
            PVF_VARIANT_CASE(12, TAPS, EPI)
            PVF_VARIANT_CASE(13, TAPS, EPI)
            PVF_VARIANT_CASE(14, TAPS, EPI)
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int f32_variant_count() { return kNumVariants; }

bool f32_variant_ok(int v, int n, int taps, Epi epi)
{
    if (v < 0 || v >= kNumVariants) return false;
    const Variant& x = kVariants[v];
    const int bn = x.wn * x.tnw * 16;
    // the head reduces over all channels inside one wave's columns
    if (epi == EPI_HEAD) return (v <= 3 || v == 5 || v == 11 || v == 12 || v == 14) && bn == n && x.wn == 1;
    (void)taps;
    return bn <= (n < 32 ? 32 : n);
}

// Defaults from a sweep on MI355X at 1000 events: the 256 x 32 tile with the
// fewest registers (most blocks per CU) wins every 5-tap layer; the
// transposed convs prefer wider N tiles.
int f32_default_variant(int n, int cin, int taps, Epi epi)
{
    if (epi == EPI_CONVT && taps == 1) return n >= 64 ? 5 : 0;
    if (epi == EPI_HEAD) return n == 64 ? 3 : 0;
    if (epi == EPI_STORE && cin >= 128 && n >= 128) return 3;
    if (n == 64 && cin <= 32) return 5;
    return 0;
}

std::string f32_kernel_name(int v, int taps, Epi epi)
{
    const Variant& x = kVariants[v];
    if (x.pf == 2)
        return "conv_mfma_f32_db<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " +
               std::to_string(x.tmw) + ", " + std::to_string(x.tnw) + ", " + std::to_string(taps) + ", " +
               std::to_string((int)epi) + ">";
    return "conv_mfma_f32<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) +
           ", " + std::to_string(x.tnw) + ", " + std::to_string(x.pf) + ", " + std::to_string(taps) + ", " +
           std::to_string((int)epi) + ">";
}

hipError_t launch_conv_f32(const ConvArgs& a, int taps, Epi epi, int variant, hipStream_t s)
{
    if (a.cin % KC != 0 || a.m_rows <= 0 || !f32_variant_ok(variant, a.n, taps, epi)) return hipErrorInvalidValue;
    if (taps == 5) {
        switch (epi) {
        case EPI_STORE: return dispatch<5, EPI_STORE>(variant, a, s);
        case EPI_POOL: return dispatch<5, EPI_POOL>(variant, a, s);
        case EPI_HEAD: return dispatch<5, EPI_HEAD>(variant, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (taps == 1 && epi == EPI_CONVT) return dispatch<1, EPI_CONVT>(variant, a, s);
    return hipErrorInvalidValue;
}

}  // namespace pvf
