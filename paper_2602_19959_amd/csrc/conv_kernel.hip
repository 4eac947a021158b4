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
//
// conv_mfma_f32_first runs enc0.c2 with the first convolution (one input
// channel, five taps) computed in its halo staging from the histogram rows,
// so that 32-channel tensor never goes through HBM.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 16;         // input channels per LDS stage = 4 chunks of 16 B

// LDS rows are KC floats (4 chunks of 16 B) with no padding; chunk q of row r
// is stored at position q ^ swz(r), swz(r) = 2 * bit 3 of r.  Read-pattern
// probes on gfx950 show that bits 1..2 of r would make every fragment read
// conflict-free (with this one only the halo reads of tap 0 are), yet the
// dominant FP32 layer ran slower with it in repeated A/B runs: 6% with the
// weight rows in (column, tap) order, under 1% with the tap-major rows used
// now (cause not pinned down).
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

// Epilogue shared by the FP32 kernels, straight from the accumulators.  The
// kernels issue the MFMA as D^T = W X^T (weight fragment in the A slot), so
// lane (li, lg) of a 16 x 16 tile holds channels 4 lg + v (v = 0..3) of tile
// row li: four consecutive outputs of one position, one 16-byte store.
template <int WM, int TMW, int TNW, int EPI>
__device__ __forceinline__ void f32_epilogue(const f32x4 (&acc)[TMW][TNW], const ConvArgs& a, int64_t m0, int n0,
                                             int tid)
{
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rw = (wave % WM) * TMW * 16;
    const int cbase = n0 + (wave / WM) * TNW * 16 + 4 * lg;   // this lane's first channel of tile j = 0
    const RowMap rows(m0, a.r_in);
    float* out = static_cast<float*>(a.out);
    float* pout = static_cast<float*>(a.pool_out);

    if constexpr (EPI == EPI_HEAD) {
        // the block holds every channel of its rows (BN == n, one wave in N)
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < TNW; ++j) {
                const int c = cbase + j * 16;
#pragma unroll
                for (int v = 0; v < 4; ++v) s += lrelu(acc[i][j][v] + a.bias[c + v], a.slope) * a.head_w[c + v];
            }
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            const int t = rw + i * 16 + li;
            if (lg == 0 && m0 + t < a.m_rows) {
                int64_t e;
                int loc;
                rows.at(t, e, loc);
                if (loc >= kGuard && loc < a.r_in - kGuard)
                    a.prob[e * a.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(s + a.head_b)));
            }
        }
        return;
    }

#pragma unroll
    for (int i = 0; i < TMW; ++i) {
        const int t = rw + i * 16 + li;
        int64_t e;
        int loc;
        rows.at(t, e, loc);
        const bool ok = m0 + t < a.m_rows && loc >= kGuard && loc < a.r_in - kGuard;
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int c = cbase + j * 16;
            const bool col_ok = c < a.n;            // n % 4 == 0: a lane's four channels are all in or all out
            const int cc = col_ok ? c : 0;
            if constexpr (EPI == EPI_CONVT) {
                const int tj = cc / a.cout;          // which of the two output rows
                const int o = cc - tj * a.cout;
                f32x4 y;
#pragma unroll
                for (int v = 0; v < 4; ++v) y[v] = acc[i][j][v] + a.bias[o + v];
                if (ok && col_ok) {
                    const int64_t ro = e * a.r_out + kGuard + 2 * (loc - kGuard) + tj;
                    *reinterpret_cast<f32x4*>(out + ro * a.ld_out + o) = y;
                }
            } else {
                f32x4 y;
#pragma unroll
                for (int v = 0; v < 4; ++v) y[v] = lrelu(acc[i][j][v] + a.bias[cc + v], a.slope);
                if (ok && col_ok) *reinterpret_cast<f32x4*>(out + (m0 + t) * a.ld_out + c) = y;
                if constexpr (EPI == EPI_POOL) {
                    // rows per event and the guard are even, so an even row is
                    // the first of a pooling pair; its partner is lane li ^ 1
                    f32x4 p;
#pragma unroll
                    for (int v = 0; v < 4; ++v) p[v] = fmaxf(y[v], __shfl_xor(y[v], 1));
                    if (ok && col_ok && (li & 1) == 0) {
                        const int64_t rp = e * a.r_pool + kGuard + (loc - kGuard) / 2;
                        *reinterpret_cast<f32x4*>(pout + rp * a.ld_pool + c) = p;
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
// FC: enc0.c2 with the first convolution fused into the staging: each halo
// chunk is computed from five histogram rows (first_conv_at, the operation
// order of the standalone kernel, so the bits match) instead of read back;
// guard rows are zero, as in the stored tensor.
template <int WM, int WN, int TMW, int TNW, int PF, int TAPS, int EPI, bool FC>
__device__ __forceinline__ void conv_f32_tile(const ConvArgs& a)
{
    static_assert(!FC || (TAPS == kTaps && PF == 0), "the fused first convolution feeds a 5-tap, unprefetched tile");
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
    // stage and compute in turn (fewer registers, more blocks per CU), every
    // load of a stage in flight before the first LDS store.
    // Thread tid owns chunk q = tid % 4 of LDS rows tid / 4 + u * RS in the halo
    // tile and in the tap-major weight tile (row = tap * BN + column); its
    // sources are fixed apart from the stage's channel offset.  Halo rows
    // outside the batch and columns beyond n are clamped to valid ones: they
    // only feed outputs the epilogue discards.
    constexpr int RS = NT / 4;
    constexpr int WROWS = TAPS * BN;
    static_assert(RS % 16 == 0, "chunk rows of one thread share their swizzle");
    const int q = tid % 4, row0 = tid / 4;
    const int lds0 = lds_at(row0, q);             // + u * RS * KC for chunk u
    auto x_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= XROWS || row0 + u * RS < XROWS; };
    auto w_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= WROWS || row0 + u * RS < WROWS; };
    const float* xsrc[XPT];
    const float* wsrc[WPT];
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
        int64_t g = m0 - RAD + min(row0 + u * RS, XROWS - 1);
        g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
        xsrc[u] = in + g * a.ld_in + 4 * q;
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int wr = min(row0 + u * RS, WROWS - 1);
        const int tap = wr / BN, nn = wr % BN;
        const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
        wsrc[u] = wt + (int64_t)n * kw + tap * a.cin + 4 * q;
    }
    f32x4 xr[FC ? 1 : XPT], wr[WPT];
    auto fetch = [&](int c0) __attribute__((always_inline)) {
        if constexpr (!FC) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) xr[u] = *reinterpret_cast<const f32x4*>(xsrc[u] + c0);
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) wr[u] = *reinterpret_cast<const f32x4*>(wsrc[u] + c0);
    };
    // FC: the halo chunks of stage c0 are computed and stored one at a time,
    // while the stage's weight loads are in flight.
    auto stage = [&](int c0) __attribute__((always_inline)) {
        if constexpr (FC) {
            const int c = c0 + 4 * q;                 // this thread's 4 channels
            float fw[4][kTaps], fb[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                fb[v] = a.first_b[c + v];
#pragma unroll
                for (int j = 0; j < kTaps; ++j) fw[v][j] = a.first_w[(c + v) * kTaps + j];
            }
            const RowMap rmap(m0, a.r_in);
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                if (!x_has(u)) continue;
                int64_t g = m0 - RAD + row0 + u * RS;
                g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
                int64_t e;
                int loc;
                rmap.at((int)(g - m0), e, loc);
                f32x4 y = {0.f, 0.f, 0.f, 0.f};
                if (loc >= kGuard && loc < a.r_in - kGuard) {
                    float x[kTaps];
#pragma unroll
                    for (int j = 0; j < kTaps; ++j) x[j] = a.first_x0[g + j - kGuard];
#pragma unroll
                    for (int v = 0; v < 4; ++v) y[v] = first_conv_at(fw[v], fb[v], x, a.slope);
                }
                *reinterpret_cast<f32x4*>(xs + lds0 + u * RS * KC) = y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < XPT; ++u)
                if (x_has(u)) *reinterpret_cast<f32x4*>(xs + lds0 + u * RS * KC) = xr[u];
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u)
            if (w_has(u)) *reinterpret_cast<f32x4*>(ws + lds0 + u * RS * KC) = wr[u];
    };

    fetch(0);
    stage(0);
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
                bv[j] = *reinterpret_cast<const f32x4*>(ws + lds_at(tap * BN + wn * TNW * 16 + j * 16 + li, lg));
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j][s], av[i][s], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            if (!PF) fetch(c0 + KC);
            stage(c0 + KC);
            __syncthreads();
        }
    }

    f32_epilogue<WM, TMW, TNW, EPI>(acc, a, m0, n0, tid);
}

template <int WM, int WN, int TMW, int TNW, int PF, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(F32Occ<WM, WN, TMW, TNW, PF, TAPS>::v)))
void conv_mfma_f32(ConvArgs a)
{
    conv_f32_tile<WM, WN, TMW, TNW, PF, TAPS, EPI, false>(a);
}

// enc0.c2 with the first convolution in its staging (max-pool epilogue); the
// first convolution's weights take registers, so the occupancy target is two
// waves per SIMD.
template <int WM, int WN, int TMW, int TNW>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(2)))
void conv_mfma_f32_first(ConvArgs a)
{
    conv_f32_tile<WM, WN, TMW, TNW, 0, kTaps, EPI_POOL, true>(a);
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

    // Wave-wide load j fills LDS rows 16 j .. 16 j + 15 of the stage (halo
    // rows first, then the tap-major weight rows tap * BN + column); this
    // wave issues j = wave + t * NW, from a per-lane source computed once.
    constexpr int NJ = XI + WI, JT = (NJ + NW - 1) / NW;
    const int lrow = lane >> 2, lpos = lane & 3;
    const float* src[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = min(wave + t * NW, NJ - 1);
        const bool xj = j < XI;
        const int row = 16 * (xj ? j : j - XI) + lrow;
        const int c = lpos ^ swz(row);
        if (xj) {
            int64_t gr = m0 - RAD + row;
            gr = gr < 0 ? 0 : (gr >= a.m_rows ? a.m_rows - 1 : gr);
            src[t] = in + gr * a.ld_in + 4 * c;
        } else {
            const int tap = row / BN, nn = row % BN;
            const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
            src[t] = wt + (int64_t)n * kw + tap * a.cin + 4 * c;
        }
    }
    auto issue = [&](int buf, int c0) __attribute__((always_inline)) {
        float* base = smem + buf * STAGE;
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            const int j = wave + t * NW;
            if ((t + 1) * NW <= NJ || j < NJ)
                __builtin_amdgcn_global_load_lds((const void*)(src[t] + c0),
                                                 (__attribute__((address_space(3))) void*)(base + 16 * j * KC), 16, 0, 0);
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
                bv[f][j] = *reinterpret_cast<const f32x4*>(ws + lds_at(tap * BN + wn * TNW * 16 + j * 16 + li, lg));
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
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tap & 1][j][s], av[tap & 1][i][s], acc[i][j],
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

template <int WM, int WN, int TMW, int TNW>
hipError_t run_first(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    hipLaunchKernelGGL((conv_mfma_f32_first<WM, WN, TMW, TNW>), grid, dim3(WM * WN * 64), 0, s, a);
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

// Variants that can take the fused first convolution: the single-buffered,
// unprefetched tiles (their halo staging goes through registers).
bool f32_first_ok(int v)
{
    return v == 0 || v == 2 || v == 3 || v == 5;
}

std::string f32_first_kernel_name(int v)
{
    const Variant& x = kVariants[v];
    return "conv_mfma_f32_first<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " +
           std::to_string(x.tmw) + ", " + std::to_string(x.tnw) + ">";
}

hipError_t launch_conv_f32_first(const ConvArgs& a, int v, hipStream_t s)
{
    if (a.cin % KC != 0 || a.m_rows <= 0 || !f32_first_ok(v) || !f32_variant_ok(v, a.n, kTaps, EPI_POOL))
        return hipErrorInvalidValue;
    switch (v) {
    case 0: return run_first<kVariants[0].wm, kVariants[0].wn, kVariants[0].tmw, kVariants[0].tnw>(a, s);
    case 2: return run_first<kVariants[2].wm, kVariants[2].wn, kVariants[2].tmw, kVariants[2].tnw>(a, s);
    case 3: return run_first<kVariants[3].wm, kVariants[3].wn, kVariants[3].tmw, kVariants[3].tnw>(a, s);
    case 5: return run_first<kVariants[5].wm, kVariants[5].wn, kVariants[5].tmw, kVariants[5].tnw>(a, s);
    default: return hipErrorInvalidValue;
    }
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
