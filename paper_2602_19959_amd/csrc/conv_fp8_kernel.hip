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
// and of its column (B).  32-byte LDS rows, two 16-byte chunks; chunk q of
// row r sits at q ^ bit 3 of r (swz32): measured on gfx950 with a read-pattern
// probe, the fragment reads (16 consecutive rows, or rows TAPS apart for the
// weights, at any tap offset) then run at the conflict-free rate, where the
// unswizzled rows took two LDS passes per read.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;            // input channels (bytes) per stage and row

__device__ __forceinline__ int swz32(int r) { return (r >> 3) & 1; }
// byte offset of the 8-byte piece p (0..3) of row r in a 32-byte-row tile
__device__ __forceinline__ int at32(int r, int p) { return r * KC + 16 * ((p >> 1) ^ swz32(r)) + 8 * (p & 1); }

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

__device__ __forceinline__ float e4m3_to_f32(uint8_t b)
{
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e ? ldexpf(1.f + m / 8.f, e - 7) : ldexpf(m / 8.f, -6);
    return (b & 0x80) ? -v : v;
}

template <int A, int B> struct Max { static constexpr int v = A > B ? A : B; };

// Occupancy target handed to the register allocator: as many waves per SIMD
// as the block's LDS allows on one CU (160 KB), at most 4 (128 registers).
constexpr int occupancy_target(int lds_bytes, int waves_per_block)
{
    const int blocks = lds_bytes > 0 ? 163840 / lds_bytes : 8;
    const int w = blocks * waves_per_block / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// Epilogue shared by the FP8 kernels (the LDS passed in is free).  The
// kernels issue the MFMA as D^T = W X^T (weight fragment in the A slot), so
// lane (li, lg) of a 16 x 16 tile holds channels 4 lg + v (v = 0..3) of tile
// row li: four consecutive FP8 outputs of one position, one 4-byte LDS store.
template <int NT, int BM, int BN, int WM, int TMW, int TNW, int EPI>
__device__ __forceinline__ void fp8_epilogue(const f32x4 (&acc)[TMW][TNW], const ConvArgs& a, void* lds, int64_t m0,
                                             int n0, int tid)
{
    constexpr int OP = BN + 16;                  // epilogue tile pitch (bytes)
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rw = (wave % WM) * TMW * 16;
    const int cw = (wave / WM) * TNW * 16;
    const RowMap rows(m0, a.r_in);
    if constexpr (EPI == EPI_HEAD) {
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < TNW; ++j) {
                const int c = n0 + cw + j * 16 + 4 * lg;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    s += lrelu(acc[i][j][v] * a.col_scale[c + v] + a.bias[c + v], a.slope) * a.head_w[c + v];
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
    } else {
        uint8_t* ot = static_cast<uint8_t*>(lds);   // [BM][OP] bytes
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int col = cw + j * 16 + 4 * lg;
            // y / a_out = LeakyReLU(acc * s_n / a_out + b / a_out): one FMA per
            // value with the folded per-column factors (n % 16 == 0, so a
            // lane's four columns are all valid or all past n)
            const int nc = min(n0 + col, a.n - 4);
            const f32x4 fs = *reinterpret_cast<const f32x4*>(a.fold_scale + nc);
            const f32x4 fb = *reinterpret_cast<const f32x4*>(a.fold_bias + nc);
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                float y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float x = fmaf(acc[i][j][v], fs[v], fb[v]);
                    if (EPI != EPI_CONVT) x = lrelu(x, a.slope);
                    y[v] = fminf(fmaxf(x, -448.f), 448.f);   // saturate (the conversion maps overflow to NaN)
                }
                // two packed conversions: channel 4 lg + v goes to byte v
                uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], (int)w, true);
                *reinterpret_cast<uint32_t*>(ot + (rw + i * 16 + li) * OP + col) = w;
            }
        }
        __syncthreads();
        uint8_t* out = static_cast<uint8_t*>(a.out);
        constexpr int CH = BN / 16;                 // 16-byte chunks per tile row
        const int n_valid = a.n - n0 < BN ? a.n - n0 : BN;
        for (int idx = tid; idx < BM * CH; idx += NT) {
            const int row = idx / CH, q = idx % CH;
            if (16 * q >= n_valid || m0 + row >= a.m_rows) continue;
            int64_t e;
            int loc;
            rows.at(row, e, loc);
            if (loc < kGuard || loc >= a.r_in - kGuard) continue;
            const uint4 v = *reinterpret_cast<const uint4*>(ot + row * OP + 16 * q);
            if constexpr (EPI == EPI_CONVT) {
                const int n = n0 + 16 * q;
                const int tj = n / a.cout, o = n - tj * a.cout;
                const int64_t ro = e * a.r_out + kGuard + 2 * (loc - kGuard) + tj;
                *reinterpret_cast<uint4*>(out + ro * a.ld_out + o) = v;
            } else {
                *reinterpret_cast<uint4*>(out + (m0 + row) * a.ld_out + n0 + 16 * q) = v;
            }
        }
        if constexpr (EPI == EPI_POOL) {
            uint8_t* pout = static_cast<uint8_t*>(a.pool_out);
            for (int idx = tid; idx < (BM / 2) * CH; idx += NT) {
                const int pr = idx / CH, q = idx % CH;
                if (16 * q >= n_valid || m0 + 2 * pr >= a.m_rows) continue;
                int64_t e;
                int loc;
                rows.at(2 * pr, e, loc);
                if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                // two whole 16-byte rows from LDS, compared in registers
                const uint4 r0 = *reinterpret_cast<const uint4*>(ot + (2 * pr) * OP + 16 * q);
                const uint4 r1 = *reinterpret_cast<const uint4*>(ot + (2 * pr + 1) * OP + 16 * q);
                const uint8_t* x0 = reinterpret_cast<const uint8_t*>(&r0);
                const uint8_t* x1 = reinterpret_cast<const uint8_t*>(&r1);
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
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(occupancy_target(
    Max<(WM * TMW * 16 + TAPS - 1) * 32 + WN * TNW * 16 * TAPS * 32,
        (EPI == EPI_HEAD ? 0 : WM * TMW * 16 * (WN * TNW * 16 + 16))>::v, WM * WN))))
void conv_mfma_fp8(ConvArgs a)
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

    // Staging: thread tid owns chunk q = tid % NCH of LDS rows tid / NCH + u * RS
    // in the halo tile and in the tap-major weight tile (row = tap * BN +
    // column); every load of a stage is in flight before the first LDS store.
    // Halo rows outside the batch and columns beyond n are clamped to valid
    // ones: they only feed outputs the epilogue discards.
    constexpr int RS = NT / NCH;
    constexpr int WROWS = TAPS * BN;
    constexpr int XPT = (XV + NT - 1) / NT, WPT = (WV + NT - 1) / NT;
    static_assert(RS % 16 == 0, "chunk rows of one thread share their swizzle");
    const int q = tid % NCH, row0 = tid / NCH;
    const int lds0 = row0 * KC + 16 * (q ^ swz32(row0));   // + u * RS * KC for chunk u
    auto x_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= XROWS || row0 + u * RS < XROWS; };
    auto w_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= WROWS || row0 + u * RS < WROWS; };
    const uint8_t* xsrc[XPT];
    const uint8_t* wsrc[WPT];
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
        int64_t g = m0 - RAD + min(row0 + u * RS, XROWS - 1);
        g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
        xsrc[u] = in + g * a.ld_in + 16 * q;
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int wr = min(row0 + u * RS, WROWS - 1);
        const int tap = wr / BN, nn = wr % BN;
        const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
        wsrc[u] = wt + (int64_t)n * kw + tap * a.cin + 16 * q;
    }

    for (int c0 = 0; c0 < a.cin; c0 += KC) {
        u32x4 xr[XPT], wr[WPT];
#pragma unroll
        for (int u = 0; u < XPT; ++u) xr[u] = *reinterpret_cast<const u32x4*>(xsrc[u] + c0);
#pragma unroll
        for (int u = 0; u < WPT; ++u) wr[u] = *reinterpret_cast<const u32x4*>(wsrc[u] + c0);
#pragma unroll
        for (int u = 0; u < XPT; ++u)
            if (x_has(u)) *reinterpret_cast<u32x4*>(xs + lds0 + u * RS * KC) = xr[u];
#pragma unroll
        for (int u = 0; u < WPT; ++u)
            if (w_has(u)) *reinterpret_cast<u32x4*>(ws + lds0 + u * RS * KC) = wr[u];
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            long av[TMW], bv[TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[i] = *reinterpret_cast<const long*>(xs + at32(wm * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[j] = *reinterpret_cast<const long*>(ws + at32(tap * BN + wn * TNW * 16 + j * 16 + li, lg));
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(bv[j], av[i], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    __syncthreads();   // the epilogue reuses the stage buffers
    fp8_epilogue<NT, BM, BN, WM, TMW, TNW, EPI>(acc, a, smem, m0, n0, tid);
}


// Double-buffered form for layers with 64 or more input channels: one stage
// = 64 channels (bytes) per row, 64-byte LDS rows as in the 16-bit kernels;
// stage k + 1 streams straight into the second LDS buffer
// (global_load_lds_dwordx4) while stage k computes, and the fragments of the
// next (chunk, tap) are read during the current MFMAs.  Same k order as
// conv_mfma_fp8 (32-channel chunk, tap), so the same bits.  Chunk c of row r
// sits at c ^ bits 2..3 of r: measured on gfx950 with a read-pattern probe,
// the 8-byte fragment reads (16 consecutive rows, or rows TAPS apart, at any
// tap offset) then run at the conflict-free rate, twice as fast as with
// c ^ 2*bit3(r).  Out-of-range rows and columns are clamped (their outputs
// are discarded).
__device__ __forceinline__ int swz64(int r) { return (r >> 2) & 3; }

template <int WM, int WN, int TMW, int TNW, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) void conv_mfma_fp8_db(ConvArgs a)
{
    constexpr int NW = WM * WN;
    constexpr int NT = NW * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int KB = 64;                       // channels (bytes) per stage and row
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int XR = (BM + TAPS - 1 + 15) / 16 * 16;
    constexpr int WRW = BN * TAPS;
    static_assert(WRW % 16 == 0, "weight rows fill whole 1 KB loads");
    constexpr int XI = XR / 16, WI = WRW / 16;
    constexpr int STAGE = (XR + WRW) * KB;
    constexpr int SMEM = Max<2 * STAGE, (EPI == EPI_HEAD ? 0 : BM * (BN + 16))>::v;
    __shared__ __attribute__((aligned(16))) uint8_t smem[SMEM];

    const uint8_t* in = static_cast<const uint8_t*>(a.in);
    const uint8_t* wt = static_cast<const uint8_t*>(a.w);
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

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Wave-wide load j fills LDS rows 16 j .. 16 j + 15 of the stage (halo
    // rows first, then the tap-major weight rows tap * BN + column); this
    // wave issues j = wave + t * NW.  Each lane's source is a 32-bit byte
    // offset, computed once, from one of two block-uniform bases (the halo's
    // first row and the N tile's first weight row; clamped rows stay at or
    // after them).
    constexpr int NJ = XI + WI, JT = (NJ + NW - 1) / NW;
    const int lrow = lane >> 2, lpos = lane & 3;
    const uint8_t* xbase = in + (m0 - RAD) * a.ld_in;
    const uint8_t* wbase = wt + (int64_t)n0 * kw;
    unsigned off[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = min(wave + t * NW, NJ - 1);
        const bool xj = j < XI;
        const int row = 16 * (xj ? j : j - XI) + lrow;
        const int c = lpos ^ swz64(row);
        if (xj) {
            int64_t gr = m0 - RAD + row;
            gr = gr < 0 ? 0 : (gr >= a.m_rows ? a.m_rows - 1 : gr);
            off[t] = (unsigned)((gr - (m0 - RAD)) * a.ld_in + 16 * c);
        } else {
            const int tap = row / BN, nn = row % BN;
            const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
            off[t] = (unsigned)((n - n0) * kw + tap * a.cin + 16 * c);
        }
    }
    auto issue = [&](int buf, int c0) __attribute__((always_inline)) {
        uint8_t* base = smem + buf * STAGE;
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            const int j = wave + t * NW;
            if ((t + 1) * NW <= NJ || j < NJ)
                __builtin_amdgcn_global_load_lds((const void*)((j < XI ? xbase : wbase) + (off[t] + (unsigned)c0)),
                                                 (__attribute__((address_space(3))) void*)(base + 16 * j * KB), 16, 0, 0);
        }
    };
    // 8-byte piece lg of 32-channel chunk `sub` of row r: byte offset in the row
    auto piece = [](int r, int sub, int lg) { return 16 * ((2 * sub + (lg >> 1)) ^ swz64(r)) + 8 * (lg & 1); };

    const int nk = a.cin / KB;
    issue(0, 0);
    for (int k = 0; k < nk; ++k) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (k + 1 < nk) issue((k + 1) & 1, (k + 1) * KB);
        const uint8_t* xs = smem + (k & 1) * STAGE;
        const uint8_t* ws = xs + XR * KB;
        long av[2][TMW], bv[2][TNW];
        auto frag = [&](int sub, int tap, int f) {
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                const int r = wm * TMW * 16 + i * 16 + li + tap;
                av[f][i] = *reinterpret_cast<const long*>(xs + r * KB + piece(r, sub, lg));
            }
#pragma unroll
            for (int j = 0; j < TNW; ++j) {
                const int r = tap * BN + wn * TNW * 16 + j * 16 + li;
                bv[f][j] = *reinterpret_cast<const long*>(ws + r * KB + piece(r, sub, lg));
            }
        };
        frag(0, 0, 0);
#pragma unroll
        for (int st = 0; st < 2 * TAPS; ++st) {          // (sub, tap) in k order
            if (st + 1 < 2 * TAPS) frag((st + 1) / TAPS, (st + 1) % TAPS, (st + 1) & 1);
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(bv[st & 1][j], av[st & 1][i], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();   // the epilogue reuses the stage buffers
    fp8_epilogue<NT, BM, BN, WM, TMW, TNW, EPI>(acc, a, smem, m0, n0, tid);
}

template <int WM, int WN, int TMW, int TNW, int DB, int TAPS, int EPI>
hipError_t run(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    if constexpr (DB)
        hipLaunchKernelGGL((conv_mfma_fp8_db<WM, WN, TMW, TNW, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    else
        hipLaunchKernelGGL((conv_mfma_fp8<WM, WN, TMW, TNW, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

struct Variant { int wm, wn, tmw, tnw, db; };
constexpr Variant kVariants[] = {
    {4, 1, 4, 2, 0},   // 0: 256 x 32
    {4, 1, 4, 4, 0},   // 1: 256 x 64
    {2, 2, 4, 4, 0},   // 2: 128 x 128
    {4, 2, 4, 4, 0},   // 3: 256 x 128 (512 threads)
    {4, 2, 4, 4, 1},   // 4: 256 x 128, double-buffered 64-channel stages
    {4, 1, 4, 4, 1},   // 5: 256 x 64, double-buffered
    {4, 1, 4, 2, 1},   // 6: 256 x 32, double-buffered
    {2, 2, 8, 4, 1},   // 7: 256 x 128, double-buffered, 128 x 64 per wave
    {8, 2, 4, 4, 1},   // 8: 512 x 128, double-buffered (1024 threads, one block per CU)
    {8, 1, 4, 2, 0},   // 9: 512 x 32 (the weight tile staged once per 512 rows)
    {8, 1, 4, 4, 0},   // 10: 512 x 64
    {8, 1, 4, 4, 1},   // 11: 512 x 64, double-buffered
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define PVF_FP8_CASE(V) \
    case V:                                                                                                  \
        return run<kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw, kVariants[V].db, TAPS, \
                   EPI>(a, s);

template <int TAPS, int EPI>
hipError_t dispatch(int v, const ConvArgs& a, hipStream_t s)
{
    if constexpr (EPI == EPI_HEAD) {
        switch (v) {
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(5)
            PVF_FP8_CASE(6)
            PVF_FP8_CASE(9)
            PVF_FP8_CASE(10)
            PVF_FP8_CASE(11)
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (v) {
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(2)
            PVF_FP8_CASE(3)
            PVF_FP8_CASE(4)
            PVF_FP8_CASE(5)
            PVF_FP8_CASE(6)
            PVF_FP8_CASE(7)
            PVF_FP8_CASE(8)
            PVF_FP8_CASE(9)
            PVF_FP8_CASE(10)
            PVF_FP8_CASE(11)
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int fp8_variant_count() { return kNumVariants; }

bool fp8_variant_ok(int v, int n, int cin, int taps, Epi epi)
{
    if (v < 0 || v >= kNumVariants) return false;
    (void)taps;
    const Variant& x = kVariants[v];
    const int bn = x.wn * x.tnw * 16;
    if (cin % (x.db ? 64 : KC) != 0) return false;
    if (epi == EPI_HEAD) return (v == 0 || v == 1 || v == 5 || v == 6 || v >= 9) && bn == n && x.wn == 1;
    return bn <= (n < 32 ? 32 : n);
}

// Picks of variant sweeps over 1000 events: the double-buffered 64-channel
// stages wherever the layer has them (cin a multiple of 64) and enough
// output channels; the single-buffered tiles for 32- and 64-channel inputs,
// 512 rows tall where the input has 32 channels (the weight tile is then
// staged once per 512 rows).
int fp8_default_variant(int n, int cin, int taps, Epi epi)
{
    if (epi == EPI_HEAD) return n == 64 ? 1 : (cin <= 32 ? 9 : 0);
    if (epi == EPI_CONVT && taps == 1) return n >= 128 ? 4 : 6;
    if (n <= 32) return cin <= 32 ? 9 : 0;
    if (cin >= 128) return 5;
    return cin <= 32 ? 10 : 1;
}

std::string fp8_kernel_name(int v, int cin, int taps, Epi epi)
{
    (void)cin;
    const Variant& x = kVariants[v];
    return std::string(x.db ? "conv_mfma_fp8_db<" : "conv_mfma_fp8<") + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) +
           ", " + std::to_string(x.tnw) + ", " + std::to_string(taps) + ", " + std::to_string((int)epi) + ">";
}

hipError_t launch_conv_fp8(const ConvArgs& a, int taps, Epi epi, int v, hipStream_t s)
{
    if (a.cin % KC != 0 || a.m_rows <= 0 || !fp8_variant_ok(v, a.n, a.cin, taps, epi) || !a.col_scale)
        return hipErrorInvalidValue;
    if (epi != EPI_HEAD && (!a.fold_scale || !a.fold_bias || a.n % 16 != 0)) return hipErrorInvalidValue;
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
