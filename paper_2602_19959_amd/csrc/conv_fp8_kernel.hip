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

constexpr int KC = 32;            // input channels (bytes) per stage and row

__device__ __forceinline__ int swz32(int r) { return (r >> 3) & 1; }
// byte offset of the 8-byte piece p (0..3) of row r in a 32-byte-row tile
__device__ __forceinline__ int at32(int r, int p) { return r * KC + 16 * ((p >> 1) ^ swz32(r)) + 8 * (p & 1); }

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

// Occupancy target handed to the register allocator: as many waves per SIMD
// as the block's LDS allows on one CU (160 KB), at most 4 (128 registers).
constexpr int occupancy_target(int lds_bytes, int waves_per_block)
{
    const int blocks = lds_bytes > 0 ? 163840 / lds_bytes : 8;
    const int w = blocks * waves_per_block / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// Epilogue shared by the FP8 kernels (the LDS passed in is free).  D layout
// of a 16x16 MFMA: lane holds rows 4*lg + v of column li.
template <int NT, int BM, int BN, int WM, int TMW, int TNW, int EPI>
__device__ __forceinline__ void fp8_epilogue(const f32x4 (&acc)[TMW][TNW], const ConvArgs& a, void* lds, int64_t m0,
                                             int n0, int tid)
{
    constexpr int OP = BN + 16;                  // epilogue tile pitch (bytes)
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rw = (wave % WM) * TMW * 16;
    const int cw = (wave / WM) * TNW * 16;
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
        uint8_t* ot = static_cast<uint8_t*>(lds);   // [BM][OP] bytes
        // A lane holds 4 rows (4 lg + v) of one column; a 4 x 4 byte transpose
        // inside each quad of lanes (two DPP exchanges, two byte permutes)
        // gives lane 4k + m row 4 lg + m of columns 4k .. 4k + 3, written as
        // one 4-byte LDS store instead of four single-byte ones.
        const int m = li & 3, kq = li >> 2;
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int col = cw + j * 16 + li;
            const int n = n0 + col;
            const int oc = EPI == EPI_CONVT ? n % a.cout : n;      // output channel
            const float cs = n < a.n ? a.col_scale[n] : 0.f;
            const float b = n < a.n ? a.bias[oc] : 0.f;
            const float inv = n < a.n ? a.out_inv_scale[oc] : 0.f;
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                uint32_t w = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float y = acc[i][j][v] * cs + b;
                    if (EPI != EPI_CONVT) y = lrelu(y, a.slope);
                    w |= (uint32_t)to_e4m3(y * inv) << (8 * v);
                }
                // quad exchange 1 (lanes m ^ 1): even m keeps bytes 0, 2 and
                // takes the partner's 0, 2; odd m the partner's 1, 3 and its own 1, 3
                const uint32_t p1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0xB1, 0xF, 0xF, false);
                const uint32_t x = __builtin_amdgcn_perm(p1, w, (m & 1) ? 0x03070105u : 0x06020400u);
                // quad exchange 2 (lanes m ^ 2)
                const uint32_t p2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
                const uint32_t y4 = __builtin_amdgcn_perm(p2, x, (m & 2) ? 0x03020706u : 0x05040100u);
                *reinterpret_cast<uint32_t*>(ot + (rw + i * 16 + 4 * lg + m) * OP + cw + j * 16 + 4 * kq) = y4;
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

    for (int c0 = 0; c0 < a.cin; c0 += KC) {
        for (int idx = tid; idx < XV; idx += NT) {
            const int row = idx / NCH, q = idx % NCH;
            const int64_t g = m0 - RAD + row;
            uint4 v = {0u, 0u, 0u, 0u};
            if (g >= 0 && g < a.m_rows) v = *reinterpret_cast<const uint4*>(in + g * a.ld_in + c0 + 16 * q);
            *reinterpret_cast<uint4*>(xs + row * KC + 16 * (q ^ swz32(row))) = v;
        }
        for (int idx = tid; idx < WV; idx += NT) {
            const int q = idx % NCH, rest = idx / NCH;
            const int tap = rest % TAPS, nn = rest / TAPS;
            uint4 v = {0u, 0u, 0u, 0u};
            if (n0 + nn < a.n)
                v = *reinterpret_cast<const uint4*>(wt + (int64_t)(n0 + nn) * kw + tap * a.cin + c0 + 16 * q);
            *reinterpret_cast<uint4*>(ws + rest * KC + 16 * (q ^ swz32(rest))) = v;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            long av[TMW], bv[TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[i] = *reinterpret_cast<const long*>(xs + at32(wm * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[j] = *reinterpret_cast<const long*>(ws + at32((wn * TNW * 16 + j * 16 + li) * TAPS + tap, lg));
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[i], bv[j], acc[i][j], 0, 0, 0);
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

    const int lrow = lane >> 2, lpos = lane & 3;
    auto issue = [&](int buf, int c0) {
        uint8_t* base = smem + buf * STAGE;
        for (int j = wave; j < XI + WI; j += NW) {
            const bool xj = j < XI;
            const int row = 16 * (xj ? j : j - XI) + lrow;
            const int c = lpos ^ swz64(row);
            const uint8_t* g;
            if (xj) {
                int64_t gr = m0 - RAD + row;
                gr = gr < 0 ? 0 : (gr >= a.m_rows ? a.m_rows - 1 : gr);
                g = in + gr * a.ld_in + c0 + 16 * c;
            } else {
                const int nn = row / TAPS, tap = row - nn * TAPS;
                const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
                g = wt + (int64_t)n * kw + tap * a.cin + c0 + 16 * c;
            }
            uint8_t* dst = base + (xj ? 16 * j * KB : XR * KB + 16 * (j - XI) * KB);
            __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
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
                const int r = (wn * TNW * 16 + j * 16 + li) * TAPS + tap;
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
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[st & 1][i], bv[st & 1][j], acc[i][j], 0, 0, 0);
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
    if (epi == EPI_HEAD) return (v == 0 || v == 1 || v == 5 || v == 6) && bn == n && x.wn == 1;
    return bn <= (n < 32 ? 32 : n);
}

// Picks of variant sweeps over 1000 events: the double-buffered 64-channel
// stages wherever the layer has them (cin a multiple of 64) and enough
// output channels; the single-buffered tiles for 32-channel inputs.
int fp8_default_variant(int n, int cin, int taps, Epi epi)
{
    if (epi == EPI_HEAD) return n == 64 ? 1 : 0;
    if (epi == EPI_CONVT && taps == 1) return n >= 256 ? 2 : (n >= 128 ? 4 : 6);
    if (n <= 32) return 0;
    if (cin >= 128) return 5;
    return 1;
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
