// UNet convolutions as implicit GEMM on the matrix cores in BF16 or FP16,
// accumulated in FP32 (mixed-precision inference, Section 5 of
// arXiv:2602.19959: FP16 on the matrix units).
//
// Same GEMM view as the FP32 kernel (m = event row, n = output channel,
// k = (tap, input channel)), with 16-bit activations and weights:
//   * one stage = 32 input channels: the (BM + 4) x 32 halo tile and the
//     BN x 5 x 32 weight tile go to LDS once (unpadded, XOR-swizzled per
//     16-byte chunk) and all five taps read them;
//   * v_mfma_f32_16x16x32_{bf16,f16}: each lane feeds 8 consecutive
//     channels of its weight column and of its position row with one 16-byte
//     LDS read; both use the same lane-to-k map, so the MFMA sums the whole
//     32-channel step.  The weights take the A slot (D^T = W X^T), which
//     leaves four consecutive output channels of one position in each lane;
//   * the k order (stage, tap, MFMA) is fixed by the kernel alone, so every
//     tile-shape variant gives the same bits and results do not depend on
//     the batch;
//   * epilogue: bias (+ LeakyReLU) in FP32, one rounding to 16 bits, then
//     the tile is staged in LDS and written back as whole 16-byte row chunks
//     (channels-last rows are contiguous), with the fused max-pool or the
//     transposed-conv row interleave; the head epilogue works on the FP32
//     accumulators and writes the FP32 probability; a decoder conv whose
//     output only feeds the next transposed conv runs that transposed conv on
//     its tile in the epilogue (EPI_UP) and stores only the upsampled rows;
//   * conv_mfma_lp_first runs enc0.c2 with the first convolution (one input
//     channel, five taps) computed in its halo staging from the histogram
//     rows, so that 32-channel tensor never goes through HBM.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <class T> struct Lp;
template <> struct Lp<__bf16> {
    using vec8 = bf16x8;
    __device__ static f32x4 mfma(vec8 a, vec8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Lp<_Float16> {
    using vec8 = f16x8;
    __device__ static f32x4 mfma(vec8 a, vec8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// LDS rows hold one stage's KC channels as NCH = KC/8 chunks of 16 B, with no
// padding; chunk c of row r sits at position c ^ swz(r): bits 1..2 of r for
// 64-byte rows, twice that for 128-byte rows.  Measured on gfx950 with a
// read-pattern probe, the fragment reads (16 consecutive rows, or rows TAPS
// apart for the weights, at any tap offset) then run at the conflict-free rate.
template <int NCH>
__device__ __forceinline__ int swz(int r)
{
    return NCH == 4 ? ((r >> 1) & 3) : (((r >> 1) & 3) << 1);
}
template <int NCH>
__device__ __forceinline__ int lds_at(int r, int c) { return (r * NCH + (c ^ swz<NCH>(r))) * 8; }   // elements

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

template <int A, int B> struct Max { static constexpr int v = A > B ? A : B; };

// Occupancy target handed to the register allocator: as many waves per SIMD
// as the block's LDS allows on one CU (160 KB), at most 4 (128 registers);
// none for the register-prefetch variants, which need the registers.
// Without it the allocator takes up to 512 registers for 4-wave blocks and
// caps a CU at two of them, where LDS would allow four or five.
constexpr int occupancy_target(int lds_bytes, int waves_per_block)
{
    const int blocks = lds_bytes > 0 ? 163840 / lds_bytes : 8;
    const int w = blocks * waves_per_block / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}
template <int T_BYTES, int BM, int BN, int KC, int TAPS, int EPI, int STAGES, int XPAD>
struct LpLds {
    static constexpr int stage = (BM + XPAD) * KC * T_BYTES + BN * TAPS * KC * T_BYTES;
    static constexpr int v = Max<STAGES * stage, (EPI == EPI_HEAD ? 0 : BM * (BN + 8) * T_BYTES)>::v;
};

// Epilogue shared by the conv kernels (the LDS passed in is free: every
// wave is past its last read of the stage buffers).  The kernels issue the
// MFMA as D^T = W X^T (weight fragment in the A slot), so lane (li, lg) of a
// 16 x 16 tile holds channels 4 lg + v (v = 0..3) of tile row li: four
// consecutive channels of one position, packed into one 8-byte LDS store.
template <class T, int NT, int BM, int BN, int WM, int TMW, int TNW, int EPI>
__device__ __forceinline__ void lp_epilogue(const f32x4 (&acc)[TMW][TNW], const ConvArgs& a, void* lds, int64_t m0,
                                            int n0, int tid)
{
    constexpr int OP = BN + 8;                  // epilogue tile pitch (elements)
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
    } else {
        T* ot = reinterpret_cast<T*>(lds);   // [BM][OP]
#pragma unroll
        for (int j = 0; j < TNW; ++j) {
            const int col = cw + j * 16 + 4 * lg;
            const int n = n0 + col;
            float b[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nv = min(n + v, a.n - 1);    // columns beyond n are never stored
                b[v] = a.bias[EPI == EPI_CONVT ? nv % a.cout : nv];
            }
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                T y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float x = acc[i][j][v] + b[v];
                    if (EPI != EPI_CONVT) x = lrelu(x, a.slope);
                    y[v] = (T)x;
                }
                *reinterpret_cast<uint2*>(ot + (rw + i * 16 + li) * OP + col) = *reinterpret_cast<const uint2*>(y);
            }
        }
        __syncthreads();
        if constexpr (EPI == EPI_UP) {
            // The transposed conv of the tile (BN == n: every channel of its
            // rows is here): column c2 = tap * up_cout + o of the upsampled
            // output is sum_c tile[row][c] up_w[c2][c], over 32-channel chunks
            // in ascending order with the weights in the A slot, as a
            // transposed-conv launch accumulates it, so the bits are the same.
            using V = typename Lp<T>::vec8;
            const T* uw = static_cast<const T*>(a.up_w);
            f32x4 up[TMW][TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j) up[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
            for (int kk = 0; kk < BN; kk += 32) {
                V av[TMW], bv[TNW];
#pragma unroll
                for (int i = 0; i < TMW; ++i)
                    av[i] = *reinterpret_cast<const V*>(ot + (rw + i * 16 + li) * OP + kk + 8 * lg);
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    bv[j] = *reinterpret_cast<const V*>(uw + (size_t)(cw + j * 16 + li) * BN + kk + 8 * lg);
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j) up[i][j] = Lp<T>::mfma(bv[j], av[i], up[i][j]);
            }
            __syncthreads();   // every wave is past its reads of the tile
            // bias, no activation, one rounding; the upsampled tile replaces it
#pragma unroll
            for (int j = 0; j < TNW; ++j) {
                const int col = cw + j * 16 + 4 * lg;
                float b[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) b[v] = a.up_b[(col + v) % a.up_cout];
#pragma unroll
                for (int i = 0; i < TMW; ++i) {
                    T y[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) y[v] = (T)(up[i][j][v] + b[v]);
                    *reinterpret_cast<uint2*>(ot + (rw + i * 16 + li) * OP + col) = *reinterpret_cast<const uint2*>(y);
                }
            }
            __syncthreads();
            // rows 2 t + tap of the destination, as a transposed-conv launch writes them
            T* uo = static_cast<T*>(a.up_out);
            constexpr int UCH = BN / 8;
            for (int idx = tid; idx < BM * UCH; idx += NT) {
                const int row = idx / UCH, q = idx % UCH;
                if (m0 + row >= a.m_rows) continue;
                int64_t e;
                int loc;
                rows.at(row, e, loc);
                if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                const uint4 v = *reinterpret_cast<const uint4*>(ot + row * OP + 8 * q);
                const int tj = (8 * q) / a.up_cout, o = 8 * q - tj * a.up_cout;
                const int64_t ro = e * a.up_r_out + kGuard + 2 * (loc - kGuard) + tj;
                *reinterpret_cast<uint4*>(uo + ro * a.up_ld + o) = v;
            }
            return;
        }
        T* out = static_cast<T*>(a.out);
        constexpr int CH = BN / 8;                  // 16-byte chunks per tile row
        const int n_valid = a.n - n0 < BN ? a.n - n0 : BN;
        for (int idx = tid; idx < BM * CH; idx += NT) {
            const int row = idx / CH, q = idx % CH;
            if (8 * q >= n_valid || m0 + row >= a.m_rows) continue;
            int64_t e;
            int loc;
            rows.at(row, e, loc);
            if (loc < kGuard || loc >= a.r_in - kGuard) continue;
            const uint4 v = *reinterpret_cast<const uint4*>(ot + row * OP + 8 * q);
            if constexpr (EPI == EPI_CONVT) {
                const int n = n0 + 8 * q;
                const int tj = n / a.cout, o = n - tj * a.cout;
                const int64_t ro = e * a.r_out + kGuard + 2 * (loc - kGuard) + tj;
                *reinterpret_cast<uint4*>(out + ro * a.ld_out + o) = v;
            } else {
                *reinterpret_cast<uint4*>(out + (m0 + row) * a.ld_out + n0 + 8 * q) = v;
            }
        }
        if constexpr (EPI == EPI_POOL) {
            T* pout = static_cast<T*>(a.pool_out);
            for (int idx = tid; idx < (BM / 2) * CH; idx += NT) {
                const int pr = idx / CH, q = idx % CH;
                if (8 * q >= n_valid || m0 + 2 * pr >= a.m_rows) continue;   // even: first row of a pooling pair
                int64_t e;
                int loc;
                rows.at(2 * pr, e, loc);
                if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                const uint4 r0 = *reinterpret_cast<const uint4*>(ot + (2 * pr) * OP + 8 * q);
                const uint4 r1 = *reinterpret_cast<const uint4*>(ot + (2 * pr + 1) * OP + 8 * q);
                const T* x0 = reinterpret_cast<const T*>(&r0);
                const T* x1 = reinterpret_cast<const T*>(&r1);
                T y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) y[u] = (float)x0[u] >= (float)x1[u] ? x0[u] : x1[u];
                const int64_t rp = e * a.r_pool + kGuard + (loc - kGuard) / 2;
                *reinterpret_cast<uint4*>(pout + rp * a.ld_pool + n0 + 8 * q) = *reinterpret_cast<const uint4*>(y);
            }
        }
    }
}

// KC: input channels per LDS stage (32 or 64); within a stage the k order is
// (32-channel chunk, tap, MFMA), the same as with KC = 32, so KC does not
// change a bit of the result.  PF = 1: the next stage is fetched into
// registers while the current one computes.
// FC: enc0.c2 with the first convolution fused into the staging: each halo
// chunk is computed from five histogram rows (first_conv_at, the operation
// order of the standalone kernel, so the bits match) instead of read back;
// guard rows are zero, as in the stored tensor.
template <class T, int WM, int WN, int TMW, int TNW, int KC, int PF, int TAPS, int EPI, bool FC>
__device__ __forceinline__ void conv_lp_tile(const ConvArgs& a)
{
    static_assert(!FC || (TAPS == kTaps && PF == 0), "the fused first convolution feeds a 5-tap, unprefetched tile");
    using V = typename Lp<T>::vec8;
    constexpr int NT = WM * WN * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int NCH = KC / 8;                 // 16-byte chunks per row and stage
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int XROWS = BM + TAPS - 1;
    constexpr int XV = XROWS * NCH;
    constexpr int WV = BN * TAPS * NCH;
    constexpr int XPT = (XV + NT - 1) / NT;
    constexpr int WPT = (WV + NT - 1) / NT;
    constexpr int OP = BN + 8;                  // epilogue tile pitch (elements)
    constexpr int STAGE = XROWS * KC + BN * TAPS * KC;
    constexpr int SMEM = Max<STAGE, (EPI == EPI_HEAD ? 0 : BM * OP)>::v;

    __shared__ __attribute__((aligned(16))) T smem[SMEM];
    T* xs = smem;
    T* ws = smem + XROWS * KC;

    const T* in = static_cast<const T*>(a.in);
    const T* wt = static_cast<const T*>(a.w);
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

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Staging: thread tid owns chunk q = tid % NCH of LDS rows tid / NCH + u * RS
    // (RS = NT / NCH), in the halo tile and in the weight tile alike.  Weight
    // rows are tap-major (row = tap * BN + column), so the chunk of stage c0
    // sits at a fixed offset from a per-thread base and the address math is
    // one add per chunk.  Halo rows outside the batch and columns beyond n are
    // clamped to valid ones: they only feed outputs the epilogue discards.
    constexpr int RS = NT / NCH;
    constexpr int WROWS = TAPS * BN;
    static_assert(RS % 8 == 0, "chunk rows of one thread share their swizzle");
    const int q = tid % NCH, row0 = tid / NCH;
    const int lds0 = lds_at<NCH>(row0, q);       // + u * RS * KC for chunk u
    // chunk u exists for this thread (a compile-time true for all but the last)
    auto x_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= XROWS || row0 + u * RS < XROWS; };
    auto w_has = [&](int u) __attribute__((always_inline)) { return (u + 1) * RS <= WROWS || row0 + u * RS < WROWS; };
    auto x_src = [&](int u) __attribute__((always_inline)) {
        const int row = (u + 1) * RS <= XROWS ? row0 + u * RS : min(row0 + u * RS, XROWS - 1);
        int64_t g = m0 - RAD + row;
        g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
        return in + g * a.ld_in + 8 * q;
    };
    auto w_src = [&](int u) __attribute__((always_inline)) {
        const int wr = (u + 1) * RS <= WROWS ? row0 + u * RS : min(row0 + u * RS, WROWS - 1);
        const int tap = wr / BN, nn = wr % BN;
        const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
        return wt + (int64_t)n * kw + tap * a.cin + 8 * q;
    };
    u32x4 xr[FC ? 1 : XPT], wr[WPT];
    auto fetch = [&](int c0) __attribute__((always_inline)) {
        if constexpr (!FC) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) xr[u] = *reinterpret_cast<const u32x4*>(x_src(u) + c0);
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) wr[u] = *reinterpret_cast<const u32x4*>(w_src(u) + c0);
    };
    // FC: the halo chunks of stage c0 are computed and stored one at a time
    // (while the stage's weight loads are in flight), so only this thread's
    // eight channels of first-convolution weights stay in registers.
    auto stage_first = [&](int c0) __attribute__((always_inline)) {
        const int c = c0 + 8 * q;
        float fw[8][kTaps], fb[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
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
            T y[8];
            if (loc < kGuard || loc >= a.r_in - kGuard) {
#pragma unroll
                for (int v = 0; v < 8; ++v) y[v] = (T)0.f;
            } else {
                float x[kTaps];
#pragma unroll
                for (int j = 0; j < kTaps; ++j) x[j] = a.first_x0[g + j - kGuard];
#pragma unroll
                for (int v = 0; v < 8; ++v) y[v] = (T)first_conv_at(fw[v], fb[v], x, a.slope);
            }
            u32x4 yv;
            __builtin_memcpy(&yv, y, sizeof(y));
            *reinterpret_cast<u32x4*>(xs + lds0 + u * RS * KC) = yv;
        }
    };
    auto stage = [&](int c0) __attribute__((always_inline)) {
        if constexpr (FC) {
            stage_first(c0);
        } else {
#pragma unroll
            for (int u = 0; u < XPT; ++u)
                if (x_has(u)) *reinterpret_cast<u32x4*>(xs + lds0 + u * RS * KC) = xr[u];
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u)
            if (w_has(u)) *reinterpret_cast<u32x4*>(ws + lds0 + u * RS * KC) = wr[u];
    };

    fetch(0);
    stage(0);
    __syncthreads();
    for (int c0 = 0; c0 < a.cin; c0 += KC) {
        const bool more = c0 + KC < a.cin;
        if constexpr (PF) {
            if (more) fetch(c0 + KC);
        }
#pragma unroll
        for (int sub = 0; sub < KC / 32; ++sub) {
#pragma unroll
            for (int tap = 0; tap < TAPS; ++tap) {
                V av[TMW], bv[TNW];
#pragma unroll
                for (int i = 0; i < TMW; ++i)
                    av[i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wm * TMW * 16 + i * 16 + li + tap, 4 * sub + lg));
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * BN + wn * TNW * 16 + j * 16 + li, 4 * sub + lg));
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
            }
        }
        __syncthreads();
        if (more) {
            if constexpr (!PF) fetch(c0 + KC);   // all loads in flight before the first store
            stage(c0 + KC);
            __syncthreads();
        }
    }

    __syncthreads();   // the epilogue reuses the stage buffers
    lp_epilogue<T, NT, BM, BN, WM, TMW, TNW, EPI>(acc, a, smem, m0, n0, tid);
}

template <class T, int WM, int WN, int TMW, int TNW, int KC, int PF, int TAPS, int EPI>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(PF ? 1 : occupancy_target(
    LpLds<(int)sizeof(T), WM * TMW * 16, WN * TNW * 16, KC, TAPS, EPI, 1, TAPS - 1>::v, WM * WN))))
void conv_mfma_lp(ConvArgs a)
{
    conv_lp_tile<T, WM, WN, TMW, TNW, KC, PF, TAPS, EPI, false>(a);
}

// enc0.c2 with the first convolution in its staging (32-channel stages,
// max-pool epilogue); the first convolution's weights take registers, so the
// occupancy target is two waves per SIMD.
template <class T, int WM, int WN, int TMW, int TNW>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(2)))
void conv_mfma_lp_first(ConvArgs a)
{
    conv_lp_tile<T, WM, WN, TMW, TNW, 32, 0, kTaps, EPI_POOL, true>(a);
}


// PF = 2 form, double-buffered: stage k + 1 streams from global memory
// straight into the second LDS buffer (global_load_lds_dwordx4: no registers,
// no LDS store instructions) while stage k is on the matrix cores, so a
// block's loads and its MFMAs overlap.  Each wave-wide load fills 1 KB of LDS
// = 16 rows x 64 B; lane L fills slot L of that block (row L / 4, position
// L % 4), so it fetches the chunk that the swizzle puts there.  Rows beyond
// the batch (first and last tile) and columns beyond n (last N tile) are
// clamped to valid addresses: they only feed outputs the epilogue discards.
// Same k order as every other variant (32-channel stage, tap, MFMA).
// NB = 1: one stage buffer, loaded (still straight into LDS) only after every
// wave is done with the previous stage; half the LDS, so more blocks share a
// CU and cover each other's load latency, and one fragment buffer per wave.
template <class T, int WM, int WN, int TMW, int TNW, int TAPS, int EPI, int NB>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(occupancy_target(
    LpLds<(int)sizeof(T), WM * TMW * 16, WN * TNW * 16, 32, TAPS, EPI, NB, 16>::v, WM * WN))))
void conv_mfma_lp_db(ConvArgs a)
{
    using V = typename Lp<T>::vec8;
    constexpr int NW = WM * WN;
    constexpr int NT = NW * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    constexpr int KC = 32, NCH = 4;
    constexpr int ROWB = KC * (int)sizeof(T);        // 64 bytes per LDS row
    constexpr int RAD = (TAPS - 1) / 2;
    constexpr int XR = (BM + TAPS - 1 + 15) / 16 * 16;
    constexpr int WRW = BN * TAPS;
    static_assert(WRW % 16 == 0, "weight rows fill whole 1 KB loads");
    constexpr int XI = XR / 16, WI = WRW / 16;      // wave-wide loads per stage
    constexpr int STAGE = (XR + WRW) * ROWB;         // bytes
    constexpr int OP = BN + 8;
    constexpr int SMEM = Max<NB * STAGE, (EPI == EPI_HEAD ? 0 : BM * OP * (int)sizeof(T))>::v;
    __shared__ __attribute__((aligned(16))) char smem[SMEM];

    const T* in = static_cast<const T*>(a.in);
    const T* wt = static_cast<const T*>(a.w);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar load loop
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
    // wave issues j = wave + t * NW.  Each lane's source is fixed apart from
    // the stage's channel offset, so it is computed once, as a 32-bit byte
    // offset from one of two block-uniform bases (the halo's first row and
    // the N tile's first weight row; clamped rows stay at or after them).
    constexpr int NJ = XI + WI, JT = (NJ + NW - 1) / NW;
    const int lrow = lane >> 2, lpos = lane & 3;
    const char* xbase = reinterpret_cast<const char*>(in + (m0 - RAD) * a.ld_in);
    const char* wbase = reinterpret_cast<const char*>(wt + (int64_t)n0 * kw);
    unsigned off[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = min(wave + t * NW, NJ - 1);
        const bool xj = j < XI;
        const int row = 16 * (xj ? j : j - XI) + lrow;       // row inside its region
        const int c = lpos ^ swz<NCH>(row);                   // chunk held by this slot
        if (xj) {
            int64_t gr = m0 - RAD + row;
            gr = gr < 0 ? 0 : (gr >= a.m_rows ? a.m_rows - 1 : gr);
            off[t] = (unsigned)(((gr - (m0 - RAD)) * a.ld_in + 8 * c) * (int64_t)sizeof(T));
        } else {
            const int tap = row / BN, nn = row % BN;
            const int n = n0 + nn < a.n ? n0 + nn : a.n - 1;
            off[t] = (unsigned)((int64_t)((n - n0) * kw + tap * a.cin + 8 * c) * (int64_t)sizeof(T));
        }
    }
    auto issue = [&](int buf, int c0) __attribute__((always_inline)) {
        char* base = smem + buf * STAGE;
        const unsigned cb = (unsigned)(c0 * (int)sizeof(T));
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            const int j = wave + t * NW;
            if ((t + 1) * NW <= NJ || j < NJ)
                __builtin_amdgcn_global_load_lds((const void*)((j < XI ? xbase : wbase) + (off[t] + cb)),
                                                 (__attribute__((address_space(3))) void*)(base + 16 * j * ROWB), 16, 0, 0);
        }
    };

    const int nk = a.cin / KC;
    issue(0, 0);
    for (int k = 0; k < nk; ++k) {
        // this wave's loads of stage k have landed; the barrier makes every
        // wave's visible and frees the other buffer (its last reads were stage k - 1)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (NB == 2 && k + 1 < nk) issue((k + 1) & 1, (k + 1) * KC);
        const T* xs = reinterpret_cast<const T*>(smem + (NB == 2 ? (k & 1) : 0) * STAGE);
        const T* ws = xs + XR * KC;
        // fragments of tap t + 1 are read while tap t is on the matrix cores
        // (blocks of 16 waves have no registers to spare for that: there the
        // other three waves of the SIMD cover the read latency)
        constexpr int FB = NW < 16 && NB == 2 ? 2 : 1;
        V av[FB][TMW], bv[FB][TNW];
        auto frag = [&](int tap, int f) {
#pragma unroll
            for (int i = 0; i < TMW; ++i)
                av[f][i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wm * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < TNW; ++j)
                bv[f][j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * BN + wn * TNW * 16 + j * 16 + li, lg));
        };
        if constexpr (FB == 2) frag(0, 0);
#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            if constexpr (FB == 2) {
                if (tap + 1 < TAPS) frag(tap + 1, (tap + 1) & 1);
            } else {
                frag(tap, 0);
            }
            const int f = FB == 2 ? (tap & 1) : 0;
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j) acc[i][j] = Lp<T>::mfma(bv[f][j], av[f][i], acc[i][j]);
        }
        if (NB == 1 && k + 1 < nk) {
            __syncthreads();   // every wave is past its reads of the buffer
            issue(0, (k + 1) * KC);
        }
    }
    __syncthreads();   // the epilogue reuses the stage buffers
    lp_epilogue<T, NT, BM, BN, WM, TMW, TNW, EPI>(acc, a, smem, m0, n0, tid);
}

// dec0.c1 and dec0.c2 + head in one launch (level 0 of the decoder, 32
// output channels each): the intermediate 32-channel tensor stays in LDS.
// A block of WM waves owns BO = 64 WM - 16 output rows starting at m0:
//   phase 1 computes dec0.c1's outputs for the BA = 64 WM rows from m0 - 2
//     (the tile and its halo), from two 32-channel stages of the
//     concatenated input, in the standalone launch's k order (chunk, tap)
//     and with its epilogue (bias, LeakyReLU, one rounding); rows that are
//     guard rows or outside the batch are set to zero, as the stored tensor
//     holds them; they go to LDS in the swizzled layout of a 32-channel halo
//     tile;
//   phase 2 runs dec0.c2 on that tile exactly as the standalone head launch
//     runs it on its staged halo (same fragments, k order and head
//     epilogue), so every bit of p is the same as from the two launches.
// c1: dec0.c1's arguments; c2: dec0.c2 + head's (in and ld_in unused).
template <class T, int WM>
__global__ __launch_bounds__(WM * 64) __attribute__((amdgpu_waves_per_eu(WM >= 8 ? 2 : 3)))
void conv_mfma_lp_dec0(ConvArgs c1, ConvArgs c2)
{
    using V = typename Lp<T>::vec8;
    constexpr int NT = WM * 64;
    constexpr int BA = WM * 64;                  // phase-1 rows per block
    constexpr int BO = BA - 16;                  // output rows per block
    constexpr int KC = 32, NCH = 4;              // one 32-channel stage, 64-byte rows
    constexpr int XR1 = BA + kTaps - 1;          // phase-1 halo rows
    constexpr int WR = kTaps * 32;               // weight rows (tap-major) of either conv
    constexpr int ATR = BA + 16;                 // intermediate tile rows (phase 2 reads up to BA + 3)
    __shared__ __attribute__((aligned(16))) T xs[(XR1 + WR) * KC];   // phase-1 stage; phase-2 weights
    __shared__ __attribute__((aligned(16))) T at[ATR * KC];          // dec0.c1's output tile
    T* ws = xs + XR1 * KC;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m_tiles = (int)((c2.m_rows + BO - 1) / BO);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = slot * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BO;
    const int64_t a0 = m0 - 2;                   // first phase-1 row

    const T* in1 = static_cast<const T*>(c1.in);
    const T* w1 = static_cast<const T*>(c1.w);
    const T* w2 = static_cast<const T*>(c2.w);

    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // ---- phase 1: dec0.c1 over rows a0 .. a0 + BA - 1, one 32-channel stage
    // at a time; the next stage's 16-byte loads (and, during the last stage,
    // dec0.c2's weights) are in flight in registers while the current stage
    // is on the matrix cores.  Halo rows outside the batch are clamped (they
    // only feed zeroed or discarded rows).
    constexpr int NC1 = (XR1 + WR) * NCH, P1 = (NC1 + NT - 1) / NT;
    constexpr int NC2 = WR * NCH, P2 = (NC2 + NT - 1) / NT;
    auto fetch1 = [&](int c0, u32x4 (&v)[P1]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < P1; ++u) {
            const int idx = min(tid + u * NT, NC1 - 1);
            const int row = idx / NCH, q = idx % NCH;
            const T* src;
            if (row < XR1) {
                int64_t g = a0 - 2 + row;
                g = g < 0 ? 0 : (g >= c1.m_rows ? c1.m_rows - 1 : g);
                src = in1 + g * c1.ld_in + c0 + 8 * q;
            } else {
                const int wr = row - XR1, tap = wr / 32, n = wr % 32;
                src = w1 + (int64_t)n * (kTaps * c1.cin) + tap * c1.cin + c0 + 8 * q;
            }
            v[u] = *reinterpret_cast<const u32x4*>(src);
        }
    };
    auto store1 = [&](const u32x4 (&v)[P1]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < P1; ++u) {
            // halo rows in xs, weight rows in ws, each region swizzled by its own row index
            const int idx = tid + u * NT;
            const int row = idx / NCH, q = idx % NCH;
            if ((u + 1) * NT <= NC1 || idx < NC1)
                *reinterpret_cast<u32x4*>(row < XR1 ? xs + lds_at<NCH>(row, q) : ws + lds_at<NCH>(row - XR1, q)) = v[u];
        }
    };
    auto fetch2 = [&](u32x4 (&v)[P2]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < P2; ++u) {
            const int idx = min(tid + u * NT, NC2 - 1);
            const int wr = idx / NCH, q = idx % NCH, tap = wr / 32, n = wr % 32;
            v[u] = *reinterpret_cast<const u32x4*>(w2 + (int64_t)n * (kTaps * c2.cin) + tap * c2.cin + 8 * q);
        }
    };
    u32x4 cur[P1], nxt[P1], wv2[P2];
    fetch1(0, cur);
    for (int c0 = 0; c0 < c1.cin; c0 += KC) {
        store1(cur);
        __syncthreads();
        if (c0 + KC < c1.cin) fetch1(c0 + KC, nxt);
        else fetch2(wv2);
#pragma unroll
        for (int tap = 0; tap < kTaps; ++tap) {
            V av[4], bv[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wave * 64 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * 32 + j * 16 + li, lg));
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P1; ++u) cur[u] = nxt[u];
    }
    // dec0.c1's epilogue into the tile: row r of the tile is row a0 + r
    {
        const RowMap rmap(a0 < 0 ? 0 : a0, c1.r_in);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wave * 64 + i * 16 + li;
            const int64_t g = a0 + r;
            bool keep = g >= 0 && g < c1.m_rows;
            if (keep) {
                int64_t e;
                int loc;
                rmap.at((int)(g - (a0 < 0 ? 0 : a0)), e, loc);
                keep = loc >= kGuard && loc < c1.r_in - kGuard;
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = j * 16 + 4 * lg;
                T y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) y[v] = keep ? (T)lrelu(acc[i][j][v] + c1.bias[col + v], c1.slope) : (T)0.f;
                *reinterpret_cast<uint2*>(at + lds_at<NCH>(r, col / 8) + (col % 8)) = *reinterpret_cast<const uint2*>(y);
            }
        }
    }
    // ---- phase 2: dec0.c2's weights, already in registers, into the free stage buffer
#pragma unroll
    for (int u = 0; u < P2; ++u) {
        const int idx = tid + u * NT;
        if ((u + 1) * NT <= NC2 || idx < NC2) *reinterpret_cast<u32x4*>(ws + lds_at<NCH>(idx / NCH, idx % NCH)) = wv2[u];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < kTaps; ++tap) {
        V av[4], bv[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const V*>(at + lds_at<NCH>(wave * 64 + i * 16 + li + tap, lg));
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * 32 + j * 16 + li, lg));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
    }
    // head epilogue: output rows t < BO of the block
    const RowMap rows(m0, c2.r_in);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float sum = 0.f;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = j * 16 + 4 * lg;
#pragma unroll
            for (int v = 0; v < 4; ++v) sum += lrelu(acc[i][j][v] + c2.bias[c + v], c2.slope) * c2.head_w[c + v];
        }
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
        const int t = wave * 64 + i * 16 + li;
        if (lg == 0 && t < BO && m0 + t < c2.m_rows) {
            int64_t e;
            int loc;
            rows.at(t, e, loc);
            if (loc >= kGuard && loc < c2.r_in - kGuard)
                c2.prob[e * c2.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(sum + c2.head_b)));
        }
    }
}

// The same fused level 0 with its stages loaded straight into LDS
// (global_load_lds_dwordx4, as the direct-to-LDS conv tiles load theirs) and
// one buffer: no staging registers, and dec0.c1's output tile takes the place
// of phase 1's halo tile (both are swizzled 32-channel tiles of the same
// rows), so a block needs 27 KB (4 waves) or 46 KB (8 waves) of LDS and more
// blocks share a CU.  Same fragments, k order and epilogues as
// conv_mfma_lp_dec0, hence the same bits.
template <class T, int WM>
__global__ __launch_bounds__(WM * 64) __attribute__((amdgpu_waves_per_eu(4)))
void conv_mfma_lp_dec0d(ConvArgs c1, ConvArgs c2)
{
    using V = typename Lp<T>::vec8;
    constexpr int NW = WM;
    constexpr int BA = WM * 64;                  // phase-1 rows per block
    constexpr int BO = BA - 16;                  // output rows per block
    constexpr int KC = 32, NCH = 4;              // 32-channel stages, 64-byte rows
    constexpr int ROWB = KC * (int)sizeof(T);
    constexpr int XRA = (BA + kTaps - 1 + 15) / 16 * 16;   // halo rows, whole 1 KB loads
    constexpr int WR = kTaps * 32;               // weight rows (tap-major) of either conv
    constexpr int XI = XRA / 16, WI = WR / 16;   // wave-wide loads of the halo and of a weight tile
    __shared__ __attribute__((aligned(16))) char smem[(XRA + WR) * ROWB];
    T* const xs = reinterpret_cast<T*>(smem);    // phase 1: halo tile; phase 2: dec0.c1's output tile
    T* const ws = xs + XRA * KC;                 // weights of the current conv

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int m_tiles = (int)((c2.m_rows + BO - 1) / BO);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = slot * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BO;
    const int64_t a0 = m0 - 2;                   // first phase-1 row

    // Wave-wide load j fills LDS rows 16 j .. 16 j + 15 (halo rows, then the
    // weight rows tap * 32 + column); lane L fills slot L % 4 of row L / 4 with
    // the chunk the swizzle puts there.  Sources: 32-bit byte offsets from the
    // halo's first row and from the weights; halo rows outside the batch are
    // clamped (they only feed zeroed or discarded rows).
    constexpr int NJ = XI + WI, JT = (NJ + NW - 1) / NW;
    const int lrow = lane >> 2, lpos = lane & 3;
    const char* xbase = reinterpret_cast<const char*>(static_cast<const T*>(c1.in) + (a0 - 2) * c1.ld_in);
    const char* w1 = static_cast<const char*>(c1.w);
    const char* w2 = static_cast<const char*>(c2.w);
    unsigned off[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = min(wave + t * NW, NJ - 1);
        const bool xj = j < XI;
        const int row = 16 * (xj ? j : j - XI) + lrow;
        const int c = lpos ^ swz<NCH>(row);
        if (xj) {
            int64_t g = a0 - 2 + row;
            g = g < 0 ? 0 : (g >= c1.m_rows ? c1.m_rows - 1 : g);
            off[t] = (unsigned)(((g - (a0 - 2)) * c1.ld_in + 8 * c) * (int64_t)sizeof(T));
        } else {
            const int tap = row / 32, n = row % 32;
            off[t] = (unsigned)((n * (kTaps * c1.cin) + tap * c1.cin + 8 * c) * (int)sizeof(T));
        }
    }
    auto issue1 = [&](int c0) __attribute__((always_inline)) {
        const unsigned cb = (unsigned)(c0 * (int)sizeof(T));
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            const int j = wave + t * NW;
            if ((t + 1) * NW <= NJ || j < NJ)
                __builtin_amdgcn_global_load_lds((const void*)((j < XI ? xbase : w1) + (off[t] + cb)),
                                                 (__attribute__((address_space(3))) void*)(smem + 16 * j * ROWB), 16,
                                                 0, 0);
        }
    };
    // dec0.c2's weights (32 input channels: one stage) into the weight rows
    auto issue2 = [&]() __attribute__((always_inline)) {
        constexpr int J2 = (WI + NW - 1) / NW;
#pragma unroll
        for (int t = 0; t < J2; ++t) {
            const int j = wave + t * NW;
            if ((t + 1) * NW <= WI || j < WI) {
                const int row = 16 * j + lrow, tap = row / 32, n = row % 32;
                const int c = lpos ^ swz<NCH>(row);
                __builtin_amdgcn_global_load_lds(
                    (const void*)(w2 + (n * (kTaps * c2.cin) + tap * c2.cin + 8 * c) * (int)sizeof(T)),
                    (__attribute__((address_space(3))) void*)(smem + (XI + j) * 16 * ROWB), 16, 0, 0);
            }
        }
    };

    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // ---- phase 1: dec0.c1 over rows a0 .. a0 + BA - 1
    issue1(0);
    for (int c0 = 0; c0 < c1.cin; c0 += KC) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < kTaps; ++tap) {
            V av[4], bv[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wave * 64 + i * 16 + li + tap, lg));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * 32 + j * 16 + li, lg));
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
        }
        __syncthreads();   // every wave is past its reads of the stage
        if (c0 + KC < c1.cin) issue1(c0 + KC);
    }
    issue2();
    // dec0.c1's epilogue into the tile (the halo's place): row r is row a0 + r
    {
        const RowMap rmap(a0 < 0 ? 0 : a0, c1.r_in);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wave * 64 + i * 16 + li;
            const int64_t g = a0 + r;
            bool keep = g >= 0 && g < c1.m_rows;
            if (keep) {
                int64_t e;
                int loc;
                rmap.at((int)(g - (a0 < 0 ? 0 : a0)), e, loc);
                keep = loc >= kGuard && loc < c1.r_in - kGuard;
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = j * 16 + 4 * lg;
                T y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) y[v] = keep ? (T)lrelu(acc[i][j][v] + c1.bias[col + v], c1.slope) : (T)0.f;
                *reinterpret_cast<uint2*>(xs + lds_at<NCH>(r, col / 8) + (col % 8)) = *reinterpret_cast<const uint2*>(y);
            }
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // ---- phase 2: dec0.c2 on the tile (rows BA .. BA + 3 of it are stale
    // halo rows: they only feed outputs t >= BO, which are not stored)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < kTaps; ++tap) {
        V av[4], bv[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wave * 64 + i * 16 + li + tap, lg));
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * 32 + j * 16 + li, lg));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
    }
    // head epilogue: output rows t < BO of the block
    const RowMap rows(m0, c2.r_in);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float sum = 0.f;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = j * 16 + 4 * lg;
#pragma unroll
            for (int v = 0; v < 4; ++v) sum += lrelu(acc[i][j][v] + c2.bias[c + v], c2.slope) * c2.head_w[c + v];
        }
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
        const int t = wave * 64 + i * 16 + li;
        if (lg == 0 && t < BO && m0 + t < c2.m_rows) {
            int64_t e;
            int loc;
            rows.at(t, e, loc);
            if (loc >= kGuard && loc < c2.r_in - kGuard)
                c2.prob[e * c2.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(sum + c2.head_b)));
        }
    }
}

// enc0.c2 (32 channels in and out) with the first convolution computed in
// its staging, the weight tile loaded straight into LDS: no staging
// registers, the first convolution's weights and biases in LDS (one copy per
// block, read by every thread), and each thread computing one 8-channel chunk
// of R consecutive halo rows from one window of R + 4 histogram values, all
// loaded while the weight tile streams in.  The arithmetic per value is
// first_conv_at and one rounding, as in the standalone kernel, and the
// 32-channel stage, k order and max-pool epilogue are those of the
// register-staged tile, so the bits are the same.
template <class T, int WM, int TMW>
__global__ __launch_bounds__(WM * 64) __attribute__((amdgpu_waves_per_eu(4)))
void conv_mfma_lp_firstd(ConvArgs a)
{
    using V = typename Lp<T>::vec8;
    constexpr int NW = WM, NT = NW * 64;
    constexpr int BM = WM * TMW * 16;
    constexpr int TNW = 2, BN = 32;              // all 32 output channels
    constexpr int KC = 32, NCH = 4;              // the one 32-channel stage, 64-byte rows
    constexpr int ROWB = KC * (int)sizeof(T);
    constexpr int XROWS = BM + kTaps - 1;
    constexpr int XR = (XROWS + 15) / 16 * 16;
    constexpr int WRW = BN * kTaps;
    constexpr int OP = BN + 8;
    constexpr int SMEM = Max<(XR + WRW) * ROWB, BM * OP * (int)sizeof(T)>::v;
    constexpr int GR = NT / NCH;                 // row groups (one per thread and chunk)
    constexpr int R = (XROWS + GR - 1) / GR;     // consecutive halo rows per thread
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    __shared__ __attribute__((aligned(16))) float fp[KC * kTaps + KC];   // first conv: weights [c][5], biases [c]
    T* const xs = reinterpret_cast<T*>(smem);
    T* const ws = xs + XR * KC;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int m_tiles = (int)((a.m_rows + BM - 1) / BM);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = slot * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BM;

    // weight tile: wave-wide load j fills weight rows 16 j .. 16 j + 15
    // (row = tap * 32 + column), lane L slot L % 4 of row L / 4
    const T* wt = static_cast<const T*>(a.w);
#pragma unroll
    for (int t = 0; t < (WRW / 16 + NW - 1) / NW; ++t) {
        const int j = wave + t * NW;
        if (j >= WRW / 16) continue;
        const int row = 16 * j + (lane >> 2), tap = row / BN, n = row % BN;
        const int c = (lane & 3) ^ swz<NCH>(row);
        __builtin_amdgcn_global_load_lds((const void*)(wt + (int64_t)n * (kTaps * a.cin) + tap * a.cin + 8 * c),
                                         (__attribute__((address_space(3))) void*)(ws + 16 * j * KC), 16, 0, 0);
    }
    // the first convolution's 160 weights and 32 biases
    if (wave == 0 && lane < KC * kTaps / 4)
        __builtin_amdgcn_global_load_lds((const void*)(a.first_w + 4 * lane),
                                         (__attribute__((address_space(3))) void*)fp, 16, 0, 0);
    if (wave == NW - 1 && lane < KC / 4)
        __builtin_amdgcn_global_load_lds((const void*)(a.first_b + 4 * lane),
                                         (__attribute__((address_space(3))) void*)(fp + KC * kTaps), 16, 0, 0);
    // this thread's rows r0 .. r0 + R - 1 (halo row r is row m0 - 2 + r) and
    // their histogram window, clamped to the batch (clamped values only feed
    // rows that are stored as zero)
    const int q = tid % NCH, r0 = (tid / NCH) * R;
    float xw[R + kTaps - 1];
#pragma unroll
    for (int k = 0; k < R + kTaps - 1; ++k) {
        int64_t g = m0 - 2 + r0 + k - kGuard;
        g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
        xw[k] = a.first_x0[g];
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    {
        const RowMap rmap(m0, a.r_in);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int r = r0 + u;
            if (r >= XROWS) break;
            int64_t g = m0 - 2 + r;
            g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
            int64_t e;
            int loc;
            rmap.at((int)(g - m0), e, loc);
            T y[8];
            if (loc < kGuard || loc >= a.r_in - kGuard) {
#pragma unroll
                for (int v = 0; v < 8; ++v) y[v] = (T)0.f;
            } else {
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int c = 8 * q + v;
                    float w5[kTaps];
#pragma unroll
                    for (int k = 0; k < kTaps; ++k) w5[k] = fp[c * kTaps + k];
                    y[v] = (T)first_conv_at(w5, fp[KC * kTaps + c], xw + u, a.slope);
                }
            }
            u32x4 yv;
            __builtin_memcpy(&yv, y, sizeof(y));
            *reinterpret_cast<u32x4*>(xs + lds_at<NCH>(r, q)) = yv;
        }
    }
    __syncthreads();

    f32x4 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < kTaps; ++tap) {
        V av[TMW], bv[TNW];
#pragma unroll
        for (int i = 0; i < TMW; ++i)
            av[i] = *reinterpret_cast<const V*>(xs + lds_at<NCH>(wave * TMW * 16 + i * 16 + li + tap, lg));
#pragma unroll
        for (int j = 0; j < TNW; ++j)
            bv[j] = *reinterpret_cast<const V*>(ws + lds_at<NCH>(tap * BN + j * 16 + li, lg));
#pragma unroll
        for (int i = 0; i < TMW; ++i)
#pragma unroll
            for (int j = 0; j < TNW; ++j) acc[i][j] = Lp<T>::mfma(bv[j], av[i], acc[i][j]);
    }
    __syncthreads();   // the epilogue reuses the stage buffer
    lp_epilogue<T, NT, BM, BN, WM, TMW, TNW, EPI_POOL>(acc, a, smem, m0, 0, tid);
}

template <class T, int WM, int WN, int TMW, int TNW, int KC, int PF, int TAPS, int EPI>
hipError_t run(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    if constexpr (PF == 2 || PF == 4)
        hipLaunchKernelGGL((conv_mfma_lp_db<T, WM, WN, TMW, TNW, TAPS, EPI, PF == 2 ? 2 : 1>), grid,
                           dim3(WM * WN * 64), 0, s, a);
    else
        hipLaunchKernelGGL((conv_mfma_lp<T, WM, WN, TMW, TNW, KC, PF, TAPS, EPI>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

template <class T, int WM, int WN, int TMW, int TNW>
hipError_t run_first(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 16;
    constexpr int BN = WN * TNW * 16;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    hipLaunchKernelGGL((conv_mfma_lp_first<T, WM, WN, TMW, TNW>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

// Tile-shape / staging variants; all give identical bits.
struct Variant { int wm, wn, tmw, tnw, kc, pf; };
constexpr Variant kVariants[] = {
    {4, 1, 4, 2, 32, 0},   //  0: 256 x 32
    {4, 1, 4, 4, 32, 0},   //  1: 256 x 64
    {2, 2, 4, 4, 32, 0},   //  2: 128 x 128
    {4, 2, 4, 4, 32, 0},   //  3: 256 x 128 (512 threads)
    {4, 1, 2, 4, 32, 0},   //  4: 128 x 64
    {2, 1, 4, 2, 32, 0},   //  5: 128 x 32 (128 threads)
    {4, 2, 4, 4, 32, 1},   //  6: 256 x 128, register prefetch
    {4, 2, 4, 4, 64, 0},   //  7: 256 x 128, 64-channel stages
    {4, 1, 4, 2, 64, 0},   //  8: 256 x 32, 64-channel stages
    {4, 1, 4, 4, 64, 1},   //  9: 256 x 64, 64-channel stages, prefetch
    {2, 2, 4, 4, 32, 1},   // 10: 128 x 128, prefetch
    {4, 1, 4, 2, 32, 1},   // 11: 256 x 32, prefetch
    {4, 2, 4, 4, 32, 2},   // 12: 256 x 128, double-buffered direct-to-LDS stages
    {4, 1, 4, 4, 32, 2},   // 13: 256 x 64, double-buffered
    {4, 1, 4, 2, 32, 2},   // 14: 256 x 32, double-buffered
    {2, 2, 4, 4, 32, 2},   // 15: 128 x 128, double-buffered
    {2, 1, 4, 2, 32, 2},   // 16: 128 x 32, double-buffered (128 threads)
    {2, 2, 8, 4, 32, 2},   // 17: 256 x 128, double-buffered, 128 x 64 per wave
    {2, 1, 8, 4, 32, 2},   // 18: 256 x 64, double-buffered, 128 x 64 per wave (128 threads)
    {8, 2, 4, 4, 32, 2},   // 19: 512 x 128, double-buffered (1024 threads, one block per CU)
    {8, 1, 4, 2, 32, 0},   // 20: 512 x 32 (the weight tile staged once per 512 rows)
    {8, 1, 4, 2, 32, 2},   // 21: 512 x 32, double-buffered
    {8, 1, 4, 4, 32, 0},   // 22: 512 x 64
    {8, 1, 4, 4, 32, 2},   // 23: 512 x 64, double-buffered
    {4, 1, 4, 2, 32, 3},   // 24: head launch with dec0.c1 fused (conv_mfma_lp_dec0, 4 waves, 240 rows)
    {8, 1, 4, 2, 32, 3},   // 25: the same with 8 waves (496 rows)
    {4, 2, 4, 4, 32, 4},   // 26: 256 x 128, single-buffered direct-to-LDS stages
    {8, 1, 4, 4, 32, 4},   // 27: 512 x 64, single-buffered direct-to-LDS
    {4, 1, 4, 4, 32, 4},   // 28: 256 x 64, single-buffered direct-to-LDS
    {4, 1, 4, 2, 32, 4},   // 29: 256 x 32, single-buffered direct-to-LDS
    {2, 2, 4, 4, 32, 4},   // 30: 128 x 128, single-buffered direct-to-LDS
    {4, 1, 4, 2, 32, 5},   // 31: head launch with dec0.c1 fused, stages straight into LDS (4 waves, 240 rows)
    {8, 1, 4, 2, 32, 5},   // 32: the same with 8 waves (496 rows)
    {2, 1, 4, 2, 32, 6},   // 33: enc0.c2 with the first conv, weight tile straight into LDS (128 x 32)
    {4, 1, 4, 2, 32, 6},   // 34: the same, 256 x 32
    {8, 1, 4, 2, 32, 6},   // 35: the same, 512 x 32
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define PVF_LP_CASE(V)                                                                                     \
    case V:                                                                                                \
        return run<T, kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw, kVariants[V].kc, \
                   kVariants[V].pf, TAPS, EPI>(a, s);

template <class T, int TAPS, int EPI>
hipError_t dispatch(int v, const ConvArgs& a, hipStream_t s)
{
    if constexpr (EPI == EPI_UP) {
        switch (v) {
            PVF_LP_CASE(1)
            PVF_LP_CASE(2)
            PVF_LP_CASE(3)
            PVF_LP_CASE(4)
            PVF_LP_CASE(9)
            PVF_LP_CASE(12)
            PVF_LP_CASE(13)
            PVF_LP_CASE(15)
            PVF_LP_CASE(19)
            PVF_LP_CASE(22)
            PVF_LP_CASE(23)
            PVF_LP_CASE(26)
            PVF_LP_CASE(27)
            PVF_LP_CASE(28)
            PVF_LP_CASE(30)
        default: return hipErrorInvalidValue;
        }
    } else if constexpr (EPI == EPI_HEAD) {
        switch (v) {
            PVF_LP_CASE(0)
            PVF_LP_CASE(1)
            PVF_LP_CASE(4)
            PVF_LP_CASE(5)
            PVF_LP_CASE(11)
            PVF_LP_CASE(13)
            PVF_LP_CASE(14)
            PVF_LP_CASE(16)
            PVF_LP_CASE(20)
            PVF_LP_CASE(21)
            PVF_LP_CASE(22)
            PVF_LP_CASE(23)
            PVF_LP_CASE(27)
            PVF_LP_CASE(28)
            PVF_LP_CASE(29)
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (v) {
            PVF_LP_CASE(0)
            PVF_LP_CASE(1)
            PVF_LP_CASE(2)
            PVF_LP_CASE(3)
            PVF_LP_CASE(4)
            PVF_LP_CASE(5)
            PVF_LP_CASE(6)
            PVF_LP_CASE(7)
            PVF_LP_CASE(8)
            PVF_LP_CASE(9)
            PVF_LP_CASE(10)
            PVF_LP_CASE(11)
            PVF_LP_CASE(12)
            PVF_LP_CASE(13)
            PVF_LP_CASE(14)
            PVF_LP_CASE(15)
            PVF_LP_CASE(16)
            PVF_LP_CASE(17)
            PVF_LP_CASE(18)
            PVF_LP_CASE(19)
            PVF_LP_CASE(20)
            PVF_LP_CASE(21)
            PVF_LP_CASE(22)
            PVF_LP_CASE(23)
            PVF_LP_CASE(26)
            PVF_LP_CASE(27)
            PVF_LP_CASE(28)
            PVF_LP_CASE(29)
            PVF_LP_CASE(30)
        // 33-35 run as the register-staged tile of the same shape when
        // enc0.c2 does not compute the first convolution (calibration)
        case 33: return run<T, 2, 1, 4, 2, 32, 0, TAPS, EPI>(a, s);
        case 34: return run<T, 4, 1, 4, 2, 32, 0, TAPS, EPI>(a, s);
        case 35: return run<T, 8, 1, 4, 2, 32, 0, TAPS, EPI>(a, s);
        default: return hipErrorInvalidValue;
        }
    }
}

template <class T>
hipError_t launch_typed(const ConvArgs& a, int taps, Epi epi, int v, hipStream_t s)
{
    if (taps == 5) {
        switch (epi) {
        case EPI_STORE: return dispatch<T, 5, EPI_STORE>(v, a, s);
        case EPI_POOL: return dispatch<T, 5, EPI_POOL>(v, a, s);
        case EPI_HEAD: return dispatch<T, 5, EPI_HEAD>(v, a, s);
        case EPI_UP: return dispatch<T, 5, EPI_UP>(v, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (taps == 1 && epi == EPI_CONVT) return dispatch<T, 1, EPI_CONVT>(v, a, s);
    return hipErrorInvalidValue;
}

}  // namespace

int lp_variant_count() { return kNumVariants; }

bool lp_variant_ok(int v, int n, int cin, int taps, Epi epi)
{
    if (v < 0 || v >= kNumVariants) return false;
    const Variant& x = kVariants[v];
    if (x.pf == 3 || x.pf == 5) return epi == EPI_HEAD && n == 32 && cin == 32 && taps == kTaps;   // dec0 fused: 32-channel head
    if (x.pf == 6) return epi == EPI_POOL && n == 32 && cin == 32 && taps == kTaps;   // enc0.c2 of 32 channels
    const int bn = x.wn * x.tnw * 16;
    if (cin % x.kc != 0) return false;
    if (epi == EPI_HEAD)
        return (v == 0 || v == 1 || v == 4 || v == 5 || v == 11 || v == 13 || v == 14 || v == 16 || v >= 20) &&
               bn == n && x.wn == 1;
    if (epi == EPI_UP)   // the tile must hold every channel of its rows
        return (v == 1 || v == 2 || v == 3 || v == 4 || v == 9 || v == 12 || v == 13 || v == 15 || v == 19 ||
                v == 22 || v == 23 || v == 26 || v == 27 || v == 28 || v == 30) && bn == n;
    return bn <= (n < 32 ? 32 : n);
}

// Defaults from the autotuner's BF16 picks on MI355X at 1000 events.  The
// small-channel layers take the 512-row, 128-row or 64-channel-stage tiles
// (the 32-channel enc0.c2: the 512-row tile that computes the first
// convolution with its weight tile loaded straight into LDS);
// from 64 output channels and 64 input channels on, the single-buffered
// direct-to-LDS 256 x 64 tile (four blocks per CU; also the 64-channel head),
// except the 128-channel layer over 64 input channels (256 x 128, single
// stage, register-staged); the 1x1 transposed convs the double-buffered
// 128 x 128 tile.
int lp_default_variant(int n, int cin, int taps, Epi epi)
{
    if (epi == EPI_HEAD) return n == 64 ? 28 : 20;
    if (epi == EPI_CONVT && taps == 1) return n >= 512 ? 17 : (n >= 128 ? 15 : (cin % 64 == 0 ? 8 : 4));
    if (n <= 32) return epi == EPI_POOL ? (n == 32 && cin == 32 ? 35 : 5) : (cin % 64 == 0 ? 8 : 14);
    if (cin <= 32) return 22;
    if (n > 64 && cin < 128) return 3;
    return 28;
}

// Decoder convs that run the following transposed conv in their epilogue
// need a tile of all their output channels; the autotuner's BF16 picks at
// 1000 events: 512 x 64 for 64 channels, the single-buffered direct-to-LDS
// 256 x 128 for 128; -1 where no such variant fits.
int lp_default_up_variant(int n, int cin)
{
    const int v = n == 64 ? 22 : (n == 128 ? 26 : -1);
    return v >= 0 && lp_variant_ok(v, n, cin, kTaps, EPI_UP) ? v : -1;
}

bool lp_dec0_ok(int v) { return v >= 0 && v < kNumVariants && (kVariants[v].pf == 3 || kVariants[v].pf == 5); }

hipError_t launch_conv_lp_dec0(int dtype, const ConvArgs& c1, const ConvArgs& c2, int v, hipStream_t s)
{
    if (!lp_dec0_ok(v) || c1.cin % 32 != 0 || c1.n != 32 || c2.cin != 32 || c2.n != 32 || c1.m_rows != c2.m_rows ||
        c1.r_in != c2.r_in || c2.m_rows <= 0 || !c2.prob || !c2.head_w)
        return hipErrorInvalidValue;
    const int wm = kVariants[v].wm;
    const bool dma = kVariants[v].pf == 5;
    const int bo = wm * 64 - 16;
    const unsigned m_tiles = (unsigned)((c2.m_rows + bo - 1) / bo);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds);
    auto go = [&](auto tag) {
        using T = decltype(tag);
        if (dma) {
            if (wm == 4) hipLaunchKernelGGL((conv_mfma_lp_dec0d<T, 4>), grid, dim3(256), 0, s, c1, c2);
            else hipLaunchKernelGGL((conv_mfma_lp_dec0d<T, 8>), grid, dim3(512), 0, s, c1, c2);
        } else {
            if (wm == 4) hipLaunchKernelGGL((conv_mfma_lp_dec0<T, 4>), grid, dim3(256), 0, s, c1, c2);
            else hipLaunchKernelGGL((conv_mfma_lp_dec0<T, 8>), grid, dim3(512), 0, s, c1, c2);
        }
    };
    if (dtype == PVF_BF16) go(__bf16{});
    else if (dtype == PVF_FP16) go(_Float16{});
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

std::string lp_kernel_name(int dtype, int v, int taps, Epi epi)
{
    const Variant& x = kVariants[v];
    if (x.pf == 6)   // not fused: the register-staged tile of the same shape runs
        return std::string("conv_mfma_lp<") + (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " +
               std::to_string(x.wm) + ", 1, " + std::to_string(x.tmw) + ", 2, 32, 0, " + std::to_string(taps) + ", " +
               std::to_string((int)epi) + ">";
    if (x.pf == 3 || x.pf == 5)
        return std::string(x.pf == 3 ? "conv_mfma_lp_dec0<" : "conv_mfma_lp_dec0d<") +
               (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " + std::to_string(x.wm) + ">";
    if (x.pf == 2 || x.pf == 4)
        return std::string("conv_mfma_lp_db<") + (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " +
               std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) + ", " +
               std::to_string(x.tnw) + ", " + std::to_string(taps) + ", " + std::to_string((int)epi) + ", " +
               (x.pf == 2 ? "2" : "1") + ">";
    return std::string("conv_mfma_lp<") + (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " +
           std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) + ", " +
           std::to_string(x.tnw) + ", " + std::to_string(x.kc) + ", " + std::to_string(x.pf) + ", " +
           std::to_string(taps) + ", " + std::to_string((int)epi) + ">";
}

// Variants that can take the fused first convolution: the single-buffered,
// unprefetched 32-channel-stage tiles (their halo staging goes through
// registers; the double-buffered ones load straight into LDS).
bool lp_first_ok(int v)
{
    return v == 0 || v == 1 || v == 5 || v == 20 || v == 22 || v == 33 || v == 34 || v == 35;
}

std::string lp_first_kernel_name(int dtype, int v)
{
    const Variant& x = kVariants[v];
    if (x.pf == 6)
        return std::string("conv_mfma_lp_firstd<") + (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " +
               std::to_string(x.wm) + ", " + std::to_string(x.tmw) + ">";
    return std::string("conv_mfma_lp_first<") + (dtype == PVF_BF16 ? "__bf16" : "_Float16") + ", " +
           std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) + ", " +
           std::to_string(x.tnw) + ">";
}

hipError_t launch_conv_lp_first(int dtype, const ConvArgs& a, int v, hipStream_t s)
{
    if (a.cin % 32 != 0 || a.m_rows <= 0 || !lp_first_ok(v) || !lp_variant_ok(v, a.n, a.cin, kTaps, EPI_POOL))
        return hipErrorInvalidValue;
    if (dtype != PVF_BF16 && dtype != PVF_FP16) return hipErrorInvalidValue;
    if (kVariants[v].pf == 6) {
        if (a.n != 32 || a.cin != 32) return hipErrorInvalidValue;
        const int wm = kVariants[v].wm, bm = wm * 64;
        const unsigned m_tiles = (unsigned)((a.m_rows + bm - 1) / bm);
        dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds);
        auto go = [&](auto tag) {
            using T = decltype(tag);
            if (wm == 2) hipLaunchKernelGGL((conv_mfma_lp_firstd<T, 2, 4>), grid, dim3(128), 0, s, a);
            else if (wm == 4) hipLaunchKernelGGL((conv_mfma_lp_firstd<T, 4, 4>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((conv_mfma_lp_firstd<T, 8, 4>), grid, dim3(512), 0, s, a);
        };
        if (dtype == PVF_BF16) go(__bf16{});
        else go(_Float16{});
        return hipGetLastError();
    }
#define PVF_LP_FIRST(V, TYPE)                                                                                  \
    case V:                                                                                                \
        return run_first<TYPE, kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw>(a, s);
    if (dtype == PVF_BF16) {
        switch (v) {
            PVF_LP_FIRST(0, __bf16)
            PVF_LP_FIRST(1, __bf16)
            PVF_LP_FIRST(5, __bf16)
            PVF_LP_FIRST(20, __bf16)
            PVF_LP_FIRST(22, __bf16)
        default: return hipErrorInvalidValue;
        }
    }
    switch (v) {
        PVF_LP_FIRST(0, _Float16)
        PVF_LP_FIRST(1, _Float16)
        PVF_LP_FIRST(5, _Float16)
        PVF_LP_FIRST(20, _Float16)
        PVF_LP_FIRST(22, _Float16)
    default: return hipErrorInvalidValue;
    }
#undef PVF_LP_FIRST
}

hipError_t launch_conv_lp(int dtype, const ConvArgs& a, int taps, Epi epi, int v, hipStream_t s)
{
    if (a.cin % 32 != 0 || a.m_rows <= 0 || !lp_variant_ok(v, a.n, a.cin, taps, epi)) return hipErrorInvalidValue;
    if (epi == EPI_CONVT && a.cout % 8 != 0) return hipErrorInvalidValue;
    if (epi == EPI_UP && (!a.up_w || !a.up_b || !a.up_out || a.up_cout % 8 != 0 || 2 * a.up_cout != a.n))
        return hipErrorInvalidValue;
    if (dtype == PVF_BF16) return launch_typed<__bf16>(a, taps, epi, v, s);
    if (dtype == PVF_FP16) return launch_typed<_Float16>(a, taps, epi, v, s);
    return hipErrorInvalidValue;
}

}  // namespace pvf
