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
// MFMA: v_mfma_f32_32x32x64_f8f6f4 with both operands e4m3 and no block
// scale, the gfx950 matrix instruction that runs FP8 at twice the 16-bit
// rate (measured at 4.6 PFLOP/s register to register, 4.5 with its operands
// read from LDS in 64 x 64 tiles per wave).  The GEMM k axis of a 5-tap
// convolution is cut into 32-byte slices, one (32-channel chunk, tap) pair
// each, in the order (chunk, tap); one MFMA takes two consecutive slices,
// lanes 0-31 the first and lanes 32-63 the second (32 bytes per lane, the
// instruction's k layout).  A stage holds KB = 64 channels (10 slices, five
// MFMAs per 32 x 32 block) when the input has a multiple of 64 channels,
// else KB = 32 (5 slices: the third MFMA's second half is zero).  Each
// layer has one stage width, so every tile variant of a layer pairs the same
// slices and gives the same bits.  The weights take the A slot (D^T = W X^T):
// lane l of a 32 x 32 block then holds position l % 32 and, in register v,
// output channel 8 (v / 4) + 4 (l / 32) + v % 4 (four consecutive channels per
// register quad).
//
// Stages are double-buffered (NB = 2): stage k + 1 streams from global memory
// straight into the second LDS buffer (16-byte global_load_lds) while stage k
// is on the matrix cores.  Single-buffered variants (NB = 1) load a stage only
// after every wave is done with the previous one; they take half the LDS, so
// more blocks share a CU, which is what hides the load latency in layers of
// one or two stages (at most 128 input channels).  LDS rows hold KB bytes in
// 16-byte chunks, chunk c of row r at c ^ s(r) (s = bits 2..3 of r for 64-byte
// rows, bit 3 for 32-byte rows).
//
// A decoder conv whose output only feeds the next transposed conv runs that
// transposed conv on its FP8 output tile in the epilogue (EPI_UP) and stores
// only the upsampled rows.
#include "pvf_internal.h"

namespace pvf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float lrelu(float x, float s) { return x >= 0.f ? x : s * x; }

__device__ __forceinline__ float e4m3_to_f32(uint8_t b)
{
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e ? ldexpf(1.f + m / 8.f, e - 7) : ldexpf(m / 8.f, -6);
    return (b & 0x80) ? -v : v;
}

template <int A, int B> struct Max { static constexpr int v = A > B ? A : B; };

template <int KB>
__device__ __forceinline__ int swz(int r) { return KB == 64 ? ((r >> 2) & 3) : ((r >> 3) & 1); }

__device__ __forceinline__ i32x8 join(u32x4 lo, u32x4 hi)
{
    return i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
}

// Fragment buffers: two (the next MFMA step's fragments are read while the
// current one computes), or one in 16-wave blocks, whose four waves per SIMD
// leave 128 registers a lane and cover the read latency themselves, and in
// the single-buffered variants, which aim at more waves per SIMD.
constexpr int frag_bufs(int waves, int nb) { return waves >= 16 || nb == 1 ? 1 : 2; }

// Occupancy target handed to the register allocator: as many waves per SIMD
// as both the block's LDS (160 KB per CU) and an estimate of its registers
// (accumulators, fragments, addressing; 512 per lane and SIMD) allow, at
// most 4, and at least what one block puts on each SIMD.
constexpr int occupancy_target(int lds_bytes, int waves_per_block, int tmw, int tnw, int nb)
{
    const int blocks = lds_bytes > 0 ? 163840 / lds_bytes : 8;
    int w = blocks * waves_per_block / 4;
    const int regs = tmw * tnw * 16 + frag_bufs(waves_per_block, nb) * (tmw + tnw) * 8 + 48;
    w = w < 512 / regs ? w : 512 / regs;
    w = w < 1 ? 1 : (w > 4 ? 4 : w);
    const int need = (waves_per_block + 3) / 4;
    return w < need ? need : w;
}

template <int BM, int BN, int KB, int TAPS, int EPI, int NB>
struct F8Lds {
    static constexpr int RPL = 1024 / KB;
    static constexpr int XR = (BM + TAPS - 1 + RPL - 1) / RPL * RPL;
    static constexpr int STAGE = (XR + BN * TAPS) * KB;
    static constexpr int v = Max<NB * STAGE, (EPI == EPI_HEAD ? 0 : BM * (BN + 16))>::v;
};

// FC: enc0.c2 with the first convolution computed in its staging (one
// 32-channel stage): the first convolution's weights, biases and output
// scales go to LDS with the weight tile, each thread computes one 16-channel
// chunk of R consecutive halo rows from one window of R + 4 histogram values
// (loaded while the tiles stream in), with first_conv_at and the standalone
// kernel's scaling and saturation, so the codes, and every bit after them,
// are the same; guard rows and rows outside the batch are zero, as in the
// stored tensor.
template <int WM, int WN, int TMW, int TNW, int KB, int TAPS, int EPI, int NB, bool FC>
__device__ __forceinline__ void fp8_tile(const ConvArgs& a)
{
    static_assert(!FC || (TAPS == kTaps && EPI == EPI_POOL && KB == 32), "the first convolution feeds enc0.c2");
    constexpr int NW = WM * WN;
    constexpr int NT = NW * 64;
    constexpr int BM = WM * TMW * 32;
    constexpr int BN = WN * TNW * 32;
    constexpr int NS = KB / 32;                  // 32-channel chunks per stage
    constexpr int SL = NS * TAPS;                // 32-byte k slices per stage
    constexpr int STEPS = (SL + 1) / 2;          // MFMAs per 32 x 32 block and stage
    constexpr int RPL = 1024 / KB;               // LDS rows per wave-wide 1 KB load
    constexpr int CPR = KB / 16;                 // 16-byte chunks per row
    constexpr int RAD = (TAPS - 1) / 2;
    using L = F8Lds<BM, BN, KB, TAPS, EPI, NB>;
    constexpr int XR = L::XR;
    constexpr int WRW = BN * TAPS;
    static_assert(WRW % RPL == 0, "weight rows fill whole 1 KB loads");
    constexpr int XI = XR / RPL, WI = WRW / RPL;
    constexpr int STAGE = L::STAGE;
    constexpr int OP = BN + 16;                  // epilogue tile pitch (bytes)
    __shared__ __attribute__((aligned(16))) uint8_t smem[L::v];
    __shared__ __attribute__((aligned(16))) float fp[FC ? 7 * KB : 4];   // FC: weights [c][5], biases, 1 / output scales

    const uint8_t* in = static_cast<const uint8_t*>(a.in);
    const uint8_t* wt = static_cast<const uint8_t*>(a.w);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WM;
    const int wn = wave / WM;
    const int r32 = lane & 31;
    const int h = lane >> 5;
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

    f32x16 acc[TMW][TNW];
#pragma unroll
    for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    // Wave-wide load j fills LDS rows RPL j .. RPL j + RPL - 1 of the stage
    // (halo rows first, then the tap-major weight rows tap * BN + column);
    // this wave issues j = wave + t * NW.  Lane L fills slot L % CPR of row
    // L / CPR, i.e. the chunk the swizzle puts there.  Sources are 32-bit
    // byte offsets from two block-uniform bases; halo rows outside the batch
    // and columns beyond n are clamped to valid ones (their outputs are
    // discarded by the epilogue).
    constexpr int NJ = XI + WI, JT = (NJ + NW - 1) / NW;
    const int lrow = lane / CPR, lpos = lane % CPR;
    const uint8_t* xbase = in + (m0 - RAD) * a.ld_in;
    const uint8_t* wbase = wt + (int64_t)n0 * kw;
    unsigned off[JT];
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = min(wave + t * NW, NJ - 1);
        const bool xj = j < XI;
        const int row = RPL * (xj ? j : j - XI) + lrow;
        const int c = lpos ^ swz<KB>(row);
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
            if (((t + 1) * NW <= NJ || j < NJ) && !(FC && j < XI))
                __builtin_amdgcn_global_load_lds((const void*)((j < XI ? xbase : wbase) + (off[t] + (unsigned)c0)),
                                                 (__attribute__((address_space(3))) void*)(base + 1024 * j), 16, 0, 0);
        }
    };

    const int nk = a.cin / KB;
    issue(0, 0);
    if constexpr (FC) {
        constexpr int HR = BM + TAPS - 1;              // halo rows the MFMAs read
        constexpr int GR = NT / CPR;                   // row groups: one per thread and 16-channel chunk
        constexpr int R = (HR + GR - 1) / GR;          // consecutive rows per thread
        if (wave == 0 && lane < KB * kTaps / 4)
            __builtin_amdgcn_global_load_lds((const void*)(a.first_w + 4 * lane),
                                             (__attribute__((address_space(3))) void*)fp, 16, 0, 0);
        if (wave == NW - 1 && lane < KB / 4)
            __builtin_amdgcn_global_load_lds((const void*)(a.first_b + 4 * lane),
                                             (__attribute__((address_space(3))) void*)(fp + 5 * KB), 16, 0, 0);
        if (wave == NW - 1 && lane < KB / 4)
            __builtin_amdgcn_global_load_lds((const void*)(a.first_inv_scale + 4 * lane),
                                             (__attribute__((address_space(3))) void*)(fp + 6 * KB), 16, 0, 0);
        const int q = tid % CPR, r0 = (tid / CPR) * R;
        float xw[R + kTaps - 1];
#pragma unroll
        for (int k = 0; k < R + kTaps - 1; ++k) {
            int64_t g = m0 - RAD + r0 + k - kGuard;
            g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
            xw[k] = a.first_x0[g];
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        const RowMap rmap(m0, a.r_in);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int r = r0 + u;
            if (r >= HR) break;
            int64_t g = m0 - RAD + r;
            g = g < 0 ? 0 : (g >= a.m_rows ? a.m_rows - 1 : g);
            int64_t e;
            int loc;
            rmap.at((int)(g - m0), e, loc);
            uint32_t w4[4] = {0u, 0u, 0u, 0u};
            if (loc >= kGuard && loc < a.r_in - kGuard) {
                // four codes per register, two per conversion (each code as
                // e4m3_sat gives it in the standalone kernel)
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    float y[4];
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const int c = 16 * q + 4 * p + k4;
                        float w5[kTaps];
#pragma unroll
                        for (int k = 0; k < kTaps; ++k) w5[k] = fp[c * kTaps + k];
                        const float act = first_conv_at(w5, fp[5 * KB + c], xw + u, a.slope);
                        y[k4] = fminf(fmaxf(act * fp[6 * KB + c], -448.f), 448.f);
                    }
                    uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                    w4[p] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], (int)w, true);
                }
            }
            *reinterpret_cast<u32x4*>(smem + r * KB + 16 * (q ^ swz<KB>(r))) = u32x4{w4[0], w4[1], w4[2], w4[3]};
        }
    }
    for (int k = 0; k < nk; ++k) {
        // this wave's loads of stage k have landed; the barrier makes every
        // wave's visible and (NB = 2) frees the other buffer (last read in
        // stage k - 1)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (NB == 2 && k + 1 < nk) issue((k + 1) & 1, (k + 1) * KB);
        const uint8_t* xs = smem + (NB == 2 ? (k & 1) : 0) * STAGE;
        const uint8_t* ws = xs + XR * KB;
        constexpr int FB = frag_bufs(NW, NB);
        i32x8 av[FB][TMW], bv[FB][TNW];
        // fragments of MFMA step p: this lane's slice 2 p + h (clamped; the
        // half past the last slice is zero)
        auto frag = [&](int p, int f) __attribute__((always_inline)) {
            const int s0 = 2 * p + h;
            const bool pad = s0 >= SL;
            const int s = pad ? SL - 1 : s0;
            const int sub = s / TAPS, tap = s - sub * TAPS;
#pragma unroll
            for (int i = 0; i < TMW; ++i) {
                const int r = wm * TMW * 32 + i * 32 + r32 + tap;
                const u32x4 lo = *reinterpret_cast<const u32x4*>(xs + r * KB + 16 * ((2 * sub) ^ swz<KB>(r)));
                const u32x4 hi = *reinterpret_cast<const u32x4*>(xs + r * KB + 16 * ((2 * sub + 1) ^ swz<KB>(r)));
                av[f][i] = pad ? i32x8{0, 0, 0, 0, 0, 0, 0, 0} : join(lo, hi);
            }
#pragma unroll
            for (int j = 0; j < TNW; ++j) {
                const int r = tap * BN + wn * TNW * 32 + j * 32 + r32;
                const u32x4 lo = *reinterpret_cast<const u32x4*>(ws + r * KB + 16 * ((2 * sub) ^ swz<KB>(r)));
                const u32x4 hi = *reinterpret_cast<const u32x4*>(ws + r * KB + 16 * ((2 * sub + 1) ^ swz<KB>(r)));
                bv[f][j] = pad ? i32x8{0, 0, 0, 0, 0, 0, 0, 0} : join(lo, hi);
            }
        };
        if constexpr (FB == 2) frag(0, 0);
#pragma unroll
        for (int p = 0; p < STEPS; ++p) {
            if constexpr (FB == 2) {
                if (p + 1 < STEPS) frag(p + 1, (p + 1) & 1);
            } else {
                frag(p, 0);
            }
            const int f = FB == 2 ? (p & 1) : 0;
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bv[f][j], av[f][i], acc[i][j], 0, 0,
                                                                                0, 0, 0, 0);
        }
        if (NB == 1 && k + 1 < nk) {
            __syncthreads();   // every wave is past its reads of the buffer
            issue(0, (k + 1) * KB);
        }
    }
    __syncthreads();   // the epilogue reuses the stage buffers

    // ---- epilogue
    const int rw = wm * TMW * 32;
    const int cw = wn * TNW * 32;
    const RowMap rows(m0, a.r_in);
    if constexpr (EPI == EPI_HEAD) {
        // logit = sum over channels of LeakyReLU(acc s_n + b_n) w_n; the two
        // lane halves hold the two halves of each block's channels
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < TNW; ++j)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = n0 + cw + j * 32 + 8 * g + 4 * h + v;
                        s += lrelu(acc[i][j][4 * g + v] * a.col_scale[c] + a.bias[c], a.slope) * a.head_w[c];
                    }
            s += __shfl_xor(s, 32);
            const int t = rw + i * 32 + r32;
            if (h == 0 && m0 + t < a.m_rows) {
                int64_t e;
                int loc;
                rows.at(t, e, loc);
                if (loc >= kGuard && loc < a.r_in - kGuard)
                    a.prob[e * a.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(s + a.head_b)));
            }
        }
        return;
    } else {
        uint8_t* ot = smem;   // [BM][OP] bytes
#pragma unroll
        for (int j = 0; j < TNW; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                // y / a_out = LeakyReLU(acc * s_n / a_out + b / a_out): one FMA
                // per value with the folded per-column factors (columns come in
                // groups of four, all valid or all past n)
                const int col = cw + j * 32 + 8 * g + 4 * h;
                const int nc = min(n0 + col, a.n - 4);
                const f32x4 fs = *reinterpret_cast<const f32x4*>(a.fold_scale + nc);
                const f32x4 fb = *reinterpret_cast<const f32x4*>(a.fold_bias + nc);
#pragma unroll
                for (int i = 0; i < TMW; ++i) {
                    float y[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        float x = fmaf(acc[i][j][4 * g + v], fs[v], fb[v]);
                        if (EPI != EPI_CONVT) x = lrelu(x, a.slope);
                        y[v] = fminf(fmaxf(x, -448.f), 448.f);   // saturate (the conversion maps overflow to NaN)
                    }
                    uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                    w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], (int)w, true);
                    *reinterpret_cast<uint32_t*>(ot + (rw + i * 32 + r32) * OP + col) = w;
                }
            }
        __syncthreads();
        if constexpr (EPI == EPI_UP) {
            // The transposed conv of the tile (BN == n: every channel of its
            // rows is here): per 64 channels one MFMA whose lane halves take
            // the two 32-channel chunks, weights in the A slot, as a
            // transposed-conv launch pairs them, so the bits are the same.
            // The tile holds the stored FP8 values (x / a_out), which the
            // transposed conv's weights were folded for.
            const uint8_t* uw = static_cast<const uint8_t*>(a.up_w);
            f32x16 up[TMW][TNW];
#pragma unroll
            for (int i = 0; i < TMW; ++i)
#pragma unroll
                for (int j = 0; j < TNW; ++j)
#pragma unroll
                    for (int v = 0; v < 16; ++v) up[i][j][v] = 0.f;
            for (int kk = 0; kk < BN; kk += 64) {
                i32x8 xv[TMW], wv[TNW];
#pragma unroll
                for (int i = 0; i < TMW; ++i) {
                    const uint8_t* r = ot + (rw + i * 32 + r32) * OP + kk + 32 * h;
                    xv[i] = join(*reinterpret_cast<const u32x4*>(r), *reinterpret_cast<const u32x4*>(r + 16));
                }
#pragma unroll
                for (int j = 0; j < TNW; ++j) {
                    const uint8_t* r = uw + (size_t)(cw + j * 32 + r32) * BN + kk + 32 * h;
                    wv[j] = join(*reinterpret_cast<const u32x4*>(r), *reinterpret_cast<const u32x4*>(r + 16));
                }
#pragma unroll
                for (int i = 0; i < TMW; ++i)
#pragma unroll
                    for (int j = 0; j < TNW; ++j)
                        up[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wv[j], xv[i], up[i][j], 0, 0, 0, 0,
                                                                                   0, 0);
            }
            __syncthreads();   // every wave is past its reads of the tile
            // folded scale and bias of the transposed conv, no activation
#pragma unroll
            for (int j = 0; j < TNW; ++j)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int col = cw + j * 32 + 8 * g + 4 * h;
                    const f32x4 fs = *reinterpret_cast<const f32x4*>(a.up_fold_scale + col);
                    const f32x4 fb = *reinterpret_cast<const f32x4*>(a.up_fold_bias + col);
#pragma unroll
                    for (int i = 0; i < TMW; ++i) {
                        float y[4];
#pragma unroll
                        for (int v = 0; v < 4; ++v) y[v] = fminf(fmaxf(fmaf(up[i][j][4 * g + v], fs[v], fb[v]), -448.f), 448.f);
                        uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                        w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], (int)w, true);
                        *reinterpret_cast<uint32_t*>(ot + (rw + i * 32 + r32) * OP + col) = w;
                    }
                }
            __syncthreads();
            // rows 2 t + tap of the destination, as a transposed-conv launch writes them
            uint8_t* uo = static_cast<uint8_t*>(a.up_out);
            constexpr int UCH = BN / 16;
            for (int idx = tid; idx < BM * UCH; idx += NT) {
                const int row = idx / UCH, q = idx % UCH;
                if (m0 + row >= a.m_rows) continue;
                int64_t e;
                int loc;
                rows.at(row, e, loc);
                if (loc < kGuard || loc >= a.r_in - kGuard) continue;
                const uint4 v = *reinterpret_cast<const uint4*>(ot + row * OP + 16 * q);
                const int tj = (16 * q) / a.up_cout, o = 16 * q - tj * a.up_cout;
                const int64_t ro = e * a.up_r_out + kGuard + 2 * (loc - kGuard) + tj;
                *reinterpret_cast<uint4*>(uo + ro * a.up_ld + o) = v;
            }
            return;
        }
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
                const uint4 q0 = *reinterpret_cast<const uint4*>(ot + (2 * pr) * OP + 16 * q);
                const uint4 q1 = *reinterpret_cast<const uint4*>(ot + (2 * pr + 1) * OP + 16 * q);
                const uint8_t* x0 = reinterpret_cast<const uint8_t*>(&q0);
                const uint8_t* x1 = reinterpret_cast<const uint8_t*>(&q1);
                uint8_t y[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) y[u] = e4m3_to_f32(x0[u]) >= e4m3_to_f32(x1[u]) ? x0[u] : x1[u];
                const int64_t rp = e * a.r_pool + kGuard + (loc - kGuard) / 2;
                *reinterpret_cast<uint4*>(pout + rp * a.ld_pool + n0 + 16 * q) = *reinterpret_cast<const uint4*>(y);
            }
        }
    }
}

// dec0.c1 and dec0.c2 + head in one launch (32 level-0 channels): the
// intermediate tensor stays in LDS as FP8.  A block of WM waves owns
// BO = 64 WM - 16 output rows from m0:
//   phase 1 runs dec0.c1 (64 input channels: one 64-channel stage) on the
//     BA = 64 WM rows from m0 - 2, in its standalone launch's slice order,
//     with its stored-output epilogue (folded scale and bias, LeakyReLU,
//     saturation, e4m3); rows that are guard rows or outside the batch are
//     zero, as in the stored tensor.  The codes go to LDS as a 32-channel
//     tile (32-byte rows, the 32-channel stage's swizzle) in the halo tile's
//     place;
//   phase 2 runs dec0.c2 and the head on that tile as the standalone head
//     launch runs them on its staged halo (32-channel stage: five slices, the
//     last MFMA's second half zero; same head epilogue), so every bit of p is
//     the same as from the two launches.
// Both stages and both weight tiles go straight into LDS (global_load_lds).
// c1: dec0.c1's arguments; c2: dec0.c2 + head's (in and ld_in unused).
template <int WM>
__global__ __launch_bounds__(WM * 64) __attribute__((amdgpu_waves_per_eu(4)))
void conv_mfma_fp8x64_dec0(ConvArgs c1, ConvArgs c2)
{
    constexpr int NW = WM;
    constexpr int BA = WM * 64;                   // phase-1 rows per block
    constexpr int BO = BA - 16;                   // output rows per block
    constexpr int K1 = 64, K2 = 32;               // row bytes of the two stages
    constexpr int XRA = (BA + kTaps - 1 + 15) / 16 * 16;   // halo rows, whole 1 KB loads of 64-byte rows
    constexpr int WR = kTaps * 32;                // weight rows (tap-major) of either conv
    constexpr int HALO = XRA * K1;
    __shared__ __attribute__((aligned(16))) uint8_t smem[HALO + WR * K1];
    uint8_t* const xs = smem;                     // phase 1: halo; phase 2: dec0.c1's tile (32-byte rows)
    uint8_t* const ws = smem + HALO;              // phase 1: dec0.c1's weights; phase 2: dec0.c2's

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r32 = lane & 31;
    const int h = lane >> 5;
    const int m_tiles = (int)((c2.m_rows + BO - 1) / BO);
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int m_tile = slot * kXcds + xcd;
    if (m_tile >= m_tiles) return;
    const int64_t m0 = (int64_t)m_tile * BO;
    const int64_t a0 = m0 - 2;                    // first phase-1 row

    // phase-1 loads: wave-wide load j fills 16 rows of 64 bytes (halo rows,
    // then the weight rows tap * 32 + column); lane L fills slot L % 4 of row
    // L / 4 with the chunk the swizzle puts there
    constexpr int NJ = XRA / 16 + WR / 16, JT = (NJ + NW - 1) / NW;
    const uint8_t* xbase = static_cast<const uint8_t*>(c1.in) + (a0 - 2) * c1.ld_in;
    const uint8_t* w1 = static_cast<const uint8_t*>(c1.w);
    const uint8_t* w2 = static_cast<const uint8_t*>(c2.w);
#pragma unroll
    for (int t = 0; t < JT; ++t) {
        const int j = wave + t * NW;
        if (!((t + 1) * NW <= NJ || j < NJ)) continue;
        const bool xj = j < XRA / 16;
        const int row = 16 * (xj ? j : j - XRA / 16) + (lane >> 2);
        const int c = (lane & 3) ^ swz<K1>(row);
        unsigned off;
        if (xj) {
            int64_t g = a0 - 2 + row;
            g = g < 0 ? 0 : (g >= c1.m_rows ? c1.m_rows - 1 : g);
            off = (unsigned)((g - (a0 - 2)) * c1.ld_in + 16 * c);
        } else {
            const int tap = row / 32, n = row % 32;
            off = (unsigned)(n * (kTaps * c1.cin) + tap * c1.cin + 16 * c);
        }
        __builtin_amdgcn_global_load_lds((const void*)((xj ? xbase : w1) + off),
                                         (__attribute__((address_space(3))) void*)(smem + 1024 * j), 16, 0, 0);
    }

    f32x16 acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;

    // ---- phase 1: ten (32-channel chunk, tap) slices, five MFMAs per block
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        const int sidx = 2 * p + h, sub = sidx / kTaps, tap = sidx - sub * kTaps;
        const int rw = tap * 32 + r32;
        const i32x8 bv = join(*reinterpret_cast<const u32x4*>(ws + rw * K1 + 16 * ((2 * sub) ^ swz<K1>(rw))),
                              *reinterpret_cast<const u32x4*>(ws + rw * K1 + 16 * ((2 * sub + 1) ^ swz<K1>(rw))));
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wave * 64 + i * 32 + r32 + tap;
            const i32x8 av = join(*reinterpret_cast<const u32x4*>(xs + r * K1 + 16 * ((2 * sub) ^ swz<K1>(r))),
                                  *reinterpret_cast<const u32x4*>(xs + r * K1 + 16 * ((2 * sub + 1) ^ swz<K1>(r))));
            acc[i] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bv, av, acc[i], 0, 0, 0, 0, 0, 0);
        }
    }
    __syncthreads();   // every wave is past its reads of the halo and of dec0.c1's weights
    // dec0.c2's weights (32-byte rows: 32 per 1 KB load, 2 slots per row)
#pragma unroll
    for (int t = 0; t < (WR / 32 + NW - 1) / NW; ++t) {
        const int j = wave + t * NW;
        if (j >= WR / 32) continue;
        const int row = 32 * j + (lane >> 1), tap = row / 32, n = row % 32;
        const int c = (lane & 1) ^ swz<K2>(row);
        __builtin_amdgcn_global_load_lds((const void*)(w2 + n * (kTaps * c2.cin) + tap * c2.cin + 16 * c),
                                         (__attribute__((address_space(3))) void*)(ws + 1024 * j), 16, 0, 0);
    }
    // dec0.c1's stored-output epilogue into the tile: row r is row a0 + r
    {
        const RowMap rmap(a0 < 0 ? 0 : a0, c1.r_in);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wave * 64 + i * 32 + r32;
            const int64_t g = a0 + r;
            bool keep = g >= 0 && g < c1.m_rows;
            if (keep) {
                int64_t e;
                int loc;
                rmap.at((int)(g - (a0 < 0 ? 0 : a0)), e, loc);
                keep = loc >= kGuard && loc < c1.r_in - kGuard;
            }
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                const int col = 8 * gq + 4 * h;
                const f32x4 fs = *reinterpret_cast<const f32x4*>(c1.fold_scale + col);
                const f32x4 fb = *reinterpret_cast<const f32x4*>(c1.fold_bias + col);
                float y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    y[v] = fminf(fmaxf(lrelu(fmaf(acc[i][4 * gq + v], fs[v], fb[v]), c1.slope), -448.f), 448.f);
                uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], (int)w, true);
                *reinterpret_cast<uint32_t*>(xs + r * K2 + 16 * ((col / 16) ^ swz<K2>(r)) + col % 16) = keep ? w : 0u;
            }
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // ---- phase 2: dec0.c2 on the tile (five slices, three MFMAs; rows BA ..
    // BA + 3 of the tile are stale and feed only outputs t >= BO)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int s0 = 2 * p + h;
        const bool pad = s0 >= kTaps;
        const int tap = pad ? kTaps - 1 : s0;
        const int rw = tap * 32 + r32;
        const i32x8 bv = pad ? i32x8{0, 0, 0, 0, 0, 0, 0, 0}
                             : join(*reinterpret_cast<const u32x4*>(ws + rw * K2 + 16 * (0 ^ swz<K2>(rw))),
                                    *reinterpret_cast<const u32x4*>(ws + rw * K2 + 16 * (1 ^ swz<K2>(rw))));
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wave * 64 + i * 32 + r32 + tap;
            const i32x8 av = pad ? i32x8{0, 0, 0, 0, 0, 0, 0, 0}
                                 : join(*reinterpret_cast<const u32x4*>(xs + r * K2 + 16 * (0 ^ swz<K2>(r))),
                                        *reinterpret_cast<const u32x4*>(xs + r * K2 + 16 * (1 ^ swz<K2>(r))));
            acc[i] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bv, av, acc[i], 0, 0, 0, 0, 0, 0);
        }
    }
    // head epilogue, as the standalone head launch's
    const RowMap rows(m0, c2.r_in);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float sum = 0.f;
#pragma unroll
        for (int gq = 0; gq < 4; ++gq)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 8 * gq + 4 * h + v;
                sum += lrelu(acc[i][4 * gq + v] * c2.col_scale[c] + c2.bias[c], c2.slope) * c2.head_w[c];
            }
        sum += __shfl_xor(sum, 32);
        const int t = wave * 64 + i * 32 + r32;
        if (h == 0 && t < BO && m0 + t < c2.m_rows) {
            int64_t e;
            int loc;
            rows.at(t, e, loc);
            if (loc >= kGuard && loc < c2.r_in - kGuard)
                c2.prob[e * c2.l_out + (loc - kGuard)] = 1.f / (1.f + expf(-(sum + c2.head_b)));
        }
    }
}

template <int WM, int WN, int TMW, int TNW, int KB, int TAPS, int EPI, int NB>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(occupancy_target(
    F8Lds<WM * TMW * 32, WN * TNW * 32, KB, TAPS, EPI, NB>::v, WM * WN, TMW, TNW, NB))))
void conv_mfma_fp8x64(ConvArgs a)
{
    fp8_tile<WM, WN, TMW, TNW, KB, TAPS, EPI, NB, false>(a);
}

template <int WM, int WN, int TMW, int TNW, int NB>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(occupancy_target(
    F8Lds<WM * TMW * 32, WN * TNW * 32, 32, kTaps, EPI_POOL, NB>::v, WM * WN, TMW, TNW, NB))))
void conv_mfma_fp8x64_first(ConvArgs a)
{
    fp8_tile<WM, WN, TMW, TNW, 32, kTaps, EPI_POOL, NB, true>(a);
}

template <int WM, int WN, int TMW, int TNW, int KB, int NB, int TAPS, int EPI>
hipError_t run(const ConvArgs& a, hipStream_t s)
{
    constexpr int BM = WM * TMW * 32;
    constexpr int BN = WN * TNW * 32;
    const unsigned m_tiles = (unsigned)((a.m_rows + BM - 1) / BM);
    const unsigned n_tiles = (unsigned)((a.n + BN - 1) / BN);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds * n_tiles);
    hipLaunchKernelGGL((conv_mfma_fp8x64<WM, WN, TMW, TNW, KB, TAPS, EPI, NB>), grid, dim3(WM * WN * 64), 0, s, a);
    return hipGetLastError();
}

// Tile variants: waves (WM x WN), 32 x 32 blocks per wave (TMW x TNW), stage
// width KB (fixed by the layer's input channels, so a layer's variants all
// give the same bits), LDS stage buffers NB.
struct Variant { int wm, wn, tmw, tnw, kb, nb; };
constexpr Variant kVariants[] = {
    {4, 1, 2, 1, 64, 2},   //  0: 256 x 32
    {4, 1, 2, 2, 64, 2},   //  1: 256 x 64
    {2, 2, 2, 2, 64, 2},   //  2: 128 x 128
    {4, 2, 2, 2, 64, 2},   //  3: 256 x 128 (512 threads)
    {8, 1, 2, 2, 64, 2},   //  4: 512 x 64 (512 threads)
    {2, 2, 2, 1, 64, 2},   //  5: 128 x 64, 64 x 32 per wave
    {2, 1, 2, 2, 64, 2},   //  6: 128 x 64 (128 threads)
    {2, 2, 4, 2, 64, 2},   //  7: 256 x 128, 128 x 64 per wave
    {4, 1, 4, 2, 64, 2},   //  8: 512 x 64, 128 x 64 per wave
    {4, 1, 2, 1, 32, 2},   //  9: 256 x 32, 32-channel stages
    {4, 1, 2, 2, 32, 2},   // 10: 256 x 64, 32-channel stages
    {8, 1, 2, 1, 32, 2},   // 11: 512 x 32, 32-channel stages
    {8, 1, 2, 2, 32, 2},   // 12: 512 x 64, 32-channel stages
    {2, 1, 2, 1, 32, 2},   // 13: 128 x 32, 32-channel stages (128 threads)
    {4, 1, 2, 2, 64, 1},   // 14: 256 x 64, single-buffered
    {4, 1, 2, 1, 64, 1},   // 15: 256 x 32, single-buffered
    {2, 2, 2, 2, 64, 1},   // 16: 128 x 128, single-buffered
    {4, 1, 2, 2, 32, 1},   // 17: 256 x 64, 32-channel stages, single-buffered
    {4, 1, 2, 1, 32, 1},   // 18: 256 x 32, 32-channel stages, single-buffered
    {2, 1, 2, 2, 64, 1},   // 19: 128 x 64, single-buffered (128 threads)
    {4, 1, 2, 1, 32, 3},   // 20: head launch with dec0.c1 fused (conv_mfma_fp8x64_dec0, 4 waves, 240 rows)
    {8, 1, 2, 1, 32, 3},   // 21: the same with 8 waves (496 rows)
    {8, 1, 2, 1, 32, 1},   // 22: 512 x 32, 32-channel stages, single-buffered
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define PVF_FP8_CASE(V)                                                                                          \
    case V:                                                                                                      \
        return run<kVariants[V].wm, kVariants[V].wn, kVariants[V].tmw, kVariants[V].tnw, kVariants[V].kb,      \
                   kVariants[V].nb, TAPS, EPI>(a, s);

template <int TAPS, int EPI>
hipError_t dispatch(int v, const ConvArgs& a, hipStream_t s)
{
    if constexpr (EPI == EPI_UP) {
        switch (v) {   // 64-channel stages, tiles of 64 or 128 columns
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(2)
            PVF_FP8_CASE(3)
            PVF_FP8_CASE(4)
            PVF_FP8_CASE(6)
            PVF_FP8_CASE(7)
            PVF_FP8_CASE(8)
            PVF_FP8_CASE(14)
            PVF_FP8_CASE(16)
            PVF_FP8_CASE(19)
        default: return hipErrorInvalidValue;
        }
    } else if constexpr (EPI == EPI_HEAD) {
        switch (v) {
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(4)
            PVF_FP8_CASE(6)
            PVF_FP8_CASE(8)
            PVF_FP8_CASE(9)
            PVF_FP8_CASE(10)
            PVF_FP8_CASE(11)
            PVF_FP8_CASE(12)
            PVF_FP8_CASE(13)
            PVF_FP8_CASE(14)
            PVF_FP8_CASE(15)
            PVF_FP8_CASE(17)
            PVF_FP8_CASE(18)
            PVF_FP8_CASE(19)
            PVF_FP8_CASE(22)
        default: return hipErrorInvalidValue;
        }
    } else if constexpr (TAPS == 1) {
        switch (v) {   // the transposed convolutions read 2 C >= 64 channels
            PVF_FP8_CASE(0)
            PVF_FP8_CASE(1)
            PVF_FP8_CASE(2)
            PVF_FP8_CASE(3)
            PVF_FP8_CASE(4)
            PVF_FP8_CASE(5)
            PVF_FP8_CASE(6)
            PVF_FP8_CASE(7)
            PVF_FP8_CASE(8)
            PVF_FP8_CASE(14)
            PVF_FP8_CASE(15)
            PVF_FP8_CASE(16)
            PVF_FP8_CASE(19)
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
            PVF_FP8_CASE(12)
            PVF_FP8_CASE(13)
            PVF_FP8_CASE(14)
            PVF_FP8_CASE(15)
            PVF_FP8_CASE(16)
            PVF_FP8_CASE(17)
            PVF_FP8_CASE(18)
            PVF_FP8_CASE(19)
            PVF_FP8_CASE(22)
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int fp8_variant_count() { return kNumVariants; }

bool fp8_variant_ok(int v, int n, int cin, int taps, Epi epi)
{
    if (v < 0 || v >= kNumVariants) return false;
    const Variant& x = kVariants[v];
    if (x.nb == 3) return epi == EPI_HEAD && n == 32 && cin == 32 && taps == kTaps;   // dec0 fused: 32-channel head
    const int bn = x.wn * x.tnw * 32;
    // the stage width follows the input channels: 64 when they allow it
    if (cin % 32 != 0 || (x.kb == 64) != (cin % 64 == 0)) return false;
    if (taps == 1 && x.kb != 64) return false;
    if (epi == EPI_HEAD)
        return x.wn == 1 && bn == n && (v == 0 || v == 1 || v == 4 || v == 6 || v == 8 || v >= 9);
    if (epi == EPI_UP)   // the tile must hold every channel of its rows
        return (v == 1 || v == 2 || v == 3 || v == 4 || v == 6 || v == 7 || v == 8 || v == 14 || v == 16 ||
                v == 19) &&
               bn == n && taps == 5;
    return bn <= n;
}

// Picks of the autotuner over 1000 events: the single-buffered tiles (more
// blocks per CU) on the 5-tap layers but the 32-channel head (enc0.c2: the
// single-buffered 256 x 32 tile that computes the first convolution), 256 x 64 (64 x 64 per wave) where the
// layer has 64 or more output channels, 256 x 32 or 128 x 32 where it has 32,
// 128 x 128 and 256 x 128 on the wide transposed convolutions; a decoder conv
// that runs the following transposed conv in its epilogue needs a tile of all
// its output channels: 256 x 64 for 64, 128 x 128 for 128.
int fp8_default_variant(int n, int cin, int taps, Epi epi)
{
    const bool k64 = cin % 64 == 0;
    if (epi == EPI_HEAD) return n == 64 ? (k64 ? 14 : 10) : (k64 ? 0 : 13);
    if (taps == 1) return n >= 256 ? 2 : (n >= 128 ? 3 : 0);
    if (n <= 32) return k64 ? 15 : (epi == EPI_POOL ? 18 : 9);
    return k64 ? 14 : 17;
}

int fp8_default_up_variant(int n, int cin)
{
    const int v = n == 64 ? 14 : (n == 128 ? 16 : -1);
    return v >= 0 && fp8_variant_ok(v, n, cin, kTaps, EPI_UP) ? v : -1;
}

std::string fp8_kernel_name(int v, int cin, int taps, Epi epi)
{
    (void)cin;
    const Variant& x = kVariants[v];
    if (x.nb == 3) return "conv_mfma_fp8x64_dec0<" + std::to_string(x.wm) + ">";
    return "conv_mfma_fp8x64<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " + std::to_string(x.tmw) +
           ", " + std::to_string(x.tnw) + ", " + std::to_string(x.kb) + ", " + std::to_string(taps) + ", " +
           std::to_string((int)epi) + ", " + std::to_string(x.nb) + ">";
}

bool fp8_dec0_ok(int v) { return v >= 0 && v < kNumVariants && kVariants[v].nb == 3; }

// enc0.c2 tiles that compute the first convolution in their staging: 32
// output columns and one 32-channel stage (the 32-channel network's level
// 0); the double-buffered 128- and 512-row tiles keep the standalone first
// convolution, so level 0 has a variant of each kind.
bool fp8_first_ok(int v) { return v == 9 || v == 18 || v == 22; }

std::string fp8_first_kernel_name(int v)
{
    const Variant& x = kVariants[v];
    return "conv_mfma_fp8x64_first<" + std::to_string(x.wm) + ", " + std::to_string(x.wn) + ", " +
           std::to_string(x.tmw) + ", " + std::to_string(x.tnw) + ", " + std::to_string(x.nb) + ">";
}

hipError_t launch_conv_fp8_first(const ConvArgs& a, int v, hipStream_t s)
{
    if (!fp8_first_ok(v) || a.m_rows <= 0 || a.cin != 32 || a.n != 32 || !a.first_x0 || !a.first_w || !a.first_b ||
        !a.first_inv_scale || !a.col_scale || !a.fold_scale || !a.fold_bias)
        return hipErrorInvalidValue;
    const int bm = kVariants[v].wm * 64;
    const unsigned m_tiles = (unsigned)((a.m_rows + bm - 1) / bm);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds);
    if (v == 9) hipLaunchKernelGGL((conv_mfma_fp8x64_first<4, 1, 2, 1, 2>), grid, dim3(256), 0, s, a);
    else if (v == 18) hipLaunchKernelGGL((conv_mfma_fp8x64_first<4, 1, 2, 1, 1>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((conv_mfma_fp8x64_first<8, 1, 2, 1, 1>), grid, dim3(512), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_conv_fp8_dec0(const ConvArgs& c1, const ConvArgs& c2, int v, hipStream_t s)
{
    if (!fp8_dec0_ok(v) || c1.cin != 64 || c1.n != 32 || c2.cin != 32 || c2.n != 32 || c1.m_rows != c2.m_rows ||
        c1.r_in != c2.r_in || c2.m_rows <= 0 || !c1.fold_scale || !c1.fold_bias || !c2.col_scale || !c2.prob ||
        !c2.head_w)
        return hipErrorInvalidValue;
    const int wm = kVariants[v].wm;
    const int bo = wm * 64 - 16;
    const unsigned m_tiles = (unsigned)((c2.m_rows + bo - 1) / bo);
    dim3 grid((m_tiles + kXcds - 1) / kXcds * kXcds);
    if (wm == 4) hipLaunchKernelGGL(conv_mfma_fp8x64_dec0<4>, grid, dim3(256), 0, s, c1, c2);
    else hipLaunchKernelGGL(conv_mfma_fp8x64_dec0<8>, grid, dim3(512), 0, s, c1, c2);
    return hipGetLastError();
}

hipError_t launch_conv_fp8(const ConvArgs& a, int taps, Epi epi, int v, hipStream_t s)
{
    if (a.cin % 32 != 0 || a.m_rows <= 0 || !fp8_variant_ok(v, a.n, a.cin, taps, epi) || !a.col_scale)
        return hipErrorInvalidValue;
    if (epi != EPI_HEAD && (!a.fold_scale || !a.fold_bias || a.n % 16 != 0)) return hipErrorInvalidValue;
    if (epi == EPI_CONVT && a.cout % 16 != 0) return hipErrorInvalidValue;
    if (epi == EPI_UP && (!a.up_w || !a.up_fold_scale || !a.up_fold_bias || !a.up_out || a.up_cout % 16 != 0 ||
                          2 * a.up_cout != a.n))
        return hipErrorInvalidValue;
    if (taps == 5) {
        switch (epi) {
        case EPI_STORE: return dispatch<5, EPI_STORE>(v, a, s);
        case EPI_POOL: return dispatch<5, EPI_POOL>(v, a, s);
        case EPI_HEAD: return dispatch<5, EPI_HEAD>(v, a, s);
        case EPI_UP: return dispatch<5, EPI_UP>(v, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (taps == 1 && epi == EPI_CONVT) return dispatch<1, EPI_CONVT>(v, a, s);
    return hipErrorInvalidValue;
}

}  // namespace pvf
