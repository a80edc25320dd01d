// BF16 MFMA implicit-GEMM convolutions (forward, data gradient, weight
// gradient) with FP32 accumulation for gfx950, plus the element-wise kernels
// of the surrogate network.
//
// Tensors are NHWC bf16 with C a multiple of 8; weights are [Co][kh][kw][Ci]
// (K = kh*kw*Ci contiguous per output channel).  One GEMM kernel template
// serves the three products:
//   forward   C[pixel][co]       = sum_k im2col(x)[pixel][k] * W[co][k]
//   data grad C[in pixel][ci]    = sum_k gather(dy)[in pixel][k] * WT[ci][k]
//                                  (k = (r, s, co); WT = [Ci][kh][kw][Co])
//   weight gr C[co][(r, s, ci)]  = sum_pixels dy[pixel][co] * x(shifted)[pixel][ci]
// A block tile (BM x BN) is built from 4 waves, each owning FM x FN tiles of
// v_mfma_f32_16x16x32_bf16.  The forward / data-gradient operands are
// contiguous along K: they go from global memory straight into a three-stage
// LDS ring by DMA (global_load_lds, 16 bytes a lane, two K steps ahead; no
// staging registers), in unpadded 64-byte rows whose 16-byte chunks are
// XOR-swizzled so the MFMA operand reads are free of bank conflicts.  Where the
// channel count is a multiple of 32 each K step is one tap's 32 channels, and
// the gather addresses are set once per tap.  The weight-gradient operands are
// contiguous along the channel (M / N) axis and are transposed into
// double-buffered LDS (rows padded to 80 bytes) through registers.  The weight
// gradient splits K (pixels) over blocks and sums the partial tiles in a fixed
// order (deterministic).
// A conv may read its input through a nearest-neighbour x2 upsampling
// (decoder layers): the gather maps (h, w) to (h / 2, w / 2).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstring>
#include <type_traits>

#include "surrogate_internal.h"

namespace sg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte staging chunk

constexpr int kThreads = 256;

// conv epilogue activation: 0 none, 1 ReLU, 2 leaky ReLU (slope kLeakySlope)
__device__ __forceinline__ float activate(float y, int act)
{
    if (act == 1) return fmaxf(y, 0.f);
    if (act == 2) return y > 0.f ? y : kLeakySlope * y;
    return y;
}
// the same with the activation known at compile time (epilogue loops instantiated per activation,
// so no per-element branch)
template <int ACT>
__device__ __forceinline__ float activate_c(float y)
{
    if constexpr (ACT == 1) return fmaxf(y, 0.f);
    else if constexpr (ACT == 2) return y > 0.f ? y : kLeakySlope * y;
    else return y;
}
constexpr int kBK = 32;           // K per MFMA step
constexpr int kBKP = kBK + 8;     // padded LDS row (bf16)

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
// two floats to packed bf16 (lo in bits 0..15) by the hardware conversion, round to nearest even:
// the bits of f2bf for finite inputs (checked on gfx950 over random finite patterns, exact ties,
// denormals and values next to the largest finite), one instruction for the pair
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    const f32x2v v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}
// bf16(a + b) for the two bf16 halves of each of two packed words
__device__ __forceinline__ uint32_t add_bf16x2(uint32_t a, uint32_t b)
{
    return pack_bf16x2(__uint_as_float(a << 16) + __uint_as_float(b << 16),
                       __uint_as_float(a & 0xFFFF0000u) + __uint_as_float(b & 0xFFFF0000u));
}

enum Mode { kFwd = 0, kDgrad = 1, kWgrad = 2 };

// LDS DMA operand rows are 64 bytes (four 16-byte K chunks) with no padding; K chunk q of row
// r sits in slot q ^ swz(r).  The 16 rows read by one MFMA operand load then put their chunks
// in 16 distinct 16-byte bank groups of 256 bytes (and any 8 consecutive rows in 8 of 128).
__device__ __forceinline__ int swz(int r) { return ((r >> 2) ^ (r >> 1)) & 3; }
// source of the DMA loads of padding and out-of-tile chunks (the DMA writes what it reads):
// 4096 bf16, so that a padding chunk can be advanced by any channel offset below C (C <= 4096)
__device__ __attribute__((aligned(16))) uint16_t g_zero_buf[4096];
// one 16-byte global -> LDS DMA load per lane: lane i of the wave writes dst_wave + 16 i, where
// dst_wave must be the same for the whole wave (it goes through M0).  A function of its own: the
// builtin called straight from a lambda inside a kernel template leaves that kernel without a
// host launch stub, with no diagnostic.
__device__ __forceinline__ void dma16(const uint16_t* src, uint16_t* dst_wave)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst_wave, 16, 0, 0);
}
// s_waitcnt immediate with expcnt and lgkmcnt at their maxima: OR in a vmcnt below 16
constexpr int kWaitVm0 = 0x0F70;

template <int MODE, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(kThreads) void k_conv_gemm(ConvGeom g0, ConvArgs a)
{
    ConvGeom g = g0;
    if (MODE == kDgrad && g0.par == 4) {   // parity class blockIdx.z of a stride-2 data gradient
        const int par = blockIdx.z, pa = par >> 1, pb = par & 1;
        g.par = par;
        g.Hc = g0.hc4[par];
        g.Wc = g0.wc4[par];
        g.f_hinwin = g0.f_hw4[par];
        g.f_win = g0.f_w4[par];
        g.M = (g0.Kw / ((int64_t)g0.Ho * g0.Wo)) * g.Hc * g.Wc;
        g.K = (pa + 1) * (pb + 1) * g0.Co;
        if ((int64_t)blockIdx.x * BM >= g.M) return;   // this class has fewer row tiles
    }
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile");
    // staged per K step: K-contiguous operands in (row, 8 k) 16-byte chunks
    // (one per register); the weight gradient's in tasks of 8 rows x 4 k, four
    // 16-byte (8 rows, k) chunks per task, transposed in registers into one
    // 8-byte (row, 4 k) LDS store per row
    constexpr int CA = (MODE == kWgrad) ? (BM / 8) * (kBK / 4) : BM * (kBK / 8);
    constexpr int CB = (MODE == kWgrad) ? (BN / 8) * (kBK / 4) : BN * (kBK / 8);
    constexpr int RPC = (MODE == kWgrad) ? 4 : 1;   // registers per chunk or task
    constexpr int PA = RPC * ((CA + kThreads - 1) / kThreads);
    constexpr int PB = RPC * ((CB + kThreads - 1) / kThreads);
    constexpr int AM8 = BM / 8, BN8 = BN / 8;   // weight-gradient row groups

    // operand tiles: the K-contiguous products fill a three-stage ring of unpadded 64-byte rows
    // straight from global memory (LDS DMA); the weight gradient double-buffers padded rows
    // through registers.  The forward epilogue reuses the space for its output tile.
    constexpr bool DMA = MODE != kWgrad;
    constexpr int NS = DMA ? 3 : 2, RL = DMA ? kBK : kBKP;   // stages, LDS row length
    constexpr int SMEM_OPS = NS * (BM + BN) * RL, SMEM_OUT = (MODE == kFwd) ? BM * (BN + 8) : 0;
    __shared__ __attribute__((aligned(16))) uint16_t smem[SMEM_OPS > SMEM_OUT ? SMEM_OPS : SMEM_OUT];
    uint16_t (*sA)[BM * RL] = reinterpret_cast<uint16_t (*)[BM * RL]>(smem);
    uint16_t (*sB)[BN * RL] = reinterpret_cast<uint16_t (*)[BN * RL]>(smem + NS * BM * RL);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int m_base = (int)blockIdx.x * BM;    // M < 2^31
    const int n_base = blockIdx.y * BN;
    const uint16_t* __restrict__ A = a.a;
    const uint16_t* __restrict__ B = a.b;
    const u32x4 zero = {0u, 0u, 0u, 0u};

    // K range of this block (split-K for the weight gradient)
    int64_t k_begin = 0, k_end = (MODE == kWgrad) ? g.Kw : g.K;
    if constexpr (MODE == kWgrad) {
        k_begin = (int64_t)blockIdx.z * a.k_chunk;
        k_end = min(k_end, k_begin + a.k_chunk);
    }
    const int nk = (int)((k_end - k_begin + kBK - 1) / kBK);
    const int Hin = g.up ? 2 * g.H : g.H, Win = g.up ? 2 * g.W : g.W;

    // ---- per-thread chunk bookkeeping, fixed over the K loop ----
    // K-contiguous modes: chunk c = tid + i * 256 -> LDS row c / 4, 16-byte slot c % 4, which holds
    // K chunk k8 = slot ^ swz(row); swz depends on row bits 1..3 only, so k8 is fixed per thread
    const int k8 = DMA ? (tid & 3) ^ swz(tid >> 2) : tid & 3;
    int a_hb[PA], a_wb[PA];       // forward: ho*s - pad, wo*s - pad; data grad: h + pad, w + pad
    int64_t a_base[PA];           // element offset of the row's image (or -1: row outside M)
    // weight gradient: fixed channel group of A (dy) and of B (x)
    const int wg_m0 = m_base + (tid % AM8) * 8;
    const int wg_n0 = n_base + (tid % BN8) * 8;
    int wg_r = 0, wg_s = 0, wg_ci0 = 0;
    if constexpr (MODE == kWgrad) {
        if (wg_n0 < g.N) {
            const int t = (int)fdiv((uint32_t)wg_n0, g.f_c);
            wg_ci0 = wg_n0 - t * g.C;
            wg_r = (int)fdiv((uint32_t)t, g.f_kw);
            wg_s = t - wg_r * g.kw;
        }
    } else {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int row = (tid >> 2) + i * (kThreads / 4);
            const int m = m_base + row;
            a_base[i] = -1;
            a_hb[i] = a_wb[i] = 0;
            if (row < BM && m < g.M) {
                if constexpr (MODE == kFwd) {
                    const int n = (int)fdiv((uint32_t)m, g.f_howo);
                    const int rem = m - n * g.Ho * g.Wo;
                    const int ho = (int)fdiv((uint32_t)rem, g.f_wo);
                    const int wo = rem - ho * g.Wo;
                    a_hb[i] = ho * g.stride - g.pad;
                    a_wb[i] = wo * g.stride - g.pad;
                    a_base[i] = (int64_t)n * g.H * g.W * g.C;
                } else {
                    // pixel (h, w) of image n; a parity class counts only its own pixels
                    const bool pc = g.par >= 0;
                    const int n = (int)fdiv((uint32_t)m, g.f_hinwin);
                    const int rem = m - n * (pc ? g.Hc * g.Wc : Hin * Win);
                    const int qh = (int)fdiv((uint32_t)rem, g.f_win);
                    const int qw = rem - qh * (pc ? g.Wc : Win);
                    const int h = pc ? 2 * qh + (g.par >> 1) : qh, w = pc ? 2 * qw + (g.par & 1) : qw;
                    a_hb[i] = h + g.pad;
                    a_wb[i] = w + g.pad;
                    a_base[i] = (int64_t)n * g.Ho * g.Wo * g.Co;
                }
            }
        }
    }

    u32x4 ra[PA], rb[PB];

    auto load_tiles = [&](int64_t k0) __attribute__((always_inline)) {
        if constexpr (MODE == kWgrad) {
#pragma unroll
            for (int i = 0; i < PA; ++i) {
                const int c = tid + (i / 4) * kThreads;   // task: rows wg_m0.., k = 4 (c / AM8) + i % 4
                const int64_t k = k0 + 4 * (c / AM8) + (i & 3);
                ra[i] = (c < CA && wg_m0 < g.M && k < k_end)
                            ? *reinterpret_cast<const u32x4*>(A + k * g.Co + wg_m0)
                            : zero;
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const int c = tid + (i / 4) * kThreads;
                const int64_t k = k0 + 4 * (c / BN8) + (i & 3);
                rb[i] = zero;
                if (c < CB && wg_n0 < g.N && k < k_end) {
                    const int p = (int)k;
                    const int n = (int)fdiv((uint32_t)p, g.f_howo);
                    const int rem = p - n * g.Ho * g.Wo;
                    const int ho = (int)fdiv((uint32_t)rem, g.f_wo);
                    const int wo = rem - ho * g.Wo;
                    int hi = ho * g.stride - g.pad + wg_r, wi = wo * g.stride - g.pad + wg_s;
                    if (hi >= 0 && wi >= 0 && hi < Hin && wi < Win) {
                        if (g.up) {
                            hi >>= 1;
                            wi >>= 1;
                        }
                        rb[i] = *reinterpret_cast<const u32x4*>(B + (((int64_t)n * g.H + hi) * g.W + wi) * g.C + wg_ci0);
                    }
                }
            }
            return;
        }
        // K-contiguous: one tap / channel split per K step (k8 fixed per thread)
        const int k = (int)k0 + k8 * 8;
        const bool kin = k < g.K;
        int r = 0, s = 0, c0 = 0, kf = k;   // kf: the column of B (all taps)
        if (kin) {
            const FastDiv fc = (MODE == kFwd) ? g.f_c : g.f_co;
            const int cc = (MODE == kFwd) ? g.C : g.Co;
            const int t = (int)fdiv((uint32_t)k, fc);
            c0 = k - t * cc;
            if (MODE == kDgrad && g.par >= 0) {
                // class taps: rows r in {1} (even h) or {0, 2} (odd h), columns s likewise, row-major
                const int pa = g.par >> 1, pb = g.par & 1;
                const int tr = pb ? t >> 1 : t, ts = pb ? t & 1 : 0;
                r = pa ? 2 * tr : 1;
                s = pb ? 2 * ts : 1;
                kf = (r * 3 + s) * cc + c0;
            } else {
                r = (int)fdiv((uint32_t)t, g.f_kw);
                s = t - r * g.kw;
            }
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            ra[i] = zero;
            if (!kin || a_base[i] < 0) continue;
            if constexpr (MODE == kFwd) {
                int hi = a_hb[i] + r, wi = a_wb[i] + s;
                if (hi < 0 || wi < 0 || hi >= Hin || wi >= Win) continue;
                if (g.up) {
                    hi >>= 1;
                    wi >>= 1;
                }
                ra[i] = *reinterpret_cast<const u32x4*>(A + a_base[i] + ((int64_t)hi * g.W + wi) * g.C + c0);
            } else {
                const int hh = a_hb[i] - r, ww = a_wb[i] - s;
                if (hh < 0 || ww < 0) continue;
                const int ho = (int)fdiv((uint32_t)hh, g.f_stride), wo = (int)fdiv((uint32_t)ww, g.f_stride);
                if (ho * g.stride != hh || wo * g.stride != ww || ho >= g.Ho || wo >= g.Wo) continue;
                ra[i] = *reinterpret_cast<const u32x4*>(A + a_base[i] + ((int64_t)ho * g.Wo + wo) * g.Co + c0);
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int col = n_base + (tid >> 2) + i * (kThreads / 4);
            rb[i] = (kin && (tid >> 2) + i * (kThreads / 4) < BN && col < g.N)
                        ? *reinterpret_cast<const u32x4*>(B + (int64_t)col * g.kb + kf)
                        : zero;
        }
    };
    // one stage of the LDS-DMA ring: each lane fetches its 16-byte chunk (a zero chunk where the
    // operand is padding or past the tile) into slot c of the stage; the 64 lanes of a wave fill
    // 64 consecutive slots, so the LDS address passed is the wave's first slot, a scalar.
    // The zero buffer's address is taken once (readfirstlane returns int: each half goes through
    // uint32_t, or the low half sign-extends).
    const uint64_t zp = reinterpret_cast<uint64_t>(g_zero_buf);
    const uint32_t zhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(zp >> 32));
    const uint32_t zlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)zp);
    const uint16_t* zsrc = reinterpret_cast<const uint16_t*>(((uint64_t)zhi << 32) | zlo);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const FastDiv fcc = (MODE == kFwd) ? g.f_c : g.f_co;
    const int cc = (MODE == kFwd) ? g.C : g.Co;   // channels of one tap along K
    // tap (r, s) of tap index t, and the column of B where the tap's channels start
    auto tap_of = [&](int t, int& r, int& s, int& kfb) __attribute__((always_inline)) {
        if (MODE == kDgrad && g.par >= 0) {
            // class taps: rows r in {1} (even h) or {0, 2} (odd h), columns s likewise, row-major
            const int pa = g.par >> 1, pb = g.par & 1;
            const int tr = pb ? t >> 1 : t, ts = pb ? t & 1 : 0;
            r = pa ? 2 * tr : 1;
            s = pb ? 2 * ts : 1;
            kfb = (r * 3 + s) * cc;
        } else {
            r = (int)fdiv((uint32_t)t, g.f_kw);
            s = t - r * g.kw;
            kfb = t * cc;
        }
    };
    // element offset of tap (r, s), channel c0, inside row i's image; false where it is padding
    auto a_tap = [&](int i, int r, int s, int c0, int& off) __attribute__((always_inline)) -> bool {
        if constexpr (MODE == kFwd) {
            const int hi = a_hb[i] + r, wi = a_wb[i] + s;
            off = ((hi >> g.up) * g.W + (wi >> g.up)) * g.C + c0;
            return a_base[i] >= 0 && (unsigned)hi < (unsigned)Hin && (unsigned)wi < (unsigned)Win;
        } else {
            const int hh = a_hb[i] - r, ww = a_wb[i] - s;
            const int ho = (int)fdiv((uint32_t)hh, g.f_stride), wo = (int)fdiv((uint32_t)ww, g.f_stride);
            off = (ho * g.Wo + wo) * g.Co + c0;
            return a_base[i] >= 0 && hh >= 0 && ww >= 0 && ho * g.stride == hh && wo * g.stride == ww &&
                   ho < g.Ho && wo < g.Wo;
        }
    };
    // general K steps (C not a multiple of 32: a step's chunks may fall in different taps, or past K)
    auto issue_stage = [&](int64_t k0, int st) __attribute__((always_inline)) {
        const int k = (int)k0 + k8 * 8;
        const bool kin = k < g.K;
        int r = 0, s = 0, c0 = 0, kf = k;
        if (kin) {
            const int t = (int)fdiv((uint32_t)k, fcc);
            c0 = k - t * cc;
            int kfb;
            tap_of(t, r, s, kfb);
            kf = kfb + c0;
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            if (wv * 64 + i * kThreads >= CA) continue;   // CA is a multiple of 64
            int off;
            const bool ok = a_tap(i, r, s, c0, off) && kin;
            dma16(ok ? A + a_base[i] + off : zsrc, &sA[st][(wv * 64 + i * kThreads) * 8]);
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            if (wv * 64 + i * kThreads >= CB) continue;
            const int col = n_base + ((tid + i * kThreads) >> 2);
            dma16((kin && col < g.N) ? B + (int64_t)col * g.kb + kf : zsrc, &sB[st][(wv * 64 + i * kThreads) * 8]);
        }
    };
    // tap steps (C a multiple of 32: each K step is 32 channels of one tap, and K = nk * 32): the
    // chunk pointers are set once per tap (pointing at channel 0 plus this lane's 8 k, or into the
    // zero buffer) and a step adds its channel offset
    const uint16_t* tpa[PA];
    const uint16_t* tpb[PB];
    int cur_t = -1;
    auto issue_tap = [&](int64_t k0, int st) __attribute__((always_inline)) {
        const int t = (int)fdiv((uint32_t)k0, fcc);
        const int c0 = (int)k0 - t * cc;
        if (t != cur_t) {
            cur_t = t;
            int r, s, kfb;
            tap_of(t, r, s, kfb);
#pragma unroll
            for (int i = 0; i < PA; ++i) {
                if (wv * 64 + i * kThreads >= CA) continue;
                int off;
                const bool ok = a_tap(i, r, s, 0, off);
                tpa[i] = (ok ? A + a_base[i] + off : zsrc) + k8 * 8;
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                if (wv * 64 + i * kThreads >= CB) continue;
                const int col = n_base + ((tid + i * kThreads) >> 2);
                tpb[i] = (col < g.N ? B + (int64_t)col * g.kb + kfb : zsrc) + k8 * 8;
            }
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            if (wv * 64 + i * kThreads >= CA) continue;
            dma16(tpa[i] + c0, &sA[st][(wv * 64 + i * kThreads) * 8]);
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            if (wv * 64 + i * kThreads >= CB) continue;
            dma16(tpb[i] + c0, &sB[st][(wv * 64 + i * kThreads) * 8]);
        }
    };
    const bool tap_steps = cc % kBK == 0;
    auto issue = [&](int64_t k0, int st) __attribute__((always_inline)) {
        if (tap_steps) issue_tap(k0, st);
        else issue_stage(k0, st);
    };
    // four (8 rows, k) chunks of consecutive k -> row j's 4 k as one 8-byte value
    auto transpose_store = [&](uint16_t* dst, const u32x4* r, int row0, int kk) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int w = j >> 1;
            const uint32_t lo = (j & 1) ? ((r[0][w] >> 16) | (r[1][w] & 0xFFFF0000u))
                                        : ((r[0][w] & 0xFFFFu) | (r[1][w] << 16));
            const uint32_t hi = (j & 1) ? ((r[2][w] >> 16) | (r[3][w] & 0xFFFF0000u))
                                        : ((r[2][w] & 0xFFFFu) | (r[3][w] << 16));
            *reinterpret_cast<uint2*>(&dst[(row0 + j) * kBKP + kk]) = make_uint2(lo, hi);
        }
    };
    auto store_tiles = [&](int buf) __attribute__((always_inline)) {
        if constexpr (MODE == kWgrad) {
#pragma unroll
            for (int i = 0; i < PA / 4; ++i) {
                const int c = tid + i * kThreads;
                if (c < CA) transpose_store(sA[buf], ra + 4 * i, (c % AM8) * 8, 4 * (c / AM8));
            }
#pragma unroll
            for (int i = 0; i < PB / 4; ++i) {
                const int c = tid + i * kThreads;
                if (c < CB) transpose_store(sB[buf], rb + 4 * i, (c % BN8) * 8, 4 * (c / BN8));
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int c = tid + i * kThreads;
            if (c >= CA) continue;
            *reinterpret_cast<u32x4*>(&sA[buf][(c >> 2) * kBKP + k8 * 8]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int c = tid + i * kThreads;
            if (c >= CB) continue;
            *reinterpret_cast<u32x4*>(&sB[buf][(c >> 2) * kBKP + k8 * 8]) = rb[i];
        }
    };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the forward epilogue's bias, read once here (in the epilogue a load after a possibly
    // aliasing store would be repeated, each waiting for memory)
    float bias_r[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = n_base + wn * TN + j * 16 + (lane & 15);
        bias_r[j] = (MODE == kFwd && a.bias && col < g.N) ? a.bias[col] : 0.f;
    }

    const int frow = lane & 15, fk = (lane >> 4) * 8;
    if constexpr (DMA) {
        // a wave waits for its own DMA of stage kt (vmcnt counts in issue order: at most the next
        // stage's loads may remain), then the barrier makes every wave's chunks visible and
        // retires the reads of the stage the next issue overwrites.  LW is the fewest DMA loads
        // any wave issues per stage (wave 3's, whose first chunk is 192); a wave with more waits
        // for part of the next stage too.  The barrier is the bare s_barrier: __syncthreads()
        // would add a wait for every outstanding load (vmcnt(0)) and drain the ring; the empty
        // asm statements keep the compiler from moving LDS accesses across it.
        constexpr int LW = ((CA - 192 + kThreads - 1) / kThreads) + (CB > 192 ? (CB - 192 + kThreads - 1) / kThreads : 0);
        static_assert(LW >= 1 && LW < 16, "per-wave DMA loads per stage");
        const int rd = frow * kBK + (((lane >> 4) ^ swz(frow)) * 8);
        if (nk > 0) issue(k_begin, 0);
        if (nk > 1) issue(k_begin + kBK, 1);
        for (int kt = 0; kt < nk; ++kt) {
            const int st = kt % 3;
            if (kt + 1 < nk) __builtin_amdgcn_s_waitcnt(kWaitVm0 | LW);
            else __builtin_amdgcn_s_waitcnt(kWaitVm0);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (kt + 2 < nk) issue(k_begin + (int64_t)(kt + 2) * kBK, (kt + 2) % 3);
            bf16x8 fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                fa[i] = *reinterpret_cast<const bf16x8*>(&sA[st][(wm * TM + i * 16) * kBK + rd]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                fb[j] = *reinterpret_cast<const bf16x8*>(&sB[st][(wn * TN + j * 16) * kBK + rd]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
    } else {
    if (nk > 0) {
        load_tiles(k_begin);
        store_tiles(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_tiles(k_begin + (int64_t)(kt + 1) * kBK);
        bf16x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            fa[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][(wm * TM + i * 16 + frow) * RL + fk]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            fb[j] = *reinterpret_cast<const bf16x8*>(&sB[buf][(wn * TN + j * 16 + frow) * RL + fk]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) store_tiles(buf ^ 1);
        __syncthreads();
    }
    }

    // epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each tile
    if constexpr (MODE == kFwd) {
        // the bf16 outputs go through an LDS tile [BM][BN + 8] to 16-byte stores; the skip tensor's
        // chunks are all loaded before the first store (a load issued after a store waits for it:
        // one memory round trip per element otherwise)
        constexpr int TP = BN + 8;
        uint16_t* sT = smem;
        __syncthreads();   // every wave is done with the operand tiles
        // (one instantiation per activation; a lane's rows r, r + 1 share one bf16 conversion)
        auto write_tile = [&](auto act_c) __attribute__((always_inline)) {
            constexpr int ACT = decltype(act_c)::value;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int cl = wn * TN + j * 16 + (lane & 15), col = n_base + cl;
#pragma unroll
                    for (int r = 0; r < 4; r += 2) {
                        const int rl = wm * TM + i * 16 + (lane >> 4) * 4 + r;
                        const float y0 = activate_c<ACT>(acc[i][j][r] + bias_r[j]);
                        const float y1 = activate_c<ACT>(acc[i][j][r + 1] + bias_r[j]);
                        const uint32_t pk = pack_bf16x2(y0, y1);
                        sT[rl * TP + cl] = (uint16_t)pk;
                        sT[(rl + 1) * TP + cl] = (uint16_t)(pk >> 16);
                        if (a.out_f32) {
                            const int64_t row = (int64_t)m_base + rl;
                            if (row < g.M && col < g.N) a.out_f32[row * g.Co + col] = y0;
                            if (row + 1 < g.M && col < g.N) a.out_f32[(row + 1) * g.Co + col] = y1;
                        }
                    }
                }
        };
        if (a.relu == 1) write_tile(std::integral_constant<int, 1>{});
        else if (a.relu == 2) write_tile(std::integral_constant<int, 2>{});
        else write_tile(std::integral_constant<int, 0>{});
        __syncthreads();
        constexpr int CH = BM * BN / 8, CPT = (CH + kThreads - 1) / kThreads;   // 16-byte chunks
        const int ld2 = a.ld_out2 ? a.ld_out2 : g.Co;
        // chunk u of this thread: tile row rl, columns 8 c8.. (Co is a multiple of 8, so a chunk is
        // wholly inside or past column N); separate loops with and without the skip tensor, so the
        // stores of the plain one wait for no load
        if (a.skip && a.out2_bf16) {
            u32x4 kv[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = tid + u * kThreads, rl = c / (BN / 8), c8 = c % (BN / 8);
                const int64_t row = (int64_t)m_base + rl;
                const int col = n_base + c8 * 8;
                kv[u] = (c < CH && row < g.M && col < g.N)
                            ? *reinterpret_cast<const u32x4*>(a.skip + row * g.Co + col)
                            : zero;
            }
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = tid + u * kThreads, rl = c / (BN / 8), c8 = c % (BN / 8);
                const int64_t row = (int64_t)m_base + rl;
                const int col = n_base + c8 * 8;
                if (c >= CH || row >= g.M || col >= g.N) continue;
                const u32x4 v = *reinterpret_cast<const u32x4*>(&sT[rl * TP + c8 * 8]);
                if (a.out_bf16) *reinterpret_cast<u32x4*>(a.out_bf16 + row * g.Co + col) = v;
                u32x4 o;
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q] = add_bf16x2(v[q], kv[u][q]);
                *reinterpret_cast<u32x4*>(a.out2_bf16 + row * ld2 + col) = o;
            }
        } else if (a.out_bf16) {
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = tid + u * kThreads, rl = c / (BN / 8), c8 = c % (BN / 8);
                const int64_t row = (int64_t)m_base + rl;
                const int col = n_base + c8 * 8;
                if (c >= CH || row >= g.M || col >= g.N) continue;
                *reinterpret_cast<u32x4*>(a.out_bf16 + row * g.Co + col) =
                    *reinterpret_cast<const u32x4*>(&sT[rl * TP + c8 * 8]);
            }
        }
        return;
    }
    // data and weight gradients: FP32 straight from the accumulators.  Output pixel of row r of row
    // tile i (a parity class's rows are a quarter of the pixels), -1 past the last row:
    auto pixel = [&](int i, int r) __attribute__((always_inline)) -> int64_t {
        const int64_t row = (int64_t)m_base + wm * TM + i * 16 + (lane >> 4) * 4 + r;
        if (row >= g.M) return -1;
        if constexpr (MODE == kDgrad) {
            if (g.par >= 0) {
                const int n = (int)fdiv((uint32_t)row, g.f_hinwin);
                const int rem = (int)row - n * g.Hc * g.Wc;
                const int qh = (int)fdiv((uint32_t)rem, g.f_win);
                const int qw = rem - qh * g.Wc;
                return ((int64_t)n * g.H + 2 * qh + (g.par >> 1)) * g.W + 2 * qw + (g.par & 1);
            }
        }
        return row;
    };
    if (MODE == kDgrad && a.accumulate) {
        // per row tile, the old values are all loaded before the tile's first store (a load issued
        // after a store waits for it)
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            int64_t px[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) px[r] = pixel(i, r);
            float pre[FN][4];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = n_base + wn * TN + j * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    pre[j][r] = (col < g.N && px[r] >= 0) ? a.out_f32[px[r] * g.C + col] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = n_base + wn * TN + j * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (col < g.N && px[r] >= 0) a.out_f32[px[r] * g.C + col] = pre[j][r] + acc[i][j][r];
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t px = pixel(i, r);
            if (px < 0) continue;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = n_base + wn * TN + j * 16 + (lane & 15);
                if (col >= g.N) continue;
                if constexpr (MODE == kDgrad)
                    a.out_f32[px * g.C + col] = acc[i][j][r];
                else
                    a.out_f32[(int64_t)blockIdx.z * g.M * g.N + px * g.N + col] = acc[i][j][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Direct 3x3 convolution (stride 1, pad 1) for few channels.  A block of TH / 2
// waves computes a TH x 32 pixel output tile of one image for all CO output
// channels.  The
// input tile with its one-pixel halo ((TH + 2) x 34 pixels, zero outside the image;
// with upsampling, fine pixel (h, w) reads stored pixel (h / 2, w / 2)) and
// all weights are staged in LDS once (by DMA, every chunk in flight at once),
// and the MFMA operands are read from there, so each input pixel leaves global
// memory once per tile instead of once per tap.  LDS pixel and weight rows are odd multiples of 16 bytes, so
// the 16-byte operand reads of a wave are free of bank conflicts.  The output
// tile is staged through LDS for 16-byte stores; the skip sum and a 1x1 head
// with one output can be fused.
// 16 x 32 tiles (eight waves): against 8 x 32 ones, the weights staged per
// block serve twice the pixels and the halo adds 1/8 instead of 1/4 of the
// input rows (the 1024-frame forward's tiled layers took 3.3 instead of
// 3.6 ms; 32-row tiles were slower again)
constexpr int kTileH = 16, kTileW = 32;

template <int C, int CO, bool UP, bool DIL = false, bool ACC = false, int TH = kTileH>
__global__ __launch_bounds__(32 * TH) void k_conv3x3_tile(ConvGeom g, ConvArgs a)
{
    // DIL: the input is dy of a stride-2 conv dilated by zeros: virtual pixel (h, w) is stored pixel
    // (h / 2, w / 2) when both are even, else 0 (the data gradient of that conv as a stride-1 conv)
    // UP: the input is read upsampled x2; the tile stages the stored pixels it
    // covers (fine halo pixel (hy, wx) of the (TH + 2) x 34 window is stored pixel
    // ((hy + 1) / 2, (wx + 1) / 2) of a (TH / 2 + 2) x 18 window, tile origins being even)
    constexpr int NT = 32 * TH;   // threads: TH / 2 waves of two output rows each
    constexpr int HP = UP ? TH / 2 + 2 : TH + 2, WP = UP ? kTileW / 2 + 2 : kTileW + 2;
    constexpr int C8 = C / 8;
    constexpr int PS = (C8 % 2 == 0) ? C + 8 : C;   // LDS pixel stride (bf16)
    constexpr int K8 = 9 * C8;                       // 8-wide K groups
    constexpr int NKS = (K8 + 3) / 4;                // MFMA K steps of 32
    constexpr int KP = NKS * 32 + 8;                 // LDS weight row (bf16), zero beyond K
    constexpr int FN = CO / 16;
    constexpr int CO8 = CO / 8;
    // staged by LDS DMA in 16-byte slots, whole waves at a time: the regions are rounded up to
    // 64 slots (512 bf16), the slots past the data (and the pad slot of each pixel and weight
    // row) filled from the zero buffer
    constexpr int SPP = PS / 8, KPS = KP / 8;        // slots per staged pixel, per weight row
    constexpr int NXS = HP * WP * SPP, NWS = CO * KPS;
    constexpr int XS = (NXS + 63) / 64 * 512, OS = TH * kTileW * CO;
    __shared__ __attribute__((aligned(16))) uint16_t sX[XS > OS ? XS : OS];
    __shared__ __attribute__((aligned(16))) uint16_t sW[(NWS + 63) / 64 * 512];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int tiles_x = (g.Wo + kTileW - 1) / kTileW, tiles_y = (g.Ho + TH - 1) / TH;
    // neighbouring tiles on the same XCD (blocks are dealt round-robin over 8)
    int64_t b = blockIdx.x;
    const int64_t nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int64_t per_img = (int64_t)tiles_x * tiles_y;
    const int64_t n = b / per_img;
    const int t_in = (int)(b - n * per_img);
    const int ty = t_in / tiles_x, tx = t_in - ty * tiles_x;
    const int ho0 = ty * TH, wo0 = tx * kTileW;
    const int Hin = g.up ? 2 * g.H : g.H, Win = g.up ? 2 * g.W : g.W;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    // the epilogue's bias, read here, where its latency overlaps the staging (in the epilogue a
    // load after a possibly aliasing store would be repeated, each waiting for memory)
    float bias_r[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) bias_r[j] = a.bias ? a.bias[16 * j + lr] : 0.f;

    // staging: every slot of the halo tile and of the weights is one DMA load, all in flight
    // together (no staging registers); halo slot j is pixel j / SPP, channel group j % SPP (the
    // pad group where that is C8), weight slot j is row j / KPS, K group j % KPS
    const uint64_t zp = reinterpret_cast<uint64_t>(g_zero_buf);
    const uint32_t zhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(zp >> 32));
    const uint32_t zlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)zp);
    const uint16_t* zsrc = reinterpret_cast<const uint16_t*>(((uint64_t)zhi << 32) | zlo);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // (each source is one select between the operand and the zero buffer, computed without early
    // returns: with divergent returns the compiler reused the zero pointer's register on the
    // padding lanes' path and those lanes loaded from a garbage address)
    auto x_src = [&](int j) __attribute__((always_inline)) -> const uint16_t* {
        const int pix = j / SPP, c8 = j - pix * SPP;
        const int hy = pix / WP, wx = pix - hy * WP;
        bool ok = j < NXS && c8 < C8;
        int hi, wi;
        if constexpr (UP) {   // stored pixels (ho0 / 2 - 1 + hy, wo0 / 2 - 1 + wx), zero outside
            hi = ho0 / 2 - 1 + hy;
            wi = wo0 / 2 - 1 + wx;
            ok = ok && (unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W;
        } else if constexpr (DIL) {
            const int h2 = ho0 - 1 + hy, w2 = wo0 - 1 + wx;
            ok = ok && h2 >= 0 && w2 >= 0 && !(h2 & 1) && !(w2 & 1) && (h2 >> 1) < g.H && (w2 >> 1) < g.W;
            hi = h2 >> 1;
            wi = w2 >> 1;
        } else {
            const int h2 = ho0 - 1 + hy, w2 = wo0 - 1 + wx;
            ok = ok && (unsigned)h2 < (unsigned)Hin && (unsigned)w2 < (unsigned)Win;
            hi = h2 >> g.up;
            wi = w2 >> g.up;
        }
        const int64_t off = ((n * g.H + hi) * g.W + wi) * C + c8 * 8;
        return ok ? a.a + off : zsrc;
    };
    auto w_src = [&](int j) __attribute__((always_inline)) -> const uint16_t* {
        const int co = j / KPS, k8 = j - co * KPS;
        // k8 = tap * C8 + channel group; mirrored: tap 8 - tap of the transposed copy
        const int ks = a.flip ? (8 - k8 / C8) * C8 + k8 % C8 : k8;
        return (j < NWS && k8 < K8) ? a.b + (int64_t)co * (9 * C) + ks * 8 : zsrc;
    };
#pragma unroll
    for (int u = 0; u < (NWS + NT - 1) / NT; ++u) {
        const int base = wv * 64 + NT * u;   // first slot of this wave's load
        if (base < NWS) dma16(w_src(base + lane), &sW[base * 8]);
    }
#pragma unroll
    for (int u = 0; u < (NXS + NT - 1) / NT; ++u) {
        const int base = wv * 64 + NT * u;
        if (base < NXS) dma16(x_src(base + lane), &sX[base * 8]);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();

    f32x4 acc[4][FN];
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[gi][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // operand of row group gi (output rows rr = 2 wave + gi / 2, columns cc = 16 (gi % 2) + lr) at
    // tap (r, s): staged pixel (sy, sx) = (rr + r, cc + s), or with UP ((rr + r + 1) / 2,
    // (cc + s + 1) / 2) = (wave + (gi / 2 + r + 1) / 2, 8 (gi % 2) + lr / 2 + (lr % 2 + s + 1) / 2).
    // Either way the LDS offset is a per-lane part fixed over the K loop plus a per-step part that
    // depends on gi only through gi / 2.
    int gofs[4];
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
        gofs[gi] = UP ? (wave * WP + (gi & 1) * 8 + (lr >> 1)) * PS
                      : ((2 * wave + (gi >> 1)) * WP + (gi & 1) * 16 + lr) * PS;
#pragma unroll 3
    for (int ks = 0; ks < NKS; ++ks) {
        const int k8 = ks * 4 + lk;
        int r = 0, s = 0, c0 = 0;
        if (k8 < K8) {   // beyond K the weights are zero; read tap 0
            const int tap = k8 / C8;
            c0 = (k8 - tap * C8) * 8;
            r = tap / 3;
            s = tap - r * 3;
        }
        int tofs[2];
        if constexpr (UP) {
            const int sxo = ((lr & 1) + s + 1) >> 1;
            tofs[0] = (((r + 1) >> 1) * WP + sxo) * PS + c0;
            tofs[1] = (((r + 2) >> 1) * WP + sxo) * PS + c0;
        } else {
            tofs[0] = tofs[1] = (r * WP + s) * PS + c0;
        }
        bf16x8 fb[FN];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = *reinterpret_cast<const bf16x8*>(&sW[(16 * j + lr) * KP + k8 * 8]);
#pragma unroll
        for (int gi = 0; gi < 4; ++gi) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&sX[gofs[gi] + tofs[gi >> 1]]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[gi][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[gi][j], 0, 0, 0);
        }
    }
    __syncthreads();   // sX is reused for the output tile

    uint16_t* sO = sX;   // [TH * kTileW][CO]
    const bool pool = a.out_f32 && a.pool2;
    if (pool) {
        // data gradient of an upsampled input: each 2 x 2 output block summed into one pixel of the
        // half-size out_f32, as (top pair) + (bottom pair).  Wave w holds output rows 2 w (row tile
        // gi = h) and 2 w + 1 (gi = h + 2) of column half h; a lane the column pairs (q, q + 1), q = 0, 2.
        const int Hc = g.Ho >> 1, Wc = g.Wo >> 1, hc = (ho0 >> 1) + wave;
        float pv[ACC ? FN : 1][2][2];   // ACC: the old values, all loaded before the stores
        if constexpr (ACC) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int pr = 0; pr < 2; ++pr) {
                        const int wc = ((wo0 + h * 16 + 4 * lk) >> 1) + pr;
                        pv[j][h][pr] = (hc < Hc && wc < Wc) ? a.out_f32[((n * Hc + hc) * Wc + wc) * CO + 16 * j + lr]
                                                            : 0.f;
                    }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int pr = 0; pr < 2; ++pr) {
                    const int wc = ((wo0 + h * 16 + 4 * lk) >> 1) + pr;
                    const float y00 = activate(acc[h][j][2 * pr] + bias_r[j], a.relu);
                    const float y01 = activate(acc[h][j][2 * pr + 1] + bias_r[j], a.relu);
                    const float y10 = activate(acc[h + 2][j][2 * pr] + bias_r[j], a.relu);
                    const float y11 = activate(acc[h + 2][j][2 * pr + 1] + bias_r[j], a.relu);
                    float sum = (y00 + y01) + (y10 + y11);
                    if constexpr (ACC) sum = pv[j][h][pr] + sum;
                    if (hc < Hc && wc < Wc) a.out_f32[((n * Hc + hc) * Wc + wc) * CO + 16 * j + lr] = sum;
                }
    }
    // (one instantiation of the loop per activation; two outputs of a lane, neighbouring pixels of
    // one channel, share one bf16 conversion)
    auto write_tile = [&](auto act_c) __attribute__((always_inline)) {
        constexpr int ACT = decltype(act_c)::value;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        const int rr = 2 * wave + (gi >> 1), ho = ho0 + rr;
        // ACC (an FP32 output accumulated into, a.accumulate): the old values of this row group,
        // all loaded before its stores (a load issued after a store waits for it)
        float prev[ACC ? FN : 1][4];
        if constexpr (ACC) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int wo = wo0 + (gi & 1) * 16 + 4 * lk + q;
                    prev[j][q] = (!pool && ho < g.Ho && wo < g.Wo)
                                     ? a.out_f32[((n * g.Ho + ho) * g.Wo + wo) * CO + 16 * j + lr]
                                     : 0.f;
                }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int co = 16 * j + lr;
#pragma unroll
            for (int q = 0; q < 4; q += 2) {
                const int cc = (gi & 1) * 16 + 4 * lk + q;
                const float y0 = activate_c<ACT>(acc[gi][j][q] + bias_r[j]);
                const float y1 = activate_c<ACT>(acc[gi][j][q + 1] + bias_r[j]);
                const uint32_t pk = pack_bf16x2(y0, y1);
                sO[(rr * kTileW + cc) * CO + co] = (uint16_t)pk;
                sO[(rr * kTileW + cc + 1) * CO + co] = (uint16_t)(pk >> 16);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int wo = wo0 + cc + t;
                    if (a.out_f32 && !pool && ho < g.Ho && wo < g.Wo) {
                        float yo = t ? y1 : y0;
                        if constexpr (ACC) yo = prev[j][q + t] + yo;
                        a.out_f32[((n * g.Ho + ho) * g.Wo + wo) * CO + co] = yo;
                    }
                }
            }
        }
    }
    };
    if (a.relu == 1) write_tile(std::integral_constant<int, 1>{});
    else if (a.relu == 2) write_tile(std::integral_constant<int, 2>{});
    else write_tile(std::integral_constant<int, 0>{});
    __syncthreads();
    const int ld2 = a.ld_out2 ? a.ld_out2 : CO;
    // 16-byte output chunks: thread tid takes chunks tid + NT u; the skip tensor's chunks are all
    // loaded before the first store
    static_assert(TH * kTileW == NT, "one output pixel per thread and channel group");
    // one extra chunk per pixel (the depth integral into S0): pixel tid's, loaded with the skip
    // chunks before the first store
    const bool extra1 = a.extra && a.out2_bf16 && a.extra_c == 8;
    const int64_t op_t = (n * g.Ho + ho0 + tid / kTileW) * g.Wo + wo0 + tid % kTileW;
    const bool in_t = ho0 + tid / kTileW < g.Ho && wo0 + tid % kTileW < g.Wo;
    const u32x4 ev = (extra1 && in_t) ? *reinterpret_cast<const u32x4*>(a.extra + op_t * 8) : zero;
    u32x4 kv[CO8];
#pragma unroll
    for (int u = 0; u < CO8; ++u) {
        const int i = tid + NT * u, c8 = i % CO8, pix = i / CO8;
        const int rr = pix / kTileW, cc = pix - rr * kTileW;
        const int ho = ho0 + rr, wo = wo0 + cc;
        kv[u] = (a.skip && a.out2_bf16 && ho < g.Ho && wo < g.Wo)
                    ? *reinterpret_cast<const u32x4*>(a.skip + ((n * g.Ho + ho) * g.Wo + wo) * CO + c8 * 8)
                    : zero;
    }
#pragma unroll
    for (int u = 0; u < CO8; ++u) {
        const int i = tid + NT * u, c8 = i % CO8, pix = i / CO8;
        const int rr = pix / kTileW, cc = pix - rr * kTileW;
        const int ho = ho0 + rr, wo = wo0 + cc;
        if (ho >= g.Ho || wo >= g.Wo) continue;
        const int64_t op = (n * g.Ho + ho) * g.Wo + wo;
        const u32x4 v = *reinterpret_cast<const u32x4*>(&sO[pix * CO + c8 * 8]);
        if (a.out_bf16) *reinterpret_cast<u32x4*>(a.out_bf16 + op * CO + c8 * 8) = v;
        if (a.skip && a.out2_bf16) {
            const u32x4 k = kv[u];
            u32x4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = add_bf16x2(v[j], k[j]);
            *reinterpret_cast<u32x4*>(a.out2_bf16 + op * ld2 + c8 * 8) = o;
        }
    }
    if (extra1) {
        if (in_t) *reinterpret_cast<u32x4*>(a.out2_bf16 + op_t * ld2 + CO) = ev;
    } else if (a.extra && a.out2_bf16) {
        const int E8 = a.extra_c / 8;
        for (int i = tid; i < TH * kTileW * E8; i += NT) {
            const int e8 = i % E8, pix = i / E8;
            const int rr = pix / kTileW, cc = pix - rr * kTileW;
            const int ho = ho0 + rr, wo = wo0 + cc;
            if (ho >= g.Ho || wo >= g.Wo) continue;
            const int64_t op = (n * g.Ho + ho) * g.Wo + wo;
            *reinterpret_cast<u32x4*>(a.out2_bf16 + op * ld2 + CO + e8 * 8) =
                *reinterpret_cast<const u32x4*>(a.extra + op * a.extra_c + e8 * 8);
        }
    }
    if (a.head_out && tid < TH * kTileW) {
        const int rr = tid / kTileW, cc = tid - rr * kTileW;
        const int ho = ho0 + rr, wo = wo0 + cc;
        if (ho < g.Ho && wo < g.Wo) {
            float sum = 0.f;
#pragma unroll
            for (int co = 0; co < CO; ++co) sum += bf2f(a.head_w[co]) * bf2f(sO[tid * CO + co]);
            a.head_out[(n * g.Ho + ho) * g.Wo + wo] = sum + a.head_b[0];
        }
    }
}

// Direct 3x3 weight gradient (pad 1; stride 1, or 2 with S2): dW[co][r][s][ci] = sum over
// output pixels p of dy[p][co] x[p + (r - 1, s - 1)][ci], for a group of CI in
// {8, 16, 24, 32} input and CO in {16, 32} output channels (block y: input
// group, block z: output group, of a layer with g.C and g.Co channels).  A block stages, per tile of
// 8 x 32 output pixels, the 10 x 34 halo of x and the tile of dy once in LDS,
// both transposed to channel planes (pixels contiguous; a thread packs two
// neighbouring pixels per 4-byte LDS store), so the MFMA operands of one
// output row are 32 consecutive pixels of a channel: A = dy (m = co), B = x
// shifted by the tap's column (n = ci), built from one aligned 16-byte and
// one 4-byte LDS read by byte alignment in registers.  A wave takes one 16-channel group of co and
// 8 CO / 64 consecutive output rows with all nine taps (every offset a
// compile-time constant, each staged x row read once per column shift for
// all its output rows) and keeps its accumulators in registers across the
// block's tiles; the next tile's chunks are loaded into
// registers while the current one is multiplied.  Tiles are dealt out with a
// static stride; at the end the four waves are summed in LDS in a fixed order
// and the block writes one partial dW, which a fixed-order reduction sums.
// UP: x is read upsampled x2 (fine pixel (h, w) is stored pixel (h/2, w/2)).
// S2: stride 2 (x pixel (2 h + r - 1, 2 w + s - 1) meets output pixel (h, w)).
constexpr int kWgH = 8, kWgW = 32;
constexpr int kWgXR = kWgH + 2, kWgXC = kWgW + 2;   // staged halo rows and columns
constexpr int kWgPitch = 40;                        // LDS row pitch (bf16)
constexpr int kWgXPlane = kWgXR * kWgPitch + 8;     // 204 dwords per channel: banks 12 apart
constexpr int kWgDPlane = kWgH * kWgPitch + 8;      // 164 dwords per channel: banks 4 apart
// stride 2: tiles of 4 x 32 outputs; their 9 x 65 input window is staged with the even and the odd
// columns in separate halves of an 80-element row, so the operands of all three column taps are
// aligned reads again (tap 0: even half; tap 1: odd half; tap 2: even half one column on)
constexpr int kWgH2 = 4;
constexpr int kWgXR2 = 2 * kWgH2 + 1, kWgRow2 = 80, kWgQ2 = 17;   // rows, row length, 4-column items
constexpr int kWgXPlane2 = kWgXR2 * kWgRow2 + 8;                  // 364 dwords: banks 44 apart
constexpr int kWgDPlane2 = kWgH2 * kWgPitch + 8;                  // 84 dwords: banks 20 apart

template <int CI, int CO, bool UP, bool S2>
__global__ __launch_bounds__(256) void k_wgrad3x3_tile(ConvGeom g, const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ dy, float* __restrict__ part)
{
    static_assert(!(UP && S2), "stride 2 reads its input directly");
    constexpr int NB = (CI + 15) / 16, CB = CO / 16, CIP = NB * 16;
    constexpr int CI8 = CI / 8, CO8 = CO / 8;
    constexpr int TH = S2 ? kWgH2 : kWgH;               // output rows per tile
    constexpr int XROW = S2 ? kWgRow2 : kWgPitch;       // LDS elements per staged input row
    constexpr int XPL = S2 ? kWgXPlane2 : kWgXPlane, DPL = S2 ? kWgDPlane2 : kWgDPlane;
    constexpr int RW = TH * CB / 4;   // output rows per wave (the waves split co groups x row groups)
    // items of one tile's operands and each thread's share: stride 1, 8 channels of two neighbouring
    // pixels; stride 2 input, 8 channels of four neighbouring pixels
    constexpr int XN = S2 ? kWgXR2 * kWgQ2 * CI8 : kWgXR * (kWgXC / 2) * CI8, DN = TH * (kWgW / 2) * CO8;
    constexpr int XE = S2 ? 4 : 2;    // pixels per input item
    constexpr int XI = (XN + 255) / 256, DI = (DN + 255) / 256;
    constexpr int SX = CIP * XPL, SD = CO * DPL, NW = CO * 9 * CI;
    static_assert(NW * 4 <= (SX + SD) * 2, "the cross-wave sum reuses the operand planes");
    __shared__ __attribute__((aligned(16))) uint16_t smem[SX + SD];
    uint16_t* sX = smem;
    uint16_t* sD = smem + SX;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int Hin = UP ? 2 * g.H : g.H, Win = UP ? 2 * g.W : g.W;
    const int tiles_x = (g.Wo + kWgW - 1) / kWgW, tiles_y = (g.Ho + TH - 1) / TH;
    const int64_t per_img = (int64_t)tiles_x * tiles_y;
    const int64_t total = (g.Kw / ((int64_t)g.Ho * g.Wo)) * per_img;   // Kw = N * Ho * Wo
    const uint16_t* xg = x + blockIdx.y * CI;    // the block's input channel group
    const uint16_t* dyg = dy + blockIdx.z * CO;  // and output channel group
    if constexpr (CIP != CI) {   // channels CI .. CIP - 1 stay zero
        for (int i = tid; i < (CIP - CI) * XPL; i += 256) sX[CI * XPL + i] = 0;
    }
    const int cbw = wave % CB, r0 = (wave / CB) * RW;   // the wave's co group and first output row
    f32x4 acc[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[t][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    u32x4 xv[XI][XE], dv[DI][2];
    auto load = [&](int64_t t) {
        const int64_t n = t / per_img;
        const int t_in = (int)(t - n * per_img);
        const int ty = t_in / tiles_x, tx = t_in - ty * tiles_x;
        const int ho0 = ty * TH, wo0 = tx * kWgW;
#pragma unroll
        for (int k = 0; k < XI; ++k) {
            const int i = tid + 256 * k;
            const int c8 = i % CI8, pr = i / CI8;
            constexpr int XQ = S2 ? kWgQ2 : kWgXC / 2;
            const int hy = pr / XQ, wx = XE * (pr - hy * XQ);
            const int hi = (S2 ? 2 * ho0 : ho0) - 1 + hy;
#pragma unroll
            for (int e = 0; e < XE; ++e) {
                const int wi = (S2 ? 2 * wo0 : wo0) - 1 + wx + e;
                xv[k][e] = zero;
                if (i < XN && hi >= 0 && wi >= 0 && hi < Hin && wi < Win) {
                    const int hs = UP ? hi >> 1 : hi, ws = UP ? wi >> 1 : wi;
                    xv[k][e] = *reinterpret_cast<const u32x4*>(xg + ((n * g.H + hs) * g.W + ws) * g.C + c8 * 8);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < DI; ++k) {
            const int i = tid + 256 * k;
            const int c8 = i % CO8, pr = i / CO8;
            const int r = pr / (kWgW / 2), c = 2 * (pr - r * (kWgW / 2));
            const int ho = ho0 + r;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int wo = wo0 + c + e;
                dv[k][e] = zero;
                if (i < DN && ho < g.Ho && wo < g.Wo)
                    dv[k][e] = *reinterpret_cast<const u32x4*>(dyg + ((n * g.Ho + ho) * g.Wo + wo) * g.Co + c8 * 8);
            }
        }
    };
    // transpose into the channel planes: channel 2j of a pixel pair is the low halves of dword j,
    // channel 2j + 1 the high halves (LDS positions do not depend on the tile)
    auto store = [&]() {
#pragma unroll
        for (int k = 0; k < XI; ++k) {
            const int i = tid + 256 * k;
            if (i < XN) {
                const int c8 = i % CI8, pr = i / CI8;
                constexpr int XQ = S2 ? kWgQ2 : kWgXC / 2;
                const int hy = pr / XQ, q = pr - hy * XQ;
                if constexpr (S2) {
                    // columns 4q .. 4q + 3: even ones to half 0 at 2q, 2q + 1; odd ones to half 1
                    uint32_t* d = reinterpret_cast<uint32_t*>(&sX[(c8 * 8) * XPL + hy * XROW + 2 * q]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        d[(2 * j) * (XPL / 2)] = __builtin_amdgcn_perm(xv[k][2][j], xv[k][0][j], 0x05040100u);
                        d[(2 * j + 1) * (XPL / 2)] = __builtin_amdgcn_perm(xv[k][2][j], xv[k][0][j], 0x07060302u);
                        d[(2 * j) * (XPL / 2) + kWgPitch / 2] =
                            __builtin_amdgcn_perm(xv[k][3][j], xv[k][1][j], 0x05040100u);
                        d[(2 * j + 1) * (XPL / 2) + kWgPitch / 2] =
                            __builtin_amdgcn_perm(xv[k][3][j], xv[k][1][j], 0x07060302u);
                    }
                } else {
                    uint32_t* d = reinterpret_cast<uint32_t*>(&sX[(c8 * 8) * XPL + hy * XROW + 2 * q]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        d[(2 * j) * (XPL / 2)] = __builtin_amdgcn_perm(xv[k][1][j], xv[k][0][j], 0x05040100u);
                        d[(2 * j + 1) * (XPL / 2)] = __builtin_amdgcn_perm(xv[k][1][j], xv[k][0][j], 0x07060302u);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < DI; ++k) {
            const int i = tid + 256 * k;
            if (i < DN) {
                const int c8 = i % CO8, pr = i / CO8;
                const int r = pr / (kWgW / 2), c = 2 * (pr - r * (kWgW / 2));
                uint32_t* d = reinterpret_cast<uint32_t*>(&sD[(c8 * 8) * DPL + r * kWgPitch + c]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    d[(2 * j) * (DPL / 2)] = __builtin_amdgcn_perm(dv[k][1][j], dv[k][0][j], 0x05040100u);
                    d[(2 * j + 1) * (DPL / 2)] = __builtin_amdgcn_perm(dv[k][1][j], dv[k][0][j], 0x07060302u);
                }
            }
        }
    };
    const uint16_t* pa = &sD[(cbw * 16 + lr) * DPL + r0 * kWgPitch + 8 * lk];                // A: output row r0
    const uint16_t* pbx = &sX[lr * XPL + (S2 ? 2 * r0 : r0) * XROW + 8 * lk];              // B: its first input row
    if ((int64_t)blockIdx.x < total) load(blockIdx.x);
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        __syncthreads();   // the previous tile's operands have been read
        store();
        __syncthreads();
        if (t + gridDim.x < total) load(t + gridDim.x);
        bf16x8 fa[RW];
#pragma unroll
        for (int rs = 0; rs < RW; ++rs) fa[rs] = *reinterpret_cast<const bf16x8*>(pa + rs * kWgPitch);
        // staged row xr feeds output row r0 + rs through tap row xr - rs (stride 2: xr - 2 rs)
        constexpr int NXR = S2 ? 2 * RW + 1 : RW + 2;
#pragma unroll
        for (int xr = 0; xr < NXR; ++xr)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                // stride 1: staged columns 8 lk .. 8 lk + 9 of the row give the three column shifts;
                // stride 2: even columns 8 lk .. 8 lk + 8 and odd columns 8 lk .. 8 lk + 7
                const uint16_t* src = pbx + nb * 16 * XPL + xr * XROW;
                const u32x4 lo = *reinterpret_cast<const u32x4*>(src);
                const uint32_t ex = *reinterpret_cast<const uint32_t*>(src + 8);
                const u32x4 sft = {__builtin_amdgcn_alignbyte(lo[1], lo[0], 2u), __builtin_amdgcn_alignbyte(lo[2], lo[1], 2u),
                                   __builtin_amdgcn_alignbyte(lo[3], lo[2], 2u), __builtin_amdgcn_alignbyte(ex, lo[3], 2u)};
                u32x4 sh[3];
                if constexpr (S2) {
                    sh[0] = lo;
                    sh[1] = *reinterpret_cast<const u32x4*>(src + kWgPitch);
                    sh[2] = sft;
                } else {
                    sh[0] = lo;
                    sh[1] = sft;
                    sh[2] = u32x4{lo[1], lo[2], lo[3], ex};
                }
#pragma unroll
                for (int dc = 0; dc < 3; ++dc) {
                    const bf16x8 fb = __builtin_bit_cast(bf16x8, sh[dc]);
#pragma unroll
                    for (int rs = 0; rs < RW; ++rs) {
                        const int dr = xr - (S2 ? 2 : 1) * rs;
                        if (dr < 0 || dr > 2) continue;
                        acc[3 * dr + dc][nb] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[rs], fb, acc[3 * dr + dc][nb], 0, 0, 0);
                    }
                }
            }
    }
    // sum over the row groups, in wave order, in the [Co][3][3][Ci] layout: lane (lr, lk),
    // element q is co = 16 cbw + 4 lk + q, ci = 16 nb + lr (waves below CB start their co group)
    float* red = reinterpret_cast<float*>(smem);
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int ci = nb * 16 + lr;
                    if (ci >= CI) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float& r = red[((cbw * 16 + 4 * lk + q) * 9 + tap) * CI + ci];
                        r = (w < CB ? 0.f : r) + acc[tap][nb][q];
                    }
                }
        }
    }
    __syncthreads();
    // the blocks with this blockIdx.x (one per channel-group pair) fill partial blockIdx.x of the whole dW
    float* pb = part + (int64_t)blockIdx.x * ((int64_t)g.Co * 9 * g.C);
    for (int i = tid; i < NW; i += 256) {
        const int ci = i % CI, q = i / CI;   // q = co * 9 + tap
        pb[((int64_t)(blockIdx.z * CO) * 9 + q) * g.C + blockIdx.y * CI + ci] = red[i];
    }
}

// Backward of the 1x1 map p = W x (W: KC x C, bf16) feeding the depth
// integral: g[pixel][c] += sum_k dp[pixel][k] W[k][c] (written once, after
// the FP32 sum over k) and the per-block partials of dW[k][c] = sum over
// pixels of dp[pixel][k] x[pixel][c].  Four threads share a pixel, each
// owning C / 4 channels, so a thread keeps KC x C / 4 accumulators; the
// pixels are dealt out in a fixed order and reduced in a fixed order.
constexpr int kProjBlocks = 1024;
template <int KC, int C>
__global__ __launch_bounds__(256) void k_proj_bwd(const uint16_t* __restrict__ dp, const uint16_t* __restrict__ x,
                                                  const uint16_t* __restrict__ w, float* __restrict__ g, int64_t P,
                                                  float* __restrict__ part)
{
    constexpr int CQ = C / 4;
    static_assert(C % 16 == 0 && KC == 8, "four 4-channel groups per thread quad; 8 map channels");
    __shared__ float red[4][KC * C];
    const int q = threadIdx.x & 3, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float wr[KC][CQ], acc[KC][CQ];
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int j = 0; j < CQ; ++j) {
            wr[k][j] = bf2f(w[k * C + q * CQ + j]);
            acc[k][j] = 0.f;
        }
    const int64_t stride = (int64_t)gridDim.x * 64;
    for (int64_t p = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2); p < P; p += stride) {
        const u32x4 dv = *reinterpret_cast<const u32x4*>(dp + p * KC);
        float d[KC];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            d[2 * j] = __uint_as_float(dv[j] << 16);
            d[2 * j + 1] = __uint_as_float(dv[j] & 0xFFFF0000u);
        }
        float xs[CQ];
        const uint16_t* xp = x + p * C + q * CQ;
#pragma unroll
        for (int j = 0; j < CQ; j += 4) {
            const uint2 v = *reinterpret_cast<const uint2*>(xp + j);
            xs[j] = __uint_as_float(v.x << 16);
            xs[j + 1] = __uint_as_float(v.x & 0xFFFF0000u);
            xs[j + 2] = __uint_as_float(v.y << 16);
            xs[j + 3] = __uint_as_float(v.y & 0xFFFF0000u);
        }
        float* gp = g + p * C + q * CQ;
#pragma unroll
        for (int j = 0; j < CQ; j += 4) {
            float4 gv = *reinterpret_cast<const float4*>(gp + j);
            float s[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float t = 0.f;
#pragma unroll
                for (int k = 0; k < KC; ++k) t = fmaf(d[k], wr[k][j + e], t);
                s[e] = t;
            }
            gv.x += s[0];
            gv.y += s[1];
            gv.z += s[2];
            gv.w += s[3];
            *reinterpret_cast<float4*>(gp + j) = gv;
        }
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int j = 0; j < CQ; ++j) acc[k][j] = fmaf(d[k], xs[j], acc[k][j]);
    }
    // the 16 threads of a wave with the same channel group, then the four waves
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int j = 0; j < CQ; ++j) {
            float v = acc[k][j];
#pragma unroll
            for (int m = 4; m < 64; m <<= 1) v += __shfl_xor(v, m);
            if (lane < 4) red[wave][k * C + q * CQ + j] = v;
        }
    __syncthreads();
    for (int i = threadIdx.x; i < KC * C; i += 256)
        part[(int64_t)blockIdx.x * (KC * C) + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// ---------------------------------------------------------------------------
// element-wise / reduction kernels

// dPre = bf16(g * [y > 0]) (ReLU) or bf16(g) (no activation)
__global__ void k_mask_to_bf16(const float* g, const uint16_t* y, uint16_t* out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = (y == nullptr || bf2f(y[i]) > 0.f) ? g[i] : 0.f;
        out[i] = f2bf(v);
    }
}

// coarse[n][h][w][c] (+)= sum of the 2x2 fine block (backward of the x2 upsample)
__global__ void k_pool2x2_sum(const float* fine, float* coarse, int N, int H, int W, int C, int accumulate)
{
    const int64_t total = (int64_t)N * H * W * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % W);
        const int64_t q = p / W;
        const int h = (int)(q % H);
        const int n = (int)(q / H);
        const int64_t base = (((int64_t)n * 2 * H + 2 * h) * 2 * W + 2 * w) * C + c;
        const int64_t rs = (int64_t)2 * W * C;
        const float s = (fine[base] + fine[base + C]) + (fine[base + rs] + fine[base + rs + C]);
        coarse[i] = accumulate ? coarse[i] + s : s;
    }
}

// Masked output gradient and bias-gradient partials in one pass over a
// [rows][C] matrix: out = bf16(g * [y > 0]) (y may be null: no mask; out may
// be null: g is already bf16 in gb), part[block][c] = sum of the block's rows
// of out.  Thread t owns column t % C for every (256 / C)-th row; the threads
// of a column are summed in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_mask_colsum(const float* g, int ldg, const uint16_t* gb, const uint16_t* y,
                                                     uint16_t* out, int64_t rows, int C, int64_t rows_per_block,
                                                     float* part, float slope)
{
    // a thread owns one 8-channel chunk of rows r_off, r_off + RP, ... (C multiple of 8, <= 256)
    __shared__ float red[256 * 8];
    const int C8 = C / 8;
    const int RP = 256 / C8;
    const int c8 = threadIdx.x % C8;
    const int r_off = threadIdx.x / C8;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    float sum[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) sum[j] = 0.f;
    if (r_off < RP) {
        // kMaskRows rows per thread at a time, all their loads issued before their stores (a load
        // issued after a store waits for it); the sums take the rows in order
        constexpr int kMaskRows = 4;
        for (int64_t rb = r0 + r_off; rb < r1; rb += kMaskRows * RP) {
            u32x4 b[kMaskRows];
            if (gb) {
#pragma unroll
                for (int k = 0; k < kMaskRows; ++k) {
                    const int64_t r = rb + k * RP;
                    b[k] = r < r1 ? *reinterpret_cast<const u32x4*>(gb + r * C + c8 * 8) : u32x4{0u, 0u, 0u, 0u};
                }
            } else {
                float4 g0[kMaskRows], g1[kMaskRows];
                u32x4 yv[kMaskRows];
#pragma unroll
                for (int k = 0; k < kMaskRows; ++k) {
                    const int64_t r = rb + k * RP;
                    yv[k] = u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};   // no mask: bf16 1.0
                    g0[k] = g1[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (r < r1) {
                        g0[k] = *reinterpret_cast<const float4*>(g + r * ldg + c8 * 8);
                        g1[k] = *reinterpret_cast<const float4*>(g + r * ldg + c8 * 8 + 4);
                        if (y) yv[k] = *reinterpret_cast<const u32x4*>(y + r * C + c8 * 8);
                    }
                }
#pragma unroll
                for (int k = 0; k < kMaskRows; ++k) {
                    const float gv[8] = {g0[k].x, g0[k].y, g0[k].z, g0[k].w, g1[k].x, g1[k].y, g1[k].z, g1[k].w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float ylo = __uint_as_float(yv[k][j] << 16), yhi = __uint_as_float(yv[k][j] & 0xFFFF0000u);
                        const uint16_t lo = f2bf(ylo > 0.f ? gv[2 * j] : (slope != 0.f ? slope * gv[2 * j] : 0.f));
                        const uint16_t hi =
                            f2bf(yhi > 0.f ? gv[2 * j + 1] : (slope != 0.f ? slope * gv[2 * j + 1] : 0.f));
                        b[k][j] = (uint32_t)lo | ((uint32_t)hi << 16);
                    }
                }
#pragma unroll
                for (int k = 0; k < kMaskRows; ++k) {
                    const int64_t r = rb + k * RP;
                    if (out && r < r1) *reinterpret_cast<u32x4*>(out + r * C + c8 * 8) = b[k];
                }
            }
#pragma unroll
            for (int k = 0; k < kMaskRows; ++k) {
                if (rb + k * RP >= r1) break;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sum[2 * j] += __uint_as_float(b[k][j] << 16);
                    sum[2 * j + 1] += __uint_as_float(b[k][j] & 0xFFFF0000u);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) red[threadIdx.x * 8 + j] = sum[j];
    __syncthreads();
    if ((int)threadIdx.x < C) {
        const int k8 = threadIdx.x / 8, j = threadIdx.x % 8;
        float t = 0.f;
        for (int q = 0; q < RP; ++q) t += red[(q * C8 + k8) * 8 + j];
        part[(int64_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

// out[i] = sum_s part[s][i] in fixed order
// Depth integral along the beam.  A block owns 32 neighbouring columns (in
// frame-major order) and splits their rows into 8 segments, one thread per
// (segment, column): each thread first sums its segment, the segment totals
// meet in LDS, and a second pass over the segment writes the running sums
// from the totals of the segments above (below, for the backward).  A wave
// covers 32 columns of two segments, so each row access is contiguous.
// Eight channels per pixel (kScanC).
constexpr int kScanC = 8;
constexpr int kScanCols = 32, kScanSeg = 8;
constexpr int kScanRows = 4;   // rows whose loads are issued together

// the 1x1 map p = b + w e of one pixel (e: 16 bf16 channels as two 16-byte chunks); w, b in LDS
__device__ __forceinline__ void depth_map(const u32x4& a0, const u32x4& a1, const float* wf, const float* bf,
                                          float* p)
{
    asm volatile("" ::: "memory");   // weights stay in LDS (broadcast reads), not in registers
    float xc[16];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        xc[2 * j] = __uint_as_float(a0[j] << 16);
        xc[2 * j + 1] = __uint_as_float(a0[j] & 0xFFFF0000u);
        xc[8 + 2 * j] = __uint_as_float(a1[j] << 16);
        xc[8 + 2 * j + 1] = __uint_as_float(a1[j] & 0xFFFF0000u);
    }
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
        float acc = bf[k];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc = fmaf(wf[k * 16 + c], xc[c], acc);
        p[k] = acc;
    }
}

// out[n][y][x][c_off + k] = bf16(scale * sum_{v < y} p_k(n, v, x)) with the
// 1x1 map p_k = b[k] + sum_c w[k][c] e[n][v][x][c] of the bf16 tensor e
// [N][H][W][16] (w bf16 [8][16], b FP32), evaluated in FP32 per pixel.
__global__ __launch_bounds__(256) void k_depth_map_scan_fwd(const uint16_t* __restrict__ e,
                                                            const uint16_t* __restrict__ w,
                                                            const float* __restrict__ b, uint16_t* __restrict__ out,
                                                            int N, int H, int W, float scale, int ld, int c_off)
{
    __shared__ float sw[kScanC * 16];
    __shared__ float sb[kScanC];
    __shared__ float tot[kScanSeg][kScanC][kScanCols + 1];
    if (threadIdx.x < kScanC * 16) sw[threadIdx.x] = bf2f(w[threadIdx.x]);
    if (threadIdx.x < kScanC) sb[threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    const int c = threadIdx.x % kScanCols, sg = threadIdx.x / kScanCols;
    const int64_t col = (int64_t)blockIdx.x * kScanCols + c;
    const bool live = col < (int64_t)N * W;
    const int64_t n = live ? col / W : 0;
    const int x = live ? (int)(col - n * W) : 0;
    const int seg = (H + kScanSeg - 1) / kScanSeg;
    const int ya = live ? min(sg * seg, H) : 0, yb = live ? min(ya + seg, H) : 0;
    const float* wf = sw;
    const float* bf = sb;
    float sum[kScanC], p[kScanC];
#pragma unroll
    for (int k = 0; k < kScanC; ++k) sum[k] = 0.f;
    const uint16_t* ec = e + (n * H * W + x) * 16;   // column base; row stride W * 16
    for (int y0 = ya; y0 < yb; y0 += kScanRows) {
        u32x4 a0[kScanRows], a1[kScanRows];
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int64_t o = (int64_t)min(y0 + q, yb - 1) * W * 16;
            a0[q] = *reinterpret_cast<const u32x4*>(ec + o);
            a1[q] = *reinterpret_cast<const u32x4*>(ec + o + 8);
        }
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            if (y0 + q >= yb) break;
            depth_map(a0[q], a1[q], wf, bf, p);
#pragma unroll
            for (int k = 0; k < kScanC; ++k) sum[k] += p[k];
        }
    }
#pragma unroll
    for (int k = 0; k < kScanC; ++k) tot[sg][k][c] = sum[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
        float o = 0.f;
        for (int q = 0; q < sg; ++q) o += tot[q][k][c];
        sum[k] = o;   // running sum over the rows above this segment
    }
    uint16_t* oc = out + (n * H * W + x) * ld + c_off;
    for (int y0 = ya; y0 < yb; y0 += kScanRows) {
        u32x4 a0[kScanRows], a1[kScanRows];
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int64_t o = (int64_t)min(y0 + q, yb - 1) * W * 16;
            a0[q] = *reinterpret_cast<const u32x4*>(ec + o);
            a1[q] = *reinterpret_cast<const u32x4*>(ec + o + 8);
        }
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int y = y0 + q;
            if (y >= yb) break;
            u32x4 ov;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                ov[j] = (uint32_t)f2bf(scale * sum[2 * j]) | ((uint32_t)f2bf(scale * sum[2 * j + 1]) << 16);
            *reinterpret_cast<u32x4*>(oc + (int64_t)y * W * ld) = ov;
            depth_map(a0[q], a1[q], wf, bf, p);
#pragma unroll
            for (int k = 0; k < kScanC; ++k) sum[k] += p[k];
        }
    }
}

// k_depth_map_scan_fwd for columns of at most kScan1Seg * kScan1Rows rows, reading e once: a block
// owns kScan1Cols neighbouring columns split into kScan1Seg segments of at most kScan1Rows rows, one
// thread per (segment, column), which keeps its rows' maps p in registers between the segment sum
// and the running sums (the two-pass kernel reads e again for those).
constexpr int kScan1Cols = 8, kScan1Seg = 32, kScan1Rows = 8;
__global__ __launch_bounds__(256) void k_depth_map_scan_fwd1(const uint16_t* __restrict__ e,
                                                             const uint16_t* __restrict__ w,
                                                             const float* __restrict__ b, uint16_t* __restrict__ out,
                                                             int N, int H, int W, float scale, int ld, int c_off)
{
    static_assert(kScan1Cols * kScan1Seg == 256, "one thread per (segment, column)");
    __shared__ float sw[kScanC * 16];
    __shared__ float sb[kScanC];
    __shared__ float tot[kScan1Seg][kScanC][kScan1Cols + 1];
    if (threadIdx.x < kScanC * 16) sw[threadIdx.x] = bf2f(w[threadIdx.x]);
    if (threadIdx.x < kScanC) sb[threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    const int c = threadIdx.x % kScan1Cols, sg = threadIdx.x / kScan1Cols;
    const int64_t col = (int64_t)blockIdx.x * kScan1Cols + c;
    const bool live = col < (int64_t)N * W;
    const int64_t n = live ? col / W : 0;
    const int x = live ? (int)(col - n * W) : 0;
    const int seg = (H + kScan1Seg - 1) / kScan1Seg;   // <= kScan1Rows (host check)
    const int ya = live ? min(sg * seg, H) : 0, yb = live ? min(ya + seg, H) : 0;
    const uint16_t* ec = e + (n * H * W + x) * 16;   // column base; row stride W * 16
    u32x4 a0[kScan1Rows], a1[kScan1Rows];
#pragma unroll
    for (int q = 0; q < kScan1Rows; ++q) {   // every row's loads before any use
        const int64_t o = (int64_t)min(ya + q, max(yb - 1, 0)) * W * 16;
        a0[q] = *reinterpret_cast<const u32x4*>(ec + o);
        a1[q] = *reinterpret_cast<const u32x4*>(ec + o + 8);
    }
    float pr[kScan1Rows][kScanC], sum[kScanC];
#pragma unroll
    for (int k = 0; k < kScanC; ++k) sum[k] = 0.f;
#pragma unroll
    for (int q = 0; q < kScan1Rows; ++q) {
        depth_map(a0[q], a1[q], sw, sb, pr[q]);
        if (ya + q < yb) {
#pragma unroll
            for (int k = 0; k < kScanC; ++k) sum[k] += pr[q][k];
        }
    }
#pragma unroll
    for (int k = 0; k < kScanC; ++k) tot[sg][k][c] = sum[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
        float o = 0.f;
        for (int q = 0; q < sg; ++q) o += tot[q][k][c];
        sum[k] = o;   // running sum over the rows above this segment
    }
    uint16_t* oc = out + (n * H * W + x) * ld + c_off;
#pragma unroll
    for (int q = 0; q < kScan1Rows; ++q) {
        const int y = ya + q;
        if (y >= yb) break;
        u32x4 ov;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            ov[j] = (uint32_t)f2bf(scale * sum[2 * j]) | ((uint32_t)f2bf(scale * sum[2 * j + 1]) << 16);
        *reinterpret_cast<u32x4*>(oc + (int64_t)y * W * ld) = ov;
#pragma unroll
        for (int k = 0; k < kScanC; ++k) sum[k] += pr[q][k];
    }
}

// Backward of k_depth_map_scan_fwd after the 1x1 map, through a tensor g
// [pixel][ld] (FP32) whose channels [c_off, c_off + 8) are the integral's
// gradient:  dp[n][v][x][k] = bf16(scale * sum_{y > v} g[n][y][x][c_off + k]),
// channels [0, c_off) copied to g_skip [pixel][c_off] (c_off multiple of 4),
// and per-block column sums of the bf16 dp (bias gradient partials) in
// part[block][8].
__global__ __launch_bounds__(256) void k_depth_scan_bwd(const float* __restrict__ g, int ld, int c_off,
                                                        float* __restrict__ g_skip, uint16_t* __restrict__ dp,
                                                        float* __restrict__ part, int N, int H, int W, float scale)
{
    __shared__ float tot[kScanSeg][kScanC][kScanCols + 1];
    __shared__ float red[kScanC][256];
    const int c = threadIdx.x % kScanCols, sg = threadIdx.x / kScanCols;
    const int64_t col = (int64_t)blockIdx.x * kScanCols + c;
    const bool live = col < (int64_t)N * W;
    const int64_t n = live ? col / W : 0;
    const int x = live ? (int)(col - n * W) : 0;
    const int seg = (H + kScanSeg - 1) / kScanSeg;
    const int ya = live ? min(sg * seg, H) : 0, yb = live ? min(ya + seg, H) : 0;
    const int64_t pc = n * H * W + x;   // column's pixel index at row 0; row stride W
    float sum[kScanC], bsum[kScanC];
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
        sum[k] = 0.f;
        bsum[k] = 0.f;
    }
    for (int y0 = ya; y0 < yb; y0 += kScanRows) {
        float4 ga[kScanRows][2];
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int64_t px = pc + (int64_t)min(y0 + q, yb - 1) * W;
            ga[q][0] = *reinterpret_cast<const float4*>(g + px * ld + c_off);
            ga[q][1] = *reinterpret_cast<const float4*>(g + px * ld + c_off + 4);
        }
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            if (y0 + q >= yb) break;
            sum[0] += ga[q][0].x; sum[1] += ga[q][0].y; sum[2] += ga[q][0].z; sum[3] += ga[q][0].w;
            sum[4] += ga[q][1].x; sum[5] += ga[q][1].y; sum[6] += ga[q][1].z; sum[7] += ga[q][1].w;
        }
    }
#pragma unroll
    for (int k = 0; k < kScanC; ++k) tot[sg][k][c] = sum[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
        float o = 0.f;
        for (int q = kScanSeg - 1; q > sg; --q) o += tot[q][k][c];
        sum[k] = o;   // running sum over the rows below this segment
    }
    for (int y0 = yb - 1; y0 >= ya; y0 -= kScanRows) {
        float4 ga[kScanRows][2];
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int64_t px = pc + (int64_t)max(y0 - q, ya) * W;
            ga[q][0] = *reinterpret_cast<const float4*>(g + px * ld + c_off);
            ga[q][1] = *reinterpret_cast<const float4*>(g + px * ld + c_off + 4);
        }
#pragma unroll
        for (int q = 0; q < kScanRows; ++q) {
            const int y = y0 - q;
            if (y < ya) break;
            const int64_t px = pc + (int64_t)y * W;
            for (int cc = 0; cc < c_off; cc += 4)
                *reinterpret_cast<float4*>(g_skip + px * c_off + cc) = *reinterpret_cast<const float4*>(g + px * ld + cc);
            u32x4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint16_t lo = f2bf(scale * sum[2 * j]), hi = f2bf(scale * sum[2 * j + 1]);
                bsum[2 * j] += bf2f(lo);
                bsum[2 * j + 1] += bf2f(hi);
                o[j] = (uint32_t)lo | ((uint32_t)hi << 16);
            }
            *reinterpret_cast<u32x4*>(dp + px * kScanC) = o;
            sum[0] += ga[q][0].x; sum[1] += ga[q][0].y; sum[2] += ga[q][0].z; sum[3] += ga[q][0].w;
            sum[4] += ga[q][1].x; sum[5] += ga[q][1].y; sum[6] += ga[q][1].z; sum[7] += ga[q][1].w;
        }
    }
#pragma unroll
    for (int k = 0; k < kScanC; ++k) red[k][threadIdx.x] = bsum[k];
    __syncthreads();
    if (threadIdx.x < kScanC) {   // fixed order over the block's threads
        float t = 0.f;
        for (int i = 0; i < 256; ++i) t += red[threadIdx.x][i];
        part[(int64_t)blockIdx.x * kScanC + threadIdx.x] = t;
    }
}

// out[i] = sum over z of part[z][i]; one thread per output, rows in order
// (for many outputs and few rows)
__global__ void k_sum_parts(const float* part, int64_t n, int splits, float* out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        int z = 0;
        for (; z + 8 <= splits; z += 8) {   // eight loads in flight, added in order
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(z + j) * n + i];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[j];
        }
        for (; z < splits; ++z) s += part[(int64_t)z * n + i];
        out[i] = s;
    }
}

// the same sum for few outputs and many rows: thread (ty, tx) of a block sums
// rows ty, ty + G, ... of output blockIdx.x * ob + tx (G = 256 / ob), then
// the G partial sums are added in order (fixed order, deterministic)
__global__ __launch_bounds__(256) void k_sum_parts_grouped(const float* part, int64_t n, int splits, float* out,
                                                           int ob)
{
    __shared__ float red[256];
    const int tx = threadIdx.x % ob, ty = threadIdx.x / ob;
    const int G = 256 / ob;
    const int64_t i = (int64_t)blockIdx.x * ob + tx;
    float s = 0.f;
    if (i < n) {
        int z = ty;
        for (; z + 7 * G < splits; z += 8 * G) {   // eight loads in flight, added in order
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(z + j * G) * n + i];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[j];
        }
        for (; z < splits; z += G) s += part[(int64_t)z * n + i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (ty == 0 && i < n) {
        float t = 0.f;
        for (int j = 0; j < G; ++j) t += red[j * ob + tx];
        out[i] = t;
    }
}

// Several reductions of per-block partials in one launch: block b computes output i of the segment
// holding it, out[out_off + i] = sum over z < splits of part[part_off + z n + i], added as
// k_sum_parts_grouped adds one output (thread t sums z = t, t + 256, ... in order, then the 256
// thread sums in order), so the results equal separate reduce_parts calls
__global__ __launch_bounds__(256) void k_reduce_segments(const float* __restrict__ part, float* __restrict__ out,
                                                         ReduceSegs t)
{
    __shared__ float red[256];
    int k = 0;
    while (k + 1 < t.count && t.s[k + 1].first <= (int)blockIdx.x) ++k;
    const ReduceSeg sg = t.s[k];
    const int64_t i = (int64_t)blockIdx.x - sg.first;
    const float* p = part + sg.part_off + i;
    float v = 0.f;
    for (int z = threadIdx.x; z < sg.splits; z += 256) v += p[(int64_t)z * sg.n];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f;
        for (int j = 0; j < 256; ++j) a += red[j];
        out[sg.out_off + i] = a;
    }
}

// 1x1 head with one output channel: y[p] = sum_c w[c] x[p][c] + b (C = 16)
__global__ __launch_bounds__(256) void k_head_fwd(const uint16_t* x, const uint16_t* w, const float* b, float* y,
                                                  int64_t P, int C)
{
    float wf[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) wf[c] = c < C ? bf2f(w[c]) : 0.f;
    const float bias = b[0];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const uint4 v0 = *reinterpret_cast<const uint4*>(x + p * 16);
        const uint4 v1 = *reinterpret_cast<const uint4*>(x + p * 16 + 8);
        const uint16_t* h0 = reinterpret_cast<const uint16_t*>(&v0);
        const uint16_t* h1 = reinterpret_cast<const uint16_t*>(&v1);
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += wf[c] * bf2f(h0[c]);
#pragma unroll
        for (int c = 0; c < 8; ++c) s += wf[8 + c] * bf2f(h1[c]);
        y[p] = s + bias;
    }
}

// head backward (C = 16): dx[p][c] = w[c] g[p]; per-block partials of
// dw[c] = sum_p x[p][c] g[p] (c < 16) and db = sum_p g[p] (entry 16)
__global__ __launch_bounds__(256) void k_head_bwd(const uint16_t* x, const uint16_t* w, const float* g, float* dx,
                                                  int64_t P, int C, int64_t rows_per_block, float* part)
{
    __shared__ float red[17][256];
    float wf[16], acc[17];
#pragma unroll
    for (int c = 0; c < 16; ++c) wf[c] = bf2f(w[c]);
#pragma unroll
    for (int c = 0; c < 17; ++c) acc[c] = 0.f;
    const int64_t p0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t p1 = min(P, p0 + rows_per_block);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const float gp = g[p];
        const uint4 v0 = *reinterpret_cast<const uint4*>(x + p * 16);
        const uint4 v1 = *reinterpret_cast<const uint4*>(x + p * 16 + 8);
        const uint16_t* h0 = reinterpret_cast<const uint16_t*>(&v0);
        const uint16_t* h1 = reinterpret_cast<const uint16_t*>(&v1);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += bf2f(h0[c]) * gp;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[8 + c] += bf2f(h1[c]) * gp;
        acc[16] += gp;
        float4* d = reinterpret_cast<float4*>(dx + p * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            d[q] = make_float4(wf[4 * q] * gp, wf[4 * q + 1] * gp, wf[4 * q + 2] * gp, wf[4 * q + 3] * gp);
    }
#pragma unroll
    for (int c = 0; c < 17; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    if (threadIdx.x < 17) {
        float t = 0.f;
        for (int j = 0; j < 256; ++j) t += red[threadIdx.x][j];
        part[(int64_t)blockIdx.x * 17 + threadIdx.x] = t;
    }
    (void)C;
}

// Discriminator input of two sets of P pixels: z[i] = (x[p] channels 0..3,
// bf16(img), 0, 0, 0) with img = y_real[p] for i = p < P and y_fake[p] for
// i = P + p (the same encoded input x[p] in both sets)
__global__ void k_disc_input(const uint16_t* x, const float* y_real, const float* y_fake, uint16_t* z, int64_t P)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * P; i += (int64_t)gridDim.x * blockDim.x) {
        const bool fake = i >= P;
        const int64_t p = fake ? i - P : i;
        const uint2 xv = *reinterpret_cast<const uint2*>(x + p * 8);
        const float img = fake ? y_fake[p] : y_real[p];
        uint4 o;
        o.x = xv.x;
        o.y = xv.y;
        o.z = (uint32_t)f2bf(img);
        o.w = 0u;
        *reinterpret_cast<uint4*>(z + i * 8) = o;
    }
}

// Binary cross-entropy on the logits l = logits[r * ld] of rows r < P_total:
// rows r < P_real have label 1 (loss w_real softplus(-l), gradient
// gscale w_real (sigmoid(l) - 1)), the rest label 0 (w_fake softplus(l),
// gscale w_fake sigmoid(l)).  grad rows hold ld floats (channel 0 the
// gradient, the others 0); part[block] = the block's loss sum.
__device__ __forceinline__ float softplus_f(float a) { return fmaxf(a, 0.f) + log1pf(expf(-fabsf(a))); }

__global__ __launch_bounds__(256) void k_bce_logits(const float* logits, int ld, int64_t P_real, int64_t P_total,
                                                    float w_real, float w_fake, float gscale, float* grad,
                                                    int64_t per_block, float* part)
{
    __shared__ float red[256];
    const int64_t r0 = (int64_t)blockIdx.x * per_block;
    const int64_t r1 = min(P_total, r0 + per_block);
    float acc = 0.f;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const float l = logits[r * ld];
        const float e = expf(-fabsf(l));
        const float sig = l >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
        const bool real = r < P_real;
        const float w = real ? w_real : w_fake;
        acc += w * softplus_f(real ? -l : l);
        grad[r * ld] = gscale * w * (real ? sig - 1.f : sig);
        for (int c = 1; c < ld; ++c) grad[r * ld + c] = 0.f;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// gy[p] += dz[p * ld + c]
__global__ void k_add_channel(float* gy, const float* dz, int ld, int c, int64_t P)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        gy[p] += dz[p * ld + c];
}

// L1 loss: per-block partial sums of |yhat - y| * scale (scale = 1 / n);
// grad = sign(yhat - y) * scale
__global__ void k_l1(const float* yhat, const float* y, int64_t n, float scale, float* grad, int64_t per_block,
                     float* part)
{
    __shared__ float red[256];
    const int64_t i0 = (int64_t)blockIdx.x * per_block;
    const int64_t i1 = min(n, i0 + per_block);
    float s = 0.f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const float d = yhat[i] - y[i];
        s += fabsf(d);
        grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * scale;   // mean over all n
}

// Adam on FP32 masters; writes the bf16 weights [Co][K] and their transpose
// WT [Ci][taps][Co] (data gradient operand)
// Adam's per-step scalars on the device, so a captured step reads them at
// replay: steps[0] (and steps[1], the discriminator's, when disc) count the
// updates; coef = {lr, 1 - b1^t, 1 - b2^t, 1 - b1^td, 1 - b2^td}
__global__ void k_adam_coef(int64_t* steps, float* coef, float lr, float b1, float b2, int disc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t t = steps[0] + 1;
    steps[0] = t;
    coef[0] = lr;
    coef[1] = 1.f - powf(b1, (float)t);
    coef[2] = 1.f - powf(b2, (float)t);
    if (disc) {
        const int64_t td = steps[1] + 1;
        steps[1] = td;
        coef[3] = 1.f - powf(b1, (float)td);
        coef[4] = 1.f - powf(b2, (float)td);
    }
}

// Adam over a parameter vector made of segments (one launch for all of a
// network's tensors): block b works on kAdamChunk elements of the segment
// whose block0 <= b; a weight segment also refreshes its bf16 copy and,
// with a transpose, the [Ci][taps][Co] copy of the data gradient
constexpr int kAdamChunk = 2048;
__global__ __launch_bounds__(256) void k_adam_multi(const AdamSeg* __restrict__ segs, int nseg, float* w, float* m,
                                                    float* v, const float* __restrict__ g, uint16_t* wb, uint16_t* wt,
                                                    const float* __restrict__ coef, int ci, float b1, float b2,
                                                    float eps)
{
    __shared__ int s_seg;
    if (threadIdx.x == 0) {
        int k = 0;
        while (k + 1 < nseg && segs[k + 1].block0 <= (int)blockIdx.x) ++k;
        s_seg = k;
    }
    __syncthreads();
    const AdamSeg sg = segs[s_seg];
    const float lr = coef[0], c1 = coef[ci], c2 = coef[ci + 1];
    const int64_t base = (int64_t)((int)blockIdx.x - sg.block0) * kAdamChunk;
    const int64_t end = min(base + (int64_t)kAdamChunk, sg.n);
    for (int64_t j = base + threadIdx.x; j < end; j += 256) {
        const int64_t i = sg.off + j;
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (sg.bf16) {
            const uint16_t bb = f2bf(wi);
            wb[i] = bb;
            if (sg.transpose) {
                // j = (co * taps + t) * Ci + ci  ->  (ci * taps + t) * Co + co
                const int cc = (int)(j % sg.Ci);
                const int64_t q = j / sg.Ci;
                const int t = (int)(q % sg.taps);
                const int co = (int)(q / sg.taps);
                wt[sg.off + ((int64_t)cc * sg.taps + t) * sg.Co + co] = bb;
            }
        }
    }
}

// the step's losses into a ring of R steps: hist[(t - 1) mod R] = loss[0..2], t = steps[0]
__global__ void k_loss_log(const float* loss, const int64_t* steps, float* hist, int R)
{
    if (threadIdx.x < 3 && blockIdx.x == 0) {
        const int64_t slot = (steps[0] - 1) % R;
        hist[slot * 3 + threadIdx.x] = loss[threadIdx.x];
    }
}

// bf16 copies of FP32 weights and the transpose (initialisation / load)
__global__ void k_weights_to_bf16(const float* w, int64_t n, uint16_t* wb, uint16_t* wt, int Co, int taps, int Ci)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t b = f2bf(w[i]);
        wb[i] = b;
        if (wt) {
            const int ci = (int)(i % Ci);
            const int64_t q = i / Ci;
            const int t = (int)(q % taps);
            const int co = (int)(q / taps);
            wt[((int64_t)ci * taps + t) * Co + co] = b;
        }
    }
}

// per-frame PSNR of clamp(yhat, 0, 1) against y (peak 1): one block per frame
__global__ void k_psnr(const float* yhat, const float* y, int64_t frame, float* psnr)
{
    __shared__ float red[256];
    const float* a = yhat + (int64_t)blockIdx.x * frame;
    const float* b = y + (int64_t)blockIdx.x * frame;
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < frame; i += blockDim.x) {
        const float d = fminf(fmaxf(a[i], 0.f), 1.f) - b[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mse = red[0] / (float)frame;
        psnr[blockIdx.x] = mse > 0.f ? -10.f * log10f(mse) : 200.f;
    }
}

// wt[ci][t][co] = w[co][t][ci] (bf16)
__global__ void k_transpose_w(const uint16_t* w, uint16_t* wt, int Co, int taps, int Ci)
{
    const int64_t n = (int64_t)Co * taps * Ci;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % Ci);
        const int64_t q = i / Ci;
        const int t = (int)(q % taps);
        const int co = (int)(q / taps);
        wt[((int64_t)ci * taps + t) * Co + co] = w[i];
    }
}

// PSNR of clamp(yhat frame idx[b], 0, 1) against target frame b (peak 1)
__global__ void k_psnr_idx(const float* yhat, const float* y, const int32_t* idx, int64_t frame, float* psnr)
{
    __shared__ float red[256];
    const float* a = yhat + (int64_t)idx[blockIdx.x] * frame;
    const float* b = y + (int64_t)blockIdx.x * frame;
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < frame; i += blockDim.x) {
        const float d = fminf(fmaxf(a[i], 0.f), 1.f) - b[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mse = red[0] / (float)frame;
        psnr[blockIdx.x] = mse > 0.f ? -10.f * log10f(mse) : 200.f;
    }
}

__global__ void k_clamp01(const float* x, float* y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fminf(fmaxf(x[i], 0.f), 1.f);
}

int64_t grid_for(int64_t n, int64_t per = 256)
{
    int64_t b = (n + per - 1) / per;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : b;
}

// sum of `splits` rows of n partial results into out, in a fixed order
hipError_t reduce_parts(const float* part, int64_t n, int splits, float* out, hipStream_t s)
{
    if (splits <= 16 || n >= 65536) {
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)grid_for(n)), dim3(256), 0, s, part, n, splits, out);
        return hipGetLastError();
    }
    int ob = 64;   // outputs per block; fewer when that leaves under 256 blocks
    while (ob > 1 && (n + ob - 1) / ob < 256) ob >>= 1;
    hipLaunchKernelGGL(k_sum_parts_grouped, dim3((unsigned)((n + ob - 1) / ob)), dim3(256), 0, s, part, n, splits,
                       out, ob);
    return hipGetLastError();
}

template <int MODE, int BM, int BN, int WM, int WN>
hipError_t launch_gemm(const ConvGeom& g, const ConvArgs& a, int splits, hipStream_t s)
{
    const int64_t gm = (g.M + BM - 1) / BM;
    const int gn = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((k_conv_gemm<MODE, BM, BN, WM, WN>), dim3((unsigned)gm, gn, splits), dim3(kThreads), 0, s,
                       g, a);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------

bool conv_tile_supported(const ConvGeom& g)
{
    const bool shape = g.kh == 3 && g.kw == 3 && g.stride == 1 && g.pad == 1 && (g.Co == 16 || g.Co == 32) &&
                       g.Ho == (g.up ? 2 * g.H : g.H) && g.Wo == (g.up ? 2 * g.W : g.W);
    // 64 input channels only upsampled, where the staged tile is the 10 x 18 stored one
    return shape && (g.C == 8 || g.C == 16 || g.C == 24 || g.C == 32 || (g.C == 64 && g.up && g.Co == 32));
}

template <int C, int CO, bool UP, bool DIL = false>
hipError_t launch_tile(const ConvGeom& g, const ConvArgs& a, hipStream_t s)
{
    constexpr int TH = kTileH;
    const int64_t tiles = (int64_t)((g.Ho + TH - 1) / TH) * ((g.Wo + kTileW - 1) / kTileW);
    const int64_t blocks = tiles * (g.Kw / ((int64_t)g.Ho * g.Wo));   // Kw = N * Ho * Wo
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    if (a.out_f32 && a.accumulate) {   // data gradients accumulated into (never upsampled)
        if constexpr (UP) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((k_conv3x3_tile<C, CO, false, DIL, true, TH>), dim3((unsigned)blocks), dim3(32 * TH), 0, s,
                                g, a);
    } else {
        hipLaunchKernelGGL((k_conv3x3_tile<C, CO, UP, DIL, false, TH>), dim3((unsigned)blocks), dim3(32 * TH), 0, s, g, a);
    }
    return hipGetLastError();
}

template <int CO>
hipError_t launch_tile_co(const ConvGeom& g, const ConvArgs& a, hipStream_t s)
{
    if (g.up) {
        switch (g.C) {
        case 8: return launch_tile<8, CO, true>(g, a, s);
        case 16: return launch_tile<16, CO, true>(g, a, s);
        case 24: return launch_tile<24, CO, true>(g, a, s);
        case 32: return launch_tile<32, CO, true>(g, a, s);
        default:
            if constexpr (CO == 32) return launch_tile<64, 32, true>(g, a, s);
            return hipErrorInvalidValue;
        }
    }
    switch (g.C) {
    case 8: return launch_tile<8, CO, false>(g, a, s);
    case 16: return launch_tile<16, CO, false>(g, a, s);
    case 24: return launch_tile<24, CO, false>(g, a, s);
    default: return launch_tile<32, CO, false>(g, a, s);
    }
}

bool dgrad_tile_supported(const ConvGeom& g)
{
    const int Hin = g.up ? 2 * g.H : g.H, Win = g.up ? 2 * g.W : g.W;
    const bool geom = g.kh == 3 && g.kw == 3 && g.pad == 1 &&
                      ((g.stride == 1 && g.Ho == Hin && g.Wo == Win) ||
                       (g.stride == 2 && !g.up && Hin == 2 * g.Ho && Win == 2 * g.Wo));
    // the forward tile conv's channels: dy's Co in, the layer's C out
    return geom && (g.Co == 8 || g.Co == 16 || g.Co == 24 || g.Co == 32) && (g.C == 16 || g.C == 32);
}

namespace {
template <int CO, bool DIL>
hipError_t launch_dgrad_tile(const ConvGeom& f, const ConvArgs& a, hipStream_t s)
{
    switch (f.C) {
    case 8: return launch_tile<8, CO, false, DIL>(f, a, s);
    case 16: return launch_tile<16, CO, false, DIL>(f, a, s);
    case 24: return launch_tile<24, CO, false, DIL>(f, a, s);
    default: return launch_tile<32, CO, false, DIL>(f, a, s);
    }
}
}  // namespace

hipError_t dgrad_tile(const ConvGeom& g, const uint16_t* dy, const uint16_t* wt, float* dx, int accumulate,
                      hipStream_t s)
{
    if (!dgrad_tile_supported(g)) return hipErrorInvalidValue;
    const int Hin = g.up ? 2 * g.H : g.H, Win = g.up ? 2 * g.W : g.W;
    ConvGeom f = g;   // forward conv: dy (Ho x Wo, Co channels) -> dx (Hin x Win, C channels)
    f.C = g.Co;
    f.Co = g.C;
    f.H = g.Ho;
    f.W = g.Wo;
    f.Ho = Hin;
    f.Wo = Win;
    f.stride = 1;
    f.up = 0;
    f.Kw = (g.Kw / ((int64_t)g.Ho * g.Wo)) * Hin * Win;   // N * Hin * Win
    ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.a = dy;
    a.b = wt;
    a.flip = 1;
    a.out_f32 = dx;
    a.accumulate = accumulate;
    a.pool2 = g.up;   // an upsampled layer's gradient at its stored input resolution
    const bool dil = g.stride == 2;
    if (f.Co == 16) return dil ? launch_dgrad_tile<16, true>(f, a, s) : launch_dgrad_tile<16, false>(f, a, s);
    return dil ? launch_dgrad_tile<32, true>(f, a, s) : launch_dgrad_tile<32, false>(f, a, s);
}

bool dgrad_parity_supported(const ConvGeom& g)
{
    return g.kh == 3 && g.kw == 3 && g.stride == 2 && g.pad == 1 && !g.up && g.Co % 8 == 0 && g.C % 8 == 0 &&
           g.H >= 2 && g.W >= 2;
}

hipError_t dgrad_parity(const ConvGeom& g, const uint16_t* dy, const uint16_t* wt, float* dx, int accumulate,
                        hipStream_t s)
{
    if (!dgrad_parity_supported(g)) return hipErrorInvalidValue;
    if (g.H < 2 || g.W < 2) return hipErrorInvalidValue;   // every class has pixels
    // one launch: class blockIdx.z; the grid covers class 0's rows, the largest class
    const int64_t N = g.Kw / ((int64_t)g.Ho * g.Wo);
    ConvGeom c = g;
    c.par = 4;
    for (int par = 0; par < 4; ++par) {
        c.hc4[par] = (g.H - (par >> 1) + 1) / 2;
        c.wc4[par] = (g.W - (par & 1) + 1) / 2;
        c.f_hw4[par] = make_fastdiv((uint32_t)(c.hc4[par] * c.wc4[par]));
        c.f_w4[par] = make_fastdiv((uint32_t)c.wc4[par]);
    }
    c.M = N * c.hc4[0] * c.wc4[0];
    c.K = 4 * g.Co;   // the largest class's (for the launch shape only)
    c.kb = 9 * g.Co;
    ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.a = dy;
    a.b = wt;
    a.out_f32 = dx;
    a.accumulate = accumulate;
    return conv_gemm(kDgrad, c, a, 1, s);
}

hipError_t conv_gemm(int mode, const ConvGeom& g, const ConvArgs& a, int splits, hipStream_t s)
{
    if (a.head_out && (mode != kFwd || !conv_tile_supported(g) || g.Co != 16 || !a.head_w || !a.head_b))
        return hipErrorInvalidValue;
    if (a.extra && (mode != kFwd || !conv_tile_supported(g) || !a.out2_bf16 || a.extra_c < 8 || a.extra_c % 8 ||
                    g.Co + a.extra_c > a.ld_out2))
        return hipErrorInvalidValue;
    if (mode == kFwd && conv_tile_supported(g))
        return g.Co == 16 ? launch_tile_co<16>(g, a, s) : launch_tile_co<32>(g, a, s);
    if (mode == kWgrad) {
        if (g.M <= 16) return launch_gemm<kWgrad, 16, 128, 1, 4>(g, a, splits, s);
        if (g.M <= 32) return launch_gemm<kWgrad, 32, 128, 1, 4>(g, a, splits, s);
        return launch_gemm<kWgrad, 64, 128, 2, 2>(g, a, splits, s);
    }
    if (mode == kFwd) {
        if (g.N <= 16) return launch_gemm<kFwd, 256, 16, 4, 1>(g, a, 1, s);
        if (g.N <= 32) return launch_gemm<kFwd, 128, 32, 4, 1>(g, a, 1, s);
        if (g.N <= 64) return launch_gemm<kFwd, 128, 64, 2, 2>(g, a, 1, s);
        return launch_gemm<kFwd, 128, 128, 2, 2>(g, a, 1, s);
    }
    // data gradient: splits = 4 only for the parity classes (g.par == 4), one per grid z
    const int nz = g.par == 4 ? 4 : 1;
    if (g.N <= 16) return launch_gemm<kDgrad, 256, 16, 4, 1>(g, a, nz, s);
    if (g.N <= 32) return launch_gemm<kDgrad, 128, 32, 4, 1>(g, a, nz, s);
    if (g.N <= 64) return launch_gemm<kDgrad, 128, 64, 2, 2>(g, a, nz, s);
    return launch_gemm<kDgrad, 128, 128, 2, 2>(g, a, nz, s);
}

bool wgrad_tile_plan(const ConvGeom& g, WgradTilePlan* plan)
{
    const bool s1 = g.stride == 1 && g.Ho == (g.up ? 2 * g.H : g.H) && g.Wo == (g.up ? 2 * g.W : g.W);
    const bool s2 = g.stride == 2 && !g.up && g.Ho == (g.H - 1) / 2 + 1 && g.Wo == (g.W - 1) / 2 + 1;
    if (!(g.kh == 3 && g.kw == 3 && g.pad == 1 && (s1 || s2))) return false;
    int ci_g = 0, co_g = 0;
    if (g.C == 8 || g.C == 16 || g.C == 24 || g.C == 32)
        ci_g = g.C;
    else if (g.C % 32 == 0 && g.Wo >= 16)   // wider layers in groups of 32 (tiles at least half full)
        ci_g = 32;
    if (g.Co == 16 || g.Co == 32)
        co_g = g.Co;
    else if (g.Co % 32 == 0 && g.Wo >= 16)
        co_g = 32;
    if (!ci_g || !co_g) return false;
    if (plan) {
        const int gy = g.C / ci_g, gz = g.Co / co_g;
        const int th = g.stride == 2 ? kWgH2 : kWgH;
        const int64_t tiles = (g.Kw / ((int64_t)g.Ho * g.Wo)) * (int64_t)((g.Ho + th - 1) / th) *
                              ((g.Wo + kWgW - 1) / kWgW);
        const int64_t want = std::max<int64_t>(1, (512 + gy * gz - 1) / (gy * gz));   // about 512 blocks
        plan->gx = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), want);
        plan->gy = gy;
        plan->gz = gz;
        plan->ci_g = ci_g;
        plan->co_g = co_g;
    }
    return true;
}

int64_t wgrad_tile_part_floats(const WgradTilePlan& p)
{
    return (int64_t)p.gx * p.gy * p.gz * p.co_g * 9 * p.ci_g;   // gx partials of the whole dW
}

namespace {
template <int CI, int CO, bool UP>
hipError_t launch_wgrad_tile3(const ConvGeom& g, const uint16_t* x, const uint16_t* dy, float* part,
                              const WgradTilePlan& p, hipStream_t s)
{
    if (g.stride == 2) {
        if constexpr (UP) return hipErrorInvalidValue;
        else
            hipLaunchKernelGGL((k_wgrad3x3_tile<CI, CO, false, true>), dim3(p.gx, p.gy, p.gz), dim3(256), 0, s, g,
                               x, dy, part);
    } else {
        hipLaunchKernelGGL((k_wgrad3x3_tile<CI, CO, UP, false>), dim3(p.gx, p.gy, p.gz), dim3(256), 0, s, g, x, dy,
                           part);
    }
    return hipGetLastError();
}

template <int CO, bool UP>
hipError_t launch_wgrad_tile2(const ConvGeom& g, const uint16_t* x, const uint16_t* dy, float* part,
                              const WgradTilePlan& p, hipStream_t s)
{
    switch (p.ci_g) {
    case 8: return launch_wgrad_tile3<8, CO, UP>(g, x, dy, part, p, s);
    case 16: return launch_wgrad_tile3<16, CO, UP>(g, x, dy, part, p, s);
    case 24: return launch_wgrad_tile3<24, CO, UP>(g, x, dy, part, p, s);
    case 32: return launch_wgrad_tile3<32, CO, UP>(g, x, dy, part, p, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t wgrad_tile(const ConvGeom& g, const uint16_t* x, const uint16_t* dy, float* part, const WgradTilePlan& p,
                      float* dw, hipStream_t s)
{
    WgradTilePlan q;
    if (!wgrad_tile_plan(g, &q) || q.gx != p.gx || q.gy != p.gy || q.gz != p.gz || q.ci_g != p.ci_g ||
        q.co_g != p.co_g)
        return hipErrorInvalidValue;
    hipError_t e;
    if (p.co_g == 16)
        e = g.up ? launch_wgrad_tile2<16, true>(g, x, dy, part, p, s) : launch_wgrad_tile2<16, false>(g, x, dy, part, p, s);
    else
        e = g.up ? launch_wgrad_tile2<32, true>(g, x, dy, part, p, s) : launch_wgrad_tile2<32, false>(g, x, dy, part, p, s);
    if (e != hipSuccess) return e;
    return reduce_parts(part, (int64_t)g.Co * 9 * g.C, p.gx, dw, s);
}

int wgrad_tile_m(int M) { return M <= 16 ? 16 : (M <= 32 ? 32 : 64); }

hipError_t mask_colsum(const float* g, int ldg, const uint16_t* y, uint16_t* out, int64_t rows, int C, float* part,
                       int blocks, float* bias_grad, hipStream_t s, float slope)
{
    if (C > 256 || C % 8 || (ldg != 0 && (ldg < C || ldg % 4))) return hipErrorInvalidValue;
    const int64_t per = (rows + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_mask_colsum, dim3(blocks), dim3(256), 0, s, g, ldg ? ldg : C, nullptr, y, out, rows, C, per,
                       part, slope);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !bias_grad) return e;
    return reduce_parts(part, C, blocks, bias_grad, s);
}

hipError_t reduce_segments(const float* part, float* out, const ReduceSegs& t, hipStream_t s)
{
    if (t.count < 1 || t.count > kMaxReduceSegs) return hipErrorInvalidValue;
    const ReduceSeg& last = t.s[t.count - 1];
    hipLaunchKernelGGL(k_reduce_segments, dim3((unsigned)(last.first + last.n)), dim3(256), 0, s, part, out, t);
    return hipGetLastError();
}

int depth_scan_blocks(int N, int W)
{
    return (int)(((int64_t)N * W + kScanCols - 1) / kScanCols);
}

hipError_t depth_map_scan_fwd(const uint16_t* e, const uint16_t* w, const float* b, uint16_t* out, int N, int H,
                              int W, float scale, int ld, int c_off, hipStream_t s)
{
    if (ld % 8 || c_off % 8 || c_off + kScanC > ld) return hipErrorInvalidValue;
    if (H <= kScan1Seg * kScan1Rows) {   // one read of e
        const int64_t blocks = ((int64_t)N * W + kScan1Cols - 1) / kScan1Cols;
        hipLaunchKernelGGL(k_depth_map_scan_fwd1, dim3((unsigned)blocks), dim3(256), 0, s, e, w, b, out, N, H, W, scale,
                           ld, c_off);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_depth_map_scan_fwd, dim3((unsigned)depth_scan_blocks(N, W)), dim3(256), 0, s, e, w, b, out, N,
                       H, W, scale, ld, c_off);
    return hipGetLastError();
}

hipError_t depth_scan_bwd(const float* g, int ld, int c_off, float* g_skip, uint16_t* dp, float* part,
                          float* bias_grad, int N, int H, int W, float scale, hipStream_t s)
{
    if (ld % 4 || c_off % 4 || c_off + kScanC > ld) return hipErrorInvalidValue;
    const int blocks = depth_scan_blocks(N, W);
    hipLaunchKernelGGL(k_depth_scan_bwd, dim3((unsigned)blocks), dim3(256), 0, s, g, ld, c_off, g_skip, dp, part, N,
                       H, W, scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, kScanC, blocks, bias_grad, s);
}

hipError_t proj_bwd(const uint16_t* dp, const uint16_t* x, const uint16_t* w, float* g, int64_t P, int KC, int C,
                    float* part, float* dw, hipStream_t s)
{
    if (KC != 8 || C != 16 || P < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_proj_bwd<8, 16>), dim3(kProjBlocks), dim3(256), 0, s, dp, x, w, g, P, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, KC * C, kProjBlocks, dw, s);
}

int proj_bwd_blocks() { return kProjBlocks; }

hipError_t mask_to_bf16(const float* g, const uint16_t* y, uint16_t* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask_to_bf16, dim3((unsigned)grid_for(n)), dim3(256), 0, s, g, y, out, n);
    return hipGetLastError();
}

hipError_t pool2x2_sum(const float* fine, float* coarse, int N, int H, int W, int C, int accumulate, hipStream_t s)
{
    const int64_t n = (int64_t)N * H * W * C;
    hipLaunchKernelGGL(k_pool2x2_sum, dim3((unsigned)grid_for(n)), dim3(256), 0, s, fine, coarse, N, H, W, C,
                       accumulate);
    return hipGetLastError();
}

hipError_t colsum_bf16(const uint16_t* x, int64_t rows, int cols, float* part, int blocks, float* out,
                       hipStream_t s)
{
    if (cols > 256 || cols % 8) return hipErrorInvalidValue;
    const int64_t per = (rows + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_mask_colsum, dim3(blocks), dim3(256), 0, s, nullptr, cols, x, nullptr, nullptr, rows, cols,
                       per, part, 0.f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, cols, blocks, out, s);
}

hipError_t sum_parts(const float* part, int64_t n, int splits, float* out, hipStream_t s)
{
    return reduce_parts(part, n, splits, out, s);
}

hipError_t head_fwd(const uint16_t* x, const uint16_t* w, const float* b, float* y, int64_t P, int C, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)grid_for(P)), dim3(256), 0, s, x, w, b, y, P, C);
    return hipGetLastError();
}

hipError_t head_bwd(const uint16_t* x, const uint16_t* w, const float* g, float* dx, int64_t P, int C, float* part,
                    int blocks, float* dwb, hipStream_t s)
{
    const int64_t per = (P + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_head_bwd, dim3(blocks), dim3(256), 0, s, x, w, g, dx, P, C, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, 17, blocks, dwb, s);
}

hipError_t l1_loss(const float* yhat, const float* y, int64_t n, float* grad, float* part, int blocks, float* loss,
                   hipStream_t s)
{
    const int64_t per = (n + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_l1, dim3(blocks), dim3(256), 0, s, yhat, y, n, 1.f / (float)n, grad, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, 1, blocks, loss, s);
}

hipError_t disc_input(const uint16_t* x, const float* y_real, const float* y_fake, uint16_t* z, int64_t P,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_disc_input, dim3((unsigned)grid_for(2 * P)), dim3(256), 0, s, x, y_real, y_fake, z, P);
    return hipGetLastError();
}

hipError_t bce_logits(const float* logits, int ld, int64_t P_real, int64_t P_total, float w_real, float w_fake,
                      float gscale, float* grad, float* part, int blocks, float* loss, hipStream_t s)
{
    const int64_t per = (P_total + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_bce_logits, dim3(blocks), dim3(256), 0, s, logits, ld, P_real, P_total, w_real, w_fake,
                       gscale, grad, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, 1, blocks, loss, s);
}

hipError_t add_channel(float* gy, const float* dz, int ld, int c, int64_t P, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_channel, dim3((unsigned)grid_for(P)), dim3(256), 0, s, gy, dz, ld, c, P);
    return hipGetLastError();
}

int adam_blocks(int64_t n) { return (int)((n + kAdamChunk - 1) / kAdamChunk); }

hipError_t adam_coef(int64_t* steps, float* coef, float lr, float b1, float b2, int disc, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam_coef, dim3(1), dim3(64), 0, s, steps, coef, lr, b1, b2, disc);
    return hipGetLastError();
}

hipError_t adam_multi(const AdamSeg* segs, int nseg, int blocks, float* w, float* m, float* v, const float* g,
                      uint16_t* wb, uint16_t* wt, const float* coef, int ci, float b1, float b2, float eps,
                      hipStream_t s)
{
    if (nseg < 1 || blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adam_multi, dim3((unsigned)blocks), dim3(256), 0, s, segs, nseg, w, m, v, g, wb, wt, coef, ci,
                       b1, b2, eps);
    return hipGetLastError();
}

hipError_t loss_log(const float* loss, const int64_t* steps, float* hist, int R, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_log, dim3(1), dim3(64), 0, s, loss, steps, hist, R);
    return hipGetLastError();
}

hipError_t weights_to_bf16(const float* w, int64_t n, uint16_t* wb, uint16_t* wt, int Co, int taps, int Ci,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_weights_to_bf16, dim3((unsigned)grid_for(n)), dim3(256), 0, s, w, n, wb, wt, Co, taps, Ci);
    return hipGetLastError();
}

hipError_t transpose_w(const uint16_t* w, uint16_t* wt, int Co, int taps, int Ci, hipStream_t s)
{
    const int64_t n = (int64_t)Co * taps * Ci;
    hipLaunchKernelGGL(k_transpose_w, dim3((unsigned)grid_for(n)), dim3(256), 0, s, w, wt, Co, taps, Ci);
    return hipGetLastError();
}

hipError_t psnr_indexed(const float* yhat, const float* y, const int32_t* idx, int n_frames, int64_t frame,
                        float* psnr, hipStream_t s)
{
    if (n_frames <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_psnr_idx, dim3(n_frames), dim3(256), 0, s, yhat, y, idx, frame, psnr);
    return hipGetLastError();
}

hipError_t clamp01(const float* x, float* y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clamp01, dim3((unsigned)grid_for(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t psnr_frames(const float* yhat, const float* y, int n_frames, int64_t frame, float* psnr, hipStream_t s)
{
    if (n_frames <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_psnr, dim3(n_frames), dim3(256), 0, s, yhat, y, frame, psnr);
    return hipGetLastError();
}

}  // namespace sg
