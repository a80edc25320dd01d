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
// v_mfma_f32_16x16x32_bf16; operands are staged through double-buffered LDS
// (rows padded to 80 bytes).  The forward / data-gradient operands are
// contiguous along K and are written to LDS with 16-byte stores; the
// weight-gradient operands are contiguous along the channel (M / N) axis and
// are transposed into LDS.  The weight gradient splits K (pixels) over
// blocks and sums the partial tiles in a fixed order (deterministic).
// A conv may read its input through a nearest-neighbour x2 upsampling
// (decoder layers): the gather maps (h, w) to (h / 2, w / 2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "surrogate_internal.h"

namespace sg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte staging chunk

constexpr int kThreads = 256;
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

enum Mode { kFwd = 0, kDgrad = 1, kWgrad = 2 };

template <int MODE, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(kThreads) void k_conv_gemm(ConvGeom g, ConvArgs a)
{
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    static_assert(WM * WN == 4, "four waves");
    static_assert(FM >= 1 && FN >= 1, "tile");
    // staged 16-byte chunks per K step: K-contiguous operands are (row, 8 k)
    // chunks, the weight gradient's are (8 rows, k) chunks
    constexpr int CA = (MODE == kWgrad) ? (BM / 8) * kBK : BM * (kBK / 8);
    constexpr int CB = (MODE == kWgrad) ? (BN / 8) * kBK : BN * (kBK / 8);
    constexpr int PA = (CA + kThreads - 1) / kThreads;
    constexpr int PB = (CB + kThreads - 1) / kThreads;
    constexpr int AM8 = BM / 8, BN8 = BN / 8;   // weight-gradient row groups

    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * kBKP];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * kBKP];

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
    // K-contiguous modes: chunk c = tid + i * 256 -> (row c / 4, k8 = tid % 4)
    const int k8 = tid & 3;
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
                    const int n = (int)fdiv((uint32_t)m, g.f_hinwin);
                    const int rem = m - n * Hin * Win;
                    const int h = (int)fdiv((uint32_t)rem, g.f_win);
                    const int w = rem - h * Win;
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
                const int c = tid + i * kThreads;
                const int64_t k = k0 + c / AM8;
                ra[i] = (c < CA && wg_m0 < g.M && k < k_end)
                            ? *reinterpret_cast<const u32x4*>(A + k * g.Co + wg_m0)
                            : zero;
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const int c = tid + i * kThreads;
                const int64_t k = k0 + c / BN8;
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
        int r = 0, s = 0, c0 = 0;
        if (kin) {
            const FastDiv fc = (MODE == kFwd) ? g.f_c : g.f_co;
            const int cc = (MODE == kFwd) ? g.C : g.Co;
            const int t = (int)fdiv((uint32_t)k, fc);
            c0 = k - t * cc;
            r = (int)fdiv((uint32_t)t, g.f_kw);
            s = t - r * g.kw;
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
                        ? *reinterpret_cast<const u32x4*>(B + (int64_t)col * g.K + k)
                        : zero;
        }
    };
    auto store_tiles = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int c = tid + i * kThreads;
            if (c >= CA) continue;
            if constexpr (MODE == kWgrad) {
                const int m8 = c % AM8, kk = c / AM8;
                const u32x4 w4 = ra[i];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    sA[buf][(m8 * 8 + j) * kBKP + kk] = (uint16_t)(w4[j >> 1] >> ((j & 1) * 16));
            } else {
                *reinterpret_cast<u32x4*>(&sA[buf][(c >> 2) * kBKP + k8 * 8]) = ra[i];
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int c = tid + i * kThreads;
            if (c >= CB) continue;
            if constexpr (MODE == kWgrad) {
                const int n8 = c % BN8, kk = c / BN8;
                const u32x4 w4 = rb[i];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    sB[buf][(n8 * 8 + j) * kBKP + kk] = (uint16_t)(w4[j >> 1] >> ((j & 1) * 16));
            } else {
                *reinterpret_cast<u32x4*>(&sB[buf][(c >> 2) * kBKP + k8 * 8]) = rb[i];
            }
        }
    };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (nk > 0) {
        load_tiles(k_begin);
        store_tiles(0);
    }
    __syncthreads();
    const int frow = lane & 15, fk = (lane >> 4) * 8;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_tiles(k_begin + (int64_t)(kt + 1) * kBK);
        bf16x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            fa[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][(wm * TM + i * 16 + frow) * kBKP + fk]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            fb[j] = *reinterpret_cast<const bf16x8*>(&sB[buf][(wn * TN + j * 16 + frow) * kBKP + fk]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) store_tiles(buf ^ 1);
        __syncthreads();
    }

    // epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each tile
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n_base + wn * TN + j * 16 + (lane & 15);
            if (col >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = (int64_t)m_base + wm * TM + i * 16 + (lane >> 4) * 4 + r;
                if (row >= g.M) continue;
                const float v = acc[i][j][r];
                if constexpr (MODE == kFwd) {
                    float y = v + (a.bias ? a.bias[col] : 0.f);
                    if (a.relu) y = fmaxf(y, 0.f);
                    const int64_t o = row * g.Co + col;
                    const uint16_t yb = f2bf(y);
                    if (a.out_bf16) a.out_bf16[o] = yb;
                    if (a.out_f32) a.out_f32[o] = y;
                    if (a.skip && a.out2_bf16)
                        a.out2_bf16[row * (a.ld_out2 ? a.ld_out2 : g.Co) + col] = f2bf(bf2f(yb) + bf2f(a.skip[o]));
                } else if constexpr (MODE == kDgrad) {
                    const int64_t o = row * g.C + col;
                    a.out_f32[o] = a.accumulate ? a.out_f32[o] + v : v;
                } else {
                    a.out_f32[(int64_t)blockIdx.z * g.M * g.N + row * g.N + col] = v;
                }
            }
        }
    }
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
                                                     float* part)
{
    __shared__ float red[256];
    const int lanes = 256 / C;
    const int c = threadIdx.x % C;
    const int r_off = threadIdx.x / C;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    float s = 0.f;
    if (r_off < lanes) {
        for (int64_t r = r0 + r_off; r < r1; r += lanes) {
            const int64_t i = r * C + c;
            uint16_t b;
            if (gb) {
                b = gb[i];
            } else {
                b = f2bf((y == nullptr || bf2f(y[i]) > 0.f) ? g[r * ldg + c] : 0.f);
                if (out) out[i] = b;
            }
            s += bf2f(b);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (r_off == 0) {
        float t = 0.f;
        for (int j = 0; j < lanes; ++j) t += red[j * C + c];
        part[(int64_t)blockIdx.x * C + c] = t;
    }
}

// out[i] = sum_s part[s][i] in fixed order
// Depth integral along the beam.  One wave per (frame, column), grid-stride
// over columns; lanes run along depth in chunks of 64 rows.  Each chunk is a
// Hillis-Steele scan over the wave (lane shuffles) plus the running total of
// the chunks already done.  Eight channels per pixel (kScanC).
constexpr int kScanC = 8;

__device__ __forceinline__ float lane_get(float v, int src) { return __shfl(v, src, 64); }

// out[n][y][x][c_off + k] = bf16(scale * sum_{v < y} p[n][v][x][k])
__global__ __launch_bounds__(256) void k_depth_scan_fwd(const float* __restrict__ p, uint16_t* __restrict__ out,
                                                        int N, int H, int W, float scale, int ld, int c_off)
{
    const int lane = threadIdx.x & 63;
    const int64_t n_cols = (int64_t)N * W;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t col = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); col < n_cols; col += waves) {
        const int64_t n = col / W;
        const int x = (int)(col - n * W);
        float carry[kScanC];
#pragma unroll
        for (int k = 0; k < kScanC; ++k) carry[k] = 0.f;
        for (int y0 = 0; y0 < H; y0 += 64) {
            const int y = y0 + lane;
            const int64_t px = (n * H + y) * W + x;
            float v[kScanC];
            if (y < H) {
                const float4 a = *reinterpret_cast<const float4*>(p + px * kScanC);
                const float4 b = *reinterpret_cast<const float4*>(p + px * kScanC + 4);
                v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
            } else {
#pragma unroll
                for (int k = 0; k < kScanC; ++k) v[k] = 0.f;
            }
            // exclusive: shift down by one lane, then an inclusive scan
#pragma unroll
            for (int k = 0; k < kScanC; ++k) {
                float e = lane_get(v[k], lane - 1);
                e = lane > 0 ? e : 0.f;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const float t = lane_get(e, lane - d);
                    if (lane >= d) e += t;
                }
                const float tot = lane_get(e + v[k], 63);
                v[k] = carry[k] + e;
                carry[k] += tot;
            }
            if (y < H) {
                u32x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    o[j] = (uint32_t)f2bf(scale * v[2 * j]) | ((uint32_t)f2bf(scale * v[2 * j + 1]) << 16);
                *reinterpret_cast<u32x4*>(out + px * ld + c_off) = o;
            }
        }
    }
}

// Backward of k_depth_scan_fwd through a tensor g [pixel][ld] (FP32) whose
// channels [c_off, c_off + 8) are the integral's gradient:
//   dp[n][v][x][k] = bf16(scale * sum_{y > v} g[n][y][x][c_off + k]),
// channels [0, c_off) copied to g_skip [pixel][c_off], and per-block column
// sums of the bf16 dp (bias gradient partials) in part[block][8].
__global__ __launch_bounds__(256) void k_depth_scan_bwd(const float* __restrict__ g, int ld, int c_off,
                                                        float* __restrict__ g_skip, uint16_t* __restrict__ dp,
                                                        float* __restrict__ part, int N, int H, int W, float scale)
{
    __shared__ float red[4][kScanC];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t n_cols = (int64_t)N * W;
    const int64_t waves = (int64_t)gridDim.x * 4;
    float bsum[kScanC];
#pragma unroll
    for (int k = 0; k < kScanC; ++k) bsum[k] = 0.f;
    for (int64_t col = (int64_t)blockIdx.x * 4 + wave; col < n_cols; col += waves) {
        const int64_t n = col / W;
        const int x = (int)(col - n * W);
        float carry[kScanC];
#pragma unroll
        for (int k = 0; k < kScanC; ++k) carry[k] = 0.f;
        const int n_chunks = (H + 63) / 64;
        for (int ch = n_chunks - 1; ch >= 0; --ch) {
            const int y = ch * 64 + lane;
            const int64_t px = (n * H + y) * W + x;
            float v[kScanC];
            if (y < H) {
                const float* src = g + px * ld;
                for (int c = 0; c < c_off; c += 4)
                    *reinterpret_cast<float4*>(g_skip + px * c_off + c) = *reinterpret_cast<const float4*>(src + c);
                const float4 a = *reinterpret_cast<const float4*>(src + c_off);
                const float4 b = *reinterpret_cast<const float4*>(src + c_off + 4);
                v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
            } else {
#pragma unroll
                for (int k = 0; k < kScanC; ++k) v[k] = 0.f;
            }
            // exclusive suffix: shift up by one lane, then an inclusive suffix scan
#pragma unroll
            for (int k = 0; k < kScanC; ++k) {
                float e = lane_get(v[k], lane + 1);
                e = lane < 63 ? e : 0.f;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const float t = lane_get(e, lane + d);
                    if (lane + d < 64) e += t;
                }
                const float tot = lane_get(e + v[k], 0);
                v[k] = carry[k] + e;
                carry[k] += tot;
            }
            if (y < H) {
                u32x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint16_t lo = f2bf(scale * v[2 * j]), hi = f2bf(scale * v[2 * j + 1]);
                    bsum[2 * j] += bf2f(lo);
                    bsum[2 * j + 1] += bf2f(hi);
                    o[j] = (uint32_t)lo | ((uint32_t)hi << 16);
                }
                *reinterpret_cast<u32x4*>(dp + px * kScanC) = o;
            }
        }
    }
    // fixed-order reduction: wave butterfly, then the block's four waves
#pragma unroll
    for (int k = 0; k < kScanC; ++k) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) bsum[k] += lane_get(bsum[k], lane ^ d);
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kScanC; ++k) red[wave][k] = bsum[k];
    __syncthreads();
    if (threadIdx.x < kScanC)
        part[(int64_t)blockIdx.x * kScanC + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void k_sum_parts(const float* part, int64_t n, int splits, float* out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + i];
        out[i] = s;
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
__global__ void k_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* wb, uint16_t* wt, int Co, int taps, int Ci)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (wb) {
            const uint16_t b = f2bf(wi);
            wb[i] = b;
            if (wt) {
                // i = (co * taps + t) * Ci + ci  ->  (ci * taps + t) * Co + co
                const int ci = (int)(i % Ci);
                const int64_t q = i / Ci;
                const int t = (int)(q % taps);
                const int co = (int)(q / taps);
                wt[((int64_t)ci * taps + t) * Co + co] = b;
            }
        }
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

hipError_t conv_gemm(int mode, const ConvGeom& g, const ConvArgs& a, int splits, hipStream_t s)
{
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
    if (g.N <= 16) return launch_gemm<kDgrad, 256, 16, 4, 1>(g, a, 1, s);
    if (g.N <= 32) return launch_gemm<kDgrad, 128, 32, 4, 1>(g, a, 1, s);
    if (g.N <= 64) return launch_gemm<kDgrad, 128, 64, 2, 2>(g, a, 1, s);
    return launch_gemm<kDgrad, 128, 128, 2, 2>(g, a, 1, s);
}

int wgrad_tile_m(int M) { return M <= 16 ? 16 : (M <= 32 ? 32 : 64); }

hipError_t mask_colsum(const float* g, int ldg, const uint16_t* y, uint16_t* out, int64_t rows, int C, float* part,
                       int blocks, float* bias_grad, hipStream_t s)
{
    if (C > 256 || (ldg != 0 && ldg < C)) return hipErrorInvalidValue;
    const int64_t per = (rows + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_mask_colsum, dim3(blocks), dim3(256), 0, s, g, ldg ? ldg : C, nullptr, y, out, rows, C, per,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)grid_for(C)), dim3(256), 0, s, part, (int64_t)C, blocks, bias_grad);
    return hipGetLastError();
}

int depth_scan_blocks(int N, int W)
{
    const int64_t b = ((int64_t)N * W + 3) / 4;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

hipError_t depth_scan_fwd(const float* p, uint16_t* out, int N, int H, int W, float scale, int ld, int c_off,
                          hipStream_t s)
{
    if (ld % 8 || c_off % 8 || c_off + kScanC > ld) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_depth_scan_fwd, dim3((unsigned)depth_scan_blocks(N, W)), dim3(256), 0, s, p, out, N, H, W,
                       scale, ld, c_off);
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
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, (int64_t)kScanC, blocks, bias_grad);
    return hipGetLastError();
}

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
    if (cols > 256) return hipErrorInvalidValue;
    const int64_t per = (rows + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_mask_colsum, dim3(blocks), dim3(256), 0, s, nullptr, cols, x, nullptr, nullptr, rows, cols,
                       per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)grid_for(cols)), dim3(256), 0, s, part, (int64_t)cols, blocks, out);
    return hipGetLastError();
}

hipError_t sum_parts(const float* part, int64_t n, int splits, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)grid_for(n)), dim3(256), 0, s, part, n, splits, out);
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, (int64_t)17, blocks, dwb);
    return hipGetLastError();
}

hipError_t l1_loss(const float* yhat, const float* y, int64_t n, float* grad, float* part, int blocks, float* loss,
                   hipStream_t s)
{
    const int64_t per = (n + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_l1, dim3(blocks), dim3(256), 0, s, yhat, y, n, 1.f / (float)n, grad, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, (int64_t)1, blocks, loss);
    return hipGetLastError();
}

hipError_t adam_step(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                     float c1, float c2, uint16_t* wb, uint16_t* wt, int Co, int taps, int Ci, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((unsigned)grid_for(n)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1, c2,
                       wb, wt, Co, taps, Ci);
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
