// Internal declarations of the surrogate network's kernels (conv_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

// Division by a fixed divisor d (1 <= d < 2^31) for dividends n < 2^31 by one
// multiply-high and a shift (Granlund & Montgomery, "Division by invariant
// integers using multiplication", PLDI 1994): q = (mulhi(n, m) + n) >> s with
// s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    const uint64_t m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, s};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.s);
}

// GEMM view of one convolution product (see conv_mfma.hip).
struct ConvGeom {
    int64_t M;      // GEMM rows
    int32_t N;      // GEMM columns
    int32_t K;      // reduction length (forward / data gradient)
    int64_t Kw;     // reduction length of the weight gradient (pixels)
    int32_t C, Co;  // input / output channels
    int32_t H, W;   // stored input size (before the optional x2 upsampling)
    int32_t Ho, Wo; // output size
    int32_t kh, kw, stride, pad, up;
    FastDiv f_c, f_co, f_kw, f_stride, f_howo, f_wo, f_hinwin, f_win;
    int32_t kb;     // elements per row of the GEMM's B operand (forward W, data gradient WT): K, or 9 Co
    // data gradient of a stride-2, pad-1 3x3 conv split by output parity (par = 2 (h % 2) + (w % 2), or
    // -1): rows are the Hc x Wc pixels (2 i + h % 2, 2 j + w % 2) of each image, K the Co x taps that
    // reach them (f_hinwin and f_win then divide by Hc Wc and Wc).  par = 4: all four classes in one
    // launch, class blockIdx.z, with its sizes and divisors in the arrays below
    int32_t par, Hc, Wc;
    int32_t hc4[4], wc4[4];
    FastDiv f_hw4[4], f_w4[4];
};

constexpr float kLeakySlope = 0.2f;   // leaky ReLU of the discriminator

struct ConvArgs {
    const uint16_t* a;       // forward: x; data gradient: dy; weight gradient: dy
    const uint16_t* b;       // forward: W [Co][K]; data gradient: WT [Ci][K]; weight gradient: x
    const float* bias;       // forward, may be null
    int32_t relu;            // forward activation: 0 none, 1 ReLU, 2 leaky ReLU (kLeakySlope)
    const uint16_t* skip;    // forward: second output = out + skip (may be null)
    uint16_t* out2_bf16;
    int32_t ld_out2;         // channels per pixel of out2 (0: Co); out2 may be wider than the conv's output
    uint16_t* out_bf16;      // forward
    float* out_f32;          // forward (optional), data gradient, weight gradient partials
    int32_t accumulate;      // data gradient: add into out_f32
    int64_t k_chunk;         // weight gradient: pixels per split (multiple of 32)
    // forward, tiled 3x3 path only (conv_tile_supported): fused 1x1 head with one output,
    // head_out[pixel] = head_b[0] + sum_co head_w[co] * bf16(out[pixel][co])
    const uint16_t* head_w;
    const float* head_b;
    float* head_out;
    // forward, tiled 3x3 path only: out2's channels [Co, Co + extra_c) are copied from extra
    // [pixel][extra_c] (extra_c multiple of 8, Co + extra_c <= ld_out2), so out2 is written whole
    const uint16_t* extra;
    int32_t extra_c;
    // tiled 3x3 path only: b is the transposed copy [C][9][Co] of a layer's weights and the taps are
    // read mirrored (the data gradient as a forward conv of dy)
    int32_t flip;
    // tiled 3x3 path only, with out_f32: the output's 2 x 2 blocks summed into one pixel of a half-size
    // out_f32 (the data gradient of an upsampled input); Ho and Wo even
    int32_t pool2;
};

// convolution shape of one layer (per batch)
struct ConvShape {
    int N, H, W, C, Co, k, stride, pad, up;
    int Hin() const { return up ? 2 * H : H; }
    int Win() const { return up ? 2 * W : W; }
    int Ho() const { return (Hin() + 2 * pad - k) / stride + 1; }
    int Wo() const { return (Win() + 2 * pad - k) / stride + 1; }
};

inline ConvGeom geom_of(const ConvShape& s, int mode)
{
    ConvGeom g;
    g.C = s.C;
    g.Co = s.Co;
    g.H = s.H;
    g.W = s.W;
    g.Ho = s.Ho();
    g.Wo = s.Wo();
    g.kh = g.kw = s.k;
    g.stride = s.stride;
    g.pad = s.pad;
    g.up = s.up;
    g.Kw = (int64_t)s.N * g.Ho * g.Wo;
    g.f_c = make_fastdiv((uint32_t)s.C);
    g.f_co = make_fastdiv((uint32_t)s.Co);
    g.f_kw = make_fastdiv((uint32_t)s.k);
    g.f_stride = make_fastdiv((uint32_t)s.stride);
    g.f_howo = make_fastdiv((uint32_t)(g.Ho * g.Wo));
    g.f_wo = make_fastdiv((uint32_t)g.Wo);
    g.f_hinwin = make_fastdiv((uint32_t)(s.Hin() * s.Win()));
    g.f_win = make_fastdiv((uint32_t)s.Win());
    if (mode == 0) {
        g.M = (int64_t)s.N * g.Ho * g.Wo;
        g.N = s.Co;
        g.K = s.k * s.k * s.C;
    } else if (mode == 1) {
        g.M = (int64_t)s.N * s.Hin() * s.Win();
        g.N = s.C;
        g.K = s.k * s.k * s.Co;
    } else {
        g.M = s.Co;
        g.N = s.k * s.k * s.C;
        g.K = 0;
    }
    g.kb = g.K;
    g.par = -1;
    g.Hc = g.Wc = 0;
    return g;
}

hipError_t conv_gemm(int mode, const ConvGeom& g, const ConvArgs& a, int splits, hipStream_t s);
// forward shapes served by the LDS-tiled direct 3x3 kernel (stride 1, pad 1, C in {8, 16, 24, 32},
// Co in {16, 32}); the fused head needs Co = 16
bool conv_tile_supported(const ConvGeom& g);
// data gradient of a 3x3 pad-1 conv (g: the layer's mode-1 geometry; stride 1, or stride 2 with even input
// sizes) as a forward tiled conv of dy with mirrored taps, over dy dilated by zeros for stride 2: dx
// [N][H][W][C] FP32 at the stored input resolution (an upsampled layer's fine-resolution gradient summed
// over 2 x 2 blocks in the epilogue), written or accumulated
bool dgrad_tile_supported(const ConvGeom& g);
// data gradient of a stride-2, pad-1 3x3 conv (g: mode-1 geometry) as four implicit GEMMs, one per output
// parity class, each over only the taps that reach it (a quarter of the full gather's products)
bool dgrad_parity_supported(const ConvGeom& g);
hipError_t dgrad_parity(const ConvGeom& g, const uint16_t* dy, const uint16_t* wt, float* dx, int accumulate,
                        hipStream_t s);
hipError_t dgrad_tile(const ConvGeom& g, const uint16_t* dy, const uint16_t* wt, float* dx, int accumulate,
                      hipStream_t s);
int wgrad_tile_m(int M);
// direct 3x3 weight gradient (stride 1 or 2, pad 1; C in {8, 16, 24, 32} or a multiple of 32, Co in {16, 32}
// or a multiple of 32, the wider ones for outputs at least 16 wide): gx x gy x gz blocks (gy input and gz
// output channel groups of ci_g and co_g) write gx partials of the whole dW (the gy x gz blocks with one
// block x index fill one partial), then a fixed-order reduction over the gx partials writes dw ([Co][3][3][C])
struct WgradTilePlan {
    int gx = 0, gy = 0, gz = 0, ci_g = 0, co_g = 0;
};
bool wgrad_tile_plan(const ConvGeom& g, WgradTilePlan* plan);
int64_t wgrad_tile_part_floats(const WgradTilePlan& p);
hipError_t wgrad_tile(const ConvGeom& g, const uint16_t* x, const uint16_t* dy, float* part, const WgradTilePlan& p,
                      float* dw, hipStream_t s);
hipError_t mask_to_bf16(const float* g, const uint16_t* y, uint16_t* out, int64_t n, hipStream_t s);
// out = bf16(g * (y > 0 ? 1 : slope)) over [rows][C] (y null: out = bf16(g)) and bias_grad[c] = sum of
// out's column c (C <= 256); g has ldg floats per row (0: C)
hipError_t mask_colsum(const float* g, int ldg, const uint16_t* y, uint16_t* out, int64_t rows, int C, float* part,
                       int blocks, float* bias_grad, hipStream_t s, float slope = 0.f);
// discriminator input of P real and P fake pixels (see k_disc_input)
hipError_t disc_input(const uint16_t* x, const float* y_real, const float* y_fake, uint16_t* z, int64_t P,
                      hipStream_t s);
// binary cross-entropy on logits (channel 0 of rows of ld floats): rows < P_real label 1, the rest label 0;
// *loss = sum of w * softplus(-+l), grad = gscale * w * (sigmoid(l) - label)
hipError_t bce_logits(const float* logits, int ld, int64_t P_real, int64_t P_total, float w_real, float w_fake,
                      float gscale, float* grad, float* part, int blocks, float* loss, hipStream_t s);
// gy[p] += dz[p * ld + c]
hipError_t add_channel(float* gy, const float* dz, int ld, int c, int64_t P, hipStream_t s);
// depth integral down each column (rows above only), times scale, of the 1x1 map p = w e + b of the bf16
// tensor e [N][H][W][16] (w bf16 [8][16], b FP32 [8]), into channels [c_off, c_off + 8) of the bf16 tensor
// out [N][H][W][ld]
hipError_t depth_map_scan_fwd(const uint16_t* e, const uint16_t* w, const float* b, uint16_t* out, int N, int H,
                              int W, float scale, int ld, int c_off, hipStream_t s);
// its backward from g [N][H][W][ld] (FP32): dp (bf16, [N][H][W][8]), the channels [0, c_off) copied to
// g_skip [N][H][W][c_off], bias_grad[8] = column sums of dp; part holds depth_scan_blocks(N, W) * 8 floats
int depth_scan_blocks(int N, int W);
// backward of the 1x1 map p = W x (KC = 8 map channels, C = 16 input channels, W bf16 [KC][C]) over
// P pixels: g [P][C] += dp W (FP32) and dw [KC][C] = sum of dp^T x (FP32, fixed order); part holds
// proj_bwd_blocks() * KC * C floats
int proj_bwd_blocks();
hipError_t proj_bwd(const uint16_t* dp, const uint16_t* x, const uint16_t* w, float* g, int64_t P, int KC, int C,
                    float* part, float* dw, hipStream_t s);
hipError_t depth_scan_bwd(const float* g, int ld, int c_off, float* g_skip, uint16_t* dp, float* part,
                          float* bias_grad, int N, int H, int W, float scale, hipStream_t s);
hipError_t pool2x2_sum(const float* fine, float* coarse, int N, int H, int W, int C, int accumulate, hipStream_t s);
hipError_t colsum_bf16(const uint16_t* x, int64_t rows, int cols, float* part, int blocks, float* out,
                       hipStream_t s);
hipError_t sum_parts(const float* part, int64_t n, int splits, float* out, hipStream_t s);
// several reductions of per-block partials ([splits][n] at part_off) into out + out_off, in one launch,
// each bit-identical to sum_parts of the same partials (n <= 65535 per segment)
constexpr int kMaxReduceSegs = 24;
struct ReduceSeg {
    int64_t part_off, out_off;
    int32_t n, splits;
    int32_t first;   // first block (output) of the segment: the sum of n over the earlier segments
};
struct ReduceSegs {
    ReduceSeg s[kMaxReduceSegs];
    int32_t count;
};
hipError_t reduce_segments(const float* part, float* out, const ReduceSegs& t, hipStream_t s);
hipError_t head_fwd(const uint16_t* x, const uint16_t* w, const float* b, float* y, int64_t P, int C, hipStream_t s);
hipError_t head_bwd(const uint16_t* x, const uint16_t* w, const float* g, float* dx, int64_t P, int C, float* part,
                    int blocks, float* dwb, hipStream_t s);
hipError_t l1_loss(const float* yhat, const float* y, int64_t n, float* grad, float* part, int blocks, float* loss,
                   hipStream_t s);
// Adam: the step counters and per-step scalars live on the device (coef = {lr, c1, c2, disc c1, disc c2});
// one launch updates all segments of a parameter vector (blocks = sum of adam_blocks(n) over segments)
struct AdamSeg {
    int64_t off, n;          // element range of the segment in the parameter vector
    int32_t block0;          // first block of the segment
    int32_t Co, taps, Ci;    // weight layout [Co][taps][Ci] (transpose only)
    int32_t bf16, transpose; // refresh the bf16 copy; also its [Ci][taps][Co] transpose
};
int adam_blocks(int64_t n);
hipError_t adam_coef(int64_t* steps, float* coef, float lr, float b1, float b2, int disc, hipStream_t s);
hipError_t adam_multi(const AdamSeg* segs, int nseg, int blocks, float* w, float* m, float* v, const float* g,
                      uint16_t* wb, uint16_t* wt, const float* coef, int ci, float b1, float b2, float eps,
                      hipStream_t s);
// losses of the step counted in steps[0] into a ring of R steps (3 floats each)
hipError_t loss_log(const float* loss, const int64_t* steps, float* hist, int R, hipStream_t s);
hipError_t weights_to_bf16(const float* w, int64_t n, uint16_t* wb, uint16_t* wt, int Co, int taps, int Ci,
                           hipStream_t s);
hipError_t psnr_frames(const float* yhat, const float* y, int n_frames, int64_t frame, float* psnr, hipStream_t s);
hipError_t psnr_indexed(const float* yhat, const float* y, const int32_t* idx, int n_frames, int64_t frame,
                        float* psnr, hipStream_t s);
hipError_t transpose_w(const uint16_t* w, uint16_t* wt, int Co, int taps, int Ci, hipStream_t s);
hipError_t clamp01(const float* x, float* y, int64_t n, hipStream_t s);

}  // namespace sg
