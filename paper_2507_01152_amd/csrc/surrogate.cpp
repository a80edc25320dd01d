// Learned surrogate of the physics simulator (C ABI in include/sonosim.h):
// conv op entry points, the encoder-decoder network, training on pairs the
// physics path renders, inference with a physics audit and fallback, and
// checkpoints.  All arithmetic runs in the kernels of conv_mfma.hip and
// physics.hip; this file only orchestrates.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "sg_host.h"
#include "surrogate_internal.h"

namespace sg {
namespace {

// tensors of the network (per frame: channels and pyramid level)
// (A0: the depth integral, stored densely before it is copied into S0's last channels)
enum { X = 0, T1, E0, T2, E1, T3, E2, T4, E3, T5, B4, U3, S3, D3, U2, S2, D2, U1, S1, D1, U0, S0, D0, A0, kNumT };
const int kTC[kNumT] = {8, 16, 16, 32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 128, 64, 64, 64, 32, 32, 32, 16, 24, 16, 8};
const int kTL[kNumT] = {0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};

struct LayerDef {
    int in, out, skip, out2, Ci, Co, stride, up;
};
// 3x3 convs with ReLU; decoder "U" layers read their input upsampled x2 and
// add the encoder tensor of the same level (out2 = out + skip).  S0 has 8
// more channels: the depth integral of a 1x1 map of E0 (kScan*).
const LayerDef kLayers[] = {
    {X, T1, -1, -1, 8, 16, 1, 0},       {T1, E0, -1, -1, 16, 16, 1, 0},
    {E0, T2, -1, -1, 16, 32, 2, 0},     {T2, E1, -1, -1, 32, 32, 1, 0},
    {E1, T3, -1, -1, 32, 64, 2, 0},     {T3, E2, -1, -1, 64, 64, 1, 0},
    {E2, T4, -1, -1, 64, 128, 2, 0},    {T4, E3, -1, -1, 128, 128, 1, 0},
    {E3, T5, -1, -1, 128, 256, 2, 0},   {T5, B4, -1, -1, 256, 256, 1, 0},
    {B4, U3, E3, S3, 256, 128, 1, 1},   {S3, D3, -1, -1, 128, 128, 1, 0},
    {D3, U2, E2, S2, 128, 64, 1, 1},    {S2, D2, -1, -1, 64, 64, 1, 0},
    {D2, U1, E1, S1, 64, 32, 1, 1},     {S1, D1, -1, -1, 32, 32, 1, 0},
    {D1, U0, E0, S0, 32, 16, 1, 1},     {S0, D0, -1, -1, 24, 16, 1, 0},
};
constexpr int kNumL = sizeof(kLayers) / sizeof(kLayers[0]);
constexpr int kHeadC = 16;
// depth integral along the beam (the exclusive sum over rows above a pixel,
// as in the energy equation of App. B.2): p = W_p E0 + b_p (1x1, 16 -> 8),
// S0[..., 16 + k] = bf16(kScanScale * sum_{v < y} p_k(v))
constexpr int kScanSrc = E0, kScanDst = S0, kScanTmp = A0, kScanC = 8, kScanOff = 16;
constexpr float kScanScale = 1.f / 16.f;
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;
constexpr int kLossRing = 4096;   // training steps whose losses stay readable on the device

// conditional patch discriminator of the adversarial term (pix2pix: the
// discriminator judges patches of an image together with the network's
// input): 3x3 convs, pad 1, leaky ReLU after all but the last, whose channel
// 0 is the patch logit (its other channels stay zero).  Input: the encoded
// input's channels 0..3 and the image in channel kDiscImageC.
struct DiscDef {
    int Ci, Co, stride;
};
const DiscDef kDisc[] = {{8, 32, 2}, {32, 64, 2}, {64, 128, 2}, {128, 128, 1}, {128, 8, 1}};
constexpr int kNumD = sizeof(kDisc) / sizeof(kDisc[0]);
constexpr int kDiscImageC = 4;
constexpr int kDiscLogitC = 8;   // channels of the last conv (channel 0: the logit)
// pyramid level of the discriminator's tensor k (k = 0: input, k = L + 1: output of layer L)
constexpr int kDiscLevel[kNumD + 1] = {0, 1, 2, 3, 3, 3};
constexpr int kDiscTC[kNumD + 1] = {8, 32, 64, 128, 128, kDiscLogitC};

}  // namespace

struct Surrogate {
    int H = 0, W = 0;
    int64_t n_params = 0;
    int64_t w_off[kNumL], b_off[kNumL], w_n[kNumL];
    int64_t proj_w = 0, proj_b = 0;
    int64_t head_w = 0, head_b = 0;
    DevBuf master, mom1, mom2, grad, wb, wt;
    int64_t step = 0;
    int cap = 0, cap_grad = 0, last_n = 0;
    DevBuf act[kNumT], gact[kNumT];
    DevBuf dpre, fine, parts, yhat, target, gy, loss, psnr, idx;
    DevBuf bias_parts;   // per-block bias-gradient partials of every layer of a backward pass, reduced at its end
    DevBuf dscan;   // bf16 gradient at the depth map's output (the integral's backward), n x H x W x kScanC
    DevBuf out32;   // FP32 frames of bf16 inference
    // CT-conditioned input: per-frame histograms and matching maps, the reference
    // (kCtBins int64 counts, then their inclusive cumulative counts) and its total
    bool ct = false;
    float adv_weight = 0.f;
    DevBuf ct_hist, ct_lut, ct_ref;
    long long ct_n_ref = 0;
    // discriminator (adv_weight > 0): FP32 masters, Adam moments, gradient, bf16 copies; tensors for up to
    // d_cap frames (d_act[k]: bf16, tensor k; d_g[k]: FP32 gradient at tensor k; logits FP32).  A step's
    // first pass (real and fake pairs, 2n frames) uses frames [0, 2n), its second pass (the generator's
    // adversarial gradient, n frames) frames [2n, 3n), so both stay readable after the step
    int64_t dn_params = 0;
    int64_t dw_off[kNumD] = {}, db_off[kNumD] = {}, dw_n[kNumD] = {};
    DevBuf d_master, d_mom1, d_mom2, d_grad, d_wb, d_wt;
    int64_t d_step = 0;
    int d_cap = 0;
    DevBuf d_act[kNumD], d_g[kNumD], d_logits, d_glog, d_dpre, d_bias_scratch;
    // training state on the device: update counters {generator, discriminator}, Adam's per-step
    // scalars, the fused Adam's segment tables, and the losses of the last kLossRing steps
    DevBuf steps, coef, segs, d_segs, hist;
    int nseg = 0, adam_nb = 0, d_nseg = 0, d_adam_nb = 0;
    // the captured training step (forward, losses, backward, Adam) for batches of g_n pairs, valid while
    // the buffers it was captured on stay in place; warm_n: shape of the last eager step
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t g_exec = nullptr;
    int g_n = 0, warm_n = 0, g_failed_n = 0;
    std::vector<const void*> g_ptrs, warm_ptrs;
    float* pinned = nullptr;   // host-pinned loss readback (3 * kLossRing floats)
    ~Surrogate();
};

Surrogate::~Surrogate()
{
    if (g_exec) (void)hipGraphExecDestroy(g_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (pinned) (void)hipHostFree(pinned);
}

void SurrogateDeleter::operator()(Surrogate* p) const { delete p; }

void surrogate_release_all(sg_ctx* c) { c->surrogates.clear(); }

namespace {

Surrogate* find_surr(sg_ctx* c, int32_t id)
{
    if (!c) return nullptr;
    auto it = c->surrogates.find(id);
    return it == c->surrogates.end() ? nullptr : it->second.get();
}

// output channels of all generator layers (the bias-gradient outputs of a backward pass)
int bias_count()
{
    int n = 0;
    for (int L = 0; L < kNumL; ++L) n += kLayers[L].Co;
    return n;
}

ConvShape layer_shape(const Surrogate& s, int L, int n)
{
    const LayerDef& d = kLayers[L];
    const int lv = kTL[d.in];
    ConvShape sh;
    sh.N = n;
    sh.H = s.H >> lv;
    sh.W = s.W >> lv;
    sh.C = d.Ci;
    sh.Co = d.Co;
    sh.k = 3;
    sh.stride = d.stride;
    sh.pad = 1;
    sh.up = d.up;
    return sh;
}

int64_t tensor_elems(const Surrogate& s, int t, int n)
{
    const int lv = kTL[t];
    return (int64_t)n * (s.H >> lv) * (s.W >> lv) * kTC[t];
}

int blocks_for(int64_t n, int cap = 1024)
{
    int64_t b = (n + 4095) / 4096;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

sg_status check(hipError_t e, const char* what) { return e == hipSuccess ? SG_OK : hip_fail(e, what); }

#define SG_TRY(x)                             \
    do {                                      \
        sg_status _s = (x);                   \
        if (_s != SG_OK) return _s;           \
    } while (0)

// weight gradient of one conv: dw (FP32) and optional bias gradient db
sg_status wgrad(sg_ctx* c, const ConvShape& sh, const uint16_t* x, const uint16_t* dy, float* dw, float* db,
                DevBuf& parts)
{
    ConvGeom g = geom_of(sh, 2);
    const int cs_blocks0 = blocks_for(g.Kw, 512);
    WgradTilePlan tp;
    if (wgrad_tile_plan(g, &tp)) {   // stride 1: direct tiled kernel, one partial per block and channel group
        const size_t need = sizeof(float) * std::max<int64_t>(wgrad_tile_part_floats(tp), (int64_t)cs_blocks0 * sh.Co);
        SG_TRY(check(parts.ensure(need), "wgrad workspace"));
        SG_TRY(check(wgrad_tile(g, x, dy, (float*)parts.p, tp, dw, c->stream), "wgrad launch"));
        if (db) SG_TRY(check(colsum_bf16(dy, g.Kw, sh.Co, (float*)parts.p, cs_blocks0, db, c->stream), "bias grad"));
        return SG_OK;
    }
    const int bm = wgrad_tile_m((int)g.M);
    const int64_t tiles = ((g.M + bm - 1) / bm) * ((g.N + 127) / 128);
    const int64_t nkt = (g.Kw + 31) / 32;
    int64_t splits = 2048 / tiles;
    if (splits < 1) splits = 1;
    if (splits > 512) splits = 512;
    if (splits > nkt) splits = nkt;
    const int64_t k_chunk = ((nkt + splits - 1) / splits) * 32;
    splits = (g.Kw + k_chunk - 1) / k_chunk;
    const int cs_blocks = blocks_for(g.Kw, 512);
    const size_t need = sizeof(float) * std::max<int64_t>(splits * g.M * g.N, (int64_t)cs_blocks * sh.Co);
    SG_TRY(check(parts.ensure(need), "wgrad workspace"));
    ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.a = dy;
    a.b = x;
    a.out_f32 = (float*)parts.p;
    a.k_chunk = k_chunk;
    SG_TRY(check(conv_gemm(2, g, a, (int)splits, c->stream), "wgrad launch"));
    SG_TRY(check(sum_parts((float*)parts.p, g.M * g.N, (int)splits, dw, c->stream), "wgrad reduce"));
    if (db) SG_TRY(check(colsum_bf16(dy, g.Kw, sh.Co, (float*)parts.p, cs_blocks, db, c->stream), "bias grad"));
    return SG_OK;
}

// data gradient of one conv into dx (stored input resolution)
sg_status dgrad(sg_ctx* c, const ConvShape& sh, const uint16_t* dy, const uint16_t* wt, float* dx, int accumulate,
                DevBuf& fine)
{
    ConvGeom g = geom_of(sh, 1);
    // few channels: the tiled forward conv of dy with mirrored taps (an upsampled layer's 2 x 2 sums in
    // its epilogue)
    if (dgrad_tile_supported(g)) return check(dgrad_tile(g, dy, wt, dx, accumulate, c->stream), "dgrad launch");
    if (dgrad_parity_supported(g))   // stride 2, wider: one GEMM per output parity class, one launch
        return check(dgrad_parity(g, dy, wt, dx, accumulate, c->stream), "dgrad launch");
    ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.a = dy;
    a.b = wt;
    if (sh.up) {
        SG_TRY(check(fine.ensure(sizeof(float) * (size_t)g.M * sh.C), "dgrad workspace"));
        a.out_f32 = (float*)fine.p;
        a.accumulate = 0;
        SG_TRY(check(conv_gemm(1, g, a, 1, c->stream), "dgrad launch"));
        return check(pool2x2_sum((float*)fine.p, dx, sh.N, sh.H, sh.W, sh.C, accumulate, c->stream), "upsample grad");
    }
    a.out_f32 = dx;
    a.accumulate = accumulate;
    return check(conv_gemm(1, g, a, 1, c->stream), "dgrad launch");
}

sg_status check_desc(const sg_conv_desc* d)
{
    if (!d) return fail(SG_EINVAL, "conv: NULL descriptor");
    if (d->N < 1 || d->H < 1 || d->W < 1 || d->C < 8 || d->C % 8 || d->Co < 8 || d->Co % 8 || d->kernel < 1 ||
        d->stride < 1 || d->pad < 0 || (d->upsample != 0 && d->upsample != 1) || d->C > 4096 || d->Co > 4096)
        return fail(SG_EINVAL, "conv: bad descriptor (C and Co multiples of 8 in [8, 4096], sizes >= 1)");
    ConvShape sh{d->N, d->H, d->W, d->C, d->Co, d->kernel, d->stride, d->pad, d->upsample};
    if (sh.Hin() + 2 * sh.pad < sh.k || sh.Win() + 2 * sh.pad < sh.k) return fail(SG_EINVAL, "conv: empty output");
    const int64_t px = (int64_t)sh.N * sh.Hin() * sh.Win();
    if (px >= (1ll << 31) || (int64_t)sh.N * sh.Ho() * sh.Wo() >= (1ll << 31))
        return fail(SG_EINVAL, "conv: more than 2^31 - 1 pixels");
    if (px * std::max(sh.C, sh.Co) >= (1ll << 40)) return fail(SG_EINVAL, "conv: tensor too large");
    if ((int64_t)sh.k * sh.k * std::max(sh.C, sh.Co) >= (1ll << 30)) return fail(SG_EINVAL, "conv: K too large");
    return SG_OK;
}

ConvShape shape_of(const sg_conv_desc* d)
{
    return ConvShape{d->N, d->H, d->W, d->C, d->Co, d->kernel, d->stride, d->pad, d->upsample};
}

// capacity for n frames; grads: also the backward buffers
sg_status ensure_capacity(Surrogate& s, int n, bool grads)
{
    if (n > s.cap) {
        for (int t = 0; t < kNumT; ++t)
            SG_TRY(check(s.act[t].ensure(sizeof(uint16_t) * tensor_elems(s, t, n)), "activation buffers"));
        const int64_t P = (int64_t)n * s.H * s.W;
        SG_TRY(check(s.yhat.ensure(sizeof(float) * P), "output buffer"));
        SG_TRY(check(s.target.ensure(sizeof(float) * P), "target buffer"));
        s.cap = n;
    }
    if (grads && n > s.cap_grad) {
        for (int t = 1; t < kNumT; ++t)
            SG_TRY(check(s.gact[t].ensure(sizeof(float) * tensor_elems(s, t, n)), "gradient buffers"));
        int64_t mx = 0;
        for (int t = 1; t < kNumT; ++t) mx = std::max(mx, tensor_elems(s, t, n));
        SG_TRY(check(s.dpre.ensure(sizeof(uint16_t) * mx), "dpre buffer"));
        SG_TRY(check(s.dscan.ensure(sizeof(uint16_t) * (size_t)n * s.H * s.W * kScanC), "depth map gradient"));
        SG_TRY(check(s.gy.ensure(sizeof(float) * (int64_t)n * s.H * s.W), "output grad"));
        s.cap_grad = n;
    }
    return SG_OK;
}

sg_status refresh_bf16(sg_ctx* c, Surrogate& s)
{
    for (int L = 0; L < kNumL; ++L) {
        const LayerDef& d = kLayers[L];
        SG_TRY(check(weights_to_bf16((float*)s.master.p + s.w_off[L], s.w_n[L], (uint16_t*)s.wb.p + s.w_off[L],
                                     (uint16_t*)s.wt.p + s.w_off[L], d.Co, 9, d.Ci, c->stream),
                     "bf16 weights"));
    }
    SG_TRY(check(weights_to_bf16((float*)s.master.p + s.proj_w, kScanC * kTC[kScanSrc], (uint16_t*)s.wb.p + s.proj_w,
                                 (uint16_t*)s.wt.p + s.proj_w, kScanC, 1, kTC[kScanSrc], c->stream),
                 "bf16 depth map"));
    return check(weights_to_bf16((float*)s.master.p + s.head_w, kHeadC, (uint16_t*)s.wb.p + s.head_w, nullptr, 1, 1,
                                 kHeadC, c->stream),
                 "bf16 head");
}

// train: also keep the pre-skip outputs of the decoder layers (ReLU masks of the backward)
sg_status forward(sg_ctx* c, Surrogate& s, int n, bool train)
{
    bool head_fused = false;
    for (int L = 0; L < kNumL; ++L) {
        const LayerDef& d = kLayers[L];
        const ConvShape sh = layer_shape(s, L, n);
        ConvArgs a;
        std::memset(&a, 0, sizeof(a));
        a.a = (const uint16_t*)s.act[d.in].p;
        a.b = (const uint16_t*)s.wb.p + s.w_off[L];
        a.bias = (const float*)s.master.p + s.b_off[L];
        a.relu = 1;
        a.out_bf16 = (d.skip >= 0 && !train) ? nullptr : (uint16_t*)s.act[d.out].p;
        if (L == kNumL - 1 && d.Co == kHeadC && conv_tile_supported(geom_of(sh, 0))) {
            // the 1x1 head in the last conv's epilogue; its input is kept for the backward only
            a.head_w = (const uint16_t*)s.wb.p + s.head_w;
            a.head_b = (const float*)s.master.p + s.head_b;
            a.head_out = (float*)s.yhat.p;
            if (!train) a.out_bf16 = nullptr;
            head_fused = true;
        }
        if (d.skip >= 0) {
            a.skip = (const uint16_t*)s.act[d.skip].p;
            a.out2_bf16 = (uint16_t*)s.act[d.out2].p;
            a.ld_out2 = kTC[d.out2];
        }
        const bool scan_here = d.out2 == kScanDst;
        const bool scan_fused = scan_here && conv_tile_supported(geom_of(sh, 0));
        if (scan_fused) {   // S0 = [U0 + E0, integral]: the conv writes whole pixels
            a.extra = (const uint16_t*)s.act[kScanTmp].p;
            a.extra_c = kScanC;
        }
        SG_TRY(check(conv_gemm(0, geom_of(sh, 0), a, 1, c->stream), "forward conv"));
        if (scan_here && !scan_fused)
            SG_TRY(check(hipMemcpy2DAsync((uint16_t*)s.act[kScanDst].p + kScanOff, sizeof(uint16_t) * kTC[kScanDst],
                                          s.act[kScanTmp].p, sizeof(uint16_t) * kScanC, sizeof(uint16_t) * kScanC,
                                          (size_t)n * s.H * s.W, hipMemcpyDeviceToDevice, c->stream),
                         "depth integral copy"));
        if (d.out == kScanSrc)   // 1x1 map of E0 and its depth integral (dense, copied into S0 later)
            SG_TRY(check(depth_map_scan_fwd((const uint16_t*)s.act[kScanSrc].p, (const uint16_t*)s.wb.p + s.proj_w,
                                            (const float*)s.master.p + s.proj_b, (uint16_t*)s.act[kScanTmp].p, n, s.H,
                                            s.W, kScanScale, kScanC, 0, c->stream),
                         "depth integral"));
    }
    if (head_fused) return SG_OK;
    return check(head_fwd((const uint16_t*)s.act[D0].p, (const uint16_t*)s.wb.p + s.head_w,
                          (const float*)s.master.p + s.head_b, (float*)s.yhat.p, (int64_t)n * s.H * s.W, kHeadC,
                          c->stream),
                 "head forward");
}

sg_status backward(sg_ctx* c, Surrogate& s, int n)
{
    bool written[kNumT] = {};
    const int64_t P = (int64_t)n * s.H * s.W;
    float* grad = (float*)s.grad.p;
    const int hb = blocks_for(P);
    SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)hb * (kHeadC + 1)), "head workspace"));
    SG_TRY(check(head_bwd((const uint16_t*)s.act[D0].p, (const uint16_t*)s.wb.p + s.head_w, (const float*)s.gy.p,
                          (float*)s.gact[D0].p, P, kHeadC, (float*)s.parts.p, hb, grad + s.head_w, c->stream),
                 "head backward"));
    written[D0] = true;
    static_assert(kNumL <= kMaxReduceSegs, "one bias segment per layer");
    ReduceSegs bseg;
    bseg.count = 0;
    int64_t boff = 0;
    int bfirst = 0;
    SG_TRY(check(s.bias_parts.ensure(sizeof(float) * 1024 * (size_t)bias_count()), "bias partials"));
    for (int L = kNumL - 1; L >= 0; --L) {
        const LayerDef& d = kLayers[L];
        const ConvShape sh = layer_shape(s, L, n);
        const int go = d.out2 >= 0 ? d.out2 : d.out;   // gradient at the layer's (skip-added) output
        const int64_t n_out = tensor_elems(s, d.out, n);
        const int64_t rows = n_out / d.Co;
        if (go == kScanDst) {
            // depth integral: dp (bf16, in dscan), its bias gradient, and the skip copy of
            // S0's first channels into E0's gradient; then the 1x1 map's two products
            const int sb = depth_scan_blocks(n, s.W);
            SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)sb * kScanC), "depth integral workspace"));
            SG_TRY(check(depth_scan_bwd((const float*)s.gact[kScanDst].p, kTC[kScanDst], kScanOff,
                                        (float*)s.gact[kScanSrc].p, (uint16_t*)s.dscan.p, (float*)s.parts.p,
                                        grad + s.proj_b, n, s.H, s.W, kScanScale, c->stream),
                         "depth integral backward"));
            SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)proj_bwd_blocks() * kScanC * kTC[kScanSrc]),
                         "depth map workspace"));
            SG_TRY(check(proj_bwd((const uint16_t*)s.dscan.p, (const uint16_t*)s.act[kScanSrc].p,
                                  (const uint16_t*)s.wb.p + s.proj_w, (float*)s.gact[kScanSrc].p,
                                  (int64_t)n * s.H * s.W, kScanC, kTC[kScanSrc], (float*)s.parts.p, grad + s.proj_w,
                                  c->stream),
                         "depth map backward"));
            written[kScanSrc] = true;
        }
        // ReLU mask; the bias gradient's per-block partials are reduced with the other layers' after the loop
        const int mb = blocks_for(rows * d.Co / 2, 1024);   // about four rows per thread
        ReduceSeg& rs = bseg.s[bseg.count++];
        rs.part_off = boff;
        rs.out_off = s.b_off[L];
        rs.n = d.Co;
        rs.splits = mb;
        rs.first = bfirst;
        boff += (int64_t)mb * d.Co;
        bfirst += d.Co;
        SG_TRY(check(mask_colsum((const float*)s.gact[go].p, kTC[go], (const uint16_t*)s.act[d.out].p,
                                 (uint16_t*)s.dpre.p, rows, d.Co, (float*)s.bias_parts.p + rs.part_off, mb, nullptr,
                                 c->stream),
                     "relu mask and bias partials"));
        if (d.skip >= 0 && go != kScanDst) {   // (S0's skip copy is done by the depth integral's backward)
            // out2 = out + skip: the skip tensor receives the same gradient
            SG_TRY(check(hipMemcpyAsync(s.gact[d.skip].p, s.gact[go].p, sizeof(float) * n_out,
                                        hipMemcpyDeviceToDevice, c->stream),
                         "skip gradient"));
            written[d.skip] = true;
        }
        SG_TRY(wgrad(c, sh, (const uint16_t*)s.act[d.in].p, (const uint16_t*)s.dpre.p, grad + s.w_off[L], nullptr,
                     s.parts));
        if (L > 0) {
            SG_TRY(dgrad(c, sh, (const uint16_t*)s.dpre.p, (const uint16_t*)s.wt.p + s.w_off[L],
                         (float*)s.gact[d.in].p, written[d.in] ? 1 : 0, s.fine));
            written[d.in] = true;
        }
    }
    return check(reduce_segments((const float*)s.bias_parts.p, grad, bseg, c->stream), "bias gradients");
}

// Adam on every generator tensor, one launch (scalars from the device, counted by adam_coef)
sg_status adam(sg_ctx* c, Surrogate& s)
{
    return check(adam_multi((const AdamSeg*)s.segs.p, s.nseg, s.adam_nb, (float*)s.master.p, (float*)s.mom1.p,
                            (float*)s.mom2.p, (const float*)s.grad.p, (uint16_t*)s.wb.p, (uint16_t*)s.wt.p,
                            (const float*)s.coef.p, 1, kBeta1, kBeta2, kEps, c->stream),
                 "adam");
}

// segment table of the fused Adam: off, n, layout and copies of each tensor, with each segment's first block
void add_seg(std::vector<AdamSeg>& t, int& blocks, int64_t off, int64_t n, int Co, int taps, int Ci, bool bf16,
             bool transpose)
{
    AdamSeg a;
    a.off = off;
    a.n = n;
    a.block0 = blocks;
    a.Co = Co;
    a.taps = taps;
    a.Ci = Ci;
    a.bf16 = bf16 ? 1 : 0;
    a.transpose = transpose ? 1 : 0;
    t.push_back(a);
    blocks += adam_blocks(n);
}

hipError_t upload_segs(DevBuf& d, const std::vector<AdamSeg>& t)
{
    hipError_t e = d.ensure(sizeof(AdamSeg) * t.size());
    if (e == hipSuccess) e = hipMemcpy(d.p, t.data(), sizeof(AdamSeg) * t.size(), hipMemcpyHostToDevice);
    return e;
}

// ---------------------------------------------------------------------------
// discriminator of the adversarial term

ConvShape disc_shape(const Surrogate& s, int L, int frames)
{
    const int lv = kDiscLevel[L];
    ConvShape sh;
    sh.N = frames;
    sh.H = s.H >> lv;
    sh.W = s.W >> lv;
    sh.C = kDisc[L].Ci;
    sh.Co = kDisc[L].Co;
    sh.k = 3;
    sh.stride = kDisc[L].stride;
    sh.pad = 1;
    sh.up = 0;
    return sh;
}

int64_t disc_elems(const Surrogate& s, int k, int frames)
{
    return (int64_t)frames * (s.H >> kDiscLevel[k]) * (s.W >> kDiscLevel[k]) * kDiscTC[k];
}

sg_status disc_capacity(Surrogate& s, int frames)
{
    if (frames <= s.d_cap) return SG_OK;
    int64_t mx = 0;
    for (int k = 0; k < kNumD; ++k) {   // (k = 0: the input z; its gradient only in the second pass)
        SG_TRY(check(s.d_act[k].ensure(sizeof(uint16_t) * disc_elems(s, k, frames)), "discriminator activations"));
        SG_TRY(check(s.d_g[k].ensure(sizeof(float) * disc_elems(s, k, frames)), "discriminator gradients"));
        mx = std::max(mx, disc_elems(s, k + 1, frames));
    }
    SG_TRY(check(s.d_logits.ensure(sizeof(float) * disc_elems(s, kNumD, frames)), "discriminator logits"));
    SG_TRY(check(s.d_glog.ensure(sizeof(float) * disc_elems(s, kNumD, frames)), "logit gradient"));
    SG_TRY(check(s.d_dpre.ensure(sizeof(uint16_t) * mx), "discriminator dpre"));
    SG_TRY(check(s.d_bias_scratch.ensure(sizeof(float) * 256), "discriminator bias scratch"));
    s.d_cap = frames;
    return SG_OK;
}

sg_status disc_refresh_bf16(sg_ctx* c, Surrogate& s)
{
    for (int L = 0; L < kNumD; ++L)
        SG_TRY(check(weights_to_bf16((float*)s.d_master.p + s.dw_off[L], s.dw_n[L], (uint16_t*)s.d_wb.p + s.dw_off[L],
                                     (uint16_t*)s.d_wt.p + s.dw_off[L], kDisc[L].Co, 9, kDisc[L].Ci, c->stream),
                     "discriminator bf16 weights"));
    return SG_OK;
}

// parameters, He-normal (last layer: channel 0 only), zero biases
sg_status disc_create(sg_ctx* c, Surrogate& s, uint64_t seed)
{
    int64_t off = 0;
    for (int L = 0; L < kNumD; ++L) {
        s.dw_off[L] = off;
        s.dw_n[L] = (int64_t)kDisc[L].Co * 9 * kDisc[L].Ci;
        off += s.dw_n[L];
        s.db_off[L] = off;
        off += kDisc[L].Co;
    }
    s.dn_params = off;
    std::vector<float> h(off, 0.f);
    std::mt19937_64 rng(seed ^ 0x9E3779B97F4A7C15ull);
    for (int L = 0; L < kNumD; ++L) {
        const bool last = L == kNumD - 1;
        std::normal_distribution<float> nd(0.f, std::sqrt((last ? 1.f : 2.f) / (9.f * kDisc[L].Ci)));
        const int64_t n = last ? 9 * kDisc[L].Ci : s.dw_n[L];   // [Co][3][3][Ci]: channel 0 first
        for (int64_t i = 0; i < n; ++i) h[s.dw_off[L] + i] = nd(rng);
    }
    const size_t bytes = sizeof(float) * off;
    hipError_t e = s.d_master.ensure(bytes);
    if (e == hipSuccess) e = s.d_mom1.ensure(bytes);
    if (e == hipSuccess) e = s.d_mom2.ensure(bytes);
    if (e == hipSuccess) e = s.d_grad.ensure(bytes);
    if (e == hipSuccess) e = s.d_wb.ensure(sizeof(uint16_t) * off);
    if (e == hipSuccess) e = s.d_wt.ensure(sizeof(uint16_t) * off);
    if (e == hipSuccess) e = hipMemcpy(s.d_master.p, h.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s.d_mom1.p, 0, bytes);
    if (e == hipSuccess) e = hipMemset(s.d_mom2.p, 0, bytes);
    if (e == hipSuccess) e = hipMemset(s.d_grad.p, 0, bytes);
    std::vector<AdamSeg> t;
    int nb = 0;
    for (int L = 0; L < kNumD; ++L) {
        add_seg(t, nb, s.dw_off[L], s.dw_n[L], kDisc[L].Co, 9, kDisc[L].Ci, true, true);
        add_seg(t, nb, s.db_off[L], kDisc[L].Co, 1, 1, 1, false, false);
    }
    if (e == hipSuccess) e = upload_segs(s.d_segs, t);
    s.d_nseg = (int)t.size();
    s.d_adam_nb = nb;
    if (e != hipSuccess) return hip_fail(e, "discriminator allocation");
    return disc_refresh_bf16(c, s);
}

// element offset of frame `off` in the discriminator's tensor k
int64_t disc_at(const Surrogate& s, int k, int off) { return disc_elems(s, k, off); }

// forward over `frames` frames of input z (bf16, [frames][H][W][8]): d_act[1..], logits, written from
// frame `off` on
sg_status disc_forward(sg_ctx* c, Surrogate& s, const uint16_t* z, int frames, int off)
{
    for (int L = 0; L < kNumD; ++L) {
        const bool last = L == kNumD - 1;
        ConvArgs a;
        std::memset(&a, 0, sizeof(a));
        a.a = L == 0 ? z : (const uint16_t*)s.d_act[L].p + disc_at(s, L, off);
        a.b = (const uint16_t*)s.d_wb.p + s.dw_off[L];
        a.bias = (const float*)s.d_master.p + s.db_off[L];
        a.relu = last ? 0 : 2;
        if (last)
            a.out_f32 = (float*)s.d_logits.p + disc_at(s, kNumD, off);
        else
            a.out_bf16 = (uint16_t*)s.d_act[L + 1].p + disc_at(s, L + 1, off);
        SG_TRY(check(conv_gemm(0, geom_of(disc_shape(s, L, frames), 0), a, 1, c->stream), "discriminator conv"));
    }
    return SG_OK;
}

// backward from the logit gradient in d_glog: parameter gradients into d_grad (weights) and the input
// gradient into d_g[0] (input_grad); tensors from frame `off` on
sg_status disc_backward(sg_ctx* c, Surrogate& s, const uint16_t* z, int frames, bool weights, bool input_grad,
                        int off)
{
    float* grad = (float*)s.d_grad.p;
    for (int L = kNumD - 1; L >= 0; --L) {
        const bool last = L == kNumD - 1;
        const ConvShape sh = disc_shape(s, L, frames);
        const int64_t rows = disc_elems(s, L + 1, frames) / kDisc[L].Co;
        const float* g_out = last ? (const float*)s.d_glog.p + disc_at(s, kNumD, off)
                                  : (const float*)s.d_g[L + 1].p + disc_at(s, L + 1, off);
        const int mb = blocks_for(rows * kDisc[L].Co / 2, 1024);   // about four rows per thread
        SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)mb * kDisc[L].Co), "bias workspace"));
        SG_TRY(check(mask_colsum(g_out, 0, last ? nullptr : (const uint16_t*)s.d_act[L + 1].p + disc_at(s, L + 1, off),
                                 (uint16_t*)s.d_dpre.p, rows, kDisc[L].Co, (float*)s.parts.p, mb,
                                 weights ? grad + s.db_off[L] : (float*)s.d_bias_scratch.p, c->stream,
                                 last ? 0.f : kLeakySlope),
                     "discriminator mask"));
        const uint16_t* x = L == 0 ? z : (const uint16_t*)s.d_act[L].p + disc_at(s, L, off);
        if (weights)
            SG_TRY(wgrad(c, sh, x, (const uint16_t*)s.d_dpre.p, grad + s.dw_off[L], nullptr, s.parts));
        if (L > 0 || input_grad)
            SG_TRY(dgrad(c, sh, (const uint16_t*)s.d_dpre.p, (const uint16_t*)s.d_wt.p + s.dw_off[L],
                         (float*)s.d_g[L].p + disc_at(s, L, off), 0, s.fine));
    }
    return SG_OK;
}

sg_status disc_adam(sg_ctx* c, Surrogate& s)
{
    return check(adam_multi((const AdamSeg*)s.d_segs.p, s.d_nseg, s.d_adam_nb, (float*)s.d_master.p,
                            (float*)s.d_mom1.p, (float*)s.d_mom2.p, (const float*)s.d_grad.p, (uint16_t*)s.d_wb.p,
                            (uint16_t*)s.d_wt.p, (const float*)s.coef.p, 3, kBeta1, kBeta2, kEps, c->stream),
                 "discriminator adam");
}

// The adversarial part of one training step (pix2pix order), after the generator's forward and L1 loss:
// discriminator step on (x, target) as real and (x, yhat) as fake, then the generator's adversarial
// gradient through the updated discriminator, added into gy.  Losses: loss[1] = L_D, loss[2] = L_adv.
sg_status adversarial_step(sg_ctx* c, Surrogate& s, int n)
{
    SG_TRY(disc_capacity(s, 3 * n));
    const int64_t P = (int64_t)n * s.H * s.W;
    const int64_t Pp = (int64_t)n * (s.H >> 3) * (s.W >> 3);   // patches per set
    uint16_t* z = (uint16_t*)s.d_act[0].p;
    SG_TRY(check(disc_input((const uint16_t*)s.act[X].p, (const float*)s.target.p, (const float*)s.yhat.p, z, P,
                            c->stream),
                 "discriminator input"));
    SG_TRY(disc_forward(c, s, z, 2 * n, 0));
    const int bb = blocks_for(2 * Pp, 256);
    SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)bb), "bce workspace"));
    const float wd = 0.5f / (float)Pp;
    SG_TRY(check(bce_logits((const float*)s.d_logits.p, kDiscLogitC, Pp, 2 * Pp, wd, wd, 1.f, (float*)s.d_glog.p,
                            (float*)s.parts.p, bb, (float*)s.loss.p + 1, c->stream),
                 "discriminator loss"));
    SG_TRY(disc_backward(c, s, z, 2 * n, true, false, 0));
    SG_TRY(disc_adam(c, s));
    // second pass on the fake half through the updated discriminator, tensors at frames [2n, 3n)
    const uint16_t* zf = z + P * 8;
    const int off = 2 * n;
    SG_TRY(disc_forward(c, s, zf, n, off));
    SG_TRY(check(bce_logits((const float*)s.d_logits.p + disc_at(s, kNumD, off), kDiscLogitC, Pp, Pp,
                            1.f / (float)Pp, 0.f, s.adv_weight, (float*)s.d_glog.p + disc_at(s, kNumD, off),
                            (float*)s.parts.p, bb, (float*)s.loss.p + 2, c->stream),
                 "adversarial loss"));
    SG_TRY(disc_backward(c, s, zf, n, false, true, off));
    return check(add_channel((float*)s.gy.p, (const float*)s.d_g[0].p + disc_at(s, 0, off), 8, kDiscImageC, P,
                             c->stream),
                 "adversarial gradient");
}

sg_status check_frames(const Surrogate& s, int32_t n, const sg_probe* probes)
{
    for (int i = 0; i < n; ++i)
        if (probes[i].W != s.W || probes[i].H != s.H || probes[i].n_elev > 1)
            return fail(SG_EINVAL, "env %d: probe %dx%d (x%d planes), the surrogate renders one %dx%d plane", i,
                        probes[i].W, probes[i].H, probes[i].n_elev, s.W, s.H);
    if (n > 65535) return fail(SG_EINVAL, "at most 65535 envs per call");
    return SG_OK;
}

sg_status check_ct_volumes(sg_ctx* c, int32_t n, const int32_t* vol_ids)
{
    for (int i = 0; i < n; ++i) {
        const int32_t v = vol_ids[i];
        if (v >= 0 && v < (int32_t)c->vols.size() && c->vols[v].live && !c->vols[v].dev.ct)
            return fail(SG_EINVAL, "env %d: volume %d has no CT (the CT-conditioned surrogate reads HU)", i, v);
    }
    return SG_OK;
}

// encode inputs of n envs into act[X] (and optionally render their targets)
sg_status encode_and_render(sg_ctx* c, Surrogate& s, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                            const double* poses, float* target)
{
    if (s.ct) {
        if (s.ct_n_ref <= 0) return fail(SG_ESTATE, "CT surrogate: no reference histogram (sg_surr_set_ct_reference)");
        SG_TRY(check_ct_volumes(c, n, vol_ids));
        SG_TRY(check(s.ct_hist.ensure(sizeof(uint32_t) * kCtBins * (size_t)n), "CT histograms"));
        SG_TRY(check(s.ct_lut.ensure(sizeof(uint16_t) * kCtBins * (size_t)n), "CT matching maps"));
    }
    std::vector<int64_t> offs(n);
    for (int i = 0; i < n; ++i) offs[i] = (int64_t)i * s.H * s.W;
    PhysArgs a;
    StageInfo info;
    SG_TRY(stage_physics(c, n, vol_ids, probes, poses, target ? target : (float*)s.yhat.p, offs.data(), nullptr, a,
                         info));
    if (s.ct)
        SG_TRY(check(launch_ct_encode(a, n, s.H * s.W, (uint32_t*)s.ct_hist.p,
                                      (const long long*)s.ct_ref.p + kCtBins, s.ct_n_ref, (uint16_t*)s.ct_lut.p,
                                      (uint16_t*)s.act[X].p, c->stream),
                     "CT encode"));
    else
        SG_TRY(check(launch_encode(a, n, s.H * s.W, (uint16_t*)s.act[X].p, c->stream), "encode"));
    if (target) SG_TRY(launch_physics(c, a, info));
    return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

// ---------------------------------------------------------------------------
// conv op entry points

extern "C" sg_status sg_conv_forward(sg_ctx* c, const sg_conv_desc* d, const uint16_t* x, const uint16_t* w,
                                     const float* bias, int32_t relu, const uint16_t* skip, uint16_t* y,
                                     uint16_t* y_skip, float* y_f32)
{
    if (!c || !x || !w || (!y && !y_f32)) return fail(SG_EINVAL, "sg_conv_forward: NULL argument");
    SG_TRY(check_desc(d));
    if (skip && !y_skip) return fail(SG_EINVAL, "sg_conv_forward: skip given without y_skip");
    (void)hipSetDevice(c->device);
    const ConvShape sh = shape_of(d);
    ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.a = x;
    a.b = w;
    a.bias = bias;
    a.relu = relu ? 1 : 0;
    a.skip = skip;
    a.out2_bf16 = y_skip;
    a.out_bf16 = y;
    a.out_f32 = y_f32;
    return check(conv_gemm(0, geom_of(sh, 0), a, 1, c->stream), "conv forward");
}

extern "C" sg_status sg_conv_backward_data(sg_ctx* c, const sg_conv_desc* d, const uint16_t* dy, const uint16_t* w,
                                           float* dx, int32_t accumulate)
{
    if (!c || !dy || !w || !dx) return fail(SG_EINVAL, "sg_conv_backward_data: NULL argument");
    SG_TRY(check_desc(d));
    (void)hipSetDevice(c->device);
    const ConvShape sh = shape_of(d);
    const int taps = sh.k * sh.k;
    SG_TRY(check(c->op_wt.ensure(sizeof(uint16_t) * (size_t)sh.Co * taps * sh.C), "weight workspace"));
    SG_TRY(check(transpose_w(w, (uint16_t*)c->op_wt.p, sh.Co, taps, sh.C, c->stream), "weight transpose"));
    return dgrad(c, sh, dy, (const uint16_t*)c->op_wt.p, dx, accumulate ? 1 : 0, c->op_fine);
}

extern "C" sg_status sg_conv_backward_weight(sg_ctx* c, const sg_conv_desc* d, const uint16_t* x, const uint16_t* dy,
                                             float* dw, float* db)
{
    if (!c || !x || !dy || !dw) return fail(SG_EINVAL, "sg_conv_backward_weight: NULL argument");
    SG_TRY(check_desc(d));
    if (db && d->Co > 256) return fail(SG_EINVAL, "sg_conv_backward_weight: bias gradient needs Co <= 256");
    (void)hipSetDevice(c->device);
    return wgrad(c, shape_of(d), x, dy, dw, db, c->op_parts);
}

// ---------------------------------------------------------------------------
// surrogate model

extern "C" sg_status sg_surr_create(sg_ctx* c, int32_t H, int32_t W, uint64_t seed, int32_t* id)
{
    if (!c || !id) return fail(SG_EINVAL, "sg_surr_create: NULL argument");
    if (H < 16 || W < 16 || H % 16 || W % 16 || H > SG_MAX_IMAGE || W > SG_MAX_IMAGE)
        return fail(SG_EINVAL, "surrogate frame %dx%d: H and W must be multiples of 16 in [16, %d]", W, H,
                    SG_MAX_IMAGE);
    (void)hipSetDevice(c->device);
    std::unique_ptr<Surrogate, SurrogateDeleter> s(new Surrogate());
    s->H = H;
    s->W = W;
    int64_t off = 0;
    for (int L = 0; L < kNumL; ++L) {
        s->w_off[L] = off;
        s->w_n[L] = (int64_t)kLayers[L].Co * 9 * kLayers[L].Ci;
        off += s->w_n[L];
        s->b_off[L] = off;
        off += kLayers[L].Co;
    }
    s->proj_w = off;
    off += kScanC * kTC[kScanSrc];
    s->proj_b = off;
    off += kScanC;
    s->head_w = off;
    off += kHeadC;
    s->head_b = off;
    off += 1;
    s->n_params = off;
    // He-normal weights, zero biases; head bias at a mid-grey level
    std::vector<float> h(off, 0.f);
    std::mt19937_64 rng(seed);
    for (int L = 0; L < kNumL; ++L) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (9.f * kLayers[L].Ci)));
        for (int64_t i = 0; i < s->w_n[L]; ++i) h[s->w_off[L] + i] = nd(rng);
    }
    std::normal_distribution<float> np_(0.f, std::sqrt(1.f / kTC[kScanSrc]));
    for (int i = 0; i < kScanC * kTC[kScanSrc]; ++i) h[s->proj_w + i] = np_(rng);
    std::normal_distribution<float> nh(0.f, std::sqrt(1.f / kHeadC));
    for (int i = 0; i < kHeadC; ++i) h[s->head_w + i] = nh(rng);
    h[s->head_b] = 0.2f;
    const size_t bytes = sizeof(float) * off;
    hipError_t e = s->master.ensure(bytes);
    if (e == hipSuccess) e = s->mom1.ensure(bytes);
    if (e == hipSuccess) e = s->mom2.ensure(bytes);
    if (e == hipSuccess) e = s->grad.ensure(bytes);
    if (e == hipSuccess) e = s->wb.ensure(sizeof(uint16_t) * off);
    if (e == hipSuccess) e = s->wt.ensure(sizeof(uint16_t) * off);
    if (e == hipSuccess) e = hipMemcpy(s->master.p, h.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->mom1.p, 0, bytes);
    if (e == hipSuccess) e = hipMemset(s->mom2.p, 0, bytes);
    if (e == hipSuccess) e = hipMemset(s->grad.p, 0, bytes);
    std::vector<AdamSeg> t;
    int nb = 0;
    for (int L = 0; L < kNumL; ++L) {
        add_seg(t, nb, s->w_off[L], s->w_n[L], kLayers[L].Co, 9, kLayers[L].Ci, true, true);
        add_seg(t, nb, s->b_off[L], kLayers[L].Co, 1, 1, 1, false, false);
    }
    add_seg(t, nb, s->proj_w, kScanC * kTC[kScanSrc], kScanC, 1, kTC[kScanSrc], true, true);
    add_seg(t, nb, s->proj_b, kScanC, 1, 1, 1, false, false);
    add_seg(t, nb, s->head_w, kHeadC, 1, 1, kHeadC, true, false);
    add_seg(t, nb, s->head_b, 1, 1, 1, 1, false, false);
    if (e == hipSuccess) e = upload_segs(s->segs, t);
    s->nseg = (int)t.size();
    s->adam_nb = nb;
    if (e == hipSuccess) e = s->steps.ensure(sizeof(int64_t) * 2);
    if (e == hipSuccess) e = hipMemset(s->steps.p, 0, sizeof(int64_t) * 2);
    if (e == hipSuccess) e = s->coef.ensure(sizeof(float) * 8);
    if (e == hipSuccess) e = hipMemset(s->coef.p, 0, sizeof(float) * 8);
    // losses {L1, L_D, L_adv}: without an adversarial term the last two stay 0
    if (e == hipSuccess) e = s->loss.ensure(sizeof(float) * 8);
    if (e == hipSuccess) e = hipMemset(s->loss.p, 0, sizeof(float) * 8);
    if (e == hipSuccess) e = s->hist.ensure(sizeof(float) * 3 * kLossRing);
    if (e == hipSuccess) e = hipMemset(s->hist.p, 0, sizeof(float) * 3 * kLossRing);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->pinned, sizeof(float) * 3 * kLossRing, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "surrogate allocation");
    SG_TRY(refresh_bf16(c, *s));
    const int32_t sid = c->next_surr++;
    c->surrogates[sid] = std::move(s);
    *id = sid;
    return SG_OK;
}

extern "C" sg_status sg_surr_create_ct(sg_ctx* c, int32_t H, int32_t W, uint64_t seed, float adv_weight, int32_t* id)
{
    if (!(adv_weight >= 0.f && adv_weight <= 1.f)) return fail(SG_EINVAL, "sg_surr_create_ct: adv_weight in [0, 1]");
    SG_TRY(sg_surr_create(c, H, W, seed, id));
    Surrogate* s = find_surr(c, *id);
    s->ct = true;
    s->adv_weight = adv_weight;
    hipError_t e = s->ct_ref.ensure(sizeof(long long) * 2 * kCtBins);
    if (e == hipSuccess) e = hipMemset(s->ct_ref.p, 0, sizeof(long long) * 2 * kCtBins);   // no reference yet
    sg_status st = e == hipSuccess ? SG_OK : hip_fail(e, "CT reference");
    if (st == SG_OK && adv_weight > 0.f) st = disc_create(c, *s, seed);
    if (st != SG_OK) c->surrogates.erase(*id);
    return st;
}

extern "C" sg_status sg_surr_set_ct_reference(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids,
                                              const sg_probe* probes, const double* poses, int64_t* hist)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !vol_ids || !probes || !poses) return fail(SG_EINVAL, "sg_surr_set_ct_reference: bad id or NULL");
    if (!s->ct) return fail(SG_EINVAL, "sg_surr_set_ct_reference: not a CT-conditioned surrogate");
    if (n < 1) return fail(SG_EINVAL, "sg_surr_set_ct_reference: n_envs must be >= 1");
    (void)hipSetDevice(c->device);
    SG_TRY(check_frames(*s, n, probes));
    SG_TRY(check_ct_volumes(c, n, vol_ids));
    DevBuf h;
    SG_TRY(check(h.ensure(sizeof(uint32_t) * kCtBins * (size_t)n), "reference histograms"));
    std::vector<int64_t> offs(n);
    for (int i = 0; i < n; ++i) offs[i] = (int64_t)i * s->H * s->W;
    SG_TRY(ensure_capacity(*s, 1, false));
    PhysArgs a;
    StageInfo info;
    SG_TRY(stage_physics(c, n, vol_ids, probes, poses, (float*)s->yhat.p, offs.data(), nullptr, a, info));
    SG_TRY(check(launch_ct_encode(a, n, s->H * s->W, (uint32_t*)h.p, nullptr, 0, nullptr, nullptr, c->stream),
                 "reference histograms"));
    SG_TRY(check(launch_ct_reference((const uint32_t*)h.p, n, (long long*)s->ct_ref.p,
                                     (long long*)s->ct_ref.p + kCtBins, c->stream),
                 "reference"));
    std::vector<long long> r(kCtBins);
    hipError_t e = hipMemcpyAsync(r.data(), s->ct_ref.p, sizeof(long long) * kCtBins, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    SG_TRY(check(e, "reference readback"));
    long long tot = 0;
    for (int b = 0; b < kCtBins; ++b) tot += r[b];
    s->ct_n_ref = tot;
    if (hist)
        for (int b = 0; b < kCtBins; ++b) hist[b] = (int64_t)r[b];
    return SG_OK;
}

extern "C" sg_status sg_surr_destroy(sg_ctx* c, int32_t id)
{
    if (!find_surr(c, id)) return fail(SG_EINVAL, "sg_surr_destroy: bad surrogate id");
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->surrogates.erase(id);
    return SG_OK;
}

extern "C" sg_status sg_surr_num_params(sg_ctx* c, int32_t id, int64_t* n)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !n) return fail(SG_EINVAL, "sg_surr_num_params: bad surrogate id or NULL");
    *n = s->n_params;
    return SG_OK;
}

namespace sg {
namespace {
// every buffer a training step touches: a captured step stays valid while none of them moved
std::vector<const void*> buffer_ptrs(const Surrogate& s)
{
    std::vector<const void*> v = {s.master.p, s.mom1.p, s.mom2.p, s.grad.p, s.wb.p, s.wt.p, s.dpre.p, s.fine.p,
                                  s.parts.p, s.yhat.p, s.target.p, s.gy.p, s.loss.p, s.dscan.p, s.steps.p, s.coef.p,
                                  s.segs.p, s.hist.p, s.bias_parts.p, s.d_master.p, s.d_mom1.p, s.d_mom2.p, s.d_grad.p, s.d_wb.p,
                                  s.d_wt.p, s.d_logits.p, s.d_glog.p, s.d_dpre.p, s.d_bias_scratch.p, s.d_segs.p};
    for (int t = 0; t < kNumT; ++t) {
        v.push_back(s.act[t].p);
        v.push_back(s.gact[t].p);
    }
    for (int k = 0; k < kNumD; ++k) {
        v.push_back(s.d_act[k].p);
        v.push_back(s.d_g[k].p);
    }
    return v;
}

void drop_graph(Surrogate& s)
{
    if (s.g_exec) (void)hipGraphExecDestroy(s.g_exec);
    s.g_exec = nullptr;
    s.g_n = 0;
    s.g_ptrs.clear();
}

// forward, L1 (and adversarial) loss, backward, Adam and the loss log on the batch in act[X] / target
sg_status train_body(sg_ctx* c, Surrogate& s, int32_t n)
{
    SG_TRY(forward(c, s, n, true));
    const int64_t P = (int64_t)n * s.H * s.W;
    const int lb = blocks_for(P);
    SG_TRY(check(s.parts.ensure(sizeof(float) * (size_t)lb), "loss workspace"));
    SG_TRY(check(l1_loss((const float*)s.yhat.p, (const float*)s.target.p, P, (float*)s.gy.p, (float*)s.parts.p, lb,
                         (float*)s.loss.p, c->stream),
                 "loss"));
    if (s.adv_weight > 0.f) SG_TRY(adversarial_step(c, s, n));
    SG_TRY(backward(c, s, n));
    SG_TRY(adam(c, s));
    return check(loss_log((const float*)s.loss.p, (const int64_t*)s.steps.p, (float*)s.hist.p, kLossRing, c->stream),
                 "loss log");
}

// capture train_body on a private stream (the caller's stream may be the legacy default stream)
hipError_t capture_step(sg_ctx* c, Surrogate& s, int32_t n)
{
    hipError_t e = hipSuccess;
    if (!s.cap_stream) e = hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipStream_t user = c->stream;
    c->stream = s.cap_stream;
    const sg_status st = train_body(c, s, n);
    c->stream = user;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s.cap_stream, &g);
    if (st != SG_OK && e == hipSuccess) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipGraphInstantiate(&s.g_exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) drop_graph(s);
    return e;
}

// Enqueue one training step on the batch in act[X] / target: the Adam scalars (counted on the device)
// first, then the step, replayed from its graph when one was captured for this shape and buffers.  A new
// shape runs eagerly once (sizing the workspaces), then is captured.  Nothing waits for the device.
sg_status enqueue_step(sg_ctx* c, Surrogate& s, int32_t n, float lr)
{
    const bool disc = s.adv_weight > 0.f;
    SG_TRY(check(adam_coef((int64_t*)s.steps.p, (float*)s.coef.p, lr, kBeta1, kBeta2, disc ? 1 : 0, c->stream),
                 "adam scalars"));
    s.step += 1;
    if (disc) s.d_step += 1;
    s.last_n = n;
    if (!s.use_graph) return train_body(c, s, n);
    const std::vector<const void*> ptrs = buffer_ptrs(s);
    if (s.g_exec && s.g_n == n && ptrs == s.g_ptrs)
        return check(hipGraphLaunch(s.g_exec, c->stream), "training graph launch");
    drop_graph(s);
    if (s.warm_n != n || ptrs != s.warm_ptrs || s.g_failed_n == n) {
        SG_TRY(train_body(c, s, n));
        s.warm_n = n;
        s.warm_ptrs = buffer_ptrs(s);
        return SG_OK;
    }
    hipError_t e = capture_step(c, s, n);
    if (e == hipSuccess && buffer_ptrs(s) != ptrs) e = hipErrorInvalidValue;   // a workspace moved during capture
    if (e != hipSuccess) {   // run this shape eagerly from now on
        drop_graph(s);
        (void)hipGetLastError();
        s.g_failed_n = n;
        return train_body(c, s, n);
    }
    s.g_n = n;
    s.g_ptrs = ptrs;
    return check(hipGraphLaunch(s.g_exec, c->stream), "training graph launch");
}

// wait for the stream, then the losses of the last step
sg_status read_last_losses(sg_ctx* c, Surrogate& s, float* out3)
{
    hipError_t e = hipMemcpyAsync(s.pinned, s.loss.p, sizeof(float) * 3, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "loss readback");
    for (int j = 0; j < 3; ++j) out3[j] = s.pinned[j];
    return SG_OK;
}

sg_status train_pairs_impl(sg_ctx* c, int32_t id, int32_t n, int32_t H, int32_t W, const uint16_t* input,
                           const float* target, float lr, Surrogate** out)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !input || !target) return fail(SG_EINVAL, "sg_surr_train_pairs: bad id or NULL");
    if (n < 1 || n > 65535) return fail(SG_EINVAL, "sg_surr_train_pairs: n in [1, 65535]");
    if (H != s->H || W != s->W)
        return fail(SG_EINVAL, "sg_surr_train_pairs: %dx%d frames, the surrogate takes %dx%d", W, H, s->W, s->H);
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(SG_EINVAL, "sg_surr_train_pairs: bad learning rate");
    (void)hipSetDevice(c->device);
    SG_TRY(ensure_capacity(*s, n, true));
    const int64_t P = (int64_t)n * s->H * s->W;
    SG_TRY(check(hipMemcpyAsync(s->act[X].p, input, sizeof(uint16_t) * 8 * P, hipMemcpyDeviceToDevice, c->stream),
                 "input copy"));
    SG_TRY(check(hipMemcpyAsync(s->target.p, target, sizeof(float) * P, hipMemcpyDeviceToDevice, c->stream),
                 "target copy"));
    *out = s;
    return enqueue_step(c, *s, n, lr);
}

sg_status train_step_impl(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                          const double* poses, float lr, Surrogate** out)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !vol_ids || !probes || !poses) return fail(SG_EINVAL, "sg_surr_train_step: bad id or NULL");
    if (n < 1) return fail(SG_EINVAL, "sg_surr_train_step: n_envs must be >= 1");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(SG_EINVAL, "sg_surr_train_step: bad learning rate");
    (void)hipSetDevice(c->device);
    SG_TRY(check_frames(*s, n, probes));
    SG_TRY(ensure_capacity(*s, n, true));
    SG_TRY(encode_and_render(c, *s, n, vol_ids, probes, poses, (float*)s->target.p));
    *out = s;
    return enqueue_step(c, *s, n, lr);
}
}  // namespace
}  // namespace sg

extern "C" sg_status sg_surr_train_step(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids,
                                        const sg_probe* probes, const double* poses, float lr, float* loss)
{
    if (!loss) return fail(SG_EINVAL, "sg_surr_train_step: NULL loss");
    Surrogate* s = nullptr;
    SG_TRY(train_step_impl(c, id, n, vol_ids, probes, poses, lr, &s));
    float l[3];
    SG_TRY(read_last_losses(c, *s, l));
    *loss = l[0];
    return SG_OK;
}

extern "C" sg_status sg_surr_train_step_async(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids,
                                              const sg_probe* probes, const double* poses, float lr)
{
    Surrogate* s = nullptr;
    return train_step_impl(c, id, n, vol_ids, probes, poses, lr, &s);
}

extern "C" sg_status sg_surr_train_pairs(sg_ctx* c, int32_t id, int32_t n, int32_t H, int32_t W,
                                         const uint16_t* input, const float* target, float lr, float* loss)
{
    if (!loss) return fail(SG_EINVAL, "sg_surr_train_pairs: NULL loss");
    Surrogate* s = nullptr;
    SG_TRY(train_pairs_impl(c, id, n, H, W, input, target, lr, &s));
    float l[3];
    SG_TRY(read_last_losses(c, *s, l));
    *loss = l[0];
    return SG_OK;
}

extern "C" sg_status sg_surr_train_pairs_async(sg_ctx* c, int32_t id, int32_t n, int32_t H, int32_t W,
                                               const uint16_t* input, const float* target, float lr)
{
    Surrogate* s = nullptr;
    return train_pairs_impl(c, id, n, H, W, input, target, lr, &s);
}

extern "C" sg_status sg_surr_loss_history(sg_ctx* c, int32_t id, int64_t first_step, int32_t count, float* out)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !out || count < 0) return fail(SG_EINVAL, "sg_surr_loss_history: bad id, NULL or negative count");
    if (count == 0) return SG_OK;
    const int64_t last = first_step + count - 1;
    if (first_step < 1 || last > s->step || s->step - first_step >= kLossRing)
        return fail(SG_ERANGE, "sg_surr_loss_history: steps %lld..%lld not held (done: %lld, ring of %d)",
                    (long long)first_step, (long long)last, (long long)s->step, kLossRing);
    (void)hipSetDevice(c->device);
    const int64_t a = (first_step - 1) % kLossRing;
    const int64_t n1 = std::min<int64_t>(count, kLossRing - a);   // up to the ring's end, then from its start
    hipError_t e = hipMemcpyAsync(s->pinned, (const float*)s->hist.p + 3 * a, sizeof(float) * 3 * n1,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && count > n1)
        e = hipMemcpyAsync(s->pinned + 3 * n1, s->hist.p, sizeof(float) * 3 * (count - n1), hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "loss history readback");
    std::memcpy(out, s->pinned, sizeof(float) * 3 * count);
    return SG_OK;
}

extern "C" sg_status sg_surr_set_graph(sg_ctx* c, int32_t id, int32_t enable)
{
    Surrogate* s = find_surr(c, id);
    if (!s) return fail(SG_EINVAL, "sg_surr_set_graph: bad id");
    s->use_graph = enable != 0;
    if (!s->use_graph) {
        (void)hipSetDevice(c->device);
        drop_graph(*s);
        s->warm_n = 0;
        s->g_failed_n = 0;
    }
    return SG_OK;
}

extern "C" sg_status sg_surr_step_count(sg_ctx* c, int32_t id, int64_t* steps)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !steps) return fail(SG_EINVAL, "sg_surr_step_count: bad id or NULL");
    *steps = s->step;
    return SG_OK;
}

extern "C" sg_status sg_audit_decide(int32_t n_audit, const float* psnr, float psnr_min, float max_fail_frac,
                                     int32_t* fallback, int32_t* whole)
{
    if (n_audit < 0 || (n_audit > 0 && (!psnr || !fallback)) || !whole)
        return fail(SG_EINVAL, "sg_audit_decide: bad arguments");
    int fails = 0;
    for (int i = 0; i < n_audit; ++i) {
        const bool bad = !(psnr[i] >= psnr_min);   // NaN fails
        fallback[i] = bad ? 1 : 0;
        fails += bad;
    }
    *whole = (n_audit > 0 && (double)fails > (double)max_fail_frac * (double)n_audit) ? 1 : 0;
    return SG_OK;
}

namespace sg {
namespace {
// audited inference into FP32 frames `out` (device, n x H x W); synchronises
sg_status infer_impl(sg_ctx* c, Surrogate* s, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                     const double* poses, float* out, const int32_t* audit_envs, int32_t n_audit, float psnr_min,
                     float max_fail_frac, float* psnr_out, int32_t* n_fallback)
{
    if (n < 1 || n_audit < 0 || n_audit > n || (n_audit > 0 && (!audit_envs || !psnr_out)))
        return fail(SG_EINVAL, "sg_surr_infer: bad sizes");
    std::vector<char> seen(n, 0);
    for (int i = 0; i < n_audit; ++i) {
        const int e = audit_envs[i];
        if (e < 0 || e >= n || seen[e]) return fail(SG_EINVAL, "sg_surr_infer: audit env %d out of range or repeated", e);
        seen[e] = 1;
    }
    (void)hipSetDevice(c->device);
    SG_TRY(check_frames(*s, n, probes));
    SG_TRY(ensure_capacity(*s, n, false));
    const int64_t HW = (int64_t)s->H * s->W;
    SG_TRY(encode_and_render(c, *s, n, vol_ids, probes, poses, nullptr));
    SG_TRY(forward(c, *s, n, false));
    SG_TRY(check(clamp01((const float*)s->yhat.p, out, (int64_t)n * HW, c->stream), "clamp"));
    *n_fallback = 0;
    if (n_audit == 0) return check(hipStreamSynchronize(c->stream), "infer");
    // render the audited envs with the physics path
    std::vector<int32_t> av(audit_envs, audit_envs + n_audit);
    std::vector<int32_t> a_vol(n_audit);
    std::vector<sg_probe> a_probe(n_audit);
    std::vector<double> a_pose(12 * (size_t)n_audit);
    std::vector<int64_t> a_off(n_audit);
    for (int i = 0; i < n_audit; ++i) {
        a_vol[i] = vol_ids[av[i]];
        a_probe[i] = probes[av[i]];
        std::memcpy(&a_pose[12 * (size_t)i], poses + 12 * (size_t)av[i], 12 * sizeof(double));
        a_off[i] = (int64_t)i * HW;
    }
    PhysArgs a;
    StageInfo info;
    SG_TRY(stage_physics(c, n_audit, a_vol.data(), a_probe.data(), a_pose.data(), (float*)s->target.p, a_off.data(),
                         nullptr, a, info));
    SG_TRY(launch_physics(c, a, info));
    SG_TRY(check(s->idx.ensure(sizeof(int32_t) * n_audit), "audit index"));
    SG_TRY(check(s->psnr.ensure(sizeof(float) * n_audit), "audit psnr"));
    SG_TRY(check(hipMemcpyAsync(s->idx.p, av.data(), sizeof(int32_t) * n_audit, hipMemcpyHostToDevice, c->stream),
                 "audit index upload"));
    SG_TRY(check(psnr_indexed(out, (const float*)s->target.p, (const int32_t*)s->idx.p, n_audit, HW,
                              (float*)s->psnr.p, c->stream),
                 "audit psnr"));
    SG_TRY(check(hipMemcpyAsync(psnr_out, s->psnr.p, sizeof(float) * n_audit, hipMemcpyDeviceToHost, c->stream),
                 "psnr readback"));
    SG_TRY(check(hipStreamSynchronize(c->stream), "audit"));
    std::vector<int32_t> fb(n_audit);
    int32_t whole = 0;
    SG_TRY(sg_audit_decide(n_audit, psnr_out, psnr_min, max_fail_frac, fb.data(), &whole));
    if (whole) {
        std::vector<int64_t> offs(n);
        for (int i = 0; i < n; ++i) offs[i] = (int64_t)i * HW;
        SG_TRY(stage_physics(c, n, vol_ids, probes, poses, out, offs.data(), nullptr, a, info));
        SG_TRY(launch_physics(c, a, info));
        *n_fallback = n;
    } else {
        int nf = 0;
        for (int i = 0; i < n_audit; ++i) {
            if (!fb[i]) continue;
            SG_TRY(check(hipMemcpyAsync(out + (int64_t)av[i] * HW, (const float*)s->target.p + (int64_t)i * HW,
                                        sizeof(float) * HW, hipMemcpyDeviceToDevice, c->stream),
                         "fallback copy"));
            ++nf;
        }
        *n_fallback = nf;
    }
    return check(hipStreamSynchronize(c->stream), "infer");
}
}  // namespace
}  // namespace sg

extern "C" sg_status sg_surr_infer(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                                   const double* poses, float* out, const int32_t* audit_envs, int32_t n_audit,
                                   float psnr_min, float max_fail_frac, float* psnr_out, int32_t* n_fallback)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !vol_ids || !probes || !poses || !out || !n_fallback)
        return fail(SG_EINVAL, "sg_surr_infer: bad id or NULL");
    return infer_impl(c, s, n, vol_ids, probes, poses, out, audit_envs, n_audit, psnr_min, max_fail_frac, psnr_out,
                      n_fallback);
}

extern "C" sg_status sg_surr_infer_bf16(sg_ctx* c, int32_t id, int32_t n, const int32_t* vol_ids,
                                        const sg_probe* probes, const double* poses, uint16_t* out_bf16,
                                        const int32_t* audit_envs, int32_t n_audit, float psnr_min,
                                        float max_fail_frac, float* psnr_out, int32_t* n_fallback)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !vol_ids || !probes || !poses || !out_bf16 || !n_fallback)
        return fail(SG_EINVAL, "sg_surr_infer_bf16: bad id or NULL");
    if (n < 1) return fail(SG_EINVAL, "sg_surr_infer_bf16: bad sizes");
    (void)hipSetDevice(c->device);
    SG_TRY(check_frames(*s, n, probes));
    const int64_t P = (int64_t)n * s->H * s->W;
    SG_TRY(check(s->out32.ensure(sizeof(float) * (size_t)P), "FP32 frames"));
    SG_TRY(infer_impl(c, s, n, vol_ids, probes, poses, (float*)s->out32.p, audit_envs, n_audit, psnr_min,
                      max_fail_frac, psnr_out, n_fallback));
    SG_TRY(check(mask_to_bf16((const float*)s->out32.p, nullptr, out_bf16, P, c->stream), "bf16 frames"));
    return check(hipStreamSynchronize(c->stream), "infer");
}

namespace {
const char kMagic[8] = {'S', 'G', 'S', 'U', 'R', 'R', '0', '1'};
const char kMagicCt[8] = {'S', 'G', 'S', 'U', 'R', 'R', 'C', '1'};    // + the CT reference counts
const char kMagicGan[8] = {'S', 'G', 'S', 'U', 'R', 'R', 'G', '1'};   // + the CT reference and the discriminator

const char* magic_of(const Surrogate& s) { return s.adv_weight > 0.f ? kMagicGan : (s.ct ? kMagicCt : kMagic); }
}

extern "C" sg_status sg_surr_save(sg_ctx* c, int32_t id, const char* path)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !path) return fail(SG_EINVAL, "sg_surr_save: bad id or NULL path");
    (void)hipSetDevice(c->device);
    const size_t n = (size_t)s->n_params;
    std::vector<float> buf(3 * n);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(buf.data(), s->master.p, sizeof(float) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + n, s->mom1.p, sizeof(float) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * n, s->mom2.p, sizeof(float) * n, hipMemcpyDeviceToHost);
    std::vector<long long> ref(s->ct ? kCtBins : 0);
    if (e == hipSuccess && s->ct)
        e = hipMemcpy(ref.data(), s->ct_ref.p, sizeof(long long) * kCtBins, hipMemcpyDeviceToHost);
    const size_t dn = (size_t)s->dn_params;
    std::vector<float> dbuf(3 * dn);
    if (e == hipSuccess && dn) e = hipMemcpy(dbuf.data(), s->d_master.p, sizeof(float) * dn, hipMemcpyDeviceToHost);
    if (e == hipSuccess && dn) e = hipMemcpy(dbuf.data() + dn, s->d_mom1.p, sizeof(float) * dn, hipMemcpyDeviceToHost);
    if (e == hipSuccess && dn)
        e = hipMemcpy(dbuf.data() + 2 * dn, s->d_mom2.p, sizeof(float) * dn, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "checkpoint readback");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SG_EINVAL, "cannot open %s for writing", path);
    const int32_t hw[2] = {s->H, s->W};
    const int64_t meta[2] = {s->n_params, s->step};
    bool ok = std::fwrite(magic_of(*s), 1, 8, f) == 8 && std::fwrite(hw, sizeof(hw), 1, f) == 1 &&
              std::fwrite(meta, sizeof(meta), 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), 3 * n, f) == 3 * n;
    if (s->ct) ok = ok && std::fwrite(ref.data(), sizeof(long long), kCtBins, f) == (size_t)kCtBins;
    if (dn) {
        const int64_t dmeta[2] = {s->dn_params, s->d_step};
        ok = ok && std::fwrite(dmeta, sizeof(dmeta), 1, f) == 1 &&
             std::fwrite(dbuf.data(), sizeof(float), 3 * dn, f) == 3 * dn;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SG_OK : fail(SG_EINVAL, "write to %s failed", path);
}

extern "C" sg_status sg_surr_load(sg_ctx* c, int32_t id, const char* path)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !path) return fail(SG_EINVAL, "sg_surr_load: bad id or NULL path");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SG_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t hw[2];
    int64_t meta[2];
    const size_t n = (size_t)s->n_params;
    std::vector<float> buf(3 * n);
    std::vector<long long> ref(2 * kCtBins, 0);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, magic_of(*s), 8) == 0 &&
              std::fread(hw, sizeof(hw), 1, f) == 1 && std::fread(meta, sizeof(meta), 1, f) == 1 &&
              hw[0] == s->H && hw[1] == s->W && meta[0] == s->n_params &&
              std::fread(buf.data(), sizeof(float), 3 * n, f) == 3 * n;
    if (s->ct) ok = ok && std::fread(ref.data(), sizeof(long long), kCtBins, f) == (size_t)kCtBins;
    const size_t dn = (size_t)s->dn_params;
    std::vector<float> dbuf(3 * dn);
    int64_t dmeta[2] = {0, 0};
    if (dn)
        ok = ok && std::fread(dmeta, sizeof(dmeta), 1, f) == 1 && dmeta[0] == s->dn_params &&
             std::fread(dbuf.data(), sizeof(float), 3 * dn, f) == 3 * dn;
    std::fclose(f);
    long long tot = 0;
    for (int b = 0; b < kCtBins && s->ct; ++b) {
        ok = ok && ref[b] >= 0;
        tot += ref[b];
        ref[kCtBins + b] = tot;
    }
    if (!ok) return fail(SG_EINVAL, "%s is not a checkpoint of this surrogate (%dx%d, %lld params)", path, s->W,
                         s->H, (long long)s->n_params);
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(s->master.p, buf.data(), sizeof(float) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->mom1.p, buf.data() + n, sizeof(float) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->mom2.p, buf.data() + 2 * n, sizeof(float) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && s->ct)
        e = hipMemcpy(s->ct_ref.p, ref.data(), sizeof(long long) * 2 * kCtBins, hipMemcpyHostToDevice);
    if (e == hipSuccess && dn) e = hipMemcpy(s->d_master.p, dbuf.data(), sizeof(float) * dn, hipMemcpyHostToDevice);
    if (e == hipSuccess && dn) e = hipMemcpy(s->d_mom1.p, dbuf.data() + dn, sizeof(float) * dn, hipMemcpyHostToDevice);
    if (e == hipSuccess && dn)
        e = hipMemcpy(s->d_mom2.p, dbuf.data() + 2 * dn, sizeof(float) * dn, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "checkpoint upload");
    s->step = meta[1];
    if (s->ct) s->ct_n_ref = tot;
    if (dn) {
        s->d_step = dmeta[1];
        SG_TRY(disc_refresh_bf16(c, *s));
    }
    const int64_t st[2] = {s->step, s->d_step};   // the device's update counters (Adam's bias correction)
    e = hipMemcpy(s->steps.p, st, sizeof(st), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "checkpoint upload");
    return refresh_bf16(c, *s);
}

extern "C" sg_status sg_surr_get_params(sg_ctx* c, int32_t id, float* host)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !host) return fail(SG_EINVAL, "sg_surr_get_params: bad id or NULL");
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host, s->master.p, sizeof(float) * s->n_params, hipMemcpyDeviceToHost);
    return check(e, "parameter readback");
}

extern "C" sg_status sg_surr_get_grads(sg_ctx* c, int32_t id, float* host)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !host) return fail(SG_EINVAL, "sg_surr_get_grads: bad id or NULL");
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host, s->grad.p, sizeof(float) * s->n_params, hipMemcpyDeviceToHost);
    return check(e, "gradient readback");
}

extern "C" sg_status sg_surr_set_params(sg_ctx* c, int32_t id, const float* host)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !host) return fail(SG_EINVAL, "sg_surr_set_params: bad id or NULL");
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(s->master.p, host, sizeof(float) * s->n_params, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");
    return refresh_bf16(c, *s);
}

extern "C" sg_status sg_surr_get_batch(sg_ctx* c, int32_t id, uint16_t* input, float* target)
{
    Surrogate* s = find_surr(c, id);
    if (!s || (!input && !target)) return fail(SG_EINVAL, "sg_surr_get_batch: bad id or NULL");
    if (s->last_n < 1) return fail(SG_ESTATE, "sg_surr_get_batch: no training step yet");
    (void)hipSetDevice(c->device);
    const int64_t P = (int64_t)s->last_n * s->H * s->W;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && input) e = hipMemcpy(input, s->act[X].p, sizeof(uint16_t) * 8 * P, hipMemcpyDeviceToHost);
    if (e == hipSuccess && target) e = hipMemcpy(target, s->target.p, sizeof(float) * P, hipMemcpyDeviceToHost);
    return check(e, "batch readback");
}

extern "C" sg_status sg_surr_tensor(sg_ctx* c, int32_t id, int32_t kind, int32_t index, void* host, int64_t* n)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !n) return fail(SG_EINVAL, "sg_surr_tensor: bad id or NULL");
    if (s->last_n < 1) return fail(SG_ESTATE, "sg_surr_tensor: no training step yet");
    const int ln = s->last_n;
    const int64_t P = (int64_t)ln * s->H * s->W;
    const bool disc = kind >= SG_SURR_T_DISC_ACT && kind <= SG_SURR_T_DISC_MOM2;
    if (disc && s->adv_weight <= 0.f) return fail(SG_EINVAL, "sg_surr_tensor: the surrogate has no discriminator");
    const void* src = nullptr;
    int64_t count = 0;
    size_t esz = sizeof(float);
    switch (kind) {
    case SG_SURR_T_ACT:
    case SG_SURR_T_GRAD:
        if (index < (kind == SG_SURR_T_GRAD ? 1 : 0) || index >= kNumT)
            return fail(SG_EINVAL, "sg_surr_tensor: tensor index %d", index);
        src = kind == SG_SURR_T_ACT ? s->act[index].p : s->gact[index].p;
        count = tensor_elems(*s, index, ln);
        if (kind == SG_SURR_T_ACT) esz = sizeof(uint16_t);
        break;
    case SG_SURR_T_YHAT: src = s->yhat.p; count = P; break;
    case SG_SURR_T_TARGET: src = s->target.p; count = P; break;
    case SG_SURR_T_GY: src = s->gy.p; count = P; break;
    case SG_SURR_T_MOM1: src = s->mom1.p; count = s->n_params; break;
    case SG_SURR_T_MOM2: src = s->mom2.p; count = s->n_params; break;
    case SG_SURR_T_DSCAN: src = s->dscan.p; count = P * kScanC; esz = sizeof(uint16_t); break;
    case SG_SURR_T_DISC_ACT:
    case SG_SURR_T_DISC_GRAD:
        if (index < 0 || index >= kNumD) return fail(SG_EINVAL, "sg_surr_tensor: discriminator tensor %d", index);
        src = kind == SG_SURR_T_DISC_ACT ? s->d_act[index].p : s->d_g[index].p;
        count = disc_elems(*s, index, 3 * ln);
        if (kind == SG_SURR_T_DISC_ACT) esz = sizeof(uint16_t);
        break;
    case SG_SURR_T_DISC_LOGITS: src = s->d_logits.p; count = disc_elems(*s, kNumD, 3 * ln); break;
    case SG_SURR_T_DISC_GLOG: src = s->d_glog.p; count = disc_elems(*s, kNumD, 3 * ln); break;
    case SG_SURR_T_DISC_MOM1: src = s->d_mom1.p; count = s->dn_params; break;
    case SG_SURR_T_DISC_MOM2: src = s->d_mom2.p; count = s->dn_params; break;
    default: return fail(SG_EINVAL, "sg_surr_tensor: kind %d", kind);
    }
    if (!host) {
        *n = count;
        return SG_OK;
    }
    if (*n != count) return fail(SG_EINVAL, "sg_surr_tensor: %lld elements asked, the tensor has %lld",
                                 (long long)*n, (long long)count);
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host, src, esz * (size_t)count, hipMemcpyDeviceToHost);
    return check(e, "tensor readback");
}

extern "C" sg_status sg_surr_gan_losses(sg_ctx* c, int32_t id, float* loss_d, float* loss_adv)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !loss_d || !loss_adv) return fail(SG_EINVAL, "sg_surr_gan_losses: bad id or NULL");
    if (s->adv_weight <= 0.f) return fail(SG_EINVAL, "sg_surr_gan_losses: the surrogate has no adversarial term");
    if (s->last_n < 1) return fail(SG_ESTATE, "sg_surr_gan_losses: no training step yet");
    (void)hipSetDevice(c->device);
    float l[3];
    SG_TRY(read_last_losses(c, *s, l));
    *loss_d = l[1];
    *loss_adv = l[2];
    return SG_OK;
}

extern "C" sg_status sg_surr_disc_num_params(sg_ctx* c, int32_t id, int64_t* n)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !n) return fail(SG_EINVAL, "sg_surr_disc_num_params: bad id or NULL");
    if (s->adv_weight <= 0.f) return fail(SG_EINVAL, "sg_surr_disc_num_params: the surrogate has no discriminator");
    *n = s->dn_params;
    return SG_OK;
}

namespace {
sg_status disc_copy(sg_ctx* c, int32_t id, float* host, int what, const char* name)
{
    Surrogate* s = find_surr(c, id);
    if (!s || !host) return fail(SG_EINVAL, "%s: bad id or NULL", name);
    if (s->adv_weight <= 0.f) return fail(SG_EINVAL, "%s: the surrogate has no discriminator", name);
    (void)hipSetDevice(c->device);
    const size_t bytes = sizeof(float) * s->dn_params;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
        if (what == 0) e = hipMemcpy(host, s->d_master.p, bytes, hipMemcpyDeviceToHost);
        if (what == 1) e = hipMemcpy(host, s->d_grad.p, bytes, hipMemcpyDeviceToHost);
        if (what == 2) e = hipMemcpy(s->d_master.p, host, bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, name);
    return what == 2 ? disc_refresh_bf16(c, *s) : SG_OK;
}
}  // namespace

extern "C" sg_status sg_surr_disc_get_params(sg_ctx* c, int32_t id, float* host)
{
    return disc_copy(c, id, host, 0, "sg_surr_disc_get_params");
}

extern "C" sg_status sg_surr_disc_get_grads(sg_ctx* c, int32_t id, float* host)
{
    return disc_copy(c, id, host, 1, "sg_surr_disc_get_grads");
}

extern "C" sg_status sg_surr_disc_set_params(sg_ctx* c, int32_t id, const float* host)
{
    return disc_copy(c, id, const_cast<float*>(host), 2, "sg_surr_disc_set_params");
}
