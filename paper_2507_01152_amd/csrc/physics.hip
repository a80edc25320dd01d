// Model-based B-mode simulation kernels for gfx950 (SonoGym, App. B.2).
//
// Two persistent work-queue kernels per step (the kernel boundary is the only
// synchronisation between them):
//  * ray kernel -- one wave64 per scanline, lanes along depth, marching down
//                  in 64-row chunks.  Per chunk: sample the plane (nearest
//                  label, optional FP64 trilinear CT), boundary indicator,
//                  reflection and transmission, wave-level scans for the
//                  transmission product and the attenuation integral
//                  (remaining energy E), per-voxel scatterer (Philox4x32-10
//                  keyed by voxel index, Box-Muller, density gate), the
//                  reflection source R' = G*E*cos(theta)*|r|.  R' and T go
//                  into a per-wave LDS ring of four chunks (the first two
//                  mirrored past its end so filter windows never wrap), and the axial
//                  Gaussian is applied one chunk behind.  The axially filtered
//                  fields and E are written scanline-major, coalesced along
//                  the scanline.  The next chunk's labels are gathered one
//                  chunk ahead.
//  * PSF kernel -- one workgroup per tile of TX scanlines x 64 rows: stages
//                  the axially filtered fields with the lateral halo in LDS,
//                  applies the lateral Gaussian, composes
//                  I = K(x)R' + E*K(x)T, log-compresses and stores the frame
//                  row-major (coalesced along image rows).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kRing = 4 * kWave;         // rows held per wave in the axial ring (power of two)
constexpr int kRingAlloc = kRing + 2 * kWave;   // + mirror of the first two chunks: windows never wrap
constexpr int kTaps = 2 * kMaxPsfRadius + 1;
constexpr int kTileRows = 64;            // PSF tile height
constexpr int kAS = kTileRows + 1;       // padded LDS column stride

// Philox4x32-10 (Salmon et al., SC'11): multipliers and Weyl key increments.
constexpr uint32_t kPhM0 = 0xD2511F53u;
constexpr uint32_t kPhM1 = 0xCD9E8D57u;
constexpr uint32_t kPhW0 = 0x9E3779B9u;
constexpr uint32_t kPhW1 = 0xBB67AE85u;

// counter (n_lo, 0, c2_in, 0): n_lo = voxel or cell index, c2_in = noise scale
__device__ __forceinline__ void philox4x32_10(uint32_t n_lo, uint32_t k0, uint32_t k1, uint32_t w[4],
                                              uint32_t c2_in = 0u)
{
    uint32_t c0 = n_lo, c1 = 0u, c2 = c2_in, c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply-add instruction per product
        const uint64_t p0 = (uint64_t)kPhM0 * c0;
        const uint64_t p1 = (uint64_t)kPhM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += kPhW0;
        k1 += kPhW1;
    }
    w[0] = c0;
    w[1] = c1;
    w[2] = c2;
    w[3] = c3;
}

__device__ __forceinline__ int32_t q16(int32_t p0, int32_t dx, int32_t dy, int x, int y)
{
    // exact for in-range planes; unsigned arithmetic keeps wrap-around defined
    return (int32_t)((uint32_t)p0 + (uint32_t)x * (uint32_t)dx + (uint32_t)y * (uint32_t)dy);
}

// nearest voxel of pixel (x, y): its linear index, -1 outside the grid, and
// (inside) its byte offset in the bricked label map
__device__ __forceinline__ int32_t voxel_at(const EnvDev& e, const VolDev& v, int x, int y, uint32_t& boff)
{
    // round half up: floor((q + 2^15) / 2^16) as an arithmetic shift
    const int32_t ix = (int32_t)((uint32_t)q16(e.P0[0], e.DX[0], e.DY[0], x, y) + 32768u) >> 16;
    const int32_t iy = (int32_t)((uint32_t)q16(e.P0[1], e.DX[1], e.DY[1], x, y) + 32768u) >> 16;
    const int32_t iz = (int32_t)((uint32_t)q16(e.P0[2], e.DX[2], e.DY[2], x, y) + 32768u) >> 16;
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    boff = in ? brick_offset(v, ix, iy, iz) : 0u;
    return in ? (iz * v.ny + iy) * v.nx + ix : -1;
}

// Volume reads through the global address space: the volume pointers are
// read from memory, so plain dereferences compile to flat loads.
template <typename T>
__device__ __forceinline__ T ld_global(const T* p, int64_t i)
{
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

// label of a voxel from voxel_at / voxel_at_q (air outside the grid)
__device__ __forceinline__ int label_of(const VolDev& v, int32_t vox, uint32_t boff)
{
    return vox >= 0 ? (int)ld_global(v.labels, (int64_t)boff) : 0;
}

__device__ __forceinline__ double ct_corner(const VolDev& v, int32_t ix, int32_t iy, int32_t iz)
{
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    return in ? (double)ld_global(v.ct, (iz * v.ny + iy) * v.nx + ix) : -1000.0;
}

// impedance from CT: max(HU + 1000, 0), HU trilinear in FP64 (successive
// linear interpolation along x, y, z; outside corners -1000 HU)
__device__ __forceinline__ double z_from_ct(const EnvDev& e, const VolDev& v, int x, int y)
{
    int32_t b[3];
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int32_t q = q16(e.P0[c], e.DX[c], e.DY[c], x, y);
        b[c] = q >> 16;
        w[c] = (double)(q & 0xFFFF) * (1.0 / 65536.0);
    }
    double cy[2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        double cx[2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const double h0 = ct_corner(v, b[0], b[1] + dy, b[2] + dz);
            const double h1 = ct_corner(v, b[0] + 1, b[1] + dy, b[2] + dz);
            cx[dy] = h0 + w[0] * (h1 - h0);
        }
        cy[dz] = cx[0] + w[1] * (cx[1] - cx[0]);
    }
    const double z = cy[0] + w[2] * (cy[1] - cy[0]) + 1000.0;
    return z > 0.0 ? z : 0.0;
}

// nearest voxel at Q16 position q: linear index (-1 outside the grid) and bricked byte offset
__device__ __forceinline__ int32_t voxel_at_q(const VolDev& v, const int32_t q[3], uint32_t& boff)
{
    const int32_t ix = (int32_t)((uint32_t)q[0] + 32768u) >> 16;
    const int32_t iy = (int32_t)((uint32_t)q[1] + 32768u) >> 16;
    const int32_t iz = (int32_t)((uint32_t)q[2] + 32768u) >> 16;
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    boff = in ? brick_offset(v, ix, iy, iz) : 0u;
    return in ? (iz * v.ny + iy) * v.nx + ix : -1;
}

// label at Q16 position q (nearest voxel, air outside)
__device__ __forceinline__ int label_at_q(const VolDev& v, int32_t q0, int32_t q1, int32_t q2)
{
    const int32_t ix = (int32_t)((uint32_t)q0 + 32768u) >> 16;
    const int32_t iy = (int32_t)((uint32_t)q1 + 32768u) >> 16;
    const int32_t iz = (int32_t)((uint32_t)q2 + 32768u) >> 16;
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    return in ? (int)ld_global(v.labels, (int64_t)brick_offset(v, ix, iy, iz)) : 0;
}

__device__ __forceinline__ float uniform24(uint32_t w)
{
    // (2*(w >> 9) + 1) * 2^-24: odd 24-bit numerator, exact in FP32
    return (float)((w >> 9) * 2u + 1u) * 0x1p-24f;
}

// Box-Muller N0 = sqrt(-2 ln u0) cos(2 pi u1) with hardware log2 / sqrt / cos(2 pi x)
__device__ __forceinline__ float box_muller(uint32_t w0, uint32_t w1)
{
    const float m2ln = __builtin_amdgcn_logf(uniform24(w0)) * -1.3862943611198906f;   // -2 ln 2
    return __builtin_amdgcn_sqrtf(m2ln) * __builtin_amdgcn_cosf(uniform24(w1));
}

// Scatterer draw of voxel (ix, iy, iz) -- index vox, scale-0 words in w --
// for a volume with S > 1 noise scales: scale s draws on cells of 2^s voxels
// (counter (cell, 0, s, 0)); n0 = sum_s N0_s / sqrt(S); the gate sums the
// integer quantised normals Q[w2_s >> 20] (units of 2^-20) exactly and tests
// the sum against the label's integer threshold floor(sqrt(S) mu1 2^20).
__device__ __forceinline__ void scatter_multiscale(const VolDev& v, const int32_t* __restrict__ q_lut, int32_t thr,
                                                int32_t ix, int32_t iy, int32_t iz, const uint32_t w[4],
                                                float& n0, bool& gate)
{
    float s0 = box_muller(w[0], w[1]);
    int32_t s1 = q_lut[w[2] >> 20];
    for (int s = 1; s < v.scales; ++s) {
        const uint32_t mx = ((uint32_t)v.nx + (1u << s) - 1u) >> s;
        const uint32_t my = ((uint32_t)v.ny + (1u << s) - 1u) >> s;
        const uint32_t cell = (((uint32_t)iz >> s) * my + ((uint32_t)iy >> s)) * mx + ((uint32_t)ix >> s);
        uint32_t ws[4];
        philox4x32_10(cell, v.key0, v.key1, ws, (uint32_t)s);
        s0 += box_muller(ws[0], ws[1]);
        s1 += q_lut[ws[2] >> 20];
    }
    n0 = s0 * (float)(1.0 / sqrt((double)v.scales));
    gate = s1 <= thr;
}

// ---- wave64 data movement on DPP (GFX9 controls) -----------------------
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
constexpr int kWaveShl1 = 0x130;   // lane i reads lane i + 1
constexpr int kWaveShr1 = 0x138;   // lane i reads lane i - 1

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_f(float old, float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWS, 0xf, false));
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp_i(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_d(double old, double v)
{
    const uint64_t o = __double_as_longlong(old), x = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)x, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(x >> 32), CTRL,
                                                              ROWS, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// inclusive scans over the 64 lanes (rows of 16 by row shifts, then the
// row totals by row broadcasts)
__device__ __forceinline__ float wave_scan_mul(float v)
{
    v *= dpp_f<kRowShr1>(1.f, v);
    v *= dpp_f<kRowShr2>(1.f, v);
    v *= dpp_f<kRowShr4>(1.f, v);
    v *= dpp_f<kRowShr8>(1.f, v);
    v *= dpp_f<kRowBcast15, 0xa>(1.f, v);
    v *= dpp_f<kRowBcast31, 0xc>(1.f, v);
    return v;
}

__device__ __forceinline__ float wave_scan_add(float v)
{
    v += dpp_f<kRowShr1>(0.f, v);
    v += dpp_f<kRowShr2>(0.f, v);
    v += dpp_f<kRowShr4>(0.f, v);
    v += dpp_f<kRowShr8>(0.f, v);
    v += dpp_f<kRowBcast15, 0xa>(0.f, v);
    v += dpp_f<kRowBcast31, 0xc>(0.f, v);
    return v;
}

__device__ __forceinline__ float lane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ double lane_d(double v, int lane)
{
    const uint64_t x = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// store the pair for ring slot `slot` (< kRing) and its mirror
__device__ __forceinline__ void ring_put(float2* ring, int slot, float2 f)
{
    ring[slot] = f;
    if (slot < kRingAlloc - kRing) ring[slot + kRing] = f;
}

__device__ __forceinline__ void wave_sync_lds()
{
    // order this wave's LDS writes before its later LDS reads (LDS executes
    // one wave's instructions in issue order; this stops compiler reordering)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// cos(theta): Sobel (1,2,1) on [label differs from the centre label] with
// clamped image coordinates, in physical units, where G is set.  Evaluated
// by the whole wave (lane = row of a 64-row chunk starting at y0) with one
// label gather per side column (x -+ 1) per lane: the side labels of rows
// y - 1 and y + 1 come from the neighbouring lanes, those of the rows just
// outside the chunk from gathers that run only when an edge lane needs them.
// q: Q16 position of (x, y); lab_up / lab_dn: labels of (x, y-1) / (x, y+1)
// (already clamped).  Every lane must call it (uniform control flow).
__device__ __forceinline__ float incidence_cos_wave(const EnvDev& e, const VolDev& v, const int32_t q[3], int x,
                                                   int y0, int lane, bool G, int lab, int lab_up, int lab_dn)
{
    const int xl = x > 0 ? -1 : 0, xr = x < e.W - 1 ? 1 : 0;
    uint32_t ol[3], orr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ol[c] = (uint32_t)(xl * e.DX[c]);
        orr[c] = (uint32_t)(xr * e.DX[c]);
    }
    const int sl = label_at_q(v, (int32_t)((uint32_t)q[0] + ol[0]), (int32_t)((uint32_t)q[1] + ol[1]),
                              (int32_t)((uint32_t)q[2] + ol[2]));
    const int sr = label_at_q(v, (int32_t)((uint32_t)q[0] + orr[0]), (int32_t)((uint32_t)q[1] + orr[1]),
                              (int32_t)((uint32_t)q[2] + orr[2]));
    // rows y - 1 and y + 1 from lanes - 1 and + 1 (lanes 0 and 63 keep their own row: the clamp at the image's
    // top and bottom rows)
    int sl_up = dpp_i<kWaveShr1>(sl, sl), sr_up = dpp_i<kWaveShr1>(sr, sr);
    int sl_dn = dpp_i<kWaveShl1>(sl, sl), sr_dn = dpp_i<kWaveShl1>(sr, sr);
    const uint64_t gm = __builtin_amdgcn_ballot_w64(G);
    const bool top = (gm & 1ull) && y0 > 0;             // lane 0 needs row y0 - 1
    const bool bot = (gm >> (kWave - 1)) & 1ull;       // lane 63 needs row y0 + 64 (G implies it is inside)
    if (top || bot) {
        const uint32_t dy = lane == 0 ? (uint32_t)(-e.DY[0]) : (uint32_t)e.DY[0];
        const uint32_t dy1 = lane == 0 ? (uint32_t)(-e.DY[1]) : (uint32_t)e.DY[1];
        const uint32_t dy2 = lane == 0 ? (uint32_t)(-e.DY[2]) : (uint32_t)e.DY[2];
        const int el = label_at_q(v, (int32_t)((uint32_t)q[0] + ol[0] + dy), (int32_t)((uint32_t)q[1] + ol[1] + dy1),
                                  (int32_t)((uint32_t)q[2] + ol[2] + dy2));
        const int er = label_at_q(v, (int32_t)((uint32_t)q[0] + orr[0] + dy),
                                  (int32_t)((uint32_t)q[1] + orr[1] + dy1), (int32_t)((uint32_t)q[2] + orr[2] + dy2));
        if (lane == 0 && top) {
            sl_up = el;
            sr_up = er;
        }
        if (lane == kWave - 1 && bot) {
            sl_dn = el;
            sr_dn = er;
        }
    }
    const int b00 = sl_up != lab, b02 = sr_up != lab, b10 = sl != lab, b12 = sr != lab;
    const int b20 = sl_dn != lab, b22 = sr_dn != lab, b01 = lab_up != lab, b21 = lab_dn != lab;
    const int sx = (b02 - b00) + 2 * (b12 - b10) + (b22 - b20);
    const int sy = (b20 - b00) + 2 * (b21 - b01) + (b22 - b02);
    // |gy| / |(gx, gy)| with gx = sx / dx, gy = sy / dy, as |sy dx| / |(sx dy, sy dx)|
    // with the hardware reciprocal square root (about 1 ulp) instead of three divisions and a square root
    const float p = (float)sx * (float)e.dy, r = (float)sy * (float)e.dx;
    const float h2 = p * p + r * r;
    return h2 == 0.f ? 1.f : fminf(fabsf(r) * __builtin_amdgcn_rsqf(h2), 1.f);
}

// Axial filter of one chunk from the ring of (R', T) pairs: lane l outputs
// row y0 + l.  Taps go in groups of four, the next group's ring reads issued
// before this group's FMAs; kax (16-byte aligned, kTaps + 7 entries) holds
// zeros past 2 ra, and a zero tap leaves a finite sum unchanged, so the sums
// are those of the taps 0..2 ra in order.
__device__ __forceinline__ void axial_from_ring(const float2* ring, const float* kax, int ra, int y0, int lane,
                                                float& aR, float& aT)
{
    float s1 = 0.f, s2 = 0.f;
    // rows y0 + lane - ra + j live at slot ((y0 - ra) mod kRing) + lane + j; the reads
    // reach j = 2 ra + 7 (one group past the last), so the slot is at most
    // (kRing - ra) + 63 + 2 ra + 7 < kRingAlloc for ra <= kMaxPsfRadius, and the row
    // at most y0 + 63 + ra + 7, inside the chunk written before this filter runs
    const float2* p = ring + ((y0 - ra + kRing) & (kRing - 1)) + lane;
    const int ng = (2 * ra + 4) >> 2;   // groups of four taps covering 0..2 ra
    const float4* k4 = reinterpret_cast<const float4*>(kax);
    // two register sets in turn: the next group's taps and ring values are read
    // before this group's FMAs (taps up to 2 ra + 7, zero past 2 ra)
    float4 ka = k4[0], kb;
    float2 a0 = p[0], a1 = p[1], a2 = p[2], a3 = p[3], b0, b1, b2, b3;
    for (int g = 0;;) {
        kb = k4[g + 1];
        b0 = p[4 * g + 4];   // read past the last group too (unused; in bounds, see above)
        b1 = p[4 * g + 5];
        b2 = p[4 * g + 6];
        b3 = p[4 * g + 7];
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the FMAs
        s1 = fmaf(ka.x, a0.x, s1);
        s2 = fmaf(ka.x, a0.y, s2);
        s1 = fmaf(ka.y, a1.x, s1);
        s2 = fmaf(ka.y, a1.y, s2);
        s1 = fmaf(ka.z, a2.x, s1);
        s2 = fmaf(ka.z, a2.y, s2);
        s1 = fmaf(ka.w, a3.x, s1);
        s2 = fmaf(ka.w, a3.y, s2);
        if (++g >= ng) break;
        ka = k4[g + 1];
        a0 = p[4 * g + 4];
        a1 = p[4 * g + 5];
        a2 = p[4 * g + 6];
        a3 = p[4 * g + 7];
        __builtin_amdgcn_sched_barrier(0);
        s1 = fmaf(kb.x, b0.x, s1);
        s2 = fmaf(kb.x, b0.y, s2);
        s1 = fmaf(kb.y, b1.x, s1);
        s2 = fmaf(kb.y, b1.y, s2);
        s1 = fmaf(kb.z, b2.x, s1);
        s2 = fmaf(kb.z, b2.y, s2);
        s1 = fmaf(kb.w, b3.x, s1);
        s2 = fmaf(kb.w, b3.y, s2);
        if (++g >= ng) break;
    }
    aR = s1;
    aT = s2;
}

// One scanline of the ray pass, executed by one wave (lane = depth row).
// MS: the volume may have several noise scales; LAB: label volume whose
// boundaries take (r, t) from the label-pair table (no CT, no FP64 impedance
// path); DBG: debug planes are written.  Separate instantiations, so the
// common code keeps its registers.
template <bool MS, bool LAB, bool DBG>
__device__ void ray_scanline(const PhysArgs& a, const EnvDev& e, const VolDev& v, const TissueDev* tab,
                             const float2* pair_rt, const float* kax, float2* ring, int x, int lane)
{
    const int H = e.H;
    float* fR = a.fR + e.scr_off + (int64_t)x * e.ld;
    float* fT = a.fT + e.scr_off + (int64_t)x * e.ld;
    float* fE = a.fE + e.scr_off + (int64_t)x * e.ld;
    if (!e.valid) {
        for (int y = lane; y < H; y += kWave) {
            fR[y] = 0.f;
            fT[y] = 0.f;
            fE[y] = 0.f;
        }
        return;
    }
    const bool ct = !LAB && v.ct != nullptr;
    const int ra = e.rax;
    // rows -64..-1 of the ring read as zeros (zero padding above the image)
    ring_put(ring, kRing - kWave + lane, make_float2(0.f, 0.f));

    float carry_t = 1.f;     // transmission product of the rows above the chunk
    float carry_a = 0.f;     // attenuation integral (sum of alpha) above the chunk,
    float carry_c = 0.f;     // with its Kahan compensation (integral = carry_a - carry_c)
    const float coef2 = (float)e.coef2;
    const bool pairs = LAB || (!ct && pair_rt != nullptr);
    const int n_lab = a.n_labels;
    float E_prev = 0.f;      // E of the previous chunk (its axial output is pending)

    uint32_t boff;
    int32_t vox = voxel_at(e, v, x, lane, boff);
    int lab = label_of(v, vox, boff);
    double Z = ct ? z_from_ct(e, v, x, lane) : 0.0;
    int32_t q[3];    // Q16 position of (x, y0 + lane)
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = q16(e.P0[c], e.DX[c], e.DY[c], x, lane);
    int lab_last_prev = 0;   // label of row y0 - 1 (previous chunk's last row)

    const int n_chunks = (H + kWave - 1) / kWave;
    for (int k = 0; k < n_chunks; ++k) {
        const int y0 = k * kWave;
        const int y = y0 + lane;
        const bool act = y < H;
        // gather the next chunk's labels (and CT) ahead of use
        int32_t qn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) qn[c] = (int32_t)((uint32_t)q[c] + (uint32_t)e.DY[c] * (uint32_t)kWave);
        uint32_t boff_n;
        const int32_t vox_n = voxel_at_q(v, qn, boff_n);
        const int lab_n = label_of(v, vox_n, boff_n);
        const double Zct_n = ct ? z_from_ct(e, v, x, y + kWave) : 0.0;

        // scatterer of this chunk's voxels (computed for every lane, selected below)
        uint32_t w[4];
        philox4x32_10((uint32_t)vox, v.key0, v.key1, w);
        const TissueDev tt = tab[lab];
        const bool inside = act && vox >= 0;
        float T;
        if (!MS || v.scales <= 1) {
            const float n0 = box_muller(w[0], w[1]);
            T = (inside && (unsigned long long)w[2] < tt.thr) ? n0 * tt.sigma0 + tt.mu0 : 0.f;
        } else {
            float n0;
            bool gate;
            scatter_multiscale(v, a.q_lut, a.ms_thr[lab * kMaxNoiseScales + v.scales - 1],
                               (int32_t)((uint32_t)q[0] + 32768u) >> 16,
                               (int32_t)((uint32_t)q[1] + 32768u) >> 16, (int32_t)((uint32_t)q[2] + 32768u) >> 16, w,
                               n0, gate);
            T = (inside && gate) ? n0 * tt.sigma0 + tt.mu0 : 0.f;
        }

        // boundary with the next row: lane i + 1, or the next chunk's first row
        const int lab_first_n = __builtin_amdgcn_readlane(lab_n, 0);
        const int lab_nr = dpp_i<kWaveShl1>(lab_first_n, lab);
        const int lab_pr = dpp_i<kWaveShr1>(y0 > 0 ? lab_last_prev : lab, lab);   // row y - 1 (clamped)
        const bool G = act && (y < H - 1) && (lab != lab_nr);
        float r = 0.f, t = 1.f;
        if (pairs) {
            // label volume: the pair table holds the FP64 expressions below, evaluated per label pair
            if (G) {
                const float2 p = pair_rt[lab * n_lab + lab_nr];
                r = p.x;
                t = p.y;
            }
        } else {
            const double Zc = ct ? Z : (double)tt.Z;
            const double Z_first_n = ct ? lane_d(Zct_n, 0) : (double)tab[lab_first_n].Z;
            const double Z_nr = dpp_d<kWaveShl1>(Z_first_n, Zc);
            if (G && Zc != Z_nr) {
                if (Zc == 0.0 || Z_nr == 0.0 || __builtin_isinf(Zc) || __builtin_isinf(Z_nr)) {
                    r = Z_nr > Zc ? 1.f : -1.f;
                    t = 0.f;
                } else {
                    const double s = Zc + Z_nr;
                    r = (float)((Z_nr - Zc) / s);
                    t = (float)((2.0 * Zc / s) * (2.0 * Z_nr / s));
                }
            }
        }
        // inclusive wave scans (FP32 transmission product and alpha sum; tree
        // order within the chunk and a compensated sum of the chunk totals, so
        // the integral's relative error stays near 9 u), shifted by one lane
        // for the exclusive prefix
        const uint64_t gmask = __builtin_amdgcn_ballot_w64(G);
        const float tp = gmask ? wave_scan_mul(act ? t : 1.f) : 1.f;
        const float as = wave_scan_add(act ? tt.alpha : 0.f);
        const float t_ex = dpp_f<kWaveShr1>(1.f, tp);
        const float a_ex = dpp_f<kWaveShr1>(0.f, as);
        // E = E0 * prod(t) * exp(-f dy alpha-integral), as 2^(-coef2 * sum)
        const float E = e.E0 * (carry_t * t_ex) * __builtin_amdgcn_exp2f(-coef2 * ((carry_a + a_ex) - carry_c));
        carry_t *= lane_f(tp, kWave - 1);
        {   // compensated running sum of the chunk totals
            const float yk = lane_f(as, kWave - 1) - carry_c;
            const float tk = carry_a + yk;
            carry_c = (tk - carry_a) - yk;
            carry_a = tk;
        }

        float cs = 1.f;
        if (gmask) {   // uniform: the wave-level Sobel reads neighbouring lanes
            const float c = incidence_cos_wave(e, v, q, x, y0, lane, G, lab, y > 0 ? lab_pr : lab, lab_nr);
            if (G) cs = c;
        }
        const float Rp = G ? E * cs * fabsf(r) : 0.f;

        // ring slot of this chunk, then the axial filter of the previous chunk
        ring_put(ring, (y0 & (kRing - 1)) + lane, act ? make_float2(Rp, T) : make_float2(0.f, 0.f));
        wave_sync_lds();
        if (k > 0) {
            float aR, aT;
            axial_from_ring(ring, kax, ra, y0 - kWave, lane, aR, aT);
            const int yp = y0 - kWave + lane;   // < H
            fR[yp] = aR;
            fT[yp] = aT;
            fE[yp] = E_prev;
        }
        E_prev = E;
        if (DBG && act) {
            const int64_t kk = e.out_off + (int64_t)y * e.W + x;
            if (a.dbg.label) a.dbg.label[kk] = (uint8_t)lab;
            if (a.dbg.voxel) a.dbg.voxel[kk] = vox;
            if (a.dbg.energy) a.dbg.energy[kk] = E;
            if (a.dbg.scatter) a.dbg.scatter[kk] = T;
            if (a.dbg.philox) {
                uint4 pw;
                pw.x = inside ? w[0] : 0u;
                pw.y = inside ? w[1] : 0u;
                pw.z = inside ? w[2] : 0u;
                pw.w = inside ? w[3] : 0u;
                reinterpret_cast<uint4*>(a.dbg.philox)[kk] = pw;
            }
        }
        lab_last_prev = __builtin_amdgcn_readlane(lab, kWave - 1);
        vox = vox_n;
        lab = lab_n;
        Z = Zct_n;
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c] = qn[c];
        wave_sync_lds();
    }
    // flush: rows below the image read as zeros
    const int y_last = (n_chunks - 1) * kWave;
    ring_put(ring, ((y_last + kWave) & (kRing - 1)) + lane, make_float2(0.f, 0.f));
    wave_sync_lds();
    float aR, aT;
    axial_from_ring(ring, kax, ra, y_last, lane, aR, aT);
    if (y_last + lane < H) {
        fR[y_last + lane] = aR;
        fT[y_last + lane] = aT;
        fE[y_last + lane] = E_prev;
    }
    wave_sync_lds();
}

// Work items of the ray kernel: block b takes item b first (no atomic: the
// blocks of a launch would otherwise all meet on the counter at once), then
// items gridDim.x + the counter's successive values.
__device__ __forceinline__ int next_item(int32_t* counter, int* s_item)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_item = (int)gridDim.x + atomicAdd(counter, 1);
    __syncthreads();
    return *s_item;
}

// Plane of a batched step's env from its current pose: lane c < 3 computes
// volume axis c with the host's arithmetic and the wave combines the three
// (the pose is rejected unless all are in range).  With store, the env's plane
// and flag are written back for the step's later consumers.
__device__ __forceinline__ void item_geometry(const PhysArgs& a, EnvDev& e, int env, bool store, int lane)
{
    int c = lane < 3 ? lane : 0;
    // opaque per item: the lane addresses below are recomputed here instead of
    // hoisted out of the item loop and held (spilled) across the scanlines
    asm volatile("" : "+v"(c));
    // per-lane voxel size read from the descriptor in global memory (a pick
    // from the wave's private copy would be indexed scratch)
    const VolDev* vg = a.vols + e.vol;
    const double s = c == 0 ? vg->sx : (c == 1 ? vg->sy : vg->sz);
    int32_t p0 = 0, ddx = 0, ddy = 0;
    const int ok_c = plane_axis(a.poses + 12 * e.pose_env, c, s, e.W, e.H, e.dx64, e.dy64, e.elev64, p0, ddx, ddy);
    const bool ok = (__ballot(ok_c != 0) & 7ull) == 7ull;
    if (!ok) p0 = ddx = ddy = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e.P0[k] = __builtin_amdgcn_readlane(p0, k);
        e.DX[k] = __builtin_amdgcn_readlane(ddx, k);
        e.DY[k] = __builtin_amdgcn_readlane(ddy, k);
    }
    e.valid = ok ? 1 : 0;
    // Other groups of the same env may load the record while it is written
    // back here; they replace its plane fields before any use (a batched
    // step never reads them from memory), so the overlap is benign.
    if (store && lane < 3) {
        EnvDev& d = a.geo_out[env];
        d.P0[lane] = p0;
        d.DX[lane] = ddx;
        d.DY[lane] = ddy;
        if (lane == 0) d.valid = e.valid;   // sg_batch_status counts the rejected poses from these flags
    }
}

// Ray kernel: items (env, group of kWaves * spw scanlines), longest first.
// Five waves per SIMD (at most 102 registers, a few spilled) hide more of the
// gather latency than four; the label-pair instantiation without debug planes
// or noise scales fits six (80 registers), the others spill too much at six.
// With a.poses (batched steps) every item computes its env's plane itself.
template <bool MS, bool LAB, bool DBG>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LAB && !DBG && !MS ? 6 : 5))) void k_ray(
    PhysArgs a, QueueDev* q)
{
    __shared__ TissueDev s_tab[SG_MAX_LABELS_DEV];
    __shared__ float2 s_pair[kPairLabels * kPairLabels];
    __shared__ __attribute__((aligned(16))) float s_kax[kTaps + 7];   // zeros past 2 rax (read ahead by a group)
    __shared__ float2 s_ring[kWaves][kRingAlloc];
    __shared__ int s_item;
    __shared__ int32_t s_geo[10];   // an item's plane (P0, DX, DY, valid), computed by wave 0
    for (int i = threadIdx.x; i < a.n_labels; i += kThreads) s_tab[i] = a.table[i];
    if (a.pair_rt)
        for (int i = threadIdx.x; i < a.n_labels * a.n_labels; i += kThreads) s_pair[i] = a.pair_rt[i];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform: scalar per-scanline values
    for (int item = (int)blockIdx.x;; item = next_item(&q->next_ray, &s_item)) {
        if (item >= a.n_ray) break;
        const ItemRay it = a.ray_items[item];
        EnvDev e = a.envs[it.env];
        const VolDev v = a.vols[e.vol];
        // batched step: wave 0 computes the plane and hands it over through LDS
        // (the other waves last read s_geo before next_item's barriers)
        if (a.poses && wave == 0) {
            item_geometry(a, e, it.env, it.x0 == 0, lane);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    s_geo[k] = e.P0[k];
                    s_geo[3 + k] = e.DX[k];
                    s_geo[6 + k] = e.DY[k];
                }
                s_geo[9] = e.valid;
            }
        }
        for (int i = threadIdx.x; i < kTaps + 7; i += kThreads) s_kax[i] = i <= 2 * e.rax ? a.coefs[e.kax + i] : 0.f;
        __syncthreads();
        if (a.poses && wave != 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                e.P0[k] = __builtin_amdgcn_readfirstlane(s_geo[k]);
                e.DX[k] = __builtin_amdgcn_readfirstlane(s_geo[3 + k]);
                e.DY[k] = __builtin_amdgcn_readfirstlane(s_geo[6 + k]);
            }
            e.valid = __builtin_amdgcn_readfirstlane(s_geo[9]);
        }
        for (int s = 0; s < a.scanlines_per_wave; ++s) {
            const int x = it.x0 + s * kWaves + wave;
            if (x < e.W)
                ray_scanline<MS, LAB, DBG>(a, e, v, s_tab, a.pair_rt ? s_pair : nullptr, s_kax, s_ring[wave], x, lane);
        }
    }
}

// PSF kernel: items (env, tile of TX scanlines x 64 rows).
// Lateral radii up to kRB take the register-window path: the kernel is
// zero-padded to 2 kRB + 1 taps and a lane keeps the kSx + 2 kRB values of its
// row that an 8-column output strip needs, so each LDS value is read once per
// strip instead of once per tap.  Larger radii use a per-pixel tap loop.
constexpr int kRB = 8;
constexpr int kSx = 8;

template <int TX>
__global__ __launch_bounds__(TX / kSx * kWave) void k_psf(PhysArgs a)
{
    static_assert(TX % kSx == 0, "strips");
    constexpr int kPW = TX / kSx;        // waves: one 8-column output strip each
    constexpr int kPT = kPW * kWave;     // threads
    extern __shared__ float lds[];
    __shared__ float s_klat[kTaps];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);   // wave-uniform: scalar column bases
    // tiles are uniform in cost: block b takes tiles b, b + G, b + 2G, ... (G: the
    // grid).  A shared work counter costs more here than it balances: its
    // same-address atomics serialise across the XCDs.
    // LDS: the staged tile, then the output tile in a region of its own, so a
    // tile needs two barriers (staged -> filter, output written -> stores): the
    // next tile's staging and taps follow the second one, which every wave
    // passes only after filtering.
    if (a.ray_queue && blockIdx.x == 0 && tid == 0) a.ray_queue->next_ray = 0;   // for the next step's ray kernel
    const int r_max = a.max_rlat < kRB ? kRB : a.max_rlat;
    float* sY = lds + kAS * (2 * (TX + 2 * r_max) + TX);   // [kTileRows][TX + 1]
    for (int item = blockIdx.x; item < a.n_psf; item += gridDim.x) {
        const ItemPsf it = a.psf_items[item];
        const EnvDev e = a.envs[it.env];
        const int W = e.W, H = e.H, rl = e.rlat, ld = e.ld;
        const int R = rl <= kRB ? kRB : rl;   // halo of the staged tile
        const int x0 = (it.tile & 0xFFFF) * TX;
        const int y0 = (it.tile >> 16) * kTileRows;
        const int CW = TX + 2 * R;
        float* sR = lds;
        float* sT = sR + CW * kAS;
        float* sE = sT + CW * kAS;
        // taps centred in a window of 2 R + 1 (zero outside the env's 2 rl + 1)
        for (int i = tid; i <= 2 * R; i += kPT) {
            const int k = i - (R - rl);
            s_klat[i] = (k >= 0 && k <= 2 * rl) ? a.coefs[e.klat + k] : 0.f;
        }
        const float* gR = a.fR + e.scr_off;
        const float* gT = a.fT + e.scr_off;
        const float* gE = a.fE + e.scr_off;
        const int gy = y0 + lane;
        const bool yin = gy < H;
        if (R == kRB) {
            // every column load of the tile in flight before the LDS stores
            constexpr int CWF = TX + 2 * kRB;
            constexpr int NCR = (CWF + kPW - 1) / kPW, NCE = (TX + kPW - 1) / kPW;
            float vr[NCR], vt[NCR], ve[NCE];
#pragma unroll
            for (int u = 0; u < NCR; ++u) {
                const int c = wave + u * kPW;            // wave-uniform column
                const int gx = x0 - kRB + c;
                const bool col = c < CWF && gx >= 0 && gx < W;
                const int64_t base = (int64_t)(col ? gx : 0) * ld;
                vr[u] = (col && yin) ? gR[base + gy] : 0.f;
                vt[u] = (col && yin) ? gT[base + gy] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < NCE; ++u) {
                const int c = wave + u * kPW;
                const int gx = x0 + c;
                const bool col = c < TX && gx < W;
                const int64_t base = (int64_t)(col ? gx : 0) * ld;
                ve[u] = (col && yin) ? gE[base + gy] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < NCR; ++u) {
                const int c = wave + u * kPW;
                if (c < CWF) {
                    sR[c * kAS + lane] = vr[u];
                    sT[c * kAS + lane] = vt[u];
                }
            }
#pragma unroll
            for (int u = 0; u < NCE; ++u) {
                const int c = wave + u * kPW;
                if (c < TX) sE[c * kAS + lane] = ve[u];
            }
        } else {
        constexpr int kU = 4;   // columns in flight per wave
        for (int c0 = wave; c0 < CW; c0 += kPW * kU) {
            float vr[kU], vt[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int c = c0 + u * kPW;
                const int gx = x0 - R + c;
                const bool in = yin && c < CW && gx >= 0 && gx < W;
                const int64_t off = in ? (int64_t)gx * ld + gy : 0;
                vr[u] = in ? gR[off] : 0.f;
                vt[u] = in ? gT[off] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int c = c0 + u * kPW;
                if (c < CW) {
                    sR[c * kAS + lane] = vr[u];
                    sT[c * kAS + lane] = vt[u];
                }
            }
        }
        for (int c0 = wave; c0 < TX; c0 += kPW * kU) {
            float ve[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int gx = x0 + c0 + u * kPW;
                const bool in = yin && c0 + u * kPW < TX && gx < W;
                ve[u] = in ? gE[(int64_t)gx * ld + gy] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (c0 + u * kPW < TX) sE[(c0 + u * kPW) * kAS + lane] = ve[u];
        }
        }
        __syncthreads();
        // lane = tile row; Y of each strip goes to registers, then through LDS to row-major stores
        constexpr int kStrips = TX / kSx;
        constexpr int kSPW = (kStrips + kPW - 1) / kPW;   // strips per wave
        float yv[kSPW][kSx];
        const int r = lane, y = y0 + r;
        if (R == kRB) {
            float kp[2 * kRB + 1];
#pragma unroll
            for (int i = 0; i <= 2 * kRB; ++i) kp[i] = s_klat[i];
#pragma unroll
            for (int q = 0; q < kSPW; ++q) {
                const int sx = wave + q * kPW;
                if (sx >= kStrips) break;
                const int cx0 = sx * kSx;
                float wr[kSx + 2 * kRB], wt[kSx + 2 * kRB];
#pragma unroll
                for (int j = 0; j < kSx + 2 * kRB; ++j) {
                    wr[j] = sR[(cx0 + j) * kAS + r];
                    wt[j] = sT[(cx0 + j) * kAS + r];
                }
#pragma unroll
                for (int o = 0; o < kSx; ++o) {
                    float s1 = 0.f, s2 = 0.f;
#pragma unroll
                    for (int i = 0; i <= 2 * kRB; ++i) {
                        s1 = fmaf(kp[i], wr[o + i], s1);
                        s2 = fmaf(kp[i], wt[o + i], s2);
                    }
                    yv[q][o] = s1 + sE[(cx0 + o) * kAS + r] * s2;   // I
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < kSPW; ++q) {
                const int sx = wave + q * kPW;
                if (sx >= kStrips) break;
                for (int o = 0; o < kSx; ++o) {
                    const int cx = sx * kSx + o;
                    float s1 = 0.f, s2 = 0.f;
                    for (int i = 0; i <= 2 * R; ++i) {
                        s1 = fmaf(s_klat[i], sR[(cx + i) * kAS + r], s1);
                        s2 = fmaf(s_klat[i], sT[(cx + i) * kAS + r], s2);
                    }
                    yv[q][o] = s1 + sE[cx * kAS + r] * s2;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kSPW; ++q) {
            const int sx = wave + q * kPW;
            if (sx >= kStrips) break;
#pragma unroll
            for (int o = 0; o < kSx; ++o) {
                const int x = x0 + sx * kSx + o;
                const float I = yv[q][o];
                float Y = 0.f;
                if (I > 0.f) {
                    // (20 / DR) log10(I / E0) as disp2 * log2(I * (1 / E0))
                    Y = 1.f + e.disp2 * __builtin_amdgcn_logf(I * e.inv_E0);
                    Y = fminf(fmaxf(Y, 0.f), 1.f);
                }
                sY[r * (TX + 1) + sx * kSx + o] = Y;
                if (a.dbg.intensity && y < H && x < W) a.dbg.intensity[e.out_off + (int64_t)y * W + x] = I;
            }
        }
        __syncthreads();
        // whole rows per wave from a scalar row base: row rr = wave + k kPW, lane = column
        for (int rr = wave; rr < kTileRows; rr += kPW) {
            const int yy = y0 + rr;
            if (yy >= H) break;
            float* orow = a.out + e.out_off + (int64_t)yy * W + x0;
            for (int cx = lane; cx < TX; cx += kWave)
                if (x0 + cx < W) orow[cx] = sY[rr * (TX + 1) + cx];
        }
    }
}

// Surrogate input of each pixel: one-hot label (channels 0..3), the
// scatterer sample of the same fixed noise field the ray pass uses (channel 4:
// N0 where the density gate passes, else 0) and the normalised depth
// (y + 0.5) / H (channel 5); bf16, 8 channels per pixel, frames packed
// [env][y][x][8] at 8 * out_off.
__device__ __forceinline__ uint16_t f2bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <bool MS>
__global__ __launch_bounds__(kThreads) void k_encode(PhysArgs a, uint16_t* enc)
{
    const int env = blockIdx.y;
    const EnvDev e = a.envs[env];
    const VolDev v = a.vols[e.vol];
    const int npx = e.W * e.H;
    for (int p = blockIdx.x * kThreads + threadIdx.x; p < npx; p += gridDim.x * kThreads) {
        const int y = p / e.W, x = p - y * e.W;
        int lab = 0;
        float sc = 0.f;
        if (e.valid) {
            uint32_t boff;
            const int32_t vox = voxel_at(e, v, x, y, boff);
            lab = label_of(v, vox, boff);
            if (vox >= 0) {
                uint32_t w[4];
                philox4x32_10((uint32_t)vox, v.key0, v.key1, w);
                const TissueDev tt = a.table[lab];
                if (!MS || v.scales <= 1) {
                    if ((unsigned long long)w[2] < tt.thr) sc = box_muller(w[0], w[1]);
                } else {
                    const int32_t ix = vox % v.nx, iy = (vox / v.nx) % v.ny, iz = vox / (v.nx * v.ny);
                    float n0;
                    bool gate;
                    scatter_multiscale(v, a.q_lut, a.ms_thr[lab * kMaxNoiseScales + v.scales - 1], ix, iy, iz, w,
                                       n0, gate);
                    if (gate) sc = n0;
                }
            }
        }
        uint4 o;
        const uint32_t one = 0x3F80u;   // bf16 1.0
        o.x = (lab == 0 ? one : 0u) | ((lab == 1 ? one : 0u) << 16);
        o.y = (lab == 2 ? one : 0u) | ((lab == 3 ? one : 0u) << 16);
        o.z = (uint32_t)f2bf16(sc) | ((uint32_t)f2bf16(((float)y + 0.5f) / (float)e.H) << 16);
        o.w = 0u;
        reinterpret_cast<uint4*>(enc)[e.out_off + p] = o;
    }
}

// CT-conditioned surrogate input.  Histogram bin of a pixel: its nearest
// voxel's HU (-1000 outside the volume) + 1024, clamped to [0, 4095].
__device__ __forceinline__ int ct_bin(const EnvDev& e, const VolDev& v, int x, int y, int32_t& vox)
{
    uint32_t boff;
    vox = voxel_at(e, v, x, y, boff);
    const int hu = (vox >= 0 && v.ct) ? (int)ld_global(v.ct, vox) : -1000;
    return min(max(hu + 1024, 0), kCtBins - 1);
}

// per-frame histograms of the bins: hist [n_envs][kCtBins], zeroed by the caller
__global__ __launch_bounds__(kThreads) void k_ct_hist(PhysArgs a, uint32_t* hist)
{
    __shared__ uint32_t h[kCtBins];
    const int env = blockIdx.y;
    const EnvDev e = a.envs[env];
    const VolDev v = a.vols[e.vol];
    for (int i = threadIdx.x; i < kCtBins; i += kThreads) h[i] = 0u;
    __syncthreads();
    const int npx = e.W * e.H;
    for (int p = blockIdx.x * kThreads + threadIdx.x; p < npx; p += gridDim.x * kThreads) {
        const int y = p / e.W, x = p - y * e.W;
        int32_t vox;
        const int b = e.valid ? ct_bin(e, v, x, y, vox) : 1024 - 1000;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kCtBins; i += kThreads)
        if (h[i]) atomicAdd(&hist[(int64_t)env * kCtBins + i], h[i]);
}

// histogram specification per frame: lut[b] = smallest r with
// refC[r] * n_src >= srcC[b] * n_ref (inclusive cumulative counts, int64)
__global__ __launch_bounds__(kThreads) void k_ct_lut(const uint32_t* hist, const long long* ref_cum, long long n_ref,
                                                     uint16_t* lut)
{
    constexpr int kPer = kCtBins / kThreads;   // 16 bins per thread
    __shared__ long long part[kThreads];
    const int env = blockIdx.x;
    const uint32_t* h = hist + (int64_t)env * kCtBins;
    long long c[kPer];
    long long run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        run += h[threadIdx.x * kPer + i];
        c[i] = run;
    }
    part[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {   // inclusive scan of the thread totals
        const long long t = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    const long long before = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    const long long n_src = part[kThreads - 1];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const long long goal = (before + c[i]) * n_ref;
        int lo = 0, hi = kCtBins - 1;   // smallest r with ref_cum[r] * n_src >= goal (ref_cum[4095] = n_ref)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ref_cum[mid] * n_src >= goal)
                hi = mid;
            else
                lo = mid + 1;
        }
        lut[(int64_t)env * kCtBins + threadIdx.x * kPer + i] = (uint16_t)lo;
    }
}

// pooled reference of the histogram matching: ref_hist[b] = sum over the n
// frames' histograms, ref_cum its inclusive cumulative counts (one block)
__global__ __launch_bounds__(kThreads) void k_ct_ref(const uint32_t* hist, int n, long long* ref_hist,
                                                     long long* ref_cum)
{
    constexpr int kPer = kCtBins / kThreads;
    __shared__ long long part[kThreads];
    long long c[kPer];
    long long run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int b = threadIdx.x * kPer + i;
        long long t = 0;
        for (int f = 0; f < n; ++f) t += hist[(int64_t)f * kCtBins + b];
        ref_hist[b] = t;
        run += t;
        c[i] = run;
    }
    part[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        const long long t = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    const long long before = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) ref_cum[threadIdx.x * kPer + i] = before + c[i];
}

// 8 bf16 channels per pixel: matched CT / 1000, N0 and N1 (quantised) of the
// voxel's noise draw (0 outside), depth (y + 0.5) / H, zeros
__global__ __launch_bounds__(kThreads) void k_encode_ct(PhysArgs a, const uint16_t* lut, uint16_t* enc)
{
    const int env = blockIdx.y;
    const EnvDev e = a.envs[env];
    const VolDev v = a.vols[e.vol];
    const int npx = e.W * e.H;
    for (int p = blockIdx.x * kThreads + threadIdx.x; p < npx; p += gridDim.x * kThreads) {
        const int y = p / e.W, x = p - y * e.W;
        int32_t vox = -1;
        const int b = e.valid ? ct_bin(e, v, x, y, vox) : 1024 - 1000;
        const int r = (int)lut[(int64_t)env * kCtBins + b];
        const float ct = (float)(r - 1024) / 1000.f;
        float n0 = 0.f, n1 = 0.f;
        if (vox >= 0) {
            uint32_t w[4];
            philox4x32_10((uint32_t)vox, v.key0, v.key1, w);
            n0 = box_muller(w[0], w[1]);
            n1 = (float)a.q_lut[w[2] >> 20] * 0x1p-20f;   // exact: |Q| < 2^24
        }
        uint4 o;
        o.x = (uint32_t)f2bf16(ct) | ((uint32_t)f2bf16(n0) << 16);
        o.y = (uint32_t)f2bf16(n1) | ((uint32_t)f2bf16(((float)y + 0.5f) / (float)e.H) << 16);
        o.z = 0u;
        o.w = 0u;
        reinterpret_cast<uint4*>(enc)[e.out_off + p] = o;
    }
}

__global__ void k_queue_reset(QueueDev* q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x].next_ray = 0;
}

// linear [nz][ny][nx] label map -> bricked layout, one thread per destination byte (padding voxels 0)
__global__ __launch_bounds__(kThreads) void k_brick_labels(const uint8_t* __restrict__ src, int32_t nx, int32_t ny,
                                                           int32_t nz, int32_t bnx, int32_t bny, int64_t n_bytes,
                                                           uint8_t* __restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n_bytes; i += (int64_t)gridDim.x * kThreads) {
        const int64_t b = i >> 7;
        const int w = (int)(i & (kBrickBytes - 1));
        const int64_t byz = b / bnx;
        const int32_t ix = (int32_t)(b - byz * bnx) * kBrickX + (w & 7);
        const int32_t iy = (int32_t)(byz % bny) * kBrickY + ((w >> 3) & 3);
        const int32_t iz = (int32_t)(byz / bny) * kBrickZ + (w >> 5);
        const bool in = ix < nx && iy < ny && iz < nz;
        dst[i] = in ? src[((int64_t)iz * ny + iy) * nx + ix] : (uint8_t)0;
    }
}

__global__ void k_max_label(const uint8_t* labels, int64_t n, int32_t* out)
{
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (int)labels[i]);
    for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_down(m, d));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

const void* psf_fn(int tx)
{
    if (tx == 16) return reinterpret_cast<const void*>(&k_psf<16>);
    if (tx == 32) return reinterpret_cast<const void*>(&k_psf<32>);
    if (tx == 64) return reinterpret_cast<const void*>(&k_psf<64>);
    return nullptr;
}

int blocks_per_cu(const void* fn, int threads, size_t lds)
{
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds) != hipSuccess) return 0;
    return n;
}

// PSF block size: one wave per 8-column strip of the tile
constexpr int psf_threads(int tx) { return tx / kSx * kWave; }

}  // namespace

size_t psf_lds_bytes(int tx, int max_rlat)
{
    const int R = max_rlat < kRB ? kRB : max_rlat;
    // staged tile (R, T with halo, E), then the output tile
    return sizeof(float) * ((size_t)kAS * (2 * (tx + 2 * R) + tx) + (size_t)kTileRows * (tx + 1));
}

bool psf_tile_supported(int tx) { return psf_fn(tx) != nullptr; }

// the instantiation of the ray kernel for a launch
template <bool MS>
const void* ray_fn(bool label_only, bool debug)
{
    if (label_only) return debug ? reinterpret_cast<const void*>(&k_ray<MS, true, true>)
                                 : reinterpret_cast<const void*>(&k_ray<MS, true, false>);
    return debug ? reinterpret_cast<const void*>(&k_ray<MS, false, true>)
                 : reinterpret_cast<const void*>(&k_ray<MS, false, false>);
}

int ray_grid(int n_cu, bool multiscale, bool label_only, bool debug)
{
    const void* fn = multiscale ? ray_fn<true>(label_only, debug) : ray_fn<false>(label_only, debug);
    return blocks_per_cu(fn, kThreads, 0) * n_cu;
}

int psf_grid(int tx, int max_rlat, int n_cu)
{
    return blocks_per_cu(psf_fn(tx), psf_threads(tx), psf_lds_bytes(tx, max_rlat)) * n_cu;
}

hipError_t launch_ray(const PhysArgs& a, QueueDev* q, int grid, hipStream_t s)
{
    if (a.n_ray <= 0) return hipSuccess;
    if (grid > a.n_ray) grid = a.n_ray;
    if (grid < 1) return hipErrorInvalidConfiguration;
    const void* fn = a.multiscale ? ray_fn<true>(ray_label_only(a), ray_debug(a)) : ray_fn<false>(ray_label_only(a), ray_debug(a));
    void* args[] = {const_cast<PhysArgs*>(&a), &q};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_psf(const PhysArgs& a, int tx, int grid, hipStream_t s)
{
    if (a.n_psf <= 0) return hipSuccess;
    if (grid > a.n_psf) grid = a.n_psf;
    if (grid < 1) return hipErrorInvalidConfiguration;
    const size_t lds = psf_lds_bytes(tx, a.max_rlat);
    if (tx == 16)
        hipLaunchKernelGGL(k_psf<16>, dim3(grid), dim3(psf_threads(16)), lds, s, a);
    else if (tx == 32)
        hipLaunchKernelGGL(k_psf<32>, dim3(grid), dim3(psf_threads(32)), lds, s, a);
    else if (tx == 64)
        hipLaunchKernelGGL(k_psf<64>, dim3(grid), dim3(psf_threads(64)), lds, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ct_encode(const PhysArgs& a, int32_t n_envs, int32_t max_pixels, uint32_t* hist,
                            const long long* ref_cum, long long n_ref, uint16_t* lut, uint16_t* enc, hipStream_t s)
{
    if (n_envs <= 0) return hipSuccess;
    int bx = (max_pixels + kThreads - 1) / kThreads;
    if (bx > 64) bx = 64;
    hipError_t e = hipMemsetAsync(hist, 0, sizeof(uint32_t) * kCtBins * (size_t)n_envs, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ct_hist, dim3(bx, n_envs), dim3(kThreads), 0, s, a, hist);
    if ((e = hipGetLastError()) != hipSuccess || !enc) return e;
    hipLaunchKernelGGL(k_ct_lut, dim3(n_envs), dim3(kThreads), 0, s, hist, ref_cum, n_ref, lut);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_encode_ct, dim3(bx, n_envs), dim3(kThreads), 0, s, a, lut, enc);
    return hipGetLastError();
}

hipError_t launch_ct_reference(const uint32_t* hist, int32_t n_envs, long long* ref_hist, long long* ref_cum,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_ct_ref, dim3(1), dim3(kThreads), 0, s, hist, n_envs, ref_hist, ref_cum);
    return hipGetLastError();
}

hipError_t launch_encode(const PhysArgs& a, int32_t n_envs, int32_t max_pixels, uint16_t* enc, hipStream_t s)
{
    if (n_envs <= 0) return hipSuccess;
    int bx = (max_pixels + kThreads - 1) / kThreads;
    if (bx > 64) bx = 64;
    if (a.multiscale)
        hipLaunchKernelGGL(k_encode<true>, dim3(bx, n_envs), dim3(kThreads), 0, s, a, enc);
    else
        hipLaunchKernelGGL(k_encode<false>, dim3(bx, n_envs), dim3(kThreads), 0, s, a, enc);
    return hipGetLastError();
}

hipError_t launch_queue_reset(QueueDev* q, int n, hipStream_t s)
{
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, q, n);
    return hipGetLastError();
}

hipError_t launch_brick_labels(const uint8_t* src, int32_t nx, int32_t ny, int32_t nz, uint8_t* dst, hipStream_t s)
{
    const int32_t bnx = (nx + kBrickX - 1) / kBrickX, bny = (ny + kBrickY - 1) / kBrickY,
                  bnz = (nz + kBrickZ - 1) / kBrickZ;
    const int64_t n_bytes = (int64_t)bnx * bny * bnz * kBrickBytes;
    const int64_t blocks = std::min<int64_t>((n_bytes + kThreads - 1) / kThreads, 65536);
    hipLaunchKernelGGL(k_brick_labels, dim3((unsigned)blocks), dim3(kThreads), 0, s, src, nx, ny, nz, bnx, bny, n_bytes,
                       dst);
    return hipGetLastError();
}

hipError_t launch_max_label(const uint8_t* labels, int64_t n, int32_t* d_out, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_max_label, dim3((unsigned)blocks), dim3(256), 0, s, labels, n, d_out);
    return hipGetLastError();
}

}  // namespace sg
