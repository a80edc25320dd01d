// Model-based B-mode simulation kernels for gfx950 (SonoGym, App. B.2).
//
// Two passes per frame:
//  * ray pass   -- one wave64 per scanline, lanes along depth.  Each 64-row
//                  chunk samples the plane (nearest label, optional trilinear
//                  CT), forms the boundary/reflection/transmission terms,
//                  runs wave-level scans for the transmission product and the
//                  attenuation integral (remaining energy E), draws the
//                  per-voxel scatterer (Philox4x32-10 keyed by voxel index,
//                  Box-Muller, density gate) and writes the reflection source
//                  R' = G*E*cos(theta)*|r|, the scattering pattern T and E to
//                  a scanline-major scratch (coalesced along the scanline).
//  * PSF pass   -- one workgroup per output tile: stages R' and T with the PSF
//                  halo through LDS, applies the separable Gaussian PSF
//                  (axial, then lateral), composes I = K(x)R' + E*K(x)T,
//                  log-compresses and stores the frame row-major (coalesced
//                  along image rows).
// A persistent kernel runs both passes from one device work queue for the
// batched path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kThreads = 256;

// Philox4x32-10 (Salmon et al., SC'11): multipliers and Weyl key increments.
constexpr uint32_t kPhM0 = 0xD2511F53u;
constexpr uint32_t kPhM1 = 0xCD9E8D57u;
constexpr uint32_t kPhW0 = 0x9E3779B9u;
constexpr uint32_t kPhW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t n_lo, uint32_t k0, uint32_t k1, uint32_t w[4])
{
    uint32_t c0 = n_lo, c1 = 0u, c2 = 0u, c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(kPhM0, c0);
        const uint32_t lo0 = kPhM0 * c0;
        const uint32_t hi1 = __umulhi(kPhM1, c2);
        const uint32_t lo1 = kPhM1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
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

// nearest voxel of pixel (x, y), -1 outside the grid
__device__ __forceinline__ int32_t voxel_at(const EnvDev& e, const VolDev& v, int x, int y)
{
    // round half up: floor((q + 2^15) / 2^16) as an arithmetic shift
    const int32_t ix = (int32_t)((uint32_t)q16(e.P0[0], e.DX[0], e.DY[0], x, y) + 32768u) >> 16;
    const int32_t iy = (int32_t)((uint32_t)q16(e.P0[1], e.DX[1], e.DY[1], x, y) + 32768u) >> 16;
    const int32_t iz = (int32_t)((uint32_t)q16(e.P0[2], e.DX[2], e.DY[2], x, y) + 32768u) >> 16;
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    return in ? (iz * v.ny + iy) * v.nx + ix : -1;
}

__device__ __forceinline__ int label_of(const VolDev& v, int32_t vox)
{
    return vox >= 0 ? (int)v.labels[vox] : 0;
}

__device__ __forceinline__ double ct_corner(const VolDev& v, int32_t ix, int32_t iy, int32_t iz)
{
    const bool in = (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny &&
                    (uint32_t)iz < (uint32_t)v.nz;
    return in ? (double)v.ct[(iz * v.ny + iy) * v.nx + ix] : -1000.0;
}

// impedance from CT: max(HU + 1000, 0), HU trilinear in FP64 (successive
// linear interpolation along x, y, z; outside corners -1000 HU)
__device__ double z_from_ct(const EnvDev& e, const VolDev& v, int x, int y)
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

// cos(theta): Sobel (1,2,1) on [label differs from the centre label] with
// clamped image coordinates, in physical units (only evaluated at G = 1)
__device__ float incidence_cos(const EnvDev& e, const VolDev& v, int x, int y, int lab)
{
    int b[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int xx = min(max(x + i - 1, 0), e.W - 1);
            const int yy = min(max(y + j - 1, 0), e.H - 1);
            b[j][i] = label_of(v, voxel_at(e, v, xx, yy)) != lab;
        }
    }
    float gx = (float)((b[0][2] - b[0][0]) + 2 * (b[1][2] - b[1][0]) + (b[2][2] - b[2][0]));
    float gy = (float)((b[2][0] - b[0][0]) + 2 * (b[2][1] - b[0][1]) + (b[2][2] - b[0][2]));
    gx = gx / e.dx;
    gy = gy / e.dy;
    const float h = sqrtf(gx * gx + gy * gy);
    return h == 0.f ? 1.f : fabsf(gy) / h;
}

__device__ __forceinline__ float uniform24(uint32_t w)
{
    // (2*(w >> 9) + 1) * 2^-24: odd 24-bit numerator, exact in FP32
    return (float)((w >> 9) * 2u + 1u) * 0x1p-24f;
}

// One scanline of the ray pass, executed by one wave (lane = depth row).
__device__ void ray_scanline(const PhysArgs& a, const EnvDev& e, const VolDev& v,
                             const TissueDev* tab, int x, int lane)
{
    const int W = e.W, H = e.H;
    (void)W;
    float* fR = a.fR + e.scr_off + (int64_t)x * H;
    float* fT = a.fT + e.scr_off + (int64_t)x * H;
    float* fE = a.fE + e.scr_off + (int64_t)x * H;
    if (!e.valid) {
        for (int y = lane; y < H; y += kWave) {
            fR[y] = 0.f;
            fT[y] = 0.f;
            fE[y] = 0.f;
        }
        return;
    }
    const bool ct = v.ct != nullptr;
    float carry_t = 1.f;     // transmission product of the rows above the chunk
    double carry_a = 0.0;    // attenuation integral (sum of alpha) above the chunk
    for (int y0 = 0; y0 < H; y0 += kWave) {
        const int y = y0 + lane;
        const bool act = y < H;
        const int32_t vox = voxel_at(e, v, x, y);
        const int lab = label_of(v, vox);
        double Z = ct ? z_from_ct(e, v, x, y) : (double)tab[lab].Z;
        // the next row's label and impedance: neighbour lane, or row y0+64
        int lab_n = __shfl_down(lab, 1);
        double Z_n = __shfl_down(Z, 1);
        if (lane == kWave - 1) {
            lab_n = label_of(v, voxel_at(e, v, x, y + 1));
            Z_n = ct ? z_from_ct(e, v, x, y + 1) : (double)tab[lab_n].Z;
        }
        const bool G = act && (y < H - 1) && (lab != lab_n);
        float r = 0.f, t = 1.f;
        if (G && Z != Z_n) {
            if (Z == 0.0 || Z_n == 0.0 || __builtin_isinf(Z) || __builtin_isinf(Z_n)) {
                r = Z_n > Z ? 1.f : -1.f;
                t = 0.f;
            } else {
                const double s = Z + Z_n;
                r = (float)((Z_n - Z) / s);
                t = (float)((2.0 * Z / s) * (2.0 * Z_n / s));
            }
        }
        // inclusive wave scans: transmission product (FP32), alpha sum (FP64)
        float tp = act ? t : 1.f;
        double as = act ? (double)tab[lab].alpha : 0.0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const float o = __shfl_up(tp, d);
            const double oa = __shfl_up(as, d);
            if (lane >= d) {
                tp *= o;
                as += oa;
            }
        }
        float t_ex = __shfl_up(tp, 1);
        double a_ex = __shfl_up(as, 1);
        if (lane == 0) {
            t_ex = 1.f;
            a_ex = 0.0;
        }
        const float E = e.E0 * (carry_t * t_ex) * expf((float)(-e.coef * (carry_a + a_ex)));
        carry_t *= __shfl(tp, kWave - 1);
        carry_a += __shfl(as, kWave - 1);

        float cs = 1.f;
        if (G) cs = incidence_cos(e, v, x, y, lab);

        float T = 0.f;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (act && vox >= 0) {
            philox4x32_10((uint32_t)vox, v.key0, v.key1, w);
            const TissueDev tt = tab[lab];
            if ((unsigned long long)w[2] < tt.thr) {
                const float n0 = sqrtf(-2.f * logf(uniform24(w[0]))) * cospif(2.f * uniform24(w[1]));
                T = n0 * tt.sigma0 + tt.mu0;
            }
        }
        const float Rp = G ? E * cs * fabsf(r) : 0.f;
        if (act) {
            fR[y] = Rp;
            fT[y] = T;
            fE[y] = E;
            const int64_t k = e.out_off + (int64_t)y * e.W + x;
            if (a.dbg.label) a.dbg.label[k] = (uint8_t)lab;
            if (a.dbg.voxel) a.dbg.voxel[k] = vox;
            if (a.dbg.energy) a.dbg.energy[k] = E;
            if (a.dbg.philox) {
                uint4 pw;
                pw.x = w[0];
                pw.y = w[1];
                pw.z = w[2];
                pw.w = w[3];
                reinterpret_cast<uint4*>(a.dbg.philox)[k] = pw;
            }
        }
    }
}

// tissue table staged in LDS for the ray pass
__device__ void stage_table(const PhysArgs& a, TissueDev* s_tab)
{
    for (int i = threadIdx.x; i < a.n_labels; i += blockDim.x) s_tab[i] = a.table[i];
}

// one ray work item: kRayWaves waves x scanlines_per_wave scanlines from x0
__device__ int ray_item(const PhysArgs& a, const ItemRay it, const TissueDev* s_tab)
{
    const EnvDev e = a.envs[it.env];
    const VolDev v = a.vols[e.vol];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int spw = a.scanlines_per_wave;
    for (int s = 0; s < spw; ++s) {
        const int x = it.x0 + s * kRayWaves + wave;
        if (x < e.W) ray_scanline(a, e, v, s_tab, x, lane);
    }
    return min(e.W - it.x0, kRayWaves * spw);
}

// one PSF tile (TX scanlines x TY rows); lds sized by psf_lds_bytes
template <int TX, int TY>
__device__ void psf_tile(const PhysArgs& a, const ItemPsf it, float* lds)
{
    const EnvDev e = a.envs[it.env];
    const int W = e.W, H = e.H, ra = e.rax, rl = e.rlat;
    const int x0 = (it.tile & 0xFFFF) * TX;
    const int y0 = (it.tile >> 16) * TY;
    const int CW = TX + 2 * rl;          // staged scanlines (with lateral halo)
    const int CH = TY + 2 * ra;          // staged rows (with axial halo)
    const int AS = TY + 1;               // padded column stride of the axial result
    float* sR = lds;
    float* sT = sR + CW * CH;
    float* aR = sT + CW * CH;
    float* aT = aR + CW * AS;
    float* sE = aT + CW * AS;
    float* kax = sE + TX * AS;
    float* klat = kax + 2 * kMaxPsfRadius + 1;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    constexpr int kWaves = kThreads / kWave;

    for (int i = tid; i <= 2 * ra; i += kThreads) kax[i] = a.coefs[e.kax + i];
    for (int i = tid; i <= 2 * rl; i += kThreads) klat[i] = a.coefs[e.klat + i];
    const float* gR = a.fR + e.scr_off;
    const float* gT = a.fT + e.scr_off;
    const float* gE = a.fE + e.scr_off;
    for (int c = wave; c < CW; c += kWaves) {
        const int gx = x0 - rl + c;
        const bool xin = gx >= 0 && gx < W;
        for (int r = lane; r < CH; r += kWave) {
            const int gy = y0 - ra + r;
            const bool in = xin && gy >= 0 && gy < H;
            const int64_t off = (int64_t)gx * H + gy;
            sR[c * CH + r] = in ? gR[off] : 0.f;
            sT[c * CH + r] = in ? gT[off] : 0.f;
        }
    }
    for (int c = wave; c < TX; c += kWaves) {
        const int gx = x0 + c;
        for (int r = lane; r < TY; r += kWave) {
            const int gy = y0 + r;
            sE[c * AS + r] = (gx < W && gy < H) ? gE[(int64_t)gx * H + gy] : 0.f;
        }
    }
    __syncthreads();
    // axial pass over every staged scanline
    for (int c = wave; c < CW; c += kWaves) {
        for (int r = lane; r < TY; r += kWave) {
            const float* pr = sR + c * CH + r;
            const float* pt = sT + c * CH + r;
            float s1 = 0.f, s2 = 0.f;
            for (int j = 0; j <= 2 * ra; ++j) {
                s1 += kax[j] * pr[j];
                s2 += kax[j] * pt[j];
            }
            aR[c * AS + r] = s1;
            aT[c * AS + r] = s2;
        }
    }
    __syncthreads();
    // lateral pass, composition, log compression, row-major store
    for (int idx = tid; idx < TX * TY; idx += kThreads) {
        const int cx = idx % TX;
        const int r = idx / TX;
        const int x = x0 + cx, y = y0 + r;
        if (x < W && y < H) {
            float s1 = 0.f, s2 = 0.f;
            for (int i = 0; i <= 2 * rl; ++i) {
                s1 += klat[i] * aR[(cx + i) * AS + r];
                s2 += klat[i] * aT[(cx + i) * AS + r];
            }
            const float I = s1 + sE[cx * AS + r] * s2;
            float Y = 0.f;
            if (I > 0.f) {
                Y = 1.f + e.disp * log10f(I / e.E0);
                Y = fminf(fmaxf(Y, 0.f), 1.f);
            }
            const int64_t k = e.out_off + (int64_t)y * W + x;
            a.out[k] = Y;
            if (a.dbg.intensity) a.dbg.intensity[k] = I;
        }
    }
    __syncthreads();   // LDS is reused by the caller's next item
}

__global__ __launch_bounds__(kThreads) void k_ray(PhysArgs a)
{
    __shared__ TissueDev s_tab[SG_MAX_LABELS_DEV];
    stage_table(a, s_tab);
    __syncthreads();
    if ((int)blockIdx.x < a.n_ray) ray_item(a, a.ray_items[blockIdx.x], s_tab);
}

template <int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_psf(PhysArgs a)
{
    extern __shared__ float lds[];
    if ((int)blockIdx.x < a.n_psf) psf_tile<TX, TY>(a, a.psf_items[blockIdx.x], lds);
}

// Persistent batched kernel: ray items first, then PSF tiles.  A tile waits
// until every scanline of its environment is finished; ray items never wait
// and are all dequeued before any tile, so every wait ends.
constexpr long long kSpinLimit = 1ll << 24;

template <int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_persistent(PhysArgs a, QueueDev* q)
{
    extern __shared__ float lds[];
    __shared__ TissueDev s_tab[SG_MAX_LABELS_DEV];
    __shared__ int s_item;
    stage_table(a, s_tab);
    const int total = a.n_ray + a.n_psf;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(&q->next, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        if (item < a.n_ray) {
            const ItemRay it = a.ray_items[item];
            const int n = ray_item(a, it, s_tab);
            __threadfence();          // publish this wave's fields at device scope
            __syncthreads();
            if (threadIdx.x == 0) atomicAdd(&q->done[it.env], n);
        } else {
            const ItemPsf it = a.psf_items[item - a.n_ray];
            if (threadIdx.x == 0) {
                const int need = a.envs[it.env].W;
                long long spins = 0;
                while (__hip_atomic_load(&q->done[it.env], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) {
                        atomicAdd(&q->timeouts, 1);
                        break;
                    }
                }
            }
            __syncthreads();
            __threadfence();          // see other workgroups' fields
            psf_tile<TX, TY>(a, it, lds);
        }
    }
}

__global__ void k_geometry(EnvDev* envs, const VolDev* vols, const double* poses, int n, QueueDev* q)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    EnvDev& d = envs[e];
    const VolDev v = vols[d.vol];
    int32_t P0[3], DX[3], DY[3];
    const int ok = plane_geometry(poses + 12 * e, v.sx, v.sy, v.sz, d.W, d.H, d.dx64, d.dy64, P0, DX, DY);
    for (int c = 0; c < 3; ++c) {
        d.P0[c] = ok ? P0[c] : 0;
        d.DX[c] = ok ? DX[c] : 0;
        d.DY[c] = ok ? DY[c] : 0;
    }
    d.valid = ok;
    if (!ok) atomicAdd(&q->n_bad, 1);
}

__global__ void k_queue_reset(QueueDev* q, int n_envs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        q->next = 0;
        q->n_bad = 0;
        q->timeouts = 0;
        q->pad = 0;
    }
    if (i < n_envs) q->done[i] = 0;
}

__global__ void k_max_label(const uint8_t* labels, int64_t n, int32_t* out)
{
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (int)labels[i]);
    for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_down(m, d));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

template <int TX, int TY>
const void* persistent_fn()
{
    return reinterpret_cast<const void*>(&k_persistent<TX, TY>);
}

}  // namespace

size_t psf_lds_bytes(int tx, int ty, int max_rax, int max_rlat)
{
    const size_t CW = tx + 2 * max_rlat, CH = ty + 2 * max_rax, AS = ty + 1;
    return sizeof(float) * (2 * CW * CH + 2 * CW * AS + tx * AS + 2 * (2 * kMaxPsfRadius + 1));
}

#define SG_TILE_SWITCH(TX_, TY_, CALL)                                        \
    if (TX_ == 32 && TY_ == 32) { CALL(32, 32); }                             \
    else if (TX_ == 64 && TY_ == 16) { CALL(64, 16); }                        \
    else if (TX_ == 16 && TY_ == 64) { CALL(16, 64); }                        \
    else if (TX_ == 64 && TY_ == 32) { CALL(64, 32); }                        \
    else { return hipErrorInvalidValue; }

hipError_t launch_ray(const PhysArgs& a, hipStream_t s)
{
    if (a.n_ray <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ray, dim3(a.n_ray), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_psf(const PhysArgs& a, int tx, int ty, hipStream_t s)
{
    if (a.n_psf <= 0) return hipSuccess;
    const size_t lds = psf_lds_bytes(tx, ty, a.max_rax, a.max_rlat);
#define SG_LAUNCH_PSF(X, Y) hipLaunchKernelGGL((k_psf<X, Y>), dim3(a.n_psf), dim3(kThreads), lds, s, a)
    SG_TILE_SWITCH(tx, ty, SG_LAUNCH_PSF)
#undef SG_LAUNCH_PSF
    return hipGetLastError();
}

hipError_t launch_persistent(const PhysArgs& a, QueueDev* q, int tx, int ty, int grid, hipStream_t s)
{
    const size_t lds = psf_lds_bytes(tx, ty, a.max_rax, a.max_rlat);
#define SG_LAUNCH_PERS(X, Y) hipLaunchKernelGGL((k_persistent<X, Y>), dim3(grid), dim3(kThreads), lds, s, a, q)
    SG_TILE_SWITCH(tx, ty, SG_LAUNCH_PERS)
#undef SG_LAUNCH_PERS
    return hipGetLastError();
}

int persistent_blocks_per_cu(int tx, int ty, int max_rax, int max_rlat)
{
    const size_t lds = psf_lds_bytes(tx, ty, max_rax, max_rlat);
    int n = 0;
    const void* fn = nullptr;
#define SG_FN(X, Y) fn = persistent_fn<X, Y>()
    if (tx == 32 && ty == 32) SG_FN(32, 32);
    else if (tx == 64 && ty == 16) SG_FN(64, 16);
    else if (tx == 16 && ty == 64) SG_FN(16, 64);
    else if (tx == 64 && ty == 32) SG_FN(64, 32);
    else return 0;
#undef SG_FN
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kThreads, lds) != hipSuccess) return 0;
    return n;
}

hipError_t launch_geometry(EnvDev* envs, const VolDev* vols, const double* poses, int32_t n, QueueDev* q,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_geometry, dim3((n + 127) / 128), dim3(128), 0, s, envs, vols, poses, n, q);
    return hipGetLastError();
}

hipError_t launch_queue_reset(QueueDev* q, int32_t n_envs, hipStream_t s)
{
    const int n = n_envs > 1 ? n_envs : 1;
    hipLaunchKernelGGL(k_queue_reset, dim3((n + 255) / 256), dim3(256), 0, s, q, n_envs);
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
