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
//                  into a per-wave LDS ring of four chunks, and the axial
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

#include "sg_internal.h"

namespace sg {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kRing = 4 * kWave;         // rows held per wave in the axial ring (power of two)
constexpr int kTaps = 2 * kMaxPsfRadius + 1;
constexpr int kTileRows = 64;            // PSF tile height
constexpr int kAS = kTileRows + 1;       // padded LDS column stride

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

// cos(theta): Sobel (1,2,1) on [label differs from the centre label] with
// clamped image coordinates, in physical units (only evaluated at G = 1)
__device__ __forceinline__ float incidence_cos(const EnvDev& e, const VolDev& v, int x, int y, int lab)
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

__device__ __forceinline__ void wave_sync_lds()
{
    // order this wave's LDS writes before its later LDS reads (LDS executes
    // one wave's instructions in issue order; this stops compiler reordering)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Axial filter of one chunk from the ring: lane l outputs row y0 + l.
__device__ __forceinline__ void axial_from_ring(const float* ringR, const float* ringT, const float* kax, int ra,
                                                int y0, int lane, float& aR, float& aT)
{
    float s1 = 0.f, s2 = 0.f;
    const int base = y0 + lane - ra + kRing;   // >= kWave - ra > 0
    for (int j = 0; j <= 2 * ra; ++j) {
        const int slot = (base + j) & (kRing - 1);
        s1 += kax[j] * ringR[slot];
        s2 += kax[j] * ringT[slot];
    }
    aR = s1;
    aT = s2;
}

// One scanline of the ray pass, executed by one wave (lane = depth row).
__device__ void ray_scanline(const PhysArgs& a, const EnvDev& e, const VolDev& v, const TissueDev* tab,
                             const float* kax, float* ringR, float* ringT, int x, int lane)
{
    const int H = e.H;
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
    const int ra = e.rax;
    // rows -64..-1 of the ring read as zeros (zero padding above the image)
    ringR[kRing - kWave + lane] = 0.f;
    ringT[kRing - kWave + lane] = 0.f;

    float carry_t = 1.f;     // transmission product of the rows above the chunk
    double carry_a = 0.0;    // attenuation integral (sum of alpha) above the chunk
    float E_prev = 0.f;      // E of the previous chunk (its axial output is pending)

    int32_t vox = voxel_at(e, v, x, lane);
    int lab = label_of(v, vox);
    double Z = ct ? z_from_ct(e, v, x, lane) : 0.0;

    const int n_chunks = (H + kWave - 1) / kWave;
    for (int k = 0; k < n_chunks; ++k) {
        const int y0 = k * kWave;
        const int y = y0 + lane;
        const bool act = y < H;
        // gather the next chunk's labels (and CT) ahead of use
        const int32_t vox_n = voxel_at(e, v, x, y + kWave);
        const int lab_n = label_of(v, vox_n);
        const double Zct_n = ct ? z_from_ct(e, v, x, y + kWave) : 0.0;

        // scatterer of this chunk's voxels (computed for every lane, selected below)
        uint32_t w[4];
        philox4x32_10((uint32_t)vox, v.key0, v.key1, w);
        const TissueDev tt = tab[lab];
        const float n0 = sqrtf(-2.f * logf(uniform24(w[0]))) * cospif(2.f * uniform24(w[1]));
        const bool inside = act && vox >= 0;
        const float T = (inside && (unsigned long long)w[2] < tt.thr) ? n0 * tt.sigma0 + tt.mu0 : 0.f;

        // boundary with the next row
        const double Zc = ct ? Z : (double)tt.Z;
        int lab_nr = __shfl_down(lab, 1);
        double Z_nr = __shfl_down(Zc, 1);
        const int lab_first_n = __shfl(lab_n, 0);
        const double Z_first_n = __shfl(ct ? Zct_n : (double)tab[lab_n].Z, 0);
        if (lane == kWave - 1) {
            lab_nr = lab_first_n;
            Z_nr = Z_first_n;
        }
        const bool G = act && (y < H - 1) && (lab != lab_nr);
        float r = 0.f, t = 1.f;
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
        // inclusive wave scans: transmission product (FP32), alpha sum (FP64)
        float tp = act ? t : 1.f;
        double as = act ? (double)tt.alpha : 0.0;
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
        const float Rp = G ? E * cs * fabsf(r) : 0.f;

        // ring slot of this chunk, then the axial filter of the previous chunk
        ringR[(y0 & (kRing - 1)) + lane] = act ? Rp : 0.f;
        ringT[(y0 & (kRing - 1)) + lane] = act ? T : 0.f;
        wave_sync_lds();
        if (k > 0) {
            float aR, aT;
            axial_from_ring(ringR, ringT, kax, ra, y0 - kWave, lane, aR, aT);
            const int yp = y0 - kWave + lane;   // < H
            fR[yp] = aR;
            fT[yp] = aT;
            fE[yp] = E_prev;
        }
        E_prev = E;
        if (act) {
            const int64_t kk = e.out_off + (int64_t)y * e.W + x;
            if (a.dbg.label) a.dbg.label[kk] = (uint8_t)lab;
            if (a.dbg.voxel) a.dbg.voxel[kk] = vox;
            if (a.dbg.energy) a.dbg.energy[kk] = E;
            if (a.dbg.philox) {
                uint4 pw;
                pw.x = inside ? w[0] : 0u;
                pw.y = inside ? w[1] : 0u;
                pw.z = inside ? w[2] : 0u;
                pw.w = inside ? w[3] : 0u;
                reinterpret_cast<uint4*>(a.dbg.philox)[kk] = pw;
            }
        }
        vox = vox_n;
        lab = lab_n;
        Z = Zct_n;
        wave_sync_lds();
    }
    // flush: rows below the image read as zeros
    const int y_last = (n_chunks - 1) * kWave;
    ringR[((y_last + kWave) & (kRing - 1)) + lane] = 0.f;
    ringT[((y_last + kWave) & (kRing - 1)) + lane] = 0.f;
    wave_sync_lds();
    float aR, aT;
    axial_from_ring(ringR, ringT, kax, ra, y_last, lane, aR, aT);
    if (y_last + lane < H) {
        fR[y_last + lane] = aR;
        fT[y_last + lane] = aT;
        fE[y_last + lane] = E_prev;
    }
    wave_sync_lds();
}

__device__ __forceinline__ int next_item(int32_t* counter, int* s_item)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
    __syncthreads();
    return *s_item;
}

// Ray kernel: items (env, group of kWaves * spw scanlines), longest first.
__global__ __launch_bounds__(kThreads) void k_ray(PhysArgs a, QueueDev* q)
{
    __shared__ TissueDev s_tab[SG_MAX_LABELS_DEV];
    __shared__ float s_kax[kTaps];
    __shared__ float s_ring[kWaves][2][kRing];
    __shared__ int s_item;
    for (int i = threadIdx.x; i < a.n_labels; i += kThreads) s_tab[i] = a.table[i];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    for (;;) {
        const int item = next_item(&q->next_ray, &s_item);
        if (item >= a.n_ray) break;
        const ItemRay it = a.ray_items[item];
        const EnvDev e = a.envs[it.env];
        const VolDev v = a.vols[e.vol];
        for (int i = threadIdx.x; i <= 2 * e.rax; i += kThreads) s_kax[i] = a.coefs[e.kax + i];
        __syncthreads();
        for (int s = 0; s < a.scanlines_per_wave; ++s) {
            const int x = it.x0 + s * kWaves + wave;
            if (x < e.W) ray_scanline(a, e, v, s_tab, s_kax, s_ring[wave][0], s_ring[wave][1], x, lane);
        }
    }
}

// PSF kernel: items (env, tile of TX scanlines x 64 rows).
template <int TX>
__global__ __launch_bounds__(kThreads) void k_psf(PhysArgs a, QueueDev* q)
{
    extern __shared__ float lds[];
    __shared__ float s_klat[kTaps];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    for (;;) {
        const int item = next_item(&q->next_psf, &s_item);
        if (item >= a.n_psf) break;
        const ItemPsf it = a.psf_items[item];
        const EnvDev e = a.envs[it.env];
        const int W = e.W, H = e.H, rl = e.rlat;
        const int x0 = (it.tile & 0xFFFF) * TX;
        const int y0 = (it.tile >> 16) * kTileRows;
        const int CW = TX + 2 * rl;
        float* sR = lds;
        float* sT = sR + CW * kAS;
        float* sE = sT + CW * kAS;
        for (int i = tid; i <= 2 * rl; i += kThreads) s_klat[i] = a.coefs[e.klat + i];
        const float* gR = a.fR + e.scr_off;
        const float* gT = a.fT + e.scr_off;
        const float* gE = a.fE + e.scr_off;
        const int gy = y0 + lane;
        const bool yin = gy < H;
        for (int c = wave; c < CW; c += kWaves) {
            const int gx = x0 - rl + c;
            const bool in = yin && gx >= 0 && gx < W;
            const int64_t off = (int64_t)gx * H + gy;
            sR[c * kAS + lane] = in ? gR[off] : 0.f;
            sT[c * kAS + lane] = in ? gT[off] : 0.f;
        }
        for (int c = wave; c < TX; c += kWaves) {
            const int gx = x0 + c;
            sE[c * kAS + lane] = (yin && gx < W) ? gE[(int64_t)gx * H + gy] : 0.f;
        }
        __syncthreads();
        for (int idx = tid; idx < TX * kTileRows; idx += kThreads) {
            const int cx = idx % TX;
            const int r = idx / TX;
            const int x = x0 + cx, y = y0 + r;
            if (x < W && y < H) {
                float s1 = 0.f, s2 = 0.f;
                for (int i = 0; i <= 2 * rl; ++i) {
                    s1 += s_klat[i] * sR[(cx + i) * kAS + r];
                    s2 += s_klat[i] * sT[(cx + i) * kAS + r];
                }
                const float I = s1 + sE[cx * kAS + r] * s2;
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

__global__ void k_queue_reset(QueueDev* q)
{
    if (threadIdx.x == 0) {
        q->next_ray = 0;
        q->next_psf = 0;
        q->n_bad = 0;
        q->pad = 0;
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

int blocks_per_cu(const void* fn, size_t lds)
{
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kThreads, lds) != hipSuccess) return 0;
    return n;
}

}  // namespace

size_t psf_lds_bytes(int tx, int max_rlat)
{
    return sizeof(float) * (size_t)kAS * (2 * (tx + 2 * max_rlat) + tx);
}

bool psf_tile_supported(int tx) { return psf_fn(tx) != nullptr; }

int ray_grid(int n_cu)
{
    return blocks_per_cu(reinterpret_cast<const void*>(&k_ray), 0) * n_cu;
}

int psf_grid(int tx, int max_rlat, int n_cu)
{
    return blocks_per_cu(psf_fn(tx), psf_lds_bytes(tx, max_rlat)) * n_cu;
}

hipError_t launch_ray(const PhysArgs& a, QueueDev* q, int grid, hipStream_t s)
{
    if (a.n_ray <= 0) return hipSuccess;
    if (grid > a.n_ray) grid = a.n_ray;
    if (grid < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_ray, dim3(grid), dim3(kThreads), 0, s, a, q);
    return hipGetLastError();
}

hipError_t launch_psf(const PhysArgs& a, QueueDev* q, int tx, int grid, hipStream_t s)
{
    if (a.n_psf <= 0) return hipSuccess;
    if (grid > a.n_psf) grid = a.n_psf;
    if (grid < 1) return hipErrorInvalidConfiguration;
    const size_t lds = psf_lds_bytes(tx, a.max_rlat);
    if (tx == 16)
        hipLaunchKernelGGL(k_psf<16>, dim3(grid), dim3(kThreads), lds, s, a, q);
    else if (tx == 32)
        hipLaunchKernelGGL(k_psf<32>, dim3(grid), dim3(kThreads), lds, s, a, q);
    else if (tx == 64)
        hipLaunchKernelGGL(k_psf<64>, dim3(grid), dim3(kThreads), lds, s, a, q);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_geometry(EnvDev* envs, const VolDev* vols, const double* poses, int32_t n, QueueDev* q,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_geometry, dim3((n + 127) / 128), dim3(128), 0, s, envs, vols, poses, n, q);
    return hipGetLastError();
}

hipError_t launch_queue_reset(QueueDev* q, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, q);
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
