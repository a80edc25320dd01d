// Internal structures shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

constexpr int kMaxPsfRadius = 32;   // axial / lateral PSF radius limit (pixels)
constexpr int kWave = 64;
constexpr int kRayWaves = 4;        // waves per ray work group (one scanline each)
#define SG_MAX_LABELS_DEV 256

// Label maps live on the device in bricks of 8 x 4 x 4 voxels (128 bytes, one
// cache line; x fastest inside a brick, bricks in x, y, z order), so a gather
// along any direction touches few lines.  The voxel's linear index
// (iz ny + iy) nx + ix stays its identity (noise counter, debug planes).
constexpr int kBrickX = 8, kBrickY = 4, kBrickZ = 4, kBrickBytes = kBrickX * kBrickY * kBrickZ;

struct VolDev {
    const uint8_t* labels;   // bricked (see kBrickX); library-owned copy
    const int16_t* ct;   // may be null
    double sx, sy, sz;   // voxel spacing, mm
    int32_t nx, ny, nz;
    int32_t bnx, bny;    // bricks along x and y
    uint32_t key0, key1; // noise-field key (low / high word of the seed)
    int32_t scales;      // noise scales S >= 1
};

constexpr int kNoiseQ = 4096;   // entries of the quantised normal (w2 >> 20)
constexpr int kCtBins = 4096;   // HU histogram bins of the CT-conditioned surrogate input (HU + 1024)
// Field-scratch scanlines start on 128-byte lines, so a 64-row segment is two whole lines
constexpr int kScrAlign = 32;
constexpr int kMaxNoiseScales = 4;

struct TissueDev {
    float Z;
    float alpha;
    float mu0;
    float sigma0;
    float mu1;                // density parameter
    unsigned long long thr;   // scatter gate: word2 < thr (thr may be 2^32)
};

// Per-environment launch parameters.  The geometry part (P0, DX, DY, valid)
// is filled either on the host (single call) or by the ray kernel from the
// current pose (batched plans).
struct EnvDev {
    int32_t P0[3], DX[3], DY[3];   // Q16 plane origin and per-pixel steps
    int32_t valid;                 // 0: pose rejected, frame is zero
    int32_t W, H;
    int32_t vol;
    int32_t rax, rlat;             // PSF radii
    int32_t kax, klat;             // offsets of the PSF taps in the coefficient pool
    float E0;
    float dx, dy;                  // pixel pitch, mm (incidence angle)
    float disp;                    // 20 / DR
    float disp2;                   // (20 / DR) * log10(2): display slope per octave
    float inv_E0;
    double coef;                   // f * dy_cm
    double coef2;                  // f * dy_cm * log2(e): attenuation in octaves
    double dx64, dy64, f64;        // for device-side geometry
    double psf64;
    double elev64;                 // elevation b of this plane, mm (volumetric probes)
    int32_t pose_env;              // caller's env whose pose this plane uses
    int32_t plane;                 // plane index within that env
    int64_t out_off;               // frame offset in the output (elements)
    int64_t scr_off;               // offset of this env in the field scratch
    int32_t ld;                    // scanline stride of the field scratch: H rounded up to kScrAlign
};

struct ItemRay { int32_t env, x0; };          // x0: first scanline of the group
struct ItemPsf { int32_t env, tile; };        // tile = ty << 16 | tx

struct DebugDev {
    uint8_t* label;
    int32_t* voxel;
    uint32_t* philox;
    float* energy;
    float* intensity;
    float* scatter;
};

// label volumes with at most this many labels take r and t from a pair table
constexpr int kPairLabels = 16;

// work-queue state of the two persistent kernels (device)
struct QueueDev {
    int32_t next_ray;    // next ray work item
    int32_t pad[3];
};

struct PhysArgs {
    const EnvDev* envs;
    const VolDev* vols;
    const TissueDev* table;
    int32_t n_labels;
    const float2* pair_rt;    // [n_labels][n_labels] (r, t) of a boundary between two labels, or null
    const int32_t* q_lut;     // [kNoiseQ] quantised normal of the multi-scale gate, units of 2^-20
    const int32_t* ms_thr;    // [label][kMaxNoiseScales]: entry S - 1 is the gate threshold of S scales
    int32_t multiscale;       // some env's volume has more than one noise scale
    int32_t any_ct;           // some env's volume has a CT (impedance from HU in FP64)
    const float* coefs;       // PSF taps pool
    const ItemRay* ray_items;
    int32_t n_ray;
    const ItemPsf* psf_items;
    int32_t n_psf;
    float* fR;                // scratch fields, scanline-major [x][y] per env
    float* fT;
    float* fE;
    float* out;
    DebugDev dbg;
    int32_t scanlines_per_wave;   // ray group = kRayWaves * scanlines_per_wave
    int32_t max_rlat;             // sizing of the PSF tile's LDS
    // batched steps: the ray kernel computes each item's plane from poses
    // (12 doubles per caller env) and the group of an env's first scanlines
    // stores it in geo_out (the envs array) for later consumers; null when the
    // host staged the geometry in envs
    const double* poses;
    EnvDev* geo_out;
    // the PSF kernel clears this ray-queue counter for the next step (the ray
    // kernel that consumed it has finished); null: the caller resets it
    QueueDev* ray_queue;
};

// Plane geometry: the pose [R|t] (probe mm -> volume mm) places pixel (x, y)
// at probe point (a + x*dx, 0, y*dy), a = -0.5*(W-1)*dx.  Origin and steps
// are converted to Q16 voxel units one rounded operation at a time
// (no contraction) and rounded half-to-even, so host and device agree
// bit for bit.  plane_axis computes volume axis c (voxel size s); it returns
// 1 if the axis is finite and every corner of the plane lies within +-2^30
// (Q16) on it, else 0 (outputs then unspecified).
__host__ __device__ inline int plane_axis(const double* pose, int c, double s, int32_t W, int32_t H, double dx,
                                          double dy, double elev, int32_t& P0, int32_t& DX, int32_t& DY)
{
#pragma clang fp contract(off)
    double a = -0.5 * (double)(W - 1);
    a = a * dx;
    const double r0 = pose[4 * c + 0], r1 = pose[4 * c + 1], r2 = pose[4 * c + 2], tc = pose[4 * c + 3];
    double u = r0 * a;
    u = tc + u;
    const double v = r1 * elev;   // elevation offset (exactly 0 for a single plane)
    u = u + v;
    u = u / s;
    u = u * 65536.0;
    double w = r0 * dx;
    w = w / s;
    w = w * 65536.0;
    double z = r2 * dy;
    z = z / s;
    z = z * 65536.0;
    // non-finite or huge values fail here
    if (!(u > -1e15 && u < 1e15) || !(w > -1e15 && w < 1e15) || !(z > -1e15 && z < 1e15)) return 0;
    const long long p0 = (long long)__builtin_rint(u);
    const long long ddx = (long long)__builtin_rint(w);
    const long long ddy = (long long)__builtin_rint(z);
    const long long lim = 1ll << 30;
    for (int k = 0; k < 4; ++k) {
        const long long qx = (k & 1) ? (long long)(W - 1) : 0;
        const long long qy = (k & 2) ? (long long)(H - 1) : 0;
        const long long q = p0 + qx * ddx + qy * ddy;
        if (q > lim || q < -lim) return 0;
    }
    P0 = (int32_t)p0;
    DX = (int32_t)ddx;
    DY = (int32_t)ddy;
    return 1;
}

// all three axes; 1 if the pose places the whole plane in range, else 0
__host__ __device__ inline int plane_geometry(const double* pose, double sx, double sy, double sz,
                                              int32_t W, int32_t H, double dx, double dy, double elev,
                                              int32_t P0[3], int32_t DX[3], int32_t DY[3])
{
    const double s[3] = {sx, sy, sz};
    for (int c = 0; c < 3; ++c)
        if (!plane_axis(pose, c, s[c], W, H, dx, dy, elev, P0[c], DX[c], DY[c])) return 0;
    return 1;
}

// launchers (physics.hip)
hipError_t launch_queue_reset(QueueDev* q, int n_queues, hipStream_t s);   // resets q[0 .. n_queues)
hipError_t launch_ray(const PhysArgs& a, QueueDev* q, int grid, hipStream_t s);
hipError_t launch_psf(const PhysArgs& a, int tile_x, int grid, hipStream_t s);
hipError_t launch_max_label(const uint8_t* labels, int64_t n, int32_t* d_out, hipStream_t s);
// copy a linear [nz][ny][nx] label map into the bricked layout (bricks = bnx * bny * bnz; padding voxels 0)
hipError_t launch_brick_labels(const uint8_t* src, int32_t nx, int32_t ny, int32_t nz, uint8_t* dst, hipStream_t s);

#if defined(__HIP__)
// byte offset of voxel (ix, iy, iz), inside the grid, in the bricked label map;
// brick counts below 2^24 (checked at registration) keep the 24-bit products exact
__device__ __forceinline__ uint32_t brick_offset(const VolDev& v, int32_t ix, int32_t iy, int32_t iz)
{
    const uint32_t b = __umul24(__umul24((uint32_t)iz >> 2, (uint32_t)v.bny) + ((uint32_t)iy >> 2), (uint32_t)v.bnx) +
                       ((uint32_t)ix >> 3);
    return (b << 7) | (((uint32_t)iz & 3u) << 5) | (((uint32_t)iy & 3u) << 3) | ((uint32_t)ix & 7u);
}
#endif
// surrogate input encoding of every pixel of n_envs frames (8 bf16 per pixel)
hipError_t launch_encode(const PhysArgs& a, int32_t n_envs, int32_t max_pixels, uint16_t* enc, hipStream_t s);
// CT-conditioned input: per-frame HU histograms (hist, n_envs x kCtBins), and when enc is given the
// matched-histogram maps (lut, n_envs x kCtBins) against the reference cumulative counts and the encoding
hipError_t launch_ct_encode(const PhysArgs& a, int32_t n_envs, int32_t max_pixels, uint32_t* hist,
                            const long long* ref_cum, long long n_ref, uint16_t* lut, uint16_t* enc, hipStream_t s);
// pooled reference histogram of n_envs per-frame histograms (int64 counts and inclusive cumulative counts)
hipError_t launch_ct_reference(const uint32_t* hist, int32_t n_envs, long long* ref_hist, long long* ref_cum,
                               hipStream_t s);
size_t psf_lds_bytes(int tile_x, int max_rlat);
bool psf_tile_supported(int tile_x);
// instantiations of the ray kernel: label-only (boundary (r, t) from the
// label-pair table, no CT volume, so no FP64 impedance work) and debug (the
// ray pass writes debug planes); each drops the code and registers the other
// cases need
inline bool ray_label_only(const PhysArgs& a) { return a.pair_rt != nullptr && a.any_ct == 0; }
inline bool ray_debug(const PhysArgs& a)
{
    return a.dbg.label || a.dbg.voxel || a.dbg.philox || a.dbg.energy || a.dbg.scatter;
}
int ray_grid(int n_cu, bool multiscale, bool label_only, bool debug);   // resident ray workgroups
int psf_grid(int tile_x, int max_rlat, int n_cu);    // resident PSF workgroups

}  // namespace sg
