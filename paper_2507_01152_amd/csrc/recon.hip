// Reconstruction observation of the bone-surface task (C ABI in
// include/sonosim.h): per-step surface points from the plan's image planes
// and their voxelisation in the current probe frame.
//
//  * update  -- one wave per (image plane, scanline): its lanes take the
//               scanline's nearest labels (the physics path's Q16 geometry) 64
//               rows at a time, a ballot finds the first bone pixel, and one
//               lane applies the keyed miss test and appends the point (FP64,
//               volume mm) to its env's list with one atomic.
//  * observe -- one workgroup per env: clears the env's 40^3 grid, then maps
//               every stored point into the current probe frame and marks its
//               cell (racing stores of the same value 1 are benign).
// Positions and cell indices are computed in FP64 in a fixed operation order
// without contraction, so they are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "sg_host.h"

namespace sg {

struct Recon {
    int32_t plan = 0;
    int32_t n_user = 0;
    int32_t capacity = 0;
    uint64_t seed = 0;
    unsigned long long keep = 0;   // floor((1 - p_miss) * 2^32)
    DevBuf points;                 // double [n_user][capacity][3]
    DevBuf counts;                 // int32 [n_user] (may exceed capacity)
    DevBuf bone;                   // uint8 [256]
};

void ReconDeleter::operator()(Recon* p) const { delete p; }

void recon_release_all(sg_ctx* c) { c->recons.clear(); }

namespace {

constexpr int kGrid = 40;
constexpr uint32_t kReconTag = 0x5245434Fu;

// Philox4x32-10 (Salmon et al., SC'11) of a full counter
__device__ __forceinline__ void philox_ctr(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                           uint32_t k1, uint32_t w[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    w[0] = c0;
    w[1] = c1;
    w[2] = c2;
    w[3] = c3;
}

__global__ __launch_bounds__(256) void k_recon_update(const EnvDev* __restrict__ envs, int n_planes,
                                                      const VolDev* __restrict__ vols, const double* __restrict__ poses,
                                                      const uint8_t* __restrict__ bone, int step, uint32_t k0, uint32_t k1,
                                                      unsigned long long keep, int capacity, double* __restrict__ pts,
                                                      int32_t* __restrict__ counts)
{
#pragma clang fp contract(off)
    __shared__ uint8_t s_bone[256];
    s_bone[threadIdx.x] = bone[threadIdx.x];
    __syncthreads();
    // one wave per scanline; its lanes look at 64 rows at a time
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.y;   // image plane (internal env)
    if (k >= n_planes) return;
    const EnvDev e = envs[k];
    const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (!e.valid || x >= e.W) return;
    const VolDev v = vols[e.vol];
    int yb = -1;
    for (int y0 = 0; y0 < e.H && yb < 0; y0 += 64) {
        const int y = y0 + lane;
        bool is_bone = false;
        if (y < e.H) {
            int32_t q[3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                q[c] = (int32_t)((uint32_t)e.P0[c] + (uint32_t)x * (uint32_t)e.DX[c] + (uint32_t)y * (uint32_t)e.DY[c]);
            const int32_t ix = (int32_t)((uint32_t)q[0] + 32768u) >> 16;
            const int32_t iy = (int32_t)((uint32_t)q[1] + 32768u) >> 16;
            const int32_t iz = (int32_t)((uint32_t)q[2] + 32768u) >> 16;
            const bool in =
                (uint32_t)ix < (uint32_t)v.nx && (uint32_t)iy < (uint32_t)v.ny && (uint32_t)iz < (uint32_t)v.nz;
            const int lab = in ? (int)v.labels[brick_offset(v, ix, iy, iz)] : 0;
            is_bone = s_bone[lab] != 0;
        }
        const unsigned long long b = __ballot(is_bone);
        if (b) yb = y0 + __ffsll((long long)b) - 1;
    }
    if (yb < 0 || lane != 0) return;
    uint32_t w[4];
    philox_ctr((uint32_t)x | ((uint32_t)e.plane << 16), (uint32_t)e.pose_env, (uint32_t)step, kReconTag, k0, k1, w);
    if (!((unsigned long long)w[0] < keep)) return;
    const double* pose = poses + 12 * e.pose_env;
    double a = -0.5 * (double)(e.W - 1);
    a = a * e.dx64;
    double px = (double)x * e.dx64;
    px = a + px;
    const double pz = (double)yb * e.dy64;
    double p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double s = pose[4 * c + 0] * px;
        const double el = pose[4 * c + 1] * e.elev64;
        s = s + el;
        const double z = pose[4 * c + 2] * pz;
        s = s + z;
        s = s + pose[4 * c + 3];
        p[c] = s;
    }
    const int idx = atomicAdd(&counts[e.pose_env], 1);
    if (idx < capacity) {
        double* o = pts + ((int64_t)e.pose_env * capacity + idx) * 3;
        o[0] = p[0];
        o[1] = p[1];
        o[2] = p[2];
    }
}

__global__ __launch_bounds__(256) void k_recon_observe(const double* __restrict__ pts, const int32_t* __restrict__ counts,
                                                       int capacity, const double* __restrict__ poses,
                                                       uint8_t* __restrict__ grids)
{
#pragma clang fp contract(off)
    const int env = blockIdx.x;
    uint8_t* g = grids + (int64_t)env * kGrid * kGrid * kGrid;
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    for (int i = threadIdx.x; i < kGrid * kGrid * kGrid / 16; i += blockDim.x) reinterpret_cast<uint4*>(g)[i] = zero;
    __syncthreads();
    const double* pose = poses + 12 * env;
    const int n = min(counts[env], capacity);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double* p = pts + ((int64_t)env * capacity + i) * 3;
        double d[3], u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = p[c] - pose[4 * c + 3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            double s = pose[0 * 4 + ax] * d[0];
            const double s1 = pose[1 * 4 + ax] * d[1];
            s = s + s1;
            const double s2 = pose[2 * 4 + ax] * d[2];
            s = s + s2;
            u[ax] = s;
        }
        const double fh = floor(u[2] / 3.0);
        const double fw = floor((u[0] + 60.0) / 3.0);
        const double fe = floor((u[1] + 60.0) / 3.0);
        if (fh >= 0.0 && fh < 40.0 && fw >= 0.0 && fw < 40.0 && fe >= 0.0 && fe < 40.0)
            g[((int)fh * kGrid + (int)fw) * kGrid + (int)fe] = 1;
    }
}

Recon* find_recon(sg_ctx* c, int32_t id)
{
    if (!c) return nullptr;
    auto it = c->recons.find(id);
    return it == c->recons.end() ? nullptr : it->second.get();
}

Plan* recon_plan(sg_ctx* c, const Recon& r)
{
    auto it = c->plans.find(r.plan);
    return it == c->plans.end() ? nullptr : it->second.get();
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_recon_create(sg_ctx* c, int32_t plan_id, int32_t capacity, const uint8_t* bone_labels,
                                     double p_miss, uint64_t seed, int32_t* recon_id)
{
    if (!c || !recon_id) return fail(SG_EINVAL, "sg_recon_create: NULL argument");
    auto it = c->plans.find(plan_id);
    if (it == c->plans.end()) return fail(SG_EINVAL, "sg_recon_create: bad plan id %d", plan_id);
    if (capacity < 1 || capacity > (1 << 24)) return fail(SG_EINVAL, "sg_recon_create: capacity in [1, 2^24]");
    if (!(p_miss >= 0.0 && p_miss <= 1.0)) return fail(SG_EINVAL, "sg_recon_create: p_miss in [0, 1]");
    (void)hipSetDevice(c->device);
    std::unique_ptr<Recon, ReconDeleter> r(new Recon());
    r->plan = plan_id;
    r->n_user = it->second->n_user;
    r->capacity = capacity;
    r->seed = seed;
    const double kp = std::floor((1.0 - p_miss) * 4294967296.0);
    r->keep = (unsigned long long)kp;
    uint8_t bone[256];
    if (bone_labels) {
        std::memcpy(bone, bone_labels, 256);
    } else {
        std::memset(bone, 0, 256);
        bone[3] = 1;
    }
    hipError_t e = r->points.ensure(sizeof(double) * 3 * (size_t)r->n_user * capacity);
    if (e == hipSuccess) e = r->counts.ensure(sizeof(int32_t) * r->n_user);
    if (e == hipSuccess) e = r->bone.ensure(256);
    if (e == hipSuccess) e = hipMemcpy(r->bone.p, bone, 256, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(r->counts.p, 0, sizeof(int32_t) * r->n_user);
    if (e != hipSuccess) return hip_fail(e, "reconstruction allocation");
    const int32_t id = c->next_recon++;
    c->recons[id] = std::move(r);
    *recon_id = id;
    return SG_OK;
}

extern "C" sg_status sg_recon_update(sg_ctx* c, int32_t id, int32_t step)
{
    Recon* r = find_recon(c, id);
    if (!r) return fail(SG_EINVAL, "sg_recon_update: bad reconstruction id");
    Plan* p = recon_plan(c, *r);
    if (!p) return fail(SG_ESTATE, "sg_recon_update: the plan was destroyed");
    (void)hipSetDevice(c->device);
    int maxW = 1;
    for (const EnvDev& e : p->envs) maxW = std::max(maxW, (int)e.W);
    const dim3 grid((unsigned)((maxW + 3) / 4), (unsigned)p->n_envs);   // a wave per scanline
    hipLaunchKernelGGL(k_recon_update, grid, dim3(256), 0, c->stream, (const EnvDev*)p->d_envs.p, p->n_envs,
                       (const VolDev*)c->d_vols.p, (const double*)p->d_poses.p, (const uint8_t*)r->bone.p, step,
                       (uint32_t)r->seed, (uint32_t)(r->seed >> 32), r->keep, r->capacity, (double*)r->points.p,
                       (int32_t*)r->counts.p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SG_OK : hip_fail(e, "reconstruction update");
}

extern "C" sg_status sg_recon_observe(sg_ctx* c, int32_t id, uint8_t* grids)
{
    Recon* r = find_recon(c, id);
    if (!r || !grids) return fail(SG_EINVAL, "sg_recon_observe: bad reconstruction id or NULL grids");
    Plan* p = recon_plan(c, *r);
    if (!p) return fail(SG_ESTATE, "sg_recon_observe: the plan was destroyed");
    if ((reinterpret_cast<uintptr_t>(grids) & 15) != 0) return fail(SG_EINVAL, "sg_recon_observe: grids not 16-byte aligned");
    (void)hipSetDevice(c->device);
    hipLaunchKernelGGL(k_recon_observe, dim3((unsigned)r->n_user), dim3(256), 0, c->stream,
                       (const double*)r->points.p, (const int32_t*)r->counts.p, r->capacity,
                       (const double*)p->d_poses.p, grids);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SG_OK : hip_fail(e, "reconstruction observation");
}

extern "C" sg_status sg_recon_counts(sg_ctx* c, int32_t id, int64_t* stored, int64_t* overflow)
{
    Recon* r = find_recon(c, id);
    if (!r) return fail(SG_EINVAL, "sg_recon_counts: bad reconstruction id");
    (void)hipSetDevice(c->device);
    std::vector<int32_t> n(r->n_user);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(n.data(), r->counts.p, sizeof(int32_t) * r->n_user, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reconstruction counts");
    for (int i = 0; i < r->n_user; ++i) {
        if (stored) stored[i] = std::min(n[i], r->capacity);
        if (overflow) overflow[i] = std::max(0, n[i] - r->capacity);
    }
    return SG_OK;
}

extern "C" sg_status sg_recon_points(sg_ctx* c, int32_t id, int32_t env, double* xyz, int64_t max_points, int64_t* n)
{
    Recon* r = find_recon(c, id);
    if (!r || !xyz || !n || env < 0 || env >= (r ? r->n_user : 0) || max_points < 0)
        return fail(SG_EINVAL, "sg_recon_points: bad arguments");
    int64_t stored = 0;
    sg_status s = SG_OK;
    std::vector<int64_t> all(r->n_user);
    s = sg_recon_counts(c, id, all.data(), nullptr);
    if (s != SG_OK) return s;
    stored = std::min<int64_t>(all[env], max_points);
    const hipError_t e = hipMemcpy(xyz, (const double*)r->points.p + (int64_t)env * r->capacity * 3,
                                   sizeof(double) * 3 * (size_t)stored, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reconstruction points");
    *n = stored;
    return SG_OK;
}

extern "C" sg_status sg_recon_reset(sg_ctx* c, int32_t id, int32_t env)
{
    Recon* r = find_recon(c, id);
    if (!r || env >= r->n_user) return fail(SG_EINVAL, "sg_recon_reset: bad reconstruction id or env");
    (void)hipSetDevice(c->device);
    int32_t* cnt = (int32_t*)r->counts.p;
    const hipError_t e = env < 0 ? hipMemsetAsync(cnt, 0, sizeof(int32_t) * r->n_user, c->stream)
                                 : hipMemsetAsync(cnt + env, 0, sizeof(int32_t), c->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, "reconstruction reset");
}

extern "C" sg_status sg_recon_destroy(sg_ctx* c, int32_t id)
{
    if (!find_recon(c, id)) return fail(SG_EINVAL, "sg_recon_destroy: bad reconstruction id");
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->recons.erase(id);
    return SG_OK;
}
