// sg_simulate without allocation (C ABI in include/sonosim.h), for callers
// that cannot allocate: code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc.  Every buffer the physics kernels use
// beyond the caller's volumes and frames -- the per-image-plane records, PSF
// taps and work lists, the ray kernel's work counter and the three FP32 field
// planes passed from the ray kernel to the PSF kernel -- lives in one
// file-scope device array, `scratch`, of kNoAllocBytes on each GPU (held
// until the process ends).  The host stages the records in a static array.
// Calls that overlap on one GPU (e.g. on two streams) race on `scratch`.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "sg_host.h"

namespace sg {
namespace {

constexpr size_t kParamBytes = size_t(2) << 20;     // records: envs | taps | ray items | PSF items
constexpr size_t kQueueOff = kParamBytes;           // the ray kernel's work counter
constexpr size_t kFieldOff = kParamBytes + 4096;    // three FP32 field planes
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;                       // guards everything below
void* g_scratch[kMaxDevices];          // device address of `scratch` on each GPU
hipEvent_t g_uploaded[kMaxDevices];    // recorded after that device's last upload from g_stage
hipEvent_t g_last = nullptr;           // the upload from g_stage that may still be reading it
alignas(256) unsigned char g_stage[kParamBytes];   // host staging of the records

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    // the host-side name of `scratch` is not a device address: take this
    // device's copy from the runtime (the caller made `device` current)
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!g_uploaded[device]) {
        e = hipEventCreateWithFlags(&g_uploaded[device], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    g_scratch[device] = p;
    return hipSuccess;
}

}  // namespace sg

using namespace sg;

extern "C" sg_status sg_simulate_noalloc(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                                         const double* poses, float* out, const int64_t* out_offsets)
{
    if (!c) return fail(SG_EINVAL, "sg_simulate_noalloc: NULL context");
    if (n < 0) return fail(SG_EINVAL, "sg_simulate_noalloc: n_envs < 0");
    if (n == 0) return SG_OK;
    if (!vol_ids || !probes || !poses || !out || !out_offsets)
        return fail(SG_EINVAL, "sg_simulate_noalloc: NULL argument");
    (void)hipSetDevice(c->device);
    sg_status s = check_envs(c, n, vol_ids, probes);
    if (s != SG_OK) return s;
    if (c->vols_dirty) return fail(SG_ESTATE, "sg_simulate_noalloc: volume table not uploaded");
    int planes = 0;
    for (int i = 0; i < n; ++i) planes += probe_planes(probes[i]);
    if (planes > kNoAllocMaxPlanes)
        return fail(SG_ERANGE, "sg_simulate_noalloc: %d image planes, at most %d per call", planes, kNoAllocMaxPlanes);

    std::lock_guard<std::mutex> lk(g_mu);
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch[c->device])
        return fail(SG_ESTATE, "sg_simulate_noalloc: no scratch on device %d", c->device);
    unsigned char* base = (unsigned char*)g_scratch[c->device];
    if (g_last) {   // the previous upload from the staging area has finished reading it
        const hipError_t e = hipEventSynchronize(g_last);
        if (e != hipSuccess) return hip_fail(e, "staging wait");
        g_last = nullptr;
    }
    // staging layout: env records | tap pool | ray items | PSF items
    EnvDev* envs = reinterpret_cast<EnvDev*>(g_stage);
    const size_t o_pool = align256(sizeof(EnvDev) * kNoAllocMaxPlanes);
    float* pool = reinterpret_cast<float*>(g_stage + o_pool);
    const int64_t pool_cap = (int64_t)kNoAllocMaxPlanes * 2 * kPsfTapsMax;
    const size_t o_items = align256(o_pool + sizeof(float) * pool_cap);
    static_assert(sizeof(ItemRay) == sizeof(ItemPsf), "one item array");
    const int64_t item_cap = (int64_t)((kParamBytes - o_items) / sizeof(ItemRay));

    int64_t pool_used = 0, scr = 0;
    int n_int = 0, max_rlat = 0, multiscale = 0, any_ct = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(poses[12 * i + k])) return fail(SG_EINVAL, "env %d: pose is not finite", i);
        if (out_offsets[i] < 0) return fail(SG_EINVAL, "env %d: negative output offset", i);
        const VolDev& v = c->vols[vol_ids[i]].dev;
        multiscale |= v.scales > 1;
        any_ct |= v.ct != nullptr;
        for (int j = 0; j < probe_planes(probes[i]); ++j) {
            EnvDev& ed = envs[n_int];
            s = fill_env_static_into(probes[i], vol_ids[i], i, j, out_offsets[i], scr, pool, pool_cap, &pool_used, ed);
            if (s != SG_OK) return s;
            ed.valid = plane_geometry(poses + 12 * i, v.sx, v.sy, v.sz, probes[i].W, probes[i].H, probes[i].dx_mm,
                                      probes[i].dy_mm, ed.elev64, ed.P0, ed.DX, ed.DY);
            if (!ed.valid)
                return fail(SG_ERANGE, "env %d plane %d: image plane outside the fixed-point range (|Q16| > 2^30)",
                            i, j);
            scr += (int64_t)probes[i].W * ed.ld;
            max_rlat = std::max(max_rlat, ed.rlat);
            ++n_int;
        }
    }
    const int64_t scr_cap = (int64_t)((kNoAllocBytes - kFieldOff) / (3 * sizeof(float)));
    if (scr > scr_cap)
        return fail(SG_ERANGE, "sg_simulate_noalloc: %lld field pixels (scanlines padded to %d rows), at most %lld",
                    (long long)scr, kScrAlign, (long long)scr_cap);
    // longest scanlines first (ray items cost ~H), then wider frames, then call order
    int order[kNoAllocMaxPlanes];
    for (int i = 0; i < n_int; ++i) order[i] = i;
    std::sort(order, order + n_int, [&](int x, int y) {
        if (envs[x].H != envs[y].H) return envs[x].H > envs[y].H;
        if (envs[x].W != envs[y].W) return envs[x].W > envs[y].W;
        return x < y;
    });
    // work lists of sg_simulate's launch shape: groups of kRayWaves scanlines, PSF tiles of 32 x 64
    constexpr int kTx = 32;
    ItemRay* rays = reinterpret_cast<ItemRay*>(g_stage + o_items);
    int64_t nr = 0;
    for (int k = 0; k < n_int; ++k) {
        const int e = order[k];
        for (int x0 = 0; x0 < envs[e].W; x0 += kRayWaves) {
            if (nr >= item_cap) return fail(SG_ERANGE, "sg_simulate_noalloc: work lists exceed the scratch");
            rays[nr++] = ItemRay{e, x0};
        }
    }
    ItemPsf* tiles = reinterpret_cast<ItemPsf*>(rays + nr);
    int64_t nt = 0;
    for (int k = 0; k < n_int; ++k) {
        const int e = order[k];
        const int tx = (envs[e].W + kTx - 1) / kTx, ty = (envs[e].H + 63) / 64;
        for (int j = 0; j < ty; ++j)
            for (int i = 0; i < tx; ++i) {
                if (nr + nt >= item_cap) return fail(SG_ERANGE, "sg_simulate_noalloc: work lists exceed the scratch");
                tiles[nt++] = ItemPsf{e, (j << 16) | i};
            }
    }
    const size_t staged = o_items + sizeof(ItemRay) * (size_t)(nr + nt);
    hipError_t e = hipMemcpyAsync(base, g_stage, staged, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(g_uploaded[c->device], c->stream);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");
    g_last = g_uploaded[c->device];

    PhysArgs a;
    std::memset(&a, 0, sizeof(a));
    a.envs = reinterpret_cast<const EnvDev*>(base);
    a.vols = (const VolDev*)c->d_vols.p;
    a.table = (const TissueDev*)c->table.p;
    a.n_labels = c->n_labels;
    a.pair_rt = c->n_labels <= kPairLabels ? (const float2*)c->pair_rt.p : nullptr;
    a.q_lut = (const int32_t*)c->q_lut.p;
    a.ms_thr = (const int32_t*)c->ms_thr.p;
    a.coefs = reinterpret_cast<const float*>(base + o_pool);
    a.ray_items = reinterpret_cast<const ItemRay*>(base + o_items);
    a.n_ray = (int32_t)nr;
    a.psf_items = reinterpret_cast<const ItemPsf*>(base + o_items + sizeof(ItemRay) * (size_t)nr);
    a.n_psf = (int32_t)nt;
    a.fR = reinterpret_cast<float*>(base + kFieldOff);
    a.fT = a.fR + scr;
    a.fE = a.fT + scr;
    a.out = out;
    a.scanlines_per_wave = 1;
    a.max_rlat = max_rlat;
    a.multiscale = multiscale;
    a.any_ct = any_ct;
    // the work counter starts at zero: cleared by a kernel (no memset node under graph capture)
    QueueDev* q = reinterpret_cast<QueueDev*>(base + kQueueOff);
    if ((e = launch_queue_reset(q, 1, c->stream)) != hipSuccess) return hip_fail(e, "queue reset");
    if ((e = launch_ray(a, q, ray_grid(c->n_cu, multiscale != 0, ray_label_only(a), false), c->stream)) != hipSuccess)
        return hip_fail(e, "ray kernel launch");
    if ((e = launch_psf(a, kTx, psf_grid(kTx, max_rlat, c->n_cu), c->stream)) != hipSuccess)
        return hip_fail(e, "PSF kernel launch");
    return SG_OK;
}
