// Host side of the C ABI declared in include/sonosim.h: contexts, volume and
// tissue registries, argument validation, plane geometry, work lists,
// staging, batched plans with HIP graph capture, and the launch-shape
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sg_internal.h"
#include "sonosim.h"
#include "sg_host.h"

namespace {

thread_local std::string g_err;

}  // namespace

namespace sg {

sg_status fail(sg_status code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

sg_status hip_fail(hipError_t e, const char* what)
{
    return fail(SG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

DevBuf::~DevBuf()
{
    if (p) (void)hipFree(p);
}

hipError_t DevBuf::ensure(size_t bytes)
{
    if (bytes <= cap) return hipSuccess;
    if (p) {
        // work already enqueued may still use the old buffer
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
}

PinnedBuf::~PinnedBuf()
{
    if (ev) (void)hipEventSynchronize(ev), (void)hipEventDestroy(ev);
    if (p) (void)hipHostFree(p);
}

hipError_t PinnedBuf::acquire(size_t bytes)
{
    if (ev) {
        hipError_t e = hipEventSynchronize(ev);   // previous upload from this buffer done
        if (e != hipSuccess) return e;
    } else {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (bytes <= cap) return hipSuccess;
    if (p) {
        (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    size_t want = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e == hipSuccess) cap = want;
    return e;
}

// normalised sampled Gaussian of std sigma; radius max(1, ceil(3 sigma));
// taps 0 .. 2r into out (room for kPsfTapsMax); returns r, or -1 beyond kMaxPsfRadius
int psf_taps_into(double sigma, float* out)
{
    int r = (int)std::ceil(3.0 * sigma);
    if (r < 1) r = 1;
    if (r > kMaxPsfRadius) return -1;
    double k[kPsfTapsMax];
    double sum = 0.0;
    for (int i = -r; i <= r; ++i) {
        k[i + r] = std::exp(-((double)i * (double)i) / (2.0 * sigma * sigma));
        sum += k[i + r];
    }
    for (int i = 0; i <= 2 * r; ++i) out[i] = (float)(k[i] / sum);
    return r;
}

unsigned long long gate_threshold(float mu1)
{
    // density gate N1 <= mu1 for N1 ~ N(0, 1) as the integer test
    // word2 < floor(Phi(mu1) * 2^32), Phi(m) = erfc(-m / sqrt 2) / 2
    const double m = (double)mu1;
    const double phi = 0.5 * std::erfc(-m / std::sqrt(2.0));
    const double x = std::floor(phi * 4294967296.0);
    if (x >= 4294967296.0) return 4294967296ull;
    if (x <= 0.0) return 0ull;
    return (unsigned long long)x;
}

int32_t multiscale_threshold(int S, float mu1)
{
    // multi-scale gate: (1 / sqrt S) sum_s Q_s 2^-20 <= mu1 with integer Q_s,
    // i.e. sum_s Q_s <= floor(sqrt(S) mu1 2^20), one FP64 rounding per step
    // in this order; clamped to int32 (sums of at most four quantised normals
    // stay far inside it)
    double x = std::sqrt((double)S);
    x = x * (double)mu1;
    x = x * 1048576.0;
    x = std::floor(x);
    if (!(x > -2147483648.0)) return INT32_MIN;
    if (x > 2147483647.0) return INT32_MAX;
    return (int32_t)x;
}

sg_status check_probe(const sg_probe& p, int idx)
{
    if (p.W < 1 || p.W > SG_MAX_IMAGE || p.H < 1 || p.H > SG_MAX_IMAGE)
        return fail(SG_EINVAL, "env %d: image size %dx%d outside [1, %d]", idx, p.W, p.H, SG_MAX_IMAGE);
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(p.dx_mm) || !pos(p.dy_mm) || !pos(p.E0) || !pos(p.psf_frac) || !pos(p.dr_db) ||
        !std::isfinite(p.f_mhz) || p.f_mhz < 0.0)
        return fail(SG_EINVAL, "env %d: probe parameters must be finite and positive", idx);
    if (p.n_elev < 0 || p.n_elev > SG_MAX_ELEV || (p.n_elev > 1 && !pos(p.elev_mm)))
        return fail(SG_EINVAL, "env %d: n_elev in [0, %d] with elev_mm > 0 for several planes", idx, SG_MAX_ELEV);
    return SG_OK;
}

int probe_planes(const sg_probe& p) { return p.n_elev > 1 ? p.n_elev : 1; }

double plane_elevation(const sg_probe& p, int j)
{
    if (probe_planes(p) == 1) return 0.0;
    return ((double)j - 0.5 * (double)(p.n_elev - 1)) * p.elev_mm;
}

// Static (pose-independent) part of an environment's parameters.
sg_status fill_env_static(const sg_probe& p, int32_t vol, int idx, int plane, int64_t out_off, int64_t scr_off,
                          std::vector<float>& pool, EnvDev& e)
{
    float taps[2 * kPsfTapsMax];
    int64_t used = 0;
    const sg_status s = fill_env_static_into(p, vol, idx, plane, out_off, scr_off, taps, 2 * kPsfTapsMax, &used, e);
    if (s != SG_OK) return s;
    e.kax += (int32_t)pool.size();
    e.klat += (int32_t)pool.size();
    pool.insert(pool.end(), taps, taps + used);
    return SG_OK;
}

sg_status fill_env_static_into(const sg_probe& p, int32_t vol, int idx, int plane, int64_t out_off, int64_t scr_off,
                               float* pool, int64_t pool_cap, int64_t* pool_used, EnvDev& e)
{
    std::memset(&e, 0, sizeof(e));
    e.pose_env = idx;
    e.plane = plane;
    e.elev64 = plane_elevation(p, plane);
    e.W = p.W;
    e.H = p.H;
    e.vol = vol;
    float kax[kPsfTapsMax], klat[kPsfTapsMax];
    e.rax = psf_taps_into(p.psf_frac * (double)p.H, kax);
    e.rlat = psf_taps_into(p.psf_frac * (double)p.W, klat);
    if (e.rax < 0 || e.rlat < 0)
        return fail(SG_EINVAL, "env %d: PSF radius exceeds %d pixels", idx, kMaxPsfRadius);
    const int64_t nax = 2 * e.rax + 1, nlat = 2 * e.rlat + 1;
    if (*pool_used + nax + nlat > pool_cap) return fail(SG_ERANGE, "env %d: PSF tap pool full", idx);
    e.kax = (int32_t)*pool_used;
    std::memcpy(pool + *pool_used, kax, sizeof(float) * nax);
    e.klat = (int32_t)(*pool_used + nax);
    std::memcpy(pool + *pool_used + nax, klat, sizeof(float) * nlat);
    *pool_used += nax + nlat;
    e.E0 = (float)p.E0;
    e.inv_E0 = (float)(1.0 / p.E0);
    e.dx = (float)p.dx_mm;
    e.dy = (float)p.dy_mm;
    e.disp = (float)(20.0 / p.dr_db);
    e.disp2 = (float)((20.0 / p.dr_db) * 0.30102999566398119521);    // log10(2)
    e.coef = p.f_mhz * (p.dy_mm / 10.0);
    e.coef2 = e.coef * 1.44269504088896340736;                        // log2(e)
    e.dx64 = p.dx_mm;
    e.dy64 = p.dy_mm;
    e.f64 = p.f_mhz;
    e.psf64 = p.psf_frac;
    e.out_off = out_off + (int64_t)plane * p.W * p.H;
    e.scr_off = scr_off;
    e.ld = (p.H + kScrAlign - 1) / kScrAlign * kScrAlign;
    return SG_OK;
}

void build_items(const std::vector<EnvDev>& envs, const std::vector<int>& order, int spw, int tx,
                 std::vector<ItemRay>& rays, std::vector<ItemPsf>& tiles)
{
    rays.clear();
    tiles.clear();
    const int group = kRayWaves * spw;
    for (int e : order) {
        for (int x0 = 0; x0 < envs[e].W; x0 += group) rays.push_back(ItemRay{e, x0});
    }
    for (int e : order) {
        const int nx = (envs[e].W + tx - 1) / tx, ny = (envs[e].H + 63) / 64;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) tiles.push_back(ItemPsf{e, (j << 16) | i});
    }
}

}  // namespace sg

using namespace sg;

// ---------------------------------------------------------------------------

extern "C" const char* sg_last_error(void) { return g_err.c_str(); }

extern "C" int32_t sg_version(void) { return 100; }

extern "C" sg_status sg_noise_quantiles(int32_t* out)
{
    if (!out) return fail(SG_EINVAL, "sg_noise_quantiles: NULL argument");
    // Phi(x) = erfc(-x / sqrt 2) / 2 is increasing: bisect to adjacent doubles
    for (int k = 0; k < kNoiseQ; ++k) {
        const double p = ((double)k + 0.5) / (double)kNoiseQ;
        double lo = -40.0, hi = 40.0;
        for (int it = 0; it < 2000; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p)
                lo = mid;
            else
                hi = mid;
        }
        // the double nearer the root of the computed Phi, in units of 2^-20
        // (an exact scaling), rounded half to even
        const double flo = std::fabs(0.5 * std::erfc(-lo / std::sqrt(2.0)) - p);
        const double fhi = std::fabs(0.5 * std::erfc(-hi / std::sqrt(2.0)) - p);
        out[k] = (int32_t)std::nearbyint((flo < fhi ? lo : hi) * 1048576.0);
    }
    return SG_OK;
}

extern "C" sg_status sg_create(sg_ctx** out, int32_t device, void* stream)
{
    if (!out) return fail(SG_EINVAL, "sg_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(SG_EINVAL, "sg_create: device %d of %d", device, n);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    sg_ctx* c = new (std::nothrow) sg_ctx();
    if (!c) return fail(SG_ENOMEM, "sg_create: out of host memory");
    c->device = device;
    c->stream = (hipStream_t)stream;
    e = noalloc_init(device);   // the no-allocation entry point's scratch on this device
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "scratch symbol");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->n_cu = prop.multiProcessorCount;
        c->arch = prop.gcnArchName;
    }
    std::vector<int32_t> q(kNoiseQ);
    (void)sg_noise_quantiles(q.data());
    e = c->q_lut.ensure(sizeof(int32_t) * kNoiseQ);
    if (e == hipSuccess) e = hipMemcpy(c->q_lut.p, q.data(), sizeof(int32_t) * kNoiseQ, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "noise table upload");
    }
    *out = c;
    return SG_OK;
}

extern "C" sg_status sg_destroy(sg_ctx* c)
{
    if (!c) return SG_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    surrogate_release_all(c);
    recon_release_all(c);
    for (HostVolume& v : c->vols) (void)hipFree(v.bricks);
    delete c;
    return SG_OK;
}

extern "C" sg_status sg_set_stream(sg_ctx* c, void* stream)
{
    if (!c) return fail(SG_EINVAL, "sg_set_stream: NULL context");
    c->stream = (hipStream_t)stream;
    for (auto& kv : c->plans) kv.second->graph_out = nullptr;   // re-capture on the new stream
    return SG_OK;
}

extern "C" sg_status sg_synchronize(sg_ctx* c)
{
    if (!c) return fail(SG_EINVAL, "sg_synchronize: NULL context");
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, "hipStreamSynchronize");
}

extern "C" sg_status sg_volume_register(sg_ctx* c, const sg_volume_desc* d, int32_t* vol_id)
{
    if (!c || !d || !vol_id) return fail(SG_EINVAL, "sg_volume_register: NULL argument");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(SG_EINVAL, "volume dims must be >= 1");
    const int64_t nvox = (int64_t)d->nx * d->ny * d->nz;
    if (nvox >= (1ll << 31)) return fail(SG_EINVAL, "volume has %lld voxels (limit 2^31 - 1)", (long long)nvox);
    for (int i = 0; i < 3; ++i)
        if (!(std::isfinite(d->spacing_mm[i]) && d->spacing_mm[i] > 0.0))
            return fail(SG_EINVAL, "voxel spacing must be finite and positive");
    if (!d->labels) return fail(SG_EINVAL, "labels pointer is NULL");
    if (d->noise_scales < 0 || d->noise_scales > kMaxNoiseScales)
        return fail(SG_EINVAL, "noise_scales %d outside [0, %d]", d->noise_scales, kMaxNoiseScales);
    (void)hipSetDevice(c->device);
    hipError_t e = c->scan.ensure(sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = hipMemsetAsync(c->scan.p, 0, sizeof(int32_t), c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    e = launch_max_label(d->labels, nvox, (int32_t*)c->scan.p, c->stream);
    if (e != hipSuccess) return hip_fail(e, "max-label scan");
    int32_t mx = 0;
    e = hipMemcpyAsync(&mx, c->scan.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "max-label readback");
    // the library's bricked copy of the label map
    const int64_t bnx = (d->nx + kBrickX - 1) / kBrickX, bny = (d->ny + kBrickY - 1) / kBrickY,
                  bnz = (d->nz + kBrickZ - 1) / kBrickZ;
    const int64_t n_bricks = bnx * bny * bnz;
    if (n_bricks >= (1ll << 24))
        return fail(SG_EINVAL, "volume needs %lld label bricks of %dx%dx%d voxels (limit 2^24 - 1)",
                    (long long)n_bricks, kBrickX, kBrickY, kBrickZ);
    uint8_t* bricks = nullptr;
    e = hipMalloc((void**)&bricks, (size_t)n_bricks * kBrickBytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (label bricks)");
    e = launch_brick_labels(d->labels, d->nx, d->ny, d->nz, bricks, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(bricks);
        return hip_fail(e, "label bricking");
    }
    HostVolume v;
    v.bricks = bricks;
    v.dev.labels = bricks;
    v.dev.bnx = (int32_t)bnx;
    v.dev.bny = (int32_t)bny;
    v.dev.ct = d->ct_hu;
    v.dev.sx = d->spacing_mm[0];
    v.dev.sy = d->spacing_mm[1];
    v.dev.sz = d->spacing_mm[2];
    v.dev.nx = d->nx;
    v.dev.ny = d->ny;
    v.dev.nz = d->nz;
    v.dev.key0 = (uint32_t)d->noise_seed;
    v.dev.key1 = (uint32_t)(d->noise_seed >> 32);
    v.dev.scales = d->noise_scales < 1 ? 1 : d->noise_scales;
    v.max_label = mx;
    v.live = true;
    c->vols.push_back(v);
    c->vols_dirty = true;
    *vol_id = (int32_t)c->vols.size() - 1;
    // the device table is brought up to date here, where allocating is
    // allowed (the entry point without allocation relies on it)
    return sync_volumes(c);
}

extern "C" sg_status sg_volume_release(sg_ctx* c, int32_t id)
{
    if (!c || id < 0 || id >= (int32_t)c->vols.size() || !c->vols[id].live)
        return fail(SG_EINVAL, "sg_volume_release: bad volume id %d", id);
    // work already enqueued may still read the bricked labels
    (void)hipSetDevice(c->device);
    const hipError_t e = hipStreamSynchronize(c->stream);
    c->vols[id].live = false;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    (void)hipFree(c->vols[id].bricks);
    c->vols[id].bricks = nullptr;
    c->vols[id].dev.labels = nullptr;
    return SG_OK;
}

extern "C" sg_status sg_tissue_table_set(sg_ctx* c, const sg_tissue* rows, int32_t n)
{
    if (!c || !rows) return fail(SG_EINVAL, "sg_tissue_table_set: NULL argument");
    if (n < 1 || n > SG_MAX_LABELS) return fail(SG_EINVAL, "table size %d outside [1, %d]", n, SG_MAX_LABELS);
    std::vector<TissueDev> t(n);
    std::vector<int32_t> ms((size_t)n * kMaxNoiseScales, 0);
    for (int i = 0; i < n; ++i) {
        const sg_tissue& r = rows[i];
        if (std::isnan(r.Z_mrayl) || r.Z_mrayl < 0.f || !std::isfinite(r.alpha_np_cm_mhz) ||
            r.alpha_np_cm_mhz < 0.f || !std::isfinite(r.mu0) || !std::isfinite(r.sigma0) || std::isnan(r.mu1))
            return fail(SG_EINVAL, "tissue row %d invalid (Z >= 0, alpha >= 0 finite, mu0/sigma0 finite)", i);
        t[i].Z = r.Z_mrayl;
        t[i].alpha = r.alpha_np_cm_mhz;
        t[i].mu0 = r.mu0;
        t[i].sigma0 = r.sigma0;
        t[i].mu1 = r.mu1;
        t[i].thr = gate_threshold(r.mu1);
        for (int s = 2; s <= kMaxNoiseScales; ++s) ms[(size_t)i * kMaxNoiseScales + s - 1] = multiscale_threshold(s, r.mu1);
    }
    // reflection and transmission of a boundary between labels i (above) and j
    // (below), for label volumes: the ray kernel's FP64 expressions, evaluated
    // here once per pair (IEEE double on both sides, so the same bits)
    std::vector<float2> rt((size_t)kPairLabels * kPairLabels, make_float2(0.f, 1.f));
    if (n <= kPairLabels) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double Zc = (double)t[i].Z, Zn = (double)t[j].Z;
                float r = 0.f, tt = 1.f;
                if (i != j && Zc != Zn) {
                    if (Zc == 0.0 || Zn == 0.0 || std::isinf(Zc) || std::isinf(Zn)) {
                        r = Zn > Zc ? 1.f : -1.f;
                        tt = 0.f;
                    } else {
                        const double s = Zc + Zn;
                        r = (float)((Zn - Zc) / s);
                        tt = (float)((2.0 * Zc / s) * (2.0 * Zn / s));
                    }
                }
                rt[(size_t)i * n + j] = make_float2(r, tt);
            }
    }
    (void)hipSetDevice(c->device);
    // the previous table may still be read by enqueued work: wait for it
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = c->table.ensure(sizeof(TissueDev) * SG_MAX_LABELS_DEV);
    if (e == hipSuccess) e = c->pair_rt.ensure(sizeof(float2) * rt.size());
    if (e == hipSuccess) e = c->ms_thr.ensure(sizeof(int32_t) * SG_MAX_LABELS_DEV * kMaxNoiseScales);
    if (e == hipSuccess) e = hipMemcpy(c->ms_thr.p, ms.data(), sizeof(int32_t) * ms.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->table.p, t.data(), sizeof(TissueDev) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->pair_rt.p, rt.data(), sizeof(float2) * rt.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "tissue table upload");
    c->n_labels = n;
    return SG_OK;
}

namespace sg {

sg_status sync_volumes(sg_ctx* c)
{
    if (!c->vols_dirty) return SG_OK;
    std::vector<VolDev> v(c->vols.size());
    for (size_t i = 0; i < v.size(); ++i) v[i] = c->vols[i].dev;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = c->d_vols.ensure(sizeof(VolDev) * std::max<size_t>(v.size(), 1));
    if (e == hipSuccess && !v.empty())
        e = hipMemcpy(c->d_vols.p, v.data(), sizeof(VolDev) * v.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "volume table upload");
    c->vols_dirty = false;
    return SG_OK;
}

sg_status check_envs(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes)
{
    if (c->n_labels < 1) return fail(SG_ESTATE, "no tissue table set");
    for (int i = 0; i < n; ++i) {
        const int v = vol_ids[i];
        if (v < 0 || v >= (int)c->vols.size() || !c->vols[v].live)
            return fail(SG_EINVAL, "env %d: bad volume id %d", i, v);
        if (c->vols[v].max_label >= c->n_labels)
            return fail(SG_EINVAL, "env %d: volume %d has label %d but the table has %d rows", i, v,
                        c->vols[v].max_label, c->n_labels);
        sg_status s = check_probe(probes[i], i);
        if (s != SG_OK) return s;
    }
    return SG_OK;
}

}  // namespace sg

namespace sg {

// Validate a call's environments, compute their geometry on the host and
// upload the parameters and work lists; fills `a` (fields scratch, queue and
// work lists of the context).  Nothing is launched.
sg_status stage_physics(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes, const double* poses,
                        float* out, const int64_t* out_offsets, const sg_debug_planes* dbg, PhysArgs& a,
                        StageInfo& info)
{
    sg_status s = check_envs(c, n, vol_ids, probes);
    if (s != SG_OK) return s;
    // one internal env per image plane (volumetric probes have several)
    std::vector<EnvDev> envs;
    std::vector<float> pool;
    int64_t scr = 0;
    int max_rlat = 0, max_px = 0, multiscale = 0, any_ct = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(poses[12 * i + k])) return fail(SG_EINVAL, "env %d: pose is not finite", i);
        if (out_offsets[i] < 0) return fail(SG_EINVAL, "env %d: negative output offset", i);
        const VolDev& v = c->vols[vol_ids[i]].dev;
        multiscale |= v.scales > 1;
        any_ct |= v.ct != nullptr;
        for (int j = 0; j < probe_planes(probes[i]); ++j) {
            EnvDev ed;
            s = fill_env_static(probes[i], vol_ids[i], i, j, out_offsets[i], scr, pool, ed);
            if (s != SG_OK) return s;
            ed.valid = plane_geometry(poses + 12 * i, v.sx, v.sy, v.sz, probes[i].W, probes[i].H, probes[i].dx_mm,
                                      probes[i].dy_mm, ed.elev64, ed.P0, ed.DX, ed.DY);
            if (!ed.valid)
                return fail(SG_ERANGE, "env %d plane %d: image plane outside the fixed-point range (|Q16| > 2^30)",
                            i, j);
            scr += (int64_t)probes[i].W * ed.ld;
            max_rlat = std::max(max_rlat, ed.rlat);
            max_px = std::max(max_px, probes[i].W * probes[i].H);
            envs.push_back(ed);
        }
    }
    const int n_int = (int)envs.size();
    s = sync_volumes(c);
    if (s != SG_OK) return s;
    // longest scanlines first (ray items cost ~H), then wider frames
    std::vector<int> order(n_int);
    for (int i = 0; i < n_int; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (envs[x].H != envs[y].H) return envs[x].H > envs[y].H;
        return envs[x].W > envs[y].W;
    });
    std::vector<ItemRay> rays;
    std::vector<ItemPsf> tiles;
    const int spw = 1, tx = 32;
    build_items(envs, order, spw, tx, rays, tiles);

    // one staging block: envs | taps | ray items | psf items
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_env = 0;
    const size_t o_pool = align(o_env + sizeof(EnvDev) * envs.size());
    const size_t o_ray = align(o_pool + sizeof(float) * pool.size());
    const size_t o_psf = align(o_ray + sizeof(ItemRay) * rays.size());
    const size_t total = align(o_psf + sizeof(ItemPsf) * tiles.size());
    hipError_t e = c->staging.acquire(total);
    if (e != hipSuccess) return hip_fail(e, "pinned staging");
    char* h = (char*)c->staging.p;
    std::memcpy(h + o_env, envs.data(), sizeof(EnvDev) * envs.size());
    std::memcpy(h + o_pool, pool.data(), sizeof(float) * pool.size());
    std::memcpy(h + o_ray, rays.data(), sizeof(ItemRay) * rays.size());
    std::memcpy(h + o_psf, tiles.data(), sizeof(ItemPsf) * tiles.size());
    if ((e = c->params.ensure(total)) != hipSuccess) return hip_fail(e, "hipMalloc params");
    if ((e = c->fields.ensure(sizeof(float) * 3 * (size_t)scr)) != hipSuccess) return hip_fail(e, "hipMalloc scratch");
    if ((e = c->queue.ensure(sizeof(QueueDev))) != hipSuccess) return hip_fail(e, "hipMalloc queue");
    e = hipMemcpyAsync(c->params.p, h, total, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->staging.ev, c->stream);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");

    char* d = (char*)c->params.p;
    std::memset(&a, 0, sizeof(a));
    a.envs = (const EnvDev*)(d + o_env);
    a.vols = (const VolDev*)c->d_vols.p;
    a.table = (const TissueDev*)c->table.p;
    a.n_labels = c->n_labels;
    a.pair_rt = c->n_labels <= kPairLabels ? (const float2*)c->pair_rt.p : nullptr;
    a.q_lut = (const int32_t*)c->q_lut.p;
    a.ms_thr = (const int32_t*)c->ms_thr.p;
    a.coefs = (const float*)(d + o_pool);
    a.ray_items = (const ItemRay*)(d + o_ray);
    a.n_ray = (int32_t)rays.size();
    a.psf_items = (const ItemPsf*)(d + o_psf);
    a.n_psf = (int32_t)tiles.size();
    a.fR = (float*)c->fields.p;
    a.fT = a.fR + scr;
    a.fE = a.fT + scr;
    a.out = out;
    if (dbg) {
        a.dbg.label = dbg->label;
        a.dbg.voxel = dbg->voxel;
        a.dbg.philox = dbg->philox;
        a.dbg.energy = dbg->energy;
        a.dbg.intensity = dbg->intensity;
        a.dbg.scatter = dbg->scatter;
    }
    a.scanlines_per_wave = spw;
    a.max_rlat = max_rlat;
    a.multiscale = multiscale;
    a.any_ct = any_ct;
    info.tile_x = tx;
    info.max_pixels = max_px;
    return SG_OK;
}

// enqueue the two physics kernels of a staged call
sg_status launch_physics(sg_ctx* c, const PhysArgs& a, const StageInfo& info)
{
    QueueDev* q = (QueueDev*)c->queue.p;
    hipError_t e;
    if ((e = launch_queue_reset(q, 1, c->stream)) != hipSuccess) return hip_fail(e, "queue reset");
    if ((e = launch_ray(a, q, ray_grid(c->n_cu, a.multiscale != 0, ray_label_only(a), ray_debug(a)), c->stream)) != hipSuccess)
        return hip_fail(e, "ray kernel launch");
    if ((e = launch_psf(a, info.tile_x, psf_grid(info.tile_x, a.max_rlat, c->n_cu), c->stream)) != hipSuccess)
        return hip_fail(e, "PSF kernel launch");
    return SG_OK;
}

}  // namespace sg

extern "C" sg_status sg_simulate(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                                 const double* poses, float* out, const int64_t* out_offsets,
                                 const sg_debug_planes* dbg)
{
    if (!c) return fail(SG_EINVAL, "sg_simulate: NULL context");
    if (n < 0) return fail(SG_EINVAL, "sg_simulate: n_envs < 0");
    if (n == 0) return SG_OK;
    if (!vol_ids || !probes || !poses || !out || !out_offsets)
        return fail(SG_EINVAL, "sg_simulate: NULL argument");
    (void)hipSetDevice(c->device);
    PhysArgs a;
    StageInfo info;
    sg_status s = stage_physics(c, n, vol_ids, probes, poses, out, out_offsets, dbg, a, info);
    if (s != SG_OK) return s;
    return launch_physics(c, a, info);
}
