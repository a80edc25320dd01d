// Batched persistent path: plans, HIP graph capture/replay and the
// launch-shape autotuner (C ABI in include/sonosim.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "sg_host.h"

namespace sg {

Plan::~Plan()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t& ev : ev_ray)
        if (ev) (void)hipEventDestroy(ev);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
}

namespace {

// Candidate launch shapes: every one yields bit-identical frames (the
// per-pixel arithmetic and summation order do not depend on the tiling or on
// the chunking).  With chunks > 1 the envs are split into that many groups of
// about equal pixel count; the PSF kernel of a group runs on a second stream
// beside the ray kernel of the next group (the ray kernel is bound by the
// VALU, the PSF kernel by memory), each kernel on part of the GPU.
const LaunchShape kShapes[] = {
    {1, 32, 1}, {2, 32, 1}, {1, 64, 1}, {2, 64, 1}, {1, 16, 1}, {4, 32, 1}, {4, 64, 1},
    {2, 32, 2}, {2, 64, 2}, {2, 32, 4}, {2, 64, 4},
};

Plan* find_plan(sg_ctx* c, int32_t id)
{
    auto it = c->plans.find(id);
    return it == c->plans.end() ? nullptr : it->second.get();
}

void drop_graph(Plan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->graph_out = nullptr;
}

sg_status apply_shape(sg_ctx* c, Plan* p, const LaunchShape& s)
{
    if (s.chunks < 1 || s.chunks > kMaxChunks) return fail(SG_EINVAL, "launch shape: %d chunks", s.chunks);
    // contiguous groups of the longest-first order with about equal pixel counts
    std::vector<ItemRay> rays;
    std::vector<ItemPsf> tiles;
    const int K = std::min<int>(s.chunks, p->n_envs);
    size_t gi = 0;
    int64_t acc = 0;
    for (int k = 0; k < kMaxChunks; ++k) p->ray_off[k] = p->ray_cnt[k] = p->tile_off[k] = p->tile_cnt[k] = 0;
    for (int k = 0; k < K; ++k) {
        std::vector<int> part;
        const int64_t goal = p->n_pixels * (k + 1) / K;
        while (gi < p->order.size() && (k == K - 1 || acc < goal || part.empty()) &&
               (int)(p->order.size() - gi) > K - 1 - k) {
            const EnvDev& e = p->envs[p->order[gi]];
            acc += (int64_t)e.W * e.H;
            part.push_back(p->order[gi++]);
            if (k < K - 1 && acc >= goal) break;
        }
        std::vector<ItemRay> r;
        std::vector<ItemPsf> t;
        build_items(p->envs, part, s.spw, s.tx, r, t);
        p->ray_off[k] = (int32_t)rays.size();
        p->ray_cnt[k] = (int32_t)r.size();
        p->tile_off[k] = (int32_t)tiles.size();
        p->tile_cnt[k] = (int32_t)t.size();
        rays.insert(rays.end(), r.begin(), r.end());
        tiles.insert(tiles.end(), t.begin(), t.end());
    }
    // occupancy only: a persistent grid's surplus blocks find the work counter spent and exit
    int gr = ray_grid(c->n_cu, p->multiscale != 0, c->n_labels <= kPairLabels && !p->any_ct, false),
        gp = psf_grid(s.tx, p->max_rlat, c->n_cu);
    if (gr < 1 || gp < 1) return fail(SG_EINVAL, "launch shape (tile %d) does not fit a compute unit", s.tx);
    p->grid_psf_last = gp;
    if (K > 1) {   // leave room on every CU for one PSF block beside the ray blocks
        const int rb = gr / c->n_cu;
        gr = std::max(1, rb - 1) * c->n_cu;
        gp = c->n_cu;
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && K > 1 && !p->aux) e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
    for (int k = 0; k < K && e == hipSuccess; ++k)
        if (!p->ev_ray[k]) e = hipEventCreateWithFlags(&p->ev_ray[k], hipEventDisableTiming);
    if (e == hipSuccess && K > 1 && !p->ev_join) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = p->d_rays.ensure(sizeof(ItemRay) * std::max<size_t>(rays.size(), 1));
    if (e == hipSuccess) e = p->d_tiles.ensure(sizeof(ItemPsf) * std::max<size_t>(tiles.size(), 1));
    if (e == hipSuccess && !rays.empty())
        e = hipMemcpy(p->d_rays.p, rays.data(), sizeof(ItemRay) * rays.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(p->d_tiles.p, tiles.data(), sizeof(ItemPsf) * tiles.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "work list upload");
    p->n_rays = (int32_t)rays.size();
    p->n_tiles = (int32_t)tiles.size();
    p->shape = s;
    p->shape.chunks = K;
    p->grid_ray = gr;
    p->grid_psf = gp;
    drop_graph(p);
    return SG_OK;
}

PhysArgs plan_args(sg_ctx* c, Plan* p, float* out)
{
    PhysArgs a;
    std::memset(&a, 0, sizeof(a));
    a.envs = (const EnvDev*)p->d_envs.p;
    a.vols = (const VolDev*)c->d_vols.p;
    a.table = (const TissueDev*)c->table.p;
    a.n_labels = c->n_labels;
    a.pair_rt = c->n_labels <= kPairLabels ? (const float2*)c->pair_rt.p : nullptr;
    a.q_lut = (const int32_t*)c->q_lut.p;
    a.ms_thr = (const int32_t*)c->ms_thr.p;
    a.coefs = (const float*)p->d_pool.p;
    a.ray_items = (const ItemRay*)p->d_rays.p;
    a.n_ray = p->n_rays;
    a.psf_items = (const ItemPsf*)p->d_tiles.p;
    a.n_psf = p->n_tiles;
    a.fR = (float*)p->fields.p;
    a.fT = a.fR + p->n_scr;
    a.fE = a.fT + p->n_scr;
    a.out = out;
    a.scanlines_per_wave = p->shape.spw;
    a.max_rlat = p->max_rlat;
    a.multiscale = p->multiscale;
    a.any_ct = p->any_ct;
    a.poses = (const double*)p->d_poses.p;   // the ray kernel computes the planes of the current poses
    a.geo_out = (EnvDev*)p->d_envs.p;
    a.ray_queue = (QueueDev*)p->d_queue.p;
    return a;
}

// enqueue one step's kernels (persistent ray kernel, which also computes the
// planes of the current poses, then persistent PSF kernel, which clears the
// ray kernel's work counter for the next step) on stream s; optional events:
// before the first ray kernel, after the last ray kernel, at the end of the
// step.  With chunks, chunk k's PSF kernel waits for its ray kernel on the
// plan's second stream, which the step joins at the end (the same code is
// captured).  Every chunk holds at least one env, so each ray kernel is
// followed by a PSF kernel that clears its counter.
hipError_t enqueue_step(sg_ctx* c, Plan* p, float* out, hipStream_t s, hipEvent_t* ev = nullptr)
{
    QueueDev* q = (QueueDev*)p->d_queue.p;
    const int K = p->shape.chunks;
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[0], s);
    if (K == 1) {
        const PhysArgs a = plan_args(c, p, out);
        if (e == hipSuccess) e = launch_ray(a, q, p->grid_ray, s);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = launch_psf(a, p->shape.tx, p->grid_psf, s);
        if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
        return e;
    }
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        PhysArgs a = plan_args(c, p, out);
        a.ray_items += p->ray_off[k];
        a.n_ray = p->ray_cnt[k];
        a.psf_items += p->tile_off[k];
        a.n_psf = p->tile_cnt[k];
        a.ray_queue = q + k;
        e = launch_ray(a, q + k, p->grid_ray, s);
        if (e == hipSuccess) e = hipEventRecord(p->ev_ray[k], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->aux, p->ev_ray[k], 0);
        if (e == hipSuccess) e = launch_psf(a, p->shape.tx, k == K - 1 ? p->grid_psf_last : p->grid_psf, p->aux);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventRecord(p->ev_join, p->aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_join, 0);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
    return e;
}

sg_status capture(sg_ctx* c, Plan* p, float* out)
{
    drop_graph(p);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = enqueue_step(c, p, out, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) {
            p->graph = g;
            e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        drop_graph(p);
        return hip_fail(e, "graph capture");
    }
    p->graph_out = out;
    p->cap_vols = c->d_vols.p;
    p->cap_labels = c->n_labels;
    return SG_OK;
}

std::string tune_key(sg_ctx* c, Plan* p)
{
    int maxW = 0, maxH = 0;
    for (auto& pr : p->probes) {
        maxW = std::max(maxW, pr.W);
        maxH = std::max(maxH, pr.H);
    }
    // the ray kernel's instantiation (noise scales, CT, label-pair table)
    // changes its occupancy, so it is part of the key
    const int pairs = c->n_labels <= kPairLabels ? 1 : 0;
    std::ostringstream k;
    k << c->arch << "|n" << p->n_envs << "|px" << p->n_pixels << "|W" << maxW << "|H" << maxH << "|ra"
      << p->max_rax << "|rl" << p->max_rlat << "|ms" << p->multiscale << "|ct" << p->any_ct << "|lp" << pairs;
    return k.str();
}

bool cache_lookup(const char* path, const std::string& key, LaunchShape* s)
{
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const std::string tag = "\"key\": \"" + key + "\"";
        if (line.find(tag) == std::string::npos) continue;
        int spw = 0, tx = 0, ty = 0, ch = 0;
        const char* q = std::strstr(line.c_str(), "\"spw\":");
        const char* x = std::strstr(line.c_str(), "\"tx\":");
        const char* y = std::strstr(line.c_str(), "\"ty\":");
        const char* z = std::strstr(line.c_str(), "\"chunks\":");
        if (q && x && y && z && std::sscanf(q, "\"spw\": %d", &spw) == 1 && std::sscanf(x, "\"tx\": %d", &tx) == 1 &&
            std::sscanf(y, "\"ty\": %d", &ty) == 1 && std::sscanf(z, "\"chunks\": %d", &ch) == 1) {
            for (const LaunchShape& k : kShapes)
                if (k.spw == spw && k.tx == tx && k.chunks == ch && ty == 64) {
                    *s = k;
                    found = true;   // keep the last matching line
                }
        }
    }
    return found;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_batch_plan_create(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes,
                                          const int64_t* out_offsets, int32_t* plan_id)
{
    if (!c || !vol_ids || !probes || !out_offsets || !plan_id)
        return fail(SG_EINVAL, "sg_batch_plan_create: NULL argument");
    if (n < 1) return fail(SG_EINVAL, "sg_batch_plan_create: n_envs must be >= 1");
    (void)hipSetDevice(c->device);
    sg_status s = check_envs(c, n, vol_ids, probes);
    if (s != SG_OK) return s;
    std::unique_ptr<Plan> p(new Plan());
    p->n_user = n;
    p->vol_ids.assign(vol_ids, vol_ids + n);
    p->probes.assign(probes, probes + n);
    p->out_offsets.assign(out_offsets, out_offsets + n);
    for (int i = 0; i < n; ++i) {   // one internal env per image plane
        if (out_offsets[i] < 0) return fail(SG_EINVAL, "env %d: negative output offset", i);
        for (int j = 0; j < probe_planes(probes[i]); ++j) {
            EnvDev ed;
            s = fill_env_static(probes[i], vol_ids[i], i, j, out_offsets[i], p->n_scr, p->pool, ed);
            if (s != SG_OK) return s;
            p->n_pixels += (int64_t)probes[i].W * probes[i].H;
            p->n_scr += (int64_t)probes[i].W * ed.ld;
            p->max_rax = std::max(p->max_rax, ed.rax);
            p->max_rlat = std::max(p->max_rlat, ed.rlat);
            p->envs.push_back(ed);
        }
        p->multiscale |= c->vols[vol_ids[i]].dev.scales > 1;
        p->any_ct |= c->vols[vol_ids[i]].dev.ct != nullptr;
    }
    p->n_envs = (int32_t)p->envs.size();
    const int ni = p->n_envs;
    // longest scanlines first (ray items cost ~H), then wider frames
    p->order.resize(ni);
    for (int i = 0; i < ni; ++i) p->order[i] = i;
    std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) {
        if (p->envs[a].H != p->envs[b].H) return p->envs[a].H > p->envs[b].H;
        return p->envs[a].W > p->envs[b].W;
    });
    hipError_t e = p->d_envs.ensure(sizeof(EnvDev) * ni);
    if (e == hipSuccess) e = p->d_pool.ensure(sizeof(float) * p->pool.size());
    if (e == hipSuccess) e = p->d_poses.ensure(sizeof(double) * 12 * n);
    if (e == hipSuccess) e = p->d_queue.ensure(sizeof(QueueDev) * kMaxChunks);
    if (e == hipSuccess) e = p->fields.ensure(sizeof(float) * 3 * (size_t)p->n_scr);
    if (e != hipSuccess) return hip_fail(e, "plan allocation");
    e = hipMemcpy(p->d_envs.p, p->envs.data(), sizeof(EnvDev) * ni, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_pool.p, p->pool.data(), sizeof(float) * p->pool.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->d_poses.p, 0, sizeof(double) * 12 * n);
    if (e == hipSuccess) e = hipMemset(p->d_queue.p, 0, sizeof(QueueDev) * kMaxChunks);   // steps leave them at 0
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    s = apply_shape(c, p.get(), kShapes[0]);
    if (s != SG_OK) return s;
    const int32_t id = c->next_plan++;
    c->plans[id] = std::move(p);
    *plan_id = id;
    return SG_OK;
}

extern "C" sg_status sg_batch_poses(sg_ctx* c, int32_t id, double** dev_poses)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p || !dev_poses) return fail(SG_EINVAL, "sg_batch_poses: bad plan id or NULL");
    *dev_poses = (double*)p->d_poses.p;
    return SG_OK;
}

extern "C" sg_status sg_batch_set_poses(sg_ctx* c, int32_t id, const double* host_poses)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p || !host_poses) return fail(SG_EINVAL, "sg_batch_set_poses: bad plan id or NULL");
    (void)hipSetDevice(c->device);
    const size_t bytes = sizeof(double) * 12 * (size_t)p->n_user;
    hipError_t e = c->staging.acquire(bytes);
    if (e != hipSuccess) return hip_fail(e, "pinned staging");
    std::memcpy(c->staging.p, host_poses, bytes);
    e = hipMemcpyAsync(p->d_poses.p, c->staging.p, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->staging.ev, c->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, "pose upload");
}

static sg_status step_checks(sg_ctx* c, Plan* p)
{
    if (c->n_labels < 1) return fail(SG_ESTATE, "no tissue table set");
    for (int i = 0; i < p->n_user; ++i) {
        const HostVolume& v = c->vols[p->vol_ids[i]];
        if (!v.live) return fail(SG_ESTATE, "env %d: volume %d was released", i, p->vol_ids[i]);
        if (v.max_label >= c->n_labels) return fail(SG_EINVAL, "env %d: label outside the table", i);
    }
    return sync_volumes(c);
}

extern "C" sg_status sg_batch_step_profiled(sg_ctx* c, int32_t id, float* out, float* ms_ray, float* ms_psf)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p || !out || !ms_ray || !ms_psf) return fail(SG_EINVAL, "sg_batch_step_profiled: bad plan id or NULL");
    (void)hipSetDevice(c->device);
    sg_status s = step_checks(c, p);
    if (s != SG_OK) return s;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    if (e == hipSuccess) {
        e = enqueue_step(c, p, out, c->stream, ev);
        // a step cut short may leave a ray counter that no PSF kernel cleared
        if (e != hipSuccess) (void)launch_queue_reset((QueueDev*)p->d_queue.p, kMaxChunks, c->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_ray, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_psf, ev[1], ev[2]);
    for (int i = 0; i < 3; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    return e == hipSuccess ? SG_OK : hip_fail(e, "profiled step");
}

extern "C" sg_status sg_batch_step(sg_ctx* c, int32_t id, float* out)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p || !out) return fail(SG_EINVAL, "sg_batch_step: bad plan id or NULL output");
    (void)hipSetDevice(c->device);
    sg_status s = step_checks(c, p);
    if (s != SG_OK) return s;
    if (!p->exec || p->graph_out != out || p->cap_vols != c->d_vols.p || p->cap_labels != c->n_labels) {
        s = capture(c, p, out);
        if (s != SG_OK) return s;
    }
    hipError_t e = hipGraphLaunch(p->exec, c->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, "hipGraphLaunch");
}

extern "C" sg_status sg_batch_status(sg_ctx* c, int32_t id, int32_t* n_bad)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p || !n_bad) return fail(SG_EINVAL, "sg_batch_status: bad plan id or NULL");
    (void)hipSetDevice(c->device);
    // the step's ray kernel flags every plane of a rejected pose; count caller envs (plane 0)
    std::vector<EnvDev> envs(p->n_envs);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(envs.data(), p->d_envs.p, sizeof(EnvDev) * envs.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status readback");
    int32_t bad = 0;
    for (const EnvDev& d : envs) bad += (!d.valid && d.plane == 0) ? 1 : 0;
    *n_bad = bad;
    return SG_OK;
}

extern "C" sg_status sg_batch_config(sg_ctx* c, int32_t id, int32_t* spw, int32_t* tx, int32_t* ty, int32_t* chunks)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p) return fail(SG_EINVAL, "sg_batch_config: bad plan id");
    if (spw) *spw = p->shape.spw * kRayWaves;
    if (tx) *tx = p->shape.tx;
    if (ty) *ty = 64;
    if (chunks) *chunks = p->shape.chunks;
    return SG_OK;
}

extern "C" sg_status sg_batch_set_config(sg_ctx* c, int32_t id, int32_t scanlines_per_item, int32_t tile_x,
                                         int32_t chunks)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p) return fail(SG_EINVAL, "sg_batch_set_config: bad plan id");
    if ((scanlines_per_item != 4 && scanlines_per_item != 8 && scanlines_per_item != 16) ||
        (tile_x != 16 && tile_x != 32 && tile_x != 64) || chunks < 1 || chunks > kMaxChunks)
        return fail(SG_EINVAL, "sg_batch_set_config: scanlines_per_item in {4, 8, 16}, tile_x in {16, 32, 64}, "
                               "chunks in [1, %d]", kMaxChunks);
    (void)hipSetDevice(c->device);
    LaunchShape s;
    s.spw = scanlines_per_item / kRayWaves;
    s.tx = tile_x;
    s.chunks = chunks;
    return apply_shape(c, p, s);
}

extern "C" sg_status sg_autotune(sg_ctx* c, int32_t id, const char* cache_path)
{
    Plan* p = c ? find_plan(c, id) : nullptr;
    if (!p) return fail(SG_EINVAL, "sg_autotune: bad plan id");
    (void)hipSetDevice(c->device);
    if (c->n_labels < 1) return fail(SG_ESTATE, "no tissue table set");
    sg_status s = sync_volumes(c);
    if (s != SG_OK) return s;
    const std::string key = tune_key(c, p);
    LaunchShape cached;
    if (cache_lookup(cache_path, key, &cached)) return apply_shape(c, p, cached);

    DevBuf scratch_out;
    hipError_t e = scratch_out.ensure(sizeof(float) * (size_t)p->n_pixels);
    if (e != hipSuccess) return hip_fail(e, "autotune output");
    // the plan's offsets may address a larger caller buffer: time into a
    // private buffer laid out densely with the same sizes.  The plan's own
    // records (p->envs) are never changed; the device copy is restored from
    // them on every exit after the dense upload.
    std::vector<EnvDev> dense = p->envs;
    int64_t off = 0;
    for (int i = 0; i < p->n_envs; ++i) {
        dense[i].out_off = off;
        off += (int64_t)dense[i].W * dense[i].H;
    }
    auto restore = [&]() -> hipError_t {
        drop_graph(p);   // captured with the dense offsets and the private buffer
        return hipMemcpy(p->d_envs.p, p->envs.data(), sizeof(EnvDev) * p->n_envs, hipMemcpyHostToDevice);
    };
    e = hipMemcpy(p->d_envs.p, dense.data(), sizeof(EnvDev) * p->n_envs, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)restore();
        return hip_fail(e, "autotune env upload");
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    LaunchShape best = p->shape;
    float best_us = 1e30f;
    for (const LaunchShape& shp : kShapes) {
        if (apply_shape(c, p, shp) != SG_OK) continue;
        if (capture(c, p, (float*)scratch_out.p) != SG_OK) continue;
        for (int w = 0; w < 3; ++w) (void)hipGraphLaunch(p->exec, c->stream);
        const int reps = 10;
        (void)hipEventRecord(t0, c->stream);
        for (int r = 0; r < reps; ++r) (void)hipGraphLaunch(p->exec, c->stream);
        (void)hipEventRecord(t1, c->stream);
        if (hipEventSynchronize(t1) != hipSuccess) continue;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        const float us = 1000.f * ms / reps;
        if (us < best_us) {
            best_us = us;
            best = shp;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    e = restore();
    if (e != hipSuccess) return hip_fail(e, "autotune env restore");
    s = apply_shape(c, p, best);
    if (s != SG_OK) return s;
    if (cache_path && best_us < 1e29f) {
        std::ofstream f(cache_path, std::ios::app);
        if (f)
            f << "{\"key\": \"" << key << "\", \"spw\": " << best.spw << ", \"tx\": " << best.tx
              << ", \"ty\": 64, \"chunks\": " << best.chunks << ", \"us\": " << best_us << "}\n";
    }
    return SG_OK;
}

extern "C" sg_status sg_batch_plan_destroy(sg_ctx* c, int32_t id)
{
    if (!c || !find_plan(c, id)) return fail(SG_EINVAL, "sg_batch_plan_destroy: bad plan id");
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->plans.erase(id);
    return SG_OK;
}
