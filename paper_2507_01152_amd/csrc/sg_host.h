// Host-side state of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "sg_internal.h"
#include "sonosim.h"

namespace sg {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    hipError_t ensure(size_t bytes);   // grow-only; synchronises the device before a regrow
};

struct PinnedBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;           // recorded after the last upload from this buffer
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf();
    hipError_t acquire(size_t bytes);  // waits for the previous upload, then grows
};

struct HostVolume {
    VolDev dev{};
    uint8_t* bricks = nullptr;   // library-owned bricked label map (dev.labels); freed on release
    int32_t max_label = 0;
    bool live = false;
};

struct LaunchShape {
    int spw = 1;      // scanlines per wave in a ray item
    int tx = 32;      // PSF tile width (scanlines); tiles are 64 rows high
    int chunks = 1;   // env chunks: the PSF kernel of chunk k runs beside the ray kernel of chunk k + 1
};
constexpr int kMaxChunks = 4;

struct Plan {
    int32_t n_envs = 0;                // internal envs: one per image plane
    int32_t n_user = 0;                // caller envs (poses, volumes, probes, offsets)
    std::vector<int32_t> vol_ids;
    std::vector<sg_probe> probes;
    std::vector<int64_t> out_offsets;
    std::vector<EnvDev> envs;          // static parts
    std::vector<float> pool;
    std::vector<int> order;            // envs, longest scanlines first
    int64_t n_pixels = 0;
    int64_t n_scr = 0;                 // field-scratch elements per field (padded scanlines)
    int max_rax = 0, max_rlat = 0;
    int multiscale = 0;                // some env's volume has several noise scales
    int any_ct = 0;                    // some env's volume has a CT
    LaunchShape shape;
    int grid_ray = 0, grid_psf = 0, grid_psf_last = 0;   // (last: the last chunk's PSF kernel runs alone)
    DevBuf d_envs, d_pool, d_rays, d_tiles, d_poses, d_queue, fields;
    int32_t n_rays = 0, n_tiles = 0;
    // per chunk: ranges of the ray and PSF work lists (one queue each)
    int32_t ray_off[kMaxChunks] = {}, ray_cnt[kMaxChunks] = {}, tile_off[kMaxChunks] = {}, tile_cnt[kMaxChunks] = {};
    hipStream_t aux = nullptr;                      // second stream of the chunked pipeline
    hipEvent_t ev_ray[kMaxChunks] = {}, ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* graph_out = nullptr;        // output pointer the graph was captured with
    const void* cap_vols = nullptr;    // volume table the graph was captured with
    int32_t cap_labels = 0;            // tissue table size the graph was captured with
    ~Plan();
};

}  // namespace sg

namespace sg {
struct Surrogate;   // surrogate.cpp
struct SurrogateDeleter {
    void operator()(Surrogate* p) const;
};
struct Recon;       // recon.hip
struct ReconDeleter {
    void operator()(Recon* p) const;
};
}  // namespace sg

struct sg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 256;
    std::string arch;
    std::vector<sg::HostVolume> vols;
    bool vols_dirty = true;
    sg::DevBuf d_vols;
    sg::DevBuf table;
    sg::DevBuf pair_rt;   // (r, t) per label pair, when n_labels <= kPairLabels
    sg::DevBuf q_lut;     // quantised normal of the multi-scale gate (kNoiseQ int32, units of 2^-20)
    sg::DevBuf ms_thr;    // multi-scale gate thresholds, [SG_MAX_LABELS_DEV][kMaxNoiseScales] int32
    int32_t n_labels = 0;
    sg::DevBuf scan, params, fields, queue;
    sg::PinnedBuf staging;
    std::map<int32_t, std::unique_ptr<sg::Plan>> plans;
    int32_t next_plan = 1;
    std::map<int32_t, std::unique_ptr<sg::Surrogate, sg::SurrogateDeleter>> surrogates;
    int32_t next_surr = 1;
    std::map<int32_t, std::unique_ptr<sg::Recon, sg::ReconDeleter>> recons;
    int32_t next_recon = 1;
    sg::DevBuf op_wt, op_fine, op_parts;   // workspaces of the conv op entry points
};

namespace sg {

sg_status fail(sg_status code, const char* fmt, ...);
sg_status hip_fail(hipError_t e, const char* what);
constexpr int kPsfTapsMax = 2 * kMaxPsfRadius + 1;
int psf_taps_into(double sigma, float* out);   // no allocation
sg_status check_probe(const sg_probe& p, int idx);
// static parameters of plane `plane` of caller env idx (frame at out_off + plane * W * H)
sg_status fill_env_static(const sg_probe& p, int32_t vol, int idx, int plane, int64_t out_off, int64_t scr_off,
                          std::vector<float>& pool, EnvDev& e);
// the same without allocation: taps appended to pool[*pool_used ..) within pool_cap floats
// (SG_ERANGE when full), e.kax / e.klat as offsets into pool
sg_status fill_env_static_into(const sg_probe& p, int32_t vol, int idx, int plane, int64_t out_off, int64_t scr_off,
                               float* pool, int64_t pool_cap, int64_t* pool_used, EnvDev& e);
int probe_planes(const sg_probe& p);                 // image planes of a probe (>= 1)
double plane_elevation(const sg_probe& p, int j);   // elevation b of plane j, mm
void build_items(const std::vector<EnvDev>& envs, const std::vector<int>& order, int spw, int tx,
                 std::vector<ItemRay>& rays, std::vector<ItemPsf>& tiles);
sg_status sync_volumes(sg_ctx* c);
// entry point without allocation (noalloc.hip): its device scratch and limits
constexpr size_t kNoAllocBytes = SG_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocMaxPlanes = SG_NOALLOC_MAX_PLANES;
hipError_t noalloc_init(int device);   // with `device` current; once per device (later calls return at once)

struct StageInfo {
    int tile_x = 32;
    int max_pixels = 0;
};
sg_status stage_physics(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes, const double* poses,
                        float* out, const int64_t* out_offsets, const sg_debug_planes* dbg, PhysArgs& a,
                        StageInfo& info);
sg_status launch_physics(sg_ctx* c, const PhysArgs& a, const StageInfo& info);
sg_status check_envs(sg_ctx* c, int32_t n, const int32_t* vol_ids, const sg_probe* probes);
void surrogate_release_all(sg_ctx* c);
void recon_release_all(sg_ctx* c);

}  // namespace sg
