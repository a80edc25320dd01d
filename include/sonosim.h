/*
 * sonosim.h -- C ABI of the MI355X (gfx950) batched ultrasound simulator.
 *
 * The problem follows SonoGym (arXiv 2507.01152), Sec. 4 "Ultrasound
 * simulation" and App. B.2: a 3D label map (optionally with a CT volume) and a
 * probe pose go in, a B-mode frame comes out, batched across parallel
 * environments.  The model-based image is I = R + B with
 *   R = PSF (x) (G * |E * cos(theta) * r|)      reflection at label boundaries,
 *   B = E * (PSF (x) T)                          backscatter of the scattering
 *                                                pattern T (per-voxel noise),
 *   E = E0 * prod(t) * exp(-f * integral alpha)  remaining energy,
 * followed by log compression to a display frame Y in [0, 1].
 *
 * Conventions (all entry points):
 *  - Every call returns an sg_status; SG_OK is 0, errors are negative and a
 *    human-readable message is available from sg_last_error() (thread-local,
 *    valid until the next failing call on the same thread).  No C++
 *    exception crosses this boundary.
 *  - "device" pointers are HIP device memory of the context's device; "host"
 *    pointers are ordinary CPU memory.  The caller owns every buffer it passes
 *    in (volumes, outputs, offsets) and must keep device buffers alive until
 *    the work that uses them has completed on the context's stream.  The
 *    library owns only its workspaces, plans, graphs and plan pose buffers.
 *  - Work is enqueued asynchronously on the context's stream unless stated.
 *  - Contexts are not thread-safe; use one context per thread or stream.
 *  - Image layout: a frame is [H][W] row-major FP32 (row = depth sample y,
 *    column = scanline x); several frames are packed into one buffer at
 *    caller-given offsets (in elements).
 */
#ifndef SONOSIM_H
#define SONOSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_ctx sg_ctx;
typedef int32_t sg_status;

#define SG_OK 0
#define SG_EINVAL (-1)  /* bad argument: size, id, NULL, NaN pose, label >= table size */
#define SG_ENOMEM (-2)  /* device or host allocation failed */
#define SG_EHIP (-3)    /* a HIP runtime call failed */
#define SG_ESTATE (-4)  /* call not valid in the current state (e.g. no tissue table) */
#define SG_ERANGE (-5)  /* a pose puts the image plane outside the fixed-point range */

/* Limits. */
#define SG_MAX_IMAGE 1024   /* W and H must lie in [1, SG_MAX_IMAGE] */
#define SG_MAX_LABELS 256

/* Message of the last failing call on this thread ("" if none). */
const char* sg_last_error(void);

/* ABI version (major * 100 + minor). */
int32_t sg_version(void);

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a
 * hipStream_t owned by the caller; NULL = the device's null stream).
 * *out receives the context.  Errors: SG_EINVAL, SG_EHIP, SG_ENOMEM. */
sg_status sg_create(sg_ctx** out, int32_t device, void* hip_stream);

/* Destroy a context and free its workspaces, plans and graphs.  Waits for
 * the context's stream.  NULL is accepted. */
sg_status sg_destroy(sg_ctx* ctx);

/* Change the stream later work is enqueued on. */
sg_status sg_set_stream(sg_ctx* ctx, void* hip_stream);

/* Block until all work enqueued by the context has completed. */
sg_status sg_synchronize(sg_ctx* ctx);

/* ------------------------------------------------------------------------
 * Volumes (Sec. 4 "Assets": CT volumes and label maps of patients).
 */
typedef struct {
    int32_t nx, ny, nz;        /* voxels; nx*ny*nz < 2^31 */
    double spacing_mm[3];      /* voxel spacing along x, y, z (> 0) */
    const uint8_t* labels;     /* device, [nz][ny][nx] (x fastest), caller-owned;
                                  read during sg_volume_register only */
    const int16_t* ct_hu;      /* device, same layout, HU; or NULL (then Z comes
                                  from the tissue table) */
    uint64_t noise_seed;       /* key of the fixed per-voxel noise fields
                                  N0, N1 (App. B.2: sampled once over 3D space) */
    int32_t noise_scales;      /* S in [0, 4]; 0 or 1: one sample per voxel.
                                  S > 1 adds coarser scales (App. B.2, multi-scale
                                  N0 and N1): scale s draws on cells of 2^s voxels
                                  per axis (Philox counter (cell, 0, s, 0)),
                                  N0 = sum_s N0_s / sqrt(S), and the density gate
                                  N1 = sum_s N1_s / sqrt(S) <= mu1 with N1_s =
                                  Q[w2_s >> 20] 2^-20 is the exact integer test
                                  sum_s Q[w2_s >> 20] <= floor(sqrt(S) mu1 2^20)
                                  (threshold rounded in FP64 on the host),
                                  Q = the table of sg_noise_quantiles. */
} sg_volume_desc;

/* Register a volume; *vol_id receives its id.  Scans the label map once on
 * the device to record its largest label, and copies it into a library-owned
 * layout of 8 x 4 x 4-voxel bricks (one 128-byte cache line each, so gathers
 * along a beam touch few lines); synchronises the stream.  The caller's label
 * buffer may be reused or freed after the call; the CT volume (ct_hu) is
 * referenced, not copied, and must stay valid while the volume is registered.
 * Errors: SG_EINVAL (also when the bricked map would need 2^24 bricks or
 * more), SG_ENOMEM / SG_EHIP. */
sg_status sg_volume_register(sg_ctx* ctx, const sg_volume_desc* desc, int32_t* vol_id);

/* Forget a registered volume: waits for the context stream, then frees the
 * library's bricked label map (the CT memory stays the caller's). */
sg_status sg_volume_release(sg_ctx* ctx, int32_t vol_id);

/* The quantised standard normal of the multi-scale density gate (host, no
 * context), in units of 2^-20: out[k] = rint(Phi^-1((k + 1/2) / 4096) 2^20)
 * for k < 4096 (half to even), with Phi^-1 solved to FP64 precision from
 * erfc.  out: host, 4096 int32.  Errors: SG_EINVAL (NULL). */
sg_status sg_noise_quantiles(int32_t* out);

/* ------------------------------------------------------------------------
 * Tissue table (App. B.2: per-tissue impedance Z, attenuation alpha and the
 * scattering parameters mu0, sigma0, mu1).  Row l describes label l.
 *   Z_mrayl          >= 0; 0 = pressure-release, +INF = rigid (both reflect
 *                    totally).  Ignored for volumes with a CT volume, where Z is
 *                    proportional to max(HU + 1000, 0).
 *   alpha_np_cm_mhz  attenuation, Np / cm / MHz (>= 0)
 *   mu0, sigma0      scatterer amplitude: T~ = N0 * sigma0 + mu0
 *   mu1              scatterer density: T = T~ where N1 <= mu1, else 0
 *                    (-INF: never, +INF: always)
 * `rows` is a host array of n_labels rows, copied.  Errors: SG_EINVAL.
 */
typedef struct {
    float Z_mrayl;
    float alpha_np_cm_mhz;
    float mu0;
    float sigma0;
    float mu1;
} sg_tissue;

sg_status sg_tissue_table_set(sg_ctx* ctx, const sg_tissue* rows, int32_t n_labels);

/* ------------------------------------------------------------------------
 * Probe / image geometry of one environment (linear probe; App. C.1 uses
 * 0.5 mm pixels).  Pixel (x, y) lies at probe-frame point
 * (a + x*dx_mm, b, y*dy_mm) with a = -0.5*(W-1)*dx_mm: x runs along the
 * probe's lateral axis, y along the beam (probe z), b along the elevation
 * (probe y).
 *   W, H      scanlines and depth samples, each in [1, SG_MAX_IMAGE]
 *   f_mhz     centre frequency (attenuation scales with f)
 *   E0        initial energy (> 0)
 *   psf_frac  PSF standard deviation as a fraction of the image size per
 *             axis (App. B.2: about 1 %), > 0
 *   dr_db     display dynamic range in dB (> 0)
 *   n_elev    planes of a volumetric probe (Sec. 4, surgery task: H x W x E
 *             images, App. C: 50 x 37 x 5 at 2 x 2 x 10 mm); 0 or 1: one
 *             plane, at most SG_MAX_ELEV.  Plane j lies at
 *             b = (j - (n_elev - 1) / 2) * elev_mm and is simulated as its own
 *             2D image; the env's output is [n_elev][H][W] at its offset.
 *   elev_mm   plane spacing (> 0 when n_elev > 1)
 */
#define SG_MAX_ELEV 64

typedef struct {
    int32_t W, H;
    double dx_mm, dy_mm, f_mhz, E0, psf_frac, dr_db;
    int32_t n_elev;
    double elev_mm;
} sg_probe;

/* Optional per-pixel outputs for checking (device pointers, each may be NULL;
 * packed like the frames at the same offsets, philox with 4 words per pixel
 * at 4*offset).  Writing them costs extra memory traffic. */
typedef struct {
    uint8_t* label;       /* nearest label (0 outside the volume) */
    int32_t* voxel;       /* linear voxel index (z*ny + y)*nx + x, -1 outside */
    uint32_t* philox;     /* Philox4x32-10 words of that voxel (0 outside) */
    float* energy;        /* remaining energy E */
    float* intensity;     /* I before log compression */
    float* scatter;       /* scattering pattern T (0 where the gate fails) */
} sg_debug_planes;

/* Simulate n_envs environments (Sec. 4 "Ultrasound simulation" pipeline:
 * pose -> image plane -> label/CT slice -> model-based image -> display).
 *   vol_ids      host, n_envs registered volume ids
 *   probes       host, n_envs probe descriptions
 *   poses        host, n_envs * 12 doubles: row-major 3x4 [R | t] mapping
 *                probe-frame mm to volume mm (volume origin at the centre of
 *                voxel (0,0,0), axes along the array indices)
 *   out          device, FP32 display frames Y in [0, 1]
 *   out_offsets  host, n_envs element offsets of each [H][W] frame in out
 *   debug        host struct of optional device planes, or NULL
 * Errors: SG_EINVAL (ids, sizes, NaN pose, a volume label >= table size),
 * SG_ERANGE (plane outside +-2^30 / 2^16 voxels), SG_ESTATE (no table),
 * SG_EHIP, SG_ENOMEM.
 */
sg_status sg_simulate(sg_ctx* ctx, int32_t n_envs, const int32_t* vol_ids,
                      const sg_probe* probes, const double* poses, float* out,
                      const int64_t* out_offsets, const sg_debug_planes* debug);

/* sg_simulate for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and frames (bit for bit), without debug planes, but it allocates
 * nothing -- no hipMalloc / hipFree / pinned or other allocating call.  The
 * per-plane records, PSF taps, work lists, work counter and the FP32 field
 * planes between the two kernels live in a file-scope device array of
 * SG_NOALLOC_SCRATCH_BYTES on each GPU, set up by sg_create and held until
 * the process ends; the records are staged in a static host array.  Each
 * call reuses its GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (e.g. on two streams) race; on one stream they are
 * ordered.  A call waits (host) until the previous call's record upload has
 * been read.  Limits: at most SG_NOALLOC_MAX_PLANES image planes (envs times
 * their planes) and 12 bytes per field pixel (scanlines padded to 32 rows)
 * within the array, e.g. 64 envs of 256 x 256.  Arguments as sg_simulate.
 * Errors: as sg_simulate; SG_ERANGE beyond the limits (nothing is enqueued). */
#define SG_NOALLOC_SCRATCH_BYTES (64u << 20)
#define SG_NOALLOC_MAX_PLANES 256
sg_status sg_simulate_noalloc(sg_ctx* ctx, int32_t n_envs, const int32_t* vol_ids, const sg_probe* probes,
                              const double* poses, float* out, const int64_t* out_offsets);

/* ------------------------------------------------------------------------
 * Batched persistent path (environments stepped in batch mode, Sec. 4):
 * a plan fixes the environments' volumes, probes and output offsets; each
 * step replays one captured HIP graph: a persistent ray kernel pulling
 * (environment, scanline group) items longest-first from a device queue,
 * each item computing its plane from the device pose, then a persistent PSF
 * kernel striding over (environment, tile) items.  Poses
 * live in a library-owned device buffer that the caller updates between
 * steps (for instance from its own kernels on the same stream).
 */

/* Create a plan.  Host arrays are copied.  *plan_id receives the id. */
sg_status sg_batch_plan_create(sg_ctx* ctx, int32_t n_envs, const int32_t* vol_ids,
                               const sg_probe* probes, const int64_t* out_offsets,
                               int32_t* plan_id);

/* Device pointer of the plan's pose buffer (n_envs * 12 doubles, layout as in
 * sg_simulate), owned by the library, valid until the plan is destroyed. */
sg_status sg_batch_poses(sg_ctx* ctx, int32_t plan_id, double** dev_poses);

/* Copy n_envs * 12 host doubles into the plan's pose buffer (asynchronous
 * on the context's stream; the host array may be reused on return). */
sg_status sg_batch_set_poses(sg_ctx* ctx, int32_t plan_id, const double* host_poses);

/* Enqueue one step: geometry from the device poses, then all environments'
 * frames into `out` (device; same offsets as the plan).  The first call (and
 * any call with a different `out` or after sg_autotune) captures the graph.
 * A pose whose plane leaves the fixed-point range produces a zero frame for
 * that environment and is reported by sg_batch_status. */
sg_status sg_batch_step(sg_ctx* ctx, int32_t plan_id, float* out);

/* Synchronise and report how many environments of the last step had a pose
 * outside the fixed-point range (or non-finite): *n_bad (host). */
sg_status sg_batch_status(sg_ctx* ctx, int32_t plan_id, int32_t* n_bad);

/* Time the candidate launch shapes for the plan on the device and keep the
 * fastest; results are cached by (device, shape bucket) in the JSON file at
 * `cache_path` (NULL: no file).  Synchronises; the poses currently in the
 * plan's buffer are used.  Output-equivalent: every candidate produces
 * bit-identical frames. */
sg_status sg_autotune(sg_ctx* ctx, int32_t plan_id, const char* cache_path);

/* Run one step without the graph, timing its persistent kernels with HIP
 * events on the context's stream; synchronises.  *ms_ray (host) receives the
 * time from the first ray kernel's start to the last one's end (with one
 * chunk: the ray kernel's duration); *ms_psf the time after that until the
 * step ends (with one chunk: the PSF kernel's duration; with more, the PSF
 * work not overlapped with ray kernels).  For measurement only; frames are
 * identical to sg_batch_step's. */
sg_status sg_batch_step_profiled(sg_ctx* ctx, int32_t plan_id, float* out, float* ms_ray, float* ms_psf);

/* Launch shape currently used by a plan (for reports): scanlines per ray
 * work item, the PSF tile (tile_x scanlines by tile_y = 64 rows) and the
 * number of env chunks (the PSF kernel of chunk k runs beside the ray kernel
 * of chunk k + 1 on a second stream).  Any pointer may be NULL. */
sg_status sg_batch_config(sg_ctx* ctx, int32_t plan_id, int32_t* scanlines_per_item,
                          int32_t* tile_x, int32_t* tile_y, int32_t* chunks);

/* Set a plan's launch shape explicitly (instead of sg_autotune):
 * scanlines_per_item in {4, 8, 16} (four waves of 1, 2 or 4 scanlines),
 * tile_x in {16, 32, 64}, chunks in [1, 4] (clamped to the env count).
 * Every shape gives bit-identical frames.  SG_EINVAL for other values;
 * synchronises the context's stream. */
sg_status sg_batch_set_config(sg_ctx* ctx, int32_t plan_id, int32_t scanlines_per_item, int32_t tile_x,
                              int32_t chunks);

sg_status sg_batch_plan_destroy(sg_ctx* ctx, int32_t plan_id);

/* ------------------------------------------------------------------------
 * Reconstruction observation of the bone-surface task (Sec. 4, task 2:
 * bone surface segmented from each frame with misses, accumulated into a
 * reconstruction M and voxelised in the current probe frame; App. C: 40^3
 * voxels of 3 mm, 20 % missing points).  Bound to a batch plan: it reads the
 * plan's device geometry and poses of the step last enqueued, so its calls
 * go on the same stream after sg_batch_step.
 *   surface point   per scanline of each image plane, the first pixel whose
 *                   nearest label is a bone label (the rest of the scanline is
 *                   in the acoustic shadow)
 *   miss            Philox4x32-10 (key = seed, counter = (x | plane << 16,
 *                   env, step, 0x5245434F)): kept when word 0 <
 *                   floor((1 - p_miss) * 2^32)
 *   stored point    the pixel's probe point (a + x*dx, b, y*dy) mapped by the
 *                   step's pose into volume mm, FP64
 *   observation     each stored point u = R^T (p - t) in the current probe
 *                   frame occupies cell (floor(u_z / 3), floor((u_x + 60) / 3),
 *                   floor((u_y + 60) / 3)) of a [40][40][40] uint8 grid
 *                   (depth, lateral, elevation), 1 = occupied.
 */

/* Create a reconstruction for the plan's envs.  capacity: stored points per
 * env (further points are counted as overflow); bone_labels: host bitmap of
 * 256 bytes (nonzero = bone), or NULL for label 3 only; p_miss in [0, 1].
 * The plan must outlive the reconstruction's use.  Errors: SG_EINVAL. */
sg_status sg_recon_create(sg_ctx* ctx, int32_t plan_id, int32_t capacity, const uint8_t* bone_labels,
                          double p_miss, uint64_t seed, int32_t* recon_id);

/* Add the surface points of the plan's current frames (step index `step`
 * keys the misses).  Asynchronous on the context's stream. */
sg_status sg_recon_update(sg_ctx* ctx, int32_t recon_id, int32_t step);

/* Voxelise every env's stored points at the plan's current pose into grids:
 * device, n_envs * 40^3 uint8, env-major.  Asynchronous. */
sg_status sg_recon_observe(sg_ctx* ctx, int32_t recon_id, uint8_t* grids);

/* Host copies (synchronising): per-env stored point counts and overflow
 * (points beyond capacity); either pointer may be NULL. */
sg_status sg_recon_counts(sg_ctx* ctx, int32_t recon_id, int64_t* stored, int64_t* overflow);

/* Host copy (synchronising) of env `env`'s stored points, xyz doubles, at
 * most max_points; *n receives the number copied.  Order is unspecified. */
sg_status sg_recon_points(sg_ctx* ctx, int32_t recon_id, int32_t env, double* xyz, int64_t max_points, int64_t* n);

/* Forget the stored points of all envs (env < 0) or of one env. */
sg_status sg_recon_reset(sg_ctx* ctx, int32_t recon_id, int32_t env);

sg_status sg_recon_destroy(sg_ctx* ctx, int32_t recon_id);


/* ------------------------------------------------------------------------
 * Learned surrogate (a label-slice -> B-mode convolutional network trained on
 * frames of the physics path; the paper's learning-based simulator, Sec. 4
 * and App. B.2 "Learning-based approach", is a pix2pix U-Net trained with an
 * L1 term).  BF16 weights and activations, FP32 accumulation; all
 * convolutions run on MFMA implicit-GEMM kernels.
 *
 * Tensors are NHWC bf16 (uint16_t storage, round-to-nearest-even) with the
 * channel count a multiple of 8; conv weights are [Co][k][k][C] bf16.
 */
typedef struct {
    int32_t N, H, W, C;       /* input: N x H x W x C (stored size) */
    int32_t Co;               /* output channels (multiple of 8) */
    int32_t kernel, stride, pad;
    int32_t upsample;         /* 1: the conv reads its input nearest-upsampled x2,
                                 i.e. at (h / 2, w / 2) of a 2H x 2W grid */
} sg_conv_desc;
/* Output size: Ho = (H' + 2 pad - kernel) / stride + 1 with H' = H (x2 if upsample). */

/* y = act(conv(x, w) + bias), bf16 (device buffers, N x Ho x Wo x Co).
 * bias (FP32, Co) may be NULL; relu 0/1; if skip (bf16, like y) is given,
 * y_skip = bf16(y + skip) is written too; y_f32 (optional) receives act(acc +
 * bias) before rounding.  Errors: SG_EINVAL. */
sg_status sg_conv_forward(sg_ctx* ctx, const sg_conv_desc* d, const uint16_t* x, const uint16_t* w,
                          const float* bias, int32_t relu, const uint16_t* skip, uint16_t* y, uint16_t* y_skip,
                          float* y_f32);

/* dx = d(sum dy * y) / dx for the conv above without activation: dy is the
 * gradient at the conv output (bf16, N x Ho x Wo x Co), dx FP32 (N x H x W x C,
 * the stored input; with upsample the four fine positions are summed).
 * accumulate 0: write, 1: add into dx. */
sg_status sg_conv_backward_data(sg_ctx* ctx, const sg_conv_desc* d, const uint16_t* dy, const uint16_t* w,
                                float* dx, int32_t accumulate);

/* dw[Co][k][k][C] = sum over output pixels of dy * shifted x (FP32), and
 * db[Co] = sum of dy (FP32, may be NULL; needs Co <= 256).  Deterministic
 * (fixed-order split-K reduction).  Limits for all three conv calls: C and Co
 * multiples of 8 up to 4096, fewer than 2^31 input and output pixels. */
sg_status sg_conv_backward_weight(sg_ctx* ctx, const sg_conv_desc* d, const uint16_t* x, const uint16_t* dy,
                                  float* dw, float* db);

/* Create a surrogate for H x W frames (multiples of 16): a five-level
 * encoder-decoder (16/32/64/128/256 channels, two 3x3 convs per level,
 * stride-2 downsampling, nearest x2 upsampling + 3x3 conv, additive skips,
 * 1x1 head), He-initialised from `seed`.  Input per pixel: one-hot label
 * (labels 0..3), the gated scatterer sample of the volume's noise field and
 * the normalised depth (y + 0.5) / H.
 * *surr_id receives the id. */
sg_status sg_surr_create(sg_ctx* ctx, int32_t H, int32_t W, uint64_t seed, int32_t* surr_id);
sg_status sg_surr_destroy(sg_ctx* ctx, int32_t surr_id);

/* CT-conditioned surrogate: the learning-based simulator translates CT slices
 * into B-mode images, and its input CT is histogram-matched to a set of
 * training CT images (Sec. 4, "Ultrasound simulation"; App. B.2, learning-based
 * approach).  Same network and training calls as sg_surr_create; the input
 * per pixel is (bf16, 8 channels):
 *   0  the nearest voxel's HU (-1000 outside the volume), binned b =
 *      clamp(HU + 1024, 0, 4095), mapped through the frame's histogram
 *      specification r(b) = the smallest bin with refC[r] * n_src >=
 *      srcC[b] * n_ref (inclusive cumulative counts of the reference and of
 *      the frame, compared exactly in 64-bit integers), as (r - 1024) / 1000;
 *   1  N0 of the voxel's noise draw (not gated), 0 outside;
 *   2  N1 of the draw as the quantised normal of sg_noise_quantiles
 *      (entry w2 >> 20, times 2^-20), 0 outside;
 *   3  depth (y + 0.5) / H;  4..7 zero.
 * Every volume it reads must carry a CT (SG_EINVAL otherwise), and the
 * reference must be set (SG_ESTATE otherwise).
 * adv_weight in [0, 1]: weight of the adversarial term (the paper trains with
 * L1 weight 1 and GAN weight 0.01); 0 trains with L1 only.  With
 * adv_weight > 0 the surrogate owns a conditional patch discriminator: five
 * 3x3 convs (pad 1) 8->32 (stride 2), 32->64 (2), 64->128 (2), 128->128,
 * 128->8, leaky ReLU (slope 0.2) after the first four, channel 0 of the last
 * one the logit of an (H/8 x W/8) patch; its input is the encoded input's
 * channels 0..3 with the image (bf16) in channel 4.  Each training step then
 * runs in pix2pix's order: generator forward; discriminator step (Adam, same
 * rate) on L_D = (mean softplus(-l_real) + mean softplus(l_fake)) / 2 with
 * (input, physics frame) as real and (input, Yhat) as fake; the generator's
 * step on L1 + adv_weight * L_adv, L_adv = mean softplus(-l) of the updated
 * discriminator on (input, Yhat).
 * Checkpoints of CT surrogates also hold the reference counts and the
 * discriminator (parameters, moments, step). */
sg_status sg_surr_create_ct(sg_ctx* ctx, int32_t H, int32_t W, uint64_t seed, float adv_weight, int32_t* surr_id);

/* Sets the reference of a CT surrogate's histogram matching: the pooled bin
 * counts of n_envs frames (H x W probes, one plane) of CT volumes at the given
 * poses.  hist (host, 4096 int64, may be NULL) receives the counts.
 * Synchronises.  Errors: SG_EINVAL (not a CT surrogate, sizes, a volume
 * without CT), SG_ERANGE (a pose outside the fixed-point range). */
sg_status sg_surr_set_ct_reference(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, const int32_t* vol_ids,
                                   const sg_probe* probes, const double* poses, int64_t* hist);

/* Number of parameters (FP32 masters: weights then bias, layer by layer). */
sg_status sg_surr_num_params(sg_ctx* ctx, int32_t surr_id, int64_t* n);

/* One training step on n_envs pairs generated on the fly: the physics path
 * renders the targets, the encoder builds the inputs, then forward, L1 loss
 * (mean |Yhat - Y|), backward and one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8) with learning rate lr.  Every probe must be H x W.  *loss (host)
 * receives the batch loss before the update (synchronises).
 * The step's network part (forward, losses, backward, Adam) is replayed from
 * a HIP graph captured for the batch size: the first step of a new batch
 * size runs kernel by kernel (sizing the workspaces), the next one is
 * captured, later ones replay it; results are bit-identical either way.
 * Adam's step count and bias corrections are kept on the device. */
sg_status sg_surr_train_step(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, const int32_t* vol_ids,
                             const sg_probe* probes, const double* poses, float lr, float* loss);

/* sg_surr_train_step without the loss readback: the step is enqueued on the
 * context's stream and the call returns without waiting for the device
 * (host staging of the physics render aside).  The losses of each step stay
 * on the device for sg_surr_loss_history. */
sg_status sg_surr_train_step_async(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, const int32_t* vol_ids,
                                   const sg_probe* probes, const double* poses, float lr);

/* Losses of training steps first_step .. first_step + count - 1 (steps are
 * counted from 1 since creation or as restored by sg_surr_load): out (host,
 * count x 3 floats) receives per step the L1 loss, L_D and L_adv (both 0
 * without an adversarial term).  The device keeps the last 4096 steps.
 * Waits for the context's stream; copies through a pinned buffer.  Errors:
 * SG_ERANGE (steps not yet enqueued or older than the last 4096). */
sg_status sg_surr_loss_history(sg_ctx* ctx, int32_t surr_id, int64_t first_step, int32_t count, float* out);

/* Training steps done (enqueued) so far, *steps (host). */
sg_status sg_surr_step_count(sg_ctx* ctx, int32_t surr_id, int64_t* steps);

/* enable = 0: train kernel by kernel (no graph); 1 (default): replay the
 * captured step.  For timing comparisons and tests; results are identical. */
sg_status sg_surr_set_graph(sg_ctx* ctx, int32_t surr_id, int32_t enable);

/* Inference with an audit (the physics path judges the network on a subset
 * and replaces failing frames).  out: device FP32, n_envs frames of H x W,
 * clamp(Yhat, 0, 1).  audit_envs (host, n_audit distinct env indices, chosen
 * by the caller) are also rendered by physics; their PSNR (peak 1) is written
 * to psnr_out (host, n_audit).  A frame whose PSNR is below psnr_min is
 * replaced by its physics frame; if more than max_fail_frac of the audited
 * frames fail, every frame is rendered by physics.  *n_fallback (host)
 * receives the number of frames that came from physics.  Synchronises. */
sg_status sg_surr_infer(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, const int32_t* vol_ids,
                        const sg_probe* probes, const double* poses, float* out, const int32_t* audit_envs,
                        int32_t n_audit, float psnr_min, float max_fail_frac, float* psnr_out,
                        int32_t* n_fallback);

/* sg_surr_infer with BF16 frames: out_bf16 (device, n_envs x H x W bf16
 * bits, caller-owned) receives bf16(round to nearest even) of the frames
 * sg_surr_infer would write, network and fallback alike; the audit judges
 * the FP32 frames (the bf16 rounding of values in [0, 1] adds at most 2^-9
 * relative error, below -60 dB).  The library keeps an FP32 staging buffer
 * of the frames.  Errors as sg_surr_infer. */
sg_status sg_surr_infer_bf16(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, const int32_t* vol_ids,
                             const sg_probe* probes, const double* poses, uint16_t* out_bf16,
                             const int32_t* audit_envs, int32_t n_audit, float psnr_min, float max_fail_frac,
                             float* psnr_out, int32_t* n_fallback);

/* Decision rule of sg_surr_infer on host data (no device work): fallback[i]
 * (host, n_audit) = psnr[i] < psnr_min (NaN counts as failing); *whole = 1
 * if the failing fraction exceeds max_fail_frac. */
sg_status sg_audit_decide(int32_t n_audit, const float* psnr, float psnr_min, float max_fail_frac,
                          int32_t* fallback, int32_t* whole);

/* One training step on caller-supplied pairs: input (device, bf16, n_envs x
 * H x W x 8, the layout the encoder writes) and target (device, FP32, n_envs
 * x H x W); H and W state the buffers' frame size and must equal the
 * surrogate's (SG_EINVAL otherwise).  Otherwise as sg_surr_train_step (both
 * buffers are copied before the step).  For a CT surrogate with an
 * adversarial term the discriminator reads input channels 0..3.
 * Synchronises. */
sg_status sg_surr_train_pairs(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, int32_t H, int32_t W,
                              const uint16_t* input, const float* target, float lr, float* loss);

/* sg_surr_train_pairs without the loss readback (see sg_surr_train_step_async):
 * the two copies and the step are enqueued; returns without waiting, so
 * input and target must stay valid until the copies have run on the
 * context's stream (work ordered after the call on that stream may reuse
 * them). */
sg_status sg_surr_train_pairs_async(sg_ctx* ctx, int32_t surr_id, int32_t n_envs, int32_t H, int32_t W,
                                    const uint16_t* input, const float* target, float lr);

/* Adversarial losses of the last training step (host): L_D before the
 * discriminator's update and L_adv (without its weight) after it.
 * SG_EINVAL without an adversarial term, SG_ESTATE before the first step. */
sg_status sg_surr_gan_losses(sg_ctx* ctx, int32_t surr_id, float* loss_d, float* loss_adv);

/* The discriminator's FP32 parameters (per layer: weights [Co][3][3][Ci],
 * then Co biases), their gradient of the last step (host copies), and
 * setting them.  SG_EINVAL without an adversarial term. */
sg_status sg_surr_disc_num_params(sg_ctx* ctx, int32_t surr_id, int64_t* n);
sg_status sg_surr_disc_get_params(sg_ctx* ctx, int32_t surr_id, float* host);
sg_status sg_surr_disc_get_grads(sg_ctx* ctx, int32_t surr_id, float* host);
sg_status sg_surr_disc_set_params(sg_ctx* ctx, int32_t surr_id, const float* host);

/* Checkpoint: FP32 masters, Adam moments, step count and frame size in one
 * file.  Loading restores them bit for bit (same frame size required). */
sg_status sg_surr_save(sg_ctx* ctx, int32_t surr_id, const char* path);
sg_status sg_surr_load(sg_ctx* ctx, int32_t surr_id, const char* path);

/* Host copies of the FP32 parameters, of the gradient of the last training
 * step, and setting the parameters (also refreshes the bf16 copies);
 * `host` holds sg_surr_num_params floats. */
sg_status sg_surr_get_params(sg_ctx* ctx, int32_t surr_id, float* host);
sg_status sg_surr_get_grads(sg_ctx* ctx, int32_t surr_id, float* host);
sg_status sg_surr_set_params(sg_ctx* ctx, int32_t surr_id, const float* host);

/* Host copies of the last training step's encoded input (bf16, n x H x W x 8)
 * and physics target (FP32, n x H x W). */
sg_status sg_surr_get_batch(sg_ctx* ctx, int32_t surr_id, uint16_t* input, float* target);

/* Host copy of a tensor the last training step left on the device (support
 * for element-wise checking of each layer; valid until the next training or
 * inference call of this surrogate).  With host == NULL, *n receives the
 * element count; otherwise *n must equal it and the elements are copied
 * (synchronises).  n frames of the last step, NHWC, H x W at level 0 and
 * (H >> l) x (W >> l) at level l:
 *   SG_SURR_T_ACT    bf16 tensor `index` (uint16 bits): 0 X (8 ch, input),
 *       1 T1 (16), 2 E0 (16), 3 T2 (32, l1), 4 E1 (32), 5 T3 (64, l2),
 *       6 E2 (64), 7 T4 (128, l3), 8 E3 (128), 9 T5 (256, l4), 10 B4 (256),
 *       11 U3 (128, l3), 12 S3 = U3 + E3, 13 D3 (128), 14 U2 (64, l2),
 *       15 S2 = U2 + E2, 16 D2, 17 U1 (32, l1), 18 S1 = U1 + E1, 19 D1,
 *       20 U0 (16, l0), 21 S0 = [U0 + E0, depth integral] (24), 22 D0 (16),
 *       23 A0 (8, the depth integral before its copy into S0)
 *   SG_SURR_T_GRAD   FP32 gradient of the loss at tensor `index` (>= 1)
 *   SG_SURR_T_YHAT, _TARGET, _GY   FP32 n x H x W: network output, physics
 *       target, gradient at the output (L1 plus the adversarial part)
 *   SG_SURR_T_MOM1, _MOM2   FP32 Adam moments (sg_surr_num_params)
 *   SG_SURR_T_DSCAN  bf16 gradient at the depth map p (n x H x W x 8): the
 *       backward of the depth integral, scale * sum of the rows below
 * With a discriminator (frames [0, 2n): the step's first pass on the real
 * then the fake pairs; frames [2n, 3n): its second pass on the fake pairs
 * through the updated discriminator; level l = 1, 2, 3, 3, 3 for k = 1..5):
 *   SG_SURR_T_DISC_ACT   bf16 input of layer `index` (0: z, 8 ch, frames
 *       [0, 2n) only; 1..4: 32, 64, 128, 128 ch after leaky ReLU)
 *   SG_SURR_T_DISC_GRAD  FP32 gradient at that tensor (index 0: second pass only)
 *   SG_SURR_T_DISC_LOGITS, _GLOG   FP32 last-layer outputs (8 ch, channel 0
 *       the logit) and their gradient, (H >> 3) x (W >> 3)
 *   SG_SURR_T_DISC_MOM1, _MOM2   FP32 Adam moments (sg_surr_disc_num_params)
 * Errors: SG_EINVAL (id, kind, index, count), SG_ESTATE (no step yet). */
#define SG_SURR_T_ACT 0
#define SG_SURR_T_GRAD 1
#define SG_SURR_T_YHAT 2
#define SG_SURR_T_TARGET 3
#define SG_SURR_T_GY 4
#define SG_SURR_T_MOM1 5
#define SG_SURR_T_MOM2 6
#define SG_SURR_T_DISC_ACT 7
#define SG_SURR_T_DISC_GRAD 8
#define SG_SURR_T_DISC_LOGITS 9
#define SG_SURR_T_DISC_GLOG 10
#define SG_SURR_T_DISC_MOM1 11
#define SG_SURR_T_DISC_MOM2 12
#define SG_SURR_T_DSCAN 13
sg_status sg_surr_tensor(sg_ctx* ctx, int32_t surr_id, int32_t kind, int32_t index, void* host, int64_t* n);

/* VALU throughput probe (measurement support for the rooflines): times
 * independent instruction chains over a grid of 8 blocks of 256 threads per
 * compute unit and writes each kind's rate in lane-operations per second to
 * rates (host, 4 doubles; best of 3 runs):
 *   [0] FP32 FMA, two-operand encoding (literal operands);
 *   [1] 32-bit xor + add pairs, two-operand encodings (2 ops per pair);
 *   [2] 32x32->64 multiply-add (the Philox product);
 *   [3] FP32 FMA, three-operand encoding (operands from registers).
 * Synchronises.  Errors: SG_EINVAL (NULL), SG_EHIP. */
sg_status sg_valu_probe(sg_ctx* ctx, double* rates);

/* HBM bandwidth probe (measurement support for the rooflines): copies bytes
 * from src to dst (device, 16-byte aligned, not overlapping; bytes a non-zero
 * multiple of 16; the caller owns both) with 16-byte vector loads and stores
 * in eight launch shapes (4 or 8 loads in flight per thread, 8 or 16 blocks
 * of 256 threads per compute unit, cached or non-temporal), four runs each, and writes the best run after
 * each shape's first as bytes read + written per second to *rate (host).  dst holds a copy of src afterwards.  Use buffers
 * well beyond the last-level cache (hundreds of MiB).  Synchronises.
 * Errors: SG_EINVAL (NULL, size, alignment or overlap), SG_EHIP. */
sg_status sg_hbm_probe(sg_ctx* ctx, const void* src, void* dst, size_t bytes, double* rate);

#ifdef __cplusplus
}
#endif

#endif /* SONOSIM_H */
