// Throughput probe of the VALU: independent chains of FP32 FMAs, of 32-bit
// xor/add pairs and of 32x32->64 multiply-adds (the Philox product), timed
// with HIP events over a grid that fills the device.  Chains with literal
// operands compile to the two-operand (VOP2) encodings, the FMA chain with
// operands from kernel arguments to the three-operand (VOP3) one; the two
// issue at different rates.  No chain can be folded at compile time (none
// is a closed-form recurrence).  A 16-byte-vector device copy measures the
// HBM bandwidth the rooflines' memory side can reach.  Entry points in
// include/sonosim.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sg_host.h"

namespace sg {
namespace {

constexpr int kProbeIters = 4096;
constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_probe_fma(float* out, float m, float c)
{
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (float)(threadIdx.x + j);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_fma_lit(float* out)
{
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (float)(threadIdx.x + j);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], 0.999f, 0.001f);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_int(uint32_t* out)
{
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x + j;
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = (a[j] ^ 0x9E3779B9u) + 0x3C6EF372u;
    }
    uint32_t s = 0u;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_mad64(uint32_t* out, uint32_t m)
{
    uint32_t a[kChains], c[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = threadIdx.x + j;
        c[j] = m ^ (uint32_t)j;
    }
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const uint64_t p = (uint64_t)m * a[j] + c[j];
            a[j] = (uint32_t)(p >> 32);
            c[j] = (uint32_t)p;
        }
    }
    uint32_t s = 0u;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= a[j] ^ c[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Grid-stride copy, U 16-byte loads in flight per thread before their
// stores; NT: non-temporal loads and stores (streamed past the caches).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_probe_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n4)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += U * stride) {
        v4f v[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (i + j * stride < n4) v[j] = NT ? __builtin_nontemporal_load(src + i + j * stride) : src[i + j * stride];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (i + j * stride < n4) {
                if (NT)
                    __builtin_nontemporal_store(v[j], dst + i + j * stride);
                else
                    dst[i + j * stride] = v[j];
            }
    }
}

template <int U, bool NT>
hipError_t launch_copy(int blocks, hipStream_t st, const void* src, void* dst, size_t n4)
{
    hipLaunchKernelGGL((k_probe_copy<U, NT>), dim3(blocks), dim3(256), 0, st, (const v4f*)src, (v4f*)dst, n4);
    return hipGetLastError();
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_valu_probe(sg_ctx* c, double* rates)
{
    if (!c || !rates) return fail(SG_EINVAL, "sg_valu_probe: NULL argument");
    (void)hipSetDevice(c->device);
    const int threads = 256, blocks = 8 * c->n_cu;   // 8 waves per SIMD
    DevBuf out;
    hipError_t e = out.ensure(sizeof(uint32_t) * (size_t)blocks * threads);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const double ops_per_iter[4] = {kChains, 2.0 * kChains, kChains, kChains};   // lane-ops per chain step
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        float best = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, c->stream);
            if (k == 0) hipLaunchKernelGGL(k_probe_fma_lit, dim3(blocks), dim3(threads), 0, c->stream, (float*)out.p);
            if (k == 1) hipLaunchKernelGGL(k_probe_int, dim3(blocks), dim3(threads), 0, c->stream, (uint32_t*)out.p);
            if (k == 3)
                hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(threads), 0, c->stream, (float*)out.p, 0.999f,
                                   0.001f);
            if (k == 2)
                hipLaunchKernelGGL(k_probe_mad64, dim3(blocks), dim3(threads), 0, c->stream, (uint32_t*)out.p,
                                   0xD2511F53u);
            if (e == hipSuccess) e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) best = std::min(best, ms);
        }
        rates[k] = (double)blocks * threads * kProbeIters * ops_per_iter[k] / (best * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e == hipSuccess ? SG_OK : hip_fail(e, "VALU probe");
}

extern "C" sg_status sg_hbm_probe(sg_ctx* c, const void* src, void* dst, size_t bytes, double* rate)
{
    if (!c || !src || !dst || !rate) return fail(SG_EINVAL, "sg_hbm_probe: NULL argument");
    if (bytes == 0 || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return fail(SG_EINVAL, "sg_hbm_probe: bytes and both pointers must be non-zero multiples of 16");
    const char* s8 = static_cast<const char*>(src);
    const char* d8 = static_cast<const char*>(dst);
    if (s8 < d8 + bytes && d8 < s8 + bytes) return fail(SG_EINVAL, "sg_hbm_probe: buffers overlap");
    (void)hipSetDevice(c->device);
    const size_t n4 = bytes / 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    // shapes: {4, 8} loads in flight x {8, 16} blocks per CU x {cached, non-temporal}; the first run of
    // each warms the TLB and is not kept
    for (int shape = 0; shape < 8 && e == hipSuccess; ++shape) {
        const int blocks = (shape & 1 ? 16 : 8) * c->n_cu;
        const bool u8 = shape & 2, nt = shape & 4;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess)
                e = nt ? (u8 ? launch_copy<8, true>(blocks, c->stream, src, dst, n4)
                             : launch_copy<4, true>(blocks, c->stream, src, dst, n4))
                       : (u8 ? launch_copy<8, false>(blocks, c->stream, src, dst, n4)
                             : launch_copy<4, false>(blocks, c->stream, src, dst, n4));
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && rep > 0) best = std::min(best, ms);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "HBM probe");
    *rate = 2.0 * (double)bytes / (best * 1e-3);
    return SG_OK;
}
