// Measurement probes.  Streaming probes of the device memory: a write-only
// and a read-only pass over a float buffer.  They measure the bandwidth that plain streaming
// kernels reach on this device, the figure the correlation's plane write
// and the harmonic gathers are compared with beside the published peak.
//
// The write is one pass of 16-byte stores, one per lane; the read is a
// grid-stride loop of 16-byte non-temporal loads on a fixed grid that fills
// every CU several times over, and keeps its loads live by summing them:
// one partial sum per workgroup, reduced through LDS.
//
// An LDS bank probe: one wave repeats one LDS access of a chosen width at
// per-lane element indices the caller picks, and reports the clock cycles
// of the loop, so access patterns can be compared for bank conflicts (the
// rules the transforms' LDS layout follows were established with it).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdas.h"
#include "fdas_internal.h"

namespace fdas {

namespace {

constexpr int kStreamThreads = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One pass, one 16-byte vector per lane: measured on gfx950 this layout
// (plain stores) writes faster than grid-stride loops or several vectors per
// lane, with or without non-temporal hints.
__global__ __launch_bounds__(kStreamThreads) void stream_write_kernel(float* __restrict__ dst,
                                                                      int64_t n, float value)
{
    const int64_t nv = n / 4;
    const int64_t i = (int64_t)blockIdx.x * kStreamThreads + threadIdx.x;
    const f32x4 v = {value, value, value, value};
    if (i < nv)
        reinterpret_cast<f32x4*>(dst)[i] = v;
    // the tail of n mod 4 floats
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * nv)
        dst[4 * nv + threadIdx.x] = value;
}

__global__ __launch_bounds__(kStreamThreads) void stream_read_kernel(const float* __restrict__ src,
                                                                     int64_t n,
                                                                     float* __restrict__ sums)
{
    __shared__ float red[kStreamThreads];
    const int64_t nv = n / 4;
    const int64_t stride = (int64_t)gridDim.x * kStreamThreads;
    const f32x4* s = reinterpret_cast<const f32x4*>(src);
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kStreamThreads + threadIdx.x; i < nv; i += stride) {
        const f32x4 v = __builtin_nontemporal_load(s + i);
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * nv)
        acc += src[4 * nv + threadIdx.x];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kStreamThreads / 2; w > 0; w /= 2) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        sums[blockIdx.x] = red[0];
    // the partials of workgroups not launched (short buffers) are zero
    if (blockIdx.x == 0)
        for (int i = gridDim.x + threadIdx.x; i < FDAS_STREAM_PARTIALS; i += kStreamThreads)
            sums[i] = 0.f;
}

int read_grid(int64_t n)
{
    const int64_t vec_blocks = (n / 4 + kStreamThreads - 1) / kStreamThreads;
    return (int)(vec_blocks < 1 ? 1 : (vec_blocks < FDAS_STREAM_PARTIALS ? vec_blocks
                                                                         : FDAS_STREAM_PARTIALS));
}

// LDS bank probe: MODE 0/1 = 64-bit write/read, 2 = 128-bit write.  Each
// lane's index is masked into the 64 KB array, so any pattern stays in
// bounds.  The loop's accesses are kept (a wave barrier between them, the
// reads summed into the output).
constexpr int kProbeBytes = 65536;

template <int MODE>
__global__ __launch_bounds__(64) void lds_probe_kernel(const int* __restrict__ pattern, int iters,
                                                       long long* __restrict__ cycles,
                                                       float* __restrict__ sink)
{
    __shared__ __align__(16) float4 buf[kProbeBytes / 16];
    const int l = threadIdx.x;
    for (int i = l; i < kProbeBytes / 16; i += 64)
        buf[i] = make_float4((float)i, 0.f, 0.f, 1.f);
    __syncthreads();
    float2* b2 = reinterpret_cast<float2*>(buf);
    const int idx = pattern[l];
    const int i2 = idx & (kProbeBytes / 8 - 1), i4 = idx & (kProbeBytes / 16 - 1);
    float acc = 0.f;
    const long long t0 = clock64();
    for (int k = 0; k < iters; ++k) {
        if constexpr (MODE == 0) {
            b2[i2] = make_float2((float)k, (float)l);
        } else if constexpr (MODE == 1) {
            const float2 v = b2[i2];
            acc += v.x + v.y;
        } else {
            buf[i4] = make_float4((float)k, (float)l, 0.f, 1.f);
        }
        __syncthreads();
    }
    const long long t1 = clock64();
    sink[blockIdx.x * 64 + l] = acc + reinterpret_cast<float*>(buf)[l];
    if (l == 0)
        cycles[blockIdx.x] = t1 - t0;
}

}  // namespace

hipError_t launch_lds_probe(const int* pattern, int mode, int iters, int groups,
                            long long* cycles, float* sink, hipStream_t s)
{
    if (mode == 0)
        hipLaunchKernelGGL(lds_probe_kernel<0>, dim3(groups), dim3(64), 0, s, pattern, iters,
                           cycles, sink);
    else if (mode == 1)
        hipLaunchKernelGGL(lds_probe_kernel<1>, dim3(groups), dim3(64), 0, s, pattern, iters,
                           cycles, sink);
    else
        hipLaunchKernelGGL(lds_probe_kernel<2>, dim3(groups), dim3(64), 0, s, pattern, iters,
                           cycles, sink);
    return hipGetLastError();
}

hipError_t launch_stream_write(float* dst, int64_t n, float value, hipStream_t s)
{
    const int64_t blocks = (n / 4 + kStreamThreads - 1) / kStreamThreads;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_write_kernel, dim3(blocks < 1 ? 1u : (unsigned)blocks),
                       dim3(kStreamThreads), 0, s, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_stream_read(const float* src, int64_t n, float* sums, hipStream_t s)
{
    hipLaunchKernelGGL(stream_read_kernel, dim3(read_grid(n)), dim3(kStreamThreads), 0, s, src,
                       n, sums);
    return hipGetLastError();
}

}  // namespace fdas
