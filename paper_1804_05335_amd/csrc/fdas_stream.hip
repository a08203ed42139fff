// Streaming probes of the device memory: a write-only and a read-only pass
// over a float buffer.  They measure the bandwidth that plain streaming
// kernels reach on this device, the figure the correlation's plane write
// and the harmonic gathers are compared with beside the published peak.
//
// The write is one pass of 16-byte stores, one per lane; the read is a
// grid-stride loop of 16-byte non-temporal loads on a fixed grid that fills
// every CU several times over, and keeps its loads live by summing them:
// one partial sum per workgroup, reduced through LDS.
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

}  // namespace

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
