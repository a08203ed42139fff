// CPU emulation of the small part of the HIP runtime and device language the
// FDAS kernels use (test infrastructure only).  Every workgroup runs as
// blockDim.x std::threads sharing `static` (= __shared__) arrays, with a
// std::barrier standing for __syncthreads; blocks run one after another.
// Device pointers are plain host pointers.  Used to check the kernels'
// indexing, masking and data flow on machines without a GPU.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__
#define __align__(n) __attribute__((aligned(n)))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))

struct float2 { float x, y; };
inline float2 make_float2(float a, float b) { return float2{a, b}; }
struct float4 { float x, y, z, w; };
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }
struct double2 { double x, y; };
inline double2 make_double2(double a, double b) { return double2{a, b}; }

inline unsigned __float_as_uint(float f) { unsigned u; std::memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(unsigned u) { float f; std::memcpy(&f, &u, 4); return f; }
inline int __float_as_int(float f) { int u; std::memcpy(&u, &f, 4); return u; }
inline float __int_as_float(int u) { float f; std::memcpy(&f, &u, 4); return f; }
#define __builtin_amdgcn_sched_barrier(x) ((void)0)

// Raw buffer resources: a byte range [base, base + bytes).  As on the GPU,
// an access whose byte offset is at or past the end is dropped (a load
// returns 0).  An access that straddles the end would be a kernel bug: it
// aborts.
struct EmuRsrc {
    unsigned char* base;
    uint32_t bytes;
};
#define __amdgpu_buffer_rsrc_t EmuRsrc
#define __builtin_amdgcn_make_buffer_rsrc emu_make_buffer_rsrc
#define __builtin_amdgcn_raw_buffer_store_b32 emu_raw_buffer_store_b32
#define __builtin_amdgcn_raw_buffer_store_b64 emu_raw_buffer_store_b64
#define __builtin_amdgcn_raw_buffer_load_b32 emu_raw_buffer_load_b32
inline EmuRsrc emu_make_buffer_rsrc(void* p, short stride, int bytes, int)
{
    if (stride != 0 || bytes < 0)
        std::abort();
    return EmuRsrc{static_cast<unsigned char*>(p), (uint32_t)bytes};
}
inline bool emu_in_range(const EmuRsrc& r, int off, int soff, uint32_t size)
{
    const uint32_t o = (uint32_t)off + (uint32_t)soff;
    if (o >= r.bytes)
        return false;
    if (o + size > r.bytes)
        std::abort();
    return true;
}
inline void emu_raw_buffer_store_b32(unsigned v, EmuRsrc r, int off, int soff, int)
{
    if (emu_in_range(r, off, soff, 4))
        std::memcpy(r.base + (uint32_t)off + (uint32_t)soff, &v, 4);
}
template <class V>
inline void emu_raw_buffer_store_b64(V v, EmuRsrc r, int off, int soff, int)
{
    static_assert(sizeof(V) == 8, "64-bit store");
    if (emu_in_range(r, off, soff, 8))
        std::memcpy(r.base + (uint32_t)off + (uint32_t)soff, &v, 8);
}
inline unsigned emu_raw_buffer_load_b32(EmuRsrc r, int off, int soff, int)
{
    unsigned v = 0;
    if (emu_in_range(r, off, soff, 4))
        std::memcpy(&v, r.base + (uint32_t)off + (uint32_t)soff, 4);
    return v;
}
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx { unsigned x = 0, y = 0, z = 0; };
inline thread_local EmuIdx threadIdx;
inline EmuIdx blockIdx, gridDim, blockDim;
inline std::barrier<>* emu_barrier = nullptr;
inline void __syncthreads() { emu_barrier->arrive_and_wait(); }
// A wave's lanes run as separate threads here, so a wave-local exchange
// through LDS needs a barrier over the wave's 64 threads (on the GPU a wave's
// LDS accesses are in order and the builtin only fences the compiler).
inline std::vector<std::barrier<>*> emu_wave_barriers;
inline void emu_wave_barrier() { emu_wave_barriers[threadIdx.x / 64]->arrive_and_wait(); }
#define __builtin_amdgcn_wave_barrier emu_wave_barrier
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)

using std::max;
using std::min;

// Cross-lane permute within a 64-lane wave (lane i reads lane (addr/4) mod 64
// of its own wave).  Emulated through a workgroup-wide buffer between two
// barriers, so every thread of the workgroup must reach it (as on the GPU,
// where the kernels call it in uniform control flow).
#define __builtin_amdgcn_ds_bpermute emu_ds_bpermute
inline int emu_perm_buf[1024];
inline int emu_ds_bpermute(int addr, int data)
{
    const unsigned t = threadIdx.x;
    emu_perm_buf[t] = data;
    __syncthreads();
    const int v = emu_perm_buf[(t & ~63u) + ((unsigned)(addr >> 2) & 63u)];
    __syncthreads();
    return v;
}
// DPP moves, for the two wave-wide patterns the kernels use: 0x130 (lane i
// reads lane i + 1; lane 63 has no source) and 0x134 (lane i reads lane
// (i + 1) mod 64).  A lane without a source gets 0 (bound_ctrl) or `old`.
// Exchanged through a per-wave buffer between two wave barriers, so every
// lane of the wave must reach it (uniform control flow, as in the kernels).
inline int emu_dpp_buf[1024];
inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    if ((ctrl != 0x130 && ctrl != 0x134) || row_mask != 0xf || bank_mask != 0xf)
        std::abort();
    const unsigned t = threadIdx.x, lane = t & 63u, base = t & ~63u;
    emu_dpp_buf[t] = src;
    emu_wave_barrier();
    int v;
    if (ctrl == 0x134 || lane < 63)
        v = emu_dpp_buf[base + ((lane + 1) & 63u)];
    else
        v = bound_ctrl ? 0 : old;
    emu_wave_barrier();
    return v;
}
inline int emu_mov_dpp(int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    return emu_update_dpp(0, src, ctrl, row_mask, bank_mask, bound_ctrl);
}
#define __builtin_amdgcn_update_dpp emu_update_dpp
#define __builtin_amdgcn_mov_dpp emu_mov_dpp
inline long long clock64() { return 0; }
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline void sincospi(double x, double* s, double* c) { *s = std::sin(M_PI * x); *c = std::cos(M_PI * x); }

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101,
       hipErrorInvalidSymbol = 13 };
// a device symbol is a host object here: its address is the device address
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym)
{
    *p = const_cast<void*>(sym);
    return hipSuccess;
}
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
typedef struct ihipStream_t* hipStream_t;
enum { hipDeviceAttributeMultiprocessorCount = 0 };
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 3; return hipSuccess; }
template <class F>
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, int) { *n = 1; return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t)
{
    std::memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

template <class K, class... A>
void emu_launch(K kernel, dim3 grid, dim3 block, A... args)
{
    gridDim = EmuIdx{grid.x, grid.y, grid.z};
    blockDim = EmuIdx{block.x, block.y, block.z};
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                blockIdx = EmuIdx{bx, by, bz};
                std::barrier<> bar(block.x);
                emu_barrier = &bar;
                std::vector<std::unique_ptr<std::barrier<>>> wbars;
                emu_wave_barriers.clear();
                for (unsigned w0 = 0; w0 < block.x; w0 += 64) {
                    wbars.emplace_back(new std::barrier<>(std::min(64u, block.x - w0)));
                    emu_wave_barriers.push_back(wbars.back().get());
                }
                std::vector<std::thread> th;
                th.reserve(block.x);
                for (unsigned t = 0; t < block.x; ++t)
                    th.emplace_back([=]() {
                        threadIdx = EmuIdx{t, 0, 0};
                        kernel(args...);
                    });
                for (auto& x : th)
                    x.join();
            }
}
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) emu_launch(k, dim3(grid), dim3(block), __VA_ARGS__)
