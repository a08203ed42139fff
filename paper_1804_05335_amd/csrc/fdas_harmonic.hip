// Harmonic summing and peak candidates on the f-fdot power plane (Sec. 3:
// a pulsed signal spreads its power over harmonics, whose powers are added
// to the fundamental's before the search for peaks, and the power is
// compared with a precomputed threshold to find candidates).
//
// A constant-fdot signal at (r, z) has its h-th harmonic at (h r, h z).  On
// a plane P[K][N] with rows z_k = (k - c) dz, c = (K - 1)/2, the H-fold sum
// at the fundamental (k, r) is S_H[k][r] = sum_{h=1}^{H} P[c + h (k - c)][h r]
// over the fundamentals whose harmonics all lie on the plane: r < ceil(N/H),
// |k - c| <= floor(c/H).  Harmonics of grid points are grid points, so the
// sums are exact gathers; they are formed in FP32 in the order h = 1..H, so
// a fold built on top of the previous one (H/2 terms already summed) equals
// the fold built from scratch bit for bit.
//
// Memory: the plane is read with stride h along a row for harmonic h, so
// each harmonic touches whole rows of the plane; folding up to 2^f reads
// about half a plane per fold on top of the previous fold's sums.  The
// kernels are plain streaming gathers (HBM-bound); a lane owns one
// fundamental column and walks its harmonics with independent loads.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdas.h"
#include "fdas_internal.h"

namespace fdas {

namespace {

constexpr int kHarmThreads = 256;

// One row of the H-fold sum per blockIdx.y, kHarmCols columns per
// blockIdx.x: lane t takes columns t + kHarmThreads j, j < kHarmCols /
// kHarmThreads, so each load instruction is coalesced and every lane keeps
// several independent gathers in flight.  With prev (the H/2-fold, KHp x
// NHp), the sum starts from it and adds harmonics H/2 + 1 .. H; without, it
// adds 1 .. H from zero.
constexpr int kHarmPerLane = 4;
constexpr int kHarmCols = kHarmThreads * kHarmPerLane;

__global__ __launch_bounds__(kHarmThreads) void harmonic_sum_kernel(
    const float* __restrict__ plane, int64_t N, int K, int H, const float* __restrict__ prev,
    int64_t NHp, int KHp, float* __restrict__ out, int64_t NH, int KH)
{
    const int64_t r0 = (int64_t)blockIdx.x * kHarmCols + threadIdx.x;
    const int c = (K - 1) / 2;
    const int krow = blockIdx.y;                       // row of the fold
    const int dk = krow - (KH - 1) / 2;                // k - c of the fundamental
    float s[kHarmPerLane];
    bool in[kHarmPerLane];
#pragma unroll
    for (int j = 0; j < kHarmPerLane; ++j) {
        in[j] = r0 + (int64_t)j * kHarmThreads < NH;
        s[j] = 0.f;
    }
    int h0 = 1;
    if (prev != nullptr) {
        const float* p = prev + (int64_t)(dk + (KHp - 1) / 2) * NHp + r0;
#pragma unroll
        for (int j = 0; j < kHarmPerLane; ++j)
            if (in[j])
                s[j] = p[(int64_t)j * kHarmThreads];
        h0 = H / 2 + 1;
    }
    for (int h = h0; h <= H; ++h) {
        const float* row = plane + (int64_t)(c + h * dk) * N + (int64_t)h * r0;
#pragma unroll
        for (int j = 0; j < kHarmPerLane; ++j)
            if (in[j])
                s[j] += row[(int64_t)h * j * kHarmThreads];
    }
    float* o = out + (int64_t)krow * NH + r0;
#pragma unroll
    for (int j = 0; j < kHarmPerLane; ++j)
        if (in[j])
            o[(int64_t)j * kHarmThreads] = s[j];
}

__global__ void zero_count_kernel(unsigned* __restrict__ count)
{
    if (threadIdx.x == 0)
        *count = 0u;
}

// Peaks of one fold: S > threshold and S >= each neighbour inside the fold.
__global__ __launch_bounds__(kHarmThreads) void candidates_kernel(
    const float* __restrict__ S, int64_t NH, int KH, float threshold, int row0,
    fdas_candidate* __restrict__ out, int capacity, unsigned* __restrict__ count)
{
    const int64_t r = (int64_t)blockIdx.x * kHarmThreads + threadIdx.x;
    const int k = blockIdx.y;
    if (r >= NH)
        return;
    const float v = S[(int64_t)k * NH + r];
    if (!(v > threshold))
        return;
    bool peak = true;
    for (int a = -1; a <= 1; ++a) {
        const int kk = k + a;
        if (kk < 0 || kk >= KH)
            continue;
        for (int b = -1; b <= 1; ++b) {
            const int64_t rr = r + b;
            if ((a == 0 && b == 0) || rr < 0 || rr >= NH)
                continue;
            peak = peak && v >= S[(int64_t)kk * NH + rr];
        }
    }
    if (!peak)
        return;
    const unsigned slot = atomicAdd(count, 1u);
    if (slot < (unsigned)capacity) {
        fdas_candidate cand;
        cand.r = r;
        cand.row = row0 + k;
        cand.power = v;
        out[slot] = cand;
    }
}

}  // namespace

void harmonic_shape(int64_t N, int K, int H, int* KH, int64_t* NH)
{
    const int c = (K - 1) / 2;
    *KH = 2 * (c / H) + 1;
    *NH = (N + H - 1) / H;
}

hipError_t launch_harmonic_sum(const float* plane, int64_t N, int K, int H, const float* prev,
                               float* out, hipStream_t s)
{
    int KH = 0, KHp = 0;
    int64_t NH = 0, NHp = 0;
    harmonic_shape(N, K, H, &KH, &NH);
    if (prev != nullptr)
        harmonic_shape(N, K, H / 2, &KHp, &NHp);
    if (NH == 0)
        return hipSuccess;
    const dim3 grid((unsigned)((NH + kHarmCols - 1) / kHarmCols), (unsigned)KH);
    hipLaunchKernelGGL(harmonic_sum_kernel, grid, dim3(kHarmThreads), 0, s, plane, N, K, H, prev,
                       NHp, KHp, out, NH, KH);
    return hipGetLastError();
}

hipError_t launch_candidates(const float* S, int64_t N, int K, int H, float threshold,
                             fdas_candidate* out, int capacity, unsigned* count, hipStream_t s)
{
    int KH = 0;
    int64_t NH = 0;
    harmonic_shape(N, K, H, &KH, &NH);
    hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || NH == 0)
        return e;
    const int row0 = (K - 1) / 2 - (KH - 1) / 2;
    const dim3 grid((unsigned)((NH + kHarmThreads - 1) / kHarmThreads), (unsigned)KH);
    hipLaunchKernelGGL(candidates_kernel, grid, dim3(kHarmThreads), 0, s, S, NH, KH, threshold,
                       row0, out, capacity, count);
    return hipGetLastError();
}

}  // namespace fdas
