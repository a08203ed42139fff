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

// ---- batched: the planes of fdas_correlate_batched (plane b at K offsets[b],
// [K][N_b]), every fold in one launch --------------------------------------------

// fold column prefix sums over the spectra: colpre[b] = sum_{b' < b}
// ceil(N_b' / H), and the same for H/2 in prevpre (one workgroup).
constexpr int kHScanThreads = 256;

__global__ __launch_bounds__(kHScanThreads) void harmonic_scan_kernel(
    const int64_t* __restrict__ offsets, int nspec, int H, int64_t* __restrict__ colpre,
    int64_t* __restrict__ prevpre)
{
    __shared__ int64_t part[2][kHScanThreads];
    __shared__ int64_t carry[2];
    const int t = threadIdx.x;
    const int Hp = H > 1 ? H / 2 : 1;
    if (t == 0) {
        carry[0] = carry[1] = 0;
        colpre[0] = prevpre[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < nspec; base += kHScanThreads) {
        const int b = base + t;
        int64_t a = 0, p = 0;
        if (b < nspec) {
            const int64_t n = offsets[b + 1] - offsets[b];
            a = n > 0 ? (n + H - 1) / H : 0;
            p = n > 0 ? (n + Hp - 1) / Hp : 0;
        }
        part[0][t] = a;
        part[1][t] = p;
        __syncthreads();
        for (int d = 1; d < kHScanThreads; d <<= 1) {
            const int64_t x = t >= d ? part[0][t - d] : 0;
            const int64_t y = t >= d ? part[1][t - d] : 0;
            __syncthreads();
            part[0][t] += x;
            part[1][t] += y;
            __syncthreads();
        }
        if (b < nspec) {
            colpre[b + 1] = carry[0] + part[0][t];
            prevpre[b + 1] = carry[1] + part[1][t];
        }
        __syncthreads();
        if (t == kHScanThreads - 1) {
            carry[0] += part[0][t];
            carry[1] += part[1][t];
        }
        __syncthreads();
    }
}

// Spectrum of fold column g: the b with colpre[b] <= g < colpre[b + 1]
// (binary search; empty spectra have equal bounds and are skipped).
__device__ __forceinline__ int column_spectrum(const int64_t* __restrict__ colpre, int nspec,
                                               int64_t g)
{
    int lo = 0, hi = nspec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (colpre[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Persistent grid: each lane takes fold columns g (stride gridDim.x x
// threads) over all spectra and walks the fold's KH rows for it, so a row's
// loads stay coalesced across the lanes.  Fold b lives at sums + KH
// colpre[b] as [KH][NH_b]; the previous fold (H/2) at prev + KHp prevpre[b].
__global__ __launch_bounds__(kHarmThreads) void harmonic_batched_kernel(
    const float* __restrict__ planes, const int64_t* __restrict__ offsets, int nspec, int K, int H,
    const float* __restrict__ prev, int KHp, const int64_t* __restrict__ colpre,
    const int64_t* __restrict__ prevpre, float* __restrict__ sums, int KH)
{
    const int64_t total = colpre[nspec];
    const int c = (K - 1) / 2;
    const int h0 = prev != nullptr ? H / 2 + 1 : 1;
    for (int64_t g = (int64_t)blockIdx.x * kHarmThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kHarmThreads) {
        const int b = column_spectrum(colpre, nspec, g);
        const int64_t Nb = offsets[b + 1] - offsets[b];
        const int64_t NH = (Nb + H - 1) / H;
        const int64_t r = g - colpre[b];
        const float* plane = planes + (int64_t)K * offsets[b];
        float* out = sums + (int64_t)KH * colpre[b] + r;
        const float* pv = nullptr;
        int64_t NHp = 0;
        if (prev != nullptr) {
            NHp = (Nb + H / 2 - 1) / (H / 2);
            pv = prev + (int64_t)KHp * prevpre[b] + r;
        }
        for (int krow = 0; krow < KH; ++krow) {
            const int dk = krow - (KH - 1) / 2;
            float s = 0.f;
            if (pv != nullptr)
                s = pv[(int64_t)(dk + (KHp - 1) / 2) * NHp];
            for (int h = h0; h <= H; ++h)
                s += plane[(int64_t)(c + h * dk) * Nb + (int64_t)h * r];
            out[(int64_t)krow * NH] = s;
        }
    }
}

// Peaks of every spectrum's fold; the record's r is the packed bin index
// offsets[b] + r, which names the spectrum too.
__global__ __launch_bounds__(kHarmThreads) void candidates_batched_kernel(
    const float* __restrict__ sums, const int64_t* __restrict__ offsets, int nspec, int H,
    const int64_t* __restrict__ colpre, int KH, float threshold, int row0,
    fdas_candidate* __restrict__ out, int capacity, unsigned* __restrict__ count)
{
    const int64_t total = colpre[nspec];
    for (int64_t g = (int64_t)blockIdx.x * kHarmThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kHarmThreads) {
        const int b = column_spectrum(colpre, nspec, g);
        const int64_t Nb = offsets[b + 1] - offsets[b];
        const int64_t NH = (Nb + H - 1) / H;
        const int64_t r = g - colpre[b];
        const float* S = sums + (int64_t)KH * colpre[b];
        for (int k = 0; k < KH; ++k) {
            const float v = S[(int64_t)k * NH + r];
            if (!(v > threshold))
                continue;
            bool peak = true;
            for (int a = -1; a <= 1; ++a) {
                const int kk = k + a;
                if (kk < 0 || kk >= KH)
                    continue;
                for (int d = -1; d <= 1; ++d) {
                    const int64_t rr = r + d;
                    if ((a == 0 && d == 0) || rr < 0 || rr >= NH)
                        continue;
                    peak = peak && v >= S[(int64_t)kk * NH + rr];
                }
            }
            if (!peak)
                continue;
            const unsigned slot = atomicAdd(count, 1u);
            if (slot < (unsigned)capacity) {
                fdas_candidate cand;
                cand.r = offsets[b] + r;
                cand.row = row0 + k;
                cand.power = v;
                out[slot] = cand;
            }
        }
    }
}

// Persistent workgroups of the batched kernels (grid-stride loops, so any
// count is correct; the host emulation of the tests builds with a small one).
#ifndef FDAS_HARM_BATCHED_GRID
#define FDAS_HARM_BATCHED_GRID 2048
#endif
constexpr int kHarmBatchedGrid = FDAS_HARM_BATCHED_GRID;

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

hipError_t launch_harmonic_batched(const float* planes, const int64_t* offsets, int nspec, int K,
                                   int H, const float* prev, float* sums, int64_t* colpre,
                                   int64_t* prevpre, hipStream_t s)
{
    int KH = 0, KHp = 0;
    int64_t NH = 0, NHp = 0;
    harmonic_shape(1, K, H, &KH, &NH);
    if (prev != nullptr)
        harmonic_shape(1, K, H / 2, &KHp, &NHp);
    hipLaunchKernelGGL(harmonic_scan_kernel, dim3(1), dim3(kHScanThreads), 0, s, offsets, nspec, H,
                       colpre, prevpre);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(harmonic_batched_kernel, dim3(kHarmBatchedGrid), dim3(kHarmThreads), 0, s,
                       planes, offsets, nspec, K, H, prev, KHp, colpre, prevpre, sums, KH);
    return hipGetLastError();
}

hipError_t launch_candidates_batched(const float* sums, const int64_t* offsets, int nspec, int K,
                                     int H, float threshold, fdas_candidate* out, int capacity,
                                     unsigned* count, int64_t* colpre, int64_t* prevpre,
                                     hipStream_t s)
{
    int KH = 0;
    int64_t NH = 0;
    harmonic_shape(1, K, H, &KH, &NH);
    hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(harmonic_scan_kernel, dim3(1), dim3(kHScanThreads), 0, s, offsets, nspec, H,
                       colpre, prevpre);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    const int row0 = (K - 1) / 2 - (KH - 1) / 2;
    hipLaunchKernelGGL(candidates_batched_kernel, dim3(kHarmBatchedGrid), dim3(kHarmThreads), 0,
                       s, sums, offsets, nspec, H, colpre, KH, threshold, row0, out, capacity,
                       count);
    return hipGetLastError();
}

}  // namespace fdas
