// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <complex>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "../../include/fdas.h"

namespace fdas {

// Record `msg` as the calling thread's last-error text and return status.
int fail_status(int status, const char* msg);

// Host FP64 response R(q, z) (templates source file).
std::complex<double> response(double q, double z);

// Bank rows H_z and the twiddle row for segment length L.
hipError_t launch_prepare_bank(const float2* taps, int K, int M, int L, float2* bank,
                               hipStream_t s);

// Fused forward correlation of one spectrum on `grid` persistent workgroups
// (0 = as many as the device holds resident); interbin selects the [K][2N]
// interbinned plane, sym a bank holding only the z >= 0 rows.
hipError_t launch_forward(const float2* spec, int64_t N, const float2* bank, int K, int M,
                          int L, float* plane, int grid, bool interbin, bool sym, hipStream_t s);

// Two-bin Fourier interpolation: the integer bank and the half-bin bank on
// one segment geometry of Mgeom taps (the half-bin tap count, M + 2), both
// inverse transforms per template, pairs written into the [K][2N] plane.
hipError_t launch_forward_dual(const float2* spec, int64_t N, const float2* bank,
                               const float2* bank_half, int K, int Mgeom, int L, float* plane2,
                               int grid, hipStream_t s);

// Batched ragged correlation: segment scan into segpre[nspec + 1] (device
// workspace), then the persistent kernel on `grid` workgroups (0 = fill the
// device at full occupancy) with E values per lane (0 = the default for L;
// batched_values_per_lane_ok lists the others).  Offsets are clamped to
// [0, cap] on the device.
bool batched_values_per_lane_ok(int L, int E);
// Workgroups of the batched kernel for (L, E, M) the current device holds
// resident (the grid that `grid = 0` launches).
hipError_t batched_resident_grid(int L, int E, int M, int* grid);
hipError_t launch_batched(const float2* specs, const int64_t* offsets, int nspec, int64_t cap,
                          const float2* bank, int K, int M, int L, int E, float* planes,
                          int64_t* segpre, int grid, hipStream_t s);

// Device address of this device's segment-prefix array for the
// allocation-free batched call (FDAS_NOALLOC_MAX_SPECTRA + 1 int64, a
// file-scope device array; looked up on the first call on each device).
hipError_t noalloc_segpre(int64_t** out);

// Adjoint: window kernel into partA [nzc][nwin][L] / partT [ceil(nwin / G)][K][M]
// (G = backward_window_group(L, M)), then
// the FP64 reductions into grad_spec [N] / grad_taps [K][M] (either may be
// null); the taps reduction sums tsplit window chunks into tpart
// [tsplit][K][M] (FP64) first.
hipError_t launch_backward(const float2* spec, int64_t N, const float2* bank, int K, int M,
                          int L, const float* dLdP, float2* grad_spec, float2* grad_taps,
                          int zchunk, float2* partA, float2* partT, int tsplit, double2* tpart,
                          hipStream_t s);

// Windows per workgroup of the two-gradient adjoint at segment length L and
// M taps (they share one taps transform per template; partT has one [K][M]
// row per group of this many windows).
int backward_window_group(int L, int M);

// Batched adjoint over the spectra of a batched forward: window scan into
// winpre [nspec + 1], the persistent window kernel into partA
// [nzc][maxwin][L] / partT [maxwin][K][M] (maxwin bounds the windows of the
// batch), then the reductions into grad_specs [cap] (packed like the
// spectra; bins outside every spectrum get 0) and grad_taps [K][M] (summed
// over the whole batch); either output may be null.
hipError_t launch_backward_batched(const float2* specs, const int64_t* offsets, int nspec,
                                   int64_t cap, const float2* bank, int K, int M, int L,
                                   const float* dLdP, float2* grad_specs, float2* grad_taps,
                                   int zchunk, int64_t maxwin, int64_t* winpre, float2* partA,
                                   float2* partT, int tsplit, double2* tpart, hipStream_t s);

// Real-to-complex front end (fdas_r2c.hip).  r2c_plan: radix bits per
// global pass for N = 2^log2N complex points (pass count, or -1 if
// unsupported).  launch_r2c: ws holds N work values.
int r2c_plan(int log2N, int bits[4]);
hipError_t launch_r2c(const float* x, int log2n, float scale, float2* spec, float2* ws,
                      hipStream_t s);
// nseries equal-length series one after another: x at stride n floats, ws at
// stride N and spec at stride N + 1 complex values; one launch per pass.
hipError_t launch_r2c_batched(const float* x, int log2n, int nseries, float scale, float2* spec,
                              float2* ws, hipStream_t s);

// Harmonic sums and candidates (fdas_harmonic.hip).
void harmonic_shape(int64_t N, int K, int H, int* KH, int64_t* NH);
hipError_t launch_harmonic_sum(const float* plane, int64_t N, int K, int H, const float* prev,
                               float* out, hipStream_t s);
hipError_t launch_candidates(const float* S, int64_t N, int K, int H, float threshold,
                             fdas_candidate* out, int capacity, unsigned* count, hipStream_t s);
// Batched folds / candidates over the planes of fdas_correlate_batched;
// colpre and prevpre ([nspec + 1] int64 each) hold the fold column prefix
// sums for H and H/2.
hipError_t launch_harmonic_batched(const float* planes, const int64_t* offsets, int nspec, int K,
                                   int H, const float* prev, float* sums, int64_t* colpre,
                                   int64_t* prevpre, hipStream_t s);
hipError_t launch_candidates_batched(const float* sums, const int64_t* offsets, int nspec, int K,
                                     int H, float threshold, fdas_candidate* out, int capacity,
                                     unsigned* count, int64_t* colpre, int64_t* prevpre,
                                     hipStream_t s);

// Streaming probes: n floats written with `value`, or read and summed into
// sums[FDAS_STREAM_PARTIALS] (one partial per workgroup).
hipError_t launch_stream_write(float* dst, int64_t n, float value, hipStream_t s);
hipError_t launch_stream_read(const float* src, int64_t n, float* sums, hipStream_t s);
// LDS bank probe (mode 0/1/2: 64-bit write / 64-bit read / 128-bit write).
hipError_t launch_lds_probe(const int* pattern, int mode, int iters, int groups,
                            long long* cycles, float* sink, hipStream_t s);

}  // namespace fdas
