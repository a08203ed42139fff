// HIP kernels for gfx950: template-bank preparation and the fused forward
// overlap-save correlation (Sec. 3, Fig. 1; Sec. 4.2).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdas_fft.hpp"
#include "fdas_internal.h"

namespace fdas {

// ---- bank preparation (off the hot path) ------------------------------------
//
// H_z[k] = (1/L) sum_j conj(T[z][j]) W_L^{((M/2 - j) mod L) k}: tap j of the
// template placed so that the filter is centred on bin 0, its two halves at
// the ends of the L-array (Sec. 3, Fig. 1).  Accumulated in FP64 with exact
// integer phase indices; one lane per (z, k).
__global__ void bank_rows_kernel(const float2* __restrict__ taps, int K, int M, int L,
                                 float2* __restrict__ bank)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (k >= L || z >= K)
        return;
    const float2* tz = taps + (int64_t)z * M;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < M; ++j) {
        int n = (M / 2 - j) % L;
        if (n < 0)
            n += L;
        const int64_t p = ((int64_t)n * k) & (L - 1);
        double s, c;
        sincospi(-2.0 * (double)p / (double)L, &s, &c);
        const float2 t = tz[j];
        const double hr = t.x, hi = -t.y;   // conj(T)
        sr += hr * c - hi * s;
        si += hr * s + hi * c;
    }
    const double inv = 1.0 / (double)L;
    bank[(int64_t)z * L + k] = make_float2((float)(sr * inv), (float)(si * inv));
}

// Twiddle row: exp(-2 pi i n / L), n in [0, L), FP64 rounded once.
__global__ void bank_twiddle_kernel(int K, int L, float2* __restrict__ bank)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L)
        return;
    double s, c;
    sincospi(-2.0 * (double)n / (double)L, &s, &c);
    bank[(int64_t)K * L + n] = make_float2((float)c, (float)s);
}

hipError_t launch_prepare_bank(const float2* taps, int K, int M, int L, float2* bank,
                               hipStream_t s)
{
    const int bs = 256;
    dim3 grid((L + bs - 1) / bs, K);
    hipLaunchKernelGGL(bank_rows_kernel, grid, dim3(bs), 0, s, taps, K, M, L, bank);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(bank_twiddle_kernel, dim3((L + bs - 1) / bs), dim3(bs), 0, s, K, L, bank);
    return hipGetLastError();
}

// ---- fused forward correlation ---------------------------------------------
//
// One workgroup per (segment s, chunk of templates).  Segment s produces the
// B = L - M outputs [s B, s B + B) from the window of input bins
// [s B - M/2, s B - M/2 + L) (zero outside [0, N)).  Per workgroup:
//   1. coalesced window load (lane t: positions t + T m);
//   2. forward FFT of the window (kept in registers for all templates);
//   3. for each template z of the chunk: multiply by H_z (natural order,
//      next H_z prefetched), inverse FFT, |.|^2, and non-temporal stores of
//      the B valid outputs to plane[z][s B + u].
// Nothing but the valid plane values reaches HBM (Sec. 4.2 first paragraph).
template <int L>
__global__ __launch_bounds__(L / Geometry<L>::E) void forward_kernel(
    const float2* __restrict__ spec, int64_t N, const float2* __restrict__ bank, int K, int M,
    int zchunk, float* __restrict__ plane)
{
    constexpr int E = Geometry<L>::E;
    using F = FFT<L, E, typename Geometry<L>::R>;
    constexpr int T = F::T;
    __shared__ float2 lds[2][LdsSize<L>::value];

    const int t = threadIdx.x;
    const int B = L - M;
    const int64_t s = blockIdx.x;
    const int64_t out0 = s * B;
    const int64_t in0 = out0 - M / 2;
    const int z0 = blockIdx.y * zchunk;
    const int z1 = min(K, z0 + zchunk);

    float2 tw[F::NTW];
    F::twiddles(tw, bank + (int64_t)K * L, t);

    float2 X[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int64_t idx = in0 + t + T * m;
        X[m] = (idx >= 0 && idx < N) ? spec[idx] : make_float2(0.f, 0.f);
    }
    float2* la = lds[0];
    float2* lb = lds[1];
    F::template run<false>(X, la, lb, tw, t);

    float2 H[E];
    {
        const float2* hz = bank + (int64_t)z0 * L + t;
#pragma unroll
        for (int m = 0; m < E; ++m)
            H[m] = hz[T * m];
    }
    for (int z = z0; z < z1; ++z) {
        float2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[m] = cmul(X[m], H[m]);
        if (z + 1 < z1) {
            const float2* hz = bank + (int64_t)(z + 1) * L + t;
#pragma unroll
            for (int m = 0; m < E; ++m)
                H[m] = hz[T * m];
        }
        F::template run<true>(v, la, lb, tw, t);
        float* row = plane + (int64_t)z * N + out0;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int u = t + T * m - M / 2;
            if (u >= 0 && u < B && out0 + u < N) {
                const float p = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                __builtin_nontemporal_store(p, row + u);
            }
        }
    }
}

int default_zchunk(int64_t nseg, int K)
{
    // Enough workgroups to fill 256 CUs several times over; each extra chunk
    // repeats one forward FFT per segment.
    const int64_t target = 4096;
    int64_t chunks = (target + nseg - 1) / (nseg > 0 ? nseg : 1);
    if (chunks < 1) chunks = 1;
    if (chunks > K) chunks = K;
    return (int)((K + chunks - 1) / chunks);
}

template <int L>
static hipError_t launch_forward_L(const float2* spec, int64_t N, const float2* bank, int K,
                                   int M, float* plane, int zchunk, hipStream_t s)
{
    const int B = L - M;
    const int64_t nseg = (N + B - 1) / B;
    const int nzc = (K + zchunk - 1) / zchunk;
    dim3 grid((unsigned)nseg, (unsigned)nzc);
    hipLaunchKernelGGL(forward_kernel<L>, grid, dim3(L / Geometry<L>::E), 0, s, spec, N, bank,
                       K, M, zchunk, plane);
    return hipGetLastError();
}

hipError_t launch_forward(const float2* spec, int64_t N, const float2* bank, int K, int M,
                          int L, float* plane, int zchunk, hipStream_t s)
{
    switch (L) {
    case 256:  return launch_forward_L<256>(spec, N, bank, K, M, plane, zchunk, s);
    case 512:  return launch_forward_L<512>(spec, N, bank, K, M, plane, zchunk, s);
    case 1024: return launch_forward_L<1024>(spec, N, bank, K, M, plane, zchunk, s);
    case 2048: return launch_forward_L<2048>(spec, N, bank, K, M, plane, zchunk, s);
    case 4096: return launch_forward_L<4096>(spec, N, bank, K, M, plane, zchunk, s);
    case 8192: return launch_forward_L<8192>(spec, N, bank, K, M, plane, zchunk, s);
    default:   return hipErrorInvalidValue;
    }
}

}  // namespace fdas
