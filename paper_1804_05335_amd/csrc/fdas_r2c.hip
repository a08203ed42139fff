// Real-to-complex front end: the n FP32 samples of a time series to the
// n/2 + 1 complex bins A[k] = scale * sum_t x[t] exp(-2 pi i k t / n),
// k = 0 .. n/2 (Sec. 4.1: the time series is taken to the Fourier domain
// by a real-to-complex FFT before the correlations).
//
// The n real samples are read as N = n/2 complex points z[m] = x[2m] +
// i x[2m+1] (no copy).  Their length-N DFT Z is computed by a few
// Stockham passes through HBM, and a last pass separates the transforms of
// the even and odd samples, E[k] = (Z[k] + conj Z[N-k])/2 and
// O[k] = (Z[k] - conj Z[N-k])/(2i), into A[k] = E[k] + W_n^k O[k].
//
// Global pass p (radix R = 16 RB, NS = product of the earlier radices):
// butterfly j in [0, N/R) gathers z[j + i N/R], i in [0, R), multiplies by
// W_{NS R}^{(j mod NS) i}, takes the R-point DFT and scatters output k to
// (j / NS) NS R + (j mod NS) + k NS.  A workgroup of 256 lanes takes G =
// 256/RB consecutive butterflies (a 4096-element tile), so every global row
// access covers G consecutive complex values; the R-point DFT inside the
// tile is DFT16 over i1, a twiddle, then DFT_RB over i2 (i = RB i1 + i2),
// with one LDS exchange.  The first pass (NS = 1) writes its tile as one
// contiguous block through LDS; later passes write G-element row chunks.
//
// Twiddles W_n^e come from two tables built in FP64 and rounded once,
// W_n^e = HI[e >> h] * LO[e & (2^h - 1)], one complex multiply each.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdas_fft.hpp"
#include "fdas_internal.h"

namespace fdas {

namespace {

constexpr int kR2cThreads = 256;
constexpr int kR2cTile = 4096;   // complex values per workgroup tile (16 per lane)

struct Twiddles {
    const float2* hi;
    const float2* lo;
    int h;        // lo has 2^h entries
    int mask;     // 2^h - 1
    int nmask;    // n - 1: exponents are taken mod n
};

__device__ __forceinline__ float2 twid(const Twiddles& tw, int e)
{
    e &= tw.nmask;
    return cmul(tw.hi[e >> tw.h], tw.lo[e & tw.mask]);
}

// HI[a] = W_n^{a 2^h}, a in [0, n >> h); LO[b] = W_n^b, b in [0, 2^h).
__global__ void r2c_twiddle_kernel(int log2n, int h, float2* __restrict__ hi,
                                   float2* __restrict__ lo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nhi = 1 << (log2n - h), nlo = 1 << h;
    const double n = (double)(1LL << log2n);
    if (i < nhi) {
        double s, c;
        sincospi(-2.0 * (double)((int64_t)i << h) / n, &s, &c);
        hi[i] = make_float2((float)c, (float)s);
    }
    if (i < nlo) {
        double s, c;
        sincospi(-2.0 * (double)i / n, &s, &c);
        lo[i] = make_float2((float)c, (float)s);
    }
}

template <int RB>
__device__ __forceinline__ void dft_small(float2 (&x)[RB])
{
    static_assert(RB == 16 || RB == 8 || RB == 4 || RB == 2, "RB in {2, 4, 8, 16}");
    float2 w[RB];
    dft_mul<RB, false, kNoMul, false>(x, w);
}

// One global Stockham pass of radix R = 16 RB over N points, reading `in`
// and writing `out`; tw_shift = log2(n / (NS R)) scales W_{NS R} exponents
// to W_n, and int_shift = log2(n / R) does the same for W_R.
template <int RB, bool FIRST>
__global__ __launch_bounds__(kR2cThreads) void r2c_pass_kernel(
    const float2* __restrict__ in, float2* __restrict__ out, int log2N, int log2NS,
    int tw_shift, int int_shift, Twiddles tw)
{
    constexpr int R = 16 * RB;
    constexpr int G = kR2cThreads / RB;          // butterflies per tile
    constexpr int PITCH = R + 1;                 // LDS row pitch (complex values)
    __shared__ float2 tile[G * PITCH];
    const int t = threadIdx.x;
    const int NS = 1 << log2NS;
    const int64_t stride = (int64_t)1 << (log2N - __builtin_ctz(R));   // N / R
    const int64_t j0 = (int64_t)blockIdx.x * G;

    // stage 1: lane (g, i2) holds i = RB i1 + i2, i1 in [0, 16)
    const int g = t % G, i2 = t / G;
    const int64_t j = j0 + g;
    const int c = (int)(j & (NS - 1));
    float2 x[16];
#pragma unroll
    for (int i1 = 0; i1 < 16; ++i1)
        x[i1] = in[j + (int64_t)(RB * i1 + i2) * stride];
    if constexpr (FIRST) {
        float2 w[16];
        dft_mul<16, false, kNoMul, false>(x, w);
    } else {
        // W_{NS R}^{c i} = W_{NS 16}^{c i1} * W_{NS R}^{c i2}: the first factor
        // goes into the DFT16's first stage, the second (constant over i1)
        // joins the inner twiddle below
        float2 w[16];
        w[0] = make_float2(1.f, 0.f);
#pragma unroll
        for (int i1 = 1; i1 < 16; ++i1)
            w[i1] = twid(tw, (c * RB * i1) << tw_shift);
        dft_mul<16, false, kMul, true>(x, w);
    }
    // inner twiddle W_R^{i2 k1} (times W_{NS R}^{c i2} after the first pass),
    // then to LDS as [g][k1 RB + i2]
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
        float2 v = x[k1];
        int e = (i2 * k1) << int_shift;
        if constexpr (!FIRST)
            e += (c * i2) << tw_shift;
        if (e != 0)
            v = cmul(v, twid(tw, e));
        tile[g * PITCH + k1 * RB + i2] = v;
    }
    __syncthreads();

    // stage 2: lane (g, q) runs DFT_RB over i2 for k1 = q*(16/RB) + r
    constexpr int KPL = 16 / RB;                 // k1 values per lane
    const int q = t / G;
    float2 y[KPL][RB];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int k1 = q * KPL + r;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            y[r][b] = tile[g * PITCH + k1 * RB + b];
        dft_small<RB>(y[r]);
    }
    // outputs k = k1 + 16 k2
    if constexpr (FIRST) {
        // out[(j0 + g) R + k]: the tile's outputs are one contiguous block
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KPL; ++r)
#pragma unroll
            for (int k2 = 0; k2 < RB; ++k2)
                tile[g * PITCH + (q * KPL + r) + 16 * k2] = y[r][k2];
        __syncthreads();
        float2* o = out + j0 * R;
#pragma unroll
        for (int m = 0; m < kR2cTile / kR2cThreads; ++m) {
            const int p = t + kR2cThreads * m;
            o[p] = tile[(p / R) * PITCH + (p % R)];
        }
    } else {
        // out[(j / NS) NS R + (j mod NS) + k NS]; NS >= G, so lanes with
        // consecutive g write consecutive addresses
        const int64_t base = (j >> log2NS) * ((int64_t)NS * R) + c;
#pragma unroll
        for (int r = 0; r < KPL; ++r)
#pragma unroll
            for (int k2 = 0; k2 < RB; ++k2)
                out[base + (int64_t)((q * KPL + r) + 16 * k2) * NS] = y[r][k2];
    }
}

// A[k] and A[N-k] from Z[k] and Z[N-k], k in [0, N/2]; Z[N] = Z[0].
__global__ void r2c_split_kernel(const float2* __restrict__ Z, int64_t N, float scale,
                                 Twiddles tw, float2* __restrict__ A)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > N / 2)
        return;
    const int64_t km = k == 0 ? 0 : N - k;
    const float2 a = Z[k], b = Z[km];
    // E = (a + conj b)/2, O = (a - conj b)/(2i), A[k] = E + W_n^k O
    const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    const float2 o = make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
    const float2 w = twid(tw, (int)k);            // W_n^k, k <= N/2 < n
    const float2 wo = cmul(o, w);
    A[k] = make_float2(scale * (e.x + wo.x), scale * (e.y + wo.y));
    // A[N-k] = E[N-k] + W_n^{N-k} O[N-k] = conj(E) - conj(W^k O)
    // (E, O Hermitian in k; W_n^{N-k} = -conj(W_n^k))
    const float2 am = make_float2(scale * (e.x - wo.x), scale * (-e.y + wo.y));
    if (k == 0)
        A[N] = am;
    else if (km != k)
        A[km] = am;
}

template <int RB>
hipError_t pass_L(const float2* in, float2* out, int log2N, int log2NS, int log2n, bool first,
                  const Twiddles& tw, hipStream_t s)
{
    constexpr int R = 16 * RB;
    constexpr int logR = 4 + (RB == 16 ? 4 : (RB == 8 ? 3 : (RB == 4 ? 2 : 1)));
    const int tw_shift = log2n - (log2NS + logR);
    const int int_shift = log2n - logR;
    const unsigned blocks = (unsigned)(((int64_t)1 << log2N) / kR2cTile);
    if (first)
        hipLaunchKernelGGL((r2c_pass_kernel<RB, true>), dim3(blocks), dim3(kR2cThreads), 0, s,
                           in, out, log2N, log2NS, tw_shift, int_shift, tw);
    else
        hipLaunchKernelGGL((r2c_pass_kernel<RB, false>), dim3(blocks), dim3(kR2cThreads), 0, s,
                           in, out, log2N, log2NS, tw_shift, int_shift, tw);
    (void)R;
    return hipGetLastError();
}

}  // namespace

// Radix bits per pass for N = 2^log2N (12 <= log2N <= 26): as few passes as
// possible, each of 5..8 bits (radix 32..256), the largest first.  A pass of
// b bits takes G = 2^(12 - b) consecutive butterflies per tile, which must
// lie in one block of NS (NS >= G, i.e. at least 12 - b bits before it) so
// its output rows are contiguous.  Returns the pass count, or -1.
int r2c_plan(int log2N, int bits[4])
{
    if (log2N < 12 || log2N > 26)
        return -1;
    const int P = (log2N + 7) / 8;
    int left = log2N, before = 0;
    for (int p = 0; p < P; ++p) {
        const int b = (left + (P - p) - 1) / (P - p);   // ceil(left / passes left)
        if (b < 5 || b > 8 || (p > 0 && before < 12 - b))
            return -1;
        bits[p] = b;
        left -= b;
        before += b;
    }
    return P;
}

size_t r2c_table_elems(int log2n)
{
    const int h = (log2n + 1) / 2;
    return ((size_t)1 << (log2n - h)) + ((size_t)1 << h);
}

hipError_t launch_r2c(const float* x, int log2n, float scale, float2* spec, float2* ws,
                      hipStream_t s)
{
    const int log2N = log2n - 1;
    const int64_t N = (int64_t)1 << log2N;
    const int h = (log2n + 1) / 2;
    Twiddles tw;
    float2* tab = ws + N;                         // after the N-point work buffer
    tw.hi = tab;
    tw.lo = tab + ((size_t)1 << (log2n - h));
    tw.h = h;
    tw.mask = (1 << h) - 1;
    tw.nmask = (1 << log2n) - 1;
    {
        const int n_entries = 1 << (log2n - h > h ? log2n - h : h);
        hipLaunchKernelGGL(r2c_twiddle_kernel, dim3((n_entries + 255) / 256), dim3(256), 0, s,
                           log2n, h, const_cast<float2*>(tw.hi), const_cast<float2*>(tw.lo));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    int bits[4];
    const int P = r2c_plan(log2N, bits);
    if (P < 1)
        return hipErrorInvalidValue;
    // buffers: the passes alternate between ws and spec so that the last
    // one writes ws, which the split pass then reads
    const float2* src = reinterpret_cast<const float2*>(x);
    int log2NS = 0;
    for (int p = 0; p < P; ++p) {
        float2* dst = ((P - 1 - p) % 2 == 0) ? ws : spec;
        hipError_t e;
        switch (bits[p]) {
        case 8: e = pass_L<16>(src, dst, log2N, log2NS, log2n, p == 0, tw, s); break;
        case 7: e = pass_L<8>(src, dst, log2N, log2NS, log2n, p == 0, tw, s); break;
        case 6: e = pass_L<4>(src, dst, log2N, log2NS, log2n, p == 0, tw, s); break;
        case 5: e = pass_L<2>(src, dst, log2N, log2NS, log2n, p == 0, tw, s); break;
        default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess)
            return e;
        src = dst;
        log2NS += bits[p];
    }
    const int bs = 256;
    const int64_t nthreads = N / 2 + 1;
    hipLaunchKernelGGL(r2c_split_kernel, dim3((unsigned)((nthreads + bs - 1) / bs)), dim3(bs), 0,
                       s, ws, N, scale, tw, spec);
    return hipGetLastError();
}

}  // namespace fdas
