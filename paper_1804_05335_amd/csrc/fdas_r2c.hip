// Real-to-complex front end: the n FP32 samples of a time series to the
// n/2 + 1 complex bins A[k] = scale * sum_t x[t] exp(-2 pi i k t / n),
// k = 0 .. n/2 (Sec. 4.1: the time series is taken to the Fourier domain
// by a real-to-complex FFT before the correlations).
//
// The n real samples are read as N = n/2 complex points z[m] = x[2m] +
// i x[2m+1] (no copy).  Their length-N DFT Z is computed by a few
// Stockham passes through HBM; the transforms of the even and odd samples,
// E[k] = (Z[k] + conj Z[N-k])/2 and O[k] = (Z[k] - conj Z[N-k])/(2i), are
// then combined into A[k] = E[k] + W_n^k O[k].  From N = 2^13 on this split
// runs inside the last pass (a workgroup takes a tile of butterflies and the
// tile of their mirrors, which hold Z[N-k] for its Z[k]); below, a separate
// kernel does it.
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
// Twiddles are computed in FP64 from exactly represented multiples of pi and
// rounded once: each pass kernel builds the ones its tile needs in LDS while
// its loads are in flight (no table, no table gathers).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdas_fft.hpp"
#include "fdas_internal.h"

namespace fdas {

namespace {

constexpr int kR2cThreads = 256;
constexpr int kR2cTile = 4096;   // complex values per workgroup tile (16 per lane)

// W_D^e = exp(-2 pi i e / D) for D = 2^log2D and 0 <= e < D; -2 e / D is
// exact in FP64, so the only errors are those of sincospi and the final
// rounding.
__device__ __forceinline__ float2 root(int64_t e, int log2D)
{
    double s, c;
    sincospi(ldexp(-(double)e, 1 - log2D), &s, &c);
    return make_float2((float)c, (float)s);
}

template <int RB>
__device__ __forceinline__ void dft_small(float2 (&x)[RB])
{
    static_assert(RB == 16 || RB == 8 || RB == 4 || RB == 2, "RB in {2, 4, 8, 16}");
    float2 w[RB];
    dft_mul<RB, false, kNoMul, false>(x, w);
}

template <int RB>
struct Shape {
    static constexpr int R = 16 * RB;
    static constexpr int logR = 4 + (RB == 16 ? 4 : (RB == 8 ? 3 : (RB == 4 ? 2 : 1)));
    static constexpr int G = kR2cThreads / RB;   // butterflies per tile
    static constexpr int PITCH = R + 1;          // LDS row pitch (complex values)
    static constexpr int KPL = 16 / RB;          // k1 values per lane in stage 2
};

// Stages 1 and 2 of a tile of G butterflies on 256 lanes.  Lane (g, i2)
// enters with x[i1] = input i = RB i1 + i2 of butterfly g; wA[i1 G + g]
// holds the DFT16 multipliers W_{16 NS}^{c i1} (unless FIRST), wR[m] =
// W_R^m and u = W_{NS R}^{c i2}, all written before the caller's last
// barrier.  With WA_IN_TILE, wA lies inside `tile`, so the multipliers are
// read before any tile write.  Leaves output k = (q KPL + r) + 16 k2 of
// butterfly g in y[r][k2] for lane (g, q).
template <int RB, bool FIRST, bool WA_IN_TILE>
__device__ __forceinline__ void tile_stages(float2 (&x)[16], int g, int i2, float2 u,
                                            const float2* wA, const float2* wR, float2* tile,
                                            float2 (&y)[Shape<RB>::KPL][RB])
{
    using S = Shape<RB>;
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
            w[i1] = wA[i1 * S::G + g];
        if constexpr (WA_IN_TILE)
            __syncthreads();
        dft_mul<16, false, kMul, true>(x, w);
    }
    // inner twiddle W_R^{i2 k1} (times u after the first pass; i2 k1 < R),
    // then to LDS as [g][k1 RB + i2]
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
        float2 w = wR[i2 * k1];
        if constexpr (!FIRST)
            w = cmul(w, u);
        tile[g * S::PITCH + k1 * RB + i2] = cmul(x[k1], w);
    }
    __syncthreads();
    // stage 2: lane (g, q) runs DFT_RB over i2 for k1 = q KPL + r
    const int q = i2;
#pragma unroll
    for (int r = 0; r < S::KPL; ++r) {
        const int k1 = q * S::KPL + r;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            y[r][b] = tile[g * S::PITCH + k1 * RB + b];
        dft_small<RB>(y[r]);
    }
}

// One global Stockham pass of radix R = 16 RB over N points, reading `in`
// and writing `out`.
template <int RB, bool FIRST>
__global__ __launch_bounds__(kR2cThreads) void r2c_pass_kernel(
    const float2* __restrict__ in, float2* __restrict__ out, int log2N, int log2NS,
    int64_t in_stride, int64_t out_stride)
{
    // series blockIdx.y of a batch (stride 0 and one series otherwise)
    in += (int64_t)blockIdx.y * in_stride;
    out += (int64_t)blockIdx.y * out_stride;
    using S = Shape<RB>;
    constexpr int R = S::R, G = S::G, PITCH = S::PITCH, KPL = S::KPL;
    __shared__ float2 tile[G * PITCH];
    __shared__ float2 wR[R];                     // W_R^m
    __shared__ float2 wA[FIRST ? 1 : 16 * G];    // W_{16 NS}^{c i1} at [i1 G + g]
    const int t = threadIdx.x;
    const int NS = 1 << log2NS;
    const int64_t stride = (int64_t)1 << (log2N - S::logR);   // N / R
    const int64_t j0 = (int64_t)blockIdx.x * G;

    const int g = t % G, i2 = t / G;
    const int64_t j = j0 + g;
    const int c = (int)(j & (NS - 1));
    float2 x[16];
#pragma unroll
    for (int i1 = 0; i1 < 16; ++i1)
        x[i1] = in[j + (int64_t)(RB * i1 + i2) * stride];
    // the tile's twiddles, while the loads are in flight; G <= NS, so the
    // tile's butterflies have the consecutive c = c0 .. c0 + G - 1
    for (int m = t; m < R; m += kR2cThreads)
        wR[m] = root(m, S::logR);
    float2 u = make_float2(1.f, 0.f);
    if constexpr (!FIRST) {
        const int c0 = (int)(j0 & (NS - 1));
        for (int idx = t; idx < 16 * G; idx += kR2cThreads)
            wA[idx] = root((int64_t)(c0 + idx % G) * (idx / G), log2NS + 4);
        u = root((int64_t)c * i2, log2NS + S::logR);
    }
    __syncthreads();
    float2 y[KPL][RB];
    tile_stages<RB, FIRST, false>(x, g, i2, u, wA, wR, tile, y);
    const int q = i2;
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

// The last pass (NS = N / R: butterfly j has c = j and outputs Z[c + k NS])
// fused with the split.  Output k of butterfly c pairs with Z[N - c - k NS],
// output R-1-k of the mirror butterfly NS - c.  Workgroup w (of NS / (2G))
// takes butterflies c = w G + g on lanes [0, 256) and their mirrors NS - c
// on lanes [256, 512), except that the mirror slot of c = 0 takes c = NS/2:
// 0 and NS/2 are their own mirrors (partners (R-k) mod R and R-1-k).  Every
// butterfly is taken once; each lane writes A[m] = scale (E + W_n^m O) for
// its own outputs m, and the lane with m = 0 also writes A[N].  W_n^m =
// W_n^c W_{2R}^k since W_n^NS = W_{2R}.  Needs NS >= 2G (N >= 2^13).
template <int RB>
__global__ __launch_bounds__(2 * kR2cThreads, 4) void r2c_last_split_kernel(
    const float2* __restrict__ in, float2* __restrict__ A, int log2N, int log2n, float scale,
    int64_t in_stride, int64_t out_stride)
{
    in += (int64_t)blockIdx.y * in_stride;
    A += (int64_t)blockIdx.y * out_stride;
    using S = Shape<RB>;
    constexpr int R = S::R, G = S::G, PITCH = S::PITCH, KPL = S::KPL;
    constexpr int kTile = G * PITCH;
    // two tiles; the DFT16 multipliers of both halves sit in the tile area
    // (read before the first tile write, see tile_stages)
    static_assert(2 * 16 * G <= 2 * kTile, "multipliers fit in the tile area");
    __shared__ float2 lds[2 * kTile];
    __shared__ float2 wR[R];                     // W_R^m
    __shared__ float2 w2R[2 * R];                // W_{2R}^k
    float2* const wA = lds;                      // [h][i1 G + g]
    const int t = threadIdx.x, h = t / kR2cThreads, tt = t % kR2cThreads;
    const int log2NS = log2N - S::logR;
    const int NS = 1 << log2NS;
    const int w = blockIdx.x;
    const int g = tt % G, i2 = tt / G;
    auto butterfly = [&](int hh, int gg) {
        return hh == 0 ? w * G + gg : (w == 0 && gg == 0 ? NS / 2 : NS - w * G - gg);
    };
    const int c = butterfly(h, g);
    float2 x[16];
#pragma unroll
    for (int i1 = 0; i1 < 16; ++i1)
        x[i1] = in[c + (int64_t)(RB * i1 + i2) * NS];
    for (int m = t; m < R; m += 2 * kR2cThreads)
        wR[m] = root(m, S::logR);
    for (int m = t; m < 2 * R; m += 2 * kR2cThreads)
        w2R[m] = root(m, S::logR + 1);
    for (int idx = t; idx < 2 * 16 * G; idx += 2 * kR2cThreads) {
        const int hh = idx / (16 * G), rem = idx % (16 * G);
        wA[idx] = root((int64_t)butterfly(hh, rem % G) * (rem / G), log2NS + 4);
    }
    // u carries the scale/2 of the split: A[m] = (scale/2) (p + W_n^m (-i) d)
    // with p = a + conj b and d = a - conj b, so the scaled outputs a, b of
    // the transform give A[m] = p + W_n^m (d.y, -d.x) directly
    const float2 u0 = root((int64_t)c * i2, log2NS + S::logR);
    const float2 u = make_float2(0.5f * scale * u0.x, 0.5f * scale * u0.y);
    const float2 wc = root(c, log2n);            // W_n^c
    __syncthreads();
    float2 y[KPL][RB];
    tile_stages<RB, false, true>(x, g, i2, u, wA + h * 16 * G, wR, lds + h * kTile, y);
    // exchange the outputs: [h][g][k] in natural k order; output 0 also goes
    // to the pad column R, where the partner index R - k of butterfly 0's
    // output 0 lands
    const int q = i2;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPL; ++r)
#pragma unroll
        for (int k2 = 0; k2 < RB; ++k2)
            lds[h * kTile + g * PITCH + (q * KPL + r) + 16 * k2] = y[r][k2];
    if (q == 0)
        lds[h * kTile + g * PITCH + R] = y[0][0];
    __syncthreads();
    // partner of output k: R - 1 - k of the mirror (own tile for the two
    // self-mirrored butterflies), R - k for butterfly 0
    const bool self = (w == 0 && g == 0);
    const float2* partner = lds + (self ? h : 1 - h) * kTile + g * PITCH +
                            (R - 1 + (self && h == 0 ? 1 : 0) - q * KPL);
    float2* const out = A + c;
#pragma unroll
    for (int r = 0; r < KPL; ++r)
#pragma unroll
        for (int k2 = 0; k2 < RB; ++k2) {
            const int k = (q * KPL + r) + 16 * k2;
            const float2 a = y[r][k2], b = partner[-(r + 16 * k2)];
            const float2 pp = make_float2(a.x + b.x, a.y - b.y);
            const float2 dd = make_float2(a.y + b.y, b.x - a.x);     // -i (a - conj b)
            const float2 wm = cmul(wc, w2R[k]);                       // W_n^(c + k NS)
            out[(int64_t)k * NS] = make_float2(fmaf(wm.x, dd.x, fmaf(-wm.y, dd.y, pp.x)),
                                               fmaf(wm.x, dd.y, fmaf(wm.y, dd.x, pp.y)));
        }
    if (c == 0 && q == 0) {
        // A[N] = scale (E[0] - O[0]) = scale (Re Z[0] - Im Z[0]); y holds
        // (scale/2) Z[0]
        const float2 a = y[0][0];
        A[(int64_t)NS * R] = make_float2(2.f * (a.x - a.y), 0.f);
    }
}

// Separate split for N < 2^13: A[k] and A[N-k] from Z[k] and Z[N-k],
// k in [0, N/2]; Z[N] = Z[0].
__global__ void r2c_split_kernel(const float2* __restrict__ Z, int64_t N, int log2n, float scale,
                                 float2* __restrict__ A, int64_t in_stride, int64_t out_stride)
{
    Z += (int64_t)blockIdx.y * in_stride;
    A += (int64_t)blockIdx.y * out_stride;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > N / 2)
        return;
    const int64_t km = k == 0 ? 0 : N - k;
    const float2 a = Z[k], b = Z[km];
    const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    const float2 o = make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
    const float2 w = root(k, log2n);              // W_n^k, k <= N/2 < n
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
hipError_t pass_L(const float2* in, float2* out, int log2N, int log2NS, bool first,
                  int64_t sin, int64_t sout, unsigned nser, hipStream_t s)
{
    const dim3 blocks((unsigned)(((int64_t)1 << log2N) / kR2cTile), nser);
    if (first)
        hipLaunchKernelGGL((r2c_pass_kernel<RB, true>), blocks, dim3(kR2cThreads), 0, s, in, out,
                           log2N, log2NS, sin, sout);
    else
        hipLaunchKernelGGL((r2c_pass_kernel<RB, false>), blocks, dim3(kR2cThreads), 0, s, in, out,
                           log2N, log2NS, sin, sout);
    return hipGetLastError();
}

template <int RB>
hipError_t last_L(const float2* in, float2* A, int log2N, int log2n, float scale, int64_t sin,
                  int64_t sout, unsigned nser, hipStream_t s)
{
    // NS / (2G) workgroups of 512 lanes per series
    const dim3 blocks((unsigned)(((int64_t)1 << log2N) / (2 * kR2cTile)), nser);
    hipLaunchKernelGGL((r2c_last_split_kernel<RB>), blocks, dim3(2 * kR2cThreads), 0, s, in, A,
                       log2N, log2n, scale, sin, sout);
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

hipError_t launch_r2c_batched(const float* x, int log2n, int nseries, float scale, float2* spec,
                              float2* ws, hipStream_t s)
{
    const int log2N = log2n - 1;
    const int64_t N = (int64_t)1 << log2N;
    int bits[4];
    const int P = r2c_plan(log2N, bits);
    if (P < 1 || nseries < 1 || nseries > 65535)
        return hipErrorInvalidValue;
    const unsigned nser = (unsigned)nseries;
    // per-series strides (complex values); with one series they are unused
    const int64_t sx = N, sws = N, ssp = N + 1;
    auto stride_of = [&](const void* p) {
        return p == (const void*)x ? sx : (p == (const void*)ws ? sws : ssp);
    };
    // From N = 2^13 on (NS >= 2G in the last pass) the last pass carries the
    // split and writes spec; the passes before it alternate so that the one
    // before the last writes ws.  Below, every pass alternates so that the
    // last writes ws, and the split kernel reads ws and writes spec.
    const bool fused = log2N >= 13;
    const int plain = fused ? P - 1 : P;
    const float2* src = reinterpret_cast<const float2*>(x);
    int log2NS = 0;
    for (int p = 0; p < plain; ++p) {
        float2* dst = ((plain - 1 - p) % 2 == 0) ? ws : spec;
        const int64_t si = stride_of(src), so = stride_of(dst);
        hipError_t e;
        switch (bits[p]) {
        case 8: e = pass_L<16>(src, dst, log2N, log2NS, p == 0, si, so, nser, s); break;
        case 7: e = pass_L<8>(src, dst, log2N, log2NS, p == 0, si, so, nser, s); break;
        case 6: e = pass_L<4>(src, dst, log2N, log2NS, p == 0, si, so, nser, s); break;
        case 5: e = pass_L<2>(src, dst, log2N, log2NS, p == 0, si, so, nser, s); break;
        default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess)
            return e;
        src = dst;
        log2NS += bits[p];
    }
    const int64_t si = stride_of(src);
    if (fused) {
        switch (bits[P - 1]) {
        case 8: return last_L<16>(src, spec, log2N, log2n, scale, si, ssp, nser, s);
        case 7: return last_L<8>(src, spec, log2N, log2n, scale, si, ssp, nser, s);
        case 6: return last_L<4>(src, spec, log2N, log2n, scale, si, ssp, nser, s);
        case 5: return last_L<2>(src, spec, log2N, log2n, scale, si, ssp, nser, s);
        default: return hipErrorInvalidValue;
        }
    }
    const int bs = 256;
    const int64_t nthreads = N / 2 + 1;
    hipLaunchKernelGGL(r2c_split_kernel, dim3((unsigned)((nthreads + bs - 1) / bs), nser), dim3(bs),
                       0, s, ws, N, log2n, scale, spec, sws, ssp);
    return hipGetLastError();
}

hipError_t launch_r2c(const float* x, int log2n, float scale, float2* spec, float2* ws,
                      hipStream_t s)
{
    return launch_r2c_batched(x, log2n, 1, scale, spec, ws, s);
}

}  // namespace fdas
