// HIP kernels for gfx950: template-bank preparation, the fused forward
// overlap-save correlation (Sec. 3, Fig. 1; Sec. 4.2), its batched ragged
// form, and the adjoint.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <type_traits>

#include "fdas_fft.hpp"
#include "fdas_internal.h"

namespace fdas {

typedef float f32x2 __attribute__((ext_vector_type(2)));


// ---- range-checked segment access ---------------------------------------------
//
// A segment's window positions q in [0, L) map to output u = q - M/2; only
// q in [M/2, M/2 + nvalid) are valid outputs (nvalid = min(B, N - out0)).
// Per-element branches are replaced by buffer instructions whose resource
// starts at position q = 0 of the row and ends after the last valid output:
// the hardware drops stores past the end and returns 0 for loads past it,
// and positions q < M/2 are given byte offset 2^31, which is past it as
// well.  Offsets are built from non-negative terms only, so no wrap-around
// is involved however the compiler splits them into register and immediate
// parts.
constexpr int kRsrcWord3 = 0x00020000;   // gfx9 raw buffer: 32-bit data format, no swizzle
constexpr int kNonTemporal = 2;          // cache policy: non-temporal

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t seg_rsrc(const void* row_q0, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row_q0), (short)0, bytes,
                                             kRsrcWord3);
}

template <int BYTES>
__device__ __forceinline__ int seg_off(int q, int half_m)
{
    return q >= half_m ? q * BYTES : (int)0x80000000u;
}

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

// DPP lane patterns (gfx9 wave-wide forms): lane i reads lane i + 1
// (lane 63 reads nothing), or lane (i + 1) mod 64.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveRol1 = 0x134;
constexpr float kQuarterPi2 = 0.61685027506808491368f;   // (pi/4)^2, interbinning

//
// Segment s produces the B = L - M outputs [s B, s B + B) from the window of
// input bins [s B - M/2, s B - M/2 + L) (zero outside [0, N)):
//   1. coalesced window load (lane t: positions t + T m);
//   2. forward FFT of the window (kept in registers for all its templates);
//   3. per template z: multiply by H_z (natural order, fused into the first
//      inverse pass), inverse FFT, |.|^2, non-temporal stores of the B valid
//      outputs to plane[z][s B + u].
// Nothing but the valid plane values reaches HBM (Sec. 4.2 first paragraph).
// The LDS ping-pong buffers la/lb keep alternating across calls, so a
// workgroup's consecutive work needs no extra barrier.
template <int L, int EV = Geometry<L>::E>
struct Fwd {
    static constexpr int E = EV;
    using F = FFT<L, E, typename Plan<L, E>::R>;
    static constexpr int T = F::T;
    static constexpr int NTW = F::NTW;
    // interbinned epilogue: waves per workgroup, and the `edge` slots
    // ([wave][E + 1]) of several waves below L = 8192 (at 8192 LDS is full:
    // the slots borrow the free exchange buffer)
    static constexpr int IB_NW = T / 64;
    static constexpr bool IB_OWN_EDGE = IB_NW > 1 && L < 8192;
    static constexpr int kEdgeAlloc = IB_OWN_EDGE ? IB_NW * (E + 1) : 1;

    __device__ static void load_row(float2 (&H)[E], const float2* __restrict__ bank, int row,
                                    int t)
    {
        const float2* h = bank + (int64_t)row * L + t;
#pragma unroll
        for (int m = 0; m < E; ++m)
            H[m] = h[T * m];
    }

    // Symmetric bank (only the rows z >= 0, template index c = (K-1)/2 on):
    // the row of template zi < c is the mirror of row c - zi, since
    // T_{-z} = conj T_z gives H_{-z}[p] = conj H_z[(L - p) mod L].  For lane
    // t and p = t + T m, (L - p) mod L = (b + T (E-1-m)) mod L with
    // b = T - t, so the mirrored row is read like a plain one from the lane
    // base b, in "load order" H[m'] = H_row[(b + T m') mod L] (only lane 0's
    // last slot wraps, to index 0), and its consumer takes
    // H_zi[t + T m] = conj(H[E-1-m]): a register renaming and a conjugate
    // that the multiply absorbs.  Rows zi >= c (row zi - c) load in natural
    // order.  The choice is uniform, so the load has no branch.
    __device__ static void load_row_sym(float2 (&H)[E], const float2* __restrict__ bank, int zi,
                                        int c, int t)
    {
        const bool mir = zi < c;
        const float2* h = bank + (int64_t)(mir ? c - zi : zi - c) * L;
        const int b = mir ? T - t : t;
#pragma unroll
        for (int m = 0; m < E - 1; ++m)
            H[m] = h[b + T * m];
        H[E - 1] = h[(b + T * (E - 1)) & (L - 1)];
    }

    template <bool SYM>
    __device__ static void load_bank_row(float2 (&H)[E], const float2* __restrict__ bank, int zi,
                                         int K, int t)
    {
        if constexpr (SYM)
            load_row_sym(H, bank, zi, (K - 1) / 2, t);
        else
            load_row(H, bank, zi, t);
    }

    __device__ static void load_window(float2 (&X)[E], const float2* __restrict__ spec,
                                       int64_t N, int64_t in0, int t)
    {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int64_t idx = in0 + t + T * m;
            X[m] = (idx >= 0 && idx < N) ? spec[idx] : make_float2(0.f, 0.f);
        }
    }

    // Templates [z0, z1) of segment s.  H holds bank row z0 on entry; each
    // template's successor row (row 0 after the last template, ready for the
    // next segment) is loaded into H as soon as the first inverse pass has
    // consumed it, so the load overlaps the rest of the transform without a
    // second register buffer.
    //
    // IB (interbinning, Sec. 3 eq. f-interp): the plane has 2N columns per
    // row; column 2r holds |y_r|^2 and column 2r+1 |(pi/4)(y_r - y_{r+1})|^2.
    // Each lane gets its right-hand neighbour's y by a DPP lane shift; the
    // segment's spare valid output supplies y_{r+1} for its last output.
    //
    // DUAL (two-bin Fourier interpolation): bank2 holds the half-bin
    // filters on the same segment geometry; per template both inverse
    // transforms run on the window's X (the half-bin row is loaded as soon
    // as the first has consumed the integer row) and the [K][2N] plane gets
    // the pair (|y_r|^2, |y_half_r|^2) in one 8-byte store.
    // DEAD: output slots m < DEAD and m >= E - DEAD hold no valid output in
    // any lane (positions below M/2 or from L - M/2 on, which needs
    // M/2 >= DEAD T); their power and stores are skipped, so the compiler
    // also drops the last butterfly operations that feed only them.
    template <bool IB, bool SYM = false, bool DUAL = false, int DEAD = 0>
    __device__ static void item(const float2* __restrict__ spec, int64_t N,
                                const float2* __restrict__ bank, int K, int M, int64_t s, int z0,
                                int z1, float* __restrict__ plane, const typename F::TW& tw,
                                float2*& la, float2*& lb, int t, float2 (&H)[E],
                                const float2* __restrict__ bank2 = nullptr,
                                float2* __restrict__ edge = nullptr)
    {
        const int B = L - M;
        const int64_t out0 = s * B;
        const int nvalid = (int)min<int64_t>(B, N - out0);   // >= 1: segment s < nseg
        float2 X[E];
        load_window(X, spec, N, out0 - M / 2, t);
        F::template run<false>(X, la, lb, tw, t);

        static_assert(!(SYM && (IB || DUAL)), "the symmetric bank is for the plain plane");
        // One template; MIR: H holds a mirrored row in load order (symmetric
        // bank, z < c), consumed reversed and conjugated.
        auto one = [&](int z, auto mir_tag) {
            constexpr bool MIR = decltype(mir_tag)::value;
            float2 v[E];
            const int znext = z + 1 == K ? 0 : z + 1;
            auto next = [&]() { load_bank_row<SYM>(H, bank, znext, K, t); };
            if constexpr (DUAL) {
                auto half = [&]() { load_row(H, bank2, z, t); };
                F::template run_mul_hook<true, kMul>(X, H, v, la, lb, tw, t, half);
                float p1[E];
#pragma unroll
                for (int m = DEAD; m < E - DEAD; ++m)
                    p1[m] = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                F::template run_mul_hook<true, kMul>(X, H, v, la, lb, tw, t, next);
                const float* row_q0 = plane + 2 * ((int64_t)z * N + out0 - M / 2);
                const auto rs = seg_rsrc(row_q0, (M / 2 + nvalid) * 8);
#pragma unroll
                for (int m = DEAD; m < E - DEAD; ++m) {
                    const float p2 = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                    const u32x2 pp = {__float_as_uint(p1[m]), __float_as_uint(p2)};
                    __builtin_amdgcn_raw_buffer_store_b64(pp, rs, seg_off<8>(t + T * m, M / 2), 0,
                                                          kNonTemporal);
                }
                return;
            }
            if constexpr (MIR) {
                float2 Hr[E];
#pragma unroll
                for (int m = 0; m < E; ++m)
                    Hr[m] = H[E - 1 - m];
                F::template run_mul_hook<true, kMulConj>(X, Hr, v, la, lb, tw, t, next);
            } else if constexpr (!IB) {
                F::template run_mul_hook<true, kMul>(X, H, v, la, lb, tw, t, next);
            } else {
                // the interbinned epilogue holds more values; the next row is
                // loaded once y has gone to LDS, which keeps H out of the
                // transform's register peak
                NoHook none;
                F::template run_mul_hook<true, kMul>(X, H, v, la, lb, tw, t, none);
            }
            if constexpr (!IB) {
                const float* row_q0 = plane + ((int64_t)z * N + out0 - M / 2);
                const auto rs = seg_rsrc(row_q0, (M / 2 + nvalid) * 4);
#pragma unroll
                for (int m = DEAD; m < E - DEAD; ++m) {
                    const float p = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(p), rs,
                                                          seg_off<4>(t + T * m, M / 2), 0,
                                                          kNonTemporal);
                }
            } else if constexpr (IB_NW == 1) {
                // one wave: y at q + 1 = (t + 1) + 64 m is lane t + 1's
                // v[m], and for lane 63 lane 0's v[m + 1]; lane 0 offers
                // v[m + 1] instead of v[m] and a rotation by one lane hands
                // every lane its neighbour (slot E, position L, is never a
                // valid output)
                next();
                const int lane = t & 63;
                const float* row_q0 = plane + 2 * ((int64_t)z * N + out0 - M / 2);
                const auto rs = seg_rsrc(row_q0, (M / 2 + nvalid) * 8);
#pragma unroll
                for (int m = DEAD; m < E - DEAD; ++m) {
                    const float2 nx = m + 1 < E ? v[m + 1] : v[m];
                    const float sx = lane == 0 ? nx.x : v[m].x;
                    const float sy = lane == 0 ? nx.y : v[m].y;
                    const float dx = __int_as_float(__builtin_amdgcn_mov_dpp(
                                         __float_as_int(sx), kDppWaveRol1, 0xf, 0xf, true)) -
                                     v[m].x;
                    const float dy = __int_as_float(__builtin_amdgcn_mov_dpp(
                                         __float_as_int(sy), kDppWaveRol1, 0xf, 0xf, true)) -
                                     v[m].y;
                    const float p = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                    const float h = kQuarterPi2 * fmaf(dx, dx, dy * dy);
                    const u32x2 ph = {__float_as_uint(p), __float_as_uint(h)};
                    __builtin_amdgcn_raw_buffer_store_b64(ph, rs, seg_off<8>(t + T * m, M / 2), 0,
                                                          kNonTemporal);
                }
            } else {
                // several waves: lanes 0..62 take lane t + 1's v[m] by a lane
                // shift; lane 63 takes the next wave's lane 0 at the same m,
                // or in the last wave wave 0's lane 0 at m + 1, from slots
                // each wave's lane 0 fills behind a barrier of their own (an
                // array of their own below L = 8192, so the exchange buffers
                // keep their parity across templates and their addresses stay
                // loop-invariant; at 8192 the free exchange buffer, which
                // then swaps parity once more per template; slot E is read
                // only for position L, never a valid output).  For valid
                // outputs q + 1 <= M/2 + B = L - M/2 stays inside the
                // segment.  Deferring lane 63's pairs to the next transform's
                // first barrier instead leaves 8-byte holes in the plane's
                // lines that a second, partial write fills: measured 1.4-1.8x
                // slower.
                constexpr int NW = IB_NW;
                const int lane = t & 63, wave = t >> 6;
                float2* const ex = IB_OWN_EDGE ? edge : la;
                if (lane == 0) {
                    // slots DEAD .. E - DEAD: the live ones and, one past
                    // them, the spare output at L - M/2
#pragma unroll
                    for (int m = DEAD; m < E - DEAD + (DEAD > 0 ? 1 : 0); ++m)
                        ex[wave * (E + 1) + m] = v[m];
                }
                next();
                __syncthreads();
                const int ew = wave + 1 < NW ? wave + 1 : 0;
                const int em = wave + 1 < NW ? 0 : 1;
                const float* row_q0 = plane + 2 * ((int64_t)z * N + out0 - M / 2);
                const auto rs = seg_rsrc(row_q0, (M / 2 + nvalid) * 8);
#pragma unroll
                for (int m = DEAD; m < E - DEAD; ++m) {
                    const float2 e = ex[ew * (E + 1) + em + m];     // broadcast read
                    // lane t + 1's v[m]; lane 63 keeps e
                    const float bx = __int_as_float(__builtin_amdgcn_update_dpp(
                        __float_as_int(e.x), __float_as_int(v[m].x), kDppWaveShl1, 0xf, 0xf, false));
                    const float by = __int_as_float(__builtin_amdgcn_update_dpp(
                        __float_as_int(e.y), __float_as_int(v[m].y), kDppWaveShl1, 0xf, 0xf, false));
                    const float p = fmaf(v[m].x, v[m].x, v[m].y * v[m].y);
                    const float dx = v[m].x - bx, dy = v[m].y - by;
                    const float h = kQuarterPi2 * fmaf(dx, dx, dy * dy);
                    const u32x2 ph = {__float_as_uint(p), __float_as_uint(h)};
                    __builtin_amdgcn_raw_buffer_store_b64(ph, rs, seg_off<8>(t + T * m, M / 2), 0,
                                                          kNonTemporal);
                }
                if constexpr (!IB_OWN_EDGE) {
                    float2* tmp = la;
                    la = lb;
                    lb = tmp;
                }
            }
        };
        if constexpr (SYM) {
            // the mirrored templates first, then the stored rows: each loop
            // has one multiply form and no per-template branch
            const int zm = min(max((K - 1) / 2, z0), z1);
            for (int z = z0; z < zm; ++z)
                one(z, std::true_type{});
            for (int z = zm; z < z1; ++z)
                one(z, std::false_type{});
        } else {
            for (int z = z0; z < z1; ++z)
                one(z, std::false_type{});
        }
    }
};

// Work partition of the persistent kernels: the flattened (segment,
// template) items [0, total) are split into gridDim.x contiguous ranges, one
// per workgroup, so every workgroup gets the same number of templates (+-1)
// and recomputes a window FFT only where its range enters a segment.
__device__ __forceinline__ void item_range(int64_t total, int64_t& i0, int64_t& i1)
{
    const int64_t P = gridDim.x, w = blockIdx.x;
    i0 = total * w / P;
    i1 = total * (w + 1) / P;
}

// One spectrum of N bins in nseg segments; persistent grid.  IB selects the
// interbinned plane ([K][2N]) instead of the plain one ([K][N]); SYM a bank
// that stores only the z >= 0 rows; DUAL adds the half-bin bank bank2 and
// writes interleaved [K][2N] pairs.
template <int L, bool IB, bool SYM, bool DUAL, int DEAD>
__global__ __launch_bounds__(Fwd<L>::T, 2) void forward_kernel(
    const float2* __restrict__ spec, int64_t N, const float2* __restrict__ bank, int K, int M,
    int64_t nseg, float* __restrict__ plane, const float2* __restrict__ bank2)
{
    using W = Fwd<L>;
    __shared__ __align__(16) float2 lds[2][LdsSize<L>::value];
    __shared__ float2 twl[W::F::kLdsTwAlloc];
    __shared__ __align__(16) float2 edge[IB ? W::kEdgeAlloc : 1];   // interbinning
    int64_t i, i1;
    item_range(nseg * K, i, i1);
    if (i >= i1)
        return;     // uniform across the workgroup, before any barrier
    const int t = threadIdx.x;
    typename W::F::TW tw;
    const int rows = SYM ? (K + 1) / 2 : K;      // bank rows before the twiddle row
    W::F::twiddles(tw, bank + (int64_t)rows * L, twl, t);
    __syncthreads();
    float2* la = lds[0];
    float2* lb = lds[1];
    float2 H[W::E];
    W::template load_bank_row<SYM>(H, bank, (int)(i % K), K, t);
    while (i < i1) {
        const int64_t s = i / K;
        const int zs = (int)(i - s * K);
        const int ze = (int)min<int64_t>(K, zs + (i1 - i));
        W::template item<IB, SYM, DUAL, DEAD>(spec, N, bank, K, M, s, zs, ze, plane, tw, la, lb,
                                               t, H, bank2, edge);
        i += ze - zs;
    }
}

// ---- batched ragged correlation --------------------------------------------
//
// Spectra b = 0..nspec-1 are packed back to back: spectrum b is
// specs[offsets[b] .. offsets[b+1]) and its plane starts at
// planes + K * offsets[b] ([K][N_b] row-major).  A single-workgroup scan
// turns the lengths into segment counts and their prefix sums segpre[0..nspec]
// (segpre[nspec] = total segments); the persistent kernel then splits the
// flattened (segment, template) items of all spectra into contiguous ranges,
// so one launch of a fixed grid covers any batch and every workgroup reaches
// the end of its range.  The offsets are read on the device, so every use
// clamps them to the caller's capacity (the bins specs holds; planes holds K
// times as many floats): an offset past it, or a negative length, makes the
// spectrum shorter or empty, never an access outside the buffers.

constexpr int kScanThreads = 1024;

// Spectrum b's first packed bin and length, clamped to [0, cap].
__device__ __forceinline__ void spec_range(const int64_t* __restrict__ offsets, int b, int64_t cap,
                                           int64_t& off, int64_t& n)
{
    int64_t o0 = offsets[b], o1 = offsets[b + 1];
    o0 = o0 < 0 ? 0 : (o0 > cap ? cap : o0);
    o1 = o1 < o0 ? o0 : (o1 > cap ? cap : o1);
    off = o0;
    n = o1 - o0;
}

// segpre[b + 1] = sum over b' <= b of ceil(N_b' / B) (segments of length B,
// or the adjoint's windows, which have the same count).
__global__ __launch_bounds__(kScanThreads) void segment_scan_kernel(
    const int64_t* __restrict__ offsets, int nspec, int64_t cap, int B, int64_t* __restrict__ segpre)
{
    __shared__ int64_t part[kScanThreads];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) {
        carry = 0;
        segpre[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < nspec; base += kScanThreads) {
        const int b = base + t;
        int64_t segs = 0;
        if (b < nspec) {
            int64_t off, n;
            spec_range(offsets, b, cap, off, n);
            segs = (n + B - 1) / B;
        }
        part[t] = segs;
        __syncthreads();
        // Hillis-Steele inclusive scan over the chunk
        for (int d = 1; d < kScanThreads; d <<= 1) {
            const int64_t add = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        if (b < nspec)
            segpre[b + 1] = carry + part[t];
        __syncthreads();
        if (t == kScanThreads - 1)
            carry += part[t];
        __syncthreads();
    }
}

// The spectrum that owns flattened segment `tile`: the last b with
// segpre[b] <= tile (segpre is non-decreasing, segpre[0] = 0 <= tile).
__device__ __forceinline__ int owner(const int64_t* __restrict__ segpre, int nspec, int64_t tile)
{
    int lo = 0, hi = nspec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segpre[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int L, int E, int DEAD>
__global__ __launch_bounds__((Fwd<L, E>::T), 2) void batched_kernel(
    const float2* __restrict__ specs, const int64_t* __restrict__ offsets,
    const int64_t* __restrict__ segpre, int nspec, int64_t cap, const float2* __restrict__ bank,
    int K, int M, float* __restrict__ planes)
{
    using W = Fwd<L, E>;
    __shared__ __align__(16) float2 lds[2][LdsSize<L>::value];
    __shared__ float2 twl[W::F::kLdsTwAlloc];
    int64_t i, i1;
    item_range(segpre[nspec] * K, i, i1);
    if (i >= i1)
        return;
    const int t = threadIdx.x;
    typename W::F::TW tw;
    W::F::twiddles(tw, bank + (int64_t)K * L, twl, t);
    __syncthreads();
    float2* la = lds[0];
    float2* lb = lds[1];
    float2 H[W::E];
    W::load_row(H, bank, (int)(i % K), t);
    while (i < i1) {
        const int64_t tile = i / K;
        const int zs = (int)(i - tile * K);
        const int ze = (int)min<int64_t>(K, zs + (i1 - i));
        const int b = owner(segpre, nspec, tile);
        int64_t off, Nb;
        spec_range(offsets, b, cap, off, Nb);
        W::template item<false, false, false, DEAD>(specs + off, Nb, bank, K, M,
                                                    tile - segpre[b], zs, ze,
                                                    planes + (int64_t)K * off, tw, la, lb, t, H);
        i += ze - zs;
    }
}

// ---- adjoint (backward) ------------------------------------------------------
//
// Loss Lw = sum_{z,r} w[z][r] P[z][r] with w = dLw/dP given.  In PyTorch's
// complex convention (grad = dLw/dRe + i dLw/dIm), with g = 2 w Y:
//   grad_A[k]    = sum_z sum_j T[z][j] g[z][k - e_j]
//   grad_T[z][j] = sum_r conj(g[z][r]) A[r + e_j].
// Per forward window s (input bins [w0, w0 + L), w0 = s B - M/2; owned outputs
// t in [M/2, M/2 + B)), the correlation is y = IFFT(X H_z) with X = FFT(a_w);
// its adjoint is IFFT(conj(H_z) FFT(g_w)), and the window's part of grad_T is
// the circular cross-correlation IFFT(conj(G) X)/L at lags e_j.  Because g_w
// is supported on the owned outputs only, neither wraps, and summing the
// windows' contributions gives the exact gradients.  Y is recomputed, never
// stored.  Window contributions go to per-(chunk, window) partial buffers and
// are summed in FP64, in a fixed order, by the two reduction kernels.
template <int L>
struct Bwd {
    using W = Fwd<L, BwdGeometry<L>::E>;
    using F = typename W::F;
    static constexpr int E = W::E;
    static constexpr int T = W::T;
    static constexpr int NTW = W::NTW;

    // Templates [z0, z1) of window s.  Hc holds bank row z0 on entry.  Per
    // template the weights w_z are loaded before the inverse transform and
    // the next bank row is loaded once the first pass of FFT(g) has started,
    // so neither load's latency sits on the critical path; row z stays live
    // for the accumulate step.  WANT_T is a compile-time switch: without the
    // taps gradient's transform the kernel needs ~80 fewer VGPRs, which buys
    // a third wave per SIMD.
    // EDGE (M/2 = T exactly): slot 0 holds the positions below M/2 and slot
    // E-1 those from L - M/2 on in every lane.  No window owns them, so g is
    // zero there (w is not read), and they are exactly the taps gradient's
    // lags, which are then stored without a per-lane test; the compiler
    // drops the transform outputs nothing reads.
    template <bool WANT_T, bool EDGE = false>
    __device__ static void item(const float2* __restrict__ spec, int64_t N,
                                const float2* __restrict__ bank, int M, int64_t s, int z0,
                                int z1, const float* __restrict__ dLdP, bool want_A,
                                float2* __restrict__ partA,
                                float2* __restrict__ partT, const typename F::TW& tw,
                                float2*& la, float2*& lb, int t, float2 (&Hc)[E])
    {
        const int B = L - M;
        const int64_t out0 = s * B;
        const int nvalid = (int)min<int64_t>(B, N - out0);   // >= 1: window s < nwin
        float2 X[E];
        W::load_window(X, spec, N, out0 - M / 2, t);
        F::template run<false>(X, la, lb, tw, t);

        float2 acc[E];
#pragma unroll
        for (int m = 0; m < E; ++m)
            acc[m] = make_float2(0.f, 0.f);

        for (int z = z0; z < z1; ++z) {
            // 2 w on the owned outputs, zero elsewhere (w is read exactly once;
            // out-of-range buffer loads return 0)
            const auto rw = seg_rsrc(dLdP + ((int64_t)z * N + out0 - M / 2), (M / 2 + nvalid) * 4);
            float wv[E];
#pragma unroll
            for (int m = 0; m < E; ++m)
                wv[m] = (EDGE && (m == 0 || m == E - 1))
                            ? 0.f
                            : 2.f * __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                        rw, seg_off<4>(t + T * m, M / 2), 0, kNonTemporal));
            float2 v[E];
            F::template run_mul<true, kMul>(X, Hc, v, la, lb, tw, t);     // y = IFFT(X H_z)
#pragma unroll
            for (int m = 0; m < E; ++m)                                   // g = 2 w y
                v[m] = (EDGE && (m == 0 || m == E - 1))
                           ? make_float2(0.f, 0.f)
                           : make_float2(wv[m] * v[m].x, wv[m] * v[m].y);
            float2 Hn[E];
            const int zn = z + 1 < z1 ? z + 1 : z0;
            auto next = [&]() { W::load_row(Hn, bank, zn, t); };
            F::template run_hook<false>(v, la, lb, tw, t, next);          // G = FFT(g)
            if (want_A) {
#pragma unroll
                for (int m = 0; m < E; ++m) {                             // acc += conj(H) G
                    acc[m].x = fmaf(v[m].x, Hc[m].x, fmaf(v[m].y, Hc[m].y, acc[m].x));
                    acc[m].y = fmaf(v[m].y, Hc[m].x, fmaf(-v[m].x, Hc[m].y, acc[m].y));
                }
            }
            if constexpr (WANT_T) {
                F::template run_mul<true, kMulConj>(X, v, v, la, lb, tw, t);  // IFFT(X conj(G))
                float2* pz = partT + (int64_t)z * M;
                if constexpr (EDGE) {
                    pz[t + M / 2] = v[0];                                 // p = t < M/2
                    pz[t] = v[E - 1];                                     // p - L + M/2 = t
                } else {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int p = t + T * m;
                        if (p < M / 2)
                            pz[p + M / 2] = v[m];
                        else if (p >= L - M / 2)
                            pz[p - L + M / 2] = v[m];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < E; ++m)
                Hc[m] = Hn[m];
        }
        if (want_A) {
            F::template run<true>(acc, la, lb, tw, t);
#pragma unroll
            for (int m = 0; m < E; ++m)
                partA[t + T * m] = acc[m];
        }
    }

    // One window of a group: its spectrum, bin count, window index in that
    // spectrum, weights and partial-gradient row.  n = 0 marks an absent
    // window (the group's tail past the last window).
    struct Win {
        const float2* spec;
        int64_t N;
        int64_t s;
        const float* dLdP;
        float2* partA;
    };

    // Both gradients for NW windows at once.  The taps gradient of template
    // z is sum_s IFFT(X_s conj(G_{z,s})) at the lags; the inverse transform
    // is linear, so the group accumulates P_z = sum_s X_s conj(G_{z,s}) in
    // the frequency domain and runs one inverse transform per template for
    // all its windows: 2 + 1/NW transforms per (window, template) instead
    // of 3, and partT holds one [K][M] row per group instead of per window.
    // The spectrum gradient is computed exactly as by item(), window by
    // window (bitwise the same partials).
    template <bool EDGE, int NW>
    __device__ static void item_group(const Win (&win)[NW], const float2* __restrict__ bank,
                                      int M, int z0, int z1, bool want_A,
                                      float2* __restrict__ partT, const typename F::TW& tw,
                                      float2*& la, float2*& lb, int t, float2 (&Hc)[E])
    {
        const int B = L - M;
        float2 X[NW][E];
        float2 acc[NW][E];
        int nvalid[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int64_t out0 = win[w].s * B;
            nvalid[w] = win[w].spec ? (int)min<int64_t>(B, win[w].N - out0) : 0;
            if (win[w].spec) {
                W::load_window(X[w], win[w].spec, win[w].N, out0 - M / 2, t);
                F::template run<false>(X[w], la, lb, tw, t);
            }
#pragma unroll
            for (int m = 0; m < E; ++m)
                acc[w][m] = make_float2(0.f, 0.f);
        }

        for (int z = z0; z < z1; ++z) {
            float2 P[E];
#pragma unroll
            for (int m = 0; m < E; ++m)
                P[m] = make_float2(0.f, 0.f);
            float2 Hn[E];
            const int zn = z + 1 < z1 ? z + 1 : z0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (!win[w].spec)           // uniform: the group's tail
                    continue;
                const int64_t out0 = win[w].s * B;
                const auto rw = seg_rsrc(win[w].dLdP + ((int64_t)z * win[w].N + out0 - M / 2),
                                         (M / 2 + nvalid[w]) * 4);
                float wv[E];
#pragma unroll
                for (int m = 0; m < E; ++m)
                    wv[m] = (EDGE && (m == 0 || m == E - 1))
                                ? 0.f
                                : 2.f * __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                            rw, seg_off<4>(t + T * m, M / 2), 0, kNonTemporal));
                float2 v[E];
                F::template run_mul<true, kMul>(X[w], Hc, v, la, lb, tw, t);   // y
#pragma unroll
                for (int m = 0; m < E; ++m)                                   // g = 2 w y
                    v[m] = (EDGE && (m == 0 || m == E - 1))
                               ? make_float2(0.f, 0.f)
                               : make_float2(wv[m] * v[m].x, wv[m] * v[m].y);
                if (w == NW - 1 || !win[w + 1 < NW ? w + 1 : w].spec) {
                    auto next = [&]() { W::load_row(Hn, bank, zn, t); };
                    F::template run_hook<false>(v, la, lb, tw, t, next);      // G = FFT(g)
                } else {
                    F::template run<false>(v, la, lb, tw, t);
                }
                if (want_A) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {                             // acc += conj(H) G
                        acc[w][m].x = fmaf(v[m].x, Hc[m].x, fmaf(v[m].y, Hc[m].y, acc[w][m].x));
                        acc[w][m].y = fmaf(v[m].y, Hc[m].x, fmaf(-v[m].x, Hc[m].y, acc[w][m].y));
                    }
                }
#pragma unroll
                for (int m = 0; m < E; ++m) {                                 // P += X conj(G)
                    P[m].x = fmaf(X[w][m].x, v[m].x, fmaf(X[w][m].y, v[m].y, P[m].x));
                    P[m].y = fmaf(X[w][m].y, v[m].x, fmaf(-X[w][m].x, v[m].y, P[m].y));
                }
            }
            F::template run<true>(P, la, lb, tw, t);                          // lags
            float2* pz = partT + (int64_t)z * M;
            if constexpr (EDGE) {
                pz[t + M / 2] = P[0];
                pz[t] = P[E - 1];
            } else {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int p = t + T * m;
                    if (p < M / 2)
                        pz[p + M / 2] = P[m];
                    else if (p >= L - M / 2)
                        pz[p - L + M / 2] = P[m];
                }
            }
#pragma unroll
            for (int m = 0; m < E; ++m)
                Hc[m] = Hn[m];
        }
        if (want_A) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (!win[w].spec)
                    continue;
                F::template run<true>(acc[w], la, lb, tw, t);
#pragma unroll
                for (int m = 0; m < E; ++m)
                    win[w].partA[t + T * m] = acc[w][m];
            }
        }
    }
};

template <int L, bool WANT_T, bool EDGE>
__global__ __launch_bounds__(Bwd<L>::T, WANT_T ? BwdGeometry<L>::kMinWaves
                                               : BwdGeometry<L>::kMinWavesSpec) void backward_kernel(
    const float2* __restrict__ spec, int64_t N, const float2* __restrict__ bank, int K, int M,
    int zchunk, int64_t nwin, const float* __restrict__ dLdP, int want_A,
    float2* __restrict__ partA, float2* __restrict__ partT)
{
    using Bk = Bwd<L>;
    __shared__ __align__(16) float2 lds[2][LdsSize<L>::value];
    __shared__ float2 twl[Bk::F::kLdsTwAlloc];
    const int t = threadIdx.x;
    typename Bk::F::TW tw;
    Bk::F::twiddles(tw, bank + (int64_t)K * L, twl, t);
    __syncthreads();
    float2* la = lds[0];
    float2* lb = lds[1];
    const int64_t s = blockIdx.x;
    const int c = blockIdx.y;
    const int z0 = c * zchunk;
    const int z1 = min(K, z0 + zchunk);
    float2 H[Bk::E];
    Bk::W::load_row(H, bank, z0, t);
    constexpr int NW = WANT_T && EDGE ? BwdGeometry<L>::kWinGroupEdge : 1;
    if constexpr (NW == 1) {
        Bk::template item<WANT_T, EDGE>(spec, N, bank, M, s, z0, z1, dLdP, want_A != 0,
                                        partA + ((int64_t)c * nwin + s) * L,
                                        partT + s * (int64_t)K * M, tw, la, lb, t, H);
    } else {
        // workgroup x takes windows x NW .. x NW + NW - 1 (those below nwin)
        typename Bk::Win win[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int64_t sw = s * NW + w;
            const bool ok = sw < nwin;
            win[w] = {ok ? spec : nullptr, N, sw, dLdP,
                      partA + ((int64_t)c * nwin + (ok ? sw : 0)) * L};
        }
        Bk::template item_group<EDGE, NW>(win, bank, M, z0, z1, want_A != 0,
                                          partT + s * (int64_t)K * M, tw, la, lb, t, H);
    }
}

// grad_A[k] = sum over chunks c and windows s covering k of
// partA[c][s][k - (s B - M/2)], summed in FP64 in (c, s) order.
__global__ void reduce_grad_spec_kernel(const float2* __restrict__ partA, int64_t N, int L, int M,
                                        int64_t nwin, int nzc, float2* __restrict__ grad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N)
        return;
    const int B = L - M;
    int64_t s_hi = (k + M / 2) / B;            // windows with s B - M/2 <= k
    if (s_hi > nwin - 1)
        s_hi = nwin - 1;
    const int64_t lo_num = k + M / 2 - L;      // windows with s B - M/2 + L > k
    const int64_t s_lo = lo_num < 0 ? 0 : lo_num / B + 1;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nzc; ++c)
        for (int64_t s = s_lo; s <= s_hi; ++s) {
            const int64_t p = k - (s * B - M / 2);
            const float2 v = partA[((int64_t)c * nwin + s) * L + p];
            sr += v.x;
            si += v.y;
        }
    grad[k] = make_float2((float)sr, (float)si);
}

// grad_T[z][j] = (1/L) sum_s partT[s][z][j] in FP64 (s: the rows of partT,
// one per window or per group of windows), in two fixed-order
// stages.  Stage 1: block (x, y) covers kTapsCols consecutive (z, j) entries
// and the windows s of chunk y; lane row q sums s = s0 + q, s0 + q +
// kTapsRows, ..., the rows are added in order q = 0, 1, ..., and the FP64
// sum goes to tpart[y][(z, j)].  Stage 2 adds the chunks in order y = 0,
// 1, ... and scales.  The chunking depends only on the geometry, so the
// result is deterministic.
constexpr int kTapsCols = 64, kTapsRows = 16;

__global__ __launch_bounds__(kTapsCols * kTapsRows) void reduce_grad_taps_kernel(
    const float2* __restrict__ partT, int64_t nwin, const int64_t* __restrict__ nwin_dev,
    int group, int64_t chunk, int KM, double2* __restrict__ tpart)
{
    __shared__ double part[kTapsRows][kTapsCols][2];
    const int c = threadIdx.x % kTapsCols, q = threadIdx.x / kTapsCols;
    const int i = blockIdx.x * kTapsCols + c;
    // rows present: nwin, or (batched) the groups of the windows actually
    // present (a device window count, rows of `group` windows, at most nwin)
    const int64_t nw = nwin_dev ? min(nwin, (*nwin_dev + group - 1) / group) : nwin;
    const int64_t s0 = (int64_t)blockIdx.y * chunk;
    const int64_t s1 = min(nw, s0 + chunk);
    double sr = 0.0, si = 0.0;
    if (i < KM)
        for (int64_t s = s0 + q; s < s1; s += kTapsRows) {
            const float2 v = partT[s * KM + i];
            sr += v.x;
            si += v.y;
        }
    part[q][c][0] = sr;
    part[q][c][1] = si;
    __syncthreads();
    if (q == 0 && i < KM) {
        double tr = 0.0, ti = 0.0;
        for (int r = 0; r < kTapsRows; ++r) {
            tr += part[r][c][0];
            ti += part[r][c][1];
        }
        tpart[(int64_t)blockIdx.y * KM + i] = make_double2(tr, ti);
    }
}

__global__ void reduce_grad_taps_final_kernel(const double2* __restrict__ tpart, int nsplit,
                                              int KM, int L, float2* __restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KM)
        return;
    double tr = 0.0, ti = 0.0;
    for (int y = 0; y < nsplit; ++y) {
        const double2 v = tpart[(int64_t)y * KM + i];
        tr += v.x;
        ti += v.y;
    }
    const double inv = 1.0 / (double)L;
    grad[i] = make_float2((float)(tr * inv), (float)(ti * inv));
}

// ---- batched adjoint -----------------------------------------------------------
//
// The adjoint over the spectra of a batched forward (packed as for
// batched_kernel, dL/dP packed like the planes).  A window of spectrum b is
// the same window as in the single-spectrum adjoint; windows of all spectra
// are numbered globally by the scan winpre (windows per spectrum =
// ceil(N_b / B), the segment count).  The grid is fixed by the host's bound
// maxwin on the window count (which only offsets that overlap could exceed)
// times the template chunks, so one launch covers any batch within the
// bound and a captured graph serves new batches.  Workgroups past the
// batch's actual window count exit at once, so no partial buffer is overrun.
// One window per workgroup (global window blockIdx.z * gridDim.x +
// blockIdx.x), as in the single-spectrum kernel, so the body allocates the
// same registers (a grid-stride loop over windows made the compiler keep
// more values live and spill).
template <int L, bool WANT_T, bool EDGE>
__global__ __launch_bounds__(Bwd<L>::T, WANT_T ? BwdGeometry<L>::kMinWaves
                                               : BwdGeometry<L>::kMinWavesSpec) void
backward_batched_kernel(const float2* __restrict__ specs, const int64_t* __restrict__ offsets,
                        const int64_t* __restrict__ winpre, int nspec, int64_t cap,
                        const float2* __restrict__ bank, int K, int M, int zchunk, int64_t maxwin,
                        const float* __restrict__ dLdP, int want_A, float2* __restrict__ partA,
                        float2* __restrict__ partT)
{
    using Bk = Bwd<L>;
    __shared__ __align__(16) float2 lds[2][LdsSize<L>::value];
    __shared__ float2 twl[Bk::F::kLdsTwAlloc];
    const int64_t nw = min(winpre[nspec], maxwin);
    const int c = blockIdx.y;
    const int z0 = c * zchunk;
    const int z1 = min(K, z0 + zchunk);
    constexpr int NW = WANT_T && EDGE ? BwdGeometry<L>::kWinGroupEdge : 1;
    const int64_t g = (int64_t)blockIdx.z * gridDim.x + blockIdx.x;   // window, or group
    if (g * NW >= nw)
        return;     // uniform across the workgroup, before any barrier
    const int t = threadIdx.x;
    typename Bk::F::TW tw;
    Bk::F::twiddles(tw, bank + (int64_t)K * L, twl, t);
    __syncthreads();
    float2* la = lds[0];
    float2* lb = lds[1];
    float2 H[Bk::E];
    Bk::W::load_row(H, bank, z0, t);
    if constexpr (NW == 1) {
        const int b = owner(winpre, nspec, g);
        int64_t off, Nb;
        spec_range(offsets, b, cap, off, Nb);
        Bk::template item<WANT_T, EDGE>(specs + off, Nb, bank, M, g - winpre[b], z0, z1,
                                        dLdP + (int64_t)K * off, want_A != 0,
                                        partA + ((int64_t)c * maxwin + g) * L,
                                        partT + g * (int64_t)K * M, tw, la, lb, t, H);
    } else {
        // group g: global windows g NW .. g NW + NW - 1 (those below the
        // batch's count), each from its own spectrum
        typename Bk::Win win[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int64_t gw = g * NW + w;
            if (gw < nw) {
                const int b = owner(winpre, nspec, gw);
                int64_t off, Nb;
                spec_range(offsets, b, cap, off, Nb);
                win[w] = {specs + off, Nb, gw - winpre[b], dLdP + (int64_t)K * off,
                          partA + ((int64_t)c * maxwin + gw) * L};
            } else {
                win[w] = {nullptr, 0, 0, nullptr, partA};
            }
        }
        Bk::template item_group<EDGE, NW>(win, bank, M, z0, z1, want_A != 0,
                                          partT + g * (int64_t)K * M, tw, la, lb, t, H);
    }
}

// grad[k] for every packed bin k < cap: the bins of spectrum b (the last b
// whose clamped range starts at or before k and contains it) sum their
// windows' partials as reduce_grad_spec_kernel does, in the same (chunk,
// window) order, so each spectrum's gradient is bitwise the single-spectrum
// one; bins outside every spectrum get 0.
__global__ void reduce_grad_spec_batched_kernel(const float2* __restrict__ partA,
                                                const int64_t* __restrict__ offsets,
                                                const int64_t* __restrict__ winpre, int nspec,
                                                int64_t cap, int L, int M, int64_t maxwin,
                                                int nzc, float2* __restrict__ grad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cap)
        return;
    if (nspec == 0) {
        grad[k] = make_float2(0.f, 0.f);
        return;
    }
    // the last spectrum whose (clamped) start is <= k
    int lo = 0, hi = nspec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        int64_t o = offsets[mid];
        o = o < 0 ? 0 : (o > cap ? cap : o);
        if (o <= k) lo = mid; else hi = mid - 1;
    }
    int64_t off, n;
    spec_range(offsets, lo, cap, off, n);
    if (k < off || k >= off + n) {
        grad[k] = make_float2(0.f, 0.f);
        return;
    }
    const int64_t kl = k - off;
    const int B = L - M;
    const int64_t nwin = (n + B - 1) / B;
    int64_t s_hi = (kl + M / 2) / B;           // windows with s B - M/2 <= kl
    if (s_hi > nwin - 1)
        s_hi = nwin - 1;
    const int64_t lo_num = kl + M / 2 - L;     // windows with s B - M/2 + L > kl
    const int64_t s_lo = lo_num < 0 ? 0 : lo_num / B + 1;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nzc; ++c)
        for (int64_t s = s_lo; s <= s_hi; ++s) {
            const int64_t g = winpre[lo] + s;
            if (g >= maxwin)
                continue;
            const int64_t p = kl - (s * B - M / 2);
            const float2 v = partA[((int64_t)c * maxwin + g) * L + p];
            sr += v.x;
            si += v.y;
        }
    grad[k] = make_float2((float)sr, (float)si);
}

// ---- launchers -------------------------------------------------------------------

// Resident workgroups of `kernel` on the current device (occupancy x CUs),
// queried once per (device, kernel) and cached so later calls -- e.g. under
// graph capture -- make no runtime queries.
template <class Kern>
static hipError_t resident_grid(Kern kernel, int threads, std::atomic<int>* cache, int* grid)
{
    constexpr int kMaxDev = 64;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev >= 0 && dev < kMaxDev) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) {
            *grid = c;
            return hipSuccess;
        }
    }
    int per_cu = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0)) !=
        hipSuccess)
        return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return e;
    *grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    if (dev >= 0 && dev < kMaxDev)
        cache[dev].store(*grid, std::memory_order_relaxed);
    return hipSuccess;
}

template <int L, bool IB, bool SYM, bool DUAL, int DEAD>
static hipError_t launch_forward_LD(const float2* spec, int64_t N, const float2* bank, int K,
                                    int M, float* plane, int grid, const float2* bank2,
                                    hipStream_t s)
{
    static std::atomic<int> cache[64];
    const int64_t nseg = (N + (L - M) - 1) / (L - M);
    if (grid <= 0) {
        hipError_t e = resident_grid(forward_kernel<L, IB, SYM, DUAL, DEAD>, Fwd<L>::T, cache,
                                     &grid);
        if (e != hipSuccess)
            return e;
    }
    if ((int64_t)grid > nseg * K)
        grid = (int)(nseg * K);
    hipLaunchKernelGGL((forward_kernel<L, IB, SYM, DUAL, DEAD>), dim3(grid), dim3(Fwd<L>::T), 0,
                       s, spec, N, bank, K, M, nseg, plane, bank2);
    return hipGetLastError();
}

// Output slots with no valid output in any lane at each end (0..2): the
// first covers positions below T, the second below 2T, all inside M/2.
template <int L, int E = Geometry<L>::E>
static int dead_slots(int M)
{
    const int d = (M / 2) / Fwd<L, E>::T;
    return d < 2 ? d : 2;
}

template <int L, bool IB, bool SYM, bool DUAL>
static hipError_t launch_forward_L(const float2* spec, int64_t N, const float2* bank, int K,
                                   int M, float* plane, int grid, const float2* bank2,
                                   hipStream_t s)
{
    switch (dead_slots<L>(M)) {
    case 0: return launch_forward_LD<L, IB, SYM, DUAL, 0>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 1: return launch_forward_LD<L, IB, SYM, DUAL, 1>(spec, N, bank, K, M, plane, grid, bank2, s);
    default: return launch_forward_LD<L, IB, SYM, DUAL, 2>(spec, N, bank, K, M, plane, grid, bank2, s);
    }
}

template <bool IB, bool SYM, bool DUAL>
static hipError_t launch_forward_ib(const float2* spec, int64_t N, const float2* bank, int K,
                                    int M, int L, float* plane, int grid, const float2* bank2,
                                    hipStream_t s)
{
    switch (L) {
    case 256:  return launch_forward_L<256, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 512:  return launch_forward_L<512, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 1024: return launch_forward_L<1024, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 2048: return launch_forward_L<2048, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 4096: return launch_forward_L<4096, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    case 8192: return launch_forward_L<8192, IB, SYM, DUAL>(spec, N, bank, K, M, plane, grid, bank2, s);
    default:   return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const float2* spec, int64_t N, const float2* bank, int K, int M,
                          int L, float* plane, int grid, bool interbin, bool sym, hipStream_t s)
{
    if (sym)   // the symmetric bank serves the plain plane only
        return interbin ? hipErrorInvalidValue
                        : launch_forward_ib<false, true, false>(spec, N, bank, K, M, L, plane,
                                                                grid, nullptr, s);
    return interbin
               ? launch_forward_ib<true, false, false>(spec, N, bank, K, M, L, plane, grid,
                                                       nullptr, s)
               : launch_forward_ib<false, false, false>(spec, N, bank, K, M, L, plane, grid,
                                                        nullptr, s);
}

hipError_t launch_forward_dual(const float2* spec, int64_t N, const float2* bank,
                               const float2* bank_half, int K, int Mgeom, int L, float* plane2,
                               int grid, hipStream_t s)
{
    return launch_forward_ib<false, false, true>(spec, N, bank, K, Mgeom, L, plane2, grid,
                                                 bank_half, s);
}

template <int L, int E, int DEAD>
static hipError_t resident_batched_LD(int* grid)
{
    static std::atomic<int> cache[64];
    return resident_grid(batched_kernel<L, E, DEAD>, Fwd<L, E>::T, cache, grid);
}

template <int L, int E>
static hipError_t resident_batched_LE(int M, int* grid)
{
    switch (dead_slots<L, E>(M)) {
    case 0: return resident_batched_LD<L, E, 0>(grid);
    case 1: return resident_batched_LD<L, E, 1>(grid);
    default: return resident_batched_LD<L, E, 2>(grid);
    }
}

template <int L>
static hipError_t resident_batched_L(int E, int M, int* grid)
{
    constexpr int E0 = Geometry<L>::E;
    if (E == 0 || E == E0)
        return resident_batched_LE<L, E0>(M, grid);
    if constexpr (L >= 1024) {
        constexpr int E1 = E0 == 16 ? 8 : 16;
        if (E == E1)
            return resident_batched_LE<L, E1>(M, grid);
    }
    return hipErrorInvalidValue;
}

hipError_t batched_resident_grid(int L, int E, int M, int* grid)
{
    switch (L) {
    case 256:  return resident_batched_L<256>(E, M, grid);
    case 512:  return resident_batched_L<512>(E, M, grid);
    case 1024: return resident_batched_L<1024>(E, M, grid);
    case 2048: return resident_batched_L<2048>(E, M, grid);
    case 4096: return resident_batched_L<4096>(E, M, grid);
    case 8192: return resident_batched_L<8192>(E, M, grid);
    default:   return hipErrorInvalidValue;
    }
}

template <int L, int E, int DEAD>
static hipError_t launch_batched_LD(const float2* specs, const int64_t* offsets, int nspec,
                                    int64_t cap, const float2* bank, int K, int M, float* planes,
                                    int64_t* segpre, int grid, hipStream_t s)
{
    if (grid <= 0) {
        hipError_t e = resident_batched_LD<L, E, DEAD>(&grid);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL((batched_kernel<L, E, DEAD>), dim3(grid), dim3(Fwd<L, E>::T), 0, s, specs,
                       offsets, segpre, nspec, cap, bank, K, M, planes);
    return hipGetLastError();
}

template <int L, int E>
static hipError_t launch_batched_LE(const float2* specs, const int64_t* offsets, int nspec,
                                    int64_t cap, const float2* bank, int K, int M, float* planes,
                                    int64_t* segpre, int grid, hipStream_t s)
{
    switch (dead_slots<L, E>(M)) {
    case 0: return launch_batched_LD<L, E, 0>(specs, offsets, nspec, cap, bank, K, M, planes, segpre, grid, s);
    case 1: return launch_batched_LD<L, E, 1>(specs, offsets, nspec, cap, bank, K, M, planes, segpre, grid, s);
    default: return launch_batched_LD<L, E, 2>(specs, offsets, nspec, cap, bank, K, M, planes, segpre, grid, s);
    }
}

template <int L>
static hipError_t launch_batched_L(const float2* specs, const int64_t* offsets, int nspec,
                                   int64_t cap, const float2* bank, int K, int M, int E,
                                   float* planes, int64_t* segpre, int grid, hipStream_t s)
{
    constexpr int E0 = Geometry<L>::E;
    if (E == 0 || E == E0)
        return launch_batched_LE<L, E0>(specs, offsets, nspec, cap, bank, K, M, planes, segpre, grid, s);
    if constexpr (L >= 1024) {
        constexpr int E1 = E0 == 16 ? 8 : 16;
        if (E == E1)
            return launch_batched_LE<L, E1>(specs, offsets, nspec, cap, bank, K, M, planes, segpre, grid, s);
    }
    return hipErrorInvalidValue;
}

bool batched_values_per_lane_ok(int L, int E)
{
    if (E == 0)
        return true;
    if (L <= 256)
        return E == 4;
    if (L == 512)
        return E == 8;
    return E == 8 || E == 16;
}

// ---- allocation-free batched correlation -------------------------------------
//
// fdas_correlate_batched_noalloc keeps the segment prefix segpre[nspec + 1]
// in this file-scope device array instead of a caller workspace.  Every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept in g_noalloc_ptr.  The scan kernel writes
// every entry the correlation kernel reads (segpre[0] = 0 and segpre[1..nspec]),
// so nothing has to be cleared between calls; calls that overlap on one GPU
// share the array and race.
static __device__ __align__(256) int64_t scratch[FDAS_NOALLOC_MAX_SPECTRA + 1];

constexpr int kMaxDevices = 64;
static std::atomic<int64_t*> g_noalloc_ptr[kMaxDevices];

hipError_t noalloc_segpre(int64_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    int64_t* p = g_noalloc_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        void* addr = nullptr;
        e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!addr)
            return hipErrorInvalidSymbol;
        p = static_cast<int64_t*>(addr);
        g_noalloc_ptr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return hipSuccess;
}

hipError_t launch_batched(const float2* specs, const int64_t* offsets, int nspec, int64_t cap,
                          const float2* bank, int K, int M, int L, int E, float* planes,
                          int64_t* segpre, int grid, hipStream_t s)
{
    if (!batched_values_per_lane_ok(L, E))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(segment_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, offsets, nspec,
                       cap, L - M, segpre);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    switch (L) {
    case 256:  return launch_batched_L<256>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    case 512:  return launch_batched_L<512>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    case 1024: return launch_batched_L<1024>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    case 2048: return launch_batched_L<2048>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    case 4096: return launch_batched_L<4096>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    case 8192: return launch_batched_L<8192>(specs, offsets, nspec, cap, bank, K, M, E, planes, segpre, grid, s);
    default:   return hipErrorInvalidValue;
    }
}

template <int L>
static hipError_t launch_backward_L(const float2* spec, int64_t N, const float2* bank, int K,
                                   int M, int zchunk, int64_t nwin, const float* dLdP,
                                   int want_A, int want_T, float2* partA, float2* partT,
                                   hipStream_t s)
{
    const int nzc = (K + zchunk - 1) / zchunk;
    const dim3 grid((unsigned)nwin, (unsigned)nzc);
    const int NW = backward_window_group(L, M);
    const dim3 grid_t((unsigned)((nwin + NW - 1) / NW), (unsigned)nzc);
    // The edge specialisation pays off with the taps transform (fewer
    // instructions and cycles); without it the compiler waits for the w
    // loads early in the transform and the kernel ran slower, so the
    // spectrum-only kernel keeps the general form.
    if (want_T && M / 2 == Bwd<L>::T)
        hipLaunchKernelGGL((backward_kernel<L, true, true>), grid_t, dim3(Bwd<L>::T), 0, s, spec,
                           N, bank, K, M, zchunk, nwin, dLdP, want_A, partA, partT);
    else if (want_T)
        hipLaunchKernelGGL((backward_kernel<L, true, false>), grid_t, dim3(Bwd<L>::T), 0, s, spec,
                           N, bank, K, M, zchunk, nwin, dLdP, want_A, partA, partT);
    else
        hipLaunchKernelGGL((backward_kernel<L, false, false>), grid, dim3(Bwd<L>::T), 0, s, spec,
                           N, bank, K, M, zchunk, nwin, dLdP, want_A, partA, partT);
    return hipGetLastError();
}

hipError_t launch_backward(const float2* spec, int64_t N, const float2* bank, int K, int M,
                          int L, const float* dLdP, float2* grad_spec, float2* grad_taps,
                          int zchunk, float2* partA, float2* partT, int tsplit, double2* tpart,
                          hipStream_t s)
{
    const int64_t nwin = (N + (L - M) - 1) / (L - M);
    const int want_A = grad_spec != nullptr, want_T = grad_taps != nullptr;
    hipError_t e = hipSuccess;
    if (nwin > 0) {
        switch (L) {
        case 256:  e = launch_backward_L<256>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        case 512:  e = launch_backward_L<512>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        case 1024: e = launch_backward_L<1024>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        case 2048: e = launch_backward_L<2048>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        case 4096: e = launch_backward_L<4096>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        case 8192: e = launch_backward_L<8192>(spec, N, bank, K, M, zchunk, nwin, dLdP, want_A, want_T, partA, partT, s); break;
        default:   return hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess)
        return e;
    const int bs = 256;
    if (want_A && N > 0) {
        const int nzc = (K + zchunk - 1) / zchunk;
        hipLaunchKernelGGL(reduce_grad_spec_kernel, dim3((unsigned)((N + bs - 1) / bs)), dim3(bs),
                           0, s, partA, N, L, M, nwin, nzc, grad_spec);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if (want_T) {
        const int KM = K * M;
        const int NW = backward_window_group(L, M);
        const int64_t ngrp = (nwin + NW - 1) / NW;       // rows of partT
        const int64_t chunk = ngrp > 0 ? (ngrp + tsplit - 1) / tsplit : 1;
        hipLaunchKernelGGL(reduce_grad_taps_kernel,
                           dim3((KM + kTapsCols - 1) / kTapsCols, (unsigned)tsplit),
                           dim3(kTapsCols * kTapsRows), 0, s, partT, ngrp,
                           (const int64_t*)nullptr, 1, chunk, KM, tpart);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(reduce_grad_taps_final_kernel, dim3((KM + bs - 1) / bs), dim3(bs), 0,
                           s, tpart, tsplit, KM, L, grad_taps);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

constexpr int64_t kMaxBwdGridX = int64_t(1) << 22;

template <int L>
static int window_group_L(int M)
{
    return M / 2 == Bwd<L>::T ? BwdGeometry<L>::kWinGroupEdge : 1;
}

int backward_window_group(int L, int M)
{
    switch (L) {
    case 256:  return window_group_L<256>(M);
    case 512:  return window_group_L<512>(M);
    case 1024: return window_group_L<1024>(M);
    case 2048: return window_group_L<2048>(M);
    case 4096: return window_group_L<4096>(M);
    default:   return window_group_L<8192>(M);
    }
}

template <int L>
static hipError_t launch_backward_batched_L(const float2* specs, const int64_t* offsets,
                                            const int64_t* winpre, int nspec, int64_t cap,
                                            const float2* bank, int K, int M, int zchunk,
                                            int64_t maxwin, const float* dLdP, int want_A,
                                            int want_T, float2* partA, float2* partT,
                                            hipStream_t s)
{
    const int nzc = (K + zchunk - 1) / zchunk;
    // one workgroup per (window, chunk), or per (group of windows, chunk)
    // with the taps gradient: items x + gridDim.x * z
    auto grid_for = [&](int64_t items) {
        const int64_t gx = items < kMaxBwdGridX ? items : kMaxBwdGridX;
        return dim3((unsigned)gx, (unsigned)nzc, (unsigned)((items + gx - 1) / (gx > 0 ? gx : 1)));
    };
    if (maxwin < 1)
        return hipSuccess;
    const dim3 grid = grid_for(maxwin);
    const int NW = backward_window_group(L, M);
    const dim3 grid_t = grid_for((maxwin + NW - 1) / NW);
    if (want_T && M / 2 == Bwd<L>::T)
        hipLaunchKernelGGL((backward_batched_kernel<L, true, true>), grid_t, dim3(Bwd<L>::T), 0,
                           s, specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP,
                           want_A, partA, partT);
    else if (want_T)
        hipLaunchKernelGGL((backward_batched_kernel<L, true, false>), grid_t, dim3(Bwd<L>::T), 0,
                           s, specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP,
                           want_A, partA, partT);
    else
        hipLaunchKernelGGL((backward_batched_kernel<L, false, false>), grid, dim3(Bwd<L>::T), 0,
                           s, specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP,
                           want_A, partA, partT);
    return hipGetLastError();
}

hipError_t launch_backward_batched(const float2* specs, const int64_t* offsets, int nspec,
                                   int64_t cap, const float2* bank, int K, int M, int L,
                                   const float* dLdP, float2* grad_specs, float2* grad_taps,
                                   int zchunk, int64_t maxwin, int64_t* winpre, float2* partA,
                                   float2* partT, int tsplit, double2* tpart, hipStream_t s)
{
    const int want_A = grad_specs != nullptr, want_T = grad_taps != nullptr;
    hipLaunchKernelGGL(segment_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, offsets, nspec,
                       cap, L - M, winpre);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    switch (L) {
    case 256:  e = launch_backward_batched_L<256>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    case 512:  e = launch_backward_batched_L<512>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    case 1024: e = launch_backward_batched_L<1024>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    case 2048: e = launch_backward_batched_L<2048>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    case 4096: e = launch_backward_batched_L<4096>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    case 8192: e = launch_backward_batched_L<8192>(specs, offsets, winpre, nspec, cap, bank, K, M, zchunk, maxwin, dLdP, want_A, want_T, partA, partT, s); break;
    default:   return hipErrorInvalidValue;
    }
    if (e != hipSuccess)
        return e;
    const int bs = 256;
    if (want_A && cap > 0) {
        const int nzc = (K + zchunk - 1) / zchunk;
        hipLaunchKernelGGL(reduce_grad_spec_batched_kernel, dim3((unsigned)((cap + bs - 1) / bs)),
                           dim3(bs), 0, s, partA, offsets, winpre, nspec, cap, L, M, maxwin, nzc,
                           grad_specs);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if (want_T) {
        const int KM = K * M;
        const int NW = backward_window_group(L, M);
        const int64_t ngrp = (maxwin + NW - 1) / NW;     // rows of partT
        const int64_t chunk = ngrp > 0 ? (ngrp + tsplit - 1) / tsplit : 1;
        hipLaunchKernelGGL(reduce_grad_taps_kernel,
                           dim3((KM + kTapsCols - 1) / kTapsCols, (unsigned)tsplit),
                           dim3(kTapsCols * kTapsRows), 0, s, partT, ngrp,
                           (const int64_t*)(winpre + nspec), NW, chunk, KM, tpart);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(reduce_grad_taps_final_kernel, dim3((KM + bs - 1) / bs), dim3(bs), 0,
                           s, tpart, tsplit, KM, L, grad_taps);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace fdas
