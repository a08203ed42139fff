// Workgroup FFTs for gfx950: register codelets plus LDS exchanges.
//
// A length-L transform runs on T = L/E lanes of one workgroup, each lane
// holding E complex values.  Between passes lane t always owns positions
// t + T*m (m in [0, E)), so every pass reads coalesced rows from LDS.  Pass
// p (radix R, NS = product of the earlier radices) is a Stockham autosort
// step: butterfly j gathers positions j + i*L/R, applies the twiddles
// W_{NS R}^{(j mod NS) i}, runs a radix-R DFT and scatters to
// (j/NS)*NS*R + (j mod NS) + i*NS.  Input and output are in natural order,
// and after the last pass each output already sits in the register that the
// first pass of the next transform reads -- so the forward transform, the
// template multiply and the inverse transform hand data over in registers
// with no reordering pass.  This is the property the paper obtains by
// pairing a decimation-in-frequency forward FFT with a decimation-in-time
// inverse (Sec. 4.2, around eqs. FFTDIT/FFTDIF); here it comes from the
// autosort formulation, so the template bank can stay in natural order.
//
// Twiddles come from a table exp(-2 pi i n/L) built in FP64 and rounded
// once (no fast-math trigonometry); each lane loads the few it needs once
// and keeps them in registers for every transform it runs.
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// multiply by the fourth root of unity of the transform direction:
// -i for the forward transform, +i for the inverse.
template <bool INV>
__device__ __forceinline__ float2 rot4(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kCos8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kSin8 = 0.38268343236508977173f;   // sin(pi/8)

// The eighth roots of unity W8^1 and W8^3 are sqrt(1/2) times a vector whose
// components are a sum and a difference of the input's.  r81/r83 return that
// unscaled vector, so the scale can be fused into the following additions:
// e +- y W8^k = fma(+-r, sqrt(1/2), e).  The inverse transform uses the
// conjugate roots.
template <bool INV>
__device__ __forceinline__ float2 r81(float2 a)
{
    return INV ? make_float2(a.x - a.y, a.x + a.y) : make_float2(a.x + a.y, a.y - a.x);
}
template <bool INV>
__device__ __forceinline__ float2 r83(float2 a)
{
    return INV ? make_float2(-(a.x + a.y), a.x - a.y) : make_float2(a.y - a.x, -(a.x + a.y));
}

// e + k r and e - k r, two FMAs per component.
__device__ __forceinline__ void fbfly(float2& hi, float2& lo, float2 e, float2 r, float k)
{
    hi = make_float2(fmaf(r.x, k, e.x), fmaf(r.y, k, e.y));
    lo = make_float2(fmaf(-r.x, k, e.x), fmaf(-r.y, k, e.y));
}

// a + b and a - b
__device__ __forceinline__ void bfly(float2& hi, float2& lo, float2 a, float2 b)
{
    hi = cadd(a, b);
    lo = csub(a, b);
}

// ---- radix-R DFT codelets, natural order in and out ----------------------
//
// Every codelet starts with radix-2 butterflies pairing element i with
// i + R/2.  That first stage is split out so a per-element multiplier (a
// twiddle, or the template H) can be fused into it with FMAs:
//   a = x_i w_i,  s = a + x_{i+R/2} w_{i+R/2} (4 FMA),  d = 2a - s (2 FMA),
// 10 instructions per pair instead of 12 (6 instead of 8 when w_i = 1).

enum MulMode { kNoMul = 0, kMul = 1, kMulConj = 2 };

template <int MODE>
__device__ __forceinline__ float2 mulw(float2 x, float2 w)
{
    if constexpr (MODE == kMul) return cmul(x, w);
    else if constexpr (MODE == kMulConj) return cmulc(x, w);
    else return x;
}

// a + x*w (or a + x*conj(w)) in 4 FMAs
template <int MODE>
__device__ __forceinline__ float2 add_mulw(float2 a, float2 x, float2 w)
{
    if constexpr (MODE == kMul)
        return make_float2(fmaf(x.x, w.x, fmaf(-x.y, w.y, a.x)), fmaf(x.x, w.y, fmaf(x.y, w.x, a.y)));
    else if constexpr (MODE == kMulConj)
        return make_float2(fmaf(x.x, w.x, fmaf(x.y, w.y, a.x)), fmaf(x.y, w.x, fmaf(-x.x, w.y, a.y)));
    else
        return cadd(a, x);
}

// First stage: x[i], x[i+R/2] <- a + b, a - b with a = x[i] w[i], b = x[i+R/2] w[i+R/2].
// FIRST_ONE: w[0] is 1 (not read).
template <int R, int MODE, bool FIRST_ONE>
__device__ __forceinline__ void stage1(float2 (&x)[R], const float2 (&w)[R])
{
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
        if constexpr (MODE == kNoMul) {
            const float2 a = x[i], b = x[i + R / 2];
            x[i] = cadd(a, b);
            x[i + R / 2] = csub(a, b);
        } else {
            const float2 a = (FIRST_ONE && i == 0) ? x[i] : mulw<MODE>(x[i], w[i]);
            const float2 sum = add_mulw<MODE>(a, x[i + R / 2], w[i + R / 2]);
            x[i] = sum;
            x[i + R / 2] = make_float2(fmaf(2.f, a.x, -sum.x), fmaf(2.f, a.y, -sum.y));
        }
    }
}

// Remaining stages, given stage1 has run.  All arithmetic is spelled out
// (the library is built without implicit FMA contraction, so every
// instantiation rounds identically).
template <bool INV>
__device__ __forceinline__ void rest4(float2& x0, float2& x1, float2& x2, float2& x3)
{
    // after stage 1: x0 = t0, x2 = t1, x1 = t2, x3 = t3' (pairs (0,2), (1,3))
    const float2 t0 = x0, t1 = x2, t2 = x1, t3 = rot4<INV>(x3);
    bfly(x0, x2, t0, t2);
    bfly(x1, x3, t1, t3);
}

// DFT4 of (a0, a1, a2, a3) given s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3,
// d13 = a1 - a3: outputs X0..X3.
template <bool INV>
__device__ __forceinline__ void dft4_tail(float2& X0, float2& X1, float2& X2, float2& X3, float2 s02,
                                          float2 d02, float2 s13, float2 d13)
{
    bfly(X0, X2, s02, s13);
    bfly(X1, X3, d02, rot4<INV>(d13));
}

template <int R, bool INV>
__device__ __forceinline__ void rest(float2 (&x)[R])
{
    if constexpr (R == 2) {
        // nothing after the single butterfly
    } else if constexpr (R == 4) {
        rest4<INV>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 8) {
        // evens e = (x0, x2, x4, x6), odds o = (x1, x3, x5, x7); stage 1 paired
        // (0,4), (2,6), (1,5), (3,7), i.e. the first stage of both radix-4 DFTs;
        // then X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]
        float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
        float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
        rest4<INV>(e0, e1, e2, e3);
        rest4<INV>(o0, o1, o2, o3);
        bfly(x[0], x[4], e0, o0);
        fbfly(x[1], x[5], e1, r81<INV>(o1), kSqrtHalf);
        bfly(x[2], x[6], e2, rot4<INV>(o2));
        fbfly(x[3], x[7], e3, r83<INV>(o3), kSqrtHalf);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.  Stage 1 paired (n2, 8+n2)
        // and (4+n2, 12+n2): the first stage of each radix-4 DFT over n1.
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2)
            rest4<INV>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);
        // x[4 k1 + n2] holds Y[n2][k1]; row k1 is a DFT4 over n2 of
        // a_n2 = Y[n2][k1] W16^(n2 k1), with the twiddle fused into its first
        // stage.  W16^2 = W8^1, W16^4 = rot4, W16^6 = W8^3, W16^9 = -W16^1.
        const float2 w1 = make_float2(kCos8, INV ? kSin8 : -kSin8);
        const float2 w3 = make_float2(kSin8, INV ? kCos8 : -kCos8);
        const float2 w9 = make_float2(-kCos8, INV ? -kSin8 : kSin8);
        float2 s02, d02, s13, d13;
        // row 0: no twiddles
        bfly(s02, d02, x[0], x[2]);
        bfly(s13, d13, x[1], x[3]);
        dft4_tail<INV>(x[0], x[1], x[2], x[3], s02, d02, s13, d13);
        // row 1: (1, W1, W2, W3)
        fbfly(s02, d02, x[4], r81<INV>(x[6]), kSqrtHalf);
        {
            const float2 a = cmul(x[5], w1);
            s13 = add_mulw<kMul>(a, x[7], w3);
            d13 = make_float2(fmaf(2.f, a.x, -s13.x), fmaf(2.f, a.y, -s13.y));
        }
        dft4_tail<INV>(x[4], x[5], x[6], x[7], s02, d02, s13, d13);
        // row 2: (1, W2, W4, W6); W2 y1 +- W6 y3 = W8^1 (y1 +- rot4(y3))
        bfly(s02, d02, x[8], rot4<INV>(x[10]));
        {
            float2 c, e;
            bfly(c, e, x[9], rot4<INV>(x[11]));
            const float2 pc = r81<INV>(c), pe = rot4<INV>(r81<INV>(e));
            fbfly(x[8], x[10], s02, pc, kSqrtHalf);
            fbfly(x[9], x[11], d02, pe, kSqrtHalf);
        }
        // row 3: (1, W3, W6, W9)
        fbfly(s02, d02, x[12], r83<INV>(x[14]), kSqrtHalf);
        {
            const float2 a = cmul(x[13], w3);
            s13 = add_mulw<kMul>(a, x[15], w9);
            d13 = make_float2(fmaf(2.f, a.x, -s13.x), fmaf(2.f, a.y, -s13.y));
        }
        dft4_tail<INV>(x[12], x[13], x[14], x[15], s02, d02, s13, d13);
        // x[4 k1 + k2] holds X[k1 + 4 k2]; transpose the 4x4 index back
        float2 y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2)
                y[k1 + 4 * k2] = x[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            x[i] = y[i];
    } else {
        static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
    }
}

// DFT_R of x[i] * w[i] (MODE selects the multiplier; FIRST_ONE: w[0] = 1).
template <int R, bool INV, int MODE, bool FIRST_ONE>
__device__ __forceinline__ void dft_mul(float2 (&x)[R], const float2 (&w)[R])
{
    stage1<R, MODE, FIRST_ONE>(x, w);
    rest<R, INV>(x);
}

// ---- transform plans ---------------------------------------------------------

template <int... Rs>
struct Radices {};

// Number of register twiddles a lane keeps for the passes from NS on (the
// pass whose stride is LNS takes its twiddles from an LDS table instead).
template <int L, int E, int NS, int LNS, class RL>
struct TwiddleCount;
template <int L, int E, int NS, int LNS>
struct TwiddleCount<L, E, NS, LNS, Radices<>> {
    static constexpr int value = 0;
};
template <int L, int E, int NS, int LNS, int R, int... Rest>
struct TwiddleCount<L, E, NS, LNS, Radices<R, Rest...>> {
    static constexpr int value = (NS > 1 && NS != LNS ? (E / R) * (R - 1) : 0) +
                                 TwiddleCount<L, E, NS * R, LNS, Radices<Rest...>>::value;
};

// LDS index of transform value idx.  gfx950 serves a 64-bit LDS read in
// two passes of 32 lanes over 64 four-byte banks, a 64-bit write in four
// passes of 16 lanes over 32 banks and a 128-bit write in eight passes of 8
// lanes (measured), so an exchange is conflict-free when each 32-lane group
// of a read touches 32 distinct values mod 32, each 16-lane group of a 64-bit
// write 16 distinct values mod 16, and each 8-lane group of a 128-bit write 8
// distinct value pairs mod 8.  Both maps XOR the low bits of idx with a
// GF(2)-linear function of h = idx >> 4, which permutes every aligned
// 16-value block (so the row reads, aligned 32-value blocks, stay
// conflict-free); the function's columns are chosen so that the strided
// writes of every plan -- stride 4, 8 or 16 in the first pass, runs of 4 or
// 8 values 16 or 64 apart in the second -- fall on distinct banks:
//   PAIR = false (64-bit writes throughout): bits 0..3 XOR G(h & 15), columns
//     G(1) = 5, G(2) = 10, G(4) = 12, G(8) = 1;
//   PAIR = true (the first pass writes adjacent pairs (2q, 2q + 1) as one
//     128-bit store, so bit 0 must stay): bits 1..3 XOR 2 G(h & 7), columns
//     G(1) = 3, G(2) = 6, G(4) = 4.
template <bool PAIR>
__device__ __forceinline__ int lds_pad(int idx)
{
    const int h = idx >> 4;
    if constexpr (PAIR) {
        const int g = ((h & 1) ? 3 : 0) ^ ((h & 2) ? 6 : 0) ^ ((h & 4) ? 4 : 0);
        return idx ^ (g << 1);
    } else {
        const int g = ((h & 1) ? 5 : 0) ^ ((h & 2) ? 10 : 0) ^ ((h & 4) ? 12 : 0) ^
                      ((h & 8) ? 1 : 0);
        return idx ^ g;
    }
}

// The first pass stores adjacent output pairs with 128-bit writes at
// L = 8192 only.  Measured: there it frees the registers that the 64-bit
// stores' extra addresses take (the 8-wave workgroups run short of them);
// at L <= 4096 the 64-bit stores timed faster.
template <int L>
struct PairWrites {
    static constexpr bool value = L >= 8192;
};

template <int L>
struct LdsSize {
    static constexpr int value = L;
};

// Load the twiddles for passes NS.. into tw[OFF..] (all but the pass of
// stride LNS).
template <int L, int E, int NS, int OFF, int NTW, int LNS, int R, int... Rest>
__device__ __forceinline__ void load_twiddles(float2 (&tw)[NTW], const float2* __restrict__ table, int t)
{
    constexpr int T = L / E, NB = E / R;
    constexpr bool REG = NS > 1 && NS != LNS;
    if constexpr (REG) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = t + u * T;
            const int base = (j & (NS - 1)) * (L / (NS * R));
#pragma unroll
            for (int i = 1; i < R; ++i)
                tw[OFF + u * (R - 1) + (i - 1)] = table[base * i];
        }
    }
    if constexpr (sizeof...(Rest) > 0)
        load_twiddles<L, E, NS * R, OFF + (REG ? NB * (R - 1) : 0), NTW, LNS, Rest...>(tw, table,
                                                                                     t);
}

// Run the passes from NS on.  The first of them reads `in` (positions
// t + T*m of this lane), the rest read v; on return v holds the transform at
// the same positions (in and v may be the same array; `in` is not written
// unless it is v).  The first pass (NS = 1) may fuse a per-element
// multiplier pre[m] (MODE0: kMul or kMulConj) into its first butterfly
// stage; later passes fuse their twiddles the same way.  Exchanges
// ping-pong between the two LDS buffers (one barrier each).
struct NoHook {
    __device__ void operator()() const {}
};

template <int L, int E, bool INV, int MODE0, int NS, int OFF, int NTW, int LNS, class Hook, int R,
          int... Rest>
__device__ __forceinline__ void run_passes(const float2 (&in)[E], const float2 (&pre)[E],
                                           float2 (&v)[E], float2*& lds_a, float2*& lds_b,
                                           const float2 (&tw)[NTW],
                                           const float2* __restrict__ twl, int t, Hook& hook)
{
    constexpr int T = L / E, NB = E / R;
    constexpr bool LAST = sizeof...(Rest) == 0;
    constexpr bool REG = NS > 1 && NS != LNS;
    constexpr bool PAIR = PairWrites<L>::value;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        float2 x[R];
#pragma unroll
        for (int i = 0; i < R; ++i)
            x[i] = in[u + i * NB];
        if constexpr (REG) {
            float2 w[R];
            w[0] = make_float2(1.f, 0.f);
#pragma unroll
            for (int i = 1; i < R; ++i)
                w[i] = tw[OFF + u * (R - 1) + (i - 1)];
            dft_mul<R, INV, INV ? kMulConj : kMul, true>(x, w);
        } else if constexpr (NS > 1) {
            // twiddles W_{NS R}^(c i), c = j mod NS, from the LDS table laid
            // out [i - 1][c] (the lanes of a row read consecutive entries)
            const int c = (t + u * T) & (NS - 1);
            float2 w[R];
            w[0] = make_float2(1.f, 0.f);
#pragma unroll
            for (int i = 1; i < R; ++i)
                w[i] = twl[(i - 1) * NS + c];
            dft_mul<R, INV, INV ? kMulConj : kMul, true>(x, w);
        } else if constexpr (MODE0 != kNoMul) {
            float2 w[R];
#pragma unroll
            for (int i = 0; i < R; ++i)
                w[i] = pre[u + i * NB];
            dft_mul<R, INV, MODE0, false>(x, w);
        } else {
            float2 w[R];
            dft_mul<R, INV, kNoMul, false>(x, w);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int i = 0; i < R; ++i)
                v[u + i * NB] = x[i];
        } else if constexpr (NS == 1 && PAIR) {
            // butterfly j's outputs are the contiguous values j R .. j R + R - 1:
            // adjacent pairs go out as single 128-bit stores
            const int j = t + u * T;
            float4* dst = reinterpret_cast<float4*>(lds_a);
#pragma unroll
            for (int q = 0; q < R / 2; ++q)
                dst[lds_pad<PAIR>(j * R + 2 * q) >> 1] =
                    make_float4(x[2 * q].x, x[2 * q].y, x[2 * q + 1].x, x[2 * q + 1].y);
        } else {
            const int j = t + u * T;
            const int idxD = (j / NS) * (NS * R) + (j & (NS - 1));
#pragma unroll
            for (int i = 0; i < R; ++i)
                lds_a[lds_pad<PAIR>(idxD + i * NS)] = x[i];
        }
    }
    if constexpr (NS == 1)
        hook();     // `in` and `pre` are no longer read: their registers may be reloaded
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[m] = lds_a[lds_pad<PAIR>(t + m * T)];
        float2* tmp = lds_a;
        lds_a = lds_b;
        lds_b = tmp;
        NoHook none;
        run_passes<L, E, INV, kNoMul, NS * R, OFF + (REG ? NB * (R - 1) : 0), NTW, LNS, NoHook,
                   Rest...>(v, pre, v, lds_a, lds_b, tw, twl, t, none);
    }
}

template <int L, int E, class RL>
struct FFT;

// Radix of the pass whose stride is NS_AT (0 if none).
template <int NS_AT, int NS, int... Rs>
struct RadixAt {
    static constexpr int value = 0;
};
template <int NS_AT, int NS, int R, int... Rest>
struct RadixAt<NS_AT, NS, R, Rest...> {
    static constexpr int value = NS == NS_AT ? R : RadixAt<NS_AT, NS * R, Rest...>::value;
};

template <int... Rs>
struct LastRadix;
template <int R>
struct LastRadix<R> {
    static constexpr int value = R;
};
template <int R, int R2, int... Rest>
struct LastRadix<R, R2, Rest...> {
    static constexpr int value = LastRadix<R2, Rest...>::value;
};

template <int L, int E, int... Rs>
struct FFT<L, E, Radices<Rs...>> {
    static constexpr int T = L / E;
    // One pass may take its twiddles from a table in LDS instead of
    // registers: at L = 8192 the last one (radix 2, stride L/2: one twiddle
    // per butterfly, a 32 KB table), which frees the registers the longest
    // transform runs short of.  (Taking the second pass's 15 twiddles per
    // lane from LDS in the interbinned kernel freed 20 VGPRs there but timed
    // 0.2 % slower.)
    static constexpr int kLNS = (L >= 8192 && LastRadix<Rs...>::value == 2) ? L / 2 : 0;
    static constexpr int kLR = kLNS > 0 ? RadixAt<kLNS, 1, Rs...>::value : 0;
    static_assert(kLNS == 0 || kLR > 0, "the LDS-twiddle stride must be a pass's");
    static constexpr int kLdsTw = kLNS > 0 ? (kLR - 1) * kLNS : 0;   // table entries
    static constexpr int kLdsTwAlloc = kLdsTw > 0 ? kLdsTw : 1;
    static constexpr int NTW = TwiddleCount<L, E, 1, kLNS, Radices<Rs...>>::value > 0
                                   ? TwiddleCount<L, E, 1, kLNS, Radices<Rs...>>::value : 1;
    static_assert((1 * ... * Rs) == L, "radices must multiply to L");
    static_assert(((E % Rs == 0) && ...), "every radix must divide E");

    // A lane's twiddles: registers, plus the workgroup's LDS table.
    struct TW {
        float2 r[NTW];
        const float2* lds;
    };

    // Load the register twiddles and, if the plan has one, fill the LDS
    // table lds_table[kLdsTw] from the twiddle row (every lane takes part;
    // the caller synchronises the workgroup before the first transform).
    __device__ static void twiddles(TW& tw, const float2* __restrict__ table, float2* lds_table,
                                    int t)
    {
        load_twiddles<L, E, 1, 0, NTW, kLNS, Rs...>(tw.r, table, t);
        if constexpr (kLdsTw > 0) {
            // entry (i - 1) kLNS + c = W_{kLNS kLR}^(c i) = W_L^(c i L / (kLNS kLR))
            for (int n = t; n < kLdsTw; n += T) {
                const int i = n / kLNS + 1, c = n % kLNS;
                lds_table[n] = table[c * i * (L / (kLNS * kLR))];
            }
        }
        tw.lds = lds_table;
    }
    // transform of v (forward: INV = false)
    template <bool INV>
    __device__ static void run(float2 (&v)[E], float2*& lds_a, float2*& lds_b, const TW& tw, int t)
    {
        NoHook none;
        run_passes<L, E, INV, kNoMul, 1, 0, NTW, kLNS, NoHook, Rs...>(v, v, v, lds_a, lds_b, tw.r,
                                                                      tw.lds, t, none);
    }
    // as run; hook() runs once the first pass has read v
    template <bool INV, class Hook>
    __device__ static void run_hook(float2 (&v)[E], float2*& lds_a, float2*& lds_b, const TW& tw,
                                    int t, Hook& hook)
    {
        run_passes<L, E, INV, kNoMul, 1, 0, NTW, kLNS, Hook, Rs...>(v, v, v, lds_a, lds_b, tw.r,
                                                                    tw.lds, t, hook);
    }
    // v = transform of in[m] * pre[m] (MODE kMul) or in[m] * conj(pre[m]) (kMulConj)
    template <bool INV, int MODE>
    __device__ static void run_mul(const float2 (&in)[E], const float2 (&pre)[E], float2 (&v)[E],
                                   float2*& lds_a, float2*& lds_b, const TW& tw, int t)
    {
        NoHook none;
        run_passes<L, E, INV, MODE, 1, 0, NTW, kLNS, NoHook, Rs...>(in, pre, v, lds_a, lds_b,
                                                                    tw.r, tw.lds, t, none);
    }
    // as run_mul; hook() runs once the first pass has consumed `in` and `pre`
    template <bool INV, int MODE, class Hook>
    __device__ static void run_mul_hook(const float2 (&in)[E], const float2 (&pre)[E],
                                        float2 (&v)[E], float2*& lds_a, float2*& lds_b,
                                        const TW& tw, int t, Hook& hook)
    {
        run_passes<L, E, INV, MODE, 1, 0, NTW, kLNS, Hook, Rs...>(in, pre, v, lds_a, lds_b, tw.r,
                                                                  tw.lds, t, hook);
    }
};

// Radix sequence for a length-L transform with E values per lane (every
// radix divides E, their product is L).
template <int L, int E>
struct Plan;
template <> struct Plan<256, 4>   { using R = Radices<4, 4, 4, 4>; };
template <> struct Plan<512, 8>   { using R = Radices<8, 8, 8>; };
template <> struct Plan<1024, 8>  { using R = Radices<8, 8, 8, 2>; };
template <> struct Plan<1024, 16> { using R = Radices<16, 16, 4>; };
template <> struct Plan<2048, 8>  { using R = Radices<8, 8, 8, 4>; };
template <> struct Plan<2048, 16> { using R = Radices<16, 16, 8>; };
template <> struct Plan<4096, 8>  { using R = Radices<8, 8, 8, 8>; };
template <> struct Plan<4096, 16> { using R = Radices<16, 16, 16>; };
template <> struct Plan<8192, 8>  { using R = Radices<8, 8, 8, 8, 2>; };
template <> struct Plan<8192, 16> { using R = Radices<16, 16, 16, 2>; };

// Values per lane of the forward kernels: 16 from L = 1024 on (two LDS
// exchanges per transform, 256 VGPRs, 2 waves per SIMD), fewer below so a
// transform still spans at least one full wave.
#ifndef FDAS_FWD_E
#define FDAS_FWD_E 16
#endif
template <int L>
struct Geometry {
    static constexpr int E = L <= 256 ? 4 : (L <= 512 ? 8 : FDAS_FWD_E);
};
// Values per lane of the adjoint, which keeps five transform-sized arrays
// live (window, accumulator, work array, two bank rows): 8 from L = 512 on,
// 16 at L = 8192 so a workgroup stays at 512 lanes.  kMinWaves is the
// occupancy (waves per SIMD) the register allocation is held to, with both
// gradients; kMinWavesSpec with the spectrum gradient only.
#ifndef FDAS_BWD_WAVES
#define FDAS_BWD_WAVES 2
#endif
#ifndef FDAS_BWD_GROUP
#define FDAS_BWD_GROUP 3
#endif
#ifndef FDAS_BWD_E8192
#define FDAS_BWD_E8192 16
#endif
template <int L>
struct BwdGeometry {
    static constexpr int E = L <= 256 ? 4 : (L >= 8192 ? FDAS_BWD_E8192 : 8);
    static constexpr int kMinWaves = L >= 8192 ? 1 : FDAS_BWD_WAVES;
    // spectrum gradient only: no taps transform, fits 168 VGPRs up to L = 2048
    static constexpr int kMinWavesSpec = L >= 8192 ? 1 : (L >= 4096 ? FDAS_BWD_WAVES : 3);
    // windows per workgroup of the two-gradient adjoint (they share one taps
    // transform per template), for the edge-specialised kernel (M/2 = T)
    // where a workgroup is a single wave: measured at L = 512, M = 128 (2^20
    // bins, K = 85) 1 / 2 / 3 / 4 windows took 0.349 / 0.387 / 0.300 /
    // 0.669 ms (two waves per SIMD from two windows on, spills at four)
    static constexpr int kWinGroupEdge = L <= 512 ? FDAS_BWD_GROUP : 1;
};

}  // namespace fdas
