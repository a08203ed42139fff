// Host FP64 template math: the predicted normalised Fourier response of a
// constant-fdot signal (Sec. 2, text before eq. 23; eq. 22 defines z as the
// number of bins drifted over the observation).
//
//   R(q, z) = int_0^1 exp(i 2 pi [q u + z (u^2 - u)/2]) du,  q = r - k.
//
// Evaluated through the Fresnel auxiliary function G(x) = g(x) + i f(x),
// defined by  C(x) + i S(x) = (1+i)/2 - G(x) exp(i pi x^2 / 2)  for x >= 0,
// which makes the closed form free of large phases and of the cancellation
// of the Fresnel integrals' 1/2 limits.  With q' = q - z/2, s = sqrt(2/z),
// x1 = s q', x2 = s (q' + z) and  exp(i pi (x2^2 - x1^2)/2) = exp(i 2 pi q):
//   x1 >= 0      : R = (G(x1) - e^{i2 pi q} G(x2)) / sqrt(2z)
//   x2 <= 0      : R = (e^{i2 pi q} G(-x2) - G(-x1)) / sqrt(2z)
//   x1 < 0 < x2  : R = ((1+i) e^{-i pi q'^2/z} - e^{i2 pi q} G(x2) - G(-x1)) / sqrt(2z)
// and R(q, z) = conj R(-q, -z) for z < 0,  R(q, 0) = (e^{i2 pi q} - 1)/(i 2 pi q).
//
// G itself: for x <= 2 from the power series
//   C(x) + i S(x) = sum_k (i pi/2)^k x^{2k+1} / (k! (2k+1)),
// and for x > 2 from G(x) = (1+i)/2 * erfcx(w), w = (sqrt(pi)/2)(1-i) x,
// with erfcx evaluated by the Laplace continued fraction (DLMF 7.9.3)
//   sqrt(pi) erfcx(w) = 2w / (2w^2+1 - 1*2/(2w^2+5 - 3*4/(2w^2+9 - ...)))
// summed by the modified Lentz method.
#include <cmath>
#include <complex>
#include <cstdint>

namespace fdas {

using cd = std::complex<double>;

static const double kPi = 3.14159265358979323846264338327950288;

// exp(i 2 pi q) with the integer part of q removed exactly first.
static cd cis_2pi(double q)
{
    double f = q - std::nearbyint(q);
    if (f == 0.0)
        return cd(1.0, 0.0);
    return cd(std::cos(2.0 * kPi * f), std::sin(2.0 * kPi * f));
}

// exp(-i pi t) with t reduced modulo 2 first.
static cd cis_minus_pi(double t)
{
    double r = std::fmod(t, 2.0);
    return cd(std::cos(kPi * r), -std::sin(kPi * r));
}

static cd fresnel_series(double x)
{
    const double t = 0.5 * kPi * x * x;
    cd term(x, 0.0);
    cd sum(0.0, 0.0);
    for (int k = 0; k < 200; ++k) {
        sum += term / double(2 * k + 1);
        term *= cd(0.0, t / double(k + 1));
        if (std::abs(term) <= 1e-18 * std::abs(sum))
            break;
    }
    return sum;
}

static cd erfcx_lentz(cd w)
{
    const double tiny = 1e-300;
    const cd w2 = 2.0 * w * w;
    cd f = w2 + 1.0;
    cd C = f, D = 0.0;
    for (int n = 1; n < 10000; ++n) {
        const double a = -double(2 * n - 1) * double(2 * n);
        const cd b = w2 + double(1 + 4 * n);
        D = b + a * D;
        if (std::abs(D) == 0.0)
            D = tiny;
        D = 1.0 / D;
        C = b + a / C;
        if (std::abs(C) == 0.0)
            C = tiny;
        const cd d = C * D;
        f *= d;
        if (std::abs(d - 1.0) < 1e-16)
            break;
    }
    return 2.0 * w / f / std::sqrt(kPi);
}

// G(x) = g(x) + i f(x), x >= 0.
static cd fresnel_aux(double x)
{
    if (x <= 2.0) {
        const cd cs = fresnel_series(x);
        const double ph = 0.5 * kPi * x * x;
        return (cd(0.5, 0.5) - cs) * cd(std::cos(ph), -std::sin(ph));
    }
    const cd w = (0.5 * std::sqrt(kPi)) * cd(1.0, -1.0) * x;
    return cd(0.5, 0.5) * erfcx_lentz(w);
}

cd response(double q, double z)
{
    if (z < 0.0)
        return std::conj(response(-q, -z));
    if (z == 0.0) {
        if (q == 0.0)
            return cd(1.0, 0.0);
        return (cis_2pi(q) - 1.0) / cd(0.0, 2.0 * kPi * q);
    }
    const double qp = q - 0.5 * z;
    const double s = std::sqrt(2.0 / z);
    const double x1 = s * qp, x2 = s * (qp + z);
    const double norm = 1.0 / std::sqrt(2.0 * z);
    const cd e2q = cis_2pi(q);
    if (x1 >= 0.0)
        return (fresnel_aux(x1) - e2q * fresnel_aux(x2)) * norm;
    if (x2 <= 0.0)
        return (e2q * fresnel_aux(-x2) - fresnel_aux(-x1)) * norm;
    const cd lead = cd(1.0, 1.0) * cis_minus_pi(qp * qp / z);
    return (lead - e2q * fresnel_aux(x2) - fresnel_aux(-x1)) * norm;
}

}  // namespace fdas
