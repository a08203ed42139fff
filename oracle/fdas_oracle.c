/*
 * Oracle: direct FP64 correlation and gradients in plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library; the GPU path never
 * does, and this file shares no code with it.
 *
 * Definition (Sec. 2, eq. 23, read with taps j in [0, M) at bin offsets
 * e_j = j - M/2 and the spectrum zero outside [0, N)):
 *     Y[z][r] = sum_j A[r + e_j] * conj(T[z][j]),  P[z][r] = |Y[z][r]|^2.
 * Gradients of Lw = sum w P (PyTorch complex convention), with
 * g[z][r] = 2 w[z][r] Y[z][r]:
 *     grad_A[k]    = sum_z sum_j T[z][j] g[z][k - e_j]
 *     grad_T[z][j] = sum_r conj(g[z][r]) A[r + e_j]
 *
 * Complex numbers are interleaved (re, im) doubles.  No FFT, no blocking:
 * each output is its defining sum, evaluated in FP64.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Y[z][r] for one (z, r): sum over taps with A = 0 outside [0, N). */
static void corr_point(const double *A, int64_t N, const double *Tz, int M,
                       int64_t r, double *yr, double *yi)
{
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < M; ++j) {
        int64_t k = r + (int64_t)j - (int64_t)(M / 2);
        if (k < 0 || k >= N)
            continue;
        double ar = A[2 * k], ai = A[2 * k + 1];
        double tr = Tz[2 * j], ti = Tz[2 * j + 1];
        /* A * conj(T) */
        sr += ar * tr + ai * ti;
        si += ai * tr - ar * ti;
    }
    *yr = sr;
    *yi = si;
}

/* Power plane rows z in [0, K), columns r in [r_lo, r_hi):
 * P[z * (r_hi - r_lo) + (r - r_lo)]. */
void oracle_power(const double *A, int64_t N, const double *T, int K, int M,
                  int64_t r_lo, int64_t r_hi, double *P)
{
    int64_t W = r_hi - r_lo;
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < K; ++z)
        for (int64_t c = 0; c < W; ++c) {
            double yr, yi;
            corr_point(A, N, T + 2 * (int64_t)z * M, M, r_lo + c, &yr, &yi);
            P[(int64_t)z * W + c] = yr * yr + yi * yi;
        }
}

/* Power at npts sampled (z, r) points. */
void oracle_power_points(const double *A, int64_t N, const double *T, int K,
                         int M, const int32_t *zi, const int64_t *ri,
                         int64_t npts, double *out)
{
    (void)K;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double yr, yi;
        corr_point(A, N, T + 2 * (int64_t)zi[p] * M, M, ri[p], &yr, &yi);
        out[p] = yr * yr + yi * yi;
    }
}

/* Interbinned plane (Sec. 3, eq. f-interp) at sampled (z, column) points of
 * the [K][2N] layout: column 2r is |Y[z][r]|^2, column 2r+1 is
 * |(pi/4)(Y[z][r] - Y[z][r+1])|^2 with Y[z][N] from the same sum. */
void oracle_interbin_points(const double *A, int64_t N, const double *T, int K, int M,
                            const int32_t *zi, const int64_t *ci, int64_t npts, double *out)
{
    (void)K;
    const double q = 0.78539816339744830962; /* pi/4 */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        const double *Tz = T + 2 * (int64_t)zi[p] * M;
        const int64_t r = ci[p] / 2;
        double yr, yi;
        corr_point(A, N, Tz, M, r, &yr, &yi);
        if ((ci[p] & 1) == 0) {
            out[p] = yr * yr + yi * yi;
        } else {
            double nr, ni;
            corr_point(A, N, Tz, M, r + 1, &nr, &ni);
            const double dr = q * (yr - nr), di = q * (yi - ni);
            out[p] = dr * dr + di * di;
        }
    }
}

/* Complex correlation Y (interleaved) for all z, r. */
void oracle_correlate(const double *A, int64_t N, const double *T, int K,
                      int M, double *Y)
{
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < K; ++z)
        for (int64_t r = 0; r < N; ++r)
            corr_point(A, N, T + 2 * (int64_t)z * M, M, r,
                       &Y[2 * ((int64_t)z * N + r)],
                       &Y[2 * ((int64_t)z * N + r) + 1]);
}

/* grad_A at npts sampled bins k, each from its defining sum:
 * grad_A[k] = sum_z sum_j T[z][j] g[z][k - e_j], g[z][r] = 2 w[z][r] Y[z][r],
 * with Y evaluated directly where needed (r in [0, N)).  w is float32 [K][N]. */
void oracle_grad_spec_points(const double *A, int64_t N, const double *T, int K, int M,
                             const float *w, const int64_t *ks, int64_t npts, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npts; ++p) {
        const int64_t k = ks[p];
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < K; ++z) {
            const double *Tz = T + 2 * (int64_t)z * M;
            for (int j = 0; j < M; ++j) {
                int64_t r = k - ((int64_t)j - (int64_t)(M / 2));
                if (r < 0 || r >= N)
                    continue;
                double yr, yi;
                corr_point(A, N, Tz, M, r, &yr, &yi);
                const double s = 2.0 * (double)w[(int64_t)z * N + r];
                const double gr = s * yr, gi = s * yi;
                const double tr = Tz[2 * j], ti = Tz[2 * j + 1];
                sr += tr * gr - ti * gi;
                si += tr * gi + ti * gr;
            }
        }
        out[2 * p] = sr;
        out[2 * p + 1] = si;
    }
}

/* Gradients of Lw = sum w P.  w is float32 [K][N]; gA is [N], gT is [K][M]
 * (interleaved complex).  Uses a scratch copy of g = 2 w Y. */
int oracle_grads(const double *A, int64_t N, const double *T, int K, int M,
                 const float *w, double *gA, double *gT)
{
    double *g = (double *)malloc(sizeof(double) * 2 * (size_t)K * (size_t)N);
    if (!g)
        return 1;
    oracle_correlate(A, N, T, K, M, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)K * N; ++i) {
        double s = 2.0 * (double)w[i];
        g[2 * i] *= s;
        g[2 * i + 1] *= s;
    }
    /* grad_A[k] = sum_z sum_j T[z][j] g[z][k - e_j] */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < K; ++z) {
            const double *Tz = T + 2 * (int64_t)z * M;
            const double *gz = g + 2 * (int64_t)z * N;
            for (int j = 0; j < M; ++j) {
                int64_t r = k - ((int64_t)j - (int64_t)(M / 2));
                if (r < 0 || r >= N)
                    continue;
                double tr = Tz[2 * j], ti = Tz[2 * j + 1];
                double gr = gz[2 * r], gi = gz[2 * r + 1];
                sr += tr * gr - ti * gi;
                si += tr * gi + ti * gr;
            }
        }
        gA[2 * k] = sr;
        gA[2 * k + 1] = si;
    }
    /* grad_T[z][j] = sum_r conj(g[z][r]) A[r + e_j] */
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < K; ++z)
        for (int j = 0; j < M; ++j) {
            const double *gz = g + 2 * (int64_t)z * N;
            double sr = 0.0, si = 0.0;
            for (int64_t r = 0; r < N; ++r) {
                int64_t k = r + (int64_t)j - (int64_t)(M / 2);
                if (k < 0 || k >= N)
                    continue;
                double gr = gz[2 * r], gi = gz[2 * r + 1];
                double ar = A[2 * k], ai = A[2 * k + 1];
                sr += gr * ar + gi * ai;
                si += gr * ai - gi * ar;
            }
            gT[2 * ((int64_t)z * M + j)] = sr;
            gT[2 * ((int64_t)z * M + j) + 1] = si;
        }
    free(g);
    return 0;
}
