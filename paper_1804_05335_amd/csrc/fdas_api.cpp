// C-ABI entry points: argument validation, status codes, dispatch.
// Every call validates before launching anything; no exception crosses the
// ABI; nothing on the hot path allocates.
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdas.h"
#include "fdas_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

int ok()
{
    g_err[0] = '\0';
    return FDAS_OK;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(FDAS_HIP_ERROR, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

constexpr int kMaxK = 4096;
constexpr int64_t kMaxN = int64_t(1) << 32;

int check_grid(double zmax, double dz, int* K)
{
    if (!(std::isfinite(zmax) && std::isfinite(dz)) || zmax < 0.0 || dz <= 0.0)
        return fail(FDAS_INVALID_ARG, "zmax must be >= 0 and dz > 0 (got %g, %g)", zmax, dz);
    const double ratio = zmax / dz;
    const double r = std::nearbyint(ratio);
    if (std::fabs(ratio - r) > 1e-9 * std::fmax(1.0, ratio))
        return fail(FDAS_INVALID_ARG, "zmax (%g) is not a multiple of dz (%g)", zmax, dz);
    if (2.0 * r + 1.0 > kMaxK)
        return fail(FDAS_UNSUPPORTED, "K = %g templates exceeds %d", 2.0 * r + 1.0, kMaxK);
    *K = (int)(2.0 * r + 1.0);
    return FDAS_OK;
}

// Geometry shared by the forward calls.
int check_geometry(int K, int M, int L)
{
    if (K < 1 || K > kMaxK)
        return fail(FDAS_UNSUPPORTED, "K = %d outside [1, %d]", K, kMaxK);
    if (!is_pow2(L) || L < 256 || L > 8192)
        return fail(FDAS_UNSUPPORTED, "L = %d is not a power of two in [256, 8192]", L);
    if (M < 2 || (M & 1) || M > L / 2)
        return fail(FDAS_UNSUPPORTED, "M = %d must be even with 2 <= M <= L/2 = %d", M, L / 2);
    return FDAS_OK;
}

void fill_templates(double dz, int K, int M, fdas_cf32* out)
{
    for (int k = 0; k < K; ++k) {
        const double z = (double(k) - 0.5 * double(K - 1)) * dz;
        for (int j = 0; j < M; ++j) {
            const std::complex<double> r = fdas::response(double(j - M / 2), z);
            out[(size_t)k * M + j].re = (float)r.real();
            out[(size_t)k * M + j].im = (float)r.imag();
        }
    }
}

}  // namespace

extern "C" {

const char* fdas_version(void) { return "fdas-gfx950 0.1.0"; }

const char* fdas_status_string(int status)
{
    switch (status) {
    case FDAS_OK: return "ok";
    case FDAS_INVALID_ARG: return "invalid argument";
    case FDAS_UNSUPPORTED: return "unsupported geometry";
    case FDAS_WORKSPACE_TOO_SMALL: return "workspace too small";
    case FDAS_HIP_ERROR: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char* fdas_last_error(void) { return g_err; }

int fdas_num_templates(double zmax, double dz, int* K)
{
    if (!K)
        return fail(FDAS_INVALID_ARG, "K pointer is NULL");
    int k = 0;
    int st = check_grid(zmax, dz, &k);
    if (st)
        return st;
    *K = k;
    return ok();
}

int fdas_template_response(double q, double z, double* re, double* im)
{
    if (!re || !im)
        return fail(FDAS_INVALID_ARG, "output pointer is NULL");
    if (!std::isfinite(q) || !std::isfinite(z))
        return fail(FDAS_INVALID_ARG, "q and z must be finite");
    const std::complex<double> r = fdas::response(q, z);
    *re = r.real();
    *im = r.imag();
    return ok();
}

int fdas_make_templates_host(double zmax, double dz, int M, fdas_cf32* taps_host)
{
    int K = 0;
    int st = check_grid(zmax, dz, &K);
    if (st)
        return st;
    if (M < 2 || (M & 1) || M > 16384)
        return fail(FDAS_UNSUPPORTED, "M = %d must be even in [2, 16384]", M);
    if (!taps_host)
        return fail(FDAS_INVALID_ARG, "taps_host is NULL");
    fill_templates(dz, K, M, taps_host);
    return ok();
}

int64_t fdas_bank_elems(int K, int L)
{
    if (K < 1 || L < 1)
        return 0;
    return (int64_t)(K + 1) * (int64_t)L;
}

int fdas_prepare_bank(const fdas_cf32* taps_dev, int K, int M, int L, fdas_cf32* bank_dev,
                      hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (!taps_dev || !bank_dev)
        return fail(FDAS_INVALID_ARG, "taps_dev and bank_dev must not be NULL");
    if (!aligned(taps_dev, 8) || !aligned(bank_dev, 16))
        return fail(FDAS_INVALID_ARG, "taps_dev must be 8-byte and bank_dev 16-byte aligned");
    hipError_t e = fdas::launch_prepare_bank(reinterpret_cast<const float2*>(taps_dev), K, M, L,
                                             reinterpret_cast<float2*>(bank_dev), stream);
    if (e != hipSuccess)
        return hip_fail(e, "prepare_bank launch");
    return ok();
}

int fdas_make_templates(double zmax, double dz, int M, int L, fdas_cf32* taps_dev,
                        fdas_cf32* bank_dev, hipStream_t stream)
{
    int K = 0;
    int st = check_grid(zmax, dz, &K);
    if (st)
        return st;
    if (!taps_dev)
        return fail(FDAS_INVALID_ARG, "taps_dev is NULL");
    if (!aligned(taps_dev, 8))
        return fail(FDAS_INVALID_ARG, "taps_dev must be 8-byte aligned");
    if (bank_dev) {
        st = check_geometry(K, M, L);
        if (st)
            return st;
        if (!aligned(bank_dev, 16))
            return fail(FDAS_INVALID_ARG, "bank_dev must be 16-byte aligned");
    } else if (M < 2 || (M & 1) || M > 16384) {
        return fail(FDAS_UNSUPPORTED, "M = %d must be even in [2, 16384]", M);
    }
    std::vector<fdas_cf32> host;
    try {
        host.resize((size_t)K * M);
    } catch (const std::bad_alloc&) {
        return fail(FDAS_INVALID_ARG, "host allocation of %d x %d taps failed", K, M);
    }
    fill_templates(dz, K, M, host.data());
    hipError_t e = hipMemcpyAsync(taps_dev, host.data(), host.size() * sizeof(fdas_cf32),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess)
        return hip_fail(e, "copy of taps to the device");
    if (bank_dev) {
        e = fdas::launch_prepare_bank(reinterpret_cast<const float2*>(taps_dev), K, M, L,
                                      reinterpret_cast<float2*>(bank_dev), stream);
        if (e != hipSuccess)
            return hip_fail(e, "prepare_bank launch");
    }
    e = hipStreamSynchronize(stream);   // the host copy must outlive the transfer
    if (e != hipSuccess)
        return hip_fail(e, "stream synchronize");
    return ok();
}

int fdas_correlate_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K,
                      int M, int L, float* plane_dev, int zchunk, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (N < 0 || N > kMaxN)
        return fail(FDAS_INVALID_ARG, "N = %lld outside [0, 2^32]", (long long)N);
    if (zchunk < 0 || zchunk > K)
        return fail(FDAS_INVALID_ARG, "zchunk = %d outside [0, K = %d]", zchunk, K);
    if (N == 0)
        return ok();
    if (!spec_dev || !bank_dev || !plane_dev)
        return fail(FDAS_INVALID_ARG, "spec_dev, bank_dev and plane_dev must not be NULL");
    if (!aligned(spec_dev, 8) || !aligned(bank_dev, 16) || !aligned(plane_dev, 4))
        return fail(FDAS_INVALID_ARG, "misaligned pointer (spec 8 B, bank 16 B, plane 4 B)");
    const int64_t nseg = (N + (L - M) - 1) / (L - M);
    if (zchunk == 0)
        zchunk = fdas::default_zchunk(nseg, K);
    hipError_t e = fdas::launch_forward(reinterpret_cast<const float2*>(spec_dev), N,
                                        reinterpret_cast<const float2*>(bank_dev), K, M, L,
                                        plane_dev, zchunk, stream);
    if (e != hipSuccess)
        return hip_fail(e, "forward launch");
    return ok();
}

int fdas_correlate(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K, int M,
                   int L, float* plane_dev, hipStream_t stream)
{
    return fdas_correlate_ex(spec_dev, N, bank_dev, K, M, L, plane_dev, 0, stream);
}

}  // extern "C"
