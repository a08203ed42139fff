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

// [a, a + na) and [b, b + nb) share a byte (NULL pointers never overlap)
bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return a && b && pa < pb + nb && pb < pa + na;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

constexpr int kMaxK = 4096;
constexpr int64_t kMaxN = int64_t(1) << 32;
constexpr int kMaxSpectra = 1 << 24;
constexpr int kMaxGrid = 1 << 20;
constexpr int64_t kMaxCapacity = int64_t(1) << 40;

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

// Half-bin taps of the two-bin Fourier interpolation, K x (M + 2): tap j of
// template z sits at bin offset j - (M+2)/2 and holds R(1/2 - offset, z) for
// the M offsets -M/2+1 .. M/2 (the bins centred on the half bin); taps 0 and
// 1 are zero.
void fill_templates_half(double dz, int K, int M, fdas_cf32* out)
{
    const int Mh = M + 2;
    for (int k = 0; k < K; ++k) {
        const double z = (double(k) - 0.5 * double(K - 1)) * dz;
        for (int j = 0; j < Mh; ++j) {
            std::complex<double> r(0.0, 0.0);
            if (j >= 2)
                r = fdas::response(0.5 - double(j - Mh / 2), z);
            out[(size_t)k * Mh + j].re = (float)r.real();
            out[(size_t)k * Mh + j].im = (float)r.imag();
        }
    }
}

}  // namespace

int fdas::fail_status(int status, const char* msg)
{
    return status == FDAS_OK ? ok() : fail(status, "%s", msg);
}

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

}  // extern "C"

namespace {

int correlate_impl(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K, int M,
                   int L, float* plane_dev, int grid, bool interbin, bool sym, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (sym && !(K & 1))
        return fail(FDAS_INVALID_ARG, "a symmetric bank needs an odd K (got %d)", K);
    if (N < 0 || N > kMaxN)
        return fail(FDAS_INVALID_ARG, "N = %lld outside [0, 2^32]", (long long)N);
    if (grid < 0 || grid > kMaxGrid)
        return fail(FDAS_INVALID_ARG, "grid = %d outside [0, %d]", grid, kMaxGrid);
    if (N == 0)
        return ok();
    if (!spec_dev || !bank_dev || !plane_dev)
        return fail(FDAS_INVALID_ARG, "spec_dev, bank_dev and plane_dev must not be NULL");
    if (!aligned(spec_dev, 8) || !aligned(bank_dev, 16) || !aligned(plane_dev, interbin ? 8 : 4))
        return fail(FDAS_INVALID_ARG,
                    "misaligned pointer (spec 8 B, bank 16 B, plane 4 B, interbinned plane 8 B)");
    hipError_t e = fdas::launch_forward(reinterpret_cast<const float2*>(spec_dev), N,
                                        reinterpret_cast<const float2*>(bank_dev), K, M, L,
                                        plane_dev, grid, interbin, sym, stream);
    if (e != hipSuccess)
        return hip_fail(e, "forward launch");
    return ok();
}

}  // namespace

extern "C" {

int fdas_correlate_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K,
                      int M, int L, float* plane_dev, int grid, hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_dev, K, M, L, plane_dev, grid, false, false, stream);
}

int fdas_correlate(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K, int M,
                   int L, float* plane_dev, hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_dev, K, M, L, plane_dev, 0, false, false, stream);
}

int fdas_correlate_interbin_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev,
                               int K, int M, int L, float* plane2_dev, int grid,
                               hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_dev, K, M, L, plane2_dev, grid, true, false, stream);
}

int fdas_correlate_interbin(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev,
                            int K, int M, int L, float* plane2_dev, hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_dev, K, M, L, plane2_dev, 0, true, false, stream);
}

int64_t fdas_bank_sym_elems(int K, int L)
{
    if (K < 1 || !(K & 1) || L < 1)
        return 0;
    return (int64_t)((K + 1) / 2 + 1) * (int64_t)L;
}

int fdas_prepare_bank_sym(const fdas_cf32* taps_dev, int K, int M, int L, fdas_cf32* bank_dev,
                          hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (!(K & 1))
        return fail(FDAS_INVALID_ARG, "a symmetric bank needs an odd K (got %d)", K);
    if (!taps_dev || !bank_dev)
        return fail(FDAS_INVALID_ARG, "taps_dev and bank_dev must not be NULL");
    if (!aligned(taps_dev, 8) || !aligned(bank_dev, 16))
        return fail(FDAS_INVALID_ARG, "taps_dev must be 8-byte and bank_dev 16-byte aligned");
    // rows z >= 0 are templates (K-1)/2 .. K-1
    const int c = (K - 1) / 2;
    hipError_t e = fdas::launch_prepare_bank(
        reinterpret_cast<const float2*>(taps_dev) + (size_t)c * M, K - c, M, L,
        reinterpret_cast<float2*>(bank_dev), stream);
    if (e != hipSuccess)
        return hip_fail(e, "prepare_bank launch");
    return ok();
}

int fdas_correlate_sym_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_sym_dev,
                          int K, int M, int L, float* plane_dev, int grid, hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_sym_dev, K, M, L, plane_dev, grid, false, true,
                          stream);
}

int fdas_correlate_sym(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_sym_dev, int K,
                       int M, int L, float* plane_dev, hipStream_t stream)
{
    return correlate_impl(spec_dev, N, bank_sym_dev, K, M, L, plane_dev, 0, false, true, stream);
}

int fdas_make_templates_half(double zmax, double dz, int M, int L, fdas_cf32* taps_half_dev,
                             fdas_cf32* bank_half_dev, hipStream_t stream)
{
    int K = 0;
    int st = check_grid(zmax, dz, &K);
    if (st)
        return st;
    st = check_geometry(K, M + 2, L);
    if (st)
        return st;
    if (M < 2 || (M & 1))
        return fail(FDAS_UNSUPPORTED, "M = %d must be even and >= 2", M);
    if (!taps_half_dev)
        return fail(FDAS_INVALID_ARG, "taps_half_dev is NULL");
    if (!aligned(taps_half_dev, 8) || (bank_half_dev && !aligned(bank_half_dev, 16)))
        return fail(FDAS_INVALID_ARG, "taps_half_dev must be 8-byte and bank_half_dev 16-byte aligned");
    std::vector<fdas_cf32> host;
    try {
        host.resize((size_t)K * (M + 2));
    } catch (const std::bad_alloc&) {
        return fail(FDAS_INVALID_ARG, "host allocation of %d x %d taps failed", K, M + 2);
    }
    fill_templates_half(dz, K, M, host.data());
    hipError_t e = hipMemcpyAsync(taps_half_dev, host.data(), host.size() * sizeof(fdas_cf32),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess)
        return hip_fail(e, "copy of half-bin taps to the device");
    if (bank_half_dev) {
        e = fdas::launch_prepare_bank(reinterpret_cast<const float2*>(taps_half_dev), K, M + 2, L,
                                      reinterpret_cast<float2*>(bank_half_dev), stream);
        if (e != hipSuccess)
            return hip_fail(e, "prepare_bank launch");
    }
    e = hipStreamSynchronize(stream);   // the host copy must outlive the transfer
    if (e != hipSuccess)
        return hip_fail(e, "stream synchronize");
    return ok();
}

int fdas_correlate_fourier2_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev,
                               const fdas_cf32* bank_half_dev, int K, int M, int L,
                               float* plane2_dev, int grid, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    st = check_geometry(K, M + 2, L);
    if (st)
        return st;
    if (N < 0 || N > kMaxN)
        return fail(FDAS_INVALID_ARG, "N = %lld outside [0, 2^32]", (long long)N);
    if (grid < 0 || grid > kMaxGrid)
        return fail(FDAS_INVALID_ARG, "grid = %d outside [0, %d]", grid, kMaxGrid);
    if (N == 0)
        return ok();
    if (!spec_dev || !bank_dev || !bank_half_dev || !plane2_dev)
        return fail(FDAS_INVALID_ARG, "spec, bank, bank_half and plane2 must not be NULL");
    if (!aligned(spec_dev, 8) || !aligned(bank_dev, 16) || !aligned(bank_half_dev, 16) ||
        !aligned(plane2_dev, 8))
        return fail(FDAS_INVALID_ARG, "misaligned pointer (spec 8 B, banks 16 B, plane2 8 B)");
    // the M-tap bank places its taps exactly where the same taps zero-padded
    // to M + 2 would go, so both banks run on the (M + 2)-tap geometry
    hipError_t e = fdas::launch_forward_dual(
        reinterpret_cast<const float2*>(spec_dev), N, reinterpret_cast<const float2*>(bank_dev),
        reinterpret_cast<const float2*>(bank_half_dev), K, M + 2, L, plane2_dev, grid, stream);
    if (e != hipSuccess)
        return hip_fail(e, "forward launch");
    return ok();
}

int fdas_correlate_fourier2(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev,
                            const fdas_cf32* bank_half_dev, int K, int M, int L, float* plane2_dev,
                            hipStream_t stream)
{
    return fdas_correlate_fourier2_ex(spec_dev, N, bank_dev, bank_half_dev, K, M, L, plane2_dev, 0,
                                      stream);
}

size_t fdas_batched_workspace_bytes(int nspec)
{
    if (nspec < 0)
        return 0;
    const size_t b = sizeof(int64_t) * ((size_t)nspec + 1);
    return (b + 255) & ~(size_t)255;
}

int fdas_correlate_batched_ex(const fdas_cf32* specs_dev, const int64_t* offsets_dev, int nspec,
                              int64_t capacity, const fdas_cf32* bank_dev, int K, int M, int L,
                              float* planes_dev, int E, int grid, void* ws_dev, size_t ws_bytes,
                              hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (nspec < 0 || nspec > kMaxSpectra)
        return fail(FDAS_INVALID_ARG, "nspec = %d outside [0, %d]", nspec, kMaxSpectra);
    if (capacity < 0 || capacity > kMaxCapacity)
        return fail(FDAS_INVALID_ARG, "capacity = %lld outside [0, 2^40]", (long long)capacity);
    if (grid < 0 || grid > kMaxGrid)
        return fail(FDAS_INVALID_ARG, "grid = %d outside [0, %d]", grid, kMaxGrid);
    if (!fdas::batched_values_per_lane_ok(L, E))
        return fail(FDAS_UNSUPPORTED, "E = %d values per lane is not supported at L = %d", E, L);
    if (nspec == 0)
        return ok();
    if (!specs_dev || !offsets_dev || !bank_dev || !planes_dev || !ws_dev)
        return fail(FDAS_INVALID_ARG, "specs, offsets, bank, planes and ws must not be NULL");
    if (!aligned(specs_dev, 8) || !aligned(offsets_dev, 8) || !aligned(bank_dev, 16) ||
        !aligned(planes_dev, 4) || !aligned(ws_dev, 8))
        return fail(FDAS_INVALID_ARG,
                    "misaligned pointer (specs 8 B, offsets 8 B, bank 16 B, planes 4 B, ws 8 B)");
    if (ws_bytes < fdas_batched_workspace_bytes(nspec))
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    fdas_batched_workspace_bytes(nspec));
    hipError_t e = fdas::launch_batched(reinterpret_cast<const float2*>(specs_dev), offsets_dev,
                                        nspec, capacity, reinterpret_cast<const float2*>(bank_dev),
                                        K, M, L, E, planes_dev, static_cast<int64_t*>(ws_dev), grid,
                                        stream);
    if (e != hipSuccess)
        return hip_fail(e, "batched launch");
    return ok();
}

int fdas_correlate_batched(const fdas_cf32* specs_dev, const int64_t* offsets_dev, int nspec,
                           int64_t capacity, const fdas_cf32* bank_dev, int K, int M, int L,
                           float* planes_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream)
{
    return fdas_correlate_batched_ex(specs_dev, offsets_dev, nspec, capacity, bank_dev, K, M, L,
                                     planes_dev, 0, 0, ws_dev, ws_bytes, stream);
}

int fdas_correlate_batched_noalloc(const fdas_cf32* specs_dev, const int64_t* offsets_dev,
                                   int nspec, int64_t capacity, const fdas_cf32* bank_dev, int K,
                                   int M, int L, float* planes_dev, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (nspec < 0 || nspec > FDAS_NOALLOC_MAX_SPECTRA)
        return fail(FDAS_INVALID_ARG,
                    "nspec = %d outside [0, %d], the allocation-free call's fixed maximum "
                    "(use fdas_correlate_batched with a workspace for more)",
                    nspec, FDAS_NOALLOC_MAX_SPECTRA);
    if (capacity < 0 || capacity > kMaxCapacity)
        return fail(FDAS_INVALID_ARG, "capacity = %lld outside [0, 2^40]", (long long)capacity);
    if (nspec == 0)
        return ok();
    if (!specs_dev || !offsets_dev || !bank_dev || !planes_dev)
        return fail(FDAS_INVALID_ARG, "specs, offsets, bank and planes must not be NULL");
    if (!aligned(specs_dev, 8) || !aligned(offsets_dev, 8) || !aligned(bank_dev, 16) ||
        !aligned(planes_dev, 4))
        return fail(FDAS_INVALID_ARG,
                    "misaligned pointer (specs 8 B, offsets 8 B, bank 16 B, planes 4 B)");
    int64_t* segpre = nullptr;
    hipError_t e = fdas::noalloc_segpre(&segpre);
    if (e != hipSuccess)
        return hip_fail(e, "allocation-free batched call: device scratch lookup");
    e = fdas::launch_batched(reinterpret_cast<const float2*>(specs_dev), offsets_dev, nspec,
                             capacity, reinterpret_cast<const float2*>(bank_dev), K, M, L, 0,
                             planes_dev, segpre, 0, stream);
    if (e != hipSuccess)
        return hip_fail(e, "allocation-free batched launch");
    return ok();
}

namespace {

int backward_zchunk(int64_t nwin, int K, int zchunk)
{
    if (zchunk > 0)
        return zchunk;
    // ~4096 workgroups, about 8 rounds of the ~512 resident on 256 CUs, so the
    // last round's tail stays small; each chunk adds one partial gradient
    // window and one recomputed forward FFT per window
    int64_t chunks = (4096 + (nwin > 0 ? nwin : 1) - 1) / (nwin > 0 ? nwin : 1);
    if (chunks < 1) chunks = 1;
    if (chunks > K) chunks = K;
    return (int)((K + chunks - 1) / chunks);
}

// Window chunks of the taps-gradient reduction: enough (64 x 16)-lane blocks
// to fill the device (~2048 over the K M / 64 column groups), each chunk at
// least 64 windows long.
int backward_tsplit(int64_t nwin, int K, int M)
{
    const int64_t groups = ((int64_t)K * M + 63) / 64;
    int64_t split = (2048 + groups - 1) / groups;
    const int64_t most = nwin / 64;
    if (split > most) split = most;
    if (split < 1) split = 1;
    return (int)split;
}

// Workspace: partA [nzc][nwin][L] complex, partT [nwin][K][M] complex, tpart
// [tsplit][K][M] FP64 complex, each 256-byte aligned.
void backward_layout(int64_t N, int K, int M, int L, int zchunk, size_t* offT, size_t* offP,
                     size_t* total)
{
    const int64_t nwin = (N + (L - M) - 1) / (L - M);
    const int zc = backward_zchunk(nwin, K, zchunk);
    const int64_t nzc = (K + zc - 1) / zc;
    const size_t a = (size_t)nzc * (size_t)nwin * (size_t)L * sizeof(fdas_cf32);
    const size_t t = (size_t)nwin * (size_t)K * (size_t)M * sizeof(fdas_cf32);
    const size_t p = (size_t)backward_tsplit(nwin, K, M) * (size_t)K * (size_t)M * 2 * sizeof(double);
    *offT = (a + 255) & ~(size_t)255;
    *offP = ((*offT + t) + 255) & ~(size_t)255;
    *total = ((*offP + p) + 255) & ~(size_t)255;
}

}  // namespace

size_t fdas_backward_workspace_bytes(int64_t N, int K, int M, int L, int zchunk)
{
    if (N < 0 || N > kMaxN || check_geometry(K, M, L) != FDAS_OK || zchunk < 0 || zchunk > K)
        return 0;
    size_t offT = 0, offP = 0, total = 0;
    backward_layout(N, K, M, L, zchunk, &offT, &offP, &total);
    return total < 256 ? 256 : total;
}

int fdas_correlate_backward_ex(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev,
                               int K, int M, int L, const float* dLdP_dev,
                               fdas_cf32* grad_spec_dev, fdas_cf32* grad_taps_dev, int zchunk,
                               void* ws_dev, size_t ws_bytes, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (N < 0 || N > kMaxN)
        return fail(FDAS_INVALID_ARG, "N = %lld outside [0, 2^32]", (long long)N);
    if (zchunk < 0 || zchunk > K)
        return fail(FDAS_INVALID_ARG, "zchunk = %d outside [0, K = %d]", zchunk, K);
    if (!grad_spec_dev && !grad_taps_dev)
        return ok();
    if (!bank_dev || !ws_dev || (N > 0 && (!spec_dev || !dLdP_dev)))
        return fail(FDAS_INVALID_ARG, "spec, bank, dLdP and ws must not be NULL");
    if ((spec_dev && !aligned(spec_dev, 8)) || !aligned(bank_dev, 16) ||
        (dLdP_dev && !aligned(dLdP_dev, 4)) || (grad_spec_dev && !aligned(grad_spec_dev, 8)) ||
        (grad_taps_dev && !aligned(grad_taps_dev, 8)) || !aligned(ws_dev, 256))
        return fail(FDAS_INVALID_ARG,
                    "misaligned pointer (spec/grads 8 B, bank 16 B, dLdP 4 B, ws 256 B)");
    const size_t need = fdas_backward_workspace_bytes(N, K, M, L, zchunk);
    if (ws_bytes < need)
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    need);
    const int64_t nwin = (N + (L - M) - 1) / (L - M);
    const int zc = backward_zchunk(nwin, K, zchunk);
    size_t offT = 0, offP = 0, total = 0;
    backward_layout(N, K, M, L, zchunk, &offT, &offP, &total);
    auto* base = static_cast<unsigned char*>(ws_dev);
    hipError_t e = fdas::launch_backward(
        reinterpret_cast<const float2*>(spec_dev), N, reinterpret_cast<const float2*>(bank_dev),
        K, M, L, dLdP_dev, reinterpret_cast<float2*>(grad_spec_dev),
        reinterpret_cast<float2*>(grad_taps_dev), zc, reinterpret_cast<float2*>(base),
        reinterpret_cast<float2*>(base + offT), backward_tsplit(nwin, K, M),
        reinterpret_cast<double2*>(base + offP), stream);
    if (e != hipSuccess)
        return hip_fail(e, "backward launch");
    return ok();
}

int fdas_correlate_backward(const fdas_cf32* spec_dev, int64_t N, const fdas_cf32* bank_dev, int K,
                            int M, int L, const float* dLdP_dev, fdas_cf32* grad_spec_dev,
                            fdas_cf32* grad_taps_dev, void* ws_dev, size_t ws_bytes,
                            hipStream_t stream)
{
    return fdas_correlate_backward_ex(spec_dev, N, bank_dev, K, M, L, dLdP_dev, grad_spec_dev,
                                      grad_taps_dev, 0, ws_dev, ws_bytes, stream);
}

namespace {

// Upper bound on the windows of a batch whose spectra lie in [0, capacity):
// sum_b ceil(N_b / B) <= capacity / B + nspec.
int64_t batched_max_windows(int64_t capacity, int nspec, int B)
{
    return capacity / B + nspec;
}

// Batched adjoint workspace: winpre [nspec + 1] int64, then (if wanted)
// partA [nzc][maxwin][L] complex, partT [maxwin][K][M] complex and tpart
// [tsplit][K][M] FP64 complex, each 256-byte aligned.
void backward_batched_layout(int64_t capacity, int nspec, int K, int M, int L, int zchunk,
                             int want, size_t* offA, size_t* offT, size_t* offP, size_t* total)
{
    const int64_t maxwin = batched_max_windows(capacity, nspec, L - M);
    const int zc = backward_zchunk(maxwin, K, zchunk);
    const int64_t nzc = (K + zc - 1) / zc;
    const size_t w = sizeof(int64_t) * ((size_t)nspec + 1);
    const size_t a = (want & FDAS_WANT_SPECTRA)
                         ? (size_t)nzc * (size_t)maxwin * (size_t)L * sizeof(fdas_cf32) : 0;
    const size_t t = (want & FDAS_WANT_TAPS)
                         ? (size_t)maxwin * (size_t)K * (size_t)M * sizeof(fdas_cf32) : 0;
    const size_t p = (want & FDAS_WANT_TAPS) ? (size_t)backward_tsplit(maxwin, K, M) * (size_t)K *
                                                   (size_t)M * 2 * sizeof(double)
                                             : 0;
    *offA = (w + 255) & ~(size_t)255;
    *offT = ((*offA + a) + 255) & ~(size_t)255;
    *offP = ((*offT + t) + 255) & ~(size_t)255;
    *total = ((*offP + p) + 255) & ~(size_t)255;
}

}  // namespace

size_t fdas_backward_batched_workspace_bytes(int64_t capacity, int nspec, int K, int M, int L,
                                             int zchunk, int want)
{
    if (capacity < 0 || capacity > kMaxCapacity || nspec < 0 || nspec > kMaxSpectra ||
        check_geometry(K, M, L) != FDAS_OK || zchunk < 0 || zchunk > K ||
        (want & ~(FDAS_WANT_SPECTRA | FDAS_WANT_TAPS)))
        return 0;
    size_t offA = 0, offT = 0, offP = 0, total = 0;
    backward_batched_layout(capacity, nspec, K, M, L, zchunk, want, &offA, &offT, &offP, &total);
    return total < 256 ? 256 : total;
}

int fdas_correlate_backward_batched(const fdas_cf32* specs_dev, const int64_t* offsets_dev,
                                    int nspec, int64_t capacity, const fdas_cf32* bank_dev, int K,
                                    int M, int L, const float* dLdP_dev,
                                    fdas_cf32* grad_specs_dev, fdas_cf32* grad_taps_dev,
                                    int zchunk, void* ws_dev, size_t ws_bytes, hipStream_t stream)
{
    int st = check_geometry(K, M, L);
    if (st)
        return st;
    if (nspec < 0 || nspec > kMaxSpectra)
        return fail(FDAS_INVALID_ARG, "nspec = %d outside [0, %d]", nspec, kMaxSpectra);
    if (capacity < 0 || capacity > kMaxCapacity)
        return fail(FDAS_INVALID_ARG, "capacity = %lld outside [0, 2^40]", (long long)capacity);
    if (zchunk < 0 || zchunk > K)
        return fail(FDAS_INVALID_ARG, "zchunk = %d outside [0, K = %d]", zchunk, K);
    if (!grad_specs_dev && !grad_taps_dev)
        return ok();
    if (!bank_dev || !ws_dev || !offsets_dev || (capacity > 0 && (!specs_dev || !dLdP_dev)))
        return fail(FDAS_INVALID_ARG, "specs, offsets, bank, dLdP and ws must not be NULL");
    if ((specs_dev && !aligned(specs_dev, 8)) || !aligned(offsets_dev, 8) ||
        !aligned(bank_dev, 16) || (dLdP_dev && !aligned(dLdP_dev, 4)) ||
        (grad_specs_dev && !aligned(grad_specs_dev, 8)) ||
        (grad_taps_dev && !aligned(grad_taps_dev, 8)) || !aligned(ws_dev, 256))
        return fail(FDAS_INVALID_ARG,
                    "misaligned pointer (specs/offsets/grads 8 B, bank 16 B, dLdP 4 B, ws 256 B)");
    const int want = (grad_specs_dev ? FDAS_WANT_SPECTRA : 0) | (grad_taps_dev ? FDAS_WANT_TAPS : 0);
    const size_t need = fdas_backward_batched_workspace_bytes(capacity, nspec, K, M, L, zchunk, want);
    if (ws_bytes < need)
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    need);
    const int64_t maxwin = batched_max_windows(capacity, nspec, L - M);
    const int zc = backward_zchunk(maxwin, K, zchunk);
    size_t offA = 0, offT = 0, offP = 0, total = 0;
    backward_batched_layout(capacity, nspec, K, M, L, zchunk, want, &offA, &offT, &offP, &total);
    auto* base = static_cast<unsigned char*>(ws_dev);
    hipError_t e = fdas::launch_backward_batched(
        reinterpret_cast<const float2*>(specs_dev), offsets_dev, nspec, capacity,
        reinterpret_cast<const float2*>(bank_dev), K, M, L, dLdP_dev,
        reinterpret_cast<float2*>(grad_specs_dev), reinterpret_cast<float2*>(grad_taps_dev), zc,
        maxwin, reinterpret_cast<int64_t*>(base), reinterpret_cast<float2*>(base + offA),
        reinterpret_cast<float2*>(base + offT), backward_tsplit(maxwin, K, M),
        reinterpret_cast<double2*>(base + offP), stream);
    if (e != hipSuccess)
        return hip_fail(e, "batched backward launch");
    return ok();
}

}  // extern "C"

// ---- real-to-complex front end ----------------------------------------------

namespace {

// log2(n) for a supported time-series length, else -1.
int r2c_log2n(int64_t n)
{
    if (n < ((int64_t)1 << 13) || n > ((int64_t)1 << 27) || (n & (n - 1)) != 0)
        return -1;
    int l = 0;
    while (((int64_t)1 << l) < n)
        ++l;
    int bits[4];
    return fdas::r2c_plan(l - 1, bits) > 0 ? l : -1;
}

}  // namespace

extern "C" {

size_t fdas_r2c_workspace_bytes(int64_t n)
{
    const int l = r2c_log2n(n);
    if (l < 0)
        return 0;
    return (size_t)(n / 2) * sizeof(fdas_cf32);
}

int fdas_r2c(const float* x_dev, int64_t n, float scale, fdas_cf32* spec_dev, void* ws_dev,
             size_t ws_bytes, hipStream_t stream)
{
    const int l = r2c_log2n(n);
    if (l < 0)
        return fail(FDAS_UNSUPPORTED, "n = %lld is not a power of two in [2^13, 2^27]",
                    (long long)n);
    if (!x_dev || !spec_dev || !ws_dev)
        return fail(FDAS_INVALID_ARG, "x, spec and ws must not be NULL");
    if (!aligned(x_dev, 8) || !aligned(spec_dev, 8) || !aligned(ws_dev, 256))
        return fail(FDAS_INVALID_ARG, "misaligned pointer (x and spec 8 B, ws 256 B)");
    const size_t need = fdas_r2c_workspace_bytes(n);
    if (ws_bytes < need)
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    need);
    const auto xb = reinterpret_cast<uintptr_t>(x_dev), sb = reinterpret_cast<uintptr_t>(spec_dev),
               wb = reinterpret_cast<uintptr_t>(ws_dev);
    const uintptr_t xe = xb + (uintptr_t)n * 4, se = sb + (uintptr_t)(n / 2 + 1) * 8,
                    we = wb + need;
    if ((xb < se && sb < xe) || (xb < we && wb < xe) || (sb < we && wb < se))
        return fail(FDAS_INVALID_ARG, "x, spec and ws must not overlap");
    hipError_t e = fdas::launch_r2c(x_dev, l, scale, reinterpret_cast<float2*>(spec_dev),
                                    reinterpret_cast<float2*>(ws_dev), stream);
    if (e != hipSuccess)
        return hip_fail(e, "r2c launch");
    return ok();
}

size_t fdas_r2c_batched_workspace_bytes(int64_t n, int nseries)
{
    const int l = r2c_log2n(n);
    if (l < 0 || nseries < 1 || nseries > 65535)
        return 0;
    return (size_t)nseries * (size_t)(n / 2) * sizeof(fdas_cf32);
}

int fdas_r2c_batched(const float* x_dev, int64_t n, int nseries, float scale,
                     fdas_cf32* spec_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream)
{
    const int l = r2c_log2n(n);
    if (l < 0)
        return fail(FDAS_UNSUPPORTED, "n = %lld is not a power of two in [2^13, 2^27]",
                    (long long)n);
    if (nseries < 1 || nseries > 65535)
        return fail(FDAS_INVALID_ARG, "nseries = %d outside [1, 65535]", nseries);
    if (!x_dev || !spec_dev || !ws_dev)
        return fail(FDAS_INVALID_ARG, "x, spec and ws must not be NULL");
    if (!aligned(x_dev, 8) || !aligned(spec_dev, 8) || !aligned(ws_dev, 256))
        return fail(FDAS_INVALID_ARG, "misaligned pointer (x and spec 8 B, ws 256 B)");
    const size_t need = fdas_r2c_batched_workspace_bytes(n, nseries);
    if (ws_bytes < need)
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    need);
    const size_t xbytes = (size_t)nseries * (size_t)n * 4;
    const size_t sbytes = (size_t)nseries * (size_t)(n / 2 + 1) * 8;
    if (overlaps(x_dev, xbytes, spec_dev, sbytes) || overlaps(x_dev, xbytes, ws_dev, need) ||
        overlaps(spec_dev, sbytes, ws_dev, need))
        return fail(FDAS_INVALID_ARG, "x, spec and ws must not overlap");
    hipError_t e = fdas::launch_r2c_batched(x_dev, l, nseries, scale,
                                            reinterpret_cast<float2*>(spec_dev),
                                            reinterpret_cast<float2*>(ws_dev), stream);
    if (e != hipSuccess)
        return hip_fail(e, "batched r2c launch");
    return ok();
}

}  // extern "C"

// ---- harmonic summing and peak candidates ---------------------------------------

namespace {

int check_harmonic(int64_t N, int K, int H)
{
    if (N < 0 || N > kMaxN)
        return fail(FDAS_INVALID_ARG, "N = %lld outside [0, 2^32]", (long long)N);
    if (K < 1 || K > kMaxK || (K & 1) == 0)
        return fail(FDAS_INVALID_ARG, "K = %d must be odd in [1, %d]", K, kMaxK);
    if (!is_pow2(H) || H > 64)
        return fail(FDAS_INVALID_ARG, "H = %d must be a power of two in [1, 64]", H);
    return FDAS_OK;
}

}  // namespace

extern "C" {

int fdas_harmonic_shape(int64_t N, int K, int H, int* KH, int64_t* NH)
{
    const int st = check_harmonic(N, K, H);
    if (st)
        return st;
    if (!KH || !NH)
        return fail(FDAS_INVALID_ARG, "KH and NH must not be NULL");
    fdas::harmonic_shape(N, K, H, KH, NH);
    return ok();
}

int fdas_harmonic_sum(const float* plane_dev, int64_t N, int K, int H, const float* prev_dev,
                      float* sums_dev, hipStream_t stream)
{
    const int st = check_harmonic(N, K, H);
    if (st)
        return st;
    if (prev_dev && H < 2)
        return fail(FDAS_INVALID_ARG, "a previous fold needs H >= 2");
    int KH = 0, KHp = 0;
    int64_t NH = 0, NHp = 0;
    fdas::harmonic_shape(N, K, H, &KH, &NH);
    if (NH == 0)
        return ok();
    if (!plane_dev || !sums_dev)
        return fail(FDAS_INVALID_ARG, "plane and sums must not be NULL");
    if (!aligned(plane_dev, 4) || !aligned(sums_dev, 4) || (prev_dev && !aligned(prev_dev, 4)))
        return fail(FDAS_INVALID_ARG, "misaligned pointer (4 B)");
    const size_t out_bytes = (size_t)KH * (size_t)NH * sizeof(float);
    if (overlaps(sums_dev, out_bytes, plane_dev, (size_t)K * (size_t)N * sizeof(float)))
        return fail(FDAS_INVALID_ARG, "sums must not overlap the plane");
    if (prev_dev) {
        fdas::harmonic_shape(N, K, H / 2, &KHp, &NHp);
        if (overlaps(sums_dev, out_bytes, prev_dev, (size_t)KHp * (size_t)NHp * sizeof(float)))
            return fail(FDAS_INVALID_ARG, "sums must not overlap the previous fold");
    }
    const hipError_t e =
        fdas::launch_harmonic_sum(plane_dev, N, K, H, prev_dev, sums_dev, stream);
    if (e != hipSuccess)
        return hip_fail(e, "harmonic sum launch");
    return ok();
}

int fdas_find_candidates(const float* sums_dev, int64_t N, int K, int H, float threshold,
                         fdas_candidate* out_dev, int capacity, unsigned* count_dev,
                         hipStream_t stream)
{
    const int st = check_harmonic(N, K, H);
    if (st)
        return st;
    if (capacity < 0)
        return fail(FDAS_INVALID_ARG, "capacity = %d must be >= 0", capacity);
    if (!count_dev || !aligned(count_dev, 4))
        return fail(FDAS_INVALID_ARG, "count must be a 4-byte aligned device pointer");
    if (capacity > 0 && (!out_dev || !aligned(out_dev, 8)))
        return fail(FDAS_INVALID_ARG, "out must be an 8-byte aligned device pointer");
    int KH = 0;
    int64_t NH = 0;
    fdas::harmonic_shape(N, K, H, &KH, &NH);
    if (NH > 0 && (!sums_dev || !aligned(sums_dev, 4)))
        return fail(FDAS_INVALID_ARG, "sums must be a 4-byte aligned device pointer");
    const hipError_t e = fdas::launch_candidates(sums_dev, N, K, H, threshold, out_dev,
                                                 capacity, count_dev, stream);
    if (e != hipSuccess)
        return hip_fail(e, "candidates launch");
    return ok();
}

}  // extern "C"

extern "C" {

size_t fdas_harmonic_batched_workspace_bytes(int nspec)
{
    if (nspec < 0 || nspec > kMaxSpectra)
        return 0;
    const size_t b = 2 * ((size_t)nspec + 1) * sizeof(int64_t);
    return (b + 255) & ~(size_t)255;
}

namespace {

int check_harmonic_batched(const int64_t* offsets_dev, int nspec, int K, int H, void* ws_dev,
                           size_t ws_bytes)
{
    const int st = check_harmonic(0, K, H);
    if (st)
        return st;
    if (nspec < 0 || nspec > kMaxSpectra)
        return fail(FDAS_INVALID_ARG, "nspec = %d outside [0, %d]", nspec, kMaxSpectra);
    if (nspec == 0)
        return FDAS_OK;
    if (!offsets_dev || !ws_dev || !aligned(offsets_dev, 8) || !aligned(ws_dev, 8))
        return fail(FDAS_INVALID_ARG, "offsets and ws must be 8-byte aligned device pointers");
    if (ws_bytes < fdas_harmonic_batched_workspace_bytes(nspec))
        return fail(FDAS_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    fdas_harmonic_batched_workspace_bytes(nspec));
    return FDAS_OK;
}

}  // namespace

int fdas_harmonic_sum_batched(const float* planes_dev, const int64_t* offsets_dev, int nspec,
                              int K, int H, const float* prev_dev, float* sums_dev, void* ws_dev,
                              size_t ws_bytes, hipStream_t stream)
{
    const int st = check_harmonic_batched(offsets_dev, nspec, K, H, ws_dev, ws_bytes);
    if (st)
        return st;
    if (prev_dev && H < 2)
        return fail(FDAS_INVALID_ARG, "a previous fold needs H >= 2");
    if (nspec == 0)
        return ok();
    if (!planes_dev || !sums_dev || !aligned(planes_dev, 4) || !aligned(sums_dev, 4) ||
        (prev_dev && !aligned(prev_dev, 4)))
        return fail(FDAS_INVALID_ARG, "planes and sums must be 4-byte aligned device pointers");
    auto* pre = static_cast<int64_t*>(ws_dev);
    const hipError_t e = fdas::launch_harmonic_batched(planes_dev, offsets_dev, nspec, K, H,
                                                       prev_dev, sums_dev, pre, pre + nspec + 1,
                                                       stream);
    if (e != hipSuccess)
        return hip_fail(e, "batched harmonic sum launch");
    return ok();
}

int fdas_find_candidates_batched(const float* sums_dev, const int64_t* offsets_dev, int nspec,
                                 int K, int H, float threshold, fdas_candidate* out_dev,
                                 int capacity, unsigned* count_dev, void* ws_dev,
                                 size_t ws_bytes, hipStream_t stream)
{
    const int st = check_harmonic_batched(offsets_dev, nspec, K, H, ws_dev, ws_bytes);
    if (st)
        return st;
    if (capacity < 0)
        return fail(FDAS_INVALID_ARG, "capacity = %d must be >= 0", capacity);
    if (!count_dev || !aligned(count_dev, 4))
        return fail(FDAS_INVALID_ARG, "count must be a 4-byte aligned device pointer");
    if (capacity > 0 && (!out_dev || !aligned(out_dev, 8)))
        return fail(FDAS_INVALID_ARG, "out must be an 8-byte aligned device pointer");
    if (nspec > 0 && (!sums_dev || !aligned(sums_dev, 4)))
        return fail(FDAS_INVALID_ARG, "sums must be a 4-byte aligned device pointer");
    if (nspec == 0) {
        // still a defined count: zero
        const hipError_t e = fdas::launch_candidates(nullptr, 0, K, H, threshold, out_dev,
                                                     capacity, count_dev, stream);
        return e == hipSuccess ? ok() : hip_fail(e, "candidates launch");
    }
    auto* pre = static_cast<int64_t*>(ws_dev);
    const hipError_t e = fdas::launch_candidates_batched(sums_dev, offsets_dev, nspec, K, H,
                                                         threshold, out_dev, capacity, count_dev,
                                                         pre, pre + nspec + 1, stream);
    if (e != hipSuccess)
        return hip_fail(e, "batched candidates launch");
    return ok();
}

int fdas_stream_write(float* dst_dev, int64_t n, float value, hipStream_t stream)
{
    if (n < 0)
        return fail(FDAS_INVALID_ARG, "n must be >= 0");
    if (n == 0)
        return ok();
    if (!dst_dev || !aligned(dst_dev, 16))
        return fail(FDAS_INVALID_ARG, "dst must be a 16-byte aligned device pointer");
    const hipError_t e = fdas::launch_stream_write(dst_dev, n, value, stream);
    return e == hipSuccess ? ok() : hip_fail(e, "stream write launch");
}

int fdas_stream_read(const float* src_dev, int64_t n, float* sums_dev, hipStream_t stream)
{
    if (n < 0)
        return fail(FDAS_INVALID_ARG, "n must be >= 0");
    if (!sums_dev || !aligned(sums_dev, 4))
        return fail(FDAS_INVALID_ARG, "sums must be a 4-byte aligned device pointer");
    if (n > 0 && (!src_dev || !aligned(src_dev, 16)))
        return fail(FDAS_INVALID_ARG, "src must be a 16-byte aligned device pointer");
    if (n > 0 && overlaps(sums_dev, FDAS_STREAM_PARTIALS * sizeof(float), src_dev,
                          (size_t)n * sizeof(float)))
        return fail(FDAS_INVALID_ARG, "sums must not overlap src");
    const hipError_t e = fdas::launch_stream_read(n > 0 ? src_dev : nullptr, n, sums_dev, stream);
    return e == hipSuccess ? ok() : hip_fail(e, "stream read launch");
}

}  // extern "C"

int fdas_lds_probe(const int* pattern_dev, int mode, int iters, int groups,
                   long long* cycles_dev, float* sink_dev, hipStream_t stream)
{
    if (mode < 0 || mode > 2)
        return fail(FDAS_INVALID_ARG, "mode = %d is not 0, 1 or 2", mode);
    if (iters < 1 || iters > (1 << 20) || groups < 1 || groups > (1 << 16))
        return fail(FDAS_INVALID_ARG, "iters = %d or groups = %d out of range", iters, groups);
    if (!pattern_dev || !cycles_dev || !sink_dev)
        return fail(FDAS_INVALID_ARG, "pattern, cycles and sink must not be NULL");
    if (!aligned(pattern_dev, 4) || !aligned(cycles_dev, 8) || !aligned(sink_dev, 4))
        return fail(FDAS_INVALID_ARG, "misaligned pointer");
    const hipError_t e = fdas::launch_lds_probe(pattern_dev, mode, iters, groups, cycles_dev,
                                                sink_dev, stream);
    if (e != hipSuccess)
        return hip_fail(e, "LDS probe launch");
    return ok();
}
