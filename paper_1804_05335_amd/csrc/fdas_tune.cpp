// Autotuner for the batched forward: picks the segment length L (and the
// persistent grid) by timing the caller's own batch.  The paper tunes the
// filter (segment) size and launch shape per card by hand (Sec. 5.1.2, and
// Sec. 4.1 on the cuFFT version); here the search runs on the device the
// call is made on and the result is cached per problem shape.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/fdas.h"
#include "fdas_internal.h"

namespace {

struct Choice {
    int L, grid;
    double ms;
};

using Key = std::tuple<int, int, int, int, int>;   // device, K, M, nspec, log2(total bins)
std::mutex g_mu;
std::map<Key, Choice> g_cache;

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

int ilog2(int64_t x)
{
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

}  // namespace

extern "C" {

size_t fdas_autotune_workspace_bytes(int K, int nspec)
{
    if (K < 1 || nspec < 0)
        return 0;
    return round256((size_t)(K + 1) * 8192 * sizeof(fdas_cf32)) +
           fdas_batched_workspace_bytes(nspec);
}

int fdas_autotune_batched(const fdas_cf32* taps_dev, int K, int M, const fdas_cf32* specs_dev,
                          const int64_t* offsets_dev, int nspec, float* planes_dev, void* ws_dev,
                          size_t ws_bytes, hipStream_t stream, int* L_out, int* grid_out,
                          double* ms_out)
{
    using fdas::fail_status;
    if (!L_out || !grid_out)
        return fail_status(FDAS_INVALID_ARG, "L_out and grid_out must not be NULL");
    if (K < 1 || K > 4096 || M < 2 || (M & 1) || M > 4096 || nspec < 1)
        return fail_status(FDAS_INVALID_ARG, "need 1 <= K <= 4096, even 2 <= M <= 4096, nspec >= 1");
    if (!taps_dev || !specs_dev || !offsets_dev || !planes_dev || !ws_dev)
        return fail_status(FDAS_INVALID_ARG, "taps, specs, offsets, planes and ws must not be NULL");
    if ((reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0)
        return fail_status(FDAS_INVALID_ARG, "ws_dev must be 256-byte aligned");
    if (ws_bytes < fdas_autotune_workspace_bytes(K, nspec))
        return fail_status(FDAS_WORKSPACE_TOO_SMALL, "autotune workspace too small");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "hipGetDevice failed");
    int64_t total = 0;
    if (hipMemcpyAsync(&total, offsets_dev + nspec, sizeof(total), hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "reading offsets[nspec] failed");
    const Key key{dev, K, M, nspec, ilog2(total > 0 ? total : 1)};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *L_out = it->second.L;
            *grid_out = it->second.grid;
            if (ms_out)
                *ms_out = it->second.ms;
            return FDAS_OK;
        }
    }
    auto* base = static_cast<unsigned char*>(ws_dev);
    auto* bank = reinterpret_cast<fdas_cf32*>(base);
    void* bws = base + round256((size_t)(K + 1) * 8192 * sizeof(fdas_cf32));
    const size_t bws_bytes = fdas_batched_workspace_bytes(nspec);

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail_status(FDAS_HIP_ERROR, "hipEventCreate failed");
    }
    Choice best{0, 0, 1e300};
    int status = FDAS_OK;
    for (int L = 512; L <= 8192 && status == FDAS_OK; L *= 2) {
        if (M > L / 2)
            continue;
        if (fdas_prepare_bank(taps_dev, K, M, L, bank, stream) != FDAS_OK) {
            status = FDAS_HIP_ERROR;
            break;
        }
        // the grid is the resident workgroup count (0): one launch to warm
        // up, then the mean of three
        if (fdas_correlate_batched_ex(specs_dev, offsets_dev, nspec, bank, K, M, L, planes_dev,
                                      0, bws, bws_bytes, stream) != FDAS_OK) {
            status = FDAS_HIP_ERROR;
            break;
        }
        const int reps = 3;
        bool okrun = hipEventRecord(e0, stream) == hipSuccess;
        for (int r = 0; r < reps && okrun; ++r)
            okrun = fdas_correlate_batched_ex(specs_dev, offsets_dev, nspec, bank, K, M, L,
                                              planes_dev, 0, bws, bws_bytes, stream) == FDAS_OK;
        okrun = okrun && hipEventRecord(e1, stream) == hipSuccess &&
                hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (!okrun || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            status = FDAS_HIP_ERROR;
            break;
        }
        if (ms / reps < best.ms)
            best = Choice{L, 0, ms / reps};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != FDAS_OK)
        return fail_status(status, "a timed trial failed");
    if (best.L == 0)
        return fail_status(FDAS_UNSUPPORTED, "no supported segment length has M <= L/2");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = best;
    }
    *L_out = best.L;
    *grid_out = best.grid;
    if (ms_out)
        *ms_out = best.ms;
    return fail_status(FDAS_OK, "");
}

}  // extern "C"
