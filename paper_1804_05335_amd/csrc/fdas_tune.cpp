// Autotuner for the batched forward: picks the segment length L, the values
// per lane E of the segment transforms and the persistent grid by timing the
// caller's own batch.  The paper tunes the filter (segment) size and the
// launch shape per card by hand (Sec. 5.1.2, and Sec. 4.1 on the cuFFT
// version); here the search runs on the device the call is made on, and the
// choice is kept in a process cache and in a JSON file that persists across
// processes, keyed by the device's architecture and compute-unit count and
// the problem's shape (K, M, and the batch size as powers of two).
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unistd.h>
#include <vector>

#include "../../include/fdas.h"
#include "fdas_internal.h"

namespace {

struct Entry {
    int L, E, grid_factor;
    double ms;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;     // this process's choices (and file entries read)

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

// Path of the persistent cache: $FDAS_TUNE_CACHE (empty: no file), else
// $XDG_CACHE_HOME/fdas/autotune.json, else $HOME/.cache/fdas/autotune.json.
std::string cache_path()
{
    if (const char* p = std::getenv("FDAS_TUNE_CACHE"))
        return p;
    std::string dir;
    if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x)
        dir = x;
    else if (const char* h = std::getenv("HOME"); h && *h)
        dir = std::string(h) + "/.cache";
    else
        return "";
    return dir + "/fdas/autotune.json";
}

void make_parent_dirs(const std::string& path)
{
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') {
            const std::string d = path.substr(0, i);
            if (::mkdir(d.c_str(), 0755) != 0 && errno != EEXIST)
                return;
        }
}

// The file is a JSON object with one entry per line:
//   "key": {"L": 2048, "E": 16, "grid_factor": 1, "ms": 27.81},
// Lines that do not parse are ignored (a damaged file only loses entries).
std::map<std::string, Entry> read_file(const std::string& path)
{
    std::map<std::string, Entry> out;
    FILE* f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!f)
        return out;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        const char* q0 = std::strchr(line, '"');
        const char* q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        if (!q1)
            continue;
        Entry e{};
        if (std::sscanf(q1 + 1, " : {\"L\": %d, \"E\": %d, \"grid_factor\": %d, \"ms\": %lf}",
                        &e.L, &e.E, &e.grid_factor, &e.ms) == 4 &&
            e.L >= 256 && e.L <= 8192 && e.grid_factor >= 1 && e.grid_factor <= 8)
            out[std::string(q0 + 1, q1)] = e;
    }
    std::fclose(f);
    return out;
}

// Merge `key` into the file (re-read first, so entries other processes
// wrote are kept) and replace the file atomically.
void write_file(const std::string& path, const std::string& key, const Entry& e)
{
    if (path.empty())
        return;
    std::map<std::string, Entry> all = read_file(path);
    all[key] = e;
    make_parent_dirs(path);
    const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f)
        return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : all) {
        std::fprintf(f, "\"%s\": {\"L\": %d, \"E\": %d, \"grid_factor\": %d, \"ms\": %.6g}%s\n",
                     kv.first.c_str(), kv.second.L, kv.second.E, kv.second.grid_factor,
                     kv.second.ms, ++i < all.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (ok)
        std::rename(tmp.c_str(), path.c_str());
    else
        std::remove(tmp.c_str());
}

// Values per lane tried at segment length L: the default first.
std::vector<int> lane_values(int L)
{
    if (L <= 256)
        return {4};
    if (L == 512)
        return {8};
    return {16, 8};
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

int fdas_autotune_candidates(int K, int M, fdas_tuning* list, int capacity, int* count)
{
    using fdas::fail_status;
    if (!count || (capacity > 0 && !list) || capacity < 0)
        return fail_status(FDAS_INVALID_ARG, "count must not be NULL; list needs capacity >= 0");
    if (K < 1 || K > 4096 || M < 2 || (M & 1) || M > 4096)
        return fail_status(FDAS_INVALID_ARG, "need 1 <= K <= 4096, even 2 <= M <= 4096");
    int n = 0;
    for (int L = 512; L <= 8192; L *= 2) {
        if (M > L / 2)
            continue;
        for (int E : lane_values(L))
            for (int gf = 1; gf <= 2; ++gf) {
                if (n < capacity)
                    list[n] = fdas_tuning{L, E, gf, 0, 0, 0.0};
                ++n;
            }
    }
    *count = n;
    return fail_status(FDAS_OK, "");
}

int fdas_autotune_batched(const fdas_cf32* taps_dev, int K, int M, const fdas_cf32* specs_dev,
                          const int64_t* offsets_dev, int nspec, int64_t capacity,
                          float* planes_dev, void* ws_dev, size_t ws_bytes, int flags,
                          hipStream_t stream, fdas_tuning* out)
{
    using fdas::fail_status;
    if (!out)
        return fail_status(FDAS_INVALID_ARG, "out must not be NULL");
    if (K < 1 || K > 4096 || M < 2 || (M & 1) || M > 4096 || nspec < 1)
        return fail_status(FDAS_INVALID_ARG, "need 1 <= K <= 4096, even 2 <= M <= 4096, nspec >= 1");
    if (capacity < 1)
        return fail_status(FDAS_INVALID_ARG, "capacity must be >= 1");
    if (flags & ~(FDAS_TUNE_NO_CACHE | FDAS_TUNE_REFRESH))
        return fail_status(FDAS_INVALID_ARG, "unknown flag bits");
    if (!taps_dev || !specs_dev || !offsets_dev || !planes_dev || !ws_dev)
        return fail_status(FDAS_INVALID_ARG, "taps, specs, offsets, planes and ws must not be NULL");
    if ((reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0)
        return fail_status(FDAS_INVALID_ARG, "ws_dev must be 256-byte aligned");
    if (ws_bytes < fdas_autotune_workspace_bytes(K, nspec))
        return fail_status(FDAS_WORKSPACE_TOO_SMALL, "autotune workspace too small");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "device query failed");
    int64_t total = 0;
    if (hipMemcpyAsync(&total, offsets_dev + nspec, sizeof(total), hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "reading offsets[nspec] failed");
    if (total > capacity)
        total = capacity;
    char keybuf[256];
    std::snprintf(keybuf, sizeof(keybuf), "%s|cu%d|K%d|M%d|n2^%d|s2^%d", prop.gcnArchName,
                  prop.multiProcessorCount, K, M, ilog2(total > 0 ? total : 1), ilog2(nspec));
    const std::string key(keybuf);
    const bool use_cache = !(flags & FDAS_TUNE_NO_CACHE);
    const bool refresh = (flags & FDAS_TUNE_REFRESH) != 0;
    const std::string path = use_cache ? cache_path() : std::string();

    auto report = [&](const Entry& e, int from_cache) {
        // grid_factor times the resident workgroup count of that kernel;
        // factor 1 is reported as 0 (the call's own default)
        int grid = 0;
        if (e.grid_factor > 1) {
            int resident = 0;
            if (fdas::batched_resident_grid(e.L, e.E, M, &resident) != hipSuccess)
                return fail_status(FDAS_HIP_ERROR, "occupancy query failed");
            grid = e.grid_factor * resident;
        }
        *out = fdas_tuning{e.L, e.E, e.grid_factor, grid, from_cache, e.ms};
        return fail_status(FDAS_OK, "");
    };

    if (use_cache && !refresh) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it == g_cache.end()) {
            for (const auto& kv : read_file(path))
                g_cache.emplace(kv.first, kv.second);
            it = g_cache.find(key);
        }
        if (it != g_cache.end() && fdas::batched_values_per_lane_ok(it->second.L, it->second.E) &&
            M <= it->second.L / 2)
            return report(it->second, 1);
    }

    auto* base = static_cast<unsigned char*>(ws_dev);
    auto* bank = reinterpret_cast<fdas_cf32*>(base);
    void* bws = base + round256((size_t)(K + 1) * 8192 * sizeof(fdas_cf32));
    const size_t bws_bytes = fdas_batched_workspace_bytes(nspec);

    int ncand = 0;
    if (fdas_autotune_candidates(K, M, nullptr, 0, &ncand) != FDAS_OK || ncand == 0)
        return fail_status(FDAS_UNSUPPORTED, "no supported segment length has M <= L/2");
    std::vector<fdas_tuning> cand(ncand);
    fdas_autotune_candidates(K, M, cand.data(), ncand, &ncand);

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail_status(FDAS_HIP_ERROR, "hipEventCreate failed");
    }
    std::vector<double> best_ms(ncand, 1e300);
    int status = FDAS_OK;
    // three rounds over the candidates (the bank is prepared once per L and
    // round), each candidate one warm-up launch and the mean of three; the
    // best of its rounds counts, so a clock change during one round does
    // not decide the choice
    for (int round = 0; round < 3 && status == FDAS_OK; ++round) {
        int bankL = 0;
        for (int c = 0; c < ncand && status == FDAS_OK; ++c) {
            const int L = cand[c].L, E = cand[c].E;
            if (L != bankL) {
                if (fdas_prepare_bank(taps_dev, K, M, L, bank, stream) != FDAS_OK) {
                    status = FDAS_HIP_ERROR;
                    break;
                }
                bankL = L;
            }
            int grid = 0;
            if (cand[c].grid_factor > 1) {
                int resident = 0;
                if (fdas::batched_resident_grid(L, E, M, &resident) != hipSuccess) {
                    status = FDAS_HIP_ERROR;
                    break;
                }
                grid = cand[c].grid_factor * resident;
            }
            auto run = [&]() {
                return fdas_correlate_batched_ex(specs_dev, offsets_dev, nspec, capacity, bank, K,
                                                 M, L, planes_dev, E, grid, bws, bws_bytes,
                                                 stream) == FDAS_OK;
            };
            const int reps = 3;
            bool okrun = run() && hipEventRecord(e0, stream) == hipSuccess;
            for (int r = 0; r < reps && okrun; ++r)
                okrun = run();
            okrun = okrun && hipEventRecord(e1, stream) == hipSuccess &&
                    hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.f;
            if (!okrun || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                status = FDAS_HIP_ERROR;
                break;
            }
            if (ms / reps < best_ms[c])
                best_ms[c] = ms / reps;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != FDAS_OK) {
        const std::string why = std::string("a timed trial failed: ") + fdas_last_error();
        return fail_status(status, why.c_str());
    }
    int bc = 0;
    for (int c = 1; c < ncand; ++c)
        if (best_ms[c] < best_ms[bc])
            bc = c;
    const Entry best{cand[bc].L, cand[bc].E, cand[bc].grid_factor, best_ms[bc]};
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = best;
        write_file(path, key, best);
    }
    return report(best, 0);
}

}  // extern "C"

extern "C" int fdas_batched_resident_grid(int L, int E, int M, int* grid)
{
    using fdas::fail_status;
    if (!grid)
        return fail_status(FDAS_INVALID_ARG, "grid must not be NULL");
    if (L < 256 || L > 8192 || (L & (L - 1)) || M < 2 || (M & 1) || M > L / 2 ||
        !fdas::batched_values_per_lane_ok(L, E))
        return fail_status(FDAS_UNSUPPORTED, "unsupported (L, E, M)");
    if (fdas::batched_resident_grid(L, E, M, grid) != hipSuccess)
        return fail_status(FDAS_HIP_ERROR, "occupancy query failed");
    return fail_status(FDAS_OK, "");
}
