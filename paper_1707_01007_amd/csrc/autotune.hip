// Autotuner tables.
//
// Products: cfpq_autotune(n) times every candidate -- the fp4 and int8 MFMA
// products and the VALU product with 8, 16 and 32-word strips -- on synthetic
// operands of the padded size for n (counter-based pseudo-random bits,
// density 1/2, made on the device), keeps the fastest in a process-wide table
// keyed by ceil(log2(npad)), and the AUTO path of cfpq_closure / cfpq_product
// uses that entry.
// Batched engine: one route per padded side (resident workgroup, or the tile
// work list with 256 or 128 tiles), filled by cfpq_batch_autotune (which
// times the candidates on the caller's own instances, batch_api.hip) or by
// hand (cfpq_batch_tune_set); cfpq_batch_closure and the server read it.
// Both tables can be saved to and loaded from a small JSON file; the
// environment variable CFPQ_TUNE_CACHE names a file loaded at first use.
// Every candidate computes the same bits, so tuning never changes a result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch_engine.h"

namespace cfpq {
namespace {

struct TuneTable {
    std::mutex mu;
    std::map<int32_t, cfpq_tune_entry> by_bucket;
    std::map<int32_t, cfpq_batch_tune_entry> batch;  // by padded side
    bool env_loaded = false;
};

TuneTable& table() {
    static TuneTable t;
    return t;
}

int32_t bucket_of(int64_t npad) {
    int32_t b = 0;
    while ((int64_t{1} << b) < npad) ++b;
    return b;
}

// splitmix64 of (seed, index): a counter-based generator, so the operands
// are the same for every launch configuration.
__global__ void fill_random_kernel(uint64_t* __restrict__ p, size_t words, uint64_t seed) {
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        p[i] = z ^ (z >> 31);
    }
}

const char* path_name(int32_t p) { return p == CFPQ_PATH_FP4 ? "fp4" : p == CFPQ_PATH_MFMA ? "mfma" : "bits"; }

const char* route_name(int32_t r) { return r == CFPQ_ROUTE_RESIDENT ? "resident" : "tiles"; }

// A batch route the engine can run: RESIDENT only up to kSmallMaxPad, TILES
// with 128 or 256 tiles, a padded side that is a positive multiple of 256.
bool batch_entry_valid(const cfpq_batch_tune_entry& e) {
    if (e.npad <= 0 || e.npad % 256 != 0) return false;
    if (e.route == CFPQ_ROUTE_RESIDENT) return e.npad <= kSmallMaxPad;
    if (e.route == CFPQ_ROUTE_TILES) return e.tile == 128 || e.tile == 256;
    return false;
}

cfpq_status load_file(const char* path, std::map<int32_t, cfpq_tune_entry>& out,
                      std::map<int32_t, cfpq_batch_tune_entry>& batch_out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(CFPQ_EINVAL, std::string("cannot open ") + path);
    char line[512];
    int n_ok = 0;
    while (std::fgets(line, sizeof line, f)) {
        {
            // {"batch_npad": P, "route": "tiles", "tile": T, "ms": X, "instances": K}
            cfpq_batch_tune_entry b;
            std::memset(&b, 0, sizeof b);
            char rname[16] = {0};
            if (std::sscanf(line, " {\"batch_npad\": %d, \"route\": \"%15[a-z]\", \"tile\": %d, \"ms\": %f, "
                                  "\"instances\": %d",
                            &b.npad, rname, &b.tile, &b.ms, &b.instances) == 5) {
                b.route = std::strcmp(rname, "resident") == 0 ? CFPQ_ROUTE_RESIDENT
                          : std::strcmp(rname, "tiles") == 0  ? CFPQ_ROUTE_TILES
                                                              : 0;
                if (b.route == CFPQ_ROUTE_RESIDENT) b.tile = 0;
                if (batch_entry_valid(b)) batch_out[b.npad] = b;
                continue;
            }
        }
        // {"bucket": B, "npad": P, "path": "mfma", "tile": T, "ms": X}
        cfpq_tune_entry e;
        std::memset(&e, 0, sizeof e);
        char name[16] = {0};
        int bucket = 0;
        if (std::sscanf(line, " {\"bucket\": %d, \"npad\": %d, \"path\": \"%15[a-z0-9]\", \"tile\": %d, \"ms\": %f",
                        &bucket, &e.npad, name, &e.tile, &e.ms) == 5) {
            if (std::strcmp(name, "mfma") == 0) e.path = CFPQ_PATH_MFMA;
            else if (std::strcmp(name, "fp4") == 0) e.path = CFPQ_PATH_FP4;
            else if (std::strcmp(name, "bits") == 0) e.path = CFPQ_PATH_BITS;
            else continue;
            if (bucket < 0 || bucket > 40 || e.npad <= 0) continue;
            out[bucket] = e;
            ++n_ok;
        }
    }
    std::fclose(f);
    (void)n_ok;
    return CFPQ_OK;
}

void ensure_env_loaded(TuneTable& t) {
    if (t.env_loaded) return;
    t.env_loaded = true;
    const char* p = std::getenv("CFPQ_TUNE_CACHE");
    if (p && *p) {
        std::map<int32_t, cfpq_tune_entry> m;
        std::map<int32_t, cfpq_batch_tune_entry> mb;
        if (load_file(p, m, mb) == CFPQ_OK) {
            for (auto& kv : m) t.by_bucket[kv.first] = kv.second;
            for (auto& kv : mb) t.batch[kv.first] = kv.second;
        }
        clear_last_error();
    }
}

}  // namespace

BatchRoute batch_route(int64_t npad, const BatchRoute* forced) {
    BatchRoute r;
    if (forced) {
        r = *forced;
    } else {
        r.route = npad <= kSmallMaxPad ? kRouteResident : kRouteTiles;
        r.tile = 256;
        TuneTable& t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        ensure_env_loaded(t);
        auto it = t.batch.find(static_cast<int32_t>(npad));
        if (it != t.batch.end()) {
            r.route = it->second.route;
            r.tile = it->second.tile;
        }
    }
    if (r.route == kRouteResident && npad > kSmallMaxPad) r = BatchRoute{};
    if (r.route == kRouteTiles && r.tile != 128) r.tile = 256;
    return r;
}

void batch_tune_record(const cfpq_batch_tune_entry& e) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    ensure_env_loaded(t);
    t.batch[e.npad] = e;
}

bool tuned_choice(const Layout& L, int32_t* path, int32_t* tile, float* ms) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    ensure_env_loaded(t);
    auto it = t.by_bucket.find(bucket_of(L.npad));
    if (it == t.by_bucket.end()) return false;
    const cfpq_tune_entry& e = it->second;
    if (reads_ct(e.path) && L.n > kMfmaMaxNodes) return false;
    if (e.path == CFPQ_PATH_FP4 && !fp4_tile_supported(e.tile)) {
        *path = CFPQ_PATH_FP4;
        *tile = 0;
        return true;
    }
    if (e.path == CFPQ_PATH_BITS && e.tile != 0 && !bits_strip_supported(e.tile, L)) {
        *path = CFPQ_PATH_BITS;
        *tile = 0;
        return true;
    }
    *path = e.path;
    *tile = e.tile;
    if (ms) *ms = e.ms;
    return true;
}

}  // namespace cfpq

using namespace cfpq;

extern "C" {

size_t cfpq_autotune_workspace_bytes(int32_t n_nodes) {
    if (n_nodes < 0) return 0;
    return static_cast<size_t>(layout_for(n_nodes).mat_words) * 8 * 4 + 256;
}

cfpq_status cfpq_autotune(int32_t n_nodes, void* stream, void* d_workspace, size_t workspace_bytes,
                          cfpq_tune_entry* out) {
    clear_last_error();
    if (n_nodes < 1 || n_nodes > CFPQ_MAX_NODES) return fail(CFPQ_EINVAL, "n_nodes out of range");
    if (!d_workspace || workspace_bytes < cfpq_autotune_workspace_bytes(n_nodes))
        return fail(CFPQ_ENOMEM, "workspace smaller than cfpq_autotune_workspace_bytes");
    const Layout L = layout_for(n_nodes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t mw = static_cast<size_t>(L.mat_words);
    auto* base = static_cast<uint64_t*>(d_workspace);
    uint64_t *B = base, *C = base + mw, *A = base + 2 * mw, *CT = base + 3 * mw;
    auto* flag = reinterpret_cast<int32_t*>(base + 4 * mw);
    fill_random_kernel<<<dim3(1024), dim3(256), 0, s>>>(base, 2 * mw, 0x5EEDull + static_cast<uint64_t>(n_nodes));
    CFPQ_HIP(hipGetLastError());
    CFPQ_HIP(launch_transpose(C, CT, L, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CFPQ_HIP(hipEventCreate(&e0));
    CFPQ_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } guard{e0, e1};
    struct Cand {
        int32_t path, tile;
    };
    std::vector<Cand> cands;
    if (L.n <= kMfmaMaxNodes) {
        cands.push_back({CFPQ_PATH_FP4, 0});  // the default pipeline depth (3 measured the same)
        cands.push_back({CFPQ_PATH_MFMA, 0});
    }
    for (int strip : {8, 16, 32})
        if (bits_strip_supported(strip, L)) cands.push_back({CFPQ_PATH_BITS, strip});
    const double work = static_cast<double>(L.npad) * L.npad * L.npad;
    const int reps = work > 1e12 ? 3 : (work > 1e10 ? 7 : 21);
    const size_t nc = std::min<size_t>(cands.size(), 8);
    auto launch = [&](size_t c) -> hipError_t {
        if (reads_ct(cands[c].path)) return launch_mfma_path(cands[c].path, B, CT, A, L, flag, s, nullptr, 1, cands[c].tile);
        return launch_bits_product(B, C, A, L, flag, s, cands[c].tile);
    };
    // Every candidate once first (code load, clocks up), then the timed
    // launches round-robin, one event pair each, so that no candidate is
    // favoured by its place in the order; the median launch of each counts.
    for (size_t c = 0; c < nc; ++c) CFPQ_HIP(launch(c));
    std::vector<std::vector<float>> times(nc);
    for (int r = 0; r < reps; ++r) {
        for (size_t c = 0; c < nc; ++c) {
            CFPQ_HIP(hipEventRecord(e0, s));
            CFPQ_HIP(launch(c));
            CFPQ_HIP(hipEventRecord(e1, s));
            CFPQ_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            CFPQ_HIP(hipEventElapsedTime(&ms, e0, e1));
            times[c].push_back(ms);
        }
    }
    cfpq_tune_entry best;
    std::memset(&best, 0, sizeof best);
    best.npad = static_cast<int32_t>(L.npad);
    best.ms = 1e30f;
    for (size_t c = 0; c < nc; ++c) {
        std::sort(times[c].begin(), times[c].end());
        const float ms = times[c][times[c].size() / 2];
        best.candidates_ms[c] = ms;
        best.candidate_path[c] = cands[c].path;
        best.candidate_tile[c] = cands[c].tile;
        if (ms < best.ms) {
            best.ms = ms;
            best.path = cands[c].path;
            best.tile = cands[c].tile;
        }
    }
    best.n_candidates = static_cast<int32_t>(std::min<size_t>(cands.size(), 8));
    {
        TuneTable& t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        ensure_env_loaded(t);
        t.by_bucket[bucket_of(L.npad)] = best;
    }
    if (out) *out = best;
    return CFPQ_OK;
}

cfpq_status cfpq_tune_get(int32_t n_nodes, cfpq_tune_entry* out) {
    clear_last_error();
    if (n_nodes < 0 || !out) return fail(CFPQ_EINVAL, "bad argument");
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    ensure_env_loaded(t);
    auto it = t.by_bucket.find(bucket_of(layout_for(n_nodes).npad));
    if (it == t.by_bucket.end()) return CFPQ_ENOTREADY;
    *out = it->second;
    return CFPQ_OK;
}

cfpq_status cfpq_tune_save(const char* path) {
    clear_last_error();
    if (!path) return fail(CFPQ_EINVAL, "path is NULL");
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(CFPQ_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [\n");
    size_t k = 0;
    for (auto& kv : t.by_bucket) {
        const cfpq_tune_entry& e = kv.second;
        std::fprintf(f, " {\"bucket\": %d, \"npad\": %d, \"path\": \"%s\", \"tile\": %d, \"ms\": %.6f}%s\n", kv.first,
                     e.npad, path_name(e.path), e.tile, e.ms, (++k < t.by_bucket.size()) ? "," : "");
    }
    std::fprintf(f, "], \"batch\": [\n");
    k = 0;
    for (auto& kv : t.batch) {
        const cfpq_batch_tune_entry& e = kv.second;
        std::fprintf(f, " {\"batch_npad\": %d, \"route\": \"%s\", \"tile\": %d, \"ms\": %.6f, \"instances\": %d}%s\n",
                     e.npad, route_name(e.route), e.tile, e.ms, e.instances, (++k < t.batch.size()) ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    return CFPQ_OK;
}

cfpq_status cfpq_tune_load(const char* path) {
    clear_last_error();
    if (!path) return fail(CFPQ_EINVAL, "path is NULL");
    std::map<int32_t, cfpq_tune_entry> m;
    std::map<int32_t, cfpq_batch_tune_entry> mb;
    cfpq_status st = load_file(path, m, mb);
    if (st != CFPQ_OK) return st;
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    t.env_loaded = true;
    for (auto& kv : m) t.by_bucket[kv.first] = kv.second;
    for (auto& kv : mb) t.batch[kv.first] = kv.second;
    return CFPQ_OK;
}

void cfpq_tune_clear(void) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    t.by_bucket.clear();
    t.batch.clear();
    t.env_loaded = true;
}

cfpq_status cfpq_batch_tune_get(int32_t npad, cfpq_batch_tune_entry* out) {
    clear_last_error();
    if (!out) return fail(CFPQ_EINVAL, "out is NULL");
    TuneTable& t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    ensure_env_loaded(t);
    auto it = t.batch.find(npad);
    if (it == t.batch.end()) return CFPQ_ENOTREADY;
    *out = it->second;
    return CFPQ_OK;
}

cfpq_status cfpq_batch_tune_set(const cfpq_batch_tune_entry* entry) {
    clear_last_error();
    if (!entry) return fail(CFPQ_EINVAL, "entry is NULL");
    TuneTable& t = table();
    if (entry->route == 0) {
        std::lock_guard<std::mutex> lk(t.mu);
        ensure_env_loaded(t);
        t.batch.erase(entry->npad);
        return CFPQ_OK;
    }
    cfpq_batch_tune_entry e = *entry;
    if (e.route == CFPQ_ROUTE_RESIDENT) e.tile = 0;
    if (!batch_entry_valid(e))
        return fail(CFPQ_EINVAL, "batch route: padded side must be a positive multiple of 256, RESIDENT at most "
                                 "512, TILES with tile 128 or 256");
    batch_tune_record(e);
    return CFPQ_OK;
}

}  // extern "C"
