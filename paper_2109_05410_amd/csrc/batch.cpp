// batch.cpp -- batched in-core heat domains: work-list table, autotuner
// with a cache file, graph of batched steps, per-domain baseline.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "abi_util.hpp"
#include "internal.hpp"
#include "oocs.h"

using oocs::fail;

struct oocs_batch {
    std::vector<oocs_domain> doms;
    std::vector<oocs::BatchDomain> table;
    oocs::BatchDomain* d_table = nullptr;
    int32_t total_wg = 0;
    float alpha = 0.1f;
    std::map<int64_t, hipGraphExec_t> graphs;  // by step count
};

namespace {

// Size bucket of a domain: by its largest side, 64..127 -> 0, 128..255 -> 1, ...
int bucket_of(const oocs_domain& d)
{
    const int64_t m = std::max(d.nx, std::max(d.ny, d.nz));
    int b = 0;
    for (int64_t s = 128; m >= s && b < 8; s *= 2) ++b;
    return b;
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

// Cache file: a JSON object {"<arch>/heat7/bucket<b>": <cfg index>, ...}.
std::map<std::string, int> read_cache(const char* path)
{
    std::map<std::string, int> m;
    if (!path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        const size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = t.substr(i + 1, j - i - 1);
        size_t k = t.find(':', j);
        if (k == std::string::npos) break;
        int v = -1;
        if (std::sscanf(t.c_str() + k + 1, "%d", &v) == 1 && v >= 0 && v < oocs::kNumTileCfgs) m[key] = v;
        i = j + 1;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m)
{
    if (!path) return;
    std::ofstream f(path);
    if (!f) return;
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : m) {
        f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
        const oocs::TileCfg& t = oocs::kTileCfgs[kv.second];
        (void)t;
    }
    f << "}\n";
}

// Time one tile configuration on a domain: median of 3 timed launches.
int time_cfg(const oocs_domain& d, float alpha, int cfg, hipStream_t s, float* ms_out)
{
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<float> t;
    int rc = OOCS_OK;
    for (int r = 0; r < 4 && rc == OOCS_OK; ++r) {
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = oocs::launch_heat_dense(d.d_u, d.d_scratch, (int)d.nx, (int)d.ny, (int)d.nz, alpha, cfg, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = oocs::hip_fail(e, "tuning launch");
        if (r > 0) t.push_back(ms);  // first launch warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return OOCS_OK;
}

}  // namespace

extern "C" {

size_t oocs_batch_table_bytes(int nd) { return nd > 0 ? (size_t)nd * sizeof(oocs::BatchDomain) : 0; }

int oocs_batch_create(const oocs_domain* doms, int nd, float alpha, void* d_table, size_t table_bytes,
                      const char* tune_cache, int tune, void* stream, oocs_batch** out)
{
    if (!doms || nd <= 0 || !d_table || !out) return fail(OOCS_E_ARG, "bad argument");
    if (table_bytes < oocs_batch_table_bytes(nd)) return fail(OOCS_E_SIZE, "table buffer too small");
    *out = nullptr;
    for (int i = 0; i < nd; ++i) {
        const oocs_domain& d = doms[i];
        if (!d.d_u || !d.d_scratch || d.nx <= 0 || d.ny <= 0 || d.nz <= 0 || d.nx > (1 << 16) || d.ny > (1 << 16) ||
            d.nz > (1 << 16) || d.nx * d.ny > ((int64_t)1 << 28))
            return fail(OOCS_E_ARG, "bad domain");
    }
    hipStream_t s = (hipStream_t)stream;
    oocs_batch* b = new (std::nothrow) oocs_batch();
    if (!b) return fail(OOCS_E_ARG, "out of host memory");
    b->doms.assign(doms, doms + nd);
    b->alpha = alpha;
    b->d_table = static_cast<oocs::BatchDomain*>(d_table);
    // autotune per size bucket
    const std::string arch = arch_name();
    std::map<std::string, int> cache = read_cache(tune_cache);
    std::map<int, int> choice;  // bucket -> cfg
    bool cache_dirty = false;
    for (int i = 0; i < nd; ++i) {
        const int bk = bucket_of(doms[i]);
        if (choice.count(bk)) continue;
        const std::string key = arch + "/heat7/bucket" + std::to_string(bk);
        auto it = cache.find(key);
        if (it != cache.end()) { choice[bk] = it->second; continue; }
        if (!tune) { choice[bk] = 0; continue; }
        // representative: the largest domain of the bucket
        int rep = i;
        for (int q = 0; q < nd; ++q)
            if (bucket_of(doms[q]) == bk && doms[q].nx * doms[q].ny * doms[q].nz > doms[rep].nx * doms[rep].ny * doms[rep].nz)
                rep = q;
        int best = 0;
        float best_ms = 0;
        for (int c = 0; c < oocs::kNumTileCfgs; ++c) {
            float ms;
            const int rc = time_cfg(doms[rep], alpha, c, s, &ms);
            if (rc) { delete b; return rc; }
            if (c == 0 || ms < best_ms) { best = c; best_ms = ms; }
        }
        choice[bk] = best;
        cache[key] = best;
        cache_dirty = true;
    }
    if (cache_dirty) write_cache(tune_cache, cache);
    int32_t total = 0;
    b->table.resize(nd);
    for (int i = 0; i < nd; ++i) {
        oocs::BatchDomain& e = b->table[i];
        e.a = doms[i].d_u;
        e.b = doms[i].d_scratch;
        e.nx = (int32_t)doms[i].nx; e.ny = (int32_t)doms[i].ny; e.nz = (int32_t)doms[i].nz;
        e.cfg = choice[bucket_of(doms[i])];
        e.wg_begin = total;
        e.pad = 0;
        const int64_t w = oocs::batch_domain_workgroups(e.nx, e.ny, e.nz, e.cfg);
        if (total + w > INT32_MAX / 2) { delete b; return fail(OOCS_E_ARG, "batch too large for one launch"); }
        total += (int32_t)w;
    }
    b->total_wg = total;
    hipError_t e = hipMemcpyAsync(b->d_table, b->table.data(), b->table.size() * sizeof(oocs::BatchDomain),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete b; return oocs::hip_fail(e, "table upload"); }
    *out = b;
    return OOCS_OK;
}

int oocs_batch_run(oocs_batch* b, int64_t steps, void* stream)
{
    if (!b || steps < 0) return fail(OOCS_E_ARG, "bad argument");
    if (steps == 0) return OOCS_OK;
    hipStream_t s = (hipStream_t)stream;
    auto it = b->graphs.find(steps);
    if (it == b->graphs.end()) {
        hipGraph_t g;
        HIP_TRY(hipGraphCreate(&g, 0));
        hipGraphNode_t prev = nullptr;
        hipError_t e = hipSuccess;
        for (int64_t t = 0; t < steps && e == hipSuccess; ++t) {
            hipGraphNode_t n;
            e = oocs::add_batch_step_node(b->d_table, (int)b->table.size(), b->total_wg, (int)(t & 1), b->alpha, g,
                                          prev ? &prev : nullptr, prev ? 1 : 0, &n);
            prev = n;
        }
        if (e == hipSuccess && (steps & 1)) {  // the state is in the scratch buffers: copy it back
            std::vector<hipGraphNode_t> copies;
            for (const oocs_domain& d : b->doms) {
                hipGraphNode_t n;
                e = hipGraphAddMemcpyNode1D(&n, g, &prev, 1, d.d_u, d.d_scratch, (size_t)(d.nx * d.ny * d.nz * 4),
                                            hipMemcpyDeviceToDevice);
                if (e != hipSuccess) break;
            }
        }
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return oocs::hip_fail(e, "batch graph");
        it = b->graphs.emplace(steps, exec).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s));
    return OOCS_OK;
}

int oocs_batch_run_per_domain(oocs_batch* b, int64_t steps, void* stream)
{
    if (!b || steps < 0) return fail(OOCS_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        const oocs_domain& d = b->doms[i];
        const int cfg = b->table[i].cfg;
        for (int64_t t = 0; t < steps; ++t) {
            const float* src = (t & 1) ? d.d_scratch : d.d_u;
            float* dst = (t & 1) ? d.d_u : d.d_scratch;
            HIP_TRY(oocs::launch_heat_dense(src, dst, (int)d.nx, (int)d.ny, (int)d.nz, b->alpha, cfg, s));
        }
        if (steps & 1)
            HIP_TRY(hipMemcpyAsync(d.d_u, d.d_scratch, (size_t)(d.nx * d.ny * d.nz * 4), hipMemcpyDeviceToDevice, s));
    }
    return OOCS_OK;
}

int oocs_batch_domain_tile(const oocs_batch* b, int domain, int* tx, int* ty, int* zc)
{
    if (!b || domain < 0 || domain >= (int)b->table.size()) return fail(OOCS_E_ARG, "bad argument");
    const oocs::TileCfg& t = oocs::kTileCfgs[b->table[domain].cfg];
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (zc) *zc = t.zc;
    return OOCS_OK;
}

int oocs_batch_destroy(oocs_batch* b)
{
    if (!b) return OOCS_OK;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    delete b;
    return OOCS_OK;
}

}  // extern "C"
