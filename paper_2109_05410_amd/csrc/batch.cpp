// batch.cpp -- batched in-core heat domains: work-list tables, autotuner of
// the tile shape (per size bucket, timed on the bucket's largest domain, with
// a cache file) and of the temporal-blocking depth (per batch, timed on one
// launch over all domains), graph of batched launches, per-domain baseline.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <climits>
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
    // two work lists: [0] every domain at the batch depth, [1] at depth 1
    // (the steps left when the step count is not a multiple of the depth)
    std::vector<oocs::BatchDomain> table[2];
    oocs::BatchDomain* d_table = nullptr;  // both lists, [0] then [1]
    int32_t* d_copy_begin = nullptr;       // nd + 1 prefix sums of copy items (persistent launches)
    uint32_t* d_sync = nullptr;            // queue, exit count, status, per-domain counts
    int32_t copy_items = 0;
    int32_t total_wg[2] = {0, 0};
    int32_t total_items[2] = {0, 0};       // persistent items of one group
    size_t lds[2] = {0, 0};
    int grid[2] = {0, 0};                  // persistent grid: [0] blocked tiles, [1] depth-1 tiles
    int depth = 1;
    float alpha = 0.1f;
    bool persistent = false;
    int64_t spin_limit = (int64_t)1 << 21;
    bool force_wait = false;
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
        if (std::sscanf(t.c_str() + k + 1, "%d", &v) == 1 && v >= 0) m[key] = v;
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
    }
    f << "}\n";
}

// Time one tile configuration on a domain: median of 3 timed launches (each
// the configuration's k steps).
int time_cfg(const oocs_domain& d, float alpha, int cfg, hipStream_t s, float* ms_out)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t ce = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);  // timing only
    if (ce == hipSuccess) ce = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (ce != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return oocs::hip_fail(ce, "tuning events");
    }
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

// Time one launch over a whole work list (the batch step at parity 0 reads
// every domain's field and writes its scratch buffer): median of 3 timed
// launches after one warm-up. The list is uploaded to the first nd entries
// of the device table, which the caller rewrites afterwards.
int time_batch(oocs::BatchDomain* d_table, const std::vector<oocs::BatchDomain>& tab, int32_t total, size_t lds,
               float alpha, hipStream_t s, float* ms_out)
{
    const int nd = (int)tab.size();
    HIP_TRY(hipMemcpyAsync(d_table, tab.data(), nd * sizeof(oocs::BatchDomain), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host list may go away on return
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t ce = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);  // timing only
    if (ce == hipSuccess) ce = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (ce != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return oocs::hip_fail(ce, "tuning events");
    }
    std::vector<float> t;
    int rc = OOCS_OK;
    for (int r = 0; r < 4 && rc == OOCS_OK; ++r) {
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = oocs::launch_batch_step(d_table, nd, total, lds, 0, alpha, s);
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

// Device buffer layout: the two work lists, the copy-item prefix sums
// (nd + 1 int32, padded to 16 bytes), then the persistent launch's counters
// (kBatchSyncWords + nd uint32).
static size_t copy_begin_offset(int nd) { return 2 * (size_t)nd * sizeof(oocs::BatchDomain); }
static size_t sync_offset(int nd) { return copy_begin_offset(nd) + ((size_t)(nd + 1) * 4 + 15) / 16 * 16; }

size_t oocs_batch_table_bytes(int nd)
{
    return nd > 0 ? sync_offset(nd) + ((size_t)oocs::kBatchSyncWords + nd) * 4 : 0;
}

int oocs_batch_create(const oocs_domain* doms, int nd, float alpha, void* d_table, size_t table_bytes,
                      const char* tune_cache, int tune, int depth, void* stream, oocs_batch** out)
{
    if (!doms || nd <= 0 || !d_table || !out) return fail(OOCS_E_ARG, "bad argument");
    if (table_bytes < oocs_batch_table_bytes(nd)) return fail(OOCS_E_SIZE, "table buffer too small");
    if (depth != 0 && depth != 1 && depth != 2 && depth != 4) return fail(OOCS_E_ARG, "depth must be 0, 1, 2 or 4");
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
    b->d_copy_begin = reinterpret_cast<int32_t*>(static_cast<char*>(d_table) + copy_begin_offset(nd));
    b->d_sync = reinterpret_cast<uint32_t*>(static_cast<char*>(d_table) + sync_offset(nd));
    const std::string arch = arch_name();
    std::map<std::string, int> cache = read_cache(tune_cache);
    bool cache_dirty = false;
    std::vector<int> depths = depth ? std::vector<int>{depth} : std::vector<int>{1, 2, 4};
    if (std::find(depths.begin(), depths.end(), 1) == depths.end()) depths.push_back(1);
    // per (bucket, depth): the best configuration and its time per step per cell (ps), or -1 if unknown
    std::map<std::pair<int, int>, std::pair<int, int64_t>> best;
    for (int i = 0; i < nd; ++i) {
        const int bk = bucket_of(doms[i]);
        for (int dk : depths) {
            if (best.count({bk, dk})) continue;
            const std::string key = arch + "/heat7/bucket" + std::to_string(bk) + "/k" + std::to_string(dk);
            auto it = cache.find(key);
            auto itp = cache.find(key + "/ps_per_cell");
            if (it != cache.end() && it->second < oocs::kNumTileCfgs && oocs::kTileCfgs[it->second].k == dk) {
                best[{bk, dk}] = {it->second, itp != cache.end() ? (int64_t)itp->second : -1};
                continue;
            }
            int first = 0;
            while (oocs::kTileCfgs[first].k != dk) ++first;
            if (!tune) { best[{bk, dk}] = {first, -1}; continue; }
            // representative: the largest domain of the bucket
            int rep = i;
            for (int q = 0; q < nd; ++q)
                if (bucket_of(doms[q]) == bk &&
                    doms[q].nx * doms[q].ny * doms[q].nz > doms[rep].nx * doms[rep].ny * doms[rep].nz)
                    rep = q;
            const double cells = (double)doms[rep].nx * doms[rep].ny * doms[rep].nz;
            int bc = first;
            float best_ms = -1;
            for (int c = 0; c < oocs::kNumTileCfgs; ++c) {
                if (oocs::kTileCfgs[c].k != dk) continue;
                float ms;
                const int rc = time_cfg(doms[rep], alpha, c, s, &ms);
                if (rc) { delete b; return rc; }
                if (best_ms < 0 || ms < best_ms) { bc = c; best_ms = ms; }
            }
            const int64_t ps = (int64_t)std::llround(best_ms * 1e9 / dk / cells);
            best[{bk, dk}] = {bc, ps};
            cache[key] = bc;
            cache[key + "/ps_per_cell"] = (int)std::min<int64_t>(ps, INT32_MAX);
            cache_dirty = true;
        }
    }
    if (cache_dirty) write_cache(tune_cache, cache);
    // work list of every domain at depth dk, with its workgroup total and LDS
    auto build_table = [&](int dk, std::vector<oocs::BatchDomain>& tab, int32_t& total, size_t& lds,
                           int32_t* items = nullptr) -> int {
        total = 0;
        lds = 0;
        int32_t nitems = 0;
        tab.resize(nd);
        for (int i = 0; i < nd; ++i) {
            oocs::BatchDomain& e = tab[i];
            e.a = doms[i].d_u;
            e.b = doms[i].d_scratch;
            e.nx = (int32_t)doms[i].nx; e.ny = (int32_t)doms[i].ny; e.nz = (int32_t)doms[i].nz;
            e.cfg = best[{bucket_of(doms[i]), dk}].first;
            e.wg_begin = total;
            e.item_begin = nitems;
            const int64_t wgs = oocs::batch_domain_workgroups(e.nx, e.ny, e.nz, e.cfg);
            if (total + wgs > INT32_MAX / 2) return fail(OOCS_E_ARG, "batch too large for one launch");
            total += (int32_t)wgs;
            nitems += (int32_t)((wgs + oocs::kBatchTilesPerItem - 1) / oocs::kBatchTilesPerItem);
            lds = std::max(lds, oocs::tile_cfg_lds(e.cfg));
        }
        if (items) *items = nitems;
        return OOCS_OK;
    };
    // depth: the forced one; else, when tuning, the one whose launch over the
    // whole batch (every domain's field read, only its scratch buffer
    // written) takes the least time per step; else the least estimated time
    b->depth = depths[0];
    if (!depth && tune) {
        double best_t = -1;
        for (int dk : depths) {
            std::vector<oocs::BatchDomain> tab;
            int32_t total;
            size_t lds;
            int rc = build_table(dk, tab, total, lds);
            float ms = 0;
            if (!rc) rc = time_batch(b->d_table, tab, total, lds, alpha, s, &ms);
            if (rc) { delete b; return rc; }
            const double t = (double)ms / dk;
            if (best_t < 0 || t < best_t) { best_t = t; b->depth = dk; }
        }
    } else if (!depth) {
        double best_t = -1;
        for (int dk : depths) {
            double t = 0;
            bool known = true;
            for (int i = 0; i < nd && known; ++i) {
                const auto& e = best[{bucket_of(doms[i]), dk}];
                if (e.second < 0) known = false;
                t += (double)e.second * doms[i].nx * doms[i].ny * doms[i].nz;
            }
            if (!known) continue;
            if (best_t < 0 || t < best_t) { best_t = t; b->depth = dk; }
        }
        if (best_t < 0) b->depth = 1;
    }
    for (int w = 0; w < 2; ++w) {
        const int rc = build_table(w == 0 ? b->depth : 1, b->table[w], b->total_wg[w], b->lds[w], &b->total_items[w]);
        if (rc) { delete b; return rc; }
    }
    // copy items of each domain (a result left in the scratch buffer is moved
    // back to u by items of kBatchCopyFloats floats)
    std::vector<int32_t> copy_begin(nd + 1, 0);
    for (int i = 0; i < nd; ++i) {
        const int64_t n = doms[i].nx * doms[i].ny * doms[i].nz;
        const int64_t items = (n + oocs::kBatchCopyFloats - 1) / oocs::kBatchCopyFloats;
        if (copy_begin[i] + items > INT32_MAX / 2) { delete b; return fail(OOCS_E_ARG, "batch too large"); }
        copy_begin[i + 1] = copy_begin[i] + (int32_t)items;
    }
    b->copy_items = copy_begin[nd];
    for (int w = 0; w < 2; ++w) {
        const int rc = oocs::batch_persistent_grid(w == 0, std::max(b->lds[0], b->lds[1]), &b->grid[w]);
        if (rc != hipSuccess) { delete b; return oocs::hip_fail((hipError_t)rc, "occupancy query"); }
    }
    hipError_t e = hipMemcpyAsync(b->d_table, b->table[0].data(), nd * sizeof(oocs::BatchDomain), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_table + nd, b->table[1].data(), nd * sizeof(oocs::BatchDomain), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_copy_begin, copy_begin.data(), (nd + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = oocs::launch_zero_words(b->d_sync, oocs::kBatchSyncWords + nd, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete b; return oocs::hip_fail(e, "table upload"); }
    *out = b;
    return OOCS_OK;
}

namespace {

// The persistent launches of a run: the groups at the batch depth, then
// those at depth 1 (steps mod depth), then the copy items if the number of
// groups is odd (with the depth-1 launch, or alone after a blocked one).
// Each launch is one kernel node; each waits for the one before.
hipError_t add_persistent_nodes(const oocs_batch* b, int64_t steps, hipGraph_t g)
{
    const int nd = (int)b->doms.size();
    const int64_t full = steps / b->depth, rest = steps % b->depth;
    const bool odd = ((full + rest) & 1) != 0;
    const size_t lds = std::max(b->lds[0], b->lds[1]);
    struct L { int w; int64_t groups; int64_t parity0; bool copy; };
    std::vector<L> ls;
    const bool tb0 = b->depth > 1;
    if (full > 0) ls.push_back({0, full, 0, odd && rest == 0 && !tb0});
    if (rest > 0) ls.push_back({1, rest, full & 1, odd});
    if (odd && !(ls.back().copy)) ls.push_back({1, 0, 0, true});
    hipGraphNode_t prev = nullptr;
    for (const L& l : ls) {
        if ((int64_t)b->total_wg[l.w] * l.groups + (l.copy ? b->copy_items : 0) >= ((int64_t)1 << 31))
            return hipErrorInvalidValue;
        oocs::BatchPersistArgs a{};
        a.tab = b->d_table + (size_t)l.w * nd;
        a.copy_begin = b->d_copy_begin;
        a.sync = b->d_sync;
        a.nd = nd;
        a.groups = (int32_t)l.groups;
        a.parity0 = (int32_t)l.parity0;
        a.total = b->total_wg[l.w];
        a.items = b->total_items[l.w];
        a.copy_items = l.copy ? b->copy_items : 0;
        a.force_wait = b->force_wait ? 1 : 0;
        a.spin_limit = b->spin_limit;
        a.alpha = b->alpha;
        const bool tb = l.w == 0 && tb0 && !l.copy;
        hipGraphNode_t n;
        const hipError_t e = oocs::add_batch_persistent_node(a, tb, b->grid[tb ? 0 : 1], lds, g, prev ? &prev : nullptr,
                                                             prev ? 1 : 0, &n);
        if (e != hipSuccess) return e;
        prev = n;
    }
    return hipSuccess;
}

}  // namespace

int oocs_batch_set_persistent(oocs_batch* b, int on)
{
    if (!b) return fail(OOCS_E_ARG, "bad argument");
    if (b->persistent != (on != 0)) {
        for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
        b->graphs.clear();
    }
    b->persistent = on != 0;
    return OOCS_OK;
}

int oocs_batch_set_wait_limit(oocs_batch* b, int64_t polls, int never_satisfied)
{
    if (!b || polls < 0) return fail(OOCS_E_ARG, "bad argument");
    b->spin_limit = polls;
    b->force_wait = never_satisfied != 0;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    return OOCS_OK;
}

int oocs_batch_check(oocs_batch* b, void* stream)
{
    if (!b) return fail(OOCS_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    uint32_t status = 0;
    HIP_TRY(hipMemcpy(&status, b->d_sync + 2, sizeof status, hipMemcpyDeviceToHost));
    if (status == 0) return OOCS_OK;
    HIP_TRY(oocs::launch_zero_words(b->d_sync, oocs::kBatchSyncWords + (int64_t)b->doms.size(), s));
    HIP_TRY(hipStreamSynchronize(s));
    return fail(OOCS_E_TIMEOUT, "a persistent batch launch gave up waiting for a dependency; the domains' states "
                                "are undefined");
}

int oocs_batch_run(oocs_batch* b, int64_t steps, void* stream)
{
    if (!b || steps < 0) return fail(OOCS_E_ARG, "bad argument");
    if (steps == 0) return OOCS_OK;
    hipStream_t s = (hipStream_t)stream;
    auto it = b->graphs.find(steps);
    if (it == b->graphs.end() && b->persistent) {
        hipGraph_t g;
        HIP_TRY(hipGraphCreate(&g, 0));
        hipError_t e = add_persistent_nodes(b, steps, g);
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return oocs::hip_fail(e, "persistent batch graph");
        it = b->graphs.emplace(steps, exec).first;
    }
    if (it == b->graphs.end()) {
        hipGraph_t g;
        HIP_TRY(hipGraphCreate(&g, 0));
        hipGraphNode_t prev = nullptr;
        hipError_t e = hipSuccess;
        const int nd = (int)b->doms.size();
        const int64_t full = steps / b->depth, rest = steps % b->depth;
        int64_t launches = 0;
        for (int64_t t = 0; t < full + rest && e == hipSuccess; ++t, ++launches) {
            const int w = t < full ? 0 : 1;
            hipGraphNode_t n;
            e = oocs::add_batch_step_node(b->d_table + (size_t)w * nd, nd, b->total_wg[w], b->lds[w], (int)(t & 1),
                                          b->alpha, g, prev ? &prev : nullptr, prev ? 1 : 0, &n);
            prev = n;
        }
        if (e == hipSuccess && (launches & 1)) {  // the state is in the scratch buffers: copy it back
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
    const int64_t full = steps / b->depth, rest = steps % b->depth;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        const oocs_domain& d = b->doms[i];
        for (int64_t t = 0; t < full + rest; ++t) {
            const int cfg = b->table[t < full ? 0 : 1][i].cfg;
            const float* src = (t & 1) ? d.d_scratch : d.d_u;
            float* dst = (t & 1) ? d.d_u : d.d_scratch;
            HIP_TRY(oocs::launch_heat_dense(src, dst, (int)d.nx, (int)d.ny, (int)d.nz, b->alpha, cfg, s));
        }
        if ((full + rest) & 1)
            HIP_TRY(hipMemcpyAsync(d.d_u, d.d_scratch, (size_t)(d.nx * d.ny * d.nz * 4), hipMemcpyDeviceToDevice, s));
    }
    return OOCS_OK;
}

int oocs_batch_domain_tile(const oocs_batch* b, int domain, int* tx, int* ty, int* zc, int* k)
{
    if (!b || domain < 0 || domain >= (int)b->doms.size()) return fail(OOCS_E_ARG, "bad argument");
    const oocs::TileCfg& t = oocs::kTileCfgs[b->table[0][domain].cfg];
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (zc) *zc = t.zc;
    if (k) *k = t.k;
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
