// host.cpp -- C ABI of liboocs (include/oocs.h): argument checks, the codec
// and stencil entry points, and the executor of the out-of-core schedule.
//
// The executor walks the planner's operation list once per residency and
// issues it on three HIP streams (Sec. V-B: three streams overlap the
// host-to-device copies, the GPU work and the device-to-host copies):
// copies with hipMemcpyAsync, the compute jobs of a tick as one fused
// launch, and the ordering edges as event records and waits. It makes no
// device allocation and no synchronisation until the last residency has
// been issued.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "oocs.h"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(OOCS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #call);    \
    } while (0)

bool dims_ok4(int64_t nx, int64_t ny, int64_t nz) { return nx > 0 && ny > 0 && nz > 0 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0; }

}  // namespace

struct oocs_plan {
    oocs::Planner P;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool runnable = false;
    hipStream_t st[3] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> ev;  // 4*nstage logical + 2*n block events (two parities)
    bool profiling = false;
    std::vector<hipEvent_t> tev;  // timing events, two per launch, grown on demand
};

extern "C" {

int oocs_version(void) { return 1; }

const char* oocs_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Codec
// ---------------------------------------------------------------------------

size_t oocs_codec_bytes(int64_t nx, int64_t ny, int64_t nz, int rate)
{
    if (!dims_ok4(nx, ny, nz) || rate < 1 || rate > OOCS_MAX_RATE) return 0;
    return (size_t)(nx / 4) * (size_t)(ny / 4) * (size_t)(nz / 4) * (size_t)rate * 8u;
}

static int codec_check(int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate, size_t bytes)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(OOCS_E_ARG, "dimensions must be positive");
    if (!dims_ok4(nx, ny, nz)) return fail(OOCS_E_ALIGN, "codec dimensions must be multiples of 4");
    if (rate < 1 || rate > OOCS_MAX_RATE) return fail(OOCS_E_RATE, "rate must be in [1, 34]");
    if (ld_y < nx || ld_z < ld_y * ny) return fail(OOCS_E_ARG, "leading dimensions too small");
    if (ld_y % 4 || ld_z % 4) return fail(OOCS_E_ALIGN, "leading dimensions must be multiples of 4");
    if (bytes < oocs_codec_bytes(nx, ny, nz, rate)) return fail(OOCS_E_SIZE, "compressed buffer too small");
    if (nx / 4 > (1 << 30) || (nx / 4) * (ny / 4) * (nz / 4) > ((int64_t)1 << 40)) return fail(OOCS_E_ARG, "field too large");
    return OOCS_OK;
}

int oocs_codec_encode(const float* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                      uint64_t* d_out, size_t out_bytes, void* stream)
{
    if (!d_in || !d_out) return fail(OOCS_E_ARG, "null pointer");
    if ((uintptr_t)d_in % 16 || (uintptr_t)d_out % 8) return fail(OOCS_E_ALIGN, "field must be 16-byte aligned, words 8-byte aligned");
    int rc = codec_check(nx, ny, nz, ld_y, ld_z, rate, out_bytes);
    if (rc) return rc;
    HIP_TRY(oocs::launch_codec_field(true, d_in, nullptr, nullptr, d_out, nx, ny, nz, ld_y, ld_z, rate,
                                     (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec_decode(const uint64_t* d_in, size_t in_bytes, int64_t nx, int64_t ny, int64_t nz, int rate, float* d_out,
                      int64_t ld_y, int64_t ld_z, void* stream)
{
    if (!d_in || !d_out) return fail(OOCS_E_ARG, "null pointer");
    if ((uintptr_t)d_out % 16 || (uintptr_t)d_in % 8) return fail(OOCS_E_ALIGN, "field must be 16-byte aligned, words 8-byte aligned");
    int rc = codec_check(nx, ny, nz, ld_y, ld_z, rate, in_bytes);
    if (rc) return rc;
    HIP_TRY(oocs::launch_codec_field(false, nullptr, d_out, d_in, nullptr, nx, ny, nz, ld_y, ld_z, rate,
                                     (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec_encode_stages(const float* d_blocks, int64_t nblocks, int rate, int32_t* d_emax, int32_t* d_q,
                             int32_t* d_t, uint32_t* d_u, uint64_t* d_planes, uint64_t* d_words, int32_t* d_bits,
                             void* stream)
{
    if (!d_blocks || nblocks < 0) return fail(OOCS_E_ARG, "bad block input");
    if (rate < 1 || rate > OOCS_MAX_RATE) return fail(OOCS_E_RATE, "rate must be in [1, 34]");
    oocs::EncStages s{d_emax, d_q, d_t, d_u, d_planes, d_words, d_bits};
    HIP_TRY(oocs::launch_encode_stages(d_blocks, nblocks, rate, s, (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec_decode_stages(const uint64_t* d_words, int64_t nblocks, int rate, int32_t* d_emax, uint64_t* d_planes,
                             uint32_t* d_u, int32_t* d_q, float* d_out, void* stream)
{
    if (!d_words || nblocks < 0) return fail(OOCS_E_ARG, "bad block input");
    if (rate < 1 || rate > OOCS_MAX_RATE) return fail(OOCS_E_RATE, "rate must be in [1, 34]");
    oocs::DecStages s{d_emax, d_planes, d_u, d_q, d_out};
    HIP_TRY(oocs::launch_decode_stages(d_words, nblocks, rate, s, (hipStream_t)stream));
    return OOCS_OK;
}

// ---------------------------------------------------------------------------
// In-core stencil steps (same level kernels as the pipeline, whole field as
// one ring with no wrap-around)
// ---------------------------------------------------------------------------

static oocs::LaunchParams base_params(int64_t nx, int64_t ny, int64_t nz, float alpha, int64_t sx, int64_t sy, int64_t sz)
{
    oocs::LaunchParams p;
    std::memset(&p, 0, sizeof p);
    p.nx = (int32_t)nx; p.ny = (int32_t)ny; p.nz = (int32_t)nz;
    p.alpha = alpha;
    const bool src = sx >= 0 && sy >= 0 && sz >= 0 && sx < nx && sy < ny && sz < nz;
    p.src_x = src ? (int32_t)sx : -1; p.src_y = src ? (int32_t)sy : -1; p.src_z = src ? (int32_t)sz : -1;
    return p;
}

static bool grid_ok(int64_t nx, int64_t ny, int64_t nz)
{
    return nx > 0 && ny > 0 && nz > 0 && nx % 4 == 0 && nx <= (1 << 20) && ny <= (1 << 20) && nz <= (1 << 20) &&
           nx * ny <= ((int64_t)1 << 31);
}

int oocs_heat7_step_k(float* d_u, float* d_tmp, int64_t nx, int64_t ny, int64_t nz, float alpha, int64_t k, void* stream)
{
    if (!d_u || !d_tmp || k < 0) return fail(OOCS_E_ARG, "bad argument");
    if (!grid_ok(nx, ny, nz)) return fail(OOCS_E_ARG, "bad grid (nx must be a multiple of 4)");
    hipStream_t s = (hipStream_t)stream;
    float* a = d_u;
    float* b = d_tmp;
    for (int64_t t = 0; t < k; ++t) {
        oocs::LaunchParams p = base_params(nx, ny, nz, alpha, -1, -1, -1);
        oocs::Job& j = p.jobs[0];
        j.kind = oocs::JOB_HEAT;
        j.z0 = 0; j.z1 = (int32_t)nz;
        j.src = {a, nz, nx * ny};
        j.dst = {b, nz, nx * ny};
        p.njobs = 1;
        HIP_TRY(oocs::launch_jobs(p, s));
        std::swap(a, b);
    }
    if (a != d_u) HIP_TRY(hipMemcpyAsync(d_u, a, (size_t)(nx * ny * nz) * 4, hipMemcpyDeviceToDevice, s));
    return OOCS_OK;
}

int oocs_wave25_step_k(float* d_p, float* d_pm, const float* d_w, int64_t nx, int64_t ny, int64_t nz, int64_t k,
                       const float* h_src, int64_t src_x, int64_t src_y, int64_t src_z, void* stream)
{
    if (!d_p || !d_pm || !d_w || k < 0) return fail(OOCS_E_ARG, "bad argument");
    if (!grid_ok(nx, ny, nz)) return fail(OOCS_E_ARG, "bad grid (nx must be a multiple of 4)");
    hipStream_t s = (hipStream_t)stream;
    float* p = d_p;
    float* pm = d_pm;
    for (int64_t t = 0; t < k; ++t) {
        oocs::LaunchParams lp = base_params(nx, ny, nz, 0.0f, src_x, src_y, src_z);
        oocs::Job& j = lp.jobs[0];
        j.kind = oocs::JOB_WAVE;
        j.z0 = 0; j.z1 = (int32_t)nz;
        j.src = {p, nz, nx * ny};
        j.src2 = {pm, nz, nx * ny};
        j.ro = {const_cast<float*>(d_w), nz, nx * ny};
        j.dst = {pm, nz, nx * ny};  // p(n+1) overwrites p(n-1) in place
        j.has_src = h_src != nullptr && lp.src_x >= 0;
        j.amp = h_src ? h_src[t] : 0.0f;
        lp.njobs = 1;
        HIP_TRY(oocs::launch_jobs(lp, s));
        std::swap(p, pm);
    }
    if (p != d_p) HIP_TRY(oocs::launch_swap(d_p, d_pm, nx * ny * nz, s));
    return OOCS_OK;
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------

int oocs_plan_create(const oocs_config* cfg, void* d_arena, size_t arena_bytes, oocs_plan** out)
{
    if (!cfg || !out) return fail(OOCS_E_ARG, "null pointer");
    *out = nullptr;
    oocs_plan* pl = new (std::nothrow) oocs_plan();
    if (!pl) return fail(OOCS_E_ARG, "out of host memory");
    std::string err;
    int rc = pl->P.init(*cfg, err);
    if (rc == OOCS_OK) rc = pl->P.choose(arena_bytes, err);
    if (rc != OOCS_OK) {
        delete pl;
        return fail(rc, err);
    }
    pl->arena = static_cast<char*>(d_arena);
    pl->arena_bytes = arena_bytes;
    if (d_arena) {
        for (int i = 0; i < 3; ++i) {
            hipError_t e = hipStreamCreateWithFlags(&pl->st[i], hipStreamNonBlocking);
            if (e != hipSuccess) { oocs_plan_destroy(pl); return hip_fail(e, "hipStreamCreateWithFlags"); }
        }
        const int nev = 4 * pl->P.nstage + 2 * pl->P.n;
        pl->ev.assign(nev, nullptr);
        for (int i = 0; i < nev; ++i) {
            hipError_t e = hipEventCreateWithFlags(&pl->ev[i], hipEventDisableTiming);
            if (e != hipSuccess) { oocs_plan_destroy(pl); return hip_fail(e, "hipEventCreateWithFlags"); }
        }
        pl->runnable = true;
    }
    *out = pl;
    return OOCS_OK;
}

int oocs_plan_destroy(oocs_plan* pl)
{
    if (!pl) return OOCS_OK;
    if (pl->runnable) {
        for (hipStream_t s : pl->st)
            if (s) (void)hipStreamSynchronize(s);
    }
    for (hipEvent_t e : pl->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->tev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : pl->st)
        if (s) (void)hipStreamDestroy(s);
    delete pl;
    return OOCS_OK;
}

int oocs_plan_get_info(const oocs_plan* pl, oocs_plan_info* out)
{
    if (!pl || !out) return fail(OOCS_E_ARG, "null pointer");
    std::memset(out, 0, sizeof *out);
    const oocs::Planner& P = pl->P;
    out->group = P.G;
    out->halo = P.h;
    out->radius = P.r;
    out->nlevels = P.nin + P.k;
    out->nrings = P.nrings();
    for (int i = 0; i < P.nrings() && i < 16; ++i) out->ring_planes[i] = P.ringW[i];
    out->plane_bytes = P.plane_elems() * 4;
    out->arena_needed = P.arena_needed;
    out->nstage = P.nstage;
    for (int f = 0; f < OOCS_MAX_FIELDS; ++f) out->store_bytes[f] = P.store_bytes(f);
    return OOCS_OK;
}

int oocs_plan_slab(const oocs_plan* pl, int i, oocs_slab_info* out)
{
    if (!pl || !out) return fail(OOCS_E_ARG, "null pointer");
    const oocs::Planner& P = pl->P;
    if (i < 0 || i >= P.n) return fail(OOCS_E_ARG, "slab index out of range");
    std::memset(out, 0, sizeof *out);
    out->z0 = P.a[i];
    out->z1 = P.a[i + 1];
    out->r0 = i == 0 ? 0 : P.a[i] + P.h;
    out->r1 = i == P.n - 1 ? P.nz : P.a[i + 1] - P.h;
    out->c0 = i == P.n - 1 ? P.nz : P.a[i + 1] - P.h;
    out->c1 = i == P.n - 1 ? P.nz : P.a[i + 1] + P.h;
    for (int f = 0; f < P.nfields; ++f) {
        const int64_t spb = P.store_plane_bytes(f);
        out->r_off[f] = out->r0 * spb;
        out->r_bytes[f] = (out->r1 - out->r0) * spb;
        out->c_off[f] = out->c0 * spb;
        out->c_bytes[f] = (out->c1 - out->c0) * spb;
    }
    return OOCS_OK;
}

int64_t oocs_plan_schedule_len(oocs_plan* pl, int kr)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    std::string err;
    const oocs::Schedule* s = pl->P.schedule(kr, err);
    if (!s) return fail(OOCS_E_ARG, err);
    return (int64_t)s->ops.size();
}

int oocs_plan_schedule_op(oocs_plan* pl, int kr, int64_t index, oocs_op* out)
{
    if (!pl || !out) return fail(OOCS_E_ARG, "null pointer");
    std::string err;
    const oocs::Schedule* s = pl->P.schedule(kr, err);
    if (!s) return fail(OOCS_E_ARG, err);
    if (index < 0 || index >= (int64_t)s->ops.size()) return fail(OOCS_E_ARG, "op index out of range");
    *out = s->ops[index];
    return OOCS_OK;
}

size_t oocs_store_bytes(const oocs_plan* pl, int field)
{
    if (!pl) return 0;
    return (size_t)pl->P.store_bytes(field);
}

// Initial compression of a field into its host store, and decompression of
// a host store, streamed through the arena in chunks of 4-plane layers.
static int store_xfer(oocs_plan* pl, int f, bool put, const float* h_field_in, float* h_field_out, const void* h_store_in,
                      void* h_store_out)
{
    const oocs::Planner& P = pl->P;
    const int64_t pb = P.plane_elems() * 4;
    const int rate = P.cfg.rate[f];
    const int64_t spb = P.store_plane_bytes(f);
    hipStream_t s = pl->st[1];
    int64_t chunk = (int64_t)(pl->arena_bytes / (size_t)(pb + spb)) / 4 * 4;
    if (chunk > P.nz) chunk = P.nz;
    if (chunk < 4) return fail(OOCS_E_CAP, "arena too small to stream the store");
    char* raw = pl->arena;
    uint64_t* comp = reinterpret_cast<uint64_t*>(pl->arena + ((chunk * pb + 255) / 256) * 256);
    for (int64_t z0 = 0; z0 < P.nz; z0 += chunk) {
        const int64_t z1 = std::min(P.nz, z0 + chunk);
        const int64_t planes = z1 - z0;
        if (put) {
            HIP_TRY(hipMemcpyAsync(raw, h_field_in + z0 * P.plane_elems(), (size_t)(planes * pb), hipMemcpyHostToDevice, s));
            HIP_TRY(oocs::launch_codec_field(true, reinterpret_cast<float*>(raw), nullptr, nullptr, comp, P.nx, P.ny, planes,
                                             P.nx, P.plane_elems(), rate, s));
            HIP_TRY(hipMemcpyAsync(static_cast<char*>(h_store_out) + z0 * spb, comp, (size_t)(planes * spb),
                                   hipMemcpyDeviceToHost, s));
        } else {
            HIP_TRY(hipMemcpyAsync(comp, static_cast<const char*>(h_store_in) + z0 * spb, (size_t)(planes * spb),
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(oocs::launch_codec_field(false, nullptr, reinterpret_cast<float*>(raw), comp, nullptr, P.nx, P.ny, planes,
                                             P.nx, P.plane_elems(), rate, s));
            HIP_TRY(hipMemcpyAsync(h_field_out + z0 * P.plane_elems(), raw, (size_t)(planes * pb), hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }
    return OOCS_OK;
}

int oocs_store_put(oocs_plan* pl, int f, const float* h_field, void* h_store)
{
    if (!pl || !h_field || !h_store) return fail(OOCS_E_ARG, "null pointer");
    if (f < 0 || f >= pl->P.nfields) return fail(OOCS_E_ARG, "field slot out of range");
    if (pl->P.cfg.rate[f] == 0) {
        std::memcpy(h_store, h_field, (size_t)pl->P.store_bytes(f));
        return OOCS_OK;
    }
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan cannot compress");
    return store_xfer(pl, f, true, h_field, nullptr, nullptr, h_store);
}

int oocs_store_get(oocs_plan* pl, int f, const void* h_store, float* h_field)
{
    if (!pl || !h_field || !h_store) return fail(OOCS_E_ARG, "null pointer");
    if (f < 0 || f >= pl->P.nfields) return fail(OOCS_E_ARG, "field slot out of range");
    if (pl->P.cfg.rate[f] == 0) {
        std::memcpy(h_field, h_store, (size_t)pl->P.store_bytes(f));
        return OOCS_OK;
    }
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan cannot decompress");
    return store_xfer(pl, f, false, nullptr, h_field, h_store, nullptr);
}

// ---------------------------------------------------------------------------
// Executor
// ---------------------------------------------------------------------------

int oocs_plan_set_profiling(oocs_plan* pl, int on)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan");
    pl->profiling = on != 0;
    return OOCS_OK;
}

// Algorithmic device-memory bytes of one job (each distinct input plane read
// once, each output plane written once).
static int64_t job_bytes(const oocs::Job& j, int64_t plane_elems)
{
    const int64_t planes = j.z1 - j.z0;
    const int64_t pb = plane_elems * 4;
    switch (j.kind) {
    case oocs::JOB_HEAT: return planes * pb * 2;        // read u, write u'
    case oocs::JOB_WAVE: return planes * pb * 4;        // read p, p(n-1), w; write p(n+1)
    case oocs::JOB_DECODE:
    case oocs::JOB_ENCODE: return planes * (pb + plane_elems * j.rate / 8);
    default: return planes * pb * 2;                    // raw copies
    }
}

int oocs_run(oocs_plan* pl, void* const* h_store, int64_t steps, const float* h_src, oocs_stats* st)
{
    if (!pl || !h_store || steps < 0) return fail(OOCS_E_ARG, "bad argument");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan cannot run");
    oocs::Planner& P = pl->P;
    for (int f : P.in_fields)
        if (!h_store[f]) return fail(OOCS_E_ARG, "missing host store pointer");
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t pe = P.plane_elems();
    auto ring = [&](int idx) {
        return oocs::Ring{reinterpret_cast<float*>(pl->arena + P.ringOff[idx]), P.ringW[idx], pe};
    };
    int64_t h2d = 0, d2h = 0, rounds = 0, launches = 0;
    int64_t kbytes[2] = {0, 0};  // codec jobs, stencil jobs
    size_t tused = 0;
    const int ns = P.nstage;
    int64_t done = 0;
    while (done < steps) {
        const int kr = (int)std::min<int64_t>(P.k, steps - done);
        std::string err;
        const oocs::Schedule* sch = P.schedule(kr, err);
        if (!sch) return fail(OOCS_E_STATE, err);
        const int parity = (int)(rounds & 1);
        auto phys = [&](int e) -> hipEvent_t {
            if (e < 4 * ns) return pl->ev[e];
            int i = e - 4 * ns;
            const bool prev = i >= P.n;
            if (prev) i -= P.n;
            const int par = prev ? 1 - parity : parity;
            return pl->ev[4 * ns + par * P.n + i];
        };
        oocs::LaunchParams lp = base_params(P.nx, P.ny, P.nz, P.cfg.alpha, P.cfg.src_x, P.cfg.src_y, P.cfg.src_z);
        for (const oocs_op& o : sch->ops) {
            switch (o.kind) {
            case OOCS_OP_H2D: {
                const int64_t spb = P.store_plane_bytes(o.field);
                const size_t bytes = (size_t)((o.z1 - o.z0) * spb);
                char* dst = pl->arena + P.in_off[o.field] + (int64_t)o.slot * P.in_slot_bytes[o.field];
                const char* src = static_cast<const char*>(h_store[o.field]) + o.z0 * spb;
                HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, pl->st[0]));
                h2d += (int64_t)bytes;
                break;
            }
            case OOCS_OP_D2H: {
                const int64_t spb = P.store_plane_bytes(o.field);
                const size_t bytes = (size_t)((o.z1 - o.z0) * spb);
                const char* src = pl->arena + P.out_off[o.field] + (int64_t)o.slot * P.out_slot_bytes[o.field];
                char* dst = static_cast<char*>(h_store[o.field]) + o.z0 * spb;
                HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, pl->st[2]));
                d2h += (int64_t)bytes;
                break;
            }
            case OOCS_OP_DECODE:
            case OOCS_OP_ENCODE: {
                const int rate = P.cfg.rate[o.field];
                if (lp.njobs >= oocs::kMaxJobs) return fail(OOCS_E_STATE, "too many jobs in a tick");
                oocs::Job& j = lp.jobs[lp.njobs++];
                std::memset(&j, 0, sizeof j);
                const bool dec = o.kind == OOCS_OP_DECODE;
                j.kind = rate ? (dec ? oocs::JOB_DECODE : oocs::JOB_ENCODE) : (dec ? oocs::JOB_COPY_IN : oocs::JOB_COPY_OUT);
                j.z0 = (int32_t)o.z0; j.z1 = (int32_t)o.z1;
                j.rate = rate;
                j.dst = ring(o.level);
                j.stage = dec ? (void*)(pl->arena + P.in_off[o.field] + (int64_t)o.slot * P.in_slot_bytes[o.field])
                              : (void*)(pl->arena + P.out_off[o.field] + (int64_t)o.slot * P.out_slot_bytes[o.field]);
                break;
            }
            case OOCS_OP_LEVEL: {
                if (lp.njobs >= oocs::kMaxJobs) return fail(OOCS_E_STATE, "too many jobs in a tick");
                oocs::Job& j = lp.jobs[lp.njobs++];
                std::memset(&j, 0, sizeof j);
                j.z0 = (int32_t)o.z0; j.z1 = (int32_t)o.z1;
                j.src = ring(o.level - 1);
                j.dst = ring(o.level);
                if (P.cfg.stencil == OOCS_HEAT7) {
                    j.kind = oocs::JOB_HEAT;
                } else {
                    j.kind = oocs::JOB_WAVE;
                    j.src2 = ring(o.level - 2);
                    j.ro = ring(P.ro_ring());
                    const int64_t step = done + (o.level - P.nin);  // index of this step within the call
                    j.has_src = h_src != nullptr && lp.src_x >= 0 && lp.src_z >= o.z0 && lp.src_z < o.z1;
                    j.amp = h_src ? h_src[step] : 0.0f;
                }
                break;
            }
            case OOCS_OP_LAUNCH:
                if (lp.njobs > 0) {
                    for (int i = 0; i < lp.njobs; ++i)
                        kbytes[oocs::is_codec_job(lp.jobs[i].kind) ? 0 : 1] += job_bytes(lp.jobs[i], pe);
                    if (pl->profiling) {
                        while (pl->tev.size() < tused + 2) {
                            hipEvent_t e;
                            HIP_TRY(hipEventCreate(&e));
                            pl->tev.push_back(e);
                        }
                        HIP_TRY(hipEventRecord(pl->tev[tused], pl->st[1]));
                    }
                    HIP_TRY(oocs::launch_jobs(lp, pl->st[1]));
                    if (pl->profiling) {
                        HIP_TRY(hipEventRecord(pl->tev[tused + 1], pl->st[1]));
                        tused += 2;
                    }
                    ++launches;
                }
                lp.njobs = 0;
                break;
            case OOCS_OP_RECORD:
                HIP_TRY(hipEventRecord(phys(o.event), pl->st[o.stream]));
                break;
            case OOCS_OP_WAIT:
                if (o.event >= P.ev_blk_prev(0) && rounds == 0) break;  // nothing written back yet in this call
                HIP_TRY(hipStreamWaitEvent(pl->st[o.stream], phys(o.event), 0));
                break;
            default:
                return fail(OOCS_E_STATE, "unknown op");
            }
        }
        done += kr;
        ++rounds;
    }
    const double enq = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int i = 0; i < 3; ++i) HIP_TRY(hipStreamSynchronize(pl->st[i]));
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    double kms = 0.0;
    for (size_t i = 0; i + 1 < tused; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pl->tev[i], pl->tev[i + 1]));
        kms += ms;
    }
    if (st) {
        st->wall_ms = wall;
        st->enqueue_ms = enq;
        st->rounds = rounds;
        st->h2d_bytes = h2d;
        st->d2h_bytes = d2h;
        st->cell_updates = P.nx * P.ny * P.nz * steps;
        st->launches = launches;
        st->codec_bytes = kbytes[0];
        st->stencil_bytes = kbytes[1];
        st->kernel_ms = kms;
    }
    return OOCS_OK;
}

}  // extern "C"
