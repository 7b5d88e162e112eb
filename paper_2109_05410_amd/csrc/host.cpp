// host.cpp -- C ABI of liboocs (include/oocs.h): argument checks, the codec
// and stencil entry points, and the executor of the out-of-core schedule.
//
// The executor walks the planner's operation list once per residency and
// issues it on three HIP streams (Sec. V-B: three streams overlap the
// host-to-device copies, the GPU work and the device-to-host copies):
// host-to-device copies with hipMemcpyAsync, device-to-host copies on an
// SDMA engine through the HSA runtime (sdma.cpp; hipMemcpyAsync where that
// is unavailable or switched off), the compute jobs of a tick as one fused
// launch, and the ordering edges as event records and waits, honoured on
// the host by default. It makes no device allocation and no synchronisation
// until the last residency has been issued.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "oocs.h"
#include "plan.hpp"
#include "sdma.hpp"

#include "abi_util.hpp"

namespace oocs {
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
}  // namespace oocs

namespace {
using oocs::fail;
using oocs::hip_fail;

bool dims_ok4(int64_t nx, int64_t ny, int64_t nz) { return nx > 0 && ny > 0 && nz > 0 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0; }

}  // namespace

// One residency's operation list built as a HIP graph (replayed once per
// residency; graph launches on one stream run one after another, so the
// waits that order a residency after the previous one are not needed inside).
struct ResidencyGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> timing;  // start/end pairs around each kernel node (profiling)
    int64_t launches = 0, codec_bytes = 0, stencil_bytes = 0, xfer_bytes = 0, h2d = 0, d2h = 0;
    int64_t timed_bytes = 0;  // algorithmic bytes of the launches that have timing nodes
};

struct oocs_plan {
    oocs::Planner P;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool runnable = false;
    hipStream_t st[3] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> ev;  // 4*nstage logical + 2*n block events (two parities)
    int profiling = 0;  // 0: off; N: time every N-th launch
    bool host_waits = true;  // eager issue: wait on the host for pending cross-stream events
    bool graphs = false;
    // device-to-host copies on SDMA engines (op-by-op issue with host waits)
    oocs::SdmaCopier sdma;
    bool sdma_on = true;
    std::vector<int64_t> ev_ticket;  // per event: SDMA ticket if last recorded on the D2H stream, else -1
    std::vector<hipEvent_t> tev;  // eager timing events, two per launch, grown on demand
    // per-stage breakdown (op-by-op issue): event pairs around every copy and
    // every stage launch, grown on demand
    bool breakdown = false;
    std::vector<hipEvent_t> bev;
    // resident read-only field: the store its ring was decoded from (null:
    // not loaded, or overwritten by store I/O through the arena)
    const void* ro_loaded = nullptr;
    // graphs by (residency length, store pointers, source on)
    std::map<std::tuple<int, const void*, const void*, const void*, bool, bool>, ResidencyGraph> gcache;
};

extern "C" {

int oocs_version(void) { return 1; }

const char* oocs_last_error(void) { return oocs::g_err.c_str(); }

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
    const bool mid = (rate & OOCS_DECODE_MIDPOINT) != 0;
    rate &= ~OOCS_DECODE_MIDPOINT;
    int rc = codec_check(nx, ny, nz, ld_y, ld_z, rate, in_bytes);
    if (rc) return rc;
    HIP_TRY(oocs::launch_codec_field(false, nullptr, d_out, d_in, nullptr, nx, ny, nz, ld_y, ld_z, rate,
                                     (hipStream_t)stream, mid));
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
    const bool mid = (rate & OOCS_DECODE_MIDPOINT) != 0;
    rate &= ~OOCS_DECODE_MIDPOINT;
    if (rate < 1 || rate > OOCS_MAX_RATE) return fail(OOCS_E_RATE, "rate must be in [1, 34]");
    oocs::DecStages s{d_emax, d_planes, d_u, d_q, d_out};
    HIP_TRY(oocs::launch_decode_stages(d_words, nblocks, rate, mid, s, (hipStream_t)stream));
    return OOCS_OK;
}

// ---------------------------------------------------------------------------
// FP64 format and FP64 wave step (codec64.hip)
// ---------------------------------------------------------------------------

size_t oocs_codec64_bytes(int64_t nx, int64_t ny, int64_t nz, int rate)
{
    if (!dims_ok4(nx, ny, nz) || rate < 1 || rate > OOCS_MAX_RATE64) return 0;
    return (size_t)(nx / 4) * (size_t)(ny / 4) * (size_t)(nz / 4) * (size_t)rate * 8u;
}

static int codec64_check(int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate, size_t bytes)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(OOCS_E_ARG, "dimensions must be positive");
    if (!dims_ok4(nx, ny, nz)) return fail(OOCS_E_ALIGN, "codec dimensions must be multiples of 4");
    if (rate < 1 || rate > OOCS_MAX_RATE64) return fail(OOCS_E_RATE, "FP64 rate must be in [1, 68]");
    if (ld_y < nx || ld_z < ld_y * ny) return fail(OOCS_E_ARG, "leading dimensions too small");
    if (bytes < oocs_codec64_bytes(nx, ny, nz, rate)) return fail(OOCS_E_SIZE, "compressed buffer too small");
    if (nx / 4 > (1 << 30) || ny / 4 > (1 << 30)) return fail(OOCS_E_ARG, "field too large");
    return OOCS_OK;
}

int oocs_codec64_encode(const double* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                        uint64_t* d_out, size_t out_bytes, void* stream)
{
    if (!d_in || !d_out) return fail(OOCS_E_ARG, "null pointer");
    if ((uintptr_t)d_in % 8 || (uintptr_t)d_out % 8) return fail(OOCS_E_ALIGN, "buffers must be 8-byte aligned");
    const int rc = codec64_check(nx, ny, nz, ld_y, ld_z, rate, out_bytes);
    if (rc) return rc;
    HIP_TRY(oocs::launch_codec64_field(true, d_in, nullptr, nullptr, d_out, nx, ny, nz, ld_y, ld_z, rate,
                                       (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec64_decode(const uint64_t* d_in, size_t in_bytes, int64_t nx, int64_t ny, int64_t nz, int rate,
                        double* d_out, int64_t ld_y, int64_t ld_z, void* stream)
{
    if (!d_in || !d_out) return fail(OOCS_E_ARG, "null pointer");
    if ((uintptr_t)d_in % 8 || (uintptr_t)d_out % 8) return fail(OOCS_E_ALIGN, "buffers must be 8-byte aligned");
    const int rc = codec64_check(nx, ny, nz, ld_y, ld_z, rate, in_bytes);
    if (rc) return rc;
    HIP_TRY(oocs::launch_codec64_field(false, nullptr, d_out, d_in, nullptr, nx, ny, nz, ld_y, ld_z, rate,
                                       (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec64_encode_stages(const double* d_blocks, int64_t nblocks, int rate, int32_t* d_emax, int64_t* d_q,
                               int64_t* d_t, uint64_t* d_u, uint64_t* d_planes, uint64_t* d_words, int32_t* d_bits,
                               void* stream)
{
    if (!d_blocks || !d_words || nblocks < 0) return fail(OOCS_E_ARG, "bad block input");
    if (rate < 1 || rate > OOCS_MAX_RATE64) return fail(OOCS_E_RATE, "FP64 rate must be in [1, 68]");
    HIP_TRY(oocs::launch_codec64_stages(true, d_blocks, nullptr, nblocks, rate, d_emax, d_q, d_t, d_u, d_planes,
                                        d_words, d_bits, nullptr, (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_codec64_decode_stages(const uint64_t* d_words, int64_t nblocks, int rate, int32_t* d_emax, uint64_t* d_planes,
                               uint64_t* d_u, int64_t* d_q, double* d_out, void* stream)
{
    if (!d_words || nblocks < 0) return fail(OOCS_E_ARG, "bad block input");
    if (rate < 1 || rate > OOCS_MAX_RATE64) return fail(OOCS_E_RATE, "FP64 rate must be in [1, 68]");
    HIP_TRY(oocs::launch_codec64_stages(false, nullptr, d_words, nblocks, rate, d_emax, d_q, nullptr, d_u, d_planes,
                                        nullptr, nullptr, d_out, (hipStream_t)stream));
    return OOCS_OK;
}

int oocs_wave25_step_k_f64(double* d_p, double* d_pm, const double* d_w, int64_t nx, int64_t ny, int64_t nz,
                           int64_t k, const double* h_src, int64_t src_x, int64_t src_y, int64_t src_z, void* stream)
{
    if (!d_p || !d_pm || !d_w || k < 0 || nx <= 0 || ny <= 0 || nz <= 0) return fail(OOCS_E_ARG, "bad argument");
    if (nx * ny * nz >= ((int64_t)1 << 40) || nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20))
        return fail(OOCS_E_ARG, "grid too large");
    if (nx * ny * 8 >= ((int64_t)1 << 32)) return fail(OOCS_E_ARG, "a plane of the wave must hold less than 4 GiB");
    const bool src_on = h_src && src_x >= 0 && src_x < nx && src_y >= 0 && src_y < ny && src_z >= 0 && src_z < nz;
    const int64_t cell = src_on ? src_x + nx * (src_y + ny * src_z) : -1;
    hipStream_t s = (hipStream_t)stream;
    double* p = d_p;
    double* pm = d_pm;
    for (int64_t t = 0; t < k; ++t) {
        HIP_TRY(oocs::launch_wave_f64(p, pm, d_w, nx, ny, nz, cell, src_on ? h_src[t] : 0.0, s));
        std::swap(p, pm);  // pm now holds p(n+1)
    }
    if (p != d_p)  // an odd number of steps: exchange the two arrays' contents (bitwise, as float pairs)
        HIP_TRY(oocs::launch_swap(reinterpret_cast<float*>(d_p), reinterpret_cast<float*>(d_pm), 2 * nx * ny * nz, s));
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
    if (((uintptr_t)d_u | (uintptr_t)d_tmp) % 16) return fail(OOCS_E_ALIGN, "fields must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    float* a = d_u;
    float* b = d_tmp;
    // Four steps per launch with the temporally blocked tiles (each cell and
    // step takes the same FP32 operations as a single level, so the bits are
    // the same) when the field gives at least 4 workgroups per compute unit
    // (a blocked workgroup marches its z chunk serially, so on small fields
    // the one-level launches are quicker), the launch's work-items fit the
    // dispatch's 32-bit grid and the cell count the tiles' 32-bit indexes;
    // the remaining k mod 4 steps, and every step otherwise, one level per
    // launch.
    int tb = -1;
    for (int c = 0; c < oocs::kNumTileCfgs; ++c)
        if (oocs::kTileCfgs[c].k == 4 && oocs::kTileCfgs[c].ty == 16 && oocs::kTileCfgs[c].zc == 64) tb = c;
    int64_t t = 0;
    if (tb >= 0 && k >= 4) {
        const oocs::TileCfg& c = oocs::kTileCfgs[tb];
        const int64_t ox = c.tx - 2 * c.k, oy = c.ty - 2 * c.k;
        const int64_t wgs = ((nx + ox - 1) / ox) * ((ny + oy - 1) / oy) * ((nz + c.zc - 1) / c.zc);
        if (wgs >= 4 * 256 && wgs * oocs::kBlockThreads < ((int64_t)1 << 32) && nx * ny * nz < ((int64_t)1 << 31))
            for (; t + 4 <= k; t += 4) {
                HIP_TRY(oocs::launch_heat_dense(a, b, (int)nx, (int)ny, (int)nz, alpha, tb, s));
                std::swap(a, b);
            }
    }
    // Small fields (up to 2^21 cells) one level per launch in short z chunks
    // (8 planes per workgroup): more workgroups, each with a shorter serial
    // march, than the level job's chunks.
    int small = -1;
    if (nx * ny * nz <= ((int64_t)1 << 21))
        for (int c = 0; c < oocs::kNumTileCfgs; ++c)
            if (oocs::kTileCfgs[c].k == 1 && oocs::kTileCfgs[c].tx == 64 && oocs::kTileCfgs[c].zc == 8) small = c;
    if (small >= 0)
        for (; t < k; ++t) {
            HIP_TRY(oocs::launch_heat_dense(a, b, (int)nx, (int)ny, (int)nz, alpha, small, s));
            std::swap(a, b);
        }
    for (; t < k; ++t) {
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
    if (nx * ny * 4 >= ((int64_t)1 << 32)) return fail(OOCS_E_ARG, "a plane of the wave must hold less than 4 GiB");
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
        pl->ev_ticket.assign(nev, -1);
        std::string why;
        (void)pl->sdma.init(d_arena, &why);  // unavailable: device-to-host copies stay on hipMemcpyAsync
        pl->runnable = true;
    }
    *out = pl;
    return OOCS_OK;
}

int oocs_plan_destroy(oocs_plan* pl)
{
    if (!pl) return OOCS_OK;
    if (pl->runnable) {
        (void)pl->sdma.drain();
        for (hipStream_t s : pl->st)
            if (s) (void)hipStreamSynchronize(s);
    }
    for (hipEvent_t e : pl->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->tev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->bev)
        if (e) (void)hipEventDestroy(e);
    for (auto& kv : pl->gcache) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        for (hipEvent_t e : kv.second.timing)
            if (e) (void)hipEventDestroy(e);
    }
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
    out->plane_bytes = P.plane_bytes();
    out->arena_needed = P.arena_needed;
    out->nstage = P.nstage;
    for (int f = 0; f < OOCS_MAX_FIELDS; ++f) out->store_bytes[f] = P.store_bytes(f);
    out->retained_planes = P.X;
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

int64_t oocs_plan_schedule_variant_len(oocs_plan* pl, int kr, int variant)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    std::string err;
    const oocs::Schedule* s = pl->P.schedule(kr, err, variant);
    if (!s) return fail(OOCS_E_ARG, err);
    return (int64_t)s->ops.size();
}

int oocs_plan_schedule_variant_op(oocs_plan* pl, int kr, int variant, int64_t index, oocs_op* out)
{
    if (!pl || !out) return fail(OOCS_E_ARG, "null pointer");
    std::string err;
    const oocs::Schedule* s = pl->P.schedule(kr, err, variant);
    if (!s) return fail(OOCS_E_ARG, err);
    if (index < 0 || index >= (int64_t)s->ops.size()) return fail(OOCS_E_ARG, "op index out of range");
    *out = s->ops[index];
    return OOCS_OK;
}

int64_t oocs_plan_schedule_len(oocs_plan* pl, int kr) { return oocs_plan_schedule_variant_len(pl, kr, 0); }

int oocs_plan_schedule_op(oocs_plan* pl, int kr, int64_t index, oocs_op* out)
{
    return oocs_plan_schedule_variant_op(pl, kr, 0, index, out);
}

size_t oocs_store_bytes(const oocs_plan* pl, int field)
{
    if (!pl) return 0;
    return (size_t)pl->P.store_bytes(field);
}

// Initial compression of a field into its host store, and decompression of
// a host store, streamed through the arena in chunks of 4-plane layers.
static int store_xfer(oocs_plan* pl, int f, bool put, const void* h_field_in, void* h_field_out, const void* h_store_in,
                      void* h_store_out)
{
    const oocs::Planner& P = pl->P;
    pl->ro_loaded = nullptr;  // the chunks below overwrite the start of the arena
    const int64_t pb = P.plane_bytes();
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
            HIP_TRY(hipMemcpyAsync(raw, static_cast<const char*>(h_field_in) + z0 * pb, (size_t)(planes * pb),
                                   hipMemcpyHostToDevice, s));
            if (P.fp64)
                HIP_TRY(oocs::launch_codec64_field(true, reinterpret_cast<double*>(raw), nullptr, nullptr, comp, P.nx,
                                                   P.ny, planes, P.nx, P.plane_elems(), rate, s));
            else
                HIP_TRY(oocs::launch_codec_field(true, reinterpret_cast<float*>(raw), nullptr, nullptr, comp, P.nx, P.ny,
                                                 planes, P.nx, P.plane_elems(), rate, s));
            HIP_TRY(hipMemcpyAsync(static_cast<char*>(h_store_out) + z0 * spb, comp, (size_t)(planes * spb),
                                   hipMemcpyDeviceToHost, s));
        } else {
            HIP_TRY(hipMemcpyAsync(comp, static_cast<const char*>(h_store_in) + z0 * spb, (size_t)(planes * spb),
                                   hipMemcpyHostToDevice, s));
            if (P.fp64)
                HIP_TRY(oocs::launch_codec64_field(false, nullptr, reinterpret_cast<double*>(raw), comp, nullptr, P.nx,
                                                   P.ny, planes, P.nx, P.plane_elems(), rate, s));
            else
                HIP_TRY(oocs::launch_codec_field(false, nullptr, reinterpret_cast<float*>(raw), comp, nullptr, P.nx,
                                                 P.ny, planes, P.nx, P.plane_elems(), rate, s, P.midpoint));
            HIP_TRY(hipMemcpyAsync(static_cast<char*>(h_field_out) + z0 * pb, raw, (size_t)(planes * pb),
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }
    return OOCS_OK;
}

int oocs_store_put(oocs_plan* pl, int f, const void* h_field, void* h_store)
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

int oocs_store_get(oocs_plan* pl, int f, const void* h_store, void* h_field)
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
    pl->profiling = on > 0 ? on : 0;
    return OOCS_OK;
}

// Stage of a job in the per-stage breakdown: 0 host-to-device transfer,
// 1 decode (or raw copy in), 2 stencil steps, 3 encode (or raw copy out),
// 4 device-to-host transfer.
static int job_stage(int kind)
{
    switch (kind) {
    case oocs::JOB_FETCH: return 0;
    case oocs::JOB_DECODE:
    case oocs::JOB_COPY_IN: return 1;
    case oocs::JOB_ENCODE:
    case oocs::JOB_COPY_OUT: return 3;
    case oocs::JOB_STORE: return 4;
    default: return 2;
    }
}

// Algorithmic device-memory bytes of one job (each distinct input plane read
// once, each output plane written once).
static int64_t job_bytes(const oocs::Job& j, int64_t plane_elems)
{
    const int64_t planes = j.z1 - j.z0;
    const int64_t pb = plane_elems * (j.f64 ? 8 : 4);
    switch (j.kind) {
    case oocs::JOB_HEAT: return planes * pb * 2;        // read u, write u'
    case oocs::JOB_HEAT_TB: return planes * pb * 2;     // read u(t), write u(t+k): k updates per cell
    case oocs::JOB_WAVE: return planes * pb * 4;        // read p, p(n-1), w; write p(n+1)
    case oocs::JOB_DECODE:
    case oocs::JOB_ENCODE: return planes * (pb + plane_elems * j.rate / 8);
    case oocs::JOB_FETCH:
    case oocs::JOB_STORE: return j.bytes;               // staging side; the other side is the host link
    default: return planes * pb * 2;                    // raw copies
    }
}

int oocs_plan_set_breakdown(oocs_plan* pl, int on)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan");
    pl->breakdown = on != 0;
    return OOCS_OK;
}

int oocs_plan_set_graphs(oocs_plan* pl, int on)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan");
    pl->graphs = on != 0;
    return OOCS_OK;
}

int oocs_plan_set_host_waits(oocs_plan* pl, int on)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan");
    pl->host_waits = on != 0;
    return OOCS_OK;
}

int oocs_plan_set_sdma(oocs_plan* pl, int on)
{
    if (!pl) return fail(OOCS_E_ARG, "null pointer");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan");
    if (on < 0 || on > 16) return fail(OOCS_E_ARG, "sdma must be 0, 1 or an engine count up to 16");
    if (on > 0 && pl->sdma.ready()) {
        const int rc = pl->sdma.drain();  // copies in flight were split the old way
        if (rc != OOCS_OK) return rc;
        (void)pl->sdma.set_engines(on);
    }
    pl->sdma_on = on != 0;
    return OOCS_OK;
}

int oocs_plan_sdma_available(const oocs_plan* pl)
{
    return pl && pl->runnable && pl->sdma.ready() ? 1 : 0;
}

int oocs_link_probe(void* d_a, void* d_b, void* h_in, void* h_out, size_t bytes, size_t chunk, int reps, int sdma,
                    double* out)
{
    if (!d_a || !d_b || !h_in || !h_out || !out || bytes == 0 || chunk == 0 || reps < 1)
        return fail(OOCS_E_ARG, "bad argument");
    const size_t n = (bytes + chunk - 1) / chunk;
    oocs::SdmaCopier cp;
    std::string why;
    uint64_t agent = 0;
    if (sdma < 0 || sdma > 16) return fail(OOCS_E_ARG, "sdma must be 0, 1 or an engine count up to 16");
    const bool use_sdma = sdma && cp.init(d_b, &why) && cp.host_agent(h_out, &agent);
    if (use_sdma) (void)cp.set_engines(sdma);
    struct Streams {
        hipStream_t s[2] = {nullptr, nullptr};
        ~Streams()
        {
            for (hipStream_t x : s)
                if (x) { (void)hipStreamSynchronize(x); (void)hipStreamDestroy(x); }
        }
    } st;
    for (hipStream_t& x : st.s) HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    auto issue = [&](int dirs) -> int {  // bit 0: host to device, bit 1: device to host
        for (size_t i = 0; i < n; ++i) {
            const size_t off = i * chunk, len = std::min(chunk, bytes - off);
            if (dirs & 1)
                HIP_TRY(hipMemcpyAsync(static_cast<char*>(d_a) + off, static_cast<const char*>(h_in) + off, len,
                                       hipMemcpyHostToDevice, st.s[0]));
            if (dirs & 2) {
                if (use_sdma) {
                    const int rc = cp.copy(static_cast<char*>(h_out) + off, agent, static_cast<const char*>(d_b) + off, len);
                    if (rc != OOCS_OK) return rc;
                } else {
                    HIP_TRY(hipMemcpyAsync(static_cast<char*>(h_out) + off, static_cast<const char*>(d_b) + off, len,
                                           hipMemcpyDeviceToHost, st.s[1]));
                }
            }
        }
        return OOCS_OK;
    };
    auto finish = [&]() -> int {
        for (hipStream_t x : st.s) HIP_TRY(hipStreamSynchronize(x));
        return cp.ready() ? cp.drain() : OOCS_OK;
    };
    double sec[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < 3; ++m) {
        const int dirs = m + 1;
        int rc = issue(dirs);  // warm-up
        if (rc == OOCS_OK) rc = finish();
        if (rc != OOCS_OK) return rc;
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < reps && rc == OOCS_OK; ++r) rc = issue(dirs);
        if (rc == OOCS_OK) rc = finish();
        if (rc != OOCS_OK) return rc;
        sec[m] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / reps;
    }
    out[0] = (double)bytes / sec[0] / 1e9;
    out[1] = (double)bytes / sec[1] / 1e9;
    out[2] = (double)bytes / sec[2] / 1e9;
    out[3] = use_sdma ? 1.0 : 0.0;
    return OOCS_OK;
}

}  // extern "C"

namespace {

// Translates the planner's copy and job ops into H2D/D2H transfers and
// launch parameters; shared by the eager and the graph executors.
struct OpTranslator {
    oocs_plan* pl;
    void* const* h_store;
    void* const* d_store;  // device addresses of the host stores (kernel-driven transfers), or null
    bool src_on;
    int variant;  // schedule variant of the residency (addressing of the retained region)
    oocs::LaunchParams lp;
    int64_t h2d = 0, d2h = 0;  // bytes of the transfer jobs added so far

    OpTranslator(oocs_plan* p, void* const* hs, void* const* ds, bool src, int var)
        : pl(p), h_store(hs), d_store(ds), src_on(src), variant(var)
    {
        const oocs::Planner& P = pl->P;
        lp = base_params(P.nx, P.ny, P.nz, P.cfg.alpha, P.cfg.src_x, P.cfg.src_y, P.cfg.src_z);
        if (src_on) {
            lp.src_table = reinterpret_cast<const float*>(pl->arena + P.src_table_off);
            lp.step_ctr = reinterpret_cast<const int32_t*>(pl->arena + P.step_ctr_off);
        }
    }
    oocs::Ring ring(int idx) const
    {
        const oocs::Planner& P = pl->P;
        return oocs::Ring{reinterpret_cast<float*>(pl->arena + P.ringOff[idx]), P.ringW[idx], P.ring_ld()};
    }
    // H2D / D2H of an op: device pointer, host pointer, bytes
    void copy_args(const oocs_op& o, void** dev, void** host, size_t* bytes) const
    {
        const oocs::Planner& P = pl->P;
        const int64_t spb = P.store_plane_bytes(o.field);
        *bytes = (size_t)((o.z1 - o.z0) * spb);
        *host = static_cast<char*>(h_store[o.field]) + o.z0 * spb;
        *dev = o.kind == OOCS_OP_H2D ? pl->arena + P.in_off[o.field] + (int64_t)o.slot * P.in_slot_bytes[o.field]
                                     : pl->arena + P.out_off[o.field] + (int64_t)o.slot * P.out_slot_bytes[o.field];
    }
    // Adds a decode/encode/level op to the pending launch; returns false on overflow.
    bool add_job(const oocs_op& o)
    {
        const oocs::Planner& P = pl->P;
        if (lp.njobs >= oocs::kMaxJobs) return false;
        oocs::Job& j = lp.jobs[lp.njobs++];
        std::memset(&j, 0, sizeof j);
        j.z0 = (int32_t)o.z0;
        j.z1 = (int32_t)o.z1;
        j.f64 = P.fp64 ? 1 : 0;
        if (o.kind == OOCS_OP_FETCH || o.kind == OOCS_OP_STORE) {
            const bool in = o.kind == OOCS_OP_FETCH;
            const int64_t spb = P.store_plane_bytes(o.field);
            j.kind = in ? oocs::JOB_FETCH : oocs::JOB_STORE;
            j.bytes = (o.z1 - o.z0) * spb;
            j.host = static_cast<char*>(d_store[o.field]) + o.z0 * spb;
            j.stage = in ? (void*)(pl->arena + P.in_off[o.field] + (int64_t)o.slot * P.in_slot_bytes[o.field])
                         : (void*)(pl->arena + P.out_off[o.field] + (int64_t)o.slot * P.out_slot_bytes[o.field]);
            (in ? h2d : d2h) += j.bytes;
        } else if (o.kind == OOCS_OP_LEVEL) {
            j.src = ring(o.level - 1);
            j.dst = ring(o.level);
            if (P.cfg.stencil == OOCS_HEAT7 && o.slot > 1) {
                j.kind = oocs::JOB_HEAT_TB;  // o.slot steps in one temporally blocked pass
                j.rate = o.slot;
            } else if (P.cfg.stencil == OOCS_HEAT7) {
                j.kind = oocs::JOB_HEAT;
            } else {
                j.kind = oocs::JOB_WAVE;
                j.src2 = ring(o.level - 2);
                j.ro = ring(P.ro_ring());
                j.has_src = src_on && lp.src_x >= 0 && lp.src_z >= o.z0 && lp.src_z < o.z1;
                j.src_off = o.level - P.nin;  // step of this level within the residency
            }
        } else {
            const bool dec = o.kind == OOCS_OP_DECODE;
            const int rate = P.cfg.rate[o.field];
            j.kind = rate ? (dec ? oocs::JOB_DECODE : oocs::JOB_ENCODE) : (dec ? oocs::JOB_COPY_IN : oocs::JOB_COPY_OUT);
            j.rate = rate;
            j.mid = dec && P.midpoint ? 1 : 0;
            j.dst = ring(o.level);
            if (o.slot == OOCS_SLOT_RETAINED)  // snake: the retained region, laid out like the host store
                j.stage = pl->arena + P.ret_off[o.field] + (o.z0 - P.ret_base(!dec, variant)) * P.store_plane_bytes(o.field);
            else if (o.slot == OOCS_SLOT_DEVICE_STORE)  // the device copy of the read-only store
                j.stage = pl->arena + P.ro_dev_off + o.z0 * P.store_plane_bytes(o.field);
            else
                j.stage = dec ? (void*)(pl->arena + P.in_off[o.field] + (int64_t)o.slot * P.in_slot_bytes[o.field])
                              : (void*)(pl->arena + P.out_off[o.field] + (int64_t)o.slot * P.out_slot_bytes[o.field]);
        }
        return true;
    }
    // algorithmic device-memory bytes of the pending launch: codec, stencil and copy, transfer jobs
    void count_bytes(int64_t* codec, int64_t* stencil, int64_t* xfer) const
    {
        for (int i = 0; i < lp.njobs; ++i) {
            const int kind = lp.jobs[i].kind;
            int64_t* b = oocs::is_codec_job(kind) ? codec : (oocs::is_xfer_job(kind) ? xfer : stencil);
            *b += job_bytes(lp.jobs[i], pl->P.plane_elems());
        }
    }
};

// Decodes the read-only store into its resident ring (OOCS_PLAN_RESIDENT_RO),
// one group of planes at a time through the field's one staging slot, on the
// compute stream. Blocking.
int load_resident_ro(oocs_plan* pl, const void* h_ro)
{
    const oocs::Planner& P = pl->P;
    const int f = 2;
    const int rate = P.cfg.rate[f];
    const int64_t spb = P.store_plane_bytes(f);
    hipStream_t s = pl->st[1];
    char* slot = pl->arena + P.in_off[f];
    for (int64_t z0 = 0; z0 < P.nz; z0 += P.G) {
        const int64_t z1 = std::min(P.nz, z0 + P.G);
        HIP_TRY(hipMemcpyAsync(slot, static_cast<const char*>(h_ro) + z0 * spb, (size_t)((z1 - z0) * spb),
                               hipMemcpyHostToDevice, s));
        oocs::LaunchParams lp = base_params(P.nx, P.ny, P.nz, P.cfg.alpha, -1, -1, -1);
        oocs::Job& j = lp.jobs[0];
        j.kind = rate ? oocs::JOB_DECODE : oocs::JOB_COPY_IN;
        j.rate = rate;
        j.mid = P.midpoint ? 1 : 0;
        j.z0 = (int32_t)z0;
        j.z1 = (int32_t)z1;
        j.dst = oocs::Ring{reinterpret_cast<float*>(pl->arena + P.ringOff[P.ro_ring()]), P.ringW[P.ro_ring()],
                           P.ring_ld()};
        j.f64 = P.fp64 ? 1 : 0;
        j.stage = slot;
        lp.njobs = 1;
        HIP_TRY(oocs::launch_jobs(lp, s));
        HIP_TRY(hipStreamSynchronize(s));  // the slot takes the next group
    }
    pl->ro_loaded = h_ro;
    return OOCS_OK;
}

// Builds the graph of one residency of kr steps.
int build_graph(oocs_plan* pl, int kr, int variant, void* const* h_store, void* const* d_store, bool src_on,
                ResidencyGraph& out)
{
    oocs::Planner& P = pl->P;
    std::string err;
    const oocs::Schedule* sch = P.schedule(kr, err, variant);
    if (!sch) return fail(OOCS_E_STATE, err);
    hipGraph_t g = nullptr;
    HIP_TRY(hipGraphCreate(&g, 0));
    struct GraphGuard { hipGraph_t g; ~GraphGuard() { if (g) (void)hipGraphDestroy(g); } } guard{g};
    hipGraphNode_t last[3] = {nullptr, nullptr, nullptr};
    std::vector<hipGraphNode_t> pending[3];
    std::map<int, hipGraphNode_t> rec;  // logical event -> node it stands for, recorded in this graph
    auto deps_of = [&](int s) {
        std::vector<hipGraphNode_t> d;
        if (last[s]) d.push_back(last[s]);
        for (hipGraphNode_t n : pending[s])
            if (n && std::find(d.begin(), d.end(), n) == d.end()) d.push_back(n);
        pending[s].clear();
        return d;
    };
    OpTranslator tr(pl, h_store, d_store, src_on, variant);
    for (const oocs_op& o : sch->ops) {
        switch (o.kind) {
        case OOCS_OP_H2D:
        case OOCS_OP_D2H: {
            void *dev, *host;
            size_t bytes;
            tr.copy_args(o, &dev, &host, &bytes);
            std::vector<hipGraphNode_t> d = deps_of(o.stream);
            hipGraphNode_t n;
            if (o.kind == OOCS_OP_H2D) {
                HIP_TRY(hipGraphAddMemcpyNode1D(&n, g, d.data(), d.size(), dev, host, bytes, hipMemcpyHostToDevice));
                out.h2d += (int64_t)bytes;
            } else {
                HIP_TRY(hipGraphAddMemcpyNode1D(&n, g, d.data(), d.size(), host, dev, bytes, hipMemcpyDeviceToHost));
                out.d2h += (int64_t)bytes;
            }
            last[o.stream] = n;
            break;
        }
        case OOCS_OP_DECODE:
        case OOCS_OP_ENCODE:
        case OOCS_OP_LEVEL:
        case OOCS_OP_FETCH:
        case OOCS_OP_STORE:
            if (!tr.add_job(o)) return fail(OOCS_E_STATE, "too many jobs in a tick");
            break;
        case OOCS_OP_LAUNCH: {
            if (tr.lp.njobs == 0) break;
            int64_t lb[3] = {0, 0, 0};
            tr.count_bytes(&lb[0], &lb[1], &lb[2]);
            out.codec_bytes += lb[0];
            out.stencil_bytes += lb[1];
            out.xfer_bytes += lb[2];
            const bool timed = pl->profiling > 0 && out.launches % pl->profiling == 0;
            if (timed) out.timed_bytes += lb[0] + lb[1] + lb[2];
            std::vector<hipGraphNode_t> d = deps_of(1);
            if (timed) {
                hipEvent_t e0, e1;
                HIP_TRY(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));  // timing only
                out.timing.push_back(e0);
                HIP_TRY(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
                out.timing.push_back(e1);
                hipGraphNode_t n0;
                HIP_TRY(hipGraphAddEventRecordNode(&n0, g, d.data(), d.size(), e0));
                d.assign(1, n0);
            }
            hipGraphNode_t n;
            HIP_TRY(oocs::add_jobs_node(tr.lp, g, d.data(), d.size(), &n));
            if (timed) {
                hipGraphNode_t n1;
                HIP_TRY(hipGraphAddEventRecordNode(&n1, g, &n, 1, out.timing.back()));
                n = n1;
            }
            last[1] = n;
            ++out.launches;
            tr.lp.njobs = 0;
            break;
        }
        case OOCS_OP_RECORD:
            if (!pending[o.stream].empty()) {  // carry waits that no node has absorbed yet
                std::vector<hipGraphNode_t> d = deps_of(o.stream);
                hipGraphNode_t n;
                HIP_TRY(hipGraphAddEmptyNode(&n, g, d.data(), d.size()));
                last[o.stream] = n;
            }
            rec[o.event] = last[o.stream];
            break;
        case OOCS_OP_WAIT: {
            auto it = rec.find(o.event);
            if (it != rec.end() && it->second) pending[o.stream].push_back(it->second);
            break;  // events of earlier residencies are complete before this graph starts
        }
        default:
            return fail(OOCS_E_STATE, "unknown op");
        }
    }
    if (src_on) {  // advance the source step counter after this residency's levels
        std::vector<hipGraphNode_t> d = deps_of(1);
        hipGraphNode_t n;
        HIP_TRY(oocs::add_step_ctr_node(reinterpret_cast<int32_t*>(pl->arena + P.step_ctr_off), true, kr, g, d.data(),
                                        d.size(), &n));
        last[1] = n;
    }
    HIP_TRY(hipGraphInstantiate(&out.exec, g, nullptr, nullptr, 0));
    out.h2d += tr.h2d;
    out.d2h += tr.d2h;
    return OOCS_OK;
}

}  // namespace

extern "C" {

int oocs_run(oocs_plan* pl, void* const* h_store, int64_t steps, const float* h_src, oocs_stats* st)
{
    if (!pl || !h_store || steps < 0) return fail(OOCS_E_ARG, "bad argument");
    if (!pl->runnable) return fail(OOCS_E_STATE, "planning-only plan cannot run");
    oocs::Planner& P = pl->P;
    for (int f : P.in_fields)
        if (!h_store[f]) return fail(OOCS_E_ARG, "missing host store pointer");
    if (P.resident_ro && !h_store[2]) return fail(OOCS_E_ARG, "missing read-only store pointer");
    const auto t_start = std::chrono::steady_clock::now();
    if (P.resident_ro && pl->ro_loaded != h_store[2]) {
        const int rc = load_resident_ro(pl, h_store[2]);
        if (rc != OOCS_OK) return rc;
    }
    if (P.ro_dev && pl->ro_loaded != h_store[2]) {  // the read-only store, copied once into the arena
        HIP_TRY(hipMemcpyAsync(pl->arena + P.ro_dev_off, h_store[2], (size_t)P.store_bytes(2), hipMemcpyHostToDevice,
                               pl->st[1]));
        HIP_TRY(hipStreamSynchronize(pl->st[1]));
        pl->ro_loaded = h_store[2];
    }
    const bool src_on = h_src != nullptr && P.cfg.stencil == OOCS_WAVE25 && P.cfg.src_x >= 0 && P.cfg.src_x < P.nx &&
                        P.cfg.src_y >= 0 && P.cfg.src_y < P.ny && P.cfg.src_z >= 0 && P.cfg.src_z < P.nz;
    int32_t* step_ctr = src_on ? reinterpret_cast<int32_t*>(pl->arena + P.step_ctr_off) : nullptr;
    float* src_table = src_on ? reinterpret_cast<float*>(pl->arena + P.src_table_off) : nullptr;
    // the source table holds a whole number of residencies
    const int64_t chunk_steps = src_on ? oocs::Planner::kSrcTable / P.k * P.k : steps;
    int64_t h2d = 0, d2h = 0, rounds = 0, launches = 0;
    int64_t kbytes[3] = {0, 0, 0};  // codec jobs, stencil and copy jobs, transfer jobs
    int64_t tbytes = 0, tlaunches = 0;  // the timed launches (profiling)
    // kernel-driven transfers address the host stores from the device
    void* d_store[OOCS_MAX_FIELDS] = {nullptr, nullptr, nullptr};
    if (!P.copy_engines || P.kernel_stores)
        for (int f = 0; f < P.nfields; ++f) {
            if (!h_store[f]) continue;
            if (hipHostGetDevicePointer(&d_store[f], h_store[f], 0) != hipSuccess || !d_store[f]) {
                (void)hipGetLastError();
                return fail(OOCS_E_ARG, "host store of field " + std::to_string(f) +
                                            " is not pinned host memory the device can address");
            }
        }
    double kms = 0.0;
    size_t tused = 0;
    const int ns = P.nstage;
    // breakdown: event pairs (start, end) with the stage each one times
    const bool bdown = pl->breakdown && !pl->graphs;
    size_t bused = 0;
    std::vector<int8_t> bstage;
    auto bevent = [&](int stage, hipStream_t s) -> int {  // records the start of a pair
        while (pl->bev.size() < bused + 2) {
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));  // timing only
            pl->bev.push_back(e);
        }
        HIP_TRY(hipEventRecord(pl->bev[bused], s));
        bstage.push_back((int8_t)stage);
        return OOCS_OK;
    };
    auto bevent_end = [&](hipStream_t s) -> int {
        HIP_TRY(hipEventRecord(pl->bev[bused + 1], s));
        bused += 2;
        return OOCS_OK;
    };
    // Device-to-host copies go to an SDMA engine when the host honours the
    // cross-stream waits itself (op-by-op issue with host waits): a wait on
    // the write-back stream then becomes a wait for the copies issued before
    // its record. Every store written back must be pinned memory of a CPU pool.
    {
        const int rc = pl->sdma.drain();  // copies left by a run that failed part-way
        if (rc != OOCS_OK) return rc;
    }
    uint64_t cpu_agent[OOCS_MAX_FIELDS] = {0, 0, 0};
    bool use_sdma = pl->sdma_on && pl->sdma.ready() && !pl->graphs && pl->host_waits && P.copy_engines && !P.kernel_stores;
    for (int f : P.out_fields)
        if (use_sdma && !pl->sdma.host_agent(h_store[f], &cpu_agent[f])) use_sdma = false;
    std::fill(pl->ev_ticket.begin(), pl->ev_ticket.end(), (int64_t)-1);
    int64_t sdma_copies = 0;
    if (use_sdma) {
        const int rc = pl->sdma.set_timing(bdown);
        if (rc != OOCS_OK) return rc;
    }

    int64_t done = 0;
    const int64_t nres = (steps + P.k - 1) / P.k;  // residencies of this call (snake variants)
    while (done < steps) {
        const int64_t chunk_end = std::min(steps, done + chunk_steps);
        if (src_on) {  // amplitudes of this chunk, counter at 0
            HIP_TRY(hipStreamSynchronize(pl->st[1]));
            HIP_TRY(hipMemcpyAsync(src_table, h_src + done, (size_t)(chunk_end - done) * 4, hipMemcpyHostToDevice,
                                   pl->st[1]));
            HIP_TRY(oocs::launch_step_ctr(step_ctr, false, 0, pl->st[1]));
        }
        int64_t chunk_round = 0;
        while (done < chunk_end) {
            const int kr = (int)std::min<int64_t>(P.k, chunk_end - done);
            const int variant = P.variant_of(rounds, nres);
            std::string err;
            const oocs::Schedule* sch = P.schedule(kr, err, variant);
            if (!sch) return fail(OOCS_E_STATE, err);
            if (pl->graphs) {
                auto key = std::make_tuple(kr + 64 * variant, (const void*)h_store[0],
                                           (const void*)(P.nfields > 1 ? h_store[1] : nullptr),
                                           (const void*)(P.nfields > 2 ? h_store[2] : nullptr), src_on, pl->profiling);
                auto it = pl->gcache.find(key);
                if (it == pl->gcache.end()) {
                    ResidencyGraph rg;
                    const int rc = build_graph(pl, kr, variant, h_store, d_store, src_on, rg);
                    if (rc != OOCS_OK) {
                        if (rg.exec) (void)hipGraphExecDestroy(rg.exec);
                        for (hipEvent_t e : rg.timing) (void)hipEventDestroy(e);
                        return rc;
                    }
                    it = pl->gcache.emplace(key, std::move(rg)).first;
                }
                ResidencyGraph& rg = it->second;
                HIP_TRY(hipGraphLaunch(rg.exec, pl->st[1]));
                h2d += rg.h2d;
                d2h += rg.d2h;
                launches += rg.launches;
                kbytes[0] += rg.codec_bytes;
                kbytes[1] += rg.stencil_bytes;
                kbytes[2] += rg.xfer_bytes;
                if (pl->profiling) {  // the timing events hold this replay's times once it completes
                    tbytes += rg.timed_bytes;
                    tlaunches += (int64_t)rg.timing.size() / 2;
                    HIP_TRY(hipStreamSynchronize(pl->st[1]));
                    for (size_t i = 0; i + 1 < rg.timing.size(); i += 2) {
                        float ms = 0.0f;
                        HIP_TRY(hipEventElapsedTime(&ms, rg.timing[i], rg.timing[i + 1]));
                        kms += ms;
                    }
                }
            } else {
                const int parity = (int)(rounds & 1);
                auto phys = [&](int e) -> int {  // index into pl->ev
                    if (e < 4 * ns) return e;
                    int i = e - 4 * ns;
                    const bool prev = i >= P.n;
                    if (prev) i -= P.n;
                    const int par = prev ? 1 - parity : parity;
                    return 4 * ns + par * P.n + i;
                };
                OpTranslator tr(pl, h_store, d_store, src_on, variant);
                for (const oocs_op& o : sch->ops) {
                    switch (o.kind) {
                    case OOCS_OP_H2D:
                    case OOCS_OP_D2H: {
                        void *dev, *host;
                        size_t bytes;
                        tr.copy_args(o, &dev, &host, &bytes);
                        if (o.kind == OOCS_OP_H2D) {
                            if (bdown && bevent(0, pl->st[0]) != OOCS_OK) return OOCS_E_HIP;
                            HIP_TRY(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, pl->st[0]));
                            if (bdown && bevent_end(pl->st[0]) != OOCS_OK) return OOCS_E_HIP;
                            h2d += (int64_t)bytes;
                        } else if (use_sdma) {
                            const int rc = pl->sdma.copy(host, cpu_agent[o.field], dev, bytes);
                            if (rc != OOCS_OK) return rc;
                            d2h += (int64_t)bytes;
                            ++sdma_copies;
                        } else {
                            if (bdown && bevent(4, pl->st[2]) != OOCS_OK) return OOCS_E_HIP;
                            HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, pl->st[2]));
                            if (bdown && bevent_end(pl->st[2]) != OOCS_OK) return OOCS_E_HIP;
                            d2h += (int64_t)bytes;
                        }
                        break;
                    }
                    case OOCS_OP_DECODE:
                    case OOCS_OP_ENCODE:
                    case OOCS_OP_LEVEL:
                    case OOCS_OP_FETCH:
                    case OOCS_OP_STORE:
                        if (!tr.add_job(o)) return fail(OOCS_E_STATE, "too many jobs in a tick");
                        break;
                    case OOCS_OP_LAUNCH:
                        if (tr.lp.njobs > 0) {
                            int64_t lb[3] = {0, 0, 0};
                            tr.count_bytes(&lb[0], &lb[1], &lb[2]);
                            for (int q = 0; q < 3; ++q) kbytes[q] += lb[q];
                            const bool timed = pl->profiling > 0 && launches % pl->profiling == 0;
                            if (timed) {
                                tbytes += lb[0] + lb[1] + lb[2];
                                ++tlaunches;
                                while (pl->tev.size() < tused + 2) {
                                    hipEvent_t e;
                                    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));  // timing only
                                    pl->tev.push_back(e);
                                }
                                HIP_TRY(hipEventRecord(pl->tev[tused], pl->st[1]));
                            }
                            if (bdown) {
                                // one launch per stage, in stage order (the jobs of a tick
                                // are independent, so any order gives the same bits)
                                for (int stage = 0; stage < 5; ++stage) {
                                    oocs::LaunchParams sub = tr.lp;
                                    sub.njobs = 0;
                                    for (int q = 0; q < tr.lp.njobs; ++q)
                                        if (job_stage(tr.lp.jobs[q].kind) == stage) sub.jobs[sub.njobs++] = tr.lp.jobs[q];
                                    if (sub.njobs == 0) continue;
                                    if (bevent(stage, pl->st[1]) != OOCS_OK) return OOCS_E_HIP;
                                    HIP_TRY(oocs::launch_jobs(sub, pl->st[1]));
                                    if (bevent_end(pl->st[1]) != OOCS_OK) return OOCS_E_HIP;
                                }
                            } else {
                                HIP_TRY(oocs::launch_jobs(tr.lp, pl->st[1]));
                            }
                            if (timed) {
                                HIP_TRY(hipEventRecord(pl->tev[tused + 1], pl->st[1]));
                                tused += 2;
                            }
                            ++launches;
                        }
                        tr.lp.njobs = 0;
                        break;
                    case OOCS_OP_RECORD: {
                        const int i = phys(o.event);
                        if (use_sdma && o.stream == 2) {
                            pl->ev_ticket[i] = pl->sdma.issued();
                        } else {
                            pl->ev_ticket[i] = -1;
                            HIP_TRY(hipEventRecord(pl->ev[i], pl->st[o.stream]));
                        }
                        break;
                    }
                    case OOCS_OP_WAIT: {
                        if (o.event >= P.ev_blk_prev(0) && chunk_round == 0 && rounds == 0) break;
                        // The host waits for the event itself instead of making the stream
                        // wait: a stream wait on a pending event from another stream costs
                        // the host ~10 us and makes the next copy call on that stream
                        // several times dearer, while the GPU is still two ticks behind
                        // by the time a lagged copy is issued. A completed event is free.
                        const int ei = phys(o.event);
                        if (pl->ev_ticket[ei] >= 0) {  // recorded behind SDMA copies
                            const int rc = pl->sdma.wait(pl->ev_ticket[ei]);
                            if (rc != OOCS_OK) return rc;
                            break;
                        }
                        const hipEvent_t e = pl->ev[ei];
                        const hipError_t q = hipEventQuery(e);
                        if (q == hipSuccess) break;
                        if (q != hipErrorNotReady) return oocs::hip_fail(q, "event query");
                        if (pl->host_waits) {
                            // poll rather than hipEventSynchronize, which may put the
                            // thread to sleep and wake it up late
                            hipError_t w;
                            while ((w = hipEventQuery(e)) == hipErrorNotReady) __builtin_ia32_pause();
                            if (w != hipSuccess) return oocs::hip_fail(w, "event query");
                        } else {
                            HIP_TRY(hipStreamWaitEvent(pl->st[o.stream], e, 0));
                        }
                        break;
                    }
                    default:
                        return fail(OOCS_E_STATE, "unknown op");
                    }
                }
                if (src_on) HIP_TRY(oocs::launch_step_ctr(step_ctr, true, kr, pl->st[1]));
                h2d += tr.h2d;
                d2h += tr.d2h;
            }
            done += kr;
            ++rounds;
            ++chunk_round;
        }
    }
    const double enq = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int i = 0; i < 3; ++i) HIP_TRY(hipStreamSynchronize(pl->st[i]));
    {
        const int rc = pl->sdma.drain();
        if (rc != OOCS_OK) return rc;
    }
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (size_t i = 0; i + 1 < tused; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pl->tev[i], pl->tev[i + 1]));
        kms += ms;
    }
    double stage_ms[5] = {0, 0, 0, 0, 0};
    for (size_t i = 0; i + 1 < bused; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pl->bev[i], pl->bev[i + 1]));
        stage_ms[bstage[i / 2]] += ms;
    }
    if (use_sdma && bdown) {
        stage_ms[4] += pl->sdma.busy_ms();
        const int rc = pl->sdma.set_timing(false);
        if (rc != OOCS_OK) return rc;
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
        st->xfer_bytes = kbytes[2];
        st->timed_launches = tlaunches;
        st->timed_bytes = tbytes;
        st->sdma_copies = sdma_copies;
        st->kernel_ms = kms;
        for (int q = 0; q < 5; ++q) st->stage_ms[q] = bdown ? stage_ms[q] : 0.0;
        st->arena_bytes = P.arena_needed;
    }
    return OOCS_OK;
}

}  // extern "C"
