// adjoint.cpp -- host orchestration of the misfit gradient: forward pass
// with checkpoints through the fixed-rate codec to host memory, backward
// pass by segments in reverse (restore, recompute on the device, adjoint).
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "abi_util.hpp"
#include "internal.hpp"
#include "oocs.h"

namespace {

using oocs::fail;

struct Layout {
    int64_t n = 0, fb = 0, cb = 0;  // cells, field bytes, compressed field bytes (0 if raw)
    int64_t nseg = 0, C = 0;
    int64_t w = 0, states = 0, lam = 0, wl = 0, gw = 0, stage = 0, total = 0;
    int64_t ckpt_field = 0, ckpt_total = 0;  // host bytes per stored field, all checkpoints
};

int64_t up256(int64_t v) { return (v + 255) / 256 * 256; }

int layout_of(const oocs_adjoint_cfg* c, Layout& L)
{
    if (!c) return fail(OOCS_E_ARG, "null config");
    if (c->nx <= 0 || c->ny <= 0 || c->nz <= 0 || c->nx % 4) return fail(OOCS_E_ARG, "bad grid (nx multiple of 4)");
    if (c->steps < 1 || c->ckpt_every < 1 || c->nrcv < 0) return fail(OOCS_E_ARG, "bad steps, ckpt_every or nrcv");
    if (c->ckpt_rate < 0 || c->ckpt_rate > OOCS_MAX_RATE) return fail(OOCS_E_RATE, "ckpt_rate outside [0, 34]");
    if (c->ckpt_rate > 0 && (c->ny % 4 || c->nz % 4)) return fail(OOCS_E_ALIGN, "compressed checkpoints need dims % 4");
    if (c->src_x < 0 || c->src_y < 0 || c->src_z < 0 || c->src_x >= c->nx || c->src_y >= c->ny || c->src_z >= c->nz)
        return fail(OOCS_E_ARG, "source cell outside the grid");
    L.n = c->nx * c->ny * c->nz;
    L.fb = up256(L.n * 4);
    L.cb = c->ckpt_rate ? up256((int64_t)oocs_codec_bytes(c->nx, c->ny, c->nz, c->ckpt_rate)) : 0;
    L.C = c->ckpt_every;
    L.nseg = (c->steps + L.C - 1) / L.C;
    int64_t off = 0;
    L.w = off; off += L.fb;
    L.states = off; off += (L.C + 2) * L.fb;
    L.lam = off; off += 3 * L.fb;
    L.wl = off; off += 2 * L.fb;
    L.gw = off; off += L.fb;
    L.stage = off; off += 2 * L.cb;
    L.total = off;
    L.ckpt_field = c->ckpt_rate ? (int64_t)oocs_codec_bytes(c->nx, c->ny, c->nz, c->ckpt_rate) : L.n * 4;
    L.ckpt_total = L.nseg * 2 * L.ckpt_field;
    return OOCS_OK;
}

// One leapfrog step on whole fields: dst = 2 cur - prev + w . L cur (+ amp)
int wave_step(const oocs_adjoint_cfg* c, float* cur, float* prev, const float* w, float* dst, float amp,
              hipStream_t s)
{
    oocs::LaunchParams p;
    std::memset(&p, 0, sizeof p);
    p.nx = (int32_t)c->nx; p.ny = (int32_t)c->ny; p.nz = (int32_t)c->nz;
    p.src_x = (int32_t)c->src_x; p.src_y = (int32_t)c->src_y; p.src_z = (int32_t)c->src_z;
    oocs::Job& j = p.jobs[0];
    j.kind = oocs::JOB_WAVE;
    j.z0 = 0; j.z1 = (int32_t)c->nz;
    const int64_t pe = c->nx * c->ny;
    j.src = {cur, c->nz, pe};
    j.src2 = {prev, c->nz, pe};
    j.ro = {const_cast<float*>(w), c->nz, pe};
    j.dst = {dst, c->nz, pe};
    j.has_src = 1;
    j.amp = amp;
    p.njobs = 1;
    HIP_TRY(oocs::launch_jobs(p, s));
    return OOCS_OK;
}

// A second stream for the checkpoint copies, with the two events that order
// it against the compute stream; synchronised and released on every exit.
struct CopyStream {
    hipStream_t s = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int init()
    {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        for (hipEvent_t& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return OOCS_OK;
    }
    ~CopyStream()
    {
        if (s) (void)hipStreamSynchronize(s);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (s) (void)hipStreamDestroy(s);
    }
};

// Order `waiter` after the work queued so far on `signaller`.
int order_after(hipStream_t waiter, hipStream_t signaller, hipEvent_t e)
{
    HIP_TRY(hipEventRecord(e, signaller));
    HIP_TRY(hipStreamWaitEvent(waiter, e, 0));
    return OOCS_OK;
}

int common_checks(const oocs_adjoint_cfg* c, const Layout& L, const void* d_v, const float* h_src, const void* d_rcv,
                  const void* d_work, size_t work_bytes, const void* h_ckpt)
{
    if (!d_v || !h_src || (c->nrcv > 0 && !d_rcv) || !d_work || !h_ckpt) return fail(OOCS_E_ARG, "null pointer");
    if ((int64_t)work_bytes < L.total) return fail(OOCS_E_SIZE, "workspace too small");
    if ((uintptr_t)d_work % 256) return fail(OOCS_E_ALIGN, "workspace must be 256-byte aligned");
    return OOCS_OK;
}

}  // namespace

extern "C" {

size_t oocs_adjoint_workspace_bytes(const oocs_adjoint_cfg* c)
{
    Layout L;
    return layout_of(c, L) == OOCS_OK ? (size_t)L.total : 0;
}

size_t oocs_adjoint_ckpt_bytes(const oocs_adjoint_cfg* c)
{
    Layout L;
    return layout_of(c, L) == OOCS_OK ? (size_t)L.ckpt_total : 0;
}

int oocs_wave_forward_ckpt(const oocs_adjoint_cfg* c, const float* d_v, const float* h_src, const int64_t* d_rcv,
                           const float* d_obs, float* d_res, void* d_work, size_t work_bytes, void* h_ckpt, double* J,
                           void* stream)
{
    Layout L;
    int rc = layout_of(c, L);
    if (rc) return rc;
    if ((rc = common_checks(c, L, d_v, h_src, d_rcv, d_work, work_bytes, h_ckpt))) return rc;
    if (c->nrcv > 0 && (!d_obs || !d_res)) return fail(OOCS_E_ARG, "null records");
    if (!J) return fail(OOCS_E_ARG, "null J");
    hipStream_t s = (hipStream_t)stream;
    char* work = static_cast<char*>(d_work);
    float* w = reinterpret_cast<float*>(work + L.w);
    float* A = reinterpret_cast<float*>(work + L.states);           // p(t-1)
    float* B = reinterpret_cast<float*>(work + L.states + L.fb);    // p(t)
    char* stage = work + L.stage;
    char* ck = static_cast<char*>(h_ckpt);
    HIP_TRY(oocs::launch_v_to_w(d_v, c->vscale, w, L.n, s));
    HIP_TRY(oocs::launch_fill(A, 0.0f, L.n, s));
    HIP_TRY(oocs::launch_fill(B, 0.0f, L.n, s));
    const int nr = c->nrcv;
    // Compressed checkpoints: each field is encoded into its staging slot on
    // the compute stream and copied to the host on the copy stream while the
    // next steps run; the slot is encoded again only after that copy. Raw
    // checkpoints are copied from the state fields on the compute stream
    // (the next step overwrites p(t-1)).
    CopyStream cs;
    if (c->ckpt_rate && (rc = cs.init())) return rc;
    bool pending[2] = {false, false};
    for (int64_t t = 0; t < c->steps; ++t) {
        if (t % L.C == 0) {
            char* slot = ck + (t / L.C) * 2 * L.ckpt_field;
            const float* f2[2] = {B, A};  // p(t), p(t-1)
            for (int f = 0; f < 2; ++f) {
                char* host = slot + f * L.ckpt_field;
                if (c->ckpt_rate == 0) {
                    HIP_TRY(hipMemcpyAsync(host, f2[f], (size_t)(L.n * 4), hipMemcpyDeviceToHost, s));
                    continue;
                }
                char* st = stage + f * L.cb;
                if (pending[f]) HIP_TRY(hipStreamWaitEvent(s, cs.ev[2 + f], 0));
                HIP_TRY(oocs::launch_codec_field(true, f2[f], nullptr, nullptr, reinterpret_cast<uint64_t*>(st), c->nx,
                                                 c->ny, c->nz, c->nx, c->nx * c->ny, c->ckpt_rate, s));
                if ((rc = order_after(cs.s, s, cs.ev[f]))) return rc;
                HIP_TRY(hipMemcpyAsync(host, st, (size_t)L.ckpt_field, hipMemcpyDeviceToHost, cs.s));
                HIP_TRY(hipEventRecord(cs.ev[2 + f], cs.s));
                pending[f] = true;
            }
        }
        if ((rc = wave_step(c, B, A, w, A, h_src[t], s))) return rc;  // p(t+1) over p(t-1)
        std::swap(A, B);
        HIP_TRY(oocs::launch_rcv_sample(B, d_rcv, nr, d_obs + t * nr, d_res + t * nr, L.n, s));
    }
    std::vector<float> res((size_t)c->steps * nr);
    if (nr > 0) HIP_TRY(hipMemcpyAsync(res.data(), d_res, res.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (cs.s) HIP_TRY(hipStreamSynchronize(cs.s));
    double j = 0.0;
    for (float r : res) j += (double)r * (double)r;
    *J = 0.5 * j;
    return OOCS_OK;
}

int oocs_wave_adjoint(const oocs_adjoint_cfg* c, const float* d_v, const float* h_src, const int64_t* d_rcv,
                      const float* d_res, void* d_work, size_t work_bytes, const void* h_ckpt, float* d_grad_v,
                      void* stream)
{
    Layout L;
    int rc = layout_of(c, L);
    if (rc) return rc;
    if ((rc = common_checks(c, L, d_v, h_src, d_rcv, d_work, work_bytes, h_ckpt))) return rc;
    if (!d_grad_v || (c->nrcv > 0 && !d_res)) return fail(OOCS_E_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    char* work = static_cast<char*>(d_work);
    float* w = reinterpret_cast<float*>(work + L.w);
    auto S = [&](int64_t i) { return reinterpret_cast<float*>(work + L.states + i * L.fb); };
    float* lam[3] = {reinterpret_cast<float*>(work + L.lam), reinterpret_cast<float*>(work + L.lam + L.fb),
                     reinterpret_cast<float*>(work + L.lam + 2 * L.fb)};
    float* wl[2] = {reinterpret_cast<float*>(work + L.wl), reinterpret_cast<float*>(work + L.wl + L.fb)};
    float* gw = reinterpret_cast<float*>(work + L.gw);
    char* stage = work + L.stage;
    const char* ck = static_cast<const char*>(h_ckpt);
    HIP_TRY(oocs::launch_v_to_w(d_v, c->vscale, w, L.n, s));
    for (int i = 0; i < 3; ++i) HIP_TRY(oocs::launch_fill(lam[i], 0.0f, L.n, s));
    for (int i = 0; i < 2; ++i) HIP_TRY(oocs::launch_fill(wl[i], 0.0f, L.n, s));
    HIP_TRY(oocs::launch_fill(gw, 0.0f, L.n, s));
    // The copy stream brings in segment seg-1's checkpoint while segment seg
    // runs: into the staging slots once they are decoded (compressed), or
    // straight into the first two state fields once the recompute has read
    // them (raw; the adjoint steps use the later states only).
    CopyStream cs;
    if ((rc = cs.init())) return rc;
    auto issue_load = [&](int64_t seg) -> int {
        const char* slot = ck + seg * 2 * L.ckpt_field;
        void* dst[2] = {c->ckpt_rate ? (void*)stage : (void*)S(1), c->ckpt_rate ? (void*)(stage + L.cb) : (void*)S(0)};
        for (int f = 0; f < 2; ++f)  // p(t0), p(t0-1)
            HIP_TRY(hipMemcpyAsync(dst[f], slot + f * L.ckpt_field, (size_t)L.ckpt_field, hipMemcpyHostToDevice, cs.s));
        return OOCS_OK;
    };
    if ((rc = order_after(cs.s, s, cs.ev[0]))) return rc;  // after the fills above
    if ((rc = issue_load(L.nseg - 1))) return rc;
    // lam[i2] = lam(t+2), lam[i1] = lam(t+1), lam[i0] = lam(t) (rotating);
    // wl[j1] = w . lam(t+1), wl[j0] = w . lam(t)
    int i0 = 0, i1 = 1, i2 = 2, j0 = 0, j1 = 1;
    for (int64_t seg = L.nseg - 1; seg >= 0; --seg) {
        const int64_t t0 = seg * L.C, t1 = std::min(c->steps, t0 + L.C);
        if ((rc = order_after(s, cs.s, cs.ev[1]))) return rc;  // this segment's checkpoint is in
        if (c->ckpt_rate) {
            for (int f = 0; f < 2; ++f)
                HIP_TRY(oocs::launch_codec_field(false, nullptr, S(1 - f), reinterpret_cast<const uint64_t*>(stage + f * L.cb),
                                                 nullptr, c->nx, c->ny, c->nz, c->nx, c->nx * c->ny, c->ckpt_rate, s));
            if (seg > 0) {
                if ((rc = order_after(cs.s, s, cs.ev[0]))) return rc;
                if ((rc = issue_load(seg - 1))) return rc;
            }
        }
        for (int64_t t = t0; t < t1; ++t)  // S(t - t0 + 1) = p(t); S(t - t0 + 2) = p(t+1)
            if ((rc = wave_step(c, S(t - t0 + 1), S(t - t0), w, S(t - t0 + 2), h_src[t], s))) return rc;
        if (!c->ckpt_rate && seg > 0) {
            if ((rc = order_after(cs.s, s, cs.ev[0]))) return rc;
            if ((rc = issue_load(seg - 1))) return rc;
        }
        for (int64_t t = t1; t > t0; --t) {
            HIP_TRY(oocs::launch_adjoint_step(lam[i1], wl[j1], lam[i2], w, S(t - t0 + 1), lam[i0], wl[j0], gw, c->nx,
                                              c->ny, c->nz, s));
            HIP_TRY(oocs::launch_rcv_inject(lam[i0], wl[j0], w, d_rcv, c->nrcv, d_res + (t - 1) * c->nrcv, L.n, s));
            const int old2 = i2;
            i2 = i1;
            i1 = i0;
            i0 = old2;
            std::swap(j0, j1);
        }
    }
    HIP_TRY(oocs::launch_grad_w_to_v(gw, d_v, c->vscale, d_grad_v, L.n, s));
    HIP_TRY(hipStreamSynchronize(s));
    return OOCS_OK;
}

}  // extern "C"
