// sdma.cpp -- SdmaCopier: HSA asynchronous copies from device to host memory.
//
// The HSA entry points are looked up in the runtime instance that is already
// loaded (the one HIP itself drives), never in a second copy: device
// pointers, agents and signals belong to that instance.
#include "sdma.hpp"

#include <dlfcn.h>

#include <algorithm>
#include <chrono>

#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include "oocs.h"

namespace oocs {
int fail(int code, const std::string& msg);
}

namespace {

struct HsaApi {
    decltype(&hsa_agent_get_info) agent_get_info = nullptr;
    decltype(&hsa_signal_create) signal_create = nullptr;
    decltype(&hsa_signal_destroy) signal_destroy = nullptr;
    decltype(&hsa_signal_load_scacquire) signal_load = nullptr;
    decltype(&hsa_signal_store_relaxed) signal_store = nullptr;
    decltype(&hsa_amd_memory_async_copy) async_copy = nullptr;
    // copies on chosen engines (optional: only split copies need them)
    decltype(&hsa_amd_memory_async_copy_on_engine) async_copy_on_engine = nullptr;
    decltype(&hsa_amd_memory_copy_engine_status) engine_status = nullptr;
    decltype(&hsa_amd_pointer_info) pointer_info = nullptr;
    // copy timing (optional: only the breakdown mode needs them)
    decltype(&hsa_amd_profiling_async_copy_enable) copy_prof_enable = nullptr;
    decltype(&hsa_amd_profiling_get_async_copy_time) copy_time = nullptr;
    decltype(&hsa_system_get_info) system_info = nullptr;
    bool ok = false;
};

const HsaApi& api()
{
    static const HsaApi a = [] {
        HsaApi r;
        // RTLD_NOLOAD: only the instance that is loaded already
        void* h = dlopen("libhsa-runtime64.so.1", RTLD_NOW | RTLD_NOLOAD);
        if (!h) return r;
        r.agent_get_info = reinterpret_cast<decltype(r.agent_get_info)>(dlsym(h, "hsa_agent_get_info"));
        r.signal_create = reinterpret_cast<decltype(r.signal_create)>(dlsym(h, "hsa_signal_create"));
        r.signal_destroy = reinterpret_cast<decltype(r.signal_destroy)>(dlsym(h, "hsa_signal_destroy"));
        r.signal_load = reinterpret_cast<decltype(r.signal_load)>(dlsym(h, "hsa_signal_load_scacquire"));
        r.signal_store = reinterpret_cast<decltype(r.signal_store)>(dlsym(h, "hsa_signal_store_relaxed"));
        r.async_copy = reinterpret_cast<decltype(r.async_copy)>(dlsym(h, "hsa_amd_memory_async_copy"));
        r.pointer_info = reinterpret_cast<decltype(r.pointer_info)>(dlsym(h, "hsa_amd_pointer_info"));
        r.async_copy_on_engine =
            reinterpret_cast<decltype(r.async_copy_on_engine)>(dlsym(h, "hsa_amd_memory_async_copy_on_engine"));
        r.engine_status = reinterpret_cast<decltype(r.engine_status)>(dlsym(h, "hsa_amd_memory_copy_engine_status"));
        r.copy_prof_enable =
            reinterpret_cast<decltype(r.copy_prof_enable)>(dlsym(h, "hsa_amd_profiling_async_copy_enable"));
        r.copy_time = reinterpret_cast<decltype(r.copy_time)>(dlsym(h, "hsa_amd_profiling_get_async_copy_time"));
        r.system_info = reinterpret_cast<decltype(r.system_info)>(dlsym(h, "hsa_system_get_info"));
        r.ok = r.agent_get_info && r.signal_create && r.signal_destroy && r.signal_load && r.signal_store &&
               r.async_copy && r.pointer_info;
        return r;
    }();
    return a;
}

// Owner agent of an allocation known to the runtime, and its device type.
bool owner_of(const void* p, hsa_agent_t* agent, hsa_device_type_t* type)
{
    const HsaApi& a = api();
    hsa_amd_pointer_info_t info{};
    info.size = sizeof info;
    if (a.pointer_info(p, &info, nullptr, nullptr, nullptr) != HSA_STATUS_SUCCESS) return false;
    if (info.type != HSA_EXT_POINTER_TYPE_HSA || info.agentOwner.handle == 0) return false;
    if (a.agent_get_info(info.agentOwner, HSA_AGENT_INFO_DEVICE, type) != HSA_STATUS_SUCCESS) return false;
    *agent = info.agentOwner;
    return true;
}

}  // namespace

namespace oocs {

SdmaCopier::~SdmaCopier()
{
    if (!ready_) return;
    (void)drain();
    if (timing_) (void)api().copy_prof_enable(false);
    for (uint64_t s : sig_) api().signal_destroy(hsa_signal_t{s});
}

bool SdmaCopier::init(const void* dev, std::string* why)
{
    const HsaApi& a = api();
    if (!a.ok) {
        *why = "HSA runtime entry points not found in the process";
        return false;
    }
    hsa_agent_t g;
    hsa_device_type_t t;
    if (!owner_of(dev, &g, &t) || t != HSA_DEVICE_TYPE_GPU) {
        *why = "device allocation has no GPU owner agent";
        return false;
    }
    for (int i = 0; i < kRing; ++i) {
        hsa_signal_t s;
        if (a.signal_create(0, 0, nullptr, &s) != HSA_STATUS_SUCCESS) {
            for (uint64_t h : sig_) a.signal_destroy(hsa_signal_t{h});
            sig_.clear();
            *why = "hsa_signal_create failed";
            return false;
        }
        sig_.push_back(s.handle);
    }
    gpu_ = g.handle;
    ready_ = true;
    return true;
}

bool SdmaCopier::host_agent(const void* host, uint64_t* agent) const
{
    if (!ready_) return false;
    hsa_agent_t c;
    hsa_device_type_t t;
    if (!owner_of(host, &c, &t) || t != HSA_DEVICE_TYPE_CPU) return false;
    *agent = c.handle;
    return true;
}

int SdmaCopier::set_timing(bool on)
{
    if (!ready_) return fail(OOCS_E_STATE, "SDMA copier not initialised");
    const HsaApi& a = api();
    if (on && (!a.copy_prof_enable || !a.copy_time || !a.system_info))
        return fail(OOCS_E_HIP, "HSA copy timing entry points not found");
    if (on == timing_) {
        busy_ms_ = 0.0;
        return OOCS_OK;
    }
    const int rc = drain();  // copies in flight were issued under the old setting
    if (rc != OOCS_OK) return rc;
    if (on && tick_ms_ == 0.0) {
        uint64_t freq = 0;
        if (a.system_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &freq) != HSA_STATUS_SUCCESS || freq == 0)
            return fail(OOCS_E_HIP, "HSA timestamp frequency unavailable");
        tick_ms_ = 1e3 / (double)freq;
    }
    if (a.copy_prof_enable(on) != HSA_STATUS_SUCCESS) return fail(OOCS_E_HIP, "hsa_amd_profiling_async_copy_enable failed");
    timing_ = on;
    busy_ms_ = 0.0;
    return OOCS_OK;
}

int SdmaCopier::advance()
{
    const HsaApi& a = api();
    while (done_ < issued_) {
        const hsa_signal_t s{sig_[done_ % kRing]};
        const hsa_signal_value_t v = a.signal_load(s);
        if (v > 0) break;
        if (v < 0) return fail(OOCS_E_HIP, "SDMA device-to-host copy reported an error");
        if (timing_) {  // before the signal can be reused by a later copy
            hsa_amd_profiling_async_copy_time_t t{};
            if (a.copy_time(s, &t) == HSA_STATUS_SUCCESS && t.end >= t.start)
                busy_ms_ += (double)(t.end - t.start) * tick_ms_;
        }
        ++done_;
    }
    return OOCS_OK;
}

int SdmaCopier::wait(int64_t t)
{
    if (t > issued_) t = issued_;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0;; ++spin) {
        const int rc = advance();
        if (rc != OOCS_OK) return rc;
        if (done_ >= t) return OOCS_OK;
        __builtin_ia32_pause();
        if ((spin & 4095u) == 4095u &&
            std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
            return fail(OOCS_E_HIP, "SDMA device-to-host copy did not complete within a minute");
    }
}

int SdmaCopier::set_engines(int n)
{
    if (n < 1 || n > 16) return fail(OOCS_E_ARG, "engine count must be in [1, 16]");
    engines_ = n;
    mask_agent_ = 0;  // looked up again at the next copy
    return OOCS_OK;
}

// The engines a split copy to CPU agent `agent` uses: the first engines_
// of those the runtime reports available for this direction.
int SdmaCopier::engines_for(uint64_t agent)
{
    if (engines_ <= 1) return 1;
    if (mask_agent_ == agent) return (int)ids_.size();
    const HsaApi& a = api();
    ids_.clear();
    uint32_t mask = 0;
    if (a.async_copy_on_engine && a.engine_status &&
        a.engine_status(hsa_agent_t{agent}, hsa_agent_t{gpu_}, &mask) == HSA_STATUS_SUCCESS)
        for (int b = 0; b < 16 && (int)ids_.size() < engines_; ++b)
            if (mask & (1u << b)) ids_.push_back(1u << b);
    if (ids_.size() < 2) ids_.clear();  // fewer than two: the runtime's own choice
    mask_agent_ = agent;
    return ids_.empty() ? 1 : (int)ids_.size();
}

int SdmaCopier::copy(void* dst, uint64_t agent, const void* src, size_t bytes)
{
    if (!ready_) return fail(OOCS_E_STATE, "SDMA copier not initialised");
    const HsaApi& a = api();
    const int parts = engines_for(agent);
    // split on 4 KiB boundaries; every part is a copy of its own
    const size_t step = ((bytes + (size_t)parts - 1) / (size_t)parts + 4095) & ~(size_t)4095;
    for (int q = 0; q < parts; ++q) {
        const size_t off = (size_t)q * step;
        if (off >= bytes && q > 0) break;
        const size_t len = parts == 1 ? bytes : std::min(step, bytes - off);
        if (issued_ - done_ >= kRing) {
            const int rc = wait(issued_ - kRing + 1);
            if (rc != OOCS_OK) return rc;
        }
        const hsa_signal_t s{sig_[issued_ % kRing]};
        a.signal_store(s, 1);
        void* d = static_cast<char*>(dst) + off;
        const void* sp = static_cast<const char*>(src) + off;
        const hsa_status_t st =
            parts == 1 ? a.async_copy(d, hsa_agent_t{agent}, sp, hsa_agent_t{gpu_}, len, 0, nullptr, s)
                       : a.async_copy_on_engine(d, hsa_agent_t{agent}, sp, hsa_agent_t{gpu_}, len, 0, nullptr, s,
                                                (hsa_amd_sdma_engine_id_t)ids_[q], false);
        if (st != HSA_STATUS_SUCCESS) {
            a.signal_store(s, 0);
            return fail(OOCS_E_HIP, "HSA device-to-host copy failed (status " + std::to_string((int)st) + ")");
        }
        ++issued_;
    }
    return OOCS_OK;
}

}  // namespace oocs
