// sdma.hpp -- device-to-host copies on the GPU's system DMA (SDMA) engines,
// issued through the HSA runtime that the process's HIP runtime has loaded.
//
// hipMemcpyAsync may carry out a device-to-host copy as a blit kernel, which
// then holds compute units beside the pipeline kernel (the HIP runtime that
// ships with PyTorch does so for every such copy). An HSA asynchronous copy
// between a GPU agent and a CPU agent runs on an SDMA engine and leaves the
// compute units to the kernels. Completion is reported through HSA signals
// that the host polls, so the executor uses these copies only where it
// already honours cross-stream dependencies on the host.
//
// Copies are numbered in issue order; a ticket t stands for "every copy
// issued before the t-th has completed". Signals live in a ring; completion
// is tracked as a prefix, so a copy that completes early is counted once all
// earlier ones have.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace oocs {

class SdmaCopier {
public:
    SdmaCopier() = default;
    SdmaCopier(const SdmaCopier&) = delete;
    SdmaCopier& operator=(const SdmaCopier&) = delete;
    ~SdmaCopier();

    // Binds to the loaded HSA runtime and to the GPU agent that owns the
    // device allocation `dev`; creates the completion signals. False (with
    // the reason in *why) if the runtime, its entry points or the agent are
    // not available; the object then stays unusable.
    bool init(const void* dev, std::string* why);
    bool ready() const { return ready_; }

    // The CPU agent owning the pinned host allocation that contains `host`,
    // as an opaque handle; false if the HSA runtime does not know the pointer
    // as memory of a CPU pool (pageable memory, for one).
    bool host_agent(const void* host, uint64_t* agent) const;

    // Issue a copy of `bytes` from device memory `src` to host memory `dst`
    // (owned by CPU agent `agent`). The source must have been released to
    // system scope by the time this is called (a completed HIP event does
    // that). Blocks only while the signal ring is full. OOCS_OK or OOCS_E_HIP.
    int copy(void* dst, uint64_t agent, const void* src, size_t bytes);

    // Split every later copy into n parts (on 4 KiB boundaries), each on
    // an engine of its own (hsa_amd_memory_async_copy_on_engine), where the
    // runtime reports n engines available for the direction (else as many
    // as it has; with fewer than two, the runtime's own choice). n = 1: one
    // copy on the engine the runtime picks (the default). Each part counts
    // as a copy for issued() and wait(). OOCS_OK or OOCS_E_ARG.
    int set_engines(int n);
    int engines() const { return engines_; }

    int64_t issued() const { return issued_; }
    // Copy timing (off by default): while on, the engine timestamps every
    // copy (hsa_amd_profiling_async_copy_enable, process-wide) and the
    // summed start-to-end durations of the copies seen completing are
    // accumulated. Turning it on resets the sum. OOCS_OK or OOCS_E_HIP.
    int set_timing(bool on);
    double busy_ms() const { return busy_ms_; }
    // Block until the first t copies have completed. OOCS_OK, or OOCS_E_HIP
    // on a copy error or after a minute without completion.
    int wait(int64_t t);
    int drain() { return wait(issued_); }

private:
    int advance();  // moves done_ over completed copies
    int engines_for(uint64_t agent);  // parts of a copy to that CPU agent (fills ids_)

    static constexpr int kRing = 64;
    bool ready_ = false;
    bool timing_ = false;
    double busy_ms_ = 0.0;
    double tick_ms_ = 0.0;  // milliseconds per HSA system timestamp tick
    uint64_t gpu_ = 0;
    std::vector<uint64_t> sig_;
    int64_t issued_ = 0, done_ = 0;
    int engines_ = 1;
    uint64_t mask_agent_ = 0;   // CPU agent ids_ was looked up for
    std::vector<uint32_t> ids_; // engine ids of a split copy
};

}  // namespace oocs
