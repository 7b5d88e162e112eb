// plan.hpp -- out-of-core planner of liboocs (host only, no HIP calls).
//
// Geometry (Sec. III): nz planes split into nslabs blocks [a_i, a_{i+1});
// one residency advances a block k steps and needs h = r*k halo planes on
// each side. Region sharing: the 2h planes around a_{i+1} (the common
// region C_i) are brought in once, by block i, and reused by block i+1.
// Separate compression (Sec. V-A): R_i and C_i are independent chunks of
// the host store.
//
// Streaming: a residency never holds a whole block. It streams planes
// through the device in groups of G planes. Every time
// level of the residency has a ring of planes; a level advances at most G
// planes per tick, one radius behind the level it reads, so that all jobs
// of a tick (decode the next input group, one z-range of every level,
// encode the next finished output group) are independent and run as one
// launch. Rings are sized exactly by a liveness sweep over the tick list,
// and G is the largest that lets rings plus staging fit the caller's arena.
#pragma once
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "oocs.h"

namespace oocs {

struct LevelRange {
    int32_t lv;         // ring written (computed level, or the output ring of fused levels)
    int64_t z0, z1;
    int32_t steps = 1;  // time steps from ring lv-1 to ring lv (fused levels: the residency length)
};

struct Tick {
    int32_t block = 0;
    int64_t in_group = -1;  // decoded this tick (all input fields), or -1
    int64_t dz0 = 0, dz1 = 0;
    std::vector<LevelRange> levels;
    int64_t out_group = -1;  // encoded this tick (all output fields), or -1
    int64_t ez0 = 0, ez1 = 0;
    int32_t out_block = 0;   // block the encoded group starts in
    bool last_out_of_block = false;  // the group completes the write-back of blocks done_b0..done_b1
    int32_t done_b0 = 0, done_b1 = -1;
};

struct GroupRec {
    int64_t z0, z1;
    int64_t tick;
    int32_t block;
    bool last_of_block;
};

struct Schedule {
    std::vector<Tick> ticks;
    std::vector<GroupRec> in_groups, out_groups;
    std::vector<oocs_op> ops;
};

class Planner {
public:
    // Validates cfg, derives geometry. Returns OOCS_OK or an error (message in err).
    int init(const oocs_config& cfg, std::string& err);
    // Lays out rings and staging for group size G; returns bytes needed, or -1 on a stall.
    int64_t layout(int64_t G, int nstage, std::string& err);
    // Picks G (cfg.group or the largest fitting arena_bytes) and fixes the layout.
    int choose(size_t arena_bytes, std::string& err);
    // Tick list for a residency of kr steps with the current G; variant:
    // OOCS_SCHED_* bits (snake plans).
    int build_ticks(int kr, int variant, Schedule& s, std::string& err) const;
    // Full operation list for kr steps and a variant (cached).
    const Schedule* schedule(int kr, std::string& err, int variant = 0);
    // Variant of residency i of R in one run (0 unless snake).
    int variant_of(int64_t i, int64_t R) const;

    // geometry
    oocs_config cfg{};
    int64_t nx = 0, ny = 0, nz = 0;
    int r = 1;         // stencil radius
    int nin = 1;       // input time levels (1 heat, 2 wave)
    bool has_ro = false;
    int n = 1;         // slabs
    int k = 1;
    bool restart = false;    // every block restarts the level fronts (halo recomputed)
    bool copy_engines = true;   // loads by hipMemcpyAsync on a copy stream (else by the kernel)
    bool kernel_stores = false; // with copy_engines: write-back by STORE jobs in the launches (else by D2H copies)
    bool fused = false;         // heat: one temporally blocked job per tick computes all k levels
    bool resident_ro = false;   // wave: the read-only field stays decoded in an nz-plane ring
    bool snake = false;         // alternating sweeps; the last block of a residency stays on the device
    bool midpoint = false;      // every decode with mid-point reconstruction
    bool ro_dev = false;        // wave: the read-only store copied once into the arena
    int64_t ro_dev_off = -1;    // its offset there
    bool fp64 = false;          // FP64 fields (wave): 8-byte values, the FP64 format
    int esize = 4;              // bytes per value
    int64_t X = 0;              // snake: planes of the retained region (whole slabs)
    bool retain_max = false;    // snake: X grown to what the arena holds
    static constexpr int kMaxFusedSteps = 4;
    int64_t slab = 0, h = 0;
    std::vector<int64_t> a;  // n+1 block bounds

    // fields
    int nfields = 1;
    std::vector<int> in_fields, out_fields;  // field slots streamed in / written back
    int in_ring(int f) const;                // ring a field is decoded into
    int out_ring(int f, int kr) const;       // ring an output field is encoded from
    int ro_ring() const { return nin + k; }
    int nrings() const { return fused ? 2 : nin + k + (has_ro ? 1 : 0); }
    int64_t plane_elems() const { return nx * ny; }
    int64_t plane_bytes() const { return nx * ny * esize; }
    int64_t ring_ld() const { return nx * ny * (esize / 4); }  // plane stride of a ring, in floats
    int64_t store_plane_bytes(int f) const;  // host-store bytes per plane of field f (compressed or raw)
    int64_t store_bytes(int f) const;

    // layout (valid after choose)
    int64_t G = 0;
    int nstage = 3;
    std::vector<int64_t> ringW, ringOff;
    int64_t in_slot_bytes[OOCS_MAX_FIELDS] = {0, 0, 0}, in_off[OOCS_MAX_FIELDS] = {0, 0, 0};
    int64_t out_slot_bytes[OOCS_MAX_FIELDS] = {0, 0, 0}, out_off[OOCS_MAX_FIELDS] = {0, 0, 0};
    int64_t ret_off[OOCS_MAX_FIELDS] = {0, 0, 0};  // snake: retained block of each read-write field
    // First plane of the retained region a decode (encode = false) or an
    // encode of a residency with schedule variant `variant` addresses: a
    // residency decodes the region it starts with (the bottom X planes when
    // it runs upward, the top X downward) and encodes the one it ends with;
    // the buffer holds plane z of a region at z - base. With X > nz / 2 the
    // regions overlap and a plane of both is encoded to another place than
    // the one it was decoded from, later in the residency than any decode
    // of what that place held (the output front trails the input front).
    int64_t ret_base(bool encode, int variant) const
    {
        return encode != ((variant & OOCS_SCHED_MIRROR) != 0) ? nz - X : 0;
    }
    int64_t arena_needed = 0;
    // wave source: amplitudes of up to kSrcTable steps and the device step counter
    static constexpr int64_t kSrcTable = 65536;
    int64_t src_table_off = -1, step_ctr_off = -1;

    // event ids used by the op lists
    int ev_loaded(int s) const { return s; }
    int ev_decoded(int s) const { return nstage + s; }
    int ev_encoded(int s) const { return 2 * nstage + s; }
    int ev_stored(int s) const { return 3 * nstage + s; }
    int ev_blk_cur(int i) const { return 4 * nstage + i; }
    int ev_blk_prev(int i) const { return 4 * nstage + n + i; }
    int nevents_logical() const { return 4 * nstage + 2 * n; }

private:
    int emit_ops(int kr, int variant, Schedule& s, std::string& err) const;
    template <class MakeOp>
    int emit_direct(int kr, Schedule& s, MakeOp op) const;
    std::map<int, Schedule> cache_;
};

}  // namespace oocs
