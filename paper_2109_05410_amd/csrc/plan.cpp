// plan.cpp -- out-of-core planner of liboocs (host only, no HIP calls).
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <climits>
#include <cstdio>
#include <deque>

namespace oocs {

namespace {
std::string fmt(const char* f, long long a = 0, long long b = 0, long long c = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
}  // namespace

int Planner::init(const oocs_config& c, std::string& err)
{
    cfg = c;
    nx = c.nx; ny = c.ny; nz = c.nz;
    if (nx <= 0 || ny <= 0 || nz <= 0) { err = "grid dimensions must be positive"; return OOCS_E_ARG; }
    if (nx % 4 || ny % 4) { err = "nx and ny must be multiples of 4"; return OOCS_E_ALIGN; }
    if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) { err = "grid dimension too large"; return OOCS_E_ARG; }
    if (c.stencil == OOCS_HEAT7) {
        r = 1; nin = 1; has_ro = false; nfields = 1;
        in_fields = {0}; out_fields = {0};
    } else if (c.stencil == OOCS_WAVE25) {
        r = 4; nin = 2; has_ro = true; nfields = 3;
        in_fields = {0, 1, 2}; out_fields = {0, 1};
    } else {
        err = "unknown stencil"; return OOCS_E_ARG;
    }
    n = c.nslabs; k = c.k;
    if (n < 1 || nz % n) { err = fmt("nslabs (%lld) must be >= 1 and divide nz (%lld)", n, nz); return OOCS_E_ARG; }
    if (k < 1 || k > 16) { err = fmt("k (%lld) must be in [1, 16]", k); return OOCS_E_ARG; }
    slab = nz / n;
    h = (int64_t)r * k;
    if (2 * h > slab && n > 1) { err = fmt("halo 2h = %lld exceeds the slab thickness %lld", 2 * h, slab); return OOCS_E_HALO; }
    fp64 = (c.flags & OOCS_PLAN_FP64) != 0;
    if (fp64 && c.stencil != OOCS_WAVE25) { err = "FP64 plans are for the wave stencil"; return OOCS_E_ARG; }
    if (fp64 && (c.flags & OOCS_PLAN_MIDPOINT)) { err = "mid-point decoding is not available in FP64"; return OOCS_E_ARG; }
    if (fp64 && (c.flags & (OOCS_PLAN_KERNEL_TRANSFERS | OOCS_PLAN_KERNEL_STORES))) {
        err = "FP64 plans move data with the copy engines (no transfer jobs)";
        return OOCS_E_ARG;
    }
    esize = fp64 ? 8 : 4;
    if (c.stencil == OOCS_WAVE25 && nx * ny * esize >= ((int64_t)1 << 32)) {
        err = "a plane of the wave must hold less than 4 GiB";  // the wave tile addresses a plane with 32-bit offsets
        return OOCS_E_ARG;
    }
    const int max_rate = fp64 ? OOCS_MAX_RATE64 : OOCS_MAX_RATE;
    bool any_rate = false;
    for (int f = 0; f < nfields; ++f) {
        if (c.rate[f] < 0 || c.rate[f] > max_rate) {
            err = fmt("rate[%lld] = %lld outside [0, %lld]", f, c.rate[f], max_rate);
            return OOCS_E_RATE;
        }
        any_rate |= c.rate[f] > 0;
    }
    for (int f = nfields; f < OOCS_MAX_FIELDS; ++f)
        if (c.rate[f] != 0) { err = "rate set for a field slot the stencil does not use"; return OOCS_E_ARG; }
    if (any_rate && (nz % 4 || slab % 4 || h % 4)) {
        err = fmt("compressed chunks need nz (%lld), the slab (%lld) and h (%lld) to be multiples of 4", nz, slab, h);
        return OOCS_E_ALIGN;
    }
    if (c.group < 0 || (c.group > 0 && any_rate && c.group % 4)) { err = "group must be a positive multiple of 4"; return OOCS_E_ALIGN; }
    if (c.nstage != 0 && (c.nstage < 2 || c.nstage > 16)) { err = "nstage must be 0 or in [2, 16]"; return OOCS_E_ARG; }
    if (c.flags & ~(OOCS_PLAN_BLOCK_RESTART | OOCS_PLAN_KERNEL_TRANSFERS | OOCS_PLAN_LEVEL_BY_LEVEL |
                    OOCS_PLAN_KERNEL_STORES | OOCS_PLAN_RESIDENT_RO | OOCS_PLAN_SNAKE | OOCS_PLAN_MIDPOINT |
                    OOCS_PLAN_FP64 | OOCS_PLAN_RO_DEVICE_STORE)) {
        err = "unknown plan flags";
        return OOCS_E_ARG;
    }
    restart = (c.flags & OOCS_PLAN_BLOCK_RESTART) != 0;
    fused = c.stencil == OOCS_HEAT7 && k <= kMaxFusedSteps && !restart && !(c.flags & OOCS_PLAN_LEVEL_BY_LEVEL);
    copy_engines = (c.flags & OOCS_PLAN_KERNEL_TRANSFERS) == 0;
    kernel_stores = copy_engines && (c.flags & OOCS_PLAN_KERNEL_STORES) != 0;
    resident_ro = (c.flags & OOCS_PLAN_RESIDENT_RO) != 0;
    if (resident_ro && !has_ro) { err = "a resident read-only field needs the wave stencil"; return OOCS_E_ARG; }
    if (resident_ro) in_fields = {0, 1};  // the read-only field is loaded once, outside the residencies
    ro_dev = (c.flags & OOCS_PLAN_RO_DEVICE_STORE) != 0;
    if (ro_dev && (!has_ro || resident_ro || !copy_engines)) {
        err = "a device-held read-only store needs the wave stencil, copy-engine transfers and no resident read-only field";
        return OOCS_E_ARG;
    }
    snake = (c.flags & OOCS_PLAN_SNAKE) != 0;
    if (snake && (!copy_engines || kernel_stores || restart || n < 2)) {
        err = "snake sweeps need copy-engine transfers, shared levels and at least two slabs";
        return OOCS_E_ARG;
    }
    // retained region: whole slabs, up to the whole grid
    if (!snake && c.retain != 0) { err = "retain needs a snake plan"; return OOCS_E_ARG; }
    retain_max = snake && c.retain == OOCS_RETAIN_MAX;
    if (snake && !retain_max && (c.retain < 0 || c.retain > n)) {
        err = fmt("retain (%lld) must be 0, OOCS_RETAIN_MAX or in [1, nslabs = %lld]", c.retain, n);
        return OOCS_E_ARG;
    }
    X = snake ? slab * (retain_max ? 1 : std::max(1, (int)c.retain)) : 0;
    midpoint = (c.flags & OOCS_PLAN_MIDPOINT) != 0;
    // kernel-driven transfers fetch one group ahead inside the launch: two slots suffice;
    // copy engines keep three groups in flight ahead of the decode
    nstage = c.nstage ? c.nstage : (copy_engines ? 4 : 2);
    a.resize(n + 1);
    for (int i = 0; i <= n; ++i) a[i] = (int64_t)i * slab;
    return OOCS_OK;
}

int Planner::in_ring(int f) const
{
    if (cfg.stencil == OOCS_HEAT7) return 0;
    return f == 0 ? 1 : (f == 1 ? 0 : ro_ring());
}

int Planner::out_ring(int f, int kr) const
{
    if (fused) return 1;                          // u(t+kr), the fused job's output ring
    if (cfg.stencil == OOCS_HEAT7) return kr;     // u(t+kr)
    return f == 0 ? kr + 1 : kr;                  // p(t+kr), p(t+kr-1)
}

int64_t Planner::store_plane_bytes(int f) const
{
    const int rate = cfg.rate[f];
    if (rate == 0) return plane_bytes();
    return (nx / 4) * (ny / 4) * (int64_t)rate * 8 / 4;  // one 4-plane layer / 4
}

int64_t Planner::store_bytes(int f) const
{
    if (f < 0 || f >= nfields) return 0;
    return store_plane_bytes(f) * nz;
}

int Planner::build_ticks(int kr, int variant, Schedule& s, std::string& err) const
{
    s.ticks.clear(); s.in_groups.clear(); s.out_groups.clear();
    // Snake variants: in pass order (z upward; a downward pass is built upward
    // and mirrored at the end) the first X planes of the input may come from
    // the retained buffer and the last X planes of the output may go to it,
    // so no group crosses those boundaries.
    const int64_t cut_in = (variant & OOCS_SCHED_RETAIN_IN) ? X : -1;
    const int64_t cut_out = (variant & OOCS_SCHED_RETAIN_OUT) ? nz - X : -1;
    const int nl = nin + kr;  // levels in use: 0 .. nl-1
    std::vector<int64_t> f(nl), lo(nl), hi(nl);
    int64_t load_front = 0;
    const int64_t align = 4;
    auto block_of = [&](int64_t z) { return (int)std::min<int64_t>(z / slab, n - 1); };
    // A pass streams the z-range [p0, p1) through all levels. With block
    // restarts every block is one pass over its extended range (levels
    // shrink by r per step inside [a_i - h, a_{i+1} + h)); with shared
    // levels the whole grid is one pass and every plane of every level is
    // computed once, the halo planes of a block being those its neighbour
    // already computed.
    const int npass = restart ? n : 1;
    for (int pi = 0; pi < npass; ++pi) {
        const int64_t p0 = restart ? a[pi] : 0;
        const int64_t p1 = restart ? a[pi + 1] : nz;
        const int64_t e_end = restart ? std::min(a[pi + 1] + h, nz) : nz;
        for (int lv = nin; lv < nl; ++lv) {
            const int64_t st = lv - nin + 1;
            lo[lv] = restart ? std::max<int64_t>(a[pi] - h + st * r, 0) : 0;
            hi[lv] = restart ? std::min<int64_t>(a[pi + 1] + h - st * r, nz) : nz;
            f[lv] = lo[lv];
        }
        if (fused) f[1] = 0;  // front of the fused output ring
        int64_t out_front = p0;
        int guard = 0;
        while (out_front < p1) {
            if (++guard > 1000000) { err = "schedule does not terminate"; return OOCS_E_STATE; }
            Tick t;
            t.block = restart ? pi : block_of(std::min(load_front, nz - 1));
            std::vector<int64_t> prev = f;
            for (int lv = 0; lv < nin; ++lv) prev[lv] = load_front;
            // decode the next input group
            if (load_front < e_end) {
                t.in_group = (int64_t)s.in_groups.size();
                t.dz0 = load_front;
                t.dz1 = std::min(load_front + G, e_end);
                if (load_front < cut_in) t.dz1 = std::min(t.dz1, cut_in);
                s.in_groups.push_back({t.dz0, t.dz1, (int64_t)s.ticks.size(), restart ? pi : block_of(t.dz0), false});
                load_front = t.dz1;
            }
            // fused levels: the output ring advances to where its inputs
            // [z - kr, z + kr] were decoded by the previous tick
            if (fused) {
                const int64_t avail = prev[0] >= nz ? nz : prev[0] - (int64_t)r * kr;
                const int64_t top = std::min(avail, prev[1] + G);
                if (top > prev[1]) {
                    LevelRange L;
                    L.lv = 1; L.z0 = prev[1]; L.z1 = top; L.steps = kr;
                    t.levels.push_back(L);
                    f[1] = top;
                }
            }
            // advance every computed level from the previous tick's fronts
            for (int lv = nin; lv < nl && !fused; ++lv) {
                const int64_t below = prev[lv - 1];
                const int64_t avail = below >= nz ? nz : below - r;
                int64_t top = std::min(std::min(hi[lv], avail), prev[lv] + G);
                if (lv >= 2) top = std::min(top, prev[lv - 2]);
                if (top > prev[lv]) {
                    t.levels.push_back({lv, prev[lv], top});
                    f[lv] = top;
                }
            }
            // encode the next finished output group: with block restarts never
            // across the pass's end; with shared levels any 4-aligned run (a
            // group may complete the write-back of a block and start the next)
            int64_t fo = nz;
            for (int fld : out_fields) {
                const int lv = out_ring(fld, kr);
                fo = std::min(fo, lv < nin ? prev[0] : prev[lv]);
            }
            const int ob = block_of(out_front);
            const int64_t bend = restart ? a[ob + 1] : nz;
            int64_t e = fo >= bend ? bend : out_front + (fo - out_front) / align * align;
            e = std::min(e, out_front + G);
            if (out_front < cut_out) e = std::min(e, cut_out);
            if (e > out_front) {
                t.out_group = (int64_t)s.out_groups.size();
                t.ez0 = out_front;
                t.ez1 = e;
                t.out_block = ob;
                // blocks whose last plane this group writes back
                t.done_b0 = block_of(out_front);
                t.done_b1 = -1;
                for (int b = t.done_b0; b < n; ++b)
                    if (a[b + 1] > out_front && a[b + 1] <= e) t.done_b1 = b;
                if (t.done_b1 < 0) t.done_b0 = 0;
                else
                    while (a[t.done_b0 + 1] <= out_front) ++t.done_b0;
                t.last_out_of_block = t.done_b1 >= 0;
                s.out_groups.push_back({out_front, e, (int64_t)s.ticks.size(), ob, t.last_out_of_block});
                out_front = e;
            }
            if (t.in_group < 0 && t.levels.empty() && t.out_group < 0) {
                err = fmt("schedule stalled in pass %lld", pi);
                return OOCS_E_STATE;
            }
            s.ticks.push_back(std::move(t));
        }
    }
    if (variant & OOCS_SCHED_MIRROR) {
        // plane z of the upward pass is plane nz - 1 - z, block b is block
        // n - 1 - b (the slabs are equal, so the mirrored slabs are slabs)
        auto mz = [&](int64_t& z0, int64_t& z1) { const int64_t t0 = z0; z0 = nz - z1; z1 = nz - t0; };
        auto mb = [&](int32_t b) { return (int32_t)(n - 1 - b); };
        for (Tick& t : s.ticks) {
            t.block = mb(t.block);
            if (t.in_group >= 0) mz(t.dz0, t.dz1);
            for (LevelRange& L : t.levels) mz(L.z0, L.z1);
            if (t.out_group >= 0) {
                mz(t.ez0, t.ez1);
                t.out_block = mb(t.out_block);
                if (t.done_b1 >= 0) {
                    const int32_t b0 = mb(t.done_b1), b1 = mb(t.done_b0);
                    t.done_b0 = b0;
                    t.done_b1 = b1;
                }
            }
        }
        for (GroupRec& g : s.in_groups) { mz(g.z0, g.z1); g.block = mb(g.block); }
        for (GroupRec& g : s.out_groups) { mz(g.z0, g.z1); g.block = mb(g.block); }
    }
    return OOCS_OK;
}

int Planner::variant_of(int64_t i, int64_t R) const
{
    if (!snake) return 0;
    return ((i & 1) ? OOCS_SCHED_MIRROR : 0) | (i > 0 ? OOCS_SCHED_RETAIN_IN : 0) |
           (i < R - 1 ? OOCS_SCHED_RETAIN_OUT : 0);
}

int64_t Planner::layout(int64_t Gc, int ns, std::string& err)
{
    G = Gc;
    nstage = ns;
    const int R = nrings();
    std::vector<int64_t> W(R, 1);
    // Size every ring by a liveness sweep over the tick lists of all
    // residency lengths 1..k (the last residency may be shorter).
    // Snake plans: also every retain variant (mirroring keeps every span).
    std::vector<int> variants{0};
    if (snake) variants = {0, OOCS_SCHED_RETAIN_IN, OOCS_SCHED_RETAIN_OUT, OOCS_SCHED_RETAIN_IN | OOCS_SCHED_RETAIN_OUT};
    for (int vi = 0; vi < (int)variants.size() * k; ++vi) {
        const int kr = vi % k + 1, variant = variants[vi / k];
        Schedule s;
        if (build_ticks(kr, variant, s, err) != OOCS_OK) return -1;
        const int64_t T = (int64_t)s.ticks.size();
        // per ring: current version of each plane -> (write tick, last read tick)
        struct Live { int64_t w = -1, rd = -1; };
        std::vector<std::vector<Live>> cur(R, std::vector<Live>(nz));
        std::vector<std::vector<std::pair<int64_t, int64_t>>> spans_lo(R), spans_hi(R);
        // intervals (z, tw, tr) collected per ring
        std::vector<std::vector<std::array<int64_t, 3>>> iv(R);
        auto close = [&](int ring, int64_t z) {
            Live& L = cur[ring][z];
            if (L.w >= 0) iv[ring].push_back({z, L.w, std::max(L.w, L.rd)});
            L = Live{};
        };
        bool bad = false;
        auto write = [&](int ring, int64_t z0, int64_t z1, int64_t tick) {
            for (int64_t z = z0; z < z1; ++z) {
                if (cur[ring][z].rd >= tick) bad = true;  // a plane may not be rewritten while still read
                close(ring, z);
                cur[ring][z].w = tick;
            }
        };
        auto read = [&](int ring, int64_t z0, int64_t z1, int64_t tick) {
            for (int64_t z = std::max<int64_t>(z0, 0); z < std::min(z1, nz); ++z) {
                Live& L = cur[ring][z];
                if (L.w < 0 || L.w >= tick) bad = true;  // must be written by an earlier tick
                L.rd = std::max(L.rd, tick);
            }
        };
        for (int64_t ti = 0; ti < T; ++ti) {
            const Tick& t = s.ticks[ti];
            for (const LevelRange& L : t.levels) {
                read(L.lv - 1, L.z0 - (int64_t)r * L.steps, L.z1 + (int64_t)r * L.steps, ti);
                if (nin == 2) {
                    read(L.lv - 2, L.z0, L.z1, ti);
                    if (!resident_ro) read(ro_ring(), L.z0, L.z1, ti);
                }
            }
            if (t.out_group >= 0)
                for (int fld : out_fields) read(out_ring(fld, kr), t.ez0, t.ez1, ti);
            if (t.in_group >= 0)
                for (int fld : in_fields) write(in_ring(fld), t.dz0, t.dz1, ti);
            for (const LevelRange& L : t.levels) write(L.lv, L.z0, L.z1, ti);
        }
        if (bad) { err = "schedule reads a plane before it is written, or rewrites it while read"; return -1; }
        for (int ring = 0; ring < R; ++ring)
            for (int64_t z = 0; z < nz; ++z) close(ring, z);
        // W = max over ticks of the span of planes live at that tick
        for (int ring = 0; ring < R; ++ring) {
            std::vector<int64_t> mn(T, INT64_MAX), mx(T, INT64_MIN);
            for (const auto& v : iv[ring])
                for (int64_t ti = v[1]; ti <= v[2]; ++ti) {
                    mn[ti] = std::min(mn[ti], v[0]);
                    mx[ti] = std::max(mx[ti], v[0]);
                }
            for (int64_t ti = 0; ti < T; ++ti)
                if (mx[ti] >= mn[ti]) W[ring] = std::max(W[ring], mx[ti] - mn[ti] + 1);
        }
    }
    if (resident_ro) W[ro_ring()] = nz;  // the whole decoded field
    ringW = W;
    ringOff.assign(R, 0);
    const int64_t pb = plane_bytes();
    int64_t off = 0;
    for (int ring = 0; ring < R; ++ring) {
        ringOff[ring] = off;
        off = align_up(off + W[ring] * pb, 256);
    }
    for (int f = 0; f < OOCS_MAX_FIELDS; ++f) { in_slot_bytes[f] = out_slot_bytes[f] = in_off[f] = out_off[f] = 0; }
    for (int fld : in_fields) {
        if (ro_dev && fld == 2) continue;  // decoded from the device copy of its store
        in_slot_bytes[fld] = align_up(G * store_plane_bytes(fld), 256);
        in_off[fld] = off;
        off += in_slot_bytes[fld] * nstage;
    }
    ro_dev_off = -1;
    if (ro_dev) {
        ro_dev_off = off;
        off = align_up(off + store_bytes(2), 256);
    }
    if (resident_ro) {  // one slot to load the read-only field group by group
        in_slot_bytes[2] = align_up(G * store_plane_bytes(2), 256);
        in_off[2] = off;
        off += in_slot_bytes[2];
    }
    for (int fld : out_fields) {
        out_slot_bytes[fld] = align_up(G * store_plane_bytes(fld), 256);
        out_off[fld] = off;
        off += out_slot_bytes[fld] * nstage;
    }
    for (int fld : out_fields) {
        ret_off[fld] = off;
        if (snake) off = align_up(off + X * store_plane_bytes(fld), 256);
    }
    src_table_off = step_ctr_off = -1;
    if (cfg.stencil == OOCS_WAVE25) {
        src_table_off = off;
        off += kSrcTable * 4;
        step_ctr_off = off;
        off += 256;
    }
    arena_needed = off;
    return off;
}

int Planner::choose(size_t arena_bytes, std::string& err)
{
    bool any_rate = false;
    for (int f = 0; f < nfields; ++f) any_rate |= cfg.rate[f] > 0;
    std::vector<int64_t> cands;
    if (cfg.group > 0) {
        cands.push_back(cfg.group);
    } else {
        // the wave's levels read 9 planes of p and write one ring each, so its
        // ticks are long already at 16 planes: larger groups only delay the
        // first transfers of a residency (1024^3 at 12 bits in 8 GiB: groups
        // of 8-16 planes ran 4-7 % faster than 20-24)
        const int64_t gmax = cfg.stencil == OOCS_WAVE25 ? 16 : 32;
        for (int64_t g = gmax; g >= 4; g -= 4) cands.push_back(g);
        if (!any_rate) { cands.push_back(2); cands.push_back(1); }
    }
    // staging depth: the caller's, else 4 then 3 slots for copy engines (a larger
    // group is worth more than a deeper queue), 2 for kernel transfers
    std::vector<int> depths;
    if (cfg.nstage) depths = {cfg.nstage};
    else if (copy_engines) depths = {4, 3};
    else depths = {2};
    int64_t best_need = -1;
    for (int64_t g : cands)
        for (int ns : depths) {
            const int64_t need = layout(g, ns, err);
            if (need < 0) return OOCS_E_STATE;
            if (best_need < 0 || need < best_need) best_need = need;
            if ((size_t)need <= arena_bytes) {
                // OOCS_RETAIN_MAX: grow the retained region slab by slab in the
                // room the pipeline leaves (it comes after G: a smaller group
                // for a larger region slows every tick)
                while (retain_max && X + slab <= nz) {
                    X += slab;
                    std::string e2;
                    const int64_t more = layout(g, ns, e2);
                    if (more < 0 || (size_t)more > arena_bytes) {  // does not fit (or cannot be scheduled)
                        X -= slab;
                        if (layout(g, ns, err) < 0) return OOCS_E_STATE;
                        break;
                    }
                }
                cache_.clear();
                return OOCS_OK;
            }
        }
    err = fmt("the pipeline needs at least %lld bytes of device arena, %lld given", best_need, (long long)arena_bytes);
    return OOCS_E_CAP;
}

int Planner::emit_ops(int kr, int variant, Schedule& s, std::string& err) const
{
    s.ops.clear();
    auto op = [&](int kind, int stream) {
        oocs_op o{};
        o.kind = kind; o.stream = stream; o.event = -1; o.slot = -1; o.field = -1; o.level = -1; o.block = -1; o.tick = -1;
        return o;
    };
    if (!copy_engines) return emit_direct(kr, s, op);
    auto block_of = [&](int64_t z) { return (int)std::min<int64_t>(z / slab, n - 1); };
    // Snake variants: the retained regions in real z. The residency takes its
    // first X planes (pass order) from the retained buffer and leaves its
    // last X planes there; a downward pass starts at the top.
    const bool mirror = (variant & OOCS_SCHED_MIRROR) != 0;
    const bool ret_in = (variant & OOCS_SCHED_RETAIN_IN) != 0, ret_out = (variant & OOCS_SCHED_RETAIN_OUT) != 0;
    auto in_retained = [&](int64_t z0, int64_t z1) {
        return ret_in && (mirror ? z0 >= nz - X : z1 <= X);
    };
    auto out_retained = [&](int64_t z0, int64_t z1) {
        return ret_out && (mirror ? z1 <= X : z0 >= nz - X);
    };
    // fields a group's load copies: all streamed inputs, or only the
    // read-only one when the read-write ones are retained
    auto loaded_fields = [&](const GroupRec& g) {
        std::vector<int> f;
        for (int fld : in_fields)
            if ((!in_retained(g.z0, g.z1) || fld == 2) && !(ro_dev && fld == 2)) f.push_back(fld);
        return f;
    };
    auto emit_h2d = [&](int64_t j, int64_t tick, std::vector<oocs_op>& out) {
        const GroupRec& g = s.in_groups[j];
        const int sl = (int)(j % nstage);
        const std::vector<int> flds = loaded_fields(g);
        if (flds.empty()) return;
        oocs_op w = op(OOCS_OP_WAIT, 0); w.event = ev_decoded(sl); w.tick = (int)tick; out.push_back(w);
        // host planes were last written by the previous residency's write-back
        // (the read-only store never is); with snake sweeps the previous
        // residency may have run the other way, so every block of the group
        if (!in_retained(g.z0, g.z1))
            for (int b = snake ? block_of(g.z0) : block_of(g.z1 - 1); b <= block_of(g.z1 - 1); ++b) {
                oocs_op w2 = op(OOCS_OP_WAIT, 0); w2.event = ev_blk_prev(b); w2.tick = (int)tick; out.push_back(w2);
            }
        for (int fld : flds) {
            oocs_op c = op(OOCS_OP_H2D, 0);
            c.field = fld; c.slot = sl; c.z0 = g.z0; c.z1 = g.z1; c.block = g.block; c.tick = (int)tick;
            c.level = in_ring(fld);
            out.push_back(c);
        }
        oocs_op rcd = op(OOCS_OP_RECORD, 0); rcd.event = ev_loaded(sl); rcd.tick = (int)tick; out.push_back(rcd);
    };
    const int64_t nin_groups = (int64_t)s.in_groups.size();
    for (int64_t j = 0; j < std::min<int64_t>(nstage, nin_groups); ++j) emit_h2d(j, -1, s.ops);
    // The copies a tick makes possible (write-back of its output group, load
    // of the group that reuses its input slot) are issued after the next
    // tick's launch, so the host issues that launch before it can block on
    // the events those copies wait for; the load of group j + nstage is then
    // issued nstage - 1 ticks before its decode. (Two ticks later measured
    // slower and unsteady: some runs lost a third of their throughput.)
    // lag < nstage keeps every wait on the record it was meant for (a slot is
    // recorded again only nstage ticks later).
    const int lag = 1;
    std::deque<std::vector<oocs_op>> lagged;
    std::vector<oocs_op> next;
    // with kernel stores: the STORE job of the previous tick's output group
    // rides in this tick's launch, and the block events it completes are
    // recorded on the compute stream after it
    int64_t pend_store = -1;
    auto emit_store = [&](int64_t m, int tick) {
        const GroupRec& g = s.out_groups[m];
        for (int fld : out_fields) {
            oocs_op c = op(OOCS_OP_STORE, 1);
            c.field = fld; c.slot = (int)(m % nstage); c.z0 = g.z0; c.z1 = g.z1; c.block = g.block; c.tick = tick;
            c.level = out_ring(fld, kr);
            s.ops.push_back(c);
        }
    };
    auto record_blocks_of = [&](int64_t m, int tick) {
        const Tick& tm = s.ticks[s.out_groups[m].tick];
        for (int b = tm.done_b0; b <= tm.done_b1; ++b) {
            oocs_op r4 = op(OOCS_OP_RECORD, 1); r4.event = ev_blk_cur(b); r4.tick = tick; r4.block = b;
            s.ops.push_back(r4);
        }
    };
    for (int64_t ti = 0; ti < (int64_t)s.ticks.size(); ++ti) {
        const Tick& t = s.ticks[ti];
        const int isl = t.in_group >= 0 ? (int)(t.in_group % nstage) : -1;
        const bool iret = isl >= 0 && in_retained(t.dz0, t.dz1);
        const bool oret = t.out_group >= 0 && out_retained(t.ez0, t.ez1);
        // a retained output group uses no staging slot and is not written back
        const int osl = t.out_group >= 0 && !oret ? (int)(t.out_group % nstage) : -1;
        const bool loaded = isl >= 0 && !loaded_fields(s.in_groups[t.in_group]).empty();
        if (loaded) { oocs_op w = op(OOCS_OP_WAIT, 1); w.event = ev_loaded(isl); w.tick = (int)ti; s.ops.push_back(w); }
        if (osl >= 0 && !kernel_stores) {
            oocs_op w = op(OOCS_OP_WAIT, 1); w.event = ev_stored(osl); w.tick = (int)ti; s.ops.push_back(w);
        }
        if (isl >= 0)
            for (int fld : in_fields) {
                oocs_op d = op(OOCS_OP_DECODE, 1);
                d.field = fld;
                d.slot = ro_dev && fld == 2 ? OOCS_SLOT_DEVICE_STORE : (iret && fld != 2 ? OOCS_SLOT_RETAINED : isl);
                d.level = in_ring(fld);
                d.z0 = t.dz0; d.z1 = t.dz1; d.block = t.block; d.tick = (int)ti;
                s.ops.push_back(d);
            }
        for (const LevelRange& L : t.levels) {
            oocs_op l = op(OOCS_OP_LEVEL, 1);
            l.level = L.lv; l.z0 = L.z0; l.z1 = L.z1; l.block = t.block; l.tick = (int)ti; l.slot = L.steps;
            s.ops.push_back(l);
        }
        if (t.out_group >= 0)
            for (int fld : out_fields) {
                oocs_op e = op(OOCS_OP_ENCODE, 1);
                e.field = fld; e.slot = oret ? OOCS_SLOT_RETAINED : osl; e.level = out_ring(fld, kr);
                e.z0 = t.ez0; e.z1 = t.ez1; e.block = t.out_block; e.tick = (int)ti;
                s.ops.push_back(e);
            }
        const int64_t stored_now = pend_store;
        if (kernel_stores && pend_store >= 0) emit_store(pend_store, (int)ti);
        { oocs_op l = op(OOCS_OP_LAUNCH, 1); l.tick = (int)ti; l.block = t.block; s.ops.push_back(l); }
        if (kernel_stores && stored_now >= 0) {
            record_blocks_of(stored_now, (int)ti);
            pend_store = -1;
        }
        if (isl >= 0) { oocs_op r2 = op(OOCS_OP_RECORD, 1); r2.event = ev_decoded(isl); r2.tick = (int)ti; s.ops.push_back(r2); }
        if (osl >= 0 && !kernel_stores) { oocs_op r2 = op(OOCS_OP_RECORD, 1); r2.event = ev_encoded(osl); r2.tick = (int)ti; s.ops.push_back(r2); }
        if (kernel_stores && osl >= 0) pend_store = t.out_group;
        if ((int)lagged.size() >= lag) {
            s.ops.insert(s.ops.end(), lagged.front().begin(), lagged.front().end());
            lagged.pop_front();
        }
        next.clear();
        if (osl >= 0 && !kernel_stores) {
            oocs_op w = op(OOCS_OP_WAIT, 2); w.event = ev_encoded(osl); w.tick = (int)ti; next.push_back(w);
            for (int fld : out_fields) {
                oocs_op c = op(OOCS_OP_D2H, 2);
                c.field = fld; c.slot = osl; c.z0 = t.ez0; c.z1 = t.ez1; c.block = t.out_block; c.tick = (int)ti;
                c.level = out_ring(fld, kr);
                next.push_back(c);
            }
            oocs_op r3 = op(OOCS_OP_RECORD, 2); r3.event = ev_stored(osl); r3.tick = (int)ti; next.push_back(r3);
            for (int b = t.done_b0; b <= t.done_b1; ++b) {
                oocs_op r4 = op(OOCS_OP_RECORD, 2); r4.event = ev_blk_cur(b); r4.tick = (int)ti; r4.block = b;
                next.push_back(r4);
            }
        }
        if (isl >= 0 && t.in_group + nstage < nin_groups) emit_h2d(t.in_group + nstage, ti, next);
        lagged.push_back(next);
    }
    if (kernel_stores && pend_store >= 0) {  // epilogue launch: the last output group
        const int tt = (int)s.ticks.size();
        emit_store(pend_store, tt);
        oocs_op l = op(OOCS_OP_LAUNCH, 1); l.tick = tt; l.block = s.out_groups[pend_store].block; s.ops.push_back(l);
        record_blocks_of(pend_store, tt);
    }
    for (const auto& blk : lagged) s.ops.insert(s.ops.end(), blk.begin(), blk.end());
    (void)err;
    return OOCS_OK;
}

// Kernel-driven transfers: one launch per tick on stream 1, holding
// FETCH of the next input group (slot j+1), DECODE of the current one
// (slot j), the levels, ENCODE of the finished output group (slot m) and
// STORE of the one encoded before it (slot m-1). A prologue launch fetches
// the first group and an epilogue launch stores the last one. Launches on
// one stream are ordered, and no two jobs of a launch touch the same slot,
// so no events are needed.
template <class MakeOp>
int Planner::emit_direct(int kr, Schedule& s, MakeOp op) const
{
    const int64_t nin_groups = (int64_t)s.in_groups.size();
    const int64_t nout_groups = (int64_t)s.out_groups.size();
    auto fetch = [&](int64_t j, int tick) {
        const GroupRec& g = s.in_groups[j];
        for (int fld : in_fields) {
            oocs_op c = op(OOCS_OP_FETCH, 1);
            c.field = fld; c.slot = (int)(j % nstage); c.z0 = g.z0; c.z1 = g.z1; c.block = g.block; c.tick = tick;
            c.level = in_ring(fld);
            s.ops.push_back(c);
        }
    };
    auto store = [&](int64_t m, int tick) {
        const GroupRec& g = s.out_groups[m];
        for (int fld : out_fields) {
            oocs_op c = op(OOCS_OP_STORE, 1);
            c.field = fld; c.slot = (int)(m % nstage); c.z0 = g.z0; c.z1 = g.z1; c.block = g.block; c.tick = tick;
            c.level = out_ring(fld, kr);
            s.ops.push_back(c);
        }
    };
    auto launch = [&](int tick, int block) { oocs_op l = op(OOCS_OP_LAUNCH, 1); l.tick = tick; l.block = block; s.ops.push_back(l); };
    if (nin_groups > 0) {
        fetch(0, -1);
        launch(-1, s.in_groups[0].block);
    }
    for (int64_t ti = 0; ti < (int64_t)s.ticks.size(); ++ti) {
        const Tick& t = s.ticks[ti];
        if (t.in_group >= 0) {
            if (t.in_group + 1 < nin_groups) fetch(t.in_group + 1, (int)ti);
            for (int fld : in_fields) {
                oocs_op d = op(OOCS_OP_DECODE, 1);
                d.field = fld; d.slot = (int)(t.in_group % nstage); d.level = in_ring(fld); d.z0 = t.dz0; d.z1 = t.dz1;
                d.block = t.block; d.tick = (int)ti;
                s.ops.push_back(d);
            }
        }
        for (const LevelRange& L : t.levels) {
            oocs_op l = op(OOCS_OP_LEVEL, 1);
            l.level = L.lv; l.z0 = L.z0; l.z1 = L.z1; l.block = t.block; l.tick = (int)ti; l.slot = L.steps;
            s.ops.push_back(l);
        }
        if (t.out_group >= 0) {
            for (int fld : out_fields) {
                oocs_op e = op(OOCS_OP_ENCODE, 1);
                e.field = fld; e.slot = (int)(t.out_group % nstage); e.level = out_ring(fld, kr); e.z0 = t.ez0; e.z1 = t.ez1;
                e.block = t.out_block; e.tick = (int)ti;
                s.ops.push_back(e);
            }
            if (t.out_group > 0) store(t.out_group - 1, (int)ti);
        }
        launch((int)ti, t.block);
    }
    if (nout_groups > 0) {
        store(nout_groups - 1, (int)s.ticks.size());
        launch((int)s.ticks.size(), s.out_groups.back().block);
    }
    return OOCS_OK;
}

const Schedule* Planner::schedule(int kr, std::string& err, int variant)
{
    if (kr < 1 || kr > k) { err = "residency length out of range"; return nullptr; }
    if (variant < 0 || variant > 7 || (variant && !snake)) { err = "schedule variant needs a snake plan"; return nullptr; }
    const int key = kr + 64 * variant;
    auto it = cache_.find(key);
    if (it != cache_.end()) return &it->second;
    Schedule s;
    if (build_ticks(kr, variant, s, err) != OOCS_OK) return nullptr;
    if (emit_ops(kr, variant, s, err) != OOCS_OK) return nullptr;
    for (const Tick& t : s.ticks) {
        const size_t per_in = copy_engines ? 1 : 2, per_out = (copy_engines && !kernel_stores) ? 1 : 2;
        const size_t jobs = t.levels.size() + (t.in_group >= 0 ? per_in * in_fields.size() : 0) +
                            (t.out_group >= 0 ? per_out * out_fields.size() : 0);
        if (jobs > 24) { err = "too many jobs in one tick"; return nullptr; }
    }
    return &cache_.emplace(key, std::move(s)).first->second;
}

}  // namespace oocs
