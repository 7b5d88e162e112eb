/*
 * oocs.h -- C ABI of liboocs, an MI355X (gfx950) library for out-of-core
 * stencil computation with on-the-fly fixed-rate compression, after
 * Shen, Wu, Okita, Ino, "Accelerating GPU-Based Out-of-Core Stencil
 * Computation with On-the-Fly Compression" (arXiv 2109.05410).
 *
 * Conventions for every call:
 *  - Return value: OOCS_OK (0) or a negative OOCS_E_* code. The text of the
 *    last error on the calling thread is returned by oocs_last_error().
 *    No C++ exception crosses this boundary.
 *  - Pointers named d_* are device (HIP) memory, h_* are host memory.
 *    Host buffers handed to oocs_run and the store calls should be pinned
 *    (hipHostMalloc, or torch pin_memory); pageable memory works but the
 *    copies are then synchronous and do not overlap.
 *  - The caller owns every buffer. The library never allocates device
 *    memory: all device scratch of the out-of-core pipeline lives in the one
 *    arena the caller passes to oocs_plan_create, so the device-memory cap is
 *    exact by construction (the paper preallocates fixed-size buffers so that
 *    nothing is allocated while it runs, Sec. IV).
 *  - Streams are hipStream_t passed as void* (NULL = the default stream).
 *    Calls that take a stream are asynchronous with respect to the host.
 *  - Fields are FP32, x fastest: cell (x, y, z) is at x + ld_y*y + ld_z*z
 *    (ld_y = nx, ld_z = nx*ny for dense fields).
 *  - A plan is not thread-safe; distinct plans may be used from distinct
 *    threads.
 */
#ifndef OOCS_H
#define OOCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OOCS_OK 0
#define OOCS_E_ARG -1    /* null pointer, unknown enum, non-positive size */
#define OOCS_E_ALIGN -2  /* a size or chunk boundary is not a multiple of 4 where the codec needs it */
#define OOCS_E_HALO -3   /* halo 2h = 2*r*k exceeds the slab thickness */
#define OOCS_E_CAP -4    /* the pipeline does not fit the device arena */
#define OOCS_E_RATE -5   /* rate outside [1, 34] (0 = uncompressed where allowed) */
#define OOCS_E_SIZE -6   /* a caller buffer is too small */
#define OOCS_E_HIP -7    /* a HIP runtime call failed (message has the HIP error) */
#define OOCS_E_STATE -8  /* the object cannot do this (e.g. a planning-only plan asked to run) */
#define OOCS_E_TIMEOUT -9 /* a bounded device-side wait gave up (the kernel still ended normally) */

#define OOCS_HEAT7 1  /* 7-point Jacobi heat stencil, radius 1 */
#define OOCS_WAVE25 2 /* 25-point 8th-order acoustic wave, radius 4, two time levels */

#define OOCS_MAX_RATE 34 /* rate at which no block is ever truncated */

/* Library version (integer, increases with every ABI change). */
int oocs_version(void);

/* Message of the last error on this thread ("" if none). Valid until the
 * next call on this thread. */
const char* oocs_last_error(void);

/* ------------------------------------------------------------------------
 * Fixed-rate codec (Sec. IV: the user fixes the number of bits kept per
 * value, so the compressed size is known in advance and buffers can be
 * preallocated). Format: 4x4x4 blocks, 64*rate bits each; block b of a
 * field (x fastest, then y, then z over blocks) occupies 64-bit words
 * [b*rate, (b+1)*rate). Inside a block: 1-bit nonzero flag, 8-bit biased
 * common exponent, block-floating-point integers with 30 fraction bits,
 * the separable 4-point decorrelating transform of Lindstrom (IEEE TVCG
 * 20(12), 2014), total-sequency ordering, negabinary, and embedded
 * bit-plane coding with group tests, truncated at the bit budget.
 * Because blocks are independent, any run of whole 4-plane layers of a
 * field is a contiguous byte range of the field's stream; the pipeline
 * relies on this to code the remainder and common region of a slab as
 * separate chunks (Sec. V-A).
 * ------------------------------------------------------------------------ */

/* Bytes of a compressed field: (nx/4)*(ny/4)*(nz/4)*rate*8. Returns 0 if a
 * dimension is not a positive multiple of 4 or rate is outside [1, 34]. */
size_t oocs_codec_bytes(int64_t nx, int64_t ny, int64_t nz, int rate);

/* Encode the FP32 field d_in (nx, ny, nz multiples of 4; leading dimensions
 * ld_y >= nx, ld_z >= ld_y*ny, in elements, both multiples of 4; d_in
 * 16-byte aligned, d_out 8-byte aligned) into d_out, which must hold
 * oocs_codec_bytes(nx, ny, nz, rate) bytes (out_bytes). Stream-ordered; no
 * allocation, no synchronisation. NaN and infinity are not supported.
 * Errors: OOCS_E_ARG, OOCS_E_ALIGN, OOCS_E_RATE, OOCS_E_SIZE, OOCS_E_HIP. */
int oocs_codec_encode(const float* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                      uint64_t* d_out, size_t out_bytes, void* stream);

/* Decode a stream made by oocs_codec_encode with the same dimensions and
 * rate into d_out. A corrupted stream decodes to some values without any
 * out-of-bounds access (every block has a fixed position and budget).
 * rate may be OR-ed with OOCS_DECODE_MIDPOINT (here and in
 * oocs_codec_decode_stages): the digits a block's budget cut off are then
 * reconstructed at the middle of their range instead of as zeros (a
 * coefficient with at least one nonzero digit read, and L digits cut off,
 * gets floor((1 - (-2)^L) / 6) added: half of the value of L negabinary
 * ones); the stream format is unchanged.
 * Errors as for encode. */
#define OOCS_DECODE_MIDPOINT 0x100
int oocs_codec_decode(const uint64_t* d_in, size_t in_bytes, int64_t nx, int64_t ny, int64_t nz, int rate, float* d_out,
                      int64_t ld_y, int64_t ld_z, void* stream);

/* Diagnostic: encode nblocks independent blocks (64 floats each, natural
 * in-block order i + 4j + 16l, block after block in d_blocks) and write every
 * intermediate stage. Any output pointer may be NULL. Per block:
 *   d_emax[b]          common exponent (INT32_MIN for an all-zero block)
 *   d_q[64b + i]       block-floating-point integers, natural order
 *   d_t[64b + i]       after the forward transform, natural order
 *   d_u[64b + k]       negabinary coefficients in sequency order
 *   d_planes[32b + p]  bit plane p as a 64-bit word (bit k = bit p of u[k])
 *   d_words[rate*b+w]  the coded block
 *   d_bits[b]          bits written before padding (header included)
 * Uses the same device code as oocs_codec_encode. */
int oocs_codec_encode_stages(const float* d_blocks, int64_t nblocks, int rate, int32_t* d_emax, int32_t* d_q,
                             int32_t* d_t, uint32_t* d_u, uint64_t* d_planes, uint64_t* d_words, int32_t* d_bits,
                             void* stream);

/* Diagnostic: decode nblocks blocks (rate words each) and write the stages:
 * d_emax[b], d_planes[32b + p], d_u[64b + k] (sequency order), d_q[64b + i]
 * (integers after the inverse transform, natural order) and the values
 * d_out[64b + i]. Any output pointer may be NULL. */
int oocs_codec_decode_stages(const uint64_t* d_words, int64_t nblocks, int rate, int32_t* d_emax, uint64_t* d_planes,
                             uint32_t* d_u, int32_t* d_q, float* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Stencil steps on device-resident fields (Sec. III: every cell is updated
 * from its neighbours each time step; cells outside the grid are zero).
 * ------------------------------------------------------------------------ */

/* k Jacobi steps of u' = u + alpha*((xm+xp)+(ym+yp)+(zm+zp) - 6u) on the
 * dense nx*ny*nz field d_u (x fastest; nx a multiple of 4). d_tmp is caller
 * scratch of the same size; both 16-byte aligned. The result is left in
 * d_u. FP32, fixed operation order, no fused multiply-add. Fields that
 * give a launch of at least 1024 workgroups take four steps per launch in
 * temporally blocked tiles, fields of up to 2^21 cells one step per launch
 * in 8-plane chunks (same bits either way).
 * Errors: OOCS_E_ARG, OOCS_E_ALIGN, OOCS_E_HIP. */
int oocs_heat7_step_k(float* d_u, float* d_tmp, int64_t nx, int64_t ny, int64_t nz, float alpha, int64_t k,
                      void* stream);

/* The same k heat steps for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): no scratch argument and no allocation of any kind. The
 * scratch field lives in a fixed array of OOCS_NOALLOC_MAX_CELLS floats
 * (64 MiB) that the library holds on every GPU it runs on until the process
 * ends; its device address is looked up on the first call on each device.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other streams or threads) race and must be ordered by the caller.
 * The array needs no clearing: each call writes all of it that it reads.
 * Errors: OOCS_E_ARG, OOCS_E_SIZE (nx*ny*nz > OOCS_NOALLOC_MAX_CELLS, checked
 * before any HIP call), OOCS_E_ALIGN, OOCS_E_HIP. */
#define OOCS_NOALLOC_MAX_CELLS (1 << 24)
int oocs_heat7_step_k_noalloc(float* d_u, int64_t nx, int64_t ny, int64_t nz, float alpha, int64_t k, void* stream);

/* k leapfrog steps of the 25-point acoustic wave (Sec. VI: two read-write
 * fields, one read-only field, radius HALO = 4):
 *   p(n+1) = 2 p(n) - p(n-1) + w * L p(n) + s(n) at the source cell,
 *   L p = 3 c0 p + sum_{m=1..4} c_m * sum_axes (p[+m] + p[-m]),
 *   c = (-205/72, 8/5, -1/5, 8/315, -1/560), w = (v dt / dx)^2.
 * On entry (d_pm, d_p) = (p(n-1), p(n)); on exit (p(n+k-1), p(n+k)).
 * h_src holds k host amplitudes (s(n) .. s(n+k-1)) or is NULL; the source
 * cell is (src_x, src_y, src_z) or any coordinate < 0 for none.
 * Errors: OOCS_E_ARG (also for planes of 4 GiB or more: nx * ny * 4 >=
 * 2^32), OOCS_E_HIP. */
int oocs_wave25_step_k(float* d_p, float* d_pm, const float* d_w, int64_t nx, int64_t ny, int64_t nz, int64_t k,
                       const float* h_src, int64_t src_x, int64_t src_y, int64_t src_z, void* stream);

/* ------------------------------------------------------------------------
 * Out-of-core plan (Sec. III and V). The grid is split along z into
 * nslabs blocks [a_i, a_{i+1}), a_i = i*nz/nslabs. One residency advances a
 * block k steps, which needs a halo of h = r*k planes on each side
 * (r = stencil radius). The 2h planes straddling each boundary a_{i+1} form
 * the common region C_i = [a_{i+1}-h, a_{i+1}+h); the rest of the block is
 * its remainder R_i. Region sharing: block i reads R_i and C_i from the host
 * and reuses C_{i-1}, still on the device from block i-1. Separate
 * compression: R_i and C_i are independent chunks of the host store, so
 * after block i the library writes back R_i and C_{i-1} (Fig. 3).
 * ------------------------------------------------------------------------ */

typedef struct oocs_plan oocs_plan;

/* Field slots: heat uses slot 0 (u). The wave uses 0 = p(n), 1 = p(n-1)
 * (both read-write) and 2 = w (read-only, compressed once, never
 * rewritten). */
#define OOCS_MAX_FIELDS 3

typedef struct {
    int64_t nx, ny, nz;             /* grid; nx, ny multiples of 4 */
    int32_t stencil;                /* OOCS_HEAT7 or OOCS_WAVE25 */
    int32_t nslabs;                 /* blocks along z; nz % nslabs == 0 */
    int32_t k;                      /* steps per residency (temporal blocking), >= 1 */
    int32_t group;                  /* planes per pipeline group (multiple of 4); 0 = the largest that fits, at most 32 (16 for the wave) */
    int32_t rate[OOCS_MAX_FIELDS];  /* bits per value of each field's host store; 0 = uncompressed */
    int32_t nstage;                 /* staging slots per direction (>= 2); 0 = default (4, or 2 with kernel transfers) */
    float alpha;                    /* heat diffusion number (u += alpha * Laplacian) */
    int32_t flags;                  /* OOCS_PLAN_* flags, or 0 */
    int64_t src_x, src_y, src_z;    /* wave source cell; any < 0 = no source */
    int32_t retain;                 /* snake plans: slabs in the retained region (see OOCS_PLAN_SNAKE); 0 = one */
} oocs_config;

/* Plan flag. Without it a residency streams the whole grid through the
 * level rings once, so the halo planes of block i at every intermediate
 * time level are the planes block i-1 already computed and stay in the
 * ring (region sharing at every level, not only at the input level): each
 * plane of each level is computed once. With it, every block restarts the
 * level fronts at its extended range [a_i - h, a_{i+1} + h) and recomputes
 * its halo as in Fig. 2. Both give bit-identical results, since every
 * computed plane has fully valid inputs either way; the flag only changes
 * the work and the tick count. The host store layout, the R_i / C_i
 * chunks and the write-back order are the same. */
#define OOCS_PLAN_BLOCK_RESTART 1

/* Plan flags: how groups cross the host link (Sec. V-B).
 * Default: the paper's three streams. Groups are loaded with hipMemcpyAsync
 * on one copy stream and written back with hipMemcpyAsync on another, both
 * ordered against the compute stream with events. The copies a tick makes
 * possible (write-back of its output group, load of the group that reuses
 * its input slot) are issued after the next tick's launch, when the events
 * they wait for have usually completed.
 * OOCS_PLAN_KERNEL_STORES: write-back by STORE jobs inside the pipeline
 * kernel instead: the launch of each tick copies the previous tick's encoded
 * group from its staging slot into the host store.
 * OOCS_PLAN_KERNEL_TRANSFERS: loads by FETCH jobs inside the kernel as well,
 * so everything runs on one stream, one launch per tick, and the host issues
 * nothing else.
 * Whenever a kernel touches the host stores they must be pinned host memory
 * that the device can address (hipHostMalloc, or a torch tensor allocated
 * with pin_memory=True). All modes give bit-identical host stores. */
#define OOCS_PLAN_KERNEL_TRANSFERS 2
#define OOCS_PLAN_KERNEL_STORES 8

/* Plan flag (heat with k <= 4): by default each tick computes all k time
 * levels of its planes in one temporally blocked job (tiles with a k-cell
 * halo, the intermediate levels held in registers and LDS), so the device
 * holds only the decoded input and the output level, and the groups can be
 * larger under the same cap. With this flag every level is its own job and
 * has its own ring of planes (always the case for the wave, for k > 4 and
 * with OOCS_PLAN_BLOCK_RESTART). Same results. */
#define OOCS_PLAN_LEVEL_BY_LEVEL 4

/* Plan flag (wave): keep the read-only field resident on the device instead
 * of streaming its chunks every residency (the paper streams it, Sec. VI).
 * Its store is decoded once into an arena buffer of nz planes, at the first
 * oocs_run after the plan is created or after any oocs_store_put /
 * oocs_store_get on the plan (those stream through the arena and overwrite
 * it), and whenever oocs_run is given a different read-only store pointer;
 * rewriting the store's contents in place between runs is not detected.
 * Each residency then moves and decodes only the two read-write fields.
 * Same results as streaming (the same decoded values are read). Needs an
 * arena that holds the whole decoded field besides the rings (OOCS_E_CAP
 * otherwise). */
#define OOCS_PLAN_RESIDENT_RO 16

/* Plan flag: snake sweeps (alternating direction). Residency i of an
 * oocs_run call streams the grid upward in z if i is even, downward if odd,
 * and the block it ends with stays on the device for the next residency,
 * which starts with it: its compressed (or raw) output is written into a
 * retained buffer of the arena instead of the host store, and the next
 * residency decodes it from there instead of loading it. The last block
 * of every residency but the call's last therefore crosses the host link
 * neither way; the read-only field is still streamed. Same results (the
 * retained planes pass through the codec exactly as the stored ones).
 * Needs the copy-engine transfers (no OOCS_PLAN_KERNEL_TRANSFERS or
 * OOCS_PLAN_KERNEL_STORES), no OOCS_PLAN_BLOCK_RESTART and nslabs >= 2.
 * oocs_config.retain sets how many slabs the retained region spans: 0 or 1
 * = the last block only; 1 < m <= nslabs = the last m blocks (a region
 * that also holds the planes a residency writes back while its pipeline
 * drains, and the next one loads while its pipeline fills, keeps both
 * phases off the host link; with m = nslabs the read-write fields cross
 * the link only in a call's first and last residency); OOCS_RETAIN_MAX =
 * the most slabs that fit in the arena beside the pipeline chosen with
 * one. A residency decodes the region it starts with from the buffer and
 * encodes the one it ends with into it, plane z of a region at place
 * z - (its first plane); beyond half the grid the two regions overlap, and
 * a plane of both is encoded to another place than the one it was decoded
 * from, after every decode of what that place held. The retained buffers
 * take retain * slab planes of every read-write field's store from the
 * arena; oocs_plan_get_info reports the planes. Any other value, or a
 * nonzero retain without this flag, is OOCS_E_ARG. */
#define OOCS_PLAN_SNAKE 32
#define OOCS_RETAIN_MAX (-1)

/* Plan flag: every decode of the plan (the residencies' decode jobs, the
 * resident read-only load, oocs_store_get) uses mid-point reconstruction
 * (OOCS_DECODE_MIDPOINT). The host stores are the same; the state a run
 * reaches is that of decode-with-mid-points o encode applied where the
 * plain plan applies decode o encode. */
#define OOCS_PLAN_MIDPOINT 64

/* Plan flag (wave): the fields are FP64 (the precision of the paper's
 * experiments, Sec. VI): device planes of doubles, raw host stores of
 * nx*ny*nz*8 bytes, compressed stores in the FP64 format (rates 1..68, see
 * oocs_codec64_encode), the FP64 wave step (oocs_wave25_step_k_f64's
 * arithmetic). oocs_store_put / oocs_store_get take double fields; source
 * amplitudes stay float (converted exactly to double). Not with
 * OOCS_PLAN_MIDPOINT, the heat stencil or transfer jobs
 * (OOCS_PLAN_KERNEL_TRANSFERS, OOCS_PLAN_KERNEL_STORES). */
#define OOCS_PLAN_FP64 128

/* Plan flag (wave): the read-only field's host store (compressed, or raw
 * at rate 0) is copied once into the arena (oocs_run copies it when the
 * read-only store pointer differs from the last one it copied; store I/O
 * on the plan forgets it), and every residency decodes the read-only
 * chunks from there instead of copying them over the host link: the
 * host-to-device traffic of a residency drops by that field's store bytes,
 * and the arena holds oocs_store_bytes(plan, 2) more bytes. Results are
 * identical. Copy-engine transfers only; not with OOCS_PLAN_RESIDENT_RO. */
#define OOCS_PLAN_RO_DEVICE_STORE 256

/* Create a plan. d_arena (arena_bytes long) is the only device memory the
 * pipeline will use; pass NULL to make a planning-only plan that can be
 * queried but not run (no HIP call is made for it). Chooses the group size
 * (when cfg->group == 0) as the largest multiple of 4, at most 32 planes (16
 * for the wave, whose ticks are long already), whose rings and staging fit
 * arena_bytes. The plan keeps d_arena; the caller keeps it
 * alive until oocs_plan_destroy.
 * Errors: OOCS_E_ARG (also a wave plane of 4 GiB or more), OOCS_E_ALIGN (a
 * compressed field with nz/nslabs or h not a multiple of 4), OOCS_E_HALO
 * (2h > nz/nslabs), OOCS_E_RATE, OOCS_E_CAP (nothing fits arena_bytes),
 * OOCS_E_HIP (stream or event creation). */
int oocs_plan_create(const oocs_config* cfg, void* d_arena, size_t arena_bytes, oocs_plan** out);

/* Release the plan's streams and events (not the arena). NULL is allowed. */
int oocs_plan_destroy(oocs_plan* plan);

typedef struct {
    int64_t group;              /* planes per pipeline group */
    int64_t halo;               /* h = r * k */
    int64_t radius;             /* r */
    int64_t nlevels;            /* time levels of a residency (inputs + k computed) */
    int64_t nrings;             /* device plane rings (levels + the read-only field) */
    int64_t ring_planes[16];    /* planes per ring; index = level, then the read-only ring */
    int64_t plane_bytes;        /* nx * ny * 4 */
    int64_t arena_needed;       /* device bytes the plan uses (<= arena size) */
    int64_t nstage;             /* staging slots per direction */
    int64_t store_bytes[OOCS_MAX_FIELDS]; /* host store bytes per field (0 for an unused slot) */
    int64_t retained_planes;    /* planes of the retained region (snake plans), else 0 */
} oocs_plan_info;

int oocs_plan_get_info(const oocs_plan* plan, oocs_plan_info* out);

typedef struct {
    int64_t z0, z1;         /* the block [a_i, a_{i+1}) */
    int64_t r0, r1;         /* remainder R_i */
    int64_t c0, c1;         /* common region C_i (empty for the last block) */
    int64_t r_off[OOCS_MAX_FIELDS], r_bytes[OOCS_MAX_FIELDS]; /* R_i in each field's host store */
    int64_t c_off[OOCS_MAX_FIELDS], c_bytes[OOCS_MAX_FIELDS]; /* C_i in each field's host store */
} oocs_slab_info;

int oocs_plan_slab(const oocs_plan* plan, int i, oocs_slab_info* out);

/* The per-residency schedule as a list of operations on three streams
 * (0 = host-to-device copies, 1 = compute, 2 = device-to-host copies),
 * exposed so that its ordering can be checked without a GPU. kr is the
 * number of steps of the residency (k, or the remainder of the last one).
 * With OOCS_PLAN_KERNEL_TRANSFERS every op is on stream 1 and the copies
 * are FETCH / STORE jobs of the launches. */
#define OOCS_OP_H2D 1     /* copy a group of host-store planes into an input staging slot */
#define OOCS_OP_DECODE 2  /* decode (or copy, if uncompressed) a staging slot into a level ring */
#define OOCS_OP_LEVEL 3   /* compute planes [z0, z1) of ring `level` from ring level-1, `slot` steps later */
#define OOCS_OP_ENCODE 4  /* encode (or copy) planes of an output level into an output staging slot */
#define OOCS_OP_D2H 5     /* copy an output staging slot to the host store */
#define OOCS_OP_LAUNCH 6  /* issue the jobs accumulated on the compute stream as one kernel launch */
#define OOCS_OP_RECORD 7  /* record event `event` on `stream` */
#define OOCS_OP_WAIT 8    /* make `stream` wait for the last record of `event` */
#define OOCS_OP_FETCH 9   /* job: copy a group of host-store planes into an input staging slot */
#define OOCS_OP_STORE 10  /* job: copy an output staging slot to the host store */

typedef struct {
    int32_t kind;    /* OOCS_OP_* */
    int32_t stream;  /* 0, 1, 2 */
    int32_t field;   /* field slot (H2D/DECODE/ENCODE/D2H) */
    int32_t level;   /* ring index: DECODE/ENCODE source or target level; LEVEL: computed level */
    int32_t slot;    /* staging slot (H2D/DECODE/ENCODE/D2H) */
    int32_t block;   /* slab index */
    int32_t tick;    /* compute tick the op belongs to */
    int32_t event;   /* RECORD/WAIT */
    int64_t z0, z1;  /* planes */
} oocs_op;

/* Number of operations of the residency schedule for kr steps (1 <= kr <= k),
 * building and caching it on first use. Returns < 0 on error. */
int64_t oocs_plan_schedule_len(oocs_plan* plan, int kr);
int oocs_plan_schedule_op(oocs_plan* plan, int kr, int64_t index, oocs_op* out);

/* Schedule variants of snake plans (OOCS_PLAN_SNAKE), OR-ed: the residency
 * runs downward in z (its op ranges and blocks are those of the upward
 * schedule mirrored), takes its first block from the retained buffer, and
 * leaves its last block there. oocs_run uses for residency i of R:
 * MIRROR if i is odd, RETAIN_IN if i > 0, RETAIN_OUT if i < R - 1. Decode
 * and encode ops on the retained buffer carry slot OOCS_SLOT_RETAINED and
 * have no copy. Variant 0 is the schedule above. */
#define OOCS_SCHED_MIRROR 1
#define OOCS_SCHED_RETAIN_IN 2
#define OOCS_SCHED_RETAIN_OUT 4
#define OOCS_SLOT_RETAINED (-2)
/* Decode ops of the read-only field in an OOCS_PLAN_RO_DEVICE_STORE plan
 * read its chunk from the device copy of the store and carry this slot. */
#define OOCS_SLOT_DEVICE_STORE (-3)
int64_t oocs_plan_schedule_variant_len(oocs_plan* plan, int kr, int variant);
int oocs_plan_schedule_variant_op(oocs_plan* plan, int kr, int variant, int64_t index, oocs_op* out);

/* Host store size for a field slot: the field's compressed stream, or
 * nx*ny*nz*4 bytes if uncompressed (nx*ny*nz*8 in an FP64 plan); 0 for an
 * unused slot. */
size_t oocs_store_bytes(const oocs_plan* plan, int field);

/* Build a field's host store from the host field h_field (nx*ny*nz values,
 * x fastest: float, or double in an FP64 plan): the initial compression,
 * done once; for the read-only field the only time it is ever compressed.
 * Streams through the plan's arena on the GPU. Blocking. */
int oocs_store_put(oocs_plan* plan, int field, const void* h_field, void* h_store);

/* Decode a field's host store into the host field h_field (float, or
 * double in an FP64 plan). Blocking. */
int oocs_store_get(oocs_plan* plan, int field, const void* h_store, void* h_field);

typedef struct {
    double wall_ms;          /* host wall time of the call */
    double enqueue_ms;       /* host time spent issuing the work (before the final wait) */
    int64_t rounds;          /* residencies executed */
    int64_t h2d_bytes;       /* bytes copied host -> device */
    int64_t d2h_bytes;       /* bytes copied device -> host */
    int64_t cell_updates;    /* nx*ny*nz*steps */
    /* Each tick is one launch of the pipeline kernel on the compute stream:
     * decode and encode jobs plus one z-range of every time level. Reported:
     * launches, the algorithmic device-memory bytes of all launches (every
     * input plane read once and every output plane written once per job:
     * heat 8 B per cell update, wave 16 B, decode and encode 4 + rate/8 B
     * per value, uncompressed copy 8 B per value), split into codec and
     * stencil jobs, and the summed GPU time of the launches measured with
     * timing events around each launch when profiling is on (0 otherwise). */
    int64_t launches;
    int64_t codec_bytes, stencil_bytes;
    double kernel_ms;
    /* FETCH / STORE jobs (kernel-driven transfers): bytes they move across
     * the host link, which are also the device-memory bytes they write or
     * read in the staging slots. Included in h2d_bytes / d2h_bytes too. */
    int64_t xfer_bytes;
    /* The launches that carried timing events (every N-th launch with
     * oocs_plan_set_profiling(plan, N)) and their algorithmic bytes:
     * kernel_ms / timed_launches is the average launch duration and
     * timed_bytes / kernel_ms the achieved algorithmic bandwidth. */
    int64_t timed_launches, timed_bytes;
    /* Device-to-host copies of this call issued on SDMA engines through the
     * HSA runtime (oocs_plan_set_sdma); the others went through hipMemcpyAsync. */
    int64_t sdma_copies;
    /* Per-stage breakdown (oocs_plan_set_breakdown on, op-by-op issue; else
     * zeros): summed durations in ms of the work of each stage of Sec. V-B,
     * [0] host-to-device copies, [1] decode jobs (raw copy-in when
     * uncompressed), [2] stencil steps, [3] encode jobs (raw copy-out),
     * [4] device-to-host copies (HIP events around each copy or launch; SDMA
     * copies by the engine's own timestamps). Stages on different engines
     * overlap, so the sum exceeds wall_ms. */
    double stage_ms[5];
    /* Device bytes the plan uses: its peak arena footprint (<= the cap). */
    int64_t arena_bytes;
} oocs_stats;

/* Per-launch kernel timing for later oocs_run calls on this plan: 0 turns it
 * off, N > 0 records timing events on the compute stream around every N-th
 * launch (N = 1: every launch). The sum of their elapsed times is returned in
 * oocs_stats.kernel_ms, with the timed launches and their bytes. */
int oocs_plan_set_profiling(oocs_plan* plan, int on);

/* Per-stage breakdown for later oocs_run calls on this plan (default 0):
 * with op-by-op issue, every tick's jobs are launched as one launch per
 * stage (decode, stencil, encode) between timing events instead of one
 * fused launch, and every copy is timed, so oocs_stats.stage_ms gives the
 * time of each stage (the breakdown of Sec. VI-B). Same results; the
 * split launches make the run slower, so time throughput with it off. */
int oocs_plan_set_breakdown(oocs_plan* plan, int on);

/* Choose how oocs_run issues a residency (default 0): as one replay of a HIP
 * graph built once per residency length and set of host stores (1), or op by
 * op on the streams (0). Both run the same kernels with the same parameters;
 * graph replays of consecutive residencies do not overlap. */
int oocs_plan_set_graphs(oocs_plan* plan, int on);

/* Op-by-op issue (graphs off): how a wait on an event of another stream that
 * has not completed yet is honoured (default 1): the host blocks until the
 * event completes and then issues the dependent work (1), or the stream is
 * made to wait with hipStreamWaitEvent (0). Waits on completed events are
 * skipped either way. Same results; (1) keeps the host's issue cost low. */
int oocs_plan_set_host_waits(oocs_plan* plan, int on);

/* Device-to-host copies of op-by-op issue with host waits (default 1): on an
 * SDMA engine through the HSA runtime that HIP has loaded (1), or with
 * hipMemcpyAsync (0), which some HIP runtimes carry out as a blit kernel that
 * holds compute units beside the pipeline kernel (Sec. V-B gives the copies
 * engines of their own). The SDMA path applies only when every written-back
 * store is pinned host memory the runtime knows and the engine is available
 * (oocs_plan_sdma_available); otherwise hipMemcpyAsync is used. Graph issue,
 * stream waits and kernel-driven transfers never use it. Same results.
 * on >= 2: every copy is split into `on` parts, each on an SDMA engine of
 * its own (as many as the runtime reports available for the direction, up
 * to `on`; one engine chosen by the runtime if it reports fewer than two);
 * at most 16. */
int oocs_plan_set_sdma(oocs_plan* plan, int on);

/* 1 if the plan found the HSA runtime and the GPU agent of its arena, else 0. */
int oocs_plan_sdma_available(const oocs_plan* plan);

/* Host-link probe, the link roofline of the pipeline's transfers (Sec. V-B:
 * copies in both directions overlap). Moves `bytes` from pinned host h_in to
 * device d_a and from device d_b to pinned host h_out in chunks of `chunk`
 * bytes, with the engines the pipeline uses: hipMemcpyAsync on one stream
 * host to device; device to host on an SDMA engine through HSA if `sdma` and
 * available (sdma >= 2: each chunk split over that many engines, as in
 * oocs_plan_set_sdma), else hipMemcpyAsync on a second stream. Each direction alone,
 * then both at once; one untimed pass, then `reps` timed ones (host wall
 * clock). out[4]: GB/s host to device alone, device to host alone, each way
 * with both at once, and 1.0 if the SDMA path was used (else 0.0). All four
 * buffers hold `bytes` bytes and stay the caller's. Blocking.
 * Errors: OOCS_E_ARG, OOCS_E_HIP. */
int oocs_link_probe(void* d_a, void* d_b, void* h_in, void* h_out, size_t bytes, size_t chunk, int reps, int sdma,
                    double* out);

/* Advance the out-of-core state held in the host stores h_store[field]
 * (one pointer per used field slot) by `steps` time steps, k per residency
 * (the last residency does steps mod k). The wave source adds h_src[s] at
 * the source cell when the field after the s-th step of this call is
 * formed (s = 0 .. steps-1); h_src holds `steps` values or is NULL. Host
 * stores are updated in place. Blocks until done; st may be NULL.
 * With OOCS_PLAN_KERNEL_STORES or OOCS_PLAN_KERNEL_TRANSFERS kernels read or
 * write the stores directly, so each must be pinned, device-addressable host
 * memory.
 * Errors: OOCS_E_ARG (also: a store the device cannot address), OOCS_E_STATE
 * (planning-only plan), OOCS_E_HIP. */
int oocs_run(oocs_plan* plan, void* const* h_store, int64_t steps, const float* h_src, oocs_stats* st);

/* ------------------------------------------------------------------------
 * FP64 (the precision of the paper's experiments, Sec. VI). The same
 * fixed-rate 4^3 block method with 64-bit integers: exponent from frexp
 * clamped at -1022, header 1 bit + (emax + 1023) in 11 bits, q =
 * trunc(x * 2^(62 - emax)) as int64, the same lifting, sequency order and
 * group-test coding over bit planes 63..0, 64 * rate - 12 bits of budget;
 * block b at word b * rate. Rates 1..68 bits per value.
 * ------------------------------------------------------------------------ */
#define OOCS_MAX_RATE64 68

/* Bytes of an FP64 field's stream; 0 on bad dims or rate. */
size_t oocs_codec64_bytes(int64_t nx, int64_t ny, int64_t nz, int rate);

/* Encode / decode an FP64 field (x fastest, leading dimensions ld_y >= nx,
 * ld_z >= ld_y * ny in elements; 8-byte aligned buffers). Stream-ordered, no
 * allocation. Errors: OOCS_E_ARG, OOCS_E_ALIGN, OOCS_E_RATE, OOCS_E_SIZE,
 * OOCS_E_HIP. */
int oocs_codec64_encode(const double* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                        uint64_t* d_out, size_t out_bytes, void* stream);
int oocs_codec64_decode(const uint64_t* d_in, size_t in_bytes, int64_t nx, int64_t ny, int64_t nz, int rate,
                        double* d_out, int64_t ld_y, int64_t ld_z, void* stream);

/* Per-block stages for parity checks (nblocks blocks of 64 values in
 * natural in-block order): as oocs_codec_encode_stages / _decode_stages
 * with 64-bit integers and 64 plane words per block. */
int oocs_codec64_encode_stages(const double* d_blocks, int64_t nblocks, int rate, int32_t* d_emax, int64_t* d_q,
                               int64_t* d_t, uint64_t* d_u, uint64_t* d_planes, uint64_t* d_words, int32_t* d_bits,
                               void* stream);
int oocs_codec64_decode_stages(const uint64_t* d_words, int64_t nblocks, int rate, int32_t* d_emax, uint64_t* d_planes,
                               uint64_t* d_u, int64_t* d_q, double* d_out, void* stream);

/* k FP64 leapfrog steps of the 25-point wave in place on (d_pm, d_p) =
 * (p(n-1), p(n)), d_w read-only; the FP32 step's formula and operation
 * order in double (the paper's precision). h_src: k amplitudes added at
 * the source cell (host memory), or NULL. Planes must hold less than 4 GiB
 * (nx * ny * 8 < 2^32), else OOCS_E_ARG. */
int oocs_wave25_step_k_f64(double* d_p, double* d_pm, const double* d_w, int64_t nx, int64_t ny, int64_t nz,
                           int64_t k, const double* h_src, int64_t src_x, int64_t src_y, int64_t src_z, void* stream);

/* ------------------------------------------------------------------------
 * Batched in-core heat domains. Many independent domains of uneven sizes
 * advance together. By default a run replays, as one HIP graph, one launch
 * per group (every tile of every domain, k steps). The persistent mode runs
 * the same work as one kernel launch: its workgroups take items (domain,
 * up to 32 consecutive tiles, group of k steps) in order from a device
 * queue, and an item of group g of a domain starts once every tile of group
 * g-1 of that domain has finished (a per-domain count of finished tiles,
 * raised after a device-scope release). Waits are bounded: a wait that
 * exceeds its poll limit sets a status word and every workgroup leaves, so
 * the kernel always ends; oocs_batch_check reports it. On a chip whose dies
 * each have their own L2, the device-scope release and acquire around every
 * item write back and invalidate that L2, which costs more than the launch
 * boundaries it saves: the persistent mode is the slower one there and
 * stays opt-in.
 * k > 1 is temporal blocking: a workgroup
 * advances its tile k steps in one pass over z, recomputing a k-cell halo,
 * so each cell crosses HBM once per k steps. The tile shape is chosen per
 * size bucket by a timing autotuner (three or more shapes per depth) whose
 * results persist in a cache file, and the depth k (1, 2 or 4) per batch.
 * ------------------------------------------------------------------------ */

typedef struct {
    float* d_u;        /* state (nz, ny, nx), x fastest; before and after a run */
    float* d_scratch;  /* caller scratch of the same size */
    int64_t nx, ny, nz;
} oocs_domain;

typedef struct oocs_batch oocs_batch;

/* Device bytes of the work-list tables and the persistent launch's counters
 * for nd domains. */
size_t oocs_batch_table_bytes(int nd);

/* Create a batch of nd domains (heat, u' = u + alpha*Laplacian, zero
 * ghosts). d_table: device memory of oocs_batch_table_bytes(nd) bytes.
 * tune: 1 = time the tile candidates of every depth on this GPU for every
 * size bucket not found in the cache (the domains' own u buffers are read,
 * their scratch buffers written; states are unchanged), 0 = use the cache,
 * else the default tiles. depth: 0 = with tune = 1, the depth whose launch
 * over the whole batch (same buffers as above) takes the least time per
 * step; with tune = 0, the least time per step estimated from the cached
 * single-domain timings (1 if unknown); or 1, 2, 4 to force it. Every depth
 * gives the same bits.
 * tune_cache: path of the cache file (NULL = no cache). The caller keeps the
 * domain buffers and d_table alive until destroy.
 * Errors: OOCS_E_ARG, OOCS_E_SIZE, OOCS_E_HIP. */
int oocs_batch_create(const oocs_domain* doms, int nd, float alpha, void* d_table, size_t table_bytes,
                      const char* tune_cache, int tune, int depth, void* stream, oocs_batch** out);

/* Advance every domain `steps` steps as one graph launch on `stream`, built
 * once per step count. Persistent mode: one kernel for the
 * steps / k groups at depth k; when steps mod k > 0, a second persistent
 * kernel for the remaining depth-1 groups; when the number of groups is
 * odd, copy items move the result from the scratch buffers to u (in the
 * depth-1 kernel, or in a third small one). Launch mode: steps / k launches
 * at depth k, then steps mod k at depth 1, then copies if needed.
 * Asynchronous; with the persistent mode call oocs_batch_check to learn
 * whether a wait gave up. */
int oocs_batch_run(oocs_batch* b, int64_t steps, void* stream);

/* 1: runs are persistent launches; 0 (default): one launch per group. */
int oocs_batch_set_persistent(oocs_batch* b, int on);

/* Poll limit of the persistent kernel's waits (default 2^21 polls, each
 * after a short sleep; seconds in all). never_satisfied = 1 is a test hook:
 * no wait is ever satisfied, so the first wait gives up after `polls`
 * polls, sets the status and every workgroup leaves. */
int oocs_batch_set_wait_limit(oocs_batch* b, int64_t polls, int never_satisfied);

/* Synchronizes `stream`, then reads the persistent launches' status word:
 * OOCS_OK, or OOCS_E_TIMEOUT if a wait gave up since the last check (the
 * status is cleared; the domains' states are then undefined). */
int oocs_batch_check(oocs_batch* b, void* stream);

/* Baseline: the same launches as separate kernel launches, domain after
 * domain. */
int oocs_batch_run_per_domain(oocs_batch* b, int64_t steps, void* stream);

/* Tile configuration chosen for a domain at the batch depth: tx, ty (threads
 * per tile for k = 1; tile cells including the halo for k > 1), planes per
 * z chunk, and the depth k. */
int oocs_batch_domain_tile(const oocs_batch* b, int domain, int* tx, int* ty, int* zc, int* k);

int oocs_batch_destroy(oocs_batch* b);

/* ------------------------------------------------------------------------
 * Misfit gradient of the wave propagator by its discrete adjoint, with
 * compressed forward checkpoints in host memory.
 *
 * Forward from rest: p(t+1) = 2p(t) - p(t-1) + w . L p(t) + s(t) at the
 * source cell, w = (v * vscale)^2 (vscale = dt/dx), t = 0..T-1; receivers
 * record r(t) = p(t) at nrcv cells for t = 1..T; J = 1/2 sum_t |r(t) - d(t)|^2.
 * Adjoint (L symmetric under zero ghosts): lam(t) = 2 lam(t+1) - lam(t+2) +
 * L(w . lam(t+1)) + S^T (r(t) - d(t)), lam(T+1) = lam(T+2) = 0;
 * dJ/dw = sum_t lam(t) . L p(t-1);  dJ/dv = dJ/dw . 2 v vscale^2.
 * The forward pass stores (p(t), p(t-1)) every ckpt_every steps through the
 * fixed-rate codec (ckpt_rate bits per value, 0 = uncompressed) into a host
 * store (the same fixed-rate format as Sec. IV, here applied to checkpoints);
 * the backward pass decodes them in reverse, recomputes each segment's
 * states on the device and runs the adjoint over it. With uncompressed
 * checkpoints the gradient is the exact FP32 gradient.
 * ------------------------------------------------------------------------ */

typedef struct {
    int64_t nx, ny, nz;          /* grid, x fastest; nx, ny, nz multiples of 4 if ckpt_rate > 0 */
    int64_t steps;               /* T >= 1 */
    int64_t ckpt_every;          /* steps between checkpoints, >= 1 */
    int32_t ckpt_rate;           /* bits per value of the checkpoints; 0 = uncompressed */
    int32_t nrcv;                /* receivers, >= 0 */
    int64_t src_x, src_y, src_z; /* source cell */
    float vscale;                /* dt / dx */
    int32_t pad0;
} oocs_adjoint_cfg;

/* Device workspace bytes the two calls below need (one caller allocation,
 * passed as d_work): w, ckpt_every + 2 state fields, three multiplier
 * fields, two fields of w . multiplier, the w-gradient field and the
 * checkpoint codec staging. The calls copy checkpoints on a second stream
 * of their own, overlapped with the steps. */
size_t oocs_adjoint_workspace_bytes(const oocs_adjoint_cfg* cfg);

/* Host checkpoint store bytes (pinned memory recommended). */
size_t oocs_adjoint_ckpt_bytes(const oocs_adjoint_cfg* cfg);

/* Forward pass. d_v: velocity field; h_src: T source amplitudes (host);
 * d_rcv: nrcv flat cell indices (device, int64; indices outside the grid
 * are ignored); d_obs: observed records
 * (device, T x nrcv, row t-1 for time t). Writes the residuals r - d into
 * d_res (device, T x nrcv), the checkpoints into h_ckpt, and J (FP64 sum of
 * the FP32 residuals) into *J. Blocking. */
int oocs_wave_forward_ckpt(const oocs_adjoint_cfg* cfg, const float* d_v, const float* h_src, const int64_t* d_rcv,
                           const float* d_obs, float* d_res, void* d_work, size_t work_bytes, void* h_ckpt, double* J,
                           void* stream);

/* Backward pass after oocs_wave_forward_ckpt with the same arguments:
 * writes dJ/dv into d_grad_v. Blocking. */
int oocs_wave_adjoint(const oocs_adjoint_cfg* cfg, const float* d_v, const float* h_src, const int64_t* d_rcv,
                      const float* d_res, void* d_work, size_t work_bytes, const void* h_ckpt, float* d_grad_v,
                      void* stream);

#ifdef __cplusplus
}
#endif
#endif /* OOCS_H */
