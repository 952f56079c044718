/*
 * spr.h — C ABI of libspr: speculative progressive isosurface raycasting of a
 * block-compressed volume on one AMD Instinct MI355X (gfx950).
 *
 * Method: Usher, Dyken, Kumar, "Speculative Progressive Raycasting for Memory
 * Constrained Isosurface Visualization of Massive Volumes" (arXiv 2309.10212).
 * The calls follow the paper's problem statement: a compressed volume is
 * uploaded once (Sec. 3 overview); every new camera or isovalue computes new
 * rays (Sec. 3.2); passes repeat until every ray has terminated, and the
 * partial image is available after each pass (Sec. 3, pipeline figure (a)-(f)).
 *
 * Conventions
 *  - Every call returns an spr_status; 0 is success.  No C++ exception
 *    crosses this boundary.  On failure spr_last_error() returns a
 *    thread-local message.  NULL handles and out-pointers are rejected with
 *    SPR_E_INVALID.
 *  - Ownership: the library copies host inputs (volume_load) and writes into
 *    caller buffers (read_*).  Device memory belongs to the handles and comes
 *    from the context's allocator (hipMalloc when none is given).  Destroy
 *    renders and batches first, then volumes, then the context.
 *  - Streams: a context issues all work on one HIP stream (spr_config.stream,
 *    0 = the null stream).  Calls are stream-ordered and return without
 *    waiting, except those documented as synchronising: render_done,
 *    render_run, batch_pass, batch_run, read_*, debug_*, mem_stats, and any
 *    call given a non-NULL spr_pass_stats.
 *  - Threading: a context and everything created from it must be used from
 *    one thread at a time.
 */
#ifndef SPR_H
#define SPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spr_status;
#define SPR_OK 0
#define SPR_E_INVALID (-1)       /* bad argument, handle or descriptor */
#define SPR_E_OOM (-2)           /* device or host allocation failed */
#define SPR_E_HIP (-3)           /* a HIP runtime call failed */
#define SPR_E_CORRUPT (-4)       /* compressed stream inconsistent with its descriptor */
#define SPR_E_CAPACITY (-5)      /* decoded-block cache cannot hold one block and its neighbours */
#define SPR_E_STATE (-6)         /* call not valid in the handle's current state */
#define SPR_E_UNIMPLEMENTED (-7)

#define SPR_NONE 0xFFFFFFFFu     /* "no block" sentinel (Sec. 3.3 uses UINT_MAX) */
#define SPR_CODEC_VERSION 1u
#define SPR_DTYPE_F32 0u
#define SPR_DTYPE_U8 1u

typedef struct spr_ctx spr_ctx;
typedef struct spr_volume spr_volume;
typedef struct spr_render spr_render;
typedef struct spr_batch spr_batch;

/* Device allocator hooks.  alloc returns a device pointer (NULL on failure);
 * free releases it.  Python passes torch's caching allocator here. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, size_t bytes, void *user);
    void *user;
} spr_allocator;

typedef struct {
    int device;            /* HIP device ordinal */
    void *stream;          /* hipStream_t; NULL = null stream */
    size_t cache_bytes;    /* decoded-block cache capacity; 256 B per slot (Sec. 3.5) */
    uint32_t spec_cap;     /* default speculation cap for new renders (Sec. 4: 64); 0 -> 64; at most 4096 */
    uint32_t flags;        /* reserved, must be 0 */
    spr_allocator alloc;   /* optional; alloc.alloc == NULL -> hipMalloc/hipFree */
} spr_config;

/* A compressed volume (Sec. 3 overview: fixed-rate block compression).
 * 2 <= nx, ny, nz <= SPR_MAX_EXTENT samples; rate_bits in 1..16 (coded) or 32 (raw float32);
 * src_dtype records what the samples were before conversion to float32;
 * codec_version must be SPR_CODEC_VERSION.  The stream holds
 * ceil(nx/4)*ceil(ny/4)*ceil(nz/4) records of 8*rate_bits bytes, block
 * (bx,by,bz) at index bx + nbx*(by + nby*bz). */
typedef struct {
    uint32_t nx, ny, nz;
    uint32_t rate_bits;
    uint32_t src_dtype;
    uint32_t codec_version;
} spr_volume_desc;

/* Pinhole camera (Sec. 3.2): eye, look-at point, up vector, vertical field
 * of view in degrees.  Coordinates are in sample units: sample (i,j,k) sits
 * at the point (i,j,k); each eye coordinate lies within +-SPR_MAX_EXTENT
 * (render creation fails with SPR_E_INVALID otherwise).  With the volume
 * extent limit this keeps every ray position below 2^20 blocks, where the
 * traversal's fp32 block estimate is exact to a quarter block. */
#define SPR_MAX_EXTENT 524288u
typedef struct {
    double eye[3], center[3], up[3];
    double vfov_deg;
} spr_camera;

/* Per-pixel hit record: ray parameter t (unit-length direction, sample
 * units), block id of the hit cell, cell index (cx&3)+4(cy&3)+16(cz&3).
 * No hit: t = +inf, block_id = cell = SPR_NONE. */
typedef struct {
    double t;
    uint32_t block_id;
    uint32_t cell;
} spr_hit;

/* Counters of one pass (Sec. 5 statistics: speculation count, utilization as
 * ray-block pairs over w*h slots, blocks visible per pass, memory). */
typedef struct {
    uint32_t pass;            /* 1-based pass index of this render */
    uint32_t n_active;        /* active rays at the start of the pass */
    uint32_t n_spec;          /* speculation count used by the pass */
    uint32_t pairs;           /* ray-block pairs written (R_BID entries != NONE) */
    uint32_t visible_blocks;  /* distinct blocks in the pairs */
    uint32_t active_blocks;   /* visible blocks plus their +x/+y/+z neighbours */
    uint32_t blocks_decoded;  /* cache misses decompressed this pass */
    uint32_t deferred_pairs;  /* pairs postponed because the cache was too small */
    uint32_t terminated;      /* rays that terminated this pass */
    uint32_t slots;           /* pair slots the pass handed out: n_active * n_spec, or the sum of the
                                 per-ray counts (SPR_SPEC_PER_RAY) */
    double utilization;       /* pairs / (w*h) */
    float ms;                 /* device time of the pass (HIP events) */
    float pad;
} spr_pass_stats;

/* Cumulative device counters of a context since its creation. */
typedef struct {
    uint64_t passes;          /* passes run (single renders and batches) */
    uint64_t blocks_decoded;  /* cache misses decompressed */
    uint64_t visible_blocks;  /* sum over passes of visible blocks */
    uint64_t active_blocks;   /* sum over passes of active blocks */
    uint64_t pairs;           /* sum over passes of ray-block pairs */
    uint64_t evicted;         /* cache slots reclaimed by LRU sweeps */
    uint64_t overflow;        /* passes whose slot supply fell short (0 by construction) */
    uint64_t rays;            /* sum over passes of active rays */
    uint64_t pair_slots;      /* sum over passes of N_act * N_spec (R_BID entries written) */
    uint64_t served_pairs;    /* sum over passes of pairs raytraced */
    uint64_t max_active_blocks; /* largest active-block count of any pass: the cache slots a pass needed */
    uint64_t walk_guard;      /* ray walks (traversal or block raytrace) ended by a step guard instead of
                                 by leaving the domain, the block, or finding their blocks; every step
                                 advances a cell index, so this is 0 unless the walk logic is broken */
    uint64_t coarse_steps;    /* coarse cells the traversal visited (Sec. 3.3): the empty-space distance
                                 byte read per visit */
    uint64_t coarse_masks;    /* of those, the cells with a candidate block, whose isovalue mask word
                                 is read too */
} spr_counters;

/* Per-render summary. */
typedef struct {
    uint32_t w, h;
    uint32_t rays_entered;    /* rays that entered the volume (Sec. 3.2) */
    uint32_t n_active;        /* rays still active */
    uint32_t n_spec;          /* speculation count of the next pass */
    uint32_t passes;          /* passes run */
    uint64_t pairs;           /* ray-block pairs over all passes */
    uint64_t bcmc_blocks;     /* blocks whose fine range contains the isovalue: what decompressing every
                                 block that may hold the surface (the BCMC comparison, Sec. 5) decodes */
    uint64_t iso_coarse_cells; /* coarse cells whose range contains the isovalue (Sec. 3.1): the ones whose
                                 blocks' fine ranges the isovalue masks read */
    uint32_t masks_built;     /* 1: this render built its isovalue masks and empty-space distances;
                                 0: it reads a set that its volume kept from an earlier render with the
                                 same isovalue (both counts above are that set's) */
} spr_render_info;

/* Accumulated device time of one kernel of the pass (profiling mode). */
typedef struct {
    const char *name;         /* static string owned by the library */
    double total_ms;
    uint64_t launches;
} spr_kernel_time;

/* Device memory by what it holds (Sec. 5.3 reports total and cache memory).
 * Kinds: SPR_MEM_COMPRESSED (compressed streams), SPR_MEM_GRIDS (macrocell
 * grids and per-block state: fine and coarse ranges, block-to-slot map, pair
 * counters, visible index, active stamps, the isovalue mask sets a volume
 * keeps), SPR_MEM_RAYS (per-render buffers: ray state, active lists, pair
 * slots, hit records, image, hit buffer, and the isovalue masks and
 * empty-space distances of a render that could not use a kept set),
 * SPR_MEM_CACHE (the decoded-block
 * cache: 256-byte slots, owners, LRU stamps, free stack), SPR_MEM_SCRATCH
 * (pass workspace, control block, batch tables, debug staging). */
#define SPR_MEM_COMPRESSED 0
#define SPR_MEM_GRIDS 1
#define SPR_MEM_RAYS 2
#define SPR_MEM_CACHE 3
#define SPR_MEM_SCRATCH 4
#define SPR_MEM_KINDS 5
typedef struct {
    size_t current[SPR_MEM_KINDS];   /* bytes held now, by kind */
    size_t at_peak[SPR_MEM_KINDS];   /* bytes by kind at the moment the total peaked (they sum to peak) */
    size_t kind_peak[SPR_MEM_KINDS]; /* each kind's own high-water mark */
    size_t total, peak;              /* as spr_mem_stats */
} spr_mem_split;

/* ---------------------------------------------------------------- context */
spr_status spr_ctx_create(const spr_config *cfg, spr_ctx **out);
spr_status spr_ctx_destroy(spr_ctx *ctx);
/* Device bytes currently held by the context and its objects, and the peak. */
spr_status spr_mem_stats(spr_ctx *ctx, size_t *current, size_t *peak);
/* The same bytes split by kind (see spr_mem_split).  With reset_peak != 0 the
 * peaks are set to the current values after they are reported, so that a
 * later call reports the peak of what ran in between.  No device call. */
spr_status spr_mem_split_get(spr_ctx *ctx, spr_mem_split *out, int reset_peak);
/* Cumulative counters (synchronises). */
spr_status spr_ctx_counters(spr_ctx *ctx, spr_counters *out);
/* Profiling mode: when enabled, passes run eagerly (not from a captured
 * graph) with a HIP event recorded on the context stream before and after
 * every kernel, also around the load-path kernels of spr_volume_build_grids
 * and the set-up kernels of spr_render_begin; the events are read back
 * lazily (no host synchronisation per pass) and per-kernel device times
 * accumulate until reset. */
spr_status spr_ctx_profile(spr_ctx *ctx, int enable, int reset);
/* Copy up to max per-kernel totals (synchronises); *n = kernels reported. */
spr_status spr_ctx_kernel_times(spr_ctx *ctx, spr_kernel_time *out, uint32_t max, uint32_t *n);

/* Launch tuning of the block raytrace (Sec. 3.7, Sec. 4.3), for batching and
 * the autotuner: each workgroup takes pairs_per_wg sorted pairs (128 or 256)
 * and stages the dual grids of up to slot_tile distinct blocks in LDS (16 or
 * 32); slot_tile 0 stages nothing: each pair reads its cells' corners from
 * the cache slots, the next cell's while the current one is tested.  The
 * image does not depend on either.  Applies to passes enqueued after the
 * call (captured pass graphs are re-recorded).  Defaults 256 / 0.
 * SPR_E_INVALID for other values. */
typedef struct {
    uint32_t pairs_per_wg;
    uint32_t slot_tile;
} spr_tuning;
spr_status spr_ctx_set_tuning(spr_ctx *ctx, const spr_tuning *t);
spr_status spr_ctx_get_tuning(spr_ctx *ctx, spr_tuning *out);

/* ----------------------------------------------------------------- volume */
/* Upload a compressed volume and build its macrocell grids (Sec. 3.1): every
 * block is decoded once to get its value range; the fine grid (one cell per
 * block) unions each block's range with its +x/+y/+z neighbours' (the 2x2x2
 * block neighbourhood), and the coarse grid (one cell per 4^3 blocks) unions
 * the fine ranges inside it.  host_stream is read before the call returns.
 * Errors: SPR_E_INVALID (bad descriptor), SPR_E_CORRUPT (bytes != expected
 * stream size), SPR_E_OOM. */
spr_status spr_volume_load(spr_ctx *ctx, const void *host_stream, size_t bytes, const spr_volume_desc *desc,
                           spr_volume **out);
spr_status spr_volume_free(spr_volume *vol);
/* Recompute the macrocell grids of a resident volume from its device stream
 * (the same load-time step as spr_volume_load, without the host upload).
 * Enqueued; must not overlap a pass that reads the grids. */
spr_status spr_volume_build_grids(spr_volume *vol);
/* Debug/parity: copy the fine (per block) and coarse (per 4^3 blocks) value
 * ranges, as interleaved (lo, hi) float pairs, into host buffers of
 * fine_count / coarse_count pairs (NULL to skip).  Synchronises. */
spr_status spr_volume_ranges(spr_volume *vol, float *fine_lohi, size_t fine_count, float *coarse_lohi,
                             size_t coarse_count);
/* Debug/parity: decode n listed blocks with the device decoder (the block
 * decompression of Sec. 3.5, run outside a pass) into host_out[i*64 ..
 * i*64+63] (raster order x + 4y + 16z).  ids and host_out are host arrays of
 * n entries and n*64 floats, owned by the caller.  SPR_E_INVALID for an id
 * outside the volume; device staging comes from the context's allocator
 * (SPR_E_OOM if it fails).  Synchronises. */
spr_status spr_debug_decode_blocks(spr_volume *vol, const uint32_t *ids, uint32_t n, float *host_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as spr_debug_decode_blocks, with the same arguments, ownership and
 * output, and no allocation.  Its device staging (the n block ids and their
 * n*64 decoded floats) is a fixed buffer that the library holds per GPU from
 * the first context created on that GPU until the process ends
 * (SPR_NOALLOC_MAX_BLOCKS * 260 bytes, 4.06 MiB plus alignment).  Every call
 * on one GPU shares that buffer, which keeps the last call's contents, so
 * calls that overlap on one GPU (several threads, or contexts on different
 * streams) race; calls from one thread at a time are safe.  SPR_E_CAPACITY
 * for n > SPR_NOALLOC_MAX_BLOCKS, SPR_E_INVALID for an id outside the volume
 * (both checked before any device work).  Synchronises. */
#define SPR_NOALLOC_MAX_BLOCKS 16384u
spr_status spr_debug_decode_blocks_noalloc(spr_volume *vol, const uint32_t *ids, uint32_t n, float *host_out);

/* Debug/parity: sqrt(x[i]) and x[i] / y[i] in fp64 on the device, compiled
 * exactly like the hit test (which relies on IEEE correctly rounded fp64
 * division and square root); n values, host arrays.  Synchronises. */
spr_status spr_debug_fp64_ops(spr_ctx *ctx, const double *x, const double *y, size_t n, double *sqrt_out,
                              double *div_out);

/* ----------------------------------------------------------------- render */
/* Start a render: computes every pixel's ray and its entry into the volume
 * (Sec. 3.2); rays that miss are terminated, the image is cleared to 0 and
 * the hit buffer to "no hit".  w*h must be < 2^24; the camera must not look
 * along its up vector.  isovalue is compared in float32.
 * The render also needs the volume's isovalue masks and empty-space
 * distances (one u64 and one byte per coarse cell, derived from the grids of
 * Sec. 3.1 and the isovalue).  A volume keeps up to 4 such sets, one per
 * isovalue (compared bitwise): a render whose isovalue has a kept set reads
 * it; otherwise it builds one into the least recently used set that no live
 * render reads, or into buffers of its own when every set is in use.
 * spr_volume_build_grids drops the kept sets' keys; spr_volume_free frees
 * them. */
spr_status spr_render_begin(spr_volume *vol, const spr_camera *cam, float isovalue, uint32_t w, uint32_t h,
                            spr_render **out);
/* Speculation cap of this render (Sec. 4 caps N_spec at 64); 1 disables
 * speculation.  Only before the first pass.  SPR_E_STATE afterwards. */
spr_status spr_render_set_spec_cap(spr_render *r, uint32_t cap);
/* Speculation policy of this render, only before the first pass
 * (SPR_E_STATE afterwards).  SPR_SPEC_UNIFORM (the default): one count for
 * every ray, N_spec = clamp(floor(w*h / N_act), 1, cap) (Sec. 4).
 * SPR_SPEC_PER_RAY: a count per ray, the per-ray speculation count that the
 * paper's conclusion leaves as future work; this library's rule gives ray i
 * n_i = min(cap, 1 + floor((w*h - N_act) * w_i / W)), where w_i =
 * 1 + floor((t_exit - t_i) / 4) is its remaining path in block lengths from
 * where its remaining walk starts (t_i) and W the sum over the active rays, so
 * every ray gets at least one slot and all of them at most w*h.  The image
 * does not depend on the policy; the passes and their work do. */
#define SPR_SPEC_UNIFORM 0u
#define SPR_SPEC_PER_RAY 1u
spr_status spr_render_set_spec_policy(spr_render *r, uint32_t policy);
/* Enqueue one pass (Sec. 3 (a)-(f), Sec. 4): speculative traversal, mark
 * visible/active blocks, LRU cache update and decompression of misses, build
 * the per-block ray lists, raytrace visible blocks, depth composite, count
 * and compact the active rays and update N_spec.  A pass on a finished
 * render does nothing.  With opt_stats != NULL the call synchronises and
 * fills the counters. */
spr_status spr_render_pass(spr_render *r, spr_pass_stats *opt_stats);
/* Synchronise and report whether every ray has terminated: the count of
 * active rays after the last pass (Sec. 3 step (f) counts the rays still
 * active; the render is complete when none is left) is 0. */
spr_status spr_render_done(spr_render *r, int *done);
/* Run passes until done or max_passes; *passes_run = passes executed.
 * Synchronises. */
spr_status spr_render_run(spr_render *r, uint32_t max_passes, uint32_t *passes_run);
/* Summary of a render (synchronises). */
spr_status spr_render_get_info(spr_render *r, spr_render_info *out);
/* Copy the RGBA8 image (w*h*4 bytes, row 0 at the top, r in the low byte)
 * or the hit buffer (w*h records) to host memory.  The image after any pass
 * is the progressive partial image (Sec. 3: pixels whose rays have
 * terminated are final, the rest are background); the hit buffer holds
 * each finished ray's hit (Sec. 3.7: parameter t, the hit block and the dual
 * cell within it).  bytes / count must equal w*h*4 / w*h (SPR_E_INVALID
 * otherwise); the caller owns the buffers.  Synchronises. */
spr_status spr_read_image(spr_render *r, uint8_t *rgba, size_t bytes);
spr_status spr_read_hits(spr_render *r, spr_hit *hits, size_t count);
/* Device pointers of the image (uint32 RGBA per pixel) and hit buffer; valid
 * until the render is freed; contents change with each pass. */
spr_status spr_render_device_ptrs(spr_render *r, void **rgba, void **hits);
spr_status spr_render_free(spr_render *r);

/* ------------------------------------------------------------------ batch */
/* A batch advances many renders (any volumes and image sizes of one
 * context) by one pass per call, with one launch sequence for all of them;
 * the launch sequence of a pass is captured once into a HIP graph and
 * replayed.  The renders stay owned by the caller and must outlive the batch;
 * each may belong to at most one live batch. */
spr_status spr_batch_create(spr_ctx *ctx, uint32_t n, spr_render *const *renders, spr_batch **out);
/* An empty batch with room for max_requests renders totalling max_pixels
 * pixels (continuous batching: members change with spr_batch_set between
 * passes while the captured pass is reused). */
spr_status spr_batch_create_empty(spr_ctx *ctx, uint32_t max_requests, uint64_t max_pixels, spr_batch **out);
/* Replace the members of a batch (0..capacity renders of the batch's
 * context; a render may belong to one batch at a time).  Renders keep their
 * progress when they join or leave.  Synchronises; SPR_E_CAPACITY if the
 * renders exceed the batch's request or pixel capacity. */
spr_status spr_batch_set(spr_batch *b, uint32_t n, spr_render *const *renders);
/* One pass of every unfinished render; synchronises and reports how many
 * renders are still unfinished. */
spr_status spr_batch_pass(spr_batch *b, uint32_t *n_unfinished);
/* Passes until every render is done or max_passes; polls completion every
 * poll_every passes (0 -> 1).  Synchronises. */
spr_status spr_batch_run(spr_batch *b, uint32_t max_passes, uint32_t poll_every, uint32_t *passes_run);
/* Progress of one batch member after the last pass. */
typedef struct {
    uint32_t n_active;    /* rays still active (0 = finished) */
    uint32_t passes;      /* passes run */
    uint32_t last_pairs;  /* ray-block pairs of the last pass */
    uint32_t n_spec;      /* N_spec for the next pass (Sec. 4) */
} spr_member_state;
/* Every member's progress, in member order (n = member count), and the
 * active blocks of the last pass: the cache slots it needed (Sec. 3.4),
 * which a server's admission control estimates from.  One gather kernel and
 * one copy; synchronises. */
spr_status spr_batch_state(spr_batch *b, spr_member_state *out, uint32_t n, uint32_t *active_blocks);
spr_status spr_batch_free(spr_batch *b);

/* Thread-local message of the last failing call on this thread. */
const char *spr_last_error(void);
/* Library version string. */
const char *spr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPR_H */
