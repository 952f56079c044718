// spr_launch.h — host-side launchers of the libspr kernels (one stream each).
#pragma once

#include "spr_internal.h"

namespace spr {

// Fixed launch shapes of a pass; every kernel loops over its device-side
// count, so one shape serves every pass and the sequence can be replayed as
// a captured graph.
struct PassGrids {
    uint32_t rays;      // 256-thread groups over the active-ray space
    uint32_t pairs;     // 256-thread groups over the pair space
    uint32_t dedupe;    // 256-thread groups over the pair space, DD_ITEMS pairs per thread
    uint32_t slots;     // 256-thread groups over cache slots (eviction sweeps)
    uint32_t assign;    // 256-thread groups assigning slots to misses
    uint32_t scatter;   // 256-thread groups scattering pairs
    uint32_t decode;    // 64-thread groups decoding misses (one thread per block)
    uint32_t rt;        // raytrace workgroups
    uint32_t rt_tile;   // sorted pairs per raytrace workgroup: 128 or 256
    uint32_t rt_lb;     // blocks staged in LDS per raytrace tile: 16 or 32, 0 = no staging
    uint64_t max_P;     // pair capacity the shape was made for
};

hipError_t launch_decode_ids(hipStream_t s, const VolDev &V, const uint32_t *ids, uint32_t n, float *out);
hipError_t launch_fp64_ops(hipStream_t s, const double *x, const double *y, uint64_t n, double *sq, double *dv);
// Load path: block ranges, fine grid, coarse grid.  ev == nullptr: plain
// launches; else ev[i] is recorded before kernel i and ev[3] after the last.
hipError_t launch_load_grids(hipStream_t s, const VolDev &V, hipEvent_t *ev = nullptr);
// Members' progress of a table into out[0..n] (see k_gather_state).
hipError_t launch_gather_state(hipStream_t s, const PassCtl *ctl, const Table &T, uint32_t n, uint4 *out);
// Stream-ordered set-up writes: *dq = q; if ds, *ds = *st (zero if st is null); if hdr, *hdr = hv.
hipError_t launch_put_req(hipStream_t s, ReqDev *dq, const ReqDev &q, ReqState *ds, const ReqState *st,
                          uint32_t *hdr, uint32_t hv);
hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t v);
hipError_t launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t n, uint64_t v);
hipError_t launch_iota_u32(hipStream_t s, uint32_t *p, uint64_t n);
hipError_t launch_release_volume(hipStream_t s, PassCtl *ctl, const Cache &C, uint32_t vol);
// Isovalue masks of the table's first request (when build_masks), then the
// initial-ray pass (pass set-up, initial rays, count, compaction); ev as for
// the load path, one event before each timed group and one after the last
// (6 events with the masks, 5 without).
hipError_t launch_init_rays(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols, uint64_t mask_words,
                            bool build_masks, hipEvent_t *ev = nullptr);
constexpr int PASS_KERNELS = 12;
extern const char *const PASS_KERNEL_NAMES[PASS_KERNELS];
// Profiling slots: the pass kernels, then the load-path and set-up kernels
// that run outside a pass.
constexpr int PROF_SLOTS = PASS_KERNELS + 5;
extern const char *const PROF_NAMES[PROF_SLOTS];
constexpr int LOAD_SLOTS[3] = {PASS_KERNELS, PASS_KERNELS + 1, PASS_KERNELS + 2};   // block ranges, fine grid, coarse grid
// masks, pass begin, initial rays, pass end, compact (INIT_SLOTS + 1: without the masks)
constexpr int INIT_SLOTS[5] = {PASS_KERNELS + 3, 0, PASS_KERNELS + 4, PASS_KERNELS - 2, PASS_KERNELS - 1};
// ev == nullptr: plain launches; else ev[i] is recorded before kernel i and
// ev[PASS_KERNELS] after the last one.
hipError_t launch_pass(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols, const Work &W,
                       const Cache &C, const PassGrids &g, hipEvent_t *ev);

}  // namespace spr
