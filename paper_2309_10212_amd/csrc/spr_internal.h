// spr_internal.h — device-side data layout and inline device routines of
// libspr (speculative progressive isosurface raycasting, arXiv 2309.10212).
//
// Everything here is GPU-path code.  It is compiled with hipcc for gfx950
// with -ffp-contract=off so that every fp64 expression below evaluates in the
// written order with IEEE rounding; the hit decision per dual cell depends on
// that (the canonical forms are documented beside each routine).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spr.h"

namespace spr {

constexpr uint32_t NONE = 0xFFFFFFFFu;          // no block / empty slot
constexpr uint32_t RAY_NOT_STARTED = 0xFFFFFFFFu;
constexpr uint32_t RAY_DONE = 0xFFFFFFFEu;
constexpr int MAX_VOLUMES = 64;
constexpr int MAX_REQS = 256;                   // requests per launch table
constexpr int WAVE = 64;

// ------------------------------------------------------------ device data --

// One loaded volume.  Block ids are local to the volume (bx + nbx*(by + nby*bz)).
struct VolDev {
    const uint32_t *stream;     // nblocks records of rec_words 32-bit words
    float2 *fine;               // per block: union of the ranges of the 2x2x2 block neighbourhood
    float2 *coarse;             // per 4^3 blocks: union of fine ranges
    uint32_t *map;              // per block: cache slot or NONE
    uint32_t *blk_cnt;          // per block: pairs on it in the current pass (0 between passes)
    uint32_t *vis_idx;          // per block: index in that pass's visible list
    uint64_t *claim;            // per coarse cell: bit (bx&3) + 4(by&3) + 16(bz&3) set once that block
                                // was claimed active in the current pass (0 between passes)
    int n[3];                   // samples per axis
    int nb[3];                  // blocks per axis, ceil(n/4)
    int nc[3];                  // coarse cells per axis, ceil(nb/4)
    int tb[3];                  // blocks that own dual cells, ceil((n-1)/4)
    int tc[3];                  // coarse cells that own dual cells, ceil(tb/4)
    int rate;                   // bits per value (32 = raw)
    int rec_words;              // 2*rate
    uint64_t nblocks;
    uint32_t live;
    uint32_t pad;
};

// Index of block (bx, by, bz) in the per-block state arrays (map, blk_cnt,
// vis_idx): the 64 blocks of a coarse cell are contiguous, at
// (bx&3) + 4(by&3) + 16(bz&3) (the order of the isovalue mask bits), and the
// coarse cells follow in raster order, so a block's +x/+y/+z neighbourhood
// mostly lies in the same 256 bytes.  Block ids everywhere else are linear,
// (bz*nb[1] + by)*nb[0] + bx.
__device__ __forceinline__ uint32_t bidx_xyz(const VolDev &V, int bx, int by, int bz) {
    const uint32_t cell = ((uint32_t)(bz >> 2) * (uint32_t)V.nc[1] + (uint32_t)(by >> 2)) * (uint32_t)V.nc[0] +
                          (uint32_t)(bx >> 2);
    return cell * 64u + (uint32_t)((bx & 3) | ((by & 3) << 2) | ((bz & 3) << 4));
}

__device__ __forceinline__ uint32_t bidx(const VolDev &V, uint32_t b) {
    const uint32_t nb0 = (uint32_t)V.nb[0], nb1 = (uint32_t)V.nb[1];
    const uint32_t r = b / nb0;
    return bidx_xyz(V, (int)(b - r * nb0), (int)(r % nb1), (int)(r / nb1));
}

// The fields of a volume that the per-block bookkeeping kernels use, read
// once into registers.  Read through a reference into device memory, they
// are reloaded after every store or atomic (the compiler cannot rule out that
// the store changed them), which puts several dependent round trips to memory
// in front of every access.
struct VolState {
    uint32_t *map, *blk_cnt, *vis_idx;
    uint64_t *claim;
    int nb0, nb1, nb2, nc0, nc1;
};

__device__ __forceinline__ VolState vol_state(const VolDev &V) {
    VolState s;
    s.map = V.map; s.blk_cnt = V.blk_cnt; s.vis_idx = V.vis_idx; s.claim = V.claim;
    s.nb0 = V.nb[0]; s.nb1 = V.nb[1]; s.nb2 = V.nb[2]; s.nc0 = V.nc[0]; s.nc1 = V.nc[1];
    return s;
}

__device__ __forceinline__ uint32_t bidx_xyz(const VolState &S, int bx, int by, int bz) {
    const uint32_t cell = ((uint32_t)(bz >> 2) * (uint32_t)S.nc1 + (uint32_t)(by >> 2)) * (uint32_t)S.nc0 +
                          (uint32_t)(bx >> 2);
    return cell * 64u + (uint32_t)((bx & 3) | ((by & 3) << 2) | ((bz & 3) << 4));
}

__device__ __forceinline__ uint32_t bidx(const VolState &S, uint32_t b) {
    const uint32_t nb0 = (uint32_t)S.nb0, nb1 = (uint32_t)S.nb1;
    const uint32_t r = b / nb0;
    return bidx_xyz(S, (int)(b - r * nb0), (int)(r % nb1), (int)(r / nb1));
}

// Entries of each per-block state array (whole coarse cells).
inline uint64_t bidx_count(const VolDev &V) { return (uint64_t)V.nc[0] * V.nc[1] * V.nc[2] * 64u; }

// Mutable per-render state kept on the device (no host round trip per pass).
struct ReqState {
    uint32_t n_act;             // active rays for the next pass
    uint32_t n_spec;            // speculation count for the next pass
    uint32_t cur;               // which of the two active-ray lists is current
    uint32_t passes;            // passes run
    uint32_t n_act_prev;        // active rays at the start of the last pass
    uint32_t last_pairs, last_deferred, last_terminated, last_nspec;
    uint32_t entered;           // rays that entered the volume (set at the first pass)
    uint32_t segs;              // traversal lanes per active ray this pass (power of two, <= 16)
    uint32_t slot_cursor;       // pair slots handed out this pass (per-ray counts: by the traversal)
    uint32_t last_slots;        // pair slots of the last pass (the sum of the rays' counts)
    uint32_t pad[1];
    unsigned long long tot_pairs;
    unsigned long long bcmc;    // blocks whose fine range contains the isovalue (set up with the masks)
    unsigned long long ccells;  // coarse cells whose range contains the isovalue (their fine ranges were read)
    unsigned long long wsum;    // sum of the active rays' weights for the next pass (per-ray counts)
};

// Speculation policy of a render: one count for every ray (Sec. 4), or
// per-ray counts from the rays' remaining paths.
constexpr uint32_t SPEC_UNIFORM = 0, SPEC_PER_RAY = 1;

// Weight of a ray whose remaining walk starts at t: its remaining path in
// block lengths, 1 + floor((t_exit - t) / 4), and 1 once t >= t_exit.
__device__ __forceinline__ uint32_t ray_weight(double t, double t_exit) {
    return t < t_exit ? 1u + (uint32_t)floor((t_exit - t) * 0.25) : 1u;
}

// Per-ray count min(cap, 1 + floor((B - N) * w / W)): at least one slot per
// ray, at most B over all N rays (W is the sum of their weights).
__device__ __forceinline__ uint32_t nspec_ray(uint32_t B, uint32_t N, unsigned long long W, uint32_t w, uint32_t cap) {
    const unsigned long long extra = (B > N && W) ? ((unsigned long long)(B - N) * w) / W : 0ull;
    const unsigned long long n = 1ull + extra;
    return n < cap ? (uint32_t)n : cap;
}

// Immutable per-render description (camera basis computed on the host).
struct ReqDev {
    double eye[3], fwd[3], right[3], upv[3];
    double sx, sy;
    float iso;
    uint32_t w, h, npix;
    uint32_t vol;               // index in the context's volume table
    uint32_t spec_cap;
    uint32_t policy;            // SPEC_UNIFORM or SPEC_PER_RAY
    uint32_t mstat_load;        // with mstat: 1 when the masks were built by an earlier render
    uint32_t *ray_state;        // per pixel: last served block, RAY_NOT_STARTED, RAY_DONE
    uint32_t *act[2];           // compacted active pixel lists
    uint32_t *pair_blk;         // per pair slot (R_BID of Sec. 3.3/4.1)
    double *tslot;              // per pair slot: the hit parameter t, written by hit pairs only
    uint64_t *best;             // per pixel: minimum over this pass's hits of
                                // pair slot << 38 | cell << 32 | rgba, ~0 for none
    uint32_t *nfound;           // per pixel: candidate blocks the traversal found this pass
    uint32_t *def_first;        // per pixel: first deferred slot of the ray this pass (NONE between passes)
    uint32_t *rbase;            // per pixel: the ray's first pair slot this pass
    uint32_t *rns;              // per pixel: the ray's speculation count this pass
    uint32_t *rw;               // per pixel: the ray's weight this pass (per-ray counts)
    uint32_t *pair_ray;         // per pair slot: active-ray index of its ray (per-ray counts)
    uint32_t *image;            // RGBA8 per pixel
    spr_hit *hits;              // per pixel
    ReqState *st;
    uint64_t *cmask64;          // per coarse cell: bit (bx&3) + 4(by&3) + 16(bz&3) set when that
                                // block's fine range contains iso (0 when the coarse range does not)
    uint8_t *cdist;             // per coarse cell: chessboard distance (in coarse cells, capped at
                                // CD_MAX) to the nearest coarse cell with a nonzero mask; a second
                                // nc bytes after it are scratch for the separable passes
    unsigned long long *mstat;  // counts of a mask set the volume keeps (bcmc, ccells), or null
                                // when the masks are the render's own
};

constexpr int CD_MAX = 15;

// Per-pass control block of a context (counters reset at each pass start).
struct PassCtl {
    uint32_t pass;              // global pass stamp (starts at 1)
    uint32_t nreq;
    uint32_t A;                 // active-ray index space of this pass (64-padded per request)
    uint32_t P;                 // pair index space of this pass
    uint32_t n_vis;             // visible blocks appended
    uint32_t v_adm;             // visible blocks admitted (served) this pass
    uint32_t n_actblk;          // active blocks appended
    uint32_t n_miss;            // misses appended
    uint32_t n_hit;
    uint32_t cursor;            // sorted-pair allocation cursor
    uint32_t served;            // served pairs
    uint32_t deferred;          // pairs on unserved blocks
    uint32_t n_slots;
    uint32_t free_top;          // entries in the free-slot stack
    uint32_t assign_base;       // misses take free_stack[assign_base + i]
    uint32_t need;              // slots to reclaim by eviction this pass
    uint32_t evict_T;           // evict occupied slots of age >= evict_T
    uint32_t evict_done_blocks; // ticket for the histogram's last block
    uint32_t evicted;
    uint32_t terminated;
    uint32_t pairs;
    uint32_t overflow;          // set if the slot supply ever fell short (never by construction)
    uint32_t assigned;          // misses that received a slot this pass
    uint32_t rays;              // active rays of this pass (unpadded)
    uint32_t A_trav;            // traversal lane space of this pass (64-padded per request)
    uint32_t guard;             // walks ended by a step guard (never by construction: every
                                // step advances a cell index within the domain)
    uint32_t csteps;            // coarse cells the traversal visited (one distance byte read each)
    uint32_t cmasks;            // of those, the nonempty ones (their mask word read too)
    uint32_t pad[4];
    uint32_t hist[64];
    // cumulative counters since context creation
    unsigned long long acc_passes, acc_decoded, acc_visible, acc_active, acc_pairs, acc_evicted, acc_overflow,
        acc_rays, acc_slots, acc_served, acc_max_active, acc_guard, acc_csteps, acc_cmasks;
};

// Launch table of a pass: the requests advanced together.
struct Table {
    ReqDev *reqs;               // up to cap entries
    uint32_t *hdr;              // hdr[0] = current number of requests (device-resident,
                                // so membership can change between graph replays)
    uint32_t *act_base;         // cap+1, 64-aligned prefix of n_act
    uint32_t *pair_base;        // cap+1, prefix of n_act*n_spec
    uint32_t *trav_base;        // cap+1, 64-aligned prefix of n_act*segs (traversal lanes)
    uint32_t *big_base;         // cap+1, prefix of n_act*segs over the requests whose segmented
                                // lanes list more candidates than the LDS buffer holds (their
                                // rows of Work::seg_buf)
    uint4 *wave_rec;            // per 64-entry wave of the A space, accumulated during a pass
                                // and cleared by its compaction: {alive rays (initial-ray pass
                                // only), pairs, deferred pairs, terminated rays}
    uint32_t *wave_off;         // exclusive prefix of the survivors
    uint32_t *wave_w;           // per wave of the A space: summed weights of its rays for the next pass
                                // (per-ray counts; cleared by the compaction like the records)
    uint32_t *host_nact;        // single-render tables: a fine-grained host word the pass end
                                // writes request 0's active-ray count to (the host polls it);
                                // null for batches
    uint32_t cap;               // request capacity
    uint32_t max_A;             // capacity of the A space (sum of padded npix)
    uint32_t max_P;             // capacity of the pair space (sum of npix)
};

// Segmented traversal (several lanes per ray, for passes with few active
// rays) of requests whose speculation count exceeds the lanes' LDS buffer:
// at most SEG_BIG_LANES such lanes per pass, each listing at most
// SEG_BIG_NS candidates.
constexpr uint32_t SEG_BIG_LANES = 65536;
constexpr uint32_t SEG_BIG_NS = 64;

// Context-level scratch for one pass, sized for the largest table.
struct Work {
    uint64_t *vis_list;         // (vol << 32) | block
    uint32_t *vis_off;          // start of the block's run in the sorted pairs
    uint64_t *miss_list;        // misses (vol << 32) | block
    uint32_t *miss_slot;
    uint32_t *pair_rank;        // per pair index: rank within its block
    uint32_t *s_ray;            // sorted pairs: (req << 24) | pixel
    uint32_t *s_q;              // sorted pairs: pair slot within the request
    uint32_t *s_vi;             // sorted pairs: visible-list index
    uint32_t *vis_nsl;          // per visible block: slots of its 2x2x2 block neighbourhood (8, NONE outside)
    uint32_t *seg_buf;          // SEG_BIG_NS x SEG_BIG_LANES: candidates of segmented traversal lanes
                                // beyond the LDS buffer, entry k of lane l at [k * SEG_BIG_LANES + l]
    uint32_t cap_P;             // pairs capacity
    uint32_t cap_K;             // active/miss list capacity
};

struct Cache {
    float *slots;               // n_slots * 64 floats
    uint64_t *owner;            // per slot: (vol << 32) | block, or ~0
    uint32_t *stamp;            // per slot: last pass used
    uint32_t *free_stack;
    uint32_t n_slots;
};

// ---------------------------------------------------------- wave helpers --

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-uniform values in scalar registers.  Fields read through generic
// pointers are otherwise treated as per-lane and kept in vector registers
// (or re-loaded inside loops); every caller guarantees the value is the same
// across the wave.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x))); }
// readfirstlane returns int: both halves are zero-extended (a sign-extended
// low word would set the upper 32 bits of every value with bit 31 set).
__device__ __forceinline__ uint64_t uni(uint64_t x) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}
__device__ __forceinline__ double uni(double x) { return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(x))); }
template <class T>
__device__ __forceinline__ T *uni(T *p) { return (T *)uni((uint64_t)p); }

// Device-memory pointers read from structures are generic (flat) pointers;
// flat accesses count against both the memory and the LDS wait counters.
// Casting to the global address space gives global_* instructions, which a
// later LDS wait does not have to drain.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p) { return (gptr<T>)p; }

// The camera and volume fields one wave needs, read once into scalar
// registers (all lanes of a wave serve the same request).
struct WaveReq {
    double eye[3], fwd[3], right[3], upv[3];
    double sx, sy;
    uint32_t w, h;
    int n[3], nb[3], nc[3], tb[3], tc[3];
};

__device__ __forceinline__ void load_wave_req(const ReqDev &q, const VolDev &V, WaveReq &u) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u.eye[a] = uni(q.eye[a]); u.fwd[a] = uni(q.fwd[a]); u.right[a] = uni(q.right[a]); u.upv[a] = uni(q.upv[a]);
        u.n[a] = uni(V.n[a]); u.nb[a] = uni(V.nb[a]); u.nc[a] = uni(V.nc[a]); u.tb[a] = uni(V.tb[a]); u.tc[a] = uni(V.tc[a]);
    }
    u.sx = uni(q.sx); u.sy = uni(q.sy);
    u.w = uni(q.w); u.h = uni(q.h);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Block-aggregated bump allocation.  Every thread of the workgroup calls it
// (block-uniform control flow) with a count and receives the start of its run
// of `cnt` entries; the workgroup issues a single atomic on *counter.  Device
// atomics on one address serialise (about 12 ns each on this chip, measured),
// so appends aggregate per workgroup, not per wave.  s_tmp: BS/64 + 1 words.
template <int BS>
__device__ __forceinline__ uint32_t block_bump(uint32_t *counter, uint32_t cnt, uint32_t *s_tmp) {
    static_assert(BS % 64 == 0 && BS <= 4096, "block_bump: workgroup of whole waves, at most 64 of them");
    constexpr uint32_t NW = BS / 64;
    const uint32_t l = lane_id(), w = threadIdx.x >> 6;
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off);
        if ((int)l >= off) incl += o;
    }
    if (l == 63) s_tmp[w] = incl;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t v = l < NW ? s_tmp[l] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t o = __shfl_up(x, off);
            if ((int)l >= off) x += o;
        }
        if (l < NW) s_tmp[l] = x - v;
        if (l == 63) s_tmp[NW] = x ? atomicAdd(counter, x) : 0u;
    }
    __syncthreads();
    const uint32_t r = s_tmp[NW] + s_tmp[w] + incl - cnt;
    __syncthreads();   // s_tmp may be reused right away
    return r;
}

// block_bump for two counters at once (one scan, both atomics issued by one
// lane back to back): returns the starts of the thread's runs of na entries
// on *ca and nb entries on *cb.  s_tmp: BS/64 + 1 entries.
template <int BS>
__device__ __forceinline__ uint2 block_bump2(uint32_t *ca, uint32_t na, uint32_t *cb, uint32_t nb, uint2 *s_tmp) {
    static_assert(BS % 64 == 0 && BS <= 4096, "block_bump2: workgroup of whole waves, at most 64 of them");
    constexpr uint32_t NW = BS / 64;
    const uint32_t l = lane_id(), w = threadIdx.x >> 6;
    uint32_t ia = na, ib = nb;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t oa = __shfl_up(ia, off), ob = __shfl_up(ib, off);
        if ((int)l >= off) { ia += oa; ib += ob; }
    }
    if (l == 63) s_tmp[w] = make_uint2(ia, ib);
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint2 v = l < NW ? s_tmp[l] : make_uint2(0u, 0u);
        uint32_t xa = v.x, xb = v.y;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t oa = __shfl_up(xa, off), ob = __shfl_up(xb, off);
            if ((int)l >= off) { xa += oa; xb += ob; }
        }
        if (l < NW) s_tmp[l] = make_uint2(xa - v.x, xb - v.y);
        if (l == 63) s_tmp[NW] = make_uint2(xa ? atomicAdd(ca, xa) : 0u, xb ? atomicAdd(cb, xb) : 0u);
    }
    __syncthreads();
    const uint2 r = make_uint2(s_tmp[NW].x + s_tmp[w].x + ia - na, s_tmp[NW].y + s_tmp[w].y + ib - nb);
    __syncthreads();   // s_tmp may be reused right away
    return r;
}

// Wave-aggregated append: every active lane calls it; lanes with want get
// consecutive indices from one atomic on *counter.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool want) {
    uint64_t m = __ballot(want);
    if (m == 0) return NONE;
    uint64_t act = __ballot(1);
    int leader = __ffsll((unsigned long long)act) - 1;
    uint32_t base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    return want ? base + (uint32_t)__popcll(m & lanemask_lt()) : NONE;
}

// ------------------------------------------------------------ ray set-up --
// Camera model (Sec. 3.2 computes per-pixel rays; the pinhole form is this
// library's reading): for pixel (px, py), row 0 at the top,
//   x = ((2(px + 1/2))/w - 1) * sx,   y = (1 - (2(py + 1/2))/h) * sy,
//   v = (fwd + x right) + y up,       d = v * (1 / sqrt((vx^2 + vy^2) + vz^2)),
// all in fp64 in exactly this order; components below 1e-290 in magnitude are
// set to 0 (the ray is parallel to that axis); r_a = 1/d_a.  t_enter/t_exit come from
// the slab test against the sample domain [0, n-1]^3 with the same plane
// parameter function tau_a(m) = (m - o_a) * r_a used by every walk level.

struct Ray {
    double o[3], d[3], r[3];
    double te, tx;
    int entered;
};

__device__ __forceinline__ double tau_at(const Ray &R, int a, int m) { return ((double)m - R.o[a]) * R.r[a]; }

template <class Cam>
__device__ inline void make_ray(const Cam &q, const int n[3], uint32_t pix, Ray &R) {
    int px = (int)(pix % q.w), py = (int)(pix / q.w);
    double ndx = (2.0 * ((double)px + 0.5)) / (double)q.w - 1.0;
    double ndy = 1.0 - (2.0 * ((double)py + 0.5)) / (double)q.h;
    double x = ndx * q.sx, y = ndy * q.sy;
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = (q.fwd[a] + x * q.right[a]) + y * q.upv[a];
    double inv = 1.0 / sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.o[a] = q.eye[a];
        R.d[a] = v[a] * inv;
        if (fabs(R.d[a]) < 1e-290) R.d[a] = 0.0;   // keeps every 1/d_a finite
        R.r[a] = R.d[a] != 0.0 ? 1.0 / R.d[a] : 0.0;
    }
    double te = 0.0, tx = __builtin_inf();
    int ent = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double np, fp;
        if (R.d[a] > 0.0) { np = tau_at(R, a, 0); fp = tau_at(R, a, n[a] - 1); }
        else if (R.d[a] < 0.0) { np = tau_at(R, a, n[a] - 1); fp = tau_at(R, a, 0); }
        else {
            if (R.o[a] < 0.0 || R.o[a] > (double)(n[a] - 1)) ent = 0;
            continue;
        }
        if (np > te) te = np;
        if (fp < tx) tx = fp;
    }
    if (te > tx) ent = 0;
    R.te = te;
    R.tx = tx;
    R.entered = ent;
}

// ------------------------------------------------- multi-level cell walk --
// A level has cells of S samples per axis (S = 1 dual cells, 4 blocks, 16
// coarse cells) and L[a] cells per axis.  Its plane m sits at S*m, except the
// top plane m = L[a], which is the domain face n-1 (so leaving the domain is
// seen identically at every level).  The cell holding the ray at parameter t
// is, for d > 0, the largest m whose lower plane has tau <= t; for d < 0 the
// smallest m whose upper plane has tau <= t; for d == 0 the cell of the
// origin.  Stepping crosses every plane with tau <= the nearest exit-plane
// parameter, so tied planes are crossed together and all levels see one
// consistent sequence.

struct Level {
    int S;
    int L[3];
    int n[3];
    double invS;   // 1/S, exact: S is 1, 4 or 16
};

__device__ __forceinline__ int plane_pos(const Level &lv, int a, int m) {
    return m >= lv.L[a] ? lv.n[a] - 1 : lv.S * m;
}

__device__ __forceinline__ double tau_plane(const Ray &R, const Level &lv, int a, int m) {
    return tau_at(R, a, plane_pos(lv, a, m));
}

// origin cell on a d == 0 axis, at level S
__device__ __forceinline__ int still_cell(const Ray &R, const Level &lv, int a) {
    double f = floor(R.o[a]);
    int m;
    if (f < 0.0) m = 0;
    else if (f > (double)(lv.n[a] - 2)) m = lv.n[a] - 2;
    else m = (int)f;
    return m / lv.S;
}

// Cell index on axis a at parameter t, within [lo, hi]: d > 0, the largest m
// whose lower plane has tau <= t; d < 0, the smallest m whose upper plane
// has tau <= t (clamped to [lo, hi] when no such m lies there).  The fp64
// position estimate floor((o + t d) / S) is that cell or a neighbour: the
// plane tests only differ from the position order within rounding of a
// plane, and ray positions stay below 2^22 samples (volume extent and eye
// coordinates are at most 2^19).  So the tests of the estimate's two planes
// decide it.
__device__ inline int cell_at(const Ray &R, const Level &lv, int a, double t, int lo, int hi) {
    if (R.d[a] == 0.0) return still_cell(R, lv, a);
    double p = R.o[a] + t * R.d[a];
    int g = (int)floor(p * lv.invS);   // == floor(p / S): S is a power of two
    g = g < lo ? lo : (g > hi ? hi : g);
    const bool lo_x = tau_plane(R, lv, a, g) <= t, hi_x = tau_plane(R, lv, a, g + 1) <= t;
    if (R.d[a] > 0.0) g += (g < hi && hi_x) ? 1 : ((g > lo && !lo_x) ? -1 : 0);
    else g += (g > lo && lo_x) ? -1 : ((g < hi && !hi_x) ? 1 : 0);
    return g;
}

// parameter where the ray leaves cell c (min over axes of the exit planes)
__device__ __forceinline__ double cell_exit(const Ray &R, const Level &lv, const int c[3]) {
    double tn = __builtin_inf();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (R.d[a] > 0.0) { double x = tau_plane(R, lv, a, c[a] + 1); if (x < tn) tn = x; }
        else if (R.d[a] < 0.0) { double x = tau_plane(R, lv, a, c[a]); if (x < tn) tn = x; }
    }
    return tn;
}

// parameter where the ray enters cell c (max of t_enter and the entry planes)
__device__ __forceinline__ double cell_entry(const Ray &R, const Level &lv, const int c[3]) {
    double t0 = R.te;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (R.d[a] > 0.0) { double e = tau_plane(R, lv, a, c[a]); if (e > t0) t0 = e; }
        else if (R.d[a] < 0.0) { double e = tau_plane(R, lv, a, c[a] + 1); if (e > t0) t0 = e; }
    }
    return t0;
}

// Incremental walk at one level: per axis the parameter of the current
// cell's exit plane (+inf where the ray is parallel to the axis), the same
// plane parameters cell_exit computes; a step only recomputes the axes that
// move, with selects instead of per-axis branches.  The step direction comes
// from the sign of d each time (no extra registers).
struct AxisWalk {
    double tex[3];
};

__device__ __forceinline__ int axis_dir(const Ray &R, int a) { return R.d[a] > 0.0 ? 1 : (R.d[a] < 0.0 ? -1 : 0); }

__device__ __forceinline__ double exit_tau(const Ray &R, const Level &lv, int a, int c) {
    const int dir = axis_dir(R, a);
    const double t = tau_plane(R, lv, a, c + (dir > 0 ? 1 : 0));
    return dir != 0 ? t : __builtin_inf();
}

__device__ __forceinline__ void walk_init(const Ray &R, const Level &lv, const int c[3], AxisWalk &w) {
#pragma unroll
    for (int a = 0; a < 3; ++a) w.tex[a] = exit_tau(R, lv, a, c[a]);
}

// exit parameter of the current cell: cell_exit's minimum
__device__ __forceinline__ double walk_exit(const AxisWalk &w) {
    double tn = w.tex[0];
    tn = w.tex[1] < tn ? w.tex[1] : tn;
    tn = w.tex[2] < tn ? w.tex[2] : tn;
    return tn;
}

// Cross every plane with parameter <= tn (tied planes together); false when
// the ray leaves [lo, hi] on some axis.  The same cell and result as
// advance().  One crossing per axis suffices: the next plane of an axis is at
// least one sample further on and |r_a| >= 1 (|d_a| <= 1), so its parameter
// exceeds tn by about |r_a| or more.
__device__ __forceinline__ bool walk_step(const Ray &R, const Level &lv, AxisWalk &w, int c[3], double tn,
                                          const int lo[3], const int hi[3]) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool st = w.tex[a] <= tn;
        c[a] += st ? axis_dir(R, a) : 0;
        ok = ok && !(st && (c[a] < lo[a] || c[a] > hi[a]));
        w.tex[a] = st ? exit_tau(R, lv, a, c[a]) : w.tex[a];
    }
    return ok;
}

// Cross every plane with tau <= tn (one per axis at most, as in walk_step).
// Returns false when the ray leaves [lo, hi] on some axis (for the full
// range: leaves the domain).
__device__ inline bool advance(const Ray &R, const Level &lv, int c[3], double tn, const int lo[3], const int hi[3]) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (R.d[a] > 0.0) {
            if (tau_plane(R, lv, a, c[a] + 1) <= tn) {
                ++c[a];
                ok = ok && c[a] <= hi[a];
            }
        } else if (R.d[a] < 0.0) {
            if (tau_plane(R, lv, a, c[a]) <= tn) {
                --c[a];
                ok = ok && c[a] >= lo[a];
            }
        }
    }
    return ok;
}

// ------------------------------------------------------------ cell test --
// Canonical hit test of dual cell (i,j,k) over [t0, t1] (Sec. 3.7, after
// Marmitt et al.): corners c_{abg} (a fastest) as fp64; local entry point
// (u0,v0,w0) = (o + t0 d) - (i,j,k); each axis factor is linear in
// s in [0, S]: X0 = (1-u0) - s dx, X1 = u0 + s dx; the cubic
// g(s) = A s^3 + B s^2 + C s + D is accumulated corner by corner in index
// order with the products grouped as written below; D -= iso.  Extrema are
// the roots of 3A s^2 + 2B s + C in (0, S); the first exact zero or strict
// sign change over {0, extrema, S} decides the hit.  The root inside the
// bracket is refined by safeguarded Newton-bisection.

struct CellHit {
    int hit;
    int refine;          // the root lies inside the bracket below: refine_hit finds it
    double s;
    double loc[3];
    double A, B, C, D, sa, sb, ga;
};

__device__ __forceinline__ double horner3(double A, double B, double C, double D, double s) {
    return ((A * s + B) * s + C) * s + D;
}

// Root of g(s) = ((A s + B) s + C) s + D in [sa, sb], where g changes sign
// (g(sa) = ga) and is monotone (the bracket lies between consecutive
// extrema).  Safeguarded Newton-Raphson (the Newton-with-bisection scheme of
// Press et al., Numerical Recipes, Sec. 9.4): keep a bracket [lo, hi] with
// g(lo) < 0 < g(hi); take the Newton step when it lands inside the bracket
// and is at most half the step before the last one, else halve the bracket;
// stop when a step is below 1e-12 (1 + |s|) or g is exactly zero.  At most
// a dozen iterations on cell-test cubics, against 40 to 60 for Newton steps
// that only move one end of the bracket.
__device__ inline double refine_root(double A, double B, double C, double D, double sa, double sb, double ga) {
    double lo = ga < 0.0 ? sa : sb, hi = ga < 0.0 ? sb : sa;
    double x = 0.5 * (sa + sb);
    double dxold = fabs(sb - sa), dx = dxold;
    double f = horner3(A, B, C, D, x), df = (3.0 * A * x + 2.0 * B) * x + C;
    for (int it = 0; it < 64; ++it) {
        if (f == 0.0) return x;
        const bool outside = ((x - hi) * df - f) * ((x - lo) * df - f) > 0.0;
        const bool slow = fabs(2.0 * f) > fabs(dxold * df);
        dxold = dx;
        if (outside || slow) {
            dx = 0.5 * (hi - lo);
            x = lo + dx;
            if (x == lo) return x;
        } else {
            dx = f / df;
            const double xp = x;
            x = x - dx;
            if (x == xp) return x;
        }
        if (fabs(dx) < 1e-12 * (1.0 + fabs(x))) return x;
        f = horner3(A, B, C, D, x);
        df = (3.0 * A * x + 2.0 * B) * x + C;
        if (f < 0.0) lo = x;
        else hi = x;
    }
    return x;
}

__device__ inline void test_cell(const Ray &R, const int c[3], double t0, double t1, const float fc[8], float iso,
                                 CellHit &res) {
    res.hit = 0;
    int above = 0, below = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        above += fc[i] > iso;
        below += fc[i] < iso;
    }
    if (above == 8 || below == 8) return;
    if (t1 < t0) return;
    double S = t1 - t0;
    double al[3][2], be[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double l = (R.o[a] + t0 * R.d[a]) - (double)c[a];
        res.loc[a] = l;
        al[a][0] = 1.0 - l;
        be[a][0] = -R.d[a];
        al[a][1] = l;
        be[a][1] = R.d[a];
    }
    double A = 0.0, B = 0.0, C = 0.0, D = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int a = i & 1, b = (i >> 1) & 1, g = (i >> 2) & 1;
        double ax = al[0][a], bx = be[0][a], ay = al[1][b], by = be[1][b], az = al[2][g], bz = be[2][g];
        double td = (ax * ay) * az;
        double tc = ((bx * ay) * az + (ax * by) * az) + (ax * ay) * bz;
        double tb = ((bx * by) * az + (bx * ay) * bz) + (ax * by) * bz;
        double ta = (bx * by) * bz;
        double cv = (double)fc[i];
        D = D + cv * td;
        C = C + cv * tc;
        B = B + cv * tb;
        A = A + cv * ta;
    }
    D = D - (double)iso;
    double cand0 = -1.0, cand1 = -1.0;
    if (A != 0.0) {
        double disc = B * B - (3.0 * A) * C;
        if (disc >= 0.0) {
            double q = -(B + copysign(sqrt(disc), B));
            cand0 = q / (3.0 * A);
            if (q != 0.0) cand1 = C / q;
        }
    } else if (B != 0.0) {
        cand0 = -C / (2.0 * B);
    }
    double e0 = 0.0, e1 = 0.0;
    int ne = 0;
    if (cand0 > 0.0 && cand0 < S) { e0 = cand0; ne = 1; }
    if (cand1 > 0.0 && cand1 < S) {
        if (ne == 0) { e0 = cand1; ne = 1; }
        else {
            if (cand1 < e0) { e1 = e0; e0 = cand1; ne = 2; }
            else if (cand1 > e0) { e1 = cand1; ne = 2; }
        }
    }
    // ordered points {0, e0 (ne >= 1), e1 (ne == 2), S}: first exact zero or
    // strict sign change wins
    double sp = 0.0;
    double gp = horner3(A, B, C, D, 0.0);
    res.refine = 0;
    if (gp == 0.0) { res.hit = 1; res.s = 0.0; return; }
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (k > ne + 1) break;
        const double sk = k == ne + 1 ? S : (k == 1 ? e0 : e1);
        const double gk = horner3(A, B, C, D, sk);
        if ((gp < 0.0 && gk > 0.0) || (gp > 0.0 && gk < 0.0)) {
            // the root is left to refine_hit, which the raytrace calls after its
            // cell loop: the lanes of a wave that hit then refine together
            res.hit = 1;
            res.refine = 1;
            res.A = A; res.B = B; res.C = C; res.D = D;
            res.sa = sp; res.sb = sk; res.ga = gp;
            res.s = sp;
            return;
        }
        if (gk == 0.0) { res.hit = 1; res.s = sk; return; }
        sp = sk;
        gp = gk;
    }
}

// The hit's position in its cell when test_cell left it to a bracket.
__device__ __forceinline__ void refine_hit(CellHit &h) {
    if (h.refine) h.s = refine_root(h.A, h.B, h.C, h.D, h.sa, h.sb, h.ga);
}

// Headlight Lambertian shading of the hit: base colour (0.90, 0.75, 0.40) x
// (0.15 + 0.85 |n.d|), n the normalised trilinear gradient; RGBA8, r low byte.
__device__ inline uint32_t shade_hit(const Ray &R, const CellHit &h, const float fc[8]) {
    double u = h.loc[0] + h.s * R.d[0], v = h.loc[1] + h.s * R.d[1], w = h.loc[2] + h.s * R.d[2];
    double U0 = 1.0 - u, U1 = u, V0 = 1.0 - v, V1 = v, W0 = 1.0 - w, W1 = w;
    double c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = (double)fc[i];
    double gx = ((c[1] - c[0]) * V0 + (c[3] - c[2]) * V1) * W0 + ((c[5] - c[4]) * V0 + (c[7] - c[6]) * V1) * W1;
    double gy = ((c[2] - c[0]) * U0 + (c[3] - c[1]) * U1) * W0 + ((c[6] - c[4]) * U0 + (c[7] - c[5]) * U1) * W1;
    double gz = ((c[4] - c[0]) * U0 + (c[5] - c[1]) * U1) * V0 + ((c[6] - c[2]) * U0 + (c[7] - c[3]) * U1) * V1;
    double len = sqrt((gx * gx + gy * gy) + gz * gz);
    double nd = len > 0.0 ? fabs((gx * R.d[0] + gy * R.d[1]) + gz * R.d[2]) / len : 1.0;
    double k = 0.15 + 0.85 * nd;
    const double base[3] = {0.90, 0.75, 0.40};
    uint32_t out = 0xFF000000u;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double x = floor(255.0 * (base[ch] * k) + 0.5);
        x = x < 0.0 ? 0.0 : (x > 255.0 ? 255.0 : x);
        out |= (uint32_t)x << (8 * ch);
    }
    return out;
}

// ------------------------------------------------------ host-side hooks --
// Kernel launchers implemented in the .hip files (all on one stream).
struct Launch;

}  // namespace spr
