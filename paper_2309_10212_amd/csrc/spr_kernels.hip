// spr_kernels.hip — gfx950 kernels of libspr.
//
// Load path (Sec. 3.1): block decode + value range, fine and coarse macrocell
// grids.  Per pass (Sec. 3 pipeline (a)-(f) with the Sec. 4 speculation
// changes): pass set-up, speculative two-level traversal with visible-block
// dedupe, mark active blocks, cache lookup + per-block pair-run allocation,
// LRU eviction (only when the free list runs short), slot assignment, miss
// decode + pair scatter, block raytrace, depth composite, ray counting and
// ordered compaction with the N_spec update.
#include "spr_launch.h"

namespace spr {

// ------------------------------------------------- codec: coefficient order --
// Embedded coding visits coefficient positions sorted by the sum of their
// per-axis transform levels (L:0, H:1, h0:2, h1:2), ties by raster index.
struct OrderTable {
    uint8_t ord[64];
};

static constexpr OrderTable make_order() {
    OrderTable t{};
    int lev[4] = {0, 1, 2, 2};
    int n = 0;
    for (int s = 0; s <= 6; ++s)
        for (int i = 0; i < 64; ++i)
            if (lev[i & 3] + lev[(i >> 2) & 3] + lev[(i >> 4) & 3] == s) t.ord[n++] = (uint8_t)i;
    return t;
}

__constant__ OrderTable c_order = make_order();

// ----------------------------------------------------- codec: wave decode --
// One wave decodes one block; lane j owns the coefficient at position j of
// the embedded order.  The bit-plane control state (read position, plane,
// significance mask, cursor) is wave-uniform; the refinement bits are read in
// parallel (lane rank among the significant set = mbcnt of the mask); the
// group-test scan finds the first set bit of a 64-bit window (ctz) and the
// target coefficient as the z-th candidate (rank by mbcnt).  The inverse
// integer transform runs on 64-bit integers in LDS, z then y then x.

__device__ __forceinline__ uint32_t rec_word(const uint32_t *s_rec, int rw, int i) {
    return i < rw ? s_rec[i] : 0u;
}

__device__ __forceinline__ uint64_t window64(const uint32_t *s_rec, int rw, uint32_t p) {
    int i = (int)(p >> 5);
    uint32_t sh = p & 31u;
    uint64_t ab = (uint64_t)rec_word(s_rec, rw, i) | ((uint64_t)rec_word(s_rec, rw, i + 1) << 32);
    if (sh == 0) return ab;
    return (ab >> sh) | ((uint64_t)rec_word(s_rec, rw, i + 2) << (64 - sh));
}

__device__ __forceinline__ int64_t floor_half64(int64_t x) { return x >> 1; }

__device__ __forceinline__ void inv_line64(int64_t *p, int stride) {
    int64_t L = p[0], H = p[stride], h0 = p[2 * stride], h1 = p[3 * stride];
    int64_t l1 = L - floor_half64(H);
    int64_t l0 = l1 + H;
    int64_t a1 = l0 - floor_half64(h0);
    int64_t a0 = a1 + h0;
    int64_t a3 = l1 - floor_half64(h1);
    int64_t a2 = a3 + h1;
    p[0] = a0; p[stride] = a1; p[2 * stride] = a2; p[3 * stride] = a3;
}

// Requires a workgroup of exactly one wave (uses __syncthreads as the wave
// barrier).  Returns this lane's decoded value at raster index lane.
__device__ float wave_decode(const uint32_t *rec, int rate, int rw, uint32_t *s_rec, int64_t *s_q) {
    const uint32_t l = lane_id();
    if (rate == 32) return __uint_as_float(rec[l]);
    if ((int)l < rw) s_rec[l] = rec[l];
    __syncthreads();
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(s_rec[0]);
    float result = 0.0f;
    if (w0 & 1u) {
        const int e = (int)((w0 >> 1) & 0xFFu) - 127;
        const uint32_t B = 64u * (uint32_t)rate;
        const uint64_t below = lanemask_lt();
        uint32_t pos = 9;
        uint64_t S = 0;
        uint32_t mag = 0, neg = 0;
        for (int k = 29; k >= 0; --k) {
            // refinement bits, one per coefficient significant before this plane
            uint32_t n = (uint32_t)__popcll(S);
            uint32_t avail = B - pos < n ? B - pos : n;
            if (n) {
                uint64_t win = window64(s_rec, rw, pos);
                uint32_t r = (uint32_t)__popcll(S & below);
                if (((S >> l) & 1ull) && r < avail) mag |= (uint32_t)((win >> r) & 1ull) << k;
            }
            pos += avail;
            if (avail < n) break;
            // significance pass: group tests from the cursor
            uint32_t c = 0;
            bool stop = false;
            for (;;) {
                uint64_t I = c >= 64 ? 0ull : (~S & (~0ull << c));
                if (I == 0) break;
                if (pos >= B) { stop = true; break; }
                uint32_t g = (uint32_t)(window64(s_rec, rw, pos) & 1ull);
                pos++;
                if (!g) break;
                uint32_t ncand = (uint32_t)__popcll(I);
                uint32_t lim = B - pos < ncand ? B - pos : ncand;
                uint64_t win = window64(s_rec, rw, pos);
                if (lim < 64) win &= (1ull << lim) - 1ull;
                if (win == 0) { stop = true; break; }
                uint32_t z = (uint32_t)__ffsll((unsigned long long)win) - 1u;
                pos += z + 1;
                // target = the z-th candidate (0-based) of I
                bool inI = (I >> l) & 1ull;
                uint32_t rk = (uint32_t)__popcll(I & below);
                uint64_t tm = __ballot(inI && rk == z);
                uint32_t target = (uint32_t)__ffsll((unsigned long long)tm) - 1u;
                if (pos >= B) { stop = true; break; }
                uint32_t sgn = (uint32_t)(window64(s_rec, rw, pos) & 1ull);
                pos++;
                if (l == target) { mag |= 1u << k; neg = sgn; }
                S |= 1ull << target;
                c = target + 1;
            }
            if (stop) break;
        }
        int64_t cval = neg ? -(int64_t)mag : (int64_t)mag;
        s_q[c_order.ord[l]] = cval;
        __syncthreads();
        if (l < 16) inv_line64(s_q + (l & 3) + 4 * (l >> 2), 16);   // z lines
        __syncthreads();
        if (l < 16) inv_line64(s_q + (l & 3) + 16 * (l >> 2), 4);   // y lines
        __syncthreads();
        if (l < 16) inv_line64(s_q + 4 * (l & 3) + 16 * (l >> 2), 1);   // x lines
        __syncthreads();
        result = (float)ldexp((double)s_q[l], e - 27);
    }
    __syncthreads();
    return result;
}

// --------------------------------------------------------- decode kernels --

// Decode listed blocks of one volume into out[i*64 ..] (debug/parity path).
__global__ __launch_bounds__(64) void k_decode_ids(VolDev V, const uint32_t *ids, uint32_t n, float *out) {
    __shared__ uint32_t s_rec[64];
    __shared__ int64_t s_q[64];
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t *rec = V.stream + (size_t)ids[i] * (size_t)V.rec_words;
        float v = wave_decode(rec, V.rate, V.rec_words, s_rec, s_q);
        out[(size_t)i * 64 + lane_id()] = v;
    }
}

// Load path: decode every block once and keep only its value range over the
// samples inside the volume (Sec. 3.1).
__global__ __launch_bounds__(64) void k_block_ranges(VolDev V, float2 *blk) {
    __shared__ uint32_t s_rec[64];
    __shared__ int64_t s_q[64];
    const uint32_t l = lane_id();
    for (uint64_t b = blockIdx.x; b < V.nblocks; b += gridDim.x) {
        const uint32_t *rec = V.stream + b * (uint64_t)V.rec_words;
        float v = wave_decode(rec, V.rate, V.rec_words, s_rec, s_q);
        int bx = (int)(b % (uint64_t)V.nb[0]);
        int by = (int)((b / (uint64_t)V.nb[0]) % (uint64_t)V.nb[1]);
        int bz = (int)(b / ((uint64_t)V.nb[0] * V.nb[1]));
        int x = 4 * bx + (int)(l & 3), y = 4 * by + (int)((l >> 2) & 3), z = 4 * bz + (int)(l >> 4);
        bool in = x < V.n[0] && y < V.n[1] && z < V.n[2];
        float lo = in ? v : __builtin_inff(), hi = in ? v : -__builtin_inff();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            float ol = __shfl_xor(lo, off), oh = __shfl_xor(hi, off);
            lo = ol < lo ? ol : lo;
            hi = oh > hi ? oh : hi;
        }
        if (l == 0) blk[b] = make_float2(lo, hi);
    }
}

// Fine grid: union of the ranges of blocks b + {0,1}^3 that exist.
__global__ void k_fine_grid(VolDev V) {
    const float2 *blk = V.blk;
    uint64_t nb = V.nblocks;
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < nb; b += (uint64_t)gridDim.x * blockDim.x) {
        int bx = (int)(b % (uint64_t)V.nb[0]);
        int by = (int)((b / (uint64_t)V.nb[0]) % (uint64_t)V.nb[1]);
        int bz = (int)(b / ((uint64_t)V.nb[0] * V.nb[1]));
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    int x = bx + dx, y = by + dy, z = bz + dz;
                    if (x >= V.nb[0] || y >= V.nb[1] || z >= V.nb[2]) continue;
                    float2 r = blk[((uint64_t)z * V.nb[1] + y) * V.nb[0] + x];
                    lo = r.x < lo ? r.x : lo;
                    hi = r.y > hi ? r.y : hi;
                }
        V.fine[b] = make_float2(lo, hi);
    }
}

// Coarse grid: union of the fine ranges of blocks 4c .. 4c+3 that exist.
__global__ void k_coarse_grid(VolDev V) {
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < nc; c += (uint64_t)gridDim.x * blockDim.x) {
        int cx = (int)(c % (uint64_t)V.nc[0]);
        int cy = (int)((c / (uint64_t)V.nc[0]) % (uint64_t)V.nc[1]);
        int cz = (int)(c / ((uint64_t)V.nc[0] * V.nc[1]));
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int z = 4 * cz; z < 4 * cz + 4 && z < V.nb[2]; ++z)
            for (int y = 4 * cy; y < 4 * cy + 4 && y < V.nb[1]; ++y)
                for (int x = 4 * cx; x < 4 * cx + 4 && x < V.nb[0]; ++x) {
                    float2 r = V.fine[((uint64_t)z * V.nb[1] + y) * V.nb[0] + x];
                    lo = r.x < lo ? r.x : lo;
                    hi = r.y > hi ? r.y : hi;
                }
        V.coarse[c] = make_float2(lo, hi);
    }
}

// Fill a u32 buffer with a value (used instead of memset so that every clear
// can live inside a captured graph).
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_u32(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

// Release every cache slot owned by volume vol (volume free).
__global__ void k_release_volume_slots(PassCtl *ctl, Cache C, uint32_t vol) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < C.n_slots; s += gridDim.x * blockDim.x) {
        uint64_t o = C.owner[s];
        bool mine = o != ~0ull && (uint32_t)(o >> 32) == vol;
        if (mine) C.owner[s] = ~0ull;
        uint32_t idx = wave_append(&ctl->free_top, mine);
        if (mine) C.free_stack[idx] = s;
    }
}

// ----------------------------------------------------------- pass helpers --

__device__ __forceinline__ uint32_t find_req(const uint32_t *base, uint32_t nreq, uint32_t p) {
    uint32_t lo = 0, hi = nreq;   // largest r with base[r] <= p
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t round64(uint32_t x) { return (x + 63u) & ~63u; }

// Wave-aggregated bump allocation of variable-size runs: returns this lane's
// start in *counter for a run of `val` entries.
__device__ __forceinline__ uint32_t wave_bump(uint32_t *counter, uint32_t val) {
    uint32_t l = lane_id();
    uint32_t incl = val;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off);
        if ((int)l >= off) incl += o;
    }
    uint32_t total = __shfl(incl, 63);
    uint32_t base = 0;
    if (l == 63) base = atomicAdd(counter, total);
    base = __shfl(base, 63);
    return base + incl - val;
}

// ---------------------------------------------------------------- K0 ------
// Pass set-up: new pass stamp, counters cleared, per-request index spaces.
__global__ void k_pass_begin(PassCtl *ctl, Table T, int is_init) {
    if (threadIdx.x < 64) ctl->hist[threadIdx.x] = 0;
    if (threadIdx.x != 0) return;
    ctl->pass += 1;
    ctl->n_vis = 0; ctl->v_adm = 0; ctl->n_actblk = 0; ctl->n_miss = 0; ctl->n_hit = 0;
    ctl->cursor = 0; ctl->served = 0; ctl->deferred = 0; ctl->need = 0; ctl->evict_T = 64;
    ctl->evict_done_blocks = 0; ctl->evicted = 0; ctl->terminated = 0; ctl->pairs = 0; ctl->overflow = 0;
    uint32_t A = 0, P = 0, rays = 0;
    for (uint32_t r = 0; r < T.nreq; ++r) {
        ReqState *st = T.reqs[r].st;
        uint32_t na = st->n_act, ns = st->n_spec;
        T.act_base[r] = A;
        T.pair_base[r] = P;
        st->n_act_prev = na;
        st->last_nspec = ns;
        st->last_pairs = 0; st->last_deferred = 0; st->last_terminated = 0;
        if (na > 0 && !is_init) {
            if (st->passes == 0) st->entered = na;
            st->passes += 1;
        }
        A += round64(na);
        P += is_init ? 0u : na * ns;
        rays += na;
    }
    ctl->rays = rays;
    T.act_base[T.nreq] = A;
    T.pair_base[T.nreq] = P;
    ctl->A = A;
    ctl->P = P;
    ctl->nreq = T.nreq;
}

// ------------------------------------------------------------ initial rays --
// Sec. 3.2: one thread per pixel computes the ray and its volume entry; rays
// that miss are terminated; image and hit buffer are cleared.  The alive
// flags feed the same count/compact kernels as a pass.
__global__ void k_init_rays(PassCtl *ctl, Table T, const VolDev *vols) {
    uint32_t A = ctl->A;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        uint32_t r = find_req(T.act_base, T.nreq, p);
        const ReqDev &q = T.reqs[r];
        uint32_t i = p - T.act_base[r];
        bool alive = false;
        if (i < q.npix) {
            Ray R;
            make_ray(q, vols[q.vol].n, i, R);
            alive = R.entered != 0;
            q.ray_state[i] = alive ? RAY_NOT_STARTED : RAY_DONE;
            q.image[i] = 0u;
            spr_hit h;
            h.t = __builtin_inf();
            h.block_id = NONE;
            h.cell = NONE;
            q.hits[i] = h;
            q.act[1][i] = i;
        }
        uint64_t m = __ballot(alive);
        if (lane_id() == 0) T.wave_cnt[p >> 6] = (uint32_t)__popcll(m);
    }
}

// ---------------------------------------------------------------- K1 ------
// Speculative two-level macrocell traversal (Sec. 3.3 and 4.1).  Each active
// ray resumes after the last block it was served (or at its volume entry),
// walks the coarse grid, descends into coarse cells whose range contains the
// isovalue and walks their blocks, and records up to N_spec blocks whose fine
// range contains the isovalue at slots i*N_spec + k; unused slots get NONE.
// First visitors of a block append it to the visible list (stamp dedupe).

__device__ __forceinline__ bool range_has(float2 r, float iso) { return r.x <= iso && iso <= r.y; }

__global__ __launch_bounds__(256) void k_traverse(PassCtl *ctl, Table T, const VolDev *vols, Work W) {
    const uint32_t A = ctl->A;
    const uint32_t pass = ctl->pass;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        uint32_t r = find_req(T.act_base, T.nreq, p);
        const ReqDev &q = T.reqs[r];
        const ReqState *st = q.st;
        uint32_t i = p - T.act_base[r];
        if (i >= st->n_act_prev) continue;
        const uint32_t ns = st->last_nspec;
        const uint32_t pix = q.act[st->cur][i];
        const VolDev &V = vols[q.vol];
        Ray R;
        make_ray(q, V.n, pix, R);
        const float iso = q.iso;
        uint32_t *slots = q.pair_blk + (size_t)i * ns;
        Level LB = {4, {V.tb[0], V.tb[1], V.tb[2]}, {V.n[0], V.n[1], V.n[2]}};
        Level LC = {16, {V.tc[0], V.tc[1], V.tc[2]}, {V.n[0], V.n[1], V.n[2]}};
        const int zero3[3] = {0, 0, 0};
        const int tbhi[3] = {V.tb[0] - 1, V.tb[1] - 1, V.tb[2] - 1};
        const int tchi[3] = {V.tc[0] - 1, V.tc[1] - 1, V.tc[2] - 1};
        int cb[3], cc[3];
        double tcur;
        bool bvalid, ctest;
        bool alive = true;
        uint32_t found = 0;
        const uint32_t state = q.ray_state[pix];
        if (state == RAY_NOT_STARTED) {
            tcur = R.te;
#pragma unroll
            for (int a = 0; a < 3; ++a) cc[a] = cell_at(R, LC, a, tcur, 0, tchi[a]);
            bvalid = false;
            ctest = true;
        } else {
            uint32_t b = state;
            cb[0] = (int)(b % (uint32_t)V.nb[0]);
            cb[1] = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
            cb[2] = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
#pragma unroll
            for (int a = 0; a < 3; ++a) cc[a] = cb[a] >> 2;
            double tn = cell_exit(R, LB, cb);
            if (tn > R.tx || !advance(R, LB, cb, tn, zero3, tbhi)) alive = false;
            tcur = tn;
            bvalid = true;
            ctest = (cb[0] >> 2) != cc[0] || (cb[1] >> 2) != cc[1] || (cb[2] >> 2) != cc[2];
            if (ctest) {
#pragma unroll
                for (int a = 0; a < 3; ++a) cc[a] = cb[a] >> 2;
            }
        }
        const int max_steps = V.tb[0] + V.tb[1] + V.tb[2] + V.tc[0] + V.tc[1] + V.tc[2] + 8;
        int steps = 0;
        while (alive && found < ns) {
            if (++steps > max_steps) { alive = false; break; }   // every step advances an index
            if (ctest) {
                const uint64_t cid = ((uint64_t)cc[2] * V.nc[1] + cc[1]) * V.nc[0] + cc[0];
                if (range_has(V.coarse[cid], iso)) {
                    if (!bvalid) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            int lo = 4 * cc[a], hi = 4 * cc[a] + 3;
                            if (hi > tbhi[a]) hi = tbhi[a];
                            cb[a] = cell_at(R, LB, a, tcur, lo, hi);
                        }
                        bvalid = true;
                    }
                    ctest = false;
                } else {
                    double tn = cell_exit(R, LC, cc);
                    if (tn > R.tx || !advance(R, LC, cc, tn, zero3, tchi)) { alive = false; break; }
                    tcur = tn;
                    bvalid = false;
                    continue;
                }
            }
            const uint32_t bid = (uint32_t)(((uint64_t)cb[2] * V.nb[1] + cb[1]) * V.nb[0] + cb[0]);
            const bool emit = range_has(V.fine[bid], iso);
            if (emit) {
                slots[found] = bid;
                found++;
                bool first = false;
                if (__hip_atomic_load(&V.vis_stamp[bid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pass)
                    first = atomicExch(&V.vis_stamp[bid], pass) != pass;
                uint32_t idx = wave_append(&ctl->n_vis, first);
                if (first) {
                    W.vis_list[idx] = ((uint64_t)q.vol << 32) | bid;
                    V.vis_idx[bid] = idx;
                    W.vis_cnt[idx] = 0;
                }
                if (found == ns) break;
            }
            double tn = cell_exit(R, LB, cb);
            if (tn > R.tx || !advance(R, LB, cb, tn, zero3, tbhi)) { alive = false; break; }
            tcur = tn;
            if ((cb[0] >> 2) != cc[0] || (cb[1] >> 2) != cc[1] || (cb[2] >> 2) != cc[2]) {
#pragma unroll
                for (int a = 0; a < 3; ++a) cc[a] = cb[a] >> 2;
                ctest = true;
            }
        }
        for (uint32_t k = found; k < ns; ++k) slots[k] = NONE;
    }
}

// ---------------------------------------------------------------- K2 ------
// Role A (per pair): rank of the pair within its visible block (atomic count,
// the N_BRays of Sec. 3.6) and served/deferred accounting.  Role B (per
// admitted visible block): mark the block and its +x/+y/+z face, edge and
// corner neighbours active (Sec. 3.4), first visitors append to the active list.

__device__ __forceinline__ uint32_t admitted_blocks(const PassCtl *ctl) {
    uint32_t nv = ctl->n_vis;
    uint32_t cap = ctl->n_slots / 8u;
    return nv < cap ? nv : cap;
}

__global__ __launch_bounds__(256) void k_mark(PassCtl *ctl, Table T, const VolDev *vols, Work W) {
    const uint32_t P = ctl->P;
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t pass = ctl->pass;
    const uint32_t total = P + vadm;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t n_served = 0, n_def = 0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        if (x < P) {
            uint32_t r = find_req(T.pair_base, T.nreq, x);
            const ReqDev &q = T.reqs[r];
            uint32_t b = q.pair_blk[x - T.pair_base[r]];
            if (b != NONE) {
                uint32_t vi = vols[q.vol].vis_idx[b];
                W.pair_rank[x] = atomicAdd(&W.vis_cnt[vi], 1u);
                if (vi < vadm) n_served++;
                else n_def++;
            }
        } else {
            uint32_t j = x - P;
            uint64_t e = W.vis_list[j];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            uint32_t b = (uint32_t)e;
            int bx = (int)(b % (uint32_t)V.nb[0]);
            int by = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
            int bz = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
            for (int o = 0; o < 8; ++o) {
                int x2 = bx + (o & 1), y2 = by + ((o >> 1) & 1), z2 = bz + (o >> 2);
                bool ok = x2 < V.nb[0] && y2 < V.nb[1] && z2 < V.nb[2];
                bool first = false;
                uint32_t nbid = 0;
                if (ok) {
                    nbid = (uint32_t)(((uint64_t)z2 * V.nb[1] + y2) * V.nb[0] + x2);
                    if (__hip_atomic_load(&V.act_stamp[nbid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pass)
                        first = atomicExch(&V.act_stamp[nbid], pass) != pass;
                }
                uint32_t idx = wave_append(&ctl->n_actblk, first);
                if (first) W.act_list[idx] = (e & 0xFFFFFFFF00000000ull) | nbid;
            }
        }
    }
    // block-level reduction of the counters
    __shared__ uint32_t s_cnt[2];
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    if (n_served) atomicAdd(&s_cnt[0], n_served);
    if (n_def) atomicAdd(&s_cnt[1], n_def);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_cnt[0]) atomicAdd(&ctl->served, s_cnt[0]);
        if (s_cnt[1]) atomicAdd(&ctl->deferred, s_cnt[1]);
    }
}

// ---------------------------------------------------------------- K3 ------
// Role A (per active block): cache lookup; a hit refreshes the slot's LRU
// stamp, a miss is appended to the miss list (Sec. 3.5).  Role B (per
// admitted visible block): allocate the block's run of sorted pairs
// (O_BRays of Sec. 3.6) by wave-aggregated bump allocation.
__global__ __launch_bounds__(256) void k_lookup(PassCtl *ctl, const VolDev *vols, Work W, Cache C) {
    const uint32_t K = ctl->n_actblk;
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t pass = ctl->pass;
    const uint32_t stride = gridDim.x * blockDim.x;
    // role B first so that whole waves stay together for the wave scan
    const uint32_t nB = round64(vadm);
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nB + K; x += stride) {
        if (x < nB) {
            uint32_t cnt = x < vadm ? W.vis_cnt[x] : 0u;
            uint32_t off = wave_bump(&ctl->cursor, cnt);
            if (x < vadm) W.vis_off[x] = off;
        } else {
            uint32_t j = x - nB;
            uint64_t e = W.act_list[j];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            uint32_t b = (uint32_t)e;
            uint32_t s = V.map[b];
            bool miss = s == NONE;
            if (!miss) C.stamp[s] = pass;
            uint32_t idx = wave_append(&ctl->n_miss, miss);
            if (miss) W.miss_list[idx] = e;
        }
    }
}

// ---------------------------------------------------------------- K4 ------
// Slot supply.  If the free stack holds fewer slots than the misses, an LRU
// sweep reclaims the oldest occupied slots not used this pass: a histogram of
// ages (pass - stamp, clamped to 63) picks the largest age threshold whose
// tail covers max(shortfall, n_slots/16) slots, and every slot at or above it
// is evicted in one sweep.
__global__ void k_alloc_plan(PassCtl *ctl) {
    if (threadIdx.x != 0) return;
    uint32_t m = ctl->n_miss, f = ctl->free_top;
    if (m > f) {
        uint32_t short_by = m - f;
        uint32_t batch = ctl->n_slots / 16u;
        ctl->need = short_by > batch ? short_by : batch;
    } else {
        ctl->need = 0;
    }
}

__global__ __launch_bounds__(256) void k_evict_hist(PassCtl *ctl, Cache C) {
    if (ctl->need == 0) return;
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t pass = ctl->pass;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < C.n_slots; s += gridDim.x * blockDim.x) {
        if (C.owner[s] == ~0ull) continue;
        uint32_t st = C.stamp[s];
        if (st == pass) continue;
        uint32_t age = pass - st;
        atomicAdd(&h[age > 63u ? 63u : age], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&ctl->hist[threadIdx.x], h[threadIdx.x]);
    __threadfence();
    __shared__ uint32_t last;
    if (threadIdx.x == 0) last = atomicAdd(&ctl->evict_done_blocks, 1u) == gridDim.x - 1;
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        uint32_t need = ctl->need, acc = 0, T = 1;
        for (int a = 63; a >= 1; --a) {
            acc += __hip_atomic_load(&ctl->hist[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (acc >= need) { T = (uint32_t)a; break; }
        }
        ctl->evict_T = T;
    }
}

__global__ __launch_bounds__(256) void k_evict(PassCtl *ctl, const VolDev *vols, Cache C) {
    if (ctl->need == 0) return;
    const uint32_t pass = ctl->pass, T = ctl->evict_T;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < round64(C.n_slots); s += gridDim.x * blockDim.x) {
        bool ev = false;
        if (s < C.n_slots) {
            uint64_t o = C.owner[s];
            if (o != ~0ull) {
                uint32_t st = C.stamp[s];
                uint32_t age = pass - st;
                if (st != pass && (age > 63u ? 63u : age) >= T) {
                    ev = true;
                    vols[(uint32_t)(o >> 32)].map[(uint32_t)o] = NONE;
                    C.owner[s] = ~0ull;
                }
            }
        }
        uint32_t idx = wave_append(&ctl->free_top, ev);
        if (ev) C.free_stack[idx] = s;
        uint64_t em = __ballot(ev);
        if (lane_id() == 0 && em) atomicAdd(&ctl->evicted, (uint32_t)__popcll(em));
    }
}

// ---------------------------------------------------------------- K5 ------
// Assign the top n_miss free slots to the misses.
__global__ __launch_bounds__(256) void k_assign(PassCtl *ctl, const VolDev *vols, Work W, Cache C) {
    const uint32_t f = ctl->free_top;
    uint32_t m = ctl->n_miss;
    if (m > f) m = f;   // cannot happen: admission keeps the active blocks within n_slots
    const uint32_t base = f - m;
    const uint32_t pass = ctl->pass;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->assigned = m;
        if (m < ctl->n_miss) ctl->overflow = 1;
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        uint64_t e = W.miss_list[i];
        uint32_t s = C.free_stack[base + i];
        vols[(uint32_t)(e >> 32)].map[(uint32_t)e] = s;
        C.owner[s] = e;
        C.stamp[s] = pass;
        W.miss_slot[i] = s;
    }
}

// ---------------------------------------------------------------- K6 ------
// Role A (waves 0 .. dec_groups-1): decode misses into their slots (Sec. 3.5).
// Role B (other workgroups): scatter served pairs into their block's run
// (the sort by block id of Sec. 3.6 / 4.2; the pair slot carries O_Spec).
__global__ __launch_bounds__(64) void k_decode_scatter(PassCtl *ctl, Table T, const VolDev *vols, Work W, Cache C,
                                                       uint32_t dec_groups) {
    __shared__ uint32_t s_rec[64];
    __shared__ int64_t s_q[64];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the slots handed out by k_assign leave the free stack
        ctl->free_top -= ctl->assigned;
    }
    if (blockIdx.x < dec_groups) {
        const uint32_t m = ctl->assigned;
        for (uint32_t i = blockIdx.x; i < m; i += dec_groups) {
            uint64_t e = W.miss_list[i];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            const uint32_t *rec = V.stream + (uint64_t)(uint32_t)e * (uint64_t)V.rec_words;
            float v = wave_decode(rec, V.rate, V.rec_words, s_rec, s_q);
            C.slots[(size_t)W.miss_slot[i] * 64 + lane_id()] = v;
        }
        return;
    }
    const uint32_t P = ctl->P;
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t nthreads = (gridDim.x - dec_groups) * blockDim.x;
    for (uint32_t x = (blockIdx.x - dec_groups) * blockDim.x + threadIdx.x; x < P; x += nthreads) {
        uint32_t r = find_req(T.pair_base, T.nreq, x);
        const ReqDev &q = T.reqs[r];
        uint32_t qq = x - T.pair_base[r];
        uint32_t b = q.pair_blk[qq];
        if (b == NONE) continue;
        uint32_t vi = vols[q.vol].vis_idx[b];
        if (vi >= vadm) continue;
        uint32_t dst = W.vis_off[vi] + W.pair_rank[x];
        const ReqState *st = q.st;
        uint32_t i = qq / st->last_nspec;
        uint32_t pix = q.act[st->cur][i];
        W.s_ray[dst] = (r << 24) | pix;
        W.s_q[dst] = qq;
        W.s_vi[dst] = vi;
    }
}

// ---------------------------------------------------------------- K9 ------
// Block raytrace (Sec. 3.7, 4.3): each served pair walks its ray through the
// dual cells of its block (Amanatides-Woo restricted to the block), tests
// each cell (corner pretest, cubic, Marmitt isolation) and writes the first
// hit (t, cell, colour) or t = +inf to the RGBZ record at its pair slot.
__device__ __forceinline__ float slot_value(const float *slots, const uint32_t ns[8], int lx, int ly, int lz) {
    int nb = (lx >> 2) | ((ly >> 2) << 1) | ((lz >> 2) << 2);
    uint32_t s = ns[nb];
    if (s == NONE) return 0.0f;   // unreachable: every neighbour of a served block holds a slot
    return slots[(size_t)s * 64 + ((lx & 3) + 4 * (ly & 3) + 16 * (lz & 3))];
}

__global__ __launch_bounds__(256) void k_raytrace(PassCtl *ctl, Table T, const VolDev *vols, Work W, Cache C) {
    const uint32_t n = ctl->served;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        uint32_t ray = W.s_ray[j];
        uint32_t r = ray >> 24, pix = ray & 0xFFFFFFu;
        uint32_t qq = W.s_q[j];
        uint64_t e = W.vis_list[W.s_vi[j]];
        const ReqDev &q = T.reqs[r];
        const VolDev &V = vols[(uint32_t)(e >> 32)];
        uint32_t b = (uint32_t)e;
        int bb[3];
        bb[0] = (int)(b % (uint32_t)V.nb[0]);
        bb[1] = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
        bb[2] = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
        uint32_t nsl[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            int x2 = bb[0] + (o & 1), y2 = bb[1] + ((o >> 1) & 1), z2 = bb[2] + (o >> 2);
            bool ok = x2 < V.nb[0] && y2 < V.nb[1] && z2 < V.nb[2];
            nsl[o] = ok ? V.map[((uint64_t)z2 * V.nb[1] + y2) * V.nb[0] + x2] : 0u;
        }
        Ray R;
        make_ray(q, V.n, pix, R);
        Level LB = {4, {V.tb[0], V.tb[1], V.tb[2]}, {V.n[0], V.n[1], V.n[2]}};
        Level L1 = {1, {V.n[0] - 1, V.n[1] - 1, V.n[2] - 1}, {V.n[0], V.n[1], V.n[2]}};
        int lo[3], hi[3], c[3];
        double tb0 = cell_entry(R, LB, bb);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = 4 * bb[a];
            hi[a] = 4 * bb[a] + 3;
            if (hi[a] > V.n[a] - 2) hi[a] = V.n[a] - 2;
            c[a] = cell_at(R, L1, a, tb0, lo[a], hi[a]);
        }
        Rgbz out;
        out.t = __builtin_inf();
        out.cell = NONE;
        out.rgba = 0u;
        for (int guard = 0; guard < 16; ++guard) {   // at most 10 cells of a 4^3 block lie on a ray
            double t0 = cell_entry(R, L1, c);
            double t1 = R.tx;
            {
                double x = cell_exit(R, L1, c);
                if (x < t1) t1 = x;
            }
            float fc[8];
            int lx = c[0] - lo[0], ly = c[1] - lo[1], lz = c[2] - lo[2];
#pragma unroll
            for (int k = 0; k < 8; ++k) fc[k] = slot_value(C.slots, nsl, lx + (k & 1), ly + ((k >> 1) & 1), lz + (k >> 2));
            CellHit h;
            test_cell(R, c, t0, t1, fc, q.iso, h);
            if (h.hit) {
                out.t = t0 + h.s;
                out.cell = (uint32_t)(lx + 4 * ly + 16 * lz);
                out.rgba = shade_hit(R, h, fc);
                break;
            }
            double tn = cell_exit(R, L1, c);
            if (tn > R.tx || !advance(R, L1, c, tn, lo, hi)) break;
        }
        q.rgbz[qq] = out;
    }
}

// --------------------------------------------------------------- K10 ------
// Depth composite (Sec. 4.4) and termination: each active ray scans its
// N_spec slots in order; slots are in traversal order, so the first hit is
// the closest (ties go to the earlier block).  An empty slot means the walk
// left the volume: the ray terminates.  A slot on a block that was not
// served this pass stops the scan: the ray keeps its progress up to the last
// served block and retries the rest next pass.  Survivor counts per wave
// feed the compaction.
__global__ __launch_bounds__(256) void k_composite(PassCtl *ctl, Table T, const VolDev *vols) {
    const uint32_t A = ctl->A;
    const uint32_t vadm = admitted_blocks(ctl);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        uint32_t r = find_req(T.act_base, T.nreq, p);
        const ReqDev &q = T.reqs[r];
        ReqState *st = q.st;
        uint32_t i = p - T.act_base[r];
        bool alive = false;
        uint32_t my_pairs = 0, my_def = 0, my_term = 0;
        if (i < st->n_act_prev) {
            const uint32_t ns = st->last_nspec;
            const uint32_t pix = q.act[st->cur][i];
            const VolDev &V = vols[q.vol];
            const uint32_t *slots = q.pair_blk + (size_t)i * ns;
            const Rgbz *res = q.rgbz + (size_t)i * ns;
            uint32_t last = NONE;
            bool term = false, stopped = false;
            for (uint32_t k = 0; k < ns; ++k) {
                uint32_t b = slots[k];
                if (b == NONE) {
                    if (!stopped && !term) term = true;
                    break;
                }
                my_pairs++;
                if (stopped || term) {
                    if (V.vis_idx[b] >= vadm) my_def++;
                    continue;
                }
                if (V.vis_idx[b] >= vadm) {
                    stopped = true;
                    my_def++;
                    continue;
                }
                Rgbz rec = res[k];
                if (rec.t < __builtin_inf()) {
                    q.image[pix] = rec.rgba;
                    spr_hit h;
                    h.t = rec.t;
                    h.block_id = b;
                    h.cell = rec.cell;
                    q.hits[pix] = h;
                    term = true;
                    continue;
                }
                last = b;
            }
            if (term) q.ray_state[pix] = RAY_DONE;
            else if (last != NONE) q.ray_state[pix] = last;
            alive = !term;
            my_term = term ? 1u : 0u;
        }
        uint64_t m = __ballot(alive);
        if (lane_id() == 0) T.wave_cnt[p >> 6] = (uint32_t)__popcll(m);
        // per-request counters (all lanes of a wave belong to one request)
        uint32_t sp = my_pairs, sd = my_def, stt = my_term;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            sp += __shfl_xor(sp, off);
            sd += __shfl_xor(sd, off);
            stt += __shfl_xor(stt, off);
        }
        if (lane_id() == 0) {
            if (sp) {
                atomicAdd(&st->last_pairs, sp);
                atomicAdd(&st->tot_pairs, (unsigned long long)sp);
                atomicAdd(&ctl->pairs, sp);
            }
            if (sd) atomicAdd(&st->last_deferred, sd);
            if (stt) { atomicAdd(&st->last_terminated, stt); atomicAdd(&ctl->terminated, stt); }
        }
    }
}

// --------------------------------------------------------------- K11 ------
// Count the surviving rays (Sec. 3 step (f)): exclusive scan of the per-wave
// survivor counts, per-request N_act, N_spec = clamp(floor(w*h / N_act), 1,
// cap) (Sec. 4), and flip to the other active-ray list.  One workgroup.
__global__ __launch_bounds__(1024) void k_pass_end(PassCtl *ctl, Table T, int is_init) {
    __shared__ uint32_t s_part[1024];
    __shared__ uint32_t s_carry;
    const uint32_t nw = ctl->A >> 6;
    const uint32_t t = threadIdx.x;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nw; base += 1024) {
        uint32_t v = base + t < nw ? T.wave_cnt[base + t] : 0u;
        s_part[t] = v;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            uint32_t o = t >= off ? s_part[t - off] : 0u;
            __syncthreads();
            s_part[t] += o;
            __syncthreads();
        }
        uint32_t incl = s_part[t];
        if (base + t < nw) T.wave_off[base + t] = s_carry + incl - v;
        __syncthreads();
        if (t == 1023) s_carry += incl;
        __syncthreads();
    }
    if (t == 0) {
        T.wave_off[nw] = s_carry;
        if (!is_init && ctl->A > 0) {
            ctl->acc_passes += 1;
            ctl->acc_decoded += ctl->assigned;
            ctl->acc_visible += ctl->n_vis;
            ctl->acc_active += ctl->n_actblk;
            ctl->acc_pairs += ctl->pairs;
            ctl->acc_evicted += ctl->evicted;
            ctl->acc_overflow += ctl->overflow;
            ctl->acc_rays += ctl->rays;
            ctl->acc_slots += ctl->P;
            ctl->acc_served += ctl->served;
        }
    }
    __syncthreads();
    for (uint32_t r = t; r < T.nreq; r += blockDim.x) {
        ReqDev &q = T.reqs[r];
        ReqState *st = q.st;
        uint32_t w0 = T.act_base[r] >> 6, w1 = T.act_base[r + 1] >> 6;
        uint32_t na = (w1 > w0 ? (w1 < nw ? T.wave_off[w1] : s_carry) - T.wave_off[w0] : 0u);
        if (st->n_act_prev > 0) st->cur ^= 1u;
        st->n_act = na;
        uint32_t ns = 0;
        if (na > 0) {
            ns = q.npix / na;
            if (ns < 1) ns = 1;
            if (ns > q.spec_cap) ns = q.spec_cap;
        }
        st->n_spec = ns;
    }
}

// --------------------------------------------------------------- K12 ------
// Ordered compaction of the surviving rays into the new active list.
__global__ __launch_bounds__(256) void k_compact(PassCtl *ctl, Table T) {
    const uint32_t A = ctl->A;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        uint32_t r = find_req(T.act_base, T.nreq, p);
        const ReqDev &q = T.reqs[r];
        const ReqState *st = q.st;
        uint32_t i = p - T.act_base[r];
        bool alive = false;
        uint32_t pix = 0;
        if (i < st->n_act_prev) {
            pix = q.act[st->cur ^ 1u][i];
            alive = q.ray_state[pix] != RAY_DONE;
        }
        uint64_t m = __ballot(alive);
        if (alive) {
            uint32_t dst = T.wave_off[p >> 6] - T.wave_off[T.act_base[r] >> 6] + (uint32_t)__popcll(m & lanemask_lt());
            q.act[st->cur][dst] = pix;
        }
    }
}

// Arithmetic probe: fp64 sqrt and division as compiled for the hit test.
__global__ void k_fp64_ops(const double *x, const double *y, uint64_t n, double *sq, double *dv) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        sq[i] = sqrt(x[i]);
        dv[i] = x[i] / y[i];
    }
}

// ------------------------------------------------------------- launchers --

static inline uint32_t grid_for(uint64_t n, uint32_t bs, uint32_t cap) {
    uint64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_decode_ids(hipStream_t s, const VolDev &V, const uint32_t *ids, uint32_t n, float *out) {
    hipLaunchKernelGGL(k_decode_ids, dim3(grid_for(n, 1, 65536)), dim3(64), 0, s, V, ids, n, out);
    return hipGetLastError();
}

hipError_t launch_fp64_ops(hipStream_t s, const double *x, const double *y, uint64_t n, double *sq, double *dv) {
    hipLaunchKernelGGL(k_fp64_ops, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, y, n, sq, dv);
    return hipGetLastError();
}

hipError_t launch_load_grids(hipStream_t s, const VolDev &V) {
    hipLaunchKernelGGL(k_block_ranges, dim3(grid_for(V.nblocks, 1, 1u << 20)), dim3(64), 0, s, V, V.blk);
    hipLaunchKernelGGL(k_fine_grid, dim3(grid_for(V.nblocks, 256, 1u << 16)), dim3(256), 0, s, V);
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    hipLaunchKernelGGL(k_coarse_grid, dim3(grid_for(nc, 256, 1u << 16)), dim3(256), 0, s, V);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t v) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t n, uint64_t v) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_iota_u32(hipStream_t s, uint32_t *p, uint64_t n) {
    hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_release_volume(hipStream_t s, PassCtl *ctl, const Cache &C, uint32_t vol) {
    hipLaunchKernelGGL(k_release_volume_slots, dim3(grid_for(C.n_slots, 256, 8192)), dim3(256), 0, s, ctl, C, vol);
    return hipGetLastError();
}

hipError_t launch_init_rays(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols) {
    hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, s, ctl, T, 1);
    hipLaunchKernelGGL(k_init_rays, dim3(grid_for(T.max_A, 256, 16384)), dim3(256), 0, s, ctl, T, vols);
    hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(1024), 0, s, ctl, T, 1);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(T.max_A, 256, 16384)), dim3(256), 0, s, ctl, T);
    return hipGetLastError();
}

const char *const PASS_KERNEL_NAMES[PASS_KERNELS] = {
    "k_pass_begin", "k_traverse", "k_mark", "k_lookup", "k_alloc_plan", "k_evict_hist", "k_evict",
    "k_assign", "k_decode_scatter", "k_raytrace", "k_composite", "k_pass_end", "k_compact"};

hipError_t launch_pass(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols, const Work &W,
                       const Cache &C, const PassGrids &g, hipEvent_t *ev) {
    int k = 0;
    auto mark = [&]() {
        if (ev) (void)hipEventRecord(ev[k], s);
        ++k;
    };
    mark(); hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, s, ctl, T, 0);
    mark(); hipLaunchKernelGGL(k_traverse, dim3(g.rays), dim3(256), 0, s, ctl, T, vols, W);
    mark(); hipLaunchKernelGGL(k_mark, dim3(g.pairs), dim3(256), 0, s, ctl, T, vols, W);
    mark(); hipLaunchKernelGGL(k_lookup, dim3(g.blocks), dim3(256), 0, s, ctl, vols, W, C);
    mark(); hipLaunchKernelGGL(k_alloc_plan, dim3(1), dim3(64), 0, s, ctl);
    mark(); hipLaunchKernelGGL(k_evict_hist, dim3(g.slots), dim3(256), 0, s, ctl, C);
    mark(); hipLaunchKernelGGL(k_evict, dim3(g.slots), dim3(256), 0, s, ctl, vols, C);
    mark(); hipLaunchKernelGGL(k_assign, dim3(g.blocks), dim3(256), 0, s, ctl, vols, W, C);
    mark(); hipLaunchKernelGGL(k_decode_scatter, dim3(g.decode + g.scatter), dim3(64), 0, s, ctl, T, vols, W, C, g.decode);
    mark(); hipLaunchKernelGGL(k_raytrace, dim3(g.pairs), dim3(256), 0, s, ctl, T, vols, W, C);
    mark(); hipLaunchKernelGGL(k_composite, dim3(g.rays), dim3(256), 0, s, ctl, T, vols);
    mark(); hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(1024), 0, s, ctl, T, 0);
    mark(); hipLaunchKernelGGL(k_compact, dim3(g.rays), dim3(256), 0, s, ctl, T);
    if (ev) (void)hipEventRecord(ev[k], s);
    return hipGetLastError();
}

}  // namespace spr
