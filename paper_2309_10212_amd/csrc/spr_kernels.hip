// spr_kernels.hip — gfx950 kernels of libspr.
//
// Load path (Sec. 3.1): block decode + value range, fine and coarse macrocell
// grids.  Per pass (Sec. 3 pipeline (a)-(f) with the Sec. 4 speculation
// changes): pass set-up, speculative two-level traversal, visible-block
// dedupe with pair ranks, active-block marking with the cache lookup and the
// per-block pair-run allocation, LRU eviction (only when the free list runs
// short), slot assignment + pair scatter, miss decode, block raytrace, depth
// composite, ray counting and ordered compaction with the N_spec update.
#include "spr_launch.h"
#include "spr_codec.h"

namespace spr {

typedef float f4v __attribute__((ext_vector_type(4)));

// Decode one block to 64 floats, stored with 16-byte stores to dst (raster order).
template <int RWMAX>
__device__ __forceinline__ void decode_to(const uint32_t *__restrict__ rec, int rate, DecodeLds<RWMAX> &L, uint32_t lane,
                                          float *__restrict__ dst) {
    // global-address 16-byte stores (a flat store would also wait on the LDS counter)
    const gptr<f4v> d4 = as_global(reinterpret_cast<f4v *>(dst));
    if (rate == 32) {
        const gptr<const f4v> s4 = as_global(reinterpret_cast<const f4v *>(rec));
#pragma unroll
        for (int i = 0; i < 16; ++i) d4[i] = s4[i];
        return;
    }
    int32_t q[64];
    int e = 0;
    if (!thread_decode<RWMAX>(rec, rate, L, lane, q, e)) {
#pragma unroll
        for (int i = 0; i < 16; ++i) d4[i] = f4v{0.f, 0.f, 0.f, 0.f};
        return;
    }
    if (e >= -99) {
        // every nonzero value is a normal float: (float)q then an exact
        // power-of-two scale equals the single rounding of q * 2^(e-27)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            d4[i] = f4v{ldexpf((float)q[4 * i], e - 27), ldexpf((float)q[4 * i + 1], e - 27),
                        ldexpf((float)q[4 * i + 2], e - 27), ldexpf((float)q[4 * i + 3], e - 27)};
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            d4[i] = f4v{(float)ldexp((double)q[4 * i], e - 27), (float)ldexp((double)q[4 * i + 1], e - 27),
                        (float)ldexp((double)q[4 * i + 2], e - 27), (float)ldexp((double)q[4 * i + 3], e - 27)};
    }
}

// --------------------------------------------------------- decode kernels --

// Decode listed blocks of one volume into out[i*64 ..] (debug/parity path).
__global__ __launch_bounds__(64) void k_decode_ids(VolDev V, const uint32_t *ids, uint32_t n, float *out) {
    __shared__ DecodeLds<32> L;
    const uint32_t lane = threadIdx.x;
    fill_dep4(L, lane);
    __syncthreads();
    for (uint32_t i = blockIdx.x * 64 + lane; i < n; i += gridDim.x * 64) {
        const uint32_t *rec = V.stream + (size_t)ids[i] * (size_t)V.rec_words;
        decode_to<32>(rec, V.rate, L, lane, out + (size_t)i * 64);
    }
}

// Coordinates of linear index v in a grid n0 wide and n1 deep, in 32-bit
// arithmetic (block and coarse-cell counts are below 2^32; a 64-bit division
// costs about a hundred instructions).
__device__ __forceinline__ void unravel3(uint32_t v, uint32_t n0, uint32_t n1, int &x, int &y, int &z) {
    const uint32_t r = v / n0;
    x = (int)(v - r * n0);
    y = (int)(r % n1);
    z = (int)(r / n1);
}

// Load path: decode every block once and keep only its value range over the
// samples inside the volume (Sec. 3.1).
template <int RWMAX>
__global__ __launch_bounds__(64) void k_block_ranges(VolDev V, float2 *blk) {
    __shared__ DecodeLds<RWMAX> L;
    const uint32_t lane = threadIdx.x;
    fill_dep4(L, lane);
    __syncthreads();
    for (uint64_t b = blockIdx.x * 64ull + lane; b < V.nblocks; b += (uint64_t)gridDim.x * 64) {
        const uint32_t *rec = V.stream + b * (uint64_t)V.rec_words;
        int bx, by, bz;
        unravel3((uint32_t)b, (uint32_t)V.nb[0], (uint32_t)V.nb[1], bx, by, bz);
        int ex = V.n[0] - 4 * bx, ey = V.n[1] - 4 * by, ez = V.n[2] - 4 * bz;   // samples inside, per axis
        float lo = __builtin_inff(), hi = -__builtin_inff();
        if (V.rate == 32) {
            const float4 *f4 = reinterpret_cast<const float4 *>(rec);
            for (int i4 = 0; i4 < 16; ++i4) {
                float4 v4 = f4[i4];
                float vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    int i = 4 * i4 + c;
                    bool in = c < ex && ((i >> 2) & 3) < ey && (i >> 4) < ez;
                    if (in) { lo = vv[c] < lo ? vv[c] : lo; hi = vv[c] > hi ? vv[c] : hi; }
                }
            }
        } else {
            int32_t q[64];
            int e = 0;
            if (!thread_decode<RWMAX>(rec, V.rate, L, lane, q, e)) {
                lo = 0.0f;
                hi = 0.0f;
            } else {
                // conversion to float is monotone: reduce the integers, convert two
                int32_t qlo = 0x7FFFFFFF, qhi = (int32_t)0x80000000;
                if (ex >= 4 && ey >= 4 && ez >= 4) {   // interior block: every sample counts
#pragma unroll
                    for (int i = 0; i < 64; ++i) { qlo = q[i] < qlo ? q[i] : qlo; qhi = q[i] > qhi ? q[i] : qhi; }
                } else {
#pragma unroll
                    for (int i = 0; i < 64; ++i) {
                        bool in = (i & 3) < ex && ((i >> 2) & 3) < ey && (i >> 4) < ez;
                        if (in) { qlo = q[i] < qlo ? q[i] : qlo; qhi = q[i] > qhi ? q[i] : qhi; }
                    }
                }
                lo = (float)ldexp((double)qlo, e - 27);
                hi = (float)ldexp((double)qhi, e - 27);
            }
        }
        blk[b] = make_float2(lo, hi);
    }
}

// Fine grid: union of the ranges of blocks b + {0,1}^3 that exist.  The box
// union is separable (min and max are exact in any order), so it runs as
// three passes over the block ranges in place, one per axis: a thread walks
// one line of blocks along the axis in increasing order and replaces entry i
// by the union of entries i and i+1, having read i+1 before it is rewritten.
// The last entry of a line has no +1 neighbour and keeps its value.  No
// second per-block array is needed.
__global__ void k_fine_axis(VolDev V, int axis) {
    float2 *f = V.fine;
    const uint32_t nb0 = (uint32_t)V.nb[0], nb1 = (uint32_t)V.nb[1], nb2 = (uint32_t)V.nb[2];
    const uint32_t len = axis == 0 ? nb0 : (axis == 1 ? nb1 : nb2);
    const uint64_t stride = axis == 0 ? 1ull : (axis == 1 ? (uint64_t)nb0 : (uint64_t)nb0 * nb1);
    const uint64_t nlines = V.nblocks / len;
    for (uint64_t ln = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; ln < nlines;
         ln += (uint64_t)gridDim.x * blockDim.x) {
        // line ln -> its first block: x lines are indexed by (y, z), y lines
        // by (x, z) and z lines by (x, y), x fastest so neighbouring threads
        // of y and z passes touch neighbouring blocks
        uint64_t b0;
        if (axis == 0) b0 = ln * nb0;
        else if (axis == 1) { const uint64_t z = ln / nb0, x = ln - z * nb0; b0 = z * nb0 * nb1 + x; }
        else b0 = ln;
        float2 cur = f[b0];
        for (uint32_t i = 0; i + 1 < len; ++i) {
            const float2 nxt = f[b0 + (uint64_t)(i + 1) * stride];
            f[b0 + (uint64_t)i * stride] = make_float2(nxt.x < cur.x ? nxt.x : cur.x, nxt.y > cur.y ? nxt.y : cur.y);
            cur = nxt;
        }
    }
}

// Coarse grid: union of the fine ranges of blocks 4c .. 4c+3 that exist.
__global__ void k_coarse_grid(VolDev V) {
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < nc; c += (uint64_t)gridDim.x * blockDim.x) {
        int cx, cy, cz;
        unravel3((uint32_t)c, (uint32_t)V.nc[0], (uint32_t)V.nc[1], cx, cy, cz);
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
// Candidates are staged in LDS and written out after the walk (or when
// TR_BUF have accumulated): on this architecture one counter tracks vector
// loads and stores alike, so a store inside the walk would make the next
// mask load wait for the store's completion as well.
constexpr uint32_t TR_BUF = 16;
// A request with few active rays walks each ray on several lanes (segments
// of its remaining parameter range), up to this many traversal lanes.
constexpr uint32_t SEG_TARGET = 262144;

// Inclusive wave scan of v; *total receives the sum over the wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t *total) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off);
        if ((int)l >= off) v += o;
    }
    *total = __shfl(v, 63);
    return v;
}

// One wave; lane i handles requests i, i + 64, ... so the per-request loads
// are issued together and the index spaces come from wave scans.
__global__ __launch_bounds__(64) void k_pass_begin(PassCtl *ctl, Table T, int is_init) {
    const uint32_t l = lane_id();
    ctl->hist[l] = 0;
    const uint32_t nreq = T.hdr[0];
    ReqState *st0 = l < nreq ? T.reqs[l].st : nullptr;
    const uint32_t na0 = st0 ? st0->n_act : 0u, ns0 = st0 ? st0->n_spec : 0u, ps0 = st0 ? st0->passes : 0u;
    // traversal lanes per ray: a power of two up to 16 while the pass stays
    // within SEG_TARGET lanes over all requests; only for requests whose
    // slots fit one lane's staging buffer (the lanes' lists are merged after
    // the walk)
    uint32_t my = na0;
    for (uint32_t r = l + 64u; r < nreq; r += 64u) my += T.reqs[r].st->n_act;
    uint32_t all_na;
    (void)wave_incl_scan(my, &all_na);
    uint32_t segs_all = 1, segs_big = 1;
    if (!is_init && all_na > 0) {
        const uint32_t want = SEG_TARGET / all_na;
        while (segs_all < 16u && 2u * segs_all <= want) segs_all *= 2u;
        // requests whose lanes may list more candidates than the LDS buffer
        // keep the excess in Work::seg_buf: all_na * segs_big <= SEG_BIG_LANES
        const uint32_t want_big = SEG_BIG_LANES / all_na;
        while (segs_big < 16u && 2u * segs_big <= want_big) segs_big *= 2u;
    }
    uint32_t A = 0, P = 0, rays = 0, AT = 0, BL = 0;   // running bases, wave-uniform
    for (uint32_t r0 = 0; r0 < nreq; r0 += 64u) {
        const uint32_t r = r0 + l;
        const bool valid = r < nreq;
        ReqState *st = r0 == 0 ? st0 : (valid ? T.reqs[r].st : nullptr);
        const uint32_t na = r0 == 0 ? na0 : (valid ? st->n_act : 0u);
        const uint32_t ns_in = r0 == 0 ? ns0 : (valid ? st->n_spec : 0u);
        const uint32_t ps = r0 == 0 ? ps0 : (valid ? st->passes : 0u);
        const uint32_t pol = valid ? T.reqs[r].policy : SPEC_UNIFORM;
        const uint32_t cap = valid ? T.reqs[r].spec_cap : 0u, npx = valid ? T.reqs[r].npix : 0u;
        // a request's first pass takes N_spec = clamp(floor(w*h / N_act), 1, cap) (Sec. 4) with its
        // current cap (the cap may change between the initial rays and the first pass)
        uint32_t ns = ns_in;
        if (!is_init && ps == 0u && na > 0u) {
            const uint32_t q0 = npx / na;
            ns = q0 < 1u ? 1u : (q0 > cap ? cap : q0);
        }
        // per-ray counts: each ray's count is at most cap and they sum to at
        // most w*h, so the request's slot space is the smaller of the two
        const uint64_t pr_space = (uint64_t)na * cap < (uint64_t)npx ? (uint64_t)na * cap : (uint64_t)npx;
        const uint32_t most = pol == SPEC_PER_RAY ? cap : ns;   // most candidates a ray lists
        const bool seg_ok = most <= TR_BUF, big_ok = !seg_ok && most <= SEG_BIG_NS;
        const uint32_t segs = na > 0 ? (seg_ok ? segs_all : (big_ok ? segs_big : 1u)) : 1u;
        const uint32_t a = round64(na), at = round64(na * segs);
        const uint32_t bl = (big_ok && segs > 1u) ? na * segs : 0u;
        const uint32_t pp = is_init ? 0u : (pol == SPEC_PER_RAY ? (uint32_t)pr_space : na * ns);
        uint32_t ta, tat, tp, tr, tb;
        const uint32_t ia = wave_incl_scan(a, &ta), iat = wave_incl_scan(at, &tat), ip = wave_incl_scan(pp, &tp);
        const uint32_t ib = wave_incl_scan(bl, &tb);
        (void)wave_incl_scan(na, &tr);
        if (valid) {
            st->segs = segs;
            st->slot_cursor = pol == SPEC_PER_RAY ? 0u : pp;   // per-ray counts: handed out by the traversal
            T.trav_base[r] = AT + iat - at;
            T.big_base[r] = BL + ib - bl;
            T.act_base[r] = A + ia - a;
            T.pair_base[r] = P + ip - pp;
            st->n_act_prev = na;
            st->last_nspec = ns;
            st->last_pairs = 0; st->last_deferred = 0; st->last_terminated = 0;
            if (na > 0 && !is_init) {
                if (ps == 0) st->entered = na;
                st->passes = ps + 1u;
            }
        }
        A += ta; P += tp; AT += tat; rays += tr; BL += tb;
    }
    if (l != 0) return;
    ctl->pass += 1;
    ctl->n_vis = 0; ctl->v_adm = 0; ctl->n_actblk = 0; ctl->n_miss = 0; ctl->n_hit = 0;
    ctl->cursor = 0; ctl->served = 0; ctl->deferred = 0; ctl->need = 0; ctl->evict_T = 64;
    ctl->evict_done_blocks = 0; ctl->evicted = 0; ctl->terminated = 0; ctl->pairs = 0; ctl->overflow = 0;
    ctl->guard = 0;
    ctl->csteps = 0;
    ctl->cmasks = 0;
    ctl->rays = rays;
    T.act_base[nreq] = A;
    T.pair_base[nreq] = P;
    T.trav_base[nreq] = AT;
    ctl->A_trav = AT;
    ctl->A = A;
    ctl->P = P;
    ctl->nreq = nreq;
}

// ----------------------------------------------------------- isovalue masks --
// Per request and coarse cell, one 64-bit word: bit (bx&3) + 4(by&3) +
// 16(bz&3) is set when that block's fine range contains the isovalue
// (inclusive, compared in float32: exactly the test the traversal needs).
// The word is 0 when the coarse range does not contain the isovalue (Sec. 3.1
// coarse grid), and a zero word lets the traversal skip the whole coarse cell.
// The walk loads one word per coarse cell and tests blocks in registers.
// The set bits also count the blocks whose fine range contains the isovalue
// (one atomic per workgroup into the request's state).
//
// A wave takes 64 consecutive coarse cells: lane l tests the coarse range of
// cell c0 + l; for the cells that pass (up to four at a time), lane i reads
// the fine range of block i of the cell, and the ballot of the lanes' tests
// is the cell's word.  Every fine range read is one of a cell whose coarse
// range contains the isovalue, and the four cells' reads are in flight
// together.  The kernel also seeds the empty-space distances: 0 for a
// nonzero word, CD_MAX otherwise.
__global__ __launch_bounds__(256) void k_iso_masks(Table T, const VolDev *vols) {
    __shared__ unsigned long long s_cnt, s_cells;
    const ReqDev &q = T.reqs[0];
    const VolDev &V = vols[uni(q.vol)];
    const float iso = uni(q.iso);
    const uint32_t nc0 = (uint32_t)uni(V.nc[0]), nc1 = (uint32_t)uni(V.nc[1]), nc2 = (uint32_t)uni(V.nc[2]);
    const int nb0 = uni(V.nb[0]), nb1 = uni(V.nb[1]), nb2 = uni(V.nb[2]);
    const uint64_t nc = (uint64_t)nc0 * nc1 * nc2;
    const float2 *__restrict__ coarse = uni(V.coarse);
    const float2 *__restrict__ fine = uni(V.fine);
    const gptr<uint64_t> out = as_global(uni(q.cmask64));
    const gptr<uint8_t> occ = as_global(uni(q.cdist) + nc);
    if (threadIdx.x == 0) { s_cnt = 0; s_cells = 0; }
    __syncthreads();
    const uint32_t lane = lane_id();
    const int ox = (int)(lane & 3u), oy = (int)((lane >> 2) & 3u), oz = (int)(lane >> 4);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    unsigned long long my = 0, mycells = 0;
    for (uint64_t c0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; c0 < nc; c0 += nwaves * 64) {
        const uint64_t c = c0 + lane;
        bool cand = false;
        if (c < nc) {
            const float2 cr = coarse[c];
            cand = cr.x <= iso && iso <= cr.y;
        }
        uint64_t todo = __ballot(cand);
        mycells += lane == 0u ? (unsigned long long)__popcll(todo) : 0ull;
        uint64_t mine = 0;
        while (todo) {
            int k[4];
            float2 r[4];
            bool in[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                k[u] = todo ? __ffsll((unsigned long long)todo) - 1 : -1;
                todo &= todo ? todo - 1 : 0ull;
                in[u] = false;
                r[u] = make_float2(1.0f, 0.0f);
                if (k[u] >= 0) {
                    int cx, cy, cz;
                    unravel3((uint32_t)(c0 + (uint64_t)k[u]), nc0, nc1, cx, cy, cz);
                    const int x = 4 * cx + ox, y = 4 * cy + oy, z = 4 * cz + oz;
                    in[u] = x < nb0 && y < nb1 && z < nb2;
                    if (in[u]) r[u] = fine[((uint64_t)z * (uint32_t)nb1 + (uint32_t)y) * (uint32_t)nb0 + (uint32_t)x];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t bits = __ballot(in[u] && r[u].x <= iso && iso <= r[u].y);
                if (k[u] >= 0 && (int)lane == k[u]) mine = bits;
            }
        }
        if (c < nc) {
            out[c] = mine;
            occ[c] = mine != 0ull ? (uint8_t)0 : (uint8_t)CD_MAX;   // input of the empty-space distances
        }
        my += (unsigned long long)__popcll(mine);
    }
    if (my) atomicAdd(&s_cnt, my);
    if (mycells) atomicAdd(&s_cells, mycells);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(&q.st->bcmc, s_cnt);
    if (threadIdx.x == 0 && s_cells) atomicAdd(&q.st->ccells, s_cells);
}

// Empty-space distances (per request, after the masks).  Chessboard distance
// is separable: with f0 = 0 on coarse cells whose mask is nonzero and CD_MAX
// elsewhere, f_{a}(c) = min over |k| <= CD_MAX of max(|k|, f_{a-1}(c + k e_a))
// along x, then y, then z gives, per cell, the distance (capped at CD_MAX) to
// the nearest nonzero cell.  Capping only underestimates: the walk then jumps
// less far, never over a nonzero cell.

// One separable pass along `axis`, tiled through LDS: a workgroup takes 32
// positions along the axis (plus the CD_MAX positions on either side) of 64
// adjacent lines, reads them once, and every output takes its 2*CD_MAX+1
// window from LDS.  Positions outside the volume read as 255, which never
// lowers a minimum.
constexpr int CD_TA = 32, CD_TL = 64, CD_SPAN = CD_TA + 2 * CD_MAX;

template <int AXIS>
__global__ __launch_bounds__(256) void k_cdist_pass(Table T, const VolDev *vols) {
    __shared__ uint8_t s_win[CD_SPAN][CD_TL];   // [position][line]
    const ReqDev &q = T.reqs[0];
    const VolDev &V = vols[uni(q.vol)];
    const int n0 = uni(V.nc[0]), n1 = uni(V.nc[1]), n2 = uni(V.nc[2]);
    const uint64_t nc = (uint64_t)n0 * n1 * n2;
    uint8_t *const cd = uni(q.cdist);
    // x: scratch -> final, y: final -> scratch, z: scratch -> final
    const uint8_t *src = AXIS == 1 ? cd : cd + nc;
    uint8_t *dst = AXIS == 1 ? cd + nc : cd;
    // the axis, the line axis (x, or y for the x pass) and the third axis
    const int na = AXIS == 0 ? n0 : (AXIS == 1 ? n1 : n2);
    const int nl = AXIS == 0 ? n1 : n0;
    const int n3 = AXIS == 2 ? n1 : n2;
    auto index = [&](int pa, int pl, int p3) -> uint64_t {
        const int x = AXIS == 0 ? pa : pl;
        const int y = AXIS == 0 ? pl : (AXIS == 1 ? pa : p3);
        const int z = AXIS == 2 ? pa : p3;
        return ((uint64_t)z * (uint32_t)n1 + (uint32_t)y) * (uint32_t)n0 + (uint32_t)x;
    };
    const int tiles_a = (na + CD_TA - 1) / CD_TA, tiles_l = (nl + CD_TL - 1) / CD_TL;
    const int ntiles = tiles_a * tiles_l * n3;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ta = tile % tiles_a, tl = (tile / tiles_a) % tiles_l, t3 = tile / (tiles_a * tiles_l);
        const int a0 = ta * CD_TA - CD_MAX, l0 = tl * CD_TL;
        for (int e = threadIdx.x; e < CD_SPAN * CD_TL; e += blockDim.x) {
            // the x pass reads along x (contiguous), the others across lines along x
            const int pos = AXIS == 0 ? e % CD_SPAN : e / CD_TL;
            const int line = AXIS == 0 ? e / CD_SPAN : e % CD_TL;
            const int pa = a0 + pos, pl = l0 + line;
            uint8_t v = 255;
            if (pa >= 0 && pa < na && pl < nl) v = src[index(pa, pl, t3)];
            s_win[pos][line] = v;
        }
        __syncthreads();
        const int line = threadIdx.x % CD_TL, pl = l0 + line;
        for (int pos = threadIdx.x / CD_TL; pos < CD_TA; pos += blockDim.x / CD_TL) {
            const int pa = ta * CD_TA + pos;
            if (pa >= na || pl >= nl) continue;
            int best = CD_MAX;
#pragma unroll
            for (int k = -CD_MAX; k <= CD_MAX; ++k) {
                const int v = s_win[pos + CD_MAX + k][line];
                const int ak = k < 0 ? -k : k;
                const int d = ak > v ? ak : v;
                best = d < best ? d : best;
            }
            dst[index(pa, pl, t3)] = (uint8_t)best;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t local_bit(const int cb[3]) {
    return (uint32_t)((cb[0] & 3) + 4 * (cb[1] & 3) + 16 * (cb[2] & 3));
}

// ------------------------------------------------------------ initial rays --
// Sec. 3.2: one thread per pixel computes the ray and its volume entry; rays
// that miss are terminated; image and hit buffer are cleared, and so is the
// per-pixel pass state.  The alive counts feed the same count/compact kernels
// as a pass.
//
// The active-ray list starts in tile order: initial index i covers the
// pixels in 8x8 tiles (one wave each), tiles left to right within bands of 8
// rows, bands top to bottom; the last band and each band's last tile may be
// smaller.  Compaction keeps the order, so the rays of a wave stay close on
// screen in every pass and walk similar cells: a wave lasts as long as its
// longest walk.  Per-pixel results do not depend on the order.
__device__ __forceinline__ uint32_t tile_pixel(uint32_t i, uint32_t w, uint32_t h) {
    const uint32_t band = i / (8u * w);
    const uint32_t y0 = 8u * band;
    const uint32_t bh = h - y0 < 8u ? h - y0 : 8u;
    const uint32_t j = i - y0 * w;       // index within the band of bh rows
    const uint32_t ct = j / (8u * bh);   // tile column; tiles before it hold 8*bh pixels each
    const uint32_t k = j - ct * 8u * bh;
    const uint32_t tw = w - 8u * ct < 8u ? w - 8u * ct : 8u;
    return (y0 + k / tw) * w + 8u * ct + k % tw;
}

__global__ void k_init_rays(PassCtl *ctl, Table T, const VolDev *vols) {
    uint32_t A = ctl->A;
    // a mask set kept by the volume carries the counts of the render that
    // built it; renders that reuse the set take them from there
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (uint32_t r = 0; r < ctl->nreq; ++r) {
            const ReqDev &q = T.reqs[r];
            unsigned long long *ms = q.mstat;
            if (ms && q.mstat_load) {
                q.st->bcmc = ms[0];
                q.st->ccells = ms[1];
            } else if (ms) {
                ms[0] = q.st->bcmc;
                ms[1] = q.st->ccells;
            }
        }
    }
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        // all lanes of a wave share a request (the A space is 64-aligned per request)
        uint32_t r = __builtin_amdgcn_readfirstlane(find_req(T.act_base, ctl->nreq, p));
        const ReqDev &q = T.reqs[r];
        uint32_t i = p - T.act_base[r];
        bool alive = false;
        uint32_t w = 0;
        if (i < q.npix) {
            const uint32_t pix = tile_pixel(i, q.w, q.h);
            Ray R;
            make_ray(q, vols[q.vol].n, pix, R);
            alive = R.entered != 0;
            w = alive ? ray_weight(R.te, R.tx) : 0u;
            q.ray_state[pix] = alive ? RAY_NOT_STARTED : RAY_DONE;
            q.act[1][i] = pix;
            // the per-pixel clears cover every pixel once: by index
            q.image[i] = 0u;
            spr_hit h;
            h.t = __builtin_inf();
            h.block_id = NONE;
            h.cell = NONE;
            q.hits[i] = h;
            q.best[i] = ~0ull;       // per-pixel pass state: no hit, nothing deferred
            q.def_first[i] = NONE;
        }
        uint64_t m = __ballot(alive);
        // the entered rays' weights (per-ray speculation counts of the first
        // pass); every lane of the wave is here
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) w += (uint32_t)__shfl_xor((int)w, off);
        if (lane_id() == 0) {
            T.wave_rec[p >> 6] = make_uint4((uint32_t)__popcll(m), 0u, 0u, 0u);
            T.wave_w[p >> 6] = w;
        }
    }
}

// ---------------------------------------------------------------- K1 ------
// Speculative two-level macrocell traversal (Sec. 3.3 and 4.1).  Each active
// ray resumes after the last block it was served (or at its volume entry),
// walks the coarse grid, descends into coarse cells whose range contains the
// isovalue and walks their blocks, and records up to N_spec blocks whose fine
// range contains the isovalue at slots i*N_spec + k; unused slots get NONE.
// The walk does no atomics: visible-block dedupe runs in its own kernel.

__device__ __forceinline__ bool range_has(float2 r, float iso) { return r.x <= iso && iso <= r.y; }


__global__ __launch_bounds__(256) void k_traverse(PassCtl *ctl, Table T, const VolDev *vols, Work W) {
    __shared__ uint32_t s_slot[TR_BUF][256];
    const uint32_t AT = ctl->A_trav;
    const uint32_t nreq = ctl->nreq;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < AT; p += gridDim.x * blockDim.x) {
        // all lanes of a wave share a request (the lane space is 64-aligned per
        // request); ray i of the request runs on lanes i*L .. i*L+L-1
        const uint32_t r = uni(find_req(T.trav_base, nreq, p));
        const ReqDev &q = T.reqs[r];
        ReqState *st = uni(q.st);
        const uint32_t L = uni(st->segs);
        const uint32_t local = p - uni(T.trav_base[r]);
        const uint32_t i = local >> __builtin_ctz(L);
        const uint32_t seg = local & (L - 1u);
        if (i >= uni(st->n_act_prev)) continue;   // whole segment groups only
        const uint32_t ns = uni(st->last_nspec);
        const uint32_t pix = uni(q.act[uni(st->cur)])[i];
        WaveReq u;
        load_wave_req(q, vols[uni(q.vol)], u);
        const gptr<const uint64_t> cmask = as_global((const uint64_t *)uni(q.cmask64));
        const gptr<const uint8_t> cdist = as_global((const uint8_t *)uni(q.cdist));
        const uint32_t state = uni(q.ray_state)[pix];
        Ray R;
        make_ray(u, u.n, pix, R);
        Level LB = {4, {u.tb[0], u.tb[1], u.tb[2]}, {u.n[0], u.n[1], u.n[2]}, 0.25};
        Level LC = {16, {u.tc[0], u.tc[1], u.tc[2]}, {u.n[0], u.n[1], u.n[2]}, 0.0625};
        const int zero3[3] = {0, 0, 0};
        const int tbhi[3] = {u.tb[0] - 1, u.tb[1] - 1, u.tb[2] - 1};
        const int tchi[3] = {u.tc[0] - 1, u.tc[1] - 1, u.tc[2] - 1};
        int cb[3], cc[3];
        AxisWalk wb;   // block-level walk state, valid while bvalid
        AxisWalk wc;   // coarse-level walk state, valid while cvalid
        double tcur;
        bool bvalid, cvalid = false;
        bool alive = true;
        uint32_t found = 0;
        if (state == RAY_NOT_STARTED) {
            tcur = R.te;
#pragma unroll
            for (int a = 0; a < 3; ++a) cc[a] = cell_at(R, LC, a, tcur, 0, tchi[a]);
            bvalid = false;
        } else {
            uint32_t b = state;
            cb[0] = (int)(b % (uint32_t)u.nb[0]);
            cb[1] = (int)((b / (uint32_t)u.nb[0]) % (uint32_t)u.nb[1]);
            cb[2] = (int)(b / ((uint32_t)u.nb[0] * (uint32_t)u.nb[1]));
            walk_init(R, LB, cb, wb);
            double tn = walk_exit(wb);
            if (tn > R.tx || !walk_step(R, LB, wb, cb, tn, zero3, tbhi)) alive = false;
            tcur = tn;
            bvalid = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) cc[a] = cb[a] >> 2;
        }
        // The ray's speculation count and pair slots.  One count for every ray
        // (Sec. 4): slots i*N_spec onwards.  Per-ray counts: the ray's weight
        // from where its remaining walk starts (tcur, the same on every lane of
        // a segment group), its count from the weight sum of the active rays,
        // and its slots from the request's cursor, one atomic per wave (ranges
        // of different rays may lie in any order; a ray's own slots stay
        // consecutive and in walk order).
        const uint32_t pol = uni(q.policy);
        uint32_t nsr = ns, rbase_i = i * ns, wi = 0;
        if (pol == SPEC_PER_RAY) {
            wi = ray_weight(tcur, R.tx);
            nsr = nspec_ray(uni(q.npix), uni(st->n_act_prev), uni((uint64_t)st->wsum), wi, uni(q.spec_cap));
            const uint32_t v = seg == 0u ? nsr : 0u;
            const uint64_t lt = lanemask_lt();
            uint32_t before = 0, total = 0;
#pragma unroll
            for (int bit = 0; bit < 13; ++bit) {   // counts <= 4096: sums of bit planes over the lanes
                const uint64_t bm = __ballot((v >> bit) & 1u);
                before += (uint32_t)__popcll(bm & lt) << bit;
                total += (uint32_t)__popcll(bm) << bit;
            }
            uint32_t base = 0;
            if ((int)lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1)
                base = atomicAdd(&st->slot_cursor, total);
            base = uni(base);
            rbase_i = base + before;
            if (L > 1u) rbase_i = (uint32_t)__shfl((int)rbase_i, (int)(lane_id() & ~(L - 1u)));
        }
        const gptr<uint32_t> slots = as_global(uni(q.pair_blk) + (size_t)rbase_i);
        const gptr<uint32_t> pray = as_global(uni(q.pair_ray) + (size_t)rbase_i);
        const bool per_ray = pol == SPEC_PER_RAY;
        // a segmented lane that may list more candidates than its LDS buffer
        // moves each full buffer to its column of seg_buf (its request has
        // rows there: big_base)
        const bool big = L > 1u && nsr > TR_BUF;
        const uint32_t bli = big ? uni(T.big_base[r]) + local : 0u;
        const gptr<uint32_t> sbuf = as_global(W.seg_buf);
        // Segments (L > 1): the rest of the ray, [t_start, t_exit], is cut at
        // t_k = t_start + (t_exit - t_start) k / L; lane k lists the blocks whose
        // entry parameter lies in [t_k, t_k+1) (the first lane everything below
        // t_1, the last everything from t_L-1 on), so every block the serial
        // walk visits belongs to exactly one lane.  Lane k > 0 starts where the
        // serial walk is at t_k: every plane with parameter <= t_k crossed
        // (cell_at), and the block found there counts only if it was entered at
        // t_k or later.
        double t_lo = -__builtin_inf(), t_hi = __builtin_inf();
        bool fresh = false;   // the next block found by cell_at needs its own entry parameter
        if (L > 1u && alive) {
            const double t0 = tcur, span = R.tx - tcur;
            if (seg + 1u < L) t_hi = t0 + span * (double)(seg + 1u) / (double)L;
            if (seg > 0u) {
                t_lo = t0 + span * (double)seg / (double)L;
                tcur = t_lo;
#pragma unroll
                for (int a = 0; a < 3; ++a) cc[a] = cell_at(R, LC, a, tcur, 0, tchi[a]);
                bvalid = false;
                cvalid = false;
                fresh = true;
            }
        }
        double tau = tcur;    // entry parameter of the current block
        uint32_t nbuf = 0, flushed = 0;   // candidates staged in LDS / already written
        const int max_steps = u.tb[0] + u.tb[1] + u.tb[2] + u.tc[0] + u.tc[1] + u.tc[2] + 16;
        int steps = 0;
        // Outer loop: one coarse cell per iteration (its mask and distance are
        // loaded here, once for the whole wave); an empty cell is left by a
        // jump or a coarse step.  Inner loop: the blocks of a nonempty coarse
        // cell, no memory access but the LDS staging.
        bool guard_hit = false;
        uint32_t csteps = 0;   // coarse cells visited (distance loaded)
        uint32_t cmasks = 0;   // nonempty coarse cells visited (mask word loaded too)
        // The walk's one exit is the loop condition (a single exit mask for the
        // compiler): oexit 1 step guard, 2 the rest is the next lane's, 3 the
        // ray left the volume; or every slot filled.
        int oexit = alive ? 0 : 3;
        while (oexit == 0 && found < nsr) {
            if (++steps > max_steps) {   // every step advances an index
                oexit = 1;
            } else if (tcur >= t_hi && !fresh) {   // the rest is the next lane's
                ++csteps;
                oexit = 2;
            } else {
                ++csteps;
                // The distance byte alone says whether the cell is empty (0 exactly for
                // a cell with a candidate block): it is loaded first and tested first,
                // so an empty cell's jump waits only for it.  The distances are 1 byte
                // per coarse cell (2 MB at 2048x2048x1920, mostly L2 hits), the mask
                // words 8 B (mostly misses).
                const uint64_t cid = ((uint64_t)cc[2] * u.nc[1] + cc[1]) * u.nc[0] + cc[0];
                const int cd = cdist[cid];
                const uint64_t cm = cmask[cid];
                if (cd != 0) {
                    bvalid = false;
                    fresh = false;   // the walk moves on to plane crossings
                    if (cd >= 2) {
                        // every coarse cell within cd-1 (chessboard) is empty: leave that box
                        // in one jump.  t* = the first crossing of one of its faces (or of
                        // the domain) - the parameter at which a cell-by-cell walk leaves
                        // the box - and the coarse cell there is the walk's cell: every
                        // plane with parameter <= t* crossed (cell_at).
                        const int rr = cd - 1;
                        double tn = __builtin_inf();
                        bool domain = false;
    #pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const int dir = axis_dir(R, a);
                            if (dir == 0) continue;
                            int face = dir > 0 ? cc[a] + rr + 1 : cc[a] - rr;
                            face = face < 0 ? 0 : (face > u.tc[a] ? u.tc[a] : face);
                            const double tf = tau_plane(R, LC, a, face);
                            const bool dom = dir > 0 ? face == u.tc[a] : face == 0;
                            if (tf < tn) { tn = tf; domain = dom; }
                            else if (tf == tn) domain = domain || dom;
                        }
                        if (tn > R.tx || domain) {
                            oexit = 3;
                        } else {
    #pragma unroll
                            for (int a = 0; a < 3; ++a) cc[a] = cell_at(R, LC, a, tn, 0, tchi[a]);
                            tcur = tn;
                            cvalid = false;
                        }
                    } else {
                        // empty coarse cell: step over it at the coarse level
                        if (!cvalid) {
                            walk_init(R, LC, cc, wc);
                            cvalid = true;
                        }
                        double tn = walk_exit(wc);
                        if (tn > R.tx || !walk_step(R, LC, wc, cc, tn, zero3, tchi)) oexit = 3;
                        else tcur = tn;
                    }
                } else {
                ++cmasks;
                if (!bvalid) {
    #pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        int lo = 4 * cc[a], hi = 4 * cc[a] + 3;
                        if (hi > tbhi[a]) hi = tbhi[a];
                        cb[a] = cell_at(R, LB, a, tcur, lo, hi);
                    }
                    walk_init(R, LB, cb, wb);
                    bvalid = true;
                    tau = fresh ? cell_entry(R, LB, cb) : tcur;
                    fresh = false;
                }
                cvalid = false;
                // One exit from the block loop, with its reason: a single exit mask
                // for the compiler to keep instead of one per break.
                //   1 the rest is the next lane's, 2 all slots filled, 3 step guard,
                //   4 the ray left the volume, 5 the walk entered another coarse cell
                int why = 0;
                do {
                    if (tau >= t_hi) {
                        why = 1;
                    } else {
                        const bool emit = tau >= t_lo && ((cm >> local_bit(cb)) & 1ull);
                        if (emit) {
                            const uint32_t bid = (uint32_t)(((uint64_t)cb[2] * u.nb[1] + cb[1]) * u.nb[0] + cb[0]);
                            s_slot[nbuf][threadIdx.x] = bid;
                            found++;
                            if (++nbuf == TR_BUF && (L == 1u || big)) {
                                if (L == 1u) {
                                    for (uint32_t k = 0; k < TR_BUF; ++k) {
                                        slots[flushed + k] = s_slot[k][threadIdx.x];
                                        if (per_ray) pray[flushed + k] = i;
                                    }
                                } else {
                                    gptr<uint32_t> d = sbuf + ((size_t)flushed * SEG_BIG_LANES + bli);
    #pragma unroll 1
                                    for (uint32_t k = 0; k < TR_BUF; ++k, d += SEG_BIG_LANES) *d = s_slot[k][threadIdx.x];
                                }
                                flushed += TR_BUF;
                                nbuf = 0;
                            }
                        }
                        if (found == nsr) {
                            why = 2;
                        } else if (++steps > max_steps) {
                            why = 3;
                        } else {
                            const double tn = walk_exit(wb);
                            if (tn > R.tx || !walk_step(R, LB, wb, cb, tn, zero3, tbhi)) {
                                why = 4;
                            } else {
                                tcur = tn;
                                tau = tn;
                                if ((cb[0] >> 2) != cc[0] || (cb[1] >> 2) != cc[1] || (cb[2] >> 2) != cc[2]) why = 5;
                            }
                        }
                    }
                } while (why == 0);
                    oexit = why == 1 ? 2 : (why == 3 ? 1 : (why == 4 ? 3 : 0));
                    if (why == 5) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) cc[a] = cb[a] >> 2;
                    }
                }
            }
        }
        guard_hit = oexit == 1;
        if (guard_hit) atomicAdd(&ctl->guard, 1u);   // counted, so that tests can assert it never happens
        // The block of pair 0 (the first active ray's first candidate) takes
        // visible-list index 0, so it is always admitted and every pass makes
        // progress under the cache-capacity rule: reserve that index.
        if (L == 1u) {
            for (uint32_t k = 0; k < nbuf; ++k) {
                slots[flushed + k] = s_slot[k][threadIdx.x];
                if (per_ray) pray[flushed + k] = i;
            }
            for (uint32_t k = found; k < nsr; ++k) slots[k] = NONE;
            if (found > 0 && T.pair_base[r] + rbase_i == 0) ctl->n_vis = 1u;
        } else {
            // merge the lanes' lists in segment order: lane k's candidates go
            // after those of lanes 0..k-1; the first ns are the ray's slots
            uint32_t incl = found;
            for (uint32_t d = 1; d < L; d <<= 1) {
                const uint32_t o = (uint32_t)__shfl_up((int)incl, d, (int)L);
                if (seg >= d) incl += o;
            }
            const uint32_t before = incl - found;
            const uint32_t total = (uint32_t)__shfl((int)incl, (int)(L - 1u), (int)L);
            const uint32_t lim = before < nsr ? (found < nsr - before ? found : nsr - before) : 0u;
            const uint32_t lim_col = lim < flushed ? lim : flushed;
            // the column-buffer part 16 entries at a time, loads issued together
            for (uint32_t k0 = 0; k0 < lim_col; k0 += 16) {
                uint32_t v[16];
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j)
                    v[j] = k0 + j < lim_col ? sbuf[(size_t)(k0 + j) * SEG_BIG_LANES + bli] : 0u;
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j)
                    if (k0 + j < lim_col) {
                        slots[before + k0 + j] = v[j];
                        if (per_ray) pray[before + k0 + j] = i;
                    }
            }
            for (uint32_t k = lim_col; k < lim; ++k) {
                slots[before + k] = s_slot[k - flushed][threadIdx.x];
                if (per_ray) pray[before + k] = i;
            }
            if (seg == 0u) {
                for (uint32_t k = total < nsr ? total : nsr; k < nsr; ++k) slots[k] = NONE;
                if (total > 0 && T.pair_base[r] + rbase_i == 0) ctl->n_vis = 1u;
            }
            found = total < nsr ? total : nsr;   // the ray's candidates (every lane of the group)
        }
        // The ray's outcome as far as the walk decides it: its candidate
        // count, which tells the pair that finishes the ray last how many to
        // wait for, and, with no candidate left, its termination (it leaves
        // the volume with no block that can hold the isovalue).  The wave's
        // pair and termination counts go to the wave record of its rays in
        // one atomic each (all rays of a traversal wave share one wave of the
        // active-ray space).
        const bool lead = seg == 0u;
        const bool term = lead && found == 0u;
        if (lead) {
            as_global(uni(q.nfound))[pix] = found;
            as_global(uni(q.rbase))[pix] = rbase_i;
            as_global(uni(q.rns))[pix] = nsr;
            if (per_ray) as_global(uni(q.rw))[pix] = wi;
            if (term) as_global(uni(q.ray_state))[pix] = RAY_DONE;
        }
        uint32_t wpairs = 0;
#pragma unroll
        for (int bit = 0; bit < 13; ++bit)   // found <= ns <= 4096: a sum of bit planes over the lanes
            wpairs += (uint32_t)__popcll(__ballot(lead && ((found >> bit) & 1u))) << bit;
        const uint32_t wterm = (uint32_t)__popcll(__ballot(term));
        uint32_t wsteps = 0, wmasks = 0;
#pragma unroll
        for (int bit = 0; bit < 16; ++bit) {   // csteps, cmasks <= max_steps < 2^16
            wsteps += (uint32_t)__popcll(__ballot((csteps >> bit) & 1u)) << bit;
            wmasks += (uint32_t)__popcll(__ballot((cmasks >> bit) & 1u)) << bit;
        }
        const uint64_t act = __ballot(1);
        if ((int)lane_id() == __ffsll((unsigned long long)act) - 1) {
            uint4 *rec = T.wave_rec + ((uni(T.act_base[r]) + i) >> 6);
            if (wpairs) atomicAdd(&rec->y, wpairs);
            if (wterm) atomicAdd(&rec->w, wterm);
            if (wsteps) atomicAdd(&ctl->csteps, wsteps);
            if (wmasks) atomicAdd(&ctl->cmasks, wmasks);
        }
    }
}

// --------------------------------------------------------------- K1b ------
// Visible blocks (Sec. 3.4) and pair ranks (the N_BRays count of Sec. 3.6) in
// one atomic per pair: the pair takes its rank within its block from the
// block's pass counter; rank 0 is the first visitor, which appends the block
// to the visible list and records its index (pair 0's block takes the
// reserved index 0).  Counters are zero between
// passes (K2 clears the ones it reads).  Each thread takes DD_ITEMS pairs, so
// a workgroup appends DD_ITEMS*256 pairs' worth of blocks with one atomic.
constexpr int DD_ITEMS = 4;

__global__ __launch_bounds__(256) void k_dedupe(PassCtl *ctl, Table T, const VolDev *vols, Work W) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint32_t P = ctl->P;
    const uint32_t nreq = ctl->nreq;
    if (P == 0) return;
    // pair 0's block owns the reserved index 0 (set up by the traversal)
    const uint32_t r0 = find_req(T.pair_base, nreq, 0u);
    const uint32_t b0 = T.reqs[r0].pair_blk[0];
    const uint32_t vol0 = T.reqs[r0].vol;
    constexpr uint32_t SPAN = 256u * DD_ITEMS;
    for (uint32_t x0 = blockIdx.x * SPAN; x0 < P; x0 += gridDim.x * SPAN) {
        uint32_t b[DD_ITEMS], vol[DD_ITEMS], bi[DD_ITEMS];
        uint32_t firsts = 0, nf = 0;
#pragma unroll
        for (int k = 0; k < DD_ITEMS; ++k) {
            const uint32_t x = x0 + (uint32_t)k * 256u + threadIdx.x;
            b[k] = NONE;
            vol[k] = 0;
            bi[k] = 0;
            if (x < P) {
                const uint32_t r = find_req(T.pair_base, nreq, x);
                const ReqDev &q = T.reqs[r];
                const uint32_t qq = x - T.pair_base[r];
                // slots past the request's cursor were not handed out this pass
                b[k] = qq < q.st->slot_cursor ? q.pair_blk[qq] : NONE;
                vol[k] = q.vol;
            }
        }
        // Ranks: one atomic per pair on its block's counter, the DD_ITEMS
        // atomics of a thread issued together; the ranks of a block are
        // exactly 0 .. count-1 in some order.
        uint32_t rank[DD_ITEMS];
#pragma unroll
        for (int k = 0; k < DD_ITEMS; ++k) {
            rank[k] = NONE;
            if (b[k] != NONE) {
                bi[k] = bidx(vol_state(vols[vol[k]]), b[k]);
                rank[k] = __hip_atomic_fetch_add(as_global(vols[vol[k]].blk_cnt) + bi[k], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            }
        }
#pragma unroll
        for (int k = 0; k < DD_ITEMS; ++k) {
            if (b[k] == NONE) continue;
            W.pair_rank[x0 + (uint32_t)k * 256u + threadIdx.x] = rank[k];
            if (rank[k] == 0) {
                if (b[k] == b0 && vol[k] == vol0) {
                    W.vis_list[0] = ((uint64_t)vol0 << 32) | b0;
                    vols[vol0].vis_idx[bi[k]] = 0u;
                } else {
                    firsts |= 1u << k;
                    nf++;
                }
            }
        }
        uint32_t idx = block_bump<256>(&ctl->n_vis, nf, s_tmp);
#pragma unroll
        for (int k = 0; k < DD_ITEMS; ++k) {
            if ((firsts >> k) & 1u) {
                W.vis_list[idx] = ((uint64_t)vol[k] << 32) | b[k];
                vols[vol[k]].vis_idx[bi[k]] = idx;
                idx++;
            }
        }
    }
}

// ---------------------------------------------------------------- K2 ------
// Per visible block: read and clear its pair count.  An admitted block
// (Sec. 3.4 cache-capacity rule) gets its run of sorted pairs (O_BRays of
// Sec. 3.6) by block-aggregated bump allocation, and marks itself and its
// +x/+y/+z face, edge and corner neighbours active (Sec. 3.4).  The first
// visitor of a block this pass (its bit in the coarse cell's claim word) also does its cache
// lookup (Sec. 3.5): a hit refreshes the slot's LRU stamp, a miss is
// appended to the miss list.  Pairs on blocks beyond the admitted prefix
// are counted as deferred.

__device__ __forceinline__ uint32_t admitted_blocks(const PassCtl *ctl) {
    uint32_t nv = ctl->n_vis;
    uint32_t cap = ctl->n_slots / 8u;
    return nv < cap ? nv : cap;
}

__global__ __launch_bounds__(256) void k_mark(PassCtl *ctl, const VolDev *vols, Work W, Cache C) {
    __shared__ uint2 s_tmp2[256 / 64 + 1];
    __shared__ uint32_t s_def, s_act;
    const uint32_t nv = ctl->n_vis;
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t pass = ctl->pass;
    if (threadIdx.x == 0) { s_def = 0; s_act = 0; }
    uint32_t my_def = 0, my_act = 0;
    for (uint32_t x0 = blockIdx.x * 256u; x0 < nv; x0 += gridDim.x * 256u) {
        const uint32_t j = x0 + threadIdx.x;
        uint32_t cnt = 0, missmask = 0, nmiss = 0;
        uint64_t e = 0;
        int bx = 0, by = 0, bz = 0;
        VolState S{};
        if (j < nv) {
            e = W.vis_list[j];
            S = vol_state(vols[(uint32_t)(e >> 32)]);
            const uint32_t b = (uint32_t)e;
            const uint32_t rr = b / (uint32_t)S.nb0;
            bx = (int)(b - rr * (uint32_t)S.nb0);
            by = (int)(rr % (uint32_t)S.nb1);
            bz = (int)(rr / (uint32_t)S.nb1);
            const uint32_t bi = bidx_xyz(S, bx, by, bz);
            const gptr<uint32_t> bc = as_global(S.blk_cnt);
            cnt = bc[bi];
            bc[bi] = 0u;
            if (j < vadm) {
                // The 8 neighbours in two straight-line steps - claims, then
                // slot map reads - so that each step's accesses go out
                // together: one round trip per step, not per neighbour.  A
                // claim sets the neighbour's bit in its coarse cell's claim
                // word; the neighbours in one coarse cell (all 8 when the
                // block is not on its cell's +x/+y/+z faces) are claimed by
                // one atomic OR, and a neighbour whose bit was clear before
                // is first.  A neighbour outside the volume takes the
                // block's own index and is masked out.
                const gptr<uint64_t> claim = as_global(S.claim);
                const gptr<const uint32_t> map = as_global((const uint32_t *)S.map);
                uint32_t nbi[8], sl[8];
                uint64_t grp[8], old[8];
                uint32_t inside = 0, lead = 0;
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int x2 = bx + (o & 1), y2 = by + ((o >> 1) & 1), z2 = bz + (o >> 2);
                    const bool ok = x2 < S.nb0 && y2 < S.nb1 && z2 < S.nb2;
                    nbi[o] = ok ? bidx_xyz(S, x2, y2, z2) : bi;
                    inside |= ok ? 1u << o : 0u;
                }
                // brick index = coarse cell * 64 + bit: group the neighbours by cell
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    grp[o] = 0ull;
                    bool first = true;
#pragma unroll
                    for (int o2 = 0; o2 < 8; ++o2) {
                        const bool same = (nbi[o2] >> 6) == (nbi[o] >> 6);
                        grp[o] |= same ? 1ull << (nbi[o2] & 63u) : 0ull;
                        if (o2 < o && same) first = false;
                    }
                    lead |= first ? 1u << o : 0u;
                }
#pragma unroll
                for (int o = 0; o < 8; ++o)
                    old[o] = ((lead >> o) & 1u) ? __hip_atomic_fetch_or(claim + (nbi[o] >> 6), grp[o], __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT)
                                                : 0ull;
#pragma unroll
                for (int o = 0; o < 8; ++o) sl[o] = map[nbi[o]];
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    // the claim word's previous value, from the atomic of o's group
                    uint64_t was = 0ull;
#pragma unroll
                    for (int o2 = 0; o2 < 8; ++o2)
                        was |= ((nbi[o2] >> 6) == (nbi[o] >> 6)) ? old[o2] : 0ull;
                    if (((inside >> o) & 1u) && !((was >> (nbi[o] & 63u)) & 1ull)) {   // first visitor: cache lookup
                        my_act++;
                        if (sl[o] == NONE) {
                            missmask |= 1u << o;
                            nmiss++;
                        } else {
                            C.stamp[sl[o]] = pass;
                        }
                    }
                }
            } else {
                my_def += cnt;
            }
        }
        const uint2 om = block_bump2<256>(&ctl->cursor, j < vadm ? cnt : 0u, &ctl->n_miss, nmiss, s_tmp2);
        if (j < vadm) W.vis_off[j] = om.x;
        uint32_t mi = om.y;
        if (missmask) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                if ((missmask >> o) & 1u) {
                    const int x2 = bx + (o & 1), y2 = by + ((o >> 1) & 1), z2 = bz + (o >> 2);
                    const uint32_t nbid = (uint32_t)(((uint64_t)z2 * (uint32_t)S.nb1 + y2) * (uint32_t)S.nb0 + x2);
                    W.miss_list[mi++] = (e & 0xFFFFFFFF00000000ull) | nbid;
                }
            }
        }
    }
    if (my_def) atomicAdd(&s_def, my_def);
    if (my_act) atomicAdd(&s_act, my_act);
    __syncthreads();
    if (threadIdx.x == 0 && s_def) atomicAdd(&ctl->deferred, s_def);
    if (threadIdx.x == 0 && s_act) atomicAdd(&ctl->n_actblk, s_act);
}

// ---------------------------------------------------------------- K4 ------
// Slot supply.  If the free stack holds fewer slots than the misses, an LRU
// sweep reclaims the oldest occupied slots not used this pass: a histogram of
// ages (pass - stamp, clamped to 63) picks the largest age threshold whose
// tail covers max(shortfall, n_slots/16) slots, and every slot at or above it
// is evicted in one sweep.
// Allocation plan, then (only when the free slots run short) the age
// histogram of the slots not used this pass.  Every workgroup computes the
// plan from the counters, which are final here; workgroup 0 publishes it.
// The admitted blocks' runs cover exactly the served pairs; eviction frees at
// least the shortfall, in batches of n_slots/16.
__global__ __launch_bounds__(256) void k_evict_hist(PassCtl *ctl, Cache C) {
    const uint32_t m = ctl->n_miss, f = ctl->free_top;
    uint32_t need = 0;
    if (m > f) {
        const uint32_t short_by = m - f, batch = ctl->n_slots / 16u;
        need = short_by > batch ? short_by : batch;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->served = ctl->cursor;
        ctl->need = need;
    }
    if (need == 0) return;
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
        uint32_t acc = 0, T = 1;
        for (int a = 63; a >= 1; --a) {
            acc += __hip_atomic_load(&ctl->hist[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (acc >= need) { T = (uint32_t)a; break; }
        }
        ctl->evict_T = T;
    }
}

__global__ __launch_bounds__(256) void k_evict(PassCtl *ctl, const VolDev *vols, Cache C) {
    if (ctl->need == 0) return;
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    __shared__ uint32_t s_ev;
    const uint32_t pass = ctl->pass, T = ctl->evict_T;
    if (threadIdx.x == 0) s_ev = 0;
    uint32_t my_ev = 0;
    for (uint32_t s0 = blockIdx.x * 256u; s0 < C.n_slots; s0 += gridDim.x * 256u) {
        const uint32_t s = s0 + threadIdx.x;
        bool ev = false;
        if (s < C.n_slots) {
            uint64_t o = C.owner[s];
            if (o != ~0ull) {
                uint32_t st = C.stamp[s];
                uint32_t age = pass - st;
                if (st != pass && (age > 63u ? 63u : age) >= T) {
                    ev = true;
                    const VolDev &V = vols[(uint32_t)(o >> 32)];
                    V.map[bidx(V, (uint32_t)o)] = NONE;
                    C.owner[s] = ~0ull;
                }
            }
        }
        const uint32_t idx = block_bump<256>(&ctl->free_top, ev ? 1u : 0u, s_tmp);
        if (ev) {
            C.free_stack[idx] = s;
            my_ev++;
        }
    }
    if (my_ev) atomicAdd(&s_ev, my_ev);
    __syncthreads();
    if (threadIdx.x == 0 && s_ev) atomicAdd(&ctl->evicted, s_ev);
}

// ---------------------------------------------------------------- K5 ------
// Role A (first assign_groups workgroups): hand the top n_miss free slots to
// the misses.  Role B (the rest): scatter served pairs into their block's run
// (the sort by block id of Sec. 3.6 / 4.2; the pair slot carries O_Spec).
__global__ __launch_bounds__(256) void k_assign_scatter(PassCtl *ctl, Table T, const VolDev *vols, Work W, Cache C,
                                                        uint32_t assign_groups) {
    if (blockIdx.x < assign_groups) {
        const uint32_t f = ctl->free_top;
        uint32_t m = ctl->n_miss;
        if (m > f) m = f;   // cannot happen: admission keeps the active blocks within n_slots
        const uint32_t base = f - m;
        const uint32_t pass = ctl->pass;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->assigned = m;
            if (m < ctl->n_miss) ctl->overflow = 1;
        }
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += assign_groups * blockDim.x) {
            uint64_t e = W.miss_list[i];
            uint32_t sl = C.free_stack[base + i];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            V.map[bidx(V, (uint32_t)e)] = sl;
            C.owner[sl] = e;
            C.stamp[sl] = pass;
            W.miss_slot[i] = sl;
        }
        return;
    }
    const uint32_t P = ctl->P;
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t nthreads = (gridDim.x - assign_groups) * blockDim.x;
    const uint32_t nreq = ctl->nreq;
    for (uint32_t x = (blockIdx.x - assign_groups) * blockDim.x + threadIdx.x; x < P; x += nthreads) {
        // loads in dependency order, all before the stores (through the
        // references they would be read again after each store)
        const uint32_t r = find_req(T.pair_base, nreq, x);
        const ReqDev &q = T.reqs[r];
        const uint32_t qq = x - T.pair_base[r];
        const uint32_t *const pblk = q.pair_blk;
        const ReqState *const st = q.st;
        const uint32_t *const act = q.act[0], *const act1 = q.act[1];
        const uint32_t rank = W.pair_rank[x];
        const VolState V = vol_state(vols[q.vol]);
        const uint32_t nsp = st->last_nspec, cur = st->cur, used = st->slot_cursor;
        const bool per_ray = q.policy == SPEC_PER_RAY;
        const uint32_t *const pray = q.pair_ray;
        if (qq >= used) continue;   // not handed out this pass (per-ray counts)
        const uint32_t b = pblk[qq];
        if (b == NONE) continue;
        const uint32_t vi = V.vis_idx[bidx(V, b)];
        const uint32_t ii = per_ray ? pray[qq] : qq / nsp;
        const uint32_t pix = (cur ? act1 : act)[ii];
        if (vi >= vadm) {
            // a pair on a block not served this pass (cache-capacity rule):
            // the ray keeps its progress up to its first such slot (k_finish
            // reads the minimum after the kernel boundary)
            atomicMin(q.def_first + pix, qq - q.rbase[pix]);
            atomicAdd(&T.wave_rec[(T.act_base[r] + ii) >> 6].z, 1u);
            continue;
        }
        const uint32_t dst = W.vis_off[vi] + rank;
        W.s_ray[dst] = (r << 24) | pix;
        W.s_q[dst] = qq;
        W.s_vi[dst] = vi;
    }
}

// ---------------------------------------------------------------- K6 ------
// Decode the misses into their slots (Sec. 3.5), one thread per block.
__global__ __launch_bounds__(64) void k_decode(PassCtl *ctl, const VolDev *vols, Work W, Cache C) {
    __shared__ DecodeLds<32> L;
    fill_dep4(L, threadIdx.x);
    __syncthreads();
    const uint32_t m = ctl->assigned;
    // The first nd workgroups decode the misses (one block per lane), the
    // others list the neighbourhoods, so that a lane's decode and its share
    // of the lists do not add up on one critical path (at most half of the
    // grid, rounded up, decodes; a longer miss list takes several blocks per
    // lane; a one-workgroup grid does both).
    const uint32_t half = (gridDim.x + 1u) / 2u;
    const uint32_t nd = (m + 63u) / 64u < half ? (m + 63u) / 64u : half;
    if (blockIdx.x < nd) {
        for (uint32_t i = blockIdx.x * 64 + threadIdx.x; i < m; i += nd * 64) {
            uint64_t e = W.miss_list[i];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            const uint32_t *rec = V.stream + (uint64_t)(uint32_t)e * (uint64_t)V.rec_words;
            decode_to<32>(rec, V.rate, L, threadIdx.x, C.slots + (size_t)W.miss_slot[i] * 64);
        }
    }
    // Per admitted visible block, the slots of its 2x2x2 neighbourhood (every
    // neighbour is active, so it holds a slot by now): the raytrace reads them
    // with the visible-list entry instead of eight map lookups after it.
    const uint32_t vadm = admitted_blocks(ctl);
    const uint32_t l0 = nd < gridDim.x ? nd : 0u;   // the list workgroups: l0 .. gridDim - 1
    const uint32_t nl = gridDim.x - l0;
    for (uint32_t v = (blockIdx.x - l0) * 64 + threadIdx.x; blockIdx.x >= l0 && v < vadm; v += nl * 64) {
        const uint64_t e = W.vis_list[v];
        const VolState V = vol_state(vols[(uint32_t)(e >> 32)]);
        const uint32_t b = (uint32_t)e;
        const uint32_t rr = b / (uint32_t)V.nb0;
        const int bx = (int)(b - rr * (uint32_t)V.nb0), by = (int)(rr % (uint32_t)V.nb1), bz = (int)(rr / (uint32_t)V.nb1);
        // eight independent reads (a neighbour outside the volume reads the
        // block's own entry and is masked), issued together
        const gptr<const uint32_t> map = as_global((const uint32_t *)V.map);
        uint32_t nsl[8];
        uint32_t inside = 0, nbi[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int x2 = bx + (o & 1), y2 = by + ((o >> 1) & 1), z2 = bz + (o >> 2);
            const bool ok = x2 < V.nb0 && y2 < V.nb1 && z2 < V.nb2;
            nbi[o] = bidx_xyz(V, ok ? x2 : bx, ok ? y2 : by, ok ? z2 : bz);
            inside |= ok ? 1u << o : 0u;
        }
#pragma unroll
        for (int o = 0; o < 8; ++o) nsl[o] = map[nbi[o]];
#pragma unroll
        for (int o = 0; o < 8; ++o) nsl[o] = ((inside >> o) & 1u) ? nsl[o] : NONE;
        // the marking's claims are done: clear the claim words this block's
        // neighbourhood set (every claimed block is in the neighbourhood of an
        // admitted visible block), so they are 0 for the next pass
        const gptr<uint64_t> claim = as_global(V.claim);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            bool first = true;
#pragma unroll
            for (int o2 = 0; o2 < o; ++o2) first = first && (nbi[o2] >> 6) != (nbi[o] >> 6);
            if (first) claim[nbi[o] >> 6] = 0ull;
        }
        uint4 *dst = reinterpret_cast<uint4 *>(W.vis_nsl + (size_t)v * 8);
        dst[0] = make_uint4(nsl[0], nsl[1], nsl[2], nsl[3]);
        dst[1] = make_uint4(nsl[4], nsl[5], nsl[6], nsl[7]);
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->free_top -= m;   // the assigned slots leave the free stack
}

// ------------------------------------------------------- finishing a ray --
// Depth composite and termination of one ray (Sec. 4.4), after the raytrace
// of its pass.  The ray's slots rbase .. rbase + nfound - 1 hold its
// candidate blocks in traversal order.  best holds the minimum hit key of the
// ray's raytraced pairs, and def_first the first slot whose block was not
// served this pass (NONE if all were).
//   - a hit in a slot before def_first is the closest hit: image, hit buffer,
//     the ray terminates;
//   - otherwise, with a deferred slot, the ray keeps its progress up to the
//     slot before it and survives;
//   - otherwise (every candidate served, no hit) the ray terminates if the
//     walk found fewer than N_spec blocks (it left the volume), and else
//     resumes after its last candidate.
// The ray's per-pixel pass state is reset for the next pass.  *w is the
// survivor's weight for the next pass (per-ray counts).
__device__ __forceinline__ bool finish_ray(const ReqDev &q, const VolDev *vols, uint32_t pix, uint32_t nf,
                                           uint32_t &w) {
    const uint32_t base = q.rbase[pix], ns = q.rns[pix];
    const uint64_t best = q.best[pix];
    const uint32_t d = q.def_first[pix];
    const uint32_t kb = best != ~0ull ? (uint32_t)(best >> 38) - base : NONE;
    bool term = false;
    uint32_t next = NONE;   // the block the ray resumes after, if it moved
    if (kb != NONE && kb < d) {
        q.image[pix] = (uint32_t)best;
        spr_hit h;
        h.t = q.tslot[base + kb];
        h.block_id = q.pair_blk[base + kb];
        h.cell = (uint32_t)(best >> 32) & 63u;
        q.hits[pix] = h;
        term = true;
    } else if (d != NONE) {
        if (d > 0u) next = q.pair_blk[base + d - 1u];
    } else if (nf < ns) {
        term = true;
    } else {
        next = q.pair_blk[base + nf - 1u];
    }
    w = 0;
    if (term) {
        q.ray_state[pix] = RAY_DONE;
    } else {
        if (next != NONE) q.ray_state[pix] = next;
        if (q.policy == SPEC_PER_RAY) {
            // the survivor's weight for the next pass: from where it leaves
            // the block it resumes after (the traversal's restart point)
            w = q.rw[pix];
            if (next != NONE) {
                const VolDev &V = vols[q.vol];
                Ray R;
                make_ray(q, V.n, pix, R);
                const Level LB = {4, {V.tb[0], V.tb[1], V.tb[2]}, {V.n[0], V.n[1], V.n[2]}, 0.25};
                const int cb[3] = {(int)(next % (uint32_t)V.nb[0]), (int)((next / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]),
                                   (int)(next / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]))};
                AxisWalk wb;
                walk_init(R, LB, cb, wb);
                w = ray_weight(walk_exit(wb), R.tx);
            }
        }
    }
    if (best != ~0ull) q.best[pix] = ~0ull;
    if (d != NONE) q.def_first[pix] = NONE;
    return term;
}

// K10: every active ray with candidates this pass is finished (finish_ray);
// the rays the traversal found no candidate for were terminated by it.  One
// thread per entry of the active-ray space, whose waves are the wave records'
// waves (64-aligned per request): a wave adds its terminations and its
// survivors' weights to its own record (no other kernel writes them now).
__global__ __launch_bounds__(256) void k_finish(PassCtl *ctl, Table T, const VolDev *vols) {
    const uint32_t A = ctl->A;
    const uint32_t nreq = ctl->nreq;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        const uint32_t r = uni(find_req(T.act_base, nreq, p));
        const ReqDev &q = T.reqs[r];
        const ReqState *st = uni(q.st);
        const uint32_t i = p - uni(T.act_base[r]);
        bool term = false;
        uint32_t w = 0;
        if (i < uni(st->n_act_prev)) {
            const uint32_t pix = uni(q.act[uni(st->cur)])[i];
            const uint32_t nf = q.nfound[pix];
            if (nf > 0u) term = finish_ray(q, vols, pix, nf, w);
        }
        const uint32_t nt = (uint32_t)__popcll(__ballot(term));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) w += (uint32_t)__shfl_xor((int)w, off);
        if (lane_id() == 0) {
            if (nt) T.wave_rec[p >> 6].w += nt;
            if (w) T.wave_w[p >> 6] += w;
        }
    }
}

// A served pair's result: with a hit, the atomic minimum of its key into the
// pixel's best word.  A ray's pair slots are consecutive and follow its
// traversal, so the pair slot orders the ray's hits as t does (ties go to the
// earlier block): the ray's first hit in slot order is the minimum of
// slot << 38 | cell << 32 | rgba over its hits (slots < 2^24).  t goes to the
// pair's slot, where the minimum's slot finds it (the second step of the
// resolve, in k_finish after the kernel boundary).
__device__ __forceinline__ void pair_done(const ReqDev &q, uint32_t pix, uint32_t qq, uint32_t cell, uint32_t rgba,
                                          double t) {
    if (cell == NONE) return;
    const uint64_t key = ((uint64_t)qq << 38) | ((uint64_t)cell << 32) | rgba;
    q.tslot[qq] = t;
    __hip_atomic_fetch_min(as_global(q.best) + pix, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- K9 ------
// Block raytrace (Sec. 3.7, 4.3): each served pair walks its ray through the
// dual cells of its block (Amanatides-Woo restricted to the block) and tests
// each cell (corner pretest, cubic, Marmitt isolation).  A pair whose ray hits
// takes the atomic minimum of its key (slot, cell, colour) into the pixel's
// best word and writes its t at its pair slot; a pair without a hit writes
// nothing.
__device__ __forceinline__ float slot_value(const float *slots, const uint32_t ns[8], int lx, int ly, int lz) {
    int nb = (lx >> 2) | ((ly >> 2) << 1) | ((lz >> 2) << 2);
    uint32_t s = ns[nb];
    if (s == NONE) return 0.0f;   // unreachable: every neighbour of a served block holds a slot
    return slots[(size_t)s * 64 + ((lx & 3) + 4 * (ly & 3) + 16 * (lz & 3))];
}

// A tile of RT_TILE sorted pairs (one workgroup; 128 or 256) covers runs of
// a few blocks.  The workgroup stages the 5^3 dual grid of each distinct
// block of the tile (up to RT_LB blocks: 16 or 32) into LDS once - the
// block's 4^3 samples plus the +x/+y/+z face, edge and corner samples of its
// neighbours (Sec. 3.7) - and every pair then reads its cell corners from
// LDS.  Pairs of blocks beyond RT_LB in a tile read the slots directly.  Both
// sizes are launch tuning: results do not depend on them.
template <int RT_TILE, int RT_LB>
__global__ __launch_bounds__(RT_TILE, 3) void k_raytrace(PassCtl *ctl, Table T, const VolDev *vols, Work W,
                                                                     Cache C) {
    __shared__ float s_grid[RT_LB][128];
    __shared__ uint32_t s_nsl[RT_LB][8];
    __shared__ int s_bb[RT_LB][4];
    __shared__ uint32_t s_scan[RT_TILE / 64];
    __shared__ uint32_t s_nloc;
    const uint32_t n = ctl->served;
    const uint32_t tid = threadIdx.x;
    for (uint32_t base = blockIdx.x * RT_TILE; base < n; base += gridDim.x * RT_TILE) {
        const uint32_t j = base + tid;
        const bool valid = j < n;
        const uint32_t vi = valid ? W.s_vi[j] : NONE;
        const uint32_t prev = (valid && tid > 0) ? W.s_vi[j - 1] : NONE;
        const bool start = valid && (tid == 0 || vi != prev);
        // workgroup exclusive scan of run starts -> local block index
        uint64_t m = __ballot(start);
        uint32_t wrank = (uint32_t)__popcll(m & lanemask_lt());
        if (lane_id() == 0) s_scan[tid >> 6] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t woff = 0, tot = 0;
        for (uint32_t w = 0; w < RT_TILE / 64; ++w) {
            uint32_t c = s_scan[w];
            if (w < (tid >> 6)) woff += c;
            tot += c;
        }
        // lb of this pair = (number of run starts at or before it) - 1
        uint32_t lb = woff + wrank + (start ? 1u : 0u) - 1u;
        {
            // pairs that are not starts: lb = starts before them - 1 (same as above minus nothing)
            uint32_t before = woff + wrank;   // starts strictly before this lane
            lb = start ? before : before - 1u;
        }
        const uint32_t nloc = tot < (uint32_t)RT_LB ? tot : (uint32_t)RT_LB;
        if (start && lb < (uint32_t)RT_LB) {
            const uint64_t e = W.vis_list[vi];
            const uint4 n0 = reinterpret_cast<const uint4 *>(W.vis_nsl + (size_t)vi * 8)[0];
            const uint4 n1 = reinterpret_cast<const uint4 *>(W.vis_nsl + (size_t)vi * 8)[1];
            const VolDev &V = vols[(uint32_t)(e >> 32)];
            uint32_t b = (uint32_t)e;
            s_bb[lb][0] = (int)(b % (uint32_t)V.nb[0]);
            s_bb[lb][1] = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
            s_bb[lb][2] = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
            s_bb[lb][3] = (int)(uint32_t)(e >> 32);
            s_nsl[lb][0] = n0.x; s_nsl[lb][1] = n0.y; s_nsl[lb][2] = n0.z; s_nsl[lb][3] = n0.w;
            s_nsl[lb][4] = n1.x; s_nsl[lb][5] = n1.y; s_nsl[lb][6] = n1.z; s_nsl[lb][7] = n1.w;
        }
        __syncthreads();
        // stage the 5^3 dual grids, four loads in flight per thread before
        // their LDS stores
        for (uint32_t x0 = tid; x0 < nloc * 125; x0 += 4 * RT_TILE) {
            float sv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t x = x0 + (uint32_t)u * RT_TILE;
                sv[u] = 0.0f;
                if (x < nloc * 125) {
                    const uint32_t l = x / 125, k = x - l * 125;
                    const int lx = (int)(k % 5), ly = (int)((k / 5) % 5), lz = (int)(k / 25);
                    const int o = (lx >> 2) | ((ly >> 2) << 1) | ((lz >> 2) << 2);
                    const uint32_t sl = s_nsl[l][o];
                    if (sl != NONE) sv[u] = C.slots[(size_t)sl * 64 + ((lx & 3) + 4 * (ly & 3) + 16 * (lz & 3))];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t x = x0 + (uint32_t)u * RT_TILE;
                if (x < nloc * 125) s_grid[x / 125][x % 125] = sv[u];
            }
        }
        __syncthreads();
        if (valid) {
            const uint32_t ray = W.s_ray[j];
            const uint32_t r = ray >> 24, pix = ray & 0xFFFFFFu;
            const uint32_t qq = W.s_q[j];
            const ReqDev &q = T.reqs[r];
            const VolDev &V = vols[q.vol];
            int bb[3];
            uint32_t nsl[8];
            const bool staged = lb < (uint32_t)RT_LB;
            if (staged) {
                bb[0] = s_bb[lb][0]; bb[1] = s_bb[lb][1]; bb[2] = s_bb[lb][2];
            } else {
                uint32_t b = (uint32_t)W.vis_list[vi];
                bb[0] = (int)(b % (uint32_t)V.nb[0]);
                bb[1] = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
                bb[2] = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
#pragma unroll
                for (int o = 0; o < 8; ++o) nsl[o] = W.vis_nsl[(size_t)vi * 8 + o];
            }
            Ray R;
            make_ray(q, V.n, pix, R);
            Level LB = {4, {V.tb[0], V.tb[1], V.tb[2]}, {V.n[0], V.n[1], V.n[2]}, 0.25};
            Level L1 = {1, {V.n[0] - 1, V.n[1] - 1, V.n[2] - 1}, {V.n[0], V.n[1], V.n[2]}, 1.0};
            int lo[3], hi[3], c[3];
            double tb0 = cell_entry(R, LB, bb);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = 4 * bb[a];
                hi[a] = 4 * bb[a] + 3;
                if (hi[a] > V.n[a] - 2) hi[a] = V.n[a] - 2;
                c[a] = cell_at(R, L1, a, tb0, lo[a], hi[a]);
            }
            // entry parameter: cell_entry for the first cell; afterwards the
            // previous cell's exit (the stepped axes' entry planes are the old
            // exit planes, every other entry plane lies before them)
            double t0 = cell_entry(R, L1, c);
            struct { double t; uint32_t cell, rgba; } out = {__builtin_inf(), NONE, 0u};
            int guard = 0;
            float fc[8];
            CellHit h;
            for (; guard < 16; ++guard) {   // at most 10 cells of a 4^3 block lie on a ray
                const double tx = cell_exit(R, L1, c);
                const double t1 = tx < R.tx ? tx : R.tx;
                int lx = c[0] - lo[0], ly = c[1] - lo[1], lz = c[2] - lo[2];
                if (staged) {
                    const float *g = s_grid[lb];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        fc[k] = g[(lx + (k & 1)) + 5 * (ly + ((k >> 1) & 1)) + 25 * (lz + (k >> 2))];
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        fc[k] = slot_value(C.slots, nsl, lx + (k & 1), ly + ((k >> 1) & 1), lz + (k >> 2));
                }
                test_cell(R, c, t0, t1, fc, q.iso, h);
                if (h.hit) {
                    out.cell = (uint32_t)(lx + 4 * ly + 16 * lz);
                    break;
                }
                if (tx > R.tx || !advance(R, L1, c, tx, lo, hi)) break;
                t0 = tx;
            }
            if (guard == 16) atomicAdd(&ctl->guard, 1u);
            // root and colour of the hit after the loop, where the wave's hit
            // lanes run them together (t0 and fc are still the hit cell's)
            if (out.cell != NONE) {
                refine_hit(h);
                out.t = t0 + h.s;
                out.rgba = shade_hit(R, h, fc);
            }
            pair_done(q, pix, qq, out.cell, out.rgba, out.t);
        }
        __syncthreads();   // the next tile reuses the LDS
    }
}

// The 8 corner values of dual cell (lx, ly, lz) of a block (local cell
// coordinates 0..3) straight from the cache slots of its 2x2x2 block
// neighbourhood: corner offset o (bit 0 x, 1 y, 2 z) lies in neighbour
// o & h, h the axes on which the cell is the block's last (its + corners are
// the neighbour's first samples).  All eight loads are issued together.
__device__ __forceinline__ void load_corners(const float *__restrict__ slots, const uint32_t nsl[8], int lx, int ly,
                                             int lz, float fc[8]) {
    const uint32_t h = (lx == 3 ? 1u : 0u) | (ly == 3 ? 2u : 0u) | (lz == 3 ? 4u : 0u);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t o = (uint32_t)k & h;
        uint32_t s = nsl[0];
        // nsl[o] with o a subset of k's bits: a short select chain per corner
#pragma unroll
        for (int m = 1; m < 8; ++m)
            if ((m & ~k) == 0) s = o == (uint32_t)m ? nsl[m] : s;
        const int x = (lx + (k & 1)) & 3, y = (ly + ((k >> 1) & 1)) & 3, z = (lz + (k >> 2)) & 3;
        fc[k] = s != NONE ? slots[(size_t)s * 64 + (uint32_t)(x + 4 * y + 16 * z)] : 0.0f;
    }
}

// Block raytrace without LDS staging: one served pair per lane.  When a
// block carries one or two pairs (the common case once speculation spreads
// the rays' slots over many blocks), staging its 125-value dual grid costs
// more loads than the pair's own corner reads (eight per cell, issued
// together; adjacent cells share a face, so the second read mostly hits the
// cache).  Same walk, cell test, shading and composite as the staged kernel.
// The camera and volume fields are read per lane: in a batch, the pairs of
// one block come from every request that sees it.
__global__ __launch_bounds__(256, 3) void k_raytrace_direct(PassCtl *ctl, Table T, const VolDev *vols, Work W,
                                                             Cache C) {
    const uint32_t n = ctl->served;
    const float *__restrict__ slots = C.slots;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const uint32_t vi = W.s_vi[j];
        const uint32_t ray = W.s_ray[j];
        const uint32_t qq = W.s_q[j];
        const uint32_t r = ray >> 24, pix = ray & 0xFFFFFFu;
        const uint4 n0 = reinterpret_cast<const uint4 *>(W.vis_nsl + (size_t)vi * 8)[0];
        const uint4 n1 = reinterpret_cast<const uint4 *>(W.vis_nsl + (size_t)vi * 8)[1];
        const uint32_t nsl[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
        const uint32_t b = (uint32_t)W.vis_list[vi];
        const ReqDev &q = T.reqs[r];
        const VolDev &V = vols[q.vol];
        const float iso = q.iso;
        int bb[3];
        bb[0] = (int)(b % (uint32_t)V.nb[0]);
        bb[1] = (int)((b / (uint32_t)V.nb[0]) % (uint32_t)V.nb[1]);
        bb[2] = (int)(b / ((uint32_t)V.nb[0] * (uint32_t)V.nb[1]));
        Ray R;
        make_ray(q, V.n, pix, R);
        const Level LB = {4, {V.tb[0], V.tb[1], V.tb[2]}, {V.n[0], V.n[1], V.n[2]}, 0.25};
        const Level L1 = {1, {V.n[0] - 1, V.n[1] - 1, V.n[2] - 1}, {V.n[0], V.n[1], V.n[2]}, 1.0};
        int lo[3], hi[3], c[3];
        const double tb0 = cell_entry(R, LB, bb);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = 4 * bb[a];
            hi[a] = 4 * bb[a] + 3;
            if (hi[a] > V.n[a] - 2) hi[a] = V.n[a] - 2;
            c[a] = cell_at(R, L1, a, tb0, lo[a], hi[a]);
        }
        // entry parameter: cell_entry for the first cell; afterwards the
        // previous cell's exit (the stepped axes' entry planes are the old
        // exit planes, every other entry plane lies before them)
        double t0 = cell_entry(R, L1, c);
        float fc[8];
        load_corners(slots, nsl, c[0] - lo[0], c[1] - lo[1], c[2] - lo[2], fc);
        double out_t = __builtin_inf();
        uint32_t out_cell = NONE, out_rgba = 0u;
        int guard = 0;
        CellHit h;
        for (; guard < 16; ++guard) {   // at most 10 cells of a 4^3 block lie on a ray
            const double tx = cell_exit(R, L1, c);
            const double t1 = tx < R.tx ? tx : R.tx;
            test_cell(R, c, t0, t1, fc, iso, h);
            if (h.hit) {
                out_cell = (uint32_t)((c[0] - lo[0]) + 4 * (c[1] - lo[1]) + 16 * (c[2] - lo[2]));
                break;
            }
            if (tx > R.tx || !advance(R, L1, c, tx, lo, hi)) break;
            load_corners(slots, nsl, c[0] - lo[0], c[1] - lo[1], c[2] - lo[2], fc);
            t0 = tx;
        }
        if (guard == 16) atomicAdd(&ctl->guard, 1u);
        // root and colour of the hit after the loop, where the wave's hit lanes
        // run them together (t0 and fc are still the hit cell's)
        if (out_cell != NONE) {
            refine_hit(h);
            out_t = t0 + h.s;
            out_rgba = shade_hit(R, h, fc);
        }
        pair_done(q, pix, qq, out_cell, out_rgba, out_t);
    }
}

// --------------------------------------------------------------- K11 ------
// Count the surviving rays (Sec. 3 step (f)): exclusive scan of the per-wave
// survivor counts, per-request N_act, N_spec = clamp(floor(w*h / N_act), 1,
// cap) (Sec. 4), the per-request pass counters, and the flip to the other
// active-ray list.  A wave's survivors are its active rays less the ones that
// terminated this pass (counted into its record by the traversal and by the
// pairs that finished rays); on the initial-ray pass the record holds the
// rays that entered the volume.  One workgroup; each thread owns a
// contiguous run of waves, sums it (splitting at request boundaries into LDS
// per-request sums), the workgroup scans the run totals, and each thread
// writes its run's offsets.
constexpr int PE_THREADS = 1024;

__global__ __launch_bounds__(PE_THREADS) void k_pass_end(PassCtl *ctl, Table T, int is_init) {
    __shared__ uint32_t s_req[4][MAX_REQS];   // survivors, pairs, deferred, terminated
    __shared__ unsigned long long s_wsum[MAX_REQS];   // survivors' weights (per-ray counts)
    __shared__ uint32_t s_wave[PE_THREADS / 64];
    const uint32_t nw = ctl->A >> 6;
    const uint32_t nreq = ctl->nreq;
    const uint32_t t = threadIdx.x;
    for (uint32_t r = t; r < nreq; r += PE_THREADS) {
        s_req[0][r] = 0; s_req[1][r] = 0; s_req[2][r] = 0; s_req[3][r] = 0;
        s_wsum[r] = 0;
    }
    __syncthreads();
    const uint32_t per = (nw + PE_THREADS - 1) / PE_THREADS;
    const uint32_t w0 = t * per < nw ? t * per : nw;
    const uint32_t w1 = w0 + per < nw ? w0 + per : nw;
    uint32_t run = 0;
    // up to PE_REG records per thread are read in two halves of PE_REG / 2,
    // each half's loads issued together, and their survivor counts kept in
    // registers for the offsets (unrolled, so the indices are compile-time;
    // 16 covers a 720p request's 14,400 waves)
    constexpr uint32_t PE_REG = 16, PE_HALF = PE_REG / 2;
    const bool in_regs = per <= PE_REG;
    uint32_t surv[PE_REG] = {};
    if (w0 < w1) {
        uint32_t r = find_req(T.act_base, nreq, w0 << 6);
        uint32_t next = (r + 1 < nreq) ? (T.act_base[r + 1] >> 6) : 0xFFFFFFFFu;
        uint32_t rbase = T.act_base[r], rna = as_global(T.reqs[r].st)->n_act_prev;
        uint4 acc = make_uint4(0u, 0u, 0u, 0u);
        unsigned long long accw = 0ull;   // the survivors' weights (per-ray counts)
        // survivors of wave w: the initial pass records them; a pass records
        // its terminations, and the wave's active rays are the request's
        // n_act_prev rays from its 64-aligned start
        auto survivors = [&](uint32_t w, const uint4 v) -> uint32_t {
            if (is_init) return v.x;
            const uint32_t lo = (w << 6) - rbase;
            const uint32_t act = lo >= rna ? 0u : (rna - lo < 64u ? rna - lo : 64u);
            return act - v.w;
        };
        auto add = [&](uint32_t w, const uint4 v, uint32_t ww) -> uint32_t {
            while (w >= next) {   // crossing into the next request's waves
                if (acc.x) atomicAdd(&s_req[0][r], acc.x);
                if (acc.y) atomicAdd(&s_req[1][r], acc.y);
                if (acc.z) atomicAdd(&s_req[2][r], acc.z);
                if (acc.w) atomicAdd(&s_req[3][r], acc.w);
                if (accw) atomicAdd(&s_wsum[r], accw);
                acc = make_uint4(0u, 0u, 0u, 0u);
                accw = 0ull;
                ++r;
                next = (r + 1 < nreq) ? (T.act_base[r + 1] >> 6) : 0xFFFFFFFFu;
                rbase = T.act_base[r];
                rna = as_global(T.reqs[r].st)->n_act_prev;
            }
            const uint32_t sv = survivors(w, v);
            acc.x += sv; acc.y += v.y; acc.z += v.z; acc.w += v.w;
            accw += ww;
            run += sv;
            return sv;
        };
        if (in_regs) {
#pragma unroll
            for (uint32_t h = 0; h < PE_REG; h += PE_HALF) {
                uint4 rv[PE_HALF];
                uint32_t wv[PE_HALF];
#pragma unroll
                for (uint32_t k = 0; k < PE_HALF; ++k) {
                    rv[k] = (w0 + h + k < w1) ? T.wave_rec[w0 + h + k] : make_uint4(0u, 0u, 0u, 0u);
                    wv[k] = (w0 + h + k < w1) ? T.wave_w[w0 + h + k] : 0u;
                }
#pragma unroll
                for (uint32_t k = 0; k < PE_HALF; ++k)
                    surv[h + k] = (w0 + h + k < w1) ? add(w0 + h + k, rv[k], wv[k]) : 0u;
            }
        } else {
            for (uint32_t w = w0; w < w1; ++w) (void)add(w, T.wave_rec[w], T.wave_w[w]);
        }
        if (acc.x) atomicAdd(&s_req[0][r], acc.x);
        if (acc.y) atomicAdd(&s_req[1][r], acc.y);
        if (acc.z) atomicAdd(&s_req[2][r], acc.z);
        if (acc.w) atomicAdd(&s_req[3][r], acc.w);
        if (accw) atomicAdd(&s_wsum[r], accw);
    }
    // workgroup exclusive scan of the run totals
    const uint32_t l = lane_id(), wv = t >> 6;
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off);
        if ((int)l >= off) incl += o;
    }
    if (l == 63) s_wave[wv] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < wv; ++k) before += s_wave[k];
    uint32_t off = before + incl - run;
    if (in_regs) {
#pragma unroll
        for (uint32_t k = 0; k < PE_REG; ++k) {
            if (w0 + k < w1) {
                T.wave_off[w0 + k] = off;
                off += surv[k];
            }
        }
    } else if (w0 < w1) {
        uint32_t r = find_req(T.act_base, nreq, w0 << 6);
        uint32_t next = (r + 1 < nreq) ? (T.act_base[r + 1] >> 6) : 0xFFFFFFFFu;
        for (uint32_t w = w0; w < w1; ++w) {
            while (w >= next) {
                ++r;
                next = (r + 1 < nreq) ? (T.act_base[r + 1] >> 6) : 0xFFFFFFFFu;
            }
            const uint4 v = T.wave_rec[w];
            uint32_t sv = v.x;
            if (!is_init) {
                const uint32_t lo = (w << 6) - T.act_base[r], rna = as_global(T.reqs[r].st)->n_act_prev;
                sv = (lo >= rna ? 0u : (rna - lo < 64u ? rna - lo : 64u)) - v.w;
            }
            T.wave_off[w] = off;
            off += sv;
        }
    }
    if (t == PE_THREADS - 1) T.wave_off[nw] = off;   // == total survivors
    __syncthreads();
    if (t == 0) {
        uint32_t pairs = 0, term = 0;
        for (uint32_t r = 0; r < nreq; ++r) {
            pairs += s_req[1][r];
            term += s_req[3][r];
        }
        ctl->pairs = pairs;
        ctl->terminated = term;
        if (!is_init && ctl->A > 0) {
            ctl->acc_passes += 1;
            ctl->acc_decoded += ctl->assigned;
            ctl->acc_visible += ctl->n_vis;
            ctl->acc_active += ctl->n_actblk;
            ctl->acc_pairs += pairs;
            ctl->acc_evicted += ctl->evicted;
            ctl->acc_overflow += ctl->overflow;
            ctl->acc_rays += ctl->rays;
            ctl->acc_slots += ctl->P;
            ctl->acc_served += ctl->served;
            if (ctl->n_actblk > ctl->acc_max_active) ctl->acc_max_active = ctl->n_actblk;
            ctl->acc_guard += ctl->guard;
            ctl->acc_csteps += ctl->csteps;
            ctl->acc_cmasks += ctl->cmasks;
        }
    }
    for (uint32_t r = t; r < nreq; r += PE_THREADS) {
        // every field read first, through a global-address pointer, then every
        // store: no wait between the stores and the loads after them
        const ReqDev &q = T.reqs[r];
        const gptr<ReqState> st = as_global(q.st);
        const uint32_t npix = q.npix, cap = q.spec_cap;
        const uint32_t prev = st->n_act_prev, cur = st->cur, cursor = st->slot_cursor;
        const unsigned long long tot = st->tot_pairs;
        const uint32_t na = s_req[0][r];
        uint32_t ns = 0;
        if (na > 0) {
            ns = npix / na;
            if (ns < 1) ns = 1;
            if (ns > cap) ns = cap;
        }
        st->cur = prev > 0 ? cur ^ 1u : cur;
        st->n_act = na;
        st->wsum = s_wsum[r];
        st->last_slots = is_init ? 0u : cursor;
        st->last_pairs = s_req[1][r];
        st->last_deferred = s_req[2][r];
        st->last_terminated = s_req[3][r];
        st->tot_pairs = tot + s_req[1][r];
        st->n_spec = ns;
        // a single render's host polls its active-ray count here
        if (r == 0 && T.host_nact) __hip_atomic_store(T.host_nact, na, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// --------------------------------------------------------------- K12 ------
// Ordered compaction of the surviving rays into the new active list.
__global__ __launch_bounds__(256) void k_compact(PassCtl *ctl, Table T) {
    const uint32_t A = ctl->A;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A; p += gridDim.x * blockDim.x) {
        // all lanes of a wave share a request (the A space is 64-aligned per request)
        uint32_t r = __builtin_amdgcn_readfirstlane(find_req(T.act_base, ctl->nreq, p));
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
        // the pass's wave records are consumed: clear them for the next pass
        // (whose active-ray space is no larger than this one's)
        if (lane_id() == 0) {
            T.wave_rec[p >> 6] = make_uint4(0u, 0u, 0u, 0u);
            T.wave_w[p >> 6] = 0u;
        }
    }
}

// Progress of the members of a launch table, for the host's scheduler: per
// request {active rays, passes run, pairs of the last pass, N_spec}, then
// {active blocks of the last pass, pass stamp, 0, 0}.  One workgroup.
// Set-up writes in stream order, from kernel arguments: a request's
// description, optionally its state and a launch table's request count.
__global__ void k_put_req(ReqDev *dq, ReqDev q, ReqState *ds, ReqState st, uint32_t *hdr, uint32_t hv) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    *dq = q;
    if (ds) *ds = st;
    if (hdr) *hdr = hv;
}

__global__ void k_gather_state(const PassCtl *ctl, Table T, uint32_t n, uint4 *out) {
    for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
        const ReqState *st = T.reqs[r].st;
        out[r] = make_uint4(st->n_act, st->passes, st->last_pairs, st->n_spec);
    }
    if (threadIdx.x == 0) out[n] = make_uint4(ctl->n_actblk, ctl->pass, 0u, 0u);
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
    hipLaunchKernelGGL(k_decode_ids, dim3(grid_for(n, 64, 8192)), dim3(64), 0, s, V, ids, n, out);
    return hipGetLastError();
}

hipError_t launch_fp64_ops(hipStream_t s, const double *x, const double *y, uint64_t n, double *sq, double *dv) {
    hipLaunchKernelGGL(k_fp64_ops, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, y, n, sq, dv);
    return hipGetLastError();
}

hipError_t launch_load_grids(hipStream_t s, const VolDev &V, hipEvent_t *ev) {
    int k = 0;
    auto mark = [&]() {
        if (ev) (void)hipEventRecord(ev[k], s);
        ++k;
    };
    dim3 g(grid_for(V.nblocks, 64, 1u << 16)), b(64);
    mark();   // block ranges go straight into the fine array, which the axis passes then widen in place
    if (V.rec_words <= 4) hipLaunchKernelGGL(k_block_ranges<4>, g, b, 0, s, V, V.fine);
    else if (V.rec_words <= 8) hipLaunchKernelGGL(k_block_ranges<8>, g, b, 0, s, V, V.fine);
    else if (V.rec_words <= 16) hipLaunchKernelGGL(k_block_ranges<16>, g, b, 0, s, V, V.fine);
    else hipLaunchKernelGGL(k_block_ranges<32>, g, b, 0, s, V, V.fine);
    mark();
    for (int a = 0; a < 3; ++a) {
        const uint64_t len = a == 0 ? (uint64_t)V.nb[0] : (a == 1 ? (uint64_t)V.nb[1] : (uint64_t)V.nb[2]);
        hipLaunchKernelGGL(k_fine_axis, dim3(grid_for(V.nblocks / len, 256, 1u << 16)), dim3(256), 0, s, V, a);
    }
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    mark(); hipLaunchKernelGGL(k_coarse_grid, dim3(grid_for(nc, 256, 1u << 16)), dim3(256), 0, s, V);
    mark();
    return hipGetLastError();
}

hipError_t launch_put_req(hipStream_t s, ReqDev *dq, const ReqDev &q, ReqState *ds, const ReqState *st,
                          uint32_t *hdr, uint32_t hv) {
    const ReqState zero{};
    hipLaunchKernelGGL(k_put_req, dim3(1), dim3(64), 0, s, dq, q, ds, st ? *st : zero, hdr, hv);
    return hipGetLastError();
}

hipError_t launch_gather_state(hipStream_t s, const PassCtl *ctl, const Table &T, uint32_t n, uint4 *out) {
    hipLaunchKernelGGL(k_gather_state, dim3(1), dim3(256), 0, s, ctl, T, n, out);
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

hipError_t launch_init_rays(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols, uint64_t mask_words,
                            bool build_masks, hipEvent_t *ev) {
    int k = 0;
    auto mark = [&]() {
        if (ev) (void)hipEventRecord(ev[k], s);
        ++k;
    };
    if (build_masks) {
        mark();   // masks, then the empty-space distances (timed together)
        hipLaunchKernelGGL(k_iso_masks, dim3(grid_for(mask_words, 256, 4096)), dim3(256), 0, s, T, vols);
        hipLaunchKernelGGL(k_cdist_pass<0>, dim3(grid_for(mask_words, CD_TA * CD_TL, 4096)), dim3(256), 0, s, T, vols);
        hipLaunchKernelGGL(k_cdist_pass<1>, dim3(grid_for(mask_words, CD_TA * CD_TL, 4096)), dim3(256), 0, s, T, vols);
        hipLaunchKernelGGL(k_cdist_pass<2>, dim3(grid_for(mask_words, CD_TA * CD_TL, 4096)), dim3(256), 0, s, T, vols);
    }
    mark(); hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, s, ctl, T, 1);
    mark(); hipLaunchKernelGGL(k_init_rays, dim3(grid_for(T.max_A, 256, 16384)), dim3(256), 0, s, ctl, T, vols);
    mark(); hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(1024), 0, s, ctl, T, 1);
    mark(); hipLaunchKernelGGL(k_compact, dim3(grid_for(T.max_A, 256, 16384)), dim3(256), 0, s, ctl, T);
    mark();
    return hipGetLastError();
}

const char *const PASS_KERNEL_NAMES[PASS_KERNELS] = {
    "k_pass_begin", "k_traverse", "k_dedupe", "k_mark", "k_evict_hist", "k_evict",
    "k_assign_scatter", "k_decode", "k_raytrace", "k_finish", "k_pass_end", "k_compact"};

const char *const PROF_NAMES[PROF_SLOTS] = {
    "k_pass_begin", "k_traverse", "k_dedupe", "k_mark", "k_evict_hist", "k_evict",
    "k_assign_scatter", "k_decode", "k_raytrace", "k_finish", "k_pass_end", "k_compact",
    "k_block_ranges", "k_fine_grid", "k_coarse_grid", "k_iso_masks", "k_init_rays"};

hipError_t launch_pass(hipStream_t s, PassCtl *ctl, const Table &T, const VolDev *vols, const Work &W,
                       const Cache &C, const PassGrids &g, hipEvent_t *ev) {
    int k = 0;
    auto mark = [&]() {
        if (ev) (void)hipEventRecord(ev[k], s);
        ++k;
    };
    mark(); hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, s, ctl, T, 0);
    mark(); hipLaunchKernelGGL(k_traverse, dim3(g.rays), dim3(256), 0, s, ctl, T, vols, W);
    mark(); hipLaunchKernelGGL(k_dedupe, dim3(g.dedupe), dim3(256), 0, s, ctl, T, vols, W);
    mark(); hipLaunchKernelGGL(k_mark, dim3(g.pairs), dim3(256), 0, s, ctl, vols, W, C);
    mark(); hipLaunchKernelGGL(k_evict_hist, dim3(g.slots), dim3(256), 0, s, ctl, C);
    mark(); hipLaunchKernelGGL(k_evict, dim3(g.slots), dim3(256), 0, s, ctl, vols, C);
    mark(); hipLaunchKernelGGL(k_assign_scatter, dim3(g.assign + g.scatter), dim3(256), 0, s, ctl, T, vols, W, C, g.assign);
    mark(); hipLaunchKernelGGL(k_decode, dim3(g.decode), dim3(64), 0, s, ctl, vols, W, C);
    mark();
    if (g.rt_lb == 0) hipLaunchKernelGGL(k_raytrace_direct, dim3(g.rt), dim3(256), 0, s, ctl, T, vols, W, C);
    else if (g.rt_tile == 128 && g.rt_lb == 16) hipLaunchKernelGGL((k_raytrace<128, 16>), dim3(g.rt), dim3(128), 0, s, ctl, T, vols, W, C);
    else if (g.rt_tile == 128) hipLaunchKernelGGL((k_raytrace<128, 32>), dim3(g.rt), dim3(128), 0, s, ctl, T, vols, W, C);
    else if (g.rt_lb == 16) hipLaunchKernelGGL((k_raytrace<256, 16>), dim3(g.rt), dim3(256), 0, s, ctl, T, vols, W, C);
    else hipLaunchKernelGGL((k_raytrace<256, 32>), dim3(g.rt), dim3(256), 0, s, ctl, T, vols, W, C);
    mark(); hipLaunchKernelGGL(k_finish, dim3(g.rays), dim3(256), 0, s, ctl, T, vols);
    mark(); hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(1024), 0, s, ctl, T, 0);
    mark(); hipLaunchKernelGGL(k_compact, dim3(g.rays), dim3(256), 0, s, ctl, T);
    if (ev) (void)hipEventRecord(ev[k], s);
    return hipGetLastError();
}

}  // namespace spr
