// spr_engine.hip — host engine and C ABI of libspr (see include/spr.h).
//
// Owns the handles, device memory, the shared decoded-block cache, the pass
// workspace and the launch tables; sequences the load path, the initial-ray
// pass and the per-pass kernels on the context's stream; captures the pass
// of a batch into a HIP graph and replays it.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "spr_launch.h"

using namespace spr;

namespace {

thread_local std::string g_err;

spr_status fail(spr_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
spr_status fail(spr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(SPR_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                        \
    do {                                 \
        spr_status s_ = (expr);          \
        if (s_ != SPR_OK) return s_;     \
    } while (0)

uint32_t round64h(uint64_t x) { return (uint32_t)((x + 63u) & ~63ull); }


// What a device allocation holds (spr_mem_split reports bytes per kind).
enum MemCat {
    MEM_COMPRESSED = 0,   // compressed streams
    MEM_GRIDS,            // macrocell grids and per-block state
    MEM_RAYS,             // per-render buffers: rays, pair slots, image, hits, masks
    MEM_CACHE,            // decoded-block cache
    MEM_SCRATCH,          // pass workspace, control block, batch tables, debug staging
    MEM_NCAT
};

}  // namespace

// Staging of the allocation-free decode (spr_debug_decode_blocks_noalloc):
// the block ids at offset 0, the decoded values at NOALLOC_OUT_OFF.  Each GPU
// holds its own copy for the life of the process.  In host code `scratch`
// names a host-side stand-in, not the device copy: kernels and copies take
// the address hipGetSymbolAddress returns for the current device
// (scratch_ptr below), never the array's name.
namespace {
constexpr size_t NOALLOC_OUT_OFF = ((size_t)SPR_NOALLOC_MAX_BLOCKS * sizeof(uint32_t) + 255) & ~(size_t)255;
constexpr size_t NOALLOC_BYTES = NOALLOC_OUT_OFF + (size_t)SPR_NOALLOC_MAX_BLOCKS * 64 * sizeof(float);
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller has made it current).
spr_status scratch_ptr(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(SPR_E_INVALID, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SPR_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return SPR_OK;
}
}  // namespace

struct spr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    spr_allocator alloc{};
    uint32_t spec_cap = 64;
    uint32_t rt_tile = 256, rt_lb = 0;    // raytrace launch tuning (spr_ctx_set_tuning)
    size_t mem_cur = 0, mem_peak = 0;
    size_t mem_cat[MEM_NCAT] = {}, mem_cat_peak[MEM_NCAT] = {}, mem_at_peak[MEM_NCAT] = {};
    PassCtl *ctl = nullptr;
    VolDev *d_vols = nullptr;
    VolDev h_vols[MAX_VOLUMES];
    spr_volume *vol_handles[MAX_VOLUMES] = {};
    Cache cache{};
    Work work{};
    uint64_t work_gen = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only to record graphs
    bool prof = false;
    // Profiling: a ring of event sets, read back only when a set is reused
    // or the totals are requested, so profiled passes need no host sync.
    static constexpr int PROF_RING = 64;
    struct ProfRec {
        hipEvent_t ev[PASS_KERNELS + 1] = {};
        const int *slots = nullptr;
        int nk = 0;
        bool pending = false;
    };
    ProfRec prof_ring[PROF_RING];
    uint32_t prof_head = 0;
    bool prof_events = false;
    double prof_ms[PROF_SLOTS] = {};
    uint64_t prof_n[PROF_SLOTS] = {};
    void *pinned = nullptr;     // small host staging area
    uint32_t *nact_host = nullptr;   // fine-grained host word: active rays after a render's last pass
    uint32_t *nact_dev = nullptr;    // its device address
    void *noalloc = nullptr;    // this device's copy of the allocation-free decode's staging
    int n_renders = 0;
};

// Isovalue masks and empty-space distances depend only on the volume's
// ranges and the isovalue, so a volume keeps the sets of its last few
// isovalues: a render whose isovalue matches a kept set (bitwise) reads that
// set instead of building its own.  A set that a live render reads is never
// rebuilt; when every set is in use, a render builds private masks.
struct MaskSet {
    uint32_t iso_bits = 0;
    bool keyed = false;          // holds (or, in stream order, will hold) the masks of iso_bits
    int users = 0;               // live renders reading it
    uint64_t last_use = 0;       // replacement order among the sets nobody reads
    void *buf = nullptr;         // counts, masks and distances, carved from one allocation
    size_t bytes = 0;
    unsigned long long *mstat = nullptr;
    uint64_t *cmask64 = nullptr;
    uint8_t *cdist = nullptr;
};
constexpr int MASK_SETS = 4;

struct spr_volume {
    spr_ctx *ctx = nullptr;
    uint32_t idx = 0;
    spr_volume_desc desc{};
    size_t stream_bytes = 0;
    int n_renders = 0;
    MaskSet msets[MASK_SETS];
    uint64_t mask_clock = 0;
};

struct spr_render {
    spr_ctx *ctx = nullptr;
    spr_volume *vol = nullptr;
    uint32_t w = 0, h = 0, npix = 0;
    ReqDev hreq{};
    ReqDev *d_req = nullptr;
    ReqState *d_st = nullptr;
    Table table{};
    PassGrids grids{};
    bool started = false;       // a pass has run
    spr_batch *batch = nullptr;
    // the request state as last read back, valid while no work that changes it
    // has been enqueued since (a pass, a batch membership)
    bool st_valid = false;
    ReqState st_cache{};
    float last_ms = 0.f;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_gen = ~0ull;
    uint64_t cwords = 0;   // isovalue mask size (one u64 per coarse cell)
    int mset = -1;         // the volume's mask set this render reads (-1: its own masks)
    bool masks_built = true;   // this render built its masks (else a kept set served them)
    void *buf = nullptr;   // every device buffer of the render, carved from one allocation
    size_t buf_bytes = 0;
};

struct spr_batch {
    spr_ctx *ctx = nullptr;
    std::vector<spr_render *> renders;
    Table table{};
    PassGrids grids{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_gen = ~0ull;
    uint64_t max_pixels = 0;
    uint4 *d_state = nullptr;   // cap + 1 gathered member records (k_gather_state)
    uint4 *h_state = nullptr;   // pinned copy
    bool state_fresh = false;   // h_state reflects the last pass and the current members
    void *buf = nullptr;        // table, member descriptions and gathered records, one allocation
    size_t buf_bytes = 0;
};

namespace {

// ------------------------------------------------------------- memory ------

spr_status dev_alloc(spr_ctx *c, MemCat cat, size_t bytes, void **out) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (c->alloc.alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
        if (!p) return fail(SPR_E_OOM, "allocator callback failed for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPR_E_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    c->mem_cur += bytes;
    c->mem_cat[cat] += bytes;
    if (c->mem_cat[cat] > c->mem_cat_peak[cat]) c->mem_cat_peak[cat] = c->mem_cat[cat];
    if (c->mem_cur > c->mem_peak) {
        c->mem_peak = c->mem_cur;
        for (int k = 0; k < MEM_NCAT; ++k) c->mem_at_peak[k] = c->mem_cat[k];
    }
    *out = p;
    return SPR_OK;
}

void dev_free(spr_ctx *c, MemCat cat, void *p, size_t bytes) {
    if (!p) return;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (c->alloc.alloc) {
        if (c->alloc.free) c->alloc.free(p, bytes, c->alloc.user);
    } else {
        (void)hipFree(p);
    }
    c->mem_cur -= bytes;
    c->mem_cat[cat] -= bytes;
}

template <typename T>
spr_status dalloc(spr_ctx *c, MemCat cat, size_t count, T **out) {
    void *p;
    CHK(dev_alloc(c, cat, count * sizeof(T), &p));
    *out = (T *)p;
    return SPR_OK;
}

template <typename T>
void dfree(spr_ctx *c, MemCat cat, T *&p, size_t count) {
    dev_free(c, cat, (void *)p, count * sizeof(T));
    p = nullptr;
}

// Several arrays carved from one device allocation (each at a 256-byte
// boundary): a render's buffers take one allocator call instead of twenty.
struct Carve {
    struct Item {
        void **ptr;
        size_t bytes;
    };
    std::vector<Item> items;
    template <typename T>
    void add(T **p, size_t count) { items.push_back({(void **)p, count * sizeof(T)}); }
    size_t total() const {
        size_t t = 0;
        for (const Item &i : items) t += (i.bytes + 255) & ~(size_t)255;
        return t;
    }
    spr_status alloc(spr_ctx *c, MemCat cat, void **base, size_t *bytes) {
        *bytes = total();
        CHK(dev_alloc(c, cat, *bytes, base));
        char *p = (char *)*base;
        for (const Item &i : items) {
            *i.ptr = p;
            p += (i.bytes + 255) & ~(size_t)255;
        }
        return SPR_OK;
    }
};

// --------------------------------------------------------- camera basis ----
// Pinhole basis in fp64 (the per-pixel part runs on the device):
// fwd = normalize(center - eye); right = normalize(fwd x up); up' = right x fwd;
// sy = tan(vfov/2), sx = sy * (w/h).  normalize(v) = v * (1 / sqrt((x^2+y^2)+z^2)).
bool make_basis(const spr_camera *c, uint32_t w, uint32_t h, ReqDev &q) {
    double f[3] = {c->center[0] - c->eye[0], c->center[1] - c->eye[1], c->center[2] - c->eye[2]};
    double fl = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    if (!(fl > 0)) return false;
    double inv = 1.0 / fl;
    for (int a = 0; a < 3; ++a) q.fwd[a] = f[a] * inv;
    double r[3] = {q.fwd[1] * c->up[2] - q.fwd[2] * c->up[1], q.fwd[2] * c->up[0] - q.fwd[0] * c->up[2],
                   q.fwd[0] * c->up[1] - q.fwd[1] * c->up[0]};
    double rl = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    if (!(rl > 0)) return false;
    inv = 1.0 / rl;
    for (int a = 0; a < 3; ++a) q.right[a] = r[a] * inv;
    q.upv[0] = q.right[1] * q.fwd[2] - q.right[2] * q.fwd[1];
    q.upv[1] = q.right[2] * q.fwd[0] - q.right[0] * q.fwd[2];
    q.upv[2] = q.right[0] * q.fwd[1] - q.right[1] * q.fwd[0];
    double th = tan((c->vfov_deg * 0.5) * (3.14159265358979323846 / 180.0));
    q.sx = th * ((double)w / (double)h);
    q.sy = th;
    for (int a = 0; a < 3; ++a) q.eye[a] = c->eye[a];
    for (int a = 0; a < 3; ++a)
        if (!isfinite(q.eye[a]) || !isfinite(q.fwd[a]) || !isfinite(q.right[a])) return false;
    for (int a = 0; a < 3; ++a)
        if (!(fabs(q.eye[a]) <= (double)SPR_MAX_EXTENT)) return false;
    return isfinite(th) && th > 0;
}

PassGrids grids_for(const spr_ctx *c, uint64_t max_A, uint64_t max_P) {
    auto g = [](uint64_t n, uint64_t per, uint32_t cap) {
        uint64_t x = (n + per - 1) / per;
        if (x < 1) x = 1;
        if (x > cap) x = cap;
        return (uint32_t)x;
    };
    PassGrids pg;
    pg.rays = g(max_A, 256, 2048);
    pg.pairs = g(max_P, 256, 2048);
    pg.dedupe = g(max_P, 1024, 2048);
    pg.slots = g(c->cache.n_slots, 256, 2048);
    pg.assign = 256;
    pg.scatter = g(max_P, 256, 2048);
    pg.decode = g(8 * max_P, 64, 4096);
    pg.max_P = max_P;
    pg.rt_tile = c->rt_tile;
    pg.rt_lb = c->rt_lb;
    pg.rt = g(max_P, c->rt_tile, 4096);
    return pg;
}

// The launch shape with the context's current raytrace tuning.
PassGrids tuned(const spr_ctx *c, const PassGrids &g0) {
    PassGrids g = g0;
    g.rt_tile = c->rt_tile;
    g.rt_lb = c->rt_lb;
    uint64_t x = (g.max_P + c->rt_tile - 1) / c->rt_tile;
    g.rt = (uint32_t)(x < 1 ? 1 : (x > 4096 ? 4096 : x));
    return g;
}

spr_status ensure_work(spr_ctx *c, uint64_t P) {
    if (P <= c->work.cap_P) return SPR_OK;
    if (P > 0xFFFFFFFFull / 8) return fail(SPR_E_INVALID, "pair space of %llu too large", (unsigned long long)P);
    HIPCHK(hipStreamSynchronize(c->stream));
    Work &W = c->work;
    size_t oP = W.cap_P, oK = W.cap_K;
    dfree(c, MEM_SCRATCH, W.vis_list, oP); dfree(c, MEM_SCRATCH, W.vis_off, oP);
    dfree(c, MEM_SCRATCH, W.miss_list, oK); dfree(c, MEM_SCRATCH, W.miss_slot, oK);
    dfree(c, MEM_SCRATCH, W.pair_rank, oP); dfree(c, MEM_SCRATCH, W.s_ray, oP); dfree(c, MEM_SCRATCH, W.s_q, oP); dfree(c, MEM_SCRATCH, W.s_vi, oP);
    dfree(c, MEM_SCRATCH, W.vis_nsl, 8 * oP);
    W.cap_P = 0; W.cap_K = 0;
    if (!W.seg_buf) CHK(dalloc(c, MEM_SCRATCH, (size_t)SEG_BIG_NS * SEG_BIG_LANES, &W.seg_buf));
    uint64_t cP = P, cK = 8 * P;
    CHK(dalloc(c, MEM_SCRATCH, cP, &W.vis_list)); CHK(dalloc(c, MEM_SCRATCH, cP, &W.vis_off));
    CHK(dalloc(c, MEM_SCRATCH, cK, &W.miss_list)); CHK(dalloc(c, MEM_SCRATCH, cK, &W.miss_slot));
    CHK(dalloc(c, MEM_SCRATCH, cP, &W.pair_rank)); CHK(dalloc(c, MEM_SCRATCH, cP, &W.s_ray)); CHK(dalloc(c, MEM_SCRATCH, cP, &W.s_q));
    CHK(dalloc(c, MEM_SCRATCH, cP, &W.s_vi)); CHK(dalloc(c, MEM_SCRATCH, 8 * cP, &W.vis_nsl));
    W.cap_P = (uint32_t)cP;
    W.cap_K = (uint32_t)cK;
    c->work_gen++;
    return SPR_OK;
}

// The arrays of a launch table, added to a carve.
void carve_table(Carve &cv, uint32_t cap, uint64_t max_A, uint64_t max_P, Table &T) {
    T.cap = cap;
    T.max_A = (uint32_t)max_A;
    T.max_P = (uint32_t)max_P;
    cv.add(&T.hdr, 1);
    cv.add(&T.act_base, cap + 1);
    cv.add(&T.pair_base, cap + 1);
    cv.add(&T.trav_base, cap + 1);
    cv.add(&T.big_base, cap + 1);
    cv.add(&T.wave_rec, max_A / 64 + 2);
    cv.add(&T.wave_off, max_A / 64 + 2);
    cv.add(&T.wave_w, max_A / 64 + 2);
}

// Wave records and weights accumulate during a pass and are cleared by its
// compaction: they start at zero.  (A render's own table needs no clearing:
// its initial-ray pass writes every record it uses.)
spr_status clear_table_records(spr_ctx *c, const Table &T) {
    HIPCHK(launch_fill_u32(c->stream, reinterpret_cast<uint32_t *>(T.wave_rec), 4 * ((uint64_t)T.max_A / 64 + 2), 0u));
    HIPCHK(launch_fill_u32(c->stream, T.wave_w, (uint64_t)T.max_A / 64 + 2, 0u));
    return SPR_OK;
}

spr_status set_table_count(spr_ctx *c, Table &T, uint32_t n) {
    HIPCHK(hipMemcpy(T.hdr, &n, sizeof(n), hipMemcpyHostToDevice));
    return SPR_OK;
}

spr_status read_state(spr_ctx *c, const ReqState *d, ReqState *h) {
    HIPCHK(hipMemcpyAsync(c->pinned, d, sizeof(ReqState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memcpy(h, c->pinned, sizeof(ReqState));
    return SPR_OK;
}

spr_status read_ctl(spr_ctx *c, PassCtl *h) {
    HIPCHK(hipMemcpyAsync((char *)c->pinned + 256, c->ctl, sizeof(PassCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memcpy(h, (char *)c->pinned + 256, sizeof(PassCtl));
    return SPR_OK;
}

// The render's state: the copy read at the end of its last run while no pass
// was enqueued since, else read back (one copy and a stream synchronisation).
static spr_status render_state(spr_render *r, ReqState *s) {
    if (r->st_valid && !r->batch) {
        *s = r->st_cache;
        return SPR_OK;
    }
    CHK(read_state(r->ctx, r->d_st, s));
    r->st_cache = *s;
    r->st_valid = !r->batch;
    return SPR_OK;
}

// One pass of a launch table replayed from a captured graph (recorded on the
// private capture stream, since the context stream may be the null stream).
spr_status graph_pass(spr_ctx *c, const Table &T, const PassGrids &g, hipGraph_t &graph, hipGraphExec_t &exec,
                      uint64_t &gen) {
    if (gen != c->work_gen || !exec) {
        if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
        if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_pass(c->cap_stream, c->ctl, T, c->d_vols, c->work, c->cache, tuned(c, g), nullptr);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gr);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return fail(SPR_E_HIP, "pass capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        graph = gr;
        HIPCHK(hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0));
        gen = c->work_gen;
    }
    HIPCHK(hipGraphLaunch(exec, c->stream));
    return SPR_OK;
}

// Profiling: add one recorded event set's kernel intervals to their slots.
constexpr int PASS_SLOTS[PASS_KERNELS] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};

spr_status prof_collect(spr_ctx *c, spr_ctx::ProfRec &rec) {
    if (!rec.pending) return SPR_OK;
    rec.pending = false;
    HIPCHK(hipEventSynchronize(rec.ev[rec.nk]));
    for (int k = 0; k < rec.nk; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, rec.ev[k], rec.ev[k + 1]));
        c->prof_ms[rec.slots[k]] += ms;
        c->prof_n[rec.slots[k]] += 1;
    }
    return SPR_OK;
}

// The next event set for nk kernels (collecting the set it replaces first).
spr_status prof_begin(spr_ctx *c, int nk, const int *slots, hipEvent_t **ev) {
    spr_ctx::ProfRec &rec = c->prof_ring[c->prof_head];
    CHK(prof_collect(c, rec));
    rec.nk = nk;
    rec.slots = slots;
    rec.pending = true;
    c->prof_head = (c->prof_head + 1) % spr_ctx::PROF_RING;
    *ev = rec.ev;
    return SPR_OK;
}

// Collect every pending set, oldest first.
spr_status prof_flush(spr_ctx *c) {
    for (int i = 0; i < spr_ctx::PROF_RING; ++i)
        CHK(prof_collect(c, c->prof_ring[(c->prof_head + i) % spr_ctx::PROF_RING]));
    return SPR_OK;
}

// One pass of a launch table, eager; in profiling mode with per-kernel events.
spr_status run_pass(spr_ctx *c, const Table &T, const PassGrids &g) {
    hipEvent_t *ev = nullptr;
    if (c->prof) CHK(prof_begin(c, PASS_KERNELS, PASS_SLOTS, &ev));
    HIPCHK(launch_pass(c->stream, c->ctl, T, c->d_vols, c->work, c->cache, tuned(c, g), ev));
    return SPR_OK;
}

}  // namespace

// ================================================================ C ABI ====

extern "C" {

const char *spr_last_error(void) { return g_err.c_str(); }

const char *spr_version(void) { return "spr 0.1 (gfx950, codec 1)"; }

spr_status spr_ctx_create(const spr_config *cfg, spr_ctx **out) {
    if (!cfg || !out) return fail(SPR_E_INVALID, "null argument");
    *out = nullptr;
    if (cfg->flags != 0) return fail(SPR_E_INVALID, "flags must be 0");
    if (cfg->spec_cap > 4096) return fail(SPR_E_INVALID, "spec cap must be in 1..4096 (0 for the default)");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(SPR_E_INVALID, "device %d out of range", cfg->device);
    uint64_t slots = cfg->cache_bytes / 256;
    if (slots < 8) return fail(SPR_E_CAPACITY, "cache of %zu bytes holds fewer than 8 blocks", cfg->cache_bytes);
    if (slots > 0x7FFFFFFFull) return fail(SPR_E_INVALID, "cache too large");
    HIPCHK(hipSetDevice(cfg->device));
    spr_ctx *c = new (std::nothrow) spr_ctx();
    if (!c) return fail(SPR_E_OOM, "host allocation failed");
    c->device = cfg->device;
    c->stream = (hipStream_t)cfg->stream;
    c->alloc = cfg->alloc;
    c->spec_cap = cfg->spec_cap ? cfg->spec_cap : 64;
    spr_status st;
#define CTX_TRY(expr)           \
    do {                        \
        st = (expr);            \
        if (st != SPR_OK) {     \
            spr_ctx_destroy(c); \
            return st;          \
        }                       \
    } while (0)
    CTX_TRY(dalloc(c, MEM_SCRATCH, 1, &c->ctl));
    CTX_TRY(dalloc(c, MEM_SCRATCH, MAX_VOLUMES, &c->d_vols));
    c->cache.n_slots = (uint32_t)slots;
    CTX_TRY(dalloc(c, MEM_CACHE, slots * 64, &c->cache.slots));
    CTX_TRY(dalloc(c, MEM_CACHE, slots, &c->cache.owner));
    CTX_TRY(dalloc(c, MEM_CACHE, slots, &c->cache.stamp));
    CTX_TRY(dalloc(c, MEM_CACHE, slots, &c->cache.free_stack));
    if (hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        spr_ctx_destroy(c);
        return fail(SPR_E_OOM, "pinned host allocation failed");
    }
    // the pass end writes a render's active-ray count here, so the host polls
    // it without a copy per pass (fine-grained: the write reaches host memory)
    if (hipHostMalloc((void **)&c->nact_host, 256, hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->nact_dev, c->nact_host, 0) != hipSuccess) {
        spr_ctx_destroy(c);
        return fail(SPR_E_OOM, "pinned host allocation failed");
    }
    bool evok = true;

    if (!evok || hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        spr_ctx_destroy(c);
        return fail(SPR_E_HIP, "hipEventCreate failed");
    }
    if ((st = scratch_ptr(c->device, &c->noalloc)) != SPR_OK) {
        spr_ctx_destroy(c);
        return st;
    }
    PassCtl h{};
    h.n_slots = (uint32_t)slots;
    h.free_top = (uint32_t)slots;
    h.evict_T = 64;
    memcpy(c->pinned, &h, sizeof(h));
    if (hipMemcpyAsync(c->ctl, c->pinned, sizeof(h), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        launch_fill_u64(c->stream, c->cache.owner, slots, ~0ull) != hipSuccess ||
        launch_fill_u32(c->stream, c->cache.stamp, slots, 0) != hipSuccess ||
        launch_iota_u32(c->stream, c->cache.free_stack, slots) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        spr_ctx_destroy(c);
        return fail(SPR_E_HIP, "context initialisation failed");
    }
#undef CTX_TRY
    *out = c;
    return SPR_OK;
}

spr_status spr_ctx_destroy(spr_ctx *c) {
    if (!c) return fail(SPR_E_INVALID, "null context");
    (void)hipSetDevice(c->device);
    if (c->stream || true) (void)hipStreamSynchronize(c->stream);
    Work &W = c->work;
    size_t oP = W.cap_P, oK = W.cap_K;
    dfree(c, MEM_SCRATCH, W.vis_list, oP); dfree(c, MEM_SCRATCH, W.vis_off, oP);
    dfree(c, MEM_SCRATCH, W.miss_list, oK); dfree(c, MEM_SCRATCH, W.miss_slot, oK);
    dfree(c, MEM_SCRATCH, W.pair_rank, oP); dfree(c, MEM_SCRATCH, W.s_ray, oP); dfree(c, MEM_SCRATCH, W.s_q, oP); dfree(c, MEM_SCRATCH, W.s_vi, oP);
    dfree(c, MEM_SCRATCH, W.vis_nsl, 8 * oP);
    dfree(c, MEM_SCRATCH, W.seg_buf, (size_t)SEG_BIG_NS * SEG_BIG_LANES);
    size_t ns = c->cache.n_slots;
    dfree(c, MEM_CACHE, c->cache.slots, ns * 64);
    dfree(c, MEM_CACHE, c->cache.owner, ns);
    dfree(c, MEM_CACHE, c->cache.stamp, ns);
    dfree(c, MEM_CACHE, c->cache.free_stack, ns);
    dfree(c, MEM_SCRATCH, c->ctl, 1);
    dfree(c, MEM_SCRATCH, c->d_vols, MAX_VOLUMES);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->nact_host) (void)hipHostFree(c->nact_host);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &rec : c->prof_ring)
        for (auto &e : rec.ev)
            if (e) (void)hipEventDestroy(e);
    delete c;
    return SPR_OK;
}

spr_status spr_mem_stats(spr_ctx *c, size_t *current, size_t *peak) {
    if (!c) return fail(SPR_E_INVALID, "null context");
    if (current) *current = c->mem_cur;
    if (peak) *peak = c->mem_peak;
    return SPR_OK;
}

spr_status spr_mem_split_get(spr_ctx *c, spr_mem_split *o, int reset_peak) {
    if (!c || !o) return fail(SPR_E_INVALID, "null argument");
    static_assert(MEM_NCAT == SPR_MEM_KINDS, "memory kinds");
    for (int k = 0; k < MEM_NCAT; ++k) {
        o->current[k] = c->mem_cat[k];
        o->at_peak[k] = c->mem_at_peak[k];
        o->kind_peak[k] = c->mem_cat_peak[k];
    }
    o->total = c->mem_cur;
    o->peak = c->mem_peak;
    if (reset_peak) {
        c->mem_peak = c->mem_cur;
        for (int k = 0; k < MEM_NCAT; ++k) {
            c->mem_cat_peak[k] = c->mem_cat[k];
            c->mem_at_peak[k] = c->mem_cat[k];
        }
    }
    return SPR_OK;
}

spr_status spr_ctx_counters(spr_ctx *c, spr_counters *o) {
    if (!c || !o) return fail(SPR_E_INVALID, "null argument");
    HIPCHK(hipSetDevice(c->device));
    PassCtl p;
    CHK(read_ctl(c, &p));
    memset(o, 0, sizeof(*o));
    o->passes = p.acc_passes;
    o->blocks_decoded = p.acc_decoded;
    o->visible_blocks = p.acc_visible;
    o->active_blocks = p.acc_active;
    o->pairs = p.acc_pairs;
    o->evicted = p.acc_evicted;
    o->overflow = p.acc_overflow;
    o->rays = p.acc_rays;
    o->pair_slots = p.acc_slots;
    o->served_pairs = p.acc_served;
    o->max_active_blocks = p.acc_max_active;
    o->walk_guard = p.acc_guard;
    o->coarse_steps = p.acc_csteps;
    o->coarse_masks = p.acc_cmasks;
    return SPR_OK;
}

spr_status spr_ctx_profile(spr_ctx *c, int enable, int reset) {
    if (!c) return fail(SPR_E_INVALID, "null context");
    HIPCHK(hipSetDevice(c->device));
    if (enable && !c->prof_events) {
        for (auto &rec : c->prof_ring)
            for (auto &e : rec.ev) HIPCHK(hipEventCreate(&e));
        c->prof_events = true;
    }
    CHK(prof_flush(c));
    c->prof = enable != 0;
    if (reset) {
        for (int k = 0; k < PROF_SLOTS; ++k) { c->prof_ms[k] = 0; c->prof_n[k] = 0; }
    }
    return SPR_OK;
}

spr_status spr_ctx_kernel_times(spr_ctx *c, spr_kernel_time *out, uint32_t max, uint32_t *n) {
    if (!c || !n || (!out && max)) return fail(SPR_E_INVALID, "null argument");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(prof_flush(c));
    uint32_t k = 0;
    for (; k < (uint32_t)PROF_SLOTS && k < max; ++k) {
        out[k].name = PROF_NAMES[k];
        out[k].total_ms = c->prof_ms[k];
        out[k].launches = c->prof_n[k];
    }
    *n = k;
    return SPR_OK;
}

spr_status spr_ctx_set_tuning(spr_ctx *c, const spr_tuning *t) {
    if (!c || !t) return fail(SPR_E_INVALID, "null argument");
    if (t->pairs_per_wg != 128 && t->pairs_per_wg != 256)
        return fail(SPR_E_INVALID, "pairs_per_wg must be 128 or 256 (got %u)", t->pairs_per_wg);
    if (t->slot_tile != 0 && t->slot_tile != 16 && t->slot_tile != 32)
        return fail(SPR_E_INVALID, "slot_tile must be 0, 16 or 32 (got %u)", t->slot_tile);
    if (t->pairs_per_wg != c->rt_tile || t->slot_tile != c->rt_lb) {
        c->rt_tile = t->pairs_per_wg;
        c->rt_lb = t->slot_tile;
        c->work_gen++;   // captured pass graphs are re-recorded with the new shape
    }
    return SPR_OK;
}

spr_status spr_ctx_get_tuning(spr_ctx *c, spr_tuning *out) {
    if (!c || !out) return fail(SPR_E_INVALID, "null argument");
    out->pairs_per_wg = c->rt_tile;
    out->slot_tile = c->rt_lb;
    return SPR_OK;
}

// ----------------------------------------------------------------- volume --

static void free_volume_buffers(spr_ctx *c, VolDev &V, size_t stream_bytes) {
    uint64_t nb = V.nblocks;
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    dev_free(c, MEM_COMPRESSED, (void *)V.stream, stream_bytes);
    V.stream = nullptr;
    dfree(c, MEM_GRIDS, V.fine, nb);
    dfree(c, MEM_GRIDS, V.coarse, nc);
    const uint64_t ns = bidx_count(V);
    dfree(c, MEM_GRIDS, V.map, ns);
    dfree(c, MEM_GRIDS, V.blk_cnt, ns);
    dfree(c, MEM_GRIDS, V.vis_idx, ns);
    dfree(c, MEM_GRIDS, V.claim, nc);
}

spr_status spr_volume_load(spr_ctx *c, const void *host_stream, size_t bytes, const spr_volume_desc *d,
                           spr_volume **out) {
    if (!c || !host_stream || !d || !out) return fail(SPR_E_INVALID, "null argument");
    *out = nullptr;
    if (d->codec_version != SPR_CODEC_VERSION) return fail(SPR_E_INVALID, "unknown codec version %u", d->codec_version);
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return fail(SPR_E_INVALID, "volume must have at least 2 samples per axis");
    if (d->nx > SPR_MAX_EXTENT || d->ny > SPR_MAX_EXTENT || d->nz > SPR_MAX_EXTENT)
        return fail(SPR_E_INVALID, "volume extent above SPR_MAX_EXTENT samples on an axis");
    if (!((d->rate_bits >= 1 && d->rate_bits <= 16) || d->rate_bits == 32))
        return fail(SPR_E_INVALID, "rate_bits %u not in 1..16 or 32", d->rate_bits);
    if (d->src_dtype != SPR_DTYPE_F32 && d->src_dtype != SPR_DTYPE_U8) return fail(SPR_E_INVALID, "bad src_dtype");
    uint64_t nbx = (d->nx + 3) / 4, nby = (d->ny + 3) / 4, nbz = (d->nz + 3) / 4;
    uint64_t nb = nbx * nby * nbz;
    if (nb >= 0xFFFFFFF0ull) return fail(SPR_E_INVALID, "too many blocks");
    uint64_t expect = nb * 8ull * d->rate_bits;
    if (bytes != expect)
        return fail(SPR_E_CORRUPT, "stream has %zu bytes, descriptor needs %llu", bytes, (unsigned long long)expect);
    int idx = -1;
    for (int i = 0; i < MAX_VOLUMES; ++i)
        if (!c->vol_handles[i]) { idx = i; break; }
    if (idx < 0) return fail(SPR_E_CAPACITY, "too many volumes in one context");
    HIPCHK(hipSetDevice(c->device));
    VolDev V{};
    V.n[0] = (int)d->nx; V.n[1] = (int)d->ny; V.n[2] = (int)d->nz;
    for (int a = 0; a < 3; ++a) {
        V.nb[a] = (V.n[a] + 3) / 4;
        V.nc[a] = (V.nb[a] + 3) / 4;
        V.tb[a] = (V.n[a] - 1 + 3) / 4;
        V.tc[a] = (V.tb[a] + 3) / 4;
    }
    if (bidx_count(V) >= 0xFFFFFFF0ull) return fail(SPR_E_INVALID, "too many blocks");
    V.rate = (int)d->rate_bits;
    V.rec_words = 2 * (int)d->rate_bits;
    V.nblocks = nb;
    V.live = 1;
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    spr_status st = SPR_OK;
    void *sp = nullptr;
    do {
        if ((st = dev_alloc(c, MEM_COMPRESSED, bytes, &sp)) != SPR_OK) break;
        V.stream = (const uint32_t *)sp;
        if ((st = dalloc(c, MEM_GRIDS, nb, &V.fine)) != SPR_OK) break;
        if ((st = dalloc(c, MEM_GRIDS, nc, &V.coarse)) != SPR_OK) break;
        if ((st = dalloc(c, MEM_GRIDS, bidx_count(V), &V.map)) != SPR_OK) break;
        if ((st = dalloc(c, MEM_GRIDS, bidx_count(V), &V.blk_cnt)) != SPR_OK) break;
        if ((st = dalloc(c, MEM_GRIDS, bidx_count(V), &V.vis_idx)) != SPR_OK) break;
        if ((st = dalloc(c, MEM_GRIDS, nc, &V.claim)) != SPR_OK) break;
    } while (0);
    if (st != SPR_OK) {
        free_volume_buffers(c, V, bytes);
        return st;
    }
    hipError_t e = hipMemcpyAsync(sp, host_stream, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fill_u32(c->stream, V.map, bidx_count(V), NONE);
    if (e == hipSuccess) e = launch_fill_u32(c->stream, V.blk_cnt, bidx_count(V), 0);
    if (e == hipSuccess) e = launch_fill_u32(c->stream, V.vis_idx, bidx_count(V), 0);
    if (e == hipSuccess) e = launch_fill_u64(c->stream, V.claim, nc, 0ull);
    if (e == hipSuccess) e = launch_load_grids(c->stream, V);
    c->h_vols[idx] = V;
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_vols + idx, &c->h_vols[idx], sizeof(VolDev), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_volume_buffers(c, V, bytes);
        return fail(SPR_E_HIP, "volume upload failed: %s", hipGetErrorString(e));
    }
    spr_volume *v = new (std::nothrow) spr_volume();
    if (!v) {
        free_volume_buffers(c, V, bytes);
        return fail(SPR_E_OOM, "host allocation failed");
    }
    v->ctx = c;
    v->idx = (uint32_t)idx;
    v->desc = *d;
    v->stream_bytes = bytes;
    c->vol_handles[idx] = v;
    *out = v;
    return SPR_OK;
}

spr_status spr_volume_free(spr_volume *v) {
    if (!v) return fail(SPR_E_INVALID, "null volume");
    spr_ctx *c = v->ctx;
    if (v->n_renders) return fail(SPR_E_STATE, "volume still has %d live renders", v->n_renders);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_release_volume(c->stream, c->ctl, c->cache, v->idx));
    VolDev &V = c->h_vols[v->idx];
    V.live = 0;
    HIPCHK(hipMemcpyAsync(c->d_vols + v->idx, &V, sizeof(VolDev), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    free_volume_buffers(c, V, v->stream_bytes);
    for (MaskSet &m : v->msets) {
        dev_free(c, MEM_GRIDS, m.buf, m.bytes);
        m = MaskSet{};
    }
    c->vol_handles[v->idx] = nullptr;
    delete v;
    return SPR_OK;
}

spr_status spr_volume_build_grids(spr_volume *v) {
    if (!v) return fail(SPR_E_INVALID, "null volume");
    spr_ctx *c = v->ctx;
    HIPCHK(hipSetDevice(c->device));
    hipEvent_t *ev = nullptr;
    if (c->prof) CHK(prof_begin(c, 3, LOAD_SLOTS, &ev));
    HIPCHK(launch_load_grids(c->stream, c->h_vols[v->idx], ev));
    // kept masks were built from the ranges just rewritten: new renders build
    // theirs again (sets in use keep serving their renders)
    for (MaskSet &m : v->msets) m.keyed = false;
    return SPR_OK;
}

spr_status spr_volume_ranges(spr_volume *v, float *fine, size_t fine_count, float *coarse, size_t coarse_count) {
    if (!v) return fail(SPR_E_INVALID, "null volume");
    spr_ctx *c = v->ctx;
    const VolDev &V = c->h_vols[v->idx];
    uint64_t nc = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    if (fine && fine_count != V.nblocks) return fail(SPR_E_INVALID, "fine_count must be %llu", (unsigned long long)V.nblocks);
    if (coarse && coarse_count != nc) return fail(SPR_E_INVALID, "coarse_count must be %llu", (unsigned long long)nc);
    HIPCHK(hipSetDevice(c->device));
    if (fine) HIPCHK(hipMemcpyAsync(fine, V.fine, V.nblocks * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
    if (coarse) HIPCHK(hipMemcpyAsync(coarse, V.coarse, nc * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPR_OK;
}

spr_status spr_debug_decode_blocks(spr_volume *v, const uint32_t *ids, uint32_t n, float *host_out) {
    if (!v || (!ids && n) || (!host_out && n)) return fail(SPR_E_INVALID, "null argument");
    if (n == 0) return SPR_OK;
    spr_ctx *c = v->ctx;
    const VolDev &V = c->h_vols[v->idx];
    for (uint32_t i = 0; i < n; ++i)
        if (ids[i] >= V.nblocks) return fail(SPR_E_INVALID, "block id %u out of range", ids[i]);
    HIPCHK(hipSetDevice(c->device));
    uint32_t *d_ids = nullptr;
    float *d_out = nullptr;
    CHK(dalloc(c, MEM_SCRATCH, n, &d_ids));
    spr_status st = dalloc(c, MEM_SCRATCH, (size_t)n * 64, &d_out);
    if (st != SPR_OK) {
        dfree(c, MEM_SCRATCH, d_ids, n);
        return st;
    }
    hipError_t e = hipMemcpyAsync(d_ids, ids, n * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_decode_ids(c->stream, V, d_ids, n, d_out);
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, d_out, (size_t)n * 64 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, MEM_SCRATCH, d_ids, n);
    dfree(c, MEM_SCRATCH, d_out, (size_t)n * 64);
    if (e != hipSuccess) return fail(SPR_E_HIP, "debug decode failed: %s", hipGetErrorString(e));
    return SPR_OK;
}

spr_status spr_debug_decode_blocks_noalloc(spr_volume *v, const uint32_t *ids, uint32_t n, float *host_out) {
    if (!v || (!ids && n) || (!host_out && n)) return fail(SPR_E_INVALID, "null argument");
    if (n > SPR_NOALLOC_MAX_BLOCKS)
        return fail(SPR_E_CAPACITY, "%u blocks exceed the allocation-free limit of %u", n, SPR_NOALLOC_MAX_BLOCKS);
    if (n == 0) return SPR_OK;
    spr_ctx *c = v->ctx;
    const VolDev &V = c->h_vols[v->idx];
    for (uint32_t i = 0; i < n; ++i)
        if (ids[i] >= V.nblocks) return fail(SPR_E_INVALID, "block id %u out of range", ids[i]);
    HIPCHK(hipSetDevice(c->device));
    // c->noalloc was looked up for this device when the context was created
    uint32_t *d_ids = (uint32_t *)c->noalloc;
    float *d_out = (float *)((unsigned char *)c->noalloc + NOALLOC_OUT_OFF);
    hipError_t e = hipMemcpyAsync(d_ids, ids, n * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_decode_ids(c->stream, V, d_ids, n, d_out);
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, d_out, (size_t)n * 64 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(SPR_E_HIP, "allocation-free decode failed: %s", hipGetErrorString(e));
    return SPR_OK;
}

spr_status spr_debug_fp64_ops(spr_ctx *c, const double *x, const double *y, size_t n, double *sq, double *dv) {
    if (!c || ((!x || !y || !sq || !dv) && n)) return fail(SPR_E_INVALID, "null argument");
    if (n == 0) return SPR_OK;
    HIPCHK(hipSetDevice(c->device));
    double *buf = nullptr;
    CHK(dalloc(c, MEM_SCRATCH, 4 * n, &buf));
    hipError_t e = hipMemcpyAsync(buf, x, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(buf + n, y, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_fp64_ops(c->stream, buf, buf + n, n, buf + 2 * n, buf + 3 * n);
    if (e == hipSuccess) e = hipMemcpyAsync(sq, buf + 2 * n, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dv, buf + 3 * n, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(c, MEM_SCRATCH, buf, 4 * n);
    if (e != hipSuccess) return fail(SPR_E_HIP, "fp64 probe failed: %s", hipGetErrorString(e));
    return SPR_OK;
}

// ----------------------------------------------------------------- render --

static void free_render_buffers(spr_ctx *c, spr_render *r) {
    dev_free(c, MEM_RAYS, r->buf, r->buf_bytes);
    r->buf = nullptr;
    r->buf_bytes = 0;
}

// The volume's mask set for iso: a kept one (*build = false), or the least
// recently used set that no live render reads, keyed to iso (*build = true,
// allocated on first use); *idx = -1 when every set is in use.
static spr_status mask_set_acquire(spr_ctx *c, spr_volume *v, float iso, uint64_t cwords, int *idx, bool *build) {
    uint32_t bits;
    memcpy(&bits, &iso, sizeof bits);
    *idx = -1;
    *build = true;
    int pick = -1;
    for (int i = 0; i < MASK_SETS && pick < 0; ++i)
        if (v->msets[i].keyed && v->msets[i].iso_bits == bits) pick = i;
    if (pick >= 0) {
        *build = false;
    } else {
        for (int i = 0; i < MASK_SETS; ++i) {
            const MaskSet &m = v->msets[i];
            if (m.users) continue;
            if (pick < 0) { pick = i; continue; }
            const MaskSet &b = v->msets[pick];
            if ((b.keyed && !m.keyed) || (b.keyed == m.keyed && m.last_use < b.last_use)) pick = i;
        }
        if (pick < 0) return SPR_OK;
        MaskSet &m = v->msets[pick];
        if (!m.buf) {
            Carve cv;
            cv.add(&m.mstat, 2);
            cv.add(&m.cmask64, cwords);
            cv.add(&m.cdist, 2 * cwords);
            CHK(cv.alloc(c, MEM_GRIDS, &m.buf, &m.bytes));
        }
        m.iso_bits = bits;
        m.keyed = true;
    }
    MaskSet &m = v->msets[pick];
    m.users++;
    m.last_use = ++v->mask_clock;
    *idx = pick;
    return SPR_OK;
}

// A render stops reading its mask set; unkey: the set was to be built by a
// render whose set-up failed, so it holds no masks.
static void mask_set_release(spr_volume *v, int idx, bool unkey) {
    if (idx < 0) return;
    MaskSet &m = v->msets[idx];
    m.users--;
    if (unkey) m.keyed = false;
}

spr_status spr_render_begin(spr_volume *v, const spr_camera *cam, float iso, uint32_t w, uint32_t h,
                            spr_render **out) {
    if (!v || !cam || !out) return fail(SPR_E_INVALID, "null argument");
    *out = nullptr;
    if (w == 0 || h == 0) return fail(SPR_E_INVALID, "empty image");
    uint64_t npix = (uint64_t)w * h;
    if (npix >= (1ull << 24)) return fail(SPR_E_INVALID, "w*h must be < 2^24");
    if (!isfinite(iso)) return fail(SPR_E_INVALID, "isovalue must be finite");
    spr_ctx *c = v->ctx;
    spr_render *r = new (std::nothrow) spr_render();
    if (!r) return fail(SPR_E_OOM, "host allocation failed");
    r->ctx = c;
    r->vol = v;
    r->w = w; r->h = h; r->npix = (uint32_t)npix;
    ReqDev &q = r->hreq;
    if (!make_basis(cam, w, h, q)) {
        delete r;
        return fail(SPR_E_INVALID, "degenerate camera (zero view direction, view along up, or eye beyond SPR_MAX_EXTENT)");
    }
    q.iso = iso;
    q.w = w; q.h = h; q.npix = (uint32_t)npix;
    q.vol = v->idx;
    q.spec_cap = c->spec_cap;
    HIPCHK(hipSetDevice(c->device));
    {
        const VolDev &V = c->h_vols[v->idx];
        r->cwords = (uint64_t)V.nc[0] * V.nc[1] * V.nc[2];
    }
    {
        spr_status ms = mask_set_acquire(c, v, iso, r->cwords, &r->mset, &r->masks_built);
        if (ms != SPR_OK) {
            delete r;
            return ms;
        }
    }
    if (r->mset >= 0) {
        const MaskSet &m = v->msets[r->mset];
        q.cmask64 = m.cmask64;
        q.cdist = m.cdist;
        q.mstat = m.mstat;
        q.mstat_load = r->masks_built ? 0u : 1u;
    }
    Carve cv;
    cv.add(&q.ray_state, npix);
    cv.add(&q.act[0], npix);
    cv.add(&q.act[1], npix);
    cv.add(&q.pair_blk, npix);
    cv.add(&q.tslot, npix);
    cv.add(&q.best, npix);
    cv.add(&q.nfound, npix);
    cv.add(&q.def_first, npix);
    cv.add(&q.rbase, npix);
    cv.add(&q.rns, npix);
    cv.add(&q.rw, npix);
    cv.add(&q.pair_ray, npix);
    cv.add(&q.image, npix);
    cv.add(&q.hits, npix);
    cv.add(&r->d_st, 1);
    cv.add(&r->d_req, 1);
    if (r->mset < 0) {
        cv.add(&q.cmask64, r->cwords);
        cv.add(&q.cdist, 2 * r->cwords);
    }
    carve_table(cv, 1, round64h(npix), npix, r->table);
    r->table.host_nact = c->nact_dev;
    spr_status st = cv.alloc(c, MEM_RAYS, &r->buf, &r->buf_bytes);
    if (st == SPR_OK) st = ensure_work(c, npix);
    if (st != SPR_OK) {
        free_render_buffers(c, r);
        mask_set_release(v, r->mset, r->masks_built);
        delete r;
        return st;
    }
    q.st = r->d_st;
    r->table.reqs = r->d_req;
    r->grids = grids_for(c, round64h(npix), npix);
    ReqState s0{};
    s0.n_act = (uint32_t)npix;
    s0.cur = 1;
    // description, initial state and request count written in stream order
    // (kernel arguments: no host synchronisation)
    hipError_t e = launch_put_req(c->stream, r->d_req, q, r->d_st, &s0, r->table.hdr, 1u);
    hipEvent_t *pev = nullptr;
    const bool build = r->masks_built;
    if (e == hipSuccess && c->prof && prof_begin(c, build ? 5 : 4, build ? INIT_SLOTS : INIT_SLOTS + 1, &pev) != SPR_OK)
        e = hipErrorUnknown;
    if (e == hipSuccess) e = launch_init_rays(c->stream, c->ctl, r->table, c->d_vols, r->cwords, build, pev);
    if (e != hipSuccess) {
        free_render_buffers(c, r);
        mask_set_release(v, r->mset, build);
        delete r;
        return fail(SPR_E_HIP, "render set-up failed: %s", hipGetErrorString(e));
    }
    v->n_renders++;
    c->n_renders++;
    *out = r;
    return SPR_OK;
}

spr_status spr_render_set_spec_cap(spr_render *r, uint32_t cap) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (cap < 1 || cap > 4096) return fail(SPR_E_INVALID, "spec cap must be in 1..4096");
    if (r->started) return fail(SPR_E_STATE, "speculation cap can only change before the first pass");
    if (r->batch) return fail(SPR_E_STATE, "render belongs to a live batch");
    if (cap == r->hreq.spec_cap) return SPR_OK;
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    // the first pass takes its count from the cap in the description
    // (k_pass_begin), so only the description changes
    r->hreq.spec_cap = cap;
    HIPCHK(launch_put_req(c->stream, r->d_req, r->hreq, nullptr, nullptr, nullptr, 0u));
    return SPR_OK;
}

spr_status spr_render_set_spec_policy(spr_render *r, uint32_t policy) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (policy != SPR_SPEC_UNIFORM && policy != SPR_SPEC_PER_RAY)
        return fail(SPR_E_INVALID, "unknown speculation policy %u", policy);
    if (r->started) return fail(SPR_E_STATE, "the speculation policy can only change before the first pass");
    if (r->batch) return fail(SPR_E_STATE, "render belongs to a live batch");
    if (policy == r->hreq.policy) return SPR_OK;
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    r->hreq.policy = policy;
    HIPCHK(launch_put_req(c->stream, r->d_req, r->hreq, nullptr, nullptr, nullptr, 0u));
    return SPR_OK;
}

static spr_status fill_stats(spr_render *r, spr_pass_stats *o, float ms) {
    spr_ctx *c = r->ctx;
    ReqState s;
    PassCtl p;
    CHK(render_state(r, &s));
    CHK(read_ctl(c, &p));
    memset(o, 0, sizeof(*o));
    o->pass = s.passes;
    o->n_active = s.n_act_prev;
    o->n_spec = s.last_nspec;
    o->pairs = s.last_pairs;
    o->visible_blocks = p.n_vis;
    o->active_blocks = p.n_actblk;
    o->blocks_decoded = p.n_miss;
    o->deferred_pairs = s.last_deferred;
    o->terminated = s.last_terminated;
    o->slots = s.last_slots;
    o->utilization = r->npix ? (double)s.last_pairs / (double)r->npix : 0.0;
    o->ms = ms;
    return SPR_OK;
}

spr_status spr_render_pass(spr_render *r, spr_pass_stats *stats) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (r->batch) return fail(SPR_E_STATE, "render belongs to a live batch");
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    r->st_valid = false;
    if (stats) HIPCHK(hipEventRecord(c->ev0, c->stream));
    if (c->prof) CHK(run_pass(c, r->table, r->grids));
    else CHK(graph_pass(c, r->table, r->grids, r->graph, r->exec, r->graph_gen));
    r->started = true;
    if (stats) {
        HIPCHK(hipEventRecord(c->ev1, c->stream));
        HIPCHK(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        CHK(fill_stats(r, stats, ms));
    }
    return SPR_OK;
}

spr_status spr_render_done(spr_render *r, int *done) {
    if (!r || !done) return fail(SPR_E_INVALID, "null argument");
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    ReqState s;
    CHK(render_state(r, &s));
    *done = s.n_act == 0;
    return SPR_OK;
}

spr_status spr_render_run(spr_render *r, uint32_t max_passes, uint32_t *passes_run) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (r->batch) return fail(SPR_E_STATE, "render belongs to a live batch");
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    // A render that has not run a pass starts at pass 0 with its active rays
    // unknown here: it is taken as not finished (a pass on a finished render
    // does no work), which saves reading the state back first.
    ReqState s0{};
    if (r->started || r->st_valid) {
        CHK(render_state(r, &s0));
    } else {
        s0.passes = 0;
        s0.n_act = r->npix;
    }
    const uint32_t start = s0.passes;
    // Keep two passes in flight: after enqueuing pass i+1, wait for pass i's
    // copy of N_act.  A pass on a finished render does no work, so the one
    // pass that may run past completion costs only its empty launches; once
    // the last N_act seen is small (the render is about to finish), keep one
    // pass in flight, which trades that empty pass for one host round trip.
    const int DEPTH = 2;
    const uint32_t NEAR_END = r->npix / 256u > 256u ? r->npix / 256u : 256u;
    hipEvent_t ev[DEPTH] = {c->ev0, c->ev1};
    // the pass end of every pass of this render writes its active-ray count
    // to this fine-grained host word; after pass i's event it holds the count
    // after pass i or a later one (counts only fall)
    volatile uint32_t *flag = (volatile uint32_t *)c->nact_host;
    uint32_t enq = 0, waited = 0, last_act = s0.n_act;
    bool done = s0.n_act == 0;
    while (!done) {
        const uint32_t depth = last_act <= NEAR_END ? 1u : (uint32_t)DEPTH;
        while (enq < max_passes && enq - waited < depth) {
            CHK(spr_render_pass(r, nullptr));
            HIPCHK(hipEventRecord(ev[enq % DEPTH], c->stream));
            ++enq;
        }
        if (waited == enq) break;   // max_passes reached
        HIPCHK(hipEventSynchronize(ev[waited % DEPTH]));
        last_act = flag[0];
        done = last_act == 0;
        ++waited;
    }
    ReqState s1;
    r->st_valid = false;
    CHK(render_state(r, &s1));   // synchronises the stream; kept for get_info and done
    if (passes_run) *passes_run = s1.passes - start;
    return SPR_OK;
}

spr_status spr_render_get_info(spr_render *r, spr_render_info *o) {
    if (!r || !o) return fail(SPR_E_INVALID, "null argument");
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    ReqState s;
    CHK(render_state(r, &s));
    memset(o, 0, sizeof(*o));
    o->w = r->w;
    o->h = r->h;
    o->rays_entered = s.passes ? s.entered : s.n_act;
    o->n_active = s.n_act;
    o->n_spec = s.n_spec;
    if (s.passes == 0 && s.n_act > 0) {
        // before the first pass the count follows the current cap (as k_pass_begin takes it)
        uint32_t ns = r->npix / s.n_act;
        o->n_spec = ns < 1u ? 1u : (ns > r->hreq.spec_cap ? r->hreq.spec_cap : ns);
    }
    o->passes = s.passes;
    o->pairs = s.tot_pairs;
    o->bcmc_blocks = s.bcmc;
    o->iso_coarse_cells = s.ccells;
    o->masks_built = r->masks_built ? 1u : 0u;
    return SPR_OK;
}

spr_status spr_read_image(spr_render *r, uint8_t *rgba, size_t bytes) {
    if (!r || !rgba) return fail(SPR_E_INVALID, "null argument");
    if (bytes != (size_t)r->npix * 4) return fail(SPR_E_INVALID, "image needs %zu bytes", (size_t)r->npix * 4);
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpyAsync(rgba, r->hreq.image, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPR_OK;
}

spr_status spr_read_hits(spr_render *r, spr_hit *hits, size_t count) {
    if (!r || !hits) return fail(SPR_E_INVALID, "null argument");
    if (count != r->npix) return fail(SPR_E_INVALID, "hit buffer needs %u records", r->npix);
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpyAsync(hits, r->hreq.hits, count * sizeof(spr_hit), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPR_OK;
}

spr_status spr_render_device_ptrs(spr_render *r, void **rgba, void **hits) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (rgba) *rgba = r->hreq.image;
    if (hits) *hits = r->hreq.hits;
    return SPR_OK;
}

spr_status spr_render_free(spr_render *r) {
    if (!r) return fail(SPR_E_INVALID, "null render");
    if (r->batch) return fail(SPR_E_STATE, "render belongs to a live batch");
    spr_ctx *c = r->ctx;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    free_render_buffers(c, r);
    mask_set_release(r->vol, r->mset, false);
    r->vol->n_renders--;
    c->n_renders--;
    delete r;
    return SPR_OK;
}

// ------------------------------------------------------------------ batch --

spr_status spr_batch_create_empty(spr_ctx *c, uint32_t max_requests, uint64_t max_pixels, spr_batch **out) {
    if (!c || !out) return fail(SPR_E_INVALID, "null argument");
    *out = nullptr;
    if (max_requests == 0 || max_requests > MAX_REQS) return fail(SPR_E_INVALID, "batch capacity must be 1..%d", MAX_REQS);
    uint64_t A = max_pixels + 64ull * max_requests, P = max_pixels;
    if (A >= 0xFFFFFFFFull || P > 0xFFFFFFFFull / 8 || max_pixels == 0) return fail(SPR_E_INVALID, "bad pixel capacity");
    HIPCHK(hipSetDevice(c->device));
    spr_batch *b = new (std::nothrow) spr_batch();
    if (!b) return fail(SPR_E_OOM, "host allocation failed");
    b->ctx = c;
    b->max_pixels = max_pixels;
    Carve cv;
    carve_table(cv, max_requests, A, P, b->table);
    cv.add(&b->table.reqs, max_requests);
    cv.add(&b->d_state, (size_t)max_requests + 1);
    spr_status st = cv.alloc(c, MEM_SCRATCH, &b->buf, &b->buf_bytes);
    if (st == SPR_OK) st = clear_table_records(c, b->table);
    if (st == SPR_OK && hipHostMalloc((void **)&b->h_state, sizeof(uint4) * ((size_t)max_requests + 1),
                                      hipHostMallocDefault) != hipSuccess) {
        b->h_state = nullptr;
        st = fail(SPR_E_OOM, "pinned host allocation failed");
    }
    if (st == SPR_OK) st = ensure_work(c, P);
    if (st == SPR_OK) st = set_table_count(c, b->table, 0);
    if (st != SPR_OK) {
        dev_free(c, MEM_SCRATCH, b->buf, b->buf_bytes);
        if (b->h_state) (void)hipHostFree(b->h_state);
        delete b;
        return st;
    }
    b->grids = grids_for(c, A, P);
    *out = b;
    return SPR_OK;
}

spr_status spr_batch_set(spr_batch *b, uint32_t n, spr_render *const *renders) {
    if (!b || (n && !renders)) return fail(SPR_E_INVALID, "null argument");
    spr_ctx *c = b->ctx;
    if (n > b->table.cap) return fail(SPR_E_CAPACITY, "%u renders exceed the batch capacity %u", n, b->table.cap);
    uint64_t pix = 0;
    for (uint32_t i = 0; i < n; ++i) {
        spr_render *r = renders[i];
        if (!r || r->ctx != c) return fail(SPR_E_INVALID, "render %u is null or from another context", i);
        if (r->batch && r->batch != b) return fail(SPR_E_STATE, "render %u belongs to another batch", i);
        for (uint32_t j = 0; j < i; ++j)
            if (renders[j] == r) return fail(SPR_E_INVALID, "render %u listed twice", i);
        pix += r->npix;
    }
    if (pix > b->max_pixels) return fail(SPR_E_CAPACITY, "renders need %llu pixels, batch holds %llu",
                                         (unsigned long long)pix, (unsigned long long)b->max_pixels);
    HIPCHK(hipSetDevice(c->device));
    std::vector<ReqDev> reqs(n);
    for (uint32_t i = 0; i < n; ++i) reqs[i] = renders[i]->hreq;
    // stream-ordered: passes already enqueued see the old table
    HIPCHK(hipStreamSynchronize(c->stream));
    if (n) HIPCHK(hipMemcpy(b->table.reqs, reqs.data(), n * sizeof(ReqDev), hipMemcpyHostToDevice));
    CHK(set_table_count(c, b->table, n));
    for (auto *r : b->renders) r->batch = nullptr;
    b->renders.assign(renders, renders + n);
    for (auto *r : b->renders) {
        r->batch = b;
        r->st_valid = false;   // batch passes change its state
    }
    b->state_fresh = false;
    return SPR_OK;
}

spr_status spr_batch_create(spr_ctx *c, uint32_t n, spr_render *const *renders, spr_batch **out) {
    if (!c || !out || (n && !renders)) return fail(SPR_E_INVALID, "null argument");
    *out = nullptr;
    if (n == 0 || n > MAX_REQS) return fail(SPR_E_INVALID, "batch size must be 1..%d", MAX_REQS);
    uint64_t P = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!renders[i] || renders[i]->ctx != c) return fail(SPR_E_INVALID, "render %u is null or from another context", i);
        P += renders[i]->npix;
    }
    spr_batch *b = nullptr;
    CHK(spr_batch_create_empty(c, n, P, &b));
    spr_status st = spr_batch_set(b, n, renders);
    if (st != SPR_OK) {
        spr_batch_free(b);
        return st;
    }
    *out = b;
    return SPR_OK;
}

static spr_status batch_launch(spr_batch *b) {
    spr_ctx *c = b->ctx;
    if (c->prof) CHK(run_pass(c, b->table, b->grids));
    else CHK(graph_pass(c, b->table, b->grids, b->graph, b->exec, b->graph_gen));
    for (auto *r : b->renders) r->started = true;
    b->state_fresh = false;
    return SPR_OK;
}

// Gather every member's progress (one kernel, one copy) into b->h_state.
static spr_status batch_gather(spr_batch *b) {
    spr_ctx *c = b->ctx;
    const uint32_t n = (uint32_t)b->renders.size();
    HIPCHK(launch_gather_state(c->stream, c->ctl, b->table, n, b->d_state));
    HIPCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(uint4) * ((size_t)n + 1), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    b->state_fresh = true;
    return SPR_OK;
}

static spr_status batch_unfinished(spr_batch *b, uint32_t *n_unfinished) {
    CHK(batch_gather(b));
    uint32_t cnt = 0;
    for (size_t i = 0; i < b->renders.size(); ++i) cnt += b->h_state[i].x > 0;
    *n_unfinished = cnt;
    return SPR_OK;
}

spr_status spr_batch_state(spr_batch *b, spr_member_state *out, uint32_t n, uint32_t *active_blocks) {
    if (!b || (n && !out)) return fail(SPR_E_INVALID, "null argument");
    if (n != b->renders.size()) return fail(SPR_E_INVALID, "n = %u, the batch has %zu members", n, b->renders.size());
    HIPCHK(hipSetDevice(b->ctx->device));
    if (!b->state_fresh) CHK(batch_gather(b));
    for (uint32_t i = 0; i < n; ++i) {
        const uint4 v = b->h_state[i];
        out[i].n_active = v.x;
        out[i].passes = v.y;
        out[i].last_pairs = v.z;
        out[i].n_spec = v.w;
    }
    if (active_blocks) *active_blocks = b->h_state[n].x;
    return SPR_OK;
}

spr_status spr_batch_pass(spr_batch *b, uint32_t *n_unfinished) {
    if (!b) return fail(SPR_E_INVALID, "null batch");
    HIPCHK(hipSetDevice(b->ctx->device));
    CHK(batch_launch(b));
    uint32_t n = 0;
    CHK(batch_unfinished(b, &n));
    if (n_unfinished) *n_unfinished = n;
    return SPR_OK;
}

spr_status spr_batch_run(spr_batch *b, uint32_t max_passes, uint32_t poll_every, uint32_t *passes_run) {
    if (!b) return fail(SPR_E_INVALID, "null batch");
    if (poll_every == 0) poll_every = 1;
    HIPCHK(hipSetDevice(b->ctx->device));
    uint32_t n = 0, left = 0;
    CHK(batch_unfinished(b, &left));
    while (left && n < max_passes) {
        for (uint32_t k = 0; k < poll_every && n < max_passes; ++k) {
            CHK(batch_launch(b));
            ++n;
        }
        CHK(batch_unfinished(b, &left));
    }
    if (passes_run) *passes_run = n;
    return SPR_OK;
}

spr_status spr_batch_free(spr_batch *b) {
    if (!b) return fail(SPR_E_INVALID, "null batch");
    spr_ctx *c = b->ctx;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    dev_free(c, MEM_SCRATCH, b->buf, b->buf_bytes);
    b->buf = nullptr;
    if (b->h_state) (void)hipHostFree(b->h_state);
    for (auto *r : b->renders) r->batch = nullptr;
    delete b;
    return SPR_OK;
}

}  // extern "C"
