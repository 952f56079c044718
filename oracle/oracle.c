/*
 * oracle.c — plain, slow, obviously-correct CPU reference for speculative
 * progressive isosurface raycasting of a block-compressed volume
 * (Usher, Dyken, Kumar, arXiv 2309.10212).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only through
 * the compressed stream that the input generator writes.
 *
 * What it computes (each by its plain definition, in fp64):
 *   - block decode of the fixed-rate codec (format version 1, the layout is
 *     written out in the input generator), one bit at a time;
 *   - whole-volume decode;
 *   - block / fine / coarse macrocell value ranges by brute force over the
 *     decoded samples (Sec. 3.1, macrocell grid construction);
 *   - per-pixel camera rays and the volume slab test (Sec. 3.2);
 *   - a march over EVERY dual cell along each ray, in order (no macrocell
 *     skipping), with the exact corner pretest, the trilinear-along-ray cubic
 *     and Marmitt-style root isolation at the cubic's extrema (Sec. 3.7), the
 *     root located by bisection in long double;
 *   - the progressive pass schedule of Sec. 3 and Sec. 4 (speculation count
 *     N_spec = floor(w*h / N_act) capped, visible / active block sets),
 *     derived from each ray's ordered list of candidate blocks;
 *   - the count of blocks whose range contains the isovalue.
 *
 * Parity pins (tests, CPU only): codec special cases and round-trip bounds;
 * the cell walk against a DDA-free box-intersection enumeration; closed-form
 * hits on planes, on (x-a)(y-b)(z-c) (exact cubic roots) and on spheres; the
 * worked speculation example of the traversal figure (6 rays, N_spec = 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_NONE 0xFFFFFFFFu

/* ======================================================== codec decode === */

static int bit_at(const uint32_t *w, uint32_t pos) { return (int)((w[pos >> 5] >> (pos & 31)) & 1u); }

/* Integer arithmetic of the inverse transform is 32-bit two's complement
 * (codec format version 1): sums wrap modulo 2^32; halving rounds toward
 * minus infinity.  Records written by the encoder never wrap (forward
 * coefficients stay below 2^30); the rule only fixes what a decoder returns
 * for any other record. */
static int32_t wrap32(int64_t x) { return (int32_t)(uint32_t)(uint64_t)x; }
static int32_t floor_div2(int32_t x) { return x >= 0 ? x / 2 : -(int32_t)(((uint32_t)(-(int64_t)x) + 1u) / 2u); }

/* coefficient order: positions sorted by lev(x)+lev(y)+lev(z), lev={0,1,2,2},
 * ties by raster index; computed by brute force over the 64 positions */
static void coeff_order(int order[64]) {
    static const int lev[4] = {0, 1, 2, 2};
    int n = 0;
    for (int s = 0; s <= 6; ++s)
        for (int i = 0; i < 64; ++i)
            if (lev[i & 3] + lev[(i >> 2) & 3] + lev[(i >> 4) & 3] == s) order[n++] = i;
}

/* inverse of the 4-point two-level integer S-transform on one line */
static void inv_line(int32_t *p, int stride) {
    int32_t L = p[0], H = p[stride], h0 = p[2 * stride], h1 = p[3 * stride];
    int32_t l1 = wrap32((int64_t)L - floor_div2(H));
    int32_t l0 = wrap32((int64_t)l1 + H);
    int32_t a1 = wrap32((int64_t)l0 - floor_div2(h0));
    int32_t a0 = wrap32((int64_t)a1 + h0);
    int32_t a3 = wrap32((int64_t)l1 - floor_div2(h1));
    int32_t a2 = wrap32((int64_t)a3 + h1);
    p[0] = a0; p[stride] = a1; p[2 * stride] = a2; p[3 * stride] = a3;
}

/* Decode one block record of 64*R bits into 64 raster-order floats. */
int orc_decode_block(const uint32_t *rec, int R, float *out) {
    if (!rec || !out) return ORC_EINVAL;
    if (R == 32) { memcpy(out, rec, 256); return ORC_OK; }
    if (R < 1 || R > 16) return ORC_EINVAL;
    const uint32_t B = 64u * (uint32_t)R;
    if (!bit_at(rec, 0)) { for (int i = 0; i < 64; ++i) out[i] = 0.0f; return ORC_OK; }
    int E = 0;
    for (int i = 0; i < 8; ++i) E |= bit_at(rec, 1 + i) << i;
    int e = E - 127;
    uint32_t pos = 9;
    uint32_t mag[64] = {0};
    int neg[64] = {0}, sig[64] = {0};
    for (int k = 29; k >= 0; --k) {
        /* refinement: one bit per coefficient that was significant before this plane */
        for (int j = 0; j < 64; ++j) {
            if (!sig[j]) continue;
            if (pos == B) goto done;
            if (bit_at(rec, pos)) mag[j] |= 1u << k;
            pos++;
        }
        /* significance: group tests over insignificant coefficients from cursor c */
        int c = 0;
        for (;;) {
            int any = 0;
            for (int j = c; j < 64; ++j) if (!sig[j]) { any = 1; break; }
            if (!any) break;
            if (pos == B) goto done;
            int g = bit_at(rec, pos++);
            if (!g) break;
            int target = -1;
            for (int j = c; j < 64; ++j) {
                if (sig[j]) continue;
                if (pos == B) goto done;
                int b = bit_at(rec, pos++);
                if (b) { target = j; break; }
            }
            if (target < 0) goto done;
            if (pos == B) goto done;
            neg[target] = bit_at(rec, pos++);
            mag[target] |= 1u << k;
            sig[target] = 1;
            c = target + 1;
        }
    }
done:;
    int order[64];
    coeff_order(order);
    int32_t q[64];
    for (int j = 0; j < 64; ++j) q[order[j]] = neg[j] ? -(int32_t)mag[j] : (int32_t)mag[j];   /* mag < 2^30 */
    for (int y = 0; y < 4; ++y) for (int x = 0; x < 4; ++x) inv_line(q + x + 4 * y, 16); /* z */
    for (int z = 0; z < 4; ++z) for (int x = 0; x < 4; ++x) inv_line(q + x + 16 * z, 4); /* y */
    for (int z = 0; z < 4; ++z) for (int y = 0; y < 4; ++y) inv_line(q + 4 * y + 16 * z, 1); /* x */
    for (int i = 0; i < 64; ++i) out[i] = (float)ldexp((double)q[i], e - 27);
    return ORC_OK;
}

static long nblk_axis(int n) { return (n + 3) / 4; }

/* Decode the listed blocks: out[i*64 .. i*64+63] = block ids[i]. */
int orc_decode_blocks(const void *stream, size_t bytes, int nx, int ny, int nz, int R,
                      const uint32_t *ids, size_t n, float *out) {
    if (!stream || !ids || !out) return ORC_EINVAL;
    size_t nb = (size_t)nblk_axis(nx) * nblk_axis(ny) * nblk_axis(nz);
    if (bytes != nb * 8u * (size_t)R) return ORC_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (ids[i] >= nb) return ORC_EINVAL;
        int rc = orc_decode_block((const uint32_t *)stream + (size_t)ids[i] * 2u * (size_t)R, R, out + 64 * i);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* Decode the whole volume into nx*ny*nz floats (x fastest). */
int orc_decode_volume(const void *stream, size_t bytes, int nx, int ny, int nz, int R, float *out) {
    if (!stream || !out || nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    if (!((R >= 1 && R <= 16) || R == 32)) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    if (bytes != (size_t)nbx * nby * nbz * 8u * (size_t)R) return ORC_EINVAL;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (long b = 0; b < nbx * nby * nbz; ++b) {
        float v[64];
        if (orc_decode_block((const uint32_t *)stream + (size_t)b * 2u * (size_t)R, R, v)) { err = 1; continue; }
        long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) {
                    long x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                    if (x < nx && y < ny && z < nz) out[(z * ny + y) * nx + x] = v[i + 4 * j + 16 * k];
                }
    }
    return err ? ORC_EINVAL : ORC_OK;
}

/* ============================================== macrocell value ranges === */

/* block_lohi[2*b]   : min/max over block b's samples inside the volume
 * fine_lohi[2*b]    : union over blocks b + {0,1}^3 that exist
 * coarse_lohi[2*c]  : union of fine ranges over blocks 4c .. 4c+3 that exist
 * (Sec. 3.1: a cell's range is its own range combined with its +x/+y/+z
 * neighbours, so the dual grid's values are covered).  Any output may be NULL. */
/* fine and coarse ranges from the block ranges (any output may be NULL) */
static void grids_from_blocks(const float *blk, long nbx, long nby, long nbz, float *fin, float *coarse_lohi) {
    if (fin) {
#pragma omp parallel for schedule(static)
        for (long bz = 0; bz < nbz; ++bz)
            for (long by = 0; by < nby; ++by)
                for (long bx = 0; bx < nbx; ++bx) {
                    float lo = INFINITY, hi = -INFINITY;
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx) {
                                long x = bx + dx, y = by + dy, z = bz + dz;
                                if (x >= nbx || y >= nby || z >= nbz) continue;
                                size_t o = (size_t)((z * nby + y) * nbx + x);
                                if (blk[2 * o] < lo) lo = blk[2 * o];
                                if (blk[2 * o + 1] > hi) hi = blk[2 * o + 1];
                            }
                    size_t b = (size_t)((bz * nby + by) * nbx + bx);
                    fin[2 * b] = lo; fin[2 * b + 1] = hi;
                }
    }
    if (coarse_lohi && fin) {
        long ncx = (nbx + 3) / 4, ncy = (nby + 3) / 4, ncz = (nbz + 3) / 4;
#pragma omp parallel for schedule(static)
        for (long cz = 0; cz < ncz; ++cz)
            for (long cy = 0; cy < ncy; ++cy)
                for (long cx = 0; cx < ncx; ++cx) {
                    float lo = INFINITY, hi = -INFINITY;
                    for (long z = 4 * cz; z < 4 * cz + 4 && z < nbz; ++z)
                        for (long y = 4 * cy; y < 4 * cy + 4 && y < nby; ++y)
                            for (long x = 4 * cx; x < 4 * cx + 4 && x < nbx; ++x) {
                                size_t o = (size_t)((z * nby + y) * nbx + x);
                                if (fin[2 * o] < lo) lo = fin[2 * o];
                                if (fin[2 * o + 1] > hi) hi = fin[2 * o + 1];
                            }
                    size_t c = (size_t)((cz * ncy + cy) * ncx + cx);
                    coarse_lohi[2 * c] = lo; coarse_lohi[2 * c + 1] = hi;
                }
    }
}

int orc_grids(const float *vol, int nx, int ny, int nz, float *block_lohi, float *fine_lohi,
              float *coarse_lohi) {
    if (!vol || nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    size_t nb = (size_t)nbx * nby * nbz;
    float *blk = (float *)malloc(sizeof(float) * 2 * nb);
    float *fin = (float *)malloc(sizeof(float) * 2 * nb);
    if (!blk || !fin) { free(blk); free(fin); return ORC_ENOMEM; }
    for (long bz = 0; bz < nbz; ++bz)
        for (long by = 0; by < nby; ++by)
            for (long bx = 0; bx < nbx; ++bx) {
                float lo = INFINITY, hi = -INFINITY;
                for (long z = 4 * bz; z < 4 * bz + 4 && z < nz; ++z)
                    for (long y = 4 * by; y < 4 * by + 4 && y < ny; ++y)
                        for (long x = 4 * bx; x < 4 * bx + 4 && x < nx; ++x) {
                            float v = vol[(z * ny + y) * nx + x];
                            if (v < lo) lo = v;
                            if (v > hi) hi = v;
                        }
                size_t b = (size_t)((bz * nby + by) * nbx + bx);
                blk[2 * b] = lo; blk[2 * b + 1] = hi;
            }
    grids_from_blocks(blk, nbx, nby, nbz, fin, coarse_lohi);
    if (block_lohi) memcpy(block_lohi, blk, sizeof(float) * 2 * nb);
    if (fine_lohi) memcpy(fine_lohi, fin, sizeof(float) * 2 * nb);
    free(blk); free(fin);
    return ORC_OK;
}

/* Block ranges straight from the compressed stream, one block decoded at a
 * time (no whole-volume buffer): min/max over each block's samples inside
 * the volume, the block_lohi of orc_grids. */
int orc_block_ranges_stream(const void *stream, size_t bytes, int nx, int ny, int nz, int R, float *block_lohi) {
    if (!stream || !block_lohi || nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    if (!((R >= 1 && R <= 16) || R == 32)) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    if (bytes != (size_t)nbx * nby * nbz * 8u * (size_t)R) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 4096)
    for (long b = 0; b < nbx * nby * nbz; ++b) {
        float v[64];
        orc_decode_block((const uint32_t *)stream + (size_t)b * 2u * (size_t)R, R, v);
        long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        float lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < 4 && 4 * bz + k < nz; ++k)
            for (int j = 0; j < 4 && 4 * by + j < ny; ++j)
                for (int i = 0; i < 4 && 4 * bx + i < nx; ++i) {
                    float x = v[i + 4 * j + 16 * k];
                    if (x < lo) lo = x;
                    if (x > hi) hi = x;
                }
        block_lohi[2 * b] = lo; block_lohi[2 * b + 1] = hi;
    }
    return ORC_OK;
}

/* Fine and coarse ranges from given block ranges (as orc_grids computes them
 * from the decoded volume).  Either output may be NULL. */
int orc_grids_from_blocks(const float *block_lohi, int nx, int ny, int nz, float *fine_lohi, float *coarse_lohi) {
    if (!block_lohi || nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    float *fin = fine_lohi;
    if (!fin) {
        fin = (float *)malloc(sizeof(float) * 2 * (size_t)nbx * nby * nbz);
        if (!fin) return ORC_ENOMEM;
    }
    grids_from_blocks(block_lohi, nbx, nby, nbz, fin, coarse_lohi);
    if (fin != fine_lohi) free(fin);
    return ORC_OK;
}

/* ================================================================ rays === */

typedef struct {
    double eye[3], center[3], up[3];
    double vfov_deg;
} orc_camera;

typedef struct {
    double eye[3], fwd[3], right[3], upv[3];
    double sx, sy;
    int w, h;
} cam_basis;

typedef struct {
    double o[3], d[3], r[3];
    double t_enter, t_exit;
    int n[3];
    int hit_volume;
} ray_t;

static int make_basis(const orc_camera *c, int w, int h, cam_basis *b) {
    double f[3] = {c->center[0] - c->eye[0], c->center[1] - c->eye[1], c->center[2] - c->eye[2]};
    double fl = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    if (!(fl > 0)) return ORC_EINVAL;
    double inv = 1.0 / fl;
    for (int a = 0; a < 3; ++a) b->fwd[a] = f[a] * inv;
    double r[3] = {b->fwd[1] * c->up[2] - b->fwd[2] * c->up[1],
                   b->fwd[2] * c->up[0] - b->fwd[0] * c->up[2],
                   b->fwd[0] * c->up[1] - b->fwd[1] * c->up[0]};
    double rl = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    if (!(rl > 0)) return ORC_EINVAL;
    inv = 1.0 / rl;
    for (int a = 0; a < 3; ++a) b->right[a] = r[a] * inv;
    b->upv[0] = b->right[1] * b->fwd[2] - b->right[2] * b->fwd[1];
    b->upv[1] = b->right[2] * b->fwd[0] - b->right[0] * b->fwd[2];
    b->upv[2] = b->right[0] * b->fwd[1] - b->right[1] * b->fwd[0];
    double th = tan((c->vfov_deg * 0.5) * (3.14159265358979323846 / 180.0));
    b->sx = th * ((double)w / (double)h);
    b->sy = th;
    for (int a = 0; a < 3; ++a) b->eye[a] = c->eye[a];
    b->w = w; b->h = h;
    return ORC_OK;
}

/* tau_a(m): parameter at which the ray crosses the plane x_a = m */
static double tau(const ray_t *ray, int a, long m) { return ((double)m - ray->o[a]) * ray->r[a]; }

static void make_ray(const cam_basis *b, int nx, int ny, int nz, int px, int py, ray_t *ray) {
    double ndx = (2.0 * ((double)px + 0.5)) / (double)b->w - 1.0;
    double ndy = 1.0 - (2.0 * ((double)py + 0.5)) / (double)b->h;
    double x = ndx * b->sx, y = ndy * b->sy;
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = (b->fwd[a] + x * b->right[a]) + y * b->upv[a];
    double inv = 1.0 / sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    ray->n[0] = nx; ray->n[1] = ny; ray->n[2] = nz;
    for (int a = 0; a < 3; ++a) {
        ray->o[a] = b->eye[a];
        ray->d[a] = v[a] * inv;
        if (fabs(ray->d[a]) < 1e-290) ray->d[a] = 0.0;   /* treated as parallel to the axis */
        ray->r[a] = ray->d[a] != 0.0 ? 1.0 / ray->d[a] : 0.0;
    }
    /* slab test against the sample domain [0, n-1]^3 */
    double te = 0.0, tx = INFINITY;
    ray->hit_volume = 1;
    for (int a = 0; a < 3; ++a) {
        double nearp, farp;
        if (ray->d[a] > 0) { nearp = tau(ray, a, 0); farp = tau(ray, a, ray->n[a] - 1); }
        else if (ray->d[a] < 0) { nearp = tau(ray, a, ray->n[a] - 1); farp = tau(ray, a, 0); }
        else {
            if (ray->o[a] < 0.0 || ray->o[a] > (double)(ray->n[a] - 1)) ray->hit_volume = 0;
            continue;
        }
        if (nearp > te) te = nearp;
        if (farp < tx) tx = farp;
    }
    if (te > tx) ray->hit_volume = 0;
    ray->t_enter = te;
    ray->t_exit = tx;
}

/* ============================================================ cell walk === */

/* Dual cell containing the ray at parameter t on axis a: for d > 0 the
 * largest m in [0, n-2] whose lower plane is crossed (tau(m) <= t); for d < 0
 * the smallest m whose upper plane m+1 is crossed; for d == 0 the cell of the
 * origin. */
static long cell_at(const ray_t *ray, int a, double t) {
    long n2 = ray->n[a] - 2;
    if (ray->d[a] > 0) {
        long m = 0;
        while (m + 1 <= n2 && tau(ray, a, m + 1) <= t) ++m;
        return m;
    } else if (ray->d[a] < 0) {
        long m = n2;
        while (m - 1 >= 0 && tau(ray, a, m) <= t) --m;
        return m;
    } else {
        double f = floor(ray->o[a]);
        long m = (long)f;
        if (m < 0) m = 0;
        if (m > n2) m = n2;
        return m;
    }
}

static void cell_interval(const ray_t *ray, const long c[3], double *t0, double *t1) {
    double a0 = ray->t_enter, a1 = ray->t_exit;
    for (int a = 0; a < 3; ++a) {
        if (ray->d[a] > 0) {
            double e = tau(ray, a, c[a]), x = tau(ray, a, c[a] + 1);
            if (e > a0) a0 = e;
            if (x < a1) a1 = x;
        } else if (ray->d[a] < 0) {
            double e = tau(ray, a, c[a] + 1), x = tau(ray, a, c[a]);
            if (e > a0) a0 = e;
            if (x < a1) a1 = x;
        }
    }
    *t0 = a0; *t1 = a1;
}

/* Advance to the next cell: cross every plane whose parameter is <= the
 * nearest exit-plane parameter (tied planes are crossed together).  Returns 0
 * when the ray leaves the volume. */
static int next_cell(const ray_t *ray, long c[3]) {
    double tn = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (ray->d[a] > 0) { double x = tau(ray, a, c[a] + 1); if (x < tn) tn = x; }
        else if (ray->d[a] < 0) { double x = tau(ray, a, c[a]); if (x < tn) tn = x; }
    }
    if (tn > ray->t_exit) return 0;
    for (int a = 0; a < 3; ++a) {
        if (ray->d[a] > 0) {
            while (tau(ray, a, c[a] + 1) <= tn) {
                c[a]++;
                if (c[a] > ray->n[a] - 2) return 0;
            }
        } else if (ray->d[a] < 0) {
            while (tau(ray, a, c[a]) <= tn) {
                c[a]--;
                if (c[a] < 0) return 0;
            }
        }
    }
    return 1;
}

/* ============================================== cell test (Sec. 3.7) === */

static double horner(double A, double B, double C, double D, double s) {
    return ((A * s + B) * s + C) * s + D;
}

static long double horner_l(double A, double B, double C, double D, long double s) {
    return (((long double)A * s + B) * s + C) * s + D;
}

/* Root of the cubic inside the bracket (sa, sb) whose end values have strictly
 * opposite signs; exactly one root lies there because the bracket is a
 * monotone piece between consecutive extrema.  Bisection in long double. */
static double bisect_root(double A, double B, double C, double D, double sa, double sb) {
    long double a = sa, b = sb;
    long double ga = horner_l(A, B, C, D, a);
    for (int it = 0; it < 200 && (b - a) > 1e-15L; ++it) {
        long double m = 0.5L * (a + b);
        long double gm = horner_l(A, B, C, D, m);
        if (gm == 0.0L) return (double)m;
        if ((gm < 0) == (ga < 0)) { a = m; ga = gm; }
        else b = m;
    }
    return (double)(0.5L * (a + b));
}

typedef struct {
    int hit;
    double s;                       /* hit offset from t0 */
    double u0, v0, w0;              /* local entry coordinates */
    double c[8];                    /* corner values, a fastest */
} cell_result;

/* Test the dual cell c along [t0, t1]; fc[a + 2b + 4g] is the sample at
 * (c0+a, c1+b, c2+g). */
static void test_cell(const float fc[8], const ray_t *ray, const long c[3], double t0, double t1,
                      float iso, cell_result *res) {
    res->hit = 0;
    int above = 0, below = 0;
    for (int i = 0; i < 8; ++i) {
        if (fc[i] > iso) above++;
        if (fc[i] < iso) below++;
    }
    if (above == 8 || below == 8) return;   /* exact pretest: no crossing possible */
    if (t1 < t0) return;
    double S = t1 - t0;
    double loc[3];
    for (int a = 0; a < 3; ++a) loc[a] = (ray->o[a] + t0 * ray->d[a]) - (double)c[a];
    /* factors along the ray: X0(s) = (1-u0) - s dx, X1(s) = u0 + s dx */
    double al[3][2], be[3][2];
    for (int a = 0; a < 3; ++a) {
        al[a][0] = 1.0 - loc[a]; be[a][0] = -ray->d[a];
        al[a][1] = loc[a];       be[a][1] = ray->d[a];
    }
    double A = 0.0, Bc = 0.0, Cc = 0.0, D = 0.0;
    for (int i = 0; i < 8; ++i) {
        int a = i & 1, b = (i >> 1) & 1, g = (i >> 2) & 1;
        double ax = al[0][a], bx = be[0][a], ay = al[1][b], by = be[1][b], az = al[2][g], bz = be[2][g];
        double td = (ax * ay) * az;
        double tc = ((bx * ay) * az + (ax * by) * az) + (ax * ay) * bz;
        double tb = ((bx * by) * az + (bx * ay) * bz) + (ax * by) * bz;
        double ta = (bx * by) * bz;
        double cv = (double)fc[i];
        D = D + cv * td;
        Cc = Cc + cv * tc;
        Bc = Bc + cv * tb;
        A = A + cv * ta;
        res->c[i] = cv;
    }
    D = D - (double)iso;
    /* extrema: roots of 3A s^2 + 2B s + C inside (0, S) */
    double cand[2];
    int nc = 0;
    if (A != 0.0) {
        double disc = Bc * Bc - (3.0 * A) * Cc;
        if (disc >= 0.0) {
            double q = -(Bc + copysign(sqrt(disc), Bc));
            cand[nc++] = q / (3.0 * A);
            if (q != 0.0) cand[nc++] = Cc / q;
        }
    } else if (Bc != 0.0) {
        cand[nc++] = -Cc / (2.0 * Bc);
    }
    double pts[4];
    int np = 0;
    pts[np++] = 0.0;
    double ext[2];
    int ne = 0;
    for (int i = 0; i < nc; ++i)
        if (cand[i] > 0.0 && cand[i] < S) ext[ne++] = cand[i];
    if (ne == 2 && ext[1] < ext[0]) { double tmp = ext[0]; ext[0] = ext[1]; ext[1] = tmp; }
    if (ne == 2 && ext[1] == ext[0]) ne = 1;
    for (int i = 0; i < ne; ++i) pts[np++] = ext[i];
    pts[np++] = S;
    double gprev = horner(A, Bc, Cc, D, pts[0]);
    res->u0 = loc[0]; res->v0 = loc[1]; res->w0 = loc[2];
    if (gprev == 0.0) { res->hit = 1; res->s = pts[0]; return; }
    for (int i = 1; i < np; ++i) {
        double gi = horner(A, Bc, Cc, D, pts[i]);
        if ((gprev < 0.0 && gi > 0.0) || (gprev > 0.0 && gi < 0.0)) {
            res->hit = 1;
            res->s = bisect_root(A, Bc, Cc, D, pts[i - 1], pts[i]);
            return;
        }
        if (gi == 0.0) { res->hit = 1; res->s = pts[i]; return; }
        gprev = gi;
    }
}

/* Headlight Lambertian shading of the hit, packed RGBA8 (r in the low byte). */
static uint32_t shade(const ray_t *ray, const cell_result *r) {
    double u = r->u0 + r->s * ray->d[0], v = r->v0 + r->s * ray->d[1], w = r->w0 + r->s * ray->d[2];
    double U0 = 1.0 - u, U1 = u, V0 = 1.0 - v, V1 = v, W0 = 1.0 - w, W1 = w;
    const double *c = r->c;
    double gx = ((c[1] - c[0]) * V0 + (c[3] - c[2]) * V1) * W0 + ((c[5] - c[4]) * V0 + (c[7] - c[6]) * V1) * W1;
    double gy = ((c[2] - c[0]) * U0 + (c[3] - c[1]) * U1) * W0 + ((c[6] - c[4]) * U0 + (c[7] - c[5]) * U1) * W1;
    double gz = ((c[4] - c[0]) * U0 + (c[5] - c[1]) * U1) * V0 + ((c[6] - c[2]) * U0 + (c[7] - c[3]) * U1) * V1;
    double len = sqrt((gx * gx + gy * gy) + gz * gz);
    double nd = len > 0.0 ? fabs((gx * ray->d[0] + gy * ray->d[1]) + gz * ray->d[2]) / len : 1.0;
    double k = 0.15 + 0.85 * nd;
    static const double base[3] = {0.90, 0.75, 0.40};
    uint32_t out = 0xFF000000u;
    for (int ch = 0; ch < 3; ++ch) {
        double x = floor(255.0 * (base[ch] * k) + 0.5);
        if (x < 0) x = 0;
        if (x > 255) x = 255;
        out |= (uint32_t)x << (8 * ch);
    }
    return out;
}

/* ============================================================= render === */

typedef struct {
    double t;
    uint32_t block, cell, rgba;
    int entered;
} pixel_result;

/* Where a march reads a dual cell's 8 corner samples: the whole decoded
 * volume, or blocks decoded on demand from the compressed stream (for
 * volumes too large to decode whole). */
typedef struct corner_src {
    void (*fetch)(struct corner_src *src, const long c[3], float fc[8]);
} corner_src;

typedef struct {
    corner_src base;
    const float *vol;
    long nx, ny;
} flat_src;

static void flat_fetch(corner_src *src, const long c[3], float fc[8]) {
    const flat_src *f = (const flat_src *)src;
    for (int g = 0; g < 2; ++g)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                fc[a + 2 * b + 4 * g] = f->vol[((c[2] + g) * f->ny + (c[1] + b)) * f->nx + (c[0] + a)];
}

#define LAZY_SLOTS 64
typedef struct {
    corner_src base;
    const uint32_t *stream;
    int R;
    long nbx, nby;
    size_t rec_words;
    long tag[LAZY_SLOTS];            /* block id held by each slot, -1 = empty */
    float val[LAZY_SLOTS][64];
} lazy_src;

/* sample (x, y, z): its block decoded into a direct-mapped slot on first use */
static float lazy_sample(lazy_src *L, long x, long y, long z) {
    long b = (x >> 2) + L->nbx * ((y >> 2) + L->nby * (z >> 2));
    int s = (int)(b % LAZY_SLOTS);
    if (L->tag[s] != b) {
        orc_decode_block(L->stream + (size_t)b * L->rec_words, L->R, L->val[s]);
        L->tag[s] = b;
    }
    return L->val[s][(x & 3) + 4 * (y & 3) + 16 * (z & 3)];
}

static void lazy_fetch(corner_src *src, const long c[3], float fc[8]) {
    lazy_src *L = (lazy_src *)src;
    for (int g = 0; g < 2; ++g)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) fc[a + 2 * b + 4 * g] = lazy_sample(L, c[0] + a, c[1] + b, c[2] + g);
}

static void trace_pixel(corner_src *src, int nx, int ny, int nz, const cam_basis *cb, float iso,
                        int px, int py, pixel_result *out) {
    ray_t ray;
    make_ray(cb, nx, ny, nz, px, py, &ray);
    out->t = INFINITY; out->block = ORC_NONE; out->cell = ORC_NONE; out->rgba = 0; out->entered = 0;
    if (!ray.hit_volume) return;
    out->entered = 1;
    long c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_at(&ray, a, ray.t_enter);
    long nbx = nblk_axis(nx), nby = nblk_axis(ny);
    do {
        double t0, t1;
        cell_interval(&ray, c, &t0, &t1);
        cell_result r;
        float fc[8];
        src->fetch(src, c, fc);
        test_cell(fc, &ray, c, t0, t1, iso, &r);
        if (r.hit) {
            out->t = t0 + r.s;
            out->block = (uint32_t)((c[0] >> 2) + nbx * ((c[1] >> 2) + nby * (c[2] >> 2)));
            out->cell = (uint32_t)((c[0] & 3) + 4 * (c[1] & 3) + 16 * (c[2] & 3));
            out->rgba = shade(&ray, &r);
            return;
        }
    } while (next_cell(&ray, c));
}

/* Render pixels.  pix = NULL renders all w*h pixels in raster order (py*w+px);
 * otherwise pix[i] is a raster pixel index.  Outputs are per listed pixel. */
int orc_render(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
               const uint32_t *pix, size_t npix, double *t_out, uint32_t *block_out, uint32_t *cell_out,
               uint32_t *rgba_out, uint8_t *entered_out) {
    if (!vol || !cam || w < 1 || h < 1 || nx < 2 || ny < 2 || nz < 2) return ORC_EINVAL;
    cam_basis cb;
    if (make_basis(cam, w, h, &cb)) return ORC_EINVAL;
    size_t n = pix ? npix : (size_t)w * h;
    if (pix)
        for (size_t i = 0; i < n; ++i)
            if (pix[i] >= (uint32_t)w * (uint32_t)h) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < (long)n; ++i) {
        uint32_t p = pix ? pix[i] : (uint32_t)i;
        pixel_result r;
        flat_src src = {{flat_fetch}, vol, nx, ny};
        trace_pixel(&src.base, nx, ny, nz, &cb, iso, (int)(p % (uint32_t)w), (int)(p / (uint32_t)w), &r);
        if (t_out) t_out[i] = r.t;
        if (block_out) block_out[i] = r.block;
        if (cell_out) cell_out[i] = r.cell;
        if (rgba_out) rgba_out[i] = r.rgba;
        if (entered_out) entered_out[i] = (uint8_t)r.entered;
    }
    return ORC_OK;
}

/* orc_render for a volume given only as its compressed stream (format of
 * orc_decode_block): the same march, reading each corner from its block
 * decoded on demand.  For sampled parity on volumes too large to decode
 * whole; results equal orc_render on the decoded volume. */
int orc_render_stream(const void *stream, size_t bytes, int nx, int ny, int nz, int R, const orc_camera *cam,
                      float iso, int w, int h, const uint32_t *pix, size_t npix, double *t_out,
                      uint32_t *block_out, uint32_t *cell_out, uint32_t *rgba_out, uint8_t *entered_out) {
    if (!stream || !cam || w < 1 || h < 1 || nx < 2 || ny < 2 || nz < 2) return ORC_EINVAL;
    if (!((R >= 1 && R <= 16) || R == 32)) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    if (bytes != (size_t)nbx * nby * nbz * 8u * (size_t)R) return ORC_EINVAL;
    cam_basis cb;
    if (make_basis(cam, w, h, &cb)) return ORC_EINVAL;
    size_t n = pix ? npix : (size_t)w * h;
    if (pix)
        for (size_t i = 0; i < n; ++i)
            if (pix[i] >= (uint32_t)w * (uint32_t)h) return ORC_EINVAL;
#pragma omp parallel
    {
        lazy_src *L = (lazy_src *)malloc(sizeof(lazy_src));
        if (L) {
            L->base.fetch = lazy_fetch;
            L->stream = (const uint32_t *)stream;
            L->R = R;
            L->nbx = nbx; L->nby = nby;
            L->rec_words = 2u * (size_t)R;
            for (int k = 0; k < LAZY_SLOTS; ++k) L->tag[k] = -1;
        }
#pragma omp for schedule(dynamic, 4)
        for (long i = 0; i < (long)n; ++i) {
            uint32_t p = pix ? pix[i] : (uint32_t)i;
            pixel_result r = {INFINITY, ORC_NONE, ORC_NONE, 0, 0};
            if (L) trace_pixel(&L->base, nx, ny, nz, &cb, iso, (int)(p % (uint32_t)w), (int)(p / (uint32_t)w), &r);
            if (t_out) t_out[i] = L ? r.t : NAN;
            if (block_out) block_out[i] = r.block;
            if (cell_out) cell_out[i] = r.cell;
            if (rgba_out) rgba_out[i] = r.rgba;
            if (entered_out) entered_out[i] = (uint8_t)r.entered;
        }
        free(L);
    }
    return ORC_OK;
}

/* The ordered dual-cell walk of one pixel's ray: cells (x,y,z) and their
 * [t0,t1].  Returns the number of cells (may exceed cap; only cap stored), or
 * -1 when the ray misses the volume. */
long orc_cell_walk(int nx, int ny, int nz, const orc_camera *cam, int w, int h, int px, int py,
                   int32_t *cells, double *t01, long cap, double *t_enter_exit) {
    cam_basis cb;
    if (!cam || make_basis(cam, w, h, &cb)) return -2;
    ray_t ray;
    make_ray(&cb, nx, ny, nz, px, py, &ray);
    if (t_enter_exit) { t_enter_exit[0] = ray.t_enter; t_enter_exit[1] = ray.t_exit; }
    if (!ray.hit_volume) return -1;
    long c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_at(&ray, a, ray.t_enter);
    long k = 0;
    do {
        if (k < cap) {
            double t0, t1;
            cell_interval(&ray, c, &t0, &t1);
            if (cells) { cells[3 * k] = (int32_t)c[0]; cells[3 * k + 1] = (int32_t)c[1]; cells[3 * k + 2] = (int32_t)c[2]; }
            if (t01) { t01[2 * k] = t0; t01[2 * k + 1] = t1; }
        }
        ++k;
    } while (next_cell(&ray, c));
    return k;
}

/* Per-pixel ray direction and entry/exit parameters (d[3], t_enter, t_exit,
 * entered) for tests of the camera model. */
int orc_ray(int nx, int ny, int nz, const orc_camera *cam, int w, int h, int px, int py, double *out6) {
    cam_basis cb;
    if (!cam || !out6 || make_basis(cam, w, h, &cb)) return ORC_EINVAL;
    ray_t ray;
    make_ray(&cb, nx, ny, nz, px, py, &ray);
    out6[0] = ray.d[0]; out6[1] = ray.d[1]; out6[2] = ray.d[2];
    out6[3] = ray.t_enter; out6[4] = ray.t_exit; out6[5] = ray.hit_volume;
    return ORC_OK;
}

/* ====================================================== pass schedule === */

/* Speculation count of Sec. 4: N_spec = floor(w*h / N_act), capped at cap and
 * at least 1. */
uint32_t orc_nspec(uint64_t slots, uint64_t n_act, uint32_t cap) {
    if (n_act == 0) return 0;
    uint64_t s = slots / n_act;
    if (s < 1) s = 1;
    if (s > cap) s = cap;
    return (uint32_t)s;
}

/* Per-ray speculation counts (the per-ray count that the paper's conclusion
 * names as future work, in place of Sec. 4's single count for all rays).
 * This build's reading: a ray's weight is its remaining path in block
 * lengths, w = 1 + floor((t_exit - t) / 4) (w = 1 once t >= t_exit), where t
 * is where its remaining walk starts: the volume entry for a ray not yet
 * started, else the parameter where it leaves its last served block.  With
 * B = w*h slots, N active rays and W the sum of their weights, ray i gets
 * n_i = min(cap, 1 + floor((B - N) * w_i / W)).  Every ray gets at least one
 * slot, the counts sum to at most B, and equal weights give floor(B / N),
 * Sec. 4's count. */
uint32_t orc_ray_weight(double t, double t_exit) {
    if (!(t < t_exit)) return 1u;
    return 1u + (uint32_t)floor((t_exit - t) * 0.25);
}

uint32_t orc_nspec_ray(uint64_t slots, uint64_t n_act, uint64_t wsum, uint32_t w, uint32_t cap) {
    if (n_act == 0 || wsum == 0) return 0;
    uint64_t extra = slots > n_act ? ((slots - n_act) * (uint64_t)w) / wsum : 0;
    uint64_t s = 1 + extra;
    if (s > cap) s = cap;
    return (uint32_t)s;
}

/* Parameter where the ray leaves block (bx,by,bz): the nearest of its exit
 * planes at block level, where block plane m sits at sample 4m except the
 * last one of an axis, which is the domain face n-1. */
static double block_exit_tau(const ray_t *ray, long bx, long by, long bz) {
    const long b[3] = {bx, by, bz};
    double tn = INFINITY;
    for (int a = 0; a < 3; ++a) {
        long nplanes = (ray->n[a] - 1 + 3) / 4;   /* blocks that own dual cells on this axis */
        long m;
        if (ray->d[a] > 0) m = b[a] + 1;
        else if (ray->d[a] < 0) m = b[a];
        else continue;
        long pos = m >= nplanes ? ray->n[a] - 1 : 4 * m;
        double x = tau(ray, a, pos);
        if (x < tn) tn = x;
    }
    return tn;
}

/* Candidate blocks of one ray: the distinct blocks of its dual-cell walk, in
 * walk order, whose fine range contains iso (Sec. 3.3: blocks whose combined
 * range does not contain the isovalue are skipped).  hit_idx = position of the
 * block holding the first hit cell, or -1. */
static long ray_candidates(const float *vol, const float *fine, int nx, int ny, int nz, const cam_basis *cb,
                           float iso, int px, int py, uint32_t **list, uint32_t **wlist, long *cap, long *hit_idx,
                           int *entered, uint32_t *w0) {
    ray_t ray;
    make_ray(cb, nx, ny, nz, px, py, &ray);
    *hit_idx = -1;
    *entered = ray.hit_volume;
    *w0 = ray.hit_volume ? orc_ray_weight(ray.t_enter, ray.t_exit) : 0u;
    if (!ray.hit_volume) return 0;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny);
    long c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_at(&ray, a, ray.t_enter);
    long n = 0;
    uint32_t last = ORC_NONE;
    int found_hit = 0;
    do {
        uint32_t b = (uint32_t)((c[0] >> 2) + nbx * ((c[1] >> 2) + nby * (c[2] >> 2)));
        if (b != last) {
            last = b;
            if (fine[2 * b] <= iso && iso <= fine[2 * b + 1]) {
                if (n == *cap) {
                    *cap = *cap ? 2 * *cap : 64;
                    *list = (uint32_t *)realloc(*list, sizeof(uint32_t) * (size_t)*cap);
                    *wlist = (uint32_t *)realloc(*wlist, sizeof(uint32_t) * (size_t)*cap);
                }
                /* the weight of a ray that resumes after this block */
                (*wlist)[n] = orc_ray_weight(block_exit_tau(&ray, c[0] >> 2, c[1] >> 2, c[2] >> 2), ray.t_exit);
                (*list)[n++] = b;
            }
        }
        if (!found_hit) {
            double t0, t1;
            cell_interval(&ray, c, &t0, &t1);
            cell_result r;
            flat_src src = {{flat_fetch}, vol, nx, ny};
            float fc[8];
            flat_fetch(&src.base, c, fc);
            test_cell(fc, &ray, c, t0, t1, iso, &r);
            if (r.hit) { found_hit = 1; *hit_idx = n - 1; }
        }
    } while (next_cell(&ray, c));
    return n;
}

/* Simulate the progressive passes (Sec. 3, Sec. 4) without a cache limit,
 * from each ray's ordered candidate-block list.  slots = w*h (the virtual GPU
 * of Sec. 4).  Ray i's list is lists[off[i] .. off[i+1]); hit[i] is the index
 * in it of the block holding the first hit (or -1); entered[i] says whether the
 * ray entered the volume.  Each pass: every active ray gets a speculation
 * count, takes its next that many candidates, and terminates if its hit block
 * is among them or if it got fewer than its count (it left the volume).
 * policy 0: one count for all rays, N_spec from the active-ray count (Sec. 4).
 * policy 1: per-ray counts (orc_nspec_ray) from weights: w0[i] before the
 * ray's first candidate, wk[off[i] + k] once it has been served candidate k
 * (w0 and wk may be NULL for policy 0).
 * Per pass p: stats[8*p ..] = {n_active, n_spec (the largest count), pairs,
 * visible blocks, active blocks (visible plus existing +x/+y/+z face, edge
 * and corner neighbours in the nbx*nby*nbz block grid), rays terminated,
 * slots (the sum of the counts), weight sum}.
 * Returns the number of passes (<= max_pass) or a negative status. */
long orc_schedule_lists_policy(uint64_t slots, size_t nray, const uint64_t *off, const uint32_t *lists,
                               const int64_t *hit, const uint8_t *entered, const uint32_t *w0, const uint32_t *wk,
                               long nbx, long nby, long nbz, uint32_t spec_cap, uint32_t policy, long max_pass,
                               uint64_t *stats) {
    if (!off || !hit || !entered || !stats || spec_cap < 1 || nbx < 1 || nby < 1 || nbz < 1) return ORC_EINVAL;
    if (policy > 1 || (policy == 1 && (!w0 || !wk))) return ORC_EINVAL;
    size_t nb = (size_t)nbx * nby * nbz;
    for (size_t i = 0; i < nray; ++i)
        for (uint64_t k = off[i]; k < off[i + 1]; ++k)
            if (lists[k] >= nb) return ORC_EINVAL;
    int64_t *pos = (int64_t *)calloc(nray ? nray : 1, sizeof(int64_t));
    char *act = (char *)calloc(nray ? nray : 1, 1);
    uint32_t *vstamp = (uint32_t *)calloc(nb, sizeof(uint32_t));
    uint32_t *astamp = (uint32_t *)calloc(nb, sizeof(uint32_t));
    if (!pos || !act || !vstamp || !astamp) {
        free(pos); free(act); free(vstamp); free(astamp);
        return ORC_ENOMEM;
    }
    uint64_t n_act = 0;
    for (size_t i = 0; i < nray; ++i) { act[i] = entered[i] ? 1 : 0; n_act += act[i]; }
    long p = 0;
    while (n_act > 0 && p < max_pass) {
        uint32_t ns = orc_nspec(slots, n_act, spec_cap);
        uint64_t wsum = 0;
        if (policy == 1)
            for (size_t i = 0; i < nray; ++i)
                if (act[i]) wsum += pos[i] == 0 ? w0[i] : wk[off[i] + (uint64_t)(pos[i] - 1)];
        uint64_t pairs = 0, vis = 0, actb = 0, term = 0, surv = 0, nslots = 0;
        uint32_t nmax = 0;
        uint32_t stamp = (uint32_t)(p + 1);
        for (size_t i = 0; i < nray; ++i) {
            if (!act[i]) continue;
            uint32_t ni = ns;
            if (policy == 1) {
                uint32_t w = pos[i] == 0 ? w0[i] : wk[off[i] + (uint64_t)(pos[i] - 1)];
                ni = orc_nspec_ray(slots, n_act, wsum, w, spec_cap);
            }
            nslots += ni;
            if (ni > nmax) nmax = ni;
            int64_t len = (int64_t)(off[i + 1] - off[i]);
            int64_t take = len - pos[i];
            if (take > (int64_t)ni) take = ni;
            for (int64_t k = 0; k < take; ++k) {
                uint32_t b = lists[off[i] + (uint64_t)(pos[i] + k)];
                pairs++;
                if (vstamp[b] != stamp) {
                    vstamp[b] = stamp;
                    vis++;
                    long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx) {
                                long x = bx + dx, y = by + dy, z = bz + dz;
                                if (x >= nbx || y >= nby || z >= nbz) continue;
                                size_t o = (size_t)((z * nby + y) * nbx + x);
                                if (astamp[o] != stamp) { astamp[o] = stamp; actb++; }
                            }
                }
            }
            int done = (hit[i] >= pos[i] && hit[i] < pos[i] + take) || take < (int64_t)ni;
            pos[i] += take;
            if (done) { act[i] = 0; term++; }
            else surv++;
        }
        uint64_t *st = stats + 8 * p;
        st[0] = n_act; st[1] = nmax; st[2] = pairs; st[3] = vis; st[4] = actb; st[5] = term; st[6] = nslots;
        st[7] = wsum;
        n_act = surv;
        ++p;
    }
    free(pos); free(act); free(vstamp); free(astamp);
    return p;
}

long orc_schedule_lists(uint64_t slots, size_t nray, const uint64_t *off, const uint32_t *lists,
                        const int64_t *hit, const uint8_t *entered, long nbx, long nby, long nbz,
                        uint32_t spec_cap, long max_pass, uint64_t *stats) {
    return orc_schedule_lists_policy(slots, nray, off, lists, hit, entered, NULL, NULL, nbx, nby, nbz, spec_cap, 0,
                                     max_pass, stats);
}

/* One pixel's candidate blocks (in walk order), the weight of the ray after
 * each (wlist) and before the first (*w0), and the index of the block that
 * holds its first hit (*hit_idx, -1 if none).  Returns the number of
 * candidates (at most cap are stored) or a negative status. */
long orc_pixel_candidates(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
                          int px, int py, uint32_t *list, uint32_t *wlist, long cap, int64_t *hit_idx, uint32_t *w0) {
    if (!vol || !cam || !list || !wlist || !hit_idx || !w0) return ORC_EINVAL;
    cam_basis cb;
    if (make_basis(cam, w, h, &cb)) return ORC_EINVAL;
    long nb = nblk_axis(nx) * nblk_axis(ny) * nblk_axis(nz);
    float *fine = (float *)malloc(sizeof(float) * 2 * (size_t)nb);
    if (!fine) return ORC_ENOMEM;
    orc_grids(vol, nx, ny, nz, NULL, fine, NULL);
    uint32_t *l = NULL, *wl = NULL;
    long lcap = 0, hi;
    int entered;
    long n = ray_candidates(vol, fine, nx, ny, nz, &cb, iso, px, py, &l, &wl, &lcap, &hi, &entered, w0);
    for (long k = 0; k < n && k < cap; ++k) { list[k] = l[k]; wlist[k] = wl[k]; }
    *hit_idx = hi;
    free(l); free(wl); free(fine);
    return n;
}

/* Candidate lists of every pixel of a render, then the pass schedule under
 * the given speculation policy (0: Sec. 4's single count, 1: per-ray counts). */
long orc_schedule_policy(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
                         uint32_t spec_cap, uint32_t policy, long max_pass, uint64_t *stats) {
    if (!vol || !cam || !stats || spec_cap < 1 || policy > 1) return ORC_EINVAL;
    cam_basis cb;
    if (make_basis(cam, w, h, &cb)) return ORC_EINVAL;
    long nbx = nblk_axis(nx), nby = nblk_axis(ny), nbz = nblk_axis(nz);
    size_t nb = (size_t)nbx * nby * nbz;
    float *fine = (float *)malloc(sizeof(float) * 2 * nb);
    if (!fine) return ORC_ENOMEM;
    orc_grids(vol, nx, ny, nz, NULL, fine, NULL);
    size_t npx = (size_t)w * h;
    uint32_t **lists = (uint32_t **)calloc(npx, sizeof(uint32_t *));
    uint32_t **wl = (uint32_t **)calloc(npx, sizeof(uint32_t *));
    long *len = (long *)calloc(npx, sizeof(long));
    int64_t *hit = (int64_t *)calloc(npx, sizeof(int64_t));
    uint8_t *ent = (uint8_t *)calloc(npx, 1);
    uint32_t *w0 = (uint32_t *)calloc(npx ? npx : 1, sizeof(uint32_t));
    uint64_t *off = (uint64_t *)calloc(npx + 1, sizeof(uint64_t));
    if (!lists || !wl || !len || !hit || !ent || !w0 || !off) {
        free(fine); free(lists); free(wl); free(len); free(hit); free(ent); free(w0); free(off);
        return ORC_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < (long)npx; ++i) {
        long cap = 0, hi;
        int entered;
        len[i] = ray_candidates(vol, fine, nx, ny, nz, &cb, iso, (int)(i % w), (int)(i / w), &lists[i], &wl[i],
                                &cap, &hi, &entered, &w0[i]);
        hit[i] = hi;
        ent[i] = (uint8_t)entered;
    }
    for (size_t i = 0; i < npx; ++i) off[i + 1] = off[i] + (uint64_t)len[i];
    uint32_t *flat = (uint32_t *)malloc(sizeof(uint32_t) * (off[npx] ? off[npx] : 1));
    uint32_t *wflat = (uint32_t *)malloc(sizeof(uint32_t) * (off[npx] ? off[npx] : 1));
    long rc = ORC_ENOMEM;
    if (flat && wflat) {
        for (size_t i = 0; i < npx; ++i)
            if (len[i]) {
                memcpy(flat + off[i], lists[i], sizeof(uint32_t) * (size_t)len[i]);
                memcpy(wflat + off[i], wl[i], sizeof(uint32_t) * (size_t)len[i]);
            }
        rc = orc_schedule_lists_policy(npx, npx, off, flat, hit, ent, w0, wflat, nbx, nby, nbz, spec_cap, policy,
                                       max_pass, stats);
    }
    for (size_t i = 0; i < npx; ++i) { free(lists[i]); free(wl[i]); }
    free(flat); free(wflat); free(fine); free(lists); free(wl); free(len); free(hit); free(ent); free(w0); free(off);
    return rc;
}

long orc_schedule(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
                  uint32_t spec_cap, long max_pass, uint64_t *stats) {
    return orc_schedule_policy(vol, nx, ny, nz, cam, iso, w, h, spec_cap, 0, max_pass, stats);
}

/* Blocks whose fine range contains iso: what an extraction method that
 * decompresses every such block would touch (comparison counter). */
uint64_t orc_blocks_containing(const float *fine_lohi, size_t nblocks, float iso) {
    uint64_t n = 0;
    for (size_t b = 0; b < nblocks; ++b)
        if (fine_lohi[2 * b] <= iso && iso <= fine_lohi[2 * b + 1]) n++;
    return n;
}
