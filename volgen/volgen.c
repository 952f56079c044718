/*
 * volgen — seeded synthetic scalar fields and the offline fixed-rate block
 * encoder that turns them into compressed volumes.
 *
 * This module produces INPUTS only.  It plays the role of the paper's offline
 * compression step (Sec. 3 overview and Sec. 5 Evaluation: data are converted
 * to float32 and compressed block-wise at a fixed rate before upload).  It
 * holds none of the rendering method's arithmetic: no decoder, no traversal,
 * no intersection.  Both the CPU oracle and the GPU library consume what it
 * writes; neither links against it.
 *
 * Pseudo-random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), one stream per seed.
 *
 * Codec (format version 1), written out in full so that independent decoders
 * can be built from this description:
 *   A volume of nx*ny*nz float32 samples (x fastest) is cut into 4x4x4 blocks;
 *   block (bx,by,bz) has linear id bx + nbx*(by + nby*bz), nb = ceil(n/4).
 *   Samples of a partial block beyond the volume edge replicate the last
 *   sample on that axis.  Block b's record is 64*R bits at byte offset b*8R,
 *   read as little-endian 32-bit words, bit i of the record = bit (i&31) of
 *   word (i>>5).
 *   R == 32 (raw): the record is the 64 float32 values, raster order
 *   (x + 4y + 16z).
 *   1 <= R <= 16 (coded):
 *     bit 0      : 1 if any value is nonzero, else the block decodes to +0.
 *     bits 1..8  : E = e + 127, e = max(frexp exponent of max|v|, -127).
 *     quantise   : q = trunc(v * 2^(27-e)) as int32 (|q| < 2^27).
 *     transform  : along x, then y, then z, every line (a0,a1,a2,a3) becomes
 *                  (L, H, h0, h1) with h0 = a0-a1, l0 = floor((a0+a1)/2),
 *                  h1 = a2-a3, l1 = floor((a2+a3)/2), H = l0-l1,
 *                  L = floor((l0+l1)/2).  |coefficient| < 2^30.
 *     order      : coefficient positions sorted by lev(x)+lev(y)+lev(z) with
 *                  lev = {0,1,2,2}, ties by raster index.
 *     planes     : sign-magnitude, planes 29 down to 0; in each plane first
 *                  one refinement bit per already significant coefficient (in
 *                  order), then group tests over the insignificant ones at or
 *                  after a cursor: bit 1 = "one of them has this plane's bit",
 *                  followed by that plane's bit of each candidate in order up
 *                  to and including the first 1, then its sign bit (1 =
 *                  negative); bit 0 ends the plane; no test is written when
 *                  no candidate is left.  Writing stops when 64R bits are
 *                  used; the rest of the record is zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VG_OK 0
#define VG_EINVAL -1
#define VG_ENOMEM -2

/* ---------------------------------------------------------------- PRNG --- */

static inline uint64_t sm64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double sm64_unit(uint64_t *s) {
    return (double)(sm64_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

static inline double sm64_range(uint64_t *s, double lo, double hi) {
    return lo + (hi - lo) * sm64_unit(s);
}

uint64_t vg_splitmix64(uint64_t *state) { return sm64_next(state); }

double vg_unit(uint64_t *state) { return sm64_unit(state); }

/* -------------------------------------------------------------- fields --- */

/* Sum of nblob Gaussian blobs: f(x) = sum a_i exp(-|x-c_i|^2 / (2 s_i^2)).
 * Centres U[n/8, 7n/8 - 1] per axis, sigma U[4,10]*(nmin/64), amplitude
 * U[0.5,1].  out has nx*ny*nz floats, x fastest. */
int vg_blobs(int nx, int ny, int nz, uint64_t seed, int nblob, float *out) {
    if (nx < 2 || ny < 2 || nz < 2 || nblob < 1 || nblob > 256 || !out) return VG_EINVAL;
    double cx[256], cy[256], cz[256], inv2s2[256], amp[256];
    uint64_t s = seed;
    int nmin = nx < ny ? (nx < nz ? nx : nz) : (ny < nz ? ny : nz);
    double sscale = (double)nmin / 64.0;
    for (int i = 0; i < nblob; ++i) {
        cx[i] = sm64_range(&s, nx / 8.0, 7.0 * nx / 8.0 - 1.0);
        cy[i] = sm64_range(&s, ny / 8.0, 7.0 * ny / 8.0 - 1.0);
        cz[i] = sm64_range(&s, nz / 8.0, 7.0 * nz / 8.0 - 1.0);
        double sig = sm64_range(&s, 4.0, 10.0) * sscale;
        inv2s2[i] = 1.0 / (2.0 * sig * sig);
        amp[i] = sm64_range(&s, 0.5, 1.0);
    }
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                double f = 0.0;
                for (int i = 0; i < nblob; ++i) {
                    double dx = x - cx[i], dy = y - cy[i], dz = z - cz[i];
                    f += amp[i] * exp(-(dx * dx + dy * dy + dz * dz) * inv2s2[i]);
                }
                out[(z * ny + y) * nx + x] = (float)f;
            }
    return VG_OK;
}

/* Turbulence-like field: nmode random Fourier modes with |k|^(-5/3) amplitude,
 * f(x) = sum_m |k_m|^(-5/3) cos(2 pi k_m . x / period + phi_m).
 * k_m integer vectors in [-kmax,kmax]^3 with 1 <= |k_m| <= kmax (rejection
 * sampled), phi_m U[0, 2pi).  Evaluated as products of per-axis complex
 * exponential tables, accumulated in double. */
int vg_fourier(int nx, int ny, int nz, uint64_t seed, int nmode, int kmax, double period,
               float *out) {
    if (nx < 2 || ny < 2 || nz < 2 || nmode < 1 || nmode > 1024 || kmax < 1 || !(period > 0) || !out)
        return VG_EINVAL;
    int kx[1024], ky[1024], kz[1024];
    double amp[1024], ph[1024];
    uint64_t s = seed;
    const double twopi = 6.283185307179586476925286766559;
    for (int m = 0; m < nmode; ++m) {
        for (;;) {
            int a = (int)(sm64_next(&s) % (uint64_t)(2 * kmax + 1)) - kmax;
            int b = (int)(sm64_next(&s) % (uint64_t)(2 * kmax + 1)) - kmax;
            int c = (int)(sm64_next(&s) % (uint64_t)(2 * kmax + 1)) - kmax;
            int k2 = a * a + b * b + c * c;
            if (k2 >= 1 && k2 <= kmax * kmax) { kx[m] = a; ky[m] = b; kz[m] = c; break; }
        }
        double kn = sqrt((double)(kx[m] * kx[m] + ky[m] * ky[m] + kz[m] * kz[m]));
        amp[m] = pow(kn, -5.0 / 3.0);
        ph[m] = twopi * sm64_unit(&s);
    }
    /* per-axis tables: e^{i 2 pi k x / period} */
    double *ex = (double *)malloc(sizeof(double) * 2 * (size_t)nmode * nx);
    double *ey = (double *)malloc(sizeof(double) * 2 * (size_t)nmode * ny);
    double *ez = (double *)malloc(sizeof(double) * 2 * (size_t)nmode * nz);
    if (!ex || !ey || !ez) { free(ex); free(ey); free(ez); return VG_ENOMEM; }
    for (int m = 0; m < nmode; ++m) {
        for (int x = 0; x < nx; ++x) {
            double a = twopi * (double)kx[m] * x / period;
            ex[2 * ((size_t)m * nx + x)] = cos(a); ex[2 * ((size_t)m * nx + x) + 1] = sin(a);
        }
        for (int y = 0; y < ny; ++y) {
            double a = twopi * (double)ky[m] * y / period;
            ey[2 * ((size_t)m * ny + y)] = cos(a); ey[2 * ((size_t)m * ny + y) + 1] = sin(a);
        }
        for (int z = 0; z < nz; ++z) {
            double a = twopi * (double)kz[m] * z / period + ph[m];
            ez[2 * ((size_t)m * nz + z)] = amp[m] * cos(a);
            ez[2 * ((size_t)m * nz + z) + 1] = amp[m] * sin(a);
        }
    }
#pragma omp parallel
    {
        double *pr = (double *)malloc(sizeof(double) * 2 * nmode);
#pragma omp for schedule(static)
        for (long zy = 0; zy < (long)nz * ny; ++zy) {
            long z = zy / ny, y = zy % ny;
            for (int m = 0; m < nmode; ++m) {
                double ar = ey[2 * ((size_t)m * ny + y)], ai = ey[2 * ((size_t)m * ny + y) + 1];
                double br = ez[2 * ((size_t)m * nz + z)], bi = ez[2 * ((size_t)m * nz + z) + 1];
                pr[2 * m] = ar * br - ai * bi;
                pr[2 * m + 1] = ar * bi + ai * br;
            }
            float *row = out + (size_t)zy * nx;
            for (int x = 0; x < nx; ++x) {
                double f = 0.0;
                for (int m = 0; m < nmode; ++m) {
                    const double *e = ex + 2 * ((size_t)m * nx + x);
                    f += pr[2 * m] * e[0] - pr[2 * m + 1] * e[1];
                }
                row[x] = (float)f;
            }
        }
        free(pr);
    }
    free(ex); free(ey); free(ez);
    return VG_OK;
}

/* Analytic fields used by the closed-form tests (exactly representable
 * samples when the parameters are small integers / dyadic rationals).
 * kind 0: plane   f = a*x + b*y + c*z + d            (p = a,b,c,d)
 * kind 1: product f = (x-a)*(y-b)*(z-c)              (p = a,b,c)
 * kind 2: sphere  f = (x-a)^2 + (y-b)^2 + (z-c)^2    (p = a,b,c) */
int vg_analytic(int nx, int ny, int nz, int kind, const double *p, float *out) {
    if (nx < 2 || ny < 2 || nz < 2 || !p || !out || kind < 0 || kind > 2) return VG_EINVAL;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                double f;
                if (kind == 0) f = p[0] * x + p[1] * y + p[2] * z + p[3];
                else if (kind == 1) f = (x - p[0]) * (y - p[1]) * (z - p[2]);
                else f = (x - p[0]) * (x - p[0]) + (y - p[1]) * (y - p[1]) + (z - p[2]) * (z - p[2]);
                out[(z * ny + y) * nx + x] = (float)f;
            }
    return VG_OK;
}

/* Quantise a float field to 0..255 integers stored as float (the u8 -> f32
 * conversion the paper applies before compression): v = clamp(round((f-lo)/
 * (hi-lo)*255), 0, 255). */
int vg_quantize_u8(float *vals, size_t n, float lo, float hi) {
    if (!vals || !(hi > lo)) return VG_EINVAL;
    double sc = 255.0 / ((double)hi - (double)lo);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)n; ++i) {
        double v = floor(((double)vals[i] - lo) * sc + 0.5);
        if (v < 0) v = 0;
        if (v > 255) v = 255;
        vals[i] = (float)v;
    }
    return VG_OK;
}

/* ----------------------------------------------------- order statistic --- */

static inline uint32_t f2key(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

static inline float key2f(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Exact k-th smallest value (0-based) of vals[0..n) by a two-round 16-bit
 * radix select on order-preserving keys. */
int vg_kth_value(const float *vals, size_t n, size_t k, float *out) {
    if (!vals || !out || k >= n) return VG_EINVAL;
    uint64_t *h = (uint64_t *)calloc(65536, sizeof(uint64_t));
    if (!h) return VG_ENOMEM;
    for (size_t i = 0; i < n; ++i) h[f2key(vals[i]) >> 16]++;
    size_t acc = 0;
    uint32_t hi = 0;
    for (uint32_t b = 0; b < 65536; ++b) {
        if (acc + h[b] > k) { hi = b; break; }
        acc += h[b];
    }
    memset(h, 0, 65536 * sizeof(uint64_t));
    for (size_t i = 0; i < n; ++i) {
        uint32_t key = f2key(vals[i]);
        if ((key >> 16) == hi) h[key & 0xffff]++;
    }
    size_t rem = k - acc;
    uint32_t lo = 0;
    for (uint32_t b = 0; b < 65536; ++b) {
        if (h[b] > rem) { lo = b; break; }
        rem -= h[b];
    }
    free(h);
    *out = key2f((hi << 16) | lo);
    return VG_OK;
}

/* ------------------------------------------------------------- encoder --- */

static int g_order[64];
static int g_order_ready = 0;

static void build_order(void) {
    if (g_order_ready) return;
    static const int lev[4] = {0, 1, 2, 2};
    int idx[64], key[64];
    for (int i = 0; i < 64; ++i) {
        idx[i] = i;
        key[i] = lev[i & 3] + lev[(i >> 2) & 3] + lev[i >> 4];
    }
    /* insertion sort by (key, index): stable on raster index */
    for (int i = 1; i < 64; ++i) {
        int v = idx[i], j = i - 1;
        while (j >= 0 && key[idx[j]] > key[v]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
    memcpy(g_order, idx, sizeof(idx));
    g_order_ready = 1;
}

static inline int32_t floor_half(int32_t s) { return s >> 1; } /* arithmetic shift */

static void fwd_line(int32_t *p, int stride) {
    int32_t a0 = p[0], a1 = p[stride], a2 = p[2 * stride], a3 = p[3 * stride];
    int32_t h0 = a0 - a1, l0 = floor_half(a0 + a1);
    int32_t h1 = a2 - a3, l1 = floor_half(a2 + a3);
    int32_t H = l0 - l1, L = floor_half(l0 + l1);
    p[0] = L; p[stride] = H; p[2 * stride] = h0; p[3 * stride] = h1;
}

typedef struct {
    uint32_t *w;
    uint32_t pos, budget;
} bitwriter;

/* returns 0 when the budget is exhausted (bit not written) */
static inline int put_bit(bitwriter *bw, uint32_t b) {
    if (bw->pos >= bw->budget) return 0;
    if (b) bw->w[bw->pos >> 5] |= 1u << (bw->pos & 31);
    bw->pos++;
    return 1;
}

static void encode_block(const float v[64], int R, uint32_t *rec) {
    if (R == 32) { memcpy(rec, v, 256); return; }
    uint32_t nwords = 2u * (uint32_t)R;
    memset(rec, 0, nwords * 4);
    float amax = 0.0f;
    for (int i = 0; i < 64; ++i) {
        float a = fabsf(v[i]);
        if (a > amax) amax = a;
    }
    if (amax == 0.0f) return;
    int e;
    frexpf(amax, &e);
    if (e < -127) e = -127;
    int32_t q[64];
    for (int i = 0; i < 64; ++i) q[i] = (int32_t)trunc(ldexp((double)v[i], 27 - e));
    for (int z = 0; z < 4; ++z) for (int y = 0; y < 4; ++y) fwd_line(q + 4 * y + 16 * z, 1);
    for (int z = 0; z < 4; ++z) for (int x = 0; x < 4; ++x) fwd_line(q + x + 16 * z, 4);
    for (int y = 0; y < 4; ++y) for (int x = 0; x < 4; ++x) fwd_line(q + x + 4 * y, 16);
    uint32_t mag[64], neg[64];
    for (int j = 0; j < 64; ++j) {
        int32_t c = q[g_order[j]];
        neg[j] = c < 0;
        mag[j] = (uint32_t)(c < 0 ? -c : c);
    }
    bitwriter bw = {rec, 0, 64u * (uint32_t)R};
    put_bit(&bw, 1);
    for (int i = 0; i < 8; ++i) put_bit(&bw, ((uint32_t)(e + 127) >> i) & 1u);
    uint8_t sig[64] = {0};
    for (int k = 29; k >= 0; --k) {
        for (int j = 0; j < 64; ++j)
            if (sig[j] && !put_bit(&bw, (mag[j] >> k) & 1u)) return;
        int c = 0;
        for (;;) {
            int any_cand = 0, any_bit = 0;
            for (int j = c; j < 64; ++j)
                if (!sig[j]) { any_cand = 1; if ((mag[j] >> k) & 1u) any_bit = 1; }
            if (!any_cand) break;
            if (!put_bit(&bw, (uint32_t)any_bit)) return;
            if (!any_bit) break;
            int target = -1;
            for (int j = c; j < 64; ++j) {
                if (sig[j]) continue;
                uint32_t b = (mag[j] >> k) & 1u;
                if (!put_bit(&bw, b)) return;
                if (b) { target = j; break; }
            }
            if (!put_bit(&bw, neg[target])) return;
            sig[target] = 1;
            c = target + 1;
        }
    }
}

/* Encode a volume.  rate in 1..16 or 32.  out must hold nblocks*8*rate bytes
 * where nblocks = ceil(nx/4)*ceil(ny/4)*ceil(nz/4). */
int vg_encode(const float *vol, int nx, int ny, int nz, int rate, void *out) {
    if (!vol || !out || nx < 1 || ny < 1 || nz < 1) return VG_EINVAL;
    if (!((rate >= 1 && rate <= 16) || rate == 32)) return VG_EINVAL;
    build_order();
    long nbx = (nx + 3) / 4, nby = (ny + 3) / 4, nbz = (nz + 3) / 4;
    long nblk = nbx * nby * nbz;
    size_t rec_words = 2u * (size_t)rate;
#pragma omp parallel for schedule(dynamic, 256)
    for (long b = 0; b < nblk; ++b) {
        long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        float v[64];
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) {
                    long x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                    if (x > nx - 1) x = nx - 1;
                    if (y > ny - 1) y = ny - 1;
                    if (z > nz - 1) z = nz - 1;
                    v[i + 4 * j + 16 * k] = vol[(z * ny + y) * nx + x];
                }
        encode_block(v, rate, (uint32_t *)out + (size_t)b * rec_words);
    }
    return VG_OK;
}

/* Encode one block of 64 raster-order values (tests). */
int vg_encode_block(const float *v64, int rate, void *rec) {
    if (!v64 || !rec || !((rate >= 1 && rate <= 16) || rate == 32)) return VG_EINVAL;
    build_order();
    encode_block(v64, rate, (uint32_t *)rec);
    return VG_OK;
}
