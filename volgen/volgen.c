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
 *     decoding   : read the planes back (a record ends after 64R bits, so a
 *                  truncated code leaves the remaining bits 0), undo the
 *                  order, invert each line as l1 = L - floor(H/2),
 *                  l0 = l1 + H, a1 = l0 - floor(h0/2), a0 = a1 + h0,
 *                  a3 = l1 - floor(h1/2), a2 = a3 + h1, along z, then y,
 *                  then x, in 32-bit two's-complement arithmetic (sums wrap
 *                  modulo 2^32), and output float(q * 2^(e-27)) rounded once.
 *                  The wrap can only matter for records this encoder never
 *                  writes (its coefficients keep every partial sum below
 *                  2^31); the rule was fixed after the first decoders were
 *                  written, without a version change, since it changes no
 *                  encoder output.
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

/* --------------------------------------------- RM-like mixing layer --- */
/* A two-fluid interface at mid-depth shaped like a Richtmyer-Meshkov mixing
 * layer:  v = clamp(round(255 * (1 + tanh(s / delta)) / 2), 0, 255),
 *   s = z - zc - h(x,y) - eta(x,y,z),  zc = (nz-1)/2,
 *   delta = 6 / (2 atanh 0.8)   (10% -> 90% over 6 samples),
 *   h = sum of 32 modes a_m sin(2 pi (p_m x + q_m y) / nx + phi_m), integer
 *       p, q in [-16,16] not both 0, a_m ~ 1/|(p,q)|, sum a_m = hsum,
 *   eta = 3-octave value noise (periods 64, 32, 16 samples; amplitudes 16, 8,
 *       4): smoothstep-weighted trilinear interpolation of hashed lattice
 *       values in [-1, 1].
 * |h| <= hsum and |eta| <= 28, so outside the band |s| > 28 + 12 the value is
 * exactly 0 or 255 and tanh is not evaluated there. */

typedef struct {
    int nx, ny, nz;
    double zc, inv_delta, hsum;
    double *h;            /* nx*ny */
    float *lat[3];        /* lattice values per octave */
    int ln[3][3];         /* lattice sizes */
    int period[3];
    double amp[3];
} rm_ctx;

static float lattice_value(uint64_t seed, int oct, int ix, int iy, int iz) {
    uint64_t s = seed * 0x9e3779b97f4a7c15ULL ^ ((uint64_t)oct << 58) ^ ((uint64_t)(uint32_t)ix << 38) ^
                 ((uint64_t)(uint32_t)iy << 19) ^ (uint64_t)(uint32_t)iz;
    return (float)(2.0 * sm64_unit(&s) - 1.0);
}

static int rm_init(rm_ctx *c, int nx, int ny, int nz, uint64_t seed, double hsum) {
    memset(c, 0, sizeof(*c));
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->zc = 0.5 * (nz - 1);
    c->inv_delta = (2.0 * atanh(0.8)) / 6.0;
    c->hsum = hsum;
    c->h = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    if (!c->h) return VG_ENOMEM;
    int pm[32], qm[32];
    double am[32], ph[32], asum = 0.0;
    uint64_t s = seed;
    const double twopi = 6.283185307179586476925286766559;
    for (int m = 0; m < 32; ++m) {
        do {
            pm[m] = (int)(sm64_next(&s) % 33ull) - 16;
            qm[m] = (int)(sm64_next(&s) % 33ull) - 16;
        } while (pm[m] == 0 && qm[m] == 0);
        am[m] = 1.0 / sqrt((double)(pm[m] * pm[m] + qm[m] * qm[m]));
        asum += am[m];
        ph[m] = twopi * sm64_unit(&s);
    }
    for (int m = 0; m < 32; ++m) am[m] *= hsum / asum;
    /* separable evaluation: sin(a + b) = sin a cos b + cos a sin b */
    double *sx = (double *)malloc(sizeof(double) * 32 * (size_t)nx), *cx = (double *)malloc(sizeof(double) * 32 * (size_t)nx);
    double *sy = (double *)malloc(sizeof(double) * 32 * (size_t)ny), *cy = (double *)malloc(sizeof(double) * 32 * (size_t)ny);
    if (!sx || !cx || !sy || !cy) { free(sx); free(cx); free(sy); free(cy); return VG_ENOMEM; }
    for (int m = 0; m < 32; ++m) {
        for (int x = 0; x < nx; ++x) {
            double a = twopi * pm[m] * x / (double)nx + ph[m];
            sx[m * (size_t)nx + x] = sin(a); cx[m * (size_t)nx + x] = cos(a);
        }
        for (int y = 0; y < ny; ++y) {
            double b = twopi * qm[m] * y / (double)nx;
            sy[m * (size_t)ny + y] = sin(b); cy[m * (size_t)ny + y] = cos(b);
        }
    }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double v = 0.0;
            for (int m = 0; m < 32; ++m)
                v += am[m] * (sx[m * (size_t)nx + x] * cy[m * (size_t)ny + y] + cx[m * (size_t)nx + x] * sy[m * (size_t)ny + y]);
            c->h[(size_t)y * nx + x] = v;
        }
    free(sx); free(cx); free(sy); free(cy);
    int periods[3] = {64, 32, 16};
    double amps[3] = {16.0, 8.0, 4.0};
    for (int o = 0; o < 3; ++o) {
        c->period[o] = periods[o];
        c->amp[o] = amps[o];
        int lx = nx / periods[o] + 2, ly = ny / periods[o] + 2, lz = nz / periods[o] + 2;
        c->ln[o][0] = lx; c->ln[o][1] = ly; c->ln[o][2] = lz;
        c->lat[o] = (float *)malloc(sizeof(float) * (size_t)lx * ly * lz);
        if (!c->lat[o]) return VG_ENOMEM;
#pragma omp parallel for schedule(static)
        for (long iz = 0; iz < lz; ++iz)
            for (int iy = 0; iy < ly; ++iy)
                for (int ix = 0; ix < lx; ++ix)
                    c->lat[o][((size_t)iz * ly + iy) * lx + ix] = lattice_value(seed, o, ix, iy, (int)iz);
    }
    return VG_OK;
}

static void rm_free(rm_ctx *c) {
    free(c->h);
    for (int o = 0; o < 3; ++o) free(c->lat[o]);
}

static inline double smooth01(double t) { return t * t * (3.0 - 2.0 * t); }

static double rm_eta(const rm_ctx *c, int x, int y, int z) {
    double eta = 0.0;
    for (int o = 0; o < 3; ++o) {
        int P = c->period[o];
        int ix = x / P, iy = y / P, iz = z / P;
        double fx = smooth01((x - ix * P) / (double)P), fy = smooth01((y - iy * P) / (double)P),
               fz = smooth01((z - iz * P) / (double)P);
        const float *L = c->lat[o];
        int lx = c->ln[o][0], ly = c->ln[o][1];
#define LV(a, b, d) (double)L[((size_t)(iz + (d)) * ly + (iy + (b))) * lx + (ix + (a))]
        double v00 = LV(0, 0, 0) + (LV(1, 0, 0) - LV(0, 0, 0)) * fx;
        double v10 = LV(0, 1, 0) + (LV(1, 1, 0) - LV(0, 1, 0)) * fx;
        double v01 = LV(0, 0, 1) + (LV(1, 0, 1) - LV(0, 0, 1)) * fx;
        double v11 = LV(0, 1, 1) + (LV(1, 1, 1) - LV(0, 1, 1)) * fx;
#undef LV
        double v0 = v00 + (v10 - v00) * fy, v1 = v01 + (v11 - v01) * fy;
        eta += c->amp[o] * (v0 + (v1 - v0) * fz);
    }
    return eta;
}

static float rm_value(const rm_ctx *c, int x, int y, int z) {
    double s0 = z - c->zc - c->h[(size_t)y * c->nx + x];
    if (s0 > 40.0) return 255.0f;
    if (s0 < -40.0) return 0.0f;
    double s = s0 - rm_eta(c, x, y, z);
    double v = floor(255.0 * 0.5 * (1.0 + tanh(s * c->inv_delta)) + 0.5);
    if (v < 0) v = 0;
    if (v > 255) v = 255;
    return (float)v;
}

/* Small volumes: the RM-like field itself (tests). */
int vg_rm_field(int nx, int ny, int nz, uint64_t seed, double hsum, float *out) {
    if (nx < 2 || ny < 2 || nz < 2 || !out) return VG_EINVAL;
    rm_ctx c;
    int rc = rm_init(&c, nx, ny, nz, seed, hsum);
    if (rc) { rm_free(&c); return rc; }
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) out[((size_t)z * ny + y) * nx + x] = rm_value(&c, x, y, (int)z);
    rm_free(&c);
    return VG_OK;
}

static void build_order(void);
static void encode_block(const float v[64], int R, uint32_t *rec);

/* Generate and encode the RM-like volume block by block (no full-size
 * buffer): out holds nblocks * 8 * rate bytes. */
int vg_rm_encode(int nx, int ny, int nz, uint64_t seed, double hsum, int rate, void *out) {
    if (nx < 2 || ny < 2 || nz < 2 || !out || !((rate >= 1 && rate <= 16) || rate == 32)) return VG_EINVAL;
    build_order();
    rm_ctx c;
    int rc = rm_init(&c, nx, ny, nz, seed, hsum);
    if (rc) { rm_free(&c); return rc; }
    long nbx = (nx + 3) / 4, nby = (ny + 3) / 4, nbz = (nz + 3) / 4;
    size_t rec_words = 2u * (size_t)rate;
    /* blocks entirely above / below the band are constant 255 / 0 */
    uint32_t full_rec[64];
    {
        float v255[64];
        for (int i = 0; i < 64; ++i) v255[i] = 255.0f;
        encode_block(v255, rate, full_rec);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (long b = 0; b < nbx * nby * nbz; ++b) {
        long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        uint32_t *dst = (uint32_t *)out + (size_t)b * rec_words;
        double hmin = 1e300, hmax = -1e300;
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i) {
                long x = 4 * bx + i, y = 4 * by + j;
                if (x > nx - 1) x = nx - 1;
                if (y > ny - 1) y = ny - 1;
                double hv = c.h[(size_t)y * nx + x];
                if (hv < hmin) hmin = hv;
                if (hv > hmax) hmax = hv;
            }
        long z0 = 4 * bz, z1 = 4 * bz + 3 > nz - 1 ? nz - 1 : 4 * bz + 3;
        if ((double)z0 - c.zc - hmax > 40.0) { memcpy(dst, full_rec, rec_words * 4); continue; }
        if ((double)z1 - c.zc - hmin < -40.0) { memset(dst, 0, rec_words * 4); continue; }
        float v[64];
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) {
                    long x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                    if (x > nx - 1) x = nx - 1;
                    if (y > ny - 1) y = ny - 1;
                    if (z > nz - 1) z = nz - 1;
                    v[i + 4 * j + 16 * k] = rm_value(&c, (int)x, (int)y, (int)z);
                }
        encode_block(v, rate, dst);
    }
    rm_free(&c);
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
    /* plane masks: bit j of pm[k] = bit k of mag[j] (order space) */
    uint64_t pm[30] = {0};
    for (int j = 0; j < 64; ++j)
        for (int k = 0; k < 30; ++k)
            if ((mag[j] >> k) & 1u) pm[k] |= 1ull << j;
    uint64_t negm = 0;
    for (int j = 0; j < 64; ++j) negm |= (uint64_t)neg[j] << j;
    uint64_t sig = 0;
    for (int k = 29; k >= 0; --k) {
        uint64_t m = sig;
        while (m) {
            int j = __builtin_ctzll(m);
            m &= m - 1;
            if (!put_bit(&bw, (uint32_t)((pm[k] >> j) & 1u))) return;
        }
        int c = 0;
        for (;;) {
            uint64_t cand = c >= 64 ? 0ull : (~sig & (~0ull << c));
            if (!cand) break;
            uint32_t any = (pm[k] & cand) != 0;
            if (!put_bit(&bw, any)) return;
            if (!any) break;
            int target = __builtin_ctzll(pm[k] & cand);
            /* one zero bit per candidate before the target, then its 1 */
            uint64_t before = cand & ((1ull << target) - 1ull);
            int nz = __builtin_popcountll(before);
            for (int z = 0; z < nz; ++z)
                if (!put_bit(&bw, 0)) return;
            if (!put_bit(&bw, 1)) return;
            if (!put_bit(&bw, (uint32_t)((negm >> target) & 1u))) return;
            sig |= 1ull << target;
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
