/*
 * sanitize_main.c — drives every entry point of the CPU oracle on small
 * seeded inputs, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitize.py compiles and runs it).  Inputs
 * come from the seeded generator; the oracle itself is linked unchanged.
 * Exit status 0 means every call returned OK and neither sanitizer fired.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eye[3], center[3], up[3];
    double vfov_deg;
} orc_camera;

/* oracle (oracle/oracle.c) */
int orc_decode_block(const uint32_t *rec, int R, float *out);
int orc_decode_blocks(const void *stream, size_t bytes, int nx, int ny, int nz, int R, const uint32_t *ids, size_t n,
                      float *out);
int orc_decode_volume(const void *stream, size_t bytes, int nx, int ny, int nz, int R, float *out);
int orc_grids(const float *vol, int nx, int ny, int nz, float *block_lohi, float *fine_lohi, float *coarse_lohi);
int orc_block_ranges_stream(const void *stream, size_t bytes, int nx, int ny, int nz, int R, float *block_lohi);
int orc_grids_from_blocks(const float *block_lohi, int nx, int ny, int nz, float *fine_lohi, float *coarse_lohi);
int orc_render(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
               const uint32_t *pix, size_t npix, double *t_out, uint32_t *block_out, uint32_t *cell_out,
               uint32_t *rgba_out, uint8_t *entered_out);
int orc_render_stream(const void *stream, size_t bytes, int nx, int ny, int nz, int R, const orc_camera *cam,
                      float iso, int w, int h, const uint32_t *pix, size_t npix, double *t_out, uint32_t *block_out,
                      uint32_t *cell_out, uint32_t *rgba_out, uint8_t *entered_out);
long orc_cell_walk(int nx, int ny, int nz, const orc_camera *cam, int w, int h, int px, int py, int32_t *cells,
                   double *t01, long cap, double *t_enter_exit);
int orc_ray(int nx, int ny, int nz, const orc_camera *cam, int w, int h, int px, int py, double *out6);
long orc_schedule(const float *vol, int nx, int ny, int nz, const orc_camera *cam, float iso, int w, int h,
                  uint32_t spec_cap, long max_pass, uint64_t *stats);
uint64_t orc_blocks_containing(const float *fine_lohi, size_t nblocks, float iso);

/* seeded inputs (volgen/volgen.c) */
int vg_blobs(int nx, int ny, int nz, uint64_t seed, int nblob, float *out);
int vg_encode(const float *vol, int nx, int ny, int nz, int rate, void *out);
uint64_t vg_splitmix64(uint64_t *state);

#define CHECK(x)                                                         \
    do {                                                                 \
        long rc_ = (long)(x);                                            \
        if (rc_ < 0) {                                                   \
            fprintf(stderr, "%s:%d: %s returned %ld\n", __FILE__, __LINE__, #x, rc_); \
            exit(1);                                                     \
        }                                                                \
    } while (0)

static void one_volume(int nx, int ny, int nz, int rate, uint64_t seed) {
    const size_t nv = (size_t)nx * ny * nz;
    const long nbx = (nx + 3) / 4, nby = (ny + 3) / 4, nbz = (nz + 3) / 4;
    const size_t nb = (size_t)nbx * nby * nbz, nc = (size_t)((nbx + 3) / 4) * ((nby + 3) / 4) * ((nbz + 3) / 4);
    const size_t bytes = nb * 8u * (size_t)rate;
    float *vol = malloc(nv * sizeof(float)), *dec = malloc(nv * sizeof(float));
    uint8_t *stream = malloc(bytes);
    float *blk = malloc(nb * 2 * sizeof(float)), *fin = malloc(nb * 2 * sizeof(float)),
          *crs = malloc(nc * 2 * sizeof(float)), *blk2 = malloc(nb * 2 * sizeof(float));
    CHECK(vg_blobs(nx, ny, nz, seed, 8, vol));
    CHECK(vg_encode(vol, nx, ny, nz, rate, stream));
    CHECK(orc_decode_volume(stream, bytes, nx, ny, nz, rate, dec));
    CHECK(orc_grids(dec, nx, ny, nz, blk, fin, crs));
    CHECK(orc_block_ranges_stream(stream, bytes, nx, ny, nz, rate, blk2));
    CHECK(orc_grids_from_blocks(blk2, nx, ny, nz, fin, crs));
    uint32_t ids[3] = {0, (uint32_t)(nb / 2), (uint32_t)(nb - 1)};
    float out[3 * 64];
    CHECK(orc_decode_blocks(stream, bytes, nx, ny, nz, rate, ids, 3, out));
    float lo = dec[0], hi = dec[0];
    for (size_t i = 0; i < nv; ++i) { lo = dec[i] < lo ? dec[i] : lo; hi = dec[i] > hi ? dec[i] : hi; }
    const float iso = lo + 0.6f * (hi - lo);
    (void)orc_blocks_containing(fin, nb, iso);
    orc_camera cam = {{-1.7 * nx, 0.4 * ny, 1.9 * nz}, {0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1)}, {0, 0, 1}, 45.0};
    const int w = 24, h = 18, np = w * h;
    double t[24 * 18];
    uint32_t b[24 * 18], c[24 * 18], rgba[24 * 18];
    uint8_t ent[24 * 18];
    CHECK(orc_render(dec, nx, ny, nz, &cam, iso, w, h, NULL, 0, t, b, c, rgba, ent));
    uint32_t pix[5] = {0, 7, 100, 211, (uint32_t)np - 1};
    CHECK(orc_render_stream(stream, bytes, nx, ny, nz, rate, &cam, iso, w, h, pix, 5, t, b, c, rgba, ent));
    int32_t cells[3 * 512];
    double t01[2 * 512], tee[2], r6[6];
    for (int p = 0; p < np; p += 37) {
        long n = orc_cell_walk(nx, ny, nz, &cam, w, h, p % w, p / w, cells, t01, 512, tee);
        if (n < -1) exit(1);
        CHECK(orc_ray(nx, ny, nz, &cam, w, h, p % w, p / w, r6));
    }
    uint64_t *stats = calloc(4096 * 8, sizeof(uint64_t));
    CHECK(orc_schedule(dec, nx, ny, nz, &cam, iso, w, h, 1, 4096, stats));
    CHECK(orc_schedule(dec, nx, ny, nz, &cam, iso, w, h, 64, 4096, stats));
    free(stats); free(vol); free(dec); free(stream); free(blk); free(fin); free(crs); free(blk2);
}

int main(void) {
    /* every rate on ragged and whole sizes */
    const int rates[] = {1, 2, 3, 4, 8, 16, 32};
    for (unsigned k = 0; k < sizeof(rates) / sizeof(rates[0]); ++k) {
        one_volume(13, 10, 7, rates[k], 20 + k);
        one_volume(16, 16, 16, rates[k], 40 + k);
    }
    /* arbitrary records at every coded rate: the decoder's paths for any bits,
     * including inverse transforms that wrap */
    uint64_t s = 12345;
    for (int R = 1; R <= 16; ++R) {
        uint32_t rec[32];
        float out[64];
        for (int it = 0; it < 2000; ++it) {
            for (int i = 0; i < 2 * R; ++i) rec[i] = (uint32_t)vg_splitmix64(&s);
            if (it % 3 == 0) rec[0] |= 1u;   /* nonzero block */
            CHECK(orc_decode_block(rec, R, out));
        }
    }
    puts("sanitize ok");
    return 0;
}
