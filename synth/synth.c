/*
 * synth.c — seeded synthetic spectral cubes (noise plus Gaussian sources).
 *
 * Input generator shared by the renderer's tests/benchmarks and by the CPU
 * reference: it produces the voxel values both sides consume and holds none of
 * the rendering arithmetic (no sampling, classification or compositing).
 *
 * The cube models a radio spectral-line cube: two sky axes (x, y) and one
 * frequency axis (z), stored as a stack of per-channel images, x fastest
 * (Sec. 2 of the paper describes the cube as a stack of images over small
 * frequency ranges).  Noise is i.i.d. N(0, sigma^2); sources are 3-D
 * Gaussians with a shared spatial width and a separate spectral width.
 *
 * Randomness comes from the counter-based generator Philox4x32-10 (Salmon,
 * Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC 2011), written here from that definition.  Because it is counter-based,
 * the value of any voxel depends only on (seed, voxel index): any sub-region
 * can be regenerated on its own and threads never change the output.
 *
 * Normal deviates use the Box-Muller transform in double precision and are
 * rounded once to float after the sources are added.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One Philox4x32 bijection with 10 rounds: ctr (4 words), key (2 words). */
void synth_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                         uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += PHILOX_W0; k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0,1) from two words. */
static inline double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) *
           (1.0 / 9007199254740992.0);
}

/* 32-bit uniform in (0,1). */
static inline double u32o(uint32_t a) { return ((double)a + 0.5) * (1.0 / 4294967296.0); }

/* Key layout: word 0 = low 32 bits of the seed, word 1 = high bits xor stream. */
static inline void make_key(uint64_t seed, uint32_t stream, uint32_t key[2]) {
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32) ^ stream;
}

#define STREAM_NOISE 0x00000000u
#define STREAM_SOURCES 0x5EED0001u
#define STREAM_AUX 0x5EED0002u

/* Standard-normal deviate for linear voxel index v (pairs share one draw). */
double synth_normal(uint64_t seed, uint64_t v) {
    uint32_t key[2], ctr[4], out[4];
    make_key(seed, STREAM_NOISE, key);
    uint64_t pair = v >> 1;
    ctr[0] = (uint32_t)pair; ctr[1] = (uint32_t)(pair >> 32); ctr[2] = 0; ctr[3] = 0;
    synth_philox4x32_10(ctr, key, out);
    double u1 = 1.0 - u53(out[0], out[1]); /* (0,1] */
    double u2 = u53(out[2], out[3]);
    double r = sqrt(-2.0 * log(u1));
    double ang = 6.283185307179586476925286766559 * u2;
    return (v & 1) ? r * sin(ang) : r * cos(ang);
}

/* Uniform deviates for auxiliary streams (camera angles, pixel subsets...):
 * out[i] = U(0,1) for counter (index, i/4). */
void synth_uniforms(uint64_t seed, uint64_t index, int64_t count, double* out) {
    uint32_t key[2], ctr[4], w[4];
    make_key(seed, STREAM_AUX, key);
    for (int64_t i = 0; i < count; i += 4) {
        ctr[0] = (uint32_t)index; ctr[1] = (uint32_t)(index >> 32);
        ctr[2] = (uint32_t)(i >> 2); ctr[3] = 0;
        synth_philox4x32_10(ctr, key, w);
        for (int j = 0; j < 4 && i + j < count; ++j) out[i + j] = u32o(w[j]);
    }
}

/*
 * Source catalogue: nsrc rows of 6 doubles (x0, y0, z0, A, sigma_s, sigma_z).
 * Centres are uniform over [0, N-1] per axis; A is uniform on [a_lo, a_hi]
 * (log-uniform when a_log != 0); sigma_s ~ U[ss_lo, ss_hi];
 * sigma_z ~ U[sz_lo, sz_hi].  Amplitudes are in units of the noise sigma.
 */
int synth_sources(uint64_t seed, int64_t nsrc, int64_t nx, int64_t ny, int64_t nz,
                  double a_lo, double a_hi, int a_log, double ss_lo, double ss_hi,
                  double sz_lo, double sz_hi, double* out) {
    if (nsrc < 0 || !out || nx < 1 || ny < 1 || nz < 1) return -1;
    uint32_t key[2], ctr[4], w0[4], w1[4];
    make_key(seed, STREAM_SOURCES, key);
    for (int64_t s = 0; s < nsrc; ++s) {
        ctr[0] = (uint32_t)s; ctr[1] = (uint32_t)(s >> 32); ctr[2] = 0; ctr[3] = 0;
        synth_philox4x32_10(ctr, key, w0);
        ctr[2] = 1;
        synth_philox4x32_10(ctr, key, w1);
        double* r = out + 6 * s;
        r[0] = u32o(w0[0]) * (double)(nx - 1);
        r[1] = u32o(w0[1]) * (double)(ny - 1);
        r[2] = u32o(w0[2]) * (double)(nz - 1);
        double ua = u32o(w0[3]);
        r[3] = a_log ? exp(log(a_lo) + ua * (log(a_hi) - log(a_lo)))
                     : a_lo + ua * (a_hi - a_lo);
        r[4] = ss_lo + u32o(w1[0]) * (ss_hi - ss_lo);
        r[5] = sz_lo + u32o(w1[1]) * (sz_hi - sz_lo);
    }
    return 0;
}

/* Sources are truncated at this many widths from their centre per axis. */
#define SYNTH_TRUNC 5.0

typedef struct {
    uint64_t seed;
    int64_t nx, ny, nz;
    double sigma;
    const double* src;
    int64_t nsrc;
    int64_t z0, nzs;
    float* out;
    int noise;
    int tid, nthreads;
} job_t;

static void* plane_worker(void* arg) {
    job_t* J = (job_t*)arg;
    const int64_t nx = J->nx, ny = J->ny;
    double* acc = (double*)malloc(sizeof(double) * (size_t)(nx * ny));
    double* fx = (double*)malloc(sizeof(double) * (size_t)nx);
    double* fy = (double*)malloc(sizeof(double) * (size_t)ny);
    if (!acc || !fx || !fy) { free(acc); free(fx); free(fy); return (void*)1; }
    for (int64_t zz = J->tid; zz < J->nzs; zz += J->nthreads) {
        int64_t z = J->z0 + zz;
        const uint64_t base = (uint64_t)z * (uint64_t)(nx * ny);
        if (J->noise) {
            for (int64_t i = 0; i < nx * ny; ++i)
                acc[i] = J->sigma * synth_normal(J->seed, base + (uint64_t)i);
        } else {
            memset(acc, 0, sizeof(double) * (size_t)(nx * ny));
        }
        for (int64_t s = 0; s < J->nsrc; ++s) {
            const double* r = J->src + 6 * s;
            double x0 = r[0], y0 = r[1], zc = r[2], A = r[3], ss = r[4], sz = r[5];
            double dz = (double)z - zc;
            if (fabs(dz) > SYNTH_TRUNC * sz) continue;
            double ez = exp(-0.5 * dz * dz / (sz * sz));
            int64_t xa = (int64_t)ceil(x0 - SYNTH_TRUNC * ss), xb = (int64_t)floor(x0 + SYNTH_TRUNC * ss);
            int64_t ya = (int64_t)ceil(y0 - SYNTH_TRUNC * ss), yb = (int64_t)floor(y0 + SYNTH_TRUNC * ss);
            if (xa < 0) xa = 0;
            if (ya < 0) ya = 0;
            if (xb > nx - 1) xb = nx - 1;
            if (yb > ny - 1) yb = ny - 1;
            if (xa > xb || ya > yb) continue;
            for (int64_t x = xa; x <= xb; ++x) {
                double dx = (double)x - x0;
                fx[x] = exp(-0.5 * dx * dx / (ss * ss));
            }
            for (int64_t y = ya; y <= yb; ++y) {
                double dy = (double)y - y0;
                fy[y] = exp(-0.5 * dy * dy / (ss * ss));
            }
            double a = A * J->sigma * ez;
            for (int64_t y = ya; y <= yb; ++y) {
                double ay = a * fy[y];
                double* row = acc + y * nx;
                for (int64_t x = xa; x <= xb; ++x) row[x] += ay * fx[x];
            }
        }
        float* o = J->out + zz * nx * ny;
        for (int64_t i = 0; i < nx * ny; ++i) o[i] = (float)acc[i];
    }
    free(acc); free(fx); free(fy);
    return NULL;
}

/*
 * Fill out[(z - z0)][y][x] for z in [z0, z0 + nzs) with
 *   v = sigma * N(0,1)  (if noise != 0)  +  sum_s A_s * sigma * G_s(x, y, z),
 * evaluated in double precision and rounded once to float.
 */
int synth_cube(uint64_t seed, int64_t nx, int64_t ny, int64_t nz, double sigma,
               const double* src, int64_t nsrc, int noise, int64_t z0, int64_t nzs,
               float* out, int nthreads) {
    if (nx < 1 || ny < 1 || nz < 1 || z0 < 0 || nzs < 0 || z0 + nzs > nz || !out) return -1;
    if (nsrc > 0 && !src) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    job_t jobs[256];
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (job_t){seed, nx, ny, nz, sigma, src, nsrc, z0, nzs, out, noise, t, nthreads};
        if (pthread_create(&th[t], NULL, plane_worker, &jobs[t]) != 0) { rc = -2; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) {
        void* r = NULL;
        pthread_join(th[t], &r);
        if (r) rc = -3;
    }
    return rc;
}
