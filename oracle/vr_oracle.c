/*
 * vr_oracle.c — plain FP64 CPU ray caster.  TEST INFRASTRUCTURE ONLY.
 *
 * This is the reference the GPU renderer is checked against.  It is written to
 * be read against the method, not to be fast: one ray per pixel, every sample
 * evaluated in double precision, no bricks, no empty-space skipping, no tiling.
 * It shares no code, header or table with the GPU path.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * What it computes (paper Sec. 2 design decision 1 and Sec. 3 process step 3:
 * ray-casting volume rendering that maps every output pixel to RGBA through a
 * pre-selected transfer function; the noise clip, compositing model, early
 * termination and maximum-intensity projection follow the renderer's stated
 * hot path):
 *
 *   box      voxel (i,j,k) is centred at integer coordinates (i,j,k) with unit
 *            spacing; the volume occupies [-1/2, N_a - 1/2] on each axis.
 *   rays     pixel (i = column, left to right; j = row, top to bottom).
 *            perspective: f = |target-eye|, r = |f x up|, u = r x f,
 *              h = tan(fovy/2), a = W/H,
 *              d = |f + (2(i+1/2)/W - 1) h a r + (1 - 2(j+1/2)/H) h u|, o = eye.
 *            orthographic: d = f, o = target + ((i+1/2)/W - 1/2) w r
 *              + (1/2 - (j+1/2)/H) h_o u; the ray is the whole line.
 *   slab     t_in/t_out from the ray-box slab test (t_in >= 0 for perspective).
 *   lattice  L = t_out - t_in, n = ceil(L / step) segments; segment k spans
 *            [t_in + k step, min(t_in + (k+1) step, t_out)] and is sampled at
 *            its midpoint; only the last segment can be short.
 *   sample   trilinear: q = clamp(p, 0, N-1), i = min(floor(q), N-2), f = q-i,
 *            lerp(a,b,f) = a + f (b-a) along x, then y, then z.
 *            nearest:   i = clamp(floor(p + 1/2), 0, N-1).
 *   classify v < clip -> (0,0,0,0); else u = clamp((v-v0)/(v1-v0) (n-1), 0, n-1),
 *            i0 = min(floor(u), n-2), g = u - i0, row = lerp(T[i0], T[i0+1], g);
 *            a row is (r, g, b, kappa) with kappa an extinction per unit length.
 *   EA       alpha_k = -expm1(-kappa_k len_k); C += T alpha_k rgb_k;
 *            T *= (1 - alpha_k); after sample k stop if 1 - T >= a_ert.
 *            Output (C_r, C_g, C_b, 1 - T); a miss gives (0,0,0,0).
 *   MIP      m = max_k v_k over the same lattice (no transfer function);
 *            output m if m >= clip else 0; a miss gives -inf.
 *
 * Sub-cube partials (Sec. 3.1, process steps 1 and 4: the cube is split into
 * sub-cubes, each rendered to its own image): with win_axis = a >= 0 only the
 * lattice samples whose position p_a lies in [win_lo, win_hi) are taken, on
 * the lattice of the whole cube (t_in, n and segment lengths unchanged).  The
 * EA partial is (C, 1 - T) of those samples; the MIP partial is m if the
 * window held a sample and m >= clip, -FLT_MAX if it held samples but none
 * at or above the clip, and -inf if it held none.  A pixel with a sample
 * within amb_window of a window edge is flagged: the sample may belong to
 * either neighbour.
 *
 * Besides the image it reports per pixel the nominal sample count n, the
 * number of samples evaluated before early termination, and flags marking
 * pixels whose result depends discontinuously on a quantity within a small
 * margin of a decision threshold (early-termination threshold, a hard clip
 * edge, a nearest-neighbour rounding tie, a grazing ray, the MIP clip floor):
 * there several results are correct, and comparisons treat them separately.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_F16 = 1, ORC_BF16 = 2, ORC_F64 = 3 };
enum { ORC_EA = 0, ORC_MIP = 1 };
enum { ORC_NEAREST = 0, ORC_TRILINEAR = 1 };

enum {
    ORC_FLAG_HIT = 1,
    ORC_FLAG_ERT_AMBIG = 2,
    ORC_FLAG_CLIP_AMBIG = 4,
    ORC_FLAG_NEAREST_AMBIG = 8,
    ORC_FLAG_GRAZE_AMBIG = 16,
    ORC_FLAG_MIPCLIP_AMBIG = 32,
    ORC_FLAG_ERT_STOPPED = 64,
    ORC_FLAG_WINDOW_AMBIG = 128,
};

typedef struct {
    int64_t nx, ny, nz;
    const void* vox;       /* [nz][ny][nx], x fastest */
    int32_t vox_dtype;     /* ORC_F32 / ORC_F16 / ORC_BF16 / ORC_F64 */
    int32_t pad0;
    double vox_scale;      /* value = decode(vox) * vox_scale */
    const double* tf;      /* tf_n rows of (r, g, b, kappa) */
    int32_t tf_n;
    int32_t mode;          /* ORC_EA / ORC_MIP */
    double v0, v1;         /* transfer-function domain */
    double clip;           /* -inf disables */
    int32_t interp;        /* ORC_NEAREST / ORC_TRILINEAR */
    int32_t ortho;
    double step;           /* lattice spacing along the ray */
    double ert;            /* early-termination opacity; >= 1 disables */
    double eye[3], target[3], up[3];
    double fovy_deg, ortho_w, ortho_h;
    int32_t width, height;
    double amb_ert, amb_clip, amb_nearest, amb_graze;  /* flag margins */
    int32_t win_axis;      /* -1: whole ray; 0/1/2: sub-cube window along x/y/z */
    int32_t pad1;
    double win_lo, win_hi; /* window [win_lo, win_hi) of sample positions on win_axis */
    double amb_window;     /* flag margin at window edges */
} orc_scene;

/* --- exact decoding of stored voxels ------------------------------------ */
double orc_decode_f16(uint16_t h) {
    int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m + 1024), e - 25);
    return s ? -v : v;
}

double orc_decode_bf16(uint16_t b) {
    uint32_t w = (uint32_t)b << 16;
    float f;
    memcpy(&f, &w, 4);
    return (double)f;
}

static inline double voxel(const orc_scene* S, int64_t x, int64_t y, int64_t z) {
    int64_t idx = (z * S->ny + y) * S->nx + x;
    double v;
    switch (S->vox_dtype) {
        case ORC_F32: v = (double)((const float*)S->vox)[idx]; break;
        case ORC_F16: v = orc_decode_f16(((const uint16_t*)S->vox)[idx]); break;
        case ORC_BF16: v = orc_decode_bf16(((const uint16_t*)S->vox)[idx]); break;
        default: v = ((const double*)S->vox)[idx]; break;
    }
    return v * S->vox_scale;
}

/* --- small vector helpers ------------------------------------------------ */
static void vsub(const double a[3], const double b[3], double o[3]) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void vcross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void vnorm(double a[3]) {
    double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* Camera basis: forward f, right r, up u. */
static void basis(const orc_scene* S, double f[3], double r[3], double u[3]) {
    vsub(S->target, S->eye, f);
    vnorm(f);
    vcross(f, S->up, r);
    vnorm(r);
    vcross(r, f, u);
}

/* Ray origin o and unit direction d for pixel (i, j). */
void orc_pixel_ray(const orc_scene* S, int64_t i, int64_t j, double o[3], double d[3]) {
    double f[3], r[3], u[3];
    basis(S, f, r, u);
    double W = (double)S->width, H = (double)S->height;
    if (S->ortho) {
        double sx = ((i + 0.5) / W - 0.5) * S->ortho_w;
        double sy = (0.5 - (j + 0.5) / H) * S->ortho_h;
        for (int a = 0; a < 3; ++a) {
            o[a] = S->target[a] + sx * r[a] + sy * u[a];
            d[a] = f[a];
        }
    } else {
        double h = tan(0.5 * S->fovy_deg * (3.14159265358979323846 / 180.0));
        double asp = W / H;
        double x = (2.0 * (i + 0.5) / W - 1.0) * h * asp;
        double y = (1.0 - 2.0 * (j + 0.5) / H) * h;
        for (int a = 0; a < 3; ++a) {
            o[a] = S->eye[a];
            d[a] = f[a] + x * r[a] + y * u[a];
        }
        vnorm(d);
    }
}

/* Slab test against [-1/2, N-1/2]^3.  Returns 1 on a hit. */
int orc_slab(const orc_scene* S, const double o[3], const double d[3], double* t_in,
             double* t_out) {
    double lo = -0.5;
    double hi[3] = {(double)S->nx - 0.5, (double)S->ny - 0.5, (double)S->nz - 0.5};
    double tin = S->ortho ? -INFINITY : 0.0, tout = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double t0 = (lo - o[a]) / d[a], t1 = (hi[a] - o[a]) / d[a];
            double tmin = t0 < t1 ? t0 : t1, tmax = t0 < t1 ? t1 : t0;
            if (tmin > tin) tin = tmin;
            if (tmax < tout) tout = tmax;
        } else if (o[a] < lo || o[a] > hi[a]) {
            return 0;
        }
    }
    if (!(tout > tin)) return 0;
    *t_in = tin;
    *t_out = tout;
    return 1;
}

static inline double clampd(double x, double lo, double hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}
static inline double lerp(double a, double b, double f) { return a + f * (b - a); }

/* Sample value at p; sets *tie when nearest rounding is within the margin of a
 * tie.  For nearest sampling, *vlo and *vhi (when non-NULL) receive the least
 * and greatest value over every voxel a tied coordinate could round to (both
 * equal the sample when there is no tie): the set of correct samples. */
static double sample(const orc_scene* S, const double p[3], int* tie, double* vlo, double* vhi) {
    const int64_t N[3] = {S->nx, S->ny, S->nz};
    if (S->interp == ORC_NEAREST) {
        int64_t i[3], alt[3];
        for (int a = 0; a < 3; ++a) {
            double s = p[a] + 0.5;
            double fl = floor(s);
            double fr = s - fl;
            int64_t k = (int64_t)fl;
            int64_t k2 = k;
            if (s > 0.0 && s < (double)N[a] && (fr < S->amb_nearest || fr > 1.0 - S->amb_nearest)) {
                *tie = 1;
                k2 = fr < 0.5 ? k - 1 : k + 1;  /* the other side of the tie */
            }
            if (k < 0) k = 0;
            if (k > N[a] - 1) k = N[a] - 1;
            if (k2 < 0) k2 = 0;
            if (k2 > N[a] - 1) k2 = N[a] - 1;
            i[a] = k;
            alt[a] = k2;
        }
        double v = voxel(S, i[0], i[1], i[2]);
        if (vlo && vhi) {
            double lo = v, hi = v;
            for (int c = 1; c < 8; ++c) {
                double w = voxel(S, (c & 1) ? alt[0] : i[0], (c & 2) ? alt[1] : i[1],
                                 (c & 4) ? alt[2] : i[2]);
                if (w < lo) lo = w;
                if (w > hi) hi = w;
            }
            *vlo = lo;
            *vhi = hi;
        }
        return v;
    }
    int64_t i[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double q = clampd(p[a], 0.0, (double)(N[a] - 1));
        int64_t k = (int64_t)floor(q);
        if (k > N[a] - 2) k = N[a] - 2;
        i[a] = k;
        f[a] = q - (double)k;
    }
    double c000 = voxel(S, i[0], i[1], i[2]), c100 = voxel(S, i[0] + 1, i[1], i[2]);
    double c010 = voxel(S, i[0], i[1] + 1, i[2]), c110 = voxel(S, i[0] + 1, i[1] + 1, i[2]);
    double c001 = voxel(S, i[0], i[1], i[2] + 1), c101 = voxel(S, i[0] + 1, i[1], i[2] + 1);
    double c011 = voxel(S, i[0], i[1] + 1, i[2] + 1), c111 = voxel(S, i[0] + 1, i[1] + 1, i[2] + 1);
    double x00 = lerp(c000, c100, f[0]), x10 = lerp(c010, c110, f[0]);
    double x01 = lerp(c001, c101, f[0]), x11 = lerp(c011, c111, f[0]);
    double y0 = lerp(x00, x10, f[1]), y1 = lerp(x01, x11, f[1]);
    double v = lerp(y0, y1, f[2]);
    if (vlo && vhi) *vlo = *vhi = v;
    return v;
}

/* Transfer-function row (r, g, b, kappa) for value v (no clip). */
void orc_classify(const orc_scene* S, double v, double out[4]) {
    int n = S->tf_n;
    double u = clampd((v - S->v0) / (S->v1 - S->v0) * (double)(n - 1), 0.0, (double)(n - 1));
    int i0 = (int)floor(u);
    if (i0 > n - 2) i0 = n - 2;
    double g = u - (double)i0;
    for (int c = 0; c < 4; ++c) out[c] = lerp(S->tf[4 * i0 + c], S->tf[4 * (i0 + 1) + c], g);
}

/* One ray.  out: 4 doubles (EA) or 1 (MIP).  bounds (MIP, nullable): the least
 * and greatest maximum over the correct choices at nearest-sampling ties. */
void orc_ray(const orc_scene* S, int64_t pi, int64_t pj, double* out, int64_t* n_nominal,
             int64_t* n_exec, int32_t* flags, double* bounds) {
    double o[3], d[3], tin, tout;
    int32_t fl = 0;
    int64_t nn = 0, ne = 0;
    orc_pixel_ray(S, pi, pj, o, d);
    const int mip = S->mode == ORC_MIP;
    if (!orc_slab(S, o, d, &tin, &tout)) {
        if (mip) out[0] = -INFINITY;
        else out[0] = out[1] = out[2] = out[3] = 0.0;
        if (bounds) bounds[0] = bounds[1] = -INFINITY;
        goto done;
    }
    fl |= ORC_FLAG_HIT;
    {
        const double L = tout - tin, step = S->step;
        const int64_t n = (int64_t)ceil(L / step);
        nn = n;
        if (L < S->amb_graze) fl |= ORC_FLAG_GRAZE_AMBIG;
        /* kappa of the transfer function exactly at the clip: a jump there
         * makes samples near the clip ambiguous */
        double rc[4] = {0, 0, 0, 0};
        int clip_jump = 0;
        if (!mip && isfinite(S->clip)) {
            orc_classify(S, S->clip, rc);
            clip_jump = rc[3] > 0.0;
        }
        double C[3] = {0.0, 0.0, 0.0}, T = 1.0, m = -INFINITY, m_lo = -INFINITY, m_hi = -INFINITY;
        const int win = S->win_axis >= 0 && S->win_axis < 3;
        int64_t in_window = 0;
        if (win) nn = 0;
        for (int64_t k = 0; k < n; ++k) {
            double a = tin + (double)k * step;
            double b = tin + (double)(k + 1) * step;
            if (b > tout) b = tout;
            double len = b - a;
            double tm = a + 0.5 * len;
            double p[3] = {o[0] + tm * d[0], o[1] + tm * d[1], o[2] + tm * d[2]};
            if (win) {
                const double pa = p[S->win_axis];
                if (fabs(pa - S->win_lo) < S->amb_window || fabs(pa - S->win_hi) < S->amb_window)
                    fl |= ORC_FLAG_WINDOW_AMBIG;
                if (!(pa >= S->win_lo && pa < S->win_hi)) continue;
                ++in_window;
                ++nn;
            }
            int tie = 0;
            double vlo, vhi;
            double v = sample(S, p, &tie, &vlo, &vhi);
            if (tie) fl |= ORC_FLAG_NEAREST_AMBIG;
            ++ne;
            if (mip) {
                if (v > m) m = v;
                if (vlo > m_lo) m_lo = vlo;
                if (vhi > m_hi) m_hi = vhi;
                continue;
            }
            if (clip_jump && fabs(v - S->clip) < S->amb_clip * fmax(1.0, fabs(S->clip)))
                fl |= ORC_FLAG_CLIP_AMBIG;
            if (v < S->clip) continue; /* classified (0,0,0,0): contributes nothing */
            double row[4];
            orc_classify(S, v, row);
            double alpha = -expm1(-row[3] * len);
            for (int c = 0; c < 3; ++c) C[c] += T * alpha * row[c];
            T *= (1.0 - alpha);
            if (fabs((1.0 - T) - S->ert) < S->amb_ert) fl |= ORC_FLAG_ERT_AMBIG;
            if (1.0 - T >= S->ert) {
                fl |= ORC_FLAG_ERT_STOPPED;
                break;
            }
        }
        if (mip) {
            if (isfinite(S->clip) && fabs(m - S->clip) < S->amb_clip * fmax(1.0, fabs(S->clip)))
                fl |= ORC_FLAG_MIPCLIP_AMBIG;
            if (win) out[0] = in_window ? ((m >= S->clip) ? m : -3.4028234663852886e38) : -INFINITY;
            else out[0] = (m >= S->clip) ? m : 0.0;
            if (bounds) {
                bounds[0] = m_lo;
                bounds[1] = m_hi;
            }
        } else {
            out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
        }
    }
done:
    if (n_nominal) *n_nominal = nn;
    if (n_exec) *n_exec = ne;
    if (flags) *flags = fl;
}

/* --- threaded driver ------------------------------------------------------ */
typedef struct {
    const orc_scene* S;
    int64_t npix;
    const int32_t* px;   /* (i, j) pairs or NULL for the full image in row order */
    double* out;
    int64_t* nn;
    int64_t* ne;
    int32_t* flags;
    double* bounds;
    volatile int64_t* next;
} drv_t;

#define ORC_CHUNK 64

static void* drv_worker(void* arg) {
    drv_t* D = (drv_t*)arg;
    const int ch = D->S->mode == ORC_MIP ? 1 : 4;
    for (;;) {
        int64_t s = __sync_fetch_and_add(D->next, (int64_t)ORC_CHUNK);
        if (s >= D->npix) break;
        int64_t e = s + ORC_CHUNK < D->npix ? s + ORC_CHUNK : D->npix;
        for (int64_t p = s; p < e; ++p) {
            int64_t i, j;
            if (D->px) { i = D->px[2 * p]; j = D->px[2 * p + 1]; }
            else { i = p % D->S->width; j = p / D->S->width; }
            orc_ray(D->S, i, j, D->out + ch * p, D->nn ? D->nn + p : NULL,
                    D->ne ? D->ne + p : NULL, D->flags ? D->flags + p : NULL,
                    D->bounds ? D->bounds + 2 * p : NULL);
        }
    }
    return NULL;
}

/*
 * Render npix pixels (px = NULL: the whole width x height image in row-major
 * order).  out holds 4 doubles per pixel (EA) or 1 (MIP).  Optional per-pixel
 * outputs: nominal sample count, executed sample count, flags, and (MIP) the
 * bounds of the correct maxima at nearest-sampling ties (2 doubles).
 * Returns 0, or -1 on invalid arguments.
 */
int orc_render(const orc_scene* S, int64_t npix, const int32_t* px, double* out,
               int64_t* n_nominal, int64_t* n_exec, int32_t* flags, double* bounds,
               int nthreads) {
    if (!S || !out || !S->vox || S->nx < 2 || S->ny < 2 || S->nz < 2) return -1;
    if (S->width < 1 || S->height < 1 || !(S->step > 0.0)) return -1;
    if (S->mode == ORC_EA && (!S->tf || S->tf_n < 2 || !(S->v1 > S->v0))) return -1;
    if (!px) npix = (int64_t)S->width * S->height;
    if (px) {
        for (int64_t p = 0; p < npix; ++p)
            if (px[2 * p] < 0 || px[2 * p] >= S->width || px[2 * p + 1] < 0 ||
                px[2 * p + 1] >= S->height)
                return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    volatile int64_t next = 0;
    drv_t D = {S, npix, px, out, n_nominal, n_exec, flags, bounds, &next};
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, drv_worker, &D) != 0) break;
        ++started;
    }
    if (started == 0) drv_worker(&D);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    return 0;
}
