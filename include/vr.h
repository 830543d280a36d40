/*
 * vr.h — C interface of the MI355X volume renderer for noisy spectral cubes.
 *
 * The renderer casts one ray per output pixel through an (x, y, frequency)
 * data cube and maps each pixel to RGBA through a pre-selected transfer
 * function (paper Sec. 3, "Framework Modules", process step 3; ray casting is
 * design decision 1 of Sec. 2).  Samples are trilinear (or nearest), values
 * below a noise clip k*sigma are treated as empty (the paper's attention to
 * low signal-to-noise data, abstract), and samples are composited front to
 * back under the emission-absorption model with early ray termination, or
 * reduced by maximum-intensity projection.  The calls below follow the
 * paper's thin-client model: the user turns interaction into rendering
 * commands (Fig. 1 caption): upload a cube, set the transfer function and
 * noise clip, set the camera, render.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Cube layout: voxel (x, y, z) of an nx*ny*nz cube lives at linear index
 *    (z*ny + y)*nx + x (x fastest; a stack of channel images).  Voxel centres
 *    sit at integer coordinates, unit spacing; the cube occupies
 *    [-1/2, n-1/2] on each axis.  Samples outside [0, n-1] clamp to the edge.
 *  * Pixels: column i left to right, row j top to bottom; an image is stored
 *    row-major, [height][width][4] float32 premultiplied RGBA (emission-
 *    absorption) or [height][width] float32 (MIP, data units; -inf where the
 *    ray misses the cube, 0 where the maximum is below the clip).
 *  * Perspective ray for pixel (i,j): f = |target-eye|, r = |f x up|,
 *    u = r x f, h = tan(fovy/2), a = width/height,
 *    d = |f + (2(i+1/2)/W - 1) h a r + (1 - 2(j+1/2)/H) h u|, origin eye,
 *    sampled for t >= 0.  Orthographic: d = f, origin target + ((i+1/2)/W -
 *    1/2) ortho_w r + (1/2 - (j+1/2)/H) ortho_h u; the whole line is sampled.
 *  * Sample lattice: with [t_in, t_out] the ray's chord through the cube and
 *    L its length, n = ceil(L/step) segments of length step (the last one
 *    shorter), each sampled at its midpoint.
 *  * Transfer function: n >= 2 rows (r, g, b, kappa), kappa an extinction
 *    coefficient per voxel length, spread evenly over [v0, v1] in data units
 *    and interpolated linearly (clamped outside).  A sample value v below the
 *    clip c contributes nothing.  Per segment alpha = 1 - exp(-kappa len);
 *    C += T alpha rgb; T *= 1 - alpha; the ray stops once 1 - T >= ert_alpha.
 *
 * Ownership and threading
 * -----------------------
 *  * The library owns brick pools, statistics, skip masks and transfer-
 *    function tables.  They are allocated through the optional allocator
 *    given to vr_create (e.g. a framework's caching allocator), otherwise
 *    with hipMalloc.  Callers own every buffer they pass in.
 *  * Device pointers passed in (out_dev, device-resident sources) must be
 *    valid on the context's device; hip_stream arguments are hipStream_t
 *    values (NULL = the default stream).
 *  * Calls on one context are serialised by an internal mutex; a context may
 *    be used from several threads.
 *  * vr_render snapshots the context's transfer function, clip and camera at
 *    call time; later set_* calls never affect work already enqueued.
 *
 * Errors
 * ------
 *  Every call returns a vr_status; no C++ exception or abort crosses this
 *  interface.  Arguments are validated before any device call.  On failure
 *  vr_last_error() describes the most recent error of the calling thread.
 *  An asynchronous device fault is reported as VR_EDEVICE by the next call
 *  that synchronises; the context must then be destroyed.
 */
#ifndef VR_H
#define VR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vr_ctx_s* vr_ctx;
typedef int32_t vr_cube;   /* cube handle, > 0; stale handles give VR_ENOTFOUND */
typedef int32_t vr_tf;     /* transfer-function handle, > 0 */
typedef int32_t vr_status;

enum {
    VR_OK = 0,
    VR_EINVAL = -1,       /* invalid argument (nothing was changed) */
    VR_ENOMEM = -2,       /* device memory or the context's budget is exhausted */
    VR_ENOTFOUND = -3,    /* unknown or released handle */
    VR_EBUSY = -4,        /* object in use by queued work */
    VR_EDEVICE = -5,      /* HIP error, or a host-only context asked for device work */
    VR_EUNSUPPORTED = -6, /* valid but not supported combination */
    VR_ESTATE = -7        /* a required piece of state (camera, transfer function) is unset */
};

enum { VR_F32 = 0, VR_F16 = 1, VR_BF16 = 2 };         /* voxel storage formats */
enum { VR_EA = 0, VR_MIP = 1 };                       /* render modes */
enum { VR_NEAREST = 0, VR_TRILINEAR = 1 };            /* interpolation */

/* Optional device allocator.  alloc returns device memory of at least
 * `bytes` bytes (256-byte aligned) or NULL; free releases it.  Both may be
 * called from any thread that calls into the library. */
typedef struct {
    void* (*alloc)(uint64_t bytes, void* user);
    void (*free)(void* ptr, uint64_t bytes, void* user);
    void* user;
} vr_allocator;

typedef struct {
    int32_t ortho;              /* 0 perspective, 1 orthographic */
    int32_t reserved;
    double eye[3];              /* voxel coordinates */
    double target[3];
    double up[3];               /* must not be parallel to target - eye */
    double fovy_deg;            /* perspective: vertical field of view, (0, 180) */
    double ortho_w, ortho_h;    /* orthographic: window size in voxels, > 0 */
} vr_camera;

typedef struct {
    int32_t mode;               /* VR_EA or VR_MIP */
    int32_t interp;             /* VR_NEAREST or VR_TRILINEAR */
    float step;                 /* lattice spacing along rays in voxels, > 0 */
    float ert_alpha;            /* early termination opacity in (0, 1]; > 1 disables */
    int32_t width, height;      /* 1 .. 16384 */
    int32_t use_skip;           /* 1: skip empty space (never changes the image), 0: off */
    int32_t reserved;
} vr_render_params;

typedef struct {
    uint64_t samples_nominal;   /* sum over pixels of the lattice size n */
    uint64_t samples_exec;      /* samples actually interpolated */
    uint64_t rays_hit;          /* rays that intersect the cube */
    uint64_t rays_ert;          /* rays stopped by early termination */
    uint64_t cells_skipped;     /* empty cells jumped over */
    float kernel_ms;            /* device time of the render kernel */
    float reserved;
} vr_stats;

typedef struct {
    int64_t nx, ny, nz;
    int32_t storage;            /* VR_F32 / VR_F16 / VR_BF16 */
    int32_t brick;              /* brick edge in voxels (32) */
    int32_t bricks_x, bricks_y, bricks_z;
    int32_t cell;               /* skip-cell edge in voxels (8) */
    double sigma_scale;         /* stored value = value / sigma_scale */
    uint64_t pool_bytes;        /* device bytes of the brick pool */
    uint64_t brick_stride;      /* bytes between brick slots */
    uint64_t aux_bytes;         /* device bytes of tables and statistics */
    float vmin, vmax;           /* range of stored values times sigma_scale */
    int32_t x_chunks;           /* 16-byte chunks of x per slot row (9 float32, 5 16-bit) */
    uint8_t resident;           /* 1 if the bricks are in device memory now */
    uint8_t registered;         /* 1 if registered with a host source (vr_cube_register) */
    uint16_t reserved;
    /* device pointers, NULL while a registered cube is not resident: */
    const void* pool;           /* brick slots; slot of brick (bx,by,bz) is
                                   (bz*bricks_y + by)*bricks_x + bx.  A slot holds local voxels
                                   lx < 16*x_chunks/elem, ly < 36, lz < 34, each the
                                   edge-clamped value of global voxel (32bx+lx, 32by+ly, 32bz+lz),
                                   in 128-byte lines of one x chunk by 4 y by 2 z: with
                                   cv = 16/elem elements per chunk, voxel (lx,ly,lz) is element
                                   (((lz/2)*9 + ly/4)*x_chunks + lx/cv)*8*cv
                                   + ((lz%2)*4 + ly%4)*cv + lx%cv */
    const float* cell_minmax;   /* per slot: 64 cells x (min, max) of stored values; cell
                                   (cx,cy,cz) in [0,3]^3 is entry (cz*4 + cy)*4 + cx and covers
                                   local voxels [8c, 8c+8] per axis */
} vr_cube_info;

/* --- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context's cubes may hold, their brick pools and per-cell
 * statistics (0 = no cap; skip masks, about 0.01 % of a pool, and scratch are
 * not counted).  Uploaded cubes count until released; registered cubes
 * (vr_cube_register) are admitted and evicted within the cap.  device = -1
 * creates a host-only context that validates arguments and keeps state but
 * rejects device work with VR_EDEVICE.  alloc may be NULL. */
vr_status vr_create(int32_t device, uint64_t hbm_budget_bytes, const vr_allocator* alloc,
                    vr_ctx* out);

/* Destroy a context, its cubes, tables and server.  Waits for queued work. */
vr_status vr_destroy(vr_ctx ctx);

/* Text of the calling thread's most recent error; valid until its next call. */
const char* vr_last_error(void);

/* Library version string. */
const char* vr_version(void);

/* --- cubes ---------------------------------------------------------------- */

/* Upload an nx*ny*nz cube (each >= 2).  src holds values of type src_dtype
 * (VR_F32, or codes of VR_F16/VR_BF16 that are stored as-is and then require
 * storage == src_dtype), in host memory (src_on_device = 0) or device memory
 * (1).  Float32 sources are converted to `storage` as round-to-nearest-even
 * of value/sigma_scale.  The cube is re-laid out into 32^3 bricks with a one-
 * voxel apron and per-8^3-cell min/max tables
 * (paper Sec. 3 process step 1: the cube is partitioned into sub-cubes).
 * Returns after src may be reused; the cube is ready for work on any stream
 * once this call returns. */
vr_status vr_cube_upload(vr_ctx ctx, const void* src, int32_t src_dtype, int32_t src_on_device,
                         int64_t nx, int64_t ny, int64_t nz, int32_t storage, double sigma_scale,
                         void* hip_stream, vr_cube* out);

/* Register a cube whose voxels stay in caller-owned host memory: src, nx, ny,
 * nz, src_dtype, storage and sigma_scale as for vr_cube_upload from host
 * memory.  Nothing is uploaded yet.  Whenever a render, batch or served
 * request needs the cube and it is not resident, the library admits it:
 * within the context's memory budget it evicts idle registered cubes, least
 * recently used first (their host copies stay with the caller), and uploads
 * this one.  A served request whose cube cannot be admitted while other
 * requests hold device memory waits in the queue until memory frees up; the
 * scheduler lets requests for resident cubes pass it for a few launches and
 * then drains the device for it, so no request starves.  This is the one-GPU
 * form of the paper's scheduling of sub-cubes of data larger than a single
 * GPU's memory onto the available GPUs (Sec. 2; Sec. 3.1, process steps 1-2).
 * A cube whose bricks alone exceed the budget is streamed instead (the
 * paper's data larger than GPU memory, abstract and Sec. 2): on first use it
 * is bricked into pinned host memory (the cell statistics stay on the
 * device), and vr_render renders it as sub-cubes of brick layers uploaded in
 * turn, two device buffers in flight, each rendered to a partial image on the
 * whole cube's lattice and integrated front to back (as vr_render_subcube and
 * vr_composite); early termination then acts within each sub-cube.  The two
 * buffers stay allocated between frames (they count against the budget and
 * give way, after other cubes' coarse levels, when an upload or admission
 * needs room, and to this cube's own coarse levels), and
 * consecutive frames take the sub-cubes in opposite orders so that a frame
 * starts on the two the frame before left on the device.  Streamed cubes are
 * rendered by vr_render only (VR_EUNSUPPORTED for batches and served
 * requests).  The caller keeps src unchanged and valid until
 * vr_cube_release.  Errors: VR_EINVAL / VR_EUNSUPPORTED as for vr_cube_upload;
 * VR_ENOMEM if even the statistics and two buffers of two brick layers
 * exceed the budget (vr_render of a streamed cube: also when the budget would
 * cut it into more than 64 sub-cubes). */
vr_status vr_cube_register(vr_ctx ctx, const void* src, int32_t src_dtype, int64_t nx, int64_t ny,
                           int64_t nz, int32_t storage, double sigma_scale, vr_cube* out);

/* --- noise-aware form --------------------------------------------------------
 * The noise of a spectral cube varies with frequency, and the paper gives
 * special attention to data of low signal-to-noise ratio (abstract; Sec. 2).
 * These calls estimate each channel's noise and store the cube in units of
 * it, so that the clip k of vr_set_noise_clip(k, 1) removes everything below
 * k*sigma(nu) channel by channel, and transfer functions are given in S/N. */

/* Robust noise level of every frequency channel (z plane) of an nx*ny*nz
 * float32 cube (x fastest) in host (src_on_device = 0) or device memory:
 * median = the lower median of the channel's nx*ny values (order statistic
 * floor((n-1)/2)), mad = the lower median of |v - median| (float32
 * deviations), sigma = 1.4826 * mad.  Computed on the device (exact order
 * statistics); each output is a host array of nz floats, any may be NULL.
 * Values must be finite.  Returns once the outputs are written.  Errors:
 * VR_EINVAL (NULL src, nx*ny >= 2^31, nz > 65536), VR_EDEVICE. */
vr_status vr_estimate_channel_noise(vr_ctx ctx, const float* src, int32_t src_on_device, int64_t nx,
                                    int64_t ny, int64_t nz, void* hip_stream, float* median_out,
                                    float* mad_out, float* sigma_out);

/* Upload a float32 cube as vr_cube_upload does, storing value / divisor[z]
 * (round to nearest even for 16-bit storage) with one positive divisor per
 * channel (host array of nz floats, e.g. the sigma of
 * vr_estimate_channel_noise).  The cube's data units are then units of each
 * channel's divisor: transfer-function domains, clips and MIP outputs are in
 * those units (sigma_scale is 1).  Errors as for vr_cube_upload; VR_EINVAL
 * for a divisor that is not positive and finite. */
vr_status vr_cube_upload_scaled(vr_ctx ctx, const float* src, int32_t src_on_device, int64_t nx,
                                int64_t ny, int64_t nz, int32_t storage, const float* channel_divisor,
                                void* hip_stream, vr_cube* out);

/* Release a cube.  VR_EBUSY if queued serving requests still reference it. */
vr_status vr_cube_release(vr_ctx ctx, vr_cube cube);

typedef struct {
    uint64_t budget_bytes;      /* the context's cap (0: none) */
    uint64_t used_bytes;        /* device bytes counted against the budget */
    uint64_t cubes;             /* live cube handles */
    uint64_t resident_cubes;    /* of which resident in device memory */
    uint64_t registered_cubes;  /* of which registered with a host source */
    uint64_t uploads;           /* on-demand admissions of registered cubes so far */
    uint64_t evictions;         /* registered cubes evicted to make room so far */
} vr_memory_stats;

/* Memory accounting of a context (admission and eviction counters). */
vr_status vr_get_memory_stats(vr_ctx ctx, vr_memory_stats* out);

/* Describe a cube (sizes, layout, device pointers for inspection). */
vr_status vr_cube_get_info(vr_ctx ctx, vr_cube cube, vr_cube_info* out);

/* --- transfer function, clip, camera --------------------------------------- */

/* Set the context's transfer function: rgbk holds n rows (r, g, b, kappa),
 * n in [2, 4096], finite, kappa >= 0, spread over [v0, v1] (v1 > v0, data
 * units).  The table is copied.  This is the pre-selected transfer function
 * through which every pixel's ray is mapped to RGBA (paper Sec. 3.1, process
 * step 3).  Errors: VR_EINVAL for a NULL table or any rule above broken. */
vr_status vr_set_transfer_function(vr_ctx ctx, const float* rgbk, int32_t n, float v0, float v1);

/* Set the noise clip c = k * sigma (data units).  k = -inf disables it.
 * sigma > 0 and finite.  Sample values below c are treated as noise and
 * contribute nothing (EA), or leave a zero pixel when the whole ray stays
 * below it (MIP): the paper's attention to data of low signal-to-noise ratio
 * (abstract; Sec. 2).  Errors: VR_EINVAL for NaN or +inf k, or a sigma that
 * is not positive and finite. */
vr_status vr_set_noise_clip(vr_ctx ctx, float k, float sigma);

/* Set the camera (validated: finite, up not parallel to the view direction,
 * perspective fovy in (0, 180), orthographic window > 0).  The camera is
 * the user's view of the cube, turned into a rendering command by the thin
 * client (paper Fig. 1 caption).  Errors: VR_EINVAL. */
vr_status vr_set_camera(vr_ctx ctx, const vr_camera* cam);

/* --- rendering ----------------------------------------------------------- */

/* Render `cube` with the context's current state into out_dev (device
 * memory of width*height*4 floats for VR_EA, width*height floats for
 * VR_MIP), enqueued on hip_stream.  One ray is cast per pixel (ray casting
 * is design decision 1 of the paper's Sec. 2; each pixel is mapped to RGBA
 * through the transfer function, Sec. 3.1 process step 3).  With stats !=
 * NULL the call waits for the render and fills the counters; otherwise it
 * returns once enqueued.  The caller keeps out_dev alive until hip_stream
 * has reached the render.  Errors: VR_EINVAL (parameters, NULL out_dev),
 * VR_ENOTFOUND (cube), VR_ESTATE if the camera (or, for VR_EA, the transfer
 * function) is unset, VR_EDEVICE on a HIP error. */
vr_status vr_render(vr_ctx ctx, vr_cube cube, const vr_render_params* params, void* out_dev,
                    void* hip_stream, vr_stats* stats);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): vr_render without
 * stats, calling no allocator.  Its dispatch-order scratch is a fixed array of
 * 1 MiB + 1 KiB in device memory (one per GPU, held until the process ends),
 * enough for 262144 tiles of 16x16 pixels (8192 x 8192).  Requires that the cube is
 * resident and that a vr_render of the same cube (same mode, transfer
 * function and clip, for its skip mask) already ran on this hip_stream, so
 * every object it reads is tracked there.  All calls on one GPU share the
 * scratch: calls that overlap on one GPU (other streams, other contexts)
 * race.  Images equal vr_render's bit for bit.  Errors: as vr_render;
 * VR_EINVAL for an image of more tiles than the scratch holds; VR_ESTATE if
 * the cube, transfer function or skip mask was not prepared on this stream. */
vr_status vr_render_noalloc(vr_ctx ctx, vr_cube cube, const vr_render_params* params,
                            void* out_dev, void* hip_stream);

/* --- sub-cubes and scene integration ---------------------------------------
 * The paper splits a cube into sub-cubes, renders each sub-cube to its own
 * image and integrates the images into the scene (Sec. 3.1, process steps 1,
 * 4 and 5); across GPUs the partials would travel to one compositor. */

/* Render the partial image of the sub-cube of voxel planes [plane_lo,
 * plane_hi) along `axis` (0 x, 1 y, 2 z): of each ray's lattice on the WHOLE
 * cube (t_in, n and segment lengths as for vr_render) only the samples whose
 * position on the axis lies in [plane_lo - 1/2, plane_hi - 1/2) are taken (the
 * window is open below when plane_lo = 0 and above when plane_hi is the axis
 * size), so the partials of sub-cubes that tile the axis take every sample
 * exactly once.  Only voxels of planes [plane_lo - 1, plane_hi] are read.
 * EA: premultiplied RGBA of those samples, (0,0,0,0) without any; early
 * termination acts within the partial.  MIP: the maximum times sigma_scale if
 * the window held a sample at or above the clip, -FLT_MAX if it held samples
 * but none reached the clip, -inf if it held none.  Other arguments, stats
 * and errors as for vr_render; VR_EINVAL unless 0 <= plane_lo < plane_hi <=
 * the axis size. */
vr_status vr_render_subcube(vr_ctx ctx, vr_cube cube, const vr_render_params* params, int32_t axis,
                            int32_t plane_lo, int32_t plane_hi, void* out_dev, void* hip_stream,
                            vr_stats* stats);

/* Integrate `count` (1..64) partial images of width x height pixels (device
 * pointers in a host array, sub-cubes in increasing plane order along `axis`)
 * into out_dev: VR_EA partials by front-to-back "over", C = C_front +
 * (1 - A_front) C_back, in the order each pixel's ray (from the context's
 * camera) crosses the sub-cubes; VR_MIP partials by their maximum, -FLT_MAX
 * becoming 0 (the clip floor).  With ERT off, the composite of a split
 * equals vr_render's image up to float rounding.  Enqueued on hip_stream.
 * Errors: VR_EINVAL (NULL pointers, count, axis or size out of range),
 * VR_ESTATE (EA without a camera), VR_EDEVICE. */
vr_status vr_composite(vr_ctx ctx, int32_t mode, const float* const* partials, int32_t count,
                       int32_t axis, int32_t width, int32_t height, void* out_dev, void* hip_stream);

/* --- progressive (coarse-to-fine) rendering ----------------------------------
 * The paper's thin client turns user interaction into rendering commands and
 * shows the results (Fig. 1 caption; Sec. 3.1, process step 4).  For such an
 * interactive loop, vr_render_progressive renders a view at a level L: an
 * image of ceil(W/2^L) x ceil(H/2^L) pixels of the level-L cube, enlarged to
 * W x H by pixel replication (output pixel (i, j) shows level pixel
 * (i >> L, j >> L)).  The level-L cube averages 2x2x2 blocks of level L - 1
 * (ceil(n/2) voxels per axis; an odd axis repeats its last voxel), float32,
 * built on the first call that needs it and kept with the cube (its device
 * memory counts against the budget and is the first to go when an upload or
 * admission needs room); level voxel (X, Y, Z) is centred at (2^L X +
 * (2^L - 1)/2, ...) of the cube, the camera is carried into level
 * coordinates and the extinction scaled by 2^L, so the level renders the same
 * rays through the same medium at 1/8^L of the samples.  A streamed cube
 * (larger than the budget) gets its level 1 from its pinned bricks, three
 * brick layers at a time, its sub-cube buffers giving way; its levels stay
 * while it is rendered, and go when two sub-cubes no longer fit beside them.
 * Where the level-L cube cannot be used (an axis below two voxels at that
 * level, no room in the budget) the level renders the full cube with a
 * lattice step 2^L times longer instead, and level_cube reports 0.  On a new view
 * (cube, parameters, camera, transfer function, clip or out_dev changed since
 * the previous call) it takes the finest level whose time, predicted from the
 * device time per sample measured on earlier calls, fits budget_ms (the
 * coarsest, max_level, when nothing is known yet or nothing fits; level 0
 * when budget_ms <= 0).  On the same view each call renders the next finer
 * level; once level 0 is shown, a call renders nothing and reports
 * converged = 1.  Level 0 is exactly vr_render's image.  The call waits for
 * the frame.  Errors: as vr_render; VR_EINVAL for max_level outside [0, 4] or
 * a non-finite budget. */
typedef struct {
    int32_t level;              /* level rendered by this call */
    int32_t converged;          /* 1: level 0 was already shown; nothing rendered */
    float ms;                   /* device time of this call (render and enlargement) */
    float predicted_ms;         /* predicted time of the level rendered */
    uint64_t samples_nominal;   /* lattice samples of the level rendered */
    int32_t level_cube;         /* 1: rendered from the level-L cube; 0: full cube */
} vr_progressive_info;

vr_status vr_render_progressive(vr_ctx ctx, vr_cube cube, const vr_render_params* params,
                                double budget_ms, int32_t max_level, void* out_dev,
                                void* hip_stream, vr_progressive_info* info);

/* --- batched rendering and serving ---------------------------------------- */

/* Transfer functions as objects, for requests that carry their own
 * (rules and citation as for vr_set_transfer_function).  vr_tf_release gives
 * VR_EBUSY while queued requests or the context's current state hold it. */
vr_status vr_tf_create(vr_ctx ctx, const float* rgbk, int32_t n, float v0, float v1, vr_tf* out);
vr_status vr_tf_release(vr_ctx ctx, vr_tf tf);

/* One view request.  tf = 0 uses the context's current transfer function;
 * clip is in data units (-inf: none). */
typedef struct {
    vr_cube cube;
    vr_tf tf;
    float clip;
    int32_t reserved;
    vr_camera camera;
    vr_render_params params;
    void* out_dev;              /* as for vr_render */
} vr_request;

/* Render `count` requests (up to 4096; any mix of cubes, sizes, modes) on
 * hip_stream: one persistent launch per class of requests present (a class is
 * a (mode, storage, interpolation) triple, each with its own specialised
 * kernel), the requests of a class taken in order, each request's tiles most
 * expensive first.  Each image equals what the request gives when rendered
 * alone in a batch of one.  Optional per-request stats as in
 * vr_render (the call then waits).  This is the one-GPU form of the paper's
 * scheduler, which maps rendering tasks onto the available GPUs (Fig. 1
 * caption; Sec. 3.1 process step 2).  Errors as for vr_render, per request
 * (the message names the request). */
vr_status vr_render_batch(vr_ctx ctx, const vr_request* reqs, int32_t count, void* hip_stream,
                          vr_stats* stats);

typedef struct {
    int32_t max_batch_requests; /* requests admitted per launch (1..4096) */
    int32_t max_batch_tiles;    /* workgroup tiles (16x16 pixels each) per launch (>= 1) */
    int32_t max_inflight;       /* launches in flight (1..4) */
    int32_t use_graphs;         /* 1: replay a captured graph per shape class */
} vr_server_cfg;

/* Start/stop the serving loop (a host thread owned by the context): the
 * scheduler server of the paper's framework (Fig. 1 caption), here batching
 * concurrent view requests into persistent launches on one GPU.  Start gives
 * VR_ESTATE if a server already runs, VR_EINVAL for a config out of range;
 * stop waits for queued work and is a no-op without a server. */
vr_status vr_server_start(vr_ctx ctx, const vr_server_cfg* cfg);
vr_status vr_server_stop(vr_ctx ctx);

/* Queue a request; returns a ticket.  Requests that arrive while others are
 * on the device join the next launch (continuous batching). */
vr_status vr_submit(vr_ctx ctx, const vr_request* req, uint64_t* ticket);

/* done = 1 once the ticket's image is complete in out_dev. */
vr_status vr_poll(vr_ctx ctx, uint64_t ticket, int32_t* done);

/* Wait for a ticket (timeout_s <= 0: forever).  latency_s (nullable) gets
 * completion time minus submission time as measured by the server. */
vr_status vr_wait(vr_ctx ctx, uint64_t ticket, double timeout_s, double* latency_s);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
