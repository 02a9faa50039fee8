/*
 * fvr.h - C ABI of the MI355X (gfx950) volumetric Fourier-transform surface
 * reconstruction library.
 *
 * Method: Alexiadis et al., "An Integrated Platform for Live 3D Human
 * Reconstruction and Motion Capturing", IEEE TCSVT 2017, Sec. III-B:
 *   1. weighted Gaussian splat of the oriented points into a vector field
 *      V(q) with density normalisation (eqs. (1)-(2));
 *   2. forward 3D FFT of V_X, V_Y, V_Z;
 *   3. integration filter j w / |w|^2 applied in the frequency domain;
 *   4. inverse 3D FFT and sum of the components -> indicator A(q);
 *   5. iso-level L = mean of A at the input sample locations;
 *   6. marching cubes on A(q) = L -> welded triangle mesh.
 *
 * Conventions (readings of points the paper leaves open):
 *   - Grid dims are (Nx, Ny, Nz).  Scalar fields are stored (Nz, Ny, Nx),
 *     x fastest: element (qx, qy, qz) at qx + Nx (qy + Ny qz).
 *   - The bbox (xmin, ymin, zmin, xmax, ymax, zmax) is the FFT's periodic
 *     domain; voxel q has centre bmin + (q + 1/2) h with h = (bmax - bmin)/N.
 *     The caller pads the bbox around the object (zero padding, Sec. III-B).
 *   - sigma1 = half the voxel diagonal, sigma2^2 = 3/2 sigma1^2, g(x; s) =
 *     exp(-x^2/s^2)/s, footprint = the 4 voxel centres per axis nearest the
 *     point (4^3 voxels, text after eq. (2)).
 *   - FFT: forward exp(-i...), unnormalised; inverse exp(+i...) / n;
 *     w_a = 2 pi kappa_a / extent_a; the derivative factor is zero on each
 *     axis's Nyquist plane; the filtered DC bin is zero.
 *   - L is the unweighted mean of the trilinearly sampled A over the
 *     accepted points, summed in double precision.
 *   - Marching cubes: inside <=> A > L (strict); one vertex per grid edge
 *     that crosses the level, numbered in (linear index of the edge's lower
 *     grid point, axis) order; triangles in (cell linear index, table) order;
 *     outward (inside -> outside) counter-clockwise winding; the table is
 *     generated from a face-consistent rule, so the mesh is closed and
 *     manifold whenever the surface does not reach the grid border.
 *
 * Memory: every array pointer is a DEVICE pointer on the context's device
 * unless stated otherwise, row-major, float32 unless stated otherwise.
 * Inputs are borrowed for the duration of the call; outputs are
 * caller-allocated.  The context owns its FFT plans, twiddle tables and
 * scratch memory; they stay resident and grow to the largest grid and point
 * count seen.  A context is used by one host thread at a time; work is
 * enqueued on the context's stream.
 *
 * Errors: every call returns an fvr_status; fvr_last_error() gives a
 * message.  On error no output array is written, except the counts that
 * FVR_E_CAPACITY reports.
 */
#ifndef FVR_H
#define FVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FVR_OK = 0,
    FVR_E_INVALID = -1,     /* bad argument or non-finite / negative input value */
    FVR_E_UNSUPPORTED = -2, /* a grid dim not of the form 2^a 3^b 5^c, or > 512 */
    FVR_E_NOMEM = -3,       /* device allocation failed */
    FVR_E_CAPACITY = -4,    /* output arrays too small; required counts written */
    FVR_E_DEVICE = -5,      /* a HIP runtime error */
    FVR_E_RANGE = -6,       /* a 16-bit spectrum value overflowed (FVR_STORAGE_FP16
                               with normals far from unit length): use float32 storage */
    /* not a status: widens the type to every int32 value, so that a value
       from a newer or older library (fvr_status_string says "unknown
       status") is a valid fvr_status in C++ too */
    FVR_STATUS_MAX_ENUM = 0x7fffffff
} fvr_status;

/* Largest point count of one frame: (2^31 - 1) / 3, so that every
 * coordinate index 3 i fits a 32-bit integer in the kernels. */
#define FVR_MAX_POINTS 715827882LL

/* fvr_mesh.flags bits */
#define FVR_FLAG_OPEN_SURFACE 1u /* a voxel on the grid's outer layer is inside:
                                    the bbox was not padded enough */

typedef struct fvr_ctx fvr_ctx;

/* One capture frame: the oriented, confidence-weighted point set of
 * Sec. III-A (points X, normals N, weights W) and the grid. */
typedef struct {
    const float *points;  /* M x 3, world units */
    const float *normals; /* M x 3 (used as given; not renormalised) */
    const float *weights; /* M, >= 0; NULL means every weight is 1 */
    int64_t n_points;     /* 0 <= M <= FVR_MAX_POINTS, else FVR_E_INVALID */
    int32_t dims[3];      /* Nx, Ny, Nz: each even, 8..512, 2^a 3^b 5^c */
    float bbox[6];        /* xmin, ymin, zmin, xmax, ymax, zmax (max > min) */
    uint32_t options;     /* FVR_SPLAT_*, FVR_STORAGE_* bits; 0: the weighted splat of
                             eqs. (1)-(2) with complex64 spectra */
} fvr_frame;

/* fvr_frame.options: the non-weighted splat of Sec. III-B ("simplest
 * version"): each point's normal goes to its nearest voxel (the grid cell
 * that contains it: floor((X - bmin)/h) in float32, clamped to the grid)
 * and V is the mean of the normals that land in a voxel (0 where none do);
 * weights are ignored (still validated). */
#define FVR_SPLAT_NEAREST 1u
/* fvr_frame.options: reduced-precision storage of the spectra between the
 * transform passes - two bfloat16 (FVR_STORAGE_BF16) or two IEEE half
 * (FVR_STORAGE_FP16) values per complex bin instead of complex64, half the
 * bytes - with every pass computing in float32.  Each forward pass stores
 * its output times 1/N_axis (the inverse's 1/n split over the passes), and
 * the angular frequencies of the derivative and the solve are taken in
 * units of 1/h_x (h_x the voxel size along x; A is scaled back at the end),
 * so the stored magnitudes do not depend on the bbox's length unit: for
 * unit normals they stay some 2^16 below FP16's largest value.  A value
 * that overflows anyway makes the call fail with FVR_E_RANGE.  V never
 * leaves the chip and A stays float32.  Every supported grid takes either
 * storage.  The indicator then
 * carries the rounding of 8-bit (bf16) or 11-bit (fp16) significands: its
 * error against an FP64 evaluation is reported with the benchmarks, and lies
 * outside the float32 tolerance. */
#define FVR_STORAGE_BF16 2u
#define FVR_STORAGE_FP16 4u

typedef struct {
    float *vertices;            /* out: capacity x 3 */
    int32_t *triangles;         /* out: capacity x 3 vertex indices */
    int64_t vertex_capacity;    /* in */
    int64_t triangle_capacity;  /* in */
    int64_t n_vertices;         /* out: written count, or the required count on FVR_E_CAPACITY */
    int64_t n_triangles;        /* out: same */
    double level;               /* out: iso-level L */
    int64_t n_rejected;         /* out: points outside the bbox (not an error) */
    uint32_t flags;             /* out: FVR_FLAG_* */
    float *normals;             /* out, optional (NULL: not computed): vertex_capacity x 3
                                   unit vertex normals -grad A (Sec. III-B lists normals
                                   among the mesh outputs): central differences of A at the
                                   edge's two grid points (one-sided on the grid's outer
                                   layer), interpolated with the vertex's t, normalised;
                                   written with the vertices */
} fvr_mesh;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
fvr_status fvr_create(int device, void *hip_stream, fvr_ctx **out);
void fvr_destroy(fvr_ctx *ctx);
/* Change the stream later calls enqueue on. */
fvr_status fvr_set_stream(fvr_ctx *ctx, void *hip_stream);

/* The whole path, Sec. III-B steps 1-6.  Enqueues on the context's stream
 * and waits for completion.  Points outside the bbox are rejected and
 * counted.  M = 0, or all points rejected, gives FVR_OK, level 0 and an
 * empty mesh.  If the mesh does not fit, returns FVR_E_CAPACITY with the
 * required n_vertices / n_triangles and writes nothing else. */
fvr_status fvr_reconstruct(fvr_ctx *ctx, const fvr_frame *frame, fvr_mesh *mesh);

/* Size of the static device scratch of fvr_reconstruct_noalloc: one array
 * per GPU the library runs on, held until the process ends.  It holds a
 * 128^3 frame of up to about a million points (with the triangle capacity
 * of its mesh); 96^3 and smaller grids hold several million. */
#define FVR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* fvr_reconstruct for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with every scratch buffer
 * carved from the device's static array of FVR_NOALLOC_SCRATCH_BYTES
 * instead of the context's own memory, and no hipMalloc, hipFree or other
 * allocation in the call (the context, made beforehand by fvr_create, owns
 * the stream and the pinned status block).  The caller passes the inputs
 * and the mesh outputs as for fvr_reconstruct.  A frame whose scratch does
 * not fit is refused with FVR_E_NOMEM before anything is enqueued.  Per-kernel
 * timing is not recorded in this call.  All calls on one GPU, from every
 * context, share that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (other threads, other streams) race and
 * must be serialised by the caller. */
fvr_status fvr_reconstruct_noalloc(fvr_ctx *ctx, const fvr_frame *frame, fvr_mesh *mesh);

/* Steps 1-5 only: the indicator A (Nz x Ny x Nx floats, device) and L.
 * Same kernels as fvr_reconstruct. */
fvr_status fvr_indicator(fvr_ctx *ctx, const fvr_frame *frame, float *field_out,
                         double *level_out);

/* Step 6 only: marching cubes of a caller field (Nz x Ny x Nx floats,
 * device) at `level`.  Any dims >= 2 are accepted (no transform-size
 * constraint) as long as 3 Nx Ny Nz < 2^31.  cases_out (optional, device, (Nz-1)(Ny-1)(Nx-1)
 * bytes, x fastest) receives each cell's case byte sum_k [A(corner k) > L]
 * 2^k with corner k at offset (k&1, (k>>1)&1, (k>>2)&1).  mesh->level is set
 * to `level`; mesh->n_rejected to 0.  Same kernels as fvr_reconstruct. */
fvr_status fvr_extract(fvr_ctx *ctx, const float *field, const int32_t dims[3],
                       const float bbox[6], float level, fvr_mesh *mesh,
                       uint8_t *cases_out);

/* Step 1 output for parity checks: V (3 x Nz x Ny x Nx floats, device,
 * component-major) written by the same splat kernel the path uses. */
fvr_status fvr_debug_splat(fvr_ctx *ctx, const fvr_frame *frame, float *v_out);

/* Batches: several frames as one unit of device work (Sec. III-B per
 * frame).  A batch owns `slots` contexts, each with its own scratch, status
 * block and stream (default priority); frame i runs on slot i mod slots, so
 * frames of different slots overlap on the device.  fvr_batch_reconstruct
 * captures the fork from the batch's stream to the slot streams, every
 * frame's stages and the join into one HIP graph, launches it and waits
 * once; a later call with the same frames (fields and pointers), outputs
 * and scratch replays the instantiated graph without capturing (up to 8
 * graphs are kept).  `hip_stream` is the stream the batch forks from (NULL:
 * a stream the batch makes; the null stream cannot be captured).  Each
 * frame's result is the one fvr_reconstruct gives for it, bit for bit.
 * Inputs and outputs are borrowed as for fvr_reconstruct.  All frames are
 * checked, and every slot's scratch grown, before anything is enqueued.
 * Returns the first frame error (FVR_E_CAPACITY: that mesh holds the
 * required counts); every mesh is filled.  A batch is used by one host
 * thread at a time. */
typedef struct fvr_batch fvr_batch;
fvr_status fvr_batch_create(int device, void *hip_stream, int slots, fvr_batch **out);
void fvr_batch_destroy(fvr_batch *batch);
fvr_status fvr_batch_set_stream(fvr_batch *batch, void *hip_stream);
/* enable = 0: enqueue the same work directly, without a graph */
fvr_status fvr_batch_use_graph(fvr_batch *batch, int enable);
fvr_status fvr_batch_reconstruct(fvr_batch *batch, const fvr_frame *frames, fvr_mesh *meshes, int n);
const char *fvr_batch_last_error(const fvr_batch *batch);

/* The front end of Sec. III-A: K depth maps (one per calibrated view) to the
 * raw oriented, confidence-weighted points that fvr_reconstruct takes.  Per
 * foreground pixel u (depth > 0 and finite): the point X = R X_loc + t with
 * X_loc = ((u_x - c_x) D / f_x, (u_y - c_y) D / f_y, D); the normal R N_loc,
 * N_loc the mean of the unit normals of the triangles of an organized
 * triangulation that contain u (each 2 x 2 pixel quad is split along the
 * diagonal whose ends differ less in depth; a triangle is kept when its three
 * pixels are foreground and no two of its depths differ by more than
 * step_threshold, the step-discontinuity constraint); the weight W = W1 W2
 * with W1 = max(<-X_loc/|X_loc|, N_loc>, 0) (viewing angle) and W2 the
 * fraction of foreground pixels in the (2 box_radius + 1)^2 square around u
 * (outside the image counts as background; silhouette confidence).  Pixels
 * in no kept triangle give no point.  Points are written view by view in
 * raster order. */
typedef struct {
    const float *depth;    /* device, views x height x width, metres along the optical axis */
    const float *cameras;  /* host, views x 16: fx, fy, cx, cy, R (3 x 3 row-major,
                              camera to world), t (camera centre in world) */
    int32_t views;         /* 1..16 */
    int32_t height, width; /* pixels per map (at most 2^24) */
    float step_threshold;  /* metres; the paper's captures: a few cm */
    int32_t box_radius;    /* pixels; 10 in the paper's experiments */
} fvr_depth_views;
/* Writes n_points points (device arrays of capacity points x 3, normals x 3,
 * weights), waiting for completion.  FVR_E_CAPACITY: *n_points holds the
 * required count and nothing is written. */
fvr_status fvr_depth_to_points(fvr_ctx *ctx, const fvr_depth_views *views, float *points, float *normals,
                               float *weights, int64_t capacity, int64_t *n_points);

/* Serving with continuous batching.  A server owns `slots` contexts (one
 * frame each at a time, each on its own stream) and a copy stream.  Requests
 * carry HOST arrays (the inputs, valid until the request's result has been
 * polled; the mesh outputs, filled before the result is returned) and wait
 * in arrival order.  A request is admitted when a slot is free and the
 * device memory the slots would then hold (scratch, inputs and mesh of each)
 * stays within hbm_budget bytes; one that cannot fit even with every other
 * slot idle is refused (result status FVR_E_NOMEM).  An admitted request's
 * upload runs on the copy stream and its stages on its slot's stream, so
 * uploads overlap compute and frames of different slots overlap; once its
 * counts are known its mesh comes back in exactly its size.  Each result is
 * the one fvr_reconstruct gives for the frame, bit for bit, whatever else
 * runs beside it.  fvr_server_poll harvests finished work, admits waiting
 * requests as slots and memory free up, and returns finished results in
 * completion order.  A server is used by one host thread at a time. */
#define FVR_REQUEST_PINNED 1u /* the request's input arrays are pinned host memory */
typedef struct {
    const float *points, *normals, *weights; /* host, M x 3, M x 3, M (weights may be NULL) */
    int64_t n_points;
    int32_t dims[3];
    float bbox[6];
    uint32_t options;                        /* FVR_SPLAT_*, FVR_STORAGE_* */
    uint32_t flags;                          /* FVR_REQUEST_* */
    float *vertices;                         /* host out: vertex_capacity x 3 */
    int32_t *triangles;                      /* host out: triangle_capacity x 3 */
    float *normals_out;                      /* host out, optional: vertex_capacity x 3 */
    int64_t vertex_capacity, triangle_capacity;
    void *user;                              /* returned in the result */
} fvr_request;
typedef struct {
    uint64_t ticket;
    fvr_status status;                       /* FVR_E_CAPACITY: n_vertices / n_triangles required */
    int64_t n_vertices, n_triangles, n_rejected;
    double level;
    uint32_t flags;                          /* FVR_FLAG_* */
    void *user;
    double submit_ms, admit_ms, done_ms;     /* host steady clock */
    char error[96];
} fvr_result;
typedef struct {
    int64_t pending, in_flight, results_waiting, admitted, completed, refused, max_in_flight;
    int64_t device_bytes, budget;
} fvr_server_stats;
typedef struct fvr_server fvr_server;
fvr_status fvr_server_create(int device, int slots, size_t hbm_budget, fvr_server **out);
void fvr_server_destroy(fvr_server *server);
/* Queue a request (checked on the host first); never waits for the device. */
fvr_status fvr_server_submit(fvr_server *server, const fvr_request *request, uint64_t *ticket);
/* Harvest, admit, and return up to max_results finished results. */
fvr_status fvr_server_poll(fvr_server *server, fvr_result *out, int max_results, int *n_results);
fvr_status fvr_server_info(const fvr_server *server, fvr_server_stats *out);
const char *fvr_server_last_error(const fvr_server *server);

/* Work counters of the context's last completed fvr_reconstruct,
 * fvr_reconstruct_noalloc or fvr_indicator call, from the status block that
 * call read back (no device work): how much of the grid the sparse passes
 * touched. */
typedef struct {
    int64_t busy_tiles, tiles;            /* splat tiles some footprint reaches / all */
    int64_t nonzero_planes, planes;       /* z planes the passes after the y transform read / all */
    int64_t mc_blocks_listed, mc_blocks;  /* marching-cubes blocks classified from the field / all
                                             (all are listed when the row ranges are not used) */
    int64_t points_used, points_rejected; /* accepted points in the level, points outside the bbox */
} fvr_stats;
fvr_status fvr_last_stats(const fvr_ctx *ctx, fvr_stats *out);

/* Plan parameters of one grid shape, as chosen by an autotuner: the radix
 * order of each axis's mixed-radix (Stockham) passes - radices from
 * {2, 3, 4, 5, 8} whose product is the axis length, at most 8 stages;
 * nstages 0 keeps the default order (8s first, then a 4 or 2, 3s, 5s) - and
 * the splat tile of ty x tz full x-rows (0 x 0 keeps the default; ty tz even,
 * ty tz Nx <= 2048, (ty + 3)(tz + 3) <= 128).  Lengths 16..256 that are
 * powers of two run register pencils whose schedule is fixed.  The radix
 * order changes the rounding of the transforms, not what they compute. */
typedef struct {
    int32_t nstages[3];
    int32_t radices[3][8];
    int32_t splat_ty, splat_tz;
} fvr_tuning;
/* Set (t != NULL) or clear (t == NULL) the tuning of grid shape `dims` for
 * the whole process: every context and batch builds its plans from it from
 * the next call on.  FVR_E_INVALID if a parameter does not fit. */
fvr_status fvr_set_tuning(const int32_t dims[3], const fvr_tuning *t);
/* The parameters plans of shape `dims` use now (tuned or default). */
fvr_status fvr_get_tuning(const int32_t dims[3], fvr_tuning *t);

/* Host-only helpers (no device work; callable without a GPU). */
/* Check dims and bbox as fvr_reconstruct would. */
fvr_status fvr_check_grid(const int32_t dims[3], const float bbox[6]);
/* Check a frame's host-side fields as fvr_reconstruct does before any
 * launch: point count (0..FVR_MAX_POINTS), the required pointers, grid and
 * bbox.  The device arrays are not read (their values are checked on the
 * device during a reconstruction). */
fvr_status fvr_check_frame(const fvr_frame *frame);
/* Copy the library's generated marching-cubes table: counts[256] triangles
 * per case and edges[256 * 15] cube-edge ids (-1 padded), cube edge
 * id = 4 axis + b_lo + 2 b_hi. */
fvr_status fvr_mc_table(uint8_t counts[256], int8_t edges[256 * 15]);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * the launches of the selected kernels (off by default).  Index i in
 * [0, fvr_timing_count()).  fvr_timing_enable selects all kernels (enable != 0)
 * or none; fvr_timing_select selects kernel i when bit i of mask is set, so a
 * caller can time one kernel without paying for events around the others. */
fvr_status fvr_timing_enable(fvr_ctx *ctx, int enable);
fvr_status fvr_timing_select(fvr_ctx *ctx, uint32_t mask);
fvr_status fvr_timing_reset(fvr_ctx *ctx);
int fvr_timing_count(void);
const char *fvr_timing_name(int i);
fvr_status fvr_timing_get(const fvr_ctx *ctx, int i, double *total_ms, int64_t *launches);

const char *fvr_status_string(fvr_status s);
const char *fvr_last_error(const fvr_ctx *ctx); /* ctx may be NULL */

#ifdef __cplusplus
}
#endif
#endif /* FVR_H */
