/*
 * radfoam.h - C ABI of the MI355X (gfx950) Voronoi ray-walk library (librf.so).
 *
 * The library renders and differentiates the Radiant Foam scene model
 * (Govindarajan, Rebain, Yi, Tagliasacchi, "Radiant Foam: Real-Time
 * Differentiable Ray Tracing", CVPR 2025):
 *   - the scene is a set of Voronoi sites x_i (Sec. 3.2, eq. (5)) with a
 *     per-cell density sigma_i and view-dependent colour given by real
 *     spherical harmonics of degree <= 3 (Sec. 3.4);
 *   - the Delaunay neighbours N(i) of every site are an input (a CSR list
 *     built on the host); the library never triangulates;
 *   - a ray starts in a given cell (Algorithm 1 starts in nn(o); the caller
 *     supplies that cell), repeatedly leaves the current cell through the
 *     nearest front-facing bisector plane (Algorithm 1, Fig. 2), and
 *     alpha-composites each segment with eq. (3)-(4) while the
 *     transmittance exceeds eps;
 *   - the backward pass returns gradients for densities, SH coefficients and
 *     site positions, geometry entering only through segment widths
 *     (Sec. 3.1, "Piecewise constant volumes").
 *
 * Conventions for every call:
 *   - All array pointers are DEVICE pointers (hipMalloc or torch CUDA
 *     memory) owned by the caller unless stated otherwise; the library keeps
 *     no reference to them after the call returns. Struct arguments
 *     themselves live in host memory.
 *   - Float arrays are IEEE binary32, row-major, densely packed.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream) unless stated otherwise.
 *   - Every call returns an rf_status and never aborts or throws. On an
 *     error nothing is launched and rf_last_error() describes it.
 *   - Per-ray anomalies are not call errors: they are reported in the
 *     per-ray `steps` output (RF_RAY_*).
 *   - Calls on different streams may run concurrently; the library holds no
 *     global mutable state besides the thread-local error string.
 */
#ifndef RADFOAM_H
#define RADFOAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RF_OK = 0,
    RF_ERR_INVALID_ARG = 1,  /* bad pointer, size, layout or CSR contents */
    RF_ERR_HIP = 2,          /* a HIP runtime call failed; see rf_last_error() */
    RF_ERR_OOM = 3,          /* device or host allocation failed */
    RF_ERR_UNSUPPORTED = 4,  /* valid but outside this build's limits */
    RF_ERR_BUSY = 5          /* serving: request not admissible right now */
} rf_status;

typedef enum { RF_F32 = 0, RF_BF16 = 1 } rf_dtype;

/* Per-ray values of `steps` (>= 0 is the number of visited cells). */
#define RF_RAY_BAD_START (-1) /* start cell outside [0, n_sites): rgb = 0, T = 1 */
#define RF_RAY_MAX_STEPS (-2) /* max_steps cells visited with T > eps before t_max */

/* Limits of this build. */
#define RF_MAX_SITES ((int64_t)1 << 24) /* cell ids fit 24 bits */
#define RF_MAX_DEGREE 255               /* Delaunay neighbours per site */
#define RF_MAX_SH_DEGREE 3

/* Thread-local description of the last error on this host thread ("" if none). */
const char *rf_last_error(void);

/* Library version string. */
const char *rf_version(void);

/* ------------------------------------------------------------------------
 * Scene (Sec. 3.2 "The Voronoi diagram", Sec. 3.4 "Training").
 *
 *   sites    float[n_sites][3]        Voronoi sites x_i.
 *   nbr_off  int32[n_sites + 1]       CSR row offsets: the neighbours of i are
 *   nbr_idx  int32[n_edges]           nbr_idx[nbr_off[i] .. nbr_off[i+1]-1].
 *                                     Rows must list the Delaunay neighbours
 *                                     of i (a superset is harmless, a missing
 *                                     neighbour is not); nbr_off[0] = 0,
 *                                     nbr_off[n_sites] = n_edges; no self loop.
 *                                     Ties between equal exit distances go to
 *                                     the first neighbour in row order.
 *   density  float[n_sites]           sigma_i >= 0 (already activated; the
 *                                     paper's softplus stays outside).
 *   sh       float[n_sites][B][3]     SH coefficients, B = (sh_degree+1)^2,
 *                                     basis l-major, m = -l..l, RGB innermost.
 *                                     Colour = sum_b sh[i][b][:] * Y_b(d), the
 *                                     real orthonormal SH basis, no offset and
 *                                     no clamp.
 * ---------------------------------------------------------------------- */
typedef struct {
    const float *sites;
    const int32_t *nbr_off;
    const int32_t *nbr_idx;
    const float *density;
    const float *sh;
    int64_t n_sites;
    int64_t n_edges;
    int32_t sh_degree; /* 0..3 */
    int32_t density_activation; /* RF_DENSITY_PLAIN: density is sigma (>= 0);
                                   RF_DENSITY_SOFTPLUS: density holds the raw
                                   parameter x, sigma = ln(1 + e^{10 x}) / 10
                                   (the paper's softplus with beta = 10, Sec. 3.4),
                                   applied by rf_pack_scene */
} rf_scene;

#define RF_DENSITY_PLAIN 0
#define RF_DENSITY_SOFTPLUS 1

/* ------------------------------------------------------------------------
 * Packed scene: device-resident records that the walk reads.
 *
 * rf_packed_bytes() gives the size of the device workspace for a scene;
 * rf_pack_scene() fills it from an rf_scene and fills the host descriptor
 * `out`. The workspace holds, per directed Delaunay edge (i -> j), the
 * bisector plane (n = x_j - x_i, c = n.(x_i + x_j)/2) and the neighbour's
 * row, and per cell one record with its SH coefficients and density (in
 * `attr_dtype`, bf16 by round-to-nearest-even) and its site. The layout is
 * private to the library. The caller owns the workspace, must keep it alive
 * and unmodified while any call that uses `out` runs, and must pack again
 * after changing the scene. Repacking into the same workspace is allowed.
 *
 * CSR contents are validated on the device: invalid entries are neutralised
 * (they can never be crossed) and counted. With validate != 0 the call
 * synchronises `stream` and returns RF_ERR_INVALID_ARG if any entry was
 * invalid (RF_ERR_UNSUPPORTED if a row exceeds RF_MAX_DEGREE); with
 * validate == 0 it stays asynchronous and rf_packed_errors() can be polled.
 * ---------------------------------------------------------------------- */
typedef struct {
    void *base;          /* device workspace (owned by the caller) */
    size_t bytes;
    int64_t n_sites;
    int64_t n_edges;
    int32_t sh_degree;
    rf_dtype attr_dtype;
    /* private section offsets (bytes from base) */
    size_t off_planes, off_adj, off_rec, off_row, off_err;
    int32_t rec_bytes;
    int32_t reserved;
} rf_packed_scene;

rf_status rf_packed_bytes(int64_t n_sites, int64_t n_edges, int32_t sh_degree, rf_dtype attr_dtype,
                          size_t *bytes);

rf_status rf_pack_scene(const rf_scene *scene, rf_dtype attr_dtype, void *workspace, size_t workspace_bytes,
                        int validate, rf_packed_scene *out, void *stream);

/* Synchronously reads the validation counters written by the last pack:
 * errors[0] = invalid CSR entries, errors[1] = rows longer than RF_MAX_DEGREE. */
rf_status rf_packed_errors(const rf_packed_scene *packed, int32_t errors[2], void *stream);

/* ------------------------------------------------------------------------
 * Rays (Algorithm 1 "Render(o, d)").
 *
 *   origin     float[n_rays][3]   o
 *   dir        float[n_rays][3]   d, unit length (not renormalised)
 *   t_max      float[n_rays]      finite end of the ray, >= 0 (the segment
 *                                 reaching it is clipped, eq. (1)'s t_max)
 *   start_cell int32[n_rays]      the cell containing o (nn(o))
 * ---------------------------------------------------------------------- */
typedef struct {
    const float *origin;
    const float *dir;
    const float *t_max;
    const int32_t *start_cell;
    int64_t n_rays;
} rf_rays;

typedef struct {
    float eps;         /* transmittance threshold of Algorithm 1 (default 1e-4); T > eps is tested
                          before each cell */
    int32_t max_steps; /* cap on visited cells per ray (default 8192) */
} rf_params;

/* ------------------------------------------------------------------------
 * Camera rays, in 8x8 screen-tile order: tiles row-major over the image,
 * pixels row-major inside a tile, partial edge tiles holding only the pixels
 * inside the image. Ray r covers pixel pixel[r] = y*width + x. With
 * (u, v) = (x + 0.5 - width/2, y + 0.5 - height/2) and R the rotation in pose
 * (columns right, down, forward), its direction is
 *   RF_CAMERA_PINHOLE: R (u, v, f) normalised, f = (width/2)/tan(fov/2);
 *   RF_CAMERA_FISHEYE (equidistant; the non-linear camera of the ray-based
 *     effects, Fig. 3): R (sin(a) u/rho, sin(a) v/rho, cos(a)) with
 *     rho = |(u, v)| and a = rho (fov/2)/(width/2), so the angle from the
 *     axis grows linearly with rho and the left and right edges are at fov/2.
 * t_max is the distance at which the ray leaves the bound (the origin must
 * be inside it). start_cell is filled with `start` (the caller's nn(origin)
 * for the camera position).
 * ---------------------------------------------------------------------- */
#define RF_CAMERA_PINHOLE 0
#define RF_CAMERA_FISHEYE 1

typedef struct {
    float pose[12];   /* row-major 3x4 [R | position] */
    float fov_deg;    /* horizontal field of view: pinhole (0, 180), fisheye (0, 360] */
    int32_t width, height;
    int32_t model;    /* RF_CAMERA_* (0, the pinhole, when zero-initialised) */
} rf_camera;

typedef struct {
    int32_t kind;     /* 0: box [p0,p1,p2] .. [p3,p4,p5]; 1: sphere about the origin, radius p0 */
    float p[6];
} rf_bound;

rf_status rf_raygen(const rf_camera *camera, const rf_bound *bound, int32_t start, float *origin, float *dir,
                    float *t_max, int32_t *start_cell, int32_t *pixel /* nullable */, void *stream);

/* ------------------------------------------------------------------------
 * Forward walk (Algorithm 1 with eq. (3)-(4)).
 *   rgb      float[n_rays][3]  composited colour C (no background)
 *   t_final  float[n_rays]     final transmittance T
 *   steps    int32[n_rays]     visited cells, or RF_RAY_* (< 0)
 * Deterministic: the same inputs give bitwise the same outputs.
 * ---------------------------------------------------------------------- */
rf_status rf_render_forward(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                            float *rgb, float *t_final, int32_t *steps, void *stream);

/* ------------------------------------------------------------------------
 * Backward walk: gradients of L = sum_r grad_rgb[r].rgb[r] + grad_t_final[r] T[r]
 * (Sec. 3.1: geometry receives gradients only through the segment widths).
 * The walk is recomputed from the inputs (rf_render_backward_logged reads
 * it from a walk log instead); rgb, t_final and steps must be the outputs of
 * rf_render_forward for the same scene, rays and params.
 *   steps         int32[n_rays]        nullable: the forward's steps
 *   mismatches    int32[1]             nullable, device: incremented (atomically)
 *                                      once for every ray whose recomputed walk
 *                                      ends with a final transmittance that
 *                                      differs from t_final (bitwise) or, when
 *                                      steps is given, a visit count or status
 *                                      that differs from steps; 0 after a
 *                                      consistent call (the caller zeroes it)
 *   grad_rgb      float[n_rays][3]
 *   grad_t_final  float[n_rays]        nullable (treated as 0)
 *   grad_sites    float[n_sites][3]    ACCUMULATED (+=); caller zeroes
 *   grad_density  float[n_sites]       ACCUMULATED (+=)
 *   grad_sh       float[n_sites][B][3] ACCUMULATED (+=)
 * Per-site sums use float atomics: results are deterministic only up to
 * the order of additions.
 * `mode` selects the gradient reduction: 0 = reduce across the wavefront
 * per cell before the atomics (default), 1 = one atomic per lane and value.
 * ---------------------------------------------------------------------- */
rf_status rf_render_backward(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                             const float *rgb, const float *t_final, const int32_t *steps, const float *grad_rgb,
                             const float *grad_t_final, float *grad_sites, float *grad_density, float *grad_sh,
                             int32_t mode, int32_t *mismatches, void *stream);

/* ------------------------------------------------------------------------
 * Start-cell location: the cell containing each point, i.e. its nearest
 * site (eq. (5)); Algorithm 1 starts the walk of a ray in the cell of its
 * origin. A greedy walk over the Delaunay graph from seed[q] (cell 0 when
 * seed is NULL) moves to the neighbour nearest the point while one is
 * nearer, first in FP32 across the bisector planes, then with squared
 * distances in double (ties go to the lower index). On a Delaunay graph a
 * site that is not the nearest always has a nearer neighbour, so the walk
 * ends at the nearest site; it takes O(distance / cell size) steps.
 *   points  float[n_points][3]  device
 *   seed    int32[n_points]     device, nullable
 *   cells   int32[n_points]     out: nearest site; -1 seed out of range;
 *                               -2 max_steps steps were not enough
 * ---------------------------------------------------------------------- */
rf_status rf_locate(const rf_packed_scene *scene, const float *points, int64_t n_points, const int32_t *seed,
                    int32_t max_steps, int32_t *cells, void *stream);

/* ------------------------------------------------------------------------
 * Walk log: what the backward needs of each visit, saved by the forward so
 * that the backward (Sec. 3.1 gradients, in the forward order of Algorithm 1)
 * does not repeat the face scans. Step-major: visit n (0-based) of ray r is
 * entry n * n_rays + r, for n < capacity.
 *   code    uint32[capacity][n_rays]  visited cell (bits 0..28) |
 *                                     exit-moves << 31 | walk-ended-here << 30
 *                                     | surface-crossing << 29 (the exit moves
 *                                     with its face when t0 <= t1 < t_max and
 *                                     no surface crossing ends the segment)
 *   t_exit  double[capacity][n_rays]  the visit's clamped exit distance te
 *                                     (along the visit's leg)
 *   tail    int32[n_rays][4]          the packed row reference (2 words) of
 *                                     the cell after the logged visits, the
 *                                     number of visited cells, the number of
 *                                     surface crossings (0 without a surface)
 * A ray with more than `capacity` visits logs the first `capacity`; the
 * backward walks that ray again from its start cell. Memory:
 * n_rays * (12 * capacity + 16) bytes, device, owned by the caller; t_exit
 * 8-byte, code 4-byte and tail 16-byte aligned. A log is valid only with the
 * scene, rays and params of the forward that wrote it, until the scene is
 * packed again.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t *code;
    double *t_exit;
    int32_t *tail;
    int32_t capacity;  /* >= 0; 0 logs nothing (the backward recomputes every visit) */
} rf_walk_log;

/* rf_render_forward that also writes `log`. Same outputs, bit for bit. */
rf_status rf_render_forward_logged(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                                   float *rgb, float *t_final, int32_t *steps, const rf_walk_log *log,
                                   void *stream);

/* rf_render_backward reading the visits from `log` (written by
 * rf_render_forward_logged for the same scene, rays and params) instead of
 * recomputing them. Same gradients as rf_render_backward up to the order of
 * the float atomic additions. */
rf_status rf_render_backward_logged(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                                    const float *rgb, const float *t_final, const float *grad_rgb,
                                    const float *grad_t_final, const rf_walk_log *log, float *grad_sites,
                                    float *grad_density, float *grad_sh, int32_t mode, void *stream);

/* ------------------------------------------------------------------------
 * Quantile regulariser (Sec. 3.4, training objectives): per ray, the loss
 * |W^-1(u1) - W^-1(u2)|, where W^-1 is the quantile function of the
 * normalised distribution of the volume-rendering weights along the ray
 * (W(t) = 1 - exp(-tau(t)) divided by the ray's opacity 1 - T_final; inside
 * a cell the density is constant, so W is exponential there) and u1, u2 are
 * the ray's two uniform draws. A ray with zero opacity has loss 0.
 *   draws    float[n_rays][2]  u1, u2 in [0, 1] (the caller's random numbers)
 *   t        float[n_rays][2]  out: W^-1(u1), W^-1(u2) (0 with zero opacity)
 *   segment  int32[n_rays][2]  out: the visit index holding each quantile (-1: none)
 *   sigma    float[n_rays][2]  out: that visit's density
 * The t, segment and sigma arrays are what the backward needs.
 * ---------------------------------------------------------------------- */
typedef struct {
    const float *draws;
    float *t;
    int32_t *segment;
    float *sigma;
} rf_quantiles;

/* Quantiles and per-ray loss (float[n_rays]) of the walks in `log` (written
 * by rf_render_forward_logged with the same scene, rays and params, whose
 * t_final is passed; walks longer than the log are walked again). */
rf_status rf_quantile_forward(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                              const float *t_final, const rf_walk_log *log, const rf_quantiles *q, float *loss,
                              void *stream);

/* rf_render_backward_logged for L = sum grad_rgb.rgb + sum grad_t_final T
 * + sum grad_loss loss: the quantile term's gradients flow to the densities
 * and, through the exit distances, to the sites. `q` holds the outputs of
 * rf_quantile_forward for the same log; grad_loss is float[n_rays]. */
rf_status rf_render_backward_quantile(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                                      const float *rgb, const float *t_final, const float *grad_rgb,
                                      const float *grad_t_final, const rf_walk_log *log, const rf_quantiles *q,
                                      const float *grad_loss, float *grad_sites, float *grad_density,
                                      float *grad_sh, int32_t mode, void *stream);

/* ------------------------------------------------------------------------
 * Secondary rays (the reflections and refractions of the ray-based effects,
 * Fig. 3): one analytic sphere in the scene, a mirror or a glass interface
 * (refractive index `ior` inside, 1 outside). The foam fills space on both
 * sides. Where a ray's current leg crosses the sphere inside cell i, the
 * segment ends at the crossing (an exit that does not move with the sites),
 * and the walk continues in cell i along the reflected direction
 * d - 2 (d.N) N, or the refracted one by Snell's law (total internal
 * reflection reflects); the new leg measures t from the crossing and ends
 * where it leaves `bound` (the first leg keeps the ray's own t_max). The
 * crossing splits the cell's visit, and the T > eps test is not repeated for
 * its second part. Crossings after the first max_bounces are ignored, so
 * max_bounces = 0 renders as rf_render_forward, bit for bit. Leg geometry
 * (crossing, normal, new direction, new t_max) is computed in double; the
 * new leg's origin and direction are then rounded to float.
 *
 * rf_render_forward_surface: the forward outputs; with a `log` (nullable)
 * it also writes the walk log, whose code words flag each crossing (bit 29;
 * the cell id takes bits 0..28) and whose tail's fourth value counts the
 * crossings. rf_render_backward_surface: the gradients of
 * sum grad_rgb.rgb + sum grad_t_final T (accumulated, caller-zeroed, as
 * rf_render_backward; the sphere itself is fixed), reading `log` if given
 * (written by rf_render_forward_surface with the same arguments) and
 * recomputing the walks otherwise or where they outgrew it; the wavefront
 * reduction is always used. The quantile regulariser gives rays with
 * crossings no loss and no gradient (its quantiles are defined along one
 * leg). Errors: RF_ERR_INVALID_ARG for a NULL or invalid surface (kind not
 * mirror or glass, radius <= 0, glass ior <= 0, max_bounces outside
 * [0, RF_MAX_BOUNCES], bound kind not 0 or 1) and as rf_render_forward /
 * rf_render_backward otherwise.
 * ---------------------------------------------------------------------- */
#define RF_SURFACE_MIRROR 1
#define RF_SURFACE_GLASS 2
#define RF_MAX_BOUNCES 1024

typedef struct {
    int32_t kind;         /* RF_SURFACE_* */
    int32_t max_bounces;  /* crossings handled per ray */
    float centre[3];
    float radius;         /* > 0 */
    float ior;            /* glass: refractive index inside the sphere, > 0 */
    rf_bound bound;       /* where the legs after a crossing end */
} rf_surface;

rf_status rf_render_forward_surface(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                                    const rf_surface *surface, float *rgb, float *t_final, int32_t *steps,
                                    const rf_walk_log *log /* nullable */, void *stream);
rf_status rf_render_backward_surface(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                                     const rf_surface *surface, const float *rgb, const float *t_final,
                                     const float *grad_rgb, const float *grad_t_final /* nullable */,
                                     const rf_walk_log *log /* nullable */, float *grad_sites,
                                     float *grad_density, float *grad_sh, void *stream);

/* ------------------------------------------------------------------------
 * Traced forward walk, for tests: the forward outputs plus, per ray, the
 * visited cells and each segment's clamped exit distance.
 *   cells   int32[n_rays][max_len]  (entries past the visit count untouched)
 *   t_exit  float[n_rays][max_len]
 * ---------------------------------------------------------------------- */
rf_status rf_render_trace(const rf_packed_scene *scene, const rf_rays *rays, const rf_params *params,
                          int32_t max_len, float *rgb, float *t_final, int32_t *steps, int32_t *cells,
                          float *t_exit, void *stream);

/* ------------------------------------------------------------------------
 * Training-step pieces around the walk (Sec. 3.3 and the implementation
 * details of Sec. 3.4). Parameters are grouped as positions, density, SH of
 * order 0 and SH of the higher orders.
 *
 * rf_train_schedule fills the Adam settings of 0-based `iteration` of a
 * `total`-iteration run with the paper's schedule: cosine annealing of each
 * group's learning rate, lr_end + (lr_0 - lr_end)(1 + cos(pi it / total))/2,
 * from 2e-4 to 2e-6 (positions), 1e-1 to 1e-2 (density), 5e-3 to 5e-4 (SH);
 * the higher SH orders held (lr 0) for the first total/4 iterations and the
 * positions from iteration total - total/10 on (the paper's last 2k of 20k);
 * t = each group's step count including this step (held steps do not
 * count); betas 0.9 and 0.999; eps 1e-15; softplus density.
 *
 * rf_adam_step applies one Adam step in place: for each value of a group with
 * lr > 0, m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); a held group
 * (lr = 0) keeps its values and moments. With softplus_density, `density`
 * holds the raw parameter x and grad_density is taken w.r.t. sigma (what the
 * backward returns), chained by d sigma / dx = 1 / (1 + e^{-10 x}). Arrays:
 * sites [n][3], density [n], sh [n][B][3], their gradients, and the moments
 * of each (caller-zeroed before the first step, caller-owned device memory;
 * 16-byte aligned arrays are streamed four values per thread). FP32.
 *
 * rf_densify_scores: per cell, |dL/dx_i| times its approximate radius, half
 * the mean distance to its Delaunay neighbours (0 for a cell without any).
 *
 * rf_sample_cells: n_draws densification candidates from the multinomial
 * distribution proportional to `scores` (>= 0, not all 0): draw k (u in
 * [0, 1)) picks the first cell whose cumulative score exceeds u times the
 * total, so a cell owns [C_{i-1}, C_i) and a zero score is never picked.
 * The cumulative sum is formed in double in the caller's workspace of
 * rf_sample_workspace(n) bytes (8-byte aligned).
 *
 * rf_prune_mask: mask[i] = 1 where density[i] (sigma) and the density of
 * every Delaunay neighbour are below `threshold` (cells that neither carry
 * nor bound a surface), else 0.
 *
 * The score and the mask skip neighbour ids outside [0, n_sites) (the CSR
 * is not validated here; rf_pack_scene does that for the walk). Offsets must
 * be monotone and within the idx array.
 *
 * All run on `stream`; errors: RF_ERR_INVALID_ARG for NULL arrays, negative
 * sizes, a schedule iteration outside [0, total), betas outside [0, 1),
 * eps < 0, lr < 0, or a moving group with t < 1.
 * ---------------------------------------------------------------------- */
typedef struct {
    float lr[4];      /* positions, density, SH order 0, SH orders >= 1; 0 holds the group */
    int32_t t[4];     /* each group's Adam step count including this step */
    float beta1, beta2, eps;
    int32_t softplus_density;
} rf_adam_args;

typedef struct {
    float *m_sites, *v_sites;      /* [n][3] */
    float *m_density, *v_density;  /* [n] */
    float *m_sh, *v_sh;            /* [n][B][3] */
} rf_adam_state;

rf_status rf_train_schedule(int32_t iteration, int32_t total, rf_adam_args *out);
rf_status rf_adam_step(int64_t n_sites, int32_t sh_degree, const rf_adam_args *args, float *sites, float *density,
                       float *sh, const float *grad_sites, const float *grad_density, const float *grad_sh,
                       const rf_adam_state *state, void *stream);
rf_status rf_densify_scores(const float *sites, const int32_t *nbr_off, const int32_t *nbr_idx, int64_t n_sites,
                            const float *grad_sites, float *scores, void *stream);
rf_status rf_sample_workspace(int64_t n, size_t *bytes);
rf_status rf_sample_cells(const float *scores, int64_t n, const float *draws, int64_t n_draws, int32_t *cells,
                          void *workspace, size_t workspace_bytes, void *stream);
rf_status rf_prune_mask(const float *density, const int32_t *nbr_off, const int32_t *nbr_idx, int64_t n_sites,
                        float threshold, uint8_t *mask, void *stream);

/* Densification applied (Sec. 3.3): a new site inside the cell of each
 * drawn candidate. new_sites[k] = x_p + frac r_p u_k with p = parents[k],
 * r_p half the distance from x_p to its nearest Delaunay neighbour (the
 * largest ball about x_p inside its Voronoi cell) and u_k = offsets[k] a
 * point of the unit ball (the caller's draws), so the new site lies strictly
 * inside the parent's cell for 0 <= frac < 1. Formed in double, rounded to
 * FP32. A parent outside [0, n_sites) gives NaN coordinates.
 *   sites     float[n_sites][3], nbr_off/nbr_idx the scene's CSR (device)
 *   parents   int32[n_new], offsets float[n_new][3], new_sites float[n_new][3] out
 * The caller appends the new sites (and their parents' attributes, see
 * rf_gather_rows) and rebuilds the Delaunay graph. */
rf_status rf_insert_sites(const float *sites, const int32_t *nbr_off, const int32_t *nbr_idx, int64_t n_sites,
                          const int32_t *parents, const float *offsets, int64_t n_new, float frac, float *new_sites,
                          void *stream);

/* out[k][:] = in[rows[k]][:] for rows of `width` floats (device arrays): the
 * parents' attributes for new sites, or the kept rows after pruning. A row
 * index outside [0, n_rows_in) gives a row of NaN. */
rf_status rf_gather_rows(const float *in, int64_t n_rows_in, int32_t width, const int32_t *rows, int64_t n_rows_out,
                         float *out, void *stream);

/* Pruning applied (Sec. 3.3): the indices i with keep[i] != 0, in increasing
 * order, into kept[0 .. *n_kept) (kept holds n entries; n_kept is a device
 * int64 written by the call). workspace: rf_keep_workspace(n) bytes, device,
 * 8-byte aligned. */
rf_status rf_keep_workspace(int64_t n, size_t *bytes);
rf_status rf_keep_index(const uint8_t *keep, int64_t n, int32_t *kept, int64_t *n_kept, void *workspace,
                        size_t workspace_bytes, void *stream);

/* rf_sample_cells for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same kernels and the same cells bit for bit, with the
 * scan's workspace in a fixed scratch array inside the library instead of
 * the caller's buffer. The call allocates nothing. Limit: n <= 4,194,304
 * cells (RF_ERR_UNSUPPORTED beyond; the scratch is 33.6 MB, held by every
 * GPU the library runs on until the process ends). Calls on one GPU share
 * that GPU's scratch: calls that overlap on one GPU (different streams, or
 * host threads) race and must be serialised by the caller. The scratch
 * keeps the last call's contents; nothing in it needs clearing. scores,
 * draws and cells as in rf_sample_cells (device pointers). */
rf_status rf_sample_cells_noalloc(const float *scores, int64_t n, const float *draws, int64_t n_draws,
                                  int32_t *cells, void *stream);

/* Copies the packed face planes (float4 per directed edge, CSR order) into
 * planes[n_edges][4]; for tests of the packing step. */
rf_status rf_packed_planes(const rf_packed_scene *scene, float *planes, void *stream);

/* Copies the packed density and SH back as float (bf16 widened exactly):
 * density[n_sites], sh[n_sites][B][3]; for tests of the packing step. */
rf_status rf_packed_attributes(const rf_packed_scene *scene, float *density, float *sh, void *stream);

/* ------------------------------------------------------------------------
 * Continuous-batching render server (forward only; the paper's renderer,
 * Sec. 3.4, measured frame rates with a low-overhead renderer).
 *
 * The packed scene stays resident (the caller keeps it alive and unmodified
 * until rf_server_destroy returns). Admitted requests are cut into 8x8
 * screen tiles. A scheduler thread owned by the server builds each kernel
 * launch from the pending tiles of all admitted requests (oldest request
 * first, up to 8192 tiles per launch) and keeps two launches queued on the
 * server's own stream, so requests that arrive while others are on the GPU
 * join the next launch and their work overlaps. Results land in a pinned
 * host output pool owned by the server: per pixel, image row-major, RGBA
 * floats = (r, g, b, final transmittance). Every pixel is computed by the same
 * ray generation and walk as rf_raygen + rf_render_forward, so a request's
 * image does not depend on what else is in flight.
 *
 * rf_server_submit admits a request immediately or returns RF_ERR_BUSY: it
 * needs a free slot (at most max_inflight <= 64 requests in flight) and W*H*16
 * contiguous bytes of the pool (pool_bytes). Callers that need FIFO order keep
 * their own queue and retry its head. start_cell is the cell containing the
 * camera position; with start_cell < 0 the server locates it on the device
 * (as rf_locate, seeded from a 16^3 grid of cells located over the bound when
 * the server is created) before the request's first tiles run.
 * rf_server_poll lists finished requests not yet collected; rf_server_result
 * copies one into `rgba` (host memory, >= W*H*16 bytes; NULL discards it) and
 * frees its slot and pool range; the copy runs outside the server's lock, so
 * the server keeps scheduling while a result is copied (a second call for the
 * same request meanwhile fails with RF_ERR_BUSY). rf_server_destroy finishes
 * admitted requests, stops the scheduler and frees the server. Every call but
 * rf_server_destroy may come from any host thread at any time (they serialise
 * on the server's lock); rf_server_destroy must not overlap another call.
 * ---------------------------------------------------------------------- */
typedef struct rf_server rf_server;

typedef struct {
    int64_t submitted, completed, rejected_busy, rays_done;
    int64_t pool_used_bytes, pool_bytes;
    int64_t launches, inflight;
} rf_server_stats;

rf_status rf_server_create(const rf_packed_scene *scene, const rf_params *params, const rf_bound *bound,
                           size_t pool_bytes, int32_t max_inflight, rf_server **out);
/* rf_server_create with a choice of form (mode):
 *   RF_SERVE_LAUNCHES    a host scheduler thread batches the pending tiles of
 *                        all admitted requests into ordinary kernel launches
 *                        (rf_server_create);
 *   RF_SERVE_PERSISTENT  one persistent kernel (the paper's low-overhead
 *                        renderer, Sec. 3.4) serves requests as they arrive:
 *                        a dispatcher wavefront reads request records from a
 *                        ring in coherent host memory and opens their slots,
 *                        worker wavefronts claim tiles of the oldest open
 *                        request and signal each completed request through
 *                        host memory. Every wait in the kernel is bounded: it
 *                        leaves 2 ms after its last request once everything
 *                        admitted is done, or after 1 s without a request,
 *                        and the scheduler relaunches it when requests wait.
 * Results are bitwise the same in both forms (the same ray generation and
 * walk). rf_server_destroy waits for admitted requests (at most 60 s) and,
 * in the persistent form, for the kernel to leave (at most 30 s; on a
 * timeout it returns RF_ERR_HIP and keeps the server's memory). */
#define RF_SERVE_LAUNCHES 0
#define RF_SERVE_PERSISTENT 1
rf_status rf_server_create_mode(const rf_packed_scene *scene, const rf_params *params, const rf_bound *bound,
                                size_t pool_bytes, int32_t max_inflight, int32_t mode, rf_server **server);
rf_status rf_server_submit(rf_server *server, const rf_camera *camera, int32_t start_cell, uint64_t *req_id);
rf_status rf_server_poll(rf_server *server, uint64_t *done_ids, int32_t cap, int32_t *n_done);
rf_status rf_server_result(rf_server *server, uint64_t req_id, float *rgba, size_t bytes);
rf_status rf_server_stats_get(rf_server *server, rf_server_stats *stats);
rf_status rf_server_destroy(rf_server *server);

#ifdef __cplusplus
}
#endif

#endif /* RADFOAM_H */
