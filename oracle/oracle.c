/*
 * FP64 CPU oracle for the differentiable Voronoi ray walk.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, double-precision
 * statement of what the GPU path computes. Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (Radiant Foam, Sec. 3):
 *   - Voronoi cells, eq. (5): cell i is the set of points whose nearest site
 *     is site i. A ray leaves cell i through the bisector plane of (x_i, x_j)
 *     for some Delaunay neighbour j (Sec. 3.2, Fig. 2 "ray_tracing").
 *   - The ray tracing procedure of Algorithm 1 ("Render(o, d)"): start in the
 *     cell of the origin, repeatedly take the nearest front-facing face, and
 *     composite the segment with eq. (3)-(4) while transmittance exceeds eps.
 *   - Colour of a cell: real spherical harmonics of degree <= 3 evaluated at
 *     the ray direction (Sec. 3.4).
 *   - The analytic gradient of the composited colour w.r.t. densities, SH
 *     coefficients and site positions; geometry enters only through the
 *     segment widths (Sec. 3.1, last paragraph).
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - front face <=> (x_j - x_i) . d > 0 strictly; exit distance
 *     t = (x_j - x_i).((x_i + x_j)/2 - o) / ((x_j - x_i).d).
 *   - ties t_j == t_1 keep the first face in CSR order (strict <).
 *   - transmittance before a segment multiplies the previous segments only
 *     (Algorithm 1's order); eq. (3)'s stray "dt" is ignored.
 *   - rays end at t_max: the segment that reaches t_max is clipped and the
 *     walk stops; a cell with no front face also ends at t_max.
 *   - the exit is clamped to be >= the entry: te = max(t0, min(t1, t_max)).
 *   - the face shared with the previous cell is skipped.
 *   - T > eps is tested before each cell; at most max_steps cells are visited.
 *   - tau = sigma * delta, with tau = 0 when sigma == 0.
 *   - secondary rays (the ray-based effects of Fig. 3): a scene may hold one
 *     analytic sphere, a mirror or a glass interface (refractive index eta
 *     inside, 1 outside). Where a ray crosses it inside cell i, the segment
 *     ends there, and the walk continues in cell i along the reflected or
 *     refracted ray (Snell's law; total internal reflection reflects), which
 *     starts a new leg with t = 0 at the crossing and its own t_max at the
 *     scene bound. The crossing splits the cell's visit in two; the
 *     transmittance test before each cell is not repeated for the second
 *     part. The foam fills the sphere too; one ray continues (no Fresnel
 *     split); crossings after the first max_bounces are ignored.
 *
 * Per-ray status (steps[]): >= 0 the number of visited cells; -1 the start
 * cell is out of range; -2 the walk stopped because max_steps cells were
 * visited while T > eps and the ray had not reached t_max.
 *
 * Return codes: 0 ok, 1 invalid argument, 2 out of memory.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

#define ORC_BAD_START (-1)
#define ORC_MAX_STEPS (-2)

#define ORC_SURF_NONE 0
#define ORC_SURF_MIRROR 1
#define ORC_SURF_GLASS 2

typedef struct {
    int32_t kind;        /* ORC_SURF_* */
    int32_t max_bounces; /* crossings handled per ray */
    double centre[3], radius;
    double ior;          /* glass: refractive index inside the sphere (outside: 1) */
    int32_t bound_kind;  /* where the legs after a crossing end (see exit_distance) */
    double bound[6];
    int32_t fp32_legs;   /* 1: each new leg's origin and direction are rounded to FP32
                            (a leg is then a ray like the caller's, whose origin and
                            direction are FP32); 0: exact FP64 legs */
} orc_surface;

typedef struct {
    const double *sites;   /* [N,3] */
    const int32_t *off;    /* [N+1] */
    const int32_t *idx;    /* [E] */
    const double *density; /* [N] */
    const double *sh;      /* [N,B,3] */
    int64_t n_sites;
    int32_t sh_deg;
    const orc_surface *surf; /* NULL: no surface */
} orc_scene;

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3, l-major, m = -l..l.               */
/* Textbook real form (with the Condon-Shortley phase folded in), written   */
/* as polynomials of the unit direction (x, y, z).                          */
/* ------------------------------------------------------------------------ */

static int sh_count(int deg) { return (deg + 1) * (deg + 1); }

static void sh_basis(int deg, const double d[3], double *Y)
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    Y[0] = 0.5 * sqrt(1.0 / pi);
    if (deg < 1) return;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = k1 * y;
    Y[2] = k1 * z;
    Y[3] = k1 * x;
    if (deg < 2) return;
    Y[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    Y[5] = 0.5 * sqrt(15.0 / pi) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = 0.5 * sqrt(15.0 / pi) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    if (deg < 3) return;
    Y[9] = 0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = 0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    Y[13] = 0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = 0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

int orc_sh_basis(int deg, const double *dirs, int64_t n, double *out)
{
    if (deg < 0 || deg > 3 || n < 0) return ORC_EINVAL;
    const int B = sh_count(deg);
    for (int64_t r = 0; r < n; ++r) sh_basis(deg, dirs + 3 * r, out + B * r);
    return ORC_OK;
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------------ */
/* Camera rays: pinhole, 8x8 screen tiles in row-major order, pixels        */
/* row-major inside a tile; partial tiles at the right/bottom edges hold    */
/* only the pixels inside the image.                                        */
/* ------------------------------------------------------------------------ */

static void tile_pixel(int64_t r, int W, int H, int *px, int *py)
{
    const int64_t band = 8 * (int64_t)W;           /* rays in a full band of tile rows */
    const int ty = (int)(r / band);
    int64_t rem = r - (int64_t)ty * band;
    const int h = (H - 8 * ty) < 8 ? (H - 8 * ty) : 8;
    const int tx = (int)(rem / (8 * h));
    rem -= (int64_t)tx * 8 * h;
    const int w = (W - 8 * tx) < 8 ? (W - 8 * tx) : 8;
    *py = 8 * ty + (int)(rem / w);
    *px = 8 * tx + (int)(rem % w);
}

/* bound_kind 0: axis-aligned box, params = lo[3], hi[3]; 1: sphere about the
 * world origin, params[0] = radius. The origin must lie inside. */
static double exit_distance(int bound_kind, const double *bp, const double o[3], const double d[3])
{
    if (bound_kind == 0) {
        double t = INFINITY;
        for (int a = 0; a < 3; ++a) {
            if (d[a] > 0.0) t = fmin(t, (bp[3 + a] - o[a]) / d[a]);
            else if (d[a] < 0.0) t = fmin(t, (bp[a] - o[a]) / d[a]);
        }
        return fmax(t, 0.0);
    }
    const double b = dot3(o, d);
    const double c = dot3(o, o) - bp[0] * bp[0];
    const double disc = b * b - c;
    return disc > 0.0 ? fmax(-b + sqrt(disc), 0.0) : 0.0;
}

/* model 0, pinhole: the pixel centre's offset (u, v) from the image centre,
 * in pixels, maps to the camera-frame direction (u / f, v / f, 1) normalised,
 * f = (W/2) / tan(fov/2).
 * model 1, equidistant fisheye (a non-linear camera, Fig. 3): the angle from
 * the optical axis grows linearly with the distance rho = |(u, v)| from the
 * image centre, theta = rho (fov/2) / (W/2), so the left and right image
 * edges are at fov/2; the direction is (sin theta u/rho, sin theta v/rho,
 * cos theta) (the axis itself at rho = 0). */
int orc_raygen(const double *pose, double fov_deg, int W, int H, int model, int bound_kind,
               const double *bound_params, double *origin, double *dir, double *tmax, int32_t *pixel)
{
    if (W <= 0 || H <= 0 || bound_kind < 0 || bound_kind > 1 || model < 0 || model > 1) return ORC_EINVAL;
    if (model == 0 && !(fov_deg > 0.0 && fov_deg < 180.0)) return ORC_EINVAL;
    if (model == 1 && !(fov_deg > 0.0 && fov_deg <= 360.0)) return ORC_EINVAL;
    const double half = 0.5 * fov_deg * M_PI / 180.0;
    const double f = 0.5 * W / tan(half);
    const double p[3] = {pose[3], pose[7], pose[11]};
    const int64_t R = (int64_t)W * H;
    for (int64_t r = 0; r < R; ++r) {
        int px, py;
        tile_pixel(r, W, H, &px, &py);
        const double u = px + 0.5 - 0.5 * W, v = py + 0.5 - 0.5 * H;
        double cam[3] = {u / f, v / f, 1.0};
        if (model == 1) {
            const double rho = sqrt(u * u + v * v);
            const double theta = rho * half / (0.5 * W);
            cam[0] = rho > 0.0 ? sin(theta) * u / rho : 0.0;
            cam[1] = rho > 0.0 ? sin(theta) * v / rho : 0.0;
            cam[2] = cos(theta);
        }
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = pose[4 * a + 0] * cam[0] + pose[4 * a + 1] * cam[1] + pose[4 * a + 2] * cam[2];
        const double len = sqrt(dot3(d, d));
        for (int a = 0; a < 3; ++a) {
            d[a] /= len;
            origin[3 * r + a] = p[a];
            dir[3 * r + a] = d[a];
        }
        tmax[r] = exit_distance(bound_kind, bound_params, p, d);
        pixel[r] = py * W + px;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Face planes of the directed Delaunay edges: n = x_j - x_i and            */
/* c = n.(x_i + x_j)/2, so that the bisector is {p : n.p = c}.              */
/* ------------------------------------------------------------------------ */

int orc_face_planes(const double *sites, const int32_t *off, const int32_t *idx, int64_t n_sites, double *planes)
{
    for (int64_t i = 0; i < n_sites; ++i) {
        const double *xi = sites + 3 * i;
        for (int32_t k = off[i]; k < off[i + 1]; ++k) {
            const double *xj = sites + 3 * (int64_t)idx[k];
            double n[3], m[3];
            for (int a = 0; a < 3; ++a) {
                n[a] = xj[a] - xi[a];
                m[a] = 0.5 * (xi[a] + xj[a]);
            }
            planes[4 * (int64_t)k + 0] = n[0];
            planes[4 * (int64_t)k + 1] = n[1];
            planes[4 * (int64_t)k + 2] = n[2];
            planes[4 * (int64_t)k + 3] = dot3(n, m);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The cell containing a point (eq. (5)): its nearest site, by exhaustive   */
/* search over all sites; the lowest index wins an exact tie. gap (if not   */
/* NULL) receives (d2_second - d2_best) / d2_second, the relative distance  */
/* of the runner-up (0 for an exact tie, 1 when the point is a site).       */
/* ------------------------------------------------------------------------ */
int orc_nearest_site(const double *sites, int64_t n_sites, const double *points, int64_t n_points, int32_t *out,
                     double *gap)
{
    if (!sites || n_sites < 1 || n_points < 0 || (n_points > 0 && (!points || !out))) return ORC_EINVAL;
    for (int64_t q = 0; q < n_points; ++q) {
        const double *p = points + 3 * q;
        int64_t best = -1;
        double d_best = INFINITY, d_second = INFINITY;
        for (int64_t i = 0; i < n_sites; ++i) {
            const double dx = p[0] - sites[3 * i], dy = p[1] - sites[3 * i + 1], dz = p[2] - sites[3 * i + 2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < d_best) {
                d_second = d_best;
                d_best = d2;
                best = i;
            } else if (d2 < d_second) {
                d_second = d2;
            }
        }
        out[q] = (int32_t)best;
        if (gap) gap[q] = d_second > 0.0 ? (d_second - d_best) / d_second : 0.0;
    }
    return ORC_OK;
}

/* IEEE binary32 -> bfloat16 with round-to-nearest-even (NaN stays NaN). */
void orc_bf16_round(const float *in, uint16_t *out, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        uint32_t u;
        memcpy(&u, &in[k], 4);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
            out[k] = (uint16_t)((u >> 16) | 0x0040u);
            continue;
        }
        const uint32_t lsb = (u >> 16) & 1u;
        out[k] = (uint16_t)((u + 0x7fffu + lsb) >> 16);
    }
}

int orc_check_csr(const int32_t *off, const int32_t *idx, int64_t n_sites, int64_t n_edges)
{
    if (n_sites < 1 || off[0] != 0 || off[n_sites] != n_edges) return ORC_EINVAL;
    for (int64_t i = 0; i < n_sites; ++i) {
        if (off[i + 1] < off[i]) return ORC_EINVAL;
        for (int32_t k = off[i]; k < off[i + 1]; ++k)
            if (idx[k] < 0 || idx[k] >= n_sites || idx[k] == i) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The walk (Algorithm 1) in FP64, with optional per-visit records.         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t cell;      /* i_n */
    int32_t next;      /* i' (or -1 when no front face) */
    double t0, t1, te; /* entry, nearest front-face distance, clamped exit */
    double den;        /* (x_next - x_cell) . d of the exit face */
    double tau;        /* sigma * delta */
    double T;          /* transmittance before the segment */
    double c[3];       /* cell colour along d */
    int moves;         /* the exit is t1 itself (not clamped, not clipped, not at the surface) */
    int bounce;        /* the segment ends where the leg crosses the surface */
    double o[3], d[3]; /* the leg: t is measured from o along d */
} visit_t;

typedef struct {
    visit_t *v;
    int64_t len, cap;
} visit_buf;

typedef struct {
    double margin;   /* min over decisions of the scaled gap to the runner-up face / t_max */
    double graze;    /* min |cos| over non-front faces other than the entry face */
    double term;     /* min |ln T - ln eps| over the transmittance tests */
    double surf;     /* min over surface decisions: |cos| at a crossing, |1 - eta^2 sin^2| at a
                        refraction, the scaled gap between the crossing and the nearest face / t_max */
    double exit_cos; /* min |cos| of the exit faces whose exits move (the conditioning of the
                        site gradient, which divides by the exit face's n.d) */
} margins_t;

/* Decisions of a walk that FP32 arithmetic may take either way, and walks
 * that take a given alternative at such a decision.
 *
 * A decision is identified by its visit n and its kind: the transmittance
 * test before visit n (kind 0), or the choice of the exit of visit n (kind
 * 1) among the front faces and the end of the ray at t_max. A choice code is
 * a neighbour id (leave through the face to it), ORC_CH_CLIP (the ray ends
 * in this cell at t_max), ORC_CH_STOP or ORC_CH_GO (the transmittance test
 * fails or passes). A decision is a near tie when the exact winner's margin
 * to an alternative is below kappa_t (faces and t_max, in the units of the
 * margin below) or kappa_T (|ln T - ln eps|). */
#define ORC_CH_CLIP (-3)
#define ORC_CH_STOP (-4)
#define ORC_CH_GO (-5)

typedef struct {
    const int32_t *f_visit, *f_choice; /* forced choices, in walk order */
    int32_t nf;
    double kappa_t, kappa_T;
    int32_t *nt_visit, *nt_choice; /* near ties after the last forced decision (alternatives to the exact choice) */
    int32_t nt_cap, nt_len;        /* nt_len = -1: more than nt_cap */
    int bad;                       /* a forced choice was not available */
} walk_ctl;

static void note_tie(walk_ctl *c, int32_t n, int32_t choice)
{
    if (c->nt_len < 0) return;
    if (c->nt_len == c->nt_cap) {
        c->nt_len = -1;
        return;
    }
    c->nt_visit[c->nt_len] = n;
    c->nt_choice[c->nt_len] = choice;
    ++c->nt_len;
}

static void push_visit(visit_buf *b, const visit_t *v)
{
    if (b->len == b->cap) {
        int64_t cap = b->cap ? 2 * b->cap : 256;
        visit_t *p = (visit_t *)realloc(b->v, (size_t)cap * sizeof(visit_t));
        if (!p) abort(); /* the oracle has no graceful path for exhausted host memory */
        b->v = p;
        b->cap = cap;
    }
    b->v[b->len++] = *v;
}

/* Distance along the leg (o, d) to its next crossing of the surface, +inf
 * if none: the far root of |o + t d - c| = radius when the leg starts inside
 * the sphere, the near positive root when it starts outside (a leg leaving
 * the surface outwards has no positive near root). */
static double surface_hit(const orc_surface *sf, const double o[3], const double d[3], int inside)
{
    double oc[3];
    for (int a = 0; a < 3; ++a) oc[a] = o[a] - sf->centre[a];
    const double b = dot3(oc, d);
    const double c = dot3(oc, oc) - sf->radius * sf->radius;
    const double disc = b * b - c;
    if (!(disc > 0.0)) return INFINITY;
    const double t = inside ? -b + sqrt(disc) : -b - sqrt(disc);
    return t > 0.0 ? t : INFINITY;
}

/* The leg after a crossing at p with incoming direction d: the outward unit
 * normal N = (p - c)/|p - c|; a mirror reflects, d' = d - 2 (d.N) N; glass
 * refracts by Snell's law with n1/n2 = 1/eta entering and eta leaving,
 * d' = (n1/n2) d + ((n1/n2) cos_i - cos_t) N_i with N_i the normal against
 * d, cos_i = -d.N_i and cos_t = sqrt(1 - (n1/n2)^2 (1 - cos_i^2)); when the
 * root's argument is negative the ray is totally reflected. Returns the new
 * inside flag; *cos_i and *root report the decision's margins. */
static int surface_turn(const orc_surface *sf, const double p[3], const double d[3], int inside, double dn[3],
                        double *cos_i, double *root)
{
    double N[3];
    for (int a = 0; a < 3; ++a) N[a] = p[a] - sf->centre[a];
    const double len = sqrt(dot3(N, N));
    for (int a = 0; a < 3; ++a) N[a] /= len;
    const double dN = dot3(d, N);
    *cos_i = fabs(dN);
    *root = INFINITY;
    int reflect = sf->kind == ORC_SURF_MIRROR;
    if (!reflect) {
        const double sgn = dN < 0.0 ? 1.0 : -1.0;          /* N_i = sgn N points against d */
        const double eta = dN < 0.0 ? 1.0 / sf->ior : sf->ior; /* n1/n2 */
        const double ci = -sgn * dN;
        const double k = 1.0 - eta * eta * (1.0 - ci * ci);
        *root = fabs(k);
        if (k < 0.0) {
            reflect = 1;
        } else {
            for (int a = 0; a < 3; ++a) dn[a] = eta * d[a] + (eta * ci - sqrt(k)) * sgn * N[a];
            inside = !inside;
        }
    }
    if (reflect)
        for (int a = 0; a < 3; ++a) dn[a] = d[a] - 2.0 * dN * N[a];
    const double l = sqrt(dot3(dn, dn));
    for (int a = 0; a < 3; ++a) dn[a] /= l;
    return inside;
}

/* Walks one ray. Returns the status code written to steps[]. */
static int32_t walk_ray(const orc_scene *s, const double o[3], const double d[3], double tmax, int32_t start,
                        double eps, int32_t max_steps, double rgb[3], double *t_final,
                        visit_buf *rec, margins_t *mg, walk_ctl *ctl)
{
    /* position of a decision in walk order: 2 n + kind */
    int32_t fi = 0;
    const int64_t last_forced =
        (ctl && ctl->nf > 0)
            ? 2 * (int64_t)ctl->f_visit[ctl->nf - 1] +
                  ((ctl->f_choice[ctl->nf - 1] == ORC_CH_STOP || ctl->f_choice[ctl->nf - 1] == ORC_CH_GO) ? 0 : 1)
            : -1;
    const int B = sh_count(s->sh_deg);
    double Y[16];
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    *t_final = 1.0;
    if (mg) {
        mg->margin = INFINITY;
        mg->graze = INFINITY;
        mg->term = INFINITY;
        mg->surf = INFINITY;
        mg->exit_cos = INFINITY;
    }
    if (start < 0 || start >= s->n_sites) return ORC_BAD_START;

    /* the current leg */
    const orc_surface *sf = (s->surf && s->surf->kind != ORC_SURF_NONE) ? s->surf : NULL;
    double lo[3] = {o[0], o[1], o[2]}, ld[3] = {d[0], d[1], d[2]};
    sh_basis(s->sh_deg, ld, Y);
    int inside = 0, bounces = 0;
    double ts = INFINITY;
    if (sf) {
        double oc[3];
        for (int a = 0; a < 3; ++a) oc[a] = o[a] - sf->centre[a];
        inside = dot3(oc, oc) < sf->radius * sf->radius;
        if (sf->max_bounces > 0) ts = surface_hit(sf, lo, ld, inside);
    }

    double t0 = 0.0, T = 1.0;
    int32_t i = start, prev = -1, n = 0, status = 0;
    double scale0 = 1.0 + sqrt(dot3(o, o));
    int cont = 0; /* the visit continues a cell after a crossing: no new transmittance test */
    for (;;) {
        if (!cont) {
            if (mg && eps > 0.0) mg->term = fmin(mg->term, fabs(log(T) - log(eps)));
            int stop = !(T > eps);
            if (ctl) {
                if (fi < ctl->nf && ctl->f_visit[fi] == n &&
                    (ctl->f_choice[fi] == ORC_CH_STOP || ctl->f_choice[fi] == ORC_CH_GO)) {
                    stop = ctl->f_choice[fi] == ORC_CH_STOP;
                    ++fi;
                } else if (2 * (int64_t)n > last_forced && eps > 0.0 && fabs(log(T) - log(eps)) < ctl->kappa_T) {
                    note_tie(ctl, n, stop ? ORC_CH_GO : ORC_CH_STOP);
                }
            }
            if (stop) break;
        }
        cont = 0;
        if (n == max_steps) {
            status = ORC_MAX_STEPS;
            break;
        }

        const double *x = s->sites + 3 * (int64_t)i;
        double t1 = INFINITY, den1 = 0.0, nlen1 = 1.0;
        int32_t inext = -1;
        /* nearest front face; runner-ups are kept for the decision margins */
        double cand_t[512], cand_cos[512];
        int32_t cand_j[512];
        int ncand = 0, win = -1;
        for (int32_t k = s->off[i]; k < s->off[i + 1]; ++k) {
            const int32_t j = s->idx[k];
            if (j == prev) continue;
            const double *xj = s->sites + 3 * (int64_t)j;
            double nv[3], mo[3];
            for (int a = 0; a < 3; ++a) {
                nv[a] = xj[a] - x[a];
                mo[a] = 0.5 * (x[a] + xj[a]) - lo[a];
            }
            const double den = dot3(nv, ld);
            const double nlen = sqrt(dot3(nv, nv));
            if (!(den > 0.0)) {
                if (mg) mg->graze = fmin(mg->graze, fabs(den) / nlen);
                continue;
            }
            const double t = dot3(nv, mo) / den;
            if ((mg || ctl) && ncand < 512) {
                cand_t[ncand] = t;
                cand_cos[ncand] = den / nlen;
                cand_j[ncand] = j;
                ++ncand;
            }
            if (t < t1) {
                t1 = t;
                inext = j;
                den1 = den;
                nlen1 = nlen;
                win = ncand - 1;
            }
        }

        /* near ties of this exit, and a forced choice */
        int force_clip = 0;
        if (ctl) {
            const int64_t pos = 2 * (int64_t)n + 1;
            if (fi < ctl->nf && ctl->f_visit[fi] == n && ctl->f_choice[fi] != ORC_CH_STOP &&
                ctl->f_choice[fi] != ORC_CH_GO) {
                const int32_t c = ctl->f_choice[fi++];
                if (c == ORC_CH_CLIP) {
                    force_clip = 1;
                } else {
                    int q = 0;
                    while (q < ncand && cand_j[q] != c) ++q;
                    if (q < ncand) {
                        /* leave through the face to c; its den as the scan computed it */
                        double nv[3];
                        for (int a = 0; a < 3; ++a) nv[a] = s->sites[3 * (int64_t)c + a] - x[a];
                        t1 = cand_t[q];
                        inext = c;
                        den1 = dot3(nv, ld);
                        nlen1 = sqrt(dot3(nv, nv));
                        win = q;
                        /* the face taken instead of the end of the ray: its exit lies at t_max */
                        if (t1 >= tmax) t1 = nextafter(tmax, -INFINITY);
                    } else {
                        ctl->bad = 1;
                    }
                }
            } else if (pos > last_forced && inext >= 0) {
                const double scale = scale0 + fabs(t1);
                const double cos1 = den1 / nlen1;
                if (t1 < tmax) {
                    for (int q = 0; q < ncand; ++q) {
                        if (q == win || !(cand_t[q] < tmax)) continue;
                        if ((cand_t[q] - t1) / (scale * (1.0 / cos1 + 1.0 / cand_cos[q])) < ctl->kappa_t)
                            note_tie(ctl, n, cand_j[q]);
                    }
                    if ((tmax - t1) * cos1 / scale < ctl->kappa_t) note_tie(ctl, n, ORC_CH_CLIP);
                } else if ((t1 - tmax) * cos1 / scale < ctl->kappa_t) {
                    note_tie(ctl, n, inext);
                }
            }
        }
        double te = force_clip ? fmax(t0, tmax) : fmax(t0, fmin(t1, tmax));
        /* the leg crosses the surface inside this cell */
        const int bounce = ts < te;
        if (mg && sf && isfinite(ts)) {
            const double scale = scale0 + ts;
            mg->surf = fmin(mg->surf, fabs(ts - fmin(t1, tmax)) / scale);
        }
        if (bounce) te = ts;
        const double delta = te - t0;
        const double sigma = s->density[i];
        const double tau = (sigma == 0.0) ? 0.0 : sigma * delta;
        const double alpha = -expm1(-tau);
        double c[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < B; ++b)
            for (int ch = 0; ch < 3; ++ch) c[ch] += s->sh[(3 * (int64_t)B) * i + 3 * b + ch] * Y[b];
        for (int ch = 0; ch < 3; ++ch) rgb[ch] += T * alpha * c[ch];

        const int clipped = !bounce && ((inext < 0) || (t1 >= tmax) || force_clip);
        if (mg && inext >= 0 && !bounce) {
            const double scale = scale0 + fabs(t1);
            const double cos1 = den1 / nlen1;
            for (int q = 0; q < ncand; ++q) {
                if (q == win) continue;
                const double m = (cand_t[q] - t1) / (scale * (1.0 / cos1 + 1.0 / cand_cos[q]));
                mg->margin = fmin(mg->margin, m);
            }
            mg->margin = fmin(mg->margin, fabs(t1 - tmax) * cos1 / scale);
            if (!clipped && t1 >= t0) mg->exit_cos = fmin(mg->exit_cos, cos1);
        }
        if (rec) {
            visit_t v;
            v.cell = i;
            v.next = inext;
            v.t0 = t0;
            v.t1 = t1;
            v.te = te;
            v.den = den1;
            v.tau = tau;
            v.T = T;
            v.c[0] = c[0];
            v.c[1] = c[1];
            v.c[2] = c[2];
            v.moves = (!clipped) && (!bounce) && (t1 >= t0);
            v.bounce = bounce;
            for (int a = 0; a < 3; ++a) {
                v.o[a] = lo[a];
                v.d[a] = ld[a];
            }
            push_visit(rec, &v);
        }
        T *= exp(-tau);
        ++n;
        if (clipped) break;
        if (bounce) {
            /* a new leg from the crossing, in the same cell; every face of
               the cell is a candidate again */
            double p[3], dn[3], ci, root;
            for (int a = 0; a < 3; ++a) p[a] = lo[a] + ts * ld[a];
            inside = surface_turn(sf, p, ld, inside, dn, &ci, &root);
            if (mg) mg->surf = fmin(mg->surf, fmin(ci, root));
            for (int a = 0; a < 3; ++a) {
                lo[a] = sf->fp32_legs ? (double)(float)p[a] : p[a];
                ld[a] = sf->fp32_legs ? (double)(float)dn[a] : dn[a];
            }
            sh_basis(s->sh_deg, ld, Y);
            tmax = exit_distance(sf->bound_kind, sf->bound, lo, ld);
            ++bounces;
            ts = bounces < sf->max_bounces ? surface_hit(sf, lo, ld, inside) : INFINITY;
            scale0 = 1.0 + sqrt(dot3(lo, lo));
            prev = -1;
            t0 = 0.0;
            cont = 1;
            continue;
        }
        prev = i;
        i = inext;
        t0 = te;
    }
    *t_final = T;
    return status ? status : n;
}

/* ------------------------------------------------------------------------ */
/* Analytic gradient of one ray (from its stored visits).                   */
/*   w_n = T_n alpha_n, R_n = sum_{k>n} w_k c_k                             */
/*   dL/dtau_n = g.(T_{n+1} c_n - R_n) - gT T_final                          */
/*   dL/dsigma_{i_n} += delta_n dL/dtau_n                                   */
/*   dL/dK_{i_n,b,ch} += g_ch w_n Y_b                                       */
/*   for an exit that moves with t1:                                        */
/*     dL/dt_n = sigma_n dL/dtau_n - sigma_{n+1} dL/dtau_{n+1}              */
/*     dt/dx_{i_n} = (p - x_{i_n})/den, dt/dx_{i_{n+1}} = (x_{i_{n+1}} - p)/den */
/*     with p = o + t_n d and den = (x_{i_{n+1}} - x_{i_n}).d, o and d the   */
/*     visit's leg (its SH basis Y is the leg's too)                        */
/* ------------------------------------------------------------------------ */

static void ray_gradient(const orc_scene *s, const visit_t *v, int64_t nv, double T_final, const double g[3],
                         double gT, double *gsites, double *gdens, double *gsh)
{
    const int B = sh_count(s->sh_deg);
    double Y[16];
    double *R = (double *)malloc((size_t)(nv > 0 ? nv : 1) * 3 * sizeof(double));
    double *dtau = (double *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(double));
    if (!R || !dtau) {
        free(R);
        free(dtau);
        return;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t n = nv - 1; n >= 0; --n) {
        const double w = v[n].T * (-expm1(-v[n].tau));
        for (int ch = 0; ch < 3; ++ch) {
            R[3 * n + ch] = acc[ch];
            acc[ch] += w * v[n].c[ch];
        }
    }
    for (int64_t n = 0; n < nv; ++n) {
        const double Tn1 = v[n].T * exp(-v[n].tau);
        double s_ = 0.0;
        for (int ch = 0; ch < 3; ++ch) s_ += g[ch] * (Tn1 * v[n].c[ch] - R[3 * n + ch]);
        dtau[n] = s_ - gT * T_final;
        const int32_t i = v[n].cell;
        const double w = v[n].T * (-expm1(-v[n].tau));
        gdens[i] += (v[n].te - v[n].t0) * dtau[n];
        sh_basis(s->sh_deg, v[n].d, Y); /* the basis of the visit's leg */
        for (int b = 0; b < B; ++b)
            for (int ch = 0; ch < 3; ++ch) gsh[(3 * (int64_t)B) * i + 3 * b + ch] += g[ch] * w * Y[b];
    }
    for (int64_t n = 0; n < nv; ++n) {
        if (!v[n].moves) continue;
        const int32_t i = v[n].cell, j = v[n].next;
        double gt = s->density[i] * dtau[n];
        if (n + 1 < nv) gt -= s->density[v[n + 1].cell] * dtau[n + 1];
        const double *xi = s->sites + 3 * (int64_t)i;
        const double *xj = s->sites + 3 * (int64_t)j;
        for (int a = 0; a < 3; ++a) {
            const double p = v[n].o[a] + v[n].t1 * v[n].d[a];
            gsites[3 * (int64_t)i + a] += gt * (p - xi[a]) / v[n].den;
            gsites[3 * (int64_t)j + a] += gt * (xj[a] - p) / v[n].den;
        }
    }
    free(R);
    free(dtau);
}

/* ------------------------------------------------------------------------ */
/* Threaded drivers.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_scene *s;
    const double *o, *d, *tmax;
    const int32_t *start;
    int64_t r0, r1;
    double eps;
    int32_t max_steps;
    /* forward */
    double *rgb, *t_final;
    int32_t *steps;
    /* trace */
    int32_t max_len;
    int32_t *cells;
    double *t_exit;
    int32_t *len;
    double *margin, *graze, *term;
    int8_t *bounce;   /* [R][max_len], nullable */
    double *legs;     /* [R][max_len][6]: each visit's leg origin and direction, nullable */
    double *surf_margin;
    double *exit_cos;
    /* backward */
    const double *grad_rgb, *grad_t;
    double *gsites, *gdens, *gsh;
    /* quantile regulariser */
    const double *u, *grad_loss;
    double *tq, *loss;
    /* forced choices (per ray, or per job of orc_walk_forced) and near ties */
    const int32_t *ray_idx;
    const int64_t *f_off;
    const int32_t *f_visit, *f_choice;
    double kappa_t, kappa_T;
    int32_t nt_cap;
    int32_t *nt_visit, *nt_choice, *nt_len, *bad;
    int status;
} job_t;

static int check_inputs(const orc_scene *s, const double *d, int64_t n_rays)
{
    if (!s || s->n_sites < 1 || s->sh_deg < 0 || s->sh_deg > 3 || n_rays < 0) return ORC_EINVAL;
    if (s->surf) {
        const orc_surface *sf = s->surf;
        if (sf->kind < ORC_SURF_NONE || sf->kind > ORC_SURF_GLASS || sf->max_bounces < 0 || !(sf->radius > 0.0) ||
            (sf->kind == ORC_SURF_GLASS && !(sf->ior > 0.0)) || sf->bound_kind < 0 || sf->bound_kind > 1)
            return ORC_EINVAL;
    }
    if (orc_check_csr(s->off, s->idx, s->n_sites, s->off[s->n_sites]) != ORC_OK) return ORC_EINVAL;
    for (int64_t i = 0; i < s->n_sites; ++i)
        if (s->off[i + 1] - s->off[i] > 512) return ORC_EINVAL; /* decision-margin buffer */
    for (int64_t r = 0; r < n_rays; ++r)
        if (fabs(sqrt(dot3(d + 3 * r, d + 3 * r)) - 1.0) > 1e-5) return ORC_EINVAL;
    for (int64_t i = 0; i < s->n_sites; ++i)
        if (!(s->density[i] >= 0.0)) return ORC_EINVAL;
    return ORC_OK;
}

static void *forward_worker(void *arg)
{
    job_t *j = (job_t *)arg;
    visit_buf buf = {0, 0, 0};
    for (int64_t r = j->r0; r < j->r1; ++r) {
        margins_t mg;
        const int tracing = j->cells != NULL;
        buf.len = 0;
        j->steps[r] = walk_ray(j->s, j->o + 3 * r, j->d + 3 * r, j->tmax[r], j->start[r], j->eps, j->max_steps,
                               j->rgb + 3 * r, j->t_final + r, tracing ? &buf : NULL, tracing ? &mg : NULL, NULL);
        if (tracing) {
            const int64_t L = buf.len < j->max_len ? buf.len : j->max_len;
            for (int64_t n = 0; n < L; ++n) {
                j->cells[r * j->max_len + n] = buf.v[n].cell;
                j->t_exit[r * j->max_len + n] = buf.v[n].te;
                if (j->bounce) j->bounce[r * j->max_len + n] = (int8_t)buf.v[n].bounce;
                if (j->legs)
                    for (int a = 0; a < 3; ++a) {
                        j->legs[(r * j->max_len + n) * 6 + a] = buf.v[n].o[a];
                        j->legs[(r * j->max_len + n) * 6 + 3 + a] = buf.v[n].d[a];
                    }
            }
            j->len[r] = (int32_t)buf.len;
            j->margin[r] = mg.margin;
            j->graze[r] = mg.graze;
            j->term[r] = mg.term;
            if (j->surf_margin) j->surf_margin[r] = mg.surf;
            if (j->exit_cos) j->exit_cos[r] = mg.exit_cos;
        }
    }
    free(buf.v);
    return NULL;
}

static void *backward_worker(void *arg)
{
    job_t *j = (job_t *)arg;
    visit_buf buf = {0, 0, 0};
    for (int64_t r = j->r0; r < j->r1; ++r) {
        double rgb[3], tf;
        buf.len = 0;
        walk_ctl ctl;
        memset(&ctl, 0, sizeof ctl);
        if (j->f_off) {
            ctl.f_visit = j->f_visit + j->f_off[r];
            ctl.f_choice = j->f_choice + j->f_off[r];
            ctl.nf = (int32_t)(j->f_off[r + 1] - j->f_off[r]);
            ctl.nt_len = -1; /* nothing recorded */
        }
        const int32_t st = walk_ray(j->s, j->o + 3 * r, j->d + 3 * r, j->tmax[r], j->start[r], j->eps, j->max_steps,
                                    rgb, &tf, &buf, NULL, j->f_off ? &ctl : NULL);
        if (st == ORC_BAD_START) continue;
        const double gT = j->grad_t ? j->grad_t[r] : 0.0;
        ray_gradient(j->s, buf.v, buf.len, tf, j->grad_rgb + 3 * r, gT, j->gsites, j->gdens, j->gsh);
    }
    free(buf.v);
    return NULL;
}

/* Walks of orc_walk_forced: job q walks ray ray_idx[q] with the forced
 * choices f_visit/f_choice[f_off[q] .. f_off[q+1]) and records its cells and
 * the near ties after the last forced decision. */
static void *forced_worker(void *arg)
{
    job_t *j = (job_t *)arg;
    visit_buf buf = {0, 0, 0};
    for (int64_t q = j->r0; q < j->r1; ++q) {
        const int64_t r = j->ray_idx[q];
        walk_ctl ctl;
        memset(&ctl, 0, sizeof ctl);
        ctl.f_visit = j->f_visit + j->f_off[q];
        ctl.f_choice = j->f_choice + j->f_off[q];
        ctl.nf = (int32_t)(j->f_off[q + 1] - j->f_off[q]);
        ctl.kappa_t = j->kappa_t;
        ctl.kappa_T = j->kappa_T;
        ctl.nt_visit = j->nt_visit + q * j->nt_cap;
        ctl.nt_choice = j->nt_choice + q * j->nt_cap;
        ctl.nt_cap = j->nt_cap;
        buf.len = 0;
        j->steps[q] = walk_ray(j->s, j->o + 3 * r, j->d + 3 * r, j->tmax[r], j->start[r], j->eps, j->max_steps,
                               j->rgb + 3 * q, j->t_final + q, &buf, NULL, &ctl);
        const int64_t L = buf.len < j->max_len ? buf.len : j->max_len;
        for (int64_t n = 0; n < L; ++n) j->cells[q * j->max_len + n] = buf.v[n].cell;
        j->len[q] = (int32_t)buf.len;
        j->nt_len[q] = ctl.nt_len;
        j->bad[q] = ctl.bad;
    }
    free(buf.v);
    return NULL;
}

/* ------------------------------------------------------------------------ */
/* Quantile regulariser (Sec. 3.4, training objectives): for a ray with     */
/* composited segments n (weights w_n = T_n alpha_n), W(t) is the weight    */
/* accumulated up to distance t; inside a segment the density is constant,  */
/* so W(t) = W(t0_n) + T_n (1 - exp(-sigma_n (t - t0_n))). The quantile      */
/* W^-1(u) of the normalised distribution is the t at which W(t) reaches     */
/* u A, A = sum of the w_n (the ray's opacity, 1 - T_final). The loss of a   */
/* ray is |W^-1(u1) - W^-1(u2)| for its two draws u1, u2.                   */
/* ------------------------------------------------------------------------ */

/* W^-1(u) for the visits v[0..nv): returns the segment index (-1 if A = 0). */
static int64_t quantile_point(const orc_scene *s, const visit_t *v, int64_t nv, double u, double *tstar)
{
    double A = 0.0;
    for (int64_t n = 0; n < nv; ++n) A += v[n].T * (-expm1(-v[n].tau));
    *tstar = 0.0;
    if (!(A > 0.0)) return -1;
    const double m = u * A;
    double cum = 0.0;
    int64_t last = -1;
    for (int64_t n = 0; n < nv; ++n) {
        const double w = v[n].T * (-expm1(-v[n].tau));
        if (!(w > 0.0)) continue;
        last = n;
        if (cum + w >= m) {
            const double sigma = s->density[v[n].cell];
            double t = v[n].t0 - log1p(-(m - cum) / v[n].T) / sigma;
            if (t > v[n].te) t = v[n].te;
            if (t < v[n].t0) t = v[n].t0;
            *tstar = t;
            return n;
        }
        cum += w;
    }
    *tstar = v[last].te; /* u A beyond the rounded total: the end of the last weighted segment */
    return last;
}

/* Adds c (d t_star / d theta) to the density and site gradients, by implicit
 * differentiation of W(t_star) = u A: d t_star = (u dA - dW(t_star)) / (T(t_star) sigma_k),
 * where T(t_star) = 1 - W(t_star) and theta ranges over the densities and the exit
 * distances of moving faces (whose site gradients follow as in ray_gradient). */
static void quantile_gradient(const orc_scene *s, const double o[3], const double d[3], const visit_t *v, int64_t nv,
                              double u, double tstar, int64_t k, double c, double *gsites, double *gdens)
{
    double A = 0.0;
    for (int64_t n = 0; n < nv; ++n) A += v[n].T * (-expm1(-v[n].tau));
    const double Tf = 1.0 - A;
    const double sk = s->density[v[k].cell];
    const double Tstar = v[k].T * exp(-sk * (tstar - v[k].t0));
    const double den = Tstar * sk;
    for (int64_t n = 0; n < nv; ++n) {
        const double delta = v[n].te - v[n].t0;
        const double dA = Tf * delta;
        const double dW = n < k ? Tstar * delta : (n == k ? Tstar * (tstar - v[k].t0) : 0.0);
        gdens[v[n].cell] += c * (u * dA - dW) / den;
    }
    for (int64_t m = 0; m < nv; ++m) {
        if (!v[m].moves) continue;
        const double sm = s->density[v[m].cell];
        const double sm1 = m + 1 < nv ? s->density[v[m + 1].cell] : 0.0;
        const double dA = Tf * (sm - sm1);
        const double dW = m + 1 < k ? Tstar * (sm - sm1) : (m + 1 == k ? Tstar * (sm - sk) : 0.0);
        const double gt = c * (u * dA - dW) / den;
        const int32_t i = v[m].cell, j = v[m].next;
        const double *xi = s->sites + 3 * (int64_t)i;
        const double *xj = s->sites + 3 * (int64_t)j;
        for (int a = 0; a < 3; ++a) {
            const double p = o[a] + v[m].t1 * d[a];
            gsites[3 * (int64_t)i + a] += gt * (p - xi[a]) / v[m].den;
            gsites[3 * (int64_t)j + a] += gt * (xj[a] - p) / v[m].den;
        }
    }
}

static void *quantile_worker(void *arg)
{
    job_t *j = (job_t *)arg;
    visit_buf buf = {0, 0, 0};
    for (int64_t r = j->r0; r < j->r1; ++r) {
        double rgb[3], tf, t[2];
        int64_t k[2];
        buf.len = 0;
        const int32_t st = walk_ray(j->s, j->o + 3 * r, j->d + 3 * r, j->tmax[r], j->start[r], j->eps, j->max_steps,
                                    rgb, &tf, &buf, NULL, NULL);
        for (int q = 0; q < 2; ++q) {
            k[q] = st == ORC_BAD_START ? -1 : quantile_point(j->s, buf.v, buf.len, j->u[2 * r + q], &t[q]);
            if (k[q] < 0) t[q] = 0.0;
            j->tq[2 * r + q] = t[q];
        }
        j->loss[r] = (k[0] < 0 || k[1] < 0) ? 0.0 : fabs(t[0] - t[1]);
        if (!j->grad_loss || k[0] < 0 || k[1] < 0 || t[0] == t[1]) continue;
        const double sg = t[0] > t[1] ? 1.0 : -1.0;
        for (int q = 0; q < 2; ++q)
            quantile_gradient(j->s, j->o + 3 * r, j->d + 3 * r, buf.v, buf.len, j->u[2 * r + q], t[q], k[q],
                              (q == 0 ? sg : -sg) * j->grad_loss[r], j->gsites, j->gdens);
    }
    free(buf.v);
    return NULL;
}

static int run_jobs(job_t *proto, int64_t n_rays, int nthreads, void *(*fn)(void *), int with_grad_buffers)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (n_rays < nthreads) nthreads = n_rays > 0 ? (int)n_rays : 1;
    job_t jobs[256];
    pthread_t th[256];
    const int64_t N = proto->s->n_sites;
    const int64_t B = sh_count(proto->s->sh_deg);
    const int64_t per = 3 * N + N + 3 * B * N;
    double *grad_mem = NULL;
    if (with_grad_buffers && nthreads > 1) {
        grad_mem = (double *)calloc((size_t)(nthreads - 1) * (size_t)per, sizeof(double));
        if (!grad_mem) return ORC_ENOMEM;
    }
    /* contiguous chunks of screen tiles: chunk boundaries are multiples of 64 rays */
    int64_t chunk = (n_rays + nthreads - 1) / nthreads;
    chunk = (chunk + 63) / 64 * 64;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].r0 = t * chunk < n_rays ? t * chunk : n_rays;
        jobs[t].r1 = (t + 1) * chunk < n_rays ? (t + 1) * chunk : n_rays;
        if (grad_mem && t > 0) {
            double *base = grad_mem + (int64_t)(t - 1) * per;
            jobs[t].gsites = base;
            jobs[t].gdens = base + 3 * N;
            jobs[t].gsh = base + 4 * N;
        }
        pthread_create(&th[t], NULL, fn, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    if (grad_mem) {
        for (int t = 1; t < nthreads; ++t) {
            const double *base = grad_mem + (int64_t)(t - 1) * per;
            for (int64_t k = 0; k < 3 * N; ++k) proto->gsites[k] += base[k];
            for (int64_t k = 0; k < N; ++k) proto->gdens[k] += base[3 * N + k];
            for (int64_t k = 0; k < 3 * B * N; ++k) proto->gsh[k] += base[4 * N + k];
        }
        free(grad_mem);
    }
    return ORC_OK;
}

int orc_forward(const orc_scene *s, const double *o, const double *d, const double *tmax, const int32_t *start,
                int64_t n_rays, double eps, int32_t max_steps, int nthreads, double *rgb, double *t_final,
                int32_t *steps)
{
    if (check_inputs(s, d, n_rays) != ORC_OK || max_steps < 1) return ORC_EINVAL;
    job_t j;
    memset(&j, 0, sizeof j);
    j.s = s;
    j.o = o;
    j.d = d;
    j.tmax = tmax;
    j.start = start;
    j.eps = eps;
    j.max_steps = max_steps;
    j.rgb = rgb;
    j.t_final = t_final;
    j.steps = steps;
    return run_jobs(&j, n_rays, nthreads, forward_worker, 0);
}

/* bounce, legs, surf_margin and exit_cos are optional (NULL) outputs. */
int orc_trace(const orc_scene *s, const double *o, const double *d, const double *tmax, const int32_t *start,
              int64_t n_rays, double eps, int32_t max_steps, int32_t max_len, int nthreads, double *rgb,
              double *t_final, int32_t *steps, int32_t *cells, double *t_exit, int32_t *len, double *margin,
              double *graze, double *term, int8_t *bounce, double *legs, double *surf_margin, double *exit_cos)
{
    if (check_inputs(s, d, n_rays) != ORC_OK || max_steps < 1 || max_len < 1) return ORC_EINVAL;
    job_t j;
    memset(&j, 0, sizeof j);
    j.s = s;
    j.o = o;
    j.d = d;
    j.tmax = tmax;
    j.start = start;
    j.eps = eps;
    j.max_steps = max_steps;
    j.rgb = rgb;
    j.t_final = t_final;
    j.steps = steps;
    j.max_len = max_len;
    j.cells = cells;
    j.t_exit = t_exit;
    j.len = len;
    j.margin = margin;
    j.graze = graze;
    j.term = term;
    j.bounce = bounce;
    j.legs = legs;
    j.surf_margin = surf_margin;
    j.exit_cos = exit_cos;
    return run_jobs(&j, n_rays, nthreads, forward_worker, 0);
}

/* Walks of rays with forced choices (see walk_ctl): job q walks ray
 * ray_idx[q] taking the choices f_visit/f_choice[f_off[q] .. f_off[q+1]) (in
 * walk order) and reports its colour, transmittance, status, cells (the
 * first max_len) and visit count, the near ties after its last forced
 * decision (up to nt_cap; nt_len = -1 if more) and whether a forced choice was
 * not available (bad). */
int orc_walk_forced(const orc_scene *s, const double *o, const double *d, const double *tmax, const int32_t *start,
                    int64_t n_rays, const int32_t *ray_idx, int64_t n_jobs, const int64_t *f_off,
                    const int32_t *f_visit, const int32_t *f_choice, double eps, int32_t max_steps, double kappa_t,
                    double kappa_T, int32_t max_len, int32_t nt_cap, int nthreads, double *rgb, double *t_final,
                    int32_t *steps, int32_t *cells, int32_t *len, int32_t *nt_visit, int32_t *nt_choice,
                    int32_t *nt_len, int32_t *bad)
{
    if (check_inputs(s, d, n_rays) != ORC_OK || max_steps < 1 || max_len < 1 || nt_cap < 0 || n_jobs < 0)
        return ORC_EINVAL;
    for (int64_t q = 0; q < n_jobs; ++q)
        if (ray_idx[q] < 0 || ray_idx[q] >= n_rays || f_off[q + 1] < f_off[q]) return ORC_EINVAL;
    job_t j;
    memset(&j, 0, sizeof j);
    j.s = s;
    j.o = o;
    j.d = d;
    j.tmax = tmax;
    j.start = start;
    j.eps = eps;
    j.max_steps = max_steps;
    j.ray_idx = ray_idx;
    j.f_off = f_off;
    j.f_visit = f_visit;
    j.f_choice = f_choice;
    j.kappa_t = kappa_t;
    j.kappa_T = kappa_T;
    j.max_len = max_len;
    j.nt_cap = nt_cap;
    j.rgb = rgb;
    j.t_final = t_final;
    j.steps = steps;
    j.cells = cells;
    j.len = len;
    j.nt_visit = nt_visit;
    j.nt_choice = nt_choice;
    j.nt_len = nt_len;
    j.bad = bad;
    return run_jobs(&j, n_jobs, nthreads, forced_worker, 0);
}

/* Gradients are accumulated (+=) into the caller's buffers. With f_off
 * (nullable) ray r takes the forced choices f_visit/f_choice[f_off[r] ..
 * f_off[r+1]) (see orc_walk_forced). */
int orc_backward(const orc_scene *s, const double *o, const double *d, const double *tmax, const int32_t *start,
                 int64_t n_rays, double eps, int32_t max_steps, const double *grad_rgb, const double *grad_t,
                 int nthreads, double *grad_sites, double *grad_density, double *grad_sh, const int64_t *f_off,
                 const int32_t *f_visit, const int32_t *f_choice)
{
    if (check_inputs(s, d, n_rays) != ORC_OK || max_steps < 1) return ORC_EINVAL;
    job_t j;
    memset(&j, 0, sizeof j);
    j.s = s;
    j.o = o;
    j.d = d;
    j.tmax = tmax;
    j.start = start;
    j.eps = eps;
    j.max_steps = max_steps;
    j.grad_rgb = grad_rgb;
    j.grad_t = grad_t;
    j.gsites = grad_sites;
    j.gdens = grad_density;
    j.gsh = grad_sh;
    j.f_off = f_off;
    j.f_visit = f_visit;
    j.f_choice = f_choice;
    return run_jobs(&j, n_rays, nthreads, backward_worker, 1);
}

int orc_quantile(const orc_scene *s, const double *o, const double *d, const double *tmax, const int32_t *start,
                 int64_t n_rays, double eps, int32_t max_steps, const double *u, const double *grad_loss, int nthreads,
                 double *tq, double *loss, double *grad_sites, double *grad_density)
{
    if (check_inputs(s, d, n_rays) != ORC_OK || max_steps < 1 || !u || !tq || !loss) return ORC_EINVAL;
    if (s->surf && s->surf->kind != ORC_SURF_NONE) return ORC_EINVAL; /* quantiles along one leg only */
    for (int64_t r = 0; r < 2 * n_rays; ++r)
        if (!(u[r] >= 0.0 && u[r] <= 1.0)) return ORC_EINVAL;
    if (grad_loss && (!grad_sites || !grad_density)) return ORC_EINVAL;
    job_t j;
    memset(&j, 0, sizeof j);
    j.s = s;
    j.o = o;
    j.d = d;
    j.tmax = tmax;
    j.start = start;
    j.eps = eps;
    j.max_steps = max_steps;
    j.u = u;
    j.grad_loss = grad_loss;
    j.tq = tq;
    j.loss = loss;
    double *dummy_sh = NULL, *dummy_s = NULL, *dummy_d = NULL;
    if (grad_loss) {
        j.gsites = grad_sites;
        j.gdens = grad_density;
    } else {
        dummy_s = (double *)calloc((size_t)3 * s->n_sites, sizeof(double));
        dummy_d = (double *)calloc((size_t)s->n_sites, sizeof(double));
        j.gsites = dummy_s;
        j.gdens = dummy_d;
    }
    dummy_sh = (double *)calloc((size_t)3 * sh_count(s->sh_deg) * s->n_sites, sizeof(double));
    j.gsh = dummy_sh;
    int rc = (!dummy_sh || !j.gsites || !j.gdens) ? ORC_ENOMEM
                                                    : run_jobs(&j, n_rays, nthreads, quantile_worker, 1);
    free(dummy_sh);
    free(dummy_s);
    free(dummy_d);
    return rc;
}
