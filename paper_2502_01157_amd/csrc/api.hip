// C ABI of librf.so: argument validation, workspace layout, dispatch.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "radfoam.h"
#include "rf_device.hpp"
#include "rf_kernels.hpp"

namespace {

thread_local char g_err[512] = "";

rf_status fail(rf_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

rf_status ok()
{
    g_err[0] = '\0';
    return RF_OK;
}

rf_status hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return ok();
    return fail(RF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t planes, adj, row, rec, err, total;
    int rec_bytes;
};

Layout layout(int64_t n, int64_t e, int deg, bool bf16)
{
    Layout L;
    L.rec_bytes = rf::rec_bytes(deg, bf16);
    size_t p = 0;
    L.planes = p;
    p = align256(p + ((size_t)e + 4) * 16);  // 4 padding faces: the scan reads in batches of four
    L.adj = p;
    p = align256(p + (size_t)e * 8);
    L.row = p;
    p = align256(p + (size_t)n * 8);
    L.rec = p;
    p = align256(p + (size_t)n * L.rec_bytes);
    L.err = p;
    p = align256(p + 8);
    L.total = p;
    return L;
}

rf_status check_packed(const rf_packed_scene* s)
{
    if (!s || !s->base) return fail(RF_ERR_INVALID_ARG, "packed scene is NULL or has no workspace");
    if (s->sh_degree < 0 || s->sh_degree > RF_MAX_SH_DEGREE)
        return fail(RF_ERR_INVALID_ARG, "packed scene has sh_degree %d", s->sh_degree);
    if (s->attr_dtype != RF_F32 && s->attr_dtype != RF_BF16)
        return fail(RF_ERR_INVALID_ARG, "packed scene has attr_dtype %d", (int)s->attr_dtype);
    if (s->n_sites < 1 || s->n_sites > RF_MAX_SITES || s->n_edges < 0 || s->n_edges > INT32_MAX)
        return fail(RF_ERR_INVALID_ARG, "packed scene sizes out of range");
    const Layout L = layout(s->n_sites, s->n_edges, s->sh_degree, s->attr_dtype == RF_BF16);
    if (s->bytes < L.total || s->off_planes != L.planes || s->off_adj != L.adj || s->off_row != L.row ||
        s->off_rec != L.rec || s->off_err != L.err || s->rec_bytes != L.rec_bytes)
        return fail(RF_ERR_INVALID_ARG, "packed scene descriptor does not match its sizes (not from rf_pack_scene?)");
    return RF_OK;
}

rf::SceneView view(const rf_packed_scene* s)
{
    const unsigned char* b = static_cast<const unsigned char*>(s->base);
    rf::SceneView v;
    v.planes = reinterpret_cast<const float4*>(b + s->off_planes);
    v.adj = reinterpret_cast<const uint2*>(b + s->off_adj);
    v.row = reinterpret_cast<const uint2*>(b + s->off_row);
    v.rec = b + s->off_rec;
    v.n_sites = s->n_sites;
    v.n_edges = s->n_edges;
    return v;
}

rf_status check_rays(const rf_rays* rays)
{
    if (!rays) return fail(RF_ERR_INVALID_ARG, "rays is NULL");
    if (rays->n_rays < 0 || rays->n_rays > ((int64_t)1 << 37))
        return fail(RF_ERR_INVALID_ARG, "n_rays = %lld out of range", (long long)rays->n_rays);
    if (rays->n_rays > 0 && (!rays->origin || !rays->dir || !rays->t_max || !rays->start_cell))
        return fail(RF_ERR_INVALID_ARG, "a ray array is NULL");
    return RF_OK;
}

rf_status check_params(const rf_params* p)
{
    if (!p) return fail(RF_ERR_INVALID_ARG, "params is NULL");
    if (!(p->eps >= 0.0f) || !isfinite(p->eps)) return fail(RF_ERR_INVALID_ARG, "eps must be finite and >= 0");
    if (p->max_steps < 1) return fail(RF_ERR_INVALID_ARG, "max_steps must be >= 1");
    return RF_OK;
}

rf::WalkArgs walk_args(const rf_packed_scene* s, const rf_rays* r, const rf_params* p)
{
    rf::WalkArgs a;
    memset(&a, 0, sizeof a);
    a.s = view(s);
    a.origin = r->origin;
    a.dir = r->dir;
    a.t_max = r->t_max;
    a.start = r->start_cell;
    a.n_rays = r->n_rays;
    a.eps = p->eps;
    a.max_steps = p->max_steps;
    return a;
}

}  // namespace

void rf::set_error(const char* msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
}

extern "C" {

const char* rf_last_error(void) { return g_err; }

const char* rf_version(void) { return "radfoam-mi355x 0.1 (gfx950)"; }

rf_status rf_packed_bytes(int64_t n_sites, int64_t n_edges, int32_t sh_degree, rf_dtype attr_dtype, size_t* bytes)
{
    if (!bytes) return fail(RF_ERR_INVALID_ARG, "bytes is NULL");
    if (n_sites < 1 || n_edges < 0 || n_edges > INT32_MAX) return fail(RF_ERR_INVALID_ARG, "sizes out of range");
    if (n_sites > RF_MAX_SITES) return fail(RF_ERR_UNSUPPORTED, "n_sites > %lld", (long long)RF_MAX_SITES);
    if (sh_degree < 0 || sh_degree > RF_MAX_SH_DEGREE) return fail(RF_ERR_INVALID_ARG, "sh_degree out of range");
    if (attr_dtype != RF_F32 && attr_dtype != RF_BF16) return fail(RF_ERR_INVALID_ARG, "bad attr_dtype");
    *bytes = layout(n_sites, n_edges, sh_degree, attr_dtype == RF_BF16).total;
    return ok();
}

rf_status rf_pack_scene(const rf_scene* scene, rf_dtype attr_dtype, void* workspace, size_t workspace_bytes,
                        int validate, rf_packed_scene* out, void* stream)
{
    if (!scene || !out) return fail(RF_ERR_INVALID_ARG, "scene or out is NULL");
    size_t need = 0;
    rf_status st = rf_packed_bytes(scene->n_sites, scene->n_edges, scene->sh_degree, attr_dtype, &need);
    if (st != RF_OK) return st;
    if (!workspace || workspace_bytes < need)
        return fail(RF_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
    if (((uintptr_t)workspace & 255) != 0) return fail(RF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (scene->density_activation != RF_DENSITY_PLAIN && scene->density_activation != RF_DENSITY_SOFTPLUS)
        return fail(RF_ERR_INVALID_ARG, "density_activation must be RF_DENSITY_PLAIN or RF_DENSITY_SOFTPLUS");
    if (!scene->sites || !scene->nbr_off || !scene->density || !scene->sh || (scene->n_edges > 0 && !scene->nbr_idx))
        return fail(RF_ERR_INVALID_ARG, "a scene array is NULL");
    const bool bf16 = attr_dtype == RF_BF16;
    const Layout L = layout(scene->n_sites, scene->n_edges, scene->sh_degree, bf16);
    unsigned char* b = static_cast<unsigned char*>(workspace);
    rf::PackArgs a;
    a.density_act = scene->density_activation;
    a.sites = scene->sites;
    a.off = scene->nbr_off;
    a.idx = scene->nbr_idx;
    a.density = scene->density;
    a.sh = scene->sh;
    a.n_sites = scene->n_sites;
    a.n_edges = scene->n_edges;
    a.planes = reinterpret_cast<float4*>(b + L.planes);
    a.adj = reinterpret_cast<uint2*>(b + L.adj);
    a.row = reinterpret_cast<uint2*>(b + L.row);
    a.rec = b + L.rec;
    a.err = reinterpret_cast<int32_t*>(b + L.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = hip_status(rf::launch_pack(scene->sh_degree, bf16, a, s), "pack kernels");
    if (st != RF_OK) return st;
    out->base = workspace;
    out->bytes = workspace_bytes;
    out->n_sites = scene->n_sites;
    out->n_edges = scene->n_edges;
    out->sh_degree = scene->sh_degree;
    out->attr_dtype = attr_dtype;
    out->off_planes = L.planes;
    out->off_adj = L.adj;
    out->off_row = L.row;
    out->off_rec = L.rec;
    out->off_err = L.err;
    out->rec_bytes = L.rec_bytes;
    out->reserved = 0;
    if (validate) {
        int32_t errs[2];
        st = rf_packed_errors(out, errs, stream);
        if (st != RF_OK) return st;
        if (errs[1]) return fail(RF_ERR_UNSUPPORTED, "%d rows have more than %d neighbours", errs[1], RF_MAX_DEGREE);
        if (errs[0]) return fail(RF_ERR_INVALID_ARG, "CSR has %d invalid entries", errs[0]);
    }
    return ok();
}

rf_status rf_packed_errors(const rf_packed_scene* packed, int32_t errors[2], void* stream)
{
    rf_status st = check_packed(packed);
    if (st != RF_OK) return st;
    if (!errors) return fail(RF_ERR_INVALID_ARG, "errors is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned char* b = static_cast<const unsigned char*>(packed->base);
    hipError_t e = hipMemcpyAsync(errors, b + packed->off_err, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_status(e, "reading pack counters");
}

rf_status rf_raygen(const rf_camera* cam, const rf_bound* bound, int32_t start, float* origin, float* dir,
                    float* t_max, int32_t* start_cell, int32_t* pixel, void* stream)
{
    if (!cam || !bound) return fail(RF_ERR_INVALID_ARG, "camera or bound is NULL");
    if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > ((int64_t)1 << 31))
        return fail(RF_ERR_INVALID_ARG, "image size %d x %d out of range", cam->width, cam->height);
    if (cam->model != 0 && cam->model != 1) return fail(RF_ERR_INVALID_ARG, "camera model must be 0 or 1");
    if (!rf::camera_fov_ok(cam->model, cam->fov_deg))
        return fail(RF_ERR_INVALID_ARG, "fov must be in (0, 180) for a pinhole, (0, 360] for a fisheye");
    if (bound->kind != 0 && bound->kind != 1) return fail(RF_ERR_INVALID_ARG, "bound kind must be 0 or 1");
    if (!origin || !dir || !t_max || !start_cell) return fail(RF_ERR_INVALID_ARG, "an output array is NULL");
    rf::RaygenArgs a;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) a.rot[3 * r + c] = cam->pose[4 * r + c];
        a.pos[r] = cam->pose[4 * r + 3];
    }
    a.model = cam->model;
    a.focal = rf::camera_focal(cam->model, cam->fov_deg, cam->width);
    a.width = cam->width;
    a.height = cam->height;
    a.bound_kind = bound->kind;
    for (int k = 0; k < 6; ++k) a.bound[k] = bound->p[k];
    a.start = start;
    a.origin = origin;
    a.dir = dir;
    a.t_max = t_max;
    a.start_cell = start_cell;
    a.pixel = pixel;
    return hip_status(rf::launch_raygen(a, static_cast<hipStream_t>(stream)), "raygen kernel");
}

rf_status rf_render_forward(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params, float* rgb,
                            float* t_final, int32_t* steps, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (rays->n_rays > 0 && (!rgb || !t_final || !steps)) return fail(RF_ERR_INVALID_ARG, "an output array is NULL");
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb = rgb;
    a.t_final = t_final;
    a.steps = steps;
    return hip_status(rf::launch_walk(rf::kForward, scene->sh_degree, scene->attr_dtype == RF_BF16, a,
                                      static_cast<hipStream_t>(stream)),
                      "forward walk");
}

rf_status rf_render_trace(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params, int32_t max_len,
                          float* rgb, float* t_final, int32_t* steps, int32_t* cells, float* t_exit, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (max_len < 1) return fail(RF_ERR_INVALID_ARG, "max_len must be >= 1");
    if (rays->n_rays > 0 && (!rgb || !t_final || !steps || !cells || !t_exit))
        return fail(RF_ERR_INVALID_ARG, "an output array is NULL");
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb = rgb;
    a.t_final = t_final;
    a.steps = steps;
    a.max_len = max_len;
    a.cells = cells;
    a.t_exit = t_exit;
    return hip_status(rf::launch_walk(rf::kTrace, scene->sh_degree, scene->attr_dtype == RF_BF16, a,
                                      static_cast<hipStream_t>(stream)),
                      "traced walk");
}

rf_status rf_render_backward(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                             const float* rgb, const float* t_final, const int32_t* steps, const float* grad_rgb,
                             const float* grad_t_final, float* grad_sites, float* grad_density, float* grad_sh,
                             int32_t mode, int32_t* mismatches, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (mode != 0 && mode != 1) return fail(RF_ERR_INVALID_ARG, "mode must be 0 or 1");
    if (rays->n_rays > 0 && (!rgb || !t_final || !grad_rgb))
        return fail(RF_ERR_INVALID_ARG, "rgb, t_final and grad_rgb are required");
    if (!grad_sites || !grad_density || !grad_sh) return fail(RF_ERR_INVALID_ARG, "a gradient array is NULL");
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb_in = rgb;
    a.t_final_in = t_final;
    a.grad_rgb = grad_rgb;
    a.grad_t = grad_t_final;
    a.steps_in = steps;
    a.mismatch = mismatches;
    a.g_sites = grad_sites;
    a.g_density = grad_density;
    a.g_sh = grad_sh;
    return hip_status(rf::launch_walk(mode == 0 ? rf::kBackwardReduce : rf::kBackwardAtomic, scene->sh_degree,
                                      scene->attr_dtype == RF_BF16, a, static_cast<hipStream_t>(stream)),
                      "backward walk");
}

static rf_status check_log(const rf_walk_log* log, int64_t n_rays)
{
    if (!log) return fail(RF_ERR_INVALID_ARG, "log is NULL");
    if (log->capacity < 0) return fail(RF_ERR_INVALID_ARG, "log capacity must be >= 0");
    if (n_rays > 0 && !log->tail) return fail(RF_ERR_INVALID_ARG, "log tail is NULL");
    if (n_rays > 0 && log->capacity > 0 && (!log->code || !log->t_exit))
        return fail(RF_ERR_INVALID_ARG, "log code or t_exit is NULL");
    if ((reinterpret_cast<uintptr_t>(log->t_exit) & 7) || (reinterpret_cast<uintptr_t>(log->code) & 3) ||
        (reinterpret_cast<uintptr_t>(log->tail) & 15))
        return fail(RF_ERR_INVALID_ARG, "log arrays must be aligned to their element size (tail: 16 bytes)");
    return RF_OK;
}

static void set_log(rf::WalkArgs& a, const rf_walk_log* log)
{
    a.log_code = log->code;
    a.log_te = log->t_exit;
    a.log_tail = reinterpret_cast<int4*>(log->tail);
    a.log_cap = log->capacity;
}

rf_status rf_render_forward_logged(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                                   float* rgb, float* t_final, int32_t* steps, const rf_walk_log* log, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (rays->n_rays > 0 && (!rgb || !t_final || !steps)) return fail(RF_ERR_INVALID_ARG, "an output array is NULL");
    if ((st = check_log(log, rays->n_rays)) != RF_OK) return st;
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb = rgb;
    a.t_final = t_final;
    a.steps = steps;
    set_log(a, log);
    return hip_status(rf::launch_walk(rf::kForwardLog, scene->sh_degree, scene->attr_dtype == RF_BF16, a,
                                      static_cast<hipStream_t>(stream)),
                      "logged forward walk");
}

rf_status rf_render_backward_logged(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                                    const float* rgb, const float* t_final, const float* grad_rgb,
                                    const float* grad_t_final, const rf_walk_log* log, float* grad_sites,
                                    float* grad_density, float* grad_sh, int32_t mode, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (mode != 0 && mode != 1) return fail(RF_ERR_INVALID_ARG, "mode must be 0 or 1");
    if (rays->n_rays > 0 && (!rgb || !t_final || !grad_rgb))
        return fail(RF_ERR_INVALID_ARG, "rgb, t_final and grad_rgb are required");
    if (!grad_sites || !grad_density || !grad_sh) return fail(RF_ERR_INVALID_ARG, "a gradient array is NULL");
    if ((st = check_log(log, rays->n_rays)) != RF_OK) return st;
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb_in = rgb;
    a.t_final_in = t_final;
    a.grad_rgb = grad_rgb;
    a.grad_t = grad_t_final;
    a.g_sites = grad_sites;
    a.g_density = grad_density;
    a.g_sh = grad_sh;
    set_log(a, log);
    return hip_status(rf::launch_walk(mode == 0 ? rf::kBackwardLogReduce : rf::kBackwardLogAtomic, scene->sh_degree,
                                      scene->attr_dtype == RF_BF16, a, static_cast<hipStream_t>(stream)),
                      "logged backward walk");
}

static rf_status check_quantiles(const rf_quantiles* q, int64_t n_rays)
{
    if (!q) return fail(RF_ERR_INVALID_ARG, "quantiles is NULL");
    if (n_rays > 0 && (!q->draws || !q->t || !q->segment || !q->sigma))
        return fail(RF_ERR_INVALID_ARG, "a quantile array is NULL");
    return RF_OK;
}

static void set_quantiles(rf::WalkArgs& a, const rf_quantiles* q)
{
    a.q_u = q->draws;
    a.q_t = q->t;
    a.q_seg = q->segment;
    a.q_sig = q->sigma;
}

rf_status rf_quantile_forward(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                              const float* t_final, const rf_walk_log* log, const rf_quantiles* q, float* loss,
                              void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if ((st = check_log(log, rays->n_rays)) != RF_OK || (st = check_quantiles(q, rays->n_rays)) != RF_OK) return st;
    if (rays->n_rays > 0 && (!t_final || !loss)) return fail(RF_ERR_INVALID_ARG, "t_final or loss is NULL");
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.t_final_in = t_final;
    set_log(a, log);
    set_quantiles(a, q);
    a.q_loss = loss;
    return hip_status(rf::launch_walk(rf::kQuantile, scene->sh_degree, scene->attr_dtype == RF_BF16, a,
                                      static_cast<hipStream_t>(stream)),
                      "quantile forward");
}

rf_status rf_render_backward_quantile(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                                      const float* rgb, const float* t_final, const float* grad_rgb,
                                      const float* grad_t_final, const rf_walk_log* log, const rf_quantiles* q,
                                      const float* grad_loss, float* grad_sites, float* grad_density, float* grad_sh,
                                      int32_t mode, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if (mode != 0 && mode != 1) return fail(RF_ERR_INVALID_ARG, "mode must be 0 or 1");
    if (rays->n_rays > 0 && (!rgb || !t_final || !grad_rgb || !grad_loss))
        return fail(RF_ERR_INVALID_ARG, "rgb, t_final, grad_rgb and grad_loss are required");
    if (!grad_sites || !grad_density || !grad_sh) return fail(RF_ERR_INVALID_ARG, "a gradient array is NULL");
    if ((st = check_log(log, rays->n_rays)) != RF_OK || (st = check_quantiles(q, rays->n_rays)) != RF_OK) return st;
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb_in = rgb;
    a.t_final_in = t_final;
    a.grad_rgb = grad_rgb;
    a.grad_t = grad_t_final;
    a.g_sites = grad_sites;
    a.g_density = grad_density;
    a.g_sh = grad_sh;
    set_log(a, log);
    set_quantiles(a, q);
    a.grad_q = grad_loss;
    return hip_status(rf::launch_walk(mode == 0 ? rf::kBackwardLogReduce : rf::kBackwardLogAtomic, scene->sh_degree,
                                      scene->attr_dtype == RF_BF16, a, static_cast<hipStream_t>(stream)),
                      "backward walk with the quantile term");
}

static rf_status check_surface(const rf_surface* sf)
{
    if (!sf) return fail(RF_ERR_INVALID_ARG, "surface is NULL");
    if (sf->kind != RF_SURFACE_MIRROR && sf->kind != RF_SURFACE_GLASS)
        return fail(RF_ERR_INVALID_ARG, "surface kind must be RF_SURFACE_MIRROR or RF_SURFACE_GLASS");
    if (sf->max_bounces < 0 || sf->max_bounces > RF_MAX_BOUNCES)
        return fail(RF_ERR_INVALID_ARG, "max_bounces must be in [0, %d]", RF_MAX_BOUNCES);
    if (!(sf->radius > 0.0f) || !isfinite(sf->radius) || !isfinite(sf->centre[0]) ||
        !isfinite(sf->centre[1]) || !isfinite(sf->centre[2]))
        return fail(RF_ERR_INVALID_ARG, "the sphere needs a finite centre and a radius > 0");
    if (sf->kind == RF_SURFACE_GLASS && !(sf->ior > 0.0f && isfinite(sf->ior)))
        return fail(RF_ERR_INVALID_ARG, "glass needs a refractive index > 0");
    if (sf->bound.kind != 0 && sf->bound.kind != 1) return fail(RF_ERR_INVALID_ARG, "bound kind must be 0 or 1");
    return RF_OK;
}

static void set_surface(rf::WalkArgs& a, const rf_surface* sf)
{
    a.surf.kind = sf->kind;
    a.surf.max_bounces = sf->max_bounces;
    for (int k = 0; k < 3; ++k) a.surf.centre[k] = sf->centre[k];
    a.surf.radius = sf->radius;
    a.surf.ior = sf->ior;
    a.surf.bound_kind = sf->bound.kind;
    for (int k = 0; k < 6; ++k) a.surf.bound[k] = sf->bound.p[k];
}

rf_status rf_render_forward_surface(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                                    const rf_surface* surface, float* rgb, float* t_final, int32_t* steps,
                                    const rf_walk_log* log, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if ((st = check_surface(surface)) != RF_OK) return st;
    if (rays->n_rays > 0 && (!rgb || !t_final || !steps)) return fail(RF_ERR_INVALID_ARG, "an output array is NULL");
    if (log && (st = check_log(log, rays->n_rays)) != RF_OK) return st;
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb = rgb;
    a.t_final = t_final;
    a.steps = steps;
    set_surface(a, surface);
    if (log) set_log(a, log);
    return hip_status(rf::launch_walk(log ? rf::kForwardLogSurf : rf::kForwardSurf, scene->sh_degree,
                                      scene->attr_dtype == RF_BF16, a, static_cast<hipStream_t>(stream)),
                      "forward walk with a surface");
}

rf_status rf_render_backward_surface(const rf_packed_scene* scene, const rf_rays* rays, const rf_params* params,
                                     const rf_surface* surface, const float* rgb, const float* t_final,
                                     const float* grad_rgb, const float* grad_t_final, const rf_walk_log* log,
                                     float* grad_sites, float* grad_density, float* grad_sh, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK || (st = check_rays(rays)) != RF_OK || (st = check_params(params)) != RF_OK)
        return st;
    if ((st = check_surface(surface)) != RF_OK) return st;
    if (rays->n_rays > 0 && (!rgb || !t_final || !grad_rgb))
        return fail(RF_ERR_INVALID_ARG, "rgb, t_final and grad_rgb are required");
    if (!grad_sites || !grad_density || !grad_sh) return fail(RF_ERR_INVALID_ARG, "a gradient array is NULL");
    if (log && (st = check_log(log, rays->n_rays)) != RF_OK) return st;
    rf::WalkArgs a = walk_args(scene, rays, params);
    a.rgb_in = rgb;
    a.t_final_in = t_final;
    a.grad_rgb = grad_rgb;
    a.grad_t = grad_t_final;
    a.g_sites = grad_sites;
    a.g_density = grad_density;
    a.g_sh = grad_sh;
    set_surface(a, surface);
    if (log) set_log(a, log);
    return hip_status(rf::launch_walk(log ? rf::kBackwardLogSurf : rf::kBackwardSurf, scene->sh_degree,
                                      scene->attr_dtype == RF_BF16, a, static_cast<hipStream_t>(stream)),
                      "backward walk with a surface");
}

rf_status rf_locate(const rf_packed_scene* scene, const float* points, int64_t n_points, const int32_t* seed,
                    int32_t max_steps, int32_t* cells, void* stream)
{
    rf_status st;
    if ((st = check_packed(scene)) != RF_OK) return st;
    if (n_points < 0 || n_points > ((int64_t)1 << 37))
        return fail(RF_ERR_INVALID_ARG, "n_points = %lld out of range", (long long)n_points);
    if (n_points > 0 && (!points || !cells)) return fail(RF_ERR_INVALID_ARG, "points or cells is NULL");
    if (max_steps < 1) return fail(RF_ERR_INVALID_ARG, "max_steps must be >= 1");
    rf::LocateArgs a;
    memset(&a, 0, sizeof a);
    a.s = view(scene);
    a.points = points;
    a.seed = seed;
    a.n_points = n_points;
    a.max_steps = max_steps;
    a.cells = cells;
    return hip_status(rf::launch_locate(scene->sh_degree, scene->attr_dtype == RF_BF16, a,
                                        static_cast<hipStream_t>(stream)),
                      "locate");
}

rf_status rf_train_schedule(int32_t iteration, int32_t total, rf_adam_args* out)
{
    if (!out) return fail(RF_ERR_INVALID_ARG, "out is NULL");
    if (total < 1 || iteration < 0 || iteration >= total)
        return fail(RF_ERR_INVALID_ARG, "iteration %d outside [0, %d)", iteration, total);
    static const double lr0[4] = {2e-4, 1e-1, 5e-3, 5e-3}, lr1[4] = {2e-6, 1e-2, 5e-4, 5e-4};
    const int32_t warm = total / 4, freeze = total - total / 10;
    const double w = (1.0 + cos(M_PI * (double)iteration / (double)total)) / 2.0;
    for (int g = 0; g < 4; ++g) out->lr[g] = (float)(lr1[g] + (lr0[g] - lr1[g]) * w);
    out->t[0] = iteration + 1 < freeze ? iteration + 1 : freeze;
    out->t[1] = iteration + 1;
    out->t[2] = iteration + 1;
    out->t[3] = iteration + 1 - warm > 0 ? iteration + 1 - warm : 0;
    if (iteration >= freeze) out->lr[0] = 0.0f;
    if (iteration < warm) out->lr[3] = 0.0f;
    out->beta1 = 0.9f;
    out->beta2 = 0.999f;
    out->eps = 1e-15f;
    out->softplus_density = 1;
    return ok();
}

rf_status rf_adam_step(int64_t n_sites, int32_t sh_degree, const rf_adam_args* args, float* sites, float* density,
                       float* sh, const float* grad_sites, const float* grad_density, const float* grad_sh,
                       const rf_adam_state* state, void* stream)
{
    if (!args || !state) return fail(RF_ERR_INVALID_ARG, "args or state is NULL");
    if (n_sites < 0 || sh_degree < 0 || sh_degree > 3) return fail(RF_ERR_INVALID_ARG, "bad n_sites or sh_degree");
    if (n_sites == 0) return ok();
    if (!sites || !density || !sh || !grad_sites || !grad_density || !grad_sh || !state->m_sites ||
        !state->v_sites || !state->m_density || !state->v_density || !state->m_sh || !state->v_sh)
        return fail(RF_ERR_INVALID_ARG, "a parameter, gradient or moment array is NULL");
    if (!(args->beta1 >= 0.0f && args->beta1 < 1.0f && args->beta2 >= 0.0f && args->beta2 < 1.0f &&
          args->eps >= 0.0f))
        return fail(RF_ERR_INVALID_ARG, "betas must be in [0, 1) and eps >= 0");
    for (int g = 0; g < 4; ++g)
        if (!(args->lr[g] >= 0.0f) || (args->lr[g] > 0.0f && args->t[g] < 1))
            return fail(RF_ERR_INVALID_ARG, "group %d: lr must be >= 0, with a step count >= 1 when it moves", g);
    const int B = (sh_degree + 1) * (sh_degree + 1);
    auto corr = [](float beta, int32_t t) { return t > 0 ? (float)(1.0 / (1.0 - pow((double)beta, t))) : 1.0f; };
    rf::AdamGroup g[3];
    for (int q = 0; q < 3; ++q) {
        g[q].beta1 = args->beta1;
        g[q].beta2 = args->beta2;
        g[q].eps = args->eps;
        g[q].B = B;
    }
    // positions
    g[0].x = sites; g[0].g = grad_sites; g[0].m = state->m_sites; g[0].v = state->v_sites; g[0].n = 3 * n_sites;
    g[0].kind = 0;
    // density
    g[1].x = density; g[1].g = grad_density; g[1].m = state->m_density; g[1].v = state->v_density;
    g[1].n = n_sites;
    g[1].kind = args->softplus_density ? 1 : 0;
    for (int q = 0; q < 2; ++q)
        for (int s2 = 0; s2 < 2; ++s2) {
            g[q].lr[s2] = args->lr[q];
            g[q].c1[s2] = corr(args->beta1, args->t[q]);
            g[q].c2[s2] = corr(args->beta2, args->t[q]);
        }
    // SH: order 0 and the higher orders
    g[2].x = sh; g[2].g = grad_sh; g[2].m = state->m_sh; g[2].v = state->v_sh; g[2].n = 3 * (int64_t)B * n_sites;
    g[2].kind = 2;
    for (int s2 = 0; s2 < 2; ++s2) {
        g[2].lr[s2] = args->lr[2 + s2];
        g[2].c1[s2] = corr(args->beta1, args->t[2 + s2]);
        g[2].c2[s2] = corr(args->beta2, args->t[2 + s2]);
    }
    const hipError_t e = rf::launch_adam(g, static_cast<hipStream_t>(stream));
    return hip_status(e, "adam step");
}

rf_status rf_densify_scores(const float* sites, const int32_t* nbr_off, const int32_t* nbr_idx, int64_t n_sites,
                            const float* grad_sites, float* scores, void* stream)
{
    if (n_sites < 0) return fail(RF_ERR_INVALID_ARG, "n_sites < 0");
    if (n_sites > 0 && (!sites || !nbr_off || !nbr_idx || !grad_sites || !scores))
        return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    return hip_status(rf::launch_densify_score(sites, nbr_off, nbr_idx, n_sites, grad_sites, scores,
                                               static_cast<hipStream_t>(stream)),
                      "densification scores");
}

rf_status rf_sample_workspace(int64_t n, size_t* bytes)
{
    if (n < 0 || !bytes) return fail(RF_ERR_INVALID_ARG, "n < 0 or bytes is NULL");
    *bytes = (size_t)rf::sample_workspace_doubles(n) * sizeof(double);
    return ok();
}

rf_status rf_sample_cells(const float* scores, int64_t n, const float* draws, int64_t n_draws, int32_t* cells,
                          void* workspace, size_t workspace_bytes, void* stream)
{
    if (n < 1 || n > INT32_MAX || n_draws < 0) return fail(RF_ERR_INVALID_ARG, "need 1 <= n <= 2^31 - 1, n_draws >= 0");
    if (n_draws == 0) return ok();
    if (!scores || !draws || !cells || !workspace) return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    if (workspace_bytes < (size_t)rf::sample_workspace_doubles(n) * sizeof(double) ||
        (reinterpret_cast<uintptr_t>(workspace) & 7))
        return fail(RF_ERR_INVALID_ARG, "workspace too small (see rf_sample_workspace) or not 8-byte aligned");
    return hip_status(rf::launch_sample(scores, n, draws, n_draws, cells, static_cast<double*>(workspace),
                                        static_cast<hipStream_t>(stream)),
                      "candidate sampling");
}

rf_status rf_insert_sites(const float* sites, const int32_t* nbr_off, const int32_t* nbr_idx, int64_t n_sites,
                          const int32_t* parents, const float* offsets, int64_t n_new, float frac, float* new_sites,
                          void* stream)
{
    if (n_sites < 1 || n_new < 0) return fail(RF_ERR_INVALID_ARG, "need n_sites >= 1, n_new >= 0");
    if (!(frac >= 0.0f && frac < 1.0f)) return fail(RF_ERR_INVALID_ARG, "frac must lie in [0, 1)");
    if (n_new == 0) return ok();
    if (!sites || !nbr_off || !nbr_idx || !parents || !offsets || !new_sites)
        return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    return hip_status(rf::launch_insert_sites(sites, nbr_off, nbr_idx, n_sites, parents, offsets, n_new, frac,
                                              new_sites, static_cast<hipStream_t>(stream)),
                      "site insertion");
}

rf_status rf_gather_rows(const float* in, int64_t n_rows_in, int32_t width, const int32_t* rows, int64_t n_rows_out,
                         float* out, void* stream)
{
    if (n_rows_in < 0 || n_rows_out < 0 || width < 1) return fail(RF_ERR_INVALID_ARG, "bad sizes");
    if (n_rows_out == 0) return ok();
    if (!in || !rows || !out) return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    return hip_status(rf::launch_gather_rows(in, n_rows_in, width, rows, n_rows_out, out,
                                             static_cast<hipStream_t>(stream)),
                      "row gather");
}

rf_status rf_keep_workspace(int64_t n, size_t* bytes)
{
    if (n < 0 || !bytes) return fail(RF_ERR_INVALID_ARG, "n < 0 or bytes is NULL");
    *bytes = (size_t)rf::keep_workspace_count(n) * sizeof(int64_t);
    return ok();
}

rf_status rf_keep_index(const uint8_t* keep, int64_t n, int32_t* kept, int64_t* n_kept, void* workspace,
                        size_t workspace_bytes, void* stream)
{
    if (n < 0 || n > INT32_MAX) return fail(RF_ERR_INVALID_ARG, "need 0 <= n <= 2^31 - 1");
    if (!n_kept) return fail(RF_ERR_INVALID_ARG, "n_kept is NULL");
    if (n > 0 && (!keep || !kept || !workspace)) return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    if (workspace_bytes < (size_t)rf::keep_workspace_count(n) * sizeof(int64_t) ||
        (reinterpret_cast<uintptr_t>(workspace) & 7) || (reinterpret_cast<uintptr_t>(n_kept) & 7))
        return fail(RF_ERR_INVALID_ARG, "workspace too small (see rf_keep_workspace) or not 8-byte aligned");
    return hip_status(rf::launch_keep_index(keep, n, kept, n_kept, static_cast<int64_t*>(workspace),
                                            static_cast<hipStream_t>(stream)),
                      "keep index");
}

rf_status rf_sample_cells_noalloc(const float* scores, int64_t n, const float* draws, int64_t n_draws,
                                  int32_t* cells, void* stream)
{
    if (n < 1 || n_draws < 0) return fail(RF_ERR_INVALID_ARG, "need n >= 1, n_draws >= 0");
    if (n > rf::sample_noalloc_max_cells())
        return fail(RF_ERR_UNSUPPORTED, "n = %lld exceeds the allocation-free sampler's limit of %lld cells",
                    (long long)n, (long long)rf::sample_noalloc_max_cells());
    if (n_draws == 0) return ok();
    if (!scores || !draws || !cells) return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    double* ws = nullptr;
    const hipError_t e = rf::sample_scratch(&ws);
    if (e != hipSuccess) return hip_status(e, "scratch address of the allocation-free sampler");
    return hip_status(rf::launch_sample(scores, n, draws, n_draws, cells, ws, static_cast<hipStream_t>(stream)),
                      "candidate sampling (allocation-free)");
}

rf_status rf_prune_mask(const float* density, const int32_t* nbr_off, const int32_t* nbr_idx, int64_t n_sites,
                        float threshold, uint8_t* mask, void* stream)
{
    if (n_sites < 0) return fail(RF_ERR_INVALID_ARG, "n_sites < 0");
    if (n_sites > 0 && (!density || !nbr_off || !nbr_idx || !mask)) return fail(RF_ERR_INVALID_ARG, "an array is NULL");
    return hip_status(rf::launch_prune_mask(density, nbr_off, nbr_idx, n_sites, threshold, mask,
                                            static_cast<hipStream_t>(stream)),
                      "pruning mask");
}

rf_status rf_packed_planes(const rf_packed_scene* scene, float* planes, void* stream)
{
    rf_status st = check_packed(scene);
    if (st != RF_OK) return st;
    if (!planes && scene->n_edges > 0) return fail(RF_ERR_INVALID_ARG, "planes is NULL");
    return hip_status(rf::launch_unpack(scene->sh_degree, scene->attr_dtype == RF_BF16, view(scene), planes, nullptr,
                                        nullptr, static_cast<hipStream_t>(stream)),
                      "plane read-back");
}

rf_status rf_packed_attributes(const rf_packed_scene* scene, float* density, float* sh, void* stream)
{
    rf_status st = check_packed(scene);
    if (st != RF_OK) return st;
    if (!density || !sh) return fail(RF_ERR_INVALID_ARG, "density or sh is NULL");
    return hip_status(rf::launch_unpack(scene->sh_degree, scene->attr_dtype == RF_BF16, view(scene), nullptr, density,
                                        sh, static_cast<hipStream_t>(stream)),
                      "attribute read-back");
}

}  // extern "C"
