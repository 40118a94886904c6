// Launch interface between the C ABI (api.hip) and the kernels (walk.hip, pack.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rf {

struct SceneView {
    const float4* planes;
    const uint2* adj;
    const uint2* row;
    const unsigned char* rec;
    int64_t n_sites;
    int64_t n_edges;
};

// An analytic sphere that bends rays (secondary rays): kind 1 mirror,
// 2 glass of refractive index `ior` inside (1 outside); legs after a
// crossing end at the bound (kind 0 box lo = b[0..2], hi = b[3..5]; kind 1
// sphere of radius b[0] about the world origin).
struct SurfaceArgs {
    int32_t kind;
    int32_t max_bounces;
    float centre[3];
    float radius;
    float ior;
    int32_t bound_kind;
    float bound[6];
};

struct WalkArgs {
    SceneView s;
    const float* origin;
    const float* dir;
    const float* t_max;
    const int32_t* start;
    int64_t n_rays;
    float eps;
    int32_t max_steps;
    // forward outputs
    float* rgb;
    float* t_final;
    int32_t* steps;
    // trace outputs
    int32_t max_len;
    int32_t* cells;
    float* t_exit;
    // backward inputs / outputs
    const float* rgb_in;
    const float* t_final_in;
    const float* grad_rgb;
    const float* grad_t;
    const int32_t* steps_in;  // the forward's steps (nullable), checked against the recomputed walk
    int32_t* mismatch;        // counts rays whose recomputed walk disagrees with the saved outputs (nullable)
    float* g_sites;
    float* g_density;
    float* g_sh;
    // walk log: written by a logged forward, read by a logged backward
    uint32_t* log_code;  // [log_cap][n_rays] cell | moves << 31 | clipped << 30 | crossing << 29
    double* log_te;      // [log_cap][n_rays] clamped exit distance of the visit (along its leg)
    int4* log_tail;      // [n_rays] (row of the cell after the logged visits, visited cells, crossings)
    int32_t log_cap;
    // quantile regulariser: two draws per ray in, quantiles and their visit out
    const float* q_u;    // [n_rays][2]
    float* q_t;          // [n_rays][2] W^-1(u)
    int32_t* q_seg;      // [n_rays][2] visit index holding it, -1 none
    float* q_sig;        // [n_rays][2] that visit's density
    float* q_loss;       // [n_rays]
    const float* grad_q; // [n_rays] upstream gradient of the loss (backward)
    // secondary rays (the kinds with a surface)
    SurfaceArgs surf;
};

struct PackArgs {
    const float* sites;
    const int32_t* off;
    const int32_t* idx;
    const float* density;
    int32_t density_act;  // 1: density holds x, sigma = softplus_10(x)
    const float* sh;
    int64_t n_sites;
    int64_t n_edges;
    float4* planes;
    uint2* adj;
    uint2* row;
    unsigned char* rec;
    int32_t* err;
};

struct RaygenArgs {
    float rot[9];
    float pos[3];
    int32_t model;  // 0 pinhole, 1 equidistant fisheye
    float focal;    // pinhole: focal length in pixels; fisheye: radians per pixel
    int32_t width, height;
    int32_t bound_kind;
    float bound[6];
    int32_t start;
    float* origin;
    float* dir;
    float* t_max;
    int32_t* start_cell;
    int32_t* pixel;
};

struct LocateArgs {
    SceneView s;
    const float* points;  // [n_points][3]
    const int32_t* seed;  // [n_points], or null: the seed grid's cell, or cell 0 without a grid
    int64_t n_points;
    int32_t max_steps;
    int32_t* cells;       // [n_points] nearest site, -1 bad seed, -2 max_steps reached
    // optional seed grid: grid_n^3 located cells of a regular grid over
    // [grid_lo, grid_lo + grid_n / grid_inv), x fastest
    const int32_t* grid;
    int32_t grid_n;
    float grid_lo[3];
    float grid_inv[3];
};

enum WalkKind {
    kForward = 0,
    kTrace = 1,
    kBackwardReduce = 2,
    kBackwardAtomic = 3,
    kForwardLog = 4,
    kBackwardLogReduce = 5,
    kBackwardLogAtomic = 6,
    kQuantile = 7,
    // with a surface (secondary rays); the backward always reduces per wavefront
    kForwardSurf = 8,
    kForwardLogSurf = 9,
    kBackwardSurf = 10,
    kBackwardLogSurf = 11
};

// Camera models (host side): the field of view each accepts, and the focal
// value the camera ray takes (pinhole: focal length in pixels; fisheye:
// radians per pixel, so that the left and right edges are at fov/2).
inline bool camera_fov_ok(int model, float fov_deg)
{
    return model == 0 ? (fov_deg > 0.0f && fov_deg < 180.0f) : (model == 1 && fov_deg > 0.0f && fov_deg <= 360.0f);
}

inline float camera_focal(int model, float fov_deg, int width)
{
    const double half = 0.5 * (double)fov_deg * 3.14159265358979323846 / 180.0;
    return model == 1 ? (float)(half / (0.5 * width)) : (float)(0.5 * width / tan(half));
}

// Records an error message for rf_last_error() on this host thread.
void set_error(const char* msg);

hipError_t launch_walk(WalkKind kind, int sh_degree, bool bf16, const WalkArgs& a, hipStream_t stream);
hipError_t launch_pack(int sh_degree, bool bf16, const PackArgs& a, hipStream_t stream);
hipError_t launch_raygen(const RaygenArgs& a, hipStream_t stream);
hipError_t launch_locate(int sh_degree, bool bf16, const LocateArgs& a, hipStream_t stream);

// Training-step kernels (train.hip).
// One parameter group of an Adam step over n floats: lr == 0 holds a value
// (neither it nor its moments change); c1, c2 are the bias corrections
// 1 / (1 - beta^t) of the group's step count t.
struct AdamGroup {
    float* x;
    const float* g;
    float* m;
    float* v;
    int64_t n;
    // SH values with basis index b > 0 use the second set
    float lr[2], c1[2], c2[2];
    int32_t kind;  // 0 plain, 1 density under softplus (chain the gradient), 2 SH with B basis functions
    int32_t B;
    float beta1, beta2, eps;
};
hipError_t launch_adam(const AdamGroup groups[3], hipStream_t stream);  // positions, density, SH
hipError_t launch_densify_score(const float* sites, const int32_t* off, const int32_t* idx, int64_t n,
                                const float* grad_sites, float* score, hipStream_t stream);
hipError_t launch_prune_mask(const float* density, const int32_t* off, const int32_t* idx, int64_t n,
                             float threshold, uint8_t* mask, hipStream_t stream);
hipError_t launch_insert_sites(const float* sites, const int32_t* off, const int32_t* idx, int64_t n_sites,
                               const int32_t* parents, const float* u, int64_t n_new, float frac, float* out,
                               hipStream_t stream);
hipError_t launch_gather_rows(const float* in, int64_t n_in, int width, const int32_t* rows, int64_t n_out,
                              float* out, hipStream_t stream);
int64_t keep_workspace_count(int64_t n);  // int64 values of the keep-index workspace
hipError_t launch_keep_index(const uint8_t* keep, int64_t n, int32_t* kept, int64_t* n_kept, int64_t* workspace,
                             hipStream_t stream);
int64_t sample_workspace_doubles(int64_t n);
int64_t sample_noalloc_max_cells();
// the per-device address of the allocation-free sampler's scratch (current device)
hipError_t sample_scratch(double** out);
hipError_t launch_sample(const float* score, int64_t n, const float* draws, int64_t n_draws, int32_t* out,
                         double* workspace, hipStream_t stream);
hipError_t launch_unpack(int sh_degree, bool bf16, const SceneView& s, float* planes_out, float* density_out,
                         float* sh_out, hipStream_t stream);

}  // namespace rf
