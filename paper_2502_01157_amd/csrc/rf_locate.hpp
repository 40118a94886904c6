// Location of the cell containing a point (its nearest site, eq. (5)), the
// start cell of a ray in Algorithm 1: a greedy walk over the Delaunay graph,
// first in FP32 across the packed bisector planes, then with squared distances
// to the sites in double (see locate.hip). Shared by the location kernel and
// the persistent render server.
#pragma once

#include "rf_device.hpp"
#include "rf_kernels.hpp"

namespace rf {

__device__ inline double dist2(const float* x, double px, double py, double pz)
{
    const double dx = px - (double)x[0], dy = py - (double)x[1], dz = pz - (double)x[2];
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// The located cell of the seed grid's cell containing the point (clamped to the grid).
__device__ inline int grid_seed(const int32_t* grid, int grid_n, const float* grid_lo, const float* grid_inv, float px,
                                float py, float pz)
{
    int ix[3];
    const float pp[3] = {px, py, pz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // clamped in float, so that NaN and far-away points convert safely
        const float f = (pp[k] - grid_lo[k]) * grid_inv[k];
        ix[k] = f >= (float)(grid_n - 1) ? grid_n - 1 : (f >= 1.0f ? (int)f : 0);
    }
    return grid[((int64_t)ix[2] * grid_n + ix[1]) * grid_n + ix[0]];
}

// The nearest site of (px, py, pz) walking from `seed`: -1 for a seed out of
// range, -2 if max_steps steps were not enough.
template <int DEG, bool BF16>
__device__ inline int locate_point(const SceneView& s, float px, float py, float pz, int seed, int max_steps)
{
    if (seed < 0 || (int64_t)seed >= s.n_sites) return -1;
    uint2 ref = s.row[seed];
    int steps = 0;
    // phase 1: FP32 steps across bisector planes
    for (; steps < max_steps; ++steps) {
        const int beg = ref_beg(ref), deg = ref_deg(ref);
        float best = 0.0f;
        int bk = -1;
        for (int k = 0; k < deg; ++k) {
            const float4 pl = s.planes[beg + k];
            const float gain = fmaf(pl.z, pz, fmaf(pl.y, py, pl.x * px)) - pl.w;
            if (gain > best) {
                best = gain;
                bk = k;
            }
        }
        if (bk < 0) break;
        ref = s.adj[beg + bk];
    }
    // phase 2: FP64 squared distances to the sites
    int cur = ref_cell(ref);
    float xc[3];
    load_site<DEG, BF16>(s.rec, cur, xc);
    double dcur = dist2(xc, px, py, pz);
    for (; steps < max_steps; ++steps) {
        const int beg = ref_beg(ref), deg = ref_deg(ref);
        int bj = cur;
        double bd = dcur;
        uint2 bref = ref;
        for (int k = 0; k < deg; ++k) {
            const uint2 nb = s.adj[beg + k];
            const int j = ref_cell(nb);
            float xj[3];
            load_site<DEG, BF16>(s.rec, j, xj);
            const double dj = dist2(xj, px, py, pz);
            if (dj < bd || (dj == bd && j < bj)) {
                bd = dj;
                bj = j;
                bref = nb;
            }
        }
        if (bj == cur) break;
        cur = bj;
        dcur = bd;
        ref = bref;
    }
    return steps < max_steps ? cur : -2;
}

}  // namespace rf
