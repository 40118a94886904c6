// Start-cell location: the cell containing each point (its nearest site,
// eq. (5)), which Algorithm 1 needs as the cell of the ray origin.
//
// Greedy walk over the Delaunay graph: from a seed cell, move to the
// neighbour nearest the point while some neighbour is nearer. A site that is
// not the point's nearest always has a nearer Delaunay neighbour (the segment
// from the site to the point leaves its Voronoi cell through a face shared
// with a neighbour j, and the exit point is as far from x_j as from x_i), so
// the walk ends at the nearest site.
//
// Phase 1 steps in FP32 across the packed bisector planes: neighbour j is
// nearer than cell i exactly when n.p > c (n = x_j - x_i, c = n.(x_i+x_j)/2),
// and |p - x_j|^2 = |p - x_i|^2 - 2 (n.p - c), so the largest n.p - c > 0 is
// the nearest neighbour. The planes of (i, j) and (j, i) are exact negations
// and the dot product is formed the same way, so two cells never both look
// nearer than each other. Phase 2 finishes with squared distances to the
// sites in double, moving while a neighbour is strictly nearer (or equally
// near with a lower index), which settles what FP32 could not resolve.
//
// A walk starts from the caller's seed cell, else from the cell of a coarse
// seed grid (the located nearest sites of a regular grid of points) that
// contains the point, else from cell 0. One point per lane; each step reads
// one row of planes (phase 1) or of neighbour ids and sites (phase 2).

#include "rf_device.hpp"
#include "rf_kernels.hpp"
#include "rf_locate.hpp"

namespace rf {

template <int DEG, bool BF16>
__global__ __launch_bounds__(kBlock) void k_locate(LocateArgs a)
{
    const int64_t q = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (q >= a.n_points) return;
    const float px = a.points[3 * q], py = a.points[3 * q + 1], pz = a.points[3 * q + 2];
    int seed = 0;
    if (a.seed)
        seed = a.seed[q];
    else if (a.grid)
        seed = grid_seed(a.grid, a.grid_n, a.grid_lo, a.grid_inv, px, py, pz);
    a.cells[q] = locate_point<DEG, BF16>(a.s, px, py, pz, seed, a.max_steps);
}

template <int DEG, bool BF16>
static hipError_t launch_locate_t(const LocateArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.n_points + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_locate<DEG, BF16>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_locate(int sh_degree, bool bf16, const LocateArgs& a, hipStream_t stream)
{
    switch (sh_degree * 2 + (bf16 ? 1 : 0)) {
    case 0: return launch_locate_t<0, false>(a, stream);
    case 1: return launch_locate_t<0, true>(a, stream);
    case 2: return launch_locate_t<1, false>(a, stream);
    case 3: return launch_locate_t<1, true>(a, stream);
    case 4: return launch_locate_t<2, false>(a, stream);
    case 5: return launch_locate_t<2, true>(a, stream);
    case 6: return launch_locate_t<3, false>(a, stream);
    case 7: return launch_locate_t<3, true>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace rf
