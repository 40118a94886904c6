// Scene packing (face planes, neighbour rows, per-cell records) and camera
// ray generation for gfx950.

#include <limits.h>

#include "rf_device.hpp"
#include "rf_kernels.hpp"
#include "rf_walk.hpp"

namespace rf {

// Row range [beg, beg + deg) of cell i from the CSR, clamped so that a corrupt
// CSR can never send a later read outside [0, E). Returns false if the row was
// invalid (out of range or longer than 255 neighbours); the row is then empty.
__device__ inline bool checked_row(const int32_t* __restrict__ off, int64_t i, int64_t E, int* beg, int* deg,
                                   bool* too_long)
{
    const int64_t b = off[i], e = off[i + 1];
    *too_long = false;
    if (b < 0 || e < b || e > E) {
        *beg = (int)(b < 0 ? 0 : (b > E ? E : b));
        *deg = 0;
        return false;
    }
    if (e - b > 255) {
        *beg = (int)b;
        *deg = 0;
        *too_long = true;
        return false;
    }
    *beg = (int)b;
    *deg = (int)(e - b);
    return true;
}

__global__ void k_zero_err(int32_t* err)
{
    if (threadIdx.x < 2) err[threadIdx.x] = 0;
}

// One thread per cell: its row reference and the CSR checks.
__global__ __launch_bounds__(256) void k_pack_rows(PackArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_sites) return;
    int beg, deg;
    bool too_long;
    const bool ok = checked_row(a.off, i, a.n_edges, &beg, &deg, &too_long);
    if (!ok) atomicAdd(&a.err[too_long ? 1 : 0], 1);
    if (i == 0 && a.off[0] != 0) atomicAdd(&a.err[0], 1);
    if (i == a.n_sites - 1 && a.off[a.n_sites] != a.n_edges) atomicAdd(&a.err[0], 1);
    a.row[i] = make_uint2((uint32_t)i | ((uint32_t)deg << 24), (uint32_t)beg);
}

// One thread per 16-byte chunk of a cell record, so that consecutive threads
// write consecutive chunks and read consecutive SH values.
// Density activation (Sec. 3.4, implementation details): softplus with
// beta = 10, ln(1 + e^{10 x}) / 10, which is x itself to FP32 precision once
// 10 x > 20. Evaluated in double: in FP32 the rounding of 10 x alone would
// put a relative error of |10 x| eps32 on e^{10 x}.
__device__ inline float softplus10(float x)
{
    const double z = 10.0 * (double)x;
    return z > 20.0 ? x : (float)(log1p(exp(z)) / 10.0);
}

template <int DEG, bool BF16>
__global__ __launch_bounds__(256) void k_pack_records(PackArgs a)
{
    using R = Rec<DEG, BF16>;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / R::CHUNKS;
    const int c = (int)(t - i * R::CHUNKS);
    if (i >= a.n_sites) return;
    const float* sh = a.sh + i * R::NSH;
    const float sigma = a.density_act ? softplus10(a.density[i]) : a.density[i];
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // byte offset of word q of this chunk inside the record
        const int byte = 16 * c + 4 * q;
        uint32_t v = 0u;
        if (byte >= R::SITE_OFF && byte < R::SITE_OFF + 12) {
            v = __float_as_uint(a.sites[3 * i + (byte - R::SITE_OFF) / 4]);
        } else if constexpr (BF16) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = byte / 2 + h;  // bf16 element index
                if (k < R::NSH) v |= f32_to_bf16_rne(sh[k]) << (16 * h);
                else if (k == R::NSH) v |= f32_to_bf16_rne(sigma) << (16 * h);
            }
        } else {
            const int k = byte / 4;
            if (k < R::NSH) v = __float_as_uint(sh[k]);
            else if (k == R::NSH) v = __float_as_uint(sigma);
        }
        w[q] = v;
    }
    reinterpret_cast<uint4*>(a.rec + i * R::BYTES)[c] = make_uint4(w[0], w[1], w[2], w[3]);
}

// One wavefront per 64 consecutive cells; its lanes stride over the cells'
// directed edges (contiguous in the CSR), so idx reads and plane/adj writes
// are coalesced. Each lane finds its edge's owner among the 64 row offsets
// by binary search over the wave's registers.
// n = x_j - x_i and c = n . ((x_i + x_j) / 2) are evaluated with the same
// instruction sequence for (i, j) and (j, i), so the two planes of a face are
// exact negations of each other.
__global__ __launch_bounds__(256) void k_pack_faces(PackArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave;
    if (c0 >= a.n_sites) return;
    const int64_t mine = c0 + lane;
    int beg = 0, deg = 0;
    bool too_long = false;
    if (mine < a.n_sites) checked_row(a.off, mine, a.n_edges, &beg, &deg, &too_long);
    // the wave's edge range: from the first valid row start to the last valid row end
    const int end = beg + deg;
    int lo_e = mine < a.n_sites ? beg : INT_MAX, hi_e = mine < a.n_sites ? end : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        lo_e = min(lo_e, __shfl_xor(lo_e, m));
        hi_e = max(hi_e, __shfl_xor(hi_e, m));
    }
    // row starts for the owner search: lanes past the last cell sort last
    const int key = mine < a.n_sites ? beg : INT_MAX;
    for (int64_t base = lo_e; base < hi_e; base += kWave) {
        const int64_t k = base + lane;
        // owner: the lane q whose row [beg_q, beg_q + deg_q) contains k. In a
        // valid CSR the row starts rise with q, so it is the last q with
        // beg_q <= k (binary search over the wavefront's registers); where
        // that row does not contain k (a corrupted CSR), a scan of all 64 rows
        // keeps every edge of every row owned, as the walk needs.
        int q = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1) {
            const int cand = q + step;
            if (__shfl(key, cand) <= k) q = cand;
        }
        const int bq = __shfl(beg, q), dq = __shfl(deg, q);
        int owner = (k >= bq && k < bq + dq) ? q : -1;
        if (ballot(k < hi_e && owner < 0)) {
            // (wavefront-uniform, so every lane takes part in the shuffles)
            int scan = -1;
            for (int r = 0; r < kWave; ++r) {
                const int br = __shfl(beg, r), dr = __shfl(deg, r);
                if (k >= br && k < br + dr) scan = r;
            }
            if (owner < 0) owner = scan;
        }
        if (k >= hi_e || owner < 0) continue;
        const int64_t i = c0 + owner;
        const float xi = a.sites[3 * i], yi = a.sites[3 * i + 1], zi = a.sites[3 * i + 2];
        const int64_t j = a.idx[k];
        int jb = 0, jd = 0;
        bool jl;
        const bool valid = j >= 0 && j < a.n_sites && j != i && checked_row(a.off, j, a.n_edges, &jb, &jd, &jl);
        if (!valid) {
            if (!(j >= 0 && j < a.n_sites && j != i)) atomicAdd(&a.err[0], 1);
            const int ib = __shfl(beg, owner), id = __shfl(deg, owner);
            a.planes[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // den = 0: never a front face
            a.adj[k] = make_uint2((uint32_t)i | ((uint32_t)id << 24), (uint32_t)ib);
            continue;
        }
        const float xj = a.sites[3 * j], yj = a.sites[3 * j + 1], zj = a.sites[3 * j + 2];
        const float nx = xj - xi, ny = yj - yi, nz = zj - zi;
        const float mx = (xi + xj) * 0.5f, my = (yi + yj) * 0.5f, mz = (zi + zj) * 0.5f;
        const float cc = fmaf(nz, mz, fmaf(ny, my, nx * mx));
        a.planes[k] = make_float4(nx, ny, nz, cc);
        a.adj[k] = make_uint2((uint32_t)j | ((uint32_t)jd << 24), (uint32_t)jb);
    }
}

template <int DEG, bool BF16>
static hipError_t launch_pack_t(const PackArgs& a, hipStream_t stream)
{
    using R = Rec<DEG, BF16>;
    hipLaunchKernelGGL(k_zero_err, dim3(1), dim3(64), 0, stream, a.err);
    const unsigned blocks = (unsigned)((a.n_sites + 255) / 256);
    hipLaunchKernelGGL(k_pack_rows, dim3(blocks), dim3(256), 0, stream, a);
    const unsigned rblocks = (unsigned)((a.n_sites * R::CHUNKS + 255) / 256);
    hipLaunchKernelGGL((k_pack_records<DEG, BF16>), dim3(rblocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_pack_faces, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_pack(int sh_degree, bool bf16, const PackArgs& a, hipStream_t stream)
{
    switch (sh_degree * 2 + (bf16 ? 1 : 0)) {
    case 0: return launch_pack_t<0, false>(a, stream);
    case 1: return launch_pack_t<0, true>(a, stream);
    case 2: return launch_pack_t<1, false>(a, stream);
    case 3: return launch_pack_t<1, true>(a, stream);
    case 4: return launch_pack_t<2, false>(a, stream);
    case 5: return launch_pack_t<2, true>(a, stream);
    case 6: return launch_pack_t<3, false>(a, stream);
    case 7: return launch_pack_t<3, true>(a, stream);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Read-back of packed data (tests of the packing step).
// ---------------------------------------------------------------------------
template <int DEG, bool BF16>
__global__ void k_unpack_attr(SceneView s, float* density, float* sh)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_sites) return;
    Attr<DEG> at;
    load_record<DEG, BF16>(s.rec, (int)i, at);
    density[i] = at.sigma;
    for (int k = 0; k < 3 * sh_count(DEG); ++k) sh[i * 3 * sh_count(DEG) + k] = at.sh[k];
}

__global__ void k_unpack_planes(SceneView s, float* planes)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.n_edges) return;
    const float4 p = s.planes[k];
    planes[4 * k] = p.x;
    planes[4 * k + 1] = p.y;
    planes[4 * k + 2] = p.z;
    planes[4 * k + 3] = p.w;
}

template <int DEG, bool BF16>
static void launch_unpack_attr_t(const SceneView& s, float* density, float* sh, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((s.n_sites + 255) / 256);
    hipLaunchKernelGGL((k_unpack_attr<DEG, BF16>), dim3(blocks), dim3(256), 0, stream, s, density, sh);
}

hipError_t launch_unpack(int sh_degree, bool bf16, const SceneView& s, float* planes_out, float* density_out,
                         float* sh_out, hipStream_t stream)
{
    if (planes_out && s.n_edges > 0) {
        const unsigned blocks = (unsigned)((s.n_edges + 255) / 256);
        hipLaunchKernelGGL(k_unpack_planes, dim3(blocks), dim3(256), 0, stream, s, planes_out);
    }
    if (density_out && sh_out) {
        switch (sh_degree * 2 + (bf16 ? 1 : 0)) {
        case 0: launch_unpack_attr_t<0, false>(s, density_out, sh_out, stream); break;
        case 1: launch_unpack_attr_t<0, true>(s, density_out, sh_out, stream); break;
        case 2: launch_unpack_attr_t<1, false>(s, density_out, sh_out, stream); break;
        case 3: launch_unpack_attr_t<1, true>(s, density_out, sh_out, stream); break;
        case 4: launch_unpack_attr_t<2, false>(s, density_out, sh_out, stream); break;
        case 5: launch_unpack_attr_t<2, true>(s, density_out, sh_out, stream); break;
        case 6: launch_unpack_attr_t<3, false>(s, density_out, sh_out, stream); break;
        case 7: launch_unpack_attr_t<3, true>(s, density_out, sh_out, stream); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Camera rays in 8x8 tile order.
// ---------------------------------------------------------------------------
__device__ inline void tile_pixel(int64_t r, int W, int H, int* px, int* py)
{
    const int64_t band = 8 * (int64_t)W;  // rays in one full band of tile rows
    const int ty = (int)(r / band);
    int64_t rem = r - (int64_t)ty * band;
    const int h = min(8, H - 8 * ty);
    const int tx = (int)(rem / (8 * h));
    rem -= (int64_t)tx * 8 * h;
    const int w = min(8, W - 8 * tx);
    *py = 8 * ty + (int)(rem / w);
    *px = 8 * tx + (int)(rem % w);
}

__global__ __launch_bounds__(256) void k_raygen(RaygenArgs g)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = (int64_t)g.width * g.height;
    if (r >= R) return;
    int px, py;
    tile_pixel(r, g.width, g.height, &px, &py);
    float d[3], t;
    camera_ray(g.rot, g.pos, g.model, g.focal, g.width, g.height, px, py, g.bound_kind, g.bound, d, &t);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.origin[3 * r + k] = g.pos[k];
        g.dir[3 * r + k] = d[k];
    }
    g.t_max[r] = t;
    g.start_cell[r] = g.start;
    if (g.pixel) g.pixel[r] = py * g.width + px;
}

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t stream)
{
    const int64_t R = (int64_t)a.width * a.height;
    const unsigned blocks = (unsigned)((R + 255) / 256);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raygen, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace rf
