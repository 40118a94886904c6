// Scene packing (face planes, neighbour rows, per-cell records) and camera
// ray generation for gfx950.

#include "rf_device.hpp"
#include "rf_kernels.hpp"

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

// One thread per cell: its row reference and its record.
template <int DEG, bool BF16>
__global__ __launch_bounds__(256) void k_pack_cells(PackArgs a)
{
    using R = Rec<DEG, BF16>;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_sites) return;
    int beg, deg;
    bool too_long;
    const bool ok = checked_row(a.off, i, a.n_edges, &beg, &deg, &too_long);
    if (!ok) atomicAdd(&a.err[too_long ? 1 : 0], 1);
    if (i == 0 && a.off[0] != 0) atomicAdd(&a.err[0], 1);
    if (i == a.n_sites - 1 && a.off[a.n_sites] != a.n_edges) atomicAdd(&a.err[0], 1);
    a.row[i] = make_uint2((uint32_t)i | ((uint32_t)deg << 24), (uint32_t)beg);

    uint32_t w[4 * R::CHUNKS];
#pragma unroll
    for (int k = 0; k < 4 * R::CHUNKS; ++k) w[k] = 0u;
    const float* sh = a.sh + i * R::NSH;
    if constexpr (BF16) {
#pragma unroll
        for (int k = 0; k <= R::NSH; ++k) {
            const float v = k < R::NSH ? sh[k] : a.density[i];
            w[k >> 1] |= f32_to_bf16_rne(v) << ((k & 1) * 16);
        }
    } else {
#pragma unroll
        for (int k = 0; k < R::NSH; ++k) w[k] = __float_as_uint(sh[k]);
        w[R::NSH] = __float_as_uint(a.density[i]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) w[R::SITE_OFF / 4 + k] = __float_as_uint(a.sites[3 * i + k]);
    uint4* dst = reinterpret_cast<uint4*>(a.rec + i * R::BYTES);
#pragma unroll
    for (int c = 0; c < R::CHUNKS; ++c) dst[c] = make_uint4(w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]);
}

// One thread per cell: the planes and neighbour rows of its directed edges.
// n = x_j - x_i and c = n . ((x_i + x_j) / 2) are evaluated with the same
// instruction sequence for (i, j) and (j, i), so the two planes of a face are
// exact negations of each other.
__global__ __launch_bounds__(256) void k_pack_faces(PackArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_sites) return;
    int beg, deg;
    bool too_long;
    const bool ok = checked_row(a.off, i, a.n_edges, &beg, &deg, &too_long);
    if (!ok) return;
    const uint2 self = make_uint2((uint32_t)i | ((uint32_t)deg << 24), (uint32_t)beg);
    const float xi = a.sites[3 * i], yi = a.sites[3 * i + 1], zi = a.sites[3 * i + 2];
    for (int k = beg; k < beg + deg; ++k) {
        const int64_t j = a.idx[k];
        int jb = 0, jd = 0;
        bool jl;
        const bool valid = j >= 0 && j < a.n_sites && j != i && checked_row(a.off, j, a.n_edges, &jb, &jd, &jl);
        if (!valid) {
            if (!(j >= 0 && j < a.n_sites && j != i)) atomicAdd(&a.err[0], 1);
            a.planes[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // den = 0: never a front face
            a.adj[k] = self;
            continue;
        }
        const float xj = a.sites[3 * j], yj = a.sites[3 * j + 1], zj = a.sites[3 * j + 2];
        const float nx = xj - xi, ny = yj - yi, nz = zj - zi;
        const float mx = (xi + xj) * 0.5f, my = (yi + yj) * 0.5f, mz = (zi + zj) * 0.5f;
        const float c = fmaf(nz, mz, fmaf(ny, my, nx * mx));
        a.planes[k] = make_float4(nx, ny, nz, c);
        a.adj[k] = make_uint2((uint32_t)j | ((uint32_t)jd << 24), (uint32_t)jb);
    }
}

template <int DEG, bool BF16>
static hipError_t launch_pack_t(const PackArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_err, dim3(1), dim3(64), 0, stream, a.err);
    const unsigned blocks = (unsigned)((a.n_sites + 255) / 256);
    hipLaunchKernelGGL((k_pack_cells<DEG, BF16>), dim3(blocks), dim3(256), 0, stream, a);
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
    const float u = ((float)px + 0.5f - 0.5f * (float)g.width) / g.focal;
    const float v = ((float)py + 0.5f - 0.5f * (float)g.height) / g.focal;
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = fmaf(g.rot[3 * k], u, fmaf(g.rot[3 * k + 1], v, g.rot[3 * k + 2]));
    const float inv = 1.0f / sqrtf(fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2])));
    d[0] *= inv;
    d[1] *= inv;
    d[2] *= inv;
    float t;
    if (g.bound_kind == 0) {
        t = INFINITY;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (d[k] > 0.0f) t = fminf(t, (g.bound[3 + k] - g.pos[k]) / d[k]);
            else if (d[k] < 0.0f) t = fminf(t, (g.bound[k] - g.pos[k]) / d[k]);
        }
    } else {
        const float b = fmaf(g.pos[0], d[0], fmaf(g.pos[1], d[1], g.pos[2] * d[2]));
        const float c = fmaf(g.pos[0], g.pos[0], fmaf(g.pos[1], g.pos[1], g.pos[2] * g.pos[2])) - g.bound[0] * g.bound[0];
        const float disc = b * b - c;
        t = disc > 0.0f ? sqrtf(disc) - b : 0.0f;
    }
    t = fmaxf(t, 0.0f);
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
