// Training-step kernels around the walk (Sec. 3.3 and the implementation
// details of Sec. 3.4): the Adam update of positions, density and SH with
// per-group learning rates, the densification score and multinomial
// sampling of densification candidates, and the pruning mask.
//
// Adam is a pure stream over the parameters (read x, g, m, v; write x, m, v:
// 28 bytes per value), so it is written for HBM: one launch for all groups,
// each thread four consecutive values with non-temporal 16-byte loads and
// stores where the group's arrays are 16-byte aligned. The score and the mask read each
// cell's CSR row (one thread per cell). Sampling scans the scores in double
// (per block of 1024, then the block totals in one block, then the offsets) and inverts
// the cumulative sum at each draw by binary search.

#include <mutex>

#include "rf_device.hpp"
#include "rf_kernels.hpp"

namespace rf {

constexpr int kTrainBlock = 256;

// ---------------------------------------------------------------------------
// Adam: one launch over the three groups (positions, density, SH); block b
// belongs to the group whose block range holds it. Each thread streams four
// consecutive values with non-temporal 16-byte accesses (nothing is reused
// within the step) when the group's arrays are 16-byte aligned.
// ---------------------------------------------------------------------------
__device__ inline void adam_one(const AdamGroup& a, int s, float& x, float g, float& m, float& v)
{
    const float lr = a.lr[s];
    if (lr == 0.0f) return;  // a held group keeps its values and moments
    if (a.kind == 1) {
        // softplus_10(x) has derivative 1 / (1 + e^{-10 x}) (in double, as the pack's softplus)
        g = (float)((double)g / (1.0 + exp(-10.0 * (double)x)));
    }
    m = fmaf(a.beta1, m, (1.0f - a.beta1) * g);
    v = fmaf(a.beta2, v, (1.0f - a.beta2) * g * g);
    x = x - lr * (m * a.c1[s]) / (sqrtf(v * a.c2[s]) + a.eps);
}

__device__ inline float4 ld_nt(const float* p, int64_t i)
{
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + i);
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ inline void st_nt(float* p, int64_t i, float4 v)
{
    __builtin_nontemporal_store(f32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<f32x4*>(p) + i);
}

struct AdamLaunch {
    AdamGroup g[3];
    int64_t first_block[3];  // first block of each group
    int32_t vec[3];          // the group's arrays are 16-byte aligned
};

__global__ __launch_bounds__(kTrainBlock) void k_adam(AdamLaunch L)
{
    const int gi = blockIdx.x >= L.first_block[2] ? 2 : (blockIdx.x >= L.first_block[1] ? 1 : 0);
    const AdamGroup& a = L.g[gi];
    const int64_t t = ((int64_t)blockIdx.x - L.first_block[gi]) * kTrainBlock + threadIdx.x;
    const int64_t k0 = 4 * t;
    if (k0 >= a.n) return;
    // SH values pick their order's parameters by basis index b = (k / 3) mod B,
    // stepped along the thread's four values (32-bit: n < 2^32)
    int sel[4] = {0, 0, 0, 0};
    if (a.kind == 2) {
        const uint32_t q = (uint32_t)k0 / 3u;
        uint32_t r3 = (uint32_t)k0 - 3u * q, b = q % (uint32_t)a.B;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sel[u] = b != 0;
            if (++r3 == 3u) {
                r3 = 0;
                if (++b == (uint32_t)a.B) b = 0;
            }
        }
    }
    if (L.vec[gi] && k0 + 4 <= a.n) {
        float4 x = ld_nt(a.x, t), m = ld_nt(a.m, t), v = ld_nt(a.v, t);
        const float4 g = ld_nt(a.g, t);
        adam_one(a, sel[0], x.x, g.x, m.x, v.x);
        adam_one(a, sel[1], x.y, g.y, m.y, v.y);
        adam_one(a, sel[2], x.z, g.z, m.z, v.z);
        adam_one(a, sel[3], x.w, g.w, m.w, v.w);
        st_nt(a.x, t, x);
        st_nt(a.m, t, m);
        st_nt(a.v, t, v);
        return;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t k = k0 + u;
        if (k >= a.n) break;
        float x = a.x[k], m = a.m[k], v = a.v[k];
        adam_one(a, sel[u], x, a.g[k], m, v);
        a.x[k] = x;
        a.m[k] = m;
        a.v[k] = v;
    }
}

hipError_t launch_adam(const AdamGroup groups[3], hipStream_t stream)
{
    AdamLaunch L;
    int64_t blocks = 0;
    for (int q = 0; q < 3; ++q) {
        L.g[q] = groups[q];
        L.first_block[q] = blocks;
        blocks += ((groups[q].n + 3) / 4 + kTrainBlock - 1) / kTrainBlock;
        L.vec[q] = ((reinterpret_cast<uintptr_t>(groups[q].x) | reinterpret_cast<uintptr_t>(groups[q].g) |
                     reinterpret_cast<uintptr_t>(groups[q].m) | reinterpret_cast<uintptr_t>(groups[q].v)) & 15) == 0;
    }
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kTrainBlock), 0, stream, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Densification score and pruning mask (one thread per cell).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTrainBlock) void k_densify_score(const float* __restrict__ sites,
                                                               const int32_t* __restrict__ off,
                                                               const int32_t* __restrict__ idx, int64_t n,
                                                               const float* __restrict__ grad_sites,
                                                               float* __restrict__ score)
{
    const int64_t i = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (i >= n) return;
    const float xi = sites[3 * i], yi = sites[3 * i + 1], zi = sites[3 * i + 2];
    const int beg = off[i], end = off[i + 1];
    float sum = 0.0f;
    int cnt = 0;
    for (int k = beg; k < end; ++k) {
        const int64_t j = idx[k];
        if (j < 0 || j >= n) continue;  // an invalid neighbour id is skipped
        const float dx = sites[3 * j] - xi, dy = sites[3 * j + 1] - yi, dz = sites[3 * j + 2] - zi;
        sum += sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        ++cnt;
    }
    const float r = cnt > 0 ? 0.5f * sum / (float)cnt : 0.0f;
    const float gx = grad_sites[3 * i], gy = grad_sites[3 * i + 1], gz = grad_sites[3 * i + 2];
    score[i] = sqrtf(fmaf(gz, gz, fmaf(gy, gy, gx * gx))) * r;
}

__global__ __launch_bounds__(kTrainBlock) void k_prune_mask(const float* __restrict__ density,
                                                            const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ idx, int64_t n,
                                                            float threshold, uint8_t* __restrict__ mask)
{
    const int64_t i = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (i >= n) return;
    bool prune = density[i] < threshold;
    for (int k = off[i]; prune && k < off[i + 1]; ++k) {
        const int64_t j = idx[k];
        if (j >= 0 && j < n) prune = density[j] < threshold;  // an invalid neighbour id is skipped
    }
    mask[i] = prune ? 1 : 0;
}

hipError_t launch_densify_score(const float* sites, const int32_t* off, const int32_t* idx, int64_t n,
                                const float* grad_sites, float* score, hipStream_t stream)
{
    const int64_t blocks = (n + kTrainBlock - 1) / kTrainBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_densify_score, dim3((unsigned)blocks), dim3(kTrainBlock), 0, stream, sites, off, idx, n,
                       grad_sites, score);
    return hipGetLastError();
}

hipError_t launch_prune_mask(const float* density, const int32_t* off, const int32_t* idx, int64_t n,
                             float threshold, uint8_t* mask, hipStream_t stream)
{
    const int64_t blocks = (n + kTrainBlock - 1) / kTrainBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prune_mask, dim3((unsigned)blocks), dim3(kTrainBlock), 0, stream, density, off, idx, n,
                       threshold, mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inserting and removing sites (densification and pruning applied).
// ---------------------------------------------------------------------------
// A new site inside its parent's cell: x_p + frac r_p u, with r_p the radius
// of the largest ball about x_p inside the cell, half the distance to the
// nearest Delaunay neighbour (the nearest bisector plane). Formed in double,
// rounded once to FP32. A parent out of range gives NaN coordinates.
__global__ __launch_bounds__(kTrainBlock) void k_insert_sites(const float* __restrict__ sites,
                                                              const int32_t* __restrict__ off,
                                                              const int32_t* __restrict__ idx, int64_t n_sites,
                                                              const int32_t* __restrict__ parents,
                                                              const float* __restrict__ u, int64_t n_new, float frac,
                                                              float* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (k >= n_new) return;
    const int p = parents[k];
    if (p < 0 || p >= n_sites) {
        out[3 * k] = out[3 * k + 1] = out[3 * k + 2] = __int_as_float(0x7fc00000);
        return;
    }
    const double x[3] = {sites[3 * (int64_t)p], sites[3 * (int64_t)p + 1], sites[3 * (int64_t)p + 2]};
    double best = INFINITY;
    for (int e = off[p]; e < off[p + 1]; ++e) {
        const int j = idx[e];
        if (j < 0 || j >= n_sites || j == p) continue;
        const double dx = sites[3 * (int64_t)j] - x[0], dy = sites[3 * (int64_t)j + 1] - x[1],
                     dz = sites[3 * (int64_t)j + 2] - x[2];
        best = fmin(best, fma(dz, dz, fma(dy, dy, dx * dx)));
    }
    const double s = isfinite(best) ? (double)frac * 0.5 * sqrt(best) : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[3 * k + c] = (float)fma(s, (double)u[3 * k + c], x[c]);
}

// out[k][:] = in[rows[k]][:] for rows of `width` floats; a row index out of
// range gives a row of NaN.
__global__ __launch_bounds__(kTrainBlock) void k_gather_rows(const float* __restrict__ in, int64_t n_in, int width,
                                                             const int32_t* __restrict__ rows, int64_t n_out,
                                                             float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (e >= n_out * width) return;
    const int64_t k = e / width;
    const int c = (int)(e - k * width);
    const int r = rows[k];
    out[e] = (r >= 0 && r < n_in) ? in[(int64_t)r * width + c] : __int_as_float(0x7fc00000);
}

// The kept indices of a mask, in order: per tile of kKeepTile flags a count,
// an exclusive scan of the counts (one block), then every kept index written
// at its tile's offset plus its rank in the tile.
constexpr int kKeepPer = 4;
constexpr int kKeepTile = kTrainBlock * kKeepPer;

__device__ inline int block_exclusive_scan(int v, int* wave_sum, int& total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int incl = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sum[w] = incl;
    __syncthreads();
    int before = incl - v;
    total = 0;
    for (int q = 0; q < kTrainBlock / kWave; ++q) {
        if (q < w) before += wave_sum[q];
        total += wave_sum[q];
    }
    return before;
}

__global__ __launch_bounds__(kTrainBlock) void k_keep_count(const uint8_t* __restrict__ keep, int64_t n,
                                                            int64_t* __restrict__ counts)
{
    __shared__ int wave_sum[kTrainBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kKeepTile + (int64_t)threadIdx.x * kKeepPer;
    int c = 0;
#pragma unroll
    for (int q = 0; q < kKeepPer; ++q) c += (base + q < n && keep[base + q]) ? 1 : 0;
    int total;
    (void)block_exclusive_scan(c, wave_sum, total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Exclusive scan of the tile counts in place (one block); the sum into *n_kept.
__global__ __launch_bounds__(kTrainBlock) void k_keep_offsets(int64_t* counts, int64_t n_tiles, int64_t* n_kept)
{
    __shared__ int64_t wave_sum[kTrainBlock / kWave];
    const int64_t per = (n_tiles + kTrainBlock - 1) / kTrainBlock;
    const int64_t beg = (int64_t)threadIdx.x * per;
    const int64_t end = beg + per < n_tiles ? beg + per : n_tiles;
    int64_t run = 0;
    for (int64_t b = beg; b < end; ++b) run += counts[b];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t incl = run;
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sum[w] = incl;
    __syncthreads();
    int64_t acc = incl - run;
    for (int q = 0; q < w; ++q) acc += wave_sum[q];
    for (int64_t b = beg; b < end; ++b) {
        const int64_t t = counts[b];
        counts[b] = acc;
        acc += t;
    }
    if (threadIdx.x == kTrainBlock - 1) *n_kept = acc;
}

__global__ __launch_bounds__(kTrainBlock) void k_keep_scatter(const uint8_t* __restrict__ keep, int64_t n,
                                                              const int64_t* __restrict__ offsets,
                                                              int32_t* __restrict__ kept)
{
    __shared__ int wave_sum[kTrainBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kKeepTile + (int64_t)threadIdx.x * kKeepPer;
    bool f[kKeepPer];
    int c = 0;
#pragma unroll
    for (int q = 0; q < kKeepPer; ++q) {
        f[q] = base + q < n && keep[base + q];
        c += f[q] ? 1 : 0;
    }
    int total;
    int64_t pos = offsets[blockIdx.x] + block_exclusive_scan(c, wave_sum, total);
#pragma unroll
    for (int q = 0; q < kKeepPer; ++q)
        if (f[q]) kept[pos++] = (int32_t)(base + q);
}

hipError_t launch_insert_sites(const float* sites, const int32_t* off, const int32_t* idx, int64_t n_sites,
                               const int32_t* parents, const float* u, int64_t n_new, float frac, float* out,
                               hipStream_t stream)
{
    const int64_t blocks = (n_new + kTrainBlock - 1) / kTrainBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_insert_sites, dim3((unsigned)blocks), dim3(kTrainBlock), 0, stream, sites, off, idx, n_sites,
                       parents, u, n_new, frac, out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* in, int64_t n_in, int width, const int32_t* rows, int64_t n_out,
                              float* out, hipStream_t stream)
{
    const int64_t blocks = (n_out * width + kTrainBlock - 1) / kTrainBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks), dim3(kTrainBlock), 0, stream, in, n_in, width, rows,
                       n_out, out);
    return hipGetLastError();
}

int64_t keep_workspace_count(int64_t n) { return (n + kKeepTile - 1) / kKeepTile; }

hipError_t launch_keep_index(const uint8_t* keep, int64_t n, int32_t* kept, int64_t* n_kept, int64_t* workspace,
                             hipStream_t stream)
{
    const int64_t tiles = keep_workspace_count(n);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    if (tiles > 0)
        hipLaunchKernelGGL(k_keep_count, dim3((unsigned)tiles), dim3(kTrainBlock), 0, stream, keep, n, workspace);
    // (with no tiles this only writes *n_kept = 0)
    hipLaunchKernelGGL(k_keep_offsets, dim3(1), dim3(kTrainBlock), 0, stream, workspace, tiles, n_kept);
    if (tiles > 0)
        hipLaunchKernelGGL(k_keep_scatter, dim3((unsigned)tiles), dim3(kTrainBlock), 0, stream, keep, n, workspace,
                           kept);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Multinomial sampling by inverting the cumulative score (double).
// ---------------------------------------------------------------------------
constexpr int kScanPer = 4;                          // values per thread
constexpr int kScanTile = kTrainBlock * kScanPer;    // values per block

// Inclusive scan of one tile of scores into cdf; the tile's total into totals[block].
__global__ __launch_bounds__(kTrainBlock) void k_scan_tiles(const float* __restrict__ score, int64_t n,
                                                            double* __restrict__ cdf, double* __restrict__ totals)
{
    __shared__ double wave_sum[kTrainBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    double v[kScanPer];
    double run = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        run += base + q < n ? (double)score[base + q] : 0.0;
        v[q] = run;
    }
    // exclusive prefix of the threads' sums: within the wavefront, then across wavefronts
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double incl = run;
    for (int d = 1; d < kWave; d <<= 1) {
        const double o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sum[w] = incl;
    __syncthreads();
    double before = incl - run;
    for (int q = 0; q < w; ++q) before += wave_sum[q];
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < n) cdf[base + q] = before + v[q];
    if (threadIdx.x == kTrainBlock - 1) totals[blockIdx.x] = before + run;
}

// Exclusive prefix of the tile totals, in place, by one block: each thread
// sums a contiguous run of totals, the block scans the runs' sums, and each
// thread rewrites its run with the offsets.
__global__ __launch_bounds__(kTrainBlock) void k_scan_totals(double* totals, int64_t n_tiles)
{
    __shared__ double wave_sum[kTrainBlock / kWave];
    const int64_t per = (n_tiles + kTrainBlock - 1) / kTrainBlock;
    const int64_t beg = (int64_t)threadIdx.x * per;
    const int64_t end = beg + per < n_tiles ? beg + per : n_tiles;
    double run = 0.0;
    for (int64_t b = beg; b < end; ++b) run += totals[b];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double incl = run;
    for (int d = 1; d < kWave; d <<= 1) {
        const double o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sum[w] = incl;
    __syncthreads();
    double acc = incl - run;
    for (int q = 0; q < w; ++q) acc += wave_sum[q];
    for (int64_t b = beg; b < end; ++b) {
        const double t = totals[b];
        totals[b] = acc;
        acc += t;
    }
}

__global__ __launch_bounds__(kTrainBlock) void k_scan_add(double* __restrict__ cdf, int64_t n,
                                                          const double* __restrict__ offsets)
{
    const int64_t k = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (k >= n) return;
    cdf[k] += offsets[k / kScanTile];
}

// Cell of each draw: the first index whose cumulative score exceeds u * total.
__global__ __launch_bounds__(kTrainBlock) void k_sample(const double* __restrict__ cdf, int64_t n,
                                                        const float* __restrict__ draws, int64_t n_draws,
                                                        int32_t* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kTrainBlock + threadIdx.x;
    if (k >= n_draws) return;
    const double target = (double)draws[k] * cdf[n - 1];
    int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    out[k] = (int32_t)(lo < n ? lo : n - 1);
}

int64_t sample_workspace_doubles(int64_t n)
{
    return n + (n + kScanTile - 1) / kScanTile;
}

// Scratch of the allocation-free sampler (rf_sample_cells_noalloc): the
// cumulative scores and tile offsets of up to kNoAllocMaxCells cells. Every
// GPU the library runs on holds its own copy until the process ends; calls on
// one GPU share it, so calls that overlap on one GPU race. Nothing needs
// clearing: each call writes every value it reads before reading it.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 22;
constexpr int64_t kNoAllocScratchDoubles = kNoAllocMaxCells + (kNoAllocMaxCells + kScanTile - 1) / kScanTile;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

// The device address of `scratch` on each device, looked up once per device
// with that device current (in host code the array's name is not a device
// address).
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxScratchDevices] = {};

int64_t sample_noalloc_max_cells() { return kNoAllocMaxCells; }

hipError_t sample_scratch(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_sample(const float* score, int64_t n, const float* draws, int64_t n_draws, int32_t* out,
                         double* workspace, hipStream_t stream)
{
    if (n == 0 || n_draws == 0) return hipSuccess;
    double* cdf = workspace;
    double* totals = workspace + n;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kTrainBlock), 0, stream, score, n, cdf, totals);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kTrainBlock), 0, stream, totals, tiles);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + kTrainBlock - 1) / kTrainBlock)), dim3(kTrainBlock), 0,
                       stream, cdf, n, totals);
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((n_draws + kTrainBlock - 1) / kTrainBlock)), dim3(kTrainBlock), 0,
                       stream, cdf, n, draws, n_draws, out);
    return hipGetLastError();
}

}  // namespace rf
