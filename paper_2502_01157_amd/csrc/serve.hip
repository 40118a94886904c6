// Continuous-batching render server.
//
// The packed scene stays resident. Admitted requests are cut into 8x8 screen
// tiles; a host scheduler thread repeatedly builds one launch from the
// pending tiles of every admitted request (oldest request first, newer
// requests fill the rest of the launch), so tiles of requests that arrived
// while others were on the GPU share launches with theirs. Two launches are
// kept queued on the server's stream so the GPU never waits for the host.
// Each launch is an ordinary kernel over a list of tile descriptors: one
// wavefront per tile renders its 64 pixels with the same ray generation and
// walk as rf_raygen + rf_render_forward and writes RGBA (colour, final
// transmittance) straight into the request's region of a pinned host output
// pool. Nothing on the device waits for anything: every launch ends when its
// tiles are done. The host retires a launch when its event completes, and a
// request when all its tiles are retired (the kernel's completion makes its
// host-memory writes visible).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "radfoam.h"
#include "rf_device.hpp"
#include "rf_kernels.hpp"
#include "rf_locate.hpp"
#include "rf_walk.hpp"
#include "serve_protocol.hpp"

namespace rf {

constexpr int kMaxSlots = 64;           // in-flight requests
constexpr int kMaxBatchTiles = 8192;    // tiles per launch (524,288 rays)
constexpr int kLaunchesInFlight = 2;
constexpr int kLocalTileBits = 25;      // descriptor = slot << 25 | tile within the request
constexpr int kSeedGrid = 16;           // seed grid for locating camera cells on the device
constexpr int kStagedMinTiles = 8192;   // launches of at least this many tiles use the staged walk
constexpr int kPersistStagedMinTiles = 8192;  // persistent form: requests of at least this many tiles

struct ReqRecord {
    float rot[9];
    float pos[3];
    int32_t model;
    float focal;
    int32_t width, height, start;
    int64_t out_offset;  // floats from the pool base
};

struct BatchArgs {
    SceneView s;
    float eps;
    int32_t max_steps;
    int32_t bound_kind;
    float bound[6];
    const ReqRecord* reqs;  // device table, one record per slot
    const uint32_t* desc;   // device tile descriptors
    int32_t n_tiles;
    float* pool;            // pinned host output pool (device-visible pointer)
};

// One tile per wavefront and per block, so that a block's slots are released
// when its own tile is done. STAGED: the walk stages its cells in LDS (as the
// batch forward does): more tiles per second once the chip is full, a longer
// walk for a lone wavefront (each step waits for its copies); the same
// results bit for bit either way. Only full launches stage: on the 512-request
// replay, staging launches from 4,096 tiles up raised the median latency
// (2.30 -> 2.38 ms), from 8,192 lowered it (2.19 ms).
template <int DEG, bool BF16, bool STAGED>
__global__ __launch_bounds__(kWave) void k_serve_tiles(BatchArgs a)
{
    const int lane = threadIdx.x;
    const int tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    const uint32_t desc = a.desc[tile];
    const int slot = (int)(desc >> kLocalTileBits);
    const int local = (int)(desc & ((1u << kLocalTileBits) - 1));
    const ReqRecord& rq = a.reqs[slot];
    const int W = rq.width, H = rq.height;
    const int tiles_x = (W + 7) / 8;
    const int px = (local % tiles_x) * 8 + (lane & 7);
    const int py = (local / tiles_x) * 8 + (lane >> 3);
    const bool live = px < W && py < H;
    float d[3], tmax;
    RayResult res;
    if constexpr (STAGED) {
        // every lane takes part in the staging, lanes past the image's edge without a ray
        using SL = StageLayout<DEG, BF16>;
        __shared__ __align__(16) unsigned char stage_mem[SL::kBytes];
        camera_ray(rq.rot, rq.pos, rq.model, rq.focal, W, H, px, py, a.bound_kind, a.bound, d, &tmax);
        walk_forward_staged<DEG, BF16, false, false>(a.s, live, rq.pos[0], rq.pos[1], rq.pos[2], d[0], d[1], d[2],
                                                     tmax, rq.start, a.eps, a.max_steps, nullptr, nullptr, 0, res,
                                                     nullptr, 0, (lds_u8*)stage_mem);
        if (!live) return;
    } else {
        if (!live) return;
        camera_ray(rq.rot, rq.pos, rq.model, rq.focal, W, H, px, py, a.bound_kind, a.bound, d, &tmax);
        walk_forward<DEG, BF16, false>(a.s, rq.pos[0], rq.pos[1], rq.pos[2], d[0], d[1], d[2], tmax, rq.start,
                                       a.eps, a.max_steps, nullptr, nullptr, 0, res);
    }
    float4* out = reinterpret_cast<float4*>(a.pool + rq.out_offset) + ((int64_t)py * W + px);
    *out = make_float4(res.C[0], res.C[1], res.C[2], res.T);
}

template <int DEG, bool BF16>
static hipError_t launch_batch_t(const BatchArgs& a, hipStream_t stream)
{
    if (a.n_tiles >= kStagedMinTiles)
        hipLaunchKernelGGL((k_serve_tiles<DEG, BF16, true>), dim3((unsigned)a.n_tiles), dim3(kWave), 0, stream, a);
    else
        hipLaunchKernelGGL((k_serve_tiles<DEG, BF16, false>), dim3((unsigned)a.n_tiles), dim3(kWave), 0, stream, a);
    return hipGetLastError();
}

static hipError_t launch_batch(int deg, bool bf16, const BatchArgs& a, hipStream_t stream)
{
    switch (deg * 2 + (bf16 ? 1 : 0)) {
    case 0: return launch_batch_t<0, false>(a, stream);
    case 1: return launch_batch_t<0, true>(a, stream);
    case 2: return launch_batch_t<1, false>(a, stream);
    case 3: return launch_batch_t<1, true>(a, stream);
    case 4: return launch_batch_t<2, false>(a, stream);
    case 5: return launch_batch_t<2, true>(a, stream);
    case 6: return launch_batch_t<3, false>(a, stream);
    case 7: return launch_batch_t<3, true>(a, stream);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Persistent form: one launch serves requests as they arrive.
//
// Block 0 is the dispatcher wavefront; every other block is one worker
// wavefront. The protocol (request ring in coherent host memory, slot
// records and claim/done words in device memory) is in serve_protocol.hpp.
// Workers take the oldest open request (its 64 slots are inspected by the 64
// lanes at once), claim up to kClaimTiles tiles of it (fewer when its tiles
// left are fewer than that per worker), render each tile exactly as
// k_serve_tiles does, and report the claim done once. An idle worker polls
// one word (the count of openings) and naps between polls, longer once it
// has been idle for a while. Every wait is bounded: the dispatcher leaves
// when the host asks, or once no request has arrived for `idle_ticks` and
// every admitted request is done, or after `hard_ticks` without a new
// request; a worker leaves when the dispatcher has left and no request is
// open, or after `hard_ticks` without a tile; both also leave after
// kIdleIterCap units of idle polling whatever the clock says. The host
// relaunches the kernel when requests wait and no launch is running.
// ---------------------------------------------------------------------------
constexpr int kClaimTiles = 4;
constexpr uint32_t kIdleIterCap = 1u << 22;  // idle polling in units of ~1 us: ~4 s

struct DevEnv {
    __device__ static uint64_t dev_load_acquire(const uint64_t* p)
    {
        return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static uint64_t dev_load_relaxed(const uint64_t* p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void dev_fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ static void dev_store_relaxed(uint64_t* p, uint64_t v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void dev_store_release(uint64_t* p, uint64_t v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void dev_fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
    __device__ static uint64_t dev_fetch_add_acq_rel(uint64_t* p, uint64_t v)
    {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static uint64_t dev_fetch_add_acquire(uint64_t* p, uint64_t v)
    {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // a release at system scope: a release fence of that scope before the
    // addition (the word itself is only ever shared by the device)
    __device__ static uint64_t sys_fetch_add_release(uint64_t* p, uint64_t v)
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void sys_store_release(uint64_t* p, uint64_t v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __device__ static uint32_t word_load(const uint32_t* p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};
using Proto = sp::Protocol<DevEnv>;

__device__ inline int64_t uniform(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
}

struct PersistArgs {
    SceneView s;
    float eps;
    int32_t max_steps;
    int32_t bound_kind;
    float bound[6];
    sp::HostCtl* host;  // coherent host memory (device-visible pointer)
    sp::DevCtl* dev;
    float* pool;        // pinned host output pool
    const int32_t* grid;  // seed grid of located cells (requests without a start cell)
    int32_t grid_n;
    float grid_lo[3], grid_inv[3];
    int64_t consumed0;  // records consumed before this launch
    uint64_t idle_ticks, hard_ticks;  // wall-clock ticks
};

template <int DEG, bool BF16>
__device__ void persistent_dispatcher(const PersistArgs& a, int lane)
{
    int64_t consumed = a.consumed0;
    uint64_t last = wall_clock64();
    uint32_t idle_iters = 0;
    while (idle_iters < kIdleIterCap) {
        // polled relaxed (an acquire at system scope would invalidate this
        // XCD's L2 on every poll); acquired once a record is there
        // (lane 0's value for the whole wavefront: the control flow below stays uniform)
        const int64_t n_req = uniform(__hip_atomic_load(&a.host->n_requests, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
        // the host never has more than kSlots records unconsumed; anything else is not a count it wrote
        if (n_req < consumed || n_req - consumed > sp::kReqRing) break;
        if (consumed < n_req) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            // the record, one word per lane, from the host ring
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&a.host->ring[consumed % sp::kReqRing]);
            uint32_t w = 0;
            if (lane < sp::kReqWords) w = __hip_atomic_load(src + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const int slot = __shfl((int)w, (int)(offsetof(sp::Req, slot) / 4));
            const uint32_t gen = (uint32_t)__shfl((int)w, (int)(offsetof(sp::Req, gen) / 4));
            int start = __shfl((int)w, (int)(offsetof(sp::Req, start) / 4));
            if (start < 0) {
                // the camera's cell, located from the seed grid
                const float px = __int_as_float(__shfl((int)w, (int)(offsetof(sp::Req, pos) / 4)));
                const float py = __int_as_float(__shfl((int)w, (int)(offsetof(sp::Req, pos) / 4) + 1));
                const float pz = __int_as_float(__shfl((int)w, (int)(offsetof(sp::Req, pos) / 4) + 2));
                if (lane == 0)
                    start = locate_point<DEG, BF16>(a.s, px, py, pz,
                                                    grid_seed(a.grid, a.grid_n, a.grid_lo, a.grid_inv, px, py, pz),
                                                    1 << 20);
                start = __shfl(start, 0);
                if (lane == (int)(offsetof(sp::Req, start) / 4)) w = (uint32_t)start;
            }
            const int n_tiles = __shfl((int)w, (int)(offsetof(sp::Req, n_tiles) / 4));
            if (slot >= 0 && slot < sp::kSlots && gen != 0 && n_tiles > 0) {
                // the record, one word per lane (no claim reads the slot
                // before the activation below: its last request completed)
                uint32_t* dst = reinterpret_cast<uint32_t*>(&a.dev->slots[slot]);
                if (lane < sp::kReqWords)
                    __hip_atomic_store(dst + lane, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // every lane's words ordered before lane 0's release of the slot
                __syncthreads();
                if (lane == 0) Proto::activate(a.dev, slot, gen, n_tiles);
            }
            ++consumed;
            if (lane == 0)
                __hip_atomic_store(&a.host->consumed, consumed, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            last = wall_clock64();
            idle_iters = 0;
            continue;
        }
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(&a.host->shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)))
            break;
        const uint64_t quiet = wall_clock64() - last;
        if (quiet > a.idle_ticks) {
            const bool idle = Proto::slot_idle(a.dev, lane);  // lane = slot (kSlots == kWave)
            if (ballot(!idle) == 0) break;                 // everything admitted is done
            if (quiet > a.hard_ticks) break;                 // no request for long: the host relaunches
        }
        ++idle_iters;
        __builtin_amdgcn_s_sleep(16);
    }
    if (lane == 0) __hip_atomic_store(&a.dev->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DEG, bool BF16>
__device__ void persistent_worker(const PersistArgs& a, int lane, lds_u8* region)
{
    uint64_t last = wall_clock64();
    uint32_t idle_units = 0;  // idle polls, in units of ~1 us
    uint32_t naps = 0;        // consecutive polls that found nothing new
    uint64_t seen = ~0ull;    // openings counted before the last scan that found nothing open
    bool fenced = true;       // the next scan follows an acquire fence
    while (idle_units < kIdleIterCap) {
        // the count's low 32 bits (an idle nap does not span 2^32 openings)
        const uint64_t o = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)Proto::opened(a.dev));
        if (o == seen) {
            // nothing opened since a scan found every slot closed or fully claimed
            if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(&a.dev->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
                break;
            if (wall_clock64() - last > a.hard_ticks) break;
            // short naps first, then ~50 us between polls: a few thousand idle
            // wavefronts polling at once would crowd the memory channel of
            // these words, which the working wavefronts need too
            if (naps < 64) {
                __builtin_amdgcn_s_sleep(127);
                idle_units += 4;
            } else {
                for (int r = 0; r < 16; ++r) __builtin_amdgcn_s_sleep(127);
                idle_units += 64;
            }
            ++naps;
            continue;
        }
        // a working wavefront scans without a fence (claim() validates what
        // the scan picks); a scan that finds nothing open is trusted only
        // after one that followed a fence
        if (fenced) DevEnv::dev_fence_acquire();
        uint64_t seq = ~0ull;
        int64_t left = 0;
        const bool op = Proto::open(a.dev, lane, &seq, &left);  // lane = slot
        if (!op) seq = ~0ull;
        const uint64_t open_lanes = ballot(op);
        if (open_lanes == 0) {
            if (fenced) seen = o;
            fenced = true;
            ++idle_units;
            continue;
        }
        seen = ~0ull;
        fenced = false;
        naps = 0;
        // the oldest open request
        uint64_t m = seq;
#pragma unroll
        for (int off = kWave / 2; off >= 1; off >>= 1) {
            const uint64_t x = __shfl_xor(m, off);
            m = x < m ? x : m;
        }
        const int slot = __builtin_ctzll(ballot(op && seq == m));
        // up to kClaimTiles tiles, fewer while the request's tiles left do not
        // give every worker that many: a small request is spread over the chip
        const int64_t slot_left = __shfl(left, slot);
        const int64_t per_worker = slot_left / (int64_t)(gridDim.x - 1);
        const int k = (int)(per_worker < 1 ? 1 : per_worker > kClaimTiles ? kClaimTiles : per_worker);
        sp::Claim c = {0, 0, 0, 0, 0};
        int cnt = 0;
        if (lane == 0) cnt = Proto::claim(a.dev, slot, k, &c);
        cnt = __builtin_amdgcn_readfirstlane(cnt);
        if (cnt == 0) {
            ++idle_units;
            continue;
        }
        c.first = __builtin_amdgcn_readfirstlane(c.first);
        c.count = cnt;
        // the claimed request's record, which stays in the slot while the
        // claim is outstanding: lane 0's loads (ordered by its claim's
        // acquire), broadcast to the wavefront
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(&a.dev->slots[slot]);
        auto word = [&](size_t off) { return __builtin_amdgcn_readfirstlane(DevEnv::word_load(rw + off / 4)); };
        float rot[9], pos[3];
        for (int k = 0; k < 9; ++k) rot[k] = __uint_as_float(word(offsetof(sp::Req, rot) + 4 * k));
        for (int k = 0; k < 3; ++k) pos[k] = __uint_as_float(word(offsetof(sp::Req, pos) + 4 * k));
        const int model = (int)word(offsetof(sp::Req, model));
        const float focal = __uint_as_float(word(offsetof(sp::Req, focal)));
        const int W = (int)word(offsetof(sp::Req, width)), H = (int)word(offsetof(sp::Req, height));
        const int start = (int)word(offsetof(sp::Req, start));
        const int64_t out_off = (int64_t)(((uint64_t)word(offsetof(sp::Req, out_offset_hi)) << 32) |
                                          word(offsetof(sp::Req, out_offset_lo)));
        const int tiles_x = (W + 7) / 8;
        float* out_base = a.pool + out_off;
        // a large request's tiles walk with their cells staged in LDS, as
        // the launches' full launches do (the same bits either way); the
        // staged walk needs the whole wavefront, so the choice is lane 0's
        const bool staged = __builtin_amdgcn_readfirstlane(c.n_tiles) >= kPersistStagedMinTiles;
        for (int j = 0; j < cnt; ++j) {
            const int local = c.first + j;
            const int px = (local % tiles_x) * 8 + (lane & 7);
            const int py = (local / tiles_x) * 8 + (lane >> 3);
            const bool live = px < W && py < H;
            float d[3], tmax;
            RayResult res;
            if (staged) {
                camera_ray(rot, pos, model, focal, W, H, px, py, a.bound_kind, a.bound, d, &tmax);
                walk_forward_staged<DEG, BF16, false, false>(a.s, live, pos[0], pos[1], pos[2], d[0], d[1], d[2], tmax,
                                                             start, a.eps, a.max_steps, nullptr, nullptr, 0, res,
                                                             nullptr, 0, region);
            } else if (live) {
                camera_ray(rot, pos, model, focal, W, H, px, py, a.bound_kind, a.bound, d, &tmax);
                walk_forward<DEG, BF16, false>(a.s, pos[0], pos[1], pos[2], d[0], d[1], d[2], tmax, start, a.eps,
                                               a.max_steps, nullptr, nullptr, 0, res);
            }
            if (live) {
                float4* out = reinterpret_cast<float4*>(out_base) + ((int64_t)py * W + px);
                *out = make_float4(res.C[0], res.C[1], res.C[2], res.T);
            }
        }
        // every lane's pixels ordered before lane 0's release of the claim
        __syncthreads();
        if (lane == 0) (void)Proto::tiles_done(a.dev, a.host, slot, c);
        last = wall_clock64();
        idle_units = 0;
    }
}

template <int DEG, bool BF16>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_serve_persistent(PersistArgs a)
{
    const int lane = threadIdx.x;
    __shared__ __align__(16) unsigned char stage_mem[StageLayout<DEG, BF16>::kBytes];
    if (blockIdx.x == 0)
        persistent_dispatcher<DEG, BF16>(a, lane);
    else
        persistent_worker<DEG, BF16>(a, lane, (lds_u8*)stage_mem);
}

static const void* persistent_kernel(int deg, bool bf16)
{
    switch (deg * 2 + (bf16 ? 1 : 0)) {
    case 0: return reinterpret_cast<const void*>(&k_serve_persistent<0, false>);
    case 1: return reinterpret_cast<const void*>(&k_serve_persistent<0, true>);
    case 2: return reinterpret_cast<const void*>(&k_serve_persistent<1, false>);
    case 3: return reinterpret_cast<const void*>(&k_serve_persistent<1, true>);
    case 4: return reinterpret_cast<const void*>(&k_serve_persistent<2, false>);
    case 5: return reinterpret_cast<const void*>(&k_serve_persistent<2, true>);
    case 6: return reinterpret_cast<const void*>(&k_serve_persistent<3, false>);
    case 7: return reinterpret_cast<const void*>(&k_serve_persistent<3, true>);
    }
    return nullptr;
}

static hipError_t launch_persistent(int deg, bool bf16, const PersistArgs& a, int blocks, hipStream_t stream)
{
    const void* f = persistent_kernel(deg, bf16);
    if (!f || blocks < 2) return hipErrorInvalidValue;
    PersistArgs args = a;
    void* params[] = {&args};
    return hipLaunchKernel(f, dim3((unsigned)blocks), dim3(kWave), params, 0, stream);
}

__global__ void k_clear_stop(sp::DevCtl* d) { __hip_atomic_store(&d->stop, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

static hipError_t launch_clear_stop(sp::DevCtl* d, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_stop, dim3(1), dim3(1), 0, stream, d);
    return hipGetLastError();
}

// Blocks of the persistent grid: as many one-wavefront blocks as the device
// holds at once (so the dispatcher and every worker are resident together).
static hipError_t persistent_blocks(int deg, bool bf16, int device, int* blocks)
{
    const void* f = persistent_kernel(deg, bf16);
    if (!f) return hipErrorInvalidValue;
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kWave, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    *blocks = std::max(2, std::min(per_cu * cus, 8192));
    return hipSuccess;
}

}  // namespace rf

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct rf_server {
    rf_packed_scene scene;
    rf_params params;
    rf_bound bound;
    int device = 0;
    hipStream_t stream = nullptr;
    float* pool = nullptr;               // pinned host, W*H*4 floats per request
    size_t pool_floats = 0;
    rf::ReqRecord* dev_reqs = nullptr;    // device table
    rf::ReqRecord* host_reqs = nullptr;   // pinned staging of the table
    int32_t* dev_grid = nullptr;          // located seed cells of a kSeedGrid^3 grid over the bound
    float grid_lo[3] = {0, 0, 0}, grid_inv[3] = {0, 0, 0};
    uint32_t* dev_desc[rf::kLaunchesInFlight] = {nullptr, nullptr};
    uint32_t* host_desc[rf::kLaunchesInFlight] = {nullptr, nullptr};
    hipEvent_t done_ev[rf::kLaunchesInFlight] = {nullptr, nullptr};
    int max_inflight = 0;
    // persistent form (mode RF_SERVE_PERSISTENT)
    int mode = RF_SERVE_LAUNCHES;
    rf::sp::HostCtl* hctl = nullptr;  // coherent pinned host memory
    rf::sp::DevCtl* dctl = nullptr;
    hipEvent_t pk_ev = nullptr;       // completion of the running persistent launch
    bool pk_running = false;
    int pk_blocks = 0;
    int64_t written = 0;              // records written into the host ring
    uint64_t idle_ticks = 0, hard_ticks = 0;
    std::chrono::steady_clock::time_point stop_deadline;  // destroy stops waiting for admitted requests then

    enum State { FREE = 0, QUEUED, DONE, COPYING };  // COPYING: its result is being copied out
    struct Slot {
        State state = FREE;
        bool uploaded = false;
        uint64_t seq = 0;
        int64_t offset = 0, floats = 0;
        int32_t width = 0, height = 0;
        int64_t n_tiles = 0, issued = 0, retired = 0;
    };
    struct Launch {
        bool busy = false;
        std::vector<std::pair<int, int64_t>> parts;  // (slot, tiles)
    };

    std::mutex mu;
    std::condition_variable cv;
    std::vector<Slot> slots;
    std::deque<int> fifo;                      // admitted slots with tiles not yet issued, oldest first
    Launch launches[rf::kLaunchesInFlight];
    int next_launch = 0;
    std::map<int64_t, int64_t> free_ranges;    // pool offset -> length (floats), coalesced
    uint64_t next_seq = 1;
    rf_server_stats stats{};
    std::thread worker;
    bool stop = false;
    rf_status worker_status = RF_OK;
    char worker_err[256] = "";
};

namespace {

thread_local char g_serr[512] = "";

rf_status sfail(rf_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_serr, sizeof g_serr, fmt, ap);
    va_end(ap);
    rf::set_error(g_serr);
    return st;
}

bool pool_alloc(rf_server* s, int64_t n, int64_t* off)
{
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
        if (it->second >= n) {
            *off = it->first;
            const int64_t rest = it->second - n;
            const int64_t start = it->first + n;
            s->free_ranges.erase(it);
            if (rest > 0) s->free_ranges[start] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(rf_server* s, int64_t off, int64_t n)
{
    auto next = s->free_ranges.lower_bound(off);
    if (next != s->free_ranges.end() && off + n == next->first) {
        n += next->second;
        next = s->free_ranges.erase(next);
    }
    if (next != s->free_ranges.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += n;
            return;
        }
    }
    s->free_ranges[off] = n;
}

// Retires finished launches. Called with the lock held.
void retire(rf_server* s)
{
    for (int b = 0; b < rf::kLaunchesInFlight; ++b) {
        rf_server::Launch& L = s->launches[b];
        if (!L.busy) continue;
        const hipError_t q = hipEventQuery(s->done_ev[b]);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess && s->worker_status == RF_OK) {
            s->worker_status = RF_ERR_HIP;
            snprintf(s->worker_err, sizeof s->worker_err, "server launch failed: %s", hipGetErrorString(q));
        }
        for (auto& part : L.parts) {
            rf_server::Slot& sl = s->slots[part.first];
            sl.retired += part.second;
            if (sl.retired == sl.n_tiles && sl.state == rf_server::QUEUED) {
                sl.state = rf_server::DONE;
                s->stats.completed++;
                s->stats.rays_done += (int64_t)sl.width * sl.height;
            }
        }
        L.parts.clear();
        L.busy = false;
    }
}

rf::SceneView scene_view(const rf_server* s)
{
    rf::SceneView v;
    const unsigned char* base = static_cast<const unsigned char*>(s->scene.base);
    v.planes = reinterpret_cast<const float4*>(base + s->scene.off_planes);
    v.adj = reinterpret_cast<const uint2*>(base + s->scene.off_adj);
    v.row = reinterpret_cast<const uint2*>(base + s->scene.off_row);
    v.rec = base + s->scene.off_rec;
    v.n_sites = s->scene.n_sites;
    v.n_edges = s->scene.n_edges;
    return v;
}

rf::LocateArgs locate_args(const rf_server* s)
{
    rf::LocateArgs a;
    memset(&a, 0, sizeof a);
    a.s = scene_view(s);
    a.max_steps = 1 << 20;
    a.grid_n = rf::kSeedGrid;
    for (int k = 0; k < 3; ++k) {
        a.grid_lo[k] = s->grid_lo[k];
        a.grid_inv[k] = s->grid_inv[k];
    }
    return a;
}

// Builds and enqueues one launch from the pending tiles, oldest request first.
// Called with the lock held; returns false if there was nothing to launch.
bool launch_next(rf_server* s)
{
    const int b = s->next_launch;
    rf_server::Launch& L = s->launches[b];
    if (L.busy || s->fifo.empty()) return false;
    hipError_t e = hipSuccess;
    // request records not yet on the device
    for (int slot : s->fifo) {
        rf_server::Slot& sl = s->slots[slot];
        if (!sl.uploaded && e == hipSuccess) {
            e = hipMemcpyAsync(&s->dev_reqs[slot], &s->host_reqs[slot], sizeof(rf::ReqRecord),
                               hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess && s->host_reqs[slot].start < 0) {
                // the camera's cell, located on the device into the record
                rf::LocateArgs la = locate_args(s);
                la.points = s->dev_reqs[slot].pos;
                la.n_points = 1;
                la.cells = &s->dev_reqs[slot].start;
                la.grid = s->dev_grid;
                e = rf::launch_locate(s->scene.sh_degree, s->scene.attr_dtype == RF_BF16, la, s->stream);
            }
            sl.uploaded = true;
        }
    }
    int n = 0;
    while (!s->fifo.empty() && n < rf::kMaxBatchTiles) {
        const int slot = s->fifo.front();
        rf_server::Slot& sl = s->slots[slot];
        const int64_t take = std::min<int64_t>(sl.n_tiles - sl.issued, rf::kMaxBatchTiles - n);
        for (int64_t k = 0; k < take; ++k)
            s->host_desc[b][n + k] = ((uint32_t)slot << rf::kLocalTileBits) | (uint32_t)(sl.issued + k);
        L.parts.emplace_back(slot, take);
        sl.issued += take;
        n += (int)take;
        if (sl.issued == sl.n_tiles) s->fifo.pop_front();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->dev_desc[b], s->host_desc[b], sizeof(uint32_t) * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        rf::BatchArgs a;
        a.s = scene_view(s);
        a.eps = s->params.eps;
        a.max_steps = s->params.max_steps;
        a.bound_kind = s->bound.kind;
        for (int k = 0; k < 6; ++k) a.bound[k] = s->bound.p[k];
        a.reqs = s->dev_reqs;
        a.desc = s->dev_desc[b];
        a.n_tiles = n;
        a.pool = s->pool;
        e = rf::launch_batch(s->scene.sh_degree, s->scene.attr_dtype == RF_BF16, a, s->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(s->done_ev[b], s->stream);
    if (e != hipSuccess && s->worker_status == RF_OK) {
        s->worker_status = RF_ERR_HIP;
        snprintf(s->worker_err, sizeof s->worker_err, "server launch: %s", hipGetErrorString(e));
    }
    L.busy = true;  // retired through its event (or the error path) like any launch
    s->next_launch = (b + 1) % rf::kLaunchesInFlight;
    s->stats.launches++;
    return true;
}

// Persistent form: marks the requests whose completion word shows their
// sequence number done, and relaunches the kernel when requests wait and no
// launch is running. Called with the lock held.
void persistent_step(rf_server* s)
{
    for (int k = 0; k < s->max_inflight; ++k) {
        rf_server::Slot& sl = s->slots[k];
        if (sl.state != rf_server::QUEUED) continue;
        if (__atomic_load_n(&s->hctl->done_seq[k], __ATOMIC_ACQUIRE) == sl.seq) {
            sl.state = rf_server::DONE;
            sl.retired = sl.n_tiles;
            s->stats.completed++;
            s->stats.rays_done += (int64_t)sl.width * sl.height;
        }
    }
    if (s->pk_running) {
        const hipError_t q = hipEventQuery(s->pk_ev);
        if (q == hipErrorNotReady) return;
        s->pk_running = false;
        if (q != hipSuccess && s->worker_status == RF_OK) {
            s->worker_status = RF_ERR_HIP;
            snprintf(s->worker_err, sizeof s->worker_err, "persistent launch failed: %s", hipGetErrorString(q));
            return;
        }
    }
    const int64_t consumed = __atomic_load_n(&s->hctl->consumed, __ATOMIC_ACQUIRE);
    if (consumed >= s->written || s->worker_status != RF_OK) return;
    rf::PersistArgs a;
    memset(&a, 0, sizeof a);
    a.s = scene_view(s);
    a.eps = s->params.eps;
    a.max_steps = s->params.max_steps;
    a.bound_kind = s->bound.kind;
    for (int k = 0; k < 6; ++k) a.bound[k] = s->bound.p[k];
    a.host = s->hctl;
    a.dev = s->dctl;
    a.pool = s->pool;
    a.grid = s->dev_grid;
    a.grid_n = rf::kSeedGrid;
    for (int k = 0; k < 3; ++k) {
        a.grid_lo[k] = s->grid_lo[k];
        a.grid_inv[k] = s->grid_inv[k];
    }
    a.consumed0 = consumed;
    a.idle_ticks = s->idle_ticks;
    a.hard_ticks = s->hard_ticks;
    // the previous launch's stop flag is cleared by a small kernel (no memset node), then the launch
    hipError_t e = rf::launch_clear_stop(s->dctl, s->stream);
    if (e == hipSuccess)
        e = rf::launch_persistent(s->scene.sh_degree, s->scene.attr_dtype == RF_BF16, a, s->pk_blocks, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->pk_ev, s->stream);
    if (e != hipSuccess) {
        s->worker_status = RF_ERR_HIP;
        snprintf(s->worker_err, sizeof s->worker_err, "persistent launch: %s", hipGetErrorString(e));
        return;
    }
    s->pk_running = true;
    s->stats.launches++;
}

void scheduler_persistent(rf_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        persistent_step(s);
        bool queued = false;
        for (int k = 0; k < s->max_inflight; ++k) queued |= s->slots[k].state == rf_server::QUEUED;
        if (s->stop && (!queued || s->worker_status != RF_OK || std::chrono::steady_clock::now() > s->stop_deadline))
            break;
        // completions are polled every 20 us while requests are queued
        s->cv.wait_for(lock, std::chrono::microseconds(queued ? 20 : 2000));
    }
}

void scheduler(rf_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        retire(s);
        bool launched = false;
        while (s->worker_status == RF_OK && launch_next(s)) launched = true;
        bool busy = false;
        for (auto& L : s->launches) busy |= L.busy;
        if (s->stop && !busy && (s->fifo.empty() || s->worker_status != RF_OK)) break;
        if (!launched) {
            // wake on new work, or poll the launch events every 50 us
            s->cv.wait_for(lock, std::chrono::microseconds(busy ? 50 : 2000));
        }
    }
}

// The seed grid: cell centres of a kSeedGrid^3 grid over the bound's box,
// each located once from cell 0; a request's camera cell is then located from
// the grid cell that contains the camera, a few steps away.
hipError_t build_seed_grid(rf_server* s)
{
    constexpr int G = rf::kSeedGrid;
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = s->bound.kind == 0 ? s->bound.p[k] : -s->bound.p[0];
        hi[k] = s->bound.kind == 0 ? s->bound.p[3 + k] : s->bound.p[0];
        s->grid_lo[k] = lo[k];
        s->grid_inv[k] = hi[k] > lo[k] ? (float)G / (hi[k] - lo[k]) : 0.0f;
    }
    std::vector<float> pts((size_t)G * G * G * 3);
    for (int z = 0; z < G; ++z)
        for (int y = 0; y < G; ++y)
            for (int x = 0; x < G; ++x) {
                const int c[3] = {x, y, z};
                float* p = &pts[(((size_t)z * G + y) * G + x) * 3];
                for (int k = 0; k < 3; ++k) p[k] = lo[k] + (c[k] + 0.5f) * (hi[k] - lo[k]) / G;
            }
    float* dev_pts = nullptr;
    hipError_t e = hipMalloc((void**)&s->dev_grid, sizeof(int32_t) * G * G * G);
    if (e == hipSuccess) e = hipMalloc((void**)&dev_pts, sizeof(float) * pts.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(dev_pts, pts.data(), sizeof(float) * pts.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        rf::LocateArgs a = locate_args(s);
        a.points = dev_pts;
        a.n_points = (int64_t)G * G * G;
        a.cells = s->dev_grid;
        a.grid = nullptr;  // from cell 0
        e = rf::launch_locate(s->scene.sh_degree, s->scene.attr_dtype == RF_BF16, a, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (dev_pts) (void)hipFree(dev_pts);
    return e;
}

void release(rf_server* s)
{
    if (s->pk_ev) (void)hipEventDestroy(s->pk_ev);
    if (s->dctl) (void)hipFree(s->dctl);
    if (s->hctl) (void)hipHostFree(s->hctl);
    for (int b = 0; b < rf::kLaunchesInFlight; ++b) {
        if (s->done_ev[b]) (void)hipEventDestroy(s->done_ev[b]);
        if (s->dev_desc[b]) (void)hipFree(s->dev_desc[b]);
        if (s->host_desc[b]) (void)hipHostFree(s->host_desc[b]);
    }
    if (s->dev_reqs) (void)hipFree(s->dev_reqs);
    if (s->dev_grid) (void)hipFree(s->dev_grid);
    if (s->host_reqs) (void)hipHostFree(s->host_reqs);
    if (s->pool) (void)hipHostFree(s->pool);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

}  // namespace

extern "C" {

rf_status rf_server_create(const rf_packed_scene* scene, const rf_params* params, const rf_bound* bound,
                           size_t pool_bytes, int32_t max_inflight, rf_server** out)
{
    return rf_server_create_mode(scene, params, bound, pool_bytes, max_inflight, RF_SERVE_LAUNCHES, out);
}

rf_status rf_server_create_mode(const rf_packed_scene* scene, const rf_params* params, const rf_bound* bound,
                                size_t pool_bytes, int32_t max_inflight, int32_t mode, rf_server** out)
{
    if (mode != RF_SERVE_LAUNCHES && mode != RF_SERVE_PERSISTENT)
        return sfail(RF_ERR_INVALID_ARG, "mode must be RF_SERVE_LAUNCHES or RF_SERVE_PERSISTENT");
    if (!scene || !params || !bound || !out) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!scene->base || scene->sh_degree < 0 || scene->sh_degree > 3 || scene->n_sites < 1)
        return sfail(RF_ERR_INVALID_ARG, "invalid packed scene");
    if (!(params->eps >= 0.0f) || params->max_steps < 1) return sfail(RF_ERR_INVALID_ARG, "invalid params");
    if (bound->kind != 0 && bound->kind != 1) return sfail(RF_ERR_INVALID_ARG, "bound kind must be 0 or 1");
    if (max_inflight < 1 || max_inflight > rf::kMaxSlots)
        return sfail(RF_ERR_INVALID_ARG, "max_inflight must be in [1, %d]", rf::kMaxSlots);
    if (pool_bytes < 1024 || pool_bytes > ((size_t)1 << 36))
        return sfail(RF_ERR_INVALID_ARG, "pool_bytes must be in [1024, 2^36]");
    rf_server* s = new (std::nothrow) rf_server();
    if (!s) return sfail(RF_ERR_OOM, "host allocation failed");
    s->scene = *scene;
    s->params = *params;
    s->bound = *bound;
    s->max_inflight = max_inflight;
    s->mode = mode;
    s->slots.resize(max_inflight);
    s->pool_floats = pool_bytes / 16 * 4;
    s->free_ranges[0] = (int64_t)s->pool_floats;
    s->stats.pool_bytes = (int64_t)(s->pool_floats * 4);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->pool, s->pool_floats * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s->dev_reqs, sizeof(rf::ReqRecord) * rf::kMaxSlots);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->host_reqs, sizeof(rf::ReqRecord) * rf::kMaxSlots, hipHostMallocDefault);
    for (int b = 0; b < rf::kLaunchesInFlight && e == hipSuccess; ++b) {
        e = hipMalloc((void**)&s->dev_desc[b], sizeof(uint32_t) * rf::kMaxBatchTiles);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&s->host_desc[b], sizeof(uint32_t) * rf::kMaxBatchTiles, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done_ev[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = build_seed_grid(s);
    if (e == hipSuccess && mode == RF_SERVE_PERSISTENT) {
        e = hipHostMalloc((void**)&s->hctl, sizeof(rf::sp::HostCtl), hipHostMallocCoherent);
        if (e == hipSuccess) {
            memset(s->hctl, 0, sizeof(rf::sp::HostCtl));
            e = hipMalloc((void**)&s->dctl, sizeof(rf::sp::DevCtl));
        }
        if (e == hipSuccess) e = hipMemset(s->dctl, 0, sizeof(rf::sp::DevCtl));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->pk_ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = rf::persistent_blocks(s->scene.sh_degree, s->scene.attr_dtype == RF_BF16, s->device, &s->pk_blocks);
        int khz = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device);
        if (e == hipSuccess && khz <= 0) e = hipErrorInvalidValue;
        // leave 2 ms after the last request once everything is done; 1 s without requests at most
        s->idle_ticks = (uint64_t)khz * 2;
        s->hard_ticks = (uint64_t)khz * 1000;
    }
    if (e != hipSuccess) {
        release(s);
        delete s;
        return sfail(e == hipErrorOutOfMemory ? RF_ERR_OOM : RF_ERR_HIP, "server allocation: %s", hipGetErrorString(e));
    }
    try {
        s->worker = std::thread(mode == RF_SERVE_PERSISTENT ? scheduler_persistent : scheduler, s);
    } catch (...) {
        release(s);
        delete s;
        return sfail(RF_ERR_OOM, "could not start the scheduler thread");
    }
    *out = s;
    return RF_OK;
}

rf_status rf_server_submit(rf_server* s, const rf_camera* cam, int32_t start_cell, uint64_t* req_id)
{
    if (!s || !cam || !req_id) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    if (cam->width <= 0 || cam->height <= 0 || !rf::camera_fov_ok(cam->model, cam->fov_deg))
        return sfail(RF_ERR_INVALID_ARG, "invalid camera");
    const int64_t pixels = (int64_t)cam->width * cam->height;
    const int64_t n_tiles = (int64_t)((cam->width + 7) / 8) * ((cam->height + 7) / 8);
    if (n_tiles >= ((int64_t)1 << rf::kLocalTileBits) || pixels * 4 > (int64_t)s->pool_floats)
        return sfail(RF_ERR_UNSUPPORTED, "image of %d x %d does not fit the server", cam->width, cam->height);
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->worker_status != RF_OK) return sfail(s->worker_status, "%s", s->worker_err);
    int slot = -1;
    for (int k = 0; k < s->max_inflight; ++k)
        if (s->slots[k].state == rf_server::FREE) {
            slot = k;
            break;
        }
    int64_t off = 0;
    if (slot < 0 || !pool_alloc(s, pixels * 4, &off)) {
        s->stats.rejected_busy++;
        return sfail(RF_ERR_BUSY, slot < 0 ? "no free request slot" : "output pool full");
    }
    rf_server::Slot& sl = s->slots[slot];
    sl.state = rf_server::QUEUED;
    sl.uploaded = false;
    sl.seq = s->next_seq++;
    sl.offset = off;
    sl.floats = pixels * 4;
    sl.width = cam->width;
    sl.height = cam->height;
    sl.n_tiles = n_tiles;
    sl.issued = 0;
    sl.retired = 0;
    rf::ReqRecord& r = s->host_reqs[slot];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) r.rot[3 * i + j] = cam->pose[4 * i + j];
        r.pos[i] = cam->pose[4 * i + 3];
    }
    r.model = cam->model;
    r.focal = rf::camera_focal(cam->model, cam->fov_deg, cam->width);
    r.width = cam->width;
    r.height = cam->height;
    r.start = start_cell;
    r.out_offset = off;
    if (s->mode == RF_SERVE_PERSISTENT) {
        rf::sp::Req q;
        memset(&q, 0, sizeof q);
        memcpy(q.rot, r.rot, sizeof q.rot);
        memcpy(q.pos, r.pos, sizeof q.pos);
        q.model = r.model;
        q.focal = r.focal;
        q.width = r.width;
        q.height = r.height;
        q.start = r.start;
        q.slot = slot;
        q.out_offset_lo = (int32_t)(uint32_t)((uint64_t)off & 0xffffffffu);
        q.out_offset_hi = (int32_t)(uint32_t)((uint64_t)off >> 32);
        q.seq_lo = (uint32_t)sl.seq;
        q.seq_hi = (uint32_t)(sl.seq >> 32);
        q.gen = (uint32_t)(1 + (sl.seq - 1) % 0xfffffffeull);  // nonzero, differs between a slot's requests
        q.n_tiles = (int32_t)n_tiles;
        // the record, then its count (the dispatcher reads the record after acquiring the count)
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s->hctl->ring[s->written % rf::sp::kReqRing]);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&q);
        for (int k = 0; k < rf::sp::kReqWords; ++k) __atomic_store_n(dst + k, src[k], __ATOMIC_RELAXED);
        ++s->written;
        __atomic_store_n(&s->hctl->n_requests, s->written, __ATOMIC_RELEASE);
    } else {
        s->fifo.push_back(slot);
    }
    s->stats.submitted++;
    s->stats.inflight++;
    s->stats.pool_used_bytes += pixels * 16;
    *req_id = sl.seq;
    s->cv.notify_one();
    return RF_OK;
}

rf_status rf_server_poll(rf_server* s, uint64_t* done_ids, int32_t cap, int32_t* n_done)
{
    if (!s || !n_done || (cap > 0 && !done_ids)) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->worker_status != RF_OK) return sfail(s->worker_status, "%s", s->worker_err);
    int n = 0;
    for (int k = 0; k < s->max_inflight && n < cap; ++k)
        if (s->slots[k].state == rf_server::DONE) done_ids[n++] = s->slots[k].seq;
    *n_done = n;
    return RF_OK;
}

// The copy runs outside the server's lock (a 1080p result is 33 MB): the
// slot is marked COPYING, which keeps it and its pool range out of every
// other call's reach, and freed afterwards, so the scheduler keeps launching
// and observing completions while a result is copied.
rf_status rf_server_result(rf_server* s, uint64_t req_id, float* rgba, size_t bytes)
{
    if (!s) return sfail(RF_ERR_INVALID_ARG, "NULL server");
    rf_server::Slot* sl = nullptr;
    size_t need = 0;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        for (int k = 0; k < s->max_inflight && !sl; ++k) {
            rf_server::Slot& c = s->slots[k];
            if (c.state == rf_server::FREE || c.seq != req_id) continue;
            if (c.state == rf_server::COPYING)
                return sfail(RF_ERR_BUSY, "request %llu is being collected", (unsigned long long)req_id);
            if (c.state != rf_server::DONE)
                return sfail(RF_ERR_BUSY, "request %llu not finished", (unsigned long long)req_id);
            need = (size_t)c.floats * 4;
            if (rgba && bytes < need)
                return sfail(RF_ERR_INVALID_ARG, "result buffer of %zu bytes < %zu", bytes, need);
            c.state = rf_server::COPYING;
            sl = &c;
        }
        if (!sl) return sfail(RF_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)req_id);
    }
    if (rgba) memcpy(rgba, s->pool + sl->offset, need);
    std::lock_guard<std::mutex> lock(s->mu);
    pool_free(s, sl->offset, sl->floats);
    s->stats.pool_used_bytes -= (int64_t)need;
    s->stats.inflight--;
    sl->state = rf_server::FREE;
    return RF_OK;
}

rf_status rf_server_stats_get(rf_server* s, rf_server_stats* out)
{
    if (!s || !out) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    return RF_OK;
}

rf_status rf_server_destroy(rf_server* s)
{
    if (!s) return RF_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->stop_deadline = std::chrono::steady_clock::now() + std::chrono::seconds(60);
        s->cv.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();  // finishes admitted requests, then returns
    if (s->mode == RF_SERVE_PERSISTENT) {
        // ask the running launch to leave, and wait for it a bounded time (it
        // leaves by itself within about a second of idling in any case)
        __atomic_store_n(&s->hctl->shutdown, 1, __ATOMIC_RELEASE);
        const auto until = std::chrono::steady_clock::now() + std::chrono::seconds(30);
        while (s->pk_running && hipEventQuery(s->pk_ev) == hipErrorNotReady) {
            if (std::chrono::steady_clock::now() > until) {
                // the launch still runs: keep its memory (leak it) rather than free it under the kernel
                sfail(RF_ERR_HIP, "persistent server kernel did not stop within 30 s");
                return RF_ERR_HIP;
            }
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        }
    }
    const hipError_t e = hipStreamSynchronize(s->stream);
    rf_status st = s->worker_status;
    if (st != RF_OK)
        sfail(st, "%s", s->worker_err);
    else if (e != hipSuccess)
        st = sfail(RF_ERR_HIP, "server stream: %s", hipGetErrorString(e));
    release(s);
    delete s;
    return st;
}

}  // extern "C"
