// Continuous-batching render server: one persistent kernel keeps the packed
// scene resident and renders 8x8 screen tiles of every admitted request.
//
// Host -> device: the host writes a request record (camera, image size, start
// cell, output offset) into a ring in pinned host memory and bumps a counter.
// One dispatcher wavefront polls that counter, copies each new record into
// the request's slot in device memory, appends the request's tile
// descriptors to a device tile ring and publishes the new tile count.
//
// Workers: every other wavefront takes a ticket (a global tile number) from a
// device counter, waits until that tile is published, renders the tile's 64
// pixels with the same ray generation and forward walk as the batch kernels,
// writes RGBA (colour, final transmittance) straight into the request's
// region of a pinned host output pool, and counts the tile done. The last
// tile of a request writes the request's sequence number into a pinned
// completion word, which the host polls.
//
// Every wave exits when the host raises the shutdown flag (tickets taken after
// it are abandoned); no wave waits on anything else. A host thread bumps a
// heartbeat word every 20 ms; if the dispatcher sees no heartbeat for the
// watchdog period (5 s) it raises the shutdown flag itself, so the grid drains
// even if the host stops responding.
//
// The control block and the output pool are coherent (fine-grained) pinned
// host memory: with the default (non-coherent) pinned memory a running kernel
// is not guaranteed to observe host writes, nor the host the kernel's.

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <iterator>
#include <thread>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "radfoam.h"
#include "rf_device.hpp"
#include "rf_kernels.hpp"
#include "rf_walk.hpp"

namespace rf {

constexpr int kMaxSlots = 64;                 // in-flight requests
constexpr int kHostRing = 128;                // request records in the host ring (>= kMaxSlots)
constexpr int64_t kTileRing = 1 << 22;        // tile descriptors in flight (>= pool pixels / 64)
constexpr int kLocalTileBits = 25;            // descriptor = slot << 25 | tile within the request

struct ReqRecord {
    float rot[9];
    float pos[3];
    float focal;
    int32_t width, height, start;
    int32_t n_tiles, slot;
    int64_t out_offset;  // in floats from the pool base
    uint64_t seq;        // 1-based request sequence number
};

struct HostCtl {  // coherent pinned host memory
    int64_t written;    // records written into the ring (host)
    int64_t heartbeat;  // bumped by the host's heartbeat thread
    int32_t shutdown;   // set by the host
    int32_t stopped;    // set by the dispatcher: 1 on shutdown, 2 when the watchdog fired
    uint64_t done_seq[kMaxSlots];  // written by the device when a request completes
    ReqRecord ring[kHostRing];
};

struct DevCtl {  // device memory
    int64_t tile_cursor;
    int64_t tiles_published;
    uint64_t dispatcher_tick;  // wall clock of the dispatcher's last loop (0: not started)
    int32_t shutdown;
    int32_t pad;
    int32_t tiles_done[kMaxSlots];
    ReqRecord slots[kMaxSlots];
};

struct ServeArgs {
    SceneView s;
    uint64_t watchdog_ticks;  // wall-clock ticks without a heartbeat before the kernel stops itself
    float eps;
    int32_t max_steps;
    int32_t bound_kind;
    float bound[6];
    HostCtl* host;
    DevCtl* dev;
    uint32_t* tiles;
    float* pool;
};

__device__ inline int64_t sys_load(const int64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline int32_t sys_load32(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ void stop_all(const ServeArgs& a, int lane, int why)
{
    if (lane == 0) {
        __hip_atomic_store(&a.dev->shutdown, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.host->stopped, why, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__device__ void dispatcher(const ServeArgs& a, int lane)
{
    int64_t consumed = 0, tiles_pub = 0;
    int64_t beat = sys_load(&a.host->heartbeat);
    uint64_t beat_time = wall_clock64();
    for (;;) {
        const int64_t b = sys_load(&a.host->heartbeat);
        const uint64_t now = wall_clock64();
        if (lane == 0) __hip_atomic_store(&a.dev->dispatcher_tick, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (b != beat) {
            beat = b;
            beat_time = now;
        } else if (now - beat_time > a.watchdog_ticks) {
            stop_all(a, lane, 2);
            return;
        }
        const int64_t written = sys_load(&a.host->written);
        bool published = false;
        while (consumed < written) {
            // the record, one word per lane, read with system-scope loads (host memory)
            constexpr int kWords = (int)(sizeof(ReqRecord) / 4);
            static_assert(kWords <= kWave, "record must fit one word per lane");
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&a.host->ring[consumed % kHostRing]);
            uint32_t word = 0;
            if (lane < kWords) word = __hip_atomic_load(src + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const int n_tiles = __shfl((int)word, (int)(offsetof(ReqRecord, n_tiles) / 4));
            const int slot = __shfl((int)word, (int)(offsetof(ReqRecord, slot) / 4));
            uint32_t* dst = reinterpret_cast<uint32_t*>(&a.dev->slots[slot]);
            if (lane < kWords) dst[lane] = word;
            if (lane == 0) a.dev->tiles_done[slot] = 0;
            for (int k = lane; k < n_tiles; k += kWave)
                a.tiles[(tiles_pub + k) % kTileRing] = ((uint32_t)slot << kLocalTileBits) | (uint32_t)k;
            tiles_pub += n_tiles;
            ++consumed;
            published = true;
        }
        if (published) {
            // slot records and tile descriptors before the new tile count
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) __hip_atomic_store(&a.dev->tiles_published, tiles_pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (sys_load32(&a.host->shutdown)) {
            stop_all(a, lane, 1);
            return;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

template <int DEG, bool BF16>
__global__ __launch_bounds__(kBlock) void k_serve(ServeArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    if (blockIdx.x == 0 && wave == 0) {
        dispatcher(a, lane);
        return;
    }
    const uint64_t born = wall_clock64();
    for (;;) {
        int64_t t = 0;
        if (lane == 0) t = __hip_atomic_fetch_add(&a.dev->tile_cursor, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = __shfl(t, 0);
        bool stop = false;
        for (int polls = 0;; ++polls) {
            int64_t pub = 0;
            int32_t sd = 0;
            if (lane == 0) {
                pub = __hip_atomic_load(&a.dev->tiles_published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                sd = __hip_atomic_load(&a.dev->shutdown, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if ((polls & 1023) == 1023) {
                    // the dispatcher must show signs of life; otherwise leave
                    const uint64_t tick = __hip_atomic_load(&a.dev->dispatcher_tick, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t now = wall_clock64();
                    const uint64_t ref = tick ? tick : born;
                    if (now > ref && now - ref > 2 * a.watchdog_ticks) sd = 1;
                }
            }
            pub = __shfl(pub, 0);
            sd = __shfl(sd, 0);
            if (sd) {
                stop = true;
                break;
            }
            if (t < pub) break;
            __builtin_amdgcn_s_sleep(20);  // ~1 us between polls of the tile count
        }
        if (stop) return;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint32_t desc = __hip_atomic_load(&a.tiles[t % kTileRing], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int slot = (int)(desc >> kLocalTileBits);
        const int local = (int)(desc & ((1u << kLocalTileBits) - 1));
        const ReqRecord& rq = a.dev->slots[slot];
        const int W = rq.width, H = rq.height;
        const int tiles_x = (W + 7) / 8;
        const int px = (local % tiles_x) * 8 + (lane & 7);
        const int py = (local / tiles_x) * 8 + (lane >> 3);
        if (px < W && py < H) {
            float d[3], tmax;
            camera_ray(rq.rot, rq.pos, rq.focal, W, H, px, py, a.bound_kind, a.bound, d, &tmax);
            RayResult res;
            walk_forward<DEG, BF16, false>(a.s, rq.pos[0], rq.pos[1], rq.pos[2], d[0], d[1], d[2], tmax, rq.start,
                                           a.eps, a.max_steps, nullptr, nullptr, 0, res);
            float4* out = reinterpret_cast<float4*>(a.pool + rq.out_offset) + ((int64_t)py * W + px);
            *out = make_float4(res.C[0], res.C[1], res.C[2], res.T);
        }
        // make this tile's pixels visible to the host before counting it done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            const int done = __hip_atomic_fetch_add(&a.dev->tiles_done[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM) + 1;
            if (done == rq.n_tiles)
                __hip_atomic_store(&a.host->done_seq[slot], rq.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

template <int DEG, bool BF16>
static hipError_t launch_serve_t(const ServeArgs& a, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((k_serve<DEG, BF16>), dim3(blocks), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

static hipError_t launch_serve(int deg, bool bf16, const ServeArgs& a, int blocks, hipStream_t stream)
{
    switch (deg * 2 + (bf16 ? 1 : 0)) {
    case 0: return launch_serve_t<0, false>(a, blocks, stream);
    case 1: return launch_serve_t<0, true>(a, blocks, stream);
    case 2: return launch_serve_t<1, false>(a, blocks, stream);
    case 3: return launch_serve_t<1, true>(a, blocks, stream);
    case 4: return launch_serve_t<2, false>(a, blocks, stream);
    case 5: return launch_serve_t<2, true>(a, blocks, stream);
    case 6: return launch_serve_t<3, false>(a, blocks, stream);
    case 7: return launch_serve_t<3, true>(a, blocks, stream);
    }
    return hipErrorInvalidValue;
}

static hipError_t serve_occupancy(int deg, bool bf16, int* blocks_per_cu)
{
    const void* f = nullptr;
    switch (deg * 2 + (bf16 ? 1 : 0)) {
    case 0: f = (const void*)k_serve<0, false>; break;
    case 1: f = (const void*)k_serve<0, true>; break;
    case 2: f = (const void*)k_serve<1, false>; break;
    case 3: f = (const void*)k_serve<1, true>; break;
    case 4: f = (const void*)k_serve<2, false>; break;
    case 5: f = (const void*)k_serve<2, true>; break;
    case 6: f = (const void*)k_serve<3, false>; break;
    case 7: f = (const void*)k_serve<3, true>; break;
    default: return hipErrorInvalidValue;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, kBlock, 0);
}

}  // namespace rf

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct rf_server {
    rf_packed_scene scene;
    rf_params params;
    rf_bound bound;
    hipStream_t stream = nullptr;
    rf::HostCtl* host = nullptr;
    rf::DevCtl* dev = nullptr;
    uint32_t* tiles = nullptr;
    float* pool = nullptr;
    size_t pool_floats = 0;
    int max_inflight = 0;
    int blocks = 0;
    bool running = false;
    std::mutex mu;
    struct Slot {
        bool busy = false;
        bool done = false;
        uint64_t seq = 0;
        int64_t offset = 0;  // floats
        int64_t floats = 0;
        int32_t width = 0, height = 0;
        int64_t tiles = 0;
    };
    std::vector<Slot> slots;
    std::map<int64_t, int64_t> free_ranges;  // offset -> length (floats), coalesced
    uint64_t next_seq = 1;
    int64_t tiles_inflight = 0;
    std::thread heartbeat;
    std::atomic<bool> heartbeat_stop{false};
    rf_server_stats stats{};
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

void stop_heartbeat(rf_server* s)
{
    if (s->heartbeat.joinable()) {
        s->heartbeat_stop.store(true);
        s->heartbeat.join();
    }
}

void release(rf_server* s)
{
    stop_heartbeat(s);
    if (s->host) (void)hipHostFree(s->host);
    if (s->pool) (void)hipHostFree(s->pool);
    if (s->dev) (void)hipFree(s->dev);
    if (s->tiles) (void)hipFree(s->tiles);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

void collect_done(rf_server* s)
{
    for (int k = 0; k < s->max_inflight; ++k) {
        rf_server::Slot& sl = s->slots[k];
        if (sl.busy && !sl.done) {
            const uint64_t v = __atomic_load_n(&s->host->done_seq[k], __ATOMIC_ACQUIRE);
            if (v == sl.seq) {
                sl.done = true;
                s->stats.completed++;
                s->stats.rays_done += (int64_t)sl.width * sl.height;
            }
        }
    }
}

}  // namespace

extern "C" {

rf_status rf_server_create(const rf_packed_scene* scene, const rf_params* params, const rf_bound* bound,
                           size_t pool_bytes, int32_t max_inflight, int32_t workgroups, rf_server** out)
{
    if (!scene || !params || !bound || !out) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!scene->base || scene->sh_degree < 0 || scene->sh_degree > 3)
        return sfail(RF_ERR_INVALID_ARG, "invalid packed scene");
    if (!(params->eps >= 0.0f) || params->max_steps < 1) return sfail(RF_ERR_INVALID_ARG, "invalid params");
    if (bound->kind != 0 && bound->kind != 1) return sfail(RF_ERR_INVALID_ARG, "bound kind must be 0 or 1");
    if (max_inflight < 1 || max_inflight > rf::kMaxSlots)
        return sfail(RF_ERR_INVALID_ARG, "max_inflight must be in [1, %d]", rf::kMaxSlots);
    const size_t max_pool = (size_t)rf::kTileRing * 64 * 16;
    if (pool_bytes < 16 * 64 || pool_bytes > max_pool)
        return sfail(RF_ERR_INVALID_ARG, "pool_bytes must be in [1024, %zu]", max_pool);
    rf_server* s = new (std::nothrow) rf_server();
    if (!s) return sfail(RF_ERR_OOM, "host allocation failed");
    s->scene = *scene;
    s->params = *params;
    s->bound = *bound;
    s->max_inflight = max_inflight;
    s->slots.resize(max_inflight);
    s->pool_floats = pool_bytes / 4 / 4 * 4;
    s->free_ranges[0] = (int64_t)s->pool_floats;
    s->stats.pool_bytes = (int64_t)(s->pool_floats * 4);
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->host, sizeof(rf::HostCtl), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->pool, s->pool_floats * 4, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipMalloc((void**)&s->dev, sizeof(rf::DevCtl));
    if (e == hipSuccess) e = hipMalloc((void**)&s->tiles, sizeof(uint32_t) * rf::kTileRing);
    if (e != hipSuccess) {
        release(s);
        delete s;
        return sfail(e == hipErrorOutOfMemory ? RF_ERR_OOM : RF_ERR_HIP, "server allocation: %s", hipGetErrorString(e));
    }
    memset(s->host, 0, sizeof(rf::HostCtl));
    e = hipMemsetAsync(s->dev, 0, sizeof(rf::DevCtl), s->stream);
    int per_cu = 0, dev_id = 0, n_cu = 0, clock_khz = 0;
    if (e == hipSuccess) e = rf::serve_occupancy(scene->sh_degree, scene->attr_dtype == RF_BF16, &per_cu);
    if (e == hipSuccess) e = hipGetDevice(&dev_id);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev_id);
    if (e == hipSuccess && clock_khz <= 0) e = hipErrorInvalidValue;
    if (e == hipSuccess) {
        // heartbeat: a host thread bumps the word the dispatcher watches
        rf::HostCtl* h = s->host;
        std::atomic<bool>* stop = &s->heartbeat_stop;
        s->heartbeat = std::thread([h, stop]() {
            int64_t k = 0;
            while (!stop->load()) {
                __atomic_store_n(&h->heartbeat, ++k, __ATOMIC_RELEASE);
                std::this_thread::sleep_for(std::chrono::milliseconds(20));
            }
        });
    }
    if (e == hipSuccess) {
        const int fill = per_cu * n_cu;
        s->blocks = workgroups > 0 ? (workgroups < fill ? workgroups : fill) : fill;
        if (s->blocks < 2) s->blocks = 2;
        rf::ServeArgs a;
        a.watchdog_ticks = (uint64_t)clock_khz * 1000ull * 5ull;
        const unsigned char* b = static_cast<const unsigned char*>(scene->base);
        a.s.planes = reinterpret_cast<const float4*>(b + scene->off_planes);
        a.s.adj = reinterpret_cast<const uint2*>(b + scene->off_adj);
        a.s.row = reinterpret_cast<const uint2*>(b + scene->off_row);
        a.s.rec = b + scene->off_rec;
        a.s.n_sites = scene->n_sites;
        a.s.n_edges = scene->n_edges;
        a.eps = params->eps;
        a.max_steps = params->max_steps;
        a.bound_kind = bound->kind;
        for (int k = 0; k < 6; ++k) a.bound[k] = bound->p[k];
        a.host = s->host;
        a.dev = s->dev;
        a.tiles = s->tiles;
        a.pool = s->pool;
        e = rf::launch_serve(scene->sh_degree, scene->attr_dtype == RF_BF16, a, s->blocks, s->stream);
    }
    if (e != hipSuccess) {
        if (s->host) __atomic_store_n(&s->host->shutdown, 1, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(s->stream);
        release(s);
        delete s;
        return sfail(RF_ERR_HIP, "server launch: %s", hipGetErrorString(e));
    }
    s->running = true;
    s->stats.workgroups = s->blocks;
    *out = s;
    return RF_OK;
}

rf_status rf_server_submit(rf_server* s, const rf_camera* cam, int32_t start_cell, uint64_t* req_id)
{
    if (!s || !cam || !req_id) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    if (cam->width <= 0 || cam->height <= 0 || !(cam->fov_deg > 0.0f && cam->fov_deg < 180.0f))
        return sfail(RF_ERR_INVALID_ARG, "invalid camera");
    const int64_t pixels = (int64_t)cam->width * cam->height;
    const int64_t n_tiles = (int64_t)((cam->width + 7) / 8) * ((cam->height + 7) / 8);
    if (n_tiles >= ((int64_t)1 << rf::kLocalTileBits) || pixels * 4 > (int64_t)s->pool_floats)
        return sfail(RF_ERR_UNSUPPORTED, "image of %d x %d does not fit the server", cam->width, cam->height);
    std::lock_guard<std::mutex> lock(s->mu);
    if (__atomic_load_n(&s->host->stopped, __ATOMIC_ACQUIRE) != 0)
        return sfail(RF_ERR_HIP, "server kernel has stopped (watchdog: no host heartbeat)");
    collect_done(s);
    int slot = -1;
    for (int k = 0; k < s->max_inflight; ++k)
        if (!s->slots[k].busy) {
            slot = k;
            break;
        }
    int64_t off = 0;
    if (slot < 0 || s->tiles_inflight + n_tiles > rf::kTileRing || !pool_alloc(s, pixels * 4, &off)) {
        s->stats.rejected_busy++;
        return sfail(RF_ERR_BUSY, slot < 0 ? "no free request slot" : "output pool full");
    }
    s->tiles_inflight += n_tiles;
    rf_server::Slot& sl = s->slots[slot];
    sl.busy = true;
    sl.done = false;
    sl.seq = s->next_seq++;
    sl.offset = off;
    sl.floats = pixels * 4;
    sl.width = cam->width;
    sl.height = cam->height;
    sl.tiles = n_tiles;
    rf::ReqRecord r;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) r.rot[3 * i + j] = cam->pose[4 * i + j];
        r.pos[i] = cam->pose[4 * i + 3];
    }
    r.focal = (float)(0.5 * cam->width / tan(0.5 * (double)cam->fov_deg * M_PI / 180.0));
    r.width = cam->width;
    r.height = cam->height;
    r.start = start_cell;
    r.n_tiles = (int32_t)n_tiles;
    r.slot = slot;
    r.out_offset = off;
    r.seq = sl.seq;
    const int64_t w = s->host->written;
    memcpy(&s->host->ring[w % rf::kHostRing], &r, sizeof r);
    __atomic_store_n(&s->host->written, w + 1, __ATOMIC_RELEASE);
    s->stats.submitted++;
    s->stats.inflight++;
    s->stats.pool_used_bytes += pixels * 16;
    *req_id = sl.seq;
    return RF_OK;
}

rf_status rf_server_poll(rf_server* s, uint64_t* done_ids, int32_t cap, int32_t* n_done)
{
    if (!s || !n_done || (cap > 0 && !done_ids)) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    collect_done(s);
    int n = 0;
    for (int k = 0; k < s->max_inflight && n < cap; ++k)
        if (s->slots[k].busy && s->slots[k].done) done_ids[n++] = s->slots[k].seq;
    *n_done = n;
    return RF_OK;
}

rf_status rf_server_result(rf_server* s, uint64_t req_id, float* rgba, size_t bytes)
{
    if (!s) return sfail(RF_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    collect_done(s);
    for (int k = 0; k < s->max_inflight; ++k) {
        rf_server::Slot& sl = s->slots[k];
        if (!sl.busy || sl.seq != req_id) continue;
        if (!sl.done) return sfail(RF_ERR_BUSY, "request %llu not finished", (unsigned long long)req_id);
        const size_t need = (size_t)sl.floats * 4;
        if (rgba) {
            if (bytes < need) return sfail(RF_ERR_INVALID_ARG, "result buffer of %zu bytes < %zu", bytes, need);
            memcpy(rgba, s->pool + sl.offset, need);
        }
        pool_free(s, sl.offset, sl.floats);
        s->tiles_inflight -= sl.tiles;
        s->stats.pool_used_bytes -= (int64_t)need;
        s->stats.inflight--;
        sl.busy = false;
        sl.done = false;
        return RF_OK;
    }
    return sfail(RF_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)req_id);
}

rf_status rf_server_stats_get(rf_server* s, rf_server_stats* out)
{
    if (!s || !out) return sfail(RF_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    collect_done(s);
    *out = s->stats;
    return RF_OK;
}

rf_status rf_server_destroy(rf_server* s)
{
    if (!s) return RF_OK;
    rf_status st = RF_OK;
    if (s->running) {
        // let admitted requests finish (bounded wait), then stop every wave
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            bool pending = false;
            {
                std::lock_guard<std::mutex> lock(s->mu);
                collect_done(s);
                for (auto& sl : s->slots) pending |= sl.busy && !sl.done;
            }
            if (!pending) break;
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) {
                st = sfail(RF_ERR_HIP, "requests still in flight after 10 s at shutdown");
                break;
            }
        }
        __atomic_store_n(&s->host->shutdown, 1, __ATOMIC_RELEASE);
        const hipError_t e = hipStreamSynchronize(s->stream);
        if (__atomic_load_n(&s->host->stopped, __ATOMIC_ACQUIRE) == 2 && st == RF_OK)
            st = sfail(RF_ERR_HIP, "server kernel had stopped itself (no host heartbeat)");
        if (e != hipSuccess && st == RF_OK) st = sfail(RF_ERR_HIP, "server kernel: %s", hipGetErrorString(e));
        s->running = false;
    }
    release(s);
    delete s;
    return st;
}

}  // extern "C"
