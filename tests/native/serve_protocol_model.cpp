// Host-thread model of the persistent render server's protocol
// (serve_protocol.hpp): a dispatcher thread and worker threads run the same
// protocol calls as the kernel's dispatcher and worker wavefronts, with the
// same memory orders, against a host thread that submits requests, polls
// their completion words, checks every pixel and recycles slots, and
// relaunches the "kernel" (the thread group) when requests wait and no launch
// is running. Built with ThreadSanitizer by the test suite.
//
// Checks: every request completes exactly once; every tile is rendered
// exactly once; the record a claim renders from is its request's, whole,
// for as long as the claim is outstanding (not torn by the next record's
// write into the slot); every pixel the host reads after a completion was written by
// its worker (ordered by the protocol's release and acquire); the launches
// leave by themselves (idle and hard limits) and on shutdown.

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstddef>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "serve_protocol.hpp"

using namespace rf::sp;
using Clock = std::chrono::steady_clock;

// Each operation may be delayed (a yield, now and then a pause of up to
// 50 us): the threads interleave at every step of the protocol, as
// wavefronts that are descheduled or wait on memory do.
static void jitter()
{
    thread_local std::mt19937 rng(std::hash<std::thread::id>()(std::this_thread::get_id()));
    const uint32_t r = rng();
    if (r % 16 == 0) std::this_thread::yield();
    if (r % 512 == 1) std::this_thread::sleep_for(std::chrono::microseconds(r % 50));
}

struct HostEnv {
    static uint64_t dev_load_acquire(const uint64_t* p) { jitter(); return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
    static uint64_t dev_load_relaxed(const uint64_t* p) { jitter(); return __atomic_load_n(p, __ATOMIC_RELAXED); }
    static void dev_fence_acquire() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
    static void dev_store_relaxed(uint64_t* p, uint64_t v) { jitter(); __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    static void dev_store_release(uint64_t* p, uint64_t v) { jitter(); __atomic_store_n(p, v, __ATOMIC_RELEASE); }
    static void dev_fence_release() { __atomic_thread_fence(__ATOMIC_RELEASE); }
    static uint64_t dev_fetch_add_acq_rel(uint64_t* p, uint64_t v)
    {
        jitter();
        return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL);
    }
    static uint64_t dev_fetch_add_acquire(uint64_t* p, uint64_t v)
    {
        jitter();
        return __atomic_fetch_add(p, v, __ATOMIC_ACQUIRE);
    }
    static uint64_t sys_fetch_add_release(uint64_t* p, uint64_t v)
    {
        jitter();
        return __atomic_fetch_add(p, v, __ATOMIC_RELEASE);
    }
    static void sys_store_release(uint64_t* p, uint64_t v) { jitter(); __atomic_store_n(p, v, __ATOMIC_RELEASE); }
    static uint32_t word_load(const uint32_t* p) { jitter(); return __atomic_load_n(p, __ATOMIC_RELAXED); }
};
using P = Protocol<HostEnv>;

// A record read word by word as a wavefront's lanes read it: in a random
// order, with pauses (a record may change while it is being read).
static void read_record(Req* dst, const Req* src, std::mt19937& rng)
{
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    int order[kReqWords];
    for (int k = 0; k < kReqWords; ++k) order[k] = k;
    std::shuffle(order, order + kReqWords, rng);
    for (int j = 0; j < kReqWords; ++j) {
        d[order[j]] = HostEnv::word_load(s + order[j]);
        if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 40));
    }
}

constexpr int kRequests = 12000;
constexpr int kMaxInflight = 3;
constexpr int kWorkers = 6;
constexpr int kClaim = 3;
constexpr int kMaxTiles = 40;
constexpr uint32_t kIdleCap = 1u << 22;

static HostCtl* H;
static DevCtl* D;
static std::vector<std::vector<std::atomic<int>>> rendered;  // [request][tile] render count
static std::vector<std::vector<uint64_t>> pixels;            // [request][tile] plain "pixels"
static std::atomic<int> dev_stop_seen{0};
static std::atomic<int> torn{0};

// The words of request r's record that the protocol does not use: each a
// distinct function of r, so that a copy mixing two records shows.
static uint32_t fill_word(int r, int k) { return (uint32_t)r * 2654435761u + (uint32_t)k * 40503u + 1u; }
static bool is_fill_word(int k)
{
    const int proto[] = {(int)(offsetof(Req, slot) / 4), (int)(offsetof(Req, seq_lo) / 4),
                         (int)(offsetof(Req, seq_hi) / 4), (int)(offsetof(Req, gen) / 4),
                         (int)(offsetof(Req, n_tiles) / 4)};
    for (int p : proto)
        if (k == p) return false;
    return true;
}

static const auto kIdle = std::chrono::microseconds(300);
static const auto kHard = std::chrono::milliseconds(200);

static void dispatcher(int64_t consumed)
{
    std::mt19937 rng((unsigned)consumed + 7);
    auto last = Clock::now();
    uint32_t idle = 0;
    while (idle < kIdleCap) {
        const int64_t n = __atomic_load_n(&H->n_requests, __ATOMIC_ACQUIRE);
        if (consumed < n) {
            Req rec;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&H->ring[consumed % kReqRing]);
            uint32_t* w = reinterpret_cast<uint32_t*>(&rec);
            for (int k = 0; k < kReqWords; ++k) w[k] = __atomic_load_n(src + k, __ATOMIC_RELAXED);
            if (rec.slot >= 0 && rec.slot < kSlots && rec.gen != 0 && rec.n_tiles > 0) {
                uint32_t* dst = reinterpret_cast<uint32_t*>(&D->slots[rec.slot]);
                // the words in any order (a wavefront's store lands in no fixed
                // order), with pauses, while late claims land on the slot
                int order[kReqWords];
                for (int k = 0; k < kReqWords; ++k) order[k] = k;
                std::shuffle(order, order + kReqWords, rng);
                for (int j = 0; j < kReqWords; ++j) {
                    const int k = order[j];
                    __atomic_store_n(dst + k, w[k], __ATOMIC_RELAXED);
                    if (rng() % 16 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 20));
                }
                // a slow dispatcher: the new record sits in the slot before the slot reopens
                if (rng() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 60));
                P::activate(D, rec.slot, rec.gen, rec.n_tiles);
            }
            ++consumed;
            __atomic_store_n(&H->consumed, consumed, __ATOMIC_RELEASE);
            last = Clock::now();
            idle = 0;
            continue;
        }
        if (__atomic_load_n(&H->shutdown, __ATOMIC_ACQUIRE)) break;
        const auto quiet = Clock::now() - last;
        if (quiet > kIdle) {
            bool all_idle = true;
            for (int s = 0; s < kSlots; ++s) all_idle &= P::slot_idle(D, s);
            if (all_idle) break;
            if (quiet > kHard) break;
        }
        ++idle;
        std::this_thread::yield();
    }
    __atomic_store_n(&D->stop, 1, __ATOMIC_RELEASE);
}

static void worker(unsigned seed)
{
    std::mt19937 rng(seed);
    auto last = Clock::now();
    uint32_t idle = 0;
    uint64_t seen = ~0ull;  // openings counted before the last scan that found nothing open
    bool fenced = true;     // the next scan follows an acquire fence
    while (idle < kIdleCap) {
        const uint64_t o = P::opened(D);
        if (o == seen) {
            if (__atomic_load_n(&D->stop, __ATOMIC_RELAXED)) {
                dev_stop_seen.fetch_add(1);
                break;
            }
            if (Clock::now() - last > kHard) break;
            ++idle;
            std::this_thread::yield();
            continue;
        }
        if (fenced) HostEnv::dev_fence_acquire();
        int best = -1;
        uint64_t best_seq = ~0ull;
        for (int s = 0; s < kSlots; ++s) {
            uint64_t seq;
            int64_t left;
            if (P::open(D, s, &seq, &left) && seq < best_seq) {
                best_seq = seq;
                best = s;
            }
        }
        if (best < 0) {
            if (fenced) seen = o;  // a scan without a fence is not trusted to find nothing
            fenced = true;
            ++idle;
            continue;
        }
        seen = ~0ull;
        fenced = false;
        // a worker may stall between seeing a slot open and claiming (the
        // slot can finish and be recycled meanwhile: the claim must notice)
        if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 80));
        Claim c;
        const int cnt = P::claim(D, best, kClaim, &c);
        if (cnt == 0) {
            ++idle;
            continue;
        }
        // the record as lane 0 reads it while the claim is outstanding
        Req rec;
        read_record(&rec, &D->slots[best], rng);
        const uint64_t seq = c.seq;
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(&rec);
        bool whole = seq >= 1 && seq <= (uint64_t)kRequests && c.gen == (uint32_t)seq && rec.gen == c.gen &&
                     req_seq(rec) == seq && rec.n_tiles == c.n_tiles && c.first + cnt <= c.n_tiles;
        for (int k = 0; whole && k < kReqWords; ++k) whole = !is_fill_word(k) || rw[k] == fill_word((int)seq - 1, k);
        if (!whole || c.first + cnt > (int)rendered[seq - 1].size()) {
            if (torn.fetch_add(1) == 0)
                fprintf(stderr, "claim of %d tiles with a torn or changed record (seq %llu, gen %u, first %d)\n", cnt,
                        (unsigned long long)seq, c.gen, c.first);
            continue;
        }
        for (int j = 0; j < cnt; ++j) {
            const int tile = c.first + j;
            rendered[seq - 1][tile].fetch_add(1, std::memory_order_relaxed);
            pixels[seq - 1][tile] = seq * 1000003ull + tile;  // plain write, published by the protocol
            if (rng() % 7 == 0) std::this_thread::yield();
        }
        P::tiles_done(D, H, best, c);
        last = Clock::now();
        idle = 0;
    }
}

struct Launch {
    std::vector<std::thread> th;
    std::atomic<int> left{0};
};

int main()
{
    H = new HostCtl();
    D = new DevCtl();
    memset(H, 0, sizeof *H);
    memset(D, 0, sizeof *D);
    std::mt19937 rng(12345);
    std::vector<int> tiles(kRequests);
    rendered = std::vector<std::vector<std::atomic<int>>>(kRequests);
    pixels.resize(kRequests);
    for (int r = 0; r < kRequests; ++r) {
        tiles[r] = 1 + (int)(rng() % kMaxTiles);
        rendered[r] = std::vector<std::atomic<int>>(tiles[r]);
        pixels[r].assign(tiles[r], 0);
    }
    int slot_req[kSlots];
    for (int s = 0; s < kSlots; ++s) slot_req[s] = -1;
    std::vector<int> done_count(kRequests, 0);
    int submitted = 0, completed = 0, launches = 0;
    int64_t written = 0;
    Launch* running = nullptr;
    auto launch_alive = [&]() {
        return running && running->left.load() > 0;
    };
    const auto t_end = Clock::now() + std::chrono::seconds(60);
    auto t_progress = Clock::now();
    int completed_before = 0;
    while (completed < kRequests && Clock::now() < t_end) {
        // a request left waiting with nothing else happening: an opening that no worker saw
        if (completed != completed_before) {
            completed_before = completed;
            t_progress = Clock::now();
        } else if (submitted > completed && Clock::now() - t_progress > std::chrono::seconds(3)) {
            fprintf(stderr, "no request completed for 3 s with %d in flight\n", submitted - completed);
            return 1;
        }
        // submit while slots are free (bursts, then pauses so that launches idle out)
        int inflight = 0;
        for (int s = 0; s < kMaxInflight; ++s) inflight += slot_req[s] >= 0;
        if (submitted < kRequests && inflight < kMaxInflight && rng() % 3 != 0) {
            int s = 0;
            while (slot_req[s] >= 0) ++s;
            const int r = submitted++;
            Req q;
            memset(&q, 0, sizeof q);
            q.slot = s;
            q.seq_lo = (uint32_t)(r + 1);
            q.gen = (uint32_t)(r + 1);
            q.n_tiles = tiles[r];
            uint32_t* qw = reinterpret_cast<uint32_t*>(&q);
            for (int k = 0; k < kReqWords; ++k)
                if (is_fill_word(k)) qw[k] = fill_word(r, k);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&H->ring[written % kReqRing]);
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&q);
            for (int k = 0; k < kReqWords; ++k) __atomic_store_n(dst + k, src[k], __ATOMIC_RELAXED);
            ++written;
            __atomic_store_n(&H->n_requests, written, __ATOMIC_RELEASE);
            slot_req[s] = r;
        }
        // completions
        for (int s = 0; s < kMaxInflight; ++s) {
            const int r = slot_req[s];
            if (r < 0) continue;
            if (__atomic_load_n(&H->done_seq[s], __ATOMIC_ACQUIRE) != (uint64_t)(r + 1)) continue;
            for (int t = 0; t < tiles[r]; ++t) {
                if (rendered[r][t].load(std::memory_order_relaxed) != 1 || pixels[r][t] != (uint64_t)(r + 1) * 1000003ull + t) {
                    fprintf(stderr, "request %d tile %d: rendered %d times, pixel %llu\n", r, t,
                            rendered[r][t].load(), (unsigned long long)pixels[r][t]);
                    return 1;
                }
            }
            ++done_count[r];
            ++completed;
            slot_req[s] = -1;  // recycled
        }
        // (re)launch when requests wait and no launch runs
        if (!launch_alive() && __atomic_load_n(&H->consumed, __ATOMIC_ACQUIRE) < written) {
            if (running) {
                for (auto& t : running->th) t.join();
                delete running;
            }
            running = new Launch();
            __atomic_store_n(&D->stop, 0, __ATOMIC_RELAXED);
            const int64_t c0 = __atomic_load_n(&H->consumed, __ATOMIC_ACQUIRE);
            running->left = kWorkers + 1;
            Launch* L = running;
            L->th.emplace_back([L, c0] { dispatcher(c0); L->left.fetch_sub(1); });
            for (int w = 0; w < kWorkers; ++w)
                L->th.emplace_back([L, w, launches] { worker(1000u * launches + w); L->left.fetch_sub(1); });
            ++launches;
        }
        if (rng() % 50 == 0) std::this_thread::sleep_for(std::chrono::milliseconds(1));  // let launches idle out
    }
    __atomic_store_n(&H->shutdown, 1, __ATOMIC_RELEASE);
    const auto t_stop = Clock::now();
    if (running) {
        for (auto& t : running->th) t.join();
        delete running;
    }
    const double stop_ms = std::chrono::duration<double, std::milli>(Clock::now() - t_stop).count();
    if (torn.load()) {
        fprintf(stderr, "%d claims read a torn record\n", torn.load());
        return 1;
    }
    for (int r = 0; r < kRequests; ++r)
        if (done_count[r] != 1) {
            fprintf(stderr, "request %d completed %d times\n", r, done_count[r]);
            return 1;
        }
    if (__atomic_load_n(&H->consumed, __ATOMIC_ACQUIRE) != written) {
        fprintf(stderr, "consumed %lld of %lld records\n", (long long)H->consumed, (long long)written);
        return 1;
    }
    printf("model: %d requests, %d launches, all tiles rendered once, stopped in %.1f ms\n", kRequests, launches,
           stop_ms);
    return launches > 1 ? 0 : 2;  // the launches must have idled out and been relaunched at least once
}
