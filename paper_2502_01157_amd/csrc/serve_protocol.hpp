// Protocol of the persistent render server, written once for the device (one
// lane of a wavefront) and for a host-thread model of it (tests).
//
// Host -> dispatcher: the host writes request records into a ring in
// coherent host memory and publishes their count (n_requests) with a release
// store. One dispatcher wavefront reads each new record (acquire on the
// count), copies it into the request's slot in device memory, resets the
// slot's done counter, opens the slot with a release store of its claim word
// and counts the opening in `opened`.
//
// Dispatcher -> workers: a slot's claim word is (tile count << 32 | tiles
// claimed); a tile count of 0 means the slot has never been opened. Workers
// claim tiles with an acquiring fetch-and-add on the claim word: the value it
// returns tells, in one atomic step, whether the claim counts (tiles claimed
// before it below the tile count of the request the word belongs to). A claim
// that counts holds the request open, since the request completes only once
// every counted claim is done, and a slot is rewritten only after its request
// completed; so the slot keeps the claim's record, which the acquire made
// visible, for as long as the claim is outstanding. A claim that lands after
// the slot reopened claims the new request's tiles, under the same rule. A
// claim that does not count (the request fully claimed or finished) reads
// nothing from the slot. A worker lands at most one such claim per opening of
// a slot (its next read of the word sees its own addition), so the claimed
// count stays far below 2^32.
//
// Workers -> host: a worker renders its claim's tiles into host memory and
// adds their number to the slot's done counter (generation << 32 | tiles
// done) with a release at system scope. The claim that completes the request
// acquires every other claim's release (all additions after the reset are
// read-modify-writes, so each one's release sequence reaches the last) and
// stores the request's sequence number into the slot's completion word in
// host memory (release), which the host polls (acquire).
//
// Idle workers poll `opened` alone, and scan the slots only when it has
// changed since their last scan that found nothing open: a slot opens only
// by an activation, and tiles once claimed stay claimed. The scan is a hint:
// claim() validates what it takes.
//
// Every shared word is accessed with atomic operations of explicit order and
// scope (records word by word, relaxed, ordered by the claim word's release
// and acquire); nothing waits on anything without a bound (the waits live in
// the kernel and the model, not here).
#pragma once

#include <stdint.h>

namespace rf {
namespace sp {

constexpr int kSlots = 64;        // requests in flight (one per lane of a wavefront)
constexpr int kReqRing = 256;     // host ring of request records (> kSlots)
constexpr uint64_t kCountMask = 0xffffffffull;

// A request as the host writes it and the device keeps it (32-bit words).
struct Req {
    float rot[9];
    float pos[3];
    int32_t model;
    float focal;
    int32_t width, height, start, slot;
    int32_t out_offset_lo, out_offset_hi;  // floats from the pool base
    uint32_t seq_lo, seq_hi;               // 1-based request sequence number
    uint32_t gen;                          // nonzero generation of the slot
    int32_t n_tiles;                       // 1 .. 2^31 - 1
};
constexpr int kReqWords = (int)(sizeof(Req) / 4);
static_assert(sizeof(Req) % 4 == 0 && kReqWords <= 64, "a record is read one word per lane");

struct HostCtl {              // coherent host memory
    int64_t n_requests;       // records written (host, release)
    int64_t consumed;         // records consumed (dispatcher, release)
    int32_t shutdown;         // host: stop now
    int32_t pad;
    uint64_t done_seq[kSlots];  // device: sequence number of the last completed request per slot
    Req ring[kReqRing];
};

struct DevCtl {               // device memory
    uint64_t claim[kSlots];
    uint64_t done[kSlots];
    uint64_t opened;          // activations so far (dispatcher, release)
    int32_t stop;             // dispatcher: no more requests in this launch
    int32_t pad;
    Req slots[kSlots];
};

// What a worker holds of a claim (the rest of the record stays in the slot).
struct Claim {
    int32_t first, count, n_tiles;
    uint32_t gen;
    uint64_t seq;
};

inline __host__ __device__ int64_t req_out_offset(const Req& r)
{
    return (int64_t)(((uint64_t)(uint32_t)r.out_offset_hi << 32) | (uint32_t)r.out_offset_lo);
}
inline __host__ __device__ uint64_t req_seq(const Req& r) { return ((uint64_t)r.seq_hi << 32) | r.seq_lo; }

// Env supplies the atomics: dev_* at the scope shared by the workers (the
// device), sys_* at the scope shared with the host, and relaxed word loads
// at device scope.
template <class Env>
struct Protocol {
    // Dispatcher, once the words of a new record are in slot s (relaxed
    // stores, ordered before this call): reset the done counter, open the
    // slot to claims of the record's n_tiles tiles, and count the opening.
    static __host__ __device__ void activate(DevCtl* d, int slot, uint32_t gen, int32_t n_tiles)
    {
        Env::dev_store_relaxed(&d->done[slot], (uint64_t)gen << 32);
        Env::dev_fence_release();
        Env::dev_store_release(&d->claim[slot], (uint64_t)(uint32_t)n_tiles << 32);
        (void)Env::dev_fetch_add_acq_rel(&d->opened, (uint64_t)1);
    }

    // Worker: activations so far. Before a scan of the slots that is to be
    // trusted when it finds nothing open, the worker reads this, then fences
    // (acquire): the scan sees every opening counted.
    static __host__ __device__ uint64_t opened(DevCtl* d) { return Env::dev_load_relaxed(&d->opened); }

    // Worker: is slot s open with tiles left? (its sequence number in *seq,
    // the tiles not yet claimed in *left) A hint only, read without
    // ordering (the sequence number may even be another request's).
    static __host__ __device__ bool open(DevCtl* d, int s, uint64_t* seq, int64_t* left)
    {
        const uint64_t c = Env::dev_load_relaxed(&d->claim[s]);
        const int64_t n = (int64_t)(c >> 32), claimed = (int64_t)(c & kCountMask);
        if (claimed >= n) return false;
        const Req* r = &d->slots[s];
        *seq = ((uint64_t)Env::word_load(&r->seq_hi) << 32) | Env::word_load(&r->seq_lo);
        *left = n - claimed;
        return true;
    }

    // Worker: claims up to k tiles of slot s. Returns the number of tiles
    // claimed (0: none), described in *out. While a claim that counted is
    // outstanding the slot keeps its request's record, visible to the
    // claiming thread.
    static __host__ __device__ int claim(DevCtl* d, int s, int k, Claim* out)
    {
        const uint64_t old = Env::dev_fetch_add_acquire(&d->claim[s], (uint64_t)k);
        const int64_t n = (int64_t)(old >> 32), c = (int64_t)(old & kCountMask);
        if (c >= n) return 0;  // nothing left, or never opened
        const Req* r = &d->slots[s];
        const int64_t left = n - c;
        out->first = (int32_t)c;
        out->count = (int32_t)(left < k ? left : k);
        out->n_tiles = (int32_t)n;
        out->gen = Env::word_load(&r->gen);
        out->seq = ((uint64_t)Env::word_load(&r->seq_hi) << 32) | Env::word_load(&r->seq_lo);
        return out->count;
    }

    // Worker: the tiles of claim `c` in slot s done. Every pixel of the claim
    // must be ordered before this call (they are released here at system
    // scope). Returns true if it completed the request.
    static __host__ __device__ bool tiles_done(DevCtl* d, HostCtl* h, int s, const Claim& c)
    {
        const uint64_t old = Env::sys_fetch_add_release(&d->done[s], (uint64_t)c.count);
        if ((uint32_t)(old >> 32) != c.gen) return false;  // cannot happen: the slot is not recycled before
        if ((int64_t)(old & kCountMask) + c.count != c.n_tiles) return false;
        // the last claim: acquire the other claims' releases (this reads our
        // own addition, the end of each of their release sequences)
        (void)Env::dev_load_acquire(&d->done[s]);
        Env::sys_store_release(&h->done_seq[s], c.seq);
        return true;
    }

    // Dispatcher: has the request last activated in slot s completed? (only
    // the dispatcher activates, so the done counter it reads is that request's)
    static __host__ __device__ bool slot_idle(DevCtl* d, int s)
    {
        const uint64_t c = Env::dev_load_acquire(&d->claim[s]);
        const int64_t n = (int64_t)(c >> 32);
        if (n == 0) return true;
        const uint64_t dn = Env::dev_load_acquire(&d->done[s]);
        return (int64_t)(dn & kCountMask) >= n;
    }
};

}  // namespace sp
}  // namespace rf
