// Protocol of the persistent render server, written once for the device (one
// lane of a wavefront) and for a host-thread model of it (tests).
//
// Host -> dispatcher: the host writes request records into a ring in
// coherent host memory and publishes their count (n_requests) with a release
// store. One dispatcher wavefront reads each new record (acquire on the
// count), copies it into the request's slot in device memory, resets the
// slot's done counter, opens the slot for claims with a release store of its
// claim word and counts the opening in `opened`. Dispatcher -> workers: a
// slot's claim word is (generation << 32 | tiles claimed); a request's
// generation is nonzero and unique among the requests a slot has held.
// Workers claim tiles with fetch-and-add on the claim word and keep a claim
// only if it hit the generation the slot's record still holds and lies below
// its tile count: a claim that lands on a finished or recycled generation
// claims nothing. A worker renders the tiles of its claim, releases their
// pixels to the host, and adds their number to the slot's done counter
// (generation << 32 | tiles done); the claim that completes the request
// stores the request's sequence number into the slot's completion word in
// host memory (release), which the host polls. A slot is recycled only after
// its request completed, so the record of a claim that counted stays in its
// slot until that claim is done.
//
// A claim that lands after completion can still read the slot while the
// dispatcher writes the next record into it, so a record is written as a
// sequence lock on its generation word: the dispatcher clears the word,
// writes the other words, then stores the new generation; a claimer reads
// the record's tile count after its claim, fences, and reads the generation,
// and keeps the claim only if the generation equals the claim word's
// (generations of a slot never repeat, so a read that saw any word of a newer
// record fails the check).
//
// Idle workers poll `opened` alone, and scan the slots only when it has
// changed since their last scan that found nothing open: a slot opens only
// by an activation, and tiles once claimed stay claimed.
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
    int32_t n_tiles;
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
// and stores at device scope.
template <class Env>
struct Protocol {
    // Dispatcher, before writing the words of a new record into slot s
    // (the generation word excluded): mark the slot's record as being written.
    static __host__ __device__ void begin_record(DevCtl* d, int s)
    {
        Env::word_store_relaxed(&d->slots[s].gen, 0u);
        Env::dev_fence_release();
    }

    // Dispatcher, after writing them: publish the record's generation.
    static __host__ __device__ void end_record(DevCtl* d, int s, uint32_t gen)
    {
        Env::dev_fence_release();
        Env::word_store_relaxed(&d->slots[s].gen, gen);
    }

    // Dispatcher, after end_record: reset the done counter, open the slot to
    // claims of generation gen, and count the opening.
    static __host__ __device__ void activate(DevCtl* d, int slot, uint32_t gen)
    {
        Env::dev_store_relaxed(&d->done[slot], (uint64_t)gen << 32);
        Env::dev_fence_release();
        Env::dev_store_release(&d->claim[slot], (uint64_t)gen << 32);
        (void)Env::dev_fetch_add_acq_rel(&d->opened, (uint64_t)1);
    }

    // Worker: activations so far. Before a scan of the slots the worker reads
    // this, then fences (acquire): the scan sees every opening counted.
    static __host__ __device__ uint64_t opened(DevCtl* d) { return Env::dev_load_relaxed(&d->opened); }

    // Worker: is slot s open with tiles left? (its sequence number in *seq,
    // the tiles not yet claimed in *left) A hint only, read without
    // ordering: claim() validates what it takes.
    static __host__ __device__ bool open(DevCtl* d, int s, uint64_t* seq, int64_t* left)
    {
        const uint64_t c = Env::dev_load_relaxed(&d->claim[s]);
        const uint32_t g = (uint32_t)(c >> 32);
        if (g == 0) return false;
        const Req* r = &d->slots[s];
        if (Env::word_load(&r->gen) != g) return false;
        const int32_t n = (int32_t)Env::word_load((const uint32_t*)&r->n_tiles);
        if ((int64_t)(c & kCountMask) >= (int64_t)n) return false;
        *seq = ((uint64_t)Env::word_load(&r->seq_hi) << 32) | Env::word_load(&r->seq_lo);
        *left = (int64_t)n - (int64_t)(c & kCountMask);
        return true;
    }

    // Worker: claims up to k tiles of slot s. Returns the number of tiles
    // claimed (0: none), described in *out. While the claim is outstanding the
    // slot keeps the claimed request's record: every lane may then read it
    // (after an acquire fence of its own).
    static __host__ __device__ int claim(DevCtl* d, int s, int k, Claim* out)
    {
        const uint64_t old = Env::dev_fetch_add_acq_rel(&d->claim[s], (uint64_t)k);
        const uint32_t g = (uint32_t)(old >> 32);
        if (g == 0) return 0;
        const Req* r = &d->slots[s];
        const int64_t n = (int32_t)Env::word_load((const uint32_t*)&r->n_tiles);
        const uint64_t seq = ((uint64_t)Env::word_load(&r->seq_hi) << 32) | Env::word_load(&r->seq_lo);
        Env::dev_fence_acquire();
        // the generation after the reads: any word of a newer record read above shows here
        if (Env::word_load(&r->gen) != g) return 0;
        const int64_t c = (int64_t)(old & kCountMask);
        if (c >= n) return 0;  // nothing left
        const int64_t left = n - c;
        out->first = (int32_t)c;
        out->count = (int32_t)(left < k ? left : k);
        out->n_tiles = (int32_t)n;
        out->gen = g;
        out->seq = seq;
        return out->count;
    }

    // Worker: the tiles of claim `c` in slot s done (their pixels already
    // released to the host). Returns true if it completed the request.
    static __host__ __device__ bool tiles_done(DevCtl* d, HostCtl* h, int s, const Claim& c)
    {
        const uint64_t old = Env::dev_fetch_add_acq_rel(&d->done[s], (uint64_t)c.count);
        if ((uint32_t)(old >> 32) != c.gen) return false;  // cannot happen: the slot is not recycled before
        if ((int64_t)(old & kCountMask) + c.count != c.n_tiles) return false;
        Env::sys_store_release(&h->done_seq[s], c.seq);
        return true;
    }

    // Dispatcher: has every request activated in a slot completed? (s: one slot)
    static __host__ __device__ bool slot_idle(DevCtl* d, int s)
    {
        const uint64_t c = Env::dev_load_acquire(&d->claim[s]);
        if ((uint32_t)(c >> 32) == 0) return true;
        const uint64_t dn = Env::dev_load_acquire(&d->done[s]);
        const int32_t n = (int32_t)Env::word_load((const uint32_t*)&d->slots[s].n_tiles);
        return (uint32_t)(dn >> 32) == (uint32_t)(c >> 32) && (int64_t)(dn & kCountMask) >= (int64_t)n;
    }
};

}  // namespace sp
}  // namespace rf
