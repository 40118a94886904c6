// Protocol of the persistent render server, written once for the device (one
// lane of a wavefront) and for a host-thread model of it (tests).
//
// Host -> dispatcher: the host writes request records into a ring in
// coherent host memory and publishes their count (n_requests) with a release
// store. One dispatcher wavefront reads each new record (acquire on the
// count), copies it into the request's slot in device memory, resets the
// slot's done counter and opens the slot for claims with a release store of
// its claim word. Dispatcher -> workers: a slot's claim word is
// (generation << 32 | tiles claimed); a request's generation is nonzero and
// unique among the requests a slot has held. Workers claim tiles with
// fetch-and-add on the claim word and keep a claim only if it hit the
// generation of the record they then read and lies below its tile count: a
// claim that lands on a finished or recycled generation claims nothing. A
// worker renders its tiles, releases their pixels to the host, and adds one
// per tile to the slot's done counter (generation << 32 | tiles done); the
// tile that completes the request stores the request's sequence number into
// the slot's completion word in host memory (release), which the host polls.
// A slot is recycled only after its request completed, so every claim that
// counted has been rendered before the slot's record changes.
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
    int32_t stop;             // dispatcher: no more requests in this launch
    int32_t pad;
    Req slots[kSlots];
};

inline __host__ __device__ int64_t req_out_offset(const Req& r)
{
    return (int64_t)(((uint64_t)(uint32_t)r.out_offset_hi << 32) | (uint32_t)r.out_offset_lo);
}
inline __host__ __device__ uint64_t req_seq(const Req& r) { return ((uint64_t)r.seq_hi << 32) | r.seq_lo; }

// Env supplies the atomics: dev_* at the scope shared by the workers (the
// device), sys_* at the scope shared with the host, and word copies.
template <class Env>
struct Protocol {
    // Dispatcher, after copying record `rec` into d->slots[slot]: reset the
    // done counter and open the slot to claims of generation rec.gen.
    static __host__ __device__ void activate(DevCtl* d, int slot, uint32_t gen)
    {
        Env::dev_store_relaxed(&d->done[slot], (uint64_t)gen << 32);
        Env::dev_fence_release();
        Env::dev_store_release(&d->claim[slot], (uint64_t)gen << 32);
    }

    // Worker: is slot s open with tiles left? (its sequence number in *seq)
    static __host__ __device__ bool open(DevCtl* d, int s, uint64_t* seq)
    {
        const uint64_t c = Env::dev_load_acquire(&d->claim[s]);
        const uint32_t g = (uint32_t)(c >> 32);
        if (g == 0) return false;
        const Req* r = &d->slots[s];
        if (Env::word_load(&r->gen) != g) return false;
        const int32_t n = (int32_t)Env::word_load((const uint32_t*)&r->n_tiles);
        if ((int64_t)(c & kCountMask) >= (int64_t)n) return false;
        *seq = ((uint64_t)Env::word_load(&r->seq_hi) << 32) | Env::word_load(&r->seq_lo);
        return true;
    }

    // Worker: claims up to k tiles of slot s. Returns the number of tiles
    // claimed (0: none) with the first in *first and the record in *rec.
    static __host__ __device__ int claim(DevCtl* d, int s, int k, int32_t* first, Req* rec)
    {
        const uint64_t old = Env::dev_fetch_add_acq_rel(&d->claim[s], (uint64_t)k);
        Env::copy_record(rec, &d->slots[s]);
        if ((uint32_t)(old >> 32) != rec->gen) return 0;  // a generation that is gone
        const int64_t c = (int64_t)(old & kCountMask);
        if (c >= rec->n_tiles) return 0;                   // nothing left
        *first = (int32_t)c;
        const int64_t left = rec->n_tiles - c;
        return (int)(left < k ? left : k);
    }

    // Worker: one tile of `rec` done (its pixels already released to the
    // host). Returns true if it completed the request.
    static __host__ __device__ bool tile_done(DevCtl* d, HostCtl* h, const Req& rec)
    {
        const uint64_t old = Env::dev_fetch_add_acq_rel(&d->done[rec.slot], (uint64_t)1);
        if ((uint32_t)(old >> 32) != rec.gen) return false;  // cannot happen: the slot is not recycled before
        if ((int64_t)(old & kCountMask) + 1 != rec.n_tiles) return false;
        Env::sys_store_release(&h->done_seq[rec.slot], req_seq(rec));
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
