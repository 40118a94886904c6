// Device functions of the walk shared by the batch kernels and the serving kernel.
#pragma once

#include "rf_device.hpp"
#include "rf_kernels.hpp"

namespace rf {

struct FaceHit {
    float num, den;
    int k;       // index within the row, -1 if no front face
    uint2 next;  // the winning neighbour's row
};

// Nearest front face of a cell: den = n.d > 0 and the smallest
// t = (c - n.o) / den, compared without division (ties keep the first face).
// Faces are read four at a time from the row's base (in the plane array or a
// wavefront's LDS copy of the row) with immediate offsets; a batch may run up
// to three faces past the row's end (the plane array is padded, an LDS row is
// followed by more of the wavefront's LDS), and those faces are masked by
// k < deg.
// UNROLL: the first six batches are unrolled, so that each face's index is
// an immediate instead of a register move per face (the plain forward's
// staged scan: 3 % faster there; the kernels that keep more registers live
// lose a wavefront per SIMD to it).
// The face's offset from the ray origin, c - n.o (FP32, always this sequence).
__device__ inline float face_num(float4 p, float ox, float oy, float oz)
{
    return p.w - fmaf(p.z, oz, fmaf(p.y, oy, p.x * ox));
}

// NUM = true: the row's fourth component already holds face_num for this
// ray's origin (staged rows of a wavefront whose rays share their origin).
template <bool UNROLL = false, bool NUM = false, typename P>
__device__ inline FaceHit scan_row(P row, int deg, float ox, float oy, float oz, float dx, float dy, float dz)
{
    float bn = 1.0f, bd = 0.0f;
    int bk = -1;
    auto batch = [&](int k) {
        float4 p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = ld16(row + k + u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float den = fmaf(p[u].z, dz, fmaf(p[u].y, dy, p[u].x * dx));
            const float num = NUM ? p[u].w : face_num(p[u], ox, oy, oz);
            const bool better = (k + u < deg) && (den > 0.0f) && (num * bd < bn * den);
            bn = better ? num : bn;
            bd = better ? den : bd;
            bk = better ? k + u : bk;
        }
    };
    int k0 = 0;
    if constexpr (UNROLL) {
#pragma unroll
        for (int k = 0; k < 24; k += 4) {
            if (k >= deg) break;
            batch(k);
        }
        k0 = 24;
    }
    for (int k = k0; k < deg; k += 4) batch(k);
    return {bn, bd, bk, make_uint2(0u, 0u)};
}

__device__ inline FaceHit nearest_front_face(const float4* __restrict__ planes, int beg, int deg, float ox, float oy,
                                             float oz, float dx, float dy, float dz)
{
    return scan_row(planes + beg, deg, ox, oy, oz, dx, dy, dz);
}

template <int DEG>
__device__ inline void colour(const Attr<DEG>& at, const float* Y, float c[3])
{
    c[0] = c[1] = c[2] = 0.0f;
#pragma unroll
    for (int b = 0; b < sh_count(DEG); ++b) {
        c[0] = fmaf(at.sh[3 * b + 0], Y[b], c[0]);
        c[1] = fmaf(at.sh[3 * b + 1], Y[b], c[1]);
        c[2] = fmaf(at.sh[3 * b + 2], Y[b], c[2]);
    }
}

struct RayResult {
    float C[3];
    float T;
    int status;  // visited cells, -1 bad start, -2 max_steps reached
};

// Exit distance through the winning face, in double precision: the plane
// through m = x_i + n/2 with normal n (the stored n = x_j - x_i), so that
// t = n.(m - o) / n.d is formed from differences of nearby points instead of
// the FP32 offset c - n.o, whose cancellation costs ~eps32 (|o| + t)/cos.
// The ray is taken in double: a caller's FP32 ray widened exactly, or a
// secondary leg kept in double (see Leg).
__device__ inline double exit_distance(float4 p, const float* site, double ox, double oy, double oz, double dx,
                                       double dy, double dz)
{
    const double nx = p.x, ny = p.y, nz = p.z;
    const double mx = fma(0.5, nx, (double)site[0]) - (double)ox;
    const double my = fma(0.5, ny, (double)site[1]) - (double)oy;
    const double mz = fma(0.5, nz, (double)site[2]) - (double)oz;
    const double num = fma(nz, mz, fma(ny, my, nx * mx));
    const double den = fma(nz, dz, fma(ny, dy, nx * dx));
    return num / den;
}

// One visited cell of Algorithm 1: nearest front face (FP32 decision), exact
// exit distance of that face, clamped segment [t0, te], its optical depth,
// opacity and colour. Shared by the forward, backward and serving walks so
// that the backward recomputes bit-identical segments.
template <int DEG>
struct Visit {
    Attr<DEG> at;
    FaceHit h;
    double t1;     // exit distance of the winning face, +inf if none
    double te;     // max(t0, min(t1, t_max))
    float delta, tau, alpha;
    float c[3];
    bool clipped;  // no front face or t1 >= t_max: the walk ends in this cell
};

// The segment of a visit whose clamped exit te is known: width, optical depth,
// opacity and colour (eq. (3)-(4)).
template <int DEG>
__device__ inline void segment(double t0, const float* Y, Visit<DEG>& v)
{
    v.delta = (float)(v.te - t0);
    v.tau = v.at.sigma > 0.0f ? v.at.sigma * v.delta : 0.0f;
    v.alpha = -expm1f(-v.tau);
    colour<DEG>(v.at, Y, v.c);
}

// `hi` (nullable): the ray in double, {o, d, t_max}, for the exit distance and
// the clipping of a secondary leg; the face decision always uses the FP32 ray.
template <int DEG, bool BF16>
__device__ inline void visit_cell(const SceneView& s, uint2 ref, double t0, float tmax, float ox, float oy, float oz,
                                  float dx, float dy, float dz, const float* Y, Visit<DEG>& v,
                                  const double* hi = nullptr)
{
    const int cell = ref_cell(ref), beg = ref_beg(ref);
    v.h = nearest_front_face(s.planes, beg, ref_deg(ref), ox, oy, oz, dx, dy, dz);
    // the cell's record, the winning plane and the neighbour's row are
    // independent loads issued together after the scan
    float4 wp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (v.h.k >= 0) {
        wp = s.planes[beg + v.h.k];
        v.h.next = s.adj[beg + v.h.k];
    }
    load_record<DEG, BF16>(s.rec, cell, v.at);
    v.t1 = INFINITY;
    if (v.h.k >= 0) {
        if (hi)
            v.t1 = exit_distance(wp, v.at.site, hi[0], hi[1], hi[2], hi[3], hi[4], hi[5]);
        else
            v.t1 = exit_distance(wp, v.at.site, ox, oy, oz, dx, dy, dz);
    }
    const double tm = hi ? hi[6] : (double)tmax;
    v.clipped = (v.h.k < 0) || (v.t1 >= tm);
    v.te = fmax(t0, fmin(v.t1, tm));
    segment<DEG>(t0, Y, v);
}

// n.d of the face between cells with sites xi and xj, n = xj - xi, for the
// exit-distance derivative dt/dx = (p - x)/(n.d) of the backward. Formed in
// double: the difference of two FP32 sites is exact there, so n.d keeps full
// precision even for a nearly grazing exit face, where an FP32 dot product
// would lose a relative ~2^-24/cos to cancellation (and that face's site
// gradient is the largest of the ray's).
__device__ inline double face_den(const float* xi, const float* xj, double dx, double dy, double dz)
{
    const double nx = (double)xj[0] - (double)xi[0], ny = (double)xj[1] - (double)xi[1],
                 nz = (double)xj[2] - (double)xi[2];
    return fma(nz, dz, fma(ny, dy, nx * dx));
}

// ---------------------------------------------------------------------------
// Wavefront staging of the visited cells' data in LDS.
//
// The lanes of a wavefront (one 8x8 tile) are mostly in the same few cells at
// each step (about 9 distinct cells and 155 distinct faces for 64 lanes at
// 1M sites). Loading a row of planes per lane costs the vector memory path
// per active lane; instead, each distinct cell's row and record are copied
// once into the wavefront's LDS region by direct global-to-LDS loads (one
// 16-byte chunk per lane), and every lane then reads its own cell's copy.
// Cells that do not fit the region are read from global memory as before.
// ---------------------------------------------------------------------------
// Each wavefront's region is 10 KiB, so that sixteen one-wavefront blocks
// fill the 160 KiB of LDS (four wavefronts per SIMD, what the registers
// allow). A wavefront step touches 9.5 distinct cells on average on the
// clustered 1M-site frame (p90: 17), and the region keeps cells from step to
// step (StageCache). A staged record takes only its used bytes (208 of the
// 256 of an FP32 record at degree 3, 112 of 128 in BF16). The split between
// record and face slots, 22 records beside 352 faces in FP32 and 28 beside
// 444 in BF16, was the fastest measured there (20 / 24 records: 2 % slower
// forwards; 16 or 18 FP32 records: 4-8 % slower).
template <int DEG, bool BF16>
struct StageLayout {
    using R = Rec<DEG, BF16>;
    static constexpr int kBudget = 10240;
    static constexpr int kRecs = BF16 ? 28 : 22;                       // record slots
    static constexpr int kRecStride = R::CHUNKS * 16;                         // the record's used bytes
    static constexpr int kFaces = (kBudget - kRecs * kRecStride) / 16 / 4 * 4;  // face slots (16 B each)
    static constexpr int kRecOff = kFaces * 16;
    static constexpr int kBytes = kRecOff + kRecs * kRecStride;
    static_assert(kBytes <= kBudget, "stage region over budget");
};


// The cells a wavefront has staged, kept from step to step: the lanes of a
// tile reach many cells a step or two after other lanes of the tile left
// them (on the clustered 1M-site frame 80 % of a step's cells were staged
// the step before), so a cell found here needs no copy. Entry e (lane e of
// `key` and `face`, e < n) is cell `key` (its ref.x), its row at face slot
// `face` and its record in record slot e. Slots are handed out in order and
// all freed together when a step starts with less room left than a step
// usually needs.
struct StageCache {
    uint32_t key = 0;
    int face = 0;
    uint64_t valid = 0;  // entries in use (wavefront-uniform): bit e for e < n
    int n = 0;
    int faces = 0;       // face slots in use
};

// Called with every lane of the wavefront active. Lanes with `want` need the
// row and record of their cell `ref` in `region`; each distinct cell is
// looked up in the cache, and copied in (direct global-to-LDS loads) if it is
// not there. On return face_slot / rec_slot give the position of the copy
// (-1: the cell did not fit, read from global memory).
// With `num` (wavefront-uniform: every walking lane's ray has the origin
// (sx, sy, sz), bit for bit, for as long as the cache lives) each staged
// plane's offset c is replaced by face_num for that origin, computed once
// per staged face instead of once per lane, face and step: the scans then
// read the same bits they would have computed.
template <int DEG, bool BF16>
__device__ inline void stage_cells(const SceneView& s, bool want, uint2 ref, lds_u8* region, StageCache& cache,
                                   int& face_slot, int& rec_slot, bool num = false, float sx = 0.0f,
                                   float sy = 0.0f, float sz = 0.0f)
{
    using SL = StageLayout<DEG, BF16>;
    using R = Rec<DEG, BF16>;
    const int lane = __lane_id();
    const uint32_t lane16 = 16u * (uint32_t)lane;
    // start afresh only once the region is (nearly) full: the longer cells
    // stay, the more steps find them (flushing with room for ~5 cells left
    // made the forward 5 % slower, with ~3 left 3 %); a step whose new cells
    // do not all fit reads those from global memory
    if (cache.faces > SL::kFaces - 16 || cache.n == SL::kRecs) {
        cache.n = 0;
        cache.faces = 0;
        cache.valid = 0;
    }
    const int first_new = cache.faces, first_entry = cache.n;
    uint64_t pend = ballot(want);
    face_slot = -1;
    rec_slot = -1;
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        // ref.x = cell | deg << 24 identifies the cell
        const uint32_t kx = __builtin_amdgcn_readlane(ref.x, leader);
        // the lanes still pending with this cell (a ballot of the bare
        // compare, masked in scalar registers); kept per lane as well, as
        // testing the mask's bit costs five VALU instructions
        const bool mine = want && ref.x == kx;
        const uint64_t members = ballot(ref.x == kx) & pend;
        pend &= ~members;
        const uint64_t hit = ballot(cache.key == kx) & cache.valid;
        int e, fo;
        if (hit) {
            e = __builtin_ctzll(hit);
            fo = __builtin_amdgcn_readlane(cache.face, e);
        } else {
            const int gdeg = (int)(kx >> 24);
            if (cache.faces + gdeg > SL::kFaces || cache.n == SL::kRecs) continue;
            const int gbeg = __builtin_amdgcn_readlane(ref.y, leader);
            const int key = (int)(kx & 0xffffffu);
            e = cache.n;
            fo = cache.faces;
            for (int k0 = 0; k0 < gdeg; k0 += kWave)
                if (k0 + lane < gdeg)
                    copy16_to_lds(s.planes + gbeg + k0, 16u * kWave, lane16, region + (fo + k0) * 16);
            if (lane < R::CHUNKS)
                copy16_to_lds(s.rec + (size_t)key * R::BYTES, R::BYTES, lane16, region + SL::kRecOff + e * SL::kRecStride);
            if (lane == e) {
                cache.key = kx;
                cache.face = fo;
            }
            cache.valid |= 1ull << e;
            ++cache.n;
            cache.faces += gdeg;
        }
        if (mine) {
            face_slot = fo;
            rec_slot = e;
        }
    }
    if (cache.n != first_entry) {
        __builtin_amdgcn_s_waitcnt(0);  // the copies have landed in LDS
        __builtin_amdgcn_wave_barrier();
        if (num) {
            for (int f = first_new + lane; f < cache.faces; f += kWave) {
                const f32x4 p = *(reinterpret_cast<lds_f32x4*>(region) + f);
                reinterpret_cast<__attribute__((address_space(3))) float*>(region)[4 * f + 3] =
                    face_num(make_float4(p.x, p.y, p.z, p.w), sx, sy, sz);
            }
            // (one wavefront's LDS accesses complete in order: the scans read the new values)
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// visit_cell reading the staged copies where there are any.
// `num`: the staged rows hold face_num for this ray's origin (wavefront-uniform).
template <int DEG, bool BF16, bool UNROLL = false>
__device__ inline void visit_cell_staged(const SceneView& s, uint2 ref, int face_slot, int rec_slot,
                                         lds_u8* region, double t0, float tmax, float ox, float oy, float oz,
                                         float dx, float dy, float dz, const float* Y, Visit<DEG>& v,
                                         const double* hi = nullptr, bool num = false)
{
    using SL = StageLayout<DEG, BF16>;
    const int cell = ref_cell(ref), beg = ref_beg(ref), deg = ref_deg(ref);
    lds_f32x4* lrow = reinterpret_cast<lds_f32x4*>(region) + face_slot;
    if (face_slot >= 0 && num)
        v.h = scan_row<UNROLL, true>(lrow, deg, ox, oy, oz, dx, dy, dz);
    else if (face_slot >= 0)
        v.h = scan_row<UNROLL>(lrow, deg, ox, oy, oz, dx, dy, dz);
    else
        v.h = nearest_front_face(s.planes, beg, deg, ox, oy, oz, dx, dy, dz);
    float4 wp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (v.h.k >= 0) {
        wp = face_slot >= 0 ? ld16(lrow + v.h.k) : s.planes[beg + v.h.k];
        v.h.next = s.adj[beg + v.h.k];
    }
    if (rec_slot >= 0)
        unpack_record<DEG, BF16>(reinterpret_cast<lds_u32x4*>(region + SL::kRecOff + rec_slot * SL::kRecStride), v.at);
    else
        load_record<DEG, BF16>(s.rec, cell, v.at);
    v.t1 = INFINITY;
    if (v.h.k >= 0) {
        if (hi)
            v.t1 = exit_distance(wp, v.at.site, hi[0], hi[1], hi[2], hi[3], hi[4], hi[5]);
        else
            v.t1 = exit_distance(wp, v.at.site, ox, oy, oz, dx, dy, dz);
    }
    const double tm = hi ? hi[6] : (double)tmax;
    v.clipped = (v.h.k < 0) || (v.t1 >= tm);
    v.te = fmax(t0, fmin(v.t1, tm));
    segment<DEG>(t0, Y, v);
}

// Where a logged walk records its visits: visit n of ray r at [n * stride + r]
// (step-major, so the lanes of a wavefront, which advance in lock step, write
// contiguous words), the first `cap` visits only; tail[r] holds the row of the
// cell after the last logged visit (where a longer walk resumes, or the cell
// whose site the last exit gradient needs) and the number of visited cells.
struct LogView {
    uint32_t* code;
    double* te;
    int4* tail;
    int32_t cap;
    int64_t stride;
};

constexpr uint32_t kLogMoves = 1u << 31;    // the exit moves with its face (t0 <= t1 < t_max)
constexpr uint32_t kLogClipped = 1u << 30;  // no front face or t1 >= t_max: the walk ended here
constexpr uint32_t kLogCross = 1u << 29;    // the segment ended at the surface: a new leg follows
constexpr uint32_t kLogCell = kLogCross - 1u;

// ---------------------------------------------------------------------------
// Secondary rays: an analytic sphere (mirror or glass) that bends the walk.
// Where the current leg (o, d) crosses the sphere inside a cell, the segment
// ends at the crossing, and the walk continues in the same cell along the
// reflected or refracted direction, measuring t from the crossing again, up
// to the scene bound. The leg arithmetic is in double and shared by the
// forward and the backward, so both build the same legs bit for bit.
// A leg after a crossing is kept in double (origin, unit direction, t_max):
// its exit distances, clipping and next crossing are computed from that, and
// only the face decisions and the SH basis use its FP32 rounding, so the
// legs are those of the exact reflection and refraction laws up to double
// rounding (a face decision near a tie may still go either way, as for any
// FP32 ray).
// ---------------------------------------------------------------------------
struct Leg {
    double ts;    // distance along the leg to its next crossing, +inf if none
    int inside;   // the leg starts inside the sphere
    int bounces;  // crossings so far
    double hi[7]; // the leg in double: origin, direction, t_max
};

// Next crossing of the leg: the far root of |o + t d - c| = r from inside,
// the near positive root from outside (a leg leaving the surface outwards
// has none).
__device__ inline double surface_hit(const SurfaceArgs& sf, const double* o, const double* d, int inside,
                                     int bounces)
{
    if (bounces >= sf.max_bounces) return INFINITY;
    const double cx = o[0] - sf.centre[0], cy = o[1] - sf.centre[1], cz = o[2] - sf.centre[2];
    const double b = fma(cz, d[2], fma(cy, d[1], cx * d[0]));
    const double r = sf.radius;
    const double c = fma(cz, cz, fma(cy, cy, cx * cx)) - r * r;
    const double disc = b * b - c;
    if (!(disc > 0.0)) return INFINITY;
    const double t = inside ? sqrt(disc) - b : -b - sqrt(disc);
    return t > 0.0 ? t : INFINITY;
}

__device__ inline void leg_start(const SurfaceArgs& sf, float ox, float oy, float oz, float dx, float dy, float dz,
                                 float tmax, Leg& L)
{
    L.hi[0] = ox;
    L.hi[1] = oy;
    L.hi[2] = oz;
    L.hi[3] = dx;
    L.hi[4] = dy;
    L.hi[5] = dz;
    L.hi[6] = tmax;
    const double cx = L.hi[0] - sf.centre[0], cy = L.hi[1] - sf.centre[1], cz = L.hi[2] - sf.centre[2];
    const double r = sf.radius;
    L.inside = fma(cz, cz, fma(cy, cy, cx * cx)) < r * r;
    L.bounces = 0;
    L.ts = surface_hit(sf, L.hi, L.hi + 3, L.inside, 0);
}

// Distance from o along d to the bound (box or sphere about the origin).
__device__ inline double bound_exit(int kind, const float* b, const double o[3], const double d[3])
{
    if (kind == 0) {
        double t = INFINITY;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (d[k] > 0.0) t = fmin(t, ((double)b[3 + k] - o[k]) / d[k]);
            else if (d[k] < 0.0) t = fmin(t, ((double)b[k] - o[k]) / d[k]);
        }
        return fmax(t, 0.0);
    }
    const double bb = fma(o[2], d[2], fma(o[1], d[1], o[0] * d[0]));
    const double c = fma(o[2], o[2], fma(o[1], o[1], o[0] * o[0])) - (double)b[0] * (double)b[0];
    const double disc = bb * bb - c;
    return disc > 0.0 ? fmax(sqrt(disc) - bb, 0.0) : 0.0;
}

// The leg after the crossing at t = L.ts: mirror d' = d - 2 (d.N) N; glass by
// Snell's law with n1/n2 = 1/ior entering and ior leaving (total internal
// reflection when the refracted cosine is imaginary). Updates the leg's
// origin, direction, t_max and crossing state.
// The new leg is kept in L.hi; ox..dz and tmax receive its FP32 rounding.
__device__ inline void surface_turn(const SurfaceArgs& sf, Leg& L, float& ox, float& oy, float& oz, float& dx,
                                    float& dy, float& dz, float& tmax)
{
    const double d[3] = {L.hi[3], L.hi[4], L.hi[5]};
    double p[3], N[3];
    p[0] = fma(L.ts, d[0], L.hi[0]);
    p[1] = fma(L.ts, d[1], L.hi[1]);
    p[2] = fma(L.ts, d[2], L.hi[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) N[k] = p[k] - (double)sf.centre[k];
    const double inv = 1.0 / sqrt(fma(N[2], N[2], fma(N[1], N[1], N[0] * N[0])));
#pragma unroll
    for (int k = 0; k < 3; ++k) N[k] *= inv;
    const double dN = fma(d[2], N[2], fma(d[1], N[1], d[0] * N[0]));
    double dn[3];
    bool reflect = sf.kind == 1;
    if (!reflect) {
        const double sgn = dN < 0.0 ? 1.0 : -1.0;  // sgn N points against d
        const double eta = dN < 0.0 ? 1.0 / (double)sf.ior : (double)sf.ior;
        const double ci = -sgn * dN;
        const double k = 1.0 - eta * eta * (1.0 - ci * ci);
        if (k < 0.0) {
            reflect = true;
        } else {
            const double m = (eta * ci - sqrt(k)) * sgn;
#pragma unroll
            for (int q = 0; q < 3; ++q) dn[q] = fma(eta, d[q], m * N[q]);
            L.inside = !L.inside;
        }
    }
    if (reflect) {
#pragma unroll
        for (int q = 0; q < 3; ++q) dn[q] = fma(-2.0 * dN, N[q], d[q]);
    }
    const double il = 1.0 / sqrt(fma(dn[2], dn[2], fma(dn[1], dn[1], dn[0] * dn[0])));
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        L.hi[q] = p[q];
        L.hi[3 + q] = dn[q] * il;
    }
    L.hi[6] = bound_exit(sf.bound_kind, sf.bound, L.hi, L.hi + 3);
    ox = (float)L.hi[0];
    oy = (float)L.hi[1];
    oz = (float)L.hi[2];
    dx = (float)L.hi[3];
    dy = (float)L.hi[4];
    dz = (float)L.hi[5];
    tmax = (float)L.hi[6];
    ++L.bounces;
    L.ts = surface_hit(sf, L.hi, L.hi + 3, L.inside, L.bounces);
}

// Algorithm 1 for one ray: start in `start`, take the nearest front face of
// each cell, composite the segment with eq. (3)-(4) while T > eps.
template <int DEG, bool BF16, bool TRACE, bool LOG = false>
__device__ inline void walk_forward(const SceneView& s, float ox, float oy, float oz, float dx, float dy, float dz,
                                    float tmax, int start, float eps, int max_steps, int32_t* cells, float* t_exit,
                                    int max_len, RayResult& res, const LogView* lg = nullptr, int64_t r = 0)
{
    res.C[0] = res.C[1] = res.C[2] = 0.0f;
    res.T = 1.0f;
    if (start < 0 || (int64_t)start >= s.n_sites) {
        res.status = -1;
        if constexpr (LOG) lg->tail[r] = make_int4(0, 0, 0, 0);
        return;
    }
    float Y[sh_count(DEG)];
    sh_basis<DEG>(dx, dy, dz, Y);
    uint2 ref = s.row[start];
    uint2 tail = ref;
    double t0 = 0.0;
    float T = 1.0f;
    int n = 0;
    for (;;) {
        if (!(T > eps)) {
            res.status = n;
            break;
        }
        if (n == max_steps) {
            res.status = -2;
            break;
        }
        if constexpr (LOG) {
            if (n == lg->cap) tail = ref;
        }
        Visit<DEG> v;
        visit_cell<DEG, BF16>(s, ref, t0, tmax, ox, oy, oz, dx, dy, dz, Y, v);
        const float w = T * v.alpha;
        res.C[0] = fmaf(w, v.c[0], res.C[0]);
        res.C[1] = fmaf(w, v.c[1], res.C[1]);
        res.C[2] = fmaf(w, v.c[2], res.C[2]);
        T *= expf(-v.tau);
        if constexpr (TRACE) {
            if (n < max_len) {
                cells[n] = ref_cell(ref);
                t_exit[n] = (float)v.te;
            }
        }
        if constexpr (LOG) {
            if (n < lg->cap) {
                const bool moves = !v.clipped && (v.t1 >= t0);
                lg->code[n * lg->stride + r] =
                    (uint32_t)ref_cell(ref) | (moves ? kLogMoves : 0u) | (v.clipped ? kLogClipped : 0u);
                lg->te[n * lg->stride + r] = v.te;
            }
        }
        ++n;
        if (v.clipped) {
            res.status = n;
            break;
        }
        ref = v.h.next;
        t0 = v.te;
    }
    res.T = T;
    if constexpr (LOG) {
        if (n <= lg->cap) tail = ref;
        lg->tail[r] = make_int4((int)tail.x, (int)tail.y, n, 0);
    }
}

// walk_forward with wavefront staging: the loop runs until every lane of the
// wavefront is done, so that all 64 lanes take part in each staging round;
// `live` is false for lanes without a ray. Same arithmetic as walk_forward,
// so the same outputs bit for bit.
// With SURF the walk bends at the surface `sf` (see surface_turn); the
// transmittance test is not repeated for the part of a cell after a crossing.
template <int DEG, bool BF16, bool TRACE, bool LOG, bool SURF = false>
__device__ inline void walk_forward_staged(const SceneView& s, bool live, float ox, float oy, float oz, float dx,
                                           float dy, float dz, float tmax, int start, float eps, int max_steps,
                                           int32_t* cells, float* t_exit, int max_len, RayResult& res,
                                           const LogView* lg, int64_t r, lds_u8* region,
                                           const SurfaceArgs* sf = nullptr)
{
    res.C[0] = res.C[1] = res.C[2] = 0.0f;
    res.T = 1.0f;
    res.status = 0;
    if (live && (start < 0 || (int64_t)start >= s.n_sites)) {
        res.status = -1;
        if constexpr (LOG) lg->tail[r] = make_int4(0, 0, 0, 0);
        live = false;
    }
    const bool logged = live;
    float Y[sh_count(DEG)];
    sh_basis<DEG>(dx, dy, dz, Y);
    uint2 ref = live ? s.row[start] : make_uint2(0u, 0u);
    uint2 tail = ref;
    double t0 = 0.0;
    float T = 1.0f;
    int n = 0;
    Leg leg = {};  // no crossing yet, no bounces (the tail reports leg.bounces)
    leg.ts = INFINITY;
    bool cont = false;  // the visit continues a cell after a crossing
    if constexpr (SURF) {
        if (live) leg_start(*sf, ox, oy, oz, dx, dy, dz, tmax, leg);
    }
    // Rays of one camera share their origin: then the staging computes each
    // face's offset from it once (bent legs have origins of their own)
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    bool shared = false;
    if constexpr (!SURF) {
        const uint64_t lv = ballot(live);
        if (lv) {
            const int l0 = __builtin_ctzll(lv);
            const uint32_t bx = __builtin_amdgcn_readlane(__float_as_uint(ox), l0);
            const uint32_t by = __builtin_amdgcn_readlane(__float_as_uint(oy), l0);
            const uint32_t bz = __builtin_amdgcn_readlane(__float_as_uint(oz), l0);
            shared = ballot(live && (__float_as_uint(ox) != bx || __float_as_uint(oy) != by ||
                                     __float_as_uint(oz) != bz)) == 0;
            sx = __uint_as_float(bx);
            sy = __uint_as_float(by);
            sz = __uint_as_float(bz);
        }
    }
    StageCache cache;
    while (ballot(live)) {
        if (live) {
            if (!cont && !(T > eps)) {
                res.status = n;
                live = false;
            } else if (n == max_steps) {
                res.status = -2;
                live = false;
            }
        }
        int face_slot, rec_slot;
        stage_cells<DEG, BF16>(s, live, ref, region, cache, face_slot, rec_slot, shared, sx, sy, sz);
        if (live) {
            if constexpr (LOG) {
                if (n == lg->cap) tail = ref;
            }
            if constexpr (SURF) {
                // the leg's FP32 rounding for the face scan, taken afresh from
                // the double leg (so that only the double leg stays live)
                ox = (float)leg.hi[0];
                oy = (float)leg.hi[1];
                oz = (float)leg.hi[2];
                dx = (float)leg.hi[3];
                dy = (float)leg.hi[4];
                dz = (float)leg.hi[5];
            }
            Visit<DEG> v;
            visit_cell_staged<DEG, BF16, !TRACE && !LOG && !SURF>(s, ref, face_slot, rec_slot, region, t0, tmax, ox,
                                                                  oy, oz, dx, dy, dz, Y, v, SURF ? leg.hi : nullptr,
                                                                  shared);
            bool cross = false;
            if constexpr (SURF) {
                if (leg.ts < v.te) {
                    // the leg crosses the surface inside this cell
                    cross = true;
                    v.te = leg.ts;
                    v.clipped = false;
                    segment<DEG>(t0, Y, v);
                }
            }
            cont = false;
            const float w = T * v.alpha;
            res.C[0] = fmaf(w, v.c[0], res.C[0]);
            res.C[1] = fmaf(w, v.c[1], res.C[1]);
            res.C[2] = fmaf(w, v.c[2], res.C[2]);
            T *= expf(-v.tau);
            if constexpr (TRACE) {
                if (n < max_len) {
                    cells[n] = ref_cell(ref);
                    t_exit[n] = (float)v.te;
                }
            }
            if constexpr (LOG) {
                if (n < lg->cap) {
                    const bool moves = !v.clipped && !cross && (v.t1 >= t0);
                    lg->code[n * lg->stride + r] = (uint32_t)ref_cell(ref) | (moves ? kLogMoves : 0u) |
                                                   (v.clipped ? kLogClipped : 0u) | (cross ? kLogCross : 0u);
                    lg->te[n * lg->stride + r] = v.te;
                }
            }
            ++n;
            if (v.clipped) {
                res.status = n;
                live = false;
            } else if (cross) {
                if constexpr (SURF) {
                    // a new leg from the crossing, in the same cell
                    surface_turn(*sf, leg, ox, oy, oz, dx, dy, dz, tmax);
                    sh_basis<DEG>(dx, dy, dz, Y);
                    t0 = 0.0;
                    cont = true;
                }
            } else {
                ref = v.h.next;
                t0 = v.te;
            }
        }
        // the next round's copies may overwrite this round's: every lane has read its own
        __builtin_amdgcn_wave_barrier();
    }
    res.T = T;
    if constexpr (LOG) {
        if (logged) {
            if (n <= lg->cap) tail = ref;
            lg->tail[r] = make_int4((int)tail.x, (int)tail.y, n, leg.bounces);
        }
    }
}

// Camera ray through the centre of pixel (px, py). Model 0, pinhole:
// direction R (px + 0.5 - W/2, py + 0.5 - H/2, f) normalised; t_max is where the ray
// leaves the bound (kind 0: box lo=b[0..2], hi=b[3..5]; kind 1: sphere of
// radius b[0] about the world origin).
//
// model 1, equidistant fisheye: the angle from the optical axis is
// proportional to the pixel's distance rho from the image centre,
// theta = rho * focal (focal: radians per pixel), and the camera-frame
// direction is (sin theta u/rho, sin theta v/rho, cos theta).
__device__ inline void camera_ray(const float* rot, const float* pos, int model, float focal, int W, int H, int px,
                                  int py, int bound_kind, const float* bound, float d[3], float* tmax)
{
    const float pu = (float)px + 0.5f - 0.5f * (float)W;
    const float pv = (float)py + 0.5f - 0.5f * (float)H;
    float u, v, w;
    if (model == 1) {
        const float rho = sqrtf(fmaf(pu, pu, pv * pv));
        const float theta = rho * focal;
        const float sr = rho > 0.0f ? sinf(theta) / rho : 0.0f;
        u = sr * pu;
        v = sr * pv;
        w = cosf(theta);
    } else {
        u = pu / focal;
        v = pv / focal;
        w = 1.0f;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = fmaf(rot[3 * k], u, fmaf(rot[3 * k + 1], v, rot[3 * k + 2] * w));
    const float inv = 1.0f / sqrtf(fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2])));
    d[0] *= inv;
    d[1] *= inv;
    d[2] *= inv;
    float t;
    if (bound_kind == 0) {
        t = INFINITY;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (d[k] > 0.0f) t = fminf(t, (bound[3 + k] - pos[k]) / d[k]);
            else if (d[k] < 0.0f) t = fminf(t, (bound[k] - pos[k]) / d[k]);
        }
    } else {
        const float b = fmaf(pos[0], d[0], fmaf(pos[1], d[1], pos[2] * d[2]));
        const float c = fmaf(pos[0], pos[0], fmaf(pos[1], pos[1], pos[2] * pos[2])) - bound[0] * bound[0];
        const float disc = b * b - c;
        t = disc > 0.0f ? sqrtf(disc) - b : 0.0f;
    }
    *tmax = fmaxf(t, 0.0f);
}

}  // namespace rf
