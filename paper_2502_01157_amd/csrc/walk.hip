// The forward and backward Voronoi ray walk (Algorithm 1 and its gradient) for gfx950.
//
// One ray per lane; rays arrive in 8x8 screen-tile order, so a wavefront is
// one tile and its lanes walk mostly the same cells at the same time. The
// forward kernels exploit that: at each step the wavefront copies the face
// rows and records of its lanes' distinct cells into its LDS region once
// (direct global-to-LDS loads) and every lane scans its cell from there.
//
// Per visited cell i the walk
//   1. scans the cell's face planes (one float4 per Delaunay neighbour),
//      keeping the nearest front face: den = n.d > 0 and the smallest
//      t = (c - n.o) / den, compared without division as
//      num_k * den_best < num_best * den_k (ties keep the first face),
//   2. loads the cell's record (SH and density, fp32 or bf16) and composites
//      the segment [t0, te], te = max(t0, min(t1, t_max)), with eq. (3)-(4):
//      C += T (1 - exp(-sigma delta)) c, T *= exp(-sigma delta),
//   3. follows the winning face to the neighbour (its row comes with the face).
// The face the ray came through is never re-taken: its plane seen from the new
// cell is the exact negation of the entry plane, so its den is exactly negative.
//
// The backward pass recomputes the same walk (same code, same rounding) and
// differentiates eq. (3)-(4) in forward order using the saved output colour:
//   R_n = C_out - sum_{k<=n} w_k c_k,  w_n = T_n alpha_n,
//   dL/dtau_n = g.(T_{n+1} c_n - R_n) - g_T T_final,
//   dL/dsigma_i += delta_n dL/dtau_n,   dL/dk_{i,b} += g w_n Y_b,
//   an exit t_n that moves with its face (t0 <= t1 < t_max) gets
//   dL/dt_n = sigma_n dL/dtau_n - sigma_{n+1} dL/dtau_{n+1}, and with
//   p = o + t_n d, den = (x_j - x_i).d:  dt/dx_i = (p - x_i)/den,
//   dt/dx_j = (x_j - p)/den   (geometry enters only through the segment
//   widths, Sec. 3.1).
// A training forward can log each visit (cell and flags, te in double) in a
// step-major walk log; the backward then reads the visits instead of
// repeating the face scans (same records, same te, so the same segments bit
// for bit), and a second launch recomputes only the walks that outgrew the
// log. The exit face's n.d is rebuilt from the two sites (in double), so both
// paths use the same value.
// Each visit's gradients for one cell (3B SH values, density, site) form a
// package that is emitted one iteration later, when the following visit has
// fixed the exit gradient. Packages are summed across the wavefront per cell
// (lanes grouped by ballot, columns summed through LDS) before one coalesced
// float atomic per value and group.

#include "rf_device.hpp"
#include "rf_kernels.hpp"
#include "rf_walk.hpp"

namespace rf {

// ---------------------------------------------------------------------------
// Forward (and traced forward).
// ---------------------------------------------------------------------------
// One wavefront (one screen tile) per block: a block's LDS and slots are
// released as soon as its own walks end (a block of four tiles holds them
// until the longest of its four walks ends: 5-6% slower walks).
constexpr int kWalkBlock = kWave;
__device__ inline int64_t ray_index()
{
    return xcd_block<32>(blockIdx.x, gridDim.x) * kWalkBlock + threadIdx.x;
}

// The staging region (10 KiB per wavefront) allows four wavefronts per SIMD;
// the walks that do not bend keep their registers within that (the logged
// FP32 walk needs 130 and would run three), the bent ones (150-160) run three.
template <int DEG, bool BF16, bool TRACE, bool LOG, bool SURF = false>
__global__ __launch_bounds__(kWalkBlock) __attribute__((amdgpu_waves_per_eu(SURF ? 3 : 4))) void k_forward(WalkArgs a)
{
    using SL = StageLayout<DEG, BF16>;
    __shared__ __align__(16) unsigned char stage_mem[(kWalkBlock / kWave) * SL::kBytes];
    lds_u8* region = (lds_u8*)(stage_mem + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * SL::kBytes);
    const int64_t r = ray_index();
    const bool valid = r < a.n_rays;  // lanes past the end still take part in the staging
    const int64_t q = valid ? r : 0;
    RayResult res;
    const LogView lg = {a.log_code, a.log_te, a.log_tail, a.log_cap, a.n_rays};
    walk_forward_staged<DEG, BF16, TRACE, LOG, SURF>(
        a.s, valid, a.origin[3 * q], a.origin[3 * q + 1], a.origin[3 * q + 2], a.dir[3 * q], a.dir[3 * q + 1],
        a.dir[3 * q + 2], a.t_max[q], a.start[q], a.eps, a.max_steps, TRACE ? a.cells + q * a.max_len : nullptr,
        TRACE ? a.t_exit + q * a.max_len : nullptr, a.max_len, res, &lg, q, region, &a.surf);
    if (!valid) return;
    a.rgb[3 * r + 0] = res.C[0];
    a.rgb[3 * r + 1] = res.C[1];
    a.rgb[3 * r + 2] = res.C[2];
    a.t_final[r] = res.T;
    a.steps[r] = res.status;
}

// ---------------------------------------------------------------------------
// Backward.
// ---------------------------------------------------------------------------

// One cell's gradient package: SH gradient is gw[ch] * Y[b] (rank one).
struct Package {
    int cell;
    float gw[3];
    float dsig;
    float dx[3];
};

template <int DEG>
__device__ inline void emit_atomic(bool has, const Package& p, const float* Y, const WalkArgs& a)
{
    if (!has) return;
    constexpr int B = sh_count(DEG);
    float* gsh = a.g_sh + (size_t)p.cell * 3 * B;
    if (p.gw[0] != 0.0f || p.gw[1] != 0.0f || p.gw[2] != 0.0f) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            unsafeAtomicAdd(gsh + 3 * b + 0, p.gw[0] * Y[b]);
            unsafeAtomicAdd(gsh + 3 * b + 1, p.gw[1] * Y[b]);
            unsafeAtomicAdd(gsh + 3 * b + 2, p.gw[2] * Y[b]);
        }
    }
    unsafeAtomicAdd(a.g_density + p.cell, p.dsig);
    unsafeAtomicAdd(a.g_sites + 3 * (size_t)p.cell + 0, p.dx[0]);
    unsafeAtomicAdd(a.g_sites + 3 * (size_t)p.cell + 1, p.dx[1]);
    unsafeAtomicAdd(a.g_sites + 3 * (size_t)p.cell + 2, p.dx[2]);
}

// Gradient emission of one wavefront, called with every lane active.
//
// Lanes holding a package for the same cell are grouped (leader by ballot).
// Every lane writes its row (Y[0..B-1], gw[0..2], dsig, dx[0..2], 1) once,
// at a position that makes each group's rows contiguous (groups in the order
// of their lowest lane, members in lane order), and for each group lane
// q < 3B+4 sums column q over the group's rows (row addresses are immediate
// offsets from the group's first row, no per-member index arithmetic).
// The group's sums then go into a per-wavefront cache of gradient rows in LDS
// (kSlots rows keyed by cell, first-in first-out): the 64 rays of a tile
// visit only a few hundred distinct cells over their whole walks, each many
// times, so summing in LDS and flushing a row with one coalesced atomic
// instruction when it is evicted (or at the end) replaces most atomics.
// The slot keys live in one register across lanes 0..kSlots-1, so a lookup is
// one ballot. Members are summed in lane order, one fused multiply-add each.
template <int DEG, int SLOTS>
struct EmitLayout {
    static constexpr int B = sh_count(DEG);
    static constexpr int S = (B + 8 + 3) & ~3;  // row stride: whole float4s
    static constexpr int NOUT = 3 * B + 4;
    static constexpr int kSlots = SLOTS;
    static constexpr int FLOATS = kWave * S + kSlots * NOUT;  // per wavefront
};

// PRIO: the wavefront raises its issue priority while it emits, so that
// its chain of dependent ballots and LDS round trips is not held up behind
// the other wavefronts' walks (with four wavefronts per SIMD: BF16
// recomputing backward 10.07 -> 9.94 ms, logged 7.44 -> 7.23 ms; with three
// it gains nothing).
template <int DEG, int SLOTS, bool PRIO = false>
struct Emitter {
    using E = EmitLayout<DEG, SLOTS>;
    float* rows;   // LDS, kWave x S
    float* cache;  // LDS, kSlots x NOUT
    int lane;
    int colA, colB;  // this lane's column: row[colA] * row[colB]
    float* base;     // its destination: base + cell * stride
    int stride;
    int slot_key;    // key of slot `lane` (lanes < kSlots), -1 empty
    int next_slot;   // wavefront-uniform FIFO position

    // lds: the wavefront's E::FLOATS floats of LDS (16-byte aligned)
    __device__ void init(float* lds, int lane_, const WalkArgs& a)
    {
        constexpr int B = E::B;
        rows = lds;
        cache = lds + kWave * E::S;
        lane = lane_;
        if (lane < 3 * B) {
            colA = lane / 3;
            colB = B + lane % 3;
            base = a.g_sh + lane;
            stride = 3 * B;
        } else if (lane == 3 * B) {
            colA = B + 3;
            colB = B + 7;
            base = a.g_density;
            stride = 1;
        } else {
            const int q = min(lane - 3 * B - 1, 2);
            colA = B + 4 + q;
            colB = B + 7;
            base = a.g_sites + q;
            stride = 3;
        }
        slot_key = -1;
        next_slot = 0;
    }

    // Sum over the group's rows first..first+m-1 of this lane's column product,
    // in row order. The last batch of fewer than four rows reads past the
    // group (at most two rows past the wavefront's 64, into its cache rows)
    // and keeps only its own rows' terms.
    __device__ float column_sum(int first, int m) const
    {
        const float* pa = rows + first * E::S + colA;
        const float* pb = rows + first * E::S + colB;
        float acc = 0.0f;
        int q = 0;
        for (; q + 4 <= m; q += 4) {
            float va[4], vb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                va[u] = pa[(q + u) * E::S];
                vb[u] = pb[(q + u) * E::S];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = fmaf(va[u], vb[u], acc);
        }
        if (q < m) {
            float va[3], vb[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                va[u] = pa[(q + u) * E::S];
                vb[u] = pb[(q + u) * E::S];
            }
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const float t = fmaf(va[u], vb[u], acc);
                acc = q + u < m ? t : acc;
            }
        }
        return acc;
    }

    // Adds the wavefront's column sums for `key` to its cache row, evicting
    // (flushing) the oldest row when the cell has none.
    __device__ void accumulate(int key, float acc)
    {
        // (lanes past kSlots hold no key: slot_key stays -1 there, and keys are cells >= 0)
        const uint64_t hit = ballot(slot_key == key);
        if (hit) {
            // each lane owns its column, so the add needs no result and no wait
            const int slot = __builtin_ctzll(hit);
            if (lane < E::NOUT) cache[slot * E::NOUT + lane] += acc;
            return;
        }
        const int slot = next_slot;
        next_slot = next_slot + 1 == E::kSlots ? 0 : next_slot + 1;
        const int old = __builtin_amdgcn_readlane(slot_key, slot);
        if (lane < E::NOUT) {
            if (old >= 0) {
                const float v = cache[slot * E::NOUT + lane];
                if (v != 0.0f) unsafeAtomicAdd(base + (size_t)old * stride, v);
            }
            cache[slot * E::NOUT + lane] = acc;
        }
        if (lane == slot) slot_key = key;
    }

    // Emits the lanes' packages; Y is each lane's SH basis for its package.
    __device__ void emit(bool has, const Package& p, const float* Y)
    {
        constexpr int B = E::B;
        uint64_t pend = ballot(has);
        if (pend == 0) return;
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
        const int key_cell = has ? p.cell : -1;
        // each member's row: the groups in the order of their lowest lane,
        // the members of a group in lane order
        int pos = 0;
        {
            uint64_t rest = pend;
            int first = 0;
            while (rest) {
                const int key = __builtin_amdgcn_readlane(key_cell, __builtin_ctzll(rest));
                const uint64_t ma = ballot(key_cell == key) & rest;
                rest &= ~ma;
                if (key_cell == key)
                    pos = first + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
                first += __popcll(ma);
            }
        }
        if (has) {
            float v[E::S];
#pragma unroll
            for (int b = 0; b < B; ++b) v[b] = Y[b];
            v[B + 0] = p.gw[0];
            v[B + 1] = p.gw[1];
            v[B + 2] = p.gw[2];
            v[B + 3] = p.dsig;
            v[B + 4] = p.dx[0];
            v[B + 5] = p.dx[1];
            v[B + 6] = p.dx[2];
            v[B + 7] = 1.0f;
#pragma unroll
            for (int c = B + 8; c < E::S; ++c) v[c] = 0.0f;
            float4* row = reinterpret_cast<float4*>(rows + pos * E::S);
#pragma unroll
            for (int c = 0; c < E::S / 4; ++c) row[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int first = 0;
        while (pend) {
            const int key = __builtin_amdgcn_readlane(key_cell, __builtin_ctzll(pend));
            const uint64_t ma = ballot(key_cell == key) & pend;
            pend &= ~ma;
            const int m = __popcll(ma);
            const float acc = column_sum(first, m);
            first += m;
            accumulate(key, acc);
        }
        // the next emission's rows overwrite these
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    }

    // Flushes every cached row (at the end of the wavefront's walks).
    __device__ void flush()
    {
        for (int slot = 0; slot < E::kSlots; ++slot) {
            const int key = __builtin_amdgcn_readlane(slot_key, slot);
            if (key < 0) continue;
            if (lane < E::NOUT) {
                const float v = cache[slot * E::NOUT + lane];
                if (v != 0.0f) unsafeAtomicAdd(base + (size_t)key * stride, v);
            }
        }
    }
};

// Offsets of the exit point p = o + t d from the two sites of the face, formed
// in double so that p - x does not lose the digits of |o| + t.
__device__ inline void exit_offsets(double t, double ox, double oy, double oz, double dx, double dy, double dz,
                                    const float* xa, const float* xb, float* pa, float* pb)
{
    const double o[3] = {ox, oy, oz}, d[3] = {dx, dy, dz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pa[k] = (float)fma(t, d[k], o[k] - (double)xa[k]);
        pb[k] = (float)fma(t, d[k], o[k] - (double)xb[k]);
    }
}

// The plain reducing backward with BF16 attributes runs 4 wavefronts per SIMD,
// which needs the wavefront's LDS within 10 KiB: 19 gradient-cache rows
// instead of 32 (measured on the clustered 1M-site frame: the logged backward
// 7.53 -> 7.10 ms, the recomputing one 11.25 -> 10.03 ms). With FP32
// attributes, or with the quantile or surface terms, the registers spilled at
// 4 wavefronts cost more than the extra wavefront hides (FP32 logged: 7.83 ->
// 8.73 ms), so those keep 3 wavefronts and 32 rows.
constexpr bool four_waves(bool bf16, bool reduce, bool surf, bool quant)
{
    return bf16 && reduce && !surf && !quant;
}

// With SURF the walks bend at the surface as in the forward: each crossing
// (logged, or found again by the recomputing walk) turns the leg with the
// same arithmetic, and the colour of the next visits uses the new leg's
// basis; the crossing visit's package is emitted in its own iteration, before
// the lane's basis turns, since nothing after the crossing changes it.
// QUANT = false leaves out the quantile regulariser's terms (and their 13
// registers) for calls without them. CHECK = true (a recomputing walk with a
// mismatch counter) compares each recomputed walk's final transmittance and
// status with the forward's; it is a separate instantiation because its
// registers cost the four-wavefront BF16 kernel 12 bytes more of spills.
template <int DEG, bool BF16, bool REDUCE, bool LOG, bool SURF = false, bool QUANT = true, bool CHECK = false>
__global__ __launch_bounds__(kWalkBlock) __attribute__((amdgpu_waves_per_eu(four_waves(BF16, REDUCE, SURF, QUANT) ? 4 : 3)))
void k_backward(WalkArgs a)
{
    constexpr int B = sh_count(DEG);
    constexpr int kSlots = four_waves(BF16, REDUCE, SURF, QUANT) ? 19 : 32;
    using E = EmitLayout<DEG, kSlots>;
    static_assert(REDUCE || !SURF, "bent walks emit through the wavefront reduction");
    __shared__ __align__(16) float lds[REDUCE ? (kWalkBlock / kWave) * E::FLOATS : 1];
    const int lane = threadIdx.x & (kWave - 1);
    Emitter<DEG, kSlots, four_waves(BF16, REDUCE, SURF, QUANT)> em;
    if constexpr (REDUCE) em.init(lds + (threadIdx.x / kWave) * E::FLOATS, lane, a);

    const int64_t r = ray_index();
    // lane state: 0 walking, 1 emit the last visit, 2 emit the next cell's entry term, 3 done
    int state = 3;
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 1, tmax = 0;
    float g[3] = {0, 0, 0}, gT = 0, Cout[3] = {0, 0, 0}, Tfin = 1;
    uint2 ref = make_uint2(0, 0);
    int n_total = 0;  // visited cells of the logged forward
    if (r < a.n_rays) {
        const int start = a.start[r];
        if (start >= 0 && (int64_t)start < a.s.n_sites) {
            state = 0;
            ox = a.origin[3 * r];
            oy = a.origin[3 * r + 1];
            oz = a.origin[3 * r + 2];
            dx = a.dir[3 * r];
            dy = a.dir[3 * r + 1];
            dz = a.dir[3 * r + 2];
            tmax = a.t_max[r];
            g[0] = a.grad_rgb[3 * r];
            g[1] = a.grad_rgb[3 * r + 1];
            g[2] = a.grad_rgb[3 * r + 2];
            gT = a.grad_t ? a.grad_t[r] : 0.0f;
            Cout[0] = a.rgb_in[3 * r];
            Cout[1] = a.rgb_in[3 * r + 1];
            Cout[2] = a.rgb_in[3 * r + 2];
            Tfin = a.t_final_in[r];
            ref = a.s.row[start];
            if (a.log_tail) {
                // a logged walk: the log kernel takes the rays whose visits
                // are all in the log, the recompute kernel the longer ones
                const int4 tl = a.log_tail[r];
                const bool in_log = tl.z >= 0 && tl.z <= a.log_cap;
                if (LOG) {
                    ref = make_uint2((uint32_t)tl.x, (uint32_t)tl.y);  // the cell after the last visit
                    n_total = tl.z;
                }
                if (in_log != LOG) state = 3;
            }
        }
    }
    float Y[B];
    sh_basis<DEG>(dx, dy, dz, Y);
    Leg leg = {};  // no crossing yet, no bounces (the tail reports leg.bounces)
    leg.ts = INFINITY;
    bool cont = false;    // the next visit continues a cell after a crossing
    bool turned = false;  // this visit ended at the surface: the leg has turned, Y has not yet
    if constexpr (SURF) {
        if (state == 0) leg_start(a.surf, ox, oy, oz, dx, dy, dz, tmax, leg);
    }

    // quantile regulariser, if requested: with D = u T_f / (1 - u + u T_f)
    // (dL/dtau_total of L = -ln(1 - u A)) and the quantile's visit k, density
    // sigma_k, t = t0_k + (L - tau_<k) / sigma_k gives, for a loss gradient c,
    // dtau_n += c (D - [n < k]) / sigma_k, plus the two terms outside tau:
    // dsigma_k -= c (t - t0_k) / sigma_k and the exit before k moves t by c.
    float qc[2] = {0.0f, 0.0f}, qD[2] = {0.0f, 0.0f}, qs[2] = {1.0f, 1.0f}, qt[2] = {0.0f, 0.0f};
    int qk[2] = {-1, -1};
    if (QUANT && state == 0 && a.grad_q) {
        const float t_a = a.q_t[2 * r], t_b = a.q_t[2 * r + 1];
        const int k_a = a.q_seg[2 * r], k_b = a.q_seg[2 * r + 1];
        if (k_a >= 0 && k_b >= 0 && t_a != t_b) {
            const float sg = t_a > t_b ? a.grad_q[r] : -a.grad_q[r];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const float u = a.q_u[2 * r + j];
                qc[j] = j == 0 ? sg : -sg;
                qD[j] = u * Tfin / (1.0f - u + u * Tfin);
                qs[j] = a.q_sig[2 * r + j];
                qt[j] = a.q_t[2 * r + j];
                qk[j] = a.q_seg[2 * r + j];
            }
        }
    }

    float T = 1.0f, Cacc[3] = {0.0f, 0.0f, 0.0f};
    double t0 = 0.0;
    int n = 0;
    // the log entry of visit n, loaded one visit ahead
    uint32_t pf_code = 0;
    double pf_te = 0.0;
    if (LOG && state == 0 && n_total > 0) {
        pf_code = a.log_code[r];
        pf_te = a.log_te[r];
    }
    // previous visit, awaiting its exit gradient
    bool have_prev = false, p_moves = false;
    Package prev = {0, {0, 0, 0}, 0, {0, 0, 0}};
    float p_site[3] = {0, 0, 0}, p_sdt = 0;
    double p_t1 = 0.0;
    // entry term of the cell after the last visit
    Package entry = {0, {0, 0, 0}, 0, {0, 0, 0}};
    bool entry_valid = false;

    int status = 0;  // the recomputed walk's status, as the forward reports it in steps
    while (ballot(state != 3)) {
        bool has = false;
        Package out = prev;
        bool stop = false;
        if (state == 0) {
            if constexpr (LOG) {
                stop = (n == n_total);
            } else if (!cont && !(T > a.eps)) {
                stop = true;
                if constexpr (CHECK) status = n;
            } else if (n == a.max_steps) {
                stop = true;
                if constexpr (CHECK) status = -2;  // max_steps cells visited with T > eps, as the forward flags it
            }
        }
        if (state == 0) {
            if (!stop) {
                Visit<DEG> v;
                int cell;
                bool moves, cross = false;
                cont = false;
                if constexpr (LOG) {
                    // the visit as the forward logged it: same record, same te,
                    // so the same segment bit for bit, without the face scan
                    const uint32_t code = pf_code;
                    v.te = pf_te;
                    cell = min((int)(code & kLogCell), (int)(a.s.n_sites - 1));
                    load_record<DEG, BF16>(a.s.rec, cell, v.at);
                    // the next visit's entry, issued after the record loads so
                    // that waiting for the record does not wait for it (loads
                    // complete in issue order)
                    // (unconditional, so that the wait counts stay exact: the
                    // last visit reloads its own entry)
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t nxt = (int64_t)(n + 1 < n_total ? n + 1 : n) * a.n_rays + r;
                    pf_code = a.log_code[nxt];
                    pf_te = a.log_te[nxt];
                    v.t1 = v.te;  // a moving exit is unclamped: te = t1
                    v.clipped = (code & kLogClipped) != 0;
                    moves = (code & kLogMoves) != 0;
                    if constexpr (SURF) {
                        cross = (code & kLogCross) != 0;
                        if (cross) leg.ts = v.te;  // the crossing as the forward found it
                    }
                    segment<DEG>(t0, Y, v);
                } else {
                    cell = ref_cell(ref);
                    if constexpr (SURF) {
                        ox = (float)leg.hi[0];
                        oy = (float)leg.hi[1];
                        oz = (float)leg.hi[2];
                        dx = (float)leg.hi[3];
                        dy = (float)leg.hi[4];
                        dz = (float)leg.hi[5];
                    }
                    visit_cell<DEG, BF16>(a.s, ref, t0, tmax, ox, oy, oz, dx, dy, dz, Y, v, SURF ? leg.hi : nullptr);
                    if constexpr (SURF) {
                        if (leg.ts < v.te) {
                            cross = true;
                            v.te = leg.ts;
                            v.clipped = false;
                            segment<DEG>(t0, Y, v);
                        }
                    }
                    moves = !v.clipped && !cross && (v.t1 >= t0);
                }
                const Attr<DEG>& at = v.at;
                const float w = T * v.alpha;
                Cacc[0] = fmaf(w, v.c[0], Cacc[0]);
                Cacc[1] = fmaf(w, v.c[1], Cacc[1]);
                Cacc[2] = fmaf(w, v.c[2], Cacc[2]);
                const float Tn = T * expf(-v.tau);
                float dtau = -gT * Tfin;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dtau = fmaf(g[ch], Tn * v.c[ch] - (Cout[ch] - Cacc[ch]), dtau);
                float dsig_q = 0.0f, gt_q = 0.0f;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (QUANT && qc[j] != 0.0f) {
                        dtau += qc[j] * (qD[j] - (n < qk[j] ? 1.0f : 0.0f)) / qs[j];
                        if (n == qk[j]) {
                            dsig_q -= qc[j] * (float)((double)qt[j] - t0) / qs[j];
                            gt_q += qc[j];
                        }
                    }
                }
                const float sdt = at.sigma * dtau;
                float edx[3] = {0.0f, 0.0f, 0.0f};
                if (have_prev) {
                    if (p_moves) {
                        // exit point relative to both sites, in double: p - x = (o - x) + t d
                        const float gt = p_sdt - sdt + gt_q;
                        float pa[3], pb[3];
                        float s;
                        if constexpr (SURF) {
                            s = (float)((double)gt / face_den(p_site, at.site, leg.hi[3], leg.hi[4], leg.hi[5]));
                            exit_offsets(p_t1, leg.hi[0], leg.hi[1], leg.hi[2], leg.hi[3], leg.hi[4], leg.hi[5],
                                         p_site, at.site, pa, pb);
                        } else {
                            s = (float)((double)gt / face_den(p_site, at.site, dx, dy, dz));
                            exit_offsets(p_t1, ox, oy, oz, dx, dy, dz, p_site, at.site, pa, pb);
                        }
                        prev.dx[0] = fmaf(s, pa[0], prev.dx[0]);
                        prev.dx[1] = fmaf(s, pa[1], prev.dx[1]);
                        prev.dx[2] = fmaf(s, pa[2], prev.dx[2]);
                        edx[0] = -s * pb[0];
                        edx[1] = -s * pb[1];
                        edx[2] = -s * pb[2];
                    }
                    has = true;
                    out = prev;
                }
                prev.cell = cell;
                prev.gw[0] = g[0] * w;
                prev.gw[1] = g[1] * w;
                prev.gw[2] = g[2] * w;
                prev.dsig = fmaf(v.delta, dtau, dsig_q);
                prev.dx[0] = edx[0];
                prev.dx[1] = edx[1];
                prev.dx[2] = edx[2];
                p_site[0] = at.site[0];
                p_site[1] = at.site[1];
                p_site[2] = at.site[2];
                p_t1 = v.t1;
                p_sdt = sdt;
                p_moves = moves;
                have_prev = true;
                T = Tn;
                ++n;
                if (v.clipped) {
                    stop = true;
                    if constexpr (CHECK) status = n;
                } else if (cross) {
                    if constexpr (SURF) {
                        // a new leg from the crossing, in the same cell; the
                        // crossing's exit does not move, so nothing links the
                        // two legs' gradients (the basis turns after this
                        // iteration's emissions, which still need the old one)
                        surface_turn(a.surf, leg, ox, oy, oz, dx, dy, dz, tmax);
                        t0 = 0.0;
                        cont = true;
                        turned = true;
                    }
                } else {
                    if (!LOG) ref = v.h.next;
                    t0 = v.te;
                }
            }
            if (stop) {
                if constexpr (CHECK && !LOG) {
                    // consistency of the recomputation: the same final
                    // transmittance (bit for bit) and visit count as the forward's
                    if (__float_as_uint(T) != __float_as_uint(Tfin) || (a.steps_in && a.steps_in[r] != status))
                        atomicAdd(a.mismatch, 1);
                }
                if (have_prev && p_moves) {
                    // the last exit moved with its face but no segment follows it
                    float xj[3], pa[3], pb[3];
                    // (kept in range, so that a log not written by the forward
                    // cannot address outside the scene)
                    entry.cell = min(ref_cell(ref), (int)(a.s.n_sites - 1));
                    load_site<DEG, BF16>(a.s.rec, entry.cell, xj);
                    float s;
                    if constexpr (SURF) {
                        s = (float)((double)p_sdt / face_den(p_site, xj, leg.hi[3], leg.hi[4], leg.hi[5]));
                        exit_offsets(p_t1, leg.hi[0], leg.hi[1], leg.hi[2], leg.hi[3], leg.hi[4], leg.hi[5], p_site,
                                     xj, pa, pb);
                    } else {
                        s = (float)((double)p_sdt / face_den(p_site, xj, dx, dy, dz));
                        exit_offsets(p_t1, ox, oy, oz, dx, dy, dz, p_site, xj, pa, pb);
                    }
                    prev.dx[0] = fmaf(s, pa[0], prev.dx[0]);
                    prev.dx[1] = fmaf(s, pa[1], prev.dx[1]);
                    prev.dx[2] = fmaf(s, pa[2], prev.dx[2]);
                    entry.dx[0] = -s * pb[0];
                    entry.dx[1] = -s * pb[1];
                    entry.dx[2] = -s * pb[2];
                    entry_valid = true;
                }
                state = have_prev ? 1 : 3;
            }
        } else if (state == 1) {
            has = true;
            out = prev;
            state = entry_valid ? 2 : 3;
        } else if (state == 2) {
            has = true;
            out = entry;
            state = 3;
        }
        if constexpr (REDUCE)
            em.emit(has, out, Y);
        else
            emit_atomic<DEG>(has, out, Y, a);
        if constexpr (SURF) {
            // a crossing's package is complete when its visit ends (its exit
            // does not move), so it goes out now, with the old leg's basis,
            // and the lane's basis turns with the leg
            if (ballot(turned)) {
                em.emit(turned, prev, Y);
                if (turned) {
                    sh_basis<DEG>(dx, dy, dz, Y);
                    have_prev = false;
                    turned = false;
                }
            }
        }
    }
    if constexpr (REDUCE) em.flush();
}

// ---------------------------------------------------------------------------
// Quantile regulariser (Sec. 3.4): W^-1(u) of the normalised weight
// distribution along a ray. With W(t) = 1 - exp(-tau(t)) (constant density in
// a cell) and A = 1 - T_final, W(t) = u A exactly where the accumulated
// optical depth reaches L = -ln(1 - u A), so the quantile lies in the first
// weighted segment k whose depth crosses L, at t0_k + (L - tau_<k) / sigma_k.
// The visits come from the walk log (one density gather per visit); a walk
// longer than the log is walked again.
// ---------------------------------------------------------------------------
struct QuantileScan {
    float L[2];
    bool found[2] = {false, false};
    int seg[2] = {-1, -1};
    float sig[2] = {0.0f, 0.0f};
    double t[2] = {0.0, 0.0};
    float tau_cum = 0.0f;
    int last = -1;  // last weighted visit
    float last_sig = 0.0f;
    double last_te = 0.0;

    __device__ void visit(int n, float sigma, double t0, double te, float tau)
    {
        if (tau > 0.0f) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!found[j] && tau_cum + tau >= L[j]) {
                    found[j] = true;
                    seg[j] = n;
                    sig[j] = sigma;
                    t[j] = fmin(fmax(t0 + (double)((L[j] - tau_cum) / sigma), t0), te);
                }
            }
            last = n;
            last_sig = sigma;
            last_te = te;
        }
        tau_cum += tau;
    }

    __device__ void finish()
    {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (!found[j] && last >= 0) {  // u A beyond the rounded total depth
                seg[j] = last;
                sig[j] = last_sig;
                t[j] = last_te;
            }
        }
    }
};

template <int DEG, bool BF16>
__global__ __launch_bounds__(kWalkBlock) void k_quantile(WalkArgs a)
{
    const int64_t r = ray_index();
    if (r >= a.n_rays) return;
    QuantileScan q;
    const int start = a.start[r];
    const float A = 1.0f - a.t_final_in[r];
    if (start >= 0 && (int64_t)start < a.s.n_sites && A > 0.0f) {
        q.L[0] = -log1pf(-a.q_u[2 * r] * A);
        q.L[1] = -log1pf(-a.q_u[2 * r + 1] * A);
        const int4 tl = a.log_tail[r];
        if (tl.w != 0) {
            // a bent walk (surface crossings): the quantiles are defined along one leg only
        } else if (tl.z >= 0 && tl.z <= a.log_cap) {
            double t0 = 0.0;
            for (int n = 0; n < tl.z; ++n) {
                const uint32_t code = a.log_code[(int64_t)n * a.n_rays + r];
                const double te = a.log_te[(int64_t)n * a.n_rays + r];
                const float sigma = load_sigma<DEG, BF16>(a.s.rec, min((int)(code & kLogCell), (int)(a.s.n_sites - 1)));
                const float delta = (float)(te - t0);
                q.visit(n, sigma, t0, te, sigma > 0.0f ? sigma * delta : 0.0f);
                t0 = te;
            }
        } else {
            // the walk outgrew the log: walk it again (same visits as the forward)
            const float ox = a.origin[3 * r], oy = a.origin[3 * r + 1], oz = a.origin[3 * r + 2];
            const float dx = a.dir[3 * r], dy = a.dir[3 * r + 1], dz = a.dir[3 * r + 2];
            float Y[sh_count(DEG)];
            sh_basis<DEG>(dx, dy, dz, Y);
            uint2 ref = a.s.row[start];
            double t0 = 0.0;
            float T = 1.0f;
            for (int n = 0; T > a.eps && n < a.max_steps; ++n) {
                Visit<DEG> v;
                visit_cell<DEG, BF16>(a.s, ref, t0, a.t_max[r], ox, oy, oz, dx, dy, dz, Y, v);
                q.visit(n, v.at.sigma, t0, v.te, v.tau);
                T *= expf(-v.tau);
                if (v.clipped) break;
                ref = v.h.next;
                t0 = v.te;
            }
        }
        q.finish();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        a.q_t[2 * r + j] = (float)q.t[j];
        a.q_seg[2 * r + j] = q.seg[j];
        a.q_sig[2 * r + j] = q.sig[j];
    }
    a.q_loss[r] = (q.seg[0] >= 0 && q.seg[1] >= 0) ? fabsf((float)q.t[0] - (float)q.t[1]) : 0.0f;
}

// ---------------------------------------------------------------------------
// Dispatch.
// ---------------------------------------------------------------------------
template <int DEG, bool BF16>
static hipError_t launch_walk_t(WalkKind kind, const WalkArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.n_rays + kWalkBlock - 1) / kWalkBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kWalkBlock);
    switch (kind) {
    case kForward:
        hipLaunchKernelGGL((k_forward<DEG, BF16, false, false>), grid, block, 0, stream, a);
        break;
    case kTrace:
        hipLaunchKernelGGL((k_forward<DEG, BF16, true, false>), grid, block, 0, stream, a);
        break;
    case kForwardLog:
        hipLaunchKernelGGL((k_forward<DEG, BF16, false, true>), grid, block, 0, stream, a);
        break;
    case kBackwardReduce:
        if (a.grad_q)
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, false>), grid, block, 0, stream, a);
        else if (a.mismatch)
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, false, false, false, true>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, false, false, false>), grid, block, 0, stream, a);
        break;
    case kBackwardAtomic:
        if (a.mismatch)
            hipLaunchKernelGGL((k_backward<DEG, BF16, false, false, false, true, true>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_backward<DEG, BF16, false, false>), grid, block, 0, stream, a);
        break;
    case kBackwardLogReduce:
        // rays within the log, then the rays whose walks outgrew it (recomputed)
        if (a.grad_q) {
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, true>), grid, block, 0, stream, a);
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, false>), grid, block, 0, stream, a);
        } else {
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, true, false, false>), grid, block, 0, stream, a);
            hipLaunchKernelGGL((k_backward<DEG, BF16, true, false, false, false>), grid, block, 0, stream, a);
        }
        break;
    case kBackwardLogAtomic:
        hipLaunchKernelGGL((k_backward<DEG, BF16, false, true>), grid, block, 0, stream, a);
        hipLaunchKernelGGL((k_backward<DEG, BF16, false, false>), grid, block, 0, stream, a);
        break;
    case kQuantile:
        hipLaunchKernelGGL((k_quantile<DEG, BF16>), grid, block, 0, stream, a);
        break;
    case kForwardSurf:
        hipLaunchKernelGGL((k_forward<DEG, BF16, false, false, true>), grid, block, 0, stream, a);
        break;
    case kForwardLogSurf:
        hipLaunchKernelGGL((k_forward<DEG, BF16, false, true, true>), grid, block, 0, stream, a);
        break;
    case kBackwardSurf:
        hipLaunchKernelGGL((k_backward<DEG, BF16, true, false, true>), grid, block, 0, stream, a);
        break;
    case kBackwardLogSurf:
        hipLaunchKernelGGL((k_backward<DEG, BF16, true, true, true>), grid, block, 0, stream, a);
        hipLaunchKernelGGL((k_backward<DEG, BF16, true, false, true>), grid, block, 0, stream, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_walk(WalkKind kind, int sh_degree, bool bf16, const WalkArgs& a, hipStream_t stream)
{
    switch (sh_degree * 2 + (bf16 ? 1 : 0)) {
    case 0: return launch_walk_t<0, false>(kind, a, stream);
    case 1: return launch_walk_t<0, true>(kind, a, stream);
    case 2: return launch_walk_t<1, false>(kind, a, stream);
    case 3: return launch_walk_t<1, true>(kind, a, stream);
    case 4: return launch_walk_t<2, false>(kind, a, stream);
    case 5: return launch_walk_t<2, true>(kind, a, stream);
    case 6: return launch_walk_t<3, false>(kind, a, stream);
    case 7: return launch_walk_t<3, true>(kind, a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace rf
