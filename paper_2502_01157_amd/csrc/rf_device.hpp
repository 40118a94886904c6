// Device-side building blocks of the Voronoi ray walk for gfx950 (CDNA4).
//
// Packed scene layout (all sections 256-byte aligned inside one workspace):
//   planes  float4[E]  per directed Delaunay edge (i -> j), in CSR order:
//                      n = x_j - x_i and c = n . (x_i + x_j) / 2, so the
//                      bisector of the two sites (the shared Voronoi face,
//                      eq. (5)) is {p : n.p = c} and cell i is the side n.p < c.
//   adj     uint2[E]   the neighbour's row: x = j | deg_j << 24, y = off_j.
//   row     uint2[N]   the same reference for every cell (used for start cells).
//   rec     N records  SH coefficients and density (fp32 or bf16) and the
//                      site (always fp32); record size is a power of two so a
//                      record never straddles more 128-byte lines than needed.
//   err     int32[2]   validation counters written by the pack kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rf {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // block of the point-location kernel (the walks run one wavefront per block)

__host__ __device__ constexpr int sh_count(int deg) { return (deg + 1) * (deg + 1); }

__host__ __device__ constexpr int pow2_at_least(int v, int lo)
{
    int p = lo;
    while (p < v) p *= 2;
    return p;
}

// Per-cell record geometry for SH degree DEG and storage BF16 (else fp32).
template <int DEG, bool BF16>
struct Rec {
    static constexpr int B = sh_count(DEG);
    static constexpr int NSH = 3 * B;                              // SH values, [b][rgb]
    static constexpr int ATTR_BYTES = (BF16 ? 2 : 4) * (NSH + 1);  // SH then density
    static constexpr int SITE_OFF = (ATTR_BYTES + 3) & ~3;         // fp32 x, y, z
    static constexpr int USED = SITE_OFF + 12;
    static constexpr int BYTES = pow2_at_least(USED, 32);
    static constexpr int CHUNKS = (USED + 15) / 16;                // uint4 loads per record
};

__host__ __device__ inline int rec_bytes(int deg, bool bf16)
{
    const int nsh = 3 * sh_count(deg);
    const int attr = (bf16 ? 2 : 4) * (nsh + 1);
    const int used = ((attr + 3) & ~3) + 12;
    return pow2_at_least(used, 32);
}

__host__ __device__ inline int rec_site_off(int deg, bool bf16)
{
    const int nsh = 3 * sh_count(deg);
    return (((bf16 ? 2 : 4) * (nsh + 1)) + 3) & ~3;
}

// ---------------------------------------------------------------------------
// bf16 storage: round to nearest even on the way in, exact widening on the way out.
// ---------------------------------------------------------------------------
__device__ inline uint32_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x0040u;  // quiet NaN
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Mask of the active lanes whose predicate holds. The builtin takes the
// predicate as the compare's lane mask; HIP's __ballot(int) widens it to an
// integer and compares that again (two more VALU instructions per ballot).
__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Unpacked attributes of one cell.
template <int DEG>
struct Attr {
    float sh[3 * sh_count(DEG)];
    float sigma;
    float site[3];
};

// LDS pointers (address space 3) for data staged by a wavefront; 16-byte LDS
// elements are read as native vectors (HIP's vector classes do not copy from
// address-space-qualified references).
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) void lds_void;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const f32x4 lds_f32x4;
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;

// Direct global-to-LDS load of 16 bytes per active lane: lane i writes
// dst + 16 i (dst must be the same for every lane of the wavefront).
__device__ inline void copy16_to_lds(const void* src, lds_u8* dst)
{
    __builtin_amdgcn_global_load_lds(src, (lds_void*)dst, 16, 0, 0);
}

// The same through a buffer descriptor of `bytes` bytes at the wavefront-
// uniform address `base` (built with scalar instructions): each active lane
// loads the 16 bytes at base + lane_offset and writes dst + 16 i.
__device__ inline void copy16_to_lds(const void* base, uint32_t bytes, uint32_t lane_offset, lds_u8* dst)
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)dst, 16, lane_offset, 0, 0, 0);
}

__device__ inline float4 ld16(const float4* p) { return *p; }
__device__ inline uint4 ld16(const uint4* p) { return *p; }
__device__ inline float4 ld16(lds_f32x4* p)
{
    const f32x4 v = *p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline uint4 ld16(lds_u32x4* p)
{
    const u32x4 v = *p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Unpacks a record from its 16-byte chunks, read through P (a global or an
// LDS pointer).
template <int DEG, bool BF16, typename P>
__device__ inline void unpack_record(P p, Attr<DEG>& a)
{
    using R = Rec<DEG, BF16>;
    uint32_t w[4 * R::CHUNKS];
#pragma unroll
    for (int c = 0; c < R::CHUNKS; ++c) {
        const uint4 v = ld16(p + c);
        w[4 * c + 0] = v.x;
        w[4 * c + 1] = v.y;
        w[4 * c + 2] = v.z;
        w[4 * c + 3] = v.w;
    }
    if constexpr (BF16) {
#pragma unroll
        for (int k = 0; k < R::NSH; ++k) a.sh[k] = (k & 1) ? bf16_hi(w[k >> 1]) : bf16_lo(w[k >> 1]);
        a.sigma = (R::NSH & 1) ? bf16_hi(w[R::NSH >> 1]) : bf16_lo(w[R::NSH >> 1]);
    } else {
#pragma unroll
        for (int k = 0; k < R::NSH; ++k) a.sh[k] = __uint_as_float(w[k]);
        a.sigma = __uint_as_float(w[R::NSH]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) a.site[k] = __uint_as_float(w[R::SITE_OFF / 4 + k]);
}

template <int DEG, bool BF16>
__device__ inline void load_record(const unsigned char* __restrict__ rec_base, int cell, Attr<DEG>& a)
{
    using R = Rec<DEG, BF16>;
    unpack_record<DEG, BF16>(reinterpret_cast<const uint4*>(rec_base + (size_t)cell * R::BYTES), a);
}

template <int DEG, bool BF16>
__device__ inline void load_site(const unsigned char* __restrict__ rec_base, int cell, float s[3])
{
    using R = Rec<DEG, BF16>;
    const float* p = reinterpret_cast<const float*>(rec_base + (size_t)cell * R::BYTES + R::SITE_OFF);
    s[0] = p[0];
    s[1] = p[1];
    s[2] = p[2];
}

// The density of a cell (exactly as unpack_record widens it).
template <int DEG, bool BF16>
__device__ inline float load_sigma(const unsigned char* __restrict__ rec_base, int cell)
{
    using R = Rec<DEG, BF16>;
    const unsigned char* p = rec_base + (size_t)cell * R::BYTES;
    if constexpr (BF16) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(p + 4 * (R::NSH >> 1));
        return (R::NSH & 1) ? bf16_hi(w) : bf16_lo(w);
    } else {
        return *reinterpret_cast<const float*>(p + 4 * R::NSH);
    }
}

// ---------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, l-major with m = -l..l, textbook
// normalisation (orthonormal on the sphere), as polynomials of the unit
// direction. The view-dependent colour of a cell is sum_b k_b Y_b(d) (Sec. 3.4).
// ---------------------------------------------------------------------------
template <int DEG>
__device__ inline void sh_basis(float x, float y, float z, float* Y)
{
    Y[0] = 0.28209479177387814f;
    if constexpr (DEG >= 1) {
        Y[1] = 0.4886025119029199f * y;
        Y[2] = 0.4886025119029199f * z;
        Y[3] = 0.4886025119029199f * x;
    }
    if constexpr (DEG >= 2) {
        Y[4] = 1.0925484305920792f * (x * y);
        Y[5] = 1.0925484305920792f * (y * z);
        Y[6] = 0.31539156525252005f * (3.0f * z * z - 1.0f);
        Y[7] = 1.0925484305920792f * (x * z);
        Y[8] = 0.5462742152960396f * (x * x - y * y);
    }
    if constexpr (DEG >= 3) {
        Y[9] = 0.5900435899266435f * y * (3.0f * x * x - y * y);
        Y[10] = 2.890611442640554f * (x * y * z);
        Y[11] = 0.4570457994644658f * y * (5.0f * z * z - 1.0f);
        Y[12] = 0.3731763325901154f * z * (5.0f * z * z - 3.0f);
        Y[13] = 0.4570457994644658f * x * (5.0f * z * z - 1.0f);
        Y[14] = 1.445305721320277f * z * (x * x - y * y);
        Y[15] = 0.5900435899266435f * x * (x * x - 3.0f * y * y);
    }
}

// Cell reference packed into the adjacency and row arrays.
__device__ inline int ref_cell(uint2 r) { return (int)(r.x & 0xffffffu); }
__device__ inline int ref_deg(uint2 r) { return (int)(r.x >> 24); }
__device__ inline int ref_beg(uint2 r) { return (int)r.y; }

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Remap so that each XCD works on chunks of CHUNK consecutive blocks (the
// walks use 32 one-tile blocks: neighbouring tiles walk the same cells, so a
// chunk's records are shared in one XCD's L2), with the chunks dealt to the
// XCDs in turn so that every XCD gets work from all over the frame. (One
// contiguous eighth of the frame per XCD leaves the XCDs with the lighter
// bands idle at the end: 15% slower walks on a 1080p frame.) Blocks past the
// last whole round of chunks keep their place.
template <int64_t CHUNK = 8>
__device__ inline int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t full = nb / (8 * CHUNK) * (8 * CHUNK);
    if (b >= full) return b;
    const int64_t x = b % 8, m = b / 8;
    return ((m / CHUNK) * 8 + x) * CHUNK + m % CHUNK;
}

}  // namespace rf
