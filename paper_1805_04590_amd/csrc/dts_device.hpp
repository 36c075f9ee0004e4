// Device helpers shared by the libdts kernels (gfx950, wave64).
//
// Every 1-D recursive pass of the domain-transform filter is a chain of affine maps
//   causal      J[n] = w[n] J[n-1] + (1 - w[n]) f[n]
//   anticausal  K[n] = w[n+1] K[n+1] + (1 - w[n+1]) J[n]
// so a line is scanned by composing maps x -> a x + b:
//   (a2, b2) o (a1, b1) = (a2 a1, a2 b1 + b2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dts {

constexpr int kWave = 64;

// Bounded waits: a poll loop gives up after this many polls (each followed by a short
// sleep), records a device-side failure and lets the wave finish, so no kernel can spin
// forever even if a co-residency assumption were violated.
constexpr int kSpinLimit = 1 << 21;

// Status word layout in the workspace header.
constexpr int kErrSpinTimeout = 1;
constexpr int kErrBadTicket = 2;

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// Weight w = a^d = 2^(d log2 a).
__device__ __forceinline__ float weight(float d, float log2a) { return exp2_fast(d * log2a); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Workgroups of a dispatch go to the 8 XCDs in turn (workgroup b to XCD b % 8), and each
// XCD has its own L2.  This bijection of [0, n) gives XCD x a contiguous band of indices,
// visited in order, so neighbouring rows meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_band_index(int b, int n) {
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, j = b / kXcds;
    return x * q + min(x, r) + j;
}

// Inclusive scan of affine maps from lane 0 upwards: lane l ends with the composition of
// the maps of lanes 0..l (lane l's map applied last).
__device__ __forceinline__ void scan_maps_up(float& a, float& b, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const float pa = __shfl_up(a, d);
        const float pb = __shfl_up(b, d);
        if (lane >= d) {
            b = fmaf(a, pb, b);
            a = a * pa;
        }
    }
}

// Inclusive scan of affine maps from lane 63 downwards: lane l ends with the composition
// of the maps of lanes 63..l (lane l's map applied last).
__device__ __forceinline__ void scan_maps_down(float& a, float& b, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const float na = __shfl_down(a, d);
        const float nb = __shfl_down(b, d);
        if (lane + d < kWave) {
            b = fmaf(a, nb, b);
            a = a * na;
        }
    }
}

// DPP move of a float within rows of 16 lanes; lanes whose source lane is outside their
// row (or outside ROWMASK) receive `old`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp_f(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL,
                                                      ROWMASK, 0xf, false));
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Compose the map (pa, pb) in front of (a, b): x -> a (pa x + pb) + b.
__device__ __forceinline__ void compose_after(float& a, float& b, float pa, float pb) {
    b = fmaf(a, pb, b);
    a = a * pa;
}

// Inclusive scan of affine maps, lane 0 upwards (lane l: maps of lanes 0..l, lane l's
// applied last): DPP shifts inside each row of 16 lanes, then the row totals (lanes 15,
// 31, 47) are read as scalars and composed in front of the later rows.
__device__ __forceinline__ void scan_up_dpp(float& a, float& b, int lane) {
    compose_after(a, b, dpp_f<0x111>(1.f, a), dpp_f<0x111>(0.f, b));
    compose_after(a, b, dpp_f<0x112>(1.f, a), dpp_f<0x112>(0.f, b));
    compose_after(a, b, dpp_f<0x114>(1.f, a), dpp_f<0x114>(0.f, b));
    compose_after(a, b, dpp_f<0x118>(1.f, a), dpp_f<0x118>(0.f, b));
    const float a0 = readlane_f(a, 15), b0 = readlane_f(b, 15);
    const float a1 = readlane_f(a, 31), b1 = readlane_f(b, 31);
    const float a2 = readlane_f(a, 47), b2 = readlane_f(b, 47);
    // prefixes of rows: row 1 gets row 0; row 2 gets rows 0..1; row 3 gets rows 0..2
    float p1a = a0, p1b = b0;
    float p2a = a1, p2b = b1;
    compose_after(p2a, p2b, p1a, p1b);
    float p3a = a2, p3b = b2;
    compose_after(p3a, p3b, p2a, p2b);
    const int row = lane >> 4;
    const float pa = row == 0 ? 1.f : row == 1 ? p1a : row == 2 ? p2a : p3a;
    const float pb = row == 0 ? 0.f : row == 1 ? p1b : row == 2 ? p2b : p3b;
    compose_after(a, b, pa, pb);
}

// Inclusive scan of affine maps, lane 63 downwards (lane l: maps of lanes 63..l, lane l's
// applied last).
__device__ __forceinline__ void scan_down_dpp(float& a, float& b, int lane) {
    compose_after(a, b, dpp_f<0x101>(1.f, a), dpp_f<0x101>(0.f, b));
    compose_after(a, b, dpp_f<0x102>(1.f, a), dpp_f<0x102>(0.f, b));
    compose_after(a, b, dpp_f<0x104>(1.f, a), dpp_f<0x104>(0.f, b));
    compose_after(a, b, dpp_f<0x108>(1.f, a), dpp_f<0x108>(0.f, b));
    const float a1 = readlane_f(a, 16), b1 = readlane_f(b, 16);
    const float a2 = readlane_f(a, 32), b2 = readlane_f(b, 32);
    const float a3 = readlane_f(a, 48), b3 = readlane_f(b, 48);
    // suffixes of rows: row 2 gets row 3; row 1 gets rows 3..2; row 0 gets rows 3..1
    float s2a = a3, s2b = b3;
    float s1a = a2, s1b = b2;
    compose_after(s1a, s1b, s2a, s2b);
    float s0a = a1, s0b = b1;
    compose_after(s0a, s0b, s1a, s1b);
    const int row = lane >> 4;
    const float sa = row == 3 ? 1.f : row == 2 ? s2a : row == 1 ? s1a : s0a;
    const float sb = row == 3 ? 0.f : row == 2 ? s2b : row == 1 ? s1b : s0b;
    compose_after(a, b, sa, sb);
}

// Carry words: a float value tagged with the epoch of the launch that wrote it, stored
// and loaded as one 64-bit device-scope atomic so a reader never sees a value without its
// tag.  Words from older launches carry older epochs and read as "not yet written".
// They are addressed as global memory explicitly: a kernel that takes the carry area's
// address from a table in memory would otherwise access them as generic (flat) memory,
// and every later LDS wait of the workgroup would also wait for those accesses.
typedef __attribute__((address_space(1))) unsigned long long gword;

__device__ __forceinline__ gword* global_word(unsigned long long* p) { return (gword*)p; }

__device__ __forceinline__ void publish(gword* p, unsigned epoch, float v) {
    const unsigned long long word =
        (static_cast<unsigned long long>(epoch) << 32) | __float_as_uint(v);
    __hip_atomic_store(p, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool peek(gword* p, unsigned epoch, float& v) {
    const unsigned long long word = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = __uint_as_float(static_cast<unsigned>(word));
    return static_cast<unsigned>(word >> 32) == epoch;
}

__device__ __forceinline__ void flag_error(int* status, int code) {
    __hip_atomic_fetch_or(status, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Four floats at a 4-byte aligned address, moved as one 16-byte access: dword alignment is
// all that multi-dword global and buffer accesses need, so rows whose length is not a
// multiple of 4 (and whose starts are therefore not 16-byte aligned) still move 16 bytes
// per lane and instruction instead of 4.
typedef float float4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// S (a multiple of 4) consecutive row elements starting at n0 (a multiple of S); elements
// at or beyond W read as `fill`, and store_seg writes only those below W.
template <int S>
__device__ __forceinline__ void load_seg(const float* row, int n0, int W, float fill, float (&v)[S]) {
    static_assert(S % 4 == 0, "segments are whole groups of 4");
    if (n0 + S <= W) {
#pragma unroll
        for (int e = 0; e < S; e += 4) {
            const float4_a4 q = *reinterpret_cast<const float4_a4*>(row + n0 + e);
            v[e] = q[0];
            v[e + 1] = q[1];
            v[e + 2] = q[2];
            v[e + 3] = q[3];
        }
    } else {
#pragma unroll
        for (int e = 0; e < S; ++e) v[e] = (n0 + e < W) ? row[n0 + e] : fill;
    }
}

template <int S>
__device__ __forceinline__ void store_seg(float* row, int n0, int W, const float (&v)[S]) {
    static_assert(S % 4 == 0, "segments are whole groups of 4");
    if (n0 + S <= W) {
        // element stores that the backend merges into 16-byte stores (a vector store here
        // is scheduled with more registers live)
#pragma unroll
        for (int e = 0; e < S; ++e) row[n0 + e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < S; ++e)
            if (n0 + e < W) row[n0 + e] = v[e];
    }
}

// Raw buffer access.  A resource covers one plane; lanes whose voffset is kInvalidOffset
// fall outside every plane (planes are < 2 GiB), so their loads return 0 and their stores
// are dropped by the hardware range check.
constexpr unsigned kInvalidOffset = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                             static_cast<int>(bytes), 0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                       float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// S consecutive floats of a row through a buffer resource over the whole plane: lane
// elements [n0, n0 + S) of the row at byte offset `row` (elements at or past `n` read 0
// and are not written), in 128-bit accesses at 4-byte aligned offsets.  Buffer accesses
// count on the vector memory counter only, so waiting for them never waits on LDS or
// scalar traffic (and the reverse), unlike generic (flat) accesses through pointers
// loaded from memory.
template <int S>
__device__ __forceinline__ void bload_seg(__amdgpu_buffer_rsrc_t r, unsigned row, int n0, int n, float (&v)[S]) {
    static_assert(S % 4 == 0, "segments are whole groups of 4");
    // 16-byte loads at 4-byte aligned offsets; a group that runs past n reads the first
    // elements of the next row, or past the end of the plane zeros (the range check applies
    // to each dword of the access), and those elements are replaced by 0
#pragma unroll
    for (int e = 0; e < S; e += 4) {
        const unsigned o = (n0 + e < n) ? row + static_cast<unsigned>(n0 + e) * 4u : kInvalidOffset;
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) v[e + k] = (n0 + e + k < n) ? __uint_as_float(q[k]) : 0.f;
    }
}

template <int S>
__device__ __forceinline__ void bstore_seg(__amdgpu_buffer_rsrc_t r, unsigned row, int n0, int n,
                                           const float (&v)[S]) {
    static_assert(S % 4 == 0, "segments are whole groups of 4");
    // whole groups as 16-byte stores at 4-byte aligned offsets, a group that reaches past n
    // element by element
#pragma unroll
    for (int e = 0; e < S; e += 4) {
        if (n0 + e + 4 <= n) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 q = {__float_as_uint(v[e]), __float_as_uint(v[e + 1]), __float_as_uint(v[e + 2]),
                             __float_as_uint(v[e + 3])};
            __builtin_amdgcn_raw_buffer_store_b128(q, r, row + static_cast<unsigned>(n0 + e) * 4u, 0, 0);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                bstore(r, (n0 + e + k < n) ? row + static_cast<unsigned>(n0 + e + k) * 4u : kInvalidOffset, 0,
                       v[e + k]);
        }
    }
}

// Scalar add the compiler cannot fold away, so a row offset advances as one running SGPR
// instead of one precomputed SGPR per unrolled row.
__device__ __forceinline__ unsigned opaque_add(unsigned x, unsigned y) {
    unsigned r = x + y;
    asm volatile("" : "+s"(r));
    return r;
}

// Vector add the compiler cannot fold or common up: unrolled row loops advance one running
// offset register instead of keeping one precomputed address register per row alive.
__device__ __forceinline__ unsigned opaque_vadd(unsigned x, unsigned y) {
    unsigned r = x + y;
    asm volatile("" : "+v"(r));
    return r;
}

// Integers the compiler cannot see through (VGPR / SGPR); used inside persistent loops so
// per-row constants are rebuilt each iteration instead of being hoisted and kept live.
__device__ __forceinline__ int opaque_v(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ int opaque_s(int x) {
    asm volatile("" : "+s"(x));
    return x;
}

// A float the compiler cannot see through: starting a product chain from it stops the
// compiler from keeping every partial product of an identical earlier chain alive.
__device__ __forceinline__ float opaque(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ float get(const float4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

}  // namespace dts

namespace dts {

// Affine-map scans with one shared factor and NB offsets: lane l ends with the maps of
// lanes 0..l (up) or 63..l (down), its own applied last.  Used where several recurrences
// share their weights (a signal and its adjoint, or several channels).
template <int NB>
__device__ __forceinline__ void compose_after_n(float& a, float (&b)[NB], float pa, const float (&pb)[NB]) {
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = fmaf(a, pb[i], b[i]);
    a = a * pa;
}

template <int CTRL, int NB>
__device__ __forceinline__ void dpp_step_n(float& a, float (&b)[NB]) {
    float pb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) pb[i] = dpp_f<CTRL>(0.f, b[i]);
    compose_after_n<NB>(a, b, dpp_f<CTRL>(1.f, a), pb);
}

template <int NB>
__device__ __forceinline__ void scan_up_dpp_n(float& a, float (&b)[NB], int lane) {
    dpp_step_n<0x111, NB>(a, b);
    dpp_step_n<0x112, NB>(a, b);
    dpp_step_n<0x114, NB>(a, b);
    dpp_step_n<0x118, NB>(a, b);
    float ra[3], rb[3][NB];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        ra[r] = readlane_f(a, 16 * r + 15);
#pragma unroll
        for (int i = 0; i < NB; ++i) rb[r][i] = readlane_f(b[i], 16 * r + 15);
    }
    // prefix of rows before row r: row 1 <- row 0, row 2 <- rows 0..1, row 3 <- rows 0..2
    float pa[4], pb[4][NB];
    pa[0] = 1.f;
#pragma unroll
    for (int i = 0; i < NB; ++i) pb[0][i] = 0.f;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        pa[r] = ra[r - 1];
#pragma unroll
        for (int i = 0; i < NB; ++i) pb[r][i] = rb[r - 1][i];
        compose_after_n<NB>(pa[r], pb[r], pa[r - 1], pb[r - 1]);
    }
    const int row = lane >> 4;
    float qa = pa[0], qb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) qb[i] = pb[0][i];
#pragma unroll
    for (int r = 1; r < 4; ++r)
        if (row == r) {
            qa = pa[r];
#pragma unroll
            for (int i = 0; i < NB; ++i) qb[i] = pb[r][i];
        }
    compose_after_n<NB>(a, b, qa, qb);
}

template <int NB>
__device__ __forceinline__ void scan_down_dpp_n(float& a, float (&b)[NB], int lane) {
    dpp_step_n<0x101, NB>(a, b);
    dpp_step_n<0x102, NB>(a, b);
    dpp_step_n<0x104, NB>(a, b);
    dpp_step_n<0x108, NB>(a, b);
    float ra[4], rb[4][NB];
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        ra[r] = readlane_f(a, 16 * r);
#pragma unroll
        for (int i = 0; i < NB; ++i) rb[r][i] = readlane_f(b[i], 16 * r);
    }
    // suffix of rows after row r: row 2 <- row 3, row 1 <- rows 3..2, row 0 <- rows 3..1
    float sa[4], sb[4][NB];
    sa[3] = 1.f;
#pragma unroll
    for (int i = 0; i < NB; ++i) sb[3][i] = 0.f;
#pragma unroll
    for (int r = 2; r >= 0; --r) {
        sa[r] = ra[r + 1];
#pragma unroll
        for (int i = 0; i < NB; ++i) sb[r][i] = rb[r + 1][i];
        compose_after_n<NB>(sa[r], sb[r], sa[r + 1], sb[r + 1]);
    }
    const int row = lane >> 4;
    float qa = sa[3], qb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) qb[i] = sb[3][i];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        if (row == r) {
            qa = sa[r];
#pragma unroll
            for (int i = 0; i < NB; ++i) qb[i] = sb[r][i];
        }
    compose_after_n<NB>(a, b, qa, qb);
}

}  // namespace dts
