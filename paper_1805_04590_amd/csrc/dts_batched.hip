// Many independent solves of uneven size in one persistent launch (not in the paper;
// every instance is the Eq. (3) gradient descent with the recursive domain-transform
// filter of Sec. 3.2, exactly as dts_solve runs it).
//
// Phase 0 computes the transformed distances of every instance (Eq. (8)-(9)); phase
// p > 0 is the (p-1)-th pass of every instance (the row and column passes of each filter
// iteration, solver iteration after solver iteration).  All workgroups of a grid that
// fits on the device at once work through the phases in lockstep: inside a phase they
// take tiles from the phase's atomic ticket counter (instance 0's tiles first, then
// instance 1's, ...), and between phases they meet at a grid barrier whose release and
// acquire make the phase's stores visible to every XCD.  A row tile is a band of rows of
// one instance: rows up to kBatchSoloWidth pixels are filtered by one wave each with no
// barrier, wider rows by groups of row_gw waves.  A column tile is one chunk of one
// 64-column strip (chunks of a strip are consecutive tickets) and exchanges carries with
// the strip's other chunks through epoch-tagged words.
//
// Progress: a workgroup takes its next ticket only when its current tile can no longer
// wait (at the start of a row or distance tile, after the carries of a column tile are
// resolved), so every chunk that a waiting chunk needs is either running or held by a
// workgroup that will start it; a strip has at most as many chunks as the grid has
// workgroups.  Every wait is bounded and flags the workspace status when it gives up.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dts.h"
#include "dts_batched.hpp"
#include "dts_chunks.hpp"
#include "dts_device.hpp"
#include "dts_internal.hpp"
#include "dts_tiles.hpp"

namespace dts {

constexpr int kBarrierSpinLimit = 1 << 25;

__device__ __forceinline__ int upper_index(const int* v, int n, int x) {
    // largest j in [0, n) with v[j] <= x (v sorted ascending, v[0] <= x)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (v[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Barrier counters: counts[0] counts the workgroup groups that finished a phase, and
// counts[kBarrierStride * (1 + g)] the workgroups of group g = blockIdx % 8 (the XCD a
// workgroup is dispatched to); all are cumulative over the phases of a launch.
constexpr int kBarrierGroups = 8;
constexpr int kBarrierStride = 16;  // 64 bytes between counters

// All workgroups of the grid: every store issued before the call is visible to every
// workgroup after it.  `phase` counts the barriers of this launch from 1.  Each workgroup
// bumps its group's counter and the last of a group bumps the global one, so no counter
// takes more than grid / 8 + 1 same-address atomics per phase (a single counter bumped by
// every workgroup serialises them: measured 45 us against 13 us per barrier at 768
// workgroups).
__device__ __forceinline__ void grid_barrier(unsigned* counts, unsigned phase, int* status) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned n = gridDim.x;
        const unsigned g = blockIdx.x % kBarrierGroups;
        const unsigned members = n / kBarrierGroups + (g < n % kBarrierGroups ? 1u : 0u);
        const unsigned groups = n < kBarrierGroups ? n : kBarrierGroups;
        const unsigned old = __hip_atomic_fetch_add(counts + kBarrierStride * (1 + g), 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == phase * members)
            __hip_atomic_fetch_add(counts, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = phase * groups;
        int spins = 0, backoff = 1;
        while (__hip_atomic_load(counts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            spins += backoff;
            if (spins > kBarrierSpinLimit) {
                flag_error(status, kErrSpinTimeout);
                break;
            }
            for (int q = 0; q < backoff; ++q) __builtin_amdgcn_s_sleep(1);
            backoff = backoff < 16 ? backoff * 2 : 16;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

struct RowLds {
    float2 fagg[kBatchWaves];
    float2 bagg[kBatchWaves];
    float wfirst[2 * kBatchWaves];
};

// Rows y0 + v, y0 + v + kBatchWaves, ... of [y0, y1), each filtered by wave v alone.
template <int S>
__device__ __forceinline__ void row_band_solo(const RowArgs& a, int y0, int y1, int wave) {
    for (int y = y0 + wave; y < y1; y += kBatchWaves)
        row_line<S, false, true, false, true>(a, y, 0, 0, 1, true, nullptr, nullptr, nullptr);
}

// Rows [y0, y1) of one instance.  gw == 1: one wave per row (row_band_solo); otherwise
// kBatchWaves / gw groups of gw waves filter rows side by side.
template <int S>
__device__ __forceinline__ void row_band(const RowArgs& ra, int y0, int y1, int gw, RowLds& RL) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (gw == 1) {
        row_band_solo<S>(ra, y0, y1, wave);
        return;
    }
    const int rg = wave / gw;
    const int gwv = wave - rg * gw;
    const int groups = kBatchWaves / gw;
    for (int y = y0; y < y1; y += groups) {
        const int yy = y + rg;
        const bool live = yy < y1;
        row_line<S, false, false, false, true>(ra, live ? yy : 0, 0, gwv, gw, live, RL.fagg + rg * gw,
                                  RL.bagg + rg * gw, RL.wfirst + rg * (gw + 1));
    }
}

// Rows of kBatchSoloWidth < W <= 2 kBatchSoloWidth pixels, each filtered by one wave alone
// in two sections of kBatchSoloWidth pixels (lane l owns pixels 16 l + [0, 16) of each):
// the causal recurrence runs through section 0 and on through section 1 from J at the
// section boundary, the anticausal one back through section 1 and on through section 0
// from K there.  Section 0's weights and causal output wait in the wave's LDS stash while
// section 1 is in registers, so the wave never holds more than one section and, as for
// rows of at most kBatchSoloWidth pixels, the waves of a workgroup filter their rows
// independently, with no workgroup barrier.
constexpr int kWideS = kBatchSoloWidth / kWave;  // pixels per lane and section
constexpr int kWideQ = kWideS / 4;               // float4 per lane and section
typedef float wide4 __attribute__((ext_vector_type(4)));
struct WideStash {
    wide4 w[kWideQ][kWave];  // section 0 weights
    wide4 j[kWideQ][kWave];  // section 0 causal output of the current channel
};

__device__ __forceinline__ void stash_put(wide4 (&s)[kWideQ][kWave], const float (&v)[kWideS], int lane) {
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) s[q][lane] = wide4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
}

__device__ __forceinline__ void stash_get(const wide4 (&s)[kWideQ][kWave], float (&v)[kWideS], int lane) {
#pragma unroll
    for (int q = 0; q < kWideQ; ++q) {
        const wide4 x = s[q][lane];
        v[4 * q] = x[0];
        v[4 * q + 1] = x[1];
        v[4 * q + 2] = x[2];
        v[4 * q + 3] = x[3];
    }
}

// causal sweep of one section: f (the signal) becomes J, starting from J = jin before the
// section's first pixel
__device__ __forceinline__ void wide_causal(const float (&w)[kWideS], float (&f)[kWideS], float jin, int lane) {
    float la = 1.f, lb = 0.f;
#pragma unroll
    for (int e = 0; e < kWideS; ++e) {
        lb = fmaf(w[e], lb - f[e], f[e]);
        la *= w[e];
    }
    scan_up_dpp(la, lb, lane);
    const float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
    float j = (lane == 0) ? jin : fmaf(xa, jin, xb);
#pragma unroll
    for (int e = 0; e < kWideS; ++e) {
        j = fmaf(w[e], j - f[e], f[e]);
        f[e] = j;
    }
}

// anticausal sweep of one section: f (J) becomes K, starting from K = kin after the
// section's last pixel, which links to it with weight wl on lane 63 (each lane's wl is
// the weight of the pixel after its last)
__device__ __forceinline__ void wide_anticausal(const float (&w)[kWideS], float wl, float (&f)[kWideS], float kin,
                                                int lane) {
    float la = 1.f, lb = 0.f;
#pragma unroll
    for (int e = kWideS - 1; e >= 0; --e) {
        const float wn = (e == kWideS - 1) ? wl : w[e < kWideS - 1 ? e + 1 : e];
        lb = fmaf(wn, lb - f[e], f[e]);
        la *= wn;
    }
    scan_down_dpp(la, lb, lane);
    const float xa = __shfl_down(la, 1), xb = __shfl_down(lb, 1);
    float k = (lane == kWave - 1) ? kin : fmaf(xa, kin, xb);
#pragma unroll
    for (int e = kWideS - 1; e >= 0; --e) {
        const float wn = (e == kWideS - 1) ? wl : w[e < kWideS - 1 ? e + 1 : e];
        k = fmaf(wn, k - f[e], f[e]);
        f[e] = k;
    }
}

__device__ __forceinline__ void row_line_wide(const RowArgs& a, int y, WideStash& st) {
    constexpr int S = kWideS;
    const int lane = lane_id();
    const int W = a.W;
    const size_t plane = static_cast<size_t>(a.H) * W;
    const unsigned rowoff = static_cast<unsigned>(y) * static_cast<unsigned>(W) * 4u;
    const int n0 = lane * S, n1 = kBatchSoloWidth + lane * S;
    const auto rs = [&](const float* base, int c) {
        return plane_rsrc(base + static_cast<size_t>(c) * plane, plane * sizeof(float));
    };
    float w[S], w1[S], f0[S], f1[S];
    bload_seg<S>(rs(a.d, 0), rowoff, n0, W, w);
    if (a.C > 0) bload_seg<S>(rs(a.src, 0), rowoff, n0, W, f0);
    bload_seg<S>(rs(a.d, 0), rowoff, n1, W, w1);
    if (a.C > 0) bload_seg<S>(rs(a.src, 0), rowoff, n1, W, f1);
#pragma unroll
    for (int e = 0; e < S; ++e) {
        w[e] = (n0 + e > 0) ? weight(w[e], a.log2a) : 0.f;  // section 0 lies inside the row
        w1[e] = (n1 + e < W) ? weight(w1[e], a.log2a) : 0.f;
    }
    // weight of the pixel after each lane's last: section 0's lane 63 links to section 1's
    // first pixel, section 1's lane 63 to nothing
    const float wsec = readlane_f(w1[0], 0);
    float wl0 = __shfl_down(w[0], 1), wl1 = __shfl_down(w1[0], 1);
    if (lane == kWave - 1) {
        wl0 = wsec;
        wl1 = 0.f;
    }
    stash_put(st.w, w, lane);
    for (int c = 0; c < a.C; ++c) {
        // section 0's weights come back from LDS for every channel, so they hold no
        // registers while section 1 is filtered
        __asm__ volatile("" ::: "memory");
        stash_get(st.w, w, lane);
        wide_causal(w, f0, 0.f, lane);
        const float jsec = readlane_f(f0[S - 1], kWave - 1);  // J at the last pixel of section 0
        stash_put(st.j, f0, lane);
        if (c + 1 < a.C) bload_seg<S>(rs(a.src, c + 1), rowoff, n0, W, f0);
        wide_causal(w1, f1, jsec, lane);
        wide_anticausal(w1, wl1, f1, 0.f, lane);
        const float ksec = readlane_f(f1[0], 0);  // K at the first pixel of section 1
        bstore_seg<S>(rs(a.dst, c), rowoff, n1, W, f1);
        __asm__ volatile("" ::: "memory");
        stash_get(st.j, f1, lane);
        stash_get(st.w, w, lane);
        wide_anticausal(w, wl0, f1, ksec, lane);
        bstore_seg<S>(rs(a.dst, c), rowoff, n0, W, f1);
        if (c + 1 < a.C) bload_seg<S>(rs(a.src, c + 1), rowoff, n1, W, f1);
    }
}

// Rows y0 + v, y0 + v + kBatchWaves, ... of [y0, y1), each filtered by wave v alone in two
// sections (row_line_wide).
__device__ __forceinline__ void row_band_wide(const RowArgs& ra, int y0, int y1, WideStash (&st)[kBatchWaves]) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int y = y0 + wave; y < y1; y += kBatchWaves) row_line_wide(ra, y, st[wave]);
}

template <int CTM>
union BatchLds {
    ChunkLds<CTM, kBatchWaves> chunk;  // column tiles
    WideStash wide[kBatchWaves];       // rows of two sections, one stash per wave
};

// Transformed distances (Eq. (8)-(9)) of rows [y0, y1): one pixel per thread, guide bands
// four at a time (their loads in flight together, the sums in band order); at x = 0
// (y = 0) the missing neighbour is the pixel itself, so the distance is 1.  Consecutive
// rows of a band share the workgroup's L2, where the row above is re-read.
__device__ __forceinline__ void dist_band(const BInst& I, int y0, int y1) {
    const int W = I.W, Cg = I.Cg;
    const size_t plane = static_cast<size_t>(I.H) * W;
    // global, not generic, accesses: the planes' addresses come from the descriptor table
    typedef __attribute__((address_space(1))) const float gcfloat;
    typedef __attribute__((address_space(1))) float gfloat;
    gcfloat* __restrict__ guide = (gcfloat*)I.guide;
    gfloat* __restrict__ dx = (gfloat*)I.dx;
    gfloat* __restrict__ dy = (gfloat*)I.dy;
    const float s2 = I.s2;
    constexpr int kU = 4;
    for (int y = y0; y < y1; ++y) {
        for (int x = threadIdx.x; x < W; x += kWave * kBatchWaves) {
            const size_t o = static_cast<size_t>(y) * W + x;
            const ptrdiff_t dl = (x > 0) ? 1 : 0;
            const ptrdiff_t du = (y > 0) ? W : 0;
            float ax = 0.f, ay = 0.f;
            gcfloat* g = guide + o;
            int k = 0;
            for (; k + kU <= Cg; k += kU) {
                float v[kU], l[kU], u[kU];
#pragma unroll
                for (int q = 0; q < kU; ++q) {
                    gcfloat* gq = g + q * plane;
                    v[q] = gq[0];
                    l[q] = gq[-dl];
                    u[q] = gq[-du];
                }
#pragma unroll
                for (int q = 0; q < kU; ++q) {
                    const float ex = v[q] - l[q];
                    const float ey = v[q] - u[q];
                    ax = fmaf(ex, ex, ax);
                    ay = fmaf(ey, ey, ay);
                }
                g += kU * plane;
            }
            for (; k < Cg; ++k) {
                const float v = g[0];
                const float ex = v - g[-dl];
                const float ey = v - g[-du];
                ax = fmaf(ex, ex, ax);
                ay = fmaf(ey, ey, ay);
                g += plane;
            }
            dx[o] = sqrtf(fmaf(s2, ax, 1.f));
            dy[o] = sqrtf(fmaf(s2, ay, 1.f));
        }
    }
}

// OCC: waves per SIMD the register allocation must allow (OCC workgroups per CU).
template <int R, int CTM, int OCC>
__global__ void __launch_bounds__(kWave * kBatchWaves) __attribute__((amdgpu_waves_per_eu(OCC, 8)))
batched_kernel(BatchArgs a) {
    __shared__ BatchLds<CTM> U;
    __shared__ RowLds RL;
    __shared__ int s_pre[kBatchMaxProblems + 1];
    __shared__ unsigned s_t;
    const unsigned launch = __hip_atomic_load(const_cast<unsigned*>(a.launch), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    const int n = a.n;
    for (int p = 0; p < a.n_phases; ++p) {
        unsigned* tickets = a.tickets + p;
        const int* pre = a.phase_prefix + static_cast<size_t>(p) * (n + 1);
        for (int j = threadIdx.x; j <= n; j += blockDim.x) s_pre[j] = pre[j];
        if (threadIdx.x == 0) s_t = atomicAdd(tickets, 1u);
        __syncthreads();
        const int total = s_pre[n];
        int t = static_cast<int>(__builtin_amdgcn_readfirstlane(s_t));
        unsigned nxt = 0u;  // thread 0: the next ticket, taken while the tile runs
        while (t < total) {
            const int i = __builtin_amdgcn_readfirstlane(upper_index(s_pre, n + 1, t));
            const int tile = t - s_pre[i];
            const BInst& I = a.inst[i];
            if (p == 0) {
                if (threadIdx.x == 0) nxt = atomicAdd(tickets, 1u);
                const int y0 = tile * I.dist_rows;
                dist_band(I, y0, min(I.H, y0 + I.dist_rows));
                __syncthreads();  // every wave has read s_t
            } else {
                const int pass = p - 1;
                const int per_iter = 2 * I.N;
                const int k = pass / per_iter;
                const int q = pass % per_iter;
                const int fi = q / 2 + 1;  // filter iteration 1..N
                const float* zk = (k == 0) ? I.target : I.out;
                if ((q & 1) == 0) {
                    if (threadIdx.x == 0) nxt = atomicAdd(tickets, 1u);
                    RowArgs ra;
                    ra.src = (fi == 1) ? zk : I.tmp;
                    ra.dst = I.tmp;
                    ra.d = I.dx;
                    ra.guide = nullptr;
                    ra.dx_out = nullptr;
                    ra.dy_out = nullptr;
                    ra.Cg = I.Cg;
                    ra.s2 = I.s2;
                    ra.C = I.Ct;
                    ra.H = I.H;
                    ra.W = I.W;
                    ra.log2a = I.log2a[fi - 1];
                    const int y0 = tile * I.row_rows;
                    const int y1 = min(I.H, y0 + I.row_rows);
                    if (I.row_S == 8) row_band<8>(ra, y0, y1, I.row_gw, RL);
                    else if (I.row_S == 16) row_band<16>(ra, y0, y1, I.row_gw, RL);
                    else row_band_wide(ra, y0, y1, U.wide);
                    __syncthreads();  // every wave has read s_t
                } else {
                    ColArgs ca;
                    const bool epi = (fi == I.N);
                    ca.src = I.tmp;
                    ca.dst = epi ? I.out : I.tmp;
                    ca.d = I.dy;
                    ca.C = I.Ct;
                    ca.H = I.H;
                    ca.W = I.W;
                    ca.log2a = I.log2a[fi - 1];
                    ca.G = I.G;
                    ca.S = I.S;
                    ca.NG = I.NG;
                    ca.batch = 1;
                    ca.groups = 1;
                    ca.carry = I.carry;
                    ca.epoch = launch * static_cast<unsigned>(a.n_phases + 1) + static_cast<unsigned>(p) + 1u;
                    ca.status = a.status;
                    ca.zk = zk;
                    ca.tgt = I.target;
                    ca.conf = I.conf;
                    ca.Cc = I.Cc;
                    ca.dst2 = nullptr;
                    ca.lambda = a.lambda;
                    ca.step = a.step;
                    const CarryCtx cctx{ca.carry, ca.epoch, ca.status, ca.G, ca.S, ca.NG, a.spin_limit, a.tag_xor};
                    const int chunk = tile % I.G;
                    const int rest = tile / I.G;
                    const int strip = rest % I.S;
                    const int grp = rest / I.S;
                    auto take_next = [&]() {
                        if (threadIdx.x == 0) nxt = atomicAdd(tickets, 1u);
                    };
                    if (epi) col_tile<CTM, R, kBatchWaves, 1>(ca, cctx, U.chunk, chunk, strip, grp, 0, take_next);
                    else col_tile<CTM, R, kBatchWaves, 0>(ca, cctx, U.chunk, chunk, strip, grp, 0, take_next);
                }
            }
            // every wave has read s_t (a barrier of the tile lies in between)
            if (threadIdx.x == 0) s_t = nxt;
            __syncthreads();
            t = static_cast<int>(__builtin_amdgcn_readfirstlane(s_t));
        }
        if (p + 1 < a.n_phases)
            grid_barrier(a.barrier, static_cast<unsigned>(p + 1), a.status);
    }
}

__global__ void batched_reset_kernel(unsigned* tickets, int n_phases, unsigned* barrier, unsigned* launch,
                                     int* status) {
    for (int i = threadIdx.x; i < n_phases; i += blockDim.x) tickets[i] = 0u;
    if (threadIdx.x <= kBarrierGroups) barrier[kBarrierStride * threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        *launch = *launch + 1u;
        *status = 0;
    }
}

// ---------------------------------------------------------------------------------------
// Variants (chosen by the autotuner): rows per wave R of the column chunks, channels per
// column group CTM, and the target size of a row tile in pixels x channels
// ---------------------------------------------------------------------------------------
struct BatchVariant {
    int R, ctm, row_px;
    void (*launch)(const BatchArgs&, unsigned, hipStream_t);
    int (*capacity)();
};

template <int R, int CTM, int OCC>
static void batched_launch_v(const BatchArgs& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((batched_kernel<R, CTM, OCC>), dim3(grid), dim3(kWave * kBatchWaves), 0, s, a);
}

template <int R, int CTM, int OCC>
static int batched_capacity_v() {
    static int cached[64] = {0};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel<R, CTM, OCC>,
                                                         kWave * kBatchWaves, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

// Row tiles of 8192 pixels x channels: on the 64 uneven solves the row phase took 511 us
// against 528 at 16384 (finer tiles even out the phase's tail), 521 at 4096, 543 at 2048.
// Two workgroups per CU with 128-row two-channel chunks (32, 2, 2) replaced (16, 1, 4),
// which spills 52 registers since rows of 1025-2048 pixels are filtered by one wave.
#define DTS_BV(R, CT, OCC, PX) {R, CT, PX, batched_launch_v<R, CT, OCC>, batched_capacity_v<R, CT, OCC>}
static const BatchVariant kBatchVariants[] = {
    DTS_BV(32, 1, 3, 8192), DTS_BV(32, 2, 2, 8192), DTS_BV(16, 2, 3, 8192), DTS_BV(8, 3, 3, 8192),
    DTS_BV(16, 3, 2, 8192),
};
#undef DTS_BV
constexpr int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);

int num_batch_variants() { return kNumBatchVariants; }

int batch_variant_info(int v, int* rows_per_wave, int* group_channels, int* row_tile_pixels) {
    if (v < 0 || v >= kNumBatchVariants) return DTS_EINVAL;
    *rows_per_wave = kBatchVariants[v].R;
    *group_channels = kBatchVariants[v].ctm;
    *row_tile_pixels = kBatchVariants[v].row_px;
    return DTS_OK;
}

// ---------------------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------------------
namespace {
constexpr size_t kBAlign = 256;
size_t bal(size_t v) { return (v + kBAlign - 1) / kBAlign * kBAlign; }

struct Geo {
    int row_S, row_gw, row_rows, dist_rows, dist_tiles, G, S, NG, rows_tiles, col_tiles, phases;
    size_t dx, dy, tmp, carry, carry_bytes;
};
}  // namespace

static int check_problem(const dts_problem& q) {
    if (!q.guide || !q.target || !q.conf || !q.out) return DTS_EINVAL;
    if (q.H < 1 || q.W < 1 || q.Cg < 1 || q.Cg > DTS_MAX_CHANNELS || q.Ct < 1 || q.Ct > DTS_MAX_CHANNELS)
        return DTS_EINVAL;
    if (q.Cc != 1 && q.Cc != q.Ct) return DTS_EINVAL;
    if (!(std::isfinite(q.sigma_s) && q.sigma_s > 0) || !(std::isfinite(q.sigma_r) && q.sigma_r > 0))
        return DTS_EINVAL;
    if (q.filter_iters < 1 || q.solver_iters < 1) return DTS_EINVAL;
    if (q.filter_iters > kBatchMaxN || q.W > kBatchMaxWidth || q.H > DTS_MAX_HEIGHT) return DTS_ENOTSUP;
    if (static_cast<long long>(q.filter_iters) * q.solver_iters > (1 << 20)) return DTS_ENOTSUP;
    if ((static_cast<size_t>(q.H) + 64) * static_cast<size_t>(q.W) * 4 >= (static_cast<size_t>(1) << 31))
        return DTS_ENOTSUP;
    return DTS_OK;
}

static Geo geometry(const dts_problem& q, const BatchVariant& v) {
    Geo g{};
    if (q.W <= kBatchSoloWidth) {
        g.row_S = q.W <= 512 ? 8 : 16;
        g.row_gw = 1;
    } else if (q.W <= 2 * kBatchSoloWidth) {
        // one wave per row in two sections (row_line_wide)
        g.row_S = kBatchWideS;
        g.row_gw = 1;
    } else {
        // wider rows: the whole workgroup on one row at a time, 16 pixels per lane
        g.row_S = 16;
        g.row_gw = kBatchWaves;
    }
    const int side = kBatchWaves / g.row_gw;  // rows processed side by side
    const long long per_round = static_cast<long long>(q.W) * q.Ct * side;
    long long rounds = (v.row_px + per_round - 1) / per_round;
    rounds = std::max(1LL, std::min(rounds, static_cast<long long>(std::max(1, 64 / side))));
    g.row_rows = static_cast<int>(rounds) * side;
    const long long dist_row = static_cast<long long>(q.W) * q.Cg;
    g.dist_rows = static_cast<int>(std::max(1LL, std::min(256LL, (4LL * v.row_px + dist_row - 1) / dist_row)));
    g.dist_tiles = (q.H + g.dist_rows - 1) / g.dist_rows;
    const int rows = v.R * kBatchWaves;
    g.G = (q.H + rows - 1) / rows;
    g.S = (q.W + kWave - 1) / kWave;
    g.NG = (q.Ct + v.ctm - 1) / v.ctm;
    g.rows_tiles = (q.H + g.row_rows - 1) / g.row_rows;
    g.col_tiles = g.NG * g.S * g.G;
    g.phases = 1 + 2 * q.filter_iters * q.solver_iters;  // distances, then the passes
    return g;
}

struct BatchLayout {
    size_t inst = 0, prefix = 0, tickets = 0, bufs = 0, total = 0;
    int n_phases = 0, total_tiles = 0, max_G = 0;
    std::vector<Geo> geo;
};

static int make_batch_layout(const dts_problem* probs, int n, const BatchVariant& v, BatchLayout& L) {
    if (n < 1 || n > kBatchMaxProblems) return DTS_ENOTSUP;
    L.geo.resize(n);
    long long tiles = 0;
    for (int i = 0; i < n; ++i) {
        int rc = check_problem(probs[i]);
        if (rc) return rc;
        L.geo[i] = geometry(probs[i], v);
        L.n_phases = std::max(L.n_phases, L.geo[i].phases);
        L.max_G = std::max(L.max_G, L.geo[i].G);
        tiles += L.geo[i].dist_tiles + static_cast<long long>(probs[i].filter_iters) *
                                           probs[i].solver_iters * (L.geo[i].rows_tiles + L.geo[i].col_tiles);
    }
    if (tiles > (1LL << 30)) return DTS_ENOTSUP;
    L.total_tiles = static_cast<int>(tiles);
    size_t off = 1024;  // header: status, launch count, barrier counters
    L.inst = off;
    off = bal(off + sizeof(BInst) * n);
    L.prefix = off;
    off = bal(off + sizeof(int) * static_cast<size_t>(L.n_phases) * (n + 1));
    L.tickets = off;
    off = bal(off + sizeof(unsigned) * static_cast<size_t>(L.n_phases));
    L.bufs = off;
    for (int i = 0; i < n; ++i) {
        const dts_problem& q = probs[i];
        Geo& g = L.geo[i];
        const size_t plane = static_cast<size_t>(q.H) * q.W * sizeof(float);
        g.dx = off;
        off = bal(off + plane);
        g.dy = off;
        off = bal(off + plane);
        g.tmp = off;
        off = bal(off + plane * q.Ct);
        g.carry = off;
        g.carry_bytes = bal(static_cast<size_t>(g.NG) * g.S * g.G * carry_words_per_chunk(v.ctm) * kWave *
                            sizeof(unsigned long long));
        off += g.carry_bytes;
    }
    L.total = off;
    return DTS_OK;
}

constexpr size_t kBBarrier = 256, kBLaunch = 128;  // barrier: 9 counters 64 bytes apart

}  // namespace dts

using namespace dts;

extern "C" {

int dts_batched_variant_count(void) { return num_batch_variants(); }

int dts_batched_variant_info(int variant, int* rows_per_wave, int* group_channels, int* row_tile_pixels) {
    if (!rows_per_wave || !group_channels || !row_tile_pixels) return DTS_EINVAL;
    return batch_variant_info(variant, rows_per_wave, group_channels, row_tile_pixels);
}

size_t dts_batched_workspace_bytes(const dts_problem* probs, int n, int variant) {
    if (!probs || n < 1 || variant < 0 || variant >= kNumBatchVariants) return 0;
    BatchLayout L;
    if (make_batch_layout(probs, n, kBatchVariants[variant], L)) return 0;
    return L.total;
}

int dts_batched_prepare(const dts_problem* probs, int n, float lambda, float step, int variant,
                        void* workspace, size_t workspace_bytes, dts_batched_plan* plan, void* stream) {
    if (!probs || n < 1 || !plan || !std::isfinite(lambda) || !std::isfinite(step)) return DTS_EINVAL;
    if (variant < 0 || variant >= kNumBatchVariants) return DTS_EINVAL;
    const BatchVariant& v = kBatchVariants[variant];
    BatchLayout L;
    int rc = make_batch_layout(probs, n, v, L);
    if (rc) return rc;
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return DTS_EWORKSPACE;
    const int cap = v.capacity();
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (L.max_G > cap) return DTS_ENOTSUP;
    char* base = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);

    // tables, built on the host and copied once
    std::vector<char> img(L.bufs - L.inst, 0);
    auto at = [&](size_t off) { return img.data() + (off - L.inst); };
    BInst* inst = reinterpret_cast<BInst*>(at(L.inst));
    for (int i = 0; i < n; ++i) {
        const dts_problem& q = probs[i];
        const Geo& g = L.geo[i];
        BInst& I = inst[i];
        I.guide = q.guide;
        I.target = q.target;
        I.conf = q.conf;
        I.out = q.out;
        I.dx = reinterpret_cast<float*>(base + g.dx);
        I.dy = reinterpret_cast<float*>(base + g.dy);
        I.tmp = reinterpret_cast<float*>(base + g.tmp);
        I.carry = reinterpret_cast<unsigned long long*>(base + g.carry);
        I.H = q.H;
        I.W = q.W;
        I.Cg = q.Cg;
        I.Ct = q.Ct;
        I.Cc = q.Cc;
        I.N = q.filter_iters;
        I.T = q.solver_iters;
        I.row_S = g.row_S;
        I.row_gw = g.row_gw;
        I.row_rows = g.row_rows;
        I.dist_rows = g.dist_rows;
        I.G = g.G;
        I.S = g.S;
        I.NG = g.NG;
        const double r = static_cast<double>(q.sigma_s) / q.sigma_r;
        I.s2 = static_cast<float>(r * r);
        for (int f = 0; f < kBatchMaxN; ++f) {
            if (f < q.filter_iters) {
                const double sh = q.sigma_s * std::sqrt(3.0) * std::ldexp(1.0, q.filter_iters - 1 - f) /
                                  std::sqrt(std::ldexp(1.0, 2 * q.filter_iters) - 1.0);
                I.log2a[f] = static_cast<float>(-std::sqrt(2.0) / sh / std::log(2.0));
            } else {
                I.log2a[f] = 0.f;
            }
        }
    }
    int* pre = reinterpret_cast<int*>(at(L.prefix));
    for (int p = 0; p < L.n_phases; ++p) {
        int local = 0;
        for (int i = 0; i < n; ++i) {
            const Geo& g = L.geo[i];
            pre[static_cast<size_t>(p) * (n + 1) + i] = local;
            int tiles = 0;
            if (p == 0) tiles = g.dist_tiles;
            else if (p < g.phases) tiles = ((p - 1) & 1) ? g.col_tiles : g.rows_tiles;
            local += tiles;
        }
        pre[static_cast<size_t>(p) * (n + 1) + n] = local;
    }
    if ((rc = launch_zero(base, L.inst, s))) return rc;
    if ((rc = hip_fail(hipMemcpyAsync(base + L.inst, img.data(), img.size(), hipMemcpyHostToDevice, s))))
        return rc;
    for (int i = 0; i < n; ++i)
        if ((rc = launch_zero(base + L.geo[i].carry, L.geo[i].carry_bytes, s))) return rc;
    if ((rc = hip_fail(hipStreamSynchronize(s)))) return rc;  // img is host memory

    memset(plan, 0, sizeof(*plan));
    plan->n = n;
    plan->variant = variant;
    plan->n_phases = L.n_phases;
    plan->total_tiles = L.total_tiles;
    plan->grid = cap;  // all co-resident: the phases meet at grid barriers
    plan->workspace_bytes = L.total;
    plan->off_inst = L.inst;
    plan->off_prefix = L.prefix;
    plan->off_tickets = L.tickets;
    plan->lambda = lambda;
    plan->step = step;
    return DTS_OK;
}

int dts_solve_batched(const dts_batched_plan* plan, void* workspace, void* stream) {
    if (!plan || !workspace || plan->n < 1 || plan->variant < 0 || plan->variant >= kNumBatchVariants)
        return DTS_EINVAL;
    char* base = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan->grid < 1 || plan->grid > kBatchVariants[plan->variant].capacity()) return DTS_EINVAL;
    BatchArgs a;
    a.inst = reinterpret_cast<const BInst*>(base + plan->off_inst);
    a.phase_prefix = reinterpret_cast<const int*>(base + plan->off_prefix);
    a.tickets = reinterpret_cast<unsigned*>(base + plan->off_tickets);
    a.barrier = reinterpret_cast<unsigned*>(base + kBBarrier);
    a.launch = reinterpret_cast<const unsigned*>(base + kBLaunch);
    a.status = reinterpret_cast<int*>(base);
    a.spin_limit = spin_limit();
    a.tag_xor = spin_tag_xor();
    a.n = plan->n;
    a.n_phases = plan->n_phases;
    a.lambda = plan->lambda;
    a.step = plan->step;
    hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(256), 0, s, a.tickets, a.n_phases, a.barrier,
                       reinterpret_cast<unsigned*>(base + kBLaunch), a.status);
    int rc = hip_fail(hipGetLastError());
    if (rc) return rc;
    ProfScope prof("batched_solve", 0.0, s);
    kBatchVariants[plan->variant].launch(a, static_cast<unsigned>(plan->grid), s);
    return hip_fail(hipGetLastError());
}

}  // extern "C"
