// Forward kernels of the domain-transform filter on gfx950.
//
// Method (Bapat & Frahm, "The Domain Transform Solver", ECCV 2018): the edge-aware mean of
// Sec. 3.2 computed with the recursive domain-transform filter -- per-pixel transformed
// distances from the guide's channel differences (Eq. (8)-(9)), weights a^d, and
// alternating causal+anticausal first-order recursive passes along rows and columns.
//
// Row pass: one workgroup per row (one-channel signals: a persistent grid walking the
// rows, each workgroup loading its next row while it scans the current one).  Lane l of
// wave v owns S consecutive pixels (float4 accesses).  Each direction of the recurrence is a chain of affine maps: a serial
// composition over the lane's S pixels, one 64-lane scan (DPP inside rows of 16 lanes,
// scalar reads across rows), one exchange of wave totals through LDS, then a serial sweep
// from the lane's exact carry-in.
//
// Column pass: lanes are columns (every access is a coalesced 256-byte row segment per
// wave), each workgroup owns a chunk of R rows of its strip and keeps it in registers.
// Chunks exchange carries through tagged 64-bit words in device memory: a decoupled
// look-back resolves the causal carry from earlier chunks, then a look-ahead resolves the
// anticausal carry from later chunks, so every element is read and written exactly once.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>

#include "../../include/dts.h"
#include "dts_chunks.hpp"
#include "dts_device.hpp"
#include "dts_internal.hpp"
#include "dts_tiles.hpp"

namespace dts {

// ---------------------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------------------
// SQ: the first pass of a variance (Eq. (7)): a.C output channels, the pairs z, z^2 of
// a.C / 2 input channels.
template <int S, bool DIST, bool SQ>
__global__ void __launch_bounds__(1024) row_pass_kernel(RowArgs a) {
    // the fused distance pass reads each guide row twice (as row y and as the row above
    // row y + 1): XCD bands keep the second read in L2
    const int y = DIST ? xcd_band_index(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
    row_tile<S, DIST, SQ>(a, y, blockIdx.y);
}


// Persistent row pass for one-channel signals: each workgroup walks rows r, r + grid, ...
// of the batch and issues the loads of its next row before it scans the current one, so
// the next row's loads are in flight during the current row's scans, barriers and
// stores.  Every LDS slot is rewritten only after a barrier that follows all reads of its
// previous contents, so consecutive rows need no extra barrier.
template <int S>
__global__ void __launch_bounds__(1024) row_pass_stream_kernel(RowArgs a, int rows) {
    __shared__ float2 fagg[kMaxRowWaves];
    __shared__ float2 bagg[kMaxRowWaves];
    __shared__ float wfirst[kMaxRowWaves + 1];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int W = a.W;
    const int n0 = (wave * kWave + lane) * S;
    float fN[S], dN[S];
    int r = blockIdx.x;
    if (r < rows) {
        load_seg<S>(a.src + static_cast<size_t>(r) * W, n0, W, 0.f, fN);
        load_seg<S>(a.d + static_cast<size_t>(r) * W, n0, W, 1.f, dN);
    }
    for (; r < rows; r += gridDim.x) {
        float f[S], w[S];
#pragma unroll
        for (int e = 0; e < S; ++e) {
            f[e] = fN[e];
            const int n = n0 + e;
            w[e] = (n > 0 && n < W) ? weight(dN[e], a.log2a) : 0.f;
        }
        const int rn = r + gridDim.x;
        if (rn < rows) {
            load_seg<S>(a.src + static_cast<size_t>(rn) * W, n0, W, 0.f, fN);
            load_seg<S>(a.d + static_cast<size_t>(rn) * W, n0, W, 1.f, dN);
        }
        float wlast = __shfl_down(w[0], 1);
        if (lane == 0) wfirst[wave] = w[0];
        if (wave == 0 && lane == 0) wfirst[nw] = 0.f;
        __syncthreads();
        if (lane == kWave - 1) wlast = wfirst[wave + 1];
        float la = 1.f, lb = 0.f;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            lb = fmaf(w[e], lb - f[e], f[e]);
            la *= w[e];
        }
        scan_up_dpp(la, lb, lane);
        float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
        if (lane == kWave - 1) fagg[wave] = make_float2(la, lb);
        __syncthreads();
        float jin = 0.f;
        for (int u = 0; u < wave; ++u) {
            const float2 g = fagg[u];
            jin = fmaf(g.x, jin, g.y);
        }
        float j = (lane == 0) ? jin : fmaf(xa, jin, xb);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            j = fmaf(w[e], j - f[e], f[e]);
            f[e] = j;
        }
        la = 1.f;
        lb = 0.f;
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            lb = fmaf(wn, lb - f[e], f[e]);
            la *= wn;
        }
        scan_down_dpp(la, lb, lane);
        xa = __shfl_down(la, 1);
        xb = __shfl_down(lb, 1);
        if (lane == 0) bagg[wave] = make_float2(la, lb);
        __syncthreads();
        float kin = 0.f;
        for (int u = nw - 1; u > wave; --u) {
            const float2 g = bagg[u];
            kin = fmaf(g.x, kin, g.y);
        }
        float k = (lane == kWave - 1) ? kin : fmaf(xa, kin, xb);
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            k = fmaf(wn, k - f[e], f[e]);
            f[e] = k;
        }
        store_seg<S>(a.dst + static_cast<size_t>(r) * W, n0, W, f);
    }
}

// Resident workgroups of the streaming row pass on the current device (its grid).
template <int S>
static int row_stream_grid(int threads) {
    static int cached[64][kMaxRowWaves + 1] = {};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    const int nw = threads / kWave;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev][nw] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, row_pass_stream_kernel<S>, threads, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev][nw] = std::max(1, per_cu * cus);
    }
    return cached[dev][nw];
}

template <int S, bool DIST, bool SQ = false>
static void launch_row_t(const RowArgs& a, int nw, int batch, int H, hipStream_t s) {
    // algorithmic bytes: signal in and out (C planes), distances in -- or, on the fused
    // first pass, the guide in (Cg planes) and both distance planes out instead
    const double px = static_cast<double>(batch) * H * a.W;
    const double cin = SQ ? 0.5 * a.C : a.C;  // planes read for a.C planes written
    const double bytes = DIST ? px * 4.0 * (cin + a.C + a.Cg + 2.0) : px * 4.0 * (cin + a.C + 1.0);
    ProfScope prof(SQ ? "row_pass_dist_square" : DIST ? "row_pass_dist" : "row_pass", bytes, s);
    if constexpr (!DIST && !SQ) {
        // one channel: the streaming kernel; several channels share each row's distances
        // in the per-row kernel instead
        const int grid = (a.C == 1) ? row_stream_grid<S>(nw * kWave) : 0;
        if (grid > 0) {
            const int rows = batch * H;
            hipLaunchKernelGGL((row_pass_stream_kernel<S>), dim3(std::min(rows, grid)), dim3(nw * kWave), 0, s, a,
                               rows);
            return;
        }
    }
    hipLaunchKernelGGL((row_pass_kernel<S, DIST, SQ>), dim3(H, batch), dim3(nw * kWave), 0, s, a);
}

// Pixels per lane for a row of width W: long rows use longer lane segments so one wave
// scan covers more pixels; at most 16 waves per row.
static int g_row_pin = 0;

static int row_segment(int W) {
    if (g_row_pin && (W + kWave * g_row_pin - 1) / (kWave * g_row_pin) <= kMaxRowWaves) return g_row_pin;
    return W > 4096 ? 16 : W > 1024 ? 8 : 4;
}

int tune_row_segment(int S) {
    if (S != 0 && S != 4 && S != 8 && S != 16) return DTS_EINVAL;
    g_row_pin = S;
    return DTS_OK;
}

int launch_row_pass(const RowPass& p, Ctx& ctx) {
    RowArgs a;
    a.src = p.src;
    a.dst = p.dst;
    a.d = p.d;
    a.guide = p.guide;
    a.dx_out = p.dx_out;
    a.dy_out = p.dy_out;
    a.Cg = p.Cg;
    a.s2 = p.s2;
    a.C = p.C;
    a.H = p.H;
    a.W = p.W;
    a.log2a = p.log2a;
    const bool dist = p.guide != nullptr;
    const hipStream_t s = ctx.stream;
    const int S = row_segment(p.W);
    const int nw = (p.W + kWave * S - 1) / (kWave * S);
    if (nw > kMaxRowWaves) return DTS_ENOTSUP;
    if (p.sq) {  // first pass of a variance: always with the distances
        if (!dist || (p.C & 1)) return DTS_EINVAL;
        switch (S) {
            case 4: launch_row_t<4, true, true>(a, nw, p.batch, p.H, s); break;
            case 8: launch_row_t<8, true, true>(a, nw, p.batch, p.H, s); break;
            default: launch_row_t<16, true, true>(a, nw, p.batch, p.H, s); break;
        }
        return hip_fail(hipGetLastError());
    }
    switch (S) {
        case 4: dist ? launch_row_t<4, true>(a, nw, p.batch, p.H, s) : launch_row_t<4, false>(a, nw, p.batch, p.H, s); break;
        case 8: dist ? launch_row_t<8, true>(a, nw, p.batch, p.H, s) : launch_row_t<8, false>(a, nw, p.batch, p.H, s); break;
        default: dist ? launch_row_t<16, true>(a, nw, p.batch, p.H, s) : launch_row_t<16, false>(a, nw, p.batch, p.H, s); break;
    }
    return hip_fail(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// Column pass
// ---------------------------------------------------------------------------------------
// Waves per SIMD the register allocation must leave room for: the 40-row single-channel
// chunk only pays off with two 8-wave workgroups per CU, i.e. at most 128 VGPRs.
template <int CT, int R, int NWV>
constexpr int col_min_waves() { return (CT == 1 && R == 40 && NWV == 8) ? 4 : 1; }

template <int CT, int R, int NWV, int EPI>
__global__ void __launch_bounds__(kWave * NWV, (col_min_waves<CT, R, NWV>())) col_pass_kernel(ColArgs a) {
    __shared__ ChunkLds<CT, NWV> L;
    const CarryCtx cctx{a.carry, a.epoch, a.status, a.G, a.S, a.NG, a.spin_limit, a.tag_xor};
    // Persistent grid: a workgroup always processes the same chunk of the strips
    // group, group + groups, ...; every strip's chunks are thus held by G workgroups of
    // the same launch that are all running, and none ever waits on one not yet started.
    const ChunkSlot slot = chunk_slot(static_cast<int>(blockIdx.x), a.G, a.xcd);
    const int chunk = slot.chunk;
    const int group = slot.group;
    if (group >= a.groups) return;
    const int n_strips = a.batch * a.NG * a.S;
#pragma unroll 1
    for (int sid = group; sid < n_strips; sid += a.groups) {
        const int strip = sid % a.S;
        const int grp = (sid / a.S) % a.NG;
        const int b = sid / (a.S * a.NG);
        col_tile<CT, R, NWV, EPI>(a, cctx, L, chunk, strip, grp, b);
    }
}

// ---------------------------------------------------------------------------------------
// Column-pass variants: rows per wave R and waves per workgroup NWV (a chunk is R * NWV
// rows of one 64-column strip) for each channel-group size CT.  The default choice per
// shape comes from col_variant(); dts_tune_col_variant() can pin another one.
// ---------------------------------------------------------------------------------------
struct ColVariant {
    int ct, R, nwv;
    int (*launch)(const ColArgs&, unsigned, hipStream_t, int);  // mode: col_tile's EPI
    int (*capacity)(int);
};

template <int CT, int R, int NWV, int EPI>
static int col_capacity_t() {
    static int cached[64] = {0};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, col_pass_kernel<CT, R, NWV, EPI>,
                                                         kWave * NWV, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

template <int CT, int R, int NWV>
static int col_capacity_v(int mode) {
    if (mode == 3) {
        if constexpr (CT % 2 == 0) return col_capacity_t<CT, R, NWV, 3>();
        else return 0;
    }
    return mode == 2 ? col_capacity_t<CT, R, NWV, 2>()
                     : mode == 1 ? col_capacity_t<CT, R, NWV, 1>() : col_capacity_t<CT, R, NWV, 0>();
}

template <int CT, int R, int NWV>
static int col_launch_v(const ColArgs& a, unsigned n, hipStream_t s, int mode) {
    if (mode == 3) {
        if constexpr (CT % 2 == 0)  // the variance epilogue takes channel pairs
            hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, 3>), dim3(n), dim3(kWave * NWV), 0, s, a);
        else
            return DTS_ENOTSUP;
    } else if (mode == 2) {
        if constexpr (CT == 1)  // the data-gradient update serves single-channel solves
            hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, 2>), dim3(n), dim3(kWave * NWV), 0, s, a);
        else
            return DTS_ENOTSUP;
    } else if (mode == 1) {
        hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, 1>), dim3(n), dim3(kWave * NWV), 0, s, a);
    } else {
        hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, 0>), dim3(n), dim3(kWave * NWV), 0, s, a);
    }
    return hip_fail(hipGetLastError());
}

#define DTS_COL_VARIANT(CT, R, NWV) \
    ColVariant { CT, R, NWV, col_launch_v<CT, R, NWV>, col_capacity_v<CT, R, NWV> }

static const ColVariant kColVariants[] = {
    DTS_COL_VARIANT(1, 32, 8),   // 0: 256-row chunks
    DTS_COL_VARIANT(1, 16, 8),   // 1: 128
    DTS_COL_VARIANT(1, 32, 4),   // 2: 128
    DTS_COL_VARIANT(1, 16, 16),  // 3: 256
    DTS_COL_VARIANT(1, 32, 16),  // 4: 512
    DTS_COL_VARIANT(2, 24, 8),   // 5: 192
    DTS_COL_VARIANT(2, 16, 8),   // 6: 128
    DTS_COL_VARIANT(3, 16, 8),   // 7: 128
    DTS_COL_VARIANT(3, 8, 16),   // 8: 128
    DTS_COL_VARIANT(4, 16, 8),   // 9: 128
    DTS_COL_VARIANT(1, 40, 8),   // 10: 320, held to 128 VGPRs
};
constexpr int kNumColVariants = sizeof(kColVariants) / sizeof(kColVariants[0]);
constexpr int kMinChunkRows = 128;   // smallest R * NWV above: sizes the carry area

static int col_group(int C) { return C < 4 ? C : 4; }

static int g_col_pin[5] = {-1, -1, -1, -1, -1};   // per channel-group size, -1 = default

// Default variant per channel-group size.  Single-channel passes over images of 2048 rows
// or more take the 320-row chunk: more bytes in flight per workgroup and fewer chunks per
// strip (10240 rows: 32 chunks, so 16 strips fill the 512 resident workgroups exactly).
// Shorter images keep the 256-row chunk, whose extra chunks give them more parallelism.
static int col_variant(int C, int H) {
    const int ct = col_group(C);
    const int pin = g_col_pin[ct];
    if (pin >= 0 && pin < kNumColVariants && kColVariants[pin].ct == ct) return pin;
    switch (ct) {
        case 1: return H >= 2048 ? 10 : 0;
        case 2: return 6;
        case 3: return 7;
        default: return 9;
    }
}

int tune_col_variant(int ct, int variant) {
    if (ct < 1 || ct > 4) return DTS_EINVAL;
    if (variant >= kNumColVariants || (variant >= 0 && kColVariants[variant].ct != ct)) return DTS_EINVAL;
    g_col_pin[ct] = variant < 0 ? -1 : variant;
    return DTS_OK;
}

int col_variant_info(int variant, int* ct, int* rows_per_wave, int* waves) {
    if (variant < 0 || variant >= kNumColVariants) return DTS_EINVAL;
    *ct = kColVariants[variant].ct;
    *rows_per_wave = kColVariants[variant].R;
    *waves = kColVariants[variant].nwv;
    return DTS_OK;
}

int num_col_variants() { return kNumColVariants; }

static int g_spin_limit = kSpinLimit;
static unsigned g_spin_tag_xor = 0u;

int tune_spin_limit(int polls) {
    if (polls == 0) {
        g_spin_limit = kSpinLimit;
        g_spin_tag_xor = 0u;
    } else if (polls > 0) {
        g_spin_limit = polls;
        g_spin_tag_xor = 0u;
    } else {
        g_spin_limit = polls == INT_MIN ? INT_MAX : -polls;
        g_spin_tag_xor = 0x80000000u;
    }
    return DTS_OK;
}

int spin_limit() { return g_spin_limit; }
unsigned spin_tag_xor() { return g_spin_tag_xor; }

static int g_col_xcd = 1;

int tune_col_xcd(int on) {
    g_col_xcd = on ? 1 : 0;
    return DTS_OK;
}

static int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cached[dev] = cus;
    }
    return cached[dev];
}

// Strips in flight and grid size of a persistent column pass.  The XCD-local form needs
// the CUs split evenly over the XCDs and a strip's G chunks to fit in one XCD's share of
// the capacity; its grid is a whole number of rounds of the 8 XCDs, and the workgroups of
// groups past n_strips exit at once.
ColGrid col_grid(int cap, int G, long long n_strips) {
    ColGrid g{};
    const int cus = device_cus();
    const int per_xcd = (cus > 0 && cus % kXcds == 0) ? cap / kXcds : 0;
    if (g_col_xcd && per_xcd >= G) {
        const long long groups = std::min<long long>(static_cast<long long>(per_xcd / G) * kXcds, n_strips);
        const long long rounds = (groups + kXcds - 1) / kXcds;
        g.groups = static_cast<int>(groups);
        g.n = static_cast<unsigned>(rounds * kXcds * G);
        g.xcd = 1;
        return g;
    }
    g.groups = static_cast<int>(std::min<long long>(cap / G, n_strips));
    g.n = static_cast<unsigned>(g.groups) * G;
    g.xcd = 0;
    return g;
}

size_t col_carry_words(int batch, int H, int W, int C) {
    // sized for the smallest chunk of any variant so every variant fits
    const int ct = col_group(C);
    const size_t G = (H + kMinChunkRows - 1) / kMinChunkRows;
    const size_t S = (W + kWave - 1) / kWave;
    const size_t NG = (C + ct - 1) / ct;
    return static_cast<size_t>(batch) * NG * S * G * carry_words_per_chunk(ct) * kWave;
}

int launch_col_pass(const ColPass& p, Ctx& ctx) {
    const ColVariant& v = kColVariants[col_variant(p.C, p.H)];
    ColArgs a;
    a.src = p.src;
    a.dst = p.dst;
    a.d = p.d;
    a.C = p.C;
    a.H = p.H;
    a.W = p.W;
    a.log2a = p.log2a;
    const int ct = v.ct;
    const int rows = v.R * v.nwv;
    a.G = (p.H + rows - 1) / rows;
    a.S = (p.W + kWave - 1) / kWave;
    a.NG = (p.C + ct - 1) / ct;
    a.batch = p.batch;
    a.carry = ctx.carry;
    a.epoch = ++ctx.epoch;
    a.status = ctx.status;
    a.spin_limit = spin_limit();
    a.tag_xor = spin_tag_xor();
    a.zk = p.zk;
    a.tgt = p.tgt;
    a.conf = p.conf;
    a.Cc = p.Cc;
    a.dst2 = p.dst2;
    a.lambda = p.lambda;
    a.step = p.step;
    a.var_k = p.var_k;
    // every workgroup of the grid must be resident at once: size the grid to the
    // device's capacity for this kernel, in whole strips of G chunks
    const int mode = p.variance ? 3 : !p.epilogue ? 0 : p.data_grad ? 2 : 1;
    if (mode == 2 && v.ct != 1) return DTS_ENOTSUP;
    if (mode == 3 && ((p.C & 1) || (v.ct & 1))) return DTS_EINVAL;
    const int cap = v.capacity(mode);
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (a.G > cap) return DTS_ENOTSUP;
    const ColGrid grid = col_grid(cap, a.G, static_cast<long long>(p.batch) * a.NG * a.S);
    a.groups = grid.groups;
    a.xcd = grid.xcd;
    const unsigned n = grid.n;
    // algorithmic bytes: signal in and out, distances in; the update epilogue also reads
    // z^k, the target and the confidence (or z^k and the data-term gradient)
    const double px = static_cast<double>(p.batch) * a.H * a.W;
    const double bytes = mode == 1   ? px * 4.0 * (4.0 * a.C + 1.0 + (a.Cc == 1 ? 1.0 : a.C))
                         : mode == 2 ? px * 4.0 * (4.0 * a.C + 1.0)
                         : mode == 3 ? px * 4.0 * (1.5 * a.C + 1.0)  // pairs and distances in, C / 2 out
                                     : px * 4.0 * (2.0 * a.C + 1.0);
    ProfScope prof(mode == 1   ? "col_pass_update"
                   : mode == 2 ? "col_pass_update_grad"
                   : mode == 3 ? "col_pass_variance_conf"
                               : "col_pass",
                   bytes, ctx.stream);
    return v.launch(a, n, ctx.stream, mode);
}

// ---------------------------------------------------------------------------------------
// Small utility kernels (fills instead of hipMemsetAsync so calls stay graph-capturable)
// ---------------------------------------------------------------------------------------
__global__ void zero_kernel(uint4* p, size_t n16) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void zero_bytes_kernel(unsigned char* p, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

__global__ void copy_kernel(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// Eq. (7): c = exp(-V / (2 sigma_c^2)) with V = DT(z^2) - DT(z)^2, taken in the last
// column pass of the variance filter (col_tile's EPI 3) as exp2(k V) with
// k = -log2(e) / (2 sigma_c^2), rounded once from double.
float variance_k(float sigma_c) {
    return static_cast<float>(-1.0 / (2.0 * static_cast<double>(sigma_c) * sigma_c * std::log(2.0)));
}

// Data-term gradient of the stereo objective (Eq. (11)) at the disparity z, one pixel per
// thread:  D = c rho'(z - t) + gamma sum_k (I_L,k - I_R,k(x - z)) dI_R,k/dx (x - z), with
// rho(r) = sqrt(r^2 + eps^2).  I_R is read linearly along the pixel's row at x - z; the
// position is clamped to [0, W - 1] and the slope is 0 where it was clamped.
__global__ void __launch_bounds__(256) stereo_data_grad_kernel(const float* __restrict__ z,
                                                                const float* __restrict__ t,
                                                                const float* __restrict__ c,
                                                                const float* __restrict__ left,
                                                                const float* __restrict__ right,
                                                                float* __restrict__ D, int Cg, int H, int W,
                                                                size_t total, float gamma, float eps2) {
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
        const size_t b = e / plane;
        const size_t i = e - b * plane;
        const int y = static_cast<int>(i / W);
        const int x = static_cast<int>(i - static_cast<size_t>(y) * W);
        const float zz = z[e];
        const float r = zz - t[e];
        const float g = c[e] * r / sqrtf(fmaf(r, r, eps2));
        const float xs = static_cast<float>(x) - zz;
        const float xc = fminf(fmaxf(xs, 0.f), static_cast<float>(W - 1));
        const bool inside = xs >= 0.f && xs <= static_cast<float>(W - 1);
        const int x0 = W > 1 ? min(static_cast<int>(floorf(xc)), W - 2) : 0;
        const int x1 = W > 1 ? x0 + 1 : 0;
        const float fr = xc - static_cast<float>(x0);
        float photo = 0.f;
        for (int k = 0; k < Cg; ++k) {
            const size_t row = ((b * Cg + k) * H + y) * static_cast<size_t>(W);
            const float r0 = right[row + x0];
            const float r1 = right[row + x1];
            const float val = fmaf(fr, r1 - r0, r0);
            const float slope = inside ? r1 - r0 : 0.f;
            photo = fmaf(left[row + x] - val, slope, photo);
        }
        D[e] = fmaf(gamma, photo, g);
    }
}

int launch_stereo_data_grad(const float* z, const float* t, const float* c, const float* left, const float* right,
                            float* D, int Cg, int batch, int H, int W, float gamma, float eps, hipStream_t s) {
    const size_t total = static_cast<size_t>(batch) * H * W;
    const size_t blocks = std::min<size_t>((total + 255) / 256, 65536);
    // z, t, c in, D out, the left image and two right-image samples per band (read once
    // from HBM when the disparity varies slowly along the row)
    ProfScope prof("stereo_data_grad", static_cast<double>(total) * 4.0 * (4.0 + 2.0 * Cg), s);
    hipLaunchKernelGGL(stereo_data_grad_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, z, t, c,
                       left, right, D, Cg, H, W, total, gamma, eps * eps);
    return hip_fail(hipGetLastError());
}

// Clears `bytes` bytes at any alignment: 16-byte stores over the aligned middle, byte
// stores over the unaligned head and tail.
int launch_zero(void* ptr, size_t bytes, hipStream_t s) {
    if (bytes == 0) return 0;
    unsigned char* p = static_cast<unsigned char*>(ptr);
    const size_t head = std::min<size_t>((16 - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u, bytes);
    const size_t n16 = (bytes - head) / 16;
    const size_t tail = bytes - head - n16 * 16;
    if (n16) {
        const size_t blocks = (n16 + 255) / 256;
        const unsigned g = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
        hipLaunchKernelGGL(zero_kernel, dim3(g), dim3(256), 0, s, reinterpret_cast<uint4*>(p + head), n16);
    }
    if (head) hipLaunchKernelGGL(zero_bytes_kernel, dim3(1), dim3(64), 0, s, p, head);
    if (tail) hipLaunchKernelGGL(zero_bytes_kernel, dim3(1), dim3(64), 0, s, p + head + n16 * 16, tail);
    return hip_fail(hipGetLastError());
}

int launch_copy(float* dst, const float* src, size_t n, hipStream_t s) {
    if (n == 0) return 0;
    const size_t blocks = (n + 255) / 256;
    const unsigned g = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(copy_kernel, dim3(g), dim3(256), 0, s, dst, src, n);
    return hip_fail(hipGetLastError());
}

}  // namespace dts
