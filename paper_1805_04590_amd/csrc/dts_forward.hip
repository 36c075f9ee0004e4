// Forward kernels of the domain-transform filter on gfx950.
//
// Method (Bapat & Frahm, "The Domain Transform Solver", ECCV 2018): the edge-aware mean of
// Sec. 3.2 computed with the recursive domain-transform filter -- per-pixel transformed
// distances from the guide's channel differences (Eq. (8)-(9)), weights a^d, and
// alternating causal+anticausal first-order recursive passes along rows and columns.
//
// Row pass: one workgroup per row.  Lane l of wave v owns S consecutive pixels (float4
// accesses).  Each direction of the recurrence is a chain of affine maps: a serial
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
#include <mutex>

#include "../../include/dts.h"
#include "dts_chunks.hpp"
#include "dts_device.hpp"
#include "dts_internal.hpp"

namespace dts {

// ---------------------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------------------
struct RowArgs {
    const float* src;
    float* dst;
    const float* d;
    const float* guide;
    float* dx_out;
    float* dy_out;
    int Cg;
    float s2;
    int C, H, W;
    float log2a;
};

constexpr int kMaxRowWaves = 16;

template <int S>
__device__ __forceinline__ void load_seg(const float* row, int n0, int W, bool vec, float fill,
                                         float (&v)[S]) {
    if (vec && n0 + S <= W) {
#pragma unroll
        for (int e = 0; e < S; e += 4) {
            const float4 q = *reinterpret_cast<const float4*>(row + n0 + e);
            v[e] = q.x;
            v[e + 1] = q.y;
            v[e + 2] = q.z;
            v[e + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < S; ++e) v[e] = (n0 + e < W) ? row[n0 + e] : fill;
    }
}

template <int S>
__device__ __forceinline__ void store_seg(float* row, int n0, int W, bool vec, const float (&v)[S]) {
    if (vec && n0 + S <= W) {
#pragma unroll
        for (int e = 0; e < S; e += 4)
            *reinterpret_cast<float4*>(row + n0 + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    } else {
#pragma unroll
        for (int e = 0; e < S; ++e)
            if (n0 + e < W) row[n0 + e] = v[e];
    }
}

// One workgroup per row; lane l of wave v owns the S consecutive pixels starting at
// (64 v + l) S.  Per direction: a serial composition of the lane's S maps, one 64-lane
// scan, one exchange of wave totals through LDS, and a serial sweep that produces the
// final values.
template <int S, bool DIST>
__global__ void __launch_bounds__(1024) row_pass_kernel(RowArgs a) {
    __shared__ float2 fagg[kMaxRowWaves];
    __shared__ float2 bagg[kMaxRowWaves];
    __shared__ float wfirst[kMaxRowWaves + 1];

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int y = blockIdx.x;
    const int b = blockIdx.y;
    const int H = a.H, W = a.W;
    const size_t plane = static_cast<size_t>(H) * W;
    const int n0 = (wave * kWave + lane) * S;
    const bool vec = (W & 3) == 0;

    float w[S];
    if constexpr (DIST) {
        float ax[S], ay[S];
#pragma unroll
        for (int e = 0; e < S; ++e) ax[e] = ay[e] = 0.f;
        for (int k = 0; k < a.Cg; ++k) {
            const float* g = a.guide + (static_cast<size_t>(b) * a.Cg + k) * plane +
                             static_cast<size_t>(y) * W;
            const float* gu = (y > 0) ? g - W : g;
            float v[S], u[S];
            load_seg<S>(g, n0, W, vec, 0.f, v);
            load_seg<S>(gu, n0, W, vec, 0.f, u);
            float prev = __shfl_up(v[S - 1], 1);
            if (lane == 0) prev = (n0 > 0 && n0 <= W) ? g[n0 - 1] : v[0];
#pragma unroll
            for (int e = 0; e < S; ++e) {
                const float ex = v[e] - (e == 0 ? prev : v[e > 0 ? e - 1 : 0]);
                const float ey = v[e] - u[e];
                ax[e] = fmaf(ex, ex, ax[e]);
                ay[e] = fmaf(ey, ey, ay[e]);
            }
        }
        float* dxr = a.dx_out + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
        float* dyr = a.dy_out + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            ax[e] = sqrtf(fmaf(a.s2, ax[e], 1.f));
            ay[e] = sqrtf(fmaf(a.s2, ay[e], 1.f));
        }
        store_seg<S>(dxr, n0, W, vec, ax);
        store_seg<S>(dyr, n0, W, vec, ay);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < W) ? weight(ax[e], a.log2a) : 0.f;
        }
    } else {
        const float* dr = a.d + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
        float dv[S];
        load_seg<S>(dr, n0, W, vec, 1.f, dv);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < W) ? weight(dv[e], a.log2a) : 0.f;
        }
    }
    // weight linking each lane's last pixel to the next pixel (0 past the end of the row)
    if (lane == 0) wfirst[wave] = w[0];
    if (threadIdx.x == 0) wfirst[nw] = 0.f;
    __syncthreads();
    float wlast = __shfl_down(w[0], 1);
    if (lane == kWave - 1) wlast = wfirst[wave + 1];

    for (int c = 0; c < a.C; ++c) {
        const size_t roff = (static_cast<size_t>(b) * a.C + c) * plane + static_cast<size_t>(y) * W;
        float f[S];
        load_seg<S>(a.src + roff, n0, W, vec, 0.f, f);

        // causal: J[n] = w[n] J[n-1] + (1 - w[n]) f[n]
        float la = 1.f, lb = 0.f;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            lb = fmaf(w[e], lb - f[e], f[e]);
            la *= w[e];
        }
        scan_up_dpp(la, lb, lane);
        if (lane == kWave - 1) fagg[wave] = make_float2(la, lb);
        float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
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

        // anticausal: K[n] = w[n+1] K[n+1] + (1 - w[n+1]) J[n]
        la = 1.f;
        lb = 0.f;
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            lb = fmaf(wn, lb - f[e], f[e]);
            la *= wn;
        }
        scan_down_dpp(la, lb, lane);
        if (lane == 0) bagg[wave] = make_float2(la, lb);
        xa = __shfl_down(la, 1);
        xb = __shfl_down(lb, 1);
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
        store_seg<S>(a.dst + roff, n0, W, vec, f);
    }
}

template <int S, bool DIST>
static void launch_row_t(const RowArgs& a, int nw, int batch, int H, hipStream_t s) {
    // algorithmic bytes: signal in and out (C planes), distances in -- or, on the fused
    // first pass, the guide in (Cg planes) and both distance planes out instead
    const double px = static_cast<double>(batch) * H * a.W;
    const double bytes = DIST ? px * 4.0 * (2.0 * a.C + a.Cg + 2.0) : px * 4.0 * (2.0 * a.C + 1.0);
    ProfScope prof(DIST ? "row_pass_dist" : "row_pass", bytes, s);
    hipLaunchKernelGGL((row_pass_kernel<S, DIST>), dim3(H, batch), dim3(nw * kWave), 0, s, a);
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
struct ColArgs {
    const float* src;
    float* dst;
    const float* d;
    int C, H, W;
    float log2a;
    int G, S, NG, batch;
    int groups;  // strips processed at once: the grid holds groups * G workgroups
    unsigned long long* carry;
    unsigned epoch;
    int* status;
    const float* zk;
    const float* tgt;
    const float* conf;
    int Cc;
    float* dst2;
    float lambda, step;
};

// One workgroup = NWV waves stacked vertically over one 64-column strip: wave v owns rows
// [r0 + v R, r0 + (v+1) R) of the chunk, one column per lane, all in registers.
template <int CT, int R, int NWV, bool EPI>
__global__ void __launch_bounds__(kWave * NWV) col_pass_kernel(ColArgs a) {
    __shared__ ChunkLds<CT, NWV> L;
    const CarryCtx cctx{a.carry, a.epoch, a.status, a.G, a.S, a.NG};
    // Persistent grid: workgroup p always processes chunk p % G, for the strips
    // p / G, p / G + groups, ...; every strip's chunks are thus held by G workgroups of
    // the same launch that are all running, and none ever waits on one not yet started.
    const int chunk = static_cast<int>(blockIdx.x % a.G);
    const int group = static_cast<int>(blockIdx.x / a.G);
    const int n_strips = a.batch * a.NG * a.S;
#pragma unroll 1
    for (int sid = group; sid < n_strips; sid += a.groups) {
    const int strip = sid % a.S;
    const int grp = (sid / a.S) % a.NG;
    const int b = sid / (a.S * a.NG);

    const int lane = opaque_v(lane_id());
    const int wave = opaque_s(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    const int H = a.H, W = a.W;
    const int x = strip * kWave + lane;
    const bool valid = x < W;
    const int r0 = (chunk * NWV + wave) * R;   // first row of this wave
    const int nr = min(R, max(H - r0, 0));
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t pbytes = plane * sizeof(float);
    const int c0 = grp * CT;
    const int ncv = min(CT, a.C - c0);

    // Row r of the wave sits at byte offset voff + r * rowb of a plane; lanes past the
    // right edge and rows past the bottom edge fall outside the plane's buffer range, so
    // their loads read 0 and their stores are dropped.
    const unsigned rowb = static_cast<unsigned>(W) * 4u;
    const unsigned voff = (valid ? static_cast<unsigned>(x) * 4u : kInvalidOffset) +
                          static_cast<unsigned>(min(r0, H)) * rowb;

    // Weights of the wave's rows and of the row after them.  The first row of the image
    // and rows past the bottom edge get weight 0: that is the boundary J[0] = f[0] going
    // down and K[H-1] = J[H-1] going up, and it makes padded rows drop out of both
    // recurrences.
    float w[R];
    const auto drs = plane_rsrc(a.d + static_cast<size_t>(b) * plane, pbytes);
    {
        unsigned vo = voff;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float keep = fminf(fmaxf(static_cast<float>(nr - r), 0.f), 1.f);
            w[r] = weight(bload(drs, vo, 0), a.log2a) * keep;
            vo = opaque_vadd(vo, rowb);
        }
    }
    if (r0 == 0) w[0] = 0.f;
    const float wnext = weight(bload(drs, voff + static_cast<unsigned>(nr) * rowb, 0), a.log2a) *
                        ((r0 + R < H) ? 1.f : 0.f);

    float f[CT][R];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int ch = (c < ncv) ? c0 + c : c0;
        const auto srs = plane_rsrc(a.src + (static_cast<size_t>(b) * a.C + ch) * plane, pbytes);
        unsigned vo = voff;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            f[c][r] = bload(srs, vo, 0);
            vo = opaque_vadd(vo, rowb);
        }
    }

    // phase 1: causal scan of the wave's rows with zero carry-in, plus the anticausal
    // coefficients:  K[first] = BJ + BQ * J_carry + P * K_carry
    float Q = 1.f, pi = 1.f, BQ = 0.f;
    float J[CT], BJ[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) J[c] = BJ[c] = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float wr = w[r];
        const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
        Q *= wr;
        const float coef = fmaf(-pi, wn, pi);   // pi (1 - wn)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            J[c] = fmaf(wr, J[c] - f[c][r], f[c][r]);
            f[c][r] = J[c];
            BJ[c] = fmaf(coef, J[c], BJ[c]);
        }
        BQ = fmaf(coef, Q, BQ);
        pi *= wn;
    }
    L.A[wave][lane] = Q;
    L.P[wave][lane] = pi;
    L.BQ[wave][lane] = BQ;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        L.B[wave][c][lane] = J[c];
        L.BJ[wave][c][lane] = BJ[c];
    }
    __syncthreads();
    if (wave == 0) chunk_carries<CT, NWV>(cctx, L, b, grp, strip, chunk, lane, valid, ncv);
    __syncthreads();

    float Jin[CT], Kin[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        Jin[c] = L.Jin[wave][c][lane];
        Kin[c] = L.Kin[wave][c][lane];
    }

    // phase 3: causal values with the true carry, then the anticausal sweep and the store
    {
        float q = opaque(1.f);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            q *= w[r];
#pragma unroll
            for (int c = 0; c < CT; ++c) f[c][r] = fmaf(q, Jin[c], f[c][r]);
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        if (c < ncv) {
            float K = Kin[c];
            const size_t pidx = static_cast<size_t>(b) * a.C + c0 + c;
            const auto ors = plane_rsrc(a.dst + pidx * plane, pbytes);
            unsigned vo = voff + static_cast<unsigned>(R - 1) * rowb;
            if constexpr (EPI) {
                const int cc = (a.Cc == 1) ? 0 : c0 + c;
                const auto zrs = plane_rsrc(a.zk + pidx * plane, pbytes);
                const auto trs = plane_rsrc(a.tgt + pidx * plane, pbytes);
                const auto crs = plane_rsrc(a.conf + (static_cast<size_t>(b) * a.Cc + cc) * plane, pbytes);
                const auto o2rs = plane_rsrc(a.dst2 ? a.dst2 + pidx * plane : a.dst, a.dst2 ? pbytes : 0);
                // rows in blocks of kEpiBlock, bottom block first: all loads of a block are
                // issued before any of its stores, so a block costs one memory round trip
                constexpr int kEpiBlock = R < 8 ? R : 8;
                static_assert(R % kEpiBlock == 0, "chunk rows must be a multiple of the block");
#pragma unroll
                for (int blk = R / kEpiBlock - 1; blk >= 0; --blk) {
                    float z[kEpiBlock], tt[kEpiBlock], cf[kEpiBlock];
                    unsigned vl = voff + static_cast<unsigned>(blk * kEpiBlock) * rowb;
#pragma unroll
                    for (int q = 0; q < kEpiBlock; ++q) {
                        z[q] = bload(zrs, vl, 0);
                        tt[q] = bload(trs, vl, 0);
                        cf[q] = bload(crs, vl, 0);
                        vl = opaque_vadd(vl, rowb);
                    }
#pragma unroll
                    for (int q = kEpiBlock - 1; q >= 0; --q) {
                        const int r = blk * kEpiBlock + q;
                        const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                        K = fmaf(wn, K - f[c][r], f[c][r]);
                        const float upd = fmaf(a.lambda, z[q] - K, cf[q] * (z[q] - tt[q]));
                        const float zn = fmaf(-a.step, upd, z[q]);
                        bstore(ors, vo, 0, zn);
                        bstore(o2rs, vo, 0, zn);
                        vo = opaque_vadd(vo, 0u - rowb);
                    }
                }
            } else {
#pragma unroll
                for (int r = R - 1; r >= 0; --r) {
                    const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                    K = fmaf(wn, K - f[c][r], f[c][r]);
                    bstore(ors, vo, 0, K);
                    vo = opaque_vadd(vo, 0u - rowb);
                }
            }
        }
    }
    }  // strips of this group
}

// ---------------------------------------------------------------------------------------
// Column-pass variants: rows per wave R and waves per workgroup NWV (a chunk is R * NWV
// rows of one 64-column strip) for each channel-group size CT.  The default choice per
// shape comes from col_variant(); dts_tune_col_variant() can pin another one.
// ---------------------------------------------------------------------------------------
struct ColVariant {
    int ct, R, nwv;
    int (*launch)(const ColArgs&, unsigned, hipStream_t, bool);
    int (*capacity)(bool);
};

template <int CT, int R, int NWV, bool EPI>
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
static int col_capacity_v(bool epi) {
    return epi ? col_capacity_t<CT, R, NWV, true>() : col_capacity_t<CT, R, NWV, false>();
}

template <int CT, int R, int NWV>
static int col_launch_v(const ColArgs& a, unsigned n, hipStream_t s, bool epi) {
    if (epi)
        hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, true>), dim3(n), dim3(kWave * NWV), 0, s, a);
    else
        hipLaunchKernelGGL((col_pass_kernel<CT, R, NWV, false>), dim3(n), dim3(kWave * NWV), 0, s, a);
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
};
constexpr int kNumColVariants = sizeof(kColVariants) / sizeof(kColVariants[0]);
constexpr int kMinChunkRows = 128;   // smallest R * NWV above: sizes the carry area

static int col_group(int C) { return C < 4 ? C : 4; }

static int g_col_pin[5] = {-1, -1, -1, -1, -1};   // per channel-group size, -1 = default

static int col_variant(int C) {
    const int ct = col_group(C);
    const int pin = g_col_pin[ct];
    if (pin >= 0 && pin < kNumColVariants && kColVariants[pin].ct == ct) return pin;
    switch (ct) {
        case 1: return 0;
        case 2: return 5;
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

size_t col_carry_words(int batch, int H, int W, int C) {
    // sized for the smallest chunk of any variant so every variant fits
    const int ct = col_group(C);
    const size_t G = (H + kMinChunkRows - 1) / kMinChunkRows;
    const size_t S = (W + kWave - 1) / kWave;
    const size_t NG = (C + ct - 1) / ct;
    return static_cast<size_t>(batch) * NG * S * G * carry_words_per_chunk(ct) * kWave;
}

int launch_col_pass(const ColPass& p, Ctx& ctx) {
    const ColVariant& v = kColVariants[col_variant(p.C)];
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
    a.zk = p.zk;
    a.tgt = p.tgt;
    a.conf = p.conf;
    a.Cc = p.Cc;
    a.dst2 = p.dst2;
    a.lambda = p.lambda;
    a.step = p.step;
    // every workgroup of the grid must be resident at once: size the grid to the
    // device's capacity for this kernel, in whole strips of G chunks
    const int cap = v.capacity(p.epilogue);
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (a.G > cap) return DTS_ENOTSUP;
    const long long n_strips = static_cast<long long>(p.batch) * a.NG * a.S;
    a.groups = static_cast<int>(std::min<long long>(cap / a.G, n_strips));
    const unsigned n = static_cast<unsigned>(a.groups) * a.G;
    // algorithmic bytes: signal in and out, distances in; the update epilogue also reads
    // z^k, the target and the confidence
    const double px = static_cast<double>(p.batch) * a.H * a.W;
    const double bytes = p.epilogue ? px * 4.0 * (4.0 * a.C + 1.0 + (a.Cc == 1 ? 1.0 : a.C))
                                    : px * 4.0 * (2.0 * a.C + 1.0);
    ProfScope prof(p.epilogue ? "col_pass_update" : "col_pass", bytes, ctx.stream);
    return v.launch(a, n, ctx.stream, p.epilogue);
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
