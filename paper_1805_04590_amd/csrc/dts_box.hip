// Box form of the edge-aware mean (Sec. 3.2, Eq. (10) as written): the kernel H is the
// indicator of |DT_i - DT_j| <= r on the transformed coordinate of a line, so each 1-D
// pass is the mean of the samples whose coordinate lies within r of the pixel's (a
// normalised box convolution).  The radius r_i = sqrt(3) sigma_Hi is the box with the
// variance of the recursive form's iteration i; passes alternate rows and columns.
//
// Membership is decided on integers, so that it cannot depend on summation order:
//   q = rint(256 d), d = sqrt(1 + s2 sum_k (I_k[n] - I_k[n-1])^2) in float32 with every
//   operation rounded to nearest (no contraction, bands summed in order), the coordinate
//   is the integer running sum of q along the line, R_i = floor(256 r_i), and j is in the
//   box of i iff |ct_i - ct_j| <= R_i.  Codes are capped at 65536, above every accepted
//   radius, which changes no decision (a step larger than R excludes the pair either way).
// Since d >= 1, a box never reaches more than h_i = R_i / 256 pixels from its centre.
//
// Kernels:
//   box_codes_kernel        guide -> qx, qy (four consecutive pixels per thread)
//   box_bounds_row_kernel   qx -> per pixel and iteration, the box as two u8 offsets
//                           (a row segment's prefix of codes in LDS, searches)
//   box_bounds_colwin_kernel  qy -> the column boxes for h_1 <= kWinMaxH (a window's
//                           prefix of codes down 64 columns in LDS, searches)
//   box_transpose_kernel    for wider boxes the column bounds are the row bounds of the
//                           transposed codes, transposed back (64 x 64 LDS tiles)
//   box_rowwin_kernel       one row pass for h <= kWinMaxH: a wave per 512 outputs, the
//                           FP64 prefix S of the segment and its halo in LDS,
//                           mean = (S[hi + 1] - S[lo]) / (hi - lo + 1)
//   box_colwin_kernel<EPI>  one column pass for h <= kWinMaxH: 64 columns x 128 output rows
//                           per workgroup, the window's rows in LDS as float32 prefixes
//                           within 32-row blocks plus FP64 block sums.  EPI: the update of
//                           Eq. (3).
//   box_row_kernel          row pass for wider boxes (h <= 255): FP64 prefix of a
//                           1024-pixel segment and its halo in LDS
//   box_col_kernel<EPI>     column pass with the update for wider boxes: one column per
//                           lane walking down its rows; an LDS ring keeps the float32
//                           prefix within 32-row blocks and the FP64 prefix at block
//                           starts, so a box sum only carries the rounding of its own
//                           additions
//   box_colprefix_kernel,   plain column pass for wider boxes: the block prefix written
//   box_colmean_kernel      out, then a gather of each box's ends and block totals
// The bounds depend on the guide only and are computed once per call; every pass then
// reads its signal and two bytes of bounds per pixel and writes its result.
#include <algorithm>
#include <mutex>

#include "../../include/dts.h"
#include "dts_device.hpp"
#include "dts_internal.hpp"

namespace dts {

constexpr int kBoxSeg = 1024;          // row-pass outputs per workgroup
constexpr int kBoxRowThreads = 256;
constexpr int kBoxRowSpan = 2048;      // segment plus halo: 1024 + 2 * 255 < 2048
constexpr int kBoxRowChunk = kBoxRowSpan / kBoxRowThreads;
constexpr int kBoxLoad = 32;           // rows loaded per step of the column kernels
constexpr int kBoxEmit = 8;            // outputs per block of the column pass
constexpr unsigned kBoxCodeCap = 65536u;
constexpr int kWinMaxH = 64;           // widest half-width of the window passes

// ---------------------------------------------------------------------------------------
// Integer codes of the arc-length increments
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned box_code(float acc, float s2) {
#pragma clang fp contract(off)
    const float d = sqrtf(1.0f + s2 * acc);
    const float q = rintf(d * 256.0f);
    return (q < 65536.0f) ? static_cast<unsigned>(q) : kBoxCodeCap;  // NaN takes the cap
}

// Four consecutive pixels per thread (float4 loads where the row allows them); every
// pixel's arithmetic is the same sequence of rounded operations as for one pixel alone.
constexpr int kCodePx = 4;

__global__ void __launch_bounds__(256) box_codes_kernel(const float* __restrict__ guide, int Cg, int H, int W,
                                                        float s2, unsigned* __restrict__ qx,
                                                        unsigned* __restrict__ qy) {
#pragma clang fp contract(off)
    // Workgroups take (row, segment) units in XCD-contiguous bands: workgroup i runs on
    // XCD i mod 8, and a row's read of the row above then usually hits that XCD's L2.
    const int segs = (W + 256 * kCodePx - 1) / (256 * kCodePx);
    const int unit = xcd_band_index(static_cast<int>(blockIdx.x), segs * H);
    const int y = unit / segs, b = blockIdx.z;
    const int x0 = ((unit - y * segs) * 256 + threadIdx.x) * kCodePx;
    if (x0 >= W) return;
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t i0 = static_cast<size_t>(y) * W + x0;
    const float* g = guide + static_cast<size_t>(b) * Cg * plane + i0;
    const bool whole = x0 + kCodePx <= W;  // the lane's pixels all lie inside the row
    float ax[kCodePx], ay[kCodePx];
#pragma unroll
    for (int e = 0; e < kCodePx; ++e) ax[e] = ay[e] = 0.0f;
    for (int k = 0; k < Cg; ++k) {
        const float* gk = g + static_cast<size_t>(k) * plane;
        float v[kCodePx], u[kCodePx];
        if (whole) {
            const float4_a4 a = *reinterpret_cast<const float4_a4*>(gk);
            v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
            if (y > 0) {
                const float4_a4 c = *reinterpret_cast<const float4_a4*>(gk - W);
                u[0] = c[0]; u[1] = c[1]; u[2] = c[2]; u[3] = c[3];
            }
        } else {
#pragma unroll
            for (int e = 0; e < kCodePx; ++e) {
                v[e] = (x0 + e < W) ? gk[e] : 0.0f;
                if (y > 0) u[e] = (x0 + e < W) ? gk[static_cast<ptrdiff_t>(e) - W] : 0.0f;
            }
        }
        const float left = (x0 > 0) ? gk[-1] : v[0];
#pragma unroll
        for (int e = 0; e < kCodePx; ++e) {
            const float ex = v[e] - (e == 0 ? left : v[e > 0 ? e - 1 : 0]);
            ax[e] = ax[e] + ex * ex;
            if (y > 0) {
                const float ey = v[e] - u[e];
                ay[e] = ay[e] + ey * ey;
            }
        }
    }
    const size_t e0 = static_cast<size_t>(b) * plane + i0;
#pragma unroll
    for (int e = 0; e < kCodePx; ++e) {
        if (x0 + e < W) {
            qx[e0 + e] = (x0 + e > 0) ? box_code(ax[e], s2) : 0u;
            qy[e0 + e] = (y > 0) ? box_code(ay[e], s2) : 0u;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Workgroup scans (256 threads = 4 waves): exclusive prefix of one value per thread
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wtot) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const T u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) wtot[wave] = incl;
    __syncthreads();
    T off = 0;
    for (int u = 0; u < wave; ++u) off += wtot[u];
    __syncthreads();
    return off + incl - v;
}

// Ring slot of the row `rel` rows after the row in slot `slot` (|rel| < RB).
__device__ __forceinline__ int ring_slot(int slot, int rel, int RB) {
    int v = slot + rel;
    v += (v < 0) ? RB : 0;
    v -= (v >= RB) ? RB : 0;
    return v;
}

// Offsets of the boxes of K local indexes li among the prefix coordinates Q[0..n): the
// first j in [li - h, li] with Q[li] - Q[j] <= R and the last j in [li, li + h] with
// Q[j] - Q[li] <= R, packed as (li - first) | (last - li) << 8.  Q is strictly increasing
// (every code >= 1), so both predicates are monotone.  The searches take a fixed number
// of steps, ceil(log2(h + 1)), the same on every lane, so the 2K searches of a step issue
// their LDS reads together instead of as K dependent chains.  A lower search keeps jl
// below the first j that passes (every j <= jl fails), an upper one keeps jh on the last
// j found to pass.
template <int K, typename Get>
__device__ __forceinline__ void box_offsets_k(Get Q, const int (&li)[K], int first, int last, unsigned R, int h,
                                              unsigned (&out)[K]) {
    int steps = 0;
    while ((1 << steps) <= h) ++steps;  // 2^steps >= h + 1, the widest search range
    unsigned qi[K];
    int jl[K], jh[K], top[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        qi[k] = Q(li[k]);
        jl[k] = max(li[k] - h, first) - 1;
        jh[k] = li[k];
        top[k] = min(li[k] + h, last);
    }
    for (int sb = steps - 1; sb >= 0; --sb) {
        const int st = 1 << sb;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // candidates clamped into the search ranges, so the reads are unconditional: a
            // lower candidate clamped to li fails (qi - qi = 0 <= R), and an upper one
            // clamped to top passes only if top is the answer, which later steps keep
            const int cl = min(jl[k] + st, li[k]), ch = min(jh[k] + st, top[k]);
            const unsigned ql = Q(cl), qh = Q(ch);
            if (qi[k] - ql > R) jl[k] = cl;
            if (qh - qi[k] <= R) jh[k] = ch;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        out[k] = static_cast<unsigned>(li[k] - jl[k] - 1) | (static_cast<unsigned>(jh[k] - li[k]) << 8);
}

struct BoxBoundsArgs {
    const unsigned* q;        // codes [batch][H][W]
    unsigned short* bounds;   // [iters][batch][H][W]
    int H, W, iters;
    unsigned cap;             // R_1 + 1
    int h1;                   // R_1 / 256
    unsigned R[kBoxMaxIters];
};

__global__ void __launch_bounds__(kBoxRowThreads) box_bounds_row_kernel(BoxBoundsArgs a) {
    __shared__ unsigned Q[kBoxRowSpan];
    __shared__ unsigned wtot[kBoxRowThreads / kWave];
    const int x0 = blockIdx.x * kBoxSeg, y = blockIdx.y, b = blockIdx.z;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const int s0 = max(x0 - a.h1, 0), s1 = min(x0 + kBoxSeg + a.h1, a.W);
    const int n = s1 - s0;
    const int E = (n + kBoxRowThreads - 1) / kBoxRowThreads;
    const unsigned* row = a.q + b * plane + static_cast<size_t>(y) * a.W + s0;
    unsigned v[kBoxRowChunk], tot = 0;
#pragma unroll
    for (int e = 0; e < kBoxRowChunk; ++e) {
        const int j = threadIdx.x * E + e;
        v[e] = (e < E && j < n && j > 0) ? min(row[j], a.cap) : 0u;
        tot += v[e];
    }
    unsigned run = block_exclusive_scan(tot, wtot);
#pragma unroll
    for (int e = 0; e < kBoxRowChunk; ++e) {
        const int j = threadIdx.x * E + e;
        run += v[e];
        if (e < E && j < n) Q[j] = run;
    }
    __syncthreads();
    auto get = [&](int m) { return Q[m]; };
    // thread t takes pixels x0 + t + 256 j, so that neighbouring lanes search neighbouring
    // LDS words (four consecutive pixels per thread put lanes four words apart: an 8-way
    // bank conflict on every read), and its kPer searches run side by side
    constexpr int kPer = kBoxSeg / kBoxRowThreads;
    int li[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) li[j] = min(x0 + static_cast<int>(threadIdx.x) + kBoxRowThreads * j, a.W - 1) - s0;
    for (int it = 0; it < a.iters; ++it) {
        unsigned bd[kPer];
        box_offsets_k<kPer>(get, li, 0, n - 1, a.R[it], static_cast<int>(a.R[it] >> 8), bd);
        unsigned short* out = a.bounds + (static_cast<size_t>(it) * gridDim.z + b) * plane + static_cast<size_t>(y) * a.W;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int x = x0 + static_cast<int>(threadIdx.x) + kBoxRowThreads * j;
            if (x < a.W) out[x] = static_cast<unsigned short>(bd[j]);
        }
    }
}

// Tiled transpose of `planes` planes [rows][cols] -> [cols][rows] through LDS (64 x 64
// tiles, coalesced on both sides): the column bounds are the row bounds of the
// transposed codes, transposed back.
template <typename T>
__global__ void __launch_bounds__(256) box_transpose_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                            int rows, int cols) {
    __shared__ T tile[64][65];
    const size_t plane = static_cast<size_t>(rows) * cols;
    const T* sp = src + blockIdx.z * plane;
    T* dp = dst + blockIdx.z * plane;
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int k = ty; k < 64; k += 4) {
        const int r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = sp[static_cast<size_t>(r) * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int c = c0 + k, r = r0 + tx;
        if (c < cols && r < rows) dp[static_cast<size_t>(c) * rows + r] = tile[tx][k];
    }
}

// ---------------------------------------------------------------------------------------
// Passes
// ---------------------------------------------------------------------------------------
struct BoxPassArgs {
    const float* src;               // [batch][C][H][W]
    float* dst;
    const unsigned short* bounds;   // [batch][H][W] of this pass's iteration
    int C, H, W, h;
    int seg, ring, nbase;           // column pass: output rows per workgroup, ring rows, base slots
    // update epilogue (column pass): dst = z - step (lambda (z - mean) + c (z - t))
    const float* zk;
    const float* tgt;
    const float* conf;
    int Cc;
    float lambda, step;
};

__global__ void __launch_bounds__(kBoxRowThreads) box_row_kernel(BoxPassArgs a) {
    __shared__ double P[kBoxRowSpan + 1];
    __shared__ double wtot[kBoxRowThreads / kWave];
    const int x0 = blockIdx.x * kBoxSeg, y = blockIdx.y, b = blockIdx.z;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const int s0 = max(x0 - a.h, 0), s1 = min(x0 + kBoxSeg + a.h, a.W);
    const int n = s1 - s0;
    const int E = (n + kBoxRowThreads - 1) / kBoxRowThreads;
    constexpr int kOut = kBoxSeg / kBoxRowThreads;
    unsigned bd[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        const int x = x0 + threadIdx.x + o * kBoxRowThreads;
        bd[o] = (x < a.W) ? a.bounds[b * plane + static_cast<size_t>(y) * a.W + x] : 0u;
    }
    for (int c = 0; c < a.C; ++c) {
        const size_t roff = (static_cast<size_t>(b) * a.C + c) * plane + static_cast<size_t>(y) * a.W;
        const float* row = a.src + roff + s0;
        float v[kBoxRowChunk];
        double tot = 0.0;
#pragma unroll
        for (int e = 0; e < kBoxRowChunk; ++e) {
            const int j = threadIdx.x * E + e;
            v[e] = (e < E && j < n) ? row[j] : 0.0f;
            tot += static_cast<double>(v[e]);
        }
        double run = block_exclusive_scan(tot, wtot);
        if (threadIdx.x == 0) P[0] = 0.0;
#pragma unroll
        for (int e = 0; e < kBoxRowChunk; ++e) {
            const int j = threadIdx.x * E + e;
            run += static_cast<double>(v[e]);
            if (e < E && j < n) P[j + 1] = run;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < kOut; ++o) {
            const int x = x0 + threadIdx.x + o * kBoxRowThreads;
            if (x < a.W) {
                const int li = x - s0;
                const int lo = li - static_cast<int>(bd[o] & 255u), hi = li + static_cast<int>(bd[o] >> 8);
                a.dst[roff + x] = static_cast<float>(P[hi + 1] - P[lo]) *
                                  __builtin_amdgcn_rcpf(static_cast<float>(hi - lo + 1));
            }
        }
        __syncthreads();  // P is rebuilt for the next channel
    }
}

// Row pass for half-widths h <= kWinMaxH (the same limit as the window column pass): one
// wave per kRowWinSeg outputs of a row, many waves in flight per CU.  The wave loads its
// window (the segment and h pixels on either side) with coalesced loads and stages it in
// LDS; each lane takes the FP64 prefix of kRowWinPer consecutive samples, a wave scan adds
// the lane totals before it, and the window's exclusive FP64 prefix S (S[0] = 0) goes back
// to LDS over the staged samples.  mean = (S[hi + 1] - S[lo]) / (hi - lo + 1), the numbers
// of box_row_kernel up to FP64 rounding.
constexpr int kRowWinSeg = 512;
constexpr int kRowWinSpan = kRowWinSeg + 2 * kWinMaxH;  // segment plus the widest halo
constexpr int kRowWinPer = kRowWinSpan / kWave;    // samples per lane (loads per lane)
constexpr int kRowWinOut = kRowWinSeg / kWave;     // outputs per lane
static_assert(kRowWinSpan % kWave == 0 && kRowWinSeg % kWave == 0, "row window shape");

__global__ void __launch_bounds__(kWave) box_rowwin_kernel(BoxPassArgs a, int segs) {
    __shared__ double S[kRowWinSpan + 1];
    float* stage = reinterpret_cast<float*>(S);  // the window's samples, before S is written
    const int lane = threadIdx.x;
    // units (row, segment) of one image in XCD-contiguous bands: a halo is then mostly
    // the neighbouring segment's pixels, read on the same XCD
    const int unit = xcd_band_index(static_cast<int>(blockIdx.x), segs * a.H);
    const int y = unit / segs, sg = unit - y * segs;
    const int b = blockIdx.z;
    const int x0 = sg * kRowWinSeg;
    const int s0 = max(x0 - a.h, 0);
    const int n = min(x0 + kRowWinSeg + a.h, a.W) - s0;  // window pixels
    const int oEnd = min(x0 + kRowWinSeg, a.W);
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const size_t yoff = static_cast<size_t>(y) * a.W;
    const unsigned short* brow = a.bounds + static_cast<size_t>(b) * plane + yoff;
    unsigned bd[kRowWinOut];
#pragma unroll
    for (int m = 0; m < kRowWinOut; ++m) {
        const int x = x0 + lane + kWave * m;
        bd[m] = (x < oEnd) ? brow[x] : 0u;
    }
    float v[kRowWinPer];
    auto load = [&](int c) {
        const float* row = a.src + (static_cast<size_t>(b) * a.C + c) * plane + yoff + s0;
#pragma unroll
        for (int m = 0; m < kRowWinPer; ++m) {
            const int e = lane + kWave * m;
            v[m] = (e < n) ? row[e] : 0.0f;
        }
    };
    load(0);
    for (int c = 0; c < a.C; ++c) {
#pragma unroll
        for (int m = 0; m < kRowWinPer; ++m) stage[lane + kWave * m] = v[m];
        __syncthreads();
        float w[kRowWinPer];
#pragma unroll
        for (int u = 0; u < kRowWinPer; ++u) w[u] = stage[lane * kRowWinPer + u];
        __syncthreads();  // S is written over the staged samples
        if (c + 1 < a.C) load(c + 1);
        double run = 0.0;
#pragma unroll
        for (int u = 0; u < kRowWinPer; ++u) run += static_cast<double>(w[u]);
        double incl = run;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const double t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        double base = __shfl_up(incl, 1);
        if (lane == 0) base = 0.0;
#pragma unroll
        for (int u = 0; u < kRowWinPer; ++u) {
            base += static_cast<double>(w[u]);
            S[lane * kRowWinPer + u + 1] = base;
        }
        if (lane == 0) S[0] = 0.0;
        __syncthreads();
        float* drow = a.dst + (static_cast<size_t>(b) * a.C + c) * plane + yoff;
#pragma unroll
        for (int m = 0; m < kRowWinOut; ++m) {
            const int x = x0 + lane + kWave * m;
            if (x < oEnd) {
                // a box never leaves the row or reaches beyond h, so it lies in the window;
                // the clamps only keep the LDS reads inside it
                const int li = x - s0;
                const int lo = max(li - static_cast<int>(bd[m] & 255u), 0);
                const int hi = min(li + static_cast<int>(bd[m] >> 8), n - 1);
                drow[x] = static_cast<float>(S[hi + 1] - S[lo]) *
                          __builtin_amdgcn_rcpf(static_cast<float>(hi - lo + 1));
            }
        }
        __syncthreads();  // the next channel's samples are staged over S
    }
}

template <int EPI>
__global__ void __launch_bounds__(kWave) box_col_kernel(BoxPassArgs a) {
    extern __shared__ unsigned char box_smem[];
    const int RB = a.ring;
    const int bmask = a.nbase - 1;  // base slots: a power of two
    float* ring = reinterpret_cast<float*>(box_smem);                                      // [RB][64]
    double* base = reinterpret_cast<double*>(box_smem + static_cast<size_t>(RB) * kWave * 4);  // [nbase][64]
    const int lane = threadIdx.x;
    const int col = blockIdx.x * kWave + lane;
    const bool valid = col < a.W;
    const int y0 = blockIdx.y * a.seg;
    const int bc = blockIdx.z;  // image * C + channel
    const int b = bc / a.C, c = bc - b * a.C;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const int h = a.h;
    const int sIn = max(y0 - h, 0);
    const int rEnd = min(y0 + a.seg + h, a.H) - 1;
    const int oEnd = min(y0 + a.seg, a.H) - 1;
    const int cx = valid ? col : 0;
    const float* sc = a.src + static_cast<size_t>(bc) * plane + cx;
    float* dc = a.dst + static_cast<size_t>(bc) * plane + cx;
    const unsigned short* bdc = a.bounds + static_cast<size_t>(b) * plane + cx;
    [[maybe_unused]] const float* zc = EPI ? a.zk + static_cast<size_t>(bc) * plane + cx : nullptr;
    [[maybe_unused]] const float* tc = EPI ? a.tgt + static_cast<size_t>(bc) * plane + cx : nullptr;
    [[maybe_unused]] const float* cc =
        EPI ? a.conf + (static_cast<size_t>(b) * a.Cc + (a.Cc == 1 ? 0 : c)) * plane + cx : nullptr;

    float run = 0.0f;
    double bsum = 0.0;
    int wslot = 0;                        // slot of the next row written
    int nextb = y0, oslot = y0 - sIn;     // next output block and the slot of its first row

    // mean of the box of output row o (slot so), from the ring
    auto box_mean = [&](int o, int so, unsigned bd) -> float {
        const int lo_off = static_cast<int>(bd & 255u), hi_off = static_cast<int>(bd >> 8);
        const int ol = o - sIn;
        const int lh = ol + hi_off, ll = ol - lo_off - 1;
        const double ph = base[((lh >> 5) & bmask) * kWave + lane] +
                          static_cast<double>(ring[ring_slot(so, hi_off, RB) * kWave + lane]);
        const double pl = (ll < 0) ? 0.0
                                   : base[((ll >> 5) & bmask) * kWave + lane] +
                                         static_cast<double>(ring[ring_slot(so, -lo_off - 1, RB) * kWave + lane]);
        return static_cast<float>(ph - pl) * __builtin_amdgcn_rcpf(static_cast<float>(lo_off + hi_off + 1));
    };
    auto put = [&](int o, float mean, float z, float t, float cf) {
        const size_t po = static_cast<size_t>(o) * a.W;
        if constexpr (EPI) {
            const float upd = fmaf(a.lambda, z - mean, cf * (z - t));
            dc[po] = fmaf(-a.step, upd, z);
        } else {
            dc[po] = mean;
        }
    };
    auto ready = [&](int loaded) {
        return nextb <= oEnd && (min(nextb + kBoxEmit - 1, oEnd) + h <= loaded || loaded == a.H - 1);
    };

    float fv[kBoxLoad];
#pragma unroll
    for (int u = 0; u < kBoxLoad; ++u) {
        const int r = sIn + u;
        fv[u] = (valid && r <= rEnd) ? sc[static_cast<size_t>(r) * a.W] : 0.0f;
    }
    for (int r0 = sIn; r0 <= rEnd; r0 += kBoxLoad) {
        // Operands of the output rows this group can complete, issued before the prefetch
        // of the next group: loads return in order, so waiting for them does not wait for
        // the prefetch.
        unsigned bdp[kBoxLoad];
        [[maybe_unused]] float zp[kBoxLoad], tp[kBoxLoad], cp[kBoxLoad];
#pragma unroll
        for (int k = 0; k < kBoxLoad; ++k) {
            const int o = nextb + k;
            const bool in = valid && o <= oEnd;
            const size_t po = static_cast<size_t>(in ? o : 0) * a.W;
            bdp[k] = in ? bdc[po] : 0u;
            if constexpr (EPI) {
                zp[k] = in ? zc[po] : 0.0f;
                tp[k] = in ? tc[po] : 0.0f;
                cp[k] = in ? cc[po] : 0.0f;
            }
        }
        float fn[kBoxLoad];
#pragma unroll
        for (int u = 0; u < kBoxLoad; ++u) {
            const int r = r0 + kBoxLoad + u;
            fn[u] = (valid && r <= rEnd) ? sc[static_cast<size_t>(r) * a.W] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kBoxLoad; ++u) {
            const int l = r0 + u - sIn;
            if (r0 + u <= rEnd) {
                if ((l & 31) == 0) {
                    bsum += static_cast<double>(run);
                    run = 0.0f;
                    base[((l >> 5) & bmask) * kWave + lane] = bsum;
                }
                run += fv[u];
                ring[wslot * kWave + lane] = run;
                wslot = (wslot + 1 == RB) ? 0 : wslot + 1;
            }
        }
        const int loaded = min(r0 + kBoxLoad - 1, rEnd);
        // blocks are emitted in order once every box of them is loaded; the first
        // kBoxLoad / kBoxEmit of them use the operands loaded above
        bool go = true;
#pragma unroll
        for (int j = 0; j < kBoxLoad / kBoxEmit; ++j) {
            go = go && ready(loaded);
            if (go) {
#pragma unroll
                for (int q = 0; q < kBoxEmit; ++q) {
                    const int o = nextb + q;
                    if (o <= oEnd) {
                        const float m = box_mean(o, ring_slot(oslot, q, RB), bdp[j * kBoxEmit + q]);
                        if (valid) {
                            if constexpr (EPI) put(o, m, zp[j * kBoxEmit + q], tp[j * kBoxEmit + q], cp[j * kBoxEmit + q]);
                            else put(o, m, 0.f, 0.f, 0.f);
                        }
                    }
                }
                nextb += kBoxEmit;
                oslot = ring_slot(oslot, kBoxEmit, RB);
            }
        }
        // at the bottom of the image the last group completes every remaining block
        while (ready(loaded)) {
#pragma unroll
            for (int q = 0; q < kBoxEmit; ++q) {
                const int o = nextb + q;
                if (o <= oEnd) {
                    const size_t po = static_cast<size_t>(o) * a.W;
                    const unsigned bd = valid ? bdc[po] : 0u;
                    const float m = box_mean(o, ring_slot(oslot, q, RB), bd);
                    if (valid) {
                        if constexpr (EPI) put(o, m, zc[po], tc[po], cc[po]);
                        else put(o, m, 0.f, 0.f, 0.f);
                    }
                }
            }
            nextb += kBoxEmit;
            oslot = ring_slot(oslot, kBoxEmit, RB);
        }
#pragma unroll
        for (int u = 0; u < kBoxLoad; ++u) fv[u] = fn[u];
    }
}

// Plain column pass in two streaming kernels.
//   box_colprefix_kernel: P[y] = sum of f over rows 32 (y / 32) .. y of the column (the
//     prefix within aligned 32-row blocks, float32), one thread per column and block;
//   box_colmean_kernel: the box sum of row o is P[hi] - P[lo - 1] plus the totals
//     P[32 k + 31] of the blocks k from (lo - 1) / 32 to hi / 32 - 1, added in FP64: a sum
//     carries only the float32 rounding of its own additions, as in box_col_kernel.
// Both kernels run at full occupancy; the gathers of the second stay within a few rows
// of the output row and are served by the caches.
constexpr int kBoxPrefixRows = 32;

__global__ void __launch_bounds__(256) box_colprefix_kernel(const float* __restrict__ src, float* __restrict__ P,
                                                            int H, int W) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= W) return;
    const size_t plane = static_cast<size_t>(H) * W;
    const int y0 = blockIdx.y * kBoxPrefixRows;
    const int n = min(kBoxPrefixRows, H - y0);
    const float* sc = src + blockIdx.z * plane + static_cast<size_t>(y0) * W + x;
    float* pc = P + blockIdx.z * plane + static_cast<size_t>(y0) * W + x;
    float v[kBoxPrefixRows];
#pragma unroll
    for (int r = 0; r < kBoxPrefixRows; ++r) v[r] = (r < n) ? sc[static_cast<size_t>(r) * W] : 0.0f;
    float run = 0.0f;
#pragma unroll
    for (int r = 0; r < kBoxPrefixRows; ++r) {
        run += v[r];
        if (r < n) pc[static_cast<size_t>(r) * W] = run;
    }
}

constexpr int kBoxMeanRows = 8;  // output rows per thread

__global__ void __launch_bounds__(256) box_colmean_kernel(const float* __restrict__ P,
                                                          const unsigned short* __restrict__ bounds,
                                                          float* __restrict__ dst, int C, int H, int W) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= W) return;
    const size_t plane = static_cast<size_t>(H) * W;
    const int bc = blockIdx.z, b = bc / C;
    const int o0 = blockIdx.y * kBoxMeanRows;
    const float* pc = P + static_cast<size_t>(bc) * plane + x;
    const unsigned short* bdc = bounds + static_cast<size_t>(b) * plane + x;
    float* dc = dst + static_cast<size_t>(bc) * plane + x;
    unsigned bd[kBoxMeanRows];
#pragma unroll
    for (int q = 0; q < kBoxMeanRows; ++q) {
        const int o = o0 + q;
        bd[q] = (o < H) ? bdc[static_cast<size_t>(o) * W] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kBoxMeanRows; ++q) {
        const int o = o0 + q;
        if (o < H) {
            const int lo = o - static_cast<int>(bd[q] & 255u), hi = o + static_cast<int>(bd[q] >> 8);
            double sum = static_cast<double>(pc[static_cast<size_t>(hi) * W]);
            int k = 0;
            if (lo > 0) {
                sum -= static_cast<double>(pc[static_cast<size_t>(lo - 1) * W]);
                k = (lo - 1) >> 5;
            }
            for (; k < (hi >> 5); ++k)
                sum += static_cast<double>(pc[static_cast<size_t>(32 * k + 31) * W]);
            dc[static_cast<size_t>(o) * W] =
                static_cast<float>(sum) * __builtin_amdgcn_rcpf(static_cast<float>(hi - lo + 1));
        }
    }
}

// ---------------------------------------------------------------------------------------
// Column pass in one kernel for half-widths h <= kWinMaxH: a workgroup owns 64 columns
// (one per lane) and kWinRows output rows.  It loads its window, the output rows and h
// rows on either side, as float32 prefixes within 32-row blocks (block k holds window
// rows 32k .. 32k + 31), sums the block totals before each block in FP64, and reads a box
// sum off the window as S(hi) - S(lo - 1) with S(j) = (FP64 total of the blocks before
// j's) + (float32 prefix of j within its block): the rounding is that of the ring kernel.
// Every output pixel costs one signal read and two bytes of bounds from HBM; the halo
// rows are the neighbouring tiles' rows, and the tile order (a run of consecutive tiles
// down a column strip per XCD) keeps both readers of a halo on one L2.  The operands of
// the output rows are loaded up front and stay in flight across the two barriers, which
// wait for LDS only.
// ---------------------------------------------------------------------------------------
constexpr int kWinRows = 128;
constexpr int kWinWaves = 8;
constexpr int kWinSpan = kWinRows + 2 * kWinMaxH;    // window rows
constexpr int kWinBlocks = kWinSpan / 32;
constexpr int kWinBlocksPerWave = (kWinBlocks + kWinWaves - 1) / kWinWaves;
constexpr int kWinOutPerWave = kWinRows / kWinWaves;
static_assert(kWinSpan % 32 == 0 && kWinRows % kWinWaves == 0, "window shape");

struct BoxWinArgs {
    BoxPassArgs p;
    int tiles_x, tiles_y;   // 64-column strips, kWinRows-row tiles per strip
    int tiles;              // tiles_x * tiles_y * batch * C
    int per_xcd;            // workgroups per XCD (the grid is 8 per_xcd)
};

// Geometry of tile T: strip-major, tiles down a strip consecutive.
struct WinTile {
    int bc, b, c;          // image * C + channel, image, channel
    int cx;                // the lane's column (0 for lanes beyond the image)
    int valid;             // the lane's column lies in the image (0 or 1)
    int y0, s0, n, nb;     // first output row, first window row, window rows, 32-row blocks
    int oEnd;              // one past the last output row
};

__device__ __forceinline__ WinTile win_tile(const BoxWinArgs& w, int T, int lane) {
    const BoxPassArgs& a = w.p;
    WinTile t;
    const int ty = T % w.tiles_y;
    const int rest = T / w.tiles_y;
    const int tx = rest % w.tiles_x;
    t.bc = rest / w.tiles_x;
    t.b = t.bc / a.C;
    t.c = t.bc - t.b * a.C;
    const int col = tx * kWave + lane;
    t.valid = col < a.W;
    t.cx = t.valid ? col : 0;
    t.y0 = ty * kWinRows;
    t.s0 = max(t.y0 - a.h, 0);
    t.n = min(t.y0 + kWinRows + a.h, a.H) - t.s0;
    t.nb = (t.n + 31) >> 5;
    t.oEnd = min(t.y0 + kWinRows, a.H);
    return t;
}

// Operands of one tile through raw buffer resources over its planes: a lane's column is a
// per-lane byte offset (kInvalidOffset beyond the image), a row a uniform (scalar) offset,
// and rows outside the window or the tile read 0 through an invalid lane offset.
struct WinRes {
    __amdgpu_buffer_rsrc_t sig, bnd, dst;
    unsigned lv4, lv2;  // the lane's byte offset in a float plane and in the bounds plane
};

__device__ __forceinline__ WinRes win_res(const BoxPassArgs& a, const WinTile& t) {
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    WinRes r;
    r.sig = plane_rsrc(a.src + static_cast<size_t>(t.bc) * plane, plane * 4);
    r.dst = plane_rsrc(a.dst + static_cast<size_t>(t.bc) * plane, plane * 4);
    r.bnd = plane_rsrc(a.bounds + static_cast<size_t>(t.b) * plane, plane * 2);
    r.lv4 = t.valid ? static_cast<unsigned>(t.cx) * 4u : kInvalidOffset;
    r.lv2 = t.valid ? static_cast<unsigned>(t.cx) * 2u : kInvalidOffset;
    return r;
}

// The wave's 32-row blocks of the window (block k = wave + kWinWaves i).
__device__ __forceinline__ void win_load_signal(const BoxPassArgs& a, const WinTile& t, const WinRes& rs, int wave,
                                                float (&v)[kWinBlocksPerWave][32]) {
    const unsigned pitch = static_cast<unsigned>(a.W) * 4u;
#pragma unroll
    for (int i = 0; i < kWinBlocksPerWave; ++i) {
        const int k = wave + kWinWaves * i;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int r = 32 * k + u;
            const unsigned row = static_cast<unsigned>(t.s0 + min(r, t.n - 1)) * pitch;
            v[i][u] = bload(rs.sig, (r < t.n) ? rs.lv4 : kInvalidOffset, row);
        }
    }
}

// Bounds of the wave's output rows (row y0 + wave + kWinWaves q).
__device__ __forceinline__ void win_load_bounds(const BoxPassArgs& a, const WinTile& t, const WinRes& rs, int wave,
                                                unsigned (&bd)[kWinOutPerWave]) {
    const unsigned pitch = static_cast<unsigned>(a.W) * 2u;
#pragma unroll
    for (int q = 0; q < kWinOutPerWave; ++q) {
        const int o = t.y0 + wave + kWinWaves * q;
        const unsigned row = static_cast<unsigned>(min(o, t.oEnd - 1)) * pitch;
        bd[q] = __builtin_amdgcn_raw_buffer_load_b16(rs.bnd, (o < t.oEnd) ? rs.lv2 : kInvalidOffset, row, 0);
    }
}

// Persistent over tiles: XCD x owns a contiguous band of tiles and its per_xcd workgroups
// take every per_xcd-th of them, so the tiles in flight on one XCD are neighbours down a
// strip.  While a tile's block sums and outputs are computed, the next tile's window and
// bounds are already in flight (registers; the barriers wait for LDS only).
template <int EPI>
__global__ void __launch_bounds__(kWinWaves* kWave) box_colwin_kernel(BoxWinArgs w) {
    __shared__ float pf[kWinSpan * kWave];      // [row][lane]
    __shared__ float btot[kWinBlocks * kWave];  // block totals (float32 prefix at the block's end)
    __shared__ double bpre[kWinBlocks * kWave]; // FP64 sum of the totals of the blocks before
    const BoxPassArgs& a = w.p;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int x = static_cast<int>(blockIdx.x % kXcds), j = static_cast<int>(blockIdx.x / kXcds);
    const int q8 = w.tiles / kXcds, r8 = w.tiles % kXcds;
    const int t_end = x * q8 + min(x, r8) + q8 + (x < r8 ? 1 : 0);
    int T = x * q8 + min(x, r8) + j;
    if (T >= t_end) return;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const unsigned pitch = static_cast<unsigned>(a.W) * 4u;

    WinTile t = win_tile(w, T, lane);
    WinRes rs = win_res(a, t);
    float v[kWinBlocksPerWave][32];
    unsigned bd[kWinOutPerWave];
    win_load_signal(a, t, rs, wave, v);
    win_load_bounds(a, t, rs, wave, bd);
    for (;;) {
        [[maybe_unused]] float zv[kWinOutPerWave], tv[kWinOutPerWave], cv[kWinOutPerWave];
        if constexpr (EPI) {
            const auto zr = plane_rsrc(a.zk + static_cast<size_t>(t.bc) * plane, plane * 4);
            const auto tr = plane_rsrc(a.tgt + static_cast<size_t>(t.bc) * plane, plane * 4);
            const auto cr = plane_rsrc(a.conf + (static_cast<size_t>(t.b) * a.Cc + (a.Cc == 1 ? 0 : t.c)) * plane,
                                       plane * 4);
#pragma unroll
            for (int q = 0; q < kWinOutPerWave; ++q) {
                const int o = t.y0 + wave + kWinWaves * q;
                const unsigned row = static_cast<unsigned>(min(o, t.oEnd - 1)) * pitch;
                const unsigned lv = (o < t.oEnd) ? rs.lv4 : kInvalidOffset;
                zv[q] = bload(zr, lv, row);
                tv[q] = bload(tr, lv, row);
                cv[q] = bload(cr, lv, row);
            }
        }
        // float32 prefixes within the wave's blocks
#pragma unroll
        for (int i = 0; i < kWinBlocksPerWave; ++i) {
            const int k = wave + kWinWaves * i;
            if (k < t.nb) {
                float run = 0.0f;
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    run += v[i][u];
                    pf[(32 * k + u) * kWave + lane] = run;
                }
                btot[k * kWave + lane] = run;
            }
        }
        // the next tile's operands, in flight during this tile's block sums and outputs
        // (the update's operands leave no registers for them: that kernel takes one tile
        // per workgroup)
        const int Tn = T + w.per_xcd;
        const bool more = !EPI && Tn < t_end;
        WinTile tn = t;
        WinRes rn = rs;
        [[maybe_unused]] unsigned bdn[kWinOutPerWave];
        if constexpr (EPI == 0) {
            if (more) {
                tn = win_tile(w, Tn, lane);
                rn = win_res(a, tn);
                win_load_signal(a, tn, rn, wave, v);
                win_load_bounds(a, tn, rn, wave, bdn);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kWinBlocksPerWave; ++i) {
            const int k = wave + kWinWaves * i;
            if (k < t.nb) {
                double acc = 0.0;
                for (int jb = 0; jb < k; ++jb) acc += static_cast<double>(btot[jb * kWave + lane]);
                bpre[k * kWave + lane] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kWinOutPerWave; ++q) {
            const int o = t.y0 + wave + kWinWaves * q;
            if (o < t.oEnd) {
                const int lo_off = static_cast<int>(bd[q] & 255u), hi_off = static_cast<int>(bd[q] >> 8);
                // a box never leaves the image or reaches beyond h, so it lies in the
                // window; the clamps only keep the LDS reads inside it
                const int jh = min(o - t.s0 + hi_off, t.n - 1);
                const int jl = max(o - t.s0 - lo_off - 1, -1);
                const double ph = bpre[(jh >> 5) * kWave + lane] + static_cast<double>(pf[jh * kWave + lane]);
                const double pl =
                    (jl < 0) ? 0.0 : bpre[(jl >> 5) * kWave + lane] + static_cast<double>(pf[jl * kWave + lane]);
                const float mean =
                    static_cast<float>(ph - pl) * __builtin_amdgcn_rcpf(static_cast<float>(lo_off + hi_off + 1));
                float res = mean;
                if constexpr (EPI) res = fmaf(-a.step, fmaf(a.lambda, zv[q] - mean, cv[q] * (zv[q] - tv[q])), zv[q]);
                bstore(rs.dst, rs.lv4, static_cast<unsigned>(o) * pitch, res);
            }
        }
        if (!more) break;
        __syncthreads();  // the LDS window is rebuilt for the next tile
        T = Tn;
        t = tn;
        rs = rn;
        if constexpr (EPI == 0) {
            for (int q = 0; q < kWinOutPerWave; ++q) bd[q] = bdn[q];  // a register rename
        }
    }
}

// ---------------------------------------------------------------------------------------
// Column bounds for h_1 <= kWinMaxH without transposes: a workgroup owns 64 columns (one
// per lane) and kWinRows output rows, builds the integer coordinate prefix of its window
// (the output rows and h_1 rows on either side) in LDS from the column codes, and places
// every box by the search of box_bounds_row_kernel along its lane's column: a binary
// search for a wave's first output row, and for the following rows ends that only move
// forward.  Integer sums, so the boxes are those of the transposed row kernel exactly.
// ---------------------------------------------------------------------------------------
constexpr int kBndRowsPerWave = kWinRows / kWinWaves;  // consecutive output rows of a wave

__global__ void __launch_bounds__(kWinWaves* kWave) box_bounds_colwin_kernel(BoxBoundsArgs a, int batch,
                                                                             int tiles_x, int tiles_y, int tiles) {
    __shared__ unsigned P[kWinSpan * kWave];      // [row][lane]: coordinate relative to the window start
    __shared__ unsigned btot[kWinBlocks * kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int T = xcd_band_index(static_cast<int>(blockIdx.x), tiles);
    const int ty = T % tiles_y, rest = T / tiles_y;
    const int tx = rest % tiles_x, b = rest / tiles_x;
    const int col = tx * kWave + lane;
    const bool valid = col < a.W;
    const int cx = valid ? col : 0;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const int y0 = ty * kWinRows;
    const int s0 = max(y0 - a.h1, 0);
    const int n = min(y0 + kWinRows + a.h1, a.H) - s0;
    const int nb = (n + 31) >> 5;
    const int oEnd = min(y0 + kWinRows, a.H);
    const unsigned* qc = a.q + static_cast<size_t>(b) * plane + cx;

    // codes of the wave's block (the window's first row contributes none), capped at
    // R_1 + 1 as in the row kernel, and their prefix within the block
    unsigned loc[32];
    const int k = wave;
    static_assert(kWinBlocksPerWave == 1, "one block per wave");
    if (k < nb) {
        unsigned run = 0;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int r = 32 * k + u;
            const unsigned c = (valid && r > 0 && r < n) ? min(qc[static_cast<size_t>(s0 + r) * a.W], a.cap) : 0u;
            run += c;
            loc[u] = run;
        }
        btot[k * kWave + lane] = run;
    }
    __syncthreads();
    if (k < nb) {
        unsigned base = 0;
        for (int jb = 0; jb < k; ++jb) base += btot[jb * kWave + lane];
#pragma unroll
        for (int u = 0; u < 32; ++u) P[(32 * k + u) * kWave + lane] = base + loc[u];
    }
    __syncthreads();

    auto get = [&](int m) { return P[m * kWave + lane]; };
    // the wave's output rows, kBndGroup at a time with their searches side by side
    constexpr int kBndGroup = 8;
    static_assert(kBndRowsPerWave % kBndGroup == 0, "whole groups");
    for (int g0 = 0; g0 < kBndRowsPerWave; g0 += kBndGroup) {
        const int o0 = y0 + wave * kBndRowsPerWave + g0;
        if (o0 >= oEnd) break;
        int li[kBndGroup];
#pragma unroll
        for (int j = 0; j < kBndGroup; ++j) li[j] = min(o0 + j, oEnd - 1) - s0;
        for (int it = 0; it < a.iters; ++it) {
            unsigned bd[kBndGroup];
            box_offsets_k<kBndGroup>(get, li, 0, n - 1, a.R[it], static_cast<int>(a.R[it] >> 8), bd);
            unsigned short* out = a.bounds + (static_cast<size_t>(it) * batch + b) * plane + col;
#pragma unroll
            for (int j = 0; j < kBndGroup; ++j)
                if (valid && o0 + j < oEnd) out[static_cast<size_t>(o0 + j) * a.W] = static_cast<unsigned short>(bd[j]);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
static int max_lds_per_block() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return 65536;
        cached = v;
    }
    return cached;
}

// Ring rows of a column kernel with half-width h: the rows a box can reach on both sides
// of the oldest output still pending, the pending block and one loaded group.
static int box_ring_rows(int h) { return (2 * h + kBoxLoad + kBoxEmit + 1 + 7) / 8 * 8; }
// Slots of 32-row block bases: a power of two covering every block the ring spans.
static int box_base_slots(int h) {
    int n = 1;
    while (n < box_ring_rows(h) / 32 + 2) n <<= 1;
    return n;
}
static size_t box_col_lds(int h) {
    return static_cast<size_t>(box_ring_rows(h)) * kWave * 4 + static_cast<size_t>(box_base_slots(h)) * kWave * 8;
}

// Output rows per column workgroup: enough workgroups to fill the chip, whole groups.
static int box_col_seg(int batch_planes, int H, int W) {
    const long strips = static_cast<long>((W + kWave - 1) / kWave) * batch_planes;
    int seg = 1024;
    while (seg > 32 && strips * ((H + seg - 1) / seg) < 2048) seg >>= 1;
    return seg;
}

int box_check_radius(int h1) {
    if (h1 > 255) return DTS_ENOTSUP;  // offsets are stored in one byte
    if (box_col_lds(h1) > static_cast<size_t>(max_lds_per_block())) return DTS_ENOTSUP;
    return DTS_OK;
}

int launch_box_codes(const float* guide, int Cg, int batch, int H, int W, float s2, unsigned* qx, unsigned* qy,
                     hipStream_t s) {
    const double total = static_cast<double>(batch) * H * W;
    ProfScope prof("box_codes", total * 4.0 * (Cg + 2), s);
    const unsigned units = static_cast<unsigned>((W + 256 * kCodePx - 1) / (256 * kCodePx)) * static_cast<unsigned>(H);
    hipLaunchKernelGGL(box_codes_kernel, dim3(units, 1, batch), dim3(256), 0, s, guide, Cg, H, W, s2, qx, qy);
    return hip_fail(hipGetLastError());
}

template <typename T>
static int launch_transpose(const T* src, T* dst, int planes, int rows, int cols, const char* name, hipStream_t s) {
    ProfScope prof(name, 2.0 * sizeof(T) * planes * static_cast<double>(rows) * cols, s);
    hipLaunchKernelGGL(box_transpose_kernel<T>, dim3((cols + 63) / 64, (rows + 63) / 64, planes), dim3(256), 0, s,
                       src, dst, rows, cols);
    return hip_fail(hipGetLastError());
}

static int launch_bounds_rows(const unsigned* q, unsigned short* bounds, int batch, int H, int W,
                              const BoxBoundsArgs& base, const char* name, hipStream_t s) {
    BoxBoundsArgs a = base;
    a.q = q;
    a.bounds = bounds;
    a.H = H;
    a.W = W;
    ProfScope prof(name, static_cast<double>(batch) * H * W * (4.0 + 2.0 * a.iters), s);
    hipLaunchKernelGGL(box_bounds_row_kernel, dim3((W + kBoxSeg - 1) / kBoxSeg, H, batch), dim3(kBoxRowThreads), 0, s,
                       a);
    return hip_fail(hipGetLastError());
}

// Row bounds from qx.  Column bounds straight from qy when h_1 fits the window kernel,
// else as the row bounds of the transposed qy (written over qx, no longer needed),
// transposed back through `bt` (iters planes of the batch).
int launch_box_bounds(unsigned* qx, const unsigned* qy, unsigned short* bx, unsigned short* by, unsigned short* bt,
                      int batch, int H, int W, const unsigned* R, int iters, hipStream_t s) {
    BoxBoundsArgs a{};
    a.iters = iters;
    a.cap = R[0] + 1;
    a.h1 = static_cast<int>(R[0] >> 8);
    for (int i = 0; i < iters; ++i) a.R[i] = R[i];
    if (int rc = box_check_radius(a.h1)) return rc;
    int rc = launch_bounds_rows(qx, bx, batch, H, W, a, "box_bounds_row", s);
    if (rc) return rc;
    if (box_window_fits(a.h1)) {
        BoxBoundsArgs c = a;
        c.q = qy;
        c.bounds = by;
        c.H = H;
        c.W = W;
        const int tiles_x = (W + kWave - 1) / kWave, tiles_y = (H + kWinRows - 1) / kWinRows;
        const long long tiles = static_cast<long long>(tiles_x) * tiles_y * batch;
        if (tiles > 0x7fffffffLL) return DTS_ENOTSUP;
        ProfScope prof("box_bounds_col_window", static_cast<double>(batch) * H * W * (4.0 + 2.0 * iters), s);
        hipLaunchKernelGGL(box_bounds_colwin_kernel, dim3(static_cast<unsigned>(tiles)), dim3(kWinWaves * kWave), 0,
                           s, c, batch, tiles_x, tiles_y, static_cast<int>(tiles));
        return hip_fail(hipGetLastError());
    }
    if ((rc = launch_transpose<unsigned>(qy, qx, batch, H, W, "box_transpose_codes", s))) return rc;
    if ((rc = launch_bounds_rows(qx, bt, batch, W, H, a, "box_bounds_col", s))) return rc;
    return launch_transpose<unsigned short>(bt, by, iters * batch, W, H, "box_transpose_bounds", s);
}

int launch_box_row(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W, int h,
                   hipStream_t s) {
    BoxPassArgs a{};
    a.src = src;
    a.dst = dst;
    a.bounds = bounds;
    a.C = C;
    a.H = H;
    a.W = W;
    a.h = h;
    const double px = static_cast<double>(batch) * H * W;
    if (box_window_fits(h)) {
        const int segs = (W + kRowWinSeg - 1) / kRowWinSeg;
        if (static_cast<long long>(segs) * H > 0x7fffffffLL) return DTS_ENOTSUP;
        ProfScope prof("box_row_window", px * (8.0 * C + 2.0), s);
        hipLaunchKernelGGL(box_rowwin_kernel, dim3(static_cast<unsigned>(segs * H), 1, batch), dim3(kWave), 0, s, a,
                           segs);
        return hip_fail(hipGetLastError());
    }
    ProfScope prof("box_row", px * (8.0 * C + 2.0), s);
    hipLaunchKernelGGL(box_row_kernel, dim3((W + kBoxSeg - 1) / kBoxSeg, H, batch), dim3(kBoxRowThreads), 0, s, a);
    return hip_fail(hipGetLastError());
}

int launch_box_col_prefixed(const float* src, float* P, float* dst, const unsigned short* bounds, int C, int batch,
                            int H, int W, hipStream_t s) {
    const double px = static_cast<double>(batch) * H * W;
    const unsigned gx = static_cast<unsigned>((W + 255) / 256);
    {
        ProfScope prof("box_col_prefix", px * 8.0 * C, s);
        hipLaunchKernelGGL(box_colprefix_kernel, dim3(gx, (H + kBoxPrefixRows - 1) / kBoxPrefixRows, batch * C),
                           dim3(256), 0, s, src, P, H, W);
        if (int rc = hip_fail(hipGetLastError())) return rc;
    }
    // prefix in once, bounds in, mean out (the gathers beyond the first read are cache hits)
    ProfScope prof("box_col_mean", px * 10.0 * C, s);
    hipLaunchKernelGGL(box_colmean_kernel, dim3(gx, (H + kBoxMeanRows - 1) / kBoxMeanRows, batch * C), dim3(256), 0,
                       s, P, bounds, dst, C, H, W);
    return hip_fail(hipGetLastError());
}

// Co-resident workgroups of the window column kernel on the current device (0 if unknown).
template <int EPI>
static int box_win_slots() {
    static std::mutex mu;
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, box_colwin_kernel<EPI>, kWinWaves * kWave, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = std::max(1, per_cu * cus);
    }
    return cached[dev];
}

static bool g_box_window = true;

int tune_box_window(int on) {
    g_box_window = on != 0;
    return DTS_OK;
}

bool box_window_fits(int h) { return g_box_window && h >= 0 && h <= kWinMaxH; }

int launch_box_col_window(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W,
                          int h, const float* zk, const float* tgt, const float* conf, int Cc, float lambda,
                          float step, hipStream_t s) {
    if (h < 0 || h > kWinMaxH) return DTS_EINVAL;
    BoxWinArgs w{};
    BoxPassArgs& a = w.p;
    a.src = src;
    a.dst = dst;
    a.bounds = bounds;
    a.C = C;
    a.H = H;
    a.W = W;
    a.h = h;
    a.zk = zk;
    a.tgt = tgt;
    a.conf = conf;
    a.Cc = Cc;
    a.lambda = lambda;
    a.step = step;
    w.tiles_x = (W + kWave - 1) / kWave;
    w.tiles_y = (H + kWinRows - 1) / kWinRows;
    const unsigned long long tiles =
        static_cast<unsigned long long>(w.tiles_x) * static_cast<unsigned long long>(w.tiles_y) * batch * C;
    if (tiles == 0) return DTS_OK;
    if (tiles > 0x7fffffffull) return DTS_ENOTSUP;
    w.tiles = static_cast<int>(tiles);
    // the plain pass runs persistent (as many workgroups as fit, each taking a run of tiles
    // with the next one prefetched); the pass with the update takes one tile per workgroup
    w.per_xcd = (w.tiles + kXcds - 1) / kXcds;
    if (!zk) w.per_xcd = std::max(1, std::min(w.per_xcd, box_win_slots<0>() / kXcds));
    const dim3 grid(static_cast<unsigned>(kXcds * w.per_xcd));
    const double px = static_cast<double>(batch) * H * W;
    if (zk) {
        ProfScope prof("box_col_window_update", px * (18.0 * C + 4.0 * Cc), s);
        hipLaunchKernelGGL(box_colwin_kernel<1>, grid, dim3(kWinWaves * kWave), 0, s, w);
    } else {
        ProfScope prof("box_col_window", px * 10.0 * C, s);
        hipLaunchKernelGGL(box_colwin_kernel<0>, grid, dim3(kWinWaves * kWave), 0, s, w);
    }
    return hip_fail(hipGetLastError());
}

int launch_box_col(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W, int h,
                   const float* zk, const float* tgt, const float* conf, int Cc, float lambda, float step,
                   hipStream_t s) {
    if (int rc = box_check_radius(h)) return rc;
    BoxPassArgs a{};
    a.src = src;
    a.dst = dst;
    a.bounds = bounds;
    a.C = C;
    a.H = H;
    a.W = W;
    a.h = h;
    a.seg = box_col_seg(batch * C, H, W);
    a.ring = box_ring_rows(h);
    a.nbase = box_base_slots(h);
    a.zk = zk;
    a.tgt = tgt;
    a.conf = conf;
    a.Cc = Cc;
    a.lambda = lambda;
    a.step = step;
    const size_t lds = box_col_lds(h);
    const dim3 grid((W + kWave - 1) / kWave, (H + a.seg - 1) / a.seg, batch * C);
    const double px = static_cast<double>(batch) * H * W;
    if (zk) {
        // per channel: signal, bounds, z^k and t in, z^{k+1} out; the confidence planes in
        ProfScope prof("box_col_update", px * (18.0 * C + 4.0 * Cc), s);
        hipLaunchKernelGGL(box_col_kernel<1>, grid, dim3(kWave), lds, s, a);
    } else {
        ProfScope prof("box_col", px * 10.0 * C, s);
        hipLaunchKernelGGL(box_col_kernel<0>, grid, dim3(kWave), lds, s, a);
    }
    return hip_fail(hipGetLastError());
}

}  // namespace dts
