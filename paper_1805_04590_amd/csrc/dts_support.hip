// Support of the edge-aware kernel and the support-weighted confidence (Sec. 3.1, the
// comparison with the bilateral solver after Eq. (6)): the confidence of a gradient-descent
// update is divided by sum_j W_ij, the mass of the kernel around pixel i.
//
// W is the unnormalised form of the domain-transform kernel: each 1-D pass sums products
// of the weights a^d over both sides of a pixel, the pixel itself once,
//     S[n] = y[n] + v[n] - x[n],   y[n] = x[n] + w[n] y[n-1],   v[n] = x[n] + w[n+1] v[n+1],
// applied to ones with the filter's alternation of rows and columns over its N
// iterations.  Each pass is scaled by m_i = (1 - a_i) / (1 + a_i), the inverse of a flat
// interior pixel's pass sum, so the result is the support relative to a flat region, in
// (0, 1].  The support depends on the guide alone: it is a one-off pass before a solve.
//
// Row pass: one workgroup per row, lane l of wave v owning S consecutive pixels, both
// directions as 64-lane affine-map scans with a cross-wave exchange through LDS (the
// layout of the filter's row pass).
// Column pass: reduce, carry, apply.  Each chunk of kChunk rows of every column first
// reduces to its two affine aggregates, one thread per column per chunk; one thread per
// column then composes them down and up the column into every chunk's carries; the apply
// kernel reruns both recurrences of the chunk from its carries and writes the scaled sum.
// Every launch is independent of the others' scheduling: no waits, no flags.
#include <algorithm>

#include "../../include/dts.h"
#include "dts_device.hpp"
#include "dts_internal.hpp"
#include "dts_tiles.hpp"

namespace dts {

constexpr int kSupChunk = 32;       // rows per column chunk
constexpr int kSupColThreads = 256;  // columns per workgroup of the column kernels

// ---------------------------------------------------------------------------------------
// Row pass: dst = m * (y + v - x) along every row; x = src, or ones when src is null.
// ---------------------------------------------------------------------------------------
template <int S>
__global__ void __launch_bounds__(1024) support_row_kernel(const float* __restrict__ src,
                                                           const float* __restrict__ dx,
                                                           float* __restrict__ dst, int H, int W,
                                                           float log2a, float m) {
    __shared__ float2 fagg[kMaxRowWaves];
    __shared__ float2 bagg[kMaxRowWaves];
    __shared__ float wfirst[kMaxRowWaves + 1];
    const int y = blockIdx.x, b = blockIdx.y;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const size_t off = (static_cast<size_t>(b) * H + y) * W;
    const int n0 = (wave * kWave + lane) * S;

    float w[S], x[S];
    {
        float dv[S];
        load_seg<S>(dx + off, n0, W, 1.f, dv);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < W) ? weight(dv[e], log2a) : 0.f;
        }
    }
    if (src) {
        load_seg<S>(src + off, n0, W, 0.f, x);
    } else {
#pragma unroll
        for (int e = 0; e < S; ++e) x[e] = (n0 + e < W) ? 1.f : 0.f;
    }
    // weight linking each lane's last pixel to the next one (0 past the end of the row)
    float wlast = __shfl_down(w[0], 1);
    if (lane == 0) wfirst[wave] = w[0];
    if (wave == 0 && lane == 0) wfirst[nw] = 0.f;
    __syncthreads();
    if (lane == kWave - 1) wlast = wfirst[wave + 1];

    // causal: y[n] = w[n] y[n-1] + x[n]
    float la = 1.f, lb = 0.f;
#pragma unroll
    for (int e = 0; e < S; ++e) {
        lb = fmaf(w[e], lb, x[e]);
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
    float yv[S];
    {
        float j = (lane == 0) ? jin : fmaf(xa, jin, xb);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            j = fmaf(w[e], j, x[e]);
            yv[e] = j;
        }
    }

    // anticausal: v[n] = w[n+1] v[n+1] + x[n]
    la = 1.f;
    lb = 0.f;
#pragma unroll
    for (int e = S - 1; e >= 0; --e) {
        const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
        lb = fmaf(wn, lb, x[e]);
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
        k = fmaf(wn, k, x[e]);
        yv[e] = m * (yv[e] + k - x[e]);
    }
    store_seg<S>(dst + off, n0, W, yv);
}

// ---------------------------------------------------------------------------------------
// Column pass.  Chunk g of a column covers rows [s, e], s = g kChunk.  Its aggregates:
//   forward   y[e] = Af y[s-1] + Bf,   Af = prod_{n=s..e} w[n]       (w[0] = 0)
//   backward  v[s] = Ab v[e+1] + Bb,   Ab = prod_{n=s+1..e+1} w[n]   (w[H] = 0)
// with Bf, Bb the chunk's own recurrences from zero carries.
// ---------------------------------------------------------------------------------------
struct SupCol {
    const float* src;   // x; ones when null
    const float* dy;
    float* dst;
    float4* agg;        // [batch][G][W]: Af, Bf, Ab, Bb
    float2* carry;      // [batch][G][W]: y[s-1], v[e+1]
    const float* conf;  // optional: conf_out = conf / s (apply only)
    float* conf_out;
    int Cc;
    int H, W, G;
    float log2a, m;
};

// Loads of one chunk of one column: x[r] and w[r] for rows s + r, and the weight of the
// row after the chunk (0 past the bottom).  Rows past the bottom read x = 0, w = 0.
__device__ __forceinline__ void sup_chunk_load(const SupCol& a, int b, int g, int col, float (&x)[kSupChunk],
                                               float (&w)[kSupChunk], float& wnext) {
    const int s = g * kSupChunk;
    const size_t base = static_cast<size_t>(b) * a.H * a.W + col;
#pragma unroll
    for (int r = 0; r < kSupChunk; ++r) {
        const int n = s + r;
        const bool in = n < a.H;
        const size_t idx = base + static_cast<size_t>(in ? n : 0) * a.W;
        w[r] = (in && n > 0) ? weight(a.dy[idx], a.log2a) : 0.f;
        x[r] = in ? (a.src ? a.src[idx] : 1.f) : 0.f;
    }
    const int n = s + kSupChunk;
    wnext = (n < a.H) ? weight(a.dy[base + static_cast<size_t>(n) * a.W], a.log2a) : 0.f;
}

__global__ void __launch_bounds__(kSupColThreads) support_col_reduce_kernel(SupCol a) {
    const int col = blockIdx.x * kSupColThreads + threadIdx.x;
    const int g = blockIdx.y, b = blockIdx.z;
    if (col >= a.W) return;
    float x[kSupChunk], w[kSupChunk], wnext;
    sup_chunk_load(a, b, g, col, x, w, wnext);
    float Af = 1.f, Bf = 0.f, Ab = 1.f, Bb = 0.f;
#pragma unroll
    for (int r = 0; r < kSupChunk; ++r) {
        Bf = fmaf(w[r], Bf, x[r]);
        Af *= w[r];
    }
#pragma unroll
    for (int r = kSupChunk - 1; r >= 0; --r) {
        const float wn = (r + 1 < kSupChunk) ? w[r + 1 < kSupChunk ? r + 1 : r] : wnext;
        Bb = fmaf(wn, Bb, x[r]);
        Ab *= wn;
    }
    a.agg[(static_cast<size_t>(b) * a.G + g) * a.W + col] = make_float4(Af, Bf, Ab, Bb);
}

// One thread per column: compose the chunk aggregates down the column (forward carries)
// and up the column (backward carries).  Loads are issued kCarryBatch chunks at a time so
// their latencies overlap; the compositions themselves are a short serial chain.
constexpr int kCarryBatch = 16;

__global__ void __launch_bounds__(kSupColThreads) support_col_carry_kernel(SupCol a) {
    const int col = blockIdx.x * kSupColThreads + threadIdx.x;
    const int b = blockIdx.y;
    if (col >= a.W) return;
    const size_t base = static_cast<size_t>(b) * a.G * a.W + col;
    float Cf = 0.f;
    for (int g0 = 0; g0 < a.G; g0 += kCarryBatch) {
        float4 q[kCarryBatch];
#pragma unroll
        for (int i = 0; i < kCarryBatch; ++i)
            if (g0 + i < a.G) q[i] = a.agg[base + static_cast<size_t>(g0 + i) * a.W];
#pragma unroll
        for (int i = 0; i < kCarryBatch; ++i)
            if (g0 + i < a.G) {
                a.carry[base + static_cast<size_t>(g0 + i) * a.W].x = Cf;
                Cf = fmaf(q[i].x, Cf, q[i].y);
            }
    }
    float Cb = 0.f;
    for (int g1 = a.G - 1; g1 >= 0; g1 -= kCarryBatch) {
        float4 q[kCarryBatch];
#pragma unroll
        for (int i = 0; i < kCarryBatch; ++i)
            if (g1 - i >= 0) q[i] = a.agg[base + static_cast<size_t>(g1 - i) * a.W];
#pragma unroll
        for (int i = 0; i < kCarryBatch; ++i)
            if (g1 - i >= 0) {
                a.carry[base + static_cast<size_t>(g1 - i) * a.W].y = Cb;
                Cb = fmaf(q[i].z, Cb, q[i].w);
            }
    }
}

__global__ void __launch_bounds__(kSupColThreads) support_col_apply_kernel(SupCol a) {
    const int col = blockIdx.x * kSupColThreads + threadIdx.x;
    const int g = blockIdx.y, b = blockIdx.z;
    if (col >= a.W) return;
    float x[kSupChunk], w[kSupChunk], wnext;
    sup_chunk_load(a, b, g, col, x, w, wnext);
    const float2 c = a.carry[(static_cast<size_t>(b) * a.G + g) * a.W + col];
    float yv[kSupChunk];
    float y = c.x;
#pragma unroll
    for (int r = 0; r < kSupChunk; ++r) {
        y = fmaf(w[r], y, x[r]);
        yv[r] = y;
    }
    const int s = g * kSupChunk;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const size_t base = static_cast<size_t>(b) * plane + col;
    float v = c.y;
#pragma unroll
    for (int r = kSupChunk - 1; r >= 0; --r) {
        const float wn = (r + 1 < kSupChunk) ? w[r + 1 < kSupChunk ? r + 1 : r] : wnext;
        v = fmaf(wn, v, x[r]);
        const int n = s + r;
        if (n < a.H) {
            const float sv = a.m * (yv[r] + v - x[r]);
            const size_t idx = base + static_cast<size_t>(n) * a.W;
            a.dst[idx] = sv;
            if (a.conf) {
                const float inv = 1.f / sv;
                for (int k = 0; k < a.Cc; ++k) {
                    const size_t ci = (static_cast<size_t>(b) * a.Cc + k) * plane + static_cast<size_t>(n) * a.W + col;
                    a.conf_out[ci] = a.conf[ci] * inv;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
size_t support_chunks(int H) { return static_cast<size_t>((H + kSupChunk - 1) / kSupChunk); }

int launch_support_row(const float* src, const float* dx, float* dst, int batch, int H, int W, float log2a,
                       float m, hipStream_t s) {
    const int S = W > 4096 ? 16 : W > 1024 ? 8 : 4;
    const int nw = (W + kWave * S - 1) / (kWave * S);
    if (nw > kMaxRowWaves) return DTS_ENOTSUP;
    const double px = static_cast<double>(batch) * H * W;
    ProfScope prof("support_row", px * 4.0 * (src ? 3.0 : 2.0), s);
    const dim3 grid(H, batch), block(nw * kWave);
    switch (S) {
        case 4: hipLaunchKernelGGL(support_row_kernel<4>, grid, block, 0, s, src, dx, dst, H, W, log2a, m); break;
        case 8: hipLaunchKernelGGL(support_row_kernel<8>, grid, block, 0, s, src, dx, dst, H, W, log2a, m); break;
        default: hipLaunchKernelGGL(support_row_kernel<16>, grid, block, 0, s, src, dx, dst, H, W, log2a, m); break;
    }
    return hip_fail(hipGetLastError());
}

int launch_support_col(const float* src, const float* dy, float* dst, void* agg, void* carry, const float* conf,
                       int Cc, float* conf_out, int batch, int H, int W, float log2a, float m, hipStream_t s) {
    SupCol a;
    a.src = src;
    a.dy = dy;
    a.dst = dst;
    a.agg = static_cast<float4*>(agg);
    a.carry = static_cast<float2*>(carry);
    a.conf = conf;
    a.conf_out = conf_out;
    a.Cc = conf ? Cc : 0;
    a.H = H;
    a.W = W;
    a.G = static_cast<int>(support_chunks(H));
    a.log2a = log2a;
    a.m = m;
    const double px = static_cast<double>(batch) * H * W;
    const unsigned cb = static_cast<unsigned>((W + kSupColThreads - 1) / kSupColThreads);
    const double xin = src ? 4.0 : 0.0;
    {
        // one plane of distances (and the signal) in, 16 bytes of aggregates per chunk out
        ProfScope prof("support_col_reduce", px * (4.0 + xin) + 16.0 * batch * a.G * static_cast<double>(W), s);
        hipLaunchKernelGGL(support_col_reduce_kernel, dim3(cb, a.G, batch), dim3(kSupColThreads), 0, s, a);
        if (int rc = hip_fail(hipGetLastError())) return rc;
    }
    {
        ProfScope prof("support_col_carry", 24.0 * batch * a.G * static_cast<double>(W), s);
        hipLaunchKernelGGL(support_col_carry_kernel, dim3(cb, batch), dim3(kSupColThreads), 0, s, a);
        if (int rc = hip_fail(hipGetLastError())) return rc;
    }
    ProfScope prof("support_col_apply", px * (8.0 + xin + 8.0 * a.Cc), s);
    hipLaunchKernelGGL(support_col_apply_kernel, dim3(cb, a.G, batch), dim3(kSupColThreads), 0, s, a);
    return hip_fail(hipGetLastError());
}

}  // namespace dts
