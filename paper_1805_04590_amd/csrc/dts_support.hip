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
// Column pass: the filter's persistent chunked column pass (dts_chunks.hpp), each chunk of
// a 64-column strip in registers, one column per lane.  A wave's rows reduce to the
// aggregates of both recurrences (y: factor A, value B at the last row from a zero carry;
// v: factor P, value BJ at the first row from a zero carry; the two do not feed each
// other, so BQ = 0), the chunk engine resolves every wave's carry-ins from the
// neighbouring chunks' aggregates, and the wave reruns both recurrences from them and
// writes the scaled sum: every plane is read once.
#include <algorithm>

#include <mutex>

#include "../../include/dts.h"
#include "dts_chunks.hpp"
#include "dts_device.hpp"
#include "dts_internal.hpp"
#include "dts_tiles.hpp"

namespace dts {

constexpr int kSupRows = 24;   // rows per wave of a column chunk
constexpr int kSupWaves = 8;   // waves per workgroup: chunks of 192 rows
constexpr int kSupChunkRows = kSupRows * kSupWaves;

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
// Column pass: dst = m * (y + v - x) along every column, and, when conf is set,
// conf_out = conf / dst.
// ---------------------------------------------------------------------------------------
struct SupColArgs {
    const float* src;   // x; ones when null
    const float* dy;
    float* dst;
    const float* conf;  // optional: conf_out = conf / s
    float* conf_out;
    int Cc;
    int H, W, batch;
    float log2a, m;
    int G, S, groups, xcd;  // chunks per strip, strips per plane, strips in flight, chunk_slot form
    unsigned long long* carry;
    unsigned epoch;
    int* status;
    int spin_limit;
    unsigned tag_xor;
};

template <int R, int NWV>
__global__ void __launch_bounds__(kWave * NWV, 4) support_col_kernel(SupColArgs a) {
    __shared__ ChunkLds<1, NWV> L;
    const CarryCtx cctx{a.carry, a.epoch, a.status, a.G, a.S, 1, a.spin_limit, a.tag_xor};
    // persistent grid, as the filter's column pass: a workgroup always takes the same chunk
    // of the strips group, group + groups, ...
    const ChunkSlot slot = chunk_slot(static_cast<int>(blockIdx.x), a.G, a.xcd);
    const int chunk = slot.chunk;
    const int group = slot.group;
    if (group >= a.groups) return;
    const int lane = opaque_v(lane_id());
    const int wave = opaque_s(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    const int H = a.H, W = a.W;
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t pbytes = plane * sizeof(float);
    const unsigned rowb = static_cast<unsigned>(W) * 4u;
    const int r0 = (chunk * NWV + wave) * R;  // first row of this wave
    const int nr = min(R, max(H - r0, 0));
    const int n_strips = a.batch * a.S;
#pragma unroll 1
    for (int sid = group; sid < n_strips; sid += a.groups) {
        const int strip = sid % a.S;
        const int b = sid / a.S;
        const int x = strip * kWave + lane;
        const bool valid = x < W;
        // rows past the bottom and lanes past the right edge read 0 (buffer range check)
        const unsigned voff = (valid ? static_cast<unsigned>(x) * 4u : kInvalidOffset) +
                              static_cast<unsigned>(min(r0, H)) * rowb;
        const auto drs = plane_rsrc(a.dy + static_cast<size_t>(b) * plane, pbytes);
        float w[R], xv[R];
        {
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float keep = (r < nr) ? 1.f : 0.f;
                w[r] = weight(bload(drs, vo, 0), a.log2a) * keep;
                vo = opaque_vadd(vo, rowb);
            }
        }
        if (r0 == 0) w[0] = 0.f;  // y[0] = x[0]
        // weight linking the wave's last row to the next one (0 past the bottom: v[H-1] = x)
        const float wnext = weight(bload(drs, voff + static_cast<unsigned>(nr) * rowb, 0), a.log2a) *
                            ((r0 + R < H) ? 1.f : 0.f);
        if (a.src) {
            const auto srs = plane_rsrc(a.src + static_cast<size_t>(b) * plane, pbytes);
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xv[r] = bload(srs, vo, 0);
                vo = opaque_vadd(vo, rowb);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) xv[r] = (r < nr) ? 1.f : 0.f;
        }

        // the wave's aggregates from zero carries
        float A = 1.f, yl = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            yl = fmaf(w[r], yl, xv[r]);
            A *= w[r];
        }
        float P = 1.f, vl = 0.f;
#pragma unroll
        for (int r = R - 1; r >= 0; --r) {
            const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
            vl = fmaf(wn, vl, xv[r]);
            P *= wn;
        }
        L.A[wave][lane] = A;
        L.B[wave][0][lane] = yl;
        L.P[wave][lane] = P;
        L.BQ[wave][lane] = 0.f;
        L.BJ[wave][0][lane] = vl;
        __syncthreads();
        chunk_carries<1, NWV>(cctx, L, b, 0, strip, chunk, lane, wave, valid, 1);
        __syncthreads();
        const float yin = L.Jin[wave][0][lane];  // y of the row before the wave's first
        const float vin = L.Kin[wave][0][lane];  // v of the row after the wave's last

        // both recurrences from the true carries; the scaled sum overwrites xv
        float yv[R];
        {
            float y = yin;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                y = fmaf(w[r], y, xv[r]);
                yv[r] = y;
            }
        }
        {
            float v = vin;
#pragma unroll
            for (int r = R - 1; r >= 0; --r) {
                const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                v = fmaf(wn, v, xv[r]);
                xv[r] = a.m * (yv[r] + v - xv[r]);
            }
        }
        const auto ors = plane_rsrc(a.dst + static_cast<size_t>(b) * plane, pbytes);
        {
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bstore(ors, vo, 0, xv[r]);
                vo = opaque_vadd(vo, rowb);
            }
        }
        for (int k = 0; k < a.Cc; ++k) {
            const size_t pl = (static_cast<size_t>(b) * a.Cc + k) * plane;
            const auto crs = plane_rsrc(a.conf + pl, pbytes);
            const auto cors = plane_rsrc(a.conf_out + pl, pbytes);
            float cv[R];
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cv[r] = bload(crs, vo, 0);
                vo = opaque_vadd(vo, rowb);
            }
            vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bstore(cors, vo, 0, cv[r] / xv[r]);
                vo = opaque_vadd(vo, rowb);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
size_t support_carry_words(int batch, int H, int W) {
    const size_t G = (H + kSupChunkRows - 1) / kSupChunkRows;
    const size_t S = (W + kWave - 1) / kWave;
    return static_cast<size_t>(batch) * S * G * carry_words_per_chunk(1) * kWave;
}

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

static int support_col_capacity() {
    static int cached[64] = {0};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, support_col_kernel<kSupRows, kSupWaves>,
                                                         kWave * kSupWaves, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

int launch_support_col(const float* src, const float* dy, float* dst, const float* conf, int Cc, float* conf_out,
                       int batch, int H, int W, float log2a, float m, Ctx& ctx) {
    SupColArgs a;
    a.src = src;
    a.dy = dy;
    a.dst = dst;
    a.conf = conf;
    a.conf_out = conf_out;
    a.Cc = conf ? Cc : 0;
    a.H = H;
    a.W = W;
    a.batch = batch;
    a.log2a = log2a;
    a.m = m;
    a.G = (H + kSupChunkRows - 1) / kSupChunkRows;
    a.S = (W + kWave - 1) / kWave;
    a.carry = ctx.carry;
    a.epoch = ++ctx.epoch;
    a.status = ctx.status;
    a.spin_limit = spin_limit();
    a.tag_xor = spin_tag_xor();
    const int cap = support_col_capacity();
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (a.G > cap) return DTS_ENOTSUP;
    const ColGrid grid = col_grid(cap, a.G, static_cast<long long>(batch) * a.S);
    a.groups = grid.groups;
    a.xcd = grid.xcd;
    // distances and the signal in, the support out; conf in and conf / s out
    const double px = static_cast<double>(batch) * H * W;
    ProfScope prof("support_col", px * 4.0 * (2.0 + (src ? 1.0 : 0.0) + 2.0 * a.Cc), ctx.stream);
    hipLaunchKernelGGL((support_col_kernel<kSupRows, kSupWaves>), dim3(grid.n), dim3(kWave * kSupWaves), 0,
                       ctx.stream, a);
    return hip_fail(hipGetLastError());
}

}  // namespace dts
