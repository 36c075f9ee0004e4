// Adjoint kernels: reverse-mode derivative of the domain-transform solve on gfx950.
//
// Not in the paper (Bapat & Frahm, ECCV 2018, whose solver is Eq. (3) gradient descent
// with the recursive domain-transform filter of Sec. 3.2); derived here by the chain rule.
// For one causal+anticausal pass on a line,
//   J[n] = w[n] J[n-1] + (1 - w[n]) f[n],      K[n] = w[n+1] K[n+1] + (1 - w[n+1]) J[n],
// and an output gradient g = dL/dK, the adjoint runs two more recurrences with the same
// weights,
//   rho[n]   = w[n] rho[n-1] + g[n]                        (forward in n)
//   sigma[n] = w[n+1] sigma[n+1] + (1 - w[n+1]) rho[n]      (backward in n)
// and gives dL/df[n] = (1 - w[n]) sigma[n] and
//   dL/dw[n] = sigma[n] (J[n-1] - f[n]) + rho[n-1] (K[n] - J[n-1]),
// then dL/dd = dL/dw * w * ln a.  rho has the form of J with input g (no 1 - w factor) and
// sigma the form of K, so each adjoint pass scans the pairs (J, rho) forward and
// (K, sigma) backward with shared factors, exactly like the forward passes.
#include <algorithm>
#include <mutex>

#include "../../include/dts.h"
#include "dts_chunks.hpp"
#include "dts_device.hpp"
#include "dts_internal.hpp"

namespace dts {

// ---------------------------------------------------------------------------------------
// Row adjoint: one workgroup per row, S pixels per lane (as the forward row pass)
// ---------------------------------------------------------------------------------------
struct RowAdjArgs {
    const float* gk;  // dL/dK [batch][C][H][W]
    float gk_scale;
    const float* f;   // pass input [batch][C][H][W]
    const float* d;   // dx [batch][H][W]
    float* gout;      // dL/df [batch][C][H][W] (unused with the update epilogue)
    float* gd;        // dL/d(dx) accumulator [batch][H][W], or null
    int C, H, W;
    float log2a, ln_a;
    // update epilogue (first pass of a solver iteration):
    //   gz <- (1 - step lam - step c) gz + dL/df,  gt += step c gz_old (+ new gz at k = 0),
    //   gc += step (t - z^k) gz_old  (summed over channels when Cc = 1)
    float* gz;
    const float* tgt;
    const float* conf;
    float* gt;
    float* gc;
    int Cc;
    float lambda, step;
    int last;
};

constexpr int kMaxRowWavesAdj = 16;

template <int S, bool EPI>
__global__ void __launch_bounds__(1024) row_adjoint_kernel(RowAdjArgs a) {
    __shared__ float fag[kMaxRowWavesAdj][3];
    __shared__ float bag[kMaxRowWavesAdj][3];
    __shared__ float wfirst[kMaxRowWavesAdj + 1];

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int y = blockIdx.x;
    const int b = blockIdx.y;
    const int H = a.H, W = a.W;
    const size_t plane = static_cast<size_t>(H) * W;
    const int n0 = (wave * kWave + lane) * S;
    const size_t prow = static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;

    float w[S];
    {
        float dv[S];
        load_seg<S>(a.d + prow, n0, W, 0.f, dv);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < W) ? weight(dv[e], a.log2a) : 0.f;
        }
    }
    if (lane == 0) wfirst[wave] = w[0];
    if (threadIdx.x == 0) wfirst[nw] = 0.f;
    __syncthreads();
    float wlast = __shfl_down(w[0], 1);
    if (lane == kWave - 1) wlast = wfirst[wave + 1];

    float gdacc[S];
#pragma unroll
    for (int e = 0; e < S; ++e) gdacc[e] = 0.f;

    for (int c = 0; c < a.C; ++c) {
        const size_t roff = (static_cast<size_t>(b) * a.C + c) * plane + static_cast<size_t>(y) * W;
        float f[S], g[S];
        load_seg<S>(a.f + roff, n0, W, 0.f, f);
        load_seg<S>(a.gk + roff, n0, W, 0.f, g);
#pragma unroll
        for (int e = 0; e < S; ++e) g[e] *= a.gk_scale;

        // forward pair: J (from f) and rho (from g), shared factor w
        float la = 1.f, lb[2] = {0.f, 0.f};
#pragma unroll
        for (int e = 0; e < S; ++e) {
            lb[0] = fmaf(w[e], lb[0] - f[e], f[e]);
            lb[1] = fmaf(w[e], lb[1], g[e]);
            la *= w[e];
        }
        scan_up_dpp_n<2>(la, lb, lane);
        if (lane == kWave - 1) {
            fag[wave][0] = la;
            fag[wave][1] = lb[0];
            fag[wave][2] = lb[1];
        }
        const float xa = __shfl_up(la, 1), xj = __shfl_up(lb[0], 1), xr = __shfl_up(lb[1], 1);
        __syncthreads();
        float jin = 0.f, rin = 0.f;
        for (int u = 0; u < wave; ++u) {
            jin = fmaf(fag[u][0], jin, fag[u][1]);
            rin = fmaf(fag[u][0], rin, fag[u][2]);
        }
        // values just before the lane's first pixel
        const float jprev = (lane == 0) ? jin : fmaf(xa, jin, xj);
        const float rprev = (lane == 0) ? rin : fmaf(xa, rin, xr);
        float J[S], rho[S];
        {
            float jj = jprev, rr = rprev;
#pragma unroll
            for (int e = 0; e < S; ++e) {
                jj = fmaf(w[e], jj - f[e], f[e]);
                rr = fmaf(w[e], rr, g[e]);
                J[e] = jj;
                rho[e] = rr;
            }
        }

        // backward pair: K (from J) and sigma (from rho), shared factor w[n+1]
        la = 1.f;
        lb[0] = lb[1] = 0.f;
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            lb[0] = fmaf(wn, lb[0] - J[e], J[e]);
            lb[1] = fmaf(wn, lb[1] - rho[e], rho[e]);
            la *= wn;
        }
        scan_down_dpp_n<2>(la, lb, lane);
        if (lane == 0) {
            bag[wave][0] = la;
            bag[wave][1] = lb[0];
            bag[wave][2] = lb[1];
        }
        const float ya = __shfl_down(la, 1), yk = __shfl_down(lb[0], 1), ys = __shfl_down(lb[1], 1);
        __syncthreads();
        float kin = 0.f, sin_ = 0.f;
        for (int u = nw - 1; u > wave; --u) {
            kin = fmaf(bag[u][0], kin, bag[u][1]);
            sin_ = fmaf(bag[u][0], sin_, bag[u][2]);
        }
        float kk = (lane == kWave - 1) ? kin : fmaf(ya, kin, yk);
        float ss = (lane == kWave - 1) ? sin_ : fmaf(ya, sin_, ys);
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            kk = fmaf(wn, kk - J[e], J[e]);
            ss = fmaf(wn, ss - rho[e], rho[e]);
            const float jm = (e == 0) ? jprev : J[e > 0 ? e - 1 : 0];
            const float rm = (e == 0) ? rprev : rho[e > 0 ? e - 1 : 0];
            const float gw = fmaf(ss, jm - f[e], rm * (kk - jm));
            gdacc[e] = fmaf(gw * w[e], a.ln_a, gdacc[e]);
            f[e] = fmaf(-w[e], ss, ss);  // f now holds dL/df = (1 - w) sigma
        }
        if constexpr (EPI) {
            // update adjoint in groups of 4 pixels; z^k of this iteration is the pass input
            const int cc = (a.Cc == 1) ? 0 : c;
            const size_t coff = (static_cast<size_t>(b) * a.Cc + cc) * plane + static_cast<size_t>(y) * W;
            float zk[S];
            load_seg<S>(a.f + roff, n0, W, 0.f, zk);
#pragma unroll
            for (int e0 = 0; e0 < S; e0 += 4) {
                float gzo[4], tt[4], cf[4], gto[4] = {0.f, 0.f, 0.f, 0.f}, gco[4] = {0.f, 0.f, 0.f, 0.f};
                load_seg<4>(a.gz + roff, n0 + e0, W, 0.f, gzo);
                load_seg<4>(a.tgt + roff, n0 + e0, W, 0.f, tt);
                load_seg<4>(a.conf + coff, n0 + e0, W, 0.f, cf);
                if (a.gt) load_seg<4>(a.gt + roff, n0 + e0, W, 0.f, gto);
                if (a.gc) load_seg<4>(a.gc + coff, n0 + e0, W, 0.f, gco);
                float gzn[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float sc = a.step * cf[q];
                    gzn[q] = fmaf(1.f - a.step * a.lambda - sc, gzo[q], f[e0 + q]);
                    gto[q] = fmaf(sc, gzo[q], gto[q]);
                    if (a.last) gto[q] += gzn[q];
                    gco[q] = fmaf(a.step * (tt[q] - zk[e0 + q]), gzo[q], gco[q]);
                }
                store_seg<4>(a.gz + roff, n0 + e0, W, gzn);
                if (a.gt) store_seg<4>(a.gt + roff, n0 + e0, W, gto);
                if (a.gc) store_seg<4>(a.gc + coff, n0 + e0, W, gco);
            }
        } else {
            store_seg<S>(a.gout + roff, n0, W, f);
        }
        __syncthreads();  // fag / bag reused by the next channel
    }
    if (a.gd) {
        float cur[S];
        load_seg<S>(a.gd + prow, n0, W, 0.f, cur);
#pragma unroll
        for (int e = 0; e < S; ++e) cur[e] += gdacc[e];
        store_seg<S>(a.gd + prow, n0, W, cur);
    }
}

static int row_adj_segment(int W) { return W > 8192 ? 16 : W > 1024 ? 8 : 4; }

template <int S, bool EPI>
static void launch_row_adj_t(const RowAdjArgs& a, int nw, int batch, hipStream_t s, double bytes) {
    ProfScope prof(EPI ? "row_adjoint_update" : "row_adjoint", bytes, s);
    hipLaunchKernelGGL((row_adjoint_kernel<S, EPI>), dim3(a.H, batch), dim3(nw * kWave), 0, s, a);
}

int launch_row_adjoint(const RowAdj& p, Ctx& ctx) {
    RowAdjArgs a;
    a.gk = p.gk;
    a.gk_scale = p.gk_scale;
    a.f = p.f;
    a.d = p.d;
    a.gout = p.gout;
    a.gd = p.gd;
    a.C = p.C;
    a.H = p.H;
    a.W = p.W;
    a.log2a = p.log2a;
    a.ln_a = p.log2a * 0.69314718055994530942f;
    a.gz = p.gz;
    a.tgt = p.tgt;
    a.conf = p.conf;
    a.gt = p.gt;
    a.gc = p.gc;
    a.Cc = p.Cc;
    a.lambda = p.lambda;
    a.step = p.step;
    a.last = p.last;
    const int S = row_adj_segment(p.W);
    const int nw = (p.W + kWave * S - 1) / (kWave * S);
    if (nw > kMaxRowWavesAdj) return DTS_ENOTSUP;
    const bool epi = p.gz != nullptr;
    // algorithmic bytes: g, f in and dL/df out (C planes), dx in, dL/d(dx) read+write;
    // the update epilogue reads gz, t, c, dL/dt, dL/dc and writes gz, dL/dt, dL/dc instead
    const double px = static_cast<double>(p.batch) * p.H * p.W;
    double planes = 3.0 * p.C + 1.0 + (p.gd ? 2.0 : 0.0);
    if (epi) planes += 4.0 * p.C + 2.0 * (p.Cc == 1 ? 1.0 : p.C) + (p.gc ? 1.0 : 0.0) * (p.Cc == 1 ? 1.0 : p.C);
    const double bytes = px * 4.0 * planes;
    const hipStream_t s = ctx.stream;
    switch (S) {
        case 4: epi ? launch_row_adj_t<4, true>(a, nw, p.batch, s, bytes) : launch_row_adj_t<4, false>(a, nw, p.batch, s, bytes); break;
        case 8: epi ? launch_row_adj_t<8, true>(a, nw, p.batch, s, bytes) : launch_row_adj_t<8, false>(a, nw, p.batch, s, bytes); break;
        default: epi ? launch_row_adj_t<16, true>(a, nw, p.batch, s, bytes) : launch_row_adj_t<16, false>(a, nw, p.batch, s, bytes); break;
    }
    return hip_fail(hipGetLastError());
}

// ---------------------------------------------------------------------------------------
// Column adjoint: persistent chunked column pass with 2 carry channels per target channel
// (channel 2c: J / K of target channel c, channel 2c+1: rho / sigma)
// ---------------------------------------------------------------------------------------
struct ColAdjArgs {
    const float* gk;
    float gk_scale;
    const float* f;
    const float* d;   // dy [batch][H][W]
    float* gout;
    float* gd;        // dL/d(dy) accumulator, one plane set per channel group, or null
    int C, H, W, batch;
    float log2a, ln_a;
    int G, S, NG, groups, xcd;
    unsigned long long* carry;
    unsigned epoch;
    int* status;
    int spin_limit;
    unsigned tag_xor;
};

template <int CTA, int R, int NWV>
__global__ void __launch_bounds__(kWave * NWV) col_adjoint_kernel(ColAdjArgs a) {
    constexpr int NCH = 2 * CTA;
    __shared__ ChunkLds<NCH, NWV> L;
    const CarryCtx cctx{a.carry, a.epoch, a.status, a.G, a.S, a.NG, a.spin_limit, a.tag_xor};
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
        const int lane = opaque_v(lane_id());
        const int wave = opaque_s(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
        const int H = a.H, W = a.W;
        const int x = strip * kWave + lane;
        const bool valid = x < W;
        const int r0 = (chunk * NWV + wave) * R;
        const int nr = min(R, max(H - r0, 0));
        const size_t plane = static_cast<size_t>(H) * W;
        const size_t pbytes = plane * sizeof(float);
        const int c0 = grp * CTA;
        const int ncv = min(CTA, a.C - c0);
        const unsigned rowb = static_cast<unsigned>(W) * 4u;
        const unsigned voff = (valid ? static_cast<unsigned>(x) * 4u : kInvalidOffset) +
                              static_cast<unsigned>(min(r0, H)) * rowb;

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
        const float wnext =
            weight(bload(drs, voff + static_cast<unsigned>(nr) * rowb, 0), a.log2a) *
            ((r0 + R < H) ? 1.f : 0.f);

        float f[CTA][R], X[NCH][R];
#pragma unroll
        for (int c = 0; c < CTA; ++c) {
            const int ch = (c < ncv) ? c0 + c : c0;
            const size_t pidx = static_cast<size_t>(b) * a.C + ch;
            const auto frs = plane_rsrc(a.f + pidx * plane, pbytes);
            const auto grs = plane_rsrc(a.gk + pidx * plane, pbytes);
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                f[c][r] = bload(frs, vo, 0);
                X[2 * c + 1][r] = bload(grs, vo, 0) * a.gk_scale;
                vo = opaque_vadd(vo, rowb);
            }
        }

        // phase 1: forward scans with zero carry-in and the backward coefficients
        float Q = 1.f, pi = 1.f, BQ = 0.f;
        float Xl[NCH], BJ[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) Xl[c] = BJ[c] = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float wr = w[r];
            const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
            Q *= wr;
            const float coef = fmaf(-pi, wn, pi);
#pragma unroll
            for (int c = 0; c < CTA; ++c) {
                Xl[2 * c] = fmaf(wr, Xl[2 * c] - f[c][r], f[c][r]);
                Xl[2 * c + 1] = fmaf(wr, Xl[2 * c + 1], X[2 * c + 1][r]);
                X[2 * c][r] = Xl[2 * c];
                X[2 * c + 1][r] = Xl[2 * c + 1];
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) BJ[c] = fmaf(coef, Xl[c], BJ[c]);
            BQ = fmaf(coef, Q, BQ);
            pi *= wn;
        }
        L.A[wave][lane] = Q;
        L.P[wave][lane] = pi;
        L.BQ[wave][lane] = BQ;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            L.B[wave][c][lane] = Xl[c];
            L.BJ[wave][c][lane] = BJ[c];
        }
        // The distance-gradient accumulator is read here so that its loads are in flight
        // during the carry exchange; it is updated and written back at the end.
        float gacc[R];
        const auto gdrs = plane_rsrc(a.gd ? a.gd + (static_cast<size_t>(grp) * a.batch + b) * plane : a.d,
                                     a.gd ? pbytes : 0);
        {
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                gacc[r] = bload(gdrs, vo, 0);
                vo = opaque_vadd(vo, rowb);
            }
        }
        __syncthreads();
        chunk_carries<NCH, NWV>(cctx, L, b, grp, strip, chunk, lane, wave, valid, 2 * ncv);
        __syncthreads();

        float Xin[NCH], Yin[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            Xin[c] = L.Jin[wave][c][lane];
            Yin[c] = L.Kin[wave][c][lane];
        }
        {
            float q = opaque(1.f);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                q *= w[r];
#pragma unroll
                for (int c = 0; c < NCH; ++c) X[c][r] = fmaf(q, Xin[c], X[c][r]);
            }
        }
        // backward sweep: K and sigma, then dL/df and dL/dw per row
#pragma unroll
        for (int c = 0; c < CTA; ++c) {
            if (c < ncv) {
                float kk = Yin[2 * c], ss = Yin[2 * c + 1];
                const size_t pidx = static_cast<size_t>(b) * a.C + c0 + c;
                const auto ors = plane_rsrc(a.gout + pidx * plane, pbytes);
                unsigned vo = voff + static_cast<unsigned>(R - 1) * rowb;
#pragma unroll
                for (int r = R - 1; r >= 0; --r) {
                    const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                    const float jr = X[2 * c][r], rr = X[2 * c + 1][r];
                    kk = fmaf(wn, kk - jr, jr);
                    ss = fmaf(wn, ss - rr, rr);
                    bstore(ors, vo, 0, fmaf(-w[r], ss, ss));
                    const float jm = (r == 0) ? Xin[2 * c] : X[2 * c][r > 0 ? r - 1 : 0];
                    const float rm = (r == 0) ? Xin[2 * c + 1] : X[2 * c + 1][r > 0 ? r - 1 : 0];
                    const float gw = fmaf(ss, jm - f[c][r], rm * (kk - jm));
                    gacc[r] = fmaf(gw * w[r], a.ln_a, gacc[r]);
                    vo = opaque_vadd(vo, 0u - rowb);
                }
            }
        }
        if (a.gd) {
            unsigned vo = voff;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bstore(gdrs, vo, 0, gacc[r]);
                vo = opaque_vadd(vo, rowb);
            }
        }
    }
}

template <int CTA, int R, int NWV>
static int col_adj_capacity() {
    static int cached[64] = {0};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, col_adjoint_kernel<CTA, R, NWV>,
                                                         kWave * NWV, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

// target channels per group, rows per wave, waves per workgroup.  One channel per
// group: a group of two needs 185 VGPRs, i.e. one 8-wave workgroup per CU, against 124
// and two per CU for one channel; the extra distance and gradient reads of the smaller
// groups cost less than the lost occupancy (8 x 1024^2, 3 channels, T = 15: forward +
// backward 20.61 ms with groups of two, 19.95 ms with groups of one).
constexpr int kAdjGroupChannels = 1;
constexpr int kAdjRowsPerWave = 16;
constexpr int kAdjWaves = 8;
constexpr int kAdjChunkRows = kAdjRowsPerWave * kAdjWaves;

int col_adjoint_groups(int C) { return (C + kAdjGroupChannels - 1) / kAdjGroupChannels; }

size_t col_adjoint_carry_words(int batch, int H, int W, int C) {
    const int cta = kAdjGroupChannels;
    const size_t G = (H + kAdjChunkRows - 1) / kAdjChunkRows;
    const size_t S = (W + kWave - 1) / kWave;
    const size_t NG = (C + cta - 1) / cta;
    return static_cast<size_t>(batch) * NG * S * G * carry_words_per_chunk(2 * cta) * kWave;
}

template <int CTA>
static int launch_col_adj_t(ColAdjArgs a, hipStream_t s, double bytes) {
    const int cap = col_adj_capacity<CTA, kAdjRowsPerWave, kAdjWaves>();
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (a.G > cap) return DTS_ENOTSUP;
    const ColGrid grid = col_grid(cap, a.G, static_cast<long long>(a.batch) * a.NG * a.S);
    a.groups = grid.groups;
    a.xcd = grid.xcd;
    const unsigned n = grid.n;
    ProfScope prof("col_adjoint", bytes, s);
    hipLaunchKernelGGL((col_adjoint_kernel<CTA, kAdjRowsPerWave, kAdjWaves>), dim3(n),
                       dim3(kWave * kAdjWaves), 0, s, a);
    return hip_fail(hipGetLastError());
}

int launch_col_adjoint(const ColAdj& p, Ctx& ctx) {
    ColAdjArgs a;
    a.gk = p.gk;
    a.gk_scale = p.gk_scale;
    a.f = p.f;
    a.d = p.d;
    a.gout = p.gout;
    a.gd = p.gd;
    a.C = p.C;
    a.H = p.H;
    a.W = p.W;
    a.batch = p.batch;
    a.log2a = p.log2a;
    a.ln_a = p.log2a * 0.69314718055994530942f;
    const int cta = kAdjGroupChannels;
    a.G = (p.H + kAdjChunkRows - 1) / kAdjChunkRows;
    a.S = (p.W + kWave - 1) / kWave;
    a.NG = (p.C + cta - 1) / cta;
    a.carry = ctx.carry;
    a.epoch = ++ctx.epoch;
    a.status = ctx.status;
    a.spin_limit = spin_limit();
    a.tag_xor = spin_tag_xor();
    const double px = static_cast<double>(p.batch) * p.H * p.W;
    const double bytes = px * 4.0 * (3.0 * p.C + 1.0 + (p.gd ? 2.0 : 0.0));
    return launch_col_adj_t<kAdjGroupChannels>(a, ctx.stream, bytes);
}

// ---------------------------------------------------------------------------------------
// Distance adjoint: dL/dguide from dL/d(dx) and dL/d(dy)
//   d = sqrt(1 + s2 sum_k D_k^2)  =>  dd/dD_k = s2 D_k / d,  D_k = I_k[p] - I_k[p - 1]
// ---------------------------------------------------------------------------------------
struct DistAdjArgs {
    const float* guide;
    const float* dx;
    const float* dy;
    const float* gdx;
    const float* gdy;   // ngy partial planes sets, summed here
    int ngy;
    float* gg;
    int Cg, H, W, batch;
    float s2;
};

__global__ void __launch_bounds__(256) dist_adjoint_kernel(DistAdjArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int b = blockIdx.z;
    if (x >= a.W) return;
    const int H = a.H, W = a.W;
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t bp = static_cast<size_t>(b) * plane;
    const size_t i = static_cast<size_t>(y) * W + x;
    auto gy_at = [&](size_t idx) {
        float s = 0.f;
        for (int g = 0; g < a.ngy; ++g) s += a.gdy[(static_cast<size_t>(g) * a.batch + b) * plane + idx];
        return s;
    };
    // factors e = dL/dd * s2 / d at this pixel and at its right / lower neighbour
    const float ex0 = (x > 0) ? a.gdx[bp + i] * a.s2 / a.dx[bp + i] : 0.f;
    const float ex1 = (x + 1 < W) ? a.gdx[bp + i + 1] * a.s2 / a.dx[bp + i + 1] : 0.f;
    const float ey0 = (y > 0) ? gy_at(i) * a.s2 / a.dy[bp + i] : 0.f;
    const float ey1 = (y + 1 < H) ? gy_at(i + W) * a.s2 / a.dy[bp + i + W] : 0.f;
    for (int k = 0; k < a.Cg; ++k) {
        const float* g = a.guide + (static_cast<size_t>(b) * a.Cg + k) * plane;
        const float c = g[i];
        float acc = 0.f;
        if (x > 0) acc = fmaf(ex0, c - g[i - 1], acc);
        if (x + 1 < W) acc = fmaf(-ex1, g[i + 1] - c, acc);
        if (y > 0) acc = fmaf(ey0, c - g[i - W], acc);
        if (y + 1 < H) acc = fmaf(-ey1, g[i + W] - c, acc);
        a.gg[(static_cast<size_t>(b) * a.Cg + k) * plane + i] = acc;
    }
}

int launch_dist_adjoint(const DistAdj& p, Ctx& ctx) {
    DistAdjArgs a{p.guide, p.dx, p.dy, p.gdx, p.gdy, p.ngy, p.gg, p.Cg, p.H, p.W, p.batch, p.s2};
    const double px = static_cast<double>(p.batch) * p.H * p.W;
    ProfScope prof("dist_adjoint", px * 4.0 * (2.0 * p.Cg + 4.0), ctx.stream);
    hipLaunchKernelGGL(dist_adjoint_kernel, dim3((p.W + 255) / 256, p.H, p.batch), dim3(256), 0,
                       ctx.stream, a);
    return hip_fail(hipGetLastError());
}

}  // namespace dts
