// Tile bodies of the forward passes, shared by the per-pass kernels (dts_forward.hip)
// and the persistent batched kernel (dts_batched.hip).
//
// row_line / row_tile: one image row per group of waves (row_tile: the whole workgroup).
//   Lane l of wave v owns S consecutive pixels.
//   Each direction of the recurrence is a chain of affine maps: a serial composition over
//   the lane's S pixels, one 64-lane scan (DPP inside rows of 16 lanes, scalar reads
//   across rows), one exchange of wave totals through LDS, then a serial sweep from the
//   lane's exact carry-in.  With DIST the tile first computes the transformed distances
//   of its row from all guide bands (Eq. (8)-(9)) and stores dx and dy.
// col_tile: one chunk of R * NWV rows of a 64-column strip, one column per lane, the
//   chunk in registers; carries through LDS between waves and through tagged words
//   between chunks (dts_chunks.hpp).  With EPI the anticausal sweep ends in the solver
//   update of Eq. (3).
#pragma once

#include "dts_chunks.hpp"
#include "dts_device.hpp"

namespace dts {

struct RowArgs {
    const float* src;
    float* dst;
    const float* d;
    const float* guide;
    float* dx_out;
    float* dy_out;
    int Cg;
    float s2;
    int C, H, W;  // C: output channels
    float log2a;
};

constexpr int kMaxRowWaves = 16;

// Both directions of the recurrence over one row held by one wave (lane l owns pixels
// [l S, (l+1) S)), in registers: w[e] links pixel e to the one before it, wlast links
// the lane's last pixel to the next lane's first (0 for lane 63).  f is replaced by K.
template <int S>
__device__ __forceinline__ void row_filter_solo(const float (&w)[S], float wlast, float (&f)[S], int lane) {
    float la = 1.f, lb = 0.f;
#pragma unroll
    for (int e = 0; e < S; ++e) {
        lb = fmaf(w[e], lb - f[e], f[e]);
        la *= w[e];
    }
    scan_up_dpp(la, lb, lane);
    const float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
    float j = (lane == 0) ? 0.f : xb;
    (void)xa;
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
    const float yb = __shfl_down(lb, 1);
    float k = (lane == kWave - 1) ? 0.f : yb;
#pragma unroll
    for (int e = S - 1; e >= 0; --e) {
        const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
        k = fmaf(wn, k - f[e], f[e]);
        f[e] = k;
    }
}

// One image row processed by a group of `nw` waves of the workgroup; lane l of group wave
// v owns the S consecutive pixels starting at (64 v + l) S.  Per direction: a serial
// composition of the lane's S maps, one 64-lane scan, one exchange of wave totals through
// the group's LDS slots (fagg/bagg: nw entries, wfirst: nw + 1), and a serial sweep that
// produces the final values.  Every wave of the workgroup must call it the same number of
// times (it holds workgroup barriers); a group with `live` false reads and writes no
// pixel.
//
// SOLO: the row belongs to one wave alone (nw = 1): no LDS, no barrier, and the waves of
// a workgroup may call it independently.  SQ: src holds C / 2 channels and output channel
// c filters src channel c / 2, squared when c is odd (the pairs z, z^2 of Eq. (7)).
// BUF: the distances and the signal move through buffer resources (bload_seg /
// bstore_seg), for callers whose pointers come from memory: accessed through them
// directly they compile to generic (flat) accesses, which every LDS wait of the scans
// would also wait for.
template <int S, bool DIST, bool SOLO = false, bool SQ = false, bool BUF = false>
__device__ __forceinline__ void row_line(const RowArgs& a, int y, int b, int wave, int nw, bool live,
                                         float2* fagg, float2* bagg, float* wfirst) {
    static_assert(!(DIST && BUF), "the buffer path serves plain row passes only");
    const int lane = lane_id();
    const int H = a.H, W = a.W;
    const int We = live ? W : 0;  // pixels of the row this group touches
    const size_t plane = static_cast<size_t>(H) * W;
    const int n0 = (wave * kWave + lane) * S;

    // BUF: each channel's row is loaded one channel ahead (channel 0 with the distances),
    // so its loads are in flight while the previous channel is scanned: a row then costs
    // about one memory round trip instead of one per channel plus one for the distances.
    const int cin = SQ ? a.C >> 1 : a.C;
    [[maybe_unused]] const unsigned rowoff = static_cast<unsigned>(y) * static_cast<unsigned>(W) * 4u;
    [[maybe_unused]] const auto load_ch = [&](int c, float (&v)[S]) {
        const size_t pl = static_cast<size_t>(b) * cin + (SQ ? c >> 1 : c);
        bload_seg<S>(plane_rsrc(a.src + pl * plane, plane * sizeof(float)), rowoff, n0, We, v);
    };
    float f[S];

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
            load_seg<S>(g, n0, We, 0.f, v);
            load_seg<S>(gu, n0, We, 0.f, u);
            float prev = __shfl_up(v[S - 1], 1);
            if (lane == 0) prev = (n0 > 0 && n0 <= We) ? g[n0 - 1] : v[0];
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
        store_seg<S>(dxr, n0, We, ax);
        store_seg<S>(dyr, n0, We, ay);
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < We) ? weight(ax[e], a.log2a) : 0.f;
        }
    } else {
        float dv[S];
        if constexpr (BUF) {
            bload_seg<S>(plane_rsrc(a.d + static_cast<size_t>(b) * plane, plane * sizeof(float)), rowoff, n0,
                         We, dv);
            if (a.C > 0) load_ch(0, f);
        } else {
            const float* dr = a.d + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
            load_seg<S>(dr, n0, We, 1.f, dv);
        }
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int n = n0 + e;
            w[e] = (n > 0 && n < We) ? weight(dv[e], a.log2a) : 0.f;
        }
    }
    // weight linking each lane's last pixel to the next pixel (0 past the end of the row)
    float wlast = __shfl_down(w[0], 1);
    if constexpr (SOLO) {
        if (lane == kWave - 1) wlast = 0.f;
    } else {
        if (lane == 0) wfirst[wave] = w[0];
        if (wave == 0 && lane == 0) wfirst[nw] = 0.f;
        __syncthreads();
        if (lane == kWave - 1) wlast = wfirst[wave + 1];
    }

    for (int c = 0; c < a.C; ++c) {
        const size_t roff = (static_cast<size_t>(b) * a.C + c) * plane + static_cast<size_t>(y) * W;
        [[maybe_unused]] float fn[S];
        if constexpr (BUF) {
            if (c + 1 < a.C) load_ch(c + 1, fn);
        } else {
            const size_t soff =
                (static_cast<size_t>(b) * cin + (SQ ? c >> 1 : c)) * plane + static_cast<size_t>(y) * W;
            load_seg<S>(a.src + soff, n0, We, 0.f, f);
        }
        if (SQ && (c & 1)) {
#pragma unroll
            for (int e = 0; e < S; ++e) f[e] *= f[e];
        }

        // causal: J[n] = w[n] J[n-1] + (1 - w[n]) f[n]
        float la = 1.f, lb = 0.f;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            lb = fmaf(w[e], lb - f[e], f[e]);
            la *= w[e];
        }
        scan_up_dpp(la, lb, lane);
        float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
        float jin = 0.f;
        if constexpr (!SOLO) {
            if (lane == kWave - 1) fagg[wave] = make_float2(la, lb);
            __syncthreads();
            for (int u = 0; u < wave; ++u) {
                const float2 g = fagg[u];
                jin = fmaf(g.x, jin, g.y);
            }
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
        xa = __shfl_down(la, 1);
        xb = __shfl_down(lb, 1);
        float kin = 0.f;
        if constexpr (!SOLO) {
            if (lane == 0) bagg[wave] = make_float2(la, lb);
            __syncthreads();
            for (int u = nw - 1; u > wave; --u) {
                const float2 g = bagg[u];
                kin = fmaf(g.x, kin, g.y);
            }
        }
        float k = (lane == kWave - 1) ? kin : fmaf(xa, kin, xb);
#pragma unroll
        for (int e = S - 1; e >= 0; --e) {
            const float wn = (e == S - 1) ? wlast : w[e < S - 1 ? e + 1 : e];
            k = fmaf(wn, k - f[e], f[e]);
            f[e] = k;
        }
        if constexpr (BUF) {
            bstore_seg<S>(plane_rsrc(a.dst + (roff - static_cast<size_t>(y) * W), plane * sizeof(float)), rowoff,
                          n0, We, f);
            if (c + 1 < a.C) {
#pragma unroll
                for (int e = 0; e < S; ++e) f[e] = fn[e];
            }
        } else {
            store_seg<S>(a.dst + roff, n0, We, f);
        }
    }
}

// One workgroup per row (all of its waves form one group).
template <int S, bool DIST, bool SQ = false>
__device__ __forceinline__ void row_tile(const RowArgs& a, int y, int b) {
    __shared__ float2 fagg[kMaxRowWaves];
    __shared__ float2 bagg[kMaxRowWaves];
    __shared__ float wfirst[kMaxRowWaves + 1];
    row_line<S, DIST, false, SQ>(a, y, b, threadIdx.x >> 6, blockDim.x >> 6, true, fagg, bagg, wfirst);
}


struct ColArgs {
    const float* src;
    float* dst;
    const float* d;
    int C, H, W;
    float log2a;
    int G, S, NG, batch;
    int groups;  // strips processed at once
    int xcd;     // 1: every strip's chunks on one XCD (chunk_slot)
    unsigned long long* carry;
    unsigned epoch;
    int* status;
    int spin_limit;
    unsigned tag_xor;
    const float* zk;
    const float* tgt;
    const float* conf;
    int Cc;
    float* dst2;
    float lambda, step;
    float var_k;  // EPI 3: -log2(e) / (2 sigma_c^2)
};

struct NoHook {
    __device__ void operator()() const {}
};

// One workgroup = NWV waves stacked vertically over one 64-column strip: wave v owns rows
// [r0 + v R, r0 + (v+1) R) of the chunk, one column per lane, all in registers.  `hook`
// runs on every thread once the chunk's carries are known, i.e. once the tile no longer
// waits on any other tile.
// EPI: 0 plain pass; 1 the solver update of Eq. (3) (reads z^k, t, c); 2 the update with
// a precomputed data-term gradient D in place of c (z - t) (reads z^k and D from `tgt`);
// 3 the confidence of Eq. (7) from channel pairs (DT(z), DT(z^2)) of an even group size:
// writes exp(-(DT(z^2) - DT(z)^2) / (2 sigma_c^2)) to channel c / 2 of `dst` (C / 2
// planes) instead of the pair.
template <int CT, int R, int NWV, int EPI, typename Hook = NoHook>
__device__ __forceinline__ void col_tile(const ColArgs& a, const CarryCtx& cctx, ChunkLds<CT, NWV>& L,
                                         int chunk, int strip, int grp, int b, Hook hook = Hook{}) {
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
    // The chunk's loads are issued at raised wave priority, so the issue of a workgroup
    // starting its tile is not held back by the ALU work of the CU's other workgroups
    // (10240^2 one-channel column pass 298 -> 293 us, 16-band solve 19.25 -> 19.10 ms).
    __builtin_amdgcn_s_setprio(3);
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

    __builtin_amdgcn_s_setprio(0);
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
    chunk_carries<CT, NWV>(cctx, L, b, grp, strip, chunk, lane, wave, valid, ncv);
    __syncthreads();
    hook();

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
    if constexpr (EPI == 3) {
        static_assert(CT % 2 == 0, "the variance epilogue takes channel pairs");
#pragma unroll
        for (int c = 0; c < CT; c += 2) {
            if (c < ncv) {  // ncv is even: C and the group's first channel are
                float K0 = Kin[c], K1 = Kin[c + 1];
                const size_t pidx = (static_cast<size_t>(b) * a.C + c0 + c) >> 1;
                const auto ors = plane_rsrc(a.dst + pidx * plane, pbytes);
                unsigned vo = voff + static_cast<unsigned>(R - 1) * rowb;
#pragma unroll
                for (int r = R - 1; r >= 0; --r) {
                    const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                    K0 = fmaf(wn, K0 - f[c][r], f[c][r]);
                    K1 = fmaf(wn, K1 - f[c + 1][r], f[c + 1][r]);
                    bstore(ors, vo, 0, exp2_fast(fmaf(-K0, K0, K1) * a.var_k));
                    vo = opaque_vadd(vo, 0u - rowb);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        if (c < ncv) {
            float K = Kin[c];
            const size_t pidx = static_cast<size_t>(b) * a.C + c0 + c;
            const auto ors = plane_rsrc(a.dst + pidx * plane, pbytes);
            unsigned vo = voff + static_cast<unsigned>(R - 1) * rowb;
            if constexpr (EPI != 0) {
                const auto zrs = plane_rsrc(a.zk + pidx * plane, pbytes);
                const auto trs = plane_rsrc(a.tgt + pidx * plane, pbytes);
                [[maybe_unused]] const auto crs = plane_rsrc(
                    EPI == 1 ? a.conf + (static_cast<size_t>(b) * a.Cc + ((a.Cc == 1) ? 0 : c0 + c)) * plane : a.tgt,
                    pbytes);
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
                        if constexpr (EPI == 1) cf[q] = bload(crs, vl, 0);
                        vl = opaque_vadd(vl, rowb);
                    }
#pragma unroll
                    for (int q = kEpiBlock - 1; q >= 0; --q) {
                        const int r = blk * kEpiBlock + q;
                        const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                        K = fmaf(wn, K - f[c][r], f[c][r]);
                        const float upd = (EPI == 1) ? fmaf(a.lambda, z[q] - K, cf[q] * (z[q] - tt[q]))
                                                     : fmaf(a.lambda, z[q] - K, tt[q]);
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
}

}  // namespace dts
