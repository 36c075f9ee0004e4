// Forward kernels of the domain-transform filter on gfx950.
//
// Method (Bapat & Frahm, "The Domain Transform Solver", ECCV 2018): the edge-aware mean of
// Sec. 3.2 computed with the recursive domain-transform filter -- per-pixel transformed
// distances from the guide's channel differences (Eq. (8)-(9)), weights a^d, and
// alternating causal+anticausal first-order recursive passes along rows and columns.
//
// Row pass: one workgroup per row.  The row is cut into tiles of 256 elements; lane l of a
// wave owns elements 4l..4l+3 of a tile (one coalesced float4 access per lane).  Each
// tile is scanned as a chain of affine maps: a serial composition over the lane's four
// elements, then a 64-lane shuffle scan, then the carry from the previous tile.  Waves own
// consecutive tiles; wave carries cross through LDS once per direction.
//
// Column pass: lanes are columns (every access is a coalesced 256-byte row segment per
// wave), each workgroup owns a chunk of R rows of its strip and keeps it in registers.
// Chunks exchange carries through tagged 64-bit words in device memory: a decoupled
// look-back resolves the causal carry from earlier chunks, then a look-ahead resolves the
// anticausal carry from later chunks, so every element is read and written exactly once.
#include <mutex>

#include "../../include/dts.h"
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
    int tpw;  // tiles per wave
};

constexpr int kTile = 256;
constexpr int kMaxRowWaves = 16;

// Up to 16 waves of 64 lanes per row, each owning up to TPW tiles of 256 elements.
template <int TPW, bool DIST>
__global__ void __launch_bounds__(1024) row_pass_kernel(RowArgs a) {
    __shared__ float2 fagg[kMaxRowWaves];
    __shared__ float2 bagg[kMaxRowWaves];
    __shared__ float wfirst[kMaxRowWaves];

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int y = blockIdx.x;
    const int b = blockIdx.y;
    const int H = a.H, W = a.W;
    const size_t plane = static_cast<size_t>(H) * W;
    const int ntiles = (W + kTile - 1) / kTile;
    const int t0 = wave * a.tpw;
    const int nt = max(0, min(a.tpw, ntiles - t0));
    const bool vec = (W & 3) == 0;

    float w[TPW][4];
    if constexpr (DIST) {
        float ax[TPW][4], ay[TPW][4];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) ax[i][e] = ay[i][e] = 0.f;
        for (int k = 0; k < a.Cg; ++k) {
            const float* g = a.guide + (static_cast<size_t>(b) * a.Cg + k) * plane +
                             static_cast<size_t>(y) * W;
            const float* gu = (y > 0) ? g - W : g;
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                if (i < nt) {
                    const int n0 = (t0 + i) * kTile + 4 * lane;
                    const float4 v = load4(g, n0, W, vec, 0.f);
                    const float4 u = load4(gu, n0, W, vec, 0.f);
                    float prev = __shfl_up(v.w, 1);
                    if (lane == 0) prev = (n0 > 0) ? g[n0 - 1] : v.x;
                    const float ex0 = v.x - prev, ex1 = v.y - v.x, ex2 = v.z - v.y,
                                ex3 = v.w - v.z;
                    ax[i][0] = fmaf(ex0, ex0, ax[i][0]);
                    ax[i][1] = fmaf(ex1, ex1, ax[i][1]);
                    ax[i][2] = fmaf(ex2, ex2, ax[i][2]);
                    ax[i][3] = fmaf(ex3, ex3, ax[i][3]);
                    const float ey0 = v.x - u.x, ey1 = v.y - u.y, ey2 = v.z - u.z,
                                ey3 = v.w - u.w;
                    ay[i][0] = fmaf(ey0, ey0, ay[i][0]);
                    ay[i][1] = fmaf(ey1, ey1, ay[i][1]);
                    ay[i][2] = fmaf(ey2, ey2, ay[i][2]);
                    ay[i][3] = fmaf(ey3, ey3, ay[i][3]);
                }
            }
        }
        float* dxr = a.dx_out + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
        float* dyr = a.dy_out + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                const int n0 = (t0 + i) * kTile + 4 * lane;
                float4 vx, vy;
                vx.x = sqrtf(fmaf(a.s2, ax[i][0], 1.f));
                vx.y = sqrtf(fmaf(a.s2, ax[i][1], 1.f));
                vx.z = sqrtf(fmaf(a.s2, ax[i][2], 1.f));
                vx.w = sqrtf(fmaf(a.s2, ax[i][3], 1.f));
                vy.x = sqrtf(fmaf(a.s2, ay[i][0], 1.f));
                vy.y = sqrtf(fmaf(a.s2, ay[i][1], 1.f));
                vy.z = sqrtf(fmaf(a.s2, ay[i][2], 1.f));
                vy.w = sqrtf(fmaf(a.s2, ay[i][3], 1.f));
                store4(dxr, n0, W, vec, vx);
                store4(dyr, n0, W, vec, vy);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int n = n0 + e;
                    w[i][e] = (n > 0 && n < W) ? weight(get(vx, e), a.log2a) : 0.f;
                }
            }
        }
    } else {
        const float* dr = a.d + static_cast<size_t>(b) * plane + static_cast<size_t>(y) * W;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                const int n0 = (t0 + i) * kTile + 4 * lane;
                const float4 dv = load4(dr, n0, W, vec, 1.f);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int n = n0 + e;
                    w[i][e] = (n > 0 && n < W) ? weight(get(dv, e), a.log2a) : 0.f;
                }
            }
        }
    }

    // weight of the first element after this wave's tiles (0 past the end of the row)
    if (lane == 0 && nt > 0) wfirst[wave] = w[0][0];
    __syncthreads();
    float w_after = 0.f;
    if (nt > 0 && (t0 + nt) * kTile < W) w_after = wfirst[wave + 1];

    for (int c = 0; c < a.C; ++c) {
        const size_t roff = (static_cast<size_t>(b) * a.C + c) * plane + static_cast<size_t>(y) * W;
        const float* srow = a.src + roff;
        float* drow = a.dst + roff;
        float f[TPW][4];
        float qs[TPW];     // causal: the lane's state factor just before its first element
        float ps[TPW];     // anticausal: the lane's state factor just after its last element
        float wl[TPW];     // weight linking the lane's last element to the next element
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                const float4 v = load4(srow, (t0 + i) * kTile + 4 * lane, W, vec, 0.f);
                f[i][0] = v.x;
                f[i][1] = v.y;
                f[i][2] = v.z;
                f[i][3] = v.w;
            }
        }
        // causal: state (Q, J) with J_actual = J + Q * J_in, J_in = J before the wave's tiles
        float SQ = 1.f, SJ = 0.f;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                float la = 1.f, lb = 0.f;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    lb = fmaf(w[i][e], lb - f[i][e], f[i][e]);
                    la *= w[i][e];
                }
                scan_maps_up(la, lb, lane);
                float xa = __shfl_up(la, 1), xb = __shfl_up(lb, 1);
                if (lane == 0) {
                    xa = 1.f;
                    xb = 0.f;
                }
                float qq = xa * SQ, jj = fmaf(xa, SJ, xb);
                qs[i] = qq;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    qq *= w[i][e];
                    jj = fmaf(w[i][e], jj - f[i][e], f[i][e]);
                    f[i][e] = jj;
                }
                SQ = __shfl(qq, kWave - 1);
                SJ = __shfl(jj, kWave - 1);
            }
        }
        if (lane == 0) fagg[wave] = make_float2(SQ, SJ);
        __syncthreads();
        float jin = 0.f;
        for (int u = 0; u < wave; ++u) {
            const float2 g = fagg[u];
            jin = fmaf(g.x, jin, g.y);
        }
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                float qq = qs[i];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    qq *= w[i][e];
                    f[i][e] = fmaf(qq, jin, f[i][e]);
                }
            }
        }

        // anticausal: state (P, K) with K_actual = K + P * K_in, K_in = K after the tiles
        float SP = 1.f, SK = 0.f;
#pragma unroll
        for (int i = TPW - 1; i >= 0; --i) {
            if (i < nt) {
                const float from_next_lane = __shfl_down(w[i][0], 1);
                float tile_next = w_after;
                if (i + 1 < TPW && i + 1 < nt) tile_next = __shfl(w[(i + 1 < TPW) ? i + 1 : i][0], 0);
                const float wn3 = (lane == kWave - 1) ? tile_next : from_next_lane;
                wl[i] = wn3;
                const float wn[4] = {w[i][1], w[i][2], w[i][3], wn3};
                float la = 1.f, lb = 0.f;
#pragma unroll
                for (int e = 3; e >= 0; --e) {
                    lb = fmaf(wn[e], lb - f[i][e], f[i][e]);
                    la *= wn[e];
                }
                scan_maps_down(la, lb, lane);
                float xa = __shfl_down(la, 1), xb = __shfl_down(lb, 1);
                if (lane == kWave - 1) {
                    xa = 1.f;
                    xb = 0.f;
                }
                float pp = xa * SP, kk = fmaf(xa, SK, xb);
                ps[i] = pp;
#pragma unroll
                for (int e = 3; e >= 0; --e) {
                    pp *= wn[e];
                    kk = fmaf(wn[e], kk - f[i][e], f[i][e]);
                    f[i][e] = kk;
                }
                SP = __shfl(pp, 0);
                SK = __shfl(kk, 0);
            }
        }
        if (lane == 0) bagg[wave] = make_float2(SP, SK);
        __syncthreads();
        float kin = 0.f;
        for (int u = nw - 1; u > wave; --u) {
            const float2 g = bagg[u];
            kin = fmaf(g.x, kin, g.y);
        }
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < nt) {
                const float wn[4] = {w[i][1], w[i][2], w[i][3], wl[i]};
                float pp = ps[i];
                float4 v;
                pp *= wn[3];
                v.w = fmaf(pp, kin, f[i][3]);
                pp *= wn[2];
                v.z = fmaf(pp, kin, f[i][2]);
                pp *= wn[1];
                v.y = fmaf(pp, kin, f[i][1]);
                pp *= wn[0];
                v.x = fmaf(pp, kin, f[i][0]);
                store4(drow, (t0 + i) * kTile + 4 * lane, W, vec, v);
            }
        }
    }
}

template <int TPW, bool DIST>
static void launch_row_t(const RowArgs& a, int nw, int batch, int H, hipStream_t s) {
    // algorithmic bytes: signal in and out (C planes), distances in -- or, on the fused
    // first pass, the guide in (Cg planes) and both distance planes out instead
    const double px = static_cast<double>(batch) * H * a.W;
    const double bytes = DIST ? px * 4.0 * (2.0 * a.C + a.Cg + 2.0) : px * 4.0 * (2.0 * a.C + 1.0);
    ProfScope prof(DIST ? "row_pass_dist" : "row_pass", bytes, s);
    hipLaunchKernelGGL((row_pass_kernel<TPW, DIST>), dim3(H, batch), dim3(nw * kWave), 0, s, a);
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
    const int ntiles = (p.W + kTile - 1) / kTile;
    const bool dist = p.guide != nullptr;
    const hipStream_t s = ctx.stream;
    int tpw = 1;
    if (ntiles <= 16) tpw = 1;
    else if (ntiles <= 32) tpw = 2;
    else if (ntiles <= 64) tpw = 4;
    else return DTS_ENOTSUP;
    const int nw = (ntiles + tpw - 1) / tpw;
    a.tpw = tpw;
    switch (tpw) {
        case 1: dist ? launch_row_t<1, true>(a, nw, p.batch, p.H, s) : launch_row_t<1, false>(a, nw, p.batch, p.H, s); break;
        case 2: dist ? launch_row_t<2, true>(a, nw, p.batch, p.H, s) : launch_row_t<2, false>(a, nw, p.batch, p.H, s); break;
        case 4: dist ? launch_row_t<4, true>(a, nw, p.batch, p.H, s) : launch_row_t<4, false>(a, nw, p.batch, p.H, s); break;
        default: dist ? launch_row_t<4, true>(a, nw, p.batch, p.H, s) : launch_row_t<4, false>(a, nw, p.batch, p.H, s); break;
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
    int G, S, NG;
    unsigned n_tickets;
    unsigned* ticket;
    unsigned ticket_base;
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

template <int CT>
struct CarryWords {
    static constexpr int kFwdA = 0;                 // product of the chunk's weights
    static constexpr int kFwdB = 1;                 // + c: causal output, zero carry-in
    static constexpr int kFwdIncl = 1 + CT;         // + c: causal output at the chunk end
    static constexpr int kBwdP = 1 + 2 * CT;        // anticausal carry factor
    static constexpr int kBwdAlpha = 2 + 2 * CT;    // + c: anticausal output, zero carry-in
    static constexpr int kBwdIncl = 2 + 3 * CT;     // + c: anticausal output at chunk start
    static constexpr int kWords = 2 + 4 * CT;
};

template <int CT, int R, int NWC, bool EPI>
__global__ void __launch_bounds__(kWave * NWC) col_pass_kernel(ColArgs a) {
    using CW = CarryWords<CT>;
    constexpr int SW = kWave * NWC;
    __shared__ unsigned s_ticket;
    if (threadIdx.x == 0) s_ticket = atomicAdd(a.ticket, 1u) - a.ticket_base;
    __syncthreads();
    const unsigned t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= a.n_tickets) {  // never taken when the counter was cleared for this call
        if (threadIdx.x == 0) flag_error(a.status, kErrBadTicket);
        return;
    }
    const int chunk = static_cast<int>(t % a.G);
    unsigned rest = t / a.G;
    const int strip = static_cast<int>(rest % a.S);
    rest /= a.S;
    const int grp = static_cast<int>(rest % a.NG);
    const int b = static_cast<int>(rest / a.NG);

    const int lane = lane_id();
    const int col = (threadIdx.x >> 6) * kWave + lane;
    const int H = a.H, W = a.W;
    const int x = strip * SW + col;
    const bool valid = x < W;
    const int r0 = chunk * R;
    const int nr = min(R, H - r0);
    const size_t plane = static_cast<size_t>(H) * W;
    const size_t pbytes = plane * sizeof(float);
    const int c0 = grp * CT;
    const int ncv = min(CT, a.C - c0);
    // Row r of the chunk sits at byte offset voff + r * rowb of a plane; lanes past the
    // right edge and rows past the bottom edge fall outside the plane's buffer range, so
    // their loads read 0 and their stores are dropped.
    const unsigned voff = (valid ? static_cast<unsigned>(x) * 4u : kInvalidOffset) +
                          static_cast<unsigned>(r0) * static_cast<unsigned>(W) * 4u;
    const unsigned rowb = static_cast<unsigned>(W) * 4u;

    // Weights of the chunk's rows.  The first row of the image and rows past the bottom
    // edge get weight 0: that is the boundary J[0] = f[0] going down and K[H-1] = J[H-1]
    // going up, and it makes padded rows drop out of both recurrences.
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
    const float wnext = weight(bload(drs, voff + static_cast<unsigned>(R) * rowb, 0), a.log2a) *
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

    // phase 1: causal scan with zero carry-in, plus the anticausal coefficients
    //   K[first] = BJ + BQ * J_carry + P * K_carry
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

    const size_t strip_base =
        ((static_cast<size_t>(b) * a.NG + grp) * a.S + strip) * static_cast<size_t>(a.G);
    auto word = [&](int j, int k) -> unsigned long long* {
        return a.carry + ((strip_base + j) * CW::kWords + k) * SW + col;
    };
    const unsigned ep = a.epoch;

    // causal carry: decoupled look-back over earlier chunks
    float Jc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) Jc[c] = 0.f;
    if (chunk > 0 && valid) {
        publish(word(chunk, CW::kFwdA), ep, Q);
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < ncv) publish(word(chunk, CW::kFwdB + c), ep, J[c]);
        float GA = 1.f, GB[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) GB[c] = 0.f;
        int j = chunk - 1;
        int spins = 0;
        while (true) {
            float v[CT];
            bool ok = true;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < ncv) ok = peek(word(j, CW::kFwdIncl + c), ep, v[c]) && ok;
            if (ok) {
#pragma unroll
                for (int c = 0; c < CT; ++c) Jc[c] = fmaf(GA, (c < ncv) ? v[c] : 0.f, GB[c]);
                break;
            }
            float A;
            ok = peek(word(j, CW::kFwdA), ep, A);
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < ncv) ok = peek(word(j, CW::kFwdB + c), ep, v[c]) && ok;
            if (ok) {
#pragma unroll
                for (int c = 0; c < CT; ++c) GB[c] = fmaf(GA, (c < ncv) ? v[c] : 0.f, GB[c]);
                GA *= A;
                spins = 0;
                if (--j < 0) {
#pragma unroll
                    for (int c = 0; c < CT; ++c) Jc[c] = GB[c];
                    break;
                }
                continue;
            }
            if (++spins > kSpinLimit) {
                flag_error(a.status, kErrSpinTimeout);
#pragma unroll
                for (int c = 0; c < CT; ++c) Jc[c] = GB[c];
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (valid) {
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < ncv) publish(word(chunk, CW::kFwdIncl + c), ep, fmaf(Q, Jc[c], J[c]));
    }

    // anticausal carry: look-ahead over later chunks
    float alpha[CT], Kc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        alpha[c] = fmaf(BQ, Jc[c], BJ[c]);
        Kc[c] = 0.f;
    }
    if (chunk < a.G - 1 && valid) {
        publish(word(chunk, CW::kBwdP), ep, pi);
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < ncv) publish(word(chunk, CW::kBwdAlpha + c), ep, alpha[c]);
        float GA = 1.f, GB[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) GB[c] = 0.f;
        int j = chunk + 1;
        int spins = 0;
        while (true) {
            float v[CT];
            bool ok = true;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < ncv) ok = peek(word(j, CW::kBwdIncl + c), ep, v[c]) && ok;
            if (ok) {
#pragma unroll
                for (int c = 0; c < CT; ++c) Kc[c] = fmaf(GA, (c < ncv) ? v[c] : 0.f, GB[c]);
                break;
            }
            float P;
            ok = peek(word(j, CW::kBwdP), ep, P);
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < ncv) ok = peek(word(j, CW::kBwdAlpha + c), ep, v[c]) && ok;
            if (ok) {
#pragma unroll
                for (int c = 0; c < CT; ++c) GB[c] = fmaf(GA, (c < ncv) ? v[c] : 0.f, GB[c]);
                GA *= P;
                spins = 0;
                if (++j >= a.G) {
#pragma unroll
                    for (int c = 0; c < CT; ++c) Kc[c] = GB[c];
                    break;
                }
                continue;
            }
            if (++spins > kSpinLimit) {
                flag_error(a.status, kErrSpinTimeout);
#pragma unroll
                for (int c = 0; c < CT; ++c) Kc[c] = GB[c];
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (valid) {
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < ncv) publish(word(chunk, CW::kBwdIncl + c), ep, fmaf(pi, Kc[c], alpha[c]));
    }

    // phase 3: causal values with the true carry, then the anticausal sweep and the store
    {
        float q = opaque(1.f);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            q *= w[r];
#pragma unroll
            for (int c = 0; c < CT; ++c) f[c][r] = fmaf(q, Jc[c], f[c][r]);
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        if (c < ncv) {
            float K = Kc[c];
            const size_t pidx = static_cast<size_t>(b) * a.C + c0 + c;
            const auto ors = plane_rsrc(a.dst + pidx * plane, pbytes);
            unsigned vo = voff + static_cast<unsigned>(R - 1) * rowb;
            if constexpr (EPI) {
                const int cc = (a.Cc == 1) ? 0 : c0 + c;
                const auto zrs = plane_rsrc(a.zk + pidx * plane, pbytes);
                const auto trs = plane_rsrc(a.tgt + pidx * plane, pbytes);
                const auto crs = plane_rsrc(a.conf + (static_cast<size_t>(b) * a.Cc + cc) * plane, pbytes);
                const auto o2rs = plane_rsrc(a.dst2 ? a.dst2 + pidx * plane : a.dst, a.dst2 ? pbytes : 0);
#pragma unroll
                for (int r = R - 1; r >= 0; --r) {
                    const float wn = (r + 1 < R) ? w[(r + 1 < R) ? r + 1 : r] : wnext;
                    K = fmaf(wn, K - f[c][r], f[c][r]);
                    const float z = bload(zrs, vo, 0);
                    const float tt = bload(trs, vo, 0);
                    const float cf = bload(crs, vo, 0);
                    const float upd = fmaf(a.lambda, z - K, cf * (z - tt));
                    const float zn = fmaf(-a.step, upd, z);
                    bstore(ors, vo, 0, zn);
                    bstore(o2rs, vo, 0, zn);
                    vo = opaque_vadd(vo, 0u - rowb);
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

template <int CT>
struct ColShape;
template <>
struct ColShape<1> {
    static constexpr int R = 32;
};
template <>
struct ColShape<2> {
    static constexpr int R = 24;
};
template <>
struct ColShape<3> {
    static constexpr int R = 16;
};
template <>
struct ColShape<4> {
    static constexpr int R = 16;
};

constexpr int kColWaves = 1;

static int col_group(int C) { return C < 4 ? C : 4; }

static int col_rows(int C) {
    switch (col_group(C)) {
        case 1: return ColShape<1>::R;
        case 2: return ColShape<2>::R;
        case 3: return ColShape<3>::R;
        default: return ColShape<4>::R;
    }
}

size_t col_carry_words(int batch, int H, int W, int C) {
    const int ct = col_group(C);
    const int R = col_rows(C);
    const size_t G = (H + R - 1) / R;
    const size_t SW = kWave * kColWaves;
    const size_t S = (W + SW - 1) / SW;
    const size_t NG = (C + ct - 1) / ct;
    return static_cast<size_t>(batch) * NG * S * G * (2 + 4 * ct) * SW;
}

// Workgroups of one column-pass launch that can be resident at once on this device.  A
// strip's chunks wait on each other (earlier ones for the causal carry, later ones for
// the anticausal carry), and tickets are handed out in order to running workgroups only,
// so the launch always completes when a whole strip's chunks fit on the device at once.
template <int CT, bool EPI>
static int col_capacity() {
    static int cached[64] = {0};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, col_pass_kernel<CT, ColShape<CT>::R, kColWaves, EPI>,
                kWave * kColWaves, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus;
    }
    return cached[dev];
}

template <int CT, bool EPI>
static int launch_col_t(const ColArgs& a, unsigned n, hipStream_t s) {
    const int cap = col_capacity<CT, EPI>();
    if (cap <= 0) return hip_fail(hipErrorNoDevice);
    if (a.G > cap) return DTS_ENOTSUP;
    // algorithmic bytes: signal in and out, distances in; the update epilogue also reads
    // z^k, the target and the confidence
    const double px = static_cast<double>(n) / (static_cast<double>(a.NG) * a.S * a.G) * a.H * a.W;
    const double bytes = EPI ? px * 4.0 * (4.0 * a.C + 1.0 + (a.Cc == 1 ? 1.0 : a.C))
                             : px * 4.0 * (2.0 * a.C + 1.0);
    ProfScope prof(EPI ? "col_pass_update" : "col_pass", bytes, s);
    hipLaunchKernelGGL((col_pass_kernel<CT, ColShape<CT>::R, kColWaves, EPI>), dim3(n),
                       dim3(kWave * kColWaves), 0, s, a);
    return hip_fail(hipGetLastError());
}

int launch_col_pass(const ColPass& p, Ctx& ctx) {
    ColArgs a;
    a.src = p.src;
    a.dst = p.dst;
    a.d = p.d;
    a.C = p.C;
    a.H = p.H;
    a.W = p.W;
    a.log2a = p.log2a;
    const int ct = col_group(p.C);
    const int R = col_rows(p.C);
    const int SW = kWave * kColWaves;
    a.G = (p.H + R - 1) / R;
    a.S = (p.W + SW - 1) / SW;
    a.NG = (p.C + ct - 1) / ct;
    a.ticket = ctx.ticket;
    a.ticket_base = ctx.ticket_base;
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
    const unsigned n = static_cast<unsigned>(p.batch) * a.NG * a.S * a.G;
    a.n_tickets = n;
    ctx.ticket_base += n;
    switch (ct) {
        case 1: return p.epilogue ? launch_col_t<1, true>(a, n, ctx.stream) : launch_col_t<1, false>(a, n, ctx.stream);
        case 2: return p.epilogue ? launch_col_t<2, true>(a, n, ctx.stream) : launch_col_t<2, false>(a, n, ctx.stream);
        case 3: return p.epilogue ? launch_col_t<3, true>(a, n, ctx.stream) : launch_col_t<3, false>(a, n, ctx.stream);
        default: return p.epilogue ? launch_col_t<4, true>(a, n, ctx.stream) : launch_col_t<4, false>(a, n, ctx.stream);
    }
}

// ---------------------------------------------------------------------------------------
// Small utility kernels (fills instead of hipMemsetAsync so calls stay graph-capturable)
// ---------------------------------------------------------------------------------------
__global__ void zero_kernel(uint4* p, size_t n16) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void copy_kernel(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

int launch_zero(void* ptr, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return 0;
    const size_t blocks = (n16 + 255) / 256;
    const unsigned g = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(zero_kernel, dim3(g), dim3(256), 0, s, static_cast<uint4*>(ptr), n16);
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
