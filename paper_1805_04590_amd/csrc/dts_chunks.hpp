// Chunked carry exchange shared by the column passes (forward and adjoint).
//
// A column strip (64 columns, one per lane) is cut into chunks of rows, one chunk per
// workgroup, and each chunk into per-wave row segments.  A column pass evaluates NCH
// first-order recurrences per column that share their weights:
//   forward  X[n] = w[n] X[n-1] + u[n]                 (u = (1 - w) f for the filter's
//                                                         causal scan, u = g for an adjoint)
//   backward Y[n] = w[n+1] Y[n+1] + (1 - w[n+1]) X[n]
// After a chunk has run both recurrences with zero carries it knows, per channel,
//   X[end]   = A X_in + B,      Y[first] = BJ + BQ X_in + P Y_in,
// where X_in is X at the row above the chunk and Y_in is Y at the row below it, A the
// product of the chunk's weights and P the product of the weights that link its rows to
// the row below.  Each chunk publishes these five aggregates as soon as its own rows are
// scanned, and then resolves both carries from its neighbours' aggregates alone:
//   X_in(k) = B(k-1) + A(k-1) (B(k-2) + A(k-2) (...)),
//   Y_in(k) = sum_{j>k} [prod_{k<m<j} P(m)] (BJ(j) + BQ(j) X_in(j)),
// with X_in(j) carried forward from X_in(k + 1) = A(k) X_in(k) + B(k).  No chunk waits
// for another chunk's carries, only for its aggregates.
//
// Every weight is a^d with a < 1 and d >= 1 (Eq. (8)-(9)), so a carry fades by at least a
// factor a per row.  A walk stops once the product of the factors still to be applied
// falls below 2^-40: what it leaves out is below 2^-40 of the largest magnitude the
// recurrence takes on the line (for a filter pass, of the largest input; for an adjoint
// pass at most 1 / (1 - a) times the largest input gradient), far under one fp32
// rounding of the result.  Where the product does not fall that
// far, the walk runs to the first or last chunk and is exact.  Which neighbours a chunk
// composes, and in which order, depends on the data only, so a given launch shape gives
// bitwise-identical results on every run.
#pragma once

#include "dts_device.hpp"

namespace dts {

struct CarryCtx {
    unsigned long long* carry;  // carry words of this launch's strips
    unsigned epoch;             // tag of this launch
    int* status;                // device-side status word
    int G, S, NG;               // chunks per strip, strips per plane, channel groups
    int spin_limit;             // polls before a wait gives up
    unsigned tag_xor;           // 0; non-zero only to exercise the timeout path (no tag matches)
};

template <int NCH>
struct CarryWords {
    static constexpr int kA = 0;            // product of the chunk's weights
    static constexpr int kB = 1;            // + c: forward output at the chunk end, zero carry-in
    static constexpr int kP = 1 + NCH;      // backward carry factor
    static constexpr int kBQ = 2 + NCH;     // backward output's factor on the forward carry-in
    static constexpr int kBJ = 3 + NCH;     // + c: backward output at the chunk start, zero carries
    static constexpr int kWords = 3 + 2 * NCH;
};

// A walk stops once the product of the factors still to be applied is below this.
constexpr float kCarryNegligible = 0x1p-40f;

template <int NCH>
__device__ __forceinline__ gword* carry_word(const CarryCtx& a, size_t strip_base, int j, int k, int col) {
    return global_word(a.carry + ((strip_base + j) * CarryWords<NCH>::kWords + k) * kWave + col);
}

// Per-wave aggregates of one chunk (written by every wave), and, in a union, the staging
// area of the exchange and the carries into every wave (written by wave 0 once the
// exchange is over), one column per lane.  In each round trip of the exchange, wave v of
// the first half stages the aggregates of the v-th earlier neighbour still to be
// composed, and wave NWV/2 + v those of the v-th later one.
template <int NCH, int NWV>
struct ChunkLds {
    float A[NWV][kWave], P[NWV][kWave], BQ[NWV][kWave];
    float B[NWV][NCH][kWave], BJ[NWV][NCH][kWave];
    union {
        struct {
            float Jin[NWV][NCH][kWave];
            float Kin[NWV][NCH][kWave];
        };
        struct {
            float A[NWV][kWave], P[NWV][kWave], BQ[NWV][kWave];
            float B[NWV][NCH][kWave], BJ[NWV][NCH][kWave];
            int ok[NWV][kWave];   // the staged neighbour's words were all written
        } n;
    };
    // State of the two walks per lane, kept here between round trips so that it holds no
    // registers while the staging loads are in flight (see chunk_carries).
    float FA[kWave], PA[kWave], V[kWave], GXa[kWave];
    float FB[NCH][kWave], U[NCH][kWave], GXb[NCH][kWave];
    int fj[kWave], bj[kWave];     // per lane: next neighbour of each walk, or kWalkDone
    int more;                     // some lane of wave 0 is still walking
};

constexpr int kWalkDone = -0x40000000;

// True when the first `ncv` of the tagged words carry the tag `ep`.
template <int NCH>
__device__ __forceinline__ bool tags_ok(const unsigned long long (&w)[NCH], int ncv, unsigned ep) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        if (c < ncv) ok = ok && static_cast<unsigned>(w[c] >> 32) == ep;
    return ok;
}

__device__ __forceinline__ unsigned long long load_word(gword* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float word_value(unsigned long long w) {
    return __uint_as_float(static_cast<unsigned>(w));
}

// All waves of a chunk's workgroup: wave 0 composes the waves into the chunk aggregates
// and publishes them; all waves stage neighbours' aggregates; wave 0 resolves the carries
// and writes every wave's carry-in X_in (L.Jin) and Y_in (L.Kin).  `ncv` channels are
// valid; `valid` is false for lanes past the right edge of the image.
template <int NCH, int NWV>
__device__ void chunk_carries(const CarryCtx& a, ChunkLds<NCH, NWV>& L, int b, int grp, int strip,
                              int chunk, int lane, int wave, bool valid, int ncv) {
    static_assert(NWV >= 2 && NWV % 2 == 0, "the exchange splits the waves in two halves");
    using CW = CarryWords<NCH>;
    constexpr int NH = NWV / 2;
    const size_t strip_base =
        ((static_cast<size_t>(b) * a.NG + grp) * a.S + strip) * static_cast<size_t>(a.G);
    const unsigned ep = a.epoch;        // tag written
    const unsigned want = ep ^ a.tag_xor;  // tag a reader accepts
    const int G = a.G;

    // chunk aggregates: wave 0 composes the waves top to bottom and leaves them in the
    // staging area (free until the exchange starts); then every wave publishes some of
    // the words, so no wave holds them all in registers
    if (wave == 0) {
        float CA = 1.f, CP = 1.f, CBQ = 0.f, CB[NCH], CBJ[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) CB[c] = CBJ[c] = 0.f;
#pragma unroll
        for (int v = 0; v < NWV; ++v) {
            // wave v's forward carry-in is CA X_in + CB (before wave v is composed in)
            const float BQv = L.BQ[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) CBJ[c] = fmaf(CP, fmaf(BQv, CB[c], L.BJ[v][c][lane]), CBJ[c]);
            CBQ = fmaf(CP, BQv * CA, CBQ);
            CP *= L.P[v][lane];
            const float Av = L.A[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) CB[c] = fmaf(Av, CB[c], L.B[v][c][lane]);
            CA *= Av;
        }
        L.n.A[0][lane] = CA;
        L.n.P[0][lane] = CP;
        L.n.BQ[0][lane] = CBQ;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            L.n.B[0][c][lane] = CB[c];
            L.n.BJ[0][c][lane] = CBJ[c];
        }
    }

    // the exchange.  Forward walk: X_in = FB + FA * (rest).  Backward walk:
    // Y_in = U + V X_in(k + 1) + PA * (rest), with X_in(j) = GXa X_in(k + 1) + GXb for the
    // next neighbour j.  Wave 0 owns the walks; their state lives in LDS.
    if (wave == 0) {
        L.FA[lane] = 1.f;
        L.PA[lane] = 1.f;
        L.V[lane] = 0.f;
        L.GXa[lane] = 1.f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) L.FB[c][lane] = L.U[c][lane] = L.GXb[c][lane] = 0.f;
        L.fj[lane] = (valid && chunk > 0) ? chunk - 1 : kWalkDone;
        L.bj[lane] = (valid && chunk + 1 < G) ? chunk + 1 : kWalkDone;
    }
    __syncthreads();
    if (valid) {
        for (int k = wave; k < CW::kWords; k += NWV) {  // a trip count set by the wave
            float v;
            bool live = true;
            if (k == CW::kA) {
                v = L.n.A[0][lane];
            } else if (k < CW::kP) {
                v = L.n.B[0][k - CW::kB][lane];
                live = k - CW::kB < ncv;
            } else if (k == CW::kP) {
                v = L.n.P[0][lane];
            } else if (k == CW::kBQ) {
                v = L.n.BQ[0][lane];
            } else {
                v = L.n.BJ[0][k - CW::kBJ][lane];
                live = k - CW::kBJ < ncv;
            }
            if (live) publish(carry_word<NCH>(a, strip_base, chunk, k, lane), ep, v);
        }
    }
    int spins = 0;
    while (true) {
        __syncthreads();
        {
            const bool fwd = wave < NH;
            const int q = fwd ? wave : wave - NH;
            const int jl = fwd ? L.fj[lane] : L.bj[lane];
            const int jq = fwd ? jl - q : jl + q;
            bool ok = false;
            if (jl != kWalkDone && jq >= 0 && jq < G) {
                unsigned long long wb[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    if (c < ncv) wb[c] = load_word(carry_word<NCH>(a, strip_base, jq, CW::kB + c, lane));
                const unsigned long long wa = load_word(carry_word<NCH>(a, strip_base, jq, CW::kA, lane));
                ok = static_cast<unsigned>(wa >> 32) == want && tags_ok<NCH>(wb, ncv, want);
                L.n.A[wave][lane] = word_value(wa);
#pragma unroll
                for (int c = 0; c < NCH; ++c) L.n.B[wave][c][lane] = (c < ncv) ? word_value(wb[c]) : 0.f;
                if (!fwd) {
                    unsigned long long wj[NCH];
#pragma unroll
                    for (int c = 0; c < NCH; ++c)
                        if (c < ncv) wj[c] = load_word(carry_word<NCH>(a, strip_base, jq, CW::kBJ + c, lane));
                    const unsigned long long wp = load_word(carry_word<NCH>(a, strip_base, jq, CW::kP, lane));
                    const unsigned long long wq = load_word(carry_word<NCH>(a, strip_base, jq, CW::kBQ, lane));
                    ok = ok && static_cast<unsigned>(wp >> 32) == want && static_cast<unsigned>(wq >> 32) == want &&
                         tags_ok<NCH>(wj, ncv, want);
                    L.n.P[wave][lane] = word_value(wp);
                    L.n.BQ[wave][lane] = word_value(wq);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) L.n.BJ[wave][c][lane] = (c < ncv) ? word_value(wj[c]) : 0.f;
                }
            }
            L.n.ok[wave][lane] = ok ? 1 : 0;
        }
        __syncthreads();
        if (wave == 0) {
            int fj = L.fj[lane], bj = L.bj[lane];
            bool fstall = false, bstall = false, progressed = false;
            if (fj != kWalkDone) {
                float FA = L.FA[lane], FB[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) FB[c] = L.FB[c][lane];
#pragma unroll
                for (int q = 0; q < NH; ++q) {
                    if (fj == kWalkDone || fstall) continue;
                    if (fj < 0 || FA < kCarryNegligible) {
                        fj = kWalkDone;
                    } else if (L.n.ok[q][lane]) {
#pragma unroll
                        for (int c = 0; c < NCH; ++c) FB[c] = fmaf(FA, L.n.B[q][c][lane], FB[c]);
                        FA *= L.n.A[q][lane];
                        --fj;
                        progressed = true;
                    } else {
                        fstall = true;
                    }
                }
                if (fj != kWalkDone && (fj < 0 || FA < kCarryNegligible)) fj = kWalkDone;
                L.FA[lane] = FA;
#pragma unroll
                for (int c = 0; c < NCH; ++c) L.FB[c][lane] = FB[c];
            }
            if (bj != kWalkDone) {
                float PA = L.PA[lane], V = L.V[lane], GXa = L.GXa[lane], U[NCH], GXb[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    U[c] = L.U[c][lane];
                    GXb[c] = L.GXb[c][lane];
                }
#pragma unroll
                for (int q = NH; q < NWV; ++q) {
                    if (bj == kWalkDone || bstall) continue;
                    if (bj >= G || PA < kCarryNegligible) {
                        bj = kWalkDone;
                    } else if (L.n.ok[q][lane]) {
                        const float bq = L.n.BQ[q][lane], aj = L.n.A[q][lane];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            U[c] = fmaf(PA, fmaf(bq, GXb[c], L.n.BJ[q][c][lane]), U[c]);
                            GXb[c] = fmaf(aj, GXb[c], L.n.B[q][c][lane]);
                        }
                        V = fmaf(PA, bq * GXa, V);
                        GXa *= aj;
                        PA *= L.n.P[q][lane];
                        ++bj;
                        progressed = true;
                    } else {
                        bstall = true;
                    }
                }
                if (bj != kWalkDone && (bj >= G || PA < kCarryNegligible)) bj = kWalkDone;
                L.PA[lane] = PA;
                L.V[lane] = V;
                L.GXa[lane] = GXa;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    L.U[c][lane] = U[c];
                    L.GXb[c][lane] = GXb[c];
                }
            }
            if (progressed) spins = 0;
            if (fstall || bstall) {
                // Wait for the blocking neighbour gently: poll only its first word,
                // sleeping longer and longer between polls, and stage the next round trip
                // once it has been written.
                gword* pw = carry_word<NCH>(a, strip_base, fstall ? fj : bj, CW::kA, lane);
                int backoff = 1;
                while (true) {
                    if (static_cast<unsigned>(load_word(pw) >> 32) == want) break;
                    spins += backoff;
                    if (spins > a.spin_limit) break;
                    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(2);
                    backoff = backoff < 32 ? backoff * 2 : 32;
                }
                if (spins > a.spin_limit) {
                    flag_error(a.status, kErrSpinTimeout);
                    fj = bj = kWalkDone;
                }
            }
            L.fj[lane] = fj;
            L.bj[lane] = bj;
            const bool any = __ballot(fj != kWalkDone || bj != kWalkDone) != 0;
            if (lane == 0) L.more = any ? 1 : 0;
        }
        __syncthreads();
        if (L.more == 0) break;
    }

    if (wave == 0) {
        // forward carry into every wave, then the backward carry from the bottom wave up
        float xe[NCH], kv[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) xe[c] = L.FB[c][lane];
#pragma unroll
        for (int v = 0; v < NWV; ++v) {
            const float Av = L.A[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                L.Jin[v][c][lane] = xe[c];
                xe[c] = fmaf(Av, xe[c], L.B[v][c][lane]);
            }
        }
        // xe is now X_in of the next chunk
#pragma unroll
        for (int c = 0; c < NCH; ++c) kv[c] = fmaf(L.V[lane], xe[c], L.U[c][lane]);
#pragma unroll
        for (int v = NWV - 1; v >= 0; --v) {
            const float Pv = L.P[v][lane], BQv = L.BQ[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                L.Kin[v][c][lane] = kv[c];
                kv[c] = fmaf(Pv, kv[c], fmaf(BQv, L.Jin[v][c][lane], L.BJ[v][c][lane]));
            }
        }
    }
}

// Chunk and strip group of workgroup p in a persistent column grid with G chunks per
// strip.  With `xcd` set, strip groups are dealt to the XCDs in turn and all G chunks of a
// group run on that group's XCD (workgroup p runs on XCD p % 8), so the carry words a
// chunk polls were written by workgroups of its own XCD; otherwise workgroup p takes
// chunk p % G of group p / G.  Groups at or past the launch's group count have no work.
struct ChunkSlot {
    int chunk, group;
};
__device__ __forceinline__ ChunkSlot chunk_slot(int p, int G, int xcd) {
    if (xcd) {
        const int k = p / kXcds;
        return ChunkSlot{k % G, (k / G) * kXcds + p % kXcds};
    }
    return ChunkSlot{p % G, p / G};
}

// Words of carry area per (strip, chunk) for NCH channels, for workspace sizing.
constexpr int carry_words_per_chunk(int nch) { return 3 + 2 * nch; }

}  // namespace dts
