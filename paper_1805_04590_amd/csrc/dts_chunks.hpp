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
// where X_in is X at the row above the chunk and Y_in is Y at the row below it.  The
// chunks of a strip exchange these through tagged 64-bit words in device memory: first a
// look-back resolves X_in from earlier chunks, then a look-ahead resolves Y_in from later
// chunks; every wave of the workgroup reads one neighbour per round trip.  Within a
// workgroup the same algebra composes the waves through LDS.
#pragma once

#include "dts_device.hpp"

namespace dts {

struct CarryCtx {
    unsigned long long* carry;  // carry words of this launch's strips
    unsigned epoch;             // tag of this launch
    int* status;                // device-side status word
    int G, S, NG;               // chunks per strip, strips per plane, channel groups
};

template <int NCH>
struct CarryWords {
    static constexpr int kFwdA = 0;                  // product of the chunk's weights
    static constexpr int kFwdB = 1;                  // + c: forward output, zero carry-in
    static constexpr int kFwdIncl = 1 + NCH;         // + c: forward output at the chunk end
    static constexpr int kBwdP = 1 + 2 * NCH;        // backward carry factor
    static constexpr int kBwdAlpha = 2 + 2 * NCH;    // + c: backward output, zero carry-in
    static constexpr int kBwdIncl = 2 + 3 * NCH;     // + c: backward output at chunk start
    static constexpr int kWords = 2 + 4 * NCH;
};

template <int NCH>
__device__ __forceinline__ gword* carry_word(const CarryCtx& a, size_t strip_base, int j, int k, int col) {
    return global_word(a.carry + ((strip_base + j) * CarryWords<NCH>::kWords + k) * kWave + col);
}

// Per-wave aggregates of one chunk (written by every wave), the carries into every wave
// (written by wave 0 after the exchange), one column per lane, and the staging area of
// the look-back / look-ahead: in each round trip wave v reads the words of the v-th
// neighbour still to be composed and leaves here what it found.
template <int NCH, int NWV>
struct ChunkLds {
    float A[NWV][kWave], P[NWV][kWave], BQ[NWV][kWave];
    float B[NWV][NCH][kWave], BJ[NWV][NCH][kWave];
    float Jin[NWV][NCH][kWave];
    union {                      // Kin is written only once both walks are over
        float Kin[NWV][NCH][kWave];
        float nV[NWV][NCH][kWave];  // neighbour's inclusive value if nS == 2, else its aggregate offset
    };
    float nA[NWV][kWave];        // neighbour's aggregate factor
    int nS[NWV][kWave];          // 2 inclusive written, 1 aggregate written, 0 neither yet
    int nJ[kWave];               // per lane: the next neighbour to read, or kWalkDone
    int more;                    // some lane of wave 0 is still walking
};

constexpr int kWalkDone = -0x40000000;

// Resolve one chunk's carry from its neighbours, one column per lane, with all NWV waves
// of the workgroup (every wave must call it; the result is valid in wave 0).  Going away
// from the chunk (towards chunk 0 for the forward carry, towards the last chunk for the
// backward one), each neighbour j contributes either its inclusive value (which ends the
// walk) or its affine aggregate x -> A x + B (composed in, walk on).  One round trip reads
// NWV neighbours, one per wave, and wave 0 composes them in order.  Lanes with `live`
// false (columns past the right edge) take no part.
template <int NCH, int NWV>
__device__ void resolve_carry(const CarryCtx& a, ChunkLds<NCH, NWV>& L, size_t strip_base, int col,
                              int wave, int chunk, int dir, int wA, int wB, int wIncl, int ncv,
                              bool live, float (&carry)[NCH]) {
    const unsigned ep = a.epoch;
    const int G = a.G;
    float GA = 1.f, GB[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) GB[c] = carry[c] = 0.f;
    int j = chunk + dir;           // wave 0: next neighbour of this lane
    bool done = !live;
    int spins = 0;
    while (true) {
        if (wave == 0) L.nJ[col] = done ? kWalkDone : j;
        __syncthreads();
        {
            const int jl = L.nJ[col];
            const int jq = jl + wave * dir;
            int st = 0;
            if (jl != kWalkDone && jq >= 0 && jq < G) {
                unsigned long long wi[NCH], wb[NCH];
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    if (c < ncv) {
                        wi[c] = __hip_atomic_load(carry_word<NCH>(a, strip_base, jq, wIncl + c, col),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        wb[c] = __hip_atomic_load(carry_word<NCH>(a, strip_base, jq, wB + c, col),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                const unsigned long long wa = __hip_atomic_load(
                    carry_word<NCH>(a, strip_base, jq, wA, col), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool inc_ok = true, agg_ok = static_cast<unsigned>(wa >> 32) == ep;
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    if (c < ncv) {
                        inc_ok = inc_ok && static_cast<unsigned>(wi[c] >> 32) == ep;
                        agg_ok = agg_ok && static_cast<unsigned>(wb[c] >> 32) == ep;
                    }
                st = inc_ok ? 2 : agg_ok ? 1 : 0;
                L.nA[wave][col] = __uint_as_float(static_cast<unsigned>(wa));
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    L.nV[wave][c][col] =
                        (c < ncv) ? __uint_as_float(static_cast<unsigned>(inc_ok ? wi[c] : wb[c])) : 0.f;
            }
            L.nS[wave][col] = st;
        }
        __syncthreads();
        if (wave == 0) {
            bool stalled = false;
#pragma unroll
            for (int q = 0; q < NWV; ++q) {
                if (done || stalled) continue;
                if (j < 0 || j >= G) {  // walked past the first / last chunk: the aggregate is exact
#pragma unroll
                    for (int c = 0; c < NCH; ++c) carry[c] = GB[c];
                    done = true;
                    continue;
                }
                const int st = L.nS[q][col];
                if (st == 2) {
#pragma unroll
                    for (int c = 0; c < NCH; ++c) carry[c] = fmaf(GA, L.nV[q][c][col], GB[c]);
                    done = true;
                } else if (st == 1) {
#pragma unroll
                    for (int c = 0; c < NCH; ++c) GB[c] = fmaf(GA, L.nV[q][c][col], GB[c]);
                    GA *= L.nA[q][col];
                    j += dir;
                } else {
                    stalled = true;
                }
            }
            if (!done && (j < 0 || j >= G)) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) carry[c] = GB[c];
                done = true;
            }
            if (!done && stalled) {
                // Wait for the blocking neighbour j gently: poll only its first inclusive
                // word and its aggregate factor, sleeping longer and longer between polls,
                // and stage the next round trip only once one of them has been written.
                gword* pi0 = carry_word<NCH>(a, strip_base, j, wIncl, col);
                gword* pa0 = carry_word<NCH>(a, strip_base, j, wA, col);
                int backoff = 1;
                while (true) {
                    const unsigned long long u =
                        __hip_atomic_load(pi0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned long long v =
                        __hip_atomic_load(pa0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (static_cast<unsigned>(u >> 32) == ep || static_cast<unsigned>(v >> 32) == ep) break;
                    spins += backoff;
                    if (spins > kSpinLimit) break;
                    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(2);
                    backoff = backoff < 32 ? backoff * 2 : 32;
                }
                if (spins > kSpinLimit) {
                    flag_error(a.status, kErrSpinTimeout);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) carry[c] = GB[c];
                    done = true;
                }
            } else if (!stalled) {
                spins = 0;
            }
            const bool any = __ballot(!done) != 0;
            if (col == 0) L.more = any ? 1 : 0;
        }
        __syncthreads();
        if (L.more == 0) break;
    }
}

// All waves of a chunk's workgroup: wave 0 composes the waves into the chunk aggregates
// and publishes them, all waves take part in the exchange of carries with the other
// chunks of the strip, and wave 0 writes every wave's carry-in X_in (L.Jin) and Y_in
// (L.Kin).  `ncv` channels are valid; `valid` is false for lanes past the right edge of
// the image.
template <int NCH, int NWV>
__device__ void chunk_carries(const CarryCtx& a, ChunkLds<NCH, NWV>& L, int b, int grp, int strip,
                              int chunk, int lane, int wave, bool valid, int ncv) {
    using CW = CarryWords<NCH>;
    const size_t strip_base =
        ((static_cast<size_t>(b) * a.NG + grp) * a.S + strip) * static_cast<size_t>(a.G);
    const unsigned ep = a.epoch;
    // chunk-level forward aggregate: compose the waves in order
    float CA = 1.f, CB[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) CB[c] = 0.f;
    if (wave == 0) {
#pragma unroll
        for (int v = 0; v < NWV; ++v) {
            const float Av = L.A[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) CB[c] = fmaf(Av, CB[c], L.B[v][c][lane]);
            CA *= Av;
        }
        if (chunk > 0 && valid) {
            publish(carry_word<NCH>(a, strip_base, chunk, CW::kFwdA, lane), ep, CA);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c < ncv) publish(carry_word<NCH>(a, strip_base, chunk, CW::kFwdB + c, lane), ep, CB[c]);
        }
    }
    float Jc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) Jc[c] = 0.f;
    if (chunk > 0)
        resolve_carry<NCH, NWV>(a, L, strip_base, lane, wave, chunk, -1, CW::kFwdA, CW::kFwdB, CW::kFwdIncl,
                                ncv, valid, Jc);
    float CP = 1.f, alpha[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) alpha[c] = 0.f;
    if (wave == 0) {
        if (valid) {
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c < ncv)
                    publish(carry_word<NCH>(a, strip_base, chunk, CW::kFwdIncl + c, lane), ep,
                            fmaf(CA, Jc[c], CB[c]));
        }
        // forward carry into every wave, and the chunk-level backward aggregate
        float jv[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) jv[c] = Jc[c];
#pragma unroll
        for (int v = 0; v < NWV; ++v) {
            const float Av = L.A[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                L.Jin[v][c][lane] = jv[c];
                jv[c] = fmaf(Av, jv[c], L.B[v][c][lane]);
            }
        }
#pragma unroll
        for (int v = NWV - 1; v >= 0; --v) {
            const float Pv = L.P[v][lane], BQv = L.BQ[v][lane];
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                alpha[c] = fmaf(Pv, alpha[c], fmaf(BQv, L.Jin[v][c][lane], L.BJ[v][c][lane]));
            CP *= Pv;
        }
        if (chunk < a.G - 1 && valid) {
            publish(carry_word<NCH>(a, strip_base, chunk, CW::kBwdP, lane), ep, CP);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c < ncv)
                    publish(carry_word<NCH>(a, strip_base, chunk, CW::kBwdAlpha + c, lane), ep, alpha[c]);
        }
    }
    float Kc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) Kc[c] = 0.f;
    if (chunk < a.G - 1)
        resolve_carry<NCH, NWV>(a, L, strip_base, lane, wave, chunk, +1, CW::kBwdP, CW::kBwdAlpha,
                                CW::kBwdIncl, ncv, valid, Kc);
    if (wave == 0) {
        if (valid) {
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c < ncv)
                    publish(carry_word<NCH>(a, strip_base, chunk, CW::kBwdIncl + c, lane), ep,
                            fmaf(CP, Kc[c], alpha[c]));
        }
        // backward carry into every wave (Y at the row after the wave's last row)
        float kv[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) kv[c] = Kc[c];
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

// Words of carry area per (strip, chunk) for NCH channels, for workspace sizing.
constexpr int carry_words_per_chunk(int nch) { return 2 + 4 * nch; }

}  // namespace dts
