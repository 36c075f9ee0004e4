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
// chunks.  Within a workgroup the same algebra composes the waves through LDS.
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
__device__ __forceinline__ unsigned long long* carry_word(const CarryCtx& a, size_t strip_base, int j,
                                                          int k, int col) {
    return a.carry + ((strip_base + j) * CarryWords<NCH>::kWords + k) * kWave + col;
}

// Look-back and look-ahead read this many neighbouring chunks per round trip.
constexpr int kLookBatch = 4;

// Resolve one chunk's carry from its neighbours (run by one wave, one column per lane).
// Going away from the chunk (towards chunk 0 for the forward carry, towards the last
// chunk for the backward one), each neighbour j contributes either its inclusive value
// (which ends the walk) or its affine aggregate x -> A x + B (composed in, walk on).
template <int NCH>
__device__ void resolve_carry(const CarryCtx& a, size_t strip_base, int col, int chunk, int dir,
                              int wA, int wB, int wIncl, int ncv, float (&carry)[NCH]) {
    const unsigned ep = a.epoch;
    float GA = 1.f, GB[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) GB[c] = 0.f;
    int j = chunk + dir;
    int spins = 0;
    const int G = a.G;
    while (true) {
        unsigned long long wi[kLookBatch][NCH], wa[kLookBatch], wb[kLookBatch][NCH];
#pragma unroll
        for (int q = 0; q < kLookBatch; ++q) {
            const int jq = j + q * dir;
            if (jq >= 0 && jq < G) {
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    if (c < ncv) {
                        wi[q][c] = __hip_atomic_load(carry_word<NCH>(a, strip_base, jq, wIncl + c, col),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        wb[q][c] = __hip_atomic_load(carry_word<NCH>(a, strip_base, jq, wB + c, col),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                wa[q] = __hip_atomic_load(carry_word<NCH>(a, strip_base, jq, wA, col), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        bool done = false, stalled = false;
#pragma unroll
        for (int q = 0; q < kLookBatch; ++q) {
            if (done || stalled || j < 0 || j >= G) continue;
            bool inc_ok = true, agg_ok = static_cast<unsigned>(wa[q] >> 32) == ep;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (c < ncv) {
                    inc_ok = inc_ok && static_cast<unsigned>(wi[q][c] >> 32) == ep;
                    agg_ok = agg_ok && static_cast<unsigned>(wb[q][c] >> 32) == ep;
                }
            if (inc_ok) {
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    carry[c] = fmaf(GA, (c < ncv) ? __uint_as_float(static_cast<unsigned>(wi[q][c])) : 0.f, GB[c]);
                done = true;
            } else if (agg_ok) {
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    GB[c] = fmaf(GA, (c < ncv) ? __uint_as_float(static_cast<unsigned>(wb[q][c])) : 0.f, GB[c]);
                GA *= __uint_as_float(static_cast<unsigned>(wa[q]));
                j += dir;
            } else {
                stalled = true;
            }
        }
        if (done) break;
        if (j < 0 || j >= G) {  // walked past the first / last chunk: the aggregate is exact
#pragma unroll
            for (int c = 0; c < NCH; ++c) carry[c] = GB[c];
            break;
        }
        if (stalled) {
            // Wait for the blocking neighbour j gently: poll only its first inclusive word
            // and its aggregate factor, sleeping longer and longer between polls, and
            // re-read the whole batch only once one of them has been written.
            unsigned long long* pi0 = carry_word<NCH>(a, strip_base, j, wIncl, col);
            unsigned long long* pa0 = carry_word<NCH>(a, strip_base, j, wA, col);
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
                break;
            }
        } else {
            spins = 0;
        }
    }
}

// Per-wave aggregates of one chunk (written by every wave) and the carries into every
// wave (written by wave 0 after the exchange), one column per lane.
template <int NCH, int NWV>
struct ChunkLds {
    float A[NWV][kWave], P[NWV][kWave], BQ[NWV][kWave];
    float B[NWV][NCH][kWave], BJ[NWV][NCH][kWave];
    float Jin[NWV][NCH][kWave], Kin[NWV][NCH][kWave];
};

// Wave 0 of a chunk's workgroup: compose the waves into the chunk aggregate, exchange
// carries with the other chunks of the strip, and write every wave's carry-in X_in
// (L.Jin) and Y_in (L.Kin).  `ncv` channels are valid; `valid` is false for lanes past
// the right edge of the image.
template <int NCH, int NWV>
__device__ void chunk_carries(const CarryCtx& a, ChunkLds<NCH, NWV>& L, int b, int grp, int strip,
                              int chunk, int lane, bool valid, int ncv) {
    using CW = CarryWords<NCH>;
    const size_t strip_base =
        ((static_cast<size_t>(b) * a.NG + grp) * a.S + strip) * static_cast<size_t>(a.G);
    const unsigned ep = a.epoch;
    // chunk-level forward aggregate: compose the waves in order
    float CA = 1.f, CB[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) CB[c] = 0.f;
#pragma unroll
    for (int v = 0; v < NWV; ++v) {
        const float Av = L.A[v][lane];
#pragma unroll
        for (int c = 0; c < NCH; ++c) CB[c] = fmaf(Av, CB[c], L.B[v][c][lane]);
        CA *= Av;
    }
    float Jc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) Jc[c] = 0.f;
    if (chunk > 0 && valid) {
        publish(carry_word<NCH>(a, strip_base, chunk, CW::kFwdA, lane), ep, CA);
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c < ncv) publish(carry_word<NCH>(a, strip_base, chunk, CW::kFwdB + c, lane), ep, CB[c]);
        resolve_carry<NCH>(a, strip_base, lane, chunk, -1, CW::kFwdA, CW::kFwdB, CW::kFwdIncl, ncv, Jc);
    }
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
    float CP = 1.f, alpha[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) alpha[c] = 0.f;
#pragma unroll
    for (int v = NWV - 1; v >= 0; --v) {
        const float Pv = L.P[v][lane], BQv = L.BQ[v][lane];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            alpha[c] = fmaf(Pv, alpha[c], fmaf(BQv, L.Jin[v][c][lane], L.BJ[v][c][lane]));
        CP *= Pv;
    }
    float Kc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) Kc[c] = 0.f;
    if (chunk < a.G - 1 && valid) {
        publish(carry_word<NCH>(a, strip_base, chunk, CW::kBwdP, lane), ep, CP);
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c < ncv) publish(carry_word<NCH>(a, strip_base, chunk, CW::kBwdAlpha + c, lane), ep, alpha[c]);
        resolve_carry<NCH>(a, strip_base, lane, chunk, +1, CW::kBwdP, CW::kBwdAlpha, CW::kBwdIncl, ncv, Kc);
    }
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

// Words of carry area per (strip, chunk) for NCH channels, for workspace sizing.
constexpr int carry_words_per_chunk(int nch) { return 2 + 4 * nch; }

}  // namespace dts
