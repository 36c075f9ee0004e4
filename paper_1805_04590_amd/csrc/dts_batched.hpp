// Device-side tables of the persistent batched solve (host fills them in the workspace).
#pragma once

namespace dts {

constexpr int kBatchMaxN = 8;        // filter iterations per instance
constexpr int kBatchWaves = 8;       // waves per workgroup of the batched kernel
constexpr int kBatchMaxWidth = kBatchWaves * 64 * 16;

struct BInst {
    const float* guide;
    const float* target;
    const float* conf;
    float* out;
    float* dx;
    float* dy;
    float* tmp;
    unsigned long long* carry;
    int H, W, Cg, Ct, Cc, N, T;
    int row_S;       // pixels per lane of the row tiles
    int G, S, NG;    // column chunks per strip, strips, channel groups
    float s2;
    float log2a[kBatchMaxN];
};

struct BatchArgs {
    const BInst* inst;
    const int* phase_base;    // [n_phases + 1] first ticket of each phase
    const int* phase_prefix;  // [n_phases][n + 1] first tile of each instance in a phase
    const int* need;          // [n_phases][n] tiles of the instance done before the phase
    unsigned* done;           // [n] completed tiles per instance
    unsigned* ticket;
    const unsigned* launch;   // launch counter (epoch base of the carry words)
    int* status;
    int n, n_phases, total;
    float lambda, step;
};

}  // namespace dts
