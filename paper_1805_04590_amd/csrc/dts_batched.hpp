// Device-side tables of the persistent batched solve (host fills them in the workspace).
#pragma once

namespace dts {

constexpr int kBatchMaxN = 8;          // filter iterations per instance
constexpr int kBatchWaves = 4;         // waves per workgroup of the batched kernel
constexpr int kBatchSoloWidth = 64 * 16;              // widest row one wave filters alone
constexpr int kBatchMaxWidth = kBatchWaves * kBatchSoloWidth;
constexpr int kBatchWideS = 32;  // row_S code of the two-section rows
constexpr int kBatchMaxProblems = 1024;

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
    int row_S;       // pixels per lane of a row: 8 or 16, or kBatchWideS for rows of one
                     // wave in two sections of kBatchSoloWidth pixels (16 per lane each)
    int row_gw;      // waves per row (1 or kBatchWaves); kBatchWaves / row_gw rows side by side
    int row_rows;    // rows per row tile (a multiple of kBatchWaves / row_gw)
    int dist_rows;   // rows per tile of the distance phase
    int G, S, NG;    // column chunks per strip, strips, channel groups
    float s2;
    float log2a[kBatchMaxN];
};

struct BatchArgs {
    const BInst* inst;
    const int* phase_prefix;  // [n_phases][n + 1] first tile of each instance in a phase
    unsigned* tickets;        // [n_phases] tile counters, zeroed by the reset kernel
    unsigned* barrier;        // barrier counters: groups, then workgroups per group (cumulative)
    const unsigned* launch;   // launch counter (epoch base of the carry words)
    int* status;
    int n, n_phases;
    float lambda, step;
    int spin_limit;
    unsigned tag_xor;
};

}  // namespace dts
