// Internal (non-ABI) interface between the libdts entry points and its kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dts {

// Per-call launch context: the stream, the workspace's device status word and the
// carry-word area of the column passes.  The host counts epochs so every column-pass
// launch of one call tags its carry words with a fresh epoch.
struct Ctx {
    hipStream_t stream = nullptr;
    int* status = nullptr;
    unsigned long long* carry = nullptr;
    size_t carry_words = 0;
    unsigned epoch = 0;
};

// One pass along rows (fused distance computation when `guide` is non-null).
struct RowPass {
    const float* src;
    float* dst;
    const float* d;   // dx [batch][H][W]; ignored when computing distances
    const float* guide;
    float* dx_out;
    float* dy_out;
    int Cg;
    float s2;         // (sigma_s / sigma_r)^2
    int C, H, W, batch;  // C: output channels
    float log2a;
    int sq;               // 1: the first pass of a variance: src holds C / 2 channels, see RowArgs
};

// One pass along columns (optional update epilogue of the solver).
struct ColPass {
    const float* src;
    float* dst;
    const float* d;   // dy [batch][H][W]
    int C, H, W, batch;
    float log2a;
    // epilogue: dst = z - step (lambda (z - K) + c (z - t)), also written to dst2 if set;
    // with data_grad (single-channel signals only): dst = z - step (lambda (z - K) + D),
    // D read from tgt
    bool epilogue;
    bool data_grad;
    const float* zk;
    const float* tgt;
    const float* conf;
    int Cc;
    float* dst2;
    float lambda, step;
    // variance (C even, in place of the epilogue): dst = exp2(var_k (K_{2c+1} - K_{2c}^2)),
    // the confidence of Eq. (7) from the filtered pairs (DT(z), DT(z^2)), C / 2 planes
    bool variance;
    float var_k;
};

// Adjoint of one row pass (update-adjoint epilogue when gz is set).
struct RowAdj {
    const float* gk;
    float gk_scale;
    const float* f;
    const float* d;
    float* gout;
    float* gd;
    int C, H, W, batch;
    float log2a;
    float* gz;
    const float* tgt;
    const float* conf;
    float* gt;
    float* gc;
    int Cc;
    float lambda, step;
    int last;
};

// Adjoint of one column pass.
struct ColAdj {
    const float* gk;
    float gk_scale;
    const float* f;
    const float* d;
    float* gout;
    float* gd;
    int C, H, W, batch;
    float log2a;
};

// Guide gradient from the distance gradients.
struct DistAdj {
    const float* guide;
    const float* dx;
    const float* dy;
    const float* gdx;
    const float* gdy;
    int ngy;
    float* gg;
    int Cg, H, W, batch;
    float s2;
};

int launch_row_adjoint(const RowAdj& p, Ctx& ctx);
int launch_col_adjoint(const ColAdj& p, Ctx& ctx);
int launch_dist_adjoint(const DistAdj& p, Ctx& ctx);
int col_adjoint_groups(int C);
size_t col_adjoint_carry_words(int batch, int H, int W, int C);

int launch_row_pass(const RowPass& p, Ctx& ctx);
int launch_col_pass(const ColPass& p, Ctx& ctx);
size_t col_carry_words(int batch, int H, int W, int C);
int tune_col_variant(int ct, int variant);
int col_variant_info(int variant, int* ct, int* rows_per_wave, int* waves);
int num_col_variants();
int num_batch_variants();
int batch_variant_info(int v, int* rows_per_wave, int* group_channels, int* row_tile_pixels);
int tune_row_segment(int S);
int launch_zero(void* ptr, size_t bytes, hipStream_t s);
int launch_stereo_data_grad(const float* z, const float* t, const float* c, const float* left, const float* right,
                            float* D, int Cg, int batch, int H, int W, float gamma, float eps, hipStream_t s);
float variance_k(float sigma_c);
int launch_copy(float* dst, const float* src, size_t n, hipStream_t s);
constexpr int kBoxMaxIters = 8;
int box_check_radius(int h1);
int launch_box_codes(const float* guide, int Cg, int batch, int H, int W, float s2, unsigned* qx, unsigned* qy,
                     hipStream_t s);
int launch_box_bounds(unsigned* qx, const unsigned* qy, unsigned short* bx, unsigned short* by, unsigned short* bt,
                      int batch, int H, int W, const unsigned* R, int iters, hipStream_t s);
int launch_box_row(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W, int h,
                   hipStream_t s);
int launch_box_col_prefixed(const float* src, float* P, float* dst, const unsigned short* bounds, int C, int batch,
                            int H, int W, hipStream_t s);
int launch_box_col(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W, int h,
                   const float* zk, const float* tgt, const float* conf, int Cc, float lambda, float step,
                   hipStream_t s);
// One-kernel column pass over a window of rows in LDS, for half-widths up to a limit
// (box_window_fits); wider boxes take launch_box_col / launch_box_col_prefixed.  Writes a
// buffer other than the one it reads.
bool box_window_fits(int h);
int tune_box_window(int on);
int launch_box_col_window(const float* src, float* dst, const unsigned short* bounds, int C, int batch, int H, int W,
                          int h, const float* zk, const float* tgt, const float* conf, int Cc, float lambda,
                          float step, hipStream_t s);
size_t support_carry_words(int batch, int H, int W);
int launch_support_row(const float* src, const float* dx, float* dst, int batch, int H, int W, float log2a,
                       float m, hipStream_t s);
int launch_support_col(const float* src, const float* dy, float* dst, const float* conf, int Cc, float* conf_out,
                       int batch, int H, int W, float log2a, float m, Ctx& ctx);

// RAII launch timer: records a start event on construction and a stop event on
// destruction (both on `s`) when timing is enabled; a no-op otherwise.
class ProfScope {
   public:
    ProfScope(const char* name, double bytes, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

   private:
    hipStream_t stream_;
    long index_ = -1;
};

// Grid of a persistent column pass: `groups` strips in flight, `n` workgroups, and
// whether the chunks of each strip are kept on one XCD (see chunk_slot).  `cap` is the
// kernel's co-resident workgroup capacity, G the chunks per strip.
struct ColGrid {
    int groups;
    unsigned n;
    int xcd;
};
ColGrid col_grid(int cap, int G, long long n_strips);
int tune_col_xcd(int on);
// Bounded waits of the carry exchange (see dts_tune_spin_limit).
int tune_spin_limit(int polls);
int spin_limit();
unsigned spin_tag_xor();

// Error bookkeeping shared by the translation units.
int hip_fail(hipError_t e);

}  // namespace dts
