// libdts C ABI: argument checks, workspace layout and pass orchestration.
//
// Method: Bapat & Frahm, "The Domain Transform Solver", ECCV 2018.  dts_filter is the
// edge-aware mean of Sec. 3.2 (the recursive domain-transform filter: distances of
// Eq. (8)-(9), weights a^d, rows then columns per iteration); dts_solve is gradient
// descent along the Eq. (3) direction on the objective of Eq. (2), starting from the
// target (Sec. 3.1), with the hyper-parameters of Sec. 4 as defaults on the Python side.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "../../include/dts.h"
#include "dts_device.hpp"
#include "dts_internal.hpp"

namespace dts {

static thread_local char g_last_hip[256] = "no HIP error";

int hip_fail(hipError_t e) {
    if (e == hipSuccess) return DTS_OK;
    snprintf(g_last_hip, sizeof(g_last_hip), "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
    return DTS_EHIP;
}

constexpr size_t kAlign = 256;
constexpr size_t kHeaderBytes = 256;
constexpr int kMaxFilterIters = 64;
constexpr long long kMaxSolverIters = 1 << 20;

static size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace: [header | dx | dy | tmp (solve only) | carry words]
struct Layout {
    size_t dx = 0, dy = 0, tmp = 0, carry = 0, carry_bytes = 0, total = 0;
};

static Layout make_layout(int batch, int H, int W, int C, bool with_tmp) {
    Layout L;
    const size_t plane = static_cast<size_t>(batch) * H * W * sizeof(float);
    size_t off = kHeaderBytes;
    L.dx = off;
    off = align_up(off + plane);
    L.dy = off;
    off = align_up(off + plane);
    if (with_tmp) {
        L.tmp = off;
        off = align_up(off + plane * C);
    }
    L.carry = off;
    L.carry_bytes = align_up(col_carry_words(batch, H, W, C) * sizeof(unsigned long long));
    off += L.carry_bytes;
    L.total = off;
    return L;
}

// Backward workspace: [header | dx | dy | gdx | gdy (one plane set per adjoint channel
// group) | tape of the 2N-1 pass inputs after the first | gz | ga | gb | carry words]
struct BwdLayout {
    size_t dx, dy, gdx, gdy, tape, gz, ga, gb, carry, carry_bytes, total;
    int ngy;
};

static BwdLayout make_backward_layout(int batch, int H, int W, int Ct, int N) {
    BwdLayout L;
    const size_t plane = static_cast<size_t>(batch) * H * W * sizeof(float);
    const size_t sig = plane * Ct;
    L.ngy = col_adjoint_groups(Ct);
    size_t off = kHeaderBytes;
    L.dx = off;
    off = align_up(off + plane);
    L.dy = off;
    off = align_up(off + plane);
    L.gdx = off;
    off = align_up(off + plane);
    L.gdy = off;
    off = align_up(off + plane * L.ngy);
    L.tape = off;
    off = align_up(off + sig * (2 * N - 1));
    L.gz = off;
    off = align_up(off + sig);
    L.ga = off;
    off = align_up(off + sig);
    L.gb = off;
    off = align_up(off + sig);
    L.carry = off;
    const size_t words = std::max(col_carry_words(batch, H, W, Ct), col_adjoint_carry_words(batch, H, W, Ct));
    L.carry_bytes = align_up(words * sizeof(unsigned long long));
    off += L.carry_bytes;
    L.total = off;
    return L;
}

static bool finite_pos(float v) { return isfinite(v) && v > 0.f; }

static int check_shape(int batch, int H, int W) {
    if (batch < 1 || H < 1 || W < 1) return DTS_EINVAL;
    if (H > DTS_MAX_HEIGHT || W > DTS_MAX_WIDTH) return DTS_ENOTSUP;
    // column passes address a plane through one buffer resource with 32-bit offsets and
    // mask lanes by pushing their offset past 2^31: keep every plane offset below 2^31
    if ((static_cast<size_t>(H) + 64) * static_cast<size_t>(W) * 4 >= (static_cast<size_t>(1) << 31))
        return DTS_ENOTSUP;
    return DTS_OK;
}

static int check_channels(int C) { return (C >= 1 && C <= DTS_MAX_CHANNELS) ? DTS_OK : DTS_EINVAL; }

// log2 of the feedback coefficient of filter iteration i (1-based) of N:
// a_i = exp(-sqrt(2)/sigma_Hi), sigma_Hi = sigma_s sqrt(3) 2^(N-i) / sqrt(4^N - 1).
static float log2_feedback(double sigma_s, int i, int N) {
    const double sigma_h = sigma_s * sqrt(3.0) * ldexp(1.0, N - i) / sqrt(ldexp(1.0, 2 * N) - 1.0);
    return static_cast<float>(-sqrt(2.0) / sigma_h / log(2.0));
}

// a_i itself, in double
static double feedback(double sigma_s, int i, int N) {
    const double sigma_h = sigma_s * sqrt(3.0) * ldexp(1.0, N - i) / sqrt(ldexp(1.0, 2 * N) - 1.0);
    return exp(-sqrt(2.0) / sigma_h);
}

// Support workspace: [header | dx | dy | tmp | chunk aggregates (float4) | carries (float2)]
struct SupportLayout {
    size_t dx, dy, tmp, carry, carry_bytes, total;
};

static SupportLayout make_support_layout(int batch, int H, int W) {
    SupportLayout L;
    const size_t plane = static_cast<size_t>(batch) * H * W * sizeof(float);
    size_t off = kHeaderBytes;
    L.dx = off;
    off = align_up(off + plane);
    L.dy = off;
    off = align_up(off + plane);
    L.tmp = off;
    off = align_up(off + plane);
    L.carry = off;
    L.carry_bytes = align_up(support_carry_words(batch, H, W) * sizeof(unsigned long long));
    off += L.carry_bytes;
    L.total = off;
    return L;
}

// Box workspace: [header | qx | qy (u32 codes) | bx | by | bt (u16 bounds, one plane per
// iteration; bt holds the transposed column bounds) | t1 | t2 (C planes each)]
struct BoxLayout {
    size_t qx, qy, bx, by, bt, t1, t2, total;
};

static BoxLayout make_box_layout(int batch, int H, int W, int C, int N) {
    BoxLayout L;
    const size_t px = static_cast<size_t>(batch) * H * W;
    size_t off = kHeaderBytes;
    L.qx = off;
    off = align_up(off + px * 4);
    L.qy = off;
    off = align_up(off + px * 4);
    L.bx = off;
    off = align_up(off + px * 2 * N);
    L.by = off;
    off = align_up(off + px * 2 * N);
    L.bt = off;
    off = align_up(off + px * 2 * N);
    L.t1 = off;
    off = align_up(off + px * 4 * C);
    L.t2 = off;
    off = align_up(off + px * 4 * C);
    L.total = off;
    return L;
}

// Box radii in units of 1/256 pixel: R_i = floor(256 sqrt(3) sigma_Hi), the box with the
// variance of the recursive filter's iteration i.
static int box_radii(double sigma_s, int N, unsigned* R) {
    for (int i = 1; i <= N; ++i) {
        const double sigma_h = sigma_s * sqrt(3.0) * ldexp(1.0, N - i) / sqrt(ldexp(1.0, 2 * N) - 1.0);
        const double r = floor(sigma_h * sqrt(3.0) * 256.0);
        if (!(r < 65536.0)) return DTS_ENOTSUP;  // the box offsets are stored in one byte
        R[i - 1] = static_cast<unsigned>(r);
    }
    return box_check_radius(static_cast<int>(R[0] >> 8));
}

static float box_s2(float sigma_s, float sigma_r) {
    const double q = static_cast<double>(sigma_s) / static_cast<double>(sigma_r);
    return static_cast<float>(q * q);
}

// Codes and bounds of one call, then N (row, column) passes from src; the last column
// pass writes dst, with the solver update when zk is set.
struct BoxCall {
    unsigned R[kBoxMaxIters];
    unsigned* qx;
    unsigned* qy;
    unsigned short* bx;
    unsigned short* by;
    unsigned short* bt;
    float* t1;
    float* t2;
};

static int box_begin(BoxCall& B, const float* guide, int Cg, int C, int batch, int H, int W, float sigma_s,
                     float sigma_r, int N, void* ws, size_t ws_bytes, hipStream_t st) {
    const BoxLayout L = make_box_layout(batch, H, W, C, N);
    if (ws == nullptr || ws_bytes < L.total) return DTS_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) & 15u) != 0) return DTS_EWORKSPACE;
    int rc = box_radii(sigma_s, N, B.R);
    if (rc) return rc;
    char* base = static_cast<char*>(ws);
    // no kernel of the box path reports a device-side failure: start from a clean status
    if ((rc = launch_zero(base, kHeaderBytes, st))) return rc;
    B.qx = reinterpret_cast<unsigned*>(base + L.qx);
    B.qy = reinterpret_cast<unsigned*>(base + L.qy);
    B.bx = reinterpret_cast<unsigned short*>(base + L.bx);
    B.by = reinterpret_cast<unsigned short*>(base + L.by);
    B.bt = reinterpret_cast<unsigned short*>(base + L.bt);
    B.t1 = reinterpret_cast<float*>(base + L.t1);
    B.t2 = reinterpret_cast<float*>(base + L.t2);
    if ((rc = launch_box_codes(guide, Cg, batch, H, W, box_s2(sigma_s, sigma_r), B.qx, B.qy, st))) return rc;
    return launch_box_bounds(B.qx, B.qy, B.bx, B.by, B.bt, batch, H, W, B.R, N, st);
}

static int box_mean(const BoxCall& B, const float* src, float* dst, int C, int batch, int H, int W, int N,
                    const float* zk, const float* tgt, const float* conf, int Cc, float lambda, float step,
                    hipStream_t st) {
    const size_t px = static_cast<size_t>(batch) * H * W;
    const float* x = src;
    for (int i = 0; i < N; ++i) {
        const int h = static_cast<int>(B.R[i] >> 8);
        // the row pass writes y (never the buffer it reads).  The window column pass writes
        // the other buffer (its halos are other tiles' rows of y); the wide-box passes build
        // their block prefix in the other buffer and write the mean back over y, or run the
        // ring kernel with the update.
        float* y = (x == B.t1) ? B.t2 : B.t1;
        float* other = (y == B.t1) ? B.t2 : B.t1;
        int rc = launch_box_row(x, y, B.bx + px * i, C, batch, H, W, h, st);
        if (rc) return rc;
        const bool last = i == N - 1;
        const bool upd = last && zk;
        if (box_window_fits(h)) {
            float* out = last ? dst : other;
            rc = launch_box_col_window(y, out, B.by + px * i, C, batch, H, W, h, upd ? zk : nullptr, tgt, conf, Cc,
                                       lambda, step, st);
            x = out;
        } else if (upd) {
            rc = launch_box_col(y, dst, B.by + px * i, C, batch, H, W, h, zk, tgt, conf, Cc, lambda, step, st);
        } else {
            rc = launch_box_col_prefixed(y, other, last ? dst : y, B.by + px * i, C, batch, H, W, st);
            x = y;
        }
        if (rc) return rc;
    }
    return DTS_OK;
}

struct Setup {
    Ctx ctx;
    Layout L;
    float* dx;
    float* dy;
    float* tmp;
};

static int begin_call(Setup& S, void* ws, size_t ws_bytes, int batch, int H, int W, int C,
                      bool with_tmp, void* stream) {
    S.L = make_layout(batch, H, W, C, with_tmp);
    if (ws == nullptr || ws_bytes < S.L.total) return DTS_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) & 15u) != 0) return DTS_EWORKSPACE;
    char* base = static_cast<char*>(ws);
    S.ctx.stream = static_cast<hipStream_t>(stream);
    S.ctx.status = reinterpret_cast<int*>(base);
    S.ctx.carry = reinterpret_cast<unsigned long long*>(base + S.L.carry);
    S.ctx.carry_words = S.L.carry_bytes / sizeof(unsigned long long);
    S.dx = reinterpret_cast<float*>(base + S.L.dx);
    S.dy = reinterpret_cast<float*>(base + S.L.dy);
    S.tmp = with_tmp ? reinterpret_cast<float*>(base + S.L.tmp) : nullptr;
    // the status word and the carry words start from zero on every call, so the
    // status read back afterwards describes the most recent call on this workspace
    int rc = launch_zero(base, kHeaderBytes, S.ctx.stream);
    if (rc) return rc;
    return launch_zero(base + S.L.carry, S.L.carry_bytes, S.ctx.stream);
}

// Scratch memory of dts_solve_noalloc: the workspace of one solve lives in this array,
// which every device the library runs on holds once (from module load to process end).
// Host code must never pass the array's name to a kernel or a copy: on the host it only
// names the symbol.  Its device address comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kScratchBytes = static_cast<size_t>(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static int scratch_address(void** out) {
    static void* ptrs[64] = {};
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= 64) return DTS_ENOTSUP;
    std::lock_guard<std::mutex> lock(mu);
    if (ptrs[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (ptr == nullptr) return hip_fail(hipErrorInvalidSymbol);
        ptrs[dev] = ptr;
    }
    *out = ptrs[dev];
    return DTS_OK;
}

}  // namespace dts

using namespace dts;

extern "C" {

size_t dts_filter_workspace_bytes(int batch, int H, int W, int Cs) {
    if (check_shape(batch, H, W) || check_channels(Cs)) return 0;
    return make_layout(batch, H, W, Cs, false).total;
}

size_t dts_solve_workspace_bytes(int batch, int H, int W, int Ct, const dts_params* p) {
    (void)p;
    if (check_shape(batch, H, W) || check_channels(Ct)) return 0;
    return make_layout(batch, H, W, Ct, true).total;
}

size_t dts_solve_backward_workspace_bytes(int batch, int H, int W, int Cg, int Ct,
                                          const dts_params* p) {
    if (!p || check_shape(batch, H, W) || check_channels(Cg) || check_channels(Ct)) return 0;
    if (p->filter_iters < 1 || p->filter_iters > kMaxFilterIters) return 0;
    return make_backward_layout(batch, H, W, Ct, p->filter_iters).total;
}

int dts_filter(const float* guide, int Cg, const float* src, float* dst, int Cs, int batch, int H,
               int W, float sigma_s, float sigma_r, int filter_iters, void* workspace,
               size_t workspace_bytes, void* stream) {
    if (!guide || !src || !dst) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || check_channels(Cs)) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return DTS_EINVAL;
    if (filter_iters < 1 || filter_iters > kMaxFilterIters) return DTS_EINVAL;
    Setup S;
    rc = begin_call(S, workspace, workspace_bytes, batch, H, W, Cs, false, stream);
    if (rc) return rc;
    const float s2 = static_cast<float>((static_cast<double>(sigma_s) / sigma_r) *
                                        (static_cast<double>(sigma_s) / sigma_r));
    for (int i = 1; i <= filter_iters; ++i) {
        const float l2a = log2_feedback(sigma_s, i, filter_iters);
        RowPass rp{};
        rp.src = (i == 1) ? src : dst;
        rp.dst = dst;
        rp.d = S.dx;
        rp.guide = (i == 1) ? guide : nullptr;
        rp.dx_out = S.dx;
        rp.dy_out = S.dy;
        rp.Cg = Cg;
        rp.s2 = s2;
        rp.C = Cs;
        rp.H = H;
        rp.W = W;
        rp.batch = batch;
        rp.log2a = l2a;
        if ((rc = launch_row_pass(rp, S.ctx))) return rc;
        ColPass cp{};
        cp.src = dst;
        cp.dst = dst;
        cp.d = S.dy;
        cp.C = Cs;
        cp.H = H;
        cp.W = W;
        cp.batch = batch;
        cp.log2a = l2a;
        cp.epilogue = false;
        if ((rc = launch_col_pass(cp, S.ctx))) return rc;
    }
    return DTS_OK;
}

// The solve of Eq. (3).  With `tape` (T > 0 needs checkpoints too) the outputs of the
// first 2N - 1 passes of every iteration go to tape[k][pass - 1] instead of the
// workspace's pass buffer: the same bytes move, and dts_solve_backward_tape reads them
// back instead of recomputing them.
static int solve_impl(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
                      int batch, int H, int W, const dts_params* p, float* out, float* checkpoints, float* tape,
                      void* workspace, size_t workspace_bytes, void* stream) {
    if (!guide || !target || !conf || !out || !p) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || check_channels(Ct)) return DTS_EINVAL;
    if (Cc != 1 && Cc != Ct) return DTS_EINVAL;
    if (!finite_pos(p->sigma_s) || !finite_pos(p->sigma_r)) return DTS_EINVAL;
    if (p->filter_iters < 1 || p->filter_iters > kMaxFilterIters) return DTS_EINVAL;
    if (p->solver_iters < 0 || p->solver_iters > kMaxSolverIters) return DTS_EINVAL;
    if (!isfinite(p->lambda) || !isfinite(p->step)) return DTS_EINVAL;
    const int T = p->solver_iters, N = p->filter_iters;
    Setup S;
    rc = begin_call(S, workspace, workspace_bytes, batch, H, W, Ct, true, stream);
    if (rc) return rc;
    const size_t sig = static_cast<size_t>(batch) * Ct * H * W;
    if (T == 0) return launch_copy(out, target, sig, S.ctx.stream);
    if (checkpoints && (rc = launch_copy(checkpoints, target, sig, S.ctx.stream))) return rc;
    const float s2 = static_cast<float>((static_cast<double>(p->sigma_s) / p->sigma_r) *
                                        (static_cast<double>(p->sigma_s) / p->sigma_r));
    const int npass = 2 * N;
    for (int k = 0; k < T; ++k) {
        const float* zk = (k == 0) ? target : (checkpoints ? checkpoints + k * sig : out);
        float* znext = (k == T - 1) ? out : (checkpoints ? checkpoints + (k + 1) * sig : out);
        // output of pass q (1 <= q < 2N) of this iteration
        float* const tk = tape ? tape + static_cast<size_t>(k) * (npass - 1) * sig : nullptr;
        const auto pass_out = [&](int q) -> float* { return tk ? tk + static_cast<size_t>(q - 1) * sig : S.tmp; };
        for (int i = 1; i <= N; ++i) {
            const float l2a = log2_feedback(p->sigma_s, i, N);
            RowPass rp{};
            rp.src = (i == 1) ? zk : pass_out(2 * i - 2);
            rp.dst = pass_out(2 * i - 1);
            rp.d = S.dx;
            rp.guide = (k == 0 && i == 1) ? guide : nullptr;
            rp.dx_out = S.dx;
            rp.dy_out = S.dy;
            rp.Cg = Cg;
            rp.s2 = s2;
            rp.C = Ct;
            rp.H = H;
            rp.W = W;
            rp.batch = batch;
            rp.log2a = l2a;
            if ((rc = launch_row_pass(rp, S.ctx))) return rc;
            ColPass cp{};
            cp.src = pass_out(2 * i - 1);
            cp.dst = (i == N) ? znext : pass_out(2 * i);
            cp.d = S.dy;
            cp.C = Ct;
            cp.H = H;
            cp.W = W;
            cp.batch = batch;
            cp.log2a = l2a;
            cp.epilogue = (i == N);
            cp.zk = zk;
            cp.tgt = target;
            cp.conf = conf;
            cp.Cc = Cc;
            cp.dst2 = nullptr;
            cp.lambda = p->lambda;
            cp.step = p->step;
            if ((rc = launch_col_pass(cp, S.ctx))) return rc;
        }
    }
    return DTS_OK;
}

int dts_solve(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
              int batch, int H, int W, const dts_params* p, float* out, float* checkpoints,
              void* workspace, size_t workspace_bytes, void* stream) {
    return solve_impl(guide, Cg, target, conf, Cc, Ct, batch, H, W, p, out, checkpoints, nullptr, workspace,
                      workspace_bytes, stream);
}

int dts_solve_tape(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
                   int batch, int H, int W, const dts_params* p, float* out, float* checkpoints, float* tape,
                   void* workspace, size_t workspace_bytes, void* stream) {
    if (!p) return DTS_EINVAL;
    if (p->solver_iters > 0 && (!checkpoints || !tape)) return DTS_EINVAL;
    return solve_impl(guide, Cg, target, conf, Cc, Ct, batch, H, W, p, out, checkpoints, tape, workspace,
                      workspace_bytes, stream);
}

int dts_solve_noalloc(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
                      int batch, int H, int W, const dts_params* p, float* out, float* checkpoints,
                      void* stream) {
    if (!p) return DTS_EINVAL;
    const size_t need = dts_solve_workspace_bytes(batch, H, W, Ct, p);
    if (need == 0) return DTS_EINVAL;
    if (need > kScratchBytes) return DTS_ENOTSUP;
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return dts_solve(guide, Cg, target, conf, Cc, Ct, batch, H, W, p, out, checkpoints, ws, kScratchBytes,
                     stream);
}

// The adjoint of solve_impl.  With `tape_ext` (written by dts_solve_tape) the inputs of
// every iteration's passes are read from it; without, they are recomputed from the
// checkpoint into the workspace's tape.
static int backward_impl(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
                         int batch, int H, int W, const dts_params* p, const float* checkpoints,
                         const float* tape_ext, const float* grad_out, float* grad_target, float* grad_conf,
                         float* grad_guide, void* workspace, size_t workspace_bytes, void* stream) {
    if (!guide || !target || !conf || !grad_out || !p) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || check_channels(Ct)) return DTS_EINVAL;
    if (Cc != 1 && Cc != Ct) return DTS_EINVAL;
    if (!finite_pos(p->sigma_s) || !finite_pos(p->sigma_r)) return DTS_EINVAL;
    if (p->filter_iters < 1 || p->filter_iters > kMaxFilterIters) return DTS_EINVAL;
    if (p->solver_iters < 0 || p->solver_iters > kMaxSolverIters) return DTS_EINVAL;
    if (!isfinite(p->lambda) || !isfinite(p->step)) return DTS_EINVAL;
    const int T = p->solver_iters, N = p->filter_iters;
    if (T > 0 && !checkpoints) return DTS_EINVAL;
    const float* const tape_in = tape_ext;
    const BwdLayout L = make_backward_layout(batch, H, W, Ct, N);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 15u))
        return DTS_EWORKSPACE;
    char* base = static_cast<char*>(workspace);
    Ctx ctx;
    ctx.stream = static_cast<hipStream_t>(stream);
    ctx.status = reinterpret_cast<int*>(base);
    ctx.carry = reinterpret_cast<unsigned long long*>(base + L.carry);
    ctx.carry_words = L.carry_bytes / sizeof(unsigned long long);
    float* dx = reinterpret_cast<float*>(base + L.dx);
    float* dy = reinterpret_cast<float*>(base + L.dy);
    float* gdx = grad_guide ? reinterpret_cast<float*>(base + L.gdx) : nullptr;
    float* gdy = grad_guide ? reinterpret_cast<float*>(base + L.gdy) : nullptr;
    float* ws_tape = reinterpret_cast<float*>(base + L.tape);
    float* gz = reinterpret_cast<float*>(base + L.gz);
    float* gab[2] = {reinterpret_cast<float*>(base + L.ga), reinterpret_cast<float*>(base + L.gb)};
    const size_t plane = static_cast<size_t>(batch) * H * W;
    const size_t sig = plane * Ct;
    const hipStream_t s = ctx.stream;

    if ((rc = launch_zero(base, kHeaderBytes, s))) return rc;
    if ((rc = launch_zero(base + L.carry, L.carry_bytes, s))) return rc;
    if (grad_guide && (rc = launch_zero(base + L.gdx, L.tape - L.gdx, s))) return rc;
    if (grad_target && (rc = launch_zero(grad_target, sig * sizeof(float), s))) return rc;
    if (grad_conf && (rc = launch_zero(grad_conf, plane * Cc * sizeof(float), s))) return rc;
    if (T == 0) {
        if (grad_target && (rc = launch_copy(grad_target, grad_out, sig, s))) return rc;
        if (grad_guide && (rc = launch_zero(grad_guide, plane * Cg * sizeof(float), s))) return rc;
        return DTS_OK;
    }
    const float s2 = static_cast<float>((static_cast<double>(p->sigma_s) / p->sigma_r) *
                                        (static_cast<double>(p->sigma_s) / p->sigma_r));
    // distances once
    {
        RowPass rp{};
        rp.guide = guide;
        rp.dx_out = dx;
        rp.dy_out = dy;
        rp.Cg = Cg;
        rp.s2 = s2;
        rp.C = 0;
        rp.H = H;
        rp.W = W;
        rp.batch = batch;
        if ((rc = launch_row_pass(rp, ctx))) return rc;
    }
    if ((rc = launch_copy(gz, grad_out, sig, s))) return rc;
    const int npass = 2 * N;
    for (int k = T - 1; k >= 0; --k) {
        const float* zk = checkpoints + static_cast<size_t>(k) * sig;
        // inputs of passes 2..2N of DT(z^k): pass p reads in(p) and writes in(p+1), kept by
        // the forward in the caller's tape or recomputed here into the workspace's
        const float* const tk = tape_in ? tape_in + static_cast<size_t>(k) * (npass - 1) * sig : ws_tape;
        auto in = [&](int pass) -> const float* {
            return pass == 1 ? zk : tk + static_cast<size_t>(pass - 2) * sig;
        };
        for (int pass = 1; pass < npass && !tape_in; ++pass) {
            const int i = (pass + 1) / 2;
            const float l2a = log2_feedback(p->sigma_s, i, N);
            float* out = ws_tape + static_cast<size_t>(pass - 1) * sig;
            if (pass & 1) {
                RowPass rp{};
                rp.src = in(pass);
                rp.dst = out;
                rp.d = dx;
                rp.C = Ct;
                rp.H = H;
                rp.W = W;
                rp.batch = batch;
                rp.log2a = l2a;
                if ((rc = launch_row_pass(rp, ctx))) return rc;
            } else {
                ColPass cp{};
                cp.src = in(pass);
                cp.dst = out;
                cp.d = dy;
                cp.C = Ct;
                cp.H = H;
                cp.W = W;
                cp.batch = batch;
                cp.log2a = l2a;
                if ((rc = launch_col_pass(cp, ctx))) return rc;
            }
        }
        // adjoint passes in reverse order; the last one carries the update adjoint
        const float* gin = gz;
        float gscale = p->step * p->lambda;
        int flip = 0;
        for (int pass = npass; pass >= 1; --pass) {
            const int i = (pass + 1) / 2;
            const float l2a = log2_feedback(p->sigma_s, i, N);
            float* gout = gab[flip];
            if (pass & 1) {
                RowAdj ra{};
                ra.gk = gin;
                ra.gk_scale = gscale;
                ra.f = in(pass);
                ra.d = dx;
                ra.gout = gout;
                ra.gd = gdx;
                ra.C = Ct;
                ra.H = H;
                ra.W = W;
                ra.batch = batch;
                ra.log2a = l2a;
                if (pass == 1) {
                    ra.gz = gz;
                    ra.tgt = target;
                    ra.conf = conf;
                    ra.gt = grad_target;
                    ra.gc = grad_conf;
                    ra.Cc = Cc;
                    ra.lambda = p->lambda;
                    ra.step = p->step;
                    ra.last = (k == 0);
                }
                if ((rc = launch_row_adjoint(ra, ctx))) return rc;
            } else {
                ColAdj ca{};
                ca.gk = gin;
                ca.gk_scale = gscale;
                ca.f = in(pass);
                ca.d = dy;
                ca.gout = gout;
                ca.gd = gdy;
                ca.C = Ct;
                ca.H = H;
                ca.W = W;
                ca.batch = batch;
                ca.log2a = l2a;
                if ((rc = launch_col_adjoint(ca, ctx))) return rc;
            }
            gin = gout;
            gscale = 1.f;
            flip ^= 1;
        }
    }
    if (grad_guide) {
        DistAdj da{guide, dx, dy, gdx, gdy, L.ngy, grad_guide, Cg, H, W, batch, s2};
        if ((rc = launch_dist_adjoint(da, ctx))) return rc;
    }
    return DTS_OK;
}

int dts_solve_backward(const float* guide, int Cg, const float* target, const float* conf, int Cc,
                       int Ct, int batch, int H, int W, const dts_params* p,
                       const float* checkpoints, const float* grad_out, float* grad_target,
                       float* grad_conf, float* grad_guide, void* workspace,
                       size_t workspace_bytes, void* stream) {
    return backward_impl(guide, Cg, target, conf, Cc, Ct, batch, H, W, p, checkpoints, nullptr, grad_out,
                         grad_target, grad_conf, grad_guide, workspace, workspace_bytes, stream);
}

int dts_solve_backward_tape(const float* guide, int Cg, const float* target, const float* conf, int Cc,
                            int Ct, int batch, int H, int W, const dts_params* p, const float* checkpoints,
                            const float* tape, const float* grad_out, float* grad_target, float* grad_conf,
                            float* grad_guide, void* workspace, size_t workspace_bytes, void* stream) {
    if (!p) return DTS_EINVAL;
    if (p->solver_iters > 0 && !tape) return DTS_EINVAL;
    return backward_impl(guide, Cg, target, conf, Cc, Ct, batch, H, W, p, checkpoints, tape, grad_out,
                         grad_target, grad_conf, grad_guide, workspace, workspace_bytes, stream);
}

static size_t stereo_workspace_bytes(int batch, int H, int W) {
    return make_layout(batch, H, W, 1, true).total + align_up(static_cast<size_t>(batch) * H * W * sizeof(float));
}

size_t dts_solve_stereo_workspace_bytes(int batch, int H, int W) {
    if (check_shape(batch, H, W)) return 0;
    return stereo_workspace_bytes(batch, H, W);
}

int dts_solve_stereo(const float* left, const float* right, int Cg, const float* target, const float* conf,
                     const float* init, int batch, int H, int W, const dts_params* p, float gamma, float epsilon,
                     float* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!left || !right || !target || !conf || !out || !p) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg)) return DTS_EINVAL;
    if (!finite_pos(p->sigma_s) || !finite_pos(p->sigma_r) || !finite_pos(epsilon)) return DTS_EINVAL;
    if (!isfinite(gamma) || gamma < 0.f) return DTS_EINVAL;
    if (p->filter_iters < 1 || p->filter_iters > kMaxFilterIters) return DTS_EINVAL;
    if (p->solver_iters < 0 || p->solver_iters > kMaxSolverIters) return DTS_EINVAL;
    if (!isfinite(p->lambda) || !isfinite(p->step)) return DTS_EINVAL;
    if (workspace_bytes < stereo_workspace_bytes(batch, H, W)) return DTS_EWORKSPACE;
    const int T = p->solver_iters, N = p->filter_iters;
    Setup S;
    rc = begin_call(S, workspace, workspace_bytes, batch, H, W, 1, true, stream);
    if (rc) return rc;
    float* D = reinterpret_cast<float*>(static_cast<char*>(workspace) + S.L.total);
    const size_t sig = static_cast<size_t>(batch) * H * W;
    const float* z0 = init ? init : target;
    if (T == 0) return launch_copy(out, z0, sig, S.ctx.stream);
    const float s2 = static_cast<float>((static_cast<double>(p->sigma_s) / p->sigma_r) *
                                        (static_cast<double>(p->sigma_s) / p->sigma_r));
    for (int k = 0; k < T; ++k) {
        const float* zk = (k == 0) ? z0 : out;
        if ((rc = launch_stereo_data_grad(zk, target, conf, left, right, D, Cg, batch, H, W, gamma, epsilon,
                                          S.ctx.stream)))
            return rc;
        for (int i = 1; i <= N; ++i) {
            const float l2a = log2_feedback(p->sigma_s, i, N);
            RowPass rp{};
            rp.src = (i == 1) ? zk : S.tmp;
            rp.dst = S.tmp;
            rp.d = S.dx;
            rp.guide = (k == 0 && i == 1) ? left : nullptr;
            rp.dx_out = S.dx;
            rp.dy_out = S.dy;
            rp.Cg = Cg;
            rp.s2 = s2;
            rp.C = 1;
            rp.H = H;
            rp.W = W;
            rp.batch = batch;
            rp.log2a = l2a;
            if ((rc = launch_row_pass(rp, S.ctx))) return rc;
            ColPass cp{};
            cp.src = S.tmp;
            cp.dst = (i == N) ? out : S.tmp;
            cp.d = S.dy;
            cp.C = 1;
            cp.H = H;
            cp.W = W;
            cp.batch = batch;
            cp.log2a = l2a;
            cp.epilogue = (i == N);
            cp.data_grad = true;
            cp.zk = zk;
            cp.tgt = D;
            cp.Cc = 1;
            cp.dst2 = nullptr;
            cp.lambda = p->lambda;
            cp.step = p->step;
            if ((rc = launch_col_pass(cp, S.ctx))) return rc;
        }
    }
    return DTS_OK;
}

size_t dts_variance_confidence_workspace_bytes(int batch, int H, int W, int C) {
    if (batch < 1 || H < 1 || W < 1 || C < 1 || 2 * C > DTS_MAX_CHANNELS) return 0;
    return make_layout(batch, H, W, 2 * C, true).total;
}

int dts_variance_confidence(const float* guide, int Cg, const float* z, float* conf, int C, int batch,
                            int H, int W, float sigma_s, float sigma_r, int filter_iters, float sigma_c,
                            void* workspace, size_t workspace_bytes, void* stream) {
    if (!guide || !z || !conf) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || C < 1 || 2 * C > DTS_MAX_CHANNELS) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r) || !finite_pos(sigma_c)) return DTS_EINVAL;
    if (filter_iters < 1 || filter_iters > kMaxFilterIters) return DTS_EINVAL;
    Setup S;
    rc = begin_call(S, workspace, workspace_bytes, batch, H, W, 2 * C, true, stream);
    if (rc) return rc;
    const float s2 = static_cast<float>((static_cast<double>(sigma_s) / sigma_r) *
                                        (static_cast<double>(sigma_s) / sigma_r));
    float* m = S.tmp;  // [batch][2C][H][W]: DT(z_c), DT(z_c^2) interleaved
    for (int i = 1; i <= filter_iters; ++i) {
        const float l2a = log2_feedback(sigma_s, i, filter_iters);
        RowPass rp{};
        rp.src = (i == 1) ? z : m;
        rp.dst = m;
        rp.d = S.dx;
        rp.guide = (i == 1) ? guide : nullptr;
        rp.dx_out = S.dx;
        rp.dy_out = S.dy;
        rp.Cg = Cg;
        rp.s2 = s2;
        rp.C = 2 * C;
        rp.H = H;
        rp.W = W;
        rp.batch = batch;
        rp.log2a = l2a;
        rp.sq = (i == 1) ? 1 : 0;
        if ((rc = launch_row_pass(rp, S.ctx))) return rc;
        ColPass cp{};
        cp.src = m;
        cp.dst = m;
        cp.d = S.dy;
        cp.C = 2 * C;
        cp.H = H;
        cp.W = W;
        cp.batch = batch;
        cp.log2a = l2a;
        cp.epilogue = false;
        if (i == filter_iters) {
            // the last column pass writes the confidences from the filtered pairs
            cp.dst = conf;
            cp.variance = true;
            cp.var_k = variance_k(sigma_c);
        }
        if ((rc = launch_col_pass(cp, S.ctx))) return rc;
    }
    return DTS_OK;
}

size_t dts_box_workspace_bytes(int batch, int H, int W, int C, int filter_iters) {
    if (check_shape(batch, H, W) || check_channels(C)) return 0;
    if (filter_iters < 1 || filter_iters > kBoxMaxIters) return 0;
    return make_box_layout(batch, H, W, C, filter_iters).total;
}

int dts_box_codes(const float* guide, int Cg, int batch, int H, int W, float sigma_s, float sigma_r,
                  unsigned* qx, unsigned* qy, void* stream) {
    if (!guide || !qx || !qy) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg)) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return DTS_EINVAL;
    return launch_box_codes(guide, Cg, batch, H, W, box_s2(sigma_s, sigma_r), qx, qy,
                            static_cast<hipStream_t>(stream));
}

int dts_filter_box(const float* guide, int Cg, const float* src, float* dst, int C, int batch, int H, int W,
                   float sigma_s, float sigma_r, int filter_iters, void* workspace, size_t workspace_bytes,
                   void* stream) {
    if (!guide || !src || !dst || src == dst) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || check_channels(C)) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return DTS_EINVAL;
    if (filter_iters < 1 || filter_iters > kBoxMaxIters) return DTS_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BoxCall B;
    if ((rc = box_begin(B, guide, Cg, C, batch, H, W, sigma_s, sigma_r, filter_iters, workspace, workspace_bytes,
                        st)))
        return rc;
    return box_mean(B, src, dst, C, batch, H, W, filter_iters, nullptr, nullptr, nullptr, 0, 0.f, 0.f, st);
}

int dts_solve_box(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct, int batch,
                  int H, int W, const dts_params* p, float* out, void* workspace, size_t workspace_bytes,
                  void* stream) {
    if (!guide || !target || !conf || !out || !p || out == target || out == conf) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg) || check_channels(Ct)) return DTS_EINVAL;
    if (Cc != 1 && Cc != Ct) return DTS_EINVAL;
    if (!finite_pos(p->sigma_s) || !finite_pos(p->sigma_r)) return DTS_EINVAL;
    if (p->filter_iters < 1 || p->filter_iters > kBoxMaxIters) return DTS_EINVAL;
    if (p->solver_iters < 0 || p->solver_iters > kMaxSolverIters) return DTS_EINVAL;
    if (!isfinite(p->lambda) || !isfinite(p->step)) return DTS_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t sig = static_cast<size_t>(batch) * Ct * H * W;
    BoxCall B;
    if ((rc = box_begin(B, guide, Cg, Ct, batch, H, W, p->sigma_s, p->sigma_r, p->filter_iters, workspace,
                        workspace_bytes, st)))
        return rc;
    if (p->solver_iters == 0) return launch_copy(out, target, sig, st);
    for (int k = 0; k < p->solver_iters; ++k) {
        // z^k is the target at k = 0 and `out` afterwards; the update reads z^k and writes
        // z^{k+1} at the same pixel, so it can run in place
        const float* zk = (k == 0) ? target : out;
        if ((rc = box_mean(B, zk, out, Ct, batch, H, W, p->filter_iters, zk, target, conf, Cc, p->lambda, p->step,
                           st)))
            return rc;
    }
    return DTS_OK;
}

size_t dts_support_workspace_bytes(int batch, int H, int W) {
    if (check_shape(batch, H, W)) return 0;
    return make_support_layout(batch, H, W).total;
}

int dts_support(const float* guide, int Cg, int batch, int H, int W, float sigma_s, float sigma_r,
                int filter_iters, float* support, const float* conf, int Cc, float* conf_out, void* workspace,
                size_t workspace_bytes, void* stream) {
    if (!guide || !support) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg)) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return DTS_EINVAL;
    if (filter_iters < 1 || filter_iters > kMaxFilterIters) return DTS_EINVAL;
    if (conf && (!conf_out || check_channels(Cc))) return DTS_EINVAL;
    if (conf && (conf == support || conf_out == support)) return DTS_EINVAL;
    const SupportLayout L = make_support_layout(batch, H, W);
    if (workspace == nullptr || workspace_bytes < L.total) return DTS_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(workspace) & 15u) != 0) return DTS_EWORKSPACE;
    char* base = static_cast<char*>(workspace);
    float* dx = reinterpret_cast<float*>(base + L.dx);
    float* dy = reinterpret_cast<float*>(base + L.dy);
    float* tmp = reinterpret_cast<float*>(base + L.tmp);
    Ctx ctx;
    ctx.stream = static_cast<hipStream_t>(stream);
    ctx.status = reinterpret_cast<int*>(base);
    ctx.carry = reinterpret_cast<unsigned long long*>(base + L.carry);
    ctx.carry_words = L.carry_bytes / sizeof(unsigned long long);
    // status and carry words start from zero: the status read back afterwards describes
    // this call (a bounded wait of the column passes that gave up)
    if ((rc = launch_zero(base, kHeaderBytes, ctx.stream))) return rc;
    if ((rc = launch_zero(base + L.carry, L.carry_bytes, ctx.stream))) return rc;
    RowPass rp{};
    rp.guide = guide;
    rp.dx_out = dx;
    rp.dy_out = dy;
    rp.Cg = Cg;
    rp.s2 = static_cast<float>((static_cast<double>(sigma_s) / sigma_r) *
                               (static_cast<double>(sigma_s) / sigma_r));
    rp.C = 0;  // distances only
    rp.H = H;
    rp.W = W;
    rp.batch = batch;
    if ((rc = launch_row_pass(rp, ctx))) return rc;
    for (int i = 1; i <= filter_iters; ++i) {
        const float l2a = log2_feedback(sigma_s, i, filter_iters);
        const double a = feedback(sigma_s, i, filter_iters);
        const float m = static_cast<float>((1.0 - a) / (1.0 + a));
        if ((rc = launch_support_row(i == 1 ? nullptr : support, dx, tmp, batch, H, W, l2a, m, ctx.stream)))
            return rc;
        const bool last = i == filter_iters;
        if ((rc = launch_support_col(tmp, dy, support, last ? conf : nullptr, Cc, last ? conf_out : nullptr, batch,
                                     H, W, l2a, m, ctx)))
            return rc;
    }
    return DTS_OK;
}

int dts_distances(const float* guide, int Cg, int batch, int H, int W, float sigma_s,
                  float sigma_r, float* dx, float* dy, void* stream) {
    if (!guide || !dx || !dy) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(Cg)) return DTS_EINVAL;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return DTS_EINVAL;
    Ctx ctx;
    ctx.stream = static_cast<hipStream_t>(stream);
    RowPass rp{};
    rp.guide = guide;
    rp.dx_out = dx;
    rp.dy_out = dy;
    rp.Cg = Cg;
    rp.s2 = static_cast<float>((static_cast<double>(sigma_s) / sigma_r) *
                               (static_cast<double>(sigma_s) / sigma_r));
    rp.C = 0;  // distances only: no signal channel is filtered
    rp.H = H;
    rp.W = W;
    rp.batch = batch;
    rp.log2a = 0.f;
    return launch_row_pass(rp, ctx);
}

size_t dts_pass_workspace_bytes(int batch, int H, int W, int C) {
    if (check_shape(batch, H, W) || check_channels(C)) return 0;
    return kHeaderBytes + align_up(col_carry_words(batch, H, W, C) * sizeof(unsigned long long));
}

static int check_pass(const float* src, const float* dst, const float* d, int C, int batch, int H,
                      int W, float sigma_s, int iter, int N) {
    if (!src || !dst || !d) return DTS_EINVAL;
    int rc = check_shape(batch, H, W);
    if (rc) return rc;
    if (check_channels(C)) return DTS_EINVAL;
    if (!finite_pos(sigma_s)) return DTS_EINVAL;
    if (N < 1 || N > kMaxFilterIters || iter < 1 || iter > N) return DTS_EINVAL;
    return DTS_OK;
}

int dts_row_pass(const float* src, float* dst, const float* dx, int C, int batch, int H, int W,
                 float sigma_s, int iter, int filter_iters, void* stream) {
    int rc = check_pass(src, dst, dx, C, batch, H, W, sigma_s, iter, filter_iters);
    if (rc) return rc;
    Ctx ctx;
    ctx.stream = static_cast<hipStream_t>(stream);
    RowPass rp{};
    rp.src = src;
    rp.dst = dst;
    rp.d = dx;
    rp.C = C;
    rp.H = H;
    rp.W = W;
    rp.batch = batch;
    rp.log2a = log2_feedback(sigma_s, iter, filter_iters);
    return launch_row_pass(rp, ctx);
}

int dts_col_pass(const float* src, float* dst, const float* dy, int C, int batch, int H, int W,
                 float sigma_s, int iter, int filter_iters, void* workspace,
                 size_t workspace_bytes, void* stream) {
    int rc = check_pass(src, dst, dy, C, batch, H, W, sigma_s, iter, filter_iters);
    if (rc) return rc;
    const size_t need = dts_pass_workspace_bytes(batch, H, W, C);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 15u))
        return DTS_EWORKSPACE;
    char* base = static_cast<char*>(workspace);
    Ctx ctx;
    ctx.stream = static_cast<hipStream_t>(stream);
    ctx.status = reinterpret_cast<int*>(base);
    ctx.carry = reinterpret_cast<unsigned long long*>(base + kHeaderBytes);
    ctx.carry_words = (need - kHeaderBytes) / sizeof(unsigned long long);
    if ((rc = launch_zero(base, need, ctx.stream))) return rc;
    ColPass cp{};
    cp.src = src;
    cp.dst = dst;
    cp.d = dy;
    cp.C = C;
    cp.H = H;
    cp.W = W;
    cp.batch = batch;
    cp.log2a = log2_feedback(sigma_s, iter, filter_iters);
    cp.epilogue = false;
    return launch_col_pass(cp, ctx);
}

int dts_col_variant_count(void) { return num_col_variants(); }

int dts_col_variant_info(int variant, int* group_channels, int* rows_per_wave, int* waves) {
    if (!group_channels || !rows_per_wave || !waves) return DTS_EINVAL;
    return col_variant_info(variant, group_channels, rows_per_wave, waves);
}

int dts_tune_col_variant(int group_channels, int variant) {
    return tune_col_variant(group_channels, variant);
}

int dts_tune_col_xcd(int on) { return tune_col_xcd(on); }

int dts_tune_spin_limit(int polls) { return tune_spin_limit(polls); }

int dts_tune_row_segment(int pixels_per_lane) { return tune_row_segment(pixels_per_lane); }
int dts_tune_box_window(int on) { return tune_box_window(on); }

int dts_workspace_status(void* workspace, void* stream) {
    if (!workspace) return DTS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int status = 0;
    int rc = hip_fail(hipMemcpyAsync(&status, workspace, sizeof(int), hipMemcpyDeviceToHost, s));
    if (rc) return rc;
    if ((rc = hip_fail(hipStreamSynchronize(s)))) return rc;
    if (status != 0) {
        if ((rc = launch_zero(workspace, 16, s))) return rc;
        if ((rc = hip_fail(hipStreamSynchronize(s)))) return rc;
        return DTS_EDEVICE;
    }
    return DTS_OK;
}

const char* dts_strerror(int code) {
    switch (code) {
        case DTS_OK: return "success";
        case DTS_EINVAL: return "invalid argument";
        case DTS_EWORKSPACE: return "workspace missing, misaligned or too small";
        case DTS_EHIP: return "HIP runtime error (see dts_last_hip_error)";
        case DTS_ENOTSUP: return "shape or option not supported";
        case DTS_EDEVICE: return "device-side failure reported by a kernel";
        default: return "unknown error";
    }
}

const char* dts_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
