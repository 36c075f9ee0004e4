// Launch timing for libdts: when enabled, every kernel launch is bracketed by a pair of
// HIP events recorded on the stream the kernel runs on, and tagged with the algorithmic
// bytes that launch must move.  dts_profile_read aggregates them per kernel variant.
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dts.h"
#include "dts_internal.hpp"

namespace dts {

namespace {
struct Rec {
    std::string name;
    hipEvent_t start, stop;
    double bytes;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
}  // namespace

ProfScope::ProfScope(const char* name, double bytes, hipStream_t s) : stream_(s) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_on) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    if (hipEventRecord(a, s) != hipSuccess) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return;
    }
    g_recs.push_back(Rec{name, a, b, bytes});
    index_ = static_cast<long>(g_recs.size()) - 1;
}

ProfScope::~ProfScope() {
    if (index_ < 0) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (index_ < static_cast<long>(g_recs.size())) (void)hipEventRecord(g_recs[index_].stop, stream_);
}

static void clear_locked() {
    for (auto& r : g_recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_recs.clear();
}

}  // namespace dts

using namespace dts;

extern "C" int dts_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (on) clear_locked();
    g_on = on != 0;
    return DTS_OK;
}

extern "C" int dts_profile_read(dts_kernel_stat* rows, int max_rows) {
    if (max_rows < 0 || (max_rows > 0 && !rows)) return DTS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    struct Acc {
        int n = 0;
        double ms = 0, bytes = 0;
    };
    std::map<std::string, Acc> agg;
    for (auto& r : g_recs) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return hip_fail(hipGetLastError());
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return hip_fail(hipGetLastError());
        Acc& a = agg[r.name];
        a.n += 1;
        a.ms += ms;
        a.bytes += r.bytes;
    }
    int i = 0;
    for (auto& kv : agg) {
        if (i < max_rows) {
            memset(&rows[i], 0, sizeof(rows[i]));
            strncpy(rows[i].name, kv.first.c_str(), sizeof(rows[i].name) - 1);
            rows[i].launches = kv.second.n;
            rows[i].total_ms = kv.second.ms;
            rows[i].bytes = kv.second.bytes;
        }
        ++i;
    }
    return i;
}
