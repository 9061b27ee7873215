// Per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when enabled, every instrumented launch records an
// event pair around itself, and bmpc_profile_read() resolves the pairs
// (synchronising on the events) into per-kernel totals.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bmpc_internal.hpp"
#include "profile.hpp"

namespace bmpc {

namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<Rec> g_pending;
std::map<std::string, std::pair<double, int>> g_tot;
std::string g_only;  // empty: every launch

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void resolve_locked()
{
    for (auto& r : g_pending) {
        float ms = 0.f;
        if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto& t = g_tot[r.name];
            t.first += ms;
            t.second += 1;
        }
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_pending.clear();
}
}  // namespace

bool profiling_enabled() { return g_on; }

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s)
{
    if (!g_on) return;
    // no event pairs inside a stream capture: they would become graph nodes
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_only.empty() && g_only != name) return;
    a_ = take_event();
    if (a_) (void)hipEventRecord(a_, s_);
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (b) (void)hipEventRecord(b, s_);
    g_pending.push_back(Rec{name_, a_, b});
}

}  // namespace bmpc

using namespace bmpc;

extern "C" {

BMPC_API bmpc_status bmpc_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_locked();
    g_tot.clear();
    g_on = on != 0;
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_profile_only(const char* name)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_only = name ? name : "";
    return BMPC_OK;
}

BMPC_API int32_t bmpc_profile_read(char* names, double* total_ms, int32_t* launches, int32_t cap)
{
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_locked();
    int i = 0;
    for (auto& kv : g_tot) {
        if (i < cap) {
            if (names) {
                std::strncpy(names + 64 * i, kv.first.c_str(), 63);
                names[64 * i + 63] = 0;
            }
            if (total_ms) total_ms[i] = kv.second.first;
            if (launches) launches[i] = kv.second.second;
        }
        ++i;
    }
    g_tot.clear();
    return i;
}

}  // extern "C"
