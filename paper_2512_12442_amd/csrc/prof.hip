// Stage timer: when enabled, launches of the selected stages are bracketed by hipEvents
// recorded on the stream they run on; lcp_profile_end sums the elapsed times per stage.
#include <mutex>
#include <vector>

#include "lcp_internal.h"

namespace lcp {

namespace {

struct Rec {
    hipEvent_t a, b;
    int stage;
};

std::mutex g_mu;
bool g_on = false;
unsigned g_mask = 0;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
constexpr size_t kMaxRecs = 1 << 16;

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

}  // namespace

StageScope::StageScope(hipStream_t s, int stage) : s_(s), idx_(-1)
{
    if (!g_on || !(g_mask & (1u << stage))) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_recs.size() >= kMaxRecs) return;
    Rec r{take_event(), take_event(), stage};
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    idx_ = (int)g_recs.size();
    g_recs.push_back(r);
}

StageScope::~StageScope()
{
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(g_recs[idx_].b, s_);
}

}  // namespace lcp

extern "C" {

int lcp_profile_begin(unsigned stage_mask)
{
    std::lock_guard<std::mutex> lk(lcp::g_mu);
    for (auto& r : lcp::g_recs) {
        lcp::g_pool.push_back(r.a);
        lcp::g_pool.push_back(r.b);
    }
    lcp::g_recs.clear();
    lcp::g_mask = stage_mask;
    lcp::g_on = true;
    return LCP_OK;
}

int lcp_profile_end(double* ms, int64_t* launches, int n_stages)
{
    std::lock_guard<std::mutex> lk(lcp::g_mu);
    lcp::g_on = false;
    for (int i = 0; i < n_stages; ++i) {
        if (ms) ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    int rc = LCP_OK;
    for (auto& r : lcp::g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) { rc = LCP_EDEVICE; continue; }
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) { rc = LCP_EDEVICE; continue; }
        if (r.stage < n_stages) {
            if (ms) ms[r.stage] += t;
            if (launches) launches[r.stage] += 1;
        }
    }
    return rc;
}

}  // extern "C"
