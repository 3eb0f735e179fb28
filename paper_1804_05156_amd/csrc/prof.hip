// prof.hip -- optional per-kernel timing with HIP events.
//
// When enabled, every instrumented launch is bracketed by two events recorded on
// its own stream; fe_prof_read synchronizes them and aggregates elapsed times by
// kernel name.  Launches made while the stream is being captured into a graph are
// not timed.  Off by default: a disabled timer costs one branch per launch, and
// switching it off destroys its events.
#include <cstring>
#include <mutex>
#include <vector>

#include "fe_internal.h"

namespace {

struct Rec {
    const char *name;
    hipEvent_t a, b;
    bool closed;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

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

void recycle_all()
{
    for (Rec &r : g_recs) {
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_recs.clear();
}

// Destroy every pooled event (timing switched off: nothing of the timer stays
// alive in the runtime until process exit).
void release_pool()
{
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    g_pool.shrink_to_fit();
}

}  // namespace

int fe_prof_begin(const char *name, hipStream_t s)
{
    if (!g_on) return -1;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec r{name, take_event(), take_event(), false};
    if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) {
        g_recs.push_back(r);
        return -1;
    }
    g_recs.push_back(r);
    return (int)g_recs.size() - 1;
}

void fe_prof_end(int tok, hipStream_t s)
{
    if (tok < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (tok >= (int)g_recs.size()) return;
    if (hipEventRecord(g_recs[tok].b, s) == hipSuccess) g_recs[tok].closed = true;
}

extern "C" int fe_prof_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (Rec &r : g_recs)
        if (r.closed) (void)hipEventSynchronize(r.b);
    recycle_all();
    g_on = on != 0;
    if (!g_on) release_pool();
    return FE_OK;
}

extern "C" int fe_prof_read(fe_prof_entry *out, int32_t cap, int32_t *count)
{
    if (!count || cap < 0 || (cap > 0 && !out)) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<fe_prof_entry> agg;
    for (Rec &r : g_recs) {
        if (!r.closed) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return FE_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return FE_EHIP;
        fe_prof_entry *e = nullptr;
        for (fe_prof_entry &x : agg)
            if (strncmp(x.name, r.name, sizeof(x.name)) == 0) e = &x;
        if (!e) {
            fe_prof_entry z{};
            strncpy(z.name, r.name, sizeof(z.name) - 1);
            z.min_ms = 1e300;
            agg.push_back(z);
            e = &agg.back();
        }
        e->launches += 1;
        e->total_ms += ms;
        if (ms < e->min_ms) e->min_ms = ms;
        if (ms > e->max_ms) e->max_ms = ms;
    }
    recycle_all();
    *count = (int32_t)agg.size();
    for (int32_t k = 0; k < cap && k < (int32_t)agg.size(); ++k) out[k] = agg[k];
    return FE_OK;
}
