// Kernel timing with HIP events, recorded on each kernel's launch stream.
//
// When enabled (bolt_prof_enable), every instrumented launch records a start
// and a stop event around itself (only launches whose name starts with the
// prefix given to bolt_prof_only, when one is given: each pair of events
// costs stream time); bolt_prof_read waits for the
// recorded events and returns, per kernel name, the number of launches and
// their total duration.  Disabled, the instrumentation is a single branch per
// launch.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace {

struct Pending {
    std::string name;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::string g_only;   // name prefix of the timed launches (empty: all)
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<int64_t, double>> g_totals;   // name -> (launches, ms)

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence when the event is recorded (the
    // default one writes back and invalidates the caches at every record,
    // which slows the work that follows; results are read after a full
    // synchronisation, never through these events)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
        return nullptr;
    return e;
}

void drain_locked()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            auto &t = g_totals[p.name];
            t.first += 1;
            t.second += ms;
        }
        g_pool.push_back(p.start);
        g_pool.push_back(p.stop);
    }
    g_pending.clear();
}

}  // namespace

namespace bolt {

bool prof_on() { return g_on; }

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s), start_(nullptr)
{
    if (!g_on)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_only.empty() && g_only.compare(0, g_only.size(), name, 0, g_only.size()) != 0)
        return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return;   // no timing inside graph capture
    start_ = take_event();
    if (start_ && hipEventRecord(reinterpret_cast<hipEvent_t>(start_), s) != hipSuccess)
        start_ = nullptr;
}

ProfScope::~ProfScope()
{
    if (!start_)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t stop = take_event();
    if (!stop || hipEventRecord(stop, s_) != hipSuccess) {
        g_pool.push_back(reinterpret_cast<hipEvent_t>(start_));
        return;
    }
    g_pending.push_back({name_, reinterpret_cast<hipEvent_t>(start_), stop});
    if (g_pending.size() > 4096)
        drain_locked();
}

}  // namespace bolt

extern "C" int bolt_prof_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return BOLT_OK;
}

extern "C" int bolt_prof_only(const char *prefix)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_only = prefix ? prefix : "";
    return BOLT_OK;
}

// Totals since the last reset.  names: buffer receiving "name=launches:ms;..."
extern "C" int bolt_prof_read(char *names, size_t cap, int32_t reset)
{
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    std::string out;
    for (auto &kv : g_totals) {
        out += kv.first + "=" + std::to_string(kv.second.first) + ":" + std::to_string(kv.second.second) + ";";
    }
    if (reset)
        g_totals.clear();
    if (names && cap) {
        const size_t n = out.size() < cap - 1 ? out.size() : cap - 1;
        out.copy(names, n);
        names[n] = 0;
    }
    return (int)out.size();
}
