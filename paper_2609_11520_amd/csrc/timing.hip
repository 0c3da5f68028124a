// Per-kernel timing hooks: when enabled, every launch wrapped in a TimingScope is
// bracketed by HIP events recorded on the launch stream; durations accumulate per
// kernel name and are read back with fio_timing_query.
#include "timing.h"

#include <map>
#include <string>

namespace fio {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
struct Acc {
    long n = 0;
    double ms = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Acc> g_acc;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    FIO_HIP(hipEventCreate(&e));
    return e;
}

void drain_locked() {
    for (auto &p : g_pending) {
        FIO_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        FIO_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        Acc &a = g_acc[p.name];
        a.n += 1;
        a.ms += ms;
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

bool timing_on() { return g_on; }

TimingScope::TimingScope(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = get_event();
    b_ = get_event();
    FIO_HIP(hipEventRecord(a_, s_));
    active_ = true;
}

TimingScope::~TimingScope() {
    if (!active_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipEventRecord(b_, s_) == hipSuccess) g_pending.push_back(Pending{name_, a_, b_});
}

}  // namespace fio

using namespace fio;

extern "C" void fio_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
}

extern "C" void fio_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    try {
        drain_locked();
    } catch (const Err &) {
    }
    g_acc.clear();
}

extern "C" int fio_timing_query(const char *kernel, long *launches, double *total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    try {
        drain_locked();
    } catch (const Err &e) {
        return e.st;
    }
    auto it = g_acc.find(kernel ? kernel : "");
    long n = it == g_acc.end() ? 0 : it->second.n;
    double ms = it == g_acc.end() ? 0.0 : it->second.ms;
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return FIO_OK;
}

extern "C" int fio_timing_names(char *buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_mu);
    try {
        drain_locked();
    } catch (const Err &e) {
        return e.st;
    }
    std::string s;
    for (auto &kv : g_acc) {
        if (!s.empty()) s += ",";
        s += kv.first;
    }
    if (buf && len) {
        size_t n = s.size() < len - 1 ? s.size() : len - 1;
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size();
}
