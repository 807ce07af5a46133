// Per-kernel timing: a process-wide record of (kernel name, start, stop)
// event pairs filled by launch() while enabled (for every launch, or for the
// launch names mesh_timing_select lists), and read back by mesh_timing_read.
// Guarded by a mutex; events are created lazily on the device current at the
// time and reused.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mesh_neighbors.h"
#include "launch.hpp"

namespace mnb {

namespace {

constexpr size_t MAX_PENDING = 1 << 16;

struct Pending {
    std::string name;  // copied: launch names may live in the caller's stack buffer
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_enabled = false;
std::vector<hipEvent_t> g_pool;
std::vector<Pending> g_pending;
std::vector<std::string> g_select;  // launch names timed; empty: all
thread_local int t_untimed = 0;
constexpr size_t MAX_SELECT_CHARS = 1024;
constexpr size_t MAX_SELECT_NAMES = 32;

}  // namespace

UntimedScope::UntimedScope() { ++t_untimed; }
UntimedScope::~UntimedScope() { --t_untimed; }

bool timing_enabled(const char* name) {
    if (t_untimed) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_enabled) return false;
    if (g_select.empty()) return true;
    for (const std::string& s : g_select)
        if (s == name) return true;
    return false;
}

bool timing_begin(hipEvent_t* start, hipEvent_t* stop) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_enabled || g_pending.size() >= MAX_PENDING) return false;
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (!g_pool.empty()) {
            ev[i] = g_pool.back();
            g_pool.pop_back();
        } else if (hipEventCreate(&ev[i]) != hipSuccess) {
            if (i == 1) g_pool.push_back(ev[0]);
            return false;
        }
    }
    *start = ev[0];
    *stop = ev[1];
    return true;
}

void timing_commit(const char* name, hipEvent_t start, hipEvent_t stop) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name, start, stop});
}

}  // namespace mnb

using namespace mnb;

extern "C" {

mesh_status mesh_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = enable != 0;
    return MESH_OK;
}

mesh_status mesh_timing_select(const char* names) {
    std::vector<std::string> sel;
    if (names) {
        const size_t n = std::strlen(names);
        if (n > MAX_SELECT_CHARS) return MESH_ERR_INVALID_ARG;
        size_t a = 0;
        while (a <= n) {
            size_t b = a;
            while (b < n && names[b] != ',') ++b;
            if (b > a) sel.emplace_back(names + a, b - a);
            a = b + 1;
        }
        if (sel.size() > MAX_SELECT_NAMES) return MESH_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_select.swap(sel);
    return MESH_OK;
}

int32_t mesh_timing_read(mesh_kernel_time* out, int32_t max_entries) {
    std::vector<Pending> pending;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        pending.swap(g_pending);
    }
    std::vector<mesh_kernel_time> agg;
    int32_t status = 0;
    for (const Pending& p : pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) != hipSuccess || hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess)
            status = -1;
        size_t k = 0;
        while (k < agg.size() && std::string(agg[k].name) != p.name.substr(0, sizeof(agg[k].name) - 1)) ++k;
        if (k == agg.size()) {
            mesh_kernel_time t{};
            std::snprintf(t.name, sizeof(t.name), "%s", p.name.c_str());
            t.min_ms = 1e300;
            agg.push_back(t);
        }
        mesh_kernel_time& t = agg[k];
        t.launches += 1;
        t.total_ms += ms;
        t.min_ms = ms < t.min_ms ? ms : t.min_ms;
        t.max_ms = ms > t.max_ms ? ms : t.max_ms;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Pending& p : pending) {
            g_pool.push_back(p.start);
            g_pool.push_back(p.stop);
        }
    }
    if (status != 0) return -1;
    const int32_t n = (int32_t)agg.size();
    for (int32_t i = 0; i < n && i < max_entries && out; ++i) out[i] = agg[i];
    return n;
}

}  // extern "C"
