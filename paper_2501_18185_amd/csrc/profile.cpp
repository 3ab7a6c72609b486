// Optional per-kernel timing with HIP events recorded on the launch stream.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mw_internal.h"

namespace mw {

struct ProfRec {
    hipEvent_t a, b;
};

static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::map<std::string, std::vector<ProfRec>> g_prof;

// launches recorded into a HIP graph must not record events
static thread_local int g_prof_suppress = 0;

ProfSuppress::ProfSuppress() { g_prof_suppress++; }
ProfSuppress::~ProfSuppress() { g_prof_suppress--; }

bool prof_enabled() { return g_prof_on && !g_prof_suppress; }

ProfToken prof_begin(const char *name, hipStream_t s)
{
    ProfToken t{nullptr, nullptr, name};
    if (!g_prof_on || g_prof_suppress) return t;
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) return ProfToken{nullptr, nullptr, name};
    hipEventRecord(t.a, s);
    return t;
}

void prof_end(const ProfToken &t, hipStream_t s)
{
    if (!t.a) return;
    hipEventRecord(t.b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[t.name].push_back(ProfRec{t.a, t.b});
}

static void clear_all()
{
    for (auto &kv : g_prof)
        for (auto &r : kv.second) {
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
    g_prof.clear();
}

}  // namespace mw

using namespace mw;

extern "C" mw_status mw_profile(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (enable) clear_all();
    g_prof_on = enable != 0;
    return MW_OK;
}

extern "C" mw_status mw_profile_read(const char *kernel, int64_t *launches, double *total_ms)
{
    if (!kernel || !launches || !total_ms) return fail(MW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *launches = 0;
    *total_ms = 0.0;
    auto it = g_prof.find(kernel);
    if (it == g_prof.end()) return MW_OK;
    for (auto &r : it->second) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(MW_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(MW_EHIP, "hipEventElapsedTime failed");
        *total_ms += ms;
        (*launches)++;
    }
    return MW_OK;
}
