// Batched sigma (many problems, one persistent launch, replayed from a HIP
// graph) and the autotuner for the launch parameters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "mw_internal.h"

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);
extern "C" void mw_internal_set_tune(mw_plan plan, int32_t u, int32_t gl);

void mw::batch_set_gather(BatchSet &b, int gl)
{
    BatchArgs &a = b.all;
    b.gl = gl;
    a.blk_start[0] = 0;
    for (int k = 0; k < a.nprob; k++) a.blk_start[k + 1] = a.blk_start[k] + (a.ndet[k] * a.R[k] * gl + 255) / 256;
}

namespace {

struct BatchKey {
    std::vector<uintptr_t> v;
    bool operator<(const BatchKey &o) const { return v < o.v; }
};

struct BatchEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int bpc = 0;  // persistent blocks per compute unit used when captured
    int u4 = 0;   // four-root partner unroll used when captured
    int gl = 0;   // gather lanes used when captured
    uint64_t used = 0;  // last use, for the eviction of the least recent
};

// Graphs are keyed by the argument tuple (their kernels hold the device
// pointers of c and sigma); at most BATCH_GRAPHS are kept, the least
// recently used dropped first, so new output buffers on every call do not
// accumulate graphs.
constexpr size_t BATCH_GRAPHS = 16;
std::mutex g_mu;
std::map<BatchKey, BatchEntry> g_cache;
uint64_t g_clock = 0;
struct Tuned {
    int bpc, u4, gl;
};
std::map<BatchKey, Tuned> g_tuned;  // autotuned launch parameters, by batch
hipStream_t g_capture_stream = nullptr;
int g_num_cu = 0;

int num_cu()
{
    if (!g_num_cu) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_num_cu = n;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

mw_status make_args(int32_t nprob, const mw_plan *plans, const int32_t *nroots, const void *const *c,
                    void *const *sigma, BatchSet &b, bool &cplx, BatchKey &key)
{
    if (nprob < 1 || nprob > MW_MAXB) return fail(MW_EUNSUPPORTED, "nprob must be in 1..32");
    if (!plans || !nroots || !c || !sigma) return fail(MW_EINVAL, "NULL argument");
    std::vector<const DevPlan *> d(nprob);
    for (int i = 0; i < nprob; i++) {
        d[i] = mw_internal_devplan(plans[i]);
        if (!d[i]) return fail(MW_EWORKSPACE, "plan " + std::to_string(i) + " has no workspace");
        if (nroots[i] < 1 || nroots[i] > d[i]->max_roots) return fail(MW_EINVAL, "nroots out of range");
        if (!c[i] || !sigma[i] || c[i] == sigma[i]) return fail(MW_EINVAL, "bad c/sigma pointer");
        if (d[i]->kind != d[0]->kind) return fail(MW_EINVAL, "all plans of a batch must be of one kind");
        for (int j = 0; j < i; j++)
            if (plans[j] == plans[i]) return fail(MW_EINVAL, "a plan may appear once per batch");
    }
    cplx = d[0]->kind == MW_SPINOR;
    // largest problems first
    std::vector<int> ord(nprob);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x]->nmem > d[y]->nmem; });
    BatchArgs &a = b.all;
    a = BatchArgs{};
    a.nprob = nprob;
    a.pk_start[0] = 0;
    a.pkd_start[0] = 0;
    a.pks_start[0] = 0;
    a.blk_start[0] = 0;
    for (int k = 0; k < nprob; k++) {
        int i = ord[k];
        a.plans[k] = d[i]->self;
        a.c[k] = c[i];
        a.sigma[k] = sigma[i];
        a.R[k] = nroots[i];
        a.ndet[k] = d[i]->ndet;
        a.pk_start[k + 1] = a.pk_start[k] + d[i]->npacket;
        a.pkd_start[k + 1] = a.pkd_start[k] + d[i]->npacket_double;
        a.pks_start[k + 1] = a.pks_start[k] + (d[i]->npacket - d[i]->npacket_double);
    }
    batch_set_gather(b, cplx ? 32 : 16);  // the plain default width of the kind
    // one dispatch counts its work-items in 32 bits (gather laid out for the
    // widest width the tuner tries)
    int64_t blk32 = 0;
    for (int k = 0; k < nprob; k++) blk32 += (a.ndet[k] * a.R[k] * 32 + 255) / 256;
    if (a.pk_start[nprob] * 64 >= 0xffffffffLL - (1 << 20) || (blk32 + 8) * 256 >= 0xffffffffLL)
        return fail(MW_EUNSUPPORTED, "too many packets in one batch");
    a.counter = d[ord[0]]->counter;
    // per root-chunk width: problems with a chunk of 4, 2 or 1 roots
    for (int cl = 0; cl < 3; cl++) {
        BatchArgs &e = b.cls[cl];
        e = BatchArgs{};
        e.pk_start[0] = 0;
        e.pkd_start[0] = 0;
        e.pks_start[0] = 0;
        e.counter = a.counter + 8 * cl;
        for (int k = 0; k < nprob; k++) {
            const int R = a.R[k];
            bool has = false;
            for (int r0 = 0; r0 < R; r0 += 4) {
                const int left = R - r0, wd = left == 1 ? 1 : (left == 2 ? 2 : 4);
                has = has || wd == (cl == 0 ? 4 : (cl == 1 ? 2 : 1));
            }
            if (!has) continue;
            const int j = e.nprob++;
            e.plans[j] = a.plans[k];
            e.c[j] = a.c[k];
            e.sigma[j] = a.sigma[k];
            e.R[j] = R;
            e.pk_start[j + 1] = e.pk_start[j] + (a.pk_start[k + 1] - a.pk_start[k]);
            e.pkd_start[j + 1] = e.pkd_start[j] + (a.pkd_start[k + 1] - a.pkd_start[k]);
            e.pks_start[j + 1] = e.pks_start[j] + (a.pks_start[k + 1] - a.pks_start[k]);
        }
    }
    key.v.clear();
    for (int i = 0; i < nprob; i++) {
        key.v.push_back((uintptr_t)plans[i]);
        key.v.push_back((uintptr_t)c[i]);
        key.v.push_back((uintptr_t)sigma[i]);
        key.v.push_back((uintptr_t)nroots[i]);
    }
    return MW_OK;
}

mw_status capture(const BatchSet &a, bool cplx, int bpc, BatchEntry &e)
{
    if (!g_capture_stream && hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(MW_EHIP, "hipStreamCreateWithFlags failed");
    if (hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(MW_EHIP, "hipStreamBeginCapture failed");
    mw_status st = launch_batched(a, cplx, num_cu() * bpc, g_capture_stream, false);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(g_capture_stream, &g);
    if (st != MW_OK) return st;
    if (ce != hipSuccess || !g) return fail(MW_EHIP, "hipStreamEndCapture failed");
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return fail(MW_EHIP, "hipGraphInstantiate failed");
    }
    e.graph = g;
    e.exec = ex;
    e.bpc = bpc;
    e.u4 = a.u4;
    e.gl = a.gl;
    return MW_OK;
}

void drop(BatchEntry &e)
{
    if (e.exec) hipGraphExecDestroy(e.exec);
    if (e.graph) hipGraphDestroy(e.graph);
    e = BatchEntry{};
}

}  // namespace

void mw_internal_grad_forget(mw_plan plan);

// Forget captured graphs that reference a plan (called when the plan is
// destroyed or re-bound: the graphs hold its device addresses).
void mw_internal_batched_forget(mw_plan plan)
{
    mw_internal_grad_forget(plan);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        bool hit = false;
        for (size_t i = 0; i < it->first.v.size(); i += 4) hit = hit || it->first.v[i] == (uintptr_t)plan;
        if (hit) {
            drop(it->second);
            it = g_cache.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = g_tuned.begin(); it != g_tuned.end();) {
        bool hit = false;
        for (size_t i = 0; i < it->first.v.size(); i += 4) hit = hit || it->first.v[i] == (uintptr_t)plan;
        it = hit ? g_tuned.erase(it) : std::next(it);
    }
}

extern "C" mw_status mw_sigma_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                                      const void *const *c, void *const *sigma, mw_stream_t stream)
{
    BatchSet a;
    bool cplx;
    BatchKey key;
    mw_status st = make_args(nprob, plans, nroots, c, sigma, a, cplx, key);
    if (st != MW_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    int bpc = 8;
    auto tb = g_tuned.find(key);
    if (tb != g_tuned.end()) {
        bpc = tb->second.bpc;
        a.u4 = tb->second.u4;
        batch_set_gather(a, tb->second.gl);
    }
    auto it = g_cache.find(key);
    if (it != g_cache.end() && (it->second.bpc != bpc || it->second.u4 != a.u4 || it->second.gl != a.gl)) {
        drop(it->second);
        g_cache.erase(it);
        it = g_cache.end();
    }
    if (it == g_cache.end()) {
        BatchEntry e;
        st = capture(a, cplx, bpc, e);
        if (st != MW_OK) return st;
        if (g_cache.size() >= BATCH_GRAPHS) {
            auto lru = g_cache.begin();
            for (auto jt = g_cache.begin(); jt != g_cache.end(); ++jt)
                if (jt->second.used < lru->second.used) lru = jt;
            drop(lru->second);
            g_cache.erase(lru);
        }
        it = g_cache.emplace(key, e).first;
    }
    it->second.used = ++g_clock;
    if (hipGraphLaunch(it->second.exec, (hipStream_t)stream) != hipSuccess) return fail(MW_EHIP, "hipGraphLaunch failed");
    return MW_OK;
}

// Direct (uncaptured) batched launch with an explicit persistent grid; used
// by the tuner and for timing.
extern "C" mw_status mw_sigma_batched_direct(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                                             const void *const *c, void *const *sigma, int32_t blocks_per_cu,
                                             mw_stream_t stream)
{
    BatchSet a;
    bool cplx;
    BatchKey key;
    mw_status st = make_args(nprob, plans, nroots, c, sigma, a, cplx, key);
    if (st != MW_OK) return st;
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(MW_EINVAL, "blocks_per_cu must be in 0..64");
    return launch_batched(a, cplx, num_cu() * blocks_per_cu, (hipStream_t)stream, true);
}

static double time_ms(hipStream_t s, int reps, const std::function<mw_status()> &f, mw_status *err)
{
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    *err = f();  // warm-up
    std::vector<float> ts;
    for (int r = 0; r < reps && *err == MW_OK; r++) {
        hipEventRecord(e0, s);
        *err = f();
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (ts.empty()) return 1e30;
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

// Autotuner for plain sigma: tries the partner-loop unroll and the gather
// width on the caller's vectors, keeps the fastest in the plan.  *choice
// (host, may be NULL) receives unroll * 100 + gather lanes.
extern "C" mw_status mw_autotune(mw_plan plan, int32_t nroots, const void *c, void *sigma, mw_stream_t stream,
                                 int32_t *choice)
{
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    hipStream_t s = (hipStream_t)stream;
    const int us[3] = {4, 8, 16};
    const int gls[3] = {8, 16, 32};
    double best = 1e30;
    int bu = 8, bg = 16;
    mw_status err = MW_OK;
    for (int u : us) {
        if (u == 16 && d->kind == MW_SPINOR) continue;
        for (int gl : gls) {
            mw_internal_set_tune(plan, u, gl);
            double t = time_ms(s, 3, [&]() { return mw_sigma(plan, nroots, c, sigma, stream); }, &err);
            if (err != MW_OK) return err;
            if (t < best) { best = t; bu = u; bg = gl; }
        }
    }
    mw_internal_set_tune(plan, bu, bg);
    if (choice) *choice = bu * 100 + bg;
    return MW_OK;
}

// Autotuner for batched sigma: tries the persistent grid (blocks per CU) or
// the flat grid, the partner unroll of the four-root launch and the gather
// width, keeps the fastest for this batch; the captured graph is rebuilt
// with it.
extern "C" mw_status mw_autotune_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                                         const void *const *c, void *const *sigma, mw_stream_t stream,
                                         int32_t *blocks_per_cu)
{
    BatchSet a;
    bool cplx;
    BatchKey key;
    mw_status st = make_args(nprob, plans, nroots, c, sigma, a, cplx, key);
    if (st != MW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double best = 1e30;
    int bb = 8, bu = 4, bg = 16;
    mw_status err = MW_OK;
    for (int gl : {8, 16, 32}) {
        batch_set_gather(a, gl);
        for (int u4 : {4, 8}) {
            a.u4 = u4;
            // bpc 0: the flat (hardware-dispatched) grid instead of the work queue
            for (int bpc : {0, 1, 2, 4, 8, 16}) {
                double t = time_ms(s, 3, [&]() { return launch_batched(a, cplx, num_cu() * bpc, s, false); }, &err);
                if (err != MW_OK) return err;
                if (t < best) { best = t; bb = bpc; bu = u4; bg = gl; }
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[key] = Tuned{bb, bu, bg};
    if (blocks_per_cu) *blocks_per_cu = bb;
    return MW_OK;
}
