// Energies and gradients of E = c^H H c and of sigma = H c with respect to
// c and the integrals, for the differentiable layer above the ABI.
//
// For the Hamiltonian of section 2.1, Eq. (1), E = sum h_PQ gamma_PQ +
// 1/2 sum (PQ|RS) Gamma_PQRS with gamma, Gamma the density matrices of c, so
//   dE/dh = gamma,  dE/dg = Gamma / 2,  dE/dc = 2 H c.
// sigma = H c is linear in c and in the integrals; for an upstream gradient
// y of sigma its vector-Jacobian products are H y (H Hermitian) and the
// transition density matrices between y and c (conjugated for complex
// problems, the convention of gradients of real losses w.r.t. complex
// inputs: dL = Re sum conj(grad) dz).
//
//  k_energy_part, k_energy_final: e_k = Re sum_I conj(c_Ik) sigma_Ik, a
//      two-stage fixed-order reduction (block partials in the plan's
//      scratch, then one block per root), so repeated calls give the same
//      bits.
//  k_scale_roots: grad_c = 2 ge_k sigma (ge on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "dev_common.h"
#include "mw_internal.h"

namespace mw {

__device__ __forceinline__ double re_dot(double a, double b) { return a * b; }
__device__ __forceinline__ double re_dot(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }

// fixed 256-wide tree reduction in LDS; the result is valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    return lds[0];
}

// block b sums rows [b chunk, (b + 1) chunk) of every root: thread t takes
// rows lo + t, lo + t + 256, ... in order; part[b][k]
template <bool CPLX>
__global__ __launch_bounds__(256) void k_energy_part(int64_t ndet, int R, int64_t chunk,
                                                     const typename Scal<CPLX>::T *__restrict__ c,
                                                     const typename Scal<CPLX>::T *__restrict__ sigma,
                                                     double *__restrict__ part)
{
    __shared__ double lds[256];
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(ndet, lo + chunk);
    for (int k = 0; k < R; k++) {
        double acc = 0.0;
        for (int64_t I = lo + threadIdx.x; I < hi; I += 256) acc += re_dot(c[I * R + k], sigma[I * R + k]);
        const double s = block_sum256(acc, lds);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * R + k] = s;
        __syncthreads();
    }
}

// block k: e[k] = sum over the nblk block partials of root k (fixed order)
__global__ __launch_bounds__(256) void k_energy_final(int nblk, int R, const double *__restrict__ part,
                                                      double *__restrict__ e)
{
    __shared__ double lds[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(int64_t)b * R + k];
    const double s = block_sum256(acc, lds);
    if (threadIdx.x == 0) e[k] = s;
}

// out[I][k] = fac ge[k] x[I][k]
template <typename T>
__global__ __launch_bounds__(256) void k_scale_roots(int64_t n, int R, double fac, const double *__restrict__ ge,
                                                     const T *__restrict__ x, T *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * R) return;
    const double f = fac * ge[t % R];
    if constexpr (sizeof(T) == 16) {
        const double2 v = ((const double2 *)x)[t];
        ((double2 *)out)[t] = make_double2(f * v.x, f * v.y);
    } else {
        out[t] = f * x[t];
    }
}

mw_status launch_energy(const DevPlan &p, int R, const void *c, const void *sigma, double *e, hipStream_t s)
{
    // block partials go to the plan's per-call scratch
    const int64_t cap = (int64_t)(p.scratch_bytes / (8 * (size_t)R));
    const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>({1024, (p.ndet + 255) / 256, cap}));
    const int64_t chunk = (p.ndet + nblk - 1) / nblk;
    double *part = (double *)p.partial;
    if (p.kind == MW_SPINOR)
        hipLaunchKernelGGL(k_energy_part<true>, dim3((unsigned)nblk), dim3(256), 0, s, p.ndet, R, chunk,
                           (const double2 *)c, (const double2 *)sigma, part);
    else
        hipLaunchKernelGGL(k_energy_part<false>, dim3((unsigned)nblk), dim3(256), 0, s, p.ndet, R, chunk,
                           (const double *)c, (const double *)sigma, part);
    hipLaunchKernelGGL(k_energy_final, dim3((unsigned)R), dim3(256), 0, s, (int)nblk, R, (const double *)part, e);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "energy kernel launch failed");
    return MW_OK;
}

// the gradients of L = sum_k ge_k E_k (arguments checked by the caller)
mw_status launch_energy_backward(const DevPlan &p, int R, const void *c, const void *sigma, const double *ge,
                                 void *grad_c, void *grad_h, void *grad_g, hipStream_t s)
{
    if (grad_c) {
        const int64_t n = p.ndet * R;
        const unsigned grid = (unsigned)((n + 255) / 256);
        if (p.kind == MW_SPINOR)
            hipLaunchKernelGGL(k_scale_roots<double2>, dim3(grid), dim3(256), 0, s, p.ndet, R, 2.0, ge,
                               (const double2 *)sigma, (double2 *)grad_c);
        else
            hipLaunchKernelGGL(k_scale_roots<double>, dim3(grid), dim3(256), 0, s, p.ndet, R, 2.0, ge,
                               (const double *)sigma, (double *)grad_c);
        if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "gradient kernel launch failed");
    }
    if (grad_h) return launch_rdm(p, R, c, c, nullptr, ge, grad_h, grad_g, 0.5, true, s);
    return MW_OK;
}

}  // namespace mw

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);

static mw_status bound(mw_plan plan, int32_t nroots, const DevPlan **out)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace: call mw_plan_upload first");
    if (nroots < 1 || nroots > d->max_roots || nroots > 64) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    *out = d;
    return MW_OK;
}

extern "C" {

mw_status mw_energy(mw_plan plan, int32_t nroots, const void *c, const void *sigma, double *e, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound(plan, nroots, &d);
    if (st != MW_OK) return st;
    if (!c || !sigma || !e) return fail(MW_EINVAL, "NULL device pointer");
    if (d->ndet == 0) return fail(MW_EINVAL, "empty space");
    return launch_energy(*d, nroots, c, sigma, e, (hipStream_t)stream);
}

mw_status mw_energy_backward(mw_plan plan, int32_t nroots, const void *c, const void *sigma, const double *ge,
                             void *grad_c, void *grad_h, void *grad_g, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound(plan, nroots, &d);
    if (st != MW_OK) return st;
    if (!c || !ge) return fail(MW_EINVAL, "c and ge must be device pointers");
    if ((grad_h == nullptr) != (grad_g == nullptr)) return fail(MW_EINVAL, "grad_h and grad_g go together");
    if (grad_c && !sigma) return fail(MW_EINVAL, "grad_c needs sigma");
    return launch_energy_backward(*d, nroots, c, sigma, ge, grad_c, grad_h, grad_g, (hipStream_t)stream);
}

mw_status mw_sigma_backward(mw_plan plan, int32_t nroots, const void *c, const void *gs, void *grad_c, void *grad_h,
                            void *grad_g, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound(plan, nroots, &d);
    if (st != MW_OK) return st;
    if (!c || !gs) return fail(MW_EINVAL, "c and gs must be device pointers");
    if ((grad_h == nullptr) != (grad_g == nullptr)) return fail(MW_EINVAL, "grad_h and grad_g go together");
    if (grad_c == gs) return fail(MW_EINVAL, "grad_c and gs must not overlap");
    hipStream_t s = (hipStream_t)stream;
    if (grad_c) {
        st = launch_sigma(*d, nroots, gs, grad_c, s);
        if (st != MW_OK) return st;
    }
    if (grad_h) return launch_rdm(*d, nroots, gs, c, nullptr, nullptr, grad_h, grad_g, 0.5, true, s);
    return MW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of problems
// ---------------------------------------------------------------------------

namespace {

// Captured gradient graphs, keyed by every argument of the call (the kernels
// hold the device pointers); at most GRAD_GRAPHS are kept, the least
// recently used dropped first.
constexpr size_t GRAD_GRAPHS = 16;
struct GradGraph {
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
std::mutex g_grad_mu;
std::vector<GradGraph> g_grad;
uint64_t g_grad_clock = 0;
hipStream_t g_grad_stream = nullptr;
// the second branch of the density-matrix backward inside the captures
hipStream_t g_grad_side = nullptr;
hipEvent_t g_grad_ev[3] = {nullptr, nullptr, nullptr};

void drop_graph(GradGraph &e)
{
    if (e.exec) hipGraphExecDestroy(e.exec);
    if (e.graph) hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

mw_status batch_plans(int32_t nprob, const mw_plan *plans, const int32_t *nroots, std::vector<const DevPlan *> &d)
{
    if (nprob < 1 || nprob > MW_MAXB) return fail(MW_EUNSUPPORTED, "nprob must be in 1..32");
    if (!plans || !nroots) return fail(MW_EINVAL, "NULL argument");
    d.resize(nprob);
    for (int i = 0; i < nprob; i++) {
        d[i] = mw_internal_devplan(plans[i]);
        if (!d[i]) return fail(MW_EWORKSPACE, "plan " + std::to_string(i) + " has no workspace");
        if (nroots[i] < 1 || nroots[i] > d[i]->max_roots || nroots[i] > 64)
            return fail(MW_EINVAL, "nroots out of range for plan " + std::to_string(i));
        for (int j = 0; j < i; j++)
            if (plans[j] == plans[i]) return fail(MW_EINVAL, "a plan may appear once per batch");
    }
    return MW_OK;
}

}  // namespace

// drop the captured gradient graphs that reference a plan (destroyed or
// re-bound)
void mw_internal_grad_forget(mw_plan plan)
{
    std::lock_guard<std::mutex> lk(g_grad_mu);
    for (auto it = g_grad.begin(); it != g_grad.end();) {
        if (!it->key.empty() && std::find(it->key.begin(), it->key.end(), (uintptr_t)plan) != it->key.end()) {
            drop_graph(*it);
            it = g_grad.erase(it);
        } else {
            ++it;
        }
    }
}

extern "C" {

mw_status mw_energy_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots, const void *const *c,
                            const void *const *sigma, double *const *e, mw_stream_t stream)
{
    std::vector<const DevPlan *> d;
    mw_status st = batch_plans(nprob, plans, nroots, d);
    if (st != MW_OK) return st;
    if (!c || !sigma || !e) return fail(MW_EINVAL, "NULL argument");
    for (int i = 0; i < nprob; i++) {
        if (!c[i] || !sigma[i] || !e[i]) return fail(MW_EINVAL, "NULL device pointer");
        if (d[i]->ndet == 0) return fail(MW_EINVAL, "empty space");
    }
    for (int i = 0; i < nprob; i++)
        if ((st = launch_energy(*d[i], nroots[i], c[i], sigma[i], e[i], (hipStream_t)stream)) != MW_OK) return st;
    return MW_OK;
}

mw_status mw_energy_backward_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots, const void *const *c,
                                     const void *const *sigma, const double *const *ge, void *const *grad_c,
                                     void *const *grad_h, void *const *grad_g, mw_stream_t stream)
{
    std::vector<const DevPlan *> d;
    mw_status st = batch_plans(nprob, plans, nroots, d);
    if (st != MW_OK) return st;
    if (!c || !sigma || !ge || !grad_c || !grad_h || !grad_g) return fail(MW_EINVAL, "NULL argument array");
    std::vector<uintptr_t> key;
    for (int i = 0; i < nprob; i++) {
        if (!c[i] || !ge[i]) return fail(MW_EINVAL, "c and ge must be device pointers");
        if ((grad_h[i] == nullptr) != (grad_g[i] == nullptr)) return fail(MW_EINVAL, "grad_h and grad_g go together");
        if (grad_c[i] && !sigma[i]) return fail(MW_EINVAL, "grad_c needs sigma");
        for (uintptr_t v : {(uintptr_t)plans[i], (uintptr_t)nroots[i], (uintptr_t)c[i], (uintptr_t)sigma[i],
                            (uintptr_t)ge[i], (uintptr_t)grad_c[i], (uintptr_t)grad_h[i], (uintptr_t)grad_g[i],
                            (uintptr_t)d[i]->rdm_fixed})
            key.push_back(v);
    }
    std::lock_guard<std::mutex> lk(g_grad_mu);
    GradGraph *hit = nullptr;
    for (auto &e : g_grad)
        if (e.key == key) hit = &e;
    if (!hit) {
        if (!g_grad_stream && hipStreamCreateWithFlags(&g_grad_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(MW_EHIP, "hipStreamCreateWithFlags failed");
        if (!g_grad_side) {
            hipStream_t t = nullptr;
            if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess)
                return fail(MW_EHIP, "hipStreamCreateWithFlags failed");
            for (auto &e : g_grad_ev)
                if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                    return fail(MW_EHIP, "hipEventCreateWithFlags failed");
            g_grad_side = t;
        }
        if (hipStreamBeginCapture(g_grad_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(MW_EHIP, "hipStreamBeginCapture failed");
        {
            ProfSuppress quiet;
            RdmCaptureSide branch(g_grad_side, g_grad_ev[0], g_grad_ev[1], g_grad_ev[2]);
            for (int i = 0; i < nprob && st == MW_OK; i++)
                st = launch_energy_backward(*d[i], nroots[i], c[i], sigma[i], ge[i], grad_c[i], grad_h[i], grad_g[i],
                                            g_grad_stream);
        }
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(g_grad_stream, &g);
        if (st != MW_OK) {
            if (g) hipGraphDestroy(g);
            return st;
        }
        if (ce != hipSuccess || !g) return fail(MW_EHIP, "hipStreamEndCapture failed");
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return fail(MW_EHIP, "hipGraphInstantiate failed");
        }
        if (g_grad.size() >= GRAD_GRAPHS) {
            auto lru = std::min_element(g_grad.begin(), g_grad.end(),
                                        [](const GradGraph &x, const GradGraph &y) { return x.used < y.used; });
            drop_graph(*lru);
            g_grad.erase(lru);
        }
        g_grad.push_back(GradGraph{key, g, ex, 0});
        hit = &g_grad.back();
    }
    hit->used = ++g_grad_clock;
    if (hipGraphLaunch(hit->exec, (hipStream_t)stream) != hipSuccess) return fail(MW_EHIP, "hipGraphLaunch failed");
    return MW_OK;
}

}  // extern "C"
