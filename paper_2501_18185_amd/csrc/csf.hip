// Spin-adapted basis: configuration state functions (CSFs) over the
// configurations of a spin-free plan's determinants (section 2.3: an orbital
// configuration generates several CSFs, told apart by their spin coupling;
// the Yamanouchi-Kotani phase lets doubly occupied orbitals move freely).
//
// Convention (M_S = S, N_alpha - N_beta = 2S).  A configuration is the pair
// (doubly occupied orbitals d_1 < ... < d_m, open orbitals o_1 < ... < o_k).
// Its CSF mu is
//   sum over spin products s of Theta_mu(s) a+_{d_1 a} a+_{d_1 b} ... a+_{d_m b}
//                                           a+_{o_1 s_1} ... a+_{o_k s_k} |vac>,
// Theta_mu the genealogical function of coupling path mu (intermediate spins
// S_1 .. S_k = S, paths ordered lexicographically with the step up first):
// the product of the Clebsch-Gordan coefficients of adding one spin 1/2 at a
// time (Condon-Shortley phase).  Rewriting the operator product in the
// determinant order of the space (ascending positions, alpha orbital p at p,
// beta orbital p at n + p) costs a sign with two factors: one fixed by the
// configuration (m(m-1)/2 + m t + #{(d, o): o < d}, t the open alpha count)
// and one by the spin product (pairs of open shells i < j with s_i beta and
// s_j alpha).  Configurations are numbered in the order of their first
// determinant, CSFs of one configuration by path.
//
// The basis lives inside the span of the space's determinants when every
// determinant of each configuration is present, so with T the [ndet][ncsf]
// expansion sigma_CSF = T^T (H (T c)) exactly: the determinant sigma of the
// plan runs unchanged between two block-diagonal transforms.
//
// Host: configurations by hashing (docc, open), a completeness check, the
// coupling tables per open-shell count k (rows = placements of the t open
// alpha spins, in increasing bit-pattern order; columns = paths), and the
// per-determinant (configuration, sign, placement rank).
// Device: k_csf_to_det (one thread per determinant and root: a row of the
// table times the configuration's CSF coefficients) and k_csf_from_det (one
// thread per CSF and root: a column of the table against the
// configuration's determinants) for configurations of few determinants;
// configurations of CSF_BIG_ROWS determinants or more go by open-shell
// count through k_csf_to_det_cls / k_csf_from_det_cls, which stage a batch
// of configurations in LDS so that each table row is read once per batch
// (the block-diagonal transform is then a product of the shared table with
// the batch's coefficients).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mw_internal.h"

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);
extern "C" int mw_internal_space(mw_plan plan, const uint64_t **dets, int64_t *ndet, int32_t *kind, int32_t *n,
                                 int32_t *na, int32_t *nb);

namespace mw_csf_impl {

constexpr int CSF_MAXOPEN = 14;   // largest table: 14 open shells at S = 1, C(14,8) x 1001 doubles = 24 MB

struct DevCsf {
    int64_t ndet, ncsf, ncfg;
    const uint2 *det_info;     // [ndet] {configuration | negative << 31, placement rank}
    const uint32_t *cfg_det;   // [ncfg+1] offsets into cfg_dets
    const uint32_t *cfg_dets;  // [ndet] determinant | negative << 31, by configuration then rank
    const uint32_t *cfg_csf;   // [ncfg+1] first CSF of each configuration
    const uint32_t *cfg_tab;   // [ncfg] offset of its table (doubles)
    const uint32_t *csf_cfg;   // [ncsf] configuration of each CSF
    const double *tab;         // coupling tables, [placements][paths] per open-shell count
    const double *tabT;        // the same tables transposed, [paths][placements], same offsets
    const uint32_t *cls_dets;  // determinants of the class kernels' configurations (see CsfClass)
    const uint32_t *cls_csf0;  // first CSF of each of those configurations
};

// Configurations with this many determinants or more (8 open shells and up
// at S = 0) are transformed by the class kernels: a block stages a batch of
// configurations of one open-shell count and reads each table row once for
// the whole batch, instead of once per configuration.
constexpr uint32_t CSF_BIG_ROWS = 64;

// the configurations of one open-shell count handled by the class kernels
struct CsfClass {
    const uint32_t *dets;  // [count][nd]: determinant | negative << 31, by configuration then rank
    const uint32_t *csf0;  // [count]: first CSF of each configuration
    uint32_t count, nd, f, toff;
};

template <class T>
size_t take(size_t &off, size_t n)
{
    off = (off + 255) & ~(size_t)255;
    size_t at = off;
    off += n * sizeof(T);
    return at;
}

// <S1 M1; 1/2 ms | S M>, doubled arguments
double cg_half(int s1, int m1, int ms, int s, int m)
{
    if (m1 + ms != m || std::abs(m) > s || std::abs(m1) > s1) return 0.0;
    const double S = 0.5 * s, M = 0.5 * m, h = 0.5 * ms;
    if (s == s1 + 1) return std::sqrt((S + 2.0 * h * M) / (2.0 * S));
    if (s == s1 - 1) return -2.0 * h * std::sqrt((S + 1.0 - 2.0 * h * M) / (2.0 * S + 2.0));
    return 0.0;
}

// coupling paths of k spins ending at 2S = s, step up first
void enumerate_paths(int k, int s, std::vector<int> &cur, std::vector<std::vector<int>> &out)
{
    const int i = (int)cur.size();
    if (i == k) {
        if ((cur.empty() ? 0 : cur.back()) == s) out.push_back(cur);
        return;
    }
    const int b = cur.empty() ? 0 : cur.back();
    for (int step : {1, -1}) {
        const int nb = b + step;
        if (nb < 0 || std::abs(nb - s) > k - i - 1) continue;
        cur.push_back(nb);
        enumerate_paths(k, s, cur, out);
        cur.pop_back();
    }
}

int64_t binom(int n, int r)
{
    if (r < 0 || r > n) return 0;
    int64_t v = 1;
    for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
    return v;
}

struct PairHash {
    size_t operator()(const std::pair<uint64_t, uint64_t> &k) const
    {
        uint64_t x = k.first * 0x9E3779B97F4A7C15ULL ^ (k.second + 0x632BE59BD9B4E019ULL);
        x ^= x >> 31;
        x *= 0xbf58476d1ce4e5b9ULL;
        x ^= x >> 29;
        return (size_t)x;
    }
};

__global__ __launch_bounds__(256) void k_csf_to_det(DevCsf q, int R, const double *__restrict__ x,
                                                     double *__restrict__ y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q.ndet * R) return;
    const int64_t I = t / R;
    const int r = (int)(t - I * R);
    const uint2 info = q.det_info[I];
    const uint32_t cfg = info.x & 0x7fffffffu;
    if (q.cfg_det[cfg + 1] - q.cfg_det[cfg] >= CSF_BIG_ROWS) return;  // class kernel
    const uint32_t c0 = q.cfg_csf[cfg], f = q.cfg_csf[cfg + 1] - c0;
    const double *row = q.tab + q.cfg_tab[cfg] + (size_t)info.y * f;
    const double *xc = x + (size_t)c0 * R + r;
    double acc = 0.0;
    for (uint32_t mu = 0; mu < f; mu++) acc = fma(row[mu], xc[(size_t)mu * R], acc);
    y[t] = (info.x >> 31) ? -acc : acc;
}

__global__ __launch_bounds__(256) void k_csf_from_det(DevCsf q, int R, const double *__restrict__ y,
                                                       double *__restrict__ x)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q.ncsf * R) return;
    const int64_t j = t / R;
    const int r = (int)(t - j * R);
    const uint32_t cfg = q.csf_cfg[j];
    const uint32_t c0 = q.cfg_csf[cfg], f = q.cfg_csf[cfg + 1] - c0, mu = (uint32_t)j - c0;
    const uint32_t d0 = q.cfg_det[cfg], nd = q.cfg_det[cfg + 1] - d0;
    if (nd >= CSF_BIG_ROWS) return;  // class kernel
    const double *col = q.tab + q.cfg_tab[cfg] + mu;
    double acc = 0.0;
    for (uint32_t k = 0; k < nd; k++) {
        const uint32_t e = q.cfg_dets[d0 + k];
        const double v = y[(size_t)(e & 0x7fffffffu) * R + r];
        acc = fma(col[(size_t)k * f], (e >> 31) ? -v : v, acc);
    }
    x[t] = acc;
}

// The class kernels: block column by = a batch of NB configurations of one
// open-shell count (RC roots from r0), grid-strided over the batches; the
// last batch repeats its last configuration in the unused places (computed,
// not written), so the inner loops carry no bounds tests.
// to_det: a thread per table row (placement) accumulates the row times the
// batch's CSF coefficients, staged in LDS, over the paths in increasing
// order (the order of k_csf_to_det, so the values are the same bits).
template <int RC, int NB>
__global__ __launch_bounds__(256) void k_csf_to_det_cls(DevCsf q, CsfClass cl, int R, int r0,
                                                        const double *__restrict__ x, double *__restrict__ y)
{
    extern __shared__ double xs[];  // [NB][f][RC]
    const uint32_t f = cl.f, nd = cl.nd;
    const uint32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t by = blockIdx.y; by * (uint32_t)NB < cl.count; by += gridDim.y) {
        const uint32_t b0 = by * (uint32_t)NB;
        const uint32_t nb = min((uint32_t)NB, cl.count - b0);
        for (uint32_t i = threadIdx.x; i < (uint32_t)NB * f * RC; i += blockDim.x) {
            const uint32_t cb = i / (f * RC), rem = i - cb * f * RC, mu = rem / RC, r = rem - mu * RC;
            xs[i] = x[(size_t)(cl.csf0[b0 + min(cb, nb - 1)] + mu) * R + r0 + r];
        }
        __syncthreads();
        if (row < nd) {
            double acc[NB * RC];
#pragma unroll
            for (int i = 0; i < NB * RC; i++) acc[i] = 0.0;
            const double *col = q.tabT + cl.toff + row;  // T[row][mu] = tabT[mu][row]
#pragma unroll 2
            for (uint32_t mu = 0; mu < f; mu++) {
                const double t = col[(size_t)mu * nd];
#pragma unroll
                for (int i = 0; i < NB * RC; i++) acc[i] = fma(t, xs[((size_t)(i / RC) * f + mu) * RC + i % RC], acc[i]);
            }
#pragma unroll
            for (int cb = 0; cb < NB; cb++)
                if ((uint32_t)cb < nb) {
                    const uint32_t e = cl.dets[(size_t)(b0 + cb) * nd + row];
                    double *out = y + (size_t)(e & 0x7fffffffu) * R + r0;
#pragma unroll
                    for (int r = 0; r < RC; r++) out[r] = (e >> 31) ? -acc[cb * RC + r] : acc[cb * RC + r];
                }
        }
        __syncthreads();
    }
}

// from_det: a thread per path mu accumulates the table column against the
// batch's signed determinant values, staged in LDS, over the placements in
// increasing order (the order of k_csf_from_det).
template <int RC, int NB>
__global__ __launch_bounds__(256) void k_csf_from_det_cls(DevCsf q, CsfClass cl, int R, int r0,
                                                          const double *__restrict__ y, double *__restrict__ x)
{
    extern __shared__ double ys[];  // [NB][nd][RC]
    const uint32_t f = cl.f, nd = cl.nd;
    const uint32_t mu = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t by = blockIdx.y; by * (uint32_t)NB < cl.count; by += gridDim.y) {
        const uint32_t b0 = by * (uint32_t)NB;
        const uint32_t nb = min((uint32_t)NB, cl.count - b0);
        for (uint32_t i = threadIdx.x; i < (uint32_t)NB * nd * RC; i += blockDim.x) {
            const uint32_t cb = i / (nd * RC), rem = i - cb * nd * RC, k = rem / RC, r = rem - k * RC;
            const uint32_t e = cl.dets[(size_t)(b0 + min(cb, nb - 1)) * nd + k];
            const double v = y[(size_t)(e & 0x7fffffffu) * R + r0 + r];
            ys[i] = (e >> 31) ? -v : v;
        }
        __syncthreads();
        if (mu < f) {
            double acc[NB * RC];
#pragma unroll
            for (int i = 0; i < NB * RC; i++) acc[i] = 0.0;
            const double *col = q.tab + cl.toff + mu;
#pragma unroll 2
            for (uint32_t k = 0; k < nd; k++) {
                const double t = col[(size_t)k * f];
#pragma unroll
                for (int i = 0; i < NB * RC; i++) acc[i] = fma(t, ys[((size_t)(i / RC) * nd + k) * RC + i % RC], acc[i]);
            }
#pragma unroll
            for (int cb = 0; cb < NB; cb++)
                if ((uint32_t)cb < nb) {
                    double *out = x + (size_t)(cl.csf0[b0 + cb] + mu) * R + r0;
#pragma unroll
                    for (int r = 0; r < RC; r++) out[r] = acc[cb * RC + r];
                }
        }
        __syncthreads();
    }
}

// D_mu = sum over the configuration's determinants of T_I,mu^2 H_II
__global__ __launch_bounds__(256) void k_csf_diag(DevCsf q, const double *__restrict__ hdiag,
                                                   double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q.ncsf) return;
    const uint32_t cfg = q.csf_cfg[j];
    const uint32_t c0 = q.cfg_csf[cfg], f = q.cfg_csf[cfg + 1] - c0, mu = (uint32_t)j - c0;
    const uint32_t d0 = q.cfg_det[cfg], nd = q.cfg_det[cfg + 1] - d0;
    const double *col = q.tab + q.cfg_tab[cfg] + mu;
    double acc = 0.0;
    for (uint32_t k = 0; k < nd; k++) {
        const double t = col[(size_t)k * f];
        acc = fma(t * t, hdiag[q.cfg_dets[d0 + k] & 0x7fffffffu], acc);
    }
    out[j] = acc;
}

}  // namespace mw_csf_impl

using namespace mw_csf_impl;

struct mw_csf_s {
    mw_plan plan = nullptr;
    int32_t two_s = 0, max_open = 0;
    int64_t ndet = 0, ncsf = 0, ncfg = 0;
    std::vector<uint2> det_info;
    std::vector<uint32_t> cfg_det, cfg_dets, cfg_csf, cfg_tab, csf_cfg;
    std::vector<double> tab, tabT;
    // class kernels: configurations with CSF_BIG_ROWS determinants or more,
    // by open-shell count; the others go through the per-element kernels
    std::vector<uint32_t> cls_dets, cls_csf0;
    struct Cls {
        uint32_t first, count, nd, f, toff;  // first: index of its first configuration in cls_csf0
        size_t dfirst;                       // index of its first determinant in cls_dets
    };
    std::vector<Cls> cls;
    int64_t small_det = 0, small_csf = 0;
    bool bound = false;
    DevCsf dev{};

    size_t layout(DevCsf *d, char *base) const
    {
        size_t off = 0;
        DevCsf t{};
        t.ndet = ndet;
        t.ncsf = ncsf;
        t.ncfg = ncfg;
        size_t a_info = take<uint2>(off, det_info.size()), a_cd = take<uint32_t>(off, cfg_det.size()),
               a_cds = take<uint32_t>(off, cfg_dets.size()), a_cc = take<uint32_t>(off, cfg_csf.size()),
               a_ct = take<uint32_t>(off, cfg_tab.size()), a_sc = take<uint32_t>(off, csf_cfg.size()),
               a_tab = take<double>(off, tab.size()), a_tabT = take<double>(off, tabT.size()),
               a_cld = take<uint32_t>(off, cls_dets.size()), a_clc = take<uint32_t>(off, cls_csf0.size());
        if (d && base) {
            t.det_info = (const uint2 *)(base + a_info);
            t.cfg_det = (const uint32_t *)(base + a_cd);
            t.cfg_dets = (const uint32_t *)(base + a_cds);
            t.cfg_csf = (const uint32_t *)(base + a_cc);
            t.cfg_tab = (const uint32_t *)(base + a_ct);
            t.csf_cfg = (const uint32_t *)(base + a_sc);
            t.tab = (const double *)(base + a_tab);
            t.tabT = (const double *)(base + a_tabT);
            t.cls_dets = (const uint32_t *)(base + a_cld);
            t.cls_csf0 = (const uint32_t *)(base + a_clc);
            *d = t;
        }
        return off + 256;
    }
};

static mw_status build_csf(mw_csf_s &C, const uint64_t *dets, int64_t N, int n, int na, int nb)
{
    const int s = C.two_s;
    // configurations in the order of their first determinant
    std::unordered_map<std::pair<uint64_t, uint64_t>, uint32_t, PairHash> id;
    id.reserve((size_t)N);
    std::vector<uint32_t> of(N);
    std::vector<std::pair<uint64_t, uint64_t>> cfgs;
    for (int64_t i = 0; i < N; i++) {
        const uint64_t A = dets[2 * i], B = dets[2 * i + 1];
        auto key = std::make_pair(A & B, A ^ B);
        auto it = id.find(key);
        if (it == id.end()) {
            it = id.emplace(key, (uint32_t)cfgs.size()).first;
            cfgs.push_back(key);
        }
        of[i] = it->second;
    }
    const int64_t ncfg = (int64_t)cfgs.size();
    // open-shell counts, CSF and determinant offsets
    std::vector<int> kc(ncfg);
    C.cfg_det.assign(ncfg + 1, 0);
    C.cfg_csf.assign(ncfg + 1, 0);
    std::vector<int64_t> fk(CSF_MAXOPEN + 1, 0);
    for (int k = 0; k <= CSF_MAXOPEN; k++)
        if (k >= s && (k - s) % 2 == 0) fk[k] = binom(k, (k - s) / 2) - binom(k, (k - s) / 2 - 1);
    int max_open = 0;
    int64_t ncsf = 0;
    for (int64_t c = 0; c < ncfg; c++) {
        const int k = __builtin_popcountll(cfgs[c].second);
        if (k > CSF_MAXOPEN)
            return fail(MW_EUNSUPPORTED, "a configuration has more than 14 open shells");
        kc[c] = k;
        max_open = std::max(max_open, k);
        const int t = (k + s) / 2;   // open alpha spins (N_alpha - N_beta = 2S)
        C.cfg_det[c + 1] = C.cfg_det[c] + (uint32_t)binom(k, t);
        ncsf += fk[k];
        if (ncsf > 0x7fffffffLL) return fail(MW_EUNSUPPORTED, "more than 2^31 - 1 CSFs");
        C.cfg_csf[c + 1] = (uint32_t)ncsf;
    }
    if ((int64_t)C.cfg_det[ncfg] != N) {
        // some configuration misses determinants: find one to report
        std::vector<uint32_t> cnt(ncfg, 0);
        for (int64_t i = 0; i < N; i++) cnt[of[i]]++;
        for (int64_t c = 0; c < ncfg; c++)
            if (cnt[c] != C.cfg_det[c + 1] - C.cfg_det[c])
                return fail(MW_EINVAL, "configuration " + std::to_string(c) + " (of its first determinant's order) holds " +
                                           std::to_string(cnt[c]) + " of its " +
                                           std::to_string(C.cfg_det[c + 1] - C.cfg_det[c]) +
                                           " determinants: the space must contain every determinant of its configurations");
        return fail(MW_EINVAL, "configuration count mismatch");
    }
    // coupling tables per open-shell count: [placements in increasing
    // alpha-pattern order][paths], each entry the genealogical coefficient
    // times the sign of the open-shell reordering
    std::vector<int64_t> toff(CSF_MAXOPEN + 1, -1);
    std::vector<char> used(CSF_MAXOPEN + 1, 0);
    for (int64_t c = 0; c < ncfg; c++) used[kc[c]] = 1;
    C.tab.clear();
    for (int k = 0; k <= CSF_MAXOPEN; k++) {
        if (!used[k]) continue;
        const int t = (k + s) / 2;
        std::vector<std::vector<int>> paths;
        std::vector<int> cur;
        enumerate_paths(k, s, cur, paths);
        if ((int64_t)paths.size() != fk[k]) return fail(MW_EINVAL, "internal: path count");
        toff[k] = (int64_t)C.tab.size();
        if (C.tab.size() + (size_t)binom(k, t) * paths.size() > 0xffffffffULL)
            return fail(MW_EUNSUPPORTED, "coupling tables too large");
        for (uint32_t pat = 0; pat < (1u << k); pat++) {
            if (__builtin_popcount(pat) != t) continue;
            // open shell i is alpha when bit i of pat is set
            int inv = 0, betas = 0;
            for (int i = 0; i < k; i++) {
                if ((pat >> i) & 1) inv += betas;
                else betas++;
            }
            const double sg = (inv & 1) ? -1.0 : 1.0;
            for (const auto &path : paths) {
                double v = 1.0;
                int b = 0, m = 0;
                for (int i = 0; i < k && v != 0.0; i++) {
                    const int ms = ((pat >> i) & 1) ? 1 : -1;
                    v *= cg_half(b, m, ms, path[i], m + ms);
                    b = path[i];
                    m += ms;
                }
                C.tab.push_back(sg * v);
            }
        }
    }
    C.cfg_tab.resize(ncfg);
    for (int64_t c = 0; c < ncfg; c++) C.cfg_tab[c] = (uint32_t)toff[kc[c]];
    // transposed tables, and the configurations of the class kernels
    C.tabT.assign(C.tab.size(), 0.0);
    C.cls.clear();
    C.cls_dets.clear();
    C.cls_csf0.clear();
    C.small_det = C.small_csf = 0;
    for (int k = 0; k <= CSF_MAXOPEN; k++) {
        if (!used[k]) continue;
        const int64_t nd = binom(k, (k + s) / 2), f = fk[k];
        for (int64_t r = 0; r < nd; r++)
            for (int64_t mu = 0; mu < f; mu++) C.tabT[toff[k] + mu * nd + r] = C.tab[toff[k] + r * f + mu];
        if (nd < (int64_t)CSF_BIG_ROWS) continue;
        mw_csf_s::Cls cl{(uint32_t)C.cls_csf0.size(), 0, (uint32_t)nd, (uint32_t)f, (uint32_t)toff[k], 0};
        for (int64_t c = 0; c < ncfg; c++)
            if (kc[c] == k) C.cls_csf0.push_back((uint32_t)c);  // configuration ids for now
        cl.count = (uint32_t)C.cls_csf0.size() - cl.first;
        C.cls.push_back(cl);
    }
    for (int64_t c = 0; c < ncfg; c++)
        if (C.cfg_det[c + 1] - C.cfg_det[c] < CSF_BIG_ROWS) {
            C.small_det += C.cfg_det[c + 1] - C.cfg_det[c];
            C.small_csf += C.cfg_csf[c + 1] - C.cfg_csf[c];
        }
    C.csf_cfg.resize(ncsf);
    for (int64_t c = 0; c < ncfg; c++)
        for (uint32_t j = C.cfg_csf[c]; j < C.cfg_csf[c + 1]; j++) C.csf_cfg[j] = (uint32_t)c;
    // per determinant: placement rank (combinatorial number system over the
    // open shells) and the configuration's reordering sign
    C.det_info.resize(N);
    C.cfg_dets.assign(N, 0xffffffffu);
    for (int64_t i = 0; i < N; i++) {
        const uint64_t A = dets[2 * i], B = dets[2 * i + 1];
        const uint64_t docc = A & B, open = A ^ B, up = A & ~B;
        const int m = __builtin_popcountll(docc), t = __builtin_popcountll(up);
        int64_t rank = 0;
        int idx = 0, seen = 0;
        for (uint64_t x = open; x; x &= x - 1, idx++) {
            const int p = __builtin_ctzll(x);
            if ((up >> p) & 1) rank += binom(idx, ++seen);
        }
        int64_t below = 0;   // pairs (d, o) with o < d
        for (uint64_t x = docc; x; x &= x - 1) {
            const int d = __builtin_ctzll(x);
            below += __builtin_popcountll(open & ((1ULL << d) - 1));
        }
        const int64_t e = (int64_t)m * (m - 1) / 2 + (int64_t)m * t + below;
        const uint32_t neg = (uint32_t)(e & 1);
        const uint32_t c = of[i];
        if (rank >= (int64_t)(C.cfg_det[c + 1] - C.cfg_det[c])) return fail(MW_EINVAL, "internal: placement rank");
        C.det_info[i] = uint2{c | (neg << 31), (uint32_t)rank};
        uint32_t &slot = C.cfg_dets[C.cfg_det[c] + rank];
        if (slot != 0xffffffffu) return fail(MW_EINVAL, "internal: two determinants share a placement");
        slot = (uint32_t)i | (neg << 31);
    }
    // the class kernels' determinant lists (configuration ids become first CSFs)
    for (auto &cl : C.cls) {
        cl.dfirst = C.cls_dets.size();
        for (uint32_t i = cl.first; i < cl.first + cl.count; i++) {
            const uint32_t c = C.cls_csf0[i];
            C.cls_dets.insert(C.cls_dets.end(), C.cfg_dets.begin() + C.cfg_det[c], C.cfg_dets.begin() + C.cfg_det[c + 1]);
            C.cls_csf0[i] = C.cfg_csf[c];
        }
    }
    (void)n;
    (void)na;
    (void)nb;
    C.ndet = N;
    C.ncsf = ncsf;
    C.ncfg = ncfg;
    C.max_open = max_open;
    return MW_OK;
}

// Device scratch of mw_csf_sigma_noalloc (for callers that cannot allocate):
// the determinant vectors T c and H T c of one call, 2 ndet nroots doubles
// at most CSF_SCRATCH_DOUBLES (32 MiB).  Each device holds its own copy of
// this array from the library's load until the process ends.  Host code
// never passes the array's name to a kernel: its device address is taken
// once per device with hipGetSymbolAddress and kept in g_scratch_dev.
constexpr size_t CSF_SCRATCH_DOUBLES = (size_t)1 << 22;
static __device__ __align__(256) double scratch[CSF_SCRATCH_DOUBLES];

constexpr int CSF_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[CSF_MAX_DEVICES];

// device address of the scratch array on the current device
static mw_status scratch_address(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= CSF_MAX_DEVICES) return fail(MW_EUNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MW_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return MW_OK;
}

static mw_status csf_bound(mw_csf csf, int32_t nroots)
{
    if (!csf) return fail(MW_EINVAL, "csf is NULL");
    if (!csf->bound) return fail(MW_EWORKSPACE, "CSF basis has no workspace: call mw_csf_upload first");
    if (nroots < 1) return fail(MW_EINVAL, "nroots must be >= 1");
    return MW_OK;
}

static unsigned grid_of(int64_t items)
{
    return (unsigned)((items + 255) / 256);
}

// the class kernels for RC roots from r0 (to_det: x CSF -> y determinants)
template <int RC, int NB>
static mw_status launch_cls_nb(const DevCsf &dev, const mw_csf_s::Cls &k, const CsfClass &cl, size_t lds, int R,
                               int r0, const double *in, double *out, hipStream_t s, bool to_det)
{
    if (lds > 64 * 1024) {
        // one configuration of up to 3432 placements and 4 roots (set on the
        // current device before each such launch)
        const void *fn = to_det ? reinterpret_cast<const void *>(&k_csf_to_det_cls<RC, NB>)
                                : reinterpret_cast<const void *>(&k_csf_from_det_cls<RC, NB>);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(MW_EHIP, "CSF class kernel: LDS attribute not set");
    }
    const unsigned ny = (unsigned)std::min<uint32_t>((k.count + NB - 1) / NB, 65535u);
    if (to_det)
        hipLaunchKernelGGL((k_csf_to_det_cls<RC, NB>), dim3((k.nd + 255) / 256, ny), dim3(256), lds, s, dev,
                           cl, R, r0, in, out);
    else {
        const unsigned bx = std::min<unsigned>(256, (k.f + 63) / 64 * 64);
        hipLaunchKernelGGL((k_csf_from_det_cls<RC, NB>), dim3((k.f + bx - 1) / bx, ny), dim3(bx), lds, s,
                           dev, cl, R, r0, in, out);
    }
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "CSF class kernel launch failed");
    return MW_OK;
}

template <int RC>
static mw_status launch_cls_rc(const mw_csf_s &C, int R, int r0, const double *in, double *out, hipStream_t s,
                               bool to_det)
{
    for (const auto &k : C.cls) {
        if (!to_det && k.f == 0) continue;  // no CSF to write (to_det still writes the zeros)
        const CsfClass cl{C.dev.cls_dets + k.dfirst, C.dev.cls_csf0 + k.first, k.count, k.nd, k.f, k.toff};
        // LDS per configuration
        const size_t per = std::max<size_t>(1, (size_t)(to_det ? k.f : k.nd)) * RC * sizeof(double);
        // configurations per block (a power of two): bounded by the
        // accumulators and 48 KB of LDS, and small enough to leave about
        // 512 blocks for the GPU
        const size_t gx = to_det ? (k.nd + 255) / 256 : (k.f + 255) / 256;
        const size_t cap = std::min<size_t>(std::min<size_t>(16 / RC, 49152 / per),
                                            std::max<size_t>(1, (size_t)k.count * gx / 512));
        int nb = 1;
        while (nb * 2 <= (int)cap) nb *= 2;
        const size_t lds = (size_t)nb * per;
        if (lds > 160 * 1024) return fail(MW_EUNSUPPORTED, "CSF class kernel: configuration too large for LDS");
        const DevCsf &d = C.dev;
        mw_status st = MW_OK;
        bool done = false;
        if constexpr (RC == 1)
            if (nb >= 16) st = launch_cls_nb<RC, 16>(d, k, cl, lds, R, r0, in, out, s, to_det), done = true;
        if constexpr (RC <= 2)
            if (!done && nb >= 8) st = launch_cls_nb<RC, 8>(d, k, cl, lds, R, r0, in, out, s, to_det), done = true;
        if (!done && nb >= 4) st = launch_cls_nb<RC, 4>(d, k, cl, lds, R, r0, in, out, s, to_det);
        else if (!done && nb >= 2) st = launch_cls_nb<RC, 2>(d, k, cl, lds, R, r0, in, out, s, to_det);
        else if (!done) st = launch_cls_nb<RC, 1>(d, k, cl, lds, R, r0, in, out, s, to_det);
        if (st != MW_OK) return st;
    }
    return MW_OK;
}

static mw_status launch_cls(const mw_csf_s &C, int R, const double *in, double *out, hipStream_t s, bool to_det)
{
    for (int r0 = 0; r0 < R; r0 += 4) {
        const int rc = std::min(4, R - r0);
        mw_status st = rc == 1   ? launch_cls_rc<1>(C, R, r0, in, out, s, to_det)
                       : rc == 2 ? launch_cls_rc<2>(C, R, r0, in, out, s, to_det)
                       : rc == 3 ? launch_cls_rc<3>(C, R, r0, in, out, s, to_det)
                                 : launch_cls_rc<4>(C, R, r0, in, out, s, to_det);
        if (st != MW_OK) return st;
    }
    return MW_OK;
}

// accessors for the Davidson driver (not exported)
extern "C" __attribute__((visibility("hidden"))) int mw_internal_csf_dims(mw_csf csf, mw_plan *plan, int64_t *ndet,
                                                                         int64_t *ncsf)
{
    if (!csf || !csf->bound) return 0;
    *plan = csf->plan;
    *ndet = csf->ndet;
    *ncsf = csf->ncsf;
    return 1;
}

extern "C" __attribute__((visibility("hidden"))) mw_status mw_internal_csf_diag(mw_csf csf, const double *hdiag,
                                                                               double *out, hipStream_t s)
{
    if (!csf || !csf->bound) return fail(MW_EWORKSPACE, "CSF basis has no workspace");
    if (csf->ncsf == 0) return MW_OK;
    hipLaunchKernelGGL(k_csf_diag, dim3(grid_of(csf->ncsf)), dim3(256), 0, s, csf->dev, hdiag, out);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "CSF kernel launch failed");
    return MW_OK;
}

extern "C" {

mw_status mw_csf_create(mw_plan plan, int32_t two_s, mw_csf *out)
{
    if (!out) return fail(MW_EINVAL, "out is NULL");
    *out = nullptr;
    const uint64_t *dets;
    int64_t N;
    int32_t kind, n, na, nb;
    if (!plan || !mw_internal_space(plan, &dets, &N, &kind, &n, &na, &nb)) return fail(MW_EINVAL, "plan is NULL");
    if (kind != MW_SPIN_FREE) return fail(MW_EUNSUPPORTED, "CSFs are built for spin-free plans");
    if (two_s < 0 || na - nb != two_s)
        return fail(MW_EINVAL, "2S must equal N_alpha - N_beta (CSFs are built at M_S = S)");
    if (N > 0x7fffffffLL) return fail(MW_EUNSUPPORTED, "more than 2^31 - 1 determinants");
    try {
        std::unique_ptr<mw_csf_s> C(new mw_csf_s());
        C->plan = plan;
        C->two_s = two_s;
        mw_status st = build_csf(*C, dets, N, n, na, nb);
        if (st != MW_OK) return st;
        *out = C.release();
    } catch (const std::bad_alloc &) {
        return fail(MW_EUNSUPPORTED, "host memory exhausted while building the CSF basis");
    }
    return MW_OK;
}

int64_t mw_csf_info(mw_csf csf, int32_t what)
{
    if (!csf) return -1;
    switch (what) {
    case 0: return csf->ncsf;
    case 1: return csf->ncfg;
    case 2: return csf->max_open;
    case 3: return (int64_t)csf->layout(nullptr, nullptr);
    case 4: return (int64_t)csf->tab.size();
    case 5: return csf->ndet;
    default: return -1;
    }
}

mw_status mw_csf_workspace_bytes(mw_csf csf, size_t *bytes)
{
    if (!csf || !bytes) return fail(MW_EINVAL, "NULL argument");
    *bytes = csf->layout(nullptr, nullptr);
    return MW_OK;
}

mw_status mw_csf_upload(mw_csf csf, void *workspace, size_t bytes, mw_stream_t stream)
{
    if (!csf || !workspace) return fail(MW_EINVAL, "NULL argument");
    const size_t need = csf->layout(nullptr, nullptr);
    if (bytes < need) return fail(MW_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace) & 255) return fail(MW_EWORKSPACE, "workspace must be 256-byte aligned");
    DevCsf d{};
    csf->layout(&d, (char *)workspace);
    hipStream_t s = (hipStream_t)stream;
    auto up = [&](const void *dst, const void *src, size_t nb) -> bool {
        if (!nb) return true;
        return hipMemcpyAsync((void *)dst, src, nb, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    const mw_csf_s &C = *csf;
    bool ok = up(d.det_info, C.det_info.data(), C.det_info.size() * sizeof(uint2)) &&
              up(d.cfg_det, C.cfg_det.data(), C.cfg_det.size() * 4) &&
              up(d.cfg_dets, C.cfg_dets.data(), C.cfg_dets.size() * 4) &&
              up(d.cfg_csf, C.cfg_csf.data(), C.cfg_csf.size() * 4) &&
              up(d.cfg_tab, C.cfg_tab.data(), C.cfg_tab.size() * 4) &&
              up(d.csf_cfg, C.csf_cfg.data(), C.csf_cfg.size() * 4) && up(d.tab, C.tab.data(), C.tab.size() * 8) &&
              up(d.tabT, C.tabT.data(), C.tabT.size() * 8) && up(d.cls_dets, C.cls_dets.data(), C.cls_dets.size() * 4) &&
              up(d.cls_csf0, C.cls_csf0.data(), C.cls_csf0.size() * 4);
    if (!ok) return fail(MW_EHIP, "hipMemcpyAsync failed during CSF upload");
    // the host vectors are read by the copies above: wait before returning
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "hipStreamSynchronize failed after CSF upload");
    csf->dev = d;
    csf->bound = true;
    return MW_OK;
}

mw_status mw_csf_to_det(mw_csf csf, int32_t nroots, const double *x, double *y, mw_stream_t stream)
{
    mw_status st = csf_bound(csf, nroots);
    if (st != MW_OK) return st;
    if (!x || !y) return fail(MW_EINVAL, "x and y must be device pointers");
    const int64_t items = csf->ndet * nroots;
    if (items == 0) return MW_OK;
    // one dispatch counts its work-items in 32 bits
    if (items > ((int64_t)1 << 32) - 256) return fail(MW_EUNSUPPORTED, "too many determinants x roots");
    if (csf->small_det > 0) {
        hipLaunchKernelGGL(k_csf_to_det, dim3(grid_of(items)), dim3(256), 0, (hipStream_t)stream, csf->dev, nroots, x,
                           y);
        if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "CSF kernel launch failed");
    }
    return launch_cls(*csf, nroots, x, y, (hipStream_t)stream, true);
}

mw_status mw_csf_from_det(mw_csf csf, int32_t nroots, const double *y, double *x, mw_stream_t stream)
{
    mw_status st = csf_bound(csf, nroots);
    if (st != MW_OK) return st;
    if (!x || !y) return fail(MW_EINVAL, "x and y must be device pointers");
    const int64_t items = csf->ncsf * nroots;
    if (items == 0) return MW_OK;
    if (items > ((int64_t)1 << 32) - 256) return fail(MW_EUNSUPPORTED, "too many CSFs x roots");
    if (csf->small_csf > 0) {
        hipLaunchKernelGGL(k_csf_from_det, dim3(grid_of(items)), dim3(256), 0, (hipStream_t)stream, csf->dev, nroots,
                           y, x);
        if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "CSF kernel launch failed");
    }
    return launch_cls(*csf, nroots, y, x, (hipStream_t)stream, false);
}

mw_status mw_csf_sigma(mw_csf csf, int32_t nroots, const double *c, double *sigma, double *work, mw_stream_t stream)
{
    mw_status st = csf_bound(csf, nroots);
    if (st != MW_OK) return st;
    if (!c || !sigma || !work) return fail(MW_EINVAL, "c, sigma and work must be device pointers");
    const DevPlan *d = mw_internal_devplan(csf->plan);
    if (!d) return fail(MW_EWORKSPACE, "the plan has no workspace: call mw_plan_upload first");
    if (nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots of the plan");
    double *cd = work, *sd = work + (size_t)csf->ndet * nroots;
    if ((st = mw_csf_to_det(csf, nroots, c, cd, stream)) != MW_OK) return st;
    if (csf->ndet > 0 && (st = launch_sigma(*d, nroots, cd, sd, (hipStream_t)stream)) != MW_OK) return st;
    return mw_csf_from_det(csf, nroots, sd, sigma, stream);
}

mw_status mw_csf_sigma_noalloc(mw_csf csf, int32_t nroots, const double *c, double *sigma, mw_stream_t stream)
{
    mw_status st = csf_bound(csf, nroots);
    if (st != MW_OK) return st;
    if (!c || !sigma) return fail(MW_EINVAL, "c and sigma must be device pointers");
    const DevPlan *d = mw_internal_devplan(csf->plan);
    if (!d) return fail(MW_EWORKSPACE, "the plan has no workspace: call mw_plan_upload first");
    if (nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots of the plan");
    const size_t need = 2 * (size_t)csf->ndet * (size_t)nroots;
    if (need > CSF_SCRATCH_DOUBLES)
        return fail(MW_EWORKSPACE, "mw_csf_sigma_noalloc: 2 ndet nroots = " + std::to_string(need) +
                                       " doubles exceeds the static scratch of " +
                                       std::to_string(CSF_SCRATCH_DOUBLES) + " doubles; use mw_csf_sigma");
    double *work = nullptr;
    if ((st = scratch_address(&work)) != MW_OK) return st;
    double *cd = work, *sd = work + (size_t)csf->ndet * nroots;
    if ((st = mw_csf_to_det(csf, nroots, c, cd, stream)) != MW_OK) return st;
    if (csf->ndet > 0 && (st = launch_sigma(*d, nroots, cd, sd, (hipStream_t)stream)) != MW_OK) return st;
    return mw_csf_from_det(csf, nroots, sd, sigma, stream);
}

mw_status mw_csf_destroy(mw_csf csf)
{
    delete csf;
    return MW_OK;
}

}  // extern "C"
