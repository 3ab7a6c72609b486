// Host side of libmw: problem validation, the grouping of determinants by
// shared (N-1)/(N-2)-electron strings, integral repacking, workspace layout
// and the C ABI entry points that do not launch kernels themselves.
//
// Grouping (MetaWave section 2.3, reduced pairs and the "bunch" scheme).
// Two determinants I, J with |I ^ J| = 4 (a double excitation) share exactly
// one (N-2)-electron string K = I & J; with |I ^ J| = 2 (a single) they share
// exactly one (N-1)-electron string.  Every determinant D is entered into the
// group of each string D minus one occupied position (N groups) and D minus
// two occupied positions (N(N-1)/2 groups).  Inside a double group each member
// is K plus an added pair (X < Y); members with disjoint pairs are exactly
// the doubly excited pairs with common part K, each pair found in one group
// only.  Inside a single group members are K plus one position, and every two
// members form a single excitation.  Groups with one member are dropped.  The
// phase of every element factorises over the group: with
// pi_K(X) = (-1)^{#K below X},  <I|a+_P a+_R a_S a_Q|J> = phi_I phi_J where
// phi = pi_K(X) pi_K(Y), and <I|a+_P a_Q|J> = pi_K(P) pi_K(Q).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "plan_host.h"

namespace mw {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string &msg) { g_last_error = msg; }
mw_status fail(mw_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

static unsigned n_threads()
{
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 4;
    if (t > 64) t = 64;
    return t;
}

// Run f(begin, end, thread) over [0, n) split into contiguous chunks.
static void parallel_for(int64_t n, const std::function<void(int64_t, int64_t, unsigned)> &f)
{
    unsigned T = n_threads();
    if (n < 4096 || T == 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + T - 1) / T;
    for (unsigned t = 0; t < T; t++) {
        int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(f, b, e, t);
    }
    for (auto &x : th) x.join();
}

// dynamic-scheduled variant for uneven work items
static void parallel_items(int64_t n, const std::function<void(int64_t)> &f)
{
    unsigned T = n_threads();
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; t++)
        th.emplace_back([&]() {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                f(i);
            }
        });
    for (auto &x : th) x.join();
}

// Sort under a strict total order: contiguous chunks in parallel, then
// pairwise merges of neighbouring chunks.
template <class T, class Less>
static void parallel_sort(std::vector<T> &v, Less less)
{
    const int64_t n = (int64_t)v.size();
    const int64_t T_ = std::min<int64_t>(n_threads(), std::max<int64_t>(1, n >> 16));
    if (T_ <= 1) {
        std::sort(v.begin(), v.end(), less);
        return;
    }
    std::vector<int64_t> cut(T_ + 1);
    for (int64_t t = 0; t <= T_; t++) cut[t] = n * t / T_;
    parallel_items(T_, [&](int64_t t) { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1], less); });
    for (int64_t w = 1; w < T_; w *= 2) {
        std::vector<int64_t> jobs;
        for (int64_t t = 0; t + w < T_; t += 2 * w) jobs.push_back(t);
        parallel_items((int64_t)jobs.size(), [&](int64_t k) {
            const int64_t t = jobs[k];
            std::inplace_merge(v.begin() + cut[t], v.begin() + cut[t + w], v.begin() + cut[std::min(t + 2 * w, T_)],
                               less);
        });
    }
}

static inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

struct KeyEntry {
    uint64_t k0, k1;   // the shared string K (two words)
    uint32_t det;
    uint16_t pos;      // X | Y << 8 (Y = 255 for single groups)
    uint16_t pad;
};

static inline bool key_less(const KeyEntry &a, const KeyEntry &b)
{
    if (a.k0 != b.k0) return a.k0 < b.k0;
    if (a.k1 != b.k1) return a.k1 < b.k1;
    return a.det < b.det;
}


// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

// integral symmetry: h Hermitian, (PQ|RS) = (RS|PQ) = conj((QP|SR)); real
// problems 8-fold; all to 1e-12 relative to the largest element
static mw_status validate_integrals(int kind, int n, const double *hin, const double *gin)
{
    if (!hin || !gin) return fail(MW_EINVAL, "h and g must be host pointers");
    if (kind == MW_SPIN_FREE) {
        const double *h = hin, *g = gin;
        double hmax = 0, gmax = 0;
        for (int i = 0; i < n * n; i++) hmax = std::max(hmax, std::fabs(h[i]));
        const size_t n4 = (size_t)n * n * n * n;
        for (size_t i = 0; i < n4; i++) gmax = std::max(gmax, std::fabs(g[i]));
        double th = 1e-12 * std::max(hmax, 1e-300), tg = 1e-12 * std::max(gmax, 1e-300);
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++)
                if (std::fabs(h[a * n + b] - h[b * n + a]) > th)
                    return fail(MW_ESYM, "h is not symmetric");
        std::atomic<bool> bad{false};
        parallel_for(n, [&](int64_t b0, int64_t b1, unsigned) {
            for (int64_t P = b0; P < b1 && !bad; P++)
                for (int Q = 0; Q < n; Q++)
                    for (int R = 0; R < n; R++)
                        for (int S = 0; S < n; S++) {
                            auto G = [&](int a, int b, int c, int e) { return g[(((size_t)a * n + b) * n + c) * n + e]; };
                            double v = G(P, Q, R, S);
                            if (std::fabs(v - G(Q, P, R, S)) > tg || std::fabs(v - G(P, Q, S, R)) > tg ||
                                std::fabs(v - G(R, S, P, Q)) > tg)
                                bad = true;
                        }
        });
        if (bad) return fail(MW_ESYM, "g lacks the real 8-fold permutation symmetry");
    } else {
        const int Mm = 2 * n;
        const std::complex<double> *h = reinterpret_cast<const std::complex<double> *>(hin);
        const std::complex<double> *g = reinterpret_cast<const std::complex<double> *>(gin);
        double hmax = 0, gmax = 0;
        for (int i = 0; i < Mm * Mm; i++) hmax = std::max(hmax, std::abs(h[i]));
        const size_t m4 = (size_t)Mm * Mm * Mm * Mm;
        for (size_t i = 0; i < m4; i++) gmax = std::max(gmax, std::abs(g[i]));
        double th = 1e-12 * std::max(hmax, 1e-300), tg = 1e-12 * std::max(gmax, 1e-300);
        for (int a = 0; a < Mm; a++)
            for (int b = 0; b < Mm; b++)
                if (std::abs(h[a * Mm + b] - std::conj(h[b * Mm + a])) > th)
                    return fail(MW_ESYM, "h is not Hermitian");
        std::atomic<bool> bad{false};
        parallel_for(Mm, [&](int64_t b0, int64_t b1, unsigned) {
            for (int64_t P = b0; P < b1 && !bad; P++)
                for (int Q = 0; Q < Mm; Q++)
                    for (int R = 0; R < Mm; R++)
                        for (int S = 0; S < Mm; S++) {
                            auto G = [&](int a, int b, int c, int e) { return g[(((size_t)a * Mm + b) * Mm + c) * Mm + e]; };
                            std::complex<double> v = G(P, Q, R, S);
                            if (std::abs(v - G(R, S, P, Q)) > tg || std::abs(v - std::conj(G(Q, P, S, R))) > tg)
                                bad = true;
                        }
        });
        if (bad) return fail(MW_ESYM, "g lacks (PQ|RS) = (RS|PQ) = conj((QP|SR))");
    }
    return MW_OK;
}

static mw_status validate(const mw_problem *p, int32_t max_roots)
{
    if (!p) return fail(MW_EINVAL, "problem is NULL");
    if (p->kind != MW_SPIN_FREE && p->kind != MW_SPINOR) return fail(MW_EINVAL, "unknown kind");
    if (p->norb < 1 || p->norb > 64) return fail(MW_EUNSUPPORTED, "norb must be in 1..64");
    if (p->ndet < 1 || p->ndet > 0x7fffffffLL) return fail(MW_EUNSUPPORTED, "ndet must be in 1..2^31-1");
    if (!p->dets || !p->h || !p->g) return fail(MW_EINVAL, "dets, h and g must be host pointers");
    if (max_roots < 1 || max_roots > 64) return fail(MW_EINVAL, "max_roots must be in 1..64");
    const int n = p->norb;
    if (p->kind == MW_SPIN_FREE) {
        if (p->nalpha < 0 || p->nalpha > n || p->nbeta < 0 || p->nbeta > n)
            return fail(MW_EELEC, "electron counts out of range");
    } else {
        if (p->nbeta != -1) return fail(MW_EINVAL, "spinor problems take nbeta = -1");
        if (p->nalpha < 0 || p->nalpha > 2 * n) return fail(MW_EELEC, "electron count out of range");
    }
    const uint64_t mask = n == 64 ? ~0ULL : ((1ULL << n) - 1);
    const uint64_t *d = p->dets;
    for (int64_t i = 0; i < p->ndet; i++) {
        uint64_t a = d[2 * i], b = d[2 * i + 1];
        if ((a & ~mask) || (b & ~mask))
            return fail(MW_EELEC, "determinant " + std::to_string(i) + " has bits beyond norb");
        int na = __builtin_popcountll(a), nb = __builtin_popcountll(b);
        bool ok = p->kind == MW_SPIN_FREE ? (na == p->nalpha && nb == p->nbeta) : (na + nb == p->nalpha);
        if (!ok) return fail(MW_EELEC, "determinant " + std::to_string(i) + " has the wrong electron count");
        if (i > 0) {
            uint64_t pa = d[2 * i - 2], pb = d[2 * i - 1];
            if (!(pa < a || (pa == a && pb < b)))
                return fail(MW_ENOTSORTED, "determinants not strictly ascending at index " + std::to_string(i));
        }
    }
    return validate_integrals(p->kind, n, p->h, p->g);
}

// ---------------------------------------------------------------------------
// grouping
// ---------------------------------------------------------------------------

static inline int occupied_positions(uint64_t w0, uint64_t w1, int n, int *occ)
{
    int k = 0;
    for (uint64_t x = w0; x; x &= x - 1) occ[k++] = __builtin_ctzll(x);
    for (uint64_t x = w1; x; x &= x - 1) occ[k++] = n + __builtin_ctzll(x);
    return k;
}

static inline void remove_pos(uint64_t &w0, uint64_t &w1, int n, int X)
{
    if (X < n) w0 &= ~(1ULL << X);
    else w1 &= ~(1ULL << (X - n));
}

// (-1)^{# of K's positions below global position X}
static inline int pi_sign(uint64_t k0, uint64_t k1, int n, int X)
{
    int c;
    if (X < n) c = __builtin_popcountll(k0 & ((1ULL << X) - 1));
    else {
        int b = X - n;
        c = __builtin_popcountll(k0) + __builtin_popcountll(k1 & (b == 64 ? ~0ULL : ((1ULL << b) - 1)));
    }
    return (c & 1) ? -1 : 1;
}

static mw_status build_groups(HostPlan &P)
{
    const int n = P.n;
    const int64_t N = P.ndet;
    const int nel = P.kind == MW_SPIN_FREE ? P.nalpha + P.nbeta : P.nalpha;
    const int64_t per_det = nel + (int64_t)nel * (nel - 1) / 2;
    const int64_t total = N * per_det;
    if (nel == 0 || total == 0) {
        P.grp_off.assign(1, 0);
        P.pk_off.assign(1, 0);
        P.rowptr.assign(N + 1, 0);
        return MW_OK;
    }
    const int PB = 10;                      // 1024 hash partitions
    const int NPART = 1 << PB;
    const unsigned T = n_threads();
    const int64_t chunk = (N + T - 1) / T;
    std::vector<int64_t> counts((size_t)T * NPART, 0);

    auto for_each_key = [&](int64_t i, auto &&emit) {
        int occ[128];
        uint64_t w0 = P.dets[2 * i], w1 = P.dets[2 * i + 1];
        int k = occupied_positions(w0, w1, n, occ);
        for (int a = 0; a < k; a++) {
            uint64_t k0 = w0, k1 = w1;
            remove_pos(k0, k1, n, occ[a]);
            emit(k0, k1, (uint16_t)(occ[a] | (255 << 8)));
            for (int b = a + 1; b < k; b++) {
                uint64_t m0 = k0, m1 = k1;
                remove_pos(m0, m1, n, occ[b]);
                emit(m0, m1, (uint16_t)(occ[a] | (occ[b] << 8)));
            }
        }
    };
    auto part_of = [&](uint64_t k0, uint64_t k1) { return (int)(mix64(k0 ^ mix64(k1 + 0x9E3779B97F4A7C15ULL)) >> (64 - PB)); };

    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; t++)
        th.emplace_back([&, t]() {
            int64_t b = t * chunk, e = std::min<int64_t>(N, b + chunk);
            int64_t *cnt = &counts[(size_t)t * NPART];
            for (int64_t i = b; i < e; i++)
                for_each_key(i, [&](uint64_t k0, uint64_t k1, uint16_t) { cnt[part_of(k0, k1)]++; });
        });
    for (auto &x : th) x.join();
    th.clear();
    // offsets: partition-major, thread-minor
    std::vector<int64_t> off((size_t)T * NPART);
    std::vector<int64_t> part_start(NPART + 1, 0);
    int64_t acc = 0;
    for (int p = 0; p < NPART; p++) {
        part_start[p] = acc;
        for (unsigned t = 0; t < T; t++) {
            off[(size_t)t * NPART + p] = acc;
            acc += counts[(size_t)t * NPART + p];
        }
    }
    part_start[NPART] = acc;
    std::vector<KeyEntry> ent;
    try {
        ent.resize((size_t)total);
    } catch (...) {
        return fail(MW_EUNSUPPORTED, "host memory exhausted while grouping determinants");
    }
    for (unsigned t = 0; t < T; t++)
        th.emplace_back([&, t]() {
            int64_t b = t * chunk, e = std::min<int64_t>(N, b + chunk);
            int64_t *o = &off[(size_t)t * NPART];
            for (int64_t i = b; i < e; i++)
                for_each_key(i, [&](uint64_t k0, uint64_t k1, uint16_t pos) {
                    int p = part_of(k0, k1);
                    ent[o[p]++] = KeyEntry{k0, k1, (uint32_t)i, pos, 0};
                });
        });
    for (auto &x : th) x.join();
    th.clear();

    // sort each partition; collect runs of length >= 2 with their ordering
    // keys: single or double, kind (which spins lost the electrons), first
    // member (the smallest determinant index)
    struct Run { int64_t start; uint32_t len, det; uint8_t single, kind; };
    std::vector<std::vector<Run>> runs(NPART);
    parallel_items(NPART, [&](int64_t p) {
        auto b = ent.begin() + part_start[p], e = ent.begin() + part_start[p + 1];
        std::sort(b, e, key_less);
        int64_t s = part_start[p], E = part_start[p + 1];
        while (s < E) {
            int64_t t = s + 1;
            while (t < E && ent[t].k0 == ent[s].k0 && ent[t].k1 == ent[s].k1) t++;
            if (t - s >= 2) {
                const int X = ent[s].pos & 255, Y = ent[s].pos >> 8;
                const uint8_t single = Y == 255;
                const uint8_t kind = single ? (X < n ? 0 : 1) : ((X < n && Y < n) ? 0 : (X >= n && Y >= n) ? 1 : 2);
                runs[p].push_back(Run{s, (uint32_t)(t - s), ent[s].det, single, kind});
            }
            s = t;
        }
    });
    std::vector<Run> all;
    for (auto &r : runs) all.insert(all.end(), r.begin(), r.end());
    runs.clear();
    runs.shrink_to_fit();
    // double groups before single groups, largest first within each class
    // (longest-processing-time order).  Groups of one size are ordered by
    // kind and then by their first member, so that determinants close in the
    // given order find their partial sums close together when the gather
    // reads them (and a packet's members read neighbouring coefficients);
    // remaining ties by the shared string K (first word, then second), so the
    // order is total and does not depend on how the keys were partitioned.
    parallel_sort(all, [&](const Run &a, const Run &b) {
        if (a.single != b.single) return a.single < b.single;
        if (a.len != b.len) return a.len > b.len;
        if (a.kind != b.kind) return a.kind < b.kind;
        if (a.det != b.det) return a.det < b.det;
        return key_less(ent[a.start], ent[b.start]);
    });

    const int64_t ngroup = (int64_t)all.size();
    P.grp_off.resize(ngroup + 1);
    int64_t m = 0;
    for (int64_t gi = 0; gi < ngroup; gi++) {
        P.grp_off[gi] = (uint32_t)m;
        m += all[gi].len;
        if (m > 0xffffffffLL) return fail(MW_EUNSUPPORTED, "more than 2^32 group memberships");
    }
    P.grp_off[ngroup] = (uint32_t)m;
    const int64_t nmem = m;
    P.grp_key.resize(2 * ngroup);
    P.grp_type.resize(ngroup);
    P.mem.resize(nmem);
    P.mem_grp.resize(nmem);
    std::vector<int64_t> single_pairs(ngroup), double_pairs(ngroup);
    parallel_items((ngroup + 1023) / 1024, [&](int64_t blk) {
        int64_t g0 = blk * 1024, g1 = std::min<int64_t>(ngroup, g0 + 1024);
        std::vector<int> freq(128);
        for (int64_t gi = g0; gi < g1; gi++) {
            const Run &r = all[gi];
            const KeyEntry &e0 = ent[r.start];
            uint64_t k0 = e0.k0, k1 = e0.k1;
            P.grp_key[2 * gi] = k0;
            P.grp_key[2 * gi + 1] = k1;
            int X0 = e0.pos & 255, Y0 = e0.pos >> 8;
            bool single = Y0 == 255;
            uint8_t type;
            if (P.kind == MW_SPIN_FREE) {
                if (single) type = X0 < n ? G_SINGLE_A : G_SINGLE_B;
                else type = (X0 < n && Y0 < n) ? G_AA : (X0 >= n && Y0 >= n) ? G_BB : G_AB;
            } else {
                type = single ? G_SINGLE_S : G_DOUBLE_S;
            }
            P.grp_type[gi] = type;
            std::fill(freq.begin(), freq.end(), 0);
            for (uint32_t t = 0; t < r.len; t++) {
                const KeyEntry &e = ent[r.start + t];
                int X = e.pos & 255, Y = e.pos >> 8;
                int phi = pi_sign(k0, k1, n, X) * (single ? 1 : pi_sign(k0, k1, n, Y));
                int64_t mi = P.grp_off[gi] + t;
                P.mem[mi] = uint2{e.det, (uint32_t)(X | (Y << 8) | (phi < 0 ? (1u << 16) : 0u))};
                P.mem_grp[mi] = (uint32_t)gi;
                freq[X]++;
                if (!single) freq[Y]++;
            }
            int64_t k = r.len;
            if (!single) {
                // integral layout per member: the kernel reads the integrals
                // of member i at a column of a row fixed by the partner, so
                // the members of one wave should sit at neighbouring
                // columns.  Within the member's 64-member window (its packet)
                // count the members sharing its first added position X and
                // those sharing the second Y; the larger run decides which
                // index varies fastest: layout 0 keeps Y fastest for
                // alpha-beta groups (X fastest for pair tables, colex order),
                // layout 1 is the transposed column order.
                const bool ab = type == G_AB;
                const int64_t g0 = P.grp_off[gi];
                for (uint32_t t = 0; t < r.len; t++) {
                    const int64_t w0 = g0 + (t / 64) * 64, w1 = std::min<int64_t>(g0 + r.len, w0 + 64);
                    const int64_t mi = g0 + t;
                    const int X = P.mem[mi].y & 255, Y = (P.mem[mi].y >> 8) & 255;
                    int cx = 0, cy = 0;
                    for (int64_t o = w0; o < w1; o++) {
                        if (o == mi) continue;
                        cx += (int)((P.mem[o].y & 255) == (uint32_t)X);
                        cy += (int)(((P.mem[o].y >> 8) & 255) == (uint32_t)Y);
                    }
                    // X shared -> Y varies: alpha-beta layout 0, pairs layout 1
                    const int lay = cx >= cy ? (ab ? 0 : 1) : (ab ? 1 : 0);
                    if (lay == 1) P.mem[mi].y |= 1u << 17;
                }
                // groups of fewer than 64 members (double and single): the
                // member's index in the group (bits 18-23) and the group size
                // (bits 24-29), so the kernels find the partners without the
                // group tables; 0 in bits 24-29 marks a large group
                if (k < 64)
                    for (uint32_t t = 0; t < r.len; t++) P.mem[g0 + t].y |= (t << 18) | ((uint32_t)k << 24);
            }
            if (single) {
                single_pairs[gi] = k * (k - 1);
                // as for double groups: index in the group and group size
                if (k < 64) {
                    const int64_t s0 = P.grp_off[gi];
                    for (uint32_t t = 0; t < r.len; t++) P.mem[s0 + t].y |= (t << 18) | ((uint32_t)k << 24);
                }
            } else {
                int64_t dp = 0;
                for (uint32_t t = 0; t < r.len; t++) {
                    const KeyEntry &e = ent[r.start + t];
                    int X = e.pos & 255, Y = e.pos >> 8;
                    dp += k - (freq[X] + freq[Y] - 1);
                }
                double_pairs[gi] = dp;
            }
        }
    });
    ent.clear();
    ent.shrink_to_fit();
    P.n_single_pairs = P.n_double_pairs = P.n_evals = P.n_double_pairs_large = 0;
    for (int64_t gi = 0; gi < ngroup; gi++) {
        P.n_single_pairs += single_pairs[gi];
        P.n_double_pairs += double_pairs[gi];
        if (all[gi].len >= 64) P.n_double_pairs_large += double_pairs[gi];
        P.n_evals += (int64_t)all[gi].len * all[gi].len;
    }
    // packets: <= 64 consecutive members; large groups are cut into chunks of
    // 64, small groups are packed whole
    P.pk_off.clear();
    P.pk_off.push_back(0);
    P.npacket_double = 0;
    {
        uint32_t cur_start = 0, cur_cnt = 0;
        bool in_single = false;
        for (int64_t gi = 0; gi < ngroup; gi++) {
            uint32_t k = all[gi].len, s = P.grp_off[gi];
            const uint8_t ty = P.grp_type[gi];
            if (!in_single && (ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S)) {
                in_single = true;
                // class boundary: close the open packet; packets before this
                // point hold double groups only
                if (cur_cnt) { P.pk_off.push_back(cur_start + cur_cnt); cur_cnt = 0; }
                P.npacket_double = (int64_t)P.pk_off.size() - 1;
                cur_start = s;
            }
            if (k >= 64) {
                if (cur_cnt) { P.pk_off.push_back(cur_start + cur_cnt); cur_cnt = 0; }
                for (uint32_t c = 0; c < k; c += 64) P.pk_off.push_back(s + std::min<uint32_t>(k, c + 64));
                cur_start = s + k;
            } else {
                if (cur_cnt + k > 64) { P.pk_off.push_back(cur_start + cur_cnt); cur_start += cur_cnt; cur_cnt = 0; }
                if (cur_cnt == 0) cur_start = s;
                cur_cnt += k;
            }
        }
        if (cur_cnt) P.pk_off.push_back(cur_start + cur_cnt);
        if (!in_single) P.npacket_double = (int64_t)P.pk_off.size() - 1;
    }
    // one wave per packet in one dispatch, whose work-item count is 32 bits
    if (((int64_t)P.pk_off.size() + 1024) * 64 > 0xffffffffLL)
        return fail(MW_EUNSUPPORTED, "too many packets for one launch");
    // Column partials of large double groups (k >= 64).  Their packets are
    // the 64-member blocks of the group; the wave of block a evaluates each
    // unordered pair with a partner in a block b >= a once (Hermiticity), keeps
    // the row sum and hands H_ji c_i summed over its lanes to member j of
    // block b > a through slot col(a, j) = nmem + grp_col[g] + a k -
    // 32 a (a + 1) + (t_j - 64 (a + 1)), t_j the member's index in the group.
    P.grp_col.assign(ngroup, 0);
    int64_t ncol = 0;
    for (int64_t gi = 0; gi < ngroup; gi++) {
        const int64_t k = (int64_t)P.grp_off[gi + 1] - P.grp_off[gi];
        const uint8_t ty = P.grp_type[gi];
        if (k < 64 || ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S) continue;
        P.grp_col[gi] = (uint32_t)ncol;
        const int64_t nb = (k + 63) / 64;
        for (int64_t a = 0; a + 1 < nb; a++) ncol += k - 64 * (a + 1);
        if (nmem + ncol > 0xffffffffLL) return fail(MW_EUNSUPPORTED, "too many partial sums");
    }
    P.ncol = ncol;
    // determinant-major list of each determinant's partial sums: its
    // memberships (row sums) and the column partials of its large groups
    P.rowptr.assign(N + 1, 0);
    for (int64_t mi = 0; mi < nmem; mi++) {
        const uint32_t gi = P.mem_grp[mi];
        const int64_t t = (int64_t)mi - P.grp_off[gi];
        const int64_t k = (int64_t)P.grp_off[gi + 1] - P.grp_off[gi];
        const uint8_t ty = P.grp_type[gi];
        const bool big = k >= 64 && !(ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S);
        P.rowptr[P.mem[mi].x + 1] += 1 + (big ? t / 64 : 0);
    }
    for (int64_t i = 0; i < N; i++) P.rowptr[i + 1] += P.rowptr[i];
    // Placement of the partial sums.  A logical slot (membership m, or nmem
    // plus a column-partial index) is stored at slot_pos[slot].  Positions
    // are grouped in regions of consecutive determinants holding about 2 MB
    // of partials: determinant i belongs to region rowptr[i] / reg_slots
    // (the gather gives each XCD a contiguous eighth of the
    // determinants, so the region it is summing stays in its L2), and inside
    // a region by the XCD whose waves write them, in packet order: every
    // region has one write frontier per XCD, written by that XCD only, whose
    // lines fill in its L2 before they are written back.
    const int64_t nslot = nmem + ncol;
    const int sbytes = (P.cplx ? 16 : 8) * P.max_roots;
    const int64_t reg_slots = std::max<int64_t>(4096, ((int64_t)2 << 20) / sbytes);
    std::vector<uint32_t> reg_of(N);
    for (int64_t i = 0; i < N; i++) reg_of[i] = (uint32_t)(P.rowptr[i] / reg_slots);
    const int64_t nreg = N > 0 ? (int64_t)reg_of[N - 1] + 1 : 1;
    // writer XCD of a packet: double-group packets w are launched with the
    // XCD-aware block order (logical block w / 4 runs on XCD (w / 64) % 8),
    // single-group packets in plain order (block (w - npd) / 4 on XCD
    // block % 8)
    const int64_t npk = (int64_t)P.pk_off.size() - 1, npd = P.npacket_double;
    auto xcd_of = [&](int64_t w) -> int { return w < npd ? (int)((w / 64) % 8) : (int)(((w - npd) / 4) % 8); };
    // the column-partial slots written by a packet: block a of a large
    // double group writes [col0, col0 + k - 64 (a + 1))
    auto col_range = [&](int64_t w, int64_t &c0, int64_t &c1, uint32_t &g, int64_t &k, int64_t &a) {
        c0 = c1 = 0;
        const uint32_t m0 = P.pk_off[w];
        g = P.mem_grp[m0];
        k = (int64_t)P.grp_off[g + 1] - P.grp_off[g];
        const uint8_t ty = P.grp_type[g];
        if (w >= npd || k < 64 || ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S) return;
        a = ((int64_t)m0 - P.grp_off[g]) / 64;
        c0 = nmem + P.grp_col[g] + a * k - 32 * a * (a + 1);
        c1 = c0 + (k - 64 * (a + 1));
    };
    std::vector<int64_t> start((size_t)nreg * 8 + 1, 0);
    for (int64_t w = 0; w < npk; w++) {
        const int x = xcd_of(w);
        for (uint32_t m = P.pk_off[w]; m < P.pk_off[w + 1]; m++) start[(size_t)reg_of[P.mem[m].x] * 8 + x + 1]++;
        int64_t c0, c1, k, a;
        uint32_t g;
        col_range(w, c0, c1, g, k, a);
        for (int64_t cs = c0; cs < c1; cs++) {
            const int64_t t = 64 * (a + 1) + (cs - c0);  // partner j's index in the group
            start[(size_t)reg_of[P.mem[P.grp_off[g] + t].x] * 8 + x + 1]++;
        }
    }
    for (size_t i = 1; i < start.size(); i++) start[i] += start[i - 1];
    if (start.back() != nslot) return fail(MW_EINVAL, "internal: partial slots miscounted");
    P.slot_pos.assign((size_t)nslot, 0);
    for (int64_t w = 0; w < npk; w++) {
        const int x = xcd_of(w);
        for (uint32_t m = P.pk_off[w]; m < P.pk_off[w + 1]; m++)
            P.slot_pos[m] = (uint32_t)start[(size_t)reg_of[P.mem[m].x] * 8 + x]++;
        int64_t c0, c1, k, a;
        uint32_t g;
        col_range(w, c0, c1, g, k, a);
        for (int64_t cs = c0; cs < c1; cs++) {
            const int64_t t = 64 * (a + 1) + (cs - c0);
            P.slot_pos[cs] = (uint32_t)start[(size_t)reg_of[P.mem[P.grp_off[g] + t].x] * 8 + x]++;
        }
    }
    std::vector<uint32_t> fillc(P.rowptr.begin(), P.rowptr.end() - 1);
    P.slot_mem.resize(P.rowptr[N]);
    for (int64_t mi = 0; mi < nmem; mi++) {
        const uint32_t det = P.mem[mi].x;
        P.slot_mem[fillc[det]++] = P.slot_pos[mi];
        const uint32_t gi = P.mem_grp[mi];
        const int64_t t = (int64_t)mi - P.grp_off[gi];
        const int64_t k = (int64_t)P.grp_off[gi + 1] - P.grp_off[gi];
        const uint8_t ty = P.grp_type[gi];
        if (k < 64 || ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S) continue;
        for (int64_t a = 0; a < t / 64; a++)
            P.slot_mem[fillc[det]++] = P.slot_pos[nmem + P.grp_col[gi] + a * k - 32 * a * (a + 1) + (t - 64 * (a + 1))];
    }
    return MW_OK;
}

// ---------------------------------------------------------------------------
// integral repacking
// ---------------------------------------------------------------------------

static inline int pair_index(int lo, int hi) { return hi * (hi - 1) / 2 + lo; }
// lexicographic index of the pair lo < hi among m positions
static inline int pair_lex(int lo, int hi, int m) { return lo * (2 * m - lo - 1) / 2 + (hi - lo - 1); }

// ---------------------------------------------------------------------------
// density-matrix rows
// ---------------------------------------------------------------------------

// The double-pair accumulators of the density matrices are filled row by
// row.  The row of a connected pair (I, J) is the pair added in J: alpha-beta
// (X, Y) -> X n + Y - n, same-spin and spinor pairs -> their colex index
// (after the n^2 alpha-beta rows of a spin-free plan).  Every double
// membership j is listed under its row, as the partner of the pairs it forms
// with the other members of its group; one workgroup sums a run of a row's
// list in LDS and adds the row to the accumulator once, instead of one
// device atomic per pair.  A row's list holds first the memberships of
// groups of RDM_WIDE members or more (a wave walks the group, a member per
// lane), then the others by increasing group size (a lane per membership,
// so that the lanes of a wave loop alike), each in membership order; the
// lists are cut into chunks of about RDM_CHUNK_WORK partner visits, the
// alpha-beta chunks first, each class by decreasing work.  The single
// memberships are listed the same way under the row of their added orbital
// (spin-free, both spins) or spinor, whose accumulators (S, C, E) are
// indexed by the partner's position first.
static mw_status build_rdm_rows(HostPlan &P)
{
    P.rdm_ent.clear();
    P.rdm_chunk.clear();
    P.rdm_pos.clear();
    P.rdm_ent_det.clear();
    P.rdm_skey.clear();
    P.rdm_single_e0 = 0;
    for (auto &c : P.rdm_cls) c = 0;
    const int64_t nmd = P.npacket_double > 0 ? (int64_t)P.pk_off[P.npacket_double] : 0;
    const int64_t nmem = (int64_t)P.mem.size();
    P.nmem_double = nmd;
    if (nmem == 0) return MW_OK;
    const int n = P.n;
    const bool sf = P.kind == MW_SPIN_FREE;
    // pairs of same-spin orbitals (spin-free) or of spinors (set again by repack)
    const int64_t npair = sf ? (int64_t)n * (n - 1) / 2 : (int64_t)P.M * (P.M - 1) / 2;
    const int64_t nab = sf ? (int64_t)n * n : 0, nrow_d = nab + npair;
    // single rows: the partner's added orbital (spin-free, both spins) or spinor
    const int64_t nrow = nrow_d + (sf ? n : P.M);
    constexpr int NC = RDM_WIDE;  // class 0: wide groups; class L: groups of L < RDM_WIDE members
    std::vector<uint32_t> key((size_t)nmem);
    parallel_for(nmem, [&](int64_t b0, int64_t b1, unsigned) {
        for (int64_t j = b0; j < b1; j++) {
            const uint32_t g = P.mem_grp[j];
            const uint32_t L = P.grp_off[g + 1] - P.grp_off[g];
            if (L < 2) { key[j] = 0xffffffffu; continue; }
            const int X = P.mem[j].y & 255, Y = (P.mem[j].y >> 8) & 255;
            const uint8_t ty = P.grp_type[g];
            int64_t row;
            if (j >= nmd) row = nrow_d + (ty == G_SINGLE_B ? X - n : X);
            else if (!sf) row = pair_index(X, Y);
            else if (ty == G_AB) row = (int64_t)X * n + (Y - n);
            else row = nab + (ty == G_BB ? pair_index(X - n, Y - n) : pair_index(X, Y));
            key[j] = (uint32_t)(row * NC + (L >= (uint32_t)RDM_WIDE ? 0 : L));
        }
    });
    // stable counting sort by key, in parallel: per-thread counts over the
    // contiguous membership ranges of parallel_for, then each thread
    // scatters its range from its own offsets (membership order kept)
    const int64_t nbin = nrow * NC;
    const unsigned T = n_threads();
    std::vector<uint32_t> cnt((size_t)T * nbin, 0);
    std::atomic<bool> too_large{false};
    parallel_for(nmem, [&](int64_t b0, int64_t b1, unsigned t) {
        uint32_t *c = cnt.data() + (size_t)t * nbin;
        for (int64_t j = b0; j < b1; j++) {
            if (key[j] == 0xffffffffu) continue;
            c[key[j]]++;
            const uint32_t g = P.mem_grp[j];
            if (P.grp_off[g + 1] - P.grp_off[g] >= 65536) too_large = true;
        }
    });
    if (too_large) return fail(MW_EUNSUPPORTED, "group too large for the density rows");
    std::vector<int64_t> start((size_t)(nbin + 1), 0);
    {
        int64_t acc = 0;
        for (int64_t b = 0; b < nbin; b++) {
            start[b] = acc;
            for (unsigned t = 0; t < T; t++) {
                const uint32_t c = cnt[(size_t)t * nbin + b];
                cnt[(size_t)t * nbin + b] = (uint32_t)acc;  // this thread's first slot in bin b
                acc += c;
                if (acc > 0xffffffffLL) return fail(MW_EUNSUPPORTED, "too many memberships for the density rows");
            }
        }
        start[nbin] = acc;
    }
    const int64_t nent = start.back();
    if (P.ndet >= (int64_t)1 << 31) return fail(MW_EUNSUPPORTED, "too many determinants for the density rows");
    P.rdm_ent.resize((size_t)nent);
    P.rdm_ent_det.resize((size_t)nent);
    parallel_for(nmem, [&](int64_t b0, int64_t b1, unsigned t) {
        uint32_t *fill = cnt.data() + (size_t)t * nbin;
        for (int64_t j = b0; j < b1; j++) {
            if (key[j] == 0xffffffffu) continue;
            const uint32_t g = P.mem_grp[j];
            const uint32_t j0 = P.grp_off[g], L = P.grp_off[g + 1] - j0;
            const int64_t e = fill[key[j]]++;
            P.rdm_ent[e] = make_uint2(j0, (uint32_t)(j - j0) | (L << 16));
            // the partner's determinant and sign (bit 31)
            P.rdm_ent_det[e] = P.mem[j].x | (((P.mem[j].y >> 16) & 1u) << 31);
        }
    });
    cnt.clear();
    cnt.shrink_to_fit();
    // single entries (the rows after the double rows): the group's string K
    // and the spin of a spin-free group, so the kernel reads no group table
    P.rdm_single_e0 = start[nrow_d * NC];
    P.rdm_skey.resize((size_t)(nent - P.rdm_single_e0));
    parallel_for(nent - P.rdm_single_e0, [&](int64_t b0, int64_t b1, unsigned) {
        for (int64_t t = b0; t < b1; t++) {
            uint2 &en = P.rdm_ent[P.rdm_single_e0 + t];
            const uint32_t g = P.mem_grp[en.x];
            P.rdm_skey[t] = make_ulonglong2(P.grp_key[2 * (size_t)g], P.grp_key[2 * (size_t)g + 1]);
            if (P.grp_type[g] == G_SINGLE_B) en.y |= 1u << 15;
        }
    });
    key.clear();
    key.shrink_to_fit();
    P.rdm_pos.resize((size_t)nmem);
    parallel_for(nmem, [&](int64_t b0, int64_t b1, unsigned) {
        for (int64_t j = b0; j < b1; j++) P.rdm_pos[j] = (uint16_t)(P.mem[j].y & 0xffffu);
    });
    struct Ch {
        uint4 c;
        int64_t work;
    };
    // alpha-beta wide, alpha-beta small, pair wide, pair small, singles
    std::vector<Ch> cls[5];
    for (int64_t row = 0; row < nrow; row++) {
        for (int part = 0; part < 2; part++) {
            // part 0: the wide class; part 1: classes 1 .. NC-1 (contiguous)
            const int64_t e0 = start[row * NC + (part ? 1 : 0)], e1 = start[row * NC + (part ? NC : 1)];
            const uint32_t flags = row < nab ? 1u : 0u;
            const uint32_t r = (uint32_t)(row < nab ? row : (row < nrow_d ? row - nab : row - nrow_d));
            std::vector<Ch> &out = cls[row >= nrow_d ? 4 : (row < nab ? 0 : 2) + part];
            int64_t a = e0, work = 0;
            for (int64_t e = e0; e < e1; e++) {
                work += (P.rdm_ent[e].y >> 16) - 1;
                if (work >= RDM_CHUNK_WORK || e + 1 == e1) {
                    out.push_back(Ch{make_uint4(r, flags, (uint32_t)a, (uint32_t)(e + 1)), work});
                    a = e + 1;
                    work = 0;
                }
            }
        }
    }
    auto by_work = [](const Ch &x, const Ch &y) { return x.work > y.work; };
    size_t tot = 0;
    for (auto &v : cls) tot += v.size();
    P.rdm_chunk.reserve(tot);
    for (int c = 0; c < 5; c++) {
        std::stable_sort(cls[c].begin(), cls[c].end(), by_work);
        P.rdm_cls[c] = (int64_t)P.rdm_chunk.size();
        for (auto &x : cls[c]) P.rdm_chunk.push_back(x.c);
    }
    P.rdm_cls[5] = (int64_t)P.rdm_chunk.size();
    return MW_OK;
}

// |z| with each product rounded on its own (no fused multiply-add), the
// rounding the screening's other magnitudes use
static double cabs_rounded(double re, double im)
{
#pragma clang fp contract(off)
    const double a = re * re;
    const double b = im * im;
    return std::sqrt(a + b);
}

// Spinor plans: B[a][b][c][d] = the largest |(PQ|RS)| over P in Kramers pair
// a, Q in b, R in c, S in d with P != R and Q != S, the |(ab|cd)| of
// Table 1 when every vertex carries both Kramers partners.  The bound of a
// doubly excited configuration pair with particles i, k and holes j, l is
// max(B[i][j][k][l], B[i][l][k][j]).
static void bound_table(HostPlan &P, const std::complex<double> *g)
{
    const int n = P.n, Mm = 2 * n;
    P.g_bound.assign((size_t)n * n * n * n, 0.0);
    parallel_for(n, [&](int64_t a0, int64_t a1, unsigned) {
        for (int64_t a = a0; a < a1; a++)
            for (int b = 0; b < n; b++)
                for (int c = 0; c < n; c++)
                    for (int d = 0; d < n; d++) {
                        double m = 0.0;
                        for (int Pp = (int)a; Pp < Mm; Pp += n)
                            for (int Q = b; Q < Mm; Q += n)
                                for (int R = c; R < Mm; R += n)
                                    for (int S = d; S < Mm; S += n) {
                                        if (Pp == R || Q == S) continue;
                                        const std::complex<double> v =
                                            g[(((size_t)Pp * Mm + Q) * Mm + R) * Mm + S];
                                        m = std::max(m, cabs_rounded(v.real(), v.imag()));
                                    }
                        P.g_bound[(((size_t)a * n + b) * n + c) * n + d] = m;
                    }
    });
}

static void repack(HostPlan &P, const mw_problem *p)
{
    const int n = P.n;
    if (P.kind == MW_SPIN_FREE) {
        const double *h = p->h, *g = p->g;
        auto G = [&](int a, int b, int c, int d) { return g[(((size_t)a * n + b) * n + c) * n + d]; };
        P.h.assign(h, h + (size_t)n * n);
        P.w_same.resize((size_t)n * n * n);
        P.w_opp.resize((size_t)n * n * n);
        for (int r = 0; r < n; r++)
            for (int a = 0; a < n; a++)
                for (int b = 0; b < n; b++) {
                    P.w_same[((size_t)r * n + a) * n + b] = G(a, b, r, r) - G(a, r, r, b);
                    P.w_opp[((size_t)r * n + a) * n + b] = G(a, b, r, r);
                }
        P.g_ab.resize((size_t)n * n * n * n);
        parallel_for(n, [&](int64_t q0, int64_t q1, unsigned) {
            for (int64_t q = q0; q < q1; q++)
                for (int s = 0; s < n; s++)
                    for (int a = 0; a < n; a++)
                        for (int r = 0; r < n; r++)
                            P.g_ab[(((size_t)q * n + s) * n + a) * n + r] = G(a, q, r, s);
        });
        const int np = n * (n - 1) / 2;
        P.npair = np;
        P.a_pair.resize((size_t)np * np);
        P.a_pair1.resize((size_t)np * np);
        // one item per x1 (its work grows with x1), taken dynamically
        parallel_items(n, [&](int64_t x1) {
            for (int x0 = 0; x0 < x1; x0++)
                for (int y1 = 1; y1 < n; y1++)
                    for (int y0 = 0; y0 < y1; y0++) {
                        const double v = G(x0, y0, (int)x1, y1) - G(x0, y1, (int)x1, y0);
                        P.a_pair[(size_t)pair_index(x0, (int)x1) * np + pair_index(y0, y1)] = v;
                        P.a_pair1[(size_t)pair_index(x0, (int)x1) * np + pair_lex(y0, y1, n)] = v;
                    }
        });
    } else {
        const int Mm = 2 * n;
        using cd = std::complex<double>;
        const cd *g = reinterpret_cast<const cd *>(p->g);
        auto G = [&](int a, int b, int c, int d) { return g[(((size_t)a * Mm + b) * Mm + c) * Mm + d]; };
        P.h.assign(p->h, p->h + 2 * (size_t)Mm * Mm);
        P.w_same.resize(2 * (size_t)Mm * Mm * Mm);
        for (int r = 0; r < Mm; r++)
            for (int a = 0; a < Mm; a++)
                for (int b = 0; b < Mm; b++) {
                    cd v = G(a, b, r, r) - G(a, r, r, b);
                    size_t k = ((size_t)r * Mm + a) * Mm + b;
                    P.w_same[2 * k] = v.real();
                    P.w_same[2 * k + 1] = v.imag();
                }
        const int np = Mm * (Mm - 1) / 2;
        P.npair = np;
        P.a_pair.resize(2 * (size_t)np * np);
        P.a_pair1.resize(2 * (size_t)np * np);
        parallel_items(Mm, [&](int64_t x1) {
            for (int x0 = 0; x0 < x1; x0++)
                for (int y1 = 1; y1 < Mm; y1++)
                    for (int y0 = 0; y0 < y1; y0++) {
                        cd v = G(x0, y0, (int)x1, y1) - G(x0, y1, (int)x1, y0);
                        size_t k = (size_t)pair_index(x0, (int)x1) * np + pair_index(y0, y1);
                        size_t k1 = (size_t)pair_index(x0, (int)x1) * np + pair_lex(y0, y1, Mm);
                        P.a_pair[2 * k] = v.real();
                        P.a_pair[2 * k + 1] = v.imag();
                        P.a_pair1[2 * k1] = v.real();
                        P.a_pair1[2 * k1 + 1] = v.imag();
                    }
        });
        bound_table(P, g);
    }
}

// Reference string omega for single elements (the closed-shell reference
// idea of section 2.3): every position occupied in more than half of the
// determinants.  F^omega = h + sum_{R in omega} [(PQ|RR) - (PR|RQ)] is
// tabulated once; a single group with string K then needs only the
// positions where K and omega differ:
//   F^K = F^omega + sum_{R in K\omega} w_R - sum_{R in omega\K} w_R.
static void reference(HostPlan &P)
{
    const int n = P.n;
    std::vector<int64_t> cnt(2 * 64, 0);
    for (int64_t i = 0; i < P.ndet; i++)
        for (int w = 0; w < 2; w++)
            for (uint64_t x = P.dets[2 * i + w]; x; x &= x - 1) cnt[w * 64 + __builtin_ctzll(x)]++;
    P.ref0 = P.ref1 = 0;
    for (int b = 0; b < n; b++) {
        if (2 * cnt[b] > P.ndet) P.ref0 |= 1ULL << b;
        if (2 * cnt[64 + b] > P.ndet) P.ref1 |= 1ULL << b;
    }
    if (P.kind == MW_SPIN_FREE) {
        // f_ref[s][p][q]: s = 0 for alpha single groups, 1 for beta
        P.f_ref.assign(2 * (size_t)n * n, 0.0);
        for (int s = 0; s < 2; s++) {
            uint64_t same = s == 0 ? P.ref0 : P.ref1, opp = s == 0 ? P.ref1 : P.ref0;
            for (int a = 0; a < n; a++)
                for (int b = 0; b < n; b++) {
                    double f = P.h[(size_t)a * n + b];
                    for (uint64_t x = same; x; x &= x - 1) f += P.w_same[((size_t)__builtin_ctzll(x) * n + a) * n + b];
                    for (uint64_t x = opp; x; x &= x - 1) f += P.w_opp[((size_t)__builtin_ctzll(x) * n + a) * n + b];
                    P.f_ref[((size_t)s * n + a) * n + b] = f;
                }
        }
    } else {
        const int Mm = 2 * n;
        P.f_ref.assign(2 * (size_t)Mm * Mm, 0.0);
        for (int a = 0; a < Mm; a++)
            for (int b = 0; b < Mm; b++) {
                double re = P.h[2 * ((size_t)a * Mm + b)], im = P.h[2 * ((size_t)a * Mm + b) + 1];
                for (int w = 0; w < 2; w++)
                    for (uint64_t x = w ? P.ref1 : P.ref0; x; x &= x - 1) {
                        size_t k = ((size_t)(w * n + __builtin_ctzll(x)) * Mm + a) * Mm + b;
                        re += P.w_same[2 * k];
                        im += P.w_same[2 * k + 1];
                    }
                P.f_ref[2 * ((size_t)a * Mm + b)] = re;
                P.f_ref[2 * ((size_t)a * Mm + b) + 1] = im;
            }
    }
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

Counts HostPlan::counts() const
{
    if (dix.on) return dix.cnt;
    Counts c;
    c.ngroup = (int64_t)grp_type.size();
    c.nmem = (int64_t)mem.size();
    c.nslot_mem = (int64_t)slot_mem.size();
    c.nslot = (int64_t)slot_pos.size();
    c.npk = (int64_t)pk_off.size() - 1;
    c.nrdm_ent = (int64_t)rdm_ent.size();
    c.nrdm_chunk = (int64_t)rdm_chunk.size();
    c.nrdm_skey = (int64_t)rdm_skey.size();
    return c;
}

size_t HostPlan::layout(DevPlan *d, char *base) const
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t sb = scalar_bytes();
    const Counts c = counts();
    const size_t ng = (size_t)c.ngroup, nm = (size_t)c.nmem;
    DevPlan t{};
    t.kind = kind; t.n = n; t.M = M; t.npair = npair; t.ndet = ndet;
    t.nmem = c.nmem;
    t.npacket = c.npk;
    t.max_roots = max_roots;
    t.ecore = ecore;
    t.grp_off = (const uint32_t *)take((ng + 1) * 4);
    t.grp_key = (const uint64_t *)take(ng * 16);
    t.grp_type = (const uint8_t *)take(ng);
    t.grp_col = (const uint32_t *)take(ng * 4);
    t.ncol = ncol;
    t.mem = (const uint2 *)take(nm * 8);
    t.mem_grp = (const uint32_t *)take(nm * 4);
    t.slot_mem = (const uint32_t *)take((size_t)c.nslot_mem * 4);
    t.slot_pos = (const uint32_t *)take((size_t)c.nslot * 4);
    t.pk_off = (const uint32_t *)take(((size_t)c.npk + 1) * 4);
    t.rowptr = (const uint32_t *)take(((size_t)ndet + 1) * 4);
    t.dets = (const uint64_t *)take(dets.size() * 8);
    t.diag = (void *)take((size_t)ndet * sb);
    t.h = (const void *)take(h.size() * 8);
    t.w_same = (const void *)take(w_same.size() * 8);
    t.w_opp = (const void *)take(w_opp.size() * 8);
    t.g_ab = (const void *)take(g_ab.size() * 8);
    t.a_pair = (const void *)take(a_pair.size() * 8);
    t.a_pair1 = (const void *)take(a_pair1.size() * 8);
    t.f_ref = (const void *)take(f_ref.size() * 8);
    t.g_bound = g_bound.empty() ? nullptr : (const double *)take(g_bound.size() * 8);
    t.ref0 = ref0;
    t.ref1 = ref1;
    t.npacket_double = npacket_double;
    t.nmem_double = nmem_double;
    t.rdm_ent = (const uint2 *)take((size_t)c.nrdm_ent * 8);
    t.rdm_chunk = (const uint4 *)take((size_t)c.nrdm_chunk * 16);
    t.rdm_pos = (const uint16_t *)take(nm * 2);
    t.rdm_ent_det = (const uint32_t *)take((size_t)c.nrdm_ent * 4);
    t.rdm_skey = (const ulonglong2 *)take((size_t)c.nrdm_skey * 16);
    t.rdm_single_e0 = rdm_single_e0;
    for (int c = 0; c < 6; c++) t.rdm_cls[c] = rdm_cls[c];
    // per-call scratch: sigma partials, or the density-matrix accumulators
    // (double pairs, RDM_COPIES copies of S and the single corrections (n^3
    // or M^3), occupation correlations and their 256 per-chunk partials)
    // followed by the bra coefficients gathered per double membership and
    // the fixed-point scale
    const size_t mm = (size_t)M * M;
    size_t rdm_bytes = kind == MW_SPIN_FREE
                           ? ((size_t)n * n * n * n + 2 * (size_t)npair * npair +
                              RDM_COPIES * (2 * (size_t)n * n + 2 * (size_t)n * n * n) + 257 * mm) * 8
                           : (2 * (size_t)npair * npair + RDM_COPIES * (mm + mm * M) + 257 * mm) * 16;
    rdm_bytes = ((rdm_bytes + 255) & ~(size_t)255) + ((nm * max_roots * sb + 255) & ~(size_t)255) + RDM_FX_BYTES;
    t.scratch_bytes = std::max(std::max<size_t>(1, nm + (size_t)ncol) * (size_t)max_roots * sb, rdm_bytes);
    t.partial = (void *)take(t.scratch_bytes);
    t.self = (DevPlan *)take(sizeof(DevPlan));
    t.counter = (uint32_t *)take(256);
    t.tune_u = tune_u;
    t.tune_gl = tune_gl ? tune_gl : (kind == MW_SPINOR ? 32 : 16);
    t.rdm_fixed = rdm_fixed;
    if (d) *d = t;
    return off + 256;
}

}  // namespace mw

using namespace mw;

struct mw_plan_s {
    HostPlan p;
};

void mw_internal_batched_forget(mw_plan plan);

extern "C" {

const char *mw_last_error(void) { return g_last_error.c_str(); }

static mw_status plan_create(const mw_problem *prob, int32_t max_roots, bool device, hipStream_t s, mw_plan *out)
{
    if (!out) return fail(MW_EINVAL, "out is NULL");
    *out = nullptr;
    mw_status st = validate(prob, max_roots);
    if (st != MW_OK) return st;
    std::unique_ptr<mw_plan_s> pl;
    try {
        pl.reset(new mw_plan_s());
        HostPlan &P = pl->p;
        P.kind = prob->kind;
        P.n = prob->norb;
        P.M = 2 * prob->norb;
        P.nalpha = prob->nalpha;
        P.nbeta = prob->nbeta;
        P.ndet = prob->ndet;
        P.ecore = prob->ecore;
        P.cplx = prob->kind == MW_SPINOR;
        P.max_roots = max_roots;
        P.dets.assign(prob->dets, prob->dets + 2 * prob->ndet);
        if (device) {
            st = build_index_device(P, s);
            if (st != MW_OK) {
                P.dix.release();
                return st;
            }
        } else {
            st = build_groups(P);
            if (st != MW_OK) return st;
            st = build_rdm_rows(P);
            if (st != MW_OK) return st;
        }
        repack(P, prob);
        reference(P);
    } catch (const std::bad_alloc &) {
        if (pl) pl->p.dix.release();
        return fail(MW_EUNSUPPORTED, "host memory exhausted while building the plan");
    } catch (const std::exception &e) {
        if (pl) pl->p.dix.release();
        return fail(MW_EINVAL, std::string("plan build failed: ") + e.what());
    }
    *out = pl.release();
    return MW_OK;
}

mw_status mw_plan_create(const mw_problem *prob, int32_t max_roots, mw_plan *out)
{
    return plan_create(prob, max_roots, false, nullptr, out);
}

mw_status mw_plan_create_device(const mw_problem *prob, int32_t max_roots, mw_stream_t stream, mw_plan *out)
{
    return plan_create(prob, max_roots, true, (hipStream_t)stream, out);
}

mw_status mw_plan_array(mw_plan plan, int32_t which, size_t *offset, size_t *bytes)
{
    if (!plan || !offset || !bytes) return fail(MW_EINVAL, "NULL argument");
    const HostPlan &P = plan->p;
    if (!P.bound) return fail(MW_EINVAL, "plan is not uploaded");
    const DevPlan &d = P.dev;
    const Counts c = P.counts();
    const size_t ng = (size_t)c.ngroup, nm = (size_t)c.nmem;
    const void *ptr = nullptr;
    size_t nb = 0;
    switch (which) {
    case 0: ptr = d.grp_off; nb = (ng + 1) * 4; break;
    case 1: ptr = d.grp_key; nb = ng * 16; break;
    case 2: ptr = d.grp_type; nb = ng; break;
    case 3: ptr = d.grp_col; nb = ng * 4; break;
    case 4: ptr = d.mem; nb = nm * 8; break;
    case 5: ptr = d.mem_grp; nb = nm * 4; break;
    case 6: ptr = d.slot_mem; nb = (size_t)c.nslot_mem * 4; break;
    case 7: ptr = d.slot_pos; nb = (size_t)c.nslot * 4; break;
    case 8: ptr = d.pk_off; nb = ((size_t)c.npk + 1) * 4; break;
    case 9: ptr = d.rowptr; nb = ((size_t)P.ndet + 1) * 4; break;
    case 10: ptr = d.rdm_ent; nb = (size_t)c.nrdm_ent * 8; break;
    case 11: ptr = d.rdm_chunk; nb = (size_t)c.nrdm_chunk * 16; break;
    case 12: ptr = d.rdm_pos; nb = nm * 2; break;
    case 13: ptr = d.rdm_ent_det; nb = (size_t)c.nrdm_ent * 4; break;
    case 14: ptr = d.rdm_skey; nb = (size_t)c.nrdm_skey * 16; break;
    default: return fail(MW_EINVAL, "array index out of range (0 .. 14)");
    }
    *offset = (size_t)((const char *)ptr - (const char *)P.ws);
    *bytes = nb;
    return MW_OK;
}

mw_status mw_plan_workspace_bytes(mw_plan plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(MW_EINVAL, "NULL argument");
    *bytes = plan->p.layout(nullptr, nullptr);
    return MW_OK;
}

mw_status mw_plan_upload(mw_plan plan, void *workspace, size_t bytes, mw_stream_t stream)
{
    if (!plan || !workspace) return fail(MW_EINVAL, "NULL argument");
    mw_internal_batched_forget(plan);
    HostPlan &P = plan->p;
    size_t need = P.layout(nullptr, nullptr);
    if (bytes < need) return fail(MW_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace) & 255) return fail(MW_EWORKSPACE, "workspace must be 256-byte aligned");
    DevPlan d;
    P.layout(&d, (char *)workspace);
    hipStream_t s = (hipStream_t)stream;
    auto up = [&](const void *dst, const void *src, size_t nb) -> bool {
        if (!nb) return true;
        return hipMemcpyAsync((void *)dst, src, nb, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    if (P.dix.on && P.moved)
        return fail(MW_EINVAL, "a plan built on the device is uploaded once (its index now lives in the first workspace)");
    if (P.dix.on) {
        // device-built index: copied inside the device, then released
        const DevIndex &x = P.dix;
        const Counts &c = x.cnt;
        auto dd = [&](const void *dst, const void *src, size_t nb) -> bool {
            if (!nb) return true;
            return hipMemcpyAsync((void *)dst, src, nb, hipMemcpyDeviceToDevice, s) == hipSuccess;
        };
        const size_t ng = (size_t)c.ngroup, nm = (size_t)c.nmem;
        bool ok = dd(d.grp_off, x.grp_off, (ng + 1) * 4) && dd(d.grp_key, x.grp_key, ng * 16) &&
                  dd(d.grp_type, x.grp_type, ng) && dd(d.grp_col, x.grp_col, ng * 4) && dd(d.mem, x.mem, nm * 8) &&
                  dd(d.mem_grp, x.mem_grp, nm * 4) && dd(d.slot_mem, x.slot_mem, (size_t)c.nslot_mem * 4) &&
                  dd(d.slot_pos, x.slot_pos, (size_t)c.nslot * 4) &&
                  dd(d.pk_off, x.pk_off, ((size_t)c.npk + 1) * 4) &&
                  dd(d.rowptr, x.rowptr, ((size_t)P.ndet + 1) * 4) &&
                  dd(d.rdm_ent, x.rdm_ent, (size_t)c.nrdm_ent * 8) &&
                  dd(d.rdm_chunk, x.rdm_chunk, (size_t)c.nrdm_chunk * 16) && dd(d.rdm_pos, x.rdm_pos, nm * 2) &&
                  dd(d.rdm_ent_det, x.rdm_ent_det, (size_t)c.nrdm_ent * 4) &&
                  dd(d.rdm_skey, x.rdm_skey, (size_t)c.nrdm_skey * 16) &&
                  up(d.dets, P.dets.data(), P.dets.size() * 8) && up(d.h, P.h.data(), P.h.size() * 8) &&
                  up(d.w_same, P.w_same.data(), P.w_same.size() * 8) &&
                  up(d.w_opp, P.w_opp.data(), P.w_opp.size() * 8) && up(d.g_ab, P.g_ab.data(), P.g_ab.size() * 8) &&
                  up(d.a_pair, P.a_pair.data(), P.a_pair.size() * 8) &&
                  up(d.a_pair1, P.a_pair1.data(), P.a_pair1.size() * 8) &&
                  up(d.f_ref, P.f_ref.data(), P.f_ref.size() * 8) &&
                  up(d.g_bound, P.g_bound.data(), P.g_bound.size() * 8) &&
                  hipMemcpyAsync(d.self, &d, sizeof(DevPlan), hipMemcpyHostToDevice, s) == hipSuccess;
        if (!ok) return fail(MW_EHIP, "hipMemcpyAsync failed during plan upload");
        mw_status st = launch_diag(d, s);
        if (st != MW_OK) return st;
        if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "hipStreamSynchronize failed after upload");
        P.dix.release();
        P.moved = true;
        P.ws = workspace;
        P.ws_bytes = bytes;
        P.dev = d;
        P.bound = true;
        return MW_OK;
    }
    bool ok = up(d.grp_off, P.grp_off.data(), P.grp_off.size() * 4) &&
              up(d.grp_key, P.grp_key.data(), P.grp_key.size() * 8) &&
              up(d.grp_type, P.grp_type.data(), P.grp_type.size()) &&
              up(d.grp_col, P.grp_col.data(), P.grp_col.size() * 4) &&
              up(d.mem, P.mem.data(), P.mem.size() * 8) &&
              up(d.mem_grp, P.mem_grp.data(), P.mem_grp.size() * 4) &&
              up(d.slot_mem, P.slot_mem.data(), P.slot_mem.size() * 4) &&
              up(d.slot_pos, P.slot_pos.data(), P.slot_pos.size() * 4) &&
              up(d.pk_off, P.pk_off.data(), P.pk_off.size() * 4) &&
              up(d.rowptr, P.rowptr.data(), P.rowptr.size() * 4) &&
              up(d.dets, P.dets.data(), P.dets.size() * 8) &&
              up(d.h, P.h.data(), P.h.size() * 8) &&
              up(d.w_same, P.w_same.data(), P.w_same.size() * 8) &&
              up(d.w_opp, P.w_opp.data(), P.w_opp.size() * 8) &&
              up(d.g_ab, P.g_ab.data(), P.g_ab.size() * 8) &&
              up(d.a_pair, P.a_pair.data(), P.a_pair.size() * 8) &&
              up(d.a_pair1, P.a_pair1.data(), P.a_pair1.size() * 8) &&
              up(d.f_ref, P.f_ref.data(), P.f_ref.size() * 8) &&
              up(d.g_bound, P.g_bound.data(), P.g_bound.size() * 8) &&
              up(d.rdm_ent, P.rdm_ent.data(), P.rdm_ent.size() * 8) &&
              up(d.rdm_chunk, P.rdm_chunk.data(), P.rdm_chunk.size() * 16) &&
              up(d.rdm_pos, P.rdm_pos.data(), P.rdm_pos.size() * 2) &&
              up(d.rdm_ent_det, P.rdm_ent_det.data(), P.rdm_ent_det.size() * 4) &&
              up(d.rdm_skey, P.rdm_skey.data(), P.rdm_skey.size() * 16);
    if (!ok) return fail(MW_EHIP, "hipMemcpyAsync failed during plan upload");
    if (hipMemcpyAsync(d.self, &d, sizeof(DevPlan), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(MW_EHIP, "hipMemcpyAsync failed during plan upload");
    mw_status st = launch_diag(d, s);
    if (st != MW_OK) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "hipStreamSynchronize failed after upload");
    P.ws = workspace;
    P.ws_bytes = bytes;
    P.dev = d;
    P.bound = true;
    return MW_OK;
}

mw_status mw_plan_update_integrals(mw_plan plan, const double *h, const double *g, double ecore, mw_stream_t stream)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    HostPlan &P = plan->p;
    if (!P.bound) return fail(MW_EWORKSPACE, "plan has no workspace: call mw_plan_upload first");
    mw_status st = validate_integrals(P.kind, P.n, h, g);
    if (st != MW_OK) return st;
    mw_problem q{};
    q.kind = P.kind;
    q.norb = P.n;
    q.h = h;
    q.g = g;
    try {
        repack(P, &q);
        reference(P);
    } catch (const std::bad_alloc &) {
        return fail(MW_EUNSUPPORTED, "host memory exhausted while repacking integrals");
    }
    P.ecore = ecore;
    P.dev.ecore = ecore;
    const DevPlan &d = P.dev;
    hipStream_t s = (hipStream_t)stream;
    auto up = [&](const void *dst, const void *src, size_t nb) -> bool {
        if (!nb) return true;
        return hipMemcpyAsync((void *)dst, src, nb, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = up(d.h, P.h.data(), P.h.size() * 8) && up(d.w_same, P.w_same.data(), P.w_same.size() * 8) &&
              up(d.w_opp, P.w_opp.data(), P.w_opp.size() * 8) && up(d.g_ab, P.g_ab.data(), P.g_ab.size() * 8) &&
              up(d.a_pair1, P.a_pair1.data(), P.a_pair1.size() * 8) &&
              up(d.a_pair, P.a_pair.data(), P.a_pair.size() * 8) && up(d.f_ref, P.f_ref.data(), P.f_ref.size() * 8) &&
              up(d.g_bound, P.g_bound.data(), P.g_bound.size() * 8) && up(d.self, &P.dev, sizeof(DevPlan));
    if (!ok) return fail(MW_EHIP, "hipMemcpyAsync failed during integral update");
    st = launch_diag(d, s);
    if (st != MW_OK) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "hipStreamSynchronize failed");
    return MW_OK;
}

mw_status mw_plan_destroy(mw_plan plan)
{
    if (plan) {
        mw_internal_batched_forget(plan);
        plan->p.dix.release();
    }
    delete plan;
    return MW_OK;
}

int64_t mw_plan_info(mw_plan plan, int32_t what)
{
    if (!plan) return -1;
    const HostPlan &P = plan->p;
    switch (what) {
    case 0: return P.ndet;
    case 1: return P.counts().ngroup;
    case 2: return P.counts().nmem;
    case 3: return P.n_single_pairs + P.n_double_pairs;
    case 4: return P.n_single_pairs;
    case 5: return P.n_double_pairs;
    case 6: return P.n_evals;
    case 7: return (int64_t)P.layout(nullptr, nullptr);
    case 8: return (int64_t)P.scalar_bytes();
    case 9: return P.n;
    case 10: return P.kind;
    case 11: return P.counts().npk;
    case 12: return P.npacket_double;
    case 13: return P.ncol;
    case 14: return P.n_double_pairs_large;
    case 15: return P.counts().nrdm_ent;
    case 16: return P.counts().nrdm_chunk;
    case 17: return P.dix.on ? 1 : 0;
    case 18: return P.rdm_fixed;
    default: return -1;
    }
}

// accessors for the other translation units (not exported)
__attribute__((visibility("hidden"))) const mw::DevPlan *mw_internal_devplan(mw_plan plan)
{
    if (!plan || !plan->p.bound) return nullptr;
    return &plan->p.dev;
}

// the host copy of the space: sorted determinants, orbitals, electron counts
__attribute__((visibility("hidden"))) int mw_internal_space(mw_plan plan, const uint64_t **dets, int64_t *ndet,
                                                            int32_t *kind, int32_t *n, int32_t *na, int32_t *nb)
{
    if (!plan) return 0;
    *dets = plan->p.dets.data();
    *ndet = plan->p.ndet;
    *kind = plan->p.kind;
    *n = plan->p.n;
    *na = plan->p.nalpha;
    *nb = plan->p.nbeta;
    return 1;
}

mw_status mw_plan_get_tuning(mw_plan plan, int32_t *code)
{
    if (!plan || !code) return fail(MW_EINVAL, "NULL argument");
    const HostPlan &P = plan->p;
    const int gl = P.tune_gl ? P.tune_gl : (P.kind == MW_SPINOR ? 32 : 16);
    *code = P.tune_u * 100 + gl;
    return MW_OK;
}

mw_status mw_plan_set_tuning(mw_plan plan, int32_t code)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const int u = code / 100, gl = code % 100;
    if ((u != 4 && u != 8 && u != 16) || (gl != 8 && gl != 16 && gl != 32))
        return fail(MW_EINVAL, "tuning code must be unroll*100+lanes, unroll 4/8/16, lanes 8/16/32");
    if (u == 16 && plan->p.kind == MW_SPINOR) return fail(MW_EINVAL, "unroll 16 is for real plans only");
    HostPlan &P = plan->p;
    P.tune_u = u;
    P.tune_gl = gl;
    P.dev.tune_u = u;
    P.dev.tune_gl = gl;
    return MW_OK;
}

mw_status mw_plan_set_rdm_mode(mw_plan plan, int32_t mode)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    if (mode != 0 && mode != 1) return fail(MW_EINVAL, "density-matrix mode must be 0 (atomic) or 1 (fixed point)");
    plan->p.rdm_fixed = mode;
    plan->p.dev.rdm_fixed = mode;
    return MW_OK;
}

// set the tunables (host copy; the device copy keeps the upload values,
// which only the batched kernels read and they do not use these fields)
__attribute__((visibility("hidden"))) void mw_internal_set_tune(mw_plan plan, int32_t u, int32_t gl)
{
    if (!plan) return;
    plan->p.tune_u = u;
    plan->p.tune_gl = gl;
    plan->p.dev.tune_u = u;
    plan->p.dev.tune_gl = gl;
}

}  // extern "C"
