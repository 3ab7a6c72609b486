// Epstein-Nesbet second-order energy over the external space (section 2.5,
// Eq. (ENPT2E), primary space = the whole variational space P):
//
//   E2_k = sum_{A in Q} |sum_{J in P} H_AJ c_Jk|^2 / (E0_k - H_AA),
//
// Q = determinants outside P reached from P by one or two excitations.
// The paper splits the space W of all such excitations into disjoint
// subspaces W_i (by constraints on the highest occupied orbitals), stores
// the connections of a batch of W_i, sorts them to find each A with its
// partners J, and deletes the connection of a doubly excited configuration
// A to J when Table 1's bound is below Q_min / max|C| over J's
// configuration.  Here the disjoint subspaces are hash buckets of A: every
// (A, J) pair generated from a J of P lands in the bucket of A, so one
// bucket holds every partner of its A's.
//
//   k_cfg_*           configurations of P (hash table): max|C| over each
//   k_pt2_enum<0>     every J lists its excitations (one workgroup per J),
//                     drops A in P (exact hash set of the space) and counts
//                     the kept pairs (configuration doubles screened)
//   k_pt2_enum<1>     the same pairs, counted per bucket
//   k_pt2_enum<2>     the pairs of the buckets of one pass, written as
//                     records {A, J} with H_AJ c_J at the bucket's offset
//   k_pt2_bucket_wave one wave per bucket (up to 1024 records): sorts its
//                     records by (hash bits of A, J) in registers, sums each
//                     run's numerator across the wave by segmented scans,
//                     adds |num|^2 / (E0 - H_AA) per external A
//   k_pt2_bucket_big  the same for larger buckets of any size, one
//                     workgroup each, sorting in global memory
//   k_sel_*           the iCIPT2 selection: the same walk, the tests per
//                     pair, kept keys bucketed, sorted, and decided per
//                     (external determinant, configuration of P)
//   k_pt2_sum1/2      per pass: bucket partial sums in a fixed order
//
// Passes over bucket ranges keep the records within the caller's work
// buffer (the pipelined memory bound of the paper's procedure).  Every sum
// has a fixed order, so repeated calls give identical bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "dev_common.h"
#include "mw_internal.h"

namespace mw {

namespace {

constexpr int PT2_WCAP = 1024;     // records of a bucket sorted by one wave in registers;
                                   // larger buckets: one workgroup, sorted in global memory
constexpr int SEL_CAP = 1024;      // selection keys of a bucket sorted in LDS; larger: global
constexpr int PT2_MEAN = 400;      // target records per bucket
constexpr int PT2_MAXR = 8;        // roots per call

struct alignas(16) Rec {
    uint64_t a0, a1;
    double haa;    // H_AA from this record's partner J (the first J of A is used)
    uint64_t key;  // low 32 bits of the hash of A (high word), then J
};

// Excitation classes of a determinant of the space; the counts are equal
// for every J (fixed particle numbers).  Spin-free: sector 0 = alpha
// positions, 1 = beta; classes single a, single b, double aa, double bb,
// double ab.  Spinor: one sector; classes single, double.
struct ExcClasses {
    int nclass;
    int type[5];      // 0 single, 1 double in one sector, 2 alpha-beta double
    int sec[5];
    int start[6];     // prefix of the class sizes (fewer than 2^31 per J)
    int no[2], nv[2];
};

struct Roots {
    double e0[PT2_MAXR];
};

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // SplitMix64 finaliser (Steele, Lea and Flood, 2014)
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ULL;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

__device__ __forceinline__ uint64_t hash_det(uint64_t a0, uint64_t a1)
{
    return mix64(a0 ^ mix64(a1 + 0x9E3779B97F4A7C15ULL));
}

// bucket = the top lognb bits of the hash
__device__ __forceinline__ uint32_t bucket_of(uint64_t h, int lognb)
{
    return lognb ? (uint32_t)(h >> (64 - lognb)) : 0u;
}

// Exact membership in the space: open addressing on the low hash bits,
// linear probing, keys {a0, a1}, empty slots all ones (no determinant of a
// space with excitations has every position occupied).
struct DetSet {
    const ulonglong2 *key;
    uint64_t mask;
};

__device__ __forceinline__ bool in_set(const DetSet &s, uint64_t h, uint64_t a0, uint64_t a1)
{
    for (uint64_t i = h & s.mask;; i = (i + 1) & s.mask) {
        const ulonglong2 k = s.key[i];
        if (k.x == a0 && k.y == a1) return true;
        if (k.x == ~0ULL && k.y == ~0ULL) return false;
    }
}

__global__ __launch_bounds__(256) void k_set_insert(const uint64_t *__restrict__ dets, int64_t ndet, uint32_t *slot,
                                                    uint64_t mask)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndet) return;
    const uint64_t a0 = dets[2 * i], a1 = dets[2 * i + 1];
    // at most ndet < table size / 2 insertions: a free slot is always found
    for (uint64_t s = hash_det(a0, a1) & mask;; s = (s + 1) & mask)
        if (atomicCAS(&slot[s], 0xffffffffu, (uint32_t)i) == 0xffffffffu) return;
}

__global__ __launch_bounds__(256) void k_set_keys(const uint64_t *__restrict__ dets, const uint32_t *__restrict__ slot,
                                                  uint64_t size, ulonglong2 *key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)size) return;
    const uint32_t d = slot[i];
    key[i] = d == 0xffffffffu ? make_ulonglong2(~0ULL, ~0ULL) : make_ulonglong2(dets[2 * (size_t)d], dets[2 * (size_t)d + 1]);
}

__device__ __forceinline__ double mag(double v) { return fabs(v); }
// |v| without contraction, as re*re + im*im rounded term by term
__device__ __forceinline__ double mag(double2 v) { return sqrt(__dadd_rn(__dmul_rn(v.x, v.x), __dmul_rn(v.y, v.y))); }

// Configurations of the space (section 2.2): a determinant's configuration
// is its occupied mask and doubly occupied mask over orbitals (spin-free) or
// Kramers pairs (spinor).  An open-addressing table holds, per
// configuration, the index of a determinant inserted with it; cslot[j] is
// the slot of determinant j's configuration (the configuration's id here),
// cmaxb[slot] the largest |c| over its determinants and the roots (as the
// bits of a non-negative double, so an integer maximum orders them).
__device__ __forceinline__ uint64_t cfg_hash(uint64_t d0, uint64_t d1)
{
    return hash_det(d0 | d1, d0 & d1);
}

__global__ __launch_bounds__(256) void k_cfg_insert(const uint64_t *__restrict__ dets, int64_t ndet, uint32_t *slot,
                                                    uint64_t mask, uint32_t *cslot)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ndet) return;
    const uint64_t o = dets[2 * j] | dets[2 * j + 1], d = dets[2 * j] & dets[2 * j + 1];
    // at most ndet < table size / 2 configurations: a free slot is found
    for (uint64_t s = cfg_hash(dets[2 * j], dets[2 * j + 1]) & mask;; s = (s + 1) & mask) {
        const uint32_t cur = atomicCAS(&slot[s], 0xffffffffu, (uint32_t)j);
        if (cur == 0xffffffffu) {
            cslot[j] = (uint32_t)s;
            return;
        }
        const uint64_t x0 = dets[2 * (size_t)cur], x1 = dets[2 * (size_t)cur + 1];
        if ((x0 | x1) == o && (x0 & x1) == d) {
            cslot[j] = (uint32_t)s;
            return;
        }
    }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_cfg_max(int64_t ndet, int R, const typename Scal<CPLX>::T *__restrict__ c,
                                                 const uint32_t *__restrict__ cslot, unsigned long long *cmaxb)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ndet) return;
    double m = 0.0;
    for (int k = 0; k < R; k++) m = fmax(m, mag(c[(size_t)j * R + k]));
    atomicMax(&cmaxb[cslot[j]], (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(256) void k_cfg_gather(int64_t ndet, const uint32_t *__restrict__ cslot,
                                                    const unsigned long long *__restrict__ cmaxb, double *cm)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ndet) return;
    cm[j] = __longlong_as_double((long long)cmaxb[cslot[j]]);
}

// Table 1 (SD column) for the double excitation of J with holes Q, S and
// particles P, R (global positions): 0 when the configuration of A is not
// doubly excited from J's (a hole and a particle on one orbital or Kramers
// pair cancel), else the bound max(|(pq|rs)|, |(ps|rq)|) over the orbitals
// (spinor: the Kramers-pair table of the plan).  With particles i, k and
// holes j, l this one formula gives IntC 1-3 max(|(ij|kl)|, |(il|kj)|),
// IntC 4-5 |(ij|kj)| (l = j), IntC 6 |(il|ij)| (k = i) and IntC 7
// |(ij|ij)|, because the two integrals coincide by symmetry in those cases.
template <bool CPLX>
__device__ __forceinline__ bool cfg_double(const DevPlan &p, int Q, int S, int P, int R, double &bound)
{
    const int n = p.n;
    const int q = Q % n, s = S % n, a = P % n, r = R % n;
    if (q == a || q == r || s == a || s == r) return false;
    if constexpr (CPLX) {
        const double *t = p.g_bound;
        bound = fmax(t[(((size_t)a * n + q) * n + r) * n + s], t[(((size_t)a * n + s) * n + r) * n + q]);
    } else {
        // g_ab[q][s][p][r] = (pq|rs)
        const double *g = (const double *)p.g_ab;
        bound = fmax(fabs(g[(((size_t)q * n + s) * n + a) * n + r]), fabs(g[(((size_t)s * n + q) * n + a) * n + r]));
    }
    return true;
}

// colex pair k -> (lo, hi), k = hi (hi - 1) / 2 + lo
__device__ __forceinline__ void pair_of(int k, int &lo, int &hi)
{
    int b = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)k)) * 0.5f);
    while (b * (b - 1) / 2 > k) b--;
    while ((b + 1) * b / 2 <= k) b++;
    hi = b;
    lo = k - b * (b - 1) / 2;
}

__device__ __forceinline__ void flip(uint64_t &d0, uint64_t &d1, int n, int X)
{
    if (X < n) d0 ^= 1ULL << X;
    else d1 ^= 1ULL << (X - n);
}

// occupied positions of (d0, d1) below global position X
__device__ __forceinline__ int below(uint64_t d0, uint64_t d1, int n, int X)
{
    if (X < n) return __popcll(d0 & ((1ULL << X) - 1));
    return __popcll(d0) + __popcll(d1 & ((1ULL << (X - n)) - 1));
}

__device__ __forceinline__ bool occ(uint64_t d0, uint64_t d1, int n, int X)
{
    return X < n ? (d0 >> X) & 1 : (d1 >> (X - n)) & 1;
}

// occupied positions strictly between a and b
__device__ __forceinline__ int between(uint64_t d0, uint64_t d1, int n, int a, int b)
{
    const int lo = min(a, b), hi = max(a, b);
    return below(d0, d1, n, hi) - below(d0, d1, n, lo) - (int)occ(d0, d1, n, lo);
}


// Antisymmetrised double integral (PQ|RS) - (PS|RQ) for particles P < R
// (in A) and holes Q < S (in J), without the phase.
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T double_value(const DevPlan &p, int P, int Q, int R, int S)
{
    using T = typename Scal<CPLX>::T;
    const int n = p.n;
    if constexpr (!CPLX) {
        if (P < n && R >= n)  // alpha-beta: (pq|rs), p q alpha, r s beta
            return ((const double *)p.g_ab)[(((size_t)Q * n + (S - n)) * n + P) * n + (R - n)];
        const int off = P >= n ? n : 0;
        return ((const double *)p.a_pair)[(size_t)pair_idx(P - off, R - off) * p.npair +
                                          pair_idx(Q - off, S - off)];
    } else {
        return ((const T *)p.a_pair)[(size_t)pair_idx(P, R) * p.npair + pair_idx(Q, S)];
    }
}

// Decode item e of the excitation list of J (occupied / virtual position
// lists of each sector in LDS) into holes Q (< S) and particles P (< R);
// S = R = -1 for a single.
__device__ __forceinline__ void decode(const ExcClasses &ex, const uint8_t (*ol)[128], const uint8_t (*vl)[128],
                                       int e, int &Q, int &S, int &P, int &R)
{
    int c = 0;
    while (e >= ex.start[c + 1]) c++;
    const int i = e - ex.start[c];
    const int t = ex.type[c], s = ex.sec[c];
    if (t == 0) {
        const int nv = ex.nv[s];
        Q = ol[s][i / nv];
        P = vl[s][i % nv];
        S = R = -1;
    } else if (t == 1) {
        const int nv = ex.nv[s];
        const int vp = nv * (nv - 1) / 2;
        int a, b, x, y;
        pair_of(i / vp, a, b);
        pair_of(i % vp, x, y);
        Q = ol[s][a];
        S = ol[s][b];
        P = vl[s][x];
        R = vl[s][y];
    } else {
        const int nvv = ex.nv[0] * ex.nv[1];
        const int hp = i / nvv, vp = i % nvv;
        Q = ol[0][hp / ex.no[1]];
        S = ol[1][hp % ex.no[1]];
        P = vl[0][vp / ex.nv[1]];
        R = vl[1][vp % ex.nv[1]];
    }
}

// H_AA - H_JJ for A = J with holes Q (< S) replaced by particles P (< R)
// (S = R = -1: a single), from the orbital energies of J, eps_X = h_XX +
// sum_{Y in J, Y != X} V(X, Y), and V(X, Y) = (XX|YY) - (XY|YX):
//   single  eps_P - eps_Q - V_PQ
//   double  eps_P + eps_R - eps_Q - eps_S - V_PQ - V_PS - V_RQ - V_RS + V_PR + V_QS
__device__ __forceinline__ double diag_delta(const double *eps, const double *__restrict__ vg, int M, int Q, int S,
                                             int P, int R)
{
    auto V = [&](int X, int Y) { return vg[(size_t)X * M + Y]; };
    if (S < 0) return (eps[P] - eps[Q]) - V(P, Q);
    return (eps[P] + eps[R]) - (eps[Q] + eps[S]) - ((V(P, Q) + V(P, S)) + (V(R, Q) + V(R, S))) + (V(P, R) + V(Q, S));
}

// <A|H|J> for A = J with holes Q (< S) replaced by particles P (< R)
// (S = R = -1: a single): the integral with the phase of
// a+_P a_Q or a+_P a+_R a_S a_Q on J.
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T exc_value(const DevPlan &p, uint64_t j0, uint64_t j1, int Q,
                                                            int S, int P, int R)
{
    const int n = p.n;
    if (S < 0) {
        uint64_t k0 = j0, k1 = j1;
        flip(k0, k1, n, Q);
        const uint8_t type = CPLX ? G_SINGLE_S : (P < n ? G_SINGLE_A : G_SINGLE_B);
        return sc_neg(single_element<CPLX>(p, type, k0, k1, P, Q), between(j0, j1, n, P, Q) & 1);
    }
    // R <- S first, then P <- Q on the result
    int sg = between(j0, j1, n, R, S);
    uint64_t k0 = j0, k1 = j1;
    flip(k0, k1, n, S);
    flip(k0, k1, n, R);
    sg += between(k0, k1, n, P, Q);
    return sc_neg(double_value<CPLX>(p, P, Q, R, S), sg & 1);
}

// Pairs with A in P are dropped here (exact hash-set test).
// MODE 0: total kept pairs (atomic per workgroup); 1: per-bucket counts;
// 2: records {A, J} of buckets [b0, b1) at off[b] + running fill, with
// val[record][k] = H_AJ c_Jk (the integral rows are read by neighbouring
// lanes here, not scattered over the buckets).
template <bool CPLX, int MODE>
__global__ __launch_bounds__(256) void k_pt2_enum(DevPlan p, ExcClasses ex, DetSet inP, int R,
                                                  const typename Scal<CPLX>::T *__restrict__ c, double qmin,
                                                  int lognb, uint32_t b0, uint32_t b1, uint32_t *cnt,
                                                  const uint64_t *__restrict__ off, unsigned long long *fill, Rec *rec,
                                                  typename Scal<CPLX>::T *val, const double *__restrict__ eps,
                                                  const double *__restrict__ vg, unsigned long long *total,
                                                  int64_t jbase, uint32_t kmask, const double *__restrict__ cm)
{
    using T = typename Scal<CPLX>::T;
    __shared__ uint8_t ol[2][128], vl[2][128];
    __shared__ double s_qlim;
    __shared__ T s_c[PT2_MAXR];
    __shared__ double s_eps[128];
    __shared__ unsigned long long s_tot;
    const int64_t J = jbase + blockIdx.x;
    const uint64_t j0 = p.dets[2 * J], j1 = p.dets[2 * J + 1];
    const int n = p.n;
    if (MODE == 2 && (int)threadIdx.x < p.M) s_eps[threadIdx.x] = eps[J * p.M + threadIdx.x];
    if (threadIdx.x == 0) {
        // sector lists: spin-free sector 0 = alpha, 1 = beta; spinor one sector
        int no[2] = {0, 0}, nv[2] = {0, 0};
        for (int X = 0; X < 2 * n; X++) {
            const int s = CPLX ? 0 : X / n;
            if (occ(j0, j1, n, X)) ol[s][no[s]++] = (uint8_t)X;
            else vl[s][nv[s]++] = (uint8_t)X;
        }
        // section 2.5, step 4: a configuration double goes when its bound
        // is below qmin / max|C| over the determinants of J's configuration
        s_qlim = qmin > 0.0 ? qmin / cm[J] : 0.0;
        for (int k = 0; k < R; k++) s_c[k] = c[(size_t)J * R + k];
        s_tot = 0;
    }
    __syncthreads();
    const double qlim = s_qlim;
    const int E = ex.start[ex.nclass];
    unsigned long long mine = 0;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        int Q, S, P, Rr;
        decode(ex, ol, vl, e, Q, S, P, Rr);
        if (S >= 0 && qmin > 0.0) {
            double bound;
            if (cfg_double<CPLX>(p, Q, S, P, Rr, bound) && bound < qlim) continue;
        }
        uint64_t a0 = j0, a1 = j1;
        flip(a0, a1, n, Q);
        flip(a0, a1, n, P);
        if (S >= 0) {
            flip(a0, a1, n, S);
            flip(a0, a1, n, Rr);
        }
        const uint64_t h = hash_det(a0, a1);
        if (in_set(inP, h, a0, a1)) continue;  // A in P: not external
        if constexpr (MODE == 0) {
            mine++;
        } else {
            const uint32_t b = bucket_of(h, lognb);
            if constexpr (MODE == 1) {
                atomicAdd(&cnt[b], 1u);
            } else {
                if (b < b0 || b >= b1) continue;
                // one 64-bit word per bucket: the claim count below, the
                // bucket's capacity above, so the claim needs no second read
                const unsigned long long wv = atomicAdd(&fill[b], 1ULL);
                const uint32_t k = (uint32_t)wv;
                if (k >= (uint32_t)(wv >> 32)) continue;
                const uint64_t slot = off[b] + k;
                double hjj;
                if constexpr (CPLX) hjj = ((const double2 *)p.diag)[J].x;
                else hjj = ((const double *)p.diag)[J];
                // records and values are scattered here and read only by
                // the bucket kernels: non-temporal stores, the record as two
                // 16-byte halves (written bytes 11 % and the exact energy
                // 2 % below four 8-byte stores on the 20,000-determinant
                // n = 64 space; plain stores were 9 % slower)
                Rec *rp = rec + slot;
                {
                    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
                    u64x2 lo, hi;
                    lo.x = a0;
                    lo.y = a1;
                    hi.x = (unsigned long long)__double_as_longlong(hjj + diag_delta(s_eps, vg, p.M, Q, S, P, Rr));
                    hi.y = ((h & kmask) << 32) | (uint64_t)(uint32_t)J;
                    __builtin_nontemporal_store(lo, (u64x2 *)&rp->a0);
                    __builtin_nontemporal_store(hi, (u64x2 *)&rp->haa);
                }
                const T v = exc_value<CPLX>(p, j0, j1, Q, S, P, Rr);
                for (int q = 0; q < R; q++) {
                    const T w = sc_mul(v, s_c[q]);
                    if constexpr (CPLX) {
                        __builtin_nontemporal_store(w.x, &val[slot * R + q].x);
                        __builtin_nontemporal_store(w.y, &val[slot * R + q].y);
                    } else {
                        __builtin_nontemporal_store(w, &val[slot * R + q]);
                    }
                }
            }
        }
    }
    if constexpr (MODE == 0) {
        atomicAdd(&s_tot, mine);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(total, s_tot);
    }
}

// eps[J][X] = h_XX + sum_{Y in J, Y != X} V(X, Y) and vg[X][Y] = V(X, Y),
// V(X, Y) = (XX|YY) - (XY|YX) (spin-free: the exchange only for equal
// spins); then H_AA = H_JJ + the difference of a single or double
// excitation in O(1) (diag_delta).
template <bool CPLX>
__device__ __forceinline__ double vpair(const DevPlan &p, int X, int Y)
{
    const int n = p.n;
    if constexpr (CPLX) {
        const int M = p.M;
        return ((const double2 *)p.w_same)[((size_t)Y * M + X) * M + X].x;
    } else {
        const int x = X % n, y = Y % n;
        const double *w = (const double *)((X < n) == (Y < n) ? p.w_same : p.w_opp);
        return w[((size_t)y * n + x) * n + x];
    }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_pt2_tables(DevPlan p, double *eps, double *vg)
{
    const int M = p.M, n = p.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)M * M) {
        const int X = (int)(t / M), Y = (int)(t % M);
        vg[t] = X == Y ? 0.0 : vpair<CPLX>(p, X, Y);
    }
    if (t >= p.ndet * M) return;
    const int64_t J = t / M;
    const int X = (int)(t % M);
    const uint64_t j0 = p.dets[2 * J], j1 = p.dets[2 * J + 1];
    double e;
    if constexpr (CPLX) e = ((const double2 *)p.h)[(size_t)X * M + X].x;
    else e = ((const double *)p.h)[(size_t)(X % n) * n + (X % n)];
    for (int Y = 0; Y < M; Y++)
        if (Y != X && occ(j0, j1, n, Y)) e += vpair<CPLX>(p, X, Y);
    eps[t] = e;
}


// One wave per bucket of at most PT2_WCAP records (four buckets per block):
// the records are sorted in registers by a bitonic network over one 64-bit
// key (22 hash bits of A, then J, then the record's index), E = 1, 2, 4, 8
// or 16 keys per lane at positions lane * E + r, exchanged between lanes by
// shuffles.  The sorted keys go to LDS (one barrier); the runs are then
// reduced across the wave's lanes (below), so a long run of a much-connected
// external determinant does not serialise one lane; the energy and the
// counts of the bucket are summed over the wave by a fixed butterfly.
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src), hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&v)[16], int lane)
{
    constexpr int N = 64 * E;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int q = 0; q < E; q++) {
                    const int pq = q ^ j;
                    if (pq > q) {
                        const bool up = (((lane * E + q) & k) == 0);
                        const uint64_t x = v[q], y = v[pq];
                        if ((x > y) == up) {
                            v[q] = y;
                            v[pq] = x;
                        }
                    }
                }
            } else {
                const int lj = j / E;
                const bool lower = (lane & lj) == 0;
#pragma unroll
                for (int q = 0; q < E; q++) {
                    const uint64_t o = shfl64(v[q], lane ^ lj);
                    const bool up = (((lane * E + q) & k) == 0);
                    v[q] = (lower == up) ? (v[q] < o ? v[q] : o) : (v[q] > o ? v[q] : o);
                }
            }
        }
    }
}

// Sum the external determinants of one bucket from its records in sorted
// order, over the lanes of one wave: sorted positions [0, m), hib_at(p) the
// hash bits of the record at position p (equal within a run, one run per
// external A unless hash bits collide), rid_at(p) its record index.  Adds
// |num|^2 / (E0 - H_AA) per external determinant into the lane's acc, and
// the kept pairs and external determinants into kept and nq.
template <bool CPLX, int RM, class HibF, class RidF>
__device__ __forceinline__ void wave_runs(int m, uint64_t base, HibF hib_at, RidF rid_at, int R, const Roots &roots,
                                          const Rec *__restrict__ rec,
                                          const typename Scal<CPLX>::T *__restrict__ val, int lane,
                                          double (&acc)[RM], uint32_t &kept, uint32_t &nq)
{
    using T = typename Scal<CPLX>::T;
    // |sum over the records of run [i, e) whose A is (a0, a1), in run order
    // (ascending J)|^2 / (E0 - H_AA), H_AA from the first of them
    auto add_a = [&](int i, int e, uint64_t a0, uint64_t a1) {
        T num[RM];
#pragma unroll
        for (int k = 0; k < RM; k++) num[k] = sc_zero(T());
        int first = -1;
        for (int u = i; u < e; u++) {
            const int ru = rid_at(u);
            const Rec &x = rec[base + ru];
            if (x.a0 != a0 || x.a1 != a1) continue;
            if (first < 0) first = ru;
            const T *vv = val + (base + ru) * R;
#pragma unroll
            for (int k = 0; k < RM; k++)
                if (k < R) num[k] = sc_add(num[k], vv[k]);
            kept++;
        }
        nq++;
        const double haa = rec[base + first].haa;
#pragma unroll
        for (int k = 0; k < RM; k++) {
            if (k >= R) continue;
            double q;
            if constexpr (CPLX) q = num[k].x * num[k].x + num[k].y * num[k].y;
            else q = num[k] * num[k];
            acc[k] += q / (roots.e0[k] - haa);
        }
    };
    // Runs by a segmented reduction over the sorted positions, 64 per round
    // (lane = position - t0): the values of a run, its length, the H_AA of
    // its first record, its first position and whether any record has
    // another A than the one before it are combined left to right by a fixed
    // butterfly, and the state of the run still open at the end of a round
    // carries into the next.  A run of one A then adds its term at its last
    // position; the rare run shared by several A takes the serial path.
    auto shT = [](T x, int src) {
        if constexpr (CPLX) return make_double2(__shfl(x.x, src), __shfl(x.y, src));
        else return __shfl(x, src);
    };
    T cs[RM];
#pragma unroll
    for (int k = 0; k < RM; k++) cs[k] = sc_zero(T());
    uint32_t ccnt = 0;
    double chaa = 0.0;
    int chead = 0, cmul = 0;
    uint64_t ca0 = 0, ca1 = 0;
    for (int t0 = 0; t0 < m; t0 += 64) {
        const int p = t0 + lane;
        const bool act = p < m;
        T x[RM];
#pragma unroll
        for (int k = 0; k < RM; k++) x[k] = sc_zero(T());
        uint64_t a0 = 0, a1 = 0;
        double hh = 0.0;
        if (act) {
            const uint64_t ri = base + (uint64_t)rid_at(p);
            a0 = rec[ri].a0;
            a1 = rec[ri].a1;
            hh = rec[ri].haa;
#pragma unroll
            for (int k = 0; k < RM; k++)
                if (k < R) x[k] = val[ri * R + k];
        }
        const uint64_t u0 = shfl64(a0, lane ? lane - 1 : 0), u1 = shfl64(a1, lane ? lane - 1 : 0);
        const uint64_t pa0 = lane ? u0 : ca0, pa1 = lane ? u1 : ca1;
        const uint32_t hk = act ? hib_at(p) : 0u;
        const bool head = act && (p == 0 || hib_at(p - 1) != hk);
        int mul = (act && !head && (a0 != pa0 || a1 != pa1)) ? 1 : 0;
        uint32_t cn = act ? 1u : 0u;
        int hp = p;
        if (lane == 0 && act && !head) {
            // the run began in an earlier round: fold in its state
#pragma unroll
            for (int k = 0; k < RM; k++) x[k] = sc_add(cs[k], x[k]);
            cn += ccnt;
            hh = chaa;
            hp = chead;
            mul |= cmul;
        }
        int fl = (head || lane == 0 || !act) ? 1 : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int src = lane >= d ? lane - d : lane;
            T xu[RM];
#pragma unroll
            for (int k = 0; k < RM; k++)
                if (k < R) xu[k] = shT(x[k], src);
            const int fu = __shfl(fl, src), mu = __shfl(mul, src), hpu = __shfl(hp, src);
            const uint32_t cu = (uint32_t)__shfl((int)cn, src);
            const double hu = __shfl(hh, src);
            if (lane >= d && !fl) {
#pragma unroll
                for (int k = 0; k < RM; k++)
                    if (k < R) x[k] = sc_add(xu[k], x[k]);
                cn += cu;
                hh = hu;
                hp = hpu;
                mul |= mu;
                fl = fu;
            }
        }
        const bool last = act && (p == m - 1 || hib_at(p + 1) != hk);
        if (last) {
            if (!mul) {
#pragma unroll
                for (int k = 0; k < RM; k++) {
                    if (k >= R) continue;
                    double q;
                    if constexpr (CPLX) q = x[k].x * x[k].x + x[k].y * x[k].y;
                    else q = x[k] * x[k];
                    acc[k] += q / (roots.e0[k] - hh);
                }
                kept += cn;
                nq++;
            } else {
                // several A in the run [hp, p]: each in ascending (a0, a1)
                const int i = hp, e = p + 1;
                bool have = false;
                uint64_t c0 = 0, c1 = 0;
                for (;;) {
                    bool found = false;
                    uint64_t n0 = 0, n1 = 0;
                    for (int u = i; u < e; u++) {
                        const Rec &y = rec[base + rid_at(u)];
                        if (have && (y.a0 < c0 || (y.a0 == c0 && y.a1 <= c1))) continue;
                        if (!found || y.a0 < n0 || (y.a0 == n0 && y.a1 < n1)) { n0 = y.a0; n1 = y.a1; found = true; }
                    }
                    if (!found) break;
                    c0 = n0;
                    c1 = n1;
                    add_a(i, e, c0, c1);
                    have = true;
                }
            }
        }
        // state of the run open at the end of this round
#pragma unroll
        for (int k = 0; k < RM; k++)
            if (k < R) cs[k] = shT(x[k], 63);
        ccnt = (uint32_t)__shfl((int)cn, 63);
        chaa = __shfl(hh, 63);
        chead = __shfl(hp, 63);
        cmul = __shfl(mul, 63);
        ca0 = shfl64(a0, 63);
        ca1 = shfl64(a1, 63);
    }
}

// fixed butterfly over the wave; lane 0 writes the bucket's energies and
// counts to slot
template <int RM>
__device__ __forceinline__ void wave_store(double (&acc)[RM], uint32_t kept, uint32_t nq, int R, int lane,
                                           uint64_t slot, double *__restrict__ part,
                                           unsigned long long *__restrict__ partc)
{
#pragma unroll
    for (int k = 0; k < RM; k++) {
        if (k >= R) continue;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kept += (uint32_t)__shfl_xor((int)kept, o);
        nq += (uint32_t)__shfl_xor((int)nq, o);
    }
    if (lane == 0) {
        for (int k = 0; k < R; k++) part[slot * R + k] = acc[k];
        partc[2 * slot] = kept;
        partc[2 * slot + 1] = nq;
    }
}

template <bool CPLX, int RM>
__global__ __launch_bounds__(256) void k_pt2_bucket_wave(int R, Roots roots, uint32_t b0, int64_t nb,
                                                         const uint32_t *__restrict__ cnt,
                                                         const uint64_t *__restrict__ off, const Rec *__restrict__ rec,
                                                         const typename Scal<CPLX>::T *__restrict__ val,
                                                         double *__restrict__ part,
                                                         unsigned long long *__restrict__ partc, int64_t boff)
{
    __shared__ uint64_t sk[4][PT2_WCAP];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t bi = boff + (int64_t)blockIdx.x * 4 + wv;  // wave-uniform
    const uint32_t b = b0 + (uint32_t)(bi < nb ? bi : 0);
    const int m = bi < nb ? (int)cnt[b] : 0;
    const bool mine = bi < nb && m <= PT2_WCAP;  // larger buckets: k_pt2_bucket_big
    const uint64_t base = mine ? off[b] : 0;
    if (mine) {
        int E = 1;
        while (64 * E < m) E <<= 1;
        uint64_t v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int i = lane * E + q;
            v[q] = ~0ULL;
            if (q < E && i < m) {
                const uint64_t key = rec[base + i].key;
                v[q] = (((key >> 32) & 0x3FFFFFULL) << 42) | ((key & 0xFFFFFFFFULL) << 10) | (uint64_t)i;
            }
        }
        if (E == 1) wave_bitonic<1>(v, lane);
        else if (E == 2) wave_bitonic<2>(v, lane);
        else if (E == 4) wave_bitonic<4>(v, lane);
        else if (E == 8) wave_bitonic<8>(v, lane);
        else wave_bitonic<16>(v, lane);
#pragma unroll
        for (int q = 0; q < 16; q++)
            if (q < E) sk[wv][lane * E + q] = v[q];
    }
    __syncthreads();
    if (!mine) return;
    double acc[RM];
#pragma unroll
    for (int k = 0; k < RM; k++) acc[k] = 0.0;
    uint32_t kept = 0, nq = 0;
    const uint64_t *s = sk[wv];
    wave_runs<CPLX, RM>(
        m, base, [&](int q) { return (uint32_t)(s[q] >> 42); }, [&](int q) { return (int)(s[q] & 1023); }, R, roots,
        rec, val, lane, acc, kept, nq);
    wave_store<RM>(acc, kept, nq, R, lane, (uint64_t)bi, part, partc);
}

// Ascending sort of the pairs (K[i], X[i]), i < np2 (a power of two), in
// global memory by one workgroup: a bitonic network whose steps are
// separated by barriers; in one step every pair of positions is handled by
// one thread.
__device__ __forceinline__ void block_bitonic(uint64_t *K, uint32_t *X, int64_t np2)
{
    for (int64_t k = 2; k <= np2; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t i = threadIdx.x; i < np2; i += blockDim.x) {
                const int64_t l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t ki = K[i], kl = K[l];
                    const uint32_t xi = X[i], xl = X[l];
                    if ((ki != kl ? ki > kl : xi > xl) == up) {
                        K[i] = kl;
                        K[l] = ki;
                        X[i] = xl;
                        X[l] = xi;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Buckets of more than PT2_WCAP records (any size: an external determinant
// with very many partners, or a hash bucket far above the mean), one
// workgroup each: the records' keys (hash bits of A, then J) and indices
// are copied to the bucket's scratch (K, X at soff), sorted there, and one
// wave sums the runs as the wave kernel does.  Every record of an external
// determinant lies in its bucket, so its numerator is summed whole, in
// ascending J.
template <bool CPLX, int RM>
__global__ __launch_bounds__(256) void k_pt2_bucket_big(int R, Roots roots, uint32_t b0,
                                                        const uint32_t *__restrict__ list,
                                                        const uint64_t *__restrict__ soff,
                                                        const uint32_t *__restrict__ cnt,
                                                        const uint64_t *__restrict__ off, const Rec *__restrict__ rec,
                                                        const typename Scal<CPLX>::T *__restrict__ val, uint64_t *skey,
                                                        uint32_t *sidx, double *__restrict__ part,
                                                        unsigned long long *__restrict__ partc)
{
    const uint32_t b = list[blockIdx.x];
    const int m = (int)cnt[b];
    const uint64_t base = off[b];
    int64_t np2 = 1;
    while (np2 < m) np2 <<= 1;
    uint64_t *K = skey + soff[blockIdx.x];
    uint32_t *X = sidx + soff[blockIdx.x];
    for (int64_t i = threadIdx.x; i < np2; i += blockDim.x) {
        K[i] = i < m ? rec[base + i].key : ~0ULL;
        X[i] = (uint32_t)i;
    }
    __syncthreads();
    block_bitonic(K, X, np2);
    if (threadIdx.x >= 64) return;  // one wave sums the runs; no barrier follows
    const int lane = threadIdx.x;
    double acc[RM];
#pragma unroll
    for (int k = 0; k < RM; k++) acc[k] = 0.0;
    uint32_t kept = 0, nq = 0;
    wave_runs<CPLX, RM>(
        m, base, [&](int q) { return (uint32_t)(K[q] >> 32); }, [&](int q) { return (int)X[q]; }, R, roots, rec,
        val, lane, acc, kept, nq);
    wave_store<RM>(acc, kept, nq, R, lane, (uint64_t)(b - b0), part, partc);
}

// Fixed-order sums over the nb buckets of a pass in two stages: block g of
// k_pt2_sum1 reduces buckets [g*chunk, (g+1)*chunk) into tmp[g][R + 2]
// (R energies, then the two counts as doubles-free integers); k_pt2_sum2
// reduces the blocks.
constexpr int PT2_SUMB = 256;

__global__ __launch_bounds__(256) void k_pt2_sum1(int64_t nb, int R, const double *__restrict__ part,
                                                  const unsigned long long *__restrict__ partc, double *tmp,
                                                  unsigned long long *tmpc)
{
    __shared__ double red[256];
    __shared__ unsigned long long redc[256];
    const int64_t chunk = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(nb, lo + chunk);
    for (int k = 0; k < R + 2; k++) {
        double a = 0.0;
        unsigned long long ac = 0;
        for (int64_t b = lo + threadIdx.x; b < hi; b += blockDim.x) {
            if (k < R) a += part[b * R + k];
            else ac += partc[2 * b + (k - R)];
        }
        red[threadIdx.x] = a;
        redc[threadIdx.x] = ac;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[threadIdx.x] += red[threadIdx.x + s];
                redc[threadIdx.x] += redc[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (k < R) tmp[(size_t)blockIdx.x * R + k] = red[0];
            else tmpc[2 * (size_t)blockIdx.x + (k - R)] = redc[0];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_pt2_sum2(int R, const double *__restrict__ tmp,
                                                  const unsigned long long *__restrict__ tmpc, double *out,
                                                  unsigned long long *outc)
{
    __shared__ double red[256];
    __shared__ unsigned long long redc[256];
    for (int k = 0; k < R + 2; k++) {
        red[threadIdx.x] = k < R ? tmp[(size_t)threadIdx.x * R + k] : 0.0;
        redc[threadIdx.x] = k < R ? 0ULL : tmpc[2 * (size_t)threadIdx.x + (k - R)];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[threadIdx.x] += red[threadIdx.x + s];
                redc[threadIdx.x] += redc[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (k < R) out[k] = red[0];
            else outc[k - R] = redc[0];
        }
        __syncthreads();
    }
}

__global__ void k_fill_u32(uint32_t *x, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// claim words of the emit pass: capacity (the bucket's count) in the high
// half, claims (0) in the low half
__global__ void k_fill_cap(unsigned long long *w, const uint32_t *cnt, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = (unsigned long long)cnt[i] << 32;
}

void fill_u32(uint32_t *x, int64_t n, hipStream_t s, uint32_t v = 0u)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
}


int64_t choose(int a, int b)
{
    if (b < 0 || b > a) return 0;
    int64_t r = 1;
    for (int i = 1; i <= b; i++) r = r * (a - b + i) / i;
    return r;
}

bool classes(const DevPlan &d, int na, int nb_, ExcClasses &ex)
{
    ex = ExcClasses{};
    int64_t cntc[5];
    if (d.kind == MW_SPIN_FREE) {
        ex.no[0] = na; ex.nv[0] = d.n - na;
        ex.no[1] = nb_; ex.nv[1] = d.n - nb_;
        ex.nclass = 5;
        const int t[5] = {0, 0, 1, 1, 2}, s[5] = {0, 1, 0, 1, 0};
        for (int c = 0; c < 5; c++) { ex.type[c] = t[c]; ex.sec[c] = s[c]; }
        cntc[0] = (int64_t)ex.no[0] * ex.nv[0];
        cntc[1] = (int64_t)ex.no[1] * ex.nv[1];
        cntc[2] = choose(ex.no[0], 2) * choose(ex.nv[0], 2);
        cntc[3] = choose(ex.no[1], 2) * choose(ex.nv[1], 2);
        cntc[4] = (int64_t)ex.no[0] * ex.no[1] * ex.nv[0] * ex.nv[1];
    } else {
        ex.no[0] = na; ex.nv[0] = d.M - na;
        ex.nclass = 2;
        ex.type[0] = 0; ex.type[1] = 1; ex.sec[0] = ex.sec[1] = 0;
        cntc[0] = (int64_t)ex.no[0] * ex.nv[0];
        cntc[1] = choose(ex.no[0], 2) * choose(ex.nv[0], 2);
    }
    int64_t acc = 0;
    ex.start[0] = 0;
    for (int c = 0; c < ex.nclass; c++) {
        acc += cntc[c];
        if (acc >= ((int64_t)1 << 31)) return false;
        ex.start[c + 1] = (int)acc;
    }
    for (int c = ex.nclass + 1; c < 6; c++) ex.start[c] = ex.start[ex.nclass];
    return true;
}

uint64_t set_size(int64_t ndet)
{
    uint64_t z = 256;
    while (z < 2 * (uint64_t)ndet) z <<= 1;
    return z;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// configuration table of the space: slots, slot of each determinant, the
// largest |c| per slot, and per determinant the largest |c| over its
// configuration
size_t cfg_bytes(int64_t ndet)
{
    return align256(4 * set_size(ndet)) + align256(4 * (size_t)ndet) + align256(8 * set_size(ndet)) +
           align256(8 * (size_t)ndet);
}

struct CfgTable {
    uint32_t *slot, *cslot;
    unsigned long long *cmaxb;
    double *cm;
};

// carve the configuration table out of the work buffer (take: the buffer's
// bump allocator) and fill it for the vectors c
template <bool CPLX, class Take>
CfgTable cfg_table(const DevPlan &d, int R, const typename Scal<CPLX>::T *c, Take take, hipStream_t s)
{
    CfgTable t;
    const uint64_t zs = set_size(d.ndet);
    t.slot = (uint32_t *)take(4 * zs);
    t.cslot = (uint32_t *)take(4 * (size_t)d.ndet);
    t.cmaxb = (unsigned long long *)take(8 * zs);
    t.cm = (double *)take(8 * (size_t)d.ndet);
    if (d.ndet == 0) return t;
    fill_u32(t.slot, (int64_t)zs, s, 0xffffffffu);
    fill_u32((uint32_t *)t.cmaxb, 2 * (int64_t)zs, s, 0u);
    const unsigned g = (unsigned)((d.ndet + 255) / 256);
    hipLaunchKernelGGL(k_cfg_insert, dim3(g), dim3(256), 0, s, d.dets, d.ndet, t.slot, zs - 1, t.cslot);
    hipLaunchKernelGGL(k_cfg_max<CPLX>, dim3(g), dim3(256), 0, s, d.ndet, R, c, (const uint32_t *)t.cslot, t.cmaxb);
    hipLaunchKernelGGL(k_cfg_gather, dim3(g), dim3(256), 0, s, d.ndet, (const uint32_t *)t.cslot,
                       (const unsigned long long *)t.cmaxb, t.cm);
    return t;
}

// work-buffer layout (both the call and the size query use these)
size_t fixed_bytes(int64_t ndet, int M)
{
    return align256(8 * 16) + align256(8 * (PT2_MAXR + 2)) + align256(8 * (size_t)PT2_SUMB * PT2_MAXR) +
           align256(16 * (size_t)PT2_SUMB) + align256(8 * (size_t)ndet * M) + align256(8 * (size_t)M * M) +
           align256(4 * set_size(ndet)) + align256(16 * set_size(ndet)) + cfg_bytes(ndet);
}

// selection: 16 buckets per determinant of the space to start with
int sel_lognb(int64_t ndet)
{
    int lognb = 4;
    while (((int64_t)1 << lognb) < ndet * 16 && lognb < 24) lognb++;
    return lognb;
}

// selection bucket tables: cnt, fill, ucnt, big (4 B); off, uoff, bigoff (8 B)
size_t sel_table_bytes(int64_t NB) { return 4 * align256(4 * (size_t)NB) + 3 * align256(8 * (size_t)NB) + 1024; }

size_t table_bytes(int64_t NB, int R)
{
    // cnt, big; fill, off, bigoff; part; partc
    return align256(4 * (size_t)NB) * 2 + align256(8 * (size_t)NB) * 3 + align256(8 * (size_t)NB * R) +
           align256(16 * (size_t)NB) + 1024 + 512;
}

// ---------------------------------------------------------------------------
// selection of external determinants (iCIPT2 criterion, section 2.4)
// ---------------------------------------------------------------------------

// Eqs. (iCI_Selection-1) and (iCI_Selection-2) per pair (A, nu), nu a
// determinant of configuration J of P: the first test max_k |H c| >= cmin,
// the second max_k |H c / (E0_k - H_AA)| >= cmin; when A's configuration is
// doubly excited from J's (case B) the pair also needs H~ max|C| >= cmin,
// Table 1's bound times the largest |C| over J's configuration, a test
// shared by every determinant of J.  A is selected when one configuration J
// has a pair passing the first test and a pair passing the second (the
// maxima over nu of each test).  A pair passing neither cannot help and is
// not kept; with one root the two tests compare one quantity |H c| with
// two thresholds, so a configuration passes both exactly when one of its
// pairs does, and only such pairs are kept.  Kept pairs carry the key A and
// kx = configuration id << 2 | first << 1 | second.  MODE 0: count kept
// pairs; 1: per bucket; 2: write the keys of the buckets [b0, b1).
template <bool CPLX, int MODE>
__global__ __launch_bounds__(256) void k_sel_enum(DevPlan p, ExcClasses ex, DetSet inP, int R,
                                                  const typename Scal<CPLX>::T *__restrict__ c, Roots roots,
                                                  double cmin, int lognb, uint32_t b0, uint32_t b1, uint32_t *cnt,
                                                  const uint64_t *__restrict__ off, uint32_t *fill, ulonglong2 *keys,
                                                  unsigned long long *kx, const double *__restrict__ eps,
                                                  const double *__restrict__ vg, unsigned long long *total,
                                                  int64_t jbase, const double *__restrict__ cm,
                                                  const uint32_t *__restrict__ cslot)
{
    using T = typename Scal<CPLX>::T;
    __shared__ uint8_t ol[2][128], vl[2][128];
    __shared__ T s_c[PT2_MAXR];
    __shared__ double s_eps[128];
    __shared__ unsigned long long s_tot;
    const int64_t J = jbase + blockIdx.x;
    const uint64_t j0 = p.dets[2 * J], j1 = p.dets[2 * J + 1];
    const int n = p.n;
    if ((int)threadIdx.x < p.M) s_eps[threadIdx.x] = eps[J * p.M + threadIdx.x];
    if (threadIdx.x == 0) {
        int no[2] = {0, 0}, nv[2] = {0, 0};
        for (int X = 0; X < 2 * n; X++) {
            const int s = CPLX ? 0 : X / n;
            if (occ(j0, j1, n, X)) ol[s][no[s]++] = (uint8_t)X;
            else vl[s][nv[s]++] = (uint8_t)X;
        }
        for (int k = 0; k < R; k++) s_c[k] = c[(size_t)J * R + k];
        s_tot = 0;
    }
    __syncthreads();
    double hjj;
    if constexpr (CPLX) hjj = ((const double2 *)p.diag)[J].x;
    else hjj = ((const double *)p.diag)[J];
    const double cmj = cm[J];
    const unsigned long long cfg = (unsigned long long)cslot[J] << 2;
    const int E = ex.start[ex.nclass];
    unsigned long long mine = 0;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        int Q, S, P, Rr;
        decode(ex, ol, vl, e, Q, S, P, Rr);
        uint64_t a0 = j0, a1 = j1;
        flip(a0, a1, n, Q);
        flip(a0, a1, n, P);
        if (S >= 0) {
            flip(a0, a1, n, S);
            flip(a0, a1, n, Rr);
        }
        const uint64_t h = hash_det(a0, a1);
        if (in_set(inP, h, a0, a1)) continue;
        if (S >= 0) {
            double bound;
            if (cfg_double<CPLX>(p, Q, S, P, Rr, bound) && !(bound * cmj >= cmin)) continue;
        }
        const T v = exc_value<CPLX>(p, j0, j1, Q, S, P, Rr);
        const double haa = hjj + diag_delta(s_eps, vg, p.M, Q, S, P, Rr);
        double m1 = 0.0, m2 = 0.0;
        for (int k = 0; k < R; k++) {
            const double a = mag(sc_mul(v, s_c[k]));
            m1 = fmax(m1, a);
            m2 = fmax(m2, a / fabs(roots.e0[k] - haa));
        }
        const bool t1 = m1 >= cmin, t2 = m2 >= cmin;
        if (R == 1 ? !(t1 && t2) : !(t1 || t2)) continue;
        if constexpr (MODE == 0) {
            mine++;
        } else {
            const uint32_t b = bucket_of(h, lognb);
            if constexpr (MODE == 1) {
                atomicAdd(&cnt[b], 1u);
            } else {
                if (b < b0 || b >= b1) continue;
                const uint32_t k = atomicAdd(&fill[b], 1u);
                if (k < cnt[b]) {
                    __builtin_nontemporal_store(a0, &keys[off[b] + k].x);
                    __builtin_nontemporal_store(a1, &keys[off[b] + k].y);
                    __builtin_nontemporal_store(cfg | (t1 ? 2ULL : 0ULL) | (t2 ? 1ULL : 0ULL), &kx[off[b] + k]);
                }
            }
        }
    }
    if constexpr (MODE == 0) {
        atomicAdd(&s_tot, mine);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(total, s_tot);
    }
}

// The selected determinants of one bucket from its keys sorted by (a0, a1,
// kx) at positions [0, m): a distinct A is selected when, within one
// configuration group of its records (equal kx >> 2), one record passed
// the first test and one the second.  The workgroup's threads take
// contiguous position ranges (a run starting in a thread's range is that
// thread's, read to its end); an exclusive scan of their counts places the
// selected A in sorted order at out.  Returns the count (every thread).
template <class Get>
__device__ uint32_t sel_compact(int64_t m, Get get, ulonglong2 *out, uint32_t *sc)
{
    const int64_t per = (m + 255) / 256;
    const int64_t lo = min(m, (int64_t)threadIdx.x * per), hi = min(m, lo + per);
    auto starts = [&](int64_t i) {
        if (i == 0) return true;
        const ulonglong2 x = get(i).k, y = get(i - 1).k;
        return x.x != y.x || x.y != y.y;
    };
    auto selected = [&](int64_t i) {
        const ulonglong2 a = get(i).k;
        int64_t g0 = i;
        while (g0 < m) {
            const auto r0 = get(g0);
            if (r0.k.x != a.x || r0.k.y != a.y) break;
            const unsigned long long cfg = r0.x >> 2;
            unsigned long long f = 0;
            int64_t g1 = g0;
            while (g1 < m) {
                const auto r = get(g1);
                if (r.k.x != a.x || r.k.y != a.y || (r.x >> 2) != cfg) break;
                f |= r.x & 3ULL;
                g1++;
            }
            if (f == 3) return true;
            g0 = g1;
        }
        return false;
    };
    uint32_t cnt = 0;
    for (int64_t i = lo; i < hi; i++)
        if (starts(i) && selected(i)) cnt++;
    sc[threadIdx.x] = cnt;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t v = (int)threadIdx.x >= o ? sc[threadIdx.x - o] : 0u;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t u = sc[threadIdx.x] - cnt;
    const uint32_t total = sc[255];
    for (int64_t i = lo; i < hi; i++)
        if (starts(i) && selected(i)) out[u++] = get(i).k;
    return total;
}

struct SelKey {
    ulonglong2 k;
    unsigned long long x;
};

// Buckets of at most SEL_CAP keys, one workgroup each: the keys sorted in
// LDS by (a0, a1, kx), the selected A written back to the front of the
// bucket's slice, ucnt[b] = how many.
__global__ __launch_bounds__(256) void k_sel_unique(uint32_t b0, const uint32_t *__restrict__ cnt,
                                                    const uint64_t *__restrict__ off, ulonglong2 *keys,
                                                    const unsigned long long *__restrict__ kx, uint32_t *ucnt,
                                                    uint32_t boff)
{
    __shared__ uint64_t s0[SEL_CAP], s1[SEL_CAP], s2[SEL_CAP];
    __shared__ uint32_t sc[256];
    const uint32_t b = b0 + boff + blockIdx.x;
    const int m = (int)cnt[b];
    if (m > SEL_CAP) return;  // k_sel_unique_big
    ulonglong2 *kb = keys + off[b];
    const unsigned long long *xb = kx + off[b];
    int np2 = 1;
    while (np2 < m) np2 <<= 1;
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        if (i < m) {
            const ulonglong2 k = kb[i];
            s0[i] = k.x;
            s1[i] = k.y;
            s2[i] = xb[i];
        } else {
            s0[i] = s1[i] = s2[i] = ~0ULL;
        }
    }
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < np2; i += blockDim.x) {
                const int l = i ^ jj;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t x0 = s0[i], x1 = s1[i], x2 = s2[i], y0 = s0[l], y1 = s1[l], y2 = s2[l];
                    const bool gt = x0 != y0 ? x0 > y0 : (x1 != y1 ? x1 > y1 : x2 > y2);
                    if (gt == up) {
                        s0[i] = y0; s1[i] = y1; s2[i] = y2;
                        s0[l] = x0; s1[l] = x1; s2[l] = x2;
                    }
                }
            }
            __syncthreads();
        }
    }
    const uint32_t u = sel_compact(
        m, [&](int64_t i) { return SelKey{make_ulonglong2(s0[i], s1[i]), s2[i]}; }, kb, sc);
    if (threadIdx.x == 0) ucnt[b] = u;
}

// Buckets of more than SEL_CAP keys (any size), one workgroup each: the
// keys copied to the bucket's scratch (K0, K1, K2 at soff), sorted there by
// a bitonic network in global memory, then compacted as above.
__global__ __launch_bounds__(256) void k_sel_unique_big(const uint32_t *__restrict__ list,
                                                        const uint64_t *__restrict__ soff,
                                                        const uint32_t *__restrict__ cnt,
                                                        const uint64_t *__restrict__ off, ulonglong2 *keys,
                                                        const unsigned long long *__restrict__ kx, uint64_t *scr,
                                                        uint64_t nscr, uint32_t *ucnt)
{
    __shared__ uint32_t sc[256];
    const uint32_t b = list[blockIdx.x];
    const int64_t m = cnt[b];
    ulonglong2 *kb = keys + off[b];
    const unsigned long long *xb = kx + off[b];
    int64_t np2 = 1;
    while (np2 < m) np2 <<= 1;
    uint64_t *K0 = scr + soff[blockIdx.x], *K1 = K0 + nscr, *K2 = K1 + nscr;
    for (int64_t i = threadIdx.x; i < np2; i += blockDim.x) {
        if (i < m) {
            const ulonglong2 k = kb[i];
            K0[i] = k.x;
            K1[i] = k.y;
            K2[i] = xb[i];
        } else {
            K0[i] = K1[i] = K2[i] = ~0ULL;
        }
    }
    __syncthreads();
    for (int64_t k = 2; k <= np2; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t i = threadIdx.x; i < np2; i += blockDim.x) {
                const int64_t l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t x0 = K0[i], x1 = K1[i], x2 = K2[i], y0 = K0[l], y1 = K1[l], y2 = K2[l];
                    const bool gt = x0 != y0 ? x0 > y0 : (x1 != y1 ? x1 > y1 : x2 > y2);
                    if (gt == up) {
                        K0[i] = y0; K1[i] = y1; K2[i] = y2;
                        K0[l] = x0; K1[l] = x1; K2[l] = x2;
                    }
                }
            }
            __syncthreads();
        }
    }
    const uint32_t u = sel_compact(
        m, [&](int64_t i) { return SelKey{make_ulonglong2(K0[i], K1[i]), K2[i]}; }, kb, sc);
    if (threadIdx.x == 0) ucnt[b] = u;
}

// out[uoff[b] + i] = the i-th distinct key of bucket b (b in [b0, b0 + nb))
__global__ __launch_bounds__(256) void k_sel_copy(uint32_t b0, int64_t nb, const uint32_t *__restrict__ ucnt,
                                                  const uint64_t *__restrict__ off, const uint64_t *__restrict__ uoff,
                                                  const ulonglong2 *__restrict__ keys, uint64_t *out, uint64_t max_out,
                                                  uint32_t boff)
{
    const int64_t bi = (int64_t)boff + blockIdx.x;
    if (bi >= nb) return;
    const uint32_t b = b0 + (uint32_t)bi;
    const uint32_t u = ucnt[b];
    for (uint32_t i = threadIdx.x; i < u; i += blockDim.x) {
        const uint64_t o = uoff[b] + i;
        if (o < max_out) {
            const ulonglong2 k = keys[off[b] + i];
            out[2 * o] = k.x;
            out[2 * o + 1] = k.y;
        }
    }
}

// A dispatch counts its work-items in 32 bits: grids are cut into chunks of
// at most 2^22 workgroups of 256.
constexpr int64_t PT2_MAXGRID = (int64_t)1 << 22;

template <bool CPLX, int MODE>
void launch_enum(const DevPlan &d, const ExcClasses &ex, const DetSet &inP, int R, const typename Scal<CPLX>::T *c,
                 double qmin, int lognb, uint32_t b0, uint32_t b1, uint32_t *cnt, const uint64_t *off,
                 unsigned long long *fill,
                 Rec *rec, typename Scal<CPLX>::T *val, const double *eps, const double *vg, unsigned long long *tot,
                 const double *cm, hipStream_t s)
{
    // hash bits kept in the records' sort key: all 32, or fewer when the
    // environment sets MW_PT2_KEY_BITS (1..31) to test runs of several A
    uint32_t kmask = 0xffffffffu;
    if (const char *e = getenv("MW_PT2_KEY_BITS")) {
        const int bits = atoi(e);
        if (bits >= 1 && bits < 32) kmask = (1u << bits) - 1u;
    }
    for (int64_t j = 0; j < d.ndet; j += PT2_MAXGRID) {
        const unsigned g = (unsigned)std::min<int64_t>(PT2_MAXGRID, d.ndet - j);
        hipLaunchKernelGGL((k_pt2_enum<CPLX, MODE>), dim3(g), dim3(256), 0, s, d, ex, inP, R, c, qmin, lognb, b0, b1,
                           cnt, off, fill, rec, val, eps, vg, tot, j, kmask, cm);
    }
}

template <bool CPLX>
void launch_bucket_wave(int64_t nb, int R, const Roots &roots, uint32_t b0, const uint32_t *cnt, const uint64_t *off,
                        const Rec *rec, const typename Scal<CPLX>::T *val, double *part, unsigned long long *partc,
                        hipStream_t s)
{
    const int64_t nblocks = (nb + 3) / 4;
    for (int64_t o = 0; o < nblocks; o += PT2_MAXGRID) {
        const unsigned g = (unsigned)std::min<int64_t>(PT2_MAXGRID, nblocks - o);
        // one root: arrays of one slot (fewer registers, more waves)
        if (R == 1)
            hipLaunchKernelGGL((k_pt2_bucket_wave<CPLX, 1>), dim3(g), dim3(256), 0, s, R, roots, b0, nb, cnt, off, rec,
                               val, part, partc, o * 4);
        else
            hipLaunchKernelGGL((k_pt2_bucket_wave<CPLX, PT2_MAXR>), dim3(g), dim3(256), 0, s, R, roots, b0, nb, cnt, off,
                               rec, val, part, partc, o * 4);
    }
}

template <bool CPLX>
mw_status pt2_t(const DevPlan &d, int R, const void *cv, const double *e0, double qmin, void *work,
                size_t work_bytes, double *e2, int64_t *stats, hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    const T *c = (const T *)cv;
    // particle numbers from the first determinant
    uint64_t first[2];
    if (hipMemcpyAsync(first, d.dets, 16, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(MW_EHIP, "pt2: reading the space failed");
    const int na = __builtin_popcountll(first[0]) + (CPLX ? __builtin_popcountll(first[1]) : 0);
    const int nbeta = CPLX ? 0 : __builtin_popcountll(first[1]);
    ExcClasses ex;
    if (!classes(d, na, nbeta, ex)) return fail(MW_EUNSUPPORTED, "pt2: more than 2^31 excitations per determinant");
    Roots roots{};
    for (int k = 0; k < R; k++) roots.e0[k] = e0[k];
    for (int k = 0; k < R; k++) e2[k] = 0.0;
    int64_t st[5] = {0, 0, 0, 0, 0};  // kept pairs, external A, passes, buckets, excitations enumerated

    char *w = (char *)work;
    size_t used = 0;
    auto take = [&](size_t bytes) -> char * {
        char *x = w + used;
        used += align256(bytes);
        return x;
    };
    unsigned long long *tot = (unsigned long long *)take(8 * 16);
    double *sums = (double *)take(8 * (PT2_MAXR + 2));
    unsigned long long *sumc = (unsigned long long *)(sums + PT2_MAXR);
    double *stmp = (double *)take(8 * (size_t)PT2_SUMB * PT2_MAXR);
    unsigned long long *stmpc = (unsigned long long *)take(16 * (size_t)PT2_SUMB);
    double *eps = (double *)take(8 * (size_t)d.ndet * d.M);
    double *vg = (double *)take(8 * (size_t)d.M * d.M);
    const uint64_t zs = set_size(d.ndet);
    uint32_t *sslot = (uint32_t *)take(4 * zs);
    ulonglong2 *skey = (ulonglong2 *)take(16 * zs);
    if (used + cfg_bytes(d.ndet) > work_bytes) return fail(MW_EWORKSPACE, "pt2: work buffer too small");
    const DetSet inP{skey, zs - 1};
    if (d.ndet > 0 && ex.start[ex.nclass] > 0) {
        fill_u32(sslot, (int64_t)zs, s, 0xffffffffu);
        hipLaunchKernelGGL(k_set_insert, dim3((unsigned)((d.ndet + 255) / 256)), dim3(256), 0, s, d.dets, d.ndet, sslot,
                           zs - 1);
        hipLaunchKernelGGL(k_set_keys, dim3((unsigned)((zs + 255) / 256)), dim3(256), 0, s, d.dets,
                           (const uint32_t *)sslot, zs, skey);
        const int64_t nt = std::max<int64_t>(d.ndet * d.M, (int64_t)d.M * d.M);
        hipLaunchKernelGGL(k_pt2_tables<CPLX>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, d, eps, vg);
        // the largest |C| over every configuration (screening only)
        const double *cm = nullptr;
        if (qmin > 0.0) cm = cfg_table<CPLX>(d, R, c, take, s).cm;
        // kept pairs: counted when screening, else bounded by every excitation
        unsigned long long T_ = (unsigned long long)d.ndet * (unsigned long long)ex.start[ex.nclass];
        if (qmin > 0.0) {
            hipMemsetAsync(tot, 0, 8, s);
            launch_enum<CPLX, 0>(d, ex, inP, R, c, qmin, 0, 0u, 0u, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, tot, cm, s);
            if (hipMemcpyAsync(&T_, tot, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(MW_EHIP, "pt2: counting pass failed");
        }
        st[4] = d.ndet * (int64_t)ex.start[ex.nclass];  // excitations enumerated per pass
        if (T_ > 0) {
            // buckets of about PT2_MEAN records; any bucket, however large,
            // is handled (over PT2_WCAP records by k_pt2_bucket_big), so the
            // count is sized once
            int lognb = 0;
            while (((uint64_t)PT2_MEAN << lognb) < T_ && lognb < 32) lognb++;
            const int64_t NB = (int64_t)1 << lognb;
            uint32_t *cnt = (uint32_t *)take(4 * (size_t)NB);
            unsigned long long *fill = (unsigned long long *)take(8 * (size_t)NB);
            uint64_t *off = (uint64_t *)take(8 * (size_t)NB);
            double *part = (double *)take(8 * (size_t)NB * R);
            unsigned long long *partc = (unsigned long long *)take(16 * (size_t)NB);
            uint32_t *big = (uint32_t *)take(4 * (size_t)NB);
            uint64_t *bigoff = (uint64_t *)take(8 * (size_t)NB);
            if (used + 1024 > work_bytes) return fail(MW_EWORKSPACE, "pt2: work buffer too small for the bucket tables");
            fill_u32(cnt, NB, s);
            launch_enum<CPLX, 1>(d, ex, inP, R, c, qmin, lognb, 0u, 0u, cnt, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, cm, s);
            if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "pt2: counting launch failed");
            std::vector<uint32_t> hc(NB);
            if (hipMemcpyAsync(hc.data(), cnt, 4 * (size_t)NB, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(MW_EHIP, "pt2: bucket counting failed");
            // passes over bucket ranges whose records (32 B + R values each)
            // and, for the large buckets, sort scratch (12 B per position of
            // the power-of-two range) fit the rest of the buffer
            const size_t avail = work_bytes - used - 1024;
            auto np2_of = [](uint64_t m) {
                uint64_t q = 1;
                while (q < m) q <<= 1;
                return q;
            };
            auto pass_bytes = [&](uint64_t nrec, uint64_t nscr) {
                return align256(nrec * sizeof(Rec)) + align256(nrec * R * sizeof(T)) + align256(8 * nscr) +
                       align256(4 * nscr);
            };
            std::vector<uint64_t> ho(NB);
            int64_t b0 = 0;
            while (b0 < NB) {
                uint64_t acc = 0, scr = 0;
                int64_t b1 = b0;
                std::vector<uint32_t> hb;
                std::vector<uint64_t> hbo;
                while (b1 < NB) {
                    const uint64_t add = hc[b1] > (uint32_t)PT2_WCAP ? np2_of(hc[b1]) : 0;
                    if (pass_bytes(acc + hc[b1], scr + add) > avail) break;
                    ho[b1] = acc;
                    acc += hc[b1];
                    if (add) {
                        hb.push_back((uint32_t)b1);
                        hbo.push_back(scr);
                    }
                    scr += add;
                    b1++;
                }
                if (b1 == b0) return fail(MW_EWORKSPACE, "pt2: work buffer too small for one bucket");
                Rec *rec = (Rec *)(w + used);
                T *val = (T *)((char *)rec + align256(acc * sizeof(Rec)));
                uint64_t *skey2 = (uint64_t *)((char *)val + align256(acc * R * sizeof(T)));
                uint32_t *sidx = (uint32_t *)((char *)skey2 + align256(8 * scr));
                hipMemcpyAsync(off + b0, ho.data() + b0, 8 * (size_t)(b1 - b0), hipMemcpyHostToDevice, s);
                hipLaunchKernelGGL(k_fill_cap, dim3((unsigned)((b1 - b0 + 255) / 256)), dim3(256), 0, s, fill + b0,
                                   (const uint32_t *)cnt + b0, (int64_t)(b1 - b0));
                ProfToken t = prof_begin("pt2_enum", s);
                launch_enum<CPLX, 2>(d, ex, inP, R, c, qmin, lognb, (uint32_t)b0, (uint32_t)b1, cnt, off, fill, rec,
                                     val, eps, vg, nullptr, cm, s);
                prof_end(t, s);
                t = prof_begin("pt2_bucket", s);
                launch_bucket_wave<CPLX>(b1 - b0, R, roots, (uint32_t)b0, cnt, off, rec, val, part, partc, s);
                prof_end(t, s);
                if (!hb.empty()) {
                    // one workgroup per large bucket (a grid of at most 2^22
                    // workgroups per dispatch)
                    hipMemcpyAsync(big, hb.data(), 4 * hb.size(), hipMemcpyHostToDevice, s);
                    hipMemcpyAsync(bigoff, hbo.data(), 8 * hbo.size(), hipMemcpyHostToDevice, s);
                    t = prof_begin("pt2_bucket_big", s);
                    for (int64_t o = 0; o < (int64_t)hb.size(); o += PT2_MAXGRID) {
                        const unsigned g = (unsigned)std::min<int64_t>(PT2_MAXGRID, (int64_t)hb.size() - o);
                        if (R == 1)
                            hipLaunchKernelGGL((k_pt2_bucket_big<CPLX, 1>), dim3(g), dim3(256), 0, s, R, roots,
                                               (uint32_t)b0, (const uint32_t *)big + o, (const uint64_t *)bigoff + o,
                                               (const uint32_t *)cnt, (const uint64_t *)off, (const Rec *)rec,
                                               (const T *)val, skey2, sidx, part, partc);
                        else
                            hipLaunchKernelGGL((k_pt2_bucket_big<CPLX, PT2_MAXR>), dim3(g), dim3(256), 0, s, R, roots,
                                               (uint32_t)b0, (const uint32_t *)big + o, (const uint64_t *)bigoff + o,
                                               (const uint32_t *)cnt, (const uint64_t *)off, (const Rec *)rec,
                                               (const T *)val, skey2, sidx, part, partc);
                    }
                    prof_end(t, s);
                }
                if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "pt2: pass launch failed");
                hipLaunchKernelGGL(k_pt2_sum1, dim3(PT2_SUMB), dim3(256), 0, s, b1 - b0, R, (const double *)part,
                                   (const unsigned long long *)partc, stmp, stmpc);
                hipLaunchKernelGGL(k_pt2_sum2, dim3(1), dim3(PT2_SUMB), 0, s, R, (const double *)stmp,
                                   (const unsigned long long *)stmpc, sums, sumc);
                double hs[PT2_MAXR + 2];
                if (hipMemcpyAsync(hs, sums, 8 * (PT2_MAXR + 2), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return fail(MW_EHIP, "pt2: pass failed");
                for (int k = 0; k < R; k++) e2[k] += hs[k];
                unsigned long long hcnt[2];
                memcpy(hcnt, hs + PT2_MAXR, 16);
                st[0] += (int64_t)hcnt[0];
                st[1] += (int64_t)hcnt[1];
                st[2]++;
                b0 = b1;
            }
            st[3] = NB;
        }
    }
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "pt2 kernel launch failed");
    if (stats)
        for (int i = 0; i < 5; i++) stats[i] = st[i];
    return MW_OK;
}

template <bool CPLX>
mw_status select_t(const DevPlan &d, int R, const void *cv, const double *e0, double cmin, void *work,
                   size_t work_bytes, uint64_t *out, int64_t max_out, int64_t *count, hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    const T *c = (const T *)cv;
    uint64_t first[2];
    if (hipMemcpyAsync(first, d.dets, 16, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(MW_EHIP, "select: reading the space failed");
    const int na = __builtin_popcountll(first[0]) + (CPLX ? __builtin_popcountll(first[1]) : 0);
    const int nbeta = CPLX ? 0 : __builtin_popcountll(first[1]);
    ExcClasses ex;
    if (!classes(d, na, nbeta, ex)) return fail(MW_EUNSUPPORTED, "select: more than 2^31 excitations per determinant");
    Roots roots{};
    for (int k = 0; k < R; k++) roots.e0[k] = e0[k];
    *count = 0;
    char *w = (char *)work;
    size_t used = 0;
    auto take = [&](size_t bytes) -> char * {
        char *x = w + used;
        used += align256(bytes);
        return x;
    };
    unsigned long long *tot = (unsigned long long *)take(8 * 16);
    double *eps = (double *)take(8 * (size_t)d.ndet * d.M);
    double *vg = (double *)take(8 * (size_t)d.M * d.M);
    const uint64_t zs = set_size(d.ndet);
    uint32_t *sslot = (uint32_t *)take(4 * zs);
    ulonglong2 *skey = (ulonglong2 *)take(16 * zs);
    if (used + cfg_bytes(d.ndet) > work_bytes) return fail(MW_EWORKSPACE, "select: work buffer too small");
    const DetSet inP{skey, zs - 1};
    if (d.ndet == 0 || ex.start[ex.nclass] == 0) return MW_OK;
    fill_u32(sslot, (int64_t)zs, s, 0xffffffffu);
    hipLaunchKernelGGL(k_set_insert, dim3((unsigned)((d.ndet + 255) / 256)), dim3(256), 0, s, d.dets, d.ndet, sslot,
                       zs - 1);
    hipLaunchKernelGGL(k_set_keys, dim3((unsigned)((zs + 255) / 256)), dim3(256), 0, s, d.dets, (const uint32_t *)sslot,
                       zs, skey);
    const int64_t nt = std::max<int64_t>(d.ndet * d.M, (int64_t)d.M * d.M);
    hipLaunchKernelGGL(k_pt2_tables<CPLX>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, d, eps, vg);
    // configuration ids and the largest |C| over every configuration
    const CfgTable cfg = cfg_table<CPLX>(d, R, c, take, s);
    auto enumerate = [&](auto mode, int lognb, uint32_t b0, uint32_t b1, uint32_t *cnt, const uint64_t *off,
                         uint32_t *fill, ulonglong2 *keys, unsigned long long *kx) {
        constexpr int MODE = decltype(mode)::value;
        for (int64_t j = 0; j < d.ndet; j += PT2_MAXGRID) {
            const unsigned g = (unsigned)std::min<int64_t>(PT2_MAXGRID, d.ndet - j);
            hipLaunchKernelGGL((k_sel_enum<CPLX, MODE>), dim3(g), dim3(256), 0, s, d, ex, inP, R, c, roots, cmin, lognb,
                               b0, b1, cnt, off, fill, keys, kx, (const double *)eps, (const double *)vg, tot, j,
                               (const double *)cfg.cm, (const uint32_t *)cfg.cslot);
        }
    };
    // bucket count: 16 per determinant of the space to start with; the
    // per-bucket counting pass gives the total too, and when the buckets
    // average more than 4 PT2_MEAN keys the count is redone once with
    // buckets sized from that total.  Buckets of any size are handled.
    int lognb = sel_lognb(d.ndet);
    const size_t fixed = used;
    std::vector<uint32_t> hc, hu;
    for (int attempt = 0;; attempt++) {
        const int64_t NB = (int64_t)1 << lognb;
        used = fixed;
        uint32_t *cnt = (uint32_t *)take(4 * (size_t)NB);
        uint32_t *fill = (uint32_t *)take(4 * (size_t)NB);
        uint32_t *ucnt = (uint32_t *)take(4 * (size_t)NB);
        uint32_t *big = (uint32_t *)take(4 * (size_t)NB);
        uint64_t *off = (uint64_t *)take(8 * (size_t)NB);
        uint64_t *uoff = (uint64_t *)take(8 * (size_t)NB);
        uint64_t *bigoff = (uint64_t *)take(8 * (size_t)NB);
        if (used + 1024 > work_bytes) return fail(MW_EWORKSPACE, "select: work buffer too small for the bucket tables");
        fill_u32(cnt, NB, s);
        enumerate(std::integral_constant<int, 1>(), lognb, 0u, 0u, cnt, nullptr, nullptr, nullptr, nullptr);
        if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "select: counting launch failed");
        hc.resize(NB);
        if (hipMemcpyAsync(hc.data(), cnt, 4 * (size_t)NB, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MW_EHIP, "select: bucket counting failed");
        uint64_t T_ = 0;
        for (uint32_t x : hc) T_ += x;
        if (T_ == 0) return MW_OK;
        if (attempt == 0 && T_ > (uint64_t)NB * 4 * PT2_MEAN && lognb < 32) {
            while (((uint64_t)PT2_MEAN << lognb) < T_ && lognb < 32) lognb++;
            continue;
        }
        // passes over bucket ranges whose keys (16 B + 8 B each) and, for the
        // large buckets, sort scratch (24 B per position of the power-of-two
        // range) fit the rest of the buffer
        const size_t avail = work_bytes - used - 1024;
        auto np2_of = [](uint64_t m) {
            uint64_t q = 1;
            while (q < m) q <<= 1;
            return q;
        };
        auto pass_bytes = [&](uint64_t nk, uint64_t nscr) {
            return align256(16 * nk) + align256(8 * nk) + align256(24 * nscr);
        };
        std::vector<uint64_t> ho(NB), huo(NB);
        hu.resize(NB);
        uint64_t written = 0;
        int64_t b0 = 0;
        while (b0 < NB) {
            uint64_t acc = 0, scr = 0;
            int64_t b1 = b0;
            std::vector<uint32_t> hb;
            std::vector<uint64_t> hbo;
            while (b1 < NB) {
                const uint64_t add = hc[b1] > (uint32_t)SEL_CAP ? np2_of(hc[b1]) : 0;
                if (pass_bytes(acc + hc[b1], scr + add) > avail) break;
                ho[b1] = acc;
                acc += hc[b1];
                if (add) {
                    hb.push_back((uint32_t)b1);
                    hbo.push_back(scr);
                }
                scr += add;
                b1++;
            }
            if (b1 == b0) return fail(MW_EWORKSPACE, "select: work buffer too small for one bucket");
            ulonglong2 *keys = (ulonglong2 *)(w + used);
            unsigned long long *kx = (unsigned long long *)((char *)keys + align256(16 * acc));
            uint64_t *scrp = (uint64_t *)((char *)kx + align256(8 * acc));
            hipMemcpyAsync(off + b0, ho.data() + b0, 8 * (size_t)(b1 - b0), hipMemcpyHostToDevice, s);
            fill_u32(fill + b0, b1 - b0, s);
            enumerate(std::integral_constant<int, 2>(), lognb, (uint32_t)b0, (uint32_t)b1, cnt, off, fill, keys, kx);
            for (int64_t o = 0; o < b1 - b0; o += PT2_MAXGRID)
                hipLaunchKernelGGL(k_sel_unique, dim3((unsigned)std::min<int64_t>(PT2_MAXGRID, b1 - b0 - o)), dim3(256),
                                   0, s, (uint32_t)b0, (const uint32_t *)cnt, (const uint64_t *)off, keys,
                                   (const unsigned long long *)kx, ucnt, (uint32_t)o);
            if (!hb.empty()) {
                hipMemcpyAsync(big, hb.data(), 4 * hb.size(), hipMemcpyHostToDevice, s);
                hipMemcpyAsync(bigoff, hbo.data(), 8 * hbo.size(), hipMemcpyHostToDevice, s);
                ProfToken t = prof_begin("sel_unique_big", s);
                for (int64_t o = 0; o < (int64_t)hb.size(); o += PT2_MAXGRID)
                    hipLaunchKernelGGL(k_sel_unique_big,
                                       dim3((unsigned)std::min<int64_t>(PT2_MAXGRID, (int64_t)hb.size() - o)), dim3(256),
                                       0, s, (const uint32_t *)big + o, (const uint64_t *)bigoff + o,
                                       (const uint32_t *)cnt, (const uint64_t *)off, keys,
                                       (const unsigned long long *)kx, scrp, scr, ucnt);
                prof_end(t, s);
            }
            if (hipMemcpyAsync(hu.data() + b0, ucnt + b0, 4 * (size_t)(b1 - b0), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(MW_EHIP, "select: pass failed");
            for (int64_t b = b0; b < b1; b++) {
                huo[b] = written;
                written += hu[b];
            }
            if (out && max_out > 0) {
                hipMemcpyAsync(uoff + b0, huo.data() + b0, 8 * (size_t)(b1 - b0), hipMemcpyHostToDevice, s);
                for (int64_t o = 0; o < b1 - b0; o += PT2_MAXGRID)
                    hipLaunchKernelGGL(k_sel_copy, dim3((unsigned)std::min<int64_t>(PT2_MAXGRID, b1 - b0 - o)), dim3(256),
                                       0, s, (uint32_t)b0, b1 - b0, (const uint32_t *)ucnt, (const uint64_t *)off,
                                       (const uint64_t *)uoff, (const ulonglong2 *)keys, out, (uint64_t)max_out,
                                       (uint32_t)o);
                if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "select: copy failed");
            }
            if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "select: pass launch failed");
            b0 = b1;
        }
        *count = (int64_t)written;
        break;
    }
    return MW_OK;
}

}  // namespace

}  // namespace mw

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);

extern "C" mw_status mw_pt2_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes)
{
    using namespace mw;
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (!bytes) return fail(MW_EINVAL, "NULL bytes");
    if (nroots < 1 || nroots > PT2_MAXR) return fail(MW_EUNSUPPORTED, "pt2: nroots must be in 1..8");
    // one pass without screening: every excitation of every J as a record
    uint64_t first[2];
    if (hipMemcpy(first, d->dets, 16, hipMemcpyDeviceToHost) != hipSuccess) return fail(MW_EHIP, "reading the space failed");
    const bool cplx = d->kind == MW_SPINOR;
    const int na = __builtin_popcountll(first[0]) + (cplx ? __builtin_popcountll(first[1]) : 0);
    const int nbeta = cplx ? 0 : __builtin_popcountll(first[1]);
    ExcClasses ex;
    if (!classes(*d, na, nbeta, ex)) return fail(MW_EUNSUPPORTED, "pt2: more than 2^31 excitations per determinant");
    const uint64_t T = (uint64_t)d->ndet * (uint64_t)ex.start[ex.nclass];
    uint64_t NB = 1;
    while (NB * PT2_MEAN < T) NB <<= 1;
    const size_t sc = cplx ? 16 : 8;
    // the larger of the second-order energy's bucket tables and the
    // selection's, so that the size serves mw_select too
    const size_t tables = std::max(table_bytes((int64_t)NB, nroots), sel_table_bytes((int64_t)1 << sel_lognb(d->ndet)));
    *bytes = fixed_bytes(d->ndet, d->M) + tables + 256 + T * (sizeof(Rec) + sc * nroots);
    return MW_OK;
}

extern "C" mw_status mw_pt2(mw_plan plan, int32_t nroots, const void *c, const double *e0, double qmin,
                            void *work, size_t work_bytes, double *e2, int64_t *stats, mw_stream_t stream)
{
    using namespace mw;
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > PT2_MAXR) return fail(MW_EUNSUPPORTED, "pt2: nroots must be in 1..8");
    if (!c || !e0 || !e2 || !work) return fail(MW_EINVAL, "NULL argument");
    if (!(qmin >= 0.0)) return fail(MW_EINVAL, "qmin must be >= 0");
    if (d->ndet > 0x7fffffffLL) return fail(MW_EUNSUPPORTED, "pt2: at most 2^31 - 1 determinants");
    hipStream_t s = (hipStream_t)stream;
    return d->kind == MW_SPINOR ? pt2_t<true>(*d, nroots, c, e0, qmin, work, work_bytes, e2, stats, s)
                                : pt2_t<false>(*d, nroots, c, e0, qmin, work, work_bytes, e2, stats, s);
}

extern "C" mw_status mw_select(mw_plan plan, int32_t nroots, const void *c, const double *e0, double cmin, void *work,
                               size_t work_bytes, uint64_t *out, int64_t max_out, int64_t *count, mw_stream_t stream)
{
    using namespace mw;
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > PT2_MAXR) return fail(MW_EUNSUPPORTED, "select: nroots must be in 1..8");
    if (!c || !e0 || !work || !count || (max_out > 0 && !out)) return fail(MW_EINVAL, "NULL argument");
    if (!(cmin >= 0.0)) return fail(MW_EINVAL, "cmin must be >= 0");
    if (d->ndet > 0x7fffffffLL) return fail(MW_EUNSUPPORTED, "select: at most 2^31 - 1 determinants");
    hipStream_t s = (hipStream_t)stream;
    return d->kind == MW_SPINOR ? select_t<true>(*d, nroots, c, e0, cmin, work, work_bytes, out, max_out, count, s)
                                : select_t<false>(*d, nroots, c, e0, cmin, work, work_bytes, out, max_out, count, s);
}
