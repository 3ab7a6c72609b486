// Transition one- and two-particle density matrices: the adjoint of sigma
// with respect to the integrals (E = sum h gamma + 1/2 sum g Gamma for the
// Hamiltonian of section 2.1).  The connectivity is recomputed from the same
// groups as sigma, never stored.
//
// Every ordered pair (I, J) connected inside a group contributes
// w_IJ = phi_I phi_J sum_k w_k conj(bra_Ik) ket_Jk:
//  double group, I adds (P<R), J adds (Q<S):  Gamma_PQRS += w, Gamma_RSPQ += w,
//      Gamma_PSRQ -= w, Gamma_RQPS -= w, collected in an accumulator
//      (spin-free alpha-beta: a full [n]^4 array G_ab; same spin and
//      spinor: the antisymmetric pair matrix D[(P,R)][(Q,S)]) that a final
//      pass expands into Gamma.
//  single group, I adds P, J adds Q (K the common N-1 string):
//      gamma_PQ += w and, for every X in K, Gamma_PQXX += w, Gamma_XXPQ += w,
//      Gamma_PXXQ -= w, Gamma_XQPX -= w (spin-free: the exchange-like two
//      only for X of the spin of P).  The sum over K is split into the
//      reference string omega (applied once at the end through the
//      accumulated S_PQ = sum of w) plus the few positions where K and omega
//      differ (compact C and E arrays).
//  diagonal I = J: gamma_PP += w, Gamma_PPRR += w, Gamma_PRRP -= w (P != R),
//      from the occupation correlations of every determinant.
//  One vector as bra and ket: each unordered pair once; the final pass adds
//  the mirror image (the reversed pair's weight is the conjugate).
// The pair accumulators are filled row by row (the row of a pair is the
// partner J's added pair or position): the plan lists every membership
// under its row, a workgroup sums a chunk of a row's list in LDS and adds the
// row to the accumulator once.
#include <hip/hip_runtime.h>
#include <mutex>

#include <algorithm>
#include <type_traits>

#include "dev_common.h"
#include "mw_internal.h"

namespace mw {

// Root weights w_k: host values passed by value, or (dev != nullptr) read
// from device memory, so that an upstream gradient already on the device
// weighs the roots without a copy to the host.
struct RdmWeights {
    double w[64];
    const double *dev;
};

template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T pair_weight(const typename Scal<CPLX>::T *bra,
                                                              const typename Scal<CPLX>::T *ket, int R, uint32_t I,
                                                              uint32_t J, const RdmWeights &W)
{
    using T = typename Scal<CPLX>::T;
    T s = sc_zero(T());
    for (int k = 0; k < R; k++) {
        T t = sc_mul(sc_conj(bra[(size_t)I * R + k]), ket[(size_t)J * R + k]);
        const double wk = W.dev ? W.dev[k] : W.w[k];
        if constexpr (CPLX) s = make_double2(s.x + wk * t.x, s.y + wk * t.y);
        else s += wk * t;
    }
    return s;
}

__device__ __forceinline__ void atom_add(double *a, double v) { atomicAdd(a, v); }

__device__ __forceinline__ int rdm_pair_lex(int lo, int hi, int m) { return lo * (2 * m - lo - 1) / 2 + (hi - lo - 1); }

__device__ __forceinline__ void atom_add(double2 *a, double2 v)
{
    atomicAdd(&a->x, v.x);
    atomicAdd(&a->y, v.y);
}

// output index of Gamma_ABCD (spin-free: spatial orbitals, spin-summed)
__device__ __forceinline__ size_t g4(int m, int a, int b, int c, int d)
{
    return (((size_t)a * m + b) * m + c) * m + d;
}

// Double pairs, accumulated row by row.  The accumulator entry of a pair
// (member i adding (P, R), partner j adding (Q, S)) has its row from j and
// its column from i: alpha-beta D_ab[q][s][p][r] (row q n + s - n, column
// p n + r - n) holds G(p,q,r,s); same-spin and spinor pairs the transposed
// antisymmetric pair matrix, D[(P,R)][(Q,S)] = DT0[QS][PR] (colex pair
// indices; DT1, the lexicographic half used by the final pass, stays zero).
// The plan lists every double membership j under the row of its pair, in
// chunks; a workgroup takes one chunk, adds w_ij of every member i of j's
// group that is connected to j into an LDS copy of the row (LDS atomics:
// the waves share it), then adds the row's nonzero entries to the
// accumulator, one device atomic per entry and chunk instead of one per
// pair.  w_ij = x_i y_j with x_i = phi_i conj(bra_i) gathered per membership
// beforehand (so that a group's members are read contiguously) and y_j =
// phi_j w_k ket_j.
// SYM (bra and ket are one vector): the reversed pair (J, I) adds the
// complex conjugate of w_IJ to the mirrored entry, so each unordered pair is
// visited once (members i before j in the group) and the final pass adds
// the mirror image.

// x[m][k] = phi_m conj(bra[det_m][k]) for every membership m
template <bool CPLX>
__global__ __launch_bounds__(256) void k_rdm_x(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                               typename Scal<CPLX>::T *__restrict__ x)
{
    const int64_t nx = p.nmem * R;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nx; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = t / R;
        const int k = (int)(t - m * R);
        const uint2 me = p.mem[m];
        x[t] = sc_neg(sc_conj(bra[(size_t)me.x * R + k]), ((me.y >> 16) & 1) != 0);
    }
}

__device__ __forceinline__ void lds_add(double *a, double v) { atomicAdd(a, v); }
__device__ __forceinline__ void lds_add(double2 *a, double2 v)
{
    atomicAdd(&a->x, v.x);
    atomicAdd(&a->y, v.y);
}
__device__ __forceinline__ bool sc_nonzero(double v) { return v != 0.0; }
__device__ __forceinline__ bool sc_nonzero(double2 v) { return v.x != 0.0 || v.y != 0.0; }

// How the pair weights are summed.  FX = false: floating-point atomics, in
// the order of arrival.  FX = true: each contribution v becomes the integer
// nearest v sc (sc = 2^s, set per call from a bound on every accumulated
// entry) and is added with 64-bit integer atomics, which are exact and
// associative (in two's complement also where a partial sum wraps), so the
// sums, and the doubles they are converted back to, do not depend on the
// order of arrival.  An accumulator slot of A has the size of the scalar T.
__device__ __forceinline__ unsigned long long fx_of(double v, double sc)
{
    return (unsigned long long)__double2ll_rn(v * sc);
}
template <bool CPLX, bool FX>
struct RdmAcc;
template <bool CPLX>
struct RdmAcc<CPLX, false> {
    using T = typename Scal<CPLX>::T;
    using A = T;
    static __device__ __forceinline__ A zero() { return sc_zero(T()); }
    static __device__ __forceinline__ bool nz(A v) { return sc_nonzero(v); }
    static __device__ __forceinline__ void lds(A *a, T v, double) { lds_add(a, v); }
    static __device__ __forceinline__ void dev(T *a, T v, double) { atom_add(a, v); }
    static __device__ __forceinline__ void flush(T *a, A v) { atom_add(a, v); }
    static __device__ __forceinline__ T value(A v, double) { return v; }
};
template <>
struct RdmAcc<false, true> {
    using A = unsigned long long;
    static __device__ __forceinline__ A zero() { return 0ULL; }
    static __device__ __forceinline__ bool nz(A v) { return v != 0ULL; }
    static __device__ __forceinline__ void lds(A *a, double v, double sc) { atomicAdd(a, fx_of(v, sc)); }
    static __device__ __forceinline__ void dev(double *a, double v, double sc) { atomicAdd((A *)a, fx_of(v, sc)); }
    static __device__ __forceinline__ void flush(double *a, A v) { atomicAdd((A *)a, v); }
    static __device__ __forceinline__ double value(A v, double inv) { return (double)(long long)v * inv; }
};
template <>
struct RdmAcc<true, true> {
    using A = ulonglong2;
    static __device__ __forceinline__ A zero() { return make_ulonglong2(0ULL, 0ULL); }
    static __device__ __forceinline__ bool nz(A v) { return v.x != 0ULL || v.y != 0ULL; }
    static __device__ __forceinline__ void lds(A *a, double2 v, double sc)
    {
        atomicAdd(&a->x, fx_of(v.x, sc));
        atomicAdd(&a->y, fx_of(v.y, sc));
    }
    static __device__ __forceinline__ void dev(double2 *a, double2 v, double sc) { lds((A *)a, v, sc); }
    static __device__ __forceinline__ void flush(double2 *a, A v)
    {
        A *d = (A *)a;
        atomicAdd(&d->x, v.x);
        atomicAdd(&d->y, v.y);
    }
    static __device__ __forceinline__ double2 value(A v, double inv)
    {
        return make_double2((double)(long long)v.x * inv, (double)(long long)v.y * inv);
    }
};
__device__ __forceinline__ double lane_get(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l), hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 lane_get(double2 v, int l) { return make_double2(lane_get(v.x, l), lane_get(v.y, l)); }
__device__ __forceinline__ uint32_t lane_get(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
// the value of lane l (per lane)
__device__ __forceinline__ uint32_t lane_from(uint32_t v, int l) { return (uint32_t)__shfl((int)v, l, 64); }
__device__ __forceinline__ double lane_from(double v, int l) { return __shfl(v, l, 64); }
__device__ __forceinline__ double2 lane_from(double2 v, int l) { return make_double2(__shfl(v.x, l, 64), __shfl(v.y, l, 64)); }
__device__ __forceinline__ uint64_t lane_from(uint64_t v, int l)
{
    return ((uint64_t)lane_from((uint32_t)(v >> 32), l) << 32) | lane_from((uint32_t)v, l);
}

// A wave takes a batch of 64 entries, one per lane with cnt visits; incl is
// the inclusive prefix of cnt over the lanes.  Visit v (0 <= v < incl of
// lane 63) belongs to the entry of the returned lane (binary search over the
// prefix), so that all lanes walk the batch's visits together.
__device__ __forceinline__ int visit_entry(uint32_t incl, uint32_t v)
{
    int t = 0;
#pragma unroll
    for (int b = 32; b >= 1; b >>= 1)
        if (lane_from(incl, t + b - 1) <= v) t += b;
    return t;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// y_j = phi_j sum-weight w_k ket_jk for root k
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T rdm_y(const typename Scal<CPLX>::T *__restrict__ ket, int R, int k,
                                                        uint2 mj, const RdmWeights &W)
{
    using T = typename Scal<CPLX>::T;
    const T v = ket[(size_t)mj.x * R + k];
    const double wk = W.dev ? W.dev[k] : W.w[k];
    T r;
    if constexpr (CPLX) r = make_double2(wk * v.x, wk * v.y);
    else r = wk * v;
    return sc_neg(r, ((mj.y >> 16) & 1) != 0);
}

// y_jk of roots k < RY (zero beyond R) for a partner record mj
template <bool CPLX, int RY>
__device__ __forceinline__ void partner_ys(const typename Scal<CPLX>::T *__restrict__ ket, int R, uint2 mj,
                                           const RdmWeights &W, bool ok, typename Scal<CPLX>::T (&y)[RY])
{
#pragma unroll
    for (int k = 0; k < RY; k++) y[k] = (ok && k < R) ? rdm_y<CPLX>(ket, R, k, mj, W) : sc_zero(typename Scal<CPLX>::T());
}

// w = sum over roots of x_ik y_jk: RM = 1 (one root), 4 (up to four roots,
// the partner's y in registers) or 0 (any count, y_jk read per pair)
template <bool CPLX, int RM, int RY>
__device__ __forceinline__ typename Scal<CPLX>::T pair_w(const typename Scal<CPLX>::T (&xv)[RY],
                                                         const typename Scal<CPLX>::T (&yv)[RY],
                                                         const typename Scal<CPLX>::T *__restrict__ x,
                                                         const typename Scal<CPLX>::T *__restrict__ ket, int R,
                                                         uint32_t i, uint2 mj, const RdmWeights &W)
{
    using T = typename Scal<CPLX>::T;
    if constexpr (RM == 0) {
        T w = sc_zero(T());
        for (int k = 0; k < R; k++) w = sc_add(w, sc_mul(x[(size_t)i * R + k], rdm_y<CPLX>(ket, R, k, mj, W)));
        return w;
    } else {
        T w = sc_mul(xv[0], yv[0]);
#pragma unroll
        for (int k = 1; k < RY; k++) w = sc_add(w, sc_mul(xv[k], yv[k]));
        return w;
    }
}

// the pair (a < b) of positions of a colex pair index r = b (b - 1) / 2 + a
__device__ __forceinline__ void pair_of_index(int r, int &a, int &b)
{
    int hi = (int)((1.0 + sqrt(1.0 + 8.0 * (double)r)) * 0.5);
    while (hi * (hi - 1) / 2 > r) hi--;
    while ((hi + 1) * hi / 2 <= r) hi++;
    b = hi;
    a = r - hi * (hi - 1) / 2;
}

// column of member i's pair in its row
template <bool CPLX>
__device__ __forceinline__ int rdm_col(bool ab, int n, int X, int Y)
{
    if (ab) return X * n + (Y - n);
    if constexpr (CPLX) return pair_idx(X, Y);
    else return X >= n ? pair_idx(X - n, Y - n) : pair_idx(X, Y);
}

// (wide groups: 256 threads per workgroup; the flattened visits of small
// groups, longer-latency chains per batch: 512, more waves per LDS row)
// The row's pair is the partner's: alpha-beta row r = a n + b - n, pair
// row r = b (b - 1) / 2 + a (same-spin positions reduced by n for beta);
// member i of the same group is connected to the partner when their pairs
// share no position.
template <bool CPLX, bool SYM, bool WIDE, int RM, bool FX>
__global__ __launch_bounds__(WIDE ? 256 : 512) void k_rdm_rows(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ ket,
                                                  const typename Scal<CPLX>::T *__restrict__ x, RdmWeights W,
                                                  typename Scal<CPLX>::T *__restrict__ acc, int ncols, int64_t c0,
                                                  const double *__restrict__ fx)
{
    using T = typename Scal<CPLX>::T;
    using AC = RdmAcc<CPLX, FX>;
    using A = typename AC::A;
    constexpr int RY = RM == 4 ? 4 : 1;
    constexpr int UW = 8, US = 4;  // steps of 64 visits in flight per wave (wide, small)
    extern __shared__ __align__(16) double rdm_lds_raw[];
    A *row = (A *)rdm_lds_raw;
    const double sc = FX ? fx[0] : 0.0;
    const uint4 ch = p.rdm_chunk[c0 + blockIdx.x];
    const bool ab = (ch.y & 1) != 0;
    const int n = p.n;
    int pa, pb;
    if (ab) {
        pa = (int)ch.x / n;
        pb = n + (int)ch.x % n;
    } else {
        pair_of_index((int)ch.x, pa, pb);
    }
    // member positions in the row's space, and the connection test
    auto reduce = [&](uint32_t pos, int &xi, int &yi) {
        xi = pos & 255;
        yi = (pos >> 8) & 255;
        if (!CPLX && !ab && xi >= n) {
            xi -= n;
            yi -= n;
        }
    };
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) row[t] = AC::zero();
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t stride = blockDim.x;  // 64 entries per wave
    if constexpr (WIDE) {
        // groups of RDM_WIDE members or more: a wave loads the records of 64
        // entries (a lane each), then walks their members in steps of 64
        // (a member per lane), UW steps in flight
        for (uint32_t base = ch.z + 64u * wv; base < ch.w; base += stride) {
            const uint32_t e = base + lane;
            const bool ok = e < ch.w;
            const uint2 en = ok ? p.rdm_ent[e] : make_uint2(0u, 0u);
            const uint32_t j0 = en.x, L = en.y >> 16;
            const uint32_t dj = ok ? p.rdm_ent_det[e] : 0u;
            T y[RY];
            partner_ys<CPLX, RY>(ket, R, make_uint2(dj & 0x7fffffffu, (dj >> 31) << 16), W, ok, y);
            const uint32_t cnt = ok ? (SYM ? (en.y & 0xffffu) : L) : 0u;  // members visited: [j0, j0 + cnt)
            const uint32_t nb = (cnt + 63) / 64;
            // inclusive prefix of the step counts over the lanes
            const uint32_t incl = wave_incl_scan(nb, lane);
            const uint32_t total = lane_get(incl, 63);
            for (uint32_t s0 = 0; s0 < total; s0 += UW) {
                uint32_t pi[UW], ii[UW], djs[UW];
                T xv[UW][RY], yv[UW][RY];
                bool act[UW];
#pragma unroll
                for (int u = 0; u < UW; u++) {
                    const uint32_t st = s0 + u;
                    // the entry of step st: the lanes whose inclusive prefix
                    // is <= st come before it
                    const int t0 = (int)__popcll(__ballot(incl <= st));
                    const int t = t0 < 64 ? t0 : 63;
                    const uint32_t off = (st - (lane_get(incl, t) - lane_get(nb, t))) * 64 + lane;
                    act[u] = st < total && off < lane_get(cnt, t);
                    ii[u] = lane_get(j0, t) + off;
                    djs[u] = lane_get(dj, t);
#pragma unroll
                    for (int k = 0; k < RY; k++) {
                        yv[u][k] = lane_get(y[k], t);
                        xv[u][k] = act[u] && k < R ? x[(size_t)ii[u] * R + k] : sc_zero(T());
                    }
                    pi[u] = act[u] ? (uint32_t)p.rdm_pos[ii[u]] : 0u;
                }
#pragma unroll
                for (int u = 0; u < UW; u++) {
                    int xi, yi;
                    reduce(pi[u], xi, yi);
                    if (!act[u] || xi == pa || xi == pb || yi == pa || yi == pb) continue;
                    const T w = pair_w<CPLX, RM, RY>(xv[u], yv[u], x, ket, R, ii[u],
                                                      make_uint2(djs[u] & 0x7fffffffu, (djs[u] >> 31) << 16), W);
                    AC::lds(&row[rdm_col<CPLX>(ab, n, pi[u] & 255, (pi[u] >> 8) & 255)], w, sc);
                }
            }
        }
    } else {
        // smaller groups: the visits of 64 entries (a lane each) are walked
        // by the lanes together, 64 at a time, US steps in flight
        for (uint32_t base = ch.z + 64u * wv; base < ch.w; base += stride) {
            const uint32_t e = base + lane;
            const bool ok = e < ch.w;
            const uint2 en = ok ? p.rdm_ent[e] : make_uint2(0u, 0u);
            const uint32_t j0 = en.x, jo = en.y & 0xffffu, L = en.y >> 16;
            const uint32_t dj = ok && !(SYM && RM == 1) ? p.rdm_ent_det[e] : 0u;
            const uint32_t cnt = ok ? (SYM ? jo : L) : 0u;
            T y[RY];
            if (SYM && RM == 1) {
                // one vector, one root: y_j = w_0 conj(x_j), read from the
                // lines of the members it pairs with (no determinant gather);
                // entries without visits read nothing
                const double w0 = W.dev ? W.dev[0] : W.w[0];
                const T xj = cnt ? sc_conj(x[j0 + jo]) : sc_zero(T());
                if constexpr (CPLX) y[0] = make_double2(w0 * xj.x, w0 * xj.y);
                else y[0] = w0 * xj;
            } else {
                partner_ys<CPLX, RY>(ket, R, make_uint2(dj & 0x7fffffffu, (dj >> 31) << 16), W, ok, y);
            }
            const uint32_t incl = wave_incl_scan(cnt, lane);
            const uint32_t total = lane_get(incl, 63);
            for (uint32_t v0 = 0; v0 < total; v0 += 64u * US) {
                uint32_t pi[US], ii[US], djs[US];
                T xv[US][RY], yv[US][RY];
                bool act[US];
#pragma unroll
                for (int u = 0; u < US; u++) {
                    const uint32_t v = v0 + 64u * u + lane;
                    act[u] = v < total;
                    const int t = visit_entry(incl, v);
                    ii[u] = lane_from(j0, t) + (v - (lane_from(incl, t) - lane_from(cnt, t)));
                    djs[u] = lane_from(dj, t);
#pragma unroll
                    for (int k = 0; k < RY; k++) {
                        yv[u][k] = lane_from(y[k], t);
                        xv[u][k] = act[u] && k < R ? x[(size_t)ii[u] * R + k] : sc_zero(T());
                    }
                    pi[u] = act[u] ? (uint32_t)p.rdm_pos[ii[u]] : 0u;
                }
#pragma unroll
                for (int u = 0; u < US; u++) {
                    int xi, yi;
                    reduce(pi[u], xi, yi);
                    if (!act[u] || xi == pa || xi == pb || yi == pa || yi == pb) continue;
                    const T w = pair_w<CPLX, RM, RY>(xv[u], yv[u], x, ket, R, ii[u],
                                                      make_uint2(djs[u] & 0x7fffffffu, (djs[u] >> 31) << 16), W);
                    AC::lds(&row[rdm_col<CPLX>(ab, n, pi[u] & 255, (pi[u] >> 8) & 255)], w, sc);
                }
            }
        }
    }
    __syncthreads();
    T *dst = acc + (size_t)ch.x * ncols;
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) {
        const A v = row[t];
        if (AC::nz(v)) AC::flush(&dst[t], v);
    }
}

// The contributions of one single pair (member i with det me.x adding
// position Xi, partner with record o adding Xj; K the group's string).
template <bool CPLX, bool FX>
__device__ __forceinline__ void rdm_single_pair(const DevPlan &p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                const typename Scal<CPLX>::T *__restrict__ ket, const RdmWeights &W,
                                                typename Scal<CPLX>::T *__restrict__ S,
                                                typename Scal<CPLX>::T *__restrict__ Cc, double *__restrict__ Ee,
                                                uint8_t type, uint64_t k0, uint64_t k1, uint2 me, int Xi, uint32_t negi,
                                                uint2 o, double sc)
{
    using T = typename Scal<CPLX>::T;
    using AC = RdmAcc<CPLX, FX>;
    const int n = p.n;
    const int Xj = o.y & 255;
    T w = pair_weight<CPLX>(bra, ket, R, me.x, o.x, W);
    w = sc_neg(w, (negi ^ ((o.y >> 16) & 1)) != 0);
    if constexpr (!CPLX) {
        const int s = type == G_SINGLE_A ? 0 : 1;
        const int pp = Xi - s * n, qq = Xj - s * n;
        // the member's orbital p (varying across the lanes of a large
        // group, whose partner q is uniform) is the innermost index of
        // every single accumulator, so the lanes' atomics coalesce
        AC::dev(&S[((size_t)s * n + qq) * n + pp], w, sc);
        // positions where K and omega differ: words (same spin, other
        // spin); C[q][x][p] collects the Coulomb-like terms of every X,
        // E[q][x][p] the exchange-like ones of X of the same spin (both
        // n^3, L2-resident; expanded into Gamma by the final pass)
        double *Cq = Cc + (size_t)qq * n * n + pp, *Eq = Ee + (size_t)qq * n * n + pp;
        for (int part = 0; part < 4; part++) {
            const bool same = part < 2;
            const uint64_t kw = (same == (s == 0)) ? k0 : k1;
            const uint64_t rw = (same == (s == 0)) ? p.ref0 : p.ref1;
            const uint64_t bits = (part & 1) ? (rw & ~kw) : (kw & ~rw);
            const double sw = (part & 1) ? -w : w;
            for (uint64_t x = bits; x; x &= x - 1) {
                const int xx = __builtin_ctzll(x);
                AC::dev(&Cq[(size_t)xx * n], sw, sc);
                if (same) AC::dev(&Eq[(size_t)xx * n], sw, sc);
            }
        }
    } else {
        const int M = p.M;
        AC::dev(&S[(size_t)Xj * M + Xi], w, sc);
        // C[Q][X][P] (M^3, P innermost) collects the four terms of every X
        T *Cq = Cc + (size_t)Xj * M * M + Xi;
        for (int part = 0; part < 4; part++) {
            const uint64_t kw = (part < 2) ? k0 : k1;
            const uint64_t rw = (part < 2) ? p.ref0 : p.ref1;
            const int base = (part < 2) ? 0 : n;
            const uint64_t bits = (part & 1) ? (rw & ~kw) : (kw & ~rw);
            const T sw = sc_neg(w, (part & 1) != 0);
            for (uint64_t x = bits; x; x &= x - 1) AC::dev(&Cq[(size_t)(base + __builtin_ctzll(x)) * M], sw, sc);
        }
    }
}

template <bool CPLX, bool SYM, bool FX>
__global__ __launch_bounds__(256) void k_rdm_single(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                    const typename Scal<CPLX>::T *__restrict__ ket, RdmWeights W,
                                                    typename Scal<CPLX>::T *__restrict__ S,
                                                    typename Scal<CPLX>::T *__restrict__ Cc,
                                                    double *__restrict__ Ee, int64_t copy_stride,
                                                    const double *__restrict__ fx)
{
    const double sc = FX ? fx[0] : 0.0;
    const int64_t wave = p.npacket_double + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= p.npacket) return;
    // the few S, C, E entries take many additions: spread them over
    // RDM_COPIES copies (folded before the final pass) by block
    {
        const int64_t o = (int64_t)(blockIdx.x % RDM_COPIES) * copy_stride;
        S += o;
        Cc += o;
        if (Ee) Ee += o;
    }
    const uint32_t mfirst = p.pk_off[wave], mend = p.pk_off[wave + 1];
    const uint32_t m = mfirst + lane;
    if (((p.mem[mfirst].y >> 24) & 63) == 0) {
        // a 64-member block of a large group: every lane visits the same
        // partner in the same step (SYM: partners after the lane's member
        // masked), so the lanes' atomics into S, C, E, whose innermost index
        // is the member's position, coalesce into few requests
        const uint32_t g = p.mem_grp[mfirst];
        const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
        const uint8_t type = p.grp_type[g];
        const uint64_t k0 = p.grp_key[2 * g], k1 = p.grp_key[2 * g + 1];
        const bool act = m < mend;
        const uint2 me = p.mem[act ? m : mfirst];
        const int Xi = me.y & 255;
        const uint32_t negi = (me.y >> 16) & 1;
        for (uint32_t j = SYM ? mfirst + 1 : j0; j < j1; j++) {
            const uint2 o = p.mem[j];
            if (!act || (o.y & 255) == (uint32_t)Xi || (SYM && j <= m)) continue;
            rdm_single_pair<CPLX, FX>(p, R, bra, ket, W, S, Cc, Ee, type, k0, k1, me, Xi, negi, o, sc);
        }
        return;
    }
    if (m >= mend) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255;
    const uint32_t negi = (me.y >> 16) & 1;
    const uint64_t k0 = p.grp_key[2 * g], k1 = p.grp_key[2 * g + 1];
    // SYM: partners after i only; k_rdm_mirror adds the reversed pairs
    for (uint32_t j = SYM ? max(j0, m + 1) : j0; j < j1; j++) {
        const uint2 o = p.mem[j];
        if ((int)(o.y & 255) == Xi) continue;
        rdm_single_pair<CPLX, FX>(p, R, bra, ket, W, S, Cc, Ee, type, k0, k1, me, Xi, negi, o, sc);
    }
}

// Single pairs, accumulated row by row like the double pairs.  The row is
// the partner j's added orbital q (spin-free, either spin) or spinor Q; a
// workgroup holds in LDS the row's S entries (S[s][q][p] for both spins;
// spinor S[Q][P]) and its C and E blocks (C[q][x][p], E[q][x][p]; spinor
// C[Q][X][P]), walks the visits of its chunk's entries with all lanes (64
// entries per wave batch, four steps in flight), and adds the nonzero
// entries to copy 0 of the accumulators.  Per pair the same terms as
// rdm_single_pair: S, then the positions where the group's string K and
// the reference omega differ.
template <bool CPLX, bool SYM, int RM, bool FX>
__global__ __launch_bounds__(256) void k_rdm_single_rows(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ ket,
                                                         const typename Scal<CPLX>::T *__restrict__ x, RdmWeights W,
                                                         typename Scal<CPLX>::T *__restrict__ S,
                                                         typename Scal<CPLX>::T *__restrict__ Cc,
                                                         double *__restrict__ Ee, int64_t c0,
                                                         const double *__restrict__ fx)
{
    using T = typename Scal<CPLX>::T;
    using AC = RdmAcc<CPLX, FX>;
    using AR = RdmAcc<false, FX>;  // the real E block (spin-free)
    using A = typename AC::A;
    constexpr int RY = RM == 4 ? 4 : 1;
    extern __shared__ __align__(16) double rdm_lds_raw[];
    const double sc = FX ? fx[0] : 0.0;
    const int n = p.n, M = p.M;
    const int nS = CPLX ? M : 2 * n, nC = CPLX ? M * M : n * n;
    const int ncols = CPLX ? nS + nC : nS + 2 * nC;
    A *lS = (A *)rdm_lds_raw, *lC = lS + nS;
    typename AR::A *lE = CPLX ? nullptr : (typename AR::A *)(lS + nS + nC);
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) lS[t] = AC::zero();
    __syncthreads();
    const uint4 ch = p.rdm_chunk[c0 + blockIdx.x];
    const int q = (int)ch.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (uint32_t base = ch.z + 64u * wv; base < ch.w; base += 256u) {
        const uint32_t e = base + lane;
        const bool ok = e < ch.w;
        const uint2 en = ok ? p.rdm_ent[e] : make_uint2(0u, 0u);
        const uint32_t j0 = en.x, jo = en.y & 0x7fffu, L = en.y >> 16;
        const uint32_t sb = (en.y >> 15) & 1u;
        const uint32_t cnt = ok ? (SYM ? jo : L) : 0u;
        // the entry carries the group's string, the spin and the partner's
        // determinant; the partner's position is the row's
        const ulonglong2 kk = ok ? p.rdm_skey[e - p.rdm_single_e0] : make_ulonglong2(0ULL, 0ULL);
        const uint64_t k0 = kk.x, k1 = kk.y;
        const uint32_t dj = ok && !(SYM && RM == 1) ? p.rdm_ent_det[e] : 0u;
        const uint2 mj = make_uint2(dj & 0x7fffffffu, ((dj >> 31) << 16) | (uint32_t)(q + (CPLX ? 0 : (int)sb * n)));
        T y[RY];
        if (SYM && RM == 1) {
            // one vector, one root: y_j = w_0 conj(x_j) from the lines of the
            // members it pairs with
            const double w0 = W.dev ? W.dev[0] : W.w[0];
            const T xj = cnt ? sc_conj(x[j0 + jo]) : sc_zero(T());
            if constexpr (CPLX) y[0] = make_double2(w0 * xj.x, w0 * xj.y);
            else y[0] = w0 * xj;
        } else {
            partner_ys<CPLX, RY>(ket, R, mj, W, ok, y);
        }
        const uint32_t incl = wave_incl_scan(cnt, lane);
        const uint32_t total = lane_get(incl, 63);
        for (uint32_t v0 = 0; v0 < total; v0 += 256u) {
            uint32_t pi[4], pj[4], ii[4], dj[4], sp[4];
            uint64_t kk0[4], kk1[4];
            T xv[4][RY], yv[4][RY];
            bool act[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t v = v0 + 64u * u + lane;
                act[u] = v < total;
                const int t = visit_entry(incl, v);
                ii[u] = lane_from(j0, t) + (v - (lane_from(incl, t) - lane_from(cnt, t)));
                pj[u] = lane_from(mj.y, t);
                dj[u] = lane_from(mj.x, t);
                sp[u] = lane_from(sb, t);
                kk0[u] = lane_from(k0, t);
                kk1[u] = lane_from(k1, t);
#pragma unroll
                for (int k = 0; k < RY; k++) {
                    yv[u][k] = lane_from(y[k], t);
                    xv[u][k] = act[u] && k < R ? x[(size_t)ii[u] * R + k] : sc_zero(T());
                }
                pi[u] = act[u] ? (uint32_t)p.rdm_pos[ii[u]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int Xi = pi[u] & 255, Xj = pj[u] & 255;
                if (!act[u] || Xi == Xj) continue;
                const T w = pair_w<CPLX, RM, RY>(xv[u], yv[u], x, ket, R, ii[u], make_uint2(dj[u], pj[u]), W);
                if constexpr (!CPLX) {
                    const int s = (int)sp[u], pp = Xi - s * n;
                    AC::lds(&lS[s * n + pp], w, sc);
                    for (int part = 0; part < 4; part++) {
                        const bool same = part < 2;
                        const uint64_t kw = (same == (s == 0)) ? kk0[u] : kk1[u];
                        const uint64_t rw = (same == (s == 0)) ? p.ref0 : p.ref1;
                        const uint64_t bits = (part & 1) ? (rw & ~kw) : (kw & ~rw);
                        const double sw = (part & 1) ? -w : w;
                        for (uint64_t b = bits; b; b &= b - 1) {
                            const int xx = __builtin_ctzll(b);
                            AC::lds(&lC[xx * n + pp], sw, sc);
                            if (same) AR::lds(&lE[xx * n + pp], sw, sc);
                        }
                    }
                } else {
                    AC::lds(&lS[Xi], w, sc);
                    for (int part = 0; part < 4; part++) {
                        const uint64_t kw = (part < 2) ? kk0[u] : kk1[u];
                        const uint64_t rw = (part < 2) ? p.ref0 : p.ref1;
                        const int bpos = (part < 2) ? 0 : n;
                        const uint64_t bits = (part & 1) ? (rw & ~kw) : (kw & ~rw);
                        const T sw = sc_neg(w, (part & 1) != 0);
                        for (uint64_t b = bits; b; b &= b - 1) AC::lds(&lC[(bpos + __builtin_ctzll(b)) * M + Xi], sw, sc);
                    }
                }
            }
        }
    }
    __syncthreads();
    // S: spin-free S[s][q][p] (lS[s n + p]); spinor S[Q][P]; C (and E) rows
    // of q: C + q nC
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) {
        const A v = lS[t];
        if (!AC::nz(v)) continue;
        if (t < nS) {
            if constexpr (CPLX) AC::flush(&S[(size_t)q * M + t], v);
            else AC::flush(&S[((size_t)(t / n) * n + q) * n + (t % n)], v);
        } else if (t < nS + nC) {
            AC::flush(&Cc[(size_t)q * nC + (t - nS)], v);
        } else {
            if constexpr (!CPLX) AC::flush(&Ee[(size_t)q * nC + (t - nS - nC)], v);
        }
    }
}

// Diagonal terms: with w_I = sum_k w_k conj(bra_Ik) ket_Ik, the occupation
// correlation D[A][B] = sum_I w_I n_A(I) n_B(I) over global positions gives
// gamma_AA = D[A][A] and the diagonal parts of Gamma (Gamma_AABB += D[A][B],
// Gamma_ABBA -= D[A][B] for A != B; spin-free: summed over spins, the
// exchange-like part for equal spins only).  One partial matrix per
// determinant chunk, reduced in a fixed order.
constexpr int RDM_OCC_CHUNKS = 256;

// position of the k-th (from 0) set bit of w, k < popcount(w): the largest
// p with at most k set bits below it (binary lifting over the bit index)
__device__ __forceinline__ int nth_bit(uint64_t w, int k)
{
    int pos = 0;
#pragma unroll
    for (int step = 32; step; step >>= 1)
        if (__popcll(w & ((1ULL << (pos + step)) - 1)) <= k) pos += step;
    return pos;
}

// Block (x, y) of 1024 threads adds w_I into an LDS copy of rows
// [A0, A0 + ROWS) of D for every determinant of chunk x, a wave per
// determinant over its pairs of occupied positions (LDS atomics: the 16
// waves take different determinants); then it writes its rows of the
// chunk's partial matrix (FX: the exact fixed-point sums, converted).
template <bool CPLX, bool FX>
__global__ __launch_bounds__(1024) void k_rdm_occ_lds(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                      const typename Scal<CPLX>::T *__restrict__ ket, RdmWeights W,
                                                      typename Scal<CPLX>::T *__restrict__ part,
                                                      const double *__restrict__ fx)
{
    using T = typename Scal<CPLX>::T;
    using AC = RdmAcc<CPLX, FX>;
    using AT = typename AC::A;
    constexpr int ROWS = CPLX ? 64 : 128;
    constexpr int MP = 129;  // LDS row stride: rows of one column fall in different banks (132 KB)
    __shared__ AT ds[ROWS * MP];
    const double sc = FX ? fx[0] : 0.0, inv = FX ? fx[1] : 0.0;
    const int n = p.n, M = p.M;
    const int A0 = (int)blockIdx.y * ROWS, A1 = min(M, A0 + ROWS);
    const int rows = A1 - A0;
    for (int t = threadIdx.x; t < rows * MP; t += blockDim.x) ds[t] = AC::zero();
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t chunk = (p.ndet + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(p.ndet, lo + chunk);
    // occupied global positions of the row range, as two masks over the words
    auto rowmask = [&](uint64_t d0, uint64_t d1, uint64_t &m0, uint64_t &m1) {
        // word 0 holds positions [0, n), word 1 positions [n, 2n)
        auto range = [](int a, int b) -> uint64_t {  // bits [a, b) of a word, 0 <= a <= b <= 64
            if (a >= b) return 0ULL;
            const uint64_t hi_ = b >= 64 ? ~0ULL : ((1ULL << b) - 1);
            return hi_ & ~((1ULL << a) - 1);
        };
        m0 = d0 & range(min(A0, n), min(A1, n));
        m1 = d1 & range(max(A0 - n, 0), max(min(A1 - n, 64), 0));
    };
    // a wave takes 64 consecutive determinants at a time: each lane loads
    // one determinant and its weight, then the wave walks them one by one
    // (one memory round trip per 64 determinants)
    for (int64_t Ib = lo + 64 * (int64_t)wv; Ib < hi; Ib += 64 * (int64_t)nw) {
      const int64_t Il = Ib + lane;
      const bool okl = Il < hi;
      const uint64_t dl0 = okl ? p.dets[2 * Il] : 0ULL, dl1 = okl ? p.dets[2 * Il + 1] : 0ULL;
      const T wl = okl ? pair_weight<CPLX>(bra, ket, R, (uint32_t)Il, (uint32_t)Il, W) : sc_zero(T());
      const int cnt = (int)min<int64_t>(64, hi - Ib);
      for (int tdet = 0; tdet < cnt; tdet++) {
        const uint64_t d0 = ((uint64_t)lane_get((uint32_t)(dl0 >> 32), tdet) << 32) | lane_get((uint32_t)dl0, tdet);
        const uint64_t d1 = ((uint64_t)lane_get((uint32_t)(dl1 >> 32), tdet) << 32) | lane_get((uint32_t)dl1, tdet);
        const T w = lane_get(wl, tdet);
        const int c0 = __popcll(d0), nocc = c0 + __popcll(d1);
        if (nocc <= 64) {
            // lane l holds the l-th occupied global position; the wave then
            // adds w at every (A, B) pair of occupied positions, 64 pairs per
            // instruction (instead of one instruction per A over all B)
            int pos = 0;
            if (lane < c0) pos = nth_bit(d0, lane);
            else if (lane < nocc) pos = n + nth_bit(d1, lane - c0);
            const int np2 = nocc * nocc;
            for (int k0 = 0; k0 < np2; k0 += 64) {
                const int k = k0 + lane;
                const int a = k < np2 ? k / nocc : 0, b = k < np2 ? k - a * nocc : 0;
                const int A = __shfl(pos, a, 64), B = __shfl(pos, b, 64);
                if (k < np2 && A >= A0 && A < A1) AC::lds(ds + (size_t)(A - A0) * MP + B, w, sc);
            }
            continue;
        }
        const int B0 = lane, B1 = lane + 64;
        const bool o0 = B0 < M && (B0 < n ? (d0 >> B0) & 1 : (d1 >> (B0 - n)) & 1);
        const bool o1 = B1 < M && (B1 < n ? (d0 >> B1) & 1 : (d1 >> (B1 - n)) & 1);
        uint64_t m0, m1;
        rowmask(d0, d1, m0, m1);
        for (int word = 0; word < 2; word++) {
            for (uint64_t x = word ? m1 : m0; x; x &= x - 1) {
                const int A = __builtin_ctzll(x) + (word ? n : 0);
                AT *row = ds + (size_t)(A - A0) * MP;
                if (o0) AC::lds(row + B0, w, sc);
                if (o1) AC::lds(row + B1, w, sc);
            }
        }
      }
    }
    __syncthreads();
    T *out = part + (size_t)blockIdx.x * M * M + (size_t)A0 * M;
    for (int t = threadIdx.x; t < rows * M; t += blockDim.x) out[t] = AC::value(ds[(t / M) * MP + t % M], inv);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rdm_occ_reduce(int M, int nchunk, const T *__restrict__ part, T *__restrict__ D)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    T s = sc_zero(T());
    for (int c = 0; c < nchunk; c++) s = sc_add(s, part[(size_t)c * M * M + t]);
    D[t] = s;
}

// D[(P,R)][(Q,S)] (P<R added in the bra determinant, Q<S in the ket one)
// from the transposed accumulators
template <typename T>
__device__ __forceinline__ T d_pair(const T *dt0, const T *dt1, int np, int m, int p, int r, int q, int s)
{
    const size_t row = (size_t)pair_idx(q, s) * np;
    return sc_add(dt0[row + pair_idx(p, r)], dt1[row + rdm_pair_lex(p, r, m)]);
}

// D-term of Gamma_abcd: the one tuple of the expansion that lands on (a,b,c,d)
template <typename T>
__device__ __forceinline__ T d_term(const T *dt0, const T *dt1, int np, int m, int a, int b, int c, int d)
{
    if (a == c || b == d) return sc_zero(T());
    if (a < c) {
        if (b < d) return d_pair(dt0, dt1, np, m, a, c, b, d);
        return sc_neg(d_pair(dt0, dt1, np, m, a, c, d, b), true);
    }
    if (d < b) return d_pair(dt0, dt1, np, m, c, a, d, b);
    return sc_neg(d_pair(dt0, dt1, np, m, c, a, b, d), true);
}

// X[t] = sum of the copies X[c * stride + t], c = 0 .. copies-1, in order
template <class T>
__global__ __launch_bounds__(256) void k_rdm_fold(T *X, int64_t stride, int copies)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= stride) return;
    T v = X[t];
    for (int c = 1; c < copies; c++) v = sc_add(v, X[c * stride + t]);
    X[t] = v;
}

// SYM pass for the single-excitation accumulators: X[P][Q][x] and
// X[Q][P][x] (P < Q; x over `inner` entries) both become their sum with the
// other's conjugate.  `outer` blocks of the matrix (spin-free: the two spin
// blocks of S) are independent.
template <class T>
__global__ __launch_bounds__(256) void k_rdm_mirror(T *X, int m, int inner, int outer)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)m * m * inner;
    if (t >= per * outer) return;
    const int64_t o = t / per, r = t % per;
    const int x = (int)(r % inner);
    const int P = (int)(r / inner / m), Q = (int)(r / inner % m);
    if (P >= Q) return;
    T *a = X + o * per + ((int64_t)P * m + Q) * inner + x;
    T *b = X + o * per + ((int64_t)Q * m + P) * inner + x;
    const T va = *a, vb = *b;
    *a = sc_add(va, sc_conj(vb));
    *b = sc_add(vb, sc_conj(va));
}

// SYM pass for X[Q][x][P] (P innermost, x over m entries): X[Q][x][P] and
// X[P][x][Q] (P < Q) both become their sum with the other's conjugate; the
// `outer` blocks are independent.
template <class T>
__global__ __launch_bounds__(256) void k_rdm_mirror_qxp(T *X, int m, int outer)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)m * m * m;
    if (t >= per * outer) return;
    const int64_t o = t / per, r = t % per;
    const int Q = (int)(r / ((int64_t)m * m)), x = (int)(r / m % m), P = (int)(r % m);
    if (P >= Q) return;
    T *a = X + o * per + ((int64_t)Q * m + x) * m + P;
    T *b = X + o * per + ((int64_t)P * m + x) * m + Q;
    const T va = *a, vb = *b;
    *a = sc_add(va, sc_conj(vb));
    *b = sc_add(vb, sc_conj(va));
}

__global__ __launch_bounds__(256) void k_rdm_finalize_sf(DevPlan p, const double *__restrict__ dab,
                                                         const double *__restrict__ dt0,
                                                         const double *__restrict__ dt1, const double *__restrict__ S,
                                                         const double *__restrict__ Cc, const double *__restrict__ Ee,
                                                         const double *__restrict__ D, double *__restrict__ gam,
                                                         double *__restrict__ Gam, int sym, double fac_g)
{
    const int n = p.n, M = p.M;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = (int64_t)n * n * n * n;
    if (t >= n4) return;
    const int dd = t % n, c = (t / n) % n, b = (t / n / n) % n, a = (int)(t / n / n / n);
    // G(p,q,r,s) lives at dab[q][s][p][r]; with sym the double pairs were
    // visited once and the reversed ones add the entry (q,p,s,r)
    double v = dab[g4(n, b, dd, a, c)] + dab[g4(n, dd, b, c, a)] + d_term(dt0, dt1, p.npair, n, a, b, c, dd);
    if (sym) v += dab[g4(n, a, c, b, dd)] + dab[g4(n, c, a, dd, b)] + d_term(dt0, dt1, p.npair, n, b, a, dd, c);
    // S[s][q][p], C[q][x][p], E[q][x][p] (p innermost)
    const double *S0 = S, *S1 = S + (size_t)n * n;
    auto occ = [&](uint64_t w, int x) { return (double)((w >> x) & 1); };
    auto sg = [&](const double *X, int pp, int qq) { return X[(size_t)qq * n + pp]; };
    auto cpq = [&](const double *X, int pp, int qq, int xx) { return X[((size_t)qq * n + xx) * n + pp]; };
    // single excitations: reference string omega (through S) + corrections
    if (c == dd) v += (sg(S0, a, b) + sg(S1, a, b)) * (occ(p.ref0, c) + occ(p.ref1, c)) + cpq(Cc, a, b, c);
    if (a == b) v += (sg(S0, c, dd) + sg(S1, c, dd)) * (occ(p.ref0, a) + occ(p.ref1, a)) + cpq(Cc, c, dd, a);
    if (b == c) v -= sg(S0, a, dd) * occ(p.ref0, b) + sg(S1, a, dd) * occ(p.ref1, b) + cpq(Ee, a, dd, b);
    if (a == dd) v -= sg(S0, c, b) * occ(p.ref0, a) + sg(S1, c, b) * occ(p.ref1, a) + cpq(Ee, c, b, a);
    // diagonal terms from the occupation correlations D over 2n positions
    auto Dg = [&](int A, int B) { return D[(size_t)A * M + B]; };
    if (a == b && c == dd) {
        double s = Dg(a, n + c) + Dg(n + a, c);
        if (a != c) s += Dg(a, c) + Dg(n + a, n + c);
        v += s;
    }
    if (a == dd && b == c && a != b) v -= Dg(a, b) + Dg(n + a, n + b);
    Gam[t] = fac_g * v;
    if (t < (int64_t)n * n) {
        const int pa = (int)(t / n), qa = (int)(t % n);
        gam[t] = sg(S0, pa, qa) + sg(S1, pa, qa) + (pa == qa ? Dg(pa, pa) + Dg(n + pa, n + pa) : 0.0);
    }
}

__global__ __launch_bounds__(256) void k_rdm_finalize_spinor(DevPlan p, const double2 *__restrict__ dt0,
                                                             const double2 *__restrict__ dt1,
                                                             const double2 *__restrict__ S,
                                                             const double2 *__restrict__ Cc,
                                                             const double2 *__restrict__ D,
                                                             double2 *__restrict__ gam, double2 *__restrict__ Gam,
                                                             int sym, double fac_g, int conj)
{
    const int M = p.M, n = p.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m4 = (int64_t)M * M * M * M;
    if (t >= m4) return;
    const int dd = t % M, c = (t / M) % M, b = (t / M / M) % M, a = (int)(t / M / M / M);
    double2 v = d_term(dt0, dt1, p.npair, M, a, b, c, dd);
    if (sym) v = sc_add(v, sc_conj(d_term(dt0, dt1, p.npair, M, b, a, dd, c)));
    auto inref = [&](int X) { return X < n ? ((p.ref0 >> X) & 1) : ((p.ref1 >> (X - n)) & 1); };
    // S[Q][P], C[Q][X][P] (P innermost)
    auto cpq = [&](int P, int Q, int X) { return Cc[((size_t)Q * M + X) * M + P]; };
    auto sg = [&](int P, int Q) { return S[(size_t)Q * M + P]; };
    if (c == dd) v = sc_add(v, sc_add(inref(c) ? sg(a, b) : sc_zero(double2()), cpq(a, b, c)));
    if (a == b) v = sc_add(v, sc_add(inref(a) ? sg(c, dd) : sc_zero(double2()), cpq(c, dd, a)));
    if (b == c) v = sc_add(v, sc_neg(sc_add(inref(b) ? sg(a, dd) : sc_zero(double2()), cpq(a, dd, b)), true));
    if (a == dd) v = sc_add(v, sc_neg(sc_add(inref(a) ? sg(c, b) : sc_zero(double2()), cpq(c, b, a)), true));
    if (a == b && c == dd && a != c) v = sc_add(v, D[(size_t)a * M + c]);
    if (a == dd && b == c && a != b) v = sc_add(v, sc_neg(D[(size_t)a * M + b], true));
    if (conj) v = sc_conj(v);
    Gam[t] = make_double2(fac_g * v.x, fac_g * v.y);
    if (t < (int64_t)M * M) {
        const int A = (int)(t / M), B = (int)(t % M);
        const double2 gv = sc_add(sg(A, B), A == B ? D[t] : sc_zero(double2()));
        gam[t] = conj ? sc_conj(gv) : gv;
    }
}

__global__ void k_zero(double *x, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = 0.0;
}

static void zero(double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
}

// Fixed-point scale sc = 2^s.  Every accumulated entry is a sum over a
// subset of the connected pairs of one operator index of w_IJ = sum_k w_k
// conj(bra_Ik) ket_Jk, and that operator takes each determinant to at most
// one other, so by Cauchy-Schwarz |entry| <= B = max_k |w_k| ||bra||_F
// ||ket||_F; with B in [2^(e-1), 2^e), s = 60 - e keeps |entry sc| < 2^60.
// The norms are kept as (m, q): the largest magnitude m and the sum q of
// (x / m)^2, so that ||x||^2 = m^2 q neither overflows nor underflows (the
// scaled sum of square of two-norm routines), over a fixed partition (a
// grid-stride loop of RDM_FX_BLOCKS blocks, a tree in LDS) combined in
// block order by one block, so the scale is the same on every call, and
// scaling bra or ket by 2^k shifts s by exactly k.
__device__ __forceinline__ void norm_add(double &m, double &q, double x)
{
    x = fabs(x);
    if (x == 0.0) return;
    if (x > m) {
        const double r = m / x;
        q = 1.0 + q * r * r;
        m = x;
    } else {
        const double r = x / m;
        q += r * r;
    }
}

__device__ __forceinline__ void norm_merge(double &m, double &q, double m2, double q2)
{
    if (m2 == 0.0) return;
    if (m2 > m) {
        const double r = m / m2;
        q = q2 + q * r * r;
        m = m2;
    } else {
        const double r = m2 / m;
        q += q2 * r * r;
    }
}

// the four (m, q) of bra and ket over the block, into lane 0's slots
__device__ __forceinline__ void block_tree_norms(double *mb, double *qb, double *mk, double *qk)
{
    for (int o = 128; o > 0; o >>= 1) {
        const int t = (int)threadIdx.x;
        if (t < o) {
            norm_merge(mb[t], qb[t], mb[t + o], qb[t + o]);
            norm_merge(mk[t], qk[t], mk[t + o], qk[t + o]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rdm_fx_norms(int64_t nb, const double *__restrict__ bra, int64_t nk,
                                                      const double *__restrict__ ket, double *__restrict__ part)
{
    __shared__ double smb[256], sqb[256], smk[256], sqk[256];
    const int64_t G = (int64_t)gridDim.x * blockDim.x;
    double mb = 0.0, qb = 0.0, mk = 0.0, qk = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nb; t += G) norm_add(mb, qb, bra[t]);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nk; t += G) norm_add(mk, qk, ket[t]);
    smb[threadIdx.x] = mb;
    sqb[threadIdx.x] = qb;
    smk[threadIdx.x] = mk;
    sqk[threadIdx.x] = qk;
    __syncthreads();
    block_tree_norms(smb, sqb, smk, sqk);
    if (threadIdx.x == 0) {
        double *o = part + 4 * (size_t)blockIdx.x;
        o[0] = smb[0];
        o[1] = sqb[0];
        o[2] = smk[0];
        o[3] = sqk[0];
    }
}

// fx[0] = 2^s, fx[1] = 2^-s (sym: the ket is the bra)
__global__ __launch_bounds__(256) void k_rdm_fx_scale(const double *__restrict__ part, int sym, RdmWeights W, int R,
                                                      double *__restrict__ fx)
{
    __shared__ double smb[256], sqb[256], smk[256], sqk[256];
    double mb = 0.0, qb = 0.0, mk = 0.0, qk = 0.0;
    for (int i = threadIdx.x; i < RDM_FX_BLOCKS; i += blockDim.x) {
        norm_merge(mb, qb, part[4 * i], part[4 * i + 1]);
        norm_merge(mk, qk, part[4 * i + 2], part[4 * i + 3]);
    }
    smb[threadIdx.x] = mb;
    sqb[threadIdx.x] = qb;
    smk[threadIdx.x] = mk;
    sqk[threadIdx.x] = qk;
    __syncthreads();
    block_tree_norms(smb, sqb, smk, sqk);
    if (threadIdx.x != 0) return;
    double wmax = 0.0;
    for (int k = 0; k < R; k++) wmax = fmax(wmax, fabs(W.dev ? W.dev[k] : W.w[k]));
    double f[5] = {wmax, smb[0], sqrt(sqb[0]), sym ? smb[0] : smk[0], sqrt(sym ? sqb[0] : sqk[0])};
    const double big = 1.79e308;
    bool ok = true;
    for (double v : f) ok = ok && v > 0.0 && v <= big;
    int s = 0;
    if (ok) {
        // the exponent of the product of the five factors without forming it
        int e = 0, ei;
        double mant = 1.0;
        for (double v : f) {
            mant *= frexp(v, &ei);
            e += ei;
        }
        frexp(mant, &ei);
        s = max(-1000, min(1000, 60 - (e + ei)));
    }
    fx[0] = ldexp(1.0, s);
    fx[1] = ldexp(1.0, -s);
}

// the fixed-point accumulators back to doubles, in place
__global__ __launch_bounds__(256) void k_rdm_fx_float(double *X, int64_t n, const double *__restrict__ fx)
{
    const double inv = fx[1];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        X[t] = (double)__double_as_longlong(X[t]) * inv;
}

static void fx_float(double *x, int64_t n, const double *fx, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_rdm_fx_float, dim3((unsigned)blocks), dim3(256), 0, s, x, n, fx);
}

// scale of one call: norms of bra and ket (nd doubles each)
static void fx_scale(const void *bra, const void *ket, int64_t nd, bool sym, const RdmWeights &W, int R, double *fx,
                     hipStream_t s)
{
    double *part = fx + 32;  // RDM_FX_BLOCKS x (m, q of bra, m, q of ket)
    hipLaunchKernelGGL(k_rdm_fx_norms, dim3(RDM_FX_BLOCKS), dim3(256), 0, s, nd, (const double *)bra,
                       sym ? (int64_t)0 : nd, (const double *)ket, part);
    hipLaunchKernelGGL(k_rdm_fx_scale, dim3(1), dim3(256), 0, s, (const double *)part, (int)sym, W, R, fx);
}

// x per membership (k_rdm_x), before the row kernels
template <bool CPLX>
static void launch_rdm_x(const DevPlan &p, int R, const typename Scal<CPLX>::T *bra, typename Scal<CPLX>::T *x,
                         hipStream_t s)
{
    if (p.rdm_cls[5] == 0) return;
    const int64_t nx = p.nmem * R;
    hipLaunchKernelGGL(k_rdm_x<CPLX>, dim3((unsigned)std::min<int64_t>((nx + 255) / 256, 1 << 20)), dim3(256), 0, s, p,
                       R, bra, x);
}

// the single-pair accumulators (copy 0 of S, C, E), row by row; the
// per-pair atomic kernel over the single packets when a row does not fit
// in the LDS of a workgroup (spinor spaces of more than 100 spinors)
template <bool CPLX>
static mw_status launch_rdm_single_rows(const DevPlan &p, int R, const typename Scal<CPLX>::T *bra,
                                        const typename Scal<CPLX>::T *ket, const RdmWeights &W, bool sym,
                                        typename Scal<CPLX>::T *S, typename Scal<CPLX>::T *Cc, double *Ee,
                                        const typename Scal<CPLX>::T *x, int64_t copy_stride, const double *fx,
                                        hipStream_t s)
{
    const int n = p.n, M = p.M;
    const bool fxm = fx != nullptr;
    const size_t lds = CPLX ? (size_t)(M + (size_t)M * M) * 16 : (size_t)(2 * n + 2 * (size_t)n * n) * 8;
    if (lds <= 160 * 1024) {
        const int64_t c0 = p.rdm_cls[4], nch = p.rdm_cls[5] - c0;
        if (nch <= 0) return MW_OK;
        auto pick = [&](auto rm, auto fc) {
            constexpr int RM = decltype(rm)::value;
            constexpr bool F = decltype(fc)::value;
            return sym ? k_rdm_single_rows<CPLX, true, RM, F> : k_rdm_single_rows<CPLX, false, RM, F>;
        };
        auto pickr = [&](auto fc) {
            return R == 1 ? pick(std::integral_constant<int, 1>{}, fc)
                          : (R <= 4 ? pick(std::integral_constant<int, 4>{}, fc)
                                    : pick(std::integral_constant<int, 0>{}, fc));
        };
        auto kern = fxm ? pickr(std::true_type{}) : pickr(std::false_type{});
        if (lds > 65536 &&
            hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(MW_EHIP, "hipFuncSetAttribute failed");
        hipLaunchKernelGGL(kern, dim3((unsigned)nch), dim3(256), lds, s, p, R, ket, x, W, S, Cc, Ee, c0, fx);
        return MW_OK;
    }
    const unsigned gs = (unsigned)((p.npacket - p.npacket_double + 3) / 4);
    if (gs == 0) return MW_OK;
    auto kern = sym ? (fxm ? k_rdm_single<CPLX, true, true> : k_rdm_single<CPLX, true, false>)
                    : (fxm ? k_rdm_single<CPLX, false, true> : k_rdm_single<CPLX, false, false>);
    hipLaunchKernelGGL(kern, dim3(gs), dim3(256), 0, s, p, R, bra, ket, W, S, Cc, Ee, copy_stride, fx);
    return MW_OK;
}

// the double-pair accumulators, row by row (k_rdm_rows over the alpha-beta
// chunks into acc_ab and the pair chunks into acc_pair)
// (an LDS row of up to 160 KB: n^2 doubles, or npair scalars)
template <bool CPLX>
static mw_status launch_rdm_rows(const DevPlan &p, int R, const typename Scal<CPLX>::T *bra,
                                 const typename Scal<CPLX>::T *ket, const RdmWeights &W, bool sym,
                                 typename Scal<CPLX>::T *acc_ab, typename Scal<CPLX>::T *acc_pair,
                                 typename Scal<CPLX>::T *x, const double *fx, hipStream_t s)
{
    const bool fxm = fx != nullptr;
    using T = typename Scal<CPLX>::T;
    (void)bra;
    auto go = [&](int c, T *acc, int ncols) -> mw_status {
        const int64_t c0 = p.rdm_cls[c], nch = p.rdm_cls[c + 1] - c0;
        if (nch <= 0) return MW_OK;
        const size_t lds = (size_t)ncols * sizeof(T);
        if (lds > 160 * 1024) return fail(MW_EUNSUPPORTED, "density-matrix row exceeds the LDS of a workgroup");
        const bool wide = (c & 1) == 0;
        auto pick = [&](auto rm, auto fc) {
            constexpr int RM = decltype(rm)::value;
            constexpr bool F = decltype(fc)::value;
            return sym ? (wide ? k_rdm_rows<CPLX, true, true, RM, F> : k_rdm_rows<CPLX, true, false, RM, F>)
                       : (wide ? k_rdm_rows<CPLX, false, true, RM, F> : k_rdm_rows<CPLX, false, false, RM, F>);
        };
        auto pickr = [&](auto fc) {
            return R == 1 ? pick(std::integral_constant<int, 1>{}, fc)
                          : (R <= 4 ? pick(std::integral_constant<int, 4>{}, fc)
                                    : pick(std::integral_constant<int, 0>{}, fc));
        };
        auto kern = fxm ? pickr(std::true_type{}) : pickr(std::false_type{});
        if (lds > 65536 &&
            hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(MW_EHIP, "hipFuncSetAttribute failed");
        hipLaunchKernelGGL(kern, dim3((unsigned)nch), dim3(wide ? 256 : 512), lds, s, p, R, ket, x, W, acc, ncols, c0,
                           fx);
        return MW_OK;
    };
    for (int c = 0; c < 4; c++) {
        mw_status st = go(c, c < 2 ? acc_ab : acc_pair, c < 2 ? p.n * p.n : p.npair);
        if (st != MW_OK) return st;
    }
    return MW_OK;
}

// The device's second stream (the one sigma's single groups use) for the
// occupation correlations and the single-pair rows: they fill other accumulators than the double-pair rows,
// so they run beside the bra gather and the double rows (the single rows
// after the gather, which they read) and are joined before the final pass.  The fork and
// join events are shared, so the launch sequence holds a lock.  A caller
// stream that is being captured into a graph gets the serial order, unless
// the capturing thread lends a stream of its own (RdmCaptureSide), which
// then joins the capture as the second branch.
namespace {
struct RdmSide {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, xready = nullptr, join = nullptr;
    bool failed = false;
};
std::mutex g_rdm_side_mu;
RdmSide g_rdm_side[64];
thread_local RdmSide t_rdm_cap;  // lent by a capturer (RdmCaptureSide)

RdmSide *rdm_side_locked()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    RdmSide &x = g_rdm_side[dev];
    if (!x.s && !x.failed) {
        // the device's side stream, shared with sigma's single groups
        if (!(x.s = device_side_stream()) ||
            hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&x.xready, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&x.join, hipEventDisableTiming) != hipSuccess) {
            x.failed = true;
            x.s = nullptr;
        }
    }
    return x.s ? &x : nullptr;
}

// the side stream waits for the gathered bra (k_rdm_x on s)
bool rdm_wait_x(hipStream_t s, RdmSide *x)
{
    if (!x) return true;
    return hipEventRecord(x->xready, s) == hipSuccess && hipStreamWaitEvent(x->s, x->xready, 0) == hipSuccess;
}

// fork: work enqueued on the returned stream runs beside s (s itself when
// s is being captured or no side stream exists); the lock stays held
hipStream_t rdm_fork(hipStream_t s, std::unique_lock<std::mutex> &lk, RdmSide *&x)
{
    x = nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return s;
    if (cap != hipStreamCaptureStatusNone) {
        // a capture: the lent stream joins it through the fork event
        RdmSide *y = &t_rdm_cap;
        if (cap != hipStreamCaptureStatusActive || !y->s || hipEventRecord(y->fork, s) != hipSuccess ||
            hipStreamWaitEvent(y->s, y->fork, 0) != hipSuccess)
            return s;
        x = y;
        return y->s;
    }
    lk.lock();
    RdmSide *y = rdm_side_locked();
    if (!y || hipEventRecord(y->fork, s) != hipSuccess || hipStreamWaitEvent(y->s, y->fork, 0) != hipSuccess)
        return s;
    x = y;
    return y->s;
}

bool rdm_join(hipStream_t s, RdmSide *x)
{
    if (!x) return true;
    return hipEventRecord(x->join, x->s) == hipSuccess && hipStreamWaitEvent(s, x->join, 0) == hipSuccess;
}
}  // namespace

RdmCaptureSide::RdmCaptureSide(hipStream_t side, hipEvent_t fork, hipEvent_t xready, hipEvent_t join)
{
    t_rdm_cap.s = side;
    t_rdm_cap.fork = fork;
    t_rdm_cap.xready = xready;
    t_rdm_cap.join = join;
}

RdmCaptureSide::~RdmCaptureSide() { t_rdm_cap = RdmSide(); }

mw_status launch_rdm(const DevPlan &p, int R, const void *bra, const void *ket, const double *weights,
                     const double *dev_weights, void *gamma, void *Gamma, double fac_g, bool conj, hipStream_t s)
{
    RdmWeights W;
    for (int k = 0; k < 64; k++) W.w[k] = (weights && k < R) ? weights[k] : 1.0;
    W.dev = dev_weights;
    // one vector as bra and ket (real weights): w_JI = conj(w_IJ)
    const bool sym = bra == ket;
    const int n = p.n, M = p.M;
    const int64_t mm = (int64_t)M * M;
    const unsigned gred = (unsigned)((mm + 255) / 256);
    if (p.kind == MW_SPIN_FREE) {
        const int64_t n4 = (int64_t)n * n * n * n, np2 = (int64_t)p.npair * p.npair, n3 = (int64_t)n * n * n;
        // S | C | E, RDM_COPIES times
        const int64_t cs = 2 * (int64_t)n * n + 2 * n3;
        double *dab = (double *)p.partial, *dt0 = dab + n4, *dt1 = dt0 + np2, *S = dt1 + np2;
        double *Cc = S + 2 * (int64_t)n * n, *Ee = Cc + n3, *D = S + RDM_COPIES * cs, *part = D + mm;
        // bra coefficients per double membership, after the accumulators
        double *xb = (double *)((char *)p.partial + ((((size_t)(part - dab) + RDM_OCC_CHUNKS * mm) * 8 + 255) &
                                                     ~(size_t)255));
        // fixed point: the scale after the gathered bra
        double *fx = p.rdm_fixed ? (double *)((char *)xb + (((size_t)p.nmem * p.max_roots * 8 + 255) & ~(size_t)255))
                                 : nullptr;
        zero(dab, n4 + 2 * np2 + RDM_COPIES * cs, s);
        if (fx) {
            ProfToken ts = prof_begin("rdm_fx_scale", s);
            fx_scale(bra, ket, p.ndet * R, sym, W, R, fx, s);
            prof_end(ts, s);
        }
        std::unique_lock<std::mutex> lk(g_rdm_side_mu, std::defer_lock);
        RdmSide *side = nullptr;
        const hipStream_t s2 = rdm_fork(s, lk, side);
        // beside the bra gather and the double rows (s2): the occupation
        // correlations, then (once the gathered bra is there) the single
        // rows and their folds
        ProfToken t = prof_begin("rdm_diag", s2);
        auto occk = fx ? k_rdm_occ_lds<false, true> : k_rdm_occ_lds<false, false>;
        hipLaunchKernelGGL(occk, dim3(RDM_OCC_CHUNKS, (unsigned)((M + 127) / 128)), dim3(1024), 0, s2, p, R,
                           (const double *)bra, (const double *)ket, W, part, (const double *)fx);
        hipLaunchKernelGGL(k_rdm_occ_reduce<double>, dim3(gred), dim3(256), 0, s2, M, RDM_OCC_CHUNKS,
                           (const double *)part, D);
        prof_end(t, s2);
        launch_rdm_x<false>(p, R, (const double *)bra, xb, s);
        if (!rdm_wait_x(s, side)) return fail(MW_EHIP, "ordering the density-matrix side stream failed");
        t = prof_begin("rdm_single", s2);
        mw_status st = launch_rdm_single_rows<false>(p, R, (const double *)bra, (const double *)ket, W, sym, S, Cc, Ee,
                                                     xb, cs, fx, s2);
        prof_end(t, s2);
        if (st != MW_OK) return st;
        if (fx) fx_float(S, RDM_COPIES * cs, fx, s2);
        hipLaunchKernelGGL(k_rdm_fold<double>, dim3((unsigned)((cs + 255) / 256)), dim3(256), 0, s2, S, cs,
                           RDM_COPIES);
        if (sym) {
            hipLaunchKernelGGL(k_rdm_mirror<double>, dim3((unsigned)((2 * (int64_t)n * n + 255) / 256)), dim3(256), 0,
                               s2, S, n, 1, 2);
            hipLaunchKernelGGL(k_rdm_mirror_qxp<double>, dim3((unsigned)((2 * n3 + 255) / 256)), dim3(256), 0, s2, Cc,
                               n, 2);
        }
        t = prof_begin("rdm_double", s);
        st = launch_rdm_rows<false>(p, R, (const double *)bra, (const double *)ket, W, sym, dab, dt0, xb, fx, s);
        prof_end(t, s);
        if (st != MW_OK) return st;
        if (fx) fx_float(dab, n4 + np2, fx, s);  // dab and dt0 (dt1 stays zero)
        if (!rdm_join(s, side)) return fail(MW_EHIP, "joining the density-matrix side stream failed");
        t = prof_begin("rdm_final", s);
        hipLaunchKernelGGL(k_rdm_finalize_sf, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, p, dab, dt0, dt1,
                           S, Cc, Ee, D, (double *)gamma, (double *)Gamma, (int)sym, fac_g);
        prof_end(t, s);
    } else {
        const int64_t m4 = mm * mm, np2 = (int64_t)p.npair * p.npair, m3 = mm * M;
        // S | C, RDM_COPIES times
        const int64_t cs = mm + m3;
        double2 *dt0 = (double2 *)p.partial, *dt1 = dt0 + np2, *S = dt1 + np2, *Cc = S + mm,
                *D = S + RDM_COPIES * cs, *part = D + mm;
        double2 *xb = (double2 *)((char *)p.partial + ((((size_t)(part - dt0) + RDM_OCC_CHUNKS * mm) * 16 + 255) &
                                                       ~(size_t)255));
        double *fx = p.rdm_fixed
                         ? (double *)((char *)xb + (((size_t)p.nmem * p.max_roots * 16 + 255) & ~(size_t)255))
                         : nullptr;
        zero((double *)dt0, 2 * (2 * np2 + RDM_COPIES * cs), s);
        if (fx) {
            ProfToken ts = prof_begin("rdm_fx_scale", s);
            fx_scale(bra, ket, 2 * p.ndet * R, sym, W, R, fx, s);
            prof_end(ts, s);
        }
        std::unique_lock<std::mutex> lk(g_rdm_side_mu, std::defer_lock);
        RdmSide *side = nullptr;
        const hipStream_t s2 = rdm_fork(s, lk, side);
        ProfToken t = prof_begin("rdm_diag", s2);
        auto occk = fx ? k_rdm_occ_lds<true, true> : k_rdm_occ_lds<true, false>;
        hipLaunchKernelGGL(occk, dim3(RDM_OCC_CHUNKS, (unsigned)((M + 63) / 64)), dim3(1024), 0, s2, p, R,
                           (const double2 *)bra, (const double2 *)ket, W, part, (const double *)fx);
        hipLaunchKernelGGL(k_rdm_occ_reduce<double2>, dim3(gred), dim3(256), 0, s2, M, RDM_OCC_CHUNKS,
                           (const double2 *)part, D);
        prof_end(t, s2);
        launch_rdm_x<true>(p, R, (const double2 *)bra, xb, s);
        if (!rdm_wait_x(s, side)) return fail(MW_EHIP, "ordering the density-matrix side stream failed");
        t = prof_begin("rdm_single", s2);
        mw_status st = launch_rdm_single_rows<true>(p, R, (const double2 *)bra, (const double2 *)ket, W, sym, S, Cc,
                                                    (double *)nullptr, xb, cs, fx, s2);
        prof_end(t, s2);
        if (st != MW_OK) return st;
        if (fx) fx_float((double *)S, 2 * RDM_COPIES * cs, fx, s2);
        hipLaunchKernelGGL(k_rdm_fold<double2>, dim3((unsigned)((cs + 255) / 256)), dim3(256), 0, s2, S, cs,
                           RDM_COPIES);
        if (sym) {
            hipLaunchKernelGGL(k_rdm_mirror<double2>, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s2, S, M, 1,
                               1);
            hipLaunchKernelGGL(k_rdm_mirror_qxp<double2>, dim3((unsigned)((m3 + 255) / 256)), dim3(256), 0, s2, Cc, M,
                               1);
        }
        t = prof_begin("rdm_double", s);
        st = launch_rdm_rows<true>(p, R, (const double2 *)bra, (const double2 *)ket, W, sym, (double2 *)nullptr, dt0,
                                   xb, fx, s);
        prof_end(t, s);
        if (st != MW_OK) return st;
        if (fx) fx_float((double *)dt0, 2 * np2, fx, s);
        if (!rdm_join(s, side)) return fail(MW_EHIP, "joining the density-matrix side stream failed");
        t = prof_begin("rdm_final", s);
        hipLaunchKernelGGL(k_rdm_finalize_spinor, dim3((unsigned)((m4 + 255) / 256)), dim3(256), 0, s, p, dt0, dt1, S,
                           Cc, D, (double2 *)gamma, (double2 *)Gamma, (int)sym, fac_g, (int)conj);
        prof_end(t, s);
    }
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "rdm kernel launch failed");
    return MW_OK;
}

}  // namespace mw

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);

extern "C" mw_status mw_rdm_backward(mw_plan plan, int32_t nroots, const void *bra, const void *ket,
                                     const double *weights, void *gamma, void *Gamma, mw_stream_t stream)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace: call mw_plan_upload first");
    if (nroots < 1 || nroots > d->max_roots || nroots > 64) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    if (!bra || !ket || !gamma || !Gamma) return fail(MW_EINVAL, "NULL device pointer");
    return launch_rdm(*d, nroots, bra, ket, weights, nullptr, gamma, Gamma, 1.0, false, (hipStream_t)stream);
}
