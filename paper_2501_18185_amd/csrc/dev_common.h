// Device helpers shared by the HIP translation units of libmw.
#pragma once

#include <hip/hip_runtime.h>

#include "mw_internal.h"

namespace mw {

// ---------------------------------------------------------------------------
// scalar helpers (double or complex as double2)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sc_zero(double) { return 0.0; }
__device__ __forceinline__ double2 sc_zero(double2) { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double sc_add(double a, double b) { return a + b; }
__device__ __forceinline__ double2 sc_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double sc_mul(double a, double b) { return a * b; }
__device__ __forceinline__ double2 sc_mul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double sc_conj(double a) { return a; }
__device__ __forceinline__ double2 sc_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double sc_neg(double a, bool n) { return n ? -a : a; }
__device__ __forceinline__ double2 sc_neg(double2 a, bool n) { return n ? make_double2(-a.x, -a.y) : a; }

template <bool C> struct Scal;
template <> struct Scal<false> { using T = double; };
template <> struct Scal<true> { using T = double2; };

__device__ __forceinline__ int pair_idx(int lo, int hi) { return hi * (hi - 1) / 2 + lo; }

// ---------------------------------------------------------------------------
// Slater-Condon pieces shared by sigma, the density matrices and PT2
// ---------------------------------------------------------------------------

// H_DD of the determinant (d0, d1) by Slater-Condon: ecore + sum h_AA +
// sum over pairs A < B of (AA|BB) - (AB|BA), positions ascending, fixed order.
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T diag_value(const DevPlan &p, uint64_t d0, uint64_t d1)
{
    using T = typename Scal<CPLX>::T;
    const int n = p.n;
    const T *h = (const T *)p.h;
    const T *w = (const T *)p.w_same;
    const T *wo = (const T *)p.w_opp;
    T e = sc_zero(T());
    if constexpr (CPLX) e = make_double2(p.ecore, 0.0);
    else e = p.ecore;
    const int M = p.M;
    // positions ascending: word 0 then word 1
    for (int wa = 0; wa < 2; wa++) {
        for (uint64_t xa = wa ? d1 : d0; xa; xa &= xa - 1) {
            int a = __builtin_ctzll(xa);
            int A = wa * n + a;
            if constexpr (CPLX) e = sc_add(e, h[(size_t)A * M + A]);
            else e = sc_add(e, h[(size_t)a * n + a]);
            // partners B > A
            for (int wb = wa; wb < 2; wb++) {
                uint64_t xb = wb ? d1 : d0;
                if (wb == wa) xb &= (a == 63) ? 0ULL : ~((2ULL << a) - 1);
                for (; xb; xb &= xb - 1) {
                    int b = __builtin_ctzll(xb);
                    int B = wb * n + b;
                    if constexpr (CPLX) e = sc_add(e, w[((size_t)B * M + A) * M + A]);
                    else e = sc_add(e, (wb == wa) ? w[((size_t)b * n + a) * n + a] : wo[((size_t)b * n + a) * n + a]);
                }
            }
        }
    }
    return e;
}

// Single-excitation element <K+P_i| H |K+P_j> / (phi_i phi_j), read as the
// (j, i) entry and conjugated:  F^K_{P_j P_i} = h_{P_j P_i} + sum_{R in K}
// [(P_j P_i|R R) - (P_j R|R P_i)]  (spin-free: the exchange part only for R
// of the same spin).  Evaluated from the reference table F^omega plus the
// positions where K and omega differ.
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T single_element(const DevPlan &p, uint8_t type, uint64_t k0,
                                                                  uint64_t k1, int Xi, int Xj)
{
    using T = typename Scal<CPLX>::T;
    const T *w = (const T *)p.w_same;
    const int n = p.n;
    if constexpr (CPLX) {
        const int M = p.M;
        const size_t base = (size_t)Xj * M + Xi, stride = (size_t)M * M;
        T f = ((const T *)p.f_ref)[base];
        T add = sc_zero(T()), sub = sc_zero(T());
        for (uint64_t x = k0 & ~p.ref0; x; x &= x - 1) add = sc_add(add, w[(size_t)__builtin_ctzll(x) * stride + base]);
        for (uint64_t x = k1 & ~p.ref1; x; x &= x - 1) add = sc_add(add, w[(size_t)(n + __builtin_ctzll(x)) * stride + base]);
        for (uint64_t x = p.ref0 & ~k0; x; x &= x - 1) sub = sc_add(sub, w[(size_t)__builtin_ctzll(x) * stride + base]);
        for (uint64_t x = p.ref1 & ~k1; x; x &= x - 1) sub = sc_add(sub, w[(size_t)(n + __builtin_ctzll(x)) * stride + base]);
        f = sc_add(f, add);
        f = make_double2(f.x - sub.x, f.y - sub.y);
        return sc_conj(f);
    } else {
        const T *wo = (const T *)p.w_opp;
        const int s = type == G_SINGLE_A ? 0 : 1;
        const int pi = Xi - s * n, pj = Xj - s * n;
        const size_t base = (size_t)pj * n + pi, stride = (size_t)n * n;
        T f = ((const T *)p.f_ref)[(size_t)s * stride + base];
        const uint64_t ks = s ? k1 : k0, ko = s ? k0 : k1;
        const uint64_t rs = s ? p.ref1 : p.ref0, ro = s ? p.ref0 : p.ref1;
        T add = 0.0, sub = 0.0;
        for (uint64_t x = ks & ~rs; x; x &= x - 1) add += w[(size_t)__builtin_ctzll(x) * stride + base];
        for (uint64_t x = ko & ~ro; x; x &= x - 1) add += wo[(size_t)__builtin_ctzll(x) * stride + base];
        for (uint64_t x = rs & ~ks; x; x &= x - 1) sub += w[(size_t)__builtin_ctzll(x) * stride + base];
        for (uint64_t x = ro & ~ko; x; x &= x - 1) sub += wo[(size_t)__builtin_ctzll(x) * stride + base];
        return (f + add) - sub;
    }
}



}  // namespace mw
