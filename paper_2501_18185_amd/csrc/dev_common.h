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


}  // namespace mw
