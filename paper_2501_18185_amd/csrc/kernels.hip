// HIP kernels of libmw for gfx950 (CDNA4, wave64).
//
// sigma = H c is evaluated group by group (MetaWave section 2.3, "bunch"
// scheme: classify pairs by what they share, fetch the integrals of the
// class, contract).  The plan groups determinants by a shared (N-1)- or
// (N-2)-electron string K; members of a group are K plus an added position
// (single groups) or an added pair (double groups).
//
//  k_group_sigma  (one wave per packet of <= 64 consecutive members; lane =
//                  member i, loop over the members j of i's group):
//      partial_i += H_ij c_j   for every j connected to i in this group,
//      H_ij = phi_i phi_j A(pair_i, pair_j) (doubles) or phi_i phi_j F^K
//      (singles).  The integral is read through Hermiticity as the entry
//      (row = j, column = i) and conjugated, so that for a fixed j the lanes
//      of a wave read consecutive columns of one row.  No atomics.
//  k_gather       (one thread per determinant and root):
//      sigma_I = H_II c_I + sum of I's partials (fixed order), one write.
//  k_diag         (one thread per determinant): H_II by Slater-Condon.
//
// All sums are in a fixed order, so repeated calls give identical bits.
#include <hip/hip_runtime.h>

#include <vector>

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
// diagonal
// ---------------------------------------------------------------------------

template <bool CPLX>
__global__ __launch_bounds__(256) void k_diag(DevPlan p)
{
    using T = typename Scal<CPLX>::T;
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p.ndet) return;
    const int n = p.n;
    const T *h = (const T *)p.h;
    const T *w = (const T *)p.w_same;
    const T *wo = (const T *)p.w_opp;
    uint64_t d0 = p.dets[2 * I], d1 = p.dets[2 * I + 1];
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
    ((T *)p.diag)[I] = e;
}

mw_status launch_diag(const DevPlan &p, hipStream_t s)
{
    if (p.ndet == 0) return MW_OK;
    unsigned grid = (unsigned)((p.ndet + 255) / 256);
    if (p.kind == MW_SPINOR) hipLaunchKernelGGL(k_diag<true>, dim3(grid), dim3(256), 0, s, p);
    else hipLaunchKernelGGL(k_diag<false>, dim3(grid), dim3(256), 0, s, p);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "k_diag launch failed");
    return MW_OK;
}

// ---------------------------------------------------------------------------
// group contraction
// ---------------------------------------------------------------------------

// Single-excitation element <K+P_i| H |K+P_j> / (phi_i phi_j), read as the
// (j, i) entry and conjugated:  F^K_{P_j P_i} = h_{P_j P_i} + sum_{R in K}
// [(P_j P_i|R R) - (P_j R|R P_i)]  (spin-free: the exchange part only for R
// of the same spin).
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T single_element(const DevPlan &p, uint8_t type, uint64_t k0,
                                                                  uint64_t k1, int Xi, int Xj)
{
    using T = typename Scal<CPLX>::T;
    const T *h = (const T *)p.h;
    const T *w = (const T *)p.w_same;
    const int n = p.n;
    if constexpr (CPLX) {
        const int M = p.M;
        T f = h[(size_t)Xj * M + Xi];
        const T *row = w + (size_t)Xj * M + Xi;
        const size_t stride = (size_t)M * M;
        for (uint64_t x = k0; x; x &= x - 1) f = sc_add(f, row[(size_t)__builtin_ctzll(x) * stride]);
        for (uint64_t x = k1; x; x &= x - 1) f = sc_add(f, row[(size_t)(n + __builtin_ctzll(x)) * stride]);
        return sc_conj(f);
    } else {
        const T *wo = (const T *)p.w_opp;
        const int pi = Xi % n, pj = Xj % n;
        const size_t base = (size_t)pj * n + pi, stride = (size_t)n * n;
        T f = h[base];
        uint64_t same = type == G_SINGLE_A ? k0 : k1;
        uint64_t opp = type == G_SINGLE_A ? k1 : k0;
        for (uint64_t x = same; x; x &= x - 1) f += w[(size_t)__builtin_ctzll(x) * stride + base];
        for (uint64_t x = opp; x; x &= x - 1) f += wo[(size_t)__builtin_ctzll(x) * stride + base];
        return f;
    }
}

// Double-excitation integral A(pair_i, pair_j) = (P Q|R S) - (P S|R Q) with
// (P,R) the pair added in i and (Q,S) the pair added in j, read as the
// (j, i) entry of the table and conjugated.
template <bool CPLX>
__device__ __forceinline__ typename Scal<CPLX>::T double_element(const DevPlan &p, uint8_t type, int Xi, int Yi,
                                                                  int Xj, int Yj)
{
    using T = typename Scal<CPLX>::T;
    const T *a = (const T *)p.a_pair;
    if constexpr (CPLX) {
        return sc_conj(a[(size_t)pair_idx(Xj, Yj) * p.npair + pair_idx(Xi, Yi)]);
    } else {
        const int n = p.n;
        if (type == G_AB) {
            // (p_i q_j | r_i s_j) stored as g_ab[q][s][p][r]
            const T *g = (const T *)p.g_ab;
            return g[(((size_t)Xj * n + (Yj - n)) * n + Xi) * n + (Yi - n)];
        }
        const int o = type == G_BB ? n : 0;
        return a[(size_t)pair_idx(Xj - o, Yj - o) * p.npair + pair_idx(Xi - o, Yi - o)];
    }
}

template <bool CPLX, int RC>
__global__ __launch_bounds__(256) void k_group_sigma(DevPlan p, int R, int r0,
                                                     const typename Scal<CPLX>::T *__restrict__ c,
                                                     typename Scal<CPLX>::T *__restrict__ partial)
{
    using T = typename Scal<CPLX>::T;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= p.npacket) return;
    const uint32_t m = p.pk_off[wave] + lane;
    if (m >= p.pk_off[wave + 1]) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    const bool negi = (me.y >> 16) & 1;
    T acc[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) acc[k] = sc_zero(T());
    const int nr = min(RC, R - r0);
    if (type == G_SINGLE_A || type == G_SINGLE_B || type == G_SINGLE_S) {
        const uint64_t k0 = p.grp_key[2 * g], k1 = p.grp_key[2 * g + 1];
        for (uint32_t j = j0; j < j1; j++) {
            const uint2 o = p.mem[j];
            const int Xj = o.y & 255;
            if (Xj == Xi) continue;
            T v = single_element<CPLX>(p, type, k0, k1, Xi, Xj);
            v = sc_neg(v, negi ^ (bool)((o.y >> 16) & 1));
            const T *cj = c + (size_t)o.x * R + r0;
#pragma unroll
            for (int k = 0; k < RC; k++)
                if (k < nr) acc[k] = sc_add(acc[k], sc_mul(v, cj[k]));
        }
    } else {
        for (uint32_t j = j0; j < j1; j++) {
            const uint2 o = p.mem[j];
            const int Xj = o.y & 255, Yj = (o.y >> 8) & 255;
            if (Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi) continue;
            T v = double_element<CPLX>(p, type, Xi, Yi, Xj, Yj);
            v = sc_neg(v, negi ^ (bool)((o.y >> 16) & 1));
            const T *cj = c + (size_t)o.x * R + r0;
#pragma unroll
            for (int k = 0; k < RC; k++)
                if (k < nr) acc[k] = sc_add(acc[k], sc_mul(v, cj[k]));
        }
    }
    T *out = partial + (size_t)p.mem_slot[m] * R + r0;
#pragma unroll
    for (int k = 0; k < RC; k++)
        if (k < nr) out[k] = acc[k];
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_gather(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ c,
                                                const typename Scal<CPLX>::T *__restrict__ partial,
                                                typename Scal<CPLX>::T *__restrict__ sigma)
{
    using T = typename Scal<CPLX>::T;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.ndet * R) return;
    int64_t I = t / R;
    int k = (int)(t - I * R);
    T acc = sc_mul(((const T *)p.diag)[I], c[t]);
    const uint32_t s0 = p.rowptr[I], s1 = p.rowptr[I + 1];
    for (uint32_t s = s0; s < s1; s++) acc = sc_add(acc, partial[(size_t)s * R + k]);
    sigma[t] = acc;
}

template <bool CPLX>
static mw_status sigma_t(const DevPlan &p, int R, const void *c, void *sigma, hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    const T *cc = (const T *)c;
    T *part = (T *)p.partial;
    if (p.npacket > 0) {
        unsigned grid = (unsigned)((p.npacket + 3) / 4);
        for (int r0 = 0; r0 < R; r0 += 4) {
            int left = R - r0;
            if (left == 1) hipLaunchKernelGGL((k_group_sigma<CPLX, 1>), dim3(grid), dim3(256), 0, s, p, R, r0, cc, part);
            else if (left == 2) hipLaunchKernelGGL((k_group_sigma<CPLX, 2>), dim3(grid), dim3(256), 0, s, p, R, r0, cc, part);
            else hipLaunchKernelGGL((k_group_sigma<CPLX, 4>), dim3(grid), dim3(256), 0, s, p, R, r0, cc, part);
        }
    }
    int64_t tot = p.ndet * R;
    hipLaunchKernelGGL(k_gather<CPLX>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, R, cc, part, (T *)sigma);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "sigma kernel launch failed");
    return MW_OK;
}

mw_status launch_sigma(const DevPlan &p, int R, const void *c, void *sigma, hipStream_t s)
{
    return p.kind == MW_SPINOR ? sigma_t<true>(p, R, c, sigma, s) : sigma_t<false>(p, R, c, sigma, s);
}

// ---------------------------------------------------------------------------
// connectivity dump (debug)
// ---------------------------------------------------------------------------

// mode 0: count connected partners of every member; mode 1: write records at
// the member's offset.  Records: I, J, P, Q, R, S, sign.
__global__ __launch_bounds__(256) void k_connect(DevPlan p, int mode, uint32_t *cnt, const uint64_t *offs,
                                                 int64_t *out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= p.nmem) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const bool single = type == G_SINGLE_A || type == G_SINGLE_B || type == G_SINGLE_S;
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    const bool negi = (me.y >> 16) & 1;
    uint32_t c = 0;
    int64_t *o = mode ? out + 7 * offs[m] : nullptr;
    for (uint32_t j = j0; j < j1; j++) {
        const uint2 q = p.mem[j];
        const int Xj = q.y & 255, Yj = (q.y >> 8) & 255;
        bool hit = single ? (Xj != Xi) : !(Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi);
        if (!hit) continue;
        if (mode) {
            int sg = (negi ^ (bool)((q.y >> 16) & 1)) ? -1 : 1;
            o[0] = me.x; o[1] = q.x; o[2] = Xi; o[3] = Xj;
            o[4] = single ? -1 : Yi; o[5] = single ? -1 : Yj; o[6] = sg;
            o += 7;
        }
        c++;
    }
    if (!mode) cnt[m] = c;
}

mw_status launch_connect(const DevPlan &p, int64_t *count, int64_t *out, hipStream_t s)
{
    // the per-member counts and offsets live in the partial scratch region,
    // which holds at least nmem doubles
    if (p.nmem == 0) {
        *count = 0;
        return MW_OK;
    }
    uint32_t *cnt = (uint32_t *)p.partial;
    unsigned grid = (unsigned)((p.nmem + 255) / 256);
    hipLaunchKernelGGL(k_connect, dim3(grid), dim3(256), 0, s, p, 0, cnt, (const uint64_t *)nullptr, (int64_t *)nullptr);
    std::vector<uint32_t> hc(p.nmem);
    if (hipMemcpyAsync(hc.data(), cnt, p.nmem * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MW_EHIP, "connect count copy failed");
    std::vector<uint64_t> off(p.nmem);
    uint64_t acc = 0;
    for (int64_t m = 0; m < p.nmem; m++) {
        off[m] = acc;
        acc += hc[m];
    }
    *count = (int64_t)acc;
    if (!out) return MW_OK;
    // offsets go after the counts in the scratch region when it is large
    // enough (nmem * max_roots * scalar >= 12 bytes per member); otherwise
    // they are not needed beyond this call, so reuse the count slots' space
    size_t scratch = (size_t)p.nmem * p.max_roots * (p.kind == MW_SPINOR ? 16 : 8);
    if (scratch < (size_t)p.nmem * 8) return fail(MW_EWORKSPACE, "scratch too small for the dump");
    uint64_t *doff = (uint64_t *)p.partial;
    if (hipMemcpyAsync(doff, off.data(), p.nmem * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(MW_EHIP, "connect offset copy failed");
    hipLaunchKernelGGL(k_connect, dim3(grid), dim3(256), 0, s, p, 1, (uint32_t *)nullptr, (const uint64_t *)doff, out);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(MW_EHIP, "connect dump failed");
    return MW_OK;
}

}  // namespace mw
