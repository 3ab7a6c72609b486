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
//  k_gather       (a few lanes per determinant and root):
//      sigma_I = H_II c_I + sum of I's partials (fixed order), one write.
//      Partials are written in member order (coalesced) and gathered
//      through the determinant-major membership list.
//  k_diag         (one thread per determinant): H_II by Slater-Condon.
//
// All sums are in a fixed order, so repeated calls give identical bits.
#include <hip/hip_runtime.h>

#include <vector>

#include "mw_internal.h"
#include "dev_common.h"

namespace mw {

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

// Offset of the double-excitation integral A(pair_i, pair_j) = (P Q|R S) -
// (P S|R Q), with (P,R) added in i and (Q,S) added in j, read as the (j, i)
// entry of its table: column part (depends on i only) + row part (j only).
// Each member carries a layout bit choosing between two tables that hold
// the same values with transposed column order, so that the members of a
// wave read runs of consecutive columns.
struct DoubleIndex {
    size_t col;
    size_t row_stride;
    int n, off, ab;
    __device__ __forceinline__ size_t row(int Xj, int Yj) const
    {
        if (ab) return ((size_t)Xj * n + (Yj - n)) * row_stride;
        return (size_t)pair_idx(Xj - off, Yj - off) * row_stride;
    }
};

__device__ __forceinline__ int pair_lex_d(int lo, int hi, int m) { return lo * (2 * m - lo - 1) / 2 + (hi - lo - 1); }

template <bool CPLX>
__device__ __forceinline__ DoubleIndex double_index(const DevPlan &p, uint8_t type, int Xi, int Yi, bool lay)
{
    DoubleIndex d;
    d.n = p.n;
    if (!CPLX && type == G_AB) {
        // (p_i q_j | r_i s_j) stored as g_ab[q][s][p][r] (layout 0) or
        // g_ab1[q][s][r][p] (layout 1)
        d.ab = 1;
        d.off = 0;
        d.row_stride = (size_t)p.n * p.n;
        const int pi = Xi, ri = Yi - p.n;
        d.col = lay ? (size_t)ri * p.n + pi : (size_t)pi * p.n + ri;
    } else {
        d.ab = 0;
        d.off = (!CPLX && type == G_BB) ? p.n : 0;
        d.row_stride = p.npair;
        const int m = CPLX ? p.M : p.n;
        d.col = lay ? pair_lex_d(Xi - d.off, Yi - d.off, m) : pair_idx(Xi - d.off, Yi - d.off);
    }
    return d;
}

// Double groups.  Lane = member i; the partner loop is unrolled by U so that
// U member records, U integrals and U coefficient rows are in flight at once
// (the loop is bound by memory latency, not arithmetic).
template <bool CPLX, int RC, int U>
__device__ __forceinline__ void group_double_body(const DevPlan &p, int64_t wave, int lane, int R, int r0,
                                                  const typename Scal<CPLX>::T *__restrict__ c,
                                                  typename Scal<CPLX>::T *__restrict__ partial)
{
    using T = typename Scal<CPLX>::T;
    const uint32_t m = p.pk_off[wave] + lane;
    if (m >= p.pk_off[wave + 1]) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    const uint32_t negi = (me.y >> 16) & 1;
    const bool lay = (me.y >> 17) & 1;
    const DoubleIndex di = double_index<CPLX>(p, type, Xi, Yi, lay);
    const T *tab = (const T *)((!CPLX && type == G_AB) ? (lay ? p.g_ab1 : p.g_ab) : (lay ? p.a_pair1 : p.a_pair));
    T acc[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) acc[k] = sc_zero(T());
    const int nr = min(RC, R - r0);
    for (uint32_t j = j0; j < j1; j += U) {
        uint2 o[U];
        bool hit[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool in = j + u < j1;
            o[u] = p.mem[in ? j + u : j0];
            const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
            hit[u] = in && !(Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi);
        }
        T v[U];
        T cj[U][RC];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
            const size_t idx = hit[u] ? di.row(Xj, Yj) + di.col : 0;
            v[u] = tab[idx];
            const T *cr = c + (size_t)(hit[u] ? o[u].x : 0) * R + r0;
#pragma unroll
            for (int k = 0; k < RC; k++) cj[u][k] = cr[k < nr ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!hit[u]) continue;
            T x = sc_neg(CPLX ? sc_conj(v[u]) : v[u], (negi ^ ((o[u].y >> 16) & 1)) != 0);
#pragma unroll
            for (int k = 0; k < RC; k++) acc[k] = sc_add(acc[k], sc_mul(x, cj[u][k]));
        }
    }
    T *out = partial + (size_t)m * R + r0;
#pragma unroll
    for (int k = 0; k < RC; k++)
        if (k < nr) out[k] = acc[k];
}

// Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD b % 8).
// Remap so that runs of XCD_CHUNK consecutive logical blocks (the packets of
// one large group, which read the same partner records and coefficients)
// share an XCD and its L2, while successive runs rotate over the XCDs.  The
// grid is a multiple of 8 * XCD_CHUNK, so the map is a bijection.
constexpr int XCD_CHUNK = 16;
__device__ __forceinline__ int64_t xcd_block(int64_t b)
{
    const int64_t x = b & 7, r = b >> 3;
    return ((r / XCD_CHUNK) * 8 + x) * XCD_CHUNK + (r % XCD_CHUNK);
}

static inline unsigned xcd_grid(int64_t blocks)
{
    const int64_t q = 8 * XCD_CHUNK;
    return (unsigned)((blocks + q - 1) / q * q);
}

template <bool CPLX, int RC, int U>
__global__ __launch_bounds__(256) void k_group_double(DevPlan p, int R, int r0,
                                                      const typename Scal<CPLX>::T *__restrict__ c,
                                                      typename Scal<CPLX>::T *__restrict__ partial)
{
    const int64_t wave = xcd_block(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (wave >= p.npacket_double) return;
    group_double_body<CPLX, RC, U>(p, wave, threadIdx.x & 63, R, r0, c, partial);
}

// Single groups (few pairs; each element needs the reference correction).
template <bool CPLX, int RC>
__device__ __forceinline__ void group_single_body(const DevPlan &p, int64_t wave, int lane, int R, int r0,
                                                  const typename Scal<CPLX>::T *__restrict__ c,
                                                  typename Scal<CPLX>::T *__restrict__ partial)
{
    using T = typename Scal<CPLX>::T;
    const uint32_t m = p.pk_off[wave] + lane;
    if (m >= p.pk_off[wave + 1]) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255;
    const uint32_t negi = (me.y >> 16) & 1;
    const uint64_t k0 = p.grp_key[2 * g], k1 = p.grp_key[2 * g + 1];
    T acc[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) acc[k] = sc_zero(T());
    const int nr = min(RC, R - r0);
    for (uint32_t j = j0; j < j1; j++) {
        const uint2 o = p.mem[j];
        const int Xj = o.y & 255;
        if (Xj == Xi) continue;
        T v = single_element<CPLX>(p, type, k0, k1, Xi, Xj);
        v = sc_neg(v, (negi ^ ((o.y >> 16) & 1)) != 0);
        const T *cj = c + (size_t)o.x * R + r0;
#pragma unroll
        for (int k = 0; k < RC; k++)
            if (k < nr) acc[k] = sc_add(acc[k], sc_mul(v, cj[k]));
    }
    T *out = partial + (size_t)m * R + r0;
#pragma unroll
    for (int k = 0; k < RC; k++)
        if (k < nr) out[k] = acc[k];
}

template <bool CPLX, int RC>
__global__ __launch_bounds__(256) void k_group_single(DevPlan p, int R, int r0,
                                                      const typename Scal<CPLX>::T *__restrict__ c,
                                                      typename Scal<CPLX>::T *__restrict__ partial)
{
    const int64_t wave = p.npacket_double + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (wave >= p.npacket) return;
    group_single_body<CPLX, RC>(p, wave, threadIdx.x & 63, R, r0, c, partial);
}

// sigma_I = H_II c_I + sum of I's partials.  GL lanes per (I, root); each
// lane sums a strided subset of the slots, then a fixed butterfly reduces
// them (deterministic order).
template <bool CPLX, int GL>
__device__ __forceinline__ void gather_body(const DevPlan &p, int64_t gt, int R,
                                            const typename Scal<CPLX>::T *__restrict__ c,
                                            const typename Scal<CPLX>::T *__restrict__ partial,
                                            typename Scal<CPLX>::T *__restrict__ sigma)
{
    using T = typename Scal<CPLX>::T;
    const int64_t t = gt / GL;
    const int sub = (int)(gt % GL);
    const bool active = t < p.ndet * R;
    T acc = sc_zero(T());
    int64_t I = 0;
    int k = 0;
    if (active) {
        I = t / R;
        k = (int)(t - I * R);
        const uint32_t s0 = p.rowptr[I], s1 = p.rowptr[I + 1];
        for (uint32_t s = s0 + sub; s < s1; s += GL) acc = sc_add(acc, partial[(size_t)p.slot_mem[s] * R + k]);
    }
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
        if constexpr (CPLX) {
            acc.x += __shfl_xor(acc.x, off, GL);
            acc.y += __shfl_xor(acc.y, off, GL);
        } else {
            acc += __shfl_xor(acc, off, GL);
        }
    }
    if (active && sub == 0) sigma[t] = sc_add(sc_mul(((const T *)p.diag)[I], c[t]), acc);
}

template <bool CPLX, int GL>
__global__ __launch_bounds__(256) void k_gather(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ c,
                                                const typename Scal<CPLX>::T *__restrict__ partial,
                                                typename Scal<CPLX>::T *__restrict__ sigma)
{
    gather_body<CPLX, GL>(p, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, R, c, partial, sigma);
}

template <bool CPLX, int RC, int U>
static void launch_double(const DevPlan &p, int R, int r0, const typename Scal<CPLX>::T *c,
                          typename Scal<CPLX>::T *part, hipStream_t s)
{
    unsigned grid = xcd_grid((p.npacket_double + 3) / 4);
    hipLaunchKernelGGL((k_group_double<CPLX, RC, U>), dim3(grid), dim3(256), 0, s, p, R, r0, c, part);
}

template <bool CPLX, int RC>
static void launch_groups(const DevPlan &p, int R, int r0, const typename Scal<CPLX>::T *c,
                          typename Scal<CPLX>::T *part, hipStream_t s)
{
    if (p.npacket_double > 0) {
        ProfToken t = prof_begin("group_sigma", s);
        // partner-loop unroll: tunable (mw_autotune)
        if (p.tune_u <= 4) launch_double<CPLX, RC, 4>(p, R, r0, c, part, s);
        else if (p.tune_u <= 8 || CPLX) launch_double<CPLX, RC, 8>(p, R, r0, c, part, s);
        else launch_double<CPLX, RC, 16>(p, R, r0, c, part, s);
        prof_end(t, s);
    }
    const int64_t ns = p.npacket - p.npacket_double;
    if (ns > 0) {
        ProfToken t = prof_begin("group_single", s);
        unsigned grid = (unsigned)((ns + 3) / 4);
        hipLaunchKernelGGL((k_group_single<CPLX, RC>), dim3(grid), dim3(256), 0, s, p, R, r0, c, part);
        prof_end(t, s);
    }
}

template <bool CPLX, int GL>
static void launch_gather(const DevPlan &p, int R, const typename Scal<CPLX>::T *c,
                          const typename Scal<CPLX>::T *part, typename Scal<CPLX>::T *sigma, hipStream_t s)
{
    int64_t tot = p.ndet * R * GL;
    hipLaunchKernelGGL((k_gather<CPLX, GL>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, R, c, part,
                       sigma);
}

template <bool CPLX>
static mw_status sigma_t(const DevPlan &p, int R, const void *c, void *sigma, hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    const T *cc = (const T *)c;
    T *part = (T *)p.partial;
    for (int r0 = 0; r0 < R; r0 += 4) {
        int left = R - r0;
        if (left == 1) launch_groups<CPLX, 1>(p, R, r0, cc, part, s);
        else if (left == 2) launch_groups<CPLX, 2>(p, R, r0, cc, part, s);
        else launch_groups<CPLX, 4>(p, R, r0, cc, part, s);
    }
    ProfToken t = prof_begin("gather", s);
    if (p.tune_gl <= 8) launch_gather<CPLX, 8>(p, R, cc, part, (T *)sigma, s);
    else if (p.tune_gl <= 16) launch_gather<CPLX, 16>(p, R, cc, part, (T *)sigma, s);
    else launch_gather<CPLX, 32>(p, R, cc, part, (T *)sigma, s);
    prof_end(t, s);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "sigma kernel launch failed");
    return MW_OK;
}

mw_status launch_sigma(const DevPlan &p, int R, const void *c, void *sigma, hipStream_t s)
{
    return p.kind == MW_SPINOR ? sigma_t<true>(p, R, c, sigma, s) : sigma_t<false>(p, R, c, sigma, s);
}

// ---------------------------------------------------------------------------
// batched sigma: one persistent launch over the packets of every problem
// ---------------------------------------------------------------------------

// Waves pull packet indices from one device counter (the dynamic schedule of
// the paper's OpenMP/MPI task loops, section 3.1.2, as a GPU work queue);
// problems are ordered by decreasing work and each problem's packets by
// decreasing group size.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_batched_groups(BatchArgs a)
{
    using T = typename Scal<CPLX>::T;
    const int lane = threadIdx.x & 63;
    const int64_t total = a.pk_start[a.nprob];
    // Work queue per XCD (block b runs on XCD b % 8): the packet sequence is
    // cut into chunks of CHUNK packets and chunk ch belongs to XCD ch % 8,
    // so the packets of one group meet in one L2.  A wave claims the next
    // chunk of its own XCD; when that queue is empty it takes chunks from
    // the others.  All counters start at zero.
    constexpr uint32_t CHUNK = 16;
    const int64_t nchunk = (total + CHUNK - 1) / CHUNK;
    const int home = blockIdx.x & 7;
    for (int qi = 0; qi < 8; qi++) {
        const int xq = (home + qi) & 7;
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.counter[xq], 1u);
            t = __shfl(t, 0);
            const int64_t ch = (int64_t)t * 8 + xq;
            if (ch >= nchunk) break;
            const int64_t u1 = min<int64_t>(total, (ch + 1) * CHUNK);
            for (int64_t u = ch * CHUNK; u < u1; u++) {
                int q = 0;
                while (u >= a.pk_start[q + 1]) q++;
                const DevPlan &p = *a.plans[q];
                const int64_t w = u - a.pk_start[q];
                const int R = a.R[q];
                const T *c = (const T *)a.c[q];
                T *part = (T *)p.partial;
                for (int r0 = 0; r0 < R; r0 += 4) {
                    // unroll 4: four roots of four partners keep the register
                    // count at the plain kernel's occupancy
                    if (w < p.npacket_double) group_double_body<CPLX, 4, 4>(p, w, lane, R, r0, c, part);
                    else group_single_body<CPLX, 4>(p, w, lane, R, r0, c, part);
                }
            }
        }
    }
}

// Gather for all problems: block b belongs to the problem whose block range
// holds b (block-uniform, so the plan fields are scalar loads).
template <bool CPLX>
__global__ __launch_bounds__(256) void k_batched_gather(BatchArgs a)
{
    using T = typename Scal<CPLX>::T;
    constexpr int GL = 16;
    const int64_t b = blockIdx.x;
    int q = 0;
    while (b >= a.blk_start[q + 1]) q++;
    const DevPlan &p = *a.plans[q];
    const int64_t local = (b - a.blk_start[q]) * blockDim.x + threadIdx.x;
    gather_body<CPLX, GL>(p, local, a.R[q], (const T *)a.c[q], (const T *)p.partial, (T *)a.sigma[q]);
}

__global__ void k_reset_counter(uint32_t *ctr)
{
    if (threadIdx.x < 8) ctr[threadIdx.x] = 0u;
}

mw_status launch_batched(const BatchArgs &a, bool cplx, int blocks, hipStream_t s, bool timing)
{
    if (a.nprob == 0) return MW_OK;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, a.counter);
    ProfToken t = timing ? prof_begin("batched_groups", s) : ProfToken{nullptr, nullptr, ""};
    if (cplx) hipLaunchKernelGGL(k_batched_groups<true>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_batched_groups<false>, dim3(blocks), dim3(256), 0, s, a);
    prof_end(t, s);
    if (timing) t = prof_begin("batched_gather", s);
    const unsigned gg = (unsigned)a.blk_start[a.nprob];
    if (cplx) hipLaunchKernelGGL(k_batched_gather<true>, dim3(gg), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_batched_gather<false>, dim3(gg), dim3(256), 0, s, a);
    prof_end(t, s);
    if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "batched launch failed");
    return MW_OK;
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
