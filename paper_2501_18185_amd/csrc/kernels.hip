// HIP kernels of libmw for gfx950 (CDNA4, wave64).
//
// sigma = H c is evaluated group by group (MetaWave section 2.3, "bunch"
// scheme: classify pairs by what they share, fetch the integrals of the
// class, contract).  The plan groups determinants by a shared (N-1)- or
// (N-2)-electron string K; members of a group are K plus an added position
// (single groups) or an added pair (double groups).
//
//  k_group_double, k_group_single (one wave per packet of <= 64 consecutive
//                  members; lane = member i, loop over the members j of i's
//                  group):
//      partial_i += H_ij c_j   for every j connected to i in this group,
//      H_ij = phi_i phi_j A(pair_i, pair_j) (doubles) or phi_i phi_j F^K
//      (singles).  The integral is read through Hermiticity as the entry
//      (row = j, column = i) and conjugated, so that for a fixed j the lanes
//      of a wave read consecutive columns of one row.  Small groups are
//      packed whole, so their partners are lanes of the same wave (records
//      by shuffles); large groups are cut into 64-member blocks and evaluate
//      each unordered pair once, the mirrored term going to a column
//      partial.  No atomics.
//  k_gather       (a few lanes per determinant and root):
//      sigma_I = H_II c_I + sum of I's partials (fixed order), one write.
//      Partials are placed by determinant region (about 2 MB each) and
//      writing XCD, and gathered through the determinant-major list of
//      their positions: the region an XCD sums stays in its L2.
//  k_diag         (one thread per determinant): H_II by Slater-Condon.
//  k_batched_*    the same bodies over the packets of many problems.
//
// All sums are in a fixed order, so repeated calls give identical bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "mw_internal.h"
#include "dev_common.h"

// Partial sums are written once and read only by the gather, after the
// group kernels.  Their positions (the plan's slot_pos) are grouped by
// determinant region and writing XCD, so a wave's stores are scattered over
// the write frontiers of many regions; plain stores let L2 merge each
// frontier line before it is written back (non-temporal stores measured
// slower with this placement: sigma 9.74 against 9.62 ms).
template <typename T> __device__ __forceinline__ void store_partial(T v, T *p) { *p = v; }

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
    ((T *)p.diag)[I] = diag_value<CPLX>(p, p.dets[2 * I], p.dets[2 * I + 1]);
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

// Offset of the double-excitation integral A(pair_i, pair_j) = (P Q|R S) -
// (P S|R Q), with (P,R) added in i and (Q,S) added in j, read as the (j, i)
// entry of its table: column part (depends on i only) + row part (j only).
// Each member carries a layout bit choosing between two tables that hold
// the same values with transposed column order, so that the members of a
// wave read runs of consecutive columns.
struct DoubleIndex {
    uint32_t col;
    uint32_t row_stride;
    int n, offx, offy, ab, lay;
    // element index (below 2^32 for every table), without branches: the
    // lanes of a wave mix group types and layouts
    __device__ __forceinline__ uint32_t at(int Xj, int Yj) const
    {
        const int x = Xj - offx, y = Yj - offy;
        // alpha-beta, layout 1: the row (s_j, q_j) of the same table holds
        // the row (q_j, s_j) with the column indices transposed
        const uint32_t rab = lay ? (uint32_t)(y * n + x) : (uint32_t)(x * n + y);
        const uint32_t rpr = (uint32_t)((y * (y - 1)) >> 1) + (uint32_t)x;
        return (ab ? rab : rpr) * row_stride + col;
    }
};

__device__ __forceinline__ int pair_lex_d(int lo, int hi, int m) { return lo * (2 * m - lo - 1) / 2 + (hi - lo - 1); }

template <bool CPLX>
__device__ __forceinline__ DoubleIndex double_index(const DevPlan &p, uint8_t type, int Xi, int Yi, bool lay)
{
    DoubleIndex d;
    d.n = p.n;
    d.lay = lay;
    if (!CPLX && type == G_AB) {
        // (p_i q_j | r_i s_j) = g_ab[q][s][p][r] (layout 0) = g_ab[s][q][r][p]
        // (layout 1: p fastest across the lanes)
        d.ab = 1;
        d.offx = 0;
        d.offy = p.n;
        d.row_stride = (uint32_t)(p.n * p.n);
        const int pi = Xi, ri = Yi - p.n;
        d.col = lay ? (uint32_t)(ri * p.n + pi) : (uint32_t)(pi * p.n + ri);
    } else {
        d.ab = 0;
        d.offx = d.offy = (!CPLX && type == G_BB) ? p.n : 0;
        d.row_stride = (uint32_t)p.npair;
        const int m = CPLX ? p.M : p.n;
        d.col = lay ? (uint32_t)pair_lex_d(Xi - d.offx, Yi - d.offx, m) : (uint32_t)pair_idx(Xi - d.offx, Yi - d.offx);
    }
    return d;
}

// Double groups.  Lane = member i; the partner loop is unrolled by U so that
// U member records, U integrals and U coefficient rows are in flight at once
// (the loop is bound by memory latency, not arithmetic).
// ---------------------------------------------------------------------------
// Large double groups (k >= 64): each unordered pair once
// ---------------------------------------------------------------------------

// Wave sum of 8 values per lane, scattered: afterwards lane l holds the sum
// over all 64 lanes of value vi(l) = 4 b5 + 2 b4 + b3 (bits of l); the 8
// lanes that differ only in bits 0-2 hold the same value.  Fixed butterfly
// (10 shuffles), so the result does not depend on timing.
__device__ __forceinline__ double shx(double v, int m) { return __shfl_xor(v, m); }
__device__ __forceinline__ double2 shx(double2 v, int m) { return make_double2(__shfl_xor(v.x, m), __shfl_xor(v.y, m)); }
__device__ __forceinline__ double shl(double v, int s) { return __shfl(v, s); }
__device__ __forceinline__ double2 shl(double2 v, int s) { return make_double2(__shfl(v.x, s), __shfl(v.y, s)); }

constexpr int RS_NV = 8;

template <typename T>
__device__ __forceinline__ T reduce_scatter8(const T (&col)[RS_NV], int lane)
{
    T w4[4], w2[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
#pragma unroll
    for (int v = 0; v < 4; v++) w4[v] = sc_add(h5 ? col[v + 4] : col[v], shx(h5 ? col[v] : col[v + 4], 32));
#pragma unroll
    for (int v = 0; v < 2; v++) w2[v] = sc_add(h4 ? w4[v + 2] : w4[v], shx(h4 ? w4[v] : w4[v + 2], 16));
    T w = sc_add(h3 ? w2[1] : w2[0], shx(h3 ? w2[0] : w2[1], 8));
    w = sc_add(w, shx(w, 4));
    w = sc_add(w, shx(w, 2));
    return sc_add(w, shx(w, 1));
}

__device__ __forceinline__ int rs_value_of_lane(int l) { return ((l >> 5) & 1) * 4 + ((l >> 4) & 1) * 2 + ((l >> 3) & 1); }
__device__ __forceinline__ int rs_lane_of_value(int v) { return ((v >> 2) & 1) << 5 | ((v >> 1) & 1) << 4 | (v & 1) << 3; }

// One wave = block a (64 consecutive members) of a group with k >= 64
// members.  It visits the partners in blocks b >= a (strictly later members
// inside block a), evaluates H_ij once per unordered pair, adds H_ij c_j to
// the row sum of i, and sums H_ji c_i = conj(H_ij) c_i over its lanes: for
// b == a the sum goes to the lane holding j, for b > a it is written to the
// column-partial slot of (a, j) that the gather adds to j's determinant.
template <bool CPLX, int RC>
__device__ __forceinline__ void group_double_half(const DevPlan &p, uint32_t mfirst, uint32_t mend, int lane, int R,
                                                  int r0, const typename Scal<CPLX>::T *__restrict__ c,
                                                  typename Scal<CPLX>::T *__restrict__ partial)
{
    using T = typename Scal<CPLX>::T;
    constexpr int JS = RS_NV / RC;         // partners per reduction pass (all loaded at once)
    const uint32_t g = p.mem_grp[mfirst];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint32_t k = j1 - j0;
    const uint32_t a = (mfirst - j0) >> 6;
    const uint8_t type = p.grp_type[g];
    const uint32_t m = mfirst + lane;
    const bool act = m < mend;
    const uint2 me = p.mem[act ? m : mfirst];
    // where this member's row partial goes (loaded now, used at the end)
    const uint32_t mpos = act ? p.slot_pos[m] : 0u;
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    const uint32_t negi = (me.y >> 16) & 1;
    const bool lay = (me.y >> 17) & 1;
    const DoubleIndex di = double_index<CPLX>(p, type, Xi, Yi, lay);
    const T *tab = (const T *)((!CPLX && type == G_AB) ? p.g_ab : (lay ? p.a_pair1 : p.a_pair));
    const int nr = min(RC, R - r0);
    // acc: row sum in partner order; dacc: the one column sum delivered from
    // the member's own block, added at the end so that the result does not
    // depend on how partners are batched into passes
    T ci[RC], acc[RC], dacc[RC];
#pragma unroll
    for (int kk = 0; kk < RC; kk++) {
        ci[kk] = act ? c[(size_t)me.x * R + r0 + (kk < nr ? kk : 0)] : sc_zero(T());
        acc[kk] = sc_zero(T());
        dacc[kk] = sc_zero(T());
    }
    const size_t colbase = (size_t)p.nmem + p.grp_col[g] + (size_t)a * k - 32 * (size_t)a * (a + 1);
    // passes of JS partners over the blocks b >= a (64 is a multiple of JS,
    // so a pass never straddles two blocks), from the group's last pass down:
    // since 64 is a multiple of JS, every block of the group starts at the
    // same pass and the blocks walk the same partners at about the same
    // time, so the partner records and coefficients one block reads are in
    // L2 for the others (spinor sigma 11.5 -> 11.2 ms).  The partner records
    // of the next pass (wave-uniform) are loaded while this pass runs.
    const uint32_t jfirst = j0 + 64 * a;
    const uint32_t jlast = jfirst + (j1 - 1 - jfirst) / JS * JS;  // start of the last pass
    uint2 onext[JS];
#pragma unroll
    for (int u = 0; u < JS; u++) onext[u] = p.mem[min(jlast + u, j1 - 1)];
    // one pass over partners jj .. jj + JS - 1 per iteration, loading the
    // records of the pass starting at jnext meanwhile (the body stays inside
    // the loop: as a lambda it spilled scalar registers)
    for (uint32_t jj = jlast + JS; jj > jfirst;) {
        jj -= JS;
        const uint32_t jnext = jj > jfirst ? jj - JS : jj;
        const uint32_t b = (jj - j0) >> 6;
        const uint32_t jb0 = j0 + 64 * b, jb1 = min(j1, jb0 + 64);
        // position of the column partial this lane writes at the end of the
        // pass (b > a), loaded before the pass's partner loads
        uint32_t cpos = 0;
        if (b > a && (lane & 7) == 0) {
            const int vi = rs_value_of_lane(lane);
            const uint32_t j = jj + vi / RC;
            if (j < jb1 && vi % RC < nr) cpos = p.slot_pos[colbase + (j - j0) - 64 * (a + 1)];
        }
        {
            T col[RS_NV];
            {
                uint2 o[JS];
                bool hit[JS];
                T v[JS];
                T cj[JS][RC];
#pragma unroll
                for (int u = 0; u < JS; u++) {
                    o[u] = onext[u];
                    onext[u] = p.mem[min(jnext + u, j1 - 1)];
                }
#pragma unroll
                for (int u = 0; u < JS; u++) {
                    const uint32_t j = jj + u;
                    const bool in = act && j < jb1 && (b > a || j > m);
                    const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
                    hit[u] = in && !(Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi);
                    v[u] = tab[hit[u] ? di.at(Xj, Yj) : 0u];
                    const T *cr = c + (size_t)(hit[u] ? o[u].x : 0) * R + r0;
#pragma unroll
                    for (int kk = 0; kk < RC; kk++) cj[u][kk] = cr[kk < nr ? kk : 0];
                }
#pragma unroll
                for (int u = 0; u < JS; u++) {
                    T x = sc_neg(CPLX ? sc_conj(v[u]) : v[u], (negi ^ ((o[u].y >> 16) & 1)) != 0);
                    if (!hit[u]) x = sc_zero(T());
                    const T xh = CPLX ? sc_conj(x) : x;
#pragma unroll
                    for (int kk = 0; kk < RC; kk++) {
                        acc[kk] = sc_add(acc[kk], sc_mul(x, cj[u][kk]));
                        col[u * RC + kk] = sc_mul(xh, ci[kk]);
                    }
                }
            }
            const T s = reduce_scatter8(col, lane);
            if (b == a) {
                // members jj .. jj+JS-1 live in lanes jj-jb0 .. of this wave
                const int t0 = (int)(jj - jb0);
                const bool tgt = lane >= t0 && lane < t0 + JS;
#pragma unroll
                for (int kk = 0; kk < RC; kk++) {
                    const int vi = (tgt ? lane - t0 : 0) * RC + kk;
                    const T got = shl(s, rs_lane_of_value(vi));
                    if (tgt && kk < nr) dacc[kk] = got;
                }
            } else if ((lane & 7) == 0) {
                const int vi = rs_value_of_lane(lane);
                const uint32_t j = jj + vi / RC;
                const int kk = vi % RC;
                if (j < jb1 && kk < nr) store_partial(s, &partial[(size_t)cpos * R + r0 + kk]);
            }
        }
    }
    if (act) {
        T *out = partial + (size_t)mpos * R + r0;
#pragma unroll
        for (int kk = 0; kk < RC; kk++)
            if (kk < nr) store_partial(sc_add(acc[kk], dacc[kk]), &out[kk]);
    }
}

template <bool CPLX, int RC, int U>
__device__ __forceinline__ void group_double_body(const DevPlan &p, int64_t wave, int lane, int R, int r0,
                                                  const typename Scal<CPLX>::T *__restrict__ c,
                                                  typename Scal<CPLX>::T *__restrict__ partial)
{
    using T = typename Scal<CPLX>::T;
    const uint32_t mfirst = p.pk_off[wave], mend = p.pk_off[wave + 1];
    // a packet of a large group is one 64-member block of it (uniform); its
    // members carry 0 as group size.  Every root-chunk width (1, 2 or 4
    // roots per pass) takes the Hermitian half-work on large groups.
    if (((p.mem[mfirst].y >> 24) & 63) == 0) {
        group_double_half<CPLX, RC>(p, mfirst, mend, lane, R, r0, c, partial);
        return;
    }
    // small groups: the packet holds whole groups in decreasing size, so a
    // member's partners are other lanes of this wave (their records come by
    // shuffles) and the first group is the largest: every lane runs that
    // many partner steps, so the shuffles see the whole wave
    const uint32_t kmax = (p.mem[mfirst].y >> 24) & 63;
    const uint32_t m = mfirst + lane;
    const bool live = m < mend;
    const uint2 me = p.mem[live ? m : mfirst];
    const uint32_t mpos = live ? p.slot_pos[m] : 0u;
    const uint32_t kk = live ? (me.y >> 24) & 63 : 0u;  // partners of this lane: steps [0, kk)
    const int lane0 = lane - (int)((me.y >> 18) & 63);  // lane of its group's first member
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    // the group kind follows from the added positions (two alpha, two beta
    // or one of each)
    const int n_ = p.n;
    const uint8_t type = CPLX ? (uint8_t)G_DOUBLE_S
                              : (uint8_t)((Xi < n_ && Yi < n_) ? G_AA : (Xi >= n_ && Yi >= n_) ? G_BB : G_AB);
    const uint32_t negi = (me.y >> 16) & 1;
    const bool lay = (me.y >> 17) & 1;
    const DoubleIndex di = double_index<CPLX>(p, type, Xi, Yi, lay);
    const T *tab = (const T *)((!CPLX && type == G_AB) ? p.g_ab : (lay ? p.a_pair1 : p.a_pair));
    T acc[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) acc[k] = sc_zero(T());
    const int nr = min(RC, R - r0);
    for (uint32_t t = 0; t < kmax; t += U) {
        uint2 o[U];
        bool hit[U];
        // all partner records first, then coefficients and integrals
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int src = t + u < kk ? lane0 + (int)(t + u) : lane;
            o[u].x = (uint32_t)__shfl((int)me.x, src);
            o[u].y = (uint32_t)__shfl((int)me.y, src);
        }
        T v[U];
        T cj[U][RC];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const T *cr = c + (size_t)o[u].x * R + r0;
#pragma unroll
            for (int k = 0; k < RC; k++) cj[u][k] = cr[k < nr ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
            hit[u] = t + u < kk && !(Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi);
            v[u] = tab[hit[u] ? di.at(Xj, Yj) : 0u];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!hit[u]) continue;
            T x = sc_neg(CPLX ? sc_conj(v[u]) : v[u], (negi ^ ((o[u].y >> 16) & 1)) != 0);
#pragma unroll
            for (int k = 0; k < RC; k++) acc[k] = sc_add(acc[k], sc_mul(x, cj[u][k]));
        }
    }
    if (!live) return;
    T *out = partial + (size_t)mpos * R + r0;
#pragma unroll
    for (int k = 0; k < RC; k++)
        if (k < nr) store_partial(acc[k], &out[k]);
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

// Gather launches: each XCD takes one contiguous eighth of the logical
// blocks (grid a multiple of 8), so determinants that are neighbours in the
// given order, whose partial sums the plan places close together, share an L2.
__device__ __forceinline__ int64_t xcd_range_block(int64_t b, int64_t grid)
{
    return (b & 7) * (grid >> 3) + (b >> 3);
}

// Real one-root launches fit six waves per SIMD in 80 registers without
// spilling (measured faster than the five the compiler picks by itself).
template <bool CPLX, int RC, int U>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((!CPLX && RC == 1 && U <= 8) ? 6 : 1))) void k_group_double(DevPlan p, int R, int r0,
                                                      const typename Scal<CPLX>::T *__restrict__ c,
                                                      typename Scal<CPLX>::T *__restrict__ partial)
{
    // wave-uniform packet index, kept in a scalar register
    const int64_t wave = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(xcd_block(blockIdx.x) * 4 + (threadIdx.x >> 6)));
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
    const uint32_t mfirst = p.pk_off[wave], mend = p.pk_off[wave + 1];
    const uint32_t m = mfirst + lane;
    const uint32_t mpos = m < mend ? p.slot_pos[m] : 0u;
    T acc[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) acc[k] = sc_zero(T());
    const int nr = min(RC, R - r0);
    // size of the packet's first (largest) group; 0 marks a large group
    const uint32_t kmax = (p.mem[mfirst].y >> 24) & 63;
    if (kmax == 0) {
        // a block of a large group: group tables, partner records from memory
        if (m >= mend) return;
        const uint32_t g = p.mem_grp[m];
        const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
        const uint8_t type = p.grp_type[g];
        const uint2 me = p.mem[m];
        const int Xi = me.y & 255;
        const uint32_t negi = (me.y >> 16) & 1;
        const uint64_t k0 = p.grp_key[2 * g], k1 = p.grp_key[2 * g + 1];
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
    } else {
        // whole small groups in decreasing size: partners are lanes of this
        // wave (records by shuffles), K is the member's determinant without
        // its added position, the kind follows from that position
        const bool live = m < mend;
        const uint2 me = p.mem[live ? m : mfirst];
        const uint32_t kk = live ? (me.y >> 24) & 63 : 0u;
        const int lane0 = lane - (int)((me.y >> 18) & 63);
        const int Xi = me.y & 255;
        const uint32_t negi = (me.y >> 16) & 1;
        const int n = p.n;
        uint64_t k0 = p.dets[2 * (size_t)me.x], k1 = p.dets[2 * (size_t)me.x + 1];
        if (Xi < n) k0 &= ~(1ULL << Xi);
        else k1 &= ~(1ULL << (Xi - n));
        const uint8_t type = CPLX ? (uint8_t)G_SINGLE_S : (uint8_t)(Xi < n ? G_SINGLE_A : G_SINGLE_B);
        for (uint32_t t = 0; t < kmax; t++) {
            const int src = t < kk ? lane0 + (int)t : lane;
            const uint32_t ox = (uint32_t)__shfl((int)me.x, src), oy = (uint32_t)__shfl((int)me.y, src);
            const int Xj = oy & 255;
            if (t >= kk || Xj == Xi) continue;
            T v = single_element<CPLX>(p, type, k0, k1, Xi, Xj);
            v = sc_neg(v, (negi ^ ((oy >> 16) & 1)) != 0);
            const T *cj = c + (size_t)ox * R + r0;
#pragma unroll
            for (int k = 0; k < RC; k++)
                if (k < nr) acc[k] = sc_add(acc[k], sc_mul(v, cj[k]));
        }
        if (!live) return;
    }
    T *out = partial + (size_t)mpos * R + r0;
#pragma unroll
    for (int k = 0; k < RC; k++)
        if (k < nr) store_partial(acc[k], &out[k]);
}

template <bool CPLX, int RC>
__global__ __launch_bounds__(256) void k_group_single(DevPlan p, int R, int r0,
                                                      const typename Scal<CPLX>::T *__restrict__ c,
                                                      typename Scal<CPLX>::T *__restrict__ partial)
{
    const int64_t wave =
        p.npacket_double + (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
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
        const uint64_t s0 = p.rowptr[I], s1 = p.rowptr[I + 1];
        // eight slots in flight per lane: all eight positions are loaded,
        // then all eight partials, so a determinant of up to 8 GL slots
        // costs two dependent memory round trips after its row pointer; the
        // additions keep the slot order (a slot past the end adds nothing)
        constexpr int W = 8;
        for (uint64_t s = s0 + sub; s < s1; s += W * GL) {
            uint32_t ix[W];
            T v[W];
#pragma unroll
            for (int j = 0; j < W; j++) ix[j] = s + (uint64_t)j * GL < s1 ? p.slot_mem[s + (uint64_t)j * GL] : 0u;
#pragma unroll
            for (int j = 0; j < W; j++)
                v[j] = s + (uint64_t)j * GL < s1 ? partial[(size_t)ix[j] * R + k] : sc_zero(T());
#pragma unroll
            for (int j = 0; j < W; j++)
                if (s + (uint64_t)j * GL < s1) acc = sc_add(acc, v[j]);
        }
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
                                                typename Scal<CPLX>::T *__restrict__ sigma, int64_t base)
{
    gather_body<CPLX, GL>(p, base + xcd_range_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x, R, c, partial,
                          sigma);
}

template <bool CPLX, int RC, int U>
static void launch_double(const DevPlan &p, int R, int r0, const typename Scal<CPLX>::T *c,
                          typename Scal<CPLX>::T *part, hipStream_t s)
{
    unsigned grid = xcd_grid((p.npacket_double + 3) / 4);
    hipLaunchKernelGGL((k_group_double<CPLX, RC, U>), dim3(grid), dim3(256), 0, s, p, R, r0, c, part);
}

template <bool CPLX, int RC>
static void launch_double_groups(const DevPlan &p, int R, int r0, const typename Scal<CPLX>::T *c,
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
}

template <bool CPLX, int RC>
static void launch_single_groups(const DevPlan &p, int R, int r0, const typename Scal<CPLX>::T *c,
                                 typename Scal<CPLX>::T *part, hipStream_t s)
{
    const int64_t ns = p.npacket - p.npacket_double;
    if (ns > 0) {
        ProfToken t = prof_begin("group_single", s);
        unsigned grid = (unsigned)((ns + 3) / 4);
        hipLaunchKernelGGL((k_group_single<CPLX, RC>), dim3(grid), dim3(256), 0, s, p, R, r0, c, part);
        prof_end(t, s);
    }
}

template <bool CPLX, bool DBL>
static void launch_chunks(const DevPlan &p, int R, const typename Scal<CPLX>::T *c, typename Scal<CPLX>::T *part,
                          hipStream_t s)
{
    for (int r0 = 0; r0 < R; r0 += 4) {
        const int left = R - r0;
        if constexpr (DBL) {
            if (left == 1) launch_double_groups<CPLX, 1>(p, R, r0, c, part, s);
            else if (left == 2) launch_double_groups<CPLX, 2>(p, R, r0, c, part, s);
            else launch_double_groups<CPLX, 4>(p, R, r0, c, part, s);
        } else {
            if (left == 1) launch_single_groups<CPLX, 1>(p, R, r0, c, part, s);
            else if (left == 2) launch_single_groups<CPLX, 2>(p, R, r0, c, part, s);
            else launch_single_groups<CPLX, 4>(p, R, r0, c, part, s);
        }
    }
}

// A second stream per device for the single-group kernels: they write
// other partial sums than the double-group kernel, so the two run side by
// side (the singles fill the compute units the memory-bound double kernel
// leaves idle, and its tail) and are joined before the gather.  The fork
// and join are enqueued under one lock (the events are shared); a caller
// stream that is being captured into a graph gets the serial order instead,
// so the side stream never becomes part of a capture.
namespace {
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool failed = false;
};
std::mutex g_side_mu;
SideStream g_side[64];

SideStream *side_stream_locked()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    SideStream &x = g_side[dev];
    if (!x.s && !x.failed) {
        if (hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&x.join, hipEventDisableTiming) != hipSuccess) {
            x.failed = true;
            x.s = nullptr;
        }
    }
    return x.s ? &x : nullptr;
}
}  // namespace

hipStream_t device_side_stream()
{
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStream *x = side_stream_locked();
    return x ? x->s : nullptr;
}

template <bool CPLX, int GL>
static void launch_gather(const DevPlan &p, int R, const typename Scal<CPLX>::T *c,
                          const typename Scal<CPLX>::T *part, typename Scal<CPLX>::T *sigma, hipStream_t s)
{
    // a dispatch counts its work-items in 32 bits: at most 2^22 blocks each.
    // Only the last chunk is partial; its grid is rounded up to a multiple of
    // 8 and the extra blocks lie past the end (inactive).
    const int64_t tot = p.ndet * R * GL, chunk = (int64_t)256 << 22;
    for (int64_t b = 0; b < tot; b += chunk) {
        const int64_t n = std::min<int64_t>(chunk, tot - b);
        hipLaunchKernelGGL((k_gather<CPLX, GL>), dim3((unsigned)((n + 2047) / 2048 * 8)), dim3(256), 0, s, p, R, c,
                           part, sigma, b);
    }
}

template <bool CPLX>
static mw_status sigma_t(const DevPlan &p, int R, const void *c, void *sigma, hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    const T *cc = (const T *)c;
    T *part = (T *)p.partial;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool both = p.npacket_double > 0 && p.npacket > p.npacket_double;
    if (both && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
        std::lock_guard<std::mutex> lk(g_side_mu);
        SideStream *x = side_stream_locked();
        if (x && hipEventRecord(x->fork, s) == hipSuccess && hipStreamWaitEvent(x->s, x->fork, 0) == hipSuccess) {
            launch_chunks<CPLX, false>(p, R, cc, part, x->s);
            launch_chunks<CPLX, true>(p, R, cc, part, s);
            if (hipEventRecord(x->join, x->s) != hipSuccess || hipStreamWaitEvent(s, x->join, 0) != hipSuccess)
                return fail(MW_EHIP, "joining the single-group stream failed");
        } else {
            launch_chunks<CPLX, true>(p, R, cc, part, s);
            launch_chunks<CPLX, false>(p, R, cc, part, s);
        }
    } else {
        launch_chunks<CPLX, true>(p, R, cc, part, s);
        launch_chunks<CPLX, false>(p, R, cc, part, s);
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
// One launch per root-chunk width (4, 2 or 1 roots per pass, the widths
// the plain launches use, so that both give identical bits); each launch
// only visits the problems that have a chunk of its width, and has its own
// register budget.
template <bool CPLX, int RC, int U>
__global__ __launch_bounds__(256) void k_batched_groups(BatchArgs a)
{
    using T = typename Scal<CPLX>::T;
    const int lane = threadIdx.x & 63;
    const int64_t total = a.pk_start[a.nprob];
    // Work queue per XCD (block b runs on XCD b % 8): the packet sequence is
    // cut into chunks of CHUNK packets, and runs of SUPER chunks (the
    // packets of the same 64 x 16 members as one XCD slice of the plain
    // launch) belong to XCD (run index) % 8, so the packets of one group
    // meet in one L2.  A wave claims the next chunk of its own XCD; when
    // that queue is empty it takes chunks from the others.  All counters
    // start at zero.
    constexpr uint32_t CHUNK = 16, SUPER = 4;
    const int64_t nchunk = (total + CHUNK - 1) / CHUNK;
    const int home = blockIdx.x & 7;
    for (int qi = 0; qi < 8; qi++) {
        const int xq = (home + qi) & 7;
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.counter[xq], 1u);
            t = __builtin_amdgcn_readfirstlane(t);
            const int64_t ch = ((int64_t)(t / SUPER) * 8 + xq) * SUPER + t % SUPER;
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
                    const int left = R - r0;
                    if ((left == 1 ? 1 : (left == 2 ? 2 : 4)) != RC) continue;
                    if (w < p.npacket_double) group_double_body<CPLX, RC, U>(p, w, lane, R, r0, c, part);
                    else group_single_body<CPLX, RC>(p, w, lane, R, r0, c, part);
                }
            }
        }
    }
}

// Flat variant: one wave per packet over the packets of every problem
// (hardware-dispatched, with the same XCD-aware block order as the plain
// launches), the double-group and the single-group packets in launches of
// their own (each with its own register budget, as the plain launches);
// the tuner picks it or the work queue above.
template <bool CPLX, int RC, int U, bool SGL, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_batched_flat(BatchArgs a)
{
    using T = typename Scal<CPLX>::T;
    const int64_t *pre = SGL ? a.pks_start : a.pkd_start;
    const int64_t u = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(xcd_block(blockIdx.x) * 4 + (threadIdx.x >> 6)));
    if (u >= pre[a.nprob]) return;
    const int lane = threadIdx.x & 63;
    int q = 0;
    while (u >= pre[q + 1]) q++;
    const DevPlan &p = *a.plans[q];
    const int64_t w = (SGL ? p.npacket_double : 0) + (u - pre[q]);
    const int R = a.R[q];
    const T *c = (const T *)a.c[q];
    T *part = (T *)p.partial;
    for (int r0 = 0; r0 < R; r0 += 4) {
        const int left = R - r0;
        if ((left == 1 ? 1 : (left == 2 ? 2 : 4)) != RC) continue;
        if constexpr (SGL) group_single_body<CPLX, RC>(p, w, lane, R, r0, c, part);
        else group_double_body<CPLX, RC, U>(p, w, lane, R, r0, c, part);
    }
}

// Gather for all problems: block b belongs to the problem whose block range
// holds b (block-uniform, so the plan fields are scalar loads).
template <bool CPLX, int GL>
__global__ __launch_bounds__(256) void k_batched_gather(BatchArgs a)
{
    using T = typename Scal<CPLX>::T;
    const int64_t b = xcd_range_block(blockIdx.x, gridDim.x);
    if (b >= a.blk_start[a.nprob]) return;
    int q = 0;
    while (b >= a.blk_start[q + 1]) q++;
    const DevPlan &p = *a.plans[q];
    const int64_t local = (b - a.blk_start[q]) * blockDim.x + threadIdx.x;
    gather_body<CPLX, GL>(p, local, a.R[q], (const T *)a.c[q], (const T *)p.partial, (T *)a.sigma[q]);
}

__global__ void k_reset_counter(uint32_t *ctr)
{
    if (threadIdx.x < 8 * 3) ctr[threadIdx.x] = 0u;
}

// WAVES: minimum waves per SIMD the register allocation must allow (the
// plain launches of the same bodies reach it; the batched bookkeeping
// would otherwise cost a wave)
template <bool CPLX, int RC, int U, int WAVES>
static void launch_flat_class(const BatchArgs &a, hipStream_t s)
{
    const int64_t nd = a.pkd_start[a.nprob], ns = a.pks_start[a.nprob];
    if (nd > 0)
        hipLaunchKernelGGL((k_batched_flat<CPLX, RC, U, false, WAVES>), dim3(xcd_grid((nd + 3) / 4)), dim3(256), 0, s, a);
    if (ns > 0)
        hipLaunchKernelGGL((k_batched_flat<CPLX, RC, U, true, 1>), dim3(xcd_grid((ns + 3) / 4)), dim3(256), 0, s, a);
}

template <bool CPLX>
static void launch_batched_flat(const BatchSet &b, hipStream_t s)
{
    if (b.cls[0].nprob) {
        if (b.u4 == 8) launch_flat_class<CPLX, 4, 8, CPLX ? 2 : 3>(b.cls[0], s);
        else launch_flat_class<CPLX, 4, 4, CPLX ? 3 : 5>(b.cls[0], s);
    }
    if (b.cls[1].nprob) launch_flat_class<CPLX, 2, 8, CPLX ? 3 : 5>(b.cls[1], s);
    if (b.cls[2].nprob) launch_flat_class<CPLX, 1, 8, CPLX ? 3 : 5>(b.cls[2], s);
}

template <bool CPLX>
static void launch_batched_groups(const BatchSet &b, int blocks, hipStream_t s)
{
    if (blocks <= 0) {
        launch_batched_flat<CPLX>(b, s);
        return;
    }
    // four-root chunks: partner unroll 4 or 8 (tuned; registers vs loads in flight)
    if (b.cls[0].nprob) {
        if (b.u4 == 8) hipLaunchKernelGGL((k_batched_groups<CPLX, 4, 8>), dim3(blocks), dim3(256), 0, s, b.cls[0]);
        else hipLaunchKernelGGL((k_batched_groups<CPLX, 4, 4>), dim3(blocks), dim3(256), 0, s, b.cls[0]);
    }
    if (b.cls[1].nprob) hipLaunchKernelGGL((k_batched_groups<CPLX, 2, 8>), dim3(blocks), dim3(256), 0, s, b.cls[1]);
    if (b.cls[2].nprob) hipLaunchKernelGGL((k_batched_groups<CPLX, 1, 8>), dim3(blocks), dim3(256), 0, s, b.cls[2]);
}

mw_status launch_batched(const BatchSet &b, bool cplx, int blocks, hipStream_t s, bool timing)
{
    const BatchArgs &a = b.all;
    if (a.nprob == 0) return MW_OK;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, a.counter);
    ProfToken t = timing ? prof_begin("batched_groups", s) : ProfToken{nullptr, nullptr, ""};
    if (cplx) launch_batched_groups<true>(b, blocks, s);
    else launch_batched_groups<false>(b, blocks, s);
    prof_end(t, s);
    if (timing) t = prof_begin("batched_gather", s);
    // gather lanes per determinant: the width blk_start was laid out for
    const unsigned gg = (unsigned)((a.blk_start[a.nprob] + 7) / 8 * 8);
    if (b.gl == 8) {
        if (cplx) hipLaunchKernelGGL((k_batched_gather<true, 8>), dim3(gg), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_batched_gather<false, 8>), dim3(gg), dim3(256), 0, s, a);
    } else if (b.gl == 32) {
        if (cplx) hipLaunchKernelGGL((k_batched_gather<true, 32>), dim3(gg), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_batched_gather<false, 32>), dim3(gg), dim3(256), 0, s, a);
    } else {
        if (cplx) hipLaunchKernelGGL((k_batched_gather<true, 16>), dim3(gg), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_batched_gather<false, 16>), dim3(gg), dim3(256), 0, s, a);
    }
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
