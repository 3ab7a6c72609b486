// Transition one- and two-particle density matrices: the adjoint of sigma
// with respect to the integrals (E = sum h gamma + 1/2 sum g Gamma for the
// Hamiltonian of section 2.1).  The connectivity is recomputed from the same
// groups as sigma, never stored.
//
// Every ordered pair (I, J) connected inside a group contributes
// w_IJ = phi_I phi_J sum_k w_k conj(bra_Ik) ket_Jk:
//  double group, I adds (P<R), J adds (Q<S):  Gamma_PQRS += w, Gamma_RSPQ += w,
//      Gamma_PSRQ -= w, Gamma_RQPS -= w.  One device atomic per pair goes to
//      an accumulator (spin-free alpha-beta: a full [n]^4 array G_ab; same
//      spin and spinor: the antisymmetric pair matrix D[(P,R)][(Q,S)]); a
//      final pass expands it into Gamma.
//  single group, I adds P, J adds Q (K the common N-1 string):
//      gamma_PQ += w and, for every X in K, Gamma_PQXX += w, Gamma_XXPQ += w,
//      Gamma_PXXQ -= w, Gamma_XQPX -= w (spin-free: the exchange-like two
//      only for X of the spin of P).  The sum over K is split into the
//      reference string omega (applied once at the end through the
//      accumulated S_PQ = sum of w) plus the few positions where K and omega
//      differ (direct atomics into compact C and E arrays, spread over
//      copies that are folded before the final pass).
//  diagonal I = J: gamma_PP += w, Gamma_PPRR += w, Gamma_PRRP -= w (P != R),
//      from the occupation correlations of every determinant.
//  One vector as bra and ket: each unordered pair once; the final pass adds
//  the mirror image (the reversed pair's weight is the conjugate).
#include <hip/hip_runtime.h>

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

// same XCD-aware block order as the sigma kernels
__device__ __forceinline__ int64_t xcd_block_r(int64_t b)
{
    const int64_t x = b & 7, r = b >> 3;
    return ((r / 16) * 8 + x) * 16 + (r % 16);
}
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

// Double pairs.  The accumulators are laid out like the integral tables of
// sigma (row from the partner j, column from the member i) and use the same
// per-member layout bit, so the 64 lanes of a wave add into a run of
// neighbouring entries.  Alpha-beta: D_ab[q][s][p][r] holds G(p,q,r,s) =
// sum of w over pairs with i adding (p alpha, r beta) and j adding (q, s);
// layout-1 lanes add into D_ab[s][q][r][p], i.e. G(r,s,p,q), which changes
// nothing because Gamma only needs G(p,q,r,s) + G(r,s,p,q).  Pair
// accumulators DT0 (colex columns) and DT1 (lex columns) hold the
// transposed antisymmetric pair matrix, D[(P,R)][(Q,S)] = DT0[QS][PR] +
// DT1[QS][lex PR].
// SYM (bra and ket are one vector): the reversed pair (J, I) adds the
// complex conjugate of w_IJ to the mirrored entry, so each unordered pair is
// visited once (partners j after i in the group) and the final pass adds
// the mirror image.
template <bool CPLX, int U, bool SYM>
__global__ __launch_bounds__(256) void k_rdm_double(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                    const typename Scal<CPLX>::T *__restrict__ ket, RdmWeights W,
                                                    double *__restrict__ dab, typename Scal<CPLX>::T *__restrict__ dt0,
                                                    typename Scal<CPLX>::T *__restrict__ dt1)
{
    using T = typename Scal<CPLX>::T;
    const int64_t wave = xcd_block_r(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= p.npacket_double) return;
    const uint32_t m = p.pk_off[wave] + lane;
    if (m >= p.pk_off[wave + 1]) return;
    const uint32_t g = p.mem_grp[m];
    const uint32_t j0 = p.grp_off[g], j1 = p.grp_off[g + 1];
    const uint8_t type = p.grp_type[g];
    const uint2 me = p.mem[m];
    const int Xi = me.y & 255, Yi = (me.y >> 8) & 255;
    const uint32_t negi = (me.y >> 16) & 1;
    const bool lay = (me.y >> 17) & 1;
    const int n = p.n;
    const bool ab = !CPLX && type == G_AB;
    const int off = (!CPLX && type == G_BB) ? n : 0;
    const int mpos = CPLX ? p.M : n;
    size_t col;
    if (ab) col = lay ? (size_t)(Yi - n) * n + Xi : (size_t)Xi * n + (Yi - n);
    else col = lay ? (size_t)rdm_pair_lex(Xi - off, Yi - off, mpos) : (size_t)pair_idx(Xi - off, Yi - off);
    T *dst_pair = lay ? dt1 : dt0;
    // SYM: a large group's blocks before this packet hold no later partner
    const uint32_t js = SYM ? max(j0, p.pk_off[wave]) : j0;
    for (uint32_t j = js; j < j1; j += U) {
        uint2 o[U];
        bool hit[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool in = j + u < j1 && (!SYM || j + u > m);
            o[u] = p.mem[in ? j + u : j0];
            const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
            hit[u] = in && !(Xj == Xi || Xj == Yi || Yj == Xi || Yj == Yi);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!hit[u]) continue;
            const int Xj = o[u].y & 255, Yj = (o[u].y >> 8) & 255;
            T w = pair_weight<CPLX>(bra, ket, R, me.x, o[u].x, W);
            w = sc_neg(w, (negi ^ ((o[u].y >> 16) & 1)) != 0);
            if constexpr (!CPLX) {
                if (ab) {
                    const size_t row = lay ? (size_t)(Yj - n) * n + Xj : (size_t)Xj * n + (Yj - n);
                    atomicAdd(&dab[row * n * n + col], w);
                    continue;
                }
            }
            atom_add(&dst_pair[(size_t)pair_idx(Xj - off, Yj - off) * p.npair + col], w);
        }
    }
}

// The contributions of one single pair (member i with det me.x adding
// position Xi, partner with record o adding Xj; K the group's string).
template <bool CPLX>
__device__ __forceinline__ void rdm_single_pair(const DevPlan &p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                const typename Scal<CPLX>::T *__restrict__ ket, const RdmWeights &W,
                                                typename Scal<CPLX>::T *__restrict__ S,
                                                typename Scal<CPLX>::T *__restrict__ Cc, double *__restrict__ Ee,
                                                uint8_t type, uint64_t k0, uint64_t k1, uint2 me, int Xi, uint32_t negi,
                                                uint2 o)
{
    using T = typename Scal<CPLX>::T;
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
        atomicAdd(&S[((size_t)s * n + qq) * n + pp], w);
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
                atomicAdd(&Cq[(size_t)xx * n], sw);
                if (same) atomicAdd(&Eq[(size_t)xx * n], sw);
            }
        }
    } else {
        const int M = p.M;
        atom_add(&S[(size_t)Xj * M + Xi], w);
        // C[Q][X][P] (M^3, P innermost) collects the four terms of every X
        T *Cq = Cc + (size_t)Xj * M * M + Xi;
        for (int part = 0; part < 4; part++) {
            const uint64_t kw = (part < 2) ? k0 : k1;
            const uint64_t rw = (part < 2) ? p.ref0 : p.ref1;
            const int base = (part < 2) ? 0 : n;
            const uint64_t bits = (part & 1) ? (rw & ~kw) : (kw & ~rw);
            const T sw = sc_neg(w, (part & 1) != 0);
            for (uint64_t x = bits; x; x &= x - 1) atom_add(&Cq[(size_t)(base + __builtin_ctzll(x)) * M], sw);
        }
    }
}

template <bool CPLX, bool SYM>
__global__ __launch_bounds__(256) void k_rdm_single(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                    const typename Scal<CPLX>::T *__restrict__ ket, RdmWeights W,
                                                    typename Scal<CPLX>::T *__restrict__ S,
                                                    typename Scal<CPLX>::T *__restrict__ Cc,
                                                    double *__restrict__ Ee, int64_t copy_stride)
{
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
            rdm_single_pair<CPLX>(p, R, bra, ket, W, S, Cc, Ee, type, k0, k1, me, Xi, negi, o);
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
        rdm_single_pair<CPLX>(p, R, bra, ket, W, S, Cc, Ee, type, k0, k1, me, Xi, negi, o);
    }
}

// Diagonal terms: with w_I = sum_k w_k conj(bra_Ik) ket_Ik, the occupation
// correlation D[A][B] = sum_I w_I n_A(I) n_B(I) over global positions gives
// gamma_AA = D[A][A] and the diagonal parts of Gamma (Gamma_AABB += D[A][B],
// Gamma_ABBA -= D[A][B] for A != B; spin-free: summed over spins, the
// exchange-like part for equal spins only).  One partial matrix per
// determinant chunk, reduced in a fixed order.
constexpr int RDM_OCC_CHUNKS = 256;

// Block (x, y) of 1024 threads adds w_I into an LDS copy of rows
// [A0, A0 + ROWS) of D for every determinant of chunk x, each lane holding
// B = lane, lane + 64 and the wave walking the occupied A of the
// determinant (LDS atomics: the 16 waves take different determinants); then
// it writes its rows of the chunk's partial matrix.
template <bool CPLX>
__global__ __launch_bounds__(1024) void k_rdm_occ_lds(DevPlan p, int R, const typename Scal<CPLX>::T *__restrict__ bra,
                                                      const typename Scal<CPLX>::T *__restrict__ ket, RdmWeights W,
                                                      typename Scal<CPLX>::T *__restrict__ part)
{
    using T = typename Scal<CPLX>::T;
    constexpr int ROWS = CPLX ? 64 : 128;  // 128 KB of LDS
    __shared__ T ds[ROWS * 128];
    const int n = p.n, M = p.M;
    const int A0 = (int)blockIdx.y * ROWS, A1 = min(M, A0 + ROWS);
    const int rows = A1 - A0;
    for (int t = threadIdx.x; t < rows * M; t += blockDim.x) ds[t] = sc_zero(T());
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
    for (int64_t I = lo + wv; I < hi; I += nw) {
        const uint64_t d0 = p.dets[2 * I], d1 = p.dets[2 * I + 1];
        const T w = pair_weight<CPLX>(bra, ket, R, (uint32_t)I, (uint32_t)I, W);
        const int B0 = lane, B1 = lane + 64;
        const bool o0 = B0 < M && (B0 < n ? (d0 >> B0) & 1 : (d1 >> (B0 - n)) & 1);
        const bool o1 = B1 < M && (B1 < n ? (d0 >> B1) & 1 : (d1 >> (B1 - n)) & 1);
        uint64_t m0, m1;
        rowmask(d0, d1, m0, m1);
        for (int word = 0; word < 2; word++) {
            for (uint64_t x = word ? m1 : m0; x; x &= x - 1) {
                const int A = __builtin_ctzll(x) + (word ? n : 0);
                T *row = ds + (size_t)(A - A0) * M;
                if (o0) atom_add(row + B0, w);
                if (o1) atom_add(row + B1, w);
            }
        }
    }
    __syncthreads();
    T *out = part + (size_t)blockIdx.x * M * M + (size_t)A0 * M;
    for (int t = threadIdx.x; t < rows * M; t += blockDim.x) out[t] = ds[t];
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

static unsigned xcd_grid_r(int64_t blocks)
{
    const int64_t q = 8 * 16;
    return (unsigned)((blocks + q - 1) / q * q);
}

static void zero(double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
}

mw_status launch_rdm(const DevPlan &p, int R, const void *bra, const void *ket, const double *weights,
                     const double *dev_weights, void *gamma, void *Gamma, double fac_g, bool conj, hipStream_t s)
{
    RdmWeights W;
    for (int k = 0; k < 64; k++) W.w[k] = (weights && k < R) ? weights[k] : 1.0;
    W.dev = dev_weights;
    // one vector as bra and ket (real weights): w_JI = conj(w_IJ)
    const bool sym = bra == ket;
    const int n = p.n, M = p.M;
    const unsigned gd = (unsigned)((p.npacket_double + 3) / 4);
    const unsigned gs = (unsigned)((p.npacket - p.npacket_double + 3) / 4);
    const unsigned gdx = xcd_grid_r((p.npacket_double + 3) / 4);
    const int64_t mm = (int64_t)M * M;
    const unsigned gred = (unsigned)((mm + 255) / 256);
    if (p.kind == MW_SPIN_FREE) {
        const int64_t n4 = (int64_t)n * n * n * n, np2 = (int64_t)p.npair * p.npair, n3 = (int64_t)n * n * n;
        // S | C | E, RDM_COPIES times
        const int64_t cs = 2 * (int64_t)n * n + 2 * n3;
        double *dab = (double *)p.partial, *dt0 = dab + n4, *dt1 = dt0 + np2, *S = dt1 + np2;
        double *Cc = S + 2 * (int64_t)n * n, *Ee = Cc + n3, *D = S + RDM_COPIES * cs, *part = D + mm;
        zero(dab, n4 + 2 * np2 + RDM_COPIES * cs, s);
        ProfToken t = prof_begin("rdm_double", s);
        if (gd) {
            if (sym)
                hipLaunchKernelGGL((k_rdm_double<false, 8, true>), dim3(gdx), dim3(256), 0, s, p, R,
                                   (const double *)bra, (const double *)ket, W, dab, dt0, dt1);
            else
                hipLaunchKernelGGL((k_rdm_double<false, 8, false>), dim3(gdx), dim3(256), 0, s, p, R,
                                   (const double *)bra, (const double *)ket, W, dab, dt0, dt1);
        }
        prof_end(t, s);
        t = prof_begin("rdm_single", s);
        if (gs) {
            if (sym)
                hipLaunchKernelGGL((k_rdm_single<false, true>), dim3(gs), dim3(256), 0, s, p, R,
                                   (const double *)bra, (const double *)ket, W, S, Cc, Ee, cs);
            else
                hipLaunchKernelGGL((k_rdm_single<false, false>), dim3(gs), dim3(256), 0, s, p, R,
                                   (const double *)bra, (const double *)ket, W, S, Cc, Ee, cs);
        }
        prof_end(t, s);
        hipLaunchKernelGGL(k_rdm_fold<double>, dim3((unsigned)((cs + 255) / 256)), dim3(256), 0, s, S, cs,
                           RDM_COPIES);
        if (sym) {
            hipLaunchKernelGGL(k_rdm_mirror<double>, dim3((unsigned)((2 * (int64_t)n * n + 255) / 256)), dim3(256), 0,
                               s, S, n, 1, 2);
            hipLaunchKernelGGL(k_rdm_mirror_qxp<double>, dim3((unsigned)((2 * n3 + 255) / 256)), dim3(256), 0, s, Cc,
                               n, 2);
        }
        t = prof_begin("rdm_diag", s);
        hipLaunchKernelGGL(k_rdm_occ_lds<false>, dim3(RDM_OCC_CHUNKS, (unsigned)((M + 127) / 128)), dim3(1024), 0, s,
                           p, R, (const double *)bra, (const double *)ket, W, part);
        hipLaunchKernelGGL(k_rdm_occ_reduce<double>, dim3(gred), dim3(256), 0, s, M, RDM_OCC_CHUNKS,
                           (const double *)part, D);
        hipLaunchKernelGGL(k_rdm_finalize_sf, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, p, dab, dt0, dt1,
                           S, Cc, Ee, D, (double *)gamma, (double *)Gamma, (int)sym, fac_g);
        prof_end(t, s);
    } else {
        const int64_t m4 = mm * mm, np2 = (int64_t)p.npair * p.npair, m3 = mm * M;
        // S | C, RDM_COPIES times
        const int64_t cs = mm + m3;
        double2 *dt0 = (double2 *)p.partial, *dt1 = dt0 + np2, *S = dt1 + np2, *Cc = S + mm,
                *D = S + RDM_COPIES * cs, *part = D + mm;
        zero((double *)dt0, 2 * (2 * np2 + RDM_COPIES * cs), s);
        ProfToken t = prof_begin("rdm_double", s);
        if (gd) {
            if (sym)
                hipLaunchKernelGGL((k_rdm_double<true, 4, true>), dim3(gdx), dim3(256), 0, s, p, R,
                                   (const double2 *)bra, (const double2 *)ket, W, (double *)nullptr, dt0, dt1);
            else
                hipLaunchKernelGGL((k_rdm_double<true, 4, false>), dim3(gdx), dim3(256), 0, s, p, R,
                                   (const double2 *)bra, (const double2 *)ket, W, (double *)nullptr, dt0, dt1);
        }
        prof_end(t, s);
        t = prof_begin("rdm_single", s);
        if (gs) {
            if (sym)
                hipLaunchKernelGGL((k_rdm_single<true, true>), dim3(gs), dim3(256), 0, s, p, R,
                                   (const double2 *)bra, (const double2 *)ket, W, S, Cc, (double *)nullptr, cs);
            else
                hipLaunchKernelGGL((k_rdm_single<true, false>), dim3(gs), dim3(256), 0, s, p, R,
                                   (const double2 *)bra, (const double2 *)ket, W, S, Cc, (double *)nullptr, cs);
        }
        prof_end(t, s);
        hipLaunchKernelGGL(k_rdm_fold<double2>, dim3((unsigned)((cs + 255) / 256)), dim3(256), 0, s, S, cs,
                           RDM_COPIES);
        if (sym) {
            hipLaunchKernelGGL(k_rdm_mirror<double2>, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, S, M, 1, 1);
            hipLaunchKernelGGL(k_rdm_mirror_qxp<double2>, dim3((unsigned)((m3 + 255) / 256)), dim3(256), 0, s, Cc, M,
                               1);
        }
        t = prof_begin("rdm_diag", s);
        hipLaunchKernelGGL(k_rdm_occ_lds<true>, dim3(RDM_OCC_CHUNKS, (unsigned)((M + 63) / 64)), dim3(1024), 0, s, p,
                           R, (const double2 *)bra, (const double2 *)ket, W, part);
        hipLaunchKernelGGL(k_rdm_occ_reduce<double2>, dim3(gred), dim3(256), 0, s, M, RDM_OCC_CHUNKS,
                           (const double2 *)part, D);
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
