// Device build of a plan's index: the grouping of determinants by shared
// (N-1)/(N-2)-electron strings (MetaWave section 2.3), the packets, the
// placement of the partial sums and the density-matrix rows, as radix sorts,
// scans and per-element kernels on the GPU.  Every rule of the host build in
// plan.cpp is kept, so the arrays are the same bit for bit:
//
//  1. key entries: determinant D emits, in a fixed order, D minus each
//     occupied position a (single) and D minus each pair a < b (double);
//     entry e belongs to determinant e / per_det, so only its index is kept;
//  2. two stable radix sorts (second word of the string, then the first)
//     order the entries by (K, determinant);
//  3. runs of equal K with two or more entries are the groups; a stable
//     sort on (single, decreasing size, kind, first member) over runs
//     listed in K order gives the host's group order (ties by K);
//  4. members, phases, the integral-layout bit and pair counts per group;
//  5. packets: large groups cut into 64-member blocks, small groups packed
//     greedily; with sizes non-increasing inside each class the greedy
//     packing is periodic, so a packet start follows from the group's index
//     in its class and two numbers per class computed on the host;
//  6. column partials, the determinant-major slot lists (a stable sort of
//     memberships by determinant) and the slot placement (a stable sort of
//     the slots, in packet order, by region and writing XCD);
//  7. density rows: a stable sort of memberships by accumulator row and
//     class, chunks cut greedily per row segment (binary searches over the
//     prefix sums of the partner visits) and ordered by work on the host.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "plan_host.h"

namespace mw {

void DevIndex::release()
{
    void *ptrs[] = {grp_off, grp_col, mem_grp, slot_mem, slot_pos, pk_off, rowptr, rdm_ent_det,
                    grp_key, grp_type, mem, rdm_ent, rdm_chunk, rdm_pos, rdm_skey};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    grp_off = grp_col = mem_grp = slot_mem = slot_pos = pk_off = rowptr = rdm_ent_det = nullptr;
    grp_key = nullptr;
    grp_type = nullptr;
    mem = rdm_ent = nullptr;
    rdm_chunk = nullptr;
    rdm_pos = nullptr;
    rdm_skey = nullptr;
}

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(int64_t n)
{
    const int64_t b = (n + TPB - 1) / TPB;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 20));
}

inline int bits_for(uint64_t maxval)  // bits to hold values 0 .. maxval
{
    int b = 1;
    while (b < 64 && (maxval >> b)) b++;
    return b;
}

// temporary device memory, freed at scope exit (after the stream drained)
struct Temp {
    hipStream_t s;
    std::vector<void *> v;
    explicit Temp(hipStream_t st) : s(st) {}
    ~Temp()
    {
        (void)hipStreamSynchronize(s);
        for (void *p : v) (void)hipFree(p);
    }
    template <class T> T *get(size_t n)
    {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        v.push_back(p);
        return (T *)p;
    }
    void drop(void *p)
    {
        auto it = std::find(v.begin(), v.end(), p);
        if (it == v.end()) return;
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
        v.erase(it);
    }
};

template <class T> T *dalloc(size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    return (T *)p;
}

template <class K, class V>
hipError_t sort_pairs(const K *ki, K *ko, const V *vi, V *vo, size_t n, int bits, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t tb = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, tb, ki, ko, vi, vo, n, 0u, (unsigned)bits, s);
    if (e != hipSuccess) return e;
    void *tmp = nullptr;
    if ((e = hipMalloc(&tmp, std::max<size_t>(tb, 1))) != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(tmp, tb, ki, ko, vi, vo, n, 0u, (unsigned)bits, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e != hipSuccess ? e : e2;
}

template <class T> hipError_t excl_scan(const T *in, T *out, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t tb = 0;
    hipError_t e = rocprim::exclusive_scan(nullptr, tb, in, out, (T)0, n, rocprim::plus<T>(), s);
    if (e != hipSuccess) return e;
    void *tmp = nullptr;
    if ((e = hipMalloc(&tmp, std::max<size_t>(tb, 1))) != hipSuccess) return e;
    e = rocprim::exclusive_scan(tmp, tb, in, out, (T)0, n, rocprim::plus<T>(), s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e != hipSuccess ? e : e2;
}

// ---------------------------------------------------------------------------
// string helpers (positions: first word 0 .. n-1, second word n .. 2n-1)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int nth_set(uint64_t w, int k)
{
    for (int i = 0; i < k; i++) w &= w - 1;
    return __builtin_ctzll(w);
}

__device__ __forceinline__ int occ_pos(uint64_t w0, uint64_t w1, int n, int k)
{
    const int c0 = __builtin_popcountll(w0);
    return k < c0 ? nth_set(w0, k) : n + nth_set(w1, k - c0);
}

__device__ __forceinline__ void drop_pos(uint64_t &w0, uint64_t &w1, int n, int X)
{
    if (X < n) w0 &= ~(1ULL << X);
    else w1 &= ~(1ULL << (X - n));
}

__device__ __forceinline__ int pi_odd(uint64_t k0, uint64_t k1, int n, int X)
{
    int c;
    if (X < n) c = __builtin_popcountll(k0 & ((1ULL << X) - 1));
    else {
        const int b = X - n;
        c = __builtin_popcountll(k0) + __builtin_popcountll(k1 & (b == 64 ? ~0ULL : ((1ULL << b) - 1)));
    }
    return c & 1;
}

struct Space {
    const uint64_t *dets;
    const uint16_t *lab;  // local entry index -> a | b << 8 (b = 255: single)
    uint32_t per_det;
    int n;
};

// entry e: its determinant, removed positions X, Y (Y = 255 for a single)
// and the string K
__device__ __forceinline__ void decode(const Space &sp, uint32_t e, uint32_t &det, int &X, int &Y, uint64_t &k0,
                                       uint64_t &k1)
{
    det = e / sp.per_det;
    const uint32_t l = e - det * sp.per_det;
    const uint16_t ab = sp.lab[l];
    const int a = ab & 255, b = ab >> 8;
    const uint64_t w0 = sp.dets[2 * (size_t)det], w1 = sp.dets[2 * (size_t)det + 1];
    X = occ_pos(w0, w1, sp.n, a);
    Y = b == 255 ? 255 : occ_pos(w0, w1, sp.n, b);
    k0 = w0;
    k1 = w1;
    drop_pos(k0, k1, sp.n, X);
    if (Y != 255) drop_pos(k0, k1, sp.n, Y);
}

// ---------------------------------------------------------------------------
// 1-3: entries, sorts, runs
// ---------------------------------------------------------------------------

__global__ void k_entries(Space sp, uint32_t total, uint64_t *key, uint32_t *val)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t det;
        int X, Y;
        uint64_t k0, k1;
        decode(sp, (uint32_t)e, det, X, Y, k0, k1);
        key[e] = k1;
        val[e] = (uint32_t)e;
    }
}

__global__ void k_first_word(Space sp, uint32_t total, const uint32_t *idx, uint64_t *key)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t det;
        int X, Y;
        uint64_t k0, k1;
        decode(sp, idx[i], det, X, Y, k0, k1);
        key[i] = k0;
    }
}

// head[i] = 1 where a new string K starts in the sorted order
__global__ void k_heads(Space sp, uint32_t total, const uint64_t *k0s, const uint32_t *idx, uint8_t *head)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        uint8_t h = 1;
        if (i > 0 && k0s[i] == k0s[i - 1]) {
            uint32_t det;
            int X, Y;
            uint64_t a0, a1, b0, b1;
            decode(sp, idx[i], det, X, Y, a0, a1);
            decode(sp, idx[i - 1], det, X, Y, b0, b1);
            h = a1 != b1;
        }
        head[i] = h;
    }
}

// flag[i] = 1 where a run of two or more entries starts; flag[total] = 0
__global__ void k_run_flags(uint32_t total, const uint8_t *head, uint32_t *flag)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= total; i += (uint64_t)gridDim.x * blockDim.x)
        flag[i] = (i + 1 < total && head[i] && !head[i + 1]) ? 1u : 0u;
}

__global__ void k_scatter_flagged(uint32_t total, const uint32_t *flag, const uint32_t *pos, uint32_t *out)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x)
        if (flag[i]) out[pos[i]] = (uint32_t)i;
}

// the ordering key of each run: single, decreasing size, kind, first member
constexpr uint32_t LMAX = (1u << 20) - 1;
__global__ void k_run_keys(Space sp, uint32_t total, uint32_t nrun, const uint32_t *start, const uint8_t *head,
                           const uint32_t *idx, uint32_t *len, uint64_t *key, uint32_t *val, uint32_t *err)
{
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < nrun; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s0 = start[r];
        uint32_t t = s0 + 1;
        while (t < total && !head[t]) t++;
        const uint32_t L = t - s0;
        uint32_t det;
        int X, Y;
        uint64_t k0, k1;
        decode(sp, idx[s0], det, X, Y, k0, k1);
        const int n = sp.n;
        const uint32_t single = Y == 255;
        const uint32_t kind = single ? (X < n ? 0u : 1u) : ((X < n && Y < n) ? 0u : (X >= n && Y >= n) ? 1u : 2u);
        if (L > LMAX) atomicOr(err, 1u);
        len[r] = L;
        key[r] = ((uint64_t)single << 54) | ((uint64_t)(LMAX - min(L, LMAX)) << 34) | ((uint64_t)kind << 32) | det;
        val[r] = (uint32_t)r;
    }
}

__global__ void k_group_len(uint32_t ngroup, const uint32_t *order, const uint32_t *rlen, uint32_t *glen)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g <= ngroup; g += (uint64_t)gridDim.x * blockDim.x)
        glen[g] = g < ngroup ? rlen[order[g]] : 0u;
}

// ---------------------------------------------------------------------------
// 4: members (one thread per group; large groups' layout bits and pair
// counts in k_large)
// ---------------------------------------------------------------------------

struct GroupOut {
    uint32_t *grp_off;
    uint64_t *grp_key;
    uint8_t *grp_type;
    uint2 *mem;
    uint32_t *mem_grp;
    uint64_t *pairs;   // per group: single pairs k (k - 1) or double pairs
};

__global__ void k_members(Space sp, int spinfree, uint32_t ngroup, const uint32_t *order, const uint32_t *rstart,
                          const uint32_t *idx, GroupOut o)
{
    const int n = sp.n;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroup; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = order[g];
        const uint32_t s0 = rstart[r];
        const uint32_t m0 = o.grp_off[g], k = o.grp_off[g + 1] - m0;
        bool single = false;
        uint8_t type = 0;
        for (uint32_t t = 0; t < k; t++) {
            uint32_t det;
            int X, Y;
            uint64_t k0, k1;
            decode(sp, idx[s0 + t], det, X, Y, k0, k1);
            if (t == 0) {
                single = Y == 255;
                o.grp_key[2 * (size_t)g] = k0;
                o.grp_key[2 * (size_t)g + 1] = k1;
                if (spinfree) {
                    if (single) type = X < n ? G_SINGLE_A : G_SINGLE_B;
                    else type = (X < n && Y < n) ? G_AA : (X >= n && Y >= n) ? G_BB : G_AB;
                } else {
                    type = single ? G_SINGLE_S : G_DOUBLE_S;
                }
                o.grp_type[g] = type;
            }
            const int odd = pi_odd(k0, k1, n, X) ^ (single ? 0 : pi_odd(k0, k1, n, Y));
            o.mem[m0 + t] = make_uint2(det, (uint32_t)(X | (Y << 8) | (odd ? (1u << 16) : 0u)));
            o.mem_grp[m0 + t] = (uint32_t)g;
        }
        if (single) {
            o.pairs[g] = (uint64_t)k * (k - 1);
            if (k < 64)
                for (uint32_t t = 0; t < k; t++) o.mem[m0 + t].y |= (t << 18) | (k << 24);
            continue;
        }
        if (k >= 64) continue;  // k_large
        // small double group: its 64-member window is the whole group
        const bool ab = type == G_AB;
        uint64_t dp = 0;
        for (uint32_t t = 0; t < k; t++) {
            const uint32_t yt = o.mem[m0 + t].y;
            const uint32_t Xt = yt & 255, Yt = (yt >> 8) & 255;
            int fx = 0, fy = 0, cx = 0, cy = 0;
            for (uint32_t u = 0; u < k; u++) {
                const uint32_t yu = o.mem[m0 + u].y;
                const uint32_t Xu = yu & 255, Yu = (yu >> 8) & 255;
                fx += (Xu == Xt) + (Yu == Xt);
                fy += (Xu == Yt) + (Yu == Yt);
                if (u != t) {
                    cx += Xu == Xt;
                    cy += Yu == Yt;
                }
            }
            dp += (uint64_t)((int)k - (fx + fy - 1));
            const int lay = cx >= cy ? (ab ? 0 : 1) : (ab ? 1 : 0);
            o.mem[m0 + t].y = yt | (lay ? (1u << 17) : 0u) | (t << 18) | (k << 24);
        }
        o.pairs[g] = dp;
    }
}

// large double groups [0, nlarge): one workgroup each; double pairs from
// the position histogram (sum over members of k - (f_X + f_Y - 1) =
// k (k + 1) - sum_x f_x^2) and the layout bit of every 64-member window
__global__ void __launch_bounds__(TPB) k_large(uint32_t nlarge, GroupOut o)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t hx[4][256], hy[4][256];
    __shared__ uint64_t part[TPB / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (uint32_t g = blockIdx.x; g < nlarge; g += gridDim.x) {
        const uint32_t m0 = o.grp_off[g], k = o.grp_off[g + 1] - m0;
        const bool ab = o.grp_type[g] == G_AB;
        for (int i = threadIdx.x; i < 256; i += TPB) hist[i] = 0;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < k; t += TPB) {
            const uint32_t y = o.mem[m0 + t].y;
            atomicAdd(&hist[y & 255], 1u);
            atomicAdd(&hist[(y >> 8) & 255], 1u);
        }
        __syncthreads();
        uint64_t sq = 0;
        for (int i = threadIdx.x; i < 256; i += TPB) sq += (uint64_t)hist[i] * hist[i];
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
        if (lane == 0) part[wv] = sq;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t tot = 0;
            for (int i = 0; i < TPB / 64; i++) tot += part[i];
            o.pairs[g] = (uint64_t)k * (k + 1) - tot;
        }
        // windows of 64 members, four at a time (one per wave)
        const uint32_t nw = (k + 63) / 64;
        for (uint32_t w0 = 0; w0 < nw; w0 += 4) {
            const uint32_t w = w0 + wv;
            for (int i = lane; i < 256; i += 64) hx[wv][i] = hy[wv][i] = 0;
            __syncthreads();
            const uint32_t t = w * 64 + lane;
            const bool live = w < nw && t < k;
            uint32_t y = 0;
            if (live) {
                y = o.mem[m0 + t].y;
                atomicAdd(&hx[wv][y & 255], 1u);
                atomicAdd(&hy[wv][(y >> 8) & 255], 1u);
            }
            __syncthreads();
            if (live) {
                const int cx = (int)hx[wv][y & 255] - 1, cy = (int)hy[wv][(y >> 8) & 255] - 1;
                const int lay = cx >= cy ? (ab ? 0 : 1) : (ab ? 1 : 0);
                if (lay) o.mem[m0 + t].y = y | (1u << 17);
            }
            __syncthreads();
        }
    }
}

// totals: single pairs, double pairs, double pairs of large groups, sum k^2
__global__ void k_pair_totals(uint32_t ngroup, const uint32_t *grp_off, const uint8_t *grp_type,
                              const uint64_t *pairs, unsigned long long *tot)
{
    __shared__ unsigned long long sh[4][TPB / 64];
    unsigned long long a[4] = {0, 0, 0, 0};
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroup; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = grp_off[g + 1] - grp_off[g];
        const uint8_t ty = grp_type[g];
        const bool single = ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S;
        if (single) a[0] += pairs[g];
        else {
            a[1] += pairs[g];
            if (k >= 64) a[2] += pairs[g];
        }
        a[3] += (unsigned long long)k * k;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = 0; c < 4; c++) {
        unsigned long long v = a[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long v = 0;
        for (int i = 0; i < TPB / 64; i++) v += sh[threadIdx.x][i];
        atomicAdd(&tot[threadIdx.x], v);
    }
}

// ---------------------------------------------------------------------------
// 5: packets
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool is_single(uint8_t ty) { return ty == G_SINGLE_A || ty == G_SINGLE_B || ty == G_SINGLE_S; }

// class of a group: single * 65 + min(size, 64) (64: a large group)
__global__ void k_class_first(uint32_t ngroup, const uint32_t *grp_off, const uint8_t *grp_type, uint32_t *first)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroup; g += (uint64_t)gridDim.x * blockDim.x) {
        auto cls = [&](uint64_t h) {
            const uint32_t k = grp_off[h + 1] - grp_off[h];
            return (is_single(grp_type[h]) ? 65u : 0u) + min(k, 64u);
        };
        const uint32_t c = cls(g);
        if (g == 0 || cls(g - 1) != c) first[c] = (uint32_t)g;
    }
}

struct PackClass {
    uint32_t first, a, q, pad;
};

__global__ void k_packet_counts(uint32_t ngroup, const uint32_t *grp_off, const uint8_t *grp_type,
                                const PackClass *pc, uint32_t *cnt)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g <= ngroup; g += (uint64_t)gridDim.x * blockDim.x) {
        if (g == ngroup) {
            cnt[g] = 0;
            continue;
        }
        const uint32_t k = grp_off[g + 1] - grp_off[g];
        if (k >= 64) {
            cnt[g] = (k + 63) / 64;
            continue;
        }
        const PackClass c = pc[(is_single(grp_type[g]) ? 65u : 0u) + k];
        const uint32_t j = (uint32_t)g - c.first;
        cnt[g] = (j >= c.a && (j - c.a) % c.q == 0) ? 1u : 0u;
    }
}

__global__ void k_packet_offsets(uint32_t ngroup, const uint32_t *grp_off, const uint32_t *cnt, const uint32_t *pstart,
                                 uint32_t *pk_off)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroup; g += (uint64_t)gridDim.x * blockDim.x)
        for (uint32_t c = 0; c < cnt[g]; c++) pk_off[pstart[g] + c] = grp_off[g] + 64 * c;
}

// ---------------------------------------------------------------------------
// 6: column partials, slot lists, placement
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool is_big(uint32_t k, uint8_t ty) { return k >= 64 && !is_single(ty); }

__global__ void k_col_counts(uint32_t ngroup, const uint32_t *grp_off, const uint8_t *grp_type, uint64_t *cc)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g <= ngroup; g += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t v = 0;
        if (g < ngroup) {
            const uint64_t k = grp_off[g + 1] - grp_off[g];
            if (is_big((uint32_t)k, grp_type[g])) {
                const uint64_t nb = (k + 63) / 64;
                v = (nb - 1) * k - 32 * (nb - 1) * nb;
            }
        }
        cc[g] = v;
    }
}

__global__ void k_col_start(uint32_t ngroup, const uint32_t *grp_off, const uint8_t *grp_type, const uint64_t *cs,
                            uint32_t *grp_col)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroup; g += (uint64_t)gridDim.x * blockDim.x)
        grp_col[g] = is_big(grp_off[g + 1] - grp_off[g], grp_type[g]) ? (uint32_t)cs[g] : 0u;
}

__device__ __forceinline__ uint32_t slots_of_member(const uint32_t *grp_off, const uint8_t *grp_type,
                                                    const uint32_t *mem_grp, uint32_t mi)
{
    const uint32_t g = mem_grp[mi];
    const uint32_t k = grp_off[g + 1] - grp_off[g], t = mi - grp_off[g];
    return 1 + (is_big(k, grp_type[g]) ? t / 64 : 0);
}

__global__ void k_row_counts(uint32_t nmem, const uint32_t *grp_off, const uint8_t *grp_type, const uint2 *mem,
                             const uint32_t *mem_grp, uint32_t *rc)
{
    for (uint64_t mi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; mi < nmem; mi += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&rc[mem[mi].x], slots_of_member(grp_off, grp_type, mem_grp, (uint32_t)mi));
}

struct PackGeom {
    const uint32_t *pk_off, *grp_off, *mem_grp, *grp_col, *rowptr;
    const uint8_t *grp_type;
    const uint2 *mem;
    int64_t npd;
    uint32_t nmem;
    uint32_t reg_slots;
};

// column slots [c0, c1) written by packet w (block a of a large double group)
__device__ __forceinline__ void col_range(const PackGeom &q, uint64_t w, uint64_t &c0, uint64_t &c1, uint32_t &g,
                                          uint64_t &a)
{
    c0 = c1 = 0;
    a = 0;
    const uint32_t m0 = q.pk_off[w];
    g = q.mem_grp[m0];
    const uint64_t k = q.grp_off[g + 1] - q.grp_off[g];
    if ((int64_t)w >= q.npd || !is_big((uint32_t)k, q.grp_type[g])) return;
    a = (m0 - q.grp_off[g]) / 64;
    c0 = q.nmem + (uint64_t)q.grp_col[g] + a * k - 32 * a * (a + 1);
    c1 = c0 + (k > 64 * (a + 1) ? k - 64 * (a + 1) : 0);  // the last block hands on nothing
}

__global__ void k_packet_items(uint32_t npk, PackGeom q, uint32_t *cnt)
{
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w <= npk; w += (uint64_t)gridDim.x * blockDim.x) {
        if (w == npk) {
            cnt[w] = 0;
            continue;
        }
        uint64_t c0, c1, a;
        uint32_t g;
        col_range(q, w, c0, c1, g, a);
        cnt[w] = (q.pk_off[w + 1] - q.pk_off[w]) + (uint32_t)(c1 - c0);
    }
}

// items in packet order (members, then column slots), keyed by the region
// of the slot's determinant and the packet's writing XCD
__global__ void k_packet_fill(uint32_t npk, PackGeom q, const uint32_t *ioff, uint32_t *key, uint32_t *val)
{
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < npk; w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = (int64_t)w < q.npd ? (uint32_t)((w / 64) % 8) : (uint32_t)(((w - q.npd) / 4) % 8);
        uint32_t off = ioff[w];
        for (uint32_t m = q.pk_off[w]; m < q.pk_off[w + 1]; m++, off++) {
            key[off] = (q.rowptr[q.mem[m].x] / q.reg_slots) * 8 + x;
            val[off] = m;
        }
        uint64_t c0, c1, a;
        uint32_t g;
        col_range(q, w, c0, c1, g, a);
        for (uint64_t cs = c0; cs < c1; cs++, off++) {
            const uint64_t t = 64 * (a + 1) + (cs - c0);
            key[off] = (q.rowptr[q.mem[q.grp_off[g] + t].x] / q.reg_slots) * 8 + x;
            val[off] = (uint32_t)cs;
        }
    }
}

__global__ void k_slot_pos(uint32_t nslot, const uint32_t *sorted_slot, uint32_t *slot_pos)
{
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < nslot; p += (uint64_t)gridDim.x * blockDim.x)
        slot_pos[sorted_slot[p]] = (uint32_t)p;
}

__global__ void k_member_dets(uint32_t nmem, const uint2 *mem, uint32_t *key, uint32_t *val)
{
    for (uint64_t mi = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; mi < nmem; mi += (uint64_t)gridDim.x * blockDim.x) {
        key[mi] = mem[mi].x;
        val[mi] = (uint32_t)mi;
    }
}

__global__ void k_slot_counts(uint32_t nmem, const uint32_t *grp_off, const uint8_t *grp_type, const uint32_t *mem_grp,
                              const uint32_t *by_det, uint32_t *cnt)
{
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p <= nmem; p += (uint64_t)gridDim.x * blockDim.x)
        cnt[p] = p < nmem ? slots_of_member(grp_off, grp_type, mem_grp, by_det[p]) : 0u;
}

__global__ void k_slot_mem(uint32_t nmem, const uint32_t *grp_off, const uint8_t *grp_type, const uint32_t *mem_grp,
                           const uint32_t *grp_col, const uint32_t *by_det, const uint32_t *soff,
                           const uint32_t *slot_pos, uint32_t *slot_mem)
{
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < nmem; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t mi = by_det[p];
        uint32_t o = soff[p];
        slot_mem[o++] = slot_pos[mi];
        const uint32_t g = mem_grp[mi];
        const uint64_t k = grp_off[g + 1] - grp_off[g], t = mi - grp_off[g];
        if (!is_big((uint32_t)k, grp_type[g])) continue;
        for (uint64_t a = 0; a < t / 64; a++)
            slot_mem[o++] = slot_pos[nmem + grp_col[g] + a * k - 32 * a * (a + 1) + (t - 64 * (a + 1))];
    }
}

// ---------------------------------------------------------------------------
// 7: density rows
// ---------------------------------------------------------------------------

struct RowGeom {
    const uint32_t *grp_off, *mem_grp;
    const uint8_t *grp_type;
    const uint2 *mem;
    uint32_t nmd;      // memberships of double groups
    int n, spinfree;
    int64_t nab, nrow_d;
};

__global__ void k_rdm_keys(uint32_t nmem, RowGeom q, uint32_t *key, uint32_t *val, uint32_t *err)
{
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nmem; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = q.mem_grp[j];
        const uint32_t L = q.grp_off[g + 1] - q.grp_off[g];
        if (L >= 65536) atomicOr(err, 2u);
        const int X = q.mem[j].y & 255, Y = (q.mem[j].y >> 8) & 255;
        const uint8_t ty = q.grp_type[g];
        const int n = q.n;
        int64_t row;
        if (j >= q.nmd) row = q.nrow_d + (ty == G_SINGLE_B ? X - n : X);
        else if (!q.spinfree) row = Y * (Y - 1) / 2 + X;
        else if (ty == G_AB) row = (int64_t)X * n + (Y - n);
        else row = q.nab + (ty == G_BB ? (Y - n) * (Y - n - 1) / 2 + (X - n) : Y * (Y - 1) / 2 + X);
        key[j] = (uint32_t)(row * RDM_WIDE + (L >= (uint32_t)RDM_WIDE ? 0 : L));
        val[j] = (uint32_t)j;
    }
}

__global__ void k_rdm_entries(uint32_t nent, RowGeom q, const uint32_t *rj, uint2 *ent, uint32_t *ent_det)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nent; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t j = rj[e];
        const uint32_t g = q.mem_grp[j];
        const uint32_t j0 = q.grp_off[g], L = q.grp_off[g + 1] - j0;
        ent[e] = make_uint2(j0, (j - j0) | (L << 16));
        ent_det[e] = q.mem[j].x | (((q.mem[j].y >> 16) & 1u) << 31);
    }
}

// start[b] = first entry of bin b (bins of the sorted keys), b in [0, nbin]
__global__ void k_bin_starts(uint32_t nent, uint32_t nbin, const uint32_t *rk, uint32_t *start)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e <= nent; e += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t lo = e == 0 ? 0 : (int64_t)rk[e - 1] + 1;
        const int64_t hi = e == nent ? (int64_t)nbin : (int64_t)rk[e];
        for (int64_t b = lo; b <= hi; b++) start[b] = (uint32_t)e;
    }
}

__global__ void k_rdm_singles(uint32_t e0, uint32_t nent, const uint32_t *mem_grp, const uint64_t *grp_key,
                              const uint8_t *grp_type, uint2 *ent, ulonglong2 *skey)
{
    for (uint64_t e = e0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nent; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = mem_grp[ent[e].x];
        skey[e - e0] = make_ulonglong2(grp_key[2 * (size_t)g], grp_key[2 * (size_t)g + 1]);
        if (grp_type[g] == G_SINGLE_B) ent[e].y |= 1u << 15;
    }
}

__global__ void k_rdm_pos(uint32_t nmem, const uint2 *mem, uint16_t *pos)
{
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nmem; j += (uint64_t)gridDim.x * blockDim.x)
        pos[j] = (uint16_t)(mem[j].y & 0xffffu);
}

// segments (row, part): part 0 the wide class, part 1 the classes 1 .. 31;
// a chunk is cut after the first entry at which its partner visits reach
// RDM_CHUNK_WORK, or at the segment's end (the host rule).  With the
// visits' prefix sums pw (pw[e] = visits of entries before e) the end of
// the chunk starting at a is found by a binary search, so a thread walks
// its segment chunk by chunk instead of entry by entry.
__device__ __forceinline__ void seg_range(const uint32_t *start, uint64_t sg, uint32_t &e0, uint32_t &e1)
{
    const uint64_t row = sg / 2, part = sg % 2;
    e0 = start[row * RDM_WIDE + (part ? 1 : 0)];
    e1 = start[row * RDM_WIDE + (part ? RDM_WIDE : 1)];
}

__global__ void k_visits(uint32_t nent, const uint2 *ent, uint64_t *w)
{
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e <= nent; e += (uint64_t)gridDim.x * blockDim.x)
        w[e] = e < nent ? (uint64_t)((ent[e].y >> 16) - 1) : 0;
}

// last entry of the chunk starting at a (a < e1)
__device__ __forceinline__ uint32_t chunk_end(const uint64_t *pw, uint32_t a, uint32_t e1)
{
    const uint64_t target = pw[a] + (uint64_t)RDM_CHUNK_WORK;
    // smallest e in [a, e1) with pw[e + 1] >= target, else e1 - 1
    uint32_t lo = a, hi = e1 - 1;
    if (pw[e1] < target) return e1 - 1;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (pw[mid + 1] >= target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ void k_chunk_counts(uint32_t nseg, const uint32_t *start, const uint64_t *pw, uint32_t *cnt)
{
    for (uint64_t sg = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; sg <= nseg; sg += (uint64_t)gridDim.x * blockDim.x) {
        if (sg == nseg) {
            cnt[sg] = 0;
            continue;
        }
        uint32_t e0, e1;
        seg_range(start, sg, e0, e1);
        uint32_t c = 0;
        for (uint32_t a = e0; a < e1; c++) a = chunk_end(pw, a, e1) + 1;
        cnt[sg] = c;
    }
}

__global__ void k_chunk_fill(uint32_t nseg, int64_t nab, int64_t nrow_d, const uint32_t *start, const uint64_t *pw,
                             const uint32_t *coff, uint4 *chunk, int64_t *cwork)
{
    for (uint64_t sg = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; sg < nseg; sg += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t e0, e1;
        seg_range(start, sg, e0, e1);
        const int64_t row = (int64_t)(sg / 2);
        const uint32_t flags = row < nab ? 1u : 0u;
        const uint32_t r = (uint32_t)(row < nab ? row : (row < nrow_d ? row - nab : row - nrow_d));
        uint32_t o = coff[sg];
        for (uint32_t a = e0; a < e1; o++) {
            const uint32_t e = chunk_end(pw, a, e1);
            chunk[o] = make_uint4(r, flags, a, e + 1);
            cwork[o] = (int64_t)(pw[e + 1] - pw[a]);
            a = e + 1;
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

#define CK(x)                                                                                       \
    do {                                                                                            \
        if ((x) != hipSuccess) return fail(MW_EHIP, std::string("device plan build: ") + #x);       \
    } while (0)
#define CKL(name)                                                                                   \
    do {                                                                                            \
        if (hipGetLastError() != hipSuccess) return fail(MW_EHIP, "device plan build: launch " name); \
    } while (0)
#define NEED(p)                                                                                     \
    do {                                                                                            \
        if (!(p)) return fail(MW_EHIP, "device plan build: out of device memory");                  \
    } while (0)

template <class T> static hipError_t down(T *dst, const T *src, size_t n, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s);
    return e != hipSuccess ? e : hipStreamSynchronize(s);
}

mw_status build_index_device(HostPlan &P, hipStream_t s)
{
    DevIndex &X = P.dix;
    X.release();
    X = DevIndex{};
    X.on = true;
    const int n = P.n;
    const int64_t N = P.ndet;
    const bool sf = P.kind == MW_SPIN_FREE;
    const int nel = sf ? P.nalpha + P.nbeta : P.nalpha;
    const int64_t per_det = nel + (int64_t)nel * (nel - 1) / 2;
    const int64_t total64 = N * per_det;
    if (total64 >= ((int64_t)1 << 32) - 1)
        return fail(MW_EUNSUPPORTED, "device plan build: more than 2^32 string entries (use the host build)");
    if (N >= (int64_t)1 << 31) return fail(MW_EUNSUPPORTED, "too many determinants for the density rows");
    const uint32_t total = (uint32_t)total64;
    Temp tmp(s);

    NEED(X.rowptr = dalloc<uint32_t>((size_t)N + 1));
    uint64_t *d_dets = tmp.get<uint64_t>(2 * (size_t)N);
    NEED(d_dets);
    CK(hipMemcpyAsync(d_dets, P.dets.data(), 2 * (size_t)N * 8, hipMemcpyHostToDevice, s));
    std::vector<uint16_t> lab;
    for (int a = 0; a < nel; a++) {
        lab.push_back((uint16_t)(a | (255 << 8)));
        for (int b = a + 1; b < nel; b++) lab.push_back((uint16_t)(a | (b << 8)));
    }
    uint16_t *d_lab = tmp.get<uint16_t>(lab.size());
    NEED(d_lab);
    if (!lab.empty()) CK(hipMemcpyAsync(d_lab, lab.data(), lab.size() * 2, hipMemcpyHostToDevice, s));
    Space sp{d_dets, d_lab, (uint32_t)std::max<int64_t>(per_det, 1), n};

    // ---- 1-3: entries sorted by (K, determinant), runs ----
    uint32_t nrun = 0;
    uint32_t *idx = nullptr, *rstart = nullptr, *rlen = nullptr;
    uint8_t *head = nullptr;
    if (total > 0) {
        uint64_t *kA = tmp.get<uint64_t>(total), *kB = tmp.get<uint64_t>(total);
        uint32_t *vA = tmp.get<uint32_t>(total), *vB = tmp.get<uint32_t>(total);
        NEED(kA && kB && vA && vB);
        k_entries<<<grid_for(total), TPB, 0, s>>>(sp, total, kA, vA);
        CKL("k_entries");
        CK(sort_pairs(kA, kB, vA, vB, total, n, s));
        k_first_word<<<grid_for(total), TPB, 0, s>>>(sp, total, vB, kA);
        CKL("k_first_word");
        CK(sort_pairs(kA, kB, vB, vA, total, n, s));
        idx = vA;  // entries in (K, determinant) order; kB holds the first words
        tmp.drop(kA);
        head = tmp.get<uint8_t>(total);
        NEED(head);
        k_heads<<<grid_for(total), TPB, 0, s>>>(sp, total, kB, idx, head);
        CKL("k_heads");
        tmp.drop(kB);
        tmp.drop(vB);
        uint32_t *flag = tmp.get<uint32_t>((size_t)total + 1), *pos = tmp.get<uint32_t>((size_t)total + 1);
        NEED(flag && pos);
        k_run_flags<<<grid_for((int64_t)total + 1), TPB, 0, s>>>(total, head, flag);
        CKL("k_run_flags");
        CK(excl_scan(flag, pos, (size_t)total + 1, s));
        CK(down(&nrun, pos + total, 1, s));
        rstart = tmp.get<uint32_t>(nrun);
        NEED(rstart);
        k_scatter_flagged<<<grid_for(total), TPB, 0, s>>>(total, flag, pos, rstart);
        CKL("k_scatter_flagged");
        tmp.drop(flag);
        tmp.drop(pos);
    }
    const uint32_t ngroup = nrun;
    uint32_t *order = nullptr;
    if (ngroup > 0) {
        rlen = tmp.get<uint32_t>(ngroup);
        uint64_t *rk = tmp.get<uint64_t>(ngroup), *rks = tmp.get<uint64_t>(ngroup);
        uint32_t *rv = tmp.get<uint32_t>(ngroup);
        order = tmp.get<uint32_t>(ngroup);
        uint32_t *err = tmp.get<uint32_t>(1);
        NEED(rlen && rk && rks && rv && order && err);
        CK(hipMemsetAsync(err, 0, 4, s));
        k_run_keys<<<grid_for(ngroup), TPB, 0, s>>>(sp, total, ngroup, rstart, head, idx, rlen, rk, rv, err);
        CKL("k_run_keys");
        uint32_t herr = 0;
        CK(down(&herr, err, 1, s));
        if (herr) return fail(MW_EUNSUPPORTED, "device plan build: a group of more than 2^20 members");
        CK(sort_pairs(rk, rks, rv, order, ngroup, 55, s));
        tmp.drop(rk);
        tmp.drop(rks);
        tmp.drop(rv);
    }
    if (head) tmp.drop(head);

    // ---- 4: groups and members ----
    X.cnt.ngroup = ngroup;
    NEED(X.grp_off = dalloc<uint32_t>((size_t)ngroup + 1));
    NEED(X.grp_key = dalloc<uint64_t>(2 * (size_t)ngroup));
    NEED(X.grp_type = dalloc<uint8_t>(ngroup));
    NEED(X.grp_col = dalloc<uint32_t>(ngroup));
    uint32_t nmem = 0;
    if (ngroup > 0) {
        uint32_t *glen = tmp.get<uint32_t>((size_t)ngroup + 1);
        NEED(glen);
        k_group_len<<<grid_for((int64_t)ngroup + 1), TPB, 0, s>>>(ngroup, order, rlen, glen);
        CKL("k_group_len");
        CK(excl_scan(glen, X.grp_off, (size_t)ngroup + 1, s));
        CK(down(&nmem, X.grp_off + ngroup, 1, s));
        tmp.drop(glen);
    } else {
        CK(hipMemsetAsync(X.grp_off, 0, 4, s));
    }
    X.cnt.nmem = nmem;
    NEED(X.mem = dalloc<uint2>(nmem));
    NEED(X.mem_grp = dalloc<uint32_t>(nmem));
    uint64_t *pairs = tmp.get<uint64_t>(ngroup);
    unsigned long long *tot = tmp.get<unsigned long long>(4);
    NEED(pairs && tot);
    CK(hipMemsetAsync(tot, 0, 32, s));
    GroupOut go{X.grp_off, X.grp_key, X.grp_type, X.mem, X.mem_grp, pairs};
    std::vector<uint32_t> first(130, 0xffffffffu);
    if (ngroup > 0) {
        k_members<<<grid_for(ngroup), TPB, 0, s>>>(sp, sf ? 1 : 0, ngroup, order, rstart, idx, go);
        CKL("k_members");
        uint32_t *dfirst = tmp.get<uint32_t>(130);
        NEED(dfirst);
        k_fill_u32<<<1, TPB, 0, s>>>(dfirst, 130, 0xffffffffu);
        k_class_first<<<grid_for(ngroup), TPB, 0, s>>>(ngroup, X.grp_off, X.grp_type, dfirst);
        CKL("k_class_first");
        CK(down(first.data(), dfirst, 130, s));
        // large double groups come first (class 64 of the doubles)
        const uint32_t nlarge = first[64] == 0xffffffffu ? 0u : [&]() {
            uint32_t e = ngroup;
            for (int c = 63; c >= 2; c--)
                if (first[c] != 0xffffffffu) e = std::min(e, first[c]);
            for (int c = 65; c < 130; c++)
                if (first[c] != 0xffffffffu) e = std::min(e, first[c]);
            return e;
        }();
        if (nlarge > 0) {
            k_large<<<std::min<uint32_t>(nlarge, 1u << 16), TPB, 0, s>>>(nlarge, go);
            CKL("k_large");
        }
        k_pair_totals<<<grid_for(ngroup), TPB, 0, s>>>(ngroup, X.grp_off, X.grp_type, pairs, tot);
        CKL("k_pair_totals");
    }
    unsigned long long htot[4] = {0, 0, 0, 0};
    CK(down(htot, tot, 4, s));
    P.n_single_pairs = (int64_t)htot[0];
    P.n_double_pairs = (int64_t)htot[1];
    P.n_double_pairs_large = (int64_t)htot[2];
    P.n_evals = (int64_t)htot[3];
    // runs and sorted entries are no longer needed
    if (idx) tmp.drop(idx);
    if (rstart) tmp.drop(rstart);
    if (rlen) tmp.drop(rlen);
    if (order) tmp.drop(order);
    tmp.drop(pairs);

    // ---- 5: packets ----
    // classes in group order: doubles (large, then sizes 63 .. 2), singles
    // (large, then 63 .. 2); the count of a class runs to the next present one
    std::vector<PackClass> pcl(130, PackClass{0, 0, 1, 0});
    uint32_t first_single = ngroup;
    {
        std::vector<int> seq;
        for (int cat = 0; cat < 2; cat++) {
            seq.push_back(cat * 65 + 64);
            for (int k = 63; k >= 1; k--) seq.push_back(cat * 65 + k);
        }
        std::vector<int> present;
        for (int c : seq)
            if (first[c] != 0xffffffffu) present.push_back(c);
        for (int c : present)
            if (c >= 65) {
                first_single = first[c];
                break;
            }
        int fill = 0, cat_prev = -1;
        for (size_t i = 0; i < present.size(); i++) {
            const int c = present[i];
            const int cat = c >= 65 ? 1 : 0, k = c - cat * 65;
            if (cat != cat_prev) fill = 0;  // a class boundary closes the open packet
            cat_prev = cat;
            if (k == 64) {
                fill = 0;  // large groups leave no packet open
                continue;
            }
            const uint32_t f0 = first[c];
            const uint32_t f1 = i + 1 < present.size() ? first[present[i + 1]] : ngroup;
            const int64_t cntc = (int64_t)f1 - f0;
            const int q = 64 / k;
            const int64_t a = fill == 0 ? 0 : std::min<int64_t>(cntc, (64 - fill) / k);
            if (a == cntc) fill += (int)(cntc * k);
            else fill = (int)(((cntc - a - 1) % q + 1) * k);
            pcl[c] = PackClass{f0, (uint32_t)a, (uint32_t)q, 0};
        }
    }
    uint32_t npk = 0;
    {
        PackClass *dpc = tmp.get<PackClass>(130);
        uint32_t *pc = tmp.get<uint32_t>((size_t)ngroup + 1), *ps = tmp.get<uint32_t>((size_t)ngroup + 1);
        NEED(dpc && pc && ps);
        CK(hipMemcpyAsync(dpc, pcl.data(), 130 * sizeof(PackClass), hipMemcpyHostToDevice, s));
        k_packet_counts<<<grid_for((int64_t)ngroup + 1), TPB, 0, s>>>(ngroup, X.grp_off, X.grp_type, dpc, pc);
        CKL("k_packet_counts");
        CK(excl_scan(pc, ps, (size_t)ngroup + 1, s));
        CK(down(&npk, ps + ngroup, 1, s));
        uint32_t pd = npk;
        if (first_single < ngroup) CK(down(&pd, ps + first_single, 1, s));
        P.npacket_double = pd;
        if (((int64_t)npk + 1 + 1024) * 64 > 0xffffffffLL) return fail(MW_EUNSUPPORTED, "too many packets for one launch");
        NEED(X.pk_off = dalloc<uint32_t>((size_t)npk + 1));
        if (ngroup > 0) {
            k_packet_offsets<<<grid_for(ngroup), TPB, 0, s>>>(ngroup, X.grp_off, pc, ps, X.pk_off);
            CKL("k_packet_offsets");
        }
        CK(hipMemcpyAsync(X.pk_off + npk, &nmem, 4, hipMemcpyHostToDevice, s));
        CK(hipStreamSynchronize(s));
        tmp.drop(dpc);
        tmp.drop(pc);
        tmp.drop(ps);
    }
    X.cnt.npk = npk;

    // ---- 6: column partials, slot lists, placement ----
    uint64_t ncol = 0;
    {
        uint64_t *cc = tmp.get<uint64_t>((size_t)ngroup + 1), *cs = tmp.get<uint64_t>((size_t)ngroup + 1);
        NEED(cc && cs);
        k_col_counts<<<grid_for((int64_t)ngroup + 1), TPB, 0, s>>>(ngroup, X.grp_off, X.grp_type, cc);
        CKL("k_col_counts");
        CK(excl_scan(cc, cs, (size_t)ngroup + 1, s));
        CK(down(&ncol, cs + ngroup, 1, s));
        if (ngroup > 0) {
            k_col_start<<<grid_for(ngroup), TPB, 0, s>>>(ngroup, X.grp_off, X.grp_type, cs, X.grp_col);
            CKL("k_col_start");
        }
        tmp.drop(cc);
        tmp.drop(cs);
    }
    if ((uint64_t)nmem + ncol > 0xffffffffULL) return fail(MW_EUNSUPPORTED, "too many partial sums");
    P.ncol = (int64_t)ncol;
    const uint32_t nslot = nmem + (uint32_t)ncol;
    X.cnt.nslot = nslot;
    X.cnt.nslot_mem = nslot;
    {
        uint32_t *rc = tmp.get<uint32_t>((size_t)N + 1);
        NEED(rc);
        CK(hipMemsetAsync(rc, 0, ((size_t)N + 1) * 4, s));
        if (nmem > 0) {
            k_row_counts<<<grid_for(nmem), TPB, 0, s>>>(nmem, X.grp_off, X.grp_type, X.mem, X.mem_grp, rc);
            CKL("k_row_counts");
        }
        CK(excl_scan(rc, X.rowptr, (size_t)N + 1, s));
        tmp.drop(rc);
        uint32_t nlist = 0;
        CK(down(&nlist, X.rowptr + N, 1, s));
        if (nlist != nslot) return fail(MW_EINVAL, "internal: slot lists miscounted (device build)");
    }
    NEED(X.slot_pos = dalloc<uint32_t>(nslot));
    NEED(X.slot_mem = dalloc<uint32_t>(nslot));
    if (nmem > 0) {
        const int sbytes = (P.cplx ? 16 : 8) * P.max_roots;
        const int64_t reg_slots = std::max<int64_t>(4096, ((int64_t)2 << 20) / sbytes);
        uint32_t last = 0;
        CK(down(&last, X.rowptr + (N - 1), 1, s));
        const uint64_t nbucket = (uint64_t)(last / reg_slots + 1) * 8;
        PackGeom q{X.pk_off, X.grp_off, X.mem_grp, X.grp_col, X.rowptr, X.grp_type, X.mem, P.npacket_double,
                   nmem, (uint32_t)reg_slots};
        uint32_t *ic = tmp.get<uint32_t>((size_t)npk + 1), *io = tmp.get<uint32_t>((size_t)npk + 1);
        NEED(ic && io);
        k_packet_items<<<grid_for((int64_t)npk + 1), TPB, 0, s>>>(npk, q, ic);
        CKL("k_packet_items");
        CK(excl_scan(ic, io, (size_t)npk + 1, s));
        uint32_t nitem = 0;
        CK(down(&nitem, io + npk, 1, s));
        if (nitem != nslot) return fail(MW_EINVAL, "internal: partial slots miscounted (device build)");
        // nslot items for the placement; nmem + 1 for the slot-list counts
        const size_t nbuf = std::max<size_t>(nslot, (size_t)nmem + 1);
        uint32_t *k1 = tmp.get<uint32_t>(nbuf), *k2 = tmp.get<uint32_t>(nbuf);
        uint32_t *v1 = tmp.get<uint32_t>(nbuf), *v2 = tmp.get<uint32_t>(nbuf);
        NEED(k1 && k2 && v1 && v2);
        k_packet_fill<<<grid_for(npk), TPB, 0, s>>>(npk, q, io, k1, v1);
        CKL("k_packet_fill");
        CK(sort_pairs(k1, k2, v1, v2, nslot, bits_for(nbucket - 1), s));
        k_slot_pos<<<grid_for(nslot), TPB, 0, s>>>(nslot, v2, X.slot_pos);
        CKL("k_slot_pos");
        // determinant-major slot lists: memberships stably sorted by determinant
        k_member_dets<<<grid_for(nmem), TPB, 0, s>>>(nmem, X.mem, k1, v1);
        CKL("k_member_dets");
        CK(sort_pairs(k1, k2, v1, v2, nmem, bits_for((uint64_t)std::max<int64_t>(N - 1, 0)), s));
        k_slot_counts<<<grid_for((int64_t)nmem + 1), TPB, 0, s>>>(nmem, X.grp_off, X.grp_type, X.mem_grp, v2, k1);
        CKL("k_slot_counts");
        CK(excl_scan(k1, v1, (size_t)nmem + 1, s));
        k_slot_mem<<<grid_for(nmem), TPB, 0, s>>>(nmem, X.grp_off, X.grp_type, X.mem_grp, X.grp_col, v2, v1,
                                                   X.slot_pos, X.slot_mem);
        CKL("k_slot_mem");
        CK(hipStreamSynchronize(s));
        tmp.drop(ic);
        tmp.drop(io);
        tmp.drop(k1);
        tmp.drop(k2);
        tmp.drop(v1);
        tmp.drop(v2);
    }

    // ---- 7: density rows ----
    uint32_t nmd = 0;  // memberships of double groups
    if (P.npacket_double > 0) CK(down(&nmd, X.pk_off + P.npacket_double, 1, s));
    P.nmem_double = nmd;
    P.rdm_single_e0 = 0;
    for (auto &c : P.rdm_cls) c = 0;
    NEED(X.rdm_pos = dalloc<uint16_t>(nmem));
    if (nmem > 0) {
        const int64_t npair = sf ? (int64_t)n * (n - 1) / 2 : (int64_t)P.M * (P.M - 1) / 2;
        const int64_t nab = sf ? (int64_t)n * n : 0, nrow_d = nab + npair;
        const int64_t nrow = nrow_d + (sf ? n : P.M);
        const int64_t nbin = nrow * RDM_WIDE;
        RowGeom q{X.grp_off, X.mem_grp, X.grp_type, X.mem, nmd, n, sf ? 1 : 0, nab, nrow_d};
        uint32_t *k1 = tmp.get<uint32_t>(nmem), *k2 = tmp.get<uint32_t>(nmem);
        uint32_t *v1 = tmp.get<uint32_t>(nmem), *v2 = tmp.get<uint32_t>(nmem);
        uint32_t *err = tmp.get<uint32_t>(1), *start = tmp.get<uint32_t>((size_t)nbin + 1);
        NEED(k1 && k2 && v1 && v2 && err && start);
        CK(hipMemsetAsync(err, 0, 4, s));
        k_rdm_keys<<<grid_for(nmem), TPB, 0, s>>>(nmem, q, k1, v1, err);
        CKL("k_rdm_keys");
        uint32_t herr = 0;
        CK(down(&herr, err, 1, s));
        if (herr) return fail(MW_EUNSUPPORTED, "group too large for the density rows");
        CK(sort_pairs(k1, k2, v1, v2, nmem, bits_for((uint64_t)nbin - 1), s));
        const uint32_t nent = nmem;
        X.cnt.nrdm_ent = nent;
        NEED(X.rdm_ent = dalloc<uint2>(nent));
        NEED(X.rdm_ent_det = dalloc<uint32_t>(nent));
        k_rdm_entries<<<grid_for(nent), TPB, 0, s>>>(nent, q, v2, X.rdm_ent, X.rdm_ent_det);
        CKL("k_rdm_entries");
        k_bin_starts<<<grid_for((int64_t)nent + 1), TPB, 0, s>>>(nent, (uint32_t)nbin, k2, start);
        CKL("k_bin_starts");
        uint32_t e0 = 0;
        CK(down(&e0, start + nrow_d * RDM_WIDE, 1, s));
        P.rdm_single_e0 = e0;
        X.cnt.nrdm_skey = nent - e0;
        NEED(X.rdm_skey = dalloc<ulonglong2>(nent - e0));
        if (nent > e0) {
            k_rdm_singles<<<grid_for(nent - e0), TPB, 0, s>>>(e0, nent, X.mem_grp, X.grp_key, X.grp_type, X.rdm_ent,
                                                               X.rdm_skey);
            CKL("k_rdm_singles");
        }
        k_rdm_pos<<<grid_for(nmem), TPB, 0, s>>>(nmem, X.mem, X.rdm_pos);
        CKL("k_rdm_pos");
        // chunks per segment, then ordered by work inside each class on the host
        const uint32_t nseg = (uint32_t)(nrow * 2);
        uint32_t *cc = tmp.get<uint32_t>((size_t)nseg + 1), *co = tmp.get<uint32_t>((size_t)nseg + 1);
        uint64_t *vis = tmp.get<uint64_t>((size_t)nent + 1), *pw = tmp.get<uint64_t>((size_t)nent + 1);
        NEED(cc && co && vis && pw);
        k_visits<<<grid_for((int64_t)nent + 1), TPB, 0, s>>>(nent, X.rdm_ent, vis);
        CKL("k_visits");
        CK(excl_scan(vis, pw, (size_t)nent + 1, s));
        k_chunk_counts<<<grid_for((int64_t)nseg + 1), TPB, 0, s>>>(nseg, start, pw, cc);
        CKL("k_chunk_counts");
        CK(excl_scan(cc, co, (size_t)nseg + 1, s));
        uint32_t nch = 0;
        CK(down(&nch, co + nseg, 1, s));
        uint4 *dch = tmp.get<uint4>(nch);
        int64_t *dwk = tmp.get<int64_t>(nch);
        NEED(dch && dwk);
        k_chunk_fill<<<grid_for(nseg), TPB, 0, s>>>(nseg, nab, nrow_d, start, pw, co, dch, dwk);
        CKL("k_chunk_fill");
        std::vector<uint4> hch(nch);
        std::vector<int64_t> hwk(nch);
        std::vector<uint32_t> hco((size_t)nseg + 1);
        CK(down(hch.data(), dch, nch, s));
        CK(down(hwk.data(), dwk, nch, s));
        CK(down(hco.data(), co, (size_t)nseg + 1, s));
        struct Ch {
            uint4 c;
            int64_t work;
        };
        std::vector<Ch> cls[5];
        for (uint32_t sg = 0; sg < nseg; sg++) {
            const int64_t row = sg / 2;
            const int part = sg % 2;
            std::vector<Ch> &out = cls[row >= nrow_d ? 4 : (row < nab ? 0 : 2) + part];
            for (uint32_t i = hco[sg]; i < hco[sg + 1]; i++) out.push_back(Ch{hch[i], hwk[i]});
        }
        std::vector<uint4> chunks;
        chunks.reserve(nch);
        for (int c = 0; c < 5; c++) {
            std::stable_sort(cls[c].begin(), cls[c].end(), [](const Ch &x, const Ch &y) { return x.work > y.work; });
            P.rdm_cls[c] = (int64_t)chunks.size();
            for (auto &x : cls[c]) chunks.push_back(x.c);
        }
        P.rdm_cls[5] = (int64_t)chunks.size();
        X.cnt.nrdm_chunk = (int64_t)chunks.size();
        NEED(X.rdm_chunk = dalloc<uint4>(chunks.size()));
        if (!chunks.empty())
            CK(hipMemcpyAsync(X.rdm_chunk, chunks.data(), chunks.size() * 16, hipMemcpyHostToDevice, s));
        CK(hipStreamSynchronize(s));
    } else {
        X.cnt.nrdm_ent = X.cnt.nrdm_chunk = X.cnt.nrdm_skey = 0;
    }
    CK(hipStreamSynchronize(s));
    return MW_OK;
}

}  // namespace mw
