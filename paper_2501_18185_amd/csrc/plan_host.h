// Host-side plan of libmw (internal, not part of the ABI): the grouping of a
// determinant space built on the host (plan.cpp) or on the device
// (plan_dev.hip), its repacked integrals and its binding to a workspace.
#pragma once

#include <cstdint>
#include <vector>

#include "mw_internal.h"

namespace mw {

// element counts of the index arrays (host vectors or device arrays)
struct Counts {
    int64_t ngroup = 0, nmem = 0, nslot_mem = 0, nslot = 0, npk = 0;
    int64_t nrdm_ent = 0, nrdm_chunk = 0, nrdm_skey = 0;
};

// Index arrays built on the device, each its own allocation, owned by the
// plan until the first upload copies them into the workspace.
struct DevIndex {
    bool on = false;
    uint32_t *grp_off = nullptr, *grp_col = nullptr, *mem_grp = nullptr, *slot_mem = nullptr, *slot_pos = nullptr;
    uint32_t *pk_off = nullptr, *rowptr = nullptr, *rdm_ent_det = nullptr;
    uint64_t *grp_key = nullptr;
    uint8_t *grp_type = nullptr;
    uint2 *mem = nullptr, *rdm_ent = nullptr;
    uint4 *rdm_chunk = nullptr;
    uint16_t *rdm_pos = nullptr;
    ulonglong2 *rdm_skey = nullptr;
    Counts cnt;
    void release();
};

struct HostPlan {
    int32_t kind = 0, n = 0, M = 0, npair = 0, nalpha = 0, nbeta = 0, max_roots = 1;
    int64_t ndet = 0;
    double ecore = 0.0;
    bool cplx = false;
    std::vector<uint64_t> dets;
    std::vector<uint32_t> grp_off;
    std::vector<uint64_t> grp_key;
    std::vector<uint8_t> grp_type;
    std::vector<uint2> mem;
    std::vector<uint32_t> mem_grp, slot_mem, pk_off, rowptr, grp_col;
    // position of each logical partial slot (membership, then column partials)
    std::vector<uint32_t> slot_pos;
    int64_t ncol = 0;  // column partial sums of large double groups
    std::vector<double> h, w_same, w_opp, g_ab, a_pair, a_pair1, f_ref;
    // spinor plans: Table 1's |(ab|cd)| over Kramers pairs (see bound_table)
    std::vector<double> g_bound;
    uint64_t ref0 = 0, ref1 = 0;
    int64_t npacket_double = 0, nmem_double = 0;
    // density-matrix rows (see build_rdm_rows)
    std::vector<uint2> rdm_ent;
    std::vector<uint4> rdm_chunk;
    std::vector<uint16_t> rdm_pos;
    std::vector<uint32_t> rdm_ent_det;
    std::vector<ulonglong2> rdm_skey;
    int64_t rdm_single_e0 = 0;
    int64_t rdm_cls[6] = {0, 0, 0, 0, 0, 0};
    // launch defaults until mw_autotune picks its own: partner-loop unroll 4,
    // 16 gather lanes (32 for complex), the fastest measured on the n = 64
    // spin-free and 40-pair spinor spaces for one, two and four roots
    int32_t tune_u = 4, tune_gl = 0;
    int32_t rdm_fixed = 0;
    int64_t n_single_pairs = 0, n_double_pairs = 0, n_evals = 0;
    // ordered double pairs inside groups of 64 members or more, which the
    // double-group kernel evaluates once per unordered pair
    int64_t n_double_pairs_large = 0;
    // index arrays built on the device (mw_plan_create_device), moved into
    // the workspace by the first upload
    DevIndex dix;
    bool moved = false;  // a device-built index already copied into a workspace
    // device binding
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    DevPlan dev{};
    size_t layout(DevPlan *d, char *base) const;
    Counts counts() const;
    size_t scalar_bytes() const { return cplx ? 16 : 8; }
};

// Build the grouping, packets, partial-sum placement and density rows of P
// (whose space, kind and root count are set) on the current device: the
// same arrays, bit for bit, as the host build.  Temporary device memory is
// allocated and freed here; the index stays in P.dix.
mw_status build_index_device(HostPlan &P, hipStream_t s);

}  // namespace mw
