// Internal declarations shared by the host plan builder and the HIP kernels
// of libmw.  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/mw.h"

namespace mw {

// Group (bucket) kinds.  A single group collects the determinants that
// contain one (N-1)-electron string K; a double group those that contain one
// (N-2)-electron string.  Two members of a double group whose added pairs are
// disjoint differ by exactly that double excitation, and K is their common
// part; two members of a single group differ by a single excitation.
enum GroupType : uint8_t {
    G_SINGLE_A = 0,   // spin-free, added orbital alpha
    G_SINGLE_B = 1,   // spin-free, added orbital beta
    G_AA = 2,         // spin-free double, both added orbitals alpha
    G_AB = 3,         // spin-free double, one alpha one beta
    G_BB = 4,         // spin-free double, both beta
    G_SINGLE_S = 5,   // spinor single
    G_DOUBLE_S = 6,   // spinor double
};

// Device-side view of a plan (all pointers inside the workspace).
struct DevPlan {
    int32_t kind;          // mw_kind
    int32_t n;             // norb
    int32_t M;             // 2 n global positions
    int32_t npair;         // pairs of same-spin orbitals (spin-free) or of spinors
    int64_t ndet;
    int64_t nmem;          // memberships
    int64_t npacket;
    int32_t max_roots;
    double ecore;
    // groups
    const uint32_t *grp_off;   // [ngroup+1] first member of each group
    const uint64_t *grp_key;   // [ngroup][2] the shared string K
    const uint8_t *grp_type;   // [ngroup]
    const uint32_t *grp_col;   // [ngroup] first column partial of a large double group
    int64_t ncol;              // column partials (stored after the nmem row partials)
    // members (group-major)
    const uint2 *mem;          // [nmem] {det, X | Y<<8 | (phi<0)<<16 | layout<<17}
    const uint32_t *mem_grp;   // [nmem] owning group
    const uint32_t *slot_mem;  // partial-sum positions listed determinant by determinant
    const uint32_t *slot_pos;  // [nmem + ncol] position of each logical partial slot
    const uint32_t *pk_off;    // [npacket+1] packets of <= 64 consecutive members
    // determinants
    const uint32_t *rowptr;    // [ndet+1] range of each determinant in slot_mem
    const uint64_t *dets;      // [ndet][2]
    void *diag;                // [ndet] scalar (written at upload)
    // integrals (scalar = double or double2)
    const void *h;             // [M'][M'] (spin-free n x n; spinor M x M)
    const void *w_same;        // singles table [R][P][Q]: (PQ|RR) - (PR|RQ)  (spin-free n^3, spinor M^3)
    const void *w_opp;         // spin-free only: [r][p][q] (pq|rr)
    const void *g_ab;          // spin-free only: [q][s][p][r] = (pq|rs); by (pq|rs) = (rs|pq),
                               // [s][q][r][p] holds the same value (transposed column order)
    const void *a_pair;        // antisymmetrised pairs [x][y] = (X0 Y0|X1 Y1) - (X0 Y1|X1 Y0), y colex
    const void *a_pair1;       // same values with the column pair y in lexicographic order
    const void *f_ref;         // F^omega (spin-free [2][n][n] by spin of the group; spinor [M][M])
    const double *g_bound;     // spinor: Table 1 bound table [n]^4 over Kramers pairs; spin-free: null
    uint64_t ref0, ref1;       // reference string omega
    int64_t npacket_double;    // packets [0, npacket_double) hold double groups
    int64_t nmem_double;       // memberships [0, nmem_double) belong to double groups
    // density-matrix rows: each double membership j (as the partner of a
    // pair) listed under the accumulator row of its added pair, {j0, (j -
    // j0) | L << 16} with [j0, j0 + L) its group; chunks {row, flags (1:
    // alpha-beta row), first entry, end} in five classes [rdm_cls[c],
    // rdm_cls[c + 1]): alpha-beta rows of wide groups, of small groups, pair
    // rows of wide and of small groups, then the rows of the single
    // memberships (by the added orbital or spinor); rdm_pos[j] = X | Y << 8,
    // the positions added in membership j (Y = 255 for single groups);
    // rdm_ent_det[e] = the determinant of entry e's membership | sign << 31
    const uint2 *rdm_ent;
    const uint4 *rdm_chunk;
    const uint16_t *rdm_pos;
    const uint32_t *rdm_ent_det;
    // entries [rdm_single_e0, end) are single memberships: their group's
    // string K in rdm_skey[e - rdm_single_e0], and bit 15 of the entry's
    // second word set for a beta (spin-free) group
    const ulonglong2 *rdm_skey;
    int64_t rdm_single_e0;
    int64_t rdm_cls[6];
    void *partial;             // [nmem][R] per-membership partial sums, member order (also RDM accumulators)
    size_t scratch_bytes;
    DevPlan *self;             // device copy of this struct (for batched launches)
    uint32_t *counter;         // device work counter (batched launches)
    int32_t tune_u, tune_gl;   // tuned partner-loop unroll and gather lanes
    int32_t rdm_fixed;         // 1: density matrices accumulated in 64-bit fixed point (order-independent)
};

struct HostPlan;

// arguments of one batched launch (at most MW_MAXB problems)
constexpr int MW_MAXB = 32;

// copies of the single-excitation density accumulators (S, C, E) that the
// single-pair kernel spreads its atomics over
constexpr int RDM_COPIES = 32;
// density-matrix rows: groups of RDM_WIDE members or more are walked by a
// wave (a member per lane), smaller ones by one lane each; a chunk holds
// about RDM_CHUNK_WORK partner visits of one row
constexpr int RDM_WIDE = 32;
constexpr int64_t RDM_CHUNK_WORK = 1 << 17;
// fixed-point density matrices: the scale and the per-block norm partials
// of its bound, after the gathered bra coefficients in the scratch
constexpr int RDM_FX_BLOCKS = 256;
constexpr size_t RDM_FX_BYTES = 256 + RDM_FX_BLOCKS * 32;
struct BatchArgs {
    int nprob;
    const DevPlan *plans[MW_MAXB];   // device copies
    const void *c[MW_MAXB];
    void *sigma[MW_MAXB];
    int R[MW_MAXB];
    int64_t pk_start[MW_MAXB + 1];   // packet prefix over problems
    int64_t blk_start[MW_MAXB + 1];  // gather-block prefix over problems (256 threads each)
    int64_t ndet[MW_MAXB];           // determinants per problem (host side, for the gather layout)
    int64_t pkd_start[MW_MAXB + 1];  // prefix of the double-group packets over problems
    int64_t pks_start[MW_MAXB + 1];  // prefix of the single-group packets over problems
    uint32_t *counter;
};
// all problems (gather) and, per root-chunk width 4 / 2 / 1, the problems
// that have a chunk of that width (group launches; counters at +8 per class)
struct BatchSet {
    BatchArgs all;
    BatchArgs cls[3];
    int u4 = 4;  // partner unroll of the four-root launch (4 or 8)
    int gl = 16; // gather lanes per determinant (8, 16 or 32); blk_start is laid out for it
};
// lay blk_start out for gl gather lanes per determinant
void batch_set_gather(BatchSet &b, int gl);
mw_status launch_batched(const BatchSet &b, bool cplx, int blocks, hipStream_t s, bool timing);

// host side helpers (plan.cpp)
void set_error(const std::string &msg);
mw_status fail(mw_status st, const std::string &msg);

// optional event timing around launches (profile.cpp)
struct ProfToken {
    hipEvent_t a, b;
    const char *name;
};
bool prof_enabled();
ProfToken prof_begin(const char *name, hipStream_t s);
void prof_end(const ProfToken &t, hipStream_t s);
// while alive on a thread, its launches record no timing events (graph capture)
struct ProfSuppress {
    ProfSuppress();
    ~ProfSuppress();
};
// energies (energy.hip); the batched gradients replay them from a graph
mw_status launch_energy(const DevPlan &p, int R, const void *c, const void *sigma, double *e, hipStream_t s);
mw_status launch_energy_backward(const DevPlan &p, int R, const void *c, const void *sigma, const double *ge,
                                 void *grad_c, void *grad_h, void *grad_g, hipStream_t s);

// kernel launchers (kernels.hip)
mw_status launch_diag(const DevPlan &p, hipStream_t s);
mw_status launch_sigma(const DevPlan &p, int nroots, const void *c, void *sigma, hipStream_t s);
// the current device's second stream (null if it cannot be created): the
// single-group kernels of sigma and the side branch of the density-matrix
// backward share it, each with its own fork and join events, so that the
// library adds one stream per device (hardware queues are few and streams
// are spread over them in creation order)
hipStream_t device_side_stream();
mw_status launch_sigma_batched(int nprob, const DevPlan *const *plans, const int *nroots,
                               const void *const *c, void *const *sigma, hipStream_t s);
// transition density matrices; weights (host) or dev_weights (device) per
// root, nullable; Gamma is written scaled by fac_g and, when conj is set
// (complex only), gamma and Gamma are written conjugated
mw_status launch_rdm(const DevPlan &p, int nroots, const void *bra, const void *ket, const double *weights,
                     const double *dev_weights, void *gamma, void *Gamma, double fac_g, bool conj, hipStream_t s);
// While alive on a thread, launch_rdm on a stream that this thread is
// capturing puts its side branch (occupation correlations, single rows) on
// `side`, a stream that is used only inside captures, joined through the
// three events; without it a capture gets the serial order.
struct RdmCaptureSide {
    RdmCaptureSide(hipStream_t side, hipEvent_t fork, hipEvent_t xready, hipEvent_t join);
    ~RdmCaptureSide();
};
mw_status launch_connect(const DevPlan &p, int64_t *count, int64_t *out, hipStream_t s);

}  // namespace mw
