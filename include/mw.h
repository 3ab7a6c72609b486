/*
 * mw.h - C ABI of libmw: the Hamiltonian-vector product sigma = H c over a
 * (selected) space of Slater determinants on one MI355X (gfx950) GPU.
 *
 * H is the generic second-quantised Hamiltonian of MetaWave (section 2.1,
 * Eq. (1)):  H = sum_PQ h_PQ a+_P a_Q + 1/2 sum_PQRS (PQ|RS) a+_P a+_R a_S a_Q,
 * Mulliken notation, with the operator symmetries of Eq. (2).  Matrix
 * elements between determinants are never stored: every call recomputes them
 * from occupation bitstrings and integrals (section 2.4, last paragraph on
 * diagonalisation through sigma = H X).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Determinant: two 64-bit words {w0, w1}.  Spin-free (MW_SPIN_FREE, tag
 * "nonrelativistic"): w0 = alpha string, w1 = beta string, spatial orbital p
 * at bit p.  Spinor (MW_SPINOR, Kramers pairs of section 2.1): w0 = unbarred
 * (A) spinors, w1 = barred (B) spinors, pair k at bit k.  The global position
 * of word w, bit b is w*norb + b, and |D> = prod_{P in D, ascending} a+_P |vac>
 * (all of w0 before w1).  The space is strictly ascending as unsigned 128-bit
 * keys with w0 the more significant word.
 *
 * Scalars: spin-free problems are real FP64; spinor problems are complex128
 * stored as interleaved (re, im) doubles.  CI vectors c and sigma are laid
 * out [ndet][nroots] (roots contiguous), in that scalar type.
 *
 * Memory ownership: problem data (dets, h, g) are HOST pointers read only
 * during mw_plan_create (or mw_plan_create_device).  Every other buffer
 * argument is a DEVICE pointer owned by the caller unless marked host.  A
 * plan lives in a caller-provided device workspace; libmw allocates device
 * memory only inside mw_plan_create_device (its sort temporaries, freed
 * before it returns, and the index it hands to the first mw_plan_upload,
 * freed there).
 *
 * Streams: device work is enqueued on the given hipStream_t (0 = default
 * stream) and is asynchronous unless stated otherwise.
 *
 * Errors: every call returns an mw_status; on failure nothing has been
 * enqueued unless stated, outputs are unspecified and mw_last_error() gives
 * a message (thread-local).  No C++ exception crosses the ABI.
 */
#ifndef MW_H
#define MW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *mw_stream_t; /* a hipStream_t */

typedef enum {
    MW_OK = 0,
    MW_EINVAL = -1,       /* bad argument (null pointer, size, nroots...) */
    MW_ENOTSORTED = -2,   /* determinants not strictly ascending          */
    MW_EELEC = -3,        /* wrong electron count or bits beyond norb      */
    MW_ESYM = -4,         /* integrals violate the required symmetry       */
    MW_EWORKSPACE = -5,   /* workspace missing, too small or misaligned    */
    MW_EHIP = -6,         /* a HIP runtime call failed                     */
    MW_ENOCONV = -7,      /* Davidson did not converge (best result kept)  */
    MW_EUNSUPPORTED = -8  /* outside the supported sizes                   */
} mw_status;

typedef enum { MW_SPIN_FREE = 0, MW_SPINOR = 1 } mw_kind;

typedef struct {
    int32_t kind;        /* mw_kind                                               */
    int32_t norb;        /* spatial orbitals (spin-free) or Kramers pairs (spinor), 1..64 */
    int32_t nalpha;      /* spin-free: N_alpha; spinor: total electron count N     */
    int32_t nbeta;       /* spin-free: N_beta;  spinor: must be -1                 */
    int64_t ndet;        /* number of determinants, 1 .. 2^31-1                    */
    const uint64_t *dets;/* HOST [ndet][2], see conventions                        */
    const double *h;     /* HOST one-body integrals h_PQ.  Spin-free: real [n][n].
                            Spinor: complex [M][M], M = 2n (A_k at k, B_k at n+k)  */
    const double *g;     /* HOST two-body integrals (PQ|RS) at [((P*m+Q)*m+R)*m+S],
                            m = n (spin-free, real) or M (spinor, complex)         */
    double ecore;        /* constant added to every diagonal element               */
} mw_problem;

typedef struct mw_plan_s *mw_plan;

/* Build a plan for a problem (section 2.3: classify determinant pairs by the
 * part they share and group them, so that pairs of one group reuse the same
 * integrals).  Host-side only: validates the problem, groups determinants by
 * the (N-1)- and (N-2)-electron strings they contain, repacks the integrals
 * and allocates HOST memory for the result.  Checks: norb in 1..64, electron
 * counts per determinant (MW_EELEC), strictly ascending dets (MW_ENOTSORTED),
 * h Hermitian, (PQ|RS) = (RS|PQ) = conj((QP|SR)) and, for spin-free
 * problems, the real 8-fold symmetry, all to 1e-12 relative (MW_ESYM).
 * max_roots (>= 1) bounds nroots of later calls.  *out receives the plan. */
mw_status mw_plan_create(const mw_problem *prob, int32_t max_roots, mw_plan *out);

/* The same plan with its grouping built on the current device (section 2.3
 * grouping, done as radix sorts of the (N-1)/(N-2)-electron strings, scans
 * and per-group kernels): the determinants, packets, partial-sum placement
 * and density-matrix rows come out bit for bit as mw_plan_create's, so
 * every product of the plan is bitwise the same.  Validation and the
 * integral repacking stay on the host.  Allocates temporary DEVICE memory
 * (about 24 bytes per string entry, N (n_e + n_e (n_e - 1) / 2) entries for
 * n_e electrons) and keeps the index in device allocations owned by the
 * plan until the first mw_plan_upload copies it into the workspace and
 * frees them; such a plan is uploaded once (a second upload returns
 * MW_EINVAL).  Runs on `stream` and synchronises it.  MW_EUNSUPPORTED when
 * the entries reach 2^32 or a group exceeds 2^20 members (the host build
 * has neither limit), MW_EHIP on a failed allocation or launch. */
mw_status mw_plan_create_device(const mw_problem *prob, int32_t max_roots, mw_stream_t stream, mw_plan *out);

/* Where index array `which` of a bound plan lives in its workspace: byte
 * offset and size (host outs), to compare plans or read them back.  which =
 * 0 group offsets, 1 group strings, 2 group kinds, 3 column-partial starts,
 * 4 memberships, 5 membership groups, 6 determinant-major slot lists, 7 slot
 * positions, 8 packet offsets, 9 slot-list row pointers, 10 density-row
 * entries, 11 density-row chunks, 12 density-row positions, 13 density-row
 * determinants, 14 density-row single strings.  MW_EINVAL for an unbound
 * plan or an index outside 0..14. */
mw_status mw_plan_array(mw_plan plan, int32_t which, size_t *offset, size_t *bytes);

/* Device workspace size (bytes, host out) the plan needs, including the
 * per-call scratch for max_roots roots. */
mw_status mw_plan_workspace_bytes(mw_plan plan, size_t *bytes);

/* Bind the plan to a device workspace of at least mw_plan_workspace_bytes
 * bytes, 256-byte aligned, and upload its tables; computes the diagonal H_II
 * on the device.  Synchronises the stream before returning.  The workspace
 * must stay allocated and untouched until mw_plan_destroy or a new upload.
 * A plan is bound to one workspace at a time and must not be used from two
 * streams concurrently. */
mw_status mw_plan_upload(mw_plan plan, void *workspace, size_t bytes, mw_stream_t stream);

/* Replace the integrals (and ecore) of a bound plan without regrouping the
 * determinants: validates them as mw_plan_create does, repacks them into the
 * workspace and recomputes the diagonal.  h, g are HOST pointers laid out as
 * in mw_problem.  Synchronises the stream.  Used when the same space is
 * evaluated for several Hamiltonians (finite differences, orbital updates). */
mw_status mw_plan_update_integrals(mw_plan plan, const double *h, const double *g, double ecore,
                                   mw_stream_t stream);

/* Free the plan's host memory (the workspace stays the caller's). */
mw_status mw_plan_destroy(mw_plan plan);

/* Plan statistics (host): what = 0 ndet, 1 number of groups (buckets),
 * 2 memberships, 3 structurally connected ordered pairs I != J, 4 pairs of
 * single excitations, 5 pairs of double excitations, 6 determinant-pair
 * evaluations per sigma (including the discarded ones), 7 workspace bytes,
 * 8 scalar size in bytes (8 or 16), 9 norb, 10 kind, 11 packets (waves of
 * the group launches), 12 packets of double groups, 13 column partial sums
 * of the large double groups, 14 ordered double-excitation pairs inside
 * groups of 64 members or more (evaluated once per unordered pair), 15
 * double memberships listed under the density-matrix rows of their added
 * pairs, 16 chunks of those lists (workgroups of the double-pair density
 * kernel), 17 1 when the grouping was built on the device, else 0,
 * 18 the density-matrix mode (mw_plan_set_rdm_mode).
 * Returns -1 for an unknown plan or index. */
int64_t mw_plan_info(mw_plan plan, int32_t what);

/* sigma_I = sum_J H_IJ c_J for nroots (1..max_roots) vectors: the product of
 * section 2.4 over the nonzero elements of H, recomputed on every call.
 * c, sigma: device [ndet][nroots] scalars; they must not overlap.
 * Enqueues the product on stream; bitwise reproducible between calls. */
mw_status mw_sigma(mw_plan plan, int32_t nroots, const void *c, void *sigma, mw_stream_t stream);

/* The same product for nprob (1..32) independent plans of one kind in one
 * launch sequence: per root-chunk width one launch over the work units of
 * all problems (a persistent grid whose waves pull them from per-XCD device
 * counters, the dynamic task scheduling of the paper's parallel templates,
 * section 3.1.2, or a flat grid, as tuned), then one gather launch.
 * plans, nroots, c, sigma are HOST arrays of length nprob (c[i], sigma[i]
 * device pointers; each plan at most once).  The launch sequence is captured
 * once into a HIP graph keyed by the argument tuple and replayed on later
 * calls with the same tuple (at most 16 graphs are kept, the least recently
 * used dropped first); destroying or re-binding a plan drops its graphs.  With the default launch parameters results equal nprob separate
 * mw_sigma calls with default parameters bit for bit; a tuned gather width
 * sums each determinant's partials in another fixed order. */
mw_status mw_sigma_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                           const void *const *c, void *const *sigma, mw_stream_t stream);

/* The batched product with an explicit persistent grid (blocks_per_cu x the
 * number of compute units, each wave pulling packets from per-XCD work
 * queues) or, with blocks_per_cu = 0, one hardware-dispatched wave per
 * packet of all problems; launched directly without graph capture. */
mw_status mw_sigma_batched_direct(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                                  const void *const *c, void *const *sigma, int32_t blocks_per_cu,
                                  mw_stream_t stream);

/* Autotuner for mw_sigma: times the partner-loop unroll (4, 8, 16) and the
 * gather width (8, 16, 32 lanes per determinant) on the caller's vectors and
 * keeps the fastest in the plan; *choice (host, nullable) = unroll*100+lanes.
 * Overwrites sigma; synchronises the stream. */
mw_status mw_autotune(mw_plan plan, int32_t nroots, const void *c, void *sigma, mw_stream_t stream,
                      int32_t *choice);

/* The launch parameters of mw_sigma as one code, unroll * 100 + lanes (the
 * value mw_autotune reports), so that a tuned choice can be kept with the
 * problem and restored without timing again: mw_plan_get_tuning writes the
 * plan's current code to *code (host), mw_plan_set_tuning sets it (unroll
 * 4, 8 or 16, 16 for real plans only; lanes 8, 16 or 32; MW_EINVAL
 * otherwise).  Host only; results do not depend on the choice. */
mw_status mw_plan_get_tuning(mw_plan plan, int32_t *code);
mw_status mw_plan_set_tuning(mw_plan plan, int32_t code);

/* Autotuner for mw_sigma_batched: times the flat grid and persistent grids
 * of 1, 2, 4, 8, 16 blocks per compute unit, a partner unroll of 4 or 8 for
 * four-root passes and a gather width of 8, 16 or 32 lanes per determinant,
 * for this argument tuple, and uses the fastest for its graph from then on;
 * *blocks_per_cu (host, nullable) receives the grid (0 = flat). */
mw_status mw_autotune_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots,
                              const void *const *c, void *const *sigma, mw_stream_t stream,
                              int32_t *blocks_per_cu);

/* Diagonal H_II (device [ndet] scalars, imaginary part zero for spinor). */
mw_status mw_diag(mw_plan plan, void *out, mw_stream_t stream);

/* Transition density matrices, the adjoint of sigma with respect to the
 * integrals (density matrices are listed among the paper's functionality,
 * section 3.4):  gamma_PQ = sum_k w_k sum_IJ conj(bra_Ik) ket_Jk <I|a+_P a_Q|J>,
 * Gamma_PQRS = sum_k w_k sum_IJ conj(bra_Ik) ket_Jk <I|a+_P a+_R a_S a_Q|J>.
 * Spin-free results are spin-summed over spatial orbitals: gamma [n][n],
 * Gamma [n][n][n][n] real; spinor: [M][M] and [M]^4 complex.  bra, ket
 * device [ndet][nroots]; weights HOST [nroots] or NULL (all 1); gamma, Gamma
 * device outputs, overwritten.  For E = c^H H c, dE/dh = gamma and dE/dg =
 * Gamma / 2.  Connectivity is recomputed, never stored.  The plan's
 * density-matrix mode (mw_plan_set_rdm_mode) decides how contributions are
 * summed: floating-point atomics (default; reproducible to rounding, not
 * bitwise) or 64-bit fixed point (the same bits on every call).  When bra and ket are
 * the same pointer, each unordered pair is visited once and the reversed
 * pair's contribution (the complex conjugate) is added in the final pass:
 * the same matrices to rounding, half the atomics. */
mw_status mw_rdm_backward(mw_plan plan, int32_t nroots, const void *bra, const void *ket,
                          const double *weights, void *gamma, void *Gamma, mw_stream_t stream);

/* Density-matrix mode of the plan, for mw_rdm_backward, mw_energy_backward,
 * mw_sigma_backward and the batched backward.  The sums of section 3.4's
 * density matrices over connected pairs are order-independent in exact
 * arithmetic; in floating point the atomics make them depend on arrival
 * order.  mode 0 (default): floating-point atomics.  mode 1: every
 * contribution v is rounded to the integer nearest v 2^s and summed with
 * 64-bit integer atomics (exact and associative, also where a partial sum
 * wraps), then scaled back by 2^-s, so the results do not depend on the
 * order of arrival, the launch configuration or stream overlap: the same
 * inputs give the same bits.  s is set per call on the device from
 * B = max_k |w_k| ||bra||_F ||ket||_F, which bounds every accumulated entry:
 * s = 60 - e for B in [2^(e-1), 2^e), so each contribution is rounded to
 * at most B 2^-60 (absolute).  The norms are computed as a largest
 * magnitude times a scaled sum of squares, so no square overflows or
 * underflows; scaling bra or ket by a power of two scales the results
 * exactly.  Host only; MW_EINVAL for other modes. */
mw_status mw_plan_set_rdm_mode(mw_plan plan, int32_t mode);

/* Energies e_k = Re sum_I conj(c_Ik) sigma_Ik (the expectation value
 * c^H H c of section 2.4 when sigma = H c, unnormalised), one per root:
 * c, sigma device [ndet][nroots]; e device [nroots] doubles, overwritten.
 * A two-stage reduction in a fixed order (block partials in the plan's
 * per-call scratch, so it must not overlap another call on the plan):
 * repeated calls give the same bits.  Asynchronous on stream. */
mw_status mw_energy(mw_plan plan, int32_t nroots, const void *c, const void *sigma, double *e, mw_stream_t stream);

/* Gradients of the energies E_k = c_k^H H c_k weighted by the upstream
 * gradients ge (device [nroots] doubles), L = sum_k ge_k E_k:
 *   grad_c[I][k] = 2 ge_k sigma[I][k]          (sigma = H c from mw_sigma)
 *   grad_h = sum_k ge_k gamma_k,  grad_g = 1/2 sum_k ge_k Gamma_k
 * with gamma_k, Gamma_k the density matrices of root k (as mw_rdm_backward
 * with bra = ket = c), since E = sum h gamma + 1/2 sum (PQ|RS) Gamma for
 * Eq. (1).  Complex problems: grad_h and grad_g are conjugated (gradient of
 * a real loss w.r.t. complex inputs, dL = Re sum conj(grad) dz).
 * grad_c device [ndet][nroots] or NULL (then sigma may be NULL); grad_h
 * [M][M] and grad_g [M]^4 (M = n spin-free, 2n spinor) both device or both
 * NULL.  Connectivity is recomputed; uses the plan's per-call scratch.
 * Asynchronous on stream; device atomics make the integral gradients
 * reproducible to rounding. */
mw_status mw_energy_backward(mw_plan plan, int32_t nroots, const void *c, const void *sigma, const double *ge,
                             void *grad_c, void *grad_h, void *grad_g, mw_stream_t stream);

/* Vector-Jacobian products of sigma = H c for an upstream gradient gs
 * (device [ndet][nroots], the gradient of a loss with respect to sigma):
 *   grad_c = H gs  (H Hermitian),
 *   grad_h = conj(gamma(gs, c)),  grad_g = 1/2 conj(Gamma(gs, c))
 * with gamma(gs, c), Gamma(gs, c) the transition density matrices of
 * mw_rdm_backward with bra = gs, ket = c, summed over the roots
 * (conjugation only for complex problems).  grad_c device [ndet][nroots]
 * or NULL (must not overlap gs); grad_h, grad_g both device or both NULL.
 * Uses the plan's per-call scratch; asynchronous on stream. */
mw_status mw_sigma_backward(mw_plan plan, int32_t nroots, const void *c, const void *gs, void *grad_c, void *grad_h,
                            void *grad_g, mw_stream_t stream);

/* Batched energies and gradients (the differentiable batched path):
 * nprob (1..32) plans, each at most once; plans, nroots and every pointer
 * array are HOST arrays of length nprob whose entries are device pointers
 * laid out as for mw_energy / mw_energy_backward.
 * mw_energy_batched: e[i][k] = Re c_i,k^H sigma_i,k for every problem
 * (after mw_sigma_batched), launched directly.
 * mw_energy_backward_batched: mw_energy_backward for every problem (grad_c,
 * grad_h, grad_g of L = sum_k ge[i][k] E_i,k; each entry may be NULL as for
 * the single call).  The launch sequence of all problems is captured once
 * into a HIP graph keyed by the argument tuple and replayed on later calls
 * with the same tuple (at most 16 graphs are kept, the least recently used
 * dropped first; destroying or re-binding a plan drops its graphs), so the
 * many small kernels of the density-matrix passes cost one launch. */
mw_status mw_energy_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots, const void *const *c,
                            const void *const *sigma, double *const *e, mw_stream_t stream);
mw_status mw_energy_backward_batched(int32_t nprob, const mw_plan *plans, const int32_t *nroots, const void *const *c,
                                     const void *const *sigma, const double *const *ge, void *const *grad_c,
                                     void *const *grad_h, void *const *grad_g, mw_stream_t stream);

/* Lowest nroots eigenpairs by block Davidson-Liu over mw_sigma (section 2.4
 * uses sigma = H X products for the diagonalisation).  c0: device
 * [ndet][nroots] start vectors (orthonormalised internally).  work: device
 * scratch of mw_davidson_work_bytes bytes.  c_out: device [ndet][nroots]
 * Ritz vectors; evals: HOST [nroots]; iters: HOST.  Convergence when every
 * residual 2-norm <= tol; subspace collapse above max(8 nroots, 24) vectors.
 * Host-driven, synchronises once per iteration.  Returns MW_ENOCONV with
 * the best vectors and values when max_iter is reached. */
mw_status mw_davidson_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes);
mw_status mw_davidson(mw_plan plan, int32_t nroots, const void *c0, void *c_out, double *evals,
                      double tol, int32_t max_iter, int32_t *iters, void *work, size_t work_bytes,
                      mw_stream_t stream);

/* Iterative vector interaction (section 2.4: trial vectors from
 * perturbation theory and conjugate gradients, a search space of fixed
 * dimension set by the number of roots, direct access to interior roots).
 * The space holds the current R vectors X, their first-order corrections
 * t_k = (r_k - eps_k x_k) / (theta_k - H_II) (r_k the residual, eps_k
 * Olsen's: t_k orthogonal to x_k) and the previous step's
 * directions (the part of the new X outside the old one), 3R vectors at
 * most; each step diagonalises H there and keeps R Ritz pairs: the lowest
 * when target is NaN, otherwise the R nearest target (energy-selected), so
 * roots below the target are never computed.  c0: device [ndet][nroots]
 * start vectors (orthonormalised internally; for a target, e.g. unit
 * vectors on the determinants whose H_II is nearest it); c_out: device
 * [ndet][nroots] Ritz vectors; evals, iters: HOST.  Convergence when every
 * residual 2-norm <= tol.  work: device scratch of mw_ivi_work_bytes
 * bytes, 256-byte aligned (4 nroots vectors and their H products).
 * Host-driven, synchronises once per step; MW_ENOCONV with the last Ritz
 * pairs when max_iter is reached.  Interior roots need a diagonally
 * dominant H (the corrections divide by theta - H_II) and a target whose
 * roots are separated from their neighbours; inside a dense cluster of
 * eigenvalues the energy selection can move between states of the
 * cluster and the iteration may not converge. */
mw_status mw_ivi_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes);
mw_status mw_ivi(mw_plan plan, int32_t nroots, double target, const void *c0, void *c_out, double *evals,
                 double tol, int32_t max_iter, int32_t *iters, void *work, size_t work_bytes, mw_stream_t stream);

/* Epstein-Nesbet second-order energies (section 2.5, Eq. (ENPT2E), with
 * the primary space equal to the plan's space P):
 *   e2[k] = sum_{A in Q} |sum_{J in P} H_AJ c[J][k]|^2 / (e0[k] - H_AA),
 * Q = every determinant outside P that one or two excitations reach from a
 * J of P (spin-free: N_alpha and N_beta kept).  Screening as in the paper's
 * PT2 procedure (step 4): the pair (A, J) is left out when the configuration
 * of A (orbital or Kramers-pair occupations 0/1/2) is doubly excited from
 * that of J and Table 1's upper bound H~ (SD column, IntC 1-7; spinor: the
 * largest integral over the Kramers partners) is below qmin / max |c[nu][k]|
 * over the determinants nu of J's configuration and the roots (qmin = 0
 * keeps every pair).
 * c: device [ndet][nroots] (complex for spinor plans), 1 <= nroots <= 8;
 * e0, e2: HOST [nroots].  work: device scratch of work_bytes bytes; the
 * connections are generated in passes over hash buckets of A sized to fit
 * it (mw_pt2_work_bytes gives the size for one pass without screening when
 * no bucket exceeds 1024 records; a larger bucket, of any size, is sorted in
 * 12 bytes of scratch per position of its power-of-two range; less memory
 * means more passes; MW_EWORKSPACE if too small for the bucket tables or
 * one bucket).  stats: HOST int64[5], nullable: kept (A, J)
 * pairs with A in Q, number of A in Q, passes, buckets, excitations
 * enumerated per pass (ndet x singles and doubles of one determinant).
 * Host-driven, synchronises the stream; repeated calls give identical bits.
 * Testing knob: the environment variable MW_PT2_KEY_BITS (1..31) keeps only
 * that many hash bits of A in the records' sort key, so that many external
 * determinants share a run (the result is the same to rounding). */
mw_status mw_pt2_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes);
mw_status mw_pt2(mw_plan plan, int32_t nroots, const void *c, const double *e0, double qmin, void *work,
                 size_t work_bytes, double *e2, int64_t *stats, mw_stream_t stream);

/* Selection of external determinants by the iCIPT2 criterion (section 2.4,
 * Eqs. (iCI_Selection-1) and (iCI_Selection-2)): A outside the plan's space
 * P, reached from P by one or two excitations, is selected when for some
 * configuration J of P, with nu over J's determinants in P,
 *   max_{nu,k} |H_A,nu c[nu][k]| >= cmin  and
 *   max_{nu,k} |H_A,nu c[nu][k] / (e0[k] - H_AA)| >= cmin
 * and, when A's configuration is doubly excited from J's (case B),
 *   H~ max_{nu,k} |c[nu][k]| >= cmin  (Table 1's bound, as for mw_pt2).
 * c: device [ndet][nroots] (complex for spinor plans), 1 <= nroots <= 8;
 * e0: HOST [nroots].  work / work_bytes: device scratch as for mw_pt2 (the
 * size mw_pt2_work_bytes gives is enough for one pass).  out: device
 * [max_out][2] uint64 receiving the distinct selected determinants (grouped
 * by hash bucket, sorted within a bucket; the same order on every call);
 * *count (HOST) = how many were selected; when it exceeds max_out only the
 * first max_out are written.  Host-driven, synchronises the stream. */
mw_status mw_select(mw_plan plan, int32_t nroots, const void *c, const double *e0, double cmin, void *work,
                    size_t work_bytes, uint64_t *out, int64_t max_out, int64_t *count, mw_stream_t stream);

/* Spin-adapted basis: configuration state functions (section 2.3: an orbital
 * configuration generates several CSFs, told apart by their spin coupling,
 * with the Yamanouchi-Kotani phase; section 2.2 stores a configuration as its
 * doubly and singly occupied orbitals).  Built over the configurations of a
 * spin-free plan's determinants at M_S = S, 2S = N_alpha - N_beta.
 * Configuration (d_1 < .. < d_m doubly occupied, o_1 < .. < o_k open); CSF mu =
 *   sum_s Theta_mu(s) a+_{d_1 alpha} a+_{d_1 beta} .. a+_{d_m beta} a+_{o_1 s_1} .. a+_{o_k s_k} |vac>,
 * Theta_mu the genealogical spin function of coupling path mu (intermediate
 * spins S_1 .. S_k = S, one spin 1/2 added at a time with Condon-Shortley
 * Clebsch-Gordan coefficients), written in the plan's determinants (the sign
 * of reordering the operators into ascending positions included).
 * Numbering: configurations in the order of their first determinant; the
 * paths of one configuration lexicographically, step up before step down.
 * With T [ndet][ncsf] that expansion, the calls below give T x, T^T y and
 * sigma_CSF = T^T H T c, which equals the Hamiltonian in the CSF basis
 * applied to c because the space holds every determinant of each of its
 * configurations (checked).
 *
 * mw_csf_create (host only): plan from mw_plan_create (spin-free), two_s =
 * N_alpha - N_beta >= 0.  MW_EINVAL if 2S differs or a configuration lacks
 * one of its C(k, (k + 2S)/2) determinants; MW_EUNSUPPORTED for spinor
 * plans, more than 14 open shells in a configuration, or more than 2^31 - 1
 * determinants or CSFs.  The CSF basis keeps the plan handle: the plan must
 * outlive it.
 * mw_csf_info: 0 ncsf, 1 configurations, 2 largest open-shell count,
 * 3 workspace bytes, 4 coupling-table entries, 5 ndet; -1 otherwise.
 * mw_csf_upload: binds a device workspace (>= mw_csf_workspace_bytes,
 * 256-byte aligned, caller-owned, untouched until destroy) and copies the
 * tables; synchronises the stream.
 * mw_csf_to_det: y [ndet][nroots] = T x, x [ncsf][nroots] (device, FP64).
 * mw_csf_from_det: x [ncsf][nroots] = T^T y.
 * mw_csf_sigma: sigma [ncsf][nroots] = T^T H T c; work: device scratch of
 * 2 ndet nroots doubles; the plan must be uploaded and nroots <= its
 * max_roots.  Asynchronous on stream; repeated calls give identical bits. */
typedef struct mw_csf_s *mw_csf;
mw_status mw_csf_create(mw_plan plan, int32_t two_s, mw_csf *out);
int64_t mw_csf_info(mw_csf csf, int32_t what);
mw_status mw_csf_workspace_bytes(mw_csf csf, size_t *bytes);
mw_status mw_csf_upload(mw_csf csf, void *workspace, size_t bytes, mw_stream_t stream);
mw_status mw_csf_to_det(mw_csf csf, int32_t nroots, const double *x, double *y, mw_stream_t stream);
mw_status mw_csf_from_det(mw_csf csf, int32_t nroots, const double *y, double *x, mw_stream_t stream);
mw_status mw_csf_sigma(mw_csf csf, int32_t nroots, const double *c, double *sigma, double *work,
                       mw_stream_t stream);
mw_status mw_csf_destroy(mw_csf csf);

/* mw_csf_sigma without a work argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  T c and H T c go to a static device array of
 * 2^22 doubles (32 MiB) that the library holds on each device it runs on
 * until the process ends; its address is taken once per device, on the
 * first call with that device current (the device of the CSF basis and its
 * plan).  Limit: 2 ndet nroots <= 2^22, else MW_EWORKSPACE and nothing is
 * enqueued.  Calls no allocating routine.  Every call on a device shares
 * that device's array: calls that overlap on one device (two streams, two
 * threads) race and give wrong results; calls in one stream are ordered.
 * The same results as mw_csf_sigma, bit for bit. */
mw_status mw_csf_sigma_noalloc(mw_csf csf, int32_t nroots, const double *c, double *sigma, mw_stream_t stream);

/* Lowest nroots eigenpairs of the Hamiltonian in the CSF basis (spin-pure
 * states of spin S): the block Davidson-Liu of mw_davidson over
 * mw_csf_sigma, preconditioned with D_mu = sum_I T_I,mu^2 H_II.  c0, c_out:
 * device [ncsf][nroots] FP64; evals, iters: HOST.  work: device scratch of
 * mw_csf_davidson_work_bytes bytes, 256-byte aligned (Davidson vectors over
 * the CSFs, two determinant vectors per root and the diagonal).  Both the
 * CSF basis and its plan must be uploaded; nroots <= the plan's max_roots.
 * Host-driven, synchronises once per iteration; MW_ENOCONV with the best
 * vectors and values when max_iter is reached. */
mw_status mw_csf_davidson_work_bytes(mw_csf csf, int32_t nroots, size_t *bytes);
mw_status mw_csf_davidson(mw_csf csf, int32_t nroots, const double *c0, double *c_out, double *evals, double tol,
                          int32_t max_iter, int32_t *iters, void *work, size_t work_bytes, mw_stream_t stream);

/* The iterative vector interaction of mw_ivi (same search space, selection
 * and stop) in the CSF basis: spin-pure lowest roots (target NaN) or the
 * spin-S roots nearest target, preconditioned as mw_csf_davidson.  c0,
 * c_out: device [ncsf][nroots]; work: mw_csf_ivi_work_bytes bytes. */
mw_status mw_csf_ivi_work_bytes(mw_csf csf, int32_t nroots, size_t *bytes);
mw_status mw_csf_ivi(mw_csf csf, int32_t nroots, double target, const double *c0, double *c_out, double *evals,
                     double tol, int32_t max_iter, int32_t *iters, void *work, size_t work_bytes, mw_stream_t stream);

/* Debug: connected pairs of all rows with their phases, as int64 records
 * [I, J, P, Q, R, S, sign] (R = S = -1 for singles; P, R particles in I; Q, S
 * holes in J; ascending within each pair).  Call with out = NULL to get the
 * count in *count (host); then with a device buffer of 7*count int64.
 * Synchronises the stream.  Order of records is unspecified. */
mw_status mw_connect_dump(mw_plan plan, int64_t *count, int64_t *out, mw_stream_t stream);

/* Optional timing: while enabled, every kernel launch of the calls above is
 * bracketed by HIP events recorded on its stream ("group_sigma",
 * "group_single", "gather", "rdm_double", "rdm_single", "rdm_diag",
 * "batched_groups", "batched_gather", "pt2_enum", "pt2_bucket",
 * "pt2_bucket_big", "sel_unique_big").  Enabling
 * clears earlier records.  mw_profile_read synchronises on the recorded
 * events and returns the number of launches and their summed duration (ms,
 * host outputs) for one kernel name. */
mw_status mw_profile(int32_t enable);
mw_status mw_profile_read(const char *kernel, int64_t *launches, double *total_ms);

/* Thread-local description of the last error (never NULL). */
const char *mw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MW_H */
