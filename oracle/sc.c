/*
 * Determinant-CI oracle, tier B: textbook Slater-Condon rules.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests and the CPU baseline can check the
 * GPU library against a plain, slow, obviously correct evaluation.  It shares
 * no code with the library.
 *
 * What it computes (MetaWave, section 2.1, Eq. (1)):
 *   H = sum_PQ h_PQ a+_P a_Q + 1/2 sum_PQRS (PQ|RS) a+_P a+_R a_S a_Q
 * between determinants of a space, sigma_I = sum_J H_IJ c_J for every root,
 * the diagonal H_II, the list of connected pairs with their phases, and the
 * transition one- and two-particle density matrices
 *   gamma_PQ   = sum_IJ conj(bra_I) ket_J <I|a+_P a_Q|J>
 *   Gamma_PQRS = sum_IJ conj(bra_I) ket_J <I|a+_P a+_R a_S a_Q|J>.
 *
 * Conventions:
 *  - A determinant is two words; global spin-orbital (spinor) position P
 *    lives in word P/n at bit P%n.  |D> = prod_{P in D, ascending} a+_P |vac>.
 *  - Spin-free: P < n is (p, alpha), P >= n is (p, beta); h_PQ and (PQ|RS)
 *    vanish unless the spins pair up as in the spin-free Hamiltonian.
 *  - Spinor: h is M x M, g is M^4 (M = 2n), complex, used as given.
 *
 * Method: for every requested row I, every J of the space is visited in
 * ascending order; the excitation level follows from the popcount of I^J;
 * the phase is counted literally, position by position.  All arithmetic is
 * FP64 (complex as explicit re/im pairs); build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cx;

static cx cx_add(cx a, cx b) { cx r = {a.re + b.re, a.im + b.im}; return r; }
static cx cx_sub(cx a, cx b) { cx r = {a.re - b.re, a.im - b.im}; return r; }
static cx cx_mul(cx a, cx b) { cx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static cx cx_conj(cx a) { cx r = {a.re, -a.im}; return r; }
static cx cx_sgn(int s, cx a) { cx r = {s * a.re, s * a.im}; return r; }
static const cx CX0 = {0.0, 0.0};

typedef struct {
    int kind;          /* 0 spin-free (real h n x n, g n^4), 1 spinor (complex M x M, M^4) */
    int n;             /* bits used per word */
    const double *h;   /* spin-free: real; spinor: interleaved re,im */
    const double *g;
    double ecore;
} ham_t;

static int spin_of(const ham_t *H, int P) { return P / H->n; }

static cx h_so(const ham_t *H, int P, int Q)
{
    int n = H->n;
    if (H->kind == 0) {
        if (spin_of(H, P) != spin_of(H, Q)) return CX0;
        cx r = {H->h[(P % n) * n + (Q % n)], 0.0};
        return r;
    }
    int M = 2 * n;
    cx r = {H->h[2 * ((size_t)P * M + Q)], H->h[2 * ((size_t)P * M + Q) + 1]};
    return r;
}

/* (PQ|RS) in the spin-orbital / spinor basis */
static cx g_so(const ham_t *H, int P, int Q, int R, int S)
{
    int n = H->n;
    if (H->kind == 0) {
        if (spin_of(H, P) != spin_of(H, Q) || spin_of(H, R) != spin_of(H, S)) return CX0;
        size_t p = P % n, q = Q % n, r = R % n, s = S % n;
        cx v = {H->g[((p * n + q) * n + r) * n + s], 0.0};
        return v;
    }
    size_t M = 2 * (size_t)n;
    size_t k = (((size_t)P * M + Q) * M + R) * M + S;
    cx v = {H->g[2 * k], H->g[2 * k + 1]};
    return v;
}

static int occupied(const uint64_t *d, int n, int P) { return (int)((d[P / n] >> (P % n)) & 1u); }

/* number of occupied positions strictly between lo and hi */
static int between(const uint64_t *d, int n, int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a, c = 0;
    for (int X = lo + 1; X < hi; X++) c += occupied(d, n, X);
    return c;
}

static int parity(int c) { return (c & 1) ? -1 : 1; }

/* positions occupied in x but not in y, ascending; returns count */
static int diff_positions(const uint64_t *x, const uint64_t *y, int n, int *out, int cap)
{
    int k = 0;
    for (int P = 0; P < 2 * n; P++)
        if (occupied(x, n, P) && !occupied(y, n, P)) {
            if (k < cap) out[k] = P;
            k++;
        }
    return k;
}

/* Excitation analysis of the pair (I, J).  Returns the level (0, 1, 2) or
 * -1 when the pair is not connected by H.  For level 1: P (in I), Q (in J).
 * For level 2: particles P < R (in I), holes Q < S (in J).  sign is
 * <I| a+_P a_Q |J> or <I| a+_P a+_R a_S a_Q |J>. */
static int excitation(const uint64_t *I, const uint64_t *J, int n,
                      int *P, int *Q, int *R, int *S, int *sign)
{
    int nel_i = __builtin_popcountll(I[0]) + __builtin_popcountll(I[1]);
    int nel_j = __builtin_popcountll(J[0]) + __builtin_popcountll(J[1]);
    if (nel_i != nel_j) return -1;
    int pc = __builtin_popcountll(I[0] ^ J[0]) + __builtin_popcountll(I[1] ^ J[1]);
    if (pc == 0) { *sign = 1; return 0; }
    if (pc > 4) return -1;
    int part[2], hole[2];
    int np = diff_positions(I, J, n, part, 2);
    int nh = diff_positions(J, I, n, hole, 2);
    if (np != nh) return -1;
    if (np == 1) {
        *P = part[0]; *Q = hole[0];
        *sign = parity(between(J, n, *P, *Q));
        return 1;
    }
    *P = part[0]; *R = part[1]; *Q = hole[0]; *S = hole[1];
    /* a+_P a+_R a_S a_Q = (a+_P a_Q)(a+_R a_S) since Q != R: apply R<-S to J
     * first, then P<-Q to the result */
    uint64_t K[2] = {J[0], J[1]};
    int s1 = parity(between(K, n, *R, *S));
    K[*S / n] &= ~(1ull << (*S % n));
    K[*R / n] |= (1ull << (*R % n));
    int s2 = parity(between(K, n, *P, *Q));
    *sign = s1 * s2;
    return 2;
}

static cx hij(const ham_t *H, const uint64_t *I, const uint64_t *J, int n)
{
    int P = -1, Q = -1, R = -1, S = -1, sign = 0;
    int lvl = excitation(I, J, n, &P, &Q, &R, &S, &sign);
    if (lvl < 0) return CX0;
    if (lvl == 0) {
        /* occupied positions ascending, then every pair A < B */
        int occ[128], no = 0;
        for (int A = 0; A < 2 * n; A++)
            if (occupied(I, n, A)) occ[no++] = A;
        cx e = {H->ecore, 0.0};
        for (int a = 0; a < no; a++) {
            int A = occ[a];
            e = cx_add(e, h_so(H, A, A));
            for (int b = a + 1; b < no; b++) {
                int B = occ[b];
                e = cx_add(e, cx_sub(g_so(H, A, A, B, B), g_so(H, A, B, B, A)));
            }
        }
        return e;
    }
    if (lvl == 1) {
        cx e = h_so(H, P, Q);
        for (int X = 0; X < 2 * n; X++) {
            if (X == Q || !occupied(J, n, X)) continue;
            e = cx_add(e, cx_sub(g_so(H, P, Q, X, X), g_so(H, P, X, X, Q)));
        }
        return cx_sgn(sign, e);
    }
    return cx_sgn(sign, cx_sub(g_so(H, P, Q, R, S), g_so(H, P, S, R, Q)));
}

/* ------------------------------------------------------------------------ */

/* set the threads the OpenMP loops of this library use (n <= 0: leave) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* threads an OpenMP loop of this library uses */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sigma[r][k] = sum_J H_{I_r J} c[J][k] for each requested row I_r.
 * c, sigma interleaved complex, [ndet][nroots] and [nrows][nroots]. */
void orc_sigma_rows(int kind, int n, const double *h, const double *g, double ecore,
                    long ndet, const uint64_t *dets, int nroots, const double *c,
                    long nrows, const long *rows, double *sigma)
{
    ham_t H = {kind, n, h, g, ecore};
    #pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < nrows; r++) {
        const uint64_t *I = dets + 2 * rows[r];
        cx *acc = (cx *)calloc((size_t)nroots, sizeof(cx));
        for (long j = 0; j < ndet; j++) {
            const uint64_t *J = dets + 2 * j;
            int pc = __builtin_popcountll(I[0] ^ J[0]) + __builtin_popcountll(I[1] ^ J[1]);
            if (pc > 4) continue;
            cx v = hij(&H, I, J, n);
            for (int k = 0; k < nroots; k++) {
                cx cj = {c[2 * (j * nroots + k)], c[2 * (j * nroots + k) + 1]};
                acc[k] = cx_add(acc[k], cx_mul(v, cj));
            }
        }
        for (int k = 0; k < nroots; k++) {
            sigma[2 * (r * nroots + k)] = acc[k].re;
            sigma[2 * (r * nroots + k) + 1] = acc[k].im;
        }
        free(acc);
    }
}

/* Matrix elements H_{I J} for explicit (I, J) index pairs. */
void orc_hij_pairs(int kind, int n, const double *h, const double *g, double ecore,
                   const uint64_t *dets, long npairs, const long *ij, double *out)
{
    ham_t H = {kind, n, h, g, ecore};
    #pragma omp parallel for schedule(static)
    for (long t = 0; t < npairs; t++) {
        cx v = hij(&H, dets + 2 * ij[2 * t], dets + 2 * ij[2 * t + 1], n);
        out[2 * t] = v.re;
        out[2 * t + 1] = v.im;
    }
}

/* Number of connected J != I for each requested row (level 1 or 2). */
void orc_degree_rows(int n, long ndet, const uint64_t *dets, long nrows, const long *rows, long *deg)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < nrows; r++) {
        const uint64_t *I = dets + 2 * rows[r];
        long cnt = 0;
        for (long j = 0; j < ndet; j++) {
            int P, Q, R, S, sg;
            if (j == rows[r]) continue;
            int lvl = excitation(I, dets + 2 * j, n, &P, &Q, &R, &S, &sg);
            if (lvl == 1 || lvl == 2) cnt++;
        }
        deg[r] = cnt;
    }
}

/* Number of ordered pairs (I, J), I != J, of the whole space that H
 * connects, split by excitation level: out[0] singles, out[1] doubles.
 * Every determinant of a space holds the same electron counts (spin-free:
 * the same N_alpha and N_beta, which the caller checks), so the number of
 * electrons moved is popcount(I xor J) / 2 and the pair is connected when
 * that is 1 or 2 (section 2.3: zero-, one- and two-electron differences).
 * Every pair is visited; only the counting loop uses the popcount
 * instruction, so the timed rows of orc_sigma_rows are built as before. */
__attribute__((target("popcnt")))
void orc_pair_counts(long ndet, const uint64_t *dets, long *out)
{
    long c1 = 0, c2 = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(+ : c1, c2)
    for (long i = 0; i < ndet; i++) {
        const uint64_t a0 = dets[2 * i], a1 = dets[2 * i + 1];
        long s1 = 0, s2 = 0;
        for (long j = 0; j < ndet; j++) {
            const int x = __builtin_popcountll(a0 ^ dets[2 * j]) + __builtin_popcountll(a1 ^ dets[2 * j + 1]);
            s1 += (x == 2);
            s2 += (x == 4);
        }
        c1 += s1;
        c2 += s2;
    }
    out[0] = c1;
    out[1] = c2;
}

/* Connected pairs of the requested rows, J ascending.  Record layout
 * (int64 x 7): I, J, P, Q, R, S, sign  (R = S = -1 for singles).
 * First call with out == NULL returns the count. */
long orc_connect_rows(int n, long ndet, const uint64_t *dets, long nrows, const long *rows,
                      long *out)
{
    long total = 0;
    for (long r = 0; r < nrows; r++) {
        const uint64_t *I = dets + 2 * rows[r];
        for (long j = 0; j < ndet; j++) {
            int P = -1, Q = -1, R = -1, S = -1, sg = 0;
            if (j == rows[r]) continue;
            int lvl = excitation(I, dets + 2 * j, n, &P, &Q, &R, &S, &sg);
            if (lvl != 1 && lvl != 2) continue;
            if (out) {
                long *o = out + 7 * total;
                o[0] = rows[r]; o[1] = j; o[2] = P; o[3] = Q;
                o[4] = lvl == 2 ? R : -1; o[5] = lvl == 2 ? S : -1; o[6] = sg;
            }
            total++;
        }
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Transition density matrices.  For every connected (I, J) all index tuples
 * with a nonzero operator element are listed structurally and their phase is
 * obtained by applying the operators one by one to J.                        */

/* apply a_X (create=0) or a+_X (create=1) to string d in place; returns the
 * sign, or 0 when the result vanishes */
static int apply_op(uint64_t *d, int n, int X, int create)
{
    int occ = occupied(d, n, X);
    if (create == occ) return 0;
    int below = 0;
    for (int Y = 0; Y < X; Y++) below += occupied(d, n, Y);
    d[X / n] ^= (1ull << (X % n));
    return parity(below);
}

/* <I| a+_P a+_R a_S a_Q |J> by literal application */
static int op2(const uint64_t *I, const uint64_t *J, int n, int P, int Q, int R, int S)
{
    uint64_t d[2] = {J[0], J[1]};
    int s = apply_op(d, n, Q, 0); if (!s) return 0;
    int t = apply_op(d, n, S, 0); if (!t) return 0; s *= t;
    t = apply_op(d, n, R, 1); if (!t) return 0; s *= t;
    t = apply_op(d, n, P, 1); if (!t) return 0; s *= t;
    return (d[0] == I[0] && d[1] == I[1]) ? s : 0;
}

static int op1(const uint64_t *I, const uint64_t *J, int n, int P, int Q)
{
    uint64_t d[2] = {J[0], J[1]};
    int s = apply_op(d, n, Q, 0); if (!s) return 0;
    int t = apply_op(d, n, P, 1); if (!t) return 0; s *= t;
    return (d[0] == I[0] && d[1] == I[1]) ? s : 0;
}

/* Output index maps: spin-free results are spin-summed over the spatial
 * orbitals (gamma_pq, Gamma_pqrs over n); spinor results are over M. */
static size_t idx2(int kind, int n, int P, int Q)
{
    if (kind == 0) return (size_t)(P % n) * n + (Q % n);
    return (size_t)P * (2 * n) + Q;
}
static size_t idx4(int kind, int n, int P, int Q, int R, int S)
{
    size_t m = kind == 0 ? (size_t)n : (size_t)2 * n;
    size_t p = kind == 0 ? P % n : P, q = kind == 0 ? Q % n : Q;
    size_t r = kind == 0 ? R % n : R, s = kind == 0 ? S % n : S;
    return ((p * m + q) * m + r) * m + s;
}

/* Accumulate for the requested bra rows (all J).  gamma, Gamma interleaved
 * complex, zero-initialised by the caller.  Single-threaded so that the
 * summation order is fixed. */
void orc_rdm_rows(int kind, int n, long ndet, const uint64_t *dets, int nroots,
                  const double *bra, const double *ket, const double *weights,
                  long nrows, const long *rows, double *gamma, double *Gamma)
{
    int M = 2 * n;
    int (*tup)[4] = (int (*)[4])malloc(sizeof(int[4]) * (size_t)(2 * M * M + 16));
    for (long r = 0; r < nrows; r++) {
        long i = rows[r];
        const uint64_t *I = dets + 2 * i;
        for (long j = 0; j < ndet; j++) {
            const uint64_t *J = dets + 2 * j;
            int P = -1, Q = -1, R = -1, S = -1, sg = 0;
            int lvl = excitation(I, J, n, &P, &Q, &R, &S, &sg);
            if (lvl < 0) continue;
            cx w = CX0;
            for (int k = 0; k < nroots; k++) {
                cx b = {bra[2 * (i * nroots + k)], bra[2 * (i * nroots + k) + 1]};
                cx kt = {ket[2 * (j * nroots + k)], ket[2 * (j * nroots + k) + 1]};
                cx t = cx_mul(cx_conj(b), kt);
                double wk = weights ? weights[k] : 1.0;
                cx wt = {wk * t.re, wk * t.im};
                w = cx_add(w, wt);
            }
            /* tuples (A,B,C,D) meaning a+_A a+_C a_D a_B */
            int nt = 0;
            if (lvl == 0) {
                for (int A = 0; A < M; A++) {
                    if (!occupied(I, n, A)) continue;
                    int s = op1(I, J, n, A, A);
                    size_t k1 = idx2(kind, n, A, A);
                    gamma[2 * k1] += s * w.re; gamma[2 * k1 + 1] += s * w.im;
                    for (int C = 0; C < M; C++) {
                        if (C == A || !occupied(I, n, C)) continue;
                        tup[nt][0] = A; tup[nt][1] = A; tup[nt][2] = C; tup[nt][3] = C; nt++;
                        tup[nt][0] = A; tup[nt][1] = C; tup[nt][2] = C; tup[nt][3] = A; nt++;
                    }
                }
            } else if (lvl == 1) {
                int s = op1(I, J, n, P, Q);
                size_t k1 = idx2(kind, n, P, Q);
                gamma[2 * k1] += s * w.re; gamma[2 * k1 + 1] += s * w.im;
                for (int X = 0; X < M; X++) {
                    if (X == Q || !occupied(J, n, X)) continue;
                    int t4[4][4] = {{P, Q, X, X}, {P, X, X, Q}, {X, Q, P, X}, {X, X, P, Q}};
                    for (int u = 0; u < 4; u++) { memcpy(tup[nt], t4[u], sizeof t4[u]); nt++; }
                }
            } else {
                int t4[4][4] = {{P, Q, R, S}, {R, S, P, Q}, {P, S, R, Q}, {R, Q, P, S}};
                for (int u = 0; u < 4; u++) { memcpy(tup[nt], t4[u], sizeof t4[u]); nt++; }
            }
            for (int u = 0; u < nt; u++) {
                /* the spin-summed spin-free Gamma_pqrs only pairs P with Q
                 * and R with S of equal spin */
                if (kind == 0 && (tup[u][0] / n != tup[u][1] / n || tup[u][2] / n != tup[u][3] / n))
                    continue;
                int s = op2(I, J, n, tup[u][0], tup[u][1], tup[u][2], tup[u][3]);
                if (!s) continue;
                size_t k4 = idx4(kind, n, tup[u][0], tup[u][1], tup[u][2], tup[u][3]);
                Gamma[2 * k4] += s * w.re; Gamma[2 * k4 + 1] += s * w.im;
            }
        }
    }
    free(tup);
}

/* ------------------------------------------------------------------------ */
/* Epstein-Nesbet second-order energy (section 2.5, Eq. (ENPT2E)) with the
 * primary space equal to the whole space P:
 *   E2_k = sum_{A in Q} |sum_{J in P} H_AJ c_Jk|^2 / (E0_k - H_AA),
 * Q = the determinants outside P that one or two excitations reach from
 * some J in P (spin-free: N_alpha and N_beta kept).  Screening as in the
 * paper's PT2 procedure (step 4): the pair (A, J) is left out when the
 * configuration of A is doubly excited from that of J and Table 1's bound
 * H~ is below qmin / max_{nu,k} |C^J_{nu,k}| (the maximum over the
 * determinants nu of J's configuration and the roots); qmin = 0 keeps
 * everything.
 * Steps: every J lists its excitations A outside P; the (A, J) list is
 * sorted by A, then J; each numerator is summed in ascending J; the
 * contributions are added in ascending A. */

typedef struct { uint64_t a0, a1; long j; } pt2_rec;

static int rec_cmp(const void *x, const void *y)
{
    const pt2_rec *a = (const pt2_rec *)x, *b = (const pt2_rec *)y;
    if (a->a0 != b->a0) return a->a0 < b->a0 ? -1 : 1;
    if (a->a1 != b->a1) return a->a1 < b->a1 ? -1 : 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* is (d0, d1) one of the sorted determinants? */
static int in_space(long ndet, const uint64_t *dets, uint64_t d0, uint64_t d1)
{
    long lo = 0, hi = ndet;
    while (lo < hi) {
        long mid = lo + (hi - lo) / 2;
        uint64_t m0 = dets[2 * mid], m1 = dets[2 * mid + 1];
        if (m0 < d0 || (m0 == d0 && m1 < d1)) lo = mid + 1;
        else hi = mid;
    }
    return lo < ndet && dets[2 * lo] == d0 && dets[2 * lo + 1] == d1;
}

static double cx_abs(cx a) { return sqrt(a.re * a.re + a.im * a.im); }

/* ------------------------------------------------------------------------ */
/* Configurations (section 2.2) and the upper bounds of Table 1.
 * The configuration of a determinant gives every spatial orbital (spin-free)
 * or Kramers pair (spinor) p the occupation n_p = (bit p of word 0) + (bit p
 * of word 1), 0, 1 or 2. */
static int occ_num(const uint64_t *d, int p) { return (int)((d[0] >> p) & 1u) + (int)((d[1] >> p) & 1u); }

/* Excitation level between the configurations of J and I: the electrons
 * that move, sum over p of max(0, n_p(J) - n_p(I)).  For level 2, the
 * orbitals that gain electrons in I (particles i <= k) and those that lose
 * them (holes j <= l); an orbital whose occupation changes by 2 is listed
 * twice. */
static int cfg_excitation(const uint64_t *I, const uint64_t *J, int n, int *i, int *k, int *j, int *l)
{
    int part[4], hole[4], np = 0, nh = 0;
    for (int p = 0; p < n; p++) {
        int d = occ_num(I, p) - occ_num(J, p);
        while (d > 0 && np < 4) { part[np++] = p; d--; }
        while (d < 0 && nh < 4) { hole[nh++] = p; d++; }
    }
    if (np == 2 && nh == 2) { *i = part[0]; *k = part[1]; *j = hole[0]; *l = hole[1]; }
    return nh;
}

/* |(ab|cd)| as Table 1 uses it.  Spin-free: the spatial integral.  Spinor
 * (every vertex has both Kramers partners): the largest |(PQ|RS)| over P in
 * pair a, Q in b, R in c, S in d, with P != R and Q != S (two electrons of
 * one pair sit in both of its spinors). */
static double g_bound(const ham_t *H, int a, int b, int c, int d)
{
    const int n = H->n;
    if (H->kind == 0) return fabs(H->g[(((size_t)a * n + b) * n + c) * n + d]);
    double m = 0.0;
    for (int P = a; P < 2 * n; P += n)
        for (int Q = b; Q < 2 * n; Q += n)
            for (int R = c; R < 2 * n; R += n)
                for (int S = d; S < 2 * n; S += n) {
                    if (P == R || Q == S) continue;
                    double v = cx_abs(g_so(H, P, Q, R, S));
                    if (v > m) m = v;
                }
    return m;
}

/* Table 1, SD column: the upper bound H~ of |H_{I mu, J nu}| over the
 * determinants of two configurations, I doubly excited from J, particles
 * i, k and holes j, l. */
static double table1_sd(const ham_t *H, int i, int k, int j, int l)
{
    if (i != k && j != l) {                   /* IntC 1-3: e_ij,kl and e_il,kj */
        double x = g_bound(H, i, j, k, l), y = g_bound(H, i, l, k, j);
        return x > y ? x : y;
    }
    if (i != k) return g_bound(H, i, j, k, j); /* IntC 4-5: e_ij,kj (l = j) */
    if (j != l) return g_bound(H, i, l, i, j); /* IntC 6: e_il,ij (k = i) */
    return g_bound(H, i, j, i, j);             /* IntC 7: e_ij,ij */
}

/* cm[j] = max over the roots k and over the determinants nu of the space
 * with the configuration of determinant j of |c[nu][k]| (the
 * max_{nu,k} |C^J_{nu,k}| of the screening).  Determinants are grouped by
 * their configuration (occupied mask, doubly occupied mask) by sorting. */
typedef struct { uint64_t occ, dbl; long j; } cfg_ent;

static int cfg_ent_cmp(const void *x, const void *y)
{
    const cfg_ent *a = (const cfg_ent *)x, *b = (const cfg_ent *)y;
    if (a->occ != b->occ) return a->occ < b->occ ? -1 : 1;
    if (a->dbl != b->dbl) return a->dbl < b->dbl ? -1 : 1;
    return (a->j > b->j) - (a->j < b->j);
}

static void cfg_cmax(long ndet, const uint64_t *dets, int nroots, const double *c, double *cm)
{
    cfg_ent *e = (cfg_ent *)malloc(sizeof(cfg_ent) * (size_t)(ndet > 0 ? ndet : 1));
    for (long j = 0; j < ndet; j++) {
        e[j].occ = dets[2 * j] | dets[2 * j + 1];
        e[j].dbl = dets[2 * j] & dets[2 * j + 1];
        e[j].j = j;
    }
    qsort(e, (size_t)ndet, sizeof(cfg_ent), cfg_ent_cmp);
    for (long s = 0; s < ndet;) {
        long t = s;
        double m = 0.0;
        while (t < ndet && e[t].occ == e[s].occ && e[t].dbl == e[s].dbl) {
            for (int k = 0; k < nroots; k++) {
                long j = e[t].j;
                cx cj = {c[2 * (j * nroots + k)], c[2 * (j * nroots + k) + 1]};
                double a = cx_abs(cj);
                if (a > m) m = a;
            }
            t++;
        }
        for (long u = s; u < t; u++) cm[e[u].j] = m;
        s = t;
    }
    free(e);
}

/* Screening test of section 2.5 (step 4) for a determinant pair (A, J):
 * true when the configuration of A is doubly excited from that of J and
 * Table 1's bound is below qmin / max_{nu,k} |C^J_{nu,k}| (cmj). */
static int pt2_screened(const ham_t *H, const uint64_t *A, const uint64_t *J, double cmj, double qmin)
{
    int i = -1, k = -1, j = -1, l = -1;
    if (cfg_excitation(A, J, H->n, &i, &k, &j, &l) != 2) return 0;
    return table1_sd(H, i, k, j, l) < qmin / cmj;
}

typedef struct { pt2_rec *r; long n, cap; } rec_buf;

static void rec_push(rec_buf *b, uint64_t a0, uint64_t a1, long j)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->r = (pt2_rec *)realloc(b->r, sizeof(pt2_rec) * (size_t)b->cap);
    }
    b->r[b->n].a0 = a0; b->r[b->n].a1 = a1; b->r[b->n].j = j;
    b->n++;
}

static void flip(uint64_t *d, int n, int X) { d[X / n] ^= (1ull << (X % n)); }

/* stats (nullable): [0] kept (A, J) pairs, [1] distinct A in Q */
void orc_pt2(int kind, int n, const double *h, const double *g, double ecore,
             long ndet, const uint64_t *dets, int nroots, const double *c,
             const double *e0, double qmin, double *e2, long *stats)
{
    ham_t H = {kind, n, h, g, ecore};
    const int M = 2 * n;
    rec_buf B = {NULL, 0, 0};
    for (long j = 0; j < ndet; j++) {
        const uint64_t *J = dets + 2 * j;
        for (int Q = 0; Q < M; Q++) {
            if (!occupied(J, n, Q)) continue;
            /* singles Q -> P */
            for (int P = 0; P < M; P++) {
                if (occupied(J, n, P)) continue;
                if (kind == 0 && P / n != Q / n) continue;
                uint64_t A[2] = {J[0], J[1]};
                flip(A, n, Q); flip(A, n, P);
                if (!in_space(ndet, dets, A[0], A[1])) rec_push(&B, A[0], A[1], j);
            }
            /* doubles Q < S -> P < R */
            for (int S = Q + 1; S < M; S++) {
                if (!occupied(J, n, S)) continue;
                for (int P = 0; P < M; P++) {
                    if (occupied(J, n, P)) continue;
                    for (int R = P + 1; R < M; R++) {
                        if (occupied(J, n, R)) continue;
                        if (kind == 0) {
                            int hs = (Q / n) + (S / n), ps = (P / n) + (R / n);
                            if (hs != ps) continue;
                        }
                        uint64_t A[2] = {J[0], J[1]};
                        flip(A, n, Q); flip(A, n, S); flip(A, n, P); flip(A, n, R);
                        if (!in_space(ndet, dets, A[0], A[1])) rec_push(&B, A[0], A[1], j);
                    }
                }
            }
        }
    }
    qsort(B.r, (size_t)B.n, sizeof(pt2_rec), rec_cmp);
    /* largest |C| over the roots and the determinants of J's configuration */
    double *cmax = (double *)calloc((size_t)(ndet > 0 ? ndet : 1), sizeof(double));
    cfg_cmax(ndet, dets, nroots, c, cmax);
    /* first record of every distinct A */
    long nA = 0;
    long *head = (long *)malloc(sizeof(long) * (size_t)(B.n + 1));
    for (long s = 0; s < B.n; s++)
        if (s == 0 || B.r[s].a0 != B.r[s - 1].a0 || B.r[s].a1 != B.r[s - 1].a1) head[nA++] = s;
    head[nA] = B.n;
    /* per-A contributions (independent, any thread), then summed in ascending A */
    double *contrib = (double *)calloc((size_t)(nA > 0 ? nA : 1) * (size_t)(nroots > 0 ? nroots : 1), sizeof(double));
    long *used = (long *)calloc((size_t)(nA > 0 ? nA : 1), sizeof(long));
    #pragma omp parallel for schedule(dynamic, 256)
    for (long a = 0; a < nA; a++) {
        cx num[64];
        const uint64_t A[2] = {B.r[head[a]].a0, B.r[head[a]].a1};
        for (int k = 0; k < nroots; k++) num[k] = CX0;
        long u_cnt = 0;
        for (long u = head[a]; u < head[a + 1]; u++) {
            long j = B.r[u].j;
            const uint64_t *J = dets + 2 * j;
            if (pt2_screened(&H, A, J, cmax[j], qmin)) continue;
            cx v = hij(&H, A, J, n);
            u_cnt++;
            for (int k = 0; k < nroots; k++) {
                cx cj = {c[2 * (j * nroots + k)], c[2 * (j * nroots + k) + 1]};
                num[k] = cx_add(num[k], cx_mul(v, cj));
            }
        }
        used[a] = u_cnt;
        if (u_cnt) {
            double haa = hij(&H, A, A, n).re;
            for (int k = 0; k < nroots; k++)
                contrib[a * nroots + k] = (num[k].re * num[k].re + num[k].im * num[k].im) / (e0[k] - haa);
        }
    }
    /* millions of terms: compensated (Neumaier) summation in ascending A, so
     * that the total carries no O(N eps) accumulation error */
    long kept = 0, nq = 0;
    for (int k = 0; k < nroots; k++) {
        double s = 0.0, comp = 0.0;
        for (long a = 0; a < nA; a++) {
            if (!used[a]) continue;
            double x = contrib[a * nroots + k], t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
        e2[k] = s + comp;
    }
    for (long a = 0; a < nA; a++)
        if (used[a]) { kept += used[a]; nq++; }
    if (stats) { stats[0] = kept; stats[1] = nq; }
    free(head);
    free(contrib);
    free(used);
    free(cmax);
    free(B.r);
}

/* ------------------------------------------------------------------------ */
/* Selection of external determinants by the iCIPT2 criterion (section 2.4,
 * Eqs. (iCI_Selection-1) and (iCI_Selection-2)).  A outside P is selected
 * when some configuration J of P (its determinants nu that the space holds)
 * gives f(A, J) true:
 *   max_{nu,k} |H_{A nu} C_{nu,k}| >= cmin  and
 *   max_{nu,k} |H_{A nu} C_{nu,k} / (E0_k - H_AA)| >= cmin,
 * and, when the configuration of A is doubly excited from J (case B),
 *   max_{nu,k} |H~ C_{nu,k}| = H~ max_{nu,k} |C_{nu,k}| >= cmin
 * with H~ Table 1's bound.  Steps: every determinant nu of P lists its
 * single and double excitations A outside P with the two per-pair tests
 * (pairs failing the bound test, or both per-pair tests, cannot make f
 * true and are not kept); the list is sorted by A and J's configuration;
 * A is selected when one configuration group has a pair passing the first
 * test and a pair passing the second.  out (nullable): [max_out][2];
 * returns the number of distinct selected determinants, written sorted. */
typedef struct { uint64_t a0, a1; } det_key;
typedef struct { uint64_t a0, a1, occ, dbl; int t1, t2; } sel_rec;

static int sel_cmp(const void *x, const void *y)
{
    const sel_rec *a = (const sel_rec *)x, *b = (const sel_rec *)y;
    if (a->a0 != b->a0) return a->a0 < b->a0 ? -1 : 1;
    if (a->a1 != b->a1) return a->a1 < b->a1 ? -1 : 1;
    if (a->occ != b->occ) return a->occ < b->occ ? -1 : 1;
    if (a->dbl != b->dbl) return a->dbl < b->dbl ? -1 : 1;
    if (a->t1 != b->t1) return a->t1 - b->t1;
    return a->t2 - b->t2;
}

long orc_select(int kind, int n, const double *h, const double *g, double ecore,
                long ndet, const uint64_t *dets, int nroots, const double *c,
                const double *e0, double cmin, uint64_t *out, long max_out)
{
    ham_t H = {kind, n, h, g, ecore};
    const int M = 2 * n;
    double *cm = (double *)calloc((size_t)(ndet > 0 ? ndet : 1), sizeof(double));
    cfg_cmax(ndet, dets, nroots, c, cm);
    sel_rec *rec = NULL;
    long nr = 0, cap = 0;
    /* every J independently (any thread), its pairs appended in turn */
    #pragma omp parallel
    {
        sel_rec *mine = NULL;
        long nm = 0, cmn = 0;
        #pragma omp for schedule(dynamic, 1)
        for (long j = 0; j < ndet; j++) {
            const uint64_t *J = dets + 2 * j;
            for (int Q = 0; Q < M; Q++) {
                if (!occupied(J, n, Q)) continue;
                for (int S = Q; S < M; S++) {          /* S == Q: a single */
                    if (!occupied(J, n, S)) continue;
                    for (int P = 0; P < M; P++) {
                        if (occupied(J, n, P)) continue;
                        for (int R = (S == Q ? P : P + 1); R < M; R++) {
                            if (S == Q && R != P) break;
                            if (S != Q && occupied(J, n, R)) continue;
                            if (kind == 0) {
                                int hs = (Q / n) + (S == Q ? Q / n : S / n);
                                int ps = (P / n) + (S == Q ? P / n : R / n);
                                if (hs != ps) continue;
                            }
                            uint64_t A[2] = {J[0], J[1]};
                            flip(A, n, Q); flip(A, n, P);
                            if (S != Q) { flip(A, n, S); flip(A, n, R); }
                            if (in_space(ndet, dets, A[0], A[1])) continue;
                            int ci = -1, ck = -1, cj = -1, cl = -1;
                            if (cfg_excitation(A, J, n, &ci, &ck, &cj, &cl) == 2 &&
                                !(table1_sd(&H, ci, ck, cj, cl) * cm[j] >= cmin))
                                continue;                     /* case (B): the bound test */
                            cx v = hij(&H, A, J, n);
                            double haa = hij(&H, A, A, n).re;
                            double m1 = 0.0, m2 = 0.0;
                            for (int k = 0; k < nroots; k++) {
                                cx cj_ = {c[2 * (j * nroots + k)], c[2 * (j * nroots + k) + 1]};
                                double a = cx_abs(cx_mul(v, cj_));
                                if (a > m1) m1 = a;
                                double b = a / fabs(e0[k] - haa);
                                if (b > m2) m2 = b;
                            }
                            int t1 = m1 >= cmin, t2 = m2 >= cmin;
                            if (!t1 && !t2) continue;
                            if (nm == cmn) {
                                cmn = cmn ? 2 * cmn : 1024;
                                mine = (sel_rec *)realloc(mine, sizeof(sel_rec) * (size_t)cmn);
                            }
                            mine[nm].a0 = A[0]; mine[nm].a1 = A[1];
                            mine[nm].occ = J[0] | J[1]; mine[nm].dbl = J[0] & J[1];
                            mine[nm].t1 = t1; mine[nm].t2 = t2;
                            nm++;
                        }
                    }
                }
            }
        }
        #pragma omp critical
        {
            if (nr + nm > cap) {
                cap = nr + nm;
                rec = (sel_rec *)realloc(rec, sizeof(sel_rec) * (size_t)(cap > 0 ? cap : 1));
            }
            if (nm) memcpy(rec + nr, mine, sizeof(sel_rec) * (size_t)nm);
            nr += nm;
        }
        free(mine);
    }
    qsort(rec, (size_t)nr, sizeof(sel_rec), sel_cmp);
    long u = 0;
    for (long s = 0; s < nr;) {
        /* the run of one A */
        long e = s;
        while (e < nr && rec[e].a0 == rec[s].a0 && rec[e].a1 == rec[s].a1) e++;
        int selected = 0;
        for (long g0 = s; g0 < e;) {
            /* the group of one configuration of P */
            long g1 = g0;
            int any1 = 0, any2 = 0;
            while (g1 < e && rec[g1].occ == rec[g0].occ && rec[g1].dbl == rec[g0].dbl) {
                any1 |= rec[g1].t1;
                any2 |= rec[g1].t2;
                g1++;
            }
            if (any1 && any2) selected = 1;
            g0 = g1;
        }
        if (selected) {
            if (out && u < max_out) { out[2 * u] = rec[s].a0; out[2 * u + 1] = rec[s].a1; }
            u++;
        }
        s = e;
    }
    free(rec);
    free(cm);
    return u;
}
