"""Seeded synthetic inputs: integrals, determinant spaces and CI vectors.

This module is shared by the CPU oracle tests and the GPU path.  It holds
none of the method's arithmetic (no matrix elements, phases or contractions):
it only draws numbers and builds sorted occupation bitstrings.

Conventions (shared with the C ABI in ``include/mw.h``):

* A determinant is two 64-bit words ``(w0, w1)``.  Spin-free: ``w0`` holds the
  alpha string and ``w1`` the beta string, spatial orbital ``p`` at bit ``p``.
  Spinor (Kramers-paired spinors, paper section 2.1): ``w0`` holds the
  unbarred (A) spinors and ``w1`` the barred (B) ones, pair ``k`` at bit ``k``.
  This is the determinant analogue of the occupation bitstrings of section 2.2
  (orbital 0 in the lowest bit).
* Spaces are sorted strictly ascending as unsigned 128-bit keys, ``w0`` major.
* Global spin-orbital / spinor position of word ``w`` bit ``b`` is ``w*n + b``.

Seeds follow ``SeedSequence([2501, 18185, k, i, j])`` with ``k`` the workload
index, ``i`` the problem index inside a batch and ``j`` the stream
(0: h, 1: g, 2: space, 3: c).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

SEED_H, SEED_G, SEED_SPACE, SEED_C = 0, 1, 2, 3


def rng_for(k: int, i: int, j: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2501, 18185, k, i, j]))


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------

def _orbit_canon_real(n: int):
    """For every (p,q,r,s) the smallest flat index of its 8-fold orbit."""
    p, q, r, s = np.meshgrid(*(np.arange(n, dtype=np.int64),) * 4, indexing="ij")
    def flat(a, b, c, d):
        return ((a * n + b) * n + c) * n + d
    cands = [flat(p, q, r, s), flat(q, p, r, s), flat(p, q, s, r), flat(q, p, s, r),
             flat(r, s, p, q), flat(s, r, p, q), flat(r, s, q, p), flat(s, r, q, p)]
    canon = cands[0]
    for c_ in cands[1:]:
        canon = np.minimum(canon, c_)
    return canon.reshape(-1)


def one_body_real(n: int, rng: np.random.Generator) -> np.ndarray:
    """Symmetric h: diagonal ascending linearly over [-2, 1], off-diagonal N(0, 0.05^2)."""
    h = np.zeros((n, n))
    diag = np.array([-2.0 + 3.0 * p / (n - 1) for p in range(n)]) if n > 1 else np.array([-2.0])
    off = rng.normal(0.0, 0.05, size=(n, n))
    iu = np.triu_indices(n, 1)
    h[iu] = off[iu]
    h = h + h.T
    h[np.diag_indices(n)] = diag
    return h


def two_body_real(n: int, rng: np.random.Generator) -> np.ndarray:
    """8-fold symmetric (pq|rs), shape (n,n,n,n).

    Orbits with p==q and r==s draw U(0.3, 0.7) (Coulomb-like); every other
    orbit draws N(0, 0.02^2) * exp(-|p-q|/4) with (p,q) of its canonical
    (smallest flat index) member.
    """
    canon = _orbit_canon_real(n)
    m = n ** 4
    uni = rng.uniform(0.3, 0.7, size=m)
    nor = rng.normal(0.0, 0.02, size=m)
    cp = canon // (n ** 3)
    cq = (canon // (n ** 2)) % n
    cr = (canon // n) % n
    cs = canon % n
    coul = (cp == cq) & (cr == cs)
    val_canon = np.where(coul, uni[canon], nor[canon] * np.exp(-np.abs(cp - cq) / 4.0))
    return val_canon.reshape(n, n, n, n)


def chemistry_like_real(n: int, rng: np.random.Generator, off: float = 0.03):
    """(h, g) with the structure of molecular integrals: orbital energies
    h_pp = -2 + 0.6 p on the diagonal, Coulomb-like (pp|qq) = 0.3 added,
    and the random integrals of ``one_body_real``/``two_body_real`` scaled
    by ``off`` elsewhere, so the determinant Hamiltonian is diagonally
    dominant (off-diagonal row sums ~0.1 against a diagonal spread ~10)."""
    h = off * one_body_real(n, rng)
    h[np.diag_indices(n)] = -2.0 + 0.6 * np.arange(n)
    g = off * two_body_real(n, rng)
    idx = np.arange(n)
    g[idx[:, None], idx[:, None], idx[None, :], idx[None, :]] += 0.3
    return h, g


def one_body_spinor(nk: int, rng: np.random.Generator) -> np.ndarray:
    """Hermitian h over M = 2*nk spinors (A_k at k, B_k at nk+k).

    Kramers-degenerate diagonal h[A_k,A_k] = h[B_k,B_k] ascending over [-2, 1];
    off-diagonal magnitude N(0, 0.05^2) with a uniform phase.
    """
    M = 2 * nk
    diag = np.array([-2.0 + 3.0 * k / (nk - 1) for k in range(nk)]) if nk > 1 else np.array([-2.0])
    mag = rng.normal(0.0, 0.05, size=(M, M))
    ph = rng.uniform(0.0, 2 * np.pi, size=(M, M))
    h = np.zeros((M, M), dtype=np.complex128)
    iu = np.triu_indices(M, 1)
    h[iu] = (mag * np.exp(1j * ph))[iu]
    h = h + h.conj().T
    h[np.diag_indices(M)] = np.concatenate([diag, diag])
    return h


def two_body_spinor(nk: int, rng: np.random.Generator) -> np.ndarray:
    """Complex (PQ|RS) over M = 2*nk spinors with (PQ|RS) = (RS|PQ) = (QP|SR)*.

    Orbits {(PQ|RS), (RS|PQ), (QP|SR)*, (SR|QP)*} share one value.  Orbits
    with P==Q and R==S are real U(0.3, 0.7); other self-conjugate orbits
    (P==S and Q==R) are real N(0, 0.02^2) * exp(-|k(P)-k(Q)|/4); the rest
    carry that magnitude times a uniform phase.  k(P) is the Kramers pair.
    """
    M = 2 * nk
    P, Q, R, S = np.meshgrid(*(np.arange(M, dtype=np.int64),) * 4, indexing="ij")
    def flat(a, b, c, d):
        return ((a * M + b) * M + c) * M + d
    f1 = flat(P, Q, R, S).reshape(-1)
    f2 = flat(R, S, P, Q).reshape(-1)
    f3 = flat(Q, P, S, R).reshape(-1)
    f4 = flat(S, R, Q, P).reshape(-1)
    del P, Q, R, S
    canon = np.minimum(np.minimum(f1, f2), np.minimum(f3, f4))
    conj = (canon == f3) | (canon == f4)
    del f1, f2, f3, f4
    m = M ** 4
    uni = rng.uniform(0.3, 0.7, size=m)
    nor = rng.normal(0.0, 0.02, size=m)
    ph = rng.uniform(0.0, 2 * np.pi, size=m)
    cp = canon // (M ** 3)
    cq = (canon // (M ** 2)) % M
    cr = (canon // M) % M
    cs = canon % M
    coul = (cp == cq) & (cr == cs)
    selfc = coul | ((cp == cs) & (cq == cr))
    kp, kq = cp % nk, cq % nk
    mag = nor[canon] * np.exp(-np.abs(kp - kq) / 4.0)
    val = np.where(coul, uni[canon] + 0j, np.where(selfc, mag + 0j, mag * np.exp(1j * ph[canon])))
    val = np.where(conj & ~selfc, val.conj(), val)
    return val.reshape(M, M, M, M)


# ---------------------------------------------------------------------------
# determinant spaces
# ---------------------------------------------------------------------------

def _words(pos: np.ndarray, n: int):
    """Global positions (..., k) with -1 padding -> (w0, w1) uint64 masks."""
    pos = np.asarray(pos, dtype=np.int64)
    valid = pos >= 0
    word = np.where(valid, pos // n, 0)
    bit = np.where(valid, pos % n, 0).astype(np.uint64)
    one = np.where(valid, np.left_shift(np.uint64(1), bit), np.uint64(0))
    w0 = np.bitwise_or.reduce(np.where(word == 0, one, np.uint64(0)), axis=-1)
    w1 = np.bitwise_or.reduce(np.where(word == 1, one, np.uint64(0)), axis=-1)
    return w0.astype(np.uint64), w1.astype(np.uint64)


def sort_unique(w0: np.ndarray, w1: np.ndarray) -> np.ndarray:
    d = np.stack([np.asarray(w0, np.uint64), np.asarray(w1, np.uint64)], axis=1)
    order = np.lexsort((d[:, 1], d[:, 0]))
    d = d[order]
    if len(d) > 1:
        keep = np.ones(len(d), bool)
        keep[1:] = (d[1:, 0] != d[:-1, 0]) | (d[1:, 1] != d[:-1, 1])
        d = d[keep]
    return np.ascontiguousarray(d)


def space_fci(n: int, na: int, nb: int) -> np.ndarray:
    """Every determinant with na alpha and nb beta electrons in n orbitals."""
    def strings(k):
        out = []
        for occ in itertools.combinations(range(n), k):
            v = 0
            for p in occ:
                v |= 1 << p
            out.append(v)
        return np.array(sorted(out), dtype=np.uint64)
    a, b = strings(na), strings(nb)
    w0 = np.repeat(a, len(b))
    w1 = np.tile(b, len(a))
    return sort_unique(w0, w1)


def _excite(hf0, hf1, n, holes, parts):
    """Apply hole/particle global-position lists (-1 padded) to the HF words."""
    h0, h1 = _words(holes, n)
    p0, p1 = _words(parts, n)
    return (hf0 ^ h0) | p0, (hf1 ^ h1) | p1


def _all_excitations(occ, vir, k):
    """All (holes, particles) of rank k from occ x vir (global positions)."""
    hs = list(itertools.combinations(occ, k))
    ps = list(itertools.combinations(vir, k))
    if not hs or not ps:
        return np.zeros((0, k), np.int64), np.zeros((0, k), np.int64)
    H = np.repeat(np.array(hs, np.int64), len(ps), axis=0)
    Pp = np.tile(np.array(ps, np.int64), (len(hs), 1))
    return H, Pp


def _hf_and_sd_spinfree(n, na, nb):
    occa = list(range(na)); vira = list(range(na, n))
    occb = [n + p for p in range(nb)]; virb = [n + p for p in range(nb, n)]
    hf0 = np.uint64((1 << na) - 1); hf1 = np.uint64((1 << nb) - 1)
    ws0 = [np.array([hf0], np.uint64)]; ws1 = [np.array([hf1], np.uint64)]
    for occ, vir in ((occa, vira), (occb, virb)):
        for k in (1, 2):
            H, Pp = _all_excitations(occ, vir, k)
            if len(H):
                a, b = _excite(hf0, hf1, n, H, Pp)
                ws0.append(a); ws1.append(b)
    Ha, Pa = _all_excitations(occa, vira, 1)
    Hb, Pb = _all_excitations(occb, virb, 1)
    if len(Ha) and len(Hb):
        H = np.concatenate([np.repeat(Ha, len(Hb), 0), np.tile(Hb, (len(Ha), 1))], 1)
        Pp = np.concatenate([np.repeat(Pa, len(Pb), 0), np.tile(Pb, (len(Pa), 1))], 1)
        a, b = _excite(hf0, hf1, n, H, Pp)
        ws0.append(a); ws1.append(b)
    return hf0, hf1, np.concatenate(ws0), np.concatenate(ws1)


def _random_subsets(rng, m, pool, kmax):
    """m rows of kmax distinct entries of pool, uniformly without replacement."""
    pool = np.asarray(pool, np.int64)
    if len(pool) < kmax:
        raise ValueError("pool too small")
    idx = np.argsort(rng.random((m, len(pool))), axis=1)[:, :kmax]
    return pool[idx]


def _fill_random(base0, base1, target, gen_batch):
    """Append unique random determinants from gen_batch() until target."""
    have = sort_unique(base0, base1)
    if len(have) > target:
        raise ValueError(f"singles+doubles ({len(have)}) exceed target {target}")
    new0, new1 = [], []
    need = target - len(have)
    seen = have
    stalls = 0
    while need > 0:
        if stalls > 20:
            raise ValueError(f"cannot reach {target} distinct determinants with this recipe")
        c0, c1 = gen_batch(int(need * 1.15) + 64)
        allk = np.concatenate([np.stack([seen[:, 0], seen[:, 1]], 1), np.stack([c0, c1], 1)])
        rec = np.empty(len(allk), dtype=[("a", "<u8"), ("b", "<u8")])
        rec["a"], rec["b"] = allk[:, 0], allk[:, 1]
        _, first = np.unique(rec, return_index=True)
        first = np.sort(first[first >= len(seen)]) - len(seen)
        first = first[:need]
        stalls = stalls + 1 if len(first) * 50 < need else 0
        new0.append(c0[first]); new1.append(c1[first])
        need -= len(first)
        seen = sort_unique(np.concatenate([seen[:, 0], c0[first]]),
                           np.concatenate([seen[:, 1], c1[first]]))
    if new0:
        return sort_unique(np.concatenate([have[:, 0]] + new0), np.concatenate([have[:, 1]] + new1))
    return have


def space_selected_spinfree(n, na, nb, target, rng, ranks=(3, 4)):
    """HF + all singles + all doubles + random higher excitations up to target.

    Random rank uniform over ``ranks``; alpha/beta split uniform over the
    feasible (k_alpha, k_beta); holes and particles uniform without
    replacement; duplicates rejected.
    """
    hf0, hf1, w0, w1 = _hf_and_sd_spinfree(n, na, nb)
    occa = np.arange(na); vira = np.arange(na, n)
    occb = n + np.arange(nb); virb = n + np.arange(nb, n)
    kmax = max(ranks)

    def gen(m):
        rank = rng.choice(np.array(ranks), size=m)
        ka = np.empty(m, np.int64)
        for r in ranks:
            feas = [a for a in range(r + 1)
                    if a <= min(na, n - na) and (r - a) <= min(nb, n - nb)]
            sel = rank == r
            ka[sel] = rng.choice(np.array(feas), size=int(sel.sum()))
        kb = rank - ka
        ha = _random_subsets(rng, m, occa, min(kmax, na))
        pa = _random_subsets(rng, m, vira, min(kmax, n - na))
        hb = _random_subsets(rng, m, occb, min(kmax, nb))
        pb = _random_subsets(rng, m, virb, min(kmax, n - nb))
        cols = np.arange(ha.shape[1]); colsp = np.arange(pa.shape[1])
        colb = np.arange(hb.shape[1]); colpb = np.arange(pb.shape[1])
        ha = np.where(cols[None, :] < ka[:, None], ha, -1)
        pa = np.where(colsp[None, :] < ka[:, None], pa, -1)
        hb = np.where(colb[None, :] < kb[:, None], hb, -1)
        pb = np.where(colpb[None, :] < kb[:, None], pb, -1)
        H = np.concatenate([ha, hb], 1); Pp = np.concatenate([pa, pb], 1)
        return _excite(hf0, hf1, n, H, Pp)

    return _fill_random(w0, w1, target, gen)


def space_truncated_spinfree(n, na, nb, target, rng):
    """HF + all singles + random doubles up to target (a small variational
    space whose external space is dominated by its doubles' excitations).

    Double spin split uniform over the feasible (k_alpha, k_beta); holes and
    particles uniform without replacement; duplicates rejected."""
    hf0 = np.uint64((1 << na) - 1); hf1 = np.uint64((1 << nb) - 1)
    occa = np.arange(na); vira = np.arange(na, n)
    occb = n + np.arange(nb); virb = n + np.arange(nb, n)
    ws0 = [np.array([hf0], np.uint64)]; ws1 = [np.array([hf1], np.uint64)]
    for occ, vir in ((list(occa), list(vira)), (list(occb), list(virb))):
        H, Pp = _all_excitations(occ, vir, 1)
        if len(H):
            a, b = _excite(hf0, hf1, n, H, Pp)
            ws0.append(a); ws1.append(b)
    feas = np.array([a for a in range(3) if a <= min(na, n - na) and (2 - a) <= min(nb, n - nb)])

    def gen(m):
        ka = rng.choice(feas, size=m)
        kb = 2 - ka
        ha = _random_subsets(rng, m, occa, min(2, na))
        pa = _random_subsets(rng, m, vira, min(2, n - na))
        hb = _random_subsets(rng, m, occb, min(2, nb))
        pb = _random_subsets(rng, m, virb, min(2, n - nb))
        ha = np.where(np.arange(ha.shape[1])[None, :] < ka[:, None], ha, -1)
        pa = np.where(np.arange(pa.shape[1])[None, :] < ka[:, None], pa, -1)
        hb = np.where(np.arange(hb.shape[1])[None, :] < kb[:, None], hb, -1)
        pb = np.where(np.arange(pb.shape[1])[None, :] < kb[:, None], pb, -1)
        H = np.concatenate([ha, hb], 1); Pp = np.concatenate([pa, pb], 1)
        return _excite(hf0, hf1, n, H, Pp)

    return _fill_random(np.concatenate(ws0), np.concatenate(ws1), target, gen)


def space_selected_spinor(nk, nel, target, rng, ranks=(3,)):
    """Spinor space over M = 2*nk spinors: HF (pairs 0..nel/2-1 in A and B)
    + all singles + all doubles + random higher excitations (total N kept)."""
    if nel % 2:
        raise ValueError("closed-shell Kramers HF needs even nel")
    half = nel // 2
    occ = list(range(half)) + [nk + k for k in range(half)]
    vir = [p for p in range(2 * nk) if p not in occ]
    hf0 = np.uint64((1 << half) - 1); hf1 = np.uint64((1 << half) - 1)
    ws0 = [np.array([hf0], np.uint64)]; ws1 = [np.array([hf1], np.uint64)]
    for k in (1, 2):
        H, Pp = _all_excitations(occ, vir, k)
        a, b = _excite(hf0, hf1, nk, H, Pp)
        ws0.append(a); ws1.append(b)
    w0, w1 = np.concatenate(ws0), np.concatenate(ws1)
    kmax = max(ranks)

    def gen(m):
        rank = rng.choice(np.array(ranks), size=m)
        H = _random_subsets(rng, m, occ, kmax)
        Pp = _random_subsets(rng, m, vir, kmax)
        cols = np.arange(kmax)
        H = np.where(cols[None, :] < rank[:, None], H, -1)
        Pp = np.where(cols[None, :] < rank[:, None], Pp, -1)
        return _excite(hf0, hf1, nk, H, Pp)

    return _fill_random(w0, w1, target, gen)


def complete_configurations(dets, n):
    """Close a spin-free space over its configurations: for every
    determinant, all determinants with the same doubly occupied orbitals,
    the same singly occupied (open) orbitals and the same number of alpha
    electrons (every placement of the alpha spins over the open shells)."""
    d = np.asarray(dets, np.uint64).reshape(-1, 2)
    if len(d) == 0:
        return d
    a, b = d[:, 0], d[:, 1]
    docc, opn = a & b, a ^ b
    cfg = np.unique(np.stack([docc, opn], 1), axis=0)
    na = int(np.bitwise_count(a[0]))
    nd = np.bitwise_count(cfg[:, 0]).astype(np.int64)
    k = np.bitwise_count(cfg[:, 1]).astype(np.int64)
    out0, out1 = [], []
    for kk in np.unique(k):
        sel = cfg[k == kk]
        nup = na - int(nd[k == kk][0])
        # open positions, ascending, one row per configuration
        pos = np.zeros((len(sel), kk), np.int64)
        col = np.zeros(len(sel), np.int64)
        for p in range(n):
            hit = (sel[:, 1] >> np.uint64(p)) & np.uint64(1) == 1
            pos[hit, col[hit]] = p
            col[hit] += 1
        for combo in itertools.combinations(range(int(kk)), nup):
            up = np.zeros(len(sel), np.uint64)
            for j in combo:
                up |= np.left_shift(np.uint64(1), pos[:, j].astype(np.uint64))
            out0.append(sel[:, 0] | up)
            out1.append(sel[:, 0] | (sel[:, 1] & ~up))
    return sort_unique(np.concatenate(out0), np.concatenate(out1))


def space_open_shell_rich(n, na, opens, nconf, rng):
    """nconf distinct random configurations of 2 na electrons in n orbitals
    for each open-shell count in ``opens`` (na - k/2 doubly occupied
    orbitals, k open ones, chosen uniformly without overlap), closed over
    their spin placements at M_S = 0."""
    w0, w1 = [], []
    for k in opens:
        nd = na - k // 2
        seen = set()
        while len(seen) < nconf:
            perm = rng.permutation(n)
            docc = int(sum(1 << int(p) for p in perm[:nd]))
            opn = int(sum(1 << int(p) for p in perm[nd:nd + k]))
            if (docc, opn) in seen:
                continue
            seen.add((docc, opn))
            # one determinant per configuration: the lowest k/2 open orbitals alpha
            op = [p for p in range(n) if opn >> p & 1]
            up = sum(1 << p for p in op[:k // 2])
            w0.append(docc | up)
            w1.append(docc | (opn & ~up))
    seed = sort_unique(np.array(w0, np.uint64), np.array(w1, np.uint64))
    return complete_configurations(seed, n)


def random_space_spinfree(n, na, nb, ndet, rng):
    """ndet distinct determinants drawn uniformly from the full space (tiny n)."""
    full = space_fci(n, na, nb)
    idx = np.sort(rng.choice(len(full), size=min(ndet, len(full)), replace=False))
    return np.ascontiguousarray(full[idx])


def ci_vectors(ndet, nroots, rng, complex_=False):
    """[ndet][nroots] N(0,1) entries, each root column normalised to 1."""
    if complex_:
        c = rng.normal(size=(ndet, nroots)) + 1j * rng.normal(size=(ndet, nroots))
    else:
        c = rng.normal(size=(ndet, nroots))
    c = c / np.linalg.norm(c, axis=0, keepdims=True)
    return np.ascontiguousarray(c)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    kind: str                 # "spinfree" | "spinor"
    norb: int                 # spatial orbitals or Kramers pairs
    nalpha: int               # N_alpha (spin-free) or total N (spinor)
    nbeta: int                # N_beta (spin-free) or -1 (spinor)
    dets: np.ndarray          # [ndet][2] uint64, sorted
    h: np.ndarray
    g: np.ndarray
    ecore: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def ndet(self):
        return len(self.dets)

    @property
    def is_complex(self):
        return self.kind == "spinor"

    @property
    def nelec(self):
        return self.nalpha + (self.nbeta if self.kind == "spinfree" else 0)


def batch_shapes(i: int):
    """Shape of problem i of the 16-problem batch."""
    n = 16 + (32 * i) // 15
    ne = 6 + (6 * i) // 15
    nd = int(round(1e4 * 50 ** (i / 15)))
    return n, ne, nd


def workload(k: int, i: int = 0, scale: float = 1.0) -> Problem:
    """Workload k (0 FCI n=8 4a4b; 1 selected n=64 10a10b 2e6; 2 spinor
    40 pairs N=20 1e6; 3 batch problem i; 4 FD case n=10 3a3b FCI; 5 the
    variational space of the second-order energy, n=64 10a10b 2e4; 6 the
    singles-and-doubles space of n=64 10a10b, complete over its
    configurations, for the CSF basis; 7 an open-shell-rich
    configuration-complete space, n=32 8a8b with 10 and 12 open shells).

    ``scale`` < 1 shrinks the random part of selected spaces (for tests)."""
    if k == 0:
        n, na, nb = 8, 4, 4
        return Problem("spinfree", n, na, nb, space_fci(n, na, nb),
                       one_body_real(n, rng_for(0, 0, SEED_H)),
                       two_body_real(n, rng_for(0, 0, SEED_G)), name="fci-n8-4a4b")
    if k == 1:
        n, na = 64, 10
        target = int(2_000_000 * scale)
        d = space_selected_spinfree(n, na, na, max(target, 421_471), rng_for(1, 0, SEED_SPACE))
        return Problem("spinfree", n, na, na, d, one_body_real(n, rng_for(1, 0, SEED_H)),
                       two_body_real(n, rng_for(1, 0, SEED_G)), name="sci-n64-10a10b")
    if k == 2:
        nk, ne = 40, 20
        target = int(1_000_000 * scale)
        d = space_selected_spinor(nk, ne, max(target, 337_501), rng_for(2, 0, SEED_SPACE))
        return Problem("spinor", nk, ne, -1, d, one_body_spinor(nk, rng_for(2, 0, SEED_H)),
                       two_body_spinor(nk, rng_for(2, 0, SEED_G)), name="spinor-40kp-20e")
    if k == 3:
        n, ne, nd = batch_shapes(i)
        nd = int(nd * scale) if scale != 1.0 else nd
        d = space_selected_spinfree(n, ne, ne, nd, rng_for(3, i, SEED_SPACE))
        return Problem("spinfree", n, ne, ne, d, one_body_real(n, rng_for(3, i, SEED_H)),
                       two_body_real(n, rng_for(3, i, SEED_G)), name=f"batch{i}-n{n}-{ne}a{ne}b")
    if k == 5:
        # variational space of the second-order energy: n=64 10a10b with the
        # integrals of workload 1, HF + singles + random doubles
        n, na = 64, 10
        target = int(20_000 * scale)
        d = space_truncated_spinfree(n, na, na, max(target, 1081), rng_for(5, 0, SEED_SPACE))
        return Problem("spinfree", n, na, na, d, one_body_real(n, rng_for(1, 0, SEED_H)),
                       two_body_real(n, rng_for(1, 0, SEED_G)), name="pt2-n64-10a10b")
    if k == 6:
        # configuration-complete space for the CSF basis: HF, all singles and
        # all doubles of n=64 10a10b (closed under the configurations) with
        # the integrals of workload 1
        n, na = 64, 10
        _, _, w0, w1 = _hf_and_sd_spinfree(n, na, na)
        return Problem("spinfree", n, na, na, sort_unique(w0, w1), one_body_real(n, rng_for(1, 0, SEED_H)),
                       two_body_real(n, rng_for(1, 0, SEED_G)), name="sd-n64-10a10b")
    if k == 7:
        # open-shell-rich configuration-complete space for the CSF basis:
        # n=32 8a8b, random configurations with 10 or 12 open shells (3 or
        # 2 doubly occupied orbitals), every spin placement of each
        n, na = 32, 8
        nconf = int(1000 * scale) if scale != 1.0 else 1000
        d = space_open_shell_rich(n, na, (10, 12), nconf, rng_for(7, 0, SEED_SPACE))
        return Problem("spinfree", n, na, na, d, one_body_real(n, rng_for(7, 0, SEED_H)),
                       two_body_real(n, rng_for(7, 0, SEED_G)), name="open-n32-8a8b")
    if k == 4:
        n, na, nb = 10, 3, 3
        return Problem("spinfree", n, na, nb, space_fci(n, na, nb),
                       one_body_real(n, rng_for(4, 0, SEED_H)),
                       two_body_real(n, rng_for(4, 0, SEED_G)), name="fci-n10-3a3b")
    raise ValueError(k)
