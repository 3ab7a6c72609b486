"""Tier A: the Hamiltonian of section 2.1, Eq. (1), applied literally.

Test infrastructure only (see the package docstring).

Every term h_PQ a+_P a_Q and 1/2 (PQ|RS) a+_P a+_R a_S a_Q (the operator
e_{PQ,RS} of Eq. (2)) is applied, operator by operator, to every ket of the
space.  A determinant is packed into one integer with global position P at
bit P (all positions below 64), |D> = prod_{P in D ascending} a+_P |vac>, so
a+_X / a_X carry the sign (-1)^{#occupied positions below X}.  No
Slater-Condon rule and no integral symmetry is used.  Cost O(N M^4): small
spaces only.
"""
from __future__ import annotations

import numpy as np


def spin_orbital_integrals(prob):
    """h_PQ and (PQ|RS) over the M = 2n global positions.

    Spin-free: position p is (p, alpha), n+p is (p, beta); h_PQ and (PQ|RS)
    vanish unless the spins of P,Q (and R,S) agree.  Spinor: as given."""
    n = prob.norb
    if prob.kind == "spinor":
        return np.asarray(prob.h, np.complex128), np.asarray(prob.g, np.complex128)
    M = 2 * n
    h = np.zeros((M, M))
    g = np.zeros((M, M, M, M))
    for s in (0, 1):
        h[s * n:(s + 1) * n, s * n:(s + 1) * n] = prob.h
        for t in (0, 1):
            g[s * n:(s + 1) * n, s * n:(s + 1) * n, t * n:(t + 1) * n, t * n:(t + 1) * n] = prob.g
    return h, g


def packed(prob):
    n = prob.norb
    if 2 * n > 63:
        raise ValueError("tier A handles at most 31 orbitals per word")
    d = np.asarray(prob.dets, np.uint64)
    return (d[:, 0] | (d[:, 1] << np.uint64(n))).astype(np.uint64)


def _annihilate(x, sign, ok, X):
    bit = np.uint64(1) << np.uint64(X)
    ok = ok & ((x & bit) != 0)
    below = np.bitwise_count(x & (bit - np.uint64(1))).astype(np.int64)
    sign = sign * np.where(below % 2 == 1, -1, 1)
    return x & ~bit, sign, ok


def _create(x, sign, ok, X):
    bit = np.uint64(1) << np.uint64(X)
    ok = ok & ((x & bit) == 0)
    below = np.bitwise_count(x & (bit - np.uint64(1))).astype(np.int64)
    sign = sign * np.where(below % 2 == 1, -1, 1)
    return x | bit, sign, ok


class _Index:
    def __init__(self, keys):
        self.order = np.argsort(keys)
        self.sorted = keys[self.order]

    def lookup(self, x):
        pos = np.searchsorted(self.sorted, x)
        pos = np.minimum(pos, len(self.sorted) - 1)
        found = self.sorted[pos] == x
        return self.order[pos], found


def _apply(x0, ops):
    """ops: list of (position, create?) applied right to left as written
    (the last entry acts first)."""
    x = x0.copy()
    sign = np.ones(len(x0), np.int64)
    ok = np.ones(len(x0), bool)
    for X, cr in reversed(ops):
        x, sign, ok = (_create if cr else _annihilate)(x, sign, ok, X)
    return x, sign, ok


def hamiltonian(prob, tol=0.0):
    """Dense H_IJ = <I|H|J> over the space, from Eq. (1) term by term."""
    h, g = spin_orbital_integrals(prob)
    M = h.shape[0]
    x0 = packed(prob)
    N = len(x0)
    idx = _Index(x0)
    cplx = np.iscomplexobj(h) or np.iscomplexobj(g)
    H = np.zeros((N, N), dtype=np.complex128 if cplx else np.float64)
    cols = np.arange(N)
    for P in range(M):
        for Q in range(M):
            if abs(h[P, Q]) <= tol:
                continue
            x, s, ok = _apply(x0, [(P, True), (Q, False)])
            I, found = idx.lookup(x)
            m = ok & found
            np.add.at(H, (I[m], cols[m]), h[P, Q] * s[m])
    for P in range(M):
        for Q in range(M):
            for R in range(M):
                for S in range(M):
                    v = g[P, Q, R, S]
                    if abs(v) <= tol:
                        continue
                    x, s, ok = _apply(x0, [(P, True), (R, True), (S, False), (Q, False)])
                    I, found = idx.lookup(x)
                    m = ok & found
                    if m.any():
                        np.add.at(H, (I[m], cols[m]), 0.5 * v * s[m])
    H[np.diag_indices(N)] += prob.ecore
    return H


def operator_matrices_1(prob):
    """A[P][Q] = matrix of a+_P a_Q in the space basis (dict of sparse
    triplets), used for density matrices."""
    x0 = packed(prob)
    idx = _Index(x0)
    M = 2 * prob.norb
    cols = np.arange(len(x0))
    out = {}
    for P in range(M):
        for Q in range(M):
            x, s, ok = _apply(x0, [(P, True), (Q, False)])
            I, found = idx.lookup(x)
            m = ok & found
            if m.any():
                out[(P, Q)] = (I[m], cols[m], s[m])
    return out


def rdm(prob, bra, ket):
    """Transition gamma_PQ = <bra|a+_P a_Q|ket>, Gamma_PQRS =
    <bra|a+_P a+_R a_S a_Q|ket> over the M global positions (no spin sum)."""
    x0 = packed(prob)
    idx = _Index(x0)
    M = 2 * prob.norb
    cols = np.arange(len(x0))
    bra = np.asarray(bra).conj()
    ket = np.asarray(ket)
    gam = np.zeros((M, M), dtype=np.complex128)
    Gam = np.zeros((M, M, M, M), dtype=np.complex128)
    for P in range(M):
        for Q in range(M):
            x, s, ok = _apply(x0, [(P, True), (Q, False)])
            I, found = idx.lookup(x)
            m = ok & found
            gam[P, Q] = np.sum(bra[I[m]] * s[m] * ket[cols[m]])
    for P in range(M):
        for Q in range(M):
            for R in range(M):
                for S in range(M):
                    x, s, ok = _apply(x0, [(P, True), (R, True), (S, False), (Q, False)])
                    I, found = idx.lookup(x)
                    m = ok & found
                    if m.any():
                        Gam[P, Q, R, S] = np.sum(bra[I[m]] * s[m] * ket[cols[m]])
    return gam, Gam


def spin_sum(prob, gam, Gam):
    """Spin-free: gamma_pq = sum_s gamma_{ps,qs}; Gamma_pqrs = sum_{s,t}
    Gamma_{ps qs rt st}."""
    n = prob.norb
    g1 = np.zeros((n, n), dtype=gam.dtype)
    g2 = np.zeros((n, n, n, n), dtype=Gam.dtype)
    for s in (0, 1):
        g1 += gam[s * n:(s + 1) * n, s * n:(s + 1) * n]
        for t in (0, 1):
            g2 += Gam[s * n:(s + 1) * n, s * n:(s + 1) * n, t * n:(t + 1) * n, t * n:(t + 1) * n]
    return g1, g2
