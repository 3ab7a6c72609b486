"""Configuration state functions (CSFs) written out in determinants.

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU library never
loads this module.

Section 2.3: an orbital configuration (oCFG) generates several many-electron
functions, CSFs for spin-free problems, distinguished by their spin coupling,
and the Yamanouchi-Kotani phase lets orbitals that are doubly occupied in a
configuration be moved freely.  Section 2.2 stores a configuration as its
doubly occupied and singly occupied orbitals.  The definition followed here,
for a space with N_alpha - N_beta = 2S (M_S = S):

* configuration: doubly occupied orbitals d_1 < ... < d_m and singly
  occupied (open) orbitals o_1 < ... < o_k of a determinant (alpha word A,
  beta word B): docc = A & B, open = A ^ B;
* spin function: the genealogical (Yamanouchi-Kotani) coupling of the k
  open-shell spins in orbital order.  A path is the list of intermediate
  spins 2S_1, ..., 2S_k (S_1 = 1/2, each step +-1/2, never negative,
  S_k = S); the coefficient of the spin product (s_1, ..., s_k) is the
  product of Clebsch-Gordan coefficients <S_{i-1} M_{i-1}; 1/2 s_i | S_i M_i>,
  M_i = s_1 + ... + s_i (Condon-Shortley phase);
* CSF |I mu> = sum over spin products of that coefficient times
  a+_{d_1 a} a+_{d_1 b} ... a+_{d_m a} a+_{d_m b} a+_{o_1 s_1} ... a+_{o_k s_k} |vac>,
  rewritten in the determinant convention of the space (creation operators
  in ascending global position, alpha orbital p at p and beta orbital p at
  n + p), which costs the sign of the sorting permutation;
* order: configurations by their first determinant in the space order;
  the paths of one configuration lexicographically, step up before step
  down.

Nothing here is tuned: every coefficient is a Python loop over spin
products.  Small spaces only.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def cg_half(two_s1, two_m1, two_ms, two_s, two_m):
    """<S1 M1; 1/2 ms | S M>, all arguments doubled (Condon-Shortley).

    Coupling a spin 1/2 to S1: S = S1 + 1/2 gives sqrt((S + 2 ms M) / 2S),
    S = S1 - 1/2 gives -2 ms sqrt((S + 1 - 2 ms M) / (2S + 2))."""
    if two_m1 + two_ms != two_m or abs(two_m) > two_s or abs(two_m1) > two_s1 or abs(two_ms) != 1:
        return 0.0
    S, M, ms = two_s / 2.0, two_m / 2.0, two_ms / 2.0
    if two_s == two_s1 + 1:
        return math.sqrt((S + 2.0 * ms * M) / (2.0 * S))
    if two_s == two_s1 - 1:
        return -2.0 * ms * math.sqrt((S + 1.0 - 2.0 * ms * M) / (2.0 * S + 2.0))
    return 0.0


def paths(k, two_s):
    """Coupling paths (2S_1, ..., 2S_k) ending at 2S, step up first."""
    out = []

    def walk(prefix, b):
        i = len(prefix)
        if i == k:
            if b == two_s:
                out.append(tuple(prefix))
            return
        for step in (1, -1):
            nb = b + step
            if nb < 0 or abs(nb - two_s) > k - i - 1:
                continue
            walk(prefix + [nb], nb)

    walk([], 0)
    return out


def spin_coefficient(path, spins):
    """Genealogical coefficient of the spin product ``spins`` (+1 alpha,
    -1 beta, doubled) on ``path``."""
    b, m, v = 0, 0, 1.0
    for bi, s in zip(path, spins):
        v *= cg_half(b, m, s, bi, m + s)
        if v == 0.0:
            return 0.0
        b, m = bi, m + s
    return v


def operator_determinant(docc, opn, spins, n):
    """The product of creation operators of one spin product, in the
    configuration's order (pairs first, then open shells), as (sign, alpha
    word, beta word) in ascending-position order.  The sign is that of the
    sorting permutation (its inversion count)."""
    seq = []
    for d in docc:
        seq += [d, n + d]
    for o, s in zip(opn, spins):
        seq.append(o if s > 0 else n + o)
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    w0 = sum(1 << p for p in seq if p < n)
    w1 = sum(1 << (p - n) for p in seq if p >= n)
    return (-1) ** inv, w0, w1


def _bits(x):
    return [p for p in range(128) if (x >> p) & 1]


def configurations(dets):
    """(doubly occupied mask, open mask) of every configuration, in the
    order of its first determinant, and the configuration of each determinant."""
    seen, cfgs, of = {}, [], []
    for a, b in dets:
        a, b = int(a), int(b)
        key = (a & b, a ^ b)
        if key not in seen:
            seen[key] = len(cfgs)
            cfgs.append(key)
        of.append(seen[key])
    return cfgs, np.array(of, np.int64)


def config_block(dmask, omask, n, two_s):
    """The CSFs of one configuration (doubly occupied and open orbital
    masks) as entries (mu, alpha word, beta word, coefficient), and their
    number."""
    docc, opn = _bits(dmask), _bits(omask)
    k = len(opn)
    products = [s for s in itertools.product((1, -1), repeat=k) if sum(s) == two_s]
    out = []
    ps = paths(k, two_s)
    for mu, path in enumerate(ps):
        for spins in products:
            v = spin_coefficient(path, spins)
            if v == 0.0:
                continue
            sign, w0, w1 = operator_determinant(docc, opn, spins, n)
            out.append((mu, w0, w1, sign * v))
    return out, len(ps)


def expansion(prob, two_s):
    """The CSF basis of the space: T [ndet][ncsf] (scipy CSC) with column
    mu of configuration I holding |I mu> in determinants, and the first CSF
    of each configuration ([ncfg + 1]).

    Raises ValueError unless the space is spin-free with N_alpha - N_beta =
    2S and holds every determinant of each of its configurations."""
    import scipy.sparse as sp
    if prob.kind != "spinfree":
        raise ValueError("CSFs are defined for spin-free problems")
    if prob.nalpha - prob.nbeta != two_s or two_s < 0:
        raise ValueError("the space must have N_alpha - N_beta = 2S")
    n = prob.norb
    dets = [(int(a), int(b)) for a, b in np.asarray(prob.dets, np.uint64)]
    index = {d: i for i, d in enumerate(dets)}
    cfgs, of = configurations(dets)
    count = np.bincount(of, minlength=len(cfgs))
    rows, cols, vals, first = [], [], [], [0]
    col = 0
    for ci, (dmask, omask) in enumerate(cfgs):
        k = bin(omask).count("1")
        nup = (k + two_s) // 2
        if count[ci] != math.comb(k, nup):
            raise ValueError("configuration %d holds %d of its %d determinants" % (ci, count[ci], math.comb(k, nup)))
        block, f = config_block(dmask, omask, n, two_s)
        for mu, w0, w1, v in block:
            rows.append(index[(w0, w1)])
            cols.append(col + mu)
            vals.append(v)
        col += f
        first.append(col)
    T = sp.csc_matrix((np.array(vals, np.float64), (np.array(rows, np.int64), np.array(cols, np.int64))),
                      shape=(len(dets), col))
    return T, np.array(first, np.int64)


def to_det(prob, two_s, x):
    """Determinant coefficients of the CSF vector(s) x: T x."""
    T, _ = expansion(prob, two_s)
    return T @ np.asarray(x, np.float64)


def from_det(prob, two_s, y):
    """CSF components of the determinant vector(s) y: T^T y."""
    T, _ = expansion(prob, two_s)
    return T.T @ np.asarray(y, np.float64)


def sigma(prob, two_s, c, sigma_det):
    """sigma in the CSF basis: T^T H T c, with ``sigma_det`` the
    determinant-basis product (a callback, e.g. the Slater-Condon tier).
    Exact because the CSFs lie in the span of the space's determinants."""
    T, _ = expansion(prob, two_s)
    c = np.asarray(c, np.float64)
    return T.T @ np.asarray(sigma_det(prob, T @ c), np.float64)
