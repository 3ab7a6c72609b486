"""Pins of the CSF oracle (``oracle/csf.py``) against facts it does not
produce itself: the general Clebsch-Gordan formula, the branching-rule
count of spin functions, textbook spin functions, orthonormality, the
total-spin operator built from creation and annihilation operators, and the
spin-resolved spectrum of the determinant Hamiltonian."""
import itertools
import math

import numpy as np
import pytest

from paper_2501_18185_amd import synth
from oracle import csf, literal, sc


def _prob(n, na, nb, dets, seed=3):
    rng = np.random.default_rng(seed)
    h, g = synth.one_body_real(n, rng), synth.two_body_real(n, rng)
    return synth.Problem("spinfree", n, na, nb, np.ascontiguousarray(dets, np.uint64), h, g, 0.25)


def _racah_cg(j1, m1, j2, m2, J, M):
    """<j1 m1; j2 m2 | J M> by Racah's closed formula (sum over k)."""
    if abs(m1 + m2 - M) > 1e-9 or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    f = math.factorial

    def F(x):
        return f(int(round(x)))

    pre = math.sqrt((2 * J + 1) * F(J + j1 - j2) * F(J - j1 + j2) * F(j1 + j2 - J) / F(j1 + j2 + J + 1))
    pre *= math.sqrt(F(J + M) * F(J - M) * F(j1 - m1) * F(j1 + m1) * F(j2 - m2) * F(j2 + m2))
    s = 0.0
    for k in range(0, 100):
        args = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if any(a < -1e-9 for a in args):
            continue
        if args[1] < 0 or args[2] < 0 or args[3] < 0:
            break
        s += (-1) ** k / np.prod([F(a) for a in args])
    return pre * s


def test_cg_half_equals_racah():
    """The spin-1/2 coupling coefficients equal the general formula."""
    for two_s1 in range(0, 11):
        for two_s in (two_s1 - 1, two_s1 + 1):
            if two_s < 0:
                continue
            for two_m in range(-two_s, two_s + 1, 2):
                for two_ms in (1, -1):
                    two_m1 = two_m - two_ms
                    if abs(two_m1) > two_s1:
                        continue
                    ref = _racah_cg(two_s1 / 2, two_m1 / 2, 0.5, two_ms / 2, two_s / 2, two_m / 2)
                    assert abs(csf.cg_half(two_s1, two_m1, two_ms, two_s, two_m) - ref) < 1e-13


def test_path_count_branching_rule():
    """Number of spin functions of k open shells at spin S:
    C(k, k/2 - S) - C(k, k/2 - S - 1)."""
    for k in range(0, 13):
        for two_s in range(k % 2, k + 1, 2):
            lo = (k - two_s) // 2
            ref = math.comb(k, lo) - (math.comb(k, lo - 1) if lo >= 1 else 0)
            assert len(csf.paths(k, two_s)) == ref


def _fn(path, k, two_s):
    return {s: csf.spin_coefficient(path, s)
            for s in itertools.product((1, -1), repeat=k) if sum(s) == two_s}


def test_textbook_spin_functions():
    """Genealogical spin functions of two to four spins (e.g. Pauncz, Spin
    Eigenfunctions, ch. 3; alpha = +1, beta = -1, spins in orbital order)."""
    r2, r6 = math.sqrt(2.0), math.sqrt(6.0)
    # two spins: singlet (ab - ba)/sqrt2; triplet M = 1: aa
    f = _fn((1, 0), 2, 0)
    assert abs(f[(1, -1)] - 1 / r2) < 1e-15 and abs(f[(-1, 1)] + 1 / r2) < 1e-15
    assert _fn((1, 2), 2, 2) == {(1, 1): 1.0}
    # three spins, S = 1/2: (2aab - aba - baa)/sqrt6 and (aba - baa)/sqrt2
    assert csf.paths(3, 1) == [(1, 2, 1), (1, 0, 1)]
    f = _fn((1, 2, 1), 3, 1)
    assert abs(f[(1, 1, -1)] - 2 / r6) < 1e-15
    assert abs(f[(1, -1, 1)] + 1 / r6) < 1e-15 and abs(f[(-1, 1, 1)] + 1 / r6) < 1e-15
    f = _fn((1, 0, 1), 3, 1)
    assert f[(1, 1, -1)] == 0.0
    assert abs(f[(1, -1, 1)] - 1 / r2) < 1e-15 and abs(f[(-1, 1, 1)] + 1 / r2) < 1e-15
    # four spins, singlet of two singlet pairs: the product (ab - ba)(ab - ba)/2
    f = _fn((1, 0, 1, 0), 4, 0)
    for s, v in f.items():
        pair = lambda a, b: (a == 1 and b == -1) - (a == -1 and b == 1)
        assert abs(v - pair(s[0], s[1]) * pair(s[2], s[3]) / 2.0) < 1e-15
    # four spins, the other singlet (first pair a triplet): proportional to
    # 2aabb + 2bbaa - abab - abba - baab - baba, norm 1
    f = _fn((1, 2, 1, 0), 4, 0)
    ref = {(1, 1, -1, -1): 2, (-1, -1, 1, 1): 2, (1, -1, 1, -1): -1, (1, -1, -1, 1): -1,
           (-1, 1, 1, -1): -1, (-1, 1, -1, 1): -1}
    scale = f[(1, 1, -1, -1)] / 2
    assert abs(abs(scale) - 1 / math.sqrt(12.0)) < 1e-15
    for s, v in ref.items():
        assert abs(f[s] - scale * v) < 1e-15


def test_operator_sign_brute_force():
    """The determinant sign equals applying the creation operators one by
    one to the vacuum, right to left (the tier-A operator routine)."""
    n = 5
    rng = np.random.default_rng(7)
    for _ in range(40):
        orbs = rng.permutation(n)
        m, k = rng.integers(0, 3), rng.integers(0, 4)
        docc, opn = sorted(orbs[:m].tolist()), sorted(orbs[m:m + k].tolist())
        spins = tuple(int(x) for x in rng.choice([1, -1], size=k))
        sign, w0, w1 = csf.operator_determinant(docc, opn, spins, n)
        ops = []
        for d in docc:
            ops += [(d, True), (n + d, True)]
        for o, s in zip(opn, spins):
            ops.append((o if s > 0 else n + o, True))
        x, sg, ok = literal._apply(np.zeros(1, np.uint64), ops)
        assert ok[0] and int(x[0]) == (w0 | (w1 << n)) and int(sg[0]) == sign


SPACES = [(5, 3, 2), (6, 3, 3), (6, 4, 2), (5, 4, 1), (6, 2, 2)]


def _s_minus(prob):
    """S_- = sum_p a+_{p beta} a_{p alpha} from the space into the images
    (tier-A operator application); returns the matrix and nothing else."""
    n = prob.norb
    x0 = literal.packed(prob)
    cols, rows, vals, index = [], [], [], {}
    for p in range(n):
        x, s, ok = literal._apply(x0, [(n + p, True), (p, False)])
        for j in np.nonzero(ok)[0]:
            key = int(x[j])
            if key not in index:
                index[key] = len(index)
            rows.append(index[key]); cols.append(j); vals.append(s[j])
    S = np.zeros((max(len(index), 1), len(x0)))
    np.add.at(S, (rows, cols), vals)
    return S


@pytest.mark.parametrize("n,na,nb", SPACES)
def test_expansion_orthonormal_spin_eigenfunctions(n, na, nb):
    """T^T T = 1, and S^2 T = S(S+1) T with S^2 = S_+ S_- + S_z^2 - S_z,
    S_+ = S_-^T, on FCI spaces (M_S = S)."""
    p = _prob(n, na, nb, synth.space_fci(n, na, nb))
    two_s = na - nb
    T, first = csf.expansion(p, two_s)
    T = T.toarray()
    assert np.abs(T.T @ T - np.eye(T.shape[1])).max() < 1e-13
    Sm = _s_minus(p)
    S, M = two_s / 2, two_s / 2
    S2 = Sm.T @ Sm + (M * M - M) * np.eye(p.ndet)
    assert np.abs(S2 @ T - S * (S + 1) * T).max() < 1e-12
    # every spin-S state of the space is reached: dim = number of CSFs
    w = np.linalg.eigvalsh(S2)
    assert int(np.sum(np.abs(w - S * (S + 1)) < 1e-8)) == T.shape[1]


@pytest.mark.parametrize("n,na,nb", SPACES[:4])
def test_spectrum_equals_spin_sector(n, na, nb):
    """eig(T^T H T) = the eigenvalues of H on its S(S+1) eigenspace of S^2."""
    p = _prob(n, na, nb, synth.space_fci(n, na, nb), seed=n + na)
    two_s = na - nb
    T = csf.expansion(p, two_s)[0].toarray()
    H = literal.hamiltonian(p)
    Sm = _s_minus(p)
    M = two_s / 2
    w, V = np.linalg.eigh(Sm.T @ Sm + (M * M - M) * np.eye(p.ndet))
    Vs = V[:, np.abs(w - M * (M + 1)) < 1e-8]
    e1 = np.linalg.eigvalsh(T.T @ H @ T)
    e2 = np.linalg.eigvalsh(Vs.T @ H @ Vs)
    assert np.abs(e1 - e2).max() < 1e-11


def test_selected_space_sigma_and_completeness():
    """On a configuration-complete selected space: T^T T = 1, the CSF sigma
    through tier B equals T^T H T c with H from tier A, and a space missing
    one determinant of a configuration is refused."""
    n, na, nb = 8, 3, 3
    rng = np.random.default_rng(11)
    base = synth.random_space_spinfree(n, na, nb, 60, rng)
    d = synth.complete_configurations(base, n)
    p = _prob(n, na, nb, d, seed=5)
    T, first = csf.expansion(p, 0)
    assert np.abs((T.T @ T).toarray() - np.eye(T.shape[1])).max() < 1e-13
    c = np.random.default_rng(1).standard_normal((T.shape[1], 2))
    got = csf.sigma(p, 0, c, sc.sigma)
    Td = T.toarray()
    ref = Td.T @ literal.hamiltonian(p) @ Td @ c
    assert np.abs(got - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
    # configurations in the order of their first determinant
    cfgs, of = csf.configurations(p.dets)
    assert np.all(np.diff(np.unique(of, return_index=True)[1]) > 0)
    # a missing determinant of an open-shell configuration
    k = np.bitwise_count(d[:, 0] ^ d[:, 1])
    drop = int(np.nonzero(k >= 2)[0][0])
    q = _prob(n, na, nb, np.delete(d, drop, axis=0))
    with pytest.raises(ValueError):
        csf.expansion(q, 0)
    with pytest.raises(ValueError):
        csf.expansion(p, 2)


def test_open_shell_rich_space_recipe():
    """The open-shell-rich input recipe: electron counts per spin, only the
    requested open-shell counts, closed over configurations, and the
    expected number of spin placements per configuration."""
    from math import comb
    n, na = 12, 4
    d = synth.space_open_shell_rich(n, na, (4, 6), 20, np.random.default_rng(5))
    a, b = d[:, 0], d[:, 1]
    assert (np.bitwise_count(a) == na).all() and (np.bitwise_count(b) == na).all()
    k = np.bitwise_count(a ^ b)
    assert set(np.unique(k).tolist()) == {4, 6}
    assert np.array_equal(synth.complete_configurations(d, n), d)
    # 20 configurations of each kind, C(k, k/2) placements each
    assert (k == 4).sum() == 20 * comb(4, 2) and (k == 6).sum() == 20 * comb(6, 3)
