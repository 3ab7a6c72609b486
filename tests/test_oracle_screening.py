"""Pins of the second-order energy screening and of the selection criterion
against hand-built problems whose results follow on paper from section 2.5
(step 4), Eqs. (iCI_Selection-1), (iCI_Selection-2) and Table 1 (SD column).

Each case is built so that the per-determinant rule |H_AJ| max_k |c_Jk|
(the earlier reading) gives a different kept set or energy: a same-spin
double whose integrals have opposite signs (|element| above the bound), an
alpha-beta double whose element is below the threshold while the exchange
integral in the bound is above it, a determinant double that is a
configuration single (never screened), the maximum over the determinants of
a configuration, a Kramers-partner integral in the spinor bound, the
selection's extra bound test of case (B), and the selection's maxima over
a configuration's determinants taken separately for its two tests.
"""
import numpy as np

from paper_2501_18185_amd import synth
from oracle import sc

REL = 1e-12


def _orbit8(g, p, q, r, s, v):
    for a, b, c, d in {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r), (r, s, p, q), (s, r, p, q),
                       (r, s, q, p), (s, r, q, p)}:
        g[a, b, c, d] = v


def _det(alpha, beta):
    return [sum(1 << p for p in alpha), sum(1 << p for p in beta)]


def _prob(n, na, nb, dets, h, g):
    d = np.array(sorted(dets, key=lambda x: (x[0], x[1])), dtype=np.uint64)
    return synth.Problem("spinfree", n, na, nb, d, h, g, 0.0)


def _h(n, diag):
    return np.diag(np.asarray(diag, dtype=float)) if len(diag) == n else None


def test_same_spin_double_opposite_signs():
    """n = 4, two alpha electrons, P = {alpha 0,1}, c = 1, E0 = H_JJ = -2.
    Only (20|31) = a and (21|30) = b are nonzero.  The double to alpha 2,3
    has |H_AJ| = |a - b| = 1.2e-3 and bound max(|a|, |b|) = 0.6e-3; the four
    singles have zero elements.  E2 = (a - b)^2 / (E0 - H_AA) = 1.44e-6 / (-3)
    at qmin = 0; at qmin = 1e-3 the double goes (bound < qmin / 1): E2 = 0,
    four kept pairs."""
    n = 4
    h = np.diag([-1.0, -1.0, 0.5, 0.5])
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 0, 3, 1, 0.6e-3)
    _orbit8(g, 2, 1, 3, 0, -0.6e-3)
    p = _prob(n, 2, 0, [_det([0, 1], [])], h, g)
    e2, kept, nq = sc.pt2(p, [1.0], -2.0, qmin=0.0)
    assert (kept, nq) == (5, 5)
    assert abs(e2[0] - 1.44e-6 / -3.0) <= REL * 1.44e-6 / 3.0
    e2, kept, nq = sc.pt2(p, [1.0], -2.0, qmin=1e-3)
    assert (kept, nq) == (4, 4)
    assert e2[0] == 0.0


def test_alpha_beta_double_kept_by_exchange_bound():
    """n = 4, one alpha one beta, P = {alpha 0, beta 1}, c = 1, E0 = -2.5.
    (20|31) = a = 0.5e-3 couples alpha 2 beta 3 (element a, below qmin =
    1e-3); (21|30) = b = 2e-3 couples alpha 3 beta 2 (element b); both lie in
    the configuration pair {0,1} -> {2,3}, bound max(|a|, |b|) = 2e-3, so
    both stay.  (10|31) = d = 0.2e-3 couples alpha 1 beta 3, a configuration
    single (orbital 0 -> 3), which is never screened.  H_AA = 1 for the first
    two, -0.5 for the third:  E2 = -(a^2 + b^2)/3.5 - d^2/2 at qmin = 0 and
    1e-3.  Of the 15 external determinants only alpha 2 beta 2 and alpha 3
    beta 3 (configuration doubles with bound 0) go at qmin = 1e-3."""
    n = 4
    a, b, d = 0.5e-3, 2e-3, 0.2e-3
    h = np.diag([-1.0, -1.0, 0.5, 0.5])
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 0, 3, 1, a)
    _orbit8(g, 2, 1, 3, 0, b)
    _orbit8(g, 1, 0, 3, 1, d)
    p = _prob(n, 1, 1, [_det([0], [1])], h, g)
    ref = -(a * a + b * b) / 3.5 - d * d / 2.0
    e2, kept, nq = sc.pt2(p, [1.0], -2.5, qmin=0.0)
    assert (kept, nq) == (15, 15)
    assert abs(e2[0] - ref) <= REL * abs(ref)
    e2, kept, nq = sc.pt2(p, [1.0], -2.5, qmin=1e-3)
    assert (kept, nq) == (13, 13)
    assert abs(e2[0] - ref) <= REL * abs(ref)


def test_configuration_maximum_over_determinants():
    """n = 4, one alpha one beta, P = {alpha 0 beta 1 (c = 1e-2), alpha 1 beta
    0 (c = 1)}: one configuration.  Only (20|31) = a = 1e-2 is nonzero, so
    A = alpha 2 beta 3 couples to the first (element a, |a c| = 1e-4 <
    qmin = 1e-3) and A' = alpha 3 beta 2 to the second (element a).  The bound
    of the configuration pair is 1e-2 and max|C| over the configuration is 1,
    so every pair into {2,3} stays: E2 is the same at qmin = 0 and 1e-3
    (the pairs that go have zero elements), ((a 1e-2)^2 + a^2) / (E0 - 1),
    E0 = -2.5."""
    n = 4
    a = 1e-2
    h = np.diag([-1.0, -1.0, 0.5, 0.5])
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 0, 3, 1, a)
    p = _prob(n, 1, 1, [_det([0], [1]), _det([1], [0])], h, g)
    # sorted: alpha 0 beta 1 = (1, 2) first, alpha 1 beta 0 = (2, 1) second
    c = np.array([1e-2, 1.0])
    e0 = -2.5
    ref = ((a * 1e-2) ** 2 + a ** 2) / (e0 - 1.0)
    e2a, _, _ = sc.pt2(p, c, e0, qmin=0.0)
    e2b, _, _ = sc.pt2(p, c, e0, qmin=1e-3)
    assert abs(e2a[0] - ref) <= REL * abs(ref)
    assert abs(e2b[0] - ref) <= REL * abs(ref)


def test_spinor_bound_takes_kramers_partners():
    """Spinor, 4 Kramers pairs, N = 2, P = {A0, A1} (positions 0 and 1),
    c = 1, E0 = -2.5.  Only (6 0|3 1) = 2e-3 and its partners under (PQ|RS) = (RS|PQ) =
    conj((QP|SR)) are nonzero; position 6 is the barred partner of pair 2.
    The 15 doubles of P include six configuration doubles: four into pairs
    {2, 3} (bound 2e-3 over the partners, kept at qmin = 1e-3 although three
    have zero elements) and two into {2, 2} or {3, 3} (bound 0, dropped):
    27 external determinants at qmin = 0, 25 at qmin = 1e-3."""
    nk = 4
    M = 2 * nk
    h = np.diag(np.array([-1.0, -1.0, 0.5, 0.5] * 2)).astype(complex)
    g = np.zeros((M,) * 4, complex)
    for P, Q, R, S in [(6, 0, 3, 1), (3, 1, 6, 0), (0, 6, 1, 3), (1, 3, 0, 6)]:
        g[P, Q, R, S] = 2e-3
    d = np.array([[0b11, 0]], np.uint64)
    p = synth.Problem("spinor", nk, 2, -1, d, h, g, 0.0)
    e2a, kept, nq = sc.pt2(p, [1.0], -2.5, qmin=0.0)
    assert (kept, nq) == (27, 27)
    e2b, kept, nq = sc.pt2(p, [1.0], -2.5, qmin=1e-3)
    assert (kept, nq) == (25, 25)
    assert abs(e2a[0] - e2b[0]) <= REL * abs(e2a[0])


def test_select_case_b_bound_test():
    """Selection from the same-spin problem of the first test with E0 = 0.5
    (|E0 - H_AA| = 0.5): the double alpha 2,3 passes both per-pair tests
    (|H c| = 1.2e-3, |H c / 0.5| = 2.4e-3 >= cmin = 1e-3) but its bound
    0.6e-3 times max|C| = 1 is below cmin: nothing is selected.  With a =
    1.2e-3, b = 0 the bound is 1.2e-3 and it is selected."""
    n = 4
    h = np.diag([-1.0, -1.0, 0.5, 0.5])
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 0, 3, 1, 0.6e-3)
    _orbit8(g, 2, 1, 3, 0, -0.6e-3)
    p = _prob(n, 2, 0, [_det([0, 1], [])], h, g)
    assert len(sc.select(p, [1.0], 0.5, 1e-3)) == 0
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 0, 3, 1, 1.2e-3)
    p = _prob(n, 2, 0, [_det([0, 1], [])], h, g)
    assert sc.select(p, [1.0], 0.5, 1e-3).tolist() == [_det([2, 3], [])]


def test_select_configuration_maxima_per_test():
    """Two roots, n = 3, one alpha one beta, P = {alpha 0 beta 1 with c =
    (1, 0), alpha 1 beta 0 with c = (0, 1)}, one configuration.  h_20 = x =
    2e-3 and (21|10) = y = 0.5e-3 couple A = alpha 2 beta 1 (a configuration
    single: case A) to the first by x and to the second by y; H_AA = 0.5,
    E0 = (H_AA - 4, H_AA - 0.25).  The first determinant passes only the
    first test (|x| >= cmin, |x| / 4 < cmin), the second only the second
    (|y| < cmin, |y| / 0.25 >= cmin); the maxima over the configuration's
    determinants pass both, so A is selected (cmin = 1e-3)."""
    n = 3
    x, y = 2e-3, 0.5e-3
    h = np.diag([0.0, 0.0, 0.5])
    h[2, 0] = h[0, 2] = x
    g = np.zeros((n,) * 4)
    _orbit8(g, 2, 1, 1, 0, y)
    p = _prob(n, 1, 1, [_det([0], [1]), _det([1], [0])], h, g)
    c = np.array([[1.0, 0.0], [0.0, 1.0]])
    e0 = np.array([0.5 - 4.0, 0.5 - 0.25])
    sel = sc.select(p, c, e0, 1e-3).tolist()
    assert _det([2], [1]) in sel
