"""GPU tests of the fixed-point density-matrix mode (mw_plan_set_rdm_mode 1).

Bar: against the oracle within 1e-12 of the largest entry (as the atomic
mode); within 1e-12 of the atomic mode; the same bits on repeated calls, in
a captured graph (the serial launch order) and eagerly (the single rows
and occupation correlations on a second stream beside the double rows);
bra and ket scaled by powers of two give exactly scaled matrices; a zero
bra gives exact zeros.  Spaces: spin-free FCI and selected spaces, complex
spinor spaces, the 102-spinor space whose single rows exceed the LDS of a
workgroup (the per-pair kernel), and the 2,000,000-determinant n=64 space.
"""
import sys

import numpy as np
import pytest

from paper_2501_18185_amd import synth
from oracle import sc

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def _prob(kind, n, na, nb, dets, h, g, ecore=0.0):
    return synth.Problem(kind, n, na, nb, np.ascontiguousarray(dets, np.uint64), h, g, ecore)


def _spinor_problem(nk, nel, target, seed):
    rng = np.random.default_rng(seed)
    d = synth.space_selected_spinor(nk, nel, target, rng)
    return _prob("spinor", nk, nel, -1, d, synth.one_body_spinor(nk, rng), synth.two_body_spinor(nk, rng))


def _spinor_pairs_102():
    """All 5,151 two-electron determinants over 102 spinors: single rows of
    168 KB, beyond a workgroup's LDS, so the per-pair kernel runs."""
    nk = 51
    M = 2 * nk
    dets = []
    for a in range(M):
        for b in range(a + 1, M):
            w = [0, 0]
            for x in (a, b):
                w[x // nk] |= 1 << (x % nk)
            dets.append(w)
    dets.sort(key=lambda d: (d[0], d[1]))
    h = np.diag(np.linspace(-2.0, 1.0, M)).astype(np.complex128)
    g = np.zeros((M, M, M, M), np.complex128)
    return synth.Problem("spinor", nk, 2, -1, np.array(dets, np.uint64), h, g, 0.0)


def _case(name):
    """(problem, bra, ket or None for ket = bra, weights, max_roots)"""
    if name == "fci-n8":
        p = synth.workload(0)
        c = synth.ci_vectors(p.ndet, 1, np.random.default_rng(1))
        return p, c, None, None, 1
    if name == "sci-3roots":
        p = synth.workload(4)
        c = synth.ci_vectors(p.ndet, 3, np.random.default_rng(2))
        k = synth.ci_vectors(p.ndet, 3, np.random.default_rng(3))
        return p, c, k, [0.5, 0.3, 0.2], 3
    if name == "sci-6roots":
        p = synth.workload(4)
        c = synth.ci_vectors(p.ndet, 6, np.random.default_rng(4))
        return p, c, None, list(np.linspace(0.9, 0.1, 6)), 6
    if name == "spinor":
        p = _spinor_problem(8, 6, 2000, 3)
        c = synth.ci_vectors(p.ndet, 1, np.random.default_rng(5), complex_=True)
        return p, c, None, None, 1
    if name == "spinor-2roots":
        p = _spinor_problem(8, 6, 2000, 3)
        c = synth.ci_vectors(p.ndet, 2, np.random.default_rng(6), complex_=True)
        k = synth.ci_vectors(p.ndet, 2, np.random.default_rng(7), complex_=True)
        return p, c, k, [0.75, 0.25], 2
    if name == "spinor-102":
        p = _spinor_pairs_102()
        c = synth.ci_vectors(p.ndet, 1, np.random.default_rng(8), complex_=True)
        return p, c, None, None, 1
    raise KeyError(name)


def _rdm(pl, bd, kd, w):
    return pl.rdm(bd, bd if kd is None else kd, weights=w)


@pytest.mark.parametrize("name", ["fci-n8", "sci-3roots", "sci-6roots", "spinor", "spinor-2roots", "spinor-102"])
def test_fixed_point_rdm_equals_oracle_and_repeats_bitwise(torch, name):
    from paper_2501_18185_amd import mw
    p, c, k, w, R = _case(name)
    _say(f"[rdm-fixed] {name}: ndet={p.ndet} roots={c.shape[1]} one vector={k is None}")
    pl = mw.Plan(p, max_roots=R)
    bd = _dev(torch, c)
    kd = None if k is None else _dev(torch, k)
    mw.profile(True)
    a1, a2 = (x.cpu().numpy() for x in _rdm(pl, bd, kd, w))
    mw.profile(False)
    assert mw.profile_read("rdm_fx_scale")[0] == 0  # float atomics: no fixed-point scale
    pl.rdm_fixed_point = True
    mw.profile(True)
    f1, f2 = (x.cpu().numpy() for x in _rdm(pl, bd, kd, w))
    mw.profile(False)
    assert mw.profile_read("rdm_fx_scale")[0] == 1  # the fixed-point path ran
    for _ in range(2):
        g1, g2 = (x.cpu().numpy() for x in _rdm(pl, bd, kd, w))
        assert np.array_equal(g1, f1) and np.array_equal(g2, f2), name
    if name == "spinor-102":
        rows = np.arange(p.ndet)
        r1, r2 = sc.rdm(p, c, c, weights=w, rows=rows[:: 17])
        # the oracle over a subset of bra rows: compare the same restriction
        cs = np.zeros_like(c)
        cs[rows[:: 17]] = c[rows[:: 17]]
        s1, s2 = (x.cpu().numpy() for x in pl.rdm(_dev(torch, cs), bd, weights=w))
        assert _rel(s1, r1) <= TOL and _rel(s2, r2) <= TOL
    else:
        r1, r2 = sc.rdm(p, c, c if k is None else k, weights=w)
        assert _rel(f1, r1) <= TOL and _rel(f2, r2) <= TOL, (name, _rel(f1, r1), _rel(f2, r2))
    assert _rel(f1, a1) <= TOL and _rel(f2, a2) <= TOL
    _say(f"[rdm-fixed] {name}: fixed vs atomic {_rel(f1, a1):.2e} {_rel(f2, a2):.2e}")


@pytest.mark.parametrize("name", ["sci-3roots", "spinor-2roots"])
def test_fixed_point_rdm_scales_exactly(torch, name):
    """bra 2^7 and ket 2^-3: both matrices exactly 2^4 times the unscaled;
    bra 2^-600 and 2^700 likewise; a zero bra gives exact zeros."""
    from paper_2501_18185_amd import mw
    p, c, k, w, R = _case(name)
    pl = mw.Plan(p, max_roots=R)
    pl.rdm_fixed_point = True
    g1, g2 = (x.cpu().numpy() for x in pl.rdm(_dev(torch, c), _dev(torch, k), weights=w))
    h1, h2 = (x.cpu().numpy() for x in pl.rdm(_dev(torch, c * 128.0), _dev(torch, k / 8.0), weights=w))
    assert np.array_equal(h1, 16.0 * g1) and np.array_equal(h2, 16.0 * g2)
    # far from 1, where the squares of the coefficients underflow (2^-600)
    # or overflow (2^700) in double: the scale follows the bound's exponent
    for e in (-600, 700):
        f = 2.0 ** e
        h1, h2 = (x.cpu().numpy() for x in pl.rdm(_dev(torch, c * f), _dev(torch, k), weights=w))
        assert np.array_equal(h1, f * g1) and np.array_equal(h2, f * g2), e
    z1, z2 = (x.cpu().numpy() for x in pl.rdm(_dev(torch, 0.0 * c), _dev(torch, k), weights=w))
    assert not np.any(z1) and not np.any(z2)


def test_fixed_point_rdm_graph_replays_equal_eager(torch):
    """Captured (one stream, serial order) and eager (second stream beside
    the double rows): the same bits, on every replay."""
    from paper_2501_18185_amd import mw
    p, c, _, _, _ = _case("fci-n8")
    pl = mw.Plan(p)
    pl.rdm_fixed_point = True
    bd = _dev(torch, c)
    e1, e2 = pl.rdm(bd, bd)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pl.rdm(bd, bd)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        o1, o2 = pl.rdm(bd, bd)
    for rep in range(3):
        o1.fill_(7.0)
        o2.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        x1, x2 = pl.rdm(bd, bd)
        torch.cuda.synchronize()
        assert torch.equal(o1, e1) and torch.equal(o2, e2), rep
        assert torch.equal(x1, e1) and torch.equal(x2, e2), rep


def test_fixed_point_energy_gradients_repeat_bitwise(torch):
    """mw_energy_backward and the batched backward (a captured graph keyed
    by the mode) in fixed point: the same bits on repeated calls, and the
    integral gradients within 1e-12 of the atomic mode's."""
    from paper_2501_18185_amd import mw
    p = synth.workload(4)
    pl = mw.Plan(p, max_roots=2)
    c = _dev(torch, synth.ci_vectors(p.ndet, 2, np.random.default_rng(9)))
    sig = pl.sigma(c)
    ge = torch.tensor([0.7, 0.3], dtype=torch.float64, device="cuda")
    _, ah, ag = pl.energy_backward(c, sig, ge)
    ba = mw.energy_backward_batched([pl], [c], [sig], [ge])
    pl.rdm_fixed_point = True
    _, fh, fg = pl.energy_backward(c, sig, ge)
    for _ in range(2):
        _, h2, g2 = pl.energy_backward(c, sig, ge)
        assert torch.equal(h2, fh) and torch.equal(g2, fg)
    bf = mw.energy_backward_batched([pl], [c], [sig], [ge])
    bf2 = mw.energy_backward_batched([pl], [c], [sig], [ge])
    torch.cuda.synchronize()
    assert torch.equal(bf[1][0], fh) and torch.equal(bf[2][0], fg)
    assert torch.equal(bf2[1][0], fh) and torch.equal(bf2[2][0], fg)
    for x, y in ((fh, ah), (fg, ag), (bf[1][0], ba[1][0]), (bf[2][0], ba[2][0])):
        assert _rel(x.cpu().numpy(), y.cpu().numpy()) <= TOL


def test_fixed_point_rdm_full_n64(torch):
    """The 2,000,000-determinant n=64 10a10b space: fixed point within 1e-12
    of the atomic mode (whose sampled rows the oracle checks), the same bits
    on a second call, and E = sum h gamma + 1/2 sum g Gamma equal to c.sigma."""
    from paper_2501_18185_amd import mw
    p = synth.workload(1)
    pl = mw.Plan(p)
    ch = synth.ci_vectors(p.ndet, 1, np.random.default_rng(10))[:, 0]
    c = _dev(torch, ch)
    a1, a2 = pl.rdm(c, c)
    pl.rdm_fixed_point = True
    f1, f2 = pl.rdm(c, c)
    g1, g2 = pl.rdm(c, c)
    torch.cuda.synchronize()
    assert torch.equal(f1, g1) and torch.equal(f2, g2)
    x1, x2 = f1.cpu().numpy(), f2.cpu().numpy()
    assert _rel(x1, a1.cpu().numpy()) <= TOL and _rel(x2, a2.cpu().numpy()) <= TOL
    N = 20
    assert abs(np.trace(x1) - N) < 1e-11
    assert abs(np.einsum("pprr->", x2) - N * (N - 1)) < 1e-9
    e_sigma = float(np.dot(ch, pl.sigma(c).cpu().numpy()))
    e_rdm = float(np.sum(p.h * x1) + 0.5 * np.sum(p.g * x2))
    _say("[rdm-fixed] n64 E sigma", e_sigma, "E rdm", e_rdm)
    assert abs(e_sigma - e_rdm) <= 1e-12 * abs(e_sigma)
