"""Plans grouped on the device (mw_plan_create_device) against the host build.

Bar: every index array of the plan (groups, memberships, packets, column
partials, slot lists and placement, density rows) byte-identical to the host
build's, the plan statistics equal, and sigma bitwise equal on the same
vector; the density matrices (device atomics, arrival order) within 1e-12.
Spaces: FCI, selected spin-free spaces with groups of 64 members or more,
a spinor space, spaces without any group, one electron, and the
2,000,000-determinant n=64 space at full size.
"""
import sys
import time

import numpy as np
import pytest

from paper_2501_18185_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _prob(kind, n, na, nb, dets, h, g, ecore=0.0):
    return synth.Problem(kind, n, na, nb, np.ascontiguousarray(dets, np.uint64), h, g, ecore)


def _real(n, rng):
    return synth.one_body_real(n, rng), synth.two_body_real(n, rng)


def _spaces():
    out = []
    out.append(("fci-n8", synth.workload(0)))
    rng = np.random.default_rng(11)
    d = synth.space_selected_spinfree(24, 5, 5, 30000, rng)
    out.append(("sci-n24", _prob("spinfree", 24, 5, 5, d, *_real(24, rng))))
    rng = np.random.default_rng(12)
    d = synth.space_selected_spinfree(40, 6, 4, 60000, rng)
    out.append(("sci-n40-6a4b", _prob("spinfree", 40, 6, 4, d, *_real(40, rng))))
    rng = np.random.default_rng(13)
    d = synth.space_selected_spinor(12, 6, 4000, rng)
    out.append(("spinor-12", _prob("spinor", 12, 6, -1, d, synth.one_body_spinor(12, rng),
                                   synth.two_body_spinor(12, rng))))
    rng = np.random.default_rng(14)
    out.append(("fci-n6-1a0b", _prob("spinfree", 6, 1, 0, synth.space_fci(6, 1, 0), *_real(6, rng))))
    rng = np.random.default_rng(15)
    out.append(("one-det", _prob("spinfree", 6, 2, 2, synth.space_fci(6, 2, 2)[:1], *_real(6, rng))))
    # determinants pairwise more than a double excitation apart: no group
    rng = np.random.default_rng(16)
    w = np.array([[0b000111, 0b000111], [0b111000, 0b111000]], dtype=np.uint64)
    out.append(("no-groups", _prob("spinfree", 6, 3, 3, w, *_real(6, rng))))
    return out


def _compare(torch, mw, name, prob, max_roots=1):
    t0 = time.perf_counter()
    ph = mw.Plan(prob, max_roots=max_roots, build="host")
    t1 = time.perf_counter()
    pd = mw.Plan(prob, max_roots=max_roots, build="device")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _say(f"[plan-device] {name}: ndet={prob.ndet} groups={ph.info('groups')} host {t1 - t0:.2f}s "
         f"device {t2 - t1:.2f}s")
    assert pd.info("built_on_device") == 1 and ph.info("built_on_device") == 0
    for what in mw.INFO:
        if what == "built_on_device":
            continue
        assert pd.info(what) == ph.info(what), (name, what, pd.info(what), ph.info(what))
    for arr in mw.PLAN_ARRAYS:
        a, b = pd.array(arr).cpu().numpy(), ph.array(arr).cpu().numpy()
        assert a.shape == b.shape, (name, arr, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            pytest.fail(f"{name}: {arr} differs at {bad.size} bytes, first at byte {bad[0]} of {a.size}")
    return ph, pd


def test_device_plan_equals_host_plan(torch):
    from paper_2501_18185_amd import mw
    for name, prob in _spaces():
        ph, pd = _compare(torch, mw, name, prob)
        rng = np.random.default_rng(3)
        c = synth.ci_vectors(prob.ndet, 1, rng, complex_=ph.is_complex)
        ct = torch.from_numpy(c).cuda()
        sh, sd = ph.sigma(ct), pd.sigma(ct)
        torch.cuda.synchronize()
        assert torch.equal(sh, sd), name
        if ph.info("memberships") > 0:
            gh, Gh = ph.rdm(ct, ct)
            gd, Gd = pd.rdm(ct, ct)
            for x, y in ((gh, gd), (Gh, Gd)):
                x, y = x.cpu().numpy(), y.cpu().numpy()
                assert np.abs(x - y).max() <= 1e-12 * max(np.abs(x).max(), 1.0), name
        _say(f"[plan-device] {name}: arrays, sigma and density matrices agree")


def test_device_plan_several_roots(torch):
    """The partial-sum placement depends on the root count (2 MB regions)."""
    from paper_2501_18185_amd import mw
    rng = np.random.default_rng(21)
    d = synth.space_selected_spinfree(24, 5, 5, 30000, rng)
    prob = _prob("spinfree", 24, 5, 5, d, *_real(24, rng))
    ph, pd = _compare(torch, mw, "sci-n24-R4", prob, max_roots=4)
    c = torch.from_numpy(synth.ci_vectors(prob.ndet, 4, np.random.default_rng(4))).cuda()
    assert torch.equal(ph.sigma(c), pd.sigma(c))


def test_device_plan_uploads_once(torch):
    from paper_2501_18185_amd import mw
    pd = mw.Plan(synth.workload(0), build="device")
    with pytest.raises(mw.MWError):
        pd.upload()


def test_device_plan_full_size(torch):
    """The 2,000,000-determinant n=64 10a10b space: the same arrays."""
    from paper_2501_18185_amd import mw
    prob = synth.workload(1)
    ph, pd = _compare(torch, mw, "sci-n64-2e6", prob)
    c = torch.from_numpy(synth.ci_vectors(prob.ndet, 1, np.random.default_rng(5))).cuda()
    assert torch.equal(ph.sigma(c), pd.sigma(c))


def test_device_plan_full_size_spinor(torch):
    """The 1,000,000-determinant 40-pair spinor space: the same arrays."""
    from paper_2501_18185_amd import mw
    prob = synth.workload(2)
    ph, pd = _compare(torch, mw, "spinor-40kp-1e6", prob)
    c = torch.from_numpy(synth.ci_vectors(prob.ndet, 1, np.random.default_rng(6), complex_=True)).cuda()
    assert torch.equal(ph.sigma(c), pd.sigma(c))
