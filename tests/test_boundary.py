"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and its host-side validation turns malformed problems into status
codes before any device work.  Plan statistics equal the oracle's counts."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2501_18185_amd import mw, synth
from oracle import sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mw.h")).read()
    names = set(re.findall(r"\b(mw_[a-z0-9_]+)\s*\(", hdr))
    names.discard("mw_status")
    assert len(names) >= 15
    L = mw.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    out = os.popen(f"nm -D --defined-only {mw.LIB_PATH}").read()
    exported = set(re.findall(r" T (mw_[a-z0-9_]+)", out))
    assert exported == names, (exported - names, names - exported)


def _problem(**kw):
    p = synth.workload(0)
    d = dict(kind=p.kind, norb=p.norb, nalpha=p.nalpha, nbeta=p.nbeta, dets=p.dets, h=p.h, g=p.g, ecore=0.0)
    d.update(kw)
    return synth.Problem(d["kind"], d["norb"], d["nalpha"], d["nbeta"], d["dets"], d["h"], d["g"], d["ecore"])


def _status(prob, max_roots=1):
    try:
        mw.Plan(prob, max_roots=max_roots, upload=False)
    except mw.MWError as e:
        return e.status
    return 0


def test_validation_status_codes():
    p = synth.workload(0)
    assert _status(_problem()) == 0
    assert _status(_problem(dets=p.dets[::-1].copy())) == -2            # not ascending
    dup = np.concatenate([p.dets[:1], p.dets[:-1]])
    assert _status(_problem(dets=dup)) == -2                             # duplicate
    bad = p.dets.copy(); bad[5, 0] ^= np.uint64(1 << 7) | np.uint64(1)   # wrong popcount
    assert _status(_problem(dets=np.sort(bad.view("u8,u8"), axis=0).view(np.uint64).reshape(-1, 2))) in (-2, -3)
    beyond = p.dets.copy(); beyond[-1, 1] = np.uint64(0xF << 8)           # bits beyond norb
    assert _status(_problem(dets=beyond)) == -3
    h = p.h.copy(); h[0, 1] += 1e-6
    assert _status(_problem(h=h)) == -4                                  # h not symmetric
    g = p.g.copy(); g[0, 1, 2, 3] += 1e-6
    assert _status(_problem(g=g)) == -4                                  # g not 8-fold
    assert _status(_problem(norb=65)) == -8
    assert _status(_problem(), max_roots=0) == -1
    assert _status(_problem(kind="spinor")) in (-1, -4)                 # nbeta must be -1


def test_sigma_without_workspace_is_an_error():
    pl = mw.Plan(synth.workload(0), upload=False)
    st = mw.lib().mw_sigma(pl._plan, 1, C.c_void_p(16), C.c_void_p(32), None)
    assert st == -5


@pytest.mark.parametrize("k", [0, 4])
def test_plan_pair_counts_equal_oracle(k):
    p = synth.workload(k)
    pl = mw.Plan(p, upload=False)
    deg = sc.degree_rows(p)
    assert pl.info("pairs") == deg.sum()
    rec = sc.connect_rows(p, np.arange(0, p.ndet, 3))
    assert pl.info("single_pairs") + pl.info("double_pairs") == pl.info("pairs")
    assert pl.info("evaluations") >= pl.info("pairs")


def test_plan_pair_counts_spinor():
    rng = np.random.default_rng(1)
    d = synth.space_selected_spinor(8, 6, 2000, rng)
    p = synth.Problem("spinor", 8, 6, -1, d, synth.one_body_spinor(8, rng), synth.two_body_spinor(8, rng))
    pl = mw.Plan(p, upload=False)
    assert pl.info("pairs") == sc.degree_rows(p).sum()


def test_csf_host_counts_and_errors():
    """mw_csf_create on the host: CSF and configuration counts equal the
    oracle's expansion; 2S, spinor plans and incomplete configurations are
    refused with status codes; transforms need an uploaded basis."""
    from oracle import csf
    n, na, nb = 6, 4, 2
    rng = np.random.default_rng(3)
    d = synth.space_fci(n, na, nb)
    p = synth.Problem("spinfree", n, na, nb, d, synth.one_body_real(n, rng), synth.two_body_real(n, rng))
    pl = mw.Plan(p, upload=False)
    cb = mw.Csf(pl, 2, upload=False)
    T, first = csf.expansion(p, 2)
    assert cb.ncsf == T.shape[1] and cb.info("configurations") == len(first) - 1
    assert cb.info("max_open") == 6 and cb.info("ndet") == len(d)
    h = C.c_void_p()
    assert mw.lib().mw_csf_create(pl._plan, 0, C.byref(h)) == -1          # 2S != Na - Nb
    assert mw.lib().mw_csf_to_det(cb._csf, 1, C.c_void_p(16), C.c_void_p(32), None) == -5
    # one determinant of a configuration with four open shells (four
    # determinants at S = 1) missing
    k = np.bitwise_count(d[:, 0] ^ d[:, 1])
    q = synth.Problem("spinfree", n, na, nb, np.delete(d, int(np.nonzero(k == 4)[0][0]), axis=0), p.h, p.g)
    assert mw.lib().mw_csf_create(mw.Plan(q, upload=False)._plan, 2, C.byref(h)) == -1
    sp = synth.workload(0)
    nk = 3
    rs = np.random.default_rng(4)
    pos = np.array([[0, 1, 4], [0, 2, 5]], np.int64)
    ds = synth.sort_unique(*synth._words(pos, nk))
    ps = synth.Problem("spinor", nk, 3, -1, ds, synth.one_body_spinor(nk, rs), synth.two_body_spinor(nk, rs))
    assert mw.lib().mw_csf_create(mw.Plan(ps, upload=False)._plan, 1, C.byref(h)) == -8
    del sp


def test_ivi_needs_uploaded_plan():
    """mw_ivi and its work size refuse a plan without a workspace."""
    pl = mw.Plan(synth.workload(0), upload=False)
    nb = C.c_size_t()
    assert mw.lib().mw_ivi_work_bytes(pl._plan, 1, C.byref(nb)) == -5
    ev = (C.c_double * 1)()
    it = C.c_int32()
    assert mw.lib().mw_ivi(pl._plan, 1, float("nan"), C.c_void_p(16), C.c_void_p(32), ev, 1e-8, 10, C.byref(it),
                           C.c_void_p(256), 1 << 20, None) == -5


def test_tuning_code_round_trip():
    """The sigma launch parameters are read and restored as one code
    (unroll * 100 + lanes) on the host; invalid codes are refused."""
    from paper_2501_18185_amd import mw
    pl = mw.Plan(synth.workload(0), upload=False)
    assert pl.tuning == 416  # defaults: unroll 4, 16 gather lanes (real)
    for code in (408, 816, 1632):
        pl.tuning = code
        assert pl.tuning == code
    for bad in (0, 316, 412, 1664, 2016):
        with pytest.raises(mw.MWError):
            pl.tuning = bad
    assert pl.tuning == 1632
    q = mw.Plan(synth.workload(0), upload=False)
    q.tuning = pl.tuning  # a saved choice restored on another plan
    assert q.tuning == 1632


def test_tuning_cache_file(tmp_path):
    """A tuned code stored in a cache file under (architecture, shape) is
    applied to a plan of the same shape and not to another shape."""
    from paper_2501_18185_amd import mw
    cache = str(tmp_path / "tuning.json")
    a = mw.Plan(synth.workload(0), upload=False)
    assert not a.load_tuning(cache, 1, "gfx950")
    a.tuning = 832
    a.save_tuning(cache, 1, "gfx950")
    b = mw.Plan(synth.workload(0), upload=False)
    assert b.load_tuning(cache, 1, "gfx950") and b.tuning == 832
    assert not b.load_tuning(cache, 2, "gfx950")   # other root count
    assert not b.load_tuning(cache, 1, "gfx942")   # other architecture
    other = mw.Plan(synth.workload(4), upload=False)
    assert not other.load_tuning(cache, 1, "gfx950")


def test_rdm_mode_is_host_state_with_status_codes():
    """mw_plan_set_rdm_mode: 0 and 1 accepted (read back as statistic 18),
    anything else MW_EINVAL, a NULL plan MW_EINVAL; no device needed."""
    pl = mw.Plan(synth.workload(0), upload=False)
    assert pl.info("rdm_fixed") == 0 and not pl.rdm_fixed_point
    pl.rdm_fixed_point = True
    assert pl.info("rdm_fixed") == 1 and pl.rdm_fixed_point
    assert mw.lib().mw_plan_set_rdm_mode(pl._plan, 2) == -1
    assert mw.lib().mw_plan_set_rdm_mode(None, 1) == -1
    assert pl.info("rdm_fixed") == 1
    pl.rdm_fixed_point = False
    assert pl.info("rdm_fixed") == 0
