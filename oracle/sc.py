"""ctypes front end of the tier-B Slater-Condon oracle (``sc.c``).

Test infrastructure only (see the package docstring).  Every function takes a
problem object with the attributes ``kind`` ("spinfree" | "spinor"),
``norb``, ``dets`` ([ndet][2] uint64), ``h``, ``g`` and ``ecore``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = C.CDLL(path)
        dp, lp, up = C.POINTER(C.c_double), C.POINTER(C.c_long), C.POINTER(C.c_uint64)
        L.orc_sigma_rows.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_long, up, C.c_int,
                                     dp, C.c_long, lp, dp]
        L.orc_hij_pairs.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, up, C.c_long, lp, dp]
        L.orc_degree_rows.argtypes = [C.c_int, C.c_long, up, C.c_long, lp, lp]
        L.orc_connect_rows.argtypes = [C.c_int, C.c_long, up, C.c_long, lp, lp]
        L.orc_connect_rows.restype = C.c_long
        L.orc_pair_counts.argtypes = [C.c_long, up, lp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_rdm_rows.argtypes = [C.c_int, C.c_int, C.c_long, up, C.c_int, dp, dp, dp, C.c_long,
                                   lp, dp, dp]
        L.orc_pt2.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_long, up, C.c_int, dp, dp,
                              C.c_double, dp, lp]
        L.orc_select.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_long, up, C.c_int, dp, dp,
                                 C.c_double, up, C.c_long]
        L.orc_select.restype = C.c_long
        _lib = L
    return _lib


def num_threads():
    """OpenMP threads the row loops use."""
    return int(lib().orc_num_threads())


def set_threads(n):
    """Threads for the row loops from now on."""
    lib().orc_set_threads(int(n))


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _ham(prob):
    kind = 0 if prob.kind == "spinfree" else 1
    if kind == 0:
        h = np.ascontiguousarray(np.real_if_close(prob.h), dtype=np.float64)
        g = np.ascontiguousarray(np.real_if_close(prob.g), dtype=np.float64)
    else:
        h = np.ascontiguousarray(prob.h, dtype=np.complex128).view(np.float64)
        g = np.ascontiguousarray(prob.g, dtype=np.complex128).view(np.float64)
    return kind, h, g


def _rows(rows, ndet):
    if rows is None:
        rows = np.arange(ndet)
    return np.ascontiguousarray(rows, dtype=np.int64)


def sigma(prob, c, rows=None):
    """sigma_I = sum_J H_IJ c_J for the requested rows (all by default).

    ``c`` is [ndet] or [ndet][nroots]; the result has the matching shape
    (restricted to ``rows``) and is complex for spinor problems or complex c.
    """
    kind, h, g = _ham(prob)
    c = np.asarray(c)
    vec = c.ndim == 1
    c2 = c.reshape(len(c), -1)
    nroots = c2.shape[1]
    cc = np.ascontiguousarray(c2, dtype=np.complex128)
    rows = _rows(rows, prob.ndet)
    out = np.zeros((len(rows), nroots), dtype=np.complex128)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    lib().orc_sigma_rows(kind, prob.norb, _p(h, C.c_double), _p(g, C.c_double), float(prob.ecore),
                         len(dets), _p(dets, C.c_uint64), nroots, _p(cc.view(np.float64), C.c_double),
                         len(rows), _p(rows, C.c_long), _p(out.view(np.float64), C.c_double))
    if kind == 0 and not np.iscomplexobj(c):
        assert not np.any(out.imag), "real problem produced an imaginary part"
        out = out.real.copy()
    return out[:, 0] if vec else out


def hij_pairs(prob, pairs):
    kind, h, g = _ham(prob)
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    out = np.zeros(len(pairs), dtype=np.complex128)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    lib().orc_hij_pairs(kind, prob.norb, _p(h, C.c_double), _p(g, C.c_double), float(prob.ecore),
                        _p(dets, C.c_uint64), len(pairs), _p(pairs, C.c_long),
                        _p(out.view(np.float64), C.c_double))
    return out.real.copy() if kind == 0 else out


def dense_h(prob):
    """Full H built from Slater-Condon elements (small spaces only)."""
    N = prob.ndet
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    v = hij_pairs(prob, np.stack([I.ravel(), J.ravel()], 1))
    return v.reshape(N, N)


def diag(prob):
    idx = np.arange(prob.ndet)
    return hij_pairs(prob, np.stack([idx, idx], 1))


def degree_rows(prob, rows=None):
    rows = _rows(rows, prob.ndet)
    out = np.zeros(len(rows), dtype=np.int64)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    lib().orc_degree_rows(prob.norb, len(dets), _p(dets, C.c_uint64), len(rows), _p(rows, C.c_long),
                          _p(out, C.c_long))
    return out


def pair_counts(prob):
    """Ordered connected pairs (I != J) of the whole space by excitation
    level: (singles, doubles).  Every pair of the space is visited."""
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    pc = np.vectorize(lambda x: bin(int(x)).count("1"), otypes=[np.int64])
    if len(dets):
        if prob.kind == "spinfree":
            na, nb = pc(dets[:, 0]), pc(dets[:, 1])
            if na.min() != na.max() or nb.min() != nb.max():
                raise ValueError("spin-free determinants must share N_alpha and N_beta")
        else:
            ne = pc(dets[:, 0]) + pc(dets[:, 1])
            if ne.min() != ne.max():
                raise ValueError("determinants must share the electron count")
    out = np.zeros(2, dtype=np.int64)
    lib().orc_pair_counts(len(dets), _p(dets, C.c_uint64), _p(out, C.c_long))
    return int(out[0]), int(out[1])


def connect_rows(prob, rows=None):
    """Connected pairs of the requested rows: int64 [npairs][7] with columns
    I, J, P, Q, R, S, sign (R = S = -1 for single excitations)."""
    rows = _rows(rows, prob.ndet)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    L = lib()
    nul = C.POINTER(C.c_long)()
    cnt = L.orc_connect_rows(prob.norb, len(dets), _p(dets, C.c_uint64), len(rows), _p(rows, C.c_long), nul)
    out = np.zeros((cnt, 7), dtype=np.int64)
    L.orc_connect_rows(prob.norb, len(dets), _p(dets, C.c_uint64), len(rows), _p(rows, C.c_long),
                       _p(out, C.c_long))
    return out


def rdm(prob, bra, ket, weights=None, rows=None):
    """Transition density matrices (gamma, Gamma) summed over the bra rows.

    Spin-free: spin-summed over spatial orbitals, gamma [n][n] and Gamma
    [n][n][n][n] with Gamma_pqrs pairing a+_p a+_r a_s a_q.  Spinor: over
    the M = 2n spinors.  bra, ket: [ndet] or [ndet][nroots]."""
    kind = 0 if prob.kind == "spinfree" else 1
    bra = np.asarray(bra); ket = np.asarray(ket)
    b2 = np.ascontiguousarray(bra.reshape(len(bra), -1), dtype=np.complex128)
    k2 = np.ascontiguousarray(ket.reshape(len(ket), -1), dtype=np.complex128)
    nroots = b2.shape[1]
    m = prob.norb if kind == 0 else 2 * prob.norb
    gam = np.zeros((m, m), dtype=np.complex128)
    Gam = np.zeros((m, m, m, m), dtype=np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    rows = _rows(rows, prob.ndet)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    lib().orc_rdm_rows(kind, prob.norb, len(dets), _p(dets, C.c_uint64), nroots,
                       _p(b2.view(np.float64), C.c_double), _p(k2.view(np.float64), C.c_double),
                       _p(w, C.c_double) if w is not None else C.POINTER(C.c_double)(),
                       len(rows), _p(rows, C.c_long),
                       _p(gam.view(np.float64), C.c_double), _p(Gam.view(np.float64), C.c_double))
    if kind == 0 and not (np.iscomplexobj(bra) or np.iscomplexobj(ket)):
        return gam.real.copy(), Gam.real.copy()
    return gam, Gam


def pt2(prob, c, e0, qmin=0.0):
    """Epstein-Nesbet second-order energies E2_k over the determinants that
    single and double excitations reach from the space (outside it), with
    the screening of section 2.5: (A, J) is left out when A's configuration
    is doubly excited from J's and Table 1's bound is below qmin / max|C|
    over J's configuration.  ``c`` [ndet] or
    [ndet][nroots], ``e0`` scalar or [nroots].  Returns (e2 [nroots],
    kept (A, J) pairs, number of external A)."""
    kind, h, g = _ham(prob)
    c = np.asarray(c)
    c2 = np.ascontiguousarray(c.reshape(len(c), -1), dtype=np.complex128)
    nroots = c2.shape[1]
    if nroots > 64:
        raise ValueError("at most 64 roots")
    e0 = np.ascontiguousarray(np.broadcast_to(np.asarray(e0, np.float64), (nroots,)))
    e2 = np.zeros(nroots)
    stats = np.zeros(2, dtype=np.int64)
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    lib().orc_pt2(kind, prob.norb, _p(h, C.c_double), _p(g, C.c_double), float(prob.ecore), len(dets),
                  _p(dets, C.c_uint64), nroots, _p(c2.view(np.float64), C.c_double), _p(e0, C.c_double),
                  float(qmin), _p(e2, C.c_double), _p(stats, C.c_long))
    return e2, int(stats[0]), int(stats[1])


def select(prob, c, e0, cmin):
    """Determinants outside the space selected by the iCIPT2 criterion of
    section 2.4 for some configuration J of the space (max over J's
    determinants and the roots of |H c| >= cmin and of |H c / (E0 - H_AA)|
    >= cmin; for a doubly excited configuration also Table 1's bound times
    max|C| >= cmin); sorted [nsel][2] uint64."""
    kind, h, g = _ham(prob)
    c = np.asarray(c)
    c2 = np.ascontiguousarray(c.reshape(len(c), -1), dtype=np.complex128)
    nroots = c2.shape[1]
    e0 = np.ascontiguousarray(np.broadcast_to(np.asarray(e0, np.float64), (nroots,)))
    dets = np.ascontiguousarray(prob.dets, dtype=np.uint64)
    args = (kind, prob.norb, _p(h, C.c_double), _p(g, C.c_double), float(prob.ecore), len(dets),
            _p(dets, C.c_uint64), nroots, _p(c2.view(np.float64), C.c_double), _p(e0, C.c_double), float(cmin))
    n = lib().orc_select(*args, C.POINTER(C.c_uint64)(), 0)
    out = np.zeros((max(n, 1), 2), dtype=np.uint64)
    lib().orc_select(*args, _p(out, C.c_uint64), n)
    return out[:n]
