"""Block Davidson-Liu for the lowest roots of H (oracle version).

Test infrastructure only (see the package docstring).  The paper diagonalises
through products sigma = H X that use only nonzero elements of H, recomputed
whenever needed (section 2.4, last paragraph); this is the standard
Davidson-Liu iteration over such products:

1. V = orthonormalised start vectors; W = H V.
2. G = V^H W; lowest ``nroots`` eigenpairs (theta_k, y_k) of G.
3. r_k = W y_k - theta_k V y_k; converged when every ||r_k||_2 <= tol.
4. t_k = r_k / (theta_k - H_II), each |denominator| clamped to >= 1e-12
   with its sign kept.
5. Two passes of Gram-Schmidt of t_k against V (and earlier t's); t_k is
   dropped when its norm falls below 1e-10.
6. When the subspace would exceed max(8 nroots, 24) vectors it collapses to
   the current Ritz vectors.
"""
from __future__ import annotations

import numpy as np


def diagonal_guess(diag, nroots):
    """Unit vectors on the nroots lowest diagonal elements (ties broken by
    index), the usual start for a diagonally dominant H."""
    diag = np.asarray(diag).real
    order = np.lexsort((np.arange(len(diag)), diag))[:nroots]
    c0 = np.zeros((len(diag), nroots))
    c0[order, np.arange(nroots)] = 1.0
    return c0


def _orthonormalize(V):
    Q, _ = np.linalg.qr(V)
    return Q


def davidson(sigma_fn, diag, c0, tol=1e-8, max_iter=100):
    c0 = np.asarray(c0)
    if c0.ndim == 1:
        c0 = c0[:, None]
    nroots = c0.shape[1]
    max_sub = max(8 * nroots, 24)
    V = _orthonormalize(c0)
    W = np.asarray(sigma_fn(V)).reshape(V.shape)
    diag = np.asarray(diag).real
    theta = None
    X = V
    for it in range(1, max_iter + 1):
        G = V.conj().T @ W
        G = 0.5 * (G + G.conj().T)
        evals, Y = np.linalg.eigh(G)
        theta = evals[:nroots]
        Yk = Y[:, :nroots]
        X = V @ Yk
        AX = W @ Yk
        R = AX - X * theta[None, :]
        rnorm = np.linalg.norm(R, axis=0)
        if np.all(rnorm <= tol):
            return theta, X, it, True
        T = []
        for k in range(nroots):
            if rnorm[k] <= tol:
                continue
            den = theta[k] - diag
            den = np.where(np.abs(den) < 1e-12, np.where(den < 0, -1e-12, 1e-12), den)
            t = R[:, k] / den
            T.append(t)
        if V.shape[1] + len(T) > max_sub:
            V, W = X, AX
        kept = []
        for t in T:
            for _ in range(2):
                t = t - V @ (V.conj().T @ t)
                for u in kept:
                    t = t - u * (u.conj() @ t)
            nt = np.linalg.norm(t)
            if nt < 1e-10:
                continue
            kept.append(t / nt)
        if not kept:
            return theta, X, it, False
        Tm = np.stack(kept, axis=1)
        V = np.concatenate([V, Tm], axis=1)
        W = np.concatenate([W, np.asarray(sigma_fn(Tm)).reshape(Tm.shape)], axis=1)
    return theta, X, max_iter, False
