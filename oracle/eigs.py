"""Lowest eigenpairs of a graph Laplacian -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never imports it.

What is computed (Section 6.4, the eigensolver: the K lowest eigenpairs of
A): for a connected graph the null space of the Laplacian is spanned by the
constant vector (Section 1), so the eigensolver's result is the k smallest
eigenvalues of A on the zero-sum subspace and an orthonormal basis of their
eigenvectors.  That result has a plain definition, written out here: the
Laplacian as a dense matrix from the weighted edge list (Section 1: a_uv =
-w_uv off the diagonal, a_uu = sum of the weights at u, duplicate pairs
summed), its full symmetric eigendecomposition (a library primitive,
numpy.linalg.eigh), and the eigenpairs after the single zero eigenvalue.
Pinned in the CPU tests by closed-form spectra (paths, grids, cycles,
complete graphs and stars) and the path's cosine eigenvectors.
"""
from __future__ import annotations

import numpy as np


def dense_laplacian(n: int, eu, ev, w) -> np.ndarray:
    """Dense FP64 Laplacian of a weighted undirected edge list."""
    a = np.zeros((n, n), np.float64)
    for u, v, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w, np.float64).tolist()):
        if u == v:
            continue
        a[u, v] -= x
        a[v, u] -= x
        a[u, u] += x
        a[v, v] += x
    return a


def lowest_eigenpairs(a: np.ndarray, k: int):
    """The k smallest eigenvalues of a connected graph's Laplacian on the
    zero-sum subspace and their orthonormal eigenvectors ([n, k]).  Also
    returns the next eigenvalue (for the gap test of the comparison)."""
    lam, vec = np.linalg.eigh(a)
    scale = max(1.0, float(np.abs(np.diag(a)).max()))
    if abs(lam[0]) > 1e-9 * scale or (a.shape[0] > 1 and lam[1] <= 1e-9 * scale):
        raise ValueError("not the Laplacian of a connected graph")
    nxt = float(lam[k + 1]) if k + 1 < a.shape[0] else float("inf")
    return lam[1:k + 1].copy(), vec[:, 1:k + 1].copy(), nxt
