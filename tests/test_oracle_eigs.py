"""CPU pins of the eigenpair oracle (Section 6.4) against closed-form spectra."""
import math

import numpy as np
import pytest

from oracle import eigs as E


def path(m):
    return m, np.arange(m - 1), np.arange(1, m), np.ones(m - 1)


def grid(a, b):
    eu, ev = [], []
    for j in range(b):
        for i in range(a):
            u = i + a * j
            if i + 1 < a:
                eu.append(u); ev.append(u + 1)
            if j + 1 < b:
                eu.append(u); ev.append(u + a)
    return a * b, np.array(eu), np.array(ev), np.ones(len(eu))


def path_spectrum(m):
    return np.array([2 - 2 * math.cos(math.pi * j / m) for j in range(m)])


def test_path_eigenvalues_and_vectors():
    m, k = 30, 5
    lam, vec, nxt = E.lowest_eigenpairs(E.dense_laplacian(*path(m)), k)
    ref = path_spectrum(m)
    assert np.allclose(lam, ref[1:k + 1], rtol=1e-12, atol=1e-14)
    assert nxt == pytest.approx(ref[k + 1], rel=1e-12)
    # eigenvector j of the path: cos(pi j (u + 1/2) / m)
    u = np.arange(m) + 0.5
    for j in range(1, k + 1):
        c = np.cos(math.pi * j * u / m)
        c /= np.linalg.norm(c)
        assert abs(float(c @ vec[:, j - 1])) == pytest.approx(1.0, abs=1e-12)
    assert np.allclose(vec.T @ vec, np.eye(k), atol=1e-12)
    assert np.allclose(vec.sum(axis=0), 0, atol=1e-12)


def test_grid_spectrum_is_sum_of_paths():
    a, b, k = 9, 6, 8
    lam, _, _ = E.lowest_eigenpairs(E.dense_laplacian(*grid(a, b)), k)
    pa, pb = path_spectrum(a), path_spectrum(b)
    ref = np.sort((pa[:, None] + pb[None, :]).ravel())
    assert np.allclose(lam, ref[1:k + 1], rtol=1e-12, atol=1e-13)


def test_cycle_complete_and_star():
    n = 16
    eu = np.arange(n); ev = (eu + 1) % n
    lam, _, _ = E.lowest_eigenpairs(E.dense_laplacian(n, eu, ev, np.ones(n)), 4)
    ref = np.sort([2 - 2 * math.cos(2 * math.pi * j / n) for j in range(n)])
    assert np.allclose(lam, ref[1:5], rtol=1e-12)
    iu, iv = np.triu_indices(7, 1)
    lam, _, _ = E.lowest_eigenpairs(E.dense_laplacian(7, iu, iv, np.full(iu.size, 0.5)), 3)
    assert np.allclose(lam, 3.5, rtol=1e-12)  # K_n with weight w: n w, multiplicity n - 1
    s = 6
    lam, _, nxt = E.lowest_eigenpairs(E.dense_laplacian(s + 1, np.zeros(s, int), np.arange(1, s + 1), np.ones(s)), s - 1)
    assert np.allclose(lam, 1.0, rtol=1e-12) and nxt == pytest.approx(s + 1, rel=1e-12)


def test_weights_scale_and_duplicates_sum():
    n, eu, ev, w = path(12)
    base, _, _ = E.lowest_eigenpairs(E.dense_laplacian(n, eu, ev, w), 3)
    dup, _, _ = E.lowest_eigenpairs(E.dense_laplacian(n, np.r_[eu, ev], np.r_[ev, eu], np.r_[w, 2 * w]), 3)
    assert np.allclose(dup, 3 * base, rtol=1e-12)


def test_disconnected_rejected():
    with pytest.raises(ValueError):
        E.lowest_eigenpairs(E.dense_laplacian(4, [0, 2], [1, 3], [1.0, 1.0]), 1)
