"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the
paper's worked example, closed forms, dense linear algebra (numpy), brute
force on tiny inputs or invariants the paper states.  None of these call the
HIP library.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_graph(n, extra, seed, wlo=0.1, whi=1.0):
    """Connected random graph: a random spanning tree plus extra random edges."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    eu = [perm[i] for i in range(1, n)]
    ev = [perm[rng.integers(0, i)] for i in range(1, n)]
    a = rng.integers(0, n, extra)
    b = rng.integers(0, n, extra)
    keep = a != b
    eu = np.concatenate([eu, a[keep]]).astype(np.int32)
    ev = np.concatenate([ev, b[keep]]).astype(np.int32)
    w = rng.uniform(wlo, whi, eu.shape[0])
    return eu, ev, w


def dense_from_coo(n, eu, ev, w):
    A = np.zeros((n, n))
    for u, v, x in zip(eu, ev, w):
        A[u, v] -= x
        A[v, u] -= x
        A[u, u] += x
        A[v, v] += x
    return A


# ----------------------------------------------------------------- Laplacian
def test_five_node_example(ora):
    """Section 1, Fig. simple_graph: the printed 5x5 Laplacian, exactly."""
    d = json.load(open(os.path.join(GOLDEN, "five_node_laplacian.json")))
    e = np.array(d["edges_1based"])
    A = ora.laplacian(5, e[:, 0].astype(int) - 1, e[:, 1].astype(int) - 1, e[:, 2])
    assert np.array_equal(A.dense(), np.array(d["laplacian"], float))
    m = e.shape[0]
    assert A.col.shape[0] + A.n == 2 * m + 5 == 17  # 2m + n non-zeros
    # spectrum derived by hand: {0, 7 -/+ 2 sqrt 6, 4 -/+ sqrt 3}
    ev = np.linalg.eigvalsh(A.dense())
    want = sorted([0, 7 - 2 * math.sqrt(6), 4 - math.sqrt(3), 4 + math.sqrt(3), 7 + 2 * math.sqrt(6)])
    assert np.allclose(ev, want, atol=1e-13)


def test_laplacian_invariants_and_energy(ora):
    """Zero row sums, symmetry, 1 in the null space, energy identity (eq. energy)."""
    for seed in range(5):
        n = 40 + 7 * seed
        eu, ev, w = random_graph(n, 3 * n, seed)
        A = ora.laplacian(n, eu, ev, w)
        D = A.dense()
        assert np.allclose(D, D.T, atol=0)
        assert np.abs(D.sum(axis=1)).max() < 1e-13
        assert np.allclose(D, dense_from_coo(n, eu, ev, w), atol=1e-13)
        x = np.random.default_rng(seed).standard_normal(n)
        # duplicates are summed, so the energy uses the merged weights
        lhs = x @ D @ x
        rhs = sum(wi * (x[u] - x[v]) ** 2 for u, v, wi in zip(eu, ev, w))
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
        assert np.linalg.matrix_rank(D) == n - 1  # connected: null space span(1)


def test_duplicates_summed_and_input_rejected(ora):
    """Section 5.1: both directions of a pair are summed.  Invalid input is refused."""
    A = ora.laplacian(3, [0, 1, 1, 2], [1, 0, 2, 1], [1.0, 2.0, 0.5, 0.25])
    assert np.array_equal(A.dense(), np.array([[3, -3, 0], [-3, 3.75, -0.75], [0, -0.75, 0.75]]))
    assert ora.laplacian_status(3, [0], [0], [1.0]) == 1       # self-loop
    assert ora.laplacian_status(3, [0], [3], [1.0]) == 1       # out of range
    assert ora.laplacian_status(3, [0], [1], [0.0]) == 2       # w <= 0
    assert ora.laplacian_status(3, [0], [1], [np.nan]) == 2    # NaN weight
    A = ora.laplacian(4, [0, 2], [1, 3], [1.0, 1.0])
    assert not ora.connected(A)


# ------------------------------------------------------------ shared pieces
def test_splitmix64_reference_vector(ora):
    """splitmix64 (Steele, Lea & Flood 2014) from state 0: first output 0xE220A8397B1DCDAF.
    hash5 chains the finaliser; h(0,...) starts from sm64(0)."""
    # sm64(0) is the first output of the published generator seeded with 0
    def sm64(x):
        M = (1 << 64) - 1
        z = (x + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)
    assert sm64(0) == 0xE220A8397B1DCDAF
    h = sm64(0)
    for v in (1, 2, 3, 4):
        h = sm64(h ^ v)
    assert ora.hash5(0, 1, 2, 3, 4) == h
    u = ora.unit_pm1(ora.hash5(5, 3, 0, 0, 0))
    assert -1.0 <= u < 1.0
    assert ora.unit_pm1(0) == -1.0 and ora.unit_pm1((1 << 64) - 1) == 1.0 - 2.0 ** -52


def test_row_reduce_order(ora):
    """Row sums: exact for integer-valued terms, within the summation error
    bound otherwise; short rows sum left to right."""
    rng = np.random.default_rng(0)
    for n in (1, 5, 64, 65, 130, 1000, 4097):
        t = rng.integers(-1000, 1000, n).astype(float)
        assert ora.row_reduce(t) == float(t.sum())
        t = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        s = ora.row_reduce(t)
        assert abs(s - math.fsum(t)) <= (n + 8) * 2.0 ** -53 * np.abs(t).sum()
        if n <= 64:
            acc = 0.0
            for v in t:
                acc += v
            assert s == acc


# ----------------------------------------------------------------- colouring
def test_colouring_proper_and_jp_equal(ora):
    for seed in range(4):
        n = 200
        eu, ev, w = random_graph(n, 4 * n, seed)
        A = ora.laplacian(n, eu, ev, w)
        c = ora.colour(A, seed=seed, level=seed)
        rows = np.repeat(np.arange(n), np.diff(A.ptr))
        assert np.all(c[rows] != c[A.col])               # proper
        assert c.max() + 1 <= np.diff(A.ptr).max() + 1   # <= maxdeg + 1
        cj, rounds = ora.colour_jp(A, seed=seed, level=seed)
        assert np.array_equal(c, cj)                     # JP rounds == sequential
        assert rounds >= c.max() + 1


def test_colouring_first_fit_in_priority_order(ora):
    """Brute force: every node has the smallest colour unused by its
    higher-priority neighbours (degree desc, hash asc, id asc)."""
    n = 120
    eu, ev, w = random_graph(n, 3 * n, 11)
    A = ora.laplacian(n, eu, ev, w)
    seed, level = 9, 2
    c = ora.colour(A, seed=seed, level=level)
    deg = np.diff(A.ptr)
    h = [ora.hash5(seed, 7, level, 0, u) for u in range(n)]
    key = lambda u: (-deg[u], h[u], u)
    for u in range(n):
        nb = A.col[A.ptr[u]:A.ptr[u + 1]]
        used = {c[v] for v in nb if key(v) < key(u)}
        k = 0
        while k in used:
            k += 1
        assert c[u] == k


# -------------------------------------------------------------- Gauss-Seidel
def test_gs_lexicographic_is_triangular_solve(ora):
    """One sweep of eq. gs equals (D - N_L)^-1 (b + N_U x) by a dense triangular solve."""
    import scipy.linalg as sl
    for seed in range(3):
        n = 60
        eu, ev, w = random_graph(n, 3 * n, seed)
        A = ora.laplacian(n, eu, ev, w)
        D = A.dense()
        rng = np.random.default_rng(seed)
        b = rng.standard_normal(n)
        b -= b.mean()
        x = rng.standard_normal(n)
        x1 = ora.gs(A, b, x)
        lower = np.tril(D)
        upper = -np.triu(D, 1)
        want = sl.solve_triangular(lower, b + upper @ x, lower=True)
        assert np.allclose(x1, want, rtol=1e-12, atol=1e-12)


def test_gs_energy_never_increases(ora):
    """GS is exact coordinate minimisation of eq. quad: E_tot never increases."""
    n = 300
    eu, ev, w = random_graph(n, 5 * n, 3)
    A = ora.laplacian(n, eu, ev, w)
    D = A.dense()
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    b -= b.mean()
    x = rng.standard_normal(n)
    E = lambda v: 0.5 * v @ D @ v - v @ b
    prev = E(x)
    for _ in range(20):
        x = ora.gs(A, b, x)
        e = E(x)
        assert e <= prev + 1e-12 * abs(prev)
        prev = e


def test_multicolour_equals_lexicographic_on_permuted(ora):
    n = 150
    eu, ev, w = random_graph(n, 4 * n, 5)
    A = ora.laplacian(n, eu, ev, w)
    c = ora.colour(A, seed=1)
    perm = np.lexsort((np.arange(n), c))  # colour-major, then id
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n)
    x = rng.standard_normal(n)
    xm = ora.gs_multicolour(A, c, b, x)
    Ap = ora.laplacian(n, inv[eu], inv[ev], w)
    xp = ora.gs(Ap, b[perm], x[perm])
    assert np.allclose(xm[perm], xp, rtol=1e-13, atol=1e-13)


def test_residual_matches_dense(ora):
    n = 80
    eu, ev, w = random_graph(n, 3 * n, 8)
    A = ora.laplacian(n, eu, ev, w)
    rng = np.random.default_rng(1)
    b, x = rng.standard_normal(n), rng.standard_normal(n)
    assert np.allclose(ora.residual(A, b, x), b - A.dense() @ x, atol=1e-12)


# --------------------------------------------------------------- elimination
def test_elimination_schur_complement(ora):
    """Section 3.2, eq. elim: F independent with degree <= 4; A^c equals the
    dense Schur complement A_CC - A_CF A_FF^-1 A_FC and is a Laplacian;
    eliminate + back-substitute equals pinv(A) b."""
    for seed in range(4):
        n = 90
        eu, ev, w = random_graph(n, n // 2, seed)
        A = ora.laplacian(n, eu, ev, w)
        inF = ora.elim_select(A, 4).astype(bool)
        deg = np.diff(A.ptr)
        rows = np.repeat(np.arange(n), deg)
        assert inF.sum() > 0
        assert np.all(deg[inF] <= 4)
        assert not np.any(inF[rows] & inF[A.col])  # independent
        # greedy maximality: every eligible non-F node has an F neighbour
        for u in np.where(~inF & (deg <= 4))[0]:
            assert inF[A.col[A.ptr[u]:A.ptr[u + 1]]].any()
        Ac, crank = ora.schur(A, inF)
        D = A.dense()
        F, Cn = np.where(inF)[0], np.where(~inF)[0]
        S = D[np.ix_(Cn, Cn)] - D[np.ix_(Cn, F)] @ np.linalg.solve(D[np.ix_(F, F)], D[np.ix_(F, Cn)])
        assert np.allclose(Ac.dense(), S, atol=1e-12)
        assert np.array_equal(crank[Cn], np.arange(Cn.shape[0]))
        assert np.abs(Ac.dense().sum(axis=1)).max() < 1e-12
        # exact elimination solve
        b = np.random.default_rng(seed).standard_normal(n)
        b -= b.mean()
        P = np.zeros((n, Cn.shape[0]))
        P[Cn, np.arange(Cn.shape[0])] = 1
        P[np.ix_(F, np.arange(Cn.shape[0]))] = -np.linalg.solve(D[np.ix_(F, F)], D[np.ix_(F, Cn)])
        assert np.allclose(P.sum(axis=1), 1, atol=1e-13)  # P 1 = 1
        xc = np.linalg.pinv(S) @ (P.T @ b)
        x = P @ xc
        x[F] += b[F] / np.diag(D)[F]
        xs = np.linalg.pinv(D) @ b
        assert np.allclose(x - x.mean(), xs, atol=1e-10)


# ----------------------------------------------------------------- Galerkin
def test_galerkin_equals_dense(ora):
    for seed in range(3):
        n = 70
        eu, ev, w = random_graph(n, 2 * n, seed)
        A = ora.laplacian(n, eu, ev, w)
        rng = np.random.default_rng(seed)
        nc = 20
        agg = np.concatenate([np.arange(nc), rng.integers(0, nc, n - nc)]).astype(np.int32)
        rng.shuffle(agg)
        Ac = ora.galerkin(A, agg, nc)
        P = np.zeros((n, nc))
        P[np.arange(n), agg] = 1
        assert np.allclose(Ac.dense(), P.T @ A.dense() @ P, atol=1e-13)
        rows = np.repeat(np.arange(n), np.diff(A.ptr))
        cut = A.val[agg[rows] != agg[A.col]].sum()
        assert abs(Ac.val.sum() - cut) < 1e-12 * cut  # inter-aggregate weight conserved


def test_path_energy_inflation(ora):
    """Section 3.4.3, eq. q: pairwise aggregation of a path and a linear error
    gives q = E(P T e)/E(e) = (2n-4)/(n-1) (n=10: 16/9), approaching 2."""
    for n in (10, 20, 100):
        eu = np.arange(n - 1)
        ev = eu + 1
        A = ora.laplacian(n, eu, ev, np.ones(n - 1))
        agg = (np.arange(n) // 2).astype(np.int32)
        Ac = ora.galerkin(A, agg, n // 2)
        e = np.arange(n, dtype=float)
        Te = np.array([e[agg == U].mean() for U in range(n // 2)])
        q = (Te @ Ac.dense() @ Te) / (e @ A.dense() @ e)
        assert abs(q - (2 * n - 4) / (n - 1)) < 1e-13
    mu_opt = lambda Q: 2 * Q / (Q + 1)  # eq. optimal_mu
    Q = 2.0
    assert mu_opt(Q) == 4 / 3
    # ACF of the smoothest error with mu_opt: max(|1-mu|, |1-mu/Q|) = 1/3
    assert abs(max(abs(1 - mu_opt(Q)), abs(1 - mu_opt(Q) / Q)) - 1 / 3) < 1e-15
