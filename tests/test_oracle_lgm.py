"""Pins of the oracle's lean geometric multigrid (Section 5.3): the periodic
Poisson grid, its red-black order, the closed form of the 2 x 2 Galerkin
operators, the transfer maps, and the published efficiency of the cycle
(a convergence factor of about 0.5 per unit of work), mesh-independent."""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module")
def lgm64():
    return O.Hierarchy.lgm(64)


def _natural(L, side):
    """The level's CSR in natural grid order (undo the colour order)."""
    n = side * side
    A = np.zeros((n, n))
    p = L.perm
    for u in range(n):
        for t in range(L.A.ptr[u], L.A.ptr[u + 1]):
            A[p[u], p[L.A.col[t]]] = -L.A.val[t]
        A[p[u], p[u]] = L.A.diag[u]
    return A


def periodic_laplacian(side, w=1.0):
    n = side * side
    A = np.zeros((n, n))
    for j in range(side):
        for i in range(side):
            u = i + side * j
            for v in ((i + 1) % side + side * j, i + side * ((j + 1) % side)):
                A[u, v] -= w
                A[v, u] -= w
                A[u, u] += w
                A[v, v] += w
    return A


def test_levels_red_black_and_galerkin_closed_form(lgm64):
    H = lgm64
    sides = [64, 32, 16, 8]
    assert H.num_levels == 4
    for l, sd in enumerate(sides):
        L = H.level(l)
        n = sd * sd
        assert L.A.n == n and L.ncol == 2 and list(L.cptr) == [0, n // 2, n]
        # red first, then black; each class an independent set
        for k, (a, z) in enumerate(((0, n // 2), (n // 2, n))):
            for u in range(a, z):
                p = int(L.perm[u])
                assert ((p % sd) + (p // sd)) % 2 == k
                assert all(not (a <= L.A.col[t] < z) for t in range(L.A.ptr[u], L.A.ptr[u + 1]))
        # level l = 2^l x (periodic 5-point Laplacian of the level's grid):
        # two fine edges cross each side of a 2 x 2 block
        assert np.array_equal(_natural(L, sd), periodic_laplacian(sd, float(2 ** l)))
    for l in range(3):
        assert H.dims(l)["gamma"] == 1.5


def test_transfer_maps_are_2x2_blocks(lgm64):
    H = lgm64
    for l, sd in enumerate([64, 32, 16]):
        F, C = H.level(l), H.level(l + 1)
        agg = C.transfer  # fine level order -> coarse level order
        sc = sd // 2
        for u in range(F.A.n):
            p = int(F.perm[u])
            q = int(C.perm[agg[u]])
            assert q == (p % sd) // 2 + sc * ((p // sd) // 2)


def _efficiency(H, side):
    """ACF of a solve and the work of one cycle in finest relaxation sweeps:
    (nu_pre + nu_post) x sum over relaxed levels of visits x n_l / n_0."""
    rng = np.random.default_rng(side)
    b = rng.standard_normal(side * side)
    x, info, hist = H.solve(b)
    visits = H.visit_counts()
    n0 = side * side
    W = sum(3 * visits[l] * H.dims(l)["n"] / n0 for l in range(H.num_levels - 1))
    return info["acf"], W, info


def test_published_efficiency_and_mesh_independence():
    """Section 5.3: about 0.5 per unit of work (read with the unit = one
    finest-level relaxation sweep), the same at every grid size."""
    acfs = []
    for side in (64, 128, 256):
        H = O.Hierarchy.lgm(side)
        acf, W, info = _efficiency(H, side)
        assert info["cycles"] <= 8 and info["rel_residual"] <= 1e-8
        eff = acf ** (1.0 / W)
        assert 0.42 <= eff <= 0.55, (side, acf, W, eff)
        acfs.append(acf)
    assert max(acfs) / min(acfs) < 1.05, acfs


def test_flat_mu_is_two_and_solution_exact():
    """The cycle solves the periodic problem: the zero-mean solution against
    the dense pseudo-inverse (side 16)."""
    side = 16
    H = O.Hierarchy.lgm(side)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(side * side)
    x, info, _ = H.solve(b)
    A = periodic_laplacian(side)
    xr = np.linalg.pinv(A) @ (b - b.mean())
    assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr)
    assert abs(info["removed_mean"] - b.mean()) <= 1e-15
