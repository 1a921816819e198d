"""Lean geometric multigrid (Section 5.3) on the GPU against the oracle: the
hierarchy (red-black order, 2 x 2 Galerkin operators, transfer maps, cycle
indices) bit for bit, one cycle to rounding, solves in the oracle's cycle
count, and at 1024 x 1024 the published efficiency of about 0.5 per unit of
work."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _case(name):
    print(f"[case] {name}", flush=True)


@pytest.fixture(scope="module")
def lg():
    from paper_1108_1310_amd import lamg
    lamg.lib()
    return lamg


def periodic_edges(side):
    u = np.arange(side * side)
    i, j = u % side, u // side
    eu = np.concatenate([u, u]).astype(np.int32)
    ev = np.concatenate([(i + 1) % side + side * j, i + side * ((j + 1) % side)]).astype(np.int32)
    return eu, ev, np.ones(eu.shape[0])


@pytest.mark.parametrize("side", [4, 16, 64, 256])
def test_lgm_hierarchy_bit_exact(ora, lg, side):
    _case(f"lgm hierarchy {side}")
    Ho = ora.Hierarchy.lgm(side)
    Hg = lg.Hierarchy.lgm(side)
    assert Hg.num_levels == Ho.num_levels
    assert Hg.coarsest_relax == Ho.coarsest_relax
    for l in range(Ho.num_levels):
        do, dg = Ho.dims(l), Hg.dims(l)
        for k in ("n", "nnz", "type", "ncol"):
            assert do[k] == dg[k], (l, k, do[k], dg[k])
        assert do["gamma"] == dg["gamma"], l
        Lo, Lg = Ho.level(l), Hg.level(l)
        assert np.array_equal(Lo.A.ptr, Lg["rp"]), l
        assert np.array_equal(Lo.A.col, Lg["ci"]), l
        assert np.array_equal(Lo.cptr, Lg["cptr"]), l
        assert np.array_equal(Lo.perm, Lg["perm"]), l
        assert np.array_equal(Lo.A.val, Lg["val"]), l
        assert np.array_equal(Lo.A.diag, Lg["diag"]), l
        if l > 0:
            assert np.array_equal(Lo.transfer, Lg["transfer"]), l


@pytest.mark.parametrize("side", [64, 256])
def test_lgm_cycle_and_solve(ora, lg, side):
    _case(f"lgm solve {side}")
    Ho = ora.Hierarchy.lgm(side)
    Hg = lg.Hierarchy.lgm(side)
    n = side * side
    rng = np.random.default_rng(side)
    b = rng.standard_normal(n)
    b -= b.mean()
    xo = Ho.cycle(b, np.zeros(n))
    xg = Hg.cycle(b, np.zeros(n)).cpu().numpy()
    assert np.linalg.norm(xg - xo) <= 1e-12 * np.linalg.norm(xo)
    eu, ev, w = periodic_edges(side)
    A = ora.laplacian(n, eu, ev, w)
    b = rng.standard_normal(n) + 0.5
    for prec in (0, 1):
        xo, io, _ = Ho.solve(b, precision=prec)
        xg, ig = Hg.solve(torch.tensor(b, device="cuda"), precision=prec)
        xg = xg.cpu().numpy()
        assert ig["status"] == 0 and io["status"] == 0
        assert abs(ig["cycles"] - io["cycles"]) <= 1, (prec, ig["cycles"], io["cycles"])
        bp = b - b.mean()
        r = ora.residual(A, bp, xg)
        assert np.linalg.norm(r) <= 1.0000001e-8 * np.linalg.norm(bp)
        assert np.linalg.norm(xg - xo) <= 1e-6 * np.linalg.norm(xo)
        assert abs(ig["acf"] - io["acf"]) <= 0.02 * io["acf"], (prec, ig["acf"], io["acf"])


def test_lgm_full_size(ora, lg):
    """1024 x 1024 (the grid size of the paper's grid experiments): the
    hierarchy's shape and transfers equal the oracle's, the solve takes the
    oracle's cycle count and ACF, and the convergence factor per unit of work
    (finest relaxation sweeps) is about 0.5."""
    side = 1024
    _case(f"lgm full {side}")
    Ho = ora.Hierarchy.lgm(side)
    Hg = lg.Hierarchy.lgm(side)
    assert Hg.num_levels == Ho.num_levels
    for l in range(Ho.num_levels):
        assert Hg.dims(l)["nnz"] == Ho.dims(l)["nnz"]
        if l > 0:
            assert np.array_equal(Ho.level(l).transfer, Hg.level(l)["transfer"]), l
    n = side * side
    b = np.random.default_rng(7).standard_normal(n)
    xo, io, _ = Ho.solve(b)
    xg, ig = Hg.solve(torch.tensor(b, device="cuda"))
    assert ig["status"] == 0 and ig["cycles"] == io["cycles"]
    assert abs(ig["acf"] - io["acf"]) <= 0.02 * io["acf"]
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-6 * np.linalg.norm(xo)
    visits = Ho.visit_counts()
    W = sum(3 * visits[l] * Ho.dims(l)["n"] / n for l in range(Ho.num_levels - 1))
    eff = ig["acf"] ** (1.0 / W)
    assert 0.45 <= eff <= 0.56, (ig["acf"], W, eff)
