"""Parity of the HIP path with the CPU oracle on identical seeded inputs.

Integer outputs (colours, node orders, elimination sets, aggregates, coarse
sparsity) must agree bit for bit.  Every floating-point value that feeds a
decision is computed in the same order on both sides, so values are
compared bit for bit as well; solve results are compared through the
relative residual (<= tol) and the distance between the two solutions.
"""
import numpy as np
import pytest
import torch

from paper_1108_1310_amd import workloads as W

pytestmark = pytest.mark.gpu


def _graphs():
    from test_oracle_pins import random_graph
    out = {}
    eu, ev, w = random_graph(3000, 6000, 7)
    out["random3k"] = (3000, eu, ev, w)
    g = W.grid2d(64)
    out["grid64"] = (g.n, g.eu, g.ev, g.w)
    g = W.chung_lu(1 << 14)
    out["chung_lu16k"] = (g.n, g.eu, g.ev, g.w)
    g = W.rgg(1 << 14)
    out["rgg16k"] = (g.n, g.eu, g.ev, g.w)
    g = W.grid3d_aniso(16)
    out["grid3d16"] = (g.n, g.eu, g.ev, g.w)
    g = W.erdos_renyi(20000, 8.0, 3)
    out["er20k"] = (g.n, g.eu, g.ev, g.w)
    g = W.er_with_hubs(60000, 6.0, [40000, 5000, 3000, 1000, 600], 11)
    out["er_hubs60k"] = (g.n, g.eu, g.ev, g.w)
    return out


GRAPHS = None


def graphs():
    global GRAPHS
    if GRAPHS is None:
        GRAPHS = _graphs()
    return GRAPHS


@pytest.fixture(scope="module")
def lg():
    from paper_1108_1310_amd import lamg
    lamg.lib()
    return lamg


def _print_case(name):
    print(f"[case] {name}", flush=True)


@pytest.mark.parametrize("name", ["random3k", "grid64", "chung_lu16k", "rgg16k", "grid3d16", "er20k"])
def test_hierarchy_bit_exact(ora, lg, name):
    _print_case(name)
    n, eu, ev, w = graphs()[name]
    Ho = ora.Hierarchy(n, eu, ev, w)
    Hg = lg.Hierarchy(n, eu, ev, w)
    assert Hg.num_levels == Ho.num_levels
    assert Hg.coarsest_relax == Ho.coarsest_relax
    for l in range(Ho.num_levels):
        do, dg = Ho.dims(l), Hg.dims(l)
        for k in ("n", "nnz", "type", "ncol", "nF", "K", "stage"):
            assert do[k] == dg[k], (l, k, do[k], dg[k])
        assert do["gamma"] == dg["gamma"]
        Lo, Lg = Ho.level(l), Hg.level(l)
        assert np.array_equal(Lo.A.ptr, Lg["rp"]), l
        assert np.array_equal(Lo.A.col, Lg["ci"]), l
        assert np.array_equal(Lo.cptr, Lg["cptr"]), l
        assert np.array_equal(Lo.perm, Lg["perm"]), l
        assert np.array_equal(Lo.A.val, Lg["val"]), l
        assert np.array_equal(Lo.A.diag, Lg["diag"]), l
        if l > 0:
            assert np.array_equal(Lo.transfer, Lg["transfer"]), l
        if do["K"] > 0:  # test vectors were relaxed on this level
            Do, Dg = Ho.agg_diag(l), Hg.agg_diag(l)
            assert np.array_equal(Do["tv"], Dg["tv"]), l
            # energy ratio of the last test-vector sweep: sums in another order
            assert abs(Do["rate"] - Dg["rate"]) <= 1e-12 * Do["rate"], l
        if l + 1 < Ho.num_levels and Ho.dims(l + 1)["type"] == 2:
            Do, Dg = Ho.agg_diag(l), Hg.agg_diag(l)
            assert np.array_equal(Do["aff"], Dg["aff"]), l
            for k in ("ok", "weak", "hub", "state"):
                assert np.array_equal(Do[k], Dg[k]), (l, k)
            for k in ("delta1", "alpha1", "alpha2", "stage"):
                assert Do[k] == Dg[k], (l, k)


def test_colouring_kernel_bit_exact(ora, lg):
    _print_case("colour random3k")
    n, eu, ev, w = graphs()["random3k"]
    A = ora.laplacian(n, eu, ev, w)
    rp = torch.tensor(A.ptr.astype(np.int32), device="cuda")
    ci = torch.tensor(A.col, device="cuda")
    for seed, level in ((0, 0), (5, 3)):
        cg = lg.colour(rp, ci, n, seed=seed, level=level).cpu().numpy()
        assert np.array_equal(cg, ora.colour(A, seed=seed, level=level))


@pytest.mark.parametrize("name", ["grid64", "chung_lu16k", "er_hubs60k"])
def test_relaxation_kernels_bit_exact(ora, lg, name):
    """Multicolour GS sweeps (FP64, FP32) and the residual on the oracle's
    colour-ordered finest level, including rows longer than 64 entries (one
    wavefront each), rows longer than 512 (a workgroup, chunks spread over
    its wavefronts) and one of 40,001 entries (more chunks than one pass of
    the workgroup stages)."""
    _print_case(name)
    n, eu, ev, w = graphs()[name]
    Ho = ora.Hierarchy(n, eu, ev, w)
    L = Ho.level(0)
    A = L.A
    rng = np.random.default_rng(1)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    rp, ci = d(A.ptr.astype(np.int32), torch.int32), d(A.col, torch.int32)
    xg = lg.gs(rp, ci, d(A.val), d(A.diag), L.cptr, d(b), d(x0), sweeps=3).cpu().numpy()
    xo = ora.gs(A, b, x0, sweeps=3)
    assert np.array_equal(xg, xo)
    rg = lg.residual(rp, ci, d(A.val), d(A.diag), d(b), d(xo)).cpu().numpy()
    assert np.array_equal(rg, ora.residual(A, b, xo))
    v32, d32 = A.val.astype(np.float32), A.diag.astype(np.float32)
    xg32 = lg.gs(rp, ci, d(v32, torch.float32), d(d32, torch.float32), L.cptr, d(b, torch.float32),
                 d(x0, torch.float32), sweeps=2).cpu().numpy()
    xo32 = ora.gs32(A, v32, d32, b.astype(np.float32), x0.astype(np.float32), sweeps=2)
    assert np.array_equal(xg32, xo32)


@pytest.mark.parametrize("name", ["grid64", "chung_lu16k", "rgg16k", "er_hubs60k"])
def test_gs_from_zero_bit_exact(lg, name):
    """Below the finest level the cycle's first sweep starts from the zero
    fill and skips the gathers of colours not yet relaxed (they hold +0):
    the sweeps must equal the plain ones from a zero iterate bit for bit, on
    every level, hub path included, FP64 and FP32."""
    _print_case(name)
    n, eu, ev, w = graphs()[name]
    Hg = lg.Hierarchy(n, eu, ev, w)
    rng = np.random.default_rng(7)
    for l in range(Hg.num_levels):
        nl = Hg.dims(l)["n"]
        b = rng.standard_normal(nl)
        for prec in (0, 1):
            xa = Hg.level_gs(l, b, np.zeros(nl), sweeps=3, precision=prec).cpu().numpy()
            xb = Hg.level_gs_zero(l, b, sweeps=3, precision=prec).cpu().numpy()
            assert np.array_equal(xa.view(np.uint8), xb.view(np.uint8)), (l, prec)


@pytest.mark.parametrize("name", ["random3k", "grid64", "chung_lu16k", "rgg16k", "er20k", "grid3d16"])
def test_one_cycle_matches_oracle(ora, lg, name):
    """One cycle, then a second from its result, element by element against
    the oracle: |x_g - x_o|_i <= tol * max|x_o|.  The GS sweeps are bit-exact;
    the recombination sums and norms are reduced in another order, and the
    cycle carries that rounding.  Measured: <= 1.4e-14 on the 2-D grid, RGG,
    Chung-Lu and ER graphs, 9e-13 on the anisotropic 3-D grid, whose weights
    span 1 to 5e-5, hence tol 1e-13 and 1e-11 there."""
    _print_case(name)
    n, eu, ev, w = graphs()[name]
    Ho = ora.Hierarchy(n, eu, ev, w)
    Hg = lg.Hierarchy(n, eu, ev, w)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    b -= b.mean()
    x0 = np.zeros(n)
    tol = 1e-11 if name.startswith("grid3d") else 1e-13
    xo = Ho.cycle(b, x0)
    xg = Hg.cycle(b, x0).cpu().numpy()
    assert np.abs(xg - xo).max() <= tol * np.abs(xo).max()
    xo2 = Ho.cycle(b, xo)
    xg2 = Hg.cycle(b, xg).cpu().numpy()
    assert np.abs(xg2 - xo2).max() <= tol * np.abs(xo2).max()


@pytest.mark.parametrize("name", ["random3k", "grid64", "chung_lu16k", "rgg16k", "grid3d16", "er20k"])
@pytest.mark.parametrize("precision", [0, 1])
def test_solve_matches_oracle(ora, lg, name, precision):
    _print_case(f"{name} precision={precision}")
    n, eu, ev, w = graphs()[name]
    Ho = ora.Hierarchy(n, eu, ev, w)
    Hg = lg.Hierarchy(n, eu, ev, w)
    b = W.rhs_normal(n, 1, 11) + 0.25
    xo, io, _ = Ho.solve(b, precision=precision)
    xg, ig = Hg.solve(torch.tensor(b, device="cuda"), precision=precision)
    xg = xg.cpu().numpy()
    assert ig["status"] == 0 and io["status"] == 0
    assert ig["rel_residual"] <= 1e-8
    A = ora.laplacian(n, eu, ev, w)
    bp = b - b.mean()
    r = ora.residual(A, bp, xg)
    assert np.linalg.norm(r) <= 1.0000001e-8 * np.linalg.norm(bp)
    assert abs(xg.mean()) <= 1e-12 * np.abs(xg).max()
    assert abs(ig["removed_mean"] - b.mean()) <= 1e-15
    assert abs(ig["cycles"] - io["cycles"]) <= 1
    assert np.linalg.norm(xg - xo) <= 1e-6 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["grid3d16", "rgg16k"])
def test_energy_recombination_matches_oracle(ora, lg, name):
    """Iterate recombination in the energy norm (recomb_norm = 1): one cycle
    through the multi-launch path and through the single-workgroup tail
    against the oracle's cycle, and solves in FP64, FP32 + refinement and the
    persistent many-graph launch in the oracle's cycles."""
    _print_case(f"energy recombination {name}")
    n, eu, ev, w = graphs()[name]
    Ho = ora.Hierarchy(n, eu, ev, w, recomb_norm=1)
    b = W.rhs_normal(n, 1, 23)
    xo = Ho.cycle(b, np.zeros(n))
    tol = 1e-10 if name.startswith("grid3d") else 1e-12
    for tail in (4096, 0):
        Hg = lg.Hierarchy(n, eu, ev, w, recomb_norm=1, tail_max_n=tail)
        xg = Hg.cycle(b, np.zeros(n)).cpu().numpy()
        assert np.linalg.norm(xg - xo) <= tol * np.linalg.norm(xo), tail
    Hg = lg.Hierarchy(n, eu, ev, w, recomb_norm=1)
    for precision in (0, 1):
        xs, io, _ = Ho.solve(b, precision=precision)
        xg, ig = Hg.solve(torch.tensor(b, device="cuda"), precision=precision)
        assert ig["status"] == 0 and io["status"] == 0
        assert abs(ig["cycles"] - io["cycles"]) <= 1, (precision, ig["cycles"], io["cycles"])
        assert np.linalg.norm(xg.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)
    # the same graph twice in one persistent launch (two handles), FP64
    Hg.set_solve_options(precision=0)
    H2 = lg.Hierarchy(n, eu, ev, w, recomb_norm=1)
    X, infos, rc = lg.solve_batch([Hg, H2], [b, b])
    assert rc == 0
    xs, io, _ = Ho.solve(b)
    for i in range(2):
        assert abs(infos[i]["cycles"] - io["cycles"]) <= 1
        assert np.linalg.norm(X[i].cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)


def test_coarsest_solve_matches(ora, lg):
    _print_case("coarsest")
    n, eu, ev, w = graphs()["grid64"]
    Ho = ora.Hierarchy(n, eu, ev, w)
    Hg = lg.Hierarchy(n, eu, ev, w)
    nL = Ho.dims(Ho.num_levels - 1)["n"]
    b = np.random.default_rng(2).standard_normal(nL)
    b -= b.mean()
    xo = Ho.coarsest_solve(b)
    xg = Hg.coarsest_solve(torch.tensor(b, device="cuda")).cpu().numpy()
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


def test_input_errors(lg):
    _print_case("errors")
    d = lambda a, t: torch.tensor(a, dtype=t, device="cuda")
    cases = [
        (4, [0, 1], [1, 4], [1.0, 1.0], lg.E_INVALID_ARG),    # index out of range
        (4, [0, 1], [1, 1], [1.0, 1.0], lg.E_INVALID_ARG),    # self-loop
        (3, [0, 1], [1, 2], [1.0, -1.0], lg.E_BAD_WEIGHT),    # negative weight
        (3, [0, 1], [1, 2], [1.0, float("nan")], lg.E_BAD_WEIGHT),
        (4, [0, 2], [1, 3], [1.0, 1.0], lg.E_NOT_CONNECTED),  # two components
    ]
    for n, eu, ev, w, want in cases:
        with pytest.raises(lg.LamgError) as ei:
            lg.Hierarchy(n, d(eu, torch.int32), d(ev, torch.int32), d(w, torch.float64))
        assert ei.value.status == want
    # a single node and a single edge are valid problems
    H = lg.Hierarchy(1, d([], torch.int32), d([], torch.int32), d([], torch.float64))
    x, info = H.solve(torch.tensor([3.0], device="cuda"))
    assert x.item() == 0.0 and info["status"] == 0
    H = lg.Hierarchy(2, d([0], torch.int32), d([1], torch.int32), d([2.0], torch.float64))
    x, info = H.solve(torch.tensor([1.0, -1.0], device="cuda"))
    assert np.allclose(x.cpu().numpy(), [0.25, -0.25], atol=1e-14)
    # non-finite right-hand side: breakdown, reported not raised
    x, info = H.solve(torch.tensor([float("nan"), 1.0], device="cuda"), check=False)
    assert info["status"] == lg.E_BREAKDOWN


def test_degenerate_rhs(lg):
    """b = 0 and a constant b (zero after the mean removal): x = 0 in no
    cycles, FP64 and FP32 + refinement; the removed mean is reported."""
    _print_case("degenerate rhs")
    n, eu, ev, w = graphs()["chung_lu16k"]
    H = lg.Hierarchy(n, eu, ev, w)
    for prec in (0, 1):
        for c in (0.0, 2.5):
            x, info = H.solve(torch.full((n,), c, dtype=torch.float64, device="cuda"), precision=prec)
            assert info["status"] == 0 and info["cycles"] == 0, (prec, c, info)
            assert torch.count_nonzero(x).item() == 0
            assert abs(info["removed_mean"] - c) <= 1e-15 * max(1.0, c)
    # the same columns beside a regular one in a multi-vector solve
    B = np.zeros((n, 3))
    B[:, 0] = 2.5
    B[:, 1] = W.rhs_normal(n, 1, 4)
    X, info, cols, rc = H.solve_multi(B)
    assert rc == 0
    assert list(cols["cycles"][[0, 2]]) == [0, 0] and cols["cycles"][1] > 0
    X = X.cpu().numpy()
    assert np.count_nonzero(X[:, 0]) == 0 and np.count_nonzero(X[:, 2]) == 0
    assert cols["removed_mean"][0] == 2.5


def test_multi_rhs_equals_single(ora, lg):
    _print_case("multi-rhs")
    n, eu, ev, w = graphs()["grid64"]
    Hg = lg.Hierarchy(n, eu, ev, w)
    B = W.rhs_normal(n, 4, 5)
    X, infos, rc = lg.solve_batch([Hg], [torch.tensor(B, device="cuda")])
    assert rc == 0
    X = X[0].cpu().numpy()
    for j in range(4):
        xj, ij = Hg.solve(torch.tensor(B[:, j].copy(), device="cuda"))
        assert np.linalg.norm(X[:, j] - xj.cpu().numpy()) <= 1e-12 * np.linalg.norm(X[:, j])


@pytest.mark.parametrize("name", ["grid64", "rgg16k", "grid3d16"])
def test_tail_matches_multilaunch(ora, lg, name):
    """The single-workgroup tail program gives the cycle of the per-kernel
    launches (same operations; only a few row sums are ordered differently)."""
    _print_case(f"tail {name}")
    n, eu, ev, w = graphs()[name]
    Ht = lg.Hierarchy(n, eu, ev, w)                 # default: coarse levels in the tail
    Hm = lg.Hierarchy(n, eu, ev, w, tail_max_n=0)   # every level launches its kernels
    rng = np.random.default_rng(9)
    b = rng.standard_normal(n)
    b -= b.mean()
    xt = Ht.cycle(b, np.zeros(n)).cpu().numpy()
    xm = Hm.cycle(b, np.zeros(n)).cpu().numpy()
    # recombination Gram sums are reduced in another tree order
    assert np.linalg.norm(xt - xm) <= 1e-10 * np.linalg.norm(xm)
    for prec in (0, 1):
        xt, it = Ht.solve(torch.tensor(b, device="cuda"), precision=prec)
        xm, im = Hm.solve(torch.tensor(b, device="cuda"), precision=prec)
        assert it["status"] == 0 and im["status"] == 0
        assert abs(it["cycles"] - im["cycles"]) <= 1
        assert torch.linalg.norm(xt - xm) <= 1e-7 * torch.linalg.norm(xm)
