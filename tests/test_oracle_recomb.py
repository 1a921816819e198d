"""Pins of the oracle's iterate recombination (Section 3.4.5, eq. recomb) in
both norms (the residual 2-norm printed there, the default, and the energy
norm of the error, an option), of
the cycle index and fractional visit schedule (Section 4.2, eq.
cycle_index) against hand-evaluated values, and of the fixed row-sum order
(a rounding choice only: the hierarchies and cycle counts do not depend on
it)."""
import json
import os

import numpy as np
import pytest

from paper_1108_1310_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _dense(ora, g):
    A = ora.laplacian(g.n, g.eu, g.ev, g.w)
    return A, A.dense()


def _case(ora, n=300, seed=3):
    g = W.erdos_renyi(n, 6.0, seed)
    A, D = _dense(ora, g)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(g.n)
    b -= b.mean()
    # iterates shaped like a cycle's: smoothed by a few GS sweeps from noise
    x = ora.gs(A, b, rng.standard_normal(g.n), sweeps=2)
    X0 = ora.gs(A, b, x + 0.3 * rng.standard_normal(g.n), sweeps=1)
    X1 = ora.gs(A, b, x + 0.3 * rng.standard_normal(g.n), sweeps=1)
    return A, D, b, x, X0, X1


@pytest.mark.parametrize("th", [1, 2])
def test_recombination_is_the_least_squares_solution(ora, th):
    """Residual norm (as printed): alpha minimises
    ||b - A(x + sum_i alpha_i (X_i - x))||_2: equal to numpy's least-squares
    solution of [R_i - r] alpha = -r, and y is the stated combination."""
    A, D, b, x, X0, X1 = _case(ora)
    Xs = np.stack([X0, X1][:th], axis=1)
    y, alpha = ora.recombine(A, b, x, Xs, norm=0)
    r = b - D @ x
    M = np.stack([(b - D @ Xs[:, i]) - r for i in range(th)], axis=1)
    ref, *_ = np.linalg.lstsq(M, -r, rcond=None)
    assert np.allclose(alpha, ref, rtol=1e-9, atol=1e-12), (alpha, ref)
    yref = x + sum(alpha[i] * (Xs[:, i] - x) for i in range(th))
    assert np.allclose(y, yref, rtol=0, atol=1e-12 * np.abs(yref).max())
    # the minimum over the combination space
    ry = np.linalg.norm(b - D @ y)
    for t in np.linspace(-2, 2, 9):
        trial = x + t * (Xs[:, 0] - x)
        assert ry <= np.linalg.norm(b - D @ trial) * (1 + 1e-12)


@pytest.mark.parametrize("th", [1, 2])
def test_energy_recombination_minimises_the_error_energy(ora, th):
    """Energy norm (the option): alpha minimises (y - x*)^T A (y - x*) over
    the combinations, i.e. solves (D^T A D) alpha = D^T r with D = [X_i - x]
    (numpy on the dense Laplacian); y has the smallest error energy of any
    step along X_0 - x, and the error energy never exceeds that of x or of
    any X_i."""
    A, Dn, b, x, X0, X1 = _case(ora)
    Xs = np.stack([X0, X1][:th], axis=1)
    y, alpha = ora.recombine(A, b, x, Xs, norm=1)
    Dm = Xs - x[:, None]
    ref = np.linalg.solve(Dm.T @ Dn @ Dm, Dm.T @ (b - Dn @ x))
    assert np.allclose(alpha, ref, rtol=1e-8, atol=1e-12), (alpha, ref)
    assert np.allclose(y, x + Dm @ alpha, rtol=0, atol=1e-12 * np.abs(y).max())
    xs = np.linalg.lstsq(Dn, b, rcond=None)[0]
    err = lambda z: float((z - xs) @ Dn @ (z - xs))
    ey = err(y)
    for t in np.linspace(-2, 2, 9):
        assert ey <= err(x + t * (Xs[:, 0] - x)) * (1 + 1e-9) + 1e-20
    assert ey <= min([err(x)] + [err(Xs[:, i]) for i in range(th)]) * (1 + 1e-9)
    # the residual-norm choice generally differs
    _, a0 = ora.recombine(A, b, x, Xs, norm=0)
    assert not np.allclose(a0, alpha)


@pytest.mark.parametrize("th", [1, 2])
def test_recombination_never_increases_the_residual(ora, th):
    """alpha = 0 (keep x) and alpha = e_i (take X_i) are feasible, so the
    recombined residual (residual norm) is at most the smallest of those
    residuals."""
    for seed in range(5):
        A, D, b, x, X0, X1 = _case(ora, 200, 10 + seed)
        Xs = np.stack([X0, X1][:th], axis=1)
        y, _ = ora.recombine(A, b, x, Xs, norm=0)
        ry = np.linalg.norm(b - D @ y)
        bound = min([np.linalg.norm(b - D @ x)] + [np.linalg.norm(b - D @ Xs[:, i]) for i in range(th)])
        assert ry <= bound * (1 + 1e-12), (seed, ry, bound)


def test_recombination_degenerate_directions(ora):
    """Saved iterates equal to each other (a singular 2 x 2 system) or to x
    (a zero direction): the dropped direction gets alpha = 0 and the
    residual still does not increase."""
    A, D, b, x, X0, X1 = _case(ora)
    for norm in (0, 1):
        y, alpha = ora.recombine(A, b, x, np.stack([X0, X0], axis=1), norm=norm)
        assert alpha[1] == 0.0 and alpha[0] != 0.0
        r1, _ = ora.recombine(A, b, x, X0[:, None], norm=norm)
        assert np.allclose(y, r1, rtol=0, atol=1e-13 * np.abs(y).max())
        y, alpha = ora.recombine(A, b, x, x[:, None].copy(), norm=norm)
        assert alpha[0] == 0.0 and np.array_equal(y, x)


def test_cycle_index_against_hand_values(ora):
    """gamma^l and the per-level body counts of one finest cycle equal the
    values evaluated by hand from eq. cycle_index and the fractional cycle
    index (tests/golden/cycle_index_hand.json)."""
    gold = json.load(open(os.path.join(HERE, "golden", "cycle_index_hand.json")))
    graphs = {"grid2d_64": lambda: W.grid2d(64), "rgg_2p14": lambda: W.rgg(1 << 14)}
    for case in gold["cases"]:
        g = graphs[case["graph"]]()
        H = ora.Hierarchy(g.n, g.eu, g.ev, g.w)
        dims = [H.dims(l) for l in range(H.num_levels)]
        assert [d["nnz"] for d in dims] == case["edges"], case["graph"]
        assert [d["type"] for d in dims] == case["types"], case["graph"]
        for l, want in enumerate(case["gamma"]):
            assert abs(dims[l]["gamma"] - want) <= 1e-14 * want, (case["graph"], l, dims[l]["gamma"], want)
        assert list(H.visit_counts()) == case["bodies"], case["graph"]


def test_row_order_is_rounding_only(ora):
    """The fixed chunked order of long rows (shared with the GPU path) against
    plain left-to-right sums: on graphs with rows far longer than 64 entries
    (Chung-Lu hubs) and without, every level's size, pattern, transfer and
    cycle count is the same; the solutions differ by rounding."""
    cases = {"chung_lu_2p16": W.chung_lu(1 << 16), "rgg_2p14": W.rgg(1 << 14),
             "er": W.erdos_renyi(20000, 8, 5), "grid3d_aniso_16": W.grid3d_aniso(16)}

    def snap(g):
        H = ora.Hierarchy(g.n, g.eu, g.ev, g.w)
        lv = []
        for l in range(H.num_levels):
            L = H.level(l)
            lv.append((H.dims(l), L.A.ptr, L.A.col, getattr(L, "transfer", None)))
        b = W.rhs_normal(g.n, 1, 11)
        x, info, _ = H.solve(b)
        return lv, info, x

    try:
        for name, g in cases.items():
            ora.set_plain_rows(False)
            a = snap(g)
            ora.set_plain_rows(True)
            p = snap(g)
            assert len(a[0]) == len(p[0]), name
            for la, lp in zip(a[0], p[0]):
                assert la[0] == lp[0], name
                assert np.array_equal(la[1], lp[1]) and np.array_equal(la[2], lp[2]), name
                assert (la[3] is None) == (lp[3] is None) and (la[3] is None or np.array_equal(la[3], lp[3])), name
            assert a[1]["cycles"] == p[1]["cycles"] and a[1]["status"] == p[1]["status"] == 0, name
            assert np.linalg.norm(a[2] - p[2]) <= 1e-12 * np.linalg.norm(a[2]), name
        # the long rows do exist: the chunked order differs from the plain one
        t = np.random.default_rng(1).standard_normal(4000)
        ora.set_plain_rows(False)
        chunked = ora.row_reduce(t)
        ora.set_plain_rows(True)
        plain = ora.row_reduce(t)
        assert plain == sum(t.tolist()) and abs(chunked - plain) <= 1e-12 * np.abs(t).sum()
        assert W.chung_lu(1 << 16).n and max(np.bincount(cases["chung_lu_2p16"].eu)) > 512
    finally:
        ora.set_plain_rows(False)
