"""Run-to-run determinism of the HIP path and properness of its colourings:
two independent setups of a graph give bitwise the same hierarchy (every
level's CSR, diagonal, colour classes, node order and transfer), every level's
colour classes hold no edge, and repeated solves (FP64, FP32 with refinement,
multi-vector) return bitwise the same iterate and the same statistics.  All
reductions use fixed grids and fixed orders, so no result depends on timing."""
import numpy as np
import pytest
import torch

from paper_1108_1310_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lg():
    from paper_1108_1310_amd import lamg
    lamg.lib()
    return lamg


def _graph(name):
    return {"chung_lu16k": lambda: W.chung_lu(1 << 14), "rgg16k": lambda: W.rgg(1 << 14),
            "grid3d16": lambda: W.grid3d_aniso(16), "er20k": lambda: W.erdos_renyi(20000, 8.0, 3)}[name]()


@pytest.mark.parametrize("name", ["chung_lu16k", "rgg16k", "grid3d16", "er20k"])
def test_setup_and_solve_deterministic(lg, name):
    print(f"[case] determinism {name}", flush=True)
    g = _graph(name)
    H1 = lg.Hierarchy(g.n, g.eu, g.ev, g.w)
    H2 = lg.Hierarchy(g.n, g.eu, g.ev, g.w)
    assert H1.num_levels == H2.num_levels
    for l in range(H1.num_levels):
        a, b = H1.level(l), H2.level(l)
        for key in ("rp", "ci", "val", "diag", "cptr", "perm"):
            assert np.array_equal(a[key], b[key]), (l, key)
        if l > 0:
            assert np.array_equal(a["transfer"], b["transfer"]), l
        # the colour classes are independent sets
        colour = np.repeat(np.arange(len(a["cptr"]) - 1), np.diff(a["cptr"]))
        rows = np.repeat(np.arange(a["n"]), np.diff(a["rp"]))
        assert len(colour) == a["n"] and not np.any(colour[rows] == colour[a["ci"]]), l
    b = torch.tensor(W.rhs_normal(g.n, 1, 29), device="cuda")
    for prec in (0, 1):
        x1, i1 = H1.solve(b, precision=prec)
        x2, i2 = H1.solve(b, precision=prec)
        x3, i3 = H2.solve(b, precision=prec)
        assert torch.equal(x1, x2) and torch.equal(x1, x3), prec
        for k in ("cycles", "rel_residual", "acf", "removed_mean", "status"):
            assert i1[k] == i2[k] == i3[k], (prec, k)
    B = torch.tensor(W.rhs_normal(g.n, 4, 31), device="cuda")
    X1, _, c1, _ = H1.solve_multi(B, precision=0)
    X2, _, c2, _ = H2.solve_multi(B, precision=0)
    assert torch.equal(X1, X2) and np.array_equal(c1["cycles"], c2["cycles"])
