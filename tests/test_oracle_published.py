"""The oracle against a published table entry (Section 5.2, table of grid
Laplacians on 1024 x 1024 grids, case (a)): the 5-point Laplacian with
Neumann boundary conditions -- the unit-weight grid graph, m = 2,095,104 --
is solved at an asymptotic convergence factor of 0.216.  The oracle's ACF on
seeded right-hand sides must be close to it.  (The paper's level count, 19,
is not compared: this implementation counts every elimination level as a
level of its own and has 23.)"""
import numpy as np

from oracle import oracle as O
from paper_1108_1310_amd import workloads as W


def test_grid_1024_acf_matches_table():
    g = W.grid2d(1024)
    assert g.m == 2095104
    H = O.Hierarchy(g.n, g.eu, g.ev, g.w)
    acfs = []
    for seed in (1, 2):
        x, info, _ = H.solve(W.rhs_normal(g.n, 1, seed))
        assert info["status"] == 0 and info["rel_residual"] <= 1e-8
        acfs.append(info["acf"])
    acf = float(np.mean(acfs))
    assert 0.18 <= acf <= 0.25, acfs
