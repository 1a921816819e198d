"""Differentiable solve: the adjoint gradients of the HIP path against a dense
pseudo-inverse gradient, the CPU oracle's adjoint, and finite differences."""
import numpy as np
import pytest
import torch

from paper_1108_1310_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    print(f"[case] {name}", flush=True)


def _loss_setup(g, frac=0.01, seed=105):
    lab, hold = W.label_split(g.n, frac, seed)
    b = W.rhs_labels(g.n, lab, seed)
    return b, hold


def test_adjoint_matches_dense_gradient(ora):
    """Tight check on a small random geometric graph (n ~ 2000): gradients of
    L = sum_{h in H} x_h^2 w.r.t. b and every edge weight."""
    _case("dense gradient rgg2k")
    from paper_1108_1310_amd import lamg
    g = W.rgg(2048, seed=7)
    b, hold = _loss_setup(g, 0.02, 7)
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    bt = d(b).requires_grad_(True)
    wt = d(g.w).requires_grad_(True)
    eu, ev = d(g.eu, torch.int32), d(g.ev, torch.int32)
    x = lamg.laplacian_solve(bt, wt, eu, ev, g.n, tol=1e-13)
    L = (x[torch.tensor(hold, device="cuda")] ** 2).sum()
    L.backward()
    A = ora.laplacian(g.n, g.eu, g.ev, g.w).dense()
    Ap = np.linalg.pinv(A)
    bp = b - b.mean()
    xd = Ap @ bp
    gx = np.zeros(g.n)
    gx[hold] = 2 * xd[hold]
    lam = Ap @ gx
    assert np.linalg.norm(bt.grad.cpu().numpy() - lam) <= 1e-9 * np.linalg.norm(lam)
    gw = -(lam[g.eu] - lam[g.ev]) * (xd[g.eu] - xd[g.ev])
    got = wt.grad.cpu().numpy()
    assert np.linalg.norm(got - gw) <= 1e-9 * np.linalg.norm(gw)


def test_adjoint_matches_oracle(ora):
    _case("oracle adjoint rgg16k")
    from paper_1108_1310_amd import lamg
    g = W.rgg(1 << 14, seed=11)
    b, hold = _loss_setup(g, 0.01, 11)
    Ho = ora.Hierarchy(g.n, g.eu, g.ev, g.w, tol=1e-12)
    xo, io, _ = Ho.solve(b)
    go = np.zeros(g.n)
    go[hold] = 2 * xo[hold]
    gbo, gwo, rc = Ho.adjoint(xo, go)
    assert rc == 0
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    bt = d(b).requires_grad_(True)
    wt = d(g.w).requires_grad_(True)
    x = lamg.laplacian_solve(bt, wt, d(g.eu, torch.int32), d(g.ev, torch.int32), g.n, tol=1e-12)
    (x[torch.tensor(hold, device="cuda")] ** 2).sum().backward()
    assert np.linalg.norm(bt.grad.cpu().numpy() - gbo) <= 1e-8 * np.linalg.norm(gbo)
    assert np.linalg.norm(wt.grad.cpu().numpy() - gwo) <= 1e-8 * np.linalg.norm(gwo)


def test_adjoint_finite_differences():
    """Central differences with h_e = 1e-4 w_e on sampled edges (half uniform,
    half incident to labelled or held-out nodes); each perturbed problem is
    set up again and solved to 1e-13."""
    _case("finite differences rgg8k")
    from paper_1108_1310_amd import lamg
    g = W.rgg(1 << 13, seed=5)
    b, hold = _loss_setup(g, 0.01, 5)
    lab, _ = W.label_split(g.n, 0.01, 5)
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    eu, ev, bt = d(g.eu, torch.int32), d(g.ev, torch.int32), d(b)
    ht = torch.tensor(hold, device="cuda")
    wt = d(g.w).requires_grad_(True)
    x = lamg.laplacian_solve(bt, wt, eu, ev, g.n, tol=1e-13)
    (x[ht] ** 2).sum().backward()
    ga = wt.grad.cpu().numpy()
    rng = np.random.default_rng(64)
    touch = np.isin(g.eu, np.concatenate([lab, hold])) | np.isin(g.ev, np.concatenate([lab, hold]))
    edges = np.concatenate([rng.choice(g.m, 8, replace=False), rng.choice(np.where(touch)[0], 8, replace=False)])

    def loss(w):
        H = lamg.Hierarchy(g.n, eu, ev, d(w), tol=1e-13)
        xx, info = H.solve(bt)
        assert info["status"] == 0
        return float((xx[ht] ** 2).sum())

    scale = np.abs(ga).max()
    for e in edges:
        h = 1e-4 * g.w[e]
        wp, wm = g.w.copy(), g.w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert abs(fd - ga[e]) <= 1e-4 * max(abs(ga[e]), 1e-3 * scale), (e, fd, ga[e])
