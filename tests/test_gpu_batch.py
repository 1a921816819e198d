"""Many graphs in one persistent launch: every graph's solve against the
oracle's solve of that graph, launch configurations against each other, and
the batch entry's bookkeeping (mixed precisions, multi-RHS entries, warm
starts, statuses)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1108_1310_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    print(f"[case] {name}", flush=True)


@pytest.fixture(scope="module")
def lg():
    from paper_1108_1310_amd import lamg
    lamg.lib()
    return lamg


_B = {}


def batch(count, nmin, nmax, seed):
    key = (count, nmin, nmax, seed)
    if key not in _B:
        gs = W.graph_batch(count, nmin, nmax, seed)
        bs = [W.rhs_normal(g.n, 1, 1000 + i) + 0.1 * i for i, g in enumerate(gs)]
        _B[key] = (gs, bs)
    return _B[key]


def _hier(lg, g, **kw):
    return lg.Hierarchy(g.n, g.eu, g.ev, g.w, **kw)


def test_batch_matches_oracle(ora, lg):
    """12 uneven graphs (grid / ER / RGG, n in [300, 6000]), FP64 and FP32
    refinement mixed in one launch: each graph meets its tolerance, in the
    oracle's cycles, at the oracle's solution."""
    _case("batch oracle 12 graphs")
    gs, bs = batch(12, 300, 6000, 31)
    hs = [_hier(lg, g) for g in gs]
    for i, h in enumerate(hs):
        h.set_solve_options(precision=i % 2)
    X, infos, rc = lg.solve_batch(hs, bs)
    assert rc == 0
    for i, (g, b, h) in enumerate(zip(gs, bs, hs)):
        Ho = ora.Hierarchy(g.n, g.eu, g.ev, g.w)
        xo, io, _ = Ho.solve(b, precision=i % 2)
        assert io["status"] == 0
        x = X[i].cpu().numpy()
        bp = b - b.mean()
        A = ora.laplacian(g.n, g.eu, g.ev, g.w)
        assert np.linalg.norm(ora.residual(A, bp, x)) <= 1.0000001e-8 * np.linalg.norm(bp), i
        assert infos[i]["rel_residual"] <= 1e-8
        assert abs(infos[i]["cycles"] - io["cycles"]) <= 1, (i, infos[i]["cycles"], io["cycles"])
        assert abs(infos[i]["removed_mean"] - b.mean()) <= 1e-14 * max(1.0, abs(b.mean()))
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo), i


def test_batch_configs_identical(lg):
    """Every launch configuration the tuner may pick gives bitwise the same
    solutions (the same sums in the same order); only the time differs."""
    _case("batch configs")
    from paper_1108_1310_amd.lamg import lib
    gs, bs = batch(10, 500, 20000, 37)
    hs = [_hier(lg, g) for g in gs]
    ref = None
    try:
        for c in range(lg.BATCH_CONFIGS):
            assert lib().lamg_t_batch_config(c) == 0
            X, infos, rc = lg.solve_batch(hs, bs)
            assert rc == 0
            got = [x.cpu().numpy() for x in X], [i["cycles"] for i in infos]
            if ref is None:
                ref = got
            else:
                assert got[1] == ref[1]
                for a, b in zip(got[0], ref[0]):
                    assert np.array_equal(a, b)
    finally:
        lib().lamg_t_batch_config(-1)
    # the tuned path (first call times every configuration) gives the same
    X, infos, rc = lg.solve_batch(hs, bs)
    assert rc == 0
    for a, b in zip([x.cpu().numpy() for x in X], ref[0]):
        assert np.array_equal(a, b)


def test_batch_equals_single_solves(lg):
    """The persistent launch and the multi-launch single solve agree (norms
    and means are reduced in another order, so to rounding)."""
    _case("batch vs single")
    gs, bs = batch(6, 1000, 30000, 41)
    hs = [_hier(lg, g) for g in gs]
    X, infos, rc = lg.solve_batch(hs, bs)
    assert rc == 0
    for i, (h, b) in enumerate(zip(hs, bs)):
        x1, i1 = h.solve(torch.tensor(b, device="cuda"))
        assert i1["status"] == 0
        assert abs(i1["cycles"] - infos[i]["cycles"]) <= 1
        assert torch.linalg.norm(x1 - X[i]) <= 1e-7 * torch.linalg.norm(x1)


def test_batch_mixed_entries_and_status(ora, lg):
    """A multi-RHS entry and single-RHS entries in one call; a graph with a
    cycle limit reports not-converged while the others converge; a warm start
    from converged solutions takes no cycle."""
    _case("batch mixed")
    gs, bs = batch(5, 400, 4000, 43)
    hs = [_hier(lg, g) for g in gs]
    hs[2].set_solve_options(max_cycles=2)
    Bm = W.rhs_normal(gs[4].n, 3, 77)
    ins = bs[:4] + [Bm]
    X, infos, rc = lg.solve_batch(hs, ins)
    assert rc == 4
    assert infos[2]["cycles"] == 2 and infos[2]["rel_residual"] > 1e-8
    for i in (0, 1, 3):
        assert infos[i]["rel_residual"] <= 1e-8
    assert X[4].shape == (gs[4].n, 3)
    A = ora.laplacian(gs[4].n, gs[4].eu, gs[4].ev, gs[4].w)
    for j in range(3):
        bj = Bm[:, j] - Bm[:, j].mean()
        assert np.linalg.norm(ora.residual(A, bj, X[4][:, j].cpu().numpy())) <= 1.0000001e-8 * np.linalg.norm(bj)
    hs[2].set_solve_options(max_cycles=100)
    X, infos, rc = lg.solve_batch(hs[:4], bs[:4])
    assert rc == 0
    Xw, iw, rc = lg.solve_batch(hs[:4], bs[:4], X)
    assert rc == 0
    assert all(i["cycles"] == 0 for i in iw)
    for a, b in zip(Xw, X):
        assert torch.equal(a, b)


def test_batch_rejects_duplicate_handles(lg):
    _case("batch duplicates")
    from paper_1108_1310_amd.lamg import Info, lib
    gs, bs = batch(5, 400, 4000, 43)
    h = _hier(lg, gs[0])
    b = torch.tensor(bs[0], device="cuda")
    x = torch.zeros_like(b)
    hp = (C.c_void_p * 2)(h.h.value, h.h.value)
    bp = (C.c_void_p * 2)(b.data_ptr(), b.data_ptr())
    xp = (C.c_void_p * 2)(x.data_ptr(), x.data_ptr())
    assert lib().lamg_solve_batch(2, hp, (C.c_int32 * 2)(1, 1), bp, xp, (Info * 2)()) == 1


def test_tune_cache_persists(tmp_path):
    """The tuner's choice for a batch shape is written to LAMG_TUNE_CACHE and
    read back by a later process, which then does not tune again (the file
    gains no line); both processes return the same solutions."""
    import os
    import subprocess
    import sys
    print("[case] batch tune cache", flush=True)
    cache = tmp_path / "tune.txt"
    out = [tmp_path / "x0.npy", tmp_path / "x1.npy"]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, numpy as np, torch\n"
        f"sys.path.insert(0, {root!r})\n"
        "from paper_1108_1310_amd import lamg, workloads as W\n"
        "gs = W.graph_batch(6, 500, 5000, 53)\n"
        "hs = [lamg.Hierarchy(g.n, g.eu, g.ev, g.w) for g in gs]\n"
        "bs = [W.rhs_normal(g.n, 1, 60 + i) for i, g in enumerate(gs)]\n"
        "X, infos, rc = lamg.solve_batch(hs, bs)\n"
        "assert rc == 0\n"
        "np.save(sys.argv[1], np.concatenate([x.cpu().numpy() for x in X]))\n")
    env = dict(os.environ, LAMG_TUNE_CACHE=str(cache))
    for i in range(2):
        r = subprocess.run([sys.executable, "-c", code, str(out[i])], env=env, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-3000:]
        lines = cache.read_text().split("\n")
        lines = [l for l in lines if l.strip()]
        assert len(lines) == 1, lines  # tuned once, reused by the second process
        key, cfg = lines[0].split()
        assert 0 <= int(cfg) < 10 and len(key) == 16
    assert np.array_equal(np.load(out[0]), np.load(out[1]))
