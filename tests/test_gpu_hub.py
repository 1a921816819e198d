"""The hub sweep of power-law levels: the split (first hub colour, hub rows,
hub-to-hub entries) is recomputed from the oracle's colour-ordered level and
must match exactly; the solve's GS sweeps through it must equal the oracle's
sequential sweeps on the same level to rounding (the hub rows add their sums
in another order: low colours first, then the hub-to-hub entries)."""
import numpy as np
import pytest
import torch

from paper_1108_1310_amd import workloads as W

pytestmark = pytest.mark.gpu

HUB_MAX_ROWS, HUB_MIN_COLOURS = 4096, 8


def _case(name):
    print(f"[case] {name}", flush=True)


@pytest.fixture(scope="module")
def lg():
    from paper_1108_1310_amd import lamg
    lamg.lib()
    return lamg


_G = {}


def chung_lu(n0):
    if n0 not in _G:
        _G[n0] = W.chung_lu(n0)
    return _G[n0]


HUB_CHUNK, HUB_COST_LAUNCH, HUB_COST_CHUNK = 4096, 100, 18


def _hub_counts(ptr, col, r0, n):
    """Per row of [r0, n): entries into columns >= r0."""
    return np.array([int(np.count_nonzero(col[ptr[u]:ptr[u + 1]] >= r0)) for u in range(r0, n)], np.int64)


def _chunks(cptr, K, cnt):
    """Chunks of whole rows of one colour with at most HUB_CHUNK entries."""
    r0 = int(cptr[K])
    hr = np.concatenate([[0], np.cumsum(cnt)])
    total = 0
    for c in range(K, len(cptr) - 1):
        a, z = int(cptr[c]) - r0, int(cptr[c + 1]) - r0
        first = a
        for u in range(a, z):
            if hr[u + 1] - hr[first] > HUB_CHUNK:
                total += 1
                first = u
        total += 1
    return total


def expected_split(cptr, A):
    """The split rule: K0 = the smallest K >= 1 whose colours >= K hold at
    most HUB_MAX_ROWS rows (at least HUB_MIN_COLOURS hub colours needed);
    then the K >= K0 (keeping HUB_MIN_COLOURS hub colours) minimising
    (K - K0) launches + chunks, priced 100 / 18 (ties: the smallest K).  The
    hub-to-hub entries are those of rows >= cptr[K] into columns >= cptr[K]."""
    nc = len(cptr) - 1
    n = int(cptr[-1])
    if n <= HUB_MAX_ROWS or nc < HUB_MIN_COLOURS:
        return None
    K0 = nc
    for c in range(nc - 1, 0, -1):
        if n - cptr[c] > HUB_MAX_ROWS:
            break
        K0 = c
    if nc - K0 < HUB_MIN_COLOURS:
        return None
    ptr, col = np.asarray(A.ptr), np.asarray(A.col)
    best, K = None, K0
    for K2 in range(K0, nc - HUB_MIN_COLOURS + 1):
        r2 = int(cptr[K2])
        cost = (K2 - K0) * HUB_COST_LAUNCH + _chunks(cptr, K2, _hub_counts(ptr, col, r2, n)) * HUB_COST_CHUNK
        if best is None or cost < best:
            best, K = cost, K2
    r0 = int(cptr[K])
    nnz = int(np.count_nonzero(col[ptr[r0]:ptr[n]] >= r0))
    return dict(k=K, r0=r0, n=n - r0, nnz=nnz)


@pytest.mark.parametrize("n0", [1 << 14, 1 << 16])
def test_hub_split_and_sweeps(ora, lg, n0):
    _case(f"hub chung_lu n0={n0}")
    g = chung_lu(n0)
    Ho = ora.Hierarchy(g.n, g.eu, g.ev, g.w)
    Hg = lg.Hierarchy(g.n, g.eu, g.ev, g.w)
    assert Hg.num_levels == Ho.num_levels
    taken = 0
    for l in range(Ho.num_levels):
        L = Ho.level(l)
        exp = expected_split(np.asarray(L.cptr), L.A)
        got = Hg.hub_info(l)
        if exp is None:
            assert got["k"] == -1, l
            continue
        assert got == exp, (l, got, exp)
        taken += 1
        n = L.A.n
        rng = np.random.default_rng(100 + l)
        b = rng.standard_normal(n)
        x0 = rng.standard_normal(n)
        xo = ora.gs(L.A, b, x0, sweeps=3)
        xg = Hg.level_gs(l, b, x0, sweeps=3, precision=0).cpu().numpy()
        scale = np.abs(xo).max()
        assert np.abs(xg - xo).max() <= 1e-12 * scale, (l, np.abs(xg - xo).max() / scale)
        # rows below the hub colours see the same operands in the same order
        # in the first sweep: bitwise equal there
        x1o = ora.gs(L.A, b, x0, sweeps=1)
        x1g = Hg.level_gs(l, b, x0, sweeps=1, precision=0).cpu().numpy()
        assert np.array_equal(x1g[:exp["r0"]], x1o[:exp["r0"]]), l
        assert np.abs(x1g - x1o).max() <= 1e-13 * np.abs(x1o).max(), l
        # b = 0 (the smoothing of a homogeneous error)
        xz = Hg.level_gs(l, None, x0, sweeps=2, precision=0).cpu().numpy()
        xzo = ora.gs(L.A, None, x0, sweeps=2)
        assert np.abs(xz - xzo).max() <= 1e-12 * np.abs(xzo).max(), l
        # FP32 on the level's FP32 copy, against the oracle's FP32 sweeps
        v32, d32 = L.A.val.astype(np.float32), L.A.diag.astype(np.float32)
        x32o = ora.gs32(L.A, v32, d32, b.astype(np.float32), x0.astype(np.float32), sweeps=2)
        x32g = Hg.level_gs(l, b, x0, sweeps=2, precision=1).cpu().numpy()
        assert np.abs(x32g.astype(np.float64) - x32o).max() <= 1e-5 * np.abs(x32o).max(), l
    assert taken >= 1


def test_hub_solve_matches_oracle(ora, lg):
    """A whole solve through hub sweeps (Chung-Lu n0 = 2^16): the oracle's
    cycle count (+-1) and solution."""
    _case("hub solve chung_lu 2^16")
    g = chung_lu(1 << 16)
    Hg = lg.Hierarchy(g.n, g.eu, g.ev, g.w)
    assert any(Hg.hub_info(l)["k"] >= 0 for l in range(Hg.num_levels))
    b = W.rhs_normal(g.n, 1, 5)
    Ho = ora.Hierarchy(g.n, g.eu, g.ev, g.w)
    xo, io, _ = Ho.solve(b)
    for prec in (0, 1):
        x, info = Hg.solve(torch.tensor(b, device="cuda"), precision=prec)
        assert info["status"] == 0
        assert abs(info["cycles"] - io["cycles"]) <= 1
        x = x.cpu().numpy()
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
