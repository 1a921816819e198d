"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only), driven through its setup, cycles, solves in both
precisions, recombination in both norms, the elimination and Galerkin
building blocks, the geometric multigrid and the negative-weight path, in a
child process with the ASan runtime preloaded.  Any invalid access, leak of
a freed pointer or undefined operation aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
from oracle import oracle as O
from paper_1108_1310_amd import workloads as W
for g in (W.grid2d(24), W.rgg(1 << 11), W.chung_lu(1 << 11), W.grid3d_aniso(8), W.erdos_renyi(600, 6.0, 2)):
    for norm in (0, 1):
        H = O.Hierarchy(g.n, g.eu, g.ev, g.w, recomb_norm=norm)
        b = W.rhs_normal(g.n, 1, 3)
        for prec in (0, 1):
            x, info, _ = H.solve(b, precision=prec)
            assert info["status"] == 0, info
        H.cycle(b, np.zeros(g.n))
        H.visit_counts()
        for l in range(H.num_levels):
            H.level(l)
    A = O.laplacian(g.n, g.eu, g.ev, g.w)
    O.colour(A); O.colour_jp(A)
    f = O.elim_select(A)
    O.schur(A, f)
    O.galerkin(A, np.arange(g.n) // 2, (g.n + 1) // 2)
    O.recombine(A, b, np.zeros(g.n), np.stack([b, 2 * b], axis=1), norm=1)
    H = O.Hierarchy(g.n, g.eu, g.ev, g.w)
    lam = H.solve(b)[0]
    H.adjoint(lam, b)
Hl = O.Hierarchy.lgm(32)
Hl.solve(W.rhs_normal(32 * 32, 1, 4))
gn = W.grid_stencil(24, "b")
Hn = O.Hierarchy(gn.n, gn.eu, gn.ev, gn.w, allow_negative=1)
Hn.solve(W.rhs_normal(gn.n, 1, 5))
O.set_plain_rows(True); O.row_reduce(np.arange(1000.0)); O.set_plain_rows(False)
assert O.laplacian_status(3, np.array([0, 1]), np.array([1, 1]), np.array([1.0, 1.0])) != 0
print("SANITIZED_OK")
"""


@pytest.mark.skipif(not sys.platform.startswith("linux"), reason="gcc sanitizer runtimes")
def test_oracle_under_asan_ubsan():
    from oracle import oracle as O
    lib = O.build(force=True, sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("no ASan runtime")
    env = dict(os.environ, LAMG_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", "ROOT = %r\n" % ROOT + SCRIPT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
