"""Device memory through the allocator hooks of lamg_options (torch's caching
allocator via the binding's TorchAllocator): setup temporaries, the
hierarchy, the multi-vector workspace and the batch buffers all come from
the hook and all return to it; results are bitwise those of a hierarchy on
the library's own allocations."""
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


def test_torch_allocator_hook(lg):
    print("[case] torch allocator hook", flush=True)
    A = lg.TorchAllocator()
    g = W.chung_lu(1 << 14)   # elimination, aggregation, hub sweeps, tail
    h = W.grid2d(40)
    H1 = lg.Hierarchy(g.n, g.eu, g.ev, g.w, allocator=A)
    H0 = lg.Hierarchy(g.n, g.eu, g.ev, g.w)
    after_setup = len(A.live)
    assert A.allocs > after_setup > 0          # the setup's temporaries went through the hook and back
    b = torch.tensor(W.rhs_normal(g.n, 1, 5), device="cuda")
    for prec in (0, 1):
        x1, i1 = H1.solve(b, precision=prec)
        x0, i0 = H0.solve(b, precision=prec)
        assert i1["status"] == 0 and i1["cycles"] == i0["cycles"]
        assert torch.equal(x1, x0)
    B = torch.tensor(W.rhs_normal(g.n, 4, 9), device="cuda")
    X1, _, _, rc1 = H1.solve_multi(B)
    X0, _, _, rc0 = H0.solve_multi(B)
    assert rc1 == 0 and rc0 == 0 and torch.equal(X1, X0)
    assert len(A.live) > after_setup              # the multi-vector workspace
    G1 = lg.Hierarchy(h.n, h.eu, h.ev, h.w, allocator=A)
    G0 = lg.Hierarchy(h.n, h.eu, h.ev, h.w)
    bh = W.rhs_normal(h.n, 1, 6)
    before = A.allocs
    Xa, ia, rca = lg.solve_batch([H1, G1], [b.cpu().numpy(), bh])
    Xb, ib, rcb = lg.solve_batch([H0, G0], [b.cpu().numpy(), bh])
    assert rca == 0 and rcb == 0
    assert A.allocs > before                      # the batch call's buffers
    for xa, xb in zip(Xa, Xb):
        assert torch.equal(xa, xb)
    H1.close()
    G1.close()
    assert not A.live and A.frees == A.allocs
    H0.close()
    G0.close()
