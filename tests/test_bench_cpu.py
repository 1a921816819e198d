"""Host logic of bench.py (no GPU): the one-GPU refusal and the work-unit
count of a cycle, checked against the oracle's own visit counters."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cycle_work_units_match_oracle_visits():
    import bench
    from oracle import oracle as O
    for side in (64, 256):
        H = O.Hierarchy.lgm(side)
        ns = [H.dims(l)["n"] for l in range(H.num_levels)]
        gammas = [H.dims(l)["gamma"] for l in range(H.num_levels)]
        visits = H.visit_counts()
        want = sum(3 * visits[l] * ns[l] / ns[0] for l in range(H.num_levels - 1))
        assert bench.cycle_work_units(ns, gammas, 3) == want
