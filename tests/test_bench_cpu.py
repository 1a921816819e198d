"""Host logic of bench.py (no GPU): the one-GPU refusal, the work-unit
count of a cycle, checked against the oracle's own visit counters, and the
rule that a recorded HBM traffic figure holds only for the kernel sources and
hub split it was measured on."""
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


class _FakeH:
    """Hub splits of a hierarchy, as bench.recorded_traffic reads them."""

    def __init__(self, ks):
        self._ks = ks
        self.num_levels = len(ks)

    def hub_info(self, l):
        return {"k": self._ks[l]}


def test_recorded_traffic_follows_the_kernel_sources():
    import bench
    t = dict(bench.TRAFFIC["chung_lu_2p20"])
    saved = bench.TRAFFIC["chung_lu_2p20"]
    H = _FakeH(t["hub_split"])
    try:
        # the record holds while the kernel sources hash to its digest ...
        bench.TRAFFIC["chung_lu_2p20"] = dict(t, kernel_sha=bench.kernel_source_hash(t["source"]))
        assert bench.recorded_traffic("chung_lu_2p20", H) == t["bytes_per_launch"]
        # ... and lapses when a source changes or the hub split differs
        bench.TRAFFIC["chung_lu_2p20"] = dict(t, kernel_sha="0" * 16)
        assert bench.recorded_traffic("chung_lu_2p20", H) is None
        bench.TRAFFIC["chung_lu_2p20"] = dict(t, kernel_sha=bench.kernel_source_hash(t["source"]))
        assert bench.recorded_traffic("chung_lu_2p20", _FakeH([0, 0])) is None
    finally:
        bench.TRAFFIC["chung_lu_2p20"] = saved
    assert bench.recorded_traffic("no_such_workload", H) is None
    # the digest covers every listed file, in order
    assert bench.kernel_source_hash(["lamg_relax.hpp"]) != bench.kernel_source_hash(t["source"])
