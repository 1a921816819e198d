"""LAMG solve benchmark on one MI355X.

One step = one complete solve of A x = b to a relative residual of 1e-8 on
the Chung-Lu power-law graph (n0 = 2^20, exponent 2.1, mean degree 16,
largest component, weights U[0.1, 1], one zero-sum N(0,1) right-hand side),
with the hierarchy built once beforehand (setup is reported separately).
The FP64 path is the headline; FP32 cycles with FP64 refinement are timed on
the same hierarchy and reported beside it.

value = edges * cycles / second over the timed steps (edges = m of the input
graph); GB/s = algorithmic bytes of the timed cycles / time.  The roofline
object covers the dominant kernel (the multicolour Gauss-Seidel relaxation),
timed live with HIP events on the solve stream around each run of its
back-to-back launches (one span per sweep's launched colours, behind a
bounded wait kernel that lets the host queue the span's launches first), in
a second pass over the same solves that launches the cycle eagerly; kernel
shares are kernel time over the wall time of the plain solves.  Beside the
two-level headline, a multilevel graph (RGG 2^20) is solved with per-kernel
spans; the CPU oracle runs on the headline's own graph and right-hand side.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="chung_lu_2p20",
                   choices=["chung_lu_2p20", "grid2d_64", "rgg_2p20", "grid3d_128_k32", "graph_batch_256", "lgm_1024",
                            "negative_grid_1024"])
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--no-multilevel", action="store_true",
                   help="skip the multilevel (RGG 2^20) solve timed beside the Chung-Lu headline")
    p.add_argument("--eigs", type=int, default=4,
                   help="lowest eigenpairs timed beside the solve on the same hierarchy (0: skip)")
    p.add_argument("--copy-bytes", type=int, default=0,
                   help="only run a plain device copy of this many bytes (HBM counter calibration) and exit")
    return p.parse_args()


def copy_calibration(nbytes):
    """A plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of its
    dispatches against nbytes give the counters' scale."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 8, "launches": 3}), flush=True)


# HBM traffic of the relaxation kernel from hardware counters (rocprofv3
# --pmc FETCH_SIZE, then WRITE_SIZE, on this benchmark), scaled by the same
# counters on a plain copy; valid only while the kernel source is unchanged
# and, where recorded, the levels split their colours at the same hub colour
# (the split sets which colours the kernel's launches cover).
TRAFFIC = {
    # profiles/gs_fp64_chung_lu_2p20.md: FETCH_SIZE 12068.9 KiB x 1.9999 + WRITE_SIZE 228.8 KiB x 1.0000
    "chung_lu_2p20": {"bytes_per_launch": 24950581, "kernel_sha": "845c5036e8e18a77",
                      "source": ["lamg_relax.hpp", "lamg_device.hpp"], "hub_split": [24, 27]},
    # profiles/mv_grid3d_128_k32.md: k_relax_mv<float, 0, 4>, FETCH_SIZE 6463.9 KiB x 1.9999 + WRITE_SIZE 1625.6 KiB x 1.0
    "grid3d_128_k32": {"bytes_per_launch": 14902339, "kernel_sha": "6e584f88a5ee283d",
                       "source": ["lamg_mv.hip", "lamg_device.hpp"]},
}


def kernel_source_hash(names=("lamg_relax.hpp", "lamg_device.hpp")):
    """First 16 hex digits of the sha256 of the named kernel sources, read in
    the order given (the kernel file and the device helpers it inlines)."""
    import hashlib
    h = hashlib.sha256()
    for name in ([names] if isinstance(names, str) else names):
        with open(os.path.join(ROOT, "paper_1108_1310_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, H):
    t = TRAFFIC.get(workload)
    if not t or t["kernel_sha"] != kernel_source_hash(t["source"]):
        return None
    if "hub_split" in t and [H.hub_info(l)["k"] for l in range(H.num_levels)] != t["hub_split"]:
        return None
    return t["bytes_per_launch"]


def workload(name):
    from paper_1108_1310_amd import workloads as W
    g, b = W.config(name)
    return g, b


def timed_solves(H, b, precision, steps, warmup, lamg, instrument=False):
    """Time `steps` full solves.  Plain runs replay the captured cycle graphs;
    instrumented runs launch every kernel eagerly with a HIP event pair (same
    stream) around each run of back-to-back relaxation launches (one span per
    sweep's launched colours, behind a bounded wait that lets the host queue
    the span first), which yields the kernel's summed duration, launch count
    and algorithmic bytes."""
    import torch
    H.set_solve_options(precision=precision)
    for _ in range(warmup):
        H.solve(b)
    torch.cuda.synchronize()
    kid = 0 if precision == lamg.FP64 else 2
    lamg.prof_enable(instrument)
    cycles, byts, worst, acf = 0, 0, 0.0, 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info = H.solve(b)
        acf = info["acf"]
        cycles += info["cycles"]
        byts += info["bytes_moved"]
        worst = max(worst, info["rel_residual"])
        if info["status"] != 0:
            raise RuntimeError(f"solve status {info['status']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = lamg.prof_read(kid)
    hub = lamg.prof_read(8 if precision == lamg.FP64 else 9)
    lamg.prof_enable(False)
    return dict(seconds=dt, cycles=cycles, bytes=byts, rel_residual=worst, acf=acf, prof=prof, hub=hub, x=x)


def mvm_time_us(H, lamg, reps=20):
    """Time of one finest-level FP64 matrix-vector product (r = b - A x over
    the finest CSR, the residual kernel of the solve), the paper's work unit
    (Section 5.1): kernel time from the instrumentation spans."""
    import torch
    L = H.level(0)
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    rp, ci, val, dg = d(L["rp"], torch.int32), d(L["ci"], torch.int32), d(L["val"]), d(L["diag"])
    x = torch.randn(H.n, dtype=torch.float64, device="cuda")
    bb = torch.randn(H.n, dtype=torch.float64, device="cuda")
    lamg.residual(rp, ci, val, dg, bb, x)
    torch.cuda.synchronize()
    lamg.prof_enable(True)
    for _ in range(reps):
        lamg.residual(rp, ci, val, dg, bb, x)
    torch.cuda.synchronize()
    p = lamg.prof_read(1)
    lamg.prof_enable(False)
    return 1e3 * p["ms"] / max(1, p["launches"])


def timed_multi(H, B, precision, steps, warmup, lamg, instrument=False):
    """Time `steps` multi-vector solves of all columns of B (one hierarchy)."""
    import torch
    H.set_solve_options(precision=precision)
    for _ in range(warmup):
        H.solve_multi(B)
    torch.cuda.synchronize()
    kid = 4 if precision == lamg.FP64 else 6
    lamg.prof_enable(instrument)
    cycles, col_cycles, byts, worst = 0, 0, 0, 0.0
    t0 = time.perf_counter()
    for i in range(steps):
        X, info, cols, rc = H.solve_multi(B)
        if rc != 0:
            raise RuntimeError(f"multi-vector solve status {rc}")
        print(f"[bench] multi-vector solve {i + 1}/{steps}: {info['cycles']} cycles", file=sys.stderr, flush=True)
        cycles += info["cycles"]
        col_cycles += int(cols["cycles"].sum())
        byts += info["bytes_moved"]
        worst = max(worst, info["rel_residual"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = lamg.prof_read(kid)
    lamg.prof_enable(False)
    return dict(seconds=dt, cycles=cycles, col_cycles=col_cycles, bytes=byts, rel_residual=worst, prof=prof, x=X)


def main_multi(a, g, B):
    """Multi-vector workload: k right-hand sides as one n x k batch on one
    hierarchy.  FP32 cycles with FP64 refinement are the headline for this
    configuration; plain FP64 multi-vector solves are timed beside them."""
    import torch
    from paper_1108_1310_amd import lamg
    k = B.shape[1]
    Bd = torch.tensor(B, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = lamg.Hierarchy(g.n, g.eu, g.ev, g.w)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    print(f"[bench] setup {setup_ms:.1f} ms, {H.num_levels} levels", file=sys.stderr, flush=True)
    r32 = timed_multi(H, Bd, lamg.FP32_REFINE, a.steps, a.warmup, lamg)
    print(f"[bench] mv fp32+refine {r32['seconds']:.3f}s cycles={r32['cycles']}", file=sys.stderr, flush=True)
    i32 = timed_multi(H, Bd, lamg.FP32_REFINE, a.steps, 0, lamg, instrument=True)
    print(f"[bench] mv fp32+refine instrumented {i32['seconds']:.3f}s", file=sys.stderr, flush=True)
    r64 = timed_multi(H, Bd, lamg.FP64, a.steps, a.warmup, lamg)
    print(f"[bench] mv fp64 {r64['seconds']:.3f}s cycles={r64['cycles']}", file=sys.stderr, flush=True)
    x64 = r64["x"]
    err = float(torch.linalg.norm(r32["x"] - x64) / torch.linalg.norm(x64))
    p = i32["prof"]
    achieved = p["bytes"] / (p["ms"] * 1e6) if p["ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(a.workload, H),
                "kernel": "k_relax_mv<float,0,4> (multi-vector multicolour GS, FP32)",
                "avg_launch_us": 1e3 * p["ms"] / max(1, p["launches"]), "launches": p["launches"],
                "bytes_per_launch": p["bytes"] / max(1, p["launches"]),
                # kernel time over the wall time of the plain (graph-replayed) solves
                "kernel_share_of_step": p["ms"] / (r32["seconds"] * 1e3),
                "instrumented_ms_per_step": i32["seconds"] * 1e3 / a.steps}
    cpu = None
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.workload)
    value = g.m * k * r32["cycles"] / r32["seconds"]
    rec = {
        "metric": "edges*cycles/s to 1e-8 rel. residual (multi-vector: edges x columns x cycles; FP32+refine, FP64 beside)",
        "value": value,
        "unit": "edges*cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["seconds"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": g.n, "m": g.m, "k": k, "precision": "fp32+fp64-refine",
                   "tol": 1e-8, "levels": H.num_levels, "setup_ms": setup_ms},
        "gbps": r32["bytes"] / r32["seconds"] / 1e9,
        "cycles_per_solve": r32["cycles"] / a.steps,
        "column_cycles_per_solve": r32["col_cycles"] / a.steps,
        "rel_residual": r32["rel_residual"],
        "err_vs_fp64": err,
        "fp64": {"value": g.m * k * r64["cycles"] / r64["seconds"], "ms_per_step": r64["seconds"] * 1e3 / a.steps,
                 "cycles_per_solve": r64["cycles"] / a.steps, "gbps": r64["bytes"] / r64["seconds"] / 1e9,
                 "rel_residual": r64["rel_residual"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def main_batch(a):
    """Many-graph workload: 256 independent uneven graphs, one right-hand side
    each, solved in one persistent launch per step (FP64 and FP32+refine);
    the same graphs solved one after another with the multi-launch cycle are
    timed once beside it."""
    import torch
    from paper_1108_1310_amd import lamg, workloads as W
    gs = W.graph_batch()
    bs = [torch.tensor(W.rhs_normal(g.n, 1, 1000 + i), device="cuda") for i, g in enumerate(gs)]
    m_tot = sum(g.m for g in gs)
    n_tot = sum(g.n for g in gs)
    print(f"[bench] batch of {len(gs)} graphs: n={n_tot} m={m_tot}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = [lamg.Hierarchy(g.n, g.eu, g.ev, g.w) for g in gs]
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    print(f"[bench] setup {setup_ms:.1f} ms", file=sys.stderr, flush=True)
    res = {}
    for prec in (lamg.FP64, lamg.FP32_REFINE):
        for h in hs:
            h.set_solve_options(precision=prec)
        for _ in range(a.warmup):
            lamg.solve_batch(hs, bs)  # the first call also autotunes the launch
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        edge_cycles, byts, worst, cyc = 0, 0, 0.0, 0
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(a.steps):
            X, infos, rc = lamg.solve_batch(hs, bs)
            if rc != 0:
                raise RuntimeError(f"batch status {rc}")
            edge_cycles += sum(g.m * i["cycles"] for g, i in zip(gs, infos))
            byts += sum(i["bytes_moved"] for i in infos)
            worst = max(worst, max(i["rel_residual"] for i in infos))
            cyc += sum(i["cycles"] for i in infos)
        ev1.record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = dict(seconds=dt, event_ms=ev0.elapsed_time(ev1), edge_cycles=edge_cycles, bytes=byts, worst=worst,
                         cycles=cyc, X=X)
        print(f"[bench] batch precision={prec} {dt:.3f}s", file=sys.stderr, flush=True)
    # the same graphs one after another (multi-launch single solves), FP64
    for h in hs:
        h.set_solve_options(precision=lamg.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_ec = 0
    for g, h, b in zip(gs, hs, bs):
        x, i = h.solve(b)
        seq_ec += g.m * i["cycles"]
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    print(f"[bench] sequential fp64 {seq:.3f}s", file=sys.stderr, flush=True)
    r64, r32 = res[lamg.FP64], res[lamg.FP32_REFINE]
    achieved = r64["bytes"] / (r64["event_ms"] * 1e6)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_batch (persistent many-graph solve, FP64)",
                "avg_launch_us": 1e3 * r64["event_ms"] / a.steps, "launches": a.steps,
                "bytes_per_launch": r64["bytes"] / a.steps}
    cpu = None
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.workload)
    rec = {
        "metric": "edges*cycles/s to 1e-8 rel. residual (sum over the batch's graphs; FP64, FP32+refine beside)",
        "value": r64["edge_cycles"] / r64["seconds"],
        "unit": "edges*cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["seconds"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "graphs": len(gs), "n": n_tot, "m": m_tot, "precision": "fp64",
                   "tol": 1e-8, "setup_ms": setup_ms},
        "gbps": r64["bytes"] / r64["seconds"] / 1e9,
        "cycles_per_graph": r64["cycles"] / (a.steps * len(gs)),
        "rel_residual": r64["worst"],
        "fp32_refine": {"value": r32["edge_cycles"] / r32["seconds"], "ms_per_step": r32["seconds"] * 1e3 / a.steps,
                        "gbps": r32["bytes"] / r32["seconds"] / 1e9, "rel_residual": r32["worst"]},
        "sequential_fp64": {"value": seq_ec / seq, "ms": seq * 1e3},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def adjoint_step(g, b, steps, warmup):
    """One gradient evaluation of the differentiable solve: setup on the
    weights, forward solve, loss = sum of x^2 on the held-out nodes, backward
    (adjoint solve on the same hierarchy + edge-gradient kernel)."""
    import torch
    from paper_1108_1310_amd import lamg, workloads as W
    _, hold = W.label_split(g.n)
    d = lambda a, t=torch.float64: torch.tensor(a, dtype=t, device="cuda")
    eu, ev, bt, ht = d(g.eu, torch.int32), d(g.ev, torch.int32), d(b), torch.tensor(hold, device="cuda")

    def one():
        wt = d(g.w).requires_grad_(True)
        x = lamg.laplacian_solve(bt, wt, eu, ev, g.n)
        (x[ht] ** 2).sum().backward()
        return wt.grad

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gw = one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"ms_per_gradient": dt * 1e3 / steps, "includes": "setup + forward solve + adjoint solve + edge gradient",
            "grad_norm": float(torch.linalg.norm(gw))}


CPU_MIN_S = 10.0  # timed oracle solve work per baseline (right-hand sides added until reached)


def _oracle_rhs_loop(H, g, rhs, max_solves):
    """Solve seeded right-hand sides rhs(j) one after another on the oracle
    hierarchy until CPU_MIN_S of solve time (or max_solves); setup untimed.
    Returns the solve time, cycles, solves and mean digits gained."""
    dt, cyc, k, dig = 0.0, 0, 0, 0.0
    while dt < CPU_MIN_S and k < max_solves:
        b = rhs(k)
        t0 = time.perf_counter()
        x, info, _ = H.solve(b)
        dt += time.perf_counter() - t0
        cyc += info["cycles"]
        dig += -math.log10(max(info["rel_residual"], 1e-300))
        k += 1
    return dt, cyc, k, dig / max(1, k)


def host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def copy_ceiling_gbps():
    """Measured device-copy bandwidth (1 GiB read + 1 GiB written per copy):
    the practical HBM ceiling beside the 8 TB/s spec."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * a.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e6)
    del a, b
    torch.cuda.empty_cache()
    return gbps


def cpu_baseline_same_input(name, gpu_cycles=None):
    """The CPU reference (serial C++) on the benchmark's own input: the same
    graph and right-hand side, setup untimed, one FP64 solve to 1e-8 timed
    (its cycle count is compared with the GPU's).  The half-size sample of
    the same recipe (several right-hand sides) is reported beside it."""
    from oracle import oracle as O
    from paper_1108_1310_amd import workloads as W
    g, b = W.config(name)
    b = b.reshape(-1)
    t0 = time.perf_counter()
    H = O.Hierarchy(g.n, g.eu, g.ev, g.w)
    setup_s = time.perf_counter() - t0
    print(f"[bench] cpu oracle setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    x, info, _ = H.solve(b)
    dt = time.perf_counter() - t0
    A0 = H.level(0).A
    xr, br = W.rhs_normal(g.n, 1, 7), W.rhs_normal(g.n, 1, 8)
    O.residual(A0, br, xr)
    t1 = time.perf_counter()
    for _ in range(3):
        O.residual(A0, br, xr)
    mvm_s = (time.perf_counter() - t1) / 3
    digits = -math.log10(max(info["rel_residual"], 1e-300))
    del H
    half = cpu_baseline("chung_lu_2p19")
    return {"value": g.m * info["cycles"] / dt, "unit": "edges*cycles/s", "cores": 1, "kind": "oracle",
            "sample": "the benchmark's own graph and right-hand side, one FP64 solve to 1e-8, 1 thread "
                      "(setup not timed)",
            "cycles": info["cycles"], "gpu_cycles": gpu_cycles,
            "cycles_match": gpu_cycles is None or int(round(gpu_cycles)) == info["cycles"],
            "rel_residual": info["rel_residual"], "solve_s": dt, "edges": g.m, "host": host_cpu(),
            "setup_s": setup_s, "mvm_ms": mvm_s * 1e3, "setup_mvm": setup_s / mvm_s,
            "solve_mvm_per_digit": dt / mvm_s / digits, "half_size_sample": half}


def cpu_baseline(name, gpu_cycles=None):
    """The CPU reference (serial C++) on a bounded sample of the same workload
    recipe: seeded right-hand sides solved one after another until about
    CPU_MIN_S seconds of solve work (the Chung-Lu headline: its own input)."""
    from oracle import oracle as O
    from paper_1108_1310_amd import workloads as W
    if name == "graph_batch_256":
        gs = W.graph_batch()[:24]
        Hs = [O.Hierarchy(g.n, g.eu, g.ev, g.w) for g in gs]
        dt, ec, k = 0.0, 0, 0
        while dt < CPU_MIN_S and k < 64:
            for i, (g, H) in enumerate(zip(gs, Hs)):
                t0 = time.perf_counter()
                x, info, _ = H.solve(W.rhs_normal(g.n, 1, 1000 + i + 7919 * k))
                dt += time.perf_counter() - t0
                ec += g.m * info["cycles"]
            k += 1
        sample = (f"the first 24 graphs of the batch, {k} right-hand side(s) each, FP64 solves to 1e-8 one after "
                  "another, 1 thread (setup not timed)")
        return {"value": ec / dt, "unit": "edges*cycles/s", "cores": 1, "kind": "oracle", "sample": sample,
                "solve_s": dt, "host": host_cpu()}
    if name == "chung_lu_2p20":
        return cpu_baseline_same_input(name, gpu_cycles)
    if name == "chung_lu_2p19":
        g = W.chung_lu(1 << 19)
        seed, what, cap = W.SEEDS["chung_lu"], "Chung-Lu recipe at n0 = 2^19 (half the workload)", 64
    elif name == "rgg_2p20":
        g = W.rgg(1 << 19)
        seed, what, cap = W.SEEDS["rgg"], "RGG recipe at 2^19 points (half the workload)", 64
    elif name == "grid3d_128_k32":
        g = W.grid3d_aniso(64)
        seed, what, cap = W.SEEDS["grid3d_aniso"], "anisotropic 3D grid recipe at 64^3 (1/8 of the workload)", 32
    else:
        g, _ = W.config(name)
        seed, what, cap = 0, "full workload", 4096
    t0 = time.perf_counter()
    if name == "lgm_1024":
        H = O.Hierarchy.lgm(1024)
    else:
        neg = name == "negative_grid_1024"
        H = O.Hierarchy(g.n, g.eu, g.ev, g.w, allow_negative=1 if neg else 0, ec=1 if neg else 0)
    setup_s = time.perf_counter() - t0
    dt, cyc, k, dig = _oracle_rhs_loop(H, g, lambda j: W.rhs_normal(g.n, 1, seed + 7919 * j), cap)
    # the oracle's finest-level matrix-vector product (its residual), the paper's work unit
    A0 = H.level(0).A
    xr, br = W.rhs_normal(g.n, 1, seed + 1), W.rhs_normal(g.n, 1, seed + 2)
    O.residual(A0, br, xr)
    t0 = time.perf_counter()
    for _ in range(5):
        O.residual(A0, br, xr)
    mvm_s = (time.perf_counter() - t0) / 5
    sample = f"{what}, {k} seeded right-hand side(s) solved one after another, FP64 to 1e-8, 1 thread (setup not timed)"
    return {"value": g.m * cyc / dt, "unit": "edges*cycles/s", "cores": 1, "kind": "oracle", "sample": sample,
            "cycles": cyc, "solves": k, "solve_s": dt, "edges": g.m, "host": host_cpu(),
            "setup_s": setup_s, "mvm_ms": mvm_s * 1e3, "setup_mvm": setup_s / mvm_s,
            "solve_mvm_per_digit": dt / k / mvm_s / dig}


def negative_grid_table(lamg):
    """The four 1024 x 1024 grid Laplacians of the paper's negative-weight
    table (ACF 0.216, 0.262, 0.816, 0.870 there): one untimed solve each with
    the default cycle (iterate recombination) and with the flat correction."""
    import torch
    from paper_1108_1310_amd import workloads as W
    out = {}
    for case in "abcd":
        g = W.grid_stencil(1024, case)
        b = torch.tensor(W.rhs_normal(g.n, 1, W.SEEDS["negative"]), device="cuda")
        row = {"m": g.m}
        for tag, kw in (("default", {}), ("flat_mu", dict(ec=lamg.EC_FLAT_MU, max_cycles=400))):
            H = lamg.Hierarchy(g.n, g.eu, g.ev, g.w, allow_negative_weights=1, **kw)
            t0 = time.perf_counter()
            x, info = H.solve(b, check=False)
            torch.cuda.synchronize()
            row[tag] = {"levels": H.num_levels, "cycles": info["cycles"], "acf": info["acf"],
                        "rel_residual": info["rel_residual"], "status": info["status"],
                        "ms": 1e3 * (time.perf_counter() - t0)}
            H.close()
        out[case] = row
        print(f"[bench] table case {case}: {row}", file=sys.stderr, flush=True)
    return out


def eigs_step(H, g, k, lamg, precision):
    """The eigensolver (LOBPCG preconditioned by one LAMG cycle, run in
    `precision`) on the workload's hierarchy: one untimed call, then one
    timed call from the same seeded block.  No CPU leg: the dense
    eigen-decomposition the oracle uses does not fit graphs of this size."""
    import torch
    from paper_1108_1310_amd import workloads as W
    x0 = torch.tensor(W.rhs_normal(g.n, k, seed=101), device="cuda")
    prec = H.opts.precision
    H.set_solve_options(precision=precision)
    H.eigs(k, x0, tol=1e-8, max_iter=500, cycles=1, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, X, info = H.eigs(k, x0, tol=1e-8, max_iter=500, cycles=1, check=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    H.set_solve_options(precision=prec)
    return {"k": k, "tol": 1e-8, "cycle": "fp64" if precision == lamg.FP64 else "fp32+refine", "status": lamg.lib().lamg_status_str(info["status"]).decode(),
            "iterations": info["iters"], "ms": ms,
            "ms_per_iteration": ms / max(1, info["iters"]), "eigenvalues": [float(v) for v in ev],
            "rel_residuals": [float(v) for v in info["resid"]]}


def eigs_cpu_sample(k, lamg, n0=1 << 12):
    """The eigenpair oracle (dense Laplacian, full symmetric eigendecomposition,
    one BLAS thread) on a bounded sample: a Chung-Lu graph of the workload's
    recipe at n0 = 2^12, beside the GPU eigensolver on the same graph."""
    from threadpoolctl import threadpool_limits
    from oracle import eigs as OE
    from paper_1108_1310_amd import workloads as W
    gs = W.chung_lu(n0)
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        lam, _, _ = OE.lowest_eigenpairs(OE.dense_laplacian(gs.n, gs.eu, gs.ev, gs.w), k)
    cpu_ms = (time.perf_counter() - t0) * 1e3
    Hs = lamg.Hierarchy(gs.n, gs.eu, gs.ev, gs.w)
    e = eigs_step(Hs, gs, k, lamg, lamg.FP64)
    Hs.close()
    rel = max(abs(x - y) / y for x, y in zip(e["eigenvalues"], lam))
    return {"kind": "oracle", "sample": f"Chung-Lu recipe at n0 = 2^12 (n = {gs.n}), dense eigh, k = {k}",
            "cores": 1, "ms": cpu_ms, "gpu_ms_same_sample": e["ms"], "gpu_iterations": e["iterations"],
            "max_rel_eigenvalue_diff": rel}


def cycle_work_units(ns, gammas, nu):
    """Relaxation work of one cycle in finest-level sweeps: nu sweeps per body
    of every level above the coarsest, times its visits (the fractional
    cycle index of each level: body c of level l visits level l+1
    ceil((c+1) gamma_l) - ceil(c gamma_l) times), scaled by n_l / n_0."""
    L = len(ns)
    count, visits = [0] * L, [0] * L

    def body(l):
        visits[l] += 1
        if l == L - 1:
            return
        c = count[l]
        count[l] += 1
        th = math.ceil((c + 1) * gammas[l]) - math.ceil(c * gammas[l])
        for _ in range(th if l + 1 < L - 1 else 1):
            body(l + 1)

    body(0)
    return sum(nu * visits[l] * ns[l] / ns[0] for l in range(L - 1))


def main():
    a = parse()
    if a.copy_bytes:
        return copy_calibration(a.copy_bytes)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1108_1310_amd import lamg
    torch.cuda.set_device(0)
    print(f"[bench] generating {a.workload}", file=sys.stderr, flush=True)
    if a.workload == "graph_batch_256":
        return main_batch(a)
    g, b = workload(a.workload)
    if b.ndim == 2 and b.shape[1] > 1:
        print(f"[bench] n={g.n} m={g.m} k={b.shape[1]}", file=sys.stderr, flush=True)
        return main_multi(a, g, b)
    b = b.reshape(-1)
    bd = torch.tensor(b, device="cuda")
    print(f"[bench] setup n={g.n} m={g.m}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if a.workload == "lgm_1024":
        H = lamg.Hierarchy.lgm(1024)  # geometric hierarchy of the same periodic grid
    else:
        # negative weights: iterate recombination stalls on most right-hand
        # sides of this problem (oracle and GPU alike), so the timed solve
        # uses the flat energy correction
        neg = a.workload == "negative_grid_1024"
        H = lamg.Hierarchy(g.n, g.eu, g.ev, g.w, allow_negative_weights=1 if neg else 0,
                           ec=lamg.EC_FLAT_MU if neg else lamg.EC_RECOMBINE)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    levels = [H.dims(l) for l in range(H.num_levels)]
    print(f"[bench] setup {setup_ms:.1f} ms, {len(levels)} levels", file=sys.stderr, flush=True)

    r64 = timed_solves(H, bd, lamg.FP64, a.steps, a.warmup, lamg)
    print(f"[bench] fp64 {r64['seconds']:.3f}s cycles={r64['cycles']}", file=sys.stderr, flush=True)
    i64 = timed_solves(H, bd, lamg.FP64, a.steps, 0, lamg, instrument=True)
    print(f"[bench] fp64 instrumented {i64['seconds']:.3f}s", file=sys.stderr, flush=True)
    out32 = None
    if not a.no_fp32:
        r32 = timed_solves(H, bd, lamg.FP32_REFINE, a.steps, a.warmup, lamg)
        i32 = timed_solves(H, bd, lamg.FP32_REFINE, a.steps, 0, lamg, instrument=True)
        x64 = r64["x"].double()
        err = float(torch.linalg.norm(r32["x"] - x64) / torch.linalg.norm(x64))
        out32 = {"value": g.m * r32["cycles"] / r32["seconds"], "ms_per_step": r32["seconds"] * 1e3 / a.steps,
                 "cycles_per_solve": r32["cycles"] / a.steps, "gbps": r32["bytes"] / r32["seconds"] / 1e9,
                 "rel_residual": r32["rel_residual"], "err_vs_fp64": err,
                 "gs_kernel": {"gbps": i32["prof"]["bytes"] / (i32["prof"]["ms"] * 1e6) if i32["prof"]["ms"] else None,
                               "avg_us": 1e3 * i32["prof"]["ms"] / max(1, i32["prof"]["launches"]),
                               "launches_per_step": i32["prof"]["launches"] / a.steps}}
        print(f"[bench] fp32+refine {r32['seconds']:.3f}s cycles={r32['cycles']}", file=sys.stderr, flush=True)

    p = i64["prof"]
    achieved = p["bytes"] / (p["ms"] * 1e6) if p["ms"] > 0 else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
                "traffic": recorded_traffic(a.workload, H),
                "kernel": "k_relax<double,0> (multicolour GS)" if achieved is not None else
                          "none: every level runs in the single-workgroup tail (latency-bound)",
                "avg_launch_us": 1e3 * p["ms"] / max(1, p["launches"]), "launches": p["launches"],
                "bytes_per_launch": p["bytes"] / max(1, p["launches"]),
                # kernel time over the wall time of the plain (graph-replayed) solves
                "kernel_share_of_step": p["ms"] / (r64["seconds"] * 1e3),
                "instrumented_ms_per_step": i64["seconds"] * 1e3 / a.steps}
    hb = i64["hub"]
    if hb["launches"] > 0:
        # the hub colours of every sweep (partial-sum launch + single-workgroup phases)
        roofline["hub_sweep"] = {"ms_per_step": hb["ms"] / a.steps, "launches": hb["launches"],
                                 "gbps": hb["bytes"] / (hb["ms"] * 1e6),
                                 "share_of_step": hb["ms"] / (r64["seconds"] * 1e3)}
    mvm_us = mvm_time_us(H, lamg)
    ms64 = r64["seconds"] * 1e3 / a.steps
    digits = -math.log10(max(r64["rel_residual"], 1e-300))
    mvm = {"mvm_us": mvm_us, "solve_mvm": 1e3 * ms64 / mvm_us,
           "solve_mvm_per_digit": 1e3 * ms64 / mvm_us / digits, "digits": digits,
           "setup_mvm": 1e3 * setup_ms / mvm_us}
    ceil = copy_ceiling_gbps()
    roofline["copy_ceiling_gbps"] = ceil
    roofline["frac_of_copy"] = achieved / ceil if achieved is not None else None
    vcyc = None
    if a.workload == "grid2d_64":
        # the literal V(1,2) cycle (gamma = 1) beside the paper's gamma = 1.5
        Hv = lamg.Hierarchy(g.n, g.eu, g.ev, g.w, gamma=1.0)
        rv = timed_solves(Hv, bd, lamg.FP64, a.steps, a.warmup, lamg)
        vcyc = {"gamma": 1.0, "value": g.m * rv["cycles"] / rv["seconds"],
                "ms_per_step": rv["seconds"] * 1e3 / a.steps, "cycles_per_solve": rv["cycles"] / a.steps,
                "acf": rv["acf"], "rel_residual": rv["rel_residual"]}
        Hv.close()
    lgm = None
    if a.workload == "lgm_1024":
        # convergence factor per unit of work (one finest relaxation sweep)
        W = cycle_work_units([d["n"] for d in levels], [d["gamma"] for d in levels],
                             H.opts.nu_pre + H.opts.nu_post)
        lgm = {"work_units_per_cycle": W, "acf": r64["acf"], "factor_per_work_unit": r64["acf"] ** (1.0 / W),
               "paper_factor_per_work_unit": 0.5}
    table = None
    if a.workload == "negative_grid_1024":
        table = negative_grid_table(lamg)
    adj = None
    if a.workload == "rgg_2p20":
        adj = adjoint_step(g, b, a.steps, a.warmup)
        print(f"[bench] gradient {adj['ms_per_gradient']:.1f} ms", file=sys.stderr, flush=True)
    eig = None
    if a.eigs > 0 and a.workload not in ("lgm_1024", "negative_grid_1024"):
        eig = {}
        for prec, key in ((lamg.FP64, "fp64_cycle"), (lamg.FP32_REFINE, "fp32_cycle")):
            e = eigs_step(H, g, a.eigs, lamg, prec)
            e["mvm_units"] = 1e3 * e["ms"] / mvm_us
            eig[key] = e
            print(f"[bench] eigs ({key}) {e['ms']:.1f} ms, {e['iterations']} iterations", file=sys.stderr, flush=True)
        if not a.no_cpu:
            eig["cpu_baseline"] = eigs_cpu_sample(a.eigs, lamg)
            print(f"[bench] eigs oracle sample {eig['cpu_baseline']}", file=sys.stderr, flush=True)
    ml = None
    if a.workload == "chung_lu_2p20" and not a.no_multilevel:
        ml = multilevel_rgg(a, lamg)
    cpu = None
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.workload, r64["cycles"] / a.steps)
    value = g.m * r64["cycles"] / r64["seconds"]
    rec = {
        "metric": "edges*cycles/s to 1e-8 rel. residual (FP64; FP32+refine beside)",
        "value": value,
        "unit": "edges*cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["seconds"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": g.n, "m": g.m, "precision": "fp64", "tol": 1e-8,
                   "energy_correction": "flat_mu" if H.opts.ec == lamg.EC_FLAT_MU else "recombination",
                   "levels": len(levels), "setup_ms": setup_ms},
        "gbps": r64["bytes"] / r64["seconds"] / 1e9,
        "cycles_per_solve": r64["cycles"] / a.steps,
        "acf": r64["acf"],
        "rel_residual": r64["rel_residual"],
        "edges_solved_per_s": g.m * a.steps / r64["seconds"],
        "mvm_units": mvm,
        "v_cycle": vcyc,
        "fp32_refine": out32,
        "adjoint": adj,
        "lgm": lgm,
        "negative_grid_table": table,
        "eigs": eig,
        "multilevel_rgg_2p20": ml,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def multilevel_rgg(a, lamg, steps_cap=5):
    """A multilevel workload beside the two-level headline: the random
    geometric graph of 2^20 points (20 levels: aggregation transfers, iterate
    recombination and the single-workgroup tail all run), FP64 solves to 1e-8
    timed as the headline is, then the same solves instrumented with HIP event
    spans per kernel: GS, residual, aggregation restriction and interpolation
    (time, launches, algorithmic bytes) and the tail launches (time only)."""
    import torch
    g, b = workload("rgg_2p20")
    bd = torch.tensor(b.reshape(-1), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = lamg.Hierarchy(g.n, g.eu, g.ev, g.w)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    steps = max(1, min(a.steps, steps_cap))
    r = timed_solves(H, bd, lamg.FP64, steps, 1, lamg)
    print(f"[bench] multilevel rgg_2p20 fp64 {r['seconds']:.3f}s cycles={r['cycles']}", file=sys.stderr, flush=True)
    lamg.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        H.solve(bd)
    torch.cuda.synchronize()
    inst_ms = (time.perf_counter() - t0) * 1e3
    kernels = {}
    for name, kid in (("gs", 0), ("residual", 1), ("restrict_agg", 10), ("interp_agg", 12), ("tail", 14)):
        p = lamg.prof_read(kid)
        kernels[name] = {"ms_per_solve": p["ms"] / steps, "launches_per_solve": p["launches"] / steps,
                         "avg_us": 1e3 * p["ms"] / max(1, p["launches"]),
                         "share_of_step": p["ms"] / (r["seconds"] * 1e3),
                         "gbps": p["bytes"] / (p["ms"] * 1e6) if p["ms"] > 0 and p["bytes"] > 0 else None,
                         "bytes_per_launch": p["bytes"] / max(1, p["launches"]) if p["bytes"] > 0 else None}
    lamg.prof_enable(False)
    cyc = r["cycles"] / steps
    kernels["tail"]["us_per_cycle"] = 1e3 * kernels["tail"]["ms_per_solve"] / max(cyc, 1)
    out = {"workload": "rgg_2p20", "n": g.n, "m": g.m, "levels": H.num_levels, "setup_ms": setup_ms,
           "value": g.m * r["cycles"] / r["seconds"], "unit": "edges*cycles/s",
           "ms_per_solve": r["seconds"] * 1e3 / steps, "cycles_per_solve": cyc, "acf": r["acf"],
           "rel_residual": r["rel_residual"], "gbps": r["bytes"] / r["seconds"] / 1e9,
           "instrumented_ms_per_solve": inst_ms / steps, "kernels": kernels}
    H.close()
    return out


if __name__ == "__main__":
    main()
