"""Benchmark: LSERK4 time stepping of the compressible Navier-Stokes DG residual on the mixed
48^3-cell periodic mesh (414,720 hex/prism/pyramid/tet elements, N = 4, FP64, BR1 lifting,
Lax-Friedrichs flux) on one MI355X.

Reports the paper's performance index (Eq. (2)): PID = wall * #ranks / (#DOF * #steps *
#RK-stages) with #DOF = sum over elements of (N+1)^3 and #ranks = 1 GPU, as DOF-updates/s =
1/PID (the JSON `value`), plus the roofline position of the dominant kernel (device-timed inside
this run) and the FP64 CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import (config_mesh, config_params, node_noise, tgv_primitive,  # noqa: E402
                       time_step)
from workloads.device import tgv_state  # noqa: E402


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(mesh, N, prm, max_seconds=25.0):
    """FP64 oracle residual on a compact sample of the same workload, single-threaded."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle.dg import DGOracle
    t0 = time.time()
    ora = DGOracle(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                   Rgas=prm["R"])
    setup = time.time() - t0
    C = mesh.C
    rng = np.random.Generator(np.random.PCG64(11))
    c0 = rng.integers(0, C, size=3)
    # sample: the elements of one cell and of its 6 face-neighbour cells (compact, so that
    # the gradients of neighbours are shared)
    cells = [c0.copy()]
    for a in range(3):
        for d in (-1, 1):
            c = c0.copy()
            c[a] = (c[a] + d) % C
            cells.append(c)
    cell_ids = {int(c[0] + C * (c[1] + C * c[2])) for c in cells}
    sample = [e for e in np.nonzero(np.isin(mesh.elem_cell, list(cell_ids)))[0]]
    need = set(sample)
    for e in sample:
        need.update(ora.neighbours(e))
    need2 = set(need)
    for e in need:
        need2.update(ora.neighbours(e))
    U = ora.initial_state(tgv_primitive, lambda es: node_noise(1, (N + 1) ** 3, es), elems=sorted(need2))
    # warm the geometry caches, then time one residual of the sample
    for e in need2:
        ora.elem_geo(e)
    t0 = time.time()
    ora.residual(U, elems=sample)
    wall = time.time() - t0
    dof = len(sample) * (N + 1) ** 3
    return dict(value=dof / wall, unit="DOF-updates/s", cores=1, kind="oracle",
                sample=(f"one RK-stage residual of {len(sample)} elements ({dof} DOF) of 7 "
                        f"face-adjacent cells of the 48^3 mesh, NS N=4, incl. the BR1 gradients "
                        f"of their neighbours; {wall:.1f} s single-threaded (setup {setup:.0f} s "
                        f"not timed)"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cells", type=int, default=None, help="override the cube edge (testing)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is design-only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2511_08020_amd import perfmodel
    from paper_2511_08020_amd.binding import PolyDG

    prm = config_params(2)
    N = prm["N"]
    log("building mesh")
    mesh = config_mesh(2, C=args.cells)
    log(f"{mesh.n_elems} elements, types {mesh.type_counts().tolist()}; creating context")
    t0 = time.time()
    dg = PolyDG.from_mesh(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                          R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2))
    log(f"context ready in {time.time() - t0:.1f} s; {dg.n_doubles} stored doubles")
    U = tgv_state(dg, prm["gamma"], prm["mach"])
    K = dg.zeros_state()
    dt = time_step(mesh, N, cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
    stream = dg.stream
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps, dt = {dt:.4e}")
    dg.rk_steps(U, K, dt, args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    dg.rk_steps(U, K, dt, args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = start.elapsed_time(end) * 1e-3
    finite = bool(torch.isfinite(U).all().item())
    dof = mesh.n_elems * (N + 1) ** 3
    stages = 5 * args.steps
    value = dof * stages / wall
    log(f"{args.steps} steps in {wall:.3f} s; PID {1.0 / value:.3e} s; finite={finite}")

    # device-timed kernels: average launch duration per (phase, type) on the context stream
    costs, phase_ms = dg.measure_costs(U, reps=5)
    fl = np.zeros((3, 4))
    by = np.zeros((3, 4))
    for ph in range(3):
        fl[ph], by[ph] = perfmodel.phase_work(ph, dg.elem_type, dg.elem_sides, N, True)
    ph, t = np.unravel_index(np.argmax(phase_ms), phase_ms.shape)
    sec = phase_ms[ph, t] * 1e-3
    t_alu = fl[ph, t] / (perfmodel.PEAK_FP64_TFLOPS * 1e12)
    t_hbm = by[ph, t] / (perfmodel.PEAK_HBM_GBS * 1e9)
    tname = ("hex", "prism", "pyramid", "tet")[t]
    if t_alu >= t_hbm:
        roof = dict(bound="alu", achieved=fl[ph, t] / sec / 1e12, peak=perfmodel.PEAK_FP64_TFLOPS,
                    unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=by[ph, t] / sec / 1e9, peak=perfmodel.PEAK_HBM_GBS,
                    unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = f"{perfmodel.PHASES[ph]}[{tname}] (k_{perfmodel.PHASES[ph]}<{t},{N},NS>)"
    roof["avg_launch_ms"] = float(phase_ms[ph, t])
    stage_ms = float(phase_ms.sum())
    log("phase ms [trace, volume, surface] x [hex, prism, pyr, tet]:\n" + str(np.round(phase_ms, 3)))

    out = {
        "metric": "DOF-updates/s (1/PID, PID = wall*ranks/(DOF*steps*RK-stages)), FP64 NS mixed mesh N=4",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ns_mixed_48c_N4: periodic 48^3-cell cube, 4^3-cell blocks split "
                               "25% each hex/prism/pyramid/tet (414,720 elements), N=4, BR1, LF, "
                               "LSERK4, TGV initial field + 1e-3 noise",
                   "n_elems": int(mesh.n_elems), "dof": int(dof), "N": N, "dt": dt},
        "pid_s": 1.0 / value,
        "state_finite": finite,
        "stage_ms_sum_of_kernels": stage_ms,
        "per_type_cost_s_per_elem": costs.tolist(),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(mesh, N, prm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
