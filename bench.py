"""Benchmark: LSERK4 time stepping of the compressible Navier-Stokes DG residual on the mixed
48^3-cell periodic mesh (414,720 hex/prism/pyramid/tet elements, N = 4, FP64, BR1 lifting,
Lax-Friedrichs flux) on one MI355X.

Reports the paper's performance index (Eq. (2)): PID = wall * #ranks / (#DOF * #steps *
#RK-stages) with #DOF = sum over elements of (N+1)^3 and #ranks = 1 GPU, as DOF-updates/s =
1/PID (the JSON `value`), plus
  roofline      the dominant kernel's algorithmic work per launch (perfmodel.algorithmic_work,
                the phase's share of the method's per-element work) over its average launch
                duration, from HIP events around every kernel of the timed steps; the kernels'
                own formulation count is reported beside it (formulation_frac);
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload, single-threaded and
                on all usable host cores;
  adjoint       the gradient of the kinetic energy after 20 steps with respect to the initial
                state (Navier-Stokes, 24^3-cell mixed mesh, N = 3, checkpoints every 5 steps):
                PID of the whole reverse run;
  batched       64 uneven Euler meshes of degrees 2..6 in one graph launch per step against the
                same problems advanced one after the other;
  imbalance     the 64^3 sphere mesh, N = 5: weighted against unweighted work queues built from
                device-timed per-type costs (Sec. 3, Listing 1), and a dynamic rebalance;
  curved        a 24^3-cell hexahedron/pyramid mesh, N = 4, stepped affine and with trilinear
                (curved) elements: per-node metrics and a mass matrix per element (Alg. 1).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-adjoint]
                       [--no-split] [--no-batched] [--batch-steps S] [--batch-meshes M]
                       [--batch-small] [--no-imbalance] [--imbalance-steps S]
                       [--imbalance-queues 256,4096] [--rebalances R] [--no-curved]
                       [--curved-steps S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import (batched_configs, config_mesh, config_params, make_mesh,  # noqa: E402
                       node_noise, tgv_primitive, time_step)
from workloads.device import tgv_state  # noqa: E402

KERNEL_SOURCES = ("device.h", "phases.h", "kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_08020_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken
    with the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_ns48.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else float(k["fetch_bytes"] + k["write_bytes"])


# ------------------------------------------------------------------------------ CPU oracle
def _oracle_sample(N, prm, block_seed=11):
    """The FP64 oracle on the 48^3 mesh and a compact sample of it: the elements of a 3x3x3 block
    of cells, with a state on them and on two rings of neighbours (the BR1 gradients of the
    neighbours enter the sample's residual)."""
    from oracle.dg import DGOracle
    mesh = config_mesh(2)
    ora = DGOracle(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"], Rgas=prm["R"])
    C = mesh.C
    c0 = np.random.Generator(np.random.PCG64(block_seed)).integers(0, C, size=3)
    cell_ids = set()
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                c = (c0 + np.array([dx, dy, dz])) % C
                cell_ids.add(int(c[0] + C * (c[1] + C * c[2])))
    sample = [int(e) for e in np.nonzero(np.isin(mesh.elem_cell, list(cell_ids)))[0]]
    ring = set(sample)
    for _ in range(2):
        ring |= {nb for e in list(ring) for nb in ora.neighbours(e)}
    U = ora.initial_state(tgv_primitive, lambda es: node_noise(1, (N + 1) ** 3, es), elems=sorted(ring))
    return ora, U, sample


def _time_sample(target_seconds):
    """Single-threaded oracle timing of the sample (the first evaluation, which builds the
    oracle's face and element tables, is not timed): (reps, dof, wall, setup)."""
    from threadpoolctl import threadpool_limits
    prm = config_params(2)
    N = prm["N"]
    with threadpool_limits(limits=1):
        t0 = time.time()
        ora, U, sample = _oracle_sample(N, prm)
        ora.residual(U, elems=sample)
        setup = time.time() - t0
        reps, wall = 0, 0.0
        while wall < target_seconds:
            t1 = time.time()
            ora.residual(U, elems=sample)
            wall += time.time() - t1
            reps += 1
    return reps, len(sample) * (N + 1) ** 3, wall, setup


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(target_seconds=15.0, max_workers=16):
    """The FP64 oracle timed on the host's cores, on a bounded sample of the plain workload (one
    RK-stage residual of a 3x3x3-cell block of the 48^3 mesh, NS N=4): first single-threaded, then
    on all usable cores at once (one single-threaded oracle process per core, each timing the same
    sample for target_seconds); the aggregate is the all-core throughput, and the paper's
    convention PID = wall x cores / (DOF x stages) gives its per-core PID."""
    import subprocess
    reps, dof, wall, setup = _time_sample(target_seconds)
    single = reps * dof / wall
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    workers = max(1, min(usable, max_workers))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(target_seconds)],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env, text=True)
             for _ in range(workers)]
    rates = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode == 0 and out.strip():
            r = json.loads(out.strip().splitlines()[-1])
            rates.append(r["reps"] * r["dof"] / r["wall"])
    agg = float(sum(rates))
    return dict(value=agg, unit="DOF-updates/s", cores=len(rates), kind="oracle",
                sample=(f"one RK-stage residual of the {dof // 125} elements ({dof} DOF) of a 3x3x3-cell "
                        f"block of the 48^3 mesh, NS N=4, incl. the BR1 gradients of their neighbours, "
                        f"repeated for {target_seconds:.0f} s per process; {len(rates)} single-threaded "
                        f"oracle processes at once (one per usable core; table setup not timed)"),
                pid_per_core_s=len(rates) / agg if agg > 0 else None,
                cpu_model=_cpu_model(), nproc=nproc, usable_cores=usable,
                single_thread={"value": single, "unit": "DOF-updates/s", "cores": 1, "reps": reps,
                               "wall_s": wall, "pid_s": 1.0 / single, "setup_s": setup})


# ------------------------------------------------------------------------------ plain form
def run_plain(args, torch, PolyDG, perfmodel):
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
    dg.timing_start()
    start.record(stream)
    dg.rk_steps(U, K, dt, args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = start.elapsed_time(end) * 1e-3
    total_ms, launches = dg.timing_stop()
    finite = bool(torch.isfinite(U).all().item())
    dof = mesh.n_elems * (N + 1) ** 3
    value = dof * 5 * args.steps / wall
    log(f"{args.steps} steps in {wall:.3f} s; PID {1.0 / value:.3e} s; finite={finite}")

    phase_ms = total_ms / np.maximum(launches, 1)
    # algorithmic work per launch (the method's count, perfmodel.algorithmic_*) and the work of
    # the kernels' own formulation (perfmodel.phase_work), per phase and type
    fl = np.zeros((3, 4))
    by = np.zeros((3, 4))
    ffl = np.zeros((3, 4))
    fby = np.zeros((3, 4))
    for ph in range(3):
        fl[ph], by[ph] = perfmodel.algorithmic_phase_work(ph, dg.elem_type, dg.elem_sides, N, True)
        ffl[ph], fby[ph] = perfmodel.phase_work(ph, dg.elem_type, dg.elem_sides, N, True)
    ph, t = np.unravel_index(np.argmax(total_ms), total_ms.shape)
    sec = phase_ms[ph, t] * 1e-3
    kname = f"pdg::k_{perfmodel.PHASES[ph]}<{t}, {N}{', true' if ph else ''}>"
    peak_f, peak_b = perfmodel.PEAK_FP64_TFLOPS, perfmodel.PEAK_HBM_GBS
    if fl[ph, t] / (peak_f * 1e12) >= by[ph, t] / (peak_b * 1e9):
        roof = dict(bound="alu", achieved=fl[ph, t] / sec / 1e12, peak=peak_f, unit="TFLOP/s")
        roof["formulation_frac"] = ffl[ph, t] / sec / 1e12 / peak_f
    else:
        roof = dict(bound="hbm", achieved=by[ph, t] / sec / 1e9, peak=peak_b, unit="GB/s")
        roof["formulation_frac"] = fby[ph, t] / sec / 1e9 / peak_b
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(kname)
    roof["kernel"] = kname
    roof["avg_launch_ms"] = float(phase_ms[ph, t])
    roof["algorithmic_flops_per_launch"] = float(fl[ph, t])
    roof["algorithmic_bytes_per_launch"] = float(by[ph, t])
    roof["formulation_flops_per_launch"] = float(ffl[ph, t])
    roof["formulation_bytes_per_launch"] = float(fby[ph, t])
    roof["launches_timed"] = int(launches[ph, t])
    roof["work_model"] = "algorithmic: per element and RK stage (perfmodel.algorithmic_work), the phase's share"
    # whole stage: algorithmic t* = max(flops at the FP64 peak, bytes at the HBM peak) against
    # the measured time per stage; and the formulation's sum over kernels of max(flop, byte time)
    F_st, B_st, t_star = perfmodel.algorithmic_stage(dg.elem_type, dg.elem_sides, N, True)
    t_form = float(np.maximum(ffl / (peak_f * 1e12), fby / (peak_b * 1e9)).sum())
    stage_s = wall / (5 * args.steps)
    stage_kernel_ms = float(phase_ms.sum())
    log("launch ms [trace, volume, surface] x [hex, prism, pyr, tet]:\n" + str(np.round(phase_ms, 3)))
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
        "launch_ms": {"phases": list(perfmodel.PHASES), "types": ["hex", "prism", "pyramid", "tet"],
                      "avg": np.round(phase_ms, 4).tolist()},
        "stage_roofline": {"algorithmic_gflop": F_st / 1e9, "algorithmic_gb": B_st / 1e9,
                           "t_star_ms": t_star * 1e3, "stage_ms": stage_s * 1e3, "kernels_ms": stage_kernel_ms,
                           "frac": t_star / stage_s, "formulation_gflop": float(ffl.sum()) / 1e9,
                           "formulation_t_star_ms": t_form * 1e3,
                           "formulation_frac": t_form * 1e3 / stage_kernel_ms},
        "roofline": roof,
    }
    del U, K, dg
    return mesh, prm, out


def stage_work(perfmodel, dg, ns):
    """Algorithmic (flops, bytes, t*) of one RK stage of context dg (perfmodel.algorithmic_stage)."""
    return perfmodel.algorithmic_stage(dg.elem_type, dg.elem_sides, dg.N, ns)


# ------------------------------------------------------------------------------ split form
def run_split(args, torch, PolyDG, perfmodel, mesh, prm):
    """The same workload with the entropy-stable split-form volume integral: whole-step rate
    and the dominant split volume kernel against the FP64 vector peak."""
    N = prm["N"]
    dg = PolyDG.from_mesh(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                          R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2), volume_form="split")
    U = tgv_state(dg, prm["gamma"], prm["mach"])
    K = dg.zeros_state()
    dt = time_step(mesh, N, cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
    stream = dg.stream
    dg.rk_steps(U, K, dt, 1)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    dg.timing_start()
    ev[0].record(stream)
    dg.rk_steps(U, K, dt, args.split_steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    wall = ev[0].elapsed_time(ev[1]) * 1e-3
    total_ms, launches = dg.timing_stop()
    phase_ms = total_ms / np.maximum(launches, 1)
    dof = mesh.n_elems * (N + 1) ** 3
    # algorithmic: the weak form's volume phase plus the flux differencing; formulation: the
    # split kernel's own count
    fl, _ = perfmodel.algorithmic_phase_work(1, dg.elem_type, dg.elem_sides, N, True)
    cnt = np.bincount(dg.elem_type, minlength=4)
    fl = fl + cnt * np.array([perfmodel.algorithmic_split_extra(t, N, True) for t in range(4)])
    ffl, _ = perfmodel.phase_work(1, dg.elem_type, dg.elem_sides, N, True, split=True)
    t = int(np.argmax(total_ms[1]))
    sec = phase_ms[1, t] * 1e-3
    ach = fl[t] / sec / 1e12
    out = {"workload": "ns_mixed_48c_N4 with the split-form volume integral (Chandrashekar flux "
                       "on Gauss-Lobatto lines)",
           "steps": args.split_steps, "ms_per_step": wall / args.split_steps * 1e3,
           "value": dof * 5 * args.split_steps / wall, "unit": "DOF-updates/s",
           "finite": bool(torch.isfinite(U).all().item()),
           "volume_launch_ms": np.round(phase_ms[1], 4).tolist(),
           "dominant_volume_kernel": {"kernel": f"pdg::k_volume_split<{t}, {N}, true>",
                                      "avg_launch_ms": float(phase_ms[1, t]),
                                      "algorithmic_flops_per_launch": float(fl[t]),
                                      "achieved_tflops": ach, "peak_tflops": perfmodel.PEAK_FP64_TFLOPS,
                                      "frac": ach / perfmodel.PEAK_FP64_TFLOPS,
                                      "formulation_flops_per_launch": float(ffl[t]),
                                      "formulation_frac": ffl[t] / sec / 1e12 / perfmodel.PEAK_FP64_TFLOPS}}
    log(f"split form: {out['ms_per_step']:.1f} ms/step, volume ms {out['volume_launch_ms']}")
    del U, K, dg
    return out


# --------------------------------------------------------------------------- curved elements
def run_curved(torch, PolyDG, perfmodel, steps, C=24, N=4):
    """Curved elements (per-node metrics, per-face-point normals, a mass-matrix inverse per modal
    element): one periodic C^3-cell mesh of hexahedron and pyramid cells (conforming, seeded),
    stepped affine, with every vertex moved by workloads.deformed, and moving (workloads.motion:
    the geometry and every pyramid's mass matrix rebuilt on the device at each RK stage time),
    NS at N; each run against the affine one and against the affine algorithmic stage t* (the
    extra per-node and per-element tables are not algorithmic work)."""
    import time as _time
    from workloads import deformed, make_mesh, motion
    prm = config_params(2)
    rng = np.random.Generator(np.random.PCG64(5))
    kinds = np.array((0, 2), np.int8)[rng.permutation(np.arange(C ** 3) % 2)]
    base = make_mesh(C, kinds)
    out = {"workload": f"ns_hexpyr_{C}c_N{N}: periodic {C}^3-cell cube, half hexahedron and half "
                       f"pyramid-split cells (seeded), N={N}, BR1, LF, LSERK4, TGV state; curved: every "
                       f"vertex moved by 0.15 h (sin ky sin kz, sin kz sin kx, sin kx sin ky); moving: the "
                       f"curved mesh with corners x0 + 0.1 h (sin k(y+z), sin k(z+x), sin k(x+y)) sin(2 t)",
           "steps": steps}
    curved = deformed(base, 0.15)
    for name, mesh in (("affine", base), ("curved", curved), ("moving", curved)):
        t0 = _time.time()
        dg = PolyDG.from_mesh(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                              R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2))
        if name == "moving":
            dg.set_motion(motion(mesh, 0.1), 2.0)
        setup = _time.time() - t0
        U = tgv_state(dg, prm["gamma"], prm["mach"])
        K = dg.zeros_state()
        dt = time_step(mesh, N, cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
        dg.rk_steps(U, K, dt, 1)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        dg.timing_start()
        ev[0].record(dg.stream)
        dg.rk_steps(U, K, dt, steps)
        ev[1].record(dg.stream)
        torch.cuda.synchronize()
        wall = ev[0].elapsed_time(ev[1]) * 1e-3
        total_ms, launches = dg.timing_stop()
        dof = mesh.n_elems * (N + 1) ** 3
        _, _, t_star = stage_work(perfmodel, dg, True)
        out[name] = {"setup_s": setup, "ms_per_step": wall / steps * 1e3, "pid_s": wall / (dof * steps * 5),
                     "value": dof * 5 * steps / wall, "unit": "DOF-updates/s",
                     "finite": bool(torch.isfinite(U).all().item()),
                     "launch_ms": np.round(total_ms / np.maximum(launches, 1), 4).tolist(),
                     "stage_frac": t_star / (wall / (steps * 5))}
        log(f"curved leg, {name}: {out[name]['ms_per_step']:.1f} ms/step (setup {setup:.1f} s)")
        del U, K
        dg.close()
    out["curved_over_affine"] = out["curved"]["ms_per_step"] / out["affine"]["ms_per_step"]
    out["moving_over_curved"] = out["moving"]["ms_per_step"] / out["curved"]["ms_per_step"]
    return out


# ---------------------------------------------------------------------------- adjoint form
def run_adjoint(torch, PolyDG, perfmodel, steps=20, checkpoint_every=5):
    from paper_2511_08020_amd import autograd as pag
    prm = config_params(4)
    N = prm["N"]
    mesh = config_mesh(4)
    dg = PolyDG.from_mesh(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                          R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2))
    dt = time_step(mesh, N, cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
    U0 = tgv_state(dg, prm["gamma"], prm["mach"])
    wJ = dg.node_weights()
    stream = dg.stream

    def gradient():
        U = U0.clone().requires_grad_(True)
        E = pag.kinetic_energy(dg, pag.rk_solve(dg, U, dt, steps, checkpoint_every), wJ)
        E.backward()
        return U.grad

    gradient()  # warm-up
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    g = gradient()
    b.record(stream)
    torch.cuda.synchronize()
    wall = a.elapsed_time(b) * 1e-3
    # forward stepping alone, for the ratio
    U = U0.clone()
    K = dg.zeros_state()
    a.record(stream)
    dg.rk_steps(U, K, dt, steps)
    b.record(stream)
    torch.cuda.synchronize()
    fwd = a.elapsed_time(b) * 1e-3
    dof = mesh.n_elems * (N + 1) ** 3
    # roofline position: the forward stage's algorithmic work for the forward stages of the run
    # (the checkpointed forward pass and the segment recomputation: 2 x 5 x steps) and, per
    # reverse stage (5 x steps), three forward stages' worth (the recomputed forward quantities
    # plus the transposed volume and face products)
    F_fwd, _, t_fwd = stage_work(perfmodel, dg, True)
    t_star = t_fwd * (2 * 5 * steps + 3 * 5 * steps)
    return {"workload": "ns_mixed_24c_N3_adjoint: 24^3 cells, equal type fractions (51,840 "
                        "elements), N=3; d KE(U_20)/d U_0, checkpoints every 5 steps",
            "value": dof * 5 * steps / wall, "unit": "DOF-updates/s (gradient run)",
            "pid_s": wall / (dof * 5 * steps), "wall_s": wall, "forward_only_s": fwd,
            "gradient_over_forward": wall / fwd, "grad_finite": bool(torch.isfinite(g).all().item()),
            "roofline": {"bound": "alu", "t_star_s": t_star, "frac": t_star / wall,
                         "achieved_tflops": F_fwd * 25 * steps / wall / 1e12,
                         "forward_frac": t_fwd * 5 * steps / fwd,
                         "model": "algorithmic forward stage t* x (2 forward + 3 per reverse stage) x 5 x steps"}}


# ---------------------------------------------------------------------------- batched form
def run_batched(torch, PolyDG, PolyBatch, perfmodel, steps, n_meshes=64, min_edge=8, max_edge=32):
    cfgs = batched_configs(n_meshes, min_edge=min_edge, max_edge=max_edge)
    probs, Us, dts, dofs = [], [], [], 0
    t0 = time.time()
    for c in cfgs:
        mesh = make_mesh(c["C"], c["kinds"])
        dg = PolyDG.from_mesh(mesh, c["N"], p_ref=1.0 / (1.4 * 0.01))
        probs.append(dg)
        Us.append(tgv_state(dg, noise_seed=1 + c["index"]))
        dts.append(time_step(mesh, c["N"]))
        dofs += mesh.n_elems * (c["N"] + 1) ** 3
        if c["index"] % 8 == 7:
            log(f"batched: {c['index'] + 1} problems set up ({time.time() - t0:.0f} s)")
    torch.cuda.synchronize()
    log(f"batched: {n_meshes} problems, {dofs} DOF, set up in {time.time() - t0:.0f} s")
    Ks = [p.zeros_state() for p in probs]
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    # sequential plain solves
    U_seq = [U.clone() for U in Us]
    for p, U, K, dt in zip(probs, U_seq, Ks, dts):
        p.rk_steps(U, K, dt, 1)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for p, U, K, dt in zip(probs, U_seq, Ks, dts):
        p.rk_steps(U, K, dt, steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    seq = ev[0].elapsed_time(ev[1]) * 1e-3
    del U_seq
    batch = PolyBatch(probs, stream=stream)
    t1 = time.time()
    tiles = batch.autotune(Us, Ks, dts, reps=2)
    solo = batch.solo()
    tune_s = time.time() - t1
    log(f"batched: tiles chosen, problems with >= {solo} elements run alone")
    batch.rk_steps(Us, Ks, dts, 1)
    torch.cuda.synchronize()
    ev[0].record(stream)
    batch.rk_steps(Us, Ks, dts, steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    bat = ev[0].elapsed_time(ev[1]) * 1e-3
    finite = all(bool(torch.isfinite(U).all().item()) for U in Us)
    batch.close()
    work = [stage_work(perfmodel, p, False) for p in probs]
    flops = sum(w[0] for w in work) * 5 * steps
    t_star = sum(w[2] for w in work) * 5 * steps
    return {"workload": f"euler_batched_{n_meshes}meshes: cube edges {min_edge}..{max_edge}, "
                        f"Dirichlet type fractions, N in 2..6 (seeded)",
            "dof": int(dofs), "steps": steps,
            "value": dofs * 5 * steps / bat, "unit": "DOF-updates/s",
            "pid_s": bat / (dofs * 5 * steps), "wall_s": bat,
            "sequential_wall_s": seq, "speedup_vs_sequential": seq / bat,
            "tiles": tiles.tolist(), "solo_min_elems": solo, "autotune_s": tune_s, "state_finite": finite,
            "roofline": {"bound": "alu", "t_star_s": t_star, "frac": t_star / bat,
                         "achieved_tflops": flops / bat / 1e12,
                         "model": "sum over problems of the algorithmic stage t* x 5 x steps"}}


# ------------------------------------------------------------------ load balance (config 5)
def run_imbalance(torch, PolyDG, steps, queues=(256,), rebalances=1):
    """Load balance of the work-queue schedule (one workgroup per contiguous segment of the
    Hilbert-ordered elements).  For each queue count: unit weights; then the dynamic loop's
    threshold-triggered rebalance from the per-queue device timers of the previous run, twice;
    and the static split by per-type costs from per-type launch timers.  Each schedule is timed
    over `steps` LSERK4 steps and its measured imbalance read from the queue timers.  The
    per-type launch schedule is timed alongside."""
    prm = config_params(5)
    N = prm["N"]
    mesh = config_mesh(5)
    log(f"imbalance: {mesh.n_elems} elements, types {mesh.type_counts().tolist()}")
    dg = PolyDG.from_mesh(mesh, N, equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                          R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2))
    U0 = tgv_state(dg, prm["gamma"], prm["mach"])
    dt = time_step(mesh, N, cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
    costs, _ = dg.measure_costs(U0, reps=3)
    w_elem, w_type = dg.type_weights(costs)
    stream = dg.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed():
        U = U0.clone()
        K = dg.zeros_state()
        dg.rk_steps(U, K, dt, 1)
        torch.cuda.synchronize()
        ev[0].record(stream)
        dg.rk_steps(U, K, dt, steps)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) * 1e-3

    def measured():
        ms, _ = dg.queue_times()
        return float(ms.max(axis=1).sum() / ms.mean(axis=1).sum() - 1.0)

    def phase_imbalance():
        # per phase (trace, volume, surface): slowest queue over the mean queue, minus 1
        ms, _ = dg.queue_times()
        return (ms.max(axis=1) / ms.mean(axis=1) - 1.0).round(4).tolist()

    dof = mesh.n_elems * (N + 1) ** 3
    out = {"workload": "ns_sphere_64c_N5: 64^3 cells, sphere of radius 0.3L 90% tet-split, "
                       "outside 90% hex (seeded), N=5",
           "n_elems": int(mesh.n_elems), "type_counts": mesh.type_counts().tolist(), "steps": steps,
           "cost_s_per_elem": costs.tolist(), "weights": w_type.astype(int).tolist()}
    wall = timed()
    out["per_type_launches"] = {"wall_s": wall, "pid_s": wall / (dof * 5 * steps)}

    def record(key, wall, **extra):
        out[key] = {"wall_s": wall, "pid_s": wall / (dof * 5 * steps), "measured_imbalance": measured(),
                    "phase_imbalance": phase_imbalance(), **extra}
        log(f"imbalance: {key}: {wall:.3f} s, measured imbalance {out[key]['measured_imbalance']:.3f}")

    for Q in queues:
        dg.set_schedule(dg.partition(torch.ones(mesh.n_elems, dtype=torch.int32), Q))
        record(f"unweighted_Q{Q}", timed())
        for it in range(1, rebalances + 1):
            info = dg.rebalance(0.0)
            record(f"rebalanced{it}_Q{Q}", timed(), predicted_imbalance=info["predicted"])
        dg.set_schedule(dg.partition(w_elem, Q))
        record(f"type_weighted_Q{Q}", timed())
        dg.set_schedule(None)
    del U0, dg
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--split-steps", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-meshes", type=int, default=64)
    ap.add_argument("--batch-small", action="store_true", help="also 64 small meshes (edges 3..6)")
    ap.add_argument("--no-imbalance", action="store_true")
    ap.add_argument("--no-curved", action="store_true")
    ap.add_argument("--curved-steps", type=int, default=5)
    ap.add_argument("--imbalance-steps", type=int, default=5)
    ap.add_argument("--imbalance-queues", type=str, default="256")
    ap.add_argument("--rebalances", type=int, default=1)
    ap.add_argument("--cells", type=int, default=None, help="override the cube edge (testing)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run 3 device copies of 512 MiB (reference for HBM byte counters)")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:  # one process of the all-core oracle timing (no GPU use)
        reps, dof, wall, setup = _time_sample(args.cpu_worker)
        print(json.dumps({"reps": reps, "dof": dof, "wall": wall, "setup": setup}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "libpolydg runs on one GPU; the multi-GPU sharding is described, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2511_08020_amd import perfmodel
    from paper_2511_08020_amd.binding import PolyBatch, PolyDG

    if args.copy_calibration:
        x = torch.full((1 << 26,), 1.0, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 device copies of {x.numel() * 8} bytes each")
        del x, y
    mesh, prm, out = run_plain(args, torch, PolyDG, perfmodel)
    torch.cuda.empty_cache()
    if not args.no_split:
        out["split_form"] = run_split(args, torch, PolyDG, perfmodel, mesh, prm)
        torch.cuda.empty_cache()
    if not args.no_curved:
        out["curved"] = run_curved(torch, PolyDG, perfmodel, args.curved_steps)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        log("adjoint: gradient through 20 steps, config 4")
        out["adjoint"] = run_adjoint(torch, PolyDG, perfmodel)
        log(f"adjoint: {out['adjoint']['wall_s']:.3f} s, "
            f"{out['adjoint']['gradient_over_forward']:.2f}x forward")
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = run_batched(torch, PolyDG, PolyBatch, perfmodel, args.batch_steps,
                                     n_meshes=args.batch_meshes)
        log(f"batched: {out['batched']['wall_s']:.3f} s vs sequential "
            f"{out['batched']['sequential_wall_s']:.3f} s")
        torch.cuda.empty_cache()
        if args.batch_small:
            # the same construction with small meshes (edges 3..6), where one mesh cannot fill the GPU
            out["batched_small"] = run_batched(torch, PolyDG, PolyBatch, perfmodel, 20, min_edge=3, max_edge=6)
            log(f"batched small meshes: {out['batched_small']['wall_s']:.3f} s vs sequential "
                f"{out['batched_small']['sequential_wall_s']:.3f} s")
    if not args.no_imbalance:
        queues = tuple(int(q) for q in args.imbalance_queues.split(","))
        out["imbalance"] = run_imbalance(torch, PolyDG, args.imbalance_steps, queues, args.rebalances)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
