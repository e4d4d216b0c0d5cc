"""Moving meshes on the device against the FP64 oracle, through the C ABI: every corner of a
periodic mesh moves as x0 + d sin(omega t) (workloads.motion), so the Jacobian, the contravariant
vectors, the face normals and the prisms' and pyramids' mass matrices V^T W J V change in time
(Alg. 1) and are rebuilt on the device at every RK stage time; the residual carries the flux
relative to the grid and the dJ/dt source.  Parity bound as for fixed meshes: per conservative
variable max|x_gpu - x_oracle| / max|x_oracle| <= 1e-12.  Combinations the library does not take
fail with PDG_ENOTSUP."""
import numpy as np
import pytest

from helpers import varwise_rel_err
from oracle.dg import DGOracle
from oracle.moving import MovingDG
from workloads import deformed, make_mesh, motion, node_noise, tgv_primitive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)
TOL = 1e-12
OMEGA = 2.0


def _mesh(C=3, t=0, amp=0.15):
    if t == "hex+pyr":
        rng = np.random.Generator(np.random.PCG64(3))
        kinds = np.array((0, 2), np.int8)[rng.permutation(np.arange(C ** 3) % 2)]
        m = make_mesh(C, kinds)
    else:
        m = make_mesh(C, np.full(C ** 3, t, np.int8))
    return deformed(m, amp) if amp else m


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


def _state(ora, N, seed=1):
    return ora.initial_state(tgv_primitive, lambda es: node_noise(seed, (N + 1) ** 3, es))


@pytest.mark.parametrize("t,N,equations", [
    (0, 2, "euler"), (0, 3, "ns"), (0, 4, "euler"), (1, 2, "euler"), (1, 3, "ns"),
    (2, 2, "ns"), (2, 3, "euler"), (2, 4, "ns"), ("hex+pyr", 3, "euler"), ("hex+pyr", 4, "ns"),
    (1, 5, "ns"), (3, 5, "euler")])
def test_moving_residual_vs_oracle(t, N, equations):
    print(f"case: moving cells {t}, 3^3 cells, {equations}, N={N}, t=0.3", flush=True)
    mesh = _mesh(t=t)
    disp = motion(mesh, 0.2)
    mv = MovingDG(mesh, N, disp, OMEGA, equations=equations)
    ora = mv.at(0.3)
    U0 = _state(ora, N, seed=4)
    dg = _dg(mesh, N, equations=equations)
    dg.set_motion(disp, OMEGA)
    dg.set_time(0.3)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.to_input_order(dg.residual(U).cpu().numpy())
    err = varwise_rel_err(R, ora.residual(U0), ora.offset)
    print(f"rel err {err:.3e} tol {TOL:.0e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("t,equations", [(0, "ns"), ("hex+pyr", "euler"), (2, "ns")])
def test_moving_rk_steps_vs_oracle(t, equations):
    """Three LSERK4 steps from t = 0.1: every stage with the geometry at its own time."""
    print(f"case: moving cells {t}, 3^3 cells, {equations} N=3, 3 LSERK4 steps", flush=True)
    mesh = _mesh(t=t)
    N, dt, t0 = 3, 2e-3, 0.1
    disp = motion(mesh, 0.2)
    mv = MovingDG(mesh, N, disp, OMEGA, equations=equations)
    ora0 = mv.at(t0)
    U0 = _state(ora0, N, seed=5)
    U_ora = mv.rk_steps(U0, t0, dt, 3)[0]
    dg = _dg(mesh, N, equations=equations)
    dg.set_motion(disp, OMEGA)
    dg.set_time(t0)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    dg.rk_steps(U, dg.zeros_state(), dt, 3)
    assert abs(dg.time - (t0 + 3 * dt)) <= 1e-15
    err = varwise_rel_err(dg.to_input_order(U.cpu().numpy()), U_ora, ora0.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= TOL


def test_moving_affine_mesh_vs_oracle():
    """An affine mesh set in motion takes the curved kernels from then on."""
    print("case: affine hexahedron/pyramid mesh set in motion, euler N=3", flush=True)
    mesh = _mesh(t="hex+pyr", amp=0.0)
    disp = motion(mesh, 0.2)
    mv = MovingDG(mesh, 3, disp, OMEGA)
    ora = mv.at(0.45)
    U0 = _state(ora, 3, seed=6)
    dg = _dg(mesh, 3)
    dg.set_motion(disp, OMEGA)
    dg.set_time(0.45)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    err = varwise_rel_err(dg.to_input_order(dg.residual(U).cpu().numpy()), ora.residual(U0), ora.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("t", [0, 1, 2])
def test_moving_free_stream_and_geometry(t):
    """A constant state stays constant on the moving mesh (R below 1e-13 of max|U|); the node
    coordinates are the oracle's at the context's time and the node weights w J sum to the box
    volume (the moving elements tile it)."""
    print(f"case: moving cells {t}, 3^3 cells, free stream, N=3", flush=True)
    mesh = _mesh(t=t)
    disp = motion(mesh, 0.2)
    dg = _dg(mesh, 3, equations="ns")
    dg.set_motion(disp, OMEGA)
    dg.set_time(0.3)
    x = dg.node_coords()
    ora = MovingDG(mesh, 3, disp, OMEGA).at(0.3)
    xo = np.stack([ora.elem_geo(e)["x"] for e in range(mesh.n_elems)])
    xs = x.cpu().numpy()[np.argsort(dg.perm)]
    assert np.abs(xs - xo).max() <= 1e-13 * mesh.L
    o = torch.ones_like(x[..., 0])
    q = torch.stack([o, 0.3 * o, -0.2 * o, 0.1 * o, P_REF / 0.4 * o + 0.5 * (0.09 + 0.04 + 0.01)], dim=1)
    U = dg.project(q)
    R = dg.residual(U)
    print(f"  max|R| {torch.abs(R).max().item():.2e}, max|U| {torch.abs(U).max().item():.2e}", flush=True)
    assert torch.abs(R).max().item() < 1e-13 * torch.abs(U).max().item()
    vol = dg.node_weights().sum().item()
    assert abs(vol - mesh.L ** 3) <= 1e-12 * mesh.L ** 3


def test_zero_motion_is_the_fixed_curved_mesh():
    """Zero displacement gives the fixed curved mesh's residual up to rounding: the fixed mesh's
    M_e^-1 comes from the host set-up (long-double Cholesky), the moving mesh's from the device's
    Gauss-Jordan elimination in FP64 (measured 3.0e-14)."""
    print("case: zero motion on curved pyramids, ns N=3", flush=True)
    mesh = _mesh(t=2)
    ora = DGOracle(mesh, 3, equations="ns")
    U0 = _state(ora, 3, seed=7)
    fixed = _dg(mesh, 3, equations="ns")
    moving = _dg(mesh, 3, equations="ns")
    moving.set_motion(np.zeros_like(mesh.corner_xyz), OMEGA)
    moving.set_time(0.8)
    R_f = fixed.residual(torch.tensor(fixed.from_input_order(U0), device="cuda")).cpu().numpy()
    R_m = moving.residual(torch.tensor(moving.from_input_order(U0), device="cuda")).cpu().numpy()
    err = varwise_rel_err(R_m, R_f, fixed.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= 1e-13


def test_moving_queue_schedule_matches():
    print("case: moving hexahedra, queue schedule, euler N=3", flush=True)
    mesh = _mesh()
    disp = motion(mesh, 0.2)
    dg = _dg(mesh, 3)
    dg.set_motion(disp, OMEGA)
    dg.set_time(0.2)
    U = torch.tensor(dg.from_input_order(_state(MovingDG(mesh, 3, disp, OMEGA).at(0.2), 3, seed=8)), device="cuda")
    R_def = dg.residual(U).cpu().numpy()
    dg.set_schedule(dg.partition(torch.ones(dg.n_elems, dtype=torch.int32), 7))
    R_q = dg.residual(U).cpu().numpy()
    dg.set_schedule(None)
    assert varwise_rel_err(R_q, R_def, dg.offset) <= 1e-14


def test_moving_unsupported_combinations_are_refused():
    from paper_2511_08020_amd.binding import PDG_EINVAL, PDG_ENOTSUP, PdgError
    print("case: motion on a mortar mesh, N=6, split form; stage and vjp on a moving mesh", flush=True)
    rng = np.random.Generator(np.random.PCG64(3))
    mortar = make_mesh(3, np.array((0, 3), np.int8)[rng.permutation(np.arange(27) % 2)])
    dg = _dg(mortar, 2)
    with pytest.raises(PdgError) as ei:
        dg.set_motion(motion(mortar, 0.2), OMEGA)
    assert ei.value.code == PDG_ENOTSUP
    with pytest.raises(PdgError) as ei:
        dg.set_time(0.1)
    assert ei.value.code == PDG_EINVAL
    mesh = _mesh(amp=0.0)
    for kw in (dict(N=6), dict(N=2, volume_form="split")):
        d = _dg(mesh, kw.pop("N"), **kw)
        with pytest.raises(PdgError) as ei:
            d.set_motion(motion(mesh, 0.2), OMEGA)
        assert ei.value.code == PDG_ENOTSUP
    dg = _dg(mesh, 2)
    torn = motion(mesh, 0.2).copy()
    torn[0, 7] += 0.01          # one corner of a shared vertex moves apart from the others
    with pytest.raises(PdgError) as ei:
        dg.set_motion(torn, OMEGA)
    assert ei.value.code == PDG_EINVAL
    dg.set_motion(motion(mesh, 0.2), OMEGA)
    U = dg.project(torch.ones((dg.n_elems, 5, 27), dtype=torch.float64, device="cuda") + 10.0)
    with pytest.raises(PdgError) as ei:
        dg.vjp(U, torch.ones_like(U))
    assert ei.value.code == PDG_ENOTSUP


def test_batch_member_set_in_motion_is_refused():
    """A batch captures its members' fixed geometry: once a member moves, stepping the batch
    fails with PDG_ENOTSUP instead of advancing a stale mesh."""
    from paper_2511_08020_amd.binding import PDG_ENOTSUP, PdgError, PolyBatch
    print("case: batch of two affine contexts, one then set in motion", flush=True)
    mesh = _mesh(amp=0.0)
    a, b = _dg(mesh, 2), _dg(mesh, 3)
    batch = PolyBatch([a, b])
    Us = [a.project(torch.ones((a.n_elems, 5, 27), dtype=torch.float64, device="cuda") + 10.0),
          b.project(torch.ones((b.n_elems, 5, 64), dtype=torch.float64, device="cuda") + 10.0)]
    Ks = [a.zeros_state(), b.zeros_state()]
    batch.rk_steps(Us, Ks, [1e-3, 1e-3], 1)
    b.set_motion(motion(mesh, 0.2), OMEGA)
    with pytest.raises(PdgError) as ei:
        batch.rk_steps(Us, Ks, [1e-3, 1e-3], 1)
    assert ei.value.code == PDG_ENOTSUP
    batch.close()


def test_moving_density_wave_converges():
    """The density wave advected to t = 0.5 on moving curved hexahedra (the same absolute
    deformation and motion at both sizes), N = 3, 6^3 -> 12^3 cells: the L2 error of the density
    against the exact solution at the nodes' final positions falls at order >= 3 (measured 3.53;
    3.39 on the fixed curved mesh).  Every stage takes the geometry at its own time, so a wrong stage time
    or grid-velocity term shows here without the oracle."""
    from workloads import density_wave_primitive
    print("case: density wave on moving curved hexahedra, N=3, 6^3 -> 12^3", flush=True)
    errs = []
    N, T = 3, 0.5
    for C in (6, 12):
        mesh = _mesh(C, amp=0.15 * C / 6)
        dg = _dg(mesh, N, p_ref=1.0)
        dg.set_motion(motion(mesh, 0.2 * C / 6), OMEGA)

        def exact(t):
            x = dg.node_coords()
            rho, u, v, w, p = density_wave_primitive(x[..., 0], x[..., 1], x[..., 2], t=t, xp=torch)
            return torch.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)], dim=1)

        U = dg.project(exact(0.0))
        dt0 = 0.5 * 0.41 * mesh.h / ((2 * N + 1) * (0.5 * np.sqrt(3) + np.sqrt(1.4 / 0.8) + 0.4))
        n_steps = int(np.ceil(T / dt0))
        dg.rk_steps(U, dg.zeros_state(), T / n_steps, n_steps)
        wJ = dg.node_weights()
        errs.append(torch.sqrt((wJ * (dg.nodal(U)[:, 0] - exact(T)[:, 0]) ** 2).sum()).item())
        dg.close()
    order = np.log(errs[0] / errs[1]) / np.log(2.0)
    print(f"  L2 errors {errs[0]:.3e} -> {errs[1]:.3e}, order {order:.2f}", flush=True)
    assert order >= 3.0


def test_motion_that_inverts_elements_is_reported():
    """A displacement of two cells folds the mesh: the geometry kernels flag the non-positive
    Jacobian (no kernel fails) and pdg_set_time / pdg_set_motion return PDG_EMESH; at t = 0 the
    same motion is valid again, and non-finite displacements are rejected up front."""
    from paper_2511_08020_amd.binding import PDG_EINVAL, PDG_EMESH, PdgError
    print("case: folding motion on affine hexahedra, N=2", flush=True)
    mesh = _mesh(amp=0.0)
    dg = _dg(mesh, 2)
    bad = motion(mesh, 2.0)
    nan = bad.copy()
    nan[1, 2, 0] = np.nan
    with pytest.raises(PdgError) as ei:
        dg.set_motion(nan, OMEGA)
    assert ei.value.code == PDG_EINVAL
    dg.set_motion(bad, OMEGA)                      # t = 0: x = x0, valid
    with pytest.raises(PdgError) as ei:
        dg.set_time(np.pi / (2 * OMEGA))           # full displacement: folded
    assert ei.value.code == PDG_EMESH
    dg.set_time(0.0)                               # valid again
    assert dg.time == 0.0



def test_second_motion_replaces_the_first():
    """pdg_set_motion called again (another displacement field and frequency) rebuilds the
    geometry and the mass-matrix coefficients: the residual on pyramids at the context's time
    then matches the oracle for the second motion alone, to the fixed 1e-12."""
    print("case: pyramids, 3^3 cells, NS N=3, motion replaced at t=0.3", flush=True)
    mesh = _mesh(t=2)
    N, omega2 = 3, 3.0
    first = motion(mesh, 0.2)
    second = motion(mesh, 0.1) * np.array([1.0, -1.0, 0.5])
    ora = MovingDG(mesh, N, second, omega2, equations="ns").at(0.3)
    U0 = _state(ora, N, seed=6)
    dg = _dg(mesh, N, equations="ns")
    dg.set_motion(first, OMEGA)
    dg.set_time(0.3)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    dg.residual(U)
    dg.set_motion(second, omega2)
    assert dg.time == 0.3
    R = dg.to_input_order(dg.residual(U).cpu().numpy())
    err = varwise_rel_err(R, ora.residual(U0), ora.offset)
    print(f"rel err {err:.3e} tol {TOL:.0e}", flush=True)
    assert err <= TOL
    dg.close()


def _bench_mesh():
    """The curved and moving workload at full size: 24^3 cells split evenly and at random (seed 5)
    into hexahedra and pyramids, 48,384 elements, corners deformed by 0.15 h."""
    C = 24
    rng = np.random.Generator(np.random.PCG64(5))
    return deformed(make_mesh(C, np.array((0, 2), np.int8)[rng.permutation(np.arange(C ** 3) % 2)]), 0.15)


def _bench_dg(mesh, prm):
    from paper_2511_08020_amd.binding import PolyDG
    return PolyDG.from_mesh(mesh, prm["N"], equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"],
                            R=prm["R"], p_ref=1.0 / (prm["gamma"] * prm["mach"] ** 2))


def _bench_params():
    from workloads import config_params
    prm = dict(config_params(2))
    prm["N"] = 4
    return prm




def _bench_residual_case(moving, steps=0):
    """Residual of the seeded coefficient state (the full-size configurations' state) on the
    bench mesh, fixed, or moving at t = 0.3, or moving after `steps` device LSERK4 steps of the
    projected Taylor-Green state from t = 0 (the geometry rebuilt at every stage), against the
    oracle on a seeded element sample, at the time the device reached."""
    from test_gpu_fullsize import _sample, _sampled_floor, _sub_err
    from workloads import coefficient_state, time_step
    from workloads.device import tgv_state
    prm = _bench_params()
    mesh = _bench_mesh()
    U0, off = coefficient_state(mesh, prm["N"])
    dg = _bench_dg(mesh, prm)
    kw = dict(equations="ns", gamma=prm["gamma"], mu=prm["mu"], Pr=prm["Pr"], Rgas=prm["R"])
    ora = DGOracle(mesh, prm["N"], **kw)
    if moving:
        disp = motion(mesh, 0.1)
        dg.set_motion(disp, OMEGA)
        if steps:
            V = tgv_state(dg, prm["gamma"], prm["mach"])
            dt = time_step(mesh, prm["N"], cfl=prm["cfl"], gamma=prm["gamma"], mach=prm["mach"])
            dg.rk_steps(V, dg.zeros_state(), dt, steps)
            assert bool(torch.isfinite(V).all())
        else:
            dg.set_time(0.3)
        print(f"  t = {dg.time:.6e}", flush=True)
        ora = MovingDG(mesh, prm["N"], disp, OMEGA, **kw).at(dg.time)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.to_input_order(dg.residual(U).cpu().numpy())
    S = _sample(mesh, per_type=3)
    floor, R_ora = _sampled_floor(lambda u: ora.residual(u, elems=S), U0, off, S)
    err = _sub_err(R, R_ora, off, S)
    print(f"  sample {S}: rel err {err:.3e} fp64 floor {floor:.2e}", flush=True)
    dg.close()
    return err


def test_curved_bench_mesh_sampled():
    """The curved workload at full size (NS, N = 4, fixed corners), to the fixed 1e-12."""
    print("case: curved 24^3 hexahedron/pyramid mesh, NS N=4, coefficient state, sampled elements", flush=True)
    assert _bench_residual_case(False) <= TOL


def test_moving_bench_mesh_residual_sampled():
    """The moving workload at full size (corners moving 0.1 h at omega = 2, t = 0.3), to the
    fixed 1e-12."""
    print("case: moving 24^3 hexahedron/pyramid mesh, NS N=4, coefficient state at t=0.3, sampled elements",
          flush=True)
    assert _bench_residual_case(True) <= TOL


def test_moving_bench_mesh_after_steps_sampled():
    """The moving workload as the benchmark runs it: two device LSERK4 steps from t = 0 (ten
    geometry rebuilds at the stage times), then the residual at the reached time, to the fixed
    1e-12: the device's clock and its rebuilt geometry agree with the oracle's mesh at that time."""
    print("case: moving 24^3 hexahedron/pyramid mesh, NS N=4, 2 LSERK4 steps, then coefficient state, "
          "sampled elements", flush=True)
    assert _bench_residual_case(True, steps=2) <= TOL
