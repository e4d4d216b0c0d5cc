"""Curved (trilinear) elements on the device against the FP64 oracle, through the C ABI: every
vertex of a periodic mesh moved by a smooth periodic field (workloads.deformed), so the Jacobian
and the contravariant vectors vary from node to node, the quadrilateral faces are bilinear
patches whose normal turns across the face, and the prisms' and pyramids' mass matrices
V^T W J V differ from element to element (Alg. 1).  The device takes per-node metric tables,
per-face-point normals and a mass-matrix inverse per modal element.  Parity bound as for the
affine meshes: per conservative variable max|x_gpu - x_oracle| / max|x_oracle| <= 1e-12.
Combinations the library does not take (a curved mesh with quadrilateral-triangle mortars, the
split form, the adjoint) fail with PDG_ENOTSUP."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle.dg import DGOracle
from workloads import deformed, density_wave_primitive, make_mesh, node_noise, tgv_primitive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)
TOL = 1e-12


def _mesh(C=3, t=0, amp=0.15):
    """Curved mesh of one cell kind t, or of hexahedron and pyramid cells (t = "hex+pyr",
    conforming: the pyramids' bases meet the hexahedra's faces)."""
    if t == "hex+pyr":
        rng = np.random.Generator(np.random.PCG64(3))
        kinds = np.array((0, 2), np.int8)[rng.permutation(np.arange(C ** 3) % 2)]
        return deformed(make_mesh(C, kinds), amp)
    return deformed(make_mesh(C, np.full(C ** 3, t, np.int8)), amp)


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


def _state(ora, N, seed=1):
    return ora.initial_state(tgv_primitive, lambda es: node_noise(seed, (N + 1) ** 3, es))


@pytest.mark.parametrize("t,N,equations", [
    (0, 2, "euler"), (0, 3, "euler"), (0, 4, "euler"), (0, 2, "ns"), (0, 3, "ns"), (0, 4, "ns"),
    (1, 2, "euler"), (1, 3, "ns"), (2, 2, "euler"), (2, 3, "ns"), (2, 4, "ns"),
    ("hex+pyr", 3, "euler"), ("hex+pyr", 4, "ns"), (3, 3, "ns"), (3, 5, "euler"), (1, 5, "ns")])
def test_curved_residual_vs_oracle(t, N, equations):
    print(f"case: curved cells {t}, 3^3 cells, {equations}, N={N}", flush=True)
    mesh = _mesh(t=t)
    ora = DGOracle(mesh, N, equations=equations)
    U0 = _state(ora, N, seed=4)
    dg = _dg(mesh, N, equations=equations)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.to_input_order(dg.residual(U).cpu().numpy())
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(R, R_ora, ora.offset)
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {TOL:.0e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("t", [0, "hex+pyr"])
def test_curved_rk_steps_vs_oracle(t):
    print(f"case: curved cells {t}, 3^3 cells, ns N=3, 3 LSERK4 steps", flush=True)
    mesh = _mesh(t=t)
    N = 3
    ora = DGOracle(mesh, N, equations="ns")
    U0 = _state(ora, N, seed=5)
    dt = 2e-3
    U_ora = ora.rk_steps(U0, dt, 3)[0]
    dg = _dg(mesh, N, equations="ns")
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    dg.rk_steps(U, dg.zeros_state(), dt, 3)
    err = varwise_rel_err(dg.to_input_order(U.cpu().numpy()), U_ora, ora.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("t", [0, 1, 2])
def test_curved_free_stream_and_node_weights(t):
    """A constant state stays constant (R below 1e-13 of the state's largest entry, the energy's
    constant-mode coefficient: rounding), and the node weights w J sum to the box volume (the
    trilinear elements tile it)."""
    print(f"case: curved cells {t}, 3^3 cells, free stream, N=3", flush=True)
    mesh = _mesh(t=t)
    dg = _dg(mesh, 3, equations="ns")
    x = dg.node_coords()
    o = torch.ones_like(x[..., 0])
    q = torch.stack([o, 0.3 * o, -0.2 * o, 0.1 * o, P_REF / 0.4 * o + 0.5 * (0.09 + 0.04 + 0.01)], dim=1)
    U = dg.project(q)
    R = dg.residual(U)
    print(f"  max|R| {torch.abs(R).max().item():.2e}, max|U| {torch.abs(U).max().item():.2e}", flush=True)
    assert torch.abs(R).max().item() < 1e-13 * torch.abs(U).max().item()
    vol = dg.node_weights().sum().item()
    assert abs(vol - mesh.L ** 3) <= 1e-12 * mesh.L ** 3


def test_curved_queue_schedule_matches():
    """The work-queue kernels run the same element code: residual equal to the per-type launch."""
    print("case: curved hexahedra, queue schedule, euler N=3", flush=True)
    mesh = _mesh()
    dg = _dg(mesh, 3)
    ora = DGOracle(mesh, 3)
    U = torch.tensor(dg.from_input_order(_state(ora, 3, seed=6)), device="cuda")
    R_def = dg.residual(U).cpu().numpy()
    qb = dg.partition(torch.ones(dg.n_elems, dtype=torch.int32), 7)
    dg.set_schedule(qb)
    R_q = dg.residual(U).cpu().numpy()
    dg.set_schedule(None)
    assert varwise_rel_err(R_q, R_def, dg.offset) <= 1e-14


def test_curved_density_wave_converges():
    """The density wave advected to t = 0.5 on curved hexahedra (the same absolute deformation at
    both sizes), N = 3, 6^3 -> 12^3 cells: L2 error of the density falls at order >= 3 (hexahedra
    reach N + 1 on affine meshes)."""
    print("case: density wave on curved hexahedra, N=3, 6^3 -> 12^3", flush=True)
    errs = []
    N, T = 3, 0.5
    for C in (6, 12):
        mesh = _mesh(C, amp=0.15 * C / 6)
        dg = _dg(mesh, N, p_ref=1.0)
        x = dg.node_coords()
        wJ = dg.node_weights()

        def exact(t):
            rho, u, v, w, p = density_wave_primitive(x[..., 0], x[..., 1], x[..., 2], t=t, xp=torch)
            return torch.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)], dim=1)

        U = dg.project(exact(0.0))
        dt0 = 0.5 * 0.41 * mesh.h / ((2 * N + 1) * (0.5 * np.sqrt(3) + np.sqrt(1.4 / 0.8)))
        n_steps = int(np.ceil(T / dt0))
        dg.rk_steps(U, dg.zeros_state(), T / n_steps, n_steps)
        errs.append(torch.sqrt((wJ * (dg.nodal(U)[:, 0] - exact(T)[:, 0]) ** 2).sum()).item())
        dg.close()
    order = np.log(errs[0] / errs[1]) / np.log(2.0)
    print(f"  L2 errors {errs[0]:.3e} -> {errs[1]:.3e}, order {order:.2f}", flush=True)
    assert order >= 3.0


@pytest.mark.parametrize("t,N,equations,flux", [
    (0, 3, "euler", "lf"), (0, 2, "ns", "lf"), (0, 3, "euler", "ec"), (1, 3, "euler", "lf"),
    (2, 3, "ns", "lf"), ("hex+pyr", 3, "euler", "ec")])
def test_curved_split_form_vs_oracle(t, N, equations, flux):
    """The entropy-stable split form on curved elements: each two-point flux takes the mean of
    the two nodes' contravariant vectors (every direction of hexahedra, the Gauss-Lobatto
    directions of the other types); with the entropy-conservative surface flux as well.  (At
    N = 4 the oracle's own FP64 floor for this state is 2.0e-12 on curved and affine hexahedra
    alike, above the fixed bar; measured there 1.3e-12.)"""
    print(f"case: curved cells {t}, 3^3 cells, split form, {equations} {flux}, N={N}", flush=True)
    mesh = _mesh(t=t)
    ora = DGOracle(mesh, N, equations=equations, volume_form="split", surface_flux=flux)
    U0 = _state(ora, N, seed=9)
    dg = _dg(mesh, N, equations=equations, volume_form="split", flux=flux)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.to_input_order(dg.residual(U).cpu().numpy())
    err = varwise_rel_err(R, ora.residual(U0), ora.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= TOL


def test_curved_unsupported_combinations_are_refused():
    from paper_2511_08020_amd.binding import PDG_ENOTSUP, PdgError
    print("case: curved mortars, curved adjoint", flush=True)
    rng = np.random.Generator(np.random.PCG64(3))
    kinds = np.array((0, 3), np.int8)[rng.permutation(np.arange(27) % 2)]
    with pytest.raises(PdgError) as ei:
        _dg(deformed(make_mesh(3, kinds), 0.15), 2)       # hexahedra next to tetrahedron pairs
    assert ei.value.code == PDG_ENOTSUP
    dg = _dg(_mesh(), 2)
    ora = DGOracle(_mesh(), 2)
    U = torch.tensor(dg.from_input_order(_state(ora, 2)), device="cuda")
    with pytest.raises(PdgError) as ei:
        dg.vjp(U, torch.ones_like(U))
    assert ei.value.code == PDG_ENOTSUP
