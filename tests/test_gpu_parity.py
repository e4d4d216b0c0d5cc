"""GPU residual / time-integration parity against the FP64 oracle (through the C ABI).

Metric (per conservative variable): max|x_gpu - x_oracle| / max|x_oracle|.  Bound: 1e-12 on
the 4^3-cell workload (residual and 10 LSERK4 steps) and on the degree sweep over 3^3-cell
meshes.  Each case also prints the problem's own FP64 floor (helpers.ulp_floor: the change of
the oracle's result under one-ulp perturbations of its input); at Mach 0.1 the pressure ~71
cancels in the momentum residual, and the device keeps the energy relative to the reference
state so that this cancellation costs no rounding of the mean pressure."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle.dg import DGOracle
from workloads import config_mesh, make_mesh, node_noise, tgv_primitive, time_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


P_REF = 1.0 / (1.4 * 0.1 ** 2)  # mean pressure of the Mach-0.1 Taylor-Green state


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


def _state(ora, N, seed=1):
    return ora.initial_state(tgv_primitive, lambda es: node_noise(seed, (N + 1) ** 3, es))


def _gpu_residual(dg, U0):
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.residual(U)
    torch.cuda.synchronize()
    return dg.to_input_order(R.cpu().numpy())


def _mixed_mesh(C, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_mesh(C, rng.permutation(np.arange(C ** 3) % 4).astype(np.int8))


@pytest.fixture(scope="module")
def cfg1():
    mesh = config_mesh(1)
    ora = DGOracle(mesh, 3)
    U0 = _state(ora, 3)
    return mesh, ora, U0


def test_residual_euler_config1(cfg1):
    mesh, ora, U0 = cfg1
    print("case: euler config-1 residual, N=3, 160 elements", flush=True)
    dg = _dg(mesh, 3)
    R = _gpu_residual(dg, U0)
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(R, R_ora, ora.offset)
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {TOL:.0e}")
    assert err <= TOL


def test_rk10_euler_config1(cfg1):
    mesh, ora, U0 = cfg1
    print("case: euler config-1, 10 LSERK4 steps at CFL 0.5", flush=True)
    dt = time_step(mesh, 3)
    dg = _dg(mesh, 3)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    K = torch.full_like(U, float("nan"))  # ignored: the first stage has A_0 = 0
    dg.rk_steps(U, K, dt, 10)
    torch.cuda.synchronize()
    U10 = dg.to_input_order(U.cpu().numpy())
    floor, U10_ora = ulp_floor(lambda u: ora.rk_steps(u, dt, 10)[0], U0, ora.offset)
    err = varwise_rel_err(U10, U10_ora, ora.offset)
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {TOL:.0e}")
    assert err <= TOL


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_residual_euler_degrees(N):
    print(f"case: euler mixed 3^3 cells residual, N={N}", flush=True)
    mesh = _mixed_mesh(3)
    ora = DGOracle(mesh, N)
    U0 = _state(ora, N, seed=5)
    R = _gpu_residual(_dg(mesh, N), U0)
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(R, R_ora, ora.offset)
    tol = TOL
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_residual_ns(N):
    print(f"case: navier-stokes mixed 3^3 cells residual, N={N}", flush=True)
    mesh = _mixed_mesh(3, seed=7)
    ora = DGOracle(mesh, N, equations="ns")
    U0 = _state(ora, N, seed=6)
    R = _gpu_residual(_dg(mesh, N, equations="ns"), U0)
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(R, R_ora, ora.offset)
    tol = TOL
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {tol:.2e}")
    assert err <= tol


def test_free_stream_gpu():
    print("case: free stream, euler mixed 4^3 cells N=3", flush=True)
    mesh = config_mesh(1)
    ora = DGOracle(mesh, 3)
    const = lambda x, y, z: (np.full_like(x, 1.2), np.full_like(x, 0.3), np.full_like(x, -0.2),
                             np.full_like(x, 0.1), np.full_like(x, 2.0))
    U0 = ora.initial_state(const)
    R = _gpu_residual(_dg(mesh, 3), U0)
    assert np.abs(R).max() <= 1e-12 * 10.0


def test_projection_and_nodal(cfg1):
    mesh, ora, U0 = cfg1
    print("case: modal projection of nodal values", flush=True)
    dg = _dg(mesh, 3)
    q = np.stack([ora.nodal(U0, e) for e in range(mesh.n_elems)]).astype(np.float64)  # input order
    qd = torch.tensor(np.ascontiguousarray(q[dg.perm]), device="cuda")
    U = dg.project(qd)
    back = dg.nodal(U)
    torch.cuda.synchronize()
    Ug = dg.to_input_order(U.cpu().numpy())
    assert varwise_rel_err(Ug, U0, ora.offset) <= TOL
    assert np.abs(back.cpu().numpy() - q[dg.perm]).max() <= 1e-12 * np.abs(q).max()
