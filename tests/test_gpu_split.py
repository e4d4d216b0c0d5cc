"""Entropy-stable split form on the device (through the C ABI) against the oracle's split
form, plus properties the oracle does not enter: discrete entropy conservation of the device
residual with the entropy-conservative surface flux on a hexahedral mesh, bitwise equality of
the work-queue schedule, and the forms the adjoint and the batch refuse.

Parity metric and bound as in the weak-form parity tests: per conservative variable
max|x_gpu - x_oracle| / max|x_oracle| <= 1e-12 (the oracle's own FP64 floor is printed)."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle import physics as ph
from oracle.dg import DGOracle
from workloads import make_mesh, node_noise, tgv_primitive, time_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


def _mixed_mesh(C, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_mesh(C, rng.permutation(np.arange(C ** 3) % 4).astype(np.int8))


def _gpu_residual(dg, U0):
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R = dg.residual(U)
    torch.cuda.synchronize()
    return dg.to_input_order(R.cpu().numpy())


def _parity(mesh, N, eq, flux="lf", amp=1e-3):
    ora = DGOracle(mesh, N, equations=eq, volume_form="split", surface_flux=flux)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(1, (N + 1) ** 3, es, amp=amp))
    dg = _dg(mesh, N, equations=eq, volume_form="split", flux=flux)
    R = _gpu_residual(dg, U0)
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(R, R_ora, ora.offset)
    tol = 1e-12
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {tol:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_split_residual_euler(N):
    print(f"case: split form, euler, mixed 3^3 cells, N={N}", flush=True)
    _parity(_mixed_mesh(3), N, "euler")


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_split_residual_ns(N):
    print(f"case: split form, ns, mixed 3^3 cells, N={N}", flush=True)
    _parity(_mixed_mesh(3), N, "ns")


def test_split_residual_entropy_conservative_surface_flux():
    """Both sides with the two-point flux at the faces as well; larger noise so that the
    logarithmic means leave their series branch at many point pairs."""
    print("case: split form + EC surface flux, euler, mixed 3^3 cells, N=3, noise 0.2", flush=True)
    _parity(_mixed_mesh(3), 3, "euler", flux="ec", amp=0.2)


def test_split_rk_steps():
    print("case: split form, euler, mixed 3^3 cells, N=3, 2 LSERK4 steps", flush=True)
    mesh = _mixed_mesh(3)
    N = 3
    ora = DGOracle(mesh, N, volume_form="split")
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(1, 64, es))
    dt = time_step(mesh, N)
    U_ora, _ = ora.rk_steps(U0, dt, 2)
    dg = _dg(mesh, N, volume_form="split")
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    K = dg.zeros_state()
    dg.rk_steps(U, K, dt, 2)
    torch.cuda.synchronize()
    err = varwise_rel_err(dg.to_input_order(U.cpu().numpy()), U_ora, ora.offset)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("N", [3, 4])
def test_device_entropy_conservation_on_hexahedra(N):
    """Periodic hexahedral mesh, split form and entropy-conservative surface flux: the device
    residual satisfies sum_e sum_k w_k J_k v(q_k) . dq_k/dt = 0 to rounding (computed here
    from the device's U and R only); the weak form with the same flux does not."""
    print(f"case: entropy rate on 4^3 hexahedra, N={N}", flush=True)
    mesh = make_mesh(4, np.zeros(64, np.int8))
    from workloads.device import tgv_state
    rates = {}
    for vf in ("split", "weak"):
        dg = _dg(mesh, N, volume_form=vf, flux="ec")
        U = tgv_state(dg, noise_seed=2)
        U = U + 0.05 * torch.sin(7.0 * torch.arange(U.numel(), device="cuda", dtype=torch.float64))
        R = dg.residual(U)
        q = U.reshape(-1, 5, (N + 1) ** 3).cpu().numpy()
        r = R.reshape(-1, 5, (N + 1) ** 3).cpu().numpy()
        w = dg.node_weights().cpu().numpy()
        v = np.stack([ph.entropy_variables(q[e], 1.4) for e in range(q.shape[0])])
        terms = (v * r).sum(axis=1) * w
        rates[vf] = (terms.sum(), np.abs(terms).sum())
        print(vf, rates[vf], flush=True)
    tot, scale = rates["split"]
    assert abs(tot) < 1e-13 * scale
    tot, scale = rates["weak"]
    assert abs(tot) > 1e-8 * scale


@pytest.mark.parametrize("eq,N", [("euler", 4), ("ns", 4), ("ns", 5)])
def test_split_queue_schedule_bitwise(eq, N):
    print(f"case: split form, queue schedule vs per-type launches, {eq} N={N}", flush=True)
    mesh = _mixed_mesh(4)
    dg = _dg(mesh, N, equations=eq, volume_form="split")
    from workloads.device import tgv_state
    U = tgv_state(dg)
    R_type = dg.residual(U)
    qb = dg.partition(torch.ones(dg.n_elems, dtype=torch.int32), 16)
    dg.set_schedule(qb)
    R_queue = dg.residual(U)
    dg.set_schedule(None)
    torch.cuda.synchronize()
    assert torch.equal(R_type, R_queue)


def test_split_and_ec_queue_schedule_with_rebalancing_bitwise():
    """Split form with the two-point surface flux on the work-queue kernels, stepped through the
    dynamic balance loop (the queue boundaries move twice): bitwise the per-type launches."""
    print("case: split + EC flux, queue schedule + rebalancing vs per-type, euler N=3", flush=True)
    mesh = _mixed_mesh(4)
    dg = _dg(mesh, 3, volume_form="split", flux="ec")
    from workloads.device import tgv_state
    U0 = tgv_state(dg)
    dt = time_step(mesh, 3)
    U_ref, K_ref = U0.clone(), dg.zeros_state()
    dg.rk_steps(U_ref, K_ref, dt, 3)
    dg.set_schedule(dg.partition(torch.ones(dg.n_elems, dtype=torch.int32), 24))
    U, K = U0.clone(), dg.zeros_state()
    log = dg.rk_steps_balanced(U, K, dt, 3, interval=1, threshold=0.0)
    dg.set_schedule(None)
    torch.cuda.synchronize()
    print(log, flush=True)
    assert len(log) == 2 and all(r["rebalanced"] for r in log)
    assert torch.equal(U, U_ref) and torch.equal(K, K_ref)


def test_adjoint_and_batch_refuse_the_split_form():
    from paper_2511_08020_amd.binding import PdgError, PolyBatch
    mesh = _mixed_mesh(3)
    for kw in (dict(volume_form="split"), dict(flux="ec")):
        dg = _dg(mesh, 2, **kw)
        U = dg.zeros_state()
        with pytest.raises(PdgError):
            dg.vjp(U + 1.0, U)
        with pytest.raises(PdgError):
            PolyBatch([dg])
