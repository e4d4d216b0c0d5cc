"""GPU Hilbert keys, element order and weighted partition: bit-exact against the oracle;
queue-scheduled residual against the oracle."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle import sfc
from oracle.dg import DGOracle
from workloads import config_mesh, node_noise, tgv_primitive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


P_REF = 1.0 / (1.4 * 0.1 ** 2)  # mean pressure of the Mach-0.1 Taylor-Green state


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


@pytest.mark.parametrize("cfg", [1, 4, 5])
def test_keys_order_bitexact(cfg):
    print(f"case: hilbert keys and order, workload {cfg}", flush=True)
    mesh = config_mesh(cfg)
    dg = _dg(mesh, 2)
    lo, scale = sfc.bbox_scale(mesh.centroid)
    keys = dg.sfc_keys(lo, scale)
    torch.cuda.synchronize()
    kg = keys.cpu().numpy().view(np.uint64)
    ko = sfc.sfc_keys(mesh.centroid, lo, scale)
    assert np.array_equal(kg, ko)
    assert np.array_equal(dg.perm, sfc.sfc_order(ko))


@pytest.mark.parametrize("cfg,Q", [(1, 7), (4, 256), (5, 256)])
def test_partition_bitexact(cfg, Q):
    print(f"case: weighted partition, workload {cfg}, {Q} queues", flush=True)
    mesh = config_mesh(cfg)
    dg = _dg(mesh, 2)
    rng = np.random.default_rng(cfg)
    costs = rng.uniform(0.5, 3.0, size=4)
    w = sfc.type_weights(costs)[dg.elem_type]
    qb = dg.partition(torch.tensor(w.astype(np.int32)), Q)
    torch.cuda.synchronize()
    assert np.array_equal(qb.cpu().numpy().astype(np.int64), sfc.partition(w, Q))
    # unweighted
    qb1 = dg.partition(torch.ones(dg.n_elems, dtype=torch.int32), Q)
    torch.cuda.synchronize()
    assert np.array_equal(qb1.cpu().numpy().astype(np.int64), sfc.partition(np.ones(dg.n_elems, np.uint32), Q))


def test_partition_bitexact_zero_and_huge_weights():
    """Trailing and leading zero weights (queue_begin[Q] = n), and weights near 2^32 with 4096
    queues (Q (2 S + w) beyond 63 bits): bit-exact against the oracle."""
    print("case: weighted partition, zero weights (workload 1) and huge weights (workload 5)", flush=True)
    dg = _dg(config_mesh(1), 2)
    n = dg.n_elems
    for w in (np.r_[np.ones(n - 5), np.zeros(5)], np.r_[np.zeros(7), np.arange(n - 7) % 3],
              np.zeros(n)):
        w = w.astype(np.uint32)
        for Q in (1, 7, 64):
            qb = dg.partition(torch.tensor(w.view(np.int32)), Q)
            torch.cuda.synchronize()
            assert np.array_equal(qb.cpu().numpy().astype(np.int64), sfc.partition(w, Q)), (Q, w[:10])
    dg5 = _dg(config_mesh(5), 2)
    rng = np.random.default_rng(3)
    w = (np.uint64(2 ** 32 - 1) - rng.integers(0, 10 ** 6, size=dg5.n_elems).astype(np.uint64)).astype(np.uint32)
    qb = dg5.partition(torch.tensor(w.view(np.int32)), 4096)
    torch.cuda.synchronize()
    assert np.array_equal(qb.cpu().numpy().astype(np.int64), sfc.partition(w, 4096))


@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_queue_schedule_residual(eq):
    print(f"case: queue-scheduled residual, {eq}, workload 1", flush=True)
    mesh = config_mesh(1)
    N = 3
    ora = DGOracle(mesh, N, equations=eq)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(1, (N + 1) ** 3, es))
    dg = _dg(mesh, N, equations=eq)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R_def = dg.residual(U).cpu().numpy()
    w = sfc.type_weights([1.0, 1.5, 1.4, 1.2])[dg.elem_type]
    qb = dg.partition(torch.tensor(w.astype(np.int32)), 13)
    dg.set_schedule(qb)
    R_q = dg.residual(U).cpu().numpy()
    dg.set_schedule(None)
    torch.cuda.synchronize()
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(dg.to_input_order(R_q), R_ora, ora.offset)
    print(f"rel err {err:.3e} fp64 floor {floor:.2e}")
    assert err <= 1e-12
    assert varwise_rel_err(R_q, R_def, dg.offset) <= 1e-14


def test_schedule_rejects_bad_bounds():
    from paper_2511_08020_amd.binding import PdgError
    mesh = config_mesh(1)
    dg = _dg(mesh, 2)
    bad = torch.tensor([0, 5, 3, dg.n_elems], dtype=torch.int32)
    with pytest.raises(PdgError):
        dg.set_schedule(bad)
