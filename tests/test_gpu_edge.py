"""Edge cases through the C ABI: single-type meshes (every other type empty), the smallest
periodic mesh, the largest degrees, more queues than elements (empty queues), zero and
skewed weights, and the argument checks that must fail cleanly."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle import sfc
from oracle.dg import DGOracle
from workloads import make_mesh, node_noise, tgv_primitive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)


def _dg(mesh, N, **kw):
    from paper_2511_08020_amd.binding import PolyDG
    kw.setdefault("p_ref", P_REF)
    return PolyDG.from_mesh(mesh, N, **kw)


def _parity(mesh, N, eq="euler"):
    ora = DGOracle(mesh, N, equations=eq)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(3, (N + 1) ** 3, es))
    dg = _dg(mesh, N, equations=eq)
    R = dg.residual(torch.tensor(dg.from_input_order(U0), device="cuda"))
    torch.cuda.synchronize()
    Rg = dg.to_input_order(R.cpu().numpy())
    floor, R_ora = ulp_floor(ora.residual, U0, ora.offset)
    err = varwise_rel_err(Rg, R_ora, ora.offset)
    tol = 1e-12
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {tol:.2e}")
    assert err <= tol


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_single_type_mesh(kind, eq):
    """Meshes of one cell kind only: three of the four per-type launches are empty."""
    print(f"case: 3^3 cells all of kind {kind}, {eq}, N=3", flush=True)
    _parity(make_mesh(3, np.full(27, kind, dtype=np.int8)), 3, eq)


def test_two_types_with_mortars():
    """Hexahedra next to tet-split cells only (every shared face a quad/two-triangle mortar)."""
    print("case: 3^3 cells, hex / tet-split checkerboard, euler N=4", flush=True)
    kinds = (np.indices((3, 3, 3)).sum(axis=0).ravel() % 2 * 3).astype(np.int8)
    _parity(make_mesh(3, kinds), 4)


def test_more_queues_than_elements():
    """Q > n_elems leaves empty queues; the schedule still covers every element once."""
    print("case: 160 elements, 1000 queues, euler N=2", flush=True)
    rng = np.random.Generator(np.random.PCG64(5))
    mesh = make_mesh(4, rng.permutation(np.arange(64) % 4).astype(np.int8))
    dg = _dg(mesh, 2)
    w = rng.integers(1, 9, size=mesh.n_elems).astype(np.uint32)
    qb = dg.partition(torch.tensor(w.astype(np.int32)), 1000)
    torch.cuda.synchronize()
    assert np.array_equal(qb.cpu().numpy().astype(np.int64), sfc.partition(w, 1000))
    ora = DGOracle(mesh, 2)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(3, 27, es))
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    R_type = dg.residual(U)
    dg.set_schedule(qb)
    R_queue = dg.residual(U)
    dg.set_schedule(None)
    torch.cuda.synchronize()
    assert torch.equal(R_type, R_queue)


def test_zero_and_skewed_weights():
    """All-zero weights give empty queues but one covering segment; one huge weight."""
    rng = np.random.Generator(np.random.PCG64(6))
    mesh = make_mesh(3, rng.permutation(np.arange(27) % 4).astype(np.int8))
    dg = _dg(mesh, 2)
    for w in (np.zeros(mesh.n_elems, np.uint32),
              np.where(np.arange(mesh.n_elems) == 17, 4_000_000_000, 1).astype(np.uint32)):
        qb = dg.partition(torch.tensor(w.view(np.int32)), 8)
        torch.cuda.synchronize()
        assert np.array_equal(qb.cpu().numpy().astype(np.int64), sfc.partition(w, 8))


def test_argument_errors():
    from paper_2511_08020_amd.binding import PdgError
    rng = np.random.Generator(np.random.PCG64(7))
    mesh = make_mesh(3, rng.permutation(np.arange(27) % 4).astype(np.int8))
    with pytest.raises(PdgError):
        _dg(mesh, 7)                       # degree out of range
    with pytest.raises(PdgError):
        _dg(mesh, 6, equations="ns")       # Navier-Stokes limited to N <= 5
    dg = _dg(mesh, 2)
    U = dg.zeros_state()
    with pytest.raises(PdgError):
        dg.residual(U, out=U)              # aliasing input and output
    with pytest.raises(PdgError):
        dg.rk_steps(U, U, 1e-3, 1)         # U and K must differ
    with pytest.raises(PdgError):
        dg.rk_stage(U, dg.zeros_state(), 1e-3, 5)   # stage out of range
    with pytest.raises(PdgError):
        dg.vjp(U, U, out=U)                # gradient aliasing its inputs
    with pytest.raises(ValueError):
        dg.residual(torch.zeros(5, dtype=torch.float64, device="cuda"))
