"""pdg_vjp_static (the vector-Jacobian product with the library's static device workspace, for
callers that cannot allocate) against pdg_vjp, through the C ABI: two calls in a row on one GPU,
the second on a smaller mesh, then the first mesh again; and a mesh whose workspace exceeds the
static array is rejected with PDG_EINVAL before any device work."""
import numpy as np
import pytest

from helpers import varwise_rel_err
from workloads import config_mesh, make_mesh, node_noise, tgv_primitive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)


def _mixed_mesh(C, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_mesh(C, rng.permutation(np.arange(C ** 3) % 4).astype(np.int8))


def _case(mesh, N, eq, seed):
    from oracle.dg import DGOracle
    from paper_2511_08020_amd.binding import PolyDG
    ora = DGOracle(mesh, N, equations=eq)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(seed, (N + 1) ** 3, es))
    lam = np.random.default_rng(30 + seed).standard_normal(ora.size)
    dg = PolyDG.from_mesh(mesh, N, equations=eq, p_ref=P_REF)
    U = torch.tensor(dg.from_input_order(U0), device="cuda")
    cot = torch.tensor(dg.from_input_order(lam), device="cuda")
    return dg, U, cot, ora.offset


def _compare(dg, U, cot, offsets):
    ref = dg.vjp(U, cot)
    out = torch.full_like(ref, float("nan"))
    dg.vjp_static(U, cot, out)
    torch.cuda.synchronize()
    a = dg.to_input_order(out.cpu().numpy())
    b = dg.to_input_order(ref.cpu().numpy())
    err = varwise_rel_err(a, b, offsets)
    print(f"vjp_static vs vjp: rel err {err:.3e}, bitwise equal {np.array_equal(a, b)}", flush=True)
    assert np.all(np.isfinite(a))
    assert err <= 1e-12


def test_vjp_static_matches_vjp_two_calls():
    print("case: pdg_vjp_static, NS mixed 4^3 N=3, then Euler 4^3 config mesh N=3, then NS again", flush=True)
    big = _case(_mixed_mesh(4), 3, "ns", 1)
    small = _case(config_mesh(1), 3, "euler", 2)
    _compare(*big)
    _compare(*small)
    _compare(*big)
    big[0].close()
    small[0].close()


def test_vjp_static_rejects_oversized_mesh():
    from paper_2511_08020_amd import binding
    from paper_2511_08020_amd.binding import PolyDG
    print("case: pdg_vjp_static size rejection, NS mixed 16^3 N=4", flush=True)
    mesh = _mixed_mesh(16)
    dg = PolyDG.from_mesh(mesh, 4, equations="ns", p_ref=P_REF)
    U = dg.zeros_state()
    cot = dg.zeros_state()
    out = dg.zeros_state()
    rc = dg.lib.pdg_vjp_static(dg.handle, binding._ptr(U), binding._ptr(cot), binding._ptr(out))
    assert rc == binding.PDG_EINVAL
    assert b"static workspace" in dg.lib.pdg_last_error()
    dg.close()
