"""Batched form (pdg_batch_*): several independent meshes of different sizes, degrees and
equations advanced by one graph launch per step.  The batch runs the residual kernels'
per-element code on the same data, so its states must equal, bit for bit, those of the plain
per-problem time stepping (whose parity against the oracle is tested elsewhere); one member is
also checked against the oracle directly."""
import numpy as np
import pytest

from helpers import ulp_floor, varwise_rel_err
from oracle.dg import DGOracle
from workloads import config_mesh, make_mesh, node_noise, time_step, tgv_primitive
from workloads.device import tgv_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P_REF = 1.0 / (1.4 * 0.1 ** 2)
# (edge, N, equations, seed) of the members: uneven sizes, every degree, both equation sets
MEMBERS = [(3, 2, "euler", 1), (5, 3, "euler", 2), (4, 4, "euler", 3), (3, 5, "euler", 4),
           (3, 6, "euler", 5), (4, 3, "ns", 6), (3, 4, "ns", 7)]


def _problem(C, N, eq, seed):
    from paper_2511_08020_amd.binding import PolyDG
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = rng.dirichlet(np.ones(4))
    mesh = make_mesh(C, rng.choice(4, size=C ** 3, p=frac).astype(np.int8))
    dg = PolyDG.from_mesh(mesh, N, equations=eq, p_ref=P_REF)
    return mesh, dg


@pytest.fixture(scope="module")
def members():
    out = []
    for C, N, eq, seed in MEMBERS:
        mesh, dg = _problem(C, N, eq, seed)
        U0 = tgv_state(dg, noise_seed=seed)
        out.append((mesh, dg, U0, time_step(mesh, N)))
    torch.cuda.synchronize()
    return out


def _sequential(members, n_steps):
    outs = []
    for mesh, dg, U0, dt in members:
        U, K = U0.clone(), dg.zeros_state()
        dg.rk_steps(U, K, dt, n_steps)
        outs.append((U, K))
    torch.cuda.synchronize()
    return outs


def _batched(members, n_steps, tiles=None, autotune=False):
    from paper_2511_08020_amd.binding import PolyBatch
    b = PolyBatch([m[1] for m in members])
    Us = [m[2].clone() for m in members]
    Ks = [m[1].zeros_state() for m in members]
    dts = [m[3] for m in members]
    chosen = None
    if tiles is not None:
        b.set_tiles(tiles)
    if autotune:
        before = [U.clone() for U in Us]
        chosen = b.autotune(Us, Ks, dts, reps=2)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c) for a, c in zip(before, Us)), "autotuning changed a state"
    b.rk_steps(Us, Ks, dts, n_steps)
    torch.cuda.synchronize()
    b.close()
    return list(zip(Us, Ks)), chosen


def test_batch_equals_sequential(members):
    print(f"case: batch of {len(MEMBERS)} problems, 3 steps, tiles 1", flush=True)
    seq = _sequential(members, 3)
    bat, _ = _batched(members, 3)
    for i, ((Us, Ks), (Ub, Kb)) in enumerate(zip(seq, bat)):
        assert torch.isfinite(Ub).all()
        assert torch.equal(Us, Ub), f"member {i}: U differs"
        assert torch.equal(Ks, Kb), f"member {i}: K differs"


def test_batch_tiles_and_repeated_launches(members):
    print("case: batch with tiles 1..8 per (type, N), 2 + 2 steps", flush=True)
    from paper_2511_08020_amd.binding import PolyBatch
    tiles = np.random.default_rng(3).choice([1, 2, 3, 5, 8], size=(4, 7)).astype(np.int32)
    seq = _sequential(members, 4)
    b = PolyBatch([m[1] for m in members])
    b.set_tiles(tiles)
    assert np.array_equal(b.tiles()[:, 2:], tiles[:, 2:])
    Us = [m[2].clone() for m in members]
    Ks = [m[1].zeros_state() for m in members]
    dts = [m[3] for m in members]
    b.rk_steps(Us, Ks, dts, 2)
    b.rk_steps(Us, Ks, dts, 2)  # replays the captured graph
    torch.cuda.synchronize()
    b.close()
    for (Useq, _), Ub in zip(seq, Us):
        assert torch.equal(Useq, Ub)


@pytest.mark.parametrize("solo", [0, 100, 2 ** 31 - 1])
def test_batch_solo_problems(members, solo):
    """Problems with at least `solo` elements run their phases alone (0: all, 100: the larger
    ones, 2^31-1: none), with odd tiles for the merged rest: bitwise the plain stepping."""
    print(f"case: batch with solo threshold {solo}, tiles 3, 2 steps", flush=True)
    from paper_2511_08020_amd.binding import PolyBatch
    seq = _sequential(members, 2)
    b = PolyBatch([m[1] for m in members])
    b.set_tiles(np.full((4, 7), 3, np.int32))
    b.set_solo(solo)
    assert b.solo() == solo
    Us = [m[2].clone() for m in members]
    Ks = [m[1].zeros_state() for m in members]
    b.rk_steps(Us, Ks, [m[3] for m in members], 2)
    torch.cuda.synchronize()
    b.close()
    for (Useq, Kseq), Ub, Kb in zip(seq, Us, Ks):
        assert torch.equal(Useq, Ub) and torch.equal(Kseq, Kb)


def test_batch_solo_graph_recaptured_when_arguments_change(members):
    """Solo problems hold their arguments in the captured graph: new state buffers (and a new
    time step) must be picked up on the next call."""
    print("case: batch with solo problems, arguments changed between calls", flush=True)
    from paper_2511_08020_amd.binding import PolyBatch
    b = PolyBatch([m[1] for m in members])
    b.set_solo(100)
    dts = [m[3] for m in members]
    Us = [m[2].clone() for m in members]
    Ks = [m[1].zeros_state() for m in members]
    b.rk_steps(Us, Ks, dts, 1)
    # continue in fresh buffers with half the time step
    Us2 = [U.clone() for U in Us]
    Ks2 = [K.clone() for K in Ks]
    b.rk_steps(Us2, Ks2, [0.5 * dt for dt in dts], 1)
    torch.cuda.synchronize()
    b.close()
    for (mesh, dg, U0, dt), Ub, Kb in zip(members, Us2, Ks2):
        U, K = U0.clone(), dg.zeros_state()
        dg.rk_steps(U, K, dt, 1)
        dg.rk_steps(U, K, 0.5 * dt, 1)
        torch.cuda.synchronize()
        assert torch.equal(U, Ub) and torch.equal(K, Kb)


def test_batch_autotune(members):
    print("case: batch autotuner, then 2 steps", flush=True)
    seq = _sequential(members, 2)
    bat, tiles = _batched(members, 2, autotune=True)
    print("tiles [type][N]:\n", tiles)
    assert set(np.unique(tiles[:, 2:])) <= {1, 2, 4, 8}
    for (Useq, _), (Ub, _) in zip(seq, bat):
        assert torch.equal(Useq, Ub)


def test_batch_member_vs_oracle():
    print("case: config-1 mesh (euler N=3) inside a batch with two other problems, 2 steps", flush=True)
    from paper_2511_08020_amd.binding import PolyBatch, PolyDG
    mesh = config_mesh(1)
    ora = DGOracle(mesh, 3)
    U0 = ora.initial_state(tgv_primitive, lambda es: node_noise(1, 64, es))
    dt = time_step(mesh, 3)
    dg = PolyDG.from_mesh(mesh, 3, p_ref=P_REF)
    others = [_problem(3, 2, "euler", 8)[1], _problem(3, 5, "euler", 9)[1]]
    probs = [others[0], dg, others[1]]
    Us = [tgv_state(others[0]), torch.tensor(dg.from_input_order(U0), device="cuda"), tgv_state(others[1])]
    Ks = [p.zeros_state() for p in probs]
    b = PolyBatch(probs)
    b.rk_steps(Us, Ks, [1e-3, dt, 1e-3], 2)
    torch.cuda.synchronize()
    U2 = dg.to_input_order(Us[1].cpu().numpy())
    floor, U2_ora = ulp_floor(lambda u: ora.rk_steps(u, dt, 2)[0], U0, ora.offset, draws=1)
    err = varwise_rel_err(U2, U2_ora, ora.offset)
    tol = 1e-12
    print(f"rel err {err:.3e} fp64 floor {floor:.2e} tol {tol:.2e}")
    assert err <= tol
    b.close()


def test_batch_rejects_duplicates(members):
    from paper_2511_08020_amd.binding import PdgError, PolyBatch
    with pytest.raises(PdgError):
        PolyBatch([members[0][1], members[0][1]])


def test_batch_with_curved_members_equals_sequential():
    """Curved members (per-node metrics, per-element mass matrices) batched with affine ones: the
    curved problems form their own (type, N, equations) groups; states equal the per-problem
    stepping bit for bit, with tiles of 1 and 4 and with the largest problem run on its own.
    A moving member is refused."""
    from paper_2511_08020_amd.binding import PDG_ENOTSUP, PdgError, PolyBatch, PolyDG
    from workloads import deformed, motion
    print("case: batch of curved and affine meshes (hexahedra, pyramids; N 3, 4; euler, ns)", flush=True)
    members = []
    for C, N, eq, seed, t, amp in ((3, 3, "euler", 11, 0, 0.15), (4, 4, "ns", 12, 2, 0.15),
                                   (3, 4, "euler", 13, 2, 0.0), (4, 3, "euler", 14, 0, 0.1)):
        mesh = make_mesh(C, np.full(C ** 3, t, np.int8))
        if amp:
            mesh = deformed(mesh, amp)
        dg = PolyDG.from_mesh(mesh, N, equations=eq, p_ref=P_REF)
        members.append((mesh, dg, tgv_state(dg, noise_seed=seed), time_step(mesh, N)))
    torch.cuda.synchronize()
    ref = _sequential(members, 2)
    for tiles, solo in ((None, None), ([[4] * 7] * 4, None), (None, 200)):
        b = PolyBatch([m[1] for m in members])
        if tiles is not None:
            b.set_tiles(tiles)
        if solo is not None:
            b.set_solo(solo)
        Us = [m[2].clone() for m in members]
        Ks = [m[1].zeros_state() for m in members]
        b.rk_steps(Us, Ks, [m[3] for m in members], 2)
        torch.cuda.synchronize()
        b.close()
        for (U, K), (Ur, Kr) in zip(zip(Us, Ks), ref):
            assert torch.equal(U, Ur) and torch.equal(K, Kr)
    moving = members[0][1]
    moving.set_motion(motion(members[0][0], 0.1), 2.0)
    with pytest.raises(PdgError) as ei:
        PolyBatch([moving, members[1][1]])
    assert ei.value.code == PDG_ENOTSUP
