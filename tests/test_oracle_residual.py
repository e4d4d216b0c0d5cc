"""Pins of the oracle residual and LSERK4 against what the discretisation fixes:
free-stream preservation, discrete conservation, convergence on a smooth exact solution,
and the Runge-Kutta order conditions."""
import numpy as np
import pytest

from oracle import physics
from oracle.dg import LSERK_A, LSERK_B, LSERK_C, DGOracle
from workloads import config_mesh, density_wave_primitive, make_mesh, node_noise, tgv_primitive


def _const(x, y, z):
    return (np.full_like(x, 1.2), np.full_like(x, 0.3), np.full_like(x, -0.2),
            np.full_like(x, 0.1), np.full_like(x, 71.4))


def _mixed(C, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_mesh(C, rng.permutation(np.arange(C ** 3) % 4).astype(np.int8))


@pytest.fixture(scope="module")
def mesh1():
    return config_mesh(1)


@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_free_stream(mesh1, eq):
    """A constant state has zero residual on the mixed mesh with mortar faces (every
    quadrature integrates the constant-flux integrand exactly for N >= 2)."""
    o = DGOracle(mesh1, 3, equations=eq)
    U = o.initial_state(_const)
    R = o.residual(U)
    flux_scale = 71.4 + 1.2 * 0.3 ** 2  # |F| of the state
    assert np.abs(R).max() < 1e-13 * flux_scale * 10


@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_discrete_conservation(mesh1, eq):
    """sum_e int_e dU/dt = 0 per variable (fluxes cancel pairwise on every face)."""
    o = DGOracle(mesh1, 3, equations=eq)
    U = o.initial_state(tgv_primitive, lambda es: node_noise(1, 64, es))
    R = o.residual(U)
    tot = o.integral(R)
    # rounding scale: the face fluxes that cancel pairwise, |F| (pressure ~ 71) times the
    # total face area seen from both sides
    area = 2.0 * sum(o.face_geo(fi)["ws"].sum() for fi in range(len(o.faces)))
    scale = 75.0 * area
    assert np.all(np.abs(tot) <= 1e-15 * scale), (tot, scale)


def test_conservation_over_rk_steps(mesh1):
    o = DGOracle(mesh1, 2)
    U = o.initial_state(tgv_primitive, lambda es: node_noise(1, 27, es))
    I0 = o.integral(U)
    U2, _ = o.rk_steps(U, 0.02, 2)
    np.testing.assert_allclose(o.integral(U2), I0, rtol=1e-13, atol=1e-12)


def test_subset_residual_matches_full(mesh1):
    o = DGOracle(mesh1, 3, equations="ns")
    U = o.initial_state(tgv_primitive, lambda es: node_noise(1, 64, es))
    R = o.residual(U)
    Rs = o.residual(U, elems=[3, 50, 121, 159])
    ok = np.isfinite(Rs)
    assert ok.sum() > 0
    assert np.array_equal(Rs[ok], R[ok])


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_mortar_rule_integrates_quad_side_integrands(N):
    """The two chunks of each triangle half of a mortar face integrate x^a y^b over the unit
    square exactly for a, b <= 2N, a + b <= 3N (the quadrilateral side's test functions, degree
    N per direction, times a degree-N flux; a + b <= 3N - 1 at N = 6), and a constant exactly on
    each half alone; the triangle's own n x n rule misses the degree-(2N+1) products."""
    from oracle import faces
    n = N + 1
    ld = np.longdouble
    A, B, C, D = (np.array(v, dtype=ld) for v in ([0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]))

    def rule(chunks):
        pts, ws = [], []
        for X, Y, Z in ((A, B, D), (A, C, D)):
            for ch in chunks:
                s, t, w = faces.face_rule("tri", n, "R1", ch)
                P, _, jac = faces.face_points("tri", X, Y, Z, np.asarray(s, ld), np.asarray(t, ld))
                pts.append(P)
                ws.append(np.asarray(w, ld) * jac)
        return np.vstack(pts), np.concatenate(ws)

    deg = 3 * N if N <= 5 else 3 * N - 1
    P, W = rule((0, 1))
    worst = 0.0
    for a in range(2 * N + 1):
        for b in range(2 * N + 1):
            if a + b <= deg:
                worst = max(worst, abs(float((W * P[:, 0] ** a * P[:, 1] ** b).sum()) - 1.0 / ((a + 1) * (b + 1))))
    assert worst < 1e-15, worst
    P1, W1 = rule((-1,))
    miss = abs(float((W1 * P1[:, 0] ** N * P1[:, 1] ** (N + 1)).sum()) - 1.0 / ((N + 1) * (N + 2)))
    assert miss > 1e-10


def _exact_cons(t):
    return lambda x, y, z: physics.primitive_to_conservative(*density_wave_primitive(x, y, z, t=t), 1.4)


@pytest.mark.parametrize("N", [2, 3])
def test_projection_converges_at_order_N_plus_1(N):
    """Modal projection (Algorithm 1) of a smooth field on mixed meshes: L2 error O(h^(N+1))."""
    errs = []
    Cs = [4, 6]
    for C in Cs:
        o = DGOracle(_mixed(C), N)
        U = o.initial_state(density_wave_primitive)
        errs.append(o.l2_error(U, _exact_cons(0.0), 0))
    rate = np.log(errs[0] / errs[1]) / np.log(Cs[1] / Cs[0])
    assert rate > N + 0.6, (errs, rate)


def test_residual_truncation_converges():
    """dU/dt of the projected exact density wave against the exact time derivative:
    hexahedra converge at O(h^N); collapsed types at no less than O(h^(N-1)) (the nodal
    quadrature of Algorithm 1's mass matrix is inexact for the highest modes)."""
    N = 2
    exR = lambda x, y, z: np.stack([-3 * 0.5 * 0.2 * np.cos(x + y + z)] * 5)
    rates = {}
    for name, kinds_fn in (("hex", lambda C: np.zeros(C ** 3, np.int8)),
                           ("mixed", lambda C: np.random.Generator(np.random.PCG64(3)).permutation(
                               np.arange(C ** 3) % 4).astype(np.int8))):
        errs = []
        for C in (3, 6):
            o = DGOracle(make_mesh(C, kinds_fn(C)), N)
            U = o.initial_state(density_wave_primitive)
            errs.append(o.l2_error(o.residual(U), exR, 0))
        rates[name] = np.log(errs[0] / errs[1]) / np.log(2.0)
    assert rates["hex"] > N - 0.2, rates
    assert rates["mixed"] > N - 1 - 0.1, rates


def _truncation_rates(t, N):
    exR = lambda x, y, z: np.stack([-3 * 0.5 * 0.2 * np.cos(x + y + z)] * 5)  # noqa: E731
    rate = {}
    for fam in ("R1", "LG"):
        errs = []
        for C in (3, 6):
            o = DGOracle(make_mesh(C, np.full(C ** 3, t, np.int8)), N, node_family=fam)
            U = o.initial_state(density_wave_primitive)
            errs.append(o.l2_error(o.residual(U), exR, 0))
        rate[fam] = np.log(errs[0] / errs[1]) / np.log(2.0)
    return rate


def test_residual_truncation_node_families():
    """What the R1 nodes cost (the reading of the workloads' collapsed Gauss-Lobatto nodes): on
    pyramids, whose Gauss-Radau volume lines and Gauss-Lobatto quadrilateral-face points fall one
    degree short of a discrete Gauss theorem, the residual truncation error converges at about
    N - 1 (measured N = 2: 1.06), while the Gauss-Legendre family (volume and quadrilateral-face
    points) keeps order N (1.99).  Pyramid mesh, N = 2, 3^3 -> 6^3 cells."""
    N = 2
    rate = _truncation_rates(2, N)
    assert rate["LG"] >= N - 0.2, rate
    assert rate["R1"] <= N - 0.5, rate


@pytest.mark.slow
@pytest.mark.parametrize("t", [2, 3])
def test_residual_truncation_node_families_N3(t):
    """The same at N = 3 on pyramids and tetrahedra (measured R1 2.17, 2.17; LG 2.90, 2.92)."""
    N = 3
    rate = _truncation_rates(t, N)
    assert rate["LG"] >= N - 0.2, rate
    assert rate["R1"] <= N - 0.5, rate


@pytest.mark.slow
def test_time_integrated_error_converges_at_N_plus_1_on_hexahedra():
    """Hexahedral mesh, N = 3, density wave advected to t = 1 from the nodal state: the L2 error
    falls at order >= N + 0.8 from 6^3 to 12^3 cells.  (The collapsed types reach N and mortar
    faces about one; the device path measures those orders at larger sizes.)"""
    N, T = 3, 1.0
    errs = []
    Cs = (6, 12)
    for C in Cs:
        o = DGOracle(make_mesh(C, np.zeros(C ** 3, np.int8)), N)
        U = o.initial_state(density_wave_primitive)
        dt0 = 0.5 * o.mesh.h / ((2 * N + 1) * (0.5 * np.sqrt(3) + np.sqrt(1.4 / 0.8)))
        ns = int(np.ceil(T / dt0))
        U, _ = o.rk_steps(U, T / ns, ns)
        errs.append(o.l2_error(U, _exact_cons(T), 0))
    rate = np.log(errs[0] / errs[1]) / np.log(Cs[1] / Cs[0])
    assert rate >= N + 0.8, (errs, rate)


def test_lserk4_order_conditions():
    """Applied to y' = z y, one LSERK step is the stability polynomial
    1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200 (fourth order), and the stage times are c."""
    # coefficients of the step polynomial by propagating polynomials in z through the stages
    U = np.zeros(7); U[0] = 1.0
    K = np.zeros(7)
    for s in range(5):
        K = LSERK_A[s] * K + np.concatenate([[0.0], U[:-1]])  # K <- A K + z U
        U = U + LSERK_B[s] * K
    np.testing.assert_allclose(U[:6], [1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200], rtol=1e-13, atol=1e-15)
    # stage times: t_s of the stage-s evaluation for y' = 1
    t, k, times = 0.0, 0.0, []
    for s in range(5):
        times.append(t)
        k = LSERK_A[s] * k + 1.0
        t = t + LSERK_B[s] * k
    np.testing.assert_allclose(times, LSERK_C, rtol=1e-12, atol=1e-15)
    assert abs(t - 1.0) < 1e-14
