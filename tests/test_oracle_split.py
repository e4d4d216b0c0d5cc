"""Pins of the oracle's entropy-stable split form (the paper's stabilisation, Sec. 2, with
Chandrashekar's two-point flux): the logarithmic mean against closed forms and inequalities,
the two-point flux against consistency, symmetry and the entropy-conservation identity, the
split volume term against the weak one where the SBP property makes them equal, and the
residual against discrete entropy conservation (hexahedra), free-stream preservation and
conservation (mixed meshes)."""
import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle.dg import DGOracle
from workloads import config_mesh, make_mesh, node_noise, tgv_primitive

G = 1.4


def _states(P, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(0.3, 3.0, P)
    u = rng.normal(0.0, 0.7, (3, P))
    p = rng.uniform(0.2, 5.0, P)
    return ph.primitive_to_conservative(rho, u[0], u[1], u[2], p, G)


def test_log_mean_closed_forms():
    assert ph.log_mean(1.0, math.e) == pytest.approx(math.e - 1.0, rel=1e-15)
    assert ph.log_mean(1.0, math.e ** 2) == pytest.approx((math.e ** 2 - 1.0) / 2.0, rel=1e-15)
    assert ph.log_mean(2.5, 2.5) == 2.5
    # close arguments: L(a, a(1+h)) = a (1 + h/2 - h^2/12 + h^3/24 + ...)
    for h in (1e-3, 1e-6, 1e-9, 1e-12):
        exact = 1.0 + h / 2 - h * h / 12 + h ** 3 / 24
        assert ph.log_mean(1.0, 1.0 + h) == pytest.approx(exact, rel=2e-16)


def test_log_mean_symmetry_homogeneity_and_bounds():
    rng = np.random.Generator(np.random.PCG64(3))
    a, b = rng.uniform(0.01, 10, 1000), rng.uniform(0.01, 10, 1000)
    L = ph.log_mean(a, b)
    assert np.array_equal(L, ph.log_mean(b, a)) or np.allclose(L, ph.log_mean(b, a), rtol=1e-15)
    assert np.allclose(ph.log_mean(3.7 * a, 3.7 * b), 3.7 * L, rtol=1e-14)
    assert np.all(L >= np.sqrt(a * b) * (1 - 1e-15)) and np.all(L <= 0.5 * (a + b) * (1 + 1e-15))


def test_two_point_flux_consistent_and_symmetric():
    qL, qR = _states(500, 1), _states(500, 2)
    n = np.random.Generator(np.random.PCG64(4)).normal(size=(3, 500))
    F = ph.chandrashekar_flux(qL, qL, n, G)
    assert np.allclose(F, ph.normal_flux(ph.euler_flux(qL, G), n), rtol=1e-14, atol=1e-14)
    assert np.allclose(ph.chandrashekar_flux(qL, qR, n, G), ph.chandrashekar_flux(qR, qL, n, G),
                       rtol=1e-14, atol=1e-14)


def test_two_point_flux_entropy_conservative():
    """(v_R - v_L).F#(qL, qR) = psi_R - psi_L (Tadmor's condition) for random state pairs;
    the entropy variables are checked against finite differences of S first."""
    q = _states(50, 5)
    v = ph.entropy_variables(q, G)
    for j in range(5):
        h = 1e-6 * np.maximum(1.0, np.abs(q[j]))
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        fd = (ph.entropy(qp, G) - ph.entropy(qm, G)) / (2 * h)
        assert np.allclose(fd, v[j], rtol=1e-7, atol=1e-7)
    qL, qR = _states(2000, 6), _states(2000, 7)
    n = np.random.Generator(np.random.PCG64(8)).normal(size=(3, 2000))
    F = ph.chandrashekar_flux(qL, qR, n, G)
    lhs = ((ph.entropy_variables(qR, G) - ph.entropy_variables(qL, G)) * F).sum(axis=0)
    rhs = ph.entropy_potential(qR, n) - ph.entropy_potential(qL, n)
    scale = np.abs(ph.entropy_variables(qR, G) * F).sum(axis=0) + 1.0
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-14


@pytest.mark.parametrize("N", [2, 3, 5])
def test_split_equals_weak_for_the_central_flux_on_hexahedra(N):
    """With F# = (F(qa) + F(qb))/2 and constant metrics, Q + Q^T = B diagonal (Gauss-Lobatto)
    makes the flux-differencing term equal the weak volume term exactly."""
    mesh = make_mesh(3, np.zeros(27, np.int8))
    o = DGOracle(mesh, N)
    U = o.initial_state(tgv_primitive, lambda es: node_noise(3, (N + 1) ** 3, es, amp=5e-2))
    q = o.nodal(U, 3)

    def central(qa, qb, nv):
        return 0.5 * (ph.normal_flux(ph.euler_flux(qa, G), nv) + ph.normal_flux(ph.euler_flux(qb, G), nv))

    rw = o._volume(q, 3)
    rs = o._volume_split(q, 3, two_point=central)
    assert np.max(np.abs(rw - rs)) <= 1e-14 * np.max(np.abs(rw))


def _entropy_rate(o, U, R):
    tot = scale = 0.0
    for e in range(o.mesh.n_elems):
        g = o.elem_geo(e)
        q = np.asarray(o.nodal(U, e), dtype=float)
        w = np.asarray(o.tref[int(o.mesh.elem_type[e])]["w"] * g["J"], dtype=float)
        v = ph.entropy_variables(q, G)
        Re = R[o.offset[e]:o.offset[e + 1]].reshape(5, -1)
        if o.mesh.elem_type[e] != 0:
            Re = Re @ np.asarray(o.tref[int(o.mesh.elem_type[e])]["V"], dtype=float).T
        tot += float(((v * Re).sum(axis=0) * w).sum())
        scale += float((np.abs(v * Re).sum(axis=0) * w).sum())
    return tot, scale


def test_entropy_conservation_on_hexahedra():
    """Periodic hexahedral mesh, split form with the entropy-conservative surface flux: the
    discrete entropy rate sum w J v(q).dq/dt vanishes to rounding; the weak form with the same
    surface flux does not, and the Lax-Friedrichs surface flux dissipates."""
    mesh = make_mesh(3, np.zeros(27, np.int8))
    rates = {}
    for vf, sf in (("split", "ec"), ("weak", "ec"), ("split", "lf")):
        o = DGOracle(mesh, 3, volume_form=vf, surface_flux=sf)
        U = o.initial_state(tgv_primitive, lambda es: node_noise(3, 64, es, amp=5e-2))
        rates[(vf, sf)] = _entropy_rate(o, U, o.residual(U))
    tot, scale = rates[("split", "ec")]
    assert abs(tot) < 1e-14 * scale
    tot, scale = rates[("weak", "ec")]
    assert abs(tot) > 1e-7 * scale
    tot, scale = rates[("split", "lf")]
    assert tot < -1e-4 * scale


@pytest.mark.parametrize("eq", ["euler", "ns"])
def test_split_free_stream_and_conservation_on_mixed_mesh(eq):
    """Constant states stay constant on every element type (the metric average in the
    two-point term is what makes this hold on collapsed elements); the integral of the
    residual vanishes (conservation)."""
    mesh = config_mesh(1)
    o = DGOracle(mesh, 3, equations=eq, volume_form="split")

    def const(x, y, z):
        one = np.ones_like(x)
        return 1.1 * one, 0.3 * one, -0.2 * one, 0.1 * one, 2.0 * one

    R = o.residual(o.initial_state(const))
    assert np.max(np.abs(R)) < 1e-12
    U = o.initial_state(tgv_primitive, lambda es: node_noise(3, 64, es, amp=1e-2))
    R = o.residual(U)
    assert np.max(np.abs(o.integral(R))) < 1e-13 * max(1.0, np.max(np.abs(R)))
