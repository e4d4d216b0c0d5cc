"""Pins of the oracle adjoint: the pointwise Jacobians against central differences of the
flux functions in extended precision, the residual's vector-Jacobian product against
central-difference Jacobian-vector products of the residual (the dot-product test
<lam, J v> = <J^T lam, v>), the element-subset form against the full form, and the
gradient through LSERK4 steps against differences of the objective."""
import numpy as np
import pytest

from oracle import adjoint, physics
from oracle.dg import DGOracle
from workloads import make_mesh, node_noise, tgv_primitive

LD = np.longdouble


def _states(seed, n=7):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.3 * rng.random(n)
    u = 0.4 * rng.standard_normal((3, n))
    p = 1.0 + rng.random(n)
    q = physics.primitive_to_conservative(rho, u[0], u[1], u[2], p, 1.4)
    return q.astype(LD)


def _fd(fun, q, h=LD(1e-7)):
    """Central differences d fun / d q[w] in extended precision: array [..., w, points]."""
    cols = []
    for w in range(q.shape[0]):
        e = np.zeros_like(q)
        e[w] = h * np.maximum(1.0, np.abs(q[w]))
        cols.append((fun(q + e) - fun(q - e)) / (2 * e[w]))
    return np.stack(cols, axis=-2)


def _close(a, b, tol=1e-9):
    a = np.asarray(a, dtype=LD)
    b = np.asarray(b, dtype=LD)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)) < tol


def test_euler_flux_jacobian():
    q = _states(1)
    assert _close(physics.euler_flux_jacobian(q, 1.4), _fd(lambda x: physics.euler_flux(x, 1.4), q))


def test_lax_friedrichs_jacobians():
    qL, qR = _states(2), _states(3)
    nrm = np.array([0.48, -0.6, 0.64], dtype=LD)
    JL, JR = physics.lax_friedrichs_jacobians(qL, qR, nrm, 1.4)
    assert _close(JL, _fd(lambda x: physics.lax_friedrichs(x, qR, nrm, 1.4), qL))
    assert _close(JR, _fd(lambda x: physics.lax_friedrichs(qL, x, nrm, 1.4), qR))


def test_lifting_jacobian():
    q = _states(4)
    assert _close(physics.lifting_jacobian(q, 1.4, 1.0),
                  _fd(lambda x: physics.lifting_variables(x, 1.4, 1.0), q))


def test_viscous_flux_jacobians():
    q = _states(5)
    grad = np.asarray(np.random.default_rng(6).standard_normal((4, 3, q.shape[1])), dtype=LD)
    dq, dg = physics.viscous_flux_jacobians(q, grad, 1.4, 0.05, 0.71, 1.0)
    assert _close(dq, _fd(lambda x: physics.viscous_flux(x, grad, 1.4, 0.05, 0.71, 1.0), q))
    # linear in the gradients: the Jacobian reproduces the flux exactly
    Fv = physics.viscous_flux(q, grad, 1.4, 0.05, 0.71, 1.0)
    assert _close(np.einsum("cvsdp,sdp->cvp", dg, grad), Fv, 1e-15)


def _mixed(C, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_mesh(C, rng.permutation(np.arange(C ** 3) % 4).astype(np.int8))


@pytest.fixture(scope="module")
def mesh3():
    return _mixed(3)


def _setup(mesh, eq, N, mu):
    o = DGOracle(mesh, N, equations=eq, mu=mu)
    U = o.initial_state(tgv_primitive, lambda es: node_noise(1, (N + 1) ** 3, es))
    return o, U


# The residual has kinks (|u.n| and the maximum wave speed); the seeded states keep every
# face point at least ~1e-7 away from them relative to the step below, so the differences
# see a smooth function and agree to the rounding of the FP64 residual (~1e-8 here).
@pytest.mark.parametrize("eq,N,mu", [("euler", 3, 0.0), ("ns", 2, 0.05), ("ns", 3, 1.0 / 1600.0)])
def test_vjp_dot_product(mesh3, eq, N, mu):
    o, U = _setup(mesh3, eq, N, mu)
    rng = np.random.default_rng(11)
    lam = rng.standard_normal(o.size)
    g = adjoint.vjp(o, U, lam)
    for _ in range(2):
        v = rng.standard_normal(o.size)
        h = 1e-8
        jv = (o.residual(U + h * v) - o.residual(U - h * v)) / (2 * h)
        a, b = lam @ jv, g @ v
        assert abs(a - b) <= 1e-6 * abs(a), (a, b)


def test_vjp_subset(mesh3):
    o, U = _setup(mesh3, "ns", 2, 0.05)
    lam = np.random.default_rng(12).standard_normal(o.size)
    full = adjoint.vjp(o, U, lam)
    S = [0, 17, 40]
    part = adjoint.vjp(o, U, lam, elems=S)
    for e in S:
        a, b = o.offset[e], o.offset[e + 1]
        assert np.allclose(part[a:b], full[a:b], rtol=0, atol=1e-12 * np.abs(full).max())
    assert np.isnan(part[o.offset[1]])


def test_kinetic_energy_grad(mesh3):
    o, U = _setup(mesh3, "euler", 2, 0.0)
    v = np.random.default_rng(13).standard_normal(o.size)
    g = adjoint.kinetic_energy_grad(o, U)
    h = 1e-6
    fd = (o.kinetic_energy(U + h * v) - o.kinetic_energy(U - h * v)) / (2 * h)
    assert abs(g @ v - fd) <= 1e-7 * abs(fd)


def test_rk_vjp(mesh3):
    """d E(U_2) / d U_0 through two LSERK4 steps, against central differences of E."""
    o, U = _setup(mesh3, "ns", 2, 0.05)
    dt = 0.02
    U2, _ = o.rk_steps(U, dt, 2)
    grad = adjoint.rk_vjp(o, U, dt, 2, adjoint.kinetic_energy_grad(o, U2))
    v = np.random.default_rng(14).standard_normal(o.size)
    h = 1e-7
    Ep = o.kinetic_energy(o.rk_steps(U + h * v, dt, 2)[0])
    Em = o.kinetic_energy(o.rk_steps(U - h * v, dt, 2)[0])
    fd = (Ep - Em) / (2 * h)
    assert abs(grad @ v - fd) <= 1e-6 * abs(fd), (grad @ v, fd)
