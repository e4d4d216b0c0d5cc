"""Oracle pins on curved (trilinear) elements: every vertex of a periodic mesh moved by a smooth
periodic field (workloads.deformed), so hexahedra are trilinear, quadrilateral faces bilinear
patches with a normal that turns across the face, and the mass matrix V^T W J V varies from
element to element through the Jacobian at the nodes (Alg. 1).  Each check is against something
the oracle does not compute itself: the divergence theorem for a closed surface, an independent
tensor Gauss quadrature of the trilinear Jacobian, the volume of the periodic box, free stream,
discrete conservation and convergence to the exact time derivative."""
import numpy as np
import pytest

from oracle.dg import DGOracle
from workloads import density_wave_primitive, deformed, make_mesh, node_noise, tgv_primitive

AMP = 0.15


def _mesh(t, C=3, amp=AMP):
    return deformed(make_mesh(C, np.full(C ** 3, t, np.int8)), amp)


def _trilinear_volume(X):
    """Volume of the trilinear hexahedron with corners X[8][3] (corner slot a + 2b + 4c at
    reference (2a-1, 2b-1, 2c-1)) by a 6-point Gauss-Legendre tensor rule of det(dx/dxi)."""
    g, w = np.polynomial.legendre.leggauss(6)
    vol = 0.0
    for i, xi in enumerate(g):
        for j, eta in enumerate(g):
            for k, zeta in enumerate(g):
                D = np.zeros((3, 3))
                for slot in range(8):
                    a, b, c = slot & 1, (slot >> 1) & 1, (slot >> 2) & 1
                    sa, sb, sc = 2 * a - 1, 2 * b - 1, 2 * c - 1
                    fa, fb, fc = (1 + sa * xi) / 2, (1 + sb * eta) / 2, (1 + sc * zeta) / 2
                    D[:, 0] += X[slot] * sa / 2 * fb * fc
                    D[:, 1] += X[slot] * fa * sb / 2 * fc
                    D[:, 2] += X[slot] * fa * fb * sc / 2
                vol += w[i] * w[j] * w[k] * np.linalg.det(D)
    return vol


@pytest.mark.parametrize("t", [0, 1, 2])
def test_curved_faces_close_and_bend(t):
    """Per element, the outward n dS of all its faces sums to zero (the divergence theorem for a
    constant field; exact for bilinear patches under the Gauss-Lobatto face rule), and some
    quadrilateral face normal turns by more than 0.01 rad across the face (the faces are not flat:
    a parallelogram stand-in would fail the first check)."""
    m = _mesh(t)
    ora = DGOracle(m, 3)
    worst, turn = 0.0, 0.0
    for e in range(m.n_elems):
        acc, area = np.zeros(3), 0.0
        for fi, side in ora.elem_faces[e]:
            fg = ora.face_geo(fi)
            nout = fg["normal"] if side == 0 else -fg["normal"]
            acc += (nout * fg["ws"][None, :]).sum(axis=1)
            area += fg["ws"].sum()
            if ora.faces[fi].kind == "quad":
                c = np.clip(nout.T @ nout, -1.0, 1.0)
                turn = max(turn, float(np.arccos(c.min())))
        worst = max(worst, float(np.abs(acc).max() / area))
    print(f"closed-surface residual {worst:.2e}, largest normal turn {turn:.3f} rad")
    assert worst < 1e-14
    assert turn > 0.01


def test_curved_hexahedron_volumes():
    """Sum of w_k J_k over each element's nodes equals an independent tensor Gauss quadrature of
    the trilinear Jacobian (exact for N >= 2 nodes per direction and for the 6-point rule), and the
    elements tile the periodic box: total volume L^3."""
    m = _mesh(0)
    ora = DGOracle(m, 3)
    total = 0.0
    for e in range(m.n_elems):
        g = ora.elem_geo(e)
        v_ora = float(np.sum(ora.tref[0]["w"] * g["J"]))
        v_ind = _trilinear_volume(m.corner_xyz[e])
        assert abs(v_ora - v_ind) <= 1e-13 * v_ind
        total += v_ora
    assert abs(total - m.L ** 3) <= 1e-12 * m.L ** 3


@pytest.mark.parametrize("t,equations", [(0, "euler"), (0, "ns"), (1, "euler"), (2, "ns")])
def test_curved_free_stream(t, equations):
    """A constant state has zero residual on curved elements (per-node metric terms and per-point
    face normals of the same trilinear map): below 1e-13 of the pressure scale."""
    m = _mesh(t)
    ora = DGOracle(m, 3, equations=equations)
    p = 1.0 / (1.4 * 0.01)

    def prim(x, y, z):
        o = np.ones_like(x)
        return o, 0.3 * o, -0.2 * o, 0.1 * o, p * o

    R = ora.residual(ora.initial_state(prim))
    assert np.abs(R).max() < 1e-13 * p


@pytest.mark.parametrize("equations", ["euler", "ns"])
def test_curved_conservation(equations):
    """The integral of dU/dt over the mesh vanishes for a noisy state (the two sides of every
    curved face use the same per-point normals and weights)."""
    m = _mesh(0)
    N = 3
    ora = DGOracle(m, N, equations=equations)
    U = ora.initial_state(tgv_primitive, lambda es: node_noise(2, (N + 1) ** 3, es))
    R = ora.residual(U)
    tot = np.asarray(ora.integral(R), dtype=float)
    scale = np.asarray(ora.integral(np.abs(R)), dtype=float)
    assert np.all(np.abs(tot) <= 1e-12 * scale), (tot, scale)


@pytest.mark.parametrize("N,order", [(2, 1.6), (3, 2.4)])
def test_curved_hexahedra_truncation_converges(N, order):
    """dU/dt of the projected density wave against its exact time derivative on curved hexahedra
    (the same absolute deformation on 3^3 and 6^3 cells): measured orders 1.76 (N = 2) and 2.54
    (N = 3); a wrong metric term or face normal stops convergence."""
    exR = lambda x, y, z: np.stack([-3 * 0.5 * 0.2 * np.cos(x + y + z)] * 5)  # noqa: E731
    errs = []
    for C in (3, 6):
        o = DGOracle(_mesh(0, C, AMP * C / 3), N)
        U = o.initial_state(density_wave_primitive)
        errs.append(o.l2_error(o.residual(U), exR, 0))
    rate = np.log(errs[0] / errs[1]) / np.log(2.0)
    print(f"N={N}: errors {errs[0]:.3e} -> {errs[1]:.3e}, order {rate:.2f}")
    assert rate >= order


def test_curved_split_form_conserves_entropy():
    """The split form with the entropy-conservative surface flux on curved hexahedra: the discrete
    entropy rate sum w J v(q).dq/dt vanishes to rounding (the two-point fluxes average the two
    nodes' contravariant vectors, which the trilinear map's metric identity makes consistent);
    the weak form with the same surface flux does not (measured 9e-19 against 3e-5)."""
    from test_oracle_split import _entropy_rate
    m = _mesh(0)
    rates = {}
    for vf in ("split", "weak"):
        o = DGOracle(m, 3, volume_form=vf, surface_flux="ec")
        U = o.initial_state(tgv_primitive, lambda es: node_noise(3, 64, es, amp=5e-2))
        rates[vf] = _entropy_rate(o, U, o.residual(U))
    tot, scale = rates["split"]
    assert abs(tot) < 1e-14 * scale
    tot, scale = rates["weak"]
    assert abs(tot) > 1e-7 * scale
