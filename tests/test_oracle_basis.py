"""Pins of the modal bases, nodes and the modal <-> nodal transforms (Algorithm 1)."""
import numpy as np
import pytest

from oracle import basis, geometry
from oracle.geometry import HEX, PRISM, PYR, TET

MODAL = [PRISM, PYR, TET]


@pytest.mark.parametrize("N", range(2, 7))
def test_mode_counts(N):
    n = N + 1
    assert basis.n_modes(TET, N) == n * (n + 1) * (n + 2) // 6
    assert basis.n_modes(PRISM, N) == n * n * (n + 1) // 2
    assert basis.n_modes(PYR, N) == n * (n + 1) * (2 * n + 1) // 6


def _closed_norm2(t, p, q, r):
    # int (1-x)^a (P_n^(a,0))^2 dx = 2^(a+1)/(2n+a+1), collapsed weights of each reference element
    if t == TET:
        return 2 / (2 * p + 1) * 1 / (p + q + 1) * 2 / (2 * (p + q + r) + 3)
    if t == PRISM:
        return 2 / (2 * p + 1) * 2 / (2 * q + 1) * 1 / (p + r + 1)
    m = max(p, q)
    return 2 / (2 * p + 1) * 2 / (2 * q + 1) * 2 / (2 * (m + r) + 3)


@pytest.mark.parametrize("t", MODAL)
@pytest.mark.parametrize("N", [2, 4, 6])
def test_basis_orthonormal_and_closed_form_norms(t, N):
    G = basis.reference_gram(t, N)
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-13)
    Graw = basis.reference_gram(t, N, scaled=False)
    expect = [_closed_norm2(t, *pqr) for pqr in basis.modes(t, N)]
    np.testing.assert_allclose(np.diag(Graw), expect, rtol=1e-13)


def _ref_xi(t, eta):
    return geometry.map_points(geometry.REF_CORNERS[t], eta)


@pytest.mark.parametrize("t", MODAL)
@pytest.mark.parametrize("N", [2, 3, 5])
def test_span_contains_total_degree_polynomials(t, N):
    """P^N(xi) lies in the span of the basis: least-squares fit at the nodes is exact."""
    eta, w = geometry.volume_nodes(t, N + 1)
    xi = _ref_xi(t, eta)
    V = basis.psi(t, N, eta).astype(np.float64)
    xi = xi.astype(np.float64)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1 - a - b):
                f = xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c
                coef, *_ = np.linalg.lstsq(V, f, rcond=None)
                assert np.abs(V @ coef - f).max() < 1e-12


@pytest.mark.parametrize("t", MODAL)
@pytest.mark.parametrize("N", range(2, 7))
def test_mass_matrix_full_rank_with_radau_nodes_singular_with_lobatto(t, N):
    """Reading of the node family: Gauss-Lobatto nodes in a collapsing direction put nodes on
    the collapsed face (J = 0) and make M = V^T W J V singular; left Gauss-Radau there does not."""
    n = N + 1
    eta, w = geometry.volume_nodes(t, n)
    J, _ = geometry.metrics(geometry.REF_CORNERS[t], eta)
    assert np.all(J > 0)
    V = basis.psi(t, N, eta)
    M = (V.T @ (V * (w * J)[:, None])).astype(np.float64)
    assert np.linalg.matrix_rank(M) == V.shape[1]
    assert np.linalg.cond(M) < 1e3
    # all-Lobatto variant
    from oracle import rules
    x, wl = rules.gauss_lobatto(n)
    l, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    e2 = np.stack([x[i.ravel()], x[j.ravel()], x[l.ravel()]], axis=1)
    w2 = wl[i.ravel()] * wl[j.ravel()] * wl[l.ravel()]
    J2, _ = geometry.metrics(geometry.REF_CORNERS[t], e2)
    V2 = basis.psi(t, N, e2)
    M2 = (V2.T @ (V2 * (w2 * J2)[:, None])).astype(np.float64)
    assert np.linalg.matrix_rank(M2, tol=1e-10 * np.abs(M2).max()) < V2.shape[1]


@pytest.mark.parametrize("t", MODAL)
@pytest.mark.parametrize("N", [2, 3, 4])
def test_round_trips(t, N):
    """P V = I (modal -> nodal -> modal), and V P q = q for q in P^N sampled at the nodes."""
    eta, w = geometry.volume_nodes(t, N + 1)
    corners = geometry.REF_CORNERS[t] * np.array([0.7, 1.3, 0.9]) + np.array([0.2, -0.1, 0.4])
    J, _ = geometry.metrics(corners, eta)
    V = basis.psi(t, N, eta).astype(np.float64)
    M = V.T @ (V * (w * J).astype(np.float64)[:, None])
    P = np.linalg.solve(M, V.T * (w * J).astype(np.float64)[None, :])
    np.testing.assert_allclose(P @ V, np.eye(V.shape[1]), atol=1e-12)
    x = geometry.map_points(corners, eta).astype(np.float64)
    q = 1 + x[:, 0] ** N - 2 * x[:, 1] * x[:, 2] ** (N - 1) + x[:, 0] * x[:, 1]
    np.testing.assert_allclose(V @ (P @ q), q, atol=1e-12 * np.abs(q).max())


@pytest.mark.parametrize("t", [HEX, PRISM, PYR, TET])
def test_element_volume_and_metric_identity(t):
    """sum_m w_m J_m is the exact element volume; sum_a d/deta_a a^a = 0 at every node."""
    from workloads import make_mesh
    kinds = np.full(27, t, dtype=np.int8)
    mesh = make_mesh(3, kinds, L=3.0)
    vol = {HEX: 1.0, PRISM: 0.5, PYR: 1 / 6, TET: 1 / 6}[t]
    n = 4
    eta, w = geometry.volume_nodes(t, n)
    dL = geometry.lagrange3d_grad(t, n, eta)  # [m, k, a]
    for e in range(min(mesh.n_elems, 12)):
        J, acon = geometry.metrics(mesh.corner_xyz[e], eta)
        assert abs((w * J).sum() - vol) < 1e-13
        div = np.einsum("mka,kac->mc", dL, acon)
        assert np.abs(div).max() < 1e-12
