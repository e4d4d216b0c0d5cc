"""Failure detection through the C ABI: a blown-up state (NaN or infinity) is reported with the
first bad stored index, broken meshes are rejected with PDG_EMESH (a face shared by three
elements, a hole, an inverted element), and a curved element on a mesh with
quadrilateral-triangle mortars with PDG_ENOTSUP.
Every case is an invalid input the library itself turns into an error code; no kernel is made
to fail."""
import numpy as np
import pytest

from workloads import make_mesh
from workloads.device import tgv_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mesh():
    rng = np.random.Generator(np.random.PCG64(11))
    return make_mesh(3, rng.permutation(np.arange(27) % 4).astype(np.int8))


def _create(et, ec, xyz, cen, nv, N=2):
    from paper_2511_08020_amd.binding import PolyDG
    return PolyDG(et, ec, xyz, cen, nv, N, p_ref=1.0 / (1.4 * 0.01))


def test_nonfinite_state_is_reported_with_its_first_index():
    from paper_2511_08020_amd.binding import PDG_ENONFINITE, PdgError
    print("case: finiteness check, 3^3 mixed cells, N=2", flush=True)
    m = _mesh()
    dg = _create(m.elem_type, m.elem_corner, m.corner_xyz, m.centroid, m.n_vertices)
    U = tgv_state(dg)
    assert dg.check_finite(U) is None
    n = U.numel()
    for bad, val in ((n - 1, float("inf")), (n // 3, float("nan")), (7, float("-inf"))):
        U2 = U.clone()
        U2[bad] = val
        U2[min(n - 1, bad + 5)] = float("nan")
        with pytest.raises(PdgError) as ei:
            dg.check_finite(U2)
        assert ei.value.code == PDG_ENONFINITE
        assert f"index {bad}" in str(ei.value)
    # a step taken from a blown-up state stays blown up, and the check catches it
    U3 = U.clone()
    U3[100] = float("nan")
    K = dg.zeros_state()
    dg.rk_steps(U3, K, 1e-4, 1)
    with pytest.raises(PdgError):
        dg.check_finite(U3)


def _expect_mesh_error(et, ec, xyz, cen, nv):
    from paper_2511_08020_amd.binding import PDG_EMESH, PdgError
    with pytest.raises(PdgError) as ei:
        _create(et, ec, xyz, cen, nv)
    print("rejected:", ei.value, flush=True)
    assert ei.value.code == PDG_EMESH


def test_face_shared_by_three_elements_is_rejected():
    print("case: duplicated element", flush=True)
    m = _mesh()
    i = [*range(m.n_elems), 0]
    _expect_mesh_error(m.elem_type[i], m.elem_corner[i], m.corner_xyz[i], m.centroid[i], m.n_vertices)


def test_hole_is_rejected():
    print("case: element removed", flush=True)
    m = _mesh()
    i = list(range(1, m.n_elems))
    _expect_mesh_error(m.elem_type[i], m.elem_corner[i], m.corner_xyz[i], m.centroid[i], m.n_vertices)


def test_inverted_element_is_rejected():
    """A hexahedron mirrored in its first reference direction has a negative Jacobian."""
    print("case: inverted hexahedron", flush=True)
    m = _mesh()
    e = int(np.nonzero(m.elem_type == 0)[0][0])
    ec, xyz = m.elem_corner.copy(), m.corner_xyz.copy()
    swap = [1, 0, 3, 2, 5, 4, 7, 6]
    ec[e] = ec[e][swap]
    xyz[e] = xyz[e][swap]
    _expect_mesh_error(m.elem_type, ec, xyz, m.centroid, m.n_vertices)


def test_curved_element_next_to_mortars_is_refused():
    """Moving one vertex of a hexahedron (in every element that holds it) makes the elements
    around it trilinear.  Curved elements are taken on conforming meshes only (a bilinear
    quadrilateral has no straight diagonal for a mortar's two triangles); this mesh has
    hexahedron-tetrahedron mortars, so creation fails with PDG_ENOTSUP (not a wrong residual)."""
    print("case: one vertex moved off the affine grid", flush=True)
    from paper_2511_08020_amd.binding import PDG_ENOTSUP, PdgError
    m = _mesh()
    e = int(np.nonzero(m.elem_type == 0)[0][0])
    vid = int(m.elem_corner[e][7])
    xyz = m.corner_xyz.copy()
    h = m.L / m.C
    xyz[m.elem_corner == vid] += np.array([0.1, 0.05, -0.07]) * h
    with pytest.raises(PdgError) as ei:
        _create(m.elem_type, m.elem_corner, xyz, m.centroid, m.n_vertices)
    print("refused:", ei.value, flush=True)
    assert ei.value.code == PDG_ENOTSUP
