"""Workload generator: element counts of the configured meshes and the seeded noise stream."""
import numpy as np

from workloads import config_mesh, make_mesh, node_noise


def test_config1_counts():
    m = config_mesh(1)
    # 32 hex cells, 16 prism-split (2 each), 8 pyramid-split (6 each), 8 tet-split (6 each)
    assert m.type_counts().tolist() == [32, 32, 48, 48]


def test_config4_counts():
    m = config_mesh(4)
    assert m.type_counts().tolist() == [3456, 6912, 20736, 20736]


def test_noise_subsets_match_full_stream():
    full = node_noise(1, 27, np.arange(20))
    sub = node_noise(1, 27, [7, 3, 4, 19])
    assert np.array_equal(sub, full[[7, 3, 4, 19]])
    assert np.abs(full).max() <= 1e-3


def test_split_elements_have_positive_orientation():
    from oracle import geometry
    m = make_mesh(3, np.arange(27) % 4)
    eta = np.array([[0.0, 0.0, -0.5]])
    for e in range(m.n_elems):
        J, _ = geometry.metrics(m.corner_xyz[e], eta)
        assert J[0] > 0


def test_motion_moves_every_vertex_alike():
    """workloads.motion gives every corner that is one vertex (periodic images included) the same
    displacement, to the 1e-12 of the largest entry that pdg_set_motion checks, on a mixed mesh."""
    import numpy as np
    from workloads import make_mesh, motion
    rng = np.random.Generator(np.random.PCG64(4))
    m = make_mesh(4, rng.permutation(np.arange(64) % 4).astype(np.int8))
    d = motion(m, 0.2).reshape(-1, 3)
    ids = m.elem_corner.ravel()
    tol = 1e-12 * np.abs(d).max()
    for v in np.unique(ids):
        rows = d[ids == v]
        assert np.abs(rows - rows[0]).max() <= tol
