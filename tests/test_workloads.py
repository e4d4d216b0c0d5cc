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
