"""Pins of the Hilbert keys, the weighted partition and the Listing 1 attribution."""
import itertools

import numpy as np
import pytest

from oracle import sfc


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5])
def test_hilbert_bijection_and_adjacency(bits):
    n = 1 << bits
    g = np.array(list(itertools.product(range(n), repeat=3)), dtype=np.uint64)[:, ::-1]
    k = sfc.hilbert_keys(g, bits)
    assert sorted(k.tolist()) == list(range(n ** 3))
    o = np.argsort(k)
    steps = np.abs(np.diff(g[o].astype(np.int64), axis=0)).sum(axis=1)
    assert np.all(steps == 1)  # consecutive cells along the curve share a face


def test_hilbert_curve_starts_at_origin():
    g = np.array([[0, 0, 0]], dtype=np.uint64)
    assert int(sfc.hilbert_keys(g, 21)[0]) == 0


def test_quantisation_clamps_and_floors():
    lo = np.array([0.0, 0.0, 0.0])
    c = np.array([[0.0, 0.5, 1.0], [-1e-9, 0.25, 0.999999]])
    q = sfc.quantise(c, lo, 8.0, bits=3)
    assert q.tolist() == [[0, 4, 7], [0, 2, 7]]


def test_stable_order_on_ties():
    keys = np.array([5, 3, 5, 3, 1], dtype=np.uint64)
    assert sfc.sfc_order(keys).tolist() == [4, 1, 3, 0, 2]


def test_partition_hand_example():
    # weights 1 1 1 1 4 1 1 1 1 1 (W = 13), three queues: midpoints (2S+w)/2W * 3
    qb = sfc.partition(np.array([1, 1, 1, 1, 4, 1, 1, 1, 1, 1]), 3)
    assert qb.tolist() == [0, 4, 6, 10]


@pytest.mark.parametrize("seed", range(5))
def test_partition_invariants(seed):
    rng = np.random.default_rng(seed)
    n, Q = int(rng.integers(1, 3000)), int(rng.integers(1, 300))
    w = rng.integers(1, 2000, size=n).astype(np.uint32)
    qb = sfc.partition(w, Q)
    assert qb[0] == 0 and qb[-1] == n and np.all(np.diff(qb) >= 0)
    S = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
    W = int(S[-1])
    loads = S[qb[1:]] - S[qb[:-1]]
    assert loads.sum() == W
    assert np.all(np.abs(loads - W / Q) <= w.max() + 1e-9)


def test_partition_zero_weights():
    # trailing zero weights: their midpoint is W, capped into the last queue; queue_begin[Q] = n
    assert sfc.partition(np.array([1, 1, 0]), 2).tolist() == [0, 1, 3]
    assert sfc.partition(np.array([0, 1, 1]), 2).tolist() == [0, 2, 3]
    assert sfc.partition(np.array([0, 0, 0]), 3).tolist() == [0, 0, 0, 3]
    rng = np.random.default_rng(7)
    for _ in range(20):
        n, Q = int(rng.integers(1, 400)), int(rng.integers(1, 40))
        w = rng.integers(0, 5, size=n).astype(np.uint32)
        w[-int(rng.integers(0, n)):] = 0 if rng.random() < 0.5 else w[-1]
        qb = sfc.partition(w, Q)
        assert qb[0] == 0 and qb[-1] == n and np.all(np.diff(qb) >= 0)
        S = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
        if S[-1]:
            loads = S[qb[1:]] - S[qb[:-1]]
            assert np.all(np.abs(loads - S[-1] / Q) <= w.max() + 1e-9)


def test_partition_exact_beyond_64bit_products():
    """Weights near 2^32 with many queues: Q (2 S + w) exceeds 2^64, the split stays exact
    (every queue load within one element weight of W/Q)."""
    rng = np.random.default_rng(11)
    n, Q = 600_000, 4096
    w = (np.uint64(2 ** 32 - 1) - rng.integers(0, 1000, size=n).astype(np.uint64)).astype(np.uint32)
    qb = sfc.partition(w, Q)
    S = np.concatenate([[0], np.cumsum(w.astype(object))])
    W = S[-1]
    assert Q * 2 * W >= 2 ** 64
    assert qb[0] == 0 and qb[-1] == n and np.all(np.diff(qb) >= 0)
    loads = np.array([S[b] - S[a] for a, b in zip(qb[:-1], qb[1:])], dtype=object)
    assert max(abs(2 * Q * l - 2 * W) for l in loads) <= 2 * Q * int(w.max())


def test_listing1_attribution_hand_example():
    # 3 elements (element 2 modal), 4 sides with SideToElem = [0, 1, 1, 2]
    t = sfc.listing1_attribution(t_elems=3.0, t_sides=4.0, t_modal=2.0,
                                 modal=[False, False, True], side_to_elem=[0, 1, 1, 2], n_elems=3)
    np.testing.assert_allclose(t, [1.0 + 1.0, 1.0 + 2.0, 1.0 + 2.0 + 1.0])
    assert abs(t.sum() - (3.0 + 4.0 + 2.0)) < 1e-15


def test_type_weights():
    w = sfc.type_weights([2.0, 3.0, 2.5, 1.0])
    assert w.tolist() == [1024, 1536, 1280, 512]
