"""Host logic of the dynamic load balance (pdg_balance_weights, no device): per-type costs
fitted from per-queue times, attribution of queue time to elements, integer weights, and the
measured imbalance; the re-partition of the weights (the oracle's prefix-sum split) balances
the true loads.  Synthetic per-queue times stand in for the queue kernels' device timers."""
import numpy as np
import pytest

from oracle import sfc
from paper_2511_08020_amd.binding import PdgError, balance_weights

# cost per element and phase (trace, volume, surface) of hex, prism, pyramid, tet: the modal
# types cost several times a hexahedron, as the paper's transform overhead makes them
COSTS = np.array([[1.0, 3.0, 2.5, 1.5],
                  [4.0, 19.0, 15.0, 8.0],
                  [2.0, 9.0, 7.0, 4.0]])


def _mesh_types(n, seed):
    """Types along the Hilbert order: hex runs and modal clusters, as around a tet-split sphere."""
    rng = np.random.Generator(np.random.PCG64(seed))
    et = np.zeros(n, dtype=np.int8)
    pos = 0
    while pos < n:
        run = int(rng.integers(5, 60))
        if rng.random() < 0.4:
            et[pos:pos + run] = rng.integers(1, 4, size=min(run, n - pos))
        pos += run
    return et


def _queue_ms(et, qb, costs):
    nq = len(qb) - 1
    ms = np.zeros((3, nq))
    for q in range(nq):
        seg = et[qb[q]:qb[q + 1]]
        for ph in range(3):
            ms[ph, q] = costs[ph][seg].sum()
    return ms


def _imbalance(ms):
    return ms.max(axis=1).sum() / ms.mean(axis=1).sum() - 1.0


def test_fit_recovers_type_costs_and_weights():
    n, nq = 3000, 48
    et = _mesh_types(n, 1)
    qb = np.linspace(0, n, nq + 1).astype(np.int32)
    ms = _queue_ms(et, qb, COSTS)
    w, tc, imb = balance_weights(et, qb, ms)
    assert np.allclose(tc, COSTS, rtol=1e-8)
    assert imb == pytest.approx(_imbalance(ms), rel=1e-12)
    tot = COSTS.sum(axis=0)[et]
    expect = np.maximum(1, np.round(1024 * tot / tot.mean()))
    assert np.array_equal(w, expect.astype(np.uint32))


def test_repartition_balances_true_loads():
    """Unit weights give a large imbalance; one rebalance from the measured times brings the
    true per-queue loads to within the granularity of single elements."""
    n, nq = 4000, 32
    et = _mesh_types(n, 2)
    qb0 = sfc.partition(np.ones(n, np.uint32), nq).astype(np.int32)
    ms0 = _queue_ms(et, qb0, COSTS)
    before = _imbalance(ms0)
    assert before > 0.15
    w, _, imb = balance_weights(et, qb0, ms0)
    assert imb == pytest.approx(before, rel=1e-12)
    qb1 = sfc.partition(w, nq).astype(np.int32)
    after = _imbalance(_queue_ms(et, qb1, COSTS))
    heaviest = COSTS.sum(axis=0).max()
    mean_load = COSTS.sum(axis=0)[et].sum() / nq
    assert after < 0.25 * before
    assert after <= 2 * heaviest / mean_load


def test_spatial_variation_of_one_type():
    """A single-type mesh whose cost varies along the curve (e.g. boundary work): the time of
    each queue is shared equally by its elements, so weights follow the per-queue average."""
    n, nq = 1200, 12
    et = np.zeros(n, dtype=np.int8)
    qb = np.linspace(0, n, nq + 1).astype(np.int32)
    per_q = 1.0 + np.arange(nq) / nq
    ms = np.stack([per_q * 100.0, per_q * 400.0, per_q * 200.0])
    w, tc, imb = balance_weights(et, qb, ms)
    cost = np.repeat(per_q * 700.0 / 100.0, 100)
    assert np.array_equal(w, np.maximum(1, np.round(1024 * cost / cost.mean())).astype(np.uint32))
    assert tc[:, 1:].max() == 0.0 and np.all(tc[:, 0] > 0)
    assert imb == pytest.approx(per_q.max() / per_q.mean() - 1.0, rel=1e-12)


def test_nonnegative_fit():
    """Times that a plain least-squares fit explains with a negative pyramid cost: the fit keeps
    every cost positive and the attributed element costs still reproduce each queue's time."""
    et = np.array([0] * 10 + [2] * 10 + [0, 2] * 5, dtype=np.int8)
    qb = np.array([0, 10, 20, 30], dtype=np.int32)
    ms = np.array([[10.0, 0.5, 3.0]] * 3)    # unconstrained fit: hex 0.925, pyramid -0.025
    w, tc, _ = balance_weights(et, qb, ms)
    assert np.allclose(tc[:, 0], 115.0 / 125.0, rtol=1e-12)      # hex fitted alone
    assert np.allclose(tc[:, 2], 1e-3 * tc[:, 0], rtol=1e-12)    # pyramid kept at the floor
    assert np.all(tc[:, [1, 3]] == 0)
    # element weights of a queue sum to its share of the total time
    tot = ms.sum(axis=0)
    share = np.array([w[qb[q]:qb[q + 1]].sum() for q in range(3)], dtype=float)
    assert np.allclose(share / share.sum(), tot / tot.sum(), rtol=0.02)


def test_balanced_times_give_zero_imbalance():
    n, nq = 800, 16
    et = _mesh_types(n, 3)
    qb = np.linspace(0, n, nq + 1).astype(np.int32)
    ms = np.full((3, nq), 2.0)
    _, _, imb = balance_weights(et, qb, ms)
    assert imb == pytest.approx(0.0, abs=1e-15)


def test_empty_queues_are_ignored_in_attribution():
    et = _mesh_types(300, 4)
    qb = np.array([0, 0, 100, 100, 300, 300], dtype=np.int32)
    ms = _queue_ms(et, qb, COSTS)
    ms[:, [0, 2, 4]] = 0.01            # launch overhead of empty workgroups
    w, tc, _ = balance_weights(et, qb, ms)
    assert np.all(w >= 1) and w.shape == (300,)


@pytest.mark.parametrize("case", ["schedule_end", "decreasing", "type", "negative", "nan", "zero", "shape"])
def test_invalid_inputs(case):
    n, nq = 100, 4
    et = np.zeros(n, dtype=np.int8)
    qb = np.array([0, 25, 50, 75, 100], dtype=np.int32)
    ms = np.ones((3, nq))
    if case == "schedule_end":
        qb = np.array([0, 25, 50, 75, 99], dtype=np.int32)
    elif case == "decreasing":
        qb = np.array([0, 50, 25, 75, 100], dtype=np.int32)
    elif case == "type":
        et[7] = 4
    elif case == "negative":
        ms[1, 2] = -1.0
    elif case == "nan":
        ms[0, 0] = np.nan
    elif case == "zero":
        ms[:] = 0.0
    elif case == "shape":
        with pytest.raises(ValueError):
            balance_weights(et, qb, np.ones((3, nq + 1)))
        return
    with pytest.raises(PdgError):
        balance_weights(et, qb, ms)


def test_attribution_reproduces_listing1_when_loop_costs_follow_type():
    """The paper's attribution (Listing 1) shares each rank's loop time among the elements taking
    part: t_elems / nElems to every element, t_modal / nModalElems to every modal element, and
    t_sides / nSides to the element of every side.  With queues as ranks and per-queue loop
    timers generated by such loops (element-loop cost a, modal cost b, cost c per side, sides
    per element fixed by the type), the per-type fit of pdg_balance_weights attributes to every
    element the Listing 1 time, exactly up to one deliberate difference: a type the fit finds no
    time for in a phase (hexahedra in the modal loop) keeps a floor of 1e-3 of that phase's
    largest type cost, so no element's share of a queue's time is exactly zero."""
    n, nq = 2400, 40
    et = _mesh_types(n, 5)
    sides = np.array([6, 5, 5, 4])[et]
    modal = et != 0
    qb = np.linspace(0, n, nq + 1).astype(np.int32)
    a, b, c = 2.0, 7.0, 0.5
    ms = np.zeros((3, nq))
    t_listing1 = np.zeros(n)
    for q in range(nq):
        seg = slice(qb[q], qb[q + 1])
        ne, nm, ns = qb[q + 1] - qb[q], int(modal[seg].sum()), int(sides[seg].sum())
        t_E, t_M, t_S = a * ne, b * nm, c * ns
        ms[:, q] = (t_S, t_E, t_M)        # phases: side loop, element loop, modal loop
        ste = np.repeat(np.arange(ne), sides[seg])
        t_listing1[seg] = sfc.listing1_attribution(t_E, t_S, t_M, modal[seg], ste, ne)
    w, tc, _ = balance_weights(et, qb, ms)
    np.testing.assert_allclose(tc[:2], [[6 * c, 5 * c, 5 * c, 4 * c], [a, a, a, a]], rtol=1e-10)
    np.testing.assert_allclose(tc[2], [1e-3 * b, b, b, b], rtol=1e-10)
    floor = np.where(et == 0, 1e-3 * b, 0.0)
    t_product = tc.sum(axis=0)[et]
    np.testing.assert_allclose(t_product - floor, t_listing1, rtol=1e-10)
    # the integer weights against those of the Listing 1 times (the floor shifts them by < 1 %)
    assert np.abs(w / np.round(1024 * t_listing1 / t_listing1.mean()) - 1).max() < 1e-2


def test_attribution_resolves_type_costs_that_listing1_averages():
    """Where they differ: when the element loop costs differ by type, Listing 1 gives every
    element of a rank the rank's average element-loop time, while the per-type fit recovers the
    per-type costs (the modal overhead inside the element loop is resolved per type)."""
    n, nq = 2400, 40
    et = _mesh_types(n, 6)
    qb = np.linspace(0, n, nq + 1).astype(np.int32)
    a_t = np.array([1.0, 4.0, 3.0, 2.0])
    ms = np.zeros((3, nq))
    for q in range(nq):
        ms[1, q] = a_t[et[qb[q]:qb[q + 1]]].sum()
    _, tc, _ = balance_weights(et, qb, ms)
    np.testing.assert_allclose(tc[1], a_t, rtol=1e-8)
    q = int(np.argmax([len(set(et[qb[i]:qb[i + 1]].tolist())) for i in range(nq)]))
    seg = et[qb[q]:qb[q + 1]]
    t1 = sfc.listing1_attribution(ms[1, q], 0.0, 0.0, seg != 0, [], seg.size)
    assert np.ptp(t1) == 0.0 and np.ptp(tc[1][seg]) > 0.0
