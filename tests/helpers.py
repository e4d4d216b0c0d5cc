"""Shared helpers of the test suite (no arithmetic of the method)."""
import numpy as np


def varwise_rel_err(a, b, offsets):
    """max over the 5 variables of max|a_v - b_v| / max|b_v|, on states with per-element
    blocks [5][ndof] at `offsets`."""
    a = np.asarray(a)
    b = np.asarray(b)
    sizes = np.diff(offsets) // 5
    var = np.concatenate([np.repeat(np.arange(5), s) for s in sizes])
    worst = 0.0
    for v in range(5):
        m = var == v
        den = np.abs(b[m]).max()
        num = np.abs(a[m] - b[m]).max()
        worst = max(worst, num / den if den > 0 else num)
    return worst


def stored_nodal(q_input_order, perm):
    """[n_elems, 5, n^3] nodal values in input order -> stored (library) order."""
    return np.ascontiguousarray(np.asarray(q_input_order)[perm])


def ulp_floor(residual_fn, U0, offsets, draws=2, seed=1):
    """FP64 conditioning floor of a map at U0: the per-variable relative change of
    residual_fn(U) when every entry of U0 is perturbed by about one unit in the last place.
    Any FP64 evaluation of the map carries errors of this size, whatever its operation order."""
    import numpy as _np
    base = residual_fn(U0)
    rng = _np.random.default_rng(seed)
    vals = []
    for _ in range(draws):
        U1 = U0 * (1.0 + 2.2e-16 * rng.standard_normal(U0.shape))
        vals.append(varwise_rel_err(residual_fn(U1), base, offsets))
    return float(_np.mean(vals)), base

