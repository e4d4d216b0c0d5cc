"""Hilbert space-filling-curve keys, SFC order, weighted contiguous partition (integer work).

Test infrastructure of the oracle.  The paper orders elements along a Hilbert curve and
splits the ordered list into contiguous, non-overlapping segments (Sec. 3, Fig. 1a); the
load per element comes from timers attributed by loop participation (Listing 1).

Keys: each centroid coordinate is quantised with one FP64 subtraction and one FP64
multiplication, k_a = min(floor((c_a - lo_a) * scale), 2^b - 1), b = 21, and the three
b-bit integers are mapped to a 3b-bit Hilbert index with J. Skilling's transpose method
("Programming the Hilbert curve", AIP Conf. Proc. 707, 2004): undo excess work, Gray
encode, then interleave the transposed bits most significant first in axis order x, y, z.
"""
from __future__ import annotations

import numpy as np

BITS = 21


def quantise(centroid, lo, scale, bits=BITS):
    """Integer cell coordinates of each centroid (uint64 [n, 3])."""
    c = np.asarray(centroid, dtype=np.float64)
    v = np.floor((c - np.asarray(lo, np.float64)[None, :]) * np.float64(scale))
    v = np.clip(v, 0, (1 << bits) - 1)
    return v.astype(np.uint64)


def axes_to_transpose(X, bits):
    """Skilling's AxestoTranspose on the columns of X (uint64 [n, 3]), vectorised over rows."""
    X = X.copy()
    n = X.shape[1]
    M = np.uint64(1 << (bits - 1))
    Q = M
    while Q > 1:
        P = Q - np.uint64(1)
        for i in range(n):
            hit = (X[:, i] & Q) != 0
            # invert low bits of X0 where bit Q of Xi is set
            X[hit, 0] ^= P
            # exchange low bits of X0 and Xi elsewhere
            miss = ~hit
            t = (X[miss, 0] ^ X[miss, i]) & P
            X[miss, 0] ^= t
            X[miss, i] ^= t
        Q >>= np.uint64(1)
    for i in range(1, n):
        X[:, i] ^= X[:, i - 1]
    t = np.zeros(X.shape[0], dtype=np.uint64)
    Q = M
    while Q > 1:
        hit = (X[:, n - 1] & Q) != 0
        t[hit] ^= Q - np.uint64(1)
        Q >>= np.uint64(1)
    for i in range(n):
        X[:, i] ^= t
    return X


def interleave(T, bits):
    key = np.zeros(T.shape[0], dtype=np.uint64)
    for j in range(bits - 1, -1, -1):
        for i in range(T.shape[1]):
            key = (key << np.uint64(1)) | ((T[:, i] >> np.uint64(j)) & np.uint64(1))
    return key


def hilbert_keys(ints, bits=BITS):
    return interleave(axes_to_transpose(np.asarray(ints, dtype=np.uint64), bits), bits)


def bbox_scale(centroid, bits=BITS):
    """lo = componentwise minimum, scale = 2^bits / (largest extent) (isotropic)."""
    c = np.asarray(centroid, dtype=np.float64)
    lo = c.min(axis=0)
    ext = float((c.max(axis=0) - lo).max())
    scale = float(1 << bits) / ext if ext > 0 else 1.0
    return lo, scale


def sfc_keys(centroid, lo, scale, bits=BITS):
    return hilbert_keys(quantise(centroid, lo, scale, bits), bits)


def sfc_order(keys):
    """Stable sort by (key, input index): perm[i] = input index of the i-th element."""
    return np.argsort(np.asarray(keys, dtype=np.uint64), kind="stable")


# ------------------------------------------------------------------------ costs and partition

def listing1_attribution(t_elems, t_sides, t_modal, modal, side_to_elem, n_elems):
    """Per-element time from loop timers, attributed by loop participation (Listing 1):
    every element gets t_elems/nElems, every modal element t_modal/nModalElems, and the
    element SideToElem(s) of every side s gets t_sides/nSides."""
    modal = np.asarray(modal, dtype=bool)
    t = np.full(n_elems, t_elems / n_elems)
    nm = int(modal.sum())
    if nm:
        t[modal] += t_modal / nm
    ste = np.asarray(side_to_elem)
    for e in ste:
        t[e] += t_sides / ste.size
    return t


def type_weights(cost_per_elem, scale=1024):
    """Integer weights w_t = max(1, round(scale * c_t / c_hex)) from per-type costs (c_hex replaced
    by the smallest positive cost without hexahedra; ties round to even; capped at 2^24 so that
    weight sums stay far inside 64 bits)."""
    c = np.asarray(cost_per_elem, dtype=np.float64)
    ref = c[0] if c[0] > 0 else c[c > 0].min()
    return np.minimum(np.maximum(1, np.rint(scale * c / ref)), 2 ** 24).astype(np.uint32)


def partition(weight, n_queues):
    """Contiguous weighted split: S_i = exclusive prefix sum of w, W = sum w,
    queue(i) = min(Q - 1, floor(Q (2 S_i + w_i) / (2W))) (element midpoints; the cap only
    moves trailing zero-weight elements, whose midpoint is W, into the last queue), and
    queue_begin[q] = first i with queue(i) >= q, queue_begin[Q] = n.  Exact integer
    arithmetic at any size."""
    w = np.asarray(weight, dtype=np.uint64)
    n = w.size
    S = np.concatenate([[0], np.cumsum(w, dtype=np.uint64)[:-1]]).astype(np.uint64)
    W = int(w.sum(dtype=np.uint64))
    Q = int(n_queues)
    qb = np.empty(Q + 1, dtype=np.int64)
    if W == 0:
        qb[:] = 0
        qb[Q] = n
        return qb
    if Q * 2 * W < (1 << 63):
        qi = (np.uint64(Q) * (np.uint64(2) * S + w)) // np.uint64(2 * W)
    else:   # Python integers: no 64-bit overflow
        qi = np.array([(Q * (2 * int(a) + int(b))) // (2 * W) for a, b in zip(S, w)], dtype=np.uint64)
    qi = np.minimum(qi, np.uint64(Q - 1))
    for q in range(Q + 1):
        qb[q] = int(np.searchsorted(qi, np.uint64(q), side="left"))
    return qb


def imbalance(load_per_queue):
    l = np.asarray(load_per_queue, dtype=np.float64)
    return float(l.max() / l.mean() - 1.0)
