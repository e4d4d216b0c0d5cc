"""Work of the residual kernels, per element, for roofline accounting.

Two counts.  `algorithmic_*`: the method's work per element and stage, independent of the
kernels (the reference for roofline fractions).  `*_work` / `phase_work`: the work of the
kernels' own formulation (kernels.hip), reported alongside as the formulation fraction:
FP64 flops with a fused multiply-add
counted as 2, divisions and square roots as 1; bytes are the compulsory HBM reads and writes
of each kernel's per-element inputs and outputs (state blocks, face traces, partial residual,
RK registers).  Operator tables shared by all elements of a type (V, P^, face operators) are
not counted: they stay cache-resident.  S = face sides of the element (a mortar half counts as
one), Sd = sides that interpolate (not collocated with volume nodes).

MI355X peaks used for fractions: HBM3E 8.0 TB/s; FP64 vector 78.6 TFLOP/s
(256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU).
"""
from __future__ import annotations

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def n_modes(t, N):
    n = N + 1
    return [n ** 3, n * n * (n + 1) // 2, n * (n + 1) * (2 * n + 1) // 6, n * (n + 1) * (n + 2) // 6][t]


def trace_work(t, N, S, Sd, ns=False):
    n = N + 1
    n2, m = n * n, n_modes(t, N)
    if t == 0:
        flops = Sd * n2 * n2 * 5 * 2
    else:
        flops = S * n2 * m * 5 * 2
    byts = 8 * (5 * m + S * 5 * n2)
    return flops, byts


def volume_work(t, N, S, Sd, ns):
    n = N + 1
    n2, nn, m = n * n, n ** 3, n_modes(t, N)
    modal = t != 0
    fl = nn * (30 + 75 + (75 if modal else 0))        # Euler flux, reference flux, contravariant
    fl += nn * 3 * n * 5 * 2                           # weak derivative
    if modal:
        fl += 2 * nn * m * 5 * 2                       # V u~ and P^ d
    else:
        fl += 5 * nn
    byts = 8 * (2 * 5 * m)                             # read U_e, write partial residual
    if ns:
        fl += nn * 12                                  # lifting variables
        fl += nn * 3 * n * 4 * (7 if modal else 2)     # weak gradient, reference directions
        fl += nn * 60                                  # reference -> physical gradient
        fl += S * n2 * 40                              # face averages of lifting variables
        if modal:
            fl += 2 * m * nn * 12 * 2                  # P^ and V on the 12 gradient fields
            fl += S * m * n2 * 12 * 2                  # modal lift of the face terms
            fl += S * n2 * (m * 12 * 2 + 85)           # gradient traces and viscous normal flux
        else:
            fl += (S - Sd) * n2 * 12 + Sd * n2 * n2 * 12 * 2 + nn * 36
            fl += (S - Sd) * n2 * 85 + Sd * n2 * (n2 * 12 * 2 + 85)
        fl += nn * (70 + 15)                           # viscous flux at the nodes
        byts += 8 * (2 * S * 5 * n2 + S * 5 * n2)      # read both sides' traces, write Fv.n
    return fl, byts


# directions on Gauss-Lobatto lines (the split form applies there), per type
SBP_DIRS = (3, 2, 2, 1)


def volume_split_work(t, N, S, Sd, ns):
    """Volume phase in the split form: the weak kernel's work without the weak derivative of
    the inviscid flux along the Gauss-Lobatto directions (Euler; hexahedra then need no
    pointwise flux at all), plus per node the two-point quantities (and on modal elements
    the contravariant vectors of those directions); per unordered node pair on each such line
    one two-point flux (it is symmetric): 73 flops (two logarithmic means in their series form
    with one division each, averages, the five flux components), 6 more for the metric average
    on modal elements; per ordered pair the weighted accumulation, 10 flops."""
    fl, byts = volume_work(t, N, S, Sd, ns)
    n = N + 1
    nn = n ** 3
    nsd = SBP_DIRS[t]
    if not ns:
        fl -= nn * nsd * n * 5 * 2
        if t == 0:
            fl -= nn * (30 + 75)
    fl += nn * (15 + (27 * nsd if t else 0))
    fl += nn * nsd * (n - 1) // 2 * (73 + (6 if t else 0))
    fl += nn * nsd * (n - 1) * 10
    return fl, byts


def surface_work(t, N, S, Sd, ns):
    n = N + 1
    n2, m = n * n, n_modes(t, N)
    fl = S * n2 * (165 if ns else 150)                 # LF flux (+ viscous average) and weights
    if t == 0:
        fl += (S - Sd) * n2 * 5 + Sd * n2 * n2 * 5 * 2
    else:
        fl += S * m * n2 * 5 * 2
    fl += 5 * m * 8                                     # residual assembly and RK update
    byts = 8 * (2 * S * 5 * n2 * (2 if ns else 1) + 5 * 5 * m)
    return fl, byts


# ------------------------------------------------------------------------------------------
# The algorithmic work model of the hot path (the reference count the roofline fractions use):
# per element and RK stage, independent of how the kernels are written.  Flops: the dense
# transforms q = V u~ and the projection (2 n^3 m nV each, modal types), the point flux
# (120 n^3), the sum-factorised volume integral (6 n^4 nV), the Lax-Friedrichs flux (100 per
# face point, shared by the two sides: 50 per side point), face interpolation and lift on modal
# sides (4 n^2 nV per point, half each), the RK update (4 nV m) and, for hexahedra, the nodal
# mass division and assembly (18 n^3); Navier-Stokes adds 15 n^3 + 72 n^4 + 72 n^3 + 60 n^3
# (lifting variables, gradients, viscous flux) and per side point 70 (viscous normal flux) plus,
# on modal sides, 63 n^2 (interpolation and lift of the lifting variables and gradients).
# Bytes: the state U and the RK register K read and written once, 4 x 8 x nV x stored dofs;
# face traces and gradients are recomputable, not algorithmic.  With the nominal face counts
# (6, 5, 5, 4) this reproduces, per element, 23k/97k/84k/65k flops (Euler, N = 3),
# 46k/292k/241k/177k (Euler, N = 4), 120k/560k/510k/405k (NS, N = 4) and
# 224k/1296k/1144k/880k (NS, N = 5) for hex/prism/pyramid/tet.
# Each term is charged to the phase that computes it: trace = face interpolation; volume =
# transforms, point and viscous fluxes, volume integral, gradients and gradient traces, and the
# read of U; surface = Riemann flux, lift, RK update and the remaining three state accesses.

NOMINAL_SIDES = (6, 5, 5, 4)


def algorithmic_work(t, N, S, ns):
    """Per-element algorithmic (flops, bytes) of one RK stage by phase: two arrays [3] (trace,
    volume, surface); S face sides (mortar halves count as sides)."""
    n = N + 1
    n2, n3, n4, nV, m = n * n, n ** 3, n ** 4, 5, n_modes(t, N)
    modal = t != 0
    fl = [0.0, 0.0, 0.0]
    fl[0] = 2 * n2 * nV * S * n2 if modal else 0
    fl[1] = (4 * n3 * m * nV if modal else 0) + 120 * n3 + 6 * n4 * nV
    fl[2] = 50 * S * n2 + (2 * n2 * nV * S * n2 if modal else 18 * n3) + 4 * nV * m
    if ns:
        fl[1] += 15 * n3 + 72 * n4 + 72 * n3 + 60 * n3 + S * n2 * (70 + (63 * n2 if modal else 0))
    by = [0.0, 8.0 * nV * m, 3 * 8.0 * nV * m]
    return fl, by


def algorithmic_split_extra(t, N, ns):
    """Algorithmic flops per element that the split-form volume integral adds to the weak form's
    volume phase: on each Gauss-Lobatto line one two-point flux per unordered node pair (73
    flops, 6 more for the averaged metric on modal elements) and the weighted accumulation per
    ordered pair (10); Euler drops the weak derivative of the inviscid flux along those
    directions (2 n^4 nV each).  Navier-Stokes keeps it for the viscous flux."""
    n = N + 1
    n3, n4, nsd = n ** 3, n ** 4, SBP_DIRS[t]
    fl = n3 * nsd * (n - 1) // 2 * (73 + (6 if t else 0)) + n3 * nsd * (n - 1) * 10
    if not ns:
        fl -= 2 * n4 * 5 * nsd
    return fl


def algorithmic_phase_work(phase, elem_type, elem_sides, N, ns):
    """Algorithmic (flops, bytes) of `phase` over all elements of each type: arrays [4]."""
    import numpy as np
    fl = np.zeros(4)
    by = np.zeros(4)
    for t in range(4):
        sel = elem_type == t
        if not sel.any():
            continue
        S, cnt = np.unique(elem_sides[sel, 0], return_counts=True)
        for s, c in zip(S, cnt):
            a, b = algorithmic_work(t, N, int(s), ns)
            fl[t] += c * a[phase]
            by[t] += c * b[phase]
    return fl, by


def algorithmic_stage(elem_type, elem_sides, N, ns):
    """(flops, bytes, t*) of one RK stage over the whole mesh: t* = max(flops at the FP64 peak,
    bytes at the HBM peak), the types overlapping in time."""
    F = B = 0.0
    for ph in range(3):
        f, b = algorithmic_phase_work(ph, elem_type, elem_sides, N, ns)
        F += float(f.sum())
        B += float(b.sum())
    return F, B, max(F / (PEAK_FP64_TFLOPS * 1e12), B / (PEAK_HBM_GBS * 1e9))


PHASES = ("trace", "volume", "surface")
_WORK = (trace_work, volume_work, surface_work)


def phase_work(phase, elem_type, elem_sides, N, ns, split=False):
    """(flops, bytes) per launch of `phase` over all elements of each type: arrays [4]."""
    import numpy as np
    fl = np.zeros(4)
    by = np.zeros(4)
    f = volume_split_work if (split and phase == 1) else _WORK[phase]
    for t in range(4):
        sel = elem_type == t
        if not sel.any():
            continue
        S = elem_sides[sel, 0]
        Sd = elem_sides[sel, 1]
        # the counts are affine in (S, Sd): evaluate per distinct pair
        pairs, cnt = np.unique(np.stack([S, Sd], axis=1), axis=0, return_counts=True)
        for (s, sd), c in zip(pairs, cnt):
            a, b = f(t, N, int(s), int(sd), ns)
            fl[t] += c * a
            by[t] += c * b
    return fl, by
