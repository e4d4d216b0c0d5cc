"""Initial states built on the device through the library (for GPU-only tests and the
benchmark): the Taylor-Green field at the library's volume nodes plus the seeded node noise
(the same stream as node_noise, scattered to the library's element order), projected with
the library's own projection."""
from __future__ import annotations

import numpy as np

from .meshgen import node_noise, tgv_primitive


def tgv_state(dg, gamma=1.4, mach=0.1, noise_seed=1, chunk=65536):
    import torch
    x = dg.node_coords()
    rho, u, v, w, p = tgv_primitive(x[..., 0], x[..., 1], x[..., 2], gamma=gamma, mach=mach, xp=torch)
    q = torch.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], dim=1)
    del x, rho, u, v, w, p
    nn = dg.n ** 3
    inv = np.empty_like(dg.perm)
    inv[dg.perm] = np.arange(dg.n_elems, dtype=dg.perm.dtype)
    for s in range(0, dg.n_elems, chunk):
        idx = np.arange(s, min(dg.n_elems, s + chunk))
        nz = torch.from_numpy(node_noise(noise_seed, nn, idx)).to(q.device)
        q[torch.from_numpy(inv[idx].astype(np.int64)).to(q.device)] += nz
    U = dg.project(q)
    del q
    return U
