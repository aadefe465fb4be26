"""Coefficients and forcing of a workload evaluated on a torch device, for sizes whose
host evaluation would take minutes (805 million elements at 513^3 nodes).  The same
seeded field and the same element centroids as the host evaluation (fields.py,
lattice.py), computed with torch operations; input generation only."""

from __future__ import annotations


def device_inputs(w, dev, chunk: int = 1 << 25):
    """(per-element nu of every level 0..L, forcing (ncomp, 6 n_L^3) flattened) on dev."""
    import torch
    from .lattice import element_centroids_torch
    field = w.make_field()
    nus = []
    for l in range(w.L + 1):
        E = 6 * (2 ** (l + 1)) ** 3
        out = torch.empty(E, dtype=torch.float64, device=dev)
        for s0 in range(0, E, chunk):
            s1 = min(E, s0 + chunk)
            out[s0:s1] = field.nu_torch(element_centroids_torch(l, s0, s1, dev))
        nus.append(out)
    E = nus[-1].numel()
    f = torch.zeros((w.ncomp, E), dtype=torch.float64, device=dev)
    for s0 in range(0, E, chunk):
        s1 = min(E, s0 + chunk)
        f[-1, s0:s1] = -field.xi_torch(element_centroids_torch(w.L, s0, s1, dev))
    return nus, f.reshape(-1)
