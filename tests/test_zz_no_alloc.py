"""agca_macro_gradient_noalloc (no device allocation; a fixed device scratch array)
against agca_macro_gradient (which allocates its scratch per call), through the C ABI:
two calls in a row, the second on a smaller lattice, bit-identical to the allocating
entry point and within 1e-12 of the oracle's gradient test of eq. (2.8)."""

import numpy as np
import pytest
import torch

from oracle import agca, mesh
from workloads import Sinkers

pytestmark = pytest.mark.gpu


def _node_xyz(L):
    n = 2 ** (L + 1)
    p = np.arange((n + 1) ** 3)
    return np.stack([p % (n + 1), (p // (n + 1)) % (n + 1), p // (n + 1) ** 2], axis=1) / n


def test_noalloc_matches_allocating_entry_point():
    from paper_2511_13109_amd import AGCAError, macro_gradient
    field = Sinkers(4, 2, radius=0.15, width=0.05, contrast=1e6)
    for L in (4, 2):             # the second call on a smaller input
        print(f"\n[macro gradient, no allocation, L={L}]", flush=True)
        eta = torch.from_numpy(field.nu(_node_xyz(L))).cuda()
        g_noalloc = macro_gradient(L, eta, noalloc=True)
        g_alloc = macro_gradient(L, eta)
        assert np.array_equal(g_noalloc, g_alloc)
        g_ref = agca.macro_gradient_max(mesh.hierarchy(L), eta.cpu().numpy())
        assert np.abs(g_noalloc - g_ref).max() <= 1e-12 * g_ref.max()
        # a repeated call starts from cleared slots (the previous call's maxima are gone)
        assert np.array_equal(macro_gradient(L, eta, noalloc=True), g_alloc)
    # a flat field after a steep one: every maximum is 0, so nothing survives in the slots
    flat = torch.ones((2 ** 3 + 1) ** 3, dtype=torch.float64, device="cuda")
    assert np.array_equal(macro_gradient(2, flat, noalloc=True), np.zeros(48))
    # L beyond 9 is rejected before anything runs
    import ctypes as C
    from paper_2511_13109_amd import _lib
    out = np.zeros(48)
    with pytest.raises(AGCAError, match="AGCA_E_INVALID"):
        _lib.check(_lib.load().agca_macro_gradient_noalloc(10, C.c_void_p(flat.data_ptr()),
                                                           out.ctypes.data_as(C.c_void_p), None),
                   "agca_macro_gradient_noalloc")
