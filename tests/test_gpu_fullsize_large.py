"""Full-size checks at the two largest workloads, through the C ABI, each sample
recomputed by the element-by-element oracle (oracle/sample.py):

* 513^3 nodes (9 levels, 4.0e8 DoFs, 64 sinkers of radii 0.02-0.06, contrast 1e6) with
  the mixed-precision hierarchy (FP32 V-cycle, BF16 finest coefficient): the FP64 fine
  apply and the FP32/BF16 fine apply at sampled nodes, flags at sampled points of the
  coarse levels, the FP64 Galerkin blocks behind them, and the energy-norm contraction
  of one V-cycle;
* Stokes with velocity 257^3 / pressure 129^3 nodes and 16 sinkers: the divergence B,
  its transpose and the 1/nu lumped pressure mass at sampled interior nodes, and the
  velocity block's fine apply at sampled nodes.

The inputs are generated on the device (workloads.device, the same seeded fields as
the host evaluation) and only the entries a sample needs are read back.
"""

import numpy as np
import pytest
import torch

from oracle import sample
from workloads import workload
from workloads.device import device_inputs

pytestmark = pytest.mark.gpu


class _Gather:
    """Host view of a device vector indexed like a numpy array: only the requested
    entries are copied back (optionally transformed on the host)."""

    def __init__(self, t, fn=None):
        self.t, self.fn = t, fn

    def __getitem__(self, idx):
        a = np.asarray(idx, dtype=np.int64)
        v = self.t[torch.from_numpy(a.reshape(-1)).to(self.t.device)].double().cpu().numpy()
        if self.fn is not None:
            v = self.fn(v)
        return v.reshape(a.shape) if a.ndim else float(v[0])


def _bf16(x):
    # one rounding of the float64 value to 8 significant bits, ties to even
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0), e - 8)


def _pid(node, n):
    return node[0] + (n + 1) * (node[1] + (n + 1) * node[2])


def _nodes(field, n, rng, k_random=3, k_sinkers=3):
    """Interior lattice nodes (n cells per axis): random ones plus nodes on the surfaces
    of the first sinkers, where the coefficient jumps."""
    pts = [tuple(int(v) for v in rng.integers(1, n, 3)) for _ in range(k_random)]
    for c, r in zip(field.centres[:k_sinkers], field.radii[:k_sinkers]):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        q = np.clip(np.rint((c + r * d) * n).astype(int), 1, n - 1)
        pts.append(tuple(int(v) for v in q))
    return pts


# ---------------------------------------------------------------------------
# 513^3 vector sinkers, mixed-precision hierarchy
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def big():
    from paper_2511_13109_amd import Hierarchy
    w = workload("sinker513")
    print(f"\n[case sinker513 L={w.L} vector, mixed precision, full size]", flush=True)
    nus, f = device_inputs(w, "cuda")
    del f
    G = Hierarchy(w.L, 3, nus[w.L], nus[:w.L], mg_dtype="f32", mg_nu_dtype="bf16",
                  smoother="chebyshev")
    yield w, w.make_field(), nus, G
    G.close()


def test_fine_apply_sampled_513(big):
    w, field, nus, G = big
    L, n = w.L, w.n
    nn = (n + 1) ** 3
    gen = torch.Generator(device="cuda").manual_seed(0)
    u = torch.randn(3 * nn, generator=gen, device="cuda", dtype=torch.float64)
    v = G.apply(L, u)
    u32 = u.float()
    v32 = G.apply(L, u32)
    rng = np.random.default_rng(0)
    for node in _nodes(field, n, rng):
        x = np.array(node) / n
        idx = torch.tensor([c * nn + _pid(node, n) for c in range(3)], device="cuda")
        ref = sample.apply_at_node(L, x, _Gather(nus[L]), 3, _Gather(u))
        got = v[idx].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), node
        # the FP32 apply with the BF16 coefficient: the oracle in FP64 on the same rounded
        # inputs; FP32 arithmetic over the 24 elements of the star stays far below 1e-4,
        # while a coefficient off by one BF16 place would move the row by about 4e-3
        ref32 = sample.apply_at_node(L, x, _Gather(nus[L], _bf16), 3, _Gather(u32))
        got32 = v32[idx].double().cpu().numpy()
        assert np.abs(got32 - ref32).max() <= 1e-4 * np.abs(ref32).max(), node
    print(f"[sinker513] fine apply sampled at {len(_nodes(field, n, np.random.default_rng(0)))} nodes",
          flush=True)


def test_flags_and_blocks_sampled_513(big):
    w, field, nus, G = big
    L = w.L
    nuh = _Gather(nus[L])
    rng = np.random.default_rng(7)
    pts = []
    for c, r in zip(field.centres[:6], field.radii[:6]):   # on and inside sinker surfaces
        d = rng.standard_normal(3)
        pts.append(c + r * d / np.linalg.norm(d))
        pts.append(c + 0.3 * r * d / np.linalg.norm(d))
    pts += list(rng.random((2, 3)))
    nflag = 0
    for level in range(3, L):
        ids = G.flags(level)
        # the blocks of a level are copied whole: levels up to 5 (a few tens of MB here)
        blocks = G.blocks(level) if (ids.size and level <= 5) else None
        k = {3: 2, 4: 4}.get(level, len(pts))      # a level-l element has 8^(L-l) descendants
        for p in pts[:k]:
            eid, fl = sample.flag_at_point(level, L, p, nuh)
            j = np.searchsorted(ids, eid)
            got = bool(j < ids.size and ids[j] == eid)
            assert got == fl, (level, eid)
            nflag += fl
            if fl and blocks is not None:
                _, B = sample.block_at_point(level, L, p, nuh, 3)
                assert np.abs(blocks[j] - B).max() <= 1e-12 * np.abs(B).max(), (level, eid)
    assert nflag > 0        # the surface points must meet flagged elements


def test_vcycle_contracts_513(big):
    # one FP32 V-cycle as an error propagator I - B A reduces a random error in the
    # energy norm of the FP64 operator
    w, field, nus, G = big
    L, n = w.L, w.n
    nn = (n + 1) ** 3
    gen = torch.Generator(device="cuda").manual_seed(1)
    e = torch.randn(3 * nn, generator=gen, device="cuda", dtype=torch.float64)
    Ae = G.apply(L, e)
    e1 = e - G.vcycle(Ae.float()).double()

    def anorm(x):
        return float(torch.dot(x, G.apply(L, x))) ** 0.5
    ratio = anorm(e1) / anorm(e)
    print(f"[sinker513] V-cycle energy-norm contraction of a random error {ratio:.4f}", flush=True)
    assert ratio < 1.0


# ---------------------------------------------------------------------------
# Stokes, velocity 257^3 / pressure 129^3
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def stokes257():
    from paper_2511_13109_amd import Hierarchy, Stokes
    w = workload("stokes257")
    print(f"\n[case stokes257 L={w.L}, full size]", flush=True)
    nus, f = device_inputs(w, "cuda")
    del f
    G = Hierarchy(w.L, 3, nus[w.L], nus[:w.L])
    yield w, w.make_field(), nus, Stokes(G)
    G.close()


def test_stokes_rows_sampled_257(stokes257):
    w, field, nus, S = stokes257
    L, n = w.L, w.n
    npc = n // 2                                   # pressure cells per axis
    nn = (n + 1) ** 3
    gen = torch.Generator(device="cuda").manual_seed(2)
    u = torch.randn(3 * nn, generator=gen, device="cuda", dtype=torch.float64)
    q = S.div(u)            # boundary velocity slots hold random values: they must be ignored
    p = torch.randn((npc + 1) ** 3, generator=gen, device="cuda", dtype=torch.float64)
    g = S.grad(p)
    m = S.mass()
    rng = np.random.default_rng(3)
    pres = _nodes(field, npc, rng)
    qs = [(float(q[_pid(k, npc)]), sample.div_at_pressure_node(L, np.array(k) / npc, _Gather(u)))
          for k in pres]
    scale = max(abs(r) for _, r in qs)
    for (got, ref), k in zip(qs, pres):
        assert abs(got - ref) <= 1e-12 * scale, k
        ref_m = sample.mass_at_pressure_node(L, np.array(k) / npc, _Gather(nus[L]))
        assert abs(float(m[_pid(k, npc)]) - ref_m) <= 1e-12 * ref_m, k
    for j in _nodes(field, n, rng):
        idx = torch.tensor([c * nn + _pid(j, n) for c in range(3)], device="cuda")
        ref = sample.grad_at_velocity_node(L, np.array(j) / n, _Gather(p))
        got = g[idx].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), j
    print(f"[stokes257] B, mass at {len(pres)} pressure nodes; B^T at velocity nodes", flush=True)


def test_fine_apply_sampled_257(stokes257):
    # the velocity block's element loop at 257^3 nodes, including the last, partly
    # filled tiles in x (9 node columns after eight full 31-wide tiles)
    w, field, nus, S = stokes257
    L, n = w.L, w.n
    nn = (n + 1) ** 3
    gen = torch.Generator(device="cuda").manual_seed(4)
    u = torch.randn(3 * nn, generator=gen, device="cuda", dtype=torch.float64)
    v = S.H.apply(L, u)
    rng = np.random.default_rng(5)
    nodes = _nodes(field, n, rng, k_random=2, k_sinkers=2)
    nodes += [(n - 1, int(rng.integers(1, n)), int(rng.integers(1, n))), (248, 17, 200),
              (252, n - 1, 1), (247, 1, n - 1)]
    for node in nodes:
        idx = torch.tensor([c * nn + _pid(node, n) for c in range(3)], device="cuda")
        ref = sample.apply_at_node(L, np.array(node) / n, _Gather(nus[L]), 3, _Gather(u))
        got = v[idx].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), node
