"""Pins of the oracle's grid (paper Section 2.1, eq. (2.2), Fig. 2)."""

import numpy as np
import pytest

from oracle import mesh


@pytest.fixture(scope="module")
def levels():
    return mesh.hierarchy(3)


def _volumes(lv):
    V = lv.coords[lv.tets]
    e = V[:, 1:] - V[:, :1]
    return np.abs(np.linalg.det(e)) / 6.0


def test_counts_and_unique_ids(levels):
    for lv in levels:
        n = lv.n
        assert lv.tets.shape[0] == 6 * n ** 3 == 48 * 8 ** lv.level
        assert lv.coords.shape[0] == (n + 1) ** 3
        assert np.array_equal(np.sort(lv.elem_id), np.arange(6 * n ** 3))
        assert np.array_equal(np.sort(lv.node_id), np.arange((n + 1) ** 3))


def test_volumes_children_eighth_and_partition(levels):
    for lv in levels:
        vol = _volumes(lv)
        assert abs(vol.sum() - 1.0) < 1e-13
        assert np.allclose(vol, 1.0 / (6 * lv.n ** 3), rtol=1e-12, atol=0)
        if lv.level > 0:
            pv = _volumes(levels[lv.level - 1])
            assert np.allclose(vol, pv[lv.parent] / 8.0, rtol=1e-12)


def test_children_inside_parent(levels):
    for l in range(1, len(levels)):
        lv, pv = levels[l], levels[l - 1]
        cen = lv.coords[lv.tets].mean(axis=1)
        P = pv.coords[pv.tets][lv.parent]                    # parent vertices per child
        M = np.ones((cen.shape[0], 4, 4))
        M[:, 1:, :] = P.transpose(0, 2, 1)
        lam = np.linalg.solve(M, np.concatenate([np.ones((cen.shape[0], 1)), cen], 1)[..., None])[..., 0]
        assert lam.min() > 1e-9


def test_conformity_faces_shared_by_two(levels):
    lv = levels[2]
    faces = np.sort(np.concatenate([lv.tets[:, [1, 2, 3]], lv.tets[:, [0, 2, 3]],
                                    lv.tets[:, [0, 1, 3]], lv.tets[:, [0, 1, 2]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(counts.tolist()) <= {1, 2}
    # boundary faces: 6 sides x n^2 squares x 2 triangles
    assert (counts == 1).sum() == 6 * lv.n ** 2 * 2


def test_kuhn_child_rule_matches_geometry(levels):
    """Arithmetic child rule of a Kuhn simplex (cube C, step order p): the 8 children sit in
    sub-cubes 2C + offset with step orders
      (0, p), (e_p1, p), (e_p1, (p2,p3,p1)), (e_p1, (p2,p1,p3)),
      (e_p1+e_p2, p), (e_p1+e_p2, (p3,p1,p2)), (e_p1+e_p2, (p1,p3,p2)), ((1,1,1), p).
    Checked against the geometric parent map of Bey refinement."""
    perms = mesh.PERMS
    pidx = {p: s for s, p in enumerate(perms)}
    for l in range(1, len(levels)):
        lv, pv = levels[l], levels[l - 1]
        nf, nc = lv.n, pv.n
        expect = {}
        for e in range(6 * nc ** 3):
            s, c = e % 6, e // 6
            C = np.array([c % nc, (c // nc) % nc, c // (nc * nc)])
            p = perms[s]
            E = np.eye(3, dtype=int)
            kids = [(0 * E[0], p), (E[p[0]], p), (E[p[0]], (p[1], p[2], p[0])),
                    (E[p[0]], (p[1], p[0], p[2])), (E[p[0]] + E[p[1]], p),
                    (E[p[0]] + E[p[1]], (p[2], p[0], p[1])),
                    (E[p[0]] + E[p[1]], (p[0], p[2], p[1])), (np.ones(3, int), p)]
            ids = []
            for off, q in kids:
                cc = 2 * C + off
                ids.append(pidx[tuple(q)] + 6 * (cc[0] + nf * (cc[1] + nf * cc[2])))
            expect[e] = sorted(ids)
        got = {}
        for k in range(lv.tets.shape[0]):
            got.setdefault(int(pv.elem_id[lv.parent[k]]), []).append(int(lv.elem_id[k]))
        for e, ids in got.items():
            assert sorted(ids) == expect[e]


def test_free_nodes(levels):
    for lv in levels:
        assert mesh.free_node_mask(lv).sum() == (lv.n - 1) ** 3
