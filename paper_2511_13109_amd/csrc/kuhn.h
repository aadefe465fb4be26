// Kuhn-simplex arithmetic of the uniformly refined cube lattice.
//
// A level with n cells per axis has the lattice nodes (x,y,z), 0 <= x,y,z <= n,
// and 6 n^3 tetrahedra: in every cell C, one simplex per axis order
// s = 0..5 (0 xyz, 1 xzy, 2 yxz, 3 yzx, 4 zxy, 5 zyx) with path vertices
//   v0 = C, v1 = v0 + e_a1, v2 = v1 + e_a2, v3 = v2 + e_a3 = C + (1,1,1).
// Cell corner k = dx + 2 dy + 4 dz; the path corners are 0, 1<<a1,
// (1<<a1)|(1<<a2), 7.
//
// With barycentric gradients scaled by the mesh width h:
//   g0 = -e_a1, g1 = e_a1 - e_a2, g2 = e_a2 - e_a3, g3 = e_a3,
// and volume h^3/6, the unit-coefficient element matrix of the scalar operator
// (paper eq. (2.3)) is (h/6) times the path Laplacian, and that of the
// symmetric-gradient operator (eq. (3.5)) is
//   (h/6) [ delta_cd g_a.g_b + g_a[d] g_b[c] ].
//
// Uniform (Bey) refinement of simplex (C, s) with path vertices x0..x3 gives 8
// children, again Kuhn simplices, in the cells 2C + offset:
//   k=0  [x0,  x01, x02, x03]  offset 0            order (a1,a2,a3)
//   k=1  [x01, x1,  x12, x13]  offset e_a1         order (a1,a2,a3)
//   k=2  [x02, x12, x2,  x23]  offset e_a1+e_a2    order (a1,a2,a3)
//   k=3  [x03, x13, x23, x3 ]  offset (1,1,1)      order (a1,a2,a3)
//   k=4  [x01, x02, x03, x13]  offset e_a1         order (a2,a3,a1)
//   k=5  [x01, x02, x12, x13]  offset e_a1         order (a2,a1,a3)
//   k=6  [x02, x03, x13, x23]  offset e_a1+e_a2    order (a3,a1,a2)
//   k=7  [x02, x12, x13, x23]  offset e_a1+e_a2    order (a1,a3,a2)
// (children listed in their own path order).  The local interpolation of eq.
// (2.4) from the parent to child k therefore is a constant 4x4 matrix whose
// row a holds the parent hat values at the child's a-th vertex (1 at a parent
// vertex, 1/2 and 1/2 at an edge midpoint), kP2 below in units of 1/2.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define AGCA_HDC __host__ __device__
#else
#define AGCA_HDC
#endif

namespace agca {

AGCA_HDC constexpr int axis1(int s) { return s >> 1; }
AGCA_HDC constexpr int axis2(int s) {
    return (s & 1) ? ((s >> 1) == 2 ? 1 : 2) : ((s >> 1) == 0 ? 1 : 0);
}
AGCA_HDC constexpr int axis3(int s) { return 3 - axis1(s) - axis2(s); }
AGCA_HDC constexpr int axis(int s, int j) {
    return j == 0 ? axis1(s) : (j == 1 ? axis2(s) : axis3(s));
}
// index s of the axis order (a, b, c)
AGCA_HDC constexpr int order_index(int a, int b, int c) { return 2 * a + (b > c ? 1 : 0); }

// path corner j (0..3) of simplex s inside its cell
AGCA_HDC constexpr int path_corner(int s, int j) {
    return j == 0 ? 0
         : j == 1 ? (1 << axis1(s))
         : j == 2 ? ((1 << axis1(s)) | (1 << axis2(s)))
                  : 7;
}

// gradient component c of vertex a (scaled by h), in {-1, 0, 1}
AGCA_HDC constexpr int grad(int s, int a, int c) {
    return a == 0 ? -(c == axis1(s))
         : a == 1 ? (c == axis1(s)) - (c == axis2(s))
         : a == 2 ? (c == axis2(s)) - (c == axis3(s))
                  : (c == axis3(s));
}

// (g_a . g_b) for a Kuhn simplex: the path Laplacian
AGCA_HDC constexpr int path_lap(int a, int b) {
    return a == b ? ((a == 0 || a == 3) ? 1 : 2) : ((a - b == 1 || b - a == 1) ? -1 : 0);
}

// unit element matrix entry of the vector operator (component c vertex a, component d
// vertex b), without h/6
AGCA_HDC constexpr int unit_entry(int s, int c, int a, int d, int b) {
    return (c == d ? path_lap(a, b) : 0) + grad(s, a, d) * grad(s, b, c);
}

// unit element matrix entry for ncomp = 1 (scalar: path Laplacian) or 3 (vector)
AGCA_HDC constexpr int elem_entry(int ncomp, int s, int c, int a, int d, int b) {
    return ncomp == 1 ? path_lap(a, b) : unit_entry(s, c, a, d, b);
}

// children: cell offset bits (x=1, y=2, z=4) and axis order of child k of s
AGCA_HDC constexpr int child_offset(int s, int k) {
    return (k == 0) ? 0
         : (k == 1 || k == 4 || k == 5) ? (1 << axis1(s))
         : (k == 3) ? 7
                    : ((1 << axis1(s)) | (1 << axis2(s)));
}
AGCA_HDC constexpr int child_order(int s, int k) {
    return (k <= 3) ? s
         : (k == 4) ? order_index(axis2(s), axis3(s), axis1(s))
         : (k == 5) ? order_index(axis2(s), axis1(s), axis3(s))
         : (k == 6) ? order_index(axis3(s), axis1(s), axis2(s))
                    : order_index(axis1(s), axis3(s), axis2(s));
}

// local interpolation parent -> child k, in units of 1/2: kP2[k][child vertex][parent vertex]
AGCA_HDC constexpr int kP2(int k, int a, int i) {
    // parent vertices hit by child k's vertex a: encoded as two indices (equal = vertex)
    constexpr int tab[8][4][2] = {
        {{0, 0}, {0, 1}, {0, 2}, {0, 3}},
        {{0, 1}, {1, 1}, {1, 2}, {1, 3}},
        {{0, 2}, {1, 2}, {2, 2}, {2, 3}},
        {{0, 3}, {1, 3}, {2, 3}, {3, 3}},
        {{0, 1}, {0, 2}, {0, 3}, {1, 3}},
        {{0, 1}, {0, 2}, {1, 2}, {1, 3}},
        {{0, 2}, {0, 3}, {1, 3}, {2, 3}},
        {{0, 2}, {1, 2}, {1, 3}, {2, 3}},
    };
    return (tab[k][a][0] == i) + (tab[k][a][1] == i);
}

// The 15 nodes coupled to a node by the simplices around it: the node itself and
// the offsets +m and -m for the 7 non-zero cell-corner masks m (x=1, y=2, z=4).
// Neighbour index 0 is the node, m is +m, 7 + m is -m.
AGCA_HDC constexpr int nbr_mask(int k) { return k == 0 ? 0 : (k <= 7 ? k : k - 7); }
AGCA_HDC constexpr int nbr_sign(int k) { return k > 7 ? -1 : 1; }
// neighbour index of path vertex b seen from path vertex a of one simplex: the path
// corners are nested bit sets, so their difference is +-(one corner mask)
AGCA_HDC constexpr int nbr_of(int s, int a, int b) {
    return a == b ? 0
         : b > a ? (path_corner(s, b) ^ path_corner(s, a))
                 : 7 + (path_corner(s, a) ^ path_corner(s, b));
}

// canonical ids
AGCA_HDC inline int64_t node_id(int64_t n, int64_t x, int64_t y, int64_t z) {
    return x + (n + 1) * (y + (n + 1) * z);
}
AGCA_HDC inline int64_t elem_id(int64_t n, int64_t cx, int64_t cy, int64_t cz, int s) {
    return s + 6 * (cx + n * (cy + n * cz));
}
// Internal storage of per-element data.  Element-id order (slot 6 cell + s) keeps the
// six coefficients of a cell in one contiguous 48-byte run, which streams better along
// the element loop's z march than six separate planes (slot s cells + cell); the
// plane layout stays available at compile time for measurements.
#ifndef AGCA_ELEM_SOA
#define AGCA_ELEM_SOA 0
#endif
AGCA_HDC inline int64_t elem_slot(int s, int64_t cell, int64_t cells) {
    return AGCA_ELEM_SOA ? s * cells + cell : 6 * cell + s;
}
AGCA_HDC inline int64_t elem_index(int64_t e, int64_t cells) {
    return elem_slot((int)(e % 6), e / 6, cells);
}

// lattice coordinates of node p = x + (n+1)(y + (n+1) z) on a level with n cells per
// axis, in 32-bit arithmetic (a level holds at most 1025^3 < 2^32 nodes; 64-bit
// division would cost several times the instructions of the kernels that use this)
AGCA_HDC inline void node_coords(int64_t p, int n, int& x, int& y, int& z) {
    const uint32_t q = (uint32_t)p, n1 = (uint32_t)(n + 1);
    const uint32_t r = q / n1;
    x = (int)(q - r * n1);
    y = (int)(r % n1);
    z = (int)(r / n1);
}

// id of child k of element e on a level with n cells (children on the level with 2n cells)
AGCA_HDC inline int64_t child_id(int64_t n, int64_t e, int k) {
    const int s = (int)(e % 6);
    int64_t c = e / 6;
    const int64_t cx = c % n;
    c /= n;
    const int64_t cy = c % n;
    const int64_t cz = c / n;
    const int off = child_offset(s, k);
    return elem_id(2 * n, 2 * cx + (off & 1), 2 * cy + ((off >> 1) & 1), 2 * cz + ((off >> 2) & 1),
                   child_order(s, k));
}

}  // namespace agca
