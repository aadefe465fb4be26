// Stencil form of the BFBT pressure operator Z = B W^-1 B^T (eq. (4.2)) and of its
// Galerkin coarsenings on the pressure lattice (host and device).
//
// B couples a pressure node k with the velocity nodes within one Kuhn edge of the fine
// node 2k, so Z couples k with k + o for o a sum of two Kuhn-lattice edges (edges are
// offsets in {0,1}^3 or {0,-1}^3): the 65 offsets o in [-2,2]^3 with
// max(o, 0) - min(o, 0) <= 2.  Linear interpolation keeps that set under P^T Z P.
// Offsets are ordered z, then y, then x ascending, so o_{64-i} = -o_i and the centre is
// o_32.  Z is symmetric, so a level stores only the centre and the 32 offsets after it
// (slot j = i - 32), offset-major over a lattice padded by 2 nodes on every side:
//   S[j * NP + kp] = Z(k, k + o_{32+j}),  kp = (x+2) + (n+5)((y+2) + (n+5)(z+2)),
// NP = (n+5)^3, 0 in the padding and where k + o leaves the lattice.  The entry of a
// lower offset is read from the neighbour: Z(k, k - o) = S[j * NP + kp - pad(o)], which
// the padding makes 0 wherever k - o leaves the lattice.
//
// Probing: colour(k) = (x + 34 y + 44 z) mod 65 gives the 65 nodes k + o (o in the
// stencil) 65 distinct colours for every k (no nonzero difference of two stencil
// offsets is a multiple of 65 under this form), so Z applied to the indicator of
// colour c returns, at node k, the single entry Z(k, k + o) whose colour is c.
#pragma once

#include "kuhn.h"   // AGCA_HDC

namespace agca {

constexpr int kZOffsets = 65;
constexpr int kZCentre = 32;
constexpr int kZStored = 33;  // the centre and the 32 offsets after it
constexpr int kZPad = 2;

AGCA_HDC constexpr int64_t z_padded_nodes(int n) {
    return (int64_t)(n + 1 + 2 * kZPad) * (n + 1 + 2 * kZPad) * (n + 1 + 2 * kZPad);
}
constexpr int kZColours = 65;
constexpr int kZColourY = 34;
constexpr int kZColourZ = 44;

struct ZOffsetTable {
    signed char dx[kZOffsets], dy[kZOffsets], dz[kZOffsets];
    signed char by_colour[kZColours];   // offset index whose colour is c
};

AGCA_HDC constexpr int z_colour_mod(int v) { return ((v % kZColours) + kZColours) % kZColours; }

AGCA_HDC constexpr int z_colour(int x, int y, int z) {
    return z_colour_mod(x + kZColourY * y + kZColourZ * z);
}

constexpr ZOffsetTable make_z_offsets() {
    ZOffsetTable t{};
    int i = 0;
    for (int dz = -2; dz <= 2; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                int mx = 0, mn = 0;
                for (int v : {dx, dy, dz}) {
                    mx = v > mx ? v : mx;
                    mn = v < mn ? v : mn;
                }
                if (mx - mn > 2) continue;
                t.dx[i] = (signed char)dx;
                t.dy[i] = (signed char)dy;
                t.dz[i] = (signed char)dz;
                ++i;
            }
    for (int c = 0; c < kZColours; ++c) t.by_colour[c] = -1;
    for (int j = 0; j < kZOffsets; ++j) t.by_colour[z_colour(t.dx[j], t.dy[j], t.dz[j])] = (signed char)j;
    return t;
}

constexpr ZOffsetTable kZTable = make_z_offsets();

constexpr bool z_colours_distinct() {
    for (int c = 0; c < kZColours; ++c)
        if (kZTable.by_colour[c] < 0) return false;   // 65 offsets on 65 colours: none shared
    return true;
}
static_assert(z_colours_distinct(), "the probing colours must separate the stencil offsets");
static_assert(kZTable.dx[kZCentre] == 0 && kZTable.dy[kZCentre] == 0 && kZTable.dz[kZCentre] == 0,
              "the centre is the middle offset");
constexpr bool z_offsets_antisymmetric() {
    for (int i = 0; i < kZOffsets; ++i)
        if (kZTable.dx[kZOffsets - 1 - i] != -kZTable.dx[i] || kZTable.dy[kZOffsets - 1 - i] != -kZTable.dy[i] ||
            kZTable.dz[kZOffsets - 1 - i] != -kZTable.dz[i])
            return false;
    return true;
}
static_assert(z_offsets_antisymmetric(), "o_{64-i} = -o_i");

}  // namespace agca
