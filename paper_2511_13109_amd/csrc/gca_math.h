// Local Galerkin triple products of the element-wise recursion (paper eq. (2.7)).
//
// For one component block (c,d) (eq. (B.2): each block is coarsened with the
// scalar interpolation), the Galerkin matrix of an element m is
//   G_m = sum_k P_k^T G_{child k} P_k,
// with the constant 4x4 local interpolations P_k of kuhn.h and, on the finest
// level, G = nu_e (h/6) K(s) the element matrix.  Compiled for the device and,
// in tests, for the host.
#pragma once

#include "cube_math.h"

namespace agca {

// G += P_k^T K P_k
AGCA_HD void add_ptkp(int k, const double (&K)[16], double (&G)[16]) {
    double P[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) P[a][i] = 0.5 * (double)kP2(k, a, i);
    double Y[16];  // K P
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) s += K[4 * a + b] * P[b][j];
            Y[4 * a + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) s += P[a][i] * Y[4 * a + j];
            G[4 * i + j] += s;
        }
}

// component block (c,d) of the finest element matrix of simplex s, scaled by w
AGCA_HD void fine_block(int ncomp, int s, int c, int d, double w, double (&K)[16]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) K[4 * a + b] = w * (double)elem_entry(ncomp, s, c, a, d, b);
}

}  // namespace agca
