// Per-cell element arithmetic of the matrix-free operator (paper eq. (2.3)).
//
// A lattice cell holds 6 Kuhn simplices.  Given the 8 corner values U[k][c]
// (corner k = dx + 2 dy + 4 dz, component c) these routines add each simplex's
// contribution A_e u_e to the corner accumulators F[k][c].
//
// Scalar (-div nu grad u): the unit element matrix is (h/6) times the path
// Laplacian, so simplex s with path corners k0..k3 contributes the fluxes
// g_j = w (U[k_j] - U[k_{j-1}]), w = nu_e h / 6:  F[k_{j-1}] -= g_j, F[k_j] += g_j.
//
// Vector (-div 2 nu eps(u)): with path differences d_j = U[k_j] - U[k_{j-1}]
// (j = 1..3) the displacement gradient in the simplex's axis frame is
// G[i][j] = d_j[a_i] / h.  The stress 2 nu eps = nu (G + G^T) tested against the
// barycentric gradients g0 = -e_a1, g1 = e_a1 - e_a2, ... gives the same flux
// structure, now with vector fluxes q_j[a_i] = w (d_j[a_i] + d_i[a_j]).
//
// Compiled for the device and, in tests, for the host.
#pragma once

#include "kuhn.h"

#if defined(__HIPCC__)
#define AGCA_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define AGCA_HD inline
using std::fma;
#endif

namespace agca {

template <int S, int NC, typename T>
AGCA_HD void tet_dca(const T (&U)[8][NC], T w, T (&F)[8][NC]) {
    constexpr int a1 = axis1(S), a2 = axis2(S), a3 = axis3(S);
    constexpr int k0 = 0, k1 = 1 << a1, k2 = (1 << a1) | (1 << a2), k3 = 7;
    if constexpr (NC == 1) {
        const T d1 = U[k1][0] - U[k0][0];
        const T d2 = U[k2][0] - U[k1][0];
        const T d3 = U[k3][0] - U[k2][0];
        F[k0][0] = fma(-w, d1, F[k0][0]);
        F[k1][0] = fma(w, d1 - d2, F[k1][0]);
        F[k2][0] = fma(w, d2 - d3, F[k2][0]);
        F[k3][0] = fma(w, d3, F[k3][0]);
    } else {
        constexpr int A[3] = {a1, a2, a3};
        T d[3][3];  // d[j][c]
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d[0][c] = U[k1][c] - U[k0][c];
            d[1][c] = U[k2][c] - U[k1][c];
            d[2][c] = U[k3][c] - U[k2][c];
        }
        // symmetric s[i][j] = d_j[a_i] + d_i[a_j]; the flux of path step j in component a_i
        // is w s[i][j]
        T sm[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) sm[i][i] = d[i][A[i]] + d[i][A[i]];
        sm[0][1] = sm[1][0] = d[1][A[0]] + d[0][A[1]];
        sm[0][2] = sm[2][0] = d[2][A[0]] + d[0][A[2]];
        sm[1][2] = sm[2][1] = d[2][A[1]] + d[1][A[2]];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int c = A[i];
            F[k0][c] = fma(-w, sm[i][0], F[k0][c]);
            F[k1][c] = fma(w, sm[i][0] - sm[i][1], F[k1][c]);
            F[k2][c] = fma(w, sm[i][1] - sm[i][2], F[k2][c]);
            F[k3][c] = fma(w, sm[i][2], F[k3][c]);
        }
    }
}

// stored local matrix B (row (c,a) = 4c+a, column (d,b) = 4d+b, path-ordered vertices)
template <int S, int NC, typename T, typename BT>
AGCA_HD void tet_block(const T (&U)[8][NC], const BT* __restrict__ B, T (&F)[8][NC]) {
    constexpr int M = 4 * NC;
    T x[M];
#pragma unroll
    for (int d = 0; d < NC; ++d)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) x[4 * d + bb] = U[path_corner(S, bb)][d];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        T y = T(0);
#pragma unroll
        for (int c = 0; c < M; ++c) y += T(B[r * M + c]) * x[c];
        F[path_corner(S, r & 3)][r >> 2] += y;
    }
}

// all six simplices of a cell with coefficients w[s] (already multiplied by h/6)
template <int NC, typename T>
AGCA_HD void cell_dca(const T (&U)[8][NC], const T (&w)[6], T (&F)[8][NC]) {
    tet_dca<0, NC, T>(U, w[0], F);
    tet_dca<1, NC, T>(U, w[1], F);
    tet_dca<2, NC, T>(U, w[2], F);
    tet_dca<3, NC, T>(U, w[3], F);
    tet_dca<4, NC, T>(U, w[4], F);
    tet_dca<5, NC, T>(U, w[5], F);
}

// add a precomputed local product y = B u_e (layout 4c + a) to the simplex's corners
template <int S, int NC, typename T>
AGCA_HD void tet_add_product(const T* __restrict__ y, T (&F)[8][NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < 4; ++a) F[path_corner(S, a)][c] += y[4 * c + a];
}

template <int S, int NC, typename T>
AGCA_HD void tet_mixed(const T (&U)[8][NC], T w, int32_t bi, const T* __restrict__ yblk,
                       T (&F)[8][NC]) {
    if (bi >= 0)
        tet_add_product<S, NC, T>(yblk + (int64_t)bi * (4 * NC), F);
    else
        tet_dca<S, NC, T>(U, w, F);
}

// cell with per-simplex choice: the stored block's product (computed beforehand for every
// flagged simplex) where bi[s] >= 0, DCA otherwise
template <int NC, typename T>
AGCA_HD void cell_mixed(const T (&U)[8][NC], const T (&w)[6], const int32_t (&bi)[6],
                        const T* __restrict__ yblk, T (&F)[8][NC]) {
    tet_mixed<0, NC, T>(U, w[0], bi[0], yblk, F);
    tet_mixed<1, NC, T>(U, w[1], bi[1], yblk, F);
    tet_mixed<2, NC, T>(U, w[2], bi[2], yblk, F);
    tet_mixed<3, NC, T>(U, w[3], bi[3], yblk, F);
    tet_mixed<4, NC, T>(U, w[4], bi[4], yblk, F);
    tet_mixed<5, NC, T>(U, w[5], bi[5], yblk, F);
}

}  // namespace agca

namespace agca {

// Element energy form u_e^T K_e w_e of the unit-coefficient element matrix (without h/6):
// scalar: sum_j du_j dw_j; vector: sum_ij (G_u[i][j] + G_u[j][i]) G_w[i][j].
template <int S, int NC, typename T>
AGCA_HD T tet_energy(const T (&U)[8][NC], const T (&W)[8][NC]) {
    constexpr int a1 = axis1(S), a2 = axis2(S);
    constexpr int k[4] = {0, 1 << a1, (1 << a1) | (1 << a2), 7};
    if constexpr (NC == 1) {
        T acc = T(0);
#pragma unroll
        for (int j = 1; j < 4; ++j) acc += (U[k[j]][0] - U[k[j - 1]][0]) * (W[k[j]][0] - W[k[j - 1]][0]);
        return acc;
    } else {
        constexpr int A[3] = {axis1(S), axis2(S), axis3(S)};
        T du[3][3], dw[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                du[j][c] = U[k[j + 1]][c] - U[k[j]][c];
                dw[j][c] = W[k[j + 1]][c] - W[k[j]][c];
            }
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc += (du[j][A[i]] + du[i][A[j]]) * dw[j][A[i]];
        return acc;
    }
}

template <int NC, typename T>
AGCA_HD void cell_energy(const T (&U)[8][NC], const T (&W)[8][NC], T (&e)[6]) {
    e[0] = tet_energy<0, NC, T>(U, W);
    e[1] = tet_energy<1, NC, T>(U, W);
    e[2] = tet_energy<2, NC, T>(U, W);
    e[3] = tet_energy<3, NC, T>(U, W);
    e[4] = tet_energy<4, NC, T>(U, W);
    e[5] = tet_energy<5, NC, T>(U, W);
}

}  // namespace agca
