// Per-node bodies of the small-level multigrid operations: the assembled-stencil pass,
// the restriction and the prolongation of Section 2.1, and the Chebyshev pass
// coefficients of Section 4.  The one-launch-per-operation kernels (k_stencil.hip,
// k_vec.hip) and the fused coarse-level cycle (k_coarse_cycle.hip) run these same
// bodies, so both forms compute the same arithmetic in the same order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "kuhn.h"

namespace agca {

constexpr int kStencilPoints = 15;  // the node and its 14 lattice neighbours

// Chebyshev smoother of degree m (Section 4): the Chebyshev iteration for D^-1 A on
// [lmax / 10, lmax], lmax = 1.1 x the level's eigenvalue estimate.  Pass 0 from x:
// x + D^-1 (b - A x) / theta.  Pass k >= 1: x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (b - A x_k)
// with rho_k = 1 / (2 sigma - rho_{k-1}), c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta,
// rho_0 = 1 / sigma.  Host and device form the coefficients with the same FP64 steps.
struct Cheb {
    double theta = 1.0, delta = 1.0, sigma = 1.0;
    AGCA_HDC explicit Cheb(double lam) {
        const double lmax = 1.1 * lam, lmin = lmax / 10.0;
        theta = 0.5 * (lmax + lmin);
        delta = 0.5 * (lmax - lmin);
        sigma = theta / delta;
    }
    // (c1, c2) of pass k >= 1
    AGCA_HDC void coef(int k, double* c1, double* c2) const {
        double rho = 1.0 / sigma, rho_new = rho;
        for (int i = 1; i <= k; ++i) {
            rho_new = 1.0 / (2.0 * sigma - rho);
            if (i < k) rho = rho_new;
        }
        *c1 = rho_new * rho;
        *c2 = 2.0 * rho_new / delta;
    }
};

// One stencil pass at (node p, component c) of a level with n cells, N = (n+1)^3 nodes;
// S in the k_stencil.hip layout S[((c NC + d) 15 + k) N + p].  Boundary rows write 0 and
// boundary values of u count as 0.  MODE_APPLY: A u; MODE_RESIDUAL: b - A u;
// MODE_JACOBI: alpha u + omega D^-1 (b - A u); MODE_CHEB: the same plus gamma x_prev.
// ISSUE_ALL keeps every stencil load of the row ahead of the arithmetic (a scheduling
// barrier: a workgroup alone on its compute unit has no other waves to hide them behind).
template <int NC, typename T, int MODE, bool ISSUE_ALL = false>
__device__ __forceinline__ void stencil_node(int n, int64_t p, int c, const T* __restrict__ S,
                                             const T* u, const T* b, const T* __restrict__ dinv,
                                             T* out, T omega, T alpha, T gamma, const T* xprev) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    int x, y, z;
    node_coords(p, n, x, y, z);
    const int64_t o = c * N + p;
    const bool interior = x > 0 && y > 0 && z > 0 && x < n && y < n && z < n;
    if (!interior) {
        out[o] = T(0);
        return;
    }
    // the row's stencil entries first, so all their loads are in flight together
    T sv[kStencilPoints * NC];
#pragma unroll
    for (int k = 0; k < kStencilPoints; ++k)
#pragma unroll
        for (int d = 0; d < NC; ++d) sv[k * NC + d] = S[((int64_t)(c * NC + d) * kStencilPoints + k) * N + p];
    if constexpr (ISSUE_ALL) __builtin_amdgcn_sched_barrier(0);
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < kStencilPoints; ++k) {
        const int m = nbr_mask(k), sg = nbr_sign(k);
        const int qx = x + sg * (m & 1), qy = y + sg * ((m >> 1) & 1), qz = z + sg * (m >> 2);
        const bool qin = qx > 0 && qy > 0 && qz > 0 && qx < n && qy < n && qz < n;
        const int64_t q = qx + n1 * (qy + n1 * (int64_t)qz);
#pragma unroll
        for (int d = 0; d < NC; ++d) {
            const T v = u[d * N + q];
            acc = fma(sv[k * NC + d], qin ? v : T(0), acc);
        }
    }
    // every product-sum is an explicit fma, so each kernel that runs this body rounds alike
    if constexpr (MODE == MODE_APPLY) {
        out[o] = acc;
    } else if constexpr (MODE == MODE_RESIDUAL) {
        out[o] = b[o] - acc;
    } else if constexpr (MODE == MODE_CHEB) {
        out[o] = fma(omega * dinv[o], b[o] - acc, fma(gamma, xprev[o], alpha * u[o]));
    } else {
        out[o] = fma(omega * dinv[o], b[o] - acc, alpha * u[o]);
    }
}

// r_c = P^T r_f at coarse node p (level with nc cells), all components: the node itself
// plus half of its 14 lattice neighbours on the fine level, pairwise by direction;
// boundary nodes get 0
template <int NC, typename T>
__device__ __forceinline__ void restrict_node(int nc, int64_t p, const T* rf, T* rc) {
    const int64_t nc1 = nc + 1, Nc = nc1 * nc1 * nc1;
    const int64_t nf1 = 2 * nc + 1, Nf = nf1 * nf1 * nf1;
    int x, y, z;
    node_coords(p, nc, x, y, z);
    const bool interior = x > 0 && y > 0 && z > 0 && x < nc && y < nc && z < nc;
    if (!interior) {
#pragma unroll
        for (int c = 0; c < NC; ++c) rc[c * Nc + p] = T(0);
        return;
    }
    const int64_t q = 2 * x + nf1 * (2 * y + nf1 * (int64_t)(2 * z));
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const T* f = rf + c * Nf;
        T half = T(0);
#pragma unroll
        for (int d = 1; d < 8; ++d) {
            const int64_t off = (d & 1) + nf1 * (((d >> 1) & 1) + nf1 * ((d >> 2) & 1));
            half += f[q + off] + f[q - off];
        }
        rc[c * Nc + p] = f[q] + T(0.5) * half;
    }
}

// x_f += P e_c at fine node p (level with nf cells), all components: the midpoint rule
// 0.5 (e(lo) + e(hi)) with lo = hi at the fine nodes that coincide with coarse ones
// (there 0.5 (e + e) = e exactly), so every node runs the same code; a coarse endpoint on
// the boundary counts 0 (boundary slots are not part of the input); fine boundary nodes
// are left alone.  All loads are issued before the stores.
template <int NC, typename T>
__device__ __forceinline__ void prolong_add_node(int nf, int64_t p, const T* ec, T* xf) {
    const int nc = nf / 2;
    const int64_t nc1 = nc + 1, Nc = nc1 * nc1 * nc1;
    const int64_t nf1 = nf + 1, Nf = nf1 * nf1 * nf1;
    int x, y, z;
    node_coords(p, nf, x, y, z);
    if (x == 0 || y == 0 || z == 0 || x == nf || y == nf || z == nf) return;
    const int dx = x & 1, dy = y & 1, dz = z & 1;
    const int64_t lo = ((x - dx) >> 1) + nc1 * (((y - dy) >> 1) + nc1 * (int64_t)((z - dz) >> 1));
    const int64_t hi = ((x + dx) >> 1) + nc1 * (((y + dy) >> 1) + nc1 * (int64_t)((z + dz) >> 1));
    T a[NC], b[NC], v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        a[c] = ec[c * Nc + lo];
        b[c] = ec[c * Nc + hi];
        v[c] = xf[c * Nf + p];
    }
    auto on_bd = [nc](int cx, int cy, int cz) {
        return cx == 0 || cy == 0 || cz == 0 || cx == nc || cy == nc || cz == nc;
    };
    const bool lo_bd = on_bd((x - dx) >> 1, (y - dy) >> 1, (z - dz) >> 1);
    const bool hi_bd = on_bd((x + dx) >> 1, (y + dy) >> 1, (z + dz) >> 1);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        xf[c * Nf + p] = v[c] + T(0.5) * ((lo_bd ? T(0) : a[c]) + (hi_bd ? T(0) : b[c]));
}

// the level-0 solve at slot t < 27 ncomp (n = 2: the single free node (1,1,1), id 13)
template <typename T>
__device__ __forceinline__ void coarse_solve_slot(int ncomp, int t, const double* __restrict__ ainv,
                                                  const T* b, T* x) {
    const int c = t / 27, p = t % 27;
    double v = 0.0;
    if (p == 13)
        for (int d = 0; d < ncomp; ++d) v = fma(ainv[c * ncomp + d], (double)b[d * 27 + 13], v);
    x[t] = T(v);
}

}  // namespace agca
