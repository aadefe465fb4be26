// Assembled operators of the small coarse levels.
//
// On a level with few nodes the element loop is bound by latency, not by
// bandwidth: a z march of a few steps per workgroup plus a separate pass for the
// stored-block products.  There the level operator of eq. (2.9) (DCA on unflagged
// simplices, the stored Galerkin block on flagged ones) is assembled once per
// coefficient into its 15-point node stencil, and apply, residual and the Jacobi
// sweeps become one fully parallel gather per (node, component).  The stencil
// holds exactly the sum of the element matrices, so the operator is unchanged up
// to the order of the additions.
//
// Layout: S[((c * ncomp + d) * 15 + k) * N + p] couples component c of node p to
// component d of its neighbour k (kuhn.h nbr_mask / nbr_sign), N = (n+1)^3 nodes;
// consecutive nodes are consecutive in memory, so every load is coalesced.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kuhn.h"
#include "level_ops.h"

namespace agca {
namespace {

constexpr int NT = 256;
constexpr int NNB = kStencilPoints;

// One thread per (node, component pair c, d = blockIdx.y / NC, blockIdx.y % NC);
// rows of boundary nodes stay zero.  Loops over the 8 cells around the node and the
// simplices of each cell that contain it; everything that decides a neighbour index
// is a compile-time constant after unrolling.
template <int NC>
__global__ void __launch_bounds__(NT)
k_stencil_assemble(int n, const double* __restrict__ nu, double scale, const int32_t* __restrict__ blk,
                   const double* __restrict__ blocks, double* __restrict__ S) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    const int c = blockIdx.y / NC, d = blockIdx.y % NC;
    if (p >= N) return;
    int x, y, z;
    node_coords(p, n, x, y, z);
    const bool interior = x > 0 && y > 0 && z > 0 && x < n && y < n && z < n;
    constexpr int M = 4 * NC;
    const int64_t cells = (int64_t)n * n * n;
    double acc[NNB];
#pragma unroll
    for (int k = 0; k < NNB; ++k) acc[k] = 0.0;
    if (interior) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            // the cell that has this node as its corner k
            const int cx = x - (k & 1), cy = y - ((k >> 1) & 1), cz = z - ((k >> 2) & 1);
            const int64_t cell = cx + (int64_t)n * (cy + (int64_t)n * cz);
#pragma unroll
            for (int s = 0; s < 6; ++s) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    if (path_corner(s, a) != k) continue;
                    const int64_t slot = elem_slot(s, cell, cells);
                    const int32_t bi = blk ? blk[slot] : -1;
                    if (bi >= 0) {
                        const double* row = blocks + (int64_t)bi * M * M + (4 * c + a) * M + 4 * d;
#pragma unroll
                        for (int bv = 0; bv < 4; ++bv) acc[nbr_of(s, a, bv)] += row[bv];
                    } else {
                        const double w = nu[slot] * scale;
#pragma unroll
                        for (int bv = 0; bv < 4; ++bv) {
                            // the unit entry depends on the runtime component pair
                            const int e = NC == 1 ? path_lap(a, bv) : unit_entry(s, c, a, d, bv);
                            acc[nbr_of(s, a, bv)] += w * (double)e;
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NNB; ++k) S[((int64_t)(c * NC + d) * NNB + k) * N + p] = acc[k];
}

// One thread per (node, component c = blockIdx.y); the body is stencil_node (level_ops.h).
template <int NC, typename T, int MODE>
__global__ void __launch_bounds__(NT)
k_stencil_apply(int n, const T* __restrict__ S, const T* __restrict__ u, const T* __restrict__ b,
                const T* __restrict__ dinv, T* __restrict__ out, T omega, T alpha, T gamma,
                const T* __restrict__ xprev) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    stencil_node<NC, T, MODE>(n, p, (int)blockIdx.y, S, u, b, dinv, out, omega, alpha, gamma, xprev);
}

template <int NC, typename T, int MODE>
hipError_t launch_mode(int n, const T* S, const T* u, const T* b, const T* dinv, T* out,
                       const Sweep<T>& sw, hipStream_t st) {
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL((k_stencil_apply<NC, T, MODE>), dim3((unsigned)((N + NT - 1) / NT), NC),
                       dim3(NT), 0, st, n, S, u, b, dinv, out, sw.omega, sw.alpha, sw.gamma, sw.xprev);
    return hipGetLastError();
}

template <int NC, typename T>
hipError_t launch_nc(int mode, int n, const T* S, const T* u, const T* b, const T* dinv, T* out,
                     const Sweep<T>& sw, hipStream_t st) {
    switch (mode) {
        case MODE_APPLY: return launch_mode<NC, T, MODE_APPLY>(n, S, u, b, dinv, out, sw, st);
        case MODE_RESIDUAL: return launch_mode<NC, T, MODE_RESIDUAL>(n, S, u, b, dinv, out, sw, st);
        case MODE_JACOBI: return launch_mode<NC, T, MODE_JACOBI>(n, S, u, b, dinv, out, sw, st);
        case MODE_CHEB: return launch_mode<NC, T, MODE_CHEB>(n, S, u, b, dinv, out, sw, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_stencil_assemble(int ncomp, int n, const double* nu, double scale,
                                   const int32_t* blk, const double* blocks, double* S,
                                   hipStream_t st) {
    if (!nu || !S || n < 2 || (blk && !blocks)) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    const dim3 grid((unsigned)((N + NT - 1) / NT), ncomp * ncomp);
    if (ncomp == 1)
        hipLaunchKernelGGL(k_stencil_assemble<1>, grid, dim3(NT), 0, st, n, nu, scale, blk, blocks, S);
    else
        hipLaunchKernelGGL(k_stencil_assemble<3>, grid, dim3(NT), 0, st, n, nu, scale, blk, blocks, S);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(int ncomp, int mode, int n, const T* S, const T* u, const T* b,
                          const T* dinv, T* out, const Sweep<T>& sw, hipStream_t st) {
    if (!S || !u || !out || n < 2) return hipErrorInvalidValue;
    if (mode != MODE_APPLY && !b) return hipErrorInvalidValue;
    if ((mode == MODE_JACOBI || mode == MODE_CHEB) && !dinv) return hipErrorInvalidValue;
    if (mode == MODE_CHEB && !sw.xprev) return hipErrorInvalidValue;
    return ncomp == 1 ? launch_nc<1, T>(mode, n, S, u, b, dinv, out, sw, st)
                      : launch_nc<3, T>(mode, n, S, u, b, dinv, out, sw, st);
}

template hipError_t launch_stencil<double>(int, int, int, const double*, const double*, const double*,
                                           const double*, double*, const Sweep<double>&, hipStream_t);
template hipError_t launch_stencil<float>(int, int, int, const float*, const float*, const float*,
                                          const float*, float*, const Sweep<float>&, hipStream_t);

}  // namespace agca
