// Geometric multigrid for the BFBT pressure operator Z = B W^-1 B^T (eq. (4.2)) on the
// pressure lattice: stencil products, damped Jacobi, probing assembly of the stencils
// and the 27-node coarse solve.  Stencil layout and the probing colours: zstencil.h.
//
// The stencil kernels are bound by HBM: a node reads its 65 stencil entries (520 bytes)
// and writes one value, the vector operands come from cache (their neighbours are the
// neighbouring threads' nodes).  One thread per node, consecutive threads along x.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kuhn.h"
#include "zstencil.h"

namespace agca {
namespace {

constexpr int NT = 256;

unsigned grid_for(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// MODE 0: out = S x;  1: out = r - S x;  2 (damped Jacobi): out = x + omega (r - S x) / S_c.
// Neighbour indices come from clamped coordinates, so every load is a lattice node; a
// neighbour outside the lattice has a stencil entry of exactly 0 (the assembly writes
// it), so its clamped stand-in adds nothing (a non-finite x stays confined to the
// nodes within two cells of it, as with the true coupling).
template <int MODE>
__global__ void __launch_bounds__(NT)
k_zstencil(int n, const double* __restrict__ S, const double* __restrict__ x,
           const double* __restrict__ r, double omega, double* __restrict__ out) {
    const int n1 = n + 1;
    const uint32_t N = (uint32_t)n1 * n1 * n1;
    const uint32_t p = blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    const int px = (int)(p % (uint32_t)n1), py = (int)((p / (uint32_t)n1) % (uint32_t)n1),
              pz = (int)(p / ((uint32_t)n1 * n1));
    uint32_t cx[5], cy[5], cz[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        cx[d] = (uint32_t)min(max(px + d - 2, 0), n);
        cy[d] = (uint32_t)min(max(py + d - 2, 0), n) * (uint32_t)n1;
        cz[d] = (uint32_t)min(max(pz + d - 2, 0), n) * (uint32_t)(n1 * n1);
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kZOffsets; ++i) {
        const int dx = kZTable.dx[i] + 2, dy = kZTable.dy[i] + 2, dz = kZTable.dz[i] + 2;
        acc = fma(S[(size_t)i * N + p], x[cx[dx] + cy[dy] + cz[dz]], acc);
    }
    if (MODE == 0)
        out[p] = acc;
    else if (MODE == 1)
        out[p] = r[p] - acc;
    else
        out[p] = x[p] + omega * (r[p] - acc) / S[(size_t)kZCentre * N + p];
}

// first Jacobi sweep from a zero guess: out = omega r / S_c
__global__ void __launch_bounds__(NT)
k_zjacobi0(int64_t N, const double* __restrict__ S, const double* __restrict__ r, double omega,
           double* __restrict__ out) {
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p < N) out[p] = omega * r[p] / S[kZCentre * N + p];
}

// indicator of the nodes of probing colour c
__global__ void __launch_bounds__(NT)
k_zprobe(int n, int c, double* __restrict__ out) {
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int px, py, pz;
    node_coords(p, n, px, py, pz);
    out[p] = z_colour(px, py, pz) == c ? 1.0 : 0.0;
}

// y = Z (indicator of colour c): at node k it is Z(k, k + o) for the one offset o whose
// node k + o has colour c; store it (0 where k + o leaves the lattice)
__global__ void __launch_bounds__(NT)
k_zextract(int n, int c, const double* __restrict__ y, double* __restrict__ S) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int px, py, pz;
    node_coords(p, n, px, py, pz);
    const int want = z_colour_mod(c - z_colour(px, py, pz));
    int oi = 0, dx = 0, dy = 0, dz = 0;
#pragma unroll
    for (int i = 0; i < kZOffsets; ++i)
        if (z_colour(kZTable.dx[i], kZTable.dy[i], kZTable.dz[i]) == want) {
            oi = i;
            dx = kZTable.dx[i];
            dy = kZTable.dy[i];
            dz = kZTable.dz[i];
        }
    const bool in = (unsigned)(px + dx) <= (unsigned)n && (unsigned)(py + dy) <= (unsigned)n &&
                    (unsigned)(pz + dz) <= (unsigned)n;
    S[oi * N + p] = in ? y[p] : 0.0;
}

// y = M r on the 27 nodes of level 0 (M row-major 27 x 27)
__global__ void __launch_bounds__(64)
k_zcoarse(const double* __restrict__ M, const double* __restrict__ r, double* __restrict__ y) {
    const int t = threadIdx.x;
    if (t >= 27) return;
    double acc = 0.0;
    for (int j = 0; j < 27; ++j) acc = fma(M[t * 27 + j], r[j], acc);
    y[t] = acc;
}

}  // namespace

hipError_t launch_zstencil(int mode, int n, const double* S, const double* x, const double* r,
                           double omega, double* out, hipStream_t st) {
    if (n < 1 || !S || !x || !out || (mode != 0 && !r) || mode < 0 || mode > 2 || x == out)
        return hipErrorInvalidValue;
    if ((int64_t)(n + 1) * (n + 1) * (n + 1) > (int64_t)UINT32_MAX / 8) return hipErrorInvalidValue;
    const unsigned g = grid_for((int64_t)(n + 1) * (n + 1) * (n + 1));
    if (mode == 0)
        hipLaunchKernelGGL(k_zstencil<0>, dim3(g), dim3(NT), 0, st, n, S, x, r, omega, out);
    else if (mode == 1)
        hipLaunchKernelGGL(k_zstencil<1>, dim3(g), dim3(NT), 0, st, n, S, x, r, omega, out);
    else
        hipLaunchKernelGGL(k_zstencil<2>, dim3(g), dim3(NT), 0, st, n, S, x, r, omega, out);
    return hipGetLastError();
}

hipError_t launch_zjacobi0(int n, const double* S, const double* r, double omega, double* out,
                           hipStream_t st) {
    if (n < 1 || !S || !r || !out) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_zjacobi0, dim3(grid_for(N)), dim3(NT), 0, st, N, S, r, omega, out);
    return hipGetLastError();
}

hipError_t launch_zprobe(int n, int colour, double* out, hipStream_t st) {
    if (n < 1 || colour < 0 || colour >= kZColours || !out) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_zprobe, dim3(grid_for(N)), dim3(NT), 0, st, n, colour, out);
    return hipGetLastError();
}

hipError_t launch_zextract(int n, int colour, const double* y, double* S, hipStream_t st) {
    if (n < 1 || colour < 0 || colour >= kZColours || !y || !S) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_zextract, dim3(grid_for(N)), dim3(NT), 0, st, n, colour, y, S);
    return hipGetLastError();
}

hipError_t launch_zcoarse(const double* M, const double* r, double* y, hipStream_t st) {
    if (!M || !r || !y || r == y) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zcoarse, dim3(1), dim3(64), 0, st, M, r, y);
    return hipGetLastError();
}

}  // namespace agca
