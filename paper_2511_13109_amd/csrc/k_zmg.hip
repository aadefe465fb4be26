// Geometric multigrid for the BFBT pressure operator Z = B W^-1 B^T (eq. (4.2)) on the
// pressure lattice: stencil products, damped Jacobi, probing assembly of the stencils
// and the 27-node coarse solve.  Stencil layout and the probing colours: zstencil.h.
//
// The stencil kernels are bound by HBM: a node reads its 33 stored stencil entries (264
// bytes; the 32 lower entries are its neighbours' stored ones, read again from cache) and
// writes one value, the vector operands come from cache (their neighbours are the
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
// S: the stored half of a symmetric stencil over the padded lattice (zstencil.h).  Each
// stored offset o contributes twice: S_o(k) x(k + o) and, for the lower offset -o,
// S_o(k - o) x(k - o), the second entry being the neighbour's own (in cache once the
// neighbouring threads have read it).  Neighbour indices of x come from clamped
// coordinates, so every load is a lattice node; wherever a neighbour leaves the lattice
// its stencil entry is exactly 0 (written by the assembly, or padding), so its clamped
// stand-in adds nothing (a non-finite x stays confined to the nodes within two cells of
// it, as with the true coupling).
template <int MODE>
__global__ void __launch_bounds__(NT)
k_zstencil(int n, const double* __restrict__ S, const double* __restrict__ x,
           const double* __restrict__ r, double omega, double* __restrict__ out) {
    const int n1 = n + 1, np1 = n + 1 + 2 * kZPad;
    const uint32_t N = (uint32_t)n1 * n1 * n1;
    const size_t NP = (size_t)np1 * np1 * np1;
    const uint32_t p = blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    const int px = (int)(p % (uint32_t)n1), py = (int)((p / (uint32_t)n1) % (uint32_t)n1),
              pz = (int)(p / ((uint32_t)n1 * n1));
    const int64_t kp = (px + kZPad) + (int64_t)np1 * ((py + kZPad) + (int64_t)np1 * (pz + kZPad));
    uint32_t cx[5], cy[5], cz[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        cx[d] = (uint32_t)min(max(px + d - 2, 0), n);
        cy[d] = (uint32_t)min(max(py + d - 2, 0), n) * (uint32_t)n1;
        cz[d] = (uint32_t)min(max(pz + d - 2, 0), n) * (uint32_t)(n1 * n1);
    }
    double acc = S[kp] * x[p];
#pragma unroll
    for (int j = 1; j < kZStored; ++j) {
        const int i = kZCentre + j;
        const int dx = kZTable.dx[i], dy = kZTable.dy[i], dz = kZTable.dz[i];
        const int64_t dp = dx + (int64_t)np1 * (dy + (int64_t)np1 * dz);
        const double* Sj = S + (size_t)j * NP;
        acc = fma(Sj[kp], x[cx[dx + 2] + cy[dy + 2] + cz[dz + 2]], acc);
        acc = fma(Sj[kp - dp], x[cx[2 - dx] + cy[2 - dy] + cz[2 - dz]], acc);
    }
    if (MODE == 0)
        out[p] = acc;
    else if (MODE == 1)
        out[p] = r[p] - acc;
    else
        out[p] = x[p] + omega * (r[p] - acc) / S[kp];
}

// first Jacobi sweep from a zero guess: out = omega r / S_c
__global__ void __launch_bounds__(NT)
k_zjacobi0(int n, const double* __restrict__ S, const double* __restrict__ r, double omega,
           double* __restrict__ out) {
    const int n1 = n + 1, np1 = n + 1 + 2 * kZPad;
    const int64_t N = (int64_t)n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int px, py, pz;
    node_coords(p, n, px, py, pz);
    const int64_t kp = (px + kZPad) + (int64_t)np1 * ((py + kZPad) + (int64_t)np1 * (pz + kZPad));
    out[p] = omega * r[p] / S[kp];
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
// node k + o has colour c; stored when o is one of the stored offsets (0 where k + o
// leaves the lattice).  A lower offset's value is the stored entry of node k + o
// (symmetry), probed with the colour of k, so each stored entry is written once.
__global__ void __launch_bounds__(NT)
k_zextract(int n, int c, const double* __restrict__ y, double* __restrict__ S) {
    const int n1 = n + 1, np1 = n + 1 + 2 * kZPad;
    const int64_t N = (int64_t)n1 * n1 * n1;
    const size_t NP = (size_t)np1 * np1 * np1;
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
    if (oi < kZCentre) return;
    const bool in = (unsigned)(px + dx) <= (unsigned)n && (unsigned)(py + dy) <= (unsigned)n &&
                    (unsigned)(pz + dz) <= (unsigned)n;
    const int64_t kp = (px + kZPad) + (int64_t)np1 * ((py + kZPad) + (int64_t)np1 * (pz + kZPad));
    S[(size_t)(oi - kZCentre) * NP + kp] = in ? y[p] : 0.0;
}

// the full 65-offset form of a stored stencil: out[i N + k] = Z(k, k + o_i)
__global__ void __launch_bounds__(NT)
k_zexpand(int n, const double* __restrict__ S, double* __restrict__ out) {
    const int n1 = n + 1, np1 = n + 1 + 2 * kZPad;
    const int64_t N = (int64_t)n1 * n1 * n1;
    const size_t NP = (size_t)np1 * np1 * np1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int px, py, pz;
    node_coords(p, n, px, py, pz);
    const int64_t kp = (px + kZPad) + (int64_t)np1 * ((py + kZPad) + (int64_t)np1 * (pz + kZPad));
#pragma unroll
    for (int i = 0; i < kZOffsets; ++i) {
        const int dx = kZTable.dx[i], dy = kZTable.dy[i], dz = kZTable.dz[i];
        const int64_t dp = dx + (int64_t)np1 * (dy + (int64_t)np1 * dz);
        // o_i stored (i >= 32) at node k; a lower o_i as -o_i = o_{64-i} at node k + o_i
        out[i * N + p] = i >= kZCentre ? S[(size_t)(i - kZCentre) * NP + kp]
                                       : S[(size_t)(kZOffsets - 1 - i - kZCentre) * NP + kp + dp];
    }
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
    hipLaunchKernelGGL(k_zjacobi0, dim3(grid_for(N)), dim3(NT), 0, st, n, S, r, omega, out);
    return hipGetLastError();
}

hipError_t launch_zexpand(int n, const double* S, double* out, hipStream_t st) {
    if (n < 1 || !S || !out) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_zexpand, dim3(grid_for(N)), dim3(NT), 0, st, n, S, out);
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
