// Hierarchy setup: viscosity-variation flags, compaction of the flagged
// elements, local Galerkin blocks (paper eqs. (2.6)-(2.7), (B.2)) and the
// Jacobi diagonals of the level operators (eq. (2.9)).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "gca_math.h"
#include "internal.h"

namespace agca {
namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// ---------------------------------------------------------------------------
// Flags.  For every element of a coarse level the minimum and maximum of the
// finest coefficient over its finest descendants, built bottom-up (min and max
// are exact, so the pyramid equals the direct definition); then the strict
// ratio test in FP64.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT)
k_minmax_from_fine(int n, const double* __restrict__ nu_fine, double* __restrict__ mn,
                   double* __restrict__ mx) {
    const int64_t ne = 6LL * n * n * n;
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    const int64_t cells_f = 8LL * n * n * n;
    double a = INFINITY, b = -INFINITY;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double v = nu_fine[elem_index(child_id(n, e, k), cells_f)];
        a = fmin(a, v);
        b = fmax(b, v);
    }
    mn[e] = a;
    mx[e] = b;
}

__global__ void __launch_bounds__(NT)
k_minmax_up(int n, const double* __restrict__ mn_f, const double* __restrict__ mx_f,
            double* __restrict__ mn, double* __restrict__ mx) {
    const int64_t ne = 6LL * n * n * n;
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    double a = INFINITY, b = -INFINITY;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t c = child_id(n, e, k);
        a = fmin(a, mn_f[c]);
        b = fmax(b, mx_f[c]);
    }
    mn[e] = a;
    mx[e] = b;
}

__global__ void __launch_bounds__(NT)
k_flag(int64_t ne, const double* __restrict__ mn, const double* __restrict__ mx, double tau,
       int mode, int32_t* __restrict__ flag) {
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    int32_t f = 0;
    if (mode == AGCA_FLAG_ALL) f = 1;
    else if (mode == AGCA_FLAG_RATIO) f = (mx[e] > tau * mn[e]) ? 1 : 0;
    flag[e] = f;
}

// Descendant means of the finest coefficient.  For P1 functions the Galerkin
// product of a coarse element (eq. (2.7)) sums the finest element matrices
// nu_d K_d of its descendants against the constant gradients of the coarse hat
// functions; all descendants have the same volume, so the block is the coarse
// element matrix with the arithmetic mean of nu_d.  The mean of equal-size
// groups is the mean of the group means, so the pyramid is exact up to rounding.
__global__ void __launch_bounds__(NT)
k_mean_from_fine(int n, const double* __restrict__ nu_fine, double* __restrict__ mean) {
    const int64_t ne = 6LL * n * n * n;
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    const int64_t cells_f = 8LL * n * n * n;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += nu_fine[elem_index(child_id(n, e, k), cells_f)];
    mean[e] = 0.125 * s;
}

__global__ void __launch_bounds__(NT)
k_mean_up(int n, const double* __restrict__ mean_f, double* __restrict__ mean) {
    const int64_t ne = 6LL * n * n * n;
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += mean_f[child_id(n, e, k)];
    mean[e] = 0.125 * s;
}

// nu_l(e) <- mean(e) on flagged elements (nu in the internal layout)
__global__ void __launch_bounds__(NT)
k_override_mean(int64_t ne, const int32_t* __restrict__ flag, const double* __restrict__ mean,
                double* __restrict__ nu) {
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne || !flag[e]) return;
    nu[elem_index(e, ne / 6)] = mean[e];
}

// Macro-element granularity (eqs. (2.8)-(2.9)).  A level-l element (cell c, order s)
// lies in the macro cube c >> l; inside that cube the Kuhn simplex with axis order
// (a1, a2, a3) is the set x_a1 >= x_a2 >= x_a3 of relative coordinates, so the macro
// simplex holding the element is the descending order of its centroid's relative
// coordinates.  In units of a quarter level-l cell that centroid is 4 (c - corner)
// plus 3, 2, 1 along the element's own a1, a2, a3: integers with distinct residues
// mod 4, hence never tied.
__device__ __forceinline__ int macro_of(int64_t e, int n, int l) {
    const int s = (int)(e % 6);
    int64_t c = e / 6;
    const int cx = (int)(c % n), cy = (int)((c / n) % n), cz = (int)(c / ((int64_t)n * n));
    const int mx = cx >> l, my = cy >> l, mz = cz >> l;
    auto w = [&](int ax) { return ax == axis1(s) ? 3 : (ax == axis2(s) ? 2 : 1); };
    const int r0 = 4 * (cx - (mx << l)) + w(0);
    const int r1 = 4 * (cy - (my << l)) + w(1);
    const int r2 = 4 * (cz - (mz << l)) + w(2);
    const int a1 = (r0 > r1) ? (r0 > r2 ? 0 : 2) : (r1 > r2 ? 1 : 2);
    const int a3 = (r0 < r1) ? (r0 < r2 ? 0 : 2) : (r1 < r2 ? 1 : 2);
    return order_index(a1, 3 - a1 - a3, a3) + 6 * (mx + 2 * (my + 2 * mz));
}

__global__ void __launch_bounds__(NT)
k_flag_macro(int64_t ne, int n, int l, uint64_t bits, int32_t* __restrict__ flag) {
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    flag[e] = (int32_t)((bits >> macro_of(e, n, l)) & 1u);
}

// max over the finest elements of each macro element of |grad eta_h| (P1 interpolant):
// along the path of simplex s the gradient components are n (eta(k_j) - eta(k_{j-1}))
// on axis a_j.  Norms are >= 0, so the maximum of their bit patterns as unsigned
// integers is the maximum of the values (exact and order-independent).
__global__ void __launch_bounds__(NT)
k_macro_grad_max(int n, int l, const double* __restrict__ eta, unsigned long long* __restrict__ gbits) {
    __shared__ unsigned long long loc[48];
    if (threadIdx.x < 48) loc[threadIdx.x] = 0ull;
    __syncthreads();
    const int64_t ne = 6LL * n * n * n;
    const int64_t n1 = n + 1;
    const double scale = (double)n;
    for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < ne; e += (int64_t)gridDim.x * NT) {
        const int s = (int)(e % 6);
        const int64_t c = e / 6;
        const int64_t cx = c % n, cy = (c / n) % n, cz = c / ((int64_t)n * n);
        const int64_t base = cx + n1 * (cy + n1 * cz);
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = path_corner(s, j);
            v[j] = eta[base + (k & 1) + n1 * (((k >> 1) & 1) + n1 * (k >> 2))];
        }
        const double g1 = scale * (v[1] - v[0]), g2 = scale * (v[2] - v[1]), g3 = scale * (v[3] - v[2]);
        const double nrm = sqrt(g1 * g1 + g2 * g2 + g3 * g3);
        atomicMax(&loc[macro_of(e, n, l)], (unsigned long long)__double_as_longlong(nrm));
    }
    __syncthreads();
    if (threadIdx.x < 48 && loc[threadIdx.x] != 0ull) atomicMax(&gbits[threadIdx.x], loc[threadIdx.x]);
}

__global__ void __launch_bounds__(NT)
k_scatter_ids(int64_t ne, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
              int32_t* __restrict__ blk, int32_t* __restrict__ blk_soa, int32_t* __restrict__ ids,
              int64_t* __restrict__ count) {
    const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (e >= ne) return;
    const int32_t f = flag[e];
    const int32_t p = pos[e];
    blk[e] = f ? p : -1;
    blk_soa[elem_index(e, ne / 6)] = f ? p : -1;  // internal layout
    if (f) ids[p] = (int32_t)e;
    if (e == ne - 1) *count = (int64_t)p + f;
}

// ---------------------------------------------------------------------------
// Local Galerkin blocks.  Component block (c,d) of an element's block follows
// the scalar recursion (B.2):  G_m = sum_k P_k^T G_child(k) P_k, with the
// constant local interpolations P_k of kuhn.h, down to the finest level where
// G is the element matrix nu_e (h/6) K(s).  One thread per (element, c, d).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_block(double* __restrict__ dst, int M, int c, int d,
                                            const double (&G)[16]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) dst[(4 * c + a) * M + 4 * d + b] = G[4 * a + b];
}

__global__ void __launch_bounds__(NT)
k_gca_fused2(int ncomp, int n, const double* __restrict__ nu_fine, double w_scale,
             const int32_t* __restrict__ blk_child, double* __restrict__ blocks_child,
             const int32_t* __restrict__ blk_self, double* __restrict__ blocks_self,
             double* __restrict__ trans_out) {
    const int64_t ne = 6LL * n * n * n;
    const int ncc = ncomp * ncomp;
    const int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (t >= ne * ncc) return;
    const int64_t e = t / ncc;
    const int cd = (int)(t % ncc);
    const int c = cd / ncomp, d = cd % ncomp;
    const int M = 4 * ncomp;
    const int64_t cells_f = 64LL * n * n * n;
    double Ge[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) Ge[i] = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int64_t ce = child_id(n, e, k);
        double Gc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) Gc[i] = 0.0;
        for (int kk = 0; kk < 8; ++kk) {
            const int64_t ge = child_id(2 * n, ce, kk);
            double K[16];
            fine_block(ncomp, (int)(ge % 6), c, d, nu_fine[elem_index(ge, cells_f)] * w_scale, K);
            add_ptkp(kk, K, Gc);
        }
        const int32_t bc = blk_child[ce];
        if (bc >= 0) store_block(blocks_child + (int64_t)bc * M * M, M, c, d, Gc);
        add_ptkp(k, Gc, Ge);
    }
    const int32_t bs = blk_self[e];
    if (bs >= 0) store_block(blocks_self + (int64_t)bs * M * M, M, c, d, Ge);
    if (trans_out) store_block(trans_out + e * M * M, M, c, d, Ge);
}

__global__ void __launch_bounds__(NT)
k_gca_from_fine(int ncomp, int n, int64_t nflag, const int32_t* __restrict__ ids,
                const double* __restrict__ nu_fine, double w_scale, double* __restrict__ blocks) {
    const int ncc = ncomp * ncomp;
    const int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (t >= nflag * ncc) return;
    const int64_t i = t / ncc;
    const int cd = (int)(t % ncc);
    const int c = cd / ncomp, d = cd % ncomp;
    const int M = 4 * ncomp;
    const int64_t e = ids[i];
    const int64_t cells_f = 8LL * n * n * n;
    double G[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) G[q] = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int64_t ge = child_id(n, e, k);
        double K[16];
        fine_block(ncomp, (int)(ge % 6), c, d, nu_fine[elem_index(ge, cells_f)] * w_scale, K);
        add_ptkp(k, K, G);
    }
    store_block(blocks + i * M * M, M, c, d, G);
}

__global__ void __launch_bounds__(NT)
k_gca_up(int ncomp, int n, const double* __restrict__ trans_in, const int32_t* __restrict__ blk_self,
         double* __restrict__ blocks_self, double* __restrict__ trans_out) {
    const int64_t ne = 6LL * n * n * n;
    const int ncc = ncomp * ncomp;
    const int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (t >= ne * ncc) return;
    const int64_t e = t / ncc;
    const int cd = (int)(t % ncc);
    const int c = cd / ncomp, d = cd % ncomp;
    const int M = 4 * ncomp;
    double G[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) G[q] = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int64_t ce = child_id(n, e, k);
        const double* src = trans_in + ce * M * M;
        double K[16];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) K[4 * a + b] = src[(4 * c + a) * M + 4 * d + b];
        add_ptkp(k, K, G);
    }
    const int32_t bs = blk_self[e];
    if (bs >= 0) store_block(blocks_self + (int64_t)bs * M * M, M, c, d, G);
    if (trans_out) store_block(trans_out + e * M * M, M, c, d, G);
}

// ---------------------------------------------------------------------------
// Diagonal of a level operator: each node gathers the diagonal entries of the
// (up to 24) simplices that contain it, from the DCA element matrix or from the
// stored block.  Boundary nodes get 0.
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(NT)
k_diagonal(int n, const double* __restrict__ nu, double scale, const int32_t* __restrict__ blk,
           const double* __restrict__ blocks, double* __restrict__ diag) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    const int x = (int)(p % n1), y = (int)((p / n1) % n1), z = (int)(p / (n1 * n1));
    const bool bd = x == 0 || y == 0 || z == 0 || x == n || y == n || z == n;
    constexpr int M = 4 * NC;
    const int64_t cells = (int64_t)n * n * n;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (!bd) {
        for (int k = 0; k < 8; ++k) {
            const int cx = x - (k & 1), cy = y - ((k >> 1) & 1), cz = z - ((k >> 2) & 1);
            const int64_t cell = cx + (int64_t)n * (cy + (int64_t)n * cz);
            for (int s = 0; s < 6; ++s) {
                int a = -1;
                for (int j = 0; j < 4; ++j)
                    if (path_corner(s, j) == k) a = j;
                if (a < 0) continue;
                const int64_t e = 6 * cell + s;
                const int32_t bi = blk ? blk[e] : -1;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (bi >= 0)
                        acc[c] += blocks[(int64_t)bi * M * M + (4 * c + a) * M + 4 * c + a];
                    else
                        acc[c] += nu[elem_slot(s, cell, cells)] * scale * (double)elem_entry(NC, s, c, a, c, a);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) diag[c * N + p] = acc[c];
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_invert_diag(int64_t count, const double* __restrict__ diag, T* __restrict__ dinv) {
    const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (i >= count) return;
    const double d = diag[i];
    dinv[i] = d > 0.0 ? T(1.0 / d) : T(0);
}

}  // namespace

hipError_t launch_minmax_from_fine(int n_coarse, const double* nu_fine, double* mn, double* mx,
                                   hipStream_t st) {
    if (!nu_fine || !mn || !mx) return hipErrorInvalidValue;
    const int64_t ne = 6LL * n_coarse * n_coarse * n_coarse;
    hipLaunchKernelGGL(k_minmax_from_fine, dim3(grid_for(ne)), dim3(NT), 0, st, n_coarse, nu_fine,
                       mn, mx);
    return hipGetLastError();
}
hipError_t launch_minmax_up(int n_coarse, const double* mn_f, const double* mx_f, double* mn,
                            double* mx, hipStream_t st) {
    if (!mn_f || !mx_f || !mn || !mx) return hipErrorInvalidValue;
    const int64_t ne = 6LL * n_coarse * n_coarse * n_coarse;
    hipLaunchKernelGGL(k_minmax_up, dim3(grid_for(ne)), dim3(NT), 0, st, n_coarse, mn_f, mx_f, mn,
                       mx);
    return hipGetLastError();
}
hipError_t launch_flag(int64_t ne, const double* mn, const double* mx, double tau, int mode,
                       int32_t* flag, hipStream_t st) {
    if (!mn || !mx || !flag) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flag, dim3(grid_for(ne)), dim3(NT), 0, st, ne, mn, mx, tau, mode, flag);
    return hipGetLastError();
}
hipError_t launch_mean_from_fine(int n_coarse, const double* nu_fine, double* mean, hipStream_t st) {
    if (!nu_fine || !mean || n_coarse < 2) return hipErrorInvalidValue;
    const int64_t ne = 6LL * n_coarse * n_coarse * n_coarse;
    hipLaunchKernelGGL(k_mean_from_fine, dim3(grid_for(ne)), dim3(NT), 0, st, n_coarse, nu_fine, mean);
    return hipGetLastError();
}
hipError_t launch_mean_up(int n_coarse, const double* mean_f, double* mean, hipStream_t st) {
    if (!mean_f || !mean || n_coarse < 2) return hipErrorInvalidValue;
    const int64_t ne = 6LL * n_coarse * n_coarse * n_coarse;
    hipLaunchKernelGGL(k_mean_up, dim3(grid_for(ne)), dim3(NT), 0, st, n_coarse, mean_f, mean);
    return hipGetLastError();
}
hipError_t launch_override_mean(int64_t ne, const int32_t* flag, const double* mean, double* nu,
                                hipStream_t st) {
    if (!flag || !mean || !nu || ne <= 0 || ne % 6) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_override_mean, dim3(grid_for(ne)), dim3(NT), 0, st, ne, flag, mean, nu);
    return hipGetLastError();
}
hipError_t launch_flag_macro(int64_t ne, int n, int l, uint64_t bits, int32_t* flag, hipStream_t st) {
    if (!flag || ne != 6LL * n * n * n || n != (2 << l)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flag_macro, dim3(grid_for(ne)), dim3(NT), 0, st, ne, n, l, bits, flag);
    return hipGetLastError();
}
hipError_t launch_macro_grad_max(int L, const double* eta, unsigned long long* gbits, hipStream_t st) {
    if (!eta || !gbits || L < 0 || L > 12) return hipErrorInvalidValue;
    const int n = 2 << L;
    const int64_t ne = 6LL * n * n * n;
    const unsigned blocks = (unsigned)std::min<int64_t>((ne + NT - 1) / NT, 4096);
    hipLaunchKernelGGL(k_macro_grad_max, dim3(blocks), dim3(NT), 0, st, n, L, eta, gbits);
    return hipGetLastError();
}
hipError_t compact_scratch_bytes(int64_t ne, size_t* bytes) {
    size_t tmp = 0;
    hipError_t err = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, (const int32_t*)nullptr,
                                                      (int32_t*)nullptr, (int)ne);
    *bytes = tmp + (size_t)ne * sizeof(int32_t) + 256;
    return err;
}
hipError_t launch_compact(int64_t ne, const int32_t* flag, int32_t* blk, int32_t* blk_soa,
                          int32_t* ids, int64_t* count_dev, void* scratch, size_t scratch_bytes,
                          hipStream_t st) {
    if (!flag || !blk || !blk_soa || !ids || !count_dev || !scratch) return hipErrorInvalidValue;
    // scratch: [pos (ne int32, 256-aligned)] [cub temp]
    int32_t* pos = static_cast<int32_t*>(scratch);
    size_t off = (((size_t)ne * sizeof(int32_t)) + 255) & ~(size_t)255;
    void* tmp = static_cast<char*>(scratch) + off;
    size_t tmp_bytes = scratch_bytes - off;
    hipError_t err = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, flag, pos, (int)ne, st);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_scatter_ids, dim3(grid_for(ne)), dim3(NT), 0, st, ne, flag, pos, blk, blk_soa,
                       ids, count_dev);
    return hipGetLastError();
}
hipError_t launch_gca_fused2(int ncomp, int n, const double* nu_fine, double h_fine,
                             const int32_t* blk_child, double* blocks_child,
                             const int32_t* blk_self, double* blocks_self, double* trans_out,
                             hipStream_t st) {
    if (!nu_fine || !blk_child || !blk_self) return hipErrorInvalidValue;
    const int64_t threads = 6LL * n * n * n * ncomp * ncomp;
    hipLaunchKernelGGL(k_gca_fused2, dim3(grid_for(threads)), dim3(NT), 0, st, ncomp, n, nu_fine,
                       h_fine / 6.0, blk_child, blocks_child, blk_self, blocks_self, trans_out);
    return hipGetLastError();
}
hipError_t launch_gca_from_fine(int ncomp, int n, int64_t nflag, const int32_t* ids,
                                const double* nu_fine, double h_fine, double* blocks,
                                hipStream_t st) {
    const int64_t threads = nflag * ncomp * ncomp;
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gca_from_fine, dim3(grid_for(threads)), dim3(NT), 0, st, ncomp, n, nflag,
                       ids, nu_fine, h_fine / 6.0, blocks);
    return hipGetLastError();
}
hipError_t launch_gca_up(int ncomp, int n, const double* trans_in, const int32_t* blk_self,
                         double* blocks_self, double* trans_out, hipStream_t st) {
    if (!trans_in || !blk_self) return hipErrorInvalidValue;
    const int64_t threads = 6LL * n * n * n * ncomp * ncomp;
    hipLaunchKernelGGL(k_gca_up, dim3(grid_for(threads)), dim3(NT), 0, st, ncomp, n, trans_in,
                       blk_self, blocks_self, trans_out);
    return hipGetLastError();
}
hipError_t launch_diagonal(int ncomp, int n, const double* nu, double scale, const int32_t* blk,
                           const double* blocks, double* diag, hipStream_t st) {
    if (!nu || !diag || (blk && !blocks)) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    if (ncomp == 1)
        hipLaunchKernelGGL(k_diagonal<1>, dim3(grid_for(N)), dim3(NT), 0, st, n, nu, scale, blk,
                           blocks, diag);
    else
        hipLaunchKernelGGL(k_diagonal<3>, dim3(grid_for(N)), dim3(NT), 0, st, n, nu, scale, blk,
                           blocks, diag);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_invert_diag(int64_t count, const double* diag, T* dinv, hipStream_t st) {
    if (!diag || !dinv) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_invert_diag<T>, dim3(grid_for(count)), dim3(NT), 0, st, count, diag, dinv);
    return hipGetLastError();
}
template hipError_t launch_invert_diag<double>(int64_t, const double*, double*, hipStream_t);
template hipError_t launch_invert_diag<float>(int64_t, const double*, float*, hipStream_t);

}  // namespace agca
