// Generalized Stokes pieces (paper Section 3.1, eqs. (3.3)-(3.5)): velocity P1 on the
// finest level L (P1-iso-P2), pressure P1 on level L-1 with every node of that level a
// degree of freedom.
//
//   B = - integral psi_k div Phi_j = -P^T B_L,
//   (B_L u)_v = sum over the simplices d containing v of |d|/4 div_d(u),
// because psi_k is linear on every fine simplex (its mean over d is the mean of its
// vertex values, which the interpolation P of eq. (2.4) gives).  On the Kuhn lattice
// |d| = h^3/6 and the barycentric gradients are grad(s, a, c) / h (kuhn.h), so
//   (B_L u)_v = h^2/24 sum_{d containing v} sum_{b, c} grad(s, b, c) u_c(b).
// B^T p = -B_L^T (P p).  The pressure preconditioner is the lumped mass weighted by
// 1/nu, m = P^T m_L, m_L(v) = h^3/24 sum_{d containing v} 1/nu_d.
//
// Every kernel gathers per node (no atomics): the simplices around a node are the
// ones of the 8 cells sharing it whose path passes through it, and their vertices
// are the node's 15 lattice neighbours (kuhn.h nbr_of).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kuhn.h"

namespace agca {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ void node_xyz(int64_t p, int n, int& x, int& y, int& z) {
    node_coords(p, n, x, y, z);
}

// cell of node (x,y,z) that has the node as its corner k, and whether it exists
__device__ __forceinline__ bool cell_of(int n, int x, int y, int z, int k, int64_t& cell) {
    const int cx = x - (k & 1), cy = y - ((k >> 1) & 1), cz = z - ((k >> 2) & 1);
    cell = cx + (int64_t)n * (cy + (int64_t)n * cz);
    return cx >= 0 && cy >= 0 && cz >= 0 && cx < n && cy < n && cz < n;
}

// q_v = -(B_L u)_v on every fine node (velocity boundary values are zero)
__global__ void __launch_bounds__(NT)
k_div_fine(int n, const double* __restrict__ u, double* __restrict__ q) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int x, y, z;
    node_xyz(p, n, x, y, z);
    // velocity at the 15 neighbours, zero outside the interior
    double U[15][3];
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        const int m = nbr_mask(k), sg = nbr_sign(k);
        const int qx = x + sg * (m & 1), qy = y + sg * ((m >> 1) & 1), qz = z + sg * (m >> 2);
        const bool in = qx > 0 && qy > 0 && qz > 0 && qx < n && qy < n && qz < n;
        const int64_t qi = in ? qx + n1 * (qy + n1 * (int64_t)qz) : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) U[k][c] = in ? u[c * N + qi] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int64_t cell;
        if (!cell_of(n, x, y, z, k, cell)) continue;
#pragma unroll
        for (int s = 0; s < 6; ++s)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (path_corner(s, a) != k) continue;
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (grad(s, b, c) != 0) acc += (double)grad(s, b, c) * U[nbr_of(s, a, b)][c];
            }
    }
    const double h = 1.0 / n;
    q[p] = -(h * h / 24.0) * acc;
}

// out[(c, j)] += -(B_L^T pf)_(j, c) on interior fine nodes
__global__ void __launch_bounds__(NT)
k_grad_fine_add(int n, const double* __restrict__ pf, double* __restrict__ out) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int x, y, z;
    node_xyz(p, n, x, y, z);
    if (x == 0 || y == 0 || z == 0 || x == n || y == n || z == n) return;
    double P[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        const int m = nbr_mask(k), sg = nbr_sign(k);
        // interior node: every neighbour lies in the lattice
        P[k] = pf[(x + sg * (m & 1)) + n1 * ((y + sg * ((m >> 1) & 1)) + n1 * (int64_t)(z + sg * (m >> 2)))];
    }
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int s = 0; s < 6; ++s)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (path_corner(s, a) != k) continue;
                double sum = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) sum += P[nbr_of(s, a, b)];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (grad(s, a, c) != 0) acc[c] += (double)grad(s, a, c) * sum;
            }
    }
    const double h = 1.0 / n;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * N + p] -= (h * h / 24.0) * acc[c];
}

// m_L(v) = h^3/24 sum_{d containing v} 1/nu_d on every fine node
__global__ void __launch_bounds__(NT)
k_mass_fine(int n, const double* __restrict__ nu, double* __restrict__ mf) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int x, y, z;
    node_xyz(p, n, x, y, z);
    const int64_t cells = (int64_t)n * n * n;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int64_t cell;
        if (!cell_of(n, x, y, z, k, cell)) continue;
#pragma unroll
        for (int s = 0; s < 6; ++s)
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (path_corner(s, a) == k) acc += 1.0 / nu[elem_slot(s, cell, cells)];
    }
    const double h = 1.0 / n;
    mf[p] = (h * h * h / 24.0) * acc;
}

// out = P^T qf over every node of the coarse level (nc cells), boundary included
__global__ void __launch_bounds__(NT)
k_restrict_all(int nc, const double* __restrict__ qf, double* __restrict__ out) {
    const int64_t nc1 = nc + 1, Nc = nc1 * nc1 * nc1;
    const int nf = 2 * nc;
    const int64_t nf1 = nf + 1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= Nc) return;
    int x, y, z;
    node_xyz(p, nc, x, y, z);
    const int X = 2 * x, Y = 2 * y, Z = 2 * z;
    double half = 0.0;
#pragma unroll
    for (int m = 1; m < 8; ++m) {
        const int dx = m & 1, dy = (m >> 1) & 1, dz = m >> 2;
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            const int qx = X + sg * dx, qy = Y + sg * dy, qz = Z + sg * dz;
            if (qx >= 0 && qy >= 0 && qz >= 0 && qx <= nf && qy <= nf && qz <= nf)
                half += qf[qx + nf1 * (qy + nf1 * (int64_t)qz)];
        }
    }
    out[p] = qf[X + nf1 * (Y + nf1 * (int64_t)Z)] + 0.5 * half;
}

// pf = P pc (ADD: pf += P pc) on every node of the fine level (nf cells), boundary included
template <bool ADD>
__global__ void __launch_bounds__(NT)
k_prolong_all(int nf, const double* __restrict__ pc, double* __restrict__ pf) {
    const int nc = nf / 2;
    const int64_t nc1 = nc + 1;
    const int64_t Nf = (int64_t)(nf + 1) * (nf + 1) * (nf + 1);
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= Nf) return;
    int x, y, z;
    node_xyz(p, nf, x, y, z);
    const int dx = x & 1, dy = y & 1, dz = z & 1;
    const int64_t lo = ((x - dx) >> 1) + nc1 * (((y - dy) >> 1) + nc1 * (int64_t)((z - dz) >> 1));
    const int64_t hi = ((x + dx) >> 1) + nc1 * (((y + dy) >> 1) + nc1 * (int64_t)((z + dz) >> 1));
    const double v = (dx | dy | dz) ? 0.5 * (pc[lo] + pc[hi]) : pc[lo];
    pf[p] = ADD ? pf[p] + v : v;
}

__global__ void __launch_bounds__(NT)
k_div_elementwise(int64_t n, const double* __restrict__ num, const double* __restrict__ den,
                  double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) out[i] = num[i] / den[i];
}

// out = a * b elementwise
__global__ void __launch_bounds__(NT)
k_mul_elementwise(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                  double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) out[i] = a[i] * b[i];
}

// Colour (x mod 3) + 3 (y mod 3) + 9 (z mod 3) of the nodes of a level with n cells per
// axis.  mode 0: out = indicator of the colour; mode 1: out = src on the colour's nodes
// (others untouched).
__global__ void __launch_bounds__(NT)
k_colour(int n, int colour, int mode, const double* __restrict__ src, double* __restrict__ out) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < N; p += stride) {
        int x, y, z;
        node_coords(p, n, x, y, z);
        const bool on = (x % 3) + 3 * (y % 3) + 9 * (z % 3) == colour;
        if (mode == 0)
            out[p] = on ? 1.0 : 0.0;
        else if (on)
            out[p] = src[p];
    }
}

// y += sign * coef[0] * x with the coefficient read from device memory
__global__ void __launch_bounds__(NT)
k_axpy_dev(int64_t n, const double* __restrict__ coef, double sign, const double* __restrict__ x,
           double* __restrict__ y) {
    const double a = sign * coef[0];
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

// Classical Gram-Schmidt against nv contiguous vectors V_i = V + i * ld (the FGMRES
// basis): one pass over w and the basis for all the dot products, one for the update.
// A workgroup owns GS_CHUNK consecutive entries; each thread keeps its GS_PER entries of
// w in registers while the workgroup walks the basis, so w is read once.  The dots of
// every workgroup are reduced in a fixed order (wavefront shuffles, then LDS), and the
// partials of all workgroups by k_gs_sum, so the results are bitwise reproducible.
constexpr int GS_PER = 8;
constexpr int GS_CHUNK = NT * GS_PER;

__device__ __forceinline__ double gs_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// partial[i * gridDim.x + block] = sum over the block's entries of w V_i (i < nv), and
// partial[nv * gridDim.x + block] = sum of w^2; a basis stored in FP32 is widened on
// the fly (the products and sums stay FP64)
template <typename VT>
__global__ void __launch_bounds__(NT)
k_gs_dots(int64_t n, const double* __restrict__ w, const VT* __restrict__ V, int64_t ld, int nv,
          double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const int64_t base = (int64_t)blockIdx.x * GS_CHUNK + threadIdx.x;
    double wv[GS_PER];
#pragma unroll
    for (int m = 0; m < GS_PER; ++m) {
        const int64_t j = base + (int64_t)m * NT;
        wv[m] = j < n ? w[j] : 0.0;
    }
    for (int i = 0; i <= nv; ++i) {
        double acc = 0.0;
        if (i < nv) {
            const VT* v = V + (int64_t)i * ld;
#pragma unroll
            for (int m = 0; m < GS_PER; ++m) {
                const int64_t j = base + (int64_t)m * NT;
                acc += wv[m] * (j < n ? (double)v[j] : 0.0);
            }
        } else {
#pragma unroll
            for (int m = 0; m < GS_PER; ++m) acc += wv[m] * wv[m];
        }
        acc = gs_wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < NT / 64; ++q) t += red[q];
            partial[(int64_t)i * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// out[i] = sum over the nb partials of row i (one workgroup per row, fixed order)
__global__ void __launch_bounds__(NT)
k_gs_sum(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    __shared__ double red[NT / 64];
    const double* row = partial + (int64_t)blockIdx.x * nb;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) acc += row[b];
    acc = gs_wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NT / 64; ++q) t += red[q];
        out[blockIdx.x] = t;
    }
}

// w -= sum_i h[i] V_i (h on the device; an FP32 basis widened on the fly)
template <typename VT>
__global__ void __launch_bounds__(NT)
k_gs_update(int64_t n, double* __restrict__ w, const VT* __restrict__ V, int64_t ld, int nv,
            const double* __restrict__ h) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t j = blockIdx.x * (int64_t)NT + threadIdx.x; j < n; j += stride) {
        double acc = 0.0;
        for (int i = 0; i < nv; ++i) acc += h[i] * (double)V[(int64_t)i * ld + j];
        w[j] -= acc;
    }
}

// The same two passes over an FP32 basis, four consecutive entries per lane and load
// (the basis vectors start at 16-byte aligned offsets, ld a multiple of 4): a wavefront
// then keeps as many bytes in flight per basis vector as the FP64 passes (with one
// 4-byte load per entry the passes ran at 3.8 TB/s against 5.3 for the FP64 basis).
// The dot pass owns GS_CHUNK_F32 = 2 GS_CHUNK entries per workgroup (gs_blocks_f32).
constexpr int GS_QUADS = 4;                   // float4 loads per lane and basis vector
constexpr int GS_CHUNK_F32 = NT * 4 * GS_QUADS;

__global__ void __launch_bounds__(NT)
k_gs_dots_f32(int64_t n, const double* __restrict__ w, const float* __restrict__ V, int64_t ld, int nv,
              double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const int64_t base = (int64_t)blockIdx.x * GS_CHUNK_F32 + 4 * threadIdx.x;
    double wv[4 * GS_QUADS];
#pragma unroll
    for (int q = 0; q < GS_QUADS; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t j = base + (int64_t)q * 4 * NT + e;
            wv[4 * q + e] = j < n ? w[j] : 0.0;
        }
    for (int i = 0; i <= nv; ++i) {
        double acc = 0.0;
        if (i < nv) {
            const float* v = V + (int64_t)i * ld;
            float4 vv[GS_QUADS];
#pragma unroll
            for (int q = 0; q < GS_QUADS; ++q) {
                // the quad starts inside the padded vector (ld >= n, a multiple of 4)
                const int64_t j = base + (int64_t)q * 4 * NT;
                vv[q] = j < n ? *reinterpret_cast<const float4*>(v + j) : float4{0.0f, 0.0f, 0.0f, 0.0f};
            }
#pragma unroll
            for (int q = 0; q < GS_QUADS; ++q) {
                const int64_t j = base + (int64_t)q * 4 * NT;
                const float f[4] = {vv[q].x, vv[q].y, vv[q].z, vv[q].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) acc += wv[4 * q + e] * (j + e < n ? (double)f[e] : 0.0);
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4 * GS_QUADS; ++m) acc += wv[m] * wv[m];
        }
        acc = gs_wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < NT / 64; ++q) t += red[q];
            partial[(int64_t)i * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// w -= sum_i h[i] V_i over four consecutive entries per lane, the basis loads of four
// vectors issued before their products are summed (in the order of i, as above)
__global__ void __launch_bounds__(NT)
k_gs_update_f32(int64_t n, double* __restrict__ w, const float* __restrict__ V, int64_t ld, int nv,
                const double* __restrict__ h) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t j = 4 * (blockIdx.x * (int64_t)NT + threadIdx.x); j < n; j += 4 * stride) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int i = 0; i < nv; ++i) {
            const float4 vv = *reinterpret_cast<const float4*>(V + (int64_t)i * ld + j);
            const double hi = h[i];
            a[0] += hi * (double)vv.x;
            a[1] += hi * (double)vv.y;
            a[2] += hi * (double)vv.z;
            a[3] += hi * (double)vv.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (j + e < n) w[j + e] -= a[e];
    }
}

// y = a x rounded to FP32 (a new FP32 basis vector)
__global__ void __launch_bounds__(NT)
k_scale_to_f32(int64_t n, double a, const double* __restrict__ x, float* __restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t j = blockIdx.x * (int64_t)NT + threadIdx.x; j < n; j += stride) y[j] = (float)(a * x[j]);
}

unsigned grid_for(int64_t n) { return (unsigned)((n + NT - 1) / NT); }
unsigned grid_stride(int64_t n) {
    const int64_t g = (n + NT - 1) / NT;
    return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_stokes_div_fine(int n, const double* u, double* q, hipStream_t st) {
    if (!u || !q || n < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_div_fine, dim3(grid_for(N)), dim3(NT), 0, st, n, u, q);
    return hipGetLastError();
}
hipError_t launch_stokes_grad_fine_add(int n, const double* pf, double* out, hipStream_t st) {
    if (!pf || !out || n < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_grad_fine_add, dim3(grid_for(N)), dim3(NT), 0, st, n, pf, out);
    return hipGetLastError();
}
hipError_t launch_stokes_mass_fine(int n, const double* nu, double* mf, hipStream_t st) {
    if (!nu || !mf || n < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_mass_fine, dim3(grid_for(N)), dim3(NT), 0, st, n, nu, mf);
    return hipGetLastError();
}
hipError_t launch_restrict_all(int n_coarse, const double* qf, double* out, hipStream_t st) {
    if (!qf || !out || n_coarse < 1) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n_coarse + 1) * (n_coarse + 1) * (n_coarse + 1);
    hipLaunchKernelGGL(k_restrict_all, dim3(grid_for(N)), dim3(NT), 0, st, n_coarse, qf, out);
    return hipGetLastError();
}
hipError_t launch_prolong_all(int n_fine, const double* pc, double* pf, hipStream_t st) {
    if (!pc || !pf || n_fine < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n_fine + 1) * (n_fine + 1) * (n_fine + 1);
    hipLaunchKernelGGL(k_prolong_all<false>, dim3(grid_for(N)), dim3(NT), 0, st, n_fine, pc, pf);
    return hipGetLastError();
}
hipError_t launch_prolong_all_add(int n_fine, const double* pc, double* pf, hipStream_t st) {
    if (!pc || !pf || n_fine < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n_fine + 1) * (n_fine + 1) * (n_fine + 1);
    hipLaunchKernelGGL(k_prolong_all<true>, dim3(grid_for(N)), dim3(NT), 0, st, n_fine, pc, pf);
    return hipGetLastError();
}
hipError_t launch_div_elementwise(int64_t n, const double* num, const double* den, double* out,
                                  hipStream_t st) {
    if (!num || !den || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_div_elementwise, dim3(grid_stride(n)), dim3(NT), 0, st, n, num, den, out);
    return hipGetLastError();
}

hipError_t launch_mul_elementwise(int64_t n, const double* a, const double* b, double* out,
                                  hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!a || !b || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mul_elementwise, dim3(grid_stride(n)), dim3(NT), 0, st, n, a, b, out);
    return hipGetLastError();
}

hipError_t launch_colour(int n, int colour, int mode, const double* src, double* out, hipStream_t st) {
    if (n < 1 || colour < 0 || colour > 26 || !out || (mode == 1 && !src)) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_colour, dim3(grid_stride(N)), dim3(NT), 0, st, n, colour, mode, src, out);
    return hipGetLastError();
}
int gs_blocks(int64_t n) { return (int)((n + GS_CHUNK - 1) / GS_CHUNK); }
int gs_blocks_f32(int64_t n) { return (int)((n + GS_CHUNK_F32 - 1) / GS_CHUNK_F32); }
template <typename VT>
hipError_t launch_gs_dots(int64_t n, const double* w, const VT* V, int64_t ld, int nv,
                          double* partial, hipStream_t st) {
    if (!w || !V || !partial || n <= 0 || nv < 0) return hipErrorInvalidValue;
    if constexpr (sizeof(VT) == 4) {
        // quad loads: leading dimension a multiple of 4 covering n, 16-byte aligned base
        if ((ld & 3) || ld < n || (reinterpret_cast<uintptr_t>(V) & 15)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_gs_dots_f32, dim3((unsigned)gs_blocks_f32(n)), dim3(NT), 0, st, n, w, V, ld, nv,
                           partial);
    } else {
        hipLaunchKernelGGL(k_gs_dots<VT>, dim3((unsigned)gs_blocks(n)), dim3(NT), 0, st, n, w, V, ld, nv,
                           partial);
    }
    return hipGetLastError();
}
template hipError_t launch_gs_dots<double>(int64_t, const double*, const double*, int64_t, int, double*,
                                           hipStream_t);
template hipError_t launch_gs_dots<float>(int64_t, const double*, const float*, int64_t, int, double*,
                                          hipStream_t);
hipError_t launch_gs_sum(const double* partial, int nb, int rows, double* out, hipStream_t st) {
    if (!partial || !out || nb <= 0 || rows <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gs_sum, dim3((unsigned)rows), dim3(NT), 0, st, partial, nb, out);
    return hipGetLastError();
}
template <typename VT>
hipError_t launch_gs_update(int64_t n, double* w, const VT* V, int64_t ld, int nv, const double* h,
                            hipStream_t st) {
    if (!w || !V || !h || n <= 0 || nv <= 0) return hipErrorInvalidValue;
    if constexpr (sizeof(VT) == 4) {
        if ((ld & 3) || ld < n || (reinterpret_cast<uintptr_t>(V) & 15)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_gs_update_f32, dim3(grid_stride((n + 3) / 4)), dim3(NT), 0, st, n, w, V, ld, nv, h);
    } else {
        hipLaunchKernelGGL(k_gs_update<VT>, dim3(grid_stride(n)), dim3(NT), 0, st, n, w, V, ld, nv, h);
    }
    return hipGetLastError();
}
template hipError_t launch_gs_update<double>(int64_t, double*, const double*, int64_t, int, const double*,
                                             hipStream_t);
template hipError_t launch_gs_update<float>(int64_t, double*, const float*, int64_t, int, const double*,
                                            hipStream_t);
hipError_t launch_scale_to_f32(int64_t n, double a, const double* x, float* y, hipStream_t st) {
    if (!x || !y || n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scale_to_f32, dim3(grid_stride(n)), dim3(NT), 0, st, n, a, x, y);
    return hipGetLastError();
}
hipError_t launch_axpy_dev(int64_t n, const double* coef, double sign, const double* x, double* y,
                           hipStream_t st) {
    if (!coef || !x || !y) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axpy_dev, dim3(grid_stride(n)), dim3(NT), 0, st, n, coef, sign, x, y);
    return hipGetLastError();
}

}  // namespace agca
