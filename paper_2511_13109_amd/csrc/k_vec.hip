// Grid transfers, level-0 solve, reductions, precision conversions, the adjoint
// gradient and the load vector.
#include <hip/hip_runtime.h>

#include "cube_math.h"
#include "internal.h"
#include "level_ops.h"

namespace agca {
namespace {

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// Transfers (paper Section 2.1).  Linear interpolation between nested P1 spaces
// on the Kuhn lattice: a fine node X = 2Y is a coarse node and copies its value;
// every other fine node is the midpoint of the coarse edge (Y, Y + d) with
// d = X mod 2 in {0,1}^3 (all such offsets are edges of the lattice), so
//   (P e)(X) = (e((X - d)/2) + e((X + d)/2)) / 2.
// Restriction is the transpose: a coarse node Y collects r(2Y) plus half of
// r(2Y + d) and r(2Y - d) for the 7 offsets d.  Boundary nodes stay zero.
// ---------------------------------------------------------------------------
// r_c = P^T r_f at one coarse node per thread, all components (restrict_node)
template <int NC, typename T>
__global__ void __launch_bounds__(NT)
k_restrict(int nc, const T* __restrict__ rf, T* __restrict__ rc) {
    const int64_t nc1 = nc + 1, Nc = nc1 * nc1 * nc1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= Nc) return;
    restrict_node<NC, T>(nc, p, rf, rc);
}

// x_f += P e_c at one fine node per thread, all components (prolong_add_node)
template <int NC, typename T>
__global__ void __launch_bounds__(NT)
k_prolong_add(int nf, const T* __restrict__ ec, T* __restrict__ xf) {
    const int64_t nf1 = nf + 1, Nf = nf1 * nf1 * nf1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= Nf) return;
    prolong_add_node<NC, T>(nf, p, ec, xf);
}

// level 0 has n = 2: a single free node (1,1,1), id 13 of 27
template <typename T>
__global__ void k_coarse_solve(int ncomp, const double* __restrict__ ainv, const T* __restrict__ b,
                               T* __restrict__ x) {
    const int t = threadIdx.x;
    if (t >= 27 * ncomp) return;
    coarse_solve_slot<T>(ncomp, t, ainv, b, x);
}

// ---------------------------------------------------------------------------
// Reductions: fixed-order two-pass sum (wavefront shuffle, then LDS across the
// workgroup's 4 wavefronts, then one workgroup over the partials) so results
// are bitwise reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_dot_partial(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
              double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride)
        acc += (double)x[i] * (double)y[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        partial[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(NT)
k_sum_partials(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) acc += partial[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        *out = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_axpby(int64_t n, double a, const T* __restrict__ x, double b, T* __restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    const T ta = T(a), tb = T(b);
    // b = 0 overwrites y without reading it (y may be uninitialised)
    if (b == 0.0) {
        for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) y[i] = ta * x[i];
    } else {
        for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride)
            y[i] = ta * x[i] + tb * y[i];
    }
}

__device__ __forceinline__ void block_sum_store(double v, double* __restrict__ out) {
    __shared__ double red[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        *out = s;
    }
    __syncthreads();
}

// x += alpha p, r -= alpha q with alpha = rz / pq read from the device, and r . r; with
// r32 the new residual is also stored in FP32 (the input of the FP32 V-cycle)
__global__ void __launch_bounds__(NT)
k_cg_update(int64_t n, const double* __restrict__ rz, const double* __restrict__ pq,
            const double* __restrict__ p, const double* __restrict__ q,
            double* __restrict__ x, double* __restrict__ r, float* __restrict__ r32,
            double* __restrict__ partial) {
    // a direction of zero energy (p = 0) takes no step; the caller tests p . q
    const double alpha = pq[0] != 0.0 ? rz[0] / pq[0] : 0.0;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        x[i] += alpha * p[i];
        const double r1 = r[i] - alpha * q[i];
        r[i] = r1;
        if (r32) r32[i] = (float)r1;
        acc += r1 * r1;
    }
    block_sum_store(acc, partial + blockIdx.x);
}

// z . r and (with q) z . q, z in FP64 or FP32 (the FP32 V-cycle's output, widened)
template <typename Z>
__global__ void __launch_bounds__(NT)
k_dot2(int64_t n, const Z* __restrict__ z, const double* __restrict__ r,
       const double* __restrict__ q, double* __restrict__ partial) {
    double a = 0.0, b = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        const double zi = (double)z[i];
        a += zi * r[i];
        if (q) b += zi * q[i];
    }
    block_sum_store(a, partial + blockIdx.x);
    block_sum_store(b, partial + gridDim.x + blockIdx.x);
}

// p = z + beta p with beta = sign num[0] / den[0] read from the device
template <typename Z>
__global__ void __launch_bounds__(NT)
k_zpbp_dev(int64_t n, const Z* __restrict__ z, const double* __restrict__ num,
           const double* __restrict__ den, double sign, double* __restrict__ p) {
    const double beta = den[0] != 0.0 ? sign * num[0] / den[0] : 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride)
        p[i] = (double)z[i] + beta * p[i];
}

// p = z + beta p (beta = 0: p = z without reading p), z in FP64 or FP32
template <typename Z>
__global__ void __launch_bounds__(NT)
k_zpbp(int64_t n, const Z* __restrict__ z, double beta, double* __restrict__ p) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    if (beta == 0.0) {
        for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) p[i] = (double)z[i];
    } else {
        for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride)
            p[i] = (double)z[i] + beta * p[i];
    }
}

// One Lanczos step for the pencil (A, D) with the coefficients on the device:
// w = y / d - alpha v - beta u (0 where d = 0; beta = sqrt(beta2[0]), no u term when u is
// null), and the partial sums of w . (d w).
__global__ void __launch_bounds__(NT)
k_lanczos_step(int64_t n, const double* __restrict__ y, const double* __restrict__ d,
               const double* __restrict__ v, const double* __restrict__ u,
               const double* __restrict__ alpha, const double* __restrict__ beta2,
               double* __restrict__ w, double* __restrict__ partial) {
    const double a = alpha[0];
    const double b = u ? sqrt(fmax(beta2[0], 0.0)) : 0.0;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        const double dv = d[i];
        double wi = dv > 0.0 ? y[i] / dv : 0.0;
        wi -= a * v[i];
        if (u) wi -= b * u[i];
        w[i] = wi;
        acc += wi * (dv * wi);
    }
    block_sum_store(acc, partial + blockIdx.x);
}

// out = x / sqrt(s[0])
__global__ void __launch_bounds__(NT)
k_scale_rsqrt(int64_t n, const double* __restrict__ x, const double* __restrict__ s,
              double* __restrict__ out) {
    const double r = sqrt(s[0]);
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) out[i] = x[i] / r;
}

// FP64 -> BF16 with a single round-to-nearest-even: round to FP32 with
// "round to odd" (truncate, then set the last bit if inexact), which keeps the
// information a second rounding needs, then round that FP32 value to BF16.
__device__ __forceinline__ uint16_t f64_to_bf16(double x) {
    float f = __double2float_rz(x);
    uint32_t bits = __float_as_uint(f);
    if ((double)f != x) bits |= 1u;
    const uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7fffu + lsb;
    return (uint16_t)(bits >> 16);
}

__global__ void __launch_bounds__(NT)
k_cast(int from, int to, const void* __restrict__ src, void* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        if (from == AGCA_F64 && to == AGCA_F32)
            static_cast<float*>(dst)[i] = (float)static_cast<const double*>(src)[i];
        else if (from == AGCA_F32 && to == AGCA_F64)
            static_cast<double*>(dst)[i] = (double)static_cast<const float*>(src)[i];
        else if (from == AGCA_F64 && to == AGCA_BF16)
            static_cast<uint16_t*>(dst)[i] = f64_to_bf16(static_cast<const double*>(src)[i]);
        else if (from == AGCA_F64 && to == AGCA_F64)
            static_cast<double*>(dst)[i] = static_cast<const double*>(src)[i];
        else if (from == AGCA_F32 && to == AGCA_F32)
            static_cast<float*>(dst)[i] = static_cast<const float*>(src)[i];
    }
}

// first damped-Jacobi sweep from a zero initial guess: x = omega D^-1 b
template <typename T>
__global__ void __launch_bounds__(NT)
k_first_sweep(int64_t n, T omega, const T* __restrict__ dinv, const T* __restrict__ b,
              T* __restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride)
        x[i] = omega * dinv[i] * b[i];
}

template <typename T>
__global__ void __launch_bounds__(NT) k_fill(int64_t n, T value, T* __restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) x[i] = value;
}

// (-1)^(x+y+z) at interior nodes (every component), 0 on the boundary
__global__ void __launch_bounds__(NT) k_alternating(int ncomp, int n, double* __restrict__ x) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int xx, y, z;
    node_coords(p, n, xx, y, z);
    const bool in = xx > 0 && y > 0 && z > 0 && xx < n && y < n && z < n;
    const double v = in ? (((xx + y + z) & 1) ? -1.0 : 1.0) : 0.0;
    for (int c = 0; c < ncomp; ++c) x[c * N + p] = v;
}

__global__ void __launch_bounds__(NT)
k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) out[i] = a[i] * b[i];
}

// out = y / d where d > 0, else 0 (the diagonal is 0 on boundary slots)
__global__ void __launch_bounds__(NT)
k_div_or_zero(int64_t n, const double* __restrict__ y, const double* __restrict__ d,
              double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        const double dv = d[i];
        out[i] = dv > 0.0 ? y[i] / dv : 0.0;
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_zero_boundary(int ncomp, int n, T* __restrict__ x) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int xx, y, z;
    node_coords(p, n, xx, y, z);
    if (xx == 0 || y == 0 || z == 0 || xx == n || y == n || z == n)
        for (int c = 0; c < ncomp; ++c) x[c * N + p] = T(0);
}

__global__ void __launch_bounds__(NT)
k_count_invalid(const double* __restrict__ v, int64_t n, int* __restrict__ counter) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += stride) {
        const double a = v[i];
        if (!(a > 0.0) || !isfinite(a)) ++bad;
    }
    if (bad) atomicAdd(counter, bad);
}

// ---------------------------------------------------------------------------
// Rounding floor of the residual (stopping test of eq. (4.3)).  Replacing every entry of
// x by a value within relative u = 2^-53 of it (one FP64 rounding) moves b - A x by at
// most u (sum_e |A_e| |x_e|) entrywise, and forming b - A x element by element adds
// errors of the same order; per free dof i this kernel forms
//   s_i = |b_i| + (sum_e |A_e| |x_e|)_i
// (|A_e| the entrywise absolute element matrix, nu_e h/6 times the absolute unit matrix)
// and the workgroup's partial sums of s_i^2, and also of b_i^2 over free dofs.  One
// thread per node in a grid-stride loop over a fixed grid: a fixed summation order.
// ---------------------------------------------------------------------------
// vertex index (0..3) of cell corner k on the path of simplex s, -1 if it is not on it
AGCA_HDC constexpr int path_vertex(int s, int k) {
    return path_corner(s, 0) == k ? 0
         : path_corner(s, 1) == k ? 1
         : path_corner(s, 2) == k ? 2
         : path_corner(s, 3) == k ? 3 : -1;
}

template <int NC>
__global__ void __launch_bounds__(NT)
k_floor_terms(int n, const double* __restrict__ nu, double scale, const double* __restrict__ b,
              const double* __restrict__ x, double* __restrict__ partial) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1, cells = (int64_t)n * n * n;
    const int64_t stride = (int64_t)gridDim.x * NT;
    double acc_s = 0.0, acc_b = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < N; p += stride) {
        int px, py, pz;
        node_coords(p, n, px, py, pz);
        if (px == 0 || py == 0 || pz == 0 || px == n || py == n || pz == n) continue;
        // |x| on the 3 x 3 x 3 nodes around p (boundary slots count 0)
        double ax[27][NC];
#pragma unroll
        for (int j = 0; j < 27; ++j) {
            const int qx = px + j % 3 - 1, qy = py + (j / 3) % 3 - 1, qz = pz + j / 9 - 1;
            const bool bd = qx == 0 || qy == 0 || qz == 0 || qx == n || qy == n || qz == n;
            const int64_t q = qx + n1 * (qy + n1 * (int64_t)qz);
#pragma unroll
            for (int c = 0; c < NC; ++c) ax[j][c] = bd ? 0.0 : fabs(x[c * N + q]);
        }
        double s[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) s[c] = 0.0;
        // p is corner k of the cell whose minimum corner is p - offset(k)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
            const int64_t cell = (px - kx) + (int64_t)n * ((py - ky) + (int64_t)n * (pz - kz));
#pragma unroll
            for (int sx = 0; sx < 6; ++sx) {
                const int a = path_vertex(sx, k);
                if (a < 0) continue;
                const double w = nu[elem_slot(sx, cell, cells)] * scale;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int bv = 0; bv < 4; ++bv) {
                        const int m = path_corner(sx, bv);
                        // node of corner m relative to p, in the 3 x 3 x 3 block
                        const int j = ((m & 1) - kx + 1) + 3 * (((m >> 1) & 1) - ky + 1) +
                                      9 * ((m >> 2) - kz + 1);
#pragma unroll
                        for (int d = 0; d < NC; ++d) {
                            const int e = elem_entry(NC, sx, c, a, d, bv);
                            t += (double)(e < 0 ? -e : e) * ax[j][d];
                        }
                    }
                    s[c] = fma(w, t, s[c]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double bi = b[c * N + p];
            const double si = fabs(bi) + s[c];
            acc_s = fma(si, si, acc_s);
            acc_b = fma(bi, bi, acc_b);
        }
    }
    block_sum_store(acc_s, partial + blockIdx.x);
    block_sum_store(acc_b, partial + gridDim.x + blockIdx.x);
}

// partial sums of x . y over the free dofs only (boundary slots are not part of a vector)
template <typename T>
__global__ void __launch_bounds__(NT)
k_interior_dot(int ncomp, int n, const T* __restrict__ x, const T* __restrict__ y,
               double* __restrict__ partial) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int64_t stride = (int64_t)gridDim.x * NT;
    double acc = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < N; p += stride) {
        int px, py, pz;
        node_coords(p, n, px, py, pz);
        if (px == 0 || py == 0 || pz == 0 || px == n || py == n || pz == n) continue;
        for (int c = 0; c < ncomp; ++c) acc += (double)x[c * N + p] * (double)y[c * N + p];
    }
    block_sum_store(acc, partial + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Adjoint gradient g_e = -w_e^T A_e u_e = -(nu_e h/6) * energy(u_e, w_e), one
// thread per cell (6 simplices, 6 consecutive outputs).
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(NT)
k_grad(int n, const double* __restrict__ nu, double scale, const double* __restrict__ u,
       const double* __restrict__ w, double* __restrict__ g) {
    const int64_t cells = (int64_t)n * n * n;
    const int64_t cell = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (cell >= cells) return;
    const int cx = (int)(cell % n), cy = (int)((cell / n) % n), cz = (int)(cell / ((int64_t)n * n));
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    double U[8][NC], W[8][NC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int x = cx + (k & 1), y = cy + ((k >> 1) & 1), z = cz + ((k >> 2) & 1);
        const bool bd = x == 0 || y == 0 || z == 0 || x == n || y == n || z == n;
        const int64_t p = x + n1 * (y + n1 * (int64_t)z);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            U[k][c] = bd ? 0.0 : u[c * N + p];
            W[k][c] = bd ? 0.0 : w[c * N + p];
        }
    }
    double e[6];
    cell_energy<NC, double>(U, W, e);
#pragma unroll
    for (int s = 0; s < 6; ++s) g[6 * cell + s] = -nu[elem_slot(s, cell, cells)] * scale * e[s];
}

__global__ void __launch_bounds__(NT)
k_to_internal(int64_t cells, const double* __restrict__ by_id, double* __restrict__ internal,
              int exponentiate) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < 6 * cells; i += stride) {
        const double v = by_id[i];
        internal[elem_index(i, cells)] = exponentiate ? exp(v) : v;
    }
}

// b_i = sum over the simplices containing node i of f_e |e| / 4 (per component)
template <int NC>
__global__ void __launch_bounds__(NT)
k_load_vector(int n, const double* __restrict__ f, double vol4, double* __restrict__ b) {
    const int64_t n1 = n + 1, N = n1 * n1 * n1, E = 6LL * n * n * n;
    const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
    if (p >= N) return;
    int x, y, z;
    node_coords(p, n, x, y, z);
    const bool bd = x == 0 || y == 0 || z == 0 || x == n || y == n || z == n;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (!bd) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int cx = x - (k & 1), cy = y - ((k >> 1) & 1), cz = z - ((k >> 2) & 1);
            const int64_t cell = cx + (int64_t)n * (cy + (int64_t)n * cz);
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const bool on = k == 0 || k == 7 || k == path_corner(s, 1) || k == path_corner(s, 2);
                if (on)
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[c] += f[c * E + 6 * cell + s];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) b[c * N + p] = acc[c] * vol4;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + NT - 1) / NT); }
inline unsigned grid_stride(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    return (unsigned)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

}  // namespace

template <typename T>
hipError_t launch_restrict(int ncomp, int n_fine, const T* rf, T* rc, hipStream_t st) {
    if (!rf || !rc || n_fine < 4) return hipErrorInvalidValue;
    const int nc = n_fine / 2;
    const int64_t Nc = (int64_t)(nc + 1) * (nc + 1) * (nc + 1);
    if (ncomp == 1)
        hipLaunchKernelGGL((k_restrict<1, T>), dim3(grid_for(Nc)), dim3(NT), 0, st, nc, rf, rc);
    else
        hipLaunchKernelGGL((k_restrict<3, T>), dim3(grid_for(Nc)), dim3(NT), 0, st, nc, rf, rc);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_prolong_add(int ncomp, int n_fine, const T* ec, T* xf, hipStream_t st) {
    if (!ec || !xf || n_fine < 4) return hipErrorInvalidValue;
    const int64_t Nf = (int64_t)(n_fine + 1) * (n_fine + 1) * (n_fine + 1);
    if (ncomp == 1)
        hipLaunchKernelGGL((k_prolong_add<1, T>), dim3(grid_for(Nf)), dim3(NT), 0, st, n_fine, ec, xf);
    else
        hipLaunchKernelGGL((k_prolong_add<3, T>), dim3(grid_for(Nf)), dim3(NT), 0, st, n_fine, ec, xf);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_coarse_solve(int ncomp, const double* ainv, const T* b, T* x, hipStream_t st) {
    if (!ainv || !b || !x) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(128), 0, st, ncomp, ainv, b, x);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_dot_partial(const T* x, const T* y, int64_t n, double* partial, int nblocks,
                              hipStream_t st) {
    if (!x || !y || !partial) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(nblocks), dim3(NT), 0, st, x, y, n, partial);
    return hipGetLastError();
}
hipError_t launch_sum_partials(const double* partial, int nblocks, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(NT), 0, st, partial, nblocks, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_axpby(int64_t n, double a, const T* x, double b, T* y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!x || !y) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axpby<T>, dim3(grid_stride(n)), dim3(NT), 0, st, n, a, x, b, y);
    return hipGetLastError();
}
hipError_t launch_cg_update(int64_t n, const double* rz, const double* pq, const double* p,
                            const double* q, double* x, double* r, float* r32, double* partial,
                            int nblocks, hipStream_t st) {
    if (!rz || !pq || !p || !q || !x || !r || !partial || nblocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_update, dim3(nblocks), dim3(NT), 0, st, n, rz, pq, p, q, x, r, r32, partial);
    return hipGetLastError();
}
template <typename Z>
hipError_t launch_zpbp_dev(int64_t n, const Z* z, const double* num, const double* den, double sign,
                           double* p, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!z || !num || !den || !p) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zpbp_dev<Z>, dim3(grid_stride(n)), dim3(NT), 0, st, n, z, num, den, sign, p);
    return hipGetLastError();
}
template hipError_t launch_zpbp_dev<double>(int64_t, const double*, const double*, const double*, double,
                                            double*, hipStream_t);
template hipError_t launch_zpbp_dev<float>(int64_t, const float*, const double*, const double*, double,
                                           double*, hipStream_t);
template <typename Z>
hipError_t launch_dot2(int64_t n, const Z* z, const double* r, const double* q, double* partial,
                       int nblocks, hipStream_t st) {
    if (!z || !r || !partial || nblocks <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dot2<Z>, dim3(nblocks), dim3(NT), 0, st, n, z, r, q, partial);
    return hipGetLastError();
}
template hipError_t launch_dot2<double>(int64_t, const double*, const double*, const double*, double*,
                                        int, hipStream_t);
template hipError_t launch_dot2<float>(int64_t, const float*, const double*, const double*, double*,
                                       int, hipStream_t);
template <typename Z>
hipError_t launch_zpbp(int64_t n, const Z* z, double beta, double* p, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!z || !p) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zpbp<Z>, dim3(grid_stride(n)), dim3(NT), 0, st, n, z, beta, p);
    return hipGetLastError();
}
template hipError_t launch_zpbp<double>(int64_t, const double*, double, double*, hipStream_t);
template hipError_t launch_zpbp<float>(int64_t, const float*, double, double*, hipStream_t);
hipError_t launch_lanczos_step(int64_t n, const double* y, const double* d, const double* v,
                               const double* u, const double* alpha, const double* beta2, double* w,
                               double* partial, int nblocks, hipStream_t st) {
    if (!y || !d || !v || !alpha || (u && !beta2) || !w || !partial || nblocks <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lanczos_step, dim3(nblocks), dim3(NT), 0, st, n, y, d, v, u, alpha, beta2, w,
                       partial);
    return hipGetLastError();
}
hipError_t launch_scale_rsqrt(int64_t n, const double* x, const double* s, double* out, hipStream_t st) {
    if (!x || !s || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scale_rsqrt, dim3(grid_stride(n)), dim3(NT), 0, st, n, x, s, out);
    return hipGetLastError();
}
hipError_t launch_cast(int from, int to, const void* src, void* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!src || !dst) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cast, dim3(grid_stride(n)), dim3(NT), 0, st, from, to, src, dst, n);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_first_sweep(int64_t n, T omega, const T* dinv, const T* b, T* x, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!dinv || !b || !x) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_first_sweep<T>, dim3(grid_stride(n)), dim3(NT), 0, st, n, omega, dinv, b, x);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(int64_t n, T value, T* x, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!x) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_stride(n)), dim3(NT), 0, st, n, value, x);
    return hipGetLastError();
}
hipError_t launch_alternating(int ncomp, int n, double* x, hipStream_t st) {
    if (!x || n < 2) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_alternating, dim3(grid_for(N)), dim3(NT), 0, st, ncomp, n, x);
    return hipGetLastError();
}
hipError_t launch_mul(int64_t n, const double* a, const double* b, double* out, hipStream_t st) {
    if (!a || !b || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mul, dim3(grid_stride(n)), dim3(NT), 0, st, n, a, b, out);
    return hipGetLastError();
}
hipError_t launch_div_or_zero(int64_t n, const double* y, const double* d, double* out,
                              hipStream_t st) {
    if (!y || !d || !out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_div_or_zero, dim3(grid_stride(n)), dim3(NT), 0, st, n, y, d, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_zero_boundary(int ncomp, int n, T* x, hipStream_t st) {
    if (!x) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_zero_boundary<T>, dim3(grid_for(N)), dim3(NT), 0, st, ncomp, n, x);
    return hipGetLastError();
}
hipError_t launch_count_invalid(const double* v, int64_t n, int* counter, hipStream_t st) {
    if (!v || !counter) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_count_invalid, dim3(grid_stride(n)), dim3(NT), 0, st, v, n, counter);
    return hipGetLastError();
}
hipError_t launch_to_internal(int64_t cells, const double* by_id, double* internal, bool exponentiate,
                              hipStream_t st) {
    if (cells <= 0) return hipSuccess;
    if (!by_id || !internal) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_to_internal, dim3(grid_stride(6 * cells)), dim3(NT), 0, st, cells, by_id,
                       internal, exponentiate ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_floor_terms(int ncomp, int n, const double* nu, double scale, const double* b,
                              const double* x, double* partial, int nblocks, hipStream_t st) {
    if (!nu || !b || !x || !partial || nblocks <= 0 || n < 2) return hipErrorInvalidValue;
    if (ncomp == 1)
        hipLaunchKernelGGL(k_floor_terms<1>, dim3(nblocks), dim3(NT), 0, st, n, nu, scale, b, x, partial);
    else
        hipLaunchKernelGGL(k_floor_terms<3>, dim3(nblocks), dim3(NT), 0, st, n, nu, scale, b, x, partial);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_interior_dot(int ncomp, int n, const T* x, const T* y, double* partial, int nblocks,
                               hipStream_t st) {
    if (!x || !y || !partial || nblocks <= 0 || n < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_interior_dot<T>, dim3(nblocks), dim3(NT), 0, st, ncomp, n, x, y, partial);
    return hipGetLastError();
}
template hipError_t launch_interior_dot<double>(int, int, const double*, const double*, double*, int,
                                                hipStream_t);
template hipError_t launch_interior_dot<float>(int, int, const float*, const float*, double*, int,
                                               hipStream_t);
hipError_t launch_grad(int ncomp, int n, const double* nu, double scale, const double* u,
                       const double* w, double* g, hipStream_t st) {
    if (!nu || !u || !w || !g) return hipErrorInvalidValue;
    const int64_t cells = (int64_t)n * n * n;
    if (ncomp == 1)
        hipLaunchKernelGGL(k_grad<1>, dim3(grid_for(cells)), dim3(NT), 0, st, n, nu, scale, u, w, g);
    else
        hipLaunchKernelGGL(k_grad<3>, dim3(grid_for(cells)), dim3(NT), 0, st, n, nu, scale, u, w, g);
    return hipGetLastError();
}
hipError_t launch_load_vector(int ncomp, int n, const double* f, double vol4, double* b,
                              hipStream_t st) {
    if (!f || !b) return hipErrorInvalidValue;
    const int64_t N = (int64_t)(n + 1) * (n + 1) * (n + 1);
    if (ncomp == 1)
        hipLaunchKernelGGL(k_load_vector<1>, dim3(grid_for(N)), dim3(NT), 0, st, n, f, vol4, b);
    else
        hipLaunchKernelGGL(k_load_vector<3>, dim3(grid_for(N)), dim3(NT), 0, st, n, f, vol4, b);
    return hipGetLastError();
}

#define AGCA_INST(T)                                                                           \
    template hipError_t launch_restrict<T>(int, int, const T*, T*, hipStream_t);               \
    template hipError_t launch_prolong_add<T>(int, int, const T*, T*, hipStream_t);            \
    template hipError_t launch_coarse_solve<T>(int, const double*, const T*, T*, hipStream_t); \
    template hipError_t launch_dot_partial<T>(const T*, const T*, int64_t, double*, int,       \
                                              hipStream_t);                                    \
    template hipError_t launch_axpby<T>(int64_t, double, const T*, double, T*, hipStream_t);   \
    template hipError_t launch_zero_boundary<T>(int, int, T*, hipStream_t);                    \
    template hipError_t launch_first_sweep<T>(int64_t, T, const T*, const T*, T*, hipStream_t);  \
    template hipError_t launch_fill<T>(int64_t, T, T*, hipStream_t);
AGCA_INST(double)
AGCA_INST(float)
#undef AGCA_INST

}  // namespace agca
