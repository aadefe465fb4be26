// The coarse end of the V-cycle (Section 2.1's multigrid cycle on the assembled-stencil
// levels) in one workgroup.
//
// Below 9^3 nodes a level's passes are a few hundred threads of work each, and as
// separate launches every pass costs a kernel's start and drain on the GPU (2-5 µs)
// whatever its size.  Here one workgroup runs the whole down and up sweep of levels
// K..1 plus the level-0 solve with workgroup barriers between the passes: every vector
// of these levels lives in LDS; the stencils and inverse diagonals are read from global
// memory (cache-resident after the first pass), each thread's stencil row with all its
// loads in flight at once.  The per-node arithmetic is the one of the per-launch
// kernels (level_ops.h), pass by pass in the same order, with the same roundings.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kuhn.h"
#include "level_ops.h"

namespace agca {
namespace {

constexpr int CT = 512;

__host__ __device__ constexpr int lvl_n(int j) { return 2 << j; }
__host__ __device__ constexpr int lvl_nodes(int j) { return (lvl_n(j) + 1) * (lvl_n(j) + 1) * (lvl_n(j) + 1); }

// one smoothing or residual pass over all (node, component) pairs of a level; a
// Chebyshev pass reads x_prev in place at its output node
template <int NC, typename T, int MODE>
__device__ __forceinline__ void level_pass(int l, const T* __restrict__ S, const T* u, const T* b,
                                           const T* __restrict__ dinv, T* out, T alpha, T gamma,
                                           T omega) {
    const int n = lvl_n(l), N = lvl_nodes(l);
    for (int i = threadIdx.x; i < NC * N; i += CT) {
        const int c = i / N, p = i - c * N;
        stencil_node<NC, T, MODE, true>(n, p, c, S, u, b, dinv, out, omega, alpha, gamma, out);
    }
}

template <int NC, typename T>
__device__ __forceinline__ void smooth_pass(int l, int8_t mode, const T (&c)[3], const T* S,
                                            const T* u, const T* b, const T* dinv, T* out) {
    if (mode == MODE_CHEB)
        level_pass<NC, T, MODE_CHEB>(l, S, u, b, dinv, out, c[0], c[1], c[2]);
    else
        level_pass<NC, T, MODE_JACOBI>(l, S, u, b, dinv, out, c[0], c[1], c[2]);
}

template <int NC, typename T, int K>
__global__ void __launch_bounds__(CT) k_coarse_cycle(const CoarseCycle<T> a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* const lds = reinterpret_cast<T*>(lds_raw);
    const int tid = threadIdx.x;
    // per level j = 0..K: right-hand side, iterate, second buffer (NC (n+1)^3 each)
    T* bv[K + 1];
    T* xv[K + 1];
    T* yv[K + 1];
    {
        int off = 0;
#pragma unroll
        for (int j = 0; j <= K; ++j) {
            const int len = NC * lvl_nodes(j);
            bv[j] = lds + off;
            xv[j] = lds + off + len;
            yv[j] = lds + off + 2 * len;
            off += 3 * len;
        }
    }
    for (int i = tid; i < NC * lvl_nodes(K); i += CT) bv[K][i] = a.b[i];
    __syncthreads();

    // down: smooth, residual, restrict
    T* cur_of[K + 1];
    T* alt_of[K + 1];
#pragma unroll
    for (int l = K; l >= 1; --l) {
        const T* S = a.sten[l];
        const T* dinv = a.dinv[l];
        const T* b = bv[l];
        T* cur = xv[l];
        T* alt = yv[l];
        const T om0 = a.first_omega[l];
        for (int i = tid; i < NC * lvl_nodes(l); i += CT) cur[i] = a.pre > 0 ? om0 * dinv[i] * b[i] : T(0);
        __syncthreads();
        for (int k = 1; k < a.pre; ++k) {
            smooth_pass<NC, T>(l, a.pre_mode[l][k], a.pre_c[l][k], S, cur, b, dinv, alt);
            __syncthreads();
            T* s = cur;
            cur = alt;
            alt = s;
        }
        level_pass<NC, T, MODE_RESIDUAL>(l, S, cur, b, dinv, alt, T(0), T(0), T(0));
        __syncthreads();
        for (int p = tid; p < lvl_nodes(l - 1); p += CT) restrict_node<NC, T>(lvl_n(l - 1), p, alt, bv[l - 1]);
        __syncthreads();
        cur_of[l] = cur;
        alt_of[l] = alt;
    }
    if (tid < 27 * NC) coarse_solve_slot<T>(NC, tid, a.ainv, bv[0], xv[0]);
    __syncthreads();

    // up: prolongate and add, smooth
    const T* ec = xv[0];
#pragma unroll
    for (int l = 1; l <= K; ++l) {
        const T* S = a.sten[l];
        const T* dinv = a.dinv[l];
        T* cur = cur_of[l];
        T* alt = alt_of[l];
        for (int p = tid; p < lvl_nodes(l); p += CT) prolong_add_node<NC, T>(lvl_n(l), p, ec, cur);
        __syncthreads();
        for (int k = 0; k < a.post; ++k) {
            smooth_pass<NC, T>(l, a.post_mode[l][k], a.post_c[l][k], S, cur, bv[l], dinv, alt);
            __syncthreads();
            T* s = cur;
            cur = alt;
            alt = s;
        }
        ec = cur;
    }
    for (int i = tid; i < NC * lvl_nodes(K); i += CT) a.x[i] = ec[i];
}

template <int NC, typename T>
hipError_t launch_k(int K, const CoarseCycle<T>& a, size_t lds, hipStream_t st) {
    switch (K) {
        case 1: hipLaunchKernelGGL((k_coarse_cycle<NC, T, 1>), dim3(1), dim3(CT), lds, st, a); break;
        case 2: hipLaunchKernelGGL((k_coarse_cycle<NC, T, 2>), dim3(1), dim3(CT), lds, st, a); break;
        case 3: hipLaunchKernelGGL((k_coarse_cycle<NC, T, 3>), dim3(1), dim3(CT), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

size_t coarse_cycle_lds(int ncomp, int K, size_t elem) {
    size_t v = 0;
    for (int j = 0; j <= K; ++j) v += 3 * (size_t)ncomp * lvl_nodes(j);
    return v * elem;
}

template <typename T>
hipError_t launch_coarse_cycle(int ncomp, int K, const CoarseCycle<T>& a, hipStream_t st) {
    if ((ncomp != 1 && ncomp != 3) || K < 1 || K > kCycleLevels) return hipErrorInvalidValue;
    if (a.pre < 0 || a.post < 0 || a.pre > kCyclePasses || a.post > kCyclePasses) return hipErrorInvalidValue;
    if (!a.ainv || !a.b || !a.x) return hipErrorInvalidValue;
    for (int l = 1; l <= K; ++l)
        if (!a.sten[l] || !a.dinv[l]) return hipErrorInvalidValue;
    const size_t lds = coarse_cycle_lds(ncomp, K, sizeof(T));
    if (lds > 65536) return hipErrorInvalidValue;
    return ncomp == 1 ? launch_k<1, T>(K, a, lds, st) : launch_k<3, T>(K, a, lds, st);
}

template hipError_t launch_coarse_cycle<double>(int, int, const CoarseCycle<double>&, hipStream_t);
template hipError_t launch_coarse_cycle<float>(int, int, const CoarseCycle<float>&, hipStream_t);

}  // namespace agca
