// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "agca.h"

namespace agca {

// Operator data of one level as seen by the element-loop kernels, in one precision.
template <typename T>
struct LevelOp {
    int n = 0;                 // cells per axis
    const void* nu = nullptr;  // 6 n^3 coefficients, internal layout (T, or uint16 bf16 bits)
    int nu_kind = 0;           // AGCA_F64 / AGCA_F32 / AGCA_BF16 storage of nu
    const int32_t* blk = nullptr;  // per element (internal layout): stored block index or -1
    const int32_t* ids = nullptr;  // sorted ids of the flagged elements
    int64_t nflag = 0;
    const T* blocks = nullptr;     // flagged x (4 ncomp)^2 entries
    T* yblk = nullptr;             // scratch: flagged x 4 ncomp products B u_e
    const T* dinv = nullptr;       // inverse Jacobi diagonal, level vector (0 on the boundary)
    const T* sten = nullptr;       // assembled stencil (k_stencil.hip layout) or null
};

// MODE_JACOBI0: two passes from a zero guess: the input x = omega0 D^-1 b is formed on
//               the fly (u unused; element loop only)
// MODE_CHEB:    a Chebyshev step, reads x_prev at each output node
enum CubeMode { MODE_APPLY = 0, MODE_RESIDUAL = 1, MODE_JACOBI = 2, MODE_APPLY_DOT = 3,
                MODE_JACOBI0 = 4, MODE_CHEB = 5 };

// Coefficients of a smoothing pass: x_out = alpha x + gamma x_prev + omega D^-1 (b - A x)
// (damped Jacobi: alpha = 1, gamma = 0); omega0 scales the first pass of MODE_JACOBI0.
template <typename T>
struct Sweep {
    T omega = T(0), alpha = T(1), gamma = T(0), omega0 = T(0);
    const T* xprev = nullptr;
};
template <typename T>
inline Sweep<T> jacobi_sweep(T omega) {
    Sweep<T> s;
    s.omega = omega;
    s.omega0 = omega;
    return s;
}

// v = A u / r = b - A u / x_out as above   (one element-loop pass)
template <typename T>
hipError_t launch_cube(int ncomp, int mode, const LevelOp<T>& op, const T* u, const T* b, T* out,
                       const Sweep<T>& sw, hipStream_t st);
// v = A u and per-workgroup partial sums of u . v (FP64 only); *nblocks receives the count
hipError_t launch_cube_dot(int ncomp, const LevelOp<double>& op, const double* u, double* out,
                           double* partial, int* nblocks, hipStream_t st);
// upper bound on the workgroups of the element loop on a level with n cells
int cube_grid_blocks(int n);

// assembled 15-point stencil of a coarse level (FP64): DCA on unflagged simplices,
// stored blocks (blk in the internal element layout) on flagged ones
hipError_t launch_stencil_assemble(int ncomp, int n, const double* nu, double scale,
                                   const int32_t* blk, const double* blocks, double* S,
                                   hipStream_t st);
// apply / residual / Jacobi-type passes (MODE_APPLY, MODE_RESIDUAL, MODE_JACOBI, MODE_CHEB)
// with an assembled stencil
template <typename T>
hipError_t launch_stencil(int ncomp, int mode, int n, const T* S, const T* u, const T* b,
                          const T* dinv, T* out, const Sweep<T>& sw, hipStream_t st);

// transfers (Section 2.1)
template <typename T>
hipError_t launch_restrict(int ncomp, int n_fine, const T* rf, T* rc, hipStream_t st);
template <typename T>
hipError_t launch_prolong_add(int ncomp, int n_fine, const T* ec, T* xf, hipStream_t st);

// level-0 solve: x = A0^-1 b on the single free node (ncomp x ncomp inverse in FP64)
template <typename T>
hipError_t launch_coarse_solve(int ncomp, const double* ainv, const T* b, T* x, hipStream_t st);

// The coarse end of a V-cycle in one workgroup (k_coarse_cycle.hip): levels K..1 (all
// assembled-stencil levels, level l with n = 2^(l+1) cells) and the level-0 solve, from
// the level-K right-hand side b to the level-K iterate x, with every intermediate vector
// in LDS.  Smoothing passes as in the per-launch V-cycle: pre-smoothing pass 0 is x = first_omega D^-1 b from zero (0 when
// pre = 0), pre passes 1.. and post passes 0.. write
// x_out = alpha x + gamma x_prev + omega D^-1 (b - A x) with the mode and coefficients
// given per level and pass (MODE_JACOBI ignores gamma).
constexpr int kCycleLevels = 3;  // K <= 3
constexpr int kCyclePasses = 8;  // pre, post <= 8
template <typename T>
struct CoarseCycle {
    int pre = 0, post = 0;
    const T* sten[kCycleLevels + 1] = {};
    const T* dinv[kCycleLevels + 1] = {};
    T first_omega[kCycleLevels + 1] = {};
    int8_t pre_mode[kCycleLevels + 1][kCyclePasses] = {};
    int8_t post_mode[kCycleLevels + 1][kCyclePasses] = {};
    T pre_c[kCycleLevels + 1][kCyclePasses][3] = {};   // alpha, gamma, omega
    T post_c[kCycleLevels + 1][kCyclePasses][3] = {};
    const double* ainv = nullptr;  // level-0 inverse, ncomp x ncomp
    const T* b = nullptr;          // level K, ncomp (n+1)^3 values (device)
    T* x = nullptr;                // level K, written
};
// LDS bytes of the fused cycle over levels 0..K
size_t coarse_cycle_lds(int ncomp, int K, size_t elem);
template <typename T>
hipError_t launch_coarse_cycle(int ncomp, int K, const CoarseCycle<T>& a, hipStream_t st);

// vector kernels
template <typename T>
hipError_t launch_dot_partial(const T* x, const T* y, int64_t n, double* partial, int nblocks,
                              hipStream_t st);
hipError_t launch_sum_partials(const double* partial, int nblocks, double* out, hipStream_t st);
template <typename T>
hipError_t launch_axpby(int64_t n, double a, const T* x, double b, T* y, hipStream_t st);  // y = a x + b y
// CG update: x += alpha p, r -= alpha q with alpha = rz[0] / pq[0] on the device (and r32 =
// FP32 copy of the new r if r32 != null), and partial sums of r . r over nblocks workgroups
hipError_t launch_cg_update(int64_t n, const double* rz, const double* pq, const double* p,
                            const double* q, double* x, double* r, float* r32, double* partial,
                            int nblocks, hipStream_t st);
// p = z + beta p with beta = sign num[0] / den[0] on the device
template <typename Z>
hipError_t launch_zpbp_dev(int64_t n, const Z* z, const double* num, const double* den, double sign,
                           double* p, hipStream_t st);
// partial sums of z . r and z . q (two arrays of nblocks; the second only if q != null)
template <typename Z>
hipError_t launch_dot2(int64_t n, const Z* z, const double* r, const double* q, double* partial,
                       int nblocks, hipStream_t st);
// p = z + beta p (beta = 0 overwrites p without reading it)
template <typename Z>
hipError_t launch_zpbp(int64_t n, const Z* z, double beta, double* p, hipStream_t st);
hipError_t launch_cast(int from, int to, const void* src, void* dst, int64_t n, hipStream_t st);
// Lanczos step with device coefficients: w = y / d - alpha[0] v - sqrt(beta2[0]) u (no u
// term when u is null), partial sums of w . (d w) over nblocks workgroups
hipError_t launch_lanczos_step(int64_t n, const double* y, const double* d, const double* v,
                               const double* u, const double* alpha, const double* beta2, double* w,
                               double* partial, int nblocks, hipStream_t st);
// out = x / sqrt(s[0]) (s on the device)
hipError_t launch_scale_rsqrt(int64_t n, const double* x, const double* s, double* out, hipStream_t st);
template <typename T>
hipError_t launch_zero_boundary(int ncomp, int n, T* x, hipStream_t st);
template <typename T>
hipError_t launch_first_sweep(int64_t n, T omega, const T* dinv, const T* b, T* x, hipStream_t st);
template <typename T>
hipError_t launch_fill(int64_t n, T value, T* x, hipStream_t st);
hipError_t launch_count_invalid(const double* v, int64_t n, int* counter, hipStream_t st);
// (-1)^(x+y+z) on interior nodes, 0 on the boundary; out = a * b; out = d > 0 ? y / d : 0
hipError_t launch_alternating(int ncomp, int n, double* x, hipStream_t st);
hipError_t launch_mul(int64_t n, const double* a, const double* b, double* out, hipStream_t st);
hipError_t launch_div_or_zero(int64_t n, const double* y, const double* d, double* out,
                              hipStream_t st);
// element-id order (e = s + 6 cell) -> internal per-element layout (kuhn.h elem_slot)
// (exponentiate: the input holds log nu)
hipError_t launch_to_internal(int64_t cells, const double* by_id, double* internal, bool exponentiate,
                              hipStream_t st);

// setup kernels (Sections 2.2-2.3)
hipError_t launch_minmax_from_fine(int n_coarse, const double* nu_fine, double* mn, double* mx,
                                   hipStream_t st);
hipError_t launch_minmax_up(int n_coarse, const double* mn_f, const double* mx_f, double* mn,
                            double* mx, hipStream_t st);
hipError_t launch_flag(int64_t ne, const double* mn, const double* mx, double tau, int mode,
                       int32_t* flag, hipStream_t st);
// descendant means of the finest coefficient (canonical ids), and their use as the DCA
// coefficient of the flagged elements (nu in the internal layout)
hipError_t launch_mean_from_fine(int n_coarse, const double* nu_fine, double* mean, hipStream_t st);
hipError_t launch_mean_up(int n_coarse, const double* mean_f, double* mean, hipStream_t st);
hipError_t launch_override_mean(int64_t ne, const int32_t* flag, const double* mean, double* nu,
                                hipStream_t st);
// flag = 1 for the level-l elements (n = 2^(l+1) cells per axis) inside the macro
// elements whose bit is set in `bits` (bit k = level-0 element id k)
hipError_t launch_flag_macro(int64_t ne, int n, int l, uint64_t bits, int32_t* flag, hipStream_t st);
// per macro element the largest |grad eta_h| over the finest elements of level L, as the
// bit patterns of non-negative doubles, max-combined into gbits[48] (zeroed by the caller)
hipError_t launch_macro_grad_max(int L, const double* eta, unsigned long long* gbits, hipStream_t st);
// exclusive scan of flags -> blk index (or -1) and total count (device int64)
hipError_t launch_compact(int64_t ne, const int32_t* flag, int32_t* blk, int32_t* blk_soa,
                          int32_t* ids, int64_t* count_dev, void* scratch, size_t scratch_bytes,
                          hipStream_t st);
hipError_t compact_scratch_bytes(int64_t ne, size_t* bytes);

// Galerkin blocks (eq. (2.7)), FP64.
// fused: for every element of level l = L-2 (n cells), from the finest coefficient on
// level L (4n cells): forms the blocks of its children (level L-1) and its own;
// stores flagged ones and optionally writes all of level l to trans_out.
hipError_t launch_gca_fused2(int ncomp, int n, const double* nu_fine, double h_fine,
                             const int32_t* blk_child, double* blocks_child,
                             const int32_t* blk_self, double* blocks_self, double* trans_out,
                             hipStream_t st);
// flagged elements of level L-1 only (n cells), from the finest level
hipError_t launch_gca_from_fine(int ncomp, int n, int64_t nflag, const int32_t* ids,
                                const double* nu_fine, double h_fine, double* blocks,
                                hipStream_t st);
// level l (n cells) from the transient blocks of level l+1
hipError_t launch_gca_up(int ncomp, int n, const double* trans_in, const int32_t* blk_self,
                         double* blocks_self, double* trans_out, hipStream_t st);

// diagonal of a level operator (FP64): D = sum of element diagonals (DCA or stored block)
hipError_t launch_diagonal(int ncomp, int n, const double* nu, double scale, const int32_t* blk,
                           const double* blocks, double* diag, hipStream_t st);
template <typename T>
hipError_t launch_invert_diag(int64_t count, const double* diag, T* dinv, hipStream_t st);

// Stokes pieces (k_stokes.hip): velocity on the level with n cells, pressure on n/2
hipError_t launch_stokes_div_fine(int n, const double* u, double* q, hipStream_t st);
// classical Gram-Schmidt against nv basis vectors V + i ld: gs_blocks(n) workgroups write
// (nv + 1) rows of partials (w . V_i, then w . w); gs_sum reduces `rows` rows to out;
// gs_update does w -= sum_i h[i] V_i with h on the device; the basis V is FP64 or FP32
// (widened on the fly); scale_to_f32 writes y = a x rounded to FP32
int gs_blocks(int64_t n);
int gs_blocks_f32(int64_t n);  // the dot pass over an FP32 basis (twice the entries per workgroup)
template <typename VT>
hipError_t launch_gs_dots(int64_t n, const double* w, const VT* V, int64_t ld, int nv,
                          double* partial, hipStream_t st);
hipError_t launch_gs_sum(const double* partial, int nb, int rows, double* out, hipStream_t st);
template <typename VT>
hipError_t launch_gs_update(int64_t n, double* w, const VT* V, int64_t ld, int nv, const double* h,
                            hipStream_t st);
hipError_t launch_scale_to_f32(int64_t n, double a, const double* x, float* y, hipStream_t st);
hipError_t launch_stokes_grad_fine_add(int n, const double* pf, double* out, hipStream_t st);
hipError_t launch_stokes_mass_fine(int n, const double* nu, double* mf, hipStream_t st);
hipError_t launch_restrict_all(int n_coarse, const double* qf, double* out, hipStream_t st);
hipError_t launch_prolong_all(int n_fine, const double* pc, double* pf, hipStream_t st);
hipError_t launch_prolong_all_add(int n_fine, const double* pc, double* pf, hipStream_t st);
// BFBT pressure multigrid (k_zmg.hip): mode 0 out = S x, 1 out = r - S x, 2 out = x + omega
// (r - S x) / S_c with S the stored half of a symmetric 65-offset stencil (zstencil.h); x
// and out distinct
hipError_t launch_zstencil(int mode, int n, const double* S, const double* x, const double* r,
                           double omega, double* out, hipStream_t st);
hipError_t launch_zjacobi0(int n, const double* S, const double* r, double omega, double* out,
                           hipStream_t st);
hipError_t launch_zprobe(int n, int colour, double* out, hipStream_t st);
hipError_t launch_zextract(int n, int colour, const double* y, double* S, hipStream_t st);
hipError_t launch_zcoarse(const double* M, const double* r, double* y, hipStream_t st);
hipError_t launch_zexpand(int n, const double* S, double* out, hipStream_t st);
hipError_t launch_mul_elementwise(int64_t n, const double* a, const double* b, double* out,
                                  hipStream_t st);
// 27-colouring of a level's nodes by (x mod 3, y mod 3, z mod 3): mode 0 writes the
// colour's indicator, mode 1 copies src into out on the colour's nodes only
hipError_t launch_colour(int n, int colour, int mode, const double* src, double* out, hipStream_t st);
hipError_t launch_div_elementwise(int64_t n, const double* num, const double* den, double* out,
                                  hipStream_t st);
hipError_t launch_axpy_dev(int64_t n, const double* coef, double sign, const double* x, double* y,
                           hipStream_t st);

// adjoint gradient and load vector (finest level)
// rounding-floor terms of the residual: partial[0..nblocks) = sums of (|b_i| + (sum_e |A_e||x_e|)_i)^2,
// partial[nblocks..2 nblocks) = sums of b_i^2, both over free dofs (finest level, FP64)
hipError_t launch_floor_terms(int ncomp, int n, const double* nu, double scale, const double* b,
                              const double* x, double* partial, int nblocks, hipStream_t st);
// partial sums of x . y over the free dofs of a level vector
template <typename T>
hipError_t launch_interior_dot(int ncomp, int n, const T* x, const T* y, double* partial, int nblocks,
                               hipStream_t st);
hipError_t launch_grad(int ncomp, int n, const double* nu, double scale, const double* u,
                       const double* w, double* g, hipStream_t st);
hipError_t launch_load_vector(int ncomp, int n, const double* f, double vol4, double* b,
                              hipStream_t st);

}  // namespace agca
