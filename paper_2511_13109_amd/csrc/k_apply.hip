// Matrix-free element loop on the refined Kuhn lattice (paper eq. (2.3) on the
// finest level, eq. (2.9) on coarser levels): apply, residual and damped-Jacobi sweep.
//
// Layout of the work: a 16 x 16 workgroup owns a 16 x 16 column of lattice
// cells and marches up through a chunk of z layers.  At every step a thread
// evaluates its cell's 6 simplices once (cube_math.h), producing contributions
// to the cell's 8 corners.  Corner sums are formed without atomics:
//   * x neighbours are lanes of the same 16-lane DPP row -> row_shr:1,
//   * y neighbours go through a small LDS buffer,
//   * the z direction is carried in registers from one step to the next.
// Each node is therefore finalised by exactly one thread; the extra first row
// and column of threads compute the halo cells needed by the tile's first
// nodes (15 x 15 nodes finalised per workgroup).  The u values of the cell
// corners come from a double-buffered LDS tile, so one barrier per z step
// suffices.  Every output node is written once, with coalesced stores.
#include <hip/hip_runtime.h>

#include "cube_math.h"
#include "internal.h"

namespace agca {
namespace {

constexpr int TX = 16;
constexpr int TY = 16;

template <typename T>
__device__ __forceinline__ T shr1_row(T v) {
    // value of the lane one to the left in the same 16-lane row (0 for the row's first lane)
    if constexpr (sizeof(T) == 8) {
        const unsigned long long bits = __double_as_longlong(v);
        int lo = (int)(bits & 0xffffffffull);
        int hi = (int)(bits >> 32);
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xF, 0xF, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xF, 0xF, true);
        return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    } else {
        int b = __float_as_int(v);
        b = __builtin_amdgcn_update_dpp(0, b, 0x111, 0xF, 0xF, true);
        return __int_as_float(b);
    }
}

template <typename T>
__device__ __forceinline__ void load_nu6(const double* __restrict__ p, T (&w)[6], T scale) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 a = q[0], b = q[1], c = q[2];
    w[0] = T(a.x) * scale; w[1] = T(a.y) * scale; w[2] = T(b.x) * scale;
    w[3] = T(b.y) * scale; w[4] = T(c.x) * scale; w[5] = T(c.y) * scale;
}
template <typename T>
__device__ __forceinline__ void load_nu6(const float* __restrict__ p, T (&w)[6], T scale) {
    const float2* q = reinterpret_cast<const float2*>(p);
    const float2 a = q[0], b = q[1], c = q[2];
    w[0] = T(a.x) * scale; w[1] = T(a.y) * scale; w[2] = T(b.x) * scale;
    w[3] = T(b.y) * scale; w[4] = T(c.x) * scale; w[5] = T(c.y) * scale;
}
__device__ __forceinline__ float bf16_to_float(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
template <typename T>
__device__ __forceinline__ void load_nu6(const uint16_t* __restrict__ p, T (&w)[6], T scale) {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
    const uint32_t a = q[0], b = q[1], c = q[2];
    w[0] = T(bf16_to_float(a & 0xffffu)) * scale; w[1] = T(bf16_to_float(a >> 16)) * scale;
    w[2] = T(bf16_to_float(b & 0xffffu)) * scale; w[3] = T(bf16_to_float(b >> 16)) * scale;
    w[4] = T(bf16_to_float(c & 0xffffu)) * scale; w[5] = T(bf16_to_float(c >> 16)) * scale;
}

template <int NC, typename T, typename NT, int MODE, bool BLK>
__global__ void __launch_bounds__(TX * TY)
k_cube(const int n, const int zc, const T* __restrict__ u, const NT* __restrict__ nu,
       const int32_t* __restrict__ blk, const T* __restrict__ blocks, const T* __restrict__ b,
       const T* __restrict__ dinv, T* __restrict__ out, const T scale, const T omega) {
    __shared__ T ubuf[2][NC][TY + 1][TX + 1];
    __shared__ T ybuf[2][NC][2][TY][TX];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int X0 = blockIdx.x * (TX - 1), Y0 = blockIdx.y * (TY - 1), Z0 = blockIdx.z * zc;
    const int cx = X0 - 1 + tx, cy = Y0 - 1 + ty;
    const int64_t n1 = n + 1;
    const int64_t N = n1 * n1 * n1;
    const int zend = min(Z0 + zc - 1, n);

    auto uval = [&](int x, int y, int z, int c) -> T {
        if (x <= 0 || y <= 0 || z <= 0 || x >= n || y >= n || z >= n) return T(0);
        return u[c * N + x + n1 * (y + n1 * (int64_t)z)];
    };
    auto fill = [&](int buf, int z) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            ubuf[buf][c][ty][tx] = uval(cx, cy, z, c);
            if (tx == TX - 1) ubuf[buf][c][ty][TX] = uval(cx + 1, cy, z, c);
            if (ty == TY - 1) ubuf[buf][c][TY][tx] = uval(cx, cy + 1, z, c);
            if (tx == TX - 1 && ty == TY - 1) ubuf[buf][c][TY][TX] = uval(cx + 1, cy + 1, z, c);
        }
    };

    fill((Z0 + 1) & 1, Z0 - 1);
    fill(Z0 & 1, Z0);
    __syncthreads();
    T Ulo[4][NC];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) Ulo[k][c] = ubuf[(Z0 + 1) & 1][c][ty + (k >> 1)][tx + (k & 1)];
    __syncthreads();

    T carry[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) carry[c] = T(0);

    const bool col_ok = cx >= 0 && cx < n && cy >= 0 && cy < n;
    const bool writer = tx >= 1 && ty >= 1 && cx <= n && cy <= n;
    const bool xin = cx > 0 && cx < n && cy > 0 && cy < n;

    for (int z = Z0 - 1; z <= zend; ++z) {
        const int cur = (z + 1) & 1;  // buffer holding layer z+1
        T U[8][NC];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                U[k][c] = Ulo[k][c];
                U[k + 4][c] = ubuf[cur][c][ty + (k >> 1)][tx + (k & 1)];
            }
        // next layer's values, written after this step's compute
        T nxt[NC], nxt_x[NC], nxt_y[NC], nxt_xy[NC];
        const bool need_next = z + 2 <= zend + 1;
        if (need_next) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                nxt[c] = uval(cx, cy, z + 2, c);
                if (tx == TX - 1) nxt_x[c] = uval(cx + 1, cy, z + 2, c);
                if (ty == TY - 1) nxt_y[c] = uval(cx, cy + 1, z + 2, c);
                if (tx == TX - 1 && ty == TY - 1) nxt_xy[c] = uval(cx + 1, cy + 1, z + 2, c);
            }
        }

        T F[8][NC];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) F[k][c] = T(0);
        if (col_ok && z >= 0 && z < n) {
            const int64_t cell = cx + (int64_t)n * (cy + (int64_t)n * z);
            T w[6];
            load_nu6(nu + 6 * cell, w, scale);
            if constexpr (BLK) {
                int32_t bi[6];
#pragma unroll
                for (int s = 0; s < 6; ++s) bi[s] = blk[6 * cell + s];
                cell_mixed<NC, T, T>(U, w, bi, blocks, F);
            } else {
                cell_dca<NC, T>(U, w, F);
            }
        }

        // x: add the left neighbour's dx=1 corners to my dx=0 corners -> P[dy][dz]
        T P[2][2][NC];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    P[dy][dz][c] = F[2 * dy + 4 * dz][c] + shr1_row(F[1 + 2 * dy + 4 * dz][c]);

        // y: pass my dy=1 sums up to thread ty+1; stage the next u layer
        const int yb = z & 1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            ybuf[yb][c][0][ty][tx] = P[1][0][c];
            ybuf[yb][c][1][ty][tx] = P[1][1][c];
        }
        if (need_next) {
            const int nb = z & 1;  // buffer of layer z+2 (it held layer z, read one step ago)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                ubuf[nb][c][ty][tx] = nxt[c];
                if (tx == TX - 1) ubuf[nb][c][ty][TX] = nxt_x[c];
                if (ty == TY - 1) ubuf[nb][c][TY][tx] = nxt_y[c];
                if (tx == TX - 1 && ty == TY - 1) ubuf[nb][c][TY][TX] = nxt_xy[c];
            }
        }
        __syncthreads();

        if (writer) {
            T s0[NC], s1[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                s0[c] = P[0][0][c] + ybuf[yb][c][0][ty - 1][tx];
                s1[c] = P[0][1][c] + ybuf[yb][c][1][ty - 1][tx];
            }
            if (z >= Z0) {
                const int64_t p = cx + n1 * (cy + n1 * (int64_t)z);
                const bool interior = xin && z > 0 && z < n;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const T av = carry[c] + s0[c];
                    T o;
                    if constexpr (MODE == MODE_APPLY) {
                        o = av;
                    } else if constexpr (MODE == MODE_RESIDUAL) {
                        o = interior ? b[c * N + p] - av : T(0);
                    } else {
                        o = interior ? Ulo[0][c] + omega * dinv[c * N + p] * (b[c * N + p] - av)
                                     : T(0);
                    }
                    out[c * N + p] = interior ? o : T(0);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) carry[c] = s1[c];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) Ulo[k][c] = U[k + 4][c];
    }
}

int pick_zc(int n) {
    const int g = (n + 1 + TX - 2) / (TX - 1);
    const int cols = g * g;
    int zc = 64;
    while (zc > 4 && (int64_t)cols * ((n + 1 + zc - 1) / zc) < 2048) zc /= 2;
    return zc;
}

template <int NC, typename T, typename NT, int MODE, bool BLK>
hipError_t launch_t(const LevelOp<T>& op, const T* u, const T* b, T* out, T omega,
                    hipStream_t st) {
    const int n = op.n;
    const int zc = pick_zc(n);
    dim3 block(TX, TY, 1);
    dim3 grid((n + 1 + TX - 2) / (TX - 1), (n + 1 + TY - 2) / (TY - 1), (n + 1 + zc - 1) / zc);
    const T scale = T(1.0 / (6.0 * n));
    hipLaunchKernelGGL((k_cube<NC, T, NT, MODE, BLK>), grid, block, 0, st, n, zc, u,
                       reinterpret_cast<const NT*>(op.nu), op.blk, op.blocks, b, op.dinv, out,
                       scale, omega);
    return hipGetLastError();
}

template <int NC, typename T, int MODE>
hipError_t dispatch_nu(const LevelOp<T>& op, const T* u, const T* b, T* out, T omega,
                       hipStream_t st) {
    if (!op.nu || !u || !out || op.n < 2) return hipErrorInvalidValue;
    if (MODE != MODE_APPLY && !b) return hipErrorInvalidValue;
    if (MODE == MODE_JACOBI && !op.dinv) return hipErrorInvalidValue;
    if (op.blk && !op.blocks) return hipErrorInvalidValue;
    const bool blk = op.blk != nullptr;
    if constexpr (sizeof(T) == 8) {
        if (op.nu_kind != AGCA_F64) return hipErrorInvalidValue;
        return blk ? launch_t<NC, T, double, MODE, true>(op, u, b, out, omega, st)
                   : launch_t<NC, T, double, MODE, false>(op, u, b, out, omega, st);
    } else {
        if (op.nu_kind == AGCA_F32)
            return blk ? launch_t<NC, T, float, MODE, true>(op, u, b, out, omega, st)
                       : launch_t<NC, T, float, MODE, false>(op, u, b, out, omega, st);
        if (op.nu_kind == AGCA_BF16 && !blk)
            return launch_t<NC, T, uint16_t, MODE, false>(op, u, b, out, omega, st);
        return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t launch_cube(int ncomp, int mode, const LevelOp<T>& op, const T* u, const T* b, T* out,
                       T omega, hipStream_t st) {
    if (ncomp == 1) {
        if (mode == MODE_APPLY) return dispatch_nu<1, T, MODE_APPLY>(op, u, b, out, omega, st);
        if (mode == MODE_RESIDUAL) return dispatch_nu<1, T, MODE_RESIDUAL>(op, u, b, out, omega, st);
        return dispatch_nu<1, T, MODE_JACOBI>(op, u, b, out, omega, st);
    }
    if (mode == MODE_APPLY) return dispatch_nu<3, T, MODE_APPLY>(op, u, b, out, omega, st);
    if (mode == MODE_RESIDUAL) return dispatch_nu<3, T, MODE_RESIDUAL>(op, u, b, out, omega, st);
    return dispatch_nu<3, T, MODE_JACOBI>(op, u, b, out, omega, st);
}

template hipError_t launch_cube<double>(int, int, const LevelOp<double>&, const double*,
                                        const double*, double*, double, hipStream_t);
template hipError_t launch_cube<float>(int, int, const LevelOp<float>&, const float*,
                                       const float*, float*, float, hipStream_t);

}  // namespace agca
