// Matrix-free element loop on the refined Kuhn lattice (paper eq. (2.3) on the
// finest level, eq. (2.9) on coarser levels): apply, residual and damped-Jacobi sweep.
// Jacobi-type passes write alpha x + gamma x_prev + omega D^-1 (b - A x): damped Jacobi
// (alpha = 1, gamma = 0) and the steps of the Chebyshev smoother (MODE_CHEB reads x_prev
// at the output node).  MODE_JACOBI0 folds the first pass from a zero guess
// (x = omega0 D^-1 b, formed while loading) into the second, so the first iterate is
// never stored.
//
// Layout of the work: a workgroup of 256 threads owns a TX x TY column of lattice
// cells (32 x 8 by default) and marches up through a chunk of z layers.  At every
// step a thread evaluates its cell's 6 simplices once (cube_math.h), producing
// contributions to the cell's 8 corners.  Corner sums are formed without atomics:
//   * x neighbours are adjacent lanes -> DPP wave_shr:1,
//   * y neighbours go through a small LDS buffer,
//   * the z direction is carried in registers from one step to the next.
// Each node is therefore finalised by exactly one thread; the first row and column
// of threads compute the halo cells needed by the tile's first nodes ((TX-1) x (TY-1)
// nodes finalised per workgroup).  Where a few node columns are left over in x after
// the last full tile (5 of 129), they are covered by tall 8 x 32 strip tiles in the
// same launch instead of a row of mostly idle 32 x 8 tiles.  The u values of the cell corners come from a
// three-layer LDS ring filled a step ahead, so one barrier per z step suffices; the
// global loads of a step are issued before its arithmetic and consumed after it.
// Every output node is written once, with coalesced stores.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "cube_math.h"
#include "internal.h"

namespace agca {
namespace {

// Main tiles: TX x TY cells per workgroup, TX * TY = 256; 32-wide rows read 264-byte
// segments of u per node row (16-wide ones 136 bytes), which measured faster beyond
// 129^3 nodes.  A tile finalises (TX-1) x (TY-1) node columns.
#ifndef AGCA_CUBE_TX
#define AGCA_CUBE_TX 32
#endif
constexpr int TX = AGCA_CUBE_TX;
constexpr int TY = 256 / TX;
constexpr int NTHREADS = 256;
// Strip tiles of SX x SY cells: when the node columns left after the last full main
// tile in x are fewer than SX (129 = 4 x 31 + 5), they go to narrow, tall tiles
// instead of a row of mostly idle main tiles, so fewer workgroups cover the level and
// each marches fewer z steps.  Both shapes have (T+1)(256/T+1) tile nodes, so they
// share one LDS layout.
constexpr int SX = 8;
constexpr int SY = 256 / SX;

// x neighbour exchange: DPP wave_shr:1, the value of the lane one to the left in the
// wavefront (0 for its first lane).  Tile rows are tw consecutive lanes and every
// wavefront starts a row, so the only lanes whose shifted-in value comes from another
// row are the rows' first lanes, the halo column, whose value is never used.
constexpr int kWaveShr1 = 0x138;
template <typename T>
__device__ __forceinline__ T shr1_row(T v) {
    constexpr int ctrl = kWaveShr1;
    if constexpr (sizeof(T) == 8) {
        const unsigned long long bits = __double_as_longlong(v);
        int lo = (int)(bits & 0xffffffffull);
        int hi = (int)(bits >> 32);
        lo = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, true);
        return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    } else {
        int b = __float_as_int(v);
        b = __builtin_amdgcn_update_dpp(0, b, ctrl, 0xF, 0xF, true);
        return __int_as_float(b);
    }
}

__device__ __forceinline__ float bf16_to_float(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// The six coefficients of a cell as loaded (in their storage type), decoded only when
// used: a select or conversion right after a load would make the wavefront wait for
// it at once.  AoS: three 16-byte (FP64), 8-byte (FP32) or 4-byte (BF16) loads.
template <typename NT>
struct RawNu;
template <>
struct RawNu<double> {
    double v[6];
    __device__ __forceinline__ void load(const double* __restrict__ p, int64_t stride) {
        if constexpr (AGCA_ELEM_SOA) {
#pragma unroll
            for (int s = 0; s < 6; ++s) v[s] = p[s * stride];
        } else {
            const double2* q = reinterpret_cast<const double2*>(p);
            const double2 a = q[0], b = q[1], c = q[2];
            v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
        }
    }
    template <typename T>
    __device__ __forceinline__ T get(int s) const { return T(v[s]); }
};
template <>
struct RawNu<float> {
    float v[6];
    __device__ __forceinline__ void load(const float* __restrict__ p, int64_t stride) {
        if constexpr (AGCA_ELEM_SOA) {
#pragma unroll
            for (int s = 0; s < 6; ++s) v[s] = p[s * stride];
        } else {
            const float2* q = reinterpret_cast<const float2*>(p);
            const float2 a = q[0], b = q[1], c = q[2];
            v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
        }
    }
    template <typename T>
    __device__ __forceinline__ T get(int s) const { return T(v[s]); }
};
template <>
struct RawNu<uint16_t> {
    uint32_t w[6];  // bf16 bits in the low half (SoA) or packed pairs in w[0..2] (AoS)
    __device__ __forceinline__ void load(const uint16_t* __restrict__ p, int64_t stride) {
        if constexpr (AGCA_ELEM_SOA) {
#pragma unroll
            for (int s = 0; s < 6; ++s) w[s] = p[s * stride];
        } else {
            const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
            w[0] = q[0]; w[1] = q[1]; w[2] = q[2];
        }
    }
    template <typename T>
    __device__ __forceinline__ T get(int s) const {
        if constexpr (AGCA_ELEM_SOA) return T(bf16_to_float(w[s] & 0xffffu));
        const uint32_t x = w[s >> 1];
        return T(bf16_to_float((s & 1) ? (x >> 16) : (x & 0xffffu)));
    }
};

// Workgroup -> tile mapping.  Consecutive workgroups are dispatched round-robin
// to the 8 XCDs, each with its own L2; remapping the linear id so that every XCD
// receives one contiguous range of tiles (x fastest, then y, then z chunks)
// keeps the halo rows that neighbouring tiles share in the same L2.
// cols tile columns per z chunk, gz chunks (negative: no remapping)
__device__ __forceinline__ int tile_lin(int cols, int gz) {
    const int b = blockIdx.x;
    if (gz <= 0) return b;
    const int total = cols * gz;
    const int q = total >> 3, r = total & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd * q + min(xcd, r) + j;
}

#ifndef AGCA_CUBE_PREFETCH_NODE
#define AGCA_CUBE_PREFETCH_NODE 1
#endif

#ifndef AGCA_CUBE_WAVES_F64V
#define AGCA_CUBE_WAVES_F64V 3
#endif

// occupancy target handed to the register allocator (0: compiler's choice)
template <int NC, typename T>
struct CubeWaves {
    static constexpr int value = (NC == 3 && sizeof(T) == 8) ? AGCA_CUBE_WAVES_F64V : 0;
};
// prefetch the next node's right-hand side and diagonal one step ahead (costs registers;
// off for the FP64 vector kernel, whose occupancy is register-bound)
#ifndef AGCA_CUBE_PREFETCH_NODE_F64V
#define AGCA_CUBE_PREFETCH_NODE_F64V 0
#endif
template <int NC, typename T>
struct CubePrefetchNode {
    static constexpr bool value = (NC == 3 && sizeof(T) == 8) ? AGCA_CUBE_PREFETCH_NODE_F64V
                                                              : AGCA_CUBE_PREFETCH_NODE;
};

// Whether a mode's launches use strip tiles.  The fused first two passes from zero hold
// the inverse diagonal of the prefetched layer as well and are at the register limit
// of 3 wavefronts per SIMD: the runtime tile shape would make them spill, so they keep
// the main tiles only (the shape then folds to a constant).
template <int MODE>
struct CubeStrip {
    // strips need the same number of tile nodes as the main tiles (one LDS layout);
    // a main tile width other than 32 (AGCA_CUBE_TX) turns them off
    static constexpr bool value = MODE != MODE_JACOBI0 && (SX + 1) * (SY + 1) == (TX + 1) * (TY + 1);
};

// One tile of tw x 256/tw cells (tw = TX or SX, uniform over the workgroup) whose first
// finalised node column is (X0, Y0), marching through the z layers Z0 .. Z0 + zc - 1.
// The shape is a runtime value so that both shapes share one body (and one register
// allocation).  ubuf_raw / ybuf_raw: the workgroup's LDS ring of u layers and its
// y-exchange buffer.
template <int NC, typename T, typename NT, int MODE, bool BLK>
__device__ __forceinline__ void cube_tile(T* __restrict__ ubuf_raw, T* __restrict__ ybuf_raw,
                                          double& dot_acc, const int tw, const int X0, const int Y0,
                                          const int Z0,
                                          const int n, const int zc, const T* __restrict__ u,
                                          const NT* __restrict__ nu, const int32_t* __restrict__ blk,
                                          const T* __restrict__ yblk, const T* __restrict__ b,
                                          const T* __restrict__ dinv, T* __restrict__ out,
                                          const T scale, const T omega, const T alpha, const T gamma,
                                          const T omega0, const T* __restrict__ xprev) {
    // node layers of u: layer j lives in buffer (j + 3) % 3, so a step reads two
    // buffers while the third receives the layer two steps ahead
    // (tw+1) x (256/tw+1) nodes per layer and component (297 for either shape), x
    // fastest, plus 64 slots that absorb the second tile store of the wavefronts that
    // have no second entry
    constexpr int UB = (TX + 1) * (TY + 1) + 64;
    auto ubuf = reinterpret_cast<T (*)[NC][UB]>(ubuf_raw);
    // y exchange: [buffer][component][dz][thread]; the thread above is tid - tw
    auto ybuf = reinterpret_cast<T (*)[NC][2][NTHREADS]>(ybuf_raw);
    // launches without strip tiles use a TX x TY block (the hardware supplies tx, ty);
    // the others a flat block of 256, split by the tile shape (tw is a power of two)
    const int tid = threadIdx.x + TX * threadIdx.y;
    const int tx = CubeStrip<MODE>::value ? tid & (tw - 1) : (int)threadIdx.x;
    const int ty = CubeStrip<MODE>::value ? tid >> __builtin_ctz(tw) : (int)threadIdx.y;
    const int cx = X0 - 1 + tx, cy = Y0 - 1 + ty;
    const int64_t n1 = n + 1;
    const int64_t N = n1 * n1 * n1;
    const int64_t layer = n1 * n1;          // nodes per z layer
    const int64_t cells = (int64_t)n * n * n;
    const int64_t clayer = (int64_t)n * n;  // cells per z layer
    const int zend = min(Z0 + zc - 1, n);

    // All loads are unconditional: addresses are clamped into the arrays and values
    // outside the interior are replaced by zero afterwards, so the loop has no
    // divergent branches around memory accesses.
    // u tile (TX+1) x (TY+1) per layer: entry tid for every thread, entry NTHREADS + tid
    // for the first wavefronts.  Every thread issues the second load (the others at a
    // clamped duplicate address, a cache hit) so that no branch surrounds the loads
    // and the prefetched values stay in registers; only the first wavefronts store it.
    const int TW = tw + 1;
    constexpr int TE = (TX + 1) * (TY + 1);  // the same for both shapes
    constexpr int NB = ((TE - NTHREADS + 63) / 64) * 64;  // whole wavefronts
    const int qa = tid;
    const int qb = min(NTHREADS + tid, TE - 1);
    const bool has_b = tid < NB;
    // stores of the second entry are unconditional (a branch would pull its loads
    // into it): lanes without one write a per-lane slot past the tile, never read
    const int qb_store = has_b ? qb : TE + (tid & 63);
    // Tile node q of this thread: offset x + (n+1) y of the clamped node within a z layer.
    int at_a, at_b;
    bool ina, inb;
    auto tile_node = [&](int q, int& at, bool& in_xy) {
        const int x = X0 - 1 + q % TW, y = Y0 - 1 + q / TW;
        in_xy = x > 0 && x < n && y > 0 && y < n;
        const int xc = min(max(x, 0), n), yc = min(max(y, 0), n);
        at = xc + (n + 1) * yc;
    };
    tile_node(qa, at_a, ina);
    tile_node(qb, at_b, inb);
    // The loads of a layer are issued a step before the layer is staged in LDS and are
    // consumed (masked, scaled, written to LDS) only at the end of that step, so that
    // their latency overlaps the step's arithmetic.
    struct TileRaw {
        T a[NC], b[NC];    // u (or, for MODE_JACOBI0, the right-hand side) at entries qa, qb
        T da[NC], db[NC];  // MODE_JACOBI0: inverse diagonal at entries qa, qb
    };
    auto load_tile = [&](int z, TileRaw& t) {
        const int64_t off = (int64_t)min(max(z, 0), n) * layer;
        const T* pv = (MODE == MODE_JACOBI0 ? b : u) + off;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            t.a[c] = pv[c * N + at_a];
            t.b[c] = pv[c * N + at_b];
            if constexpr (MODE == MODE_JACOBI0) {
                t.da[c] = dinv[off + c * N + at_a];
                t.db[c] = dinv[off + c * N + at_b];
            }
        }
    };
    auto store_tile = [&](int buf, int z, const TileRaw& t) {
        const bool zin = z > 0 && z < n;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            T va = t.a[c], vb = t.b[c];
            if constexpr (MODE == MODE_JACOBI0) {  // the first sweep from zero, x1 = omega0 D^-1 b
                va = omega0 * t.da[c] * va;
                vb = omega0 * t.db[c] * vb;
            }
            ubuf[buf][c][qa] = (ina && zin) ? va : T(0);
            ubuf[buf][c][qb_store] = (inb && zin) ? vb : T(0);
        }
    };

    const bool col_ok = cx >= 0 && cx < n && cy >= 0 && cy < n;
    const bool writer = tx >= 1 && ty >= 1 && cx <= n && cy <= n;
    const bool xin = cx > 0 && cx < n && cy > 0 && cy < n;
    constexpr bool IS_JACOBI = MODE == MODE_JACOBI || MODE == MODE_JACOBI0 || MODE == MODE_CHEB;
    constexpr bool NEEDS_B = MODE == MODE_RESIDUAL || IS_JACOBI;
    // cell and node columns of this thread, clamped
    const int64_t cellcol = min(max(cx, 0), n - 1) + (int64_t)n * min(max(cy, 0), n - 1);
    const NT* pnu = nu + elem_slot(0, cellcol, cells);
    const int32_t* pblk = blk ? blk + elem_slot(0, cellcol, cells) : nullptr;
    constexpr int64_t kSlotsPerCell = AGCA_ELEM_SOA ? 1 : 6;  // z-layer stride factor
    const int64_t col = min(max(cx, 0), n) + n1 * min(max(cy, 0), n);

    struct RawCell {
        RawNu<NT> nu;
        int32_t bi[6];
        bool ok;
    };
    auto load_cell = [&](int z, RawCell& r) {
        r.ok = col_ok && z >= 0 && z < n;
        const int64_t off = (int64_t)min(max(z, 0), n - 1) * clayer * kSlotsPerCell;
        r.nu.load(pnu + off, cells);
        if constexpr (BLK) {
#pragma unroll
            for (int s = 0; s < 6; ++s) r.bi[s] = pblk[off + elem_slot(s, 0, cells)];
        }
    };
    auto decode_cell = [&](const RawCell& r, T (&w)[6], int32_t (&bi)[6]) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            w[s] = r.ok ? r.nu.template get<T>(s) * scale : T(0);
            if constexpr (BLK) bi[s] = r.ok ? r.bi[s] : -1;
        }
    };
    auto load_node = [&](int z, T (&bq)[NC], T (&dq)[NC]) {
        if constexpr (NEEDS_B) {
            const bool ok = writer && xin && z > 0 && z < n && z >= Z0 && z <= zend;
            const int64_t p = col + (int64_t)min(max(z, 0), n) * layer;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T bv = b[c * N + p];
                bq[c] = ok ? bv : T(0);
                if constexpr (IS_JACOBI) {
                    const T dv = dinv[c * N + p];
                    dq[c] = ok ? dv : T(0);
                } else {
                    dq[c] = T(0);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) bq[c] = dq[c] = T(0);
        }
    };

    auto bidx = [](int layer) { return (layer + 3) % 3; };
    {
        TileRaw t;
        load_tile(Z0 - 1, t);
        store_tile(bidx(Z0 - 1), Z0 - 1, t);
        load_tile(Z0, t);
        store_tile(bidx(Z0), Z0, t);
    }
    RawCell rc;  // the cell layer of the coming step, loaded a step ahead
    load_cell(Z0 - 1, rc);
    TileRaw nxt;  // the node layer two ahead of the coming step, loaded after the
                  // previous step's barrier and staged at the end of this step
    load_tile(Z0 + 1, nxt);
    T bq[NC], dq[NC];
    load_node(Z0 - 1, bq, dq);
    __syncthreads();

    T carry[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) carry[c] = T(0);

    const int lq = ty * TW + tx;  // this thread's cell corner 0 in a ring layer
    for (int z = Z0 - 1; z <= zend; ++z) {
        const int lo = bidx(z), hi = bidx(z + 1);  // buffers holding layers z and z+1
        T U[8][NC];
        // the cell's corners in the ring: the row pitch is a constant of each shape (a
        // branch that is uniform over the workgroup), so the reads take immediate offsets
        auto gather = [&](auto pitch) {
            constexpr int PW = decltype(pitch)::value;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    U[k][c] = ubuf[lo][c][lq + (k >> 1) * PW + (k & 1)];
                    U[k + 4][c] = ubuf[hi][c][lq + (k >> 1) * PW + (k & 1)];
                }
        };
        if (!CubeStrip<MODE>::value || tw == TX)
            gather(std::integral_constant<int, TX + 1>{});
        else
            gather(std::integral_constant<int, SX + 1>{});
        T w_cur[6];
        int32_t bi_cur[6];
        decode_cell(rc, w_cur, bi_cur);
        T self[NC];  // u at this thread's output node (cell corner 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) self[c] = U[0][c];
        // issue the next step's coefficient loads first so that they overlap this step's work
        RawCell rn;
        load_cell(z + 1 <= zend ? z + 1 : -1, rn);
        // keep the scheduler from sinking these loads towards their uses at the end of
        // the step, which would expose their latency
        __builtin_amdgcn_sched_barrier(0);
        T bq_n[NC], dq_n[NC];
        if constexpr (CubePrefetchNode<NC, T>::value) load_node(z + 1, bq_n, dq_n);

        T F[8][NC];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) F[k][c] = T(0);
        if constexpr (BLK)
            cell_mixed<NC, T>(U, w_cur, bi_cur, yblk, F);
        else
            cell_dca<NC, T>(U, w_cur, F);

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
            ybuf[yb][c][0][tid] = P[1][0][c];
            ybuf[yb][c][1][tid] = P[1][1][c];
        }
        // held layer z-1, read last step; after the last step nothing reads this buffer
        // again, so the store needs no condition (a branch would pull the loads into it)
        store_tile(bidx(z + 2), z + 2, nxt);
        __syncthreads();
        // the layer after next: its loads overlap this step's output phase and the next
        // step's arithmetic (addresses are clamped into the lattice: no condition)
        load_tile(z + 3, nxt);
        __builtin_amdgcn_sched_barrier(0);

        if (writer) {
            T s0[NC], s1[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                s0[c] = P[0][0][c] + ybuf[yb][c][0][tid - tw];
                s1[c] = P[0][1][c] + ybuf[yb][c][1][tid - tw];
            }
            if (z >= Z0) {
                const int64_t p = col + (int64_t)z * layer;
                const bool interior = xin && z > 0 && z < n;
                if constexpr (!CubePrefetchNode<NC, T>::value) load_node(z, bq, dq);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const T av = carry[c] + s0[c];
                    T o;
                    if constexpr (MODE == MODE_APPLY) {
                        o = av;
                    } else if constexpr (MODE == MODE_APPLY_DOT) {
                        o = av;
                        if (interior) dot_acc += (double)self[c] * (double)av;
                    } else if constexpr (MODE == MODE_RESIDUAL) {
                        o = bq[c] - av;
                    } else if constexpr (MODE == MODE_CHEB) {
                        // Chebyshev step: alpha x + gamma x_prev + omega D^-1 (b - A x)
                        const T xp = interior ? xprev[c * N + p] : T(0);
                        o = alpha * self[c] + gamma * xp + omega * dq[c] * (bq[c] - av);
                    } else {
                        o = alpha * self[c] + omega * dq[c] * (bq[c] - av);
                    }
                    out[c * N + p] = interior ? o : T(0);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) carry[c] = s1[c];
        }
        rc = rn;
        if constexpr (CubePrefetchNode<NC, T>::value) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bq[c] = bq_n[c];
                dq[c] = dq_n[c];
            }
        }
    }
}

template <int NC, typename T, typename NT, int MODE, bool BLK>
__global__ void __launch_bounds__(NTHREADS)
__attribute__((amdgpu_waves_per_eu(CubeWaves<NC, T>::value > 0 ? CubeWaves<NC, T>::value : 1)))
k_cube(const int n, const int zc, const int gx, const int gy, const int gs, const int gz,
       const T* __restrict__ u, const NT* __restrict__ nu, const int32_t* __restrict__ blk,
       const T* __restrict__ yblk, const T* __restrict__ b, const T* __restrict__ dinv,
       T* __restrict__ out, const T scale, const T omega, const T alpha, const T gamma,
       const T omega0, const T* __restrict__ xprev, double* __restrict__ partial) {
    constexpr int UB = (TX + 1) * (TY + 1) + 64;
    static_assert(SX * SY == NTHREADS && TX * TY == NTHREADS, "both tile shapes have 256 cells");
    __shared__ T ubuf[3 * NC * UB];
    __shared__ T ybuf[2 * NC * 2 * 256];
    double dot_acc = 0.0;  // MODE_APPLY_DOT: this thread's share of u . (A u)
    // per z chunk: gx x gy main tiles, then gs strip tiles (one column of them in x)
    const int cols = gx * gy + gs;
    const int lin = tile_lin(cols, gz);
    const int bz = lin / cols, c = lin - bz * cols;
    const bool main_tile = !CubeStrip<MODE>::value || c < gx * gy;
    const int tw = main_tile ? TX : SX;
    const int X0 = main_tile ? (c % gx) * (TX - 1) : gx * (TX - 1);
    const int Y0 = main_tile ? (c / gx) * (TY - 1) : (c - gx * gy) * (SY - 1);
    cube_tile<NC, T, NT, MODE, BLK>(ubuf, ybuf, dot_acc, tw, X0, Y0, bz * zc, n, zc, u, nu, blk, yblk, b,
                                    dinv, out, scale, omega, alpha, gamma, omega0, xprev);
    if constexpr (MODE == MODE_APPLY_DOT) {
        // fixed-order workgroup reduction: wavefront shuffle, then the 4 wavefronts
        __shared__ double red[NTHREADS / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dot_acc += __shfl_down(dot_acc, off, 64);
        const int tid = threadIdx.x + TX * threadIdx.y;
        if ((tid & 63) == 0) red[tid >> 6] = dot_acc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < NTHREADS / 64; ++w) sum += red[w];
            partial[blockIdx.x] = sum;
        }
    }
}

// Products y_f = B_f u_e of the stored Galerkin blocks of all flagged simplices of a
// level, one thread per (flagged simplex, block row); the element loop then adds
// y_f to the simplex's corners.  Reads each block once, coalesced by rows.
template <int NC, typename T>
__global__ void __launch_bounds__(256)
k_block_products(const int n, const int64_t nflag, const int32_t* __restrict__ ids,
                 const T* __restrict__ blocks, const T* __restrict__ u, T* __restrict__ y) {
    constexpr int M = 4 * NC;
    const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (t >= nflag * M) return;
    const int64_t f = t / M;
    const int r = (int)(t % M);
    const int64_t e = ids[f];
    const int s = (int)(e % 6);
    int64_t cell = e / 6;
    const int cx = (int)(cell % n);
    cell /= n;
    const int cy = (int)(cell % n);
    const int cz = (int)(cell / n);
    const int64_t n1 = n + 1, N = n1 * n1 * n1;
    const int k1 = 1 << axis1(s), k2 = k1 | (1 << axis2(s));
    const int corner[4] = {0, k1, k2, 7};
    T xv[M];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int k = corner[a];
        const int x = cx + (k & 1), yy = cy + ((k >> 1) & 1), z = cz + ((k >> 2) & 1);
        const bool bd = x == 0 || yy == 0 || z == 0 || x == n || yy == n || z == n;
        const int64_t p = x + n1 * (yy + n1 * (int64_t)z);
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[4 * c + a] = bd ? T(0) : u[c * N + p];
    }
    const T* row = blocks + f * (M * M) + r * M;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < M; ++c) acc += row[c] * xv[c];
    y[t] = acc;
}

// Tile columns of a level with n cells per axis: gx x gy main tiles and gs strip tiles
// (gs = 0 when the node columns left after the last full main tile in x are none or
// more than a strip tile finalises).  AGCA_CUBE_STRIP=0 keeps main tiles only.
struct CubeGrid {
    int gx, gy, gs;
};
CubeGrid cube_grid(int n, bool allow_strip) {
    static const bool strip_env = [] {
        const char* e = getenv("AGCA_CUBE_STRIP");
        return e ? atoi(e) != 0 : true;
    }();
    const bool strip = allow_strip && strip_env;
    const int nodes = n + 1;
    const int full = nodes / (TX - 1), rest = nodes - full * (TX - 1);
    CubeGrid g;
    g.gy = (nodes + TY - 2) / (TY - 1);
    if (strip && full >= 1 && rest >= 1 && rest <= SX - 1) {
        g.gx = full;
        g.gs = (nodes + SY - 2) / (SY - 1);
    } else {
        g.gx = (nodes + TX - 2) / (TX - 1);
        g.gs = 0;
    }
    return g;
}
int tile_columns(int n, bool allow_strip = true) {
    const CubeGrid g = cube_grid(n, allow_strip);
    return g.gx * g.gy + g.gs;
}

// z layers per workgroup.  Chunks of about 16 layers amortise the halo layer each chunk
// recomputes; small levels use shorter chunks to expose more workgroups; when the
// workgroups slightly exceed what the GPU holds at once (slots), the chunks grow
// until they fit, rather than leaving a short second round.
int pick_zc(int n, int slots, bool allow_strip) {
    static const int forced = [] {
        const char* e = getenv("AGCA_CUBE_ZC");
        return e ? atoi(e) : 0;
    }();
    if (forced > 0) return forced;
    const int64_t cols = tile_columns(n, allow_strip);
    auto blocks = [&](int zc) { return cols * ((n + 1 + zc - 1) / zc); };
    int zc = 16;
    while (zc > 2 && blocks(zc) < 512) zc /= 2;
    if (slots > 0 && blocks(zc) > slots && blocks(zc) <= slots + slots / 4)
        while (blocks(zc) > slots && zc < n + 1) ++zc;
    // the shortest chunk that gives the same number of chunks (fewer z steps per
    // workgroup for the same workgroups)
    const int gz = (n + 1 + zc - 1) / zc;
    return (n + 1 + gz - 1) / gz;
}

// workgroups of one kernel that the GPU runs at once (occupancy x compute units)
template <typename K>
int resident_slots(K kernel) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NTHREADS, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

template <int NC, typename T, typename NT, int MODE, bool BLK>
hipError_t launch_t(const LevelOp<T>& op, const T* u, const T* b, T* out, const Sweep<T>& sw,
                    hipStream_t st, double* partial = nullptr, int* nblocks = nullptr) {
    const int n = op.n;
    static const int slots = resident_slots(k_cube<NC, T, NT, MODE, BLK>);
    const int zc = pick_zc(n, slots, CubeStrip<MODE>::value);
    const CubeGrid g = cube_grid(n, CubeStrip<MODE>::value);
    const int gz = (n + 1 + zc - 1) / zc;
    const int nwg = (g.gx * g.gy + g.gs) * gz;
    const dim3 block = CubeStrip<MODE>::value ? dim3(NTHREADS, 1, 1) : dim3(TX, TY, 1);
    dim3 grid((unsigned)nwg, 1, 1);
    const T scale = T(1.0 / (6.0 * n));
    if constexpr (BLK && MODE != MODE_JACOBI0) {
        if (op.nflag > 0) {
            const int64_t threads = op.nflag * 4 * NC;
            hipLaunchKernelGGL((k_block_products<NC, T>), dim3((unsigned)((threads + 255) / 256)),
                               dim3(256), 0, st, n, op.nflag, op.ids, op.blocks, u, op.yblk);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    static const bool xcd_map = [] {
        const char* e = getenv("AGCA_CUBE_XCD");
        return e ? atoi(e) != 0 : true;
    }();
    if (nblocks) *nblocks = nwg;
    hipLaunchKernelGGL((k_cube<NC, T, NT, MODE, BLK>), grid, block, 0, st, n, zc, g.gx, g.gy, g.gs,
                       xcd_map ? gz : -gz, u,
                       reinterpret_cast<const NT*>(op.nu), op.blk, op.yblk, b, op.dinv, out,
                       scale, sw.omega, sw.alpha, sw.gamma, sw.omega0, sw.xprev, partial);
    return hipGetLastError();
}

template <int NC, typename T, int MODE>
hipError_t dispatch_nu(const LevelOp<T>& op, const T* u, const T* b, T* out, const Sweep<T>& sw,
                       hipStream_t st) {
    if (!op.nu || !out || op.n < 2) return hipErrorInvalidValue;
    if (MODE != MODE_JACOBI0 && !u) return hipErrorInvalidValue;
    if (MODE != MODE_APPLY && !b) return hipErrorInvalidValue;
    if ((MODE == MODE_JACOBI || MODE == MODE_JACOBI0 || MODE == MODE_CHEB) && !op.dinv)
        return hipErrorInvalidValue;
    if (MODE == MODE_CHEB && !sw.xprev) return hipErrorInvalidValue;
    if (op.blk && (!op.blocks || !op.ids || !op.yblk || op.nflag <= 0)) return hipErrorInvalidValue;
    // the stored-block products are formed from u before the element loop, which
    // MODE_JACOBI0 never stores
    if (MODE == MODE_JACOBI0 && op.blk) return hipErrorInvalidValue;
    const bool blk = op.blk != nullptr;
    if constexpr (sizeof(T) == 8) {
        if (op.nu_kind != AGCA_F64) return hipErrorInvalidValue;
        if constexpr (MODE != MODE_JACOBI0)
            if (blk) return launch_t<NC, T, double, MODE, true>(op, u, b, out, sw, st);
        return launch_t<NC, T, double, MODE, false>(op, u, b, out, sw, st);
    } else {
        if (op.nu_kind == AGCA_F32) {
            if constexpr (MODE != MODE_JACOBI0)
                if (blk) return launch_t<NC, T, float, MODE, true>(op, u, b, out, sw, st);
            return launch_t<NC, T, float, MODE, false>(op, u, b, out, sw, st);
        }
        if (op.nu_kind == AGCA_BF16 && !blk)
            return launch_t<NC, T, uint16_t, MODE, false>(op, u, b, out, sw, st);
        return hipErrorInvalidValue;
    }
}

}  // namespace

int cube_grid_blocks(int n) {
    // upper bound of any launch's workgroups: main tiles only (at least as many
    // columns as with strips), one z layer per workgroup
    return tile_columns(n, false) * (n + 1);
}

hipError_t launch_cube_dot(int ncomp, const LevelOp<double>& op, const double* u, double* out,
                           double* partial, int* nblocks, hipStream_t st) {
    if (!op.nu || !u || !out || !partial || !nblocks || op.n < 2 || op.nu_kind != AGCA_F64)
        return hipErrorInvalidValue;
    if (op.blk && (!op.blocks || !op.ids || !op.yblk || op.nflag <= 0)) return hipErrorInvalidValue;
    if (ncomp == 1)
        return op.blk ? launch_t<1, double, double, MODE_APPLY_DOT, true>(op, u, nullptr, out, Sweep<double>{}, st,
                                                                           partial, nblocks)
                      : launch_t<1, double, double, MODE_APPLY_DOT, false>(op, u, nullptr, out, Sweep<double>{}, st,
                                                                            partial, nblocks);
    return op.blk ? launch_t<3, double, double, MODE_APPLY_DOT, true>(op, u, nullptr, out, Sweep<double>{}, st,
                                                                       partial, nblocks)
                  : launch_t<3, double, double, MODE_APPLY_DOT, false>(op, u, nullptr, out, Sweep<double>{}, st,
                                                                        partial, nblocks);
}

template <int NC, typename T>
hipError_t launch_cube_nc(int mode, const LevelOp<T>& op, const T* u, const T* b, T* out,
                          const Sweep<T>& sw, hipStream_t st) {
    switch (mode) {
        case MODE_APPLY: return dispatch_nu<NC, T, MODE_APPLY>(op, u, b, out, sw, st);
        case MODE_RESIDUAL: return dispatch_nu<NC, T, MODE_RESIDUAL>(op, u, b, out, sw, st);
        case MODE_JACOBI: return dispatch_nu<NC, T, MODE_JACOBI>(op, u, b, out, sw, st);
        case MODE_JACOBI0: return dispatch_nu<NC, T, MODE_JACOBI0>(op, u, b, out, sw, st);
        case MODE_CHEB: return dispatch_nu<NC, T, MODE_CHEB>(op, u, b, out, sw, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_cube(int ncomp, int mode, const LevelOp<T>& op, const T* u, const T* b, T* out,
                       const Sweep<T>& sw, hipStream_t st) {
    return ncomp == 1 ? launch_cube_nc<1, T>(mode, op, u, b, out, sw, st)
                      : launch_cube_nc<3, T>(mode, op, u, b, out, sw, st);
}

template hipError_t launch_cube<double>(int, int, const LevelOp<double>&, const double*,
                                        const double*, double*, const Sweep<double>&, hipStream_t);
template hipError_t launch_cube<float>(int, int, const LevelOp<float>&, const float*,
                                       const float*, float*, const Sweep<float>&, hipStream_t);

}  // namespace agca
