// C ABI of the AGCA multigrid library: hierarchy construction, level
// operations, V-cycle and FP64 outer solvers (declared in include/agca.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cube_math.h"
#include "stop_rule.h"
#include "zstencil.h"
#include "internal.h"
#include "level_ops.h"

using namespace agca;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct Level {
    int n = 0;
    int64_t nodes = 0, elems = 0;
    // per-element coefficient arrays use the internal layout of kuhn.h (elem_slot)
    double* nu64 = nullptr;      // finest: nu_L; coarse: DCA coefficient of this level
    float* nu32 = nullptr;       // FP32 copy (FP32 V-cycle)
    uint16_t* nubf = nullptr;    // BF16 copy of the finest coefficient (FP32 V-cycle option)
    int32_t* flag = nullptr;     // by element id
    int32_t* blk = nullptr;      // by element id: stored block index or -1
    int32_t* blk_soa = nullptr;  // the same in the internal layout (element loop)
    int32_t* ids = nullptr;
    int64_t nflag = 0;           // flagged elements
    int64_t nblk = 0;            // stored Galerkin blocks: nflag, or 0 when the flagged
                                 // elements' DCA coefficient carries the descendant mean
    double* blocks64 = nullptr;
    float* blocks32 = nullptr;
    double* yblk64 = nullptr;    // per-flagged-element block products (scratch)
    float* yblk32 = nullptr;
    double* diag = nullptr;
    double* dinv64 = nullptr;
    float* dinv32 = nullptr;
    double* sten64 = nullptr;    // assembled 15-point stencil (small coarse levels only)
    float* sten32 = nullptr;
    void* b = nullptr;  // V-cycle work vectors, mg precision
    void* x = nullptr;
    void* t = nullptr;
    void* r = nullptr;
    int64_t bytes = 0;
};

}  // namespace

struct agca_hier {
    agca_config cfg{};
    hipStream_t st = nullptr;
    std::vector<Level> lv;
    double* ainv0 = nullptr;
    double* partial = nullptr;
    int nb_partial = 1024;       // workgroups of the grid-stride reduction kernels
    int partial_cap = 0;
    double* red = nullptr;       // reduction results (device)
    int* counter = nullptr;      // invalid-coefficient counter (device)
    double* red_host = nullptr;  // pinned host mirror
    // FP64 solver vectors on the finest level
    double* s_r = nullptr;
    double* s_z = nullptr;
    double* s_p = nullptr;
    double* s_q = nullptr;
    float* s_r32 = nullptr;
    float* s_z32 = nullptr;
    double* trans[2] = {nullptr, nullptr};
    // Stokes (velocity: finest level, pressure: level L-1)
    std::vector<double> lam;     // Chebyshev: eigenvalue estimate of D^-1 A per level
    int64_t nu_version = 0;      // bumped by every coefficient rebuild
    int64_t mass_version = -1;   // nu_version the pressure mass was formed for
    double* st_mass = nullptr;   // lumped 1/nu pressure mass (level L-1, all nodes)
    double* st_pf = nullptr;     // fine-level scalar scratch (interpolated pressure)
    double* st_qf = nullptr;     // fine-level scalar scratch (fine divergence)
    double* st_work = nullptr;   // Krylov vectors, st_work_vecs of them
    double* st_tri = nullptr;    // during a triangular-preconditioned solve: one Stokes vector
    double* st_bfbt = nullptr;   // BFBT Schur approximation: W^-1, diag(Z) and work vectors
    int64_t bfbt_version = -1;   // nu_version W^-1 was formed for
    int st_schur_iters = 0;      // during a BFBT-preconditioned solve: CG steps per Z solve
    bool st_schur_mg = false;    // ... preconditioned by the pressure multigrid (else Jacobi)
    int st_vcycles = 1;          // during a Stokes solve: V-cycles per velocity-block inverse
    double* st_vtmp = nullptr;   // two velocity vectors for velocity_cycles > 1
    int64_t zdiag_version = -1;  // nu_version diag(Z) was formed for
    double* st_zmg = nullptr;    // pressure multigrid for Z: stencils and vectors of levels 0..L-1
    int64_t zmg_version = -1;    // nu_version the stencils were assembled for
    double* st_gs = nullptr;     // Gram-Schmidt partial sums, st_gs_cap doubles
    int64_t st_gs_cap = 0;
    int64_t st_work_vecs = 0;
    std::vector<void*> allocs;
    int64_t bytes = 0;
    bool error = false;
};

namespace {

// device reduction slots (and their pinned host mirror): Krylov coefficients of one
// Arnoldi step at the largest Stokes restart length
constexpr int AGCA_RED_SLOTS = 512;

int64_t nodes_of(int n) { return (int64_t)(n + 1) * (n + 1) * (n + 1); }
int64_t elems_of(int n) { return 6LL * n * n * n; }

#define HIPCHK(h, call)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (h)->error = true;                                                                 \
            return fail(AGCA_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
        }                                                                                      \
    } while (0)

int32_t dev_alloc(agca_hier* h, void** p, size_t bytes, int64_t* level_bytes = nullptr) {
    *p = nullptr;
    if (bytes == 0) return AGCA_OK;
    if (h->cfg.mem_limit_bytes && (uint64_t)(h->bytes + (int64_t)bytes) > h->cfg.mem_limit_bytes)
        return fail(AGCA_E_OOM, "mem_limit_bytes exceeded (" + std::to_string(h->bytes + bytes) +
                                    " > " + std::to_string(h->cfg.mem_limit_bytes) + ")");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(AGCA_E_OOM, "hipMalloc(" + std::to_string(bytes) + ") failed: " +
                                    hipGetErrorString(e));
    }
    h->allocs.push_back(*p);
    h->bytes += (int64_t)bytes;
    if (level_bytes) *level_bytes += (int64_t)bytes;
    return AGCA_OK;
}

template <typename P>
int32_t alloc_t(agca_hier* h, P** p, size_t count, int64_t* lb = nullptr) {
    void* v = nullptr;
    int32_t rc = dev_alloc(h, &v, count * sizeof(P), lb);
    *p = static_cast<P*>(v);
    return rc;
}

#define TRY(x)                       \
    do {                             \
        int32_t rc_ = (x);           \
        if (rc_ != AGCA_OK) return rc_; \
    } while (0)

bool mg32(const agca_hier* h) { return h->cfg.mg_dtype == AGCA_F32; }

// Coarse levels with at most this many cells per axis keep their operator as an
// assembled stencil (latency-bound sizes; 33^3 nodes x 135 FP64 values = 39 MB).
// AGCA_STENCIL_MAX_N overrides it (0 turns the stencils off).
int stencil_max_n() {
    static const int v = [] {
        const char* e = getenv("AGCA_STENCIL_MAX_N");
        return e ? atoi(e) : 32;
    }();
    return v;
}
size_t mg_size(const agca_hier* h) { return mg32(h) ? sizeof(float) : sizeof(double); }

template <typename T>
LevelOp<T> level_op(const agca_hier* h, int l);

template <>
LevelOp<double> level_op<double>(const agca_hier* h, int l) {
    const Level& L = h->lv[l];
    LevelOp<double> op;
    op.n = L.n;
    op.nu = L.nu64;
    op.nu_kind = AGCA_F64;
    op.blk = (l < h->cfg.L && L.nblk > 0) ? L.blk_soa : nullptr;
    op.ids = L.ids;
    op.nflag = L.nblk;
    op.blocks = L.blocks64;
    op.yblk = L.yblk64;
    op.dinv = L.dinv64;
    op.sten = L.sten64;
    return op;
}
template <>
LevelOp<float> level_op<float>(const agca_hier* h, int l) {
    const Level& L = h->lv[l];
    LevelOp<float> op;
    op.n = L.n;
    if (l == h->cfg.L && h->cfg.mg_nu_dtype == AGCA_BF16) {
        op.nu = L.nubf;
        op.nu_kind = AGCA_BF16;
    } else {
        op.nu = L.nu32;
        op.nu_kind = AGCA_F32;
    }
    op.blk = (l < h->cfg.L && L.nblk > 0) ? L.blk_soa : nullptr;
    op.ids = L.ids;
    op.nflag = L.nblk;
    op.blocks = L.blocks32;
    op.yblk = L.yblk32;
    op.dinv = L.dinv32;
    op.sten = L.sten32;
    return op;
}

int32_t check_level(const agca_hier* h, int level) {
    if (!h) return fail(AGCA_E_INVALID, "null hierarchy");
    if (h->error) return fail(AGCA_E_STATE, "hierarchy is in an error state");
    if (level < 0 || level > h->cfg.L) return fail(AGCA_E_INVALID, "level out of range");
    return AGCA_OK;
}

int32_t check_dtype(const agca_hier* h, int dtype, bool need_mg) {
    if (dtype != AGCA_F64 && dtype != AGCA_F32) return fail(AGCA_E_INVALID, "dtype must be F64 or F32");
    if (dtype == AGCA_F32 && !mg32(h)) return fail(AGCA_E_INVALID, "F32 needs mg_dtype == F32");
    if (need_mg && dtype != h->cfg.mg_dtype) return fail(AGCA_E_INVALID, "dtype must equal mg_dtype");
    return AGCA_OK;
}

// ---------------------------------------------------------------------------
// level operations (templated on the vector precision)
// ---------------------------------------------------------------------------
// one pass of the level operator: the assembled stencil where the level has one,
// the element loop otherwise
template <typename T>
int32_t do_cube(agca_hier* h, int l, int mode, const T* u, const T* b, T* out, const Sweep<T>& sw) {
    const LevelOp<T> op = level_op<T>(h, l);
    if (op.sten)
        HIPCHK(h, launch_stencil<T>(h->cfg.ncomp, mode, op.n, op.sten, u, b, op.dinv, out, sw, h->st));
    else
        HIPCHK(h, launch_cube<T>(h->cfg.ncomp, mode, op, u, b, out, sw, h->st));
    return AGCA_OK;
}
template <typename T>
int32_t do_cube(agca_hier* h, int l, int mode, const T* u, const T* b, T* out, T omega) {
    return do_cube<T>(h, l, mode, u, b, out, jacobi_sweep<T>(omega));
}

// Chebyshev pass coefficients (Cheb, level_ops.h) as a Sweep
template <typename T>
Sweep<T> cheb_sweep(const Cheb& ch, int k, const T* xprev) {
    Sweep<T> s;
    if (k == 0) {
        s.omega = T(1.0 / ch.theta);
        s.omega0 = s.omega;
        return s;
    }
    double c1, c2;
    ch.coef(k, &c1, &c2);
    s.alpha = T(1.0 + c1);
    s.gamma = T(-c1);
    s.omega = T(c2);
    s.omega0 = T(1.0 / ch.theta);  // the pass-0 scaling, for the fused first two passes
    s.xprev = xprev;
    return s;
}

// whether the first two pre-sweeps can be one pass on level l: the element loop
// without stored blocks (whose products are formed from a stored u before the pass);
// on stencil levels the separate first sweep measures as fast
template <typename T>
bool fusable(const agca_hier* h, int l) {
    const LevelOp<T> op = level_op<T>(h, l);
    return op.sten == nullptr && op.blk == nullptr;
}

// Mode and coefficients of smoothing pass k on level l (k >= 1 before the coarse
// correction, where pass 0 is formed from zero; k >= 0 after it): damped Jacobi; for
// Chebyshev, pass 0 is x + D^-1 (b - A x) / theta, pass 1 before the correction starts
// from x_prev = 0 (gamma = 0), every other pass is a Chebyshev step reading x_prev.
template <typename T>
int smooth_pass_coef(const agca_hier* h, int l, bool pre, int k, const T* xprev, Sweep<T>* sw) {
    if (h->cfg.smoother != AGCA_SMOOTH_CHEBYSHEV) {
        *sw = jacobi_sweep<T>(T(h->cfg.omega));
        return MODE_JACOBI;
    }
    const Cheb ch(h->lam[l]);
    if (k == 0) {
        *sw = cheb_sweep<T>(ch, 0, nullptr);
        return MODE_JACOBI;
    }
    *sw = cheb_sweep<T>(ch, k, xprev);
    if (pre && k == 1) {
        sw->gamma = T(0);
        sw->xprev = nullptr;
        return MODE_JACOBI;
    }
    return MODE_CHEB;
}

// Levels 1..K that the coarse end of a V-cycle runs in one workgroup (k_coarse_cycle.hip):
// consecutive assembled-stencil levels from level 1 up, each below the finest level, whose
// stencil one compute unit reads per pass in about a microsecond (at most
// kFuseStencilBytes: levels 1-2 of a scalar hierarchy, level 1 of a vector one; beyond
// that the one workgroup is slower than a launch per pass spread over the chip), with at
// most AGCA_FUSE_MAX_N cells per axis (default 8; 0 turns the fused cycle off) and the
// LDS of levels 0..K within 64 KiB; 0 when level 1 does not qualify or a smoothing phase
// has more passes than the fused cycle takes.
constexpr size_t kFuseStencilBytes = 160 * 1024;
int fuse_max_n() {
    static const int v = [] {
        const char* e = getenv("AGCA_FUSE_MAX_N");
        return e ? atoi(e) : 8;
    }();
    return v;
}
template <typename T>
int coarse_cycle_levels(const agca_hier* h) {
    if (h->cfg.pre_sweeps > kCyclePasses || h->cfg.post_sweeps > kCyclePasses) return 0;
    const int nc = h->cfg.ncomp;
    int K = 0;
    for (int l = 1; l <= kCycleLevels && l < h->cfg.L; ++l) {
        const Level& lv = h->lv[l];
        if (!level_op<T>(h, l).sten || lv.n != (2 << l) || lv.n > fuse_max_n()) break;
        if ((size_t)nc * nc * kStencilPoints * lv.nodes * sizeof(T) > kFuseStencilBytes) break;
        if (coarse_cycle_lds(nc, l, sizeof(T)) > 65536) break;
        K = l;
    }
    return K;
}

template <typename T>
int32_t do_smooth(agca_hier* h, int l, int sweeps, double omega, const T* b, T* x) {
    T* tmp = static_cast<T*>(h->lv[l].t);
    T* src = x;
    T* dst = tmp;
    for (int i = 0; i < sweeps; ++i) {
        TRY(do_cube<T>(h, l, MODE_JACOBI, src, b, dst, T(omega)));
        T* s = src;
        src = dst;
        dst = s;
    }
    if (src != x)
        HIPCHK(h, hipMemcpyAsync(x, src, sizeof(T) * h->cfg.ncomp * h->lv[l].nodes,
                                 hipMemcpyDeviceToDevice, h->st));
    return AGCA_OK;
}

// One V(pre,post)-cycle from a zero initial guess, with damped Jacobi or the Chebyshev
// smoother (pre / post = number of passes = Chebyshev degree).  On element-loop levels
// without stored blocks the first two pre-smoothing passes from zero are one kernel
// (the first, x = omega0 D^-1 b, is formed while loading; Chebyshev only for degree
// 2, whose second pass needs no stored first iterate); elsewhere the first pass is
// the elementwise x = omega0 D^-1 b.  Every further pass writes the level's other
// buffer (a Chebyshev pass reads the previous iterate from it at the same node), so
// the passes ping-pong, and on the finest level the starting buffer is chosen so
// that the last pass lands in the caller's x (no copies).
template <typename T>
int32_t do_vcycle(agca_hier* h, const T* bL, T* xL) {
    const int L = h->cfg.L, nc = h->cfg.ncomp;
    const T om = T(h->cfg.omega);
    const int pre = h->cfg.pre_sweeps, post = h->cfg.post_sweeps;
    const bool cheb = h->cfg.smoother == AGCA_SMOOTH_CHEBYSHEV;
    // pass k of a smoothing phase; xprev = the iterate before the current one
    auto pass = [&](int l, bool pre_phase, int k, const T* x, const T* bl, T* out, const T* xprev) -> int32_t {
        Sweep<T> sw;
        const int mode = smooth_pass_coef<T>(h, l, pre_phase, k, xprev, &sw);
        return do_cube<T>(h, l, mode, x, bl, out, sw);
    };
    // levels K..1 and the level-0 solve run as one workgroup-resident kernel
    const int K = coarse_cycle_levels<T>(h);
    std::vector<T*> xcur(L + 1, nullptr), xalt(L + 1, nullptr);
    for (int l = L; l > K; --l) {
        const int64_t cnt = (int64_t)nc * h->lv[l].nodes;
        const T* bl = (l == L) ? bL : static_cast<const T*>(h->lv[l].b);
        T* home = (l == L) ? xL : static_cast<T*>(h->lv[l].x);
        T* other = static_cast<T*>(h->lv[l].t);
        const bool fuse = fusable<T>(h, l) && (!cheb || pre == 2);
        // out-of-place launches that write this level's iterate after its first producer
        // (pre-sweeps after the first pass, then every post-sweep; the prolongation
        // adds in place)
        const int first = (pre >= 2 && fuse) ? 2 : (pre > 0 ? 1 : 0);
        const int launches = (pre - first) + post;
        T* cur = (launches % 2 == 0) ? home : other;
        T* alt = (cur == home) ? other : home;
        const LevelOp<T> op = level_op<T>(h, l);
        const T om0 = cheb ? T(1.0 / Cheb(h->lam[l]).theta) : om;
        if (first == 2) {
            // passes 0 and 1 from zero: x1 = om0 D^-1 b, then (x_prev = 0)
            const Sweep<T> sw = cheb ? cheb_sweep<T>(Cheb(h->lam[l]), 1, nullptr) : jacobi_sweep<T>(om);
            TRY(do_cube<T>(h, l, MODE_JACOBI0, nullptr, bl, cur, sw));
        } else if (first == 1) {
            HIPCHK(h, launch_first_sweep<T>(cnt, om0, op.dinv, bl, cur, h->st));
        } else {
            HIPCHK(h, launch_fill<T>(cnt, T(0), cur, h->st));
        }
        for (int i = first; i < pre; ++i) {
            TRY(pass(l, true, i, cur, bl, alt, alt));
            std::swap(cur, alt);
        }
        xcur[l] = cur;
        xalt[l] = alt;
        T* rl = static_cast<T*>(h->lv[l].r);
        TRY(do_cube<T>(h, l, MODE_RESIDUAL, cur, bl, rl, T(0)));
        HIPCHK(h, launch_restrict<T>(nc, h->lv[l].n, rl, static_cast<T*>(h->lv[l - 1].b), h->st));
    }
    if (K >= 1) {
        CoarseCycle<T> cc;
        cc.pre = pre;
        cc.post = post;
        for (int l = 1; l <= K; ++l) {
            const LevelOp<T> op = level_op<T>(h, l);
            cc.sten[l] = op.sten;
            cc.dinv[l] = op.dinv;
            cc.first_omega[l] = cheb ? T(1.0 / Cheb(h->lam[l]).theta) : om;
            for (int k = 0; k < kCyclePasses; ++k) {
                Sweep<T> sw;
                if (k >= 1 && k < pre) {
                    cc.pre_mode[l][k] = (int8_t)smooth_pass_coef<T>(h, l, true, k, nullptr, &sw);
                    cc.pre_c[l][k][0] = sw.alpha;
                    cc.pre_c[l][k][1] = sw.gamma;
                    cc.pre_c[l][k][2] = sw.omega;
                }
                if (k < post) {
                    cc.post_mode[l][k] = (int8_t)smooth_pass_coef<T>(h, l, false, k, nullptr, &sw);
                    cc.post_c[l][k][0] = sw.alpha;
                    cc.post_c[l][k][1] = sw.gamma;
                    cc.post_c[l][k][2] = sw.omega;
                }
            }
        }
        cc.ainv = h->ainv0;
        cc.b = static_cast<const T*>(h->lv[K].b);
        cc.x = static_cast<T*>(h->lv[K].x);
        HIPCHK(h, launch_coarse_cycle<T>(nc, K, cc, h->st));
        xcur[K] = cc.x;
    } else {
        HIPCHK(h, launch_coarse_solve<T>(nc, h->ainv0, static_cast<const T*>(h->lv[0].b),
                                         static_cast<T*>(h->lv[0].x), h->st));
        xcur[0] = static_cast<T*>(h->lv[0].x);
    }
    for (int l = K + 1; l <= L; ++l) {
        const T* bl = (l == L) ? bL : static_cast<const T*>(h->lv[l].b);
        T* cur = xcur[l];
        T* alt = xalt[l];
        HIPCHK(h, launch_prolong_add<T>(nc, h->lv[l].n, xcur[l - 1], cur, h->st));
        for (int i = 0; i < post; ++i) {
            TRY(pass(l, false, i, cur, bl, alt, alt));
            std::swap(cur, alt);
        }
        xcur[l] = cur;
    }
    if (xcur[L] != xL)  // only when pre = post = 0 parity cannot place it
        HIPCHK(h, hipMemcpyAsync(xL, xcur[L], sizeof(T) * nc * h->lv[L].nodes,
                                 hipMemcpyDeviceToDevice, h->st));
    return AGCA_OK;
}

// x . y into reduction slot `slot` (device) and *out (host); synchronises
template <typename T>
int32_t do_dot(agca_hier* h, const T* x, const T* y, int64_t count, double* out, int slot = 0) {
    HIPCHK(h, launch_dot_partial<T>(x, y, count, h->partial, h->nb_partial, h->st));
    HIPCHK(h, launch_sum_partials(h->partial, h->nb_partial, h->red + slot, h->st));
    HIPCHK(h, hipMemcpyAsync(h->red_host + slot, h->red + slot, sizeof(double), hipMemcpyDeviceToHost,
                             h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    *out = h->red_host[slot];
    return AGCA_OK;
}

// sum nb partials into red[slot] (device)
int32_t reduce_to(agca_hier* h, const double* partial, int nb, int slot) {
    HIPCHK(h, launch_sum_partials(partial, nb, h->red + slot, h->st));
    return AGCA_OK;
}
// copy red[first .. first + k) to the host and wait
int32_t fetch(agca_hier* h, int k, double* out, int first = 0) {
    HIPCHK(h, hipMemcpyAsync(h->red_host + first, h->red + first, sizeof(double) * k,
                             hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    for (int i = 0; i < k; ++i) out[i] = h->red_host[first + i];
    return AGCA_OK;
}

// reduction slots of the two helpers below and of the Krylov solvers' residual
// replacement, clear of the solvers' scalars (slots 0..4, which must survive a
// replacement in the middle of an iteration)
constexpr int kSlotFloor = 8;
constexpr int kSlotReplace = 10;

// ||b||_2 over the free dofs of a finest-level vector (boundary slots are not part of it)
int32_t interior_norm(agca_hier* h, const double* b, double* out) {
    const int L = h->cfg.L;
    HIPCHK(h, launch_interior_dot<double>(h->cfg.ncomp, h->lv[L].n, b, b, h->partial, h->nb_partial,
                                          h->st));
    TRY(reduce_to(h, h->partial, h->nb_partial, kSlotFloor));
    double v = 0.0;
    TRY(fetch(h, 1, &v, kSlotFloor));
    *out = std::sqrt(v);
    return AGCA_OK;
}

// Rounding floor of the relative residual of x (eq. (4.3) evaluated in FP64):
//   rho = u || |b| + sum_e |A_e| |x_e| ||_2 / ||b||_2  over the free dofs, u = 2^-53.
// Rounding every entry of x once more moves b - A x by at most u sum_e |A_e| |x_e|
// entrywise, so no solver can certify a relative residual much below rho for an FP64
// iterate near x.
constexpr double kUnitRoundoff = 1.1102230246251565e-16;  // 2^-53
// the two sums: s_sq = sum (|b_i| + (sum_e |A_e||x_e|)_i)^2, b_sq = sum b_i^2 (free dofs)
int32_t floor_sums(agca_hier* h, const double* b, const double* x, double* s_sq, double* b_sq) {
    const int L = h->cfg.L;
    const Level& lv = h->lv[L];
    HIPCHK(h, launch_floor_terms(h->cfg.ncomp, lv.n, lv.nu64, 1.0 / (6.0 * lv.n), b, x, h->partial,
                                 h->nb_partial, h->st));
    TRY(reduce_to(h, h->partial, h->nb_partial, kSlotFloor));
    TRY(reduce_to(h, h->partial + h->nb_partial, h->nb_partial, kSlotFloor + 1));
    double v[2] = {0.0, 0.0};
    TRY(fetch(h, 2, v, kSlotFloor));
    *s_sq = v[0];
    *b_sq = v[1];
    return AGCA_OK;
}
int32_t residual_floor(agca_hier* h, const double* b, const double* x, double* rho) {
    double s_sq = 0.0, b_sq = 0.0;
    TRY(floor_sums(h, b, x, &s_sq, &b_sq));
    *rho = b_sq > 0.0 ? kUnitRoundoff * std::sqrt(s_sq) / std::sqrt(b_sq) : 0.0;
    return AGCA_OK;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
int32_t validate(const agca_config* c) {
    if (!c) return fail(AGCA_E_INVALID, "null config");
    if (c->L < 1 || c->L > 9) return fail(AGCA_E_INVALID, "L must be in [1, 9]");
    if (c->ncomp != 1 && c->ncomp != 3) return fail(AGCA_E_INVALID, "ncomp must be 1 or 3");
    if (c->flag_mode != AGCA_FLAG_RATIO && c->flag_mode != AGCA_FLAG_MACRO &&
        c->flag_mode != AGCA_FLAG_NONE && c->flag_mode != AGCA_FLAG_ALL)
        return fail(AGCA_E_INVALID, "unknown flag_mode");
    if (c->mg_dtype != AGCA_F64 && c->mg_dtype != AGCA_F32)
        return fail(AGCA_E_INVALID, "mg_dtype must be F64 or F32");
    if (c->mg_nu_dtype != AGCA_F64 && c->mg_nu_dtype != AGCA_F32 && c->mg_nu_dtype != AGCA_BF16)
        return fail(AGCA_E_INVALID, "mg_nu_dtype must be F64, F32 or BF16");
    if (c->mg_dtype == AGCA_F64 && c->mg_nu_dtype != AGCA_F64)
        return fail(AGCA_E_INVALID, "an FP64 V-cycle needs an FP64 coefficient");
    if (c->mg_dtype == AGCA_F32 && c->mg_nu_dtype == AGCA_F64)
        return fail(AGCA_E_INVALID, "an FP32 V-cycle uses an FP32 or BF16 coefficient");
    if (c->coarse_storage != AGCA_STORE_BLOCKS && c->coarse_storage != AGCA_STORE_MEAN)
        return fail(AGCA_E_INVALID, "unknown coarse_storage");
    if (c->smoother != AGCA_SMOOTH_JACOBI && c->smoother != AGCA_SMOOTH_CHEBYSHEV)
        return fail(AGCA_E_INVALID, "unknown smoother");
    if (c->pre_sweeps < 0 || c->post_sweeps < 0 || c->pre_sweeps > 64 || c->post_sweeps > 64)
        return fail(AGCA_E_INVALID, "sweeps must be in [0, 64]");
    if (!(c->omega > 0.0 && c->omega < 2.0)) return fail(AGCA_E_INVALID, "omega must be in (0, 2)");
    if (!(c->flag_ratio >= 1.0) || !std::isfinite(c->flag_ratio))
        return fail(AGCA_E_INVALID, "flag_ratio must be finite and >= 1");
    return AGCA_OK;
}

int32_t count_invalid(agca_hier* h, const double* v, int64_t n, int* out) {
    int* cnt = h->counter;
    HIPCHK(h, hipMemsetAsync(cnt, 0, sizeof(int), h->st));
    HIPCHK(h, launch_count_invalid(v, n, cnt, h->st));
    HIPCHK(h, hipMemcpyAsync(out, cnt, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return AGCA_OK;
}

// level-0 operator on its single free node (1,1,1): ncomp x ncomp, inverted on the host
int32_t ensure_solver_vectors(agca_hier* h) {
    if (h->s_r) return AGCA_OK;
    const int64_t cnt = (int64_t)h->cfg.ncomp * h->lv[h->cfg.L].nodes;
    TRY(alloc_t(h, &h->s_r, cnt));
    TRY(alloc_t(h, &h->s_z, cnt));
    TRY(alloc_t(h, &h->s_p, cnt));
    TRY(alloc_t(h, &h->s_q, cnt));
    if (mg32(h)) {
        TRY(alloc_t(h, &h->s_r32, cnt));
        TRY(alloc_t(h, &h->s_z32, cnt));
    }
    return AGCA_OK;
}


// Largest eigenvalue of the symmetric tridiagonal matrix (diagonal a[0..m), off-diagonal
// b[0..m-1)): bisection on the Sturm count (number of eigenvalues below x = number of
// negative pivots of the LDL^T factorisation of T - x I), inside the Gershgorin bounds.
double tridiag_max_eigenvalue(const std::vector<double>& a, const std::vector<double>& b) {
    const int m = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
            d = (a[i] - x) - (i > 0 ? off / d : 0.0);
            if (d == 0.0) d = -1e-300;  // x is (to rounding) a pivot zero: count it below
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fabs(hi); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == m) hi = mid;  // every eigenvalue lies below mid
        else lo = mid;
    }
    return hi;
}

// Largest eigenvalue of D^-1 A_l for the Chebyshev smoother, levels 1..L, in FP64: the
// largest Ritz value of 20 Lanczos steps in the D inner product from (-1)^(x+y+z) on the
// free nodes (a lower bound of the eigenvalue):
//   alpha_k = v_k.A v_k, w = D^-1 A v_k - alpha_k v_k - beta_{k-1} v_{k-1},
//   beta_k = sqrt(w.Dw), v_{k+1} = w / beta_k; the process ends early when beta_k
// vanishes against alpha_k (an invariant Krylov space).
constexpr int kLanczosSteps = 20;
constexpr double kLanczosBreakdown = 1e-12;

int32_t estimate_eigenvalues(agca_hier* h) {
    TRY(ensure_solver_vectors(h));
    const int L = h->cfg.L, nc = h->cfg.ncomp;
    constexpr int K = kLanczosSteps;
    static_assert(2 * K + 1 <= AGCA_RED_SLOTS, "reduction slots");
    h->lam.assign(L + 1, 0.0);
    std::vector<double> co(2 * K + 1);
    for (int l = 1; l <= L; ++l) {
        const Level& lv = h->lv[l];
        const int64_t cnt = (int64_t)nc * lv.nodes;
        double *v = h->s_r, *vprev = h->s_z, *w = h->s_p, *y = h->s_q;
        // the whole process runs on the device (alpha_k in slot k, beta_k^2 in slot K + k,
        // the start vector's D-norm^2 in slot 2K) and is read back once
        HIPCHK(h, launch_alternating(nc, lv.n, w, h->st));
        HIPCHK(h, launch_mul(cnt, lv.diag, w, y, h->st));
        HIPCHK(h, launch_dot_partial<double>(w, y, cnt, h->partial, h->nb_partial, h->st));
        TRY(reduce_to(h, h->partial, h->nb_partial, 2 * K));
        HIPCHK(h, launch_scale_rsqrt(cnt, w, h->red + 2 * K, v, h->st));
        const LevelOp<double> op = level_op<double>(h, l);
        for (int k = 0; k < K; ++k) {
            if (op.sten) {
                TRY(do_cube<double>(h, l, MODE_APPLY, v, nullptr, y, 0.0));
                HIPCHK(h, launch_dot_partial<double>(v, y, cnt, h->partial, h->nb_partial, h->st));
                TRY(reduce_to(h, h->partial, h->nb_partial, k));
            } else {
                // element-loop level: y = A v with v . A v in the same pass
                int nbq = 0;
                HIPCHK(h, launch_cube_dot(nc, op, v, y, h->partial, &nbq, h->st));
                TRY(reduce_to(h, h->partial, nbq, k));
            }
            HIPCHK(h, launch_lanczos_step(cnt, y, lv.diag, v, k > 0 ? vprev : nullptr, h->red + k,
                                          k > 0 ? h->red + K + k - 1 : nullptr, w, h->partial,
                                          h->nb_partial, h->st));
            TRY(reduce_to(h, h->partial, h->nb_partial, K + k));
            // after a breakdown (beta_k = 0) the later steps compute non-finite values that
            // are never read: the host cuts the sequence at the breakdown
            HIPCHK(h, launch_scale_rsqrt(cnt, w, h->red + K + k, vprev, h->st));
            std::swap(v, vprev);
        }
        TRY(fetch(h, 2 * K + 1, co.data()));
        if (!(co[2 * K] > 0.0) || !std::isfinite(co[2 * K]))
            return fail(AGCA_E_NUMERIC, "eigenvalue estimate failed");
        std::vector<double> alpha, beta;
        for (int k = 0; k < K; ++k) {
            const double a = co[k], s = co[K + k];
            if (!std::isfinite(a) || !std::isfinite(s)) return fail(AGCA_E_NUMERIC, "eigenvalue estimate failed");
            alpha.push_back(a);
            const double b = std::sqrt(std::max(s, 0.0));
            if (!(b > kLanczosBreakdown * std::fabs(a))) break;
            beta.push_back(b);
        }
        beta.resize(alpha.size() - 1);
        h->lam[l] = tridiag_max_eigenvalue(alpha, beta);
        if (!(h->lam[l] > 0.0) || !std::isfinite(h->lam[l]))
            return fail(AGCA_E_NUMERIC, "eigenvalue estimate failed");
    }
    return AGCA_OK;
}

int32_t build_coarsest(agca_hier* h) {
    const int nc = h->cfg.ncomp, M = 4 * nc;
    Level& L0 = h->lv[0];
    std::vector<double> nu(48);
    HIPCHK(h, hipMemcpyAsync(nu.data(), L0.nu64, 48 * sizeof(double), hipMemcpyDeviceToHost, h->st));
    std::vector<int32_t> blk(48, -1);
    std::vector<double> blocks;
    const bool has_blocks = h->cfg.L > 0 && L0.nblk > 0;
    if (has_blocks) {
        HIPCHK(h, hipMemcpyAsync(blk.data(), L0.blk, 48 * sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
        blocks.resize((size_t)L0.nblk * M * M);
        HIPCHK(h, hipMemcpyAsync(blocks.data(), L0.blocks64, blocks.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, h->st));
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    const double scale = 1.0 / (6.0 * 2);
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    // node (1,1,1) is corner k = 7 - (cell offset bits) of each of the 8 cells
    for (int cell = 0; cell < 8; ++cell) {
        const int k = 7 - cell;  // cell (cx,cy,cz) = bits of 'cell'; node at corner 7 - cell
        for (int s = 0; s < 6; ++s) {
            int a = -1;
            for (int j = 0; j < 4; ++j)
                if (path_corner(s, j) == k) a = j;
            if (a < 0) continue;
            const int e = 6 * cell + s;
            for (int c = 0; c < nc; ++c)
                for (int d = 0; d < nc; ++d) {
                    double v;
                    if (blk[e] >= 0)
                        v = blocks[(size_t)blk[e] * M * M + (4 * c + a) * M + 4 * d + a];
                    else
                        v = nu[elem_slot(s, cell, 8)] * scale * elem_entry(nc, s, c, a, d, a);
                    A[c][d] += v;
                }
        }
    }
    double inv[9] = {0};
    if (nc == 1) {
        if (!(A[0][0] > 0)) return fail(AGCA_E_NUMERIC, "coarsest operator is not positive");
        inv[0] = 1.0 / A[0][0];
    } else {
        const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        if (!(std::fabs(det) > 0)) return fail(AGCA_E_NUMERIC, "coarsest operator is singular");
        inv[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
        inv[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
        inv[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
        inv[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
        inv[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
        inv[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
        inv[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
        inv[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
        inv[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    }
    HIPCHK(h, hipMemcpyAsync(h->ainv0, inv, sizeof(double) * nc * nc, hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return AGCA_OK;
}

// log_fine: nu_fine holds log nu (exponentiated while it is copied)
int32_t build_operators(agca_hier* h, const double* nu_fine, const double* const* nu_coarse,
                        bool log_fine = false) {
    const int L = h->cfg.L, nc = h->cfg.ncomp, M = 4 * nc;
    ++h->nu_version;
    // coefficients
    for (int l = 0; l <= L; ++l) {
        const double* src = (l == L) ? nu_fine : nu_coarse[l];
        if (!src) return fail(AGCA_E_INVALID, "null coefficient pointer for level " + std::to_string(l));
        HIPCHK(h, launch_to_internal(h->lv[l].elems / 6, src, h->lv[l].nu64, l == L && log_fine, h->st));
    }
    for (int l = 0; l <= L; ++l) {
        int bad = 0;
        TRY(count_invalid(h, h->lv[l].nu64, h->lv[l].elems, &bad));
        if (bad)
            return fail(AGCA_E_INVALID, std::to_string(bad) + " coefficient values on level " +
                                            std::to_string(l) + " are not finite and positive");
    }
    // flags: min/max pyramid from level L-1 down to 0
    {
        double *mn[2] = {nullptr, nullptr}, *mx[2] = {nullptr, nullptr}, *mean[2] = {nullptr, nullptr};
        const bool store_mean = h->cfg.coarse_storage == AGCA_STORE_MEAN;
        const int64_t emax = h->lv[L - 1].elems;
        void* scratch = nullptr;
        size_t sbytes = 0;
        HIPCHK(h, compact_scratch_bytes(emax, &sbytes));
        // transient buffers: allocated with plain hipMalloc and released at the end of setup
        std::vector<void*> tmp;
        auto talloc = [&](void** p, size_t bytes) -> int32_t {
            hipError_t e = hipMalloc(p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(AGCA_E_OOM, "transient hipMalloc failed");
            }
            tmp.push_back(*p);
            return AGCA_OK;
        };
        auto release = [&]() {
            (void)hipStreamSynchronize(h->st);
            for (void* p : tmp) (void)hipFree(p);
            tmp.clear();
        };
        uint64_t macro_bits = 0;
        for (int k = 0; k < 48; ++k)
            if (h->cfg.macro_flags[k]) macro_bits |= (uint64_t)1 << k;
        int32_t rc = AGCA_OK;
        for (int i = 0; i < 2 && rc == AGCA_OK; ++i) {
            rc = talloc((void**)&mn[i], emax * sizeof(double));
            if (rc == AGCA_OK) rc = talloc((void**)&mx[i], emax * sizeof(double));
            if (rc == AGCA_OK && store_mean) rc = talloc((void**)&mean[i], emax * sizeof(double));
        }
        if (rc == AGCA_OK) rc = talloc(&scratch, sbytes);
        int64_t* cnt_dev = nullptr;
        if (rc == AGCA_OK) rc = talloc((void**)&cnt_dev, sizeof(int64_t) * 16);
        if (rc != AGCA_OK) {
            release();
            return rc;
        }
        for (int l = L - 1; l >= 0; --l) {
            const int cur = l & 1, fin = (l + 1) & 1;
            hipError_t e = (l == L - 1)
                               ? launch_minmax_from_fine(h->lv[l].n, h->lv[L].nu64, mn[cur], mx[cur], h->st)
                               : launch_minmax_up(h->lv[l].n, mn[fin], mx[fin], mn[cur], mx[cur], h->st);
            if (e == hipSuccess)
                e = (h->cfg.flag_mode == AGCA_FLAG_MACRO)
                        ? launch_flag_macro(h->lv[l].elems, h->lv[l].n, l, macro_bits, h->lv[l].flag, h->st)
                        : launch_flag(h->lv[l].elems, mn[cur], mx[cur], h->cfg.flag_ratio, h->cfg.flag_mode,
                                      h->lv[l].flag, h->st);
            if (e == hipSuccess && store_mean) {
                // the flagged elements' Galerkin blocks equal their DCA element matrices with
                // the mean finest coefficient: keep that mean as their coefficient instead
                e = (l == L - 1) ? launch_mean_from_fine(h->lv[l].n, h->lv[L].nu64, mean[cur], h->st)
                                 : launch_mean_up(h->lv[l].n, mean[fin], mean[cur], h->st);
                if (e == hipSuccess)
                    e = launch_override_mean(h->lv[l].elems, h->lv[l].flag, mean[cur], h->lv[l].nu64, h->st);
            }
            if (e == hipSuccess)
                e = launch_compact(h->lv[l].elems, h->lv[l].flag, h->lv[l].blk, h->lv[l].blk_soa,
                                   h->lv[l].ids, cnt_dev + l, scratch, sbytes, h->st);
            if (e != hipSuccess) {
                release();
                h->error = true;
                return fail(AGCA_E_HIP, std::string("flag kernels: ") + hipGetErrorString(e));
            }
        }
        std::vector<int64_t> counts(16, 0);
        hipError_t e = hipMemcpyAsync(counts.data(), cnt_dev, sizeof(int64_t) * L,
                                      hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        release();
        if (e != hipSuccess) {
            h->error = true;
            return fail(AGCA_E_HIP, std::string("flag count readback: ") + hipGetErrorString(e));
        }
        for (int l = 0; l < L; ++l) {
            h->lv[l].nflag = counts[l];
            h->lv[l].nblk = (h->cfg.coarse_storage == AGCA_STORE_MEAN) ? 0 : counts[l];
        }
    }
    // block storage
    for (int l = 0; l < L; ++l) {
        Level& lv = h->lv[l];
        lv.blocks64 = nullptr;
        lv.blocks32 = nullptr;
        if (lv.nblk > 0) {
            TRY(alloc_t(h, &lv.blocks64, (size_t)lv.nblk * M * M, &lv.bytes));
            TRY(alloc_t(h, &lv.yblk64, (size_t)lv.nblk * M, &lv.bytes));
            if (mg32(h)) {
                TRY(alloc_t(h, &lv.blocks32, (size_t)lv.nblk * M * M, &lv.bytes));
                TRY(alloc_t(h, &lv.yblk32, (size_t)lv.nblk * M, &lv.bytes));
            }
        }
    }
    // Galerkin blocks, bottom-up (eq. (2.7))
    {
        int lowest = -1;  // coarsest... any flagged level <= L-2 ?
        for (int l = 0; l <= L - 2; ++l)
            if (h->lv[l].nblk > 0) {
                lowest = l;
                break;
            }
        const double h_fine = 1.0 / h->lv[L].n;
        if (lowest < 0) {
            if (L >= 1 && h->lv[L - 1].nblk > 0)
                HIPCHK(h, launch_gca_from_fine(nc, h->lv[L - 1].n, h->lv[L - 1].nblk, h->lv[L - 1].ids,
                                               h->lv[L].nu64, h_fine, h->lv[L - 1].blocks64, h->st));
        } else {
            // levels L-2 .. lowest need the Galerkin matrices of every element of the level
            // below them while any coarser level is flagged; transient ping-pong buffers
            std::vector<void*> tmp;
            int32_t rc = AGCA_OK;
            for (int i = 0; i < 2; ++i) {
                const int l = L - 2 - i;
                if (l < lowest + 1) break;  // trans of level l is needed only if some level < l is flagged
                void* p = nullptr;
                hipError_t e = hipMalloc(&p, (size_t)h->lv[l].elems * M * M * sizeof(double));
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    rc = fail(AGCA_E_OOM, "transient Galerkin buffer allocation failed");
                    break;
                }
                tmp.push_back(p);
                h->trans[i] = static_cast<double*>(p);
            }
            if (rc == AGCA_OK) {
                const int l2 = L - 2;
                double* out2 = (l2 > lowest) ? h->trans[0] : nullptr;
                hipError_t e = launch_gca_fused2(nc, h->lv[l2].n, h->lv[L].nu64, h_fine, h->lv[L - 1].blk,
                                                 h->lv[L - 1].blocks64, h->lv[l2].blk, h->lv[l2].blocks64,
                                                 out2, h->st);
                int cur = 0;
                for (int l = L - 3; l >= lowest && e == hipSuccess; --l) {
                    double* in = h->trans[cur];
                    // trans[1-cur] held level l+2 (no longer needed) and is large enough
                    double* out = (l > lowest) ? h->trans[1 - cur] : nullptr;
                    e = launch_gca_up(nc, h->lv[l].n, in, h->lv[l].blk, h->lv[l].blocks64, out, h->st);
                    cur = 1 - cur;
                }
                if (e == hipSuccess) e = hipStreamSynchronize(h->st);
                if (e != hipSuccess) {
                    h->error = true;
                    rc = fail(AGCA_E_HIP, std::string("Galerkin kernels: ") + hipGetErrorString(e));
                }
            }
            for (void* p : tmp) (void)hipFree(p);
            h->trans[0] = h->trans[1] = nullptr;
            if (rc != AGCA_OK) return rc;
        }
    }
    // diagonals, FP32 copies
    for (int l = 0; l <= L; ++l) {
        Level& lv = h->lv[l];
        const double scale = 1.0 / (6.0 * lv.n);
        HIPCHK(h, launch_diagonal(nc, lv.n, lv.nu64, scale, (l < L && lv.nblk > 0) ? lv.blk : nullptr,
                                  lv.blocks64, lv.diag, h->st));
        const int64_t cnt = (int64_t)nc * lv.nodes;
        if (mg32(h)) {
            HIPCHK(h, launch_invert_diag<float>(cnt, lv.diag, lv.dinv32, h->st));
            // the finest level holds either an FP32 or a BF16 copy, coarse levels an FP32 one
            if (l == L && h->cfg.mg_nu_dtype == AGCA_BF16)
                HIPCHK(h, launch_cast(AGCA_F64, AGCA_BF16, lv.nu64, lv.nubf, lv.elems, h->st));
            else
                HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, lv.nu64, lv.nu32, lv.elems, h->st));
            if (lv.blocks32)
                HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, lv.blocks64, lv.blocks32,
                                      (int64_t)lv.nblk * M * M, h->st));
        } else {
            HIPCHK(h, launch_invert_diag<double>(cnt, lv.diag, lv.dinv64, h->st));
        }
        if (lv.sten64) {
            HIPCHK(h, launch_stencil_assemble(nc, lv.n, lv.nu64, scale, lv.nblk > 0 ? lv.blk_soa : nullptr,
                                              lv.blocks64, lv.sten64, h->st));
            if (lv.sten32)
                HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, lv.sten64, lv.sten32,
                                      (int64_t)nc * nc * 15 * lv.nodes, h->st));
        }
    }
    TRY(build_coarsest(h));
    if (h->cfg.smoother == AGCA_SMOOTH_CHEBYSHEV) TRY(estimate_eigenvalues(h));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return AGCA_OK;
}

// Teardown and re-allocation paths release memory on a best-effort basis: an error
// reported by hipFree there leaves nothing for the caller to act on, so it is dropped.
void free_all(agca_hier* h) {
    if (h->st) (void)hipStreamSynchronize(h->st);
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->red_host) (void)hipHostFree(h->red_host);
    h->red_host = nullptr;
}

int32_t free_blocks(agca_hier* h) {
    // blocks are re-sized on every rebuild: drop the old ones from the allocation list
    for (auto& lv : h->lv) {
        for (void* p : {(void*)lv.blocks64, (void*)lv.blocks32, (void*)lv.yblk64, (void*)lv.yblk32}) {
            if (!p) continue;
            for (size_t i = 0; i < h->allocs.size(); ++i)
                if (h->allocs[i] == p) {
                    (void)hipFree(p);
                    h->allocs.erase(h->allocs.begin() + i);
                    break;
                }
        }
        const int M = 4 * h->cfg.ncomp;
        const int64_t freed = (lv.blocks64 ? lv.nblk * M * M * (int64_t)sizeof(double) : 0) +
                              (lv.blocks32 ? lv.nblk * M * M * (int64_t)sizeof(float) : 0) +
                              (lv.yblk64 ? lv.nblk * M * (int64_t)sizeof(double) : 0) +
                              (lv.yblk32 ? lv.nblk * M * (int64_t)sizeof(float) : 0);
        h->bytes -= freed;
        lv.bytes -= freed;
        lv.blocks64 = nullptr;
        lv.blocks32 = nullptr;
        lv.yblk64 = nullptr;
        lv.yblk32 = nullptr;
        lv.nflag = 0;
        lv.nblk = 0;
    }
    return AGCA_OK;
}

}  // namespace

// ===========================================================================
// ABI
// ===========================================================================
extern "C" {

const char* agca_last_error(void) { return g_err.c_str(); }

int32_t agca_macro_gradient(int32_t L, const double* eta_nodes, double* gmax, void* stream) {
    if (L < 1 || L > 9) return fail(AGCA_E_INVALID, "L must be in [1, 9]");
    if (!eta_nodes || !gmax) return fail(AGCA_E_INVALID, "null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long* d = nullptr;
    if (hipMalloc((void**)&d, 48 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(AGCA_E_OOM, "hipMalloc failed");
    }
    unsigned long long bits[48];
    hipError_t e = hipMemsetAsync(d, 0, sizeof(bits), st);
    if (e == hipSuccess) e = launch_macro_grad_max(L, eta_nodes, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bits, d, sizeof(bits), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(AGCA_E_HIP, std::string("macro gradient: ") + hipGetErrorString(e));
    for (int k = 0; k < 48; ++k) {
        double v;
        std::memcpy(&v, &bits[k], sizeof(v));
        if (!std::isfinite(v)) return fail(AGCA_E_INVALID, "non-finite nodal values");
        gmax[k] = v;
    }
    return AGCA_OK;
}

}  // extern "C"

// Scratch of agca_macro_gradient_noalloc: one 64-bit slot per macro element (the bit
// pattern of a non-negative double, so an unsigned atomic maximum orders the values),
// in a file-scope device array instead of a per-call allocation.  Each GPU holds its own
// copy, at its own address, until the process ends; host code uses the address from
// hipGetSymbolAddress, never the array's name (in host code the name is a host-side
// stand-in).  Every call on a GPU shares that GPU's copy.
static constexpr int kMacroScratchSlots = 48;
static __device__ __align__(256) unsigned long long scratch[kMacroScratchSlots];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device, looked up once per device
int32_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(AGCA_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(AGCA_E_INVALID, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(AGCA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return AGCA_OK;
}
}  // namespace

extern "C" {

int32_t agca_macro_gradient_noalloc(int32_t L, const double* eta_nodes, double* gmax, void* stream) {
    if (L < 1 || L > 9) return fail(AGCA_E_INVALID, "L must be in [1, 9]");
    if (!eta_nodes || !gmax) return fail(AGCA_E_INVALID, "null pointer");
    static_assert(kMacroScratchSlots >= 48, "one scratch slot per macro element");
    void* ptr = nullptr;
    TRY(scratch_address(&ptr));
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long* slots = static_cast<unsigned long long*>(ptr);
    unsigned long long bits[48];
    // the slots keep the previous call's maxima: clear them with a fill kernel (all-zero
    // bits are the double 0.0, below every norm)
    hipError_t e = launch_fill<double>(48, 0.0, static_cast<double*>(ptr), st);
    if (e == hipSuccess) e = launch_macro_grad_max(L, eta_nodes, slots, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bits, slots, sizeof(bits), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return fail(AGCA_E_HIP, std::string("macro gradient (no allocation): ") + hipGetErrorString(e));
    for (int k = 0; k < 48; ++k) {
        double v;
        std::memcpy(&v, &bits[k], sizeof(v));
        if (!std::isfinite(v)) return fail(AGCA_E_INVALID, "non-finite nodal values");
        gmax[k] = v;
    }
    return AGCA_OK;
}

void agca_default_config(agca_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->L = 3;
    c->ncomp = 1;
    c->flag_mode = AGCA_FLAG_RATIO;
    c->mg_dtype = AGCA_F64;
    c->mg_nu_dtype = AGCA_F64;
    c->pre_sweeps = 2;
    c->post_sweeps = 2;
    c->flag_ratio = 10.0;
    c->omega = 2.0 / 3.0;
    c->mem_limit_bytes = 0;
}

int32_t agca_validate_config(const agca_config* cfg) { return validate(cfg); }

int32_t agca_create(const agca_config* cfg, const double* nu_fine, const double* const* nu_coarse,
                    void* stream, agca_hier** out) {
    if (!out) return fail(AGCA_E_INVALID, "null output handle");
    *out = nullptr;
    TRY(validate(cfg));
    if (!nu_fine || !nu_coarse) return fail(AGCA_E_INVALID, "null coefficient pointer");
    agca_hier* h = new agca_hier();
    h->cfg = *cfg;
    h->st = static_cast<hipStream_t>(stream);
    const int L = cfg->L, nc = cfg->ncomp;
    const size_t ts = mg_size(h);
    auto bail = [&](int32_t rc) {
        std::string msg = g_err;
        free_all(h);
        delete h;
        g_err = msg;
        return rc;
    };
    h->lv.resize(L + 1);
    int32_t rc = AGCA_OK;
    for (int l = 0; l <= L && rc == AGCA_OK; ++l) {
        Level& lv = h->lv[l];
        lv.n = 1 << (l + 1);
        lv.nodes = nodes_of(lv.n);
        lv.elems = elems_of(lv.n);
        const int64_t nv = (int64_t)nc * lv.nodes;
        rc = alloc_t(h, &lv.nu64, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && mg32(h) && !(l == L && cfg->mg_nu_dtype == AGCA_BF16))
            rc = alloc_t(h, &lv.nu32, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && mg32(h) && l == L && cfg->mg_nu_dtype == AGCA_BF16)
            rc = alloc_t(h, &lv.nubf, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && l < L) rc = alloc_t(h, &lv.flag, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && l < L) rc = alloc_t(h, &lv.blk, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && l < L) rc = alloc_t(h, &lv.blk_soa, lv.elems, &lv.bytes);
        if (rc == AGCA_OK && l < L) rc = alloc_t(h, &lv.ids, lv.elems, &lv.bytes);
        if (rc == AGCA_OK) rc = alloc_t(h, &lv.diag, nv, &lv.bytes);
        if (rc == AGCA_OK && mg32(h)) rc = alloc_t(h, &lv.dinv32, nv, &lv.bytes);
        if (rc == AGCA_OK && !mg32(h)) rc = alloc_t(h, &lv.dinv64, nv, &lv.bytes);
        if (rc == AGCA_OK && l >= 1 && l < L && lv.n <= stencil_max_n()) {
            rc = alloc_t(h, &lv.sten64, (size_t)nv * nc * 15, &lv.bytes);
            if (rc == AGCA_OK && mg32(h)) rc = alloc_t(h, &lv.sten32, (size_t)nv * nc * 15, &lv.bytes);
        }
        if (rc == AGCA_OK && l < L) rc = dev_alloc(h, &lv.b, nv * ts, &lv.bytes);
        if (rc == AGCA_OK && l < L) rc = dev_alloc(h, &lv.x, nv * ts, &lv.bytes);
        if (rc == AGCA_OK && l > 0) rc = dev_alloc(h, &lv.t, nv * ts, &lv.bytes);
        if (rc == AGCA_OK && l > 0) rc = dev_alloc(h, &lv.r, nv * ts, &lv.bytes);
    }
    if (rc == AGCA_OK) rc = alloc_t(h, &h->ainv0, 9);
    if (rc == AGCA_OK) {
        h->partial_cap = std::max(2 * h->nb_partial, cube_grid_blocks(h->lv[L].n));
        rc = alloc_t(h, &h->partial, h->partial_cap);
    }
    if (rc == AGCA_OK) rc = alloc_t(h, &h->red, AGCA_RED_SLOTS);
    if (rc == AGCA_OK) rc = alloc_t(h, &h->counter, 4);
    if (rc == AGCA_OK) {
        hipError_t e = hipHostMalloc((void**)&h->red_host, AGCA_RED_SLOTS * sizeof(double));
        if (e != hipSuccess) rc = fail(AGCA_E_OOM, "hipHostMalloc failed");
    }
    if (rc != AGCA_OK) return bail(rc);
    rc = build_operators(h, nu_fine, nu_coarse);
    if (rc != AGCA_OK) return bail(rc);
    *out = h;
    return AGCA_OK;
}

int32_t agca_destroy(agca_hier* h) {
    if (!h) return AGCA_OK;
    free_all(h);
    delete h;
    return AGCA_OK;
}

int32_t agca_set_nu(agca_hier* h, const double* nu_fine, const double* const* nu_coarse) {
    TRY(check_level(h, 0));
    if (!nu_fine || !nu_coarse) return fail(AGCA_E_INVALID, "null coefficient pointer");
    HIPCHK(h, hipStreamSynchronize(h->st));
    free_blocks(h);
    return build_operators(h, nu_fine, nu_coarse);
}

int32_t agca_set_log_nu(agca_hier* h, const double* log_nu_fine, const double* const* nu_coarse) {
    TRY(check_level(h, 0));
    if (!log_nu_fine || !nu_coarse) return fail(AGCA_E_INVALID, "null coefficient pointer");
    HIPCHK(h, hipStreamSynchronize(h->st));
    free_blocks(h);
    return build_operators(h, log_nu_fine, nu_coarse, true);
}

int32_t agca_query(const agca_hier* h, int32_t level, agca_level_info* out) {
    TRY(check_level(h, level));
    if (!out) return fail(AGCA_E_INVALID, "null output");
    const Level& lv = h->lv[level];
    const int M = 4 * h->cfg.ncomp;
    out->n = lv.n;
    out->nodes = lv.nodes;
    out->free_nodes = (int64_t)(lv.n - 1) * (lv.n - 1) * (lv.n - 1);
    out->elements = lv.elems;
    out->flagged = level < h->cfg.L ? lv.nflag : 0;
    out->block_bytes = (lv.blocks64 ? lv.nblk * M * M * 8 : 0) + (lv.blocks32 ? lv.nblk * M * M * 4 : 0);
    out->level_bytes = lv.bytes;
    out->lambda_max = (size_t)level < h->lam.size() ? h->lam[level] : 0.0;
    return AGCA_OK;
}

int32_t agca_get_flags(const agca_hier* h, int32_t level, int32_t* ids_host, int64_t cap, int64_t* n) {
    TRY(check_level(h, level));
    if (level >= h->cfg.L) return fail(AGCA_E_INVALID, "the finest level has no flags");
    const Level& lv = h->lv[level];
    if (n) *n = lv.nflag;
    if (cap < lv.nflag || (!ids_host && lv.nflag > 0)) return fail(AGCA_E_INVALID, "ids buffer too small");
    agca_hier* hh = const_cast<agca_hier*>(h);
    if (lv.nflag > 0) {
        HIPCHK(hh, hipMemcpyAsync(ids_host, lv.ids, lv.nflag * sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hh, hipStreamSynchronize(h->st));
    }
    return AGCA_OK;
}

int32_t agca_get_blocks(const agca_hier* h, int32_t level, double* blocks_host, int64_t cap) {
    TRY(check_level(h, level));
    if (level >= h->cfg.L) return fail(AGCA_E_INVALID, "the finest level has no blocks");
    const Level& lv = h->lv[level];
    const int M = 4 * h->cfg.ncomp;
    if (h->cfg.coarse_storage == AGCA_STORE_MEAN && lv.nflag > 0)
        return fail(AGCA_E_INVALID, "no stored blocks: the hierarchy keeps the descendant mean instead");
    if (cap < lv.nblk * M * M) return fail(AGCA_E_INVALID, "blocks buffer too small");
    agca_hier* hh = const_cast<agca_hier*>(h);
    if (lv.nblk > 0) {
        HIPCHK(hh, hipMemcpyAsync(blocks_host, lv.blocks64, lv.nblk * M * M * sizeof(double),
                                  hipMemcpyDeviceToHost, h->st));
        HIPCHK(hh, hipStreamSynchronize(h->st));
    }
    return AGCA_OK;
}

int32_t agca_get_diagonal(const agca_hier* h, int32_t level, double* diag_host, int64_t cap) {
    TRY(check_level(h, level));
    const Level& lv = h->lv[level];
    const int64_t cnt = (int64_t)h->cfg.ncomp * lv.nodes;
    if (cap < cnt || !diag_host) return fail(AGCA_E_INVALID, "diagonal buffer too small");
    agca_hier* hh = const_cast<agca_hier*>(h);
    HIPCHK(hh, hipMemcpyAsync(diag_host, lv.diag, cnt * sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hh, hipStreamSynchronize(h->st));
    return AGCA_OK;
}

int32_t agca_apply(agca_hier* h, int32_t level, int32_t dtype, const void* u, void* v) {
    TRY(check_level(h, level));
    TRY(check_dtype(h, dtype, false));
    if (!u || !v || u == v) return fail(AGCA_E_INVALID, "u and v must be distinct non-null vectors");
    if (dtype == AGCA_F64)
        return do_cube<double>(h, level, MODE_APPLY, (const double*)u, nullptr, (double*)v, 0.0);
    return do_cube<float>(h, level, MODE_APPLY, (const float*)u, nullptr, (float*)v, 0.0f);
}

int32_t agca_residual(agca_hier* h, int32_t level, int32_t dtype, const void* b, const void* x, void* r) {
    TRY(check_level(h, level));
    TRY(check_dtype(h, dtype, false));
    if (!b || !x || !r || r == x) return fail(AGCA_E_INVALID, "bad vector pointers");
    if (dtype == AGCA_F64)
        return do_cube<double>(h, level, MODE_RESIDUAL, (const double*)x, (const double*)b, (double*)r, 0.0);
    return do_cube<float>(h, level, MODE_RESIDUAL, (const float*)x, (const float*)b, (float*)r, 0.0f);
}

int32_t agca_smooth(agca_hier* h, int32_t level, int32_t dtype, int32_t sweeps, double omega,
                    const void* b, void* x) {
    TRY(check_level(h, level));
    TRY(check_dtype(h, dtype, true));
    if (level == 0) return fail(AGCA_E_INVALID, "level 0 is solved directly");
    if (!b || !x || b == x) return fail(AGCA_E_INVALID, "bad vector pointers");
    if (sweeps < 0) return fail(AGCA_E_INVALID, "sweeps must be >= 0");
    if (dtype == AGCA_F64) return do_smooth<double>(h, level, sweeps, omega, (const double*)b, (double*)x);
    return do_smooth<float>(h, level, sweeps, omega, (const float*)b, (float*)x);
}

int32_t agca_restrict(agca_hier* h, int32_t fine_level, int32_t dtype, const void* r_f, void* r_c) {
    TRY(check_level(h, fine_level));
    TRY(check_dtype(h, dtype, false));
    if (fine_level == 0) return fail(AGCA_E_INVALID, "level 0 has no coarser level");
    if (!r_f || !r_c) return fail(AGCA_E_INVALID, "null vector");
    if (dtype == AGCA_F64)
        HIPCHK(h, launch_restrict<double>(h->cfg.ncomp, h->lv[fine_level].n, (const double*)r_f, (double*)r_c, h->st));
    else
        HIPCHK(h, launch_restrict<float>(h->cfg.ncomp, h->lv[fine_level].n, (const float*)r_f, (float*)r_c, h->st));
    return AGCA_OK;
}

int32_t agca_prolong_add(agca_hier* h, int32_t coarse_level, int32_t dtype, const void* e_c, void* x_f) {
    TRY(check_level(h, coarse_level));
    TRY(check_dtype(h, dtype, false));
    if (coarse_level >= h->cfg.L) return fail(AGCA_E_INVALID, "no finer level");
    if (!e_c || !x_f) return fail(AGCA_E_INVALID, "null vector");
    const int nf = h->lv[coarse_level + 1].n;
    if (dtype == AGCA_F64)
        HIPCHK(h, launch_prolong_add<double>(h->cfg.ncomp, nf, (const double*)e_c, (double*)x_f, h->st));
    else
        HIPCHK(h, launch_prolong_add<float>(h->cfg.ncomp, nf, (const float*)e_c, (float*)x_f, h->st));
    return AGCA_OK;
}

int32_t agca_vcycle(agca_hier* h, int32_t dtype, const void* b, void* x) {
    TRY(check_level(h, 0));
    TRY(check_dtype(h, dtype, true));
    if (!b || !x || b == x) return fail(AGCA_E_INVALID, "bad vector pointers");
    if (dtype == AGCA_F64) return do_vcycle<double>(h, (const double*)b, (double*)x);
    return do_vcycle<float>(h, (const float*)b, (float*)x);
}

int32_t agca_dot(agca_hier* h, int32_t level, int32_t dtype, const void* x, const void* y, double* out) {
    TRY(check_level(h, level));
    TRY(check_dtype(h, dtype, false));
    if (!x || !y || !out) return fail(AGCA_E_INVALID, "null pointer");
    const int64_t cnt = (int64_t)h->cfg.ncomp * h->lv[level].nodes;
    if (dtype == AGCA_F64) return do_dot<double>(h, (const double*)x, (const double*)y, cnt, out);
    return do_dot<float>(h, (const float*)x, (const float*)y, cnt, out);
}

int32_t agca_cast(agca_hier* h, int32_t from, int32_t to, const void* src, void* dst, int64_t count) {
    TRY(check_level(h, 0));
    const bool ok = (from == AGCA_F64 && (to == AGCA_F32 || to == AGCA_BF16 || to == AGCA_F64)) ||
                    (from == AGCA_F32 && (to == AGCA_F64 || to == AGCA_F32));
    if (!ok) return fail(AGCA_E_INVALID, "unsupported conversion");
    if (count < 0 || (count > 0 && (!src || !dst))) return fail(AGCA_E_INVALID, "bad buffers");
    if (count == 0) return AGCA_OK;
    HIPCHK(h, launch_cast(from, to, src, dst, count, h->st));
    return AGCA_OK;
}

int64_t agca_device_bytes(const agca_hier* h) { return h ? h->bytes : 0; }

int32_t agca_residual_floor(agca_hier* h, const double* b, const double* x, double* rho) {
    TRY(check_level(h, 0));
    if (!b || !x || !rho) return fail(AGCA_E_INVALID, "null pointer");
    return residual_floor(h, b, x, rho);
}

int32_t agca_grad_log_nu(agca_hier* h, const double* u, const double* w, double* g) {
    TRY(check_level(h, 0));
    if (!u || !w || !g) return fail(AGCA_E_INVALID, "null pointer");
    const Level& lv = h->lv[h->cfg.L];
    HIPCHK(h, launch_grad(h->cfg.ncomp, lv.n, lv.nu64, 1.0 / (6.0 * lv.n), u, w, g, h->st));
    return AGCA_OK;
}

int32_t agca_load_vector(agca_hier* h, const double* f, double* b) {
    TRY(check_level(h, 0));
    if (!f || !b) return fail(AGCA_E_INVALID, "null pointer");
    const Level& lv = h->lv[h->cfg.L];
    const double hh = 1.0 / lv.n;
    HIPCHK(h, launch_load_vector(h->cfg.ncomp, lv.n, f, hh * hh * hh / 6.0 / 4.0, b, h->st));
    return AGCA_OK;
}

// ---------------------------------------------------------------------------
// solvers
// ---------------------------------------------------------------------------

// z = B r with the hierarchy's V-cycle (FP32 V-cycle: cast in and out)
static int32_t precondition(agca_hier* h, const double* r, double* z) {
    if (!mg32(h)) return do_vcycle<double>(h, r, z);
    const int64_t cnt = (int64_t)h->cfg.ncomp * h->lv[h->cfg.L].nodes;
    HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, r, h->s_r32, cnt, h->st));
    TRY(do_vcycle<float>(h, h->s_r32, h->s_z32));
    HIPCHK(h, launch_cast(AGCA_F32, AGCA_F64, h->s_z32, z, cnt, h->st));
    return AGCA_OK;
}

// Residual replacement and the stopping rule of the Krylov solvers.  The recurrence's
// residual drifts away from the true residual b - A x by the rounding of every update,
// so the true residual replaces it whenever the recurrence has halved since the last
// replacement (kReplaceEvery; the search direction is kept, no restart: van der Vorst
// and Ye, SIAM J. Sci. Comput. 22, 2000), and when it reaches tol.  The iteration
// continues while the true residual is above tol and keeps improving; it ends at the
// rounding floor (floor_limited) only under the rule of stop_rule.h (the true residual
// stopped improving and is at most kFloorFactor max(tol, rho), rho the rounding
// floor of the iterate, residual_floor).  A stall above that is AGCA_E_NOCONV.  A
// replacement costs one residual pass and one dot product, against an apply, a
// V-cycle and three vector passes per iteration.

int32_t agca_solve(agca_hier* h, const agca_solve_opts* o, const double* b, double* x,
                   agca_solve_stats* stats) {
    TRY(check_level(h, 0));
    if (!o || !b || !x || !stats) return fail(AGCA_E_INVALID, "null pointer");
    if (o->max_iter < 0 || !(o->tol >= 0.0)) return fail(AGCA_E_INVALID, "bad solve options");
    if (o->solver < AGCA_SOLVER_PCG || o->solver > AGCA_SOLVER_STATIONARY)
        return fail(AGCA_E_INVALID, "unknown solver");
    if (o->n_milestones < 0 || o->n_milestones > AGCA_MAX_MILESTONES)
        return fail(AGCA_E_INVALID, "n_milestones must be in [0, " + std::to_string(AGCA_MAX_MILESTONES) + "]");
    for (int i = 0; i < o->n_milestones; ++i)
        if (!(o->milestones[i] > 0.0) || !std::isfinite(o->milestones[i]))
            return fail(AGCA_E_INVALID, "milestones must be finite and positive");
    TRY(ensure_solver_vectors(h));
    std::memset(stats, 0, sizeof(*stats));
    for (int i = 0; i < AGCA_MAX_MILESTONES; ++i) stats->milestone_iterations[i] = -1;
    const int L = h->cfg.L;
    const int64_t cnt = (int64_t)h->cfg.ncomp * h->lv[L].nodes;
    double *r = h->s_r, *z = h->s_z, *p = h->s_p, *q = h->s_q;
    auto t0 = std::chrono::steady_clock::now();
    if (!o->use_x0) HIPCHK(h, launch_fill<double>(cnt, 0.0, x, h->st));
    HIPCHK(h, launch_zero_boundary<double>(h->cfg.ncomp, h->lv[L].n, x, h->st));
    double bn = 0.0;
    TRY(interior_norm(h, b, &bn));
    if (!std::isfinite(bn)) return fail(AGCA_E_NUMERIC, "non-finite right-hand side");
    TRY(do_cube<double>(h, L, MODE_RESIDUAL, x, b, r, 0.0));
    double rr = 0.0;
    TRY(do_dot<double>(h, r, r, cnt, &rr));
    double rel = bn > 0 ? std::sqrt(rr) / bn : 0.0;
    int hist_n = 0;
    auto record = [&](double v) {
        if (o->record_history && hist_n < AGCA_MAX_HISTORY) stats->history[hist_n++] = v;
    };
    record(rel);
    int it = 0, replacements = 0;
    bool floor_limited = false, stalled = false;
    EndChecks ends;
    double rho = -1.0;  // formed at the first stall
    int32_t status = AGCA_OK;
    double rec_rel = rel;
    // milestones: record the first iteration whose verified true residual is below each
    auto note_milestones = [&](double rel_true) {
        for (int i = 0; i < o->n_milestones; ++i)
            if (stats->milestone_iterations[i] < 0 && rel_true <= o->milestones[i]) {
                stats->milestone_iterations[i] = it;
                stats->milestone_seconds[i] =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                stats->milestone_residuals[i] = rel_true;
            }
    };
    auto milestone_due = [&](double rec) {
        for (int i = 0; i < o->n_milestones; ++i)
            if (stats->milestone_iterations[i] < 0 && rec <= o->milestones[i]) return true;
        return false;
    };
    note_milestones(rel);
    if (bn == 0.0) {
        HIPCHK(h, launch_fill<double>(cnt, 0.0, x, h->st));
        rel = rec_rel = 0.0;
    } else if (rel > o->tol) {
        if (o->solver == AGCA_SOLVER_PCG || o->solver == AGCA_SOLVER_FCG) {
            // One loop for both: PCG around the FP64 V-cycle and FCG(1) around the FP32
            // one.  FCG(1): beta = z_k . (r_k - r_{k-1}) / (z_{k-1} . r_{k-1}), formed as
            // -alpha z_k . q_{k-1} / (z_{k-1} . r_{k-1}) = -z_k . q_{k-1} / (p_{k-1} . q_{k-1})
            // since r_k - r_{k-1} = -alpha q_{k-1} (no copy of the old residual).  With a
            // fixed SPD preconditioner (PCG) this equals z_k . r_k / (z_{k-1} . r_{k-1}) in
            // exact arithmetic (z_k . r_{k-1} = 0).  With the FP32 V-cycle the residual update
            // also writes the V-cycle's FP32 input, and z stays in FP32: the dot products
            // and the direction update widen it on the fly.
            const bool mixed = mg32(h);
            float *r32 = h->s_r32, *z32 = h->s_z32;
            auto vcycle = [&]() -> int32_t {
                return mixed ? do_vcycle<float>(h, r32, z32) : do_vcycle<double>(h, r, z);
            };
            auto dots = [&](const double* qq) -> hipError_t {
                return mixed ? launch_dot2<float>(cnt, z32, r, qq, h->partial, h->nb_partial, h->st)
                             : launch_dot2<double>(cnt, z, r, qq, h->partial, h->nb_partial, h->st);
            };
            auto direction = [&](double beta) -> hipError_t {
                return mixed ? launch_zpbp<float>(cnt, z32, beta, p, h->st)
                             : launch_zpbp<double>(cnt, z, beta, p, h->st);
            };
            // The scalars stay in reduction slots on the device (alpha = rz / pq and beta are
            // formed by the kernels that use them); the host reads p.q, r.r and z.r once per
            // iteration for the stopping test and the breakdown checks.
            auto direction_dev = [&](const double* num, const double* den, double sign) -> hipError_t {
                return mixed ? launch_zpbp_dev<float>(cnt, z32, num, den, sign, p, h->st)
                             : launch_zpbp_dev<double>(cnt, z, num, den, sign, p, h->st);
            };
            constexpr int PQ = 0, RR = 1, ZR = 2, ZQ = 3, RZ = 4;
            double* red = h->red;
            double tmp[5];
            double anchor = rel;  // true residual at the last replacement
            if (mixed) HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, r, r32, cnt, h->st));
            TRY(vcycle());
            HIPCHK(h, dots(nullptr));
            TRY(reduce_to(h, h->partial, h->nb_partial, RZ));
            HIPCHK(h, direction(0.0));
            while (it < o->max_iter) {
                // q = A p fused with p . q
                int nbq = 0;
                HIPCHK(h, launch_cube_dot(h->cfg.ncomp, level_op<double>(h, L), p, q, h->partial, &nbq,
                                          h->st));
                TRY(reduce_to(h, h->partial, nbq, PQ));
                // x += alpha p, r -= alpha q (and its FP32 copy), fused with r . r
                HIPCHK(h, launch_cg_update(cnt, red + RZ, red + PQ, p, q, x, r, mixed ? r32 : nullptr,
                                           h->partial, h->nb_partial, h->st));
                TRY(reduce_to(h, h->partial, h->nb_partial, RR));
                TRY(fetch(h, 5, tmp));
                if (!(tmp[RZ] > 0.0) || !std::isfinite(tmp[RZ])) {
                    status = fail(AGCA_E_NUMERIC, "preconditioned residual is not positive");
                    break;
                }
                if (!(tmp[PQ] > 0.0) || !std::isfinite(tmp[PQ])) {
                    status = fail(AGCA_E_NUMERIC, "search direction has non-positive energy");
                    break;
                }
                rr = tmp[RR];
                ++it;
                rel = rec_rel = std::sqrt(rr) / bn;
                record(rel);
                if (!std::isfinite(rel) || rel > 1e30) {
                    status = fail(AGCA_E_NUMERIC, "residual diverged");
                    break;
                }
                const bool full = rel <= kReplaceEvery * anchor;
                if (rel <= o->tol || full || milestone_due(rel)) {
                    // residual replacement: r = b - A x (and its FP32 copy); r . r goes to a
                    // slot of its own (FCG's next beta still reads p . q from slot PQ)
                    TRY(do_cube<double>(h, L, MODE_RESIDUAL, x, b, r, 0.0));
                    TRY(do_dot<double>(h, r, r, cnt, &rr, kSlotReplace));
                    if (mixed) HIPCHK(h, launch_cast(AGCA_F64, AGCA_F32, r, r32, cnt, h->st));
                    const double rel_true = std::sqrt(rr) / bn;
                    ++replacements;
                    anchor = rel_true;
                    note_milestones(rel_true);
                    if (rel_true <= o->tol) {
                        rel = rel_true;
                        break;
                    }
                    if (ends.stagnated(rel_true, it, full)) {
                        // the floor of x changes little once the solve has stalled: formed once
                        if (rho < 0.0) TRY(residual_floor(h, b, x, &rho));
                        if (at_floor(rel_true, o->tol, rho) || ends.given_up()) {
                            rel = rel_true;
                            floor_limited = at_floor(rel_true, o->tol, rho);
                            stalled = !floor_limited;
                            break;
                        }
                    }
                    rel = rec_rel = rel_true;
                }
                TRY(vcycle());
                // The new direction is A-orthogonalised against the previous one, beta =
                // -z.q / p.q, in both solvers: for PCG (fixed SPD preconditioner) that equals
                // z.r / rz_old in exact arithmetic, but the latter takes r orthogonal to the
                // previous direction, which a replaced residual near the rounding floor is
                // not; with it PCG stalled above the floor (513^3 sinkers: 1.3e-6 against a
                // floor of 7.3e-7, where the A-orthogonal form reaches 1.9e-7)
                // z . r and z . q in one pass
                HIPCHK(h, dots(q));
                TRY(reduce_to(h, h->partial, h->nb_partial, ZR));
                TRY(reduce_to(h, h->partial + h->nb_partial, h->nb_partial, ZQ));
                // beta = -alpha z.q / rz_old = -z.q / p.q
                HIPCHK(h, direction_dev(red + ZQ, red + PQ, -1.0));
                HIPCHK(h, hipMemcpyAsync(red + RZ, red + ZR, sizeof(double), hipMemcpyDeviceToDevice, h->st));
            }
        } else {
            // iterative refinement / stationary: x += B r, r = b - A x (the residual is exact)
            while (it < o->max_iter) {
                TRY(precondition(h, r, z));
                HIPCHK(h, launch_axpby<double>(cnt, 1.0, z, 1.0, x, h->st));
                TRY(do_cube<double>(h, L, MODE_RESIDUAL, x, b, r, 0.0));
                ++it;
                TRY(do_dot<double>(h, r, r, cnt, &rr));
                rel = rec_rel = std::sqrt(rr) / bn;
                record(rel);
                note_milestones(rel);
                if (!std::isfinite(rel) || rel > 1e30) {
                    status = fail(AGCA_E_NUMERIC, "residual diverged");
                    break;
                }
                if (rel <= o->tol) break;
            }
        }
    }
    // final FP64 residual with FP64 coefficients, and the rounding floor of x
    TRY(do_cube<double>(h, L, MODE_RESIDUAL, x, b, r, 0.0));
    TRY(do_dot<double>(h, r, r, cnt, &rr));
    stats->rel_residual = bn > 0 ? std::sqrt(rr) / bn : 0.0;
    rho = 0.0;
    if (bn > 0) TRY(residual_floor(h, b, x, &rho));
    stats->floor_estimate = rho;
    stats->recursive_rel_residual = rec_rel;
    stats->iterations = it;
    stats->replacements = replacements;
    stats->converged = stats->rel_residual <= o->tol || bn == 0.0;
    stats->floor_limited = (!stats->converged && floor_limited && at_floor(stats->rel_residual, o->tol, rho)) ? 1 : 0;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status != AGCA_OK) return status;
    if (stalled && !stats->converged)
        return fail(AGCA_E_NOCONV, "the true residual stalled above " + std::to_string(kFloorFactor) +
                                       " x max(tol, rounding floor)");
    if (!stats->converged && !stats->floor_limited)
        return fail(AGCA_E_NOCONV, "no convergence within max_iter");
    return AGCA_OK;
}

// ---------------------------------------------------------------------------
// Stokes: K = [[A, B^T], [B, 0]], velocity on level L (this hierarchy's operator),
// pressure on every node of level L-1.  Krylov vectors are contiguous [u | p].
// ---------------------------------------------------------------------------
struct StokesDims {
    int64_t nu = 0, np = 0, tot = 0;
    int nf = 0, nc = 0;
};

static StokesDims stokes_dims(const agca_hier* h) {
    StokesDims d;
    const int L = h->cfg.L;
    d.nf = h->lv[L].n;
    d.nc = h->lv[L - 1].n;
    d.nu = 3 * h->lv[L].nodes;
    d.np = h->lv[L - 1].nodes;
    d.tot = d.nu + d.np;
    return d;
}

static int32_t stokes_ready(agca_hier* h) {
    TRY(check_level(h, 0));
    if (h->cfg.ncomp != 3) return fail(AGCA_E_INVALID, "Stokes needs the vector hierarchy (ncomp = 3)");
    if (h->cfg.L < 2) return fail(AGCA_E_INVALID, "Stokes needs L >= 2");
    const StokesDims d = stokes_dims(h);
    if (!h->st_mass) {
        TRY(alloc_t(h, &h->st_mass, (size_t)d.np));
        TRY(alloc_t(h, &h->st_pf, (size_t)h->lv[h->cfg.L].nodes));
        TRY(alloc_t(h, &h->st_qf, (size_t)h->lv[h->cfg.L].nodes));
    }
    if (h->mass_version != h->nu_version) {
        HIPCHK(h, launch_stokes_mass_fine(d.nf, h->lv[h->cfg.L].nu64, h->st_qf, h->st));
        HIPCHK(h, launch_restrict_all(d.nc, h->st_qf, h->st_mass, h->st));
        h->mass_version = h->nu_version;
    }
    return AGCA_OK;
}

static int32_t stokes_work(agca_hier* h, int64_t vecs) {
    if (h->st_work_vecs >= vecs) return AGCA_OK;
    if (h->st_work) {
        for (size_t i = 0; i < h->allocs.size(); ++i)
            if (h->allocs[i] == h->st_work) {
                (void)hipFree(h->st_work);
                h->allocs.erase(h->allocs.begin() + i);
                h->bytes -= h->st_work_vecs * stokes_dims(h).tot * (int64_t)sizeof(double);
                break;
            }
        h->st_work = nullptr;
        h->st_work_vecs = 0;
    }
    TRY(alloc_t(h, &h->st_work, (size_t)(vecs * stokes_dims(h).tot)));
    h->st_work_vecs = vecs;
    return AGCA_OK;
}

// q (pressure) = B u
static int32_t stokes_div(agca_hier* h, const double* u, double* q) {
    const StokesDims d = stokes_dims(h);
    HIPCHK(h, launch_stokes_div_fine(d.nf, u, h->st_qf, h->st));
    HIPCHK(h, launch_restrict_all(d.nc, h->st_qf, q, h->st));
    return AGCA_OK;
}
// v (velocity) += B^T p
static int32_t stokes_grad_add(agca_hier* h, const double* p, double* v) {
    const StokesDims d = stokes_dims(h);
    HIPCHK(h, launch_prolong_all(d.nf, p, h->st_pf, h->st));
    HIPCHK(h, launch_stokes_grad_fine_add(d.nf, h->st_pf, v, h->st));
    return AGCA_OK;
}
// y = K x
static int32_t stokes_apply(agca_hier* h, const double* x, double* y) {
    const StokesDims d = stokes_dims(h);
    TRY(do_cube<double>(h, h->cfg.L, MODE_APPLY, x, nullptr, y, 0.0));
    TRY(stokes_grad_add(h, x + d.nu, y));
    TRY(stokes_div(h, x, y + d.nu));
    return AGCA_OK;
}
// ---------------------------------------------------------------------------
// diag(A)-BFBT Schur approximation (eq. (4.2)): S^-1 = Z^-1 (B W^-1 A W^-1 B^T) Z^-1,
// W = diag(A) on the free velocity dofs, Z = B W^-1 B^T on the pressure nodes.  Z has
// the constant pressure in its kernel; Z^-1 is a fixed number of Jacobi-preconditioned
// CG steps from zero (the paper uses an algebraic multigrid cycle there).
// ---------------------------------------------------------------------------
struct Bfbt {
    double *winv, *v1, *v2;                            // velocity vectors
    double *zdiag, *y1, *y2, *zr, *zz, *zp, *zq, *ztmp;  // pressure vectors
    double* zred;                                      // CG scalars (device)
};
static Bfbt bfbt_bufs(agca_hier* h) {
    const StokesDims d = stokes_dims(h);
    Bfbt w;
    double* p = h->st_bfbt;
    for (double** v : {&w.winv, &w.v1, &w.v2}) { *v = p; p += d.nu; }
    for (double** v : {&w.zdiag, &w.y1, &w.y2, &w.zr, &w.zz, &w.zp, &w.zq, &w.ztmp}) { *v = p; p += d.np; }
    w.zred = p;
    return w;
}
// out = Z y = B (W^-1 (B^T y))
static int32_t z_apply(agca_hier* h, const Bfbt& w, const double* y, double* out) {
    const StokesDims d = stokes_dims(h);
    HIPCHK(h, launch_fill<double>(d.nu, 0.0, w.v1, h->st));
    TRY(stokes_grad_add(h, y, w.v1));
    HIPCHK(h, launch_mul_elementwise(d.nu, w.v1, w.winv, w.v1, h->st));
    TRY(stokes_div(h, w.v1, out));
    return AGCA_OK;
}
// W^-1 (0 on boundary velocity dofs), once per coefficient rebuild, and with `diag`
// diag(Z) as well.  Two pressure nodes of one colour (coordinates equal mod 3) are at
// least 3 pressure cells apart, while B^T e_k lives on the velocity nodes within one
// pressure cell of node k: Z_km = 0 for distinct k, m of one colour, so Z applied to a
// colour's indicator holds Z_kk on that colour's nodes.
static int32_t bfbt_ready(agca_hier* h, bool diag) {
    const StokesDims d = stokes_dims(h);
    if (!h->st_bfbt) TRY(alloc_t(h, &h->st_bfbt, (size_t)(3 * d.nu + 8 * d.np + 8)));
    const Bfbt w = bfbt_bufs(h);
    if (h->bfbt_version != h->nu_version) {
        HIPCHK(h, launch_invert_diag<double>(d.nu, h->lv[h->cfg.L].diag, w.winv, h->st));
        h->bfbt_version = h->nu_version;
    }
    if (!diag || h->zdiag_version == h->nu_version) return AGCA_OK;
    for (int c = 0; c < 27; ++c) {
        HIPCHK(h, launch_colour(d.nc, c, 0, nullptr, w.ztmp, h->st));
        TRY(z_apply(h, w, w.ztmp, w.zq));
        HIPCHK(h, launch_colour(d.nc, c, 1, w.zq, w.zdiag, h->st));
    }
    h->zdiag_version = h->nu_version;
    return AGCA_OK;
}

// ---------------------------------------------------------------------------
// Geometric multigrid for Z on the pressure lattice (the paper solves with Z by an
// algebraic multigrid cycle inside CG): levels L-1 (the pressure space) down to 0 with
// the linear interpolation P over all nodes, Galerkin operators Z_l = P^T Z_{l+1} P
// (the constant pressure stays in every kernel), stored as symmetric 65-offset stencils
// (the centre and 32 offsets per node, zstencil.h) assembled by probing with 65 colours; damped Jacobi V(2,2) cycles,
// omega = 2/3, zero initial guesses, and on level 0 (27 nodes) the minimal-norm
// solution from the bordered system [[Z_0, 1], [1^T, 0]].
// ---------------------------------------------------------------------------
constexpr int kZSweeps = 2;
constexpr double kZOmega = 2.0 / 3.0;

struct ZLevel {
    int n = 0;
    int64_t N = 0;
    double *S = nullptr, *r = nullptr, *y = nullptr, *a = nullptr, *t = nullptr;
};
// levels 0..L-1 carved from st_zmg: per level the stored half of the stencil (33 padded
// arrays, zstencil.h) and four vectors, then the 27 x 27 coarse inverse
static std::vector<ZLevel> zmg_levels(const agca_hier* h, double** coarse = nullptr) {
    std::vector<ZLevel> z(h->cfg.L);
    double* p = h->st_zmg;
    for (int l = 0; l < h->cfg.L; ++l) {
        z[l].n = h->lv[l].n;
        z[l].N = nodes_of(z[l].n);
        z[l].S = p;
        p += (int64_t)kZStored * z_padded_nodes(z[l].n);
        for (double** v : {&z[l].r, &z[l].y, &z[l].a, &z[l].t}) {
            *v = p;
            p += z[l].N;
        }
    }
    if (coarse) *coarse = p;
    return z;
}
static int64_t zmg_doubles(const agca_hier* h) {
    int64_t c = 27 * 27;
    for (int l = 0; l < h->cfg.L; ++l) c += kZStored * z_padded_nodes(h->lv[l].n) + 4 * nodes_of(h->lv[l].n);
    return c;
}

// inverse of the bordered 28 x 28 matrix [[Z0, s 1], [s 1^T, 0]] by Gauss-Jordan
// elimination with partial pivoting; its leading 27 x 27 block maps a zero-sum r to the
// zero-sum solution of Z0 y = r (Z0's kernel is the constants), whatever s > 0: s is
// taken as the largest entry of Z0, so that the border does not dwarf the operator
static bool bordered_inverse(const std::vector<double>& Z0, std::vector<double>& M) {
    constexpr int n = 28;
    double zmax = 0.0;
    for (double v : Z0) zmax = std::max(zmax, std::fabs(v));
    if (!(zmax > 0.0)) return false;
    std::vector<double> A(n * n, 0.0), I(n * n, 0.0);
    for (int i = 0; i < 27; ++i) {
        for (int j = 0; j < 27; ++j) A[i * n + j] = Z0[i * 27 + j];
        A[i * n + 27] = zmax;
        A[27 * n + i] = zmax;
    }
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (!(std::fabs(A[piv * n + c]) > 1e-13 * scale)) return false;
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(A[c * n + j], A[piv * n + j]);
                std::swap(I[c * n + j], I[piv * n + j]);
            }
        const double inv = 1.0 / A[c * n + c];
        for (int j = 0; j < n; ++j) {
            A[c * n + j] *= inv;
            I[c * n + j] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[r * n + j] -= f * A[c * n + j];
                I[r * n + j] -= f * I[c * n + j];
            }
        }
    }
    M.assign(27 * 27, 0.0);
    for (int i = 0; i < 27; ++i)
        for (int j = 0; j < 27; ++j) M[i * 27 + j] = I[i * n + j];
    return true;
}

// assemble every level's stencil, once per coefficient rebuild: the top level probes the
// matrix-free Z = B W^-1 B^T, level l < L-1 probes P^T Z_{l+1} P with Z_{l+1}'s stencil
static int32_t zmg_ready(agca_hier* h) {
    TRY(bfbt_ready(h, false));
    if (!h->st_zmg) TRY(alloc_t(h, &h->st_zmg, (size_t)zmg_doubles(h)));
    if (h->zmg_version == h->nu_version) return AGCA_OK;
    double* coarse = nullptr;
    const std::vector<ZLevel> z = zmg_levels(h, &coarse);
    const int top = h->cfg.L - 1;
    const Bfbt w = bfbt_bufs(h);
    // padding and the entries of neighbours outside the lattice stay 0
    for (int l = 0; l <= top; ++l)
        HIPCHK(h, launch_fill<double>(kZStored * z_padded_nodes(z[l].n), 0.0, z[l].S, h->st));
    for (int c = 0; c < kZColours; ++c) {
        HIPCHK(h, launch_zprobe(z[top].n, c, w.ztmp, h->st));
        TRY(z_apply(h, w, w.ztmp, w.zq));
        HIPCHK(h, launch_zextract(z[top].n, c, w.zq, z[top].S, h->st));
    }
    for (int l = top - 1; l >= 0; --l) {
        const ZLevel &zc = z[l], &zf = z[l + 1];
        for (int c = 0; c < kZColours; ++c) {
            HIPCHK(h, launch_zprobe(zc.n, c, zc.r, h->st));
            HIPCHK(h, launch_prolong_all(zf.n, zc.r, zf.t, h->st));
            HIPCHK(h, launch_zstencil(0, zf.n, zf.S, zf.t, nullptr, 0.0, zf.a, h->st));
            HIPCHK(h, launch_restrict_all(zc.n, zf.a, zc.y, h->st));
            HIPCHK(h, launch_zextract(zc.n, c, zc.y, zc.S, h->st));
        }
    }
    // level 0 (n = 2) as a dense symmetric 27 x 27 matrix from its stored entries
    const int64_t NP0 = z_padded_nodes(2);
    const int P0 = 2 + 1 + 2 * kZPad;
    std::vector<double> S0((size_t)(kZStored * NP0)), Z0(27 * 27, 0.0), M;
    HIPCHK(h, hipMemcpyAsync(S0.data(), z[0].S, sizeof(double) * S0.size(), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    for (int k = 0; k < 27; ++k) {
        const int x = k % 3, y = (k / 3) % 3, zz = k / 9;
        const int64_t kp = (x + kZPad) + P0 * ((y + kZPad) + (int64_t)P0 * (zz + kZPad));
        for (int j = 0; j < kZStored; ++j) {
            const int i = kZCentre + j;
            const int X = x + kZTable.dx[i], Y = y + kZTable.dy[i], Zc = zz + kZTable.dz[i];
            if (X < 0 || Y < 0 || Zc < 0 || X > 2 || Y > 2 || Zc > 2) continue;
            const int m = X + 3 * (Y + 3 * Zc);
            Z0[k * 27 + m] = Z0[m * 27 + k] = S0[(size_t)j * NP0 + kp];
        }
    }
    for (double v : Z0)
        if (!std::isfinite(v)) return fail(AGCA_E_NUMERIC, "non-finite coarse pressure operator");
    if (!bordered_inverse(Z0, M))
        return fail(AGCA_E_NUMERIC, "the coarse pressure operator has a kernel beyond the constants");
    HIPCHK(h, hipMemcpyAsync(coarse, M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->zmg_version = h->nu_version;
    return AGCA_OK;
}

// y = V_l r: one V(kZSweeps, kZSweeps) cycle on level l from a zero guess (r, y distinct
// from level l's own work vectors a and t)
static int32_t zmg_cycle(agca_hier* h, const std::vector<ZLevel>& z, const double* coarse, int l,
                         const double* r, double* y) {
    if (l == 0) {
        HIPCHK(h, launch_zcoarse(coarse, r, y, h->st));
        return AGCA_OK;
    }
    const ZLevel& Z = z[l];
    // 2 kZSweeps Jacobi results in all, alternating between a and y so that the last is y
    double* cur = (2 * kZSweeps - 1) % 2 ? Z.a : y;
    auto other = [&](double* v) { return v == y ? Z.a : y; };
    HIPCHK(h, launch_zjacobi0(Z.n, Z.S, r, kZOmega, cur, h->st));
    for (int s = 1; s < kZSweeps; ++s) {
        double* nxt = other(cur);
        HIPCHK(h, launch_zstencil(2, Z.n, Z.S, cur, r, kZOmega, nxt, h->st));
        cur = nxt;
    }
    HIPCHK(h, launch_zstencil(1, Z.n, Z.S, cur, r, 0.0, Z.t, h->st));
    const ZLevel& C = z[l - 1];
    HIPCHK(h, launch_restrict_all(C.n, Z.t, C.r, h->st));
    TRY(zmg_cycle(h, z, coarse, l - 1, C.r, C.y));
    HIPCHK(h, launch_prolong_all_add(Z.n, C.y, cur, h->st));
    for (int s = 0; s < kZSweeps; ++s) {
        double* nxt = other(cur);
        HIPCHK(h, launch_zstencil(2, Z.n, Z.S, cur, r, kZOmega, nxt, h->st));
        cur = nxt;
    }
    if (cur != y) return fail(AGCA_E_STATE, "pressure V-cycle ended outside its output");
    return AGCA_OK;
}

// y = iters steps of CG on Z y = r from y = 0 preconditioned by one pressure V-cycle,
// with the assembled top-level stencil as the operator (scalars as in z_solve)
static int32_t z_solve_mg(agca_hier* h, const Bfbt& w, const double* r, double* y, int iters) {
    const int64_t np = stokes_dims(h).np;
    const int nb = h->nb_partial;
    double* coarse = nullptr;
    const std::vector<ZLevel> z = zmg_levels(h, &coarse);
    const ZLevel& T = z[h->cfg.L - 1];
    HIPCHK(h, launch_fill<double>(np, 0.0, y, h->st));
    HIPCHK(h, launch_axpby<double>(np, 1.0, r, 0.0, w.zr, h->st));
    TRY(zmg_cycle(h, z, coarse, h->cfg.L - 1, w.zr, w.zz));
    HIPCHK(h, launch_dot2<double>(np, w.zz, w.zr, nullptr, h->partial, nb, h->st));
    HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred, h->st));
    HIPCHK(h, launch_axpby<double>(np, 1.0, w.zz, 0.0, w.zp, h->st));
    int cur = 0;
    for (int k = 0; k < iters; ++k) {
        HIPCHK(h, launch_zstencil(0, T.n, T.S, w.zp, nullptr, 0.0, w.zq, h->st));
        HIPCHK(h, launch_dot2<double>(np, w.zp, w.zq, nullptr, h->partial, nb, h->st));
        HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred + 2, h->st));
        HIPCHK(h, launch_cg_update(np, w.zred + cur, w.zred + 2, w.zp, w.zq, y, w.zr, nullptr,
                                   h->partial, nb, h->st));
        if (k == iters - 1) break;
        TRY(zmg_cycle(h, z, coarse, h->cfg.L - 1, w.zr, w.zz));
        HIPCHK(h, launch_dot2<double>(np, w.zz, w.zr, nullptr, h->partial, nb, h->st));
        HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred + (1 - cur), h->st));
        HIPCHK(h, launch_zpbp_dev<double>(np, w.zz, w.zred + (1 - cur), w.zred + cur, 1.0, w.zp, h->st));
        cur = 1 - cur;
    }
    return AGCA_OK;
}

// y = iters steps of Jacobi-preconditioned CG on Z y = r from y = 0.  The scalars stay
// on the device: r.z alternates between zred[0] and zred[1], p.q is zred[2]; a step of
// zero Z-energy (r = 0) has step size zero (the update kernels' guards).
static int32_t z_solve(agca_hier* h, const Bfbt& w, const double* r, double* y, int iters) {
    const int64_t np = stokes_dims(h).np;
    const int nb = h->nb_partial;
    HIPCHK(h, launch_fill<double>(np, 0.0, y, h->st));
    HIPCHK(h, launch_axpby<double>(np, 1.0, r, 0.0, w.zr, h->st));
    HIPCHK(h, launch_div_elementwise(np, w.zr, w.zdiag, w.zz, h->st));
    HIPCHK(h, launch_dot2<double>(np, w.zz, w.zr, nullptr, h->partial, nb, h->st));
    HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred, h->st));
    HIPCHK(h, launch_axpby<double>(np, 1.0, w.zz, 0.0, w.zp, h->st));
    int cur = 0;
    for (int k = 0; k < iters; ++k) {
        TRY(z_apply(h, w, w.zp, w.zq));
        HIPCHK(h, launch_dot2<double>(np, w.zp, w.zq, nullptr, h->partial, nb, h->st));
        HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred + 2, h->st));
        HIPCHK(h, launch_cg_update(np, w.zred + cur, w.zred + 2, w.zp, w.zq, y, w.zr, nullptr,
                                   h->partial, nb, h->st));
        if (k == iters - 1) break;
        HIPCHK(h, launch_div_elementwise(np, w.zr, w.zdiag, w.zz, h->st));
        HIPCHK(h, launch_dot2<double>(np, w.zz, w.zr, nullptr, h->partial, nb, h->st));
        HIPCHK(h, launch_sum_partials(h->partial, nb, w.zred + (1 - cur), h->st));
        HIPCHK(h, launch_zpbp_dev<double>(np, w.zz, w.zred + (1 - cur), w.zred + cur, 1.0, w.zp, h->st));
        cur = 1 - cur;
    }
    return AGCA_OK;
}
// q = S^-1 rp, S the BFBT approximation, Z solves by Jacobi-CG or multigrid-CG
static int32_t bfbt_apply(agca_hier* h, const double* rp, double* q, int iters, bool mg) {
    const StokesDims d = stokes_dims(h);
    const Bfbt w = bfbt_bufs(h);
    auto zsolve = [&](const double* r, double* y) {
        return mg ? z_solve_mg(h, w, r, y, iters) : z_solve(h, w, r, y, iters);
    };
    TRY(zsolve(rp, w.y1));
    HIPCHK(h, launch_fill<double>(d.nu, 0.0, w.v2, h->st));
    TRY(stokes_grad_add(h, w.y1, w.v2));
    HIPCHK(h, launch_mul_elementwise(d.nu, w.v2, w.winv, w.v2, h->st));
    TRY(do_cube<double>(h, h->cfg.L, MODE_APPLY, w.v2, nullptr, w.v1, 0.0));
    HIPCHK(h, launch_mul_elementwise(d.nu, w.v1, w.winv, w.v1, h->st));
    TRY(stokes_div(h, w.v1, w.y2));
    TRY(zsolve(w.y2, q));
    return AGCA_OK;
}
// q = S^-1 rp: the lumped 1/nu mass, or BFBT during a solve that asked for it
static int32_t schur_inv(agca_hier* h, const double* rp, double* q) {
    if (h->st_schur_iters > 0) return bfbt_apply(h, rp, q, h->st_schur_iters, h->st_schur_mg);
    HIPCHK(h, launch_div_elementwise(stokes_dims(h).np, rp, h->st_mass, q, h->st));
    return AGCA_OK;
}

// z = A~^-1 r for the velocity block: st_vcycles V-cycles of a stationary iteration from
// zero (z = V r, then z += V (r - A z)); one V-cycle is the paper's choice (Section 4)
static int32_t velocity_inv(agca_hier* h, const double* r, double* z) {
    TRY(precondition(h, r, z));
    if (h->st_vcycles <= 1) return AGCA_OK;
    const StokesDims d = stokes_dims(h);
    if (!h->st_vtmp) TRY(alloc_t(h, &h->st_vtmp, (size_t)(2 * d.nu)));
    double *t = h->st_vtmp, *e = h->st_vtmp + d.nu;
    for (int k = 1; k < h->st_vcycles; ++k) {
        TRY(do_cube<double>(h, h->cfg.L, MODE_RESIDUAL, z, r, t, 0.0));
        TRY(precondition(h, t, e));
        HIPCHK(h, launch_axpby<double>(d.nu, 1.0, e, 1.0, z, h->st));
    }
    return AGCA_OK;
}

// z = diag(V-cycle, S^-1) r, or with the upper block-triangular preconditioner of
// eq. (4.1), z = [[V, V B^T S^-1], [0, -S^-1]] r with S approximating the positive
// B A^-1 B^T (diag(mass) or BFBT): q = S^-1 r_p, z_u = V(r_u + B^T q), z_p = -q.
static int32_t stokes_precond(agca_hier* h, const double* r, double* z) {
    const StokesDims d = stokes_dims(h);
    if (!h->st_tri) {
        TRY(velocity_inv(h, r, z));
        TRY(schur_inv(h, r + d.nu, z + d.nu));
        return AGCA_OK;
    }
    double* tu = h->st_tri;
    double* q = tu + d.nu;
    TRY(schur_inv(h, r + d.nu, q));
    HIPCHK(h, launch_axpby<double>(d.nu, 1.0, r, 0.0, tu, h->st));
    TRY(stokes_grad_add(h, q, tu));
    TRY(velocity_inv(h, tu, z));
    HIPCHK(h, launch_axpby<double>(d.np, -1.0, q, 0.0, z + d.nu, h->st));
    return AGCA_OK;
}
static int32_t stokes_norm(agca_hier* h, const double* x, double* out) {
    double v = 0.0;
    TRY(do_dot<double>(h, x, x, stokes_dims(h).tot, &v));
    *out = std::sqrt(v);
    return AGCA_OK;
}
// r = b - K x
static int32_t stokes_residual(agca_hier* h, const double* b, const double* x, double* r) {
    const int64_t tot = stokes_dims(h).tot;
    TRY(stokes_apply(h, x, r));
    HIPCHK(h, launch_axpby<double>(tot, 1.0, b, -1.0, r, h->st));
    return AGCA_OK;
}

// Right-preconditioned flexible GMRES(m).  Each Arnoldi vector is orthogonalised by
// classical Gram-Schmidt (one pass over the basis for all dot products, one for the
// update; the coefficients stay on the device), two sweeps over the basis per step
// instead of the 2 (k + 1) sweeps of modified Gram-Schmidt.  A second pass runs when
// the first removed more than 90 % of the vector's norm (the Daniel-Gragg-Kaufman-
// Stewart test with threshold 0.1; the customary 1/sqrt(2) fired on every step of the
// sinker problems without changing a single iteration count, at twice the cost).
constexpr double kDgks = 0.1;
// An FP32 basis keeps its vectors at a leading dimension that is a multiple of 4 (the
// Gram-Schmidt passes load four entries at a time), in as many FP64 vector slots as its
// bytes need.
static int64_t fp32_basis_ld(int64_t tot) { return (tot + 3) & ~(int64_t)3; }
static int64_t fp32_basis_slots(int m, int64_t tot) {
    const int64_t bytes = (int64_t)(m + 1) * fp32_basis_ld(tot) * (int64_t)sizeof(float);
    const int64_t slot = tot * (int64_t)sizeof(double);
    return (bytes + slot - 1) / slot;
}
// work vectors of FGMRES(m): the basis (m + 1 vectors), Z (m), w, r, and with an FP32
// basis the FP64 copy of the basis vector being preconditioned
static int64_t fgmres_work_vecs(int m, bool v32, int64_t tot) {
    return v32 ? fp32_basis_slots(m, tot) + m + 3 : 2 * (int64_t)m + 3;
}
static int32_t stokes_fgmres(agca_hier* h, const agca_stokes_opts* o, const double* b, double* x,
                             double bn, double* rel_out, int* it_out, std::vector<double>& hist,
                             bool* floor_out, double* rho_out) {
    const int64_t tot = stokes_dims(h).tot;
    const int m = o->restart;
    // the basis V (m + 1 vectors, FP64 or FP32), Z (m FP64 vectors), w, r, and with an FP32
    // basis an FP64 copy of the basis vector being preconditioned
    const bool v32 = o->basis_dtype == AGCA_F32;
    TRY(stokes_work(h, fgmres_work_vecs(m, v32, tot)));
    const int64_t vslots = v32 ? fp32_basis_slots(m, tot) : m + 1;
    const int64_t ld32 = fp32_basis_ld(tot);
    double* V = v32 ? nullptr : h->st_work;
    float* V32 = v32 ? reinterpret_cast<float*>(h->st_work) : nullptr;
    double* Z = h->st_work + vslots * tot;
    double* w = Z + (int64_t)m * tot;
    double* r = w + tot;
    double* vk = v32 ? r + tot : nullptr;
    auto vec = [&](double* base, int i) { return base + (int64_t)i * tot; };
    // V_i = a x
    auto set_basis = [&](int i, double a, const double* xx) -> hipError_t {
        return v32 ? launch_scale_to_f32(tot, a, xx, V32 + (int64_t)i * ld32, h->st)
                   : launch_axpby<double>(tot, a, xx, 0.0, vec(V, i), h->st);
    };
    auto gs_dots = [&](int nv) -> hipError_t {
        return v32 ? launch_gs_dots<float>(tot, w, V32, ld32, nv, h->st_gs, h->st)
                   : launch_gs_dots<double>(tot, w, V, tot, nv, h->st_gs, h->st);
    };
    auto gs_update = [&](int nv) -> hipError_t {
        return v32 ? launch_gs_update<float>(tot, w, V32, ld32, nv, h->red, h->st)
                   : launch_gs_update<double>(tot, w, V, tot, nv, h->red, h->st);
    };
    HIPCHK(h, launch_fill<double>(tot, 0.0, x, h->st));
    HIPCHK(h, launch_axpby<double>(tot, 1.0, b, 0.0, r, h->st));
    double rel = 0.0;
    TRY(stokes_norm(h, r, &rel));
    rel /= bn;
    hist.push_back(rel);
    int it = 0;
    std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), col(m + 3);
    std::vector<double> cycle_res;  // true residual after each restart cycle
    const int nb = v32 ? gs_blocks_f32(tot) : gs_blocks(tot);  // workgroups of the dot pass
    if (h->st_gs_cap < (int64_t)(m + 2) * nb) {
        for (size_t i = 0; h->st_gs && i < h->allocs.size(); ++i)
            if (h->allocs[i] == h->st_gs) {
                (void)hipFree(h->st_gs);
                h->allocs.erase(h->allocs.begin() + i);
                h->bytes -= h->st_gs_cap * (int64_t)sizeof(double);
                break;
            }
        h->st_gs = nullptr;
        h->st_gs_cap = 0;
        TRY(alloc_t(h, &h->st_gs, (size_t)(m + 2) * nb));
        h->st_gs_cap = (int64_t)(m + 2) * nb;
    }
    auto Hm = [&](int i, int k) -> double& { return H[(size_t)i * m + k]; };
    while (it < o->max_iter) {
        double beta = 0.0;
        TRY(stokes_norm(h, r, &beta));
        HIPCHK(h, set_basis(0, 1.0 / beta, r));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k_done = 0;
        for (int k = 0; k < m; ++k) {
            if (v32) {
                HIPCHK(h, launch_cast(AGCA_F32, AGCA_F64, V32 + (int64_t)k * ld32, vk, tot, h->st));
                TRY(stokes_precond(h, vk, vec(Z, k)));
            } else {
                TRY(stokes_precond(h, vec(V, k), vec(Z, k)));
            }
            TRY(stokes_apply(h, vec(Z, k), w));
            // classical Gram-Schmidt against V_0..V_k, a second pass after severe cancellation
            HIPCHK(h, gs_dots(k + 1));
            HIPCHK(h, launch_gs_sum(h->st_gs, nb, k + 2, h->red, h->st));
            HIPCHK(h, gs_update(k + 1));
            HIPCHK(h, gs_dots(0));
            HIPCHK(h, launch_gs_sum(h->st_gs, nb, 1, h->red + k + 2, h->st));
            TRY(fetch(h, k + 3, col.data()));
            for (int i = 0; i <= k; ++i) Hm(i, k) = col[i];
            double nrm2 = col[k + 2];
            if (!(std::sqrt(nrm2) >= kDgks * std::sqrt(col[k + 1]))) {
                HIPCHK(h, gs_dots(k + 1));
                HIPCHK(h, launch_gs_sum(h->st_gs, nb, k + 1, h->red, h->st));
                HIPCHK(h, gs_update(k + 1));
                HIPCHK(h, gs_dots(0));
                HIPCHK(h, launch_gs_sum(h->st_gs, nb, 1, h->red + k + 1, h->st));
                TRY(fetch(h, k + 2, col.data()));
                for (int i = 0; i <= k; ++i) Hm(i, k) += col[i];
                nrm2 = col[k + 1];
            }
            Hm(k + 1, k) = std::sqrt(nrm2);
            if (Hm(k + 1, k) > 0.0) HIPCHK(h, set_basis(k + 1, 1.0 / Hm(k + 1, k), w));
            for (int i = 0; i < k; ++i) {
                const double t = cs[i] * Hm(i, k) + sn[i] * Hm(i + 1, k);
                Hm(i + 1, k) = -sn[i] * Hm(i, k) + cs[i] * Hm(i + 1, k);
                Hm(i, k) = t;
            }
            const double dd = std::hypot(Hm(k, k), Hm(k + 1, k));
            cs[k] = Hm(k, k) / dd;
            sn[k] = Hm(k + 1, k) / dd;
            Hm(k, k) = dd;
            Hm(k + 1, k) = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            ++it;
            k_done = k + 1;
            hist.push_back(std::fabs(g[k + 1]) / bn);
            if (!std::isfinite(hist.back())) return fail(AGCA_E_NUMERIC, "FGMRES breakdown");
            if (hist.back() <= o->tol || it >= o->max_iter) break;
        }
        // y = H^-1 g (upper triangular), x += Z y
        std::vector<double> y(k_done);
        for (int i = k_done - 1; i >= 0; --i) {
            double t = g[i];
            for (int j = i + 1; j < k_done; ++j) t -= Hm(i, j) * y[j];
            y[i] = t / Hm(i, i);
        }
        for (int i = 0; i < k_done; ++i) HIPCHK(h, launch_axpby<double>(tot, y[i], vec(Z, i), 1.0, x, h->st));
        TRY(stokes_residual(h, b, x, r));
        const bool estimate_reached = hist.back() <= o->tol;
        TRY(stokes_norm(h, r, &rel));
        rel /= bn;
        hist.back() = rel;
        if (rel <= o->tol) break;
        // rounding floor: the cycle's recurrence reached the tolerance but the true
        // residual did not, it is less than 5 % better than four restart cycles ago
        // (the true residual of an FP64 iterate stagnates there while each cycle's
        // estimate keeps converging), and it is at most kFloorFactor max(tol, rho_A),
        // rho_A the rounding floor of the velocity block alone (the residual_floor
        // terms of A and the velocity right-hand side over the whole system's norm: a
        // lower bound of the full system's floor, which adds the B and B^T terms)
        cycle_res.push_back(rel);
        const size_t c = cycle_res.size();
        if (estimate_reached && c >= 5 && rel > 0.95 * cycle_res[c - 5]) {
            double s_sq = 0.0, b_sq = 0.0;
            TRY(floor_sums(h, b, x, &s_sq, &b_sq));
            *rho_out = kUnitRoundoff * std::sqrt(s_sq) / bn;
            if (at_floor(rel, o->tol, *rho_out)) {
                *floor_out = true;
                break;
            }
        }
    }
    *rel_out = rel;
    *it_out = it;
    return AGCA_OK;
}

// MINRES (Paige and Saunders, SIAM J. Numer. Anal. 12, 1975) with the block-diagonal
// preconditioner P (SPD), derived here as follows.  With P = C C^T, MINRES for
// C^T K C y = C^T b runs the Lanczos process on C^T K C; its vectors q_j are kept as
// w_j = C^-T q_j (residual space) and u_j = C q_j = P w_j (solution space):
//   v = K u_j - beta_j w_{j-1},  alpha_j = u_j . v,  v -= alpha_j w_j,
//   beta_{j+1} = sqrt(v . P v),  w_{j+1} = v / beta_{j+1},  u_{j+1} = P v / beta_{j+1},
// so that K U_k = W_{k+1} T_k, T_k tridiagonal ((k+1) x k).  The iterate x_k = U_k t_k
// minimises ||beta_1 e_1 - T_k t||.  T_k is reduced to upper triangular R_k by Givens
// rotations G_j = [[c_j, s_j], [-s_j, c_j]] on rows (j, j+1): column k holds beta_k,
// alpha_k, beta_{k+1} in rows k-1, k, k+1; G_{k-2} turns (0, beta_k) into
// (eps_k, c_{k-2} beta_k), G_{k-1} turns (c_{k-2} beta_k, alpha_k) into (sig_k, gam_k),
// and G_k (c_k = gam_k / rho_k, s_k = beta_{k+1} / rho_k, rho_k = |(gam_k, beta_{k+1})|)
// annihilates beta_{k+1}.  The same rotations take beta_1 e_1 to (tau_1 .. tau_k, gbar):
// tau_k = c_k gbar, gbar <- -s_k gbar.  With the directions D_k = U_k R_k^-1,
//   d_k = (u_k - sig_k d_{k-1} - eps_k d_{k-2}) / rho_k,   x_k = x_{k-1} + tau_k d_k.
// The stopping test (eq. (4.3)) uses the true residual b - K x_k, recomputed at every
// step (the method minimises the P^-1-norm of the residual, not its 2-norm).
static int32_t stokes_minres(agca_hier* h, const agca_stokes_opts* o, const double* b, double* x,
                             double bn, double* rel_out, int* it_out, std::vector<double>& hist) {
    const int64_t tot = stokes_dims(h).tot;
    TRY(stokes_work(h, 8));
    auto vecn = [&](int i) { return h->st_work + (int64_t)i * tot; };
    double *w_prev = vecn(0), *w = vecn(1), *u = vecn(2), *v = vecn(3), *pv = vecn(4),
           *d_last = vecn(5), *d_older = vecn(6), *res = vecn(7);
    HIPCHK(h, launch_fill<double>(tot, 0.0, x, h->st));
    hist.push_back(1.0);
    *rel_out = 1.0;
    *it_out = 0;
    // beta_1 = sqrt(b . P b), w_1 = b / beta_1, u_1 = P b / beta_1
    TRY(stokes_precond(h, b, pv));
    double t = 0.0;
    TRY(do_dot<double>(h, b, pv, tot, &t));
    if (!(t >= 0.0) || !std::isfinite(t)) return fail(AGCA_E_NUMERIC, "MINRES: preconditioner is not positive");
    const double beta1 = std::sqrt(t);
    if (beta1 == 0.0) {
        *rel_out = 0.0;
        return AGCA_OK;
    }
    HIPCHK(h, launch_axpby<double>(tot, 1.0 / beta1, b, 0.0, w, h->st));
    HIPCHK(h, launch_axpby<double>(tot, 1.0 / beta1, pv, 0.0, u, h->st));
    HIPCHK(h, launch_fill<double>(tot, 0.0, d_last, h->st));
    HIPCHK(h, launch_fill<double>(tot, 0.0, d_older, h->st));
    double beta = beta1;            // beta_k
    double c1 = 1.0, s1 = 0.0;      // rotation k-1
    double c2 = 1.0, s2 = 0.0;      // rotation k-2
    double gbar = beta1;            // last entry of the rotated right-hand side
    double rel = 1.0;
    int k = 0;
    while (k < o->max_iter) {
        ++k;
        // Lanczos: v = K u_k - beta_k w_{k-1} - alpha_k w_k, P v, beta_{k+1}
        TRY(stokes_apply(h, u, v));
        if (k > 1) HIPCHK(h, launch_axpby<double>(tot, -beta, w_prev, 1.0, v, h->st));
        double alpha = 0.0;
        TRY(do_dot<double>(h, u, v, tot, &alpha));
        HIPCHK(h, launch_axpby<double>(tot, -alpha, w, 1.0, v, h->st));
        TRY(stokes_precond(h, v, pv));
        TRY(do_dot<double>(h, v, pv, tot, &t));
        if (!std::isfinite(t) || !std::isfinite(alpha)) return fail(AGCA_E_NUMERIC, "MINRES breakdown");
        // v . P v can only vanish (or lose its sign to rounding) in an invariant space
        const double beta_next = t > 0.0 ? std::sqrt(t) : 0.0;
        // QR update of the new column (beta_k, alpha_k, beta_{k+1})
        const double bk = k > 1 ? beta : 0.0;
        const double eps = s2 * bk;
        const double bt = c2 * bk;
        const double sig = c1 * bt + s1 * alpha;
        const double gam = -s1 * bt + c1 * alpha;
        const double rho = std::hypot(gam, beta_next);
        if (!(rho > 0.0)) return fail(AGCA_E_NUMERIC, "MINRES: singular tridiagonal factor");
        const double c = gam / rho, s = beta_next / rho;
        const double tau = c * gbar;
        gbar = -s * gbar;
        // d_k = (u_k - sig d_{k-1} - eps d_{k-2}) / rho, written over d_{k-2}
        HIPCHK(h, launch_axpby<double>(tot, 1.0 / rho, u, -eps / rho, d_older, h->st));
        HIPCHK(h, launch_axpby<double>(tot, -sig / rho, d_last, 1.0, d_older, h->st));
        std::swap(d_last, d_older);
        HIPCHK(h, launch_axpby<double>(tot, tau, d_last, 1.0, x, h->st));
        c2 = c1;
        s2 = s1;
        c1 = c;
        s1 = s;
        TRY(stokes_residual(h, b, x, res));
        TRY(stokes_norm(h, res, &rel));
        rel /= bn;
        hist.push_back(rel);
        if (!std::isfinite(rel)) return fail(AGCA_E_NUMERIC, "MINRES breakdown");
        if (rel <= o->tol || beta_next == 0.0) break;
        // advance the Lanczos vectors: w_{k+1} into the buffer of w_{k-1}, u_{k+1} over u_k
        HIPCHK(h, launch_axpby<double>(tot, 1.0 / beta_next, v, 0.0, w_prev, h->st));
        std::swap(w_prev, w);
        HIPCHK(h, launch_axpby<double>(tot, 1.0 / beta_next, pv, 0.0, u, h->st));
        beta = beta_next;
    }
    *rel_out = rel;
    *it_out = k;
    return AGCA_OK;
}

int32_t agca_stokes_div(agca_hier* h, const double* u, double* q) {
    TRY(stokes_ready(h));
    if (!u || !q) return fail(AGCA_E_INVALID, "null pointer");
    return stokes_div(h, u, q);
}

int32_t agca_stokes_grad(agca_hier* h, const double* p, double* v) {
    TRY(stokes_ready(h));
    if (!p || !v) return fail(AGCA_E_INVALID, "null pointer");
    HIPCHK(h, launch_fill<double>(stokes_dims(h).nu, 0.0, v, h->st));
    return stokes_grad_add(h, p, v);
}

int32_t agca_stokes_mass(agca_hier* h, double* m) {
    TRY(stokes_ready(h));
    if (!m) return fail(AGCA_E_INVALID, "null pointer");
    HIPCHK(h, hipMemcpyAsync(m, h->st_mass, sizeof(double) * stokes_dims(h).np,
                             hipMemcpyDeviceToDevice, h->st));
    return AGCA_OK;
}

int32_t agca_stokes_schur_apply(agca_hier* h, int32_t schur, int32_t schur_iters, const double* rp,
                                double* q) {
    TRY(stokes_ready(h));
    if (!rp || !q || rp == q) return fail(AGCA_E_INVALID, "null or aliased pointer");
    const StokesDims d = stokes_dims(h);
    if (schur == AGCA_SCHUR_MASS) {
        HIPCHK(h, launch_div_elementwise(d.np, rp, h->st_mass, q, h->st));
        return AGCA_OK;
    }
    if (schur != AGCA_SCHUR_BFBT && schur != AGCA_SCHUR_BFBT_MG)
        return fail(AGCA_E_INVALID, "unknown Schur approximation");
    if (schur_iters < 1 || schur_iters > 1000) return fail(AGCA_E_INVALID, "schur_iters must be in [1, 1000]");
    const bool zmg = schur == AGCA_SCHUR_BFBT_MG;
    TRY(bfbt_ready(h, !zmg));
    if (zmg) TRY(zmg_ready(h));
    return bfbt_apply(h, rp, q, schur_iters, zmg);
}

int32_t agca_stokes_z_stencil(agca_hier* h, int32_t level, double* out) {
    TRY(stokes_ready(h));
    if (!out) return fail(AGCA_E_INVALID, "null pointer");
    if (level < 0 || level > h->cfg.L - 1) return fail(AGCA_E_INVALID, "level must be in [0, L-1]");
    TRY(zmg_ready(h));
    const std::vector<ZLevel> z = zmg_levels(h);
    HIPCHK(h, launch_zexpand(z[level].n, z[level].S, out, h->st));
    return AGCA_OK;
}

int32_t agca_stokes_z_vcycle(agca_hier* h, const double* r, double* y) {
    TRY(stokes_ready(h));
    if (!r || !y || r == y) return fail(AGCA_E_INVALID, "null or aliased pointer");
    TRY(zmg_ready(h));
    double* coarse = nullptr;
    const std::vector<ZLevel> z = zmg_levels(h, &coarse);
    const Bfbt w = bfbt_bufs(h);
    const int64_t np = stokes_dims(h).np;
    // through the solver's own buffers: the cycle's input and output stay distinct from
    // the top level's work vectors whatever the caller passes
    HIPCHK(h, launch_axpby<double>(np, 1.0, r, 0.0, w.zr, h->st));
    TRY(zmg_cycle(h, z, coarse, h->cfg.L - 1, w.zr, w.zz));
    HIPCHK(h, hipMemcpyAsync(y, w.zz, sizeof(double) * np, hipMemcpyDeviceToDevice, h->st));
    return AGCA_OK;
}

int32_t agca_stokes_solve(agca_hier* h, const agca_stokes_opts* o, const double* f, const double* g,
                          double* u, double* p, agca_solve_stats* stats) {
    TRY(stokes_ready(h));
    if (!o || !f || !g || !u || !p || !stats) return fail(AGCA_E_INVALID, "null pointer");
    if (o->max_iter < 0 || !(o->tol >= 0.0)) return fail(AGCA_E_INVALID, "bad solve options");
    if (o->solver != AGCA_STOKES_FGMRES && o->solver != AGCA_STOKES_MINRES)
        return fail(AGCA_E_INVALID, "unknown Stokes solver");
    if (o->solver == AGCA_STOKES_FGMRES && (o->restart < 1 || o->restart > AGCA_RED_SLOTS - 2))
        return fail(AGCA_E_INVALID, "restart must be in [1, " + std::to_string(AGCA_RED_SLOTS - 2) + "]");
    if (o->precond != AGCA_STOKES_DIAGONAL && o->precond != AGCA_STOKES_TRIANGULAR)
        return fail(AGCA_E_INVALID, "unknown Stokes preconditioner");
    if (o->precond == AGCA_STOKES_TRIANGULAR && o->solver != AGCA_STOKES_FGMRES)
        return fail(AGCA_E_INVALID, "the triangular preconditioner is not symmetric: FGMRES only");
    if (o->schur != AGCA_SCHUR_MASS && o->schur != AGCA_SCHUR_BFBT && o->schur != AGCA_SCHUR_BFBT_MG)
        return fail(AGCA_E_INVALID, "unknown Schur approximation");
    const bool bfbt = o->schur != AGCA_SCHUR_MASS;
    const bool zmg = o->schur == AGCA_SCHUR_BFBT_MG;
    if (bfbt && (o->schur_iters < 1 || o->schur_iters > 1000))
        return fail(AGCA_E_INVALID, "schur_iters must be in [1, 1000]");
    if (bfbt && o->solver != AGCA_STOKES_FGMRES)
        return fail(AGCA_E_INVALID, "the BFBT approximation is not a fixed linear map: FGMRES only");
    if (o->velocity_cycles < 0 || o->velocity_cycles > 8)
        return fail(AGCA_E_INVALID, "velocity_cycles must be in [0, 8]");
    if (o->basis_dtype != AGCA_F64 && o->basis_dtype != AGCA_F32)
        return fail(AGCA_E_INVALID, "basis_dtype must be F64 or F32");
    if (o->basis_dtype == AGCA_F32 && o->solver != AGCA_STOKES_FGMRES)
        return fail(AGCA_E_INVALID, "an FP32 basis is an FGMRES option");
    TRY(ensure_solver_vectors(h));
    std::memset(stats, 0, sizeof(*stats));
    const StokesDims d = stokes_dims(h);
    // contiguous right-hand side and solution in the last two work vectors' place
    const int64_t kry = (o->solver == AGCA_STOKES_FGMRES)
                            ? fgmres_work_vecs(o->restart, o->basis_dtype == AGCA_F32, d.tot) : 8;
    const bool tri = o->precond == AGCA_STOKES_TRIANGULAR;
    TRY(stokes_work(h, kry + 2 + (tri ? 1 : 0)));
    double* bvec = h->st_work + kry * d.tot;
    double* xvec = bvec + d.tot;
    h->st_tri = tri ? xvec + d.tot : nullptr;
    h->st_schur_iters = 0;
    if (bfbt) TRY(bfbt_ready(h, !zmg));
    if (zmg) TRY(zmg_ready(h));
    h->st_schur_iters = bfbt ? o->schur_iters : 0;
    h->st_schur_mg = zmg;
    h->st_vcycles = o->velocity_cycles > 1 ? o->velocity_cycles : 1;
    auto t0 = std::chrono::steady_clock::now();
    HIPCHK(h, hipMemcpyAsync(bvec, f, sizeof(double) * d.nu, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, launch_zero_boundary<double>(3, d.nf, bvec, h->st));
    HIPCHK(h, hipMemcpyAsync(bvec + d.nu, g, sizeof(double) * d.np, hipMemcpyDeviceToDevice, h->st));
    double bn = 0.0;
    TRY(stokes_norm(h, bvec, &bn));
    if (!std::isfinite(bn)) return fail(AGCA_E_NUMERIC, "non-finite right-hand side");
    std::vector<double> hist;
    double rel = 0.0;
    int it = 0;
    bool floor_limited = false;
    double rho_a = 0.0;
    if (bn == 0.0) {
        HIPCHK(h, launch_fill<double>(d.tot, 0.0, xvec, h->st));
        hist.push_back(0.0);
    } else {
        const int32_t rc = (o->solver == AGCA_STOKES_FGMRES)
                               ? stokes_fgmres(h, o, bvec, xvec, bn, &rel, &it, hist, &floor_limited, &rho_a)
                               : stokes_minres(h, o, bvec, xvec, bn, &rel, &it, hist);
        h->st_tri = nullptr;
        h->st_schur_iters = 0;
        h->st_vcycles = 1;
        if (rc != AGCA_OK) return rc;
    }
    h->st_tri = nullptr;
    h->st_schur_iters = 0;
    h->st_vcycles = 1;
    // pressure with zero mean (the constant is the kernel of B^T on free velocities)
    double psum = 0.0;
    {
        double* ones = h->st_qf;   // scratch of at least np entries
        HIPCHK(h, launch_fill<double>(d.np, 1.0, ones, h->st));
        TRY(do_dot<double>(h, xvec + d.nu, ones, d.np, &psum));
        HIPCHK(h, launch_axpby<double>(d.np, -psum / (double)d.np, ones, 1.0, xvec + d.nu, h->st));
    }
    HIPCHK(h, hipMemcpyAsync(u, xvec, sizeof(double) * d.nu, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(p, xvec + d.nu, sizeof(double) * d.np, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    stats->iterations = it;
    stats->rel_residual = rel;
    stats->recursive_rel_residual = hist.empty() ? rel : hist.back();
    stats->converged = rel <= o->tol || bn == 0.0;
    stats->floor_limited = (!stats->converged && floor_limited) ? 1 : 0;
    stats->floor_estimate = rho_a;
    for (size_t i = 0; i < hist.size() && i < (size_t)AGCA_MAX_HISTORY; ++i)
        if (o->record_history) stats->history[i] = hist[i];
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!stats->converged && !stats->floor_limited)
        return fail(AGCA_E_NOCONV, "no convergence within max_iter");
    return AGCA_OK;
}

}  // extern "C"

