// Host build of the library's per-cell arithmetic headers (kuhn.h, cube_math.h,
// gca_math.h) and of its solver stopping rule (stop_rule.h), driven by
// tests/test_host_headers.py, which compares the printed values with the CPU oracle.
// Reads one command from stdin:
//   elem  ncomp                  -> for s = 0..5 the unit element matrix (without h/6)
//                                   obtained from tet_dca on unit corner vectors,
//                                   (4 ncomp)^2 values per s, row (c,a) = 4c+a, col (d,b)
//   energy ncomp U[8*ncomp] W[8*ncomp] -> cell_energy (6 values)
//   gca ncomp l L nid ids[nid] nu[6 n_L^3]
//                                -> Galerkin blocks of level-l elements by the element-wise
//                                   recursion (fine_block + add_ptkp over child_id), FP64
//   stop tol rho k (r_i it_i f_i)*k -> after each true residual r_i of a replacement at
//                                   iteration it_i (f_i = 1: the recurrence had halved
//                                   since the last one), the decision:
//                                   0 continue, 1 floor, 2 stalled
//   zstencil                     -> the pressure stencil's 65 offsets (dx dy dz per line)
//                                   and the probing colour of every node of a 9^3 lattice
#include <cstdio>
#include <cstring>
#include <vector>

#include "gca_math.h"
#include "stop_rule.h"
#include "zstencil.h"

using namespace agca;

template <int S, int NC>
static void elem_matrix_s(std::vector<double>& out) {
    constexpr int M = 4 * NC;
    for (int col = 0; col < M; ++col) {
        const int d = col / 4, b = col % 4;
        double U[8][NC] = {}, F[8][NC] = {};
        U[path_corner(S, b)][d] = 1.0;
        tet_dca<S, NC, double>(U, 1.0, F);
        for (int row = 0; row < M; ++row) out[(size_t)row * M + col] = F[path_corner(S, row % 4)][row / 4];
    }
}

template <int NC>
static void elem_all() {
    constexpr int M = 4 * NC;
    std::vector<double> m((size_t)M * M);
    auto dump = [&]() {
        for (double v : m) std::printf("%.17g\n", v);
    };
    elem_matrix_s<0, NC>(m); dump();
    elem_matrix_s<1, NC>(m); dump();
    elem_matrix_s<2, NC>(m); dump();
    elem_matrix_s<3, NC>(m); dump();
    elem_matrix_s<4, NC>(m); dump();
    elem_matrix_s<5, NC>(m); dump();
}

template <int NC>
static void energy() {
    double U[8][NC], W[8][NC], e[6];
    for (int k = 0; k < 8; ++k)
        for (int c = 0; c < NC; ++c)
            if (std::scanf("%lf", &U[k][c]) != 1) return;
    for (int k = 0; k < 8; ++k)
        for (int c = 0; c < NC; ++c)
            if (std::scanf("%lf", &W[k][c]) != 1) return;
    cell_energy<NC, double>(U, W, e);
    for (double v : e) std::printf("%.17g\n", v);
}

// component block (c,d) of the Galerkin matrix of element e on a level with n cells,
// recursing depth levels down to the finest coefficient
static void gca_block(int ncomp, int64_t n, int64_t e, int depth, const std::vector<double>& nu,
                      double scale_fine, int c, int d, double (&G)[16]) {
    if (depth == 0) {
        fine_block(ncomp, (int)(e % 6), c, d, nu[(size_t)e] * scale_fine, G);
        return;
    }
    for (double& g : G) g = 0.0;
    for (int k = 0; k < 8; ++k) {
        double Gc[16];
        gca_block(ncomp, 2 * n, child_id(n, e, k), depth - 1, nu, scale_fine, c, d, Gc);
        add_ptkp(k, Gc, G);
    }
}

static void gca() {
    int ncomp, l, L, nid;
    if (std::scanf("%d %d %d %d", &ncomp, &l, &L, &nid) != 4) return;
    std::vector<long long> ids(nid);
    for (auto& v : ids)
        if (std::scanf("%lld", &v) != 1) return;
    const int64_t nL = 2LL << L;
    std::vector<double> nu((size_t)(6 * nL * nL * nL));
    for (auto& v : nu)
        if (std::scanf("%lf", &v) != 1) return;
    const int M = 4 * ncomp;
    for (long long e : ids) {
        std::vector<double> B((size_t)M * M);
        for (int c = 0; c < ncomp; ++c)
            for (int d = 0; d < ncomp; ++d) {
                double G[16];
                gca_block(ncomp, 2LL << l, e, L - l, nu, 1.0 / (6.0 * (double)nL), c, d, G);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) B[(size_t)(4 * c + a) * M + 4 * d + b] = G[4 * a + b];
            }
        for (double v : B) std::printf("%.17g\n", v);
    }
}

static void stop() {
    double tol, rho;
    int k;
    if (std::scanf("%lf %lf %d", &tol, &rho, &k) != 3) return;
    EndChecks ends;
    for (int i = 0; i < k; ++i) {
        double r;
        int it, full;
        if (std::scanf("%lf %d %d", &r, &it, &full) != 3) return;
        int verdict = 0;
        if (ends.stagnated(r, it, full != 0)) {
            if (at_floor(r, tol, rho))
                verdict = 1;
            else if (ends.given_up())
                verdict = 2;
        }
        std::printf("%d\n", verdict);
        if (verdict) break;
    }
}

static void zstencil() {
    for (int i = 0; i < kZOffsets; ++i) std::printf("%d %d %d\n", kZTable.dx[i], kZTable.dy[i], kZTable.dz[i]);
    for (int z = 0; z < 9; ++z)
        for (int y = 0; y < 9; ++y)
            for (int x = 0; x < 9; ++x) std::printf("%d\n", z_colour(x, y, z));
}

int main() {
    char cmd[16];
    if (std::scanf("%15s", cmd) != 1) return 1;
    int nc = 0;
    if (!std::strcmp(cmd, "elem") || !std::strcmp(cmd, "energy")) {
        if (std::scanf("%d", &nc) != 1) return 1;
    }
    if (!std::strcmp(cmd, "elem")) nc == 1 ? elem_all<1>() : elem_all<3>();
    else if (!std::strcmp(cmd, "energy")) nc == 1 ? energy<1>() : energy<3>();
    else if (!std::strcmp(cmd, "gca")) gca();
    else if (!std::strcmp(cmd, "stop")) stop();
    else if (!std::strcmp(cmd, "zstencil")) zstencil();
    else return 1;
    return 0;
}
