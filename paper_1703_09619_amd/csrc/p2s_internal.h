// p2s_internal.h -- layouts and compile-time structure shared by the host
// runtime and the HIP kernels of the product-to-sum fill.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define P2S_HD
#else
#define P2S_HD __host__ __device__
#endif

namespace p2s {

constexpr int MAXN = 8;          // largest order N (functions per direction)
constexpr int KPAD = 16;         // padded Legendre-degree extent (K = 2N-1 <= 15)
constexpr int MAXQ = 32;         // largest Gauss rule per axis
constexpr int NFAM = 3;          // 1-D families: phi, phi', psi
enum Fam : int { PHI = 0, DPHI = 1, PSI = 2 };

// Linearization tables, eq. (3): lin[t][m1][m2][k] with type t = 3*X + Y
// (X test family, Y trial family):  X_m1 Y_m2 = sum_k lin L_k.
constexpr int NTYPE = NFAM * NFAM;
constexpr int LIN_STRIDE_M1 = MAXN * KPAD;
constexpr int LIN_STRIDE_T = MAXN * MAXN * KPAD;
constexpr int LIN_SIZE = NTYPE * LIN_STRIDE_T;

// Gauss tables for Q = 1..MAXQ: x[Q][a], w[Q][a], and the moment weights
// legw[Q][k][a] = w_a L_k(x_a) for k < KPAD.
constexpr int GX_SIZE = (MAXQ + 1) * MAXQ;
constexpr int LEGW_STRIDE_Q = KPAD * MAXQ;
constexpr int LEGW_SIZE = (MAXQ + 1) * LEGW_STRIDE_Q;

P2S_HD constexpr int fam_dim(int fam, int N) { return fam == PSI ? N - 1 : N; }

// Legendre degrees present in the expansion of family member m.
P2S_HD constexpr uint32_t fam_support(int fam, int m)
{
    return fam == PHI ? (m < 2 ? 3u : ((1u << m) | (1u << (m - 2))))
         : fam == DPHI ? (m < 2 ? 1u : (1u << (m - 1)))
                       : (1u << m);
}

// Degrees k with a structurally nonzero lin[.][m1][m2][k]: the Legendre
// product L_a L_b spans degrees |a-b|, |a-b|+2, ..., a+b.
P2S_HD constexpr uint32_t prod_mask(int fx, int m1, int fy, int m2)
{
    uint32_t sx = fam_support(fx, m1), sy = fam_support(fy, m2), r = 0;
    for (int a = 0; a < KPAD; ++a) {
        if (!((sx >> a) & 1u)) continue;
        for (int b = 0; b < KPAD; ++b) {
            if (!((sy >> b) & 1u)) continue;
            int lo = a > b ? a - b : b - a;
            for (int k = lo; k <= a + b; k += 2) r |= 1u << k;
        }
    }
    return r;
}

P2S_HD constexpr int popcount32(uint32_t v)
{
    int c = 0;
    for (; v; v &= v - 1u) ++c;
    return c;
}

// Packed linearization tables: for order N and family pair (X,Y), the
// structurally nonzero coefficients lin[X,Y][p1][p2][q] in the order
// p1 < dim(X,N), p2 < dim(Y,N), q ascending -- the order in which the
// unrolled last contraction stage consumes them.
P2S_HD constexpr int packed_before(int X, int Y, int N, int P1, int P2)
{
    int c = 0;
    for (int p1 = 0; p1 < fam_dim(X, N); ++p1)
        for (int p2 = 0; p2 < fam_dim(Y, N); ++p2) {
            if (p1 == P1 && p2 == P2) return c;
            c += popcount32(prod_mask(X, p1, Y, p2));
        }
    return c;
}
P2S_HD constexpr int packed_count(int X, int Y, int N) { return packed_before(X, Y, N, -1, -1); }
// offset of the (N, X, Y) table inside the packed region, N = 2..MAXN
P2S_HD constexpr int packed_offset(int N, int X, int Y)
{
    int o = 0;
    for (int n = 2; n <= MAXN; ++n)
        for (int t = 0; t < NTYPE; ++t) {
            if (n == N && t == 3 * X + Y) return o;
            o += (packed_count(t / 3, t % 3, n) + 1) & ~1;  // keep 16-byte alignment
        }
    return o;
}
constexpr int PACKED_SIZE = packed_offset(MAXN + 1, 0, 0);

// Offsets of the device table buffer (in doubles).
constexpr int TAB_LIN = 0;
constexpr int TAB_GX = TAB_LIN + LIN_SIZE;
constexpr int TAB_GW = TAB_GX + GX_SIZE;
constexpr int TAB_LEGW = TAB_GW + GX_SIZE;
constexpr int TAB_PACK = TAB_LEGW + LEGW_SIZE;
// 1-D basis values at the Gauss points (direct quadrature):
// basis[Q][family][m][a] for family in {phi, phi', psi}
constexpr int BASIS_STRIDE_Q = NFAM * MAXN * MAXQ;
constexpr int TAB_BASIS = TAB_PACK + PACKED_SIZE;
// Tail rows of the learned-order check: for each Q, the discrete Legendre
// coefficient weights of the four highest degrees a Q-point rule resolves,
// tailw[Q][j][a] = (2d+1)/2 w_a L_d(x_a), d = Q-1-j (zero when d < 0).
constexpr int TAILW_STRIDE_Q = 4 * MAXQ;
constexpr int TAB_TAILW = TAB_BASIS + (MAXQ + 1) * BASIS_STRIDE_Q;
// Point tables of the sum-factorized direct quadrature: for order N and the
// 2N-point Gauss rule, pt[N][t][m1][m2][a] = w_a X_m1(x_a) Y_m2(x_a) (type
// t = 3X+Y), in the [t][m1][m2][.] layout of the linearization table.
constexpr int PT_STRIDE_N = NTYPE * MAXN * MAXN * KPAD;
constexpr int TAB_PT = TAB_TAILW + (MAXQ + 1) * TAILW_STRIDE_Q;
constexpr int TAB_SIZE = TAB_PT + (MAXN + 1) * PT_STRIDE_N;
// Per (element, field) tail record written by the moment stage in learned
// mode: env[axis][j] at axis*4+j (axis 0 = u, 1 = v, 2 = w), the scale of
// the tensor the axis was examined on at 12+axis.
constexpr int TAIL_REC = 16;
// the moment stage carries the four tail rows beside the 2N-1 moment rows
// in one 16-row matrix-core tile: orders up to 6
constexpr int TAIL_MAXN = 6;

// the split path samples at most this many points per axis (one MFMA
// K-block of 16)
constexpr int SPLIT_MAXQ = 16;

// Mirrors of the public enums and status bits (include/p2s.h).
enum MatKind : int { MAT_SINCOSEXP = 0, MAT_ROTDIAG = 1, MAT_PLANEWAVE = 2, ALPHA_SAMPLED = 3 };
constexpr uint32_t P2S_STATUS_DETJ_BIT = 1u;
constexpr uint32_t P2S_STATUS_NONFINITE_BIT = 2u;
constexpr uint32_t P2S_STATUS_FALLBACK_BIT = 4u;

// Learned quadrature order: network shape and parameter layout (FP32).
// Weights are stored input-major, W[i][o]: y_o = sum_i x_i W[i][o] + b_o.
constexpr int MLP_IN = 85, MLP_H = 128, MLP_NCLS = 19, MLP_OUT = 3 * MLP_NCLS;
constexpr int MLP_KMIN = 6, MLP_KMAX = MLP_KMIN + MLP_NCLS - 1;  // K in {6..24}
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_IN * MLP_H;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_OUT;
constexpr int MLP_PARAMS = MLP_OFF_B3 + MLP_OUT;

// Work item of the persistent contraction: rows (m1, ., .) of component
// `comp` of element e.
struct WorkItem {
    int32_t e;
    int16_t comp, m1;
};

// Per-element descriptor used by every kernel.
struct ElemDesc {
    int32_t N, Qu, Qv, Qw;
    int64_t out_off;    // start of the element's block in out (doubles)
    int64_t alpha_off;  // start of its coupling samples in the workspace
    int64_t mom_off;    // start of its moment tensors in the workspace
};

// Problem shape helpers (host and device).
P2S_HD constexpr int num_fields(int problem) { return problem == 0 ? 7 : 12; }
P2S_HD constexpr int num_comp(int problem) { return problem == 0 ? 1 : 3; }
// dimension of component g along axis ax
P2S_HD constexpr int comp_dim(int problem, int N, int g, int ax)
{
    return (problem == 1 && g == ax) ? N - 1 : N;
}
P2S_HD constexpr int comp_size(int problem, int N, int g)
{
    return comp_dim(problem, N, g, 0) * comp_dim(problem, N, g, 1) * comp_dim(problem, N, g, 2);
}
P2S_HD constexpr int comp_offset(int problem, int N, int g)
{
    int o = 0;
    for (int h = 0; h < g; ++h) o += comp_size(problem, N, h);
    return o;
}
P2S_HD constexpr int num_dofs(int problem, int N)
{
    return comp_offset(problem, N, num_comp(problem));
}

}  // namespace p2s
