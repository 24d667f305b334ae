// p2s_kernels.hip -- HIP kernels of the product-to-sum element-matrix fill
// for CDNA4 (gfx950, wave64).
//
// Stages (paper Section II):
//   k_coupling   geometry + coupling factor alpha_s at every Gauss point
//                (the integrand factor of eq. (2) that is not separable);
//   k_moments    the 3-D integrals of eq. (4), I_s[k,l,q], by sum
//                factorization over the three axes;
//   k_contract   eq. (4): M = sum_s sum_{k,l,q} Cu Cv Cw I_s, mode by mode,
//                with the linearization coefficients of eq. (3).
#include <hip/hip_runtime.h>

#include <utility>

#include "p2s_internal.h"
#include "p2s_kernels.h"

namespace p2s {

// ---------------------------------------------------------------------------
// Structural sparsity of the linearization tables (degrees k with a nonzero
// coefficient), evaluated at compile time.
struct MaskTable {
    uint32_t m[NTYPE][MAXN][MAXN];
    constexpr MaskTable() : m()
    {
        for (int t = 0; t < NTYPE; ++t)
            for (int a = 0; a < MAXN; ++a)
                for (int b = 0; b < MAXN; ++b) m[t][a][b] = prod_mask(t / 3, a, t % 3, b);
    }
};
__constant__ MaskTable c_masks = MaskTable();

// ---------------------------------------------------------------------------
// Geometry and coupling factors.

__device__ __forceinline__ void lagrange3(double t, double l[3], double d[3])
{
    l[0] = 0.5 * t * (t - 1.0);
    l[1] = 1.0 - t * t;
    l[2] = 0.5 * t * (t + 1.0);
    d[0] = t - 0.5;
    d[1] = -2.0 * t;
    d[2] = t + 0.5;
}

// eps(x) as a symmetric tensor (e00 e11 e22 e01 e02 e12).
__device__ __forceinline__ void permittivity(int kind, const double *p, const double x[3], double e[6])
{
    if (kind == MAT_ROTDIAG) {
        const double kx = p[9] * x[0] + p[10] * x[1] + p[11] * x[2];
        const double c3 = 2.0943951023931954923;  // 2 pi / 3
        double d[3];
        d[0] = 1.0 + 0.5 * sin(kx);
        d[1] = 1.0 + 0.5 * sin(kx + c3);
        d[2] = 1.0 + 0.5 * sin(kx + 2.0 * c3);
        // eps_rc = sum_a R[a][r] d_a R[a][c]
        const int rr[6] = {0, 1, 2, 0, 0, 1}, cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) v = fma(p[3 * a + rr[s]] * d[a], p[3 * a + cc[s]], v);
            e[s] = v;
        }
        return;
    }
    double v;
    if (kind == MAT_PLANEWAVE)
        v = 1.0 + 0.8 * sin(p[0] * x[0] + p[1] * x[1] + p[2] * x[2] + p[3]);
    else
        v = 1.0 + 0.5 * sin(p[0] * x[0]) * cos(p[0] * x[1]) * exp(-x[2]);
    e[0] = e[1] = e[2] = v;
    e[3] = e[4] = e[5] = 0.0;
}

// Coupling fields at reference point (u,v,w) of an element with nodes X.
// Returns det J; writes F fields (packed order of P2S_ALPHA_SAMPLED).
template <int PROB>
__device__ __forceinline__ double coupling_point(const double *X, int kind, const double *mp,
                                                 double u, double v, double w, double *f)
{
    double lu[3], du[3], lv[3], dv[3], lw[3], dw[3];
    lagrange3(u, lu, du);
    lagrange3(v, lv, dv);
    lagrange3(w, lw, dw);
    double x[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // contract the u-direction first
            double s[3], su[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double *Xr = X + 3 * (3 * j + 9 * k) + r;
                s[r] = lu[0] * Xr[0] + lu[1] * Xr[3] + lu[2] * Xr[6];
                su[r] = du[0] * Xr[0] + du[1] * Xr[3] + du[2] * Xr[6];
            }
            const double a0 = lv[j] * lw[k], a1 = dv[j] * lw[k], a2 = lv[j] * dw[k];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                x[r] = fma(a0, s[r], x[r]);
                J[r][0] = fma(a0, su[r], J[r][0]);
                J[r][1] = fma(a1, s[r], J[r][1]);
                J[r][2] = fma(a2, s[r], J[r][2]);
            }
        }
    // adjugate: adj[a][b] = cofactor[b][a]
    double adj[3][3];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const double rdet = 1.0 / det;
    double e[6];
    permittivity(kind, mp, x, e);
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    if (PROB == 0) {
        // eps det J J^-1 J^-T = eps adj adj^T / det
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const double g = adj[ia[s]][0] * adj[ib[s]][0] + adj[ia[s]][1] * adj[ib[s]][1] +
                             adj[ia[s]][2] * adj[ib[s]][2];
            f[s] = e[0] * g * rdet;
        }
        f[6] = e[0] * det;
    } else {
        // curl-curl: J^T J / det
#pragma unroll
        for (int s = 0; s < 6; ++s)
            f[s] = (J[0][ia[s]] * J[0][ib[s]] + J[1][ia[s]] * J[1][ib[s]] + J[2][ia[s]] * J[2][ib[s]]) * rdet;
        // mass: det J^-1 eps J^-T = adj eps adj^T / det
        double E3[3][3] = {{e[0], e[3], e[4]}, {e[3], e[1], e[5]}, {e[4], e[5], e[2]}};
        double T[3][3];  // adj * eps
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                T[a][c] = adj[a][0] * E3[0][c] + adj[a][1] * E3[1][c] + adj[a][2] * E3[2][c];
#pragma unroll
        for (int s = 0; s < 6; ++s)
            f[6 + s] = (T[ia[s]][0] * adj[ib[s]][0] + T[ia[s]][1] * adj[ib[s]][1] +
                        T[ia[s]][2] * adj[ib[s]][2]) * rdet;
    }
    return det;
}

// One workgroup per element: coupling fields at all Gauss points,
// alpha[alpha_off + f*P + (a*Qv+b)*Qw + c], unweighted.
template <int PROB>
__global__ __launch_bounds__(256) void k_coupling(const ElemDesc *__restrict__ desc, int64_t e0,
                                                  const double *__restrict__ nodes,
                                                  const double *__restrict__ mat, int kind,
                                                  int mat_stride, const double *__restrict__ tab,
                                                  double *__restrict__ alpha,
                                                  uint32_t *__restrict__ status)
{
    constexpr int F = num_fields(PROB);
    const int64_t e = e0 + blockIdx.x;
    const ElemDesc d = desc[e];
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw;
    const int P = Qu * Qv * Qw;
    double *dst = alpha + d.alpha_off;
    __shared__ double X[81];
    __shared__ double mp[16];
    if (kind == ALPHA_SAMPLED) {
        const double *src = mat + e * (int64_t)(F * P);
        for (int i = threadIdx.x; i < F * P; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x == 0) status[e] = 0u;
        return;
    }
    if (threadIdx.x < 81) X[threadIdx.x] = nodes[e * 81 + threadIdx.x];
    if (threadIdx.x < mat_stride) mp[threadIdx.x] = mat[e * mat_stride + threadIdx.x];
    __syncthreads();
    const double *gu = tab + TAB_GX + Qu * MAXQ;
    const double *gv = tab + TAB_GX + Qv * MAXQ;
    const double *gw = tab + TAB_GX + Qw * MAXQ;
    int bad = 0;
    for (int pt = threadIdx.x; pt < P; pt += blockDim.x) {
        const int c = pt % Qw;
        const int b = (pt / Qw) % Qv;
        const int a = pt / (Qw * Qv);
        double f[F];
        const double det = coupling_point<PROB>(X, kind, mp, gu[a], gv[b], gw[c], f);
        bad |= !(det > 0.0);
#pragma unroll
        for (int s = 0; s < F; ++s) dst[(int64_t)s * P + pt] = f[s];
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) status[e] = bad ? P2S_STATUS_DETJ_BIT : 0u;
}

// ---------------------------------------------------------------------------
// Moments, eq. (4): I[k][l][q] = sum_{a,b,c} Wu[k][a] Wv[l][b] Ww[q][c] alpha[a][b][c]
// with W[k][a] = w_a L_k(x_a), as three passes (contract w, then v, then u).
// One workgroup per (element, field); the sizes are runtime, the degree
// count K = 2N-1 selects a register-blocked instantiation.

template <int K>
__device__ void moments_body(const ElemDesc &d, int f, int F, const double *__restrict__ alpha,
                             const double *__restrict__ tab, double *__restrict__ mom, double *sm,
                             int p2off)
{
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw;
    const int P = Qu * Qv * Qw;
    const double *A = alpha + d.alpha_off + (int64_t)f * P;
    const double *Wu = tab + TAB_LEGW + Qu * LEGW_STRIDE_Q;
    const double *Wv = tab + TAB_LEGW + Qv * LEGW_STRIDE_Q;
    const double *Ww = tab + TAB_LEGW + Qw * LEGW_STRIDE_Q;
    constexpr int KS = K + 1;  // LDS row stride
    double *P1 = sm;          // [Qu*Qv][KS]   (q)
    double *P2 = sm + p2off;  // [Qu][K][KS]   (l, q)
    const int tid = threadIdx.x, nt = blockDim.x;
    // pass 1: contract w
    for (int ab = tid; ab < Qu * Qv; ab += nt) {
        double acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = 0.0;
        const double *Ar = A + (int64_t)ab * Qw;
        for (int c = 0; c < Qw; ++c) {
            const double x = Ar[c];
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = fma(Ww[q * MAXQ + c], x, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < K; ++q) P1[ab * KS + q] = acc[q];
    }
    __syncthreads();
    // pass 2: contract v
    for (int aq = tid; aq < Qu * K; aq += nt) {
        const int a = aq / K, q = aq - (aq / K) * K;
        double acc[K];
#pragma unroll
        for (int l = 0; l < K; ++l) acc[l] = 0.0;
        for (int b = 0; b < Qv; ++b) {
            const double x = P1[(a * Qv + b) * KS + q];
#pragma unroll
            for (int l = 0; l < K; ++l) acc[l] = fma(Wv[l * MAXQ + b], x, acc[l]);
        }
#pragma unroll
        for (int l = 0; l < K; ++l) P2[(a * K + l) * KS + q] = acc[l];
    }
    __syncthreads();
    // pass 3: contract u
    double *I = mom + d.mom_off + (int64_t)f * K * K * K;
    for (int lq = tid; lq < K * K; lq += nt) {
        const int l = lq / K, q = lq - (lq / K) * K;
        double acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = 0.0;
        for (int a = 0; a < Qu; ++a) {
            const double x = P2[(a * K + l) * KS + q];
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = fma(Wu[k * MAXQ + a], x, acc[k]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) I[k * K * K + lq] = acc[k];
    }
}

__global__ __launch_bounds__(256) void k_moments(const ElemDesc *__restrict__ desc, int64_t e0, int F,
                                                 const double *__restrict__ alpha,
                                                 const double *__restrict__ tab,
                                                 double *__restrict__ mom, int p2off)
{
    extern __shared__ double sm[];
    const ElemDesc d = desc[e0 + blockIdx.x];
    const int f = blockIdx.y;
    switch (d.N) {
    case 2: moments_body<3>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 3: moments_body<5>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 4: moments_body<7>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 5: moments_body<9>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 6: moments_body<11>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 7: moments_body<13>(d, f, F, alpha, tab, mom, sm, p2off); break;
    case 8: moments_body<15>(d, f, F, alpha, tab, mom, sm, p2off); break;
    default: break;
    }
}

// LDS layout of k_moments for the largest order and rule of a plan:
// P1 [Qu*Qv][KS] followed by P2 [Qu][K][KS], KS = K+1.
int moments_p2_offset(int maxN, int maxQuv) { return maxQuv * (2 * maxN); }
size_t moments_smem_bytes(int maxN, int maxQu, int maxQuv)
{
    const int K = 2 * maxN - 1, KS = K + 1;
    return sizeof(double) * (size_t)(moments_p2_offset(maxN, maxQuv) + maxQu * K * KS);
}

// ---------------------------------------------------------------------------
// Contraction, eq. (4), mode by mode.  One workgroup per (element, row
// component i, first-axis test index m1): it produces the full rows
// (m1, n1, p1) of component i, looping over column components j.  For the
// coupling terms s of block (i,j):
//   stage A  A_s[m2][l][q] = sum_k Cu[m1][m2][k] I_s[k][l][q]     (LDS)
//            one thread per (s, l, q): each moment is loaded once and
//            reused for every m2; coefficients are uniform (scalar loads)
//   stage B  B[q]          = sum_l Cv[n1][n2][l] A_s[m2][l][q]    (registers)
//   stage C  acc[p1][p2]  += sum_q Cw[p1][p2][q] B[q]             (registers)
// Stages B and C run one lane per (m2, n1, n2).  Stage C's sparsity is
// resolved at compile time per family pair, and its coefficients come from
// a packed table in consumption order (scalar loads at immediate offsets).

struct PackIndex {
    int16_t before[MAXN + 1][NTYPE][MAXN][MAXN];
    constexpr PackIndex() : before()
    {
        for (int n = 2; n <= MAXN; ++n)
            for (int t = 0; t < NTYPE; ++t) {
                int c = 0;
                for (int p1 = 0; p1 < fam_dim(t / 3, n); ++p1)
                    for (int p2 = 0; p2 < fam_dim(t % 3, n); ++p2) {
                        before[n][t][p1][p2] = (int16_t)c;
                        c += popcount32(prod_mask(t / 3, p1, t % 3, p2));
                    }
            }
    }
};
constexpr PackIndex kPackIndex = PackIndex();

struct PackOffsets {
    int off[MAXN + 1][NTYPE];
    constexpr PackOffsets() : off()
    {
        int o = 0;  // same running layout as packed_offset()
        for (int n = 2; n <= MAXN; ++n)
            for (int t = 0; t < NTYPE; ++t) {
                off[n][t] = o;
                o += (packed_count(t / 3, t % 3, n) + 1) & ~1;
            }
    }
};
constexpr PackOffsets kPackOffsets = PackOffsets();

template <int PROB, int N>
struct CShape {
    static constexpr int K = 2 * N - 1;
    static constexpr int KS = K + 1;  // LDS row stride (16-byte aligned rows)
    static constexpr int NC = num_comp(PROB);
    static constexpr int NDOF = num_dofs(PROB, N);
    static constexpr int NT = PROB == 0 ? 10 : 5;  // terms per block
    static constexpr int TERM_DOUBLES = N * K * KS;
    static constexpr int G = (NT * TERM_DOUBLES * 8 <= 65536) ? NT : 65536 / (TERM_DOUBLES * 8);
    static constexpr int SA = ((K * K + 63) / 64) * 64;  // stage-A threads per term
    static constexpr int max_tasks()
    {
        int m = 0;
        for (int i = 0; i < NC; ++i)
            for (int j = 0; j < NC; ++j) {
                int t = comp_dim(PROB, N, j, 0) * comp_dim(PROB, N, i, 1) * comp_dim(PROB, N, j, 1);
                m = t > m ? t : m;
            }
        return m;
    }
    static constexpr int THREADS = ((max_tasks() + 63) / 64) * 64;
    static constexpr int ROWS_PER_ELEM()
    {
        int r = 0;
        for (int i = 0; i < NC; ++i) r += comp_dim(PROB, N, i, 0);
        return r;
    }
};

// constant address space: loads through it become scalar (SMEM) loads
typedef __attribute__((address_space(4))) const double cdouble;

template <int N, int X, int Y, int P1, int P2>
__device__ __forceinline__ void stage_c_one(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                            cdouble *__restrict__ tb)
{
    if constexpr (P1 < fam_dim(X, N) && P2 < fam_dim(Y, N)) {
        constexpr uint32_t msk = prod_mask(X, P1, Y, P2);
        constexpr int base = kPackIndex.before[N][3 * X + Y][P1][P2];
#pragma unroll
        for (int q = 0; q < 2 * N - 1; ++q)
            if ((msk >> q) & 1u)
                acc[P1][P2] = fma(tb[base + popcount32(msk & ((1u << q) - 1u))], bv[q], acc[P1][P2]);
    }
}

template <int N, int X, int Y, int... Is>
__device__ __forceinline__ void stage_c_all(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                            cdouble *__restrict__ tb, std::integer_sequence<int, Is...>)
{
    (stage_c_one<N, X, Y, Is / N, Is % N>(acc, bv, tb), ...);
}

template <int N, int X, int Y>
__device__ __forceinline__ void stage_c(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                        const double *__restrict__ pack)
{
    constexpr int off = kPackOffsets.off[N][3 * X + Y];
    static_assert(off == packed_offset(N, X, Y), "packed table layout");
    cdouble *tb = (cdouble *)(pack + off);
    // keep the table base in SGPRs and opaque to loop-invariant motion, so
    // every coefficient is a scalar load at an immediate offset
    asm volatile("" : "+s"(tb));
    stage_c_all<N, X, Y>(acc, bv, tb, std::make_integer_sequence<int, N * N>{});
}

template <int PROB, int N>
__device__ __forceinline__ void stage_c_dispatch(int tw, double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                                 const double *__restrict__ pack)
{
    if constexpr (PROB == 0) {
        switch (tw) {
        case 3 * PHI + PHI: stage_c<N, PHI, PHI>(acc, bv, pack); break;
        case 3 * PHI + DPHI: stage_c<N, PHI, DPHI>(acc, bv, pack); break;
        case 3 * DPHI + PHI: stage_c<N, DPHI, PHI>(acc, bv, pack); break;
        default: stage_c<N, DPHI, DPHI>(acc, bv, pack); break;
        }
    } else {
        switch (tw) {
        case 3 * PHI + PHI: stage_c<N, PHI, PHI>(acc, bv, pack); break;
        case 3 * PHI + DPHI: stage_c<N, PHI, DPHI>(acc, bv, pack); break;
        case 3 * PHI + PSI: stage_c<N, PHI, PSI>(acc, bv, pack); break;
        case 3 * DPHI + PHI: stage_c<N, DPHI, PHI>(acc, bv, pack); break;
        case 3 * DPHI + DPHI: stage_c<N, DPHI, DPHI>(acc, bv, pack); break;
        case 3 * DPHI + PSI: stage_c<N, DPHI, PSI>(acc, bv, pack); break;
        case 3 * PSI + PHI: stage_c<N, PSI, PHI>(acc, bv, pack); break;
        case 3 * PSI + DPHI: stage_c<N, PSI, DPHI>(acc, bv, pack); break;
        default: stage_c<N, PSI, PSI>(acc, bv, pack); break;
        }
    }
}

// Work-group id -> logical work item, so that consecutive items (the row
// tiles of one element, which share its moment tensors) run on the same XCD:
// the hardware deals work-group ids round-robin over the 8 XCDs.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t total_padded)
{
    const int64_t per = total_padded >> 3;
    return (w & 7) * per + (w >> 3);
}

// Store one lane's p-block: direct rows (m1,n1,p1) x cols (m2,n2,p2), and,
// for the part above the diagonal, its mirror image (the matrix is
// symmetric), whose rows are (m2,n2,p2) and whose columns (m1,n1,p1).
template <int N, int NDOF>
__device__ __forceinline__ void store_block(double *__restrict__ base, int row0, int col0, int Np_i,
                                            int Np_j, bool mirror, const double (&acc)[N][N], bool &bad)
{
    double *o = base + (int64_t)row0 * NDOF + col0;
    const bool v2 = (NDOF % 2 == 0) && ((reinterpret_cast<uintptr_t>(o) & 15u) == 0);
#pragma unroll
    for (int p1 = 0; p1 < N; ++p1) {
        if (p1 >= Np_i) continue;
#pragma unroll
        for (int p2 = 0; p2 < N; ++p2) bad |= (p2 < Np_j) && !isfinite(acc[p1][p2]);
        double *op = o + (int64_t)p1 * NDOF;
        if (v2 && (Np_j % 2 == 0)) {
#pragma unroll
            for (int p2 = 0; p2 + 1 < N; p2 += 2)
                if (p2 + 1 < Np_j) *reinterpret_cast<double2 *>(op + p2) = make_double2(acc[p1][p2], acc[p1][p2 + 1]);
        } else {
#pragma unroll
            for (int p2 = 0; p2 < N; ++p2)
                if (p2 < Np_j) op[p2] = acc[p1][p2];
        }
    }
    if (!mirror) return;
    double *t = base + (int64_t)col0 * NDOF + row0;
    const bool t2 = (NDOF % 2 == 0) && ((reinterpret_cast<uintptr_t>(t) & 15u) == 0);
#pragma unroll
    for (int p2 = 0; p2 < N; ++p2) {
        if (p2 >= Np_j) continue;
        double *tp = t + (int64_t)p2 * NDOF;
        if (t2 && (Np_i % 2 == 0)) {
#pragma unroll
            for (int p1 = 0; p1 + 1 < N; p1 += 2)
                if (p1 + 1 < Np_i) *reinterpret_cast<double2 *>(tp + p1) = make_double2(acc[p1][p2], acc[p1 + 1][p2]);
        } else {
#pragma unroll
            for (int p1 = 0; p1 < N; ++p1)
                if (p1 < Np_i) tp[p1] = acc[p1][p2];
        }
    }
}

template <int PROB, int N>
__global__ __launch_bounds__((CShape<PROB, N>::THREADS)) void k_contract(
    const ElemDesc *__restrict__ desc, const int32_t *__restrict__ elist, int64_t e0, int64_t nitems,
    int64_t padded, const double *__restrict__ tab, const BlockDesc *__restrict__ blocks,
    const double *__restrict__ mom, double *__restrict__ out, uint32_t *__restrict__ status,
    double sK, double sM)
{
    using S = CShape<PROB, N>;
    constexpr int K = S::K, KS = S::KS, NC = S::NC, NDOF = S::NDOF, G = S::G;
    const int64_t item = xcd_remap(blockIdx.x, padded);
    if (item >= nitems) return;
    constexpr int R = S::ROWS_PER_ELEM();
    const int64_t eidx = e0 + item / R;
    const int64_t e = elist ? (int64_t)elist[eidx] : eidx;
    int rr = (int)(item % R);
    int i = 0;
    while (i + 1 < NC && rr >= comp_dim(PROB, N, i, 0)) {
        rr -= comp_dim(PROB, N, i, 0);
        ++i;
    }
    const int m1 = rr;
    const ElemDesc d = desc[e];
    const double *lin = tab + TAB_LIN;
    const double *pack = tab + TAB_PACK;
    const double *I0 = mom + d.mom_off;
    double *obase = out + d.out_off;
    __shared__ double Abuf[G][S::TERM_DOUBLES];
    const int tid = threadIdx.x;
    const int Nn_i = comp_dim(PROB, N, i, 1), Np_i = comp_dim(PROB, N, i, 2);
    const int rowbase = comp_offset(PROB, N, i) + m1 * Nn_i * Np_i;
    bool bad = false;

    // symmetric: blocks j >= i; inside the diagonal block only m2 >= m1
    for (int j = i; j < NC; ++j) {
        const int Nm_j = comp_dim(PROB, N, j, 0), Nn_j = comp_dim(PROB, N, j, 1),
                  Np_j = comp_dim(PROB, N, j, 2);
        const int m2lo = (j == i) ? m1 : 0;
        const int nm = Nm_j - m2lo;
        const int T = nm * Nn_i * Nn_j;
        const bool active = tid < T;
        const int n2 = tid % Nn_j;
        const int m2 = m2lo + (tid / Nn_j) % nm;
        const int n1 = tid / (Nn_j * nm);
        double acc[N][N];
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) acc[a][b] = 0.0;
        double bsum[K];
#pragma unroll
        for (int q = 0; q < K; ++q) bsum[q] = 0.0;
        const BlockDesc *bd = blocks + (i * 3 + j);
        const int ngroup = bd->ngroup;
        for (int g0 = 0; g0 < ngroup; g0 += G) {
            const int ng = ngroup - g0 < G ? ngroup - g0 : G;
            // stage A: worker w -> (group gl, moment entry lq); gl is wave-uniform
            for (int w = tid; w < ng * S::SA; w += S::THREADS) {
                const int gl = w / S::SA;
                const int lq = w - gl * S::SA;
                if (lq < K * K) {
                    double a[N];
#pragma unroll
                    for (int mm = 0; mm < N; ++mm) a[mm] = 0.0;
                    const int s0 = bd->gstart[g0 + gl], s1 = bd->gstart[g0 + gl + 1];
                    for (int s = s0; s < s1; ++s) {
                        const Term t = bd->t[s];
                        const double sc = (t.scale ? sM : sK) * (double)t.sign;
                        const double *I = I0 + (int64_t)t.field * K * K * K + lq;
                        double v[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) v[k] = I[k * K * K];
                        const double *Cu = lin + t.tu * LIN_STRIDE_T + m1 * LIN_STRIDE_M1;
#pragma unroll
                        for (int mm = 0; mm < N; ++mm) {
                            if (mm >= m2lo && mm < Nm_j) {
                                const uint32_t mk = c_masks.m[t.tu][m1][mm];
                                double x = 0.0;
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    if ((mk >> k) & 1u) x = fma(Cu[mm * KPAD + k], v[k], x);
                                a[mm] = fma(sc, x, a[mm]);
                            }
                        }
                    }
                    const int l = lq / K, q = lq - (lq / K) * K;
                    double *Ab = Abuf[gl] + l * KS + q;
#pragma unroll
                    for (int mm = 0; mm < N; ++mm)
                        if (mm >= m2lo && mm < Nm_j) Ab[mm * K * KS] = a[mm];
                }
            }
            __syncthreads();
            if (active) {
                for (int gl = 0; gl < ng; ++gl) {
                    const Term t = bd->t[bd->gstart[g0 + gl]];
                    // stage B, summed over the groups of one tw run
                    uint32_t ml = c_masks.m[t.tv][n1][n2];
                    const double *Cv = lin + t.tv * LIN_STRIDE_T + n1 * LIN_STRIDE_M1 + n2 * KPAD;
                    const double *Arow = Abuf[gl] + m2 * K * KS;
                    while (ml) {
                        const int l = __ffs(ml) - 1;
                        ml &= ml - 1u;
                        const double c = Cv[l];
                        const double2 *a2 = reinterpret_cast<const double2 *>(Arow + l * KS);
#pragma unroll
                        for (int h = 0; h < KS / 2; ++h) {
                            const double2 x = a2[h];
                            bsum[2 * h] = fma(c, x.x, bsum[2 * h]);
                            if (2 * h + 1 < K) bsum[2 * h + 1] = fma(c, x.y, bsum[2 * h + 1]);
                        }
                    }
                    if (bd->cflag[g0 + gl]) {
                        // stage C
                        stage_c_dispatch<PROB, N>(t.tw, acc, bsum, pack);
#pragma unroll
                        for (int q = 0; q < K; ++q) bsum[q] = 0.0;
                    }
                }
            }
            __syncthreads();
        }
        if (active) {
            const int row0 = rowbase + n1 * Np_i;
            const int col0 = comp_offset(PROB, N, j) + (m2 * Nn_j + n2) * Np_j;
            store_block<N, NDOF>(obase, row0, col0, Np_i, Np_j, j > i || m2 > m1, acc, bad);
        }
    }
    if (__syncthreads_or(bad) && tid == 0) atomicOr(status + e, P2S_STATUS_NONFINITE_BIT);
}

// ---------------------------------------------------------------------------
// Host-side launchers.

void launch_coupling(int problem, const ElemDesc *desc, int64_t e0, int64_t count,
                     const double *nodes, const double *mat, int kind, int mat_stride,
                     const double *tab, double *alpha, uint32_t *status, hipStream_t st)
{
    if (count <= 0) return;
    if (problem == 0)
        hipLaunchKernelGGL(k_coupling<0>, dim3((unsigned)count), dim3(256), 0, st, desc, e0, nodes,
                           mat, kind, mat_stride, tab, alpha, status);
    else
        hipLaunchKernelGGL(k_coupling<1>, dim3((unsigned)count), dim3(256), 0, st, desc, e0, nodes,
                           mat, kind, mat_stride, tab, alpha, status);
}

void launch_moments(int problem, int maxN, int maxQu, int maxQuv, const ElemDesc *desc, int64_t e0,
                    int64_t count, const double *alpha, const double *tab, double *mom, hipStream_t st)
{
    if (count <= 0) return;
    const int F = num_fields(problem);
    hipLaunchKernelGGL(k_moments, dim3((unsigned)count, F), dim3(256),
                       moments_smem_bytes(maxN, maxQu, maxQuv), st, desc, e0, F, alpha, tab, mom,
                       moments_p2_offset(maxN, maxQuv));
}

int prepare_kernels()
{
    // k_moments may need more than the default 64 KiB of LDS
    hipError_t r = hipFuncSetAttribute((const void *)k_moments,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return r == hipSuccess ? 0 : -1;
}

template <int PROB, int N>
static void launch_contract_t(const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                              const double *tab, const BlockDesc *terms, const double *mom, double *out,
                              uint32_t *status, double sK, double sM, hipStream_t st)
{
    using S = CShape<PROB, N>;
    const int64_t nitems = count * S::ROWS_PER_ELEM();
    const int64_t padded = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((k_contract<PROB, N>), dim3((unsigned)padded), dim3(S::THREADS), 0, st, desc, elist,
                       e0, nitems, padded, tab, terms, mom, out, status, sK, sM);
}

int launch_contract(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0,
                    int64_t count, const double *tab, const BlockDesc *terms, const double *mom, double *out,
                    uint32_t *status, double sK, double sM, hipStream_t st)
{
    if (count <= 0) return 0;
#define P2S_CASE(P, n)                                                                           \
    if (problem == P && N == n) {                                                                \
        launch_contract_t<P, n>(desc, elist, e0, count, tab, terms, mom, out, status, sK, sM, st); \
        return 0;                                                                                \
    }
    P2S_CASE(0, 2) P2S_CASE(0, 3) P2S_CASE(0, 4) P2S_CASE(0, 5) P2S_CASE(0, 6) P2S_CASE(0, 7) P2S_CASE(0, 8)
    P2S_CASE(1, 2) P2S_CASE(1, 3) P2S_CASE(1, 4) P2S_CASE(1, 5) P2S_CASE(1, 6) P2S_CASE(1, 7) P2S_CASE(1, 8)
#undef P2S_CASE
    return -1;
}

}  // namespace p2s
