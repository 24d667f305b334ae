// p2s_direct.hip -- direct quadrature of eq. (2) on the GPU: every entry
// M_ij = sum over Gauss points W * (test features)_i . alpha . (trial features)_j,
// without the product-to-sum identity.  This is the method the paper
// compares against (Section IV: direct numerical integration); it shares the
// coupling-factor stage with the product-to-sum path and uses the same
// output layout.
//
// One workgroup per (element, 64x64 output tile) above the diagonal; the
// tile below the diagonal is stored as the mirror image.  Points are taken
// in chunks of 8: for each chunk the basis features of the tile's 64 test
// rows and the alpha-weighted features of its 64 trial columns are built in
// LDS, then every thread accumulates a 4x4 register tile.
#include <hip/hip_runtime.h>

#include "p2s_internal.h"
#include "p2s_kernels.h"

namespace p2s {

constexpr int DT = 64;   // tile edge
constexpr int DPC = 8;   // points per chunk
constexpr int DF = 6;    // features per point (vector: curl 3 + value 3; scalar: grad 3 + value)

// Features of dof `r` at point (a,b,c): vector problem -> reference curl
// (3) and E_hat (3); scalar -> reference gradient (3) and value (1).
// bas[ax] is the 1-D table of axis ax's rule: [family][m][point].
template <int PROB>
__device__ __forceinline__ void dof_features(int N, int r, const int pt[3], const double *const bas[3],
                                             double f[DF])
{
    auto B = [&](int ax, int fam, int m) { return bas[ax][(fam * MAXN + m) * MAXQ + pt[ax]]; };
    if (PROB == 0) {
        const int m = r / (N * N), n = (r / N) % N, p = r % N;
        const double u = B(0, PHI, m), v = B(1, PHI, n), w = B(2, PHI, p);
        const double du = B(0, DPHI, m), dv = B(1, DPHI, n), dw = B(2, DPHI, p);
        f[0] = du * v * w;
        f[1] = u * dv * w;
        f[2] = u * v * dw;
        f[3] = u * v * w;
        f[4] = f[5] = 0.0;
        return;
    }
    int g = 0, off = 0;
    while (g < 2 && r >= off + comp_size(1, N, g)) {
        off += comp_size(1, N, g);
        ++g;
    }
    const int loc = r - off;
    const int d1 = comp_dim(1, N, g, 1), d2 = comp_dim(1, N, g, 2);
    const int idx[3] = {loc / (d1 * d2), (loc / d2) % d1, loc % d2};
    double val[3], der[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (ax == g) {
            val[ax] = B(ax, PSI, idx[ax]);
            der[ax] = 0.0;
        } else {
            val[ax] = B(ax, PHI, idx[ax]);
            der[ax] = B(ax, DPHI, idx[ax]);
        }
    }
    const double fv = val[0] * val[1] * val[2];
    const double fu = der[0] * val[1] * val[2];
    const double fvv = val[0] * der[1] * val[2];
    const double fw = val[0] * val[1] * der[2];
    // reference curl of f e_g
    f[0] = g == 0 ? 0.0 : (g == 1 ? -fw : fvv);
    f[1] = g == 0 ? fw : (g == 1 ? 0.0 : -fu);
    f[2] = g == 0 ? -fvv : (g == 1 ? fu : 0.0);
    f[3] = g == 0 ? fv : 0.0;
    f[4] = g == 1 ? fv : 0.0;
    f[5] = g == 2 ? fv : 0.0;
}

template <int PROB>
__global__ __launch_bounds__(256) void k_direct(const ElemDesc *__restrict__ desc, int64_t e0, int ntile,
                                                const double *__restrict__ tab, const double *__restrict__ alpha,
                                                double *__restrict__ out, double sK, double sM)
{
    constexpr int F = num_fields(PROB);
    const int64_t e = e0 + blockIdx.x / (ntile * (ntile + 1) / 2);
    int t = blockIdx.x % (ntile * (ntile + 1) / 2);
    int rt = 0;
    while (t >= ntile - rt) {
        t -= ntile - rt;
        ++rt;
    }
    const int ct = rt + t;  // ct >= rt
    const ElemDesc d = desc[e];
    const int N = d.N, Qu = d.Qu, Qv = d.Qv, Qw = d.Qw;
    const int P = Qu * Qv * Qw;
    const int nd = num_dofs(PROB, N);
    const double *A = alpha + d.alpha_off;
    const double *gwu = tab + TAB_GW + Qu * MAXQ, *gwv = tab + TAB_GW + Qv * MAXQ, *gww = tab + TAB_GW + Qw * MAXQ;
    const double *const bas[3] = {tab + TAB_BASIS + Qu * BASIS_STRIDE_Q, tab + TAB_BASIS + Qv * BASIS_STRIDE_Q,
                                  tab + TAB_BASIS + Qw * BASIS_STRIDE_Q};
    __shared__ __attribute__((aligned(32))) double Ft[DPC][DF][DT];
    __shared__ __attribute__((aligned(32))) double Gt[DPC][DF][DT];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double acc[4][4] = {};
    for (int p0 = 0; p0 < P; p0 += DPC) {
        // features of the tile's test rows (Ft) and trial columns (Gt)
        for (int x = tid; x < 2 * DPC * DT; x += 256) {
            const int side = x / (DPC * DT);
            const int pp = (x / DT) % DPC;
            const int rr = x % DT;
            const int dof = (side ? ct : rt) * DT + rr;
            const int pt = p0 + pp;
            double f[DF] = {0, 0, 0, 0, 0, 0};
            if (dof < nd && pt < P) {
                const int a = pt / (Qv * Qw), b = (pt / Qw) % Qv, c = pt % Qw;
                const int p3[3] = {a, b, c};
                dof_features<PROB>(N, dof, p3, bas, f);
                if (side) {
                    const double W = gwu[a] * gwv[b] * gww[c];
                    double al[12];
#pragma unroll
                    for (int s = 0; s < F; ++s) al[s] = A[(int64_t)s * P + pt];
                    double Kc[3][3] = {{al[0], al[3], al[4]}, {al[3], al[1], al[5]}, {al[4], al[5], al[2]}};
                    double g3[DF];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        g3[r] = sK * W * (Kc[r][0] * f[0] + Kc[r][1] * f[1] + Kc[r][2] * f[2]);
                    if (PROB == 0) {
                        g3[3] = sM * W * al[6] * f[3];
                        g3[4] = g3[5] = 0.0;
                    } else {
                        double Mc[3][3] = {{al[6], al[9], al[10]}, {al[9], al[7], al[11]}, {al[10], al[11], al[8]}};
#pragma unroll
                        for (int r = 0; r < 3; ++r)
                            g3[3 + r] = sM * W * (Mc[r][0] * f[3] + Mc[r][1] * f[4] + Mc[r][2] * f[5]);
                    }
#pragma unroll
                    for (int q = 0; q < DF; ++q) f[q] = g3[q];
                }
            }
            double(*dst)[DF][DT] = side ? Gt : Ft;
#pragma unroll
            for (int q = 0; q < DF; ++q) dst[pp][q][rr] = f[q];
        }
        __syncthreads();
#pragma unroll 2
        for (int pp = 0; pp < DPC; ++pp)
#pragma unroll
            for (int q = 0; q < DF; ++q) {
                const double4 av = *reinterpret_cast<const double4 *>(&Ft[pp][q][ty * 4]);
                const double4 bv = *reinterpret_cast<const double4 *>(&Gt[pp][q][tx * 4]);
                const double ar[4] = {av.x, av.y, av.z, av.w}, br[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(ar[i], br[j], acc[i][j]);
            }
        __syncthreads();
    }
    double *o = out + d.out_off;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = rt * DT + ty * 4 + i, c = ct * DT + tx * 4 + j;
            if (r < nd && c < nd) {
                o[(int64_t)r * nd + c] = acc[i][j];
                if (ct != rt) o[(int64_t)c * nd + r] = acc[i][j];
            }
        }
}

void launch_direct(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                   const double *alpha, double *out, double sK, double sM, hipStream_t st)
{
    if (count <= 0) return;
    const int nd = num_dofs(problem, N);
    const int ntile = (nd + DT - 1) / DT;
    const int64_t grid = count * (int64_t)(ntile * (ntile + 1) / 2);
    if (problem == 0)
        hipLaunchKernelGGL(k_direct<0>, dim3((unsigned)grid), dim3(256), 0, st, desc, e0, ntile, tab, alpha, out, sK, sM);
    else
        hipLaunchKernelGGL(k_direct<1>, dim3((unsigned)grid), dim3(256), 0, st, desc, e0, ntile, tab, alpha, out, sK, sM);
}

}  // namespace p2s
