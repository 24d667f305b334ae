// p2s_kernels.hip -- HIP kernels of the product-to-sum element-matrix fill
// for CDNA4 (gfx950, wave64).
//
// Stages (paper Section II):
//   k_coupling   geometry + coupling factor alpha_s at every Gauss point
//                (the integrand factor of eq. (2) that is not separable);
//   k_moments    the 3-D integrals of eq. (4), I_s[k,l,q], by sum
//                factorization over the three axes;
// (the contraction of eq. (4) is in p2s_contract.hip)
#include <hip/hip_runtime.h>

#include <utility>

#include "p2s_internal.h"
#include "p2s_kernels.h"

namespace p2s {

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
                                                  uint32_t *__restrict__ status,
                                                  const int32_t *__restrict__ only)
{
    constexpr int F = num_fields(PROB);
    const int64_t e = e0 + blockIdx.x;
    if (only && !only[e]) return;
    const ElemDesc d = desc[e];
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw;
    const int P = Qu * Qv * Qw;
    double *dst = alpha + d.alpha_off;
    __shared__ double X[81];
    __shared__ double mp[16];
    if (kind == ALPHA_SAMPLED) {
        const double *src = mat + e * (int64_t)(F * P);
        for (int i = threadIdx.x; i < F * P; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x == 0 && !only) status[e] = 0u;
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
    if (threadIdx.x == 0) {
        if (only)
            status[e] |= bad ? P2S_STATUS_DETJ_BIT : 0u;
        else
            status[e] = bad ? P2S_STATUS_DETJ_BIT : 0u;
    }
}

// ---------------------------------------------------------------------------
// Moments, eq. (4): I[k][l][q] = sum_{a,b,c} Wu[k][a] Wv[l][b] Ww[q][c] alpha[a][b][c]
// with W[k][a] = w_a L_k(x_a), as three passes (contract w, then v, then u).
// One workgroup per (element, field); the sizes are runtime, the degree
// count K = 2N-1 selects a register-blocked instantiation.
//
// TAIL (learned order): each pass whose axis is sampled below the full
// rule MLP_KMAX also takes, on every line it contracts, the discrete
// Legendre coefficients of the four highest degrees its rule resolves (w on
// the samples, v on the w-moments, u on the (v,w)-moments), keeps their
// largest magnitudes and the largest magnitude of the tensor it reads, and
// writes them as the (element, field) tail record (zeros for full axes).

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int K, bool TAIL>
__device__ void moments_body(const ElemDesc &d, int64_t e, int f, int F, const double *__restrict__ alpha,
                             const double *__restrict__ tab, double *__restrict__ mom, double *sm,
                             int p2off, double *__restrict__ tailst)
{
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw;
    const int P = Qu * Qv * Qw;
    const double *A = alpha + d.alpha_off + (int64_t)f * P;
    const double *Wu = tab + TAB_LEGW + Qu * LEGW_STRIDE_Q;
    const double *Wv = tab + TAB_LEGW + Qv * LEGW_STRIDE_Q;
    const double *Ww = tab + TAB_LEGW + Qw * LEGW_STRIDE_Q;
    const double *Tu = tab + TAB_TAILW + Qu * TAILW_STRIDE_Q;
    const double *Tv = tab + TAB_TAILW + Qv * TAILW_STRIDE_Q;
    const double *Tw = tab + TAB_TAILW + Qw * TAILW_STRIDE_Q;
    constexpr int KS = K + 1;  // LDS row stride
    double *P1 = sm;          // [Qu*Qv][KS]   (q)
    double *P2 = sm + p2off;  // [Qu][K][KS]   (l, q)
    const int tid = threadIdx.x, nt = blockDim.x;
    double rec[TAIL_REC];
#pragma unroll
    for (int i = 0; i < TAIL_REC; ++i) rec[i] = 0.0;
    // workgroup-uniform: which axes take the tail statistic
    const bool tu = TAIL && Qu < MLP_KMAX, tv = TAIL && Qv < MLP_KMAX, tw = TAIL && Qw < MLP_KMAX;
    // pass 1: contract w
    for (int ab = tid; ab < Qu * Qv; ab += nt) {
        double acc[K], tl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = 0.0;
        const double *Ar = A + (int64_t)ab * Qw;
        for (int c = 0; c < Qw; ++c) {
            const double x = Ar[c];
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = fma(Ww[q * MAXQ + c], x, acc[q]);
            if (tw) {
#pragma unroll
                for (int j = 0; j < 4; ++j) tl[j] = fma(Tw[j * MAXQ + c], x, tl[j]);
                rec[14] = fmax(rec[14], fabs(x));
            }
        }
        if (tw)
#pragma unroll
            for (int j = 0; j < 4; ++j) rec[8 + j] = fmax(rec[8 + j], fabs(tl[j]));
#pragma unroll
        for (int q = 0; q < K; ++q) P1[ab * KS + q] = acc[q];
    }
    __syncthreads();
    // pass 2: contract v
    for (int aq = tid; aq < Qu * K; aq += nt) {
        const int a = aq / K, q = aq - (aq / K) * K;
        double acc[K], tl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < K; ++l) acc[l] = 0.0;
        for (int b = 0; b < Qv; ++b) {
            const double x = P1[(a * Qv + b) * KS + q];
#pragma unroll
            for (int l = 0; l < K; ++l) acc[l] = fma(Wv[l * MAXQ + b], x, acc[l]);
            if (tv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) tl[j] = fma(Tv[j * MAXQ + b], x, tl[j]);
                rec[13] = fmax(rec[13], fabs(x));
            }
        }
        if (tv)
#pragma unroll
            for (int j = 0; j < 4; ++j) rec[4 + j] = fmax(rec[4 + j], fabs(tl[j]));
#pragma unroll
        for (int l = 0; l < K; ++l) P2[(a * K + l) * KS + q] = acc[l];
    }
    __syncthreads();
    // pass 3: contract u
    double *I = mom + d.mom_off + (int64_t)f * K * K * K;
    for (int lq = tid; lq < K * K; lq += nt) {
        const int l = lq / K, q = lq - (lq / K) * K;
        double acc[K], tl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = 0.0;
        for (int a = 0; a < Qu; ++a) {
            const double x = P2[(a * K + l) * KS + q];
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = fma(Wu[k * MAXQ + a], x, acc[k]);
            if (tu) {
#pragma unroll
                for (int j = 0; j < 4; ++j) tl[j] = fma(Tu[j * MAXQ + a], x, tl[j]);
                rec[12] = fmax(rec[12], fabs(x));
            }
        }
        if (tu)
#pragma unroll
            for (int j = 0; j < 4; ++j) rec[j] = fmax(rec[j], fabs(tl[j]));
#pragma unroll
        for (int k = 0; k < K; ++k) I[k * K * K + lq] = acc[k];
    }
    if (TAIL) {
        // block-wide maximum of the record: waves, then LDS (P1 is free now)
        __syncthreads();
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int i = 0; i < 15; ++i) {
            const double v = wave_max(rec[i]);
            if (lane == 0) sm[wave * TAIL_REC + i] = v;
        }
        __syncthreads();
        if (tid < 15) {
            double v = 0.0;
            for (int w = 0; w < (nt + 63) / 64; ++w) v = fmax(v, sm[w * TAIL_REC + tid]);
            tailst[(e * F + f) * TAIL_REC + tid] = v;
        }
    }
}

template <bool TAIL>
__global__ __launch_bounds__(256) void k_moments(const ElemDesc *__restrict__ desc, int64_t e0, int F,
                                                 const double *__restrict__ alpha,
                                                 const double *__restrict__ tab,
                                                 double *__restrict__ mom, int p2off,
                                                 const int32_t *__restrict__ only, double *__restrict__ tailst)
{
    extern __shared__ double sm[];
    const int64_t e = e0 + blockIdx.x;
    if (only && !only[e]) return;
    const ElemDesc d = desc[e];
    const int f = blockIdx.y;
    switch (d.N) {
    case 2: moments_body<3, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 3: moments_body<5, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 4: moments_body<7, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 5: moments_body<9, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 6: moments_body<11, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 7: moments_body<13, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
    case 8: moments_body<15, TAIL>(d, e, f, F, alpha, tab, mom, sm, p2off, tailst); break;
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
// Host-side launchers.

void launch_coupling(int problem, const ElemDesc *desc, int64_t e0, int64_t count,
                     const double *nodes, const double *mat, int kind, int mat_stride,
                     const double *tab, double *alpha, uint32_t *status, const int32_t *only, hipStream_t st)
{
    if (count <= 0) return;
    if (problem == 0)
        hipLaunchKernelGGL(k_coupling<0>, dim3((unsigned)count), dim3(256), 0, st, desc, e0, nodes,
                           mat, kind, mat_stride, tab, alpha, status, only);
    else
        hipLaunchKernelGGL(k_coupling<1>, dim3((unsigned)count), dim3(256), 0, st, desc, e0, nodes,
                           mat, kind, mat_stride, tab, alpha, status, only);
}

void launch_moments(int problem, int maxN, int maxQu, int maxQuv, const ElemDesc *desc, int64_t e0,
                    int64_t count, const double *alpha, const double *tab, double *mom, const int32_t *only,
                    double *tailst, hipStream_t st)
{
    if (count <= 0) return;
    const int F = num_fields(problem);
    if (tailst)
        hipLaunchKernelGGL(k_moments<true>, dim3((unsigned)count, F), dim3(256),
                           moments_smem_bytes(maxN, maxQu, maxQuv), st, desc, e0, F, alpha, tab, mom,
                           moments_p2_offset(maxN, maxQuv), only, tailst);
    else
        hipLaunchKernelGGL(k_moments<false>, dim3((unsigned)count, F), dim3(256),
                           moments_smem_bytes(maxN, maxQu, maxQuv), st, desc, e0, F, alpha, tab, mom,
                           moments_p2_offset(maxN, maxQuv), only, tailst);
}

int prepare_kernels()
{
    // k_moments may need more than the default 64 KiB of LDS
    hipError_t r = hipFuncSetAttribute((const void *)k_moments<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipError_t r2 = hipFuncSetAttribute((const void *)k_moments<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return r == hipSuccess && r2 == hipSuccess ? 0 : -1;
}

}  // namespace p2s
