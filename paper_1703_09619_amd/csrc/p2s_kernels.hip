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

// eps(x) as a symmetric tensor (e00 e11 e22 e01 e02 e12) for material KIND.
template <int KIND>
__device__ __forceinline__ void permittivity(const double *p, const double x[3], double e[6])
{
    if constexpr (KIND == MAT_ROTDIAG) {
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
    } else {
        double v;
        if constexpr (KIND == MAT_PLANEWAVE)
            v = 1.0 + 0.8 * sin(p[0] * x[0] + p[1] * x[1] + p[2] * x[2] + p[3]);
        else
            v = 1.0 + 0.5 * sin(p[0] * x[0]) * cos(p[0] * x[1]) * exp(-x[2]);
        e[0] = e[1] = e[2] = v;
        e[3] = e[4] = e[5] = 0.0;
    }
}

// Coupling fields at one point from the map value x and Jacobian
// J[r][c] = dx_r/du_c.  Returns det J; writes F fields (packed order of
// P2S_ALPHA_SAMPLED).
template <int PROB, int KIND>
__device__ __forceinline__ double coupling_fields(const double x[3], const double J[3][3], const double *mp,
                                                  double *f)
{
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
    permittivity<KIND>(mp, x, e);
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
// alpha[alpha_off + f*P + (a*Qv+b)*Qw + c], unweighted.  The triquadratic
// map is sum-factorized: a thread takes a line of points along u (fixed
// v_b, w_c), contracts the node array over the (v,w) Lagrange factors once,
//   Y[i] = sum_jk lv_j lw_k X_ijk,  Yv[i] = sum_jk dv_j lw_k X_ijk,
//   Yw[i] = sum_jk lv_j dw_k X_ijk,
// and then evaluates x and J at each point of the line from 3 terms each.
template <int PROB, int KIND>
__global__ __launch_bounds__(256) void k_coupling(const ElemDesc *__restrict__ desc, int64_t e0,
                                                  const double *__restrict__ nodes,
                                                  const double *__restrict__ mat,
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
    const int P = Qu * Qv * Qw, L = Qv * Qw;
    double *dst = alpha + d.alpha_off;
    __shared__ double X[81];
    __shared__ double mp[16];
    if constexpr (KIND == ALPHA_SAMPLED) {
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
    for (int ln = threadIdx.x; ln < L; ln += blockDim.x) {
        const int b = ln / Qw, c = ln - (ln / Qw) * Qw;
        double lv[3], dv[3], lw[3], dw[3];
        lagrange3(gv[b], lv, dv);
        lagrange3(gw[c], lw, dw);
        double Y[3][3], Yv[3][3], Yw[3][3];  // [i][r]
        // the node array is read from LDS here, line by line (held in
        // registers across the line loop it would take 162 VGPRs): an
        // opaque zero offset keeps the reads inside the loop
        int xo = 0;
        asm volatile("" : "+v"(xo));
        const double *Xv = X + xo;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double y = 0.0, yv = 0.0, yw = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    // t_j = X_ijk for j = 0..2
                    const double t0 = Xv[3 * (i + 9 * k) + r], t1 = Xv[3 * (i + 3 + 9 * k) + r],
                                 t2 = Xv[3 * (i + 6 + 9 * k) + r];
                    const double sl = lv[0] * t0 + lv[1] * t1 + lv[2] * t2;
                    const double sd = dv[0] * t0 + dv[1] * t1 + dv[2] * t2;
                    y = fma(lw[k], sl, y);
                    yv = fma(lw[k], sd, yv);
                    yw = fma(dw[k], sl, yw);
                }
                Y[i][r] = y;
                Yv[i][r] = yv;
                Yw[i][r] = yw;
            }
        for (int a = 0; a < Qu; ++a) {
            double lu[3], du[3];
            lagrange3(gu[a], lu, du);
            double x[3], J[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                x[r] = lu[0] * Y[0][r] + lu[1] * Y[1][r] + lu[2] * Y[2][r];
                J[r][0] = du[0] * Y[0][r] + du[1] * Y[1][r] + du[2] * Y[2][r];
                J[r][1] = lu[0] * Yv[0][r] + lu[1] * Yv[1][r] + lu[2] * Yv[2][r];
                J[r][2] = lu[0] * Yw[0][r] + lu[1] * Yw[1][r] + lu[2] * Yw[2][r];
            }
            double f[F];
            const double det = coupling_fields<PROB, KIND>(x, J, mp, f);
            bad |= !(det > 0.0);
            const int64_t pt = (int64_t)a * L + ln;
#pragma unroll
            for (int s = 0; s < F; ++s) dst[(int64_t)s * P + pt] = f[s];
        }
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
// with W[k][a] = w_a L_k(x_a), as three dense GEMM passes on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64), contracting u, then v, then w:
//   pass 1  P1[k][(b,c)] = sum_a Wu[k][a] alpha[a][(b,c)]   (operand B read
//           straight from HBM: 16 consecutive samples per row, coalesced)
//   pass 2  P2[k][l][c]  = sum_b Wv[l][b] P1[k][b][c]       (N = (k,c))
//   pass 3  I[k][l][q]   = sum_c Ww[q][c] P2[k][l][c]       (N = (k,l))
// Each pass is M = 16 rows (K = 2N-1 <= 15 moment degrees) by N columns in
// tiles of 16, with the summed index in steps of 4.  One workgroup (4 waves)
// per (element, field); the waves take the N tiles in turn.
//
// TAIL (learned order, K + 4 <= 16): the tail statistic of every axis
// sampled below the full rule MLP_KMAX.  Rows K..K+3 of that axis's pass
// hold the discrete Legendre coefficients of the four highest degrees its
// rule resolves (tail weights), and they are carried through the later
// passes like moment rows, so that each axis's coefficients end up
// projected onto the moment degrees of the other two axes:
//   u tail rows: P1 rows K..K+3, through passes 2 and 3 -> T_u[j][l][q]
//   v tail rows: P2 columns K..K+3 of l, through pass 3 -> T_v[k][j][q]
//   w tail rows: pass 3 rows K..K+3                      -> T_w[k][l][j]
// The workgroup keeps the largest magnitude of each T_x[j] and of the
// moment tensor and writes them as the (element, field) tail record (zeros
// for axes at the full rule).  The values do not depend on the order in
// which the axes are contracted.
//
// FP64 MFMA 16x16x4 lane layout (wave64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register i of lane l is D[4i + l/16][l%16].

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Operand-A value of row m for a pass over an axis with Q points: moment
// weights for m < K, tail weights for K <= m < K+4 when `tail`, else 0;
// column a (zero beyond Q in both tables).
__device__ __forceinline__ double pass_weight(const double *__restrict__ tab, int Q, int K, bool tail, int m, int a)
{
    if (a >= MAXQ) return 0.0;
    if (m < K) return tab[TAB_LEGW + Q * LEGW_STRIDE_Q + m * MAXQ + a];
    if (tail && m < K + 4) return tab[TAB_TAILW + Q * TAILW_STRIDE_Q + (m - K) * MAXQ + a];
    return 0.0;
}

template <bool TAIL>
__device__ void moments_body(const ElemDesc &d, int64_t e, int f, int F, const double *__restrict__ alpha,
                             const double *__restrict__ tab, double *__restrict__ mom, double *sm,
                             int p2off, double *__restrict__ tailst)
{
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw, K = 2 * d.N - 1;
    const int L = Qv * Qw, P = Qu * L;
    const int QWS = Qw | 1;  // odd row stride of P2
    const double *A = alpha + d.alpha_off + (int64_t)f * P;
    double *P1 = sm;          // [K1][Qv*Qw]   (k; b, c)
    double *P2 = sm + p2off;  // [K1][K2][QWS] (k, l; c)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    double rec[TAIL_REC];
#pragma unroll
    for (int i = 0; i < TAIL_REC; ++i) rec[i] = 0.0;
    // workgroup-uniform: which axes take the tail statistic; K1 rows of P1
    // (u moments, then u tail rows), K2 rows l' of P2 (v moments, then v
    // tail rows)
    const bool tu = TAIL && Qu < MLP_KMAX, tv = TAIL && Qv < MLP_KMAX, tw = TAIL && Qw < MLP_KMAX;
    const int K1 = K + (tu ? 4 : 0), K2 = K + (tv ? 4 : 0);
    double wa[MAXQ / 4];  // operand A of the current pass, one value per step of 4

    // pass 1: contract u; columns (b,c).  A wave takes TG consecutive column
    // tiles at a time and issues all their sample loads before the matrix
    // operations, so that many HBM loads are in flight per lane.
    constexpr int TG = 4;
    const int su = (Qu + 3) >> 2;
#pragma unroll
    for (int ks = 0; ks < MAXQ / 4; ++ks) wa[ks] = ks < su ? pass_weight(tab, Qu, K, tu, r16, 4 * ks + k4) : 0.0;
    for (int nt0 = wave * TG; nt0 * 16 < L; nt0 += nwave * TG) {
        double xs[TG][MAXQ / 4];
#pragma unroll
        for (int t = 0; t < TG; ++t) {
            const int col = (nt0 + t) * 16 + r16;
#pragma unroll
            for (int ks = 0; ks < MAXQ / 4; ++ks) {
                const int a = 4 * ks + k4;
                xs[t][ks] = (ks < su && a < Qu && col < L) ? A[(int64_t)a * L + col] : 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < TG; ++t) {
            const int col = (nt0 + t) * 16 + r16;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < MAXQ / 4; ++ks)
                if (ks < su) acc = mfma64(wa[ks], xs[t][ks], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 4 * i + k4;
                if (col < L && m < K1) P1[m * L + col] = acc[i];
            }
        }
    }
    __syncthreads();
    // pass 2: contract v; columns n = (k, c), k < K1 (moment rows, then the
    // u tail rows when u is reduced)
    const int sv = (Qv + 3) >> 2, n2 = K1 * Qw;
#pragma unroll
    for (int ks = 0; ks < MAXQ / 4; ++ks) wa[ks] = ks < sv ? pass_weight(tab, Qv, K, tv, r16, 4 * ks + k4) : 0.0;
    for (int nt = wave; nt * 16 < n2; nt += nwave) {
        const int n = nt * 16 + r16;
        const int k = n / Qw, c = n - (n / Qw) * Qw;
        // all LDS reads of the tile first, then the chain of matrix operations
        double xv[MAXQ / 4];
#pragma unroll
        for (int ks = 0; ks < MAXQ / 4; ++ks) {
            const int b = 4 * ks + k4;
            xv[ks] = (ks < sv && b < Qv && n < n2) ? P1[k * L + b * Qw + c] : 0.0;
        }
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < MAXQ / 4; ++ks)
            if (ks < sv) acc = mfma64(wa[ks], xv[ks], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * i + k4;
            if (n < n2 && m < K2) P2[(k * K2 + m) * QWS + c] = acc[i];
        }
    }
    __syncthreads();
    // pass 3: contract w; columns n = (k, l); results staged in LDS so that
    // the global write below is contiguous: in the P1 region (free after
    // pass 2) when K^3 doubles fit below P2, else after P2 (the buffer is
    // sized for that case)
    double *I = mom + d.mom_off + (int64_t)f * K * K * K;
    double *Is = (K * K * K <= p2off) ? sm : P2 + K1 * K2 * QWS;
    const int sw = (Qw + 3) >> 2, n3 = K1 * K2;
#pragma unroll
    for (int ks = 0; ks < MAXQ / 4; ++ks) wa[ks] = ks < sw ? pass_weight(tab, Qw, K, tw, r16, 4 * ks + k4) : 0.0;
    for (int nt = wave; nt * 16 < n3; nt += nwave) {
        const int n = nt * 16 + r16;
        double xw[MAXQ / 4];
#pragma unroll
        for (int ks = 0; ks < MAXQ / 4; ++ks) {
            const int c = 4 * ks + k4;
            xw[ks] = (ks < sw && c < Qw && n < n3) ? P2[n * QWS + c] : 0.0;
        }
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < MAXQ / 4; ++ks)
            if (ks < sw) acc = mfma64(wa[ks], xw[ks], acc);
        // column n = (k', l'): k' >= K is a u tail row, l' >= K a v tail row
        const int kk = n / K2, ll = n - (n / K2) * K2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * i + k4;
            if (n < n3 && m < K + (tw ? 4 : 0)) {
                if (!TAIL) {
                    Is[n * K + m] = acc[i];
                } else if (kk < K && ll < K) {
                    if (m < K) {
                        Is[(kk * K + ll) * K + m] = acc[i];
                        rec[12] = fmax(rec[12], fabs(acc[i]));
                    } else {
                        rec[8 + m - K] = fmax(rec[8 + m - K], fabs(acc[i]));  // T_w
                    }
                } else if (m < K) {
                    if (kk >= K && ll < K) rec[kk - K] = fmax(rec[kk - K], fabs(acc[i]));         // T_u
                    else if (kk < K && ll >= K) rec[4 + ll - K] = fmax(rec[4 + ll - K], fabs(acc[i]));  // T_v
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < K * K * K; i += blockDim.x) I[i] = Is[i];
    if (TAIL) {
        // block-wide maximum of the record: waves, then LDS (after the copy)
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 15; ++i) {
            const double v = wave_max(rec[i]);
            if (lane == 0) sm[wave * TAIL_REC + i] = v;
        }
        __syncthreads();
        if (tid < TAIL_REC) {
            // scale of every reduced axis: the largest moment magnitude;
            // entry 15 is unused and written as zero
            const int src = tid >= 12 ? 12 : tid;
            const bool on = tid < 12 || (tid == 12 && tu) || (tid == 13 && tv) || (tid == 14 && tw);
            double v = 0.0;
            for (int w = 0; w < nwave; ++w) v = fmax(v, sm[w * TAIL_REC + src]);
            tailst[(e * F + f) * TAIL_REC + tid] = on ? v : 0.0;
        }
    }
}

// With tail records the LDS holds the carried tail rows (about 114 KB at 24
// points per axis, one workgroup per CU), so that form runs eight waves per
// workgroup instead of four.
constexpr int MOMENTS_TAIL_THREADS = 512;

template <bool TAIL>
__global__ __launch_bounds__(TAIL ? MOMENTS_TAIL_THREADS : 256) void k_moments(const ElemDesc *__restrict__ desc,
                                                                             int64_t e0, int F,
                                                 const double *__restrict__ alpha,
                                                 const double *__restrict__ tab,
                                                 double *__restrict__ mom, int p2off,
                                                 const int32_t *__restrict__ only, double *__restrict__ tailst,
                                                 const int32_t *__restrict__ elist)
{
    extern __shared__ double sm[];
    const int64_t e = elist ? (int64_t)elist[e0 + blockIdx.x] : e0 + blockIdx.x;
    if (only && !only[e]) return;
    const ElemDesc d = desc[e];
    if (TAIL && d.Qu >= MLP_KMAX && d.Qv >= MLP_KMAX && d.Qw >= MLP_KMAX) {
        // nothing sampled below the full rule: plain moments, empty record
        moments_body<false>(d, e, blockIdx.y, F, alpha, tab, mom, sm, p2off, tailst);
        if (threadIdx.x < TAIL_REC) tailst[(e * F + blockIdx.y) * TAIL_REC + threadIdx.x] = 0.0;
        return;
    }
    moments_body<TAIL>(d, e, blockIdx.y, F, alpha, tab, mom, sm, p2off, tailst);
}

// Register-blocked vector-unit form of the same three passes (contract w,
// then v, then u; one lane per line, K accumulators per lane), used when
// every rule has at most 16 points: there the matrix-core tiles are few and
// mostly padding, and this form is faster.  No tail statistic.
template <int K>
__device__ void moments_valu(const ElemDesc &d, int f, const double *__restrict__ alpha,
                             const double *__restrict__ tab, double *__restrict__ mom, double *sm, int p2off)
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
    double *A0 = sm + p2off;  // [Qu*Qv][Qw|1] samples, dead before P2 is written
    const int tid = threadIdx.x, nt = blockDim.x;
    const int QW1 = Qw | 1;   // odd row stride: the lanes of pass 1 read distinct banks
    // stage the samples: coalesced reads, eight in flight per lane
    {
        constexpr int U = 8;
        for (int x0 = tid; x0 < P; x0 += U * nt) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = x0 + u * nt;
                v[u] = x < P ? A[x] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = x0 + u * nt;
                if (x < P) {
                    const int ab = x / Qw;
                    A0[ab * QW1 + (x - ab * Qw)] = v[u];
                }
            }
        }
    }
    __syncthreads();
    // pass 1: contract w
    for (int ab = tid; ab < Qu * Qv; ab += nt) {
        double acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = 0.0;
        const double *Ar = A0 + ab * QW1;
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

__global__ __launch_bounds__(256) void k_moments_valu(const ElemDesc *__restrict__ desc, int64_t e0,
                                                      const double *__restrict__ alpha,
                                                      const double *__restrict__ tab, double *__restrict__ mom,
                                                      int p2off, const int32_t *__restrict__ only,
                                                      const int32_t *__restrict__ elist)
{
    extern __shared__ double sm[];
    const int64_t e = elist ? (int64_t)elist[e0 + blockIdx.x] : e0 + blockIdx.x;
    if (only && !only[e]) return;
    const ElemDesc d = desc[e];
    const int f = blockIdx.y;
    switch (d.N) {
    case 2: moments_valu<3>(d, f, alpha, tab, mom, sm, p2off); break;
    case 3: moments_valu<5>(d, f, alpha, tab, mom, sm, p2off); break;
    case 4: moments_valu<7>(d, f, alpha, tab, mom, sm, p2off); break;
    case 5: moments_valu<9>(d, f, alpha, tab, mom, sm, p2off); break;
    case 6: moments_valu<11>(d, f, alpha, tab, mom, sm, p2off); break;
    case 7: moments_valu<13>(d, f, alpha, tab, mom, sm, p2off); break;
    case 8: moments_valu<15>(d, f, alpha, tab, mom, sm, p2off); break;
    default: break;
    }
}

// LDS layout of k_moments for the largest order and rule of a plan:
// P1 [K][Qv*Qw] followed by P2 [K][K][Qw | 1]; the staged K^3 tile of
// pass 3 reuses P1 when it fits there, else follows P2; at least one
// TAIL_REC per wave of the tail form (the tail-record reduction reuses the
// start).
// With tail records P1 and P2 carry four more rows per reduced axis: P1
// [K+4][Qv*Qw], P2 [K+4][K+4][Qw | 1].
int moments_p2_offset(int maxN, int maxQvw, bool tail) { return maxQvw * (2 * maxN - 1 + (tail ? 4 : 0)); }
size_t moments_smem_bytes(int maxN, int maxQw, int maxQvw, bool tail)
{
    const int K = 2 * maxN - 1, K4 = K + (tail ? 4 : 0);
    const size_t p2 = (size_t)moments_p2_offset(maxN, maxQvw, tail);
    size_t n = p2 + (size_t)(K4 * K4 * (maxQw | 1));
    if ((size_t)(K * K * K) > p2) n += (size_t)(K * K * K);
    // the tail-record reduction reuses the start: one record per wave
    const size_t red = (size_t)(MOMENTS_TAIL_THREADS / 64) * TAIL_REC;
    return sizeof(double) * (n > red ? n : red);
}
// LDS layout of k_moments_valu: P1 [Qu*Qv][K+1] followed by P2 [Qu][K][K+1],
// which first holds the staged samples [Qu*Qv][Qw|1].
static int valu_p2_offset(int maxN, int maxQuv) { return maxQuv * (2 * maxN); }
static size_t valu_smem_bytes(int maxN, int maxQu, int maxQuv, int maxQw)
{
    const int K = 2 * maxN - 1;
    const size_t p2 = (size_t)maxQu * K * (K + 1), a0 = (size_t)maxQuv * (maxQw | 1);
    return sizeof(double) * ((size_t)valu_p2_offset(maxN, maxQuv) + (p2 > a0 ? p2 : a0));
}
size_t moments_lds_bytes(const MomentShape &m)
{
    return m.maxQ <= SPLIT_MAXQ ? valu_smem_bytes(m.maxN, m.maxQu, m.maxQuv, m.maxQw)
                                : moments_smem_bytes(m.maxN, m.maxQw, m.maxQvw, false);
}

// ---------------------------------------------------------------------------
// Host-side launchers.

template <int PROB, int KIND>
static void launch_coupling_k(const ElemDesc *desc, int64_t e0, int64_t count, const double *nodes,
                              const double *mat, int mat_stride, const double *tab, double *alpha,
                              uint32_t *status, const int32_t *only, hipStream_t st)
{
    hipLaunchKernelGGL((k_coupling<PROB, KIND>), dim3((unsigned)count), dim3(256), 0, st, desc, e0, nodes, mat,
                       mat_stride, tab, alpha, status, only);
}

template <int PROB>
static void launch_coupling_p(int kind, const ElemDesc *desc, int64_t e0, int64_t count, const double *nodes,
                              const double *mat, int mat_stride, const double *tab, double *alpha,
                              uint32_t *status, const int32_t *only, hipStream_t st)
{
    switch (kind) {
    case MAT_SINCOSEXP:
        launch_coupling_k<PROB, MAT_SINCOSEXP>(desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only, st);
        break;
    case MAT_ROTDIAG:
        if constexpr (PROB == 1)
            launch_coupling_k<PROB, MAT_ROTDIAG>(desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only,
                                                 st);
        break;
    case MAT_PLANEWAVE:
        launch_coupling_k<PROB, MAT_PLANEWAVE>(desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only, st);
        break;
    default:
        launch_coupling_k<PROB, ALPHA_SAMPLED>(desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only, st);
        break;
    }
}

void launch_coupling(int problem, const ElemDesc *desc, int64_t e0, int64_t count,
                     const double *nodes, const double *mat, int kind, int mat_stride,
                     const double *tab, double *alpha, uint32_t *status, const int32_t *only, hipStream_t st)
{
    if (count <= 0) return;
    if (problem == 0)
        launch_coupling_p<0>(kind, desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only, st);
    else
        launch_coupling_p<1>(kind, desc, e0, count, nodes, mat, mat_stride, tab, alpha, status, only, st);
}

void launch_moments(int problem, const MomentShape &m, const ElemDesc *desc, int64_t e0, int64_t count,
                    const double *alpha, const double *tab, double *mom, const int32_t *only, double *tailst,
                    hipStream_t st, const int32_t *elist)
{
    if (count <= 0) return;
    const int F = num_fields(problem);
    if (tailst)
        hipLaunchKernelGGL(k_moments<true>, dim3((unsigned)count, F), dim3(MOMENTS_TAIL_THREADS),
                           moments_smem_bytes(m.maxN, m.maxQw, m.maxQvw, true), st, desc, e0, F, alpha, tab, mom,
                           moments_p2_offset(m.maxN, m.maxQvw, true), only, tailst, elist);
    else if (m.maxQ <= SPLIT_MAXQ)
        hipLaunchKernelGGL(k_moments_valu, dim3((unsigned)count, F), dim3(256),
                           valu_smem_bytes(m.maxN, m.maxQu, m.maxQuv, m.maxQw), st, desc, e0, alpha, tab, mom,
                           valu_p2_offset(m.maxN, m.maxQuv), only, elist);
    else
        hipLaunchKernelGGL(k_moments<false>, dim3((unsigned)count, F), dim3(256),
                           moments_smem_bytes(m.maxN, m.maxQw, m.maxQvw, false), st, desc, e0, F, alpha, tab, mom,
                           moments_p2_offset(m.maxN, m.maxQvw, false), only, tailst, elist);
}

int prepare_kernels()
{
    // k_moments may need more than the default 64 KiB of LDS
    hipError_t r = hipFuncSetAttribute((const void *)k_moments<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipError_t r2 = hipFuncSetAttribute((const void *)k_moments<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipError_t r3 = hipFuncSetAttribute((const void *)k_moments_valu,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return r == hipSuccess && r2 == hipSuccess && r3 == hipSuccess ? 0 : -1;
}

}  // namespace p2s
