// p2s_cheb2d.hip -- the paper's own instance of the product-to-sum method
// (Section III): 2-D curl-curl + mass element matrices of curved
// quadrilaterals with the Chebyshev vector basis of eq. (6),
//   u-functions U_m(u) T_n(v) (m < M, n <= N), v-functions T_m(u) U_n(v)
//   (m <= M, n < N), M = N,
// the entries of eqs. (8)-(15), and the two-term product formulas of eq. (16)
// with the nonsingular Chebyshev polynomials of eq. (17):
//   U_a U_b = T^ns_|a-b| - T^ns_{a+b+2},  T_a T_b = (T_|a-b| + T_{a+b}) / 2,
//   U_a T_b = (U_{a+b} + U_{a-b}) / 2,  U_-1 = 0, U_-k = -U_{k-2}.
// Every entry is then a four-term sum of "starting point" integrals (eqs.
// (18)-(19)) per coupling factor, so the contraction is a gather-add:
//   k_cheb_coupling  geometry (quartic 25-node map), J and the four coupling
//                    factors 1/(mu J), eps G_uu, eps G_uv, eps G_vv at the
//                    Q x Q Gauss points
//   k_cheb_moments   I_f[k][l] = sum_ab w_a w_b F_k(u_a) G_l(v_b) alpha_f(a,b),
//                    two sum-factorized passes; (F, G) = (T^ns, T^ns) for the
//                    stiffness factor, (T^ns, T), (U, U), (T, T^ns) for the
//                    mass factors (k, l <= 2M)
//   k_cheb_gather    each entry from at most eight moments
// and, as the baseline the paper compares against (Table I), direct 2-D
// quadrature of every entry (k_cheb_direct).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "p2s.h"
#include "p2s_internal.h"
#include "p2s_kernels.h"
#include "p2s_tables.h"

namespace p2s {

constexpr int C2_MAXM = 18;               // largest order M = N
constexpr int C2_KM = 2 * C2_MAXM + 1;    // moment indices 0..2M
constexpr int C2_NF = 4;                  // coupling factors
enum C2Fam : int { C2_T = 0, C2_U = 1, C2_TNS = 2 };

// Quartic Lagrange polynomials on the nodes -1, -1/2, 0, 1/2, 1 and their
// derivatives at t.
__device__ __forceinline__ void lagrange5(double t, double l[5], double d[5])
{
    const double z[5] = {-1.0, -0.5, 0.0, 0.5, 1.0};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double num = 1.0, den = 1.0, der = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j == i) continue;
            den *= z[i] - z[j];
            // product rule: d/dt prod_j (t - z_j)
            double p = 1.0;
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (k != i && k != j) p *= t - z[k];
            der += p;
            num *= t - z[j];
        }
        l[i] = num / den;
        d[i] = der / den;
    }
}

// One workgroup per element; alpha[e][f][a*Q + b] (a along u), unweighted.
__global__ __launch_bounds__(256) void k_cheb_coupling(int Q, const double *__restrict__ nodes,
                                                       const double *__restrict__ mat,
                                                       const double *__restrict__ gx, double *__restrict__ alpha,
                                                       uint32_t *__restrict__ status)
{
    const int64_t e = blockIdx.x;
    __shared__ double X[50];
    __shared__ double p[4];
    if (threadIdx.x < 50) X[threadIdx.x] = nodes[e * 50 + threadIdx.x];
    if (threadIdx.x < 4) p[threadIdx.x] = mat[e * 4 + threadIdx.x];
    __syncthreads();
    const int P = Q * Q;
    double *dst = alpha + e * (int64_t)C2_NF * P;
    int bad = 0;
    for (int pt = threadIdx.x; pt < P; pt += blockDim.x) {
        const int a = pt / Q, b = pt - (pt / Q) * Q;
        double lu[5], du[5], lv[5], dv[5];
        lagrange5(gx[a], lu, du);
        lagrange5(gx[b], lv, dv);
        double x = 0, y = 0, xu = 0, xv = 0, yu = 0, yv = 0;
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const double nx = X[2 * (i + 5 * j)], ny = X[2 * (i + 5 * j) + 1];
                const double w0 = lu[i] * lv[j], wu = du[i] * lv[j], wv = lu[i] * dv[j];
                x = fma(w0, nx, x);
                y = fma(w0, ny, y);
                xu = fma(wu, nx, xu);
                yu = fma(wu, ny, yu);
                xv = fma(wv, nx, xv);
                yv = fma(wv, ny, yv);
            }
        const double J = xu * yv - xv * yu;
        bad |= !(J > 0.0);
        const double rJ = 1.0 / J;
        const double eps = p[0] * exp(p[1] * x + p[2] * y + p[3]);
        dst[pt] = rJ;                                            // 1/(mu J), mu = 1
        dst[P + pt] = eps * (xv * xv + yv * yv) * rJ;            // eps G_uu
        dst[2 * P + pt] = -eps * (xu * xv + yu * yv) * rJ;       // eps G_uv
        dst[3 * P + pt] = eps * (xu * xu + yu * yu) * rJ;        // eps G_vv
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) status[e] = bad ? P2S_STATUS_DETJ_BIT : 0u;
}

// Family values at x for indices 0..KM-1 into v[fam][k] (stride C2_KM):
// three-term recurrences for T and U, and T^ns_0 = T^ns_1 = 0,
// T^ns_{k+2} = T^ns_k - U_k (eq. (16) with a factor U_0 = 1).
__device__ __forceinline__ void cheb_families(double x, int KM, double *v, int stride)
{
    double t0 = 1.0, t1 = x, u0 = 1.0, u1 = 2.0 * x;
    double s0 = 0.0, s1 = 0.0;  // T^ns_k, T^ns_{k+1}
    for (int k = 0; k < KM; ++k) {
        v[C2_T * stride + k] = t0;
        v[C2_U * stride + k] = u0;
        v[C2_TNS * stride + k] = s0;
        const double t2 = 2.0 * x * t1 - t0, u2 = 2.0 * x * u1 - u0, s2 = s0 - u0;
        t0 = t1;
        t1 = t2;
        s0 = s1;
        s1 = s2;
        u0 = u1;
        u1 = u2;
    }
}

// Moment families of each coupling factor along u and v.
__constant__ int c_c2fam[C2_NF][2] = {{C2_TNS, C2_TNS}, {C2_TNS, C2_T}, {C2_U, C2_U}, {C2_T, C2_TNS}};

// One workgroup per (element, factor): mom[e][f][k][l], k, l < KM = 2M+1.
__global__ __launch_bounds__(256) void k_cheb_moments(int Q, int KM, const double *__restrict__ gx,
                                                      const double *__restrict__ gw,
                                                      const double *__restrict__ alpha, double *__restrict__ mom)
{
    const int64_t e = blockIdx.x;
    const int f = blockIdx.y;
    __shared__ double A[MAXQ * (MAXQ + 1)];
    __shared__ double Fu[C2_KM * MAXQ], Gv[C2_KM * MAXQ];
    __shared__ double Pt[C2_KM * (MAXQ + 1)];
    const int P = Q * Q, QS = Q + 1;
    const double *src = alpha + (e * C2_NF + f) * (int64_t)P;
    for (int i = threadIdx.x; i < P; i += blockDim.x) A[(i / Q) * QS + i % Q] = src[i];
    const int fu = c_c2fam[f][0], fv = c_c2fam[f][1];
    if (threadIdx.x < Q) {
        const int a = threadIdx.x;
        double v[3 * C2_KM];
        cheb_families(gx[a], KM, v, C2_KM);
        for (int k = 0; k < KM; ++k) {
            Fu[k * MAXQ + a] = gw[a] * v[fu * C2_KM + k];
            Gv[k * MAXQ + a] = gw[a] * v[fv * C2_KM + k];
        }
    }
    __syncthreads();
    // pass 1: Pt[k][b] = sum_a Fu[k][a] A[a][b]
    for (int kb = threadIdx.x; kb < KM * Q; kb += blockDim.x) {
        const int k = kb / Q, b = kb - (kb / Q) * Q;
        double s = 0.0;
        for (int a = 0; a < Q; ++a) s = fma(Fu[k * MAXQ + a], A[a * QS + b], s);
        Pt[k * QS + b] = s;
    }
    __syncthreads();
    // pass 2: I[k][l] = sum_b Gv[l][b] Pt[k][b]
    double *I = mom + (e * C2_NF + f) * (int64_t)KM * KM;
    for (int kl = threadIdx.x; kl < KM * KM; kl += blockDim.x) {
        const int k = kl / KM, l = kl - (kl / KM) * KM;
        double s = 0.0;
        for (int b = 0; b < Q; ++b) s = fma(Gv[l * MAXQ + b], Pt[k * QS + b], s);
        I[kl] = s;
    }
}

// Two-term expansions of eq. (16): index and weight of each term (weight 0
// for an absent term).
struct Pair {
    int k0, k1;
    double w0, w1;
};
__device__ __forceinline__ Pair pair_uu(int a, int b)  // U_a U_b -> T^ns
{
    return Pair{a > b ? a - b : b - a, a + b + 2, 1.0, -1.0};
}
__device__ __forceinline__ Pair pair_tt(int a, int b)  // T_a T_b -> T
{
    return Pair{a > b ? a - b : b - a, a + b, 0.5, 0.5};
}
__device__ __forceinline__ Pair pair_ut(int a, int b)  // U_a T_b -> U
{
    const int d = a - b;
    Pair p{a + b, 0, 0.5, 0.0};
    if (d >= 0) {
        p.k1 = d;
        p.w1 = 0.5;
    } else if (d <= -2) {
        p.k1 = -d - 2;
        p.w1 = -0.5;
    }
    return p;
}
__device__ __forceinline__ double gather2(const double *I, int KM, Pair pu, Pair pv)
{
    return pu.w0 * (pv.w0 * I[pu.k0 * KM + pv.k0] + pv.w1 * I[pu.k0 * KM + pv.k1]) +
           pu.w1 * (pv.w0 * I[pu.k1 * KM + pv.k0] + pv.w1 * I[pu.k1 * KM + pv.k1]);
}

// dof index -> (v-block?, m, n)
__device__ __forceinline__ void c2_dof(int i, int M, bool &vb, int &m, int &n)
{
    const int NU = M * (M + 1);
    vb = i >= NU;
    if (!vb) {
        m = i / (M + 1);
        n = i - m * (M + 1);
    } else {
        const int r = i - NU;
        m = r / M;
        n = r - m * M;
    }
}

// One workgroup per (element, tile of ROWS rows): the element's moments in
// LDS, every entry of the tile as a gather-add, stores coalesced along rows.
constexpr int C2_ROWS = 8;
__global__ __launch_bounds__(256) void k_cheb_gather(int M, const double *__restrict__ mom,
                                                     double *__restrict__ out, uint32_t *__restrict__ status,
                                                     double sK, double sM)
{
    extern __shared__ double smem[];
    const int KM = 2 * M + 1, nd = 2 * M * (M + 1);
    const int tiles = (nd + C2_ROWS - 1) / C2_ROWS;
    const int64_t e = blockIdx.x / tiles;
    const int r0 = (int)(blockIdx.x % tiles) * C2_ROWS;
    const double *src = mom + e * (int64_t)C2_NF * KM * KM;
    for (int i = threadIdx.x; i < C2_NF * KM * KM; i += blockDim.x) smem[i] = src[i];
    __syncthreads();
    const double *IS = smem, *I1 = smem + KM * KM, *I2 = smem + 2 * KM * KM, *I3 = smem + 3 * KM * KM;
    double *o = out + e * (int64_t)nd * nd;
    bool bad = false;
    const int r1 = min(nd, r0 + C2_ROWS);
    for (int x = threadIdx.x; x < (r1 - r0) * nd; x += blockDim.x) {
        const int i = r0 + x / nd, j = x - (x / nd) * nd;
        bool vi, vj;
        int m1, n1, m2, n2;
        c2_dof(i, M, vi, m1, n1);
        c2_dof(j, M, vj, m2, n2);
        double s = 0.0, mm = 0.0;
        if (!vi && !vj) {           // eqs. (8), (12)
            if (n1 && n2) s = n1 * n2 * gather2(IS, KM, pair_uu(m1, m2), pair_uu(n1 - 1, n2 - 1));
            mm = gather2(I1, KM, pair_uu(m1, m2), pair_tt(n1, n2));
        } else if (!vi && vj) {     // eqs. (9), (13)
            if (n1 && m2) s = -n1 * m2 * gather2(IS, KM, pair_uu(m1, m2 - 1), pair_uu(n1 - 1, n2));
            mm = gather2(I2, KM, pair_ut(m1, m2), pair_ut(n2, n1));
        } else if (vi && !vj) {     // eqs. (10), (14)
            if (m1 && n2) s = -m1 * n2 * gather2(IS, KM, pair_uu(m2, m1 - 1), pair_uu(n2 - 1, n1));
            mm = gather2(I2, KM, pair_ut(m2, m1), pair_ut(n1, n2));
        } else {                    // eqs. (11), (15)
            if (m1 && m2) s = m1 * m2 * gather2(IS, KM, pair_uu(m1 - 1, m2 - 1), pair_uu(n1, n2));
            mm = gather2(I3, KM, pair_tt(m1, m2), pair_uu(n1, n2));
        }
        const double v = fma(sK, s, sM * mm);
        bad |= !isfinite(v);
        o[(int64_t)i * nd + j] = v;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(status + e, P2S_STATUS_NONFINITE_BIT);
}

// Direct quadrature of every entry of eqs. (8)-(15) (the method the paper
// compares against): one workgroup per (element, tile of rows); the four
// coupling factors (Gauss-weighted) and the 1-D T and U values at the points
// in LDS; each thread sums one entry over all Q x Q points.
__global__ __launch_bounds__(256) void k_cheb_direct(int M, int Q, const double *__restrict__ gx,
                                                     const double *__restrict__ gw,
                                                     const double *__restrict__ alpha, double *__restrict__ out,
                                                     double sK, double sM)
{
    extern __shared__ double smem[];
    const int nd = 2 * M * (M + 1), P = Q * Q, NT = M + 1;
    const int tiles = (nd + C2_ROWS - 1) / C2_ROWS;
    const int64_t e = blockIdx.x / tiles;
    const int r0 = (int)(blockIdx.x % tiles) * C2_ROWS;
    double *Al = smem;                 // [4][P], weighted
    double *Tv = smem + C2_NF * P;     // [NT][Q]
    double *Uv = Tv + NT * Q;          // [NT][Q]
    const double *src = alpha + e * (int64_t)C2_NF * P;
    for (int i = threadIdx.x; i < C2_NF * P; i += blockDim.x) {
        const int pt = i % P, a = pt / Q, b = pt - (pt / Q) * Q;
        Al[i] = gw[a] * gw[b] * src[i];
    }
    for (int i = threadIdx.x; i < NT * Q; i += blockDim.x) {
        const int k = i / Q, a = i - (i / Q) * Q;
        double t0 = 1.0, t1 = gx[a], u0 = 1.0, u1 = 2.0 * gx[a];
        for (int j = 0; j < k; ++j) {
            const double t2 = 2.0 * gx[a] * t1 - t0, u2 = 2.0 * gx[a] * u1 - u0;
            t0 = t1;
            t1 = t2;
            u0 = u1;
            u1 = u2;
        }
        Tv[i] = t0;
        Uv[i] = u0;
    }
    __syncthreads();
    double *o = out + e * (int64_t)nd * nd;
    const int r1 = min(nd, r0 + C2_ROWS);
    for (int x = threadIdx.x; x < (r1 - r0) * nd; x += blockDim.x) {
        const int i = r0 + x / nd, j = x - (x / nd) * nd;
        bool vi, vj;
        int m1, n1, m2, n2;
        c2_dof(i, M, vi, m1, n1);
        c2_dof(j, M, vj, m2, n2);
        // reference components and curls: E_u-function (m,n): (U_m T_n, 0),
        // curl -n U_m U_{n-1}; E_v-function: (0, T_m U_n), curl m U_{m-1} U_n
        const double *cu1 = vi ? (m1 ? Uv + (m1 - 1) * Q : nullptr) : Uv + m1 * Q;
        const double *cv1 = vi ? Uv + n1 * Q : (n1 ? Uv + (n1 - 1) * Q : nullptr);
        const double c1 = vi ? (double)m1 : -(double)n1;
        const double *cu2 = vj ? (m2 ? Uv + (m2 - 1) * Q : nullptr) : Uv + m2 * Q;
        const double *cv2 = vj ? Uv + n2 * Q : (n2 ? Uv + (n2 - 1) * Q : nullptr);
        const double c2 = vj ? (double)m2 : -(double)n2;
        const double *eu1 = vi ? Tv + m1 * Q : Uv + m1 * Q, *ev1 = vi ? Uv + n1 * Q : Tv + n1 * Q;
        const double *eu2 = vj ? Tv + m2 * Q : Uv + m2 * Q, *ev2 = vj ? Uv + n2 * Q : Tv + n2 * Q;
        const double *G = Al + (1 + (vi ? 1 : 0) + (vj ? 1 : 0)) * P;  // G_uu, G_uv or G_vv
        const bool curl = cu1 && cv1 && cu2 && cv2;
        double s = 0.0, mm = 0.0;
        for (int a = 0; a < Q; ++a) {
            const double pm = eu1[a] * eu2[a];
            const double ps = curl ? cu1[a] * cu2[a] : 0.0;
            for (int b = 0; b < Q; ++b) {
                mm = fma(pm * ev1[b] * ev2[b], G[a * Q + b], mm);
                if (curl) s = fma(ps * cv1[b] * cv2[b], Al[a * Q + b], s);
            }
        }
        o[(int64_t)i * nd + j] = fma(sK, c1 * c2 * s, sM * mm);
    }
}

}  // namespace p2s

using namespace p2s;

struct p2s_cheb2d_s {
    p2s_ctx ctx = nullptr;
    int device = 0;
    int64_t E = 0;
    int M = 0, Q = 0;
    double *d_gauss = nullptr;  // x[Q], w[Q]
    double *d_alpha = nullptr, *d_mom = nullptr;
    bool profile = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float ms[3] = {0.f, 0.f, 0.f};
    int runs = 0;
};

extern "C" {

int64_t p2s_cheb2d_num_dofs(int M) { return (M < 1 || M > C2_MAXM) ? -1 : 2 * (int64_t)M * (M + 1); }

int p2s_cheb2d_create(p2s_ctx ctx, int64_t E, int M, int Q, p2s_cheb2d *out)
{
    if (!ctx || !out) return P2S_EINVAL;
    *out = nullptr;
    if (E < 0) return P2S_EINVAL;
    if (M < 1 || M > C2_MAXM) return P2S_EORDER;
    if (Q < 1 || Q > P2S_MAX_Q) return P2S_EQUAD;
    std::vector<double> g(2 * Q);
    if (gauss_rule(Q, g.data(), g.data() + Q) != 0) return P2S_EQUAD;
    const int dev = p2s_context_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) return P2S_EHIP;
    auto p = new p2s_cheb2d_s();
    p->ctx = ctx;
    p->device = dev;
    p->E = E;
    p->M = M;
    p->Q = Q;
    const int KM = 2 * M + 1;
    bool ok = hipMalloc(&p->d_gauss, sizeof(double) * 2 * Q) == hipSuccess &&
              hipMalloc(&p->d_alpha, sizeof(double) * std::max<int64_t>(1, E * C2_NF * Q * Q)) == hipSuccess &&
              hipMalloc(&p->d_mom, sizeof(double) * std::max<int64_t>(1, E * C2_NF * KM * KM)) == hipSuccess &&
              hipMemcpy(p->d_gauss, g.data(), sizeof(double) * 2 * Q, hipMemcpyHostToDevice) == hipSuccess;
    for (auto &ev : p->ev) ok = ok && hipEventCreate(&ev) == hipSuccess;
    if (!ok) {
        p2s_cheb2d_destroy(p);
        return P2S_ENOMEM;
    }
    *out = p;
    return P2S_OK;
}

void p2s_cheb2d_destroy(p2s_cheb2d p)
{
    if (!p) return;
    hipFree(p->d_gauss);
    hipFree(p->d_alpha);
    hipFree(p->d_mom);
    for (auto &ev : p->ev)
        if (ev) hipEventDestroy(ev);
    delete p;
}

int p2s_cheb2d_execute(p2s_cheb2d p, int method, const double *nodes, const double *material, double stiff_scale,
                       double mass_scale, double *out, uint32_t *status, void *stream)
{
    if (!p) return P2S_EINVAL;
    if (method != P2S_METHOD_P2S && method != P2S_METHOD_DIRECT) return P2S_EINVAL;
    if (p->E == 0) return P2S_OK;
    if (!nodes || !material || !out || !status) return P2S_EINVAL;
    if (hipSetDevice(p->device) != hipSuccess) return P2S_EHIP;
    hipStream_t st = (hipStream_t)stream;
    const int M = p->M, Q = p->Q, KM = 2 * M + 1, nd = 2 * M * (M + 1);
    const int tiles = (nd + C2_ROWS - 1) / C2_ROWS;
    const double *gx = p->d_gauss, *gw = p->d_gauss + Q;
    if (p->profile) hipEventRecord(p->ev[0], st);
    hipLaunchKernelGGL(k_cheb_coupling, dim3((unsigned)p->E), dim3(256), 0, st, Q, nodes, material, gx, p->d_alpha,
                       status);
    if (p->profile) hipEventRecord(p->ev[1], st);
    if (method == P2S_METHOD_P2S) {
        hipLaunchKernelGGL(k_cheb_moments, dim3((unsigned)p->E, C2_NF), dim3(256), 0, st, Q, KM, gx, gw, p->d_alpha,
                           p->d_mom);
        if (p->profile) hipEventRecord(p->ev[2], st);
        hipLaunchKernelGGL(k_cheb_gather, dim3((unsigned)(p->E * tiles)), dim3(256),
                           sizeof(double) * C2_NF * KM * KM, st, M, p->d_mom, out, status, stiff_scale, mass_scale);
    } else {
        if (p->profile) hipEventRecord(p->ev[2], st);
        hipLaunchKernelGGL(k_cheb_direct, dim3((unsigned)(p->E * tiles)), dim3(256),
                           sizeof(double) * (C2_NF * Q * Q + 2 * (M + 1) * Q), st, M, Q, gx, gw, p->d_alpha, out,
                           stiff_scale, mass_scale);
    }
    if (p->profile) {
        hipEventRecord(p->ev[3], st);
        hipEventSynchronize(p->ev[3]);
        for (int s = 0; s < 3; ++s) {
            float t = 0.f;
            hipEventElapsedTime(&t, p->ev[s], p->ev[s + 1]);
            p->ms[s] += t;
        }
        p->runs++;
    }
    return hipGetLastError() == hipSuccess ? P2S_OK : P2S_EHIP;
}

int p2s_cheb2d_profile(p2s_cheb2d p, int enable, double *ms)
{
    if (!p) return P2S_EINVAL;
    if (ms)
        for (int s = 0; s < 3; ++s) ms[s] = p->runs ? p->ms[s] / p->runs : 0.0;
    p->profile = enable != 0;
    p->ms[0] = p->ms[1] = p->ms[2] = 0.f;
    p->runs = 0;
    return P2S_OK;
}

}  // extern "C"
