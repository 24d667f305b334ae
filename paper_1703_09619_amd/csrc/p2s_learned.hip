// p2s_learned.hip -- learned quadrature order for the moment stage.
//
// A small FP32 network (85 -> 128 -> 128 -> 57, ReLU) maps an element's
// geometry and material parameters to, per axis, a distribution over the
// Gauss rule size K in {6..24} used to sample the coupling factor before the
// moment stage (eq. (4)).  The smallest K whose predicted cumulative
// probability reaches p_cover is used; a tail check on the sampled coupling
// factor (its highest resolvable Legendre coefficients along each axis)
// sends elements it does not trust back to the full rule.
//
// Everything here runs in these kernels: features, inference, the order
// choice, the tail decision (its statistic is gathered by the moment
// stage), and training (forward with saved activations,
// softmax cross-entropy backward, weight gradients, Adam).
#include <hip/hip_runtime.h>

#include <cmath>

#include "p2s_internal.h"
#include "p2s_kernels.h"

namespace p2s {

// ---------------------------------------------------------------------------
// Features: node offsets from the nominal cube (81, scaled by 1/0.3) and the
// first four material parameters (plane wave: |k_x|, |k_y|, |k_z| / (16 pi),
// phase / (2 pi) - 1/2; the sign of a wave-vector component does not change
// how finely the field must be sampled along that axis).
__global__ void k_features(int64_t E, const double *__restrict__ nodes, const double *__restrict__ mat,
                           int kind, int stride, float *__restrict__ X)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= E * MLP_IN) return;
    const int64_t e = t / MLP_IN;
    const int f = (int)(t % MLP_IN);
    float v = 0.f;
    if (f < 81) {
        const int node = f / 3, r = f % 3;
        const int idx[3] = {node % 3, (node / 3) % 3, node / 9};
        v = (float)((nodes[e * 81 + f] - 0.5 * idx[r]) / 0.3);
    } else {
        const int q = f - 81;
        if (q < stride) {
            const double p = mat[e * stride + q];
            if (kind == MAT_PLANEWAVE)
                v = (float)(q < 3 ? fabs(p) / (16.0 * 3.14159265358979323846)
                                  : p / (2.0 * 3.14159265358979323846) - 0.5);
            else
                v = (float)p;
        }
    }
    X[t] = v;
}

// Y[b][o] = act(sum_i X[b][i] W[i][o] + bias[o])
__global__ void k_dense(int64_t B, int I, int O, const float *__restrict__ X, const float *__restrict__ W,
                        const float *__restrict__ bias, float *__restrict__ Y, int relu)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * O) return;
    const int64_t b = t / O;
    const int o = (int)(t % O);
    const float *x = X + b * I;
    float acc = bias[o];
    for (int i = 0; i < I; ++i) acc = fmaf(x[i], W[(int64_t)i * O + o], acc);
    Y[t] = relu ? fmaxf(acc, 0.f) : acc;
}

// Per-sample softmax cross-entropy summed over the three axes; dZ holds
// (softmax - onehot) / B.
__global__ void k_softmax_ce(int64_t B, const float *__restrict__ Z, const int32_t *__restrict__ labels,
                             float *__restrict__ dZ, float *__restrict__ loss)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    float l = 0.f;
    for (int ax = 0; ax < 3; ++ax) {
        const float *z = Z + b * MLP_OUT + ax * MLP_NCLS;
        float mx = z[0];
        for (int c = 1; c < MLP_NCLS; ++c) mx = fmaxf(mx, z[c]);
        float s = 0.f;
        for (int c = 0; c < MLP_NCLS; ++c) s += expf(z[c] - mx);
        const int y = min(max(labels[b * 3 + ax], 0), MLP_NCLS - 1);
        l += logf(s) - (z[y] - mx);
        if (dZ) {
            float *dz = dZ + b * MLP_OUT + ax * MLP_NCLS;
            for (int c = 0; c < MLP_NCLS; ++c) dz[c] = (expf(z[c] - mx) / s - (c == y ? 1.f : 0.f)) / (float)B;
        }
    }
    loss[b] = l;
}

// dW[i][o] = sum_b A[b][i] dY[b][o]  (i < I);  row i == I holds db[o]
__global__ void k_dense_wgrad(int64_t B, int I, int O, const float *__restrict__ A, const float *__restrict__ dY,
                              float *__restrict__ dW, float *__restrict__ db)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (I + 1) * O) return;
    const int i = t / O, o = t % O;
    float acc = 0.f;
    if (i < I) {
        for (int64_t b = 0; b < B; ++b) acc = fmaf(A[b * I + i], dY[b * O + o], acc);
        dW[(int64_t)i * O + o] = acc;
    } else {
        for (int64_t b = 0; b < B; ++b) acc += dY[b * O + o];
        db[o] = acc;
    }
}

// dX[b][i] = (sum_o dY[b][o] W[i][o]) * (A[b][i] > 0)   (A: the ReLU output)
__global__ void k_dense_xgrad(int64_t B, int I, int O, const float *__restrict__ dY, const float *__restrict__ W,
                              const float *__restrict__ A, float *__restrict__ dX)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * I) return;
    const int64_t b = t / I;
    const int i = (int)(t % I);
    float acc = 0.f;
    for (int o = 0; o < O; ++o) acc = fmaf(dY[b * O + o], W[(int64_t)i * O + o], acc);
    dX[t] = A[t] > 0.f ? acc : 0.f;
}

__global__ void k_sum(int64_t n, const float *__restrict__ x, float *__restrict__ out)
{
    __shared__ float s[256];
    float acc = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += x[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// omb1 = 1 - b1, omb2 = 1 - b2, c1 = 1 - b1^t, c2 = 1 - b2^t are formed in
// FP64 on the host: in FP32, 1 - 0.999f and 1 - 0.999f^t lose up to five
// digits to cancellation.
__global__ void k_adam(int P, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps,
                       float c1, float c2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + omb1 * gt;
    const float vt = b2 * v[t] + omb2 * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// Order choice: per element and axis, the smallest K whose cumulative
// predicted probability reaches p_cover, raised to the full rule MLP_KMAX
// when it is at least k_direct (an axis the network is that unsure of is
// sampled with the full rule at once); written to quad[e][3] and, when desc
// is given, into the element descriptors.
__global__ void k_choose(int64_t E, const float *__restrict__ Z, float p_cover, int k_direct,
                         int32_t *__restrict__ quad, ElemDesc *__restrict__ desc)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= E) return;
    int K[3];
    for (int ax = 0; ax < 3; ++ax) {
        const float *z = Z + e * MLP_OUT + ax * MLP_NCLS;
        float mx = z[0];
        for (int c = 1; c < MLP_NCLS; ++c) mx = fmaxf(mx, z[c]);
        float s = 0.f;
        for (int c = 0; c < MLP_NCLS; ++c) s += expf(z[c] - mx);
        float cdf = 0.f;
        int pick = MLP_NCLS - 1;
        for (int c = 0; c < MLP_NCLS; ++c) {
            cdf += expf(z[c] - mx) / s;
            if (cdf >= p_cover) {
                pick = c;
                break;
            }
        }
        K[ax] = MLP_KMIN + pick >= k_direct ? MLP_KMAX : MLP_KMIN + pick;
        if (quad) quad[e * 3 + ax] = K[ax];
    }
    if (desc) {
        desc[e].Qu = K[0];
        desc[e].Qv = K[1];
        desc[e].Qw = K[2];
    }
}

// ---------------------------------------------------------------------------
// Tail check.  With Q points along an axis, the moment of degree k along it
// is exact unless the integrand has Legendre content along that axis at
// degrees >= 2Q - k; the highest moment degree is K_m - 1 = 2N - 2.  The
// moment stage records, per field and axis, the envelope A_j (largest
// magnitude) of the discrete Legendre coefficients of degrees Q-1 .. Q-4
// along the axis, projected on the other two axes onto the moment degrees,
// and the scale S (largest moment magnitude).  Per axis, over the fields:
//   r2  = min(1, max(A_1/A_3, A_2/A_4))    (decay over two degrees)
//   est = max(A_1, A_2) r2^((Q - K_m + 2)/2)  (content at degree 2Q-K_m+1)
//   t   = est / S.
// Only axes sampled below the full rule can differ from the full-rule fill
// (the moment stage records nothing for the others): tau = max of t over
// those axes.  tau > theta sends the element back to the full rule
// (redo[e] = 1, descriptor set to `qfull` on every axis, fallback bit).
__global__ void k_tail_decide(ElemDesc *__restrict__ desc, int64_t e0, int64_t count, int F,
                              const double *__restrict__ tailst, double theta, int qfull,
                              int32_t *__restrict__ redo, uint32_t *__restrict__ status,
                              double *__restrict__ tau_out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t e = e0 + i;
    const ElemDesc d = desc[e];
    const int Q[3] = {d.Qu, d.Qv, d.Qw};
    const int Km = 2 * d.N - 1;
    double tau = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        if (Q[ax] >= qfull) continue;
        double A[4] = {0.0, 0.0, 0.0, 0.0}, S = 0.0;
        for (int f = 0; f < F; ++f) {
            const double *r = tailst + (e * F + f) * TAIL_REC;
#pragma unroll
            for (int j = 0; j < 4; ++j) A[j] = fmax(A[j], r[ax * 4 + j]);
            S = fmax(S, r[12 + ax]);
        }
        double r2 = fmax(A[2] > 0.0 ? A[0] / A[2] : 1.0, A[3] > 0.0 ? A[1] / A[3] : 1.0);
        r2 = fmin(r2, 1.0);
        const double expo = fmax(0.5 * (double)(Q[ax] - Km + 2), 0.0);
        const double est = fmax(A[0], A[1]) * pow(r2, expo);
        tau = fmax(tau, est / fmax(S, 1e-300));
    }
    if (tau_out) tau_out[e] = tau;
    const bool fail = !(tau <= theta);
    redo[e] = fail ? 1 : 0;
    if (fail) {
        desc[e].Qu = desc[e].Qv = desc[e].Qw = qfull;
        status[e] |= P2S_STATUS_FALLBACK_BIT;
    }
}

// Per-element relative Frobenius difference ||a - b|| / ||b|| of blocks of
// `len` doubles at element offsets off[e] (or e*len when off is null).
__global__ __launch_bounds__(256) void k_rel_error(int64_t len, const int64_t *__restrict__ off,
                                                   const double *__restrict__ a, const double *__restrict__ b,
                                                   double *__restrict__ err)
{
    const int64_t e = blockIdx.x;
    const int64_t o = off ? off[e] : e * len;
    const int64_t n = off ? off[e + 1] - off[e] : len;
    __shared__ double s[2][256];
    double d2 = 0.0, b2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = a[o + i], y = b[o + i];
        d2 = fma(x - y, x - y, d2);
        b2 = fma(y, y, b2);
    }
    s[0][threadIdx.x] = d2;
    s[1][threadIdx.x] = b2;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) err[e] = sqrt(s[0][0]) / sqrt(s[1][0]);
}

// ---------------------------------------------------------------------------
// Host launchers

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_features(int64_t E, const double *nodes, const double *mat, int kind, int stride, float *X,
                     hipStream_t st)
{
    if (E > 0)
        hipLaunchKernelGGL(k_features, dim3(nblk(E * MLP_IN, 256)), dim3(256), 0, st, E, nodes, mat, kind, stride, X);
}

void launch_mlp_forward(int64_t B, const float *params, const float *X, float *H1, float *H2, float *Z,
                        hipStream_t st)
{
    if (B <= 0) return;
    hipLaunchKernelGGL(k_dense, dim3(nblk(B * MLP_H, 256)), dim3(256), 0, st, B, MLP_IN, MLP_H, X,
                       params + MLP_OFF_W1, params + MLP_OFF_B1, H1, 1);
    hipLaunchKernelGGL(k_dense, dim3(nblk(B * MLP_H, 256)), dim3(256), 0, st, B, MLP_H, MLP_H, H1,
                       params + MLP_OFF_W2, params + MLP_OFF_B2, H2, 1);
    hipLaunchKernelGGL(k_dense, dim3(nblk(B * MLP_OUT, 256)), dim3(256), 0, st, B, MLP_H, MLP_OUT, H2,
                       params + MLP_OFF_W3, params + MLP_OFF_B3, Z, 0);
}

void launch_mlp_backward(int64_t B, const float *params, const float *X, const float *H1, const float *H2,
                         const float *Z, const int32_t *labels, float *dZ, float *dH2, float *dH1, float *grad,
                         float *loss_b, float *loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_softmax_ce, dim3(nblk(B, 256)), dim3(256), 0, st, B, Z, labels, dZ, loss_b);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, B, loss_b, loss);
    hipLaunchKernelGGL(k_dense_wgrad, dim3(nblk((MLP_H + 1) * MLP_OUT, 256)), dim3(256), 0, st, B, MLP_H, MLP_OUT,
                       H2, dZ, grad + MLP_OFF_W3, grad + MLP_OFF_B3);
    hipLaunchKernelGGL(k_dense_xgrad, dim3(nblk(B * MLP_H, 256)), dim3(256), 0, st, B, MLP_H, MLP_OUT, dZ,
                       params + MLP_OFF_W3, H2, dH2);
    hipLaunchKernelGGL(k_dense_wgrad, dim3(nblk((MLP_H + 1) * MLP_H, 256)), dim3(256), 0, st, B, MLP_H, MLP_H,
                       H1, dH2, grad + MLP_OFF_W2, grad + MLP_OFF_B2);
    hipLaunchKernelGGL(k_dense_xgrad, dim3(nblk(B * MLP_H, 256)), dim3(256), 0, st, B, MLP_H, MLP_H, dH2,
                       params + MLP_OFF_W2, H1, dH1);
    hipLaunchKernelGGL(k_dense_wgrad, dim3(nblk((MLP_IN + 1) * MLP_H, 256)), dim3(256), 0, st, B, MLP_IN, MLP_H,
                       X, dH1, grad + MLP_OFF_W1, grad + MLP_OFF_B1);
}

void launch_adam(float *params, const float *grad, float *m, float *v, float lr, int step, hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(MLP_PARAMS, 256)), dim3(256), 0, st, MLP_PARAMS, params, grad, m, v, lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

void launch_choose(int64_t E, const float *Z, float p_cover, int k_direct, int32_t *quad, ElemDesc *desc,
                   hipStream_t st)
{
    if (E > 0)
        hipLaunchKernelGGL(k_choose, dim3(nblk(E, 256)), dim3(256), 0, st, E, Z, p_cover, k_direct, quad, desc);
}

void launch_tail_decide(ElemDesc *desc, int64_t e0, int64_t count, int F, const double *tailst, double theta,
                        int qfull, int32_t *redo, uint32_t *status, double *tau, hipStream_t st)
{
    if (count > 0)
        hipLaunchKernelGGL(k_tail_decide, dim3(nblk(count, 256)), dim3(256), 0, st, desc, e0, count, F, tailst, theta,
                           qfull, redo, status, tau);
}

void launch_rel_error(int64_t E, int64_t len, const int64_t *off, const double *a, const double *b, double *err,
                      hipStream_t st)
{
    if (E > 0) hipLaunchKernelGGL(k_rel_error, dim3((unsigned)E), dim3(256), 0, st, len, off, a, b, err);
}

}  // namespace p2s
