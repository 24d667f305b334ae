// p2s_split.hip -- split-FP32 form of the moment stage (eq. (4)) and of the
// contraction, on the FP32 matrix cores of gfx950 (v_mfma_f32_16x16x4f32).
//
// Every FP64 operand x is carried as two FP32 parts, hi = fl32(x) and
// lo = fl32(x - hi); a product of two split operands is hi*hi + hi*lo + lo*hi
// and a product with an FP32 intermediate is x*hi + x*lo.  The matrix cores
// accumulate in FP32 within one K-block of 16; each product-to-sum run's
// result is added into FP64 accumulators, and the coupling samples, tables
// and final sums stay FP64.  The FP32 accumulation bounds the relative error
// near 1e-7 whatever the operand split.
//
// MFMA 16x16x4 lane layout (wave64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register i of lane l is D[4(l/16)+i][l%16].
#include <hip/hip_runtime.h>

#include "p2s_internal.h"
#include "p2s_kernels.h"
#include "p2s_terms.h"

namespace p2s {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Moments: one workgroup (4 waves) per (element, field); Q <= 16 per axis,
// K = 2N-1 <= 15.  Three GEMM passes, each a K-block of 16:
//   P1[ab][q] = sum_c alpha[ab][c] Ww[q][c]      (alpha split: 3 products)
//   P2[a][l][q] = sum_b Wv[l][b] P1[ab][q]       (2 products)
//   I[k][l][q] = sum_a Wu[k][a] P2[a][l][q]      (2 products)
// Output I in FP32 at mom32 + mom_off (the FP64 moment buffer reused).

constexpr int PS = 17;  // LDS row stride of the pass results

__global__ __launch_bounds__(256) void k_moments_split(const ElemDesc *__restrict__ desc, int64_t e0, int F,
                                                       const double *__restrict__ alpha,
                                                       const float *__restrict__ t32, float *__restrict__ mom32)
{
    __shared__ float P1[256 * PS];
    __shared__ float P2[256 * PS];
    const int64_t e = e0 + blockIdx.x;
    const int f = blockIdx.y;
    const ElemDesc d = desc[e];
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw, K = 2 * d.N - 1;
    const int P = Qu * Qv * Qw;
    const double *A = alpha + d.alpha_off + (int64_t)f * P;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    // W[k][a] = w_a L_k(x_a) split, rows k < 16, columns a < 16
    const float *Wuh = t32 + T32_LEGW_H + Qu * T32_LEGW_Q, *Wul = t32 + T32_LEGW_L + Qu * T32_LEGW_Q;
    const float *Wvh = t32 + T32_LEGW_H + Qv * T32_LEGW_Q, *Wvl = t32 + T32_LEGW_L + Qv * T32_LEGW_Q;
    const float *Wwh = t32 + T32_LEGW_H + Qw * T32_LEGW_Q, *Wwl = t32 + T32_LEGW_L + Qw * T32_LEGW_Q;

    // pass 1: M = ab (Qu*Qv <= 256 rows), K = c, N = q
    const int nab = Qu * Qv;
    for (int mt = wave; mt < 16; mt += 4) {
        f4 c = {0.f, 0.f, 0.f, 0.f};
        const int ab = mt * 16 + r16;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int cc = ks * 4 + k4;
            const double x = (ab < nab && cc < Qw) ? A[(int64_t)ab * Qw + cc] : 0.0;
            const float xh = (float)x, xl = (float)(x - (double)xh);
            const float bh = Wwh[r16 * 16 + cc], bl = Wwl[r16 * 16 + cc];
            c = mfma(xl, bh, c);
            c = mfma(xh, bl, c);
            c = mfma(xh, bh, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) P1[(mt * 16 + 4 * k4 + i) * PS + r16] = c[i];
    }
    __syncthreads();
    // pass 2: per a, M = l, K = b, N = q
    for (int a = wave; a < Qu; a += 4) {
        f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int b = ks * 4 + k4;
            const float x = b < Qv ? P1[(a * Qv + b) * PS + r16] : 0.f;
            c = mfma(Wvl[r16 * 16 + b], x, c);
            c = mfma(Wvh[r16 * 16 + b], x, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) P2[(a * 16 + 4 * k4 + i) * PS + r16] = c[i];
    }
    __syncthreads();
    // pass 3: M = k, K = a, N = (l,q) in 16 tiles of 16 (tile nt has l = nt)
    float *I = mom32 + d.mom_off + (int64_t)f * K * K * K;
    for (int nt = wave; nt < 16; nt += 4) {
        f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int a = ks * 4 + k4;
            const float x = a < Qu ? P2[(a * 16 + nt) * PS + r16] : 0.f;
            c = mfma(Wul[r16 * 16 + a], x, c);
            c = mfma(Wuh[r16 * 16 + a], x, c);
        }
        const int l = nt, q = r16;
        if (l < K && q < K)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 4 * k4 + i;
                if (k < K) I[(k * K + l) * K + q] = c[i];
            }
    }
}

// ---------------------------------------------------------------------------
// Contraction: one workgroup (4 waves) per (element, row component I, m1)
// for the block (I,J); all per-axis index ranges are padded to 8 (MAXN),
// so (n1,n2) and (p1,p2) are 64-wide.  The block's terms come grouped by
// (v,w) family pair, runs of groups share the w pair (p2s_terms.h).
//   stage A  Ag[m2][l][q] = sum_{s in g} sc_s sum_k Cu_s[m1][m2][k] I_s[k][l][q]
//            M = m2 (16, 8 used), K = k, N = (l,q) 256; once per m1
//   stage B  Bsum[n1n2][q] = sum_{g in run} sum_l Cv_g[n1n2][l] Ag[m2][l][q]
//            M = n1n2 (wave w owns rows 16w..16w+15), K = l, N = q
//   stage C  acc[n1n2][p1p2] += sum_q Bsum[n1n2][q] Cw_run[p1p2][q]
//            M = n1n2, K = q, N = p1p2 (4 tiles); FP64 accumulation
// then through LDS to the dense output rows (and the mirrored columns).

constexpr int SPLIT_TILE_STRIDE = 65;  // doubles per LDS tile row

template <int PROB, int I, int J>
__global__ __launch_bounds__(256) void k_contract_split(const ElemDesc *__restrict__ desc, int64_t e0, int64_t count,
                                                        int64_t total_padded, const float *__restrict__ t32,
                                                        const float *__restrict__ mom32, double *__restrict__ out,
                                                        uint32_t *__restrict__ status, double sK, double sM)
{
    constexpr BlockC BK = BlockOf<PROB, I, J>::B;
    constexpr int NG = BK.ngroup;
    __shared__ float Ag[NG * 8 * 256];
    __shared__ float Bt[4 * 16 * PS];
    __shared__ double tile[64 * SPLIT_TILE_STRIDE];

    // work item: consecutive items (the m1 rows of one element) on one XCD
    const int64_t w = blockIdx.x;
    const int64_t per = total_padded >> 3;
    const int64_t item = (w & 7) * per + (w >> 3);
    const ElemDesc d0 = desc[e0];
    const int N = d0.N;
    const int NM_I = comp_dim(PROB, N, I, 0), NN_I = comp_dim(PROB, N, I, 1), NP_I = comp_dim(PROB, N, I, 2);
    const int NM_J = comp_dim(PROB, N, J, 0), NN_J = comp_dim(PROB, N, J, 1), NP_J = comp_dim(PROB, N, J, 2);
    if (item >= count * NM_I) return;
    const int64_t e = e0 + item / NM_I;
    const int m1 = (int)(item % NM_I);
    const ElemDesc d = desc[e];
    const int K = 2 * N - 1, NDOF = num_dofs(PROB, N);
    const float *Im = mom32 + d.mom_off;
    double *obase = out + d.out_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const float *LH = t32 + T32_LIN_H, *LL = t32 + T32_LIN_L;
    constexpr int TS = MAXN * MAXN * KPAD, M1S = MAXN * KPAD;  // lin strides: type, first index

    // stage A
    static_for<0, NG>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        for (int nt = wave; nt < 16; nt += 4) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
            static_for<BK.gstart[g], BK.gstart[g + 1]>([&](auto sc_) {
                constexpr TermC t = BK.t[decltype(sc_)::value];
                const float sc = (float)((t.scale ? sM : sK) * (double)t.sign);
                const float *Is = Im + (int64_t)t.field * K * K * K;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = ks * 4 + k4;
                    const int m2 = r16 < MAXN ? r16 : MAXN - 1;  // rows 8..15 are padding
                    const int ci = t.tu * TS + m1 * M1S + m2 * KPAD + k;
                    const float ah = r16 < MAXN ? sc * LH[ci] : 0.f;
                    const float al = r16 < MAXN ? sc * LL[ci] : 0.f;
                    const float x = (k < K && nt < K && r16 < K) ? Is[(k * K + nt) * K + r16] : 0.f;
                    c = mfma(al, x, c);
                    c = mfma(ah, x, c);
                }
            });
            if (k4 < 2)
#pragma unroll
                for (int i = 0; i < 4; ++i) Ag[(g * 8 + 4 * k4 + i) * 256 + nt * 16 + r16] = c[i];
        }
    });
    __syncthreads();

    const int m2lo = (J == I) ? m1 : 0;
    const int rowbase = comp_offset(PROB, N, I) + m1 * NN_I * NP_I;
    bool bad = false;
    // stage B/C rows of this wave: n1n2 = 16 wave + r16 (A operand of B)
    const int bn1 = (16 * wave + r16) >> 3, bn2 = (16 * wave + r16) & 7;
    for (int m2 = m2lo; m2 < NM_J; ++m2) {
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0;
        f4 cb = {0.f, 0.f, 0.f, 0.f};
        static_for<0, NG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            constexpr int tv = BK.t[BK.gstart[g]].tv;
            constexpr int tw = BK.t[BK.gstart[g]].tw;
            // stage B for group g, accumulated over the run
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int l = ks * 4 + k4;
                const int ci = tv * TS + bn1 * M1S + bn2 * KPAD + l;
                const float x = Ag[(g * 8 + m2) * 256 + l * 16 + r16];
                cb = mfma(LL[ci], x, cb);
                cb = mfma(LH[ci], x, cb);
            }
            if constexpr (BK.cflag[g] != 0) {
                // transpose the wave's Bsum tile for use as the A operand
                float *bt = Bt + wave * 16 * PS;
#pragma unroll
                for (int i = 0; i < 4; ++i) bt[(4 * k4 + i) * PS + r16] = cb[i];
                __syncthreads();
                // stage C for this run, 4 column tiles of (p1,p2)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    f4 cc = {0.f, 0.f, 0.f, 0.f};
                    const int pp = nt * 16 + r16;
                    const int p1 = pp >> 3, p2 = pp & 7;
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int q = ks * 4 + k4;
                        const float a = bt[r16 * PS + q];
                        const int ci = tw * TS + p1 * M1S + p2 * KPAD + q;
                        cc = mfma(a, LL[ci], cc);
                        cc = mfma(a, LH[ci], cc);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[nt * 4 + i] += (double)cc[i];
                }
                __syncthreads();
                cb = f4{0.f, 0.f, 0.f, 0.f};
            }
        });
        // tile[n1n2][p1p2] in FP64
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                tile[(16 * wave + 4 * k4 + i) * SPLIT_TILE_STRIDE + nt * 16 + r16] = acc[nt * 4 + i];
        __syncthreads();
        // rows (n1,p1) of m1 against columns (n2,p2) of m2.  Threads take a
        // padded 8x8 grid: the low six bits of the thread id give the
        // contiguous pair of a row, the high bits the row (four per pass), so
        // the index arithmetic is shifts and masks only.
        const int colbase = comp_offset(PROB, N, J) + m2 * NN_J * NP_J;
        {
            const int t = threadIdx.x & 63, ta = t >> 3, tb = t & 7;  // (n2,p2) / (n1,p1) of the thread
            for (int rr = threadIdx.x >> 6; rr < 64; rr += blockDim.x >> 6) {
                const int ra = rr >> 3, rb = rr & 7;                  // (n1,p1) / (n2,p2) of the row
                // direct: row (n1,p1) = (ra,rb), column (n2,p2) = (ta,tb)
                if (ra < NN_I && rb < NP_I && ta < NN_J && tb < NP_J) {
                    const double v = tile[(ra * 8 + ta) * SPLIT_TILE_STRIDE + rb * 8 + tb];
                    bad |= !isfinite(v);
                    obase[(int64_t)(rowbase + ra * NP_I + rb) * NDOF + colbase + ta * NP_J + tb] = v;
                }
                // mirror: row colbase + (n2,p2) = (ra,rb) of J, column rowbase + (n1,p1) = (ta,tb) of I
                if ((J != I || m2 != m1) && ra < NN_J && rb < NP_J && ta < NN_I && tb < NP_I)
                    obase[(int64_t)(colbase + ra * NP_J + rb) * NDOF + rowbase + ta * NP_I + tb] =
                        tile[(ta * 8 + ra) * SPLIT_TILE_STRIDE + tb * 8 + rb];
            }
        }
        __syncthreads();
    }
    bad = __syncthreads_or(bad);
    if (bad && threadIdx.x == 0) atomicOr(status + e, P2S_STATUS_NONFINITE_BIT);
}

// ---------------------------------------------------------------------------

__global__ void k_widen(int64_t n, const float *__restrict__ src, double *__restrict__ dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

void launch_widen(int64_t n, const float *src, double *dst, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src, dst);
}

void launch_moments_split(int problem, const ElemDesc *desc, int64_t e0, int64_t count, const double *alpha,
                          const float *t32, float *mom32, hipStream_t st)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_moments_split, dim3((unsigned)count, num_fields(problem)), dim3(256), 0, st, desc, e0,
                       num_fields(problem), alpha, t32, mom32);
}

template <int PROB, int I, int J>
static void launch_block(int N, const ElemDesc *desc, int64_t e0, int64_t count, const float *t32,
                         const float *mom32, double *out, uint32_t *status, double sK, double sM, hipStream_t st)
{
    const int64_t items = count * comp_dim(PROB, N, I, 0);
    const int64_t padded = (items + 7) & ~int64_t(7);
    hipLaunchKernelGGL((k_contract_split<PROB, I, J>), dim3((unsigned)padded), dim3(256), 0, st, desc, e0, count,
                       padded, t32, mom32, out, status, sK, sM);
}

void launch_contract_split(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const float *t32,
                           const float *mom32, double *out, uint32_t *status, double sK, double sM, hipStream_t st)
{
    if (count <= 0) return;
    if (problem == 0) {
        launch_block<0, 0, 0>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
        return;
    }
    launch_block<1, 0, 0>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
    launch_block<1, 0, 1>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
    launch_block<1, 0, 2>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
    launch_block<1, 1, 1>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
    launch_block<1, 1, 2>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
    launch_block<1, 2, 2>(N, desc, e0, count, t32, mom32, out, status, sK, sM, st);
}

}  // namespace p2s
